// device.h -- device-side building blocks shared by the libscn kernels:
// counter-based random numbers, candidate poses, sphere-set transforms and the
// sphere-vs-box / sphere-vs-sphere / sphere-vs-grid tests.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scn.h"

namespace scn {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32
// S-box; multipliers 0xD2511F53 / 0xCD9E8D57, key schedule bumped by the
// Weyl constants 0x9E3779B9 / 0xBB67AE85 between rounds.
// ---------------------------------------------------------------------------
struct U4 { uint32_t a, b, c, d; };

__device__ __forceinline__ U4 philox10(U4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64 product each (v_mad_u64_u32) for both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * x.a, p1 = (uint64_t)0xCD9E8D57u * x.c;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        x = U4{hi1 ^ x.b ^ k0, lo1, hi0 ^ x.d ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x;
}

// (w >> 9) + 1/2 scaled by 2^-23: a uniform in (0,1), exact in binary32.
// Returned as the signed unit 2u - 1 in (-1, 1), also exact.
__device__ __forceinline__ float signed_unit(uint32_t w) {
    return fmaf((float)(w >> 9), 2.0f / 8388608.0f, 1.0f / 8388608.0f - 1.0f);
}
__device__ __forceinline__ float unit01(uint32_t w) {
    return ((float)(w >> 9) + 0.5f) * (1.0f / 8388608.0f);
}

// Support surface row (16 floats): R[9] support->world, t[3], hx, hy, inset, lift.
struct Support {
    float R[9], t[3], hx, hy, inset, lift;
};
__device__ __forceinline__ Support load_support(const float* __restrict__ sup, int u) {
    Support S;
    const float* p = sup + 16 * u;
#pragma unroll
    for (int i = 0; i < 9; ++i) S.R[i] = p[i];
    S.t[0] = p[9]; S.t[1] = p[10]; S.t[2] = p[11];
    S.hx = p[12]; S.hy = p[13]; S.inset = p[14]; S.lift = p[15];
    return S;
}

// Candidate pose in the support frame: position and yaw (as cos/sin).
struct Pose { float x, y, z, c, s, yaw; };

// Candidate i of attempt a for the object at position j of scene s.
__device__ __forceinline__ Pose sample_pose(uint64_t seed, uint32_t s, uint32_t j, uint32_t a,
                                            uint32_t i, float ax, float ay, float z,
                                            uint32_t* w3 = nullptr) {
    U4 w = philox10(U4{i, a, j, s}, (uint32_t)seed, (uint32_t)(seed >> 32));
    if (w3) *w3 = w.d;   // the fourth word: the stable-pose choice
    Pose p;
    p.x = ax * signed_unit(w.a);
    p.y = ay * signed_unit(w.b);
    const float u2 = unit01(w.c);
    p.yaw = 6.28318530717958647692f * u2;
    sincospif(2.0f * u2, &p.s, &p.c);
    p.z = z;
    return p;
}

// Stable pose of a candidate of an object with table rows [r0, r1): the
// first row whose cumulative weight (row entry 9) reaches u = unit01(w3)
// (exact comparisons of exact values); -1 without rows.
__device__ __forceinline__ int stable_pick(const int32_t* __restrict__ pose_off,
                                           const float* __restrict__ stable, int o, uint32_t w3) {
    if (!pose_off) return -1;
    const int r0 = pose_off[o], r1 = pose_off[o + 1];
    if (r1 <= r0) return -1;
    const float u = unit01(w3);
    int r = r0;
    while (r < r1 - 1 && !(u <= stable[12 * r + 9])) ++r;
    return r;
}

// c turned into a stable pose's resting frame: R c (R row-major).
__device__ __forceinline__ void rest_point(const float* __restrict__ R, float cx, float cy, float cz,
                                           float& x, float& y, float& z) {
    x = fmaf(R[0], cx, fmaf(R[1], cy, R[2] * cz));
    y = fmaf(R[3], cx, fmaf(R[4], cy, R[5] * cz));
    z = fmaf(R[6], cx, fmaf(R[7], cy, R[8] * cz));
}

// Object-frame point -> world: R_u (Rz(yaw) c + (x,y,z)) + t_u.
__device__ __forceinline__ void to_world(const Support& S, const Pose& P, float cx, float cy,
                                         float cz, float& wx, float& wy, float& wz) {
    const float lx = fmaf(P.c, cx, fmaf(-P.s, cy, P.x));
    const float ly = fmaf(P.s, cx, fmaf(P.c, cy, P.y));
    const float lz = cz + P.z;
    wx = fmaf(S.R[0], lx, fmaf(S.R[1], ly, fmaf(S.R[2], lz, S.t[0])));
    wy = fmaf(S.R[3], lx, fmaf(S.R[4], ly, fmaf(S.R[5], lz, S.t[1])));
    wz = fmaf(S.R[6], lx, fmaf(S.R[7], ly, fmaf(S.R[8], lz, S.t[2])));
}

// Supports that turn about z only, R = [[a, -b, 0], [b, a, 0], [0, 0, 1]]
// (the exact pattern z-rotations have in FP32), compose with the candidate's
// yaw into one planar rotation: world = [[C, -S], [S, C]] (cx, cy) + (Tx, Ty),
// and world z = (cz + z) + t_z does not depend on the candidate at all.
__device__ __forceinline__ bool yaw_support(const Support& U) {
    return U.R[2] == 0.f && U.R[5] == 0.f && U.R[6] == 0.f && U.R[7] == 0.f && U.R[8] == 1.f &&
           U.R[0] == U.R[4] && U.R[1] == -U.R[3];
}
struct Planar { float C, S, Tx, Ty; };
__device__ __forceinline__ Planar planar(const Support& U, const Pose& P) {
    const float a = U.R[0], b = U.R[3];
    Planar m;
    m.C = fmaf(a, P.c, -b * P.s);
    m.S = fmaf(b, P.c, a * P.s);
    m.Tx = fmaf(a, P.x, fmaf(-b, P.y, U.t[0]));
    m.Ty = fmaf(b, P.x, fmaf(a, P.y, U.t[1]));
    return m;
}
__device__ __forceinline__ void planar_xy(const Planar& m, float cx, float cy, float& wx, float& wy) {
    wx = fmaf(m.C, cx, fmaf(-m.S, cy, m.Tx));
    wy = fmaf(m.S, cx, fmaf(m.C, cy, m.Ty));
}

// Box row (16 floats): R[9] box->world, centre[3], half extents[3].
// Box-local excess e = |R^T (p - c)| - h.
__device__ __forceinline__ void box_excess(const float* B, float px, float py, float pz,
                                           float& ex, float& ey, float& ez) {
    const float dx = px - B[9], dy = py - B[10], dz = pz - B[11];
    const float qx = fmaf(B[0], dx, fmaf(B[3], dy, B[6] * dz));
    const float qy = fmaf(B[1], dx, fmaf(B[4], dy, B[7] * dz));
    const float qz = fmaf(B[2], dx, fmaf(B[5], dy, B[8] * dz));
    ex = fabsf(qx) - B[12];
    ey = fabsf(qy) - B[13];
    ez = fabsf(qz) - B[14];
}

// Same excess with the box held in registers (R row-major, centre c, half h).
__device__ __forceinline__ void box_excess_reg(const float* R, const float* c, const float* h,
                                               float px, float py, float pz, float& ex, float& ey,
                                               float& ez) {
    const float dx = px - c[0], dy = py - c[1], dz = pz - c[2];
    ex = fabsf(fmaf(R[0], dx, fmaf(R[3], dy, R[6] * dz))) - h[0];
    ey = fabsf(fmaf(R[1], dx, fmaf(R[4], dy, R[7] * dz))) - h[1];
    ez = fabsf(fmaf(R[2], dx, fmaf(R[5], dy, R[8] * dz))) - h[2];
}

// Exact signed distance to the box.
__device__ __forceinline__ float box_sdf(const float* B, float px, float py, float pz) {
    float ex, ey, ez;
    box_excess(B, px, py, pz, ex, ey, ez);
    const float ox = fmaxf(ex, 0.f), oy = fmaxf(ey, 0.f), oz = fmaxf(ez, 0.f);
    const float out = __builtin_amdgcn_sqrtf(fmaf(ox, ox, fmaf(oy, oy, oz * oz)));
    return out + fminf(fmaxf(ex, fmaxf(ey, ez)), 0.f);
}

// Squared outside distance |max(e,0)|^2: the sphere (radius r) comes closer
// than margin to the box iff this is < (r + margin)^2 (inside gives 0).
__device__ __forceinline__ float box_out2(const float* B, float px, float py, float pz) {
    float ex, ey, ez;
    box_excess(B, px, py, pz, ex, ey, ez);
    const float ox = fmaxf(ex, 0.f), oy = fmaxf(ey, 0.f), oz = fmaxf(ez, 0.f);
    return fmaf(ox, ox, fmaf(oy, oy, oz * oz));
}

// Boxes whose rotation keeps the z axis (R[2] = R[5] = R[6] = R[7] = 0,
// R[8] = 1): the same value as box_out2, bit for bit, with the zero terms left
// out (an FMA with a zero product adds exactly the other term).
__device__ __forceinline__ bool yaw_box(const float* B) {
    return B[2] == 0.f && B[5] == 0.f && B[6] == 0.f && B[7] == 0.f && B[8] == 1.f;
}
__device__ __forceinline__ float box_out2_yaw(const float* B, float px, float py, float pz) {
    const float dx = px - B[9], dy = py - B[10], dz = pz - B[11];
    const float ox = fmaxf(fabsf(fmaf(B[0], dx, B[3] * dy)) - B[12], 0.f);
    const float oy = fmaxf(fabsf(fmaf(B[1], dx, B[4] * dy)) - B[13], 0.f);
    const float oz = fmaxf(fabsf(dz) - B[14], 0.f);
    return fmaf(ox, ox, fmaf(oy, oy, oz * oz));
}
template <bool kYaw>
__device__ __forceinline__ float box_out2_t(const float* B, float px, float py, float pz) {
    if constexpr (kYaw) return box_out2_yaw(B, px, py, pz);
    else return box_out2(B, px, py, pz);
}

// Grid instance row (24 floats): W[9] world->grid, tw[3], origin[3], h, nx, ny, nz, pad.
// Trilinear sample of node values at a world point; +inf outside the nodes,
// NaN inside when a node it reads is not finite (non-finite input collides).
__device__ __forceinline__ float grid_sample(const float* G, const float* __restrict__ vals,
                                             float px, float py, float pz) {
    const float gx = fmaf(G[0], px, fmaf(G[1], py, fmaf(G[2], pz, G[9])));
    const float gy = fmaf(G[3], px, fmaf(G[4], py, fmaf(G[5], pz, G[10])));
    const float gz = fmaf(G[6], px, fmaf(G[7], py, fmaf(G[8], pz, G[11])));
    const float inv_h = 1.0f / G[15];
    const int nx = (int)G[16], ny = (int)G[17], nz = (int)G[18];
    const float fx = (gx - G[12]) * inv_h, fy = (gy - G[13]) * inv_h, fz = (gz - G[14]) * inv_h;
    if (!(fx >= 0.f && fy >= 0.f && fz >= 0.f && fx <= (float)(nx - 1) && fy <= (float)(ny - 1) &&
          fz <= (float)(nz - 1)))
        return __builtin_huge_valf();
    const int ix = min((int)fx, nx - 2), iy = min((int)fy, ny - 2), iz = min((int)fz, nz - 2);
    const float tx = fx - (float)ix, ty = fy - (float)iy, tz = fz - (float)iz;
    const float* v = vals + ((size_t)iz * ny + iy) * nx + ix;
    const size_t sy = nx, sz = (size_t)nx * ny;
    const float c00 = fmaf(tx, v[1] - v[0], v[0]);
    const float c10 = fmaf(tx, v[sy + 1] - v[sy], v[sy]);
    const float c01 = fmaf(tx, v[sz + 1] - v[sz], v[sz]);
    const float c11 = fmaf(tx, v[sz + sy + 1] - v[sz + sy], v[sz + sy]);
    const float c0 = fmaf(ty, c10 - c00, c00);
    const float c1 = fmaf(ty, c11 - c01, c01);
    // a non-finite node makes the interpolant non-finite (no finite weight
    // cancels an infinity or a NaN)
    const float r = fmaf(tz, c1 - c0, c0);
    return __builtin_isfinite(r) ? r : __builtin_nanf("");
}

// Every one of n floats is finite (not NaN, not an infinity).
__device__ __forceinline__ bool all_finite(const float* p, int n) {
    bool ok = true;
    for (int i = 0; i < n; ++i) ok &= __builtin_isfinite(p[i]);
    return ok;
}
__device__ __forceinline__ bool finite4(const float4& v) {
    return __builtin_isfinite(v.x) & __builtin_isfinite(v.y) & __builtin_isfinite(v.z) &
           __builtin_isfinite(v.w);
}

// Squared distance from a world point to a grid instance's node box (0 inside).
__device__ __forceinline__ float grid_box_d2(const float* G, float px, float py, float pz) {
    const float gx = fmaf(G[0], px, fmaf(G[1], py, fmaf(G[2], pz, G[9])));
    const float gy = fmaf(G[3], px, fmaf(G[4], py, fmaf(G[5], pz, G[10])));
    const float gz = fmaf(G[6], px, fmaf(G[7], py, fmaf(G[8], pz, G[11])));
    const float ex = G[15] * (G[16] - 1.f), ey = G[15] * (G[17] - 1.f), ez = G[15] * (G[18] - 1.f);
    const float dx = fmaxf(fmaxf(G[12] - gx, gx - (G[12] + ex)), 0.f);
    const float dy = fmaxf(fmaxf(G[13] - gy, gy - (G[13] + ey)), 0.f);
    const float dz = fmaxf(fmaxf(G[14] - gz, gz - (G[14] + ez)), 0.f);
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Reachability of an object frame at world position p with x axis d by the
// robot at base pose rb (R[9], t[3]) on the 4-D map (z*, theta, x*, y*):
// base-frame position turned by the object's yaw about the base z axis.
__device__ __forceinline__ bool reach_ok(const uint8_t* __restrict__ map, const scn_reach_map& m,
                                         const float* rb, float px, float py, float pz, float dx,
                                         float dy, float dz, float theta) {
    const float vx = px - rb[9], vy = py - rb[10], vz = pz - rb[11];
    const float qx = fmaf(rb[0], vx, fmaf(rb[3], vy, rb[6] * vz));
    const float qy = fmaf(rb[1], vx, fmaf(rb[4], vy, rb[7] * vz));
    const float qz = fmaf(rb[2], vx, fmaf(rb[5], vy, rb[8] * vz));
    const float ex = fmaf(rb[0], dx, fmaf(rb[3], dy, rb[6] * dz));
    const float ey = fmaf(rb[1], dx, fmaf(rb[4], dy, rb[7] * dz));
    const float n = sqrtf(fmaf(ex, ex, ey * ey));
    const float cs = n > 0.f ? ex / n : 1.f, sn = n > 0.f ? ey / n : 0.f;
    const float v[4] = {qz, theta, fmaf(cs, qx, sn * qy), fmaf(-sn, qx, cs * qy)};
    int idx[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const float f = floorf((v[a] - m.lo[a]) / m.h[a]);
        if (!(f >= 0.f) || !(f < (float)m.dims[a])) return false;
        idx[a] = (int)f;
    }
    const size_t cell = (((size_t)idx[0] * m.dims[1] + idx[1]) * m.dims[2] + idx[2]) * m.dims[3] + idx[3];
    return map[cell] != 0;
}

__device__ __forceinline__ float bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// One DPP move of v (lanes the pattern does not write keep v).
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), kCtrl, kRowMask, 0xf, false));
}

// Wave-wide max / min over all 64 lanes (call with every lane active), on the
// DPP network rather than LDS permutes: pairs and quads (quad_perm), half rows
// (row_half_mirror) and rows of 16 (row_mirror), then row 0 into row 1 and
// row 2 into row 3 (row_bcast:15), and row 1 into rows 2-3 (row_bcast:31);
// lane 63 then holds the result, returned to every lane.
template <bool kMax>
__device__ __forceinline__ float wave_extreme(float v) {
    auto op = [](float a, float b) { return kMax ? fmaxf(a, b) : fminf(a, b); };
    v = op(v, dpp_f<0xB1>(v));        // quad_perm [1, 0, 3, 2]
    v = op(v, dpp_f<0x4E>(v));        // quad_perm [2, 3, 0, 1]
    v = op(v, dpp_f<0x141>(v));       // row_half_mirror
    v = op(v, dpp_f<0x140>(v));       // row_mirror
    v = op(v, dpp_f<0x142, 0xA>(v));  // row_bcast:15 into rows 1 and 3
    v = op(v, dpp_f<0x143, 0xC>(v));  // row_bcast:31 into rows 2 and 3
    return bcast(v, kWave - 1);
}
__device__ __forceinline__ float wave_max(float v) { return wave_extreme<true>(v); }
__device__ __forceinline__ float wave_min(float v) { return wave_extreme<false>(v); }
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// ---------------------------------------------------------------------------
// Height map of a support (the learned proposal's state feature: one per
// support, over the boxes of the support's scene and the placed objects that
// rest on it): cell (ix, iy), ix along x in [0,64), iy along y,
// centre (-hx + (ix + 1/2) 2hx/64, -hy + ...); value = max(0, box tops, sphere
// tops) above the support plane, metres.  A box covers a cell when the cell
// centre at the box centre's height lies in the box's x/y extent (box frame);
// its top is the box's highest point.  A sphere (support-frame centre p,
// radius r) covers a cell when the cell centre is within r of p in x/y; its
// top there is p_z + sqrt(r^2 - d^2).
struct SupportFrame {
    float R[9], t[3], hx, hy;
};
__device__ __forceinline__ SupportFrame support_frame(const float* __restrict__ sup, int u) {
    SupportFrame F;
    const float* p = sup + 16 * (size_t)u;
    for (int i = 0; i < 9; ++i) F.R[i] = p[i];
    F.t[0] = p[9]; F.t[1] = p[10]; F.t[2] = p[11];
    F.hx = p[12]; F.hy = p[13];
    return F;
}
// world point -> support frame: R^T (p - t)
__device__ __forceinline__ void to_support(const SupportFrame& F, float x, float y, float z,
                                           float& sx, float& sy, float& sz) {
    const float dx = x - F.t[0], dy = y - F.t[1], dz = z - F.t[2];
    sx = F.R[0] * dx + F.R[3] * dy + F.R[6] * dz;
    sy = F.R[1] * dx + F.R[4] * dy + F.R[7] * dz;
    sz = F.R[2] * dx + F.R[5] * dy + F.R[8] * dz;
}
// Raise a scene's height map (64 x 64 floats at hm) by one world sphere:
// a monotone max through integer atomics on non-negative floats, so the
// result does not depend on the order of the spheres or of the callers.
// With a tile (T, an LDS window of tw x th cells from cell (tx0, ty0),
// i-major), cells inside the window are raised there and the rest in hm; the
// caller then raises hm by the window (hmap_flush_tile).  Every cell value is
// the same either way.
__device__ __forceinline__ void hmap_raise_sphere(const SupportFrame& F, float* __restrict__ hm,
                                                  float x, float y, float z, float r,
                                                  int* T = nullptr, int tx0 = 0, int ty0 = 0,
                                                  int tw = 0, int th = 0) {
    const float cw = 2.f * F.hx / 64.f, ch = 2.f * F.hy / 64.f;
    int* H = (int*)hm;
    float px, py, pz;
    to_support(F, x, y, z, px, py, pz);
    // cells whose centre can lie within r of (px, py)
    const int ix0 = max(0, (int)floorf((px - r + F.hx) / cw - 0.5f));
    const int ix1 = min(63, (int)ceilf((px + r + F.hx) / cw - 0.5f));
    const int iy0 = max(0, (int)floorf((py - r + F.hy) / ch - 0.5f));
    const int iy1 = min(63, (int)ceilf((py + r + F.hy) / ch - 0.5f));
    for (int ix = ix0; ix <= ix1; ++ix) {
        const float cx = -F.hx + (ix + 0.5f) * cw;
        for (int iy = iy0; iy <= iy1; ++iy) {
            const float cy = -F.hy + (iy + 0.5f) * ch;
            const float d2 = (cx - px) * (cx - px) + (cy - py) * (cy - py);
            if (d2 < r * r) {
                const float top = pz + sqrtf(r * r - d2);
                if (top > 0.f) {
                    const int wx = ix - tx0, wy = iy - ty0;
                    if ((unsigned)wx < (unsigned)tw && (unsigned)wy < (unsigned)th)
                        atomicMax(T + wx * th + wy, __float_as_int(top));
                    else
                        atomicMax(H + ix * 64 + iy, __float_as_int(top));
                }
            }
        }
    }
}

}  // namespace scn
