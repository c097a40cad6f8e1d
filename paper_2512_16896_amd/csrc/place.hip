// place.hip -- the persistent fused place kernel and its launcher.
//
// One workgroup of W waves owns scene s for the whole launch and places its
// objects one after another (the per-object rejection loop of the method).
// For one object the candidates of all attempts form one list in
// (attempt, index) order; the first collision-free entry of that list is the
// winner: the lowest index of the first attempt that has a collision-free
// candidate (retries only happen for a scene that found none).  Wave w walks
// the entries w, w+W, w+2W, ... in batches of 64:
//
//   batch phase (lane t <-> candidate t of the batch): the pose (Philox), the
//     world centre of the object's bounding sphere, two probe spheres tested
//     against a depth map of the placed spheres and against the boxes near
//     the bounding sphere (a probe that collides rejects its candidate), and
//     the bit mask of those near boxes (1-Lipschitz distance bounds: every
//     other box is farther than the margin from every sphere, exactly);
//   candidate phase (each candidate the batch phase left open, the object's
//     spheres across the lanes, SPL per lane): sphere tests against the boxes
//     of its mask, the depth map, and for each placed object whose bounding
//     sphere comes within reach a lane-parallel pretest of its placed
//     spheres followed by exact tests of the spheres that pass.  The
//     candidate is rejected at the first hit any lane reports (ballot).
//
// A collision-free candidate lowers the scene's best entry (LDS atomicMin);
// a wave stops once the best entry is below its next one, so every entry
// before the winner has been decided and the result is exactly the first
// collision-free one, whatever the number of waves.
#include <algorithm>
#include <climits>

#include "device.h"
#include "internal.h"

namespace scn {

// Object-object spatial relation of the object being placed (Sec. IV-F), set
// up once per object in LDS.  kind 1: the partial annulus around one anchor,
// sampled area-uniformly in the sector r^2 in [r0sq, r0sq + dr2], angle
// phi0 +- th; kind 2 ('middle'): the anchors' convex hull, sampled uniformly
// in the anchors' bounding box [lo, lo + d] and rejected outside the hull
// (edges (a, e): inside when cross(e, p - a) >= 0); kind -1: no valid region.
// Either kind rejects points outside the (eroded) support rectangle ax x ay.
// face_to turns the object's x axis to the first anchor.
struct RelState {
    int kind, face_to, nedge, pad;
    float a0x, a0y, r0sq, dr2, phi0, th;
    float lox, loy, dx, dy;
    float edge[8][4];
};

// Stable poses of the object being placed (kCons instances): its rows'
// cumulative weights, rotations and the lift that rests each turned sphere
// set on the support, staged in LDS by the object's setup.
struct StableTab {
    int n, r0;
    float cum[SCN_MAX_STABLE];
    float lift[SCN_MAX_STABLE];
    float R[SCN_MAX_STABLE][9];
};

// The stable-pose row (local index, -1 none) of the Philox word w3.
__device__ __forceinline__ int stable_row(const StableTab* st, uint32_t w3) {
    if (!st || st->n <= 0) return -1;
    const float u = unit01(w3);
    int m = 0;
    while (m < st->n - 1 && !(u <= st->cum[m])) ++m;
    return m;
}

// Relation sample from the candidate's Philox words: the pose (z = zc) and
// whether it lies in the relation's region.
__device__ __forceinline__ Pose relation_pose(const RelState& R, U4 w, float ax, float ay,
                                              float zc, bool* inside) {
    const float u0 = unit01(w.a), u1 = unit01(w.b), u2 = unit01(w.c);
    Pose p;
    bool in = R.kind > 0;
    if (R.kind == 1) {
        const float rr = sqrtf(fmaf(u0, R.dr2, R.r0sq));
        float sn, cs;
        sincosf(fmaf(R.th, fmaf(2.f, u1, -1.f), R.phi0), &sn, &cs);
        p.x = fmaf(rr, cs, R.a0x);
        p.y = fmaf(rr, sn, R.a0y);
    } else {
        p.x = fmaf(u0, R.dx, R.lox);
        p.y = fmaf(u1, R.dy, R.loy);
        for (int e = 0; e < R.nedge; ++e)
            in &= R.edge[e][2] * (p.y - R.edge[e][1]) - R.edge[e][3] * (p.x - R.edge[e][0]) >= 0.f;
    }
    in &= fabsf(p.x) <= ax && fabsf(p.y) <= ay;
    if (R.face_to) {
        const float fx = R.a0x - p.x, fy = R.a0y - p.y;
        const float n = sqrtf(fmaf(fx, fx, fy * fy));
        p.yaw = atan2f(fy, fx);
        p.c = n > 0.f ? fx / n : 1.f;
        p.s = n > 0.f ? fy / n : 0.f;
    } else {
        p.yaw = 6.28318530717958647692f * u2;
        sincospif(2.0f * u2, &p.s, &p.c);
    }
    p.z = zc;
    *inside = in;
    return p;
}

// Sets up the relation of object o (at position j of the scene whose first
// object is o0) from its row and its anchors' records; one thread.
__device__ void relation_setup(RelState& R, const float* __restrict__ row, int j, int o0,
                               const int32_t* __restrict__ obj_sup, int o,
                               const scn_pose_rec* __restrict__ rec, float ax, float ay) {
    R.kind = -1;
    R.face_to = ((int)row[15]) & 1;
    R.nedge = 0;
    const int kind = (int)row[0], n = (int)row[1];
    if (n < 1 || n > 8 || (kind != 1 && kind != 2)) return;
    float anc[8][2];
    for (int k = 0; k < n; ++k) {
        const int ja = (int)row[2 + k];
        if (ja < 0 || ja >= j || obj_sup[o0 + ja] != obj_sup[o]) return;
        anc[k][0] = rec[o0 + ja].x;
        anc[k][1] = rec[o0 + ja].y;
    }
    R.a0x = anc[0][0];
    R.a0y = anc[0][1];
    if (kind == 1) {
        float far = 0.f;
        for (int c = 0; c < 4; ++c) {
            const float cx = (c & 1 ? ax : -ax) - R.a0x, cy = (c & 2 ? ay : -ay) - R.a0y;
            far = fmaxf(far, sqrtf(fmaf(cx, cx, cy * cy)));
        }
        const float rmin = row[12], rmax = fminf(row[13], far);
        if (!(rmin < rmax)) return;
        const bool dir = row[10] != 0.f || row[11] != 0.f;
        R.th = dir ? fminf(row[14], 3.14159265358979323846f) : 3.14159265358979323846f;
        R.phi0 = dir ? atan2f(row[11], row[10]) : 0.f;
        R.r0sq = rmin * rmin;
        R.dr2 = rmax * rmax - R.r0sq;
        R.kind = 1;
        return;
    }
    if (n < 3) return;
    float lo[2] = {anc[0][0], anc[0][1]}, hi[2] = {anc[0][0], anc[0][1]};
    for (int k = 1; k < n; ++k)
        for (int d = 0; d < 2; ++d) {
            lo[d] = fminf(lo[d], anc[k][d]);
            hi[d] = fmaxf(hi[d], anc[k][d]);
        }
    R.lox = lo[0]; R.loy = lo[1];
    R.dx = hi[0] - lo[0]; R.dy = hi[1] - lo[1];
    // hull edges: (i, k) with every other anchor strictly to its left
    int ne = 0;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            if (i == k) continue;
            const float ex = anc[k][0] - anc[i][0], ey = anc[k][1] - anc[i][1];
            bool edge = true;
            for (int m = 0; m < n && edge; ++m)
                if (m != i && m != k &&
                    !(ex * (anc[m][1] - anc[i][1]) - ey * (anc[m][0] - anc[i][0]) > 0.f))
                    edge = false;
            if (edge && ne < 8) {
                R.edge[ne][0] = anc[i][0]; R.edge[ne][1] = anc[i][1];
                R.edge[ne][2] = ex; R.edge[ne][3] = ey;
                ++ne;
            }
        }
    R.nedge = ne;
    if (ne >= 3) R.kind = 2;
}

// Pose of entry g of an object's candidate list.  Entries 0..prop_k-1 are the
// learned proposal's bins in rank order: one pose drawn uniformly inside the
// bin (x cell, y cell, yaw cell of the 32 x 16 x 8 grid) with Philox counter
// (rank, 0x10000, j, s); the entries after them are the uniform attempts, entry
// prop_k + a C + i being candidate i of attempt a (counter (i, a, j, s)).
// With a stable-pose table (st), *row receives the candidate's row (fourth
// Philox word of its uniform counter; -1 without rows) and z adds that row's
// lift to zc.
__device__ __forceinline__ Pose entry_pose(int g, int prop_k, const int32_t* __restrict__ bins,
                                           int C, uint64_t seed, uint32_t s, uint32_t j, float ax,
                                           float ay, float zc, int* att, int* idx,
                                           const RelState* rs = nullptr, bool* inside = nullptr,
                                           const StableTab* st = nullptr, int* row = nullptr) {
    if (g < prop_k) {
        const int bin = min(max(bins[g], 0), 4095);
        const U4 w = philox10(U4{(uint32_t)g, 0x10000u, j, s}, (uint32_t)seed, (uint32_t)(seed >> 32));
        const float u0 = ((float)(bin >> 7) + unit01(w.a)) * (1.f / 32.f);
        const float u1 = ((float)((bin >> 3) & 15) + unit01(w.b)) * (1.f / 16.f);
        const float u2 = ((float)(bin & 7) + unit01(w.c)) * (1.f / 8.f);
        Pose p;
        p.x = ax * fmaf(2.f, u0, -1.f);
        p.y = ay * fmaf(2.f, u1, -1.f);
        p.yaw = 6.28318530717958647692f * u2;
        sincospif(2.0f * u2, &p.s, &p.c);
        p.z = zc;
        *att = -2;
        *idx = g;
        return p;
    }
    const int e = g - prop_k;
    const int a = e / C, i = e - a * C;
    *att = a;
    *idx = i;
    Pose p;
    uint32_t w3;
    if (rs) {
        const U4 w = philox10(U4{(uint32_t)i, (uint32_t)a, j, s}, (uint32_t)seed,
                              (uint32_t)(seed >> 32));
        p = relation_pose(*rs, w, ax, ay, zc, inside);
        w3 = w.d;
    } else {
        if (inside) *inside = true;
        p = sample_pose(seed, s, j, (uint32_t)a, (uint32_t)i, ax, ay, zc, &w3);
    }
    if (row) {
        *row = stable_row(st, w3);
        if (*row >= 0) p.z = zc + st->lift[*row];
    }
    return p;
}


__device__ __forceinline__ float4 bcast4(const float4& v, int lane) {
    return make_float4(bcast(v.x, lane), bcast(v.y, lane), bcast(v.z, lane), bcast(v.w, lane));
}

__device__ __forceinline__ unsigned long long bcast64(unsigned long long v, int lane) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// Depth map of a scene's placed spheres, in the frame of its (single) support:
// one int8 per voxel, a lower bound of how deep the voxel centre lies inside
// the placed spheres, max over spheres of r - |v - c| in steps of kMapQ, kept
// where it is >= -kMapReach (kMapNone elsewhere).  A probe sphere of radius rp
// centred at p in voxel v hits a placed sphere within the margin when
// depth(v) > |p - v| - rp - margin (kMapSafety more is asked): for the sphere
// that gives the depth, |p - c| <= |p - v| + |v - c| < rp + r + margin.
// Writes race without atomics: every value written is one sphere's depth, a
// valid lower bound, so a lost update only loses a rejection.  Distances use
// the hardware square root (within 1 ulp, ~1.2e-7 relative): below the
// quantisation slack of an insert (1e-3 of a step) for distances under 4 m,
// and far inside kMapSafety at any scale the map covers.
constexpr float kMapQ = 5e-4f;         // depth step (m)
constexpr float kMapReach = 0.04f;     // depths kept down to -4 cm (-80 steps)
constexpr float kMapSafety = 1e-4f;    // a rejection keeps this far inside the margin
constexpr int kMapNone = -128;
static_assert(kMapReach / kMapQ + 2.f < 128.f, "quantised depths must stay above kMapNone");
constexpr float kMapOver = 0.3f;       // mapped overhang beyond the support rectangle (m)
constexpr float kMapTop = 0.5f;        // mapped height above the support plane (m)

struct DepthMap {
    float x0, y0, h, inv_h;
    int nx, ny, nz;
};

// Voxel size: the smallest h >= 3 cm (in 5 % steps) whose grid over the
// rectangle grown by kMapOver and kMapTop of height fits kMapBytes.
__device__ __forceinline__ bool map_geometry(float ax, float ay, DepthMap& m) {
    const float ex = 2.f * (ax + kMapOver), ey = 2.f * (ay + kMapOver);
    if (!(ex > 0.f && ey > 0.f && ex < 1e4f && ey < 1e4f)) return false;
    float h = fmaxf(cbrtf(ex * ey * kMapTop / (float)kMapBytes), 0.03f);
    for (int it = 0; it < 64; ++it) {
        m.nx = (int)ceilf(ex / h);
        m.ny = (int)ceilf(ey / h);
        m.nz = (int)ceilf(kMapTop / h);
        if ((long long)m.nx * m.ny * m.nz <= kMapBytes) {
            m.h = h;
            m.inv_h = 1.f / h;
            m.x0 = -ax - kMapOver;
            m.y0 = -ay - kMapOver;
            return true;
        }
        h *= 1.05f;
    }
    return false;
}

// Adds a sphere (support frame): the voxels whose centres lie within
// r + kMapReach of its centre.  The caller writes the (i, j) columns c of the
// covering cube with c % parts == part; each column visits only the z range
// of that ball.
// The depth map's initial LDS contents: a copy of src (a map kept by an
// earlier launch) or empty (every voxel at the lowest depth).  16-byte words,
// eight loads in flight per thread before their stores, so a one-wave
// workgroup waits on three rounds of loads instead of one per word; the
// region ends on a 16-byte boundary inside kMapBytes.
static_assert(kMapBytes % 16 == 0 && kBoxLdsBytes % 16 == 0, "16-byte map words");
__device__ __forceinline__ void map_fill(int8_t* __restrict__ M, const DepthMap& m,
                                         const int8_t* __restrict__ src) {
    const int w16 = (m.nx * m.ny * m.nz + 15) >> 4;
    int4* mw = reinterpret_cast<int4*>(M);
    const int4* sw = reinterpret_cast<const int4*>(src);
    const int e = (int)0x80808080u;
    const int step = (int)blockDim.x;
    for (int i0 = (int)threadIdx.x; i0 < w16; i0 += 8 * step) {
        int4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * step;
            v[u] = src && i < w16 ? sw[i] : make_int4(e, e, e, e);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * step;
            if (i < w16) mw[i] = v[u];
        }
    }
}

__device__ __forceinline__ void map_insert(int8_t* __restrict__ M, const DepthMap& m, float cx,
                                           float cy, float cz, float r, int part, int parts) {
    if (!(fabsf(cx) < 1e4f && fabsf(cy) < 1e4f && fabsf(cz) < 1e4f && r >= 0.f && r < 1e3f)) return;
    const float e = r + kMapReach;
    const int i0 = max((int)floorf((cx - e - m.x0) * m.inv_h), 0);
    const int i1 = min((int)floorf((cx + e - m.x0) * m.inv_h), m.nx - 1);
    const int j0 = max((int)floorf((cy - e - m.y0) * m.inv_h), 0);
    const int j1 = min((int)floorf((cy + e - m.y0) * m.inv_h), m.ny - 1);
    const int k0 = max((int)floorf((cz - e) * m.inv_h), 0);
    const int k1 = min((int)floorf((cz + e) * m.inv_h), m.nz - 1);
    const int nxr = i1 - i0 + 1, nyr = j1 - j0 + 1;
    if (nxr <= 0 || nyr <= 0 || k1 < k0) return;
    static_assert(kMapBytes < 32768, "voxel indices of a cube must stay below 2^15");
    // c -> (i, j) by a float reciprocal: with c < 2^15 the quotient of
    // (c + 1/2) / nxr stays at least 1/(2 nxr) from an integer, far beyond
    // the rounding of the product, so the truncation is exact (and indices
    // below 2^15 make 24-bit multiplies exact)
    const int ncol = nxr * nyr;
    const float rx = 1.f / (float)nxr;
    const float e2 = e * e;
    for (int c = part; c < ncol; c += parts) {
        const int jj = (int)(((float)c + 0.5f) * rx);
        const int i = i0 + (c - __mul24(jj, nxr)), j = j0 + jj;
        const float dx = fmaf((float)i + 0.5f, m.h, m.x0) - cx;
        const float dy = fmaf((float)j + 0.5f, m.h, m.y0) - cy;
        const float dxy2 = fmaf(dx, dx, dy * dy);
        if (dxy2 > e2) continue;
        // voxel centres (k + 1/2) h within sqrt(e^2 - dxy2) of cz, widened by
        // one voxel each way (the depth test below decides)
        const float hz = __builtin_amdgcn_sqrtf(e2 - dxy2);
        const int ka = max((int)floorf((cz - hz) * m.inv_h - 0.5f), k0);
        const int kb = min((int)floorf((cz + hz) * m.inv_h - 0.5f) + 1, k1);
        int8_t* col = M + __mul24(j, m.nx) + i;
        const int plane = __mul24(m.ny, m.nx);
        // two z neighbours per step: both reads issue before either write
        // (different planes, so they never alias)
        for (int k = ka; k <= kb; k += 2) {
            const bool has1 = k + 1 <= kb;
            const float dz0 = ((float)k + 0.5f) * m.h - cz, dz1 = dz0 + m.h;
            const float d0 = r - __builtin_amdgcn_sqrtf(fmaf(dz0, dz0, dxy2));
            const float d1 = r - __builtin_amdgcn_sqrtf(fmaf(dz1, dz1, dxy2));
            int8_t* v0 = col + __mul24(k, plane);
            int8_t* v1 = has1 ? v0 + plane : v0;
            const int o0 = *v0, o1 = *v1;
            const int q0 = min((int)floorf(d0 * (1.f / kMapQ) - 1e-3f), 127);
            const int q1 = min((int)floorf(d1 * (1.f / kMapQ) - 1e-3f), 127);
            if (d0 >= -kMapReach && q0 > o0) *v0 = (int8_t)q0;
            if (has1 && d1 >= -kMapReach && q1 > o1) *v1 = (int8_t)q1;
        }
    }
}

__device__ __forceinline__ DepthMap map_params(const DepthMap* p) {
    const volatile DepthMap* v = p;
    DepthMap m;
    m.x0 = v->x0; m.y0 = v->y0; m.h = v->h; m.inv_h = v->inv_h;
    m.nx = v->nx; m.ny = v->ny; m.nz = v->nz;
    return m;
}

// True when a sphere of radius rp centred at (px, py, pz) (support frame)
// certainly comes within the margin of a mapped sphere.
__device__ __forceinline__ bool map_hit(const int8_t* __restrict__ M, const DepthMap& m, float px,
                                        float py, float pz, float rp, float margin) {
    const float fx = (px - m.x0) * m.inv_h, fy = (py - m.y0) * m.inv_h, fz = pz * m.inv_h;
    if (!(fx >= 0.f && fy >= 0.f && fz >= 0.f && fx < (float)m.nx && fy < (float)m.ny &&
          fz < (float)m.nz))
        return false;
    const int i = min((int)fx, m.nx - 1), j = min((int)fy, m.ny - 1), k = min((int)fz, m.nz - 1);
    const int q = M[__mul24(__mul24(k, m.ny) + j, m.nx) + i];
    if (q == kMapNone) return false;
    const float dx = fmaf((float)i + 0.5f, m.h, m.x0) - px;
    const float dy = fmaf((float)j + 0.5f, m.h, m.y0) - py;
    const float dz = ((float)k + 0.5f) * m.h - pz;
    const float dv = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    return (float)q * kMapQ > dv - rp - margin + kMapSafety;
}

// Constants of an object that depend on its sphere set only: the centre bc
// of the spheres' bounding box, the radius rho of the bounding sphere about
// bc, the lift that rests the lowest point on the support, and the probes.
// One wave computes them (all 64 lanes active).
struct ObjConsts {
    float bc[3], rho, lift;
    float4 probe, probe2;
    bool two;
};

template <int SPL, bool kProbe2>
__device__ __forceinline__ ObjConsts object_consts(const float4* __restrict__ tmpl, int sb, int S,
                                                   int lane) {
    ObjConsts K;
    float cx[SPL], cy[SPL], cz[SPL], cr[SPL];
    bool act[SPL];
    float lift = -1e30f, lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
        const int k = lane + kWave * q;
        act[q] = k < S;
        const float4 c = act[q] ? tmpl[sb + k] : make_float4(0.f, 0.f, 0.f, 0.f);
        cx[q] = c.x; cy[q] = c.y; cz[q] = c.z; cr[q] = c.w;
        if (act[q]) {
            lift = fmaxf(lift, c.w - c.z);
            lo[0] = fminf(lo[0], c.x - c.w); hi[0] = fmaxf(hi[0], c.x + c.w);
            lo[1] = fminf(lo[1], c.y - c.w); hi[1] = fmaxf(hi[1], c.y + c.w);
            lo[2] = fminf(lo[2], c.z - c.w); hi[2] = fmaxf(hi[2], c.z + c.w);
        }
    }
    K.lift = wave_max(lift);
#pragma unroll
    for (int d = 0; d < 3; ++d) K.bc[d] = 0.5f * (wave_min(lo[d]) + wave_max(hi[d]));
    float rho = 0.f;
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
        if (act[q]) {
            const float dx = cx[q] - K.bc[0], dy = cy[q] - K.bc[1], dz = cz[q] - K.bc[2];
            rho = fmaxf(rho, sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))) + cr[q]);
        }
    }
    K.rho = wave_max(rho) * (1.0f + 1e-6f) + 1e-6f;
    // Probe: the object's largest sphere (the lowest index among equals).
    // A candidate whose probe already comes within the margin of a box, a grid
    // or the depth map collides, and the batch phase settles that for 64
    // candidates at once with the same arithmetic as the full test of that
    // sphere.
    K.probe = make_float4(0.f, 0.f, 1e18f, 0.f);
    if (S > 0) {
        float rmax = -1.f;
#pragma unroll
        for (int q = 0; q < SPL; ++q)
            if (act[q]) rmax = fmaxf(rmax, cr[q]);
        rmax = wave_max(rmax);
        int kp = 0;
#pragma unroll
        for (int q = SPL - 1; q >= 0; --q) {   // the lowest slot with a hit wins
            const unsigned long long m = __ballot(act[q] && cr[q] == rmax);
            if (m) kp = kWave * q + __builtin_ctzll(m);
        }
        K.probe = tmpl[sb + uniform_int(kp)];
    }
    // A second probe on the far side: the largest sphere (lowest index among
    // equals) farther from the first probe than half the farthest sphere.
    K.probe2 = K.probe;
    K.two = false;
    if (kProbe2 && S > 1) {
        const float4 p = K.probe;
        auto d1 = [&](int q) {
            const float dx = cx[q] - p.x, dy = cy[q] - p.y, dz = cz[q] - p.z;
            return sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        };
        float dfar = 0.f;
#pragma unroll
        for (int q = 0; q < SPL; ++q)
            if (act[q]) dfar = fmaxf(dfar, d1(q));
        dfar = 0.5f * wave_max(dfar);
        float r2 = -1.f;
#pragma unroll
        for (int q = 0; q < SPL; ++q)
            if (act[q] && d1(q) > dfar) r2 = fmaxf(r2, cr[q]);
        r2 = wave_max(r2);
        if (r2 >= 0.f) {
            int kp = 0;
#pragma unroll
            for (int q = SPL - 1; q >= 0; --q) {
                const unsigned long long m = __ballot(act[q] && d1(q) > dfar && cr[q] == r2);
                if (m) kp = kWave * q + __builtin_ctzll(m);
            }
            K.probe2 = tmpl[sb + uniform_int(kp)];
            K.two = true;
        }
    }
    return K;
}

// Boxes (of the first 64) that some candidate of an object can reach: every
// candidate's bounding centre lies, in the support frame, on the rectangle
// grown by |bc_xy| at height bc_z + zc; a box whose bounding sphere stays
// farther than reach from that set is skipped by the batch phase.
__device__ __forceinline__ unsigned long long reachable_boxes(const ObjConsts& K, const Support& U,
                                                              float reach,
                                                              const float* __restrict__ box,
                                                              int b0, int nbox_mask, int lane) {
    const float ax = U.hx - U.inset, ay = U.hy - U.inset, zc = U.lift + K.lift;
    const float gx = ax + sqrtf(fmaf(K.bc[0], K.bc[0], K.bc[1] * K.bc[1]));
    const float gy = ay + sqrtf(fmaf(K.bc[0], K.bc[0], K.bc[1] * K.bc[1]));
    const float hz = K.bc[2] + zc;
    bool rel = false;
    if (lane < nbox_mask) {
        const float* B = box + 16 * (b0 + lane);
        const float dx = B[9] - U.t[0], dy = B[10] - U.t[1], dz = B[11] - U.t[2];
        const float sx = fmaf(U.R[0], dx, fmaf(U.R[3], dy, U.R[6] * dz));
        const float sy = fmaf(U.R[1], dx, fmaf(U.R[4], dy, U.R[7] * dz));
        const float sz = fmaf(U.R[2], dx, fmaf(U.R[5], dy, U.R[8] * dz));
        const float ox = fmaxf(fabsf(sx) - gx, 0.f), oy = fmaxf(fabsf(sy) - gy, 0.f);
        const float oz = sz - hz;
        const float lim = sqrtf(fmaf(B[12], B[12], fmaf(B[13], B[13], B[14] * B[14]))) + reach;
        // generous slack for the rounding of this test (it only prunes)
        rel = fmaf(ox, ox, fmaf(oy, oy, oz * oz)) < lim * lim * 1.0001f + 1e-6f;
    }
    return __ballot(rel);
}

// the kernel's static shared variables (s_best, s_found, s_dm, s_rel,
// s_stab) within the reserve the planner leaves beside the dynamic LDS
static_assert(sizeof(int) + 16 * 9 * sizeof(float) + sizeof(DepthMap) + sizeof(RelState) +
                  sizeof(StableTab) + 64 <= kPlaceStaticLds,
              "static LDS of the place kernel exceeds its reserve");

// The 4 constants the place kernel keeps per object to place (written by
// lane 0 to I[0..3]): bounding centre and radius, the two probes, and the
// lift, flags (second probe; non-finite template or support) and the mask of
// the scene's first 64 boxes some candidate can reach.  One wave per object.
template <int SPL, bool kProbe2>
__device__ __forceinline__ void object_info(const float4* __restrict__ tmpl,
                                            const int32_t* __restrict__ sph_off,
                                            const int32_t* __restrict__ obj_sup,
                                            const float* __restrict__ sup,
                                            const float* __restrict__ box, int o, int b0,
                                            int nbox_mask, float margin, int lane, float4* I) {
    const int sb = sph_off[o];
    const ObjConsts K = object_consts<SPL, kProbe2>(tmpl, sb, sph_off[o + 1] - sb, lane);
    const Support U = load_support(sup, obj_sup[o]);
    // a non-finite template sphere or support entry: every candidate of the
    // object collides
    bool fin_ok = lane < 16 ? __builtin_isfinite(sup[16 * obj_sup[o] + lane]) : true;
    for (int k = sb + lane; k < sph_off[o + 1]; k += kWave) fin_ok &= finite4(tmpl[k]);
    const bool obj_bad = __ballot(!fin_ok) != 0;
    const unsigned long long rel = reachable_boxes(K, U, K.rho + margin, box, b0, nbox_mask, lane);
    if (lane == 0) {
        I[0] = make_float4(K.bc[0], K.bc[1], K.bc[2], K.rho);
        I[1] = K.probe;
        I[2] = K.probe2;
        I[3] = make_float4(K.lift, __int_as_float((K.two ? 1 : 0) | (obj_bad ? 2 : 0)),
                           __int_as_float((int)(unsigned)rel),
                           __int_as_float((int)(unsigned)(rel >> 32)));
    }
}

// kLds = true : the scene's placed spheres live in LDS (cap_sph of them);
//               with `split`, scenes with more spheres are left to the
//               other launch, otherwise they are a capacity error.
// kLds = false: placed spheres are read from global memory (L1/L2) and only
//               the object bounds live in LDS; with `split`, scenes of at
//               most split_sph spheres are left to the LDS launch.
// kGrids: the batch has voxel-grid furniture (the grid code is compiled out
// otherwise, which keeps the register count of grid-free launches low).
// kYaw: the batch declares SCN_GEOM_YAW (supports and boxes turn about z
// only); candidate transforms and box tests take their planar form (4 instead
// of 14 instructions per sphere transform, 5 fewer per box test). A scene
// that breaks the declaration is marked invalid with kErrGeometry.
// The kernel's parameters, shared by the two entry points below.
#define SCN_PLACE_PARAMS     const int32_t* __restrict__ obj_off, const int32_t* __restrict__ sph_off, \
    const float4* __restrict__ tmpl, const int32_t* __restrict__ obj_sup, \
    const int32_t* __restrict__ obj_ncand, const float* __restrict__ sup, \
    const int32_t* __restrict__ box_off, const float* __restrict__ box, \
    float4* __restrict__ placed, int32_t* __restrict__ n_placed, int8_t* __restrict__ status, \
    scn_pose_rec* __restrict__ rec, int32_t* __restrict__ chosen, \
    unsigned long long* __restrict__ counters, const int32_t* __restrict__ order, \
    const int32_t* __restrict__ n_order, uint64_t seed, \
    float margin, int retries, int default_ncand, int max_steps, int cap_sph, int cap_obj, \
    int split, int split_sph, const int32_t* __restrict__ prop_bins, int prop_k, \
    int32_t* __restrict__ resume, int chunk, int j_cap, int32_t* __restrict__ n_active, \
    const int32_t* __restrict__ grid_off, const float* __restrict__ grid, \
    const int32_t* __restrict__ grid_src, const int64_t* __restrict__ grid_val_off, \
    const float* __restrict__ grid_val, const int32_t* __restrict__ obj_rel, \
    const float* __restrict__ rel, const float* __restrict__ obj_ratio, \
    const float* __restrict__ robot, const float* __restrict__ obj_reach, scn_reach_map rmap, \
    int8_t* __restrict__ map_keep, float4* __restrict__ bnd_keep, const float4* __restrict__ info_keep, \
    float* __restrict__ hmap, const int32_t* __restrict__ pose_off, \
    const float* __restrict__ stable, int32_t* __restrict__ rec_stable
#define SCN_PLACE_ARGS \
    obj_off, sph_off, tmpl, obj_sup, obj_ncand, sup, box_off, box, placed, n_placed, status, rec, chosen, counters, order, n_order, seed, margin, retries, default_ncand, max_steps, cap_sph, cap_obj, split, split_sph, prop_bins, prop_k, resume, chunk, j_cap, n_active, \
    grid_off, grid, grid_src, grid_val_off, grid_val, obj_rel, rel, obj_ratio, robot, obj_reach, \
    rmap, map_keep, bnd_keep, info_keep, hmap, pose_off, stable, rec_stable

// kHmap: instances of the learned launches, which raise the height map of the
// object's support at each commit (placed spheres in global memory, no
// constraints)
template <int SPL, bool kLds, bool kGrids, bool kYaw, bool kCons, bool kHmap = false>
__device__ __forceinline__ void place_scenes(SCN_PLACE_PARAMS) {
    static_assert(!kHmap || (!kLds && !kCons), "height-map instances keep spheres in global memory");
    // placed objects covered by a candidate's object mask: 64 per word; the
    // dense multi-shelf (grid) scenes carry 100 objects, so they get two words
    constexpr int kObjWords = kGrids ? 2 : 1;
    extern __shared__ float4 lds[];
    float4* lsph = lds;                        // placed spheres: (x, y, z, r + margin)
    float4* lbnd = lds + (kLds ? cap_sph : 0); // world bounding sphere of each placed object
    // per object to place: 4 constants (bounds, probes, lift and flags)
    // (a launch that places at most max_steps objects keeps that many)
    float4* linfo = lbnd + cap_obj;
    const int n_info = max_steps > 0 ? min(cap_obj, max_steps) : cap_obj;
    // the rows of the scene's first 64 boxes (kBoxLdsBytes)
    // per object the launch may place: first template sphere, sphere count,
    // candidates per attempt and support, staged once so that an object's
    // start reads them from LDS instead of through a chain of scalar loads
    int4* lobj = reinterpret_cast<int4*>(linfo + 4 * n_info);
    float* lbox = reinterpret_cast<float*>(lobj + n_info);
    // scenes without grids: the depth map after them (kMapBytes)
    constexpr bool kMap = !kGrids;
    int8_t* lmap = reinterpret_cast<int8_t*>(lbox) + kBoxLdsBytes;
    __shared__ int s_best;
    // the pose of the entry each wave found valid (a wave finds at most one
    // per object): x, y, z, c, s, yaw, attempt, index, stable-pose row
    __shared__ float s_found[16][9];
    __shared__ DepthMap s_dm;   // read where used (volatile), not held in registers
    __shared__ RelState s_rel;  // the current object's spatial relation
    __shared__ StableTab s_stab;  // the current object's stable poses

    // with n_order, only the first *n_order entries of `order` are scenes of
    // this launch (a list compacted on the device); the other workgroups leave.
    // The scene's header words are read up front, so that these independent
    // loads are in flight together instead of costing a round trip each.
    const int n_live = n_order ? *n_order : INT_MAX;
    const int s = order ? order[blockIdx.x] : (int)blockIdx.x;
    if ((int)blockIdx.x >= n_live) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform_int(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;

    const int o0 = obj_off[s], o1 = obj_off[s + 1];
    const int8_t status0 = status[s];
    const int placed0 = n_placed[s];
    const int resume_s = resume ? resume[s] : 0;
    const int b0 = box_off[s], b1 = box_off[s + 1];
    const int g0 = grid_off ? grid_off[s] : 0;
    const int g1 = grid_off ? grid_off[s + 1] : 0;
    const int nobj = o1 - o0;
    const int first = sph_off[o0];
    const int nsph = sph_off[o1] - first;
    if (split) {   // which of the two launches owns this scene
        if (kLds ? nsph > split_sph : nsph <= split_sph) return;
    }
    if (status0 != SCN_SCENE_ACTIVE) {
        if (chosen && threadIdx.x == 0) chosen[s] = -2;
        return;
    }
    // (every wave checks every object: no barrier, and the same answer in
    // each wave)
    int too_big = 0;
    for (int ob = o0 + lane; ob < o1; ob += kWave)
        too_big |= (sph_off[ob + 1] - sph_off[ob]) > kWave * SPL;
    too_big = __ballot(too_big) != 0;
    if (too_big || (kLds && nsph > cap_sph) || nobj > cap_obj) {
        if (threadIdx.x == 0) {
            atomicOr(counters + kErrorWord, (unsigned long long)kErrCapacity);
            if (chosen) chosen[s] = -2;
        }
        return;
    }
    int j = min(max(placed0, 0), nobj);
    int j_end = max_steps > 0 ? min(nobj, j + max_steps) : nobj;
    if (j_cap > 0) j_end = min(j_end, j_cap);
    if (j >= j_end && j < nobj) {   // the objects-per-scene cap stops this scene
        if (chosen && threadIdx.x == 0) chosen[s] = -1;
        return;
    }
    // entry of the current object's list to resume at (learned path)
    const int resume0 = max(resume_s, 0);
    const int j_start = j;
    int pend = 0;
    // placed sphere k of this scene, radius grown by the margin
    auto placed_sphere = [&](int k) -> float4 {
        if constexpr (kLds) {
            return lsph[k];
        } else {
            float4 q = placed[first + k];
            q.w += margin;
            return q;
        }
    };

    // Stage the already placed spheres and their objects' bounding spheres.
    const int n_stage = kLds ? sph_off[o0 + j] - first : 0;
    for (int i = threadIdx.x; i < n_stage; i += blockDim.x) {
        float4 q = placed[first + i];
        q.w += margin;
        lsph[i] = q;
    }
    // (with bnd_keep the bounding spheres recorded when each was placed)
    if (bnd_keep)
        for (int ob = threadIdx.x; ob < j; ob += blockDim.x) lbnd[ob] = bnd_keep[o0 + ob];
    for (int ob = bnd_keep ? j : wave; ob < j; ob += W) {
        const int a0 = sph_off[o0 + ob] - first, a1 = sph_off[o0 + ob + 1] - first;
        float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
        for (int k = a0 + lane; k < a1; k += kWave) {
            const float4 q = placed[first + k];
            lo[0] = fminf(lo[0], q.x - q.w); hi[0] = fmaxf(hi[0], q.x + q.w);
            lo[1] = fminf(lo[1], q.y - q.w); hi[1] = fmaxf(hi[1], q.y + q.w);
            lo[2] = fminf(lo[2], q.z - q.w); hi[2] = fmaxf(hi[2], q.z + q.w);
        }
        float c[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) c[d] = 0.5f * (wave_min(lo[d]) + wave_max(hi[d]));
        float rho = 0.f;
        for (int k = a0 + lane; k < a1; k += kWave) {
            const float4 q = placed[first + k];
            const float dx = q.x - c[0], dy = q.y - c[1], dz = q.z - c[2];
            rho = fmaxf(rho, sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))) + q.w);
        }
        rho = wave_max(rho) * (1.0f + 1e-6f) + 1e-6f;
        if (lane == 0) lbnd[ob] = make_float4(c[0], c[1], c[2], rho);
    }
    // Depth map: when every object of the scene rests on one support, in that
    // support's frame; cleared, then filled with the spheres already placed
    // (their support-frame centres from the world ones)
    bool use_map = false;
    if constexpr (kMap) {
        DepthMap dm{};
        int other = 0;
        for (int ob = o0 + (int)threadIdx.x; ob < o1; ob += blockDim.x)
            other |= obj_sup[ob] != obj_sup[o0];
        use_map = nobj > 0 && !__syncthreads_or(other);
        if (use_map) {
            const Support U0 = load_support(sup, obj_sup[o0]);
            use_map = map_geometry(U0.hx - U0.inset, U0.hy - U0.inset, dm);
            if (use_map) {
                if (threadIdx.x == 0) s_dm = dm;
                const int n_old = sph_off[o0 + j] - first;
                // with map_keep, the map the launch that placed the scene's
                // last object stored (every placing launch stores it)
                const bool kept = map_keep && j > 0;
                map_fill(lmap, dm, kept ? map_keep + (size_t)s * kMapBytes : nullptr);
                __syncthreads();
                for (int i = kept ? n_old : (int)threadIdx.x; i < n_old; i += blockDim.x) {
                    const float4 q = placed[first + i];
                    const float dx = q.x - U0.t[0], dy = q.y - U0.t[1], dz = q.z - U0.t[2];
                    map_insert(lmap, dm, fmaf(U0.R[0], dx, fmaf(U0.R[3], dy, U0.R[6] * dz)),
                               fmaf(U0.R[1], dx, fmaf(U0.R[4], dy, U0.R[7] * dz)),
                               fmaf(U0.R[2], dx, fmaf(U0.R[5], dy, U0.R[8] * dz)), q.w, 0, 1);
                }
            }
        }
    }
    __syncthreads();

    unsigned long long n_cand = 0, n_pairs = 0, n_boxp = 0, n_att = 0, n_done = 0, n_xf = 0;
    unsigned long long n_boxc = 0, n_objc = 0, n_sphc = 0, n_grid = 0;
    unsigned lane_boxp = 0;   // per-lane share of n_boxp
    int8_t fin = SCN_SCENE_ACTIVE;
    int last = -2;
    const int nbox_mask = min(b1 - b0, kWave);   // boxes covered by the batch masks
    // the first 64 box rows into LDS: the batch and candidate phases read
    // them there (the barrier below publishes them)
    for (int i = threadIdx.x; i < 16 * nbox_mask; i += blockDim.x) lbox[i] = box[16 * b0 + i];
    // Constants of every object this launch may place, once per scene with the
    // objects spread over the waves; the loads and reductions of different
    // objects overlap here instead of stalling each object's start.
    // A second probe is not used in grid batches: their placements rarely
    // collide, and its registers would cost occupancy.
    // With info_keep (computed once per generation by k_object_info) they
    // are only copied.
    for (int jj = j + (int)threadIdx.x; jj < j_end; jj += blockDim.x) {
        const int oo = o0 + jj, a = sph_off[oo];
        lobj[jj - j] = make_int4(a, sph_off[oo + 1] - a, obj_ncand ? obj_ncand[oo] : default_ncand,
                                 obj_sup[oo]);
    }
    if (info_keep) {
        for (int i = threadIdx.x; i < 4 * (j_end - j); i += blockDim.x)
            linfo[i] = info_keep[4 * (size_t)(o0 + j) + i];
    } else {
        for (int jj = j + wave; jj < j_end; jj += W)
            object_info<SPL, !kGrids>(tmpl, sph_off, obj_sup, sup, box, o0 + jj, b0, nbox_mask,
                                      margin, lane, linfo + 4 * (jj - j));
    }
    // the scene's boxes all turn about z only (then, with a support that does
    // too, the entry loop runs its planar form); each wave reads every row
    const int ngrid_mask = kGrids ? min(g1 - g0, kWave) : 0;   // grids covered by the masks
    int tilted = 0, bad_in = 0;
    for (int bi = b0 + lane; bi < b1; bi += kWave) {
        tilted |= !yaw_box(box + 16 * bi);
        bad_in |= !all_finite(box + 16 * bi, 15);
    }
    // non-finite input the whole scene is tested against (box rows, grid
    // instance rows, spheres placed before this launch): every candidate of
    // every remaining object collides
    if constexpr (kGrids)
        for (int gi = g0 + lane; gi < g1; gi += kWave) bad_in |= !all_finite(grid + 24 * gi, 19);
    const bool boxes_yaw = __ballot(tilted) == 0;
    const bool rows_bad = __ballot(bad_in) != 0;
    // (with bnd_keep every placed sphere comes from an earlier launch of the
    // same generation, which placed it only from a finite template, support
    // and pose); the barrier also publishes the box rows and object constants
    bool scene_bad = rows_bad;
    if (bnd_keep) {
        __syncthreads();
    } else {
        int bad_placed = 0;
        for (int i = threadIdx.x; i < sph_off[o0 + j] - first; i += blockDim.x)
            bad_placed |= !finite4(placed[first + i]);
        scene_bad = (__syncthreads_or(bad_placed) != 0) || rows_bad;
    }

    for (; j < j_end; ++j) {
        const int o = o0 + j;
        const int4 od = lobj[j - j_start];
        const int sb = uniform_int(od.x);
        const int S = uniform_int(od.y);
        const int osup = uniform_int(od.w);
        const int nq = (S + kWave - 1) / kWave;   // sphere slots per lane this object uses
        float cx[SPL], cy[SPL], cz[SPL], cr[SPL], rm2[SPL];
        bool act[SPL];
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            const int k = lane + kWave * q;
            act[q] = k < S;
            // Lanes without a sphere carry a zero-radius point 1e18 m up the
            // object's z axis: rigid motions keep it ~1e18 m from everything,
            // so it never tests as a hit and needs no predicate in the loops.
            const float4 c = act[q] ? tmpl[sb + k] : make_float4(0.f, 0.f, 1e18f, 0.f);
            cx[q] = c.x; cy[q] = c.y; cz[q] = c.z; cr[q] = c.w;
            rm2[q] = act[q] ? (c.w + margin) * (c.w + margin) : 0.f;
        }
        // the object's constants, computed in the prologue
        const float4* I = linfo + 4 * (j - j_start);
        const float4 I0 = I[0], I1 = I[1], I2 = I[2], I3 = I[3];
        const float bc[3] = {uniform_f(I0.x), uniform_f(I0.y), uniform_f(I0.z)};
        const float rho = uniform_f(I0.w);
        const float reach = rho + margin;
        const float4 probe = make_float4(uniform_f(I1.x), uniform_f(I1.y), uniform_f(I1.z), uniform_f(I1.w));
        const float4 probe2 = make_float4(uniform_f(I2.x), uniform_f(I2.y), uniform_f(I2.z), uniform_f(I2.w));
        const float lift = uniform_f(I3.x);
        const int oflags = uniform_int(__float_as_int(I3.y));
        const bool two = (oflags & 1) != 0;
        // stable-pose rows of the object (kCons instances)
        int nstab = 0;
        if constexpr (kCons) {
            if (pose_off) nstab = uniform_int(pose_off[o + 1] - pose_off[o]);
        }
        // boxes some candidate can reach (the mask assumes the unturned set:
        // every box for an object with stable poses)
        const unsigned long long box_rel =
            nstab > 0 ? (nbox_mask == kWave ? ~0ull : (1ull << nbox_mask) - 1ull)
                      : (((unsigned long long)(unsigned)uniform_int(__float_as_int(I3.w)) << 32) |
                         (unsigned)uniform_int(__float_as_int(I3.z)));
        const float prm2 = (probe.w + margin) * (probe.w + margin);
        const float prm2b = (probe2.w + margin) * (probe2.w + margin);

        const Support U = load_support(sup, osup);
        // ratio_on_support (Sec. IV-F): the support eroded by ratio x half
        // the shorter x / y extent of the object's sphere set
        float ero = 0.f;
        if (obj_ratio) {
            const float ratio = obj_ratio[o];
            if (ratio > 0.f) {
                float lx0 = 1e30f, hx0 = -1e30f, ly0 = 1e30f, hy0 = -1e30f;
#pragma unroll
                for (int q = 0; q < SPL; ++q)
                    if (act[q]) {
                        lx0 = fminf(lx0, cx[q] - cr[q]); hx0 = fmaxf(hx0, cx[q] + cr[q]);
                        ly0 = fminf(ly0, cy[q] - cr[q]); hy0 = fmaxf(hy0, cy[q] + cr[q]);
                    }
                const float ex = wave_max(hx0) - wave_min(lx0), ey = wave_max(hy0) - wave_min(ly0);
                ero = ratio * 0.5f * fminf(ex, ey);
            }
        }
        // z of the object's frame: the support's lift plus the rest lift of
        // the sphere set (with stable poses, the row's lift is added per
        // candidate)
        const float ax = U.hx - U.inset - ero, ay = U.hy - U.inset - ero;
        const float zc = U.lift + (nstab > 0 ? 0.f : lift);
        // spatial relations and reachability: instances for batches that
        // have them (kCons)
        const RelState* rs = nullptr;
        float reach_theta = -1.f;
        if constexpr (kCons) {
            const int rel_row = obj_rel ? obj_rel[o] : -1;
            if (rel_row >= 0 && threadIdx.x == 0)
                relation_setup(s_rel, rel + 16 * rel_row, j, o0, obj_sup, o, rec, ax, ay);
            if (rel_row >= 0) rs = &s_rel;
            if (robot && obj_reach) reach_theta = obj_reach[o];
        }
        // the object's stable poses: rotations, cumulative weights and the
        // lift of each turned sphere set (wave 0; the barrier before the
        // entry loop publishes them)
        const StableTab* st = nullptr;
        if constexpr (kCons) {
            if (nstab > SCN_MAX_STABLE) {   // more rows than the table holds
                if (threadIdx.x == 0) {
                    atomicOr(counters + kErrorWord, (unsigned long long)kErrCapacity);
                    if (chosen) chosen[s] = -2;
                }
                fin = SCN_SCENE_INVALID;
                last = -1;
                break;
            }
            if (nstab > 0) {
                if (wave == 0) {
                    const int r0 = pose_off[o];
                    for (int m = 0; m < nstab; ++m) {
                        const float* R = stable + 12 * (r0 + m);
                        float l = -__builtin_huge_valf();
#pragma unroll
                        for (int q = 0; q < SPL; ++q) {
                            if (act[q]) {
                                float x, y, z;
                                rest_point(R, cx[q], cy[q], cz[q], x, y, z);
                                l = fmaxf(l, cr[q] - z);
                            }
                        }
                        l = wave_max(l);
                        if (lane < 9) s_stab.R[m][lane] = R[lane];
                        if (lane == 0) {
                            s_stab.lift[m] = l;
                            s_stab.cum[m] = R[9];
                        }
                    }
                    if (lane == 0) {
                        s_stab.n = nstab;
                        s_stab.r0 = r0;
                    }
                }
                st = &s_stab;
            }
        }
        // planar form: supports and boxes turn about z only; world z of each
        // sphere, of the bounding centre and of the probe is then the same
        // for every candidate
        if (scene_bad || (oflags & 2)) {   // non-finite input: every candidate collides
            if (threadIdx.x == 0) {
                atomicOr(counters + kErrorWord, (unsigned long long)kErrNonFinite);
                atomicAdd(counters + kNonFinite, 1ull);
            }
            fin = SCN_SCENE_INVALID;
            last = -1;
            break;
        }
        if (kYaw && !(boxes_yaw && yaw_support(U))) {   // breaks the declared geometry
            if (threadIdx.x == 0) atomicOr(counters + kErrorWord, (unsigned long long)kErrGeometry);
            fin = SCN_SCENE_INVALID;
            last = -1;
            break;
        }
        float wz0[SPL];
#pragma unroll
        for (int q = 0; q < SPL; ++q) wz0[q] = (cz[q] + zc) + U.t[2];
        const float bz0 = (bc[2] + zc) + U.t[2], pz0 = (probe.z + zc) + U.t[2];
        const float pz02 = (probe2.z + zc) + U.t[2];
        const int C = uniform_int(od.z);
        // proposals of this scene (only when it has them this step)
        const int pk = prop_bins ? prop_k : 0;
        const int32_t* pb = prop_bins ? prop_bins + (size_t)s * prop_k : nullptr;
        const int total = pk + (C > 0 ? (retries + 1) * C : 0);   // entries of the list
        // entries [g_lo, g_hi) of the list are tried in this launch: with a
        // chunk, the proposals plus `chunk` uniform entries, then `chunk` more
        // per launch (chunk < 0: the proposals alone, then the uniform entries
        // from a later launch); earlier launches found none of the entries
        // before g_lo valid, so the lowest valid entry of [g_lo, g_hi) is the
        // first valid one of the whole list
        const int g_lo = j == j_start ? min(resume0, total) : 0;
        const int g_hi = chunk != 0 ? min(total, max(g_lo, pk) + max(chunk, 0)) : total;
        const int nob_mask = min(j, kWave * kObjWords);     // objects covered by the masks

        if (threadIdx.x == 0) s_best = INT_MAX;
        __syncthreads();

        // Exact sphere tests of the candidate (spheres wx/wy/wz in the lanes)
        // against placed object ob; true when a lane hit.
        float wx[SPL], wy[SPL], wz[SPL];
        float Gx = 0.f, Gy = 0.f, Gz = 0.f;
        auto test_object = [&](int ob, bool& hit) {
            const int a0 = sph_off[o0 + ob] - first, a1 = sph_off[o0 + ob + 1] - first;
            for (int c0 = a0; c0 < a1; c0 += kWave) {
                // lane-parallel pretest of up to 64 placed spheres; the pair
                // loop then takes each sphere from the lane that loaded it
                bool rel = false;
                float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
                if (c0 + lane < a1) {
                    q = placed_sphere(c0 + lane);
                    const float dx = q.x - Gx, dy = q.y - Gy, dz = q.z - Gz;
                    const float lim = rho + q.w;
                    rel = fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < lim * lim;
                }
                unsigned long long rm = __ballot(rel);
                n_sphc += (unsigned long long)min(kWave, a1 - c0);
                while (rm) {
                    const int l0 = __builtin_ctzll(rm);
                    rm &= rm - 1;
                    int l1 = l0;
                    if (rm) {
                        l1 = __builtin_ctzll(rm);
                        rm &= rm - 1;
                    }
                    const int k0 = c0 + l0, k1 = c0 + l1;
                    const float4 qa = bcast4(q, l0), qb = bcast4(q, l1);
                    float m = __builtin_huge_valf();
#pragma unroll
                    for (int q = 0; q < SPL; ++q) {
                        if (q > 0 && q >= nq) break;
                        {
                            const float ex = wx[q] - qa.x, ey = wy[q] - qa.y, ez = wz[q] - qa.z;
                            const float rr = cr[q] + qa.w;
                            m = fminf(m, fmaf(-rr, rr, fmaf(ex, ex, fmaf(ey, ey, ez * ez))));
                        }
                        {
                            const float ex = wx[q] - qb.x, ey = wy[q] - qb.y, ez = wz[q] - qb.z;
                            const float rr = cr[q] + qb.w;
                            m = fminf(m, fmaf(-rr, rr, fmaf(ex, ex, fmaf(ey, ey, ez * ez))));
                        }
                    }
                    hit |= m < 0.f;
                    n_pairs += (unsigned long long)S * (k1 != k0 ? 2u : 1u);
                    if (__ballot(hit)) return;
                }
            }
        };

        bool stop = false;
        for (int base = 0; !stop; base += kWave) {
            const int gb = g_lo + wave + W * base;
            if (gb >= g_hi) break;
            if (uniform_int(__hip_atomic_load(&s_best, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP)) < gb)
                break;
            // ---- batch phase: lane t holds entry g_lo + wave + W (base + t) ----
            const int g = gb + W * lane;
            const bool live = g < g_hi;
            int ga, gi;
            bool inside;
            int srow = -1;   // the candidate's stable-pose row (local index), -1 none
            const Pose L = entry_pose(live ? g : 0, pk, pb, C, seed, (uint32_t)s, (uint32_t)j, ax,
                                      ay, zc, &ga, &gi, rs, &inside, st, st ? &srow : nullptr);
            // the bounding centre and probes, turned into the candidate's
            // resting frame when it takes a stable pose
            float bx = bc[0], by = bc[1], bz = bc[2];
            float p1x = probe.x, p1y = probe.y, p1z = probe.z;
            float p2x = probe2.x, p2y = probe2.y, p2z = probe2.z;
            if constexpr (kCons) {
                if (srow >= 0) {
                    const float* R = s_stab.R[srow];
                    rest_point(R, bc[0], bc[1], bc[2], bx, by, bz);
                    rest_point(R, probe.x, probe.y, probe.z, p1x, p1y, p1z);
                    rest_point(R, probe2.x, probe2.y, probe2.z, p2x, p2y, p2z);
                }
            }
            float lx, ly, lz;   // world centre of this candidate's bounding sphere
            float qx, qy, qz;   // world centres of its probe spheres
            float ux, uy, uz;
            Planar M{};         // the candidate's planar motion (kYaw)
            if constexpr (kYaw) {
                M = planar(U, L);
                planar_xy(M, bx, by, lx, ly);
                planar_xy(M, p1x, p1y, qx, qy);
                planar_xy(M, p2x, p2y, ux, uy);
                if (kCons && srow >= 0) {
                    lz = (bz + L.z) + U.t[2];
                    qz = (p1z + L.z) + U.t[2];
                    uz = (p2z + L.z) + U.t[2];
                } else {
                    lz = bz0;
                    qz = pz0;
                    uz = pz02;
                }
            } else {
                to_world(U, L, bx, by, bz, lx, ly, lz);
                to_world(U, L, p1x, p1y, p1z, qx, qy, qz);
                to_world(U, L, p2x, p2y, p2z, ux, uy, uz);
            }
            // rejected: a point outside its relation's region, one the robot
            // cannot reach, or a probe that collides
            bool sure = !inside;
            if constexpr (kCons) {
                if (reach_theta >= 0.f && !sure) {
                    const float* rb = robot + 12 * s;
                    float ox, oy, oz, dx, dy, dz;
                    // the object's x axis: R_m e_x turned by the candidate
                    // (e_x without a stable pose)
                    float v0 = 1.f, v1 = 0.f, v2 = 0.f;
                    if (srow >= 0) {
                        const float* R = s_stab.R[srow];
                        v0 = R[0]; v1 = R[3]; v2 = R[6];
                    }
                    if constexpr (kYaw) {
                        ox = M.Tx; oy = M.Ty; oz = L.z + U.t[2];
                        if (srow >= 0) {
                            dx = fmaf(M.C, v0, -M.S * v1);
                            dy = fmaf(M.S, v0, M.C * v1);
                            dz = v2;
                        } else {
                            dx = M.C; dy = M.S; dz = 0.f;
                        }
                    } else {
                        to_world(U, L, 0.f, 0.f, 0.f, ox, oy, oz);
                        if (srow >= 0) {
                            const float l0 = fmaf(L.c, v0, -L.s * v1), l1 = fmaf(L.s, v0, L.c * v1);
                            dx = fmaf(U.R[0], l0, fmaf(U.R[1], l1, U.R[2] * v2));
                            dy = fmaf(U.R[3], l0, fmaf(U.R[4], l1, U.R[5] * v2));
                            dz = fmaf(U.R[6], l0, fmaf(U.R[7], l1, U.R[8] * v2));
                        } else {
                            dx = fmaf(U.R[0], L.c, U.R[1] * L.s);
                            dy = fmaf(U.R[3], L.c, U.R[4] * L.s);
                            dz = fmaf(U.R[6], L.c, U.R[7] * L.s);
                        }
                    }
                    sure = !reach_ok(rmap.map, rmap, rb, ox, oy, oz, dx, dy, dz, reach_theta);
                }
            }
            unsigned long long bmask = 0, gmask = 0;
            // the probes against the depth map of the placed spheres first:
            // the cheapest rejection
            if (kMap && use_map && j > 0) {
                const DepthMap dmq = map_params(&s_dm);
                if (!sure)
                    sure = map_hit(lmap, dmq, fmaf(L.c, p1x, fmaf(-L.s, p1y, L.x)),
                               fmaf(L.s, p1x, fmaf(L.c, p1y, L.y)), p1z + L.z,
                               probe.w, margin);
                if (two && !sure)
                    sure = map_hit(lmap, dmq, fmaf(L.c, p2x, fmaf(-L.s, p2y, L.x)),
                                   fmaf(L.s, p2x, fmaf(L.c, p2y, L.y)), p2z + L.z,
                                   probe2.w, margin);
                n_sphc += (two ? 2u : 1u) * __popcll(__ballot(live));
            }
            // The box and grid masks serve only candidates still open: a
            // batch the map rejected entirely skips them.
            const bool need = __ballot(live && !sure) != 0;
            if (need) {
                // boxes near the bounding sphere (box data uniform over the wave)
                for (unsigned long long rm = box_rel; rm; rm &= rm - 1) {
                    const int bi = __builtin_ctzll(rm);
                    const float* B = lbox + 16 * bi;
                    bmask |= (unsigned long long)(box_out2_t<kYaw>(B, lx, ly, lz) < reach * reach) << bi;
                }
                // the probes against the lane's own near boxes: a candidate is
                // near few boxes, so this per-lane loop runs far fewer rounds
                // than testing the probes against every box some lane is near
                const unsigned long long pm = sure ? 0ull : bmask;
                lane_boxp += live ? (two ? 2u : 1u) * (unsigned)__popcll(pm) : 0u;
                for (unsigned long long rm = pm; rm && !sure; rm &= rm - 1) {
                    const float* B = lbox + 16 * __builtin_ctzll(rm);
                    sure = box_out2_t<kYaw>(B, qx, qy, qz) < prm2;
                    if (two && !sure) sure = box_out2_t<kYaw>(B, ux, uy, uz) < prm2b;
                }
                // grids: only spheres whose centres lie inside a grid's node box
                // sample it (outside it reads +inf), so a bounding sphere that
                // misses the node box needs no sample
                if constexpr (kGrids) for (int gi = 0; gi < ngrid_mask; ++gi) {
                    const float* G = grid + 24 * (g0 + gi);
                    const bool near = grid_box_d2(G, lx, ly, lz) <= rho * rho;
                    if (near) {
                        gmask |= 1ull << gi;
                        const float* vals = grid_val + grid_val_off[grid_src[g0 + gi]];
                        if (!sure) sure = grid_sample(G, vals, qx, qy, qz) < probe.w + margin;
                        if (two && !sure) sure = grid_sample(G, vals, ux, uy, uz) < probe2.w + margin;
                    }
                    n_grid += (two ? 2u : 1u) * __popcll(__ballot(near && live));
                }
            }
            const unsigned long long sure_mask = __ballot(sure && live);
            {
                const unsigned long long nlive = __popcll(__ballot(live));
                if (need) n_boxc += nlive * (unsigned long long)(__popcll(box_rel) + ngrid_mask);
                n_xf += (two ? 2u : 1u) * nlive;   // probe transforms
            }
            // ---- candidate phase: the entries the batch phase left open, in
            // entry order; entries below position t_end are decided ----
            const unsigned long long live_mask = __ballot(live);
            unsigned long long todo = live_mask & ~sure_mask;
            int t_end = kWave;
            if (live_mask != ~0ull) stop = true;   // the entry list ends in this batch
            while (todo) {
                const int t = __builtin_ctzll(todo);
                todo &= todo - 1;
                const int gt = gb + W * t;
                if (uniform_int(__hip_atomic_load(&s_best, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP)) < gt) {
                    t_end = t;
                    stop = true;
                    break;
                }
                Pose P{};
                Planar Mt{};
                // the candidate's stable pose: the lanes' template spheres in
                // its resting frame and its z (the unturned set otherwise)
                float tx[SPL], ty[SPL], tz[SPL], twz[SPL];
                float zt = zc;
#pragma unroll
                for (int q = 0; q < SPL; ++q) {
                    tx[q] = cx[q]; ty[q] = cy[q]; tz[q] = cz[q]; twz[q] = wz0[q];
                }
                if constexpr (kCons) {
                    const int mt = st ? uniform_int(__builtin_amdgcn_readlane(srow, t)) : -1;
                    if (mt >= 0) {
                        const float* R = s_stab.R[mt];
                        zt = bcast(L.z, t);
#pragma unroll
                        for (int q = 0; q < SPL; ++q) {
                            rest_point(R, cx[q], cy[q], cz[q], tx[q], ty[q], tz[q]);
                            twz[q] = (tz[q] + zt) + U.t[2];
                        }
                    }
                }
                if constexpr (kYaw) {
                    Mt.C = bcast(M.C, t); Mt.S = bcast(M.S, t);
                    Mt.Tx = bcast(M.Tx, t); Mt.Ty = bcast(M.Ty, t);
                } else {
                    P.x = bcast(L.x, t); P.y = bcast(L.y, t); P.z = zt;
                    P.c = bcast(L.c, t); P.s = bcast(L.s, t);
                }
                Gx = bcast(lx, t); Gy = bcast(ly, t); Gz = bcast(lz, t);
                unsigned long long bm = bcast64(bmask, t), gm = bcast64(gmask, t);
                // placed objects whose bounding spheres come within reach of
                // the candidate's bounding centre (lane = object), built only
                // for candidates still open
                unsigned long long omask[kObjWords];
#pragma unroll
                for (int w = 0; w < kObjWords; ++w) {
                    const int ob = 64 * w + lane;
                    bool onear = false;
                    if (ob < nob_mask) {
                        const float4 bd = lbnd[ob];
                        const float dx = Gx - bd.x, dy = Gy - bd.y, dz = Gz - bd.z;
                        const float lim = reach + bd.w;
                        onear = fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < lim * lim;
                    }
                    omask[w] = __ballot(onear);
                }
                n_objc += (unsigned)nob_mask;
                n_xf += S;
#pragma unroll
                for (int q = 0; q < SPL; ++q) {
                    if (q > 0 && q >= nq) break;
                    if constexpr (kYaw) {
                        planar_xy(Mt, tx[q], ty[q], wx[q], wy[q]);
                        wz[q] = twz[q];
                    } else {
                        to_world(U, P, tx[q], ty[q], tz[q], wx[q], wy[q], wz[q]);
                    }
                }
                bool hit = false;
                // boxes of the mask, then any boxes beyond the first 64
                while (bm) {
                    const int bi = __builtin_ctzll(bm);
                    bm &= bm - 1;
                    const float* B = lbox + 16 * bi;
#pragma unroll
                    for (int q = 0; q < SPL; ++q)
                        if (q == 0 || q < nq) hit |= box_out2_t<kYaw>(B, wx[q], wy[q], wz[q]) < rm2[q];
                    n_boxp += S;
                    if (__ballot(hit)) break;
                }
                for (int bx = b0 + kWave; bx < b1 && !__ballot(hit); ++bx) {
                    const float* B = box + 16 * bx;
                    n_boxc += 1;
                    if (!(box_out2_t<kYaw>(B, Gx, Gy, Gz) < reach * reach)) continue;
#pragma unroll
                    for (int q = 0; q < SPL; ++q)
                        if (q == 0 || q < nq) hit |= box_out2_t<kYaw>(B, wx[q], wy[q], wz[q]) < rm2[q];
                    n_boxp += S;
                }
                // voxel grids of the mask: trilinear field minus radius vs
                // margin (a NaN sample, from a non-finite node, collides)
                if constexpr (kGrids) while (gm && !__ballot(hit)) {
                    const int gi = __builtin_ctzll(gm);
                    gm &= gm - 1;
                    const float* G = grid + 24 * (g0 + gi);
                    const float* vals = grid_val + grid_val_off[grid_src[g0 + gi]];
#pragma unroll
                    for (int q = 0; q < SPL; ++q)
                        if (q == 0 || q < nq)
                            hit |= !(grid_sample(G, vals, wx[q], wy[q], wz[q]) >= cr[q] + margin);
                    n_grid += S;
                }
                // grids beyond the first 64: the same node-box pretest on the
                // candidate's bounding sphere, then the samples
                if constexpr (kGrids) for (int gx = g0 + kWave; gx < g1 && !__ballot(hit); ++gx) {
                    const float* G = grid + 24 * gx;
                    n_boxc += 1;
                    if (!(grid_box_d2(G, Gx, Gy, Gz) <= rho * rho)) continue;
                    const float* vals = grid_val + grid_val_off[grid_src[gx]];
#pragma unroll
                    for (int q = 0; q < SPL; ++q)
                        if (q == 0 || q < nq)
                            hit |= !(grid_sample(G, vals, wx[q], wy[q], wz[q]) >= cr[q] + margin);
                    n_grid += S;
                }
                // Every sphere against the depth map: a hit there is a proven
                // collision, found without the placed spheres' pair tests
                // (support-frame coordinates R_u^T (w - t_u) of the world
                // spheres; their rounding is far inside the map's safety).
                // Objects of up to 64 spheres only: for 4 spheres per lane the
                // lookups and the registers they hold cost more than the pair
                // tests they save.
                if (kMap && SPL == 1 && use_map && j > 0 && !__ballot(hit)) {
                    const DepthMap dmq = map_params(&s_dm);
#pragma unroll
                    for (int q = 0; q < SPL; ++q) {
                        if (!(q == 0 || q < nq) || !act[q]) continue;
                        const float dx = wx[q] - U.t[0], dy = wy[q] - U.t[1];
                        float sx, sy, sz;
                        if constexpr (kYaw) {
                            sx = fmaf(U.R[0], dx, U.R[3] * dy);
                            sy = fmaf(U.R[1], dx, U.R[4] * dy);
                            sz = tz[q] + zt;
                        } else {
                            const float dz = wz[q] - U.t[2];
                            sx = fmaf(U.R[0], dx, fmaf(U.R[3], dy, U.R[6] * dz));
                            sy = fmaf(U.R[1], dx, fmaf(U.R[4], dy, U.R[7] * dz));
                            sz = fmaf(U.R[2], dx, fmaf(U.R[5], dy, U.R[8] * dz));
                        }
                        hit |= map_hit(lmap, dmq, sx, sy, sz, cr[q], margin);
                    }
                    n_sphc += S;
                }
                // placed objects of the masks, then any beyond them
                if (!__ballot(hit)) {
#pragma unroll
                    for (int w = 0; w < kObjWords; ++w) {
                        unsigned long long om = omask[w];
                        while (om) {
                            const int ob = 64 * w + __builtin_ctzll(om);
                            om &= om - 1;
                            test_object(ob, hit);
                            if (__ballot(hit)) break;
                        }
                        if (__ballot(hit)) break;
                    }
                    for (int ob = kWave * kObjWords; ob < j && !__ballot(hit); ++ob) {
                        const float4 bd = lbnd[ob];
                        const float dx = Gx - bd.x, dy = Gy - bd.y, dz = Gz - bd.z;
                        const float lim = reach + bd.w;
                        n_objc += 1;
                        if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < lim * lim) test_object(ob, hit);
                    }
                }
                if (!__ballot(hit)) {
                    if (lane == 0) atomicMin(&s_best, gt);   // first, so other waves stop early
                    // its pose for the commit, drawn again here (once per
                    // wave and object) rather than by every wave after the
                    // barrier or kept live in registers
                    int fa, fi, fr = -1;
                    bool fin_in;
                    const Pose F = entry_pose(gt, pk, pb, C, seed, (uint32_t)s, (uint32_t)j, ax,
                                              ay, zc, &fa, &fi, rs, &fin_in, st, st ? &fr : nullptr);
                    if (lane == 0) {
                        float* f = s_found[wave];
                        f[0] = F.x; f[1] = F.y; f[2] = F.z; f[3] = F.c; f[4] = F.s; f[5] = F.yaw;
                        f[6] = __int_as_float(fa); f[7] = __int_as_float(fi);
                        f[8] = __int_as_float(fr);
                    }
                    t_end = t + 1;
                    stop = true;
                    break;
                }
            }
            n_cand += __popcll(t_end == kWave ? live_mask : live_mask & ((1ull << t_end) - 1));
        }
        __syncthreads();
        const int best = s_best;
        if (best == INT_MAX && g_hi < total) {   // entries left for a later launch
            pend = g_hi;
            last = -1;
            break;
        }
        if (wave == 0)
            n_att += (pk ? 1u : 0u) +
                     (best == INT_MAX ? (unsigned)(retries + 1)
                                      : (best < pk ? 0u : (unsigned)((best - pk) / C + 1)));
        if (best == INT_MAX) { fin = SCN_SCENE_INVALID; last = -1; break; }
        // the pose the owning wave tested (entries g_lo + w + W n belong to wave w)
        Pose Pw;
        int fa, fi, fr;
        {
            const float* f = s_found[(best - g_lo) % W];
            Pw.x = f[0]; Pw.y = f[1]; Pw.z = f[2]; Pw.c = f[3]; Pw.s = f[4]; Pw.yaw = f[5];
            fa = __float_as_int(f[6]); fi = __float_as_int(f[7]); fr = __float_as_int(f[8]);
        }
        // the winner's sphere set and bounding centre in its resting frame
        float tx[SPL], ty[SPL], tz[SPL], twz[SPL];
        float tb[3] = {bc[0], bc[1], bc[2]};
        float tbz = bz0;
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            tx[q] = cx[q]; ty[q] = cy[q]; tz[q] = cz[q]; twz[q] = wz0[q];
        }
        if constexpr (kCons) {
            if (fr >= 0) {
                const float* R = s_stab.R[fr];
#pragma unroll
                for (int q = 0; q < SPL; ++q) {
                    rest_point(R, cx[q], cy[q], cz[q], tx[q], ty[q], tz[q]);
                    twz[q] = (tz[q] + Pw.z) + U.t[2];
                }
                rest_point(R, bc[0], bc[1], bc[2], tb[0], tb[1], tb[2]);
                tbz = (tb[2] + Pw.z) + U.t[2];
            }
        }
        if (wave == 0) {
            const Pose P = Pw;
            const Planar Mc = planar(U, P);   // the planar form
            // world bounding sphere of the placed object
            float gx, gy, gz;
            if constexpr (kYaw) {
                planar_xy(Mc, tb[0], tb[1], gx, gy);
                gz = tbz;
            } else {
                to_world(U, P, tb[0], tb[1], tb[2], gx, gy, gz);
            }
            // The learned proposal's height map of the object's support is
            // raised by the committed spheres (the arithmetic of k_hmap_raise).
            // The cells under the object's bounding sphere are raised in an
            // LDS window first (the box rows' space, free during the commit
            // and read again below when this launch places another object),
            // then the map once per covered cell: far fewer global atomics
            // than one per sphere and cell.
            SupportFrame F{};
            float* H = nullptr;
            int* T = reinterpret_cast<int*>(lbox);
            int tx0 = 0, ty0 = 0, tw = 0, th = 0;
            if (kHmap && hmap) {
                const int u = osup;
                F = support_frame(sup, u);
                H = hmap + (size_t)u * 4096;
                float qx, qy, qz;
                to_support(F, gx, gy, gz, qx, qy, qz);
                const float cw = 2.f * F.hx / 64.f, ch = 2.f * F.hy / 64.f;
                tx0 = max(0, (int)floorf((qx - rho + F.hx) / cw - 0.5f));
                ty0 = max(0, (int)floorf((qy - rho + F.hy) / ch - 0.5f));
                tw = min(63, (int)ceilf((qx + rho + F.hx) / cw - 0.5f)) - tx0 + 1;
                th = min(63, (int)ceilf((qy + rho + F.hy) / ch - 0.5f)) - ty0 + 1;
                if (tw <= 0 || th <= 0 || tw * th > kHmapTileCells) tw = th = 0;   // no window
                for (int c = lane; c < tw * th; c += kWave) T[c] = 0;
            }
#pragma unroll
            for (int q = 0; q < SPL; ++q) {
                if (act[q]) {
                    float px, py, pz;
                    if constexpr (kYaw) {   // the arithmetic the candidate was tested with
                        planar_xy(Mc, tx[q], ty[q], px, py);
                        pz = twz[q];
                    } else {
                        to_world(U, P, tx[q], ty[q], tz[q], px, py, pz);
                    }
                    const int k = lane + kWave * q;
                    placed[sb + k] = make_float4(px, py, pz, cr[q]);
                    if constexpr (kLds) lsph[sb - first + k] = make_float4(px, py, pz, cr[q] + margin);
                    if (kHmap && hmap) hmap_raise_sphere(F, H, px, py, pz, cr[q], T, tx0, ty0, tw, th);
                }
            }
            if (kHmap && hmap) {
                // window cell c = wx th + wy (c < 2^10: the float quotient
                // truncates exactly)
                const int ncell = tw * th;
                const float rth = 1.f / (float)max(th, 1);
                for (int c = lane; c < ncell; c += kWave) {
                    const int v = T[c];
                    if (v > 0) {
                        const int wx = (int)(((float)c + 0.5f) * rth), wy = c - wx * th;
                        atomicMax(reinterpret_cast<int*>(H) + (tx0 + wx) * 64 + ty0 + wy, v);
                    }
                }
                if (ncell > 0 && j + 1 < j_end)   // the box rows back for the next object
                    for (int i = lane; i < 16 * nbox_mask; i += kWave)
                        T[i] = __float_as_int(box[16 * b0 + i]);
            }
            if (lane == 0) {
                lbnd[j] = make_float4(gx, gy, gz, rho);
                if (bnd_keep) bnd_keep[o] = make_float4(gx, gy, gz, rho);
                rec[o] = scn_pose_rec{P.x, P.y, P.z, P.yaw, fa, fi};
                if constexpr (kCons) {
                    if (rec_stable) rec_stable[o] = fr >= 0 ? s_stab.r0 + fr : -1;
                }
            }
            ++n_done;
        }
        // the new object's spheres into the depth map (voxels split over the
        // waves); a later launch rebuilds the map from the placed spheres, or
        // with map_keep loads the one stored below
        if (kMap && use_map && (j + 1 < j_end || map_keep)) {
            const DepthMap dm = map_params(&s_dm);
#pragma unroll
            for (int q = 0; q < SPL; ++q)
                if (act[q])
                    map_insert(lmap, dm, fmaf(Pw.c, tx[q], fmaf(-Pw.s, ty[q], Pw.x)),
                               fmaf(Pw.s, tx[q], fmaf(Pw.c, ty[q], Pw.y)), tz[q] + Pw.z, cr[q], wave,
                               W);
        }
        last = fi;
        __syncthreads();
    }
    // the depth map of a scene that placed in this launch back to map_keep
    // (the barrier ending the last placement ordered every insert before)
    if constexpr (kMap) {
        if (map_keep && use_map && j > j_start) {
            const DepthMap dm = map_params(&s_dm);
            const int w16 = (dm.nx * dm.ny * dm.nz + 15) >> 4;
            int4* dst = reinterpret_cast<int4*>(map_keep + (size_t)s * kMapBytes);
            const int4* mw = reinterpret_cast<const int4*>(lmap);
            for (int i = threadIdx.x; i < w16; i += blockDim.x) dst[i] = mw[i];
        }
    }
    if (threadIdx.x == 0) {
        n_placed[s] = j;
        if (resume) resume[s] = pend;
        const int8_t st = fin != SCN_SCENE_ACTIVE ? fin
                                                  : (j == nobj ? SCN_SCENE_VALID : SCN_SCENE_ACTIVE);
        status[s] = st;
        if (n_active && st == SCN_SCENE_ACTIVE && (j_cap <= 0 || j < j_cap)) {
            atomicAdd(n_active, 1);                   // scenes with work left
            if (pend == 0) atomicAdd(n_active + 1, 1);  // of them, starting a new object
        }
        if (chosen) chosen[s] = last;
        if (st == SCN_SCENE_VALID) atomicAdd(counters + kValidScenes, 1ull);
        if (st == SCN_SCENE_INVALID) atomicAdd(counters + kInvalidScenes, 1ull);
    }
    // per-lane counts summed over the wave (every lane is active here)
    for (int m = 32; m >= 1; m >>= 1) lane_boxp += __shfl_xor(lane_boxp, m, kWave);
    n_boxp += lane_boxp;
    if (lane == 0) {
        atomicAdd(counters + kCandidates, n_cand);
        atomicAdd(counters + kSpherePairs, n_pairs);
        atomicAdd(counters + kBoxPairs, n_boxp);
        atomicAdd(counters + kTransforms, n_xf);
        atomicAdd(counters + kBoxCulls, n_boxc);
        atomicAdd(counters + kObjCulls, n_objc);
        atomicAdd(counters + kSphCulls, n_sphc);
        if (n_grid) atomicAdd(counters + kGridSamples, n_grid);
        if (n_att) atomicAdd(counters + kAttempts, n_att);
        if (n_done) atomicAdd(counters + kPlaced, n_done);
    }
}

// Entry points.  k_place: every batch but the ones below.  k_place_g5: grid
// batches with up to 128 spheres per object, asked for 5 waves per SIMD
// (their code sits a few registers above it, and a few bytes of spills cost
// less than a fifth of the waves; 256-sphere objects would spill far more).
template <int SPL, bool kLds, bool kGrids, bool kYaw, bool kCons>
__global__ __launch_bounds__(1024) void k_place(SCN_PLACE_PARAMS) {
    place_scenes<SPL, kLds, kGrids, kYaw, kCons>(SCN_PLACE_ARGS);
}
template <int SPL, bool kLds, bool kYaw>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5))) void k_place_g5(
    SCN_PLACE_PARAMS) {
    place_scenes<SPL, kLds, true, kYaw, false>(SCN_PLACE_ARGS);
}
// the learned launches' instances (height-map raise), likewise
template <int SPL, bool kGrids, bool kYaw>
__global__ __launch_bounds__(1024) void k_place_h(SCN_PLACE_PARAMS) {
    place_scenes<SPL, false, kGrids, kYaw, false, true>(SCN_PLACE_ARGS);
}
template <int SPL, bool kYaw>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5))) void k_place_hg5(
    SCN_PLACE_PARAMS) {
    place_scenes<SPL, false, true, kYaw, false, true>(SCN_PLACE_ARGS);
}

// Spatial relations, reachability and stable poses are compiled only into
// grid-free instances (kCons); a grid batch with any is refused by the
// launcher.
template <int SPL, bool kLds, bool kGrids, bool kYaw, bool kCons>
static auto place_kernel() {
    if constexpr (kGrids && SPL <= 2) return k_place_g5<SPL, kLds, kYaw>;
    else if constexpr (kGrids) return k_place<SPL, kLds, true, kYaw, false>;
    else return k_place<SPL, kLds, false, kYaw, kCons>;
}
template <int SPL, bool kGrids, bool kYaw>
static auto place_kernel_h() {
    if constexpr (kGrids && SPL <= 2) return k_place_hg5<SPL, kYaw>;
    else return k_place_h<SPL, kGrids, kYaw>;
}

template <int SPL, bool kLds>
static hipError_t launch_place_one(const scn_batch& b, const scn_gen_args& a,
                                   const PlacePlan& plan, int cap_sph, int split, int32_t* chosen,
                                   unsigned long long* ctr, hipStream_t st) {
    const bool yaw = b.geometry == SCN_GEOM_YAW;
    const bool relp = b.obj_rel != nullptr || b.robot != nullptr || b.obj_pose_off != nullptr;
    if (relp && b.grid_off) return hipErrorNotSupported;
    // the height-map raise is compiled into global-sphere, constraint-free
    // instances only
    if (plan.hmap && (kLds || relp)) return hipErrorNotSupported;
    auto kern = b.grid_off ? (yaw ? place_kernel<SPL, kLds, true, true, false>()
                                  : place_kernel<SPL, kLds, true, false, false>())
                : relp     ? (yaw ? place_kernel<SPL, kLds, false, true, true>()
                                  : place_kernel<SPL, kLds, false, false, true>())
                           : (yaw ? place_kernel<SPL, kLds, false, true, false>()
                                  : place_kernel<SPL, kLds, false, false, false>());
    if constexpr (!kLds) {
        if (plan.hmap)
            kern = b.grid_off ? (yaw ? place_kernel_h<SPL, true, true>()
                                     : place_kernel_h<SPL, true, false>())
                              : (yaw ? place_kernel_h<SPL, false, true>()
                                     : place_kernel_h<SPL, false, false>());
    }
    // the kernel's layout: placed spheres (LDS instances), a bounding sphere
    // per object, 4 constants and one index row per object the launch may
    // place, box rows, depth map (grid-free batches)
    const int n_info = plan.max_steps > 0 ? std::min(plan.cap_obj, plan.max_steps) : plan.cap_obj;
    const int bytes = 16 * ((kLds ? cap_sph : 0) + plan.cap_obj + 5 * n_info) + kBoxLdsBytes +
                      (b.grid_off ? 0 : kMapBytes);
    if (bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(b.n_scenes), dim3(kWave * plan.waves), bytes, st, b.obj_off,
                       b.sph_off, (const float4*)b.tmpl, b.obj_sup, b.obj_ncand, b.sup,
                       b.box_off, b.box, (float4*)b.placed, b.n_placed, b.status, b.rec, chosen,
                       ctr, plan.order, plan.n_order, a.seed, a.margin, a.retries, a.default_ncand,
                       plan.max_steps, cap_sph, plan.cap_obj, split, plan.split_sph,
                       plan.prop_bins, plan.prop_k, plan.resume, plan.chunk, plan.j_cap,
                       plan.n_active, b.grid_off, b.grid, b.grid_src,
                       b.grid_val_off, b.grid_val, b.obj_rel, b.rel, b.obj_ratio, b.robot,
                       b.obj_reach, b.reach, (int8_t*)plan.map_keep, (float4*)plan.bnd_keep,
                       (const float4*)plan.info_keep, plan.hmap, b.obj_pose_off, b.stable,
                       b.rec_stable);
    return hipGetLastError();
}

template <int SPL>
static hipError_t launch_place_spl(const scn_batch& b, const scn_gen_args& a,
                                   const PlacePlan& plan, int32_t* chosen,
                                   unsigned long long* ctr, hipStream_t st) {
    switch (plan.mode) {
        case kPlaceAllLds:
            return launch_place_one<SPL, true>(b, a, plan, plan.cap_sph, 0, chosen, ctr, st);
        case kPlaceAllGlobal:
            return launch_place_one<SPL, false>(b, a, plan, 0, 0, chosen, ctr, st);
        case kPlaceSplit: {
            // larger scenes first (they run longest), then the LDS-resident ones
            hipError_t e = launch_place_one<SPL, false>(b, a, plan, 0, 1, chosen, ctr, st);
            if (e != hipSuccess) return e;
            return launch_place_one<SPL, true>(b, a, plan, plan.split_sph, 1, chosen, ctr, st);
        }
        default: return hipErrorInvalidValue;
    }
}

// Every object's 4 place-kernel constants (object_info) into info, once per
// generation: one workgroup of 4 waves per scene, one wave per object.
template <int SPL, bool kProbe2>
__global__ __launch_bounds__(256) void k_object_info(
    int n, const int32_t* __restrict__ obj_off, const int32_t* __restrict__ sph_off,
    const float4* __restrict__ tmpl, const int32_t* __restrict__ obj_sup,
    const float* __restrict__ sup, const int32_t* __restrict__ box_off,
    const float* __restrict__ box, float margin, float4* __restrict__ info) {
    const int s = blockIdx.x;
    if (s >= n) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform_int(threadIdx.x >> 6), W = blockDim.x >> 6;
    const int b0 = box_off[s], nbox_mask = min(box_off[s + 1] - b0, kWave);
    for (int o = obj_off[s] + wave; o < obj_off[s + 1]; o += W)
        object_info<SPL, kProbe2>(tmpl, sph_off, obj_sup, sup, box, o, b0, nbox_mask, margin, lane,
                                  info + 4 * (size_t)o);
}

hipError_t launch_object_info(const scn_batch& b, float margin, void* info, hipStream_t st) {
    if (b.n_scenes == 0) return hipSuccess;
    const int S = b.max_spheres_per_object;
    const dim3 grid(b.n_scenes), block(256);
    auto args = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, block, 0, st, b.n_scenes, b.obj_off, b.sph_off,
                           (const float4*)b.tmpl, b.obj_sup, b.sup, b.box_off, b.box, margin,
                           (float4*)info);
    };
    const bool p2 = b.grid_off == nullptr;   // the second probe serves grid-free batches
    if (S <= 64) p2 ? args(k_object_info<1, true>) : args(k_object_info<1, false>);
    else if (S <= 128) p2 ? args(k_object_info<2, true>) : args(k_object_info<2, false>);
    else p2 ? args(k_object_info<4, true>) : args(k_object_info<4, false>);
    return hipGetLastError();
}

hipError_t launch_place(const scn_batch& b, const scn_gen_args& a, const PlacePlan& plan,
                        int32_t* chosen, int64_t* counters, hipStream_t st) {
    if (b.n_scenes == 0) return hipSuccess;
    auto* ctr = (unsigned long long*)counters;
    switch (plan.spl) {
        case 1: return launch_place_spl<1>(b, a, plan, chosen, ctr, st);
        case 2: return launch_place_spl<2>(b, a, plan, chosen, ctr, st);
        case 4: return launch_place_spl<4>(b, a, plan, chosen, ctr, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace scn
