// kernels.hip -- the libscn hot path on gfx950 (wave64, CDNA4).
//
//   k_reset   scene/record reset (graph-safe fill, no hipMemset)
//   k_sample  candidate poses of one attempt, one lane per candidate
//   k_check   dense exact clearance: sphere-pair distances on the FP32 matrix
//             cores (one wave per candidate), boxes and grids on the vector ALU
//   k_order_* longest-first scene order (counting sort by a work estimate)
// The persistent fused place kernel is in place.hip.
#include <climits>

#include "device.h"
#include "internal.h"

namespace scn {

// ---------------------------------------------------------------------------
__global__ void k_reset(int n_scenes, int n_objects, int32_t* __restrict__ n_placed,
                        int8_t* __restrict__ status, scn_pose_rec* __restrict__ rec,
                        int32_t* __restrict__ rec_stable) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    for (int s = tid; s < n_scenes; s += stride) {
        n_placed[s] = 0;
        status[s] = SCN_SCENE_ACTIVE;
    }
    if (rec) {
        const float nan = __builtin_nanf("");
        for (int o = tid; o < n_objects; o += stride) rec[o] = scn_pose_rec{nan, nan, nan, nan, -1, -1};
    }
    if (rec_stable)
        for (int o = tid; o < n_objects; o += stride) rec_stable[o] = -1;
}

__global__ void k_fill_i64(int64_t* p, int n, int64_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_reset(const scn_batch& b, hipStream_t st) {
    const int n = b.n_scenes > b.n_objects ? b.n_scenes : b.n_objects;
    if (n == 0) return hipSuccess;
    int blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, st, b.n_scenes, b.n_objects,
                       b.n_placed, b.status, b.rec, b.rec_stable);
    return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* p, int n, int64_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_i64, dim3((n + 63) / 64), dim3(64), 0, st, p, n, v);
    return hipGetLastError();
}

// Height that rests the lowest sphere of object o on its support plane.
__device__ __forceinline__ float rest_lift(const float4* __restrict__ tmpl, int k0, int k1) {
    float lift = -__builtin_huge_valf();
    for (int k = k0; k < k1; ++k) {
        const float4 c = tmpl[k];
        lift = fmaxf(lift, c.w - c.z);
    }
    return lift;
}

// ---------------------------------------------------------------------------
// Candidate poses of one attempt.  grid = (scenes, candidate tiles of 256).
__global__ __launch_bounds__(256) void k_sample(
    const int32_t* __restrict__ obj_off, const int32_t* __restrict__ sph_off,
    const float4* __restrict__ tmpl, const int32_t* __restrict__ obj_sup,
    const float* __restrict__ sup, const float* __restrict__ obj_ratio,
    const int32_t* __restrict__ obj_idx, const int32_t* __restrict__ cand_off, uint64_t seed,
    int attempt, float* __restrict__ ox, float* __restrict__ oy, float* __restrict__ oz,
    float* __restrict__ oyaw, const int32_t* __restrict__ pose_off, const float* __restrict__ stable,
    int32_t* __restrict__ ok) {
    const int s = blockIdx.x;
    const int o = obj_idx[s];
    if (o < obj_off[s] || o >= obj_off[s + 1]) return;   // -1 or not an object of scene s
    const int c0 = cand_off[s], c1 = cand_off[s + 1];
    const int t = c0 + blockIdx.y * blockDim.x + threadIdx.x;
    if (t >= c1) return;
    const Support U = load_support(sup, obj_sup[o]);
    const float lift = rest_lift(tmpl, sph_off[o], sph_off[o + 1]);
    // ratio_on_support: erosion by ratio x half the shorter x / y extent
    float ero = 0.f;
    if (obj_ratio && obj_ratio[o] > 0.f) {
        float lx = 1e30f, hx = -1e30f, ly = 1e30f, hy = -1e30f;
        for (int k = sph_off[o]; k < sph_off[o + 1]; ++k) {
            const float4 c = tmpl[k];
            lx = fminf(lx, c.x - c.w); hx = fmaxf(hx, c.x + c.w);
            ly = fminf(ly, c.y - c.w); hy = fmaxf(hy, c.y + c.w);
        }
        ero = obj_ratio[o] * 0.5f * fminf(hx - lx, hy - ly);
    }
    uint32_t w3;
    Pose P = sample_pose(seed, (uint32_t)s, (uint32_t)(o - obj_off[s]), (uint32_t)attempt,
                         (uint32_t)(t - c0), U.hx - U.inset - ero, U.hy - U.inset - ero,
                         U.lift + lift, &w3);
    // a stable pose: the lift of the turned sphere set
    const int row = stable_pick(pose_off, stable, o, w3);
    if (row >= 0) {
        const float* R = stable + 12 * row;
        float l = -__builtin_huge_valf();
        for (int k = sph_off[o]; k < sph_off[o + 1]; ++k) {
            const float4 c = tmpl[k];
            float x, y, z;
            rest_point(R, c.x, c.y, c.z, x, y, z);
            l = fmaxf(l, c.w - z);
        }
        P.z = U.lift + l;
    }
    ox[t] = P.x;
    oy[t] = P.y;
    oz[t] = P.z;
    oyaw[t] = P.yaw;
    if (ok) ok[t] = row;
}

hipError_t launch_sample(const scn_batch& b, const int32_t* obj_idx, const int32_t* cand_off,
                         int max_cand, uint64_t seed, int attempt, scn_poses out, hipStream_t st) {
    if (b.n_scenes == 0 || max_cand == 0) return hipSuccess;
    dim3 grid(b.n_scenes, (max_cand + 255) / 256);
    hipLaunchKernelGGL(k_sample, grid, dim3(256), 0, st, b.obj_off, b.sph_off,
                       (const float4*)b.tmpl, b.obj_sup, b.sup, b.obj_ratio, obj_idx, cand_off,
                       seed, attempt, out.x, out.y, out.z, out.yaw, b.obj_pose_off, b.stable,
                       out.stable);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense distance-mode check on the matrix cores.
//
// grid = (scenes, candidate tiles of kCheckTile); 4 waves per workgroup, and a
// wave takes the tile's candidates one at a time (tile start + wave, + 4, ...).
// For one candidate with world pose (Rw, tw), in the frame centred at tw:
//   p'_k = Rw c_k              (template sphere k, |p'| <= the object's reach R)
//   q'_j = q_j - tw            (placed sphere j of the scene)
//   D[k][j] = |p'_k - q'_j|^2 = |p'_k|^2 - 2 p'_k . q'_j + |q'_j|^2
// is a rank-4 product, so each 16 x 16 block of it is one
// v_mfma_f32_16x16x4_f32:
//   A row k    = (-2 p'x, -2 p'y, -2 p'z, |p'|^2)      lane l: row l % 16, entry l / 16
//   B column j = (q'x, q'y, q'z, 1)                     lane l: column l % 16, entry l / 16
//   C[.][j]    = |q'_j|^2                               lane l: rows 4 (l / 16) .. +3 of column l % 16
// and the vector ALU keeps, per lane and row, min_j (sqrt|D| - r_j).
//
// Precision.  A pair close enough to matter has |p'| <= R and |q'| <= R + d,
// so the expansion's terms and partial sums stay below 2 (R + d)^2 and its FP32
// evaluation (the squares, the products and sums of the instruction) errs by
// at most a few ulps of that: dD <= 8 * 2^-23 * 2 (R + 1 cm)^2.  The distance
// sqrt(D + dD) is then within dD / (2 d) of the true one, under 8e-6 m once
// d >= s_exact = dD / 1.6e-5 m (a few mm for objects of R ~ 0.2 m).  Every
// candidate that has a pair closer than s_exact (tracked as the minimum of
// sqrt|D| over all its pairs) has its pairs evaluated again in the direct
// form |p' - q'| on the vector ALU; that happens to a small fraction of
// candidates, since only near-concentric sphere pairs are that close.  |D|
// under the root absorbs a tiny negative value of such a pair.
//
// The running minima are kept as the bit patterns of sqrt|D| + (O - r_j) with
// O = 1 m + the scene's largest placed radius: that value is positive, so
// unsigned integer order is float order (v_min3_u32, no NaN quieting of the
// accumulator), and O is removed afterwards (FP32 rounding of the sum costs
// at most half an ulp of O, ~6e-8 m).  Rows past the object's S spheres and
// columns past the scene's placed spheres are padded with a huge |p'|^2 /
// |q'|^2.  clearance = min over rows k of (row minimum - r_k), with the boxes
// and grids (one sphere per lane, exact SDF and trilinear sample) folded in
// before the wave minimum.
constexpr int kCheckTile = 32;
constexpr int kCheckWaves = 4;
constexpr int kCheckMaxSpheres = 256;   // template spheres of one object (LDS copy)
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct CheckIn {
    const float4* stmpl;   // the object's template spheres, staged in LDS
    const float4* placed;
    __amdgpu_buffer_rsrc_t placed_rsrc;   // the scene's placed spheres; reads past them return 0
    const float* box;
    const float* grid;
    const int32_t* grid_src;
    const int64_t* grid_val_off;
    const float* grid_val;
    int S, first, pl_end, b0, b1, g0, g1;
    float off;             // offset of the running minima (1 m + largest placed radius)
    float s_exact;         // a pair closer than this sends the candidate to the direct form
};

// One candidate's sphere pairs for template rows [16 r0, 16 (r0 + NRT)):
// min over those rows k and every placed sphere j of (|p_k - q_j| - r_j - r_k),
// lane-partial (the caller takes the wave minimum).  smin receives the
// smallest sqrt|D| seen (bit pattern).
template <int NRT>
__device__ __forceinline__ float pair_rows(const CheckIn& in, const float* Rw, const float* tw,
                                           int r0, uint32_t& smin) {
    const int lane = threadIdx.x & (kWave - 1);
    const int col = lane & 15, grp = lane >> 4;
    const float kBig = 1e30f;
    const uint32_t kInfBits = 0x7f800000u;
    // one-hot weights of this lane's operand entry (x, y, z, or the 4th):
    // entry = sum of w_e * value_e, exact because the other products are +0
    const float w0 = grp == 0 ? 1.f : 0.f, w1 = grp == 1 ? 1.f : 0.f;
    const float w2 = grp == 2 ? 1.f : 0.f, w3 = grp == 3 ? 1.f : 0.f;
    // A operands: row l % 16 of each 16-row tile, entry l / 16
    float A[NRT];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) {
        const int k = 16 * (r0 + rt) + col;
        const float4 c = in.stmpl[min(k, in.S - 1)];
        const float ux = fmaf(Rw[0], c.x, fmaf(Rw[1], c.y, Rw[2] * c.z));
        const float uy = fmaf(Rw[3], c.x, fmaf(Rw[4], c.y, Rw[5] * c.z));
        const float uz = fmaf(Rw[6], c.x, fmaf(Rw[7], c.y, Rw[8] * c.z));
        const float n2 = k < in.S ? fmaf(ux, ux, fmaf(uy, uy, uz * uz)) : kBig;
        const float s2 = k < in.S ? -2.f : 0.f;
        A[rt] = fmaf(w0 * s2, ux, fmaf(w1 * s2, uy, fmaf(w2 * s2, uz, w3 * n2)));
    }
    uint32_t acc[NRT][4];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[rt][i] = kInfBits;
    uint32_t sm[NRT];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) sm[rt] = kInfBits;
    const int np = in.pl_end - in.first;
    // two 16-column tiles per step (both loads in flight, and three-way
    // minima); buffer reads past the scene's placed spheres return 0, and
    // those columns are padded with a huge |q'|^2
    for (int jb = 0; jb < np; jb += 32) {
        float4 q[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
            q[h] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(
                                                  in.placed_rsrc, 16 * (16 * h + col), 16 * jb, 0));
        float bv[2], orj[2];
        f32x4 cv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bool ok = jb + 16 * h + col < np;
            const float qx = q[h].x - tw[0], qy = q[h].y - tw[1], qz = q[h].z - tw[2];
            const float n2 = ok ? fmaf(qx, qx, fmaf(qy, qy, qz * qz)) : kBig;
            orj[h] = ok ? in.off - q[h].w : in.off;
            bv[h] = fmaf(w0, qx, fmaf(w1, qy, fmaf(w2, qz, w3)));
            cv[h] = f32x4{n2, n2, n2, n2};
        }
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) {
            const f32x4 d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(A[rt], bv[0], cv[0], 0, 0, 0);
            const f32x4 d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(A[rt], bv[1], cv[1], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float s0 = __builtin_amdgcn_sqrtf(fabsf(d0[i]));
                const float s1 = __builtin_amdgcn_sqrtf(fabsf(d1[i]));
                acc[rt][i] = min(acc[rt][i],
                                 min(__float_as_uint(s0 + orj[0]), __float_as_uint(s1 + orj[1])));
                sm[rt] = min(sm[rt], min(__float_as_uint(s0), __float_as_uint(s1)));
            }
        }
    }
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) smin = min(smin, sm[rt]);
    // rows 4 (l / 16) + i of each tile: remove the offset and the sphere's radius
    float m = __builtin_huge_valf();
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 16 * (r0 + rt) + 4 * grp + i;
            if (k < in.S && acc[rt][i] != kInfBits)
                m = fminf(m, (__uint_as_float(acc[rt][i]) - in.off) - in.stmpl[k].w);
        }
    return m;
}

// The candidates t = t0, t0 + kCheckWaves, ... < t1 of one wave.  Returns how
// many got a NaN clearance (non-finite input).
template <bool kGrids>
__device__ __forceinline__ unsigned check_candidates(const CheckIn& in, const Support& U,
                                                     unsigned& nref,
                                                     const float* __restrict__ px,
                                                     const float* __restrict__ py,
                                                     const float* __restrict__ pz,
                                                     const float* __restrict__ pyaw, int t0,
                                                     int t1, bool bad_wg, float margin,
                                                     float* __restrict__ clr_out,
                                                     uint8_t* __restrict__ col_out) {
    const int lane = threadIdx.x & (kWave - 1);
    const float inf = __builtin_huge_valf();
    const int nrt = (in.S + 15) >> 4;
    unsigned nbad = 0;
    for (int t = t0; t < t1; t += kCheckWaves) {
        const float x = px[t], y = py[t], z = pz[t], yw = pyaw[t];
        bool bad = bad_wg || !(__builtin_isfinite(x) & __builtin_isfinite(y) &
                               __builtin_isfinite(z) & __builtin_isfinite(yw));
        float sn, cs;
        sincosf(yw, &sn, &cs);
        // candidate -> world: Rw = R_u Rz(yaw), tw = R_u (x,y,z) + t_u
        float Rw[9], tw[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            Rw[3 * r + 0] = fmaf(U.R[3 * r + 0], cs, U.R[3 * r + 1] * sn);
            Rw[3 * r + 1] = fmaf(-U.R[3 * r + 0], sn, U.R[3 * r + 1] * cs);
            Rw[3 * r + 2] = U.R[3 * r + 2];
            tw[r] = fmaf(U.R[3 * r + 0], x, fmaf(U.R[3 * r + 1], y, fmaf(U.R[3 * r + 2], z, U.t[r])));
        }
        float m = inf;
        if (in.first < in.pl_end) {
            // 64 template rows (four 16-row tiles) per pass over the placed spheres
            uint32_t smin = 0x7f800000u;
            for (int r0 = 0; r0 < nrt; r0 += 4) {
                const int n = nrt - r0;
                m = fminf(m, n >= 4   ? pair_rows<4>(in, Rw, tw, r0, smin)
                             : n == 3 ? pair_rows<3>(in, Rw, tw, r0, smin)
                             : n == 2 ? pair_rows<2>(in, Rw, tw, r0, smin)
                                      : pair_rows<1>(in, Rw, tw, r0, smin));
            }
            // a pair closer than s_exact: the candidate's pairs again, in the
            // direct form (one template sphere per lane)
            if (wave_min(__uint_as_float(smin)) < in.s_exact) {
                ++nref;
                m = inf;
                for (int k = lane; k < in.S; k += kWave) {
                    const float4 c = in.stmpl[k];
                    const float ux = fmaf(Rw[0], c.x, fmaf(Rw[1], c.y, Rw[2] * c.z));
                    const float uy = fmaf(Rw[3], c.x, fmaf(Rw[4], c.y, Rw[5] * c.z));
                    const float uz = fmaf(Rw[6], c.x, fmaf(Rw[7], c.y, Rw[8] * c.z));
                    float best = inf;
                    for (int j = in.first; j < in.pl_end; ++j) {
                        const float4 q = in.placed[j];
                        const float dx = ux - (q.x - tw[0]), dy = uy - (q.y - tw[1]);
                        const float dz = uz - (q.z - tw[2]);
                        best = fminf(best, __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))) - q.w);
                    }
                    m = fminf(m, best - c.w);
                }
            }
        }
        // boxes and grids: one template sphere per lane
        for (int k = lane; k < in.S; k += kWave) {
            const float4 c = in.stmpl[k];
            const float wx = fmaf(Rw[0], c.x, fmaf(Rw[1], c.y, fmaf(Rw[2], c.z, tw[0])));
            const float wy = fmaf(Rw[3], c.x, fmaf(Rw[4], c.y, fmaf(Rw[5], c.z, tw[1])));
            const float wz = fmaf(Rw[6], c.x, fmaf(Rw[7], c.y, fmaf(Rw[8], c.z, tw[2])));
            float best = inf;
            for (int bx = in.b0; bx < in.b1; ++bx)
                best = fminf(best, box_sdf(in.box + 16 * bx, wx, wy, wz));
            if (kGrids) {
                for (int g = in.g0; g < in.g1; ++g) {
                    const float* G = in.grid + 24 * g;
                    const float v =
                        grid_sample(G, in.grid_val + in.grid_val_off[in.grid_src[g]], wx, wy, wz);
                    bad |= v != v;
                    best = fminf(best, v);
                }
            }
            m = fminf(m, best - c.w);
        }
        const float clr_w = wave_min(m);
        bad = __ballot(bad) != 0;
        const float clr = bad ? __builtin_nanf("") : clr_w;
        if (lane == 0) {
            if (clr_out) clr_out[t] = clr;
            if (col_out) col_out[t] = clr >= margin ? 0 : 1;
        }
        nbad += bad ? 1 : 0;
    }
    return nbad;
}

template <bool kGrids>
__global__ __launch_bounds__(64 * kCheckWaves) __attribute__((amdgpu_waves_per_eu(5))) void k_check(
    const int32_t* __restrict__ obj_off, const int32_t* __restrict__ sph_off,
    const float4* __restrict__ tmpl, const int32_t* __restrict__ obj_sup,
    const float* __restrict__ sup, const int32_t* __restrict__ box_off,
    const float* __restrict__ box, const int32_t* __restrict__ grid_off,
    const float* __restrict__ grid, const int32_t* __restrict__ grid_src,
    const int64_t* __restrict__ grid_val_off, const float* __restrict__ grid_val,
    const float4* __restrict__ placed, const int32_t* __restrict__ n_placed,
    const int32_t* __restrict__ obj_idx, const int32_t* __restrict__ cand_off,
    const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz,
    const float* __restrict__ pyaw, float margin, float* __restrict__ clr_out,
    uint8_t* __restrict__ col_out, unsigned long long* __restrict__ counters) {
    __shared__ float4 s_tmpl[kCheckMaxSpheres];
    __shared__ float s_rmax[kCheckWaves];
    const int s = blockIdx.x;
    const int o = obj_idx[s];
    if (o < obj_off[s] || o >= obj_off[s + 1]) return;   // -1 or not an object of scene s
    const int c0 = cand_off[s], c1 = cand_off[s + 1];
    const int tbase = c0 + blockIdx.y * kCheckTile;
    if (tbase >= c1) return;
    const int tend = min(c1, tbase + kCheckTile);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;

    const int oo = obj_off[s];
    const int first = sph_off[oo];
    const int pl_end = sph_off[oo + min(max(n_placed[s], 0), obj_off[s + 1] - oo)];
    const int b0 = box_off[s], b1 = box_off[s + 1];
    int g0 = 0, g1 = 0;
    if (kGrids) { g0 = grid_off[s]; g1 = grid_off[s + 1]; }
    const int k0 = sph_off[o], S = sph_off[o + 1] - k0;
    if (S > kCheckMaxSpheres) return;    // refused on the host
    // Non-finite input makes a candidate collide with a NaN clearance: the
    // object's support row and spheres, the scene's box and grid rows and
    // placed spheres (shared by the workgroup), the candidate's own pose, and
    // any grid sample that reads a non-finite node.  The same pass stages the
    // template in LDS and finds the largest placed radius.
    int bad_in = threadIdx.x < 16 ? !__builtin_isfinite(sup[16 * obj_sup[o] + threadIdx.x]) : 0;
    for (int k = threadIdx.x; k < S; k += blockDim.x) {
        const float4 v = tmpl[k0 + k];
        bad_in |= !finite4(v);
        s_tmpl[k] = v;
    }
    for (int bx = b0 + threadIdx.x; bx < b1; bx += blockDim.x) bad_in |= !all_finite(box + 16 * bx, 15);
    for (int g = g0 + threadIdx.x; g < g1; g += blockDim.x) bad_in |= !all_finite(grid + 24 * g, 19);
    float rmax = 0.f;
    for (int q = first + threadIdx.x; q < pl_end; q += blockDim.x) {
        const float4 v = placed[q];
        bad_in |= !finite4(v);
        rmax = fmaxf(rmax, fabsf(v.w));
    }
    rmax = wave_max(rmax);
    if (lane == 0) s_rmax[wave] = rmax;
    const bool bad_wg = __syncthreads_or(bad_in) != 0;
    for (int w = 0; w < kCheckWaves; ++w) rmax = fmaxf(rmax, s_rmax[w]);

    // the object's reach about its frame origin, which bounds |p'| (see above)
    float reach = 0.f;
    for (int k = lane; k < S; k += kWave) {
        const float4 c = s_tmpl[k];
        reach = fmaxf(reach, __builtin_amdgcn_sqrtf(fmaf(c.x, c.x, fmaf(c.y, c.y, c.z * c.z))));
    }
    reach = wave_max(reach) + 0.01f;
    const float s_exact = fmaxf(1e-4f, 8.f * 1.1920929e-7f * 2.f * reach * reach / 1.6e-5f);
    // a buffer resource over the scene's placed spheres (CDNA dword 3 of a raw
    // buffer: 0x00020000); a read at or past pl_end returns zeros
    const __amdgpu_buffer_rsrc_t prs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(placed + first), (short)0, 16 * (pl_end - first), 0x00020000);
    const CheckIn in{s_tmpl, placed, prs, box, grid, grid_src, grid_val_off, grid_val,
                     S, first, pl_end, b0, b1, g0, g1, 1.f + (bad_wg ? 0.f : rmax), s_exact};
    const Support U = load_support(sup, obj_sup[o]);
    unsigned nref = 0;
    const unsigned nbad = check_candidates<kGrids>(in, U, nref, px, py, pz, pyaw,
                                                   tbase + uniform_int(wave), tend, bad_wg,
                                                   margin, clr_out, col_out);
    if (nbad && lane == 0) {
        atomicOr(counters + kErrorWord, (unsigned long long)kErrNonFinite);
        atomicAdd(counters + kNonFinite, (unsigned long long)nbad);
    }
    if (nref && lane == 0) atomicAdd(counters + kCheckRefined, (unsigned long long)nref);
}

// Any non-finite node value in the grid assets sets the non-finite error bit
// (the samples that read it collide).
__global__ __launch_bounds__(256) void k_scan_grid_values(const int64_t* __restrict__ off,
                                                          int n_assets,
                                                          const float* __restrict__ vals,
                                                          unsigned long long* __restrict__ counters) {
    const int64_t n = off[n_assets];
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !__builtin_isfinite(vals[i]);
    if (__ballot(bad) && (threadIdx.x & (kWave - 1)) == 0)
        atomicOr(counters + kErrorWord, (unsigned long long)kErrNonFinite);
}

hipError_t launch_scan_grid_values(const scn_batch& b, int64_t* counters, hipStream_t st) {
    if (!b.grid_off || b.n_grid_assets <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_grid_values, dim3(256), dim3(256), 0, st, b.grid_val_off,
                       b.n_grid_assets, b.grid_val, (unsigned long long*)counters);
    return hipGetLastError();
}

hipError_t launch_check(const scn_batch& b, const int32_t* obj_idx, const int32_t* cand_off,
                        int max_cand, scn_poses P, float margin, float* clr, uint8_t* col,
                        int64_t* counters, hipStream_t st) {
    if (b.n_scenes == 0 || max_cand == 0) return hipSuccess;
    dim3 grid(b.n_scenes, (max_cand + kCheckTile - 1) / kCheckTile);
    auto* ctr = (unsigned long long*)counters;
    if (b.grid_off) {
        hipError_t e = launch_scan_grid_values(b, counters, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_check<true>, grid, dim3(64 * kCheckWaves), 0, st, b.obj_off,
                           b.sph_off, (const float4*)b.tmpl, b.obj_sup, b.sup, b.box_off, b.box,
                           b.grid_off, b.grid, b.grid_src, b.grid_val_off, b.grid_val,
                           (const float4*)b.placed, b.n_placed, obj_idx, cand_off, P.x, P.y, P.z,
                           P.yaw, margin, clr, col, ctr);
    } else {
        hipLaunchKernelGGL(k_check<false>, grid, dim3(64 * kCheckWaves), 0, st, b.obj_off,
                           b.sph_off, (const float4*)b.tmpl, b.obj_sup, b.sup, b.box_off, b.box,
                           nullptr, nullptr, nullptr, nullptr, nullptr, (const float4*)b.placed,
                           b.n_placed, obj_idx, cand_off, P.x, P.y, P.z, P.yaw, margin, clr, col,
                           ctr);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Longest-first order.  Work estimate of a scene: its objects times its
// spheres (the pair work of a scene grows with both), scaled by how crowded
// its first object's support is with boxes: the footprints of the boxes'
// support-frame bounding boxes that reach above the plane, clipped to the
// support rectangle, as a fraction c of its area (overlaps counted twice).
// On a crowded support more objects exhaust their attempts, and a scene
// with an object that does runs several times longer; the scale is
// 1 + 3 min(c, 1.5).  256 log-spaced buckets, largest first; scenes inside a
// bucket in arbitrary order (results do not depend on the order: scenes are
// independent).
__device__ __forceinline__ int work_bucket(const int32_t* __restrict__ obj_off,
                                           const int32_t* __restrict__ sph_off,
                                           const int32_t* __restrict__ box_off,
                                           const int32_t* __restrict__ obj_sup,
                                           const float* __restrict__ sup,
                                           const float* __restrict__ box, int s) {
    const int o0 = obj_off[s], o1 = obj_off[s + 1];
    const int b0 = box_off[s], b1 = box_off[s + 1];
    float crowd = 0.f;
    if (o1 > o0 && b1 > b0) {
        const float* U = sup + 16 * (size_t)obj_sup[o0];
        const float hx = U[12], hy = U[13];
        float cover = 0.f;
        // (unrolled: the boxes' row loads in flight together)
#pragma unroll 4
        for (int bi = b0; bi < b1; ++bi) {
            const float* B = box + 16 * (size_t)bi;
            // box centre and bounding half extents in the support frame
            const float dx = B[9] - U[9], dy = B[10] - U[10], dz = B[11] - U[11];
            float c[3], e[3];
            for (int a = 0; a < 3; ++a) {
                c[a] = U[a] * dx + U[3 + a] * dy + U[6 + a] * dz;
                // row a of U^T B_R, absolute, times the half extents
                float ea = 0.f;
                for (int k = 0; k < 3; ++k) {
                    const float m = U[a] * B[k] + U[3 + a] * B[3 + k] + U[6 + a] * B[6 + k];
                    ea += fabsf(m) * B[12 + k];
                }
                e[a] = ea;
            }
            if (!(c[2] + e[2] > 0.f)) continue;
            const float ox = fminf(hx, c[0] + e[0]) - fmaxf(-hx, c[0] - e[0]);
            const float oy = fminf(hy, c[1] + e[1]) - fmaxf(-hy, c[1] - e[1]);
            if (ox > 0.f && oy > 0.f) cover += ox * oy;
        }
        const float area = 4.f * hx * hy, f = cover / area;
        crowd = f > 0.f ? fminf(f, 1.5f) : 0.f;   // non-finite rows: no scaling
    }
    const float w = (float)(o1 - o0) * (float)(sph_off[o1] - sph_off[o0] + 16 * (b1 - b0)) *
                        (1.f + 3.f * crowd) + 1.f;
    const int bk = (int)(__log2f(w) * 6.0f);
    return kOrderBuckets - 1 - min(max(bk, 0), kOrderBuckets - 1);
}

static_assert(kOrderBuckets == 256, "the order kernels run one thread per bucket (256)");
// Many scenes share a bucket: each workgroup counts its scenes per bucket in
// LDS first and adds its counts to the global histogram with one atomic per
// bucket it uses.
__global__ __launch_bounds__(256) void k_order_hist(int n, const int32_t* __restrict__ obj_off,
                                                    const int32_t* __restrict__ sph_off,
                                                    const int32_t* __restrict__ box_off,
                                                    const int32_t* __restrict__ obj_sup,
                                                    const float* __restrict__ sup,
                                                    const float* __restrict__ box,
                                                    int32_t* __restrict__ hist) {
    __shared__ int cnt[kOrderBuckets];
    const int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + t;
    if (s < n) atomicAdd(&cnt[work_bucket(obj_off, sph_off, box_off, obj_sup, sup, box, s)], 1);
    __syncthreads();
    if (cnt[t] > 0) atomicAdd(hist + t, cnt[t]);
}

// exclusive scan of the 256 bucket counts, one workgroup of 256 threads
__global__ void k_order_scan(int32_t* __restrict__ hist) {
    __shared__ int v[kOrderBuckets];
    const int t = threadIdx.x;
    v[t] = hist[t];
    __syncthreads();
    for (int d = 1; d < kOrderBuckets; d <<= 1) {
        const int x = t >= d ? v[t - d] : 0;
        __syncthreads();
        v[t] += x;
        __syncthreads();
    }
    hist[t] = t == 0 ? 0 : v[t - 1];
}

// The scatter: each workgroup reserves, per bucket it uses, a run of slots
// with one atomic on the scanned histogram, and hands them out to its scenes
// by LDS atomics.
__global__ __launch_bounds__(256) void k_order_scatter(int n, const int32_t* __restrict__ obj_off,
                                                       const int32_t* __restrict__ sph_off,
                                                       const int32_t* __restrict__ box_off,
                                                       const int32_t* __restrict__ obj_sup,
                                                       const float* __restrict__ sup,
                                                       const float* __restrict__ box,
                                                       int32_t* __restrict__ hist,
                                                       int32_t* __restrict__ order) {
    __shared__ int cnt[kOrderBuckets], base[kOrderBuckets];
    const int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + t;
    const int bk = s < n ? work_bucket(obj_off, sph_off, box_off, obj_sup, sup, box, s) : 0;
    if (s < n) atomicAdd(&cnt[bk], 1);
    __syncthreads();
    base[t] = cnt[t] > 0 ? atomicAdd(hist + t, cnt[t]) : 0;
    __syncthreads();
    if (s < n) order[atomicAdd(&base[bk], 1)] = s;
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_longest_first(const scn_batch& b, int32_t* order, int32_t* hist,
                                hipStream_t st) {
    const int n = b.n_scenes;
    if (n == 0) return hipSuccess;
    const int g = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kOrderBuckets), 0, st, hist, kOrderBuckets, 0);
    hipLaunchKernelGGL(k_order_hist, dim3(g), dim3(256), 0, st, n, b.obj_off, b.sph_off,
                       b.box_off, b.obj_sup, b.sup, b.box, hist);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(kOrderBuckets), 0, st, hist);
    hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(256), 0, st, n, b.obj_off, b.sph_off,
                       b.box_off, b.obj_sup, b.sup, b.box, hist, order);
    return hipGetLastError();
}

}  // namespace scn
