// kernels.hip -- the libscn hot path on gfx950 (wave64, CDNA4).
//
//   k_reset   scene/record reset (graph-safe fill, no hipMemset)
//   k_sample  candidate poses of one attempt, one lane per candidate
//   k_check   dense exact clearance, one lane per candidate, obstacles
//             wave-uniform (scalar loads from the read-only tables)
//   k_order_* longest-first scene order (counting sort by a work estimate)
// The persistent fused place kernel is in place.hip.
#include <climits>

#include "device.h"
#include "internal.h"

namespace scn {

// ---------------------------------------------------------------------------
__global__ void k_reset(int n_scenes, int n_objects, int32_t* __restrict__ n_placed,
                        int8_t* __restrict__ status, scn_pose_rec* __restrict__ rec) {
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
                       b.n_placed, b.status, b.rec);
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
    const float* __restrict__ sup, const int32_t* __restrict__ obj_idx,
    const int32_t* __restrict__ cand_off, uint64_t seed, int attempt, float* __restrict__ ox,
    float* __restrict__ oy, float* __restrict__ oz, float* __restrict__ oyaw) {
    const int s = blockIdx.x;
    const int o = obj_idx[s];
    if (o < obj_off[s] || o >= obj_off[s + 1]) return;   // -1 or not an object of scene s
    const int c0 = cand_off[s], c1 = cand_off[s + 1];
    const int t = c0 + blockIdx.y * blockDim.x + threadIdx.x;
    if (t >= c1) return;
    const Support U = load_support(sup, obj_sup[o]);
    const float lift = rest_lift(tmpl, sph_off[o], sph_off[o + 1]);
    const Pose P = sample_pose(seed, (uint32_t)s, (uint32_t)(o - obj_off[s]), (uint32_t)attempt,
                               (uint32_t)(t - c0), U.hx - U.inset, U.hy - U.inset, U.lift + lift);
    ox[t] = P.x;
    oy[t] = P.y;
    oz[t] = P.z;
    oyaw[t] = P.yaw;
}

hipError_t launch_sample(const scn_batch& b, const int32_t* obj_idx, const int32_t* cand_off,
                         int max_cand, uint64_t seed, int attempt, scn_poses out, hipStream_t st) {
    if (b.n_scenes == 0 || max_cand == 0) return hipSuccess;
    dim3 grid(b.n_scenes, (max_cand + 255) / 256);
    hipLaunchKernelGGL(k_sample, grid, dim3(256), 0, st, b.obj_off, b.sph_off,
                       (const float4*)b.tmpl, b.obj_sup, b.sup, obj_idx, cand_off, seed, attempt,
                       out.x, out.y, out.z, out.yaw);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense distance-mode check.  grid = (scenes, candidate tiles of 256); every
// lane owns one candidate; spheres, boxes and placed spheres are uniform
// across the wave, so they come through scalar loads.
template <bool kGrids>
__global__ __launch_bounds__(256) void k_check(
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
    const int s = blockIdx.x;
    const int o = obj_idx[s];
    if (o < obj_off[s] || o >= obj_off[s + 1]) return;   // -1 or not an object of scene s
    const int c0 = cand_off[s], c1 = cand_off[s + 1];
    const int tbase = c0 + blockIdx.y * blockDim.x;
    if (tbase >= c1) return;
    const int t = tbase + threadIdx.x;
    const bool live = t < c1;
    const int tt = live ? t : c1 - 1;

    const int oo = obj_off[s];
    const int first = sph_off[oo];
    const int pl_end = sph_off[oo + min(max(n_placed[s], 0), obj_off[s + 1] - oo)];
    const int b0 = box_off[s], b1 = box_off[s + 1];
    int g0 = 0, g1 = 0;
    if (kGrids) { g0 = grid_off[s]; g1 = grid_off[s + 1]; }
    // Non-finite input makes a candidate collide with a NaN clearance: the
    // object's support row and spheres, the scene's box and grid rows and
    // placed spheres (shared by the workgroup), the candidate's own pose, and
    // any grid sample that reads a non-finite node.
    int bad_in = threadIdx.x < 16 ? !__builtin_isfinite(sup[16 * obj_sup[o] + threadIdx.x]) : 0;
    for (int k = sph_off[o] + threadIdx.x; k < sph_off[o + 1]; k += blockDim.x)
        bad_in |= !finite4(tmpl[k]);
    for (int bx = b0 + threadIdx.x; bx < b1; bx += blockDim.x) bad_in |= !all_finite(box + 16 * bx, 15);
    for (int g = g0 + threadIdx.x; g < g1; g += blockDim.x) bad_in |= !all_finite(grid + 24 * g, 19);
    for (int q = first + threadIdx.x; q < pl_end; q += blockDim.x) bad_in |= !finite4(placed[q]);
    bool bad = __syncthreads_or(bad_in) != 0;

    const Support U = load_support(sup, obj_sup[o]);
    float sn, cs;
    const float x = px[tt], y = py[tt], z = pz[tt], yw = pyaw[tt];
    bad |= !(__builtin_isfinite(x) & __builtin_isfinite(y) & __builtin_isfinite(z) &
             __builtin_isfinite(yw));
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
    float clr = __builtin_huge_valf();
    for (int k = sph_off[o]; k < sph_off[o + 1]; ++k) {
        const float4 c = tmpl[k];
        const float wx = fmaf(Rw[0], c.x, fmaf(Rw[1], c.y, fmaf(Rw[2], c.z, tw[0])));
        const float wy = fmaf(Rw[3], c.x, fmaf(Rw[4], c.y, fmaf(Rw[5], c.z, tw[1])));
        const float wz = fmaf(Rw[6], c.x, fmaf(Rw[7], c.y, fmaf(Rw[8], c.z, tw[2])));
        float best = __builtin_huge_valf();
        for (int bx = b0; bx < b1; ++bx) best = fminf(best, box_sdf(box + 16 * bx, wx, wy, wz));
        if (kGrids) {
            for (int g = g0; g < g1; ++g) {
                const float* G = grid + 24 * g;
                const float v = grid_sample(G, grid_val + grid_val_off[grid_src[g]], wx, wy, wz);
                bad |= v != v;
                best = fminf(best, v);
            }
        }
        int j = first;
        for (; j + 4 <= pl_end; j += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 q = placed[j + u];
                const float dx = wx - q.x, dy = wy - q.y, dz = wz - q.z;
                const float d = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
                best = fminf(best, d - q.w);
            }
        }
        for (; j < pl_end; ++j) {
            const float4 q = placed[j];
            const float dx = wx - q.x, dy = wy - q.y, dz = wz - q.z;
            const float d = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
            best = fminf(best, d - q.w);
        }
        clr = fminf(clr, best - c.w);
    }
    if (bad) clr = __builtin_nanf("");
    if (live) {
        if (clr_out) clr_out[t] = clr;
        if (col_out) col_out[t] = clr >= margin ? 0 : 1;
    }
    const unsigned long long nbad = __ballot(bad && live);
    if (nbad && (threadIdx.x & (kWave - 1)) == 0) {
        atomicOr(counters + kErrorWord, (unsigned long long)kErrNonFinite);
        atomicAdd(counters + kNonFinite, (unsigned long long)__popcll(nbad));
    }
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
    dim3 grid(b.n_scenes, (max_cand + 255) / 256);
    auto* ctr = (unsigned long long*)counters;
    if (b.grid_off) {
        hipError_t e = launch_scan_grid_values(b, counters, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_check<true>, grid, dim3(256), 0, st, b.obj_off, b.sph_off,
                           (const float4*)b.tmpl, b.obj_sup, b.sup, b.box_off, b.box, b.grid_off,
                           b.grid, b.grid_src, b.grid_val_off, b.grid_val,
                           (const float4*)b.placed, b.n_placed, obj_idx, cand_off, P.x, P.y, P.z,
                           P.yaw, margin, clr, col, ctr);
    } else {
        hipLaunchKernelGGL(k_check<false>, grid, dim3(256), 0, st, b.obj_off, b.sph_off,
                           (const float4*)b.tmpl, b.obj_sup, b.sup, b.box_off, b.box, nullptr,
                           nullptr, nullptr, nullptr, nullptr, (const float4*)b.placed,
                           b.n_placed, obj_idx, cand_off, P.x, P.y, P.z, P.yaw, margin, clr, col,
                           ctr);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Longest-first order.  Work estimate of a scene: its objects times its
// spheres (the pair work of a scene grows with both); 256 log-spaced buckets,
// largest first; scenes inside a bucket in arbitrary order (results do not
// depend on the order: scenes are independent).
__device__ __forceinline__ int work_bucket(const int32_t* __restrict__ obj_off,
                                           const int32_t* __restrict__ sph_off,
                                           const int32_t* __restrict__ box_off, int s) {
    const int o0 = obj_off[s], o1 = obj_off[s + 1];
    const float w = (float)(o1 - o0) * (float)(sph_off[o1] - sph_off[o0] + 16 * (box_off[s + 1] - box_off[s])) + 1.f;
    const int bk = (int)(__log2f(w) * 6.0f);
    return kOrderBuckets - 1 - min(max(bk, 0), kOrderBuckets - 1);
}

__global__ void k_order_hist(int n, const int32_t* __restrict__ obj_off,
                             const int32_t* __restrict__ sph_off,
                             const int32_t* __restrict__ box_off, int32_t* __restrict__ hist) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) atomicAdd(hist + work_bucket(obj_off, sph_off, box_off, s), 1);
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

__global__ void k_order_scatter(int n, const int32_t* __restrict__ obj_off,
                                const int32_t* __restrict__ sph_off,
                                const int32_t* __restrict__ box_off, int32_t* __restrict__ hist,
                                int32_t* __restrict__ order) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) order[atomicAdd(hist + work_bucket(obj_off, sph_off, box_off, s), 1)] = s;
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
                       b.box_off, hist);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(kOrderBuckets), 0, st, hist);
    hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(256), 0, st, n, b.obj_off, b.sph_off,
                       b.box_off, hist, order);
    return hipGetLastError();
}

}  // namespace scn
