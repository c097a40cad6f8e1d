// kernels.hip -- the libscn hot path on gfx950 (wave64, CDNA4).
//
//   k_reset   scene/record reset (graph-safe fill, no hipMemset)
//   k_sample  candidate poses of one attempt, one lane per candidate
//   k_check   dense exact clearance, one lane per candidate, obstacles
//             wave-uniform (scalar loads from the read-only tables)
//   k_place   persistent fused place kernel: one workgroup per scene loops
//             over the scene's objects and attempts; one wave per candidate
//             with the object's spheres across the lanes; placed spheres and
//             object bounds of the scene live in LDS; first-valid selection by
//             an LDS atomicMin over candidate indices.
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
    uint8_t* __restrict__ col_out) {
    const int s = blockIdx.x;
    const int o = obj_idx[s];
    if (o < obj_off[s] || o >= obj_off[s + 1]) return;   // -1 or not an object of scene s
    const int c0 = cand_off[s], c1 = cand_off[s + 1];
    const int tbase = c0 + blockIdx.y * blockDim.x;
    if (tbase >= c1) return;
    const int t = tbase + threadIdx.x;
    const bool live = t < c1;
    const int tt = live ? t : c1 - 1;

    const Support U = load_support(sup, obj_sup[o]);
    float sn, cs;
    sincosf(pyaw[tt], &sn, &cs);
    const float x = px[tt], y = py[tt], z = pz[tt];
    // candidate -> world: Rw = R_u Rz(yaw), tw = R_u (x,y,z) + t_u
    float Rw[9], tw[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        Rw[3 * r + 0] = fmaf(U.R[3 * r + 0], cs, U.R[3 * r + 1] * sn);
        Rw[3 * r + 1] = fmaf(-U.R[3 * r + 0], sn, U.R[3 * r + 1] * cs);
        Rw[3 * r + 2] = U.R[3 * r + 2];
        tw[r] = fmaf(U.R[3 * r + 0], x, fmaf(U.R[3 * r + 1], y, fmaf(U.R[3 * r + 2], z, U.t[r])));
    }
    const int oo = obj_off[s];
    const int first = sph_off[oo];
    const int pl_end = sph_off[oo + min(max(n_placed[s], 0), obj_off[s + 1] - oo)];
    const int b0 = box_off[s], b1 = box_off[s + 1];
    int g0 = 0, g1 = 0;
    if (kGrids) { g0 = grid_off[s]; g1 = grid_off[s + 1]; }

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
                best = fminf(best, grid_sample(G, grid_val + grid_val_off[grid_src[g]], wx, wy, wz));
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
    if (live) {
        if (clr_out) clr_out[t] = clr;
        if (col_out) col_out[t] = clr < margin ? 1 : 0;
    }
}

hipError_t launch_check(const scn_batch& b, const int32_t* obj_idx, const int32_t* cand_off,
                        int max_cand, scn_poses P, float margin, float* clr, uint8_t* col,
                        hipStream_t st) {
    if (b.n_scenes == 0 || max_cand == 0) return hipSuccess;
    dim3 grid(b.n_scenes, (max_cand + 255) / 256);
    if (b.grid_off) {
        hipLaunchKernelGGL(k_check<true>, grid, dim3(256), 0, st, b.obj_off, b.sph_off,
                           (const float4*)b.tmpl, b.obj_sup, b.sup, b.box_off, b.box, b.grid_off,
                           b.grid, b.grid_src, b.grid_val_off, b.grid_val,
                           (const float4*)b.placed, b.n_placed, obj_idx, cand_off, P.x, P.y, P.z,
                           P.yaw, margin, clr, col);
    } else {
        hipLaunchKernelGGL(k_check<false>, grid, dim3(256), 0, st, b.obj_off, b.sph_off,
                           (const float4*)b.tmpl, b.obj_sup, b.sup, b.box_off, b.box, nullptr,
                           nullptr, nullptr, nullptr, nullptr, (const float4*)b.placed,
                           b.n_placed, obj_idx, cand_off, P.x, P.y, P.z, P.yaw, margin, clr, col);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Persistent fused place kernel.
//
// One workgroup of W waves owns scene s for the whole launch.  For each of
// the scene's remaining objects (up to max_steps), attempts a = 0..retries:
// wave w evaluates candidates i = w, w+W, w+2W, ... in increasing order; a
// lane computes the pose of one of the wave's next 64 candidates (Philox in
// parallel), then the wave walks them one at a time with the object's
// spheres spread over the lanes (SPL spheres per lane).  A candidate is
// rejected at the first obstacle that any lane hits (ballot); placed objects
// whose bounding spheres are farther apart than the margin are skipped
// (exact: no sphere pair inside can be closer).  A collision-free candidate
// lowers the scene's best index (LDS atomicMin) and ends that wave's search;
// waves stop as soon as the best index is below their next candidate, so the
// result is exactly the lowest collision-free index.
template <int SPL>
__global__ __launch_bounds__(512) void k_place(
    const int32_t* __restrict__ obj_off, const int32_t* __restrict__ sph_off,
    const float4* __restrict__ tmpl, const int32_t* __restrict__ obj_sup,
    const int32_t* __restrict__ obj_ncand, const float* __restrict__ sup,
    const int32_t* __restrict__ box_off, const float* __restrict__ box,
    float4* __restrict__ placed, int32_t* __restrict__ n_placed, int8_t* __restrict__ status,
    scn_pose_rec* __restrict__ rec, int32_t* __restrict__ chosen,
    unsigned long long* __restrict__ counters, uint64_t seed, float margin, int retries,
    int default_ncand, int max_steps, int cap_sph, int cap_obj) {
    extern __shared__ float4 lds[];
    float4* lsph = lds;            // placed spheres of this scene: (x, y, z, r + margin)
    float4* lbnd = lds + cap_sph;  // world bounding sphere of each placed object
    __shared__ int s_best[2];

    const int s = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform_int(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;

    if (status[s] != SCN_SCENE_ACTIVE) {
        if (chosen && threadIdx.x == 0) chosen[s] = -2;
        return;
    }
    const int o0 = obj_off[s], o1 = obj_off[s + 1];
    const int nobj = o1 - o0;
    const int first = sph_off[o0];
    int too_big = 0;
    for (int ob = o0 + (int)threadIdx.x; ob < o1; ob += blockDim.x)
        too_big |= (sph_off[ob + 1] - sph_off[ob]) > kWave * SPL;
    too_big = __syncthreads_or(too_big);
    if (too_big || sph_off[o1] - first > cap_sph || nobj > cap_obj) {
        if (threadIdx.x == 0) {
            atomicOr(counters + kErrorWord, (unsigned long long)kErrCapacity);
            if (chosen) chosen[s] = -2;
        }
        return;
    }
    int j = min(max(n_placed[s], 0), nobj);
    const int j_end = max_steps > 0 ? min(nobj, j + max_steps) : nobj;

    // Stage the already placed spheres and their objects' bounding spheres.
    const int n_stage = sph_off[o0 + j] - first;
    for (int i = threadIdx.x; i < n_stage; i += blockDim.x) {
        float4 q = placed[first + i];
        q.w += margin;
        lsph[i] = q;
    }
    for (int ob = wave; ob < j; ob += W) {
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
    __syncthreads();

    unsigned long long n_cand = 0, n_pairs = 0, n_boxp = 0, n_att = 0, n_done = 0, n_xf = 0;
    int8_t fin = SCN_SCENE_ACTIVE;
    int last = -2;
    const int b0 = box_off[s], b1 = box_off[s + 1];
    int phase = 0;

    for (; j < j_end; ++j) {
        const int o = o0 + j;
        const int sb = sph_off[o];
        const int S = sph_off[o + 1] - sb;
        float cx[SPL], cy[SPL], cz[SPL], cr[SPL], rm2[SPL];
        bool act[SPL];
        float lift = -1e30f, lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            const int k = lane + kWave * q;
            act[q] = k < S;
            const float4 c = act[q] ? tmpl[sb + k] : make_float4(0.f, 0.f, 0.f, 0.f);
            cx[q] = c.x; cy[q] = c.y; cz[q] = c.z; cr[q] = c.w;
            rm2[q] = (c.w + margin) * (c.w + margin);
            if (act[q]) {
                lift = fmaxf(lift, c.w - c.z);
                lo[0] = fminf(lo[0], c.x - c.w); hi[0] = fmaxf(hi[0], c.x + c.w);
                lo[1] = fminf(lo[1], c.y - c.w); hi[1] = fmaxf(hi[1], c.y + c.w);
                lo[2] = fminf(lo[2], c.z - c.w); hi[2] = fmaxf(hi[2], c.z + c.w);
            }
        }
        lift = wave_max(lift);
        float bc[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) bc[d] = 0.5f * (wave_min(lo[d]) + wave_max(hi[d]));
        float rho = 0.f;
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            if (act[q]) {
                const float dx = cx[q] - bc[0], dy = cy[q] - bc[1], dz = cz[q] - bc[2];
                rho = fmaxf(rho, sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))) + cr[q]);
            }
        }
        rho = wave_max(rho) * (1.0f + 1e-6f) + 1e-6f;

        const Support U = load_support(sup, obj_sup[o]);
        const float ax = U.hx - U.inset, ay = U.hy - U.inset, zc = U.lift + lift;
        const int C = obj_ncand ? obj_ncand[o] : default_ncand;
        int found = -1, found_att = -1;

        for (int a = 0; a <= retries; ++a) {
            int* best = &s_best[phase];
            if (threadIdx.x == 0) *best = INT_MAX;
            __syncthreads();
            if (wave == 0) ++n_att;
            bool stop = false;
            for (int base = 0; !stop; base += kWave) {
                if (wave + W * base >= C) break;
                const Pose L = sample_pose(seed, (uint32_t)s, (uint32_t)j, (uint32_t)a,
                                           (uint32_t)(wave + W * (base + lane)), ax, ay, zc);
                for (int t = 0; t < kWave; ++t) {
                    const int i = wave + W * (base + t);
                    if (i >= C) { stop = true; break; }
                    const int cur = uniform_int(
                        __hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                    if (cur < i) { stop = true; break; }
                    Pose P;
                    P.x = bcast(L.x, t); P.y = bcast(L.y, t); P.z = zc;
                    P.c = bcast(L.c, t); P.s = bcast(L.s, t);
                    ++n_cand;
                    n_xf += S;
                    float wx[SPL], wy[SPL], wz[SPL];
#pragma unroll
                    for (int q = 0; q < SPL; ++q) to_world(U, P, cx[q], cy[q], cz[q], wx[q], wy[q], wz[q]);
                    bool hit = false;
                    // static boxes
                    for (int bx = b0; bx < b1; ++bx) {
                        const float* B = box + 16 * bx;
#pragma unroll
                        for (int q = 0; q < SPL; ++q)
                            hit |= act[q] && box_out2(B, wx[q], wy[q], wz[q]) < rm2[q];
                        n_boxp += S;
                        if (__ballot(hit)) break;
                    }
                    if (!__ballot(hit) && j > 0) {
                        float gx, gy, gz;
                        to_world(U, P, bc[0], bc[1], bc[2], gx, gy, gz);
                        for (int ob = 0; ob < j; ++ob) {
                            const float4 bd = lbnd[ob];
                            const float dx = gx - bd.x, dy = gy - bd.y, dz = gz - bd.z;
                            const float lim = rho + bd.w + margin;
                            if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) >= lim * lim) continue;
                            const int a0 = sph_off[o0 + ob] - first, a1 = sph_off[o0 + ob + 1] - first;
                            for (int k = a0; k < a1; ++k) {
                                const float4 qs = lsph[k];
#pragma unroll
                                for (int q = 0; q < SPL; ++q) {
                                    const float ex = wx[q] - qs.x, ey = wy[q] - qs.y, ez = wz[q] - qs.z;
                                    const float rr = cr[q] + qs.w;
                                    hit |= act[q] && fmaf(-rr, rr, fmaf(ex, ex, fmaf(ey, ey, ez * ez))) < 0.f;
                                }
                            }
                            n_pairs += (unsigned long long)S * (unsigned long long)(a1 - a0);
                            if (__ballot(hit)) break;
                        }
                    }
                    if (!__ballot(hit)) {
                        if (lane == 0) atomicMin(best, i);
                        stop = true;
                        break;
                    }
                }
            }
            __syncthreads();
            const int b = *best;
            phase ^= 1;
            if (b != INT_MAX) { found = b; found_att = a; break; }
        }
        if (found < 0) { fin = SCN_SCENE_INVALID; last = -1; break; }
        if (wave == 0) {
            const Pose P = sample_pose(seed, (uint32_t)s, (uint32_t)j, (uint32_t)found_att,
                                       (uint32_t)found, ax, ay, zc);
#pragma unroll
            for (int q = 0; q < SPL; ++q) {
                if (act[q]) {
                    float wx, wy, wz;
                    to_world(U, P, cx[q], cy[q], cz[q], wx, wy, wz);
                    const int k = lane + kWave * q;
                    placed[sb + k] = make_float4(wx, wy, wz, cr[q]);
                    lsph[sb - first + k] = make_float4(wx, wy, wz, cr[q] + margin);
                }
            }
            if (lane == 0) {
                float gx, gy, gz;
                to_world(U, P, bc[0], bc[1], bc[2], gx, gy, gz);
                lbnd[j] = make_float4(gx, gy, gz, rho);
                rec[o] = scn_pose_rec{P.x, P.y, P.z, P.yaw, found_att, found};
            }
            ++n_done;
        }
        last = found;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        n_placed[s] = j;
        status[s] = fin != SCN_SCENE_ACTIVE ? fin : (j == nobj ? SCN_SCENE_VALID : SCN_SCENE_ACTIVE);
        if (chosen) chosen[s] = last;
    }
    if (lane == 0) {
        atomicAdd(counters + kCandidates, n_cand);
        atomicAdd(counters + kSpherePairs, n_pairs);
        atomicAdd(counters + kBoxPairs, n_boxp);
        atomicAdd(counters + kTransforms, n_xf);
        if (n_att) atomicAdd(counters + kAttempts, n_att);
        if (n_done) atomicAdd(counters + kPlaced, n_done);
    }
}

int place_max_lds_bytes() { return 160 * 1024; }

hipError_t launch_place(const scn_batch& b, const scn_gen_args& a, const PlacePlan& plan,
                        int32_t* chosen, int64_t* counters, hipStream_t st) {
    if (b.n_scenes == 0) return hipSuccess;
    dim3 grid(b.n_scenes), block(kWave * plan.waves);
    auto* ctr = (unsigned long long*)counters;
#define SCN_LAUNCH_PLACE(SPLV)                                                                  \
    do {                                                                                        \
        auto kern = k_place<SPLV>;                                                              \
        if (plan.lds_bytes > 64 * 1024) {                                                       \
            hipError_t e = hipFuncSetAttribute((const void*)kern,                               \
                                               hipFuncAttributeMaxDynamicSharedMemorySize,      \
                                               plan.lds_bytes);                                 \
            if (e != hipSuccess) return e;                                                      \
        }                                                                                       \
        hipLaunchKernelGGL(kern, grid, block, plan.lds_bytes, st, b.obj_off, b.sph_off,         \
                           (const float4*)b.tmpl, b.obj_sup, b.obj_ncand, b.sup, b.box_off,     \
                           b.box, (float4*)b.placed, b.n_placed, b.status, b.rec, chosen, ctr,  \
                           a.seed, a.margin, a.retries, a.default_ncand, plan.max_steps,        \
                           plan.cap_sph, plan.cap_obj);                                         \
    } while (0)
    switch (plan.spl) {
        case 1: SCN_LAUNCH_PLACE(1); break;
        case 2: SCN_LAUNCH_PLACE(2); break;
        case 4: SCN_LAUNCH_PLACE(4); break;
        default: return hipErrorInvalidValue;
    }
#undef SCN_LAUNCH_PLACE
    return hipGetLastError();
}

}  // namespace scn
