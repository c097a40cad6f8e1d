// learned.hip -- state features, proposal ranking and label harvesting for
// the learned pose proposal.
//
//   k_descriptor     32 sphere-set moments per object (object frame)
//   k_hmap_boxes     64 x 64 height map of a scene's support from its boxes
//   k_hmap_raise     raise the map by one placed object's spheres
//   k_features       BF16 network input rows: [10 x height map, descriptor]
//   k_topk_*         top-k pose bins per state (radix selection, or a
//                    bitonic sort in LDS for large k)
//   k_harvest        uniform label candidates of a state with their bins and
//                    accept / reject from the exact checker (distance form)
#include <climits>

#include "device.h"
#include "internal.h"

namespace scn {

// ---------------------------------------------------------------------------
// Descriptor (one wave per object; values in decimetres where lengths):
//  0 S/256 | 1-4 mean/min/max/std radius x10 | 5 sum r^3 x1e3 |
//  6-8 r^3-weighted centroid x10 | 9-14 centre covariance xx,yy,zz,xy,xz,yz x100 |
//  15-17 sphere-set AABB half extents x10 | 18 rest lift x10 |
//  19 resting top height x10 | 20 footprint radius x10 | 21-31 zero
__global__ __launch_bounds__(64) void k_descriptor(int n_obj, const int32_t* __restrict__ sph_off,
                                                   const float4* __restrict__ tmpl,
                                                   float* __restrict__ desc) {
    const int o = blockIdx.x;
    if (o >= n_obj) return;
    const int lane = threadIdx.x;
    const int k0 = sph_off[o], k1 = sph_off[o + 1];
    const int S = k1 - k0;
    auto sum = [](float x) {
        for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, kWave);
        return x;
    };
    // first pass: sums, extremes and weighted sums
    float sr = 0.f, rmin = 1e30f, rmax = -1e30f, v = 0.f, wx = 0.f, wy = 0.f, wz = 0.f;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
    float lift = -1e30f, top = -1e30f, foot = 0.f;
    for (int k = k0 + lane; k < k1; k += kWave) {
        const float4 c = tmpl[k];
        const float r3 = c.w * c.w * c.w;
        sr += c.w; rmin = fminf(rmin, c.w); rmax = fmaxf(rmax, c.w);
        v += r3; wx += r3 * c.x; wy += r3 * c.y; wz += r3 * c.z;
        sx += c.x; sy += c.y; sz += c.z;
        lo[0] = fminf(lo[0], c.x - c.w); hi[0] = fmaxf(hi[0], c.x + c.w);
        lo[1] = fminf(lo[1], c.y - c.w); hi[1] = fmaxf(hi[1], c.y + c.w);
        lo[2] = fminf(lo[2], c.z - c.w); hi[2] = fmaxf(hi[2], c.z + c.w);
        lift = fmaxf(lift, c.w - c.z);
        top = fmaxf(top, c.z + c.w);
        foot = fmaxf(foot, sqrtf(c.x * c.x + c.y * c.y) + c.w);
    }
    sr = sum(sr); v = sum(v); wx = sum(wx); wy = sum(wy); wz = sum(wz);
    sx = sum(sx); sy = sum(sy); sz = sum(sz);
    rmin = wave_min(rmin); rmax = wave_max(rmax);
    for (int d = 0; d < 3; ++d) { lo[d] = wave_min(lo[d]); hi[d] = wave_max(hi[d]); }
    lift = wave_max(lift); top = wave_max(top); foot = wave_max(foot);
    const float n = (float)(S > 0 ? S : 1);
    const float mr = sr / n;
    const float mx = sx / n, my = sy / n, mz = sz / n;
    // second pass: centred second moments
    float vr = 0.f, cxx = 0.f, cyy = 0.f, czz = 0.f, cxy = 0.f, cxz = 0.f, cyz = 0.f;
    for (int k = k0 + lane; k < k1; k += kWave) {
        const float4 c = tmpl[k];
        const float dr = c.w - mr, dx = c.x - mx, dy = c.y - my, dz = c.z - mz;
        vr += dr * dr;
        cxx += dx * dx; cyy += dy * dy; czz += dz * dz;
        cxy += dx * dy; cxz += dx * dz; cyz += dy * dz;
    }
    vr = sum(vr); cxx = sum(cxx); cyy = sum(cyy); czz = sum(czz);
    cxy = sum(cxy); cxz = sum(cxz); cyz = sum(cyz);
    if (lane != 0) return;
    float* D = desc + 32 * (size_t)o;
    const float iv = v > 0.f ? 1.f / v : 0.f;
    D[0] = (float)S / 256.f;
    D[1] = 10.f * mr;
    D[2] = 10.f * (S ? rmin : 0.f);
    D[3] = 10.f * (S ? rmax : 0.f);
    D[4] = 10.f * sqrtf(vr / n);
    D[5] = 1e3f * v;
    D[6] = 10.f * wx * iv; D[7] = 10.f * wy * iv; D[8] = 10.f * wz * iv;
    D[9] = 100.f * cxx / n;
    D[10] = 100.f * cyy / n;
    D[11] = 100.f * czz / n;
    D[12] = 100.f * cxy / n;
    D[13] = 100.f * cxz / n;
    D[14] = 100.f * cyz / n;
    for (int d = 0; d < 3; ++d) D[15 + d] = 10.f * 0.5f * (S ? hi[d] - lo[d] : 0.f);
    D[18] = 10.f * (S ? lift : 0.f);
    D[19] = 10.f * (S ? top + lift : 0.f);
    D[20] = 10.f * foot;
    for (int d = 21; d < 32; ++d) D[d] = 0.f;
}

hipError_t launch_descriptor(const scn_batch& b, float* desc, hipStream_t st) {
    if (b.n_objects == 0) return hipSuccess;
    hipLaunchKernelGGL(k_descriptor, dim3(b.n_objects), dim3(64), 0, st, b.n_objects, b.sph_off,
                       (const float4*)b.tmpl, desc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Height maps, one per support (64 x 64 floats at hmap + 4096 u): cell (ix,
// iy), ix along x in [0,64), iy along y, centre (-hx + (ix + 1/2) 2hx/64,
// -hy + ...); value = max(0, box tops, sphere tops) above the support plane,
// metres.  The boxes are those of the support's scene; the spheres those of
// the scene's placed objects that rest on the support.  A box covers a cell
// when the cell centre at the box centre's height lies in the box's x/y extent
// (box frame); its top is the box's highest point.  A sphere (support-frame
// centre p, radius r) covers a cell when the cell centre is within r of p in
// x/y; its top there is p_z + sqrt(r^2 - d^2).
//
// The box part: one workgroup per scene writes the map of every support its
// objects rest on (each once: at the first object on it); supports without
// objects are not written.  A support belongs to one scene.
__global__ __launch_bounds__(256) void k_hmap_boxes(
    int n, const int32_t* __restrict__ obj_off, const int32_t* __restrict__ obj_sup,
    const float* __restrict__ sup, const int32_t* __restrict__ box_off,
    const float* __restrict__ box, float* __restrict__ hmap) {
    const int s = blockIdx.x;
    if (s >= n) return;
    const int o0 = obj_off[s], o1 = obj_off[s + 1];
    const int b0 = box_off[s], b1 = box_off[s + 1];
    for (int o = o0; o < o1; ++o) {
        const int u = obj_sup[o];
        bool seen = false;
        for (int e = o0; e < o && !seen; ++e) seen = obj_sup[e] == u;
        if (seen) continue;   // uniform: every thread reads the same entries
        const SupportFrame F = support_frame(sup, u);
        for (int cell = threadIdx.x; cell < 4096; cell += blockDim.x) {
            const int ix = cell >> 6, iy = cell & 63;
            const float cx = -F.hx + (ix + 0.5f) * (2.f * F.hx / 64.f);
            const float cy = -F.hy + (iy + 0.5f) * (2.f * F.hy / 64.f);
            float h = 0.f;
            for (int b = b0; b < b1; ++b) {
                const float* B = box + 16 * b;
                // box centre and axes in the support frame
                float bcx, bcy, bcz;
                to_support(F, B[9], B[10], B[11], bcx, bcy, bcz);
                float ax[3][3];   // ax[a] = support-frame direction of box axis a
                for (int a = 0; a < 3; ++a) {
                    float ux, uy, uz;
                    ux = F.R[0] * B[a] + F.R[3] * B[3 + a] + F.R[6] * B[6 + a];
                    uy = F.R[1] * B[a] + F.R[4] * B[3 + a] + F.R[7] * B[6 + a];
                    uz = F.R[2] * B[a] + F.R[5] * B[3 + a] + F.R[8] * B[6 + a];
                    ax[a][0] = ux; ax[a][1] = uy; ax[a][2] = uz;
                }
                const float dx = cx - bcx, dy = cy - bcy;   // at the centre's height
                const float qx = ax[0][0] * dx + ax[0][1] * dy;
                const float qy = ax[1][0] * dx + ax[1][1] * dy;
                if (fabsf(qx) <= B[12] && fabsf(qy) <= B[13]) {
                    const float topz = bcz + fabsf(ax[0][2]) * B[12] + fabsf(ax[1][2]) * B[13] +
                                       fabsf(ax[2][2]) * B[14];
                    h = fmaxf(h, topz);
                }
            }
            hmap[(size_t)u * 4096 + cell] = h;
        }
    }
}

// Raise the map of object o's support by its placed spheres (world frame,
// k0 .. k1-1).  One wave, one sphere per lane at a time; monotone max through
// integer atomics on non-negative floats.
__device__ void raise_object(int o, int k0, int k1, const int32_t* __restrict__ obj_sup,
                             const float* __restrict__ sup, const float4* __restrict__ placed,
                             float* __restrict__ hmap) {
    const int u = obj_sup[o];
    const SupportFrame F = support_frame(sup, u);
    for (int k = k0 + threadIdx.x; k < k1; k += kWave) {
        const float4 q = placed[k];
        hmap_raise_sphere(F, hmap + (size_t)u * 4096, q.x, q.y, q.z, q.w);
    }
}

// Raise the height maps by each scene's object obj_idx[s] (-1: none), or by
// its first n_state[s] objects, whose world spheres are in placed.
__global__ __launch_bounds__(64) void k_hmap_raise(
    int n, const int32_t* __restrict__ obj_off, const int32_t* __restrict__ obj_sup,
    const float* __restrict__ sup, const int32_t* __restrict__ sph_off,
    const float4* __restrict__ placed, const int32_t* __restrict__ obj_idx,
    const int32_t* __restrict__ n_state, float* __restrict__ hmap) {
    const int s = blockIdx.x;
    if (s >= n) return;
    if (n_state) {
        const int m = min(max(n_state[s], 0), obj_off[s + 1] - obj_off[s]);
        for (int o = obj_off[s]; o < obj_off[s] + m; ++o)
            raise_object(o, sph_off[o], sph_off[o + 1], obj_sup, sup, placed, hmap);
    } else {
        const int o = obj_idx[s];
        if (o < obj_off[s] || o >= obj_off[s + 1]) return;
        raise_object(o, sph_off[o], sph_off[o + 1], obj_sup, sup, placed, hmap);
    }
}

// The scene each support belongs to (sup_scene[u], -1 where no object rests
// on it); a support that objects of two scenes rest on sets
// kErrSharedSupport.  One thread per scene.
__global__ void k_support_scene(int n, const int32_t* __restrict__ obj_off,
                                const int32_t* __restrict__ obj_sup, int32_t* __restrict__ sup_scene,
                                unsigned long long* __restrict__ counters) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    bool shared = false;
    for (int o = obj_off[s]; o < obj_off[s + 1]; ++o) {
        const int prev = atomicCAS(sup_scene + obj_sup[o], -1, s);
        shared |= prev != -1 && prev != s;
    }
    if (shared) atomicOr(counters + kErrorWord, (unsigned long long)kErrSharedSupport);
}

hipError_t launch_support_scene(const scn_batch& b, int32_t* sup_scene, int64_t* counters,
                                hipStream_t st) {
    if (b.n_scenes == 0) return hipSuccess;
    if (hipError_t e = launch_fill_i32(sup_scene, b.n_supports, -1, st)) return e;
    hipLaunchKernelGGL(k_support_scene, dim3((b.n_scenes + 255) / 256), dim3(256), 0, st,
                       b.n_scenes, b.obj_off, b.obj_sup, sup_scene,
                       (unsigned long long*)counters);
    return hipGetLastError();
}

// The learned pipeline's plan of one tick: the active scenes below the
// objects cap that still have an object to place, split into those that start
// a new object (resume[s] == 0: they need proposals; list[0 ..), with the
// object in obj_idx by row) and those resuming the uniform entries of a
// pending one (list[n ..)).  count[0] and count[1] (zeroed by the caller)
// receive the two sizes.
// Appends are aggregated per wave, so the order within each list is not the
// scene order; each scene's step does not depend on it.
__global__ __launch_bounds__(256) void k_tick_plan(int n, const int32_t* __restrict__ obj_off,
                                                   const int32_t* __restrict__ n_placed,
                                                   const int8_t* __restrict__ status,
                                                   const int32_t* __restrict__ resume, int j_cap,
                                                   int32_t* __restrict__ list,
                                                   int32_t* __restrict__ obj_idx,
                                                   int32_t* __restrict__ count) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    bool fresh = false, pending = false;
    int j = 0;
    if (s < n && status[s] == SCN_SCENE_ACTIVE) {
        j = n_placed[s];
        if (j < obj_off[s + 1] - obj_off[s] && (j_cap <= 0 || j < j_cap)) {
            fresh = resume[s] == 0;
            pending = !fresh;
        }
    }
    const unsigned long long lower = lane ? (~0ull >> (kWave - lane)) : 0ull;
    const unsigned long long mf = __ballot(fresh), mp = __ballot(pending);
    int base_f = 0, base_p = 0;
    if (lane == 0) {
        if (mf) base_f = atomicAdd(count, __popcll(mf));
        if (mp) base_p = atomicAdd(count + 1, __popcll(mp));
    }
    base_f = __shfl(base_f, 0, kWave);
    base_p = __shfl(base_p, 0, kWave);
    if (fresh) {
        const int r = base_f + __popcll(mf & lower);
        list[r] = s;
        obj_idx[r] = obj_off[s] + j;
    }
    if (pending) list[n + base_p + __popcll(mp & lower)] = s;
}

hipError_t launch_tick_plan(const scn_batch& b, const int32_t* resume, int j_cap, int32_t* list,
                            int32_t* obj_idx, int32_t* count, hipStream_t st) {
    if (b.n_scenes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tick_plan, dim3((b.n_scenes + 255) / 256), dim3(256), 0, st, b.n_scenes,
                       b.obj_off, b.n_placed, b.status, resume, j_cap, list, obj_idx, count);
    return hipGetLastError();
}

hipError_t launch_hmap_boxes(const scn_batch& b, float* hmap, hipStream_t st) {
    if (b.n_scenes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hmap_boxes, dim3(b.n_scenes), dim3(256), 0, st, b.n_scenes, b.obj_off,
                       b.obj_sup, b.sup, b.box_off, b.box, hmap);
    return hipGetLastError();
}

hipError_t launch_hmap_raise(const scn_batch& b, const int32_t* obj_idx, const int32_t* n_state,
                             float* hmap, hipStream_t st) {
    if (b.n_scenes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hmap_raise, dim3(b.n_scenes), dim3(64), 0, st, b.n_scenes, b.obj_off,
                       b.obj_sup, b.sup, b.sph_off, (const float4*)b.placed, obj_idx, n_state,
                       hmap);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Feature rows x[r] = [10 * hmap[u] (4096), desc[o] (32)] as BF16 for
// object o = obj_idx[r] on support u = obj_sup[o]; zeros for rows with
// obj_idx < 0.  Row length ld >= 4128.  With m_dev only rows below *m_dev are
// written.
__global__ __launch_bounds__(256) void k_features(int n, const float* __restrict__ hmap,
                                                 const float* __restrict__ desc,
                                                 const int32_t* __restrict__ obj_idx,
                                                 const int32_t* __restrict__ obj_sup, int ld,
                                                 __bf16* __restrict__ x,
                                                 const int32_t* __restrict__ m_dev) {
    const int r = blockIdx.x;
    if (r >= n || (m_dev && r >= *m_dev)) return;
    const int o = obj_idx[r];
    const size_t u = o >= 0 ? (size_t)obj_sup[o] : 0;   // the support of feature row r
    __bf16* row = x + (size_t)r * ld;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        float v = 0.f;
        if (o >= 0) {
            if (i < 4096) v = 10.f * hmap[u * 4096 + i];
            else if (i < 4128) v = desc[32 * (size_t)o + (i - 4096)];
        }
        row[i] = (__bf16)v;
    }
}

hipError_t launch_features(int n, const float* hmap, const float* desc, const int32_t* obj_idx,
                           const int32_t* obj_sup, int ld, void* x, hipStream_t st,
                           const int32_t* m_dev) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3(n), dim3(256), 0, st, n, hmap, desc, obj_idx, obj_sup, ld,
                       (__bf16*)x, m_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Top-k bins per row of logits [M][4096]: bins in rank order (logit
// descending, ties to the lower bin; NaN ranks last).  Rows with
// active[m] < 0 are skipped (active may be nullptr).  Row m's bins go to
// bins[rows[m]] (scattered back to its scene) or bins[m]; with m_dev only
// rows below *m_dev are ranked.
//
// The rank order is the descending order of the unique 64-bit key
// (orderable(logit) << 32) | (4095 - bin).
__device__ __forceinline__ unsigned orderable(float f) {
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ unsigned logit_key(float v) {
    if (v != v) v = -__builtin_huge_valf();
    if (v == 0.f) v = 0.f;   // -0 ties with +0
    return orderable(v);
}

// k <= kSelMax: radix selection of the k-th largest 32-bit value (four 8-bit
// digits, histograms in LDS), then the values above it and the lowest-bin
// ties at it are gathered and ranked by counting.  256 threads per row, 16
// logits per thread (thread t owns bins 16t .. 16t+15).
constexpr int kSelMax = 256;
__global__ __launch_bounds__(256) void k_topk_select(int M, const float* __restrict__ logits, int k,
                                                     const int32_t* __restrict__ active,
                                                     int32_t* __restrict__ bins,
                                                     const int32_t* __restrict__ rows,
                                                     const int32_t* __restrict__ m_dev) {
    __shared__ unsigned hist[256];
    __shared__ unsigned s_prefix, s_need, s_count;
    __shared__ unsigned s_tie_count[256];
    __shared__ unsigned long long sel[kSelMax];
    const int m = blockIdx.x;
    if (m >= M || (m_dev && m >= *m_dev)) return;
    if (active && active[m] < 0) return;
    const size_t out = rows ? (size_t)rows[m] : (size_t)m;   // the row's bins go to row `out`
    const int t = threadIdx.x;
    const float4* z4 = reinterpret_cast<const float4*>(logits + (size_t)m * 4096) + 4 * t;
    unsigned v[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 f = z4[q];
        v[4 * q] = logit_key(f.x); v[4 * q + 1] = logit_key(f.y);
        v[4 * q + 2] = logit_key(f.z); v[4 * q + 3] = logit_key(f.w);
    }
    if (t == 0) { s_prefix = 0u; s_need = (unsigned)k; s_count = 0u; }
    // digit passes, most significant first: find the value T of rank k
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        const unsigned hi_mask = pass == 0 ? 0u : (0xFFFFFFFFu << (shift + 8));
        hist[t] = 0u;
        __syncthreads();
        const unsigned prefix = s_prefix;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if ((v[i] & hi_mask) == prefix) atomicAdd(&hist[(v[i] >> shift) & 0xFFu], 1u);
        __syncthreads();
        if (t < 64) {
            // wave 0 walks the digits from the top: 4 digits per lane
            unsigned c[4], tot = 0u;
#pragma unroll
            for (int d = 0; d < 4; ++d) { c[d] = hist[255 - (4 * t + d)]; tot += c[d]; }
            // inclusive scan of lane totals (lane 0 = highest digits)
            unsigned inc = tot;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned y = __shfl_up(inc, o, kWave);
                if (t >= o) inc += y;
            }
            const unsigned need = s_need;
            const unsigned before = inc - tot;
            if (before < need && inc >= need) {
                unsigned acc = before;
                for (int d = 0; d < 4; ++d) {
                    if (acc + c[d] >= need) {
                        const unsigned digit = 255u - (unsigned)(4 * t + d);
                        s_prefix = prefix | (digit << shift);
                        s_need = need - acc;
                        break;
                    }
                    acc += c[d];
                }
            }
        }
        __syncthreads();
    }
    const unsigned T = s_prefix;      // k-th largest value
    const unsigned n_tie = s_need;    // ties at T that enter, lowest bins first
    // count ties per thread, exclusive scan over threads (bin order)
    unsigned ties = 0u;
#pragma unroll
    for (int i = 0; i < 16; ++i) ties += v[i] == T;
    s_tie_count[t] = ties;
    __syncthreads();
    if (t < 64) {
        unsigned c[4], tot = 0u;
#pragma unroll
        for (int d = 0; d < 4; ++d) { c[d] = s_tie_count[4 * t + d]; tot += c[d]; }
        unsigned inc = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned y = __shfl_up(inc, o, kWave);
            if (t >= o) inc += y;
        }
        unsigned acc = inc - tot;
#pragma unroll
        for (int d = 0; d < 4; ++d) { s_tie_count[4 * t + d] = acc; acc += c[d]; }
    }
    __syncthreads();
    unsigned tie_rank = s_tie_count[t];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const unsigned bin = 16u * t + i;
        const unsigned long long key = ((unsigned long long)v[i] << 32) | (4095u - bin);
        bool take = v[i] > T;
        if (v[i] == T) { take = tie_rank < n_tie; ++tie_rank; }
        if (take) sel[atomicAdd(&s_count, 1u)] = key;
    }
    __syncthreads();
    // rank by counting (keys are unique)
    for (int i = t; i < k; i += 256) {
        const unsigned long long a = sel[i];
        int r = 0;
        for (int j = 0; j < k; ++j) r += sel[j] > a;
        bins[out * k + r] = 4095 - (int)(a & 0xFFFFFFFFu);
    }
}

// Any k: a bitonic sort of the 4096 keys in LDS, 1024 threads per row.
__global__ __launch_bounds__(1024) void k_topk_sort(int M, const float* __restrict__ logits, int k,
                                                    const int32_t* __restrict__ active,
                                                    int32_t* __restrict__ bins,
                                                    const int32_t* __restrict__ rows,
                                                    const int32_t* __restrict__ m_dev) {
    __shared__ unsigned long long key[4096];
    const int m = blockIdx.x;
    if (m >= M || (m_dev && m >= *m_dev)) return;
    if (active && active[m] < 0) return;
    const size_t out = rows ? (size_t)rows[m] : (size_t)m;
    const float* z = logits + (size_t)m * 4096;
    for (int i = threadIdx.x; i < 4096; i += blockDim.x)
        key[i] = ((unsigned long long)logit_key(z[i]) << 32) | (unsigned)(4095 - i);
    __syncthreads();
    for (int size = 2; size <= 4096; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < 4096; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    const unsigned long long a = key[i], b = key[j];
                    if (desc ? (a < b) : (a > b)) { key[i] = b; key[j] = a; }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < k; i += blockDim.x)
        bins[out * k + i] = 4095 - (int)(key[i] & 0xFFFFFFFFu);
}

hipError_t launch_topk(int M, const float* logits, int k, const int32_t* active, int32_t* bins,
                       hipStream_t st, const int32_t* rows, const int32_t* m_dev) {
    if (M == 0) return hipSuccess;
    if (k <= kSelMax && ((uintptr_t)logits & 15u) == 0)
        hipLaunchKernelGGL(k_topk_select, dim3(M), dim3(256), 0, st, M, logits, k, active, bins,
                           rows, m_dev);
    else
        hipLaunchKernelGGL(k_topk_sort, dim3(M), dim3(1024), 0, st, M, logits, k, active, bins,
                           rows, m_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Label harvesting.  For every scene s with obj_idx[s] >= 0, L uniform
// candidates of that object (Philox tag 2 in the attempt word: counter
// (i, 0x20000 | round, step, s)) are checked exactly against the scene's
// boxes, its voxel grids (trilinear) and its first n_placed[s] objects;
// bins[s][i] receives the pose bin and accept[s][i] 1 (collision-free) or 0.
// Lane per candidate, wave-uniform obstacles (like the dense checker).
// Non-finite input (the object's spheres or support row, a box row or placed
// sphere of the state) makes every label of the state a rejection, and a grid
// sample that reads a non-finite node rejects its label; either sets the
// non-finite error bit.
__global__ __launch_bounds__(64) void k_harvest(
    const int32_t* __restrict__ obj_off, const int32_t* __restrict__ sph_off,
    const float4* __restrict__ tmpl, const int32_t* __restrict__ obj_sup,
    const float* __restrict__ sup, const int32_t* __restrict__ box_off,
    const float* __restrict__ box, const float4* __restrict__ placed,
    const int32_t* __restrict__ n_state, int L, uint64_t seed, int round, float margin,
    int32_t* __restrict__ bins_out, float* __restrict__ accept_out,
    unsigned long long* __restrict__ counters, const int32_t* __restrict__ grid_off,
    const float* __restrict__ grid, const int32_t* __restrict__ grid_src,
    const int64_t* __restrict__ grid_val_off, const float* __restrict__ grid_val) {
    const int s = blockIdx.x;
    const int i = blockIdx.y * 64 + threadIdx.x;
    const int o = obj_off[s] + max(n_state[s], 0);   // the next object of the state
    if (o >= obj_off[s + 1]) {
        if (i < L) { bins_out[(size_t)s * L + i] = -1; accept_out[(size_t)s * L + i] = 0.f; }
        return;
    }
    const int ii = i < L ? i : L - 1;
    const Support U = load_support(sup, obj_sup[o]);
    float lift = -1e30f;
    for (int k = sph_off[o]; k < sph_off[o + 1]; ++k) lift = fmaxf(lift, tmpl[k].w - tmpl[k].z);
    const int j = o - obj_off[s];
    const U4 w = philox10(U4{(uint32_t)ii, 0x20000u | (uint32_t)round, (uint32_t)j, (uint32_t)s},
                          (uint32_t)seed, (uint32_t)(seed >> 32));
    const float u0 = unit01(w.a), u1 = unit01(w.b), u2 = unit01(w.c);
    Pose P;
    P.x = (U.hx - U.inset) * signed_unit(w.a);
    P.y = (U.hy - U.inset) * signed_unit(w.b);
    P.yaw = 6.28318530717958647692f * u2;
    sincospif(2.0f * u2, &P.s, &P.c);
    P.z = U.lift + lift;
    const int bin = (min((int)(u0 * 32.f), 31) * 16 + min((int)(u1 * 16.f), 15)) * 8 +
                    min((int)(u2 * 8.f), 7);
    const int first = sph_off[obj_off[s]];
    const int pl_end = sph_off[o];   // the state's placed objects precede o
    bool bad = threadIdx.x < 16 ? !__builtin_isfinite(sup[16 * obj_sup[o] + threadIdx.x]) : false;
    for (int k = sph_off[o] + threadIdx.x; k < sph_off[o + 1]; k += kWave) bad |= !finite4(tmpl[k]);
    for (int bx = box_off[s] + threadIdx.x; bx < box_off[s + 1]; bx += kWave)
        bad |= !all_finite(box + 16 * bx, 15);
    for (int q = first + threadIdx.x; q < pl_end; q += kWave) bad |= !finite4(placed[q]);
    bad = __ballot(bad) != 0;
    float clr = __builtin_huge_valf();
    const int g0 = grid_off ? grid_off[s] : 0, g1 = grid_off ? grid_off[s + 1] : 0;
    bool nan_sample = false;   // a grid sample that read a non-finite node
    for (int k = sph_off[o]; k < sph_off[o + 1]; ++k) {
        const float4 c = tmpl[k];
        float wx, wy, wz;
        to_world(U, P, c.x, c.y, c.z, wx, wy, wz);
        float best = __builtin_huge_valf();
        for (int bx = box_off[s]; bx < box_off[s + 1]; ++bx)
            best = fminf(best, box_sdf(box + 16 * bx, wx, wy, wz));
        for (int g = g0; g < g1; ++g) {
            const float v = grid_sample(grid + 24 * g, grid_val + grid_val_off[grid_src[g]], wx,
                                        wy, wz);
            nan_sample |= v != v;
            best = fminf(best, v);
        }
        for (int q = first; q < pl_end; ++q) {
            const float4 p = placed[q];
            const float dx = wx - p.x, dy = wy - p.y, dz = wz - p.z;
            best = fminf(best, __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))) - p.w);
        }
        clr = fminf(clr, best - c.w);
    }
    if (i < L) {
        bins_out[(size_t)s * L + i] = bin;
        accept_out[(size_t)s * L + i] = !bad && !nan_sample && clr >= margin ? 1.f : 0.f;
    }
    if ((bad || __ballot(nan_sample && i < L) != 0) && threadIdx.x == 0)
        atomicOr(counters + kErrorWord, (unsigned long long)kErrNonFinite);
}

hipError_t launch_harvest(const scn_batch& b, const int32_t* n_state, int L, uint64_t seed,
                          int round, float margin, int32_t* bins, float* accept,
                          int64_t* counters, hipStream_t st) {
    if (b.n_scenes == 0 || L <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_harvest, dim3(b.n_scenes, (L + 63) / 64), dim3(64), 0, st, b.obj_off,
                       b.sph_off, (const float4*)b.tmpl, b.obj_sup, b.sup, b.box_off, b.box,
                       (const float4*)b.placed, n_state, L, seed, round, margin, bins, accept,
                       (unsigned long long*)counters, b.grid_off, b.grid, b.grid_src,
                       b.grid_val_off, b.grid_val);
    return hipGetLastError();
}

}  // namespace scn
