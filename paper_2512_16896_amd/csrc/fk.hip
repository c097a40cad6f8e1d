// fk.hip -- batched forward kinematics of articulated furniture parts
// (Sec. IV-B: one transform per scene instance on every scene-graph edge, and
// a batched FK that moves the articulated parts of all instances at once;
// Sec. V-A: drawer joint states randomized per scene).
//
//   k_fk_links  one lane per scene: the scene's joints in topological order,
//               each child link = parent link * joint frame * motion(q)
//   k_fk_rows   one lane per box / support row: rows attached to a link move
//               to link * local pose
//
// Motion of a joint with unit axis a (joint frame): prismatic = translation by
// q a; revolute = rotation by q about a (Rodrigues: I + sin q K + (1 - cos q) K^2).
// Sampled joint values q = lower + u (upper - lower), u from Philox4x32-10 with
// counter (joint index within the scene, 0x30000, 0, scene).
#include "device.h"
#include "internal.h"

namespace scn {

// C = A B for rigid transforms stored R[9] (row-major), t[3].
__device__ __forceinline__ void compose(const float* A, const float* B, float* C) {
    float R[9], t[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            R[3 * r + c] = fmaf(A[3 * r + 0], B[c], fmaf(A[3 * r + 1], B[3 + c], A[3 * r + 2] * B[6 + c]));
        t[r] = fmaf(A[3 * r + 0], B[9], fmaf(A[3 * r + 1], B[10], fmaf(A[3 * r + 2], B[11], A[9 + r])));
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) C[i] = R[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) C[9 + i] = t[i];
}

__global__ __launch_bounds__(64) void k_fk_links(int n_scenes, const int32_t* __restrict__ joint_off,
                                                 const float* __restrict__ joint,
                                                 const float* __restrict__ base, uint64_t seed,
                                                 int sample, float* __restrict__ q,
                                                 float* __restrict__ link,
                                                 unsigned long long* __restrict__ counters) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_scenes) return;
    const int j0 = joint_off[s], j1 = joint_off[s + 1];
    bool bad = false;
    for (int i = j0; i < j1; ++i) {
        const float* J = joint + 24 * i;
        float qi;
        if (sample) {
            const U4 w = philox10(U4{(uint32_t)(i - j0), 0x30000u, 0u, (uint32_t)s},
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
            qi = fmaf(unit01(w.a), J[3] - J[2], J[2]);
            q[i] = qi;
        } else {
            qi = q[i];
        }
        const int parent = (int)J[1];
        float P[12];
        if (parent < -1 || parent >= i - j0) {
            // a parent that is not an earlier joint of the scene: the link is
            // left undefined (NaN) and the error is reported
            bad = true;
            for (int k = 0; k < 12; ++k) link[12 * i + k] = __builtin_nanf("");
            continue;
        }
        const float* src = parent < 0 ? base + 12 * s : link + 12 * (j0 + parent);
#pragma unroll
        for (int k = 0; k < 12; ++k) P[k] = src[k];
        float Tj[12], M[12], PT[12], L[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) Tj[k] = J[8 + k];
        const float ax = J[4], ay = J[5], az = J[6];
        if (J[0] == 0.f) {   // prismatic
            M[0] = 1.f; M[1] = 0.f; M[2] = 0.f;
            M[3] = 0.f; M[4] = 1.f; M[5] = 0.f;
            M[6] = 0.f; M[7] = 0.f; M[8] = 1.f;
            M[9] = qi * ax; M[10] = qi * ay; M[11] = qi * az;
        } else {             // revolute
            float sn, cs;
            sincosf(qi, &sn, &cs);
            const float v = 1.f - cs;
            // I + sin K + (1 - cos) K^2, K the cross-product matrix of a and
            // K^2 = a a^T - |a|^2 I
            const float n2 = fmaf(ax, ax, fmaf(ay, ay, az * az));
            M[0] = fmaf(v, ax * ax - n2, 1.f); M[1] = fmaf(v, ax * ay, -sn * az); M[2] = fmaf(v, ax * az, sn * ay);
            M[3] = fmaf(v, ax * ay, sn * az);  M[4] = fmaf(v, ay * ay - n2, 1.f); M[5] = fmaf(v, ay * az, -sn * ax);
            M[6] = fmaf(v, ax * az, -sn * ay); M[7] = fmaf(v, ay * az, sn * ax);  M[8] = fmaf(v, az * az - n2, 1.f);
            M[9] = 0.f; M[10] = 0.f; M[11] = 0.f;
        }
        compose(P, Tj, PT);
        compose(PT, M, L);
#pragma unroll
        for (int k = 0; k < 12; ++k) link[12 * i + k] = L[k];
    }
    if (bad) atomicOr(counters + kErrorWord, (unsigned long long)kErrBadJoint);
}

__global__ __launch_bounds__(256) void k_fk_rows(int n_rows, int n_joints,
                                                 const int32_t* __restrict__ row_link,
                                                 const float* __restrict__ local,
                                                 const float* __restrict__ link,
                                                 float* __restrict__ rows,
                                                 unsigned long long* __restrict__ counters) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int l = row_link[r];
    if (l < 0) return;
    if (l >= n_joints) {
        atomicOr(counters + kErrorWord, (unsigned long long)kErrBadJoint);
        return;
    }
    float A[12], B[12], W[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) { A[k] = link[12 * l + k]; B[k] = local[12 * r + k]; }
    compose(A, B, W);
#pragma unroll
    for (int k = 0; k < 12; ++k) rows[16 * r + k] = W[k];
}

hipError_t launch_fk(const scn_joints& j, uint64_t seed, int sample, float* q, float* link,
                     int n_box, const int32_t* box_link, const float* box_local, float* box,
                     int n_sup, const int32_t* sup_link, const float* sup_local, float* sup,
                     int64_t* counters, hipStream_t st) {
    auto* ctr = (unsigned long long*)counters;
    if (j.n_scenes > 0)
        hipLaunchKernelGGL(k_fk_links, dim3((j.n_scenes + 63) / 64), dim3(64), 0, st, j.n_scenes,
                           j.joint_off, j.joint, j.base, seed, sample, q, link, ctr);
    if (n_box > 0 && box_link)
        hipLaunchKernelGGL(k_fk_rows, dim3((n_box + 255) / 256), dim3(256), 0, st, n_box,
                           j.n_joints, box_link, box_local, link, box, ctr);
    if (n_sup > 0 && sup_link)
        hipLaunchKernelGGL(k_fk_rows, dim3((n_sup + 255) / 256), dim3(256), 0, st, n_sup,
                           j.n_joints, sup_link, sup_local, link, sup, ctr);
    return hipGetLastError();
}

}  // namespace scn

extern "C" int scn_forward_kinematics(scn_ctx* c, const scn_joints* j, uint64_t seed,
                                      int32_t sample_q, float* q, float* link, int32_t n_box,
                                      const int32_t* box_link, const float* box_local, float* box,
                                      int32_t n_sup, const int32_t* sup_link,
                                      const float* sup_local, float* sup, scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (!j) return scn_fail(SCN_E_INVALID_ARG, "null joints");
    if (j->n_scenes < 0 || j->n_joints < 0 || n_box < 0 || n_sup < 0)
        return scn_fail(SCN_E_INVALID_ARG, "negative size");
    if (j->n_scenes > 0 && (!j->joint_off || !j->base))
        return scn_fail(SCN_E_INVALID_ARG, "joint_off and base required");
    if (j->n_joints > 0 && (!j->joint || !q || !link))
        return scn_fail(SCN_E_INVALID_ARG, "joint, q and link required");
    if (n_box > 0 && box_link && (!box_local || !box))
        return scn_fail(SCN_E_INVALID_ARG, "box_local and box required with box_link");
    if (n_sup > 0 && sup_link && (!sup_local || !sup))
        return scn_fail(SCN_E_INVALID_ARG, "sup_local and sup required with sup_link");
    SCN_HIP(scn::launch_fk(*j, seed, sample_q ? 1 : 0, q, link, n_box, box_link, box_local, box,
                           n_sup, sup_link, sup_local, sup, c->d_counters, (hipStream_t)stream));
    return SCN_OK;
}
