// reach.hip -- batched reachability queries on the GPU (Sec. IV-E: the
// reachability map moved to the device and its queries batched).  One lane
// per query; the map lookup is device.h:reach_ok, the same one the place
// kernel applies to candidates of objects that must be reachable.
#include "device.h"
#include "internal.h"

namespace scn {

__global__ __launch_bounds__(256) void k_reach(int n, scn_reach_map m,
                                               const float* __restrict__ robot,
                                               const float* __restrict__ pose,
                                               const float* __restrict__ theta,
                                               uint8_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* P = pose + 12 * i;
    float rb[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) rb[k] = robot[12 * i + k];
    out[i] = reach_ok(m.map, m, rb, P[9], P[10], P[11], P[0], P[3], P[6], theta[i]) ? 1 : 0;
}

}  // namespace scn

extern "C" int scn_reach_query(scn_ctx* c, const scn_reach_map* m, int32_t n, const float* robot,
                               const float* pose, const float* theta, uint8_t* out,
                               scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (!m || n < 0) return scn_fail(SCN_E_INVALID_ARG, "null map or negative n");
    if (n == 0) return SCN_OK;
    if (!m->map || !robot || !pose || !theta || !out)
        return scn_fail(SCN_E_INVALID_ARG, "map, robot, pose, theta and out required");
    for (int a = 0; a < 4; ++a)
        if (m->dims[a] <= 0 || !(m->h[a] > 0.f))
            return scn_fail(SCN_E_INVALID_ARG, "map axis %d: dims and h must be > 0", a);
    hipLaunchKernelGGL(scn::k_reach, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n,
                       *m, robot, pose, theta, out);
    SCN_HIP(hipGetLastError());
    return SCN_OK;
}
