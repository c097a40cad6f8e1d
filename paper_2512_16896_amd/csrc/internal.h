// internal.h -- launch plumbing between the C ABI (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scn.h"

namespace scn {

// Device counters (int64 each), laid out like scn_counters.
enum CounterSlot {
    kCandidates = 0, kSpherePairs = 1, kBoxPairs = 2, kGridSamples = 3, kAttempts = 4,
    kPlaced = 5, kErrorWord = 6, kTransforms = 7, kNumCounters = 16
};
enum ErrorBits { kErrCapacity = 1 };

struct PlacePlan {
    int waves;        // waves per workgroup (candidates in flight per scene)
    int spl;          // template spheres per lane (1, 2 or 4)
    int cap_sph;      // placed spheres a scene may hold in LDS
    int cap_obj;      // objects a scene may hold
    int max_steps;    // objects to place per scene in this launch (<= 0: all)
    int lds_bytes;
};

hipError_t launch_reset(const scn_batch& b, hipStream_t st);
hipError_t launch_fill_i64(int64_t* p, int n, int64_t v, hipStream_t st);
hipError_t launch_sample(const scn_batch& b, const int32_t* obj_idx, const int32_t* cand_off,
                         int max_cand, uint64_t seed, int attempt, scn_poses out, hipStream_t st);
hipError_t launch_check(const scn_batch& b, const int32_t* obj_idx, const int32_t* cand_off,
                        int max_cand, scn_poses poses, float margin, float* clr, uint8_t* col,
                        hipStream_t st);
hipError_t launch_place(const scn_batch& b, const scn_gen_args& a, const PlacePlan& plan,
                        int32_t* chosen, int64_t* counters, hipStream_t st);
int place_max_lds_bytes();

}  // namespace scn
