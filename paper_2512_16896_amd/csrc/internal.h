// internal.h -- launch plumbing between the C ABI (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scn.h"

namespace scn {

// Device counters (int64 each), laid out like scn_counters.
enum CounterSlot {
    kCandidates = 0, kSpherePairs = 1, kBoxPairs = 2, kGridSamples = 3, kAttempts = 4,
    kPlaced = 5, kErrorWord = 6, kTransforms = 7, kBoxCulls = 8, kObjCulls = 9,
    kValidScenes = 10, kInvalidScenes = 11, kSphCulls = 12, kNumCounters = 16
};
enum ErrorBits { kErrCapacity = 1 };

// Where the fused place kernel keeps a scene's placed spheres.
enum PlaceMode {
    kPlaceAllLds = 0,     // every scene in LDS (LDS sized for the largest scene)
    kPlaceSplit = 1,      // scenes up to split_sph spheres in LDS, larger ones in global memory
    kPlaceAllGlobal = 2   // every scene reads placed spheres from global memory
};

struct PlacePlan {
    const int32_t* order;  // scene launch order (nullptr: batch order)
    int waves;        // waves per workgroup (candidates in flight per scene)
    int spl;          // template spheres per lane (1, 2 or 4)
    int mode;         // PlaceMode
    int cap_sph;      // placed spheres a scene may hold in LDS (all-LDS mode)
    int split_sph;    // split mode: largest scene (in spheres) kept in LDS
    int cap_obj;      // objects a scene may hold
    int max_steps;    // objects to place per scene in this launch (<= 0: all)
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
// Longest-first scene order: a counting sort of the scenes by an estimate of
// their placement work.  hist needs kOrderBuckets + 1 int32 of device memory.
constexpr int kOrderBuckets = 256;
hipError_t launch_longest_first(const scn_batch& b, int32_t* order, int32_t* hist,
                                hipStream_t st);

}  // namespace scn
