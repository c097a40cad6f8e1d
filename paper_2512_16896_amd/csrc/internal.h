// internal.h -- launch plumbing between the C ABI (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>

#include "scn.h"

// The library context (opaque in scn.h).
struct scn_ctx {
    int device;
    int lds_per_block;
    int n_cu;
    int64_t* d_counters;   // scn::kNumCounters int64
    void* ws = nullptr;    // caller-owned workspace (scn_set_workspace), never freed here
    size_t ws_bytes = 0;
    int32_t* h_flag = nullptr;   // pinned host words for small device-to-host reads
    hipStream_t cap_stream = nullptr;   // stream used only to capture graphs
    hipStream_t aux_stream = nullptr;   // second stream of the learned pipeline (default priority)
    hipEvent_t ev[2] = {nullptr, nullptr};   // its fork / join events
    std::map<std::string, hipGraphExec_t> plain_graphs;   // generation graphs per batch + plan
    struct Tuned { int schedule; float ms; };
    std::map<std::string, Tuned> tuned;   // autotuned schedule per batch shape bucket
};

// Error reporting shared by the host files: records a message for
// scn_last_error() and returns `code`.
int scn_fail(int code, const char* fmt, ...);
int scn_check_ctx(scn_ctx* c);
// The caller-owned workspace when it holds at least `bytes`, else an
// SCN_E_INVALID_ARG failure naming the sizes (nothing is allocated here).
int scn_workspace(scn_ctx* c, size_t bytes, void** out);

namespace scn {
constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
// Workspace bytes of each kind of call (scn_workspace_bytes); the calls take
// their buffers in the order these sizes are summed.
size_t ws_order_bytes(int n_scenes);                       // longest-first order + histogram
size_t ws_mlp_forward_bytes(const scn_mlp* n, int rows);   // hidden activations
size_t ws_mlp_backward_bytes(const scn_mlp* n, int rows);
size_t ws_mlp_train_bytes(const scn_mlp* n, int rows);     // backward + gradients
size_t ws_learned_bytes(const scn_batch* b, const scn_mlp* n, int top_k);
}  // namespace scn

// Network forward with the hidden activations in `act_ws`
// (ws_mlp_forward_bytes of it); used by the learned generation.  With m_dev
// the live row count min(M, *m_dev) is read on the device.
int scn_mlp_forward_ws(const scn_mlp* n, const uint16_t* x, int M, float* logits, void* act_ws,
                       hipStream_t st, const int32_t* m_dev = nullptr);

#define SCN_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return scn_fail(SCN_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

namespace scn {

// Device counters (int64 each), laid out like scn_counters.
enum CounterSlot {
    kCandidates = 0, kSpherePairs = 1, kBoxPairs = 2, kGridSamples = 3, kAttempts = 4,
    kPlaced = 5, kErrorWord = 6, kTransforms = 7, kBoxCulls = 8, kObjCulls = 9,
    kValidScenes = 10, kInvalidScenes = 11, kSphCulls = 12, kNonFinite = 13, kCheckRefined = 14,
    kNumCounters = 16
};
enum ErrorBits {
    kErrCapacity = 1,
    kErrGeometry = 2,
    kErrNonFinite = 4,
    kErrBadJoint = 8,
    kErrSharedSupport = 16   // the learned path: objects of two scenes on one support
};

// Bytes of dynamic LDS the place kernel adds for a scene's depth map (batches
// without grids).
constexpr int kMapBytes = 24576;
// 16-byte slots per object in the place kernel's LDS: its world bounding
// sphere once placed, and 4 constants and an index row while it is to be
// placed
constexpr int kObjLds = 6;
// the place kernel's LDS copy of a scene's first 64 box rows (16 floats each)
constexpr int kBoxLdsBytes = 64 * 16 * 4;
// cells of the height-map window the place kernel raises in LDS at a commit
// (it reuses the box rows' space)
constexpr int kHmapTileCells = kBoxLdsBytes / 4;
// LDS the place kernel's static shared variables may take (reserved beside
// its dynamic LDS)
constexpr int kPlaceStaticLds = 2048;

// Where the fused place kernel keeps a scene's placed spheres.
enum PlaceMode {
    kPlaceAllLds = 0,     // every scene in LDS (LDS sized for the largest scene)
    kPlaceSplit = 1,      // scenes up to split_sph spheres in LDS, larger ones in global memory
    kPlaceAllGlobal = 2   // every scene reads placed spheres from global memory
};

struct PlacePlan {
    int32_t* order;   // scene launch order (nullptr: batch order), in the workspace
    const int32_t* n_order = nullptr;   // device count of `order`'s live entries (nullptr: all)
    int32_t* hist;    // its bucket counters (kOrderBuckets + 1), in the workspace
    int waves;        // waves per workgroup (candidates in flight per scene)
    int spl;          // template spheres per lane (1, 2 or 4)
    int mode;         // PlaceMode
    int cap_sph;      // placed spheres a scene may hold in LDS (all-LDS mode)
    int split_sph;    // split mode: largest scene (in spheres) kept in LDS
    int cap_obj;      // objects a scene may hold
    int max_steps;    // objects to place per scene in this launch (<= 0: all)
    const int32_t* prop_bins = nullptr;  // learned proposal: [n_scenes][prop_k] bins, rank order
    int prop_k = 0;
    // Resumable lists (learned path): a launch tries the proposals plus
    // `chunk` uniform entries of the current object (then `chunk` per launch)
    // and, when none is valid and entries remain, leaves the object pending
    // with resume[s] = the next entry.  chunk == 0: the whole list; chunk < 0:
    // the proposals alone (the uniform entries in later launches).
    int32_t* resume = nullptr;
    int chunk = 0;
    int j_cap = 0;                 // objects per scene in total (<= 0: all)
    int32_t* n_active = nullptr;   // [2]: scenes left active with work remaining, and those
                                   // of them that start a new object next
    // State kept across the launches of one generation (learned pipeline):
    // each scene's depth map (kMapBytes), each placed object's world bounding
    // sphere (float4) and each object's constants (4 float4, k_object_info).
    void* map_keep = nullptr;
    void* bnd_keep = nullptr;
    const void* info_keep = nullptr;
    float* hmap = nullptr;   // learned proposal: height maps raised at each commit
};

// learned-proposal kernels (learned.hip)
hipError_t launch_descriptor(const scn_batch& b, float* desc, hipStream_t st);
hipError_t launch_hmap_boxes(const scn_batch& b, float* hmap, hipStream_t st);
hipError_t launch_hmap_raise(const scn_batch& b, const int32_t* obj_idx, const int32_t* n_state,
                             float* hmap, hipStream_t st);
hipError_t launch_features(int n, const float* hmap, const float* desc, const int32_t* obj_idx,
                           const int32_t* obj_sup, int ld, void* x, hipStream_t st,
                           const int32_t* m_dev = nullptr);
hipError_t launch_topk(int M, const float* logits, int k, const int32_t* active, int32_t* bins,
                       hipStream_t st, const int32_t* rows = nullptr,
                       const int32_t* m_dev = nullptr);
hipError_t launch_support_scene(const scn_batch& b, int32_t* sup_scene, int64_t* counters,
                                hipStream_t st);
hipError_t launch_tick_plan(const scn_batch& b, const int32_t* resume, int j_cap, int32_t* list,
                            int32_t* obj_idx, int32_t* count, hipStream_t st);
hipError_t launch_harvest(const scn_batch& b, const int32_t* n_state, int L, uint64_t seed,
                          int round, float margin, int32_t* bins, float* accept,
                          int64_t* counters, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t st);   // kernels.hip

hipError_t launch_reset(const scn_batch& b, hipStream_t st);
hipError_t launch_fill_i64(int64_t* p, int n, int64_t v, hipStream_t st);
hipError_t launch_sample(const scn_batch& b, const int32_t* obj_idx, const int32_t* cand_off,
                         int max_cand, uint64_t seed, int attempt, scn_poses out, hipStream_t st);
hipError_t launch_check(const scn_batch& b, const int32_t* obj_idx, const int32_t* cand_off,
                        int max_cand, scn_poses poses, float margin, float* clr, uint8_t* col,
                        int64_t* counters, hipStream_t st);
// Sets the non-finite error bit when any grid asset node value is not finite.
hipError_t launch_scan_grid_values(const scn_batch& b, int64_t* counters, hipStream_t st);
hipError_t launch_object_info(const scn_batch& b, float margin, void* info, hipStream_t st);
hipError_t launch_place(const scn_batch& b, const scn_gen_args& a, const PlacePlan& plan,
                        int32_t* chosen, int64_t* counters, hipStream_t st);
// Longest-first scene order: a counting sort of the scenes by an estimate of
// their placement work.  hist needs kOrderBuckets + 1 int32 of device memory.
constexpr int kOrderBuckets = 256;
// network kernels (mlp.hip)
hipError_t launch_gemm(int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                       const float* bias, bool relu, float* C32, void* C16, int ldc,
                       hipStream_t st, const int32_t* m_dev = nullptr);
hipError_t launch_transpose_bf16(int rows, int cols, const void* in, int ldi, void* out, int ldo,
                                 hipStream_t st);
hipError_t launch_f32_to_bf16(int n, const float* in, void* out, hipStream_t st);
hipError_t launch_bce(int M, int N, int L, const float* z, const int32_t* bins, const float* tgt,
                      float inv_count, float* dz32, float* loss, hipStream_t st);
hipError_t launch_relu_bwd(int n, const float* da, const void* act, void* dp, hipStream_t st);
hipError_t launch_colsum_bf16(int M, int N, const void* d, float* db, hipStream_t st);
hipError_t launch_colsum_f32(int M, int N, const float* d, float* db, hipStream_t st);
hipError_t launch_adamw(int rows, int cols, float* w, const float* g, float* m1, float* m2,
                        void* wb, void* wt, float lr, float b1, float b2, float eps, float wd,
                        float c1, float c2, hipStream_t st);
hipError_t launch_init_layer(int rows, int cols, uint64_t seed, int layer, float* w, void* wb,
                             void* wt, hipStream_t st);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st);

hipError_t launch_longest_first(const scn_batch& b, int32_t* order, int32_t* hist,
                                hipStream_t st);
// batched forward kinematics (fk.hip)
hipError_t launch_fk(const scn_joints& j, uint64_t seed, int sample, float* q, float* link,
                     int n_box, const int32_t* box_link, const float* box_local, float* box,
                     int n_sup, const int32_t* sup_link, const float* sup_local, float* sup,
                     int64_t* counters, hipStream_t st);

}  // namespace scn
