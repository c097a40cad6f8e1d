// api.hip -- the C ABI of libscn.so (declared in include/scn.h): argument
// validation, contexts, launch planning and error reporting.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "internal.h"
#include "scn.h"

static thread_local std::string g_err;

int scn_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int scn_check_ctx(scn_ctx* c) {
    if (!c) return scn_fail(SCN_E_INVALID_ARG, "null context");
    if (hipSetDevice(c->device) != hipSuccess) return scn_fail(SCN_E_HIP, "hipSetDevice failed");
    return SCN_OK;
}

int scn_workspace(scn_ctx* c, size_t bytes, void** out) {
    if (bytes > 0 && (!c->ws || bytes > c->ws_bytes))
        return scn_fail(SCN_E_INVALID_ARG,
                        "workspace of %zu bytes needed, %zu attached (scn_workspace_bytes, "
                        "scn_set_workspace)", bytes, c->ws ? c->ws_bytes : (size_t)0);
    *out = c->ws;
    return SCN_OK;
}

size_t scn::ws_order_bytes(int n_scenes) {
    return align256(sizeof(int32_t) * (size_t)(n_scenes > 0 ? n_scenes : 0)) +
           align256(sizeof(int32_t) * (kOrderBuckets + 1));
}

// Fixed device scratch of scn_generate_scenes_noalloc: the longest-first scene
// order and its histogram for up to SCN_NOALLOC_MAX_SCENES scenes (4 MiB + 1.25
// KiB).  Every device the library runs on holds its own copy until the process
// ends.  In host code `scratch` only names the symbol: kernels are handed the
// per-device address that hipGetSymbolAddress returned for it (g_scratch_ptr).
static constexpr size_t kScratchBytes =
    scn::align256(sizeof(int32_t) * (size_t)SCN_NOALLOC_MAX_SCENES) +
    scn::align256(sizeof(int32_t) * (scn::kOrderBuckets + 1));
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kScratchMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchMaxDevices] = {};

// Looks up this device's address of `scratch` once (the device must be
// current); called by scn_ctx_create.
static int scratch_setup(int device) {
    if (device < 0 || device >= kScratchMaxDevices)
        return scn_fail(SCN_E_NO_DEVICE, "device %d beyond the %d the library tracks", device,
                        kScratchMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return SCN_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return scn_fail(SCN_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = p;
    return SCN_OK;
}

static void* scratch_ptr(int device) {
    if (device < 0 || device >= kScratchMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

namespace {

#define fail scn_fail
#define check_ctx scn_check_ctx

int check_batch(const scn_batch* b, bool need_state) {
    if (!b) return fail(SCN_E_INVALID_ARG, "null batch");
    if (b->n_scenes < 0 || b->n_objects < 0 || b->n_spheres < 0 || b->n_supports < 0 ||
        b->n_boxes < 0 || b->n_grids < 0)
        return fail(SCN_E_INVALID_ARG, "negative batch size");
    if (b->n_scenes > 0 && (!b->obj_off || !b->box_off))
        return fail(SCN_E_INVALID_ARG, "obj_off/box_off required");
    if (b->n_objects > 0 && (!b->sph_off || !b->obj_sup || !b->sup))
        return fail(SCN_E_INVALID_ARG, "sph_off/obj_sup/sup required");
    if (b->n_spheres > 0 && !b->tmpl) return fail(SCN_E_INVALID_ARG, "tmpl required");
    if (b->n_boxes > 0 && !b->box) return fail(SCN_E_INVALID_ARG, "box required");
    if (b->grid_off && (!b->grid || !b->grid_src || !b->grid_val_off || !b->grid_val))
        return fail(SCN_E_INVALID_ARG, "grid_off given without grid tables");
    if (b->obj_pose_off && !b->stable)
        return fail(SCN_E_INVALID_ARG, "obj_pose_off given without stable");
    if (b->max_spheres_per_object < 0 || b->max_spheres_per_scene < 0 ||
        b->max_objects_per_scene < 0)
        return fail(SCN_E_INVALID_ARG, "negative planning size");
    if (need_state && b->n_scenes > 0 && (!b->n_placed || !b->status || !b->rec || !b->placed))
        return fail(SCN_E_INVALID_ARG, "placed/n_placed/status/rec required");
    return SCN_OK;
}

}  // namespace

extern "C" {

const char* scn_last_error(void) { return g_err.c_str(); }

const char* scn_status_string(int status) {
    switch (status) {
        case SCN_OK: return "ok";
        case SCN_E_INVALID_ARG: return "invalid argument";
        case SCN_E_HIP: return "HIP runtime error";
        case SCN_E_CAPACITY: return "scene exceeds the planned capacity";
        case SCN_E_NO_DEVICE: return "no usable gfx950 device";
        case SCN_E_UNSUPPORTED: return "unsupported size";
        case SCN_E_NONFINITE: return "non-finite input (treated as a collision)";
        default: return "unknown status";
    }
}

int scn_ctx_create(scn_ctx** out, int device) {
    if (!out) return fail(SCN_E_INVALID_ARG, "null output pointer");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(SCN_E_NO_DEVICE, "no HIP device");
    if (device < 0 || device >= n) return fail(SCN_E_NO_DEVICE, "device %d out of range (%d)", device, n);
    hipDeviceProp_t p;
    SCN_HIP(hipGetDeviceProperties(&p, device));
    if (strncmp(p.gcnArchName, "gfx950", 6) != 0)
        return fail(SCN_E_NO_DEVICE, "device %d is %s, not gfx950", device, p.gcnArchName);
    SCN_HIP(hipSetDevice(device));
    if (int r = scratch_setup(device)) return r;
    auto* c = new scn_ctx();
    c->device = device;
    if (hipHostMalloc((void**)&c->h_flag, 4 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(SCN_E_HIP, "hipHostMalloc(flags) failed");
    }
    c->n_cu = p.multiProcessorCount;
    c->lds_per_block = (int)p.sharedMemPerBlock;
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess &&
        optin > c->lds_per_block)
        c->lds_per_block = optin;
    if (hipMalloc((void**)&c->d_counters, sizeof(int64_t) * scn::kNumCounters) != hipSuccess) {
        (void)hipHostFree(c->h_flag);
        delete c;
        return fail(SCN_E_HIP, "hipMalloc(counters) failed");
    }
    if (hipMemset(c->d_counters, 0, sizeof(int64_t) * scn::kNumCounters) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->d_counters);
        (void)hipHostFree(c->h_flag);
        delete c;
        return fail(SCN_E_HIP, "counter init failed");
    }
    *out = c;
    return SCN_OK;
}

int scn_ctx_destroy(scn_ctx* c) {
    if (!c) return SCN_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(c->d_counters);
    if (c->h_flag) (void)hipHostFree(c->h_flag);
    for (auto& kv : c->plain_graphs) (void)hipGraphExecDestroy(kv.second);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
    for (auto e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
    return SCN_OK;
}

int scn_workspace_bytes(int kind, const scn_batch* b, const scn_mlp* net, int32_t rows,
                        int32_t top_k, size_t* bytes) {
    if (!bytes) return fail(SCN_E_INVALID_ARG, "null output pointer");
    *bytes = 0;
    auto need_net = [&]() -> int {
        if (!net) return fail(SCN_E_INVALID_ARG, "network required for this workspace kind");
        for (int l = 0; l <= SCN_MLP_LAYERS; ++l)
            if (net->dims[l] <= 0) return fail(SCN_E_INVALID_ARG, "dims[%d] must be > 0", l);
        return SCN_OK;
    };
    switch (kind) {
        case SCN_WS_GENERATE:
            if (!b || b->n_scenes < 0) return fail(SCN_E_INVALID_ARG, "batch required");
            *bytes = scn::ws_order_bytes(b->n_scenes);
            return SCN_OK;
        case SCN_WS_MLP_FORWARD:
        case SCN_WS_MLP_BACKWARD:
        case SCN_WS_MLP_TRAIN:
            if (int r = need_net()) return r;
            if (rows < 0) return fail(SCN_E_INVALID_ARG, "rows must be >= 0");
            *bytes = kind == SCN_WS_MLP_FORWARD    ? scn::ws_mlp_forward_bytes(net, rows)
                     : kind == SCN_WS_MLP_BACKWARD ? scn::ws_mlp_backward_bytes(net, rows)
                                                   : scn::ws_mlp_train_bytes(net, rows);
            return SCN_OK;
        case SCN_WS_GENERATE_LEARNED:
            if (int r = need_net()) return r;
            if (!b || b->n_scenes < 0 || b->n_objects < 0)
                return fail(SCN_E_INVALID_ARG, "batch required");
            if (top_k < 1 || top_k > SCN_BINS) return fail(SCN_E_INVALID_ARG, "top_k out of range");
            *bytes = scn::ws_learned_bytes(b, net, top_k);
            return SCN_OK;
        default:
            return fail(SCN_E_INVALID_ARG, "unknown workspace kind %d", kind);
    }
}

int scn_set_workspace(scn_ctx* c, void* ptr, size_t bytes) {
    if (!c) return fail(SCN_E_INVALID_ARG, "null context");
    if (ptr && ((uintptr_t)ptr & 255u))
        return fail(SCN_E_INVALID_ARG, "workspace must be 256-byte aligned");
    c->ws = ptr;
    c->ws_bytes = ptr ? bytes : 0;
    return SCN_OK;
}

int scn_reset_counters(scn_ctx* c, scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    SCN_HIP(scn::launch_fill_i64(c->d_counters, scn::kNumCounters, 0, (hipStream_t)stream));
    return SCN_OK;
}

int scn_read_counters(scn_ctx* c, scn_counters* out, scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (!out) return fail(SCN_E_INVALID_ARG, "null output pointer");
    int64_t h[scn::kNumCounters];
    SCN_HIP(hipMemcpyAsync(h, c->d_counters, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream));
    SCN_HIP(hipStreamSynchronize((hipStream_t)stream));
    memset(out, 0, sizeof *out);
    out->candidates = h[scn::kCandidates];
    out->sphere_pairs = h[scn::kSpherePairs];
    out->box_pairs = h[scn::kBoxPairs];
    out->grid_samples = h[scn::kGridSamples];
    out->attempts = h[scn::kAttempts];
    out->placed = h[scn::kPlaced];
    out->error_word = h[scn::kErrorWord];
    out->transforms = h[scn::kTransforms];
    out->box_culls = h[scn::kBoxCulls];
    out->object_culls = h[scn::kObjCulls];
    out->valid_scenes = h[scn::kValidScenes];
    out->invalid_scenes = h[scn::kInvalidScenes];
    out->sphere_culls = h[scn::kSphCulls];
    out->nonfinite = h[scn::kNonFinite];
    out->check_refined = h[scn::kCheckRefined];
    if (out->error_word & scn::kErrCapacity)
        return fail(SCN_E_CAPACITY, "a scene exceeded the planned capacity and was skipped");
    if (out->error_word & scn::kErrGeometry)
        return fail(SCN_E_INVALID_ARG,
                    "a scene breaks the batch's declared SCN_GEOM_YAW geometry and was marked invalid");
    if (out->error_word & scn::kErrBadJoint)
        return fail(SCN_E_INVALID_ARG,
                    "a joint's parent is not an earlier joint of its scene, or a row's link index "
                    "is out of range (those links and rows were not computed)");
    if (out->error_word & scn::kErrSharedSupport)
        return fail(SCN_E_INVALID_ARG,
                    "the learned generation found objects of two scenes on one support (its "
                    "height maps are per support)");
    if (out->error_word & scn::kErrNonFinite)
        return fail(SCN_E_NONFINITE,
                    "non-finite input: the candidates tested against it collided (%lld counted)",
                    (long long)out->nonfinite);
    return SCN_OK;
}

int scn_sample_poses(scn_ctx* c, const scn_batch* b, const int32_t* obj_idx,
                     const int32_t* cand_off, int32_t total, int32_t max_cand, uint64_t seed,
                     int32_t attempt, scn_poses out, scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (int r = check_batch(b, false)) return r;
    if (total < 0 || max_cand < 0 || attempt < 0)
        return fail(SCN_E_INVALID_ARG, "negative total/max_cand/attempt");
    if (b->n_scenes > 0 && (!obj_idx || !cand_off)) return fail(SCN_E_INVALID_ARG, "obj_idx/cand_off required");
    if (total > 0 && (!out.x || !out.y || !out.z || !out.yaw))
        return fail(SCN_E_INVALID_ARG, "output arrays required");
    if ((int64_t)max_cand > 65535LL * 256) return fail(SCN_E_UNSUPPORTED, "max_cand too large");
    SCN_HIP(scn::launch_sample(*b, obj_idx, cand_off, max_cand, seed, attempt, out, (hipStream_t)stream));
    return SCN_OK;
}

int scn_check_batch(scn_ctx* c, const scn_batch* b, const int32_t* obj_idx,
                    const int32_t* cand_off, int32_t total, int32_t max_cand, scn_poses poses,
                    float margin, float* clearance, uint8_t* collide, scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (int r = check_batch(b, false)) return r;
    if (total < 0 || max_cand < 0) return fail(SCN_E_INVALID_ARG, "negative total/max_cand");
    if (b->n_scenes > 0 && (!obj_idx || !cand_off || !b->n_placed || !b->placed))
        return fail(SCN_E_INVALID_ARG, "obj_idx/cand_off/n_placed/placed required");
    if (total > 0 && (!poses.x || !poses.y || !poses.z || !poses.yaw))
        return fail(SCN_E_INVALID_ARG, "pose arrays required");
    if (poses.stable)
        return fail(SCN_E_UNSUPPORTED, "the dense checker takes poses that turn about z only");
    if (!(margin >= 0.f)) return fail(SCN_E_INVALID_ARG, "margin must be >= 0");
    if ((int64_t)max_cand > 65535LL * 128) return fail(SCN_E_UNSUPPORTED, "max_cand too large");
    if (b->max_spheres_per_object > 256)
        return fail(SCN_E_UNSUPPORTED, "max_spheres_per_object %d > 256", b->max_spheres_per_object);
    SCN_HIP(scn::launch_check(*b, obj_idx, cand_off, max_cand, poses, margin, clearance, collide,
                              c->d_counters, (hipStream_t)stream));
    return SCN_OK;
}

int scn_reset_scenes(scn_ctx* c, scn_batch* b, scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (int r = check_batch(b, true)) return r;
    SCN_HIP(scn::launch_reset(*b, (hipStream_t)stream));
    return SCN_OK;
}

// Shape bucket of a batch for the autotuner: sphere slots per lane, then the
// largest scene, objects per scene and scene count rounded up to powers of two.
static int pow2_ceil(int v) {
    int p = 1;
    while (p < v && p < (1 << 30)) p <<= 1;
    return p;
}
static std::string shape_key(const scn_batch* b) {
    const int S = b->max_spheres_per_object;
    const int spl = S <= 64 ? 1 : (S <= 128 ? 2 : 4);
    char k[128];
    snprintf(k, sizeof k, "spl%d_sph%d_obj%d_box%d_n%d", spl, pow2_ceil(b->max_spheres_per_scene),
             pow2_ceil(b->max_objects_per_scene), pow2_ceil(b->max_boxes_per_scene),
             pow2_ceil(b->n_scenes));
    return k;
}

// 4 waves, batch order, placed spheres read from global memory: a workgroup
// then needs only its depth map and object data in LDS, so five fit on a CU
// (register-bound), which keeps more scenes in flight than LDS-resident
// spheres allow
static const int kDefaultSchedule = 4 | (SCN_SCHED_LDS_NONE << SCN_SCHED_LDS_SHIFT);

static int plan_place(scn_ctx* c, const scn_batch* b, const scn_gen_args* a, int max_steps,
                      scn::PlacePlan* plan, void* order_ws = nullptr) {
    if (!a) return fail(SCN_E_INVALID_ARG, "null args");
    if (!(a->margin >= 0.f)) return fail(SCN_E_INVALID_ARG, "margin must be >= 0");
    if (a->retries < 0) return fail(SCN_E_INVALID_ARG, "retries must be >= 0");
    if (!b->obj_ncand && a->default_ncand <= 0)
        return fail(SCN_E_INVALID_ARG, "default_ncand must be > 0 when obj_ncand is NULL");
    const int S = b->max_spheres_per_object;
    if (S > 256) return fail(SCN_E_UNSUPPORTED, "max_spheres_per_object %d > 256", S);
    if ((b->obj_rel || b->robot || b->obj_pose_off) && b->grid_off)
        return fail(SCN_E_UNSUPPORTED,
                    "spatial relations, reachability or stable poses in voxel-grid batches are "
                    "not supported");
    if (b->obj_rel && !b->rel) return fail(SCN_E_INVALID_ARG, "obj_rel given without rel");
    if (b->robot) {
        if (!b->obj_reach || !b->reach.map)
            return fail(SCN_E_INVALID_ARG, "robot given without obj_reach / reach.map");
        for (int a = 0; a < 4; ++a)
            if (b->reach.dims[a] <= 0 || !(b->reach.h[a] > 0.f))
                return fail(SCN_E_INVALID_ARG, "reach map axis %d: dims and h must be > 0", a);
    }
    plan->spl = S <= 64 ? 1 : (S <= 128 ? 2 : 4);
    int sched = a->schedule;
    if (sched == 0) {
        auto it = c->tuned.find(shape_key(b));
        sched = it != c->tuned.end() ? it->second.schedule : kDefaultSchedule;
    }
    if (sched & ~(SCN_SCHED_WAVES_MASK | SCN_SCHED_LONGEST_FIRST | SCN_SCHED_LDS_MASK))
        return fail(SCN_E_INVALID_ARG, "unknown schedule bits 0x%x", sched);
    const int w = sched & SCN_SCHED_WAVES_MASK;
    if (w < 1 || w > 16) return fail(SCN_E_INVALID_ARG, "schedule waves must be 1..16");
    plan->waves = w;
    plan->order = nullptr;
    plan->hist = nullptr;
    if (sched & SCN_SCHED_LONGEST_FIRST) {
        // the order and its histogram in the caller's workspace (order_ws:
        // the learned generation passes its own region)
        void* ws = order_ws;
        if (!ws)
            if (int r = scn_workspace(c, scn::ws_order_bytes(b->n_scenes), &ws)) return r;
        plan->order = (int32_t*)ws;
        plan->hist = (int32_t*)((char*)ws + scn::align256(sizeof(int32_t) * (size_t)b->n_scenes));
    }
    plan->cap_sph = b->max_spheres_per_scene > 0 ? b->max_spheres_per_scene : 1;
    plan->cap_obj = b->max_objects_per_scene > 0 ? b->max_objects_per_scene : 1;
    plan->max_steps = max_steps;
    // dynamic LDS available to the place kernel: the block limit minus the
    // kernel's own static shared variables
    const long long lds_cap =
        c->lds_per_block - scn::kPlaceStaticLds - scn::kBoxLdsBytes -
        (b->grid_off ? 0 : scn::kMapBytes);
    if (16LL * scn::kObjLds * plan->cap_obj + 16LL * 64 > lds_cap)
        return fail(SCN_E_UNSUPPORTED, "%d objects per scene do not fit the LDS", plan->cap_obj);
    static const int kBudgetKB[] = {0, 32, 48, 64, 80, 96};
    const int code = (sched & SCN_SCHED_LDS_MASK) >> SCN_SCHED_LDS_SHIFT;
    const long long all_bytes = 16LL * plan->cap_sph + 16LL * scn::kObjLds * plan->cap_obj;
    if (code == SCN_SCHED_LDS_NONE) {
        plan->mode = scn::kPlaceAllGlobal;
        plan->split_sph = 0;
    } else if (code <= 5) {
        long long budget = code == 0 ? all_bytes : 1024LL * kBudgetKB[code];
        if (budget > lds_cap) budget = lds_cap;
        if (all_bytes <= budget) {
            plan->mode = scn::kPlaceAllLds;
            plan->split_sph = plan->cap_sph;
        } else {
            plan->mode = scn::kPlaceSplit;
            plan->split_sph = (int)(budget / 16) - scn::kObjLds * plan->cap_obj;
            if (plan->split_sph < 1) plan->split_sph = 1;
        }
    } else {
        return fail(SCN_E_INVALID_ARG, "unknown LDS budget code %d", code);
    }
    return SCN_OK;
}

static int run_place(scn_ctx* c, scn_batch* b, const scn_gen_args* a, const scn::PlacePlan& plan,
                     int32_t* chosen, bool reset, hipStream_t st) {
    if (reset) SCN_HIP(scn::launch_reset(*b, st));
    if (plan.order) SCN_HIP(scn::launch_longest_first(*b, plan.order, plan.hist, st));
    SCN_HIP(scn::launch_scan_grid_values(*b, c->d_counters, st));
    SCN_HIP(scn::launch_place(*b, *a, plan, chosen, c->d_counters, st));
    return SCN_OK;
}

int scn_place_step(scn_ctx* c, scn_batch* b, const scn_gen_args* a, int32_t* chosen,
                   scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (int r = check_batch(b, true)) return r;
    scn::PlacePlan plan;
    if (int r = plan_place(c, b, a, 1, &plan)) return r;
    return run_place(c, b, a, plan, chosen, false, (hipStream_t)stream);
}

// One object step of the scenes rows[0 .. *n_rows) (a list compacted on the
// device; the launch covers n_scenes workgroups and the rest leave at once),
// for the learned pipeline: entries per `chunk` as in scn_place_internal.
__attribute__((visibility("hidden"))) int scn_place_rows(
    scn_ctx* c, scn_batch* b, const scn_gen_args* a, const int32_t* prop_bins, int prop_k,
    int32_t* resume, int chunk, int j_cap, const int32_t* rows, const int32_t* n_rows,
    void* map_keep, void* bnd_keep, const void* info_keep, float* hmap, hipStream_t st) {
    // the launch order is the list's: no longest-first order is computed; the
    // placed spheres stay in global memory (the kept state assumes it)
    scn_gen_args a1 = *a;
    if (a1.schedule == 0) a1.schedule = kDefaultSchedule;
    a1.schedule = (a1.schedule & ~(SCN_SCHED_LONGEST_FIRST | SCN_SCHED_LDS_MASK)) |
                  (SCN_SCHED_LDS_NONE << SCN_SCHED_LDS_SHIFT);
    a = &a1;
    scn::PlacePlan plan;
    if (int r = plan_place(c, b, a, 1, &plan, nullptr)) return r;
    plan.order = const_cast<int32_t*>(rows);   // read only by the kernel
    plan.hist = nullptr;
    plan.n_order = n_rows;
    plan.prop_bins = prop_bins;
    plan.prop_k = prop_bins ? prop_k : 0;
    plan.resume = resume;
    plan.chunk = chunk;
    plan.j_cap = j_cap;
    plan.n_active = nullptr;
    plan.map_keep = map_keep;
    plan.bnd_keep = bnd_keep;
    plan.info_keep = info_keep;
    plan.hmap = hmap;
    SCN_HIP(scn::launch_place(*b, *a, plan, nullptr, c->d_counters, st));
    return SCN_OK;
}

// The generation's launches (reset, scene order, place kernel) as a hipGraph:
// recorded on the context's capture stream, used to refresh the executable
// graph kept for this batch and plan (hipGraphExecUpdate: only the kernel
// arguments such as the seed differ between calls), then replayed on `st`.
static int run_place_graph(scn_ctx* c, scn_batch* b, const scn_gen_args* a,
                           const scn::PlacePlan& plan, hipStream_t st) {
    if (!c->cap_stream) SCN_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    SCN_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    const int r = run_place(c, b, a, plan, nullptr, true, c->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (r != SCN_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return r != SCN_OK ? r : fail(SCN_E_HIP, "generation capture: %s", hipGetErrorString(e));
    }
    char key[512];
    snprintf(key, sizeof key, "%p %p %p %p %p %p %p %p %p %p %p %p %d %d %d %d %d %d %d %d %d %p",
             (const void*)b->obj_off, (const void*)b->sph_off, (const void*)b->tmpl,
             (const void*)b->sup, (const void*)b->box, (const void*)b->grid,
             (const void*)b->placed, (const void*)b->n_placed, (const void*)b->status,
             (const void*)b->rec, (const void*)b->obj_ncand, (const void*)b->grid_off, b->n_scenes,
             b->n_objects, b->geometry, plan.mode, plan.waves, plan.spl, plan.cap_sph,
             plan.split_sph, plan.max_steps, (const void*)plan.order);
    auto it = c->plain_graphs.find(key);
    if (it != c->plain_graphs.end()) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(it->second, g, &bad, &res) != hipSuccess ||
            res != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(it->second);
            c->plain_graphs.erase(it);
            it = c->plain_graphs.end();
        }
    }
    if (it == c->plain_graphs.end()) {
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(SCN_E_HIP, "generation graph: %s", hipGetErrorString(ei));
        }
        it = c->plain_graphs.emplace(key, ex).first;
    }
    (void)hipGraphDestroy(g);
    SCN_HIP(hipGraphLaunch(it->second, st));
    return SCN_OK;
}

int scn_generate_scenes(scn_ctx* c, scn_batch* b, const scn_gen_args* a, scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (int r = check_batch(b, true)) return r;
    scn::PlacePlan plan;
    if (int r = plan_place(c, b, a, a ? a->max_steps : 0, &plan)) return r;
    if (a->use_graph) return run_place_graph(c, b, a, plan, (hipStream_t)stream);
    return run_place(c, b, a, plan, nullptr, true, (hipStream_t)stream);
}

int scn_generate_scenes_noalloc(scn_ctx* c, scn_batch* b, const scn_gen_args* a,
                                scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (!b) return fail(SCN_E_INVALID_ARG, "null batch");
    if (b->n_scenes > SCN_NOALLOC_MAX_SCENES)
        return fail(SCN_E_INVALID_ARG, "%d scenes exceed the fixed scratch of %d scenes",
                    b->n_scenes, SCN_NOALLOC_MAX_SCENES);
    if (int r = check_batch(b, true)) return r;
    if (!a) return fail(SCN_E_INVALID_ARG, "null args");
    if (a->use_graph)
        return fail(SCN_E_UNSUPPORTED, "scn_generate_scenes_noalloc launches eagerly (use_graph = 0)");
    void* ws = scratch_ptr(c->device);
    if (!ws) return fail(SCN_E_HIP, "no scratch address for device %d", c->device);
    scn::PlacePlan plan;
    if (int r = plan_place(c, b, a, a->max_steps, &plan, ws)) return r;
    return run_place(c, b, a, plan, nullptr, true, (hipStream_t)stream);
}

int scn_autotune(scn_ctx* c, scn_batch* b, const scn_gen_args* a, int32_t* best_schedule,
                 float* best_ms, scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (int r = check_batch(b, true)) return r;
    if (!a) return fail(SCN_E_INVALID_ARG, "null args");
    const hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    SCN_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SCN_E_HIP, "hipEventCreate failed");
    }
    // time one full generation under `sched`: the best of three runs after a
    // warm-up run (single runs vary by a few per cent)
    auto time_one = [&](int sched, float* ms) -> int {
        scn_gen_args t = *a;
        t.schedule = sched;
        t.max_steps = 0;
        scn::PlacePlan plan;
        if (int r = plan_place(c, b, &t, 0, &plan)) return r;
        if (int r = run_place(c, b, &t, plan, nullptr, true, st)) return r;
        for (int rep = 0; rep < 3; ++rep) {
            if (hipEventRecord(e0, st) != hipSuccess) return fail(SCN_E_HIP, "event record");
            if (int r = run_place(c, b, &t, plan, nullptr, true, st)) return r;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return fail(SCN_E_HIP, "event sync");
            float m = 0.f;
            if (hipEventElapsedTime(&m, e0, e1) != hipSuccess) return fail(SCN_E_HIP, "elapsed time");
            if (rep == 0 || m < *ms) *ms = m;
        }
        return SCN_OK;
    };
    int best = -1;
    float best_t = 0.f;
    int rc = SCN_OK;
    auto consider = [&](int sched) {
        if (rc != SCN_OK) return;
        float ms = 0.f;
        rc = time_one(sched, &ms);
        if (rc == SCN_OK && (best < 0 || ms < best_t)) { best = sched; best_t = ms; }
    };
    // Coordinate descent: LDS budget (4 waves, longest first), then waves,
    // then the scene order.
    const int lpt = SCN_SCHED_LONGEST_FIRST;
    for (int code : {0, 2, 4, (int)SCN_SCHED_LDS_NONE}) consider(4 | lpt | (code << SCN_SCHED_LDS_SHIFT));
    const int lds_bits = best & SCN_SCHED_LDS_MASK;
    for (int w : {1, 2, 8, 16}) consider(w | lpt | lds_bits);
    consider(best & ~SCN_SCHED_LONGEST_FIRST);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SCN_OK) return rc;
    c->tuned[shape_key(b)] = scn_ctx::Tuned{best, best_t};
    if (best_schedule) *best_schedule = best;
    if (best_ms) *best_ms = best_t;
    return SCN_OK;
}

int scn_autotune_save(scn_ctx* c, const char* path) {
    if (!c || !path) return fail(SCN_E_INVALID_ARG, "null context or path");
    FILE* f = fopen(path, "w");
    if (!f) return fail(SCN_E_INVALID_ARG, "cannot write %s", path);
    fprintf(f, "{\"scn_autotune\": [\n");
    size_t i = 0;
    for (const auto& kv : c->tuned) {
        fprintf(f, "  {\"shape\": \"%s\", \"schedule\": %d, \"ms\": %.4f}%s\n", kv.first.c_str(),
                kv.second.schedule, kv.second.ms, ++i < c->tuned.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    fclose(f);
    return SCN_OK;
}

int scn_autotune_load(scn_ctx* c, const char* path) {
    if (!c || !path) return fail(SCN_E_INVALID_ARG, "null context or path");
    FILE* f = fopen(path, "r");
    if (!f) return fail(SCN_E_INVALID_ARG, "cannot read %s", path);
    char line[512], shape[128];
    int sched;
    float ms;
    while (fgets(line, sizeof line, f)) {
        if (sscanf(line, " {\"shape\": \"%127[^\"]\", \"schedule\": %d, \"ms\": %f", shape, &sched,
                   &ms) == 3)
            c->tuned[shape] = scn_ctx::Tuned{sched, ms};
    }
    fclose(f);
    return SCN_OK;
}

}  // extern "C"
