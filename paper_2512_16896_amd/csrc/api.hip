// api.hip -- the C ABI of libscn.so (declared in include/scn.h): argument
// validation, contexts, launch planning and error reporting.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.h"
#include "scn.h"

struct scn_ctx {
    int device;
    int lds_per_block;
    int n_cu;
    int64_t* d_counters;   // scn::kNumCounters int64
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define SCN_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(SCN_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
    } while (0)

int check_ctx(scn_ctx* c) {
    if (!c) return fail(SCN_E_INVALID_ARG, "null context");
    if (hipSetDevice(c->device) != hipSuccess) return fail(SCN_E_HIP, "hipSetDevice failed");
    return SCN_OK;
}

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
    auto* c = new scn_ctx();
    c->device = device;
    c->n_cu = p.multiProcessorCount;
    c->lds_per_block = (int)p.sharedMemPerBlock;
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess &&
        optin > c->lds_per_block)
        c->lds_per_block = optin;
    if (hipMalloc((void**)&c->d_counters, sizeof(int64_t) * scn::kNumCounters) != hipSuccess) {
        delete c;
        return fail(SCN_E_HIP, "hipMalloc(counters) failed");
    }
    if (hipMemset(c->d_counters, 0, sizeof(int64_t) * scn::kNumCounters) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->d_counters);
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
    delete c;
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
    if (out->error_word & scn::kErrCapacity)
        return fail(SCN_E_CAPACITY, "a scene exceeded the planned capacity and was skipped");
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
    if (!(margin >= 0.f)) return fail(SCN_E_INVALID_ARG, "margin must be >= 0");
    if ((int64_t)max_cand > 65535LL * 256) return fail(SCN_E_UNSUPPORTED, "max_cand too large");
    SCN_HIP(scn::launch_check(*b, obj_idx, cand_off, max_cand, poses, margin, clearance, collide,
                              (hipStream_t)stream));
    return SCN_OK;
}

int scn_reset_scenes(scn_ctx* c, scn_batch* b, scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (int r = check_batch(b, true)) return r;
    SCN_HIP(scn::launch_reset(*b, (hipStream_t)stream));
    return SCN_OK;
}

static int plan_place(scn_ctx* c, const scn_batch* b, const scn_gen_args* a, int max_steps,
                      scn::PlacePlan* plan) {
    if (!a) return fail(SCN_E_INVALID_ARG, "null args");
    if (!(a->margin >= 0.f)) return fail(SCN_E_INVALID_ARG, "margin must be >= 0");
    if (a->retries < 0) return fail(SCN_E_INVALID_ARG, "retries must be >= 0");
    if (!b->obj_ncand && a->default_ncand <= 0)
        return fail(SCN_E_INVALID_ARG, "default_ncand must be > 0 when obj_ncand is NULL");
    const int S = b->max_spheres_per_object;
    if (S > 256) return fail(SCN_E_UNSUPPORTED, "max_spheres_per_object %d > 256", S);
    plan->spl = S <= 64 ? 1 : (S <= 128 ? 2 : 4);
    plan->waves = 4;
    if (a->schedule > 0) {
        const int w = a->schedule & 0xF;
        if (w != 1 && w != 2 && w != 4 && w != 8)
            return fail(SCN_E_INVALID_ARG, "schedule waves must be 1, 2, 4 or 8");
        plan->waves = w;
    }
    plan->cap_sph = b->max_spheres_per_scene > 0 ? b->max_spheres_per_scene : 1;
    plan->cap_obj = b->max_objects_per_scene > 0 ? b->max_objects_per_scene : 1;
    plan->max_steps = max_steps;
    const long long bytes = 16LL * plan->cap_sph + 16LL * plan->cap_obj;
    if (bytes > c->lds_per_block)
        return fail(SCN_E_UNSUPPORTED, "a scene needs %lld B of LDS (> %d)", bytes, c->lds_per_block);
    plan->lds_bytes = (int)bytes;
    return SCN_OK;
}

int scn_place_step(scn_ctx* c, scn_batch* b, const scn_gen_args* a, int32_t* chosen,
                   scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (int r = check_batch(b, true)) return r;
    scn::PlacePlan plan;
    if (int r = plan_place(c, b, a, 1, &plan)) return r;
    SCN_HIP(scn::launch_place(*b, *a, plan, chosen, c->d_counters, (hipStream_t)stream));
    return SCN_OK;
}

int scn_generate_scenes(scn_ctx* c, scn_batch* b, const scn_gen_args* a, scn_stream stream) {
    if (int r = check_ctx(c)) return r;
    if (int r = check_batch(b, true)) return r;
    scn::PlacePlan plan;
    if (int r = plan_place(c, b, a, a ? a->max_steps : 0, &plan)) return r;
    SCN_HIP(scn::launch_reset(*b, (hipStream_t)stream));
    SCN_HIP(scn::launch_place(*b, *a, plan, nullptr, c->d_counters, (hipStream_t)stream));
    return SCN_OK;
}

}  // extern "C"
