// learned_api.hip -- C ABI of the learned pose proposal: state features,
// ranking, label harvesting and the learned generation pipeline.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "scn.h"

using scn::align256;

namespace {

// The learned proposal's pose bins cover a whole support rectangle and turn
// about z only: batches whose candidates are drawn elsewhere (spatial
// relations, ratio_on_support), filtered by reachability, or turned by stable
// poses are outside what it computes.
int check_learned_batch(const scn_batch* b) {
    if (b->obj_rel || b->obj_ratio || b->robot || b->obj_pose_off)
        return scn_fail(SCN_E_UNSUPPORTED,
                        "the learned proposal does not support spatial relations, "
                        "ratio_on_support, reachability or stable poses (its bins cover the "
                        "whole support and turns about z)");
    return SCN_OK;
}

// Waves per scene of the learned pipeline's launches: the first ticks'
// new-object launch (throughput), the others (latency).  Measured on the
// 4096-scene workload (20 objects of 64 spheres, 1024 candidates per attempt):
// 19.4 ms per generation with 1 and 4, against 20-27 ms with 2 / 2-8 and
// 42 ms with 2 / 16.
constexpr int kBulkWaves = 1;
constexpr int kWideWaves = 4;

int check_scenes(const scn_batch* b) {
    if (!b) return scn_fail(SCN_E_INVALID_ARG, "null batch");
    if (b->n_scenes < 0 || b->n_objects < 0) return scn_fail(SCN_E_INVALID_ARG, "negative sizes");
    if (b->n_scenes > 0 && (!b->obj_off || !b->box_off || !b->sup || !b->obj_sup))
        return scn_fail(SCN_E_INVALID_ARG, "obj_off/box_off/sup/obj_sup required");
    if (b->n_objects > 0 && (!b->sph_off || !b->tmpl))
        return scn_fail(SCN_E_INVALID_ARG, "sph_off/tmpl required");
    if (b->n_boxes > 0 && !b->box) return scn_fail(SCN_E_INVALID_ARG, "box required");
    return SCN_OK;
}

}  // namespace

extern "C" {

int scn_descriptors(scn_ctx* c, const scn_batch* b, float* desc, scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (int r = check_scenes(b)) return r;
    if (b->n_objects > 0 && !desc) return scn_fail(SCN_E_INVALID_ARG, "desc required");
    SCN_HIP(scn::launch_descriptor(*b, desc, (hipStream_t)stream));
    return SCN_OK;
}

int scn_heightmaps(scn_ctx* c, const scn_batch* b, const int32_t* n_state, float* hmap,
                   scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (int r = check_scenes(b)) return r;
    if (b->n_scenes == 0) return SCN_OK;
    if (!hmap) return scn_fail(SCN_E_INVALID_ARG, "hmap required");
    const int32_t* ns = n_state ? n_state : b->n_placed;
    if (!ns || !b->placed) return scn_fail(SCN_E_INVALID_ARG, "n_state (or n_placed) and placed required");
    const hipStream_t st = (hipStream_t)stream;
    SCN_HIP(scn::launch_hmap_boxes(*b, hmap, st));
    SCN_HIP(scn::launch_hmap_raise(*b, nullptr, ns, hmap, st));
    return SCN_OK;
}

int scn_features(scn_ctx* c, const scn_batch* b, int32_t n, const float* hmap,
                 const float* desc, const int32_t* obj_idx, uint16_t* x, scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (!b || !b->obj_sup) return scn_fail(SCN_E_INVALID_ARG, "batch with obj_sup required");
    if (n < 0) return scn_fail(SCN_E_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!hmap || !desc || !obj_idx || !x))
        return scn_fail(SCN_E_INVALID_ARG, "hmap, desc, obj_idx and x required");
    SCN_HIP(scn::launch_features(n, hmap, desc, obj_idx, b->obj_sup, SCN_FEATURES, x,
                                 (hipStream_t)stream));
    return SCN_OK;
}

int scn_proposal_topk(scn_ctx* c, const float* logits, int32_t M, int32_t k,
                      const int32_t* active, int32_t* bins, scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (M < 0 || k < 1 || k > SCN_BINS) return scn_fail(SCN_E_INVALID_ARG, "bad M or k");
    if (M > 0 && (!logits || !bins)) return scn_fail(SCN_E_INVALID_ARG, "logits and bins required");
    SCN_HIP(scn::launch_topk(M, logits, k, active, bins, (hipStream_t)stream));
    return SCN_OK;
}

int scn_harvest_labels(scn_ctx* c, const scn_batch* b, const int32_t* n_state, int32_t L,
                       uint64_t seed, int32_t round, float margin, int32_t* bins, float* accept,
                       scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (int r = check_scenes(b)) return r;
    if (int r = check_learned_batch(b)) return r;
    if (L <= 0 || round < 0 || round > 0xFFFF || !(margin >= 0.f))
        return scn_fail(SCN_E_INVALID_ARG, "bad L, round or margin");
    if (b->n_scenes == 0) return SCN_OK;
    const int32_t* ns = n_state ? n_state : b->n_placed;
    if (!ns || !b->placed || !bins || !accept)
        return scn_fail(SCN_E_INVALID_ARG, "n_state (or n_placed), placed, bins and accept required");
    if (L > 65535 * 64) return scn_fail(SCN_E_UNSUPPORTED, "L too large");
    SCN_HIP(scn::launch_harvest(*b, ns, L, seed, round, margin, bins, accept, c->d_counters,
                                (hipStream_t)stream));
    return SCN_OK;
}

// Defined in api.hip: one object step of the fused place kernel over the
// scenes of a device-compacted list.
__attribute__((visibility("hidden"))) int scn_place_rows(
    scn_ctx* c, scn_batch* b, const scn_gen_args* a, const int32_t* prop_bins, int prop_k,
    int32_t* resume, int chunk, int j_cap, const int32_t* rows, const int32_t* n_rows,
    void* map_keep, void* bnd_keep, const void* info_keep, float* hmap, hipStream_t st);

}  // extern "C"

// Layout of the learned generation's workspace: the network's hidden
// activations, then the pipeline buffers below.
namespace {
struct LearnedWs {
    void* act;
    float* hmap;
    float* desc;
    uint16_t* x;
    float* logits;
    int32_t* bins;
    int32_t *obj_idx, *list, *count, *resume;
    void *map_keep, *bnd_keep, *info_keep;   // state the step launches keep (PlacePlan)
    int32_t* sup_scene;                       // the scene of each support (checked)
};
size_t learned_layout(const scn_batch* b, const scn_mlp* net, int top_k, char* base,
                      LearnedWs* w) {
    const size_t n = (size_t)b->n_scenes;
    size_t off = 0;
    auto take = [&](size_t sz) -> char* {
        char* q = base ? base + off : nullptr;
        off += align256(sz);
        return q;
    };
    LearnedWs t;
    t.act = take(scn::ws_mlp_forward_bytes(net, b->n_scenes));
    t.hmap = (float*)take((size_t)b->n_supports * SCN_HMAP_CELLS * 4);
    t.sup_scene = (int32_t*)take((size_t)b->n_supports * 4);
    t.desc = (float*)take((size_t)b->n_objects * SCN_DESC * 4);
    t.x = (uint16_t*)take(n * SCN_FEATURES * 2);
    t.logits = (float*)take(n * SCN_BINS * 4);
    t.bins = (int32_t*)take(n * (size_t)top_k * 4);
    t.obj_idx = (int32_t*)take(n * 4);
    t.list = (int32_t*)take(2 * n * 4);
    t.count = (int32_t*)take(8);
    t.resume = (int32_t*)take(n * 4);
    t.map_keep = take(b->grid_off ? 0 : n * (size_t)scn::kMapBytes);
    t.bnd_keep = take((size_t)b->n_objects * 16);
    t.info_keep = take((size_t)b->n_objects * 64);
    if (w) *w = t;
    return off;
}
}  // namespace

size_t scn::ws_learned_bytes(const scn_batch* b, const scn_mlp* net, int top_k) {
    return learned_layout(b, net, top_k, nullptr, nullptr);
}

extern "C" {

int scn_generate_scenes_learned(scn_ctx* c, scn_batch* b, const scn_gen_args* a,
                                const scn_mlp* net, int32_t top_k, scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (int r = check_scenes(b)) return r;
    if (!a || !net) return scn_fail(SCN_E_INVALID_ARG, "args and network required");
    if (top_k < 1 || top_k > SCN_BINS) return scn_fail(SCN_E_INVALID_ARG, "top_k out of range");
    if (net->dims[0] != SCN_FEATURES || net->dims[SCN_MLP_LAYERS] != SCN_BINS)
        return scn_fail(SCN_E_INVALID_ARG, "network must map %d features to %d bins",
                        SCN_FEATURES, SCN_BINS);
    for (int l = 0; l < SCN_MLP_LAYERS; ++l) {
        if (net->dims[l + 1] <= 0 || net->dims[l] % 32)
            return scn_fail(SCN_E_INVALID_ARG, "layer %d: dims must be positive multiples of 32", l);
        if (!net->b[l] || !net->wb[l])
            return scn_fail(SCN_E_INVALID_ARG, "layer %d tensors missing", l);
    }
    if (!b->placed || !b->n_placed || !b->status || !b->rec)
        return scn_fail(SCN_E_INVALID_ARG, "placed/n_placed/status/rec required");
    if (a->retries < 0) return scn_fail(SCN_E_INVALID_ARG, "retries must be >= 0");
    if (int r = check_learned_batch(b)) return r;
    // Launch shapes.  The first ticks (as many as a scene has objects) carry
    // nearly every scene in the new-object list: their launch runs
    // args->schedule (0: one wave per scene, placed spheres from global
    // memory), sized for throughput.  The pending list, and both lists in the
    // later ticks, hold a few scenes whose steps are latency-bound: they run
    // args->wide_schedule (0: 4 waves per scene).  None of this changes a
    // placement.
    scn_gen_args bulk = *a, wide = *a;
    if (bulk.schedule == 0) bulk.schedule = kBulkWaves | (SCN_SCHED_LDS_NONE << SCN_SCHED_LDS_SHIFT);
    wide.schedule = a->wide_schedule != 0 ? a->wide_schedule
                                          : kWideWaves | (SCN_SCHED_LDS_NONE << SCN_SCHED_LDS_SHIFT);
    a = &bulk;
    const hipStream_t st = (hipStream_t)stream;
    const int n = b->n_scenes;
    if (n == 0) return SCN_OK;
    void* ws;
    if (int r = scn_workspace(c, learned_layout(b, net, top_k, nullptr, nullptr), &ws)) return r;
    LearnedWs W;
    learned_layout(b, net, top_k, (char*)ws, &W);
    if (!c->aux_stream) SCN_HIP(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
    for (auto& e : c->ev)
        if (!e) SCN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));

    const int j_cap = a->max_steps > 0 && a->max_steps < b->max_objects_per_scene ? a->max_steps : 0;
    // uniform entries a pending object tries per tick (0: all that remain)
    const int chunk = a->fallback_chunk > 0 ? a->fallback_chunk : 0;
    // every tick makes progress on each listed scene (a placement, the
    // invalid mark, the proposals, or `chunk` more uniform entries), which
    // bounds the ticks
    long long c_max = b->max_cand_per_object > 0 ? b->max_cand_per_object : a->default_ncand;
    if (c_max < 1) c_max = 1;
    const long long per_obj = 1 + (chunk > 0 ? ((long long)(a->retries + 1) * c_max + chunk - 1) / chunk : 1);
    const long long max_ticks =
        (long long)(j_cap > 0 ? j_cap : b->max_objects_per_scene) * per_obj + 1;

    SCN_HIP(scn::launch_reset(*b, st));
    SCN_HIP(scn::launch_fill_i32(W.resume, n, 0, st));
    SCN_HIP(scn::launch_descriptor(*b, W.desc, st));
    SCN_HIP(scn::launch_support_scene(*b, W.sup_scene, c->d_counters, st));
    SCN_HIP(scn::launch_hmap_boxes(*b, W.hmap, st));
    SCN_HIP(scn::launch_object_info(*b, a->margin, W.info_keep, st));
    void* map_keep = b->grid_off ? nullptr : W.map_keep;

    int32_t* list_new = W.list;        // scenes starting an object: need proposals
    int32_t* list_pend = W.list + n;   // scenes resuming a pending object's uniform entries
    auto plan = [&](hipStream_t s) -> int {
        SCN_HIP(scn::launch_fill_i32(W.count, 2, 0, s));
        SCN_HIP(scn::launch_tick_plan(*b, W.resume, j_cap, W.list, W.obj_idx, W.count, s));
        return SCN_OK;
    };
    // One tick on stream s (and the context's second stream): the plan
    // splits the scenes with work into the two lists; the pending ones try
    // their next `chunk` uniform entries on the second stream while the new
    // ones run features, network and top-k over their compacted rows and try
    // their proposals alone; a placing step raises its scene's height map at
    // the commit.  The lists are disjoint, so the two streams never touch
    // the same scene.  Launch sizes are fixed (n rows / scenes); each kernel
    // reads its list's length on the device and the rest of its grid leaves.
    auto tick = [&](hipStream_t s, bool late) -> int {
        if (int r = plan(s)) return r;
        SCN_HIP(hipEventRecord(c->ev[0], s));
        SCN_HIP(hipStreamWaitEvent(c->aux_stream, c->ev[0], 0));
        if (int r = scn_place_rows(c, b, &wide, W.bins, top_k, W.resume, chunk, j_cap, list_pend,
                                   W.count + 1, map_keep, W.bnd_keep, W.info_keep, W.hmap,
                                   c->aux_stream))
            return r;
        SCN_HIP(hipEventRecord(c->ev[1], c->aux_stream));
        SCN_HIP(scn::launch_features(n, W.hmap, W.desc, W.obj_idx, b->obj_sup, SCN_FEATURES, W.x,
                                     s, W.count));
        if (int r = scn_mlp_forward_ws(net, W.x, n, W.logits, W.act, s, W.count)) return r;
        SCN_HIP(scn::launch_topk(n, W.logits, top_k, nullptr, W.bins, s, list_new, W.count));
        if (int r = scn_place_rows(c, b, late ? &wide : a, W.bins, top_k, W.resume, -1, j_cap,
                                   list_new, W.count, map_keep, W.bnd_keep, W.info_keep,
                                   W.hmap, s))
            return r;
        SCN_HIP(hipStreamWaitEvent(s, c->ev[1], 0));
        return SCN_OK;
    };

    // With use_graph the two kinds of tick are captured (on the context's
    // capture stream, forking to the second stream and joining back) and
    // replayed on `stream`: ticks of a kind have the same kernel arguments,
    // since the state lives in device memory.
    hipGraphExec_t exec[2] = {nullptr, nullptr};   // [first ticks, later ticks]
    auto release = [&]() {
        for (auto& e : exec)
            if (e) {
                (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
    };
    if (a->use_graph) {
        if (!c->cap_stream)
            SCN_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        for (int k = 0; k < 2; ++k) {
            SCN_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
            const int r = tick(c->cap_stream, k == 1);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
            if (r != SCN_OK || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                release();
                return r != SCN_OK ? r : scn_fail(SCN_E_HIP, "tick capture: %s", hipGetErrorString(e));
            }
            const hipError_t ei = hipGraphInstantiate(&exec[k], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ei != hipSuccess) {
                release();
                return scn_fail(SCN_E_HIP, "tick graph: %s", hipGetErrorString(ei));
            }
        }
    }

    // Ticks run in batches without a host wait; after each batch the host
    // reads the two list sizes of a fresh plan (8 bytes) and stops when both
    // are zero.  No scene can finish in fewer ticks than it has objects, so
    // the first batch is that long.
    long long done = 0;
    long long batch = b->max_objects_per_scene > 0 ? b->max_objects_per_scene : 1;
    if (j_cap > 0 && j_cap < batch) batch = j_cap;
    const long long first = batch;   // ticks of the first kind
    int r = SCN_OK;
    while (r == SCN_OK) {
        const long long m = batch < max_ticks - done ? batch : max_ticks - done;
        for (long long t = 0; t < m && r == SCN_OK; ++t) {
            const bool late = done + t >= first;
            if (exec[late])
                r = hipGraphLaunch(exec[late], st) == hipSuccess
                        ? SCN_OK
                        : scn_fail(SCN_E_HIP, "tick graph launch failed");
            else
                r = tick(st, late);
        }
        done += m;
        if (r != SCN_OK) break;
        r = plan(st);
        if (r == SCN_OK && hipMemcpyAsync(c->h_flag, W.count, 2 * sizeof(int32_t),
                                          hipMemcpyDeviceToHost, st) != hipSuccess)
            r = scn_fail(SCN_E_HIP, "list size read failed");
        if (r == SCN_OK && hipStreamSynchronize(st) != hipSuccess)
            r = scn_fail(SCN_E_HIP, "tick failed: %s", hipGetErrorString(hipGetLastError()));
        if (r != SCN_OK || (c->h_flag[0] == 0 && c->h_flag[1] == 0) || done >= max_ticks) break;
        batch = 8;
    }
    release();
    return r;
}

}  // extern "C"
