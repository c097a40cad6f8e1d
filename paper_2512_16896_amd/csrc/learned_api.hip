// learned_api.hip -- C ABI of the learned pose proposal: state features,
// ranking, label harvesting and the learned generation pipeline.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "scn.h"

using scn::align256;

namespace {

// The learned proposal's state features hold one height map over the support
// of each scene's first object, and its label harvest tests boxes and placed
// spheres only: batches with voxel grids, or more supports than scenes (some
// scene's objects on several supports), are outside what it computes.
int check_single_support(const scn_batch* b) {
    if (b->obj_rel || b->obj_ratio || b->robot)
        return scn_fail(SCN_E_UNSUPPORTED,
                        "the learned proposal does not support spatial relations, "
                        "ratio_on_support or reachability (its bins cover the whole support)");
    if (b->grid_off)
        return scn_fail(SCN_E_UNSUPPORTED, "the learned proposal does not support voxel-grid batches");
    if (b->n_supports > b->n_scenes)
        return scn_fail(SCN_E_UNSUPPORTED,
                        "the learned proposal needs one support per scene (%d supports, %d scenes)",
                        b->n_supports, b->n_scenes);
    return SCN_OK;
}

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

int scn_features(scn_ctx* c, int32_t n, const float* hmap, const float* desc,
                 const int32_t* obj_idx, uint16_t* x, scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (n < 0) return scn_fail(SCN_E_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!hmap || !desc || !obj_idx || !x))
        return scn_fail(SCN_E_INVALID_ARG, "hmap, desc, obj_idx and x required");
    SCN_HIP(scn::launch_features(n, hmap, desc, obj_idx, SCN_FEATURES, x, (hipStream_t)stream));
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
    if (int r = check_single_support(b)) return r;
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

// Defined in api.hip: plan and launch of the fused place kernel.
__attribute__((visibility("hidden"))) int scn_place_internal(
    scn_ctx* c, scn_batch* b, const scn_gen_args* a, int max_steps, int32_t* chosen, bool reset,
    const int32_t* prop_bins, int prop_k, int32_t* resume, int chunk, int j_cap,
    int32_t* n_active, void* order_ws, hipStream_t st);

}  // extern "C"

// Layout of the learned generation's workspace: the scene order region, the
// network's hidden activations, then the pipeline buffers below.
namespace {
struct LearnedWs {
    void* order;
    void* act;
    float* hmap;
    float* desc;
    uint16_t* x;
    float* logits;
    int32_t* bins;
    int32_t *obj_idx, *before, *placed_now, *resume, *n_active;
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
    t.order = take(scn::ws_order_bytes(b->n_scenes));
    t.act = take(scn::ws_mlp_forward_bytes(net, b->n_scenes));
    t.hmap = (float*)take(n * SCN_HMAP_CELLS * 4);
    t.desc = (float*)take((size_t)b->n_objects * SCN_DESC * 4);
    t.x = (uint16_t*)take(n * SCN_FEATURES * 2);
    t.logits = (float*)take(n * SCN_BINS * 4);
    t.bins = (int32_t*)take(n * (size_t)top_k * 4);
    t.obj_idx = (int32_t*)take(n * 4);
    t.before = (int32_t*)take(n * 4);
    t.placed_now = (int32_t*)take(n * 4);
    t.resume = (int32_t*)take(n * 4);
    t.n_active = (int32_t*)take(8);
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
    if (int r = check_single_support(b)) return r;
    // Schedule 0: 2 waves, batch order, placed spheres from global memory.
    // Each step launch is as long as its slowest scene's proposals and
    // fallback chunk; measured on batched-4096 this beat the plain default
    // of 4 waves (34.2 vs 37.3 ms per generation) and 1, 3 or 8 waves.
    scn_gen_args args = *a;
    if (args.schedule == 0) args.schedule = 2 | (SCN_SCHED_LDS_NONE << SCN_SCHED_LDS_SHIFT);
    a = &args;
    const hipStream_t st = (hipStream_t)stream;
    const int n = b->n_scenes;
    if (n == 0) return SCN_OK;
    void* ws;
    if (int r = scn_workspace(c, learned_layout(b, net, top_k, nullptr, nullptr), &ws)) return r;
    LearnedWs W;
    learned_layout(b, net, top_k, (char*)ws, &W);
    float* hmap = W.hmap;
    float* desc = W.desc;
    uint16_t* x = W.x;
    float* logits = W.logits;
    int32_t* bins = W.bins;
    int32_t* obj_idx = W.obj_idx;
    int32_t* before = W.before;
    int32_t* placed_now = W.placed_now;
    int32_t* resume = W.resume;
    int32_t* n_active = W.n_active;

    const int j_cap = a->max_steps > 0 && a->max_steps < b->max_objects_per_scene ? a->max_steps : 0;
    // uniform entries tried per launch: one attempt of the default size, so
    // that a launch never waits on one scene's whole fallback
    const int chunk = a->fallback_chunk < 0 ? 0
                      : a->fallback_chunk > 0 ? a->fallback_chunk
                      : (b->max_cand_per_object > 0 ? b->max_cand_per_object : a->default_ncand);
    // every launch makes progress on each active scene (a placement, the
    // invalid mark, or `chunk` more entries), which bounds the launches
    long long c_max = b->max_cand_per_object > 0 ? b->max_cand_per_object : a->default_ncand;
    if (c_max < 1) c_max = 1;
    const long long per_obj = chunk > 0 ? 1 + ((long long)(a->retries + 1) * c_max + chunk - 1) / chunk : 1;
    const long long max_launch = (long long)(j_cap > 0 ? j_cap : b->max_objects_per_scene) * per_obj + 1;

    SCN_HIP(scn::launch_reset(*b, st));
    SCN_HIP(scn::launch_fill_i32(resume, n, 0, st));
    SCN_HIP(scn::launch_descriptor(*b, desc, st));
    SCN_HIP(scn::launch_hmap_boxes(*b, hmap, st));

    // One step launch on stream s: for scenes that start a new object, the
    // features, the network and the top-k (skipped when no scene does:
    // resumed scenes need no proposal); then the place kernel, the height map
    // update of the scenes that placed, and the read-back of the two counters.
    auto enqueue_step = [&](hipStream_t s, bool with_net) -> int {
        if (with_net) {
            SCN_HIP(scn::launch_next_object(*b, resume, j_cap, obj_idx, s));
            SCN_HIP(scn::launch_features(n, hmap, desc, obj_idx, SCN_FEATURES, x, s));
            if (int r = scn_mlp_forward_ws(net, x, n, logits, W.act, s)) return r;
            SCN_HIP(scn::launch_topk(n, logits, top_k, obj_idx, bins, s));
        }
        SCN_HIP(scn::launch_copy_i32(b->n_placed, before, n, s));
        SCN_HIP(scn::launch_fill_i32(n_active, 2, 0, s));
        if (int r = scn_place_internal(c, b, a, 1, nullptr, false, bins, top_k, resume, chunk,
                                       j_cap, n_active, W.order, s))
            return r;
        SCN_HIP(scn::launch_last_object(*b, before, placed_now, s));
        SCN_HIP(scn::launch_hmap_raise(*b, placed_now, nullptr, hmap, s));
        SCN_HIP(hipMemcpyAsync(c->h_flag, n_active, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        return SCN_OK;
    };

    // With use_graph the two step variants are captured once (on the
    // context's own stream, after the first step ran eagerly and made every
    // allocation) and replayed on `stream`: every step has the same kernel
    // arguments, since the state lives in device memory.
    hipGraphExec_t exec[2] = {nullptr, nullptr};   // [with network, resume only]
    auto release = [&]() {
        for (auto& e : exec)
            if (e) {
                (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
    };
    auto capture = [&](bool with_net, hipGraphExec_t* out) -> int {
        if (!c->cap_stream)
            SCN_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        SCN_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
        const int r = enqueue_step(c->cap_stream, with_net);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (r != SCN_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return r != SCN_OK ? r : scn_fail(SCN_E_HIP, "step capture: %s", hipGetErrorString(e));
        }
        const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return scn_fail(SCN_E_HIP, "step graph: %s", hipGetErrorString(ei));
        return SCN_OK;
    };

    bool fresh = true;   // some scene starts a new object (needs the network)
    for (long long it = 0; it < max_launch; ++it) {
        int r = SCN_OK;
        if (a->use_graph && it > 0) {
            hipGraphExec_t& e = exec[fresh ? 0 : 1];
            if (!e) r = capture(fresh, &e);
            if (r == SCN_OK && hipGraphLaunch(e, st) != hipSuccess)
                r = scn_fail(SCN_E_HIP, "step graph launch failed");
        } else {
            r = enqueue_step(st, fresh);
        }
        if (r == SCN_OK && hipStreamSynchronize(st) != hipSuccess)
            r = scn_fail(SCN_E_HIP, "step failed: %s", hipGetErrorString(hipGetLastError()));
        if (r != SCN_OK) {
            release();
            return r;
        }
        if (c->h_flag[0] == 0) break;
        fresh = c->h_flag[1] > 0;
    }
    release();
    return SCN_OK;
}

}  // extern "C"
