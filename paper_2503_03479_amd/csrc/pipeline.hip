// The whole parameter-search path for one image pair (Sec. III.B): simulate the
// views of both images, extract ORB on every view, match all view pairs and pick
// the best one, as one asynchronous sequence of launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "internal.h"

namespace xa {
namespace {

struct PairWs {
    size_t arena_a, mask_a, sim_a, ext_a, arena_b, mask_b, sim_b, ext_b, total;
};

PairWs pair_layout(const xa_plan_header* a, const xa_plan_header* b) {
    PairWs w{};
    size_t o = 0;
    w.arena_a = o; o = align_up(o + size_t(a->arena_bytes));
    w.mask_a = o;  o = align_up(o + size_t(a->arena_bytes));
    w.sim_a = o;   o = align_up(o + simulate_ws_bytes(a));
    w.ext_a = o;   o = align_up(o + extract_ws_layout(a).total);
    w.arena_b = o; o = align_up(o + size_t(b->arena_bytes));
    w.mask_b = o;  o = align_up(o + size_t(b->arena_bytes));
    w.sim_b = o;   o = align_up(o + simulate_ws_bytes(b));
    w.ext_b = o;   o = align_up(o + extract_ws_layout(b).total);
    w.total = o;
    return w;
}

}  // namespace
}  // namespace xa

using namespace xa;

extern "C" size_t xa_match_pair_workspace_size(const void* plan_a_host, const void* plan_b_host) {
    PlanView a, b;
    if (plan_host_view(plan_a_host, &a) != XA_OK || plan_host_view(plan_b_host, &b) != XA_OK) return 0;
    return pair_layout(a.h, b.h).total;
}

extern "C" xa_status xa_match_pair(const void* plan_a_host, const void* plan_a_dev, const uint8_t* d_a,
                                   const void* plan_b_host, const void* plan_b_dev, const uint8_t* d_b,
                                   const int8_t* d_pattern, int32_t ratio_num, int32_t ratio_den,
                                   const xa_pair_buffers* out, void* d_ws, size_t ws_bytes, hipStream_t stream) {
    PlanView ha, hb;
    xa_status s = plan_host_view(plan_a_host, &ha);
    if (s != XA_OK) return s;
    s = plan_host_view(plan_b_host, &hb);
    if (s != XA_OK) return s;
    if (ha.h->n_features != hb.h->n_features) return fail(XA_EINVAL, "plans disagree on n_features");
    if (!plan_a_dev || !plan_b_dev || !d_a || !d_b || !d_pattern || !out) return fail(XA_EINVAL, "NULL pointer");
    if (!out->kp_a || !out->desc_a || !out->count_a || !out->kp_b || !out->desc_b || !out->count_b || !out->matches ||
        !out->pair_count || !out->best)
        return fail(XA_EINVAL, "NULL output buffer");
    if (ratio_num < 0 || ratio_den < 1 || ratio_num > (1 << 20) || ratio_den > (1 << 20))
        return fail(XA_EINVAL, "bad ratio");
    const PairWs w = pair_layout(ha.h, hb.h);
    if (ws_bytes < w.total) return fail(XA_ECAPACITY, "pair workspace needs %zu bytes, got %zu", w.total, ws_bytes);
    if (!d_ws || reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(XA_EINVAL, "workspace must be 256-byte aligned");
    uint8_t* ws = static_cast<uint8_t*>(d_ws);
    const PlanView da = plan_dev_view(plan_a_host, plan_a_dev), db = plan_dev_view(plan_b_host, plan_b_dev);
    s = launch_simulate(ha, da, d_a, ws + w.arena_a, ws + w.mask_a, nullptr,
                        reinterpret_cast<float*>(ws + w.sim_a), stream);
    if (s != XA_OK) return s;
    s = launch_simulate(hb, db, d_b, ws + w.arena_b, ws + w.mask_b, nullptr,
                        reinterpret_cast<float*>(ws + w.sim_b), stream);
    if (s != XA_OK) return s;
    // the first extraction's set-up launch also clears the matcher's pair counts
    s = launch_extract(ha, da, ws + w.arena_a, ws + w.mask_a, d_pattern, out->kp_a, out->desc_a, out->count_a,
                       ws + w.ext_a, stream, out->pair_count, ha.h->n_views * hb.h->n_views);
    if (s != XA_OK) return s;
    s = launch_extract(hb, db, ws + w.arena_b, ws + w.mask_b, d_pattern, out->kp_b, out->desc_b, out->count_b,
                       ws + w.ext_b, stream);
    if (s != XA_OK) return s;
    s = launch_match(out->desc_a, out->count_a, ha.h->n_views, out->desc_b, out->count_b, hb.h->n_views,
                     ha.h->n_features, ratio_num, ratio_den, out->matches, out->pair_count, out->best, stream, true);
    return s == XA_OK ? ok() : s;
}

// ------------------------------------------------------------------ batches

namespace xa {
namespace {

struct BatchWs {
    size_t scale, arena, mask, sim, ext, total;
};

// Scale-stage scratch, then one region per chunk buffer, each sized for the largest chunk:
// the chunks run one after another and reuse it.
BatchWs batch_layout(const void* splan_host, const PlanView* ph, int n_chunks) {
    size_t arena = 0, sim = 0, ext = 0;
    for (int c = 0; c < n_chunks; ++c) {
        arena = std::max(arena, size_t(ph[c].h->arena_bytes));
        sim = std::max(sim, simulate_ws_bytes(ph[c].h));
        ext = std::max(ext, extract_ws_layout(ph[c].h).total);
    }
    BatchWs w{};
    size_t o = 0;
    w.scale = o; o = align_up(o + (splan_host ? xa_scale_workspace_size(splan_host) : 0));
    w.arena = o; o = align_up(o + arena);
    w.mask = o;  o = align_up(o + arena);
    w.sim = o;   o = align_up(o + sim);
    w.ext = o;   o = align_up(o + ext);
    w.total = o;
    return w;
}

struct BatchArgs {
    const void *splan_host, *splan_dev;
    int n_chunks;
    const void* const* vplan_hosts;
    const void* const* vplan_devs;
    const void *mplan_host, *mplan_dev;
    uint8_t* sources;
    const int8_t* pattern;
    int32_t num, den;
    xa_batch_buffers out;
    uint8_t* ws;
    size_t ws_bytes;
};

xa_status chunk_views(int n_chunks, const void* const* hosts, std::vector<PlanView>* ph) {
    if (n_chunks < 1 || n_chunks > (1 << 20) || !hosts) return fail(XA_EINVAL, "need at least one view plan");
    ph->resize(n_chunks);
    for (int c = 0; c < n_chunks; ++c) {
        const xa_status s = plan_host_view(hosts[c], &(*ph)[c]);
        if (s != XA_OK) return s;
        if ((*ph)[c].h->n_features != (*ph)[0].h->n_features)
            return fail(XA_EINVAL, "view plans %d and 0 disagree on n_features", c);
    }
    return XA_OK;
}

xa_status batch_check(const BatchArgs& a, std::vector<PlanView>* ph, BatchWs* w) {
    if (a.splan_host && !is_scale_plan(a.splan_host)) return fail(XA_EINVAL, "not a scale plan");
    if (a.splan_host && !a.splan_dev) return fail(XA_EINVAL, "scale plan without a device copy");
    xa_status s = chunk_views(a.n_chunks, a.vplan_hosts, ph);
    if (s != XA_OK) return s;
    if (!a.vplan_devs) return fail(XA_EINVAL, "NULL device plan array");
    long long views = 0;
    for (int c = 0; c < a.n_chunks; ++c) {
        if (!a.vplan_devs[c]) return fail(XA_EINVAL, "view plan %d has no device copy", c);
        views += (*ph)[c].h->n_views;
    }
    if (views > INT32_MAX) return fail(XA_EUNSUPPORTED, "too many views");
    MatchPlanView mv;
    s = match_plan_view(a.mplan_host, &mv);
    if (s != XA_OK) return s;
    if (mv.h->n_features != (*ph)[0].h->n_features)
        return fail(XA_EINVAL, "view and match plans disagree on n_features");
    if (mv.h->views_needed > views)
        return fail(XA_EINVAL, "match plan reads %d views, the view plans hold %lld", mv.h->views_needed, views);
    if (!a.mplan_dev || !a.sources || !a.pattern) return fail(XA_EINVAL, "NULL pointer");
    const xa_batch_buffers& o = a.out;
    if (!o.kp || !o.desc || !o.count || !o.matches || !o.pair_count || !o.best)
        return fail(XA_EINVAL, "NULL output buffer");
    if (a.num < 0 || a.den < 1 || a.num > (1 << 20) || a.den > (1 << 20)) return fail(XA_EINVAL, "bad ratio");
    *w = batch_layout(a.splan_host, ph->data(), a.n_chunks);
    if (a.ws_bytes < w->total) return fail(XA_ECAPACITY, "batch workspace needs %zu bytes, got %zu", w->total, a.ws_bytes);
    if (!a.ws || reinterpret_cast<uintptr_t>(a.ws) % kAlign) return fail(XA_EINVAL, "workspace must be 256-byte aligned");
    return XA_OK;
}

xa_status batch_launch(const BatchArgs& a, const std::vector<PlanView>& ph, const BatchWs& w, hipStream_t st) {
    xa_status s = XA_OK;
    if (a.splan_host) s = launch_scale(a.splan_host, a.splan_dev, a.sources, nullptr, a.ws + w.scale, st);
    if (s != XA_OK) return s;
    const size_t N = size_t(ph[0].h->n_features);
    const int n_pairs = int(static_cast<const MatchPlanHeader*>(a.mplan_host)->total_pairs);
    size_t v0 = 0;
    for (int c = 0; c < a.n_chunks; ++c) {
        const PlanView pd = plan_dev_view(a.vplan_hosts[c], a.vplan_devs[c]);
        s = launch_simulate(ph[c], pd, a.sources, a.ws + w.arena, a.ws + w.mask, nullptr,
                            reinterpret_cast<float*>(a.ws + w.sim), st);
        if (s != XA_OK) return s;
        // the first chunk's extraction set-up also clears the matcher's pair counts
        s = launch_extract(ph[c], pd, a.ws + w.arena, a.ws + w.mask, a.pattern, a.out.kp + v0 * N,
                           a.out.desc + v0 * N * 32, a.out.count + v0, a.ws + w.ext, st,
                           c == 0 ? a.out.pair_count : nullptr, c == 0 ? n_pairs : 0);
        if (s != XA_OK) return s;
        v0 += size_t(ph[c].h->n_views);
    }
    return launch_match_plan(a.mplan_host, a.mplan_dev, a.out.desc, a.out.count, a.num, a.den, a.out.matches,
                             a.out.pair_count, a.out.best, st, true);
}

}  // namespace
}  // namespace xa

struct xa_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" size_t xa_match_batch_workspace_size(const void* splan_host, int32_t n_chunks,
                                                const void* const* vplan_hosts) {
    std::vector<PlanView> ph;
    if (chunk_views(n_chunks, vplan_hosts, &ph) != XA_OK) return 0;
    if (splan_host && !is_scale_plan(splan_host)) return 0;
    return batch_layout(splan_host, ph.data(), n_chunks).total;
}

extern "C" xa_status xa_match_batch(const void* splan_host, const void* splan_dev, int32_t n_chunks,
                                    const void* const* vplan_hosts, const void* const* vplan_devs,
                                    const void* mplan_host, const void* mplan_dev, uint8_t* d_sources,
                                    const int8_t* d_pattern, int32_t ratio_num, int32_t ratio_den,
                                    const xa_batch_buffers* out, void* d_ws, size_t ws_bytes, hipStream_t stream) {
    if (!out) return fail(XA_EINVAL, "NULL output buffers");
    const BatchArgs a{splan_host, splan_dev, n_chunks, vplan_hosts, vplan_devs, mplan_host, mplan_dev, d_sources,
                      d_pattern, ratio_num, ratio_den, *out, static_cast<uint8_t*>(d_ws), ws_bytes};
    std::vector<PlanView> ph;
    BatchWs w;
    xa_status s = batch_check(a, &ph, &w);
    if (s != XA_OK) return s;
    s = batch_launch(a, ph, w, stream);
    return s == XA_OK ? ok() : s;
}

extern "C" xa_status xa_match_batch_capture(const void* splan_host, const void* splan_dev, int32_t n_chunks,
                                            const void* const* vplan_hosts, const void* const* vplan_devs,
                                            const void* mplan_host, const void* mplan_dev, uint8_t* d_sources,
                                            const int8_t* d_pattern, int32_t ratio_num, int32_t ratio_den,
                                            const xa_batch_buffers* out, void* d_ws, size_t ws_bytes,
                                            xa_graph** graph) {
    if (!out || !graph) return fail(XA_EINVAL, "NULL pointer");
    *graph = nullptr;
    const BatchArgs a{splan_host, splan_dev, n_chunks, vplan_hosts, vplan_devs, mplan_host, mplan_dev, d_sources,
                      d_pattern, ratio_num, ratio_den, *out, static_cast<uint8_t*>(d_ws), ws_bytes};
    std::vector<PlanView> ph;
    BatchWs w;
    xa_status s = batch_check(a, &ph, &w);
    if (s != XA_OK) return s;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    auto* g = new (std::nothrow) xa_graph;
    if (!g) {
        hipStreamDestroy(cs);
        return fail(XA_EHIP, "out of host memory");
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        s = batch_launch(a, ph, w, cs);
        hipGraph_t graph_obj = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph_obj);
        g->graph = graph_obj;
        if (s == XA_OK && e2 != hipSuccess) s = hip_fail(e2, "end capture");
        if (s == XA_OK) {
            const hipError_t e3 = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
            if (e3 != hipSuccess) s = hip_fail(e3, "graph instantiate");
        }
    } else {
        s = hip_fail(e, "begin capture");
    }
    hipStreamDestroy(cs);
    if (s != XA_OK) {
        if (g->exec) hipGraphExecDestroy(g->exec);
        if (g->graph) hipGraphDestroy(g->graph);
        delete g;
        return s;
    }
    *graph = g;
    return ok();
}

extern "C" xa_status xa_graph_launch(xa_graph* graph, hipStream_t stream) {
    if (!graph || !graph->exec) return fail(XA_EINVAL, "NULL graph");
    const hipError_t e = hipGraphLaunch(graph->exec, stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return ok();
}

extern "C" xa_status xa_graph_destroy(xa_graph* graph) {
    if (!graph) return ok();
    if (graph->exec) hipGraphExecDestroy(graph->exec);
    if (graph->graph) hipGraphDestroy(graph->graph);
    delete graph;
    return ok();
}

extern "C" xa_status xa_check(hipStream_t stream) {
    // a sticky error left by an earlier asynchronous failure (cleared once reported)
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pending HIP error");
    // the stream's own state: finished, still running, or failed
    e = hipStreamQuery(stream);
    if (e != hipSuccess && e != hipErrorNotReady) return hip_fail(e, "stream");
    return ok();
}
