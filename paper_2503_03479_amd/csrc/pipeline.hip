// The whole parameter-search path for one image pair (Sec. III.B): simulate the
// views of both images, extract ORB on every view, match all view pairs and pick
// the best one, as one asynchronous sequence of launches on the caller's stream.
#include <hip/hip_runtime.h>

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
    s = launch_extract(ha, da, ws + w.arena_a, ws + w.mask_a, d_pattern, out->kp_a, out->desc_a, out->count_a,
                       ws + w.ext_a, stream);
    if (s != XA_OK) return s;
    s = launch_extract(hb, db, ws + w.arena_b, ws + w.mask_b, d_pattern, out->kp_b, out->desc_b, out->count_b,
                       ws + w.ext_b, stream);
    if (s != XA_OK) return s;
    s = launch_match(out->desc_a, out->count_a, ha.h->n_views, out->desc_b, out->count_b, hb.h->n_views,
                     ha.h->n_features, ratio_num, ratio_den, out->matches, out->pair_count, out->best, stream);
    return s == XA_OK ? ok() : s;
}
