// Host-side planning: the sampling grid of Sec. III.B, the view maps of eq. (2),
// anti-alias taps, pyramid levels, keypoint quotas and the arena / tile layout.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace xa {

// Warp tile widths per compression class (set by the caller, e.g. from xa_tune_warp_tiles; 0 =
// the built-in rule), and a per-thread override the tuner plans with.
static std::mutex g_tiles_mu;
static int32_t g_warp_tiles[XA_WARP_CLASSES] = {};
static thread_local const int32_t* t_tile_override = nullptr;

int warp_class(double t, double s) {
    const double c = t / s;
    const int k = int(std::floor(2.0 * std::log2(std::max(c, 1.0)) + 1e-9));
    return std::min(std::max(k, 0), XA_WARP_CLASSES - 1);
}

int planned_warp_tile_w(double t, double s) {
    const int k = warp_class(t, s);
    if (t_tile_override && t_tile_override[k] > 0) return t_tile_override[k];
    std::lock_guard<std::mutex> lock(g_tiles_mu);
    return g_warp_tiles[k] > 0 ? g_warp_tiles[k] : warp_tile_w(t, s);
}

void set_tile_override(const int32_t* widths) { t_tile_override = widths; }

static int32_t g_blur_rows[XA_WARP_CLASSES] = {};
static thread_local const int32_t* t_rows_override = nullptr;

int planned_blur_rows(double t, double s) {
    const int k = warp_class(t, s);
    if (t_rows_override && t_rows_override[k] > 0) return t_rows_override[k];
    std::lock_guard<std::mutex> lock(g_tiles_mu);
    return g_blur_rows[k] > 0 ? g_blur_rows[k] : kBlurRowsDefault;
}

void set_blur_rows_override(const int32_t* rows) { t_rows_override = rows; }

bool valid_warp_tile_w(int32_t w) { return w == 4 || w == 8 || w == 16 || w == 32 || w == 64; }

static thread_local std::string g_error;

xa_status fail(xa_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

xa_status ok() {
    g_error.clear();
    return XA_OK;
}

xa_status plan_host_view(const void* blob, PlanView* out) {
    if (!blob) return fail(XA_EINVAL, "plan is NULL");
    const auto* h = static_cast<const xa_plan_header*>(blob);
    if (h->magic != XA_PLAN_MAGIC || h->version != XA_PLAN_VERSION)
        return fail(XA_EINVAL, "not an xaffine plan (magic %08x version %u)", h->magic, h->version);
    const char* b = static_cast<const char*>(blob);
    out->h = h;
    out->views = reinterpret_cast<const xa_view_desc*>(b + h->off_views);
    out->levels = reinterpret_cast<const xa_level_desc*>(b + h->off_levels);
    out->taps = reinterpret_cast<const BlurTap*>(b + h->off_taps);
    out->blur_views = reinterpret_cast<const int32_t*>(b + h->off_blur_views);
    out->warp_prefix = reinterpret_cast<const int32_t*>(b + h->off_warp_prefix);
    out->level_prefix = reinterpret_cast<const int32_t*>(b + h->off_level_prefix);
    out->vl_prefix = reinterpret_cast<const int32_t*>(b + h->off_vl_prefix);
    out->blur_prefix = reinterpret_cast<const int32_t*>(b + h->off_blur_prefix);
    out->sources = reinterpret_cast<const xa_source_desc*>(b + h->off_sources);
    out->fast_flags = reinterpret_cast<const uint8_t*>(b + h->off_fast_flags);
    return XA_OK;
}

PlanView plan_dev_view(const void* blob_host, const void* blob_dev) {
    const auto* h = static_cast<const xa_plan_header*>(blob_host);
    const char* b = static_cast<const char*>(blob_dev);
    PlanView p;
    p.h = reinterpret_cast<const xa_plan_header*>(b);
    p.views = reinterpret_cast<const xa_view_desc*>(b + h->off_views);
    p.levels = reinterpret_cast<const xa_level_desc*>(b + h->off_levels);
    p.taps = reinterpret_cast<const BlurTap*>(b + h->off_taps);
    p.blur_views = reinterpret_cast<const int32_t*>(b + h->off_blur_views);
    p.warp_prefix = reinterpret_cast<const int32_t*>(b + h->off_warp_prefix);
    p.level_prefix = reinterpret_cast<const int32_t*>(b + h->off_level_prefix);
    p.vl_prefix = reinterpret_cast<const int32_t*>(b + h->off_vl_prefix);
    p.blur_prefix = reinterpret_cast<const int32_t*>(b + h->off_blur_prefix);
    p.sources = reinterpret_cast<const xa_source_desc*>(b + h->off_sources);
    p.fast_flags = reinterpret_cast<const uint8_t*>(b + h->off_fast_flags);
    return p;
}

ExtractWs extract_ws_layout(const xa_plan_header* h) {
    ExtractWs w{};
    const size_t nvl = size_t(h->n_views) * h->n_levels;
    size_t o = 0;
    w.smooth = o;      o = align_up(o + size_t(h->arena_bytes));
    w.cand = o;        o = align_up(o + size_t(h->cand_total) * sizeof(Cand));
    w.cand_count = o;  o = align_up(o + nvl * 4);
    w.harris = o;
    w.stage = o;       o = align_up(o + size_t(h->n_views) * h->n_features * 16);
    w.stage_count = o; o = align_up(o + nvl * 4);
    w.steer = o;       o = align_up(o + size_t(kOrientBins) * kBriefTests * 4);
    w.total = o;
    return w;
}

size_t simulate_ws_bytes(const xa_plan_header* h) { return align_up(size_t(h->blur_floats) * 4); }

}  // namespace xa

using namespace xa;

extern "C" const char* xa_last_error(void) { return g_error.c_str(); }

extern "C" const char* xa_version(void) { return "xaffine 1.0 (gfx950)"; }

static double tilt_of(int i) {
    // sqrt(2)^i, exact for even i so that the longitude-count test is decided exactly on its boundary
    return std::ldexp(1.0, i / 2) * ((i & 1) ? std::sqrt(2.0) : 1.0);
}

extern "C" xa_status xa_sampling_grid(int32_t n_tilt, double b_deg, xa_affine_params* out, int32_t cap,
                                      int32_t* n_out) {
    return xa_sampling_grid_scaled(n_tilt, b_deg, 0.0, out, cap, n_out);
}

extern "C" xa_status xa_sampling_grid_scaled(int32_t n_tilt, double b_deg, double delta_s, xa_affine_params* out,
                                             int32_t cap, int32_t* n_out) {
    if (n_tilt < 0 || n_tilt > 20) return fail(XA_EINVAL, "n_tilt %d out of range [0, 20]", n_tilt);
    if (!(delta_s >= 0.0) || !std::isfinite(delta_s)) return fail(XA_EINVAL, "delta_s must be >= 0");
    if (!(b_deg > 0.0) || !std::isfinite(b_deg)) return fail(XA_EINVAL, "longitude step must be > 0");
    if (!n_out || cap < 0 || (cap > 0 && !out)) return fail(XA_EINVAL, "bad output arguments");
    int32_t n = 0;
    for (int i = 0; i <= n_tilt; ++i) {
        const double t = tilt_of(i);
        for (int k = 0; double(k) * b_deg < 180.0 * t; ++k) {
            if (n < cap) {
                const double deg = double(k) * b_deg / t;
                out[n] = xa_affine_params{t, deg * (M_PI / 180.0), 0.0, 1.0 + double(i) * delta_s, 0.0, 0.0};
            }
            ++n;
        }
    }
    *n_out = n;
    if (n > cap) return fail(XA_ECAPACITY, "grid has %d views, capacity %d", n, cap);
    return ok();
}

namespace {

struct Mat2 {
    double a, b, c, d;  // [[a, b], [c, d]]
};
Mat2 mul(const Mat2& x, const Mat2& y) {
    return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}
Mat2 rot(double a) {
    const double c = std::cos(a), s = std::sin(a);
    return {c, -s, s, c};
}

struct Planned {
    xa_view_desc v;
    std::vector<BlurTap> taps;
};

// Residue mod 64 of the row stride (floats) of the warp's LDS source tile for a view.  A wave
// reads tap (j, i) of its 64 pixels at base_l + j ls + i, two dwords per lane (i, i + 1); every
// tap's pattern over the banks is the same up to a shift, so one read of the wave's base
// addresses stands for all of them.  The LDS serves a wave in two halves of 32 lanes over 32
// banks of 4 bytes, so a read costs, per half, the most distinct dwords one bank serves (at
// least 2 for 64 dwords); the residue with the least cost summed over the halves, waves and
// pixel rows of two interior sample tiles wins, the smallest on ties.  (This model matched the
// measured change of the LDS cycles, where one pass over 64 banks underestimated them.)  The tile
// footprint and the stride follow the kernel: ls = w + ((mod - w) & 63) for the footprint width
// w (16-byte chunks), or w | 1 where that would not fit the LDS stage.
int warp_ls_mod(const xa_view_desc& v) {
    if (v.interp != XA_INTERP_LANCZOS4) return 1;
    const int tw = v.warp_tile_w, th = kWarpRows * kWarpThreads / tw;
    const int W = v.src_w, H = v.src_h;
    const int tiles_x = (v.width + tw - 1) / tw, tiles_y = (v.height + th - 1) / th;
    struct Sample {
        int width, bh;
        std::vector<int> rr, cc;   // per wave-row group of 64 lanes: row and column offsets, -1 = unused lane
    };
    std::vector<Sample> samples;
    const int picks[2][2] = {{tiles_x / 3, tiles_y / 3}, {(2 * tiles_x) / 3, (2 * tiles_y) / 3}};
    for (const auto& pk : picks) {
        const int x0 = pk[0] * tw, y0 = pk[1] * th;
        const double* m = v.inv;
        const double ox = m[0] * (tw - 1), oy = m[1] * (th - 1), o2x = m[3] * (tw - 1), o2y = m[4] * (th - 1);
        const double cx0 = m[0] * x0 + m[1] * y0 + m[2], cy0 = m[3] * x0 + m[4] * y0 + m[5];
        const double pxl = cx0 + std::min(ox, 0.0) + std::min(oy, 0.0), pxh = cx0 + std::max(ox, 0.0) + std::max(oy, 0.0);
        const double pyl = cy0 + std::min(o2x, 0.0) + std::min(o2y, 0.0), pyh = cy0 + std::max(o2x, 0.0) + std::max(o2y, 0.0);
        const int bx0 = std::max(int(std::fmax(std::floor(pxl - 1e-6), -1e9)) - 3, 0);
        const int bx1 = std::min(int(std::fmin(std::floor(pxh + 1e-6), 1e9)) + 4, W - 1);
        const int by0 = std::max(int(std::fmax(std::floor(pyl - 1e-6), -1e9)) - 3, 0);
        const int by1 = std::min(int(std::fmin(std::floor(pyh + 1e-6), 1e9)) + 4, H - 1);
        if (bx1 < bx0 || by1 < by0) continue;
        const int ax0 = bx0 & ~3;
        Sample sm;
        sm.width = (((bx1 - ax0) >> 2) + 1) * 4;
        sm.bh = by1 - by0 + 1;
        for (int t = 0; t < kWarpThreads; ++t)
            for (int k = 0; k < kWarpRows; ++k) {
                const int qx = x0 + t % tw, qy = y0 + t / tw + k * (kWarpThreads / tw);
                const double px = m[0] * qx + m[1] * qy + m[2], py = m[3] * qx + m[4] * qy + m[5];
                const bool ok = qx < v.width && qy < v.height && px >= -0.5 && px <= W - 0.5 && py >= -0.5 &&
                                py <= H - 0.5;
                sm.rr.push_back(ok ? int(std::floor(py)) - 3 - by0 : -1);
                sm.cc.push_back(ok ? int(std::floor(px)) - 3 - ax0 : 0);
            }
        samples.push_back(std::move(sm));
    }
    if (samples.empty()) return 1;
    int best_mod = 1;
    long best = -1;
    // dwords already counted in the current read: a flag per footprint float (reads of border
    // pixels start up to 3 rows and columns before the staged box: offset into range)
    std::vector<uint8_t> seen(size_t(kWarpLds) * 2 + 4096, 0);
    std::vector<int> touched;
    touched.reserve(128);
    for (int mod = 0; mod < 64; ++mod) {
        long cost = 0;
        for (const Sample& sm : samples) {
            int ls = sm.width + ((mod - sm.width) & 63);
            if (int64_t(ls) * sm.bh > kWarpLds) ls = sm.width | 1;
            // lanes of one wave and pixel row: entries (wave * 64 + lane) * kWarpRows + k
            for (int wv = 0; wv < kWarpThreads / 64; ++wv)
                for (int k = 0; k < kWarpRows; ++k)
                    for (int half = 0; half < 2; ++half) {
                        int count[32] = {0};
                        int worst = 2;
                        for (int lane = 32 * half; lane < 32 * half + 32; ++lane) {
                            const size_t e = size_t(wv * 64 + lane) * kWarpRows + k;
                            if (sm.rr[e] < 0) continue;
                            const int a = sm.rr[e] * ls + sm.cc[e];
                            for (int d = 0; d < 2; ++d) {
                                const long slot = long(a + d) + 2048;
                                if (slot < 0 || slot >= long(seen.size()) || seen[size_t(slot)]) continue;
                                seen[size_t(slot)] = 1;
                                touched.push_back(int(slot));
                                worst = std::max(worst, ++count[(a + d) & 31]);
                            }
                        }
                        for (int sl : touched) seen[size_t(sl)] = 0;
                        touched.clear();
                        cost += worst;
                    }
        }
        if (best < 0 || cost < best) {
            best = cost;
            best_mod = mod;
        }
    }
    return best_mod;
}

Planned plan_one(const xa_source_desc& src, int32_t source, const xa_affine_params& p) {
    Planned out{};
    xa_view_desc& v = out.v;
    const int32_t W = src.width, H = src.height;
    v.p = p;
    v.source = source;
    v.src_w = W;
    v.src_h = H;
    v.src_pitch = src.pitch;
    v.src_offset = src.offset;
    v.src_scale = src.scale;
    // L = s R(psi) diag(1/t, 1) R(phi): R(phi) turns the longitude onto x, the tilt compresses x.
    Mat2 L = mul(mul(rot(p.psi), Mat2{1.0 / p.t, 0.0, 0.0, 1.0}), rot(p.phi));
    L = {L.a * p.s, L.b * p.s, L.c * p.s, L.d * p.s};
    const double cx[4] = {-0.5, W - 0.5, -0.5, W - 0.5};
    const double cy[4] = {-0.5, -0.5, H - 0.5, H - 0.5};
    double lox = 1e300, loy = 1e300, hix = -1e300, hiy = -1e300;
    for (int i = 0; i < 4; ++i) {
        const double x = L.a * cx[i] + L.b * cy[i];
        const double y = L.c * cx[i] + L.d * cy[i];
        lox = std::min(lox, x); hix = std::max(hix, x);
        loy = std::min(loy, y); hiy = std::max(hiy, y);
    }
    v.width = int32_t(std::ceil((hix - lox) - 1e-9));
    v.height = int32_t(std::ceil((hiy - loy) - 1e-9));
    const double tx = -lox - 0.5 + p.tx, ty = -loy - 0.5 + p.ty;
    const double det = L.a * L.d - L.b * L.c;
    const Mat2 Li{L.d / det, -L.b / det, -L.c / det, L.a / det};
    v.fwd[0] = L.a; v.fwd[1] = L.b; v.fwd[2] = tx;
    v.fwd[3] = L.c; v.fwd[4] = L.d; v.fwd[5] = ty;
    v.inv[0] = Li.a; v.inv[1] = Li.b; v.inv[2] = -(Li.a * tx + Li.b * ty);
    v.inv[3] = Li.c; v.inv[4] = Li.d; v.inv[5] = -(Li.c * tx + Li.d * ty);
    // anti-alias for the net compression t/s along u (0.8 sqrt(t^2 - 1) for s = 1)
    const double r = p.t / p.s;
    v.sigma = r > 1.0 ? 0.8 * std::sqrt(r * r - 1.0) : 0.0;
    v.ux = std::cos(p.phi);
    v.uy = -std::sin(p.phi);
    v.blur_offset = -1;
    if (v.sigma > 0.0) {
        // Sheared-line Gaussian: taps step one pixel along the major axis and m along the other.
        double m;
        if (std::fabs(v.ux) >= std::fabs(v.uy)) { v.blur_major = 0; m = v.uy / v.ux; }
        else { v.blur_major = 1; m = v.ux / v.uy; }
        const double sstep = v.sigma / std::sqrt(1.0 + m * m);
        const int K = int(std::ceil(4.0 * sstep));
        std::vector<double> g(2 * K + 1);
        double sum = 0.0;
        for (int k = -K; k <= K; ++k) {
            g[k + K] = std::exp(-double(k) * double(k) / (2.0 * sstep * sstep));
            sum += g[k + K];
        }
        for (int k = -K; k <= K; ++k) {
            const double km = double(k) * m;
            const double fl = std::floor(km);
            const double w = g[k + K] / sum, f = km - fl;
            out.taps.push_back(BlurTap{float(w * (1.0 - f)), float(w * f), k, int32_t(fl)});
        }
        v.blur_ntaps = 2 * K + 1;
        // zero taps up to a multiple of 4 (the kernel reads taps in groups of 4)
        while (out.taps.size() % 4) out.taps.push_back(BlurTap{0.0f, 0.0f, 0, 0});
    }
    return out;
}

}  // namespace

extern "C" xa_status xa_plan_views(const xa_source_desc* sources, int32_t n_sources, const int32_t* view_source,
                                   const xa_affine_params* params, int32_t n_views, int32_t n_levels, double level_scale,
                                   int32_t n_features, int32_t fast_threshold, void* blob, size_t blob_cap,
                                   size_t* blob_bytes) {
    if (!blob_bytes) return fail(XA_EINVAL, "blob_bytes is NULL");
    if (n_sources < 1 || !sources) return fail(XA_EINVAL, "need at least one source");
    for (int i = 0; i < n_sources; ++i) {
        const xa_source_desc& sd = sources[i];
        if (sd.width < 1 || sd.height < 1 || sd.width > 32768 || sd.height > 32768)
            return fail(XA_EINVAL, "source %d size %dx%d out of range [1, 32768]", i, sd.width, sd.height);
        if (sd.pitch < sd.width || sd.offset < 0) return fail(XA_EINVAL, "source %d: pitch < width or offset < 0", i);
        if (!(sd.scale > 0.0) || !std::isfinite(sd.scale)) return fail(XA_EINVAL, "source %d: scale must be > 0", i);
    }
    if (n_views < 1 || !params || !view_source) return fail(XA_EINVAL, "need at least one view");
    if (n_levels < 1 || n_levels > XA_MAX_LEVELS) return fail(XA_EINVAL, "n_levels %d not in [1, %d]", n_levels, XA_MAX_LEVELS);
    if (!(level_scale > 1.0) || !std::isfinite(level_scale)) return fail(XA_EINVAL, "level_scale must be > 1");
    if (n_features < 1 || n_features > XA_MAX_FEATURES)
        return fail(XA_EUNSUPPORTED, "n_features %d not in [1, %d]", n_features, XA_MAX_FEATURES);
    if (fast_threshold < 0 || fast_threshold > 255) return fail(XA_EINVAL, "fast_threshold must be in [0, 255]");
    for (int i = 0; i < n_views; ++i) {
        const xa_affine_params& p = params[i];
        if (view_source[i] < 0 || view_source[i] >= n_sources) return fail(XA_EINVAL, "view %d: bad source index", i);
        if (!(p.t >= 1.0) || !(p.s >= 1.0) || !std::isfinite(p.t) || !std::isfinite(p.s) || !std::isfinite(p.phi) ||
            !std::isfinite(p.psi) || !std::isfinite(p.tx) || !std::isfinite(p.ty))
            return fail(XA_EINVAL, "view %d: need finite parameters with t >= 1 and s >= 1 (reduce with the scale stage)", i);
    }
    // Per-level keypoint quotas, proportional to level area; level 0 takes the remainder.
    std::vector<int32_t> quota(n_levels, 0);
    {
        std::vector<double> r(n_levels);
        double tot = 0.0;
        for (int l = 0; l < n_levels; ++l) r[l] = std::pow(level_scale, double(-2 * l));
        for (int l = 0; l < n_levels; ++l) tot += r[l];
        int32_t rest = n_features;
        for (int l = 1; l < n_levels; ++l) {
            quota[l] = int32_t(std::floor(double(n_features) * r[l] / tot));
            rest -= quota[l];
        }
        quota[0] = rest;
        for (int l = 0; l < n_levels; ++l)
            if (quota[l] > XA_MAX_QUOTA)
                return fail(XA_EUNSUPPORTED, "level %d quota %d exceeds %d", l, quota[l], XA_MAX_QUOTA);
    }

    std::vector<Planned> pv(n_views);
    int64_t total_px = 0;
    for (int i = 0; i < n_views; ++i) {
        pv[i] = plan_one(sources[view_source[i]], view_source[i], params[i]);
        const auto& v = pv[i].v;
        if (v.width < 1 || v.height < 1 || v.width > 32768 || v.height > 32768)
            return fail(XA_EUNSUPPORTED, "view %d canvas %dx%d out of range", i, v.width, v.height);
        total_px += int64_t(v.width) * v.height;
        if (total_px > (int64_t(1) << 34)) return fail(XA_EUNSUPPORTED, "views exceed 2^34 pixels");
    }

    const int32_t nvl = n_views * n_levels;
    std::vector<xa_level_desc> lv(nvl);
    std::vector<BlurTap> taps;
    std::vector<int32_t> blur_views, blur_prefix;
    std::vector<int32_t> warp_prefix(n_views + 1, 0);
    std::vector<int32_t> level_prefix(size_t(n_levels) * (n_views + 1), 0);
    std::vector<int32_t> vl_prefix(nvl + 1, 0);
    std::vector<uint8_t> fast_flags;
    int64_t arena = 0, cand = 0, blur_floats = 0;
    int64_t warp_tiles = 0, vl_tiles = 0, blur_tiles = 0;
    std::vector<int64_t> lvl_tiles(n_levels, 0);
    std::map<std::array<double, 5>, int> ls_cache;
    for (int i = 0; i < n_views; ++i) {
        xa_view_desc& v = pv[i].v;
        if (v.sigma > 0.0) {
            v.blur_offset = blur_floats;
            blur_floats += int64_t(blur_pitch(v.src_w)) * v.src_h;
            v.blur_tap0 = int32_t(taps.size());
            taps.insert(taps.end(), pv[i].taps.begin(), pv[i].taps.end());
            blur_views.push_back(i);
            blur_prefix.push_back(int32_t(blur_tiles));
            v.blur_rows = planned_blur_rows(v.p.t, v.p.s);
            const int btw = blur_tile_w(v.blur_major, v.blur_rows), bth = blur_tile_h(v.blur_major, v.blur_rows);
            blur_tiles += int64_t((v.src_w + btw - 1) / btw) * ((v.src_h + bth - 1) / bth);
        }
        warp_prefix[i] = int32_t(warp_tiles);
        v.warp_tile_w = planned_warp_tile_w(v.p.t, v.p.s);
        {   // the residue depends on the view's linear map and tile width (the sources' sizes only
            // move the sample tiles): views that share them, as the grid's views of many pairs
            // do, share one search
            const std::array<double, 5> key = {v.inv[0], v.inv[1], v.inv[3], v.inv[4], double(v.warp_tile_w)};
            auto it = ls_cache.find(key);
            if (it == ls_cache.end()) it = ls_cache.emplace(key, warp_ls_mod(v)).first;
            v.warp_ls_mod = it->second;
        }
        const int th = kWarpRows * kWarpThreads / v.warp_tile_w;
        warp_tiles += int64_t((v.width + v.warp_tile_w - 1) / v.warp_tile_w) * ((v.height + th - 1) / th);
        int32_t kp_base = 0;
        for (int l = 0; l < n_levels; ++l) {
            xa_level_desc& d = lv[size_t(i) * n_levels + l];
            const double f = std::pow(level_scale, double(l));
            d.width = l == 0 ? v.width : std::max(1, int32_t(std::floor(v.width / f + 0.5)));
            d.height = l == 0 ? v.height : std::max(1, int32_t(std::floor(v.height / f + 0.5)));
            d.pitch = level_pitch(d.width);
            d.offset = arena;
            if (l == 0) { v.offset = arena; v.pitch = d.pitch; }
            arena = int64_t(align_up(size_t(arena + int64_t(d.pitch) * d.height), 128));
            d.quota = quota[l];
            d.kp_base = kp_base;
            kp_base += quota[l];
            d.view = i;
            d.level = l;
            d.cand_offset = cand;
            const bool detect = d.width > 2 * kBorder && d.height > 2 * kBorder;
            d.cand_cap = detect ? int64_t((d.width + 1) / 2) * ((d.height + 1) / 2) : 0;
            cand += d.cand_cap;
            level_prefix[size_t(l) * (n_views + 1) + i] = int32_t(lvl_tiles[l]);
            lvl_tiles[l] += int64_t((d.width + kPyrTX - 1) / kPyrTX) * ((d.height + kPyrTY - 1) / kPyrTY);
            vl_prefix[size_t(i) * n_levels + l] = int32_t(vl_tiles);
            const int ftx = (d.width + kFastTX - 1) / kFastTX, fty = (d.height + kFastTY - 1) / kFastTY;
            vl_tiles += int64_t(ftx) * fty;
            for (int ty = 0; ty < fty; ++ty)
                for (int tx = 0; tx < ftx; ++tx)
                    fast_flags.push_back(fast_tile_flags(v, d.width, d.height, l, tx * kFastTX, ty * kFastTY, kFastTX,
                                                         kFastTY, kBorder));
        }
    }
    warp_prefix[n_views] = int32_t(warp_tiles);
    for (int l = 0; l < n_levels; ++l) level_prefix[size_t(l) * (n_views + 1) + n_views] = int32_t(lvl_tiles[l]);
    vl_prefix[nvl] = int32_t(vl_tiles);
    blur_prefix.push_back(int32_t(blur_tiles));
    if (warp_tiles > INT32_MAX / 2 || vl_tiles > INT32_MAX / 2 || blur_tiles > INT32_MAX / 2)
        return fail(XA_EUNSUPPORTED, "too many tiles for one launch");

    xa_plan_header h{};
    h.magic = XA_PLAN_MAGIC;
    h.version = XA_PLAN_VERSION;
    h.src_w = sources[0].width;
    h.src_h = sources[0].height;
    h.n_views = n_views;
    h.n_levels = n_levels;
    h.n_features = n_features;
    h.fast_threshold = fast_threshold;
    h.level_scale = level_scale;
    h.arena_bytes = arena;
    h.cand_total = cand;
    h.blur_floats = blur_floats;
    h.n_blur = int32_t(blur_views.size());
    h.n_taps_total = int32_t(taps.size());
    h.n_sources = n_sources;
    size_t o = align_up(sizeof(xa_plan_header), 64);
    h.off_views = int64_t(o);        o = align_up(o + sizeof(xa_view_desc) * n_views, 64);
    h.off_levels = int64_t(o);       o = align_up(o + sizeof(xa_level_desc) * nvl, 64);
    h.off_taps = int64_t(o);         o = align_up(o + sizeof(BlurTap) * taps.size(), 64);
    h.off_blur_views = int64_t(o);   o = align_up(o + 4 * blur_views.size(), 64);
    h.off_warp_prefix = int64_t(o);  o = align_up(o + 4 * warp_prefix.size(), 64);
    h.off_level_prefix = int64_t(o); o = align_up(o + 4 * level_prefix.size(), 64);
    h.off_vl_prefix = int64_t(o);    o = align_up(o + 4 * vl_prefix.size(), 64);
    h.off_blur_prefix = int64_t(o);  o = align_up(o + 4 * blur_prefix.size(), 64);
    h.off_sources = int64_t(o);      o = align_up(o + sizeof(xa_source_desc) * n_sources, 64);
    h.off_fast_flags = int64_t(o);   o = align_up(o + fast_flags.size(), 64);
    h.total_bytes = int64_t(o);
    *blob_bytes = o;
    if (!blob) return ok();
    if (blob_cap < o) return fail(XA_ECAPACITY, "plan needs %zu bytes, buffer has %zu", o, blob_cap);
    char* b = static_cast<char*>(blob);
    std::memset(b, 0, o);
    std::memcpy(b, &h, sizeof(h));
    for (int i = 0; i < n_views; ++i)
        std::memcpy(b + h.off_views + sizeof(xa_view_desc) * i, &pv[i].v, sizeof(xa_view_desc));
    std::memcpy(b + h.off_levels, lv.data(), sizeof(xa_level_desc) * nvl);
    if (!taps.empty()) std::memcpy(b + h.off_taps, taps.data(), sizeof(BlurTap) * taps.size());
    if (!blur_views.empty()) std::memcpy(b + h.off_blur_views, blur_views.data(), 4 * blur_views.size());
    std::memcpy(b + h.off_warp_prefix, warp_prefix.data(), 4 * warp_prefix.size());
    std::memcpy(b + h.off_level_prefix, level_prefix.data(), 4 * level_prefix.size());
    std::memcpy(b + h.off_vl_prefix, vl_prefix.data(), 4 * vl_prefix.size());
    std::memcpy(b + h.off_blur_prefix, blur_prefix.data(), 4 * blur_prefix.size());
    std::memcpy(b + h.off_sources, sources, sizeof(xa_source_desc) * n_sources);
    if (!fast_flags.empty()) std::memcpy(b + h.off_fast_flags, fast_flags.data(), fast_flags.size());
    return ok();
}

extern "C" xa_status xa_plan_set_interp(void* plan_host, int32_t interp) {
    if (interp != XA_INTERP_LANCZOS4 && interp != XA_INTERP_NEAREST) return fail(XA_EINVAL, "unknown interpolation %d", interp);
    PlanView p;
    const xa_status s = plan_host_view(plan_host, &p);
    if (s != XA_OK) return s;
    auto* views = reinterpret_cast<xa_view_desc*>(static_cast<char*>(plan_host) + p.h->off_views);
    for (int i = 0; i < p.h->n_views; ++i) views[i].interp = interp;
    return ok();
}

extern "C" xa_status xa_plan_image(int32_t src_w, int32_t src_h, int32_t src_pitch, const xa_affine_params* params,
                                   int32_t n_views, int32_t n_levels, double level_scale, int32_t n_features,
                                   int32_t fast_threshold, void* blob, size_t blob_cap, size_t* blob_bytes) {
    const xa_source_desc src{src_w, src_h, src_pitch, 0, 0, 1.0};
    std::vector<int32_t> vs(n_views > 0 ? n_views : 0, 0);
    return xa_plan_views(&src, 1, vs.data(), params, n_views, n_levels, level_scale, n_features, fast_threshold, blob,
                         blob_cap, blob_bytes);
}

extern "C" xa_status xa_set_warp_tiles(const int32_t* widths) {
    if (widths)
        for (int k = 0; k < XA_WARP_CLASSES; ++k)
            if (widths[k] != 0 && !valid_warp_tile_w(widths[k]))
                return fail(XA_EINVAL, "warp tile width %d of class %d is not 0, 4, 8, 16, 32 or 64", widths[k], k);
    std::lock_guard<std::mutex> lock(g_tiles_mu);
    for (int k = 0; k < XA_WARP_CLASSES; ++k) g_warp_tiles[k] = widths ? widths[k] : 0;
    return ok();
}

extern "C" xa_status xa_get_warp_tiles(int32_t* widths) {
    if (!widths) return fail(XA_EINVAL, "NULL output");
    std::lock_guard<std::mutex> lock(g_tiles_mu);
    for (int k = 0; k < XA_WARP_CLASSES; ++k) {
        const double c = std::pow(2.0, 0.5 * k + 0.25);     // a compression inside class k
        widths[k] = g_warp_tiles[k] > 0 ? g_warp_tiles[k] : warp_tile_w(c, 1.0);
    }
    return ok();
}

extern "C" xa_status xa_set_blur_rows(const int32_t* rows) {
    if (rows)
        for (int k = 0; k < XA_WARP_CLASSES; ++k)
            if (rows[k] != 0 && !valid_blur_rows(rows[k]))
                return fail(XA_EINVAL, "blur rows %d of class %d are not 0, 4 or 8", rows[k], k);
    std::lock_guard<std::mutex> lock(g_tiles_mu);
    for (int k = 0; k < XA_WARP_CLASSES; ++k) g_blur_rows[k] = rows ? rows[k] : 0;
    return ok();
}

extern "C" xa_status xa_get_blur_rows(int32_t* rows) {
    if (!rows) return fail(XA_EINVAL, "NULL output");
    std::lock_guard<std::mutex> lock(g_tiles_mu);
    for (int k = 0; k < XA_WARP_CLASSES; ++k) rows[k] = g_blur_rows[k] > 0 ? g_blur_rows[k] : kBlurRowsDefault;
    return ok();
}
