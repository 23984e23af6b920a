// Internal declarations shared by the library's translation units.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>

#include "xaffine.h"

namespace xa {

// Tile shapes of the launch geometry (the plan's prefix tables are counted in these tiles).
constexpr int kWarpThreads = 256;           // warp: 256 threads per output tile
constexpr int kWarpRows = 2;                // view pixels per warp thread (tiles hold kWarpRows * 256 pixels)
constexpr int kWarpLds = 8192;              // floats of source footprint a warp tile can stage in LDS
constexpr int kPyrTX = 256, kPyrTY = 16;    // pyramid down-sampling (4 x 4 output pixels per thread)
constexpr int kFastTX = 64, kFastTY = 32;   // FAST / NMS / smoothing / Harris tiles (256 threads, 8 rows each)
constexpr int kBlurRowsDefault = 8;         // directional blur: outputs per thread across the minor axis
constexpr int kBlurTX = 64;                  // blur tile side along the taps' major axis (one wave's lanes)
constexpr int kBlurStride = 128;            // LDS row stride (floats) of a major-x blur tile
constexpr int kBlurLdsMax = 16384;          // floats of source a blur tile may stage in LDS (64 KiB)
// Blur tiles: 64 x 16 when the taps step along x (a wave's lanes take 64 columns of one row
// group), 16 x 64 when they step along y (a wave's lanes take 64 rows of one 4-column group, so
// each tap read hits 64 rows, one per LDS bank at the odd row stride).
// Blur tile: kBlurTX along the major axis by 4 waves x `rows` outputs across it.
__host__ __device__ inline int blur_tile_w(int major, int rows) { return major == 0 ? kBlurTX : 4 * rows; }
__host__ __device__ inline int blur_tile_h(int major, int rows) { return major == 0 ? 4 * rows : kBlurTX; }

// Warp tile width for a view: the output tile is w x (512 / w), narrow along the compressed
// axis so that its source footprint stays compact.
inline int warp_tile_w(double t, double s) {
    const double c = t / s;
    return c < 2.0 ? 16 : (c < 8.0 ? 8 : 4);
}
// Warp tile width the planner uses for a view: the caller's table (xa_set_warp_tiles) or the
// tuner's per-thread override for the view's compression class, else the rule above.
int warp_class(double t, double s);
int planned_warp_tile_w(double t, double s);
void set_tile_override(const int32_t* widths);   // per thread; NULL ends the override
bool valid_warp_tile_w(int32_t w);
// Blur outputs per thread the planner uses for a view of compression class warp_class(t, s): the
// caller's table (xa_set_blur_rows) or the tuner's per-thread override, else kBlurRowsDefault.
int planned_blur_rows(double t, double s);
void set_blur_rows_override(const int32_t* rows);   // per thread; NULL ends the override
inline bool valid_blur_rows(int32_t r) { return r == 4 || r == 8; }
// The hardware deals consecutive blocks of a launch round-robin to the 8 XCDs, each with its
// own L2.  For kernels whose neighbouring tiles share cache lines (narrow warp tiles), this
// remap gives each XCD one contiguous run of tiles instead: block b, the i-th on XCD b % 8,
// takes tile start(b % 8) + i, where XCD x owns the run of n / 8 (+1 for x < n % 8) tiles
// starting at start(x).  A bijection on [0, n).
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_contiguous(int b, int n) {
    const int x = b % kXcds, i = b / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + i;
}
constexpr int kBorder = 22;                 // detection border (rotated BRIEF tests reach 21 px)
constexpr size_t kAlign = 256;

// True if no point of the level-pixel rectangle [rx0, rx1] x [ry0, ry1], taken to view level-0
// coordinates (x0 = (x + 1/2) W0 / Wl - 1/2 per axis) and grown there by m pixels per axis,
// maps through inv into the source rectangle [-1/2, W - 1/2] x [-1/2, H - 1/2].  The image
// of the grown rectangle is a parallelogram; a separating axis among the source's two axes
// and the parallelogram's two edge normals decides, in fp64 with a 1e-6 px margin.
inline __host__ __device__ bool rect_misses_source(const xa_view_desc& v, double sx, double sy, double rx0, double rx1, double ry0,
                                   double ry1, double m) {
    const double ax = (rx0 + 0.5) * sx - 0.5 - m, bx = (rx1 + 0.5) * sx - 0.5 + m;
    const double ay = (ry0 + 0.5) * sy - 0.5 - m, by = (ry1 + 0.5) * sy - 0.5 + m;
    const double* G = v.inv;
    const double qx[4] = {G[0] * ax + G[1] * ay + G[2], G[0] * bx + G[1] * ay + G[2], G[0] * bx + G[1] * by + G[2],
                          G[0] * ax + G[1] * by + G[2]};
    const double qy[4] = {G[3] * ax + G[4] * ay + G[5], G[3] * bx + G[4] * ay + G[5], G[3] * bx + G[4] * by + G[5],
                          G[3] * ax + G[4] * by + G[5]};
    const double eps = 1e-6;
    const double lo_x = -0.5, hi_x = double(v.src_w) - 0.5, lo_y = -0.5, hi_y = double(v.src_h) - 0.5;
    double mnx = qx[0], mxx = qx[0], mny = qy[0], mxy = qy[0];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        mnx = fmin(mnx, qx[k]); mxx = fmax(mxx, qx[k]);
        mny = fmin(mny, qy[k]); mxy = fmax(mxy, qy[k]);
    }
    if (mxx < lo_x - eps || mnx > hi_x + eps || mxy < lo_y - eps || mny > hi_y + eps) return true;
    const double rx[4] = {lo_x, hi_x, hi_x, lo_x}, ry[4] = {lo_y, lo_y, hi_y, hi_y};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        // normal of the edge q0 -> q1 (e = 0) or q0 -> q3 (e = 1)
        const int k = e == 0 ? 1 : 3;
        const double nx = -(qy[k] - qy[0]), ny = qx[k] - qx[0];
        const double nn = sqrt(nx * nx + ny * ny);
        if (!(nn > 0.0)) continue;
        double qmn = 1e300, qmx = -1e300, rmn = 1e300, rmx = -1e300;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double pq = nx * qx[j] + ny * qy[j], pr = nx * rx[j] + ny * ry[j];
            qmn = fmin(qmn, pq); qmx = fmax(qmx, pq);
            rmn = fmin(rmn, pr); rmx = fmax(rmx, pr);
        }
        if (rmx < qmn - eps * nn || rmn > qmx + eps * nn) return true;
    }
    return false;
}

// Distance bound (view level-0 pixels per axis) between a level-l pixel whose pyramid mask is
// set and a valid level-0 pixel: each level's mask is the AND of a 2 x 2 footprint within one
// pixel of the same point one level down, and level k pixels span at most 1.25^k level-0
// pixels, so the bound is 1 + sum_{k<l} 1.25^k.
inline __host__ __device__ double mask_reach(int l) {
    double r = 1.0, f = 1.0;
    for (int k = 0; k < l; ++k) {
        r += f;
        f *= 1.25;
    }
    return r;
}

// Flags of one FAST tile (64 x 32 pixels at (x0, y0) of a level of size W x H of view v at
// level l): bit 0 = some pixel of the tile can be valid (its smoothing can be read),
// bit 1 = some pixel can pass the content filter (all four corners of its +-B box inside the
// source).  Both bits are conservative: a pyramid-mask pixel is set only within mask_reach(l)
// view pixels of a valid level-0 pixel, and the valid region is convex.
inline __host__ __device__ uint8_t fast_tile_flags(const xa_view_desc& v, int W, int H, int l, int x0, int y0,
                                                    int tile_w, int tile_h, int border) {
    const double sxl = double(v.width) / double(W), syl = double(v.height) / double(H);
    const double reach = mask_reach(l);
    const double x1 = double((x0 + tile_w < W ? x0 + tile_w : W) - 1), y1 = double((y0 + tile_h < H ? y0 + tile_h : H) - 1);
    const bool smooth = !rect_misses_source(v, sxl, syl, x0, x1, y0, y1, reach);
    bool detect = true;
    for (int c = 0; c < 4; ++c) {
        const double ox = (c & 1) ? double(border) : -double(border), oy = (c & 2) ? double(border) : -double(border);
        detect = detect && !rect_misses_source(v, sxl, syl, x0 + ox, x1 + ox, y0 + oy, y1 + oy, reach);
    }
    return uint8_t((smooth ? 1 : 0) | (detect ? 2 : 0));
}

struct BlurTap {
    float wa;       // w (1 - f): weight of the sample at the whole-pixel minor offset
    float wb;       // w f: weight of the next row / column (f = k m - floor(k m))
    int32_t dmaj;   // step along the major axis (k)
    int32_t dmin;   // floor(k m): whole-pixel step along the minor axis
};
static_assert(sizeof(BlurTap) == 16, "tap layout");
static_assert(sizeof(xa_view_desc) == 256, "view desc layout");
static_assert(sizeof(xa_source_desc) == 32, "source desc layout");
static_assert(sizeof(xa_level_desc) == 56, "level desc layout");
static_assert(sizeof(xa_plan_header) == 168, "plan header layout");
static_assert(sizeof(xa_keypoint) == 40, "keypoint layout");
static_assert(sizeof(xa_match) == 8, "match layout");

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }
inline int32_t level_pitch(int32_t w) { return (w + 15) / 16 * 16; }
// Row pitch (floats) of a blurred source: rows start 16-byte aligned so the warp stages them in float4s.
__host__ __device__ inline int32_t blur_pitch(int32_t w) { return (w + 3) & ~3; }

// Candidate record written by the FAST kernel: raster position y * W + x and Harris response.
struct Cand {
    uint32_t raster;
    uint32_t pad;
    long long harris;
};
static_assert(sizeof(Cand) == 16, "candidate layout");

// Status helpers (plan.cpp owns the thread-local message).
xa_status fail(xa_status s, const char* fmt, ...);
xa_status ok();
xa_status hip_fail(int err, const char* what);

// Validated view of a plan blob.
struct PlanView {
    const xa_plan_header* h = nullptr;
    const xa_view_desc* views = nullptr;
    const xa_level_desc* levels = nullptr;
    const BlurTap* taps = nullptr;
    const int32_t* blur_views = nullptr;
    const int32_t* warp_prefix = nullptr;
    const int32_t* level_prefix = nullptr;
    const int32_t* vl_prefix = nullptr;
    const int32_t* blur_prefix = nullptr;
    const xa_source_desc* sources = nullptr;
    const uint8_t* fast_flags = nullptr;
};
xa_status plan_host_view(const void* blob, PlanView* out);
PlanView plan_dev_view(const void* blob_host, const void* blob_dev);

// Workspace layouts.
struct ExtractWs {
    size_t smooth, cand, cand_count, harris, stage, stage_count, steer, total;
};
constexpr int kOrientBins = 30;             // orientation bins of the steered BRIEF pattern
constexpr int kBriefTests = 256;            // binary tests per descriptor
ExtractWs extract_ws_layout(const xa_plan_header* h);
size_t simulate_ws_bytes(const xa_plan_header* h);

// Stage launchers (device work only, arguments already validated).
constexpr int kStageBlur = 1, kStageWarp = 2;   // launch_simulate stage mask
xa_status launch_simulate(const PlanView& ph, const PlanView& pd, const uint8_t* sources,
                          uint8_t* arena, uint8_t* mask, float* values, float* blurred, hipStream_t st,
                          int stages = kStageBlur | kStageWarp);
// zero_extra (nullable): n_extra int32 counters the set-up launch clears as well (the matcher's
// pair counts of a pipeline, which then skips its own clearing launch).
xa_status launch_extract(const PlanView& ph, const PlanView& pd, uint8_t* arena, uint8_t* mask,
                         const int8_t* pattern, xa_keypoint* kp, uint8_t* desc, int32_t* count,
                         uint8_t* ws, hipStream_t st, int32_t* zero_extra = nullptr, int n_extra = 0);
xa_status launch_scale(const void* splan_host, const void* splan_dev, uint8_t* d_sources, float* d_values,
                       void* d_ws, hipStream_t stream);
bool is_scale_plan(const void* blob);

constexpr uint32_t kMatchMagic = 0x5841464Du;   // "XAFM"
struct MatchPlanHeader {
    uint32_t magic;
    int32_t n_groups, n_features, q, views_needed;  // views_needed = max over groups of a0 + na, b0 + nb
    long long total_blocks, total_pairs;
    int64_t off_groups, off_prefix, total_bytes;
};
struct MatchPlanView {
    const MatchPlanHeader* h = nullptr;
};
xa_status match_plan_view(const void* blob, MatchPlanView* out);
// counts_zeroed: pair_count is already zero on the stream (no clearing launch)
xa_status launch_match_plan(const void* mplan_host, const void* mplan_dev, const uint8_t* desc, const int32_t* count,
                            int32_t num, int32_t den, xa_match* matches, int32_t* pair_count, int32_t* best,
                            hipStream_t st, bool counts_zeroed = false);
xa_status launch_match(const uint8_t* desc_a, const int32_t* count_a, int32_t n_a,
                       const uint8_t* desc_b, const int32_t* count_b, int32_t n_b, int32_t n_features,
                       int32_t num, int32_t den, xa_match* matches, int32_t* pair_count, int32_t* best,
                       hipStream_t st, bool counts_zeroed = false);

}  // namespace xa
