// Internal declarations shared by the library's translation units.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "xaffine.h"

namespace xa {

// Tile shapes of the launch geometry (the plan's prefix tables are counted in these tiles).
constexpr int kWarpThreads = 256;           // warp: 256 threads per output tile
constexpr int kWarpRows = 2;                // view pixels per warp thread (tiles hold kWarpRows * 256 pixels)
constexpr int kWarpLds = 8192;              // floats of source footprint a warp tile can stage in LDS
constexpr int kPyrTX = 256, kPyrTY = 4;     // pyramid down-sampling (4 output pixels per thread)
constexpr int kFastTX = 64, kFastTY = 32;   // FAST / NMS / smoothing / Harris tiles (256 threads, 8 rows each)
constexpr int kBlurTX = 64, kBlurTY = 16;   // directional blur over the source (4 rows per thread)
constexpr int kBlurStride = 128;            // LDS row stride (floats) of a major-x blur tile
constexpr int kBlurLdsMax = 16384;          // floats of source a blur tile may stage in LDS (64 KiB)

// Warp tile width for a view: the output tile is w x (512 / w), narrow along the compressed
// axis so that its source footprint stays compact.
inline int warp_tile_w(double t, double s) {
    const double c = t / s;
    return c < 2.0 ? 16 : (c < 8.0 ? 8 : 4);
}
constexpr int kBorder = 22;                 // detection border (rotated BRIEF tests reach 21 px)
constexpr size_t kAlign = 256;

struct BlurTap {
    float wa;       // w (1 - f): weight of the sample at the whole-pixel minor offset
    float wb;       // w f: weight of the next row / column (f = k m - floor(k m))
    int32_t dmaj;   // step along the major axis (k)
    int32_t dmin;   // floor(k m): whole-pixel step along the minor axis
};
static_assert(sizeof(BlurTap) == 16, "tap layout");
static_assert(sizeof(xa_view_desc) == 248, "view desc layout");
static_assert(sizeof(xa_source_desc) == 32, "source desc layout");
static_assert(sizeof(xa_level_desc) == 56, "level desc layout");
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
};
xa_status plan_host_view(const void* blob, PlanView* out);
PlanView plan_dev_view(const void* blob_host, const void* blob_dev);

// Workspace layouts.
struct ExtractWs {
    size_t smooth, cand, cand_count, harris, stage, stage_count, total;
};
ExtractWs extract_ws_layout(const xa_plan_header* h);
size_t simulate_ws_bytes(const xa_plan_header* h);

// Stage launchers (device work only, arguments already validated).
xa_status launch_simulate(const PlanView& ph, const PlanView& pd, const uint8_t* sources,
                          uint8_t* arena, uint8_t* mask, float* values, float* blurred, hipStream_t st);
xa_status launch_extract(const PlanView& ph, const PlanView& pd, uint8_t* arena, uint8_t* mask,
                         const int8_t* pattern, xa_keypoint* kp, uint8_t* desc, int32_t* count,
                         uint8_t* ws, hipStream_t st);
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
xa_status launch_match_plan(const void* mplan_host, const void* mplan_dev, const uint8_t* desc, const int32_t* count,
                            int32_t num, int32_t den, xa_match* matches, int32_t* pair_count, int32_t* best,
                            hipStream_t st);
xa_status launch_match(const uint8_t* desc_a, const int32_t* count_a, int32_t n_a,
                       const uint8_t* desc_b, const int32_t* count_b, int32_t n_b, int32_t n_features,
                       int32_t num, int32_t den, xa_match* matches, int32_t* pair_count, int32_t* best,
                       hipStream_t st);

}  // namespace xa
