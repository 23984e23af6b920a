/*
 * xaffine -- affine view simulation, ORB extraction and all-view-pair Hamming
 * matching on AMD Instinct MI355X (gfx950).
 *
 * The library computes the parameter-search stage of "Feature Point
 * Extraction for Extra-Affine Image" (arXiv 2503.03479, Sec. III.B): views of
 * an image are simulated over a grid of tilts t and longitudes phi (the
 * camera model of eq. (2), resampled with the Lanczos kernel of eqs. (3)-(4)
 * after an anti-alias blur along the tilt direction), ORB features are
 * extracted on every view, every view of image A is matched against every
 * view of image B with a brute-force Hamming matcher and a ratio test
 * (Sec. IV.C), and the view pair with the most matches gives the optimal
 * parameter group.
 *
 * Conventions for every entry point
 *  - Pointers named d_* are device pointers owned by the caller.  The library
 *    never allocates device memory; each call that needs scratch space takes a
 *    workspace (d_ws, ws_bytes) whose minimum size a *_workspace_size query
 *    returns.  Workspaces must be 256-byte aligned.
 *  - Device work is enqueued on `stream` and is asynchronous: outputs are valid
 *    once the stream has been synchronised.  No call synchronises the stream.
 *  - A plan is a flat, relocatable byte blob written by xa_plan_views.  Calls
 *    take it twice: plan_host (host memory, used for launch geometry) and
 *    plan_dev (a byte-for-byte device copy made by the caller, read by kernels).
 *  - Images are row-major uint8 with a row pitch in bytes.  All coordinates are
 *    pixel centres: pixel (x, y) covers [x-1/2, x+1/2] x [y-1/2, y+1/2].
 *  - Errors: every call returns an xa_status; on anything but XA_OK the outputs
 *    are undefined and xa_last_error() returns a message (thread-local, valid
 *    until the next call on the same thread).  Invalid arguments are detected
 *    on the host before anything is enqueued.  Faults inside kernels surface as
 *    XA_EHIP on a later call or on the caller's own stream synchronisation.
 *  - No C++ exception crosses this interface.
 */
#ifndef XAFFINE_H
#define XAFFINE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    XA_OK = 0,
    XA_EINVAL = -1,        /* bad argument (size, pointer, parameter range, plan magic) */
    XA_ECAPACITY = -2,     /* a caller-provided buffer or workspace is too small */
    XA_EHIP = -3,          /* the HIP runtime reported an error */
    XA_EUNSUPPORTED = -4   /* a size beyond a documented library limit */
} xa_status;

#define XA_PLAN_MAGIC 0x58414650u   /* "XAFP" */
#define XA_PLAN_VERSION 6u
#define XA_MAX_LEVELS 12
#define XA_MAX_QUOTA 2048           /* keypoints per pyramid level */
#define XA_MAX_FEATURES 4096        /* keypoints per view */
#define XA_DESC_BYTES 32            /* rBRIEF-256 */

/* One simulated camera change, eq. (2): A = T R1(psi) S T_tau R2(phi).
 * t >= 1 is the tilt (latitude theta = arccos 1/t), phi the longitude and
 * psi the spin (radians), s > 0 the scale (s > 1 magnifies), (tx, ty) a
 * translation of the content inside the view canvas (pixels). */
typedef struct {
    double t, phi, psi, s, tx, ty;
} xa_affine_params;

/* A source image inside a caller-owned sources buffer (uint8, row-major).
 * scale relates its pixel coordinates to the original image the caller
 * matches: p_original = (p + 1/2) / scale - 1/2 (1 for an original image,
 * s for the output of the scale stage at scale s). */
typedef struct {
    int32_t width, height;
    int32_t pitch;              /* bytes between rows */
    int32_t pad;
    int64_t offset;             /* byte offset of pixel (0, 0) in the sources buffer */
    double scale;
} xa_source_desc;

/* A planned view of one source.  fwd maps source to view, inv view to source,
 * both 2x3 row-major (x' = m[0] x + m[1] y + m[2], y' = m[3] x + m[4] y + m[5]).
 * The linear part is s R(psi) diag(1/t, 1) R(phi); the canvas is the bounding
 * box of the source rectangle under it.  sigma is the standard deviation (in
 * source pixels) of the anti-alias Gaussian applied along (ux, uy), the
 * source direction the map compresses: sigma = 0.8 sqrt((t/s)^2 - 1) when
 * t/s > 1, else 0. */
typedef struct {
    xa_affine_params p;
    int32_t source;             /* index into the plan's source table */
    int32_t src_w, src_h, src_pitch;
    int64_t src_offset;         /* byte offset of the source in the sources buffer */
    double src_scale;           /* source -> original coordinates, see xa_source_desc */
    int32_t width, height;      /* canvas W' x H' */
    int32_t pitch;              /* row pitch of level 0 in the arena (bytes) */
    int32_t warp_tile_w;        /* width of the warp's output tiles (tiles hold 512 pixels) */
    double fwd[6];
    double inv[6];
    double sigma;
    double ux, uy;
    int64_t offset;             /* byte offset of level 0 in the pyramid arena */
    int64_t blur_offset;        /* float offset of the blurred source in the simulate workspace, -1 if none;
                                   its rows are (src_w + 3) / 4 * 4 floats apart */
    int32_t blur_major;         /* 0: taps step along x, 1: along y */
    int32_t blur_tap0;          /* first entry in the tap table */
    int32_t blur_ntaps;         /* 2K + 1, 0 if no blur */
    int32_t interp;             /* XA_INTERP_LANCZOS4 (eqs. (3)-(4)) or XA_INTERP_NEAREST */
    int32_t warp_ls_mod;        /* residue mod 64 of the row stride (floats) of the warp's LDS source tile,
                                   chosen by the planner to spread the 8 x 8 sums' reads over the LDS banks */
    int32_t blur_rows;          /* outputs per thread of the blur across the minor axis (4 or 8; 0 if no blur):
                                   the blur's tiles are 64 x 4 blur_rows (taps along x) or 4 blur_rows x 64 */
} xa_view_desc;

#define XA_INTERP_LANCZOS4 0
#define XA_INTERP_NEAREST 1

/* One pyramid level of one view.  Level sizes are round(W' / scale^l);
 * quota is the number of keypoints the level may contribute.  Pixel (x, y)
 * of the level is byte offset + y * pitch + x of the arena; pitch is the
 * width rounded up to a multiple of 16 (the padding bytes are unspecified). */
typedef struct {
    int32_t width, height;
    int32_t pitch;
    int32_t quota;
    int64_t offset;             /* byte offset of this level in the pyramid arena */
    int32_t kp_base;            /* sum of the quotas of the lower levels of the view */
    int32_t view, level;
    int32_t pad;
    int64_t cand_offset;        /* first entry of this level in the candidate arena */
    int64_t cand_cap;           /* ceil(W/2) ceil(H/2): bound on corners that survive 3x3 NMS */
} xa_level_desc;

/* Plan header; the blob holds the tables at the byte offsets given here. */
typedef struct {
    uint32_t magic, version;
    int32_t src_w, src_h;
    int32_t n_views, n_levels;
    int32_t n_features, fast_threshold;
    double level_scale;
    int64_t total_bytes;        /* size of the blob */
    int64_t arena_bytes;        /* u8 pyramid arena: every level of every view */
    int64_t cand_total;         /* entries of the candidate arena */
    int64_t blur_floats;        /* floats of blurred sources (simulate workspace) */
    int32_t n_blur;             /* views with sigma > 0 */
    int32_t n_taps_total;
    int64_t off_views;          /* xa_view_desc[n_views] */
    int64_t off_levels;         /* xa_level_desc[n_views * n_levels], view-major */
    int64_t off_taps;           /* blur taps: n_taps_total x {float wa, wb; int32 dmaj, dmin}: the tap k
                                   adds wa I(p + k v_whole) + wb I(next row / column) */
    int64_t off_blur_views;     /* int32[n_blur]: view index of each blurred view */
    int64_t off_warp_prefix;    /* int32[n_views + 1]: first warp tile of each view */
    int64_t off_level_prefix;   /* int32[n_levels][n_views + 1]: first tile of each view at each level */
    int64_t off_vl_prefix;      /* int32[n_views * n_levels + 1]: first tile of each (view, level) */
    int64_t off_blur_prefix;    /* int32[n_blur + 1]: first blur tile of each blurred view */
    int64_t off_sources;        /* xa_source_desc[n_sources] */
    int32_t n_sources;
    int32_t pad;
    int64_t off_fast_flags;     /* uint8[vl_prefix[n_views * n_levels]]: per FAST tile, bit 0 = some pixel can
                                   be valid, bit 1 = some pixel can pass the content filter */
} xa_plan_header;

/* A keypoint in canonical order within its view: level ascending, then Harris
 * response descending, then raster position (y W_l + x) ascending.  (x, y)
 * are level pixel coordinates; (xs, ys) the source-image coordinates of the
 * keypoint, (x + 1/2) W'/W_l - 1/2 (likewise y) mapped through inv. */
typedef struct {
    int32_t x, y, level, bin;
    int64_t harris;
    double xs, ys;
} xa_keypoint;

/* Nearest neighbour of one query in one view pair: t = train index of the
 * nearest descriptor (smallest index on ties), d1 its distance, d2 the
 * smallest distance to any other train descriptor.  t = -1 and d1 = d2 =
 * 65535 when the train set is empty; d2 = 65535 when it has one element. */
typedef struct {
    int32_t t;
    uint16_t d1, d2;
} xa_match;

/* Outputs of xa_match_pair (device pointers, caller-allocated):
 *  kp_a/desc_a/count_a : [n_views_a][n_features] keypoints, [..][32] bytes, [n_views_a] counts
 *  kp_b/desc_b/count_b : same for image B
 *  matches             : [n_views_a * n_views_b][n_features], pair k = i * n_views_b + j
 *  pair_count          : [n_views_a * n_views_b] accepted matches per pair
 *  best                : [4] = pair index, i, j, count of the pair with the most
 *                        matches (the lowest pair index on ties) */
typedef struct {
    xa_keypoint* kp_a; uint8_t* desc_a; int32_t* count_a;
    xa_keypoint* kp_b; uint8_t* desc_b; int32_t* count_b;
    xa_match* matches; int32_t* pair_count; int32_t* best;
} xa_pair_buffers;

const char* xa_last_error(void);
const char* xa_version(void);

/* Surfaces an asynchronous failure of work enqueued earlier: XA_EHIP (with the HIP runtime's
 * message in xa_last_error) if the runtime holds an error left by a failed launch or kernel
 * (the error is cleared by reporting it) or if `stream` itself is in an error state; XA_OK
 * otherwise, also while work is still running on `stream` (the call never waits: synchronise
 * the stream first to check completed work).  Argument errors of other calls are reported by
 * those calls on the host and leave nothing for xa_check.  stream = NULL is the null stream. */
xa_status xa_check(hipStream_t stream);

/* Sampling rule of Sec. III.B: for i = 0..n_tilt, t = sqrt(2)^i and
 * phi = k b / t for k = 0, 1, ... while k b / t < 180 deg (b in degrees);
 * psi = tx = ty = 0, s = 1.  Writes at most cap entries; *n_out receives the
 * full count (XA_ECAPACITY if it exceeds cap).  Host only. */
xa_status xa_sampling_grid(int32_t n_tilt, double b_deg, xa_affine_params* out, int32_t cap, int32_t* n_out);

/* The same grid with the scale tied to the tilt index (Sec. III.B): the views of tilt
 * t_i = sqrt(2)^i get s = 1 + i * delta_s, a magnification (eq. (11) charges them the area
 * factor (1 + i delta_s)^2).  delta_s = 0 gives xa_sampling_grid.  delta_s must be >= 0. */
xa_status xa_sampling_grid_scaled(int32_t n_tilt, double b_deg, double delta_s, xa_affine_params* out, int32_t cap,
                                  int32_t* n_out);

/* Plan simulated views of one or more source images (Sec. III.B, eq. (2)):
 * canvases, maps, blur taps, pyramid levels (n_levels at factor level_scale),
 * per-level quotas of n_features keypoints (proportional to level area) and
 * the arena layout.  View i simulates sources[view_source[i]] with params[i];
 * parameters need t >= 1 and s >= 1 (reductions go through the scale stage,
 * xa_scale_sources, whose output is then a source with scale < 1).  Host
 * only.  With blob == NULL (or blob_cap too small) only *blob_bytes is set
 * (XA_ECAPACITY for a buffer that is too small). */
xa_status xa_plan_views(const xa_source_desc* sources, int32_t n_sources, const int32_t* view_source,
                        const xa_affine_params* params, int32_t n_views, int32_t n_levels, double level_scale,
                        int32_t n_features, int32_t fast_threshold, void* blob, size_t blob_cap, size_t* blob_bytes);

/* Resampling of every view of a host plan blob: XA_INTERP_LANCZOS4 (the default of
 * xa_plan_views; eqs. (3)-(4)) or XA_INTERP_NEAREST (the search-time interpolation of
 * Sec. III: the source pixel floor(p + 1/2) per axis, clamped).  Blur, canvas and validity
 * are unchanged.  Call it before copying the blob to the device.  XA_EINVAL for another
 * value or a blob that is not a view plan. */
xa_status xa_plan_set_interp(void* plan_host, int32_t interp);

/* xa_plan_views for one src_w x src_h image at offset 0 of its buffer. */
xa_status xa_plan_image(int32_t src_w, int32_t src_h, int32_t src_pitch, const xa_affine_params* params,
                        int32_t n_views, int32_t n_levels, double level_scale, int32_t n_features,
                        int32_t fast_threshold, void* blob, size_t blob_cap, size_t* blob_bytes);

/* Simulate every planned view (anti-alias blur along the compressed direction,
 * then Lanczos-4 resampling, eqs. (3)-(4)) from the sources in d_sources.
 * Writes level 0 of each view into d_arena (u8, round-half-even of the
 * interpolated value, 0 outside the source), its content mask into d_mask
 * (1 where the view pixel maps inside the source rectangle) and, if d_values
 * is not NULL, the unquantised fp32 values at the same element offsets
 * (d_values then holds arena_bytes floats).  Pixel (x, y) of view v is element
 * offset + y * pitch + x (xa_view_desc).  d_arena and d_mask must be 128-byte
 * aligned.  Workspace: xa_simulate_workspace_size(plan_host). */
size_t xa_simulate_workspace_size(const void* plan_host);
xa_status xa_simulate_views(const void* plan_host, const void* plan_dev, const uint8_t* d_sources,
                            uint8_t* d_arena, uint8_t* d_mask, float* d_values,
                            void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Warp tile widths (the output tiles of the view warp hold 512 pixels as w x 512 / w) per
 * compression class: class k holds the views with sqrt(2)^k <= t / s < sqrt(2)^(k + 1), the
 * last class open-ended.  Plans made after xa_set_warp_tiles use its widths (0 = the built-in
 * rule: 16 below t / s = 2, 8 below 8, else 4); plans made before keep theirs.  The width
 * changes only the speed: every view pixel is computed the same way.  widths: host arrays of
 * XA_WARP_CLASSES entries in {0, 4, 8, 16, 32, 64} (NULL: the rule for every class);
 * xa_get_warp_tiles returns the widths in effect.  XA_EINVAL for other widths. */
#define XA_WARP_CLASSES 8
#define XA_WARP_CANDIDATES 5
xa_status xa_set_warp_tiles(const int32_t* widths);
xa_status xa_get_warp_tiles(int32_t* widths);

/* The autotuner of the warp tile widths: for each compression class k, the sampling grid's views
 * of tilt sqrt(2)^k (scale 1) of a src_w x src_h test image, repeated until they hold about 8 M
 * view pixels (a launch that fills the chip), are blurred once, then warped with each candidate
 * width (4, 8, 16, 32, 64), 3 timed launches each after one untimed (ms[k][c], if not NULL, the
 * mean times in milliseconds).  widths[k] gets the fastest candidate if it beats the built-in
 * rule's width by more than 3 %, else the rule's width.  The result is not
 * applied: pass it to xa_set_warp_tiles (and keep it per device).  Synchronises `stream` (it
 * uploads a plan per candidate and reads events); not to be run concurrently with other work
 * timed on the same device.  Workspace: xa_tune_warp_tiles_workspace_size(src_w, src_h) bytes,
 * 256-byte aligned (0 for sizes outside 16..8192).  XA_EINVAL for sizes or pointers out of
 * range; XA_EHIP for runtime errors. */
/* The blur's outputs per thread across the minor axis (4 or 8), per compression class as for the
 * warp tiles: xa_set_blur_rows(rows) sets the table the planner reads (rows: XA_WARP_CLASSES
 * entries in {0, 4, 8}, 0 = the default 8; NULL: the default for every class); plans made before
 * keep theirs.  Only the speed changes: each blurred sample is the same sum in the same order.
 * xa_get_blur_rows returns the table in effect.  XA_EINVAL for other values.  The tuner blurs the
 * sampling grid's views of each class k >= 1 of a src_w x src_h test image (repeated to about
 * 8 M source pixels) with 4 and 8 rows, 3 timed launches each after one untimed (ms[k][2], if not
 * NULL; class 0 has no blur and gets 0), and gives rows[k] = 4 if that beats 8 by more than 3 %,
 * else 8.  Not applied; synchronises `stream`.  Workspace: xa_tune_blur_rows_workspace_size(src_w,
 * src_h) bytes, 256-byte aligned; XA_EINVAL for sizes outside 16..8192 or bad pointers. */
xa_status xa_set_blur_rows(const int32_t* rows);
xa_status xa_get_blur_rows(int32_t* rows);
size_t xa_tune_blur_rows_workspace_size(int32_t src_w, int32_t src_h);
xa_status xa_tune_blur_rows(int32_t src_w, int32_t src_h, void* d_ws, size_t ws_bytes, hipStream_t stream,
                            int32_t* rows, float* ms);

size_t xa_tune_warp_tiles_workspace_size(int32_t src_w, int32_t src_h);
xa_status xa_tune_warp_tiles(int32_t src_w, int32_t src_h, void* d_ws, size_t ws_bytes, hipStream_t stream,
                             int32_t* widths, float* ms);

/* The two stages of xa_simulate_views, callable one at a time (to time or to
 * repeat one of them).  xa_blur_views writes the blurred fp32 planes of the
 * plan's blurred views into the workspace; xa_warp_views resamples every view
 * from those planes (unblurred views read d_sources directly) and writes what
 * xa_simulate_views writes.  xa_warp_views requires a workspace that
 * xa_blur_views filled for the same plan and sources, untouched since; the
 * workspace, arguments and errors are those of xa_simulate_views
 * (xa_blur_views takes no arena or mask). */
xa_status xa_blur_views(const void* plan_host, const void* plan_dev, const uint8_t* d_sources, void* d_ws,
                        size_t ws_bytes, hipStream_t stream);
xa_status xa_warp_views(const void* plan_host, const void* plan_dev, const uint8_t* d_sources,
                        uint8_t* d_arena, uint8_t* d_mask, float* d_values,
                        void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Scale stage for the scale parameter of the sampling group (Sec. III.B).  A
 * job resamples src into dst at factor s: for s < 1 an isotropic anti-alias
 * Gaussian of standard deviation 0.8 sqrt(1/s^2 - 1) first, then Lanczos-4
 * (eqs. (3)-(4)) at p = (q + 1/2)/s - 1/2, taps clamped to the image, rounded
 * half to even.  dst must be xa_scaled_size(src, s) = round(s W) x round(s H)
 * and should carry scale = s * src.scale, so that keypoints found on views of
 * it map back to the original image.  Supported: 1/8 <= s, outputs up to
 * 32768 pixels a side.  Both images live in the same caller-owned sources
 * buffer (d_sources); all jobs run in two launches.  If d_values is not NULL
 * it receives the unquantised fp32 output at the destination's element
 * offsets (it must span the sources buffer's element count).
 * Workspace: xa_scale_workspace_size(splan_host). */
typedef struct {
    xa_source_desc src, dst;
    double s;
} xa_scale_job;
xa_status xa_scaled_size(int32_t w, int32_t h, double s, int32_t* out_w, int32_t* out_h);
xa_status xa_plan_scales(const xa_scale_job* jobs, int32_t n_jobs, void* blob, size_t blob_cap, size_t* blob_bytes);
size_t xa_scale_workspace_size(const void* splan_host);
xa_status xa_scale_sources(const void* splan_host, const void* splan_dev, uint8_t* d_sources, float* d_values,
                           void* d_ws, size_t ws_bytes, hipStream_t stream);

/* ORB feature extraction on every simulated view of the search (Sec. III.B: ORB runs on each image
 * of the simulated group; Sec. IV.C: 1000 feature points per image in the measured setting).
 * ORB on every planned view (levels 1.. of the pyramid are written into
 * d_arena and d_mask, whose level 0 must hold the simulated views): FAST-9
 * at the plan's threshold with 3x3 non-maximum suppression and a content
 * filter, integer Harris top-N per level, 30-bin intensity-centroid
 * orientation and rBRIEF-256 with the caller's test pattern d_pattern
 * (int8[256][4] = x1, y1, x2, y2 in [-15, 15]).  Outputs are
 * [n_views][n_features] keypoints and descriptors (32 bytes, bit i in byte
 * i/8 at position i%8) and [n_views] counts.  Workspace:
 * xa_extract_workspace_size(plan_host). */
size_t xa_extract_workspace_size(const void* plan_host);
xa_status xa_extract_orb(const void* plan_host, const void* plan_dev,
                         uint8_t* d_arena, uint8_t* d_mask, const int8_t* d_pattern,
                         xa_keypoint* d_kp, uint8_t* d_desc, int32_t* d_count,
                         void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Brute-force Hamming matching of every view of A (queries) against every view
 * of B (train), Sec. III.B, with the ratio test of Sec. IV.C evaluated exactly
 * as ratio_den * d1 < ratio_num * d2 (and at least two train descriptors).
 * d_matches: [n_a * n_b][n_features]; d_pair_count: [n_a * n_b]; d_best: [4]
 * (see xa_pair_buffers).  No workspace. */
xa_status xa_match_views(const uint8_t* d_desc_a, const int32_t* d_count_a, int32_t n_a,
                         const uint8_t* d_desc_b, const int32_t* d_count_b, int32_t n_b,
                         int32_t n_features, int32_t ratio_num, int32_t ratio_den,
                         xa_match* d_matches, int32_t* d_pair_count, int32_t* d_best,
                         hipStream_t stream);

/* The brute-force Hamming matching of Sec. III.B with the ratio test of Sec. IV.C (as in
 * xa_match_views), over groups of view pairs, for many image pairs in one launch: group
 * g matches query views [a0, a0 + na) against train views [b0, b0 + nb) of one
 * descriptor set (d_desc [n_views][n_features][32], d_count [n_views]) and
 * writes its na * nb view pairs from index pair_base on (pair pair_base + i * nb
 * + j) of d_matches [P][n_features] and d_pair_count [P], P = the largest
 * pair_base + na * nb; d_best [n_groups][4] = (i * nb + j, i, j, count) of the
 * group's best pair, lowest index on ties, (-1, -1, -1, 0) for an empty group.
 * The groups' pair ranges must not overlap and their views must lie inside the
 * descriptor set (n_views): xa_plan_matches and xa_match_groups reject plans
 * that break either rule with XA_EINVAL, and xa_match_batch checks the views
 * against its view plan.  queries_per_lane selects the matcher variant (the
 * autotuner times them; all give identical results): 0 = the default (the
 * matrix-core kernel), 1, 2 or 4 = the vector-ALU popcount kernel with that many queries
 * per lane, XA_MATCH_MATRIX = the matrix-core kernel (the +-1 dot product of two
 * descriptors is 256 - 2 x their Hamming distance, contracted exactly in fp4 on
 * MFMA), XA_MATCH_MATRIX_PACKED = the same kernel with each block's sixteen 32-query
 * tiles packed across the group's query views from their device-side counts (views with
 * few keypoints share blocks; each block first scans the group's counts, so it pays where
 * many views hold far fewer keypoints than n_features; groups of more than 1024 query
 * views keep one view per block).  Match plans are blobs like view plans (host and device copies). */
#define XA_MATCH_MATRIX (-1)
#define XA_MATCH_MATRIX_PACKED (-2)
typedef struct {
    int32_t a0, na;
    int32_t b0, nb;
    int64_t pair_base;
} xa_match_group;
xa_status xa_plan_matches(const xa_match_group* groups, int32_t n_groups, int32_t n_features, int32_t queries_per_lane,
                          void* blob, size_t blob_cap, size_t* blob_bytes);
xa_status xa_match_groups(const void* mplan_host, const void* mplan_dev, const uint8_t* d_desc, const int32_t* d_count,
                          int32_t n_views, int32_t ratio_num, int32_t ratio_den, xa_match* d_matches,
                          int32_t* d_pair_count, int32_t* d_best, hipStream_t stream);

/* The matcher's autotuner: every variant (1, 2, 4 queries per lane, XA_MATCH_MATRIX,
 * XA_MATCH_MATRIX_PACKED) runs the given groups on the given descriptor set (d_desc, d_count,
 * n_views as for xa_match_groups), once untimed and `reps` times timed with HIP events;
 * *best_variant gets the fastest (ms[5], if not NULL, the mean times in milliseconds, in the
 * order above).  Every variant's results are
 * the same; d_matches, d_pair_count and d_best receive them (sized as for xa_match_groups).  The
 * workspace holds the plans' device copies: xa_tune_matcher_workspace_size(groups, n_groups,
 * n_features) bytes, 256-byte aligned.  The library keeps each result per device, keyed by the
 * group table, n_features and the per-view counts (read from d_count); with XA_TUNE_USE_CACHE in
 * `flags` a known key returns its stored result and launches nothing (the outputs are then left
 * as they are); without it the variants are timed again and the entry replaced.  Synchronises
 * `stream`.  XA_EINVAL as for xa_plan_matches / xa_match_groups, for reps outside 1..1000 or for
 * unknown flags. */
#define XA_TUNE_USE_CACHE 1
size_t xa_tune_matcher_workspace_size(const xa_match_group* groups, int32_t n_groups, int32_t n_features);
xa_status xa_tune_matcher(const xa_match_group* groups, int32_t n_groups, int32_t n_features, const uint8_t* d_desc,
                          const int32_t* d_count, int32_t n_views, int32_t reps, int32_t flags,
                          xa_match* d_matches, int32_t* d_pair_count, int32_t* d_best, void* d_ws, size_t ws_bytes,
                          hipStream_t stream, int32_t* best_variant, float* ms);

/* Exact L2 nearest-two matching of SIFT descriptors (the SIFT feature matching of Sec. III.A and
 * III.C, screened by the nearest / second-nearest distance ratio of Sec. IV.C), for descriptors in
 * their usual 8-bit form: 128 components 0..255 per descriptor, row-major, d_q [n_q][128] and
 * d_t [n_t][128], both 16-byte aligned device arrays (NULL allowed where the count is 0).
 * d_out [n_q] (device): t = the train index of the smallest squared Euclidean distance d1 (the
 * lowest index on ties; -1 if n_t = 0), d2 = the smallest squared distance to any other train
 * descriptor (may equal d1); a missing distance reads 0xFFFFFFFF.  *d_count (device) = the queries
 * that pass the ratio test on distances, d1 < (ratio_num / ratio_den) d2, evaluated exactly on the
 * squared values as ratio_den^2 d1 < ratio_num^2 d2, with at least two train descriptors (the
 * paper's threshold is 3 / 4).  Squared distances are exact: the dot products are contracted on
 * the int8 matrix cores.  d_ws: caller-owned device workspace of
 * xa_match_l2_workspace_size(n_q, n_t) bytes, 16-byte aligned (none is needed when n_q = 0).
 * Asynchronous on stream; the library allocates nothing.  XA_EINVAL for counts outside
 * 0..XA_L2_MAX_DESCRIPTORS, a ratio outside 0 <= num, 1 <= den <= 2^16, a NULL or misaligned
 * array, or a short workspace; XA_EHIP if a launch fails. */
#define XA_L2_MAX_DESCRIPTORS (1 << 20)
typedef struct {
    int32_t t;
    uint32_t d1, d2;
} xa_l2_match;
size_t xa_match_l2_workspace_size(int32_t n_q, int32_t n_t);
xa_status xa_match_l2(const uint8_t* d_q, int32_t n_q, const uint8_t* d_t, int32_t n_t, int32_t ratio_num,
                      int32_t ratio_den, xa_l2_match* d_out, int32_t* d_count, void* d_ws, size_t ws_bytes,
                      hipStream_t stream);

/* xa_match_l2 for callers that cannot allocate device memory or pass a workspace (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and
 * the same results, with the per-slice partial results in a library-owned device array of
 * XA_L2_NOALLOC_SCRATCH_BYTES per GPU (held from the first call on a device until the process
 * ends; its address is looked up once per device with that device current).  The caller still
 * owns d_q, d_t, d_out and d_count, with the layouts, alignment and limits of xa_match_l2.  No
 * hipMalloc, hipFree or allocating library routine is called.  XA_ECAPACITY when
 * xa_match_l2_workspace_size(n_q, n_t) exceeds the scratch size (it never does within
 * XA_L2_MAX_DESCRIPTORS); XA_EINVAL as for xa_match_l2.  Every call on one GPU shares that GPU's
 * scratch array and leaves its contents behind: calls that overlap on one GPU (on different
 * streams, or from different threads) race and must be serialised by the caller. */
#define XA_L2_NOALLOC_SCRATCH_BYTES (16u << 20)
xa_status xa_match_l2_noalloc(const uint8_t* d_q, int32_t n_q, const uint8_t* d_t, int32_t n_t, int32_t ratio_num,
                              int32_t ratio_den, xa_l2_match* d_out, int32_t* d_count, hipStream_t stream);

/* SIFT keypoints and descriptors of one 8-bit image (Lowe's detector and descriptor, which the
 * method uses to choose the base image, Sec. III.A, and to match the re-simulated reference
 * against the target, Sec. III.C).  Scale space: s layers per octave (s + 3 Gaussian images,
 * s + 2 DoG images), input blur sigma_in, base blur sigma0, no initial doubling,
 * floor(log2 min(W, H)) - 3 octaves unless n_octaves is given, each octave from every second
 * pixel of the previous octave's G_s; separable fp32 blurs summed from tap -r to tap r with
 * every product and sum rounded.  Keypoints: strict 26-neighbour DoG extrema, at least 5 pixels
 * from the border, refined by the quadratic fit (decisions taken on cofactors, no division),
 * rejected below |D| = 255 contrast / s or at principal-curvature ratio >= edge; one keypoint
 * per orientation peak (36 bins, >= 0.8 of the highest).  Descriptors: 4 x 4 x 8 trilinear
 * histograms, unit norm, clipped at 0.2, renormalised, min(255, floor(512 v + 1/2)).
 *
 * Order: keypoints come in the order of their DoG candidates (octave, candidate layer, row,
 * column), one candidate's orientations in bin order; the first max_keypoints are written.
 * d_img: W x H u8 at row pitch `pitch` bytes (device).  d_kp [max_keypoints], d_desc
 * [max_keypoints][128] u8, d_count [2] = {keypoints written, keypoints found}: device, caller-
 * owned.  Fitted keypoints beyond raw_capacity (default 2 max_keypoints + 1024) are dropped
 * before orientation assignment, in order, so "found" then counts only the kept ones.  The
 * outputs do not depend on thread scheduling (histograms are summed in fixed point).
 * Workspace: xa_sift_workspace_size(w, h, opts) bytes, 256-byte aligned; opts NULL = defaults.
 * XA_EINVAL for sizes, options or pointers out of range; XA_EUNSUPPORTED above 2^28 pixels. */
#define XA_SIFT_MAX_KEYPOINTS 65536
typedef struct {
    int32_t n_octaves;          /* 0: floor(log2 min(W, H)) - 3, at least 1 */
    int32_t n_layers;           /* s, 1..5 (3) */
    int32_t max_keypoints;      /* capacity of d_kp / d_desc, 1..XA_SIFT_MAX_KEYPOINTS (4096) */
    int32_t raw_capacity;       /* fitted keypoints kept for orientation; 0 = 2 max_keypoints + 1024 */
    double sigma0;              /* 1.6 */
    double sigma_in;            /* 0.5 */
    double contrast;            /* 0.04, on intensities scaled to [0, 1] */
    double edge;                /* 10 */
} xa_sift_opts;
typedef struct {
    float x, y;                 /* original-image pixel coordinates */
    float size;                 /* blur of the keypoint's scale in original pixels */
    float angle;                /* radians in [0, 2 pi), atan2 convention in image axes (y down) */
    float response;             /* |D| at the fitted extremum */
    int32_t xi, yi;             /* sample position in the octave */
    int8_t octave, layer, peak, pad;
} xa_sift_keypoint;
size_t xa_sift_workspace_size(int32_t w, int32_t h, const xa_sift_opts* opts);
xa_status xa_extract_sift(const uint8_t* d_img, int32_t w, int32_t h, int32_t pitch, const xa_sift_opts* opts,
                          xa_sift_keypoint* d_kp, uint8_t* d_desc, int32_t* d_count, void* d_ws, size_t ws_bytes,
                          hipStream_t stream);

/* The SIFT matches kept for eq. (1) (Sec. III.A) and for RANSAC (Sec. III.C): of the n_q
 * queries matched by xa_match_l2 (d_matches), those passing its ratio test (at least two train
 * rows, den^2 d1^2 < num^2 d2^2), in query order.  For the o-th kept match, d_pq[2 o..] and
 * d_pt[2 o..] are the query and train keypoints' (x, y) taken through the 2 x 3 row-major maps
 * map_q and map_t (host memory, NULL = identity; e.g. a simulated view's inverse map back to its
 * source), and d_des[o] = sqrt(d1^2), the descriptor distance.  *d_n = kept matches.  Outputs
 * hold n_q entries at most (device, caller-owned).  XA_EINVAL for counts or ratios out of range
 * or NULL pointers. */
xa_status xa_sift_match_points(const xa_sift_keypoint* d_kp_q, const xa_sift_keypoint* d_kp_t,
                               const xa_l2_match* d_matches, int32_t n_q, int32_t n_t, int32_t ratio_num,
                               int32_t ratio_den, const double* map_q, const double* map_t, double* d_pq,
                               double* d_pt, double* d_des, int32_t* d_n, hipStream_t stream);

/* The whole parameter-search path for one image pair (Sec. III.B: simulate the image group over
 * the (t, phi, s) grid, extract ORB on every image of it, match with the brute-force Hamming
 * matcher and keep the parameters of the view pair with the most matches; ratio test of
 * Sec. IV.C): simulate both images, extract ORB on every view, match all view pairs, pick the
 * best pair (the paper's single-target search is the case of plan B holding one identity view).
 * Both plans must use the same n_features.  Workspace:
 * xa_match_pair_workspace_size(plan_a_host, plan_b_host). */
size_t xa_match_pair_workspace_size(const void* plan_a_host, const void* plan_b_host);
xa_status xa_match_pair(const void* plan_a_host, const void* plan_a_dev, const uint8_t* d_a,
                        const void* plan_b_host, const void* plan_b_dev, const uint8_t* d_b,
                        const int8_t* d_pattern, int32_t ratio_num, int32_t ratio_den,
                        const xa_pair_buffers* out, void* d_ws, size_t ws_bytes, hipStream_t stream);

/* The search of Sec. III.B (with the scale parameter of the sampling group, Sec. III.B and
 * Sec. IV.D, as the scale stage) for many image pairs in one sequence of launches: each pair's
 * outputs are those xa_match_pair computes for it; the batching itself is not in the paper.
 * Many image pairs at once: the scale stage (optional: splan may be NULL), the
 * simulation and ORB of every view of every image, and the group matching of
 * every image pair (one match plan), as one sequence of launches on `stream`.
 * The views come as n_chunks view plans over one sources buffer (the scale
 * stage writes its outputs into it first); chunk c is simulated and extracted
 * with one launch per stage over all of its views, then the next chunk reuses
 * the same scratch, so the workspace holds the largest chunk, not the batch.
 * Views are numbered across the chunks in order (chunk 0's views first); the
 * outputs kp/desc/count hold all of them ([total views][n_features]...), the
 * match plan's groups use that numbering, matches/pair_count hold its view
 * pairs and best [n_groups][4] its groups' best pairs.  Every view plan and the
 * match plan must agree on n_features.  xa_match_batch_capture records the same
 * sequence into a HIP graph (on a private stream; nothing is executed) that
 * xa_graph_launch replays on any stream; the graph keeps every pointer it was
 * captured with, and the host plan blobs need not outlive the capture.
 * Workspace: xa_match_batch_workspace_size(splan_host, n_chunks, vplan_hosts)
 * (0 for invalid plans). */
typedef struct {
    xa_keypoint* kp; uint8_t* desc; int32_t* count;
    xa_match* matches; int32_t* pair_count; int32_t* best;
} xa_batch_buffers;
typedef struct xa_graph xa_graph;
size_t xa_match_batch_workspace_size(const void* splan_host, int32_t n_chunks, const void* const* vplan_hosts);
xa_status xa_match_batch(const void* splan_host, const void* splan_dev, int32_t n_chunks,
                         const void* const* vplan_hosts, const void* const* vplan_devs, const void* mplan_host,
                         const void* mplan_dev, uint8_t* d_sources, const int8_t* d_pattern, int32_t ratio_num,
                         int32_t ratio_den, const xa_batch_buffers* out, void* d_ws, size_t ws_bytes,
                         hipStream_t stream);
xa_status xa_match_batch_capture(const void* splan_host, const void* splan_dev, int32_t n_chunks,
                                 const void* const* vplan_hosts, const void* const* vplan_devs,
                                 const void* mplan_host, const void* mplan_dev, uint8_t* d_sources,
                                 const int8_t* d_pattern, int32_t ratio_num, int32_t ratio_den,
                                 const xa_batch_buffers* out, void* d_ws, size_t ws_bytes, xa_graph** graph);
xa_status xa_graph_launch(xa_graph* graph, hipStream_t stream);
xa_status xa_graph_destroy(xa_graph* graph);

/* Precision of eqs. (5)-(6) for the best pair found by xa_match_views /
 * xa_match_pair: among its accepted matches (query q of view i of A, train
 * t of view j of B), count those with |H (xs_a, ys_a) - (xs_b, ys_b)| <= th,
 * H a 3x3 row-major homography acting on source coordinates of A.
 * d_out[0] = correct, d_out[1] = accepted.  H is read from host memory. */
xa_status xa_pair_precision(const xa_keypoint* d_kp_a, const xa_keypoint* d_kp_b, const xa_match* d_matches,
                            const int32_t* d_count_a, const int32_t* d_count_b, int32_t n_b,
                            int32_t n_features, int32_t ratio_num, int32_t ratio_den,
                            const int32_t* d_best, const double* H, double th, int32_t* d_out,
                            hipStream_t stream);

/* Accepted matches of a best view pair (d_best = (pair, i, j, count) as written by
 * xa_match_views / xa_match_pair / xa_match_groups for one group) as points in original
 * image coordinates, in query order: d_pa [N][2], d_pb [N][2] fp64 (N = n_features, the
 * capacity), d_dist [N] the matches' Hamming distances (nullable), *d_n = how many were
 * written (device).  n_b = views of B in the pair layout (pair = i * n_b + j).  The same
 * acceptance rule as the pair counts (eqs. (5)-(6) use these points). */
xa_status xa_best_pair_points(const xa_keypoint* d_kp_a, const xa_keypoint* d_kp_b, const xa_match* d_matches,
                              const int32_t* d_count_a, const int32_t* d_count_b, int32_t n_b, int32_t n_features,
                              int32_t ratio_num, int32_t ratio_den, const int32_t* d_best, double* d_pa, double* d_pb,
                              int32_t* d_dist, int32_t* d_n, hipStream_t stream);

/* The scaling coefficient of eq. (1) (Sec. III.A, base-image selection) over the first
 * min(*d_n, cap) matches (d_pa, d_pb [.][2] fp64 points, d_des [.] descriptor distances,
 * as written by xa_best_pair_points): the sum over consecutive matches of
 * (|a_i a_{i+1}| - |b_i b_{i+1}|) (1 - (Des(i) + Des(i+1)) / 1000), in a fixed order, into
 * *d_f (device fp64).  f > 0 means segments are longer in image A. */
xa_status xa_scaling_coefficient(const double* d_pa, const double* d_pb, const int32_t* d_des, const int32_t* d_n,
                                 int32_t cap, double* d_f, hipStream_t stream);
/* The same with fp64 descriptor distances (the SIFT distances of xa_sift_match_points). */
xa_status xa_scaling_coefficient_f64(const double* d_pa, const double* d_pb, const double* d_des, const int32_t* d_n,
                                     int32_t cap, double* d_f, hipStream_t stream);

/* Homography RANSAC over n matched points (Sec. III.C; eq. (7) is the inlier share):
 * d_pa, d_pb [n][2] fp64; d_samples [k][4] int32 match indices (the random draws, made by
 * the caller); th the inlier distance in pixels.  A sample whose indices leave [0, n) or
 * some 3 of whose 4 points (in A or in B) span a doubled triangle area below 1 px^2 scores
 * -1; otherwise H (h33 = 1) solves the 8 x 8 system that maps its 4 points of A onto those
 * of B (partial pivoting, fp64) and scores the number of matches with |H(p_a) - p_b| <= th
 * (projective image; w <= 0 counts as an outlier).  Outputs: d_scores [k]; d_best [2] =
 * (index, score) of the best sample, the lowest index on ties, (-1, -1) if none is valid;
 * d_H [9] the homography row-major: the least-squares refit (h33 = 1, Hartley-normalised
 * coordinates) over the best sample's inliers, or the sample's own H when that has no
 * solution (zeros if there is no valid sample); d_inliers [n] u8 the best sample's inlier
 * mask (nullable).  No workspace. */
xa_status xa_ransac_homography(const double* d_pa, const double* d_pb, int32_t n, const int32_t* d_samples, int32_t k,
                               double th, int32_t* d_scores, int32_t* d_best, double* d_H, uint8_t* d_inliers,
                               hipStream_t stream);

/* The Lanczos-4 warp of eqs. (3)-(4) as a differentiable map of fp32 crops and of
 * the camera parameters of eq. (2), for photometric refinement of the grid
 * search's (t, phi).  n crops of h x w fp32 values (d_img [n][h][w], row-major,
 * no padding) and one xa_affine_params per crop (d_params [n], device memory, so
 * that an optimiser can update them without a host round trip).  The map is
 * centred: view pixel q samples the crop at p = L^-1 (q - c - T) + c with
 * L = s R(psi) diag(1/t, 1) R(phi), c = ((w - 1)/2, (h - 1)/2), T = (tx, ty);
 * the view has the crop's size.  A view pixel is valid iff p lies in
 * [-1/2, w - 1/2] x [-1/2, h - 1/2]; invalid pixels are 0 and carry no gradient.
 * Taps outside the crop are clamped; weights are normalised to sum one.
 *
 * xa_warp_f32_fwd: d_out [n][h][w] fp32, d_mask [n][h][w] u8 (nullable).
 * xa_warp_f32_bwd: given dLoss/dout (d_gout [n][h][w]), writes dLoss/dimg to
 * d_gimg [n][h][w] (overwritten; nullable) and dLoss/d(t, phi, psi, s, tx, ty)
 * to d_gparams [n][6] fp64 (nullable).  The parameter gradient is summed over
 * each crop in a fixed order (deterministic); the image gradient is summed per
 * tile in fixed point and added to d_gimg with fp32 atomics, so its last bits
 * depend on the order of arrival.
 * Workspaces (16-byte aligned; each call first writes the crops' maps and tile
 * shapes there): xa_warp_f32_fwd_workspace_size and xa_warp_f32_bwd_workspace_size.
 * XA_EINVAL for sizes below 1, NULL or misaligned buffers; XA_ECAPACITY for a short
 * workspace; XA_EUNSUPPORTED above 2^28 pixels per crop or 2^38 in all. */
/* Separable Gaussian blur of n fp32 crops h x w (d_in, d_out [n][h][w], device; may not
 * alias): taps exp(-k^2 / 2 sigma^2) for |k| <= max(1, ceil(3 sigma)), normalised, edge pixels
 * replicated, rows then columns.  The coarse-to-fine smoothing of the photometric refinement of
 * (t, phi) (crop and target smoothed alike).  Workspace: xa_blur_f32_workspace_size(n, h, w)
 * bytes (the row pass).  XA_EINVAL for sizes beyond 65535 crops or rows, or sigma outside (0, 16]. */
size_t xa_blur_f32_workspace_size(int32_t n, int32_t h, int32_t w);
xa_status xa_blur_f32(const float* d_in, int32_t n, int32_t h, int32_t w, double sigma, float* d_out, void* d_ws,
                      size_t ws_bytes, hipStream_t stream);

size_t xa_warp_f32_fwd_workspace_size(int32_t n, int32_t h, int32_t w);
xa_status xa_warp_f32_fwd(const float* d_img, int32_t n, int32_t h, int32_t w, const xa_affine_params* d_params,
                          float* d_out, uint8_t* d_mask, void* d_ws, size_t ws_bytes, hipStream_t stream);
size_t xa_warp_f32_bwd_workspace_size(int32_t n, int32_t h, int32_t w);
xa_status xa_warp_f32_bwd(const float* d_img, const float* d_gout, const xa_affine_params* d_params, int32_t n,
                          int32_t h, int32_t w, float* d_gimg, double* d_gparams, void* d_ws, size_t ws_bytes,
                          hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* XAFFINE_H */
