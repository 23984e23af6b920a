// ORB on every simulated view, on gfx950: fixed-point pyramid, FAST-9 with 3x3
// non-maximum suppression, integer Harris response, per-level top-N selection,
// 7-tap integer smoothing, intensity-centroid orientation (30 bins) and
// rBRIEF-256 packed by wave ballots.  All arithmetic is integer, so the results
// are exact.  Levels live in one arena with 16-byte aligned rows, so tiles move
// between HBM and LDS in 16-byte chunks.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <climits>

#include "internal.h"

namespace xa {
namespace {

constexpr int kNegV = -1;          // FAST score stored for pixels that are not corners
constexpr int kSelThreads = 256;
constexpr int kSelMax = XA_MAX_QUOTA;

// Integer unit vectors of the 30 orientation bins: round(2^20 cos(2 pi k / 30)),
// round(2^20 sin(2 pi k / 30)); bins k and k + 15 are exact negatives.
__constant__ int32_t c_cos[30] = {1048576, 1025662, 957922, 848316, 701634, 524288, 324028, 109606,
                                  -109606, -324028, -524288, -701634, -848316, -957922, -1025662,
                                  -1048576, -1025662, -957922, -848316, -701634, -524288, -324028, -109606,
                                  109606, 324028, 524288, 701634, 848316, 957922, 1025662};
__constant__ int32_t c_sin[30] = {0, 218011, 426494, 616338, 779244, 908093, 997255, 1042832,
                                  1042832, 997255, 908093, 779244, 616338, 426494, 218011,
                                  0, -218011, -426494, -616338, -779244, -908093, -997255, -1042832,
                                  -1042832, -997255, -908093, -779244, -616338, -426494, -218011};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Largest i in [0, n) with prefix[i] <= b, searched 64 entries at a time by the whole
// wave (every lane must be active); prefix[0] == 0 <= b < prefix[n].
__device__ __forceinline__ int find_segment_wave(const int32_t* __restrict__ prefix, int n, int b) {
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) >> 6;
        const int p = lo + lane * step;
        const bool le = p < hi && prefix[p] <= b;
        const unsigned long long bal = __ballot(le);
        const int k = 63 - __clzll(bal);            // lane 0 always qualifies (prefix[lo] <= b)
        lo = lo + k * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// ------------------------------------------------------------------ pyramid

// Bilinear source position of destination index d for an n_src -> n_dst resize:
// src = (d + 1/2) n_src / n_dst - 1/2 in 1/2048 units, rounded half up, in exact
// unsigned arithmetic (1024 ((2d+1) n_src - n_dst) / n_dst split into quotient and remainder).
// Returns i0 << 11 | w1 (the second sample is min(i0 + 1, n_src - 1) with weight w1).
__device__ __forceinline__ int resample_index(int d, int n_dst, int n_src) {
    const uint32_t A = uint32_t(2 * d + 1) * uint32_t(n_src) - uint32_t(n_dst);
    const uint32_t qa = A / uint32_t(n_dst);
    const uint32_t ra = A - qa * uint32_t(n_dst);
    const uint32_t q = 1024u * qa + (2048u * ra + uint32_t(n_dst)) / (2u * uint32_t(n_dst));
    int a = int(q >> 11), w = int(q & 2047u);
    if (a >= n_src - 1) { a = n_src - 1; w = 0; }
    return (a << 11) | w;
}

constexpr int kPyrLW = 352;        // LDS row stride of the staged source rows (bytes): 256 output columns at
                                   // scale <= 1.25 span <= 322 source columns, plus 15 of 16-byte alignment
constexpr int kPyrLH = 24;         // staged source rows (16 output rows span at most 15 * 1.25 + 2)

// Level l of every view from level l-1: (sum_{2x2} wy wx pix + 2^21) >> 22; the content
// mask of a level pixel is the AND over its 2x2 footprint.  One block per 256 x 16 output
// tile, so that its set-up (prefix search, resampling positions, staging) serves 4096 pixels;
// each thread writes columns tx + 64 k (k = 0..3) on rows ty, ty + 4, ty + 8, ty + 12, so that
// a wave's lanes read neighbouring source bytes (one pass over the LDS banks) and store 64
// consecutive bytes; the source rows the tile reads are staged in LDS in 16-byte chunks.
__global__ void __launch_bounds__(256) k_pyr(const xa_level_desc* __restrict__ levels, int n_levels, int l,
                                             const int32_t* __restrict__ prefix, int n_views,
                                             uint8_t* __restrict__ arena, uint8_t* __restrict__ mask) {
    __shared__ int scol[kPyrTX], srow[kPyrTY];
    __shared__ __align__(16) uint8_t simg[kPyrLH * kPyrLW];
    __shared__ __align__(16) uint8_t smsk[kPyrLH * kPyrLW];
    const int b = blockIdx.x;
    const int vi = find_segment_wave(prefix, n_views, b);
    const xa_level_desc d = levels[vi * n_levels + l];
    const xa_level_desc p = levels[vi * n_levels + l - 1];
    const int local = b - prefix[vi];
    const int tiles_x = (d.width + kPyrTX - 1) / kPyrTX;
    const int X0 = (local % tiles_x) * kPyrTX, Y0 = (local / tiles_x) * kPyrTY;
    const int t = threadIdx.x;
    scol[t] = X0 + t < d.width ? resample_index(X0 + t, d.width, p.width) : -1;
    if (t < kPyrTY) srow[t] = Y0 + t < d.height ? resample_index(Y0 + t, d.height, p.height) : -1;
    __syncthreads();
    const int xl = min(X0 + kPyrTX, d.width) - 1 - X0, yl = min(Y0 + kPyrTY, d.height) - 1 - Y0;
    const int c_lo = scol[0] >> 11, c_hi = min((scol[xl] >> 11) + 1, p.width - 1);
    const int r_lo = srow[0] >> 11, r_hi = min((srow[yl] >> 11) + 1, p.height - 1);
    const int cb = c_lo & ~15, nch = (((c_hi + 16) & ~15) - cb) >> 4, nr = r_hi - r_lo + 1;
    const uint8_t* P = arena + p.offset;
    const uint8_t* M = mask + p.offset;
    const bool staged = nch * 16 <= kPyrLW && nr <= kPyrLH;
    if (staged) {
        for (int e = t; e < nr * nch; e += 256) {
            const int r = e / nch, k = e - (e / nch) * nch;
            const size_t g = size_t(r_lo + r) * p.pitch + cb + 16 * k;
            *reinterpret_cast<uint4*>(simg + r * kPyrLW + 16 * k) = *reinterpret_cast<const uint4*>(P + g);
            *reinterpret_cast<uint4*>(smsk + r * kPyrLW + 16 * k) = *reinterpret_cast<const uint4*>(M + g);
        }
    }
    __syncthreads();
    const int tx = t & 63, ty = t >> 6;
    if (X0 + tx >= d.width) return;
    // the thread's columns tx + 64 k: a wave's lanes read neighbouring source bytes
    int cx0[4], cx1[4], cw0[4], cw1[4];
    bool cv_ok[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        cv_ok[k] = X0 + tx + 64 * k < d.width;
        const int cv = cv_ok[k] ? scol[tx + 64 * k] : 0;
        cx0[k] = cv >> 11;
        cw1[k] = cv & 2047;
        cw0[k] = 2048 - cw1[k];
        cx1[k] = min(cx0[k] + 1, p.width - 1);
    }
    // The staged and the direct path are separate loops, so that the staged one reads LDS with
    // LDS instructions (one loop over a pointer that may be either compiles to flat loads).
    auto rows = [&](auto fetch) {
        for (int rr = 0; rr < kPyrTY / 4; ++rr) {
            const int yr = ty + 4 * rr;
            const int y = Y0 + yr;
            if (y >= d.height) break;
            const int rv = srow[yr];
            const int y0 = rv >> 11, wy1 = rv & 2047, wy0 = 2048 - wy1, y1 = min(y0 + 1, p.height - 1);
            const size_t o = size_t(d.offset) + size_t(y) * d.pitch + X0 + tx;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!cv_ok[k]) break;
                int p00, p01, p10, p11, m;
                fetch(y0, y1, cx0[k], cx1[k], p00, p01, p10, p11, m);
                const int top = cw0[k] * p00 + cw1[k] * p01;
                const int bot = cw0[k] * p10 + cw1[k] * p11;
                arena[o + 64 * k] = uint8_t((wy0 * top + wy1 * bot + (1 << 21)) >> 22);
                mask[o + 64 * k] = uint8_t(m & 1);
            }
        }
    };
    if (staged) {
        rows([&](int y0, int y1, int x0, int x1, int& p00, int& p01, int& p10, int& p11, int& m) {
            const int a0 = (y0 - r_lo) * kPyrLW - cb, a1 = (y1 - r_lo) * kPyrLW - cb;
            p00 = simg[a0 + x0]; p01 = simg[a0 + x1]; p10 = simg[a1 + x0]; p11 = simg[a1 + x1];
            m = smsk[a0 + x0] & smsk[a0 + x1] & smsk[a1 + x0] & smsk[a1 + x1];
        });
    } else {
        rows([&](int y0, int y1, int x0, int x1, int& p00, int& p01, int& p10, int& p11, int& m) {
            const size_t a0 = size_t(y0) * p.pitch, a1 = size_t(y1) * p.pitch;
            p00 = P[a0 + x0]; p01 = P[a0 + x1]; p10 = P[a1 + x0]; p11 = P[a1 + x1];
            m = M[a0 + x0] & M[a0 + x1] & M[a1 + x0] & M[a1 + x1];
        });
    }
}

// ------------------------------------------------------------------ FAST-9 + NMS + Harris + smoothing

// Bresenham circle of radius 3, clockwise from 12 o'clock (x right, y down).
constexpr int kCircleX[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
constexpr int kCircleY[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

// FAST-9 score of an LDS pixel (row stride S): with d_k the circle pixel minus the centre,
// V = max over the 16 arcs of 9 contiguous circle pixels of the larger of the arc's min d and
// its min -d; kNegV unless V > T.  A pixel with a bright 9-arc (all d > T) has no dark one, since
// two 9-arcs of 16 share a pixel, so V is the score of the polarity that makes it a corner.
// Arc minima from three-wide minima: min over k..k+8 = min(m3[k], m3[k+3], m3[k+6]).
template <int S>
__device__ __forceinline__ int fast_score_lds(const uint8_t* p, int T) {
    const int c = p[0];
    int d[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) d[k] = int(p[kCircleY[k] * S + kCircleX[k]]) - c;
    int lo3[16], hi3[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        lo3[k] = min(min(d[k], d[(k + 1) & 15]), d[(k + 2) & 15]);
        hi3[k] = max(max(d[k], d[(k + 1) & 15]), d[(k + 2) & 15]);
    }
    int bright = INT_MIN, dark = INT_MAX;     // max over arcs of the arc min; min over arcs of the arc max
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        bright = max(bright, min(min(lo3[k], lo3[(k + 3) & 15]), lo3[(k + 6) & 15]));
        dark = min(dark, max(max(hi3[k], hi3[(k + 3) & 15]), hi3[(k + 6) & 15]));
    }
    const int v = max(bright, -dark);
    return v > T ? v : kNegV;
}

constexpr int kFH = 4;                              // halo rows above and below the tile
constexpr int kFLW = kFastTX + 32;                  // LDS row: x0 - 16 .. x0 + 79 (6 chunks of 16)
constexpr int kFLH = kFastTY + 2 * kFH;             // 40 rows
constexpr int kFChunks = kFLW / 16;
constexpr int kSW = kFastTX + 2, kSH = kFastTY + 2; // FAST scores: the tile plus a one-pixel ring
constexpr int kMaxBlockCand = kFastTX * kFastTY / 4;

// Exact pre-test of FAST-9 on the four compass pixels: any arc of 9 contiguous circle pixels
// holds two of them, so a pixel can be a corner only if two are brighter than c + T or two
// darker than c - T.  Two of the four exceed c + T iff the second largest does, and two fall
// below c - T iff the second smallest does; with the pairs (n, s) and (e, w) ordered, the second
// largest is max(min of the two maxima, both minima) and the second smallest min(max of the two
// minima, both maxima).
__device__ __forceinline__ bool fast_pretest(int c, int n, int e, int s, int w, int T) {
    const int hi1 = max(n, s), lo1 = min(n, s), hi2 = max(e, w), lo2 = min(e, w);
    const int second_hi = max(max(lo1, lo2), min(hi1, hi2));
    const int second_lo = min(min(hi1, hi2), max(lo1, lo2));
    return max(second_hi - c, c - second_lo) > T;
}

// One block per 64 x 32 tile of one (view, level) that can hold detections:
//  1. the tile plus a 4-row / 16-column halo is staged in LDS in 16-byte chunks (border
//     replicated, byte by byte, for chunks that leave the image);
//  2. one pass over the tile, thread = column, 8 rows each: the 7-tap smoothing
//     [18 34 49 54 49 34 18] / 256 (exact horizontal sums by v_dot4 over byte windows, rounded
//     vertical pass) and, from the same row words, the FAST pre-test of the tile's pixels on
//     their four compass pixels (any 9-pixel arc contains two of them); the one-pixel ring the
//     suppression also needs is pre-tested separately.  Pixels that pass are queued;
//  3. full FAST-9 scores of the queued pixels;
//  4. 3x3 non-maximum suppression (ties go to the earlier raster position) and the content
//     filter on the corners of the +-B box, then one atomic reservation per block in the
//     candidate arena and the Harris response of each survivor, 16 lanes per candidate (each
//     lane takes 3 or 4 of the 49 window positions; the integer sums are reduced across them).
// Tiles of a tilted view's empty corners skip work that cannot matter (flags from the
// planner): smoothing when no pixel of the tile can be valid, detection when no pixel can
// pass the content filter.
__global__ void __launch_bounds__(256) k_fast(const uint8_t* __restrict__ fast_flags,
                                              const xa_level_desc* __restrict__ levels, const int32_t* __restrict__ prefix,
                                              int nvl, int T, const uint8_t* __restrict__ arena,
                                              const uint8_t* __restrict__ mask, Cand* __restrict__ cand,
                                              int32_t* __restrict__ cand_count, uint8_t* __restrict__ smooth) {
    constexpr int kScoreWords = (kSH * kSW) / 4;    // 4 scores per 8-byte word
    static_assert((kSH * kSW) % 4 == 0, "score grid in whole 8-byte words");
    constexpr int kRing = 2 * kSW + 2 * kFastTY;    // ring pixels: top and bottom rows, left and right columns
    __shared__ __align__(16) uint8_t img[kFLH * kFLW];
    __shared__ __align__(16) uint8_t sm[kFastTY * kFastTX];
    __shared__ __align__(8) int16_t score[kSH * kSW];
    __shared__ int16_t queue[kSH * kSW];
    __shared__ int16_t cxy[2 * kMaxBlockCand];
    __shared__ int qn, cn, cbase;
    const int b = blockIdx.x;
    const int vl = find_segment_wave(prefix, nvl, b);
    const xa_level_desc d = levels[vl];
    if (d.cand_cap == 0) return;
    const int W = d.width, H = d.height, pitch = d.pitch;
    const int local = b - prefix[vl];
    const int tiles_x = (W + kFastTX - 1) / kFastTX;
    const int x0 = (local % tiles_x) * kFastTX, y0 = (local / tiles_x) * kFastTY;
    const uint8_t* P = arena + d.offset;
    const int t = threadIdx.x;
    // which parts of the tile can matter (decided by the planner, see fast_tile_flags)
    const uint8_t flags = fast_flags[b];
    const bool need_smooth = (flags & 1) != 0, may_detect = (flags & 2) != 0;
    if (!need_smooth && !may_detect) return;
    const bool detect = may_detect && !(x0 + kFastTX <= kBorder - 1 || x0 - 1 >= W - kBorder ||
                                        y0 + kFastTY <= kBorder - 1 || y0 - 1 >= H - kBorder);
    for (int e = t; e < kFLH * kFChunks; e += 256) {
        const int r = e / kFChunks, k = e - (e / kFChunks) * kFChunks;
        const int gy = clampi(y0 - kFH + r, 0, H - 1);
        const int gx = x0 - 16 + 16 * k;
        uint4 v;
        if (gx >= 0 && gx + 16 <= W) {
            v = *reinterpret_cast<const uint4*>(P + size_t(gy) * pitch + gx);
        } else {
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t acc = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc |= uint32_t(P[size_t(gy) * pitch + clampi(gx + 4 * q + j, 0, W - 1)]) << (8 * j);
                w[q] = acc;
            }
            v = make_uint4(w[0], w[1], w[2], w[3]);
        }
        *reinterpret_cast<uint4*>(img + r * kFLW + 16 * k) = v;
    }
    if (detect)   // every score starts at kNegV (-1: all bits set)
        for (int e = t; e < kScoreWords; e += 256) reinterpret_cast<unsigned long long*>(score)[e] = ~0ull;
    if (t == 0) { qn = 0; cn = 0; }
    __syncthreads();

    // ---- smoothing and the tile's pre-test: thread = column c, tile rows 8g .. 8g + 7
    {
        const int c = t & 63, g = __builtin_amdgcn_readfirstlane(t >> 6);   // g: the wave's row group
        const int lx = c + 16 - 3;                 // first byte of the 7-tap window
        const int a = lx & ~3, o = lx & 3;
        const uint32_t w03 = 18u | (34u << 8) | (49u << 16) | (54u << 24);
        const uint32_t w46 = 49u | (34u << 8) | (18u << 16);
        int h[14], ctr[14], wst[8], est[8];
#pragma unroll
        for (int j = 0; j < 14; ++j) {
            const uint32_t* row = reinterpret_cast<const uint32_t*>(img + (kFH + 8 * g - 3 + j) * kFLW + a);
            const uint32_t d0 = row[0], d1 = row[1], d2 = row[2];
            const uint32_t lo = __builtin_amdgcn_alignbyte(d1, d0, o);                // bytes lx .. lx + 3
            const uint32_t hi = __builtin_amdgcn_alignbyte(d2, d1, o) & 0x00FFFFFFu;  // bytes lx + 4 .. lx + 6
            h[j] = int(__builtin_amdgcn_udot4(lo, w03, __builtin_amdgcn_udot4(hi, w46, 0u, false), false));
            ctr[j] = int(lo >> 24);                                                    // the column's own byte
            if (j >= 3 && j < 11) {
                wst[j - 3] = int(lo & 0xFFu);                                          // 3 columns left
                est[j - 3] = int(hi >> 16);                                            // 3 columns right
            }
        }
        if (need_smooth) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int s = 18 * h[j] + 34 * h[j + 1] + 49 * h[j + 2] + 54 * h[j + 3] + 49 * h[j + 4] +
                              34 * h[j + 5] + 18 * h[j + 6];
                sm[(8 * g + j) * kFastTX + c] = uint8_t((s + (1 << 15)) >> 16);
            }
        }
        if (detect) {
            const int gx = x0 + c;
            const bool col_ok = gx >= kBorder - 1 && gx <= W - kBorder;
            uint32_t pass = 0;                     // bit j: tile row 8 g + j passes
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int gy = y0 + 8 * g + j;     // the same for the whole wave
                const bool ok = col_ok && gy >= kBorder - 1 && gy <= H - kBorder &&
                                fast_pretest(ctr[j + 3], ctr[j], est[j], ctr[j + 6], wst[j], T);
                pass |= uint32_t(ok) << j;
            }
            while (pass) {
                const int j = __builtin_ctz(pass);
                pass &= pass - 1;
                queue[atomicAdd(&qn, 1)] = int16_t((8 * g + j + 1) * kSW + c + 1);
            }
        }
    }
    // ---- the ring's pre-test (rows -1 and 32, columns -1 and 64 of the tile)
    if (detect) {
        for (int e = t; e < kRing; e += 256) {
            int sx, sy;
            if (e < 2 * kSW) { sy = e < kSW ? 0 : kSH - 1; sx = e < kSW ? e : e - kSW; }
            else { const int r = e - 2 * kSW; sx = r < kFastTY ? 0 : kSW - 1; sy = 1 + (r < kFastTY ? r : r - kFastTY); }
            const int gx = x0 - 1 + sx, gy = y0 - 1 + sy;
            if (gx >= kBorder - 1 && gx <= W - kBorder && gy >= kBorder - 1 && gy <= H - kBorder) {
                const uint8_t* p = img + (sy - 1 + kFH) * kFLW + sx - 1 + 16;
                if (fast_pretest(p[0], p[-3 * kFLW], p[3], p[3 * kFLW], p[-3], T))
                    queue[atomicAdd(&qn, 1)] = int16_t(sy * kSW + sx);
            }
        }
    }
    __syncthreads();
    // ---- smoothed tile out, 16 bytes per store (rows are padded to 16 bytes)
    for (int e = t; need_smooth && e < kFastTY * (kFastTX / 16); e += 256) {
        const int r = e >> 2, k = e & 3;
        const int y = y0 + r, x = x0 + 16 * k;
        if (y < H && x < W)
            *reinterpret_cast<uint4*>(smooth + d.offset + size_t(y) * pitch + x) =
                *reinterpret_cast<const uint4*>(sm + r * kFastTX + 16 * k);
    }
    if (!detect) return;
    // ---- full scores of the queued pixels
    const int nq = qn;
    for (int q = t; q < nq; q += 256) {
        const int e = queue[q];
        const int sy = e / kSW, sx = e - (e / kSW) * kSW;
        score[e] = int16_t(fast_score_lds<kFLW>(img + (sy - 1 + kFH) * kFLW + sx - 1 + 16, T));
    }
    __syncthreads();
    // ---- NMS + content filter -> block candidate list.  Only queued pixels can score above T
    // (every other pixel keeps kNegV), so the queue is walked instead of the tile.
    const uint8_t* Mk = mask + d.offset;
    for (int q = t; q < nq; q += 256) {
        const int e = queue[q];
        const int ty = e / kSW - 1, tx = e - (e / kSW) * kSW - 1;       // tile coordinates
        if (tx < 0 || tx >= kFastTX || ty < 0 || ty >= kFastTY) continue;   // ring pixel
        const int x = x0 + tx, y = y0 + ty;
        if (x < kBorder || x >= W - kBorder || y < kBorder || y >= H - kBorder) continue;
        const int vp = score[e];
        if (vp <= T) continue;
        bool keep = true;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0) continue;
                const int vq = score[e + dy * kSW + dx];
                const bool q_after = dy > 0 || (dy == 0 && dx > 0);
                keep = keep && (vp > vq || (vp == vq && q_after));
            }
        if (!keep) continue;
        const size_t r0 = size_t(y - kBorder) * pitch, r1 = size_t(y + kBorder) * pitch;
        if (!(Mk[r0 + x - kBorder] && Mk[r0 + x + kBorder] && Mk[r1 + x - kBorder] && Mk[r1 + x + kBorder])) continue;
        const int s = atomicAdd(&cn, 1);
        cxy[2 * s] = int16_t(tx);
        cxy[2 * s + 1] = int16_t(ty);
    }
    __syncthreads();
    const int nc = cn;
    if (nc == 0) return;
    if (t == 0) cbase = atomicAdd(&cand_count[vl], nc);
    __syncthreads();
    const int base = cbase;
    // Harris response: 3x3 Sobel gradients over the 7x7 window, structure tensor sums a, b, c,
    // R = 25 (a b - c^2) - (a + b)^2 in int64.  16 lanes per candidate; the group's lanes are
    // active together, so the xor shuffles below stay inside it.
    const int grp = t >> 4, sub = t & 15;
    for (int s = grp; s < nc; s += 256 / 16) {
        const int tx = cxy[2 * s], ty = cxy[2 * s + 1];
        int sa = 0, sb = 0, sc = 0;
        for (int pw = sub; pw < 49; pw += 16) {
            const int dy = pw / 7 - 3, dx = pw - (pw / 7) * 7 - 3;
            const uint8_t* p = img + (ty + kFH + dy) * kFLW + tx + 16 + dx;
            const int v00 = p[-kFLW - 1], v01 = p[-kFLW], v02 = p[-kFLW + 1];
            const int v10 = p[-1], v12 = p[1];
            const int v20 = p[kFLW - 1], v21 = p[kFLW], v22 = p[kFLW + 1];
            const int ix = (v02 + 2 * v12 + v22) - (v00 + 2 * v10 + v20);
            const int iy = (v20 + 2 * v21 + v22) - (v00 + 2 * v01 + v02);
            sa += ix * ix;
            sb += iy * iy;
            sc += ix * iy;
        }
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) {
            sa += __shfl_xor(sa, off);
            sb += __shfl_xor(sb, off);
            sc += __shfl_xor(sc, off);
        }
        if (sub == 0 && base + s < d.cand_cap) {
            const long long tr = (long long)(sa + sb);
            Cand cd;
            cd.raster = uint32_t(y0 + ty) * uint32_t(W) + uint32_t(x0 + tx);
            cd.pad = 0;
            cd.harris = 25LL * ((long long)sa * sb - (long long)sc * sc) - tr * tr;
            cand[d.cand_offset + base + s] = cd;
        }
    }
}

// ------------------------------------------------------------------ top-N per level

// order-preserving map int64 -> uint64
__device__ __forceinline__ unsigned long long okey(long long r) { return (unsigned long long)r ^ 0x8000000000000000ull; }

// Digit (0..255) holding the k-th item, counting from the top bin when descending and from
// the bottom bin otherwise, of a 256-bin histogram; every thread of a 256-thread block takes
// part.  *s_k receives the rank of the item inside that bin, *s_bin the bin's size.
__device__ int pick_digit(const int* hist, int* wsum, bool descending, int k, int* s_digit, int* s_k, int* s_bin) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int g = descending ? 255 - t : t;
    const int h = hist[g];
    int incl = h;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    for (int w = 0; w < wv; ++w) incl += wsum[w];
    const int before = incl - h;
    if (before < k && k <= incl) { *s_digit = g; *s_k = k - before; *s_bin = h; }
    __syncthreads();
    return *s_digit;
}

// The candidates of one (view, level) block: the first kSelRegs * kSelThreads live in
// registers (item i = threadIdx.x + r kSelThreads in slot r), the rest are read from memory.
constexpr int kSelRegs = 8;

struct SelItems {
    unsigned long long key[kSelRegs];   // okey(Harris response)
    uint32_t ras[kSelRegs];             // raster position
};

// Calls f(key, raster) for every candidate this thread owns.
template <typename F>
__device__ __forceinline__ void for_items(const SelItems& it, const Cand* cd, int C, F f) {
#pragma unroll
    for (int r = 0; r < kSelRegs; ++r)
        if (int(threadIdx.x) + r * kSelThreads < C) f(it.key[r], it.ras[r]);
    for (int i = threadIdx.x + kSelRegs * kSelThreads; i < C; i += kSelThreads) {
        const Cand c = cd[i];
        f(okey(c.harris), c.raster);
    }
}

// k-th value, in the order given by `descending`, among this block's candidates with
// pred(key, raster), of the field val(key, raster), by 8-bit digits of its bits
// 8 n_digits - 1 .. 0 (higher bits are taken to be shared by every such candidate and come
// back as zero).  *k_rem receives how many candidates equal to it complete k, *n_eq how many
// equal it (n_items when n_digits is 0).
template <typename Val, typename Pred>
__device__ unsigned long long radix_select(const SelItems& it, const Cand* cd, int C, int n_items, int k, int n_digits,
                                           bool descending, Val val, Pred pred, int* hist, int* wsum, int* k_rem,
                                           int* n_eq, int* s_digit, int* s_k, int* s_bin) {
    unsigned long long prefix = 0, pmask = 0;
    int eq = n_items;
    for (int shift = 8 * (n_digits - 1); shift >= 0; shift -= 8) {
        hist[threadIdx.x] = 0;
        __syncthreads();
        for_items(it, cd, C, [&](unsigned long long key, uint32_t ras) {
            const unsigned long long u = val(key, ras);
            if (pred(key, ras) && (u & pmask) == prefix) atomicAdd(&hist[(u >> shift) & 0xFF], 1);
        });
        __syncthreads();
        const int dgt = pick_digit(hist, wsum, descending, k, s_digit, s_k, s_bin);
        prefix |= (unsigned long long)dgt << shift;
        pmask |= 0xFFull << shift;
        k = *s_k;
        eq = *s_bin;
        __syncthreads();
    }
    *k_rem = k;
    *n_eq = eq;
    return prefix;
}

// 8-bit digits that cover bits 0 .. the highest set bit of x (0 for x = 0)
__device__ __forceinline__ int digits_for(unsigned long long x) { return x ? (64 - __clzll((long long)x) + 7) >> 3 : 0; }

__device__ __forceinline__ unsigned long long wave_or(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ unsigned long long wave_and(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v &= __shfl_xor(v, off);
    return v;
}

// One block per (view, level): the top `quota` candidates by (Harris response descending,
// raster ascending), in that order, into the staging slots.  The response threshold is found
// by radix selection (over the positive responses alone when there are at least `quota` of
// them, which leaves fewer distinct high bytes), ties at the threshold by a second selection
// of the raster position; the kept candidates are compacted into LDS and each is written at
// its rank, counted against the others.
__global__ void __launch_bounds__(kSelThreads) k_select(const xa_level_desc* __restrict__ levels, int n_features,
                                                        const Cand* __restrict__ cand,
                                                        const int32_t* __restrict__ cand_count,
                                                        int4* __restrict__ stage, int32_t* __restrict__ stage_count) {
    // kept entries, padded with (0, 0xFFFFFFFF) to a multiple of 8: such an entry never
    // precedes another
    __shared__ __align__(16) unsigned long long s_key[kSelMax + 8];
    __shared__ __align__(16) uint32_t s_ras[kSelMax + 8];
    __shared__ int hist[256], wsum[kSelThreads / 64];
    __shared__ unsigned long long s_red[4][kSelThreads / 64];
    __shared__ int s_digit, s_k, s_bin, s_n, s_pos;
    const int vl = blockIdx.x, t = threadIdx.x;
    const xa_level_desc d = levels[vl];
    const int C = int(min((long long)cand_count[vl], (long long)d.cand_cap));
    const int quota = d.quota;
    const Cand* cd = cand + d.cand_offset;
    const int n = min(C, quota);
    if (n <= 0) {                   // nothing to keep (no candidates, or a zero quota)
        if (t == 0) stage_count[vl] = 0;
        return;
    }
    SelItems it;
#pragma unroll
    for (int r = 0; r < kSelRegs; ++r) {
        const int i = t + r * kSelThreads;
        Cand c{};
        if (i < C) c = cd[i];
        it.key[r] = okey(c.harris);
        it.ras[r] = c.raster;
    }
    if (t == 0) { s_n = 0; s_pos = 0; }
    __syncthreads();
    unsigned long long K = 0;       // kept: key > K, or key == K and raster <= Rthr
    uint32_t Rthr = 0xFFFFFFFFu;
    if (C > n) {
        constexpr unsigned long long kPos = 0x8000000000000000ull;    // okey of a zero response
        unsigned long long o = 0, a = ~0ull, op = 0, ap = ~0ull;
        int npos = 0;
        for_items(it, cd, C, [&](unsigned long long key, uint32_t) {
            o |= key; a &= key;
            if (key > kPos) { op |= key; ap &= key; ++npos; }
        });
        o = wave_or(o); a = wave_and(a); op = wave_or(op); ap = wave_and(ap);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) npos += __shfl_xor(npos, off);
        if ((t & 63) == 0) {
            s_red[0][t >> 6] = o; s_red[1][t >> 6] = a; s_red[2][t >> 6] = op; s_red[3][t >> 6] = ap;
            atomicAdd(&s_pos, npos);
        }
        __syncthreads();
        o = 0; a = ~0ull; op = 0; ap = ~0ull;
        for (int w = 0; w < kSelThreads / 64; ++w) {
            o |= s_red[0][w]; a &= s_red[1][w]; op |= s_red[2][w]; ap &= s_red[3][w];
        }
        const bool pos_only = s_pos >= n;
        if (pos_only) { o = op; a = ap; }
        const int nd = digits_for(o ^ a);
        const unsigned long long high = nd == 8 ? 0ull : a & ~((1ull << (8 * nd)) - 1);
        const int n_items = pos_only ? s_pos : C;
        int k_eq, n_eq;
        K = high | radix_select(
            it, cd, C, n_items, n, nd, true, [](unsigned long long key, uint32_t) { return key; },
            [&](unsigned long long key, uint32_t) { return !pos_only || key > kPos; }, hist, wsum, &k_eq, &n_eq,
            &s_digit, &s_k, &s_bin);
        // among responses equal to K the first k_eq raster positions are kept: all of them when
        // k_eq covers every such candidate
        if (k_eq < n_eq) {
            int k_r, n_r;
            const uint32_t npix = uint32_t(d.width) * uint32_t(d.height);
            Rthr = uint32_t(radix_select(
                it, cd, C, n_eq, k_eq, digits_for(npix - 1), false,
                [](unsigned long long, uint32_t ras) { return (unsigned long long)ras; },
                [&](unsigned long long key, uint32_t) { return key == K; }, hist, wsum, &k_r, &n_r, &s_digit,
                &s_k, &s_bin));
        }
    }
    // compact the n kept candidates (all of them when C <= quota)
    for_items(it, cd, C, [&](unsigned long long key, uint32_t ras) {
        if (key > K || (key == K && ras <= Rthr)) {
            const int slot = atomicAdd(&s_n, 1);
            s_key[slot] = key;
            s_ras[slot] = ras;
        }
    });
    if (t < 8) { s_key[n + t] = 0ull; s_ras[n + t] = 0xFFFFFFFFu; }
    __syncthreads();
    // rank of kept entry i = entries before it in (key descending, raster ascending) order;
    // rasters are distinct, so the ranks are a permutation of 0 .. n-1.  Each thread ranks
    // entries t, t + kSelThreads, ... against 8 entries per step of 128-bit LDS reads.
    const int per = (n + kSelThreads - 1) / kSelThreads;
    unsigned long long ki[kSelRegs];
    uint32_t ri[kSelRegs];
    int rank[kSelRegs];
#pragma unroll
    for (int r = 0; r < kSelRegs; ++r) {
        const int i = t + r * kSelThreads;
        ki[r] = i < n ? s_key[i] : 0ull;
        ri[r] = i < n ? s_ras[i] : 0xFFFFFFFFu;
        rank[r] = 0;
    }
    const ulonglong2* k2 = reinterpret_cast<const ulonglong2*>(s_key);
    const uint4* r4 = reinterpret_cast<const uint4*>(s_ras);
    for (int j = 0; j < n; j += 8) {
        const ulonglong2 a0 = k2[j / 2], a1 = k2[j / 2 + 1], a2 = k2[j / 2 + 2], a3 = k2[j / 2 + 3];
        const uint4 b0 = r4[j / 4], b1 = r4[j / 4 + 1];
        const unsigned long long kj[8] = {a0.x, a0.y, a1.x, a1.y, a2.x, a2.y, a3.x, a3.y};
        const uint32_t rj[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
        for (int r = 0; r < kSelRegs; ++r) {
            if (r >= per) break;
#pragma unroll
            for (int e = 0; e < 8; ++e) rank[r] += (kj[e] > ki[r] || (kj[e] == ki[r] && rj[e] < ri[r])) ? 1 : 0;
        }
    }
    int4* st = stage + size_t(d.view) * n_features + d.kp_base;
#pragma unroll
    for (int r = 0; r < kSelRegs; ++r) {
        if (t + r * kSelThreads < n) {
            const long long R = (long long)(ki[r] ^ 0x8000000000000000ull);
            st[rank[r]] = make_int4(int(ri[r] % uint32_t(d.width)), int(ri[r] / uint32_t(d.width)),
                                    int(uint32_t(R & 0xFFFFFFFFll)), int(R >> 32));
        }
    }
    if (t == 0) stage_count[vl] = n;
}

// ------------------------------------------------------------------ orientation + rBRIEF

__device__ __forceinline__ int rnd20(int v) {
    const int a = v < 0 ? -v : v;
    const int r = (a + (1 << 19)) >> 20;
    return v < 0 ? -r : r;
}

// The rotated test offsets of the BRIEF pattern for every orientation bin: entry (b, i) packs
// (ax, ay, bx, by) of test i steered by bin b as four int8 (each within +-21: the pattern's
// coordinates are clamped to [-15, 15]).  One block per bin, one thread per test.
// The extraction's set-up in one launch: blocks 0 .. kOrientBins - 1 steer the pattern (block b:
// bin b), the rest zero the n candidate counters.
__global__ void __launch_bounds__(kBriefTests) k_steer(const int8_t* __restrict__ pattern, uint32_t* __restrict__ steer,
                                                       int32_t* __restrict__ zero, int n, int32_t* __restrict__ zero2,
                                                       int n2) {
    if (int(blockIdx.x) >= kOrientBins) {
        const int z = (blockIdx.x - kOrientBins) * kBriefTests + threadIdx.x;
        if (z < n) zero[z] = 0;
        if (z < n2) zero2[z] = 0;
        return;
    }
    const int b = blockIdx.x, i = threadIdx.x;
    const int Cb = c_cos[b], Sb = c_sin[b];
    const int x1 = clampi(pattern[4 * i], -15, 15), y1 = clampi(pattern[4 * i + 1], -15, 15);
    const int x2 = clampi(pattern[4 * i + 2], -15, 15), y2 = clampi(pattern[4 * i + 3], -15, 15);
    const int ax = rnd20(x1 * Cb - y1 * Sb), ay = rnd20(x1 * Sb + y1 * Cb);
    const int bx = rnd20(x2 * Cb - y2 * Sb), by = rnd20(x2 * Sb + y2 * Cb);
    steer[b * kBriefTests + i] = uint32_t(uint8_t(ax)) | (uint32_t(uint8_t(ay)) << 8) | (uint32_t(uint8_t(bx)) << 16) |
                                 (uint32_t(uint8_t(by)) << 24);
}


// Two keypoints per wave: intensity-centroid moments over the radius-15 disk, integer argmax
// over the 30 bins, then 256 steered binary tests on the smoothed level, packed four 64-bit
// ballots at a time.  Keypoints are written in canonical order.  The kernel is bound by its
// chain of dependent loads (counts, level, keypoint, disk, steered table, smoothed samples), so
// each step is taken for both keypoints before the next: their loads overlap.
constexpr int kKpPerWave = 2;

__global__ void __launch_bounds__(256) k_orient_brief(const xa_view_desc* __restrict__ views,
                                                      const xa_level_desc* __restrict__ levels, int n_levels,
                                                      int n_features, const uint8_t* __restrict__ arena,
                                                      const uint8_t* __restrict__ smooth, const int4* __restrict__ stage,
                                                      const int32_t* __restrict__ stage_count,
                                                      const uint32_t* __restrict__ steer, xa_keypoint* __restrict__ kp,
                                                      uint8_t* __restrict__ desc, int32_t* __restrict__ count) {
    constexpr int KW = kKpPerWave;
    const int v = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int k0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * KW;
    // the level of keypoint k: lane l < n_levels holds level l's count; an inclusive wave scan
    // gives each level's end, and the first level whose end exceeds k holds it
    const int cnt = lane < n_levels ? stage_count[v * n_levels + lane] : 0;
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    const int pre = __shfl(incl, 63);
    if (k0 == 0 && lane == 0) count[v] = pre;
    int lev[KW], x[KW], y[KW];
    long long R[KW];
    xa_level_desc d[KW];
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        const int k = k0 + u;
        const unsigned long long past = __ballot(lane < n_levels && incl > k);
        lev[u] = (past && k < n_features) ? int(__ffsll((long long)past)) - 1 : -1;
    }
    if (lev[0] < 0) return;                   // keypoints of a wave are consecutive: none is kept
#pragma unroll
    for (int u = 0; u < KW; ++u) d[u] = levels[v * n_levels + (lev[u] >= 0 ? lev[u] : lev[0])];
    int4 st4[KW];
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        const int l = lev[u] >= 0 ? lev[u] : lev[0];
        const int start = __shfl(incl - cnt, l);
        const int rank = lev[u] >= 0 ? k0 + u - start : 0;
        st4[u] = stage[size_t(v) * n_features + d[u].kp_base + rank];
    }
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        x[u] = st4[u].x;
        y[u] = st4[u].y;
        R[u] = (long long)(((unsigned long long)(uint32_t)st4[u].w << 32) | (uint32_t)st4[u].z);
    }
    // disk moments: all rows' loads of both keypoints are issued before any is used (keypoints
    // lie kBorder > 16 pixels inside the level, so offsets up to 16 stay in bounds); the disk
    // x^2 + y^2 <= 225 is applied afterwards
    const int dx = (lane & 31) - 15;
    int I[KW][16];
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        const uint8_t* row = arena + d[u].offset + size_t(y[u] - 15 + (lane >> 5)) * d[u].pitch + x[u] + dx;
#pragma unroll
        for (int it = 0; it < 16; ++it) I[u][it] = row[size_t(2 * it) * d[u].pitch];
    }
    int bin[KW];
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        int m10 = 0, m01 = 0;
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int dy = -15 + 2 * it + (lane >> 5);
            const int val = (dy <= 15 && dx * dx + dy * dy <= 225) ? I[u][it] : 0;
            m10 += dx * val;
            m01 += dy * val;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            m10 += __shfl_xor(m10, off);
            m01 += __shfl_xor(m01, off);
        }
        long long sc = lane < 30 ? (long long)m10 * c_cos[lane] + (long long)m01 * c_sin[lane] : LLONG_MIN;
        int bk = lane;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const long long os = __shfl_xor(sc, off);
            const int ob = __shfl_xor(bk, off);
            if (os > sc || (os == sc && ob < bk)) { sc = os; bk = ob; }
        }
        bin[u] = bk;
    }
    // The smoothed 43 x 43 patch the steered tests read (offsets within +-21) is staged in LDS by
    // aligned 4-byte row loads: the tests' scattered byte reads would each touch a cache line of
    // their own.  (Issued together with the disk's loads instead, the registers they hold cost
    // more than the overlap gains.)
    // Columns a .. a + 47 with a = (x - 21) & ~3 >= 0 (x >= kBorder); the row past x + 21 stays
    // inside the level's padded row or runs into the next row (y + 21 < H - 1).
    constexpr int kPR = 2 * 21 + 1, kPW = 12;          // patch rows, 4-byte words per row
    __shared__ uint32_t patch[4][KW][kPR * kPW];
    const int wv = threadIdx.x >> 6;
    int a0[KW];
    {
        uint32_t w[KW][(kPR * kPW + 63) / 64];
#pragma unroll
        for (int u = 0; u < KW; ++u) {
            a0[u] = (x[u] - 21) & ~3;
            const uint8_t* base = smooth + d[u].offset + size_t(y[u] - 21) * d[u].pitch + a0[u];
#pragma unroll
            for (int it = 0; it < (kPR * kPW + 63) / 64; ++it) {
                const int e = it * 64 + lane, r = e / kPW, c = e - (e / kPW) * kPW;
                w[u][it] = e < kPR * kPW ? *reinterpret_cast<const uint32_t*>(base + size_t(r) * d[u].pitch + 4 * c) : 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < KW; ++u)
#pragma unroll
            for (int it = 0; it < (kPR * kPW + 63) / 64; ++it) {
                const int e = it * 64 + lane;
                if (e < kPR * kPW) patch[wv][u][e] = w[u][it];
            }
    }
    // the patch is written and read by this wave alone: order its LDS writes before the reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // tests g * 64 + lane steered by the bin (k_steer)
    uint32_t pk[KW][4];
#pragma unroll
    for (int u = 0; u < KW; ++u)
#pragma unroll
        for (int g = 0; g < 4; ++g) pk[u][g] = steer[bin[u] * kBriefTests + g * 64 + lane];
    bool bit[KW][4];
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        const uint8_t* P8 = reinterpret_cast<const uint8_t*>(patch[wv][u]);
        const int cx = x[u] - a0[u];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const uint32_t q = pk[u][g];
            const int ax = int(int8_t(q & 0xFF)), ay = int(int8_t((q >> 8) & 0xFF));
            const int bx = int(int8_t((q >> 16) & 0xFF)), by = int(int8_t(q >> 24));
            bit[u][g] = P8[(ay + 21) * (4 * kPW) + cx + ax] < P8[(by + 21) * (4 * kPW) + cx + bx];
        }
    }
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        unsigned long long words[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) words[g] = __ballot(bit[u][g]);
        if (lev[u] < 0) continue;
        const size_t slot = size_t(v) * n_features + k0 + u;
        if (lane < 4) reinterpret_cast<unsigned long long*>(desc + slot * XA_DESC_BYTES)[lane] = words[lane];
        if (lane == 0) {
#pragma clang fp contract(off)     // the back-map rounds term by term, as a plain fp64 evaluation
            const xa_view_desc& vd = views[v];
            const xa_level_desc& l0 = levels[v * n_levels];
            const double x0 = (double(x[u]) + 0.5) * (double(l0.width) / double(d[u].width)) - 0.5;
            const double y0 = (double(y[u]) + 0.5) * (double(l0.height) / double(d[u].height)) - 0.5;
            xa_keypoint o;
            o.x = x[u]; o.y = y[u]; o.level = lev[u]; o.bin = bin[u]; o.harris = R[u];
            o.xs = vd.inv[0] * x0 + vd.inv[1] * y0 + vd.inv[2];
            o.ys = vd.inv[3] * x0 + vd.inv[4] * y0 + vd.inv[5];
            if (vd.src_scale != 1.0) {     // scale-stage source: back to the original image
                o.xs = (o.xs + 0.5) / vd.src_scale - 0.5;
                o.ys = (o.ys + 0.5) / vd.src_scale - 0.5;
            }
            kp[slot] = o;
        }
    }
}

}  // namespace

xa_status launch_extract(const PlanView& ph, const PlanView& pd, uint8_t* arena, uint8_t* mask,
                         const int8_t* pattern, xa_keypoint* kp, uint8_t* desc, int32_t* count,
                         uint8_t* ws, hipStream_t st, int32_t* zero_extra, int n_extra) {
    const xa_plan_header* h = ph.h;
    const int nv = h->n_views, L = h->n_levels, nvl = nv * L, N = h->n_features;
    const ExtractWs w = extract_ws_layout(h);
    uint8_t* smooth = ws + w.smooth;
    Cand* cand = reinterpret_cast<Cand*>(ws + w.cand);
    int32_t* cand_count = reinterpret_cast<int32_t*>(ws + w.cand_count);
    int4* stage = reinterpret_cast<int4*>(ws + w.stage);
    int32_t* stage_count = reinterpret_cast<int32_t*>(ws + w.stage_count);
    uint32_t* steer = reinterpret_cast<uint32_t*>(ws + w.steer);
    if (!zero_extra) n_extra = 0;
    const int nz = std::max(nvl, n_extra);   // the candidate counters, and the caller's counts to clear
    hipLaunchKernelGGL(k_steer, dim3(kOrientBins + (nz + kBriefTests - 1) / kBriefTests), dim3(kBriefTests), 0, st,
                       pattern, steer, cand_count, nvl, zero_extra, n_extra);
    for (int l = 1; l < L; ++l) {
        const int32_t* pre_h = ph.level_prefix + size_t(l) * (nv + 1);
        const int tiles = pre_h[nv];
        if (tiles > 0)
            hipLaunchKernelGGL(k_pyr, dim3(tiles), dim3(256), 0, st, pd.levels, L, l,
                               pd.level_prefix + size_t(l) * (nv + 1), nv, arena, mask);
    }
    const int vt = ph.vl_prefix[nvl];
    if (vt > 0)
        hipLaunchKernelGGL(k_fast, dim3(vt), dim3(256), 0, st, pd.fast_flags, pd.levels, pd.vl_prefix, nvl,
                           h->fast_threshold, arena, mask, cand, cand_count, smooth);
    hipLaunchKernelGGL(k_select, dim3(nvl), dim3(kSelThreads), 0, st, pd.levels, N, cand, cand_count, stage,
                       stage_count);
    hipLaunchKernelGGL(k_orient_brief, dim3((N + 4 * kKpPerWave - 1) / (4 * kKpPerWave), nv), dim3(256), 0, st, pd.views, pd.levels, L, N, arena,
                       smooth, stage, stage_count, steer, kp, desc, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "extract launch");
    return XA_OK;
}

}  // namespace xa

using namespace xa;

extern "C" size_t xa_extract_workspace_size(const void* plan_host) {
    PlanView p;
    if (plan_host_view(plan_host, &p) != XA_OK) return 0;
    return extract_ws_layout(p.h).total;
}

extern "C" xa_status xa_extract_orb(const void* plan_host, const void* plan_dev, uint8_t* d_arena, uint8_t* d_mask,
                                    const int8_t* d_pattern, xa_keypoint* d_kp, uint8_t* d_desc, int32_t* d_count,
                                    void* d_ws, size_t ws_bytes, hipStream_t stream) {
    PlanView ph;
    xa_status s = plan_host_view(plan_host, &ph);
    if (s != XA_OK) return s;
    if (!plan_dev || !d_arena || !d_mask || !d_pattern || !d_kp || !d_desc || !d_count)
        return fail(XA_EINVAL, "NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(d_arena) | reinterpret_cast<uintptr_t>(d_mask)) % 128)
        return fail(XA_EINVAL, "arena and mask must be 128-byte aligned");
    const size_t need = extract_ws_layout(ph.h).total;
    if (ws_bytes < need) return fail(XA_ECAPACITY, "extract workspace needs %zu bytes, got %zu", need, ws_bytes);
    if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) % kAlign))
        return fail(XA_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    const PlanView pd = plan_dev_view(plan_host, plan_dev);
    s = launch_extract(ph, pd, d_arena, d_mask, d_pattern, d_kp, d_desc, d_count, static_cast<uint8_t*>(d_ws), stream);
    return s == XA_OK ? ok() : s;
}
