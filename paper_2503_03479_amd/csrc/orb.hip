// ORB on every simulated view, on gfx950: fixed-point pyramid, FAST-9 with 3x3
// non-maximum suppression and wave-ballot compaction, integer Harris response with
// per-level top-N selection, 7-tap integer smoothing, intensity-centroid
// orientation (30 bins) and rBRIEF-256 packed by wave ballots.  All arithmetic
// is integer, so the results are exact.
#include <hip/hip_runtime.h>

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

__device__ __forceinline__ int find_segment(const int32_t* __restrict__ prefix, int n, int b) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ pyramid

// Bilinear source position of destination index d for an n_src -> n_dst resize:
// src = (d + 1/2) n_src / n_dst - 1/2 in 1/2048 units, rounded half up, in exact
// unsigned arithmetic (1024 ((2d+1) n_src - n_dst) / n_dst split into quotient and remainder).
__device__ __forceinline__ void resample_index(int d, int n_dst, int n_src, int& i0, int& i1, int& w1) {
    const uint32_t A = uint32_t(2 * d + 1) * uint32_t(n_src) - uint32_t(n_dst);
    const uint32_t qa = A / uint32_t(n_dst);
    const uint32_t ra = A - qa * uint32_t(n_dst);
    const uint32_t q = 1024u * qa + (2048u * ra + uint32_t(n_dst)) / (2u * uint32_t(n_dst));
    int a = int(q >> 11), w = int(q & 2047u);
    if (a >= n_src - 1) { a = n_src - 1; w = 0; }
    i0 = a;
    w1 = w;
    i1 = a + 1 < n_src ? a + 1 : n_src - 1;
}

// Level l of every view from level l-1: (sum_{2x2} wy wx pix + 2^21) >> 22; the content
// mask of a level pixel is the AND over its 2x2 footprint.
__global__ void __launch_bounds__(256) k_pyr(const xa_level_desc* __restrict__ levels, int n_levels, int l,
                                             const int32_t* __restrict__ prefix, int n_views,
                                             uint8_t* __restrict__ arena, uint8_t* __restrict__ mask) {
    __shared__ int sx0[kPyrTX], sx1[kPyrTX], swx[kPyrTX];
    __shared__ int sy0[kPyrTY], sy1[kPyrTY], swy[kPyrTY];
    const int b = blockIdx.x;
    const int vi = find_segment(prefix, n_views, b);
    const xa_level_desc d = levels[vi * n_levels + l];
    const xa_level_desc p = levels[vi * n_levels + l - 1];
    const int local = b - prefix[vi];
    const int tiles_x = (d.width + kPyrTX - 1) / kPyrTX;
    const int x0 = (local % tiles_x) * kPyrTX, y0 = (local / tiles_x) * kPyrTY;
    const int t = threadIdx.x;
    if (t < kPyrTX) {
        if (x0 + t < d.width) resample_index(x0 + t, d.width, p.width, sx0[t], sx1[t], swx[t]);
    } else if (t < kPyrTX + kPyrTY) {
        const int r = t - kPyrTX;
        if (y0 + r < d.height) resample_index(y0 + r, d.height, p.height, sy0[r], sy1[r], swy[r]);
    }
    __syncthreads();
    const int tx = t % kPyrTX, ty = t / kPyrTX;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= d.width || y >= d.height) return;
    const uint8_t* P = arena + p.offset;
    const uint8_t* M = mask + p.offset;
    const int r0 = sy0[ty] * p.width, r1 = sy1[ty] * p.width;
    const int c0 = sx0[tx], c1 = sx1[tx];
    const int wx1 = swx[tx], wx0 = 2048 - wx1, wy1 = swy[ty], wy0 = 2048 - wy1;
    const int top = wx0 * int(P[r0 + c0]) + wx1 * int(P[r0 + c1]);
    const int bot = wx0 * int(P[r1 + c0]) + wx1 * int(P[r1 + c1]);
    const int out = (wy0 * top + wy1 * bot + (1 << 21)) >> 22;
    const size_t o = size_t(d.offset) + size_t(y) * d.width + x;
    arena[o] = uint8_t(out);
    mask[o] = uint8_t(M[r0 + c0] & M[r0 + c1] & M[r1 + c0] & M[r1 + c1]);
}

// ------------------------------------------------------------------ FAST-9 + NMS + compaction

// Bresenham circle of radius 3, clockwise from 12 o'clock (x right, y down).
__constant__ int8_t c_circle_x[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
__constant__ int8_t c_circle_y[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

// True iff the 16-bit circular mask has a run of at least 9 set bits.
__device__ __forceinline__ bool has_run9(uint32_t m) {
    const uint32_t x = m | (m << 16);
    uint32_t r = x & (x >> 1);
    r &= r >> 2;
    r &= r >> 4;
    r &= x >> 8;
    return (r & 0xFFFFu) != 0;
}

// FAST-9 score of the pixel at (cx, cy) of an LDS tile: V = max over the 16 arcs of 9
// contiguous circle pixels and both polarities of the arc minimum of the signed
// difference; returns kNegV unless V > T (i.e. unless the pixel is a corner).
__device__ __forceinline__ int fast_score_lds(const uint8_t* t, int stride, int cx, int cy, int T) {
    const int c = t[cy * stride + cx];
    int d[16];
    uint32_t bm = 0, dm = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        d[k] = int(t[(cy + c_circle_y[k]) * stride + cx + c_circle_x[k]]) - c;
        bm |= uint32_t(d[k] > T) << k;
        dm |= uint32_t(d[k] < -T) << k;
    }
    if (!has_run9(bm) && !has_run9(dm)) return kNegV;
    int best = INT_MIN;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        int mn = d[s], mx = d[s];
#pragma unroll
        for (int j = 1; j < 9; ++j) {
            const int v = d[(s + j) & 15];
            mn = min(mn, v);
            mx = max(mx, v);
        }
        best = max(best, max(mn, -mx));
    }
    return best;
}

constexpr int kFastHalo = 4;                                  // circle radius 3 + 1 for the NMS ring
constexpr int kFastLW = kFastTX + 2 * kFastHalo;              // 72
constexpr int kFastLH = kFastTY + 2 * kFastHalo;              // 16
constexpr int kScoreW = kFastTX + 2, kScoreH = kFastTY + 2;   // 66 x 10
constexpr int kSmRows = kFastTY + 6;                          // rows of horizontal smoothing sums

// One block per 64 x 8 tile of one (view, level), levels that can hold detections only:
//  1. the tile plus a 4-pixel halo is staged in LDS (border replicated);
//  2. the 7-tap smoothing [18 34 49 54 49 34 18] / 256 of the tile is written out
//     (exact horizontal sums, vertical pass (sum + 2^15) >> 16);
//  3. FAST-9 scores on the tile plus a one-pixel ring: an exact pre-test on the four
//     compass pixels (any 9-pixel arc contains two of them) queues the pixels that can be
//     corners, and only those get the full score;
//  4. 3x3 non-maximum suppression (ties to the earlier raster position), the content
//     filter on the corners of the +-B box, and ballot compaction of the survivors.
__global__ void __launch_bounds__(256) k_fast(const xa_level_desc* __restrict__ levels, const int32_t* __restrict__ prefix,
                                              int nvl, int T, const uint8_t* __restrict__ arena,
                                              const uint8_t* __restrict__ mask, uint32_t* __restrict__ cand,
                                              int32_t* __restrict__ cand_count, uint8_t* __restrict__ smooth) {
    __shared__ uint8_t img[kFastLH * kFastLW];
    __shared__ int score[kScoreH * kScoreW];
    __shared__ int hs[kSmRows * kFastTX];
    __shared__ int16_t queue[kScoreH * kScoreW];
    __shared__ int qn;
    const int b = blockIdx.x;
    const int vl = find_segment(prefix, nvl, b);
    const xa_level_desc d = levels[vl];
    if (d.cand_cap == 0) return;
    const int W = d.width, H = d.height;
    const int local = b - prefix[vl];
    const int tiles_x = (W + kFastTX - 1) / kFastTX;
    const int x0 = (local % tiles_x) * kFastTX, y0 = (local / tiles_x) * kFastTY;
    const uint8_t* P = arena + d.offset;
    for (int e = threadIdx.x; e < kFastLH * kFastLW; e += 256) {
        const int ly = e / kFastLW, lx = e - (e / kFastLW) * kFastLW;
        const int gx = clampi(x0 - kFastHalo + lx, 0, W - 1), gy = clampi(y0 - kFastHalo + ly, 0, H - 1);
        img[e] = P[size_t(gy) * W + gx];
    }
    if (threadIdx.x == 0) qn = 0;
    __syncthreads();
    // smoothing: horizontal sums for rows y0-3 .. y0+10, then the vertical pass
    const int w7[7] = {18, 34, 49, 54, 49, 34, 18};
    for (int e = threadIdx.x; e < kSmRows * kFastTX; e += 256) {
        const int r = e / kFastTX, c = e - (e / kFastTX) * kFastTX;
        const uint8_t* row = img + (r + 1) * kFastLW + c + 1;
        int sum = 0;
#pragma unroll
        for (int k = 0; k < 7; ++k) sum += w7[k] * int(row[k]);
        hs[e] = sum;
    }
    // FAST pre-test over the tile and its ring; positions that cannot be compared stay non-corners
    const bool detect = !(x0 + kFastTX <= kBorder || x0 >= W - kBorder || y0 + kFastTY <= kBorder || y0 >= H - kBorder);
    if (detect) {
        for (int e = threadIdx.x; e < kScoreH * kScoreW; e += 256) {
            const int sy = e / kScoreW, sx = e - (e / kScoreW) * kScoreW;
            const int gx = x0 - 1 + sx, gy = y0 - 1 + sy;
            score[e] = kNegV;
            if (gx >= kBorder - 1 && gx <= W - kBorder && gy >= kBorder - 1 && gy <= H - kBorder) {
                const uint8_t* p = img + (sy + kFastHalo - 1) * kFastLW + sx + kFastHalo - 1;
                const int c = p[0];
                const int n = p[-3 * kFastLW], e3 = p[3], s3 = p[3 * kFastLW], w3 = p[-3];
                const int nb = (n > c + T) + (e3 > c + T) + (s3 > c + T) + (w3 > c + T);
                const int nd = (n < c - T) + (e3 < c - T) + (s3 < c - T) + (w3 < c - T);
                if (nb >= 2 || nd >= 2) queue[atomicAdd(&qn, 1)] = int16_t(e);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < kFastTY / 4; ++rr) {
        const int tx = threadIdx.x % kFastTX, ty = threadIdx.x / kFastTX + 4 * rr;
        const int x = x0 + tx, y = y0 + ty;
        if (x < W && y < H) {
            int sum = 0;
#pragma unroll
            for (int k = 0; k < 7; ++k) sum += w7[k] * hs[(ty + k) * kFastTX + tx];
            smooth[size_t(d.offset) + size_t(y) * W + x] = uint8_t((sum + (1 << 15)) >> 16);
        }
    }
    if (!detect) return;
    const int nq = qn;
    for (int q = threadIdx.x; q < nq; q += 256) {
        const int e = queue[q];
        const int sy = e / kScoreW, sx = e - (e / kScoreW) * kScoreW;
        score[e] = fast_score_lds(img, kFastLW, sx + kFastHalo - 1, sy + kFastHalo - 1, T);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint8_t* M = mask + d.offset;
#pragma unroll
    for (int rr = 0; rr < kFastTY / 4; ++rr) {
        const int tx = threadIdx.x % kFastTX, ty = threadIdx.x / kFastTX + 4 * rr;
        const int x = x0 + tx, y = y0 + ty;
        bool keep = false;
        if (x >= kBorder && x < W - kBorder && y >= kBorder && y < H - kBorder) {
            const int vp = score[(ty + 1) * kScoreW + tx + 1];
            if (vp > T) {
                keep = true;
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (dx == 0 && dy == 0) continue;
                        const int vq = score[(ty + 1 + dy) * kScoreW + tx + 1 + dx];
                        const bool q_after = dy > 0 || (dy == 0 && dx > 0);
                        keep = keep && (vp > vq || (vp == vq && q_after));
                    }
                if (keep) {
                    const size_t r0 = size_t(y - kBorder) * W, r1 = size_t(y + kBorder) * W;
                    keep = M[r0 + x - kBorder] && M[r0 + x + kBorder] && M[r1 + x - kBorder] && M[r1 + x + kBorder];
                }
            }
        }
        const unsigned long long bal = __ballot(keep);
        if (bal) {
            const int n = __popcll(bal);
            int base = 0;
            if (lane == 0) base = atomicAdd(&cand_count[vl], n);
            base = __shfl(base, 0);
            const int pos = __popcll(bal & ((1ull << lane) - 1ull));
            if (keep && base + pos < d.cand_cap) cand[d.cand_offset + base + pos] = uint32_t(y) * uint32_t(W) + uint32_t(x);
        }
    }
}

// ------------------------------------------------------------------ Harris + top-N per level

__device__ __forceinline__ long long harris_at(const uint8_t* __restrict__ P, int W, int x, int y) {
    int a = 0, b = 0, c = 0;
    for (int dy = -3; dy <= 3; ++dy) {
        const uint8_t* r0 = P + size_t(y + dy - 1) * W + x;
        const uint8_t* r1 = r0 + W;
        const uint8_t* r2 = r1 + W;
#pragma unroll
        for (int dx = -3; dx <= 3; ++dx) {
            const int ix = (int(r0[dx + 1]) + 2 * int(r1[dx + 1]) + int(r2[dx + 1])) -
                           (int(r0[dx - 1]) + 2 * int(r1[dx - 1]) + int(r2[dx - 1]));
            const int iy = (int(r2[dx - 1]) + 2 * int(r2[dx]) + int(r2[dx + 1])) -
                           (int(r0[dx - 1]) + 2 * int(r0[dx]) + int(r0[dx + 1]));
            a += ix * ix;
            b += iy * iy;
            c += ix * iy;
        }
    }
    const long long tr = (long long)(a + b);
    return 25LL * ((long long)a * b - (long long)c * c) - tr * tr;
}

// order-preserving map int64 -> uint64
__device__ __forceinline__ unsigned long long okey(long long r) { return (unsigned long long)r ^ 0x8000000000000000ull; }

// k-th largest (descending = true) or k-th smallest value among the items i < C whose
// `pred` holds, by 8-bit digit histograms from the top digit down; returns the value and
// leaves in *k_rem how many items equal to it are needed to make k.
template <typename Get, typename Pred>
__device__ unsigned long long radix_select(int C, int k, int top_bit, bool descending, Get get, Pred pred,
                                           int* hist, int* k_rem, int* s_digit, int* s_k) {
    unsigned long long prefix = 0, pmask = 0;
    for (int shift = top_bit - 7; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < C; i += blockDim.x) {
            if (!pred(i)) continue;
            const unsigned long long u = get(i);
            if ((u & pmask) != prefix) continue;
            atomicAdd(&hist[(u >> shift) & 0xFF], 1);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0, g = 0;
            for (int s = 0; s < 256; ++s) {
                g = descending ? 255 - s : s;
                if (acc + hist[g] >= k) break;
                acc += hist[g];
            }
            *s_digit = g;
            *s_k = k - acc;
        }
        __syncthreads();
        prefix |= (unsigned long long)(*s_digit) << shift;
        pmask |= 0xFFull << shift;
        k = *s_k;
        __syncthreads();
    }
    *k_rem = k;
    return prefix;
}

// One block per (view, level): Harris at every candidate, then the top `quota` by
// (response descending, raster ascending), sorted in that order, into the staging slots.
__global__ void __launch_bounds__(kSelThreads) k_select(const xa_level_desc* __restrict__ levels, int n_features,
                                                        const uint8_t* __restrict__ arena, const uint32_t* __restrict__ cand,
                                                        const int32_t* __restrict__ cand_count,
                                                        long long* __restrict__ harris, int4* __restrict__ stage,
                                                        int32_t* __restrict__ stage_count) {
    __shared__ unsigned long long s_key[kSelMax];
    __shared__ uint32_t s_ras[kSelMax];
    __shared__ int hist[256];
    __shared__ int s_digit, s_k, s_n;
    const int vl = blockIdx.x;
    const xa_level_desc d = levels[vl];
    const int C = int(min((long long)cand_count[vl], (long long)d.cand_cap));
    const int quota = d.quota;
    const uint8_t* P = arena + d.offset;
    const uint32_t* cd = cand + d.cand_offset;
    long long* hr = harris + d.cand_offset;
    for (int i = threadIdx.x; i < C; i += blockDim.x) {
        const uint32_t r = cd[i];
        hr[i] = harris_at(P, d.width, int(r % uint32_t(d.width)), int(r / uint32_t(d.width)));
    }
    __syncthreads();
    const int n = min(C, quota);
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    if (C <= quota) {
        for (int i = threadIdx.x; i < C; i += blockDim.x) {
            const int slot = atomicAdd(&s_n, 1);
            s_key[slot] = okey(hr[i]);
            s_ras[slot] = cd[i];
        }
    } else if (n > 0) {
        int k_eq;
        const unsigned long long K = radix_select(
            C, n, 63, true, [&](int i) { return okey(hr[i]); }, [](int) { return true; }, hist, &k_eq, &s_digit, &s_k);
        // among the candidates with response exactly K, the k_eq smallest raster positions
        int k_r;
        const unsigned long long Rthr = radix_select(
            C, k_eq, 31, false, [&](int i) { return (unsigned long long)cd[i]; },
            [&](int i) { return okey(hr[i]) == K; }, hist, &k_r, &s_digit, &s_k);
        for (int i = threadIdx.x; i < C; i += blockDim.x) {
            const unsigned long long u = okey(hr[i]);
            if (u > K || (u == K && cd[i] <= Rthr)) {
                const int slot = atomicAdd(&s_n, 1);
                s_key[slot] = u;
                s_ras[slot] = cd[i];
            }
        }
    }
    __syncthreads();
    // bitonic sort of n entries padded to a power of two: key descending, raster ascending
    int M = 1;
    while (M < n) M <<= 1;
    for (int i = n + threadIdx.x; i < M; i += blockDim.x) {
        s_key[i] = 0ull;
        s_ras[i] = 0xFFFFFFFFu;
    }
    __syncthreads();
    for (int k = 2; k <= M; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < M; i += blockDim.x) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const unsigned long long ka = s_key[i], kb = s_key[ixj];
                    const uint32_t ra = s_ras[i], rb = s_ras[ixj];
                    const bool a_first = ka > kb || (ka == kb && ra < rb);
                    const bool up = (i & k) == 0;
                    if (up != a_first) {
                        s_key[i] = kb; s_key[ixj] = ka;
                        s_ras[i] = rb; s_ras[ixj] = ra;
                    }
                }
            }
            __syncthreads();
        }
    }
    int4* st = stage + size_t(d.view) * n_features + d.kp_base;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t r = s_ras[i];
        const long long R = (long long)(s_key[i] ^ 0x8000000000000000ull);
        st[i] = make_int4(int(r % uint32_t(d.width)), int(r / uint32_t(d.width)), int(uint32_t(R & 0xFFFFFFFFll)),
                          int(R >> 32));
    }
    if (threadIdx.x == 0) stage_count[vl] = n;
}

// ------------------------------------------------------------------ orientation + rBRIEF

__device__ __forceinline__ int rnd20(int v) {
    const int a = v < 0 ? -v : v;
    const int r = (a + (1 << 19)) >> 20;
    return v < 0 ? -r : r;
}

// One wave per keypoint: intensity-centroid moments over the radius-15 disk, integer
// argmax over the 30 bins, then 256 steered binary tests on the smoothed level,
// packed four 64-bit ballots at a time.  Keypoints are written in canonical order.
__global__ void __launch_bounds__(256) k_orient_brief(const xa_view_desc* __restrict__ views,
                                                      const xa_level_desc* __restrict__ levels, int n_levels,
                                                      int n_features, const uint8_t* __restrict__ arena,
                                                      const uint8_t* __restrict__ smooth, const int4* __restrict__ stage,
                                                      const int32_t* __restrict__ stage_count,
                                                      const int8_t* __restrict__ pattern, xa_keypoint* __restrict__ kp,
                                                      uint8_t* __restrict__ desc, int32_t* __restrict__ count) {
    const int v = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    int pre = 0, lev = -1, rank = 0;
    for (int l = 0; l < n_levels; ++l) {
        const int c = stage_count[v * n_levels + l];
        if (lev < 0 && k < pre + c) { lev = l; rank = k - pre; }
        pre += c;
    }
    if (k == 0 && lane == 0) count[v] = pre;
    if (lev < 0) return;
    const xa_level_desc d = levels[v * n_levels + lev];
    const int4 s = stage[size_t(v) * n_features + d.kp_base + rank];
    const int x = s.x, y = s.y;
    const long long R = (long long)(((unsigned long long)(uint32_t)s.w << 32) | (uint32_t)s.z);
    const int W = d.width;
    const uint8_t* P = arena + d.offset;
    int m10 = 0, m01 = 0;
    {
        const int dx = (lane & 31) - 15;
        for (int it = 0; it < 16; ++it) {
            const int dy = -15 + 2 * it + (lane >> 5);
            if (dy <= 15 && dx * dx + dy * dy <= 225) {
                const int I = P[size_t(y + dy) * W + x + dx];
                m10 += dx * I;
                m01 += dy * I;
            }
        }
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
    const int bin = bk;
    const int Cb = c_cos[bin], Sb = c_sin[bin];
    const uint8_t* Sm = smooth + d.offset;
    unsigned long long words[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int i = g * 64 + lane;
        // pattern coordinates are clamped to the documented [-15, 15], so every test stays inside the border
        const int x1 = clampi(pattern[4 * i], -15, 15), y1 = clampi(pattern[4 * i + 1], -15, 15);
        const int x2 = clampi(pattern[4 * i + 2], -15, 15), y2 = clampi(pattern[4 * i + 3], -15, 15);
        const int ax = rnd20(x1 * Cb - y1 * Sb), ay = rnd20(x1 * Sb + y1 * Cb);
        const int bx = rnd20(x2 * Cb - y2 * Sb), by = rnd20(x2 * Sb + y2 * Cb);
        const bool bit = Sm[size_t(y + ay) * W + x + ax] < Sm[size_t(y + by) * W + x + bx];
        words[g] = __ballot(bit);
    }
    const size_t slot = size_t(v) * n_features + k;
    if (lane < 4) reinterpret_cast<unsigned long long*>(desc + slot * XA_DESC_BYTES)[lane] = words[lane];
    if (lane == 0) {
        const xa_view_desc& vd = views[v];
        const xa_level_desc& l0 = levels[v * n_levels];
        const double x0 = __dadd_rn(__dmul_rn(__dadd_rn(double(x), 0.5), double(l0.width) / double(W)), -0.5);
        const double y0 = __dadd_rn(__dmul_rn(__dadd_rn(double(y), 0.5), double(l0.height) / double(d.height)), -0.5);
        xa_keypoint o;
        o.x = x; o.y = y; o.level = lev; o.bin = bin; o.harris = R;
        o.xs = __dadd_rn(__dadd_rn(__dmul_rn(vd.inv[0], x0), __dmul_rn(vd.inv[1], y0)), vd.inv[2]);
        o.ys = __dadd_rn(__dadd_rn(__dmul_rn(vd.inv[3], x0), __dmul_rn(vd.inv[4], y0)), vd.inv[5]);
        kp[slot] = o;
    }
}

}  // namespace

xa_status launch_extract(const PlanView& ph, const PlanView& pd, uint8_t* arena, uint8_t* mask,
                         const int8_t* pattern, xa_keypoint* kp, uint8_t* desc, int32_t* count,
                         uint8_t* ws, hipStream_t st) {
    const xa_plan_header* h = ph.h;
    const int nv = h->n_views, L = h->n_levels, nvl = nv * L, N = h->n_features;
    const ExtractWs w = extract_ws_layout(h);
    uint8_t* smooth = ws + w.smooth;
    uint32_t* cand = reinterpret_cast<uint32_t*>(ws + w.cand);
    int32_t* cand_count = reinterpret_cast<int32_t*>(ws + w.cand_count);
    long long* harris = reinterpret_cast<long long*>(ws + w.harris);
    int4* stage = reinterpret_cast<int4*>(ws + w.stage);
    int32_t* stage_count = reinterpret_cast<int32_t*>(ws + w.stage_count);
    hipLaunchKernelGGL(k_fill_i32, dim3((nvl + 255) / 256), dim3(256), 0, st, cand_count, nvl, 0);
    for (int l = 1; l < L; ++l) {
        const int32_t* pre_h = ph.level_prefix + size_t(l) * (nv + 1);
        const int tiles = pre_h[nv];
        if (tiles > 0)
            hipLaunchKernelGGL(k_pyr, dim3(tiles), dim3(256), 0, st, pd.levels, L, l,
                               pd.level_prefix + size_t(l) * (nv + 1), nv, arena, mask);
    }
    const int vt = ph.vl_prefix[nvl];
    if (vt > 0) {
        hipLaunchKernelGGL(k_fast, dim3(vt), dim3(256), 0, st, pd.levels, pd.vl_prefix, nvl, h->fast_threshold,
                           arena, mask, cand, cand_count, smooth);
    }
    hipLaunchKernelGGL(k_select, dim3(nvl), dim3(kSelThreads), 0, st, pd.levels, N, arena, cand, cand_count, harris,
                       stage, stage_count);
    hipLaunchKernelGGL(k_orient_brief, dim3((N + 3) / 4, nv), dim3(256), 0, st, pd.views, pd.levels, L, N, arena,
                       smooth, stage, stage_count, pattern, kp, desc, count);
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
    const size_t need = extract_ws_layout(ph.h).total;
    if (ws_bytes < need) return fail(XA_ECAPACITY, "extract workspace needs %zu bytes, got %zu", need, ws_bytes);
    if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) % kAlign))
        return fail(XA_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    const PlanView pd = plan_dev_view(plan_host, plan_dev);
    s = launch_extract(ph, pd, d_arena, d_mask, d_pattern, d_kp, d_desc, d_count, static_cast<uint8_t*>(d_ws), stream);
    return s == XA_OK ? ok() : s;
}
