// View simulation on gfx950: anti-alias blur along the tilt direction and
// Lanczos-4 affine resampling (eqs. (3)-(4), 8x8 window per Sec. IV.C).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"
#include "lanczos.h"

namespace xa {
namespace {

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
        const int k = 63 - __clzll(bal);
        lo = lo + k * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// Source region a blur tile reads: the 64 x 16 tile grown by the tap offsets.  Taps step
// one pixel along the major axis (k = -K..K) and floor(k m) (+1 for the interpolation
// partner) along the minor axis, and floor(k m) is monotonic in k.
struct BlurRegion {
    int rx0, ry0, rw, rh, stride, floats;
};
__host__ __device__ inline BlurRegion blur_region(const xa_view_desc& v, const BlurTap* tp, int x0, int y0) {
    const int n = v.blur_ntaps, K = (n - 1) / 2;
    const int dlo = min(tp[0].dmin, tp[n - 1].dmin), dhi = max(tp[0].dmin, tp[n - 1].dmin) + 1;
    const int tw = blur_tile_w(v.blur_major, v.blur_rows), th = blur_tile_h(v.blur_major, v.blur_rows);
    BlurRegion r;
    if (v.blur_major == 0) {
        r.rx0 = x0 - K; r.rw = tw + 2 * K;
        r.ry0 = y0 + dlo; r.rh = th + dhi - dlo;
        r.stride = kBlurStride;           // the interpolation partner is one row down: a fixed offset
    } else {
        r.rx0 = x0 + dlo; r.rw = tw + dhi - dlo;
        r.ry0 = y0 - K; r.rh = th + 2 * K;
        r.stride = r.rw | 1;              // the partner is the next column; odd stride spreads rows over banks
    }
    r.floats = (v.blur_major == 0 && r.rw > kBlurStride) ? (1 << 30) : r.stride * r.rh;
    return r;
}

// The outputs of one blur tile from its staged footprint: each thread makes R outputs adjacent
// across the minor axis (rows for taps along x, columns for taps along y); tap k of them reads
// R + 1 consecutive minor samples, and each output keeps the same sum order as a one-output
// evaluation.
template <int R>
__device__ __forceinline__ void blur_outputs(const float* __restrict__ btile, const BlurRegion& g, const xa_view_desc& v,
                                             const BlurTap* __restrict__ tp, int n, int x0, int y0, int W, int H,
                                             float* __restrict__ o) {
    const int n4 = (n + 3) & ~3;           // the tap table is padded with zero taps to a multiple of 4
    const int bp = blur_pitch(W);
    float a[R];
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = 0.0f;
    if (v.blur_major == 0) {
        const int c = threadIdx.x & 63, gq = threadIdx.x >> 6;        // column, group of R rows
        const int x = x0 + c, y = y0 + R * gq;
        if (x < W && y < H) {
            constexpr int S = kBlurStride;
            const float* base = btile + (y - g.ry0) * S + (x - g.rx0);
            for (int k = 0; k < n4; k += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const BlurTap t = tp[k + u];
                    const float* q = base + t.dmin * S + t.dmaj;
                    float r[R + 1];
#pragma unroll
                    for (int i = 0; i <= R; ++i) r[i] = q[i * S];
#pragma unroll
                    for (int i = 0; i < R; ++i) a[i] = fmaf(t.wb, r[i + 1], fmaf(t.wa, r[i], a[i]));
                }
            }
            float* op = o + size_t(y) * bp + x;
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (y + i < H) op[size_t(i) * bp] = a[i];
        }
    } else {
        const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;         // row, group of R columns
        const int x = x0 + R * cg, y = y0 + r;
        if (x < W && y < H) {
            const float* base = btile + (y - g.ry0) * g.stride + (x - g.rx0);
            for (int k = 0; k < n4; k += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const BlurTap t = tp[k + u];
                    const float* q = base + t.dmaj * g.stride + t.dmin;
                    float rr[R + 1];
#pragma unroll
                    for (int i = 0; i <= R; ++i) rr[i] = q[i];
#pragma unroll
                    for (int i = 0; i < R; ++i) a[i] = fmaf(t.wb, rr[i + 1], fmaf(t.wa, rr[i], a[i]));
                }
            }
            float* op = o + size_t(y) * bp + x;
#pragma unroll
            for (int i = 0; i < R; i += 4) {
                if (x + i + 3 < W) {
                    *reinterpret_cast<float4*>(op + i) = make_float4(a[i], a[i + 1], a[i + 2], a[i + 3]);   // x + i and bp are multiples of 4
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (x + i + e < W) op[i + e] = a[i + e];
                }
            }
        }
    }
}

// Directional Gaussian over the source, one block per 64 x 4R tile of one blurred view (4R x 64
// when the taps step along y; R = blur_rows, 4 or 8).
// out(p) = sum_k w_k lerp(I, p + k v), v = (1, m) (major x) or (m, 1) (major y), written as
// sum_k wa_k I(p + k v_whole) + wb_k I(p + k v_whole + e_minor).  The tile's source footprint
// is staged in LDS as fp32 with the border replicated at load time (the same as clamping
// each tap), so each tap is one paired LDS read and two FMAs.
__global__ void __launch_bounds__(256) k_blur(const uint8_t* __restrict__ sources,
                                              const xa_view_desc* __restrict__ views,
                                              const int32_t* __restrict__ blur_views,
                                              const int32_t* __restrict__ blur_prefix, int n_blur,
                                              const BlurTap* __restrict__ taps, float* __restrict__ out,
                                              int lds_floats) {
    extern __shared__ float btile[];
    const int bi = find_segment_wave(blur_prefix, n_blur, blockIdx.x);
    const xa_view_desc& v = views[blur_views[bi]];
    const int W = v.src_w, H = v.src_h, pitch = v.src_pitch;
    const uint8_t* src = sources + v.src_offset;
    const int local = blockIdx.x - blur_prefix[bi];
    const int btw = blur_tile_w(v.blur_major, v.blur_rows), bth = blur_tile_h(v.blur_major, v.blur_rows);
    const int tiles_x = (W + btw - 1) / btw;
    const int x0 = (local % tiles_x) * btw, y0 = (local / tiles_x) * bth;
    const int tx = threadIdx.x % btw, ty0 = threadIdx.x / btw;
    const BlurTap* tp = taps + v.blur_tap0;
    const int n = v.blur_ntaps;
    const BlurRegion g = blur_region(v, tp, x0, y0);
    float* o = out + v.blur_offset;
    if (g.floats <= lds_floats) {
        if (((reinterpret_cast<uintptr_t>(src) | uintptr_t(pitch)) & 3) == 0) {
            // 4-byte-aligned sources: the footprint's rows are read as aligned words (columns
            // ax0 + 4 j .. + 3), 4 per thread before any is stored; words that leave the image are
            // assembled byte by byte with the border replicated, and columns outside the footprint
            // are dropped.  r = e / nw through a float reciprocal is exact for e < 2^14.
            const int ax0 = g.rx0 & ~3;
            const int nw = ((g.rx0 + g.rw - 1 - ax0) >> 2) + 1;
            const int n_w = nw * g.rh;
            const float rnw = 1.0f / float(nw);
            for (int e0 = 0; e0 < n_w; e0 += 4 * 256) {
                uint32_t wv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * 256 + int(threadIdx.x);
                    const int r = int((float(e) + 0.5f) * rnw), j = e - r * nw;
                    const int gx = ax0 + 4 * j;
                    const uint8_t* row = src + size_t(clampi(g.ry0 + r, 0, H - 1)) * pitch;
                    if (e < n_w) {
                        if (gx >= 0 && gx + 3 < W) {
                            wv[u] = *reinterpret_cast<const uint32_t*>(row + gx);
                        } else {
                            wv[u] = 0;
#pragma unroll
                            for (int b = 0; b < 4; ++b) wv[u] |= uint32_t(row[clampi(gx + b, 0, W - 1)]) << (8 * b);
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * 256 + int(threadIdx.x);
                    const int r = int((float(e) + 0.5f) * rnw), j = e - r * nw;
                    const int c0 = ax0 + 4 * j - g.rx0;
                    if (e < n_w) {
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            if (c0 + b >= 0 && c0 + b < g.rw) btile[r * g.stride + c0 + b] = float((wv[u] >> (8 * b)) & 0xFFu);
                    }
                }
            }
        } else {
            // loads are issued 8 per thread before any is stored, so their latencies overlap;
            // r = e / rw through a float reciprocal is exact for e < 2^14 (see the warp's staging)
            const int n_el = g.rw * g.rh;
            const float rrw = 1.0f / float(g.rw);
            for (int e0 = 0; e0 < n_el; e0 += 8 * 256) {
                float val[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * 256 + int(threadIdx.x);
                    const int r = int((float(e) + 0.5f) * rrw), c = e - r * g.rw;
                    if (e < n_el) val[u] = float(src[size_t(clampi(g.ry0 + r, 0, H - 1)) * pitch + clampi(g.rx0 + c, 0, W - 1)]);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * 256 + int(threadIdx.x);
                    const int r = int((float(e) + 0.5f) * rrw), c = e - r * g.rw;
                    if (e < n_el) btile[r * g.stride + c] = val[u];
                }
            }
        }
        __syncthreads();
        if (v.blur_rows == 4) blur_outputs<4>(btile, g, v, tp, n, x0, y0, W, H, o);
        else blur_outputs<8>(btile, g, v, tp, n, x0, y0, W, H, o);
        return;
    }
    // footprint larger than the LDS tile (very large sigma): read the taps from global memory
    for (int j = 0; j < (btw * bth) / 256; ++j) {
        const int x = x0 + tx, y = y0 + ty0 + (256 / btw) * j;
        if (x >= W || y >= H) continue;
        float acc = 0.0f;
        if (v.blur_major == 0) {
            for (int k = 0; k < n; ++k) {
                const BlurTap t = tp[k];
                const int xk = clampi(x + t.dmaj, 0, W - 1);
                const int yk = y + t.dmin;
                const float a = float(src[size_t(clampi(yk, 0, H - 1)) * pitch + xk]);
                const float b = float(src[size_t(clampi(yk + 1, 0, H - 1)) * pitch + xk]);
                acc += t.wa * a + t.wb * b;
            }
        } else {
            for (int k = 0; k < n; ++k) {
                const BlurTap t = tp[k];
                const uint8_t* row = src + size_t(clampi(y + t.dmaj, 0, H - 1)) * pitch;
                const int xk = x + t.dmin;
                const float a = float(row[clampi(xk, 0, W - 1)]);
                const float b = float(row[clampi(xk + 1, 0, W - 1)]);
                acc += t.wa * a + t.wb * b;
            }
        }
        o[size_t(y) * blur_pitch(W) + x] = acc;
    }
}

// Source coordinate of a view pixel, evaluated term by term in fp64 without contraction
// (the same rounding as a plain left-to-right evaluation of inv * q; device code is otherwise
// built with multiply-adds fused, so the operators stand under a pragma that keeps them apart).
__device__ __forceinline__ double affine_x(const double* m, double qx, double qy) {
#pragma clang fp contract(off)
    return m[0] * qx + m[1] * qy + m[2];
}

// 8 x 8 Lanczos sum of eq. (3) with normalised weights; row(j) returns a pointer such
// that row(j)[c] is the source sample at clamped column c of clamped row iy - 3 + j.
template <typename Row>
__device__ __forceinline__ float lanczos_sum(Row row, const int cols[8], const float wx[8], const float wy[8]) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const auto* r = row(j);
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < 8; ++i) s += wx[i] * float(r[cols[i]]);
        acc += wy[j] * s;
    }
    return acc;
}

// One block per 512-pixel output tile (w x 512/w, w per view), two pixels per thread, so
// that the block's serial chain (prefix search, view descriptor, footprint staging, barrier)
// is paid once per 512 pixels; all views of the plan in one launch (block -> view by prefix
// search).  The tile's source
// footprint (bounding box of its pixel centres mapped through inv, grown by the 8-tap
// window) is staged in LDS as fp32 when it fits; otherwise taps are read from global memory.
__global__ void __launch_bounds__(kWarpThreads) k_warp(const uint8_t* __restrict__ sources,
                                                       const float* __restrict__ blurred,
                                                       const xa_view_desc* __restrict__ views, int n_views,
                                                       const int32_t* __restrict__ prefix, uint8_t* __restrict__ arena,
                                                       uint8_t* __restrict__ mask, float* __restrict__ values) {
    __shared__ float tile[kWarpLds];
    const int b = xcd_contiguous(blockIdx.x, gridDim.x);
    const int vi = find_segment_wave(prefix, n_views, b);
    const xa_view_desc& v = views[vi];
    const int W = v.src_w, H = v.src_h, pitch = v.src_pitch;
    const uint8_t* src = sources + v.src_offset;
    const int local = b - prefix[vi];
    const int tw = v.warp_tile_w, th = kWarpRows * kWarpThreads / tw;
    const int tiles_x = (v.width + tw - 1) / tw;
    const int x0 = (local % tiles_x) * tw, y0 = (local / tiles_x) * th;
    if (v.interp == XA_INTERP_NEAREST) {
        // nearest neighbour (the search-time interpolation of Sec. III): one read per pixel,
        // the source pixel floor(p + 1/2) per axis, clamped; nothing is staged
        const float* nsrc = blurred + (v.blur_offset >= 0 ? v.blur_offset : 0);
        const int qx = x0 + int(threadIdx.x) % tw;
        for (int k = 0; k < kWarpRows; ++k) {
            const int qy = y0 + int(threadIdx.x) / tw + k * (kWarpThreads / tw);
            if (qx >= v.width || qy >= v.height) break;
            const size_t o = size_t(v.offset) + size_t(qy) * v.pitch + qx;
            const double px = affine_x(v.inv, double(qx), double(qy));
            const double py = affine_x(v.inv + 3, double(qx), double(qy));
            if (!(px >= -0.5 && px <= W - 0.5 && py >= -0.5 && py <= H - 0.5)) {
                arena[o] = 0;
                mask[o] = 0;
                if (values) values[o] = 0.0f;
                continue;
            }
            const int ix = clampi(int(floor(px + 0.5)), 0, W - 1), iy = clampi(int(floor(py + 0.5)), 0, H - 1);
            const float val = v.blur_offset >= 0 ? nsrc[size_t(iy) * blur_pitch(W) + ix]
                                                 : float(src[size_t(iy) * pitch + ix]);
            const float q = rintf(val);
            arena[o] = uint8_t(q < 0.0f ? 0.0f : (q > 255.0f ? 255.0f : q));
            mask[o] = 1;
            if (values) values[o] = val;
        }
        return;
    }
    // bounding box of the footprint (the tile's pixel centres through inv, grown by the
    // 8-tap window, clamped to the source): the corner (x0, y0) plus the extreme offsets of
    // the other corners; rounding here is ~1e-12 px, far inside the 1e-6 margin
    const double ox = v.inv[0] * double(tw - 1), oy = v.inv[1] * double(th - 1);
    const double o2x = v.inv[3] * double(tw - 1), o2y = v.inv[4] * double(th - 1);
    const double cx0 = affine_x(v.inv, double(x0), double(y0)), cy0 = affine_x(v.inv + 3, double(x0), double(y0));
    const double pxl = cx0 + fmin(ox, 0.0) + fmin(oy, 0.0), pxh = cx0 + fmax(ox, 0.0) + fmax(oy, 0.0);
    const double pyl = cy0 + fmin(o2x, 0.0) + fmin(o2y, 0.0), pyh = cy0 + fmax(o2x, 0.0) + fmax(o2y, 0.0);
    const int bx0 = max(int(fmax(floor(pxl - 1e-6), -1e9)) - 3, 0);
    const int bx1 = min(int(fmin(floor(pxh + 1e-6), 1e9)) + 4, W - 1);
    const int by0 = max(int(fmax(floor(pyl - 1e-6), -1e9)) - 3, 0);
    const int by1 = min(int(fmin(floor(pyh + 1e-6), 1e9)) + 4, H - 1);
    const int bh = by1 - by0 + 1;
    const bool blur = v.blur_offset >= 0;
    const float* bsrc = blurred + (blur ? v.blur_offset : 0);
    const int bp = blur_pitch(W);
    // staged columns start at a multiple of 4 so that rows load in 16-byte (blurred) or
    // 4-byte (u8) chunks; u8 sources whose rows are not 4-byte aligned load byte by byte
    const bool vec = blur || (((reinterpret_cast<uintptr_t>(src)) | uintptr_t(pitch)) & 3) == 0;
    const int ax0 = vec ? (bx0 & ~3) : bx0;
    const int nc = vec ? ((bx1 - ax0) >> 2) + 1 : bx1 - bx0 + 1;      // chunks per row
    const int cw = vec ? 4 : 1;                                         // columns per chunk
    // LDS row stride: the planner's residue mod 64 (spreads the 8 x 8 sums' reads over the banks),
    // or the odd width where that would not fit
    const int wmin = nc * cw;
    int ls = wmin + ((v.warp_ls_mod - wmin) & 63);
    if ((long long)ls * bh > kWarpLds) ls = wmin | 1;
    const bool use_lds = bx1 >= bx0 && bh > 0 && (long long)ls * bh <= kWarpLds;
    if (use_lds) {
        // chunk e = r * nc + c; each thread starts at e = tid and steps by 256 = q * nc + rem
        // chunks, so its (r, c) and both offsets advance by constants (no division per chunk);
        // up to 4 loads are in flight before their LDS stores
        const int n = nc * bh;
        const int q = kWarpThreads / nc, rem = kWarpThreads - q * nc;
        int e = int(threadIdx.x);
        int r = e / nc, c = e - r * nc;
        if (blur) {
            const float* g = bsrc + size_t(by0 + r) * bp + ax0 + 4 * c;
            int lo = r * ls + 4 * c;
            while (e < n) {
                float4 val[4];
                int los[4];
                int k = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (e < n) {
                        val[u] = *reinterpret_cast<const float4*>(g);
                        los[u] = lo;
                        ++k;
                        e += kWarpThreads;
                        c += rem;
                        g += size_t(q) * bp + 4 * rem;
                        lo += q * ls + 4 * rem;
                        if (c >= nc) {
                            c -= nc;
                            g += bp - 4 * nc;
                            lo += ls - 4 * nc;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (u < k) {
                        tile[los[u]] = val[u].x;
                        tile[los[u] + 1] = val[u].y;
                        tile[los[u] + 2] = val[u].z;
                        tile[los[u] + 3] = val[u].w;
                    }
                }
            }
        } else if (vec) {
            const uint8_t* g = src + size_t(by0 + r) * pitch + ax0 + 4 * c;
            int lo = r * ls + 4 * c;
            while (e < n) {
                uint32_t val[4];
                int los[4];
                int k = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (e < n) {
                        val[u] = *reinterpret_cast<const uint32_t*>(g);
                        los[u] = lo;
                        ++k;
                        e += kWarpThreads;
                        c += rem;
                        g += size_t(q) * pitch + 4 * rem;
                        lo += q * ls + 4 * rem;
                        if (c >= nc) {
                            c -= nc;
                            g += pitch - 4 * nc;
                            lo += ls - 4 * nc;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (u < k) {
                        tile[los[u]] = float(val[u] & 0xFF);
                        tile[los[u] + 1] = float((val[u] >> 8) & 0xFF);
                        tile[los[u] + 2] = float((val[u] >> 16) & 0xFF);
                        tile[los[u] + 3] = float(val[u] >> 24);
                    }
                }
            }
        } else {
            const uint8_t* g = src + size_t(by0 + r) * pitch + ax0 + c;
            int lo = r * ls + c;
            while (e < n) {
                tile[lo] = float(*g);
                e += kWarpThreads;
                c += rem;
                g += size_t(q) * pitch + rem;
                lo += q * ls + rem;
                if (c >= nc) {
                    c -= nc;
                    g += pitch - nc;
                    lo += ls - nc;
                }
            }
        }
    }
    __syncthreads();
    // each thread resamples kWarpRows pixels of its tile column, kWarpThreads / tw rows apart
    const int qx = x0 + int(threadIdx.x) % tw;
    for (int k = 0; k < kWarpRows; ++k) {
        const int qy = y0 + int(threadIdx.x) / tw + k * (kWarpThreads / tw);
        if (qx >= v.width || qy >= v.height) break;
        const size_t o = size_t(v.offset) + size_t(qy) * v.pitch + qx;
        const double px = affine_x(v.inv, double(qx), double(qy));
        const double py = affine_x(v.inv + 3, double(qx), double(qy));
        const bool inside = px >= -0.5 && px <= W - 0.5 && py >= -0.5 && py <= H - 0.5;
        if (!inside) {
            arena[o] = 0;
            mask[o] = 0;
            if (values) values[o] = 0.0f;
            continue;
        }
        const double fxd = floor(px), fyd = floor(py);
        const int ix = int(fxd), iy = int(fyd);
        float wx[8], wy[8];
        const float sx = lanczos4_weights(float(px - fxd), wx);
        const float sy = lanczos4_weights(float(py - fyd), wy);
        int cols[8];
        float val;
        if (use_lds && ix >= 3 && ix + 4 <= W - 1 && iy >= 3 && iy + 4 <= H - 1) {
            // interior: the 8 x 8 window needs no clamping; rows are read at immediate offsets
            const float* base = tile + (iy - 3 - by0) * ls + (ix - 3 - ax0);
            val = 0.0f;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float* r = base + j * ls;
                float sacc = 0.0f;
#pragma unroll
                for (int i = 0; i < 8; ++i) sacc += wx[i] * r[i];
                val += wy[j] * sacc;
            }
        } else if (use_lds) {
#pragma unroll
            for (int i = 0; i < 8; ++i) cols[i] = clampi(ix - 3 + i, bx0, bx1) - ax0;
            val = lanczos_sum([&](int j) { return tile + (clampi(iy - 3 + j, by0, by1) - by0) * ls; }, cols, wx, wy);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) cols[i] = clampi(ix - 3 + i, 0, W - 1);
            if (blur)
                val = lanczos_sum([&](int j) { return bsrc + size_t(clampi(iy - 3 + j, 0, H - 1)) * bp; }, cols, wx,
                                  wy);
            else
                val = lanczos_sum([&](int j) { return src + size_t(clampi(iy - 3 + j, 0, H - 1)) * pitch; }, cols,
                                  wx, wy);
        }
        val *= __builtin_amdgcn_rcpf(sx * sy);    // eq. (3) divided by the sum of the weights
        const float q = rintf(val);
        arena[o] = uint8_t(q < 0.0f ? 0.0f : (q > 255.0f ? 255.0f : q));
        mask[o] = 1;
        if (values) values[o] = val;
    }
}

}  // namespace

xa_status hip_fail(int err, const char* what) {
    return fail(XA_EHIP, "%s: %s", what, hipGetErrorString(hipError_t(err)));
}

xa_status launch_simulate(const PlanView& ph, const PlanView& pd, const uint8_t* sources,
                          uint8_t* arena, uint8_t* mask, float* values, float* blurred, hipStream_t st, int stages) {
    const xa_plan_header* h = ph.h;
    if ((stages & kStageBlur) && h->n_blur > 0) {
        const int tiles = ph.blur_prefix[h->n_blur];
        // LDS sized for the largest footprint among the blurred views (tiles away from the border
        // have the same footprint size as the first); larger ones fall back to global reads
        int lds = 0;
        for (int i = 0; i < h->n_blur; ++i) {
            const xa_view_desc& v = ph.views[ph.blur_views[i]];
            const BlurRegion g = blur_region(v, ph.taps + v.blur_tap0, 0, 0);
            if (g.floats <= kBlurLdsMax) lds = std::max(lds, g.floats);
        }
        hipLaunchKernelGGL(k_blur, dim3(tiles), dim3(256), size_t(lds) * sizeof(float), st, sources, pd.views,
                           pd.blur_views, pd.blur_prefix, h->n_blur, pd.taps, blurred, lds);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "blur launch");
    }
    const int tiles = ph.warp_prefix[h->n_views];
    if ((stages & kStageWarp) && tiles > 0) {
        hipLaunchKernelGGL(k_warp, dim3(tiles), dim3(kWarpThreads), 0, st, sources, blurred, pd.views, h->n_views,
                           pd.warp_prefix, arena, mask, values);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "warp launch");
    }
    return XA_OK;
}

}  // namespace xa

using namespace xa;

extern "C" size_t xa_simulate_workspace_size(const void* plan_host) {
    PlanView p;
    if (plan_host_view(plan_host, &p) != XA_OK) return 0;
    return simulate_ws_bytes(p.h);
}

static xa_status simulate_entry(const void* plan_host, const void* plan_dev, const uint8_t* d_sources,
                                uint8_t* d_arena, uint8_t* d_mask, float* d_values, void* d_ws, size_t ws_bytes,
                                hipStream_t stream, int stages) {
    PlanView ph;
    xa_status s = plan_host_view(plan_host, &ph);
    if (s != XA_OK) return s;
    if (!plan_dev || !d_sources) return fail(XA_EINVAL, "NULL device pointer");
    if (stages & kStageWarp) {
        if (!d_arena || !d_mask) return fail(XA_EINVAL, "NULL device pointer");
        if ((reinterpret_cast<uintptr_t>(d_arena) | reinterpret_cast<uintptr_t>(d_mask)) % 128)
            return fail(XA_EINVAL, "arena and mask must be 128-byte aligned");
    }
    const size_t need = simulate_ws_bytes(ph.h);
    if (ws_bytes < need) return fail(XA_ECAPACITY, "simulate workspace needs %zu bytes, got %zu", need, ws_bytes);
    if (need > 0 && (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) % kAlign)))
        return fail(XA_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    const PlanView pd = plan_dev_view(plan_host, plan_dev);
    s = launch_simulate(ph, pd, d_sources, d_arena, d_mask, d_values, static_cast<float*>(d_ws), stream, stages);
    return s == XA_OK ? ok() : s;
}

extern "C" xa_status xa_simulate_views(const void* plan_host, const void* plan_dev, const uint8_t* d_sources,
                                       uint8_t* d_arena, uint8_t* d_mask, float* d_values, void* d_ws,
                                       size_t ws_bytes, hipStream_t stream) {
    return simulate_entry(plan_host, plan_dev, d_sources, d_arena, d_mask, d_values, d_ws, ws_bytes, stream,
                          kStageBlur | kStageWarp);
}

extern "C" xa_status xa_blur_views(const void* plan_host, const void* plan_dev, const uint8_t* d_sources, void* d_ws,
                                   size_t ws_bytes, hipStream_t stream) {
    return simulate_entry(plan_host, plan_dev, d_sources, nullptr, nullptr, nullptr, d_ws, ws_bytes, stream,
                          kStageBlur);
}

extern "C" xa_status xa_warp_views(const void* plan_host, const void* plan_dev, const uint8_t* d_sources,
                                   uint8_t* d_arena, uint8_t* d_mask, float* d_values, void* d_ws, size_t ws_bytes,
                                   hipStream_t stream) {
    return simulate_entry(plan_host, plan_dev, d_sources, d_arena, d_mask, d_values, d_ws, ws_bytes, stream,
                          kStageWarp);
}

// ------------------------------------------------------------------ warp tile tuning

namespace xa {
namespace {

constexpr int kTuneCandidates[XA_WARP_CANDIDATES] = {4, 8, 16, 32, 64};

__global__ void __launch_bounds__(256) k_tune_fill(uint8_t* __restrict__ p, int pitch, int w, int h) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= w) return;
    uint32_t v = uint32_t(x) * 2654435761u ^ uint32_t(y) * 40503u;
    v ^= v >> 15;
    p[size_t(y) * pitch + x] = uint8_t(v);
}

// The views of compression class k: tilt sqrt(2)^k, longitudes 0, 72/t, 144/t, ... degrees below
// 180 (the sampling grid's views of that tilt), scale 1, repeated until they hold about
// kTuneViewPixels view pixels, so that each timed launch fills the chip as a real plan's does
// (one view of a small class would time launch latency, the same for every width).
constexpr double kTuneViewPixels = 8.0e6;

std::vector<xa_affine_params> class_views(int k, int w, int h) {
    std::vector<xa_affine_params> v;
    const double t = std::pow(2.0, 0.5 * k);
    const double step = 72.0 / t;
    for (int j = 0; k == 0 ? j < 1 : j * step < 180.0 - 1e-9; ++j) {
        xa_affine_params p{t, j * step * 3.141592653589793 / 180.0, 0.0, 1.0, 0.0, 0.0};
        v.push_back(p);
    }
    const double px = double(v.size()) * double(w) * double(h) / t;
    const int reps = std::max(1, int(std::ceil(kTuneViewPixels / px)));
    const size_t n = v.size();
    for (int r = 1; r < reps; ++r)
        for (size_t i = 0; i < n; ++i) v.push_back(v[i]);
    return v;
}

struct TunePlan {
    std::vector<uint8_t> blob;
};

xa_status tune_plan(int w, int h, int pitch, int k, int width, TunePlan* out, int rows = 0) {
    const std::vector<xa_affine_params> views = class_views(k, w, h);
    int32_t forced[XA_WARP_CLASSES], forced_rows[XA_WARP_CLASSES];
    for (int c = 0; c < XA_WARP_CLASSES; ++c) {
        forced[c] = width;
        forced_rows[c] = rows;
    }
    set_tile_override(forced);
    set_blur_rows_override(rows > 0 ? forced_rows : nullptr);
    size_t bytes = 0;
    xa_status s = xa_plan_image(w, h, pitch, views.data(), int32_t(views.size()), 1, 1.2, 1, 20, nullptr, 0, &bytes);
    if (s == XA_OK) {
        out->blob.assign(bytes, 0);
        s = xa_plan_image(w, h, pitch, views.data(), int32_t(views.size()), 1, 1.2, 1, 20, out->blob.data(), bytes,
                          &bytes);
    }
    set_tile_override(nullptr);
    set_blur_rows_override(nullptr);
    return s;
}

struct TuneLayout {
    size_t src, blob, ws, arena, mask, total;
    int pitch;
};

xa_status tune_layout(int w, int h, TuneLayout* L) {
    L->pitch = (w + 15) / 16 * 16;
    size_t blob = 0, ws = 0, arena = 0;
    for (int k = 0; k < XA_WARP_CLASSES; ++k) {
        for (const int rows : {4, 8}) {
            TunePlan P;
            const xa_status s = tune_plan(w, h, L->pitch, k, 8, &P, rows);
            if (s != XA_OK) return s;
            PlanView pv;
            plan_host_view(P.blob.data(), &pv);
            blob = std::max(blob, P.blob.size());
            ws = std::max(ws, simulate_ws_bytes(pv.h));
            arena = std::max(arena, size_t(pv.h->arena_bytes));
        }
    }
    size_t o = 0;
    L->src = o;   o += align_up(size_t(L->pitch) * h);
    L->blob = o;  o += align_up(blob);
    L->ws = o;    o += align_up(ws);
    L->arena = o; o += align_up(arena);
    L->mask = o;  o += align_up(arena);
    L->total = o;
    return XA_OK;
}

}  // namespace
}  // namespace xa

extern "C" size_t xa_tune_warp_tiles_workspace_size(int32_t src_w, int32_t src_h) {
    if (src_w < 16 || src_h < 16 || src_w > 8192 || src_h > 8192) return 0;
    TuneLayout L;
    return tune_layout(src_w, src_h, &L) == XA_OK ? L.total : 0;
}

extern "C" xa_status xa_tune_warp_tiles(int32_t src_w, int32_t src_h, void* d_ws, size_t ws_bytes, hipStream_t stream,
                                        int32_t* widths, float* ms) {
    if (src_w < 16 || src_h < 16 || src_w > 8192 || src_h > 8192)
        return fail(XA_EINVAL, "tuning image must be 16..8192 pixels a side");
    if (!widths) return fail(XA_EINVAL, "NULL output");
    TuneLayout L;
    xa_status s = tune_layout(src_w, src_h, &L);
    if (s != XA_OK) return s;
    if (!d_ws || ws_bytes < L.total || reinterpret_cast<uintptr_t>(d_ws) % kAlign)
        return fail(XA_EINVAL, "workspace of %zu bytes (256-byte aligned) needed, %zu given", L.total, ws_bytes);
    uint8_t* base = static_cast<uint8_t*>(d_ws);
    uint8_t* src = base + L.src;
    void* blob_dev = base + L.blob;
    float* blurred = reinterpret_cast<float*>(base + L.ws);
    uint8_t* arena = base + L.arena;
    uint8_t* mask = base + L.mask;
    hipLaunchKernelGGL(k_tune_fill, dim3(unsigned((src_w + 255) / 256), unsigned(src_h)), dim3(256), 0, stream, src,
                       L.pitch, src_w, src_h);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "event create");
    constexpr int kReps = 3;
    constexpr float kTuneMargin = 0.03f;
    for (int k = 0; k < XA_WARP_CLASSES && s == XA_OK; ++k) {
        float times[XA_WARP_CANDIDATES] = {};
        for (int c = 0; c < XA_WARP_CANDIDATES && s == XA_OK; ++c) {
            TunePlan P;
            s = tune_plan(src_w, src_h, L.pitch, k, kTuneCandidates[c], &P);
            if (s != XA_OK) break;
            if (P.blob.size() > L.ws - L.blob) {     // the plan's slot in the workspace
                s = fail(XA_EUNSUPPORTED, "tuning plan larger than its workspace slot");
                break;
            }
            e = hipMemcpyAsync(blob_dev, P.blob.data(), P.blob.size(), hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);     // the host blob goes out of scope below
            if (e != hipSuccess) { s = hip_fail(e, "plan upload"); break; }
            PlanView ph;
            plan_host_view(P.blob.data(), &ph);
            const PlanView pd = plan_dev_view(P.blob.data(), blob_dev);
            if (c == 0) s = launch_simulate(ph, pd, src, arena, mask, nullptr, blurred, stream, kStageBlur);
            if (s == XA_OK) s = launch_simulate(ph, pd, src, arena, mask, nullptr, blurred, stream, kStageWarp);
            e = hipEventRecord(e0, stream);
            for (int r = 0; r < kReps && s == XA_OK; ++r)
                s = launch_simulate(ph, pd, src, arena, mask, nullptr, blurred, stream, kStageWarp);
            if (e == hipSuccess) e = hipEventRecord(e1, stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) { s = hip_fail(e, "tuning timing"); break; }
            t /= kReps;
            if (ms) ms[k * XA_WARP_CANDIDATES + c] = t;
            times[c] = t;
        }
        if (s != XA_OK) break;
        // the rule's width stays unless a candidate is faster by more than the timing noise
        const int rule_w = warp_tile_w(std::pow(2.0, 0.5 * k), 1.0);
        int best_c = 0;
        for (int c = 1; c < XA_WARP_CANDIDATES; ++c)
            if (times[c] < times[best_c]) best_c = c;
        float rule_ms = times[best_c];
        for (int c = 0; c < XA_WARP_CANDIDATES; ++c)
            if (kTuneCandidates[c] == rule_w) rule_ms = times[c];
        widths[k] = times[best_c] < (1.0f - kTuneMargin) * rule_ms ? kTuneCandidates[best_c] : rule_w;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return s == XA_OK ? ok() : s;
}

extern "C" size_t xa_tune_blur_rows_workspace_size(int32_t src_w, int32_t src_h) {
    return xa_tune_warp_tiles_workspace_size(src_w, src_h);
}

extern "C" xa_status xa_tune_blur_rows(int32_t src_w, int32_t src_h, void* d_ws, size_t ws_bytes, hipStream_t stream,
                                       int32_t* rows, float* ms) {
    if (src_w < 16 || src_h < 16 || src_w > 8192 || src_h > 8192)
        return fail(XA_EINVAL, "tuning image must be 16..8192 pixels a side");
    if (!rows) return fail(XA_EINVAL, "NULL output");
    TuneLayout L;
    xa_status s = tune_layout(src_w, src_h, &L);
    if (s != XA_OK) return s;
    if (!d_ws || ws_bytes < L.total || reinterpret_cast<uintptr_t>(d_ws) % kAlign)
        return fail(XA_EINVAL, "workspace of %zu bytes (256-byte aligned) needed, %zu given", L.total, ws_bytes);
    uint8_t* base = static_cast<uint8_t*>(d_ws);
    uint8_t* src = base + L.src;
    void* blob_dev = base + L.blob;
    float* blurred = reinterpret_cast<float*>(base + L.ws);
    uint8_t* arena = base + L.arena;
    uint8_t* mask = base + L.mask;
    hipLaunchKernelGGL(k_tune_fill, dim3(unsigned((src_w + 255) / 256), unsigned(src_h)), dim3(256), 0, stream, src,
                       L.pitch, src_w, src_h);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "event create");
    constexpr int kReps = 3;
    constexpr float kTuneMargin = 0.03f;
    constexpr int kRows[2] = {4, 8};
    rows[0] = kBlurRowsDefault;                  // class 0 (t/s < sqrt 2) has no blur on the grid
    if (ms) ms[0] = ms[1] = 0.0f;
    for (int k = 1; k < XA_WARP_CLASSES && s == XA_OK; ++k) {
        float times[2] = {};
        for (int c = 0; c < 2 && s == XA_OK; ++c) {
            TunePlan P;
            s = tune_plan(src_w, src_h, L.pitch, k, 8, &P, kRows[c]);
            if (s != XA_OK) break;
            if (P.blob.size() > L.ws - L.blob) {     // the plan's slot in the workspace
                s = fail(XA_EUNSUPPORTED, "tuning plan larger than its workspace slot");
                break;
            }
            e = hipMemcpyAsync(blob_dev, P.blob.data(), P.blob.size(), hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);     // the host blob goes out of scope below
            if (e != hipSuccess) { s = hip_fail(e, "plan upload"); break; }
            PlanView ph;
            plan_host_view(P.blob.data(), &ph);
            const PlanView pd = plan_dev_view(P.blob.data(), blob_dev);
            s = launch_simulate(ph, pd, src, arena, mask, nullptr, blurred, stream, kStageBlur);
            e = hipEventRecord(e0, stream);
            for (int r = 0; r < kReps && s == XA_OK; ++r)
                s = launch_simulate(ph, pd, src, arena, mask, nullptr, blurred, stream, kStageBlur);
            if (e == hipSuccess) e = hipEventRecord(e1, stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) { s = hip_fail(e, "tuning timing"); break; }
            times[c] = t / kReps;
            if (ms) ms[2 * k + c] = times[c];
        }
        if (s != XA_OK) break;
        rows[k] = times[0] < (1.0f - kTuneMargin) * times[1] ? 4 : 8;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return s == XA_OK ? ok() : s;
}
