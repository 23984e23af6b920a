// The Lanczos-4 affine warp of fp32 crops as a differentiable function of the image
// and of the six camera parameters (t, phi, psi, s, tx, ty), forward and adjoint.
//
// Resampling of eqs. (3)-(4): 8 x 8 taps (i, j = -3..4), weights normalised to sum one,
// border taps clamped.  The map is the camera map of eq. (2), L = s R(psi) diag(1/t, 1)
// R(phi), centred on the crop: view pixel q samples p = L^-1 (q - c - T) + c, with
// c = ((w - 1)/2, (h - 1)/2) and T = (tx, ty).  Pixels whose p leaves
// [-1/2, w - 1/2] x [-1/2, h - 1/2] are 0 and carry no gradient.
//
// Coordinates are fp64; weights and sums fp32; per-pixel parameter gradients fp64.
// Kernel weights use sin(pi (i - f)) = -(-1)^i sin(pi f) and the angle-difference
// formula for sin(pi (i - f) / 4), so each axis needs the sine and cosine of pi f and pi f / 4 only;
// within 0.05 of a zero of the argument the weight and its derivative switch to the
// Taylor series of sinc(x) sinc(x / 4), where the closed forms cancel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace xa {
namespace {

constexpr int kDwTX = 16, kDwTY = 16;  // 256 threads, one view pixel each
constexpr int kDwLds = 8192;           // floats of source footprint a tile stages (forward) or accumulates (adjoint)

struct CropMap {
    double m[4];      // L^-1, row-major
    double dm[4][4];  // d L^-1 / d(t, phi, psi, s)
    double cx, cy, tx, ty;
};

// L^-1 = (1/s) R(-phi) diag(t, 1) R(-psi) and its derivatives; d/da R(a) = R(a) J.
__device__ void crop_map(const xa_affine_params& P, bool derivs, CropMap* C, int w, int h) {
    double sf, cf, sp, cp;
    sincos(P.phi, &sf, &cf);
    sincos(P.psi, &sp, &cp);
    const double is = 1.0 / P.s;
    // R(-phi) = [[cf, sf], [-sf, cf]], R(-psi) = [[cp, sp], [-sp, cp]]
    // A = R(-phi) diag(t, 1) = [[t cf, sf], [-t sf, cf]]
    const double a00 = P.t * cf, a01 = sf, a10 = -P.t * sf, a11 = cf;
    C->m[0] = is * (a00 * cp - a01 * sp);
    C->m[1] = is * (a00 * sp + a01 * cp);
    C->m[2] = is * (a10 * cp - a11 * sp);
    C->m[3] = is * (a10 * sp + a11 * cp);
    C->cx = 0.5 * (w - 1);
    C->cy = 0.5 * (h - 1);
    C->tx = P.tx;
    C->ty = P.ty;
    if (!derivs) return;
    // d/dt: (1/s) R(-phi) diag(1, 0) R(-psi) = (1/s) [cf; -sf] [cp, sp]
    C->dm[0][0] = is * cf * cp; C->dm[0][1] = is * cf * sp;
    C->dm[0][2] = -is * sf * cp; C->dm[0][3] = -is * sf * sp;
    // d/dphi: -(1/s) R(-phi) J diag(t, 1) R(-psi); R(-phi) J = [[sf, -cf], [cf, sf]]
    {
        const double b00 = sf * P.t, b01 = -cf, b10 = cf * P.t, b11 = sf;
        C->dm[1][0] = -is * (b00 * cp - b01 * sp);
        C->dm[1][1] = -is * (b00 * sp + b01 * cp);
        C->dm[1][2] = -is * (b10 * cp - b11 * sp);
        C->dm[1][3] = -is * (b10 * sp + b11 * cp);
    }
    // d/dpsi: -(1/s) R(-phi) diag(t, 1) R(-psi) J; R(-psi) J = [[sp, -cp], [cp, sp]]
    C->dm[2][0] = -is * (a00 * sp + a01 * cp);
    C->dm[2][1] = -is * (-a00 * cp + a01 * sp);
    C->dm[2][2] = -is * (a10 * sp + a11 * cp);
    C->dm[2][3] = -is * (-a10 * cp + a11 * sp);
    // d/ds = -L^-1 / s
    for (int k = 0; k < 4; ++k) C->dm[3][k] = -C->m[k] * is;
}

// Taylor coefficients of sinc(x) sinc(x / 4) in u = (pi x)^2.
constexpr float kC1 = -17.0f / 96.0f;
constexpr float kC2 = float(1.0 / 120 + 1.0 / 30720 + 1.0 / 576);
constexpr float kC3 = float(-1.0 / 5040 - 1.0 / 20643840 - 1.0 / 184320 - 1.0 / 11520);
constexpr float kPi = 3.14159265358979323846f;

// Weights w_i = L(i - f) and (if D) dw_i/dp = -L'(i - f) for i = -3..4; returns the sums.
template <bool D>
__device__ inline void axis_weights(float f, float* w, float* dw, float* sw, float* sdw) {
    // hardware sine / cosine take revolutions: sin(pi f) = sin(2 pi (f / 2)); absolute error ~1e-6,
    // and the closed forms below are only used at least 0.05 away from a zero of the argument
    const float s1 = __builtin_amdgcn_sinf(0.5f * f), c1 = __builtin_amdgcn_cosf(0.5f * f);
    const float s4 = __builtin_amdgcn_sinf(0.125f * f), c4 = __builtin_amdgcn_cosf(0.125f * f);
    // sin(pi i / 4), cos(pi i / 4) for i = -3..4
    constexpr float kH = 0.70710678118654752f;
    const float si[8] = {-kH, -1.0f, -kH, 0.0f, kH, 1.0f, kH, 0.0f};
    const float ci[8] = {-kH, 0.0f, kH, 1.0f, kH, 0.0f, -kH, -1.0f};
    float a = 0.0f, b = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int i = k - 3;
        const float x = float(i) - f;
        const float sgn = (i & 1) ? -1.0f : 1.0f;          // (-1)^i
        float L, Ld;
        if (fabsf(x) < 0.05f) {
            const float u = kPi * kPi * x * x;
            L = 1.0f + u * (kC1 + u * (kC2 + u * kC3));
            Ld = 2.0f * kPi * kPi * x * (kC1 + u * (2.0f * kC2 + 3.0f * u * kC3));
        } else {
            const float sx = -sgn * s1;                      // sin(pi x)
            const float cx = sgn * c1;                       // cos(pi x)
            const float sq = si[k] * c4 - ci[k] * s4;        // sin(pi x / 4)
            const float cq = ci[k] * c4 + si[k] * s4;        // cos(pi x / 4)
            const float r = 1.0f / x;
            const float k4 = 4.0f / (kPi * kPi);
            L = k4 * sx * sq * r * r;
            Ld = (k4 * (kPi * cx * sq + 0.25f * kPi * sx * cq) * r - 2.0f * L) * r;
        }
        w[k] = L;
        a += L;
        if (D) {
            dw[k] = -Ld;
            b -= Ld;
        }
    }
    *sw = a;
    if (D) *sdw = b;
}

struct Sample {
    bool valid;
    double px, py, dx, dy;
};

__device__ inline Sample sample_point(const CropMap& C, int x, int y, int w, int h) {
    Sample S;
    S.dx = double(x) - C.cx - C.tx;
    S.dy = double(y) - C.cy - C.ty;
    S.px = C.m[0] * S.dx + C.m[1] * S.dy + C.cx;
    S.py = C.m[2] * S.dx + C.m[3] * S.dy + C.cy;
    S.valid = S.px >= -0.5 && S.px <= w - 0.5 && S.py >= -0.5 && S.py <= h - 0.5;
    return S;
}

__global__ void __launch_bounds__(256) k_dw_fill(float* __restrict__ p, size_t n) {
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        p[i] = 0.0f;
}

// Source box of a 16 x 16 tile: the bounding box of its pixel centres mapped through the
// crop map, grown by the 8-tap window and clamped to the crop.  Every tap of a valid pixel of
// the tile, once clamped to the crop, lies in it.
struct Box {
    int x0, x1, y0, y1;
};
__device__ Box tile_box(const CropMap& C, int tx0, int ty0, int w, int h) {
    double pxl = 1e300, pxh = -1e300, pyl = 1e300, pyh = -1e300;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const Sample S = sample_point(C, tx0 + ((c & 1) ? kDwTX - 1 : 0), ty0 + ((c & 2) ? kDwTY - 1 : 0), w, h);
        pxl = fmin(pxl, S.px); pxh = fmax(pxh, S.px);
        pyl = fmin(pyl, S.py); pyh = fmax(pyh, S.py);
    }
    Box b;
    b.x0 = max(int(fmax(floor(pxl - 1e-6), -1e9)) - 3, 0);
    b.x1 = min(int(fmin(floor(pxh + 1e-6), 1e9)) + 4, w - 1);
    b.y0 = max(int(fmax(floor(pyl - 1e-6), -1e9)) - 3, 0);
    b.y1 = min(int(fmin(floor(pyh + 1e-6), 1e9)) + 4, h - 1);
    return b;
}

// One 16 x 16 tile per block; its source box is staged in LDS when it fits (taps then read
// from LDS), else taps are read from global memory.
__global__ void __launch_bounds__(256) k_dw_fwd(const float* __restrict__ img, const xa_affine_params* __restrict__ params,
                                                int w, int h, int tiles_x, int tiles, float* __restrict__ out,
                                                uint8_t* __restrict__ mask) {
    __shared__ CropMap sC;
    __shared__ float tile[kDwLds];
    const int crop = blockIdx.x / tiles, tl = blockIdx.x - crop * tiles;
    if (threadIdx.x == 0) crop_map(params[crop], false, &sC, w, h);
    __syncthreads();
    const int tyi = tl / tiles_x, txi = tl - tyi * tiles_x;
    const int tx0 = txi * kDwTX, ty0 = tyi * kDwTY;
    const Box bx = tile_box(sC, tx0, ty0, w, h);
    const int bw = bx.x1 - bx.x0 + 1, bh = bx.y1 - bx.y0 + 1;
    const int ls = bw | 1;
    const bool use_lds = bw > 0 && bh > 0 && ls * bh <= kDwLds;
    const float* base = img + size_t(crop) * h * w;
    if (use_lds) {
        // element e = r * bw + c, each thread stepping by 256 = q * bw + rem (no division per element)
        const int n = bw * bh, q = 256 / bw, rem = 256 - q * bw;
        int e = threadIdx.x, r = e / bw, c = e - r * bw;
        const float* g = base + size_t(bx.y0 + r) * w + bx.x0 + c;
        int lo = r * ls + c;
        while (e < n) {
            tile[lo] = *g;
            e += 256;
            c += rem;
            g += size_t(q) * w + rem;
            lo += q * ls + rem;
            if (c >= bw) {
                c -= bw;
                g += w - bw;
                lo += ls - bw;
            }
        }
    }
    __syncthreads();
    const int x = tx0 + int(threadIdx.x % kDwTX), y = ty0 + int(threadIdx.x / kDwTX);
    if (x >= w || y >= h) return;
    const size_t o = (size_t(crop) * h + y) * w + x;
    const Sample S = sample_point(sC, x, y, w, h);
    float v = 0.0f;
    if (S.valid) {
        const double fx0 = floor(S.px), fy0 = floor(S.py);
        const int ix = int(fx0), iy = int(fy0);
        float wx[8], wy[8], sx, sy;
        axis_weights<false>(float(S.px - fx0), wx, nullptr, &sx, nullptr);
        axis_weights<false>(float(S.py - fy0), wy, nullptr, &sy, nullptr);
        float acc = 0.0f;
        if (use_lds) {
            int cols[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) cols[i] = min(max(ix - 3 + i, bx.x0), bx.x1) - bx.x0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float* row = tile + (min(max(iy - 3 + j, bx.y0), bx.y1) - bx.y0) * ls;
                float r = 0.0f;
#pragma unroll
                for (int i = 0; i < 8; ++i) r = fmaf(wx[i], row[cols[i]], r);
                acc = fmaf(wy[j], r, acc);
            }
        } else {
            int cols[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) cols[i] = min(max(ix - 3 + i, 0), w - 1);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float* row = base + size_t(min(max(iy - 3 + j, 0), h - 1)) * w;
                float r = 0.0f;
#pragma unroll
                for (int i = 0; i < 8; ++i) r = fmaf(wx[i], row[cols[i]], r);
                acc = fmaf(wy[j], r, acc);
            }
        }
        v = acc / (sx * sy);
    }
    out[o] = v;
    if (mask) mask[o] = S.valid ? 1 : 0;
}

// Adjoint, one 16 x 16 tile per block.  The image gradient is accumulated in LDS over the
// tile's source box with LDS atomics when the box fits, then added to the crop's gradient with
// one global atomic per box pixel (a global atomic per tap otherwise); the parameter gradient
// is summed per block in a fixed order.
template <bool GIMG, bool GPAR>
__global__ void __launch_bounds__(256) k_dw_bwd(const float* __restrict__ img, const float* __restrict__ gout,
                                                const xa_affine_params* __restrict__ params, int w, int h,
                                                int tiles_x, int tiles, float* __restrict__ gimg,
                                                double* __restrict__ partial) {
    __shared__ CropMap sC;
    __shared__ double sRed[4][6];
    __shared__ float sMax[4];
    // the tile's image-gradient box, accumulated in LDS as fixed point (see below)
    __shared__ int accum[GIMG ? kDwLds : 1];
    // the tile's source box, staged for the parameter gradient's tap reads (as in the forward)
    // when the image gradient is not wanted: with both, the two 32 KiB arrays would leave room
    // for two blocks per CU, which costs more than the staging saves
    constexpr bool kStage = GPAR && !GIMG;
    __shared__ float stile[kStage ? kDwLds : 1];
    const int crop = blockIdx.x / tiles, tl = blockIdx.x - crop * tiles;
    if (threadIdx.x == 0) crop_map(params[crop], GPAR, &sC, w, h);
    const int tyi = tl / tiles_x, txi = tl - tyi * tiles_x;
    const int tx0 = txi * kDwTX, ty0 = tyi * kDwTY;
    const size_t cbase = size_t(crop) * h * w;
    const int x = tx0 + int(threadIdx.x % kDwTX), y = ty0 + int(threadIdx.x / kDwTX);
    const float g = (x < w && y < h) ? gout[cbase + size_t(y) * w + x] : 0.0f;
    if (GIMG) {     // m = max |g| over the tile (infinite if some g is NaN)
        float a = g != g ? INFINITY : fabsf(g);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) a = fmaxf(a, __shfl_xor(a, off));
        if ((threadIdx.x & 63) == 0) sMax[threadIdx.x >> 6] = a;
    }
    __syncthreads();
    const Box bx = tile_box(sC, tx0, ty0, w, h);
    const int bw = bx.x1 - bx.x0 + 1, bh = bx.y1 - bx.y0 + 1;
    // Integer LDS atomics run several times faster than float ones, so the box sums are kept
    // in int32 units of 1/S, S = 2^(29 - k) with 2^k <= 1024 m < 2^(k+1): one output pixel adds
    // at most |g| (sum |wx| / |sum wx|) (sum |wy| / |sum wy|) < 4 |g| to a box pixel (clamped
    // taps included) and at most 256 output pixels reach it, so every sum stays below 2^30.
    // Rounding each contribution to 1/S costs at most 2^-20 m.  A tile whose m is not finite
    // keeps float atomics (the box is then reused as float); a tile whose m is tiny keeps S at
    // 2^125.
    const float m = GIMG ? fmaxf(fmaxf(sMax[0], sMax[1]), fmaxf(sMax[2], sMax[3])) : 0.0f;
    const bool fixed = GIMG && isfinite(1024.0f * m);
    // k is held at -96 or above so that S stays a finite float for tiny gradients
    const float scale = fixed && m > 0.0f ? ldexpf(1.0f, 29 - max(ilogbf(1024.0f * m), -96)) : 1.0f;
    const bool use_acc = GIMG && bw > 0 && bh > 0 && bw * bh <= kDwLds;
    if (use_acc)
        for (int e = threadIdx.x; e < bw * bh; e += 256) accum[e] = 0;
    const int ls = bw | 1;
    const bool use_tile = kStage && bw > 0 && bh > 0 && ls * bh <= kDwLds;
    if (use_tile) {
        // element e = r * bw + c, each thread stepping by 256 = q * bw + rem (no division per element)
        const int n = bw * bh, q = 256 / bw, rem = 256 - q * bw;
        int e = threadIdx.x, r = e / bw, c = e - r * bw;
        const float* gsrc = img + cbase + size_t(bx.y0 + r) * w + bx.x0 + c;
        int lo = r * ls + c;
        while (e < n) {
            stile[lo] = *gsrc;
            e += 256;
            c += rem;
            gsrc += size_t(q) * w + rem;
            lo += q * ls + rem;
            if (c >= bw) {
                c -= bw;
                gsrc += w - bw;
                lo += ls - bw;
            }
        }
    }
    __syncthreads();
    double gp[6] = {0, 0, 0, 0, 0, 0};
    if (x < w && y < h) {
        const Sample S = sample_point(sC, x, y, w, h);
        if (S.valid && g != 0.0f) {
            const double fx0 = floor(S.px), fy0 = floor(S.py);
            const int ix = int(fx0), iy = int(fy0);
            float wx[8], wy[8], dwx[8], dwy[8], sx, sy, sdx, sdy;
            axis_weights<GPAR>(float(S.px - fx0), wx, dwx, &sx, &sdx);
            axis_weights<GPAR>(float(S.py - fy0), wy, dwy, &sy, &sdy);
            const float inv = 1.0f / (sx * sy);
            int cols[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) cols[i] = min(max(ix - 3 + i, 0), w - 1);
            float v = 0.0f, vx = 0.0f, vy = 0.0f;
            const float gn = g * inv;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int row = min(max(iy - 3 + j, 0), h - 1);
                if (GPAR) {
                    // taps of a valid pixel lie inside the tile's box (the image-gradient box relies
                    // on the same), so the staged copy serves them, at box-relative (non-negative)
                    // offsets; the LDS and global reads stay separate loops (the choice is uniform
                    // per block)
                    float r = 0.0f, rd = 0.0f;
                    if (use_tile) {
                        const float* tr = stile + (row - bx.y0) * ls;
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const float a = tr[cols[i] - bx.x0];
                            r = fmaf(wx[i], a, r);
                            rd = fmaf(dwx[i], a, rd);
                        }
                    } else {
                        const float* rp = img + cbase + size_t(row) * w;
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const float a = rp[cols[i]];
                            r = fmaf(wx[i], a, r);
                            rd = fmaf(dwx[i], a, rd);
                        }
                    }
                    v = fmaf(wy[j], r, v);
                    vx = fmaf(wy[j], rd, vx);
                    vy = fmaf(dwy[j], r, vy);
                }
                if (GIMG) {
                    const float gj = gn * wy[j];
                    if (use_acc && fixed) {     // box-relative, non-negative offsets
                        int* ar = accum + (row - bx.y0) * bw;
                        const float gs = gj * scale;
#pragma unroll
                        for (int i = 0; i < 8; ++i) atomicAdd(ar + (cols[i] - bx.x0), int(rintf(gs * wx[i])));
                    } else if (use_acc) {
                        float* ar = reinterpret_cast<float*>(accum) + (row - bx.y0) * bw;
#pragma unroll
                        for (int i = 0; i < 8; ++i) atomicAdd(ar + (cols[i] - bx.x0), gj * wx[i]);
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; ++i) unsafeAtomicAdd(gimg + cbase + size_t(row) * w + cols[i], gj * wx[i]);
                    }
                }
            }
            if (GPAR) {
                const double V = double(v) * inv;
                const double dVx = double(vx) * inv - V * double(sdx) / double(sx);
                const double dVy = double(vy) * inv - V * double(sdy) / double(sy);
                const double gd = g;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double dpx = sC.dm[k][0] * S.dx + sC.dm[k][1] * S.dy;
                    const double dpy = sC.dm[k][2] * S.dx + sC.dm[k][3] * S.dy;
                    gp[k] = gd * (dVx * dpx + dVy * dpy);
                }
                // d(q - c - T)/dtx = (-1, 0), d/dty = (0, -1)
                gp[4] = -gd * (dVx * sC.m[0] + dVy * sC.m[2]);
                gp[5] = -gd * (dVx * sC.m[1] + dVy * sC.m[3]);
            }
        }
    }
    if (GIMG && use_acc) {
        __syncthreads();
        // one global atomic per box pixel that received a contribution
        const int n = bw * bh, q = 256 / bw, rem = 256 - q * bw;
        int e = threadIdx.x, r = e / bw, c = e - r * bw;
        float* gptr = gimg + cbase + size_t(bx.y0 + r) * w + bx.x0 + c;
        const float inv_scale = 1.0f / scale;
        while (e < n) {
            const float a = fixed ? float(accum[e]) * inv_scale : __int_as_float(accum[e]);
            if (a != 0.0f) unsafeAtomicAdd(gptr, a);
            e += 256;
            c += rem;
            gptr += size_t(q) * w + rem;
            if (c >= bw) {
                c -= bw;
                gptr += w - bw;
            }
        }
    }
    if (!GPAR) return;
    // block sum in a fixed order: butterfly within the wave, then the four waves in order
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) gp[k] += __shfl_xor(gp[k], off);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 6; ++k) sRed[wave][k] = gp[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        partial[size_t(blockIdx.x) * 6 + k] = ((sRed[0][k] + sRed[1][k]) + sRed[2][k]) + sRed[3][k];
    }
}

// gparam[crop][k] = sum over the crop's tiles of partial[tile][k], in tile order.
__global__ void __launch_bounds__(256) k_dw_reduce(const double* __restrict__ partial, int tiles,
                                                   double* __restrict__ gparam) {
    __shared__ double s[256][6];
    const int crop = blockIdx.x;
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int t = threadIdx.x; t < tiles; t += 256)
#pragma unroll
        for (int k = 0; k < 6; ++k) a[k] += partial[(size_t(crop) * tiles + t) * 6 + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) s[threadIdx.x][k] = a[k];
    __syncthreads();
    for (int n = 128; n >= 1; n >>= 1) {
        if (int(threadIdx.x) < n)
#pragma unroll
            for (int k = 0; k < 6; ++k) s[threadIdx.x][k] += s[threadIdx.x + n][k];
        __syncthreads();
    }
    if (threadIdx.x < 6) gparam[size_t(crop) * 6 + threadIdx.x] = s[0][threadIdx.x];
}

struct DwGeom {
    int tiles_x, tiles;
    long long blocks;
};

xa_status dw_check(const float* img, int32_t n, int32_t h, int32_t w, const xa_affine_params* params, DwGeom* g) {
    if (n < 1 || h < 1 || w < 1) return fail(XA_EINVAL, "need n, h, w >= 1");
    if ((long long)h * w > (1LL << 28) || (long long)n * h * w > (1LL << 38))
        return fail(XA_EUNSUPPORTED, "crops too large");
    if (!img || !params) return fail(XA_EINVAL, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(img) % 4 || reinterpret_cast<uintptr_t>(params) % 8)
        return fail(XA_EINVAL, "misaligned image or parameter buffer");
    g->tiles_x = (w + kDwTX - 1) / kDwTX;
    g->tiles = g->tiles_x * ((h + kDwTY - 1) / kDwTY);
    g->blocks = (long long)g->tiles * n;
    if (g->blocks > INT32_MAX) return fail(XA_EUNSUPPORTED, "too many tiles for one launch");
    return XA_OK;
}

}  // namespace
}  // namespace xa

using namespace xa;

extern "C" xa_status xa_warp_f32_fwd(const float* d_img, int32_t n, int32_t h, int32_t w,
                                     const xa_affine_params* d_params, float* d_out, uint8_t* d_mask,
                                     hipStream_t stream) {
    DwGeom g;
    xa_status s = dw_check(d_img, n, h, w, d_params, &g);
    if (s != XA_OK) return s;
    if (!d_out) return fail(XA_EINVAL, "NULL output");
    hipLaunchKernelGGL(k_dw_fwd, dim3(unsigned(g.blocks)), dim3(256), 0, stream, d_img, d_params, w, h, g.tiles_x,
                       g.tiles, d_out, d_mask);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "warp forward launch");
}

extern "C" size_t xa_warp_f32_bwd_workspace_size(int32_t n, int32_t h, int32_t w) {
    if (n < 1 || h < 1 || w < 1) return 0;
    const long long tiles = (long long)((w + kDwTX - 1) / kDwTX) * ((h + kDwTY - 1) / kDwTY);
    return align_up(size_t(tiles) * size_t(n) * 6 * sizeof(double));
}

extern "C" xa_status xa_warp_f32_bwd(const float* d_img, const float* d_gout, const xa_affine_params* d_params,
                                     int32_t n, int32_t h, int32_t w, float* d_gimg, double* d_gparams, void* d_ws,
                                     size_t ws_bytes, hipStream_t stream) {
    DwGeom g;
    xa_status s = dw_check(d_img, n, h, w, d_params, &g);
    if (s != XA_OK) return s;
    if (!d_gout) return fail(XA_EINVAL, "NULL output gradient");
    if (reinterpret_cast<uintptr_t>(d_gout) % 4 || reinterpret_cast<uintptr_t>(d_gimg) % 4 ||
        reinterpret_cast<uintptr_t>(d_gparams) % 8)
        return fail(XA_EINVAL, "misaligned gradient buffer");
    if (!d_gimg && !d_gparams) return ok();
    double* partial = static_cast<double*>(d_ws);
    if (d_gparams) {
        const size_t need = xa_warp_f32_bwd_workspace_size(n, h, w);
        if (ws_bytes < need) return fail(XA_ECAPACITY, "warp backward needs %zu bytes of workspace, got %zu", need,
                                          ws_bytes);
        if (!d_ws || reinterpret_cast<uintptr_t>(d_ws) % 8) return fail(XA_EINVAL, "workspace NULL or misaligned");
    }
    if (d_gimg) {
        const size_t total = size_t(n) * h * w;
        const unsigned fb = unsigned(std::min<size_t>((total + 255) / 256, 65536));
        hipLaunchKernelGGL(k_dw_fill, dim3(fb), dim3(256), 0, stream, d_gimg, total);
    }
    const dim3 grid(unsigned(g.blocks)), block(256);
    if (d_gimg && d_gparams)
        hipLaunchKernelGGL((k_dw_bwd<true, true>), grid, block, 0, stream, d_img, d_gout, d_params, w, h, g.tiles_x,
                           g.tiles, d_gimg, partial);
    else if (d_gimg)
        hipLaunchKernelGGL((k_dw_bwd<true, false>), grid, block, 0, stream, d_img, d_gout, d_params, w, h, g.tiles_x,
                           g.tiles, d_gimg, partial);
    else
        hipLaunchKernelGGL((k_dw_bwd<false, true>), grid, block, 0, stream, d_img, d_gout, d_params, w, h, g.tiles_x,
                           g.tiles, d_gimg, partial);
    if (d_gparams) hipLaunchKernelGGL(k_dw_reduce, dim3(unsigned(n)), dim3(256), 0, stream, partial, g.tiles, d_gparams);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "warp backward launch");
}
