// View simulation on gfx950: anti-alias blur along the tilt direction and
// Lanczos-4 affine resampling (eqs. (3)-(4), 8x8 window per Sec. IV.C).
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace xa {
namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Largest i in [0, n) with prefix[i] <= b (prefix[0] == 0, prefix non-decreasing).
__device__ __forceinline__ int find_segment(const int32_t* __restrict__ prefix, int n, int b) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Directional Gaussian over the source: one thread per source pixel of one blurred view.
// out(p) = sum_k w_k lerp(I, p + k v) with v = (1, m) (major x) or (m, 1) (major y).
__global__ void __launch_bounds__(256) k_blur(const uint8_t* __restrict__ src, int W, int H, int pitch,
                                              const xa_view_desc* __restrict__ views,
                                              const int32_t* __restrict__ blur_views,
                                              const BlurTap* __restrict__ taps, float* __restrict__ out) {
    const int tiles_x = (W + kBlurTX - 1) / kBlurTX;
    const int x = (blockIdx.x % tiles_x) * kBlurTX + (threadIdx.x % kBlurTX);
    const int y = (blockIdx.x / tiles_x) * kBlurTY + (threadIdx.x / kBlurTX);
    if (x >= W || y >= H) return;
    const xa_view_desc& v = views[blur_views[blockIdx.y]];
    const BlurTap* tp = taps + v.blur_tap0;
    const int n = v.blur_ntaps;
    float acc = 0.0f;
    if (v.blur_major == 0) {
        for (int k = 0; k < n; ++k) {
            const BlurTap t = tp[k];
            const int xk = clampi(x + t.dmaj, 0, W - 1);
            const int y0 = y + t.dmin;
            const float a = float(src[size_t(clampi(y0, 0, H - 1)) * pitch + xk]);
            const float b = float(src[size_t(clampi(y0 + 1, 0, H - 1)) * pitch + xk]);
            acc += t.w * ((1.0f - t.frac) * a + t.frac * b);
        }
    } else {
        for (int k = 0; k < n; ++k) {
            const BlurTap t = tp[k];
            const int yk = clampi(y + t.dmaj, 0, H - 1);
            const int x0 = x + t.dmin;
            const uint8_t* row = src + size_t(yk) * pitch;
            const float a = float(row[clampi(x0, 0, W - 1)]);
            const float b = float(row[clampi(x0 + 1, 0, W - 1)]);
            acc += t.w * ((1.0f - t.frac) * a + t.frac * b);
        }
    }
    out[v.blur_offset + size_t(y) * W + x] = acc;
}

// Weights L4(i - f), i = -3..4, of eq. (4) (a = 4), normalised to sum 1.
// sin(pi (i - f)) = (-1)^(i+1) sin(pi f) and sin(pi (i - f)/4) expands with the
// angle-difference formula, so three transcendental evaluations serve all 8 taps;
// f == 0 gives the exact one-hot weights of an on-grid sample.
__device__ __forceinline__ void lanczos4_weights(float f, float w[8]) {
    if (f == 0.0f) {
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = (i == 3) ? 1.0f : 0.0f;
        return;
    }
    const float sp = sinpif(f);
    const float s4 = sinpif(0.25f * f), c4 = cospif(0.25f * f);
    // sin(pi i / 4), cos(pi i / 4) for i = -3..4
    const float si[8] = {-0.70710678f, -1.0f, -0.70710678f, 0.0f, 0.70710678f, 1.0f, 0.70710678f, 0.0f};
    const float ci[8] = {-0.70710678f, 0.0f, 0.70710678f, 1.0f, 0.70710678f, 0.0f, -0.70710678f, -1.0f};
    const float k = 4.0f / (float(M_PI) * float(M_PI));
    float sum = 0.0f;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int i = t - 3;
        const float x = float(i) - f;
        const float sgn = (i & 1) ? 1.0f : -1.0f;           // (-1)^(i+1)
        const float num = sgn * sp * (si[t] * c4 - ci[t] * s4);
        w[t] = k * num / (x * x);
        sum += w[t];
    }
    const float r = 1.0f / sum;
#pragma unroll
    for (int t = 0; t < 8; ++t) w[t] *= r;
}

// Source coordinate of a view pixel, evaluated term by term in fp64 without contraction
// (the same rounding as a plain left-to-right evaluation of inv * q).
__device__ __forceinline__ double affine_x(const double* m, double qx, double qy) {
    return __dadd_rn(__dadd_rn(__dmul_rn(m[0], qx), __dmul_rn(m[1], qy)), m[2]);
}

template <typename T>
__device__ __forceinline__ float lanczos_sample(const T* __restrict__ S, int W, int H, int ix, int iy,
                                                const float wx[8], const float wy[8]) {
    int cols[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) cols[i] = clampi(ix - 3 + i, 0, W - 1);
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const T* row = S + size_t(clampi(iy - 3 + j, 0, H - 1)) * W;
        float r = 0.0f;
#pragma unroll
        for (int i = 0; i < 8; ++i) r += wx[i] * float(row[cols[i]]);
        acc += wy[j] * r;
    }
    return acc;
}

// One thread per view pixel; all views of the plan in one launch (block -> view by prefix search).
__global__ void __launch_bounds__(256) k_warp(const uint8_t* __restrict__ src, int W, int H, int pitch,
                                              const float* __restrict__ blurred,
                                              const xa_view_desc* __restrict__ views, int n_views,
                                              const int32_t* __restrict__ prefix, uint8_t* __restrict__ arena,
                                              uint8_t* __restrict__ mask, float* __restrict__ values) {
    const int b = blockIdx.x;
    const int vi = find_segment(prefix, n_views, b);
    const xa_view_desc& v = views[vi];
    const int local = b - prefix[vi];
    const int tiles_x = (v.width + kWarpTX - 1) / kWarpTX;
    const int qx = (local % tiles_x) * kWarpTX + (threadIdx.x % kWarpTX);
    const int qy = (local / tiles_x) * kWarpTY + (threadIdx.x / kWarpTX);
    if (qx >= v.width || qy >= v.height) return;
    const size_t o = size_t(v.offset) + size_t(qy) * v.width + qx;
    const double px = affine_x(v.inv, double(qx), double(qy));
    const double py = affine_x(v.inv + 3, double(qx), double(qy));
    const bool inside = px >= -0.5 && px <= W - 0.5 && py >= -0.5 && py <= H - 0.5;
    if (!inside) {
        arena[o] = 0;
        mask[o] = 0;
        if (values) values[o] = 0.0f;
        return;
    }
    const double fxd = floor(px), fyd = floor(py);
    const int ix = int(fxd), iy = int(fyd);
    float wx[8], wy[8];
    lanczos4_weights(float(px - fxd), wx);
    lanczos4_weights(float(py - fyd), wy);
    float val;
    if (v.blur_offset >= 0) {
        val = lanczos_sample(blurred + v.blur_offset, W, H, ix, iy, wx, wy);
    } else if (pitch == W) {
        val = lanczos_sample(src, W, H, ix, iy, wx, wy);
    } else {
        // general pitch: row addressing through the pitch
        int cols[8];
        for (int i = 0; i < 8; ++i) cols[i] = clampi(ix - 3 + i, 0, W - 1);
        val = 0.0f;
        for (int j = 0; j < 8; ++j) {
            const uint8_t* row = src + size_t(clampi(iy - 3 + j, 0, H - 1)) * pitch;
            float r = 0.0f;
            for (int i = 0; i < 8; ++i) r += wx[i] * float(row[cols[i]]);
            val += wy[j] * r;
        }
    }
    const float q = rintf(val);
    arena[o] = uint8_t(q < 0.0f ? 0.0f : (q > 255.0f ? 255.0f : q));
    mask[o] = 1;
    if (values) values[o] = val;
}

}  // namespace

xa_status hip_fail(int err, const char* what) {
    return fail(XA_EHIP, "%s: %s", what, hipGetErrorString(hipError_t(err)));
}

xa_status launch_simulate(const PlanView& ph, const PlanView& pd, const uint8_t* src, int32_t pitch,
                          uint8_t* arena, uint8_t* mask, float* values, float* blurred, hipStream_t st) {
    const xa_plan_header* h = ph.h;
    const int W = h->src_w, H = h->src_h;
    if (h->n_blur > 0) {
        const int tiles = ((W + kBlurTX - 1) / kBlurTX) * ((H + kBlurTY - 1) / kBlurTY);
        hipLaunchKernelGGL(k_blur, dim3(tiles, h->n_blur), dim3(256), 0, st, src, W, H, pitch, pd.views,
                           pd.blur_views, pd.taps, blurred);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "blur launch");
    }
    const int tiles = ph.warp_prefix[h->n_views];
    if (tiles > 0) {
        hipLaunchKernelGGL(k_warp, dim3(tiles), dim3(256), 0, st, src, W, H, pitch, blurred, pd.views, h->n_views,
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

extern "C" xa_status xa_simulate_views(const void* plan_host, const void* plan_dev, const uint8_t* d_src,
                                       int32_t src_pitch, uint8_t* d_arena, uint8_t* d_mask, float* d_values,
                                       void* d_ws, size_t ws_bytes, hipStream_t stream) {
    PlanView ph;
    xa_status s = plan_host_view(plan_host, &ph);
    if (s != XA_OK) return s;
    if (!plan_dev || !d_src || !d_arena || !d_mask) return fail(XA_EINVAL, "NULL device pointer");
    if (src_pitch < ph.h->src_w) return fail(XA_EINVAL, "pitch %d < width %d", src_pitch, ph.h->src_w);
    const size_t need = simulate_ws_bytes(ph.h);
    if (ws_bytes < need) return fail(XA_ECAPACITY, "simulate workspace needs %zu bytes, got %zu", need, ws_bytes);
    if (need > 0 && (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) % kAlign)))
        return fail(XA_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    const PlanView pd = plan_dev_view(plan_host, plan_dev);
    s = launch_simulate(ph, pd, d_src, src_pitch, d_arena, d_mask, d_values, static_cast<float*>(d_ws), stream);
    return s == XA_OK ? ok() : s;
}
