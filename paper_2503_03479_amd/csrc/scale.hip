// Scale stage for the scale parameter of the sampling group (Sec. III.B): images
// are reduced (s < 1, after an isotropic anti-alias Gaussian of standard
// deviation 0.8 sqrt(1/s^2 - 1)) or magnified (s > 1) by Lanczos-4 resampling
// (eqs. (3)-(4)) onto a round(s W) x round(s H) grid at p = (q + 1/2)/s - 1/2,
// taps clamped to the image.  The output is a new source that views use with
// s = 1 in their own map.  All jobs of a plan run in two launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "lanczos.h"

namespace xa {
namespace {

constexpr uint32_t kScaleMagic = 0x58414653u;   // "XAFS"
constexpr int kSTX = 64, kSTY = 16;             // blur and resample tiles (256 threads, 4 rows each)
constexpr int kSMaxK = 26;                      // largest Gaussian half-width (s >= 1/8)
constexpr int kSLds = (kSTX + 2 * kSMaxK) * (kSTY + 2 * kSMaxK);

struct ScaleJob {
    xa_source_desc src, dst;
    double s;
    float sigma;
    int32_t K;              // Gaussian taps -K..K, 0 = no blur
    int32_t tap0;           // first Gaussian weight
    int32_t pad;
    int64_t blur_offset;    // float offset of the blurred source in the workspace, -1 if none
};

struct ScaleHeader {
    uint32_t magic, version;
    int32_t n_jobs, n_taps;
    int64_t blur_floats;
    int64_t total_bytes;
    int64_t off_jobs, off_taps, off_blur_prefix, off_warp_prefix;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

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

// Isotropic Gaussian of one job's source: the tile plus a K halo (border replicated at load)
// is staged in LDS, blurred along x into LDS, then along y into the workspace (fp32).
__global__ void __launch_bounds__(256) k_sblur(const ScaleJob* __restrict__ jobs, const int32_t* __restrict__ prefix,
                                               int n_jobs, const float* __restrict__ taps,
                                               const uint8_t* __restrict__ sources, float* __restrict__ out) {
    __shared__ float a[kSLds];
    __shared__ float hx[(kSTY + 2 * kSMaxK) * kSTX];
    const int ji = find_segment_wave(prefix, n_jobs, blockIdx.x);
    const ScaleJob& j = jobs[ji];
    const int W = j.src.width, H = j.src.height, K = j.K;
    const uint8_t* src = sources + j.src.offset;
    const int local = blockIdx.x - prefix[ji];
    const int tiles_x = (W + kSTX - 1) / kSTX;
    const int x0 = (local % tiles_x) * kSTX, y0 = (local / tiles_x) * kSTY;
    const int rw = kSTX + 2 * K, rh = kSTY + 2 * K;
    for (int e = threadIdx.x; e < rw * rh; e += 256) {
        const int r = e / rw, c = e - (e / rw) * rw;
        a[e] = float(src[size_t(clampi(y0 - K + r, 0, H - 1)) * j.src.pitch + clampi(x0 - K + c, 0, W - 1)]);
    }
    __syncthreads();
    const float* g = taps + j.tap0;
    for (int e = threadIdx.x; e < rh * kSTX; e += 256) {
        const int r = e / kSTX, c = e - (e / kSTX) * kSTX;
        float acc = 0.0f;
        for (int k = 0; k <= 2 * K; ++k) acc = fmaf(g[k], a[r * rw + c + k], acc);
        hx[e] = acc;
    }
    __syncthreads();
    float* o = out + j.blur_offset;
    for (int rr = 0; rr < kSTY / 4; ++rr) {
        const int c = threadIdx.x % kSTX, r = threadIdx.x / kSTX + 4 * rr;
        const int x = x0 + c, y = y0 + r;
        if (x >= W || y >= H) continue;
        float acc = 0.0f;
        for (int k = 0; k <= 2 * K; ++k) acc = fmaf(g[k], hx[(r + k) * kSTX + c], acc);
        o[size_t(y) * W + x] = acc;
    }
}

// Lanczos-4 resampling of one job onto its output grid: p = (q + 1/2)/s - 1/2 per axis,
// taps clamped, value normalised by the weight sums, rounded half to even into the u8 output.
__global__ void __launch_bounds__(256) k_swarp(const ScaleJob* __restrict__ jobs, const int32_t* __restrict__ prefix,
                                               int n_jobs, uint8_t* __restrict__ sources,
                                               const float* __restrict__ blurred, float* __restrict__ values) {
    const int ji = find_segment_wave(prefix, n_jobs, blockIdx.x);
    const ScaleJob& j = jobs[ji];
    const int W = j.src.width, H = j.src.height;
    const int local = blockIdx.x - prefix[ji];
    const int tiles_x = (j.dst.width + kSTX - 1) / kSTX;
    const int x = (local % tiles_x) * kSTX + threadIdx.x % kSTX;
    const int ybase = (local / tiles_x) * kSTY + threadIdx.x / kSTX;
    if (x >= j.dst.width) return;
    const double px = __dadd_rn(__dadd_rn(double(x), 0.5) / j.s, -0.5);
    const double fxd = floor(px);
    const int ix = int(fxd);
    float wx[8];
    const float sx = lanczos4_weights(float(px - fxd), wx);
    int cols[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) cols[i] = clampi(ix - 3 + i, 0, W - 1);
    for (int rr = 0; rr < kSTY / 4; ++rr) {
        const int y = ybase + 4 * rr;
        if (y >= j.dst.height) break;
        const double py = __dadd_rn(__dadd_rn(double(y), 0.5) / j.s, -0.5);
        const double fyd = floor(py);
        const int iy = int(fyd);
        float wy[8];
        const float sy = lanczos4_weights(float(py - fyd), wy);
        float acc = 0.0f;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int row = clampi(iy - 3 + r, 0, H - 1);
            float sacc = 0.0f;
            if (j.blur_offset >= 0) {
                const float* s = blurred + j.blur_offset + size_t(row) * W;
#pragma unroll
                for (int i = 0; i < 8; ++i) sacc += wx[i] * s[cols[i]];
            } else {
                const uint8_t* s = sources + j.src.offset + size_t(row) * j.src.pitch;
#pragma unroll
                for (int i = 0; i < 8; ++i) sacc += wx[i] * float(s[cols[i]]);
            }
            acc += wy[r] * sacc;
        }
        const float val = acc * __builtin_amdgcn_rcpf(sx * sy);
        const float q = rintf(val);
        sources[j.dst.offset + size_t(y) * j.dst.pitch + x] = uint8_t(q < 0.0f ? 0.0f : (q > 255.0f ? 255.0f : q));
        if (values) values[j.dst.offset + size_t(y) * j.dst.pitch + x] = val;
    }
}

struct ScaleView {
    const ScaleHeader* h;
    const ScaleJob* jobs;
    const float* taps;
    const int32_t* blur_prefix;
    const int32_t* warp_prefix;
};

ScaleView scale_view(const void* blob, const void* base) {
    const auto* h = static_cast<const ScaleHeader*>(blob);
    const char* b = static_cast<const char*>(base);
    return ScaleView{reinterpret_cast<const ScaleHeader*>(b), reinterpret_cast<const ScaleJob*>(b + h->off_jobs),
                     reinterpret_cast<const float*>(b + h->off_taps),
                     reinterpret_cast<const int32_t*>(b + h->off_blur_prefix),
                     reinterpret_cast<const int32_t*>(b + h->off_warp_prefix)};
}

bool sizes_overflow(int32_t w, int32_t h, double s) {
    return !(s > 0.0) || !std::isfinite(s) || s * w > 32768.0 || s * h > 32768.0;
}

}  // namespace
}  // namespace xa

using namespace xa;

extern "C" xa_status xa_scaled_size(int32_t w, int32_t h, double s, int32_t* out_w, int32_t* out_h) {
    if (!out_w || !out_h || w < 1 || h < 1 || sizes_overflow(w, h, s))
        return fail(XA_EINVAL, "bad size or scale");
    *out_w = std::max(1, int32_t(std::floor(s * w + 0.5)));
    *out_h = std::max(1, int32_t(std::floor(s * h + 0.5)));
    return ok();
}

extern "C" xa_status xa_plan_scales(const xa_scale_job* jobs, int32_t n_jobs, void* blob, size_t blob_cap,
                                    size_t* blob_bytes) {
    if (!blob_bytes || n_jobs < 1 || !jobs) return fail(XA_EINVAL, "need at least one job");
    std::vector<ScaleJob> js(n_jobs);
    std::vector<float> taps;
    std::vector<int32_t> wp;
    int64_t blur_floats = 0, bt = 0, wt = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const xa_scale_job& q = jobs[i];
        int32_t ow, oh;
        if (xa_scaled_size(q.src.width, q.src.height, q.s, &ow, &oh) != XA_OK)
            return fail(XA_EINVAL, "job %d: bad source size or scale", i);
        if (q.dst.width != ow || q.dst.height != oh)
            return fail(XA_EINVAL, "job %d: destination must be %dx%d", i, ow, oh);
        if (q.src.pitch < q.src.width || q.dst.pitch < q.dst.width || q.src.offset < 0 || q.dst.offset < 0)
            return fail(XA_EINVAL, "job %d: bad pitch or offset", i);
        ScaleJob& j = js[i];
        std::memset(&j, 0, sizeof(j));
        j.src = q.src;
        j.dst = q.dst;
        j.s = q.s;
        j.blur_offset = -1;
        if (q.s < 1.0) {
            const double sigma = 0.8 * std::sqrt(1.0 / (q.s * q.s) - 1.0);
            const int K = int(std::ceil(4.0 * sigma));
            if (K > kSMaxK) return fail(XA_EUNSUPPORTED, "job %d: scale %g below the supported 1/8", i, q.s);
            j.sigma = float(sigma);
            j.K = K;
            j.tap0 = int32_t(taps.size());
            double sum = 0.0;
            std::vector<double> g(2 * K + 1);
            for (int k = -K; k <= K; ++k) sum += (g[k + K] = std::exp(-double(k) * k / (2.0 * sigma * sigma)));
            for (int k = 0; k <= 2 * K; ++k) taps.push_back(float(g[k] / sum));
            j.blur_offset = blur_floats;
            blur_floats += int64_t(q.src.width) * q.src.height;
        }
        if (j.K > 0) bt += int64_t((q.src.width + kSTX - 1) / kSTX) * ((q.src.height + kSTY - 1) / kSTY);
        wp.push_back(int32_t(wt));
        wt += int64_t((ow + kSTX - 1) / kSTX) * ((oh + kSTY - 1) / kSTY);
    }
    // blur tiles per job (zero for jobs without a blur; the prefix search skips empty segments)
    std::vector<int32_t> bpa(n_jobs + 1, 0);
    {
        int64_t acc = 0;
        for (int i = 0; i < n_jobs; ++i) {
            bpa[i] = int32_t(acc);
            if (js[i].K > 0)
                acc += int64_t((js[i].src.width + kSTX - 1) / kSTX) * ((js[i].src.height + kSTY - 1) / kSTY);
        }
        bpa[n_jobs] = int32_t(acc);
    }
    wp.push_back(int32_t(wt));
    if (bt > INT32_MAX / 2 || wt > INT32_MAX / 2) return fail(XA_EUNSUPPORTED, "too many tiles");
    ScaleHeader h{};
    h.magic = kScaleMagic;
    h.version = 1;
    h.n_jobs = n_jobs;
    h.n_taps = int32_t(taps.size());
    h.blur_floats = blur_floats;
    size_t o = align_up(sizeof(ScaleHeader), 64);
    h.off_jobs = int64_t(o);        o = align_up(o + sizeof(ScaleJob) * n_jobs, 64);
    h.off_taps = int64_t(o);        o = align_up(o + sizeof(float) * taps.size(), 64);
    h.off_blur_prefix = int64_t(o); o = align_up(o + 4 * bpa.size(), 64);
    h.off_warp_prefix = int64_t(o); o = align_up(o + 4 * wp.size(), 64);
    h.total_bytes = int64_t(o);
    *blob_bytes = o;
    if (!blob) return ok();
    if (blob_cap < o) return fail(XA_ECAPACITY, "scale plan needs %zu bytes, buffer has %zu", o, blob_cap);
    char* b = static_cast<char*>(blob);
    std::memset(b, 0, o);
    std::memcpy(b, &h, sizeof(h));
    std::memcpy(b + h.off_jobs, js.data(), sizeof(ScaleJob) * n_jobs);
    if (!taps.empty()) std::memcpy(b + h.off_taps, taps.data(), sizeof(float) * taps.size());
    std::memcpy(b + h.off_blur_prefix, bpa.data(), 4 * bpa.size());
    std::memcpy(b + h.off_warp_prefix, wp.data(), 4 * wp.size());
    return ok();
}

extern "C" size_t xa_scale_workspace_size(const void* splan_host) {
    if (!splan_host || static_cast<const ScaleHeader*>(splan_host)->magic != kScaleMagic) return 0;
    return align_up(size_t(static_cast<const ScaleHeader*>(splan_host)->blur_floats) * 4);
}

namespace xa {
xa_status launch_scale(const void* splan_host, const void* splan_dev, uint8_t* d_sources, float* d_values,
                       void* d_ws, hipStream_t stream) {
    const ScaleView hv = scale_view(splan_host, splan_host), dv = scale_view(splan_host, splan_dev);
    const int n = hv.h->n_jobs;
    const int bt = hv.blur_prefix[n], wt = hv.warp_prefix[n];
    float* blurred = static_cast<float*>(d_ws);
    if (bt > 0)
        hipLaunchKernelGGL(k_sblur, dim3(bt), dim3(256), 0, stream, dv.jobs, dv.blur_prefix, n, dv.taps, d_sources,
                           blurred);
    if (wt > 0)
        hipLaunchKernelGGL(k_swarp, dim3(wt), dim3(256), 0, stream, dv.jobs, dv.warp_prefix, n, d_sources, blurred,
                           d_values);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "scale launch");
    return XA_OK;
}
bool is_scale_plan(const void* blob) {
    return blob && static_cast<const ScaleHeader*>(blob)->magic == kScaleMagic;
}
}  // namespace xa

extern "C" xa_status xa_scale_sources(const void* splan_host, const void* splan_dev, uint8_t* d_sources,
                                      float* d_values, void* d_ws, size_t ws_bytes, hipStream_t stream) {
    if (!splan_host || static_cast<const ScaleHeader*>(splan_host)->magic != kScaleMagic)
        return fail(XA_EINVAL, "not a scale plan");
    if (!splan_dev || !d_sources) return fail(XA_EINVAL, "NULL device pointer");
    const size_t need = xa_scale_workspace_size(splan_host);
    if (ws_bytes < need) return fail(XA_ECAPACITY, "scale workspace needs %zu bytes, got %zu", need, ws_bytes);
    if (need > 0 && (!d_ws || reinterpret_cast<uintptr_t>(d_ws) % kAlign))
        return fail(XA_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    const xa_status s = launch_scale(splan_host, splan_dev, d_sources, d_values, d_ws, stream);
    return s == XA_OK ? ok() : s;
}
