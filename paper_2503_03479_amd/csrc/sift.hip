// SIFT keypoints and 128-D descriptors on one 8-bit image: the detector and descriptor of Lowe
// [14] that the method uses to pick the base image (Sec. III.A, eq. (1)) and to match the
// re-simulated reference against the target (Sec. III.C).
//
// Readings of [14] (the paper does not restate SIFT): intensities as fp32 0..255, input blur
// 0.5, sigma0 = 1.6, s layers per octave (s + 3 Gaussian images, s + 2 DoG images), no initial
// doubling, floor(log2 min(W, H)) - 3 octaves, the next octave from every second pixel of G_s.
// Gaussian taps exp(-k^2 / 2 sigma^2), |k| <= ceil(4 sigma), normalised in fp64 on the host
// and rounded to fp32; replicated borders; each separable pass sums w_k v_k from k = -r to r in
// fp32 with every product and sum rounded (no fused multiply-add), rows before columns.  The
// scale space is therefore the same bits as any evaluation in that order.
//
// Candidates are strict 26-neighbour extrema of layers 1..s, 5 pixels inside the border, with
// |D| above half the contrast threshold.  The quadratic fit of [14] runs in fp64 from the fp32
// DoG values in a fixed operation order and decides without dividing: with n = -adj(H) g, a
// sample converges when |n_i| < |det| / 2 for all i, else it moves one sample towards each
// component with |n_i| >= |det| / 2 (5 fits at most, rejected when it leaves layers 1..s or the
// border region); contrast |D det + g.n / 2| >= 255 (c / s) |det|; edge tr^2 r < (r + 1)^2 det2,
// det2 > 0.  The keypoint set is therefore exact.
//
// Orientation: a 36-bin histogram of atan2(dy, dx) (image axes) over the square of radius
// round(4.5 sigma), weighted by magnitude and a Gaussian of 1.5 sigma, smoothed by
// (1 4 6 4 1) / 16, every local peak >= 0.8 of the highest, refined by a parabola.  Descriptor:
// 4 x 4 cells of 3 sigma by 8 direction bins over the window turned to the angle, Gaussian
// weight of 2 cells, trilinear spreading, unit norm, clip 0.2, renormalise, min(255,
// floor(512 v + 1/2)).  Histograms are summed as int64 fixed point in LDS (2^-40 and 2^-32
// units), so they do not depend on the order of the atomics: the outputs are deterministic, and
// they differ from an fp64 sum only by those roundings.
//
// Order: keypoints come in the order of their candidates (octave, candidate layer, row,
// column), the peaks of one candidate in bin order.  Candidates are counted per row, the counts
// scanned, then written at their row's offset in column order: no atomics decide an order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace xa {
namespace {

constexpr int kSiftBorder = 5;
constexpr int kSiftFitSteps = 5;
constexpr int kSiftMaxLayers = 5;
constexpr int kSiftMaxOctaves = 16;
constexpr int kSiftMaxTaps = 64;            // 2 r + 1 for sigma up to 7.8
constexpr int kOriBins = 36;
constexpr int kMaxPeaks = kOriBins / 2;     // local maxima of a circular 36-bin histogram
constexpr double kOriScale = 1099511627776.0;   // 2^40: orientation histogram fixed point
constexpr double kDescScale = 4294967296.0;     // 2^32: descriptor histogram fixed point
constexpr double kPi = 3.141592653589793;

struct Taps {
    float w[kSiftMaxTaps];
    int r;
};

// Raw keypoint after the fit.
struct RawKp {
    int o, k, xi, yi;
    double x, y, sigma_oct, size, response;
};

struct PeakSet {
    int n, pad;
    int bin[kMaxPeaks];
    double angle[kMaxPeaks];
};

struct Octave {
    int w, h;
    size_t gauss;      // float offset of G_0 (images of w * h floats, G_0 .. G_(s+2), then D_0 .. D_(s+1))
    int row0;          // first entry of this octave in the row-count table
    int rows;          // rows per layer scanned for candidates (h - 2 border, at least 0)
};

struct SiftGeom {
    int n_oct, s;
    Octave oct[kSiftMaxOctaves];
    size_t floats;     // scale space and a temporary image
    size_t tmp;        // float offset of the temporary image
    int total_rows;
    int raw_cap;
    // byte offsets in the workspace
    size_t off_floats, off_rowcount, off_rowoff, off_raw, off_peaks, off_kpoff, off_counters, total;
};

// ------------------------------------------------------------------ scale space

#pragma clang fp contract(off)

template <typename T>
__global__ void __launch_bounds__(256) k_sift_hblur(const T* __restrict__ src, int pitch, int w, int h, Taps t,
                                                    float* __restrict__ dst) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= w) return;
    const T* row = src + size_t(y) * pitch;
    float acc = 0.0f;
    for (int k = -t.r; k <= t.r; ++k) {
        const float v = float(row[min(max(x + k, 0), w - 1)]);
        acc = acc + t.w[k + t.r] * v;
    }
    dst[size_t(y) * w + x] = acc;
}

__global__ void __launch_bounds__(256) k_sift_vblur(const float* __restrict__ src, int w, int h, Taps t,
                                                    float* __restrict__ dst) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= w) return;
    float acc = 0.0f;
    for (int k = -t.r; k <= t.r; ++k) {
        const float v = src[size_t(min(max(y + k, 0), h - 1)) * w + x];
        acc = acc + t.w[k + t.r] * v;
    }
    dst[size_t(y) * w + x] = acc;
}

// G_0 of octave o + 1: every second pixel of G_s of octave o.
__global__ void __launch_bounds__(256) k_sift_down(const float* __restrict__ src, int ws, float* __restrict__ dst,
                                                   int w, int h) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= w) return;
    dst[size_t(y) * w + x] = src[size_t(2 * y) * ws + 2 * x];
}

// D_k = G_(k+1) - G_k for k = 0 .. n - 1.
__global__ void __launch_bounds__(256) k_sift_dog(const float* __restrict__ g, float* __restrict__ d, size_t plane,
                                                  int n) {
    const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= plane) return;
    for (int k = 0; k < n; ++k) d[size_t(k) * plane + i] = g[size_t(k + 1) * plane + i] - g[size_t(k) * plane + i];
}

// ------------------------------------------------------------------ candidates and the fit

struct FitParams {
    double pre;        // half the contrast threshold
    double thr;        // 255 c / s
    double edge;       // r
    double sigma0;
    int s;
};

__device__ inline bool is_extremum(const float* __restrict__ D, size_t plane, int w, int k, int y, int x,
                                   double pre) {
    const float c = D[size_t(k) * plane + size_t(y) * w + x];
    if (!(fabs(double(c)) > pre)) return false;
    bool mx = c > 0.0f, mn = c < 0.0f;
    for (int dk = -1; dk <= 1; ++dk)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dk == 0 && dy == 0 && dx == 0) continue;
                const float v = D[size_t(k + dk) * plane + size_t(y + dy) * w + (x + dx)];
                mx = mx && c > v;
                mn = mn && c < v;
            }
    return mx || mn;
}

// The fit of candidate (k, y, x) of one octave's DoG stack; true and *out when accepted.  The
// operation order is that of the plain definition the tests hold it to.
__device__ bool localise(const float* __restrict__ D, size_t plane, int w, int h, int o, int k, int y, int x,
                         const FitParams& P, RawKp* out) {
    bool conv = false;
    double c = 0, g0 = 0, g1 = 0, g2 = 0, dxx = 0, dyy = 0, dxy = 0, det = 0, n0 = 0, n1 = 0, n2 = 0;
    for (int it = 0; it < kSiftFitSteps; ++it) {
        const float* Dm = D + size_t(k - 1) * plane;
        const float* D0 = D + size_t(k) * plane;
        const float* Dp = D + size_t(k + 1) * plane;
        auto f = [&](const float* L, int yy, int xx) { return double(L[size_t(yy) * w + xx]); };
        c = f(D0, y, x);
        g0 = (f(D0, y, x + 1) - f(D0, y, x - 1)) * 0.5;
        g1 = (f(D0, y + 1, x) - f(D0, y - 1, x)) * 0.5;
        g2 = (f(Dp, y, x) - f(Dm, y, x)) * 0.5;
        const double v2 = c * 2.0;
        dxx = (f(D0, y, x + 1) + f(D0, y, x - 1)) - v2;
        dyy = (f(D0, y + 1, x) + f(D0, y - 1, x)) - v2;
        const double dss = (f(Dp, y, x) + f(Dm, y, x)) - v2;
        dxy = ((f(D0, y + 1, x + 1) - f(D0, y + 1, x - 1)) - (f(D0, y - 1, x + 1) - f(D0, y - 1, x - 1))) * 0.25;
        const double dxs = ((f(Dp, y, x + 1) - f(Dp, y, x - 1)) - (f(Dm, y, x + 1) - f(Dm, y, x - 1))) * 0.25;
        const double dys = ((f(Dp, y + 1, x) - f(Dp, y - 1, x)) - (f(Dm, y + 1, x) - f(Dm, y - 1, x))) * 0.25;
        const double a00 = dyy * dss - dys * dys;
        const double a01 = dxs * dys - dxy * dss;
        const double a02 = dxy * dys - dyy * dxs;
        const double a11 = dxx * dss - dxs * dxs;
        const double a12 = dxy * dxs - dxx * dys;
        const double a22 = dxx * dyy - dxy * dxy;
        det = (dxx * a00 + dxy * a01) + dxs * a02;
        n0 = -((a00 * g0 + a01 * g1) + a02 * g2);
        n1 = -((a01 * g0 + a11 * g1) + a12 * g2);
        n2 = -((a02 * g0 + a12 * g1) + a22 * g2);
        if (det == 0.0) return false;
        const double half = 0.5 * fabs(det);
        if (fabs(n0) < half && fabs(n1) < half && fabs(n2) < half) {
            conv = true;
            break;
        }
        const bool pos = det > 0.0;
        x += fabs(n0) < half ? 0 : (((n0 > 0.0) == pos) ? 1 : -1);
        y += fabs(n1) < half ? 0 : (((n1 > 0.0) == pos) ? 1 : -1);
        k += fabs(n2) < half ? 0 : (((n2 > 0.0) == pos) ? 1 : -1);
        if (k < 1 || k > P.s || x < kSiftBorder || x >= w - kSiftBorder || y < kSiftBorder || y >= h - kSiftBorder)
            return false;
    }
    if (!conv) return false;
    const double ad = fabs(det);
    const double t = (g0 * n0 + g1 * n1) + g2 * n2;
    const double lhs = fabs(c * det + 0.5 * t);
    if (lhs < P.thr * ad) return false;
    const double tr = dxx + dyy;
    const double d2 = dxx * dyy - dxy * dxy;
    if (d2 <= 0.0 || tr * tr * P.edge >= (P.edge + 1.0) * (P.edge + 1.0) * d2) return false;
    const double ox = n0 / det, oy = n1 / det, os = n2 / det;
    const double sigma_oct = P.sigma0 * pow(2.0, (double(k) + os) / double(P.s));
    const double scale = double(1 << o);
    out->o = o;
    out->k = k;
    out->xi = x;
    out->yi = y;
    out->x = (double(x) + ox) * scale;
    out->y = (double(y) + oy) * scale;
    out->sigma_oct = sigma_oct;
    out->size = sigma_oct * scale;
    out->response = lhs / ad;
    return true;
}

// Exclusive block scan of one int per thread (256 threads); returns the block total.
__device__ int block_scan(int v, int* excl) {
    __shared__ int s[256];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int a = int(threadIdx.x) >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += a;
        __syncthreads();
    }
    *excl = s[threadIdx.x] - v;
    const int total = s[255];
    __syncthreads();
    return total;
}

// One block per (layer, row) of an octave: pass 0 counts the row's accepted candidates, pass 1
// writes them (below the raw capacity) at the row's offset, in column order.
template <int PASS>
__global__ void __launch_bounds__(256) k_sift_rows(const float* __restrict__ D, int w, int h, int o, int row0,
                                                   int rows, FitParams P, int* __restrict__ rowcount,
                                                   const int* __restrict__ rowoff, int raw_cap,
                                                   RawKp* __restrict__ raw) {
    const int k = 1 + int(blockIdx.x) / rows, y = kSiftBorder + int(blockIdx.x) % rows;
    const size_t plane = size_t(w) * h;
    int base = PASS == 1 ? rowoff[row0 + blockIdx.x] : 0, count = 0;
    for (int x0 = kSiftBorder; x0 < w - kSiftBorder; x0 += 256) {
        const int x = x0 + int(threadIdx.x);
        RawKp kp;
        const bool acc = x < w - kSiftBorder && is_extremum(D, plane, w, k, y, x, P.pre) &&
                         localise(D, plane, w, h, o, k, y, x, P, &kp);
        int excl;
        const int tot = block_scan(acc ? 1 : 0, &excl);
        if (PASS == 1 && acc && base + count + excl < raw_cap) raw[base + count + excl] = kp;
        count += tot;
    }
    if (PASS == 0 && threadIdx.x == 0) rowcount[row0 + blockIdx.x] = count;
}

// Exclusive scan of n ints (one block of 256 threads, n / 256 per thread); off[n] = total.
__global__ void __launch_bounds__(256) k_sift_scan(const int* __restrict__ in, int n, int* __restrict__ off) {
    __shared__ int s[256];
    const int per = (n + 255) / 256, b = int(threadIdx.x) * per;
    int sum = 0;
    for (int i = 0; i < per && b + i < n; ++i) sum += in[b + i];
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int a = int(threadIdx.x) >= d ? s[threadIdx.x - d] : 0;
        __syncthreads();
        s[threadIdx.x] += a;
        __syncthreads();
    }
    int run = s[threadIdx.x] - sum;
    for (int i = 0; i < per && b + i < n; ++i) {
        off[b + i] = run;
        run += in[b + i];
    }
    if (threadIdx.x == 255) off[n] = s[255];
}

// ------------------------------------------------------------------ orientation and descriptor

__device__ inline const float* gauss_image(const float* fl, const Octave* oct, int o, int k) {
    return fl + oct[o].gauss + size_t(k) * size_t(oct[o].w) * oct[o].h;
}

struct OctaveTable {
    Octave oct[kSiftMaxOctaves];
};

// One wave per raw keypoint: the fixed-point histogram in LDS, then the peaks.
__global__ void __launch_bounds__(64) k_sift_orient(const float* __restrict__ fl, OctaveTable T,
                                                    const RawKp* __restrict__ raw, const int* __restrict__ n_raw,
                                                    int raw_cap, PeakSet* __restrict__ peaks) {
    __shared__ unsigned long long hist[kOriBins];
    const int i = blockIdx.x;
    const int n = min(*n_raw, raw_cap);
    if (i >= n) return;
    const RawKp kp = raw[i];
    const Octave& oc = T.oct[kp.o];
    const int w = oc.w, h = oc.h;
    const float* G = gauss_image(fl, T.oct, kp.o, kp.k);
    if (threadIdx.x < kOriBins) hist[threadIdx.x] = 0ull;
    __syncthreads();
    const int R = int(floor(4.5 * kp.sigma_oct + 0.5));
    const double sw = 1.5 * kp.sigma_oct;
    const double expf_ = -1.0 / (2.0 * sw * sw);
    const int side = 2 * R + 1;
    const double to_bin = double(kOriBins) / (2.0 * kPi);
    for (int e = threadIdx.x; e < side * side; e += 64) {
        const int ii = e / side - R, jj = e % side - R;
        const int yy = kp.yi + ii, xx = kp.xi + jj;
        if (yy <= 0 || yy >= h - 1 || xx <= 0 || xx >= w - 1) continue;
        const double dx = double(G[size_t(yy) * w + xx + 1]) - double(G[size_t(yy) * w + xx - 1]);
        const double dy = double(G[size_t(yy + 1) * w + xx]) - double(G[size_t(yy - 1) * w + xx]);
        const double wgt = exp(double(ii * ii + jj * jj) * expf_);
        const double mag = sqrt(dx * dx + dy * dy);
        const double ang = atan2(dy, dx);
        int b = int(floor(ang * to_bin + 0.5)) % kOriBins;
        if (b < 0) b += kOriBins;
        atomicAdd(&hist[b], (unsigned long long)(__double2ll_rn(wgt * mag * kOriScale)));
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double hv[kOriBins], sm[kOriBins];
    for (int b = 0; b < kOriBins; ++b) hv[b] = double((long long)hist[b]) / kOriScale;
    double mx = 0.0;
    for (int b = 0; b < kOriBins; ++b) {
        const int bm2 = (b + kOriBins - 2) % kOriBins, bm1 = (b + kOriBins - 1) % kOriBins;
        const int bp1 = (b + 1) % kOriBins, bp2 = (b + 2) % kOriBins;
        sm[b] = (hv[bm2] + hv[bp2]) * (1.0 / 16.0) + (hv[bm1] + hv[bp1]) * (4.0 / 16.0) + hv[b] * (6.0 / 16.0);
        mx = b == 0 ? sm[b] : fmax(mx, sm[b]);
    }
    PeakSet P;
    P.n = 0;
    P.pad = 0;
    for (int b = 0; b < kOriBins; ++b) {
        const double l = sm[(b + kOriBins - 1) % kOriBins], c = sm[b], r = sm[(b + 1) % kOriBins];
        if (c > l && c > r && c >= 0.8 * mx && P.n < kMaxPeaks) {
            double bf = double(b) + 0.5 * (l - r) / ((l - 2.0 * c) + r);
            if (bf < 0.0) bf += kOriBins;
            else if (bf >= kOriBins) bf -= kOriBins;
            double ang = bf * (2.0 * kPi / kOriBins);
            if (ang >= 2.0 * kPi) ang -= 2.0 * kPi;
            P.bin[P.n] = b;
            P.angle[P.n] = ang;
            ++P.n;
        }
    }
    peaks[i] = P;
}

// off[i] = oriented keypoints of raw keypoints 0..i-1 (one block), then the counts.
__global__ void __launch_bounds__(256) k_sift_scan_peaks(const PeakSet* __restrict__ peaks,
                                                         const int* __restrict__ n_raw, int raw_cap,
                                                         int* __restrict__ off, int max_kp, int* __restrict__ count) {
    __shared__ int s[256];
    const int n = min(*n_raw, raw_cap);
    const int per = (n + 255) / 256, b = int(threadIdx.x) * per;
    int sum = 0;
    for (int i = 0; i < per && b + i < n; ++i) sum += peaks[b + i].n;
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int a = int(threadIdx.x) >= d ? s[threadIdx.x - d] : 0;
        __syncthreads();
        s[threadIdx.x] += a;
        __syncthreads();
    }
    int run = s[threadIdx.x] - sum;
    for (int i = 0; i < per && b + i < n; ++i) {
        off[b + i] = run;
        run += peaks[b + i].n;
    }
    if (threadIdx.x == 255) {
        off[n] = s[255];
        count[0] = min(s[255], max_kp);
        count[1] = s[255];
    }
}

// One wave per kept keypoint: its raw keypoint and peak, the keypoint record and the descriptor.
__global__ void __launch_bounds__(64) k_sift_desc(const float* __restrict__ fl, OctaveTable T,
                                                  const RawKp* __restrict__ raw, const PeakSet* __restrict__ peaks,
                                                  const int* __restrict__ n_raw, int raw_cap,
                                                  const int* __restrict__ off, const int* __restrict__ count,
                                                  xa_sift_keypoint* __restrict__ out_kp, uint8_t* __restrict__ out_desc) {
    __shared__ unsigned long long hist[6 * 6 * 8];
    __shared__ double red[64];
    const int q = blockIdx.x;
    if (q >= count[0]) return;
    // raw keypoint r with off[r] <= q < off[r + 1]
    const int n = min(*n_raw, raw_cap);
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    const RawKp kp = raw[lo];
    const int pk = q - off[lo];
    const double theta = peaks[lo].angle[pk];
    const Octave& oc = T.oct[kp.o];
    const int w = oc.w, h = oc.h;
    const float* G = gauss_image(fl, T.oct, kp.o, kp.k);
    for (int e = threadIdx.x; e < 6 * 6 * 8; e += 64) hist[e] = 0ull;
    __syncthreads();
    constexpr int d = 4, nb = 8;
    const double hw = 3.0 * kp.sigma_oct;
    int radius = int(floor(hw * sqrt(2.0) * (d + 1) * 0.5 + 0.5));
    radius = min(radius, int(sqrt(double(w) * w + double(h) * h)));
    const double ct = cos(theta) / hw, st = sin(theta) / hw;
    const double bins_per_rad = nb / (2.0 * kPi);
    const double expf_ = -1.0 / (0.5 * d * d);
    const int side = 2 * radius + 1;
    for (int e = threadIdx.x; e < side * side; e += 64) {
        const double ii = double(e / side - radius), jj = double(e % side - radius);
        const double c_rot = jj * ct + ii * st;
        const double r_rot = ii * ct - jj * st;
        const double rbin = r_rot + (d / 2 - 0.5), cbin = c_rot + (d / 2 - 0.5);
        const int yy = kp.yi + int(ii), xx = kp.xi + int(jj);
        if (!(rbin > -1.0 && rbin < d && cbin > -1.0 && cbin < d && yy > 0 && yy < h - 1 && xx > 0 && xx < w - 1))
            continue;
        const double dx = double(G[size_t(yy) * w + xx + 1]) - double(G[size_t(yy) * w + xx - 1]);
        const double dy = double(G[size_t(yy + 1) * w + xx]) - double(G[size_t(yy - 1) * w + xx]);
        const double mag = sqrt(dx * dx + dy * dy);
        const double ang = atan2(dy, dx);
        const double wgt = exp((c_rot * c_rot + r_rot * r_rot) * expf_);
        double ob = (ang - theta) * bins_per_rad;
        if (ob < 0.0) ob += nb;
        if (ob < 0.0) ob += nb;
        if (ob >= nb) ob -= nb;
        const double v = mag * wgt;
        const double r0 = floor(rbin), c0 = floor(cbin), o0 = floor(ob);
        const double fr = rbin - r0, fc = cbin - c0, fo = ob - o0;
        const int ir = int(r0) + 1, ic = int(c0) + 1, io = int(o0) % nb;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const double wr = a ? fr : 1.0 - fr, wc = b ? fc : 1.0 - fc, wo = c ? fo : 1.0 - fo;
                    const double val = v * wr * wc * wo;
                    atomicAdd(&hist[((ir + a) * 6 + (ic + b)) * nb + (io + c) % nb],
                              (unsigned long long)(__double2ll_rn(val * kDescScale)));
                }
    }
    __syncthreads();
    // the inner 4 x 4 x 8 values, two per lane: element t = (r * 4 + c) * 8 + o
    double v[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int t = threadIdx.x + 64 * u;
        const int r = t / 32, c = (t / 8) % 4, o = t % 8;
        v[u] = double((long long)hist[((r + 1) * 6 + (c + 1)) * nb + o]) / kDescScale;
    }
    auto wave_sum = [&](double x) {
        red[threadIdx.x] = x;
        __syncthreads();
        double s = 0.0;
        for (int l = 0; l < 64; ++l) s += red[l];
        __syncthreads();
        return s;
    };
    const double nrm = sqrt(wave_sum(v[0] * v[0] + v[1] * v[1]));
    const double thr = 0.2 * nrm;
    v[0] = fmin(v[0], thr);
    v[1] = fmin(v[1], thr);
    const double nrm2 = sqrt(wave_sum(v[0] * v[0] + v[1] * v[1]));
    const double scale = 512.0 / fmax(nrm2, 1.1920928955078125e-07);
#pragma unroll
    for (int u = 0; u < 2; ++u)
        out_desc[size_t(q) * 128 + threadIdx.x + 64 * u] = uint8_t(fmin(floor(v[u] * scale + 0.5), 255.0));
    if (threadIdx.x == 0) {
        xa_sift_keypoint K;
        K.x = float(kp.x);
        K.y = float(kp.y);
        K.size = float(kp.size);
        K.angle = float(theta);
        K.response = float(kp.response);
        K.xi = kp.xi;
        K.yi = kp.yi;
        K.octave = int8_t(kp.o);
        K.layer = int8_t(kp.k);
        K.peak = int8_t(peaks[lo].bin[pk]);
        K.pad = 0;
        out_kp[q] = K;
    }
}

// Accepted L2 matches (nearest train row, ratio test den^2 d1^2 < num^2 d2^2 with at least two
// train rows, as xa_match_l2 counts them) in query order: both keypoints through their 2 x 3
// maps, and the descriptor distance sqrt(d1^2).  One block; the order comes from block scans.
struct Map2 {
    double m[6];
};
__global__ void __launch_bounds__(256) k_sift_match_points(const xa_sift_keypoint* __restrict__ kq,
                                                           const xa_sift_keypoint* __restrict__ kt,
                                                           const xa_l2_match* __restrict__ matches, int nq, int nt,
                                                           int num, int den, Map2 mq, Map2 mt, double* __restrict__ pq,
                                                           double* __restrict__ pt, double* __restrict__ des,
                                                           int32_t* __restrict__ n_out) {
    int base = 0;
    for (int q0 = 0; q0 < nq; q0 += 256) {
        const int q = q0 + int(threadIdx.x);
        xa_l2_match mm;
        mm.t = -1;
        mm.d1 = mm.d2 = 0xFFFFFFFFu;
        if (q < nq) mm = matches[q];
        const bool acc = q < nq && nt >= 2 && mm.t >= 0 && mm.t < nt && mm.d2 != 0xFFFFFFFFu &&
                         (long long)den * den * (long long)mm.d1 < (long long)num * num * (long long)mm.d2;
        int excl;
        const int tot = block_scan(acc ? 1 : 0, &excl);
        if (acc) {
            const int o = base + excl;
            const double ax = kq[q].x, ay = kq[q].y, bx = kt[mm.t].x, by = kt[mm.t].y;
            pq[2 * o] = mq.m[0] * ax + mq.m[1] * ay + mq.m[2];
            pq[2 * o + 1] = mq.m[3] * ax + mq.m[4] * ay + mq.m[5];
            pt[2 * o] = mt.m[0] * bx + mt.m[1] * by + mt.m[2];
            pt[2 * o + 1] = mt.m[3] * bx + mt.m[4] * by + mt.m[5];
            des[o] = sqrt(double(mm.d1));
        }
        base += tot;
    }
    if (threadIdx.x == 0) *n_out = base;
}

// ------------------------------------------------------------------ host side
// (still without contraction: the tap tables and blur widths follow the plain evaluation order)

Taps make_taps(double sigma) {
    Taps t;
    t.r = int(std::ceil(4.0 * sigma));
    std::vector<double> raw;
    for (int k = -t.r; k <= t.r; ++k) raw.push_back(std::exp(-double(k * k) / (2.0 * sigma * sigma)));
    double total = 0.0;
    for (double v : raw) total += v;
    for (int i = 0; i <= 2 * t.r; ++i) t.w[i] = float(raw[i] / total);
    return t;
}

xa_status sift_options(const xa_sift_opts* o, xa_sift_opts* out) {
    xa_sift_opts d;
    d.n_octaves = 0;
    d.n_layers = 3;
    d.max_keypoints = 4096;
    d.raw_capacity = 0;
    d.sigma0 = 1.6;
    d.sigma_in = 0.5;
    d.contrast = 0.04;
    d.edge = 10.0;
    if (o) d = *o;
    if (d.n_layers < 1 || d.n_layers > kSiftMaxLayers) return fail(XA_EINVAL, "n_layers must lie in 1..%d", kSiftMaxLayers);
    if (d.max_keypoints < 1 || d.max_keypoints > XA_SIFT_MAX_KEYPOINTS)
        return fail(XA_EINVAL, "max_keypoints must lie in 1..%d", XA_SIFT_MAX_KEYPOINTS);
    if (d.raw_capacity == 0) d.raw_capacity = std::min(2 * d.max_keypoints + 1024, XA_SIFT_MAX_KEYPOINTS * 2);
    if (d.raw_capacity < 1 || d.raw_capacity > 2 * XA_SIFT_MAX_KEYPOINTS)
        return fail(XA_EINVAL, "raw_capacity must lie in 1..%d", 2 * XA_SIFT_MAX_KEYPOINTS);
    if (!(d.sigma0 > d.sigma_in) || !(d.sigma_in >= 0.0) || !(d.sigma0 < 64.0))
        return fail(XA_EINVAL, "need 0 <= sigma_in < sigma0 < 64");
    if (!(d.contrast >= 0.0) || !(d.edge > 0.0)) return fail(XA_EINVAL, "need contrast >= 0 and edge > 0");
    // the largest incremental blur must fit the tap table
    const double top = d.sigma0 * std::pow(2.0, double(d.n_layers + 2) / d.n_layers);
    const double prev = d.sigma0 * std::pow(2.0, double(d.n_layers + 1) / d.n_layers);
    if (int(std::ceil(4.0 * std::sqrt(top * top - prev * prev))) * 2 + 1 > kSiftMaxTaps ||
        int(std::ceil(4.0 * std::sqrt(d.sigma0 * d.sigma0 - d.sigma_in * d.sigma_in))) * 2 + 1 > kSiftMaxTaps)
        return fail(XA_EUNSUPPORTED, "blur too wide for the %d-tap table", kSiftMaxTaps);
    *out = d;
    return XA_OK;
}

xa_status sift_geom(int w, int h, const xa_sift_opts& o, SiftGeom* G) {
    if (w < 1 || h < 1 || (long long)w * h > (1LL << 28)) return fail(XA_EUNSUPPORTED, "image size out of range");
    int n_oct = o.n_octaves;
    if (n_oct <= 0) n_oct = std::max(1, int(std::floor(std::log2(double(std::min(w, h))))) - 3);
    if (n_oct > kSiftMaxOctaves) return fail(XA_EINVAL, "at most %d octaves", kSiftMaxOctaves);
    G->n_oct = n_oct;
    G->s = o.n_layers;
    size_t fl = 0;
    int rows = 0, ow = w, oh = h;
    for (int i = 0; i < n_oct; ++i) {
        if (i > 0) {
            ow = (ow + 1) / 2;
            oh = (oh + 1) / 2;
        }
        Octave& oc = G->oct[i];
        oc.w = ow;
        oc.h = oh;
        oc.gauss = fl;
        fl += size_t(2 * o.n_layers + 5) * size_t(ow) * oh;
        oc.row0 = rows;
        oc.rows = (ow > 2 * kSiftBorder && oh > 2 * kSiftBorder) ? oh - 2 * kSiftBorder : 0;
        rows += o.n_layers * oc.rows;
    }
    G->tmp = fl;
    fl += size_t(w) * h;
    G->floats = fl;
    G->total_rows = rows;
    G->raw_cap = o.raw_capacity;
    size_t off = 0;
    G->off_floats = off;
    off += align_up(fl * sizeof(float));
    G->off_rowcount = off;
    off += align_up(size_t(rows + 1) * sizeof(int));
    G->off_rowoff = off;
    off += align_up(size_t(rows + 1) * sizeof(int));
    G->off_raw = off;
    off += align_up(size_t(G->raw_cap) * sizeof(RawKp));
    G->off_peaks = off;
    off += align_up(size_t(G->raw_cap) * sizeof(PeakSet));
    G->off_kpoff = off;
    off += align_up(size_t(G->raw_cap + 1) * sizeof(int));
    G->off_counters = off;
    off += align_up(4 * sizeof(int));
    G->total = off;
    return XA_OK;
}

void blur_into(const void* src, bool u8, int pitch, int w, int h, double sigma, float* tmp, float* dst,
               hipStream_t st) {
    const Taps t = make_taps(sigma);
    const dim3 grid(unsigned((w + 255) / 256), unsigned(h));
    if (u8)
        hipLaunchKernelGGL(k_sift_hblur<uint8_t>, grid, dim3(256), 0, st, static_cast<const uint8_t*>(src), pitch, w, h,
                           t, tmp);
    else
        hipLaunchKernelGGL(k_sift_hblur<float>, grid, dim3(256), 0, st, static_cast<const float*>(src), pitch, w, h, t,
                           tmp);
    hipLaunchKernelGGL(k_sift_vblur, grid, dim3(256), 0, st, tmp, w, h, t, dst);
}

}  // namespace
}  // namespace xa

using namespace xa;

extern "C" size_t xa_sift_workspace_size(int32_t w, int32_t h, const xa_sift_opts* opts) {
    xa_sift_opts o;
    if (sift_options(opts, &o) != XA_OK) return 0;
    SiftGeom G;
    if (sift_geom(w, h, o, &G) != XA_OK) return 0;
    return G.total;
}

extern "C" xa_status xa_extract_sift(const uint8_t* d_img, int32_t w, int32_t h, int32_t pitch,
                                     const xa_sift_opts* opts, xa_sift_keypoint* d_kp, uint8_t* d_desc,
                                     int32_t* d_count, void* d_ws, size_t ws_bytes, hipStream_t stream) {
    xa_sift_opts o;
    xa_status s = sift_options(opts, &o);
    if (s != XA_OK) return s;
    if (!d_img || !d_kp || !d_desc || !d_count) return fail(XA_EINVAL, "NULL device pointer");
    if (pitch < w) return fail(XA_EINVAL, "pitch %d below width %d", pitch, w);
    SiftGeom G;
    s = sift_geom(w, h, o, &G);
    if (s != XA_OK) return s;
    if (!d_ws || ws_bytes < G.total || reinterpret_cast<uintptr_t>(d_ws) % kAlign)
        return fail(XA_EINVAL, "workspace of %zu bytes (256-byte aligned) needed, %zu given", G.total, ws_bytes);
    uint8_t* ws = static_cast<uint8_t*>(d_ws);
    float* fl = reinterpret_cast<float*>(ws + G.off_floats);
    int* rowcount = reinterpret_cast<int*>(ws + G.off_rowcount);
    int* rowoff = reinterpret_cast<int*>(ws + G.off_rowoff);
    RawKp* raw = reinterpret_cast<RawKp*>(ws + G.off_raw);
    PeakSet* peaks = reinterpret_cast<PeakSet*>(ws + G.off_peaks);
    int* kpoff = reinterpret_cast<int*>(ws + G.off_kpoff);
    float* tmp = fl + G.tmp;
    // scale space
    const double base = std::sqrt(o.sigma0 * o.sigma0 - o.sigma_in * o.sigma_in);
    std::vector<double> inc;
    for (int k = 1; k < o.n_layers + 3; ++k) {
        const double prev = o.sigma0 * std::pow(2.0, double(k - 1) / o.n_layers);
        const double total = o.sigma0 * std::pow(2.0, double(k) / o.n_layers);
        inc.push_back(std::sqrt(total * total - prev * prev));
    }
    const int s_ = o.n_layers;
    for (int i = 0; i < G.n_oct; ++i) {
        const Octave& oc = G.oct[i];
        const size_t plane = size_t(oc.w) * oc.h;
        float* g = fl + oc.gauss;
        if (i == 0) {
            blur_into(d_img, true, pitch, oc.w, oc.h, base, tmp, g, stream);
        } else {
            const Octave& pv = G.oct[i - 1];
            hipLaunchKernelGGL(k_sift_down, dim3(unsigned((oc.w + 255) / 256), unsigned(oc.h)), dim3(256), 0, stream,
                               fl + pv.gauss + size_t(s_) * pv.w * pv.h, pv.w, g, oc.w, oc.h);
        }
        for (int k = 1; k < s_ + 3; ++k)
            blur_into(g + size_t(k - 1) * plane, false, oc.w, oc.w, oc.h, inc[k - 1], tmp, g + size_t(k) * plane, stream);
        hipLaunchKernelGGL(k_sift_dog, dim3(unsigned((plane + 255) / 256)), dim3(256), 0, stream, g,
                           g + size_t(s_ + 3) * plane, plane, s_ + 2);
    }
    // candidates and the fit: count per row, scan, write
    FitParams P;
    P.thr = o.contrast / double(o.n_layers) * 255.0;
    P.pre = 0.5 * P.thr;
    P.edge = o.edge;
    P.sigma0 = o.sigma0;
    P.s = s_;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1 && G.total_rows > 0)
            hipLaunchKernelGGL(k_sift_scan, dim3(1), dim3(256), 0, stream, rowcount, G.total_rows, rowoff);
        for (int i = 0; i < G.n_oct; ++i) {
            const Octave& oc = G.oct[i];
            if (oc.rows == 0) continue;
            const float* D = fl + oc.gauss + size_t(s_ + 3) * oc.w * oc.h;
            const dim3 grid(unsigned(s_ * oc.rows));
            if (pass == 0)
                hipLaunchKernelGGL(k_sift_rows<0>, grid, dim3(256), 0, stream, D, oc.w, oc.h, i, oc.row0, oc.rows, P,
                                   rowcount, rowoff, G.raw_cap, raw);
            else
                hipLaunchKernelGGL(k_sift_rows<1>, grid, dim3(256), 0, stream, D, oc.w, oc.h, i, oc.row0, oc.rows, P,
                                   rowcount, rowoff, G.raw_cap, raw);
        }
    }
    if (G.total_rows == 0) {   // no octave is large enough for a candidate: zero rows, zero keypoints
        hipLaunchKernelGGL(k_sift_scan, dim3(1), dim3(256), 0, stream, rowcount, 0, rowoff);
    }
    const int* n_raw = rowoff + G.total_rows;
    OctaveTable T;
    for (int i = 0; i < kSiftMaxOctaves; ++i) T.oct[i] = G.oct[i < G.n_oct ? i : 0];
    hipLaunchKernelGGL(k_sift_orient, dim3(unsigned(G.raw_cap)), dim3(64), 0, stream, fl, T, raw, n_raw, G.raw_cap,
                       peaks);
    hipLaunchKernelGGL(k_sift_scan_peaks, dim3(1), dim3(256), 0, stream, peaks, n_raw, G.raw_cap, kpoff,
                       o.max_keypoints, d_count);
    hipLaunchKernelGGL(k_sift_desc, dim3(unsigned(o.max_keypoints)), dim3(64), 0, stream, fl, T, raw, peaks, n_raw,
                       G.raw_cap, kpoff, d_count, d_kp, d_desc);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "SIFT launch");
}

extern "C" xa_status xa_sift_match_points(const xa_sift_keypoint* d_kp_q, const xa_sift_keypoint* d_kp_t,
                                          const xa_l2_match* d_matches, int32_t n_q, int32_t n_t, int32_t ratio_num,
                                          int32_t ratio_den, const double* map_q, const double* map_t, double* d_pq,
                                          double* d_pt, double* d_des, int32_t* d_n, hipStream_t stream) {
    if (n_q < 0 || n_t < 0 || n_q > XA_L2_MAX_DESCRIPTORS || n_t > XA_L2_MAX_DESCRIPTORS)
        return fail(XA_EINVAL, "counts must lie in 0..%d", XA_L2_MAX_DESCRIPTORS);
    if (ratio_num < 0 || ratio_den < 1 || ratio_num > (1 << 16) || ratio_den > (1 << 16))
        return fail(XA_EINVAL, "ratio must be num/den with 0 <= num, 1 <= den <= 2^16");
    if (!d_n || (n_q > 0 && (!d_kp_q || !d_matches || !d_pq || !d_pt || !d_des)) || (n_t > 0 && !d_kp_t))
        return fail(XA_EINVAL, "NULL device pointer");
    Map2 mq = {{1, 0, 0, 0, 1, 0}}, mt = {{1, 0, 0, 0, 1, 0}};
    if (map_q)
        for (int i = 0; i < 6; ++i) mq.m[i] = map_q[i];
    if (map_t)
        for (int i = 0; i < 6; ++i) mt.m[i] = map_t[i];
    hipLaunchKernelGGL(k_sift_match_points, dim3(1), dim3(256), 0, stream, d_kp_q, d_kp_t, d_matches, n_q, n_t,
                       ratio_num, ratio_den, mq, mt, d_pq, d_pt, d_des, d_n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "SIFT match points launch");
}
