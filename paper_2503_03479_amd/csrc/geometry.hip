// Precise-stage geometry (Sec. III.C): the accepted matches of the best view pair in
// original-image coordinates, and homography RANSAC over them with caller-drawn samples;
// eq. (7) is the share of matches RANSAC keeps.
//
// A sample (4 match indices) is degenerate when some 3 of its 4 points, in image A or B,
// span a doubled triangle area below 1 px^2, or when an index is outside [0, n); it then
// scores -1.  Otherwise H (h33 = 1) solves the 8 x 8 system mapping the 4 points of A onto
// those of B (Gaussian elimination with partial pivoting, fp64), and the score is the number
// of matches with |H(p_a) - p_b| <= th (projective image; w <= 0 is an outlier).  The best
// sample has the highest score, the lowest index on ties.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace xa {
namespace {

constexpr double kDegenerateArea = 1.0;

__device__ bool degenerate4(const double* x, const double* y) {
    const int tri[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma clang fp contract(off)
        const int a = tri[t][0], b = tri[t][1], c = tri[t][2];
        const double cross = (x[b] - x[a]) * (y[c] - y[a]) - (y[b] - y[a]) * (x[c] - x[a]);
        if (fabs(cross) < kDegenerateArea) return true;
    }
    return false;
}

// H of one sample into H[9]; false if degenerate.  M is 8 x 9 scratch (LDS) for one solver.
__device__ bool sample_homography(const double* __restrict__ pa, const double* __restrict__ pb, int n,
                                  const int32_t* __restrict__ idx, double* M, double* H) {
    double sx[4], sy[4], dx[4], dy[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = idx[i];
        if (j < 0 || j >= n) return false;
        sx[i] = pa[2 * j]; sy[i] = pa[2 * j + 1];
        dx[i] = pb[2 * j]; dy[i] = pb[2 * j + 1];
    }
    if (degenerate4(sx, sy) || degenerate4(dx, dy)) return false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double* r0 = M + (2 * i) * 9;
        double* r1 = r0 + 9;
        r0[0] = sx[i]; r0[1] = sy[i]; r0[2] = 1.0; r0[3] = 0.0; r0[4] = 0.0; r0[5] = 0.0;
        r0[6] = -dx[i] * sx[i]; r0[7] = -dx[i] * sy[i]; r0[8] = dx[i];
        r1[0] = 0.0; r1[1] = 0.0; r1[2] = 0.0; r1[3] = sx[i]; r1[4] = sy[i]; r1[5] = 1.0;
        r1[6] = -dy[i] * sx[i]; r1[7] = -dy[i] * sy[i]; r1[8] = dy[i];
    }
    for (int c = 0; c < 8; ++c) {
        int p = c;
        double best = fabs(M[c * 9 + c]);
        for (int r = c + 1; r < 8; ++r) {
            const double a = fabs(M[r * 9 + c]);
            if (a > best) { best = a; p = r; }
        }
        if (!(best > 0.0)) return false;
        if (p != c)
            for (int k = c; k < 9; ++k) {
                const double tmp = M[c * 9 + k];
                M[c * 9 + k] = M[p * 9 + k];
                M[p * 9 + k] = tmp;
            }
        for (int r = c + 1; r < 8; ++r) {
            const double f = M[r * 9 + c] / M[c * 9 + c];
            for (int k = c; k < 9; ++k) M[r * 9 + k] -= f * M[c * 9 + k];
        }
    }
    for (int r = 7; r >= 0; --r) {
        double s = M[r * 9 + 8];
        for (int k = r + 1; k < 8; ++k) s -= M[r * 9 + k] * H[k];
        H[r] = s / M[r * 9 + r];
    }
    H[8] = 1.0;
    return true;
}

// |H(p_a) - p_b| <= th, evaluated term by term without contraction (the pragma: device code
// is otherwise built with multiply-adds fused)
__device__ __forceinline__ bool is_inlier(const double* H, double x, double y, double bx, double by, double th) {
#pragma clang fp contract(off)
    const double w = H[6] * x + H[7] * y + H[8];
    if (!(w > 0.0)) return false;
    const double u = H[0] * x + H[1] * y + H[2];
    const double v = H[3] * x + H[4] * y + H[5];
    const double ex = u / w - bx, ey = v / w - by;
    return sqrt(ex * ex + ey * ey) <= th;
}

// One 64-lane block per sample: lane 0 solves, every lane counts inliers.
__global__ void __launch_bounds__(64) k_ransac_score(const double* __restrict__ pa, const double* __restrict__ pb,
                                                     int n, const int32_t* __restrict__ samples, double th,
                                                     int32_t* __restrict__ scores) {
    __shared__ double M[72];
    __shared__ double H[9];
    __shared__ int ok;
    const int k = blockIdx.x;
    if (threadIdx.x == 0) ok = sample_homography(pa, pb, n, samples + 4 * size_t(k), M, H) ? 1 : 0;
    __syncthreads();
    if (!ok) {
        if (threadIdx.x == 0) scores[k] = -1;
        return;
    }
    int c = 0;
    for (int i = threadIdx.x; i < n; i += 64) c += is_inlier(H, pa[2 * i], pa[2 * i + 1], pb[2 * i], pb[2 * i + 1], th);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if (threadIdx.x == 0) scores[k] = c;
}

// best = (index, score) of the highest score, lowest index on ties; (-1, -1) if none >= 0.
__global__ void __launch_bounds__(1024) k_ransac_best(const int32_t* __restrict__ scores, int K,
                                                      int32_t* __restrict__ best) {
    __shared__ unsigned long long s[16];
    unsigned long long key = 0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const int sc = scores[k];
        if (sc < 0) continue;
        const unsigned long long kk = ((unsigned long long)uint32_t(sc) << 32) | (0xFFFFFFFFu - uint32_t(k));
        key = key > kk ? key : kk;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off);
        key = key > o ? key : o;
    }
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) m = m > s[w] ? m : s[w];
        if (m == 0) {
            best[0] = -1;
            best[1] = -1;
        } else {
            best[0] = int(0xFFFFFFFFu - uint32_t(m & 0xFFFFFFFFull));
            best[1] = int(m >> 32);
        }
    }
}

// Sum of v over the block (256 threads) in a fixed order: butterfly inside each wave, then
// the four wave sums in order.  Every thread receives the total.
__device__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

// Solve the 8 x 8 system M (row-major 8 x 9, augmented) by partial pivoting into h; false if singular.
__device__ bool solve8(double* M, double* h) {
    for (int c = 0; c < 8; ++c) {
        int p = c;
        double best = fabs(M[c * 9 + c]);
        for (int r = c + 1; r < 8; ++r) {
            const double a = fabs(M[r * 9 + c]);
            if (a > best) { best = a; p = r; }
        }
        if (!(best > 0.0)) return false;
        if (p != c)
            for (int k = c; k < 9; ++k) {
                const double tmp = M[c * 9 + k];
                M[c * 9 + k] = M[p * 9 + k];
                M[p * 9 + k] = tmp;
            }
        for (int r = c + 1; r < 8; ++r) {
            const double f = M[r * 9 + c] / M[c * 9 + c];
            for (int k = c; k < 9; ++k) M[r * 9 + k] -= f * M[c * 9 + k];
        }
    }
    for (int r = 7; r >= 0; --r) {
        double s = M[r * 9 + 8];
        for (int k = r + 1; k < 8; ++k) s -= M[r * 9 + k] * h[k];
        h[r] = s / M[r * 9 + r];
    }
    return true;
}

// H of the best sample refitted over its inliers (least squares, h33 = 1, in Hartley-normalised
// coordinates: centroid at 0, mean distance sqrt(2); normal equations with fixed-order sums),
// or the sample's own H when there are fewer than 4 inliers or no solution; the inlier mask
// is the best sample's.  H = 0 and an empty mask when there is no valid sample.
__global__ void __launch_bounds__(256) k_ransac_final(const double* __restrict__ pa, const double* __restrict__ pb,
                                                      int n, const int32_t* __restrict__ samples, double th,
                                                      const int32_t* __restrict__ best, double* __restrict__ Hout,
                                                      uint8_t* __restrict__ inliers) {
    __shared__ double M[72];
    __shared__ double H[9];
    __shared__ double red[4];
    __shared__ double Nm[45];           // the 8 x 8 normal matrix (upper triangle, 36) and the right side (8)
    __shared__ int ok;
    const int b = best[0];
    if (threadIdx.x == 0) ok = b >= 0 && sample_homography(pa, pb, n, samples + 4 * size_t(b), M, H) ? 1 : 0;
    __syncthreads();
    if (!ok) {
        if (threadIdx.x < 9) Hout[threadIdx.x] = 0.0;
        for (int i = threadIdx.x; inliers && i < n; i += blockDim.x) inliers[i] = 0;
        return;
    }
    // centroids and count of the inliers
    double sax = 0, say = 0, sbx = 0, sby = 0, cnt = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const bool in = is_inlier(H, pa[2 * i], pa[2 * i + 1], pb[2 * i], pb[2 * i + 1], th);
        if (inliers) inliers[i] = uint8_t(in);
        if (in) {
            sax += pa[2 * i]; say += pa[2 * i + 1];
            sbx += pb[2 * i]; sby += pb[2 * i + 1];
            cnt += 1.0;
        }
    }
    const double m = block_sum(cnt, red);
    const double cax = block_sum(sax, red) / m, cay = block_sum(say, red) / m;
    const double cbx = block_sum(sbx, red) / m, cby = block_sum(sby, red) / m;
    double da = 0, db = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (is_inlier(H, pa[2 * i], pa[2 * i + 1], pb[2 * i], pb[2 * i + 1], th)) {
            da += sqrt((pa[2 * i] - cax) * (pa[2 * i] - cax) + (pa[2 * i + 1] - cay) * (pa[2 * i + 1] - cay));
            db += sqrt((pb[2 * i] - cbx) * (pb[2 * i] - cbx) + (pb[2 * i + 1] - cby) * (pb[2 * i + 1] - cby));
        }
    const double ma = block_sum(da, red) / m, mb = block_sum(db, red) / m;
    const bool refit = m >= 4.0 && ma > 0.0 && mb > 0.0;
    double h[8];
    bool solved = false;
    if (refit) {
        const double sa = sqrt(2.0) / ma, sb = sqrt(2.0) / mb;
        // normal equations: rows r1 = [x, y, 1, 0, 0, 0, -u x, -u y] -> u, r2 = [0, 0, 0, x, y, 1, -v x, -v y] -> v
        double acc[44];
#pragma unroll
        for (int e = 0; e < 44; ++e) acc[e] = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            if (!is_inlier(H, pa[2 * i], pa[2 * i + 1], pb[2 * i], pb[2 * i + 1], th)) continue;
            const double x = sa * (pa[2 * i] - cax), y = sa * (pa[2 * i + 1] - cay);
            const double u = sb * (pb[2 * i] - cbx), v = sb * (pb[2 * i + 1] - cby);
            const double r1[8] = {x, y, 1.0, 0.0, 0.0, 0.0, -u * x, -u * y};
            const double r2[8] = {0.0, 0.0, 0.0, x, y, 1.0, -v * x, -v * y};
            int e = 0;
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int c = a; c < 8; ++c) acc[e++] += r1[a] * r1[c] + r2[a] * r2[c];
#pragma unroll
            for (int a = 0; a < 8; ++a) acc[36 + a] += r1[a] * u + r2[a] * v;
        }
        for (int e = 0; e < 44; ++e) {
            const double t = block_sum(acc[e], red);
            if (threadIdx.x == 0) Nm[e] = t;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int e = 0;
            for (int a = 0; a < 8; ++a)
                for (int c = a; c < 8; ++c) {
                    M[a * 9 + c] = Nm[e];
                    M[c * 9 + a] = Nm[e];
                    ++e;
                }
            for (int a = 0; a < 8; ++a) M[a * 9 + 8] = Nm[36 + a];
            solved = solve8(M, h);
            if (solved) {
                // H = Tb^-1 Hn Ta with Ta = [[sa, 0, -sa cax], [0, sa, -sa cay], [0, 0, 1]] (Tb likewise)
                const double Hn[9] = {h[0], h[1], h[2], h[3], h[4], h[5], h[6], h[7], 1.0};
                const double Ta[9] = {sa, 0.0, -sa * cax, 0.0, sa, -sa * cay, 0.0, 0.0, 1.0};
                const double Tbi[9] = {1.0 / sb, 0.0, cbx, 0.0, 1.0 / sb, cby, 0.0, 0.0, 1.0};
                double T1[9], R[9];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        T1[r * 3 + c] = Hn[r * 3] * Ta[c] + Hn[r * 3 + 1] * Ta[3 + c] + Hn[r * 3 + 2] * Ta[6 + c];
                    }
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c)
                        R[r * 3 + c] = Tbi[r * 3] * T1[c] + Tbi[r * 3 + 1] * T1[3 + c] + Tbi[r * 3 + 2] * T1[6 + c];
                for (int k = 0; k < 9; ++k) Hout[k] = R[k] / R[8];
            }
            if (!solved)
                for (int k = 0; k < 9; ++k) Hout[k] = H[k];
        }
    } else if (threadIdx.x == 0) {
        for (int k = 0; k < 9; ++k) Hout[k] = H[k];
    }
}

// Accepted matches of the best view pair, in query order, as original-image points:
// one block; flags, a block-wide exclusive scan, then the writes.
__global__ void __launch_bounds__(1024) k_pair_points(const xa_keypoint* __restrict__ kp_a,
                                                      const xa_keypoint* __restrict__ kp_b,
                                                      const xa_match* __restrict__ matches,
                                                      const int32_t* __restrict__ count_a,
                                                      const int32_t* __restrict__ count_b, int n_b, int N, int num,
                                                      int den, const int32_t* __restrict__ best,
                                                      double* __restrict__ pa, double* __restrict__ pb,
                                                      int32_t* __restrict__ dist, int32_t* __restrict__ n_out) {
    __shared__ int wsum[16];
    __shared__ int base;
    const int pair = best[0], i = best[1], j = best[2];
    const bool valid = pair >= 0 && i >= 0 && j >= 0 && j < n_b && pair == i * n_b + j;
    const int nq = valid ? min(max(count_a[i], 0), N) : 0;
    const int nt = valid ? min(max(count_b[j], 0), N) : 0;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int q0 = 0; q0 < nq; q0 += blockDim.x) {
        const int q = q0 + int(threadIdx.x);
        bool acc = false;
        xa_match m{};
        if (q < nq) {
            m = matches[size_t(pair) * N + q];
            acc = nt >= 2 && den * int(m.d1) < num * int(m.d2) && m.t >= 0 && m.t < nt;
        }
        const unsigned long long bal = __ballot(acc);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wv] = __popcll(bal);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wv; ++w) off += wsum[w];
        if (acc) {
            const int o = off + before;
            const xa_keypoint a = kp_a[size_t(i) * N + q];
            const xa_keypoint bk = kp_b[size_t(j) * N + m.t];
            pa[2 * o] = a.xs; pa[2 * o + 1] = a.ys;
            pb[2 * o] = bk.xs; pb[2 * o + 1] = bk.ys;
            if (dist) dist[o] = int32_t(m.d1);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < int(blockDim.x >> 6); ++w) t += wsum[w];
            base += t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_out = base;
}

// Eq. (1) over the first min(*n, cap) matches: sum over consecutive pairs of the difference of
// segment lengths weighted by 1 - (Des(i) + Des(i + 1)) / 1000, in a fixed summation order.
template <typename D>
__global__ void __launch_bounds__(256) k_scaling(const double* __restrict__ pa, const double* __restrict__ pb,
                                                 const D* __restrict__ des, const int32_t* __restrict__ n_dev,
                                                 int cap, double* __restrict__ f) {
    __shared__ double red[4];
    const int n = min(max(*n_dev, 0), cap);
    double acc = 0.0;
    for (int i = threadIdx.x; i + 1 < n; i += blockDim.x) {
        const double ax = pa[2 * i + 2] - pa[2 * i], ay = pa[2 * i + 3] - pa[2 * i + 1];
        const double bx = pb[2 * i + 2] - pb[2 * i], by = pb[2 * i + 3] - pb[2 * i + 1];
        const double w = 1.0 - (double(des[i]) + double(des[i + 1])) / 1000.0;
        acc += (sqrt(ax * ax + ay * ay) - sqrt(bx * bx + by * by)) * w;
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) *f = t;
}

}  // namespace
}  // namespace xa

using namespace xa;

extern "C" xa_status xa_scaling_coefficient(const double* d_pa, const double* d_pb, const int32_t* d_des,
                                            const int32_t* d_n, int32_t cap, double* d_f, hipStream_t stream) {
    if (!d_pa || !d_pb || !d_des || !d_n || !d_f) return fail(XA_EINVAL, "NULL pointer");
    if (cap < 0) return fail(XA_EINVAL, "negative capacity");
    hipLaunchKernelGGL(k_scaling<int32_t>, dim3(1), dim3(256), 0, stream, d_pa, d_pb, d_des, d_n, cap, d_f);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "scaling coefficient launch");
}

extern "C" xa_status xa_scaling_coefficient_f64(const double* d_pa, const double* d_pb, const double* d_des,
                                                const int32_t* d_n, int32_t cap, double* d_f, hipStream_t stream) {
    if (!d_pa || !d_pb || !d_des || !d_n || !d_f) return fail(XA_EINVAL, "NULL pointer");
    if (cap < 0) return fail(XA_EINVAL, "negative capacity");
    hipLaunchKernelGGL(k_scaling<double>, dim3(1), dim3(256), 0, stream, d_pa, d_pb, d_des, d_n, cap, d_f);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "scaling coefficient launch");
}

extern "C" xa_status xa_ransac_homography(const double* d_pa, const double* d_pb, int32_t n, const int32_t* d_samples,
                                          int32_t k, double th, int32_t* d_scores, int32_t* d_best, double* d_H,
                                          uint8_t* d_inliers, hipStream_t stream) {
    if (n < 0 || k < 0) return fail(XA_EINVAL, "negative count");
    if (!(th >= 0.0)) return fail(XA_EINVAL, "threshold must be >= 0");
    if (!d_scores || !d_best || !d_H || ((!d_pa || !d_pb) && n > 0) || (!d_samples && k > 0))
        return fail(XA_EINVAL, "NULL pointer");
    if ((reinterpret_cast<uintptr_t>(d_pa) | reinterpret_cast<uintptr_t>(d_pb) | reinterpret_cast<uintptr_t>(d_H)) % 8 ||
        (reinterpret_cast<uintptr_t>(d_samples) | reinterpret_cast<uintptr_t>(d_scores) |
         reinterpret_cast<uintptr_t>(d_best)) % 4)
        return fail(XA_EINVAL, "misaligned buffer");
    if (k > 0)
        hipLaunchKernelGGL(k_ransac_score, dim3(unsigned(k)), dim3(64), 0, stream, d_pa, d_pb, n, d_samples, th,
                           d_scores);
    hipLaunchKernelGGL(k_ransac_best, dim3(1), dim3(1024), 0, stream, d_scores, k, d_best);
    hipLaunchKernelGGL(k_ransac_final, dim3(1), dim3(256), 0, stream, d_pa, d_pb, n, d_samples, th, d_best, d_H,
                       d_inliers);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "ransac launch");
}

extern "C" xa_status xa_best_pair_points(const xa_keypoint* d_kp_a, const xa_keypoint* d_kp_b, const xa_match* d_matches,
                                         const int32_t* d_count_a, const int32_t* d_count_b, int32_t n_b,
                                         int32_t n_features, int32_t ratio_num, int32_t ratio_den,
                                         const int32_t* d_best, double* d_pa, double* d_pb, int32_t* d_dist,
                                         int32_t* d_n, hipStream_t stream) {
    if (!d_kp_a || !d_kp_b || !d_matches || !d_count_a || !d_count_b || !d_best || !d_pa || !d_pb || !d_n)
        return fail(XA_EINVAL, "NULL pointer");
    if (n_b < 1 || n_features < 1 || n_features > XA_MAX_FEATURES) return fail(XA_EINVAL, "bad sizes");
    if (ratio_num < 0 || ratio_den < 1 || ratio_num > (1 << 20) || ratio_den > (1 << 20))
        return fail(XA_EINVAL, "bad ratio");
    hipLaunchKernelGGL(k_pair_points, dim3(1), dim3(1024), 0, stream, d_kp_a, d_kp_b, d_matches, d_count_a, d_count_b,
                       n_b, n_features, ratio_num, ratio_den, d_best, d_pa, d_pb, d_dist, d_n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "pair points launch");
}
