// All-view-pair brute-force Hamming matching on gfx950 (Sec. III.B) with the
// nearest / second-nearest ratio test (Sec. IV.C), the best view pair, and the
// precision of eqs. (5)-(6).  Matching is integer XOR + popcount on the vector
// ALU: queries live in registers, train descriptors stream through LDS and are
// read as wave-uniform broadcasts.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace xa {
namespace {

constexpr int kMatchThreads = 256;   // four waves per block; a block owns 256 * Q queries of one view pair
constexpr int kMatchChunk = 512;     // train descriptors per LDS chunk (16 KiB)
constexpr int kIdxBits = 13;         // train index field of the packed (distance, index) key

// popcount(x) + acc in one v_bcnt_u32_b32 (keeps the eight popcounts of a 256-bit distance a chain)
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// median of three: with m1 <= m2, med3(m1, key, m2) = min(m2, max(m1, key))
__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Block = one view pair x (kMatchThreads * Q) queries.  Each lane keeps Q queries and,
// per query, the two smallest packed keys (d << 13 | train index): the smallest key gives
// d1 and the smallest index attaining it, the second smallest gives d2 over the others.
template <int Q>
__global__ void __launch_bounds__(kMatchThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) k_match(const uint32_t* __restrict__ desc_a,
                                                         const int32_t* __restrict__ count_a,
                                                         const uint32_t* __restrict__ desc_b,
                                                         const int32_t* __restrict__ count_b, int n_b, int N,
                                                         int num, int den, xa_match* __restrict__ matches,
                                                         int32_t* __restrict__ pair_count) {
    __shared__ uint4 tr[kMatchChunk * 2];
    __shared__ int s_acc;
    const int pair = blockIdx.x;
    const int i = pair / n_b, j = pair - (pair / n_b) * n_b;
    const int nq = min(max(count_a[i], 0), N), nt = min(max(count_b[j], 0), N);
    const int q0 = blockIdx.y * kMatchThreads * Q;
    if (q0 >= nq) return;
    uint32_t q[Q][8];
    uint32_t m1[Q], m2[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const int qi = q0 + a * kMatchThreads + threadIdx.x;
        if (qi < nq) {
            const uint4* p = reinterpret_cast<const uint4*>(desc_a + (size_t(i) * N + qi) * 8);
            const uint4 u0 = p[0], u1 = p[1];
            q[a][0] = u0.x; q[a][1] = u0.y; q[a][2] = u0.z; q[a][3] = u0.w;
            q[a][4] = u1.x; q[a][5] = u1.y; q[a][6] = u1.z; q[a][7] = u1.w;
        } else {
#pragma unroll
            for (int w = 0; w < 8; ++w) q[a][w] = 0u;
        }
        m1[a] = 0xFFFFFFFFu;
        m2[a] = 0xFFFFFFFFu;
    }
    const uint4* tb = reinterpret_cast<const uint4*>(desc_b + size_t(j) * N * 8);
    for (int c0 = 0; c0 < nt; c0 += kMatchChunk) {
        const int cn = min(kMatchChunk, nt - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < cn * 2; e += kMatchThreads) tr[e] = tb[size_t(c0) * 2 + e];
        __syncthreads();
#pragma unroll 2
        for (int r = 0; r < cn; ++r) {
            const uint4 t0 = tr[2 * r], t1 = tr[2 * r + 1];
            const uint32_t idx = uint32_t(c0 + r);
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                uint32_t d = __popc(q[a][0] ^ t0.x);
                d = bcnt_acc(q[a][1] ^ t0.y, d);
                d = bcnt_acc(q[a][2] ^ t0.z, d);
                d = bcnt_acc(q[a][3] ^ t0.w, d);
                d = bcnt_acc(q[a][4] ^ t1.x, d);
                d = bcnt_acc(q[a][5] ^ t1.y, d);
                d = bcnt_acc(q[a][6] ^ t1.z, d);
                d = bcnt_acc(q[a][7] ^ t1.w, d);
                const uint32_t key = (d << kIdxBits) | idx;
                m2[a] = med3_u32(m1[a], key, m2[a]);
                m1[a] = min(m1[a], key);
            }
        }
    }
    if (threadIdx.x == 0) s_acc = 0;
    __syncthreads();
    int acc = 0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const int qi = q0 + a * kMatchThreads + threadIdx.x;
        if (qi >= nq) continue;
        xa_match m;
        m.t = nt > 0 ? int32_t(m1[a] & ((1u << kIdxBits) - 1u)) : -1;
        const int d1 = nt > 0 ? int(m1[a] >> kIdxBits) : 65535;
        const int d2 = nt > 1 ? int(m2[a] >> kIdxBits) : 65535;
        m.d1 = uint16_t(d1);
        m.d2 = uint16_t(d2);
        matches[size_t(pair) * N + qi] = m;
        acc += (nt >= 2 && den * d1 < num * d2) ? 1 : 0;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(&s_acc, acc);
    __syncthreads();
    if (threadIdx.x == 0 && s_acc) atomicAdd(&pair_count[pair], s_acc);
}

// Argmax of the pair counts, lowest pair index on ties: max over (count << 32 | ~pair).
__global__ void __launch_bounds__(1024) k_best(const int32_t* __restrict__ pair_count, int n_pairs, int n_b,
                                               int32_t* __restrict__ best) {
    __shared__ unsigned long long s[16];
    unsigned long long key = 0;
    for (int p = threadIdx.x; p < n_pairs; p += blockDim.x) {
        const unsigned long long k = ((unsigned long long)(uint32_t)pair_count[p] << 32) | (0xFFFFFFFFu - uint32_t(p));
        key = key > k ? key : k;
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
        const int p = int(0xFFFFFFFFu - uint32_t(m & 0xFFFFFFFFull));
        best[0] = p;
        best[1] = p / n_b;
        best[2] = p % n_b;
        best[3] = int(m >> 32);
    }
}

struct H9 {
    double h[9];
};

// Eqs. (5)-(6) on the best pair: correct iff |H p_a - p_b| <= th.
__global__ void __launch_bounds__(256) k_precision(const xa_keypoint* __restrict__ kp_a, const xa_keypoint* __restrict__ kp_b,
                                                   const xa_match* __restrict__ matches, const int32_t* __restrict__ count_a,
                                                   const int32_t* __restrict__ count_b, int n_b, int N, int num, int den,
                                                   const int32_t* __restrict__ best, H9 H, double th,
                                                   int32_t* __restrict__ out) {
    __shared__ int s_ok, s_n;
    if (threadIdx.x == 0) { s_ok = 0; s_n = 0; }
    __syncthreads();
    const int pair = best[0], i = best[1], j = best[2];
    const bool valid = pair >= 0 && i >= 0 && j >= 0 && j < n_b && pair == i * n_b + j;
    const int nq = valid ? min(max(count_a[i], 0), N) : 0;
    const int nt = valid ? min(max(count_b[j], 0), N) : 0;
    int ok = 0, n = 0;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
        const xa_match m = matches[size_t(pair) * N + q];
        if (!(nt >= 2 && den * int(m.d1) < num * int(m.d2)) || m.t < 0 || m.t >= nt) continue;
        const xa_keypoint a = kp_a[size_t(i) * N + q];
        const xa_keypoint b = kp_b[size_t(j) * N + m.t];
        const double w = H.h[6] * a.xs + H.h[7] * a.ys + H.h[8];
        const double px = (H.h[0] * a.xs + H.h[1] * a.ys + H.h[2]) / w;
        const double py = (H.h[3] * a.xs + H.h[4] * a.ys + H.h[5]) / w;
        const double ex = px - b.xs, ey = py - b.ys;
        n += 1;
        ok += (sqrt(ex * ex + ey * ey) <= th) ? 1 : 0;
    }
    atomicAdd(&s_ok, ok);
    atomicAdd(&s_n, n);
    __syncthreads();
    if (threadIdx.x == 0) { out[0] = s_ok; out[1] = s_n; }
}

}  // namespace

xa_status launch_match(const uint8_t* desc_a, const int32_t* count_a, int32_t n_a, const uint8_t* desc_b,
                       const int32_t* count_b, int32_t n_b, int32_t N, int32_t num, int32_t den, xa_match* matches,
                       int32_t* pair_count, int32_t* best, hipStream_t st) {
    const int n_pairs = n_a * n_b;
    hipLaunchKernelGGL(k_fill_i32, dim3((n_pairs + 255) / 256), dim3(256), 0, st, pair_count, n_pairs, 0);
    const uint32_t* da = reinterpret_cast<const uint32_t*>(desc_a);
    const uint32_t* db = reinterpret_cast<const uint32_t*>(desc_b);
    // Q queries per lane: 4 amortises each LDS broadcast of a train descriptor over 4 comparisons;
    // fewer for small N so that padding lanes do not dominate
    if (N > 2 * kMatchThreads) {
        const int gy = (N + 4 * kMatchThreads - 1) / (4 * kMatchThreads);
        hipLaunchKernelGGL(k_match<4>, dim3(n_pairs, gy), dim3(kMatchThreads), 0, st, da, count_a, db, count_b, n_b, N,
                           num, den, matches, pair_count);
    } else if (N > kMatchThreads) {
        hipLaunchKernelGGL(k_match<2>, dim3(n_pairs, 1), dim3(kMatchThreads), 0, st, da, count_a, db, count_b, n_b, N,
                           num, den, matches, pair_count);
    } else {
        hipLaunchKernelGGL(k_match<1>, dim3(n_pairs, 1), dim3(kMatchThreads), 0, st, da, count_a, db, count_b, n_b, N,
                           num, den, matches, pair_count);
    }
    hipLaunchKernelGGL(k_best, dim3(1), dim3(1024), 0, st, pair_count, n_pairs, n_b, best);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "match launch");
    return XA_OK;
}

}  // namespace xa

using namespace xa;

extern "C" xa_status xa_match_views(const uint8_t* d_desc_a, const int32_t* d_count_a, int32_t n_a,
                                    const uint8_t* d_desc_b, const int32_t* d_count_b, int32_t n_b,
                                    int32_t n_features, int32_t ratio_num, int32_t ratio_den, xa_match* d_matches,
                                    int32_t* d_pair_count, int32_t* d_best, hipStream_t stream) {
    if (n_a < 1 || n_b < 1 || int64_t(n_a) * n_b > (int64_t(1) << 30)) return fail(XA_EINVAL, "bad view counts");
    if (n_features < 1 || n_features > XA_MAX_FEATURES) return fail(XA_EUNSUPPORTED, "n_features out of range");
    if (ratio_num < 0 || ratio_den < 1 || ratio_num > (1 << 20) || ratio_den > (1 << 20))
        return fail(XA_EINVAL, "ratio must be num/den with 0 <= num, 1 <= den <= 2^20");
    if (!d_desc_a || !d_count_a || !d_desc_b || !d_count_b || !d_matches || !d_pair_count || !d_best)
        return fail(XA_EINVAL, "NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(d_desc_a) | reinterpret_cast<uintptr_t>(d_desc_b)) % 16)
        return fail(XA_EINVAL, "descriptor arrays must be 16-byte aligned");
    xa_status s = launch_match(d_desc_a, d_count_a, n_a, d_desc_b, d_count_b, n_b, n_features, ratio_num, ratio_den,
                               d_matches, d_pair_count, d_best, stream);
    return s == XA_OK ? ok() : s;
}

extern "C" xa_status xa_pair_precision(const xa_keypoint* d_kp_a, const xa_keypoint* d_kp_b, const xa_match* d_matches,
                                       const int32_t* d_count_a, const int32_t* d_count_b, int32_t n_b,
                                       int32_t n_features, int32_t ratio_num, int32_t ratio_den, const int32_t* d_best,
                                       const double* H, double th, int32_t* d_out, hipStream_t stream) {
    if (!d_kp_a || !d_kp_b || !d_matches || !d_count_a || !d_count_b || !d_best || !H || !d_out)
        return fail(XA_EINVAL, "NULL pointer");
    if (n_b < 1 || n_features < 1 || n_features > XA_MAX_FEATURES || ratio_den < 1 || ratio_num < 0)
        return fail(XA_EINVAL, "bad sizes");
    H9 h;
    for (int k = 0; k < 9; ++k) h.h[k] = H[k];
    hipLaunchKernelGGL(k_precision, dim3(1), dim3(256), 0, stream, d_kp_a, d_kp_b, d_matches, d_count_a, d_count_b, n_b,
                       n_features, ratio_num, ratio_den, d_best, h, th, d_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "precision launch");
    return ok();
}
