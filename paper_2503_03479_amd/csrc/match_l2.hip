// Exact L2 nearest-two matching of 8-bit SIFT descriptors (the SIFT matching of Sec. III.A and
// III.C, screened by the nearest / second-nearest ratio of Sec. IV.C) on the int8 matrix cores.
//
// For 128-D descriptors with components 0..255 the squared distance is an integer below 2^23.
// With the query bytes centred as q' = q - 128 and the train bytes as t'' = 127 - t (both in
// -128..127, i.e. q ^ 0x80 and t ^ 0x7F as bytes), sum (q - t)^2 = P_q + P_t + 2 sum t'' q' with
// P_q = |q|^2 - 254 S_q + 4161536 and P_t = |t|^2 - 256 S_t (S = the component sum), so one
// v_mfma_i32_32x32x32_i8 contraction per 32 x 32 tile and K-step gives every dot product
// exactly.  Per query the order of P_t + 2 sum t''q' (= d^2 - P_q, magnitude below 2^23) is the
// order of d^2; packed with the row's index inside its 128-row chunk as
// key = (P_t + 2 acc) * 128 + row = T7[row] + 256 acc, each result costs one shift-add, and the
// two smallest keys per query are kept two keys at a time with min3 and med3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <mutex>

#include "internal.h"

namespace xa {
namespace {

constexpr int kL2Threads = 256;            // four waves
constexpr int kL2QT = 2;                   // 32-query tiles per wave (each train operand feeds both)
constexpr int kL2BlockQ = (kL2Threads / 64) * 32 * kL2QT;   // queries per block
constexpr int kL2Chunk = 128;              // train rows staged in LDS per step (16 KiB of operands)
constexpr int kL2TargetBlocks = 2048;      // train slices are added until a launch has about this many blocks
constexpr int kL2Sentinel = 0x7F000000;    // key base of a row past the train range: above every real key
constexpr int kL2NoVal = 1 << 24;          // value of a missing neighbour (real values are below 2^23 in magnitude)
constexpr int kL2DescWords = 8;            // 128 bytes = 8 x 16 bytes

typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v16i_t __attribute__((ext_vector_type(16)));

// (value, index) ordered lexicographically as one int64: the index is below 2^31
__device__ __forceinline__ long long lex(int v, int i) { return (static_cast<long long>(v) << 32) | uint32_t(i); }
constexpr long long kNone = (static_cast<long long>(kL2NoVal) << 32) | uint32_t(INT_MAX);

// the two smallest of {a1 <= a2} and {b1 <= b2}, into (a1, a2)
__device__ __forceinline__ void merge2(long long& a1, long long& a2, long long b1, long long b2) {
    if (b1 < a1) {
        a2 = a1 < b2 ? a1 : b2;
        a1 = b1;
    } else {
        a2 = b1 < a2 ? b1 : a2;
    }
}

__device__ __forceinline__ int med3_i32(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

__device__ __forceinline__ v4i_t as_v4i(uint4 u, uint32_t x) {
    v4i_t v = {int(u.x ^ x), int(u.y ^ x), int(u.z ^ x), int(u.w ^ x)};
    return v;
}

__device__ __forceinline__ uint32_t udot4(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_udot4(a, b, c, false);
}

// Block (query block qb, train slice blockIdx.y): 256 queries against the slice's train rows,
// chunk by chunk; the two best (value, index) per query of the slice go to part[slice][query].
// Operand layout: K-step s of lane (h = lane / 32, m = lane % 32) is bytes 32 s + 16 h .. + 15 of
// descriptor m of the tile, for both operands, so the contraction pairs equal components
// whatever order the hardware gives the 16 bytes.  Result r of the lane is tile row
// 8 (r / 4) + 4 h + r % 4 of query column m.
__global__ void __launch_bounds__(kL2Threads)
k_match_l2(const uint4* __restrict__ q, int nq, const uint4* __restrict__ t, int nt, int chunks_per_slice,
           int4* __restrict__ part) {
    __shared__ uint4 tr[(kL2Chunk / 32) * 4 * 64];      // [tile][K-step][lane]
    __shared__ __align__(16) int t7[kL2Chunk];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane >> 5, m = lane & 31;
    const int qw = blockIdx.x * kL2BlockQ + wv * 32 * kL2QT;   // this wave's first query
    v4i_t B[kL2QT][4];
#pragma unroll
    for (int qt = 0; qt < kL2QT; ++qt) {
        const int qi = qw + qt * 32 + m;
#pragma unroll
        for (int s = 0; s < 4; ++s)
            B[qt][s] = qi < nq ? as_v4i(q[size_t(qi) * kL2DescWords + 2 * s + h], 0x80808080u) : v4i_t{0, 0, 0, 0};
    }
    long long K1[kL2QT], K2[kL2QT];
#pragma unroll
    for (int qt = 0; qt < kL2QT; ++qt) { K1[qt] = kNone; K2[qt] = kNone; }
    const int c_begin = blockIdx.y * chunks_per_slice * kL2Chunk;
    const int c_end = min(nt, c_begin + chunks_per_slice * kL2Chunk);
    // staging: thread -> chunk row r = tid / 2, its 16-byte pieces 4 (tid % 2) .. + 3; each
    // chunk's pieces are loaded one chunk ahead, so the loads overlap the previous chunk's tiles
    const int r = threadIdx.x >> 1, hf = threadIdx.x & 1;
    uint4 nx[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        nx[k] = c_begin + r < c_end ? t[size_t(c_begin + r) * kL2DescWords + hf * 4 + k] : make_uint4(0, 0, 0, 0);
    for (int c0 = c_begin; c0 < c_end; c0 += kL2Chunk) {
        __syncthreads();                                  // the previous chunk's readers are done
        {   // stage this chunk's operands and T7 (with P_t)
            const int row = c0 + r;
            const bool live = row < c_end;
            uint32_t sq = 0, s1 = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int c = hf * 4 + k;                 // piece c: K-step c / 2, half c % 2
                const uint4 w = live ? nx[k] : make_uint4(0, 0, 0, 0);
                sq = udot4(w.x, w.x, udot4(w.y, w.y, udot4(w.z, w.z, udot4(w.w, w.w, sq))));
                s1 = udot4(w.x, 0x01010101u, udot4(w.y, 0x01010101u, udot4(w.z, 0x01010101u, udot4(w.w, 0x01010101u, s1))));
                tr[((r >> 5) * 4 + (c >> 1)) * 64 + (c & 1) * 32 + (r & 31)] =
                    live ? make_uint4(w.x ^ 0x7F7F7F7Fu, w.y ^ 0x7F7F7F7Fu, w.z ^ 0x7F7F7F7Fu, w.w ^ 0x7F7F7F7Fu)
                         : make_uint4(0, 0, 0, 0);
            }
            sq += __shfl_xor(sq, 1);
            s1 += __shfl_xor(s1, 1);
            if (hf == 0) t7[r] = live ? (int(sq) - 256 * int(s1)) * 128 + r : kL2Sentinel + r;
        }
        __syncthreads();
        {
            const int row = c0 + kL2Chunk + r;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (row < c_end) nx[k] = t[size_t(row) * kL2DescWords + hf * 4 + k];
        }
        if (qw >= nq) continue;                           // wave-uniform: no query in this wave
        int m1[kL2QT], m2[kL2QT];
#pragma unroll
        for (int qt = 0; qt < kL2QT; ++qt) { m1[qt] = INT_MAX; m2[qt] = INT_MAX; }
        const int ntile = (min(kL2Chunk, c_end - c0) + 31) >> 5;
        for (int tt = 0; tt < ntile; ++tt) {
            const uint4* a = tr + tt * 4 * 64 + lane;
            const v4i_t A0 = as_v4i(a[0], 0u), A1 = as_v4i(a[64], 0u), A2 = as_v4i(a[128], 0u), A3 = as_v4i(a[192], 0u);
            const int4* tp = reinterpret_cast<const int4*>(t7 + tt * 32 + 4 * h);
            const int4 g[4] = {tp[0], tp[2], tp[4], tp[6]};   // rows 8 j + 4 h + 0..3
#pragma unroll
            for (int qt = 0; qt < kL2QT; ++qt) {
                v16i_t acc = {};
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, B[qt][0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, B[qt][1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(A2, B[qt][2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(A3, B[qt][3], acc, 0, 0, 0);
                int key[16];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    key[4 * j + 0] = g[j].x + acc[4 * j + 0] * 256;
                    key[4 * j + 1] = g[j].y + acc[4 * j + 1] * 256;
                    key[4 * j + 2] = g[j].z + acc[4 * j + 2] * 256;
                    key[4 * j + 3] = g[j].w + acc[4 * j + 3] * 256;
                }
#pragma unroll
                for (int r = 0; r < 16; r += 2) {         // the two smallest of {m1, m2, x, y}
                    m2[qt] = min(m2[qt], med3_i32(m1[qt], key[r], key[r + 1]));
                    m1[qt] = min(min(m1[qt], key[r]), key[r + 1]);
                }
            }
        }
        // the chunk's two smallest keys, decoded to (value, train index); missing rows decode
        // to values of 2^23 and above
#pragma unroll
        for (int qt = 0; qt < kL2QT; ++qt) {
            const int v1 = m1[qt] >> 7, v2 = m2[qt] >> 7;
            const long long b1 = v1 < (1 << 23) ? lex(v1, c0 + (m1[qt] & 127)) : kNone;
            const long long b2 = v2 < (1 << 23) ? lex(v2, c0 + (m2[qt] & 127)) : kNone;
            merge2(K1[qt], K2[qt], b1, b2);
        }
    }
#pragma unroll
    for (int qt = 0; qt < kL2QT; ++qt) {
        // lanes h = 0 and 1 saw disjoint rows of the same query column
        const long long o1 = __shfl_xor(K1[qt], 32), o2 = __shfl_xor(K2[qt], 32);
        merge2(K1[qt], K2[qt], o1, o2);
        const int qi = qw + qt * 32 + m;
        if (h == 0 && qi < nq)
            part[size_t(blockIdx.y) * nq + qi] =
                make_int4(int(K1[qt] >> 32), int(uint32_t(K1[qt])), int(K2[qt] >> 32), int(uint32_t(K2[qt])));
    }
}

// Per query: the slices' best pairs merged in slice order, the squared distances restored
// (d^2 = value + P_q), the ratio test den^2 d1^2 < num^2 d2^2 with at least two train rows.
__global__ void __launch_bounds__(256)
k_match_l2_final(const uint4* __restrict__ q, int nq, int nt, const int4* __restrict__ part, int n_slices, int num,
                 int den, xa_l2_match* __restrict__ out, int32_t* __restrict__ count) {
    const int qi = blockIdx.x * 256 + threadIdx.x;
    if (qi >= nq) return;
    long long K1 = kNone, K2 = kNone;
    for (int s = 0; s < n_slices; ++s) {
        const int4 p = part[size_t(s) * nq + qi];
        merge2(K1, K2, lex(p.x, p.y), lex(p.z, p.w));
    }
    uint32_t sq = 0, s1 = 0;
#pragma unroll
    for (int k = 0; k < kL2DescWords; ++k) {
        const uint4 w = q[size_t(qi) * kL2DescWords + k];
        sq = udot4(w.x, w.x, udot4(w.y, w.y, udot4(w.z, w.z, udot4(w.w, w.w, sq))));
        s1 = udot4(w.x, 0x01010101u, udot4(w.y, 0x01010101u, udot4(w.z, 0x01010101u, udot4(w.w, 0x01010101u, s1))));
    }
    const int pq = int(sq) - 254 * int(s1) + 4161536;
    const int i1 = int(uint32_t(K1)), i2 = int(uint32_t(K2));
    const bool has1 = int(K1 >> 32) < kL2NoVal, has2 = int(K2 >> 32) < kL2NoVal;
    xa_l2_match o;
    o.t = has1 ? i1 : -1;
    o.d1 = has1 ? uint32_t(int(K1 >> 32) + pq) : 0xFFFFFFFFu;
    o.d2 = has2 ? uint32_t(int(K2 >> 32) + pq) : 0xFFFFFFFFu;
    out[qi] = o;
    const bool accept = nt >= 2 && has2 &&
                        static_cast<long long>(den) * den * o.d1 < static_cast<long long>(num) * num * o.d2;
    if (accept) atomicAdd(count, 1);
}

__global__ void k_l2_zero(int32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

struct L2Launch {
    int qblocks, n_slices, chunks_per_slice;
};

L2Launch l2_launch(int nq, int nt) {
    L2Launch L;
    L.qblocks = (nq + kL2BlockQ - 1) / kL2BlockQ;
    const int n_chunks = (nt + kL2Chunk - 1) / kL2Chunk;
    int want = std::max(1, (kL2TargetBlocks + std::max(L.qblocks, 1) - 1) / std::max(L.qblocks, 1));
    want = std::min(want, std::max(n_chunks, 1));
    L.chunks_per_slice = std::max(1, (n_chunks + want - 1) / want);
    L.n_slices = std::max(1, (n_chunks + L.chunks_per_slice - 1) / L.chunks_per_slice);
    return L;
}

}  // namespace
}  // namespace xa

using namespace xa;

// Scratch of the allocation-free entry: every device the library runs on holds one copy of
// this array until the process ends.  In host code its name stands for the host-side shadow,
// not a device address, so kernels are only ever given the address hipGetSymbolAddress returns
// for the current device.
static __device__ __align__(256) int4 scratch[XA_L2_NOALLOC_SCRATCH_BYTES / sizeof(int4)];

namespace xa {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of the scratch array, looked up once per device.
xa_status scratch_for_current_device(int4** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(XA_EUNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || reinterpret_cast<uintptr_t>(p) % 256) return fail(XA_EHIP, "scratch array address not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<int4*>(g_scratch_ptr[dev]);
    return XA_OK;
}

}  // namespace
}  // namespace xa

extern "C" size_t xa_match_l2_workspace_size(int32_t n_q, int32_t n_t) {
    if (n_q < 0 || n_t < 0) return 0;
    const L2Launch L = l2_launch(n_q, n_t);
    return size_t(L.n_slices) * size_t(n_q) * sizeof(int4);
}

namespace xa {
namespace {

xa_status l2_check(const uint8_t* d_q, int32_t n_q, const uint8_t* d_t, int32_t n_t, int32_t ratio_num,
                   int32_t ratio_den, const xa_l2_match* d_out, const int32_t* d_count) {
    if (n_q < 0 || n_t < 0 || n_q > XA_L2_MAX_DESCRIPTORS || n_t > XA_L2_MAX_DESCRIPTORS)
        return fail(XA_EINVAL, "descriptor counts must lie in 0..%d", XA_L2_MAX_DESCRIPTORS);
    if (ratio_num < 0 || ratio_den < 1 || ratio_num > (1 << 16) || ratio_den > (1 << 16))
        return fail(XA_EINVAL, "ratio must be num/den with 0 <= num, 1 <= den <= 2^16");
    if (!d_count || (n_q > 0 && (!d_q || !d_out)) || (n_t > 0 && !d_t)) return fail(XA_EINVAL, "NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(d_q) | reinterpret_cast<uintptr_t>(d_t)) % 16)
        return fail(XA_EINVAL, "descriptor arrays must be 16-byte aligned");
    return XA_OK;
}

// The count is cleared by a kernel (no memset node, so the sequence can be graph-captured),
// then the slices' partial results go to part and the final pass merges them.
xa_status l2_enqueue(const uint8_t* d_q, int32_t n_q, const uint8_t* d_t, int32_t n_t, int32_t ratio_num,
                     int32_t ratio_den, xa_l2_match* d_out, int32_t* d_count, int4* part, hipStream_t stream) {
    hipLaunchKernelGGL(k_l2_zero, dim3(1), dim3(64), 0, stream, d_count);
    if (n_q > 0) {
        const L2Launch L = l2_launch(n_q, n_t);
        hipLaunchKernelGGL(k_match_l2, dim3(unsigned(L.qblocks), unsigned(L.n_slices)), dim3(kL2Threads), 0, stream,
                           reinterpret_cast<const uint4*>(d_q), n_q, reinterpret_cast<const uint4*>(d_t), n_t,
                           L.chunks_per_slice, part);
        hipLaunchKernelGGL(k_match_l2_final, dim3(unsigned((n_q + 255) / 256)), dim3(256), 0, stream,
                           reinterpret_cast<const uint4*>(d_q), n_q, n_t, part, L.n_slices, ratio_num, ratio_den,
                           d_out, d_count);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "L2 match launch");
    return ok();
}

}  // namespace
}  // namespace xa

extern "C" xa_status xa_match_l2(const uint8_t* d_q, int32_t n_q, const uint8_t* d_t, int32_t n_t, int32_t ratio_num,
                                 int32_t ratio_den, xa_l2_match* d_out, int32_t* d_count, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream) {
    const xa_status st = l2_check(d_q, n_q, d_t, n_t, ratio_num, ratio_den, d_out, d_count);
    if (st != XA_OK) return st;
    const size_t need = xa_match_l2_workspace_size(n_q, n_t);
    if (need > 0 && (!d_ws || ws_bytes < need || reinterpret_cast<uintptr_t>(d_ws) % 16))
        return fail(XA_EINVAL, "workspace of %zu bytes (16-byte aligned) needed, %zu given", need, ws_bytes);
    return l2_enqueue(d_q, n_q, d_t, n_t, ratio_num, ratio_den, d_out, d_count, static_cast<int4*>(d_ws), stream);
}

extern "C" xa_status xa_match_l2_noalloc(const uint8_t* d_q, int32_t n_q, const uint8_t* d_t, int32_t n_t,
                                         int32_t ratio_num, int32_t ratio_den, xa_l2_match* d_out, int32_t* d_count,
                                         hipStream_t stream) {
    xa_status st = l2_check(d_q, n_q, d_t, n_t, ratio_num, ratio_den, d_out, d_count);
    if (st != XA_OK) return st;
    const size_t need = xa_match_l2_workspace_size(n_q, n_t);
    if (need > XA_L2_NOALLOC_SCRATCH_BYTES)
        return fail(XA_ECAPACITY, "%d x %d descriptors need %zu bytes of scratch, above the %zu-byte maximum", n_q, n_t,
                    need, size_t(XA_L2_NOALLOC_SCRATCH_BYTES));
    int4* part = nullptr;
    st = scratch_for_current_device(&part);
    if (st != XA_OK) return st;
    return l2_enqueue(d_q, n_q, d_t, n_t, ratio_num, ratio_den, d_out, d_count, part, stream);
}
