// All-view-pair brute-force Hamming matching on gfx950 (Sec. III.B) with the
// nearest / second-nearest ratio test (Sec. IV.C), the best view pair, and the
// precision of eqs. (5)-(6).  Two families of kernels compute the same result:
// integer XOR + popcount on the vector ALU (queries in registers, train
// descriptors streamed through LDS and read as wave-uniform broadcasts), and an
// exact fp4 matrix-core contraction of the descriptors read as +-1 vectors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

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

// Block = one view pair x (kMatchThreads * Q) queries.  A group is a cross product of query
// views [a0, a0 + na) and train views [b0, b0 + nb); blocks map to (group, pair, query block)
// through a prefix table (groups == nullptr: the single group `one`).  Each lane keeps Q
// queries and, per query, the two smallest packed keys (d << 13 | train index): the smallest
// key gives d1 and the smallest index attaining it, the second smallest gives d2 over the others.
template <int Q>
__global__ void __launch_bounds__(kMatchThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_match(const uint32_t* __restrict__ desc_q, const int32_t* __restrict__ count_q, const uint32_t* __restrict__ desc_t,
        const int32_t* __restrict__ count_t, const xa_match_group* __restrict__ groups,
        const int32_t* __restrict__ block_prefix, int n_groups, xa_match_group one, int qblocks, int N, int num,
        int den, xa_match* __restrict__ matches, int32_t* __restrict__ pair_count) {
    __shared__ uint4 tr[kMatchChunk * 2];
    __shared__ int s_acc;
    xa_match_group G = one;
    int local = blockIdx.x;
    if (groups) {
        const int gi = find_segment_wave(block_prefix, n_groups, blockIdx.x);
        G = groups[gi];
        local = blockIdx.x - block_prefix[gi];
    }
    const int qb = local % qblocks, pr = local / qblocks;
    const int i = pr / G.nb, j = pr - (pr / G.nb) * G.nb;
    const long long pair = G.pair_base + pr;
    const int va = G.a0 + i, vb = G.b0 + j;
    const int nq = min(max(count_q[va], 0), N), nt = min(max(count_t[vb], 0), N);
    const int q0 = qb * kMatchThreads * Q;
    if (q0 >= nq) return;
    uint32_t q[Q][8];
    uint32_t m1[Q], m2[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const int qi = q0 + a * kMatchThreads + threadIdx.x;
        if (qi < nq) {
            const uint4* p = reinterpret_cast<const uint4*>(desc_q + (size_t(va) * N + qi) * 8);
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
    const uint4* tb = reinterpret_cast<const uint4*>(desc_t + size_t(vb) * N * 8);
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

// ------------------------------------------------------------------ matrix-core variant
//
// With descriptor bits read as +1 / -1, the dot product of two 256-bit descriptors is
// 256 - 2 x their Hamming distance, so one view pair's distance table is the product of
// two +-1 matrices: an fp4 (e2m1) MFMA contraction whose every input and partial sum is a
// small integer, hence exact in fp32.  Train descriptors are the A rows and queries the B
// columns of v_mfma_scale_f32_32x32x64_f8f6f4 (unit scales), so each lane holds one query
// column and 16 train rows of a 32 x 32 tile.  The accumulator starts at
// 512 + (16383 - j) / 2^14 for train row j, so the result dot + 512 + that fraction lies in
// (255, 769) and is exact in fp32 (10 + 14 significant bits): the largest has the smallest
// distance and, among equal distances, the smallest index.  Rows past the train count have
// zero operands and start at 1, below every real row.  Positive floats order as their bit
// patterns, so the two largest per query are kept with integer v_max / v_med3.

constexpr int kMxThreads = 256;      // four waves
constexpr int kMxQT = 4;             // 32-query tiles per wave: a block owns 512 queries of one view pair
constexpr int kMxChunk = 256;        // train descriptors expanded into LDS per step (32 KiB)
constexpr int kMxBlockQ = (kMxThreads / 64) * 32 * kMxQT;

typedef int v8i_t __attribute__((ext_vector_type(8)));
typedef float v16f_t __attribute__((ext_vector_type(16)));

// byte -> 8 fp4 values, bit i -> nibble i: +1.0 (0x2) for a set bit, -1.0 (0xA) for a clear one
__device__ __forceinline__ uint32_t byte_pm1(uint32_t b) {
    uint32_t s = (b | (b << 12)) & 0x000F000Fu;
    s = (s | (s << 6)) & 0x03030303u;
    s = (s | (s << 3)) & 0x11111111u;
    return 0xAAAAAAAAu ^ (s << 3);
}

// one 32-bit descriptor word -> the 32 fp4 values of one lane's MFMA operand
__device__ __forceinline__ uint4 word_pm1(uint32_t w) {
    return make_uint4(byte_pm1(w & 0xFFu), byte_pm1((w >> 8) & 0xFFu), byte_pm1((w >> 16) & 0xFFu), byte_pm1(w >> 24));
}

__device__ __forceinline__ v8i_t operand(uint4 u) {
    v8i_t v = {int(u.x), int(u.y), int(u.z), int(u.w), 0, 0, 0, 0};
    return v;
}

// PACK: blocks of one train view take the group's query tiles packed: the 32-query tiles of all
// its query views, concatenated in view order, sixteen to a block, so views with few keypoints
// share a block instead of each filling a block of its own with padding.  Finding its tiles
// costs each block a scan of the group's counts before its first query load, which the plain
// mapping does not pay, so the two are separate matcher variants.  A group of more query views
// than kMxPackViews (the prefix over them lives in LDS) keeps one query view per block.
constexpr int kMxPackViews = 1024;

// Outputs as k_match's.  Block mapping per group: PACK (and at most kMxPackViews query views),
// block local = b nb + j takes packed tiles [16 b, 16 b + 16) against train view j (blocks past
// the group's tiles exit); otherwise as k_match (view pair, then query block of 512).  The K
// dimension is split alike for both operands: slice s of lane l is word 2 s + l / 32 of
// descriptor (tile row or column) l % 32, so the contraction pairs equal bits whatever order
// the hardware gives the 64 values of a slice.
template <bool PACK>
__global__ void __launch_bounds__(kMxThreads) __attribute__((amdgpu_waves_per_eu(3)))
k_match_mx(const uint32_t* __restrict__ desc_q, const int32_t* __restrict__ count_q, const uint32_t* __restrict__ desc_t,
           const int32_t* __restrict__ count_t, const xa_match_group* __restrict__ groups,
           const int32_t* __restrict__ block_prefix, int n_groups, xa_match_group one, int qblocks, int N, int num,
           int den, xa_match* __restrict__ matches, int32_t* __restrict__ pair_count) {
    // [tile of 32][slice][lane] operands of one chunk of train descriptors
    __shared__ uint4 tr[(kMxChunk / 32) * 4 * 64];
    __shared__ int s_pre[PACK ? kMxPackViews + 1 : 1];    // exclusive prefix of the query views' tiles
    __shared__ int s_cnt[PACK ? kMxPackViews : 1];        // the query views' clamped counts
    __shared__ int s_wsum[kMxThreads / 64];   // the count scan's wave sums (packed); [0] the block's count (plain)
    xa_match_group G = one;
    int local = blockIdx.x;
    if (groups) {
        const int gi = find_segment_wave(block_prefix, n_groups, blockIdx.x);
        G = groups[gi];
        local = blockIdx.x - block_prefix[gi];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane >> 5, m = lane & 31;
    // The block's sixteen 32-query tiles are dealt to the waves in turn (tile wv + 4 qt of the
    // block is slot qt of wave wv), so a partly filled block keeps every SIMD busy; nqt = the
    // wave's slots holding queries (the first nqt; empty slots are skipped).  Slot qt holds rows
    // [row0[qt], row0[qt] + 32) of query view sv[qt] (sn[qt] queries), of view pair sp[qt].
    int sv[kMxQT], row0[kMxQT], sn[kMxQT];
    long long sp[kMxQT];
    const bool packed = PACK && G.na <= kMxPackViews;
    int j = 0, vb = 0, nt = 0, nqt;
    const uint4* tb = nullptr;
    uint4 n0 = make_uint4(0, 0, 0, 0), n1 = n0;                // next chunk's descriptor of this thread
    if (packed) {
        // the train view first: its count and its first chunk's rows load while the query side
        // is worked out (rows past the count are loaded too, and masked when expanded)
        j = local % G.nb;
        vb = G.b0 + j;
        nt = min(max(count_t[vb], 0), N);
        tb = reinterpret_cast<const uint4*>(desc_t + size_t(vb) * N * 8);
        if (int(threadIdx.x) < N) { n0 = tb[2 * threadIdx.x]; n1 = tb[2 * threadIdx.x + 1]; }
        const int b = local / G.nb;
        {   // s_pre[v] = tiles of query views [0, v), s_cnt[v] = view v's clamped count, four views
            // a thread: up to 256 views wave 0 scans them alone (one barrier); beyond that every
            // wave scans its share and the waves' sums are combined (two barriers)
            const bool one_wave = G.na <= 4 * 64;
            const int nscan = one_wave ? 64 : kMxThreads;
            int c[4], tsum = 0, x = 0;
            if (!one_wave || wv == 0) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int v = 4 * int(threadIdx.x) + e;
                    const int n = v < G.na ? min(max(count_q[G.a0 + v], 0), N) : 0;
                    if (v < G.na) s_cnt[v] = n;
                    c[e] = (n + 31) >> 5;
                    tsum += c[e];
                }
                x = tsum;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const int y = __shfl_up(x, off);
                    if (lane >= off) x += y;
                }
            }
            int ex = x - tsum;
            if (!one_wave) {
                if (lane == 63) s_wsum[wv] = x;
                __syncthreads();
                for (int w = 0; w < wv; ++w) ex += s_wsum[w];
            }
            if (!one_wave || wv == 0) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int v = 4 * int(threadIdx.x) + e;
                    if (v <= G.na) s_pre[v] = ex;
                    ex += c[e];
                }
                if (int(threadIdx.x) == nscan - 1 && G.na == 4 * nscan) s_pre[G.na] = ex;
            }
            __syncthreads();
        }
        const int T = s_pre[G.na];
        if (16 * b >= T) return;
        nqt = __builtin_amdgcn_readfirstlane(min(max((T - 16 * b - wv + 3) >> 2, 0), kMxQT));
        // slot qt's view i (s_pre[i] <= u < s_pre[i + 1]) is the number of views v >= 1 with
        // s_pre[v] <= u, counted by ballots over the prefix
        int le[kMxQT] = {0, 0, 0, 0};
        for (int v0 = 1; v0 < G.na; v0 += 64) {
            const int v = v0 + lane;
            const int pv = v < G.na ? s_pre[v] : INT32_MAX;
#pragma unroll
            for (int qt = 0; qt < kMxQT; ++qt) le[qt] += __popcll(__ballot(pv <= 16 * b + wv + 4 * qt));
        }
#pragma unroll
        for (int qt = 0; qt < kMxQT; ++qt) {
            sv[qt] = G.a0; row0[qt] = 0; sn[qt] = 0; sp[qt] = 0;
            if (qt < nqt) {
                const int u = 16 * b + wv + 4 * qt;      // packed tile index, below T
                const int i = __builtin_amdgcn_readfirstlane(le[qt]);
                sv[qt] = G.a0 + i;
                row0[qt] = __builtin_amdgcn_readfirstlane((u - s_pre[i]) * 32);
                sn[qt] = __builtin_amdgcn_readfirstlane(s_cnt[i]);
                sp[qt] = G.pair_base + (long long)i * G.nb + j;
            }
        }
    } else {
        const int qb = local % qblocks, pr = local / qblocks;
        const int i = pr / G.nb;
        j = pr - i * G.nb;
        vb = G.b0 + j;
        const int nq = min(max(count_q[G.a0 + i], 0), N);
        nt = min(max(count_t[vb], 0), N);
        const int q0 = qb * kMxBlockQ;
        if (q0 >= nq) return;
        const int btiles = min((nq - q0 + 31) >> 5, kMxQT * 4);
        nqt = __builtin_amdgcn_readfirstlane(min(max((btiles - wv + 3) >> 2, 0), kMxQT));
#pragma unroll
        for (int qt = 0; qt < kMxQT; ++qt) {
            sv[qt] = G.a0 + i;
            row0[qt] = q0 + (wv + 4 * qt) * 32;
            sn[qt] = qt < nqt ? nq : 0;
            sp[qt] = G.pair_base + pr;
        }
    }
    uint4 B[kMxQT][4];
#pragma unroll
    for (int qt = 0; qt < kMxQT; ++qt) {
        const int qi = row0[qt] + m;
        const uint32_t* p = desc_q + (size_t(sv[qt]) * N + qi) * 8;
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) B[qt][sl] = word_pm1(qi < sn[qt] ? p[2 * sl + h] : 0u);
    }
    if (!packed) {   // one query view: its train view's first chunk loads after the queries
        tb = reinterpret_cast<const uint4*>(desc_t + size_t(vb) * N * 8);
        if (int(threadIdx.x) < nt) { n0 = tb[2 * threadIdx.x]; n1 = tb[2 * threadIdx.x + 1]; }
    }
    uint32_t m1[kMxQT], m2[kMxQT];
#pragma unroll
    for (int qt = 0; qt < kMxQT; ++qt) { m1[qt] = 0u; m2[qt] = 0u; }
    // start value of element r (tile row 8 (r / 4) + 4 h + r % 4) of a tile at base 0
    float f0[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) f0[r] = 512.0f + float(16383 - (8 * (r >> 2) + 4 * h + (r & 3))) * (1.0f / 16384.0f);
    for (int c0 = 0; c0 < nt; c0 += kMxChunk) {
        const int cn = min(kMxChunk, nt - c0);
        __syncthreads();
        {   // expand this thread's descriptor (chunk row t) into its 8 operand slots; rows
            // past the train count get zero operands
            const int t = threadIdx.x, tt = t >> 5, tm = t & 31;
            const bool live = t < cn;
            const uint32_t w[8] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w};
#pragma unroll
            for (int k = 0; k < 8; ++k)
                tr[(tt * 4 + (k >> 1)) * 64 + (k & 1) * 32 + tm] = live ? word_pm1(w[k]) : make_uint4(0, 0, 0, 0);
        }
        __syncthreads();
        {
            const int nx = c0 + kMxChunk + int(threadIdx.x);
            if (nx < nt) { n0 = tb[2 * size_t(nx)]; n1 = tb[2 * size_t(nx) + 1]; }
        }
        if (nqt == 0) continue;
        // keys are positive floats, whose order is their bit patterns' order.  Per pair
        // {x, y}: the largest of {m1, x, y} is max3(m1, x, y) and the runner-up med3(m1, x, y);
        // the second largest of everything seen is the largest runner-up, so two pairs'
        // runners-up join m2 in one max3: five instructions for four keys.  The float median
        // is a builtin, so the compiler inserts the wait states an MFMA result needs before a
        // VALU read.
        auto update = [&](int qt, const v16f_t& k) {
#pragma unroll
            for (int r = 0; r < 16; r += 4) {
                const float mid0 = __builtin_amdgcn_fmed3f(__uint_as_float(m1[qt]), k[r], k[r + 1]);
                m1[qt] = max(max(m1[qt], __float_as_uint(k[r])), __float_as_uint(k[r + 1]));
                const float mid1 = __builtin_amdgcn_fmed3f(__uint_as_float(m1[qt]), k[r + 2], k[r + 3]);
                m1[qt] = max(max(m1[qt], __float_as_uint(k[r + 2])), __float_as_uint(k[r + 3]));
                m2[qt] = max(max(m2[qt], __float_as_uint(mid0)), __float_as_uint(mid1));
            }
        };
        // one tile of 32 train descriptors against the wave's query tiles (a partly filled
        // tile computes unused columns)
        auto contract = [&](int tt, const v16f_t& ci) {
            const uint4* a = tr + tt * 4 * 64 + lane;
            const v8i_t A0 = operand(a[0]), A1 = operand(a[64]), A2 = operand(a[128]), A3 = operand(a[192]);
            // each chain, then its updates (a slot past nqt holds no query)
#pragma unroll
            for (int qt = 0; qt < kMxQT; ++qt) {
                if (qt >= nqt) break;
                v16f_t acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A0, operand(B[qt][0]), ci, 4, 4, 0, 127, 0, 127);
                acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A1, operand(B[qt][1]), acc, 4, 4, 0, 127, 0, 127);
                acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A2, operand(B[qt][2]), acc, 4, 4, 0, 127, 0, 127);
                acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A3, operand(B[qt][3]), acc, 4, 4, 0, 127, 0, 127);
                update(qt, acc);
            }
        };
        // whole tiles first; a ragged last tile starts its rows past the train count at 1,
        // below every real key (their operands are zero)
        const int nfull = cn >> 5;
        for (int tt = 0; tt < nfull; ++tt) {
            const float fb = float(c0 + tt * 32) * (1.0f / 16384.0f);
            v16f_t ci;
#pragma unroll
            for (int r = 0; r < 16; ++r) ci[r] = f0[r] - fb;
            contract(tt, ci);
        }
        if (cn & 31) {
            const int base = c0 + nfull * 32;
            const float fb = float(base) * (1.0f / 16384.0f);
            v16f_t ci;
#pragma unroll
            for (int r = 0; r < 16; ++r) ci[r] = base + 8 * (r >> 2) + 4 * h + (r & 3) < nt ? f0[r] - fb : 1.0f;
            contract(nfull, ci);
        }
    }
    // PACK: a block may span several view pairs, so each slot adds its accepted count; the
    // plain variant's block is one view pair and adds its count once
    if constexpr (!PACK) {
        if (threadIdx.x == 0) s_wsum[0] = 0;
        __syncthreads();
    }
    int cnt = 0;
#pragma unroll
    for (int qt = 0; qt < kMxQT; ++qt) {
        if (qt >= nqt) break;
        // lanes l and l + 32 saw disjoint rows of the same query column
        const uint32_t o1 = __shfl_xor(m1[qt], 32), o2 = __shfl_xor(m2[qt], 32);
        const float b1 = __uint_as_float(max(m1[qt], o1));
        const float b2 = __uint_as_float(max(min(m1[qt], o1), max(m2[qt], o2)));
        const int qi = row0[qt] + m;
        int acc = 0;
        if (h == 0 && qi < sn[qt]) {
            xa_match r;
            int d1 = 65535, d2 = 65535;
            r.t = -1;
            if (nt > 0) {   // b1 = (256 - 2 d1) + 512 + (16383 - t) / 2^14
                const float it = floorf(b1);
                r.t = 16383 - int((b1 - it) * 16384.0f);
                d1 = (768 - int(it)) >> 1;
            }
            if (nt > 1) d2 = (768 - int(floorf(b2))) >> 1;
            r.d1 = uint16_t(d1);
            r.d2 = uint16_t(d2);
            matches[size_t(sp[qt]) * N + qi] = r;
            acc = (nt >= 2 && den * d1 < num * d2) ? 1 : 0;
        }
        if constexpr (PACK) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
            if (lane == 0 && acc) atomicAdd(&pair_count[sp[qt]], acc);
        } else {
            cnt += acc;
        }
    }
    if constexpr (!PACK) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
        if (lane == 0 && cnt) atomicAdd(&s_wsum[0], cnt);
        __syncthreads();
        if (threadIdx.x == 0 && s_wsum[0]) atomicAdd(&pair_count[sp[0]], s_wsum[0]);
    }
}

// Per group: argmax of the pair counts, lowest pair index on ties, as the max over
// (count << 32 | ~local pair); best[4 g ..] = local pair, i, j, count.
__global__ void __launch_bounds__(1024) k_best(const int32_t* __restrict__ pair_count,
                                               const xa_match_group* __restrict__ groups, xa_match_group one,
                                               int32_t* __restrict__ best) {
    __shared__ unsigned long long s[16];
    const xa_match_group G = groups ? groups[blockIdx.x] : one;
    const int n_pairs = G.na * G.nb;
    unsigned long long key = 0;
    for (int p = threadIdx.x; p < n_pairs; p += blockDim.x) {
        const unsigned long long k =
            ((unsigned long long)(uint32_t)pair_count[G.pair_base + p] << 32) | (0xFFFFFFFFu - uint32_t(p));
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
        int32_t* b = best + 4 * size_t(blockIdx.x);
        if (n_pairs > 0) {
            const int p = int(0xFFFFFFFFu - uint32_t(m & 0xFFFFFFFFull));
            b[0] = p;
            b[1] = p / G.nb;
            b[2] = p % G.nb;
            b[3] = int(m >> 32);
        } else {  // no view pairs: no best pair
            b[0] = b[1] = b[2] = -1;
            b[3] = 0;
        }
    }
}

struct H9 {
    double h[9];
};

// |H (x, y) - (bx, by)| <= th of eqs. (5)-(6), evaluated term by term without contraction, so
// that it rounds as the plain evaluation (device code is otherwise built with multiply-adds fused)
__device__ __forceinline__ bool within_th(const H9& H, double x, double y, double bx, double by, double th) {
#pragma clang fp contract(off)
    const double w = H.h[6] * x + H.h[7] * y + H.h[8];
    const double px = (H.h[0] * x + H.h[1] * y + H.h[2]) / w;
    const double py = (H.h[3] * x + H.h[4] * y + H.h[5]) / w;
    const double ex = px - bx, ey = py - by;
    return sqrt(ex * ex + ey * ey) <= th;
}

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
        n += 1;
        ok += within_th(H, a.xs, a.ys, b.xs, b.ys, th) ? 1 : 0;
    }
    atomicAdd(&s_ok, ok);
    atomicAdd(&s_n, n);
    __syncthreads();
    if (threadIdx.x == 0) { out[0] = s_ok; out[1] = s_n; }
}

}  // namespace

// the variant taken when none is named: the matrix-core kernel (about 4x the popcount
// kernels' rate at a thousand features per view)
static int pick_q(int) { return XA_MATCH_MATRIX; }

// queries one block of matcher variant Q owns (Q = XA_MATCH_MATRIX[_PACKED]: the matrix-core
// kernel; the packed form's grid keeps the bound of one 512-query block per view pair)
static int block_queries(int Q) {
    return Q == XA_MATCH_MATRIX || Q == XA_MATCH_MATRIX_PACKED ? kMxBlockQ : kMatchThreads * Q;
}

xa_status launch_match_any(const uint8_t* desc_q, const int32_t* count_q, const uint8_t* desc_t,
                           const int32_t* count_t, const xa_match_group* groups_dev, const int32_t* prefix_dev,
                           int n_groups, const xa_match_group& one, long long total_pairs, long long total_blocks,
                           int N, int Q, int num, int den, xa_match* matches, int32_t* pair_count, int32_t* best,
                           hipStream_t st, bool counts_zeroed = false) {
    if (total_blocks > INT32_MAX || total_pairs > INT32_MAX) return fail(XA_EUNSUPPORTED, "too many view pairs");
    if (total_pairs > 0 && !counts_zeroed)
        hipLaunchKernelGGL(k_fill_i32, dim3(unsigned((total_pairs + 255) / 256)), dim3(256), 0, st, pair_count,
                           int(total_pairs), 0);
    const uint32_t* dq = reinterpret_cast<const uint32_t*>(desc_q);
    const uint32_t* dt = reinterpret_cast<const uint32_t*>(desc_t);
    const int qblocks = (N + block_queries(Q) - 1) / block_queries(Q);
    if (total_blocks > 0) {
        if (Q == XA_MATCH_MATRIX_PACKED)
            hipLaunchKernelGGL(k_match_mx<true>, dim3(unsigned(total_blocks)), dim3(kMxThreads), 0, st, dq, count_q, dt,
                               count_t, groups_dev, prefix_dev, n_groups, one, qblocks, N, num, den, matches, pair_count);
        else if (Q == XA_MATCH_MATRIX)
            hipLaunchKernelGGL(k_match_mx<false>, dim3(unsigned(total_blocks)), dim3(kMxThreads), 0, st, dq, count_q, dt,
                               count_t, groups_dev, prefix_dev, n_groups, one, qblocks, N, num, den, matches, pair_count);
        else if (Q == 4)
            hipLaunchKernelGGL(k_match<4>, dim3(unsigned(total_blocks)), dim3(kMatchThreads), 0, st, dq, count_q, dt,
                               count_t, groups_dev, prefix_dev, n_groups, one, qblocks, N, num, den, matches, pair_count);
        else if (Q == 2)
            hipLaunchKernelGGL(k_match<2>, dim3(unsigned(total_blocks)), dim3(kMatchThreads), 0, st, dq, count_q, dt,
                               count_t, groups_dev, prefix_dev, n_groups, one, qblocks, N, num, den, matches, pair_count);
        else
            hipLaunchKernelGGL(k_match<1>, dim3(unsigned(total_blocks)), dim3(kMatchThreads), 0, st, dq, count_q, dt,
                               count_t, groups_dev, prefix_dev, n_groups, one, qblocks, N, num, den, matches, pair_count);
    }
    hipLaunchKernelGGL(k_best, dim3(groups_dev ? n_groups : 1), dim3(1024), 0, st, pair_count, groups_dev, one, best);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "match launch");
    return XA_OK;
}

xa_status launch_match(const uint8_t* desc_a, const int32_t* count_a, int32_t n_a, const uint8_t* desc_b,
                       const int32_t* count_b, int32_t n_b, int32_t N, int32_t num, int32_t den, xa_match* matches,
                       int32_t* pair_count, int32_t* best, hipStream_t st, bool counts_zeroed) {
    const int Q = pick_q(N);
    const int qblocks = (N + block_queries(Q) - 1) / block_queries(Q);
    const xa_match_group one{0, n_a, 0, n_b, 0};
    return launch_match_any(desc_a, count_a, desc_b, count_b, nullptr, nullptr, 1, one, (long long)n_a * n_b,
                            (long long)n_a * n_b * qblocks, N, Q, num, den, matches, pair_count, best, st,
                            counts_zeroed);
}

// ------------------------------------------------------------------ match plans

xa_status match_plan_view(const void* blob, MatchPlanView* out) {
    if (!blob) return fail(XA_EINVAL, "match plan is NULL");
    const auto* h = static_cast<const MatchPlanHeader*>(blob);
    if (h->magic != kMatchMagic) return fail(XA_EINVAL, "not a match plan");
    out->h = h;
    return XA_OK;
}

xa_status launch_match_plan(const void* mplan_host, const void* mplan_dev, const uint8_t* desc, const int32_t* count,
                            int32_t num, int32_t den, xa_match* matches, int32_t* pair_count, int32_t* best,
                            hipStream_t st, bool counts_zeroed) {
    const auto* h = static_cast<const MatchPlanHeader*>(mplan_host);
    const char* d = static_cast<const char*>(mplan_dev);
    const xa_match_group one{0, 0, 0, 0, 0};
    return launch_match_any(desc, count, desc, count, reinterpret_cast<const xa_match_group*>(d + h->off_groups),
                            reinterpret_cast<const int32_t*>(d + h->off_prefix), h->n_groups, one, h->total_pairs,
                            h->total_blocks, h->n_features, h->q, num, den, matches, pair_count, best, st,
                            counts_zeroed);
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

extern "C" xa_status xa_plan_matches(const xa_match_group* groups, int32_t n_groups, int32_t n_features,
                                     int32_t queries_per_lane, void* blob, size_t blob_cap, size_t* blob_bytes) {
    if (!blob_bytes || !groups || n_groups < 1) return fail(XA_EINVAL, "need at least one group");
    if (n_features < 1 || n_features > XA_MAX_FEATURES) return fail(XA_EUNSUPPORTED, "n_features out of range");
    const int Q = queries_per_lane == 0 ? pick_q(n_features) : queries_per_lane;
    if (Q != 1 && Q != 2 && Q != 4 && Q != XA_MATCH_MATRIX && Q != XA_MATCH_MATRIX_PACKED)
        return fail(XA_EINVAL, "queries_per_lane must be 0 (auto), 1, 2, 4, XA_MATCH_MATRIX or XA_MATCH_MATRIX_PACKED");
    const int qblocks = (n_features + block_queries(Q) - 1) / block_queries(Q);
    std::vector<int32_t> prefix(n_groups + 1, 0);
    long long blocks = 0, pairs = 0, views = 0;
    for (int g = 0; g < n_groups; ++g) {
        const xa_match_group& G = groups[g];
        if (G.na < 0 || G.nb < 0 || G.a0 < 0 || G.b0 < 0 || G.pair_base < 0)
            return fail(XA_EINVAL, "group %d: negative field", g);
        views = std::max(views, std::max((long long)G.a0 + G.na, (long long)G.b0 + G.nb));
        if (views > INT32_MAX) return fail(XA_EINVAL, "group %d: view index overflow", g);
        prefix[g] = int32_t(blocks);
        blocks += (long long)G.na * G.nb * qblocks;
        pairs = std::max(pairs, (long long)G.pair_base + (long long)G.na * G.nb);
        if (blocks > INT32_MAX / 2) return fail(XA_EUNSUPPORTED, "too many view pairs for one launch");
    }
    prefix[n_groups] = int32_t(blocks);
    {   // disjoint pair ranges: no two groups write the same view pair
        std::vector<std::pair<long long, long long>> r;
        for (int g = 0; g < n_groups; ++g)
            if (groups[g].na > 0 && groups[g].nb > 0)
                r.emplace_back(groups[g].pair_base, groups[g].pair_base + (long long)groups[g].na * groups[g].nb);
        std::sort(r.begin(), r.end());
        for (size_t i = 1; i < r.size(); ++i)
            if (r[i].first < r[i - 1].second) return fail(XA_EINVAL, "groups write overlapping pair ranges");
    }
    MatchPlanHeader h{};
    h.magic = kMatchMagic;
    h.n_groups = n_groups;
    h.n_features = n_features;
    h.q = Q;
    h.views_needed = int32_t(views);
    h.total_blocks = blocks;
    h.total_pairs = pairs;
    size_t o = align_up(sizeof(h), 64);
    h.off_groups = int64_t(o); o = align_up(o + sizeof(xa_match_group) * n_groups, 64);
    h.off_prefix = int64_t(o); o = align_up(o + 4 * prefix.size(), 64);
    h.total_bytes = int64_t(o);
    *blob_bytes = o;
    if (!blob) return ok();
    if (blob_cap < o) return fail(XA_ECAPACITY, "match plan needs %zu bytes, buffer has %zu", o, blob_cap);
    char* b = static_cast<char*>(blob);
    std::memset(b, 0, o);
    std::memcpy(b, &h, sizeof(h));
    std::memcpy(b + h.off_groups, groups, sizeof(xa_match_group) * n_groups);
    std::memcpy(b + h.off_prefix, prefix.data(), 4 * prefix.size());
    return ok();
}

extern "C" xa_status xa_match_groups(const void* mplan_host, const void* mplan_dev, const uint8_t* d_desc,
                                     const int32_t* d_count, int32_t n_views, int32_t ratio_num, int32_t ratio_den,
                                     xa_match* d_matches, int32_t* d_pair_count, int32_t* d_best, hipStream_t stream) {
    MatchPlanView mv;
    xa_status s = match_plan_view(mplan_host, &mv);
    if (s != XA_OK) return s;
    if (mv.h->views_needed > n_views)
        return fail(XA_EINVAL, "match plan reads %d views, descriptor set has %d", mv.h->views_needed, n_views);
    if (!mplan_dev || !d_desc || !d_count || !d_matches || !d_pair_count || !d_best)
        return fail(XA_EINVAL, "NULL device pointer");
    if (reinterpret_cast<uintptr_t>(d_desc) % 16) return fail(XA_EINVAL, "descriptors must be 16-byte aligned");
    if (ratio_num < 0 || ratio_den < 1 || ratio_num > (1 << 20) || ratio_den > (1 << 20))
        return fail(XA_EINVAL, "ratio must be num/den with 0 <= num, 1 <= den <= 2^20");
    s = launch_match_plan(mplan_host, mplan_dev, d_desc, d_count, ratio_num, ratio_den, d_matches, d_pair_count,
                          d_best, stream);
    return s == XA_OK ? ok() : s;
}

// the variants the tuner times, in the order of its ms[] output
static constexpr int kTuneVariants = 5;

extern "C" size_t xa_tune_matcher_workspace_size(const xa_match_group* groups, int32_t n_groups, int32_t n_features) {
    size_t most = 0;
    const int variants[kTuneVariants] = {1, 2, 4, XA_MATCH_MATRIX, XA_MATCH_MATRIX_PACKED};
    for (int v : variants) {
        size_t bytes = 0;
        if (xa_plan_matches(groups, n_groups, n_features, v, nullptr, 0, &bytes) != XA_OK) return 0;
        most = std::max(most, bytes);
    }
    return align_up(most);
}

namespace {
// The tuner's results, per device, keyed by everything the matcher's run time depends on: the
// group table, n_features and the per-view counts (the descriptor bits do not matter).
struct TuneEntry {
    int32_t best;
    float ms[kTuneVariants];
};
std::mutex g_tune_mu;
std::map<std::pair<int, uint64_t>, TuneEntry> g_tune_cache;

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const uint8_t* b = static_cast<const uint8_t*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}
}  // namespace

extern "C" xa_status xa_tune_matcher(const xa_match_group* groups, int32_t n_groups, int32_t n_features,
                                     const uint8_t* d_desc, const int32_t* d_count, int32_t n_views, int32_t reps,
                                     int32_t flags, xa_match* d_matches, int32_t* d_pair_count, int32_t* d_best,
                                     void* d_ws, size_t ws_bytes, hipStream_t stream, int32_t* best_variant,
                                     float* ms) {
    if (!best_variant) return fail(XA_EINVAL, "NULL output");
    if (reps < 1 || reps > 1000) return fail(XA_EINVAL, "reps must lie in 1..1000");
    if (flags & ~XA_TUNE_USE_CACHE) return fail(XA_EINVAL, "unknown flags 0x%x", unsigned(flags));
    const size_t need = xa_tune_matcher_workspace_size(groups, n_groups, n_features);
    if (need == 0) return fail(XA_EINVAL, "invalid match groups");
    if (!d_ws || ws_bytes < need || reinterpret_cast<uintptr_t>(d_ws) % kAlign)
        return fail(XA_EINVAL, "workspace of %zu bytes (256-byte aligned) needed, %zu given", need, ws_bytes);
    if (!d_count || n_views < 1) return fail(XA_EINVAL, "need the per-view counts");
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::vector<int32_t> counts(size_t(n_views), 0);
    e = hipMemcpyAsync(counts.data(), d_count, counts.size() * sizeof(int32_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "count download");
    uint64_t key = fnv1a(1469598103934665603ull, groups, size_t(n_groups) * sizeof(xa_match_group));
    key = fnv1a(key, &n_features, sizeof n_features);
    key = fnv1a(key, counts.data(), counts.size() * sizeof(int32_t));
    if (flags & XA_TUNE_USE_CACHE) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const auto it = g_tune_cache.find({device, key});
        if (it != g_tune_cache.end()) {
            *best_variant = it->second.best;
            if (ms) std::copy(it->second.ms, it->second.ms + kTuneVariants, ms);
            return ok();
        }
    }
    const int variants[kTuneVariants] = {1, 2, 4, XA_MATCH_MATRIX, XA_MATCH_MATRIX_PACKED};
    TuneEntry entry{};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "event create");
    xa_status s = XA_OK;
    float best = 0.0f;
    int best_v = 0;
    for (int i = 0; i < kTuneVariants && s == XA_OK; ++i) {
        size_t bytes = 0;
        s = xa_plan_matches(groups, n_groups, n_features, variants[i], nullptr, 0, &bytes);
        if (s != XA_OK) break;
        std::vector<uint8_t> blob(bytes);
        s = xa_plan_matches(groups, n_groups, n_features, variants[i], blob.data(), bytes, &bytes);
        if (s != XA_OK) break;
        e = hipMemcpyAsync(d_ws, blob.data(), bytes, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);     // the host blob goes out of scope below
        if (e != hipSuccess) { s = hip_fail(e, "plan upload"); break; }
        s = xa_match_groups(blob.data(), d_ws, d_desc, d_count, n_views, 4, 5, d_matches, d_pair_count, d_best, stream);
        e = hipEventRecord(e0, stream);
        for (int r = 0; r < reps && s == XA_OK; ++r)
            s = xa_match_groups(blob.data(), d_ws, d_desc, d_count, n_views, 4, 5, d_matches, d_pair_count, d_best,
                                stream);
        if (e == hipSuccess) e = hipEventRecord(e1, stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) { s = hip_fail(e, "matcher timing"); break; }
        t /= reps;
        entry.ms[i] = t;
        if (best_v == 0 || t < best) {
            best = t;
            best_v = variants[i];
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (s != XA_OK) return s;
    entry.best = best_v;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[{device, key}] = entry;
    }
    *best_variant = best_v;
    if (ms) std::copy(entry.ms, entry.ms + kTuneVariants, ms);
    return ok();
}
