// The Lanczos-4 affine warp of fp32 crops as a differentiable function of the image
// and of the six camera parameters (t, phi, psi, s, tx, ty), forward and adjoint.
//
// Resampling of eqs. (3)-(4): 8 x 8 taps (i, j = -3..4), weights normalised to sum one,
// border taps clamped.  The map is the camera map of eq. (2), L = s R(psi) diag(1/t, 1)
// R(phi), centred on the crop: view pixel q samples p = L^-1 (q - c - T) + c, with
// c = ((w - 1)/2, (h - 1)/2) and T = (tx, ty).  Pixels whose p leaves
// [-1/2, w - 1/2] x [-1/2, h - 1/2] are 0 and carry no gradient.
//
// Coordinates are fp64; weights and sums fp32; per-pixel parameter gradients fp64.  The tap
// weights and their derivatives in the fractional offset are the polynomial fits of lanczos.h
// (no transcendental, division or branch per tap).
//
// Launch structure.  A prologue kernel computes each crop's map (and its derivatives) once,
// together with the crop's tile shape: 512, 256 or 128 view pixels, as 2^k x (P / 2^k), the
// largest P and the k whose source box (the tile's footprint grown by the 8-tap window) fits
// the 32 KiB of LDS a block uses; crops whose box never fits read their taps from global memory
// at P = 512.  A scan gives each crop's first tile in one compact tile list, and a second
// prologue kernel writes each tile's descriptor (its source box and staging geometry, computed
// once per tile in fp64 rather than by every wave that works on it).  The main kernels launch
// one block per entry of that list's upper bound (the host does not know the crops' tile
// counts), dealt XCD-contiguously: each XCD (with its own L2) takes one contiguous eighth of the
// list, so neighbouring tiles, whose source boxes share lines, meet in one L2; blocks past the
// list's end return at once.  Each thread takes up to two pixels of a tile, 256 / 2^k rows apart.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"
#include "lanczos.h"

namespace xa {
namespace {

constexpr int kDwThreads = 256;
constexpr int kDwLds = 8192;          // 32 KiB: staged source floats (forward) or fixed-point sums (adjoint)
constexpr int kDwPixels[3] = {512, 256, 128};   // tile sizes, tried largest first
constexpr int kDwLog2Max = 8;         // tile widths 2 .. 256

struct CropMap {
    double m[4];      // L^-1, row-major
    double dm[4][4];  // d L^-1 / d(t, phi, psi, s)
    double cx, cy, tx, ty;
    int tw_log2, th;  // tile shape 2^tw_log2 x th
    int tiles_x, tiles;
    int px, log2_px;  // pixels per tile and their log2
    int pad[2];
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

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

// Tiles of a w x h crop at tile shape 2^k x th.
__host__ __device__ inline int tile_count(int w, int h, int k, int th, int* tiles_x) {
    const int tx = (w + (1 << k) - 1) >> k;
    if (tiles_x) *tiles_x = tx;
    return tx * ((h + th - 1) / th);
}

// Upper bound on the LDS words a tile's staged box takes (odd row stride, columns aligned down
// to a multiple of 4), from the extent of its pixel centres through L^-1.
__device__ inline double box_words(const CropMap& C, int tw, int th, int w, int h) {
    const double ex = (tw - 1) * fabs(C.m[0]) + (th - 1) * fabs(C.m[1]);
    const double ey = (tw - 1) * fabs(C.m[2]) + (th - 1) * fabs(C.m[3]);
    const double bw = fmin(ex + 10.0, double(w)) + 4.0;   // +3 alignment, +1 odd stride
    const double bh = fmin(ey + 10.0, double(h));
    return bw * bh;
}

// One thread per crop: the map, its derivatives and the tile shape.
__global__ void __launch_bounds__(64) k_dw_maps(const xa_affine_params* __restrict__ params, int n, int w, int h,
                                                CropMap* __restrict__ maps) {
    const int c = blockIdx.x * 64 + threadIdx.x;
    if (c >= n) return;
    CropMap C;
    crop_map(params[c], true, &C, w, h);
    int best_k = -1, best_p = 0;
    for (int pi = 0; pi < 3 && best_k < 0; ++pi) {
        const int P = kDwPixels[pi];
        double best = 1e300;
        for (int k = 1; k <= kDwLog2Max && (1 << k) < P; ++k) {
            const double a = box_words(C, 1 << k, P >> k, w, h);
            if (a < best) {
                best = a;
                best_k = k;
            }
        }
        if (best <= double(kDwLds)) best_p = P;
        else best_k = -1;
    }
    if (best_k < 0) {   // no shape fits: taps from global memory, at the largest tile
        best_p = kDwPixels[0];
        double best = 1e300;
        for (int k = 1; k <= kDwLog2Max && (1 << k) < best_p; ++k) {
            const double a = box_words(C, 1 << k, best_p >> k, w, h);
            if (a < best) {
                best = a;
                best_k = k;
            }
        }
    }
    C.tw_log2 = best_k;
    C.th = best_p >> best_k;
    C.px = best_p;
    C.log2_px = best_p == 512 ? 9 : (best_p == 256 ? 8 : 7);
    C.tiles = tile_count(w, h, best_k, C.th, &C.tiles_x);
    C.pad[0] = C.pad[1] = 0;
    maps[c] = C;
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

// A tile: its first pixel (x0, y0), its source box [bx0, bx1] x [by0, by1] (the pixel
// centres' bounding box through L^-1, grown by the 8-tap window, clamped to the crop; every
// clamped tap of a valid pixel of the tile lies in it), the staged copy's geometry (first
// column ax0, a multiple of 4 when rows load as 16 bytes; nc chunks per row; odd row stride
// ls) and flags.  Written once per tile by k_dw_tiles, read by the main kernels' blocks.
constexpr int kTileEmpty = 1;     // no pixel of the tile can be valid
constexpr int kTileStaged = 2;    // the staged box fits the LDS array (forward, adjoint without image gradient)
constexpr int kTileAccum = 4;     // the box's fixed-point sums fit the LDS array (adjoint image gradient)
struct TileDesc {
    int x0, y0, bx0, bx1, by0, by1;
    int ax0, nc, ls, flags;
    int crop, pad;
};

__device__ TileDesc make_tile(const CropMap& C, int tl, int w, int h, bool vec4) {
    TileDesc T;
    const int tw = 1 << C.tw_log2, th = C.th;
    const int tyi = tl / C.tiles_x, txi = tl - tyi * C.tiles_x;
    T.x0 = txi << C.tw_log2;
    T.y0 = tyi * th;
    const int x1 = min(T.x0 + tw, w) - 1, y1 = min(T.y0 + th, h) - 1;
    // corners of the pixel-centre parallelogram in the source
    const Sample S = sample_point(C, T.x0, T.y0, w, h);
    const double ux = C.m[0] * double(x1 - T.x0), uy = C.m[2] * double(x1 - T.x0);   // along the tile's x edge
    const double vx = C.m[1] * double(y1 - T.y0), vy = C.m[3] * double(y1 - T.y0);   // along its y edge
    const double pxl = S.px + fmin(ux, 0.0) + fmin(vx, 0.0), pxh = S.px + fmax(ux, 0.0) + fmax(vx, 0.0);
    const double pyl = S.py + fmin(uy, 0.0) + fmin(vy, 0.0), pyh = S.py + fmax(uy, 0.0) + fmax(vy, 0.0);
    const double eps = 1e-6;
    bool empty = pxh < -0.5 - eps || pxl > w - 0.5 + eps || pyh < -0.5 - eps || pyl > h - 0.5 + eps;
    // separating axes along the parallelogram's edge normals
    for (int e = 0; e < 2 && !empty; ++e) {
        const double nx = e == 0 ? -uy : -vy, ny = e == 0 ? ux : vx;
        const double nn = fabs(nx) + fabs(ny);
        if (!(nn > 0.0)) continue;
        // the parallelogram's extent along n: its two parallel edges project to a and a + d
        const double a = nx * S.px + ny * S.py;
        const double d = e == 0 ? nx * vx + ny * vy : nx * ux + ny * uy;
        const double qlo = a + fmin(d, 0.0), qhi = a + fmax(d, 0.0);
        // the crop rectangle's extent along n
        const double rlo = fmin(nx * -0.5, nx * (w - 0.5)) + fmin(ny * -0.5, ny * (h - 0.5));
        const double rhi = fmax(nx * -0.5, nx * (w - 0.5)) + fmax(ny * -0.5, ny * (h - 0.5));
        const double m = eps * nn;
        if (qhi < rlo - m || qlo > rhi + m) empty = true;
    }
    T.bx0 = max(int(fmax(floor(pxl - eps), -1e9)) - 3, 0);
    T.bx1 = min(int(fmin(floor(pxh + eps), 1e9)) + 4, w - 1);
    T.by0 = max(int(fmax(floor(pyl - eps), -1e9)) - 3, 0);
    T.by1 = min(int(fmin(floor(pyh + eps), 1e9)) + 4, h - 1);
    if (T.bx1 < T.bx0 || T.by1 < T.by0) empty = true;
    T.ax0 = vec4 ? (T.bx0 & ~3) : T.bx0;
    T.nc = vec4 ? ((T.bx1 - T.ax0) >> 2) + 1 : T.bx1 - T.bx0 + 1;
    T.ls = (T.nc * (vec4 ? 4 : 1)) | 1;
    const long long bh = T.by1 - T.by0 + 1, bw = T.bx1 - T.bx0 + 1;
    T.flags = 0;
    if (empty) T.flags = kTileEmpty;
    else {
        if ((long long)T.ls * bh <= kDwLds) T.flags |= kTileStaged;
        if (bw * bh <= kDwLds) T.flags |= kTileAccum;
    }
    T.pad = 0;
    return T;
}

// prefix[c] = tiles of crops 0..c-1 (prefix[n] = all tiles): one block, 256 crops per step.
__global__ void __launch_bounds__(256) k_dw_scan(const CropMap* __restrict__ maps, int n, int* __restrict__ prefix) {
    __shared__ int s[256];
    int carry = 0;
    for (int base = 0; base < n; base += 256) {
        const int i = base + int(threadIdx.x);
        const int v = i < n ? maps[i].tiles : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {    // inclusive scan of the step
            const int a = int(threadIdx.x) >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < n) prefix[i] = carry + s[threadIdx.x] - v;
        carry += s[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) prefix[n] = carry;
}

// Tile of block blockIdx.x, or -1: the hardware deals blocks to the 8 XCDs round-robin, so
// block b is the (b / 8)-th of XCD b % 8, which takes tiles [x q, (x + 1) q), q = ceil(total / 8).
__device__ inline int block_tile(int total) {
    const int q = (total + kXcds - 1) / kXcds;
    const int x = int(blockIdx.x) % kXcds, i = int(blockIdx.x) / kXcds;
    const int t = x * q + i;
    return i < q && t < total ? t : -1;
}

// One thread per (crop, tile slot below the most tiles any shape needs): the descriptor of the
// crop's tile tl, at its place in the compact list.
__global__ void __launch_bounds__(256) k_dw_tiles(const CropMap* __restrict__ maps, const int* __restrict__ prefix,
                                                  int n, int w, int h, int slots, int vec4,
                                                  TileDesc* __restrict__ tiles) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)n * slots) return;
    const int crop = int(i / slots), tl = int(i - (long long)crop * slots);
    const CropMap& C = maps[crop];
    if (tl >= C.tiles) return;
    TileDesc T = make_tile(C, tl, w, h, vec4 != 0);
    T.crop = crop;
    tiles[prefix[crop] + tl] = T;
}

// Stage the box rows [by0, by1], columns [ax0, ax0 + cw * nc) of the crop in LDS at row stride
// ls: 16-byte loads (cw = 4) when the crop's rows are 16-byte aligned, else 4-byte loads.
// Chunk e = r * nc + c; each thread starts at e = tid and steps by 256 = q * nc + rem chunks.
__device__ inline void stage_box(float* __restrict__ tile, const float* __restrict__ base, int w, int ax0, int by0,
                                 int nc, int bh, int ls, bool vec4) {
    const int n = nc * bh, q = kDwThreads / nc, rem = kDwThreads - q * nc;
    int e = int(threadIdx.x), r = e / nc, c = e - r * nc;
    if (vec4) {
        const float* g = base + size_t(by0 + r) * w + ax0 + 4 * c;
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
                    e += kDwThreads;
                    c += rem;
                    g += size_t(q) * w + 4 * rem;
                    lo += q * ls + 4 * rem;
                    if (c >= nc) {
                        c -= nc;
                        g += w - 4 * nc;
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
    } else {
        const float* g = base + size_t(by0 + r) * w + ax0 + c;
        int lo = r * ls + c;
        while (e < n) {
            tile[lo] = *g;
            e += kDwThreads;
            c += rem;
            g += size_t(q) * w + rem;
            lo += q * ls + rem;
            if (c >= nc) {
                c -= nc;
                g += w - nc;
                lo += ls - nc;
            }
        }
    }
}



__global__ void __launch_bounds__(kDwThreads) k_dw_fwd(const float* __restrict__ img, const CropMap* __restrict__ maps,
                                                       const TileDesc* __restrict__ tiles, const int* __restrict__ prefix,
                                                       int n, int w, int h, int vec4, float* __restrict__ out,
                                                       uint8_t* __restrict__ mask) {
    __shared__ float tile[kDwLds];
    const int t = block_tile(prefix[n]);
    if (t < 0) return;
    const TileDesc& T = tiles[t];
    const int crop = T.crop;
    const CropMap& C = maps[crop];
    const float* base = img + size_t(crop) * h * w;
    const bool empty = (T.flags & kTileEmpty) != 0, staged = (T.flags & kTileStaged) != 0;
    if (staged) {
        stage_box(tile, base, w, T.ax0, T.by0, T.nc, T.by1 - T.by0 + 1, T.ls, vec4 != 0);
        __syncthreads();
    }
    const int twm = (1 << C.tw_log2) - 1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e = int(threadIdx.x) + k * kDwThreads;
        if (e >= C.px) break;
        const int x = T.x0 + (e & twm), y = T.y0 + (e >> C.tw_log2);
        if (x >= w || y >= h) continue;
        const size_t o = (size_t(crop) * h + y) * w + x;
        float v = 0.0f;
        bool valid = false;
        if (!empty) {
            const Sample S = sample_point(C, x, y, w, h);
            valid = S.valid;
            if (valid) {
                const double fx0 = floor(S.px), fy0 = floor(S.py);
                const int ix = int(fx0), iy = int(fy0);
                float wx[8], wy[8];
                const float sx = lanczos4_weights(float(S.px - fx0), wx);
                const float sy = lanczos4_weights(float(S.py - fy0), wy);
                float acc = 0.0f;
                if (staged && ix >= 3 && ix + 4 <= w - 1 && iy >= 3 && iy + 4 <= h - 1) {
                    // interior: the window needs no clamping; rows at immediate offsets
                    const float* r0 = tile + (iy - 3 - T.by0) * T.ls + (ix - 3 - T.ax0);
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const float* r = r0 + j * T.ls;
                        float s = 0.0f;
#pragma unroll
                        for (int i = 0; i < 8; ++i) s = fmaf(wx[i], r[i], s);
                        acc = fmaf(wy[j], s, acc);
                    }
                } else if (staged) {
                    // clamped taps lie in the box: box-relative (non-negative) LDS offsets
                    int cols[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) cols[i] = clampi(ix - 3 + i, 0, w - 1) - T.ax0;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const float* r = tile + (clampi(iy - 3 + j, 0, h - 1) - T.by0) * T.ls;
                        float s = 0.0f;
#pragma unroll
                        for (int i = 0; i < 8; ++i) s = fmaf(wx[i], r[cols[i]], s);
                        acc = fmaf(wy[j], s, acc);
                    }
                } else {
                    int cols[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) cols[i] = clampi(ix - 3 + i, 0, w - 1);
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const float* r = base + size_t(clampi(iy - 3 + j, 0, h - 1)) * w;
                        float s = 0.0f;
#pragma unroll
                        for (int i = 0; i < 8; ++i) s = fmaf(wx[i], r[cols[i]], s);
                        acc = fmaf(wy[j], s, acc);
                    }
                }
                v = acc * __builtin_amdgcn_rcpf(sx * sy);
            }
        }
        out[o] = v;
        if (mask) mask[o] = valid ? 1 : 0;
    }
}

// Adjoint.  The image gradient of a tile is accumulated over its source box in LDS (integer
// atomics on a fixed-point scale, see below) when the box fits, then added to the crop's
// gradient with one global atomic per box pixel that received anything (a global atomic per tap
// otherwise).  The parameter gradient is summed per block in a fixed order into partial[slot].
// With the image gradient wanted, the parameter gradient's tap reads go to global memory (two
// 32 KiB arrays would halve the blocks per CU); without it the box is staged as in the forward.
template <bool GIMG, bool GPAR>
__global__ void __launch_bounds__(kDwThreads) k_dw_bwd(const float* __restrict__ img, const float* __restrict__ gout,
                                                       const CropMap* __restrict__ maps,
                                                       const TileDesc* __restrict__ tiles,
                                                       const int* __restrict__ prefix, int n, int w, int h, int vec4,
                                                       float* __restrict__ gimg, double* __restrict__ partial) {
    constexpr bool kStage = GPAR && !GIMG;
    __shared__ int accum[GIMG ? kDwLds : 1];
    __shared__ float stile[kStage ? kDwLds : 1];
    __shared__ double sRed[4][6];
    __shared__ float sMax[4];
    const int t = block_tile(prefix[n]);
    if (t < 0) return;
    const TileDesc& T = tiles[t];
    const int crop = T.crop;
    const CropMap& C = maps[crop];
    const bool empty = (T.flags & kTileEmpty) != 0;
    const size_t cbase = size_t(crop) * h * w;
    const int twm = (1 << C.tw_log2) - 1;
    float g[2];
    int xs[2], ys[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e = int(threadIdx.x) + k * kDwThreads;
        xs[k] = T.x0 + (e & twm);
        ys[k] = T.y0 + (e >> C.tw_log2);
        const bool in = e < C.px && xs[k] < w && ys[k] < h;
        if (!in) xs[k] = w;   // marks the slot unused
        g[k] = in ? gout[cbase + size_t(ys[k]) * w + xs[k]] : 0.0f;
    }
    // Integer LDS atomics run several times faster than float ones, so the box sums are kept
    // in int32 units of 1/S.  With m = max |g| over the tile and 2^k <= 1024 m < 2^(k+1),
    // S = 2^(37 - log2(P) - k) for a tile of P pixels: one output pixel adds at most
    // |g| (sum |wx| / |sum wx|) (sum |wy| / |sum wy|) < 4 |g| to a box pixel (clamped taps
    // included), so less than 4 m S < 2^(30 - log2 P) per pixel, and the sum over the tile's P
    // pixels stays below 2^30.  Rounding a contribution to 1/S costs at most 1/(2S) <=
    // 2^(log2(P) - 28) m (2^-19 m at P = 512, 2^-20 m at 256); a box pixel's error is at most
    // that times the number of the tile's pixels whose window holds it.
    // A tile whose m is not finite keeps float atomics (the box then holds floats); a tile whose
    // m is tiny keeps k at -96 so that S stays a finite float.
    float scale = 1.0f;
    bool fixed = false;
    if (GIMG) {
        float a = fmaxf(g[0] != g[0] ? INFINITY : fabsf(g[0]), g[1] != g[1] ? INFINITY : fabsf(g[1]));
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) a = fmaxf(a, __shfl_xor(a, off));
        if ((threadIdx.x & 63) == 0) sMax[threadIdx.x >> 6] = a;
        __syncthreads();
        const float m = fmaxf(fmaxf(sMax[0], sMax[1]), fmaxf(sMax[2], sMax[3]));
        fixed = isfinite(1024.0f * m);
        if (fixed && m > 0.0f) scale = ldexpf(1.0f, 37 - C.log2_px - max(ilogbf(1024.0f * m), -96));
    }
    const int bw = T.bx1 - T.bx0 + 1, bh = T.by1 - T.by0 + 1;
    const bool use_acc = GIMG && (T.flags & kTileAccum) != 0;
    if (use_acc)
        for (int e = threadIdx.x; e < bw * bh; e += kDwThreads) accum[e] = 0;
    const bool staged = kStage && (T.flags & kTileStaged) != 0;
    if (staged) stage_box(stile, img + cbase, w, T.ax0, T.by0, T.nc, bh, T.ls, vec4 != 0);
    if (use_acc || kStage) __syncthreads();
    double gp[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int x = xs[k], y = ys[k];
        if (empty || x >= w || g[k] == 0.0f) continue;
        const Sample S = sample_point(C, x, y, w, h);
        if (!S.valid) continue;
        const double fx0 = floor(S.px), fy0 = floor(S.py);
        const int ix = int(fx0), iy = int(fy0);
        float wx[8], wy[8], dwx[8], dwy[8], sx, sy, sdx = 0.0f, sdy = 0.0f;
        if (GPAR) {
            sx = lanczos4_weights_d(float(S.px - fx0), wx, dwx, &sdx);
            sy = lanczos4_weights_d(float(S.py - fy0), wy, dwy, &sdy);
        } else {
            sx = lanczos4_weights(float(S.px - fx0), wx);
            sy = lanczos4_weights(float(S.py - fy0), wy);
        }
        const float inv = __builtin_amdgcn_rcpf(sx * sy);
        int cols[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) cols[i] = clampi(ix - 3 + i, 0, w - 1);
        float v = 0.0f, vx = 0.0f, vy = 0.0f;
        const float gn = g[k] * inv;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int row = clampi(iy - 3 + j, 0, h - 1);
            if (GPAR) {
                // taps of a valid pixel lie inside the tile's box, so a staged copy serves them at
                // box-relative (non-negative) offsets; staged and global reads stay separate loops
                float r = 0.0f, rd = 0.0f;
                if (staged) {
                    const float* tr = stile + (row - T.by0) * T.ls;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const float a = tr[cols[i] - T.ax0];
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
                if (use_acc && fixed) {   // box-relative, non-negative offsets
                    int* ar = accum + (row - T.by0) * bw;
                    const float gs = gj * scale;
#pragma unroll
                    for (int i = 0; i < 8; ++i) atomicAdd(ar + (cols[i] - T.bx0), int(rintf(gs * wx[i])));
                } else if (use_acc) {
                    float* ar = reinterpret_cast<float*>(accum) + (row - T.by0) * bw;
#pragma unroll
                    for (int i = 0; i < 8; ++i) atomicAdd(ar + (cols[i] - T.bx0), gj * wx[i]);
                } else {
                    float* gr = gimg + cbase + size_t(row) * w;
#pragma unroll
                    for (int i = 0; i < 8; ++i) unsafeAtomicAdd(gr + cols[i], gj * wx[i]);
                }
            }
        }
        if (GPAR) {
            const double V = double(v) * inv;
            const double dVx = double(vx) * inv - V * double(sdx * __builtin_amdgcn_rcpf(sx));
            const double dVy = double(vy) * inv - V * double(sdy * __builtin_amdgcn_rcpf(sy));
            const double gd = g[k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double dpx = C.dm[q][0] * S.dx + C.dm[q][1] * S.dy;
                const double dpy = C.dm[q][2] * S.dx + C.dm[q][3] * S.dy;
                gp[q] += gd * (dVx * dpx + dVy * dpy);
            }
            // d(q - c - T)/dtx = (-1, 0), d/dty = (0, -1)
            gp[4] -= gd * (dVx * C.m[0] + dVy * C.m[2]);
            gp[5] -= gd * (dVx * C.m[1] + dVy * C.m[3]);
        }
    }
    if (use_acc) {
        __syncthreads();
        // one global atomic per box pixel that received a contribution
        const int n = bw * bh, q = kDwThreads / bw, rem = kDwThreads - q * bw;
        int e = threadIdx.x, r = e / bw, c = e - r * bw;
        float* gptr = gimg + cbase + size_t(T.by0 + r) * w + T.bx0 + c;
        const float inv_scale = 1.0f / scale;
        while (e < n) {
            const float a = fixed ? float(accum[e]) * inv_scale : __int_as_float(accum[e]);
            if (a != 0.0f) unsafeAtomicAdd(gptr, a);
            e += kDwThreads;
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
        partial[size_t(t) * 6 + k] = ((sRed[0][k] + sRed[1][k]) + sRed[2][k]) + sRed[3][k];
    }
}

// gparam[crop][k] = sum over the crop's tiles of partial[slot][k], in tile order.
__global__ void __launch_bounds__(256) k_dw_reduce(const double* __restrict__ partial, const int* __restrict__ prefix,
                                                   double* __restrict__ gparam) {
    __shared__ double s[256][6];
    const int crop = blockIdx.x;
    const int t0 = prefix[crop], tiles = prefix[crop + 1] - t0;
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int t = threadIdx.x; t < tiles; t += 256)
#pragma unroll
        for (int k = 0; k < 6; ++k) a[k] += partial[(size_t(t0) + t) * 6 + k];
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

// Block slots per crop: the most tiles any candidate shape needs.
int dw_slots(int w, int h) {
    int best = 0;
    for (int pi = 0; pi < 3; ++pi)
        for (int k = 1; k <= kDwLog2Max && (1 << k) < kDwPixels[pi]; ++k)
            best = std::max(best, tile_count(w, h, k, kDwPixels[pi] >> k, nullptr));
    return best;
}

// Separable Gaussian of fp32 crops (the coarse-to-fine smoothing of the photometric refinement):
// taps exp(-k^2 / 2 sigma^2), |k| <= max(1, ceil(3 sigma)), normalised; edge pixels replicated.
constexpr int kCropBlurMaxTaps = 97;     // sigma up to 16
struct CropTaps {
    float w[kCropBlurMaxTaps];
    int r;
};

template <bool ROWS>
__global__ void __launch_bounds__(256) k_crop_blur(const float* __restrict__ in, int h, int w, CropTaps t,
                                                   float* __restrict__ out) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, c = blockIdx.z;
    if (x >= w) return;
    const float* base = in + size_t(c) * h * w;
    float acc = 0.0f;
    for (int k = -t.r; k <= t.r; ++k) {
        const float v = ROWS ? base[size_t(y) * w + min(max(x + k, 0), w - 1)]
                             : base[size_t(min(max(y + k, 0), h - 1)) * w + x];
        acc = fmaf(t.w[k + t.r], v, acc);
    }
    out[(size_t(c) * h + y) * w + x] = acc;
}

struct DwGeom {
    int slots;
    long long slot_total;
    bool vec4;
};

xa_status dw_check(const float* img, int32_t n, int32_t h, int32_t w, const xa_affine_params* params, DwGeom* g) {
    if (n < 1 || h < 1 || w < 1) return fail(XA_EINVAL, "need n, h, w >= 1");
    if ((long long)h * w > (1LL << 28) || (long long)n * h * w > (1LL << 38))
        return fail(XA_EUNSUPPORTED, "crops too large");
    if (!img || !params) return fail(XA_EINVAL, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(img) % 4 || reinterpret_cast<uintptr_t>(params) % 8)
        return fail(XA_EINVAL, "misaligned image or parameter buffer");
    g->slots = dw_slots(w, h);
    g->slot_total = (long long)g->slots * n;
    if (g->slot_total > INT32_MAX - kXcds) return fail(XA_EUNSUPPORTED, "too many tiles for one launch");
    g->vec4 = w % 4 == 0 && reinterpret_cast<uintptr_t>(img) % 16 == 0;
    return XA_OK;
}

xa_status dw_ws_check(void* d_ws, size_t ws_bytes, size_t need, const char* what) {
    if (ws_bytes < need) return fail(XA_ECAPACITY, "%s needs %zu bytes of workspace, got %zu", what, need, ws_bytes);
    if (!d_ws || reinterpret_cast<uintptr_t>(d_ws) % 16) return fail(XA_EINVAL, "workspace NULL or misaligned");
    return XA_OK;
}

// Workspace: maps [n], prefix [n + 1], tile descriptors [n x slots] (an upper bound on the
// tiles), then (adjoint) per-tile parameter partial sums [n x slots][6].
struct DwWs {
    CropMap* maps;
    int* prefix;
    TileDesc* tiles;
    double* partial;
};
size_t ws_prologue_bytes(int32_t n, int slots) {
    return align_up(size_t(n) * sizeof(CropMap)) + align_up(size_t(n + 1) * sizeof(int)) +
           align_up(size_t(n) * size_t(slots) * sizeof(TileDesc));
}
DwWs carve(void* ws, int32_t n, int slots) {
    char* p = static_cast<char*>(ws);
    DwWs W;
    W.maps = reinterpret_cast<CropMap*>(p);
    p += align_up(size_t(n) * sizeof(CropMap));
    W.prefix = reinterpret_cast<int*>(p);
    p += align_up(size_t(n + 1) * sizeof(int));
    W.tiles = reinterpret_cast<TileDesc*>(p);
    p += align_up(size_t(n) * size_t(slots) * sizeof(TileDesc));
    W.partial = reinterpret_cast<double*>(p);
    return W;
}

void enqueue_prologue(const xa_affine_params* d_params, int32_t n, int32_t h, int32_t w, const DwGeom& g,
                      const DwWs& W, hipStream_t stream) {
    hipLaunchKernelGGL(k_dw_maps, dim3(unsigned((n + 63) / 64)), dim3(64), 0, stream, d_params, n, w, h, W.maps);
    hipLaunchKernelGGL(k_dw_scan, dim3(1), dim3(256), 0, stream, W.maps, n, W.prefix);
    hipLaunchKernelGGL(k_dw_tiles, dim3(unsigned((g.slot_total + 255) / 256)), dim3(256), 0, stream, W.maps,
                       W.prefix, n, w, h, g.slots, int(g.vec4), W.tiles);
}


}  // namespace
}  // namespace xa

using namespace xa;

extern "C" size_t xa_warp_f32_fwd_workspace_size(int32_t n, int32_t h, int32_t w) {
    if (n < 1 || h < 1 || w < 1) return 0;
    return ws_prologue_bytes(n, dw_slots(w, h));
}

extern "C" xa_status xa_warp_f32_fwd(const float* d_img, int32_t n, int32_t h, int32_t w,
                                     const xa_affine_params* d_params, float* d_out, uint8_t* d_mask, void* d_ws,
                                     size_t ws_bytes, hipStream_t stream) {
    DwGeom g;
    xa_status s = dw_check(d_img, n, h, w, d_params, &g);
    if (s != XA_OK) return s;
    if (!d_out) return fail(XA_EINVAL, "NULL output");
    if (reinterpret_cast<uintptr_t>(d_out) % 4) return fail(XA_EINVAL, "misaligned output");
    s = dw_ws_check(d_ws, ws_bytes, xa_warp_f32_fwd_workspace_size(n, h, w), "warp forward");
    if (s != XA_OK) return s;
    const unsigned grid = unsigned((g.slot_total + kXcds - 1) / kXcds * kXcds);
    const DwWs W = carve(d_ws, n, g.slots);
    enqueue_prologue(d_params, n, h, w, g, W, stream);
    hipLaunchKernelGGL(k_dw_fwd, dim3(grid), dim3(kDwThreads), 0, stream, d_img, W.maps, W.tiles, W.prefix, n, w, h,
                       int(g.vec4), d_out, d_mask);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "warp forward launch");
}

extern "C" size_t xa_warp_f32_bwd_workspace_size(int32_t n, int32_t h, int32_t w) {
    if (n < 1 || h < 1 || w < 1) return 0;
    const int slots = dw_slots(w, h);
    return ws_prologue_bytes(n, slots) + align_up(size_t(slots) * size_t(n) * 6 * sizeof(double));
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
    s = dw_ws_check(d_ws, ws_bytes, xa_warp_f32_bwd_workspace_size(n, h, w), "warp backward");
    if (s != XA_OK) return s;
    const unsigned grid = unsigned((g.slot_total + kXcds - 1) / kXcds * kXcds);
    const DwWs W = carve(d_ws, n, g.slots);
    enqueue_prologue(d_params, n, h, w, g, W, stream);
    if (d_gimg) {
        const size_t total = size_t(n) * h * w;
        const unsigned fb = unsigned(std::min<size_t>((total + 255) / 256, 65536));
        hipLaunchKernelGGL(k_dw_fill, dim3(fb), dim3(256), 0, stream, d_gimg, total);
    }
    const int v4 = int(g.vec4);
    if (d_gimg && d_gparams)
        hipLaunchKernelGGL((k_dw_bwd<true, true>), dim3(grid), dim3(kDwThreads), 0, stream, d_img, d_gout, W.maps,
                           W.tiles, W.prefix, n, w, h, v4, d_gimg, W.partial);
    else if (d_gimg)
        hipLaunchKernelGGL((k_dw_bwd<true, false>), dim3(grid), dim3(kDwThreads), 0, stream, d_img, d_gout, W.maps,
                           W.tiles, W.prefix, n, w, h, v4, d_gimg, W.partial);
    else
        hipLaunchKernelGGL((k_dw_bwd<false, true>), dim3(grid), dim3(kDwThreads), 0, stream, d_img, d_gout, W.maps,
                           W.tiles, W.prefix, n, w, h, v4, d_gimg, W.partial);
    if (d_gparams)
        hipLaunchKernelGGL(k_dw_reduce, dim3(unsigned(n)), dim3(256), 0, stream, W.partial, W.prefix, d_gparams);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "warp backward launch");
}

extern "C" size_t xa_blur_f32_workspace_size(int32_t n, int32_t h, int32_t w) {
    if (n < 1 || h < 1 || w < 1) return 0;
    return align_up(size_t(n) * h * w * sizeof(float));
}

extern "C" xa_status xa_blur_f32(const float* d_in, int32_t n, int32_t h, int32_t w, double sigma, float* d_out,
                                 void* d_ws, size_t ws_bytes, hipStream_t stream) {
    if (n < 1 || h < 1 || w < 1 || n > 65535 || h > 65535 || (long long)n * h * w > (1LL << 34))
        return fail(XA_EINVAL, "need 1 <= n, h <= 65535, w >= 1 and at most 2^34 values");
    if (!(sigma > 0.0) || !(sigma <= 16.0)) return fail(XA_EINVAL, "sigma must lie in (0, 16]");
    if (!d_in || !d_out) return fail(XA_EINVAL, "NULL pointer");
    const size_t need = xa_blur_f32_workspace_size(n, h, w);
    if (!d_ws || ws_bytes < need || reinterpret_cast<uintptr_t>(d_ws) % 4)
        return fail(XA_EINVAL, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    CropTaps t;
    t.r = std::max(1, int(std::ceil(3.0 * sigma)));
    double sum = 0.0;
    double raw[kCropBlurMaxTaps];
    for (int k = -t.r; k <= t.r; ++k) sum += (raw[k + t.r] = std::exp(-double(k) * k / (2.0 * sigma * sigma)));
    for (int k = 0; k <= 2 * t.r; ++k) t.w[k] = float(raw[k] / sum);
    const dim3 grid(unsigned((w + 255) / 256), unsigned(h), unsigned(n));
    float* tmp = static_cast<float*>(d_ws);
    hipLaunchKernelGGL(k_crop_blur<true>, grid, dim3(256), 0, stream, d_in, h, w, t, tmp);
    hipLaunchKernelGGL(k_crop_blur<false>, grid, dim3(256), 0, stream, tmp, h, w, t, d_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "crop blur launch");
}
