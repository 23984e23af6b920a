// Tap weights of the Lanczos-4 kernel of eq. (4) over the 8-tap window of eq. (3), shared by the
// view warp and the scale stage.
#pragma once

#include <hip/hip_runtime.h>

namespace xa {

// Weights proportional to L4(i - f), i = -3..4, for the fractional offset f in [0, 1]; returns
// their sum, by which the caller divides (the proportionality factor is the same for all 8 and
// positive).
//
// Only ratios matter, so two factors common to all taps drop out:
//  - sin(pi (i - f)) = (-1)^(i+1) sin(pi f), and 4 / pi^2, leaving
//    L4(i - f) ~ (-1)^(i+1) sin(pi (i - f) / 4) / (i - f)^2;
//  - multiplying all 8 by D = prod_j (j - f)^2 turns the 8 reciprocals into products:
//    w_i = (-1)^(i+1) sin(pi (i - f) / 4) prod_{j != i} (j - f)^2, formed from prefix and
//    suffix products of the squared distances (26 multiplies instead of 8 quarter-rate
//    reciprocals).
// The numerators come from C = cos(pi f / 4) and S = sin(pi f / 4) by the angle-difference
// formula, except at i = 1, whose factor sin(pi (1 - f) / 4) is evaluated directly: it vanishes as
// f -> 1, where the difference h (C - S) would cancel to noise, and near there its tap must
// dominate.  Both poles (i = 0 at f -> 0, i = 1 at f -> 1) then have accurate numerators.  The
// magnitudes stay in range: every squared distance is at most 16, so no product exceeds 16^7.
// f at most 2^-40 (the neighbouring weights are below 1e-11) and f == 1 (an fp64 fraction within
// 2^-25 of 1, rounded to fp32) give the one-hot limits at i = 0 and i = 1.
//
// The hardware sine and cosine take revolutions (sin(pi x / 4) = sin(2 pi (x / 8))); their
// absolute error, ~1e-6, moves an 8-bit intensity by far less than its rounding step.
__device__ __forceinline__ float lanczos4_weights(float f, float w[8]) {
    if (f <= 0x1p-40f || f >= 1.0f) {
        const int hot = f >= 1.0f ? 4 : 3;
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = (i == hot) ? 1.0f : 0.0f;
        return 1.0f;
    }
    constexpr float h = 0.70710678118654752440f;                  // sin(pi / 4) = cos(pi / 4)
    const float S = __builtin_amdgcn_sinf(0.125f * f);
    const float C = __builtin_amdgcn_cosf(0.125f * f);
    const float S1 = __builtin_amdgcn_sinf(0.125f - 0.125f * f); // sin(pi (1 - f) / 4)
    const float hs = h * S, hc = h * C;
    // (-1)^(i+1) sin(pi (i - f) / 4) for i = -3..4
    const float g[8] = {hs - hc, C, -(hc + hs), S, S1, -C, hc + hs, -S};
    float d[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const float x = float(t - 3) - f;
        d[t] = x * x;
    }
    float pre[8], suf[8];                    // pre[t] = prod_{j < t} d_j, suf[t] = prod_{j > t} d_j
    pre[1] = d[0];
    suf[6] = d[7];
#pragma unroll
    for (int t = 2; t < 8; ++t) pre[t] = pre[t - 1] * d[t - 1];
#pragma unroll
    for (int t = 5; t >= 0; --t) suf[t] = suf[t + 1] * d[t + 1];
    float sum = 0.0f;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const float q = t == 0 ? suf[0] : (t == 7 ? pre[7] : pre[t] * suf[t]);
        w[t] = g[t] * q;
        sum += w[t];
    }
    return sum;
}

}  // namespace xa
