// Tap weights of the Lanczos-4 kernel of eq. (4) over the 8-tap window of eq. (3), shared by the
// view warp, the scale stage and the differentiable warp (with their derivatives).
#pragma once

#include <hip/hip_runtime.h>

namespace xa {

// With g = f - 1/2, taps p and 7 - p (p = 0..3) of the window weigh L4(p - 7/2 -+ g), whose even
// and odd parts in g are E_p(h) = sum_k kLanczosEven[p][k] h^k and O_p = g sum_k kLanczosOdd[p][k]
// h^k, h = g^2.  L4 is entire, so these degree-4 least-squares fits hold to 1.4e-7 in fp32 over
// the whole of 0 <= f <= 1 (fp32 rounding of weights near 1), one-hot limits at f = 0 and 1
// included; gen_lanczos_poly.py prints this table.
constexpr float kLanczosEven[4][5] = {
    {-1.266088057e-02f, 4.956583306e-02f, 1.182281319e-02f, -3.285482526e-02f, 1.122928970e-02f},
    {5.990948528e-02f, -2.697711289e-01f, 1.186428145e-01f, 9.818997234e-03f, -9.039720520e-03f},
    {-1.664152294e-01f, 7.228511572e-01f, -2.318021953e-01f, 1.084158383e-02f, 5.296494346e-03f},
    {6.203830242e-01f, -5.134930015e-01f, 1.300900429e-01f, -8.574611507e-03f, -1.643885276e-03f},
};
constexpr float kLanczosOdd[4][5] = {
    {3.124131449e-02f, -1.518085748e-01f, 1.153091788e-01f, -3.287798539e-02f, 4.537742585e-03f},
    {-6.741748750e-02f, 3.247852325e-01f, -2.359036207e-01f, 6.402381510e-02f, -9.015359916e-03f},
    {1.677483320e-01f, -7.656255960e-01f, 4.019368887e-01f, -9.694371372e-02f, 1.325049903e-02f},
    {-1.305212140e+00f, 1.348976851e+00f, -5.413594842e-01f, 1.193514392e-01f, -1.587783545e-02f},
};

// Derivatives of the tap weights in f (the adjoint of the differentiable warp): with g and h as
// above, dw_p/df = g A_p(h) + B_p(h) and dw_{7-p}/df = g A_p(h) - B_p(h), A_p from
// kLanczosDerivOdd and B_p from kLanczosDerivEven, degree-4 least-squares fits within 1e-7 of
// -L4'(i - f); gen_lanczos_poly.py prints these tables too.
constexpr float kLanczosDerivOdd[4][5] = {
    {9.913045913e-02f, 4.737459496e-02f, -1.986290663e-01f, 9.954920411e-02f, -2.050872333e-02f},
    {-5.395411253e-01f, 4.744940400e-01f, 6.030366197e-02f, -8.131737262e-02f, 1.899872907e-02f},
    {1.445701480e+00f, -9.271550179e-01f, 6.408178061e-02f, 4.863896221e-02f, -1.323004533e-02f},
    {-1.026985645e+00f, 5.203410387e-01f, -5.110301077e-02f, -1.538309455e-02f, 4.711917136e-03f},
};
constexpr float kLanczosDerivEven[4][5] = {
    {3.124131076e-02f, -4.554252326e-01f, 5.765330791e-01f, -2.300434113e-01f, 4.059078544e-02f},
    {-6.741748005e-02f, 9.743545651e-01f, -1.179489970e+00f, 4.479415715e-01f, -8.059152216e-02f},
    {1.677483320e-01f, -2.296875238e+00f, 2.009642363e+00f, -6.782695651e-01f, 1.184374467e-01f},
    {-1.305212021e+00f, 4.046928406e+00f, -2.706747055e+00f, 8.350570202e-01f, -1.419217438e-01f},
};

// Weights L4(i - f), i = -3..4, for the fractional offset f in [0, 1] (w[i + 3]); returns their
// sum, by which the caller divides.  Per tap pair: two degree-4 Horner chains in h, one multiply
// by g, a sum and a difference; the sum of all 8 is twice the sum of the even parts.  No
// transcendental, reciprocal or branch.
__device__ __forceinline__ float lanczos4_weights(float f, float w[8]) {
    const float g = f - 0.5f, h = g * g;
    float s = 0.0f;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        float e = kLanczosEven[p][4], o = kLanczosOdd[p][4];
#pragma unroll
        for (int k = 3; k >= 0; --k) {
            e = fmaf(e, h, kLanczosEven[p][k]);
            o = fmaf(o, h, kLanczosOdd[p][k]);
        }
        o *= g;
        w[p] = e + o;
        w[7 - p] = e - o;
        s += e;
    }
    return 2.0f * s;
}

// Weights (as lanczos4_weights) and their derivatives dw[i + 3] = d L4(i - f) / df; returns the
// weights' sum and puts the derivatives' sum in *dsum.  Per tap pair four Horner chains.
__device__ __forceinline__ float lanczos4_weights_d(float f, float w[8], float dw[8], float* dsum) {
    const float g = f - 0.5f, h = g * g;
    float s = 0.0f, ds = 0.0f;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        float e = kLanczosEven[p][4], o = kLanczosOdd[p][4];
        float a = kLanczosDerivOdd[p][4], b = kLanczosDerivEven[p][4];
#pragma unroll
        for (int k = 3; k >= 0; --k) {
            e = fmaf(e, h, kLanczosEven[p][k]);
            o = fmaf(o, h, kLanczosOdd[p][k]);
            a = fmaf(a, h, kLanczosDerivOdd[p][k]);
            b = fmaf(b, h, kLanczosDerivEven[p][k]);
        }
        o *= g;
        a *= g;
        w[p] = e + o;
        w[7 - p] = e - o;
        dw[p] = a + b;
        dw[7 - p] = a - b;
        s += e;
        ds += a;
    }
    *dsum = 2.0f * ds;
    return 2.0f * s;
}

}  // namespace xa
