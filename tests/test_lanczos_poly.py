"""The polynomial Lanczos-4 tap weights of the warp and scale kernels (csrc/lanczos.h), evaluated
as the kernels do (fp32 Horner), against the oracle's closed form of eq. (4); and the header's
table against its generator."""
import os
import re

import numpy as np

from oracle.simulate import lanczos4

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2503_03479_amd", "csrc")


def _header_table(name):
    text = open(os.path.join(CSRC, "lanczos.h")).read()
    body = re.search(name + r"\[4\]\[5\] = \{(.*?)\};", text, re.S).group(1)
    return np.array([float(v) for v in re.findall(r"([-+0-9.e]+)f", body)], np.float32).reshape(4, 5)


def _header_tables():
    return _header_table("kLanczosEven"), _header_table("kLanczosOdd")


def _horner32(C, h):
    """sum_k C[k] h^k by Horner's rule in fp32 with single-rounding fmaf (emulated in fp64)."""
    v = np.full(h.shape, C[4], np.float32)
    for k in range(3, -1, -1):
        v = (v.astype(np.float64) * h + np.float64(C[k])).astype(np.float32)
    return v


def _derivs_fp32(f, A, B):
    """The derivative half of lanczos4_weights_d step by step in fp32."""
    f = np.asarray(f, np.float32)
    g = (f - np.float32(0.5)).astype(np.float32)
    h = (g * g).astype(np.float32)
    dw = np.zeros(f.shape + (8,), np.float32)
    ds = np.zeros(f.shape, np.float32)
    for p in range(4):
        a = (_horner32(A[p], h) * g).astype(np.float32)
        b = _horner32(B[p], h)
        dw[..., p] = a + b
        dw[..., 7 - p] = a - b
        ds = (ds + a).astype(np.float32)
    return dw, np.float32(2) * ds


def _weights_fp32(f, E, O):
    """lanczos4_weights step by step in fp32 (fmaf rounds once: emulated in fp64, then rounded)."""
    f = np.asarray(f, np.float32)
    g = (f - np.float32(0.5)).astype(np.float32)
    h = (g * g).astype(np.float32)
    w = np.zeros(f.shape + (8,), np.float32)
    s = np.zeros(f.shape, np.float32)
    for p in range(4):
        e = np.full(f.shape, E[p, 4], np.float32)
        o = np.full(f.shape, O[p, 4], np.float32)
        for k in range(3, -1, -1):
            e = (e.astype(np.float64) * h + np.float64(E[p, k])).astype(np.float32)
            o = (o.astype(np.float64) * h + np.float64(O[p, k])).astype(np.float32)
        o = (o * g).astype(np.float32)
        w[..., p] = e + o
        w[..., 7 - p] = e - o
        s = (s + e).astype(np.float32)
    return w, np.float32(2) * s


def test_polynomial_weights_match_the_kernel_definition():
    E, O = _header_tables()
    f = np.concatenate([np.linspace(0, 1, 100001), [0.0, 1.0, 2.0 ** -30, 1 - 2.0 ** -24]]).astype(np.float32)
    w, s = _weights_fp32(f, E, O)
    ref = lanczos4(np.arange(-3, 5)[None, :] - f.astype(np.float64)[:, None])
    assert np.abs(w - ref).max() < 2e-7
    assert np.abs(s - ref.sum(axis=1)).max() < 1e-6
    # one-hot limits: f = 0 and f = 1 select the tap at the integer coordinate to rounding level
    assert abs(w[-4 + 0, 3] - 1) < 2e-7 and np.abs(np.delete(w[-4], 3)).max() < 2e-7
    assert abs(w[-3, 4] - 1) < 2e-7 and np.abs(np.delete(w[-3], 4)).max() < 2e-7
    # symmetry: w_i(f) = w_{7-i}(1 - f)
    w2, _ = _weights_fp32(np.float32(1) - f[:100001], E, O)
    assert np.abs(w[:100001] - w2[:, ::-1]).max() < 2e-7


def test_header_table_is_the_generator_output():
    import importlib.util
    spec = importlib.util.spec_from_file_location("gen", os.path.join(CSRC, "gen_lanczos_poly.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    E, O = _header_tables()
    GE, GO = gen.coefficients()
    assert np.array_equal(E, GE) and np.array_equal(O, GO)


def test_derivative_weights_match_the_derivative_of_eq4():
    """d L4(i - f) / df = -L4'(i - f) from the oracle's closed-form derivative (the adjoint's
    weights), checked over [0, 1] in the kernel's fp32 evaluation; the sum of the derivatives is
    the derivative of the sum; at f = 0 the closed form gives -L4'(i) = -(-1)^i sinc(i / 4) / i
    for i != 0 and 0 for i = 0; the centred differences of the value polynomials agree."""
    from oracle.diffwarp import lanczos4_deriv
    A, B = _header_table("kLanczosDerivOdd"), _header_table("kLanczosDerivEven")
    f = np.concatenate([np.linspace(0, 1, 100001), [2.0 ** -30, 1 - 2.0 ** -24]]).astype(np.float32)
    dw, ds = _derivs_fp32(f, A, B)
    ref = -lanczos4_deriv(np.arange(-3, 5)[None, :] - f.astype(np.float64)[:, None])
    assert np.abs(dw - ref).max() < 5e-7
    assert np.abs(ds - ref.sum(axis=1)).max() < 2e-6
    d0, _ = _derivs_fp32(np.zeros(1, np.float32), A, B)
    i = np.arange(-3, 5)
    closed = np.where(i == 0, 0.0, -((-1.0) ** i) * np.sinc(i / 4.0) / np.where(i == 0, 1, i))
    assert np.abs(d0[0] - closed).max() < 5e-7
    # the value polynomials' centred differences (fp64 evaluation of the fp32 tables)
    E, O = _header_tables()
    fm = np.linspace(0.01, 0.99, 99)
    hstep = 1e-5

    def w64(ff):
        g = ff - 0.5
        hh = g * g
        out = np.zeros(ff.shape + (8,))
        for p in range(4):
            e = sum(float(E[p, k]) * hh ** k for k in range(5))
            o = g * sum(float(O[p, k]) * hh ** k for k in range(5))
            out[..., p], out[..., 7 - p] = e + o, e - o
        return out
    fd = (w64(fm + hstep) - w64(fm - hstep)) / (2 * hstep)
    dwm, _ = _derivs_fp32(fm.astype(np.float32), A, B)
    assert np.abs(dwm - fd).max() < 5e-6
    # symmetry: dw_i/df(f) = -dw_{7-i}/df(1 - f)
    dw2, _ = _derivs_fp32(np.float32(1) - f[:100001], A, B)
    assert np.abs(dw[:100001] + dw2[:, ::-1]).max() < 5e-7


def test_derivative_tables_are_the_generator_output():
    import importlib.util
    spec = importlib.util.spec_from_file_location("gen", os.path.join(CSRC, "gen_lanczos_poly.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    GA, GB = gen.derivative_coefficients()
    assert np.array_equal(_header_table("kLanczosDerivOdd"), GA)
    assert np.array_equal(_header_table("kLanczosDerivEven"), GB)
