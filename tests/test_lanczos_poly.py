"""The polynomial Lanczos-4 tap weights of the warp and scale kernels (csrc/lanczos.h), evaluated
as the kernels do (fp32 Horner), against the oracle's closed form of eq. (4); and the header's
table against its generator."""
import os
import re

import numpy as np

from oracle.simulate import lanczos4

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2503_03479_amd", "csrc")


def _header_tables():
    text = open(os.path.join(CSRC, "lanczos.h")).read()
    out = {}
    for name in ("kLanczosEven", "kLanczosOdd"):
        body = re.search(name + r"\[4\]\[5\] = \{(.*?)\};", text, re.S).group(1)
        out[name] = np.array([float(v) for v in re.findall(r"([-+0-9.e]+)f", body)], np.float32).reshape(4, 5)
    return out["kLanczosEven"], out["kLanczosOdd"]


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
