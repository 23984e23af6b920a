"""Coefficients of the polynomial Lanczos-4 tap weights in lanczos.h.

Over the fractional offset f in [0, 1], the taps i = -3..4 of the 8-tap window weigh
L4(i - f) with L4(x) = sinc(x) sinc(x / 4) (eq. (4), a = 4).  With g = f - 1/2, tap p (0-based,
p = 0..3) and its mirror 7 - p see L4(p - 7/2 - g) and L4(p - 7/2 + g) (L4 is even), so the pair
is E_p(g) +- O_p(g) with E_p even and O_p odd in g.  L4 is entire, so on |g| <= 1/2 low-degree
fits converge fast: E_p(g) = sum_k e_pk h^k and O_p(g) = g sum_k o_pk h^k in h = g^2, degree 4
each, fitted by least squares on a dense grid.  Evaluated in fp32 by Horner's rule they stay
within 1.4e-7 of L4, the rounding level of fp32 weights near 1.

The adjoint of the warp also needs the weights' derivatives in f (= d/dg).  For the tap pair the
derivative splits the same way: dw_p/dg = A_p(g) + B_p(g) and dw_{7-p}/dg = A_p(g) - B_p(g), with
A_p = g sum_k a_pk h^k odd and B_p = sum_k b_pk h^k even, fitted by least squares to the exact
derivative -L4'(p - 7/2 -+ g); degree 4 keeps them within 1e-7 of it.

Run as a script to print the tables that lanczos.h holds."""
import numpy as np

DEGREE = 4


def lanczos4(x):
    x = np.asarray(x, np.float64)
    return np.where(np.abs(x) < 4.0, np.sinc(x) * np.sinc(x / 4.0), 0.0)


def sinc_deriv(x):
    """d/dx sin(pi x) / (pi x) = (cos(pi x) - sinc(x)) / x, and its series -pi^2 x / 3 near 0."""
    x = np.asarray(x, np.float64)
    small = np.abs(x) < 1e-4
    xs = np.where(small, 1.0, x)
    return np.where(small, -(np.pi ** 2 / 3.0) * x, (np.cos(np.pi * xs) - np.sinc(xs)) / xs)


def lanczos4_deriv(x):
    x = np.asarray(x, np.float64)
    d = sinc_deriv(x) * np.sinc(x / 4.0) + np.sinc(x) * sinc_deriv(x / 4.0) / 4.0
    return np.where(np.abs(x) < 4.0, d, 0.0)


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


def derivative_coefficients(degree=DEGREE, n=40001):
    """(A, B): dw_p/dg = g A_p(h) + B_p(h) and dw_{7-p}/dg = g A_p(h) - B_p(h), p = 0..3."""
    g = np.linspace(0.0, 0.5, n)
    h = g * g
    even = np.vander(h, degree + 1, increasing=True)
    odd = g[:, None] * even
    A, B = [], []
    for p in range(4):
        d, dm = -lanczos4_deriv(p - 3.5 - g), -lanczos4_deriv(3.5 - p - g)
        A.append(np.linalg.lstsq(odd, 0.5 * (d + dm), rcond=None)[0])
        B.append(np.linalg.lstsq(even, 0.5 * (d - dm), rcond=None)[0])
    return np.array(A, np.float32), np.array(B, np.float32)


def table():
    E, O = coefficients()
    A, B = derivative_coefficients()
    rows = []
    for name, M in (("kLanczosEven", E), ("kLanczosOdd", O), ("kLanczosDerivOdd", A), ("kLanczosDerivEven", B)):
        rows.append(f"constexpr float {name}[4][{M.shape[1]}] = {{")
        for r in M:
            rows.append("    {" + ", ".join(f"{float(c):.9e}f" for c in r) + "},")
        rows.append("};")
    return "\n".join(rows)


if __name__ == "__main__":
    print(table())
