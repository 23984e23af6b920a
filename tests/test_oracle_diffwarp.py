"""Pins of the differentiable-warp oracle: identity, integer shifts, the kernel
derivative against central differences of np.sinc, the dot-product test of the
image adjoint, and the parameter gradient against central finite differences."""
import math

import numpy as np
import pytest

import synth
from oracle import diffwarp as D


def _crop(seed=5000, n=48):
    g = synth.rng(seed)
    img = g.random((n, n + 6))
    # smooth a little so that finite differences see a well-behaved function
    k = np.array([1, 4, 6, 4, 1], np.float64) / 16
    for ax in (0, 1):
        img = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), ax, img)
    return img


def test_identity_is_exact():
    img = _crop()
    V, mask = D.warp_forward(img, (1.0, 0.0, 0.0, 1.0, 0.0, 0.0))
    assert mask.all()
    assert np.max(np.abs(V - img)) < 1e-12


def test_integer_translation_shifts_the_image():
    img = _crop()
    V, mask = D.warp_forward(img, (1.0, 0.0, 0.0, 1.0, 3.0, -2.0))
    # view pixel q samples p = q - T: V[y, x] = img[y + 2, x - 3]
    assert np.max(np.abs(V[:-2, 3:] - img[2:, :-3])) < 1e-12
    assert not mask[:, :3].any() and not mask[-2:, :].any()


def test_quarter_turn_is_a_rotation():
    img = _crop(n=40)[:, :40]
    V, mask = D.warp_forward(img, (1.0, 0.0, math.pi / 2, 1.0, 0.0, 0.0))
    assert mask.all()
    # L = R(90 deg): q - c = R (p - c), so p = R^-1 (q - c) + c; on a square crop this is np.rot90
    assert np.max(np.abs(V - np.rot90(img, k=1))) < 1e-9 or np.max(np.abs(V - np.rot90(img, k=-1))) < 1e-9


def test_kernel_derivative_matches_central_differences():
    x = np.concatenate([np.linspace(-3.99, 3.99, 801), [0.0, 1e-6, -3e-5, 2e-4, 0.5, 1.0, -2.0]])
    h = 1e-6
    num = (D.lanczos4(x + h) - D.lanczos4(x - h)) / (2 * h)
    assert np.max(np.abs(D.lanczos4_deriv(x) - num)) < 1e-8
    assert D.lanczos4_deriv(np.array([0.0]))[0] == 0.0


def test_image_adjoint_dot_product():
    g = synth.rng(7)
    img = _crop()
    params = (1.7, 0.6, -0.4, 0.8, 1.3, -2.2)
    y = g.standard_normal(img.shape)
    Ax, _ = D.warp_forward(img, params)
    gimg, _ = D.warp_adjoint(np.zeros_like(img), y, params)
    lhs = float(np.sum(Ax * y))
    rhs = float(np.sum(img * gimg))
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))


def _fd_check(img, target, params, h, tol):
    base = np.array(params, np.float64)
    # the loss on a fixed set of pixels (valid at the base point and at every probe),
    # so that finite differences do not see the mask move
    masks = [D.warp_forward(img, base)[1]]
    for k in range(6):
        for sgn in (-1, 1):
            p = base.copy()
            p[k] += sgn * h
            masks.append(D.warp_forward(img, p)[1])
    keep = np.logical_and.reduce(masks)

    def loss(p):
        V, _ = D.warp_forward(img, p)
        r = np.where(keep, V - target, 0.0)
        return 0.5 * np.sum(r * r)

    V, _ = D.warp_forward(img, base)
    _, gp = D.warp_adjoint(img, np.where(keep, V - target, 0.0), base)
    floor = 1e-3 * np.abs(gp).max()
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        fd = (loss(base + e) - loss(base - e)) / (2 * h)
        assert abs(gp[k] - fd) <= tol * max(abs(fd), floor), (D.PARAM_NAMES[k], h, gp[k], fd)


PARAMS = [(1.7, 0.6, -0.4, 0.8, 1.3, -2.2), (3.2, 2.5, 1.1, 0.55, -4.0, 0.7), (1.05, 0.1, 0.0, 1.0, 0.25, 0.0)]


@pytest.mark.parametrize("params", PARAMS)
def test_parameter_gradient_converges_to_finite_differences(params):
    """On a rough crop the O(h^2) error of central differences is visible at h = 1e-3;
    at h = 1e-5 it is below 1e-6 of the gradient."""
    _fd_check(_crop(), _crop(seed=5001), params, 1e-5, 1e-6)


@pytest.mark.parametrize("params", PARAMS)
def test_parameter_gradient_at_h_1e_3(params):
    """Central differences with h = 1e-3 on a smooth crop agree within 1e-3."""
    img, target = _crop(), _crop(seed=5001)
    k = np.array([1, 4, 6, 4, 1], np.float64) / 16
    for _ in range(12):
        for ax in (0, 1):
            img = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), ax, img)
            target = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), ax, target)
    _fd_check(img, target, params, 1e-3, 1e-3)


def test_image_gradient_matches_finite_differences():
    img = _crop(n=24)
    target = _crop(seed=5002, n=24)
    params = (1.9, 0.7, 0.3, 0.9, 0.4, -0.6)
    loss, gimg, _ = D.l2_loss_and_grads(img, target, params)
    g = synth.rng(3)
    for _ in range(6):
        y, x = int(g.integers(0, img.shape[0])), int(g.integers(0, img.shape[1]))
        e = np.zeros_like(img)
        e[y, x] = 1e-3
        fd = (D.l2_loss_and_grads(img + e, target, params)[0] - D.l2_loss_and_grads(img - e, target, params)[0]) / 2e-3
        assert abs(gimg[y, x] - fd) < 1e-7 + 1e-6 * abs(fd)
