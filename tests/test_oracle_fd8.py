"""Pins of the oracle's eighth-order finite-difference first derivatives
(Section 3.2, the FD kernel): exact modified wavenumbers on Fourier modes,
eighth-order convergence, summation by parts between gradient and divergence,
agreement with the spectral derivative on band-limited fields, and the reduced
gradient at v = 0 in closed form with the FD8 derivative."""
import numpy as np

import oracle
import synth

from conftest import rel_l2

C = np.array([4 / 5, -1 / 5, 4 / 105, -1 / 280])


def _grid(shape):
    return np.meshgrid(*[np.arange(n) * (2 * np.pi / n) for n in shape], indexing="ij")


def _kappa(m, n):
    """FD8 symbol of d/dx on the mode e^{i m x}: (1/h) sum_q c_q 2 sin(q m h)"""
    h = 2 * np.pi / n
    return sum(C[q - 1] * 2 * np.sin(q * m * h) for q in range(1, 5)) / h


def test_fd8_modified_wavenumbers():
    shape = (16, 12, 20)
    x = _grid(shape)
    a = (3, -2, 5)
    f = np.sin(a[0] * x[0] + a[1] * x[1] + a[2] * x[2])
    c = np.cos(a[0] * x[0] + a[1] * x[1] + a[2] * x[2])
    g = oracle.fd8_grad(f)
    for d in range(3):
        assert np.abs(g[d] - _kappa(a[d], shape[d]) * c).max() < 1e-12
    # the symbol differs from the exact wavenumber (this is not the spectral derivative)
    assert abs(_kappa(5, 20) - 5) > 1e-4


def test_fd8_is_eighth_order():
    errs = []
    for n in (16, 32):
        shape = (8, 8, n)
        x = _grid(shape)
        g = oracle.fd8_grad(np.sin(x[2]))
        errs.append(np.abs(g[2] - np.cos(x[2])).max())
    ratio = errs[0] / errs[1]
    assert 200 < ratio < 300, ratio  # 2^8 = 256


def test_fd8_summation_by_parts():
    shape = (12, 10, 14)
    rng = np.random.default_rng(800)
    f = rng.standard_normal(shape)
    w = rng.standard_normal((3,) + shape)
    lhs = (oracle.fd8_grad(f) * w).sum()
    rhs = -(f * oracle.fd8_div(w)).sum()
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_fd8_matches_spectral_on_smooth_fields():
    shape = (64, 64, 64)
    f = synth.bandlimited_vector(shape, 3, 801)[0]
    e = rel_l2(oracle.fd8_grad(f), oracle.spectral_grad(f))
    assert 1e-9 < e < 1e-5, e


def test_gradient_at_zero_velocity_with_fd8():
    """v = 0: g = (m1 - m0) grad_FD8 m0, grad_FD8 from the modified wavenumbers."""
    shape = (16, 16, 16)
    x = _grid(shape)
    m0 = np.sin(x[0]) + 0.5 * np.cos(2 * x[1] + x[2])
    k1, k2, k3 = _kappa(1, 16), _kappa(2, 16), _kappa(1, 16)
    gm0 = np.stack([k1 * np.cos(x[0]), -0.5 * k2 * np.sin(2 * x[1] + x[2]),
                    -0.5 * k3 * np.sin(2 * x[1] + x[2])])
    m1 = np.cos(x[2] - x[1])
    P = oracle.Problem(shape, 3, reg=1, beta=0.1, fd8=True)
    P.set_images(m0, m1)
    P.set_velocity(np.zeros((3,) + shape))
    assert np.abs(P.gradient() - (m1 - m0) * gm0).max() < 1e-12
    Q = oracle.Problem(shape, 3, reg=1, beta=0.1)
    Q.set_images(m0, m1)
    Q.set_velocity(np.zeros((3,) + shape))
    assert np.abs(P.gradient() - Q.gradient()).max() > 1e-4  # the scheme is in use
