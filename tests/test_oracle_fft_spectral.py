"""Pins of the oracle's DFT/FFT and spectral operators against the
mathematics: brute-force non-separable DFT, numpy's FFT, Parseval, exact
derivatives of band-limited sinusoids, adjointness, projector identities."""
import numpy as np
import pytest

import oracle
import synth

from conftest import rel_l2


def _grid(shape):
    return np.meshgrid(*[np.arange(n) * (2 * np.pi / n) for n in shape], indexing="ij")


@pytest.mark.parametrize("mode", [1, 2])
def test_dft_matches_bruteforce_triple_sum(mode):
    """hat f(k) = sum_x f(x) exp(-i k.x), evaluated as one non-separable sum."""
    shape = (6, 8, 10)
    rng = np.random.default_rng(1)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    x = _grid(shape)
    ks = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = sum(np.multiply.outer(ks[d].ravel(), x[d].ravel()) for d in range(3))
    ref = (np.exp(-1j * phase) @ a.ravel()).reshape(shape)
    oracle.set_fft_mode(mode)
    try:
        got = oracle.fft3(a, -1)
    finally:
        oracle.set_fft_mode(0)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-13


@pytest.mark.parametrize("shape", [(12, 20, 24), (30, 16, 18), (8, 64, 40), (48, 10, 12)])
def test_fft_matches_numpy(shape):
    rng = np.random.default_rng(2)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    for mode in (1, 2):
        oracle.set_fft_mode(mode)
        try:
            got = oracle.fft3(a, -1)
            inv = oracle.fft3(a, +1)
        finally:
            oracle.set_fft_mode(0)
        assert np.abs(got - np.fft.fftn(a)).max() < 1e-12 * np.abs(got).max()
        assert np.abs(inv - np.fft.ifftn(a) * a.size).max() < 1e-12 * np.abs(inv).max()


def test_fft_parseval_and_roundtrip():
    shape = (20, 24, 30)
    rng = np.random.default_rng(3)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    F = oracle.fft3(a, -1)
    assert abs((np.abs(F) ** 2).sum() / a.size - (np.abs(a) ** 2).sum()) < 1e-11 * (np.abs(a) ** 2).sum()
    back = oracle.fft3(F, +1) / a.size
    assert np.abs(back - a).max() < 1e-13


def _sinusoid(shape, a, c):
    x = _grid(shape)
    ph = a[0] * x[0] + a[1] * x[1] + a[2] * x[2] + c
    return np.sin(ph), np.cos(ph)


@pytest.mark.parametrize("shape", [(16, 16, 16), (12, 20, 10)])
def test_grad_div_exact_on_bandlimited(shape):
    a, c = (3, -2, 4), 0.7
    s, co = _sinusoid(shape, a, c)
    g = oracle.spectral_grad(s)
    for d in range(3):
        assert np.abs(g[d] - a[d] * co).max() < 1e-12
    b, c2 = (-1, 4, 2), -0.3
    s2, co2 = _sinusoid(shape, b, c2)
    v = np.stack([s, s2, s + s2])
    div = oracle.spectral_div(v)
    ref = a[0] * co + b[1] * co2 + (a[2] * co + b[2] * co2)
    assert np.abs(div - ref).max() < 1e-12


@pytest.mark.parametrize("reg", [1, 2])
def test_reg_and_inverse_exact_on_bandlimited(reg):
    shape = (16, 12, 20)
    a, c = (2, -3, 5), 0.1
    s, _ = _sinusoid(shape, a, c)
    k2 = sum(x * x for x in a)
    sym = k2 if reg == 1 else k2 * k2
    A = oracle.reg_apply(s, reg)
    assert np.abs(A - sym * s).max() < 1e-10 * sym
    beta = 3e-3
    Ai = oracle.reg_inverse(s + 0.25, reg, beta)
    assert np.abs(Ai - (s / (beta * sym) + 0.25 / beta)).max() < 1e-11 / beta


def test_grad_div_adjoint_on_rough_fields():
    """<grad f, w> = -<f, div w> holds exactly for the discrete operators
    (including the Nyquist modes) -- random, non band-limited inputs."""
    shape = (10, 12, 8)
    rng = np.random.default_rng(4)
    f = rng.standard_normal(shape)
    w = rng.standard_normal((3,) + shape)
    lhs = np.sum(oracle.spectral_grad(f) * w)
    rhs = -np.sum(f * oracle.spectral_div(w))
    assert abs(lhs - rhs) < 1e-11 * np.abs(lhs)


def test_nyquist_reading():
    """First-order symbols drop the Nyquist mode; A keeps it."""
    shape = (8, 8, 8)
    x = _grid(shape)
    f = np.cos(4 * x[2])
    assert np.abs(oracle.spectral_grad(f)).max() < 1e-13
    assert np.abs(oracle.reg_apply(f, 1) - 16 * f).max() < 1e-12


def test_leray_projector_identities():
    shape = (12, 10, 16)
    rng = np.random.default_rng(5)
    w = rng.standard_normal((3,) + shape)
    u = rng.standard_normal((3,) + shape)
    P = oracle.leray(w)
    assert np.abs(oracle.spectral_div(P)).max() < 1e-11
    assert np.abs(oracle.leray(P) - P).max() < 1e-12
    assert abs(np.sum(P * u) - np.sum(w * oracle.leray(u))) < 1e-10 * np.abs(np.sum(P * u))
    phi = rng.standard_normal(shape)
    assert np.abs(oracle.leray(oracle.spectral_grad(phi))).max() < 1e-11
    # divergence-free fields are left alone: curl of a band-limited potential
    vd = synth.bandlimited_vector(shape, 3, 6, divfree=True)
    assert np.abs(oracle.leray(vd) - vd).max() < 1e-12 * np.abs(vd).max() + 1e-14


def test_leray_keeps_syn_velocity():
    """The paper's SYN velocity (component l depends only on the other two
    coordinates) is divergence free, so P leaves it unchanged."""
    m0, v = synth.syn_problem((16, 16, 16))
    assert np.abs(oracle.spectral_div(v)).max() < 1e-13
    assert rel_l2(oracle.leray(v), v) < 1e-13
