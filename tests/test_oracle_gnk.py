"""Pins of the oracle's pieces for the full Gauss-Newton-Krylov driver
(Algorithm "GNK"): trilinear interpolation (d = 1 in the Section 3.1 formula)
against nodes, cell centres and a numpy brute force, exact integer-shift
transport and its first-order convergence; the beta setter (g is affine in
beta with slope A v); the beta-continuation driver's stages and descent."""
import numpy as np

import oracle
import synth

from conftest import rel_l2


def _brute_linear(f, y):
    n = np.array(f.shape)
    h = 2 * np.pi / n
    out = np.empty(y.shape[1])
    for q in range(y.shape[1]):
        u = y[:, q] / h
        b = np.floor(u).astype(int)
        t = u - b
        s = 0.0
        for a in range(2):
            for c in range(2):
                for e in range(2):
                    w = (t[0] if a else 1 - t[0]) * (t[1] if c else 1 - t[1]) * (t[2] if e else 1 - t[2])
                    s += w * f[(b[0] + a) % n[0], (b[1] + c) % n[1], (b[2] + e) % n[2]]
        out[q] = s
    return out


def test_linear_interp_nodes_centres_brute_force():
    shape = (8, 6, 10)
    rng = np.random.default_rng(900)
    f = rng.standard_normal(shape)
    h = np.array([2 * np.pi / n for n in shape]).reshape(3, 1)
    idx = np.stack([rng.integers(0, n, 50) for n in shape])
    assert np.abs(oracle.interp_linear(f, idx * h) - f[idx[0], idx[1], idx[2]]).max() < 1e-13
    cen = oracle.interp_linear(f, (idx + 0.5) * h)
    avg = np.zeros(50)
    for a in range(2):
        for c in range(2):
            for e in range(2):
                avg += f[(idx[0] + a) % shape[0], (idx[1] + c) % shape[1], (idx[2] + e) % shape[2]]
    assert np.abs(cen - avg / 8).max() < 1e-13
    y = rng.uniform(-7, 13, (3, 200))
    assert np.abs(oracle.interp_linear(f, y) - _brute_linear(f, y)).max() < 1e-12
    assert np.abs(oracle.interp_linear(np.full(shape, 2.5), y) - 2.5).max() < 1e-13


def test_linear_transport_integer_shift_is_exact():
    shape, nt = (16, 12, 20), 4
    s = (1, -2, 3)
    v = np.stack([np.full(shape, s[c] * nt * 2 * np.pi / shape[c]) for c in range(3)])
    m0 = synth.blob_image(shape, 5, 901)
    P = oracle.Problem(shape, nt, ip=1)
    P.set_images(m0, m0)
    P.set_velocity(v)
    mt = P.transport(m0)
    assert np.abs(mt[-1] - np.roll(m0, tuple(nt * c for c in s), axis=(0, 1, 2))).max() < 1e-12


def test_linear_transport_converges_at_second_order():
    """a sub-voxel constant shift of a smooth field: the trilinear error drops
    ~4x per grid doubling (the cubic one ~16x) and exceeds the cubic error"""
    def err(n, ip):
        shape = (n, n, n)
        x = np.meshgrid(*[np.arange(n) * (2 * np.pi / n)] * 3, indexing="ij")
        d = 0.3
        v = np.stack([np.full(shape, d), np.full(shape, -0.5 * d), np.full(shape, 0.25 * d)])
        m0 = np.sin(x[0]) * np.cos(x[1] + x[2])
        P = oracle.Problem(shape, 1, ip=ip)
        P.set_images(m0, m0)
        P.set_velocity(v)
        exact = np.sin(x[0] - d) * np.cos(x[1] + 0.5 * d + x[2] - 0.25 * d)
        return np.abs(P.transport(m0)[-1] - exact).max()

    e16, e32 = err(16, 1), err(32, 1)
    assert 3.0 < e16 / e32 < 5.0, e16 / e32
    assert err(16, 3) < 0.1 * e16


def test_set_beta_makes_g_affine_in_beta():
    shape = (16, 16, 16)
    m0 = synth.sin2_template(shape, 3, 910)
    v = synth.bandlimited_vector(shape, 2, 911, max_disp=1.0)
    P = oracle.Problem(shape, 2, reg=2, beta=1e-2)
    P.set_images(m0, m0 + 0.1)
    P.set_velocity(v)
    g1 = P.gradient()
    P.set_beta(3e-2)
    g2 = P.gradient()
    assert rel_l2(g2 - g1, 2e-2 * oracle.reg_apply(v, 2)) < 1e-10


def test_gn_solve_continuation():
    shape, nt = (16, 16, 16), 2
    m0 = synth.blob_image(shape, 6, 920)
    vtrue = synth.bandlimited_vector(shape, 2, 921, max_disp=1.5)
    P = oracle.Problem(shape, nt, reg=2, beta=1e-2)
    P.set_images(m0, m0)
    P.set_velocity(vtrue)
    m1 = P.transport(m0)[-1]
    P.set_images(m0, m1)
    P.set_velocity(np.zeros((3,) + shape))
    J0 = P.objective()[1]
    v, rep = P.gn_solve(np.zeros((3,) + shape), 1e-2, eps_n=5e-2, max_gn=3, max_pcg=20)
    assert rep["stages"] == 3  # beta = 1, 0.1, 0.01
    assert rep["gn_iters"] >= 3 and rep["pcg_iters"] > 0 and rep["inner_iters"] > 0
    P.set_velocity(v)
    assert P.objective()[1] < 0.5 * J0  # the mismatch fell
    # without continuation: one stage at the target beta
    P.set_velocity(np.zeros((3,) + shape))
    _, rep1 = P.gn_solve(np.zeros((3,) + shape), 1e-2, max_gn=2, max_pcg=20, continuation=False, pc="inva")
    assert rep1["stages"] == 1 and rep1["inner_iters"] == 0
