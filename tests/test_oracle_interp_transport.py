"""Pins of the oracle's cubic interpolation, departure points, state and
adjoint transport: exactness on cubics, general Lagrange weights by brute
force, periodicity, exact rolls under integer shifts, convergence orders,
conservation of the adjoint's integral."""
import numpy as np
import pytest

import oracle
import synth


def _lagrange_general(u, nodes):
    """prod_{m != r} (u - x_m)/(x_r - x_m) for every node r."""
    w = []
    for r, xr in enumerate(nodes):
        p = 1.0
        for m, xm in enumerate(nodes):
            if m != r:
                p *= (u - xm) / (xr - xm)
        w.append(p)
    return w


def test_interp_matches_bruteforce_general_lagrange():
    shape = (6, 7, 8)
    rng = np.random.default_rng(10)
    f = rng.standard_normal(shape)
    h = np.array([2 * np.pi / n for n in shape])
    nq = 50
    u = rng.uniform(-9, 17, (3, nq))  # voxel coordinates, many wraps
    got = oracle.interp(f, u * h[:, None])
    for q in range(nq):
        s = 0.0
        b = np.floor(u[:, q]).astype(int)
        nodes = [[b[d] - 1 + r for r in range(4)] for d in range(3)]
        w = [_lagrange_general(u[d, q], nodes[d]) for d in range(3)]
        for a in range(4):
            for bb in range(4):
                for c in range(4):
                    s += f[nodes[0][a] % shape[0], nodes[1][bb] % shape[1],
                           nodes[2][c] % shape[2]] * w[0][a] * w[1][bb] * w[2][c]
        assert abs(got[q] - s) < 1e-12


def test_interp_exact_on_cubic_polynomials():
    shape = (12, 10, 14)
    rng = np.random.default_rng(11)
    coef = rng.standard_normal((3, 4))
    p = [np.polynomial.polynomial.Polynomial(coef[d]) for d in range(3)]
    idx = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    f = p[0](idx[0]) * p[1](idx[1]) * p[2](idx[2])
    h = np.array([2 * np.pi / n for n in shape])
    # queries whose 4x4x4 stencils do not wrap
    u = np.stack([rng.uniform(1, n - 3, 200) for n in shape])
    got = oracle.interp(f, u * h[:, None])
    ref = p[0](u[0]) * p[1](u[1]) * p[2](u[2])
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_interp_nodes_periodicity_partition_of_unity():
    shape = (8, 9, 10)
    rng = np.random.default_rng(12)
    f = rng.standard_normal(shape)
    x = oracle.grid_points(shape).reshape(3, -1)
    assert np.abs(oracle.interp(f, x) - f.ravel()).max() < 1e-14
    y = rng.uniform(0, 2 * np.pi, (3, 64))
    base = oracle.interp(f, y)
    for d in range(3):
        ys = y.copy()
        ys[d] += 2 * np.pi * (d + 1)
        assert np.abs(oracle.interp(f, ys) - base).max() < 1e-11
    assert np.abs(oracle.interp(np.ones(shape), y) - 1).max() < 1e-14


def test_departure_constant_velocity_exact():
    shape = (8, 8, 8)
    c = np.array([0.3, -0.7, 1.1])
    v = np.broadcast_to(c.reshape(3, 1, 1, 1), (3,) + shape).copy()
    nt = 4
    X, Xa = oracle.departure(v, nt)
    x = oracle.grid_points(shape)
    assert np.abs(X - (x - c.reshape(3, 1, 1, 1) / nt)).max() < 1e-14
    assert np.abs(Xa - (x + c.reshape(3, 1, 1, 1) / nt)).max() < 1e-14


def _exact_velocity(y):
    """smooth periodic field given in closed form (evaluated anywhere)"""
    return np.stack([0.6 * np.sin(y[1] + 0.3) + 0.2 * np.cos(y[2]),
                     0.5 * np.cos(y[0] - 0.5 * 0) * np.cos(y[2]),
                     0.4 * np.sin(y[0] + y[1])])


def test_departure_local_error_is_third_order():
    """Heun's local error on the backward trajectory dy/dt = v(y),
    y(t+dt) = x, is O(dt^3) (RK4 reference with exact v)."""
    shape = (48, 48, 48)
    x = oracle.grid_points(shape)
    v = _exact_velocity(x)
    errs = []
    for nt in (4, 8, 16):
        dt = 1.0 / nt
        X, _ = oracle.departure(v, nt)
        y = x.reshape(3, -1).copy()
        sub = 64
        hs = -dt / sub
        for _ in range(sub):
            k1 = _exact_velocity(y)
            k2 = _exact_velocity(y + 0.5 * hs * k1)
            k3 = _exact_velocity(y + 0.5 * hs * k2)
            k4 = _exact_velocity(y + hs * k3)
            y = y + hs / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        errs.append(np.abs(X.reshape(3, -1) - y).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.0 < r1 < 10.5 and 6.0 < r2 < 10.5, errs


@pytest.mark.parametrize("s", [1, -2])
def test_state_integer_shift_is_exact_roll(s):
    shape = (16, 12, 10)
    nt = 4
    h = np.array([2 * np.pi / n for n in shape])
    shift = np.array([s, 0, 2 * s])
    c = shift * h * nt  # c dt = shift voxels per step
    v = np.broadcast_to(c.reshape(3, 1, 1, 1), (3,) + shape).copy()
    rng = np.random.default_rng(13)
    m0 = rng.standard_normal(shape)
    P = oracle.Problem(shape, nt)
    P.set_images(m0, m0)
    P.set_velocity(v)
    m = P.transport(m0)
    for j in range(nt + 1):
        ref = np.roll(m0, tuple(shift * j), axis=(0, 1, 2))
        assert np.abs(m[j] - ref).max() < 1e-12
    # adjoint sweep: exact backward roll, no reaction (div v = 0)
    phi = rng.standard_normal(shape)
    lam = P.adjoint(phi)
    for j in range(nt + 1):
        ref = np.roll(phi, tuple(-shift * (nt - j)), axis=(0, 1, 2))
        assert np.abs(lam[j] - ref).max() < 1e-12


def test_state_subvoxel_shift_fourth_order_in_space():
    """Constant sub-voxel velocity: m(1) = m0(x - c) up to the cubic
    interpolation error, which falls ~16x per grid halving."""
    errs = []
    c = np.array([0.37, -0.21, 0.52])
    for n in (16, 32, 64):
        shape = (n, n, n)
        x = oracle.grid_points(shape)
        m0 = np.sin(x[0] + 2 * x[1]) + 0.5 * np.cos(x[2] - x[0])
        v = np.broadcast_to(c.reshape(3, 1, 1, 1), (3,) + shape).copy()
        P = oracle.Problem(shape, 2)
        P.set_images(m0, m0)
        P.set_velocity(v)
        m1 = P.transport(m0)[-1]
        y = x - c.reshape(3, 1, 1, 1)
        ref = np.sin(y[0] + 2 * y[1]) + 0.5 * np.cos(y[2] - y[0])
        errs.append(np.abs(m1 - ref).max())
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12, errs


def test_adjoint_conserves_integral():
    """-d_t lam - div(lam v) = 0 conserves int lam for any v, so the sweep's
    reaction term must compensate a compressible v (dropping it fails)."""
    shape = (32, 32, 32)
    v = synth.bandlimited_vector(shape, 2, 21, max_disp=3.0)
    phi = 1.0 + 0.5 * synth.bandlimited_scalar(shape, 3, 22)
    P = oracle.Problem(shape, 4)
    P.set_images(phi, phi)
    P.set_velocity(v)
    lam = P.adjoint(phi)
    s_end, s0 = phi.sum(), lam[0].sum()
    assert abs(s0 - s_end) / abs(s_end) < 2e-4
    # pure advection along Xa (reaction term dropped) drifts far more
    Xa = P.get("Xa").reshape(3, -1)
    l = phi.copy()
    for _ in range(4):
        l = oracle.interp(l, Xa).reshape(shape)
    assert abs(l.sum() - s_end) > 20 * abs(s0 - s_end)


def test_departure_points_at_chosen_points_equal_the_whole_field():
    """the point-wise departure evaluation is the whole-grid one restricted"""
    shape, nt = (16, 12, 20), 3
    v = synth.bandlimited_vector(shape, 3, 910, max_disp=2.5)
    X, Xa = oracle.departure(v, nt)
    rng = np.random.default_rng(911)
    idx = np.stack([rng.integers(0, n, 200) for n in shape])
    Xp, Xap = oracle.departure_points(v, nt, idx)
    assert np.array_equal(Xp, X[:, idx[0], idx[1], idx[2]])
    assert np.array_equal(Xap, Xa[:, idx[0], idx[1], idx[2]])
