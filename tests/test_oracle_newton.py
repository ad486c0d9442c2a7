"""Pins of the oracle's gradient, Hessian matvec, PCG and transport VJP:
closed forms at v = 0, linearity, symmetry (exact at v = 0, shrinking with
refinement otherwise), finite-difference consistency (a discretise-after-
optimise scheme: agreement to discretisation error, falling with refinement),
and Krylov optimality of the PCG iterates against a dense solve."""
import numpy as np
import pytest

import oracle
import synth

from conftest import rel_l2


def _grid(shape):
    return np.meshgrid(*[np.arange(n) * (2 * np.pi / n) for n in shape], indexing="ij")


def _closed_form_inputs(shape):
    """band-limited m0, m1, v~ with closed-form derivatives and A symbols"""
    x = _grid(shape)
    m0 = np.sin(x[0]) + 0.5 * np.cos(2 * x[1] + x[2])
    gm0 = np.stack([np.cos(x[0]), -np.sin(2 * x[1] + x[2]), -0.5 * np.sin(2 * x[1] + x[2])])
    m1 = np.cos(x[2] - x[1])
    vt = np.stack([np.sin(x[1]), np.cos(x[2] + x[0]), np.sin(2 * x[0] - x[1] + x[2])])
    k2 = np.array([1.0, 2.0, 6.0])  # |k|^2 of each component of vt
    return m0, gm0, m1, vt, k2


@pytest.mark.parametrize("reg", [1, 2])
def test_matvec_and_gradient_at_zero_velocity(reg):
    """v = 0: m~_j = -t_j v~.grad m0, lam~ = v~.grad m0, so
    H v~ = beta A v~ + (v~.grad m0) grad m0 and g = (m1 - m0) grad m0."""
    shape = (16, 16, 16)
    nt, beta = 4, 0.3
    m0, gm0, m1, vt, k2 = _closed_form_inputs(shape)
    P = oracle.Problem(shape, nt, reg=reg, beta=beta)
    P.set_images(m0, m1)
    P.set_velocity(np.zeros((3,) + shape))
    sym = k2 if reg == 1 else k2 ** 2
    proj = (vt * gm0).sum(0)
    ref = beta * sym.reshape(3, 1, 1, 1) * vt + proj * gm0
    assert np.abs(P.matvec(vt) - ref).max() < 1e-11
    mt = P.inc_state(vt)
    for j in range(nt + 1):
        assert np.abs(mt[j] + (j / nt) * proj).max() < 1e-12
    assert np.abs(P.gradient() - (m1 - m0) * gm0).max() < 1e-12
    J, mis, rg = P.objective()
    assert abs(mis - 0.5 * P.h3 * ((m0 - m1) ** 2).sum()) < 1e-12 * mis
    assert rg == 0.0


def test_leray_variant_at_zero_velocity():
    shape = (12, 12, 12)
    m0, gm0, m1, vt, k2 = _closed_form_inputs(shape)
    P = oracle.Problem(shape, 2, reg=1, beta=0.1, leray=True)
    P.set_images(m0, m1)
    P.set_velocity(np.zeros((3,) + shape))
    body = (vt * gm0).sum(0) * gm0
    ref = 0.1 * k2.reshape(3, 1, 1, 1) * vt + oracle.leray(body)
    assert np.abs(P.matvec(vt) - ref).max() < 1e-11
    # the projected part is divergence free and differs from the raw body force
    assert np.abs(oracle.spectral_div(P.matvec(vt) - 0.1 * k2.reshape(3, 1, 1, 1) * vt)).max() < 1e-10
    assert np.abs(oracle.leray(body) - body).max() > 1e-2


def _problem32(v_scale=0.5, leray=False, nt=4, n=32, reg=1, beta=1e-2):
    shape = (n, n, n)
    m0 = synth.sin2_template(shape, 4, 1000)
    vtrue = synth.bandlimited_vector(shape, 3, 1001, max_disp=0.5 * n / (2 * np.pi))
    P = oracle.Problem(shape, nt, reg=reg, beta=beta, leray=leray)
    P.set_images(m0, m0)
    P.set_velocity(vtrue)
    m1 = P.transport(m0)[-1]
    P.set_images(m0, m1)
    P.set_velocity(v_scale * vtrue)
    return P, vtrue


def test_matvec_linear():
    P, _ = _problem32()
    shape = P.shape
    a = synth.unit_rms(synth.bandlimited_vector(shape, 3, 1100))
    b = synth.unit_rms(synth.bandlimited_vector(shape, 3, 1101))
    lhs = P.matvec(2.0 * a - 0.5 * b)
    rhs = 2.0 * P.matvec(a) - 0.5 * P.matvec(b)
    assert rel_l2(lhs, rhs) < 1e-12


def test_symmetry_exact_at_zero_and_converging_otherwise():
    shape = (16, 16, 16)
    rng = np.random.default_rng(30)
    x = synth.unit_rms(synth.bandlimited_vector(shape, 3, 31))
    y = synth.unit_rms(synth.bandlimited_vector(shape, 3, 32))
    m0 = synth.sin2_template(shape, 3, 33)
    P = oracle.Problem(shape, 4, reg=2, beta=1e-3)
    P.set_images(m0, m0)
    P.set_velocity(np.zeros((3,) + shape))
    a, b = oracle.inner(P.matvec(x), y, P.h3), oracle.inner(x, P.matvec(y), P.h3)
    assert abs(a - b) < 1e-12 * abs(a)
    assert oracle.inner(P.matvec(x), x, P.h3) > 0

    def asym(n, nt):
        shp = (n, n, n)
        m0 = synth.sin2_template(shp, 3, 33)
        v = synth.bandlimited_vector(shp, 2, 34, max_disp=0.6 * n / (2 * np.pi))
        xx = synth.unit_rms(synth.bandlimited_vector(shp, 3, 31))
        yy = synth.unit_rms(synth.bandlimited_vector(shp, 3, 32))
        Q = oracle.Problem(shp, nt, reg=2, beta=1e-3)
        Q.set_images(m0, m0)
        Q.set_velocity(v)
        Hx, Hy = Q.matvec(xx), Q.matvec(yy)
        d = abs(oracle.inner(Hx, yy, Q.h3) - oracle.inner(xx, Hy, Q.h3))
        assert oracle.inner(Hx, xx, Q.h3) > 0
        return d / (np.sqrt(oracle.inner(Hx, Hx, Q.h3)) * np.sqrt(oracle.inner(yy, yy, Q.h3)))

    a1, a2 = asym(16, 4), asym(32, 8)
    assert a2 < a1, (a1, a2)


def _fd_gap(n, nt, eps=1e-3):
    P, vtrue = _problem32(n=n, nt=nt)
    v = 0.5 * vtrue
    w = synth.bandlimited_vector(P.shape, 3, 1200)
    w *= np.abs(v).max() / np.abs(w).max()
    P.set_velocity(v)
    g = P.gradient()
    gw = oracle.inner(g, w, P.h3)
    P.set_velocity(v + eps * w)
    Jp = P.objective()[0]
    P.set_velocity(v - eps * w)
    Jm = P.objective()[0]
    return abs((Jp - Jm) / (2 * eps) - gw) / abs(gw)


def test_gradient_finite_difference_consistency():
    """(J(v+ew) - J(v-ew))/2e vs <g,w>: the discretise-after-optimise gap is
    small and shrinks under refinement; a sign/scale/index error gives O(1)."""
    g1 = _fd_gap(32, 4)
    g2 = _fd_gap(48, 8)
    assert g1 < 5e-2, g1
    assert g2 < g1, (g1, g2)


def test_matvec_matches_fd_of_gradient_at_zero_residual():
    """At v = v_true (m1 from the same scheme) the residual vanishes, the
    Gauss-Newton and full Hessians agree, and (g(v+ew)-g(v-ew))/2e ~ H w."""
    P, vtrue = _problem32(v_scale=1.0, n=32, nt=4)
    w = synth.bandlimited_vector(P.shape, 3, 1300)
    w *= 0.5 * np.abs(vtrue).max() / np.abs(w).max()
    Hw = P.matvec(w)
    eps = 1e-3
    P.set_velocity(vtrue + eps * w)
    gp = P.gradient()
    P.set_velocity(vtrue - eps * w)
    gm = P.gradient()
    fd = (gp - gm) / (2 * eps)
    assert rel_l2(fd, Hw) < 5e-2


def _dense(op, n):
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(op(e))
    return np.stack(cols, 1)


def test_pcg_iterates_are_krylov_optimal():
    """k-step PCG (x0 = 0, M^-1 = (beta A)^-1) equals argmin over the Krylov
    space K_k(M^-1 H, M^-1 b) of the H-energy error, computed densely at 8^3."""
    shape = (8, 8, 8)
    n3 = 3 * 512
    m0 = synth.sin2_template(shape, 2, 40)
    P = oracle.Problem(shape, 2, reg=1, beta=5e-2)
    P.set_images(m0, m0 + 0.1)
    P.set_velocity(np.zeros((3,) + shape))
    H = _dense(lambda e: P.matvec(e.reshape((3,) + shape)).ravel(), n3)
    Minv = _dense(lambda e: oracle.reg_inverse(e.reshape((3,) + shape), 1, 5e-2).ravel(), n3)
    b = synth.bandlimited_vector(shape, 2, 41).ravel()
    xstar = np.linalg.solve(H, b)
    prev = np.inf
    K = [Minv @ b]
    for k in range(1, 6):
        V, _ = np.linalg.qr(np.stack(K, 1))
        xk = V @ np.linalg.solve(V.T @ H @ V, V.T @ b)
        xp, info = P.pcg(b.reshape((3,) + shape), k, 0.0)
        assert info["iters"] == k
        assert rel_l2(xp.ravel(), xk) < 1e-8, k
        err = (xp.ravel() - xstar) @ H @ (xp.ravel() - xstar)
        assert err <= prev * (1 + 1e-12)
        prev = err
        K.append(Minv @ (H @ K[-1]))
    # converged solve
    xp, info = P.pcg(b.reshape((3,) + shape), 300, 1e-10)
    assert rel_l2(xp.ravel(), xstar) < 1e-7


def test_transport_vjp_total_equals_gradient():
    """L = 1/2 sum (m(1)-m1)^2 + beta/2 sum (Av).v (plain sums): the VJP's
    beta A v + dL/dv reproduces the reduced gradient with K = I exactly."""
    P, vtrue = _problem32(n=16, nt=4)
    m0 = synth.sin2_template(P.shape, 4, 1000)
    m = P.transport(m0)
    P.set_images(m0, m[-1] * 0.9 + 0.05)
    gout = m[-1] - (m[-1] * 0.9 + 0.05)
    gm0, gv = P.transport_vjp(m0, gout)
    v = P.get("v")
    total = P.beta * oracle.reg_apply(v, 1) + gv
    assert rel_l2(total, P.gradient()) < 1e-12


def test_transport_vjp_finite_difference_consistency():
    P, vtrue = _problem32(n=32, nt=4)
    m0 = synth.sin2_template(P.shape, 4, 1000)
    target = synth.blob_image(P.shape, 8, 1400)
    v = P.get("v")

    def loss(mm0, vv):
        P.set_velocity(vv)
        return 0.5 * ((P.transport(mm0)[-1] - target) ** 2).sum()

    P.set_velocity(v)
    gout = P.transport(m0)[-1] - target
    gm0, gv = P.transport_vjp(m0, gout)
    w = synth.bandlimited_vector(P.shape, 3, 1401)
    w *= np.abs(v).max() / np.abs(w).max()
    eps = 1e-3
    fd = (loss(m0, v + eps * w) - loss(m0, v - eps * w)) / (2 * eps)
    assert abs(fd - (gv * w).sum()) / abs(fd) < 5e-2
    dm = synth.bandlimited_scalar(P.shape, 4, 1402)
    fd0 = (loss(m0 + eps * dm, v) - loss(m0 - eps * dm, v)) / (2 * eps)
    assert abs(fd0 - (gm0 * dm).sum()) / abs(fd0) < 5e-2


def test_gn_iteration_decreases_objective():
    P, vtrue = _problem32(v_scale=0.0, n=16, nt=4, reg=2, beta=1e-3)
    P.set_velocity(np.zeros((3,) + P.shape))
    J0 = P.objective()[0]
    v, info = P.gn_iterate(10, 0.0)
    assert info["alpha"] > 0
    assert info["J_after"] < J0
    assert abs(P.objective()[0] - info["J_after"]) < 1e-14
