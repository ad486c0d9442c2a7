"""Pins of the oracle's zero-velocity Hessian preconditioner InvH0 (Section 2
"Preconditioning", eq. h0-pc, Algorithm "PC"): H0 = beta0 A + grad m (x) grad m
with beta0 = max(beta, 5e-2) and m the deformed template m(1), against a closed
form, against the Gauss-Newton matvec at v = 0, against a construction with
numpy's FFT at a nonzero velocity; the inner solve against a dense solve and
its exact reduction to (beta0 A)^{-1} for a constant template; the outer PCG
with InvH0 against the Krylov-optimal iterates of the H0^{-1}-preconditioned
system.  The two-level variant 2LInvH0: spectral restriction and prolongation
against band-limited samples and a numpy construction, its reduction to
(beta0 A)^{-1} for a constant template, and the whole step (restrict, dense
coarse solve, prolong, high-pass) rebuilt with numpy."""
import numpy as np
import pytest

import oracle
import synth

from conftest import rel_l2


def _grid(shape):
    return np.meshgrid(*[np.arange(n) * (2 * np.pi / n) for n in shape], indexing="ij")


def _reg_numpy(s, reg):
    """A s with numpy's FFT: symbol |k|^2 (H1 seminorm) or |k|^4 (H2), per component"""
    shape = s.shape[1:]
    k = np.meshgrid(*[np.fft.fftfreq(n, 1.0 / n) for n in shape], indexing="ij")
    a = (k[0] ** 2 + k[1] ** 2 + k[2] ** 2) ** reg
    return np.stack([np.fft.ifftn(a * np.fft.fftn(c)).real for c in s])


def _h0_numpy(s, G, beta, reg):
    b0 = max(beta, 5e-2)
    return b0 * _reg_numpy(s, reg) + G * (G * s).sum(0)


@pytest.mark.parametrize("beta", [0.3, 1e-3])
def test_h0_closed_form_at_zero_velocity(beta):
    """v = 0: m(1) = m0 = sin x1 + cos(2 x2 + x3)/2, so H0 v~ = beta0 |k|^(2 reg) v~
    + (v~ . grad m0) grad m0 with beta0 = max(beta, 5e-2) (the floor below 5e-2)."""
    shape = (16, 12, 16)
    x = _grid(shape)
    m0 = np.sin(x[0]) + 0.5 * np.cos(2 * x[1] + x[2])
    gm0 = np.stack([np.cos(x[0]), -np.sin(2 * x[1] + x[2]), -0.5 * np.sin(2 * x[1] + x[2])])
    vt = np.stack([np.sin(x[1]), np.cos(x[2] + x[0]), np.sin(2 * x[0] - x[1] + x[2])])
    k2 = np.array([1.0, 2.0, 6.0])
    for reg in (1, 2):
        P = oracle.Problem(shape, 3, reg=reg, beta=beta)
        P.set_images(m0, np.cos(x[2]))
        P.set_velocity(np.zeros((3,) + shape))
        sym = k2 if reg == 1 else k2 ** 2
        ref = max(beta, 5e-2) * sym.reshape(3, 1, 1, 1) * vt + (vt * gm0).sum(0) * gm0
        assert np.abs(P.h0_apply(vt) - ref).max() < 1e-11


def test_h0_is_the_gauss_newton_hessian_at_zero_velocity():
    """At v = 0 (Leray off, beta >= 5e-2) H0 and the Gauss-Newton matvec coincide:
    the zero-velocity approximation is exact there."""
    shape = (16, 16, 16)
    m0 = synth.sin2_template(shape, 3, 700)
    P = oracle.Problem(shape, 4, reg=2, beta=0.1)
    P.set_images(m0, m0 + 0.05)
    P.set_velocity(np.zeros((3,) + shape))
    vt = synth.unit_rms(synth.bandlimited_vector(shape, 4, 701))
    assert rel_l2(P.h0_apply(vt), P.matvec(vt)) < 1e-12


def test_h0_uses_the_deformed_template_and_is_spd():
    """At v != 0 H0 is built from grad m(1), the template transported by v (not
    grad m0): equal to a numpy-FFT construction from grad m_{N_t}; symmetric in
    the h^3 inner product and positive."""
    shape = (16, 16, 16)
    nt = 4
    m0 = synth.sin2_template(shape, 3, 710)
    v = synth.bandlimited_vector(shape, 2, 711, max_disp=2.0)
    P = oracle.Problem(shape, nt, reg=1, beta=1e-3)
    P.set_images(m0, m0)
    P.set_velocity(v)
    G1 = P.get("G", nt)
    G0 = P.get("G", 0)
    a = synth.unit_rms(synth.bandlimited_vector(shape, 3, 712))
    b = synth.unit_rms(synth.bandlimited_vector(shape, 3, 713))
    Ha = P.h0_apply(a)
    assert rel_l2(Ha, _h0_numpy(a, G1, 1e-3, 1)) < 1e-11
    assert rel_l2(Ha, _h0_numpy(a, G0, 1e-3, 1)) > 1e-3  # the refresh matters
    ab, ba = oracle.inner(Ha, b, P.h3), oracle.inner(a, P.h0_apply(b), P.h3)
    assert abs(ab - ba) < 1e-12 * abs(ab)
    assert oracle.inner(Ha, a, P.h3) > 0


def _dense(op, n):
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(op(e))
    return np.stack(cols, 1)


def test_inner_solve_matches_dense_solve():
    shape = (8, 8, 8)
    n3 = 3 * 512
    m0 = synth.sin2_template(shape, 2, 720)
    v = synth.bandlimited_vector(shape, 2, 721, max_disp=0.8)
    P = oracle.Problem(shape, 2, reg=2, beta=1e-2)
    P.set_images(m0, m0)
    P.set_velocity(v)
    G1 = P.get("G", 2)
    H0 = _dense(lambda e: _h0_numpy(e.reshape((3,) + shape), G1, 1e-2, 2).ravel(), n3)
    r = synth.bandlimited_vector(shape, 3, 722)
    sstar = np.linalg.solve(H0, r.ravel())
    s, it = P.invh0(r, 1e-13, 500)
    assert 0 < it < 500
    assert rel_l2(s.ravel(), sstar) < 1e-9
    # a loose tolerance stops early with the residual it promises
    s2, it2 = P.invh0(r, 1e-2, 500)
    assert it2 < it
    res = np.linalg.norm(r.ravel() - H0 @ s2.ravel()) / np.linalg.norm(r)
    assert res <= 1e-2


def test_inner_solve_is_inva_for_a_constant_template():
    """grad m = 0: H0 = beta0 A, and the inner start (beta0 A)^{-1} r already
    solves it for a mean-free r (no iteration)."""
    shape = (12, 12, 12)
    P = oracle.Problem(shape, 2, reg=1, beta=1e-3)
    P.set_images(np.full(shape, 0.3), np.full(shape, 0.7))
    P.set_velocity(synth.bandlimited_vector(shape, 2, 730, max_disp=1.0))
    r = synth.bandlimited_vector(shape, 3, 731)  # band-limited, no zero mode
    s, it = P.invh0(r, 1e-10, 100)
    assert it == 0
    assert np.abs(s - oracle.reg_inverse(r, 1, 5e-2)).max() < 1e-13


def test_pcg_with_invh0_is_krylov_optimal():
    """Outer PCG with the inner solve run to convergence (outer rtol 0 leaves
    the inner solve only its iteration cap): the k-th iterate minimises the
    H-energy error over K_k(H0^{-1} H, H0^{-1} b), computed densely at 8^3.
    v = 0 keeps H exactly symmetric; beta = 1e-2 < 5e-2 makes H0 (beta0 = 5e-2)
    differ from H."""
    shape = (8, 8, 8)
    n3 = 3 * 512
    nt = 2
    m0 = synth.sin2_template(shape, 2, 740)
    P = oracle.Problem(shape, nt, reg=1, beta=1e-2)
    P.set_images(m0, m0 + 0.1)
    P.set_velocity(np.zeros((3,) + shape))
    H = _dense(lambda e: P.matvec(e.reshape((3,) + shape)).ravel(), n3)
    G1 = P.get("G", nt)
    H0 = _dense(lambda e: _h0_numpy(e.reshape((3,) + shape), G1, 1e-2, 1).ravel(), n3)
    assert np.abs(H0 - H).max() > 1e-3
    H0inv = np.linalg.inv(H0)
    b = synth.bandlimited_vector(shape, 2, 742).ravel()
    xstar = np.linalg.solve(H, b)
    prev = np.inf
    K = [H0inv @ b]
    for k in range(1, 5):
        V, _ = np.linalg.qr(np.stack(K, 1))
        xk = V @ np.linalg.solve(V.T @ H @ V, V.T @ b)
        xp, info = P.pcg(b.reshape((3,) + shape), k, 0.0, pc="invh0", eps_h0=1e-3, max_inner=300)
        assert info["iters"] == k and info["inner"] > 0
        assert rel_l2(xp.ravel(), xk) < 1e-8, k
        err = (xp.ravel() - xstar) @ H @ (xp.ravel() - xstar)
        assert err <= prev * (1 + 1e-12)
        prev = err
        K.append(H0inv @ (H @ K[-1]))


def test_invh0_needs_fewer_outer_iterations_than_inva():
    """The paper's point: the zero-velocity Hessian is a far better preconditioner
    than (beta A)^{-1} at small beta (same relative tolerance, same problem)."""
    shape = (16, 16, 16)
    m0 = synth.blob_image(shape, 8, 750)
    vtrue = synth.bandlimited_vector(shape, 3, 751, max_disp=1.5)
    P = oracle.Problem(shape, 4, reg=2, beta=1e-3)
    P.set_images(m0, m0)
    P.set_velocity(vtrue)
    m1 = P.transport(m0)[-1]
    P.set_images(m0, m1)
    P.set_velocity(0.5 * vtrue)
    g = P.gradient()
    _, ia = P.pcg(-g, 200, 1e-3)
    _, ih = P.pcg(-g, 200, 1e-3, pc="invh0", eps_h0=1e-3, max_inner=200)
    assert ih["iters"] < ia["iters"], (ih, ia)
    assert ih["rel_res"] <= 1e-3 and ia["rel_res"] <= 1e-3


# ---- two-level variant 2LInvH0 (Algorithm "PC", second function) ------------


def _np_restrict(f):
    """numpy: fine Fourier coefficients of |k_d| < n_d/4 onto the half grid"""
    shape = f.shape
    nc = [n // 2 for n in shape]
    F = np.fft.fftn(f)
    kc = [np.fft.fftfreq(m, 1.0 / m).astype(int) for m in nc]
    idx = np.ix_(*[k % n for k, n in zip(kc, shape)])
    mask = np.ones(nc)
    for d in range(3):
        sl = [None, None, None]
        sl[d] = slice(None)
        mask = mask * (2 * np.abs(kc[d]) != nc[d])[tuple(sl)]
    return np.fft.ifftn(F[idx] * mask * (np.prod(nc) / np.prod(shape))).real


def _np_prolong(g):
    shape = [2 * n for n in g.shape]
    G = np.fft.fftn(g)
    kc = [np.fft.fftfreq(m, 1.0 / m).astype(int) for m in g.shape]
    mask = np.ones(g.shape)
    for d in range(3):
        sl = [None, None, None]
        sl[d] = slice(None)
        mask = mask * (2 * np.abs(kc[d]) != g.shape[d])[tuple(sl)]
    F = np.zeros(shape, complex)
    F[np.ix_(*[k % n for k, n in zip(kc, shape)])] = G * mask * (np.prod(shape) / np.prod(g.shape))
    return np.fft.ifftn(F).real


def test_restrict_and_prolong_sample_band_limited_fields():
    shape = (16, 12, 20)
    x = _grid(shape)
    f = np.sin(x[0] + 2 * x[2]) + 0.3 * np.cos(2 * x[1] - x[0]) + 0.2  # |k_d| < n_d/4
    xc = _grid(tuple(n // 2 for n in shape))
    fc = np.sin(xc[0] + 2 * xc[2]) + 0.3 * np.cos(2 * xc[1] - xc[0]) + 0.2
    assert np.abs(oracle.restrict(f) - fc).max() < 1e-13
    assert np.abs(oracle.prolong(fc) - f).max() < 1e-13
    assert np.abs(oracle.restrict(oracle.prolong(fc)) - fc).max() < 1e-13
    v = np.stack([f, 2 * f, -f])
    assert np.abs(oracle.restrict(v) - np.stack([fc, 2 * fc, -fc])).max() < 1e-13


def test_high_pass_partition():
    """P R is the projector on |k_d| < n_d/4: idempotent, and f - P R f keeps no
    such mode (numpy FFT); the oracle's R and P equal the numpy construction."""
    shape = (16, 16, 12)
    rng = np.random.default_rng(760)
    f = rng.standard_normal(shape)
    lo = oracle.prolong(oracle.restrict(f))
    assert np.abs(oracle.prolong(oracle.restrict(lo)) - lo).max() < 1e-12
    F = np.fft.fftn(f - lo)
    k = np.meshgrid(*[np.fft.fftfreq(n, 1.0 / n) for n in shape], indexing="ij")
    low = (np.abs(k[0]) < 4) & (np.abs(k[1]) < 4) & (np.abs(k[2]) < 3)
    assert np.abs(F[low]).max() < 1e-10
    assert np.abs(oracle.restrict(f) - _np_restrict(f)).max() < 1e-12
    g = rng.standard_normal((8, 8, 6))
    assert np.abs(oracle.prolong(g) - _np_prolong(g)).max() < 1e-12


def test_two_level_is_inva_for_a_constant_template():
    shape = (16, 16, 16)
    P = oracle.Problem(shape, 2, reg=2, beta=1e-3)
    P.set_images(np.full(shape, 0.3), np.full(shape, 0.7))
    P.set_velocity(synth.bandlimited_vector(shape, 2, 770, max_disp=1.0))
    r = synth.bandlimited_vector(shape, 3, 771)
    s, it = P.two_level_invh0(r, 1e-10, 100)
    assert it == 0
    assert np.abs(s - oracle.reg_inverse(r, 2, 5e-2)).max() < 1e-12 * np.abs(s).max()


def test_two_level_matches_numpy_construction():
    """16^3 fine, 8^3 coarse: restriction, dense coarse H0 solve, prolongation
    and high-pass all by numpy, against the oracle run to convergence."""
    shape = (16, 16, 16)
    nt, beta, reg = 2, 1e-2, 1
    m0 = synth.sin2_template(shape, 3, 780)
    P = oracle.Problem(shape, nt, reg=reg, beta=beta)
    P.set_images(m0, m0)
    P.set_velocity(synth.bandlimited_vector(shape, 2, 781, max_disp=1.0))
    r = synth.bandlimited_vector(shape, 4, 782)
    G1 = P.get("G", nt)
    Gc = np.stack([_np_restrict(g) for g in G1])
    rc = np.stack([_np_restrict(c) for c in r])
    cshape = Gc.shape[1:]
    n3 = 3 * int(np.prod(cshape))
    H0c = _dense(lambda e: _h0_numpy(e.reshape((3,) + cshape), Gc, beta, reg).ravel(), n3)
    sc = np.linalg.solve(H0c, rc.ravel()).reshape((3,) + cshape)
    sf = _reg_inverse_numpy(r, reg, max(beta, 5e-2))
    hp = sf - np.stack([_np_prolong(_np_restrict(c)) for c in sf])
    want = np.stack([_np_prolong(c) for c in sc]) + hp
    s, it = P.two_level_invh0(r, 1e-13, 500)
    assert 0 < it < 500
    assert rel_l2(s, want) < 1e-9


def _reg_inverse_numpy(s, reg, beta):
    shape = s.shape[1:]
    k = np.meshgrid(*[np.fft.fftfreq(n, 1.0 / n) for n in shape], indexing="ij")
    a = (k[0] ** 2 + k[1] ** 2 + k[2] ** 2) ** reg
    inv = np.where(a == 0, 1.0 / beta, 1.0 / (beta * np.where(a == 0, 1.0, a)))
    return np.stack([np.fft.ifftn(inv * np.fft.fftn(c)).real for c in s])


def test_pcg_with_two_level_converges():
    shape = (32, 32, 32)
    m0 = synth.blob_image(shape, 10, 790)
    vtrue = synth.bandlimited_vector(shape, 3, 791, max_disp=2.0)
    P = oracle.Problem(shape, 2, reg=2, beta=1e-3)
    P.set_images(m0, m0)
    P.set_velocity(vtrue)
    m1 = P.transport(m0)[-1]
    P.set_images(m0, m1)
    P.set_velocity(0.5 * vtrue)
    g = P.gradient()
    _, ia = P.pcg(-g, 200, 1e-2)
    _, i2 = P.pcg(-g, 200, 1e-2, pc="2linvh0", eps_h0=1e-3, max_inner=200)
    assert i2["rel_res"] <= 1e-2 and i2["inner"] > 0
    assert i2["iters"] <= ia["iters"], (i2, ia)
