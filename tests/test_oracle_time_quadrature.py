"""Pins of the oracle's time discretisation: the trapezoid rule of the body
force (B(lam) = dt sum_j w_j lam_j grad m_j, eq. reducedgrad and eq. matvec)
and the Heun split of the incremental-state source (eq. incsta), both
readings of Section 2 "Discretization".

With a constant velocity whose step dt*v moves every point by a whole number
of voxels, every departure point lies on the grid, every cubic interpolation
returns a grid value and every characteristic is a periodic roll.  The
divergence vanishes, so the adjoint reaction term drops out.  With
band-limited sinusoidal m0, m1 and v~, whose derivatives and shifts are
exact, each field of the scheme then has a closed form:
  m_j(x)   = m0(x - j a),            a = dt v (one step),
  G_j(x)   = grad m0(x - j a),
  lam_j(x) = phi(x + (N_t - j) a),   phi = lam_{N_t},
  m~_j(x)  = -dt/2 sum_{i<j} (v~(x-(j-i)a) + v~(x-(j-i-1)a)) . grad m0(x - j a),
  b        = dt sum_j w_j lam_j G_j, w_0 = w_{N_t} = 1/2, else 1,
and g = K b (A v = 0 for a constant v), H v~ = beta A v~ + K b~ with
lam~_{N_t} = -m~_{N_t}.  The oracle must reproduce them to rounding.

The same special case fixes the order of the time discretisation without
any reading: the continuous gradient and Hessian matvec are time integrals
of products of shifted sinusoids (evaluated here by Gauss-Legendre
quadrature), and the trapezoid body force with the Heun source converges to
them at second order in dt; a left-endpoint rule or an explicit-Euler source
is first order and gives error ratios near 2 instead of 4 under halving."""
import numpy as np
import pytest

import oracle

from conftest import rel_l2

TWO_PI = 2 * np.pi


# --- band-limited analytic fields ------------------------------------------
# f(x) = sum_q amp_q * sin(k_q . x + ph_q); derivative and A symbol exact.
M0 = [(1.0, (1, 2, 0), 0.3), (0.5, (-1, 0, 1), 1.2), (0.3, (0, 0, 2), -0.4)]
M1 = [(1.0, (1, -1, 1), 0.7), (0.2, (0, 1, 0), 0.1)]
VT = [
    [(1.0, (0, 1, 0), 0.0), (0.4, (1, 0, 1), 0.5)],
    [(1.0, (1, 0, 1), 1.0), (0.3, (0, 2, -1), -0.2)],
    [(1.0, (2, -1, 1), 0.2)],
]


def ev(terms, X, shift=(0.0, 0.0, 0.0)):
    """f(X - shift) for the point array X [3][...]"""
    out = 0.0
    for amp, k, ph in terms:
        arg = sum(k[d] * (X[d] - shift[d]) for d in range(3)) + ph
        out = out + amp * np.sin(arg)
    return out


def ev_grad(terms, X, shift=(0.0, 0.0, 0.0)):
    comps = []
    for d in range(3):
        s = 0.0
        for amp, k, ph in terms:
            arg = sum(k[e] * (X[e] - shift[e]) for e in range(3)) + ph
            s = s + amp * k[d] * np.cos(arg)
        comps.append(s)
    return np.stack(comps)


def ev_vec(terms3, X, shift=(0.0, 0.0, 0.0)):
    return np.stack([ev(t, X, shift) for t in terms3])


def reg_vec(terms3, X, reg):
    """A v~ per component, A = -Laplacian (reg 1) or its square (reg 2)"""
    comps = []
    for t in terms3:
        s = 0.0
        for amp, k, ph in t:
            k2 = float(sum(kk * kk for kk in k))
            s = s + (k2 if reg == 1 else k2 * k2) * amp * np.sin(sum(k[d] * X[d] for d in range(3)) + ph)
        comps.append(s)
    return np.stack(comps)


def grid(shape):
    return np.stack(np.meshgrid(*[np.arange(n) * (TWO_PI / n) for n in shape], indexing="ij"))


def trapezoid_weights(nt):
    w = np.ones(nt + 1)
    w[0] = w[-1] = 0.5
    return w


def mt_closed(X, a, j, dt):
    """m~_j(X) of the Heun scheme under the integer shift a per step"""
    s = 0.0
    gm = ev_grad(M0, X, tuple(j * ad for ad in a))
    for i in range(j):
        vt = 0.5 * (ev_vec(VT, X, tuple((j - i) * ad for ad in a)) +
                    ev_vec(VT, X, tuple((j - i - 1) * ad for ad in a)))
        s = s + (vt * gm).sum(0)
    return -dt * s


def problem(shape, nt, steps, reg=2, beta=1e-3, leray=False):
    """oracle problem with the constant velocity moving `steps` voxels per
    time step (integers per axis); returns (P, X grid, a, v)"""
    h = np.array([TWO_PI / n for n in shape])
    a = tuple(float(steps[d] * h[d]) for d in range(3))
    v = np.stack([np.full(shape, a[d] * nt) for d in range(3)])  # dt v = a
    X = grid(shape)
    P = oracle.Problem(shape, nt, reg=reg, beta=beta, leray=leray)
    P.set_images(ev(M0, X), ev(M1, X))
    P.set_velocity(v)
    return P, X, a, v


CASES = [((16, 16, 16), 2, (1, -2, 1)), ((24, 16, 20), 3, (2, 1, -1)), ((16, 20, 24), 4, (-1, 1, 2))]


@pytest.mark.parametrize("shape,nt,steps", CASES)
def test_integer_shift_state_adjoint_exact(shape, nt, steps):
    P, X, a, v = problem(shape, nt, steps)
    for j in range(nt + 1):
        sh = tuple(j * ad for ad in a)
        assert np.abs(P.get("m", j) - ev(M0, X, sh)).max() < 1e-12, j
        assert np.abs(P.get("G", j) - ev_grad(M0, X, sh)).max() < 1e-11, j
    phi = ev(M1, X) - ev(M0, X, tuple(nt * ad for ad in a))
    lam = P.adjoint(phi)
    for j in range(nt + 1):
        want = ev(M1, X, tuple(-(nt - j) * ad for ad in a)) - ev(M0, X, tuple(j * ad for ad in a))
        assert np.abs(lam[j] - want).max() < 1e-12, j


@pytest.mark.parametrize("shape,nt,steps", CASES)
def test_integer_shift_body_force_and_gradient_exact(shape, nt, steps):
    """O9: the trapezoid in time; g = K b with A v = 0"""
    P, X, a, v = problem(shape, nt, steps)
    dt = 1.0 / nt
    w = trapezoid_weights(nt)
    b = 0.0
    for j in range(nt + 1):
        lam_j = ev(M1, X, tuple(-(nt - j) * ad for ad in a)) - ev(M0, X, tuple(j * ad for ad in a))
        b = b + w[j] * lam_j * ev_grad(M0, X, tuple(j * ad for ad in a))
    b = dt * b
    g = P.gradient()
    assert rel_l2(g, b) < 1e-12
    # the body-force step on its own, from the oracle's adjoint
    phi = ev(M1, X) - ev(M0, X, tuple(nt * ad for ad in a))
    assert rel_l2(P.body_force(P.adjoint(phi)), b) < 1e-12
    # the test separates the trapezoid from the one-sided rules
    for wl in (np.r_[np.ones(nt), 0.0], np.r_[0.0, np.ones(nt)]):
        bl = 0.0
        for j in range(nt + 1):
            lam_j = ev(M1, X, tuple(-(nt - j) * ad for ad in a)) - ev(M0, X, tuple(j * ad for ad in a))
            bl = bl + wl[j] * lam_j * ev_grad(M0, X, tuple(j * ad for ad in a))
        assert rel_l2(dt * bl, b) > 1e-2


@pytest.mark.parametrize("shape,nt,steps", CASES)
@pytest.mark.parametrize("reg", [1, 2])
def test_integer_shift_incremental_state_and_matvec_exact(shape, nt, steps, reg):
    """O12: the Heun source dt/2 (v~(X).I[G_j](X) + v~.G_{j+1}); O13 with it"""
    beta = 1e-3
    P, X, a, v = problem(shape, nt, steps, reg=reg, beta=beta)
    dt = 1.0 / nt
    vt = ev_vec(VT, X)
    mt = P.inc_state(vt)
    for j in range(nt + 1):
        assert np.abs(mt[j] - mt_closed(X, a, j, dt)).max() < 1e-12, j
    # an explicit-Euler source, m~_{j+1} = I[m~_j](X) - dt v~(X).I[G_j](X), differs
    euler = 0.0
    for i in range(nt):
        euler = euler - dt * (ev_vec(VT, X, tuple((nt - i) * ad for ad in a)) *
                              ev_grad(M0, X, tuple(nt * ad for ad in a))).sum(0)
    assert rel_l2(euler, mt[nt]) > 1e-2
    # lam~_j = -m~_N(x + (N - j) a); b~ by the trapezoid; H v~ = beta A v~ + b~
    w = trapezoid_weights(nt)
    bt = 0.0
    for j in range(nt + 1):
        Y = X + np.array([(nt - j) * ad for ad in a]).reshape(3, 1, 1, 1)
        lam_j = -mt_closed(Y, a, nt, dt)
        bt = bt + w[j] * lam_j * ev_grad(M0, X, tuple(j * ad for ad in a))
    hv = beta * reg_vec(VT, X, reg) + dt * bt
    assert rel_l2(P.matvec(vt), hv) < 1e-12


def test_integer_shift_leray_variant():
    shape, nt, steps = (16, 16, 16), 2, (1, -2, 1)
    P, X, a, v = problem(shape, nt, steps, leray=True)
    Q, _, _, _ = problem(shape, nt, steps, leray=False)
    vt = ev_vec(VT, X)
    beta = 1e-3
    b = Q.matvec(vt) - beta * reg_vec(VT, X, 2)
    assert rel_l2(P.matvec(vt), beta * reg_vec(VT, X, 2) + oracle.leray(b)) < 1e-12
    assert rel_l2(P.gradient(), oracle.leray(Q.gradient())) < 1e-12


# --- second order in time ----------------------------------------------------

def _gauss(nq=24):
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def continuous_gradient(X, c):
    """int_0^1 lam(x,t) grad m(x,t) dt, lam(x,t) = (m1 - m(.,1))(x + (1-t)c),
    m(x,t) = m0(x - tc): the reduced gradient's body force for v = c"""
    tq, wq = _gauss()
    out = 0.0
    for t, w in zip(tq, wq):
        back = tuple(-(1 - t) * cd for cd in c)
        lam = ev(M1, X, back) - ev(M0, X, tuple(cd * t for cd in c))  # m0(y - c), y = x + (1-t)c
        out = out + w * lam * ev_grad(M0, X, tuple(cd * t for cd in c))
    return out


def continuous_inc_state(Y, c):
    """m~(y, 1) = -int_0^1 v~(y - (1-tau)c) dtau . grad m0(y - c)"""
    tq, wq = _gauss()
    s = 0.0
    for tau, w in zip(tq, wq):
        s = s + w * ev_vec(VT, Y, tuple((1 - tau) * cd for cd in c))
    return -(s * ev_grad(M0, Y, tuple(c))).sum(0)


def continuous_matvec_body(X, c):
    """int_0^1 lam~(x,t) grad m(x,t) dt, lam~(x,t) = -m~(x + (1-t)c, 1)"""
    tq, wq = _gauss()
    out = 0.0
    for t, w in zip(tq, wq):
        Y = X + np.array([(1 - t) * cd for cd in c]).reshape(3, 1, 1, 1)
        out = out - w * continuous_inc_state(Y, c) * ev_grad(M0, X, tuple(cd * t for cd in c))
    return out


def test_time_discretisation_is_second_order():
    """Total displacement fixed (8, 8, 0 voxels on a 64 x 64 x 16 grid, i.e. pi/4
    along x1 and x2), N_t = 2, 4, 8 with 4, 2, 1 voxels per step: g and
    H v~ - beta A v~ approach the time integrals with error ratios of about 4
    per halving of dt (measured 4.19, 4.04 and 4.17, 4.04)."""
    shape = (64, 64, 16)
    h = TWO_PI / 64
    c = (8 * h, 8 * h, 0.0)
    X = grid(shape)
    g_ref = continuous_gradient(X, c)
    hb_ref = continuous_matvec_body(X, c)
    vt = ev_vec(VT, X)
    eg, eh = [], []
    for nt in (2, 4, 8):
        steps = (8 // nt, 8 // nt, 0)
        P, _, _, _ = problem(shape, nt, steps, reg=2, beta=1e-3)
        eg.append(rel_l2(P.gradient(), g_ref))
        eh.append(rel_l2(P.matvec(vt) - 1e-3 * reg_vec(VT, X, 2), hb_ref))
    rg = [eg[0] / eg[1], eg[1] / eg[2]]
    rh = [eh[0] / eh[1], eh[1] / eh[2]]
    print("gradient errors", eg, "ratios", rg)
    print("matvec errors", eh, "ratios", rh)
    for r in rg + rh:
        assert 3.6 < r < 4.5, (rg, rh)
    assert eg[-1] < 1e-2 and eh[-1] < 1e-2
