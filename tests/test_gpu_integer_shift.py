"""GPU reduced gradient and Hessian matvec in the integer-shift case whose
exact discrete solution is known in closed form (a constant velocity moving
whole voxels per time step, band-limited sinusoidal images and increment):
the trapezoid body force and the Heun incremental-state source of the GPU
path against that closed form and against the FP64 oracle on the same
float32 inputs."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel, say, to_dev, to_np
from paper_2008_12820_amd import Plan
from paper_2008_12820_amd import _lib as L

import test_oracle_time_quadrature as TQ

pytestmark = pytest.mark.gpu

CASES = TQ.CASES + [((32, 32, 32), 4, (1, 1, -1)), ((24, 20, 30), 8, (1, -1, 1))]


@pytest.mark.parametrize("shape,nt,steps", CASES)
@pytest.mark.parametrize("leray", [False, True])
def test_integer_shift_gradient_and_matvec(shape, nt, steps, leray):
    say(f"integer shift {shape} nt {nt} steps {steps} leray {leray}")
    reg, beta = 2, 1e-3
    dt = 1.0 / nt
    X = TQ.grid(shape)
    h = [TQ.TWO_PI / n for n in shape]
    a = tuple(steps[d] * h[d] for d in range(3))
    m0 = synth.f32(TQ.ev(TQ.M0, X))
    m1 = synth.f32(TQ.ev(TQ.M1, X))
    v = synth.f32(np.stack([np.full(shape, a[d] * nt) for d in range(3)]))
    vt = synth.f32(TQ.ev_vec(TQ.VT, X))
    P = Plan(shape, nt, reg=reg, beta=beta, leray=leray)
    P.set_images(to_dev(m0), to_dev(m1))
    P.set_velocity(to_dev(v))
    ref = oracle.Problem(shape, nt, reg=reg, beta=beta, leray=leray)
    ref.set_images(synth.f64(m0), synth.f64(m1))
    ref.set_velocity(synth.f64(v))
    # closed forms (K = I), projected for the Leray variant
    w = TQ.trapezoid_weights(nt)
    b, bt = 0.0, 0.0
    for j in range(nt + 1):
        sh = tuple(j * ad for ad in a)
        lam_j = TQ.ev(TQ.M1, X, tuple(-(nt - j) * ad for ad in a)) - TQ.ev(TQ.M0, X, sh)
        Y = X + np.array([(nt - j) * ad for ad in a]).reshape(3, 1, 1, 1)
        b = b + w[j] * lam_j * TQ.ev_grad(TQ.M0, X, sh)
        bt = bt - w[j] * TQ.mt_closed(Y, a, nt, dt) * TQ.ev_grad(TQ.M0, X, sh)
    K = oracle.leray if leray else (lambda f: f)
    g_cf = K(dt * b)
    h_cf = beta * TQ.reg_vec(TQ.VT, X, reg) + K(dt * bt)
    mN = to_np(P.get_field(L.FIELD_STATE, nt))
    e_m = rel(mN, TQ.ev(TQ.M0, X, tuple(nt * ad for ad in a)))
    g, _ = P.gradient()
    g = to_np(g)
    hv = to_np(P.hessian_matvec(to_dev(vt)))
    mt = to_np(P.get_field(L.FIELD_INC_STATE))
    e_g, e_h = rel(g, g_cf), rel(hv, h_cf)
    e_mt = rel(mt, TQ.mt_closed(X, a, nt, dt))
    e_go, e_ho = rel(g, ref.gradient()), rel(hv, ref.matvec(synth.f64(vt)))
    say(f"  closed form: m(1) {e_m:.2e} m~(1) {e_mt:.2e} g {e_g:.2e} Hv {e_h:.2e}; "
        f"oracle: g {e_go:.2e} Hv {e_ho:.2e}")
    assert e_m < 1e-6 and e_mt < 1e-5
    assert e_g < 1e-5 and e_h < 1e-5
    assert e_go < 1e-5 and e_ho < 1e-5
    P.close()
