"""GPU parity of the eighth-order finite-difference first derivatives
(Section 3.2, plans created with LDDMM_FLAG_FD8) against the FP64 oracle run
with the same scheme: grad m_j of the velocity state, the reduced gradient
and the Hessian matvec; the FD8 and spectral plans differ by the scheme's
truncation error only."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import incremental, rel, say, to_dev, to_np
from paper_2008_12820_amd import Plan
from paper_2008_12820_amd import _lib as L

pytestmark = pytest.mark.gpu


def _inputs(shape, nt, seed=1600):
    m0 = synth.f32(synth.blob_image(shape, 10, seed))
    vtrue = synth.f32(synth.bandlimited_vector(shape, 3, seed + 1, max_disp=2.0))
    ref = oracle.Problem(shape, nt, reg=2, beta=1e-3, fd8=True)
    ref.set_images(synth.f64(m0), synth.f64(m0))
    ref.set_velocity(synth.f64(vtrue))
    m1 = synth.f32(ref.transport(synth.f64(m0))[-1])
    v = synth.f32(0.5 * synth.f64(vtrue))
    ref.set_images(synth.f64(m0), synth.f64(m1))
    ref.set_velocity(synth.f64(v))
    return m0, m1, v, ref


@pytest.mark.parametrize("shape,nt", [((32, 32, 32), 4), ((24, 20, 30), 3)])
def test_fd8_plan_matches_oracle(shape, nt):
    say(f"FD8 plan {shape} nt {nt}")
    m0, m1, v, ref = _inputs(shape, nt)
    P = Plan(shape, nt, reg=2, beta=1e-3, fd8=True)
    P.set_images(to_dev(m0), to_dev(m1))
    P.set_velocity(to_dev(v))
    eg_state = rel(to_np(P.get_field(L.FIELD_GRAD_STATE, nt)), ref.get("G", nt))
    g, _ = P.gradient()
    eg = rel(to_np(g), ref.gradient())
    vt = incremental(shape, 1610)
    eh = rel(to_np(P.hessian_matvec(to_dev(vt))), ref.matvec(synth.f64(vt)))
    say(f"grad m_N {eg_state:.2e}, gradient {eg:.2e}, matvec {eh:.2e}")
    assert eg_state < 1e-5 and eg < 1e-5 and eh < 1e-5
    # the spectral plan on the same inputs differs by more than rounding
    S = Plan(shape, nt, reg=2, beta=1e-3)
    S.set_images(to_dev(m0), to_dev(m1))
    S.set_velocity(to_dev(v))
    gs, _ = S.gradient()
    assert rel(to_np(gs), to_np(g)) > 1e-5
