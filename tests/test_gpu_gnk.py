"""GPU parity of the full Gauss-Newton-Krylov driver pieces against the FP64
oracle: plans with trilinear interpolation (LDDMM_FLAG_LINEAR_IP, d = 1 in
the Section 3.1 formula), the beta setter, and the beta-continuation solve
(Algorithm "GNK") with a fixed iteration schedule; argument checks."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, incremental, rel, say, to_dev, to_np
from paper_2008_12820_amd import LddmmError, Plan
from paper_2008_12820_amd import _lib as L

pytestmark = pytest.mark.gpu


def _inputs(shape, nt, ip, seed=1700, beta=1e-3):
    m0 = synth.f32(synth.blob_image(shape, 10, seed))
    vtrue = synth.f32(synth.bandlimited_vector(shape, 3, seed + 1, max_disp=2.0))
    ref = oracle.Problem(shape, nt, reg=2, beta=beta, ip=ip)
    ref.set_images(synth.f64(m0), synth.f64(m0))
    ref.set_velocity(synth.f64(vtrue))
    m1 = synth.f32(ref.transport(synth.f64(m0))[-1])
    v = synth.f32(0.5 * synth.f64(vtrue))
    ref.set_images(synth.f64(m0), synth.f64(m1))
    ref.set_velocity(synth.f64(v))
    return m0, m1, v, ref


@pytest.mark.parametrize("shape,nt", [((32, 32, 32), 4), ((24, 20, 30), 3)])
def test_linear_ip_plan_matches_oracle(shape, nt):
    say(f"trilinear plan {shape} nt {nt}")
    m0, m1, v, ref = _inputs(shape, nt, ip=1)
    P = Plan(shape, nt, reg=2, beta=1e-3, linear_ip=True)
    P.set_images(to_dev(m0), to_dev(m1))
    P.set_velocity(to_dev(v))
    es = rel(to_np(P.get_field(L.FIELD_STATE, nt)), ref.get("m", nt))
    g, _ = P.gradient()
    eg = rel(to_np(g), ref.gradient())
    vt = incremental(shape, 1710)
    eh = rel(to_np(P.hessian_matvec(to_dev(vt))), ref.matvec(synth.f64(vt)))
    say(f"m(1) {es:.2e}, gradient {eg:.2e}, matvec {eh:.2e}")
    assert es < 1e-6 and eg < 1e-5 and eh < 1e-5


def test_linear_ip_integer_shift_is_exact():
    shape, nt = (32, 24, 40), 4
    s = (1, -2, 3)
    v = torch.stack([torch.full(shape, s[c] * nt * 2 * np.pi / shape[c], device=DEV) for c in range(3)])
    m0 = to_dev(synth.f32(synth.blob_image(shape, 6, 1720)))
    P = Plan(shape, nt, linear_ip=True)
    m1 = P.transport_forward(m0, v)
    want = torch.roll(m0, shifts=tuple(nt * c for c in s), dims=(0, 1, 2))
    assert rel(to_np(m1), to_np(want)) < 1e-6


def test_set_beta_matches_oracle():
    shape, nt = (24, 24, 24), 3
    m0, m1, v, ref = _inputs(shape, nt, ip=3, beta=1e-2)
    P = Plan(shape, nt, reg=2, beta=1e-2)
    P.set_images(to_dev(m0), to_dev(m1))
    P.set_velocity(to_dev(v))
    P.set_beta(3e-2)
    ref.set_beta(3e-2)
    g, _ = P.gradient()
    assert rel(to_np(g), ref.gradient()) < 1e-5
    with pytest.raises(LddmmError) as e:
        P.set_beta(0.0)
    assert e.value.status == L.EINVAL


def test_gn_solve_matches_oracle():
    """beta = 1, 1e-1, 1e-2 with two Newton steps each, five PCG iterations
    (InvA above beta 0.5, 2LInvH0 below, five coarse iterations): the same
    schedule on both sides."""
    shape, nt = (32, 32, 32), 2
    say("gn_solve with continuation")
    m0 = synth.f32(synth.blob_image(shape, 8, 1730))
    vtrue = synth.f32(synth.bandlimited_vector(shape, 2, 1731, max_disp=1.5))
    ref = oracle.Problem(shape, nt, reg=2, beta=1e-2)
    ref.set_images(synth.f64(m0), synth.f64(m0))
    ref.set_velocity(synth.f64(vtrue))
    m1 = synth.f32(ref.transport(synth.f64(m0))[-1])
    ref.set_images(synth.f64(m0), synth.f64(m1))
    kw = dict(eps_n=0.0, max_gn=2, max_pcg=5, rtol=1e-12, continuation=True, pc="2linvh0", eps_h0=1e-3,
              max_inner=5)
    v_ref, rep_ref = ref.gn_solve(np.zeros((3,) + shape), 1e-2, **kw)
    P = Plan(shape, nt, reg=2, beta=1e-2)
    P.set_images(to_dev(m0), to_dev(m1))
    v = torch.zeros((3,) + shape, device=DEV)
    rep = P.gn_solve(v, 1e-2, **kw)
    say(f"report {rep} vs {rep_ref}")
    for k in ("stages", "gn_iters", "pcg_iters", "inner_iters"):
        assert rep[k] == rep_ref[k], k
    e = rel(to_np(v), v_ref)
    say(f"final velocity rel {e:.2e}")
    assert e < 1e-5
    assert abs(rep["J"] - rep_ref["J"]) <= 1e-5 * abs(rep_ref["J"])


def test_gn_solve_arguments():
    P = Plan((16, 16, 16), 2, reg=2, beta=1e-2)
    v = torch.zeros((3, 16, 16, 16), device=DEV)
    with pytest.raises(LddmmError) as e:
        P.gn_solve(v, 1e-2)
    assert e.value.status == L.ESTATE
    m0 = to_dev(synth.f32(synth.blob_image((16, 16, 16), 4, 1740)))
    P.set_images(m0, m0)
    for bad in (dict(beta_target=0.0), dict(max_inner=0), dict(eps_h0=1.0), dict(max_gn=-1)):
        kw = dict(beta_target=1e-2)
        kw.update(bad)
        bt = kw.pop("beta_target")
        with pytest.raises(LddmmError) as e:
            P.gn_solve(v, bt, **kw)
        assert e.value.status == L.EINVAL, bad
