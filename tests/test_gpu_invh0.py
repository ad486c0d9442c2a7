"""GPU parity of the zero-velocity Hessian preconditioners InvH0 and 2LInvH0
(Section 2 "Preconditioning", eq. h0-pc, Algorithm "PC") against the FP64
oracle: the H0 operator, the inner PCG solve at a fixed iteration count and at
a tolerance, the two-level step, Newton steps whose PCG uses them; argument
checks."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import DEV, incremental, problem, rel, say, to_dev, to_np
from paper_2008_12820_amd import LddmmError, Plan
from paper_2008_12820_amd import _lib as L
from paper_2008_12820_amd.batch import Batch

pytestmark = pytest.mark.gpu


def _setup(shape=(24, 20, 30), nt=3, reg=2, beta=1e-3, leray=False, disp=2.0):
    m0, m1, vtrue, v, ref = problem(shape, nt, reg, beta, leray, disp=disp, nblobs=10)
    P = Plan(shape, nt, reg=reg, beta=beta, leray=leray)
    P.set_images(to_dev(m0), to_dev(m1))
    P.set_velocity(to_dev(v))
    return P, ref


@pytest.mark.parametrize("beta,reg", [(1e-3, 2), (0.2, 1)])
def test_h0_apply_matches_oracle(beta, reg):
    say(f"H0 apply beta {beta} reg {reg}")
    P, ref = _setup(beta=beta, reg=reg)
    s = incremental(P.shape, 1500)
    e = rel(to_np(P.apply_h0(to_dev(s))), ref.h0_apply(synth.f64(s)))
    say(f"H0 rel {e:.2e}")
    assert e < 1e-5


def test_inner_solve_matches_oracle():
    say("InvH0 inner solve")
    P, ref = _setup()
    r = incremental(P.shape, 1501)
    s, it = P.apply_invh0(to_dev(r), 0.0, 6)
    s_ref, it_ref = ref.invh0(synth.f64(r), 0.0, 6)
    assert it == it_ref == 6
    e = rel(to_np(s), s_ref)
    say(f"6 inner iterations: rel {e:.2e}")
    assert e < 1e-5
    # to a tolerance: the same stopping rule, so the same iteration within one.
    # The true FP64 residual of the FP32 iterate carries the FP32 rounding of s
    # times ||H0|| ~ beta0 |k_max|^4 (1.1e4 here): about 1.3e-3 of ||r|| on top
    # of the tolerance, which is what FP32 vectors can attain.
    s, it = P.apply_invh0(to_dev(r), 1e-3, 100)
    s_ref, it_ref = ref.invh0(synth.f64(r), 1e-3, 100)
    assert abs(it - it_ref) <= 1 and it > 0
    rr = synth.f64(r)
    res = np.linalg.norm(rr - ref.h0_apply(synth.f64(to_np(s)))) / np.linalg.norm(rr)
    res_ref = np.linalg.norm(rr - ref.h0_apply(s_ref)) / np.linalg.norm(rr)
    say(f"tolerance 1e-3: {it} vs {it_ref} iterations, residual {res:.2e} vs {res_ref:.2e}")
    assert res_ref <= 1e-3 and res <= 1e-3 + 1.5e-3, res


def test_newton_step_with_invh0_matches_oracle_pcg():
    say("Newton step, PCG with InvH0")
    P, ref = _setup(shape=(32, 32, 32), nt=4, reg=2, beta=5e-4)
    P.set_preconditioner("invh0", eps_h0=1e-3, max_inner=8)
    vt, info = P.newton_step(4, 1e-12)  # fixed outer count; the inner tolerance 1e-15 leaves 8 each
    vt_ref, pinfo = ref.pcg(-ref.gradient(), 4, 1e-12, pc="invh0", eps_h0=1e-3, max_inner=8)
    assert info["pcg_iters"] == pinfo["iters"] == 4
    assert info["inner_iters"] == pinfo["inner"] == 5 * 8
    e = rel(to_np(vt), vt_ref)
    say(f"newton step rel {e:.2e}")
    assert e < 1e-5
    # InvA again on the same plan
    P.set_preconditioner("inva")
    vt2, info2 = P.newton_step(4, 1e-12)
    vt2_ref, _ = ref.pcg(-ref.gradient(), 4, 1e-12)
    e2 = rel(to_np(vt2), vt2_ref)
    say(f"newton step, InvA again: rel {e2:.2e}")
    assert info2["inner_iters"] == 0 and e2 < 1e-5


def test_invh0_cuts_outer_iterations():
    say("InvH0 vs InvA outer iterations")
    P, _ = _setup(shape=(32, 32, 32), nt=4, reg=2, beta=5e-4, disp=3.0)
    _, ia = P.newton_step(200, 1e-3)
    P.set_preconditioner("invh0", eps_h0=1e-3, max_inner=50)
    _, ih = P.newton_step(200, 1e-3)
    say(f"outer: InvA {ia['pcg_iters']}, InvH0 {ih['pcg_iters']} (+{ih['inner_iters']} inner)")
    assert ih["pcg_iters"] < ia["pcg_iters"]
    assert ih["rel_res"] <= 1e-3 and ia["rel_res"] <= 1e-3


def test_preconditioner_arguments():
    P, _ = _setup(shape=(16, 16, 16), nt=2)
    for args in [(3, 1e-3, 10), (1, 0.0, 10), (1, 1.0, 10), (1, 1e-3, 0), (-1, 1e-3, 10)]:
        with pytest.raises(LddmmError) as e:
            L.lddmm_set_preconditioner(P._h, *args)
        assert e.value.status == L.EINVAL
    s = to_dev(incremental(P.shape, 1502))
    with pytest.raises(LddmmError) as e:
        L.lddmm_apply_invh0(P._h, s, -1.0, 5, P._vector())
    assert e.value.status == L.EINVAL


def test_batch_rejects_invh0():
    shapes = [(16, 16, 16), (16, 16, 16)]
    Bt = Batch(shapes, 2, reg=2, beta=1e-3, nstreams=2)
    m0 = [to_dev(synth.f32(synth.blob_image(s, 4, 1510 + b))) for b, s in enumerate(shapes)]
    Bt.set_images(m0, m0)
    vb = [to_dev(np.zeros((3,) + s, np.float32)) for s in shapes]
    Bt.set_velocity(vb)
    L.lddmm_set_preconditioner(L.lddmm_batch_plan(Bt._h, 1), 1, 1e-3, 10)
    with pytest.raises(LddmmError) as e:
        Bt.gn_iterate(vb, 2, 0.0)
    assert e.value.status == L.EUNSUPPORTED
    Bt.close()


def test_two_level_matches_oracle():
    say("2LInvH0 step")
    P, ref = _setup(shape=(32, 24, 40), nt=3, reg=2, beta=1e-3)
    r = incremental(P.shape, 1520)
    s, it = P.apply_2linvh0(to_dev(r), 0.0, 6)
    s_ref, it_ref = ref.two_level_invh0(synth.f64(r), 0.0, 6)
    assert it == it_ref == 6
    e = rel(to_np(s), s_ref)
    say(f"2L, 6 coarse iterations: rel {e:.2e}")
    assert e < 1e-5
    # the coarse restriction of grad m(1) follows a new velocity
    v2 = to_dev(synth.f32(0.5 * synth.bandlimited_vector(P.shape, 3, 1521, max_disp=2.0)))
    P.set_velocity(v2)
    ref.set_velocity(synth.f64(to_np(v2)))
    s, _ = P.apply_2linvh0(to_dev(r), 0.0, 6)
    s_ref, _ = ref.two_level_invh0(synth.f64(r), 0.0, 6)
    e = rel(to_np(s), s_ref)
    say(f"2L after a new velocity: rel {e:.2e}")
    assert e < 1e-5


def test_newton_step_with_two_level_matches_oracle_pcg():
    say("Newton step, PCG with 2LInvH0")
    P, ref = _setup(shape=(32, 32, 32), nt=4, reg=2, beta=5e-4)
    P.set_preconditioner("2linvh0", eps_h0=1e-3, max_inner=8)
    vt, info = P.newton_step(4, 1e-12)
    vt_ref, pinfo = ref.pcg(-ref.gradient(), 4, 1e-12, pc="2linvh0", eps_h0=1e-3, max_inner=8)
    assert info["pcg_iters"] == pinfo["iters"] == 4
    assert info["inner_iters"] == pinfo["inner"] == 5 * 8
    e = rel(to_np(vt), vt_ref)
    say(f"newton step (2L) rel {e:.2e}")
    assert e < 1e-5


def test_two_level_needs_a_halving_grid():
    P, _ = _setup(shape=(24, 20, 30), nt=2)
    with pytest.raises(LddmmError) as e:
        P.set_preconditioner("2linvh0")
    assert e.value.status == L.EINVAL
    with pytest.raises(LddmmError) as e:
        P.apply_2linvh0(to_dev(incremental(P.shape, 1530)), 0.0, 2)
    assert e.value.status == L.EINVAL


def test_two_level_after_set_beta_matches_oracle():
    """The half-grid H0 and (beta0 A_c)^{-1} follow a beta change of the fine
    plan: the coarse plan, created at beta = 0.2 (beta0 = 0.2), must use
    beta0 = 5e-2 after set_beta(1e-3), as the fine (beta0 A)^{-1} does."""
    say("2LInvH0 after set_beta")
    P, ref = _setup(shape=(32, 24, 40), nt=3, reg=2, beta=0.2)
    r = incremental(P.shape, 1540)
    s, _ = P.apply_2linvh0(to_dev(r), 0.0, 6)  # creates the half-grid plan at beta 0.2
    s_ref, _ = ref.two_level_invh0(synth.f64(r), 0.0, 6)
    e0 = rel(to_np(s), s_ref)
    P.set_beta(1e-3)
    ref.set_beta(1e-3)
    s, it = P.apply_2linvh0(to_dev(r), 0.0, 6)
    s_ref, it_ref = ref.two_level_invh0(synth.f64(r), 0.0, 6)
    e1 = rel(to_np(s), s_ref)
    say(f"2L beta 0.2: rel {e0:.2e}; after set_beta(1e-3): rel {e1:.2e}")
    assert it == it_ref == 6
    assert e0 < 1e-5 and e1 < 1e-5


@pytest.mark.parametrize("shape,two_level", [((16, 12, 128), False), ((32, 24, 256), True)])
def test_fused_rank_one_rows_match_oracle(shape, two_level):
    """x3 lengths with a register row plan (n3 = 128 on the grid the inner
    PCG runs on): the rank-one part of H0 goes back and forth along x3 in one
    kernel, without its physical fields in HBM; 6 inner iterations against
    the oracle, then a Newton step whose PCG uses the preconditioner."""
    say(f"fused x3 rank-one rows, {shape}, two-level {two_level}")
    P, ref = _setup(shape=shape, nt=2, reg=2, beta=1e-3)
    r = incremental(P.shape, 1550)
    if two_level:
        s, it = P.apply_2linvh0(to_dev(r), 0.0, 6)
        s_ref, it_ref = ref.two_level_invh0(synth.f64(r), 0.0, 6)
    else:
        s, it = P.apply_invh0(to_dev(r), 0.0, 6)
        s_ref, it_ref = ref.invh0(synth.f64(r), 0.0, 6)
    assert it == it_ref == 6
    e = rel(to_np(s), s_ref)
    pc = "2linvh0" if two_level else "invh0"
    P.set_preconditioner(pc, eps_h0=1e-3, max_inner=5)
    vt, info = P.newton_step(3, 1e-12)
    vt_ref, pinfo = ref.pcg(-ref.gradient(), 3, 1e-12, pc=pc, eps_h0=1e-3, max_inner=5)
    e2 = rel(to_np(vt), vt_ref)
    say(f"  6 inner iterations rel {e:.2e}; Newton step ({pc}) rel {e2:.2e}")
    assert info["pcg_iters"] == pinfo["iters"] == 3 and info["inner_iters"] == pinfo["inner"]
    assert e < 1e-5 and e2 < 1e-5
