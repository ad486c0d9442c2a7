"""GPU parity of the reduced gradient, objective, Gauss-Newton Hessian matvec,
PCG Newton step, Gauss-Newton iteration and transport VJP against the FP64
oracle on identical float32 inputs (rel-L2 <= 1e-5), plus edge cases."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, incremental, problem, rel, say, to_dev, to_np
from paper_2008_12820_amd import ENOTCONV, ESTATE, LddmmError, Plan
from paper_2008_12820_amd import _lib as L

pytestmark = pytest.mark.gpu

CASES = [
    # shape, nt, reg, beta, leray
    ((32, 32, 32), 4, 1, 1e-2, False),   # the 32^3 parity problem (H1 seminorm)
    ((32, 32, 32), 4, 2, 5e-4, True),
    ((24, 20, 30), 3, 2, 1e-3, False),   # ragged, radix 3 and 5
    ((48, 40, 36), 2, 1, 5e-2, True),
    ((16, 16, 16), 1, 2, 1e-2, False),   # a single time step
    ((24, 20, 30), 8, 2, 1e-3, True),    # N_t = 8: the other fused-epilogue instantiation
    ((64, 20, 24), 2, 2, 1e-3, True),    # x1 length with a register pass, Leray on
]


def _plan(shape, nt, reg, beta, leray, m0, m1, v):
    P = Plan(shape, nt, reg=reg, beta=beta, leray=leray)
    P.set_images(to_dev(m0), to_dev(m1))
    P.set_velocity(to_dev(v))
    return P


@pytest.mark.parametrize("shape,nt,reg,beta,leray", CASES)
def test_gradient_objective_matvec(shape, nt, reg, beta, leray):
    say(f"gradient/matvec {shape} nt {nt} reg {reg} leray {leray}")
    m0, m1, vtrue, v, ref = problem(shape, nt, reg, beta, leray, disp=2.0)
    P = _plan(shape, nt, reg, beta, leray, m0, m1, v)
    J, mis, rg = P.objective()
    Jr, misr, rgr = ref.objective()
    assert abs(mis - misr) / misr < 1e-5 and abs(rg - rgr) / rgr < 1e-5
    g, gn = P.gradient()
    g_ref = ref.gradient()
    eg = rel(to_np(g), g_ref)
    say(f"  gradient rel {eg:.2e}")
    assert eg < 1e-5
    assert abs(gn - np.sqrt(oracle.inner(g_ref, g_ref, ref.h3))) / gn < 1e-5
    for seed in (1100, 1101):
        vt = incremental(shape, seed)
        hv = to_np(P.hessian_matvec(to_dev(vt)))
        eh = rel(hv, ref.matvec(synth.f64(vt)))
        say(f"  matvec rel {eh:.2e}")
        assert eh < 1e-5, seed
        mt_ref = ref.inc_state(synth.f64(vt))[-1]
        assert rel(to_np(P.get_field(L.FIELD_INC_STATE)), mt_ref) < 1e-5


def test_matvec_at_zero_velocity_and_deterministic():
    shape, nt = (32, 32, 32), 4
    say("matvec v=0 closed form / determinism")
    m0, m1, vtrue, v, ref = problem(shape, nt, 1, 1e-2)
    zero = np.zeros((3,) + shape, np.float32)
    P = _plan(shape, nt, 1, 1e-2, False, m0, m1, zero)
    ref.set_velocity(synth.f64(zero))
    vt = incremental(shape, 1100)
    a = to_np(P.hessian_matvec(to_dev(vt)))
    b = to_np(P.hessian_matvec(to_dev(vt)))
    assert np.array_equal(a, b)  # bitwise run-to-run determinism
    gm0 = oracle.spectral_grad(synth.f64(m0))
    closed = 1e-2 * oracle.reg_apply(synth.f64(vt), 1) + (synth.f64(vt) * gm0).sum(0) * gm0
    assert rel(a, closed) < 1e-5
    assert rel(a, ref.matvec(synth.f64(vt))) < 1e-5


def test_inv_reg_and_newton_step_match_oracle_pcg():
    shape, nt = (32, 32, 32), 4
    say("newton step 10 PCG")
    m0, m1, vtrue, v, ref = problem(shape, nt, 2, 5e-4, disp=2.0, nblobs=12)
    P = _plan(shape, nt, 2, 5e-4, False, m0, m1, v)
    r = incremental(shape, 1200)
    assert rel(to_np(P.apply_inv_reg(to_dev(r))), oracle.reg_inverse(synth.f64(r), 2, 5e-4)) < 1e-5
    vt, info = P.newton_step(10, 1e-12)  # fixed iteration count
    g_ref = ref.gradient()
    vt_ref, pinfo = ref.pcg(-g_ref, 10, 1e-12)
    assert info["pcg_iters"] == pinfo["iters"] == 10
    e = rel(to_np(vt), vt_ref)
    say(f"  10-iteration Newton step rel {e:.2e}, rel_res {info['rel_res']:.6e} vs {pinfo['rel_res']:.6e}")
    assert e < 1e-5
    assert abs(info["rel_res"] - pinfo["rel_res"]) < 1e-3 * max(pinfo["rel_res"], 1e-3)


@pytest.mark.parametrize("shape,leray", [((30, 12, 20), True), ((20, 18, 10), False), ((64, 20, 24), True)])
def test_spectral_pcg_on_mixed_grids(shape, leray):
    """The spectral-domain PCG on grids with radix-3 and -5 transforms and
    x3 lengths whose half (n3/2 = 10, 5) is odd, where the Hermitian weights
    of the inner products sit on the planes k3 = 0 and k3 = n3/2 of short
    rows, and on an x1 length with a register pass (the fused p update and
    inverse x1 pass): a 6-iteration Newton step against the oracle's FP64
    PCG."""
    nt, reg, beta = 2, 2, 1e-3
    say(f"spectral PCG {shape} leray {leray}")
    m0, m1, vtrue, v, ref = problem(shape, nt, reg, beta, leray, disp=2.0)
    P = _plan(shape, nt, reg, beta, leray, m0, m1, v)
    vt, info = P.newton_step(6, 1e-12)
    vt_ref, pinfo = ref.pcg(-ref.gradient(), 6, 1e-12)
    e = rel(to_np(vt), vt_ref)
    say(f"  6-iteration Newton step rel {e:.2e}, rel_res {info['rel_res']:.6e} vs {pinfo['rel_res']:.6e}")
    assert info["pcg_iters"] == pinfo["iters"] == 6
    assert e < 1e-5


@pytest.mark.parametrize("leray", [True, False])
def test_overlapped_assembly_is_bitwise_the_same(leray):
    """With overlap on, the forward transform of the assembly's first operand
    (without the Leray projection: the whole of A v) runs on the plan's side
    stream beside the transport sweeps; gradient and matvec keep every bit,
    call after call."""
    shape, nt = (64, 24, 40), 3  # n1 = 64: the register-pass assembly
    say(f"overlap on/off, leray {leray}")
    m0, m1, vtrue, v, _ = problem(shape, nt, 2, 1e-3, disp=2.0)
    P = _plan(shape, nt, 2, 1e-3, leray, m0, m1, v)
    vt = to_dev(incremental(shape, 1400))
    g0, _ = P.gradient()
    h0 = P.hessian_matvec(vt)
    g0, h0 = to_np(g0), to_np(h0)
    P.set_overlap(True)
    for _ in range(3):
        g1, _ = P.gradient()
        h1 = P.hessian_matvec(vt)
        assert np.array_equal(to_np(g1), g0) and np.array_equal(to_np(h1), h0)
    P.set_overlap(False)
    assert np.array_equal(to_np(P.hessian_matvec(vt)), h0)


def test_gn_iterate_matches_oracle():
    shape, nt = (24, 24, 24), 4
    say("gn iterate")
    m0, m1, vtrue, v, ref = problem(shape, nt, 2, 1e-3, disp=2.0, vscale=0.0)
    P = _plan(shape, nt, 2, 1e-3, False, m0, m1, v)
    vd = to_dev(v)
    info = P.gn_iterate(vd, 5, 0.0)
    v_ref, rinfo = ref.gn_iterate(5, 0.0)
    assert info["alpha"] == rinfo["alpha"] and info["alpha"] > 0
    assert abs(info["J_after"] - rinfo["J_after"]) / rinfo["J_after"] < 1e-5
    e = rel(to_np(vd), v_ref)
    say(f"  GN iterate velocity rel {e:.2e}")
    assert e < 1e-5
    assert abs(P.objective()[0] - info["J_after"]) <= 1e-6 * info["J_after"]


@pytest.mark.parametrize("shape,nt", [((32, 32, 32), 4), ((20, 24, 16), 3)])
def test_transport_and_vjp_match_oracle(shape, nt):
    say(f"transport/vjp {shape} nt {nt}")
    m0, m1, vtrue, v, ref = problem(shape, nt, disp=2.0)
    P = Plan(shape, nt)
    ck = torch.empty((nt + 1,) + shape, device=DEV)
    m1g = to_np(P.transport_forward(to_dev(m0), to_dev(v), ck))
    mref = ref.transport(synth.f64(m0))
    assert rel(m1g, mref[-1]) < 1e-6
    assert rel(to_np(ck), mref) < 1e-6
    gout = synth.f32(synth.bandlimited_scalar(shape, 3, 77))
    gm0, gv = P.transport_vjp(ck, to_dev(v), to_dev(gout))
    gm0_ref, gv_ref = ref.transport_vjp(synth.f64(m0), synth.f64(gout))
    assert rel(to_np(gm0), gm0_ref) < 1e-5
    assert rel(to_np(gv), gv_ref) < 1e-5


def test_state_errors():
    shape = (16, 16, 16)
    P = Plan(shape, 2)
    vt = to_dev(np.zeros((3,) + shape, np.float32))
    with pytest.raises(LddmmError) as e:
        P.hessian_matvec(vt)
    assert e.value.status == ESTATE
    with pytest.raises(LddmmError):
        P.gradient()


def test_pcg_spectra_and_their_physical_images():
    """The PCG keeps r and p as spectra: before any PCG they cannot be read
    (ESTATE); after one, the residual field is the inverse transform of the
    residual spectrum, z that of (beta A)^{-1} r, and the search direction
    field the inverse transform of p's spectrum (all within FP32 transform
    rounding); ||r|| / ||r0|| of the history is that of these spectra."""
    shape, nt, reg, beta = (24, 20, 30), 2, 2, 1e-3
    say("PCG spectra and physical images")
    m0, m1, vtrue, v, ref = problem(shape, nt, reg, beta, False, disp=2.0)
    P = _plan(shape, nt, reg, beta, False, m0, m1, v)
    for f in (L.FIELD_PCG_R_HAT, L.FIELD_PCG_P_HAT, L.FIELD_PCG_R):
        with pytest.raises(LddmmError) as e:
            P.get_field(f)
        assert e.value.status == ESTATE
    g, _ = P.gradient()
    g0 = np.linalg.norm(to_np(g))
    P.newton_step(3, 1e-30)
    hats = [P.get_field(f).cpu().numpy().astype(np.complex128) for f in (L.FIELD_PCG_R_HAT, L.FIELD_PCG_P_HAT)]
    r_hat, p_hat = (np.fft.irfftn(h, s=shape, axes=(1, 2, 3)) for h in hats)
    r, z, p = (to_np(P.get_field(f)) for f in (L.FIELD_PCG_R, L.FIELD_PCG_Z, L.FIELD_PCG_P))
    er, ep = rel(r, r_hat), rel(p, p_hat)
    ez = rel(z, oracle.reg_inverse(r_hat, reg, beta))
    hist = P.pcg_history()
    eh = abs(np.linalg.norm(r_hat) / g0 - hist[-1]) / hist[-1]
    say(f"  r {er:.2e}, z {ez:.2e}, p {ep:.2e}, history {eh:.2e}")
    assert er < 1e-6 and ez < 1e-6 and ep < 1e-6 and eh < 1e-6


def test_pcg_stops_on_its_tolerance_mid_stream():
    """The PCG's stop test is read one iteration late and the iterations
    queued after a stop skip their vector kernels: a solve that meets its
    tolerance after k of at most 20 iterations must return the oracle's x_k
    (iteration count, x and relative residual), and a second solve on the same
    plan (its stop flag reset) must give the same result bitwise."""
    shape, nt, reg, beta = (24, 20, 30), 2, 2, 1e-3
    say("PCG stop on the tolerance, mid-stream")
    m0, m1, vtrue, v, ref = problem(shape, nt, reg, beta, True, disp=2.0)
    g_ref = ref.gradient()
    _, _, hist = ref.pcg_history(-g_ref, 10, 1e-30)
    # a tolerance between the residuals after iterations 5 and 6, clear of both
    k = next(i for i in range(4, 9) if hist[i - 1] / hist[i] > 1.05)
    rtol = float(np.sqrt(hist[k - 1] * hist[k]))
    x_ref, info_ref = ref.pcg(-g_ref, 20, rtol)
    assert info_ref["iters"] == k + 1
    P = _plan(shape, nt, reg, beta, True, m0, m1, v)
    vt, info = P.newton_step(20, rtol)
    x1 = to_np(vt).copy()
    e = rel(x1, x_ref)
    say(f"  stop after {info['pcg_iters']} (oracle {info_ref['iters']}) of 20, rtol {rtol:.3e}: x rel {e:.2e}, "
        f"rel_res {info['rel_res']:.4e} vs {info_ref['rel_res']:.4e}")
    assert info["pcg_iters"] == info_ref["iters"] and e < 1e-5
    assert abs(info["rel_res"] - info_ref["rel_res"]) / info_ref["rel_res"] < 1e-5
    vt2, info2 = P.newton_step(20, rtol)
    assert info2["pcg_iters"] == info["pcg_iters"] and np.array_equal(to_np(vt2), x1)


def test_negative_curvature_is_reported():
    """With the Leray projection the matvec is beta A v~ + P b~, and for a
    first search direction p = (beta A)^{-1}(-g) that is mostly curl free
    (P removes that part from b~ but not from beta A p), <p, H p> can be
    negative: here v is a gradient field, m1 the template transported by
    1.001 v, beta = 1e-4.  The oracle's first curvature is negative (cosine
    about -0.14, far beyond FP32 round-off); the GPU PCG must stop with flag 1
    and return M^{-1} r0, as the oracle does."""
    shape, nt, beta = (16, 16, 16), 2, 1e-4
    say("non-positive curvature")
    m0 = synth.f32(synth.blob_image(shape, 4, 7001))
    phi = synth.bandlimited_vector(shape, 2, 7201, max_disp=1.0)[0]
    v = oracle.spectral_grad(phi)
    v = synth.f32(v / np.abs(v).max() * (2 * np.pi / 16))
    ref = oracle.Problem(shape, nt, reg=1, beta=beta, leray=True)
    ref.set_images(synth.f64(m0), synth.f64(m0))
    ref.set_velocity(1.001 * synth.f64(v))
    m1 = synth.f32(ref.transport(synth.f64(m0))[-1])
    ref.set_images(synth.f64(m0), synth.f64(m1))
    ref.set_velocity(synth.f64(v))
    g_ref = ref.gradient()
    p = oracle.reg_inverse(-g_ref, 1, beta)
    hp = ref.matvec(p)
    cos = oracle.inner(p, hp, ref.h3) / np.sqrt(oracle.inner(p, p, ref.h3) * oracle.inner(hp, hp, ref.h3))
    x_ref, rinfo = ref.pcg(-g_ref, 5, 1e-12)
    say(f"  oracle: first curvature cosine {cos:.3f}, flags {rinfo['flags']}, iterations {rinfo['iters']}")
    assert cos < -0.1 and rinfo["flags"] == 1 and rinfo["iters"] == 1
    P = _plan(shape, nt, 1, beta, True, m0, m1, v)
    vt, info = P.newton_step(5, 1e-12, allow_notconv=True)
    g, _ = P.gradient()
    own = to_np(P.apply_inv_reg(-g))
    e_own = rel(to_np(vt), own)
    e = rel(to_np(vt), x_ref)
    # the residual m1 - m(1) is 1e-3 of the image here, so the FP32 rounding
    # of m(1) alone moves g (and M^{-1} r0) by about 6e-5 relative
    mN = ref.transport(synth.f64(m0))[-1]
    c_r = np.linalg.norm(mN) / np.linalg.norm(synth.f64(m1) - mN)
    say(f"  GPU: status {info['status']}, flags {info['flags']}, iterations {info['pcg_iters']}, "
        f"vs its own M^-1 r0 {e_own:.2e}, vs the oracle's {e:.2e} (||m(1)|| / ||m1 - m(1)|| = {c_r:.0f})")
    assert info["status"] == ENOTCONV and info["flags"] == 1 and info["pcg_iters"] == 1
    assert e_own < 1e-6
    assert e < 1e-7 * c_r


def test_non_finite_value_is_reported():
    """A non-finite velocity: PCG reports flag 2."""
    shape = (16, 16, 16)
    m0 = np.zeros(shape, np.float32)
    P = Plan(shape, 2, beta=1e-2)
    P.set_images(to_dev(m0), to_dev(m0 + 1))
    v = np.zeros((3,) + shape, np.float32)
    v[0, 3, 4, 5] = np.nan
    P.set_velocity(to_dev(v))
    vt, info = P.newton_step(3, 0.0, allow_notconv=True)
    assert info["status"] == ENOTCONV and info["flags"] & 2


@pytest.mark.parametrize("shape", [(32, 32, 32), (40, 36, 96)])
def test_gather_strategies_agree(shape):
    """Direct, LDS-staged box gathers (both tile shapes) and their pipelined
    persistent forms compute the stencil sum with the same fused multiply-adds
    in the same order: the matvec is bitwise the same for every strategy and
    matches the oracle."""
    say(f"gather strategies {shape}")
    nt = 3
    m0, m1, vtrue, v, ref = problem(shape, nt, 2, 1e-3, disp=3.0)
    P = _plan(shape, nt, 2, 1e-3, False, m0, m1, v)
    vt = incremental(shape, 1300)
    ref_hv = ref.matvec(synth.f64(vt))
    outs = []
    for mode in (0, 1, 2, 3, 4):
        P.set_gather_mode(mode)
        P.set_velocity(to_dev(v))
        outs.append(to_np(P.hessian_matvec(to_dev(vt))))
        assert rel(outs[-1], ref_hv) < 1e-5, mode
    for got in outs[1:]:
        assert np.array_equal(got, outs[0])


def test_pipelined_gathers_walk_many_tiles():
    """A grid with more tiles than resident workgroups (2250 tiles of 2x4x64,
    1150 of 4x4x64, ragged along every axis and unequal over the eight
    per-XCD ranges): every workgroup of the pipelined gathers walks several
    tiles through its two LDS boxes.  Gradient and matvec are bitwise those of
    the one-tile-per-workgroup box gathers."""
    shape, nt = (90, 100, 120), 3
    say(f"pipelined gathers {shape}")
    m0 = synth.f32(synth.blob_image(shape, 40, 2100))
    m1 = synth.f32(synth.blob_image(shape, 40, 2101))
    v = synth.f32(synth.bandlimited_vector(shape, 4, 2102, max_disp=4.0))
    P = _plan(shape, nt, 2, 1e-3, True, m0, m1, v)
    vt = incremental(shape, 1301)
    res = {}
    for mode in (1, 2, 3, 4):
        P.set_gather_mode(mode)
        P.set_velocity(to_dev(v))
        g, _ = P.gradient()
        res[mode] = (to_np(g), to_np(P.hessian_matvec(to_dev(vt))))
    for a, b in ((1, 3), (2, 4), (1, 2)):
        assert np.array_equal(res[a][0], res[b][0]), (a, b)
        assert np.array_equal(res[a][1], res[b][1]), (a, b)
    assert np.isfinite(res[3][1]).all() and np.abs(res[3][1]).max() > 0


def test_workspace_beyond_device_memory_is_enomem():
    """A plan whose workspace cannot fit in HBM (1024^3, N_t = 256: about
    10 TB) fails with ENOMEM and leaves the device usable."""
    cfg = L.make_config((1024, 1024, 1024), 256, L.REG_H2S, 1e-3)
    need = L.lddmm_workspace_bytes(cfg)
    free, total = torch.cuda.mem_get_info(DEV)
    say(f"ENOMEM: workspace {need / 1e12:.1f} TB, device {total / 1e9:.0f} GB")
    assert need > total
    with pytest.raises(LddmmError) as e:
        L.lddmm_plan_create(cfg, torch.cuda.current_stream(DEV).cuda_stream)
    assert e.value.status == L.ENOMEM
    # the device still works: a small plan runs a matvec
    shape = (16, 16, 16)
    m0, m1, vtrue, v, ref = problem(shape, 2, 1, 1e-2)
    P = _plan(shape, 2, 1, 1e-2, False, m0, m1, v)
    vt = incremental(shape, 1600)
    assert rel(to_np(P.hessian_matvec(to_dev(vt))), ref.matvec(synth.f64(vt))) < 1e-5
    P.close()
