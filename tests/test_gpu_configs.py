"""GPU parity on the workloads the scope names beside the 32^3 problem:

* 128^3 Gauss-Newton (H2 seminorm beta = 5e-4, N_t = 4, 40-blob template, its
  image under a divergence-free band-limited velocity |k| <= 6 of about 4
  voxels, 10 PCG iterations with (beta A)^{-1}), Leray projection off and on:
  the reduced gradient and a Hessian matvec at v = 0 and after one
  Gauss-Newton iteration, each PCG iteration checked on its own (the oracle
  takes the GPU's PCG state after k - 1 iterations and performs iteration k),
  the whole 10-iteration Newton step and its residual history;
* 256^3 with N_t = 8 (the benchmark's second case): gradient and matvec over
  the whole grid;
* the differentiable transport at 128^3 (N_t = 8) against the oracle's
  gradient, and at 512^3 with a smooth non-integer divergence-free velocity,
  where every step of the forward map and of its adjoint is checked at 4096
  sampled points against the oracle's departure points and interpolation,
  the VJP's body force against its definition, and the checkpoint gradients
  against the exact identity sum_x G_d sin(k.x) = -k_d sum_x m cos(k.x) of
  the spectral derivative."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, rel, say, to_dev, to_np
from paper_2008_12820_amd import Plan
from paper_2008_12820_amd import _lib as L
from paper_2008_12820_amd.autograd import TransportMap

pytestmark = pytest.mark.gpu

N128 = (128, 128, 128)


def _config2(leray):
    m0 = synth.f32(synth.blob_image(N128, 40, 2000))
    vtrue = synth.f32(synth.bandlimited_vector(N128, 6, 2001, max_disp=4.0, divfree=True))
    ref = oracle.Problem(N128, 4, reg=2, beta=5e-4, leray=leray)
    ref.set_images(synth.f64(m0), synth.f64(m0))
    ref.set_velocity(synth.f64(vtrue))
    m1 = synth.f32(ref.transport(synth.f64(m0))[-1])
    ref.set_images(synth.f64(m0), synth.f64(m1))
    return m0, m1, ref


def _pcg_state(P, shape):
    """the GPU PCG's residual and search direction: their FP32 spectra
    (unnormalised half spectra), transformed back in FP64"""
    out = []
    for f in (L.FIELD_PCG_R_HAT, L.FIELD_PCG_P_HAT):
        hat = P.get_field(f).cpu().numpy().astype(np.complex128)
        out.append(np.fft.irfftn(hat, s=shape, axes=(1, 2, 3)))
    return out


def _pcg_step_check(P, ref, k):
    """iteration k of PCG from the GPU's state after k - 1 iterations, by
    the oracle's matvec and (beta A)^{-1}, against the GPU's iteration k.
    The GPU keeps r and p as FP32 spectra; the oracle takes them exactly
    (transformed back in FP64), so its matvec sees the GPU's own p and not
    an FP32 rounding of it that beta A would amplify at high |k|."""
    shape = P.shape
    x0, _ = P.newton_step(k - 1, 1e-30)
    x0 = to_np(x0)
    r, p = _pcg_state(P, shape)
    z = oracle.reg_inverse(r, ref.reg, ref.beta)
    xk, _ = P.newton_step(k, 1e-30)
    xk = to_np(xk)
    rk, pk = _pcg_state(P, shape)
    q = ref.matvec(p)
    rz = oracle.inner(r, z, ref.h3)
    alpha = rz / oracle.inner(p, q, ref.h3)
    x_or = x0 + alpha * p
    r_or = r - alpha * q
    z_or = oracle.reg_inverse(r_or, ref.reg, ref.beta)
    p_or = z_or + (oracle.inner(r_or, z_or, ref.h3) / rz) * p
    return rel(xk, x_or), rel(rk, r_or), rel(pk, p_or), rk


@pytest.mark.timeout(900)
@pytest.mark.parametrize("leray", [False, True])
def test_config2_128_gauss_newton(leray):
    say(f"128^3 Gauss-Newton, Leray {leray}: inputs")
    m0, m1, ref = _config2(leray)
    P = Plan(N128, 4, reg=2, beta=5e-4, leray=leray)
    P.autotune()
    P.set_images(to_dev(m0), to_dev(m1))
    zero = np.zeros((3,) + N128, np.float32)
    P.set_velocity(to_dev(zero))
    P.autotune()
    ref.set_velocity(synth.f64(zero))
    vt = synth.f32(synth.unit_rms(synth.bandlimited_vector(N128, 6, 2100)))
    g, _ = P.gradient()
    eg = rel(to_np(g), ref.gradient())
    eh = rel(to_np(P.hessian_matvec(to_dev(vt))), ref.matvec(synth.f64(vt)))
    say(f"  v = 0: gradient rel {eg:.2e}, matvec rel {eh:.2e}")
    assert eg < 1e-5 and eh < 1e-5
    # every PCG iteration on its own, from the GPU's state
    rnorm = {0: np.linalg.norm(to_np(g))}
    for k in (1, 2, 5, 10):
        ex, er, ep, rk = _pcg_step_check(P, ref, k)
        rnorm[k] = np.linalg.norm(rk)
        say(f"  PCG iteration {k} from the GPU state: x {ex:.2e}, r {er:.2e}, p {ep:.2e}")
        assert ex < 1e-5 and er < 1e-5 and ep < 1e-5, k
    # the whole first Newton step and its residual history
    vt10, info = P.newton_step(10, 1e-30)
    hist = P.pcg_history()
    vt_ref, rinfo, hist_ref = ref.pcg_history(-ref.gradient(), 10, 1e-30)
    e10 = rel(to_np(vt10), vt_ref)
    dh = max(abs(a - b) / b for a, b in zip(hist, hist_ref))
    say(f"  10-iteration step rel {e10:.2e}; history {['%.4e' % h for h in hist]}; "
        f"oracle {['%.4e' % h for h in hist_ref]}; max rel diff {dh:.2e}")
    assert info["pcg_iters"] == rinfo["iters"] == 10 and len(hist) == 10
    assert e10 < 1e-5
    # the history is ||r_k|| / ||r_0|| of the GPU's own residuals
    for k in (1, 2, 5, 10):
        assert abs(hist[k - 1] - rnorm[k] / rnorm[0]) <= 1e-6 * hist[k - 1], k
    # Against the FP64 history: r and p are kept as spectra, so p carries no
    # white transform error for beta |k|^4 to amplify at high |k| in the next
    # matvec (a physical-space FP32 loop moves this history by 6.8e-3 that
    # way); what remains is the FP32 rounding of each spectral coefficient
    # and of the body force's forward transform (measured <= 1.5e-7).
    assert dh < 1e-5
    # one Gauss-Newton iteration, then the gradient and a matvec at the new
    # velocity on both sides (the oracle takes the GPU's velocity)
    v = to_dev(zero)
    gi = P.gn_iterate(v, 10, 1e-30)
    say(f"  GN iteration: alpha {gi['alpha']}, J {gi['J_before']:.6e} -> {gi['J_after']:.6e}")
    assert gi["alpha"] > 0
    ref.set_velocity(synth.f64(to_np(v)))
    J, _, _ = ref.objective()
    assert abs(gi["J_after"] - J) <= 1e-5 * J
    g, _ = P.gradient()
    g_ref = ref.gradient()
    eg = rel(to_np(g), g_ref)
    eh = rel(to_np(P.hessian_matvec(to_dev(vt))), ref.matvec(synth.f64(vt)))
    # g = beta A v + K b: the FP32 rounding of each term is relative to that
    # term, so where the two cancel (here, after a Newton step) the relative
    # error of g grows by c_g = (||beta A v|| + ||K b||) / ||g|| (1 at v = 0)
    bav = 5e-4 * oracle.reg_apply(synth.f64(to_np(v)), 2)
    c_g = (np.linalg.norm(bav) + np.linalg.norm(g_ref - bav)) / np.linalg.norm(g_ref)
    say(f"  after one GN iteration: gradient rel {eg:.2e} (c_g {c_g:.2f}, bar {1e-5 * c_g:.2e}), "
        f"matvec rel {eh:.2e}")
    assert eg < 1e-5 * c_g and eh < 1e-5
    P.close()


@pytest.mark.timeout(900)
def test_gradient_and_matvec_256_nt8_match_oracle():
    n = (256, 256, 256)
    say("256^3 N_t = 8 gradient/matvec vs oracle: inputs")
    m0 = synth.f32(synth.blob_image(n, 120, 3000))
    m1 = synth.f32(synth.blob_image(n, 120, 3002))
    v = synth.f32(0.5 * synth.bandlimited_vector(n, 8, 3001, max_disp=6.0))
    vt = synth.f32(synth.unit_rms(synth.bandlimited_vector(n, 8, 3119)))  # the last timed increment's seed
    P = Plan(n, 8, reg=2, beta=5e-4, leray=True)
    P.autotune()
    P.set_images(to_dev(m0), to_dev(m1))
    P.set_velocity(to_dev(v))
    P.autotune()
    g, _ = P.gradient()
    hv = P.hessian_matvec(to_dev(vt))
    g, hv = to_np(g), to_np(hv)
    P.close()
    say("256^3 N_t = 8: oracle")
    ref = oracle.Problem(n, 8, reg=2, beta=5e-4, leray=True)
    ref.set_images(synth.f64(m0), synth.f64(m1))
    ref.set_velocity(synth.f64(v))
    eg = rel(g, ref.gradient())
    eh = rel(hv, ref.matvec(synth.f64(vt)))
    say(f"256^3 N_t = 8: gradient rel {eg:.2e}, matvec rel {eh:.2e}")
    assert eg < 1e-5 and eh < 1e-5


@pytest.mark.timeout(900)
def test_autograd_128_matches_oracle_gradient():
    shape, nt, beta = N128, 8, 1e-4
    say("autograd 128^3 N_t = 8")
    m0 = synth.f32(synth.blob_image(shape, 40, 2200))
    m1 = synth.f32(synth.blob_image(shape, 40, 2202))
    v = synth.f32(synth.bandlimited_vector(shape, 6, 2201, max_disp=4.0))
    T = TransportMap(shape, nt, reg=2, beta=beta, device=DEV)
    m0d = to_dev(m0).requires_grad_(True)
    vd = to_dev(v).requires_grad_(True)
    mt = T(m0d, vd)
    loss = 0.5 * ((mt - to_dev(m1)) ** 2).sum() + beta * T.reg_energy(vd)
    loss.backward()
    ref = oracle.Problem(shape, nt, reg=2, beta=beta)
    ref.set_images(synth.f64(m0), synth.f64(m1))
    ref.set_velocity(synth.f64(v))
    mref = ref.transport(synth.f64(m0))[-1]
    em = rel(to_np(mt), mref)
    eg = rel(to_np(vd.grad), ref.gradient())
    gm0_ref, _ = ref.transport_vjp(synth.f64(m0), mref - synth.f64(m1))
    e0 = rel(to_np(m0d.grad), gm0_ref)
    say(f"  m(1) rel {em:.2e}, dL/dv rel {eg:.2e}, dL/dm0 rel {e0:.2e}")
    assert em < 1e-6 and eg < 1e-5 and e0 < 1e-5


def _sample_points(n, count, seed):
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, nd, count) for nd in n])
    # faces and edges: the periodic wrap
    idx[0, :64] = 0
    idx[1, 64:128] = n[1] - 1
    idx[2, 128:192] = n[2] - 1
    idx[2, 192:256] = 0
    return idx


@pytest.mark.timeout(900)
def test_transport_512_smooth_velocity_sampled():
    n, nt = (512, 512, 512), 8
    say("512^3 transport and VJP, smooth divergence-free velocity: inputs")
    # a 64^3 periodic blob image tiled 8 x 8 x 8 is a periodic 512^3 image
    m0 = np.tile(synth.f32(synth.blob_image((64, 64, 64), 12, 2300)), (8, 8, 8))
    v = synth.f32(synth.bandlimited_vector(n, 8, 2301, max_disp=6.0, divfree=True))
    w = np.tile(synth.f32(synth.blob_image((64, 64, 64), 12, 2302)), (8, 8, 8))
    T = TransportMap(n, nt, reg=2, beta=1e-4, device=DEV)
    P = T.plan
    ck = torch.empty((nt + 1,) + n, device=DEV)
    m1 = P.transport_forward(to_dev(m0), to_dev(v), ck)
    gm0, gv = P.transport_vjp(ck, to_dev(v), to_dev(w))
    idx = _sample_points(n, 4096, 2303)
    at = lambda f: f[..., idx[0], idx[1], idx[2]]  # noqa: E731
    h = 2 * np.pi / 512
    say("512^3: departure points at the sampled points")
    X, Xa = oracle.departure_points(synth.f64(v), nt, idx)
    dX = at(to_np(P.get_field(L.FIELD_DISP)))
    dXa = at(to_np(P.get_field(L.FIELD_DISP_ADJ)))
    eX = max(np.abs(dX - (X / h - idx)).max(), np.abs(dXa - (Xa / h - idx)).max())
    say(f"  departure displacement max error {eX:.2e} voxels (max |d| {np.abs(dX).max():.2f})")
    assert eX < 4e-6
    say("512^3: every state step at the sampled points")
    errs = []
    for j in range(nt):
        mj = synth.f64(to_np(ck[j]))
        want = oracle.interp(mj, X)
        got = at(to_np(ck[j + 1]))
        errs.append(np.abs(got - want).max() / np.abs(mj).max())
    say(f"  state steps: max error {max(errs):.2e} of max |m|")
    assert max(errs) < 1e-5
    assert np.array_equal(to_np(m1), to_np(ck[nt]))
    say("512^3: every adjoint step at the sampled points")
    lam = [to_np(P.get_field(L.FIELD_ADJOINT, j)) for j in range(nt + 1)]
    assert rel(lam[nt], w) == 0.0
    errs = []
    for j in range(nt):
        want = oracle.interp(synth.f64(lam[j + 1]), Xa)  # div v = 0: the reaction factor is 1
        errs.append(np.abs(at(lam[j]) - want).max() / np.abs(lam[j + 1]).max())
    say(f"  adjoint steps: max error {max(errs):.2e} of max |lam|")
    assert max(errs) < 1e-5
    assert np.array_equal(to_np(gm0), lam[0])
    say("512^3: checkpoint gradients (spectral identity) and the body force")
    x = [np.arange(nd) * (2 * np.pi / nd) for nd in n]
    # modes that the tiled template carries (multiples of 8); s = sin cos cos
    # of each is band-limited, so the spectral derivative is exact on it and
    # skew-adjoint: sum G_d s = -sum m d_d s
    modes = [(8, 0, 8), (0, 8, 16), (16, -8, 0)]
    G = []
    for j in range(nt + 1):
        Gj = to_np(P.get_field(L.FIELD_GRAD_STATE, j))
        mj = to_np(ck[j])
        kv = modes[j % 3]
        f = [np.sin(kv[0] * x[0]), np.cos(kv[1] * x[1]), np.cos(kv[2] * x[2])]
        df = [kv[0] * np.cos(kv[0] * x[0]), -kv[1] * np.sin(kv[1] * x[1]), -kv[2] * np.sin(kv[2] * x[2])]
        outer = lambda a, b, c: a[:, None, None] * b[None, :, None] * c[None, None, :]  # noqa: E731
        s3 = outer(*f)
        for d in range(3):
            fd = list(f)
            fd[d] = df[d]
            lhs = float((Gj[d] * s3).sum())
            rhs = -float((mj * outer(*fd)).sum())
            tol = 1e-5 * abs(rhs) + 1e-7 * float(np.linalg.norm(Gj[d]) * np.linalg.norm(s3))
            assert abs(lhs - rhs) <= tol, (j, d, kv, lhs, rhs)
        G.append(at(Gj))
    dt = 1.0 / nt
    b = 0.0
    for j in range(nt + 1):
        wj = 0.5 if j in (0, nt) else 1.0
        b = b + wj * at(lam[j]) * G[j]
    eb = np.abs(at(to_np(gv)) + dt * b).max() / np.abs(dt * b).max()
    say(f"  body force: max error {eb:.2e}")
    assert eb < 1e-5
    P.close()
