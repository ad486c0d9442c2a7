"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (autotuned FFT tiles and gather strategy):

* 256^3, N_t = 4, H2 seminorm beta = 5e-4, Leray on, 120-blob images and a
  band-limited velocity of about 3 voxels: the reduced gradient and one
  Gauss-Newton Hessian matvec against the FP64 oracle over the whole grid
  (rel-L2 <= 1e-5), and the interpolation of a field at the state departure
  points against the oracle's direct 64-term sum on sampled points;
* 512^3, N_t = 8, the differentiable transport: a constant velocity that
  moves every point by a whole number of voxels per step makes the forward
  map an exact periodic roll and its adjoint the opposite roll (the
  divergence vanishes), which holds at any size (up to the rounding of the
  FP32 velocity)."""
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

N256 = (256, 256, 256)


def _bench_inputs(n, seed=3000):
    m0 = synth.f32(synth.blob_image(n, 120, seed))
    m1 = synth.f32(synth.blob_image(n, 120, seed + 2))
    v = synth.f32(0.5 * synth.bandlimited_vector(n, 8, seed + 1, max_disp=6.0))
    vt = synth.f32(synth.unit_rms(synth.bandlimited_vector(n, 8, seed + 100)))
    return m0, m1, v, vt


@pytest.mark.timeout(900)
def test_gradient_and_matvec_256_match_oracle():
    say("256^3 gradient/matvec vs oracle: inputs")
    m0, m1, v, vt = _bench_inputs(N256)
    P = Plan(N256, 4, reg=2, beta=5e-4, leray=True)
    P.autotune()
    P.set_images(to_dev(m0), to_dev(m1))
    P.set_velocity(to_dev(v))
    P.autotune()  # gather strategy on the real displacement field, as timed
    g, _ = P.gradient()
    hv = P.hessian_matvec(to_dev(vt))
    g, hv = to_np(g), to_np(hv)
    say("256^3: oracle")
    ref = oracle.Problem(N256, 4, reg=2, beta=5e-4, leray=True)
    ref.set_images(synth.f64(m0), synth.f64(m1))
    ref.set_velocity(synth.f64(v))
    eg = rel(g, ref.gradient())
    eh = rel(hv, ref.matvec(synth.f64(vt)))
    say(f"256^3: gradient rel {eg:.2e}, matvec rel {eh:.2e}")
    assert eg < 1e-5 and eh < 1e-5


@pytest.mark.timeout(600)
def test_interp_256_sampled_points_match_direct_sum():
    say("256^3 interpolation at departure points, sampled")
    m0, m1, v, _ = _bench_inputs(N256)
    P = Plan(N256, 4, reg=2, beta=5e-4, leray=True)
    P.set_images(to_dev(m0), to_dev(m1))
    P.set_velocity(to_dev(v))
    P.autotune()
    disp_d = P.get_field(L.FIELD_DISP)  # voxel displacements of X, as stored
    got = to_np(P.interp(to_dev(m1), disp_d))
    disp = to_np(disp_d)
    rng = np.random.default_rng(7)
    idx = rng.integers(0, 256, size=(4096, 3))
    idx[:64, 0] = 0                   # faces and edges: the periodic wrap
    idx[64:128, 1] = 255
    idx[128:192, 2] = 255
    idx[192:256, 2] = 0
    h = 2 * np.pi / 256
    y = (idx.T + disp[:, idx[:, 0], idx[:, 1], idx[:, 2]]) * h
    want = oracle.interp(synth.f64(m1), y)
    err = np.abs(got[idx[:, 0], idx[:, 1], idx[:, 2]] - want)
    assert err.max() <= 1e-5 * np.abs(m1).max()


@pytest.mark.timeout(600)
def test_transport_512_integer_shift_is_exact_roll():
    n, nt = (512, 512, 512), 8
    say("512^3 autograd transport, integer shifts")
    s = (1, -2, 3)  # voxels per time step along x1, x2, x3
    h = 2 * np.pi / 512
    v = torch.empty((3,) + n, device=DEV)
    for c in range(3):
        v[c].fill_(s[c] * h * nt)  # c dt = s h
    m0 = torch.from_numpy(synth.f32(synth.blob_image((64, 64, 64), 12, 77))).to(DEV)
    m0 = m0.repeat(8, 8, 8).contiguous()
    T = TransportMap(n, nt, reg=2, beta=1e-4, device=DEV)
    m0r = m0.clone().requires_grad_(True)
    vr = v.clone().requires_grad_(True)
    mt = T(m0r, vr)
    shift = tuple(nt * sc for sc in s)
    # the FP32 velocity makes each step an integer shift up to rounding: the
    # interpolation weights are those of t = 0 within ~1e-7
    assert rel(to_np(mt), to_np(torch.roll(m0, shifts=shift, dims=(0, 1, 2)))) < 1e-6
    w = torch.roll(m0, shifts=(5, 0, -7), dims=(0, 1, 2))
    (mt * w).sum().backward()
    assert rel(to_np(m0r.grad), to_np(torch.roll(w, shifts=tuple(-a for a in shift), dims=(0, 1, 2)))) < 1e-6
