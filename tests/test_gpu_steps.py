"""GPU parity of each step of the path against the FP64 oracle, through the
C ABI: 3D real FFT, spectral operators, cubic interpolation, departure
points, state and its gradients.  Sizes span several LDS tiles, non-power-of-
two radices (3, 5) and ragged tails; the bar is rel-L2 <= 1e-5 (FP32)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, problem, rel, say, to_dev, to_np
from paper_2008_12820_amd import OP_DIV, OP_GRAD, OP_INVREG, OP_LERAY, OP_REG, Plan

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8, 8), (16, 12, 10), (32, 32, 32), (24, 40, 20), (48, 30, 64), (96, 80, 160)]


@pytest.mark.parametrize("shape", SHAPES)
def test_fft_r2c_matches_oracle_dft(shape):
    say(f"fft r2c {shape}")
    rng = np.random.default_rng(1)
    f = rng.standard_normal(shape).astype(np.float32)
    P = Plan(shape, 1)
    got = P.fft_r2c(to_dev(f)).cpu().numpy().astype(np.complex128)
    ref = oracle.fft3(f.astype(np.float64), -1)[:, :, : shape[2] // 2 + 1]
    assert rel(got.view(float), ref.view(float)) < 1e-6
    back = to_np(P.fft_c2r(torch.from_numpy(got.astype(np.complex64)).to(DEV)))
    assert rel(back, f) < 1e-6


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("reg", [1, 2])
def test_spectral_operators(shape, reg):
    say(f"spectral ops {shape} reg {reg}")
    rng = np.random.default_rng(2)
    f = synth.f32(synth.bandlimited_scalar(shape, 4, 3) + 0.1 * rng.standard_normal(shape))
    v = synth.f32(synth.bandlimited_vector(shape, 4, 4) + 0.1 * rng.standard_normal((3,) + shape))
    beta = 3e-3
    P = Plan(shape, 1, reg=reg, beta=beta)
    fd, vd = to_dev(f), to_dev(v)
    f64, v64 = synth.f64(f), synth.f64(v)
    assert rel(to_np(P.spectral_op(OP_GRAD, fd)), oracle.spectral_grad(f64)) < 1e-5
    assert rel(to_np(P.spectral_op(OP_DIV, vd)), oracle.spectral_div(v64)) < 1e-5
    assert rel(to_np(P.spectral_op(OP_REG, vd)), oracle.reg_apply(v64, reg)) < 1e-5
    assert rel(to_np(P.spectral_op(OP_INVREG, vd)), oracle.reg_inverse(v64, reg, beta)) < 1e-5
    assert rel(to_np(P.spectral_op(OP_LERAY, vd)), oracle.leray(v64)) < 1e-5


@pytest.mark.parametrize("shape", [(16, 16, 16), (24, 20, 30), (64, 48, 40)])
def test_interp_matches_oracle(shape):
    say(f"interp {shape}")
    rng = np.random.default_rng(5)
    f = rng.standard_normal((2,) + shape).astype(np.float32)
    disp = rng.uniform(-7.5, 7.5, (3,) + shape).astype(np.float32)
    disp[:, 0, 0, 0] = [shape[0] + 0.25, -shape[1] - 0.5, 2 * shape[2] - 0.1]  # beyond one period
    # second half of the grid: a smooth displacement, so that the LDS-staged
    # strategies take their box path there and the global fallback elsewhere
    half = shape[0] // 2
    xs = np.arange(shape[0])[half:, None, None] * (2 * np.pi / shape[0])
    ys = np.arange(shape[1])[None, :, None] * (2 * np.pi / shape[1])
    zs = np.arange(shape[2])[None, None, :] * (2 * np.pi / shape[2])
    disp[0, half:] = 2.3 * np.sin(ys + zs)
    disp[1, half:] = -1.7 * np.cos(xs + zs)
    disp[2, half:] = 3.1 * np.sin(xs + ys) + 0.5
    P = Plan(shape, 1)
    x = oracle.grid_points(shape)
    h = np.array([2 * np.pi / n for n in shape]).reshape(3, 1, 1, 1)
    y = (x + h * synth.f64(disp)).reshape(3, -1)
    ref = oracle.interp(synth.f64(f), y).reshape((2,) + shape)
    outs = []
    for mode in (-1, 0, 1, 2):  # default, direct, box tiles 2x4x64 and 4x4x64
        P.set_gather_mode(mode)
        got = to_np(P.interp(to_dev(f), to_dev(disp)))
        assert rel(got, ref) < 1e-6, mode
        assert np.abs(got - ref).max() < 1e-5, mode
        outs.append(got)
    for got in outs[2:]:
        assert np.array_equal(got, outs[1])  # same fused multiply-adds in the same order


@pytest.mark.parametrize("shape,nt", [((16, 16, 16), 4), ((24, 20, 30), 3), ((32, 32, 32), 4)])
def test_velocity_state_matches_oracle(shape, nt):
    say(f"velocity state {shape} nt {nt}")
    m0, m1, vtrue, v, ref = problem(shape, nt, disp=2.0)
    P = Plan(shape, nt)
    P.set_images(to_dev(m0), to_dev(m1))
    P.set_velocity(to_dev(v))
    from paper_2008_12820_amd import _lib as L
    assert rel(to_np(P.get_field(L.FIELD_DISP)), ref.displacement("X")) < 1e-6
    assert rel(to_np(P.get_field(L.FIELD_DISP_ADJ)), ref.displacement("Xa")) < 1e-6
    for j in range(nt + 1):
        assert rel(to_np(P.get_field(L.FIELD_STATE, j)), ref.get("m", j)) < 1e-6
        assert rel(to_np(P.get_field(L.FIELD_GRAD_STATE, j)), ref.get("G", j)) < 1e-5
    assert rel(to_np(P.get_field(L.FIELD_DIV)), ref.get("delta")) < 1e-5


def test_autotune_keeps_results_bitwise():
    """Tile shapes only change how lines are grouped into workgroups, never
    the arithmetic of a line: results before and after tuning are identical."""
    shape = (48, 40, 36)
    say("autotune")
    rng = np.random.default_rng(9)
    v = to_dev(rng.standard_normal((3,) + shape).astype(np.float32))
    P = Plan(shape, 2, reg=2, beta=1e-3, leray=True)
    before = [to_np(P.spectral_op(op, v)) for op in (OP_REG, OP_INVREG, OP_LERAY)]
    rep = P.autotune()
    assert "tuned=1" in rep
    after = [to_np(P.spectral_op(op, v)) for op in (OP_REG, OP_INVREG, OP_LERAY)]
    for a, b in zip(before, after):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape,nt,disp", [((24, 20, 30), 3, 2.0), ((90, 100, 120), 1, 3.0), ((90, 100, 120), 1, 25.0)])
def test_departure_strategies_bitwise(shape, nt, disp):
    """The departure points of the RK2 characteristics (Section 3.1) from the
    direct kernel (strategy 0) and from the LDS-staged boxes of 2x4x64 and
    4x4x64 tiles (1, 2) are bitwise equal: the same FP64 sum in the same
    order.  The ragged 90x100x120 grid ends mid-tile on every axis; at a
    25-voxel field the predictor stencils of a tile spread far beyond the box
    and most points take the global-memory path."""
    from paper_2008_12820_amd import _lib as L
    say(f"departure strategies {shape} nt {nt} disp {disp}")
    v = synth.f32(synth.bandlimited_vector(shape, 4, 2200, max_disp=disp))
    P = Plan(shape, nt)
    m0 = to_dev(synth.f32(synth.blob_image(shape, 6, 2201)))
    P.set_images(m0, m0)
    out = {}
    for mode in (0, 1, 2):
        P.set_gather_mode(mode)
        P.set_velocity(to_dev(v))
        out[mode] = (to_np(P.get_field(L.FIELD_DISP)), to_np(P.get_field(L.FIELD_DISP_ADJ)))
    for mode in (1, 2):
        assert np.array_equal(out[mode][0], out[0][0]), mode
        assert np.array_equal(out[mode][1], out[0][1]), mode
    if shape == (24, 20, 30):
        ref = oracle.Problem(shape, nt)
        ref.set_images(synth.f64(to_np(m0)), synth.f64(to_np(m0)))
        ref.set_velocity(synth.f64(v))
        assert rel(out[1][0], ref.displacement("X")) < 1e-6
        assert rel(out[2][1], ref.displacement("Xa")) < 1e-6
