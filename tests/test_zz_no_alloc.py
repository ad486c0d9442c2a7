"""The transport map without device allocation (lddmm_transport_forward_static)
against the plan entry point lddmm_transport_forward, through the C ABI: two
calls in a row, the second on a smaller grid, with and without checkpoints,
cubic and trilinear interpolation.  Both run the same kernels, so the results
agree bitwise."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, say, to_dev, to_np
from paper_2008_12820_amd import _lib as L

pytestmark = pytest.mark.gpu


def _plan_forward(cfg, m0, v, ckpt):
    stream = torch.cuda.current_stream(DEV).cuda_stream
    h = L.lddmm_plan_create(cfg, stream)
    try:
        out = torch.empty_like(m0)
        L.lddmm_transport_forward(h, m0, v, out, ckpt)
        torch.cuda.synchronize()
        return out
    finally:
        L.lddmm_plan_destroy(h)


@pytest.mark.parametrize("flags", [0, L.FLAG_LINEAR_IP])
def test_static_transport_matches_plan(flags):
    stream = torch.cuda.current_stream(DEV).cuda_stream
    for shape, nt, seed in [((48, 40, 64), 4, 4100), ((16, 24, 20), 3, 4110)]:
        say(f"static transport {shape} nt {nt} flags {flags}")
        cfg = L.make_config(shape, nt, L.REG_H2S, 1e-3, flags=flags | L.FLAG_TRANSPORT_ONLY)
        m0 = to_dev(synth.blob_image(shape, 8, seed))
        v = to_dev(synth.bandlimited_vector(shape, 3, seed + 1, max_disp=2.5))
        n = int(np.prod(shape))
        ck_ref = torch.empty(((nt + 1) * n,), device=DEV)
        ref = _plan_forward(cfg, m0, v, ck_ref)
        for with_ckpt in (False, True):
            out = torch.full_like(m0, float("nan"))
            ck = torch.full(((nt + 1) * n,), float("nan"), device=DEV) if with_ckpt else None
            L.lddmm_transport_forward_static(cfg, stream, m0, v, out, ck)
            torch.cuda.synchronize()
            a, b = to_np(out), to_np(ref)
            err = np.linalg.norm(a - b) / np.linalg.norm(b)
            say(f"  ckpt {with_ckpt}: rel {err:.2e}, bitwise {np.array_equal(a, b)}")
            assert err <= 1e-6
            assert np.array_equal(a, b)
            if with_ckpt:
                assert np.array_equal(to_np(ck), to_np(ck_ref))


def test_static_transport_rejects_large_grids():
    stream = torch.cuda.current_stream(DEV).cuda_stream
    shape = (128, 128, 160)  # 2^21 * 1.25 points: beyond the static array
    cfg = L.make_config(shape, 2, L.REG_H2S, 1e-3, flags=L.FLAG_TRANSPORT_ONLY)
    m0 = torch.zeros(shape, device=DEV)
    v = torch.zeros((3,) + shape, device=DEV)
    out = torch.empty_like(m0)
    with pytest.raises(L.LddmmError) as e:
        L.lddmm_transport_forward_static(cfg, stream, m0, v, out)
    assert e.value.status == L.EINVAL
    with pytest.raises(L.LddmmError) as e:
        L.lddmm_transport_forward_static(L.make_config((16, 16, 16), 2, flags=L.FLAG_TRANSPORT_ONLY),
                                         stream, m0, v, m0)
    assert e.value.status == L.EINVAL
