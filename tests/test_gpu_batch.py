"""GPU checks of the batched form: members of uneven grid sizes advanced by
graph-captured (and eager) batched Gauss-Newton iterations reproduce the
plain per-member lddmm_gn_iterate, and one member against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, rel, say, to_dev, to_np
from paper_2008_12820_amd import Plan
from paper_2008_12820_amd import _lib as L
from paper_2008_12820_amd.batch import Batch

pytestmark = pytest.mark.gpu

SIZES = [16, 24, 20, 32, 16]
NT, BETA = 4, 1e-3


def _member(n, seed):
    shape = (n, n, n)
    m0 = synth.f32(synth.blob_image(shape, 6, seed))
    vtrue = synth.f32(synth.bandlimited_vector(shape, 3, seed + 1, max_disp=2.0))
    ref = oracle.Problem(shape, NT, reg=2, beta=BETA)
    ref.set_images(synth.f64(m0), synth.f64(m0))
    ref.set_velocity(synth.f64(vtrue))
    m1 = synth.f32(ref.transport(synth.f64(m0))[-1])
    ref.set_images(synth.f64(m0), synth.f64(m1))
    ref.set_velocity(np.zeros((3,) + shape))
    return m0, m1, ref


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_matches_plain_gn(use_graph):
    say(f"batch vs plain, graph={use_graph}")
    mem = [_member(n, 5000 + 10 * b) for b, n in enumerate(SIZES)]
    shapes = [(n, n, n) for n in SIZES]
    Bt = Batch(shapes, NT, reg=2, beta=BETA, nstreams=3)
    m0s = [to_dev(m[0]) for m in mem]
    m1s = [to_dev(m[1]) for m in mem]
    vb = [torch.zeros((3,) + s, device=DEV) for s in shapes]
    Bt.set_images(m0s, m1s)
    Bt.set_velocity(vb)
    plans, vp = [], []
    for b, s in enumerate(shapes):
        P = Plan(s, NT, reg=2, beta=BETA)
        P.set_images(m0s[b], m1s[b])
        v = torch.zeros((3,) + s, device=DEV)
        P.set_velocity(v)
        plans.append(P)
        vp.append(v)
    for it in range(2):
        for rtol in (0.0,):  # eps_K rule (early PCG stop predicated in the batch)
            infos = Bt.gn_iterate(vb, 6, rtol, use_graph=use_graph)
            for b, P in enumerate(plans):
                pinfo = P.gn_iterate(vp[b], 6, rtol)
                assert infos[b]["pcg_iters"] == pinfo["pcg_iters"], (it, b)
                assert infos[b]["alpha"] == pinfo["alpha"], (it, b)
                assert rel(to_np(vb[b]), to_np(vp[b])) < 1e-6, (it, b)
                assert abs(infos[b]["J_after"] - pinfo["J_after"]) <= 1e-6 * abs(pinfo["J_after"])
    # one member against the oracle (two Gauss-Newton iterations)
    ref = mem[3][2]
    for it in range(2):
        v_ref, rinfo = ref.gn_iterate(6, 0.0)
    e = rel(to_np(vb[3]), v_ref)
    say(f"  member 3 after two GN iterations vs oracle: rel {e:.2e}")
    assert e < 1e-5
    Bt.close()


def test_batch_graph_follows_set_beta():
    """A member's captured iteration is recaptured after a beta change (beta
    is an argument of the captured kernels): the batch still equals the
    plain lddmm_gn_iterate at the new beta."""
    say("batch graph after set_beta")
    sizes = [16, 20]
    mem = [_member(n, 5100 + 10 * b) for b, n in enumerate(sizes)]
    shapes = [(n, n, n) for n in sizes]
    Bt = Batch(shapes, NT, reg=2, beta=BETA, nstreams=2)
    m0s = [to_dev(m[0]) for m in mem]
    m1s = [to_dev(m[1]) for m in mem]
    vb = [torch.zeros((3,) + s, device=DEV) for s in shapes]
    Bt.set_images(m0s, m1s)
    Bt.set_velocity(vb)
    plans, vp = [], []
    for b, s in enumerate(shapes):
        P = Plan(s, NT, reg=2, beta=BETA)
        P.set_images(m0s[b], m1s[b])
        v = torch.zeros((3,) + s, device=DEV)
        P.set_velocity(v)
        plans.append(P)
        vp.append(v)
    for it, beta in enumerate((BETA, 20 * BETA)):
        if it:
            for b, P in enumerate(plans):
                P.set_beta(beta)
                L.lddmm_set_beta(L.lddmm_batch_plan(Bt._h, b), beta)
        infos = Bt.gn_iterate(vb, 4, 0.0, use_graph=True)
        for b, P in enumerate(plans):
            pinfo = P.gn_iterate(vp[b], 4, 0.0)
            assert infos[b]["pcg_iters"] == pinfo["pcg_iters"], (it, b)
            assert infos[b]["alpha"] == pinfo["alpha"], (it, b)
            e = rel(to_np(vb[b]), to_np(vp[b]))
            say(f"  iteration {it} beta {beta} member {b}: rel {e:.2e}")
            assert e < 1e-6, (it, b)
    Bt.close()


@pytest.mark.timeout(900)
def test_batch_64_uneven_members_match_plain_and_oracle():
    """The batched workload: 64 registrations with grid sizes drawn from
    {64, 96, 128, 160}^3, N_t = 4, H2 beta = 1e-3, 5 Gauss-Newton iterations
    of 8 PCG iterations each (rtol 1e-30: every member runs all 8).  Each
    member's final velocity equals its plain per-plan run; four members (the
    64^3 ones first in the draw) against the FP64 oracle's five iterations."""
    rng = np.random.default_rng(4000)
    sizes = [int(x) for x in rng.choice([64, 96, 128, 160], size=64)]
    shapes = [(n, n, n) for n in sizes]
    say(f"64-member batch: sizes {dict((n, sizes.count(n)) for n in (64, 96, 128, 160))}")
    m0s, m1s, host = [], [], []
    for b, s in enumerate(shapes):
        m0 = synth.f32(synth.blob_image(s, 40, 4000 + 10 * b))
        m1 = synth.f32(synth.blob_image(s, 40, 4000 + 10 * b + 2))
        m0s.append(to_dev(m0))
        m1s.append(to_dev(m1))
        host.append((m0, m1))
    GN, PCG, TOL = 5, 8, 1e-30
    Bt = Batch(shapes, 4, reg=2, beta=1e-3, nstreams=4)
    vb = [torch.zeros((3,) + s, device=DEV) for s in shapes]
    Bt.set_images(m0s, m1s)
    Bt.set_velocity(vb)
    for _ in range(GN):
        infos = Bt.gn_iterate(vb, PCG, TOL, use_graph=True)
        assert all(i["pcg_iters"] == PCG for i in infos)
    Bt.close()
    worst = 0.0
    for b, s in enumerate(shapes):
        P = Plan(s, 4, reg=2, beta=1e-3)
        P.set_images(m0s[b], m1s[b])
        v = torch.zeros((3,) + s, device=DEV)
        P.set_velocity(v)
        for _ in range(GN):
            P.gn_iterate(v, PCG, TOL)
        e = rel(to_np(vb[b]), to_np(v))
        worst = max(worst, e)
        P.close()
    say(f"  batch vs plain, worst member rel {worst:.2e}")
    assert worst <= 1e-5
    small = [b for b, n in enumerate(sizes) if n == 64][:4]
    for b in small:
        ref = oracle.Problem(shapes[b], 4, reg=2, beta=1e-3)
        ref.set_images(synth.f64(host[b][0]), synth.f64(host[b][1]))
        ref.set_velocity(np.zeros((3,) + shapes[b]))
        for _ in range(GN):
            v_ref, _ = ref.gn_iterate(PCG, TOL)
        e = rel(to_np(vb[b]), v_ref)
        say(f"  member {b} ({sizes[b]}^3) vs oracle after {GN} iterations: rel {e:.2e}")
        assert e < 1e-5
