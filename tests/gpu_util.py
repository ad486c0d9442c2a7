"""Shared helpers of the GPU parity tests (inputs from synth, references from
the oracle, device results through the C ABI)."""
import numpy as np
import torch

import oracle
import synth

DEV = torch.device("cuda", 0)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def say(msg):
    print(msg, flush=True)


def problem(shape, nt, reg=1, beta=1e-2, leray=False, nblobs=None, K=3, disp=1.0, seed=1000,
            vscale=0.5, divfree=False):
    """Seeded registration inputs: template, velocity v_true, reference m1 =
    oracle transport of m0 by v_true, evaluation velocity v = vscale*v_true.
    Returns float32 arrays (what the GPU gets) and the oracle problem with
    images and velocity set from the same float32 values."""
    if nblobs:
        m0 = synth.f32(synth.blob_image(shape, nblobs, seed))
    else:
        m0 = synth.f32(synth.sin2_template(shape, 4, seed))
    vtrue = synth.f32(synth.bandlimited_vector(shape, K, seed + 1, max_disp=disp, divfree=divfree))
    ref = oracle.Problem(shape, nt, reg=reg, beta=beta, leray=leray)
    ref.set_images(synth.f64(m0), synth.f64(m0))
    ref.set_velocity(synth.f64(vtrue))
    m1 = synth.f32(ref.transport(synth.f64(m0))[-1])
    v = synth.f32(vscale * synth.f64(vtrue))
    ref.set_images(synth.f64(m0), synth.f64(m1))
    ref.set_velocity(synth.f64(v))
    return m0, m1, vtrue, v, ref


def incremental(shape, seed, K=3):
    return synth.f32(synth.unit_rms(synth.bandlimited_vector(shape, K, seed)))
