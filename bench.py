"""Benchmark: Gauss-Newton Hessian matvecs/s and transport grid-points/s at
256^3 FP32 on one MI355X, with the HBM roofline of the dominant kernel and
the FP64 CPU oracle timed beside it.

Workload (one "step" = one Hessian matvec, eqs. "matvec", "incsta",
"incadj" of arXiv 2008.12820, on a fresh incremental velocity):
  grid 256^3, N_t = 4 (and N_t = 8 reported alongside), cubic Lagrange
  interpolation, H2 seminorm, beta = 5e-4, Leray projection on;
  template: 120 periodic Gaussian blobs (sigma 3..12 voxels) in [0,1];
  reference: a second blob image; velocity v = v_true / 2 with v_true
  band-limited |k| <= 8 scaled to a 6-voxel maximum displacement;
  incremental velocities band-limited |k| <= 8, unit RMS (4, reused cyclically).
All inputs are resident in HBM before timing starts; the per-velocity
precompute (set_velocity) is timed separately.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_bytes(cls, n, nt):
    """Algorithmic (compulsory) bytes one Hessian matvec moves through each
    kernel class: every field read once, every output written once; a gather
    counts one read of its source field; FFT passes count their spectral
    input and output once.  Leray on (assembly: 6 fields in, 3 out)."""
    n1, n2, n3 = n
    N = n1 * n2 * n3
    S = n1 * n2 * (n3 // 2 + 1) * 8  # one FP32 half-spectrum field (complex64)
    D = 2 * S                        # the same in FP64 (the forward chain of v~)
    return {
        # incremental-state start: dX 12 + v~ 12 (gathered and read pointwise,
        # counted once) + I[G_j](X) 12 nt + G_{j+1} 12 nt; writes m~_1 and
        # the sources s_1 .. s_{nt-1}: 4 nt
        "incstate_init": (24 + 28 * nt) * N,
        # dX 12 + m~_j 4 + s_j 4 + m~_{j+1} 4
        "incstate_step": 24 * N * (nt - 1),
        # dXa 12 + lam~_{j+1} 4 + c 4 + lam~_j 4, all adjoint steps but the last
        "adj_step": 24 * N * (nt - 1),
        # last adjoint step with the body force: dXa 12 + lam~_1 4 + c 4 +
        # lam~_0 4 + lam~_2 .. lam~_nt 4 (nt - 1) + G_j 12 (nt + 1) + b~ 12
        "adj_body": (16 * nt + 44) * N,
        # (transport VJP only) lam_j (nt+1) + G_j 3 (nt+1) + b 3
        "body_force": (16 * (nt + 1) + 12) * N,
        # x3 R2C of v~ (FP32 in, FP64 out) and of b~ (FP32 in and out)
        "r2c_x3": 3 * (4 * N + D) + 3 * (4 * N + S),
        # x2 forward of v~ (FP64) and b~ (FP32), x2 inverse of the result (FP32)
        "fft_cols": 3 * 2 * D + 3 * 2 * S + 3 * 2 * S,
        # fused x1 forward (v~ FP64, b~ FP32), symbol, x1 inverse (FP32 out)
        "x1_symbol": 3 * D + 3 * S + 3 * S,
        "c2r_x3": 3 * (S + 4 * N),
    }.get(cls)


# the kernel classes one Hessian matvec launches
MATVEC_CLASSES = ("incstate_init", "incstate_step", "adj_step", "adj_body", "r2c_x3", "fft_cols",
                  "x1_symbol", "c2r_x3")


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCE = {
    "incstate_init": ["paper_2008_12820_amd/csrc/transport.hip"],
    "adj_body": ["paper_2008_12820_amd/csrc/transport.hip"],
    "incstate_step": ["paper_2008_12820_amd/csrc/transport.hip"],
    "adj_step": ["paper_2008_12820_amd/csrc/transport.hip"],
    "body_force": ["paper_2008_12820_amd/csrc/transport.hip"],
    "r2c_x3": ["paper_2008_12820_amd/csrc/fft.hip"],
    "fft_cols": ["paper_2008_12820_amd/csrc/fft.hip"],
    "x1_symbol": ["paper_2008_12820_amd/csrc/fft.hip"],
    "c2r_x3": ["paper_2008_12820_amd/csrc/fft.hip"],
}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE, copy-kernel calibrated), or None when
    no summary exists or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get(workload, {}).get(kernel)
    if not ent or ent.get("source_hash") != source_hash(KERNEL_SOURCE[kernel]):
        return None
    return ent.get("bytes_per_launch")


def measured_matvec_bytes(workload, launches):
    """HBM bytes of one matvec from the committed PMC summary: the gather
    classes' bytes per launch times their launches per matvec (`launches`,
    class -> count) plus the transform classes' bytes per matvec; None when
    a class is missing or its source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh).get(workload, {})
    total = 0.0
    for cls in MATVEC_CLASSES:
        ent = data.get(cls)
        if not ent or ent.get("source_hash") != source_hash(KERNEL_SOURCE[cls]):
            return None
        if "bytes_per_matvec" in ent:
            total += ent["bytes_per_matvec"]
        elif cls in launches:
            total += ent["bytes_per_launch"] * launches[cls]
        else:
            return None
    return total


def make_inputs(n, seed=3000):
    import numpy as np
    import synth
    log(f"generating inputs {n}")
    m0 = synth.f32(synth.blob_image(n, 120, seed))
    m1 = synth.f32(synth.blob_image(n, 120, seed + 2))
    vtrue = synth.bandlimited_vector(n, 8, seed + 1, max_disp=6.0)
    v = synth.f32(0.5 * vtrue)
    vts = [synth.f32(synth.unit_rms(synth.bandlimited_vector(n, 8, seed + 100 + r)))
           for r in range(4)]
    return m0, m1, v, vts


def time_matvecs(plan, vts_dev, steps, warmup, torch, only=None):
    """warmup untimed matvecs, then exactly steps timed ones (wall clock);
    HIP events bracket every launch (only=None) or the launches of one kernel
    class (only=name: the others run unbracketed, as in production)."""
    out = torch.empty_like(vts_dev[0])
    for i in range(warmup):
        plan.hessian_matvec(vts_dev[i % len(vts_dev)], out)
    torch.cuda.synchronize()
    plan.set_timing(True, only=only)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        plan.hessian_matvec(vts_dev[i % len(vts_dev)], out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = plan.timing()
    plan.set_timing(False)
    return t1 - t0, kt


def matvec_spread(plan, vts_dev, steps, torch):
    """Each of `steps` matvecs bracketed by HIP events on the plan's stream
    (a pass of its own after the timed region): median, minimum and mean ms."""
    import numpy as np
    out = torch.empty_like(vts_dev[0])
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    plan.hessian_matvec(vts_dev[0], out)
    torch.cuda.synchronize()
    for i in range(steps):
        ev[i][0].record()
        plan.hessian_matvec(vts_dev[i % len(vts_dev)], out)
        ev[i][1].record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"median_ms": float(np.median(t)), "min_ms": float(t.min()), "mean_ms": float(t.mean()),
            "max_ms": float(t.max()), "matvecs": steps}


def bench_config2(torch, dev):
    """The 128^3 Gauss-Newton problem (40-blob template, its image under a
    divergence-free band-limited velocity |k| <= 6 of about 4 voxels, H2
    beta = 5e-4, N_t = 4): one Newton step of exactly 10 PCG iterations with
    (beta A)^{-1} from v = 0, on the GPU (warm, mean of three).  Returns the
    GPU figures and the inputs for the oracle's run of the same step."""
    import synth
    from paper_2008_12820_amd import Plan
    n = (128, 128, 128)
    m0 = synth.f32(synth.blob_image(n, 40, 2000))
    vtrue = synth.f32(synth.bandlimited_vector(n, 6, 2001, max_disp=4.0, divfree=True))
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    T = Plan(n, 4, reg=2, beta=5e-4, device=dev, transport_only=True)
    m1 = T.transport_forward(to(m0), to(vtrue))
    T.close()
    P = Plan(n, 4, reg=2, beta=5e-4, device=dev)
    P.autotune()
    P.set_images(to(m0), m1)
    zero = torch.zeros((3,) + n, device=dev)
    P.set_velocity(zero)
    P.autotune()
    P.newton_step(10, 1e-30)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        _, info = P.newton_step(10, 1e-30)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / 3
    m1h = m1.cpu().numpy()
    tiles = P.tuning()
    P.close()
    return {"grid": list(n), "pcg_iters": info["pcg_iters"], "newton_step_ms": 1e3 * el, "fft_tiles": tiles}, (m0, m1h)


def bench_leray_off(torch, dev, n, m0d, m1d, vd, vtd, steps, warmup):
    """The same matvec with the Leray projection off (K = I): the assembly is
    pointwise in b, A v~ runs wholly beside the transport sweeps."""
    from paper_2008_12820_amd import Plan
    log("matvec, Leray projection off")
    plan = Plan(n, 4, reg=2, beta=5e-4, leray=False, device=dev)
    plan.autotune()
    plan.set_images(m0d, m1d)
    plan.set_velocity(vd)
    plan.autotune()
    out = torch.empty_like(vtd[0])
    for i in range(warmup):
        plan.hessian_matvec(vtd[i % len(vtd)], out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        plan.hessian_matvec(vtd[i % len(vtd)], out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.close()
    return {"matvecs_per_s": steps / el, "ms_per_matvec": 1e3 * el / steps, "nt": 4, "leray": False}


def dominant_class(kt, n, nt):
    return max((k for k in kt if kernel_bytes(k, n, nt) is not None), key=lambda k: kt[k][0])


# the oracle's 128^3 matvec on one thread, in a child process (the OpenMP
# thread count is fixed at the runtime's start); prints the seconds
_ONE_THREAD = r"""
import sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle, synth
n = (128, 128, 128)
m0 = synth.f32(synth.blob_image(n, 40, 3000))
m1 = synth.f32(synth.blob_image(n, 40, 3002))
v = synth.f32(0.5 * synth.bandlimited_vector(n, 8, 3001, max_disp=3.0))
vt = synth.f32(synth.unit_rms(synth.bandlimited_vector(n, 8, 3100)))
P = oracle.Problem(n, 4, reg=2, beta=5e-4, leray=True)
P.set_images(synth.f64(m0), synth.f64(m1))
P.set_velocity(synth.f64(v))
t0 = time.perf_counter()
P.matvec(synth.f64(vt))
print(time.perf_counter() - t0)
"""


def oracle_one_thread():
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_THREAD, ROOT], env=env, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        log(f"one-thread oracle run failed: {r.stderr[-400:]}")
        return None
    return float(r.stdout.strip().splitlines()[-1])


def oracle_config2(m0, m1):
    """the oracle's Newton step (10 PCG iterations, InvA, from v = 0) on the
    128^3 problem of bench_config2, with the precompute and gradient"""
    import numpy as np
    import oracle
    import synth
    n = m0.shape
    P = oracle.Problem(n, 4, reg=2, beta=5e-4)
    P.set_images(synth.f64(m0), synth.f64(m1))
    t0 = time.perf_counter()
    P.set_velocity(np.zeros((3,) + n))
    g = P.gradient()
    P.pcg(-g, 10, 1e-30)
    return time.perf_counter() - t0


def cpu_baseline(n, nt, m0, m1, v, vt, sample):
    import numpy as np
    import oracle
    import synth
    cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    shape = n if sample == "full" else tuple(s // 2 for s in n)
    if sample != "full":
        sl = (slice(None, None, 2),) * 3
        m0, m1 = m0[sl], m1[sl]
        v, vt = v[(slice(None),) + sl], vt[(slice(None),) + sl]
    P = oracle.Problem(shape, nt, reg=2, beta=5e-4, leray=True)
    P.set_images(synth.f64(m0), synth.f64(m1))
    log(f"oracle precompute {shape} (timed apart)")
    t0 = time.perf_counter()
    P.set_velocity(synth.f64(v))
    t_pre = time.perf_counter() - t0
    log("oracle matvec (timed)")
    t0 = time.perf_counter()
    P.matvec(synth.f64(vt))
    dt = time.perf_counter() - t0
    scale = float(np.prod(shape)) / float(np.prod(n))
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": scale / dt,
        "unit": "matvecs/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"one FP64 oracle Hessian matvec at {shape[0]}^3, N_t={nt} (per-velocity "
                   f"precompute untimed), {dt:.2f} s" +
                   ("" if sample == "full" else "; scaled by the point-count ratio to 256^3")),
        "seconds": dt,
        "precompute_seconds": t_pre,
        "cpu_model": cpu,
    }


def bench_batched(torch, dev):
    """64 registrations, sizes uniform over {64,96,128,160}^3, N_t = 4, H2
    beta = 1e-3, 5 Gauss-Newton iterations of exactly 8 PCG iterations:
    batched graph-captured form vs the same members run one after another
    through the plain per-plan calls."""
    import numpy as np
    import synth
    from paper_2008_12820_amd import Plan
    from paper_2008_12820_amd.batch import Batch
    rng = np.random.default_rng(4000)
    sizes = [int(x) for x in rng.choice([64, 96, 128, 160], size=64)]
    shapes = [(n, n, n) for n in sizes]
    log(f"batched: generating {len(sizes)} members")
    m0s, m1s = [], []
    for b, s in enumerate(shapes):
        if b % 16 == 0:
            log(f"batched: member {b}")
        seed = 4000 + 10 * b
        m0 = torch.from_numpy(synth.f32(synth.blob_image(s, 40, seed))).to(dev)
        vt = torch.from_numpy(synth.f32(synth.bandlimited_vector(s, 6, seed + 1, max_disp=4.0))).to(dev)
        P = Plan(s, 4, reg=2, beta=1e-3, device=dev, transport_only=True)
        m1s.append(P.transport_forward(m0, vt))
        m0s.append(m0)
        P.close()
    torch.cuda.synchronize()
    npts = sum(int(np.prod(s)) for s in shapes)
    GN, PCG, TOL = 5, 8, 1e-30  # tiny rtol: exactly 8 PCG iterations per step

    log("batched: sequential plain runs")
    plans = [Plan(s, 4, reg=2, beta=1e-3, device=dev) for s in shapes]
    vseq = [torch.zeros((3,) + s, device=dev) for s in shapes]
    for b, P in enumerate(plans):
        P.set_images(m0s[b], m1s[b])
        P.set_velocity(vseq[b])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, P in enumerate(plans):
        for _ in range(GN):
            P.gn_iterate(vseq[b], PCG, TOL)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for P in plans:
        P.close()
    del plans
    torch.cuda.empty_cache()

    log("batched: graph-captured batch")
    Bt = Batch(shapes, 4, reg=2, beta=1e-3, nstreams=8)
    vb = [torch.zeros((3,) + s, device=dev) for s in shapes]
    Bt.set_images(m0s, m1s)
    Bt.set_velocity(vb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_iter = []
    for _ in range(GN):
        ti = time.perf_counter()
        infos = Bt.gn_iterate(vb, PCG, TOL, use_graph=True)  # the first call also captures the graph
        torch.cuda.synchronize()
        t_iter.append(time.perf_counter() - ti)
    t_bat = time.perf_counter() - t0
    diff = max(float(torch.linalg.vector_norm(vb[b] - vseq[b]) /
                     torch.linalg.vector_norm(vseq[b]).clamp_min(1e-30)) for b in range(len(shapes)))
    Bt.close()
    return {
        "members": len(shapes), "sizes": {str(n): sizes.count(n) for n in (64, 96, 128, 160)},
        "gn_steps": GN, "pcg_per_step": PCG,
        "batched_s": t_bat, "sequential_s": t_seq,
        "batched_iteration_s": t_iter,
        "registrations_per_s": len(shapes) / t_bat,
        "sequential_registrations_per_s": len(shapes) / t_seq,
        "speedup": t_seq / t_bat,
        "aggregate_grid_pts_per_s": npts * GN / t_bat,
        "max_rel_l2_vs_sequential": diff,
        "accepted_steps": sum(1 for i in infos if i["alpha"] > 0),
    }


def fft_comparison(torch, dev, n):
    """One forward 3D R2C of an n^3 FP32 field: the hand-written FFT (x3, x2
    and x1 passes plus the repack into the standard half-spectrum layout)
    against torch.fft.rfftn (rocFFT through hipFFT), both timed with events
    on the current stream; context only, not part of the metric."""
    from paper_2008_12820_amd import Plan
    P = Plan(n, 1, reg=2, beta=1e-3, device=dev, transport_only=True)
    x = torch.randn(n, device=dev, dtype=torch.float32)

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    ours = timed(lambda: P.fft_r2c(x))
    try:
        ref = timed(lambda: torch.fft.rfftn(x))
        y1, y2 = P.fft_r2c(x), torch.fft.rfftn(x)
        agree = float(torch.linalg.vector_norm(y1 - y2) / torch.linalg.vector_norm(y2))
    except Exception as e:  # no hipFFT in this torch build
        log(f"rocFFT comparison unavailable: {e}")
        ref, agree = None, None
    P.close()
    return {"grid": list(n), "fft_r2c_ms": ours, "rocfft_rfftn_ms": ref, "rel_l2_vs_rocfft": agree}


def bench_autograd(torch, dev, n=512, nt=8):
    """TransportMap forward + backward at 512^3, N_t = 8, with the loss
    0.5 ||m(1) - m1||^2 + beta H2(v), beta = 1e-4, against the plain reduced
    gradient (set_velocity + gradient) on the same inputs."""
    import numpy as np
    import synth
    from paper_2008_12820_amd import Plan
    from paper_2008_12820_amd.autograd import TransportMap
    shape = (n, n, n)
    log(f"autograd: generating {shape}")
    m0 = torch.from_numpy(synth.f32(synth.blob_image(shape, 120, 5000))).to(dev)
    m1 = torch.from_numpy(synth.f32(synth.blob_image(shape, 120, 5002))).to(dev)
    v = torch.from_numpy(synth.f32(synth.bandlimited_vector(shape, 8, 5001, max_disp=6.0))).to(dev)
    beta = 1e-4
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    T = TransportMap(shape, nt, reg=2, beta=beta, device=dev)
    ws_t = Plan.workspace_bytes(shape, nt, 2, beta, transport_only=True)
    times = []
    for it in range(3):
        vv = v.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = 0.5 * ((T(m0, vv) - m1) ** 2).sum() + beta * T.reg_energy(vv)
        loss.backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    torch_peak = torch.cuda.max_memory_allocated()
    g_auto = vv.grad.detach().clone()
    T.plan.close()
    del T
    torch.cuda.empty_cache()
    log("autograd: plain reduced gradient")
    P = Plan(shape, nt, reg=2, beta=beta, device=dev)
    ws_p = Plan.workspace_bytes(shape, nt, 2, beta)
    P.set_images(m0, m1)
    tp = []
    for it in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.set_velocity(v)
        g, gn = P.gradient()
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
    # plain-sum loss gradient equals the reduced gradient (no h^3, K = I)
    rel = float(torch.linalg.vector_norm(g_auto - g) / torch.linalg.vector_norm(g))
    P.close()
    return {"grid": list(shape), "nt": nt, "forward_backward_ms": 1e3 * min(times),
            "plain_set_velocity_gradient_ms": 1e3 * min(tp),
            "transport_plan_GB": ws_t / 1e9, "plain_plan_GB": ws_p / 1e9,
            "torch_peak_GB": torch_peak / 1e9, "rel_l2_autograd_vs_plain_gradient": rel}


def bench_syn(torch, dev, n):
    """The paper's SYN problem (Section 4) as in its scaling table: 5 Gauss-
    Newton iterations of 10 PCG steps, InvA, beta = 1e-3, N_t = 4, trilinear
    interpolation, FD first derivatives; m1 = the template transported by the
    SYN velocity.  Time of the whole solve from v = 0."""
    import synth
    from paper_2008_12820_amd import Plan

    log(f"SYN workload {n}")
    m0, vsyn = synth.syn_problem(n)
    m0d = torch.from_numpy(synth.f32(m0)).to(dev)
    vd = torch.from_numpy(synth.f32(vsyn)).to(dev)
    P = Plan(n, 4, reg=2, beta=1e-3, device=dev, linear_ip=True, fd8=True)
    P.autotune()
    m1d = P.transport_forward(m0d, vd)
    P.set_images(m0d, m1d)
    v = torch.zeros_like(vd)
    kw = dict(eps_n=0.0, max_gn=5, max_pcg=10, rtol=1e-12, continuation=False, pc="inva")
    P.gn_solve(v.clone(), 1e-3, **{**kw, "max_gn": 1, "max_pcg": 2})  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = P.gn_solve(v, 1e-3, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    mis = P.objective()[1]
    P.set_velocity(torch.zeros_like(vd))
    mis0 = P.objective()[1]
    P.close()
    return {"grid": list(n), "gn_iters": rep["gn_iters"], "pcg_iters": rep["pcg_iters"], "seconds": el,
            "relative_mismatch": mis / mis0, "gnorm_rel": rep["gnorm_rel"],
            "paper_v100_1gpu_seconds": 3.32 if n == (256, 256, 256) else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--no-nt8", action="store_true")
    ap.add_argument("--no-overlap", action="store_true",
                    help="serialise the assembly's forward transform with the transport sweeps")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", choices=["full", "half"], default="full")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-member batched run")
    ap.add_argument("--no-autograd", action="store_true", help="skip the 512^3 autograd run")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the matvec lines (no Leray-off, FFT, SYN, 128^3 Newton, batched, autograd)")
    ap.add_argument("--pcg-only", action="store_true",
                    help="only Newton steps of 10 PCG iterations on the N_t = 4 plan (one warm, three timed), "
                         "e.g. under a kernel trace")
    ap.add_argument("--no-newton", action="store_true",
                    help="no Newton steps (the matvec kernels alone, e.g. for hardware counters)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU's share only (the whole grid on one device); "
              "runs on more than one GPU are not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2008_12820_amd import Plan

    n = (args.size,) * 3
    N = int(np.prod(n))
    nt = 4
    dev = torch.device("cuda", 0)
    m0, m1, v, vts = make_inputs(n)
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    m0d, m1d, vd = to(m0), to(m1), to(v)
    vtd = [to(a) for a in vts]

    res_nt = {}
    for nt_ in ([4] if args.no_nt8 else [4, 8]):
        log(f"plan {n} nt={nt_}")
        plan = Plan(n, nt_, reg=2, beta=5e-4, leray=True, device=dev)
        tuning = plan.autotune()
        log(f"autotuned: {tuning}")
        plan.set_images(m0d, m1d)
        plan.set_velocity(vd)
        tuning = plan.autotune()  # gather strategy, timed on this velocity's displacements
        plan.set_overlap(False)  # the per-class profile below attributes time without sharing
        log(f"autotuned: {tuning}")
        if args.pcg_only:
            plan.newton_step(10, 0.0)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                _, info = plan.newton_step(10, 0.0)
            torch.cuda.synchronize()
            print(json.dumps({"pcg_only": True, "grid": list(n), "nt": nt_, "pcg_iters": info["pcg_iters"],
                              "newton_step_10pcg_ms": 1e3 * (time.perf_counter() - t0) / 3}), flush=True)
            return
        # per-velocity precompute and reduced gradient, warm (the first call of
        # each loads its kernels), mean of three calls
        plan.set_velocity(vd)
        g, gn = plan.gradient()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            plan.set_velocity(vd)
        torch.cuda.synchronize()
        pre = (time.perf_counter() - t0) / 3
        t0 = time.perf_counter()
        for _ in range(3):
            g, gn = plan.gradient()
        torch.cuda.synchronize()
        tg = (time.perf_counter() - t0) / 3
        steps = args.steps if nt_ == 4 else max(5, args.steps // 2)
        # per-class profile (every launch bracketed by events), then the timed
        # region with only the dominant class bracketed
        log(f"profiling kernel classes nt={nt_}")
        prof_steps = max(4, steps // 2)
        _, kt = time_matvecs(plan, vtd, prof_steps, 1, torch)
        dom_ = dominant_class(kt, n, nt_)
        plan.set_overlap(not args.no_overlap)
        log(f"timing {steps} matvecs nt={nt_} (events on {dom_}, overlap {not args.no_overlap})")
        el, kt_dom = time_matvecs(plan, vtd, steps, args.warmup, torch, only=dom_)
        spread = matvec_spread(plan, vtd, steps, torch)
        log(f"per-matvec events nt={nt_}: {spread}")
        res_nt[nt_] = dict(elapsed=el, steps=steps, kt=kt, prof_steps=prof_steps, kt_dom=kt_dom, dom=dom_,
                           precompute_s=pre, spread=spread,
                           gradient_s=tg, tuning=tuning)
        if nt_ == 4 and not args.no_newton:
            log("newton step, 10 PCG iterations")
            vt_out, info = plan.newton_step(10, 0.0)  # warm (loads the PCG kernels)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                vt_out, info = plan.newton_step(10, 0.0)
            torch.cuda.synchronize()
            res_nt[nt_]["newton_step_s"] = (time.perf_counter() - t0) / 3
            res_nt[nt_]["newton_info"] = {k: info[k] for k in ("pcg_iters", "rel_res", "gnorm")}
            # Newton step to a fixed relative residual with each preconditioner
            # (eps_H0 = 1e-3 as the paper's NIREP runs, 1e-2 as its CLARITY
            # runs, 1e-1 beside them; the second of two calls is timed)
            pcs = {}
            for kind, eps in (("inva", 1e-3), ("invh0", 1e-3), ("2linvh0", 1e-3), ("invh0", 1e-2),
                              ("2linvh0", 1e-2), ("2linvh0", 1e-1)):
                plan.set_preconditioner(kind, eps_h0=eps, max_inner=50)
                key = kind if eps == 1e-3 else f"{kind}_eps{eps:g}"
                for _ in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, inf = plan.newton_step(100, 1e-2)
                    torch.cuda.synchronize()
                pcs[key] = {"ms": 1e3 * (time.perf_counter() - t0), "pcg_iters": inf["pcg_iters"],
                            "inner_iters": inf["inner_iters"], "rel_res": inf["rel_res"], "eps_h0": eps}
                log(f"newton step rtol 1e-2, {key}: {pcs[key]}")
            # the same step at a smaller beta (the H0 solves keep their beta0 of 5e-2)
            pcs_small = {}
            plan.set_beta(1e-4)
            for kind, eps in (("inva", 1e-3), ("2linvh0", 1e-1)):
                plan.set_preconditioner(kind, eps_h0=eps, max_inner=50)
                key = kind if kind == "inva" else f"{kind}_eps{eps:g}"
                for _ in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, inf = plan.newton_step(300, 1e-2, allow_notconv=True)
                    torch.cuda.synchronize()
                pcs_small[key] = {"ms": 1e3 * (time.perf_counter() - t0), "pcg_iters": inf["pcg_iters"],
                                  "inner_iters": inf["inner_iters"], "rel_res": inf["rel_res"], "eps_h0": eps}
                log(f"newton step rtol 1e-2, beta 1e-4, {key}: {pcs_small[key]}")
            plan.set_beta(5e-4)
            plan.set_preconditioner("inva")
            res_nt[nt_]["newton_preconditioners"] = pcs
            res_nt[nt_]["newton_preconditioners_beta1e-4"] = pcs_small
            # the eighth-order FD first derivatives (Section 3.2) in a second plan:
            # per-velocity precompute, derivative kernel time, scheme difference
            g_spec, _ = plan.gradient()
            g_spec = g_spec.clone()
            fplan = Plan(n, nt_, reg=2, beta=5e-4, leray=True, device=dev, fd8=True)
            fplan.autotune()
            fplan.set_images(m0d, m1d)
            fplan.set_velocity(vd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                fplan.set_velocity(vd)
            torch.cuda.synchronize()
            pre_fd8 = (time.perf_counter() - t0) / 3
            fplan.set_timing(True)  # the derivative kernels' own time, one more call
            fplan.set_velocity(vd)
            torch.cuda.synchronize()
            kt8 = fplan.timing()
            fplan.set_timing(False)
            g_fd8, _ = fplan.gradient()
            res_nt[nt_]["fd8"] = {
                "precompute_ms": 1e3 * pre_fd8,
                "fd8_kernel_ms_per_velocity": kt8.get("fd8", (0, 0))[0],
                "fd8_launches_per_velocity": kt8.get("fd8", (0, 0))[1],
                "gradient_rel_diff_vs_spectral": float(
                    torch.linalg.vector_norm(g_fd8 - g_spec) / torch.linalg.vector_norm(g_spec)),
            }
            log(f"fd8: {res_nt[nt_]['fd8']}")
            fplan.close()
            del fplan
        plan.close()
        del plan
        torch.cuda.empty_cache()

    r4 = res_nt[4]
    value = r4["steps"] / r4["elapsed"]
    ms = 1e3 * r4["elapsed"] / r4["steps"]

    def transport_rate(r, nt_):
        kt = r["kt"]
        t_inc = sum(kt.get(k, (0, 0))[0] for k in ("incstate_init", "incstate_step")) / r["prof_steps"]
        # the last adjoint step carries the body force
        t_adj = sum(kt.get(k, (0, 0))[0] for k in ("adj_step", "adj_body")) / r["prof_steps"]
        return {
            "incstate_pts_per_s": N * nt_ / (t_inc * 1e-3),
            "incadj_pts_per_s": N * nt_ / (t_adj * 1e-3),
            "headline_pts_per_s": 2 * N * nt_ / ((t_inc + t_adj) * 1e-3),
        }

    # dominant kernel of the N_t = 4 matvec and its roofline, from the events
    # around its launches inside the timed region
    kt = r4["kt"]
    dom = r4["dom"]
    t_dom_ms, launches = r4["kt_dom"][dom]
    per_matvec_bytes = kernel_bytes(dom, n, nt)
    launches_per_matvec = launches / r4["steps"]
    bytes_per_launch = per_matvec_bytes / launches_per_matvec
    achieved = bytes_per_launch / (t_dom_ms / launches * 1e-3) / 1e9
    workload = f"matvec_{n[0]}^3_nt{nt}"
    traffic = measured_traffic(dom, workload)
    prof_steps = r4["prof_steps"]  # matvecs of the profiling pass
    kernels = {k: {"ms_per_matvec": kt[k][0] / prof_steps,
                   "launches_per_matvec": kt[k][1] / prof_steps} for k in kt}
    for k in kernels:
        b = kernel_bytes(k, n, nt)
        if b is not None:
            kernels[k]["alg_GBps"] = b / (kernels[k]["ms_per_matvec"] * 1e-3) / 1e9
    def matvec_alg_bytes(nt_):  # whole-matvec algorithmic bytes (Leray on): the classes' sum
        return sum(kernel_bytes(k, n, nt_) for k in MATVEC_CLASSES)

    def unfused_bytes(nt_):  # the unfused step count, (136 + 132 N_t) B per grid point (Leray on)
        return (136 + 132 * nt_) * N

    # measured (FETCH_SIZE + WRITE_SIZE) bytes of one matvec from the committed counters
    meas = measured_matvec_bytes(workload, {"incstate_init": 1, "incstate_step": nt - 1, "adj_step": nt - 1,
                                            "adj_body": 1})

    out = {
        "metric": "Hessian matvecs/s and transport grid-pts/s at 256^3 FP32; % HBM roofline",
        "value": value,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": r4["steps"],
        "warmup": args.warmup,
        "ms_per_step": ms,
        "timed_s": r4["elapsed"],  # the timed region (K matvecs between two synchronisations)
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"gauss-newton hessian matvec, {n[0]}^3, N_t={nt}, cubic "
                               "Lagrange SL, H2 seminorm beta=5e-4, Leray on",
                   "grid": list(n), "nt": nt, "parallelism": "single GPU (whole grid)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": dom,
                     "bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": t_dom_ms / launches},
        "transport": transport_rate(r4, 4),
        "matvec_alg_bytes_per_pt": matvec_alg_bytes(nt) / N,
        "matvec_alg_hbm_frac": matvec_alg_bytes(nt) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "matvec_unfused_bytes_per_pt": unfused_bytes(nt) / N,
        "matvec_unfused_hbm_frac": unfused_bytes(nt) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "matvec_measured_bytes": meas,
        "matvec_measured_hbm_frac": meas / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS if meas else None,
        "matvec_events": r4["spread"],
        "kernels": kernels,
        "precompute_ms": 1e3 * r4["precompute_s"],
        "gradient_ms": 1e3 * r4["gradient_s"],
        "newton_step_10pcg_ms": 1e3 * r4["newton_step_s"] if "newton_step_s" in r4 else None,
        "newton_info": r4.get("newton_info"),
        "newton_rtol_1e-2": r4.get("newton_preconditioners"),
        "newton_rtol_1e-2_beta1e-4": r4.get("newton_preconditioners_beta1e-4"),
        "fd8": r4.get("fd8"),
        "fft_tiles": r4["tuning"],
        "overlap": not args.no_overlap,
    }
    if 8 in res_nt:
        r8 = res_nt[8]
        ms8 = 1e3 * r8["elapsed"] / r8["steps"]
        out["nt8"] = {"matvecs_per_s": r8["steps"] / r8["elapsed"], "ms_per_matvec": ms8,
                      "transport": transport_rate(r8, 8),
                      "matvec_alg_hbm_frac": matvec_alg_bytes(8) / (ms8 * 1e-3) / 1e9 / PEAK_HBM_GBS,
                      "matvec_unfused_hbm_frac": unfused_bytes(8) / (ms8 * 1e-3) / 1e9 / PEAK_HBM_GBS,
                      "matvec_events": r8["spread"],
                      "precompute_ms": 1e3 * r8["precompute_s"]}
    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        src = torch.empty(1 << 28, device=dev, dtype=torch.float32).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": 1 << 30, "bytes_written": 1 << 30,
                                   "GBps": 5 * 2 * (1 << 30) / (time.perf_counter() - t0) / 1e9}
        del src, dst
    c2_inputs = None
    if not args.no_extras:
        out["leray_off"] = bench_leray_off(torch, dev, n, m0d, m1d, vd, vtd, args.steps, args.warmup)
        out["fft_vs_rocfft"] = fft_comparison(torch, dev, n)
        out["syn_workload"] = bench_syn(torch, dev, n)
        log("128^3 Newton step (10 PCG)")
        out["newton_128"], c2_inputs = bench_config2(torch, dev)
        if not args.no_batched:
            out["batched"] = bench_batched(torch, dev)
            log(f"batched: {out['batched']}")
        if not args.no_autograd:
            out["autograd"] = bench_autograd(torch, dev)
            log(f"autograd: {out['autograd']}")
    if not args.no_cpu:
        log("cpu baseline (FP64 oracle)")
        out["cpu_baseline"] = cpu_baseline(n, nt, m0, m1, v, vts[0], args.cpu_sample)
        out["cpu_baseline"]["precompute_vs_gpu"] = out["cpu_baseline"]["precompute_seconds"] / (
            out["precompute_ms"] * 1e-3)
        if not args.no_extras:
            log("oracle: one thread, one matvec at 128^3")
            out["cpu_baseline"]["one_thread_128_matvec_s"] = oracle_one_thread()
            log("oracle: 128^3 Newton step")
            t_or = oracle_config2(*c2_inputs)
            out["newton_128"]["oracle_s"] = t_or
            out["newton_128"]["oracle_cores"] = out["cpu_baseline"]["cores"]
    else:
        out["cpu_baseline"] = None
    out["host"] = platform.node()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
