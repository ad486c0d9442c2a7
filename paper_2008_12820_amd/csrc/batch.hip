// Batched form: many independent registrations (uneven grid sizes) advanced
// together.  Each member is a full plan on one of a few library-owned HIP
// streams; one Gauss-Newton iteration of a member -- gradient, eps_K,
// fixed-count PCG with device-resident scalars, <g, v~>, and the first
// Armijo trial J(v + v~) -- is a single host-sync-free sequence, captured
// once into a hipGraph and replayed, so the members' small kernels overlap
// across streams and their launch cost is paid once per graph.  Only the
// line-search decision needs the host; rejected trials (rare) run eagerly.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.hpp"

namespace lddmm {

struct MemberGraph {
    hipGraphExec_t exec = nullptr;
    int max_pcg = -1;
    double rtol = 0.0;
    unsigned long gen = 0;  // the plan's enqueue generation at capture
};

}  // namespace lddmm

struct lddmm_batch {
    int B = 0;
    std::vector<lddmm_plan *> plans;
    std::vector<hipStream_t> streams;
    std::vector<lddmm::MemberGraph> graphs;
};

namespace lddmm {

template <class F>
static lddmm_status bguard(F &&f)
{
    try {
        f();
        return LDDMM_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.status;
    } catch (...) {
        set_last_error("unexpected exception");
        return LDDMM_EDEVICE;
    }
}

static void batch_free(lddmm_batch *Bt)
{
    if (!Bt) return;
    for (auto &g : Bt->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (lddmm_plan *p : Bt->plans)
        if (p) (void)lddmm_plan_destroy(p);
    for (hipStream_t s : Bt->streams) (void)hipStreamDestroy(s);
    delete Bt;
}

static void sync_all(lddmm_batch *Bt)
{
    for (hipStream_t s : Bt->streams) check_hip(hipStreamSynchronize(s), "stream sync");
}

static void copy_scalars_async(lddmm_plan *P)
{
    check_hip(hipMemcpyAsync(P->hscal, P->dscal, sizeof(double) * kNumScalars, hipMemcpyDeviceToHost,
                             P->stream),
              "scalar copy");
}

static void capture_member(lddmm_batch *Bt, int b, int max_pcg, double rtol)
{
    lddmm_plan *P = Bt->plans[b];
    MemberGraph &G = Bt->graphs[b];
    // kernel arguments such as beta are baked into the graph: recapture when
    // the plan's enqueue generation moved since the capture
    if (G.exec && G.max_pcg == max_pcg && G.rtol == rtol && G.gen == P->enqueue_gen) return;
    if (G.exec) {
        check_hip(hipGraphExecDestroy(G.exec), "hipGraphExecDestroy");
        G.exec = nullptr;
    }
    const bool timing = P->timing.on;
    P->timing.on = false;  // no event nodes in the graph
    hipGraph_t graph = nullptr;
    check_hip(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
        gn_trial_enqueue(P, max_pcg, rtol, P->px);
        copy_scalars_async(P);
    } catch (...) {
        (void)hipStreamEndCapture(P->stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        P->timing.on = timing;
        throw;
    }
    check_hip(hipStreamEndCapture(P->stream, &graph), "hipStreamEndCapture");
    P->timing.on = timing;
    hipError_t e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    check_hip(e, "hipGraphInstantiate");
    G.max_pcg = max_pcg;
    G.rtol = rtol;
    G.gen = P->enqueue_gen;
}

}  // namespace lddmm

using namespace lddmm;

extern "C" {

lddmm_status lddmm_batch_create(int32_t B, const lddmm_config *cfgs, int32_t nstreams, lddmm_batch **out)
{
    lddmm_batch *Bt = nullptr;
    if (out) *out = nullptr;
    lddmm_status st = bguard([&] {
        if (!out || !cfgs) fail(LDDMM_EINVAL, "NULL argument");
        if (B < 1 || B > 4096) fail(LDDMM_EINVAL, "B must be in [1, 4096]");
        if (nstreams < 1 || nstreams > 32) fail(LDDMM_EINVAL, "nstreams must be in [1, 32]");
        Bt = new lddmm_batch();
        Bt->B = B;
        const int S = std::min(nstreams, B);
        for (int s = 0; s < S; ++s) {
            hipStream_t h;
            check_hip(hipStreamCreateWithFlags(&h, hipStreamNonBlocking), "hipStreamCreate");
            Bt->streams.push_back(h);
        }
        Bt->plans.assign(B, nullptr);
        Bt->graphs.assign(B, MemberGraph{});
        for (int b = 0; b < B; ++b) {
            if (cfgs[b].flags & LDDMM_FLAG_TRANSPORT_ONLY)
                fail(LDDMM_EINVAL, "batch members need full plans");
            lddmm_status s = lddmm_plan_create(&cfgs[b], (void *)Bt->streams[b % S], &Bt->plans[b]);
            if (s != LDDMM_OK)
                fail(s, "member " + std::to_string(b) + ": " + lddmm_last_error());
            // FFT tiles per grid size (the cache makes repeated sizes free)
            s = lddmm_autotune(Bt->plans[b]);
            if (s != LDDMM_OK)
                fail(s, "member " + std::to_string(b) + " autotune: " + lddmm_last_error());
        }
        *out = Bt;
    });
    if (st != LDDMM_OK) batch_free(Bt);
    return st;
}

lddmm_status lddmm_batch_destroy(lddmm_batch *Bt)
{
    return bguard([&] {
        if (!Bt) fail(LDDMM_EINVAL, "batch is NULL");
        (void)hipDeviceSynchronize();
        batch_free(Bt);
    });
}

lddmm_status lddmm_batch_plan(lddmm_batch *Bt, int32_t b, lddmm_plan **plan)
{
    return bguard([&] {
        if (!Bt || !plan) fail(LDDMM_EINVAL, "NULL argument");
        if (b < 0 || b >= Bt->B) fail(LDDMM_EINVAL, "member index out of range");
        *plan = Bt->plans[b];
    });
}

lddmm_status lddmm_batch_set_images(lddmm_batch *Bt, const float *const *m0, const float *const *m1)
{
    return bguard([&] {
        if (!Bt || !m0 || !m1) fail(LDDMM_EINVAL, "NULL argument");
        check_hip(hipDeviceSynchronize(), "device sync");
        for (int b = 0; b < Bt->B; ++b) {
            lddmm_status s = lddmm_set_images(Bt->plans[b], m0[b], m1[b]);
            if (s != LDDMM_OK) fail(s, "member " + std::to_string(b) + ": " + lddmm_last_error());
        }
        sync_all(Bt);
    });
}

lddmm_status lddmm_batch_set_velocity(lddmm_batch *Bt, const float *const *v)
{
    return bguard([&] {
        if (!Bt || !v) fail(LDDMM_EINVAL, "NULL argument");
        check_hip(hipDeviceSynchronize(), "device sync");
        for (int b = 0; b < Bt->B; ++b) {
            lddmm_status s = lddmm_set_velocity(Bt->plans[b], v[b]);
            if (s != LDDMM_OK) fail(s, "member " + std::to_string(b) + ": " + lddmm_last_error());
        }
        sync_all(Bt);
    });
}

lddmm_status lddmm_batch_gn_iterate(lddmm_batch *Bt, int32_t max_pcg, double rtol, int32_t use_graph,
                                    float *const *v_inout, lddmm_newton_info *infos)
{
    return bguard([&] {
        if (!Bt || !v_inout) fail(LDDMM_EINVAL, "NULL argument");
        if (max_pcg < 0) fail(LDDMM_EINVAL, "max_pcg must be >= 0");
        for (int b = 0; b < Bt->B; ++b) {
            lddmm_plan *P = Bt->plans[b];
            if (!P->have_images || !P->have_velocity)
                fail(LDDMM_ESTATE, "member " + std::to_string(b) + " has no velocity state");
            if (!v_inout[b] || (uintptr_t)v_inout[b] % 16) fail(LDDMM_EINVAL, "v_inout entry NULL or misaligned");
            if (P->pc_kind != 0)
                fail(LDDMM_EUNSUPPORTED, "member " + std::to_string(b) + ": the batched iteration runs InvA only");
        }
        check_hip(hipDeviceSynchronize(), "device sync");
        // phase 1: every member's iteration up to the first Armijo trial
        for (int b = 0; b < Bt->B; ++b) {
            lddmm_plan *P = Bt->plans[b];
            if (use_graph) {
                capture_member(Bt, b, max_pcg, rtol);
                check_hip(hipGraphLaunch(Bt->graphs[b].exec, P->stream), "hipGraphLaunch");
            } else {
                gn_trial_enqueue(P, max_pcg, rtol, P->px);
                copy_scalars_async(P);
            }
        }
        sync_all(Bt);
        // phase 2: line-search decisions (Armijo, c1 = 1e-4, halving, 10 trials)
        for (int b = 0; b < Bt->B; ++b) {
            lddmm_plan *P = Bt->plans[b];
            const double *h = P->hscal;
            const long M = 3 * P->N;
            const double J0 = h[S_J0], gv = h[S_GV];
            double alpha = 1.0, Jn = h[S_J1];
            bool ok = Jn <= J0 + 1e-4 * alpha * gv;
            lddmm_newton_info info{};
            info.pcg_iters = (int)h[S_ITERS];
            info.flags = (int)h[S_FLAGS];
            info.rel_res = h[S_REL];
            info.gnorm = h[S_GNORM];
            info.gnorm_rel = h[S_G0] > 0 ? h[S_GNORM] / h[S_G0] : 1.0;
            info.J_before = J0;
            P->g0norm = h[S_G0];
            for (int tries = 1; !ok && tries < 10; ++tries) {
                alpha *= 0.5;
                axpby(P, M, 1.f, P->px, (float)alpha, P->vt, P->v);
                velocity_state(P);
                objective_enqueue(P, S_E, S_MIS, S_REG);
                Jn = fetch_scalar(P, S_E);
                ok = Jn <= J0 + 1e-4 * alpha * gv;
            }
            if (!ok) {
                copy_kernel(P, M, P->px, P->v);
                velocity_state(P);
                alpha = 0.0;
                Jn = J0;
            }
            copy_kernel(P, M, P->v, v_inout[b]);
            info.alpha = alpha;
            info.J_after = Jn;
            if (infos) infos[b] = info;
        }
        sync_all(Bt);
    });
}

}  // extern "C"
