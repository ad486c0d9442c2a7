// Batched form: many independent registrations (uneven grid sizes) advanced
// together.  Members of one configuration (grid size, N_t, regularisation,
// beta, flags) form a group whose workspaces sit in one batched plan: every
// kernel of a Gauss-Newton iteration is launched once for all members of the
// group, the member index a grid dimension (see Mb), so a phase of the
// iteration -- a transport step, a transform pass, a reduction, a PCG scalar
// update -- is one launch per group instead of one per member.  The
// iteration up to the first Armijo trial (gradient, eps_K, fixed-count PCG
// with device-resident scalars predicated per member, <g, v~>, the trial
// state and J) of every group is captured once into one hipGraph for the
// whole batch and replayed: the groups' streams fork from the first and join
// it again inside the capture, so the groups still run side by side.  Only
// the line-search decisions need the
// host; rejected trials (rare) run eagerly on the member alone, through the
// member's view of its group.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

namespace lddmm {

struct Group {
    lddmm_plan *P = nullptr;  // the batched plan of the group's members
    std::vector<int> members;  // batch indices, in member order
    unsigned long gen = 0;     // the plan's enqueue generation at the capture
};

}  // namespace lddmm

struct lddmm_batch {
    int B = 0;
    std::vector<lddmm::Group> groups;
    std::vector<hipStream_t> streams;
    // the batch's captured Gauss-Newton trial iteration, its arguments, and
    // the fork / join events of the capture (one per stream)
    hipGraphExec_t exec = nullptr;
    int max_pcg = -1;
    double rtol = 0.0;
    std::vector<hipEvent_t> ev_fork, ev_join;
    std::vector<lddmm_plan *> views;  // member b's plan: a view of its group's plan
    std::vector<int> group_of, index_of;
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
    for (lddmm_plan *V : Bt->views) view_free(V);
    if (Bt->exec) (void)hipGraphExecDestroy(Bt->exec);
    for (Group &g : Bt->groups)
        if (g.P) (void)lddmm_plan_destroy(g.P);
    for (hipEvent_t e : Bt->ev_fork) (void)hipEventDestroy(e);
    for (hipEvent_t e : Bt->ev_join) (void)hipEventDestroy(e);
    for (hipStream_t s : Bt->streams) (void)hipStreamDestroy(s);
    delete Bt;
}

static void sync_all(lddmm_batch *Bt)
{
    for (hipStream_t s : Bt->streams) check_hip(hipStreamSynchronize(s), "stream sync");
}

static bool same_config(const lddmm_config &a, const lddmm_config &b)
{
    return a.n[0] == b.n[0] && a.n[1] == b.n[1] && a.n[2] == b.n[2] && a.nt == b.nt && a.reg == b.reg &&
           a.leray == b.leray && a.flags == b.flags && a.beta == b.beta;
}

// the group's state as its members' views see it
static void to_views(lddmm_batch *Bt, const Group &g)
{
    const lddmm_plan *P = g.P;
    for (int b : g.members) {
        lddmm_plan *V = Bt->views[b];
        V->have_images = P->have_images;
        V->have_velocity = P->have_velocity;
        V->have_grad = P->have_grad;
        V->have_matvec = P->have_matvec;
        V->have_disp = P->have_disp;
        V->have_vjp = P->have_vjp;
        V->boxes_valid = P->boxes_valid;
        V->vel_gen = P->vel_gen;
        V->gather_mode = P->gather_mode;
        V->gather_mode3 = P->gather_mode3;
        V->departure_mode = P->departure_mode;
        V->gather_tuned = P->gather_tuned;
        V->fft = P->fft;
    }
}

// members' settings the group's launches take as one argument: beta (equal
// over the group), the preconditioner (InvA)
static void from_views(lddmm_batch *Bt, Group &g)
{
    lddmm_plan *P = g.P;
    const double beta = Bt->views[g.members[0]]->cfg.beta;
    for (int b : g.members) {
        const lddmm_plan *V = Bt->views[b];
        if (V->cfg.beta != beta)
            fail(LDDMM_EUNSUPPORTED, "members " + std::to_string(g.members[0]) + " and " + std::to_string(b) +
                                         " share a grid size but not beta");
        if (V->pc_kind != 0)
            fail(LDDMM_EUNSUPPORTED, "member " + std::to_string(b) + ": the batched iteration runs InvA only");
    }
    if (P->cfg.beta != beta) {
        P->cfg.beta = beta;
        ++P->enqueue_gen;  // beta is an argument of the captured kernels
    }
}

// every member's scalars into its block of the pinned host mirror
static void copy_scalars_async(lddmm_plan *P)
{
    if (P->mb.count == 1)
        check_hip(hipMemcpyAsync(P->hscal, P->dscal, sizeof(double) * kNumScalars, hipMemcpyDeviceToHost, P->stream),
                  "scalar copy");
    else
        check_hip(hipMemcpy2DAsync(P->hscal, sizeof(double) * kHostScalars, P->dscal, (size_t)P->mb.stride,
                                   sizeof(double) * kNumScalars, (size_t)P->mb.count, hipMemcpyDeviceToHost,
                                   P->stream),
                  "scalar copy");
}

// One graph for the whole batch: the first stream begins the capture, the
// others join it through an event, every group enqueues its trial iteration
// on its own stream, and the others' events join the first stream again
// before the capture ends.  Kernel arguments such as beta are baked into the
// graph: it is captured again when an argument or a group plan's enqueue
// generation moved.
static void capture_batch(lddmm_batch *Bt, int max_pcg, double rtol)
{
    bool fresh = Bt->exec && Bt->max_pcg == max_pcg && Bt->rtol == rtol;
    for (const Group &g : Bt->groups) fresh = fresh && g.gen == g.P->enqueue_gen;
    if (fresh) return;
    if (Bt->exec) {
        check_hip(hipGraphExecDestroy(Bt->exec), "hipGraphExecDestroy");
        Bt->exec = nullptr;
    }
    const size_t S = Bt->streams.size();
    while (Bt->ev_fork.size() < S) {
        hipEvent_t a = nullptr, b = nullptr;
        check_hip(hipEventCreateWithFlags(&a, hipEventDisableTiming), "hipEventCreateWithFlags");
        Bt->ev_fork.push_back(a);
        check_hip(hipEventCreateWithFlags(&b, hipEventDisableTiming), "hipEventCreateWithFlags");
        Bt->ev_join.push_back(b);
    }
    std::vector<bool> timing;
    for (Group &g : Bt->groups) {
        timing.push_back(g.P->timing.on);
        g.P->timing.on = false;  // no event nodes in the graph
    }
    hipStream_t s0 = Bt->streams[0];
    hipGraph_t graph = nullptr;
    check_hip(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
        check_hip(hipEventRecord(Bt->ev_fork[0], s0), "hipEventRecord");
        for (size_t i = 1; i < S; ++i) check_hip(hipStreamWaitEvent(Bt->streams[i], Bt->ev_fork[0], 0), "fork");
        for (Group &g : Bt->groups) {
            gn_trial_enqueue(g.P, max_pcg, rtol, g.P->px);
            copy_scalars_async(g.P);
        }
        for (size_t i = 1; i < S; ++i) {
            check_hip(hipEventRecord(Bt->ev_join[i], Bt->streams[i]), "hipEventRecord");
            check_hip(hipStreamWaitEvent(s0, Bt->ev_join[i], 0), "join");
        }
    } catch (...) {
        (void)hipStreamEndCapture(s0, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        for (size_t i = 0; i < Bt->groups.size(); ++i) Bt->groups[i].P->timing.on = timing[i];
        throw;
    }
    check_hip(hipStreamEndCapture(s0, &graph), "hipStreamEndCapture");
    for (size_t i = 0; i < Bt->groups.size(); ++i) Bt->groups[i].P->timing.on = timing[i];
    hipError_t e = hipGraphInstantiate(&Bt->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    check_hip(e, "hipGraphInstantiate");
    Bt->max_pcg = max_pcg;
    Bt->rtol = rtol;
    for (Group &g : Bt->groups) g.gen = g.P->enqueue_gen;
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
        for (int b = 0; b < B; ++b) {
            size_t bytes = 0;
            const lddmm_status s = lddmm_workspace_bytes(&cfgs[b], &bytes);
            if (s != LDDMM_OK) fail(s, "member " + std::to_string(b) + ": " + lddmm_last_error());
            if (cfgs[b].flags & LDDMM_FLAG_TRANSPORT_ONLY) fail(LDDMM_EINVAL, "batch members need full plans");
        }
        Bt = new lddmm_batch();
        Bt->B = B;
        Bt->group_of.assign(B, -1);
        Bt->index_of.assign(B, -1);
        for (int b = 0; b < B; ++b) {
            int g = 0;
            while (g < (int)Bt->groups.size() && !same_config(Bt->groups[g].P ? Bt->groups[g].P->cfg : cfgs[Bt->groups[g].members[0]], cfgs[b]))
                ++g;
            if (g == (int)Bt->groups.size()) Bt->groups.emplace_back();
            Bt->group_of[b] = g;
            Bt->index_of[b] = (int)Bt->groups[g].members.size();
            Bt->groups[g].members.push_back(b);
        }
        const int S = std::min<int>(nstreams, (int)Bt->groups.size());
        for (int s = 0; s < S; ++s) {
            hipStream_t h;
            check_hip(hipStreamCreateWithFlags(&h, hipStreamNonBlocking), "hipStreamCreate");
            Bt->streams.push_back(h);
        }
        for (int g = 0; g < (int)Bt->groups.size(); ++g) {
            Group &G = Bt->groups[g];
            G.P = create_plan(&cfgs[G.members[0]], (void *)Bt->streams[g % S], (int)G.members.size());
            // FFT tiles per grid size (timed on the batched launches)
            const lddmm_status s = lddmm_autotune(G.P);
            if (s != LDDMM_OK) fail(s, "group autotune: " + std::string(lddmm_last_error()));
        }
        Bt->views.assign(B, nullptr);
        for (int b = 0; b < B; ++b)
            Bt->views[b] = member_view(Bt->groups[Bt->group_of[b]].P, Bt->index_of[b]);
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
        *plan = Bt->views[b];
    });
}

lddmm_status lddmm_batch_set_images(lddmm_batch *Bt, const float *const *m0, const float *const *m1)
{
    return bguard([&] {
        if (!Bt || !m0 || !m1) fail(LDDMM_EINVAL, "NULL argument");
        check_hip(hipDeviceSynchronize(), "device sync");
        for (int b = 0; b < Bt->B; ++b) {
            const lddmm_status s = lddmm_set_images(Bt->views[b], m0[b], m1[b]);
            if (s != LDDMM_OK) fail(s, "member " + std::to_string(b) + ": " + lddmm_last_error());
        }
        for (Group &g : Bt->groups) {
            g.P->have_images = 1;
            g.P->have_velocity = 0;
            to_views(Bt, g);
        }
        sync_all(Bt);
    });
}

lddmm_status lddmm_batch_set_velocity(lddmm_batch *Bt, const float *const *v)
{
    return bguard([&] {
        if (!Bt || !v) fail(LDDMM_EINVAL, "NULL argument");
        for (int b = 0; b < Bt->B; ++b)
            if (!v[b] || (uintptr_t)v[b] % 16) fail(LDDMM_EINVAL, "v entry NULL or misaligned");
        for (const Group &g : Bt->groups)
            if (!g.P->have_images) fail(LDDMM_ESTATE, "set_images has not been called");
        check_hip(hipDeviceSynchronize(), "device sync");
        // each member's velocity into its workspace, then the per-velocity
        // state of all members of a group in batched launches
        for (int b = 0; b < Bt->B; ++b) {
            lddmm_plan *V = Bt->views[b];
            copy_kernel(V, 3 * V->N, v[b], V->v);
        }
        for (Group &g : Bt->groups) {
            velocity_state(g.P);
            to_views(Bt, g);
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
            const lddmm_plan *V = Bt->views[b];
            if (!V->have_images || !V->have_velocity)
                fail(LDDMM_ESTATE, "member " + std::to_string(b) + " has no velocity state");
            if (!v_inout[b] || (uintptr_t)v_inout[b] % 16) fail(LDDMM_EINVAL, "v_inout entry NULL or misaligned");
        }
        for (Group &g : Bt->groups) from_views(Bt, g);
        check_hip(hipDeviceSynchronize(), "device sync");
        // phase 1: every group's iteration up to the first Armijo trial (one
        // graph for the batch, or eagerly on the groups' streams)
        if (use_graph) {
            capture_batch(Bt, max_pcg, rtol);
            check_hip(hipGraphLaunch(Bt->exec, Bt->streams[0]), "hipGraphLaunch");
        } else {
            for (Group &g : Bt->groups) {
                gn_trial_enqueue(g.P, max_pcg, rtol, g.P->px);
                copy_scalars_async(g.P);
            }
        }
        sync_all(Bt);
        for (Group &g : Bt->groups) to_views(Bt, g);
        // phase 2: line-search decisions (Armijo, c1 = 1e-4, halving, 10 trials)
        for (int b = 0; b < Bt->B; ++b) {
            lddmm_plan *P = Bt->views[b];
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
