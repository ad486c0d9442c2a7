// C ABI of the gfx950 LDDMM library: plan management and the host-side
// sequencing of the Gauss-Newton-Krylov hot path (Algorithm "GNK" of
// arXiv 2008.12820).  No arithmetic on fields happens here; every step runs
// in the kernels of fft.hip, transport.hip and linalg.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>

#include "internal.hpp"

namespace lddmm {

static thread_local std::string g_last_error;

void fail(lddmm_status s, const std::string &msg) { throw Error{s, msg}; }
void set_last_error(const std::string &msg) { g_last_error = msg; }

void check_hip(hipError_t e, const char *what)
{
    if (e != hipSuccess) fail(LDDMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

const char *kernel_name(int id)
{
    static const char *names[K_NUM_KERNELS] = {
        "r2c_x3", "fft_cols", "x1_symbol", "c2r_x3", "departure", "state_step", "gather_vec",
        "adj_coef", "adj_step", "incstate_init", "incstate_step", "body_force", "dot", "vecop",
        "pack", "adj_body", "fd8"};
    return (id >= 0 && id < K_NUM_KERNELS) ? names[id] : "unknown";
}

Scope::Scope(lddmm_plan *p, int k) : P(p), kid(k)
{
    PlanTiming &T = P->timing;
    if (!T.on || (T.only >= 0 && T.only != k)) return;
    if (T.used == T.pool.size()) {
        hipEvent_t a, b;
        check_hip(hipEventCreate(&a), "hipEventCreate");
        check_hip(hipEventCreate(&b), "hipEventCreate");
        T.pool.emplace_back(a, b);
        T.kid.push_back(k);
    }
    slot = (int)T.used++;
    T.kid[slot] = k;
    check_hip(hipEventRecord(T.pool[slot].first, P->stream), "hipEventRecord");
}

Scope::~Scope() noexcept(false)
{
    if (slot >= 0) (void)hipEventRecord(P->timing.pool[slot].second, P->stream);
}

template <class F>
static lddmm_status guard(F &&f)
{
    try {
        f();
        return LDDMM_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return LDDMM_ENOMEM;
    } catch (...) {
        g_last_error = "unexpected exception";
        return LDDMM_EDEVICE;
    }
}

static bool smooth235(int n)
{
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

static void validate(const lddmm_config *cfg)
{
    if (!cfg) fail(LDDMM_EINVAL, "config is NULL");
    for (int d = 0; d < 3; ++d) {
        const int n = cfg->n[d];
        if (n < 8 || n > 1024 || (n & 1) || !smooth235(n))
            fail(LDDMM_EINVAL, "grid size n[" + std::to_string(d) + "] = " + std::to_string(n) +
                                   " must be even, in [8, 1024], with prime factors 2, 3, 5 only");
    }
    if (cfg->nt < 1 || cfg->nt > 256) fail(LDDMM_EINVAL, "nt must be in [1, 256]");
    if (cfg->reg != LDDMM_REG_H1S && cfg->reg != LDDMM_REG_H2S)
        fail(LDDMM_EINVAL, "reg must be LDDMM_REG_H1S or LDDMM_REG_H2S");
    if (!(std::isfinite(cfg->beta) && cfg->beta > 0.0)) fail(LDDMM_EINVAL, "beta must be finite and > 0");
    if (cfg->leray != 0 && cfg->leray != 1) fail(LDDMM_EINVAL, "leray must be 0 or 1");
    if (cfg->flags & ~(LDDMM_FLAG_TRANSPORT_ONLY | LDDMM_FLAG_FD8 | LDDMM_FLAG_LINEAR_IP))
        fail(LDDMM_EINVAL, "unknown bits in flags");
}

// Sub-allocation plan of the arena, in bytes, each piece 256-byte aligned.
struct Layout {
    size_t off[40];
    size_t len[40];
    int n = 0;
    size_t total = 0;
    size_t add(size_t bytes)
    {
        size_t o = total;
        len[n] = bytes;
        off[n++] = o;
        total += (bytes + 255) & ~size_t(255);
        return o;
    }
};

static bool transport_only(const lddmm_config *cfg) { return cfg->flags & LDDMM_FLAG_TRANSPORT_ONLY; }

static int spectral_slots(const lddmm_config *cfg)
{
    return transport_only(cfg) ? 9 : std::max(9, 4 * std::min(cfg->nt + 1, 4));
}

// Pieces the transport-only plan does not need get zero bytes.
static Layout make_layout(const lddmm_config *cfg)
{
    const size_t N = (size_t)cfg->n[0] * cfg->n[1] * cfg->n[2];
    const size_t nt = (size_t)cfg->nt;
    const size_t f = sizeof(float) * N;
    const size_t spec = sizeof(float2) * (size_t)cfg->n[0] * cfg->n[1] * (cfg->n[2] / 2 + 1);
    const size_t full = transport_only(cfg) ? 0 : 1;
    Layout L;
    L.add(full * f);                       // 0 m0
    L.add(full * f);                       // 1 m1
    L.add(3 * f);                          // 2 v
    L.add(3 * f);                          // 3 dX
    L.add(3 * f);                          // 4 dXa
    L.add((nt + 1) * f);                   // 5 m
    L.add(3 * (nt + 1) * f);               // 6 G
    L.add(full * 3 * nt * f);              // 7 GX
    L.add(f);                              // 8 delta
    L.add(f);                              // 9 coef
    L.add((nt + 1) * f);                   // 10 lam
    L.add(full * 2 * f);                   // 11 mt
    L.add(full * std::max<size_t>(nt - 1, 1) * f);  // 12 src
    L.add(3 * f);                          // 13 b
    L.add(3 * f);                          // 14 tmp3
    L.add(full * 3 * f);                   // 15 g
    // 16..21 PCG x r z p q, Newton step vt; r, z and q also hold the spectra r^,
    // p^ and (H p)^ of the spectral-domain loop, so they take either size
    const size_t rzq = std::max(3 * f, 3 * spec);
    for (int i = 0; i < 6; ++i) L.add(full * ((i == 1 || i == 2 || i == 4) ? rzq : 3 * f));
    L.add(spectral_slots(cfg) * 2 * spec);  // 22 spec (slots sized for FP64)
    // 23 red: two sets of partials, or one per x1 column tile and field
    const size_t red_len = std::max<size_t>(2 * kRedBlocks, 3 * ((size_t)cfg->n[1] * (cfg->n[2] / 2) + cfg->n[0]));
    L.add(sizeof(double) * red_len);
    L.add(sizeof(double) * 2 * kNumScalars);  // 24 dscal (two banks)
    L.add(2 * tile_boxes_bytes(cfg->n));     // 25 stencil extents per gather tile (dX, dXa)
    L.add(sizeof(double) * kHistMax);       // 26 PCG residual history
    return L;
}

static void plan_free(lddmm_plan *P)
{
    if (!P) return;
    fft_free(P);
    if (P->side) {
        (void)hipStreamSynchronize(P->side);
        (void)hipStreamDestroy(P->side);
    }
    if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
    if (P->ev_join) (void)hipEventDestroy(P->ev_join);
    if (P->h0buf) (void)hipFree(P->h0buf);
    if (P->coarse) (void)lddmm_plan_destroy(P->coarse);
    if (P->arena) (void)hipFree(P->arena);
    if (P->hscal) (void)hipHostFree(P->hscal);
    for (hipEvent_t e : P->ev_poll)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : P->ev_inner)
        if (e) (void)hipEventDestroy(e);
    for (auto &pr : P->timing.pool) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    delete P;
}

static void need(const void *p, const char *name)
{
    if (!p) fail(LDDMM_EINVAL, std::string(name) + " is NULL");
}

// device array argument: non-NULL unless optional, 16-byte aligned
static void need_dev(const void *p, const char *name, bool optional = false)
{
    if (!p) {
        if (optional) return;
        fail(LDDMM_EINVAL, std::string(name) + " is NULL");
    }
    if ((uintptr_t)p % 16 != 0) fail(LDDMM_EINVAL, std::string(name) + " is not 16-byte aligned");
}

static void need_full(const lddmm_plan *P)
{
    if (transport_only(&P->cfg))
        fail(LDDMM_EUNSUPPORTED, "this plan was created with LDDMM_FLAG_TRANSPORT_ONLY");
}

static void need_velocity(const lddmm_plan *P)
{
    need_full(P);
    if (!P->have_images) fail(LDDMM_ESTATE, "set_images has not been called");
    if (!P->have_velocity) fail(LDDMM_ESTATE, "set_velocity has not been called since the last change");
}

// device-to-device copies run as a kernel so that every sequence stays
// capturable in a graph
static void copy_dev(lddmm_plan *P, float *dst, const float *src, long count)
{
    if (dst == src) return;
    copy_kernel(P, count, src, dst);
}

static void zero_dev(lddmm_plan *P, float *dst, long count)
{
    fill(P, count, 0.f, dst);
}

// ---------------------------------------------------------------------------
// operators
// ---------------------------------------------------------------------------
// first derivatives with the plan's scheme: spectral, or the FD8 stencil
// (LDDMM_FLAG_FD8); gradients: three outputs per input
static void gradients(lddmm_plan *P, const std::vector<const float *> &in, const std::vector<float *> &out)
{
    if (!(P->cfg.flags & LDDMM_FLAG_FD8)) {
        spectral_apply(P, SOP_GRAD, in, out);
        return;
    }
    for (size_t f = 0; f < in.size(); ++f) launch_fd8_grad(P, in[f], out[3 * f], out[3 * f + 1], out[3 * f + 2]);
}

static void divergence(lddmm_plan *P, const float *v, float *out)
{
    const long N = P->N;
    if (P->cfg.flags & LDDMM_FLAG_FD8)
        launch_fd8_div(P, v, out);
    else
        spectral_apply(P, SOP_DIV, {v, v + N, v + 2 * N}, {out});
}

void velocity_state(lddmm_plan *P)
{
    const long N = P->N;
    const int nt = P->nt;
    ++P->vel_gen;
    launch_departure(P, P->v, P->dX, P->dXa);
    copy_dev(P, P->m, P->m0, N);
    for (int j = 0; j < nt; ++j)
        launch_interp(P, 1, P->m + (long)j * N, P->dX, P->m + (long)(j + 1) * N, K_STATE_STEP);
    std::vector<const float *> in;
    std::vector<float *> out;
    for (int j = 0; j <= nt; ++j) {
        in.push_back(P->m + (long)j * N);
        for (int c = 0; c < 3; ++c) out.push_back(P->G + ((long)j * 3 + c) * N);
    }
    gradients(P, in, out);
    launch_interp(P, 3 * nt, P->G, P->dX, P->GX, K_GATHER_VEC);
    divergence(P, P->v, P->delta);
    launch_adj_coef(P);
    P->have_velocity = 1;
    P->have_grad = 0;
    P->have_matvec = 0;
    P->have_disp = 1;
    P->have_vjp = 0;
}

// Without the Leray projection K = I, so the assembly is pointwise in b:
// out = beta (A w) + b.  A w (the FP64 forward chain of the regularisation
// operator) is written straight into out, which never aliases w, and b is
// not transformed at all.
static bool assemble_pointwise(const lddmm_plan *P) { return !P->cfg.leray; }

// The assembly beta A w + K b needs the forward transform of w, which depends
// on the input alone: with overlap on and outside stream capture it is started
// on the side stream (forked from the plan's stream) while the transport
// sweeps run, and the assembly joins it; without the Leray projection the
// side stream computes the whole of A w into out.  Otherwise everything stays
// on the plan's stream.
static bool assemble_prefetch(lddmm_plan *P, const float *w, float *out)
{
    if (!P->overlap) return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    check_hip(hipStreamIsCapturing(P->stream, &cs), "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) return false;
    if (!P->side) {  // created on first use, default priority
        check_hip(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking), "hipStreamCreateWithFlags");
        check_hip(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming), "hipEventCreateWithFlags");
        check_hip(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming), "hipEventCreateWithFlags");
    }
    const long N = P->N;
    check_hip(hipEventRecord(P->ev_fork, P->stream), "hipEventRecord");
    check_hip(hipStreamWaitEvent(P->side, P->ev_fork, 0), "hipStreamWaitEvent");
    hipStream_t main = P->stream;
    P->stream = P->side;
    try {
        if (assemble_pointwise(P))
            spectral_apply(P, SOP_REG, {w, w + N, w + 2 * N}, {out, out + N, out + 2 * N});
        else
            spectral_forward(P, SOP_ASSEMBLE, {w, w + N, w + 2 * N}, 3);
    } catch (...) {
        P->stream = main;
        throw;
    }
    P->stream = main;
    check_hip(hipEventRecord(P->ev_join, P->side), "hipEventRecord");
    return true;
}

static void assemble(lddmm_plan *P, const float *w, const float *b, float *out, bool w_started = false)
{
    const long N = P->N;
    if (w_started) check_hip(hipStreamWaitEvent(P->stream, P->ev_join, 0), "hipStreamWaitEvent");
    if (assemble_pointwise(P)) {
        if (!w_started) spectral_apply(P, SOP_REG, {w, w + N, w + 2 * N}, {out, out + N, out + 2 * N});
        const double beta = P->beta_sym > 0.0 ? P->beta_sym : P->cfg.beta;  // the symbol's beta
        axpby(P, 3 * N, (float)beta, out, 1.f, b, out);
        return;
    }
    spectral_apply(P, SOP_ASSEMBLE, {w, w + N, w + 2 * N, b, b + N, b + 2 * N},
                   {out, out + N, out + 2 * N}, w_started ? 3 : 0);
}

// g and <g,g> (slot S_GG), no host synchronisation
void gradient_enqueue(lddmm_plan *P, float *g)
{
    const long N = P->N;
    const int nt = P->nt;
    float *lam = P->lam;
    const bool started = assemble_prefetch(P, P->v, g);
    axpby(P, N, 1.f, P->m1, -1.f, P->m + (long)nt * N, lam + (long)nt * N);
    for (int j = nt - 1; j >= 1; --j) launch_adj_step(P, lam + (long)(j + 1) * N, lam + (long)j * N, 1.f);
    launch_adj_body(P, lam + N, 1.f, lam, lam, lam + (long)nt * N, 1.f);
    assemble(P, P->v, P->b, g, started);
    dot_async(P, g, g, 3 * N, S_GG, P->h3);
    P->have_grad = 1;
}

static double gradient_impl(lddmm_plan *P, float *g)
{
    gradient_enqueue(P, g);
    const double gn = std::sqrt(fetch_scalar(P, S_GG));
    if (P->g0norm == 0.0) {
        P->g0norm = gn;
        dev_set_scalar(P, S_G0, gn);
    }
    return gn;
}

// The transport sweeps of the matvec (eqs. incsta, incadj, matvec): the
// incremental state from vt, the incremental adjoint and the body force into
// P->b; after_start() runs once the incremental-state start is enqueued.
template <class F>
static void matvec_sweeps(lddmm_plan *P, const float *vt, F &&after_start)
{
    const long N = P->N;
    const int nt = P->nt;
    float *mt[2] = {P->mt, P->mt + N};
    launch_incstate_init(P, vt, mt[0]);
    after_start();
    for (int j = 1; j < nt; ++j)
        launch_incstate_step(P, mt[(j - 1) & 1], P->src + (long)(j - 1) * N, mt[j & 1]);
    const float *mtN = mt[(nt - 1) & 1];
    float *lam = P->lam;
    if (nt == 1) {
        launch_adj_body(P, mtN, -1.f, lam, lam, mtN, -1.f);
    } else {
        launch_adj_step(P, mtN, lam + (long)(nt - 1) * N, -1.f);
        for (int j = nt - 2; j >= 1; --j) launch_adj_step(P, lam + (long)(j + 1) * N, lam + (long)j * N, 1.f);
        launch_adj_body(P, lam + N, 1.f, lam, lam, mtN, -1.f);
    }
}

void matvec_impl(lddmm_plan *P, const float *vt, float *hvt)
{
    bool started = false;
    // the transform of vt is forked after the start gather, which streams at
    // full bandwidth: it then shares the device with the issue-bound steps
    matvec_sweeps(P, vt, [&] { started = assemble_prefetch(P, vt, hvt); });
    assemble(P, vt, P->b, hvt, started);
    P->have_matvec = 1;
}

// H p for the spectral-domain PCG: p in physical space (the transport
// sweeps) and as its spectrum ph (the beta A p term); the result stays in
// the spectral domain (qh), <p, H p> goes to S_KAPPA and alpha follows
static void matvec_spectral(lddmm_plan *P, const float *p, const float2 *ph, float2 *qh)
{
    matvec_sweeps(P, p, [] {});
    spec_forward3(P, P->b, 0);
    spcg_assemble(P, 0, ph, qh, S_KAPPA, P->cfg.leray, kAfterAlpha);
    P->have_matvec = 1;
}

void inv_reg(lddmm_plan *P, const float *r, float *s)
{
    const long N = P->N;
    spectral_apply(P, SOP_INVREG, {r, r + N, r + 2 * N}, {s, s + N, s + 2 * N});
}

static double dot_now(lddmm_plan *P, const float *a, const float *b, long n)
{
    dot_async(P, a, b, n, 1, P->h3);
    return fetch_scalar(P, 1);
}

// ---- zero-velocity Hessian preconditioner InvH0 (Section 2 "Preconditioning",
// eq. h0-pc, Algorithm "PC") ---------------------------------------------------

static double h0_beta(const lddmm_plan *P) { return P->cfg.beta < 5e-2 ? 5e-2 : P->cfg.beta; }

// out = H0 s = beta0 A s + grad m(1) (grad m(1) . s), with grad m(1) the stored
// gradient of the template transported by the current velocity
static void h0_apply(lddmm_plan *P, const float *s, float *out)
{
    const long N = P->N;
    spectral_apply(P, SOP_REG, {s, s + N, s + 2 * N}, {out, out + N, out + 2 * N});
    h0_point(P, s, P->G + (long)P->nt * 3 * N, out, (float)h0_beta(P));
}

// (beta0 A)^{-1} r: the InvA symbol with beta0 for the duration of the scope
struct Beta0Scope {
    lddmm_plan *P;
    explicit Beta0Scope(lddmm_plan *p) : P(p) { P->beta_sym = h0_beta(P); }
    ~Beta0Scope() { P->beta_sym = 0.0; }
};

// The vectors of the H0 solves, FP32 spectra of three fields each (see
// spcg_run): [0] the solution (the outer PCG's M^{-1} r), [1] the inner
// residual, [2] the inner search direction, [3] H0 p.  Allocated on first use.
static float2 *h0_vectors(lddmm_plan *P)
{
    if (!P->h0buf) {
        const size_t bytes = sizeof(float2) * 4 * 3 * (size_t)P->fft.spec_stride;
        hipError_t e = hipMalloc((void **)&P->h0buf, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            P->h0buf = nullptr;
            fail(LDDMM_ENOMEM, "InvH0 vectors of " + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
        }
    }
    return reinterpret_cast<float2 *>(P->h0buf);
}

// The stop test of a device-resident PCG loop: iteration k has been
// enqueued; the host reads the stop flag (slot S_DONE of the current bank)
// that iteration k - 1 left, through a pinned copy and an event, so the
// stream holds one iteration ahead and never drains.  An iteration queued
// after the stop is predicated off on the device.  Returns true on a stop.
struct StopPoll {
    lddmm_plan *P;
    hipEvent_t *ev;
    double *host;
    StopPoll(lddmm_plan *p, hipEvent_t *events, double *pinned) : P(p), ev(events), host(pinned)
    {
        for (int i = 0; i < 2; ++i)
            if (!ev[i]) check_hip(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming), "hipEventCreateWithFlags");
    }
    bool after(int it)
    {
        check_hip(hipMemcpyAsync(host + (it & 1), scalars(P) + S_DONE, sizeof(double), hipMemcpyDeviceToHost,
                                 P->stream),
                  "stop flag copy");
        check_hip(hipEventRecord(ev[it & 1], P->stream), "hipEventRecord");
        if (it < 1) return false;
        check_hip(hipEventSynchronize(ev[(it - 1) & 1]), "hipEventSynchronize");
        return host[(it - 1) & 1] != 0.0;
    }
};

struct BankScope {
    lddmm_plan *P;
    int keep;
    BankScope(lddmm_plan *p, int b) : P(p), keep(p->bank) { P->bank = b; }
    ~BankScope() { P->bank = keep; }
};

// the stop flags the vector kernels of P's launches test (Mb::stopped) for
// the duration of the scope: a loop's own and, for an inner solve, the outer
// loop's (either may be NULL)
struct SkipScope {
    lddmm_plan *P;
    Mb keep;
    SkipScope(lddmm_plan *p, const double *own, const double *outer) : P(p), keep(p->mb)
    {
        P->mb.done = own;
        P->mb.done2 = outer;
    }
    ~SkipScope() { P->mb = keep; }
};

// the spectra of the spectral-domain PCG live in the r, z and q buffers of
// the workspace (sized for a physical field or a spectrum): r^ in r, p^ in z,
// (H p)^ in q
static float2 *spec_r(lddmm_plan *P) { return reinterpret_cast<float2 *>(P->pr); }
static float2 *spec_p(lddmm_plan *P) { return reinterpret_cast<float2 *>(P->pz); }

// transform slots of the spectral PCG loops: the forward transforms (the
// right-hand side, the body force, G (G . p)) and the copy of p its inverse
// transform consumes
constexpr int kSlotFwd = 0, kSlotInv = 3;

// qh = H0 p for the spectrum ph of p: beta0 A p pointwise, the rank-one part
// G (G . p) (G = grad m(1)) in physical space between an inverse and a
// forward transform; with kappa, <p, H0 p> into S_KAPPA and alpha.  in: what
// slots kSlotInv.. hold on entry (kFromVector: nothing yet, kCopy: ph,
// kAfterX1: ph after its inverse x1 pass)
enum { kFromVector, kCopy, kAfterX1 };
static void h0_apply_spec(lddmm_plan *P, const float2 *ph, float2 *qh, bool kappa, int in)
{
    const long N = P->N;
    const float *G1 = P->G + (long)P->nt * 3 * N;
    if (in == kFromVector) spec_copy3(P, ph, kSlotInv, false);
    if (in != kAfterX1) x1_pass(P, kSlotInv, 3, true, false);
    x2_pass(P, kSlotInv, 3, true, false);
    if (!x3_rank1(P, kSlotInv, kSlotFwd, G1)) {  // x3 lengths without a register plan
        RealOut ro{};
        RealIn ri{};
        for (int c = 0; c < 3; ++c) {
            ro.p[c] = P->tmp3 + c * N;
            ri.p[c] = P->b + c * N;
        }
        c2r_fields(P, kSlotInv, 3, ro, (float)(1.0 / (double)N));
        h0_rank1(P, P->tmp3, G1, P->b);  // b: free outside the matvec
        r2c_fields(P, ri, 3, kSlotFwd, false);
    }
    x2_pass(P, kSlotFwd, 3, false, false);
    if (kappa && x1_fwd_h0_assemble(P, kSlotFwd, ph, qh)) return;  // x1 pass, assembly, kappa, alpha
    x1_pass(P, kSlotFwd, 3, false, false);
    spcg_assemble(P, kSlotFwd, ph, qh, kappa ? S_KAPPA : -1, 0, kappa ? kAfterAlpha : 0);
}

// sh ~= H0^{-1} rh (spectra): PCG on H0 s = r preconditioned by
// (beta0 A)^{-1}, from s = (beta0 A)^{-1} r, until ||r - H0 s|| <= tol ||r||,
// max_it iterations or <p, H0 p> <= 0; every scalar on the device (bank 1 of
// P), the stop test lagged by one iteration; the vectors as spectra (the
// preconditioner pointwise, one transform round trip per iteration for the
// rank-one part).  outer (may be NULL): the bank-0 scalars of the outer PCG
// this solve preconditions; the solve then does nothing once that PCG has
// stopped and adds its iterations to the outer S_INNER.  rh and sh must not
// be the inner vectors [1..3] of P.
static void invh0_spec(lddmm_plan *P, const float2 *rh, float2 *sh, double tol, int max_it, double *outer)
{
    const long S3 = 3 * P->fft.spec_stride;
    float2 *w = h0_vectors(P);
    float2 *ri = w + S3, *pi = w + 2 * S3, *qi = w + 3 * S3;
    Beta0Scope b0(P);
    BankScope bk(P, 1);
    StopPoll poll(P, P->ev_inner, P->hscal + kNumScalars + 2);
    SkipScope sk0(P, outer ? outer + S_DONE : nullptr, nullptr);
    dev_set_scalar(P, S_RTOL, tol);
    spec_dot(P, rh, rh, S_RR);
    dev_pcg_init(P);  // S_R0 = ||r||; stopped when r = 0
    if (outer) dev_inner_link(P, outer);
    SkipScope sk1(P, scalars(P) + S_DONE, outer ? outer + S_DONE : nullptr);
    spec_invreg3(P, rh, sh);
    h0_apply_spec(P, sh, qi, false, kFromVector);
    axpby(P, 2 * S3, 1.f, (const float *)rh, -1.f, (const float *)qi, (float *)ri);
    // <r, r> and <r, (beta0 A)^{-1} r> of the start residual, p = (beta0 A)^{-1} r
    // (copied into the slots its inverse transform reads)
    spcg_start(P, ri, P->fft.spec_stride, 1.f, nullptr, pi, kSlotInv, S_RR, S_RZ);
    dev_pcg_conv(P);  // the start may already meet the tolerance
    for (int it = 0; it < max_it; ++it) {
        h0_apply_spec(P, pi, qi, true, it == 0 ? kCopy : kAfterX1);                 // kappa, alpha
        spcg_r(P, ri, qi, nullptr, nullptr, S_RR, S_RZN, kAfterConv | kAfterBeta, nullptr);  // r; conv, beta
        spcg_p_x1(P, ri, nullptr, pi, kSlotInv, sh);  // s += alpha p, then p and its x1 pass
        if (poll.after(it)) break;
    }
    if (outer) dev_inner_accum(P, outer);
}

// iterations of the last inner solve on P (synchronises the stream)
static int inner_iterations(lddmm_plan *P)
{
    BankScope bk(P, 1);
    return (int)fetch_scalar(P, S_ITERS);
}

// ---- two-level variant 2LInvH0 (Algorithm "PC", second function) ---------

static bool halves(const lddmm_config &c)
{
    for (int d = 0; d < 3; ++d)
        if (c.n[d] % 4 != 0 || c.n[d] < 16) return false;
    return true;
}

static lddmm_plan *coarse_plan(lddmm_plan *P)
{
    if (!P->coarse) {
        lddmm_config c = P->cfg;
        for (int d = 0; d < 3; ++d) c.n[d] = P->cfg.n[d] / 2;
        lddmm_plan *C = nullptr;
        const lddmm_status st = lddmm_plan_create(&c, (void *)P->stream, &C);
        if (st != LDDMM_OK) fail(st, std::string("half-grid plan: ") + lddmm_last_error());
        P->coarse = C;
    }
    return P->coarse;
}

// three fields: out (grid of C) = Restrict / Prolong of in (grid of F), by
// FP32 transforms on both plans and spectral resampling in between
static void resample3(lddmm_plan *F, const float *in, lddmm_plan *C, float *out)
{
    RealIn ri{};
    for (int c = 0; c < 3; ++c) ri.p[c] = in + c * F->N;
    r2c_fields(F, ri, 3, 0, false);
    x2_pass(F, 0, 3, false, false);
    x1_pass(F, 0, 3, false, false);
    spectral_resample(F, 0, C, 0, 3);
    x1_pass(C, 0, 3, true, false);
    x2_pass(C, 0, 3, true, false);
    RealOut ro{};
    for (int c = 0; c < 3; ++c) ro.p[c] = out + c * C->N;
    c2r_fields(C, 0, 3, ro, (float)(1.0 / (double)C->N));
}

// sh ~= 2LInvH0(rh), spectra.  The paper's steps s_f = (b0 A)^{-1} r,
// s_c = R s_f, coarse PCG on H0_c s_c = R r from s_c, s_f = P s_c + (s_f -
// P R s_f) are run as s_f = (b0 A)^{-1} r + P (s_c - s_c0) with s_c0 =
// (b0 A_c)^{-1} R r, the same coarse start: R and (b0 A)^{-1} commute (the
// same symbol at every kept wavenumber), so R s_f = s_c0.  On spectra the
// restriction R and the prolongation P are coefficient copies (truncation,
// zero padding).  The coarse plan holds R grad m(1) in its grad m_{N_t} slot,
// refreshed per velocity.
static void twolevel_spec(lddmm_plan *P, const float2 *rh, float2 *sh, double tol, int max_it, double *outer,
                          int rz_slot, int after)
{
    lddmm_plan *C = coarse_plan(P);
    // the half-grid H0 and (beta0 A_c)^{-1} take the fine plan's beta0: the
    // identity R (beta0 A)^{-1} = (beta0 A_c)^{-1} R used below needs one beta0
    C->cfg.beta = P->cfg.beta;
    if (P->coarse_gen != P->vel_gen) {
        resample3(P, P->G + (long)P->nt * 3 * P->N, C, C->G + (long)C->nt * 3 * C->N);
        P->coarse_gen = P->vel_gen;
    }
    // the half-grid plan runs no outer PCG of its own: its r, z, q buffers
    // hold R r, s_c0 and s_c
    float2 *rc = spec_r(C), *sc0 = spec_p(C), *sc = reinterpret_cast<float2 *>(C->pq);
    {
        Beta0Scope b0(C);
        two_level_restrict(P, rh, C, rc, sc0);
    }
    invh0_spec(C, rc, sc, tol, max_it, outer);
    Beta0Scope b0(P);
    two_level_prolong(P, rh, sh, C, sc, sc0, rz_slot, after);
}

// zh = M^{-1} rh of the outer PCG for InvH0 / 2LInvH0 (tol_outer: its
// tolerance), then <r, z> into rz_slot and the scalar steps `after`; the
// inner iterations are added to the outer S_INNER
static void precondition_spec(lddmm_plan *P, const float2 *rh, float2 *zh, double tol_outer, int rz_slot, int after)
{
    if (P->pc_kind == 1) {
        invh0_spec(P, rh, zh, P->pc_eps_h0 * tol_outer, P->pc_max_inner, P->dscal);
        spec_dot(P, rh, zh, rz_slot, after);
    } else {
        twolevel_spec(P, rh, zh, P->pc_eps_h0 * tol_outer, P->pc_max_inner, P->dscal, rz_slot, after);
    }
}

// PCG on H x = sign * rhs, x0 = 0, with r, p and H p kept as FP32 spectra
// (internal layout, unnormalised) and x in physical space.  Iteration k:
// kappa = <p, H p>, alpha = <r, z> / kappa, x += alpha p, r -= alpha q,
// z = M^{-1} r, beta = <r, z>_new / <r, z>, p = z + beta p; the stop on
// ||r|| <= rtol ||r0||, max_it iterations or kappa <= 0 (then x = M^{-1} r0
// at the first iteration).  The inner products follow from Parseval's
// identity over the half spectrum, in FP64.  With M^{-1} = (beta A)^{-1}
// (InvA) the preconditioner is pointwise in k and fused into the updates;
// InvH0 and 2LInvH0 run their inner solves on spectra too.  Each iteration
// transforms the body force forward and the new p back (for the transport
// sweeps of the next matvec).  Scalars on the device (bank 0); poll: the
// lagged stop test, or NULL to enqueue max_it iterations, those after a stop
// predicated off.  Slot S_RTOL must hold the tolerance.
static void spcg_run(lddmm_plan *P, const float *rhs, float sign, int max_it, float *x, StopPoll *poll, double rtol)
{
    const long M = 3 * P->N;
    float2 *rh = spec_r(P), *ph = spec_p(P), *qh = reinterpret_cast<float2 *>(P->pq);
    const bool inva = P->pc_kind == 0;
    float2 *zh = inva ? nullptr : h0_vectors(P);
    float *p = P->pp;
    P->pcg_spectral = 1;
    spec_forward3(P, rhs, kSlotFwd);
    if (inva) {
        spcg_start(P, spec_slot(P, kSlotFwd), P->slot_bytes / 8, sign, rh, ph, kSlotInv, S_RR, S_RZ);
        dev_pcg_init(P);
    } else {
        spcg_start(P, spec_slot(P, kSlotFwd), P->slot_bytes / 8, sign, rh, nullptr, -1, S_RR, -1);
        dev_pcg_init(P);
        precondition_spec(P, rh, zh, rtol, S_RZ, 0);
        copy_kernel(P, 6 * P->fft.spec_stride, (const float *)zh, (float *)ph);
        spec_copy3(P, ph, kSlotInv, false);
    }
    spec_inverse3(P, kSlotInv, p);
    fill(P, M, 0.f, x);
    SkipScope sk(P, scalars(P) + S_DONE, nullptr);
    for (int it = 0; it < max_it; ++it) {
        matvec_spectral(P, p, ph, qh);  // kappa, alpha
        dev_pcg_x(P, M, p, x);          // (or x = p0 = M^{-1} r0 after a first-iteration curvature stop)
        const int hist = it < kHistMax ? kAfterHist : 0;
        double *hdst = hist ? P->hist + it : nullptr;
        if (inva) {
            spcg_r(P, rh, qh, nullptr, nullptr, S_RR, S_RZN, kAfterConv | hist | kAfterBeta, hdst);
        } else {
            spcg_r(P, rh, qh, nullptr, nullptr, S_RR, -1, kAfterConv | hist, hdst);
            precondition_spec(P, rh, zh, rtol, S_RZN, kAfterBeta);
        }
        spcg_p_x1(P, rh, zh, ph, kSlotInv);  // p, and its way back to physical space
        spec_inverse3(P, kSlotInv, p, true);
        if (poll && poll->after(it)) break;  // iteration it is queued, predicated off
    }
}

static int pcg_finish(lddmm_plan *P, lddmm_newton_info &info);

// the last PCG on this plan (or, for a batch member, on its group) kept r and p as spectra
static bool spectral_pcg_state(const lddmm_plan *P)
{
    return P->pr && (P->pcg_spectral || (P->view_of && P->view_of->pcg_spectral));
}

// The PCG of the Newton step (spcg_run) with the host's lagged stop test.
static int pcg_impl(lddmm_plan *P, const float *rhs, int max_it, double rtol, float *x,
                    lddmm_newton_info &info)
{
    StopPoll poll(P, P->ev_poll, P->hscal + kNumScalars);
    dev_set_scalar(P, S_RTOL, rtol);
    spcg_run(P, rhs, 1.f, max_it, x, &poll, rtol);
    return pcg_finish(P, info);
}

// the PCG's outcome from the device scalars (synchronises the stream)
static int pcg_finish(lddmm_plan *P, lddmm_newton_info &info)
{
    check_hip(hipMemcpyAsync(P->hscal, P->dscal, sizeof(double) * kNumScalars, hipMemcpyDeviceToHost, P->stream),
              "scalar copy");
    check_hip(hipStreamSynchronize(P->stream), "stream sync");
    const double *h = P->hscal;
    info.pcg_iters = (int)h[S_ITERS];
    info.rel_res = h[S_REL];
    info.inner_iters = (int)h[S_INNER];
    info.flags = (int)h[S_FLAGS];
    P->pcg_hist.assign(std::min(info.pcg_iters, kHistMax), 0.0);
    if (!P->pcg_hist.empty())
        check_hip(hipMemcpy(P->pcg_hist.data(), P->hist, sizeof(double) * P->pcg_hist.size(), hipMemcpyDeviceToHost),
                  "history copy");
    return info.flags;
}

// J into slot sj, its parts into smis and sreg; no host synchronisation
void objective_enqueue(lddmm_plan *P, int sj, int smis, int sreg)
{
    const long N = P->N;
    sqdiff_async(P, P->m + (long)P->nt * N, P->m1, N, smis, 0.5 * P->h3);
    spectral_apply(P, SOP_REG, {P->v, P->v + N, P->v + 2 * N}, {P->tmp3, P->tmp3 + N, P->tmp3 + 2 * N});
    dot_async(P, P->tmp3, P->v, 3 * N, sreg, 0.5 * P->cfg.beta * P->h3);
    dev_sum(P, sj, smis, sreg);
}

static void objective_impl(lddmm_plan *P, double &J, double &mis, double &reg)
{
    objective_enqueue(P, S_E, S_MIS, S_REG);
    mis = fetch_scalar(P, S_MIS);
    reg = fetch_scalar(P, S_REG);
    J = mis + reg;
}

// PCG on H x = -g with every scalar on the device (no host round trip):
// exactly max_it iterations are enqueued and the ones after a stop are
// predicated off, which reproduces the early exit of the host loop.
// g must hold the gradient and slot S_RTOL the tolerance.
void pcg_enqueue(lddmm_plan *P, const float *g, int max_it, float *x)
{
    spcg_run(P, g, -1.f, max_it, x, nullptr, 0.0);
}

// One Gauss-Newton iteration up to and including the first line-search
// trial (alpha = 1), all on the device: gradient, tolerance, J(v), PCG step
// into P->vt, <g, v~>, the old velocity saved in v0, v <- v0 + v~, state
// refresh and J(v0 + v~).  Scalars land in the S_* slots.
void gn_trial_enqueue(lddmm_plan *P, int max_pcg, double rtol, float *v0)
{
    const long M = 3 * P->N;
    gradient_enqueue(P, P->g);
    dev_tolerance(P, rtol);
    objective_enqueue(P, S_J0, S_MIS, S_REG);
    pcg_enqueue(P, P->g, max_pcg, P->vt);
    dot_async(P, P->g, P->vt, M, S_GV, P->h3);
    copy_dev(P, v0, P->v, M);
    axpby(P, M, 1.f, v0, 1.f, P->vt, P->v);
    velocity_state(P);
    objective_enqueue(P, S_J1, S_MIS1, S_REG1);
}

static double tolerance(lddmm_plan *P, double rtol, double gnorm)
{
    if (rtol > 0.0) return rtol;
    const double grel = P->g0norm > 0.0 ? gnorm / P->g0norm : 1.0;
    return std::min(std::sqrt(grel), 0.5);
}

// A plan for members copies of one configuration (1: a plain plan): one
// arena of members workspaces, stride bytes apart (see Mb); twiddles and tile
// choices are shared.  Throws on failure (nothing leaks).
lddmm_plan *create_plan(const lddmm_config *cfg, void *stream, int members)
{
    lddmm_plan *P = new lddmm_plan();
    try {
        P->cfg = *cfg;
        P->stream = (hipStream_t)stream;
        check_hip(hipGetDevice(&P->device), "hipGetDevice");
        P->N = (long)cfg->n[0] * cfg->n[1] * cfg->n[2];
        P->nt = cfg->nt;
        for (int d = 0; d < 3; ++d) P->h[d] = 2.0 * M_PI / cfg->n[d];
        P->h3 = P->h[0] * P->h[1] * P->h[2];
        P->dt = 1.0 / cfg->nt;
        Layout L = make_layout(cfg);
        const size_t total = L.total * (size_t)members;
        hipError_t e = hipMalloc(&P->arena, total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            P->arena = nullptr;
            fail(LDDMM_ENOMEM, "workspace of " + std::to_string(total) + " bytes: " + hipGetErrorString(e));
        }
        P->arena_bytes = total;
        P->mb.stride = members > 1 ? (long long)L.total : 0;
        P->mb.count = members;
        char *a = (char *)P->arena;
        auto F = [&](int i) { return L.len[i] ? (float *)(a + L.off[i]) : nullptr; };
        P->m0 = F(0);
        P->m1 = F(1);
        P->v = F(2);
        P->dX = F(3);
        P->dXa = F(4);
        P->m = F(5);
        P->G = F(6);
        P->GX = F(7);
        P->delta = F(8);
        P->coef = F(9);
        P->lam = F(10);
        P->mt = F(11);
        P->src = F(12);
        P->b = F(13);
        P->tmp3 = F(14);
        P->g = F(15);
        P->px = F(16);
        P->pr = F(17);
        P->pz = F(18);
        P->pp = F(19);
        P->pq = F(20);
        P->vt = F(21);
        P->spec = a + L.off[22];
        P->nspec = spectral_slots(cfg);
        P->slot_bytes = (long)sizeof(double2) * cfg->n[0] * cfg->n[1] * (cfg->n[2] / 2 + 1);
        P->red = (double *)(a + L.off[23]);
        P->red_len = (long)(L.len[23] / sizeof(double));
        P->dscal = (double *)(a + L.off[24]);
        assign_tile_boxes(P, a + L.off[25]);
        P->hist = (double *)(a + L.off[26]);
        check_hip(hipHostMalloc((void **)&P->hscal, sizeof(double) * kHostScalars * members, hipHostMallocDefault),
                  "hipHostMalloc");
        fft_init(P);
    } catch (...) {
        plan_free(P);
        throw;
    }
    return P;
}

// Member b of a batched plan as a plan of its own (host record only): every
// workspace pointer shifted to the member's copy, one member, the group's
// tables, streams and events shared.  Calls on it launch for that member
// alone.  It owns nothing the group owns (view_free releases only what was
// created on it afterwards).
lddmm_plan *member_view(const lddmm_plan *G, int b)
{
    lddmm_plan *V = new lddmm_plan(*G);
    const long long off = G->mb.offset((unsigned)b);
    auto sh = [&](auto *&p) {
        if (p) p = (std::remove_reference_t<decltype(p)>)((char *)p + off);
    };
    for (float **f : {&V->m0, &V->m1, &V->v, &V->dX, &V->dXa, &V->m, &V->G, &V->GX, &V->delta, &V->coef, &V->lam,
                      &V->mt, &V->src, &V->b, &V->tmp3, &V->g, &V->px, &V->pr, &V->pz, &V->pp, &V->pq, &V->vt})
        sh(*f);
    sh(V->spec);
    sh(V->red);
    sh(V->dscal);
    sh(V->hist);
    for (auto &row : V->boxes)
        for (void *&bx : row)
            if (bx) bx = (char *)bx + off;
    V->hscal = G->hscal + (size_t)b * kHostScalars;
    V->mb = Mb{};
    V->view_of = G;
    V->arena = nullptr;
    V->arena_bytes = 0;
    V->h0buf = nullptr;
    V->coarse = nullptr;
    V->timing = PlanTiming{};
    return V;
}

// release what a view created for itself (never the group's shared pieces)
void view_free(lddmm_plan *V)
{
    if (!V) return;
    const lddmm_plan *G = V->view_of;
    if (V->side && V->side != G->side) {
        (void)hipStreamSynchronize(V->side);
        (void)hipStreamDestroy(V->side);
    }
    if (V->ev_fork && V->ev_fork != G->ev_fork) (void)hipEventDestroy(V->ev_fork);
    if (V->ev_join && V->ev_join != G->ev_join) (void)hipEventDestroy(V->ev_join);
    for (int i = 0; i < 2; ++i) {
        if (V->ev_poll[i] && V->ev_poll[i] != G->ev_poll[i]) (void)hipEventDestroy(V->ev_poll[i]);
        if (V->ev_inner[i] && V->ev_inner[i] != G->ev_inner[i]) (void)hipEventDestroy(V->ev_inner[i]);
    }
    if (V->h0buf) (void)hipFree(V->h0buf);
    if (V->coarse) (void)lddmm_plan_destroy(V->coarse);
    for (auto &pr : V->timing.pool) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    delete V;
}

}  // namespace lddmm

using namespace lddmm;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

lddmm_status lddmm_workspace_bytes(const lddmm_config *cfg, size_t *bytes)
{
    return guard([&] {
        validate(cfg);
        need(bytes, "bytes");
        const int n[3] = {cfg->n[0], cfg->n[1], cfg->n[2]};
        size_t tw = 0;
        for (size_t cs : {sizeof(float2), sizeof(double2)}) {
            tw += ((cs * n[0] + 255) & ~size_t(255)) + ((cs * n[1] + 255) & ~size_t(255));
            tw += ((cs * (n[2] / 2) + 255) & ~size_t(255)) + ((cs * n[2] + 255) & ~size_t(255));
        }
        *bytes = make_layout(cfg).total + tw;
    });
}

lddmm_status lddmm_plan_create(const lddmm_config *cfg, void *stream, lddmm_plan **plan)
{
    if (plan) *plan = nullptr;
    return guard([&] {
        validate(cfg);
        need(plan, "plan");
        *plan = create_plan(cfg, stream, 1);
    });
}

lddmm_status lddmm_plan_destroy(lddmm_plan *plan)
{
    return guard([&] {
        need(plan, "plan");
        if (plan->view_of) fail(LDDMM_EINVAL, "a batch member's plan belongs to the batch (lddmm_batch_destroy)");
        (void)hipStreamSynchronize(plan->stream);
        plan_free(plan);
    });
}

lddmm_status lddmm_set_images(lddmm_plan *P, const float *m0, const float *m1)
{
    return guard([&] {
        need(P, "plan");
        need_dev(m0, "m0");
        need_dev(m1, "m1");
        need_full(P);
        copy_dev(P, P->m0, m0, P->N);
        copy_dev(P, P->m1, m1, P->N);
        dev_set_scalar(P, S_G0, 0.0);
        P->have_images = 1;
        P->have_velocity = 0;
        P->g0norm = 0.0;
    });
}

lddmm_status lddmm_set_velocity(lddmm_plan *P, const float *v)
{
    return guard([&] {
        need(P, "plan");
        need_dev(v, "v");
        need_full(P);
        if (!P->have_images) fail(LDDMM_ESTATE, "set_images has not been called");
        copy_dev(P, P->v, v, 3 * P->N);
        velocity_state(P);
    });
}

lddmm_status lddmm_objective(lddmm_plan *P, double *J, double *mismatch, double *reg)
{
    return guard([&] {
        need(P, "plan");
        need_velocity(P);
        double j, m, r;
        objective_impl(P, j, m, r);
        if (J) *J = j;
        if (mismatch) *mismatch = m;
        if (reg) *reg = r;
    });
}

lddmm_status lddmm_gradient(lddmm_plan *P, float *g, double *gnorm)
{
    return guard([&] {
        need(P, "plan");
        need_dev(g, "g");
        need_velocity(P);
        const double gn = gradient_impl(P, g);
        if (gnorm) *gnorm = gn;
    });
}

lddmm_status lddmm_hessian_matvec(lddmm_plan *P, const float *vt, float *hvt)
{
    return guard([&] {
        need(P, "plan");
        need_dev(vt, "vt");
        need_dev(hvt, "hvt");
        if (vt == hvt) fail(LDDMM_EINVAL, "vt and hvt must be distinct");
        need_velocity(P);
        matvec_impl(P, vt, hvt);
    });
}

lddmm_status lddmm_apply_inv_reg(lddmm_plan *P, const float *r, float *s)
{
    return guard([&] {
        need(P, "plan");
        need_dev(r, "r");
        need_dev(s, "s");
        inv_reg(P, r, s);
    });
}

lddmm_status lddmm_newton_step(lddmm_plan *P, int32_t max_pcg, double rtol, float *vt_out,
                               lddmm_newton_info *info)
{
    lddmm_newton_info loc{};
    lddmm_status st = guard([&] {
        need(P, "plan");
        need_dev(vt_out, "vt_out");
        if (max_pcg < 0) fail(LDDMM_EINVAL, "max_pcg must be >= 0");
        need_velocity(P);
        const double gn = gradient_impl(P, P->g);
        loc.gnorm = gn;
        loc.gnorm_rel = P->g0norm > 0 ? gn / P->g0norm : 1.0;
        const double tol = tolerance(P, rtol, gn);
        axpby(P, 3 * P->N, -1.f, P->g, 0.f, nullptr, P->tmp3);
        const int flags = pcg_impl(P, P->tmp3, max_pcg, tol, vt_out, loc);
        if (flags) fail(LDDMM_ENOTCONV, flags & 2 ? "PCG met a non-finite value" : "PCG met non-positive curvature");
    });
    if (info) *info = loc;
    return st;
}

}  // extern "C"

namespace lddmm {

// One Gauss-Newton iteration at the plan's velocity (Algorithm "GNK"): g, J,
// eps_K, PCG on H v~ = -g, Armijo (c1 = 1e-4, halving, 10 trials), state
// refresh.  With eps_n > 0 it returns false without a step when the
// gradient already meets ||g|| <= eps_n ||g0||.
static bool gn_iterate_impl(lddmm_plan *P, int max_pcg, double rtol, double eps_n, lddmm_newton_info &loc)
{
    const long M = 3 * P->N;
    const double gn = gradient_impl(P, P->g);
    loc.gnorm = gn;
    loc.gnorm_rel = P->g0norm > 0 ? gn / P->g0norm : 1.0;
    if (eps_n > 0.0 && gn <= eps_n * P->g0norm) return false;
    double J0, mis, rg;
    objective_impl(P, J0, mis, rg);
    loc.J_before = J0;
    const double tol = tolerance(P, rtol, gn);
    axpby(P, M, -1.f, P->g, 0.f, nullptr, P->tmp3);
    const int flags = pcg_impl(P, P->tmp3, max_pcg, tol, P->vt, loc);
    const double gv = dot_now(P, P->g, P->vt, M);
    float *v0 = P->pq, *vn = P->pp;  // PCG scratch is free now
    copy_dev(P, v0, P->v, M);
    double alpha = 1.0, Jn = J0;
    bool ok = false;
    for (int tries = 0; tries < 10; ++tries) {
        axpby(P, M, 1.f, v0, (float)alpha, P->vt, vn);
        copy_dev(P, P->v, vn, M);
        velocity_state(P);
        objective_impl(P, Jn, mis, rg);
        if (Jn <= J0 + 1e-4 * alpha * gv) {
            ok = true;
            break;
        }
        alpha *= 0.5;
    }
    if (!ok) {
        copy_dev(P, P->v, v0, M);
        velocity_state(P);
        alpha = 0.0;
        Jn = J0;
    }
    loc.alpha = alpha;
    loc.J_after = Jn;
    loc.flags = flags;
    return true;
}

static void set_beta_impl(lddmm_plan *P, double beta)
{
    P->cfg.beta = beta;
    if (P->coarse) P->coarse->cfg.beta = beta;
    P->g0norm = 0.0;
    dev_set_scalar(P, S_G0, 0.0);
    ++P->enqueue_gen;  // beta is an argument of the enqueued kernels
}

}  // namespace lddmm

extern "C" {

lddmm_status lddmm_gn_iterate(lddmm_plan *P, int32_t max_pcg, double rtol, float *v_inout,
                              lddmm_newton_info *info)
{
    lddmm_newton_info loc{};
    lddmm_status st = guard([&] {
        need(P, "plan");
        need_dev(v_inout, "v_inout");
        if (max_pcg < 0) fail(LDDMM_EINVAL, "max_pcg must be >= 0");
        need_velocity(P);
        gn_iterate_impl(P, max_pcg, rtol, 0.0, loc);
        copy_dev(P, v_inout, P->v, 3 * P->N);
        check_hip(hipStreamSynchronize(P->stream), "stream sync");
    });
    if (info) *info = loc;
    return st;
}

lddmm_status lddmm_set_beta(lddmm_plan *P, double beta)
{
    return guard([&] {
        need(P, "plan");
        if (!(beta > 0.0) || !std::isfinite(beta)) fail(LDDMM_EINVAL, "beta must be finite and > 0");
        set_beta_impl(P, beta);
    });
}

lddmm_status lddmm_gn_solve(lddmm_plan *P, const lddmm_solve_opts *o, float *v_inout, lddmm_solve_report *report)
{
    lddmm_solve_report rep{};
    lddmm_status st = guard([&] {
        need(P, "plan");
        need(o, "opts");
        need_dev(v_inout, "v_inout");
        need_full(P);
        if (!P->have_images) fail(LDDMM_ESTATE, "set_images first");
        if (!(o->beta_target > 0.0) || !std::isfinite(o->beta_target)) fail(LDDMM_EINVAL, "beta_target must be > 0");
        if (o->max_gn < 0 || o->max_pcg < 0 || o->max_inner < 1 || o->pc_kind < 0 || o->pc_kind > 2 ||
            !(o->eps_h0 > 0.0 && o->eps_h0 < 1.0) || !(o->eps_n >= 0.0))
            fail(LDDMM_EINVAL, "solve options out of range");
        if (o->pc_kind == 2 && !halves(P->cfg)) fail(LDDMM_EINVAL, "2LInvH0 needs a grid that halves");
        std::vector<double> betas;
        if (o->continuation)
            for (double b = 1.0; b > o->beta_target * (1 + 1e-12); b /= 10.0) betas.push_back(b);
        betas.push_back(o->beta_target);
        const int keep_kind = P->pc_kind, keep_inner = P->pc_max_inner;
        const double keep_eps = P->pc_eps_h0;
        const long M = 3 * P->N;
        copy_dev(P, P->v, v_inout, M);
        velocity_state(P);
        P->have_velocity = 1;
        try {
            for (double b : betas) {
                set_beta_impl(P, b);
                P->pc_kind = b > o->pc_switch ? 0 : o->pc_kind;
                P->pc_eps_h0 = o->eps_h0;
                P->pc_max_inner = o->max_inner;
                ++rep.stages;
                for (int it = 0; it < o->max_gn; ++it) {
                    lddmm_newton_info loc{};
                    if (!gn_iterate_impl(P, o->max_pcg, o->rtol, o->eps_n, loc)) break;
                    ++rep.gn_iters;
                    rep.pcg_iters += loc.pcg_iters;
                    rep.inner_iters += loc.inner_iters;
                    if (loc.alpha == 0.0) break;
                }
            }
        } catch (...) {
            P->pc_kind = keep_kind;
            P->pc_eps_h0 = keep_eps;
            P->pc_max_inner = keep_inner;
            throw;
        }
        P->pc_kind = keep_kind;
        P->pc_eps_h0 = keep_eps;
        P->pc_max_inner = keep_inner;
        const double gn = gradient_impl(P, P->g);
        rep.gnorm_rel = P->g0norm > 0 ? gn / P->g0norm : 1.0;
        double J, mis, rg;
        objective_impl(P, J, mis, rg);
        rep.J = J;
        copy_dev(P, v_inout, P->v, M);
        check_hip(hipStreamSynchronize(P->stream), "stream sync");
    });
    if (report) *report = rep;
    return st;
}

lddmm_status lddmm_transport_forward(lddmm_plan *P, const float *m0, const float *v, float *m1_out,
                                     float *ckpt)
{
    return guard([&] {
        need(P, "plan");
        need_dev(m0, "m0");
        need_dev(v, "v");
        need_dev(m1_out, "m1_out");
        const long N = P->N;
        copy_dev(P, P->v, v, 3 * N);
        P->have_velocity = 0;
        P->have_vjp = 0;
        launch_departure(P, P->v, P->dX, P->dXa);
        P->have_disp = 1;
        float *buf = ckpt ? ckpt : P->m;
        copy_dev(P, buf, m0, N);
        for (int j = 0; j < P->nt; ++j)
            launch_interp(P, 1, buf + (long)j * N, P->dX, buf + (long)(j + 1) * N, K_STATE_STEP);
        copy_dev(P, m1_out, buf + (long)P->nt * N, N);
    });
}

lddmm_status lddmm_transport_vjp(lddmm_plan *P, const float *ckpt, const float *v,
                                 const float *grad_m1, float *grad_m0, float *grad_v)
{
    return guard([&] {
        need(P, "plan");
        need_dev(ckpt, "ckpt");
        need_dev(v, "v");
        need_dev(grad_m1, "grad_m1");
        need_dev(grad_m0, "grad_m0", true);
        need_dev(grad_v, "grad_v", true);
        const long N = P->N;
        const int nt = P->nt;
        copy_dev(P, P->v, v, 3 * N);
        P->have_velocity = 0;
        P->have_vjp = 0;
        launch_departure(P, P->v, P->dX, P->dXa);
        P->have_disp = 1;
        divergence(P, P->v, P->delta);
        launch_adj_coef(P);
        float *lam = P->lam;
        copy_dev(P, lam + (long)nt * N, grad_m1, N);
        for (int j = nt - 1; j >= 0; --j) launch_adj_step(P, lam + (long)(j + 1) * N, lam + (long)j * N, 1.f);
        if (grad_m0) copy_dev(P, grad_m0, lam, N);
        if (grad_v) {
            std::vector<const float *> in;
            std::vector<float *> out;
            for (int j = 0; j <= nt; ++j) {
                in.push_back(ckpt + (long)j * N);
                for (int c = 0; c < 3; ++c) out.push_back(P->G + ((long)j * 3 + c) * N);
            }
            gradients(P, in, out);
            launch_body_force(P, lam, lam + (long)nt * N, 1.f, P->G, P->b);
            axpby(P, 3 * N, -1.f, P->b, 0.f, nullptr, grad_v);
        }
        P->have_vjp = grad_v ? 2 : 1;  // 2: the checkpoint gradients are held too
    });
}

lddmm_status lddmm_reg_energy(lddmm_plan *P, const float *v, float *Av, double *energy)
{
    return guard([&] {
        need(P, "plan");
        need_dev(v, "v");
        need_dev(Av, "Av", true);
        need(energy, "energy");
        const long N = P->N;
        float *out = Av ? Av : P->tmp3;
        spectral_apply(P, SOP_REG, {v, v + N, v + 2 * N}, {out, out + N, out + 2 * N});
        dot_async(P, out, v, 3 * N, 4, 0.5);
        *energy = fetch_scalar(P, 4);
    });
}

lddmm_status lddmm_fft_r2c(lddmm_plan *P, const float *f, float *fhat)
{
    return guard([&] {
        need(P, "plan");
        need_dev(f, "f");
        need_dev(fhat, "fhat");
        RealIn ri{};
        ri.p[0] = f;
        r2c_fields(P, ri, 1, 0, false);
        x2_pass(P, 0, 1, false, false);
        x1_pass(P, 0, 1, false, false);
        pack_standard(P, 0, (float2 *)fhat);
    });
}

lddmm_status lddmm_fft_c2r(lddmm_plan *P, const float *fhat, float *f)
{
    return guard([&] {
        need(P, "plan");
        need_dev(f, "f");
        need_dev(fhat, "fhat");
        unpack_standard(P, (const float2 *)fhat, 0);
        x1_pass(P, 0, 1, true, false);
        x2_pass(P, 0, 1, true, false);
        RealOut ro{};
        ro.p[0] = f;
        c2r_fields(P, 0, 1, ro, (float)(1.0 / (double)P->N));
    });
}

lddmm_status lddmm_spectral_op(lddmm_plan *P, int32_t op, const float *in, float *out)
{
    return guard([&] {
        need(P, "plan");
        need_dev(in, "in");
        need_dev(out, "out");
        const long N = P->N;
        int sop = 0;
        switch (op) {
        case LDDMM_OP_GRAD: sop = SOP_GRAD; break;
        case LDDMM_OP_DIV: sop = SOP_DIV; break;
        case LDDMM_OP_REG: sop = SOP_REG; break;
        case LDDMM_OP_INVREG: sop = SOP_INVREG; break;
        case LDDMM_OP_LERAY: sop = SOP_LERAY; break;
        default: fail(LDDMM_EINVAL, "unknown operator");
        }
        std::vector<const float *> vi;
        std::vector<float *> vo;
        for (int i = 0; i < op_nin(sop); ++i) vi.push_back(in + i * N);
        for (int o = 0; o < op_nout(sop); ++o) vo.push_back(out + o * N);
        // LERAY symbol is independent of cfg.leray; the plan flag only selects K
        spectral_apply(P, sop, vi, vo);
    });
}

lddmm_status lddmm_interp(lddmm_plan *P, int32_t nfields, const float *fields, const float *disp,
                          float *out)
{
    return guard([&] {
        need(P, "plan");
        need_dev(fields, "fields");
        need_dev(disp, "disp");
        need_dev(out, "out");
        if (nfields < 1) fail(LDDMM_EINVAL, "nfields must be >= 1");
        launch_interp(P, nfields, fields, disp, out, K_GATHER_VEC);
    });
}

lddmm_status lddmm_get_field(lddmm_plan *P, int32_t what, int32_t j, float *out)
{
    return guard([&] {
        need(P, "plan");
        need_dev(out, "out");
        const long N = P->N;
        const int nt = P->nt;
        auto need_v = [&] { need_velocity(P); };
        // after a transport-map call the departure points, the divergence and,
        // after a VJP, the adjoint sweep and the checkpoint gradients are held
        const bool tmap = !P->have_velocity && P->have_disp;
        switch (what) {
        case LDDMM_FIELD_DISP:
            if (!tmap) need_v();
            copy_dev(P, out, P->dX, 3 * N);
            break;
        case LDDMM_FIELD_DISP_ADJ:
            if (!tmap) need_v();
            copy_dev(P, out, P->dXa, 3 * N);
            break;
        case LDDMM_FIELD_STATE:
            need_v();
            if (j < 0 || j > nt) fail(LDDMM_EINVAL, "j out of range");
            copy_dev(P, out, P->m + (long)j * N, N);
            break;
        case LDDMM_FIELD_GRAD_STATE:
            if (!(tmap && P->have_vjp == 2)) need_v();
            if (j < 0 || j > nt) fail(LDDMM_EINVAL, "j out of range");
            copy_dev(P, out, P->G + (long)j * 3 * N, 3 * N);
            break;
        case LDDMM_FIELD_DIV:
            if (!(tmap && P->have_vjp)) need_v();
            copy_dev(P, out, P->delta, N);
            break;
        case LDDMM_FIELD_INC_STATE:
            if (!P->have_matvec) fail(LDDMM_ESTATE, "no matvec has been computed");
            copy_dev(P, out, P->mt + (long)((nt - 1) & 1) * N, N);
            break;
        case LDDMM_FIELD_PCG_R:
        case LDDMM_FIELD_PCG_Z:
            if (!spectral_pcg_state(P)) fail(LDDMM_ESTATE, "no PCG has run");
            // the inverse transforms of r and M^{-1} r (InvA: pointwise; InvH0
            // and 2LInvH0: the last inner solve's result)
            if (what == LDDMM_FIELD_PCG_Z && P->pc_kind != 0)
                spec_copy3(P, h0_vectors(P), 0, false);
            else
                spec_copy3(P, spec_r(P), 0, what == LDDMM_FIELD_PCG_Z);
            spec_inverse3(P, 0, out);
            break;
        case LDDMM_FIELD_PCG_P: copy_dev(P, out, P->pp, 3 * N); break;
        case LDDMM_FIELD_PCG_R_HAT:
        case LDDMM_FIELD_PCG_P_HAT: {
            if (!spectral_pcg_state(P)) fail(LDDMM_ESTATE, "no PCG has run");
            const long per = (long)P->cfg.n[0] * P->cfg.n[1] * (P->cfg.n[2] / 2 + 1);
            spec_copy3(P, what == LDDMM_FIELD_PCG_P_HAT ? spec_p(P) : spec_r(P), 0, false);
            for (int c = 0; c < 3; ++c) pack_standard(P, c, reinterpret_cast<float2 *>(out) + c * per);
            break;
        }
        case LDDMM_FIELD_ADJOINT:
            if (!P->have_grad && !P->have_matvec && !(tmap && P->have_vjp))
                fail(LDDMM_ESTATE, "no adjoint has been computed");
            if (j < 0 || j > nt) fail(LDDMM_EINVAL, "j out of range");
            copy_dev(P, out, P->lam + (long)j * N, N);
            break;
        default: fail(LDDMM_EINVAL, "unknown field");
        }
    });
}

lddmm_status lddmm_set_timing(lddmm_plan *P, int32_t enable)
{
    return guard([&] {
        need(P, "plan");
        check_hip(hipStreamSynchronize(P->stream), "stream sync");
        P->timing.on = enable != 0;
        P->timing.only = -1;
        P->timing.used = 0;
    });
}

lddmm_status lddmm_set_timing_only(lddmm_plan *P, int32_t kernel_id)
{
    return guard([&] {
        need(P, "plan");
        if (kernel_id < 0 || kernel_id >= K_NUM_KERNELS) fail(LDDMM_EINVAL, "kernel id out of range");
        check_hip(hipStreamSynchronize(P->stream), "stream sync");
        P->timing.on = true;
        P->timing.only = kernel_id;
        P->timing.used = 0;
    });
}

lddmm_status lddmm_get_timing(lddmm_plan *P, int32_t kernel_id, double *total_ms, int64_t *launches)
{
    return guard([&] {
        need(P, "plan");
        if (kernel_id < 0 || kernel_id >= K_NUM_KERNELS) fail(LDDMM_EINVAL, "kernel id out of range");
        check_hip(hipStreamSynchronize(P->stream), "stream sync");
        double ms = 0.0;
        int64_t cnt = 0;
        for (size_t i = 0; i < P->timing.used; ++i) {
            if (P->timing.kid[i] != kernel_id) continue;
            float t = 0.f;
            check_hip(hipEventElapsedTime(&t, P->timing.pool[i].first, P->timing.pool[i].second),
                      "hipEventElapsedTime");
            ms += t;
            ++cnt;
        }
        if (total_ms) *total_ms = ms;
        if (launches) *launches = cnt;
    });
}

lddmm_status lddmm_autotune(lddmm_plan *P)
{
    return guard([&] {
        need(P, "plan");
        check_hip(hipStreamSynchronize(P->stream), "stream sync");
        autotune_fft(P);
        // the gather strategy is timed on the real displacement field
        if (P->have_velocity) autotune_gather(P);
        ++P->enqueue_gen;
    });
}

lddmm_status lddmm_tuning(lddmm_plan *P, char *buf, size_t len)
{
    return guard([&] {
        need(P, "plan");
        need(buf, "buf");
        const std::string r = tuning_report(P) + " gather_mode=" + std::to_string(P->gather_mode) +
                              "/" + std::to_string(P->gather_mode3) + " departure_mode=" + std::to_string(P->departure_mode) +
                              (P->gather_tuned ? " (tuned)" : "");
        if (len == 0) fail(LDDMM_EINVAL, "len is 0");
        const size_t n = std::min(len - 1, r.size());
        std::memcpy(buf, r.data(), n);
        buf[n] = 0;
    });
}

lddmm_status lddmm_set_preconditioner(lddmm_plan *P, int32_t kind, double eps_h0, int32_t max_inner)
{
    return guard([&] {
        need(P, "plan");
        if (kind < 0 || kind > 2) fail(LDDMM_EINVAL, "kind must be 0 (InvA), 1 (InvH0) or 2 (2LInvH0)");
        if (kind == 2 && !halves(P->cfg))
            fail(LDDMM_EINVAL, "2LInvH0 needs every grid size divisible by 4 and at least 16");
        if (!(eps_h0 > 0.0 && eps_h0 < 1.0)) fail(LDDMM_EINVAL, "eps_h0 must lie in (0, 1)");
        if (max_inner < 1) fail(LDDMM_EINVAL, "max_inner must be >= 1");
        P->pc_kind = kind;
        P->pc_eps_h0 = eps_h0;
        P->pc_max_inner = max_inner;
        ++P->enqueue_gen;
    });
}

lddmm_status lddmm_apply_h0(lddmm_plan *P, const float *s, float *out)
{
    return guard([&] {
        need(P, "plan");
        need_dev(s, "s");
        need_dev(out, "out");
        need_full(P);
        need_velocity(P);
        h0_apply(P, s, out);
    });
}

lddmm_status lddmm_apply_invh0(lddmm_plan *P, const float *r, double tol, int32_t max_inner, float *s,
                               int32_t *iters)
{
    return guard([&] {
        need(P, "plan");
        need_dev(r, "r");
        need_dev(s, "s");
        if (!(tol >= 0.0) || max_inner < 0) fail(LDDMM_EINVAL, "tol must be >= 0 and max_inner >= 0");
        need_full(P);
        need_velocity(P);
        float2 *rh = reinterpret_cast<float2 *>(P->pq), *sh = h0_vectors(P);
        spec_forward3(P, r, kSlotFwd);
        spec_from_slots(P, kSlotFwd, rh);
        invh0_spec(P, rh, sh, tol, max_inner, nullptr);
        spec_copy3(P, sh, kSlotInv, false);
        spec_inverse3(P, kSlotInv, s);
        const int it = inner_iterations(P);
        if (iters) *iters = it;
    });
}

lddmm_status lddmm_apply_2linvh0(lddmm_plan *P, const float *r, double tol, int32_t max_inner, float *s,
                                 int32_t *iters)
{
    return guard([&] {
        need(P, "plan");
        need_dev(r, "r");
        need_dev(s, "s");
        if (!(tol >= 0.0) || max_inner < 0) fail(LDDMM_EINVAL, "tol must be >= 0 and max_inner >= 0");
        if (!halves(P->cfg)) fail(LDDMM_EINVAL, "2LInvH0 needs every grid size divisible by 4 and at least 16");
        need_full(P);
        need_velocity(P);
        float2 *rh = reinterpret_cast<float2 *>(P->pq), *sh = h0_vectors(P);
        spec_forward3(P, r, kSlotFwd);
        spec_from_slots(P, kSlotFwd, rh);
        twolevel_spec(P, rh, sh, tol, max_inner, nullptr, -1, 0);
        spec_copy3(P, sh, kSlotInv, false);
        spec_inverse3(P, kSlotInv, s);
        const int it = inner_iterations(coarse_plan(P));
        if (iters) *iters = it;
    });
}

lddmm_status lddmm_set_overlap(lddmm_plan *P, int32_t enable)
{
    return guard([&] {
        need(P, "plan");
        if (enable != 0 && enable != 1) fail(LDDMM_EINVAL, "enable must be 0 or 1");
        P->overlap = enable;
    });
}

lddmm_status lddmm_set_gather_mode(lddmm_plan *P, int32_t mode)
{
    return guard([&] {
        need(P, "plan");
        if (mode < -1 || mode > 4) fail(LDDMM_EINVAL, "mode must be -1 .. 4");
        P->gather_mode = mode;
        P->gather_mode3 = -1;
        P->departure_mode = mode < 0 ? -1 : mode == 0 ? 0 : (mode & 1) ? 1 : 2;
        ++P->enqueue_gen;
    });
}

lddmm_status lddmm_pcg_history(lddmm_plan *P, double *rel_res, int32_t len, int32_t *count)
{
    return guard([&] {
        need(P, "plan");
        if (len < 0) fail(LDDMM_EINVAL, "len must be >= 0");
        if (len > 0) need(rel_res, "rel_res");
        const int n = (int)P->pcg_hist.size();
        for (int k = 0; k < std::min(n, (int)len); ++k) rel_res[k] = P->pcg_hist[k];
        if (count) *count = n;
    });
}

int32_t lddmm_num_kernels(void) { return K_NUM_KERNELS; }

const char *lddmm_kernel_name(int32_t kernel_id) { return kernel_name(kernel_id); }

const char *lddmm_status_string(lddmm_status s)
{
    switch (s) {
    case LDDMM_OK: return "ok";
    case LDDMM_EINVAL: return "invalid argument";
    case LDDMM_ENOMEM: return "out of device memory";
    case LDDMM_EDEVICE: return "HIP device error";
    case LDDMM_ESTATE: return "call out of order";
    case LDDMM_ENOTCONV: return "PCG did not converge (non-positive curvature or non-finite value)";
    case LDDMM_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *lddmm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Transport map without device allocation (lddmm_transport_forward_static).
// The departure displacements and the state ping-pong live in one
// file-scope device array, one copy per GPU for the life of the process; its
// device address is looked up once per device and kept.  The host-side
// array name is not a device address, so only the looked-up pointer is
// handed to kernels.
// ---------------------------------------------------------------------------
namespace lddmm {

constexpr long kStaticMaxPoints = 1L << 21;  // 128^3 grid points
constexpr long kStaticFloats = 7 * kStaticMaxPoints;  // dX, dXa (3N each), one state buffer (N)
static __device__ __align__(256) float scratch[kStaticFloats];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float *g_scratch_ptr[kMaxDevices] = {};

// the current device's copy of the array (looked up on first use, with that
// device current)
static float *static_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) fail(LDDMM_EDEVICE, "device index " + std::to_string(dev) + " out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) fail(LDDMM_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = (float *)ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace lddmm

extern "C" {

lddmm_status lddmm_transport_forward_static(const lddmm_config *cfg, void *stream, const float *m0, const float *v,
                                            float *m1_out, float *ckpt)
{
    return guard([&] {
        validate(cfg);
        need_dev(m0, "m0");
        need_dev(v, "v");
        need_dev(m1_out, "m1_out");
        need_dev(ckpt, "ckpt", true);
        if (m0 == m1_out) fail(LDDMM_EINVAL, "m0 and m1_out must be distinct arrays");
        const long N = (long)cfg->n[0] * cfg->n[1] * cfg->n[2];
        if (N > kStaticMaxPoints)
            fail(LDDMM_EINVAL, "lddmm_transport_forward_static: " + std::to_string(N) + " grid points exceed its " +
                                   std::to_string(kStaticMaxPoints) + "-point maximum (use lddmm_transport_forward)");
        // a plan record on the host only: no workspace, no tile-extents tables
        // (the gathers reduce their extents themselves), timing off
        lddmm_plan T;
        T.cfg = *cfg;
        T.stream = (hipStream_t)stream;
        check_hip(hipGetDevice(&T.device), "hipGetDevice");
        T.N = N;
        T.nt = cfg->nt;
        for (int d = 0; d < 3; ++d) T.h[d] = 2.0 * M_PI / cfg->n[d];
        T.h3 = T.h[0] * T.h[1] * T.h[2];
        T.dt = 1.0 / cfg->nt;
        float *s = static_scratch(T.device);
        float *dX = s, *dXa = s + 3 * N, *buf = s + 6 * N;
        launch_departure(&T, v, dX, dXa);
        if (ckpt) {
            copy_kernel(&T, N, m0, ckpt);
            for (int j = 0; j < T.nt; ++j)
                launch_interp(&T, 1, ckpt + (long)j * N, dX, ckpt + (long)(j + 1) * N, K_STATE_STEP);
            copy_kernel(&T, N, ckpt + (long)T.nt * N, m1_out);
        } else {
            // m_j alternates between buf and m1_out so that the last step writes m1_out
            const float *cur = m0;
            for (int j = 0; j < T.nt; ++j) {
                float *dst = ((T.nt - 1 - j) % 2 == 0) ? m1_out : buf;
                launch_interp(&T, 1, cur, dX, dst, K_STATE_STEP);
                cur = dst;
            }
        }
    });
}

}  // extern "C"
