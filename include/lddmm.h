/*
 * lddmm.h -- C ABI of the MI355X (gfx950) library for the Gauss-Newton-Krylov
 * hot path of LDDMM-type diffeomorphic image registration on a periodic 3D
 * grid (Brunn, Himthani, Biros, Mehl, Mang, arXiv 2008.12820).
 *
 * Problem (eq. "problem", Section 1.1): given a template m0 and a reference
 * m1 on Omega = [0,2pi)^3 (periodic), find a stationary velocity v that
 * minimises 1/2 ||m(.,1) - m1||^2 + beta/2 <A v, v>, where m is transported
 * by d_t m + v . grad m = 0, m(.,0) = m0.  The library evaluates the
 * objective, the reduced gradient (eq. "reducedgrad"), the Gauss-Newton
 * Hessian matvec (eq. "matvec" with eqs. "incsta", "incadj"), the spectral
 * preconditioner (beta A)^{-1} (Section 2, "Preconditioning"), a PCG Newton
 * step and a globalised Gauss-Newton iteration (eq. "iter", Algorithm "GNK"),
 * and the transport map with its vector-Jacobian product.
 *
 * Conventions shared by every call:
 *  - Grid n[0] x n[1] x n[2], x3 fastest: point p = (i*n1 + j)*n2 + k sits at
 *    (i h1, j h2, k h3), hd = 2pi/nd.  Every n[d] is even, >= 8, <= 1024, and
 *    has no prime factor other than 2, 3, 5.
 *  - Scalar fields are N = n0*n1*n2 float32 values; vector fields are 3N,
 *    component-major ([3][n0][n1][n2]).
 *  - Every float pointer is a DEVICE pointer owned by the caller, 16-byte
 *    aligned (EINVAL otherwise), contiguous.  Host pointers are used only for scalars and info
 *    structs.  The plan copies what it keeps; it never retains caller pointers.
 *  - All work is enqueued on the plan's HIP stream.  Calls that return host
 *    scalars (objective, gradient norm, newton step, GN iterate, timing)
 *    synchronise that stream before returning; the others are asynchronous.
 *  - Every call returns an lddmm_status and never aborts or prints;
 *    lddmm_last_error() gives a detail string for the calling thread.
 *  - A plan is not thread-safe; distinct plans on distinct streams are.
 *  - Units: J uses the h^3 = h1 h2 h3 quadrature; inner products and norms
 *    are h^3-weighted; the fields g and H v~ carry no h^3 factor.
 */
#ifndef LDDMM_H
#define LDDMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lddmm_status {
    LDDMM_OK = 0,
    LDDMM_EINVAL = 1,       /* bad size, beta, nt, pointer or argument */
    LDDMM_ENOMEM = 2,       /* device workspace allocation failed */
    LDDMM_EDEVICE = 3,      /* a HIP runtime error (detail in lddmm_last_error) */
    LDDMM_ESTATE = 4,       /* call out of order (e.g. gradient before set_velocity) */
    LDDMM_ENOTCONV = 5,     /* PCG met non-positive curvature or a non-finite value */
    LDDMM_EUNSUPPORTED = 6  /* valid request the library does not implement */
} lddmm_status;

/* Regularisation operator A (Section 1.1: H1 seminorm by default, A the
 * vector Laplacian; the H2 seminorm uses the squared Laplacian).
 * Spectral symbols |k|^2 and |k|^4. */
typedef enum lddmm_reg { LDDMM_REG_H1S = 1, LDDMM_REG_H2S = 2 } lddmm_reg;

/* lddmm_config.flags */
enum {
    /* Allocate only what the transport map, its VJP, the spectral operators
     * and lddmm_reg_energy need; the Newton-path calls then return
     * LDDMM_EUNSUPPORTED.  (Roughly half the workspace.) */
    LDDMM_FLAG_TRANSPORT_ONLY = 1,
    /* First derivatives (grad m_j, div v, and those of the transport VJP) by
     * the eighth-order central finite-difference stencil of Section 3.2,
     * coefficients 4/5, -1/5, 4/105, -1/280 over +-1..4 points, instead of
     * spectrally.  A, (beta A)^{-1} and the Leray projection stay spectral. */
    LDDMM_FLAG_FD8 = 2,
    /* First-order (trilinear) Lagrange interpolation, d = 1 in the formula
     * of Section 3.1, in every semi-Lagrangian step and the departure
     * predictor, instead of the cubic one (the paper's tuned runs use it). */
    LDDMM_FLAG_LINEAR_IP = 4
};

typedef struct lddmm_config {
    int32_t n[3];   /* grid size */
    int32_t nt;     /* time steps N_t >= 1 (dt = 1/N_t), Section 2 "Discretization" */
    int32_t reg;    /* lddmm_reg */
    int32_t leray;  /* 1: apply the Leray projection to the body force in g and H v~ */
    int32_t flags;  /* LDDMM_FLAG_* bits, 0 for the full plan */
    double beta;    /* regularisation weight, finite and > 0 */
} lddmm_config;

typedef struct lddmm_newton_info {
    int32_t pcg_iters;  /* Hessian matvecs spent in PCG */
    int32_t flags;      /* 1: non-positive curvature, 2: non-finite value met */
    double rel_res;     /* final ||r|| / ||r0|| of PCG */
    double alpha;       /* accepted line-search step (0 when none was accepted) */
    double J_before;    /* objective at the velocity the step started from */
    double J_after;     /* objective at the accepted velocity */
    double gnorm;       /* ||g|| at the start of the step */
    double gnorm_rel;   /* ||g|| / ||g0||, g0 the first gradient after set_images */
    int32_t inner_iters;  /* H0 applications inside the InvH0 preconditioner (0 for InvA) */
    int32_t reserved;
} lddmm_newton_info;

typedef struct lddmm_plan lddmm_plan;

/* Device bytes a plan for cfg allocates (host-only arithmetic, no device
 * call).  EINVAL for an invalid cfg or bytes == NULL. */
lddmm_status lddmm_workspace_bytes(const lddmm_config *cfg, size_t *bytes);

/* Create a plan on the current HIP device; stream is a hipStream_t (NULL =
 * the null stream).  Allocates all workspace (departure points, state and
 * gradient histories, FFT scratch and twiddles, reduction buffers) up front.
 * EINVAL for an invalid cfg, ENOMEM when the allocation fails. */
lddmm_status lddmm_plan_create(const lddmm_config *cfg, void *stream, lddmm_plan **plan);
lddmm_status lddmm_plan_destroy(lddmm_plan *plan);

/* Template m0 and reference m1 (N floats each, copied in).  Invalidates the
 * velocity state and the stored ||g0||. */
lddmm_status lddmm_set_images(lddmm_plan *plan, const float *m0, const float *m1);

/* Velocity v (3N, copied in).  Computes everything that depends on v only:
 * departure points of the state and adjoint characteristics (RK2, Section 2
 * "Discretization", FP64 arithmetic), the state m_j for j = 0..N_t (eq.
 * "problem" constraint, semi-Lagrangian), grad m_j, grad m_j at the state
 * departure points, div v and the adjoint reaction coefficient.
 * ESTATE before set_images. */
lddmm_status lddmm_set_velocity(lddmm_plan *plan, const float *v);

/* J = 1/2 ||m_{N_t} - m1||^2 + beta/2 <A v, v> (eq. "problem"), and its two
 * parts; any output pointer may be NULL.  ESTATE before set_velocity. */
lddmm_status lddmm_objective(lddmm_plan *plan, double *J, double *mismatch, double *reg);

/* Reduced gradient g = beta A v + K int_0^1 lam grad m dt (eq. "reducedgrad"),
 * lam from the adjoint equation (eq. "adj-transport") with final value
 * m1 - m(1); K = Leray projection if cfg.leray else I.  g: 3N device output.
 * gnorm (host, may be NULL) receives ||g||.  ESTATE before set_velocity. */
lddmm_status lddmm_gradient(lddmm_plan *plan, float *g, double *gnorm);

/* Gauss-Newton matvec H v~ = beta A v~ + K int_0^1 lam~ grad m dt
 * (eq. "matvec"), with m~ from eq. "incsta" (m~(0) = 0) and lam~ from
 * eq. "incadj" (lam~(1) = -m~(1)).  vt, hvt: 3N device arrays (distinct).
 * ESTATE before set_velocity. */
lddmm_status lddmm_hessian_matvec(lddmm_plan *plan, const float *vt, float *hvt);

/* s = (beta A)^{-1} r (Section 2, preconditioner "InvA"; the zero mode is
 * divided by beta).  r, s: 3N device arrays (may alias). */
lddmm_status lddmm_apply_inv_reg(lddmm_plan *plan, const float *r, float *s);

/* PCG solve of H v~ = -g at the current velocity (eq. "iter"), x0 = 0,
 * preconditioner (beta A)^{-1}, at most max_pcg matvecs, stop when
 * ||r|| <= rtol ||r0||; rtol <= 0 selects eps_K = min(sqrt(||g||/||g0||), 0.5)
 * (Algorithm "GNK").  vt_out: 3N device output.  ENOTCONV (with vt_out the
 * last iterate, or M^{-1} r0 at the first iteration) on non-positive
 * curvature or a non-finite value; info may be NULL. */
lddmm_status lddmm_newton_step(lddmm_plan *plan, int32_t max_pcg, double rtol, float *vt_out,
                               lddmm_newton_info *info);

/* Residual history of the last PCG of lddmm_newton_step / lddmm_gn_iterate
 * (Algorithm "GNK", the Krylov solve of eq. "iter"): rel_res[k] (host, len
 * entries at most) = ||r|| / ||r0|| after iteration k + 1 (the value before
 * it when that iteration stopped at the curvature test); *count (host, may
 * be NULL) = the iterations recorded (the first 4096 of a solve).  Copies
 * min(len, count) entries; EINVAL for len < 0 or rel_res NULL with len > 0. */
lddmm_status lddmm_pcg_history(lddmm_plan *plan, double *rel_res, int32_t len, int32_t *count);

/* One Gauss-Newton iteration (Algorithm "GNK"): gradient, PCG step as in
 * lddmm_newton_step, Armijo line search (alpha = 1, accept
 * J(v + a v~) <= J(v) + 1e-4 a <g, v~>, else halve, at most 10 tries), then
 * v <- v + a v~ and the plan's velocity state is refreshed.  v_inout: 3N
 * device array holding v on entry (must equal the plan's velocity) and the
 * updated velocity on return.  When no step is accepted v is unchanged and
 * info->alpha = 0. */
lddmm_status lddmm_gn_iterate(lddmm_plan *plan, int32_t max_pcg, double rtol, float *v_inout,
                              lddmm_newton_info *info);

/* Transport map (m0, v) -> m(1) (constraint of eq. "problem"): sets the
 * plan's characteristics from v, writes m(1) to m1_out (N) and, when ckpt is
 * not NULL, every m_j (j = 0..N_t) to ckpt ((N_t+1) N, the per-step
 * checkpoints).  Does not need set_images; replaces the plan's velocity. */
lddmm_status lddmm_transport_forward(lddmm_plan *plan, const float *m0, const float *v,
                                     float *m1_out, float *ckpt);

/* Vector-Jacobian product of the transport map for a loss with
 * dL/dm(1) = grad_m1: lam = adjoint sweep (eq. "adj-transport") with final
 * value grad_m1; grad_m0 = lam(0) (N); grad_v = -int_0^1 lam grad m dt (3N),
 * grad m from the checkpoints ckpt ((N_t+1) N from lddmm_transport_forward
 * with the same v).  Either output may be NULL. */
lddmm_status lddmm_transport_vjp(lddmm_plan *plan, const float *ckpt, const float *v,
                                 const float *grad_m1, float *grad_m0, float *grad_v);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the transport
 * map of lddmm_transport_forward without a plan.  cfg gives the grid, N_t
 * and the interpolation order (LDDMM_FLAG_LINEAR_IP; the other flags, reg,
 * leray and beta are validated but not used); stream is a hipStream_t
 * (NULL = the null stream) on the current device.  Writes m(1) to m1_out (N)
 * and, when ckpt is not NULL, every m_j to ckpt ((N_t+1) N); m0, v, m1_out,
 * ckpt are caller-owned device arrays, m0 and m1_out distinct.  Results are
 * bitwise those of lddmm_transport_forward.  Nothing is allocated: the
 * departure displacements and a state buffer (7N floats) live in a static
 * device array of 56 MiB that each GPU the library runs on holds until the
 * process ends, so at most 2^21 grid points (128^3): EINVAL beyond that.
 * Every call on a GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other streams or threads) race, so serialise them.  Asynchronous
 * on the stream; the array is written before it is read, nothing needs
 * clearing. */
lddmm_status lddmm_transport_forward_static(const lddmm_config *cfg, void *stream, const float *m0,
                                            const float *v, float *m1_out, float *ckpt);

/* Regularisation energy E = 1/2 sum_x (A v) . v (plain sum over the grid, no
 * h^3; beta not applied) and, when Av is not NULL, A v (3N) -- the beta/2
 * reg(v) term of eq. "problem" up to the factors beta h^3, and its gradient
 * for a caller that differentiates E (e.g. an autograd loss).  v: 3N. */
lddmm_status lddmm_reg_energy(lddmm_plan *plan, const float *v, float *Av, double *energy);

/* ---- step-level calls: each step of the path on its own ---------------- */

/* Unnormalised 3D real-to-complex DFT, hat f(k) = sum_x f(x) e^{-i k.x},
 * written in the standard half-spectrum layout [n0][n1][n2/2+1] of
 * interleaved (re, im) float pairs.  f: N, fhat: 2 n0 n1 (n2/2+1) floats. */
lddmm_status lddmm_fft_r2c(lddmm_plan *plan, const float *f, float *fhat);

/* Inverse of lddmm_fft_r2c including the 1/N factor (Hermitian input). */
lddmm_status lddmm_fft_c2r(lddmm_plan *plan, const float *fhat, float *f);

/* Spectral operators (Section 2: derivatives, A, its inverse and the Leray
 * projection are diagonal in the spectral domain).  First-order symbols use
 * i k with the Nyquist wavenumber set to 0; A uses the full |k|^2 or |k|^4.
 *   LDDMM_OP_GRAD   in N   -> out 3N   grad f
 *   LDDMM_OP_DIV    in 3N  -> out N    div v
 *   LDDMM_OP_REG    in 3N  -> out 3N   A v (per component)
 *   LDDMM_OP_INVREG in 3N  -> out 3N   (beta A)^{-1} v
 *   LDDMM_OP_LERAY  in 3N  -> out 3N   (I - k k^T/|k|^2) v                  */
enum { LDDMM_OP_GRAD = 1, LDDMM_OP_DIV = 2, LDDMM_OP_REG = 3, LDDMM_OP_INVREG = 4,
       LDDMM_OP_LERAY = 5 };
lddmm_status lddmm_spectral_op(lddmm_plan *plan, int32_t op, const float *in, float *out);

/* Cubic Lagrange interpolation (Section 3.1, d = 3): out[f][p] = I[field
 * f](x_p + h * disp[:, p]) for nfields fields, disp a 3N displacement in
 * voxels.  Nodes floor(u)-1 .. floor(u)+2, periodic. */
lddmm_status lddmm_interp(lddmm_plan *plan, int32_t nfields, const float *fields,
                          const float *disp, float *out);

/* Copy a plan-held array to out: LDDMM_FIELD_DISP (state departure
 * displacement (X - x)/h, 3N), LDDMM_FIELD_DISP_ADJ (adjoint, 3N),
 * LDDMM_FIELD_STATE (m_j, N), LDDMM_FIELD_GRAD_STATE (grad m_j, 3N),
 * LDDMM_FIELD_DIV (div v, N), LDDMM_FIELD_INC_STATE (m~(1) of the last
 * matvec, N), LDDMM_FIELD_ADJOINT (lam_j of the last gradient, N).
 * LDDMM_FIELD_PCG_R, _PCG_Z, _PCG_P (3N each): the residual r, the
 * preconditioned residual z = M^{-1} r and the search direction p that the
 * last PCG of lddmm_newton_step / lddmm_gn_iterate left (after k iterations
 * without a stop: r_k, z_k and p_k = z_k + beta_k p_{k-1}, the state from
 * which iteration k + 1 starts; Algorithm "GNK" solves eq. "iter" with it).
 * The PCG keeps r and p as spectra (see below): r and z are returned as
 * their FP32 inverse transforms (z = (beta A)^{-1} r for InvA, the last
 * inner solve's result for InvH0 and 2LInvH0), p as the physical field the
 * transport sweeps of the next matvec read; ESTATE for r and z before the
 * first PCG, p unspecified then.
 * LDDMM_FIELD_PCG_R_HAT, _PCG_P_HAT (3 n1 n2 (n3/2 + 1) complex values,
 * interleaved FP32, i.e. 6 n1 n2 (n3/2 + 1) floats): the spectra of r and p
 * themselves, in the standard half-spectrum layout [c][k1][k2][k3], k3 <= n3/2,
 * unnormalised (the forward DFT, sum_x f(x) e^{-i k.x}); ESTATE before the
 * first PCG.
 * After lddmm_transport_forward or lddmm_transport_vjp (e.g. on a
 * transport-only plan) the displacements are available, and after a VJP
 * also div v, the adjoint lam_j of that sweep (final value grad_m1) and, when
 * grad_v was asked for, grad m_j of the checkpoints.
 * ESTATE when the array has not been computed. */
enum { LDDMM_FIELD_DISP = 1, LDDMM_FIELD_DISP_ADJ = 2, LDDMM_FIELD_STATE = 3,
       LDDMM_FIELD_GRAD_STATE = 4, LDDMM_FIELD_DIV = 5, LDDMM_FIELD_INC_STATE = 6,
       LDDMM_FIELD_ADJOINT = 7, LDDMM_FIELD_PCG_R = 8, LDDMM_FIELD_PCG_Z = 9,
       LDDMM_FIELD_PCG_P = 10, LDDMM_FIELD_PCG_R_HAT = 11, LDDMM_FIELD_PCG_P_HAT = 12 };
lddmm_status lddmm_get_field(lddmm_plan *plan, int32_t what, int32_t j, float *out);

/* ---- batched form --------------------------------------------------------- */

/* B independent registrations advanced together (the data-parallel
 * multi-image processing the paper cites as related work).  Members with the
 * same configuration (grid size, N_t, regularisation, beta, flags) form a
 * group whose workspaces live in one batched plan: every kernel of an
 * iteration is launched once for all members of the group, the member index
 * a grid dimension, so a transport step, a transform pass, a reduction or a
 * PCG scalar update is one launch per group.  Per Gauss-Newton iteration a
 * group's gradient, eps_K, fixed-count PCG (device-resident scalars, stops
 * predicated per member), <g, v~> and first Armijo trial are one sequence;
 * groups run on up to nstreams library-created streams (default priority).
 * With use_graph != 0 the sequences of all groups are replayed from one
 * hipGraph captured for the whole batch (the group streams fork from the
 * first stream and join it inside the capture).  The batch calls
 * synchronise the device on entry and their streams on return.  Arrays of
 * device pointers are HOST arrays of B entries.
 * lddmm_batch_plan gives member b's plan for per-member calls
 * (lddmm_objective, lddmm_get_field, lddmm_set_beta, ...), which run on that
 * member alone; it belongs to the batch (lddmm_plan_destroy on it: EINVAL).
 * Members of one group must keep equal beta (lddmm_batch_gn_iterate returns
 * EUNSUPPORTED otherwise) and the InvA preconditioner. */
typedef struct lddmm_batch lddmm_batch;

lddmm_status lddmm_batch_create(int32_t B, const lddmm_config *cfgs, int32_t nstreams,
                                lddmm_batch **batch);
lddmm_status lddmm_batch_destroy(lddmm_batch *batch);
/* member b's plan (owned by the batch) for per-member calls such as
 * lddmm_objective or lddmm_get_field */
lddmm_status lddmm_batch_plan(lddmm_batch *batch, int32_t b, lddmm_plan **plan);
lddmm_status lddmm_batch_set_images(lddmm_batch *batch, const float *const *m0,
                                    const float *const *m1);
lddmm_status lddmm_batch_set_velocity(lddmm_batch *batch, const float *const *v);
/* One Gauss-Newton iteration per member, with the semantics of
 * lddmm_gn_iterate (rtol <= 0: eps_K rule; PCG stops are predicated so the
 * result equals the early-exit loop).  v_inout[b] receives member b's new
 * velocity; infos (host, B entries, may be NULL) the per-member reports. */
lddmm_status lddmm_batch_gn_iterate(lddmm_batch *batch, int32_t max_pcg, double rtol,
                                    int32_t use_graph, float *const *v_inout,
                                    lddmm_newton_info *infos);

/* ---- measurement -------------------------------------------------------- */

/* Autotuner: times every candidate tile shape (powers of two up to the LDS
 * budget) of each FFT kernel of the plan -- x3 rows per block, x1/x2 column
 * tiles per precision and sub-array, fused x1 operator tiles -- on the
 * plan's own buffers, keeps the fastest, and caches the choice per device
 * and grid size for the process and, when the environment variable
 * LDDMM_TUNE_CACHE names a file, in that file.  Synchronises the stream. */
lddmm_status lddmm_autotune(lddmm_plan *plan);
/* Change the regularisation weight beta (finite, > 0), e.g. for a
 * beta-continuation; the velocity state stays valid (it does not depend on
 * beta) and the stored ||g0|| is cleared, so the next gradient sets it.
 * EINVAL for a bad beta. */
lddmm_status lddmm_set_beta(lddmm_plan *plan, double beta);

/* Options of lddmm_gn_solve (Algorithm "GNK" with the beta-continuation of
 * Section 2 "Preconditioning", last paragraph). */
typedef struct lddmm_solve_opts {
    double beta_target;    /* final beta, > 0 */
    double eps_n;          /* a stage stops at ||g|| <= eps_n ||g0|| (the paper: 5e-2); 0 never */
    double rtol;           /* PCG tolerance; <= 0: eps_K = min(sqrt(||g||/||g0||), 0.5) */
    double eps_h0;         /* inner tolerance factor of InvH0 / 2LInvH0, in (0, 1) */
    double pc_switch;      /* InvA while beta > pc_switch (the paper: 0.5) */
    int32_t max_gn;        /* Gauss-Newton iterations per stage, >= 0 */
    int32_t max_pcg;       /* PCG iterations per Newton step, >= 0 */
    int32_t max_inner;     /* inner iterations per preconditioner application, >= 1 */
    int32_t continuation;  /* 1: beta = 1, 1e-1, ... while above beta_target, then beta_target */
    int32_t pc_kind;       /* preconditioner below pc_switch: 0 InvA, 1 InvH0, 2 2LInvH0 */
    int32_t reserved;
} lddmm_solve_opts;

typedef struct lddmm_solve_report {
    int32_t stages;       /* beta values solved for */
    int32_t gn_iters;     /* Newton steps taken over all stages */
    int32_t pcg_iters;    /* Hessian matvecs spent in PCG */
    int32_t inner_iters;  /* H0 applications inside the preconditioners */
    double J;             /* final objective (at beta_target) */
    double gnorm_rel;     /* final ||g|| / ||g0|| of the last stage */
} lddmm_solve_report;

/* Gauss-Newton-Krylov solve from the velocity in v_inout (3N, overwritten
 * with the result): per beta stage, Gauss-Newton iterations (lddmm_gn_iterate
 * semantics, the stage's first gradient as ||g0||) until ||g|| <= eps_n
 * ||g0||, max_gn steps or a failed line search, each stage starting from the
 * previous one's velocity; the plan's own preconditioner setting is restored
 * afterwards and its beta is left at beta_target.  ESTATE before
 * set_images; EINVAL for options out of range. */
lddmm_status lddmm_gn_solve(lddmm_plan *plan, const lddmm_solve_opts *opts, float *v_inout,
                            lddmm_solve_report *report);

/* Preconditioner of the PCG in lddmm_newton_step and lddmm_gn_iterate
 * (Section 2 "Preconditioning", Algorithm "PC"):
 *   kind 0 = InvA, (beta A)^{-1} (the default);
 *   kind 1 = InvH0, an inner PCG solve of eq. h0-pc,
 *     (beta0 A + grad m (x) grad m) s = r,  beta0 = max(beta, 5e-2),
 *   with m the deformed template m(1) at the current velocity,
 *   preconditioned by (beta0 A)^{-1}, started from (beta0 A)^{-1} r, stopped
 *   at ||r - H0 s|| <= eps_h0 * eps_K * ||r|| (eps_K the outer tolerance) or
 *   after max_inner iterations; four more 3N-float vectors on first use;
 *   kind 2 = 2LInvH0, the same solve on the grid of half the resolution
 *   (lddmm_apply_2linvh0 below); every n_d divisible by 4 and at least 16.
 * EINVAL for kind outside 0..2, eps_h0 not in (0, 1), max_inner < 1, or a
 * grid kind 2 cannot halve.  The batched iteration supports InvA only. */
lddmm_status lddmm_set_preconditioner(lddmm_plan *plan, int32_t kind, double eps_h0, int32_t max_inner);
/* out = H0 s (eq. h0-pc, the operator above); 3N floats each.  ESTATE before
 * a velocity is set. */
lddmm_status lddmm_apply_h0(lddmm_plan *plan, const float *s, float *out);
/* s ~= H0^{-1} r by the inner PCG above with relative tolerance tol (>= 0; 0
 * runs exactly max_inner iterations unless the residual vanishes) and at most
 * max_inner >= 0 iterations; *iters (may be NULL) receives the iterations. */
lddmm_status lddmm_apply_invh0(lddmm_plan *plan, const float *r, double tol, int32_t max_inner, float *s,
                               int32_t *iters);
/* s ~= 2LInvH0(r) (Algorithm "PC", second function): s_f = (beta0 A)^{-1} r;
 * the H0 system restricted to the half grid (Fourier coefficients of
 * |k_d| < n_d/4, the coarse Nyquist modes dropped; grad m(1) restricted the
 * same way) solved by the inner PCG from the restricted s_f with tolerance
 * tol and at most max_inner iterations; s = Prolong(s_c) + s_f -
 * Prolong(Restrict(s_f)).  The half-grid plan (about 1/8 of the workspace) is
 * created on first use.  EINVAL unless every n_d is divisible by 4 and at
 * least 16; *iters (may be NULL) receives the coarse iterations. */
lddmm_status lddmm_apply_2linvh0(lddmm_plan *plan, const float *r, double tol, int32_t max_inner, float *s,
                                 int32_t *iters);
/* Override the gather strategy of the interpolation kernels: 0 direct
 * (one thread per point, stencil loads through L1/L2), 1 and 2 LDS-staged
 * boxes for tiles of 2x4x64 and 4x4x64 points (points whose stencil leaves
 * the box load from global memory), 3 and 4 the same tiles walked by a
 * resident grid of workgroups that stage the next tile's box while they
 * interpolate the current one (one-field gathers at the plan's own
 * departure points; other gathers take 1 or 2), -1 the default heuristic.
 * The FP64 departure-point kernel follows the tile shape (0 direct, 1 and
 * 3 boxes of 2x4x64, 2 and 4 boxes of 4x4x64).  Every strategy computes
 * the same tensor-product sum in the same order, so results are bitwise
 * equal.  lddmm_autotune picks among 0..4 (and the departure strategy on
 * its own) by timing once the plan has a velocity.
 * EINVAL for a mode outside -1..4. */
lddmm_status lddmm_set_gather_mode(lddmm_plan *plan, int32_t mode);
/* Overlap (enable = 1, the default) or serialise (0) the forward transform
 * of the assembly's first operand -- the incremental velocity in a Hessian
 * matvec (eq. matvec), the velocity in a reduced gradient (eq.
 * reducedgrad) -- with the transport sweeps: it depends on the input alone,
 * so it runs on a side stream of the plan (created on first use, default
 * priority), forked from the plan's stream after the incremental-state start
 * (matvec) or at the start (gradient) and joined back before the assembly.
 * Results are bitwise the same either way; calls made under stream capture
 * always serialise.  Kernels of the two streams then share the device, so
 * per-kernel timings of the overlapped sweeps include that sharing. */
lddmm_status lddmm_set_overlap(lddmm_plan *plan, int32_t enable);
/* NUL-terminated report of the tile shapes in use (len bytes at most). */
lddmm_status lddmm_tuning(lddmm_plan *plan, char *buf, size_t len);

/* enable != 0: bracket every kernel launch of the plan with HIP events on
 * the plan's stream.  lddmm_get_timing synchronises, then reports the summed
 * event time (ms) and launch count of kernel class id since the last reset
 * (lddmm_set_timing resets).  Ids 0 .. lddmm_num_kernels()-1. */
lddmm_status lddmm_set_timing(lddmm_plan *plan, int32_t enable);
/* The same for the launches of one kernel class only (two events per launch
 * of that class, none elsewhere); lddmm_set_timing(plan, 0) turns it off. */
lddmm_status lddmm_set_timing_only(lddmm_plan *plan, int32_t kernel_id);
lddmm_status lddmm_get_timing(lddmm_plan *plan, int32_t kernel_id, double *total_ms,
                              int64_t *launches);
int32_t lddmm_num_kernels(void);
const char *lddmm_kernel_name(int32_t kernel_id);

const char *lddmm_status_string(lddmm_status s);
const char *lddmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LDDMM_H */
