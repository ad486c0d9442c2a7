// Host-side plan and launcher declarations of the gfx950 LDDMM library.
#pragma once

#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"

namespace lddmm {

// Thrown inside the library, converted to an lddmm_status at the C boundary.
struct Error {
    lddmm_status status;
    std::string msg;
};

[[noreturn]] void fail(lddmm_status s, const std::string &msg);
void set_last_error(const std::string &msg);
void check_hip(hipError_t e, const char *what);

// Spectral layout of one real field of n1 x n2 x n3 (internal, never exposed):
//   main: [n1][n2][n3/2] complex (k3 = 0 .. n3/2-1), then
//   nyq : [n1][n2]       complex (k3 = n3/2),
// i.e. n1*n2*(n3/2+1) float2 per field.  After the x3 pass the first two
// indices are physical (x1, x2); after the x2 pass (x1, k2); after the x1
// pass (k1, k2).
struct FftCtx {
    int n1 = 0, n2 = 0, n3 = 0, m3 = 0;
    long nrow = 0;         // n1*n2
    long spec_stride = 0;  // float2 per spectral field
    RadixPlan rp1{}, rp2{}, rp3{};
    float2 *tw1 = nullptr, *tw2 = nullptr, *tw3 = nullptr, *twN3 = nullptr;      // device tables
    double2 *tw1d = nullptr, *tw2d = nullptr, *tw3d = nullptr, *twN3d = nullptr;  // FP64 tables
    // tile shapes (set from LDS-budget heuristics, refined by the autotuner)
    int tw_cols[2][2][2] = {};  // [axis: 0 = x1, 1 = x2][part: main, Nyquist][FP64]
    int tw_x1[8][2] = {};       // [spectral op][part]
    int twr_r2c[2] = {};        // rows per block of the x3 R2C pass [FP64]
    int twr_c2r = 0;            // rows per block of the x3 C2R pass
    int tuned = 0;              // 1 once the autotuner has run
};

// LDS bytes of one FFT workgroup: the default tiles stay within kLdsBudget
// (several workgroups per CU); the autotuner may go up to kLdsMax (the
// 160 KB a gfx950 workgroup can address)
constexpr size_t kLdsBudget = 64 * 1024;
constexpr size_t kLdsMax = 160 * 1024;

struct PlanTiming {
    bool on = false;
    int only = -1;  // >= 0: bracket only launches of this kernel class
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    std::vector<int> kid;  // kernel class of each used pair
    size_t used = 0;
};

}  // namespace lddmm

struct lddmm_plan {
    lddmm_config cfg{};
    hipStream_t stream = nullptr;
    // side stream and fork/join events: the forward transform of an input that
    // only the final assembly needs runs beside the transport sweeps
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int overlap = 1;  // lddmm_set_overlap (on by default)
    // preconditioner (lddmm_set_preconditioner): 0 InvA, 1 InvH0
    int pc_kind = 0, pc_max_inner = 50;
    double pc_eps_h0 = 1e-3;
    float *h0buf = nullptr;   // InvH0 inner PCG vectors r, z, p, q (4 x 3N), on first use
    lddmm_plan *coarse = nullptr;  // 2LInvH0: the plan of the half grid, on first use
    unsigned long vel_gen = 0;     // velocity states computed (grad m(1) generations)
    unsigned long coarse_gen = 0;  // vel_gen whose restricted grad m(1) the coarse plan holds
    double beta_sym = 0.0;    // > 0: beta of the (beta A)^{-1} symbol instead of cfg.beta
    int device = 0;
    // members of a batched plan (see Mb); the arena holds mb.count copies of
    // the workspace, mb.stride bytes apart
    lddmm::Mb mb;
    const lddmm_plan *view_of = nullptr;  // a batch member's plan: the batched plan it views
    long N = 0;
    int nt = 0;
    double h[3] = {0, 0, 0};
    double h3 = 0, dt = 0;
    lddmm::FftCtx fft;

    void *arena = nullptr;
    size_t arena_bytes = 0;

    float *m0 = nullptr, *m1 = nullptr, *v = nullptr, *dX = nullptr, *dXa = nullptr;
    float *m = nullptr;      // (nt+1) N, m[0] = m0
    float *G = nullptr;      // (nt+1) 3N
    float *GX = nullptr;     // nt 3N, G_j at the state departure points
    float *delta = nullptr, *coef = nullptr;
    float *lam = nullptr;    // (nt+1) N adjoint history
    float *mt = nullptr;     // 2N incremental-state ping-pong
    float *src = nullptr;    // max(nt-1,1) N incremental-state sources
    float *b = nullptr, *tmp3 = nullptr, *g = nullptr;
    float *px = nullptr, *pr = nullptr, *pz = nullptr, *pp = nullptr, *pq = nullptr, *vt = nullptr;
    char *spec = nullptr;    // spectral scratch: nspec slots of slot_bytes (FP64-sized)
    long slot_bytes = 0;
    int nspec = 0;
    int pcg_spectral = 0;    // 1: a PCG has run (its r and p spectra are in pr and pz)
    double *red = nullptr;   // reduction partials (two sets of kRedBlocks, or per x1 tile and field)
    long red_len = 0;        // doubles at red
    double *hist = nullptr;  // ||r_k|| / ||r0|| per PCG iteration (device, kHistMax)
    std::vector<double> pcg_hist;  // the last PCG's history (host)
    double *dscal = nullptr; // device scalars, two banks of kNumScalars (see ScalarSlot)
    int bank = 0;            // the bank the scalar kernels and reductions use
    double *hscal = nullptr; // pinned host mirror (kNumScalars, then the 2-slot poll rings of the PCG and the inner PCG)
    hipEvent_t ev_poll[2] = {nullptr, nullptr};   // the device-resident PCG's lagged stop test
    hipEvent_t ev_inner[2] = {nullptr, nullptr};  // the same for the InvH0 inner PCG

    int have_images = 0, have_velocity = 0, have_grad = 0, have_matvec = 0;
    // transport map calls: departure points (forward or VJP), and the adjoint
    // sweep and checkpoint gradients of the last VJP
    int have_disp = 0, have_vjp = 0;
    void *boxes[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // stencil extents per tile: [dX, dXa][2x4, 4x4]
    int boxes_valid = 0;
    int gather_mode = -1;    // 0 direct, 1/2 box tiles 2x4x64/4x4x64, 3/4 the same pipelined, -1 heuristic
    int gather_mode3 = -1;   // the same for three-field gathers; -1: follow gather_mode
    int departure_mode = -1; // 0 direct, 1/2 box tiles 2x4x64/4x4x64, -1 the gather strategy's tiles
    int gather_tuned = 0;
    int pipe_grid[2] = {0, 0};  // workgroups of the pipelined gathers [2x4, 4x4] (0: not yet sized)
    float gather_ms[1] = {0.f};
    double g0norm = 0.0;
    // bumped by every setter that changes the arguments or the choice of the
    // kernels a call enqueues (beta, tile shapes, gather strategy, ...), so
    // that a captured graph of an older generation is not replayed
    unsigned long enqueue_gen = 0;
    lddmm::PlanTiming timing;
};

namespace lddmm {

// ---- launch bracketing (per-kernel HIP events when timing is on) ----------
struct Scope {
    lddmm_plan *P;
    int kid;
    int slot = -1;
    Scope(lddmm_plan *p, int k);
    ~Scope() noexcept(false);
};

// ---- fft.hip ----------------------------------------------------------------
struct RealIn {
    const float *p[8];
};
struct RealOut {
    float *p[8];
};

void fft_init(lddmm_plan *P);
void fft_free(lddmm_plan *P);
// real fields -> spectral slots [slot0, slot0+count), FP64 or FP32 arithmetic and storage
void r2c_fields(lddmm_plan *P, const RealIn &in, int count, int slot0, bool dbl);
// x2 pass over spectral slots (forward or inverse)
void x2_pass(lddmm_plan *P, int slot0, int count, bool inverse, bool dbl);
// x1 pass without a symbol (forward or inverse)
void x1_pass(lddmm_plan *P, int slot0, int count, bool inverse, bool dbl);
// FP32 spectral slots -> real fields, times scale
void c2r_fields(lddmm_plan *P, int slot0, int count, const RealOut &out, float scale);
// three spectra in slots in0.. (after the inverse x1 and x2 passes) -> along
// x3 back, t = G (G . p) per point, forward along x3 -> slots out0.. (the
// rank-one part of H0 without a trip through HBM); false (nothing done) for
// an x3 length without a register row plan
bool x3_rank1(lddmm_plan *P, int in0, int out0, const float *G);

enum SpecOp { SOP_GRAD = 1, SOP_DIV, SOP_REG, SOP_INVREG, SOP_LERAY, SOP_ASSEMBLE, SOP_IDENT };
// x1 forward, pointwise symbol, x1 inverse in one pass: batches of the op's
// input fields at spec_in + b*nin, outputs at spec_out + b*nout.
void x1_symbol(lddmm_plan *P, int op, int spec_in, int spec_out, int nbatch, int leray);
// whole operator on real fields (in: nbatch*nin fields, out: nbatch*nout);
// fwd_done > 0 (one field set only): the forward passes of the first fwd_done
// inputs were already run by spectral_forward
void spectral_apply(lddmm_plan *P, int op, const std::vector<const float *> &in,
                    const std::vector<float *> &out, int fwd_done = 0);
// FP32 spectra of slots [s0, s0+count) of plan S resampled into slots
// [d0, ..) of plan D, a grid of half or twice the size (restriction /
// prolongation by truncation / zero padding of the Fourier coefficients)
void spectral_resample(lddmm_plan *S, int s0, lddmm_plan *D, int d0, int count);
// forward x3 and x2 passes of the first count inputs of one field set, into
// the slots spectral_apply uses for them
void spectral_forward(lddmm_plan *P, int op, const std::vector<const float *> &in, int count);
int op_nin(int op);
int op_nout(int op);
// time the candidate tile shapes of every FFT kernel of the plan and keep
// the fastest (results cached per device and shape for the process and, if
// the environment names one, in a text file)
void autotune_fft(lddmm_plan *P);
std::string tuning_report(const lddmm_plan *P);
// standard half-spectrum [n1][n2][n3/2+1] <-> internal layout
void pack_standard(lddmm_plan *P, int spec_field, float2 *dst);
void unpack_standard(lddmm_plan *P, const float2 *srcp, int spec_field);
// spectral-domain PCG with M^{-1} = (beta A)^{-1}: FP32 spectra (internal
// layout, unnormalised) of three fields, 3 * spec_stride float2 per vector.
// three real fields (stride N) -> their spectra in slots [slot0, slot0 + 3)
void spec_forward3(lddmm_plan *P, const float *in, int slot0);
// spectra in slots [slot0, slot0 + 3) (overwritten) -> three real fields;
// x1_done: the inverse x1 pass has already run on them
void spec_inverse3(lddmm_plan *P, int slot0, float *out, bool x1_done = false);
// q = K b + beta A p (b: the spectra in slots bslot..; K the Leray projection
// when leray); <p, q> into scalar kslot unless it is negative, then the
// scalar steps `after` (kAfter* bits)
void spcg_assemble(lddmm_plan *P, int bslot, const float2 *p, float2 *q, int kslot, int leray, int after);
// r = sign b (b: three spectra bstride float2 apart) unless r is NULL;
// p = M^{-1} r unless NULL, copied into slots cslot.. unless cslot < 0;
// <r, r> and <r, M^{-1} r> into scalars rr_slot, rz_slot (rz skipped when < 0)
void spcg_start(lddmm_plan *P, const float2 *b, long bstride, float sign, float2 *r, float2 *p, int cslot, int rr_slot,
                int rz_slot);
// r -= alpha q and, unless x is NULL, x += alpha p (device alpha); <r, r>
// and <r, M^{-1} r> into rr_slot, rz_slot (rz skipped when < 0), then the
// scalar steps `after` (S_REL into hist_dst for kAfterHist)
void spcg_r(lddmm_plan *P, float2 *r, const float2 *q, float2 *x, const float2 *p, int rr_slot, int rz_slot,
            int after, double *hist_dst);
// p = z + beta p (device beta, kept after a stop) with z = M^{-1} r when z is
// NULL; copied into slots cslot.. unless cslot < 0; unless sx is NULL, first
// sx += alpha p (device alpha, the p before its update)
void spcg_p(lddmm_plan *P, const float2 *r, const float2 *z, float2 *p, int cslot, float2 *sx = nullptr);
// the forward x1 pass of the spectra in slots slot0.. (t^ after the x3 and
// x2 passes) fused with the H0 assembly q = t^ + beta0 A p into the vector q,
// <p, q> into S_KAPPA and alpha; false (nothing done) without a register plan
bool x1_fwd_h0_assemble(lddmm_plan *P, int slot0, const float2 *p, float2 *q);
// the same update fused into the inverse x1 pass of p into slots slot0..
// (where the x1 length has a register plan; else the update, its copy and
// the pass apart): the slots then hold p after its inverse x1 pass
void spcg_p_x1(lddmm_plan *P, const float2 *r, const float2 *z, float2 *p, int slot0, float2 *sx = nullptr);
// <a, b> of three spectra each into scalar slot, then the steps `after`
void spec_dot(lddmm_plan *P, const float2 *a, const float2 *b, int slot, int after = 0);
// dst = M^{-1} src, three spectra each
void spec_invreg3(lddmm_plan *P, const float2 *src, float2 *dst);
// slots src_slot.. -> three contiguous spectra
void spec_from_slots(lddmm_plan *P, int src_slot, float2 *dst);
// two-level preconditioner on spectra (plans F and C of a grid and its half):
// rc = R r and sc0 = (beta0 A_c)^{-1} R r (C's symbol), from fine spectra r
void two_level_restrict(lddmm_plan *F, const float2 *r, lddmm_plan *C, float2 *rc, float2 *sc0);
// z = (beta0 A)^{-1} r + P (scs - sc0) (F's symbol); <r, z> into F's scalar
// rz_slot (unless negative), then the steps `after`
void two_level_prolong(lddmm_plan *F, const float2 *r, float2 *z, lddmm_plan *C, const float2 *scs,
                       const float2 *sc0, int rz_slot, int after);
// the FP32 view of transform slot slot
float2 *spec_slot(lddmm_plan *P, int slot);
// three spectra (3 * spec_stride float2 at src) into slots dst_slot..,
// times M^{-1} when inv
void spec_copy3(lddmm_plan *P, const float2 *src, int dst_slot, bool inv);

// ---- transport.hip ----------------------------------------------------------
void launch_departure(lddmm_plan *P, const float *v, float *dX, float *dXa);
size_t tile_boxes_bytes(const int n[3]);                // per displacement field
void assign_tile_boxes(lddmm_plan *P, char *base);      // 2 * tile_boxes_bytes at base
void launch_tile_boxes(lddmm_plan *P);
void autotune_gather(lddmm_plan *P);
void launch_interp(lddmm_plan *P, int nf, const float *fields, const float *disp, float *out,
                   int kid);
void launch_adj_coef(lddmm_plan *P);
void launch_adj_step(lddmm_plan *P, const float *lin, float *lout, float scale);
void launch_incstate_init(lddmm_plan *P, const float *vt, float *mt1);
void launch_incstate_step(lddmm_plan *P, const float *min, const float *s, float *mout);
// last adjoint step into lam0 fused with the body force into P->b
void h0_point(lddmm_plan *P, const float *s, const float *G, float *out, float beta0);
// out = G (G . s), the rank-one part of H0 (three fields each, stride N)
void h0_rank1(lddmm_plan *P, const float *s, const float *G, float *out);
// eighth-order central differences (Section 3.2): grad f into g1, g2, g3;
// div of v (three fields, stride N) into out
void launch_fd8_grad(lddmm_plan *P, const float *f, float *g1, float *g2, float *g3);
void launch_fd8_div(lddmm_plan *P, const float *v, float *out);
void launch_adj_body(lddmm_plan *P, const float *lin, float scale, float *lam0, const float *lam,
                     const float *lamN, float scaleN);
void launch_body_force(lddmm_plan *P, const float *lam, const float *lamN, float scaleN,
                       const float *G, float *b);

// ---- api.hip (sequencing shared with the batched form) ---------------------
void velocity_state(lddmm_plan *P);
void gradient_enqueue(lddmm_plan *P, float *g);
void matvec_impl(lddmm_plan *P, const float *vt, float *hvt);
void inv_reg(lddmm_plan *P, const float *r, float *s);
void objective_enqueue(lddmm_plan *P, int sj, int smis, int sreg);
void pcg_enqueue(lddmm_plan *P, const float *g, int max_it, float *x);
void gn_trial_enqueue(lddmm_plan *P, int max_pcg, double rtol, float *v0);

// ---- linalg.hip -------------------------------------------------------------
// FP64 h^3-weighted reductions; result left in P->dscal[slot] (device).
void dot_async(lddmm_plan *P, const float *a, const float *b, long n, int slot, double scale);
void sqdiff_async(lddmm_plan *P, const float *a, const float *b, long n, int slot,
                  double scale);
double fetch_scalar(lddmm_plan *P, int slot);
// out = a*x + b*y (y may be null)
void axpby(lddmm_plan *P, long n, float a, const float *x, float b, const float *y, float *out);
// out[i] = value
void fill(lddmm_plan *P, long n, float value, float *out);
constexpr int kRedBlocks = 1024;
constexpr int kNumScalars = 32;
// pinned host doubles per member: the scalars, then the 2-slot poll rings of
// the PCG and of the inner PCG
constexpr int kHostScalars = kNumScalars + 4;
constexpr int kHistMax = 4096;  // PCG iterations whose residual is recorded

// Device scalar slots (P->dscal).  0..4 serve the eager calls; the rest hold
// the state of the device-resident PCG / Gauss-Newton step, which needs no
// host round trip and can be captured in a graph.
enum ScalarSlot {
    S_GG = 0, S_DOT = 1, S_MIS = 2, S_REG = 3, S_E = 4,
    S_RR = 5, S_RZ = 6, S_KAPPA = 7, S_RZN = 8, S_R0 = 9, S_ALPHA = 10, S_BETA = 11,
    S_DONE = 12, S_ITERS = 13, S_FLAGS = 14, S_RTOL = 15, S_REL = 16, S_GNORM = 17,
    S_G0 = 18, S_GV = 19, S_J0 = 20, S_J1 = 21, S_COPYZ = 22, S_MIS1 = 23, S_REG1 = 24,
    S_INNER = 25  // inner iterations of the InvH0 / 2LInvH0 preconditioner summed over a PCG
};
// Two banks of kNumScalars slots: bank 0 holds the outer PCG / Gauss-Newton
// state, bank 1 the inner PCG of the H0 preconditioner.  The scalar kernels
// and reductions work on the plan's current bank.
inline double *scalars(lddmm_plan *P) { return P->dscal + P->bank * kNumScalars; }

// device-resident PCG pieces (single-thread scalar kernels and predicated
// vector updates; see linalg.hip)
void dev_set_scalar(lddmm_plan *P, int slot, double value);
void dev_tolerance(lddmm_plan *P, double rtol);
void dev_pcg_init(lddmm_plan *P);
// x += alpha p with the device alpha (nothing when it is 0), or x = p after
// a curvature stop at the first iteration
void dev_pcg_x(lddmm_plan *P, long n, const float *p, float *x);
// scalars(P)[slot] = scale * (sum of kRedBlocks partials)
void dev_reduce_final(lddmm_plan *P, const double *partial, int slot, double scale);
// the scalar steps of the PCG that may follow a reduction in the same launch
enum { kAfterAlpha = 1, kAfterConv = 2, kAfterHist = 4, kAfterBeta = 8 };
// slots a and b (b < 0: none) = scale * (sums of the kRedBlocks partials at
// partial and partial + kRedBlocks), then the steps named in after (alpha,
// conv, S_REL into hist_dst, beta, in that order)
void dev_reduce_final_steps(lddmm_plan *P, const double *partial, int a, int b, double scale, int after,
                            double *hist_dst, int np = kRedBlocks);
// doubles of the reduction partials (P->red)
inline long red_capacity(const lddmm_plan *P) { return P->red_len; }
void dev_pcg_conv(lddmm_plan *P);
void dev_sum(lddmm_plan *P, int dst, int a, int b);
// the inner PCG (current bank) counts as stopped when the outer one (bank-0
// scalars outer) has stopped; and adds its iterations to outer[S_INNER]
void dev_inner_link(lddmm_plan *P, double *outer);
void dev_inner_accum(lddmm_plan *P, double *outer);
void copy_kernel(lddmm_plan *P, long n, const float *x, float *out);

// ---- batched plans (api.hip) ----------------------------------------------
lddmm_plan *create_plan(const lddmm_config *cfg, void *stream, int members);
lddmm_plan *member_view(const lddmm_plan *G, int b);
void view_free(lddmm_plan *V);

}  // namespace lddmm
