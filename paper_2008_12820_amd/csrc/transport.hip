// Semi-Lagrangian transport kernels for gfx950 (Section 2 "Discretization":
// backward characteristics with RK2, interpolation at the off-grid departure
// points; Section 3.1: cubic Lagrange interpolation, d = 3).
//
// One thread per grid point, 64 consecutive x3 points per wavefront, so the
// 4x4x4 stencils of a wavefront overlap and their loads coalesce in L1/L2.
// Departure points are computed once per velocity in FP64 and stored as
// FP32 displacements in voxels, d = (X - x)/h, which keeps full FP32
// precision in the fractional offset (grid index + d is never formed in FP32).
#include "internal.hpp"

namespace lddmm {

constexpr int kPtThreads = 256;

struct Grid3 {
    int n1, n2, n3;
    int N;
};

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8), each with its own L2.  Renumber them so that each XCD sweeps
// one contiguous eighth of the grid: neighbouring rows and planes, whose
// 4x4x4 stencils overlap, then meet in the same L2.  A bijection on the
// first 8*floor(nb/8) workgroups; the remainder keeps its numbers.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int per = nb >> 3;
    if (b >= per * 8) return b;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int point_index()
{
    return xcd_block((int)blockIdx.x, (int)gridDim.x) * (int)blockDim.x + (int)threadIdx.x;
}

__device__ __forceinline__ void point_coords(const Grid3 &g, int p, int &i, int &j, int &k)
{
    k = p % g.n3;
    const int r = p / g.n3;
    j = r % g.n2;
    i = r / g.n2;
}

// Lagrange basis on the nodes -1, 0, 1, 2 at t in [0,1)
template <class T>
__device__ __forceinline__ void lagrange4(T t, T w[4])
{
    const T tm1 = t - T(1), tm2 = t - T(2), tp1 = t + T(1);
    w[0] = -t * tm1 * tm2 * T(1.0 / 6.0);
    w[1] = tp1 * tm1 * tm2 * T(0.5);
    w[2] = -tp1 * t * tm2 * T(0.5);
    w[3] = tp1 * t * tm1 * T(1.0 / 6.0);
}

// Stencil of one axis: node offsets (already multiplied by the axis stride)
// and weights for grid index i displaced by d voxels; periodic wrap.
// Returns the first node index (in [0, n)).
template <class T>
__device__ __forceinline__ int axis_stencil(int i, T d, int n, unsigned stride, unsigned o[4], T w[4])
{
    // clamp keeps the integer conversion defined for any input (NaN -> -lim);
    // the modulo below wraps every in-range displacement exactly
    const T lim = (T)1048576;
    d = d > lim ? lim : d;
    d = d >= -lim ? d : -lim;
    const T fl = floor(d);
    int b = i + (int)fl - 1;
    b %= n;
    if (b < 0) b += n;
    const int first = b;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        o[q] = (unsigned)b * stride;
        b = (b + 1 == n) ? 0 : b + 1;
    }
    lagrange4<T>(d - fl, w);
    return first;
}

template <class T>
struct Stencil {
    unsigned o1[4], o2[4], o3[4];  // element offsets of the nodes along x1, x2, x3
    bool contig;                   // x3 nodes consecutive in memory (no wrap)
    T w1[4], w2[4], w3[4];
};

template <class T>
__device__ __forceinline__ void make_stencil(const Grid3 &g, int i, int j, int k, T d1, T d2, T d3,
                                             Stencil<T> &s)
{
    axis_stencil<T>(i, d1, g.n1, (unsigned)g.n2 * (unsigned)g.n3, s.o1, s.w1);
    axis_stencil<T>(j, d2, g.n2, (unsigned)g.n3, s.o2, s.w2);
    const int b3 = axis_stencil<T>(k, d3, g.n3, 1u, s.o3, s.w3);
    s.contig = b3 + 3 < g.n3;
}

// Separable evaluation of the tensor-product sum.  When the four x3 nodes
// are contiguous (no periodic wrap) their loads come from one row pointer
// and merge into one 16-byte load; both branches add in the same order.
template <class T>
__device__ __forceinline__ T gather(const float *__restrict__ f, const Stencil<T> &s)
{
    T acc = T(0);
    if (s.contig) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            T acc2 = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float *row = f + (s.o1[a] + s.o2[b] + s.o3[0]);
                const T r = (T)row[0] * s.w3[0] + (T)row[1] * s.w3[1] + (T)row[2] * s.w3[2] +
                            (T)row[3] * s.w3[3];
                acc2 += s.w2[b] * r;
            }
            acc += s.w1[a] * acc2;
        }
    } else {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            T acc2 = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float *row = f + (s.o1[a] + s.o2[b]);
                const T r = (T)row[s.o3[0]] * s.w3[0] + (T)row[s.o3[1]] * s.w3[1] +
                            (T)row[s.o3[2]] * s.w3[2] + (T)row[s.o3[3]] * s.w3[3];
                acc2 += s.w2[b] * r;
            }
            acc += s.w1[a] * acc2;
        }
    }
    return acc;
}

__device__ __forceinline__ void load_stencil(const Grid3 &g, int p, const float *__restrict__ disp,
                                             Stencil<float> &s)
{
    int i, j, k;
    point_coords(g, p, i, j, k);
    make_stencil<float>(g, i, j, k, disp[p], disp[(long)g.N + p], disp[2L * g.N + p], s);
}

// ---------------------------------------------------------------------------
// departure points, FP64:  X = x - dt/2 (v(x) + I[v](x - dt v(x)))
//                          Xa = x + dt/2 (v(x) + I[v](x + dt v(x)))
// stored as displacements in voxels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPtThreads) void k_departure(const float *__restrict__ v,
                                                          float *__restrict__ dX,
                                                          float *__restrict__ dXa, Grid3 g, double dt,
                                                          double ih1, double ih2, double ih3)
{
    const int p = point_index();
    if (p >= g.N) return;
    int i, j, k;
    point_coords(g, p, i, j, k);
    const double ih[3] = {ih1, ih2, ih3};
    double vx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) vx[c] = (double)v[(long)c * g.N + p];
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const double sgn = dir == 0 ? -1.0 : 1.0;
        Stencil<double> s;
        make_stencil<double>(g, i, j, k, sgn * dt * vx[0] * ih[0], sgn * dt * vx[1] * ih[1],
                             sgn * dt * vx[2] * ih[2], s);
        float *out = dir == 0 ? dX : dXa;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double vi = gather<double>(v + (long)c * g.N, s);
            out[(long)c * g.N + p] = (float)(sgn * 0.5 * dt * (vx[c] + vi) * ih[c]);
        }
    }
}

// out[f][p] = I[in[f]](x_p + h disp_p) for nf fields (field stride N)
__global__ __launch_bounds__(kPtThreads) void k_interp(const float *__restrict__ in,
                                                       const float *__restrict__ disp,
                                                       float *__restrict__ out, Grid3 g, int nf)
{
    const int p = point_index();
    if (p >= g.N) return;
    Stencil<float> s;
    load_stencil(g, p, disp, s);
#pragma unroll 1
    for (int f = 0; f < nf; ++f) out[(long)f * g.N + p] = gather<float>(in + (long)f * g.N, s);
}

// adjoint reaction coefficient: one Heun step of d lam/ds = lam div v along
// the adjoint characteristic gives lam_j = c * I[lam_{j+1}](Xa) with
// c = 1 + dt/2 (delta_a + delta (1 + dt delta_a)), delta_a = I[delta](Xa)
__global__ __launch_bounds__(kPtThreads) void k_adj_coef(const float *__restrict__ delta,
                                                         const float *__restrict__ dXa,
                                                         float *__restrict__ coef, Grid3 g, float dt)
{
    const int p = point_index();
    if (p >= g.N) return;
    Stencil<float> s;
    load_stencil(g, p, dXa, s);
    const float da = gather<float>(delta, s);
    coef[p] = 1.f + 0.5f * dt * (da + delta[p] * (1.f + dt * da));
}

// lam_out = scale * c * I[lam_in](Xa)
__global__ __launch_bounds__(kPtThreads) void k_adj_step(const float *__restrict__ lin,
                                                         const float *__restrict__ dXa,
                                                         const float *__restrict__ coef,
                                                         float *__restrict__ lout, Grid3 g, float scale)
{
    const int p = point_index();
    if (p >= g.N) return;
    Stencil<float> s;
    load_stencil(g, p, dXa, s);
    lout[p] = scale * coef[p] * gather<float>(lin, s);
}

// Incremental state, first step and all sources (eq. incsta along X):
//   vX = I[v~](X),  s_j = vX . I[G_j](X) + v~ . G_{j+1}   (j = 0..nt-1)
//   m~_1 = -dt/2 s_0;  s_1..s_{nt-1} stored for the later steps
__global__ __launch_bounds__(kPtThreads) void k_incstate_init(const float *__restrict__ vt,
                                                              const float *__restrict__ dX,
                                                              const float *__restrict__ GX,
                                                              const float *__restrict__ G,
                                                              float *__restrict__ mt1,
                                                              float *__restrict__ src, Grid3 g,
                                                              int nt, float dt)
{
    const int p = point_index();
    if (p >= g.N) return;
    Stencil<float> s;
    load_stencil(g, p, dX, s);
    const long N = g.N;
    float vX[3], vp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        vX[c] = gather<float>(vt + c * N, s);
        vp[c] = vt[c * N + p];
    }
    for (int j = 0; j < nt; ++j) {
        const float *gx = GX + (long)j * 3 * N;
        const float *g1 = G + (long)(j + 1) * 3 * N;
        const float a = vX[0] * gx[p] + vX[1] * gx[N + p] + vX[2] * gx[2 * N + p];
        const float b = vp[0] * g1[p] + vp[1] * g1[N + p] + vp[2] * g1[2 * N + p];
        if (j == 0)
            mt1[p] = -0.5f * dt * (a + b);
        else
            src[(long)(j - 1) * N + p] = a + b;
    }
}

// m~_{j+1} = I[m~_j](X) - dt/2 s_j
__global__ __launch_bounds__(kPtThreads) void k_incstate_step(const float *__restrict__ min,
                                                              const float *__restrict__ dX,
                                                              const float *__restrict__ s_j,
                                                              float *__restrict__ mout, Grid3 g,
                                                              float dt)
{
    const int p = point_index();
    if (p >= g.N) return;
    Stencil<float> s;
    load_stencil(g, p, dX, s);
    mout[p] = gather<float>(min, s) - 0.5f * dt * s_j[p];
}

// b = dt * sum_j w_j lam_j G_j (trapezoid, w_0 = w_nt = 1/2); lam_nt is read
// from lamN times scaleN, lam_0..lam_{nt-1} from lam.
__global__ __launch_bounds__(kPtThreads) void k_body_force(const float *__restrict__ lam,
                                                           const float *__restrict__ lamN, float scaleN,
                                                           const float *__restrict__ G,
                                                           float *__restrict__ b, Grid3 g, int nt,
                                                           float dt)
{
    const int p = point_index();
    if (p >= g.N) return;
    const long N = g.N;
    float acc[3] = {0.f, 0.f, 0.f};
    for (int j = 0; j <= nt; ++j) {
        const float w = (j == 0 || j == nt) ? 0.5f : 1.f;
        const float l = (j == nt ? scaleN * lamN[p] : lam[(long)j * N + p]) * w;
        const float *gj = G + (long)j * 3 * N;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += l * gj[c * N + p];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) b[c * N + p] = dt * acc[c];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static Grid3 grid_of(const lddmm_plan *P)
{
    return Grid3{P->cfg.n[0], P->cfg.n[1], P->cfg.n[2], (int)P->N};
}

static dim3 blocks_of(const lddmm_plan *P)
{
    return dim3((unsigned)((P->N + kPtThreads - 1) / kPtThreads));
}

void launch_departure(lddmm_plan *P, const float *v, float *dX, float *dXa)
{
    Scope s(P, K_DEPARTURE);
    hipLaunchKernelGGL(k_departure, blocks_of(P), dim3(kPtThreads), 0, P->stream, v, dX, dXa,
                       grid_of(P), P->dt, 1.0 / P->h[0], 1.0 / P->h[1], 1.0 / P->h[2]);
    check_hip(hipGetLastError(), "k_departure");
}

void launch_interp(lddmm_plan *P, int nf, const float *fields, const float *disp, float *out, int kid)
{
    Scope s(P, kid);
    hipLaunchKernelGGL(k_interp, blocks_of(P), dim3(kPtThreads), 0, P->stream, fields, disp, out,
                       grid_of(P), nf);
    check_hip(hipGetLastError(), "k_interp");
}

void launch_adj_coef(lddmm_plan *P)
{
    Scope s(P, K_ADJ_COEF);
    hipLaunchKernelGGL(k_adj_coef, blocks_of(P), dim3(kPtThreads), 0, P->stream, P->delta, P->dXa,
                       P->coef, grid_of(P), (float)P->dt);
    check_hip(hipGetLastError(), "k_adj_coef");
}

void launch_adj_step(lddmm_plan *P, const float *lin, float *lout, float scale)
{
    Scope s(P, K_ADJ_STEP);
    hipLaunchKernelGGL(k_adj_step, blocks_of(P), dim3(kPtThreads), 0, P->stream, lin, P->dXa,
                       P->coef, lout, grid_of(P), scale);
    check_hip(hipGetLastError(), "k_adj_step");
}

void launch_incstate_init(lddmm_plan *P, const float *vt, float *mt1)
{
    Scope s(P, K_INCSTATE_INIT);
    hipLaunchKernelGGL(k_incstate_init, blocks_of(P), dim3(kPtThreads), 0, P->stream, vt, P->dX,
                       P->GX, P->G, mt1, P->src, grid_of(P), P->nt, (float)P->dt);
    check_hip(hipGetLastError(), "k_incstate_init");
}

void launch_incstate_step(lddmm_plan *P, const float *min, const float *sj, float *mout)
{
    Scope s(P, K_INCSTATE_STEP);
    hipLaunchKernelGGL(k_incstate_step, blocks_of(P), dim3(kPtThreads), 0, P->stream, min, P->dX,
                       sj, mout, grid_of(P), (float)P->dt);
    check_hip(hipGetLastError(), "k_incstate_step");
}

void launch_body_force(lddmm_plan *P, const float *lam, const float *lamN, float scaleN,
                       const float *G, float *b)
{
    Scope s(P, K_BODY_FORCE);
    hipLaunchKernelGGL(k_body_force, blocks_of(P), dim3(kPtThreads), 0, P->stream, lam, lamN,
                       scaleN, G, b, grid_of(P), P->nt, (float)P->dt);
    check_hip(hipGetLastError(), "k_body_force");
}

}  // namespace lddmm
