// Vector algebra of the PCG / Gauss-Newton loop for gfx950: FP64-accumulating
// deterministic reductions (fixed grid, fixed tree) and FP32 vector updates.
#include "internal.hpp"

namespace lddmm {

constexpr int kRedThreads = 256;

// mode 0: sum a*b;  mode 1: sum (a-b)^2
template <int MODE>
__device__ __forceinline__ double red_term(float x, float y)
{
    if (MODE == 0) return (double)x * (double)y;
    const double d = (double)x - (double)y;
    return d * d;
}

// Partial sums per workgroup over a fixed grid, in a fixed order: the result
// is bitwise reproducible.  vec: 16-byte accesses over the first n/4 groups of
// four, the n % 4 tail by the first threads of workgroup 0.
template <int MODE>
__global__ __launch_bounds__(kRedThreads) void k_reduce_partial(const float *__restrict__ a,
                                                                const float *__restrict__ b, long n,
                                                                int vec, double *__restrict__ partial, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); a = mshift(a, mo_); b = mshift(b, mo_); partial = mshift(partial, mo_);
    if (mb.stopped(mo_)) return;
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    const long stride = (long)gridDim.x * blockDim.x;
    const long i0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (vec) {
        const long n4 = n >> 2;
        const float4 *a4 = (const float4 *)a, *b4 = (const float4 *)b;
        for (long i = i0; i < n4; i += stride) {
            const float4 x = a4[i], y = b4[i];
            acc += (red_term<MODE>(x.x, y.x) + red_term<MODE>(x.y, y.y)) +
                   (red_term<MODE>(x.z, y.z) + red_term<MODE>(x.w, y.w));
        }
        if (blockIdx.x == 0 && (long)threadIdx.x < (n & 3)) {
            const long t = (n4 << 2) + threadIdx.x;
            acc += red_term<MODE>(a[t], b[t]);
        }
    } else {
        for (long i = i0; i < n; i += stride) acc += red_term<MODE>(a[i], b[i]);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double *__restrict__ partial,
                                                              int np, double *__restrict__ out,
                                                              double scale, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); partial = mshift(partial, mo_); out = mshift(out, mo_);
    if (mb.stopped(mo_)) return;
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = scale * sh[0];
}

// Elementwise updates: with vec set (every pointer 16-byte aligned) thread t
// handles the groups of four t, t + stride, ... with 16-byte accesses and the
// n % 4 tail elements go to the first threads; otherwise one element each.
template <class F4, class F1>
__device__ __forceinline__ void ew_loop(long n, int vec, F4 body4, F1 body1)
{
    const long stride = (long)gridDim.x * blockDim.x;
    const long i0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (vec) {
        const long n4 = n >> 2;
        for (long i = i0; i < n4; i += stride) body4(i);
        if (i0 < (n & 3)) body1((n4 << 2) + i0);
    } else {
        for (long i = i0; i < n; i += stride) body1(i);
    }
}

// The updates round as written with explicit fused multiply-adds, the same in
// the 16-byte and the one-element paths (a x + b y, x + alpha p: one rounding).
__device__ __forceinline__ float axpby1(float a, float x, float b, float y) { return __builtin_fmaf(b, y, a * x); }

__device__ __forceinline__ float4 f4axpby(float a, float4 x, float b, float4 y)
{
    return make_float4(axpby1(a, x.x, b, y.x), axpby1(a, x.y, b, y.y), axpby1(a, x.z, b, y.z),
                       axpby1(a, x.w, b, y.w));
}

__global__ void k_axpby(long n, int vec, float a, const float *__restrict__ x, float b,
                        const float *__restrict__ y, float *__restrict__ out, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); x = mshift(x, mo_); y = mshift(y, mo_); out = mshift(out, mo_);
    if (mb.stopped(mo_)) return;
    if (y) {
        ew_loop(
            n, vec,
            [&](long i) { ((float4 *)out)[i] = f4axpby(a, ((const float4 *)x)[i], b, ((const float4 *)y)[i]); },
            [&](long i) { out[i] = axpby1(a, x[i], b, y[i]); });
    } else {
        ew_loop(
            n, vec,
            [&](long i) {
                const float4 v = ((const float4 *)x)[i];
                ((float4 *)out)[i] = make_float4(a * v.x, a * v.y, a * v.z, a * v.w);
            },
            [&](long i) { out[i] = a * x[i]; });
    }
}

__global__ void k_fill(long n, int vec, float value, float *__restrict__ out, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); out = mshift(out, mo_);
    ew_loop(
        n, vec, [&](long i) { ((float4 *)out)[i] = make_float4(value, value, value, value); },
        [&](long i) { out[i] = value; });
}

// H0 s = beta0 A s + G (G . s) (eq. h0-pc): on entry out holds A s; three
// fields each, stride n
__global__ void k_h0_point(long n, int vec, float beta0, const float *__restrict__ s,
                           const float *__restrict__ G, float *__restrict__ out, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); s = mshift(s, mo_); G = mshift(G, mo_); out = mshift(out, mo_);
    if (mb.stopped(mo_)) return;
    ew_loop(
        n, vec,
        [&](long i) {
            const float4 s0 = ((const float4 *)s)[i], s1 = ((const float4 *)(s + n))[i],
                         s2 = ((const float4 *)(s + 2 * n))[i];
            const float4 g0 = ((const float4 *)G)[i], g1 = ((const float4 *)(G + n))[i],
                         g2 = ((const float4 *)(G + 2 * n))[i];
            float4 *o0 = (float4 *)out + i, *o1 = (float4 *)(out + n) + i, *o2 = (float4 *)(out + 2 * n) + i;
            const float4 d = make_float4(g0.x * s0.x + g1.x * s1.x + g2.x * s2.x, g0.y * s0.y + g1.y * s1.y + g2.y * s2.y,
                                         g0.z * s0.z + g1.z * s1.z + g2.z * s2.z, g0.w * s0.w + g1.w * s1.w + g2.w * s2.w);
            const float4 a0 = *o0, a1 = *o1, a2 = *o2;
            *o0 = make_float4(beta0 * a0.x + g0.x * d.x, beta0 * a0.y + g0.y * d.y, beta0 * a0.z + g0.z * d.z,
                              beta0 * a0.w + g0.w * d.w);
            *o1 = make_float4(beta0 * a1.x + g1.x * d.x, beta0 * a1.y + g1.y * d.y, beta0 * a1.z + g1.z * d.z,
                              beta0 * a1.w + g1.w * d.w);
            *o2 = make_float4(beta0 * a2.x + g2.x * d.x, beta0 * a2.y + g2.y * d.y, beta0 * a2.z + g2.z * d.z,
                              beta0 * a2.w + g2.w * d.w);
        },
        [&](long i) {
            const float d = G[i] * s[i] + G[n + i] * s[n + i] + G[2 * n + i] * s[2 * n + i];
            out[i] = beta0 * out[i] + G[i] * d;
            out[n + i] = beta0 * out[n + i] + G[n + i] * d;
            out[2 * n + i] = beta0 * out[2 * n + i] + G[2 * n + i] * d;
        });
}

// out = G (G . s): the rank-one part of H0 (eq. h0-pc); three fields each,
// stride n
__global__ void k_h0_rank1(long n, int vec, const float *__restrict__ s, const float *__restrict__ G,
                           float *__restrict__ out, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); s = mshift(s, mo_); G = mshift(G, mo_); out = mshift(out, mo_);
    if (mb.stopped(mo_)) return;
    ew_loop(
        n, vec,
        [&](long i) {
            const float4 s0 = ((const float4 *)s)[i], s1 = ((const float4 *)(s + n))[i],
                         s2 = ((const float4 *)(s + 2 * n))[i];
            const float4 g0 = ((const float4 *)G)[i], g1 = ((const float4 *)(G + n))[i],
                         g2 = ((const float4 *)(G + 2 * n))[i];
            const float4 d = make_float4(g0.x * s0.x + g1.x * s1.x + g2.x * s2.x, g0.y * s0.y + g1.y * s1.y + g2.y * s2.y,
                                         g0.z * s0.z + g1.z * s1.z + g2.z * s2.z, g0.w * s0.w + g1.w * s1.w + g2.w * s2.w);
            ((float4 *)out)[i] = make_float4(g0.x * d.x, g0.y * d.y, g0.z * d.z, g0.w * d.w);
            ((float4 *)(out + n))[i] = make_float4(g1.x * d.x, g1.y * d.y, g1.z * d.z, g1.w * d.w);
            ((float4 *)(out + 2 * n))[i] = make_float4(g2.x * d.x, g2.y * d.y, g2.z * d.z, g2.w * d.w);
        },
        [&](long i) {
            const float d = G[i] * s[i] + G[n + i] * s[n + i] + G[2 * n + i] * s[2 * n + i];
            out[i] = G[i] * d;
            out[n + i] = G[n + i] * d;
            out[2 * n + i] = G[2 * n + i] * d;
        });
}

// ---- device-resident PCG scalars ----------------------------------------
__global__ void k_set_scalar(double *d, int slot, double value, Mb mb) {
    const long long mo_ = mb.offset(blockIdx.y); d = mshift(d, mo_); d[slot] = value; }

// gnorm = sqrt(<g,g>); ||g0|| latched on first use; eps_K rule when rtol <= 0
__global__ void k_tolerance(double *d, double rtol, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); d = mshift(d, mo_);
    const double gn = sqrt(d[S_GG]);
    d[S_GNORM] = gn;
    if (d[S_G0] == 0.0) d[S_G0] = gn;
    const double grel = d[S_G0] > 0.0 ? gn / d[S_G0] : 1.0;
    d[S_RTOL] = rtol > 0.0 ? rtol : fmin(sqrt(grel), 0.5);
}

__global__ void k_pcg_init(double *d, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); d = mshift(d, mo_);
    const double r0 = sqrt(d[S_RR]);
    d[S_R0] = r0;
    d[S_DONE] = (r0 == 0.0) ? 1.0 : 0.0;
    d[S_ITERS] = 0.0;
    d[S_FLAGS] = 0.0;
    d[S_REL] = (r0 == 0.0) ? 0.0 : 1.0;  // ||r|| / ||r0|| before the first iteration
    d[S_INNER] = 0.0;
    d[S_COPYZ] = 0.0;
    d[S_ALPHA] = 0.0;
    d[S_BETA] = 0.0;
}

// after kappa = <p, H p>: alpha, or stop on non-finite / non-positive kappa
__device__ void pcg_alpha_step(double *d)
{
    if (d[S_DONE] != 0.0) {
        d[S_ALPHA] = 0.0;
        return;
    }
    d[S_ITERS] += 1.0;
    const double kappa = d[S_KAPPA];
    if (!isfinite(kappa)) {
        d[S_FLAGS] = (double)((int)d[S_FLAGS] | 2);
        d[S_DONE] = 1.0;
        d[S_ALPHA] = 0.0;
    } else if (kappa <= 0.0) {
        d[S_FLAGS] = (double)((int)d[S_FLAGS] | 1);
        d[S_DONE] = 1.0;
        d[S_ALPHA] = 0.0;
        if (d[S_ITERS] == 1.0) d[S_COPYZ] = 1.0;
    } else {
        d[S_ALPHA] = d[S_RZ] / kappa;
    }
}

// x += alpha p (alpha from the device scalars; nothing when it is 0), or
// x = p when the first iteration stopped on its curvature (slot S_COPYZ:
// then p = M^{-1} r0)
__global__ void k_pcg_x_dev(long n, int vec, const double *__restrict__ d, const float *__restrict__ p,
                            float *__restrict__ x, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); d = mshift(d, mo_); p = mshift(p, mo_); x = mshift(x, mo_);
    if (d[S_COPYZ] != 0.0) {
        ew_loop(
            n, vec, [&](long i) { ((float4 *)x)[i] = ((const float4 *)p)[i]; }, [&](long i) { x[i] = p[i]; });
        return;
    }
    const float al = (float)d[S_ALPHA];
    if (al == 0.f) return;
    ew_loop(
        n, vec,
        [&](long i) {
            float4 *x4 = (float4 *)x + i;
            const float4 pv = ((const float4 *)p)[i], xv = *x4;
            *x4 = make_float4(__builtin_fmaf(al, pv.x, xv.x), __builtin_fmaf(al, pv.y, xv.y),
                              __builtin_fmaf(al, pv.z, xv.z), __builtin_fmaf(al, pv.w, xv.w));
        },
        [&](long i) { x[i] = __builtin_fmaf(al, p[i], x[i]); });
}

// after rr = <r, r>: relative residual and the stopping test
__device__ void pcg_conv_step(double *d)
{
    if (d[S_DONE] != 0.0) return;
    const double rn = sqrt(d[S_RR]);
    if (!isfinite(rn)) {
        d[S_FLAGS] = (double)((int)d[S_FLAGS] | 2);
        d[S_DONE] = 1.0;
        return;
    }
    d[S_REL] = rn / d[S_R0];
    if (rn <= d[S_RTOL] * d[S_R0]) d[S_DONE] = 1.0;
}

__global__ void k_pcg_conv(double *d, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); d = mshift(d, mo_);
    pcg_conv_step(d);
}

__device__ void pcg_beta_step(double *d)
{
    if (d[S_DONE] != 0.0) return;
    d[S_BETA] = d[S_RZN] / d[S_RZ];
    d[S_RZ] = d[S_RZN];
}

// One or two final reductions (partial, partial + np) into scalar slots a
// and b of d (b < 0: one), then the PCG's scalar steps that follow them, in
// the order alpha, conv, the relative residual into hist_dst, beta (bits of
// `after`), by thread 0: one launch instead of up to six.
__global__ __launch_bounds__(kRedThreads) void k_reduce_final_steps(const double *__restrict__ partial, int np,
                                                                    double *__restrict__ d, int a, int b,
                                                                    double scale, int after,
                                                                    double *__restrict__ hist_dst, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); partial = mshift(partial, mo_); d = mshift(d, mo_);
    const bool skip = mb.stopped(mo_);  // the partials are stale: keep the slots, run the (predicated) steps
    hist_dst = mshift(hist_dst, mo_);
    __shared__ double sh[2][kRedThreads];
    double acc0 = 0.0, acc1 = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        acc0 += partial[i];
        if (b >= 0) acc1 += partial[np + i];
    }
    sh[0][threadIdx.x] = acc0;
    sh[1][threadIdx.x] = acc1;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (!skip) {
        d[a] = scale * sh[0][0];
        if (b >= 0) d[b] = scale * sh[1][0];
    }
    if (after & kAfterAlpha) pcg_alpha_step(d);
    if (after & kAfterConv) pcg_conv_step(d);
    if (after & kAfterHist) hist_dst[0] = d[S_REL];
    if (after & kAfterBeta) pcg_beta_step(d);
}

__global__ void k_sum2(double *d, int dst, int a, int b, Mb mb) {
    const long long mo_ = mb.offset(blockIdx.y); d = mshift(d, mo_); d[dst] = d[a] + d[b]; }
__global__ void k_inner_link(double *inner, const double *outer, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); inner = mshift(inner, mo_); outer = mshift(outer, mo_);
    if (outer[S_DONE] != 0.0) inner[S_DONE] = 1.0;
}
__global__ void k_inner_accum(const double *inner, double *outer, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); inner = mshift(inner, mo_); outer = mshift(outer, mo_);
    if (outer[S_DONE] == 0.0) outer[S_INNER] += inner[S_ITERS];
}

__global__ void k_copy(long n, int vec, const float *__restrict__ x, float *__restrict__ out, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); x = mshift(x, mo_); out = mshift(out, mo_);
    if (mb.stopped(mo_)) return;
    ew_loop(
        n, vec, [&](long i) { ((float4 *)out)[i] = ((const float4 *)x)[i]; }, [&](long i) { out[i] = x[i]; });
}

// 16-byte accesses when every pointer is 16-byte aligned
static int vec_ok(std::initializer_list<const void *> ptrs)
{
    for (const void *q : ptrs)
        if (q && ((uintptr_t)q & 15)) return 0;
    return 1;
}

// workgroups of 256 for n elements (n / 4 groups when vec), at most 8192
static unsigned vec_blocks(long n, int vec = 0)
{
    if (vec) n = (n + 3) / 4;
    long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void dot_async(lddmm_plan *P, const float *a, const float *b, long n, int slot, double scale)
{
    Scope s(P, K_DOT);
    hipLaunchKernelGGL(k_reduce_partial<0>, dim3(kRedBlocks, P->mb.count), dim3(kRedThreads), 0, P->stream, a, b,
                       n, vec_ok({a, b}), P->red, P->mb);
    check_hip(hipGetLastError(), "k_reduce_partial");
    hipLaunchKernelGGL(k_reduce_final, dim3(1, P->mb.count), dim3(kRedThreads), 0, P->stream, P->red, kRedBlocks,
                       scalars(P) + slot, scale, P->mb);
    check_hip(hipGetLastError(), "k_reduce_final");
}

void sqdiff_async(lddmm_plan *P, const float *a, const float *b, long n, int slot, double scale)
{
    Scope s(P, K_DOT);
    hipLaunchKernelGGL(k_reduce_partial<1>, dim3(kRedBlocks, P->mb.count), dim3(kRedThreads), 0, P->stream, a, b,
                       n, vec_ok({a, b}), P->red, P->mb);
    check_hip(hipGetLastError(), "k_reduce_partial");
    hipLaunchKernelGGL(k_reduce_final, dim3(1, P->mb.count), dim3(kRedThreads), 0, P->stream, P->red, kRedBlocks,
                       scalars(P) + slot, scale, P->mb);
    check_hip(hipGetLastError(), "k_reduce_final");
}

double fetch_scalar(lddmm_plan *P, int slot)
{
    check_hip(hipMemcpyAsync(P->hscal + slot, scalars(P) + slot, sizeof(double), hipMemcpyDeviceToHost,
                             P->stream),
              "scalar copy");
    check_hip(hipStreamSynchronize(P->stream), "stream sync");
    return P->hscal[slot];
}

void axpby(lddmm_plan *P, long n, float a, const float *x, float b, const float *y, float *out)
{
    Scope s(P, K_VECOP);
    const int vec = vec_ok({x, y, out});
    hipLaunchKernelGGL(k_axpby, dim3(vec_blocks(n, vec), P->mb.count), dim3(256), 0, P->stream, n, vec, a, x, b, y, out,
                       P->mb);
    check_hip(hipGetLastError(), "k_axpby");
}

void fill(lddmm_plan *P, long n, float value, float *out)
{
    Scope s(P, K_VECOP);
    const int vec = vec_ok({out});
    hipLaunchKernelGGL(k_fill, dim3(vec_blocks(n, vec), P->mb.count), dim3(256), 0, P->stream, n, vec, value, out, P->mb);
    check_hip(hipGetLastError(), "k_fill");
}

#define LAUNCH1(kern, ...)                                                                  \
    do {                                                                                    \
        Scope s_(P, K_VECOP);                                                               \
        hipLaunchKernelGGL(kern, dim3(1, P->mb.count), dim3(1), 0, P->stream, __VA_ARGS__, P->mb); \
        check_hip(hipGetLastError(), #kern);                                                \
    } while (0)

void dev_set_scalar(lddmm_plan *P, int slot, double value) { LAUNCH1(k_set_scalar, scalars(P), slot, value); }
void dev_tolerance(lddmm_plan *P, double rtol) { LAUNCH1(k_tolerance, scalars(P), rtol); }
void dev_pcg_init(lddmm_plan *P) { LAUNCH1(k_pcg_init, scalars(P)); }
void dev_pcg_conv(lddmm_plan *P) { LAUNCH1(k_pcg_conv, scalars(P)); }
void dev_sum(lddmm_plan *P, int dst, int a, int b) { LAUNCH1(k_sum2, scalars(P), dst, a, b); }
void dev_inner_link(lddmm_plan *P, double *outer) { LAUNCH1(k_inner_link, scalars(P), outer); }
void dev_inner_accum(lddmm_plan *P, double *outer) { LAUNCH1(k_inner_accum, scalars(P), outer); }

void dev_pcg_x(lddmm_plan *P, long n, const float *p, float *x)
{
    Scope s(P, K_VECOP);
    const int vec = vec_ok({p, x});
    hipLaunchKernelGGL(k_pcg_x_dev, dim3(vec_blocks(n, vec), P->mb.count), dim3(256), 0, P->stream, n, vec, scalars(P),
                       p, x, P->mb);
    check_hip(hipGetLastError(), "k_pcg_x_dev");
}

void dev_reduce_final(lddmm_plan *P, const double *partial, int slot, double scale)
{
    dev_reduce_final_steps(P, partial, slot, -1, scale, 0, nullptr);
}

void dev_reduce_final_steps(lddmm_plan *P, const double *partial, int a, int b, double scale, int after,
                            double *hist_dst, int np)
{
    Scope s(P, K_DOT);
    hipLaunchKernelGGL(k_reduce_final_steps, dim3(1, P->mb.count), dim3(kRedThreads), 0, P->stream, partial, np,
                       scalars(P), a, b, scale, after, hist_dst, P->mb);
    check_hip(hipGetLastError(), "k_reduce_final_steps");
}

void h0_point(lddmm_plan *P, const float *s, const float *G, float *out, float beta0)
{
    Scope sc(P, K_VECOP);
    const long n = P->N;
    const int vec = vec_ok({s, s + n, G, G + n, out, out + n});
    hipLaunchKernelGGL(k_h0_point, dim3(vec_blocks(n, vec), P->mb.count), dim3(256), 0, P->stream, n, vec, beta0, s, G,
                       out, P->mb);
    check_hip(hipGetLastError(), "k_h0_point");
}

void h0_rank1(lddmm_plan *P, const float *s, const float *G, float *out)
{
    Scope sc(P, K_VECOP);
    const long n = P->N;
    const int vec = vec_ok({s, s + n, G, G + n, out, out + n});
    hipLaunchKernelGGL(k_h0_rank1, dim3(vec_blocks(n, vec), P->mb.count), dim3(256), 0, P->stream, n, vec, s, G, out,
                       P->mb);
    check_hip(hipGetLastError(), "k_h0_rank1");
}

void copy_kernel(lddmm_plan *P, long n, const float *x, float *out)
{
    Scope s(P, K_VECOP);
    const int vec = vec_ok({x, out});
    hipLaunchKernelGGL(k_copy, dim3(vec_blocks(n, vec), P->mb.count), dim3(256), 0, P->stream, n, vec, x, out, P->mb);
    check_hip(hipGetLastError(), "k_copy");
}

}  // namespace lddmm
