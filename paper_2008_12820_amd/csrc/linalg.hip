// Vector algebra of the PCG / Gauss-Newton loop for gfx950: FP64-accumulating
// deterministic reductions (fixed grid, fixed tree) and FP32 vector updates.
#include "internal.hpp"

namespace lddmm {

constexpr int kRedThreads = 256;

// mode 0: sum a*b;  mode 1: sum (a-b)^2
template <int MODE>
__global__ __launch_bounds__(kRedThreads) void k_reduce_partial(const float *__restrict__ a,
                                                                const float *__restrict__ b, long n,
                                                                double *__restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (MODE == 0) {
            acc += (double)a[i] * (double)b[i];
        } else {
            const double d = (double)a[i] - (double)b[i];
            acc += d * d;
        }
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
                                                              double scale)
{
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

__global__ void k_axpby(long n, float a, const float *__restrict__ x, float b,
                        const float *__restrict__ y, float *__restrict__ out)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

__global__ void k_fill(long n, float value, float *__restrict__ out)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = value;
}

__global__ void k_pcg_xr(long n, float al, const float *__restrict__ p, const float *__restrict__ q,
                         float *__restrict__ x, float *__restrict__ r)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        x[i] += al * p[i];
        r[i] -= al * q[i];
    }
}

// ---- device-resident PCG scalars ----------------------------------------
__global__ void k_set_scalar(double *d, int slot, double value) { d[slot] = value; }

// gnorm = sqrt(<g,g>); ||g0|| latched on first use; eps_K rule when rtol <= 0
__global__ void k_tolerance(double *d, double rtol)
{
    const double gn = sqrt(d[S_GG]);
    d[S_GNORM] = gn;
    if (d[S_G0] == 0.0) d[S_G0] = gn;
    const double grel = d[S_G0] > 0.0 ? gn / d[S_G0] : 1.0;
    d[S_RTOL] = rtol > 0.0 ? rtol : fmin(sqrt(grel), 0.5);
}

__global__ void k_pcg_init(double *d)
{
    const double r0 = sqrt(d[S_RR]);
    d[S_R0] = r0;
    d[S_DONE] = (r0 == 0.0) ? 1.0 : 0.0;
    d[S_ITERS] = 0.0;
    d[S_FLAGS] = 0.0;
    d[S_REL] = 0.0;
    d[S_COPYZ] = 0.0;
    d[S_ALPHA] = 0.0;
    d[S_BETA] = 0.0;
}

// after kappa = <p, H p>: alpha, or stop on non-finite / non-positive kappa
__global__ void k_pcg_alpha(double *d)
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

__global__ void k_pcg_xr_dev(long n, const double *__restrict__ d, const float *__restrict__ p,
                             const float *__restrict__ q, float *__restrict__ x, float *__restrict__ r)
{
    const float al = (float)d[S_ALPHA];
    if (al == 0.f) return;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        x[i] += al * p[i];
        r[i] -= al * q[i];
    }
}

__global__ void k_copy_if(long n, const double *__restrict__ d, const float *__restrict__ z,
                          float *__restrict__ x)
{
    if (d[S_COPYZ] == 0.0) return;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = z[i];
}

// after rr = <r, r>: relative residual and the stopping test
__global__ void k_pcg_conv(double *d)
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

__global__ void k_pcg_beta(double *d)
{
    if (d[S_DONE] != 0.0) return;
    d[S_BETA] = d[S_RZN] / d[S_RZ];
    d[S_RZ] = d[S_RZN];
}

__global__ void k_pcg_p(long n, const double *__restrict__ d, const float *__restrict__ z,
                        float *__restrict__ p)
{
    if (d[S_DONE] != 0.0) return;
    const float be = (float)d[S_BETA];
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = z[i] + be * p[i];
}

__global__ void k_sum2(double *d, int dst, int a, int b) { d[dst] = d[a] + d[b]; }

__global__ void k_copy(long n, const float *__restrict__ x, float *__restrict__ out)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = x[i];
}

static unsigned vec_blocks(long n)
{
    long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void dot_async(lddmm_plan *P, const float *a, const float *b, long n, int slot, double scale)
{
    Scope s(P, K_DOT);
    hipLaunchKernelGGL(k_reduce_partial<0>, dim3(kRedBlocks), dim3(kRedThreads), 0, P->stream, a, b,
                       n, P->red);
    check_hip(hipGetLastError(), "k_reduce_partial");
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, P->stream, P->red, kRedBlocks,
                       P->dscal + slot, scale);
    check_hip(hipGetLastError(), "k_reduce_final");
}

void sqdiff_async(lddmm_plan *P, const float *a, const float *b, long n, int slot, double scale)
{
    Scope s(P, K_DOT);
    hipLaunchKernelGGL(k_reduce_partial<1>, dim3(kRedBlocks), dim3(kRedThreads), 0, P->stream, a, b,
                       n, P->red);
    check_hip(hipGetLastError(), "k_reduce_partial");
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, P->stream, P->red, kRedBlocks,
                       P->dscal + slot, scale);
    check_hip(hipGetLastError(), "k_reduce_final");
}

double fetch_scalar(lddmm_plan *P, int slot)
{
    check_hip(hipMemcpyAsync(P->hscal + slot, P->dscal + slot, sizeof(double), hipMemcpyDeviceToHost,
                             P->stream),
              "scalar copy");
    check_hip(hipStreamSynchronize(P->stream), "stream sync");
    return P->hscal[slot];
}

void axpby(lddmm_plan *P, long n, float a, const float *x, float b, const float *y, float *out)
{
    Scope s(P, K_VECOP);
    hipLaunchKernelGGL(k_axpby, dim3(vec_blocks(n)), dim3(256), 0, P->stream, n, a, x, b, y, out);
    check_hip(hipGetLastError(), "k_axpby");
}

void fill(lddmm_plan *P, long n, float value, float *out)
{
    Scope s(P, K_VECOP);
    hipLaunchKernelGGL(k_fill, dim3(vec_blocks(n)), dim3(256), 0, P->stream, n, value, out);
    check_hip(hipGetLastError(), "k_fill");
}

void pcg_update_xr(lddmm_plan *P, long n, float al, const float *p, const float *q, float *x, float *r)
{
    Scope s(P, K_VECOP);
    hipLaunchKernelGGL(k_pcg_xr, dim3(vec_blocks(n)), dim3(256), 0, P->stream, n, al, p, q, x, r);
    check_hip(hipGetLastError(), "k_pcg_xr");
}

#define LAUNCH1(kern, ...)                                                                  \
    do {                                                                                    \
        Scope s_(P, K_VECOP);                                                               \
        hipLaunchKernelGGL(kern, dim3(1), dim3(1), 0, P->stream, __VA_ARGS__);              \
        check_hip(hipGetLastError(), #kern);                                                \
    } while (0)

void dev_set_scalar(lddmm_plan *P, int slot, double value) { LAUNCH1(k_set_scalar, P->dscal, slot, value); }
void dev_tolerance(lddmm_plan *P, double rtol) { LAUNCH1(k_tolerance, P->dscal, rtol); }
void dev_pcg_init(lddmm_plan *P) { LAUNCH1(k_pcg_init, P->dscal); }
void dev_pcg_alpha(lddmm_plan *P) { LAUNCH1(k_pcg_alpha, P->dscal); }
void dev_pcg_conv(lddmm_plan *P) { LAUNCH1(k_pcg_conv, P->dscal); }
void dev_pcg_beta(lddmm_plan *P) { LAUNCH1(k_pcg_beta, P->dscal); }
void dev_sum(lddmm_plan *P, int dst, int a, int b) { LAUNCH1(k_sum2, P->dscal, dst, a, b); }

void dev_pcg_xr(lddmm_plan *P, long n, const float *p, const float *q, float *x, float *r)
{
    Scope s(P, K_VECOP);
    hipLaunchKernelGGL(k_pcg_xr_dev, dim3(vec_blocks(n)), dim3(256), 0, P->stream, n, P->dscal, p, q, x, r);
    check_hip(hipGetLastError(), "k_pcg_xr_dev");
}

void dev_copy_if(lddmm_plan *P, long n, const float *z, float *x)
{
    Scope s(P, K_VECOP);
    hipLaunchKernelGGL(k_copy_if, dim3(vec_blocks(n)), dim3(256), 0, P->stream, n, P->dscal, z, x);
    check_hip(hipGetLastError(), "k_copy_if");
}

void dev_pcg_p(lddmm_plan *P, long n, const float *z, float *p)
{
    Scope s(P, K_VECOP);
    hipLaunchKernelGGL(k_pcg_p, dim3(vec_blocks(n)), dim3(256), 0, P->stream, n, P->dscal, z, p);
    check_hip(hipGetLastError(), "k_pcg_p");
}

void copy_kernel(lddmm_plan *P, long n, const float *x, float *out)
{
    Scope s(P, K_VECOP);
    hipLaunchKernelGGL(k_copy, dim3(vec_blocks(n)), dim3(256), 0, P->stream, n, x, out);
    check_hip(hipGetLastError(), "k_copy");
}

}  // namespace lddmm
