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

}  // namespace lddmm
