// Shared device helpers and host-side declarations of the gfx950 LDDMM library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lddmm.h"

namespace lddmm {

// ---------------------------------------------------------------------------
// complex helpers (float2 / double2 as complex numbers)
// ---------------------------------------------------------------------------
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cmulc(float2 a, float2 b)  // a * conj(b)
{
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__host__ __device__ inline float2 cmuli(float2 a) { return make_float2(-a.y, a.x); }  // i * a

// ---------------------------------------------------------------------------
// Members of a batched plan: count copies of one plan's workspace, stride
// bytes apart (a batch of registrations of one grid size).  A kernel launched
// for all of them takes its member index from a grid dimension and shifts
// every workspace pointer it was given by index * stride; tables the members
// share (FFT twiddles) are not shifted.  A plain plan: stride 0, count 1.
// ---------------------------------------------------------------------------
// p + off bytes; NULL stays NULL
template <class T>
__device__ __forceinline__ T *mshift(T *p, long long off)
{
    return p ? reinterpret_cast<T *>(reinterpret_cast<uintptr_t>(p) + (uintptr_t)off) : p;
}

struct Mb {
    long long stride = 0;
    int count = 1;
    // Inside a device-resident PCG loop: the loop's stop flag and that of the
    // PCG it preconditions, or NULL (member 0's; the members' at the same
    // stride).  The vector kernels of an iteration queued after a stop
    // (transport gathers, transform passes, spectral updates, reductions)
    // then return at once: their results would go only to steps the stop
    // predicates off.  Both NULL outside such loops.
    const double *done = nullptr, *done2 = nullptr;
    __host__ __device__ long long offset(unsigned idx) const { return (long long)idx * stride; }
    __device__ bool stopped(long long off) const
    {
        return (done && *mshift(done, off) != 0.0) || (done2 && *mshift(done2, off) != 0.0);
    }
};

// ---------------------------------------------------------------------------
// FFT line plans
// ---------------------------------------------------------------------------
constexpr int kMaxPasses = 12;

struct RadixPlan {
    int L;                 // line length
    int np;                // number of passes
    int r[kMaxPasses];     // radix of each pass (8, 4, 2, 3 or 5)
};

RadixPlan make_radix_plan(int L);

// Kernel classes for the per-kernel event timing.
enum KernelId : int {
    K_R2C_X3 = 0,
    K_FFT_COLS,
    K_SPECTRAL_X1,
    K_C2R_X3,
    K_DEPARTURE,
    K_STATE_STEP,
    K_GATHER_VEC,
    K_ADJ_COEF,
    K_ADJ_STEP,
    K_INCSTATE_INIT,
    K_INCSTATE_STEP,
    K_BODY_FORCE,
    K_DOT,
    K_VECOP,
    K_PACK,
    K_ADJ_BODY,
    K_FD8,
    K_NUM_KERNELS
};
const char *kernel_name(int id);

}  // namespace lddmm
