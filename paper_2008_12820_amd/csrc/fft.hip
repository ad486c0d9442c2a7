// Hand-written 3D real FFT and the spectral operators of the method for gfx950.
//
// The paper applies A, (beta A)^{-1} and the Leray projection in the spectral
// domain (Section 2, "two FFTs and one Hadamard product"); first derivatives
// are spectral here as in the CPU version of the method (Section 3.2).
//
// Structure (x3 is contiguous in memory):
//   r2c_x3   : each row of n3 reals is read once, packed as n3/2 complex
//              values, transformed in LDS and split into the half spectrum
//              (k3 = 0 .. n3/2-1 in the main array, k3 = n3/2 in a separate
//              Nyquist plane so the main rows stay n3/2 wide and aligned).
//   fft_cols : complex pass along x2 (or x1) over tiles of TW adjacent k3
//              columns, staged through LDS, Stockham autosort radix 8/4/2/3/5.
//   x1_*     : forward x1 pass, pointwise symbol over all fields of the
//              operator, inverse x1 pass in one kernel -- one HBM round trip
//              instead of three.
//   c2r_x3   : the inverse of r2c_x3, with the output scale folded in.
//
// Precision: roundoff of an FP32 forward transform is spread evenly over all
// wavenumbers, and an unbounded symbol (|k|, |k|^2, |k|^4) multiplies it by up
// to |k_max|^p while the band-limited signal sits at small |k|.  So the
// forward chain (r2c, x2, x1) of every field that meets such a symbol runs in
// FP64 (FP64 storage between passes); bounded symbols (Leray, (beta A)^{-1})
// and every inverse transform run in FP32, whose roundoff is relative to the
// output.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <map>
#include <set>
#include <sstream>
#include <string>
#include <type_traits>

namespace lddmm {

// ---------------------------------------------------------------------------
// complex arithmetic templated on float2 / double2
// ---------------------------------------------------------------------------
template <class C> struct RealOf;
template <> struct RealOf<float2> { using type = float; };
template <> struct RealOf<double2> { using type = double; };
template <class R> struct CplxOf;
template <> struct CplxOf<float> { using type = float2; };
template <> struct CplxOf<double> { using type = double2; };

template <class C>
__device__ __forceinline__ C mk(typename RealOf<C>::type x, typename RealOf<C>::type y)
{
    C r;
    r.x = x;
    r.y = y;
    return r;
}
template <class C> __device__ __forceinline__ C add(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <class C> __device__ __forceinline__ C sub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <class C> __device__ __forceinline__ C mul(C a, C b)
{
    return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class C> __device__ __forceinline__ C mulc(C a, C b)  // a * conj(b)
{
    return mk<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <class C> __device__ __forceinline__ C conj_(C a) { return mk<C>(a.x, -a.y); }
template <class C> __device__ __forceinline__ C scl(C a, typename RealOf<C>::type s) { return mk<C>(a.x * s, a.y * s); }
template <class C> __device__ __forceinline__ C muli(C a) { return mk<C>(-a.y, a.x); }  // i * a
template <class C, bool INV> __device__ __forceinline__ C mul_mi(C a)  // -i a forward, +i a inverse
{
    return INV ? mk<C>(-a.y, a.x) : mk<C>(a.y, -a.x);
}
__device__ __forceinline__ float2 to_f2(double2 a) { return make_float2((float)a.x, (float)a.y); }
__device__ __forceinline__ float2 to_f2(float2 a) { return a; }

// ---------------------------------------------------------------------------
// small DFTs
// ---------------------------------------------------------------------------
template <class C, bool INV>
__device__ __forceinline__ void dft2(C *v)
{
    C a = v[0], b = v[1];
    v[0] = add(a, b);
    v[1] = sub(a, b);
}

template <class C, bool INV>
__device__ __forceinline__ void dft4(C &v0, C &v1, C &v2, C &v3)
{
    C t0 = add(v0, v2), t1 = sub(v0, v2);
    C t2 = add(v1, v3), t3 = mul_mi<C, INV>(sub(v1, v3));
    v0 = add(t0, t2);
    v2 = sub(t0, t2);
    v1 = add(t1, t3);
    v3 = sub(t1, t3);
}

template <class C, bool INV>
__device__ __forceinline__ void dft8(C *v)
{
    using R = typename RealOf<C>::type;
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<C, INV>(e0, e1, e2, e3);
    dft4<C, INV>(o0, o1, o2, o3);
    const R r = R(0.70710678118654752440);
    const C w1 = INV ? mk<C>(r, r) : mk<C>(r, -r);
    const C w3 = INV ? mk<C>(-r, r) : mk<C>(-r, -r);
    o1 = mul(o1, w1);
    o2 = mul_mi<C, INV>(o2);
    o3 = mul(o3, w3);
    v[0] = add(e0, o0);
    v[4] = sub(e0, o0);
    v[1] = add(e1, o1);
    v[5] = sub(e1, o1);
    v[2] = add(e2, o2);
    v[6] = sub(e2, o2);
    v[3] = add(e3, o3);
    v[7] = sub(e3, o3);
}

template <class C, bool INV>
__device__ __forceinline__ void dft3(C *v)
{
    using R = typename RealOf<C>::type;
    const R s = R(0.86602540378443864676);  // sin(2 pi / 3)
    C t = add(v[1], v[2]);
    C d = sub(v[1], v[2]);
    C m = mk<C>(v[0].x - R(0.5) * t.x, v[0].y - R(0.5) * t.y);
    C sd = mul_mi<C, INV>(scl(d, s));
    v[0] = add(v[0], t);
    v[1] = add(m, sd);
    v[2] = sub(m, sd);
}

template <class C, bool INV>
__device__ __forceinline__ void dft5(C *v)
{
    using R = typename RealOf<C>::type;
    const R c1 = R(0.30901699437494742410);   // cos(2 pi/5)
    const R c2 = R(-0.80901699437494742410);  // cos(4 pi/5)
    const R s1 = R(0.95105651629515357212);   // sin(2 pi/5)
    const R s2 = R(0.58778525229247312917);   // sin(4 pi/5)
    C t1 = add(v[1], v[4]), t2 = add(v[2], v[3]);
    C d1 = sub(v[1], v[4]), d2 = sub(v[2], v[3]);
    C a1 = mk<C>(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    C a2 = mk<C>(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    C b1 = mk<C>(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
    C b2 = mk<C>(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
    C ib1 = mul_mi<C, INV>(b1), ib2 = mul_mi<C, INV>(b2);
    v[0] = add(v[0], add(t1, t2));
    v[1] = add(a1, ib1);
    v[4] = sub(a1, ib1);
    v[2] = add(a2, ib2);
    v[3] = sub(a2, ib2);
}

template <int R, class C, bool INV>
__device__ __forceinline__ void dft_small(C *v)
{
    if constexpr (R == 2) dft2<C, INV>(v);
    else if constexpr (R == 4) dft4<C, INV>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<C, INV>(v);
    else if constexpr (R == 3) dft3<C, INV>(v);
    else dft5<C, INV>(v);
}

// 16-point DFT in registers, natural order in and out: DFT4 over the four
// stride-4 subsequences, twiddles W16^(n1 k2), DFT4 across, 4x4 transpose
template <class C, bool INV>
__device__ __forceinline__ void dft16(C *v)
{
    using R = typename RealOf<C>::type;
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) dft4<C, INV>(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]);
    // Y[n1][k2] sits at v[n1 + 4 k2]; W16^m = cos(pi m / 8) + sg i sin(pi m / 8)
    const R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173), h = R(0.70710678118654752440);
    const R sg = INV ? R(1) : R(-1);
    v[5] = mul(v[5], mk<C>(c1, sg * s1));     // m = 1
    v[9] = mul(v[9], mk<C>(h, sg * h));       // m = 2
    v[13] = mul(v[13], mk<C>(s1, sg * c1));   // m = 3
    v[6] = mul(v[6], mk<C>(h, sg * h));       // m = 2
    v[10] = mul_mi<C, INV>(v[10]);            // m = 4
    v[14] = mul(v[14], mk<C>(-h, sg * h));    // m = 6
    v[7] = mul(v[7], mk<C>(s1, sg * c1));     // m = 3
    v[11] = mul(v[11], mk<C>(-h, sg * h));    // m = 6
    v[15] = mul(v[15], mk<C>(-c1, -sg * s1)); // m = 9
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) dft4<C, INV>(v[4 * k2], v[4 * k2 + 1], v[4 * k2 + 2], v[4 * k2 + 3]);
    C t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) t[4 * k1 + k2] = v[4 * k2 + k1];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = t[i];
}

template <int R, class C, bool INV>
__device__ __forceinline__ void dft_reg(C *v)
{
    if constexpr (R == 16) dft16<C, INV>(v);
    else dft_small<R, C, INV>(v);
}

// ---------------------------------------------------------------------------
// Register line FFTs for the column passes.  A 256-thread workgroup owns TW
// adjacent columns of lines of L = R1 * R2 points.  Stage 1: a task (c, s)
// loads the stride-R2 subsequence n = s + R2 m of column c into registers,
// takes its DFT_R1 and multiplies by W_L^(s k1); one LDS exchange; stage 2:
// a task (c, k1) takes the DFT_R2 over s and holds X[k1 + R1 k2], k2 < R2.
// The inverse runs the two stages the other way round from that register
// layout, so a pointwise symbol can be applied in between with no exchange.
// ---------------------------------------------------------------------------
template <int L>
struct RegPlan {
    static constexpr bool ok = false;
    static constexpr int R1 = 1, R2 = 1, TW = 1;
};
template <>
struct RegPlan<64> {
    static constexpr bool ok = true;
    static constexpr int R1 = 8, R2 = 8, TW = 32;
};
template <>
struct RegPlan<128> {
    static constexpr bool ok = true;
    static constexpr int R1 = 16, R2 = 8, TW = 32;
};
template <>
struct RegPlan<256> {
    static constexpr bool ok = true;
    static constexpr int R1 = 16, R2 = 16, TW = 16;
};

template <int L>
struct RegShape {
    using P = RegPlan<L>;
    static constexpr int R1 = P::R1, R2 = P::R2, TW = P::TW;
    static constexpr int T1 = TW * R2 / 256;  // stage-1 tasks per thread
    static constexpr int T2 = TW * R1 / 256;  // stage-2 tasks per thread
    static constexpr int PITCH = R2 * TW + 1; // exchange row per k1 (+1 against bank conflicts)
    static constexpr int XCH = R1 * PITCH;    // exchange buffer, complex values
    static_assert(T1 * 256 == TW * R2 && T2 * 256 == TW * R1, "tasks must fill the workgroup");
};

// load(n, c) returns element n of column c of the tile (zero past the last
// column); on return out[u][k2] = X[k1 + R1 k2] of task u (c, k1).
template <int L, bool INV, class C, class LoadF>
__device__ __forceinline__ void reg_fft(LoadF &&load, C *X, C (&out)[RegShape<L>::T2][RegShape<L>::R2],
                                        const C *__restrict__ tw)
{
    using S = RegShape<L>;
    constexpr int R1 = S::R1, R2 = S::R2, TW = S::TW, PITCH = S::PITCH;
    __syncthreads();  // X may still be read by a previous transform
#pragma unroll
    for (int u = 0; u < S::T1; ++u) {
        const int task = (int)threadIdx.x + 256 * u, c = task % TW, s = task / TW;
        C v[R1];
#pragma unroll
        for (int m = 0; m < R1; ++m) v[m] = load(s + R2 * m, c);
        dft_reg<R1, C, INV>(v);
#pragma unroll
        for (int k1 = 1; k1 < R1; ++k1) v[k1] = INV ? mulc(v[k1], tw[s * k1]) : mul(v[k1], tw[s * k1]);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) X[k1 * PITCH + s * TW + c] = v[k1];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < S::T2; ++u) {
        const int task = (int)threadIdx.x + 256 * u, c = task % TW, k1 = task / TW;
#pragma unroll
        for (int s = 0; s < R2; ++s) out[u][s] = X[k1 * PITCH + s * TW + c];
        dft_reg<R2, C, INV>(out[u]);
    }
}

// inverse from the register layout reg_fft leaves (in is overwritten):
// store(n, c, value) for every element of the tile.
template <int L, class C, class StoreF>
__device__ __forceinline__ void reg_ifft(C (&in)[RegShape<L>::T2][RegShape<L>::R2], C *X, StoreF &&store,
                                         const C *__restrict__ tw)
{
    using S = RegShape<L>;
    constexpr int R1 = S::R1, R2 = S::R2, TW = S::TW, PITCH = S::PITCH;
    __syncthreads();  // X may still be read by a previous transform
#pragma unroll
    for (int u = 0; u < S::T2; ++u) {
        const int task = (int)threadIdx.x + 256 * u, c = task % TW, k1 = task / TW;
        dft_reg<R2, C, true>(in[u]);
#pragma unroll
        for (int na = 1; na < R2; ++na) in[u][na] = mulc(in[u][na], tw[na * k1]);
#pragma unroll
        for (int na = 0; na < R2; ++na) X[k1 * PITCH + na * TW + c] = in[u][na];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < S::T1; ++u) {
        const int task = (int)threadIdx.x + 256 * u, c = task % TW, na = task / TW;
        C v[R1];
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) v[k1] = X[k1 * PITCH + na * TW + c];
        dft_reg<R1, C, true>(v);
#pragma unroll
        for (int nb = 0; nb < R1; ++nb) store(na + R2 * nb, c, v[nb]);
    }
}

// ---------------------------------------------------------------------------
// Stockham autosort passes in LDS.  An LDS tile holds TW lines of length L;
// element (n, c) of line c sits at n*TW + c (CFAST: the columns are the
// coalesced direction) or at c*LP + n (rows contiguous).
// ---------------------------------------------------------------------------
template <int R, class C, bool INV, bool CFAST>
__device__ __forceinline__ void stockham_pass(const C *__restrict__ src, C *__restrict__ dst, int L,
                                              int TW, int logTW, int LP, int Ns,
                                              const C *__restrict__ tw, int tid, int nthr)
{
    const int LR = L / R;
    const int step = L / (Ns * R);
    const int nb = LR * TW;
    for (int b = tid; b < nb; b += nthr) {
        int j, c;
        if (CFAST) {
            c = b & (TW - 1);
            j = b >> logTW;
        } else {
            j = b % LR;
            c = b / LR;
        }
        const int jm = j % Ns;
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int n = j + r * LR;
            v[r] = src[CFAST ? (n * TW + c) : (c * LP + n)];
        }
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const C w = tw[jm * r * step];
                v[r] = INV ? mulc(v[r], w) : mul(v[r], w);
            }
        }
        dft_small<R, C, INV>(v);
        const int idxD = (j - jm) * R + jm;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int n = idxD + r * Ns;
            dst[CFAST ? (n * TW + c) : (c * LP + n)] = v[r];
        }
    }
}

// Full line FFT of a tile; the data start in A, B is scratch.  Returns the
// buffer holding the result (A for an even pass count, B for an odd one).
// Every thread of the block must call it; it ends with a barrier.
template <bool INV, bool CFAST, class C>
__device__ C *lds_fft(C *A, C *B, int TW, int logTW, int LP, const RadixPlan &rp,
                      const C *__restrict__ tw, int tid, int nthr)
{
    C *s = A, *d = B;
    int Ns = 1;
    const int L = rp.L;
    for (int p = 0; p < rp.np; ++p) {
        const int R = rp.r[p];
        switch (R) {
        case 8: stockham_pass<8, C, INV, CFAST>(s, d, L, TW, logTW, LP, Ns, tw, tid, nthr); break;
        case 4: stockham_pass<4, C, INV, CFAST>(s, d, L, TW, logTW, LP, Ns, tw, tid, nthr); break;
        case 2: stockham_pass<2, C, INV, CFAST>(s, d, L, TW, logTW, LP, Ns, tw, tid, nthr); break;
        case 3: stockham_pass<3, C, INV, CFAST>(s, d, L, TW, logTW, LP, Ns, tw, tid, nthr); break;
        default: stockham_pass<5, C, INV, CFAST>(s, d, L, TW, logTW, LP, Ns, tw, tid, nthr); break;
        }
        __syncthreads();
        C *t = s;
        s = d;
        d = t;
        Ns *= R;
    }
    return s;
}

// Compile-time line lengths: the same greedy radix sequence as
// make_radix_plan, with every pass's stride, butterfly count and twiddle
// step known at compile time (no runtime integer division in the index math).
__host__ __device__ constexpr int next_radix(int n)
{
    return n % 8 == 0 ? 8 : (n % 4 == 0 ? 4 : (n % 2 == 0 ? 2 : (n % 3 == 0 ? 3 : 5)));
}

template <int R, int L, int Ns, class C, bool INV, bool CFAST>
__device__ __forceinline__ void stockham_pass_fixed(const C *__restrict__ src, C *__restrict__ dst, int TW,
                                                    int logTW, int LP, const C *__restrict__ tw, int tid,
                                                    int nthr)
{
    constexpr int LR = L / R;
    constexpr int step = L / (Ns * R);
    const int nb = LR * TW;
    for (int b = tid; b < nb; b += nthr) {
        int j, c;
        if (CFAST) {
            c = b & (TW - 1);
            j = b >> logTW;
        } else {
            j = b % LR;
            c = b / LR;
        }
        const int jm = j % Ns;
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int n = j + r * LR;
            v[r] = src[CFAST ? (n * TW + c) : (c * LP + n)];
        }
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const C w = tw[jm * r * step];
                v[r] = INV ? mulc(v[r], w) : mul(v[r], w);
            }
        }
        dft_small<R, C, INV>(v);
        const int idxD = (j - jm) * R + jm;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int n = idxD + r * Ns;
            dst[CFAST ? (n * TW + c) : (c * LP + n)] = v[r];
        }
    }
}

template <bool INV, bool CFAST, class C, int L, int Ns = 1>
__device__ __forceinline__ C *lds_fft_fixed(C *s, C *d, int TW, int logTW, int LP, const C *__restrict__ tw,
                                            int tid, int nthr)
{
    if constexpr (Ns == L) {
        return s;
    } else {
        constexpr int R = next_radix(L / Ns);
        stockham_pass_fixed<R, L, Ns, C, INV, CFAST>(s, d, TW, logTW, LP, tw, tid, nthr);
        __syncthreads();
        return lds_fft_fixed<INV, CFAST, C, L, Ns * R>(d, s, TW, logTW, LP, tw, tid, nthr);
    }
}

// LF > 0: compile-time length LF; LF = 0: the runtime plan
template <bool INV, bool CFAST, int LF, class C>
__device__ __forceinline__ C *lds_fft_any(C *A, C *B, int TW, int logTW, int LP, const RadixPlan &rp,
                                          const C *__restrict__ tw, int tid, int nthr)
{
    if constexpr (LF > 0)
        return lds_fft_fixed<INV, CFAST, C, LF>(A, B, TW, logTW, LP, tw, tid, nthr);
    else
        return lds_fft<INV, CFAST, C>(A, B, TW, logTW, LP, rp, tw, tid, nthr);
}

// runs fn.template operator()<LF>() with LF = L for the compiled lengths, else 0
template <class Fn>
static void with_len(int L, Fn &&fn)
{
    switch (L) {
    case 32: fn.template operator()<32>(); break;
    case 48: fn.template operator()<48>(); break;
    case 64: fn.template operator()<64>(); break;
    case 80: fn.template operator()<80>(); break;
    case 96: fn.template operator()<96>(); break;
    case 128: fn.template operator()<128>(); break;
    case 160: fn.template operator()<160>(); break;
    case 256: fn.template operator()<256>(); break;
    case 512: fn.template operator()<512>(); break;
    default: fn.template operator()<0>(); break;
    }
}

// first buffer to load into so that a forward transform ends in `home`
template <class C>
__device__ __forceinline__ C *load_target(const RadixPlan &rp, C *home, C *other)
{
    return (rp.np & 1) ? other : home;
}

constexpr int kFftThreads = 256;

// Launch with dynamic LDS; above 64 KB the kernel's limit is raised (once
// per kernel) to kLdsMax.
static void allow_big_lds(const void *k)
{
    static std::set<const void *> done;
    if (done.count(k)) return;
    check_hip(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax),
              "hipFuncSetAttribute");
    done.insert(k);
}

#define FFT_LAUNCH(kern, grid, lds, stream, ...)                                   \
    do {                                                                           \
        if ((lds) > 65536) allow_big_lds((const void *)(kern));                     \
        hipLaunchKernelGGL(kern, grid, dim3(kFftThreads), lds, stream, __VA_ARGS__); \
    } while (0)

// ---------------------------------------------------------------------------
// Register Stockham passes along x3 rows (the R2C / C2R passes): a workgroup
// of RB M / 8 threads owns RB rows of M = n3/2 complex points, eight values
// per thread; task (row, j) with the butterfly index j fastest, so the
// global accesses of one element r of a pass are contiguous along the row.
// RBA and RBB: the two row counts the autotuner chooses between.
// ---------------------------------------------------------------------------
template <int M>
struct RowPlan {
    static constexpr bool ok = false;
    static constexpr int NP = 1, RBA = 1, RBB = 1;
    static constexpr int radix(int) { return 1; }
};
template <>
struct RowPlan<64> {
    static constexpr bool ok = true;
    static constexpr int NP = 2, RBA = 32, RBB = 16;
    static constexpr int radix(int) { return 8; }
};
template <>
struct RowPlan<128> {
    static constexpr bool ok = true;
    static constexpr int NP = 3, RBA = 16, RBB = 8;
    static constexpr int radix(int p) { return p == 0 ? 8 : 4; }
};
template <>
struct RowPlan<256> {
    static constexpr bool ok = true;
    static constexpr int NP = 3, RBA = 8, RBB = 4;
    static constexpr int radix(int p) { return p < 2 ? 8 : 4; }
};
template <>
struct RowPlan<512> {
    static constexpr bool ok = true;
    static constexpr int NP = 3, RBA = 4, RBB = 2;
    static constexpr int radix(int) { return 8; }
};

template <int M, int RB_>
struct RowShape {
    using P = RowPlan<M>;
    static constexpr int RB = RB_, NP = P::NP, NT = RB_ * M / 8;
    static constexpr int RPITCH = M + M / 8 + 1;  // LDS row pitch (complex values)
    static constexpr int XCH = RB * RPITCH;       // exchange buffer (complex values)
};

// LDS slot of row element e: one pad value after every eight, so that the
// stride-R writes of a pass (lanes j, j + 1 write elements R j + r) spread
// over the banks
__device__ __forceinline__ int rw_slot(int e) { return e + (e >> 3); }

template <int M, int RB, int R>
__device__ __forceinline__ int rw_line(int t)
{
    return ((int)threadIdx.x + RowShape<M, RB>::NT * t) / (M / R);
}
template <int M, int RB, int R>
__device__ __forceinline__ int rw_but(int t)
{
    return ((int)threadIdx.x + RowShape<M, RB>::NT * t) % (M / R);
}

template <int M, int RB, int R, int NS, bool INV, class C>
__device__ __forceinline__ void rw_butterflies(C *v, const C *__restrict__ tw)
{
#pragma unroll
    for (int t = 0; t < 8 / R; ++t) {
        if constexpr (NS > 1) {
            const int jm = rw_but<M, RB, R>(t) & (NS - 1);
            constexpr int step = M / (NS * R);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const C w = tw[jm * r * step];
                v[t * R + r] = INV ? mulc(v[t * R + r], w) : mul(v[t * R + r], w);
            }
        }
        dft_small<R, C, INV>(v + t * R);
    }
}

template <int M, int RB, int R, int NS>
__device__ __forceinline__ int rw_out_elem(int t, int r)
{
    const int j = rw_but<M, RB, R>(t), jm = j & (NS - 1);
    return (j - jm) * R + jm + r * NS;
}

// passes P0.. in forward (FWD) or reversed radix order, input in v as pass
// P0 reads it; the final pass leaves its outputs in v
template <int M, int RB, bool FWD, bool INV, int P0, int NS, class C>
__device__ __forceinline__ void rw_run(C *v, C *X, const C *__restrict__ tw)
{
    using S = RowShape<M, RB>;
    constexpr int R = FWD ? S::P::radix(P0) : S::P::radix(S::NP - 1 - P0);
    rw_butterflies<M, RB, R, NS, INV>(v, tw);
    if constexpr (P0 + 1 < S::NP) {
        constexpr int R2 = FWD ? S::P::radix(P0 + 1) : S::P::radix(S::NP - 2 - P0);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 8 / R; ++t)
#pragma unroll
            for (int r = 0; r < R; ++r)
                X[rw_line<M, RB, R>(t) * S::RPITCH + rw_slot(rw_out_elem<M, RB, R, NS>(t, r))] = v[t * R + r];
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 8 / R2; ++t)
#pragma unroll
            for (int r = 0; r < R2; ++r)
                v[t * R2 + r] = X[rw_line<M, RB, R2>(t) * S::RPITCH + rw_slot(rw_but<M, RB, R2>(t) + r * (M / R2))];
        rw_run<M, RB, FWD, INV, P0 + 1, NS * R>(v, X, tw);
    }
}

// R2C rows with register passes: n3 = 2M real values per row
template <class R, int M, int RB>
__global__ __launch_bounds__(RB * M / 8) void k_r2c_reg(RealIn in, char *__restrict__ spec, long slot_bytes, int slot0,
                                                 long nrow, const typename CplxOf<R>::type *__restrict__ tw_m,
                                                 const typename CplxOf<R>::type *__restrict__ tw_n, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    using C = typename CplxOf<R>::type;
    using S = RowShape<M, RB>;
    constexpr int R0 = S::P::radix(0), RL = S::P::radix(S::NP - 1);
    extern __shared__ char lds_raw[];
    C *X = reinterpret_cast<C *>(lds_raw);
    const int f = blockIdx.y;
    // the kernel-argument array is indexed by f and never copied (a copy
    // indexed at run time would live in scratch memory)
    const float2 *__restrict__ src = reinterpret_cast<const float2 *>(mshift(in.p[f], mo_));
    const long row0 = (long)blockIdx.x * S::RB;
    C v[8];
#pragma unroll
    for (int t = 0; t < 8 / R0; ++t) {
        const long row = row0 + rw_line<M, RB, R0>(t);
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int e = rw_but<M, RB, R0>(t) + r * (M / R0);
            const float2 z = row < nrow ? src[row * M + e] : make_float2(0.f, 0.f);
            v[t * R0 + r] = mk<C>((R)z.x, (R)z.y);
        }
    }
    rw_run<M, RB, true, false, 0, 1>(v, X, tw_m);
    // Z to LDS (natural order), then the pairs (k, M - k) give the half spectrum
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8 / RL; ++t)
#pragma unroll
        for (int r = 0; r < RL; ++r)
            X[rw_line<M, RB, RL>(t) * S::RPITCH + rw_slot(rw_out_elem<M, RB, RL, M / RL>(t, r))] = v[t * RL + r];
    __syncthreads();
    C *outm = reinterpret_cast<C *>(spec + (long)(slot0 + f) * slot_bytes);
    C *outq = outm + nrow * M;
    for (int idx = threadIdx.x; idx < S::RB * (M + 1); idx += S::NT) {
        const int c = idx / (M + 1), k = idx - c * (M + 1);
        const long row = row0 + c;
        if (row >= nrow) continue;
        const C zk = X[c * S::RPITCH + rw_slot(k == M ? 0 : k)];
        const C zc = conj_(X[c * S::RPITCH + rw_slot(k == 0 ? 0 : M - k)]);
        const C E = scl(add(zk, zc), R(0.5));
        const C D = scl(sub(zk, zc), R(0.5));
        const C O = mk<C>(D.y, -D.x);  // D / i
        const C Xk = add(E, mul(tw_n[k], O));
        if (k < M)
            outm[row * M + k] = Xk;
        else
            outq[row] = Xk;
    }
}

// C2R rows with register passes (FP32), times scale
template <int M, int RB>
__global__ __launch_bounds__(RB * M / 8) void k_c2r_reg(const char *__restrict__ spec, long slot_bytes, int slot0,
                                                 RealOut out, long nrow, const float2 *__restrict__ tw_m,
                                                 const float2 *__restrict__ tw_n, float scale, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    using S = RowShape<M, RB>;
    constexpr int RA = S::P::radix(S::NP - 1), R1 = S::P::radix(0);  // first and last inverse radices
    extern __shared__ char lds_raw[];
    float2 *X = reinterpret_cast<float2 *>(lds_raw);
    const int f = blockIdx.y;
    const long row0 = (long)blockIdx.x * S::RB;
    const float2 *inm = reinterpret_cast<const float2 *>(spec + (long)(slot0 + f) * slot_bytes);
    const float2 *inq = inm + nrow * M;
    for (int idx = threadIdx.x; idx < S::RB * (M + 1); idx += S::NT) {
        const int c = idx / (M + 1), k = idx - c * (M + 1);
        const long row = row0 + c;
        float2 Xv = make_float2(0.f, 0.f);
        if (row < nrow) Xv = (k < M) ? inm[row * M + k] : inq[row];
        X[c * S::RPITCH + rw_slot(k)] = Xv;
    }
    __syncthreads();
    float2 v[8];
#pragma unroll
    for (int t = 0; t < 8 / RA; ++t) {
        const int c = rw_line<M, RB, RA>(t);
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            const int k = rw_but<M, RB, RA>(t) + r * (M / RA);
            const float2 Xk = X[c * S::RPITCH + rw_slot(k)];
            const float2 Xc = conj_(X[c * S::RPITCH + rw_slot(M - k)]);
            const float2 E = add(Xk, Xc);
            const float2 O = mulc(sub(Xk, Xc), tw_n[k]);  // * exp(+2 pi i k / n3)
            v[t * RA + r] = add(E, muli(O));
        }
    }
    rw_run<M, RB, false, true, 0, 1>(v, X, tw_m);
    float *__restrict__ dst = mshift(out.p[f], mo_);
#pragma unroll
    for (int t = 0; t < 8 / R1; ++t) {
        const long row = row0 + rw_line<M, RB, R1>(t);
        if (row >= nrow) continue;
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int e = rw_out_elem<M, RB, R1, M / R1>(t, r);
            const float2 z = v[t * R1 + r];
            *reinterpret_cast<float2 *>(dst + row * 2 * M + 2 * e) = make_float2(z.x * scale, z.y * scale);
        }
    }
}

// rw_run over NF row sets at once (v[f], exchange buffer X + f XCH): one
// pair of barriers per pass for all of them, and NF independent butterfly
// chains per thread; per set the arithmetic of rw_run
template <int M, int RB, bool FWD, bool INV, int P0, int NS, int NF, class C>
__device__ __forceinline__ void rw_run_n(C (*v)[8], C *X, const C *__restrict__ tw)
{
    using S = RowShape<M, RB>;
    constexpr int R = FWD ? S::P::radix(P0) : S::P::radix(S::NP - 1 - P0);
#pragma unroll
    for (int f = 0; f < NF; ++f) rw_butterflies<M, RB, R, NS, INV>(v[f], tw);
    if constexpr (P0 + 1 < S::NP) {
        constexpr int R2 = FWD ? S::P::radix(P0 + 1) : S::P::radix(S::NP - 2 - P0);
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int t = 0; t < 8 / R; ++t)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    X[f * S::XCH + rw_line<M, RB, R>(t) * S::RPITCH + rw_slot(rw_out_elem<M, RB, R, NS>(t, r))] =
                        v[f][t * R + r];
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int t = 0; t < 8 / R2; ++t)
#pragma unroll
                for (int r = 0; r < R2; ++r)
                    v[f][t * R2 + r] =
                        X[f * S::XCH + rw_line<M, RB, R2>(t) * S::RPITCH + rw_slot(rw_but<M, RB, R2>(t) + r * (M / R2))];
        rw_run_n<M, RB, FWD, INV, P0 + 1, NS * R, NF>(v, X, tw);
    }
}

// The rank-one part of H0 (eq. h0-pc) along x3 rows: the spectra of p in
// slots in0.. (three fields, after the inverse x1 and x2 passes) go back
// along x3 as in k_c2r_reg (times scale), t = G (G . p) is formed per point
// with G = grad m(1) (three physical fields, n3 = 2M floats per row), and t
// goes forward along x3 as in k_r2c_reg (FP32) into slots out0..; p and t
// never reach HBM.  The arithmetic of c2r, k_h0_rank1 and r2c in turn; the
// three fields go through their passes together (three exchange buffers of
// XCH values in LDS).
template <int M, int RB>
__global__ __launch_bounds__(RB * M / 8) void k_x3_rank1(char *__restrict__ spec, long slot_bytes, int in0, int out0,
                                                  const float *__restrict__ G, long nrow,
                                                  const float2 *__restrict__ tw_m, const float2 *__restrict__ tw_n,
                                                  float scale, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.z);
    if (mb.stopped(mo_)) return;
    spec = mshift(spec, mo_);
    G = mshift(G, mo_);
    using S = RowShape<M, RB>;
    constexpr int RA = S::P::radix(S::NP - 1), R1 = S::P::radix(0);  // first and last inverse radices
    constexpr int R0 = R1, RL = RA;                                   // first and last forward radices
    extern __shared__ char lds_raw[];
    float2 *X = reinterpret_cast<float2 *>(lds_raw);  // field f: X + f XCH
    const long row0 = (long)blockIdx.x * S::RB;
    const long n3 = 2L * M, N = nrow * n3;
    for (int idx = threadIdx.x; idx < S::RB * (M + 1); idx += S::NT) {
        const int c = idx / (M + 1), k = idx - c * (M + 1);
        const long row = row0 + c;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float2 *inm = reinterpret_cast<const float2 *>(spec + (long)(in0 + f) * slot_bytes);
            const float2 *inq = inm + nrow * M;
            float2 Xv = make_float2(0.f, 0.f);
            if (row < nrow) Xv = (k < M) ? inm[row * M + k] : inq[row];
            X[f * S::XCH + c * S::RPITCH + rw_slot(k)] = Xv;
        }
    }
    __syncthreads();
    float2 v[3][8];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const float2 *Xf = X + f * S::XCH;
#pragma unroll
        for (int t = 0; t < 8 / RA; ++t) {
            const int c = rw_line<M, RB, RA>(t);
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                const int k = rw_but<M, RB, RA>(t) + r * (M / RA);
                const float2 Xk = Xf[c * S::RPITCH + rw_slot(k)];
                const float2 Xc = conj_(Xf[c * S::RPITCH + rw_slot(M - k)]);
                const float2 E = add(Xk, Xc);
                const float2 O = mulc(sub(Xk, Xc), tw_n[k]);
                v[f][t * RA + r] = add(E, muli(O));
            }
        }
    }
    rw_run_n<M, RB, false, true, 0, 1, 3>(v, X, tw_m);
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int i = 0; i < 8; ++i) v[f][i] = make_float2(v[f][i].x * scale, v[f][i].y * scale);
    // t = G (G . p) at the points this thread holds (x3 = 2e, 2e + 1 of its rows)
#pragma unroll
    for (int t = 0; t < 8 / R1; ++t) {
        const long row = row0 + rw_line<M, RB, R1>(t);
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int i = t * R1 + r;
            if (row >= nrow) {
                v[0][i] = v[1][i] = v[2][i] = make_float2(0.f, 0.f);
                continue;
            }
            const long o = row * n3 + 2 * rw_out_elem<M, RB, R1, M / R1>(t, r);
            const float2 g0 = *reinterpret_cast<const float2 *>(G + o), g1 = *reinterpret_cast<const float2 *>(G + N + o),
                         g2 = *reinterpret_cast<const float2 *>(G + 2 * N + o);
            const float dx = g0.x * v[0][i].x + g1.x * v[1][i].x + g2.x * v[2][i].x;
            const float dy = g0.y * v[0][i].y + g1.y * v[1][i].y + g2.y * v[2][i].y;
            v[0][i] = make_float2(g0.x * dx, g0.y * dy);
            v[1][i] = make_float2(g1.x * dx, g1.y * dy);
            v[2][i] = make_float2(g2.x * dx, g2.y * dy);
        }
    }
    // t to LDS in natural order, then the forward pass's own distribution
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int t = 0; t < 8 / R1; ++t)
#pragma unroll
            for (int r = 0; r < R1; ++r)
                X[f * S::XCH + rw_line<M, RB, R1>(t) * S::RPITCH + rw_slot(rw_out_elem<M, RB, R1, M / R1>(t, r))] =
                    v[f][t * R1 + r];
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int t = 0; t < 8 / R0; ++t)
#pragma unroll
            for (int r = 0; r < R0; ++r)
                v[f][t * R0 + r] =
                    X[f * S::XCH + rw_line<M, RB, R0>(t) * S::RPITCH + rw_slot(rw_but<M, RB, R0>(t) + r * (M / R0))];
    rw_run_n<M, RB, true, false, 0, 1, 3>(v, X, tw_m);
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int t = 0; t < 8 / RL; ++t)
#pragma unroll
            for (int r = 0; r < RL; ++r)
                X[f * S::XCH + rw_line<M, RB, RL>(t) * S::RPITCH + rw_slot(rw_out_elem<M, RB, RL, M / RL>(t, r))] =
                    v[f][t * RL + r];
    __syncthreads();
    for (int idx = threadIdx.x; idx < S::RB * (M + 1); idx += S::NT) {
        const int c = idx / (M + 1), k = idx - c * (M + 1);
        const long row = row0 + c;
        if (row >= nrow) continue;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float2 *Xf = X + f * S::XCH;
            const float2 zk = Xf[c * S::RPITCH + rw_slot(k == M ? 0 : k)];
            const float2 zc = conj_(Xf[c * S::RPITCH + rw_slot(k == 0 ? 0 : M - k)]);
            const float2 E = scl(add(zk, zc), 0.5f);
            const float2 D = scl(sub(zk, zc), 0.5f);
            const float2 O = mk<float2>(D.y, -D.x);  // D / i
            const float2 Xk = add(E, mul(tw_n[k], O));
            float2 *outm = reinterpret_cast<float2 *>(spec + (long)(out0 + f) * slot_bytes);
            if (k < M)
                outm[row * M + k] = Xk;
            else
                outm[nrow * M + row] = Xk;
        }
    }
}

// ---------------------------------------------------------------------------
// x3 pass: real rows -> half spectrum (main + Nyquist plane), computed in R
// ---------------------------------------------------------------------------
template <class R, int LF>
__global__ __launch_bounds__(kFftThreads) void k_r2c_x3(RealIn in, char *__restrict__ spec,
                                                        long slot_bytes, int slot0, long nrow, int n3_rt,
                                                        int TWR, RadixPlan rp,
                                                        const typename CplxOf<R>::type *__restrict__ tw_m3,
                                                        const typename CplxOf<R>::type *__restrict__ tw_n3, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    using C = typename CplxOf<R>::type;
    extern __shared__ char lds_raw[];
    C *lds = reinterpret_cast<C *>(lds_raw);
    const int n3 = LF > 0 ? 2 * LF : n3_rt;
    const int m3 = n3 >> 1, LP = m3 + 1;
    C *A = lds, *B = lds + TWR * LP;
    const int f = blockIdx.y;
    const float *__restrict__ src = mshift(in.p[f], mo_);
    const long row0 = (long)blockIdx.x * TWR;
    const int tid = threadIdx.x, nthr = kFftThreads;
    R *Af = reinterpret_cast<R *>(A);
    for (int idx = tid; idx < TWR * n3; idx += nthr) {
        const int c = idx / n3, x = idx - c * n3;
        const long row = row0 + c;
        Af[(c * LP + (x >> 1)) * 2 + (x & 1)] = row < nrow ? (R)src[row * n3 + x] : R(0);
    }
    __syncthreads();
    const C *Z = lds_fft_any<false, false, LF>(A, B, TWR, 0, LP, rp, tw_m3, tid, nthr);
    C *outm = reinterpret_cast<C *>(spec + (long)(slot0 + f) * slot_bytes);
    C *outq = outm + nrow * m3;
    for (int idx = tid; idx < TWR * (m3 + 1); idx += nthr) {
        const int c = idx / (m3 + 1), k = idx - c * (m3 + 1);
        const long row = row0 + c;
        if (row >= nrow) continue;
        const C zk = Z[c * LP + (k == m3 ? 0 : k)];
        const C zc = conj_(Z[c * LP + (k == 0 ? 0 : m3 - k)]);
        const C E = scl(add(zk, zc), R(0.5));
        const C D = scl(sub(zk, zc), R(0.5));
        const C O = mk<C>(D.y, -D.x);  // D / i
        const C X = add(E, mul(tw_n3[k], O));
        if (k < m3)
            outm[row * m3 + k] = X;
        else
            outq[row] = X;
    }
}

// ---------------------------------------------------------------------------
// x3 pass: half spectrum (FP32) -> real rows, times scale
// ---------------------------------------------------------------------------
template <int LF>
__global__ __launch_bounds__(kFftThreads) void k_c2r_x3(const char *__restrict__ spec, long slot_bytes,
                                                        int slot0, RealOut out, long nrow, int n3_rt,
                                                        int TWR, RadixPlan rp,
                                                        const float2 *__restrict__ tw_m3,
                                                        const float2 *__restrict__ tw_n3, float scale, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    extern __shared__ char lds_raw[];
    float2 *lds = reinterpret_cast<float2 *>(lds_raw);
    const int n3 = LF > 0 ? 2 * LF : n3_rt;
    const int m3 = n3 >> 1, LP = m3 + 1;
    float2 *A = lds, *B = lds + TWR * LP;
    const int f = blockIdx.y;
    const long row0 = (long)blockIdx.x * TWR;
    const int tid = threadIdx.x, nthr = kFftThreads;
    const float2 *inm = reinterpret_cast<const float2 *>(spec + (long)(slot0 + f) * slot_bytes);
    const float2 *inq = inm + nrow * m3;
    for (int idx = tid; idx < TWR * (m3 + 1); idx += nthr) {
        const int c = idx / (m3 + 1), k = idx - c * (m3 + 1);
        const long row = row0 + c;
        float2 X = make_float2(0.f, 0.f);
        if (row < nrow) X = (k < m3) ? inm[row * m3 + k] : inq[row];
        B[c * LP + k] = X;
    }
    __syncthreads();
    for (int idx = tid; idx < TWR * m3; idx += nthr) {
        const int c = idx / m3, k = idx - c * m3;
        const float2 Xk = B[c * LP + k];
        const float2 Xc = conj_(B[c * LP + m3 - k]);
        const float2 E = add(Xk, Xc);
        const float2 O = mulc(sub(Xk, Xc), tw_n3[k]);  // * exp(+2 pi i k / n3)
        A[c * LP + k] = add(E, muli(O));
    }
    __syncthreads();
    const float2 *z = lds_fft_any<true, false, LF>(A, B, TWR, 0, LP, rp, tw_m3, tid, nthr);
    float *__restrict__ dst = mshift(out.p[f], mo_);
    for (int idx = tid; idx < TWR * m3; idx += nthr) {
        const int c = idx / m3, n = idx - c * m3;
        const long row = row0 + c;
        if (row >= nrow) continue;
        const float2 val = z[c * LP + n];
        *reinterpret_cast<float2 *>(dst + row * n3 + 2 * n) = make_float2(val.x * scale, val.y * scale);
    }
}

// ---------------------------------------------------------------------------
// Column pass (x2 or x1) over tiles of TW adjacent columns
// ---------------------------------------------------------------------------
struct ColDesc {
    long base_off;  // offset of the sub-array (main: 0, Nyquist plane: nrow*m3), in elements
    long ostride;   // stride between outer indices
    long nstride;   // stride along the transformed line
    long cstride;   // stride between columns
    int ncols;      // columns per outer index
};

// Position of a column-pass workgroup.  Workgroups go round-robin to the 8
// XCDs (linear id mod 8); renumbering the (x, y) plane of the grid gives each
// XCD a contiguous run of column tiles, so the narrow column segments of
// neighbouring tiles, which share 128-byte lines, meet in one L2.
struct TilePos {
    int x, y;
};

__device__ __forceinline__ TilePos tile_pos()
{
    const int gx = (int)gridDim.x, tot = gx * (int)gridDim.y;
    int lin = (int)blockIdx.x + gx * (int)blockIdx.y;
    const int per = tot >> 3;
    if (lin < per * 8) lin = (lin & 7) * per + (lin >> 3);
    return TilePos{lin % gx, lin / gx};
}

template <class C>
__device__ __forceinline__ void tile_load(C *dst, const C *__restrict__ src, const ColDesc &d, int L,
                                          int TW, int logTW, int col0, int tid, int nthr)
{
    for (int idx = tid; idx < L * TW; idx += nthr) {
        const int n = idx >> logTW, c = idx & (TW - 1);
        const int col = col0 + c;
        dst[idx] = col < d.ncols ? src[n * d.nstride + col * d.cstride] : mk<C>(0, 0);
    }
}

template <class C>
__device__ __forceinline__ void tile_store(C *__restrict__ dst, const C *src, const ColDesc &d, int L,
                                           int TW, int logTW, int col0, int tid, int nthr)
{
    for (int idx = tid; idx < L * TW; idx += nthr) {
        const int n = idx >> logTW, c = idx & (TW - 1);
        const int col = col0 + c;
        if (col < d.ncols) dst[n * d.nstride + col * d.cstride] = src[idx];
    }
}

template <bool INV, class R, int LF>
__global__ __launch_bounds__(kFftThreads) void k_fft_cols(char *__restrict__ spec, long slot_bytes,
                                                          int slot0, ColDesc d, int TW, int logTW,
                                                          RadixPlan rp,
                                                          const typename CplxOf<R>::type *__restrict__ tw, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    using C = typename CplxOf<R>::type;
    extern __shared__ char lds_raw[];
    C *lds = reinterpret_cast<C *>(lds_raw);
    const int L = LF > 0 ? LF : rp.L;
    C *A = lds, *B = lds + L * TW;
    const int tid = threadIdx.x, nthr = kFftThreads;
    const TilePos tp = tile_pos();
    C *base = reinterpret_cast<C *>(spec + (long)(slot0 + bz_) * slot_bytes) + d.base_off +
              (long)tp.y * d.ostride;
    const int col0 = tp.x * TW;
    tile_load(A, base, d, L, TW, logTW, col0, tid, nthr);
    __syncthreads();
    const C *res = lds_fft_any<INV, true, LF>(A, B, TW, logTW, 0, rp, tw, tid, nthr);
    tile_store(base, res, d, L, TW, logTW, col0, tid, nthr);
}

// ---------------------------------------------------------------------------
// Register Stockham passes for the fused x1 operators: eight values per
// thread, radix <= 8.  A task (c, j) is butterfly j of column c; pass p
// (radix R, Ns = product of the earlier radices) reads elements j + r L/R,
// multiplies by W_{Ns R}^((j mod Ns) r), takes the DFT_R and writes elements
// (j - j mod Ns) R + j mod Ns + r Ns; the first pass reads the tile from
// global memory, the passes exchange through LDS.  After the last forward
// pass a thread holds X[j + r L/R_P], which is exactly the input of the
// first pass of the inverse run with the radices in reverse order, so a
// pointwise symbol is applied in registers between the two.
// ---------------------------------------------------------------------------
// TWA and TWB: the two column-tile widths (threads = TW L / 8) the
// autotuner chooses between
template <int L>
struct StPlan {
    static constexpr bool ok = false;
    static constexpr int NP = 1, TWA = 1, TWB = 1;
    static constexpr int radix(int) { return 1; }
};
template <>
struct StPlan<64> {
    static constexpr bool ok = true;
    static constexpr int NP = 2, TWA = 32, TWB = 16;
    static constexpr int radix(int) { return 8; }
};
template <>
struct StPlan<128> {
    static constexpr bool ok = true;
    static constexpr int NP = 3, TWA = 16, TWB = 8;
    static constexpr int radix(int p) { return p == 0 ? 8 : 4; }
};
template <>
struct StPlan<256> {
    static constexpr bool ok = true;
    static constexpr int NP = 3, TWA = 16, TWB = 8;
    static constexpr int radix(int p) { return p < 2 ? 8 : 4; }
};
template <>
struct StPlan<512> {
    static constexpr bool ok = true;
    static constexpr int NP = 3, TWA = 8, TWB = 4;
    static constexpr int radix(int) { return 8; }
};

template <int L, int TW_>
struct StShape {
    using P = StPlan<L>;
    static constexpr int TW = TW_, NT = TW_ * L / 8, NP = P::NP;
    static constexpr int RL = P::radix(NP - 1);  // radix of the last forward pass
    static constexpr int NTL = 8 / RL;           // butterflies a thread holds after it
    static constexpr int PITCH = TW + 1;         // LDS row pitch (complex values)
    static constexpr int XCH = L * PITCH;        // exchange buffer (complex values)
    static_assert(NT * 8 == TW * L, "eight values per thread");
};

// one pass over registers v (8 values: task t, element r at v[t R + r])
template <int L, int TW, int R, int NS, bool INV, class C>
__device__ __forceinline__ void st_butterflies(C *v, const C *__restrict__ tw)
{
    using S = StShape<L, TW>;
#pragma unroll
    for (int t = 0; t < 8 / R; ++t) {
        const int j = ((int)threadIdx.x + S::NT * t) / S::TW;
        if constexpr (NS > 1) {
            const int jm = j & (NS - 1);
            constexpr int step = L / (NS * R);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const C w = tw[jm * r * step];
                v[t * R + r] = INV ? mulc(v[t * R + r], w) : mul(v[t * R + r], w);
            }
        }
        dft_small<R, C, INV>(v + t * R);
    }
}

// element rows written by a pass (Ns = NS, radix R) for task t, value r
template <int L, int TW, int R, int NS>
__device__ __forceinline__ int st_out_row(int t, int r)
{
    using S = StShape<L, TW>;
    const int j = ((int)threadIdx.x + S::NT * t) / S::TW, jm = j & (NS - 1);
    return (j - jm) * R + jm + r * NS;
}

template <int L, int TW, int R>
__device__ __forceinline__ int st_in_row(int t, int r)
{
    using S = StShape<L, TW>;
    return ((int)threadIdx.x + S::NT * t) / S::TW + r * (L / R);
}

__device__ __forceinline__ int st_col(int t, int NT, int TW) { return ((int)threadIdx.x + NT * t) % TW; }

// passes P0.. of a transform whose input already sits in v (as pass P0
// reads it); the radices are taken in forward order (FWD) or reversed;
// intermediate results go through X; the final pass leaves its outputs in v
template <int L, int TW, bool FWD, bool INV, int P0, int NS, class C>
__device__ __forceinline__ void st_run(C *v, C *X, const C *__restrict__ tw)
{
    using S = StShape<L, TW>;
    constexpr int R = FWD ? S::P::radix(P0) : S::P::radix(S::NP - 1 - P0);
    st_butterflies<L, TW, R, NS, INV>(v, tw);
    if constexpr (P0 + 1 < S::NP) {
        constexpr int R2 = FWD ? S::P::radix(P0 + 1) : S::P::radix(S::NP - 2 - P0);
        __syncthreads();  // X free
#pragma unroll
        for (int t = 0; t < 8 / R; ++t)
#pragma unroll
            for (int r = 0; r < R; ++r)
                X[st_out_row<L, TW, R, NS>(t, r) * S::PITCH + st_col(t, S::NT, S::TW)] = v[t * R + r];
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 8 / R2; ++t)
#pragma unroll
            for (int r = 0; r < R2; ++r)
                v[t * R2 + r] = X[st_in_row<L, TW, R2>(t, r) * S::PITCH + st_col(t, S::NT, S::TW)];
        st_run<L, TW, FWD, INV, P0 + 1, NS * R>(v, X, tw);
    }
}

// forward transform: load(n, c) -> v holds X[j + r L/R_P] (task t at v[t R_P + r])
template <int L, int TW, class C, class LoadF>
__device__ __forceinline__ void st_fwd(LoadF &&load, C *v, C *X, const C *__restrict__ tw)
{
    using S = StShape<L, TW>;
    constexpr int R = S::P::radix(0);
#pragma unroll
    for (int t = 0; t < 8 / R; ++t)
#pragma unroll
        for (int r = 0; r < R; ++r) v[t * R + r] = load(st_in_row<L, TW, R>(t, r), st_col(t, S::NT, S::TW));
    st_run<L, TW, true, false, 0, 1>(v, X, tw);
}

// spectral index (x1 wavenumber index) of held value i after st_fwd
template <int L, int TW>
__device__ __forceinline__ int st_held_index(int i)
{
    using S = StShape<L, TW>;
    return st_in_row<L, TW, S::RL>(i / S::RL, i % S::RL);
}
template <int L, int TW>
__device__ __forceinline__ int st_held_col(int i)
{
    using S = StShape<L, TW>;
    return st_col(i / S::RL, S::NT, S::TW);
}

// inverse transform from the layout st_fwd leaves (v is overwritten):
// store(n, c, value) for every element of the tile
template <int L, int TW, class C, class StoreF>
__device__ __forceinline__ void st_inv(C *v, C *X, StoreF &&store, const C *__restrict__ tw)
{
    using S = StShape<L, TW>;
    st_run<L, TW, false, true, 0, 1>(v, X, tw);
    constexpr int R = S::P::radix(0);  // the inverse ends with the first forward radix
    constexpr int NS = L / R;
#pragma unroll
    for (int t = 0; t < 8 / R; ++t)
#pragma unroll
        for (int r = 0; r < R; ++r) store(st_out_row<L, TW, R, NS>(t, r), st_col(t, S::NT, S::TW), v[t * R + r]);
}

// ---------------------------------------------------------------------------
// Spectral symbols.  (l1, l2, l3) index a spectral point, l3 in [0, n3/2].
// ---------------------------------------------------------------------------
struct SymCtx {
    int n1, n2, n3;
    double scale, beta;  // scale = 1/N folds the inverse normalisation in
    int reg, leray;
};

__device__ __forceinline__ double wn_full(int l, int n) { return (double)(l <= (n >> 1) ? l : l - n); }
__device__ __forceinline__ double wn_odd(int l, int n)
{
    return (2 * l == n) ? 0.0 : (double)(l <= (n >> 1) ? l : l - n);
}
__device__ __forceinline__ double reg_symbol(const SymCtx &s, int l1, int l2, int l3)
{
    const double k1 = wn_full(l1, s.n1), k2 = wn_full(l2, s.n2), k3 = wn_full(l3, s.n3);
    const double kk = k1 * k1 + k2 * k2 + k3 * k3;
    return s.reg == 2 ? kk * kk : kk;
}

// (beta A)^{-1} symbol, as the InvA operator forms it (1/beta where A vanishes)
__device__ __forceinline__ float invreg_factor(const SymCtx &sc, int l1, int l2, int l3)
{
    const double a = reg_symbol(sc, l1, l2, l3);
    return (float)((a == 0.0) ? 1.0 / sc.beta : 1.0 / (sc.beta * a));
}

// ---------------------------------------------------------------------------
// Column pass with register line FFTs (lengths with a RegPlan)
// ---------------------------------------------------------------------------
// deterministic sums of two values over a 256-thread workgroup (fixed tree);
// the totals land in thread 0
__device__ __forceinline__ void block_sum2(double &a, double &b)
{
    __shared__ double sa[256], sb[256];
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    a = sa[0];
    b = sb[0];
}

// The search-direction update of the spectral PCG fused into the inverse x1
// pass that starts p's way back to physical space: while a column is
// loaded, p = z + beta p (z = M^{-1} r, or the given z; beta from the device
// scalars d, p kept once the PCG has stopped) is formed and written back to
// the vector; the pass then transforms it into the slots.
struct PUpd {
    const float2 *r, *z;  // z NULL: z = M^{-1} r with the symbol of sc
    float2 *p;
    long S;               // float2 per field of the vectors
    const double *d;
    SymCtx sc;
    float2 *s = nullptr;  // unless NULL: s += alpha p with p as loaded (before its update)
};

// The H0 assembly fused into the forward x1 pass that completes the
// transform of t = G (G . p): each output coefficient becomes
// q = t^ + beta0 A p (p: the vector's spectrum) and is written to the vector
// q instead of the slot, with the partial sums of <p, q> per workgroup and
// field (partial[field * gridDim.x + workgroup]).
struct QAsm {
    const float2 *p;
    float2 *q;
    long S;
    double *partial;
    SymCtx sc;
};

// Both parts of the spectrum in one launch: the tiles of the main array
// (gx0 x outer0, descriptor d0) and then those of the Nyquist plane (gx1,
// descriptor d1) along a one-dimensional grid, in the XCD order of tile_pos.
// PUPD (inverse FP32 x1 passes only): the loaded values are p = z + beta p;
// ASM (forward FP32 x1 passes only): the outputs are assembled into q.
template <bool INV, class R, int L, bool PUPD, bool ASM = false>
__global__ __launch_bounds__(256) void k_cols_reg(char *__restrict__ spec, long slot_bytes, int slot0, ColDesc d0,
                                                  ColDesc d1, int gx0, int outer0,
                                                  const typename CplxOf<R>::type *__restrict__ tw, PUpd pu, QAsm qa,
                                                  Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) {
        // after a stop only the stopping iteration's s update (alpha != 0) is left
        if constexpr (!PUPD) return;
        else if (!pu.s || mshift(pu.d, mo_)[S_ALPHA] == 0.0) return;
    }
    using C = typename CplxOf<R>::type;
    using S = RegShape<L>;
    extern __shared__ char lds_raw[];
    C *X = reinterpret_cast<C *>(lds_raw);
    const TilePos lp = tile_pos();  // gridDim.y = 1: lp.x is the linear tile index
    const int t0 = gx0 * outer0;
    const bool nyq = lp.x >= t0;
    const ColDesc &d = nyq ? d1 : d0;
    const TilePos tp = nyq ? TilePos{lp.x - t0, 0} : TilePos{lp.x % gx0, lp.x / gx0};
    C *base = reinterpret_cast<C *>(spec + (long)(slot0 + bz_) * slot_bytes) + d.base_off +
              (long)tp.y * d.ostride;
    const int col0 = tp.x * S::TW;
    C out[S::T2][S::R2];
    if constexpr (PUPD) {
        static_assert(INV && std::is_same<R, float>::value, "the update precedes an inverse FP32 pass");
        const long fo = (long)bz_ * pu.S + d.base_off + (long)tp.y * d.ostride;
        const float2 *rr = mshift(pu.r, mo_) + fo, *zz = mshift(pu.z, mo_);
        float2 *pp = mshift(pu.p, mo_) + fo;
        const double *dd = mshift(pu.d, mo_);
        if (zz) zz += fo;
        float2 *ss = mshift(pu.s, mo_);
        if (ss) ss += fo;
        const bool upd = dd[S_DONE] == 0.0;
        const float be = (float)dd[S_BETA], al = (float)dd[S_ALPHA];
        reg_fft<L, INV>(
            [&](int n, int c) {
                const int col = col0 + c;
                if (col >= d.ncols) return mk<C>(0, 0);
                const long e = n * d.nstride + col * d.cstride;
                float2 v = pp[e];
                if (ss && al != 0.f) {
                    const float2 sv = ss[e];
                    ss[e] = make_float2(__builtin_fmaf(al, v.x, sv.x), __builtin_fmaf(al, v.y, sv.y));
                }
                if (upd) {
                    float2 zv;
                    if (zz) {
                        zv = zz[e];
                    } else {
                        // x1 pass: the line index is k1; the Nyquist plane's columns are k2
                        const int l2 = nyq ? col : tp.y, l3 = nyq ? (pu.sc.n3 >> 1) : col;
                        const float m = invreg_factor(pu.sc, n, l2, l3);
                        const float2 rv = rr[e];
                        zv = make_float2(m * rv.x, m * rv.y);
                    }
                    v = make_float2(__builtin_fmaf(be, v.x, zv.x), __builtin_fmaf(be, v.y, zv.y));
                    pp[e] = v;
                }
                return v;
            },
            X, out, tw);
    } else {
        reg_fft<L, INV>(
            [&](int n, int c) {
                const int col = col0 + c;
                return col < d.ncols ? base[n * d.nstride + col * d.cstride] : mk<C>(0, 0);
            },
            X, out, tw);
    }
    if constexpr (ASM) {
        static_assert(!INV && std::is_same<R, float>::value, "the assembly follows a forward FP32 pass");
        const long fo = (long)bz_ * qa.S + d.base_off + (long)tp.y * d.ostride;
        const float2 *pp = mshift(qa.p, mo_) + fo;
        float2 *qq = mshift(qa.q, mo_) + fo;
        double acc = 0.0, unused = 0.0;
#pragma unroll
        for (int u = 0; u < S::T2; ++u) {
            const int task = (int)threadIdx.x + 256 * u, c = task % S::TW, k1 = task / S::TW;
            const int col = col0 + c;
            if (col < d.ncols) {
                const int l2 = nyq ? col : tp.y, l3 = nyq ? (qa.sc.n3 >> 1) : col;
                const double w = (nyq || col == 0) ? 1.0 : 2.0;  // Hermitian weight (l3 = 0 or n3/2: 1)
#pragma unroll
                for (int k2 = 0; k2 < S::R2; ++k2) {
                    const int n = k1 + S::R1 * k2;
                    const long e = n * d.nstride + col * d.cstride;
                    const double ba = qa.sc.beta * reg_symbol(qa.sc, n, l2, l3);
                    const float2 pv = pp[e], o = out[u][k2];
                    const float2 v = make_float2(o.x + (float)(pv.x * ba), o.y + (float)(pv.y * ba));
                    qq[e] = v;
                    acc += w * ((double)pv.x * v.x + (double)pv.y * v.y);
                }
            }
        }
        block_sum2(acc, unused);
        if (threadIdx.x == 0) mshift(qa.partial, mo_)[(long)bz_ * gridDim.x + blockIdx.x] = acc;
    } else {
#pragma unroll
        for (int u = 0; u < S::T2; ++u) {
            const int task = (int)threadIdx.x + 256 * u, c = task % S::TW, k1 = task / S::TW;
            const int col = col0 + c;
            if (col < d.ncols)
#pragma unroll
                for (int k2 = 0; k2 < S::R2; ++k2) base[(k1 + S::R1 * k2) * d.nstride + col * d.cstride] = out[u][k2];
        }
    }
}

struct ColCtx {  // how a tile position maps to (l2, l3)
    int nyq;     // 0: main array (columns are k3, the outer index is k2); 1: Nyquist plane
    int outer;   // outer index of the tile
    __device__ __forceinline__ void l23(const SymCtx &s, int col, int &l2, int &l3) const
    {
        l2 = nyq ? col : outer;
        l3 = nyq ? (s.n3 >> 1) : col;
    }
};

// per-field real symbol, forward and inverse in R
enum { SYM_REG = 0, SYM_INVREG = 1, SYM_IDENT = 2 };

template <class R, int SYM, int LF>
__global__ __launch_bounds__(kFftThreads) void k_x1_scalar(char *__restrict__ spec, long slot_bytes,
                                                           int in0, int out0, ColDesc d, int nyq,
                                                           int TW, int logTW, RadixPlan rp,
                                                           const typename CplxOf<R>::type *__restrict__ tw,
                                                           SymCtx sc, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    using C = typename CplxOf<R>::type;
    extern __shared__ char lds_raw[];
    C *lds = reinterpret_cast<C *>(lds_raw);
    const int L = LF > 0 ? LF : rp.L, tile = L * TW;
    C *A = lds, *B = lds + tile;
    const TilePos tp = tile_pos();
    const int tid = threadIdx.x, nthr = kFftThreads, col0 = tp.x * TW;
    const long off = d.base_off + (long)tp.y * d.ostride;
    const C *src = reinterpret_cast<const C *>(spec + (long)(in0 + bz_) * slot_bytes) + off;
    float2 *dst = reinterpret_cast<float2 *>(spec + (long)(out0 + bz_) * slot_bytes) + off;
    tile_load(load_target(rp, A, B), src, d, L, TW, logTW, col0, tid, nthr);
    __syncthreads();
    lds_fft_any<false, true, LF>(load_target(rp, A, B), load_target(rp, B, A), TW, logTW, 0, rp, tw, tid, nthr);
    const ColCtx cc{nyq, tp.y};
    for (int idx = tid; idx < tile; idx += nthr) {
        const int n = idx >> logTW, c = idx & (TW - 1);
        int l2, l3;
        cc.l23(sc, col0 + c, l2, l3);
        double f = sc.scale;
        if (SYM == SYM_REG) {
            f *= reg_symbol(sc, n, l2, l3);
        } else if (SYM == SYM_INVREG) {
            const double a = reg_symbol(sc, n, l2, l3);
            f *= (a == 0.0) ? 1.0 / sc.beta : 1.0 / (sc.beta * a);
        }
        A[idx] = scl(A[idx], (R)f);
    }
    __syncthreads();
    const C *res = lds_fft_any<true, true, LF>(A, B, TW, logTW, 0, rp, tw, tid, nthr);
    for (int idx = tid; idx < tile; idx += nthr) {
        const int n = idx >> logTW, c = idx & (TW - 1);
        const int col = col0 + c;
        if (col < d.ncols) dst[n * d.nstride + col * d.cstride] = to_f2(res[idx]);
    }
}

// grad: one FP64 input field -> three FP32 output fields
template <int LF>
__global__ __launch_bounds__(kFftThreads) void k_x1_grad(char *__restrict__ spec, long slot_bytes, int in0,
                                                         int out0, ColDesc d, int nyq, int TW, int logTW,
                                                         RadixPlan rp, const double2 *__restrict__ twd,
                                                         const float2 *__restrict__ twf, SymCtx sc, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    extern __shared__ char lds_raw[];
    const int L = LF > 0 ? LF : rp.L, tile = L * TW;
    double2 *WA = reinterpret_cast<double2 *>(lds_raw), *WB = WA + tile;
    float2 *O = reinterpret_cast<float2 *>(WB + tile);  // three float2 tiles
    float2 *S = reinterpret_cast<float2 *>(WA);         // float scratch once WA/WB are free
    const TilePos tp = tile_pos();
    const int tid = threadIdx.x, nthr = kFftThreads, col0 = tp.x * TW;
    const long off = d.base_off + (long)tp.y * d.ostride;
    const double2 *src = reinterpret_cast<const double2 *>(spec + (long)(in0 + bz_) * slot_bytes) + off;
    tile_load(load_target(rp, WA, WB), src, d, L, TW, logTW, col0, tid, nthr);
    __syncthreads();
    lds_fft_any<false, true, LF>(load_target(rp, WA, WB), load_target(rp, WB, WA), TW, logTW, 0, rp, twd, tid, nthr);
    const ColCtx cc{nyq, tp.y};
    for (int idx = tid; idx < tile; idx += nthr) {
        const int n = idx >> logTW, c = idx & (TW - 1);
        int l2, l3;
        cc.l23(sc, col0 + c, l2, l3);
        const double k[3] = {wn_odd(n, sc.n1), wn_odd(l2, sc.n2), wn_odd(l3, sc.n3)};
        const double2 f = scl(WA[idx], sc.scale);
#pragma unroll
        for (int q = 0; q < 3; ++q) O[q * tile + idx] = to_f2(muli(scl(f, k[q])));
    }
    __syncthreads();
    for (int q = 0; q < 3; ++q) {
        const float2 *res = lds_fft_any<true, true, LF>(O + q * tile, S, TW, logTW, 0, rp, twf, tid, nthr);
        float2 *dst = reinterpret_cast<float2 *>(spec + (long)(out0 + 3 * bz_ + q) * slot_bytes) + off;
        tile_store(dst, res, d, L, TW, logTW, col0, tid, nthr);
        __syncthreads();
    }
}

// div: three FP64 input fields -> one FP32 output field (FP64 accumulation)
template <int LF>
__global__ __launch_bounds__(kFftThreads) void k_x1_div(char *__restrict__ spec, long slot_bytes, int in0,
                                                        int out0, ColDesc d, int nyq, int TW, int logTW,
                                                        RadixPlan rp, const double2 *__restrict__ twd,
                                                        const float2 *__restrict__ twf, SymCtx sc, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    extern __shared__ char lds_raw[];
    const int L = LF > 0 ? LF : rp.L, tile = L * TW;
    double2 *WA = reinterpret_cast<double2 *>(lds_raw), *WB = WA + tile, *ACC = WB + tile;
    const TilePos tp = tile_pos();
    const int tid = threadIdx.x, nthr = kFftThreads, col0 = tp.x * TW;
    const long off = d.base_off + (long)tp.y * d.ostride;
    const ColCtx cc{nyq, tp.y};
    for (int q = 0; q < 3; ++q) {
        const double2 *src = reinterpret_cast<const double2 *>(spec + (long)(in0 + 3 * bz_ + q) * slot_bytes) + off;
        tile_load(load_target(rp, WA, WB), src, d, L, TW, logTW, col0, tid, nthr);
        __syncthreads();
        lds_fft_any<false, true, LF>(load_target(rp, WA, WB), load_target(rp, WB, WA), TW, logTW, 0, rp, twd, tid, nthr);
        for (int idx = tid; idx < tile; idx += nthr) {
            const int n = idx >> logTW, c = idx & (TW - 1);
            int l2, l3;
            cc.l23(sc, col0 + c, l2, l3);
            const double kq = q == 0 ? wn_odd(n, sc.n1) : (q == 1 ? wn_odd(l2, sc.n2) : wn_odd(l3, sc.n3));
            const double2 t = muli(scl(WA[idx], kq * sc.scale));
            ACC[idx] = q == 0 ? t : add(ACC[idx], t);
        }
        __syncthreads();
    }
    float2 *FA = reinterpret_cast<float2 *>(WA), *FB = FA + tile;
    for (int idx = tid; idx < tile; idx += nthr) FA[idx] = to_f2(ACC[idx]);
    __syncthreads();
    const float2 *res = lds_fft_any<true, true, LF>(FA, FB, TW, logTW, 0, rp, twf, tid, nthr);
    float2 *dst = reinterpret_cast<float2 *>(spec + (long)(out0 + bz_) * slot_bytes) + off;
    tile_store(dst, res, d, L, TW, logTW, col0, tid, nthr);
}

__device__ __forceinline__ void leray_coef(const SymCtx &sc, int n, int l2, int l3, double k[3], double &ikk)
{
    k[0] = wn_odd(n, sc.n1);
    k[1] = wn_odd(l2, sc.n2);
    k[2] = wn_odd(l3, sc.n3);
    const double kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    ikk = kk > 0.0 ? 1.0 / kk : 0.0;
}

// 1 / |k~|^2 in FP32 (0 where k~ = 0); |k~|^2 is an exact integer
__device__ __forceinline__ float leray_ikk(const SymCtx &sc, int n, int l2, int l3)
{
    const float k1 = (float)wn_odd(n, sc.n1), k2 = (float)wn_odd(l2, sc.n2), k3 = (float)wn_odd(l3, sc.n3);
    const float kk = k1 * k1 + k2 * k2 + k3 * k3;
    return kk > 0.f ? 1.f / kk : 0.f;
}

// Leray projection: three FP32 fields in and out
template <int LF>
__global__ __launch_bounds__(kFftThreads) void k_x1_leray(char *__restrict__ spec, long slot_bytes, int in0,
                                                          int out0, ColDesc d, int nyq, int TW, int logTW,
                                                          RadixPlan rp, const float2 *__restrict__ twf,
                                                          SymCtx sc, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    extern __shared__ char lds_raw[];
    const int L = LF > 0 ? LF : rp.L, tile = L * TW;
    float2 *T = reinterpret_cast<float2 *>(lds_raw);  // three field tiles, then scratch
    float2 *S = T + 3 * tile;
    const TilePos tp = tile_pos();
    const int tid = threadIdx.x, nthr = kFftThreads, col0 = tp.x * TW;
    const long off = d.base_off + (long)tp.y * d.ostride;
    for (int q = 0; q < 3; ++q) {
        const float2 *src = reinterpret_cast<const float2 *>(spec + (long)(in0 + 3 * bz_ + q) * slot_bytes) + off;
        float2 *home = T + q * tile;
        tile_load(load_target(rp, home, S), src, d, L, TW, logTW, col0, tid, nthr);
        __syncthreads();
        lds_fft_any<false, true, LF>(load_target(rp, home, S), load_target(rp, S, home), TW, logTW, 0, rp, twf, tid, nthr);
    }
    const ColCtx cc{nyq, tp.y};
    for (int idx = tid; idx < tile; idx += nthr) {
        const int n = idx >> logTW, c = idx & (TW - 1);
        int l2, l3;
        cc.l23(sc, col0 + c, l2, l3);
        double k[3], ikk;
        leray_coef(sc, n, l2, l3, k, ikk);
        float2 w[3] = {T[idx], T[tile + idx], T[2 * tile + idx]};
        const double sx = (k[0] * w[0].x + k[1] * w[1].x + k[2] * w[2].x) * ikk;
        const double sy = (k[0] * w[0].y + k[1] * w[1].y + k[2] * w[2].y) * ikk;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            T[q * tile + idx] = make_float2((float)((w[q].x - k[q] * sx) * sc.scale),
                                            (float)((w[q].y - k[q] * sy) * sc.scale));
    }
    __syncthreads();
    for (int q = 0; q < 3; ++q) {
        const float2 *res = lds_fft_any<true, true, LF>(T + q * tile, S, TW, logTW, 0, rp, twf, tid, nthr);
        float2 *dst = reinterpret_cast<float2 *>(spec + (long)(out0 + 3 * bz_ + q) * slot_bytes) + off;
        tile_store(dst, res, d, L, TW, logTW, col0, tid, nthr);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Fused x1 operators with register line FFTs: forward x1 transform of the
// input fields, the symbol applied to the spectra each thread holds, inverse
// x1 transform of the outputs; the same arithmetic, in the same order and
// precision, as the LDS kernels above.  blockIdx.z is the batch index.
// ---------------------------------------------------------------------------
// Both parts of the spectrum in one launch, as in k_cols_reg: the main
// array's tiles (gx0 x outer0, d0), then the Nyquist plane's (d1).
template <int OP, int L, int TW>
__global__ __launch_bounds__(TW * L / 8) void k_x1_reg(char *__restrict__ spec, long slot_bytes, int in0,
                                                         int out0, ColDesc d0, ColDesc d1, int gx0, int outer0,
                                                         const double2 *__restrict__ twd,
                                                         const float2 *__restrict__ twf, SymCtx sc, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    using S = StShape<L, TW>;
    extern __shared__ char lds_raw[];
    double2 *XD = reinterpret_cast<double2 *>(lds_raw);
    float2 *XF = reinterpret_cast<float2 *>(lds_raw);
    const TilePos lp = tile_pos();  // gridDim.y = 1: lp.x is the linear tile index
    const int t0 = gx0 * outer0, nyq = lp.x >= t0 ? 1 : 0;
    const ColDesc &d = nyq ? d1 : d0;
    const TilePos tp = nyq ? TilePos{lp.x - t0, 0} : TilePos{lp.x % gx0, lp.x / gx0};
    const int col0 = tp.x * TW, z = (int)bz_;
    const long off = d.base_off + (long)tp.y * d.ostride;
    const ColCtx cc{nyq, tp.y};
    auto load_d = [&](int slot) {
        const double2 *src = reinterpret_cast<const double2 *>(spec + (long)slot * slot_bytes) + off;
        return [=](int n, int c) {
            const int col = col0 + c;
            return col < d.ncols ? src[n * d.nstride + col * d.cstride] : mk<double2>(0, 0);
        };
    };
    auto load_f = [&](int slot) {
        const float2 *src = reinterpret_cast<const float2 *>(spec + (long)slot * slot_bytes) + off;
        return [=](int n, int c) {
            const int col = col0 + c;
            return col < d.ncols ? src[n * d.nstride + col * d.cstride] : mk<float2>(0, 0);
        };
    };
    auto store = [&](int slot) {
        float2 *dst = reinterpret_cast<float2 *>(spec + (long)slot * slot_bytes) + off;
        return [=](int n, int c, auto v) {
            const int col = col0 + c;
            if (col < d.ncols) dst[n * d.nstride + col * d.cstride] = to_f2(v);
        };
    };
    // spectral position of held value i: x1 index n(i), columns give (l2, l3)
    auto pos = [&](int i, int &n, int &l2, int &l3) {
        n = st_held_index<L, TW>(i);
        cc.l23(sc, col0 + st_held_col<L, TW>(i), l2, l3);
    };
    if constexpr (OP == SOP_GRAD) {  // one FP64 field -> three FP32 fields
        double2 f[8];
        st_fwd<L, TW>(load_d(in0 + z), f, XD, twd);
#pragma unroll 1
        for (int q = 0; q < 3; ++q) {
            float2 o[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                int n, l2, l3;
                pos(i, n, l2, l3);
                const double kq = q == 0 ? wn_odd(n, sc.n1) : (q == 1 ? wn_odd(l2, sc.n2) : wn_odd(l3, sc.n3));
                o[i] = to_f2(muli(scl(scl(f[i], sc.scale), kq)));
            }
            __syncthreads();  // the exchange buffer is reused
            st_inv<L, TW>(o, XF, store(out0 + 3 * z + q), twf);
        }
    } else if constexpr (OP == SOP_DIV) {  // three FP64 fields -> one FP32 field
        double2 acc[8];
#pragma unroll 1
        for (int q = 0; q < 3; ++q) {
            double2 f[8];
            if (q > 0) __syncthreads();
            st_fwd<L, TW>(load_d(in0 + 3 * z + q), f, XD, twd);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                int n, l2, l3;
                pos(i, n, l2, l3);
                const double kq = q == 0 ? wn_odd(n, sc.n1) : (q == 1 ? wn_odd(l2, sc.n2) : wn_odd(l3, sc.n3));
                const double2 t = muli(scl(f[i], kq * sc.scale));
                acc[i] = q == 0 ? t : add(acc[i], t);
            }
        }
        float2 o[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = to_f2(acc[i]);
        __syncthreads();
        st_inv<L, TW>(o, XF, store(out0 + z), twf);
    } else if constexpr (OP == SOP_LERAY) {  // three FP32 fields in and out
        float2 w[3][8];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (q > 0) __syncthreads();
            st_fwd<L, TW>(load_f(in0 + 3 * z + q), w[q], XF, twf);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int n, l2, l3;
            pos(i, n, l2, l3);
            double k[3], ikk;
            leray_coef(sc, n, l2, l3, k, ikk);
            const float2 a = w[0][i], b = w[1][i], c = w[2][i];
            const double sx = (k[0] * a.x + k[1] * b.x + k[2] * c.x) * ikk;
            const double sy = (k[0] * a.y + k[1] * b.y + k[2] * c.y) * ikk;
            const float2 in3[3] = {a, b, c};
#pragma unroll
            for (int q = 0; q < 3; ++q)
                w[q][i] = make_float2((float)((in3[q].x - k[q] * sx) * sc.scale),
                                      (float)((in3[q].y - k[q] * sy) * sc.scale));
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            __syncthreads();
            st_inv<L, TW>(w[q], XF, store(out0 + 3 * z + q), twf);
        }
    } else if constexpr (OP == SOP_ASSEMBLE) {  // w: 3 FP64, b: 3 FP32 -> 3 FP32
        // o_q = (K b)_q + beta A w_q: the b part first (the Leray accumulator
        // needs all three components), then the w components one at a time
        const int w0 = in0 + 6 * z, b0 = w0 + 3, o0 = out0 + 3 * z;
        float2 o[3][8], sd[8];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (q > 0) __syncthreads();
            st_fwd<L, TW>(load_f(b0 + q), o[q], XF, twf);
            if (sc.leray) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    int n, l2, l3;
                    pos(i, n, l2, l3);
                    const float kq = (float)(q == 0 ? wn_odd(n, sc.n1) : (q == 1 ? wn_odd(l2, sc.n2) : wn_odd(l3, sc.n3)));
                    const float t = kq * leray_ikk(sc, n, l2, l3);
                    const float2 tb = mk<float2>(o[q][i].x * t, o[q][i].y * t);
                    sd[i] = q == 0 ? tb : add(sd[i], tb);
                }
            }
        }
        const float fs = (float)sc.scale;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int n, l2, l3;
            pos(i, n, l2, l3);
            const float k[3] = {(float)wn_odd(n, sc.n1), (float)wn_odd(l2, sc.n2), (float)wn_odd(l3, sc.n3)};
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                float2 v = o[q][i];
                if (sc.leray) v = sub(v, mk<float2>(sd[i].x * k[q], sd[i].y * k[q]));
                o[q][i] = scl(v, fs);
            }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double2 f[8];
            __syncthreads();
            st_fwd<L, TW>(load_d(w0 + q), f, XD, twd);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                int n, l2, l3;
                pos(i, n, l2, l3);
                o[q][i] = add(o[q][i], to_f2(scl(f[i], sc.beta * reg_symbol(sc, n, l2, l3) * sc.scale)));
            }
            __syncthreads();
            st_inv<L, TW>(o[q], XF, store(o0 + q), twf);
        }
    } else {  // scalar symbols: REG (FP64), INVREG and IDENT (FP32)
        using C = typename std::conditional<OP == SOP_REG, double2, float2>::type;
        using R = typename RealOf<C>::type;
        C f[8];
        if constexpr (OP == SOP_REG)
            st_fwd<L, TW>(load_d(in0 + z), f, XD, twd);
        else
            st_fwd<L, TW>(load_f(in0 + z), f, XF, twf);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int n, l2, l3;
            pos(i, n, l2, l3);
            double fac = sc.scale;
            if (OP == SOP_REG) {
                fac *= reg_symbol(sc, n, l2, l3);
            } else if (OP == SOP_INVREG) {
                const double a = reg_symbol(sc, n, l2, l3);
                fac *= (a == 0.0) ? 1.0 / sc.beta : 1.0 / (sc.beta * a);
            }
            f[i] = scl(f[i], (R)fac);
        }
        __syncthreads();
        if constexpr (OP == SOP_REG)
            st_inv<L, TW>(f, XD, store(out0 + z), twd);
        else
            st_inv<L, TW>(f, XF, store(out0 + z), twf);
    }
}

// Assembly beta A w + K b: w three FP64 fields, b three FP32 fields, out three
// FP32 fields.  K = Leray if sc.leray.  The b components stream through one
// working tile; the Leray correction accumulates s = k.b / |k|^2.
template <int LF>
__global__ __launch_bounds__(kFftThreads) void k_x1_assemble(char *__restrict__ spec, long slot_bytes,
                                                             int w0, int b0, int out0, ColDesc d, int nyq,
                                                             int TW, int logTW, RadixPlan rp,
                                                             const double2 *__restrict__ twd,
                                                             const float2 *__restrict__ twf, SymCtx sc, Mb mb)
{
    const unsigned zc_ = gridDim.z / (unsigned)mb.count, bz_ = blockIdx.z % zc_;
    const long long mo_ = mb.offset(blockIdx.z / zc_); spec = mshift(spec, mo_);
    if (mb.stopped(mo_)) return;
    extern __shared__ char lds_raw[];
    const int L = LF > 0 ? LF : rp.L, tile = L * TW;
    double2 *WA = reinterpret_cast<double2 *>(lds_raw), *WB = WA + tile;
    float2 *FA = reinterpret_cast<float2 *>(WA), *FB = FA + tile;  // float view of the working pair
    float2 *O = reinterpret_cast<float2 *>(WB + tile);             // three output tiles
    float2 *Sd = O + 3 * tile;                                     // Leray accumulator
    const TilePos tp = tile_pos();
    const int tid = threadIdx.x, nthr = kFftThreads, col0 = tp.x * TW;
    const long off = d.base_off + (long)tp.y * d.ostride;
    const ColCtx cc{nyq, tp.y};
    for (int q = 0; q < 3; ++q) {
        const double2 *src = reinterpret_cast<const double2 *>(spec + (long)(w0 + q) * slot_bytes) + off;
        tile_load(load_target(rp, WA, WB), src, d, L, TW, logTW, col0, tid, nthr);
        __syncthreads();
        lds_fft_any<false, true, LF>(load_target(rp, WA, WB), load_target(rp, WB, WA), TW, logTW, 0, rp, twd, tid, nthr);
        for (int idx = tid; idx < tile; idx += nthr) {
            const int n = idx >> logTW, c = idx & (TW - 1);
            int l2, l3;
            cc.l23(sc, col0 + c, l2, l3);
            O[q * tile + idx] = to_f2(scl(WA[idx], sc.beta * reg_symbol(sc, n, l2, l3) * sc.scale));
        }
        __syncthreads();
    }
    for (int q = 0; q < 3; ++q) {
        const float2 *src = reinterpret_cast<const float2 *>(spec + (long)(b0 + q) * slot_bytes) + off;
        tile_load(load_target(rp, FA, FB), src, d, L, TW, logTW, col0, tid, nthr);
        __syncthreads();
        lds_fft_any<false, true, LF>(load_target(rp, FA, FB), load_target(rp, FB, FA), TW, logTW, 0, rp, twf, tid, nthr);
        for (int idx = tid; idx < tile; idx += nthr) {
            const float2 bq = FA[idx];
            const float s = (float)sc.scale;
            O[q * tile + idx] = add(O[q * tile + idx], scl(bq, s));
            if (sc.leray) {
                const int n = idx >> logTW, c = idx & (TW - 1);
                int l2, l3;
                cc.l23(sc, col0 + c, l2, l3);
                double k[3], ikk;
                leray_coef(sc, n, l2, l3, k, ikk);
                const float2 t = scl(bq, (float)(k[q] * ikk * sc.scale));
                Sd[idx] = q == 0 ? t : add(Sd[idx], t);
            }
        }
        __syncthreads();
    }
    if (sc.leray) {
        for (int idx = tid; idx < tile; idx += nthr) {
            const int n = idx >> logTW, c = idx & (TW - 1);
            int l2, l3;
            cc.l23(sc, col0 + c, l2, l3);
            double k[3], ikk;
            leray_coef(sc, n, l2, l3, k, ikk);
            const float2 s = Sd[idx];
#pragma unroll
            for (int q = 0; q < 3; ++q) O[q * tile + idx] = sub(O[q * tile + idx], scl(s, (float)k[q]));
        }
        __syncthreads();
    }
    for (int q = 0; q < 3; ++q) {
        const float2 *res = lds_fft_any<true, true, LF>(O + q * tile, FA, TW, logTW, 0, rp, twf, tid, nthr);
        float2 *dst = reinterpret_cast<float2 *>(spec + (long)(out0 + q) * slot_bytes) + off;
        tile_store(dst, res, d, L, TW, logTW, col0, tid, nthr);
        __syncthreads();
    }
}

// standard half-spectrum layout <-> internal layout (FP32 slots)
__global__ void k_pack_standard(const float2 *__restrict__ spec, float2 *__restrict__ dst, long nrow, int m3, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.z); spec = mshift(spec, mo_); dst = mshift(dst, mo_);
    const long total = nrow * (m3 + 1);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const long row = i / (m3 + 1);
        const int k = (int)(i - row * (m3 + 1));
        dst[i] = k < m3 ? spec[row * m3 + k] : spec[nrow * m3 + row];
    }
}

__global__ void k_unpack_standard(const float2 *__restrict__ srcp, float2 *__restrict__ spec, long nrow, int m3, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.z); srcp = mshift(srcp, mo_); spec = mshift(spec, mo_);
    const long total = nrow * (m3 + 1);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const long row = i / (m3 + 1);
        const int k = (int)(i - row * (m3 + 1));
        if (k < m3)
            spec[row * m3 + k] = srcp[i];
        else
            spec[nrow * m3 + row] = srcp[i];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
RadixPlan make_radix_plan(int L)
{
    RadixPlan rp{};
    rp.L = L;
    int n = L;
    while (n > 1) {
        int R = 0;
        for (int cand : {8, 4, 2, 3, 5})
            if (n % cand == 0) {
                R = cand;
                break;
            }
        if (R == 0 || rp.np >= kMaxPasses) fail(LDDMM_EINVAL, "FFT length with a prime factor other than 2, 3, 5");
        rp.r[rp.np++] = R;
        n /= R;
    }
    return rp;
}

static int floor_pow2(long x);
static int rows_per_block(int m3, size_t csize, size_t budget);
static int col_tile(int L, size_t bytes_per_elem, int ncols, size_t budget);
static void col_descs(const FftCtx &F, int axis, struct ColDesc dd[2], int outer[2]);
static size_t x1_bytes_per_elem(int op);
static void default_tiles(FftCtx &F);

// a launch grid over every member of the plan: the member index is folded
// into z (z = index within the launch + extent * member)
static dim3 mgrid(const lddmm_plan *P, dim3 g)
{
    g.z *= (unsigned)P->mb.count;
    return g;
}

template <class C>
static C *upload_twiddles(int L)
{
    std::vector<C> h(L);
    for (int m = 0; m < L; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)L;
        h[m].x = (decltype(h[m].x))std::cos(a);
        h[m].y = (decltype(h[m].y))std::sin(a);
    }
    C *d = nullptr;
    check_hip(hipMalloc(&d, sizeof(C) * L), "hipMalloc twiddles");
    check_hip(hipMemcpy(d, h.data(), sizeof(C) * L, hipMemcpyHostToDevice), "twiddle upload");
    return d;
}

void fft_init(lddmm_plan *P)
{
    FftCtx &F = P->fft;
    F.n1 = P->cfg.n[0];
    F.n2 = P->cfg.n[1];
    F.n3 = P->cfg.n[2];
    F.m3 = F.n3 / 2;
    F.nrow = (long)F.n1 * F.n2;
    F.spec_stride = F.nrow * (F.m3 + 1);
    F.rp1 = make_radix_plan(F.n1);
    F.rp2 = make_radix_plan(F.n2);
    F.rp3 = make_radix_plan(F.m3);
    F.tw1 = upload_twiddles<float2>(F.n1);
    F.tw2 = upload_twiddles<float2>(F.n2);
    F.tw3 = upload_twiddles<float2>(F.m3);
    F.twN3 = upload_twiddles<float2>(F.n3);
    F.tw1d = upload_twiddles<double2>(F.n1);
    F.tw2d = upload_twiddles<double2>(F.n2);
    F.tw3d = upload_twiddles<double2>(F.m3);
    F.twN3d = upload_twiddles<double2>(F.n3);
    default_tiles(F);
}

void fft_free(lddmm_plan *P)
{
    FftCtx &F = P->fft;
    for (void *p : {(void *)F.tw1, (void *)F.tw2, (void *)F.tw3, (void *)F.twN3, (void *)F.tw1d,
                    (void *)F.tw2d, (void *)F.tw3d, (void *)F.twN3d})
        if (p) (void)hipFree(p);
    F.tw1 = F.tw2 = F.tw3 = F.twN3 = nullptr;
    F.tw1d = F.tw2d = F.tw3d = F.twN3d = nullptr;
}

// LDS bytes per tile element of each fused x1 kernel
static size_t x1_bytes_per_elem(int op)
{
    switch (op) {
    case SOP_GRAD: return 2 * 16 + 3 * 8;
    case SOP_DIV: return 3 * 16;
    case SOP_LERAY: return 4 * 8;
    case SOP_ASSEMBLE: return 2 * 16 + 4 * 8;
    case SOP_REG: return 2 * 16;
    default: return 2 * 8;
    }
}

static int floor_pow2(long x)
{
    int p = 1;
    while ((long)p * 2 <= x) p *= 2;
    return p;
}

static int ilog2(int x)
{
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

// rows per block of the x3 passes: two buffers of TWR*(m3+1) complex values
static int rows_per_block(int m3, size_t csize, size_t budget)
{
    long cap = (long)(budget / (2 * csize * (m3 + 1)));
    int t = floor_pow2(cap < 1 ? 1 : cap);
    return t > 32 ? 32 : t;
}

// columns per tile when each column needs `bytes_per_elem` bytes of LDS per
// line element (summed over all tiles the kernel holds)
static int col_tile(int L, size_t bytes_per_elem, int ncols, size_t budget)
{
    long cap = (long)(budget / (bytes_per_elem * (size_t)L));
    int t = floor_pow2(cap < 1 ? 1 : cap);
    if (t > 32) t = 32;
    int nc = floor_pow2(ncols);
    if (nc < ncols) nc *= 2;
    if (t > nc) t = nc;
    return t;
}

// heuristic tiles: the widest power-of-two tile the LDS budget allows (<= 32)
static void default_tiles(FftCtx &F)
{
    for (int axis = 0; axis < 2; ++axis) {
        ColDesc dd[2];
        int outer[2];
        col_descs(F, axis == 1 ? 1 : 0, dd, outer);
        const int L = axis == 1 ? F.rp2.L : F.rp1.L;
        for (int part = 0; part < 2; ++part)
            for (int dbl = 0; dbl < 2; ++dbl)
                F.tw_cols[axis][part][dbl] = col_tile(L, 2 * (dbl ? 16 : 8), dd[part].ncols, kLdsBudget);
    }
    ColDesc dd[2];
    int outer[2];
    col_descs(F, 0, dd, outer);
    for (int op = 0; op < 8; ++op)
        for (int part = 0; part < 2; ++part)
            F.tw_x1[op][part] = col_tile(F.rp1.L, x1_bytes_per_elem(op), dd[part].ncols, kLdsBudget);
    F.twr_r2c[0] = rows_per_block(F.m3, sizeof(float2), kLdsBudget);
    F.twr_r2c[1] = rows_per_block(F.m3, sizeof(double2), kLdsBudget);
    F.twr_c2r = rows_per_block(F.m3, sizeof(float2), kLdsBudget);
}

static void check_lds(size_t bytes, const char *what)
{
    if (bytes > kLdsMax) fail(LDDMM_EUNSUPPORTED, std::string(what) + ": LDS tile exceeds the budget");
}

void r2c_fields(lddmm_plan *P, const RealIn &in, int count, int slot0, bool dbl)
{
    FftCtx &F = P->fft;
    const size_t cs = dbl ? sizeof(double2) : sizeof(float2);
    const int TWR = F.twr_r2c[dbl ? 1 : 0];
    const size_t lds = 2 * cs * TWR * (F.m3 + 1);
    check_lds(lds, "r2c_x3");
    dim3 grid((unsigned)((F.nrow + TWR - 1) / TWR), count);
    Scope s(P, K_R2C_X3);
    bool done = false;
    with_len(F.m3, [&]<int LF>() {
        if constexpr (RowPlan<LF>::ok) {
            auto go = [&]<int RB>() {
                using RS = RowShape<LF, RB>;
                const size_t ldsr = cs * RS::XCH;
                check_lds(ldsr, "r2c_x3");
                const dim3 gr((unsigned)((F.nrow + RB - 1) / RB), count);
                const dim3 blk(RS::NT);
                if (dbl) {
                    if (ldsr > 65536) allow_big_lds((const void *)(k_r2c_reg<double, LF, RB>));
                    hipLaunchKernelGGL((k_r2c_reg<double, LF, RB>), mgrid(P, gr), blk, ldsr, P->stream, in, P->spec,
                                       P->slot_bytes, slot0, F.nrow, F.tw3d, F.twN3d, P->mb);
                } else {
                    if (ldsr > 65536) allow_big_lds((const void *)(k_r2c_reg<float, LF, RB>));
                    hipLaunchKernelGGL((k_r2c_reg<float, LF, RB>), mgrid(P, gr), blk, ldsr, P->stream, in, P->spec,
                                       P->slot_bytes, slot0, F.nrow, F.tw3, F.twN3, P->mb);
                }
            };
            if (TWR >= RowPlan<LF>::RBA)
                go.template operator()<RowPlan<LF>::RBA>();
            else
                go.template operator()<RowPlan<LF>::RBB>();
            done = true;
        }
    });
    if (done) {
        check_hip(hipGetLastError(), "k_r2c_reg");
        return;
    }
    with_len(F.m3, [&]<int LF>() {
        if (dbl)
            FFT_LAUNCH((k_r2c_x3<double, LF>), mgrid(P, grid), lds, P->stream, in, P->spec,
                               P->slot_bytes, slot0, F.nrow, F.n3, TWR, F.rp3, F.tw3d, F.twN3d, P->mb);
        else
            FFT_LAUNCH((k_r2c_x3<float, LF>), mgrid(P, grid), lds, P->stream, in, P->spec,
                               P->slot_bytes, slot0, F.nrow, F.n3, TWR, F.rp3, F.tw3, F.twN3, P->mb);
    });
    check_hip(hipGetLastError(), "k_r2c_x3");
}

void c2r_fields(lddmm_plan *P, int slot0, int count, const RealOut &out, float scale)
{
    FftCtx &F = P->fft;
    const int TWR = F.twr_c2r;
    const size_t lds = 2 * sizeof(float2) * TWR * (F.m3 + 1);
    check_lds(lds, "c2r_x3");
    dim3 grid((unsigned)((F.nrow + TWR - 1) / TWR), count);
    Scope s(P, K_C2R_X3);
    bool done = false;
    with_len(F.m3, [&]<int LF>() {
        if constexpr (RowPlan<LF>::ok) {
            auto go = [&]<int RB>() {
                using RS = RowShape<LF, RB>;
                const size_t ldsr = sizeof(float2) * RS::XCH;
                check_lds(ldsr, "c2r_x3");
                const dim3 gr((unsigned)((F.nrow + RB - 1) / RB), count);
                if (ldsr > 65536) allow_big_lds((const void *)(k_c2r_reg<LF, RB>));
                hipLaunchKernelGGL((k_c2r_reg<LF, RB>), mgrid(P, gr), dim3(RS::NT), ldsr, P->stream, P->spec, P->slot_bytes,
                                   slot0, out, F.nrow, F.tw3, F.twN3, scale, P->mb);
            };
            if (TWR >= RowPlan<LF>::RBA)
                go.template operator()<RowPlan<LF>::RBA>();
            else
                go.template operator()<RowPlan<LF>::RBB>();
            done = true;
        }
    });
    if (done) {
        check_hip(hipGetLastError(), "k_c2r_reg");
        return;
    }
    with_len(F.m3, [&]<int LF>() {
        FFT_LAUNCH((k_c2r_x3<LF>), mgrid(P, grid), lds, P->stream, P->spec, P->slot_bytes,
                           slot0, out, F.nrow, F.n3, TWR, F.rp3, F.tw3, F.twN3, scale, P->mb);
    });
    check_hip(hipGetLastError(), "k_c2r_x3");
}

bool x3_rank1(lddmm_plan *P, int in0, int out0, const float *G)
{
    FftCtx &F = P->fft;
    bool done = false;
    with_len(F.m3, [&]<int LF>() {
        if constexpr (RowPlan<LF>::ok) {
            auto go = [&]<int RB>() {
                using RS = RowShape<LF, RB>;
                const size_t lds = sizeof(float2) * 3 * RS::XCH;  // an exchange buffer per field
                check_lds(lds, "x3_rank1");
                if (lds > 65536) allow_big_lds((const void *)(k_x3_rank1<LF, RB>));
                const dim3 gr((unsigned)((F.nrow + RB - 1) / RB), 1, P->mb.count);
                Scope s(P, K_C2R_X3);
                hipLaunchKernelGGL((k_x3_rank1<LF, RB>), gr, dim3(RS::NT), lds, P->stream, P->spec, P->slot_bytes, in0,
                                   out0, G, F.nrow, F.tw3, F.twN3, (float)(1.0 / (double)P->N), P->mb);
            };
            if (F.twr_c2r >= RowPlan<LF>::RBA)
                go.template operator()<RowPlan<LF>::RBA>();
            else
                go.template operator()<RowPlan<LF>::RBB>();
            done = true;
        }
    });
    if (done) check_hip(hipGetLastError(), "k_x3_rank1");
    return done;
}

static void col_descs(const FftCtx &F, int axis, ColDesc dd[2], int outer[2]);
static SymCtx sym_ctx(lddmm_plan *P, int leray);

void spcg_p_x1(lddmm_plan *P, const float2 *r, const float2 *z, float2 *p, int slot0, float2 *sx)
{
    FftCtx &F = P->fft;
    bool done = false;
    with_len(F.rp1.L, [&]<int LF>() {
        if constexpr (RegPlan<LF>::ok) {
            using RS = RegShape<LF>;
            ColDesc dd[2];
            int outer[2];
            col_descs(F, 0, dd, outer);
            const int g0 = (dd[0].ncols + RS::TW - 1) / RS::TW, g1 = (dd[1].ncols + RS::TW - 1) / RS::TW;
            const dim3 grid((unsigned)(g0 * outer[0] + g1), 1, 3);
            const size_t lds = sizeof(float2) * RS::XCH;
            check_lds(lds, "fft_cols");
            const PUpd pu{r, z, p, F.spec_stride, scalars(P), sym_ctx(P, 0), sx};
            Scope s(P, K_FFT_COLS);
            FFT_LAUNCH((k_cols_reg<true, float, LF, true>), mgrid(P, grid), lds, P->stream, P->spec, P->slot_bytes, slot0,
                       dd[0], dd[1], g0, outer[0], F.tw1, pu, QAsm{}, P->mb);
            done = true;
        }
    });
    if (done) {
        check_hip(hipGetLastError(), "k_cols_reg");
        return;
    }
    spcg_p(P, r, z, p, slot0, sx);
    x1_pass(P, slot0, 3, true, false);
}

bool x1_fwd_h0_assemble(lddmm_plan *P, int slot0, const float2 *p, float2 *q)
{
    FftCtx &F = P->fft;
    bool done = false;
    with_len(F.rp1.L, [&]<int LF>() {
        if constexpr (RegPlan<LF>::ok) {
            using RS = RegShape<LF>;
            ColDesc dd[2];
            int outer[2];
            col_descs(F, 0, dd, outer);
            const int g0 = (dd[0].ncols + RS::TW - 1) / RS::TW, g1 = (dd[1].ncols + RS::TW - 1) / RS::TW;
            const int tiles = g0 * outer[0] + g1;
            if (3L * tiles > red_capacity(P)) return;
            const size_t lds = sizeof(float2) * RS::XCH;
            check_lds(lds, "fft_cols");
            const QAsm qa{p, q, F.spec_stride, P->red, sym_ctx(P, 0)};
            {
                Scope s(P, K_FFT_COLS);
                FFT_LAUNCH((k_cols_reg<false, float, LF, false, true>), mgrid(P, dim3((unsigned)tiles, 1, 3)), lds,
                           P->stream, P->spec, P->slot_bytes, slot0, dd[0], dd[1], g0, outer[0], F.tw1, PUpd{}, qa, P->mb);
                check_hip(hipGetLastError(), "k_cols_reg");
            }
            dev_reduce_final_steps(P, P->red, S_KAPPA, -1, P->h3 / (double)P->N, kAfterAlpha, nullptr, 3 * tiles);
            done = true;
        }
    });
    return done;
}

// column descriptors: main array and Nyquist plane, along x2 (axis 1) or x1 (axis 0)
static void col_descs(const FftCtx &F, int axis, ColDesc dd[2], int outer[2])
{
    if (axis == 1) {
        dd[0] = {0, (long)F.n2 * F.m3, F.m3, 1, F.m3};
        outer[0] = F.n1;
        dd[1] = {F.nrow * F.m3, 0, 1, F.n2, F.n1};
        outer[1] = 1;
    } else {
        dd[0] = {0, F.m3, (long)F.n2 * F.m3, 1, F.m3};
        outer[0] = F.n2;
        dd[1] = {F.nrow * F.m3, 0, F.n2, 1, F.n2};
        outer[1] = 1;
    }
}

static void cols_pass(lddmm_plan *P, int axis, int slot0, int count, bool inverse, bool dbl,
                      int only_part = -1)
{
    FftCtx &F = P->fft;
    const RadixPlan &rp = axis == 1 ? F.rp2 : F.rp1;
    ColDesc dd[2];
    int outer[2];
    col_descs(F, axis, dd, outer);
    const size_t cs = dbl ? sizeof(double2) : sizeof(float2);
    for (int part = 0; part < 2; ++part) {
        if (only_part >= 0 && part != only_part) continue;
        const ColDesc &d = dd[part];
        Scope s(P, K_FFT_COLS);
        bool done = false;
        with_len(rp.L, [&]<int LF>() {
            if constexpr (RegPlan<LF>::ok) {
                // both parts in one launch (only_part selects one for the autotuner)
                using RS = RegShape<LF>;
                const int g0 = (dd[0].ncols + RS::TW - 1) / RS::TW, g1 = (dd[1].ncols + RS::TW - 1) / RS::TW;
                const int o0 = (only_part == 1) ? 0 : outer[0];
                const unsigned tiles = (unsigned)(g0 * o0 + (only_part == 0 ? 0 : g1));
                const dim3 grid(tiles, 1, count);
                const size_t lds = cs * RS::XCH;
                check_lds(lds, "fft_cols");
                if (dbl) {
                    const double2 *tw = axis == 1 ? F.tw2d : F.tw1d;
                    if (inverse)
                        FFT_LAUNCH((k_cols_reg<true, double, LF, false>), mgrid(P, grid), lds, P->stream, P->spec, P->slot_bytes,
                                   slot0, dd[0], dd[1], g0, o0, tw, PUpd{}, QAsm{}, P->mb);
                    else
                        FFT_LAUNCH((k_cols_reg<false, double, LF, false>), mgrid(P, grid), lds, P->stream, P->spec, P->slot_bytes,
                                   slot0, dd[0], dd[1], g0, o0, tw, PUpd{}, QAsm{}, P->mb);
                } else {
                    const float2 *tw = axis == 1 ? F.tw2 : F.tw1;
                    if (inverse)
                        FFT_LAUNCH((k_cols_reg<true, float, LF, false>), mgrid(P, grid), lds, P->stream, P->spec, P->slot_bytes,
                                   slot0, dd[0], dd[1], g0, o0, tw, PUpd{}, QAsm{}, P->mb);
                    else
                        FFT_LAUNCH((k_cols_reg<false, float, LF, false>), mgrid(P, grid), lds, P->stream, P->spec, P->slot_bytes,
                                   slot0, dd[0], dd[1], g0, o0, tw, PUpd{}, QAsm{}, P->mb);
                }
                done = true;
            }
        });
        if (done) {
            check_hip(hipGetLastError(), "k_cols_reg");
            break;  // both parts launched
        }
        const int TW = F.tw_cols[axis == 1 ? 1 : 0][part][dbl ? 1 : 0];
        const size_t lds = 2 * cs * rp.L * TW;
        check_lds(lds, "fft_cols");
        dim3 grid((unsigned)((d.ncols + TW - 1) / TW), outer[part], count);
        const int lt = ilog2(TW);
        with_len(rp.L, [&]<int LF>() {
            if (dbl) {
                const double2 *tw = axis == 1 ? F.tw2d : F.tw1d;
                if (inverse)
                    FFT_LAUNCH((k_fft_cols<true, double, LF>), mgrid(P, grid), lds, P->stream,
                                       P->spec, P->slot_bytes, slot0, d, TW, lt, rp, tw, P->mb);
                else
                    FFT_LAUNCH((k_fft_cols<false, double, LF>), mgrid(P, grid), lds, P->stream,
                                       P->spec, P->slot_bytes, slot0, d, TW, lt, rp, tw, P->mb);
            } else {
                const float2 *tw = axis == 1 ? F.tw2 : F.tw1;
                if (inverse)
                    FFT_LAUNCH((k_fft_cols<true, float, LF>), mgrid(P, grid), lds, P->stream,
                                       P->spec, P->slot_bytes, slot0, d, TW, lt, rp, tw, P->mb);
                else
                    FFT_LAUNCH((k_fft_cols<false, float, LF>), mgrid(P, grid), lds, P->stream,
                                       P->spec, P->slot_bytes, slot0, d, TW, lt, rp, tw, P->mb);
            }
        });
        check_hip(hipGetLastError(), "k_fft_cols");
    }
}

void x2_pass(lddmm_plan *P, int slot0, int count, bool inverse, bool dbl)
{
    cols_pass(P, 1, slot0, count, inverse, dbl);
}

void x1_pass(lddmm_plan *P, int slot0, int count, bool inverse, bool dbl)
{
    cols_pass(P, 0, slot0, count, inverse, dbl);
}

int op_nin(int op)
{
    switch (op) {
    case SOP_GRAD: return 1;
    case SOP_ASSEMBLE: return 6;
    case SOP_IDENT: return 1;
    default: return 3;
    }
}

int op_nout(int op)
{
    switch (op) {
    case SOP_DIV: return 1;
    case SOP_IDENT: return 1;
    default: return 3;
    }
}

// precision of the forward transform of input field i of op
static bool input_is_fp64(int op, int i)
{
    switch (op) {
    case SOP_GRAD:
    case SOP_DIV:
    case SOP_REG: return true;
    case SOP_ASSEMBLE: return i < 3;
    default: return false;
    }
}

static SymCtx sym_ctx(lddmm_plan *P, int leray)
{
    FftCtx &F = P->fft;
    SymCtx sc;
    sc.n1 = F.n1;
    sc.n2 = F.n2;
    sc.n3 = F.n3;
    sc.scale = 1.0 / ((double)F.n1 * F.n2 * F.n3);
    sc.beta = P->beta_sym > 0.0 ? P->beta_sym : P->cfg.beta;
    sc.reg = P->cfg.reg;
    sc.leray = leray;
    return sc;
}

// x1 forward, symbol, x1 inverse for nbatch batches: inputs of batch b at
// slots in0 + b*nin .. , outputs at out0 + b*nout ..
// only_part: -1 both parts of the spectrum in one launch, 0 / 1 one of them
template <int LF, int TW>
static void x1_reg_launch(lddmm_plan *P, int op, int in0, int out0, const ColDesc (&dd)[2], const int (&outer)[2],
                          int only_part, int nbatch, const SymCtx &sc)
{
    FftCtx &F = P->fft;
    using RS = StShape<LF, TW>;
    const bool fp64x = op == SOP_GRAD || op == SOP_DIV || op == SOP_ASSEMBLE || op == SOP_REG;
    const size_t lds = (fp64x ? sizeof(double2) : sizeof(float2)) * RS::XCH;
    check_lds(lds, "x1_symbol");
    const int nz = (op == SOP_REG || op == SOP_INVREG) ? 3 * nbatch : nbatch;
    const int g0 = (dd[0].ncols + TW - 1) / TW, g1 = (dd[1].ncols + TW - 1) / TW;
    const int o0 = only_part == 1 ? 0 : outer[0];
    const dim3 grid((unsigned)(g0 * o0 + (only_part == 0 ? 0 : g1)), 1, nz);
    Scope s(P, K_SPECTRAL_X1);
#define X1R(OPV)                                                                                         \
    do {                                                                                                 \
        if (lds > 65536) allow_big_lds((const void *)(k_x1_reg<OPV, LF, TW>));                           \
        hipLaunchKernelGGL((k_x1_reg<OPV, LF, TW>), mgrid(P, grid), dim3(RS::NT), lds, P->stream, P->spec,         \
                           P->slot_bytes, in0, out0, dd[0], dd[1], g0, o0, F.tw1d, F.tw1, sc, P->mb);            \
    } while (0)
    switch (op) {
    case SOP_GRAD: X1R(SOP_GRAD); break;
    case SOP_DIV: X1R(SOP_DIV); break;
    case SOP_LERAY: X1R(SOP_LERAY); break;
    case SOP_ASSEMBLE: X1R(SOP_ASSEMBLE); break;
    case SOP_REG: X1R(SOP_REG); break;
    case SOP_INVREG: X1R(SOP_INVREG); break;
    case SOP_IDENT: X1R(SOP_IDENT); break;
    default: fail(LDDMM_EINVAL, "unknown spectral operator");
    }
#undef X1R
}

static void x1_symbol_parts(lddmm_plan *P, int op, int in0, int out0, int nbatch, int leray, int only_part);

void x1_symbol(lddmm_plan *P, int op, int in0, int out0, int nbatch, int leray)
{
    x1_symbol_parts(P, op, in0, out0, nbatch, leray, -1);
}

static void x1_symbol_parts(lddmm_plan *P, int op, int in0, int out0, int nbatch, int leray, int only_part)
{
    FftCtx &F = P->fft;
    const RadixPlan &rp = F.rp1;
    const int L = rp.L;
    const SymCtx sc = sym_ctx(P, leray);
    ColDesc dd[2];
    int outer[2];
    col_descs(F, 0, dd, outer);
    for (int part = 0; part < 2; ++part) {
        if (only_part >= 0 && part != only_part) continue;
        const ColDesc &d = dd[part];
        bool done = false;
        with_len(L, [&]<int LF>() {
            if constexpr (StPlan<LF>::ok) {
                // both parts in one launch with the main part's tile width
                // (only_part selects one for the autotuner)
                using SP = StPlan<LF>;
                const bool wide = F.tw_x1[op][part] >= SP::TWA;
                if (wide)
                    x1_reg_launch<LF, SP::TWA>(P, op, in0, out0, dd, outer, only_part, nbatch, sc);
                else
                    x1_reg_launch<LF, SP::TWB>(P, op, in0, out0, dd, outer, only_part, nbatch, sc);
                done = true;
            }
        });
        if (done) {
            check_hip(hipGetLastError(), "k_x1_reg");
            break;  // both parts launched (or the one asked for)
        }
        const size_t per = x1_bytes_per_elem(op);  // LDS bytes per tile element
        const int TW = F.tw_x1[op][part];
        const size_t lds = per * L * TW;
        check_lds(lds, "x1_symbol");
        const int lt = ilog2(TW);
        const unsigned gx = (unsigned)((d.ncols + TW - 1) / TW);
        Scope s(P, K_SPECTRAL_X1);
        with_len(L, [&]<int LF>() {
            switch (op) {
            case SOP_GRAD:
                FFT_LAUNCH((k_x1_grad<LF>), mgrid(P, dim3(gx, outer[part], nbatch)), lds, P->stream, P->spec, P->slot_bytes, in0, out0, d, part, TW, lt, rp, F.tw1d,
                                   F.tw1, sc, P->mb);
                break;
            case SOP_DIV:
                FFT_LAUNCH((k_x1_div<LF>), mgrid(P, dim3(gx, outer[part], nbatch)), lds, P->stream, P->spec, P->slot_bytes, in0, out0, d, part, TW, lt, rp, F.tw1d,
                                   F.tw1, sc, P->mb);
                break;
            case SOP_LERAY:
                FFT_LAUNCH((k_x1_leray<LF>), mgrid(P, dim3(gx, outer[part], nbatch)), lds, P->stream, P->spec, P->slot_bytes, in0, out0, d, part, TW, lt, rp, F.tw1, sc, P->mb);
                break;
            case SOP_ASSEMBLE:
                for (int b = 0; b < nbatch; ++b)
                    FFT_LAUNCH((k_x1_assemble<LF>), mgrid(P, dim3(gx, outer[part], 1)), lds, P->stream, P->spec, P->slot_bytes, in0 + 6 * b, in0 + 6 * b + 3,
                                       out0 + 3 * b, d, part, TW, lt, rp, F.tw1d, F.tw1, sc, P->mb);
                break;
            case SOP_REG:  // three independent fields per batch
                FFT_LAUNCH((k_x1_scalar<double, SYM_REG, LF>), mgrid(P, dim3(gx, outer[part], 3 * nbatch)), lds, P->stream, P->spec, P->slot_bytes, in0, out0, d,
                                   part, TW, lt, rp, F.tw1d, sc, P->mb);
                break;
            case SOP_INVREG:
                FFT_LAUNCH((k_x1_scalar<float, SYM_INVREG, LF>), mgrid(P, dim3(gx, outer[part], 3 * nbatch)), lds, P->stream, P->spec, P->slot_bytes, in0, out0, d,
                                   part, TW, lt, rp, F.tw1, sc, P->mb);
                break;
            case SOP_IDENT:
                FFT_LAUNCH((k_x1_scalar<float, SYM_IDENT, LF>), mgrid(P, dim3(gx, outer[part], nbatch)), lds, P->stream, P->spec, P->slot_bytes, in0, out0, d,
                                   part, TW, lt, rp, F.tw1, sc, P->mb);
                break;
            default: fail(LDDMM_EINVAL, "unknown spectral operator");
            }
        });
        check_hip(hipGetLastError(), "x1_symbol");
    }
}

// Apply a spectral operator to real fields.  The real inputs are grouped in
// batches of op_nin(op) fields; batches are processed in chunks that fit the
// plan's spectral scratch (input slots followed by output slots).
// forward x3 and x2 passes of inputs [f0, fin) of one chunk into slots
// f0 .., grouped by precision (consecutive runs of at most eight)
static void forward_passes(lddmm_plan *P, int op, const float *const *in, int nin, int f0, int fin)
{
    while (f0 < fin) {
        const bool dbl = input_is_fp64(op, f0 % nin);
        int f1 = f0 + 1;
        while (f1 < fin && f1 - f0 < 8 && input_is_fp64(op, f1 % nin) == dbl) ++f1;
        RealIn ri{};
        for (int i = f0; i < f1; ++i) ri.p[i - f0] = in[i];
        r2c_fields(P, ri, f1 - f0, f0, dbl);
        x2_pass(P, f0, f1 - f0, false, dbl);
        f0 = f1;
    }
}

void spectral_forward(lddmm_plan *P, int op, const std::vector<const float *> &in, int count)
{
    if (count > op_nin(op) || count > (int)in.size() || P->nspec < op_nin(op) + op_nout(op))
        fail(LDDMM_EINVAL, "spectral_forward: bad field count");
    forward_passes(P, op, in.data(), op_nin(op), 0, count);
}

void spectral_apply(lddmm_plan *P, int op, const std::vector<const float *> &in,
                    const std::vector<float *> &out, int fwd_done)
{
    const int nin = op_nin(op), nout = op_nout(op);
    const int nbatch = (int)in.size() / nin;
    if ((int)in.size() != nbatch * nin || (int)out.size() != nbatch * nout)
        fail(LDDMM_EINVAL, "spectral_apply: field count mismatch");
    if (fwd_done && nbatch != 1) fail(LDDMM_EINVAL, "spectral_apply: forward passes done for one field set only");
    const int per = nin + nout;
    const int chunk = P->nspec / per;
    if (chunk < 1) fail(LDDMM_EINVAL, "spectral scratch too small");
    for (int b0 = 0; b0 < nbatch; b0 += chunk) {
        const int nb = std::min(chunk, nbatch - b0);
        const int fin = nb * nin, fout = nb * nout;
        forward_passes(P, op, in.data() + (size_t)b0 * nin, nin, fwd_done, fin);
        x1_symbol(P, op, 0, fin, nb, P->cfg.leray);
        x2_pass(P, fin, fout, true, false);
        for (int g0 = 0; g0 < fout; g0 += 8) {
            RealOut ro{};
            const int cnt = std::min(8, fout - g0);
            for (int i = 0; i < cnt; ++i) ro.p[i] = out[(size_t)b0 * nout + g0 + i];
            c2r_fields(P, fin + g0, cnt, ro, 1.0f);
        }
    }
}

// ---------------------------------------------------------------------------
// autotuner: candidate tiles are the powers of two from the LDS-budget
// maximum down to 1; each is timed with HIP events (one warm-up, three timed
// launches) on the plan's own buffers and the fastest is kept.
// ---------------------------------------------------------------------------
template <class Fn>
static float time_ms(lddmm_plan *P, Fn &&fn)
{
    hipEvent_t a, b;
    check_hip(hipEventCreate(&a), "hipEventCreate");
    check_hip(hipEventCreate(&b), "hipEventCreate");
    fn();
    check_hip(hipEventRecord(a, P->stream), "hipEventRecord");
    for (int r = 0; r < 3; ++r) fn();
    check_hip(hipEventRecord(b, P->stream), "hipEventRecord");
    check_hip(hipEventSynchronize(b), "hipEventSynchronize");
    float ms = 0.f;
    check_hip(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

template <class Fn>
static void tune_one(lddmm_plan *P, int &slot, int top, Fn &&fn, int bottom = 1)
{
    int best = top;
    float bt = 1e30f;
    for (int t = top; t >= bottom; t >>= 1) {
        slot = t;
        const float ms = time_ms(P, fn);
        if (ms < bt) {
            bt = ms;
            best = t;
        }
    }
    slot = best;
}

static std::vector<int *> tunables(FftCtx &F)
{
    std::vector<int *> v;
    for (auto &a : F.tw_cols)
        for (auto &p : a)
            for (int &x : p) v.push_back(&x);
    for (auto &o : F.tw_x1)
        for (int &x : o) v.push_back(&x);
    v.push_back(&F.twr_r2c[0]);
    v.push_back(&F.twr_r2c[1]);
    v.push_back(&F.twr_c2r);
    return v;
}

static std::string tune_key(lddmm_plan *P)
{
    hipDeviceProp_t prop;
    check_hip(hipGetDeviceProperties(&prop, P->device), "hipGetDeviceProperties");
    const FftCtx &F = P->fft;
    return std::string(prop.gcnArchName) + ":" + std::to_string(F.n1) + "x" + std::to_string(F.n2) +
           "x" + std::to_string(F.n3);
}

static std::map<std::string, std::vector<int>> &tune_cache()
{
    static std::map<std::string, std::vector<int>> c;
    return c;
}

static void load_cache_file()
{
    static bool loaded = false;
    if (loaded) return;
    loaded = true;
    const char *path = std::getenv("LDDMM_TUNE_CACHE");
    if (!path) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ss(line);
        std::string key;
        if (!(ss >> key)) continue;
        std::vector<int> vals;
        int x;
        while (ss >> x) vals.push_back(x);
        tune_cache()[key] = vals;
    }
}

void autotune_fft(lddmm_plan *P)
{
    FftCtx &F = P->fft;
    load_cache_file();
    const std::string key = tune_key(P);
    std::vector<int *> tv = tunables(F);
    auto it = tune_cache().find(key);
    if (it != tune_cache().end() && it->second.size() == tv.size()) {
        for (size_t i = 0; i < tv.size(); ++i) *tv[i] = it->second[i];
        F.tuned = 1;
        return;
    }
    const bool timing = P->timing.on;
    P->timing.on = false;
    const long N = P->N;
    RealIn ri{};
    for (int c = 0; c < 3; ++c) ri.p[c] = P->v + c * N;
    RealOut ro{};
    for (int c = 0; c < 3; ++c) ro.p[c] = P->b + c * N;
    int rba = 0, rbb = 0;  // register row-pass candidates, when n3/2 has a plan
    with_len(F.m3, [&]<int LF>() {
        if constexpr (RowPlan<LF>::ok) {
            rba = RowPlan<LF>::RBA;
            rbb = RowPlan<LF>::RBB;
        }
    });
    for (int dbl = 0; dbl < 2; ++dbl) {
        auto run = [&] { r2c_fields(P, ri, 3, 0, dbl != 0); };
        if (rba > 0)
            tune_one(P, F.twr_r2c[dbl], rba, run, rbb);
        else
            tune_one(P, F.twr_r2c[dbl], rows_per_block(F.m3, dbl ? sizeof(double2) : sizeof(float2), kLdsMax), run);
    }
    {
        auto run = [&] { c2r_fields(P, 0, 3, ro, 1.f); };
        if (rba > 0)
            tune_one(P, F.twr_c2r, rba, run, rbb);
        else
            tune_one(P, F.twr_c2r, rows_per_block(F.m3, sizeof(float2), kLdsMax), run);
    }
    for (int axis = 0; axis < 2; ++axis) {
        ColDesc dd[2];
        int outer[2];
        col_descs(F, axis == 1 ? 1 : 0, dd, outer);
        const int L = axis == 1 ? F.rp2.L : F.rp1.L;
        for (int part = 0; part < 2; ++part)
            for (int dbl = 0; dbl < 2; ++dbl)
                tune_one(P, F.tw_cols[axis][part][dbl], col_tile(L, 2 * (dbl ? 16 : 8), dd[part].ncols, kLdsMax),
                         [&] { cols_pass(P, axis == 1 ? 1 : 0, 0, 3, false, dbl != 0, part); });
    }
    ColDesc d1[2];
    int o1[2];
    col_descs(F, 0, d1, o1);
    const int ops[] = {SOP_GRAD, SOP_DIV, SOP_REG, SOP_INVREG, SOP_LERAY, SOP_ASSEMBLE};
    int twa = 0, twb = 0;  // register-pass tile widths, when the x1 length has them
    with_len(F.rp1.L, [&]<int LF>() {
        if constexpr (StPlan<LF>::ok) {
            twa = StPlan<LF>::TWA;
            twb = StPlan<LF>::TWB;
        }
    });
    for (int op : ops)
        for (int part = 0; part < 2; ++part) {
            auto run = [&] { x1_symbol_parts(P, op, 0, op_nin(op), 1, 1, part); };
            if (twa > 0)
                tune_one(P, F.tw_x1[op][part], twa, run, twb);
            else
                tune_one(P, F.tw_x1[op][part],
                         col_tile(F.rp1.L, x1_bytes_per_elem(op), d1[part].ncols, kLdsMax), run);
        }
    P->timing.on = timing;
    F.tuned = 1;
    std::vector<int> vals;
    for (int *p : tv) vals.push_back(*p);
    tune_cache()[key] = vals;
    if (const char *path = std::getenv("LDDMM_TUNE_CACHE")) {
        std::ofstream out(path, std::ios::app);
        out << key;
        for (int x : vals) out << ' ' << x;
        out << '\n';
    }
}

std::string tuning_report(const lddmm_plan *P)
{
    const FftCtx &F = P->fft;
    std::ostringstream o;
    o << "tuned=" << F.tuned << " r2c_rows=" << F.twr_r2c[0] << "/" << F.twr_r2c[1]
      << " c2r_rows=" << F.twr_c2r << " cols_x1=" << F.tw_cols[0][0][0] << "/" << F.tw_cols[0][0][1]
      << " cols_x2=" << F.tw_cols[1][0][0] << "/" << F.tw_cols[1][0][1]
      << " x1_grad=" << F.tw_x1[SOP_GRAD][0] << " x1_div=" << F.tw_x1[SOP_DIV][0]
      << " x1_reg=" << F.tw_x1[SOP_REG][0] << " x1_invreg=" << F.tw_x1[SOP_INVREG][0]
      << " x1_leray=" << F.tw_x1[SOP_LERAY][0] << " x1_assemble=" << F.tw_x1[SOP_ASSEMBLE][0];
    return o.str();
}

// Spectral resampling between a grid and its half (two-level preconditioner):
// FP32 spectra in the private layout (main [n1][n2][n3/2], then the Nyquist
// plane).  Every destination coefficient of wavenumber k takes the source
// coefficient of the same k times scale when |k_d| < nc_d/2 on every axis of
// the coarse grid nc (coarse Nyquist modes dropped), else zero.
__global__ void k_resample(const float2 *__restrict__ src, int s1, int s2, int sm3, float2 *__restrict__ dst,
                           int d1, int d2, int dm3, int c1, int c2, int cm3, float scale, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.z); src = mshift(src, mo_); dst = mshift(dst, mo_);
    const long nrow = (long)d1 * d2, total = nrow * (dm3 + 1);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        long row;
        int k;
        if (i < nrow * dm3) {
            row = i / dm3;
            k = (int)(i - row * dm3);
        } else {
            row = i - nrow * dm3;
            k = dm3;
        }
        const int l1 = (int)(row / d2), l2 = (int)(row - (long)l1 * d2);
        const int k1 = 2 * l1 <= d1 ? l1 : l1 - d1, k2 = 2 * l2 <= d2 ? l2 : l2 - d2;
        float2 v = make_float2(0.f, 0.f);
        if (2 * abs(k1) < c1 && 2 * abs(k2) < c2 && k < cm3) {
            const int m1 = k1 < 0 ? k1 + s1 : k1, m2 = k2 < 0 ? k2 + s2 : k2;
            const float2 u = src[((long)m1 * s2 + m2) * sm3 + k];  // k < cm3 <= sm3: main array
            v = make_float2(scale * u.x, scale * u.y);
        }
        dst[i < nrow * dm3 ? row * dm3 + k : nrow * dm3 + row] = v;
    }
}

void spectral_resample(lddmm_plan *S, int s0, lddmm_plan *D, int d0, int count)
{
    const FftCtx &FS = S->fft, &FD = D->fft;
    const bool down = FD.n1 < FS.n1;
    const FftCtx &FC = down ? FD : FS;  // the coarse grid
    const float scale = (float)((double)FD.n1 * FD.n2 * FD.n3 / ((double)FS.n1 * FS.n2 * FS.n3));
    Scope sc(D, K_PACK);
    for (int f = 0; f < count; ++f) {
        const float2 *src = reinterpret_cast<const float2 *>(S->spec + (long)(s0 + f) * S->slot_bytes);
        float2 *dst = reinterpret_cast<float2 *>(D->spec + (long)(d0 + f) * D->slot_bytes);
        hipLaunchKernelGGL(k_resample, mgrid(D, dim3(1024)), dim3(256), 0, D->stream, src, FS.n1, FS.n2, FS.m3, dst, FD.n1,
                           FD.n2, FD.m3, FC.n1, FC.n2, FC.m3, scale, D->mb);
    }
    check_hip(hipGetLastError(), "k_resample");
}

void pack_standard(lddmm_plan *P, int slot, float2 *dst)
{
    FftCtx &F = P->fft;
    Scope s(P, K_PACK);
    hipLaunchKernelGGL(k_pack_standard, mgrid(P, dim3(1024)), dim3(256), 0, P->stream,
                       reinterpret_cast<const float2 *>(P->spec + (long)slot * P->slot_bytes), dst, F.nrow, F.m3, P->mb);
    check_hip(hipGetLastError(), "k_pack_standard");
}

void unpack_standard(lddmm_plan *P, const float2 *srcp, int slot)
{
    FftCtx &F = P->fft;
    Scope s(P, K_PACK);
    hipLaunchKernelGGL(k_unpack_standard, mgrid(P, dim3(1024)), dim3(256), 0, P->stream, srcp,
                       reinterpret_cast<float2 *>(P->spec + (long)slot * P->slot_bytes), F.nrow, F.m3, P->mb);
    check_hip(hipGetLastError(), "k_unpack_standard");
}

// ---------------------------------------------------------------------------
// Spectral-domain PCG vectors (Algorithm "GNK").  The PCG keeps its residual
// r, search direction p and H p as FP32 spectra in the internal layout,
// unnormalised (F f, the forward transform without 1/N): the preconditioner
// (beta A)^{-1} and the beta A part of the Hessian are then pointwise in k,
// and an iteration transforms only the body force forward and the search
// direction back (for the transport sweeps).  Inner products follow from
// Parseval's identity over the half spectrum:
//   sum_x a b = (1/N) sum_k w_k Re(conj(F a)_k (F b)_k),
// w = 1 on the planes k3 = 0 and k3 = n3/2, w = 2 elsewhere.
// ---------------------------------------------------------------------------
// Two-level preconditioner on spectra (restriction R: truncation to the half
// grid's wavenumbers |k_d| < n_d/4, times N_c/N_f; prolongation P: zero
// padding, times N_f/N_c).  Fine entry (l1, l2, l3) of wavenumber k and the
// half grid's entry of the same k: (k1 mod c1, k2 mod c2, l3) when inside.
struct TwoGrid {
    int f1, f2, fm3;  // fine n1, n2, n3/2
    int c1, c2, cm3;  // coarse n1, n2, n3/2
    __device__ __forceinline__ long coarse_of(int l1, int l2, int l3) const
    {
        const int k1 = 2 * l1 <= f1 ? l1 : l1 - f1, k2 = 2 * l2 <= f2 ? l2 : l2 - f2;
        if (!(2 * abs(k1) < c1 && 2 * abs(k2) < c2 && l3 < cm3)) return -1;
        const int m1 = k1 < 0 ? k1 + c1 : k1, m2 = k2 < 0 ? k2 + c2 : k2;
        return ((long)m1 * c2 + m2) * cm3 + l3;
    }
    __device__ __forceinline__ long fine_of(int l1, int l2, int l3) const
    {
        const int k1 = 2 * l1 <= c1 ? l1 : l1 - c1, k2 = 2 * l2 <= c2 ? l2 : l2 - c2;
        if (!(2 * abs(k1) < c1 && 2 * abs(k2) < c2 && l3 < cm3)) return -1;
        const int m1 = k1 < 0 ? k1 + f1 : k1, m2 = k2 < 0 ? k2 + f2 : k2;
        return ((long)m1 * f2 + m2) * fm3 + l3;
    }
};

struct SpecIdx {
    unsigned nmain;  // n1 n2 m3 entries of the main array, then the Nyquist plane
    unsigned m3, n2;
    // spectral indices and Hermitian weight of entry e of a field
    __device__ __forceinline__ void at(unsigned e, int &l1, int &l2, int &l3, double &w) const
    {
        unsigned row;
        if (e < nmain) {
            row = e / m3;
            l3 = (int)(e - row * m3);
            w = l3 == 0 ? 1.0 : 2.0;
        } else {
            row = e - nmain;
            l3 = (int)m3;
            w = 1.0;
        }
        l1 = (int)(row / n2);
        l2 = (int)(row - (unsigned)l1 * n2);
    }
};

#define SPEC_LOOP(S)                                                                                  \
    for (unsigned e = blockIdx.x * blockDim.x + threadIdx.x; e < (unsigned)(S); e += gridDim.x * blockDim.x)

// q = K b + beta A p (K: the Leray projection when LERAY, else the identity;
// b the forward transform of the body force in transform slots, bstride
// float2 apart) and the partial sums of <p, q> (one per workgroup)
template <bool LERAY>
__global__ __launch_bounds__(256) void k_spec_assemble(const float2 *__restrict__ b, long bstride,
                                                       const float2 *__restrict__ p, float2 *__restrict__ q, long S,
                                                       SpecIdx ix, SymCtx sc, double *__restrict__ partial, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y);
    if (mb.stopped(mo_)) return;
    b = mshift(b, mo_); p = mshift(p, mo_); q = mshift(q, mo_); partial = mshift(partial, mo_);
    double acc = 0.0, unused = 0.0;
    SPEC_LOOP(S)
    {
        int l1, l2, l3;
        double w;
        ix.at(e, l1, l2, l3, w);
        float2 o[3] = {b[e], b[bstride + e], b[2 * bstride + e]};
        if constexpr (LERAY) {
            // the order of the fused assembly: s = sum_q (k_q / |k|^2) b_q,
            // then b_q - k_q s, in FP32 (|k|^2 an exact integer)
            const float ikk = leray_ikk(sc, l1, l2, l3);
            const float k[3] = {(float)wn_odd(l1, sc.n1), (float)wn_odd(l2, sc.n2), (float)wn_odd(l3, sc.n3)};
            float2 sd = make_float2(0.f, 0.f);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const float t = k[f] * ikk;
                const float2 tb = make_float2(o[f].x * t, o[f].y * t);
                sd = f == 0 ? tb : make_float2(sd.x + tb.x, sd.y + tb.y);
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) o[f] = make_float2(o[f].x - sd.x * k[f], o[f].y - sd.y * k[f]);
        }
        const double ba = sc.beta * reg_symbol(sc, l1, l2, l3);
        double d = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float2 pv = p[f * S + e];
            const float2 v = make_float2(o[f].x + (float)(pv.x * ba), o[f].y + (float)(pv.y * ba));
            q[f * S + e] = v;
            d += (double)pv.x * v.x + (double)pv.y * v.y;
        }
        acc += w * d;
    }
    block_sum2(acc, unused);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// PCG start from r = sign b (b: spectra bstride float2 apart, e.g. F(rhs) in
// transform slots): r written unless NULL; p = M^{-1} r unless NULL, with a
// copy into c (cstride apart) unless NULL; the partial sums of <r, r> and
// <r, M^{-1} r> (partial, partial + gridDim.x)
__global__ __launch_bounds__(256) void k_spcg_start(const float2 *__restrict__ b, long bstride, float sign,
                                                    float2 *__restrict__ r, float2 *__restrict__ p,
                                                    float2 *__restrict__ c, long cstride, long S, SpecIdx ix,
                                                    SymCtx sc, double *__restrict__ partial, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y);
    if (mb.stopped(mo_)) return;
    b = mshift(b, mo_); r = mshift(r, mo_); p = mshift(p, mo_); c = mshift(c, mo_); partial = mshift(partial, mo_);
    double arr = 0.0, arz = 0.0;
    SPEC_LOOP(S)
    {
        int l1, l2, l3;
        double w;
        ix.at(e, l1, l2, l3, w);
        const float m = invreg_factor(sc, l1, l2, l3);
        double srr = 0.0, srz = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float2 bv = b[f * bstride + e];
            const float2 rv = make_float2(sign * bv.x, sign * bv.y);
            const float2 zv = make_float2(m * rv.x, m * rv.y);
            if (r) r[f * S + e] = rv;
            if (p) p[f * S + e] = zv;
            if (c) c[f * cstride + e] = zv;
            srr += (double)rv.x * rv.x + (double)rv.y * rv.y;
            srz += (double)rv.x * zv.x + (double)rv.y * zv.y;
        }
        arr += w * srr;
        arz += w * srz;
    }
    block_sum2(arr, arz);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = arr;
        partial[gridDim.x + blockIdx.x] = arz;
    }
}

// r -= alpha q and, unless x is NULL, x += alpha p (alpha from the device
// scalars d; nothing changes when alpha = 0, i.e. after a stop), then the
// partial sums of <r, r> and <r, M^{-1} r>
__global__ __launch_bounds__(256) void k_spcg_r(float2 *__restrict__ r, const float2 *__restrict__ q,
                                                float2 *__restrict__ x, const float2 *__restrict__ p, long S,
                                                SpecIdx ix, SymCtx sc, const double *__restrict__ d,
                                                double *__restrict__ partial, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y);
    if (mb.stopped(mo_)) return;
    r = mshift(r, mo_); q = mshift(q, mo_); x = mshift(x, mo_); p = mshift(p, mo_); d = mshift(d, mo_);
    partial = mshift(partial, mo_);
    const float al = (float)d[S_ALPHA];
    double arr = 0.0, arz = 0.0;
    SPEC_LOOP(S)
    {
        int l1, l2, l3;
        double w;
        ix.at(e, l1, l2, l3, w);
        const float m = invreg_factor(sc, l1, l2, l3);
        double srr = 0.0, srz = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            float2 rv = r[f * S + e];
            if (al != 0.f) {
                const float2 qv = q[f * S + e];
                rv = make_float2(__builtin_fmaf(-al, qv.x, rv.x), __builtin_fmaf(-al, qv.y, rv.y));
                r[f * S + e] = rv;
                if (x) {
                    const float2 pv = p[f * S + e], xv = x[f * S + e];
                    x[f * S + e] = make_float2(__builtin_fmaf(al, pv.x, xv.x), __builtin_fmaf(al, pv.y, xv.y));
                }
            }
            const float2 zv = make_float2(m * rv.x, m * rv.y);
            srr += (double)rv.x * rv.x + (double)rv.y * rv.y;
            srz += (double)rv.x * zv.x + (double)rv.y * zv.y;
        }
        arr += w * srr;
        arz += w * srz;
    }
    block_sum2(arr, arz);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = arr;
        partial[gridDim.x + blockIdx.x] = arz;
    }
}

// p = z + beta p with z = M^{-1} r, or the given z when z is not NULL (beta
// from the device scalars d; p kept once the PCG has stopped), and a copy of
// p into c (cstride apart) unless c is NULL; unless s is NULL first s +=
// alpha p (the p before its update)
__global__ __launch_bounds__(256) void k_spcg_p(const float2 *__restrict__ r, const float2 *__restrict__ z,
                                                float2 *__restrict__ p, float2 *__restrict__ c, long cstride, long S,
                                                SpecIdx ix, SymCtx sc, const double *__restrict__ d,
                                                float2 *__restrict__ s, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y);
    // after a stop only the stopping iteration's s update (alpha != 0) is left
    if (mb.stopped(mo_) && (!s || mshift(d, mo_)[S_ALPHA] == 0.0)) return;
    r = mshift(r, mo_); z = mshift(z, mo_); p = mshift(p, mo_); c = mshift(c, mo_); d = mshift(d, mo_);
    s = mshift(s, mo_);
    const bool upd = d[S_DONE] == 0.0;
    const float be = (float)d[S_BETA], al = (float)d[S_ALPHA];
    SPEC_LOOP(S)
    {
        int l1, l2, l3;
        double w;
        ix.at(e, l1, l2, l3, w);
        const float m = (upd && !z) ? invreg_factor(sc, l1, l2, l3) : 0.f;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            float2 pv = p[f * S + e];
            if (s && al != 0.f) {
                const float2 sv = s[f * S + e];
                s[f * S + e] = make_float2(__builtin_fmaf(al, pv.x, sv.x), __builtin_fmaf(al, pv.y, sv.y));
            }
            if (upd) {
                float2 zv;
                if (z) {
                    zv = z[f * S + e];
                } else {
                    const float2 rv = r[f * S + e];
                    zv = make_float2(m * rv.x, m * rv.y);
                }
                pv = make_float2(__builtin_fmaf(be, pv.x, zv.x), __builtin_fmaf(be, pv.y, zv.y));
                p[f * S + e] = pv;
            }
            if (c) c[f * cstride + e] = pv;
        }
    }
}

// the partial sums of <a, b> over three spectra each
__global__ __launch_bounds__(256) void k_spec_dot(const float2 *__restrict__ a, const float2 *__restrict__ b, long S,
                                                  SpecIdx ix, double *__restrict__ partial, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y);
    if (mb.stopped(mo_)) return;
    a = mshift(a, mo_); b = mshift(b, mo_); partial = mshift(partial, mo_);
    double acc = 0.0, unused = 0.0;
    SPEC_LOOP(S)
    {
        int l1, l2, l3;
        double w;
        ix.at(e, l1, l2, l3, w);
        double t = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float2 u = a[f * S + e], v = b[f * S + e];
            t += (double)u.x * v.x + (double)u.y * v.y;
        }
        acc += w * t;
    }
    block_sum2(acc, unused);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}
// dst_f = src_f, or M^{-1} src_f (inv), for three spectra
__global__ __launch_bounds__(256) void k_spec_copy3(const float2 *__restrict__ src, long sstride, float2 *__restrict__ dst,
                                                    long dstride, long S, SpecIdx ix, SymCtx sc, int inv, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y);
    if (mb.stopped(mo_)) return;
    src = mshift(src, mo_); dst = mshift(dst, mo_);
    SPEC_LOOP(S)
    {
        int l1, l2, l3;
        double w;
        ix.at(e, l1, l2, l3, w);
        const float m = inv ? invreg_factor(sc, l1, l2, l3) : 1.f;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float2 v = src[f * sstride + e];
            dst[f * dstride + e] = inv ? make_float2(m * v.x, m * v.y) : v;
        }
    }
}
// R r (coarse, three spectra rc) and s_c0 = (beta0 A_c)^{-1} R r (sc0) from
// the fine spectra r; the loop runs over the coarse entries (sc: the coarse
// symbol)
__global__ __launch_bounds__(256) void k_2l_restrict(const float2 *__restrict__ r, long Sf, float2 *__restrict__ rc,
                                                     float2 *__restrict__ sc0, long Sc, SpecIdx ixc, TwoGrid tg,
                                                     float scale, SymCtx sc, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y);
    if (mb.stopped(mo_)) return;
    r = mshift(r, mo_); rc = mshift(rc, mo_); sc0 = mshift(sc0, mo_);
    SPEC_LOOP(Sc)
    {
        int l1, l2, l3;
        double w;
        ixc.at(e, l1, l2, l3, w);
        const long ef = tg.fine_of(l1, l2, l3);
        const float m = invreg_factor(sc, l1, l2, l3);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            float2 v = make_float2(0.f, 0.f);
            if (ef >= 0) {
                const float2 u = r[f * Sf + ef];
                v = make_float2(scale * u.x, scale * u.y);
            }
            rc[f * Sc + e] = v;
            sc0[f * Sc + e] = make_float2(m * v.x, m * v.y);
        }
    }
}

// z = (beta0 A)^{-1} r + P (s_c - s_c0) on the fine spectra, and the
// partial sums of <r, z> (sc: the fine symbol)
__global__ __launch_bounds__(256) void k_2l_prolong(const float2 *__restrict__ r, float2 *__restrict__ z, long Sf,
                                                    SpecIdx ixf, const float2 *__restrict__ scs,
                                                    const float2 *__restrict__ sc0, long Sc, TwoGrid tg, float scale,
                                                    SymCtx sc, double *__restrict__ partial, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y);
    if (mb.stopped(mo_)) return;
    r = mshift(r, mo_); z = mshift(z, mo_); scs = mshift(scs, mo_); sc0 = mshift(sc0, mo_);
    partial = mshift(partial, mo_);
    double acc = 0.0, unused = 0.0;
    SPEC_LOOP(Sf)
    {
        int l1, l2, l3;
        double w;
        ixf.at(e, l1, l2, l3, w);
        const long ec = tg.coarse_of(l1, l2, l3);
        const float m = invreg_factor(sc, l1, l2, l3);
        double t = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float2 rv = r[f * Sf + e];
            float2 zv = make_float2(m * rv.x, m * rv.y);
            if (ec >= 0) {
                const float2 a = scs[f * Sc + ec], b = sc0[f * Sc + ec];
                const float2 d = make_float2(a.x - b.x, a.y - b.y);
                zv = make_float2(zv.x + scale * d.x, zv.y + scale * d.y);
            }
            z[f * Sf + e] = zv;
            t += (double)rv.x * zv.x + (double)rv.y * zv.y;
        }
        acc += w * t;
    }
    block_sum2(acc, unused);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}
#undef SPEC_LOOP

static SpecIdx spec_idx(const FftCtx &F)
{
    // 32-bit entry indices (with the grid stride added once past the end)
    if (F.spec_stride >= (1L << 31)) fail(LDDMM_EINVAL, "spectral PCG: more than 2^31 coefficients per field");
    SpecIdx ix;
    ix.nmain = (unsigned)(F.nrow * F.m3);
    ix.m3 = (unsigned)F.m3;
    ix.n2 = (unsigned)F.n2;
    return ix;
}

static float2 *slot_ptr(lddmm_plan *P, int slot) { return reinterpret_cast<float2 *>(P->spec + (long)slot * P->slot_bytes); }

void spec_forward3(lddmm_plan *P, const float *in, int slot0)
{
    RealIn ri{};
    for (int c = 0; c < 3; ++c) ri.p[c] = in + c * P->N;
    r2c_fields(P, ri, 3, slot0, false);
    x2_pass(P, slot0, 3, false, false);
    x1_pass(P, slot0, 3, false, false);
}

void spec_inverse3(lddmm_plan *P, int slot0, float *out, bool x1_done)
{
    if (!x1_done) x1_pass(P, slot0, 3, true, false);
    x2_pass(P, slot0, 3, true, false);
    RealOut ro{};
    for (int c = 0; c < 3; ++c) ro.p[c] = out + c * P->N;
    c2r_fields(P, slot0, 3, ro, (float)(1.0 / (double)P->N));
}

void spcg_assemble(lddmm_plan *P, int bslot, const float2 *p, float2 *q, int kslot, int leray, int after)
{
    const FftCtx &F = P->fft;
    const SymCtx sc = sym_ctx(P, leray);
    {
        Scope s(P, K_VECOP);
        const dim3 g(kRedBlocks, P->mb.count);
        if (sc.leray)
            hipLaunchKernelGGL(k_spec_assemble<true>, g, dim3(256), 0, P->stream, slot_ptr(P, bslot), P->slot_bytes / 8, p,
                               q, F.spec_stride, spec_idx(F), sc, P->red, P->mb);
        else
            hipLaunchKernelGGL(k_spec_assemble<false>, g, dim3(256), 0, P->stream, slot_ptr(P, bslot), P->slot_bytes / 8, p,
                               q, F.spec_stride, spec_idx(F), sc, P->red, P->mb);
        check_hip(hipGetLastError(), "k_spec_assemble");
    }
    if (kslot >= 0) dev_reduce_final_steps(P, P->red, kslot, -1, P->h3 / (double)P->N, after, nullptr);
}

void spcg_start(lddmm_plan *P, const float2 *b, long bstride, float sign, float2 *r, float2 *p, int cslot, int rr_slot,
                int rz_slot)
{
    const FftCtx &F = P->fft;
    {
        Scope s(P, K_VECOP);
        hipLaunchKernelGGL(k_spcg_start, dim3(kRedBlocks, P->mb.count), dim3(256), 0, P->stream, b, bstride, sign, r, p,
                           cslot >= 0 ? slot_ptr(P, cslot) : nullptr, P->slot_bytes / 8, F.spec_stride,
                           spec_idx(F), sym_ctx(P, 0), P->red, P->mb);
        check_hip(hipGetLastError(), "k_spcg_start");
    }
    dev_reduce_final_steps(P, P->red, rr_slot, rz_slot, P->h3 / (double)P->N, 0, nullptr);
}

void spcg_r(lddmm_plan *P, float2 *r, const float2 *q, float2 *x, const float2 *p, int rr_slot, int rz_slot,
            int after, double *hist_dst)
{
    const FftCtx &F = P->fft;
    {
        Scope s(P, K_VECOP);
        hipLaunchKernelGGL(k_spcg_r, dim3(kRedBlocks, P->mb.count), dim3(256), 0, P->stream, r, q, x, p, F.spec_stride,
                           spec_idx(F), sym_ctx(P, 0), (const double *)scalars(P), P->red, P->mb);
        check_hip(hipGetLastError(), "k_spcg_r");
    }
    dev_reduce_final_steps(P, P->red, rr_slot, rz_slot, P->h3 / (double)P->N, after, hist_dst);
}

void spcg_p(lddmm_plan *P, const float2 *r, const float2 *z, float2 *p, int cslot, float2 *sx)
{
    const FftCtx &F = P->fft;
    Scope s(P, K_VECOP);
    hipLaunchKernelGGL(k_spcg_p, dim3(kRedBlocks, P->mb.count), dim3(256), 0, P->stream, r, z, p,
                       cslot >= 0 ? slot_ptr(P, cslot) : nullptr, P->slot_bytes / 8, F.spec_stride, spec_idx(F),
                       sym_ctx(P, 0), (const double *)scalars(P), sx, P->mb);
    check_hip(hipGetLastError(), "k_spcg_p");
}

float2 *spec_slot(lddmm_plan *P, int slot) { return slot_ptr(P, slot); }

static void spec_copy3_raw(lddmm_plan *P, const float2 *src, long sstride, float2 *dst, long dstride, bool inv)
{
    const FftCtx &F = P->fft;
    Scope s(P, K_VECOP);
    hipLaunchKernelGGL(k_spec_copy3, dim3(kRedBlocks, P->mb.count), dim3(256), 0, P->stream, src, sstride, dst, dstride,
                       F.spec_stride, spec_idx(F), sym_ctx(P, 0), inv ? 1 : 0, P->mb);
    check_hip(hipGetLastError(), "k_spec_copy3");
}

void spec_copy3(lddmm_plan *P, const float2 *src, int dst_slot, bool inv)
{
    spec_copy3_raw(P, src, P->fft.spec_stride, slot_ptr(P, dst_slot), P->slot_bytes / 8, inv);
}

void spec_from_slots(lddmm_plan *P, int src_slot, float2 *dst)
{
    spec_copy3_raw(P, slot_ptr(P, src_slot), P->slot_bytes / 8, dst, P->fft.spec_stride, false);
}

void spec_invreg3(lddmm_plan *P, const float2 *src, float2 *dst)
{
    spec_copy3_raw(P, src, P->fft.spec_stride, dst, P->fft.spec_stride, true);
}

void spec_dot(lddmm_plan *P, const float2 *a, const float2 *b, int slot, int after)
{
    const FftCtx &F = P->fft;
    {
        Scope s(P, K_DOT);
        hipLaunchKernelGGL(k_spec_dot, dim3(kRedBlocks, P->mb.count), dim3(256), 0, P->stream, a, b, F.spec_stride,
                           spec_idx(F), P->red, P->mb);
        check_hip(hipGetLastError(), "k_spec_dot");
    }
    dev_reduce_final_steps(P, P->red, slot, -1, P->h3 / (double)P->N, after, nullptr);
}

static TwoGrid two_grid(const FftCtx &F, const FftCtx &C)
{
    return TwoGrid{F.n1, F.n2, F.m3, C.n1, C.n2, C.m3};
}

void two_level_restrict(lddmm_plan *F, const float2 *r, lddmm_plan *C, float2 *rc, float2 *sc0)
{
    const FftCtx &FF = F->fft, &FC = C->fft;
    const float scale = (float)((double)FC.n1 * FC.n2 * FC.n3 / ((double)FF.n1 * FF.n2 * FF.n3));
    Scope s(C, K_PACK);
    hipLaunchKernelGGL(k_2l_restrict, dim3(kRedBlocks, C->mb.count), dim3(256), 0, C->stream, r, FF.spec_stride, rc, sc0,
                       FC.spec_stride, spec_idx(FC), two_grid(FF, FC), scale, sym_ctx(C, 0), C->mb);
    check_hip(hipGetLastError(), "k_2l_restrict");
}

void two_level_prolong(lddmm_plan *F, const float2 *r, float2 *z, lddmm_plan *C, const float2 *scs,
                       const float2 *sc0, int rz_slot, int after)
{
    const FftCtx &FF = F->fft, &FC = C->fft;
    const float scale = (float)((double)FF.n1 * FF.n2 * FF.n3 / ((double)FC.n1 * FC.n2 * FC.n3));
    {
        Scope s(F, K_PACK);
        hipLaunchKernelGGL(k_2l_prolong, dim3(kRedBlocks, F->mb.count), dim3(256), 0, F->stream, r, z, FF.spec_stride,
                           spec_idx(FF), scs, sc0, FC.spec_stride, two_grid(FF, FC), scale, sym_ctx(F, 0), F->red,
                           F->mb);
        check_hip(hipGetLastError(), "k_2l_prolong");
    }
    if (rz_slot >= 0) dev_reduce_final_steps(F, F->red, rz_slot, -1, F->h3 / (double)F->N, after, nullptr);
}

}  // namespace lddmm
