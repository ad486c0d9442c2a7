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
//   x1_symbol: forward x1 pass, pointwise symbol over all fields of the
//              operator, inverse x1 pass -- one HBM round trip instead of three.
//   c2r_x3   : the inverse of r2c_x3, with the output scale folded in.
#include "internal.hpp"

#include <algorithm>
#include <cmath>

namespace lddmm {

// ---------------------------------------------------------------------------
// small DFTs
// ---------------------------------------------------------------------------
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a)  // a * (-i) forward, a * (+i) inverse
{
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
__device__ __forceinline__ void dft_small(float2 *v);

template <>
__device__ __forceinline__ void dft_small<2, false>(float2 *v)
{
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}
template <>
__device__ __forceinline__ void dft_small<2, true>(float2 *v)
{
    dft_small<2, false>(v);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2 &v0, float2 &v1, float2 &v2, float2 &v3)
{
    float2 t0 = cadd(v0, v2), t1 = csub(v0, v2);
    float2 t2 = cadd(v1, v3), t3 = mul_mi<INV>(csub(v1, v3));
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, t3);
    v3 = csub(t1, t3);
}

template <>
__device__ __forceinline__ void dft_small<4, false>(float2 *v)
{
    dft4<false>(v[0], v[1], v[2], v[3]);
}
template <>
__device__ __forceinline__ void dft_small<4, true>(float2 *v)
{
    dft4<true>(v[0], v[1], v[2], v[3]);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2 *v)
{
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    const float r = 0.70710678118654752440f;
    // W8^k, W8 = exp(-+ 2 pi i / 8)
    float2 w1 = INV ? make_float2(r, r) : make_float2(r, -r);
    float2 w3 = INV ? make_float2(-r, r) : make_float2(-r, -r);
    o1 = cmul(o1, w1);
    o2 = mul_mi<INV>(o2);
    o3 = cmul(o3, w3);
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}
template <>
__device__ __forceinline__ void dft_small<8, false>(float2 *v)
{
    dft8<false>(v);
}
template <>
__device__ __forceinline__ void dft_small<8, true>(float2 *v)
{
    dft8<true>(v);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2 *v)
{
    const float s = 0.86602540378443864676f;  // sin(2 pi / 3)
    float2 t = cadd(v[1], v[2]);
    float2 d = csub(v[1], v[2]);
    float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
    float2 sd = mul_mi<INV>(cscale(d, s));  // -+ i s d
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, sd);
    v[2] = csub(m, sd);
}
template <>
__device__ __forceinline__ void dft_small<3, false>(float2 *v)
{
    dft3<false>(v);
}
template <>
__device__ __forceinline__ void dft_small<3, true>(float2 *v)
{
    dft3<true>(v);
}

template <bool INV>
__device__ __forceinline__ void dft5(float2 *v)
{
    const float c1 = 0.30901699437494742410f;   // cos(2 pi/5)
    const float c2 = -0.80901699437494742410f;  // cos(4 pi/5)
    const float s1 = 0.95105651629515357212f;   // sin(2 pi/5)
    const float s2 = 0.58778525229247312917f;   // sin(4 pi/5)
    float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    float2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    float2 a1 = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    float2 a2 = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    float2 b1 = make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
    float2 b2 = make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
    float2 ib1 = mul_mi<INV>(b1), ib2 = mul_mi<INV>(b2);  // -+ i b
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, ib1);
    v[4] = csub(a1, ib1);
    v[2] = cadd(a2, ib2);
    v[3] = csub(a2, ib2);
}
template <>
__device__ __forceinline__ void dft_small<5, false>(float2 *v)
{
    dft5<false>(v);
}
template <>
__device__ __forceinline__ void dft_small<5, true>(float2 *v)
{
    dft5<true>(v);
}

// ---------------------------------------------------------------------------
// Stockham autosort passes in LDS.  An LDS tile holds TW lines of length L;
// element (n, c) of line c sits at n*TW + c (CFAST: the columns are the
// coalesced direction) or at c*LP + n (rows contiguous).
// ---------------------------------------------------------------------------
template <int R, bool INV, bool CFAST>
__device__ __forceinline__ void stockham_pass(const float2 *__restrict__ src, float2 *__restrict__ dst,
                                              int L, int TW, int logTW, int LP, int Ns,
                                              const float2 *__restrict__ tw, int tid, int nthr)
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
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int n = j + r * LR;
            v[r] = src[CFAST ? (n * TW + c) : (c * LP + n)];
        }
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[jm * r * step];
                v[r] = INV ? cmulc(v[r], w) : cmul(v[r], w);
            }
        }
        dft_small<R, INV>(v);
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
template <bool INV, bool CFAST>
__device__ float2 *lds_fft(float2 *A, float2 *B, int TW, int logTW, int LP, const RadixPlan &rp,
                           const float2 *__restrict__ tw, int tid, int nthr)
{
    float2 *s = A, *d = B;
    int Ns = 1;
    const int L = rp.L;
    for (int p = 0; p < rp.np; ++p) {
        const int R = rp.r[p];
        switch (R) {
        case 8: stockham_pass<8, INV, CFAST>(s, d, L, TW, logTW, LP, Ns, tw, tid, nthr); break;
        case 4: stockham_pass<4, INV, CFAST>(s, d, L, TW, logTW, LP, Ns, tw, tid, nthr); break;
        case 2: stockham_pass<2, INV, CFAST>(s, d, L, TW, logTW, LP, Ns, tw, tid, nthr); break;
        case 3: stockham_pass<3, INV, CFAST>(s, d, L, TW, logTW, LP, Ns, tw, tid, nthr); break;
        default: stockham_pass<5, INV, CFAST>(s, d, L, TW, logTW, LP, Ns, tw, tid, nthr); break;
        }
        __syncthreads();
        float2 *t = s;
        s = d;
        d = t;
        Ns *= R;
    }
    return s;
}

constexpr int kFftThreads = 256;

// ---------------------------------------------------------------------------
// x3 pass: real rows -> half spectrum (main + Nyquist plane)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kFftThreads) void k_r2c_x3(RealIn in, float2 *__restrict__ spec,
                                                        long spec_stride, int field0, long nrow,
                                                        int n3, int TWR, RadixPlan rp,
                                                        const float2 *__restrict__ tw_m3,
                                                        const float2 *__restrict__ tw_n3)
{
    extern __shared__ float2 lds[];
    const int m3 = n3 >> 1, LP = m3 + 1;
    float2 *A = lds, *B = lds + TWR * LP;
    const int f = blockIdx.y;
    const float *__restrict__ src = in.p[f];
    const long row0 = (long)blockIdx.x * TWR;
    const int tid = threadIdx.x, nthr = blockDim.x;
    float *Af = reinterpret_cast<float *>(A);
    for (int idx = tid; idx < TWR * n3; idx += nthr) {
        const int c = idx / n3, x = idx - c * n3;
        const long row = row0 + c;
        Af[(c * LP + (x >> 1)) * 2 + (x & 1)] = row < nrow ? src[row * n3 + x] : 0.f;
    }
    __syncthreads();
    const float2 *Z = lds_fft<false, false>(A, B, TWR, 0, LP, rp, tw_m3, tid, nthr);
    float2 *outm = spec + (long)(field0 + f) * spec_stride;
    float2 *outq = outm + nrow * m3;
    for (int idx = tid; idx < TWR * (m3 + 1); idx += nthr) {
        const int c = idx / (m3 + 1), k = idx - c * (m3 + 1);
        const long row = row0 + c;
        if (row >= nrow) continue;
        const float2 zk = Z[c * LP + (k == m3 ? 0 : k)];
        const float2 zc = cconj(Z[c * LP + (k == 0 ? 0 : m3 - k)]);
        const float2 E = cscale(cadd(zk, zc), 0.5f);
        const float2 D = cscale(csub(zk, zc), 0.5f);
        const float2 O = make_float2(D.y, -D.x);  // D / i
        const float2 X = cadd(E, cmul(tw_n3[k], O));
        if (k < m3)
            outm[row * m3 + k] = X;
        else
            outq[row] = X;
    }
}

// ---------------------------------------------------------------------------
// x3 pass: half spectrum -> real rows, times scale
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kFftThreads) void k_c2r_x3(const float2 *__restrict__ spec,
                                                        long spec_stride, int field0, RealOut out,
                                                        long nrow, int n3, int TWR, RadixPlan rp,
                                                        const float2 *__restrict__ tw_m3,
                                                        const float2 *__restrict__ tw_n3,
                                                        float scale)
{
    extern __shared__ float2 lds[];
    const int m3 = n3 >> 1, LP = m3 + 1;
    float2 *A = lds, *B = lds + TWR * LP;
    const int f = blockIdx.y;
    const long row0 = (long)blockIdx.x * TWR;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const float2 *inm = spec + (long)(field0 + f) * spec_stride;
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
        const float2 Xc = cconj(B[c * LP + m3 - k]);
        const float2 E = cadd(Xk, Xc);
        const float2 O = cmulc(csub(Xk, Xc), tw_n3[k]);  // * exp(+2 pi i k / n3)
        A[c * LP + k] = cadd(E, cmuli(O));
    }
    __syncthreads();
    const float2 *z = lds_fft<true, false>(A, B, TWR, 0, LP, rp, tw_m3, tid, nthr);
    float *__restrict__ dst = out.p[f];
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
    long base_off;  // offset of the sub-array (main: 0, Nyquist plane: nrow*m3)
    long ostride;   // stride between outer indices (blockIdx.y)
    long nstride;   // stride along the transformed line
    long cstride;   // stride between columns
    int ncols;      // columns per outer index
};

template <bool INV>
__global__ __launch_bounds__(kFftThreads) void k_fft_cols(float2 *__restrict__ data, long fstride,
                                                          int field0, ColDesc d, int TW, int logTW,
                                                          RadixPlan rp,
                                                          const float2 *__restrict__ tw)
{
    extern __shared__ float2 lds[];
    const int L = rp.L;
    float2 *A = lds, *B = lds + L * TW;
    const int tid = threadIdx.x, nthr = blockDim.x;
    float2 *base = data + (long)(field0 + blockIdx.z) * fstride + d.base_off +
                   (long)blockIdx.y * d.ostride;
    const int col0 = blockIdx.x * TW;
    for (int idx = tid; idx < L * TW; idx += nthr) {
        const int n = idx >> logTW, c = idx & (TW - 1);
        const int col = col0 + c;
        A[idx] = col < d.ncols ? base[n * d.nstride + col * d.cstride] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const float2 *res = lds_fft<INV, true>(A, B, TW, logTW, 0, rp, tw, tid, nthr);
    for (int idx = tid; idx < L * TW; idx += nthr) {
        const int n = idx >> logTW, c = idx & (TW - 1);
        const int col = col0 + c;
        if (col < d.ncols) base[n * d.nstride + col * d.cstride] = res[idx];
    }
}

// ---------------------------------------------------------------------------
// Spectral symbols.  l1, l2, l3: indices of the spectral point (k3 index
// l3 in [0, n3/2]).  scale = 1/N folds the inverse normalisation in.
// ---------------------------------------------------------------------------
struct SymCtx {
    int n1, n2, n3;
    float scale, beta;
    int reg, leray;
};

__device__ __forceinline__ float wn_full(int l, int n) { return (float)(l <= (n >> 1) ? l : l - n); }
__device__ __forceinline__ float wn_odd(int l, int n)
{
    return (2 * l == n) ? 0.f : (float)(l <= (n >> 1) ? l : l - n);
}

__device__ __forceinline__ float reg_symbol(const SymCtx &s, int l1, int l2, int l3)
{
    const float k1 = wn_full(l1, s.n1), k2 = wn_full(l2, s.n2), k3 = wn_full(l3, s.n3);
    const float kk = k1 * k1 + k2 * k2 + k3 * k3;
    return s.reg == 2 ? kk * kk : kk;
}

__device__ __forceinline__ void leray_apply(const SymCtx &s, int l1, int l2, int l3, float2 *w)
{
    const float k[3] = {wn_odd(l1, s.n1), wn_odd(l2, s.n2), wn_odd(l3, s.n3)};
    const float kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (kk > 0.f) {
        const float ikk = 1.f / kk;
        const float2 kw = make_float2((k[0] * w[0].x + k[1] * w[1].x + k[2] * w[2].x) * ikk,
                                      (k[0] * w[0].y + k[1] * w[1].y + k[2] * w[2].y) * ikk);
#pragma unroll
        for (int c = 0; c < 3; ++c) w[c] = make_float2(w[c].x - k[c] * kw.x, w[c].y - k[c] * kw.y);
    }
}

struct OpGrad {
    static constexpr int NIN = 1, NOUT = 3;
    __device__ void operator()(const SymCtx &s, int l1, int l2, int l3, const float2 *in,
                               float2 *out) const
    {
        const float k[3] = {wn_odd(l1, s.n1), wn_odd(l2, s.n2), wn_odd(l3, s.n3)};
        const float2 f = cscale(in[0], s.scale);
#pragma unroll
        for (int d = 0; d < 3; ++d) out[d] = cmuli(cscale(f, k[d]));
    }
};

struct OpDiv {
    static constexpr int NIN = 3, NOUT = 1;
    __device__ void operator()(const SymCtx &s, int l1, int l2, int l3, const float2 *in,
                               float2 *out) const
    {
        const float k[3] = {wn_odd(l1, s.n1), wn_odd(l2, s.n2), wn_odd(l3, s.n3)};
        float2 acc = make_float2(k[0] * in[0].x + k[1] * in[1].x + k[2] * in[2].x,
                                 k[0] * in[0].y + k[1] * in[1].y + k[2] * in[2].y);
        out[0] = cmuli(cscale(acc, s.scale));
    }
};

struct OpReg {
    static constexpr int NIN = 3, NOUT = 3;
    __device__ void operator()(const SymCtx &s, int l1, int l2, int l3, const float2 *in,
                               float2 *out) const
    {
        const float a = reg_symbol(s, l1, l2, l3) * s.scale;
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = cscale(in[c], a);
    }
};

struct OpInvReg {
    static constexpr int NIN = 3, NOUT = 3;
    __device__ void operator()(const SymCtx &s, int l1, int l2, int l3, const float2 *in,
                               float2 *out) const
    {
        const float a = reg_symbol(s, l1, l2, l3);
        const float f = (a == 0.f ? 1.f / s.beta : 1.f / (s.beta * a)) * s.scale;
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = cscale(in[c], f);
    }
};

struct OpLeray {
    static constexpr int NIN = 3, NOUT = 3;
    __device__ void operator()(const SymCtx &s, int l1, int l2, int l3, const float2 *in,
                               float2 *out) const
    {
        float2 w[3] = {in[0], in[1], in[2]};
        leray_apply(s, l1, l2, l3, w);
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = cscale(w[c], s.scale);
    }
};

// beta A w + K b (K = Leray if s.leray): inputs w0..w2, b0..b2
struct OpAssemble {
    static constexpr int NIN = 6, NOUT = 3;
    __device__ void operator()(const SymCtx &s, int l1, int l2, int l3, const float2 *in,
                               float2 *out) const
    {
        const float a = s.beta * reg_symbol(s, l1, l2, l3);
        float2 b[3] = {in[3], in[4], in[5]};
        if (s.leray) leray_apply(s, l1, l2, l3, b);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            out[c] = make_float2((a * in[c].x + b[c].x) * s.scale, (a * in[c].y + b[c].y) * s.scale);
    }
};

struct OpIdent {
    static constexpr int NIN = 1, NOUT = 1;
    __device__ void operator()(const SymCtx &s, int, int, int, const float2 *in, float2 *out) const
    {
        out[0] = cscale(in[0], s.scale);
    }
};

// x1 forward -> symbol -> x1 inverse.  nyq = 0: main array, columns are k3
// and blockIdx.y is k2; nyq = 1: Nyquist plane, columns are k2, k3 = n3/2.
template <class Op>
__global__ __launch_bounds__(kFftThreads) void k_x1_symbol(const float2 *__restrict__ in, int in_first,
                                                           float2 *__restrict__ out, int out_first,
                                                           long fstride, ColDesc d, int nyq, int TW,
                                                           int logTW, RadixPlan rp,
                                                           const float2 *__restrict__ tw, SymCtx sc,
                                                           Op op)
{
    constexpr int NF = Op::NIN > Op::NOUT ? Op::NIN : Op::NOUT;
    extern __shared__ float2 lds[];
    const int L = rp.L;
    const int tile = L * TW;
    float2 *S = lds + NF * tile;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int col0 = blockIdx.x * TW;
    const long off = d.base_off + (long)blockIdx.y * d.ostride;
    const bool odd = rp.np & 1;
    for (int f = 0; f < Op::NIN; ++f) {
        const float2 *src = in + (long)(in_first + blockIdx.z * Op::NIN + f) * fstride + off;
        float2 *buf = lds + f * tile;
        float2 *first = odd ? S : buf;
        for (int idx = tid; idx < tile; idx += nthr) {
            const int n = idx >> logTW, c = idx & (TW - 1);
            const int col = col0 + c;
            first[idx] = col < d.ncols ? src[n * d.nstride + col * d.cstride] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        lds_fft<false, true>(first, odd ? buf : S, TW, logTW, 0, rp, tw, tid, nthr);
    }
    for (int idx = tid; idx < tile; idx += nthr) {
        const int n = idx >> logTW, c = idx & (TW - 1);
        const int col = col0 + c;
        if (col >= d.ncols) continue;
        const int l2 = nyq ? col : (int)blockIdx.y;
        const int l3 = nyq ? (sc.n3 >> 1) : col;
        float2 vin[Op::NIN], vout[Op::NOUT];
#pragma unroll
        for (int f = 0; f < Op::NIN; ++f) vin[f] = lds[f * tile + idx];
        op(sc, n, l2, l3, vin, vout);
#pragma unroll
        for (int o = 0; o < Op::NOUT; ++o) lds[o * tile + idx] = vout[o];
    }
    __syncthreads();
    for (int o = 0; o < Op::NOUT; ++o) {
        float2 *buf = lds + o * tile;
        const float2 *res = lds_fft<true, true>(buf, S, TW, logTW, 0, rp, tw, tid, nthr);
        float2 *dst = out + (long)(out_first + blockIdx.z * Op::NOUT + o) * fstride + off;
        for (int idx = tid; idx < tile; idx += nthr) {
            const int n = idx >> logTW, c = idx & (TW - 1);
            const int col = col0 + c;
            if (col < d.ncols) dst[n * d.nstride + col * d.cstride] = res[idx];
        }
        __syncthreads();
    }
}

// standard half-spectrum layout <-> internal layout
__global__ void k_pack_standard(const float2 *__restrict__ spec, float2 *__restrict__ dst, long nrow,
                                int m3)
{
    const long total = nrow * (m3 + 1);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long)gridDim.x * blockDim.x) {
        const long row = i / (m3 + 1);
        const int k = (int)(i - row * (m3 + 1));
        dst[i] = k < m3 ? spec[row * m3 + k] : spec[nrow * m3 + row];
    }
}

__global__ void k_unpack_standard(const float2 *__restrict__ srcp, float2 *__restrict__ spec,
                                  long nrow, int m3)
{
    const long total = nrow * (m3 + 1);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long)gridDim.x * blockDim.x) {
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

static float2 *upload_twiddles(int L, int count)
{
    std::vector<float2> h(count);
    for (int m = 0; m < count; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)L;
        h[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    float2 *d = nullptr;
    check_hip(hipMalloc(&d, sizeof(float2) * count), "hipMalloc twiddles");
    check_hip(hipMemcpy(d, h.data(), sizeof(float2) * count, hipMemcpyHostToDevice), "twiddle upload");
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
    F.rp3 = make_radix_plan(F.m3 > 1 ? F.m3 : 1);
    F.tw1 = upload_twiddles(F.n1, F.n1);
    F.tw2 = upload_twiddles(F.n2, F.n2);
    F.tw3 = upload_twiddles(F.m3, F.m3);
    F.twN3 = upload_twiddles(F.n3, F.n3);
}

void fft_free(lddmm_plan *P)
{
    FftCtx &F = P->fft;
    for (float2 *p : {F.tw1, F.tw2, F.tw3, F.twN3})
        if (p) (void)hipFree(p);
    F.tw1 = F.tw2 = F.tw3 = F.twN3 = nullptr;
}

static constexpr size_t kLdsBudget = 64 * 1024;

static int floor_pow2(long x)
{
    int p = 1;
    while ((long)p * 2 <= x) p *= 2;
    return p;
}

static int rows_per_block(int m3)
{
    // two buffers of TWR * (m3 + 1) float2
    long cap = (long)(kLdsBudget / (2 * sizeof(float2) * (m3 + 1)));
    int t = floor_pow2(cap < 1 ? 1 : cap);
    return t > 32 ? 32 : t;
}

static int col_tile(int L, int nbuf, int ncols)
{
    long cap = (long)(kLdsBudget / ((size_t)nbuf * sizeof(float2) * L));
    int t = floor_pow2(cap < 1 ? 1 : cap);
    if (t > 32) t = 32;
    int nc = floor_pow2(ncols);
    if (nc < ncols) nc *= 2;
    if (t > nc) t = nc;
    return t;
}

static int ilog2(int x)
{
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

void r2c_fields(lddmm_plan *P, const RealIn &in, int count, int spec_first)
{
    FftCtx &F = P->fft;
    const int TWR = rows_per_block(F.m3);
    const size_t lds = 2 * sizeof(float2) * TWR * (F.m3 + 1);
    dim3 grid((unsigned)((F.nrow + TWR - 1) / TWR), count);
    Scope s(P, K_R2C_X3);
    hipLaunchKernelGGL(k_r2c_x3, grid, dim3(kFftThreads), lds, P->stream, in, P->spec,
                       F.spec_stride, spec_first, F.nrow, F.n3, TWR, F.rp3, F.tw3, F.twN3);
    check_hip(hipGetLastError(), "k_r2c_x3");
}

void c2r_fields(lddmm_plan *P, int spec_first, int count, const RealOut &out, float scale)
{
    FftCtx &F = P->fft;
    const int TWR = rows_per_block(F.m3);
    const size_t lds = 2 * sizeof(float2) * TWR * (F.m3 + 1);
    dim3 grid((unsigned)((F.nrow + TWR - 1) / TWR), count);
    Scope s(P, K_C2R_X3);
    hipLaunchKernelGGL(k_c2r_x3, grid, dim3(kFftThreads), lds, P->stream, P->spec, F.spec_stride,
                       spec_first, out, F.nrow, F.n3, TWR, F.rp3, F.tw3, F.twN3, scale);
    check_hip(hipGetLastError(), "k_c2r_x3");
}

// column descriptors: main array and Nyquist plane, along x2 (axis 1) or x1 (axis 0)
static void col_descs(const FftCtx &F, int axis, ColDesc &dm, ColDesc &dq, int &outer_m, int &outer_q)
{
    if (axis == 1) {
        dm = {0, (long)F.n2 * F.m3, F.m3, 1, F.m3};
        outer_m = F.n1;
        dq = {F.nrow * F.m3, 0, 1, F.n2, F.n1};
        outer_q = 1;
    } else {
        dm = {0, F.m3, (long)F.n2 * F.m3, 1, F.m3};
        outer_m = F.n2;
        dq = {F.nrow * F.m3, 0, F.n2, 1, F.n2};
        outer_q = 1;
    }
}

static void cols_pass(lddmm_plan *P, int axis, int spec_first, int count, bool inverse)
{
    FftCtx &F = P->fft;
    const RadixPlan &rp = axis == 1 ? F.rp2 : F.rp1;
    const float2 *tw = axis == 1 ? F.tw2 : F.tw1;
    ColDesc dm, dq;
    int om, oq;
    col_descs(F, axis, dm, dq, om, oq);
    for (int part = 0; part < 2; ++part) {
        const ColDesc &d = part == 0 ? dm : dq;
        const int outer = part == 0 ? om : oq;
        const int TW = col_tile(rp.L, 2, d.ncols);
        const size_t lds = 2 * sizeof(float2) * rp.L * TW;
        dim3 grid((unsigned)((d.ncols + TW - 1) / TW), outer, count);
        Scope s(P, K_FFT_COLS);
        if (inverse)
            hipLaunchKernelGGL(k_fft_cols<true>, grid, dim3(kFftThreads), lds, P->stream, P->spec,
                               F.spec_stride, spec_first, d, TW, ilog2(TW), rp, tw);
        else
            hipLaunchKernelGGL(k_fft_cols<false>, grid, dim3(kFftThreads), lds, P->stream, P->spec,
                               F.spec_stride, spec_first, d, TW, ilog2(TW), rp, tw);
        check_hip(hipGetLastError(), "k_fft_cols");
    }
}

void x2_pass(lddmm_plan *P, int spec_first, int count, bool inverse)
{
    cols_pass(P, 1, spec_first, count, inverse);
}

void x1_pass(lddmm_plan *P, int spec_first, int count, bool inverse)
{
    cols_pass(P, 0, spec_first, count, inverse);
}

int op_nin(int op)
{
    switch (op) {
    case SOP_GRAD: return 1;
    case SOP_DIV: return 3;
    case SOP_ASSEMBLE: return 6;
    case SOP_IDENT: return 1;
    default: return 3;
    }
}

int op_nout(int op)
{
    switch (op) {
    case SOP_GRAD: return 3;
    case SOP_DIV: return 1;
    case SOP_IDENT: return 1;
    default: return 3;
    }
}

template <class Op>
static void launch_x1_symbol(lddmm_plan *P, int spec_in, int spec_out, int nbatch, const SymCtx &sc)
{
    FftCtx &F = P->fft;
    constexpr int NF = Op::NIN > Op::NOUT ? Op::NIN : Op::NOUT;
    ColDesc dm, dq;
    int om, oq;
    col_descs(F, 0, dm, dq, om, oq);
    for (int part = 0; part < 2; ++part) {
        const ColDesc &d = part == 0 ? dm : dq;
        const int outer = part == 0 ? om : oq;
        const int TW = col_tile(F.rp1.L, NF + 1, d.ncols);
        const size_t lds = (size_t)(NF + 1) * sizeof(float2) * F.rp1.L * TW;
        dim3 grid((unsigned)((d.ncols + TW - 1) / TW), outer, nbatch);
        Scope s(P, K_SPECTRAL_X1);
        hipLaunchKernelGGL(k_x1_symbol<Op>, grid, dim3(kFftThreads), lds, P->stream, P->spec,
                           spec_in, P->spec, spec_out, F.spec_stride, d, part, TW, ilog2(TW), F.rp1,
                           F.tw1, sc, Op{});
        check_hip(hipGetLastError(), "k_x1_symbol");
    }
}

void x1_symbol(lddmm_plan *P, int op, int spec_in, int spec_out, int nbatch, int leray)
{
    FftCtx &F = P->fft;
    SymCtx sc;
    sc.n1 = F.n1;
    sc.n2 = F.n2;
    sc.n3 = F.n3;
    sc.scale = (float)(1.0 / ((double)F.n1 * F.n2 * F.n3));
    sc.beta = (float)P->cfg.beta;
    sc.reg = P->cfg.reg;
    sc.leray = leray;
    switch (op) {
    case SOP_GRAD: launch_x1_symbol<OpGrad>(P, spec_in, spec_out, nbatch, sc); break;
    case SOP_DIV: launch_x1_symbol<OpDiv>(P, spec_in, spec_out, nbatch, sc); break;
    case SOP_REG: launch_x1_symbol<OpReg>(P, spec_in, spec_out, nbatch, sc); break;
    case SOP_INVREG: launch_x1_symbol<OpInvReg>(P, spec_in, spec_out, nbatch, sc); break;
    case SOP_LERAY: launch_x1_symbol<OpLeray>(P, spec_in, spec_out, nbatch, sc); break;
    case SOP_ASSEMBLE: launch_x1_symbol<OpAssemble>(P, spec_in, spec_out, nbatch, sc); break;
    case SOP_IDENT: launch_x1_symbol<OpIdent>(P, spec_in, spec_out, nbatch, sc); break;
    default: fail(LDDMM_EINVAL, "unknown spectral operator");
    }
}

// Apply a spectral operator to real fields.  The real inputs are grouped in
// batches of op_nin(op) fields; batches are processed in chunks that fit the
// plan's spectral scratch (input slots followed by output slots).
void spectral_apply(lddmm_plan *P, int op, const std::vector<const float *> &in,
                    const std::vector<float *> &out)
{
    const int nin = op_nin(op), nout = op_nout(op);
    const int nbatch = (int)in.size() / nin;
    if ((int)in.size() != nbatch * nin || (int)out.size() != nbatch * nout)
        fail(LDDMM_EINVAL, "spectral_apply: field count mismatch");
    const int per = nin + nout;
    int chunk = P->nspec / per;
    if (chunk < 1) fail(LDDMM_EINVAL, "spectral scratch too small");
    for (int b0 = 0; b0 < nbatch; b0 += chunk) {
        const int nb = std::min(chunk, nbatch - b0);
        const int fin = nb * nin, fout = nb * nout;
        for (int f0 = 0; f0 < fin; f0 += 8) {
            RealIn ri{};
            const int cnt = std::min(8, fin - f0);
            for (int i = 0; i < cnt; ++i) ri.p[i] = in[(size_t)b0 * nin + f0 + i];
            r2c_fields(P, ri, cnt, f0);
        }
        x2_pass(P, 0, fin, false);
        x1_symbol(P, op, 0, fin, nb, P->cfg.leray);
        x2_pass(P, fin, fout, true);
        for (int f0 = 0; f0 < fout; f0 += 8) {
            RealOut ro{};
            const int cnt = std::min(8, fout - f0);
            for (int i = 0; i < cnt; ++i) ro.p[i] = out[(size_t)b0 * nout + f0 + i];
            c2r_fields(P, fin + f0, cnt, ro, 1.0f);
        }
    }
}

void pack_standard(lddmm_plan *P, int spec_field, float2 *dst)
{
    FftCtx &F = P->fft;
    Scope s(P, K_PACK);
    hipLaunchKernelGGL(k_pack_standard, dim3(1024), dim3(256), 0, P->stream,
                       P->spec + (long)spec_field * F.spec_stride, dst, F.nrow, F.m3);
    check_hip(hipGetLastError(), "k_pack_standard");
}

void unpack_standard(lddmm_plan *P, const float2 *srcp, int spec_field)
{
    FftCtx &F = P->fft;
    Scope s(P, K_PACK);
    hipLaunchKernelGGL(k_unpack_standard, dim3(1024), dim3(256), 0, P->stream, srcp,
                       P->spec + (long)spec_field * F.spec_stride, F.nrow, F.m3);
    check_hip(hipGetLastError(), "k_unpack_standard");
}

}  // namespace lddmm
