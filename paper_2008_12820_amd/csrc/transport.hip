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

// Division of a point index by n3 and n2 with one multiply-high: for
// 0 <= p < 2^31 and sh = ceil(log2 d), mag = floor(2^(31+sh)/d) + 1,
// floor(p/d) = (p*mag) >> (31+sh) exactly (Granlund and Montgomery, "Division
// by invariant integers using multiplication", 1994, Theorem 4.2 with N = 31).
struct Divider {
    unsigned mag, sh;  // sh >= 1 (d >= 2)
};

struct Grid3 {
    int n1, n2, n3;
    int N;
    Divider by3, by2;
};

__device__ __forceinline__ unsigned divide(unsigned p, Divider d)
{
    return __umulhi(p, d.mag) >> (d.sh - 1);
}

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
    return xcd_block((int)blockIdx.x, (int)gridDim.x) * kPtThreads + (int)threadIdx.x;
}

__device__ __forceinline__ void point_coords(const Grid3 &g, int p, int &i, int &j, int &k)
{
    const unsigned r = divide((unsigned)p, g.by3);
    k = p - (int)r * g.n3;
    const unsigned q = divide(r, g.by2);
    j = (int)r - (int)q * g.n2;
    i = (int)q;
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
    if ((unsigned)(b + n) < (unsigned)(3 * n)) {  // |displacement| below n: one wrap
        b = b < 0 ? b + n : b;
        b = b >= n ? b - n : b;
    } else {
        b %= n;
        if (b < 0) b += n;
    }
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

// Separable evaluation of the tensor-product sum, with one rounding sequence
// shared by every gather strategy: each stencil row is contracted along x3
// by explicit fused multiply-adds, rows along x2, then planes along x1.
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class T>
__device__ __forceinline__ T row3(T f0, T f1, T f2, T f3, const T w[4])
{
    return fma_(f3, w[3], fma_(f2, w[2], fma_(f1, w[1], f0 * w[0])));
}
template <class T>
__device__ __forceinline__ T accum(int i, const T w[4], T r, T acc)
{
    return i == 0 ? w[0] * r : fma_(w[i], r, acc);
}

// When the four x3 nodes are contiguous (no periodic wrap) their loads come
// from one row pointer and merge into one 16-byte load.
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
                acc2 = accum<T>(b, s.w2, row3<T>((T)row[0], (T)row[1], (T)row[2], (T)row[3], s.w3), acc2);
            }
            acc = accum<T>(a, s.w1, acc2, acc);
        }
    } else {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            T acc2 = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float *row = f + (s.o1[a] + s.o2[b]);
                acc2 = accum<T>(b, s.w2,
                                row3<T>((T)row[s.o3[0]], (T)row[s.o3[1]], (T)row[s.o3[2]], (T)row[s.o3[3]], s.w3),
                                acc2);
            }
            acc = accum<T>(a, s.w1, acc2, acc);
        }
    }
    return acc;
}

// First-order (trilinear) interpolation, d = 1 in the Section 3.1 formula:
// nodes floor(u) and floor(u) + 1 per axis, weights 1 - t and t.
template <class T>
struct Stencil2 {
    unsigned o1[2], o2[2], o3[2];
    T w1[2], w2[2], w3[2];
};

template <class T>
__device__ __forceinline__ void axis_stencil2(int i, T d, int n, unsigned stride, unsigned o[2], T w[2])
{
    const T lim = (T)1048576;
    d = d > lim ? lim : d;
    d = d >= -lim ? d : -lim;
    const T fl = floor(d);
    int b = i + (int)fl;
    if ((unsigned)(b + n) < (unsigned)(3 * n)) {
        b = b < 0 ? b + n : b;
        b = b >= n ? b - n : b;
    } else {
        b %= n;
        if (b < 0) b += n;
    }
    o[0] = (unsigned)b * stride;
    o[1] = (unsigned)(b + 1 == n ? 0 : b + 1) * stride;
    const T t = d - fl;
    w[0] = T(1) - t;
    w[1] = t;
}

template <class T>
__device__ __forceinline__ void make_stencil2(const Grid3 &g, int i, int j, int k, T d1, T d2, T d3,
                                              Stencil2<T> &s)
{
    axis_stencil2<T>(i, d1, g.n1, (unsigned)g.n2 * (unsigned)g.n3, s.o1, s.w1);
    axis_stencil2<T>(j, d2, g.n2, (unsigned)g.n3, s.o2, s.w2);
    axis_stencil2<T>(k, d3, g.n3, 1u, s.o3, s.w3);
}

// x3 pairs, then x2, then x1, with explicit fused multiply-adds
template <class T>
__device__ __forceinline__ T gather2(const float *__restrict__ f, const Stencil2<T> &s)
{
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        T acc2 = T(0);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const float *row = f + (s.o1[a] + s.o2[b]);
            const T r = fma_((T)row[s.o3[1]], s.w3[1], (T)row[s.o3[0]] * s.w3[0]);
            acc2 = b == 0 ? s.w2[0] * r : fma_(s.w2[1], r, acc2);
        }
        acc = a == 0 ? s.w1[0] * acc2 : fma_(s.w1[1], acc2, acc);
    }
    return acc;
}

// ---------------------------------------------------------------------------
// departure points, FP64:  X = x - dt/2 (v(x) + I[v](x - dt v(x)))
//                          Xa = x + dt/2 (v(x) + I[v](x + dt v(x)))
// stored as displacements in voxels
// ---------------------------------------------------------------------------
template <int ORDER>
__global__ __launch_bounds__(kPtThreads) void k_departure(const float *__restrict__ v,
                                                          float *__restrict__ dX,
                                                          float *__restrict__ dXa, Grid3 g, double dt,
                                                          double ih1, double ih2, double ih3, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); v = mshift(v, mo_); dX = mshift(dX, mo_); dXa = mshift(dXa, mo_);
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
        float *out = dir == 0 ? dX : dXa;
        if constexpr (ORDER == 1) {
            Stencil2<double> s;
            make_stencil2<double>(g, i, j, k, sgn * dt * vx[0] * ih[0], sgn * dt * vx[1] * ih[1],
                                  sgn * dt * vx[2] * ih[2], s);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double vi = gather2<double>(v + (long)c * g.N, s);
                out[(long)c * g.N + p] = (float)(sgn * 0.5 * dt * (vx[c] + vi) * ih[c]);
            }
        } else {
            Stencil<double> s;
            make_stencil<double>(g, i, j, k, sgn * dt * vx[0] * ih[0], sgn * dt * vx[1] * ih[1],
                                 sgn * dt * vx[2] * ih[2], s);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double vi = gather<double>(v + (long)c * g.N, s);
                out[(long)c * g.N + p] = (float)(sgn * 0.5 * dt * (vx[c] + vi) * ih[c]);
            }
        }
    }
}

// b = dt * sum_j w_j lam_j G_j (trapezoid, w_0 = w_nt = 1/2); lam_nt is read
// from lamN times scaleN, lam_0..lam_{nt-1} from lam.  Four points per thread
// (16-byte accesses); NTC > 0 fixes nt at compile time so that every load of
// the sum is in flight at once.
__device__ __forceinline__ float4 f4fma(float a, float4 x, float4 y)
{
    return make_float4(a * x.x + y.x, a * x.y + y.y, a * x.z + y.z, a * x.w + y.w);
}
__device__ __forceinline__ float4 f4mul(float4 x, float4 y)
{
    return make_float4(x.x * y.x, x.y * y.y, x.z * y.z, x.w * y.w);
}
__device__ __forceinline__ float4 f4scl(float a, float4 x) { return make_float4(a * x.x, a * x.y, a * x.z, a * x.w); }
__device__ __forceinline__ float4 f4add(float4 x, float4 y)
{
    return make_float4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
}

template <int NTC>
__global__ __launch_bounds__(kPtThreads) void k_body_force(const float4 *__restrict__ lam,
                                                           const float4 *__restrict__ lamN, float scaleN,
                                                           const float4 *__restrict__ G, float4 *__restrict__ b,
                                                           long N4, int nt_rt, float dt, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); lam = mshift(lam, mo_); lamN = mshift(lamN, mo_); G = mshift(G, mo_); b = mshift(b, mo_);
    if (mb.stopped(mo_)) return;
    const int nt = NTC > 0 ? NTC : nt_rt;
    const long p = (long)xcd_block((int)blockIdx.x, (int)gridDim.x) * kPtThreads + threadIdx.x;
    if (p >= N4) return;
    float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0, a2 = a0;
#pragma unroll
    for (int j = 0; j <= nt; ++j) {
        const float w = (j == 0 || j == nt) ? 0.5f : 1.f;
        const float4 l = j == nt ? f4scl(scaleN * w, lamN[p]) : f4scl(w, lam[(long)j * N4 + p]);
        const float4 *gj = G + (long)j * 3 * N4;
        a0 = f4add(a0, f4mul(l, gj[p]));
        a1 = f4add(a1, f4mul(l, gj[N4 + p]));
        a2 = f4add(a2, f4mul(l, gj[2 * N4 + p]));
    }
    b[p] = f4scl(dt, a0);
    b[N4 + p] = f4scl(dt, a1);
    b[2 * N4 + p] = f4scl(dt, a2);
}

// Incremental-state sources from the increment vt and its values vX at the
// departure points: s_j = vX . I[G_j](X) + vt . G_{j+1}; m~_1 = -dt/2 s_0 and
// s_1 .. s_{nt-1} are stored.  Four points per thread (16-byte accesses).

// ---------------------------------------------------------------------------
// Box gathers.  A 256-thread workgroup owns an output tile of T1 x T2 rows of
// 64 x3 points; wavefront w takes the rows w, w + 4, ... (PPT points per
// thread).  The workgroup reduces the stencil extents of its points and
// stages that box of every source field, periodically wrapped, in LDS with
// coalesced row loads; the stencils are then read from LDS, where nodes never
// wrap.  The box capacity is fixed, (T1+3+H) x (T2+3+H) rows of kPad3 floats:
// a point whose stencil is not inside the staged box (displacements varying
// across the tile by more than H voxels along x1 or x2, or by more than
// kPad3 - 67 along x3) gathers from global memory instead.
// ---------------------------------------------------------------------------
constexpr int kT3 = 64;    // tile extent along x3 (one wavefront)
// Half tiles: where the last x3 tile of a row would hold at most 32 points
// (n3 mod 64 in (0, 32], e.g. n3 = 96, 160), tiles are 32 points wide and a
// wavefront takes two rows at a time (lanes 0-31 one row, lanes 32-63 the
// row PPT/2 iterations further), so no tile leaves half its lanes idle.
__host__ __device__ constexpr bool half_tiles_for(int n3) { return n3 % 64 != 0 && n3 % 64 <= 32; }
template <bool HALF>
struct TileMap {
    static constexpr int W3 = HALF ? 32 : kT3;  // x3 points per tile
    // x3 index of a lane's points in tile column t3
    __device__ static int k_of(int t3, int lane) { return t3 * W3 + (HALF ? (lane & 31) : lane); }
    // the tile row (e = 0 .. T1 T2 - 1) of a lane's point q (q < NQ)
    __device__ static int row_of(int w, int q, int lane, int nq) { return w + 4 * (HALF ? q + (lane >> 5) * nq : q); }
};
constexpr int kBoxH = 1;   // tolerated spread of floor(d) across the tile, x1 and x2
constexpr int kPad3 = 72;  // box row pitch along x3 (floats)

template <int T1, int T2>
struct BoxCfg {
    static constexpr int PPT = T1 * T2 / 4;  // points per thread
    static constexpr int BR1 = T1 + 3 + kBoxH, BR2 = T2 + 3 + kBoxH;
    static constexpr int CAP = BR1 * BR2 * kPad3;  // floats per field
};

// periodic wrap of any index: one step for [-n, 2n), a modulo beyond
__device__ __forceinline__ int wrapg(int x, int n)
{
    if ((unsigned)(x + n) < (unsigned)(3 * n)) {
        x = x < 0 ? x + n : x;
        return x >= n ? x - n : x;
    }
    x %= n;
    return x < 0 ? x + n : x;
}

// Direct global-to-LDS load of one dword per active lane: lane l's value
// lands at lds + l (the row base is wave-uniform), with no register round
// trip; completion is tracked by the vector-memory counter, so a wait on it
// precedes the barrier that publishes the box.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;
__device__ __forceinline__ void load_to_lds(const float *g, float *lds)
{
    __builtin_amdgcn_global_load_lds((glb_void_t *)const_cast<float *>(g), (lds_void_t *)lds, 4, 0, 0);
}
__device__ __forceinline__ void wait_lds_loads() { __builtin_amdgcn_s_waitcnt(0); }

// Stage the periodic box [L1, L1 + B1) x [L2, L2 + B2) x [L3, L3 + B3) of src
// into LDS rows of kPad3 floats, row (a, b) at box + (a BR2 + b) kPad3.  With
// BR2 = 8 rows per x1 plane, wavefront w stages the x2 rows w and w + 4 of
// every plane: their offsets are wrapped once and a plane's offset advances by
// one wrapped step, so a row costs the scalar unit one 64-bit add.  Lane l
// loads the columns k0 = wrap(L3 + l) and k1 = wrap(L3 + l + 64) (has0, has1:
// inside the box).
template <int BR1, int BR2>
__device__ __forceinline__ void stage_box(const float *__restrict__ src, const Grid3 &g, int L1, int L2, int B1,
                                          int B2, int w, unsigned k0, unsigned k1, bool has0, bool has1, float *box)
{
    static_assert(BR2 == 8, "four wavefronts stage two x2 rows of each plane");
    const long n23 = (long)g.n2 * g.n3;
    const long ob0 = (long)wrapg(L2 + w, g.n2) * g.n3, ob1 = (long)wrapg(L2 + w + 4, g.n2) * g.n3;
    const bool hb0 = w < B2, hb1 = w + 4 < B2;
    int ia = wrapg(L1, g.n1);
#pragma unroll
    for (int a = 0; a < BR1; ++a) {
        if (a < B1) {
            const float *plane = src + (long)ia * n23;
            float *brow = box + (a * BR2 + w) * kPad3;
            if (hb0) {
                if (has0) load_to_lds(plane + ob0 + k0, brow);
                if (has1) load_to_lds(plane + ob0 + k1, brow + 64);
            }
            if (hb1) {
                if (has0) load_to_lds(plane + ob1 + k0, brow + 4 * kPad3);
                if (has1) load_to_lds(plane + ob1 + k1, brow + 4 * kPad3 + 64);
            }
        }
        ia = ia + 1 == g.n1 ? 0 : ia + 1;
    }
}

// displacements clamped to +-2^20 voxels (NaN to the lower bound), so that
// every index derived from them stays a finite int
__device__ __forceinline__ float clamp_disp(float d)
{
    const float lim = 1048576.f;
    return fminf(fmaxf(d, -lim), lim);
}

// Epilogues: which fields are gathered and what is written per point.  Each
// splits its work into load(p), every pointwise input, and store(p, v, in):
// the gather kernels issue the loads of all of a thread's points before the
// first store, since a load placed after a store to another array cannot be
// moved above it (the arrays may alias as far as the compiler knows) and
// would cost one memory round trip per point and step.
struct NoIn {
};
struct EpiCopy {  // out = I[src]
    static constexpr int NF = 1;
    __device__ void shift(long long o) { src = mshift(src, o); dst = mshift(dst, o); }
    using In = NoIn;
    const float *src;
    float *dst;
    __device__ const float *field(int) const { return src; }
    __device__ In load(long) const { return {}; }
    __device__ void store(long p, const float *v, const In &) const { dst[p] = v[0]; }
};
struct EpiAdj {  // out = scale * c * I[src]
    static constexpr int NF = 1;
    __device__ void shift(long long o) { src = mshift(src, o); coef = mshift(coef, o); dst = mshift(dst, o); }
    struct In {
        float c;
    };
    const float *src, *coef;
    float *dst;
    float scale;
    __device__ const float *field(int) const { return src; }
    __device__ In load(long p) const { return {coef[p]}; }
    __device__ void store(long p, const float *v, const In &in) const { dst[p] = scale * in.c * v[0]; }
};
struct EpiInc {  // out = I[src] - dt/2 s
    static constexpr int NF = 1;
    __device__ void shift(long long o) { src = mshift(src, o); s = mshift(s, o); dst = mshift(dst, o); }
    struct In {
        float s;
    };
    const float *src, *s;
    float *dst;
    float hdt;
    __device__ const float *field(int) const { return src; }
    __device__ In load(long p) const { return {s[p]}; }
    __device__ void store(long p, const float *v, const In &in) const { dst[p] = v[0] - hdt * in.s; }
};
struct EpiAdjCoef {  // c = 1 + dt/2 (delta_a + delta (1 + dt delta_a)), delta_a = I[delta](Xa)
    static constexpr int NF = 1;
    __device__ void shift(long long o) { delta = mshift(delta, o); coef = mshift(coef, o); }
    struct In {
        float d;
    };
    const float *delta;
    float *coef;
    float dt;
    __device__ const float *field(int) const { return delta; }
    __device__ In load(long p) const { return {delta[p]}; }
    __device__ void store(long p, const float *v, const In &in) const
    {
        const float da = v[0];
        coef[p] = 1.f + 0.5f * dt * (da + in.d * (1.f + dt * da));
    }
};
struct EpiVec3 {  // three fields (stride N): out_c = I[src_c]
    static constexpr int NF = 3;
    __device__ void shift(long long o) { src = mshift(src, o); dst = mshift(dst, o); }
    using In = NoIn;
    const float *src;
    float *dst;
    long N;
    __device__ const float *field(int f) const { return src + f * N; }
    __device__ In load(long) const { return {}; }
    __device__ void store(long p, const float *v, const In &) const
    {
        dst[p] = v[0];
        dst[N + p] = v[1];
        dst[2 * N + p] = v[2];
    }
};
// Incremental-state start (eq. incsta, Heun along the characteristics, with
// m~_0 = 0): the gather gives v~(X) (three fields); with the per-velocity
// I[grad m_j](X) and grad m_{j+1} the epilogue forms every step's source
//   s_j = v~(X) . I[grad m_j](X) + v~ . grad m_{j+1},   j = 0 .. N_t - 1,
// writes m~_1 = -dt/2 s_0 and keeps s_1 .. s_{N_t-1} for the later steps.
// With N_t fixed at compile time (NTC > 0) all 6 N_t + 3 inputs are loaded
// before the first store.
template <int NTC>
struct EpiIncSrc {
    static constexpr int NF = 3;
    __device__ void shift(long long o) { vt = mshift(vt, o); GX = mshift(GX, o); G = mshift(G, o); mt1 = mshift(mt1, o); src = mshift(src, o); }
    struct In {
        float v[3], gx[NTC > 0 ? NTC : 1][3], g1[NTC > 0 ? NTC : 1][3];
    };
    const float *vt;        // v~ (stride N): gathered and read pointwise
    const float *GX, *G;    // I[grad m_j](X) and grad m_j, three fields per j
    float *mt1, *src;       // m~_1; s_j at src + (j - 1) N
    long N;
    int nt_rt;
    float hdt;
    __device__ const float *field(int f) const { return vt + f * N; }
    __device__ In load(long p) const
    {
        In in;
#pragma unroll
        for (int c = 0; c < 3; ++c) in.v[c] = vt[c * N + p];
        if constexpr (NTC > 0) {
#pragma unroll
            for (int j = 0; j < NTC; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    in.gx[j][c] = GX[((long)j * 3 + c) * N + p];
                    in.g1[j][c] = G[((long)(j + 1) * 3 + c) * N + p];
                }
        }
        return in;
    }
    __device__ void store(long p, const float *x, const In &in) const
    {
        const float v0 = in.v[0], v1 = in.v[1], v2 = in.v[2];
        if constexpr (NTC > 0) {
#pragma unroll
            for (int j = 0; j < NTC; ++j)
                put(p, j, (x[0] * in.gx[j][0] + x[1] * in.gx[j][1] + x[2] * in.gx[j][2]) +
                              (v0 * in.g1[j][0] + v1 * in.g1[j][1] + v2 * in.g1[j][2]));
        } else {
            for (int j = 0; j < nt_rt; ++j) {
                const float *gx = GX + (long)j * 3 * N, *g1 = G + (long)(j + 1) * 3 * N;
                put(p, j, (x[0] * gx[p] + x[1] * gx[N + p] + x[2] * gx[2 * N + p]) +
                              (v0 * g1[p] + v1 * g1[N + p] + v2 * g1[2 * N + p]));
            }
        }
    }
    __device__ void put(long p, int j, float s) const
    {
        if (j == 0)
            mt1[p] = -hdt * s;
        else
            src[(long)(j - 1) * N + p] = s;
    }
};

// Last adjoint step (eq. adj-transport, incadj) fused with the body force:
// lam_0 = scale c I[lam_1](Xa), then the trapezoid in time
//   b = dt sum_j w_j lam_j grad m_j,  w_0 = w_{N_t} = 1/2, else 1,
// with lam_0 from the gather, lam_1 .. lam_{N_t-1} from the sweep and
// lam_{N_t} = scaleN lamN.  With N_t fixed at compile time (NTC > 0) all
// inputs are loaded before the first store.
template <int NTC>
struct EpiAdjBody {
    static constexpr int NF = 1;
    __device__ void shift(long long o) { src = mshift(src, o); coef = mshift(coef, o); lam0 = mshift(lam0, o); lam = mshift(lam, o); lamN = mshift(lamN, o); G = mshift(G, o); b = mshift(b, o); }
    struct In {
        float c, lam[NTC > 0 ? NTC : 1], g[NTC > 0 ? NTC + 1 : 1][3];  // lam[j-1] = lam_j, j = 1 .. N_t
    };
    const float *src, *coef;
    float *lam0;            // lam_0 out
    float scale;
    const float *lam;       // lam_j at lam + j N, 1 <= j < N_t
    const float *lamN;
    float scaleN;
    const float *G;         // grad m_j, three fields per j
    float *b;               // body force, three fields
    long N;
    int nt_rt;
    float dt;
    __device__ const float *field(int) const { return src; }
    __device__ In load(long p) const
    {
        In in;
        in.c = coef[p];
        if constexpr (NTC > 0) {
#pragma unroll
            for (int j = 1; j <= NTC; ++j) in.lam[j - 1] = j == NTC ? lamN[p] : lam[(long)j * N + p];
#pragma unroll
            for (int j = 0; j <= NTC; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) in.g[j][c] = G[((long)j * 3 + c) * N + p];
        }
        return in;
    }
    __device__ void store(long p, const float *v, const In &in) const
    {
        const float l0 = scale * in.c * v[0];
        lam0[p] = l0;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
        if constexpr (NTC > 0) {
#pragma unroll
            for (int j = 0; j <= NTC; ++j) {
                const float w = (j == 0 || j == NTC) ? 0.5f : 1.f;
                const float l = j == 0 ? w * l0 : (j == NTC ? (scaleN * w) * in.lam[j - 1] : w * in.lam[j - 1]);
                a0 += l * in.g[j][0];
                a1 += l * in.g[j][1];
                a2 += l * in.g[j][2];
            }
        } else {
            const int nt = nt_rt;
            for (int j = 0; j <= nt; ++j) {
                const float w = (j == 0 || j == nt) ? 0.5f : 1.f;
                const float l = j == 0 ? w * l0 : (j == nt ? (scaleN * w) * lamN[p] : w * lam[(long)j * N + p]);
                const float *gj = G + (long)j * 3 * N;
                a0 += l * gj[p];
                a1 += l * gj[N + p];
                a2 += l * gj[2 * N + p];
            }
        }
        b[p] = dt * a0;
        b[N + p] = dt * a1;
        b[2 * N + p] = dt * a2;
    }
};

// one point's epilogue, its loads first
template <class Epi>
__device__ __forceinline__ void epi_finish(const Epi &epi, long p, const float *v)
{
    const typename Epi::In in = epi.load(p);
    epi.store(p, v, in);
}

// the epilogues of a thread's PPT points of a tile, in groups: a group's
// loads are all issued before its first store (out-of-grid points load
// point 0 and store nothing)
template <int PPT, class Epi>
__device__ __forceinline__ void epi_finish_tile(const Epi &epi, const long (&pp)[PPT], const bool (&ok)[PPT],
                                                const float (*val)[Epi::NF])
{
    // points per group: their inputs together within 64 floats for two points
    // per thread, 32 for four (the contraction's registers set the kernel's
    // peak there)
    constexpr int SZ = (int)(sizeof(typename Epi::In) / sizeof(float)), BUD = PPT <= 2 ? 64 : 32;
    constexpr int GRP = SZ * PPT <= BUD ? PPT : (BUD / SZ > 1 ? BUD / SZ : 1);
#pragma unroll
    for (int q0 = 0; q0 < PPT; q0 += GRP) {
        typename Epi::In in[GRP];
#pragma unroll
        for (int u = 0; u < GRP; ++u)
            if (q0 + u < PPT) in[u] = epi.load(ok[q0 + u] ? pp[q0 + u] : 0);
#pragma unroll
        for (int u = 0; u < GRP; ++u)
            if (q0 + u < PPT && ok[q0 + u]) epi.store(pp[q0 + u], val[q0 + u], in[u]);
    }
}

// Stencil extents of one tile: the smallest first node (L) and the largest
// (H) along each axis over the tile's grid points, reduced over the
// workgroup; L1 > H1 when no point of the tile is inside the grid.
template <int T1, int T2, bool HALF>
__device__ __forceinline__ void tile_extents(const Grid3 &g, const float *__restrict__ disp, int i0, int j0, int t3,
                                             int w, int lane, int (*red)[6], int L[3], int H[3])
{
    using BC = BoxCfg<T1, T2>;
    using TM = TileMap<HALF>;
    constexpr int NQ = HALF ? BC::PPT / 2 : BC::PPT;
    const long N = g.N;
    const int k = TM::k_of(t3, lane);
    int lo1 = 0x7fffffff, lo2 = 0x7fffffff, lo3 = 0x7fffffff;
    int hi1 = (int)0x80000000, hi2 = (int)0x80000000, hi3 = (int)0x80000000;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int e = TM::row_of(w, q, lane, NQ), i = i0 + e / T2, j = j0 + e % T2;
        if (i < g.n1 && j < g.n2 && k < g.n3) {
            const long p = ((long)i * g.n2 + j) * g.n3 + k;
            const int b1 = i + (int)floorf(clamp_disp(disp[p])) - 1;
            const int b2 = j + (int)floorf(clamp_disp(disp[N + p])) - 1;
            const int b3 = k + (int)floorf(clamp_disp(disp[2 * N + p])) - 1;
            lo1 = min(lo1, b1);
            hi1 = max(hi1, b1);
            lo2 = min(lo2, b2);
            hi2 = max(hi2, b2);
            lo3 = min(lo3, b3);
            hi3 = max(hi3, b3);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo1 = min(lo1, __shfl_xor(lo1, off));
        lo2 = min(lo2, __shfl_xor(lo2, off));
        lo3 = min(lo3, __shfl_xor(lo3, off));
        hi1 = max(hi1, __shfl_xor(hi1, off));
        hi2 = max(hi2, __shfl_xor(hi2, off));
        hi3 = max(hi3, __shfl_xor(hi3, off));
    }
    if (lane == 0) {
        red[w][0] = lo1;
        red[w][1] = lo2;
        red[w][2] = lo3;
        red[w][3] = hi1;
        red[w][4] = hi2;
        red[w][5] = hi3;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        L[a] = min(min(red[0][a], red[1][a]), min(red[2][a], red[3][a]));
        H[a] = max(max(red[0][a + 3], red[1][a + 3]), max(red[2][a + 3], red[3][a + 3]));
    }
}

// Per-tile stencil extents of a displacement field, computed once per
// velocity: the matvec's gathers read them instead of reducing again, so a
// workgroup starts staging its box at once.  Entry t: L[3], H[3] of tile t
// (in the numbering of the gather kernel, before the XCD renumbering).
struct TileBox {
    int L[3], H[3], pad[2];
};

template <int T1, int T2, bool HALF>
__global__ __launch_bounds__(256) void k_tile_boxes(Grid3 g, const float *__restrict__ disp, TileBox *__restrict__ out,
                                                    int nt2, int nt3, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); disp = mshift(disp, mo_); out = mshift(out, mo_);
    __shared__ int red[4][6];
    const int tid = threadIdx.x, lane = tid & 63;
    // the wavefront index, wave-uniform: the compiler keeps what derives from
    // it (the rows of a point, their bounds and base addresses) in scalars
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tb = (int)blockIdx.x;
    const int u3 = tb % nt3, rr = tb / nt3, u2 = rr % nt2, u1 = rr / nt2;
    int L[3], H[3];
    tile_extents<T1, T2, HALF>(g, disp, u1 * T1, u2 * T2, u3, w, lane, red, L, H);
    if (tid == 0) {
        TileBox b;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            b.L[a] = L[a];
            b.H[a] = H[a];
        }
        b.pad[0] = b.pad[1] = 0;
        out[tb] = b;
    }
}

// boxes != nullptr: the extents come from k_tile_boxes for this displacement field
// MB: a batched plan (the member from blockIdx.y); plain plans run the
// kernel without the member shift
// HALF: half tiles (see TileMap)
template <int T1, int T2, class Epi, bool MB, bool HALF>
__global__ __launch_bounds__(256) void k_box(Grid3 g, const float *__restrict__ disp, Epi epi, int nt2, int nt3,
                                             const TileBox *__restrict__ boxes, Mb mb)
{
    if (mb.stopped(MB ? mb.offset(blockIdx.y) : 0)) return;  // a PCG iteration after the stop
    if constexpr (MB) {
        const long long mo_ = mb.offset(blockIdx.y);
        disp = mshift(disp, mo_);
        boxes = mshift(boxes, mo_);
        epi.shift(mo_);
    }
    using BC = BoxCfg<T1, T2>;
    using TM = TileMap<HALF>;
    // points per thread: PPT rows of one tile row each, or PPT / 2 when a
    // wavefront takes two rows at a time (half tiles)
    constexpr int PPT = HALF ? BC::PPT / 2 : BC::PPT, BR1 = BC::BR1, BR2 = BC::BR2, NF = Epi::NF;
    constexpr int S1 = BR2 * kPad3;  // box stride along x1 (x2: kPad3)
    extern __shared__ float box[];   // CAP floats
    __shared__ int red[4][6];
    const int tid = threadIdx.x, lane = tid & 63;
    // the wavefront index, wave-uniform: the compiler keeps what derives from
    // it (the rows of a point, their bounds and base addresses) in scalars
    // (for full tiles; half tiles give each half of the wavefront its row)
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int t3 = tb % nt3, rr = tb / nt3, t2 = rr % nt2, t1 = rr / nt2;
    const int i0 = t1 * T1, j0 = t2 * T2, k = TM::k_of(t3, lane);
    const long N = g.N;
    int Lx[3], Hx[3];
    if (boxes) {
        const TileBox tbx = boxes[tb];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Lx[a] = tbx.L[a];
            Hx[a] = tbx.H[a];
        }
    } else {
        tile_extents<T1, T2, HALF>(g, disp, i0, j0, t3, w, lane, red, Lx, Hx);
    }
    const int L1 = Lx[0], L2 = Lx[1], L3 = Lx[2], H1 = Hx[0], H2 = Hx[1], H3 = Hx[2];
    if (L1 > H1) return;  // no point of the tile is inside the grid (uniform)
    float d1[PPT], d2[PPT], d3[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int e = TM::row_of(w, q, lane, PPT), i = i0 + e / T2, j = j0 + e % T2;
        // points outside the grid (ragged tiles) read point 0 and use d = 0;
        // their sums are formed (wrapped, valid) and never stored, so no
        // lane of the contraction branches on them
        const bool in = i < g.n1 && j < g.n2 && k < g.n3;
        const long p = in ? ((long)i * g.n2 + j) * g.n3 + k : 0;
        const float e1 = clamp_disp(disp[p]), e2 = clamp_disp(disp[N + p]), e3 = clamp_disp(disp[2 * N + p]);
        d1[q] = in ? e1 : 0.f;
        d2[q] = in ? e2 : 0.f;
        d3[q] = in ? e3 : 0.f;
    }
    // staged extents: the stencil box, cut to the capacity (64-bit: a clamped
    // displacement spans up to 2^21 nodes)
    const int B1 = (int)min((long)H1 + 4 - L1, (long)BR1);
    const int B2 = (int)min((long)H2 + 4 - L2, (long)BR2);
    const int B3 = (int)min((long)H3 + 4 - L3, (long)kPad3);
    // Staging (stage_box): a row's source pointer is uniform over the
    // wavefront, so its address arithmetic runs on the scalar unit; the x3
    // wrap of a lane's two columns is the same for every row.  Fields go
    // through the one box in turn.
    const bool has0 = lane < B3, has1 = lane + 64 < B3;
    const unsigned k0 = (unsigned)wrapg(L3 + lane, g.n3), k1 = (unsigned)wrapg(L3 + lane + 64, g.n3);
    float val[PPT][NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const float *__restrict__ src = epi.field(f);
        if (f > 0) __syncthreads();  // the previous field's stencils are read
        stage_box<BR1, BR2>(src, g, L1, L2, B1, B2, w, k0, k1, has0, has1, box);
        wait_lds_loads();
        __syncthreads();
        if constexpr (NF > 1) {
            // weights and indices are formed again per field: kept across the
            // fields they would hold 4 x 12 registers (fewer waves per SIMD)
#pragma unroll
            for (int q = 0; q < PPT; ++q) asm("" : "+v"(d1[q]), "+v"(d2[q]), "+v"(d3[q]));
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int e = TM::row_of(w, q, lane, PPT), i = i0 + e / T2, j = j0 + e % T2;
            const float f1 = floorf(d1[q]), f2 = floorf(d2[q]), f3 = floorf(d3[q]);
            float w1[4], w2[4], w3[4];
            lagrange4<float>(d1[q] - f1, w1);
            lagrange4<float>(d2[q] - f2, w2);
            lagrange4<float>(d3[q] - f3, w3);
            const int b1 = i + (int)f1 - 1, b2 = j + (int)f2 - 1, b3 = k + (int)f3 - 1;
            // >= 0 by the reduction for points inside the grid; the unsigned
            // compare sends any other stencil to the global path
            const int o1 = b1 - L1, o2 = b2 - L2, o3 = b3 - L3;
            float acc = 0.f;
            if ((unsigned)o1 <= (unsigned)(B1 - 4) && (unsigned)o2 <= (unsigned)(B2 - 4) &&
                (unsigned)o3 <= (unsigned)(B3 - 4)) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    // one base address per x1 plane: the row reads of the
                    // plane then fit the LDS instruction's offset field
                    int pa = (int)(__umul24((unsigned)(o1 + a), S1) + __umul24((unsigned)o2, kPad3)) + o3;  // 24-bit: full rate
                    asm("" : "+v"(pa));
                    const float *pl = box + pa;
                    float acc2 = 0.f;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const float *row = pl + b * kPad3;
                        acc2 = accum<float>(b, w2, row3<float>(row[0], row[1], row[2], row[3], w3), acc2);
                    }
                    acc = accum<float>(a, w1, acc2, acc);
                }
            } else {  // stencil outside the staged box: global loads, wrapped per node
#pragma unroll 1
                for (int a = 0; a < 4; ++a) {
                    const long ra = (long)wrapg(b1 + a, g.n1) * g.n2;
                    float acc2 = 0.f;
                    for (int b = 0; b < 4; ++b) {
                        const float *row = src + (ra + wrapg(b2 + b, g.n2)) * g.n3;
                        acc2 = accum<float>(b, w2,
                                            row3<float>(row[wrapg(b3, g.n3)], row[wrapg(b3 + 1, g.n3)],
                                                        row[wrapg(b3 + 2, g.n3)], row[wrapg(b3 + 3, g.n3)], w3),
                                            acc2);
                    }
                    acc = accum<float>(a, w1, acc2, acc);
                }
            }
            val[q][f] = acc;
        }
    }
    long pp[PPT];
    bool ok[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int e = TM::row_of(w, q, lane, PPT), i = i0 + e / T2, j = j0 + e % T2;
        ok[q] = i < g.n1 && j < g.n2 && k < g.n3;
        pp[q] = ((long)i * g.n2 + j) * g.n3 + k;
    }
    epi_finish_tile<PPT>(epi, pp, ok, val);
}

// Departure points through an LDS box (cubic interpolation): per direction
// the tile's predictor stencils at x -+ dt v(x) are reduced to their extents,
// the three velocity components are staged through the box in turn and the
// FP64 contraction runs from LDS in the order of gather<double>, so X and Xa
// are bitwise those of k_departure<3>.  Stencils outside the box gather from
// global memory.  Nothing per point stays in registers across
// the component and point loops; v(x) is read again where it is needed.
__device__ __forceinline__ double predictor_disp(const float *__restrict__ v, long N, long p, int c, double sdt,
                                                 double ihc)
{
    // the clamped displacement of axis_stencil<double>
    double d = sdt * (double)v[(long)c * N + p] * ihc;
    const double lim = 1048576.0;
    d = d > lim ? lim : d;
    return d >= -lim ? d : -lim;
}

template <int T1, int T2>
__global__ __launch_bounds__(256) void k_departure_box(const float *__restrict__ v, float *__restrict__ dX,
                                                       float *__restrict__ dXa, Grid3 g, int nt2, int nt3, double dt,
                                                       double ih1, double ih2, double ih3, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); v = mshift(v, mo_); dX = mshift(dX, mo_); dXa = mshift(dXa, mo_);
    using BC = BoxCfg<T1, T2>;
    constexpr int PPT = BC::PPT, BR1 = BC::BR1, BR2 = BC::BR2;
    constexpr int S1 = BR2 * kPad3;
    extern __shared__ float box[];
    __shared__ int red[4][6];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int t3 = tb % nt3, rr = tb / nt3, t2 = rr % nt2, t1 = rr / nt2;
    const int i0 = t1 * T1, j0 = t2 * T2, k = t3 * kT3 + lane;
    const long N = g.N;
    const double ih[3] = {ih1, ih2, ih3};
#pragma unroll 1
    for (int dir = 0; dir < 2; ++dir) {
        const double sgn = dir == 0 ? -1.0 : 1.0;
        float *__restrict__ out = dir == 0 ? dX : dXa;
        const double sdt = sgn * dt;
        int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff};
        int hi[3] = {(int)0x80000000, (int)0x80000000, (int)0x80000000};
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int e = w + 4 * q, i = i0 + e / T2, j = j0 + e % T2;
            if (!(i < g.n1 && j < g.n2 && k < g.n3)) continue;
            const long p = ((long)i * g.n2 + j) * g.n3 + k;
            const int ijk[3] = {i, j, k};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int b = ijk[c] + (int)floor(predictor_disp(v, N, p, c, sdt, ih[c])) - 1;
                lo[c] = min(lo[c], b);
                hi[c] = max(hi[c], b);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lo[c] = min(lo[c], __shfl_xor(lo[c], off));
                hi[c] = max(hi[c], __shfl_xor(hi[c], off));
            }
        if (dir > 0) __syncthreads();  // the first direction's box and extents are read
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                red[w][c] = lo[c];
                red[w][c + 3] = hi[c];
            }
        __syncthreads();
        int L[3], H[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            L[c] = min(min(red[0][c], red[1][c]), min(red[2][c], red[3][c]));
            H[c] = max(max(red[0][c + 3], red[1][c + 3]), max(red[2][c + 3], red[3][c + 3]));
        }
        if (L[0] > H[0]) return;  // no point of the tile inside the grid (uniform)
        const int B1 = (int)min((long)H[0] + 4 - L[0], (long)BR1);
        const int B2 = (int)min((long)H[1] + 4 - L[1], (long)BR2);
        const int B3 = (int)min((long)H[2] + 4 - L[2], (long)kPad3);
        const bool has0 = lane < B3, has1 = lane + 64 < B3;
        const unsigned k0 = (unsigned)wrapg(L[2] + lane, g.n3), k1 = (unsigned)wrapg(L[2] + lane + 64, g.n3);
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            const float *__restrict__ src = v + (long)c * N;
            const double ihc = c == 0 ? ih1 : c == 1 ? ih2 : ih3;
            if (c > 0) __syncthreads();  // the previous component's stencils are read
            stage_box<BR1, BR2>(src, g, L[0], L[1], B1, B2, w, k0, k1, has0, has1, box);
            wait_lds_loads();
            __syncthreads();
#pragma unroll 1
            for (int q = 0; q < PPT; ++q) {
                const int e = w + 4 * q, i = i0 + e / T2, j = j0 + e % T2;
                if (!(i < g.n1 && j < g.n2 && k < g.n3)) continue;
                const long p = ((long)i * g.n2 + j) * g.n3 + k;
                const double d1 = predictor_disp(v, N, p, 0, sdt, ih1), d2 = predictor_disp(v, N, p, 1, sdt, ih2),
                             d3 = predictor_disp(v, N, p, 2, sdt, ih3);
                const double f1 = floor(d1), f2 = floor(d2), f3 = floor(d3);
                double w1[4], w2[4], w3[4];
                lagrange4<double>(d1 - f1, w1);
                lagrange4<double>(d2 - f2, w2);
                lagrange4<double>(d3 - f3, w3);
                const int b1 = i + (int)f1 - 1, b2 = j + (int)f2 - 1, b3 = k + (int)f3 - 1;
                const int o1 = b1 - L[0], o2 = b2 - L[1], o3 = b3 - L[2];
                double acc = 0.0;
                if (o1 <= B1 - 4 && o2 <= B2 - 4 && o3 <= B3 - 4) {
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const float *pl = box + (o1 + a) * S1 + o2 * kPad3 + o3;
                        double acc2 = 0.0;
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const float *row = pl + b * kPad3;
                            acc2 = accum<double>(
                                b, w2,
                                row3<double>((double)row[0], (double)row[1], (double)row[2], (double)row[3], w3),
                                acc2);
                        }
                        acc = accum<double>(a, w1, acc2, acc);
                    }
                } else {  // from global memory, wrapped per node
#pragma unroll 1
                    for (int a = 0; a < 4; ++a) {
                        const long ra = (long)wrapg(b1 + a, g.n1) * g.n2;
                        double acc2 = 0.0;
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const float *row = src + (ra + wrapg(b2 + b, g.n2)) * g.n3;
                            acc2 = accum<double>(b, w2,
                                                 row3<double>((double)row[wrapg(b3, g.n3)],
                                                              (double)row[wrapg(b3 + 1, g.n3)],
                                                              (double)row[wrapg(b3 + 2, g.n3)],
                                                              (double)row[wrapg(b3 + 3, g.n3)], w3),
                                                 acc2);
                        }
                        acc = accum<double>(a, w1, acc2, acc);
                    }
                }
                out[(long)c * N + p] = (float)(sgn * 0.5 * dt * ((double)src[p] + acc) * ihc);
            }
        }
    }
}

// Persistent, software-pipelined box gathers (one field, extents table
// required): a fixed grid of workgroups walks the tiles, each XCD a
// contiguous run of them.  While a workgroup interpolates tile k from one
// LDS box, tile k+1's box rows are already in flight straight into the other
// box (global-to-LDS loads, no registers) together with its displacements;
// one wait and one barrier per tile.  Same stencil sums, bitwise, as k_box.
template <int T1, int T2, class Epi>
__global__ __launch_bounds__(256) void k_box_pipe(Grid3 g, const float *__restrict__ disp, Epi epi, int nt2,
                                                  int nt3, const TileBox *__restrict__ boxes, int ntiles, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); disp = mshift(disp, mo_); boxes = mshift(boxes, mo_); epi.shift(mo_);
    if (mb.stopped(mo_)) return;
    static_assert(Epi::NF == 1, "one field");
    using BC = BoxCfg<T1, T2>;
    constexpr int PPT = BC::PPT, BR1 = BC::BR1, BR2 = BC::BR2, CAP = BC::CAP;
    constexpr int S1 = BR2 * kPad3;
    extern __shared__ float boxes2[];  // 2 x CAP floats
    const int tid = threadIdx.x, lane = tid & 63;
    // the wavefront index, wave-uniform: the compiler keeps what derives from
    // it (the rows of a point, their bounds and base addresses) in scalars
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const long N = g.N;
    const float *__restrict__ src = epi.field(0);
    // tiles of this workgroup: XCD x = blockIdx % 8 owns tiles [x T / 8, (x+1) T / 8)
    const int G = (int)gridDim.x, per = (ntiles + 7) / 8;
    const int xcd = (int)blockIdx.x & 7, slot = (int)blockIdx.x >> 3, gx = (G + 7 - xcd) / 8;
    const int tbeg = xcd * per, tend = min(ntiles, tbeg + per);
    auto tile_at = [&](int kk) { return tbeg + slot + kk * gx; };
    // issue the box rows of tile t into bx (wavefront w: rows w, w + 4, ...)
    auto fetch_to = [&](int t, float *bx) {
        const TileBox tbx = boxes[t];
        if (tbx.L[0] > tbx.H[0]) return;  // no point of the tile inside the grid
        const int L1 = tbx.L[0], L2 = tbx.L[1], L3 = tbx.L[2];
        const int B1 = (int)min((long)tbx.H[0] + 4 - L1, (long)BR1);
        const int B2 = (int)min((long)tbx.H[1] + 4 - L2, (long)BR2);
        const int B3 = (int)min((long)tbx.H[2] + 4 - L3, (long)kPad3);
        const unsigned k0 = (unsigned)wrapg(L3 + lane, g.n3), k1 = (unsigned)wrapg(L3 + lane + 64, g.n3);
        stage_box<BR1, BR2>(src, g, L1, L2, B1, B2, w, k0, k1, lane < B3, lane + 64 < B3, bx);
    };
    // the displacements of tile t's points (points outside the grid read point 0)
    auto load_disp = [&](int t, float *e1, float *e2, float *e3) {
        const int t3 = t % nt3, rr = t / nt3, t2 = rr % nt2, t1 = rr / nt2;
        const int i0 = t1 * T1, j0 = t2 * T2, k = t3 * kT3 + lane;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int e = w + 4 * q, i = i0 + e / T2, j = j0 + e % T2;
            const long p = (i < g.n1 && j < g.n2 && k < g.n3) ? ((long)i * g.n2 + j) * g.n3 + k : 0;
            e1[q] = disp[p];
            e2[q] = disp[N + p];
            e3[q] = disp[2 * N + p];
        }
    };
    if (tile_at(0) >= tend) return;  // uniform over the workgroup
    float d1[PPT], d2[PPT], d3[PPT];
    fetch_to(tile_at(0), boxes2);
    load_disp(tile_at(0), d1, d2, d3);
    wait_lds_loads();
    __syncthreads();
    for (int kk = 0;; ++kk) {
        const int t = tile_at(kk), tn = tile_at(kk + 1);
        const bool more = tn < tend;
        const int t3 = t % nt3, rr = t / nt3, t2 = rr % nt2, t1 = rr / nt2;
        const int i0 = t1 * T1, j0 = t2 * T2, k = t3 * kT3 + lane;
        // the next tile's box goes to the buffer last read two tiles ago (every
        // wave has passed the barrier that ended that tile)
        float n1[PPT], n2[PPT], n3[PPT];
        if (more) {
            fetch_to(tn, boxes2 + ((kk + 1) & 1) * CAP);
            load_disp(tn, n1, n2, n3);
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            d1[q] = clamp_disp(d1[q]);
            d2[q] = clamp_disp(d2[q]);
            d3[q] = clamp_disp(d3[q]);
        }
        const TileBox tbx = boxes[t];
        const float *cur = boxes2 + (kk & 1) * CAP;
        const int L1 = tbx.L[0], L2 = tbx.L[1], L3 = tbx.L[2];
        const int B1 = (int)min((long)tbx.H[0] + 4 - L1, (long)BR1);
        const int B2 = (int)min((long)tbx.H[1] + 4 - L2, (long)BR2);
        const int B3 = (int)min((long)tbx.H[2] + 4 - L3, (long)kPad3);
        float val[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int e = w + 4 * q, i = i0 + e / T2, j = j0 + e % T2;
            val[q] = 0.f;
            if (!(i < g.n1 && j < g.n2 && k < g.n3)) continue;
            const float f1 = floorf(d1[q]), f2 = floorf(d2[q]), f3 = floorf(d3[q]);
            float w1[4], w2[4], w3[4];
            lagrange4<float>(d1[q] - f1, w1);
            lagrange4<float>(d2[q] - f2, w2);
            lagrange4<float>(d3[q] - f3, w3);
            const int b1 = i + (int)f1 - 1, b2 = j + (int)f2 - 1, b3 = k + (int)f3 - 1;
            const int o1 = b1 - L1, o2 = b2 - L2, o3 = b3 - L3;
            float acc = 0.f;
            if (o1 <= B1 - 4 && o2 <= B2 - 4 && o3 <= B3 - 4) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    int pa = (int)(__umul24((unsigned)(o1 + a), S1) + __umul24((unsigned)o2, kPad3)) + o3;  // 24-bit: full rate
                    asm("" : "+v"(pa));
                    const float *pl = cur + pa;
                    float acc2 = 0.f;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const float *row = pl + b * kPad3;
                        acc2 = accum<float>(b, w2, row3<float>(row[0], row[1], row[2], row[3], w3), acc2);
                    }
                    acc = accum<float>(a, w1, acc2, acc);
                }
            } else {
#pragma unroll 1
                for (int a = 0; a < 4; ++a) {
                    const long ra = (long)wrapg(b1 + a, g.n1) * g.n2;
                    float acc2 = 0.f;
                    for (int b = 0; b < 4; ++b) {
                        const float *row = src + (ra + wrapg(b2 + b, g.n2)) * g.n3;
                        acc2 = accum<float>(b, w2,
                                            row3<float>(row[wrapg(b3, g.n3)], row[wrapg(b3 + 1, g.n3)],
                                                        row[wrapg(b3 + 2, g.n3)], row[wrapg(b3 + 3, g.n3)], w3),
                                            acc2);
                    }
                    acc = accum<float>(a, w1, acc2, acc);
                }
            }
            val[q] = acc;
        }
        {
            long pp[PPT];
            bool ok[PPT];
            float vv[PPT][1];
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int e = w + 4 * q, i = i0 + e / T2, j = j0 + e % T2;
                ok[q] = i < g.n1 && j < g.n2 && k < g.n3;
                pp[q] = ((long)i * g.n2 + j) * g.n3 + k;
                vv[q][0] = val[q];
            }
            epi_finish_tile<PPT>(epi, pp, ok, vv);
        }
        if (!more) break;  // uniform
        wait_lds_loads();
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            d1[q] = n1[q];
            d2[q] = n2[q];
            d3[q] = n3[q];
        }
    }
}

// direct gathers, one thread per point, stencil loads from L1/L2
template <class Epi>
__global__ __launch_bounds__(kPtThreads) void k_direct(Grid3 g, const float *__restrict__ disp, Epi epi, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); disp = mshift(disp, mo_); epi.shift(mo_);
    if (mb.stopped(mo_)) return;
    const int p = point_index();
    if (p >= g.N) return;
    int i, j, k;
    point_coords(g, p, i, j, k);
    const long N = g.N;
    Stencil<float> s;
    make_stencil<float>(g, i, j, k, disp[p], disp[N + p], disp[2 * N + p], s);
    float v[Epi::NF];
#pragma unroll
    for (int f = 0; f < Epi::NF; ++f) v[f] = gather<float>(epi.field(f), s);
    epi_finish(epi, p, v);
}

// trilinear gathers (LDDMM_FLAG_LINEAR_IP): eight nodes per point from L1/L2
template <class Epi>
__global__ __launch_bounds__(kPtThreads) void k_direct_lin(Grid3 g, const float *__restrict__ disp, Epi epi, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.y); disp = mshift(disp, mo_); epi.shift(mo_);
    if (mb.stopped(mo_)) return;
    const int p = point_index();
    if (p >= g.N) return;
    int i, j, k;
    point_coords(g, p, i, j, k);
    const long N = g.N;
    Stencil2<float> s;
    make_stencil2<float>(g, i, j, k, disp[p], disp[N + p], disp[2 * N + p], s);
    float v[Epi::NF];
#pragma unroll
    for (int f = 0; f < Epi::NF; ++f) v[f] = gather2<float>(epi.field(f), s);
    epi_finish(epi, p, v);
}

// Eighth-order central first derivatives on the periodic grid (Section 3.2,
// the FD kernel replacing the spectral gradient and divergence):
//   df/dx ~= (1/h) sum_{q=1..4} c_q (f(x + q h) - f(x - q h)),
//   c = (4/5, -1/5, 4/105, -1/280).
// A workgroup covers 64 x3 points of 4 x2 rows of one x1 plane; the x3
// neighbours share cache lines, the x2 and x1 ones come through L2.
__device__ __forceinline__ float fd8_sum(float p1, float m1, float p2, float m2, float p3, float m3, float p4,
                                         float m4)
{
    float s = 0.8f * (p1 - m1);
    s = __builtin_fmaf(-0.2f, p2 - m2, s);
    s = __builtin_fmaf(0.038095238095238095f, p3 - m3, s);
    return __builtin_fmaf(-0.0035714285714285713f, p4 - m4, s);
}

__device__ __forceinline__ int wrap_up(int x, int n) { return x >= n ? x - n : x; }
__device__ __forceinline__ int wrap_dn(int x, int n) { return x < 0 ? x + n : x; }

// derivative along axis AX (0: x1, 1: x2, 2: x3) of f at (i, j, k)
template <int AX>
__device__ __forceinline__ float fd8_at(const float *__restrict__ f, int n1, int n2, int n3, int i, int j, int k)
{
    float p[4], m[4];
#pragma unroll
    for (int q = 1; q <= 4; ++q) {
        int ip = i, im = i, jp = j, jm = j, kp = k, km = k;
        if (AX == 0) {
            ip = wrap_up(i + q, n1);
            im = wrap_dn(i - q, n1);
        } else if (AX == 1) {
            jp = wrap_up(j + q, n2);
            jm = wrap_dn(j - q, n2);
        } else {
            kp = wrap_up(k + q, n3);
            km = wrap_dn(k - q, n3);
        }
        p[q - 1] = f[((long)ip * n2 + jp) * n3 + kp];
        m[q - 1] = f[((long)im * n2 + jm) * n3 + km];
    }
    return fd8_sum(p[0], m[0], p[1], m[1], p[2], m[2], p[3], m[3]);
}

__global__ __launch_bounds__(256) void k_fd8_grad(const float *__restrict__ f, float *__restrict__ g1,
                                                  float *__restrict__ g2, float *__restrict__ g3, int n1, int n2,
                                                  int n3, float ih1, float ih2, float ih3, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.z); f = mshift(f, mo_); g1 = mshift(g1, mo_); g2 = mshift(g2, mo_); g3 = mshift(g3, mo_);
    if (mb.stopped(mo_)) return;
    const int nkt = (n3 + 63) / 64;
    const int kt = (int)blockIdx.x % nkt, jt = (int)blockIdx.x / nkt, i = (int)blockIdx.y;
    const int k = kt * 64 + (int)(threadIdx.x & 63), j = jt * 4 + (int)(threadIdx.x >> 6);
    if (k >= n3 || j >= n2) return;
    const long p = ((long)i * n2 + j) * n3 + k;
    g1[p] = ih1 * fd8_at<0>(f, n1, n2, n3, i, j, k);
    g2[p] = ih2 * fd8_at<1>(f, n1, n2, n3, i, j, k);
    g3[p] = ih3 * fd8_at<2>(f, n1, n2, n3, i, j, k);
}

__global__ __launch_bounds__(256) void k_fd8_div(const float *__restrict__ v, float *__restrict__ out, int n1,
                                                 int n2, int n3, long N, float ih1, float ih2, float ih3, Mb mb)
{
    const long long mo_ = mb.offset(blockIdx.z); v = mshift(v, mo_); out = mshift(out, mo_);
    if (mb.stopped(mo_)) return;
    const int nkt = (n3 + 63) / 64;
    const int kt = (int)blockIdx.x % nkt, jt = (int)blockIdx.x / nkt, i = (int)blockIdx.y;
    const int k = kt * 64 + (int)(threadIdx.x & 63), j = jt * 4 + (int)(threadIdx.x >> 6);
    if (k >= n3 || j >= n2) return;
    const long p = ((long)i * n2 + j) * n3 + k;
    const float d1 = ih1 * fd8_at<0>(v, n1, n2, n3, i, j, k);
    const float d2 = ih2 * fd8_at<1>(v + N, n1, n2, n3, i, j, k);
    const float d3 = ih3 * fd8_at<2>(v + 2 * N, n1, n2, n3, i, j, k);
    out[p] = (d1 + d2) + d3;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static Divider divider(int d)
{
    unsigned sh = 0;
    while ((1u << sh) < (unsigned)d) ++sh;
    const unsigned long long mag = ((1ull << (31 + sh)) / (unsigned)d) + 1;
    return Divider{(unsigned)mag, sh};
}

static Grid3 grid_of(const lddmm_plan *P)
{
    return Grid3{P->cfg.n[0], P->cfg.n[1], P->cfg.n[2], (int)P->N, divider(P->cfg.n[2]), divider(P->cfg.n[1])};
}

static dim3 blocks_of(const lddmm_plan *P)
{
    return dim3((unsigned)((P->N + kPtThreads - 1) / kPtThreads), (unsigned)P->mb.count);
}

static dim3 fd8_grid(const lddmm_plan *P)
{
    const int n1 = P->cfg.n[0], n2 = P->cfg.n[1], n3 = P->cfg.n[2];
    return dim3((unsigned)(((n3 + 63) / 64) * ((n2 + 3) / 4)), (unsigned)n1, (unsigned)P->mb.count);
}

void launch_fd8_grad(lddmm_plan *P, const float *f, float *g1, float *g2, float *g3)
{
    Scope s(P, K_FD8);
    hipLaunchKernelGGL(k_fd8_grad, fd8_grid(P), dim3(256), 0, P->stream, f, g1, g2, g3, P->cfg.n[0], P->cfg.n[1],
                       P->cfg.n[2], (float)(1.0 / P->h[0]), (float)(1.0 / P->h[1]), (float)(1.0 / P->h[2]), P->mb);
    check_hip(hipGetLastError(), "k_fd8_grad");
}

void launch_fd8_div(lddmm_plan *P, const float *v, float *out)
{
    Scope s(P, K_FD8);
    hipLaunchKernelGGL(k_fd8_div, fd8_grid(P), dim3(256), 0, P->stream, v, out, P->cfg.n[0], P->cfg.n[1],
                       P->cfg.n[2], P->N, (float)(1.0 / P->h[0]), (float)(1.0 / P->h[1]), (float)(1.0 / P->h[2]), P->mb);
    check_hip(hipGetLastError(), "k_fd8_div");
}

static bool linear_ip(const lddmm_plan *P) { return (P->cfg.flags & LDDMM_FLAG_LINEAR_IP) != 0; }

static int gather_mode(const lddmm_plan *P);
template <int T1, int T2>
static unsigned tiles_of(const lddmm_plan *P, int &nt2, int &nt3, int w3 = kT3);
// the box gathers' tiles are half tiles on this plan's grid
static bool half_tiles(const lddmm_plan *P) { return half_tiles_for(P->cfg.n[2]); }
static int gather_w3(const lddmm_plan *P) { return half_tiles(P) ? 32 : kT3; }

// departure strategy: P->departure_mode 0 direct, 1 box tiles 2x4x64, 2 box
// tiles 4x4x64; -1 the tile shape of the gather strategy
static int departure_mode(const lddmm_plan *P)
{
    if (P->departure_mode >= 0) return P->departure_mode;
    const int m = gather_mode(P);
    return m == 0 ? 0 : (m == 1 || m == 3) ? 1 : 2;
}

template <int T1, int T2>
static void launch_departure_box(lddmm_plan *P, const float *v, float *dX, float *dXa)
{
    int nt2, nt3;
    const unsigned ntiles = tiles_of<T1, T2>(P, nt2, nt3);
    const size_t lds = sizeof(float) * BoxCfg<T1, T2>::CAP;
    hipLaunchKernelGGL((k_departure_box<T1, T2>), dim3(ntiles, P->mb.count), dim3(256), lds, P->stream, v, dX, dXa, grid_of(P),
                       nt2, nt3, P->dt, 1.0 / P->h[0], 1.0 / P->h[1], 1.0 / P->h[2], P->mb);
    check_hip(hipGetLastError(), "k_departure_box");
}

void launch_departure(lddmm_plan *P, const float *v, float *dX, float *dXa)
{
    Scope s(P, K_DEPARTURE);
    if (linear_ip(P)) {
        hipLaunchKernelGGL(k_departure<1>, blocks_of(P), dim3(kPtThreads), 0, P->stream, v, dX, dXa, grid_of(P),
                           P->dt, 1.0 / P->h[0], 1.0 / P->h[1], 1.0 / P->h[2], P->mb);
        check_hip(hipGetLastError(), "k_departure");
        return;  // the trilinear gathers stage no boxes
    }
    switch (departure_mode(P)) {
    case 0:
        hipLaunchKernelGGL(k_departure<3>, blocks_of(P), dim3(kPtThreads), 0, P->stream, v, dX, dXa, grid_of(P),
                           P->dt, 1.0 / P->h[0], 1.0 / P->h[1], 1.0 / P->h[2], P->mb);
        check_hip(hipGetLastError(), "k_departure");
        break;
    case 1: launch_departure_box<2, 4>(P, v, dX, dXa); break;
    default: launch_departure_box<4, 4>(P, v, dX, dXa); break;
    }
    if (dX == P->dX && dXa == P->dXa) launch_tile_boxes(P);
}

// gather strategy: P->gather_mode 0 direct, 1 box tiles 2x4x64, 2 box tiles
// 4x4x64, 3 and 4 the same tiles walked by persistent pipelined workgroups
// (one-field gathers at the plan's own departure points; others take 1 or
// 2); -1 before tuning: 4x4 tiles when they leave enough workgroups to fill
// the chip, else 2x4
static int gather_mode(const lddmm_plan *P)
{
    // a batched plan walks its members' tiles with one workgroup per tile
    if (P->gather_mode >= 0) return P->mb.count > 1 && P->gather_mode >= 3 ? P->gather_mode - 2 : P->gather_mode;
    const long n1 = P->cfg.n[0], n2 = P->cfg.n[1], n3 = P->cfg.n[2];
    const long tiles = ((n1 + 3) / 4) * ((n2 + 3) / 4) * ((n3 + kT3 - 1) / kT3);
    return tiles >= 4096 ? 2 : 1;
}

template <int T1, int T2>
static unsigned tiles_of(const lddmm_plan *P, int &nt2, int &nt3, int w3)
{
    const int n1 = P->cfg.n[0], n2 = P->cfg.n[1], n3 = P->cfg.n[2];
    const int nt1 = (n1 + T1 - 1) / T1;
    nt2 = (n2 + T2 - 1) / T2;
    nt3 = (n3 + w3 - 1) / w3;
    return (unsigned)((long)nt1 * nt2 * nt3);
}

// the extents table of a displacement field for tiles T1 x T2, when the plan
// holds one for that field (its own departure points)
template <int T1, int T2>
static const TileBox *boxes_for(const lddmm_plan *P, const float *disp)
{
    const int shape = (T1 == 4 && T2 == 4) ? 1 : 0;
    if (!P->boxes_valid) return nullptr;
    if (disp == P->dX) return (const TileBox *)P->boxes[0][shape];
    if (disp == P->dXa) return (const TileBox *)P->boxes[1][shape];
    return nullptr;
}

template <int T1, int T2, class Epi, bool HALF>
static void launch_box_as(lddmm_plan *P, const float *disp, const Epi &epi, int kid)
{
    int nt2, nt3;
    const unsigned ntiles = tiles_of<T1, T2>(P, nt2, nt3, TileMap<HALF>::W3);
    const size_t lds = sizeof(float) * BoxCfg<T1, T2>::CAP;
    static_assert(sizeof(float) * BoxCfg<4, 4>::CAP <= 64 * 1024, "box exceeds the default LDS limit");
    Scope s(P, kid);
    if (P->mb.count > 1)
        hipLaunchKernelGGL((k_box<T1, T2, Epi, true, HALF>), dim3(ntiles, P->mb.count), dim3(256), lds, P->stream,
                           grid_of(P), disp, epi, nt2, nt3, boxes_for<T1, T2>(P, disp), P->mb);
    else
        hipLaunchKernelGGL((k_box<T1, T2, Epi, false, HALF>), dim3(ntiles), dim3(256), lds, P->stream, grid_of(P),
                           disp, epi, nt2, nt3, boxes_for<T1, T2>(P, disp), P->mb);
    check_hip(hipGetLastError(), "k_box");
}

template <int T1, int T2, class Epi>
static void launch_box(lddmm_plan *P, const float *disp, const Epi &epi, int kid)
{
    if (half_tiles(P))
        launch_box_as<T1, T2, Epi, true>(P, disp, epi, kid);
    else
        launch_box_as<T1, T2, Epi, false>(P, disp, epi, kid);
}

// Pipelined gathers: as many workgroups as stay resident on the device at
// once (a multiple of the 8 XCDs), at most one per tile; the plain box
// kernel where no extents table exists.
template <int T1, int T2, class Epi>
static void launch_box_pipe1(lddmm_plan *P, const float *disp, const Epi &epi, int kid);

template <int T1, int T2, class Epi>
static void launch_box_pipe(lddmm_plan *P, const float *disp, const Epi &epi, int kid)
{
    if constexpr (Epi::NF != 1) {
        launch_box<T1, T2>(P, disp, epi, kid);
    } else {
        launch_box_pipe1<T1, T2>(P, disp, epi, kid);
    }
}

template <int T1, int T2, class Epi>
static void launch_box_pipe1(lddmm_plan *P, const float *disp, const Epi &epi, int kid)
{
    const TileBox *bx = boxes_for<T1, T2>(P, disp);
    if (!bx || half_tiles(P)) {  // the pipelined kernel walks full tiles only
        launch_box<T1, T2>(P, disp, epi, kid);
        return;
    }
    int nt2, nt3;
    const unsigned ntiles = tiles_of<T1, T2>(P, nt2, nt3);
    const size_t lds = 2 * sizeof(float) * BoxCfg<T1, T2>::CAP;
    static_assert(2 * sizeof(float) * BoxCfg<4, 4>::CAP <= 64 * 1024, "boxes exceed the default LDS limit");
    int &grid = P->pipe_grid[(T1 == 4 && T2 == 4) ? 1 : 0];
    if (grid == 0) {
        int per_cu = 0, cus = 0;
        check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_box_pipe<T1, T2, EpiAdj>, 256, lds),
                  "hipOccupancyMaxActiveBlocksPerMultiprocessor");
        check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device),
                  "hipDeviceGetAttribute");
        grid = std::max(8, (std::max(per_cu, 1) * cus) / 8 * 8);
    }
    const unsigned nb = std::min((unsigned)grid, ntiles);
    Scope s(P, kid);
    hipLaunchKernelGGL((k_box_pipe<T1, T2, Epi>), dim3(nb, P->mb.count), dim3(256), lds, P->stream, grid_of(P), disp, epi, nt2,
                       nt3, bx, (int)ntiles, P->mb);
    check_hip(hipGetLastError(), "k_box_pipe");
}

// extents tables of the plan's two displacement fields for both tile shapes
size_t tile_boxes_bytes(const int n[3])
{
    const int w3 = half_tiles_for(n[2]) ? 32 : kT3;
    auto cnt = [&](int T1, int T2) {
        return (size_t)((n[0] + T1 - 1) / T1) * ((n[1] + T2 - 1) / T2) * ((n[2] + w3 - 1) / w3);
    };
    return sizeof(TileBox) * (cnt(2, 4) + cnt(4, 4));
}

void assign_tile_boxes(lddmm_plan *P, char *base)
{
    int nt2, nt3;
    const size_t n24 = tiles_of<2, 4>(P, nt2, nt3, gather_w3(P)), per = tile_boxes_bytes(P->cfg.n);
    for (int f = 0; f < 2; ++f) {
        P->boxes[f][0] = base + f * per;
        P->boxes[f][1] = base + f * per + sizeof(TileBox) * n24;
    }
    P->boxes_valid = 0;
}

void launch_tile_boxes(lddmm_plan *P)
{
    if (!P->boxes[0][0]) return;
    int nt2, nt3;
    const bool half = half_tiles(P);
    const int w3 = gather_w3(P);
    for (int f = 0; f < 2; ++f) {
        const float *disp = f == 0 ? P->dX : P->dXa;
        unsigned nb = tiles_of<2, 4>(P, nt2, nt3, w3);
        if (half)
            hipLaunchKernelGGL((k_tile_boxes<2, 4, true>), dim3(nb, P->mb.count), dim3(256), 0, P->stream, grid_of(P),
                               disp, (TileBox *)P->boxes[f][0], nt2, nt3, P->mb);
        else
            hipLaunchKernelGGL((k_tile_boxes<2, 4, false>), dim3(nb, P->mb.count), dim3(256), 0, P->stream, grid_of(P),
                               disp, (TileBox *)P->boxes[f][0], nt2, nt3, P->mb);
        nb = tiles_of<4, 4>(P, nt2, nt3, w3);
        if (half)
            hipLaunchKernelGGL((k_tile_boxes<4, 4, true>), dim3(nb, P->mb.count), dim3(256), 0, P->stream, grid_of(P),
                               disp, (TileBox *)P->boxes[f][1], nt2, nt3, P->mb);
        else
            hipLaunchKernelGGL((k_tile_boxes<4, 4, false>), dim3(nb, P->mb.count), dim3(256), 0, P->stream, grid_of(P),
                               disp, (TileBox *)P->boxes[f][1], nt2, nt3, P->mb);
    }
    check_hip(hipGetLastError(), "k_tile_boxes");
    P->boxes_valid = 1;
}

template <class Epi>
static void tiled(lddmm_plan *P, const float *disp, const Epi &epi, int kid)
{
    if (linear_ip(P)) {
        Scope s(P, kid);
        hipLaunchKernelGGL((k_direct_lin<Epi>), blocks_of(P), dim3(kPtThreads), 0, P->stream, grid_of(P), disp, epi, P->mb);
        check_hip(hipGetLastError(), "k_direct_lin");
        return;
    }
    const int mode = (Epi::NF > 1 && P->gather_mode3 >= 0) ? P->gather_mode3 : gather_mode(P);
    switch (mode) {
    case 0: {
        Scope s(P, kid);
        hipLaunchKernelGGL((k_direct<Epi>), blocks_of(P), dim3(kPtThreads), 0, P->stream, grid_of(P), disp, epi, P->mb);
        check_hip(hipGetLastError(), "k_direct");
        break;
    }
    case 1: launch_box<2, 4>(P, disp, epi, kid); break;
    case 2: launch_box<4, 4>(P, disp, epi, kid); break;
    case 3: launch_box_pipe<2, 4>(P, disp, epi, kid); break;
    default: launch_box_pipe<4, 4>(P, disp, epi, kid); break;
    }
}

// time the gather strategies on the plan's adjoint displacement field (one
// adjoint step into scratch) and keep the fastest
void autotune_gather(lddmm_plan *P)
{
    const int keep = P->gather_mode;
    float best = 1e30f;
    int bm = 2;
    const float *src = P->lam;
    float *dst = P->lam + P->N;
    for (int m = 0; m < 5; ++m) {
        P->gather_mode = m;
        hipEvent_t a, b;
        check_hip(hipEventCreate(&a), "hipEventCreate");
        check_hip(hipEventCreate(&b), "hipEventCreate");
        tiled(P, P->dXa, EpiAdj{src, P->coef, dst, 1.f}, K_ADJ_STEP);
        check_hip(hipEventRecord(a, P->stream), "hipEventRecord");
        for (int r = 0; r < 3; ++r) tiled(P, P->dXa, EpiAdj{src, P->coef, dst, 1.f}, K_ADJ_STEP);
        check_hip(hipEventRecord(b, P->stream), "hipEventRecord");
        check_hip(hipEventSynchronize(b), "hipEventSynchronize");
        float ms = 0.f;
        check_hip(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (ms < best) {
            best = ms;
            bm = m;
        }
    }
    P->gather_mode = keep >= 0 ? keep : bm;
    P->gather_ms[0] = best;
    // three-field gathers (more registers per point) are tuned on their own,
    // on the incremental-state start with the velocity for v~ (its outputs
    // are matvec scratch)
    if (keep < 0 && P->v && P->GX && P->mt && P->src) {
        float best3 = 1e30f;
        int bm3 = P->gather_mode;
        for (int m = 0; m < 3; ++m) {
            P->gather_mode3 = m;
            hipEvent_t a, b;
            check_hip(hipEventCreate(&a), "hipEventCreate");
            check_hip(hipEventCreate(&b), "hipEventCreate");
            launch_incstate_init(P, P->v, P->mt);
            check_hip(hipEventRecord(a, P->stream), "hipEventRecord");
            for (int r = 0; r < 3; ++r) launch_incstate_init(P, P->v, P->mt);
            check_hip(hipEventRecord(b, P->stream), "hipEventRecord");
            check_hip(hipEventSynchronize(b), "hipEventSynchronize");
            float ms = 0.f;
            check_hip(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            if (ms < best3) {
                best3 = ms;
                bm3 = m;
            }
        }
        P->gather_mode3 = bm3;
    }
    // departure points (bitwise the same under every strategy, so the plan's
    // own fields are recomputed in place)
    if (P->departure_mode < 0 && P->v && P->dX && P->dXa) {
        float bestd = 1e30f;
        int bd = 2;
        for (int m = 0; m < 3; ++m) {
            P->departure_mode = m;
            hipEvent_t a, b;
            check_hip(hipEventCreate(&a), "hipEventCreate");
            check_hip(hipEventCreate(&b), "hipEventCreate");
            launch_departure(P, P->v, P->dX, P->dXa);
            check_hip(hipEventRecord(a, P->stream), "hipEventRecord");
            for (int r = 0; r < 3; ++r) launch_departure(P, P->v, P->dX, P->dXa);
            check_hip(hipEventRecord(b, P->stream), "hipEventRecord");
            check_hip(hipEventSynchronize(b), "hipEventSynchronize");
            float ms = 0.f;
            check_hip(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            if (ms < bestd) {
                bestd = ms;
                bd = m;
            }
        }
        P->departure_mode = bd;
    }
    P->gather_tuned = 1;
}

void launch_interp(lddmm_plan *P, int nf, const float *fields, const float *disp, float *out, int kid)
{
    const long N = P->N;
    int f = 0;
    for (; f + 3 <= nf; f += 3) tiled(P, disp, EpiVec3{fields + f * N, out + f * N, N}, kid);
    for (; f < nf; ++f) tiled(P, disp, EpiCopy{fields + f * N, out + f * N}, kid);
}

void launch_adj_coef(lddmm_plan *P)
{
    tiled(P, P->dXa, EpiAdjCoef{P->delta, P->coef, (float)P->dt}, K_ADJ_COEF);
}

void launch_adj_step(lddmm_plan *P, const float *lin, float *lout, float scale)
{
    tiled(P, P->dXa, EpiAdj{lin, P->coef, lout, scale}, K_ADJ_STEP);
}

void launch_incstate_init(lddmm_plan *P, const float *vt, float *mt1)
{
    const float hdt = 0.5f * (float)P->dt;
    switch (P->nt) {
    case 4: tiled(P, P->dX, EpiIncSrc<4>{vt, P->GX, P->G, mt1, P->src, P->N, 4, hdt}, K_INCSTATE_INIT); break;
    case 8: tiled(P, P->dX, EpiIncSrc<8>{vt, P->GX, P->G, mt1, P->src, P->N, 8, hdt}, K_INCSTATE_INIT); break;
    default: tiled(P, P->dX, EpiIncSrc<0>{vt, P->GX, P->G, mt1, P->src, P->N, P->nt, hdt}, K_INCSTATE_INIT); break;
    }
}

void launch_adj_body(lddmm_plan *P, const float *lin, float scale, float *lam0, const float *lam,
                     const float *lamN, float scaleN)
{
    const float dt = (float)P->dt;
#define ADJ_BODY(NTC, NT)                                                                                 \
    tiled(P, P->dXa, EpiAdjBody<NTC>{lin, P->coef, lam0, scale, lam, lamN, scaleN, P->G, P->b, P->N, NT, dt}, \
          K_ADJ_BODY)
    switch (P->nt) {
    case 4: ADJ_BODY(4, 4); break;
    case 8: ADJ_BODY(8, 8); break;
    default: ADJ_BODY(0, P->nt); break;
    }
#undef ADJ_BODY
}

void launch_incstate_step(lddmm_plan *P, const float *min, const float *sj, float *mout)
{
    tiled(P, P->dX, EpiInc{min, sj, mout, 0.5f * (float)P->dt}, K_INCSTATE_STEP);
}

void launch_body_force(lddmm_plan *P, const float *lam, const float *lamN, float scaleN,
                       const float *G, float *b)
{
    Scope s(P, K_BODY_FORCE);
    const long N4 = P->N / 4;
    const dim3 grid((unsigned)((N4 + kPtThreads - 1) / kPtThreads), (unsigned)P->mb.count);
#define BODY(NTC)                                                                                              \
    hipLaunchKernelGGL((k_body_force<NTC>), grid, dim3(kPtThreads), 0, P->stream, (const float4 *)lam,          \
                       (const float4 *)lamN, scaleN, (const float4 *)G, (float4 *)b, N4, P->nt, (float)P->dt, P->mb)
    switch (P->nt) {
    case 4: BODY(4); break;
    case 8: BODY(8); break;
    default: BODY(0); break;
    }
#undef BODY
    check_hip(hipGetLastError(), "k_body_force");
}

}  // namespace lddmm
