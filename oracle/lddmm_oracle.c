/*
 * lddmm_oracle.c -- plain FP64 CPU reference for the Gauss-Newton-Krylov LDDMM
 * hot path (reduced gradient, Gauss-Newton Hessian matvec, PCG, Newton step).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no source
 * with the HIP library: no header, kernel, table or helper.  It is written to
 * be read against the paper (Brunn, Himthani, Biros, Mehl, Mang, "Multi-Node
 * Multi-GPU Diffeomorphic Image Registration for Large-Scale Imaging
 * Problems", arXiv 2008.12820), not to be fast: no blocking, no fusion, no
 * reordering beyond what the definitions state.  OpenMP only distributes
 * independent grid points or FFT lines; every sum over the grid is serial.
 *
 * Conventions (Section 2 "Discretization", Table "Notation"):
 *   domain [0,2pi)^3, periodic; grid n1 x n2 x n3, x3 fastest;
 *   point p = (i*n2 + j)*n3 + k sits at x = (i*h1, j*h2, k*h3), hd = 2pi/nd;
 *   vector fields are stored component-major: v[c*N + p], c = 0,1,2;
 *   N_t time steps of size dt = 1/N_t.
 *
 * Readings where the paper is silent:
 *   RK2 = Heun; the same cubic interpolation evaluates v at the predictor;
 *   cubic Lagrange nodes floor(u)-1 .. floor(u)+2, indices mod n;
 *   the adjoint reaction term is stepped with Heun along the characteristic;
 *   incremental-state source interpolated as 4 fields (m~ and grad m);
 *   trapezoid rule in time for the body force;
 *   first-order spectral symbols use the Nyquist-zeroed wavenumber;
 *   (beta A)^{-1} takes 1/beta on the zero mode;
 *   h^3-weighted inner products; Armijo with c1 = 1e-4, halving, 10 tries;
 *   InvH0: H0 without the Leray projector (as printed), beta0 = max(beta,
 *   5e-2) in H0 and in its inner preconditioner, inner start (beta0 A)^{-1} r,
 *   inner stop relative to ||r||, tolerance eps_H0 times the outer tolerance;
 *   FD8: the standard eighth-order central stencil (coefficients 4/5, -1/5,
 *   4/105, -1/280), used for every first derivative when selected;
 *   trilinear interpolation, when selected, everywhere the cubic one is used
 *   (departure predictor included).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define OR_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------ */
/* DFT and FFT (Section 3.3 uses 3D real FFTs; here the plain complex DFT)  */
/* ------------------------------------------------------------------------ */

/* 0: naive DFT for lines of length <= 32, recursive FFT above;
 * 1: always naive DFT; 2: always recursive FFT. */
static int or_fft_mode = 0;
void or_set_fft_mode(int mode) { or_fft_mode = mode; }

/* W[e] = exp(sign * 2 pi i e / n), e = 0..n-1 */
static cplx *root_table(int n, int sign)
{
    cplx *W = malloc(sizeof(cplx) * (size_t)n);
    for (int e = 0; e < n; e++) {
        double a = 2.0 * OR_PI * (double)e / (double)n;
        W[e] = cos(a) + (double)sign * sin(a) * I;
    }
    return W;
}

/* out[k] = sum_m in[m*stride] * exp(sign 2 pi i m k / n).  W is the table
 * of the top-level length ntop (n divides ntop). */
static void dft_naive(const cplx *in, long stride, cplx *out, int n,
                      const cplx *W, int ntop)
{
    long step = ntop / n;
    for (int k = 0; k < n; k++) {
        cplx s = 0.0;
        for (int m = 0; m < n; m++)
            s += in[m * stride] * W[(((long)m * k) % n) * step];
        out[k] = s;
    }
}

static int smallest_factor(int n)
{
    if (n % 2 == 0) return 2;
    if (n % 3 == 0) return 3;
    if (n % 5 == 0) return 5;
    return n;
}

/* Textbook recursive decimation-in-time mixed-radix FFT:
 * X[k + m s] = sum_r W_n^{r (k + m s)} Y_r[k], Y_r = DFT_m(x[r::p]). */
static void fft_rec(const cplx *in, long stride, cplx *out, int n,
                    const cplx *W, int ntop)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int p = smallest_factor(n);
    if (p == n) {
        dft_naive(in, stride, out, n, W, ntop);
        return;
    }
    int m = n / p;
    for (int r = 0; r < p; r++)
        fft_rec(in + r * stride, stride * p, out + (long)r * m, m, W, ntop);
    long step = ntop / n;
    cplx tmp[n];
    for (int k = 0; k < m; k++) {
        for (int s = 0; s < p; s++) {
            long kk = k + (long)m * s;
            cplx acc = 0.0;
            for (int r = 0; r < p; r++)
                acc += W[(((long)r * kk) % n) * step] * out[(long)r * m + k];
            tmp[kk] = acc;
        }
    }
    memcpy(out, tmp, sizeof(cplx) * (size_t)n);
}

/* Transform every line of a along one axis (unnormalised). */
static void transform_axis(cplx *a, const int n[3], int axis, int sign)
{
    int L = n[axis];
    long st[3] = {(long)n[1] * n[2], n[2], 1};
    long stride = st[axis];
    long nlines = (long)n[0] * n[1] * n[2] / L;
    int naive = (or_fft_mode == 1) || (or_fft_mode == 0 && L <= 32);
    cplx *W = root_table(L, sign);
#pragma omp parallel
    {
        cplx *line = malloc(sizeof(cplx) * (size_t)L);
        cplx *out = malloc(sizeof(cplx) * (size_t)L);
#pragma omp for schedule(static)
        for (long q = 0; q < nlines; q++) {
            long base;
            if (axis == 0) {
                base = q;
            } else if (axis == 1) {
                base = (q / n[2]) * (long)n[1] * n[2] + (q % n[2]);
            } else {
                base = q * n[2];
            }
            for (int m = 0; m < L; m++) line[m] = a[base + m * stride];
            if (naive)
                dft_naive(line, 1, out, L, W, L);
            else
                fft_rec(line, 1, out, L, W, L);
            for (int k = 0; k < L; k++) a[base + k * stride] = out[k];
        }
        free(line);
        free(out);
    }
    free(W);
}

/* hat f(k) = sum_x f(x) e^{-i k.x} (sign -1) or its unnormalised inverse. */
void or_fft3(double *re_im, int n1, int n2, int n3, int sign)
{
    int n[3] = {n1, n2, n3};
    cplx *a = (cplx *)re_im;
    for (int ax = 0; ax < 3; ax++) transform_axis(a, n, ax, sign);
}

static cplx *forward_real(const double *f, const int n[3])
{
    long N = (long)n[0] * n[1] * n[2];
    cplx *F = malloc(sizeof(cplx) * (size_t)N);
    for (long p = 0; p < N; p++) F[p] = f[p];
    for (int ax = 0; ax < 3; ax++) transform_axis(F, n, ax, -1);
    return F;
}

/* f = Re(N^{-1} sum_k F(k) e^{i k.x}); F is overwritten. */
static void inverse_real(cplx *F, double *f, const int n[3])
{
    long N = (long)n[0] * n[1] * n[2];
    for (int ax = 0; ax < 3; ax++) transform_axis(F, n, ax, +1);
    for (long p = 0; p < N; p++) f[p] = creal(F[p]) / (double)N;
}

/* ------------------------------------------------------------------------ */
/* Spectral operators (Section 2: A, its inverse and the Leray projection    */
/* are applied in the spectral domain; first derivatives spectrally as in   */
/* the CPU version of the method, Section 3.2).                             */
/* ------------------------------------------------------------------------ */

/* integer wavenumber of index l along an axis of length n (domain 2pi) */
static double wavenumber(int l, int n) { return (l <= n / 2) ? (double)l : (double)(l - n); }

/* wavenumber for odd-order operators: the Nyquist index gets 0 */
static double wavenumber_odd(int l, int n) { return (2 * l == n) ? 0.0 : wavenumber(l, n); }

static void spectral_index(long p, const int n[3], int l[3])
{
    l[2] = (int)(p % n[2]);
    l[1] = (int)((p / n[2]) % n[1]);
    l[0] = (int)(p / ((long)n[1] * n[2]));
}

/* symbol of A: |k|^2 (H1 seminorm, reg=1) or |k|^4 (H2 seminorm, reg=2) */
static double reg_symbol(const int l[3], const int n[3], int reg)
{
    double k2 = 0.0;
    for (int d = 0; d < 3; d++) {
        double k = wavenumber(l[d], n[d]);
        k2 += k * k;
    }
    return reg == 2 ? k2 * k2 : k2;
}

/* g_d = d f / d x_d, d = 0,1,2 */
void or_spectral_grad(const double *f, double *g, int n1, int n2, int n3)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
    cplx *F = forward_real(f, n);
    cplx *G = malloc(sizeof(cplx) * (size_t)N);
    for (int d = 0; d < 3; d++) {
        for (long p = 0; p < N; p++) {
            int l[3];
            spectral_index(p, n, l);
            G[p] = I * wavenumber_odd(l[d], n[d]) * F[p];
        }
        inverse_real(G, g + d * N, n);
    }
    free(G);
    free(F);
}

/* div v = sum_d d v_d / d x_d */
void or_spectral_div(const double *v, double *out, int n1, int n2, int n3)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
    cplx *S = calloc((size_t)N, sizeof(cplx));
    for (int d = 0; d < 3; d++) {
        cplx *F = forward_real(v + d * N, n);
        for (long p = 0; p < N; p++) {
            int l[3];
            spectral_index(p, n, l);
            S[p] += I * wavenumber_odd(l[d], n[d]) * F[p];
        }
        free(F);
    }
    inverse_real(S, out, n);
    free(S);
}

/* Eighth-order central differences for first derivatives (Section 3.2, the
 * FD kernel that replaces the spectral gradient and divergence): on a
 * periodic axis of spacing h,
 *   df/dx ~= (1/h) sum_{j=1..4} c_j (f(x + j h) - f(x - j h)),
 *   c = (4/5, -1/5, 4/105, -1/280),
 * the unique antisymmetric 9-point stencil exact for polynomials of degree 8. */
static const double fd8_c[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

static double fd8_axis(const double *f, const int n[3], int i, int j, int k, int d)
{
    double s = 0.0, h = 2.0 * OR_PI / n[d];
    for (int q = 1; q <= 4; q++) {
        int ip = i, jp = j, kp = k, im = i, jm = j, km = k;
        if (d == 0) { ip = (i + q) % n[0]; im = (i - q + n[0]) % n[0]; }
        if (d == 1) { jp = (j + q) % n[1]; jm = (j - q + n[1]) % n[1]; }
        if (d == 2) { kp = (k + q) % n[2]; km = (k - q + n[2]) % n[2]; }
        s += fd8_c[q - 1] * (f[((long)ip * n[1] + jp) * n[2] + kp] - f[((long)im * n[1] + jm) * n[2] + km]);
    }
    return s / h;
}

void or_fd8_grad(const double *f, double *g, int n1, int n2, int n3)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
#pragma omp parallel for
    for (int i = 0; i < n1; i++)
        for (int j = 0; j < n2; j++)
            for (int k = 0; k < n3; k++) {
                long p = ((long)i * n2 + j) * n3 + k;
                for (int d = 0; d < 3; d++) g[d * N + p] = fd8_axis(f, n, i, j, k, d);
            }
}

void or_fd8_div(const double *v, double *out, int n1, int n2, int n3)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
#pragma omp parallel for
    for (int i = 0; i < n1; i++)
        for (int j = 0; j < n2; j++)
            for (int k = 0; k < n3; k++) {
                long p = ((long)i * n2 + j) * n3 + k;
                out[p] = fd8_axis(v, n, i, j, k, 0) + fd8_axis(v + N, n, i, j, k, 1) +
                         fd8_axis(v + 2 * N, n, i, j, k, 2);
            }
}

/* out_c = A v_c for each component (ncomp = 1 or 3) */
void or_reg_apply(const double *v, double *out, int ncomp, int n1, int n2, int n3, int reg)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
    for (int c = 0; c < ncomp; c++) {
        cplx *F = forward_real(v + c * N, n);
        for (long p = 0; p < N; p++) {
            int l[3];
            spectral_index(p, n, l);
            F[p] *= reg_symbol(l, n, reg);
        }
        inverse_real(F, out + c * N, n);
        free(F);
    }
}

/* out_c = (beta A)^{-1} v_c; the zero mode is divided by beta alone */
void or_reg_inverse(const double *v, double *out, int ncomp, int n1, int n2, int n3,
                    int reg, double beta)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
    for (int c = 0; c < ncomp; c++) {
        cplx *F = forward_real(v + c * N, n);
        for (long p = 0; p < N; p++) {
            int l[3];
            spectral_index(p, n, l);
            double a = reg_symbol(l, n, reg);
            F[p] *= (a == 0.0) ? 1.0 / beta : 1.0 / (beta * a);
        }
        inverse_real(F, out + c * N, n);
        free(F);
    }
}

/* Leray projection: hat(Pv) = (I - k k^T / |k|^2) hat v with the
 * Nyquist-zeroed wavenumber; identity where that wavenumber vanishes. */
void or_leray(const double *v, double *out, int n1, int n2, int n3)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
    cplx *F[3];
    for (int c = 0; c < 3; c++) F[c] = forward_real(v + c * N, n);
    cplx *Q[3];
    for (int c = 0; c < 3; c++) Q[c] = malloc(sizeof(cplx) * (size_t)N);
    for (long p = 0; p < N; p++) {
        int l[3];
        spectral_index(p, n, l);
        double k[3], kk = 0.0;
        for (int d = 0; d < 3; d++) {
            k[d] = wavenumber_odd(l[d], n[d]);
            kk += k[d] * k[d];
        }
        for (int c = 0; c < 3; c++) {
            cplx s = F[c][p];
            if (kk > 0.0) {
                cplx kv = k[0] * F[0][p] + k[1] * F[1][p] + k[2] * F[2][p];
                s -= k[c] * kv / kk;
            }
            Q[c][p] = s;
        }
    }
    for (int c = 0; c < 3; c++) {
        inverse_real(Q[c], out + c * N, n);
        free(Q[c]);
        free(F[c]);
    }
}

/* ------------------------------------------------------------------------ */
/* Cubic Lagrange interpolation (Section 3.1, formula with d = 3)            */
/* ------------------------------------------------------------------------ */

/* Lagrange basis on the nodes -1, 0, 1, 2 evaluated at t in [0,1) */
static void lagrange_cubic(double t, double w[4])
{
    w[0] = -t * (t - 1.0) * (t - 2.0) / 6.0;
    w[1] = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
    w[2] = -(t + 1.0) * t * (t - 2.0) / 2.0;
    w[3] = (t + 1.0) * t * (t - 1.0) / 6.0;
}

static long wrap_index(long i, int n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

/* out[f*nq + q] = I[field f](y_q), y given component-major y[c*nq + q]
 * in physical coordinates.  Direct 64-term tensor-product sum. */
void or_interp(const double *fields, int nf, int n1, int n2, int n3,
               const double *y, long nq, double *out)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
#pragma omp parallel for schedule(static)
    for (long q = 0; q < nq; q++) {
        double w[3][4];
        long idx[3][4];
        for (int d = 0; d < 3; d++) {
            double h = 2.0 * OR_PI / n[d];
            double u = y[d * nq + q] / h;
            double b = floor(u);
            lagrange_cubic(u - b, w[d]);
            for (int r = 0; r < 4; r++) idx[d][r] = wrap_index((long)b - 1 + r, n[d]);
        }
        for (int f = 0; f < nf; f++) {
            const double *F = fields + (long)f * N;
            double s = 0.0;
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++)
                    for (int c = 0; c < 4; c++)
                        s += F[(idx[0][a] * n2 + idx[1][b]) * n3 + idx[2][c]] *
                             w[0][a] * w[1][b] * w[2][c];
            out[(long)f * nq + q] = s;
        }
    }
}

/* The same with first-order (trilinear) Lagrange interpolation, d = 1 in
 * the formula of Section 3.1: nodes floor(u) and floor(u)+1, weights 1-t, t. */
void or_interp_linear(const double *fields, int nf, int n1, int n2, int n3,
                      const double *y, long nq, double *out)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
#pragma omp parallel for schedule(static)
    for (long q = 0; q < nq; q++) {
        double w[3][2];
        long idx[3][2];
        for (int d = 0; d < 3; d++) {
            double h = 2.0 * OR_PI / n[d];
            double u = y[d * nq + q] / h;
            double b = floor(u);
            w[d][0] = 1.0 - (u - b);
            w[d][1] = u - b;
            for (int r = 0; r < 2; r++) idx[d][r] = wrap_index((long)b + r, n[d]);
        }
        for (int f = 0; f < nf; f++) {
            const double *F = fields + (long)f * N;
            double s = 0.0;
            for (int a = 0; a < 2; a++)
                for (int b = 0; b < 2; b++)
                    for (int c = 0; c < 2; c++)
                        s += F[(idx[0][a] * n2 + idx[1][b]) * n3 + idx[2][c]] *
                             w[0][a] * w[1][b] * w[2][c];
            out[(long)f * nq + q] = s;
        }
    }
}

/* order 3 (cubic, the default) or 1 (trilinear) */
static void interp_order(int order, const double *fields, int nf, const int n[3], const double *y, long nq,
                         double *out)
{
    if (order == 1)
        or_interp_linear(fields, nf, n[0], n[1], n[2], y, nq, out);
    else
        or_interp(fields, nf, n[0], n[1], n[2], y, nq, out);
}

/* physical coordinates of all grid points, component-major */
static double *grid_points(const int n[3])
{
    long N = (long)n[0] * n[1] * n[2];
    double *x = malloc(sizeof(double) * 3 * (size_t)N);
    for (long p = 0; p < N; p++) {
        int l[3];
        spectral_index(p, n, l);
        for (int d = 0; d < 3; d++) x[d * N + p] = l[d] * (2.0 * OR_PI / n[d]);
    }
    return x;
}

/* ------------------------------------------------------------------------ */
/* Characteristics (Section 2 "Discretization": backward trajectories of    */
/* grid points, RK2 for dy/dt = v(y) with y(t+dt) = x)                      */
/* ------------------------------------------------------------------------ */

/* X  = x - dt/2 (v(x) + v(x - dt v(x)))   (state and incremental state)
 * Xa = x + dt/2 (v(x) + v(x + dt v(x)))   (adjoints: transport along -v) */
static void departure_order(int order, const double *v, int n1, int n2, int n3, int nt, double *X,
                            double *Xa);

void or_departure(const double *v, int n1, int n2, int n3, int nt, double *X, double *Xa)
{
    departure_order(3, v, n1, n2, n3, nt, X, Xa);
}

/* the departure points with the interpolation of the given order at the predictor */
static void departure_order(int order, const double *v, int n1, int n2, int n3, int nt, double *X,
                            double *Xa)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
    double dt = 1.0 / nt;
    double *x = grid_points(n);
    double *y = malloc(sizeof(double) * 3 * (size_t)N);
    double *vy = malloc(sizeof(double) * 3 * (size_t)N);
    for (int dir = 0; dir < 2; dir++) {
        double s = dir == 0 ? -1.0 : 1.0;
        double *out = dir == 0 ? X : Xa;
        for (long i = 0; i < 3 * N; i++) y[i] = x[i] + s * dt * v[i];
        interp_order(order, v, 3, n, y, N, vy);
        for (long i = 0; i < 3 * N; i++) out[i] = x[i] + s * 0.5 * dt * (v[i] + vy[i]);
    }
    free(vy);
    free(y);
    free(x);
}

/* The same two departure points (cubic predictor) at nq chosen grid points
 * only, given by their indices idx[3][nq]: for checks at grid sizes where the
 * whole field would take too long.  X, Xa: [3][nq]. */
void or_departure_points(const double *v, int n1, int n2, int n3, int nt, const long *idx, long nq,
                         double *X, double *Xa)
{
    int n[3] = {n1, n2, n3};
    long N = (long)n1 * n2 * n3;
    double dt = 1.0 / nt;
    double *x = malloc(sizeof(double) * 3 * (size_t)nq);
    double *vx = malloc(sizeof(double) * 3 * (size_t)nq);
    double *y = malloc(sizeof(double) * 3 * (size_t)nq);
    double *vy = malloc(sizeof(double) * 3 * (size_t)nq);
    for (long q = 0; q < nq; q++) {
        long p = (idx[q] * n2 + idx[nq + q]) * n3 + idx[2 * nq + q];
        for (int d = 0; d < 3; d++) {
            x[d * nq + q] = idx[d * nq + q] * (2.0 * OR_PI / n[d]);
            vx[d * nq + q] = v[d * N + p];
        }
    }
    for (int dir = 0; dir < 2; dir++) {
        double s = dir == 0 ? -1.0 : 1.0;
        double *out = dir == 0 ? X : Xa;
        for (long i = 0; i < 3 * nq; i++) y[i] = x[i] + s * dt * vx[i];
        or_interp(v, 3, n1, n2, n3, y, nq, vy);
        for (long i = 0; i < 3 * nq; i++) out[i] = x[i] + s * 0.5 * dt * (vx[i] + vy[i]);
    }
    free(vy);
    free(y);
    free(vx);
    free(x);
}

/* ------------------------------------------------------------------------ */
/* Problem context                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n[3];
    long N;
    int nt;
    int reg;
    double beta;
    int leray;
    double h3;
    double *m0, *m1, *v;  /* copies of the inputs */
    double *X, *Xa;       /* departure points, [3][N] */
    double *m;            /* state m_j, [nt+1][N] */
    double *G;            /* grad m_j, [nt+1][3][N] */
    double *delta;        /* div v */
    double *delta_a;      /* div v at Xa */
    int have_images, have_velocity;
    double g0norm;        /* norm of the first gradient after set_images */
    int fd8;              /* first derivatives: 0 spectral, 1 eighth-order FD */
    int ip;               /* interpolation order: 3 cubic (default), 1 trilinear */
} or_ctx;

static void ctx_interp(const or_ctx *c, const double *fields, int nf, const double *y, double *out)
{
    interp_order(c->ip, fields, nf, c->n, y, c->N, out);
}

/* interpolation order 3 or 1; takes effect at the next velocity */
void or_ctx_set_ip_order(or_ctx *c, int order) { c->ip = order == 1 ? 1 : 3; }

/* the regularisation weight (for beta-continuation); the velocity state does
 * not depend on it */
void or_ctx_set_beta(or_ctx *c, double beta)
{
    c->beta = beta;
    c->g0norm = 0.0;  /* a new beta starts a new Newton solve: ||g||_rel from its first gradient */
}

/* grad of a scalar and div of a vector field with the context's scheme */
static void ctx_grad(const or_ctx *c, const double *f, double *g)
{
    if (c->fd8)
        or_fd8_grad(f, g, c->n[0], c->n[1], c->n[2]);
    else
        or_spectral_grad(f, g, c->n[0], c->n[1], c->n[2]);
}

static void ctx_div(const or_ctx *c, const double *v, double *out)
{
    if (c->fd8)
        or_fd8_div(v, out, c->n[0], c->n[1], c->n[2]);
    else
        or_spectral_div(v, out, c->n[0], c->n[1], c->n[2]);
}

/* choose the first-derivative scheme; takes effect at the next velocity */
void or_ctx_set_fd8(or_ctx *c, int on) { c->fd8 = on ? 1 : 0; }

or_ctx *or_ctx_create(int n1, int n2, int n3, int nt, int reg, double beta, int leray)
{
    or_ctx *c = calloc(1, sizeof(or_ctx));
    c->n[0] = n1;
    c->n[1] = n2;
    c->n[2] = n3;
    c->N = (long)n1 * n2 * n3;
    c->nt = nt;
    c->reg = reg;
    c->beta = beta;
    c->leray = leray;
    c->ip = 3;
    c->h3 = (2.0 * OR_PI / n1) * (2.0 * OR_PI / n2) * (2.0 * OR_PI / n3);
    long N = c->N;
    c->m0 = malloc(sizeof(double) * N);
    c->m1 = malloc(sizeof(double) * N);
    c->v = malloc(sizeof(double) * 3 * N);
    c->X = malloc(sizeof(double) * 3 * N);
    c->Xa = malloc(sizeof(double) * 3 * N);
    c->m = malloc(sizeof(double) * (nt + 1) * N);
    c->G = malloc(sizeof(double) * (nt + 1) * 3 * N);
    c->delta = malloc(sizeof(double) * N);
    c->delta_a = malloc(sizeof(double) * N);
    return c;
}

void or_ctx_destroy(or_ctx *c)
{
    if (!c) return;
    free(c->m0);
    free(c->m1);
    free(c->v);
    free(c->X);
    free(c->Xa);
    free(c->m);
    free(c->G);
    free(c->delta);
    free(c->delta_a);
    free(c);
}

/* <a,b> = h^3 sum_i a_i b_i (serial, fixed order) */
double or_inner(const double *a, const double *b, long count, double h3)
{
    double s = 0.0;
    for (long i = 0; i < count; i++) s += a[i] * b[i];
    return h3 * s;
}

/* state: m_0 = m0, m_{j+1} = I[m_j](X) (transport equation, semi-Lagrangian) */
static void solve_state(const or_ctx *c, const double *m0, double *m)
{
    long N = c->N;
    memcpy(m, m0, sizeof(double) * N);
    for (int j = 0; j < c->nt; j++)
        ctx_interp(c, m + j * N, 1, c->X, m + (j + 1) * N);
}

void or_ctx_set_images(or_ctx *c, const double *m0, const double *m1)
{
    memcpy(c->m0, m0, sizeof(double) * c->N);
    memcpy(c->m1, m1, sizeof(double) * c->N);
    c->have_images = 1;
    c->have_velocity = 0;
    c->g0norm = 0.0;
}

/* everything that depends on v only: X, Xa, m_j, grad m_j, div v, div v at Xa */
void or_ctx_set_velocity(or_ctx *c, const double *v)
{
    long N = c->N;
    memcpy(c->v, v, sizeof(double) * 3 * N);
    departure_order(c->ip, c->v, c->n[0], c->n[1], c->n[2], c->nt, c->X, c->Xa);
    solve_state(c, c->m0, c->m);
    for (int j = 0; j <= c->nt; j++) ctx_grad(c, c->m + j * N, c->G + (long)j * 3 * N);
    ctx_div(c, c->v, c->delta);
    ctx_interp(c, c->delta, 1, c->Xa, c->delta_a);
    c->have_velocity = 1;
}

/* Adjoint transport (eq. adjoint): -d_t lam - div(lam v) = 0, final value phi.
 * Along the characteristics of -v the equation reads d lam/ds = lam div v;
 * one Heun step on that reaction term per time step:
 *   l = I[lam_{j+1}](Xa); r0 = l*delta(Xa); lam* = l + dt r0;
 *   r1 = lam* delta(x); lam_j = l + dt/2 (r0 + r1). */
void or_ctx_adjoint(const or_ctx *c, const double *phi, double *lam)
{
    long N = c->N;
    double dt = 1.0 / c->nt;
    memcpy(lam + (long)c->nt * N, phi, sizeof(double) * N);
    double *l = malloc(sizeof(double) * N);
    for (int j = c->nt - 1; j >= 0; j--) {
        ctx_interp(c, lam + (long)(j + 1) * N, 1, c->Xa, l);
        for (long p = 0; p < N; p++) {
            double r0 = l[p] * c->delta_a[p];
            double ls = l[p] + dt * r0;
            double r1 = ls * c->delta[p];
            lam[(long)j * N + p] = l[p] + 0.5 * dt * (r0 + r1);
        }
    }
    free(l);
}

/* body force b = int_0^1 lam grad m dt, trapezoid rule in time */
void or_ctx_body_force(const or_ctx *c, const double *lam, double *b)
{
    long N = c->N;
    double dt = 1.0 / c->nt;
    for (long i = 0; i < 3 * N; i++) b[i] = 0.0;
    for (int j = 0; j <= c->nt; j++) {
        double w = (j == 0 || j == c->nt) ? 0.5 : 1.0;
        for (int d = 0; d < 3; d++)
            for (long p = 0; p < N; p++)
                b[d * N + p] += dt * w * lam[(long)j * N + p] * c->G[((long)j * 3 + d) * N + p];
    }
}

/* beta A w + K b with K = Leray projection or identity */
static void assemble(const or_ctx *c, const double *w, const double *b, double *out)
{
    long N = c->N;
    double *Aw = malloc(sizeof(double) * 3 * N);
    or_reg_apply(w, Aw, 3, c->n[0], c->n[1], c->n[2], c->reg);
    if (c->leray) {
        double *Pb = malloc(sizeof(double) * 3 * N);
        or_leray(b, Pb, c->n[0], c->n[1], c->n[2]);
        for (long i = 0; i < 3 * N; i++) out[i] = c->beta * Aw[i] + Pb[i];
        free(Pb);
    } else {
        for (long i = 0; i < 3 * N; i++) out[i] = c->beta * Aw[i] + b[i];
    }
    free(Aw);
}

/* objective (eq. problem): J = 1/2 ||m(1) - m1||^2 + beta/2 <A v, v> */
void or_ctx_objective(const or_ctx *c, double out[3])
{
    long N = c->N;
    double *r = malloc(sizeof(double) * N);
    for (long p = 0; p < N; p++) r[p] = c->m[(long)c->nt * N + p] - c->m1[p];
    double mis = 0.5 * or_inner(r, r, N, c->h3);
    double *Av = malloc(sizeof(double) * 3 * N);
    or_reg_apply(c->v, Av, 3, c->n[0], c->n[1], c->n[2], c->reg);
    double reg = 0.5 * c->beta * or_inner(Av, c->v, 3 * N, c->h3);
    out[0] = mis + reg;
    out[1] = mis;
    out[2] = reg;
    free(Av);
    free(r);
}

/* reduced gradient (eq. reducedgrad): g = beta A v + K int lam grad m dt,
 * lam from the adjoint equation with final value m1 - m(1) */
void or_ctx_gradient(or_ctx *c, double *g)
{
    long N = c->N;
    double *phi = malloc(sizeof(double) * N);
    for (long p = 0; p < N; p++) phi[p] = c->m1[p] - c->m[(long)c->nt * N + p];
    double *lam = malloc(sizeof(double) * (c->nt + 1) * N);
    or_ctx_adjoint(c, phi, lam);
    double *b = malloc(sizeof(double) * 3 * N);
    or_ctx_body_force(c, lam, b);
    assemble(c, c->v, b, g);
    if (c->g0norm == 0.0) c->g0norm = sqrt(or_inner(g, g, 3 * N, c->h3));
    free(b);
    free(lam);
    free(phi);
}

/* incremental state (eq. incsta): d_t m~ + v.grad m~ + v~.grad m = 0, m~(0) = 0.
 * Heun along the characteristics with the source f_j = -v~ . grad m_j:
 *   m~_{j+1} = I[m~_j](X) - dt/2 ( I[v~](X) . I[grad m_j](X) + v~ . grad m_{j+1} ) */
void or_ctx_inc_state(const or_ctx *c, const double *vt, double *mt)
{
    long N = c->N;
    double dt = 1.0 / c->nt;
    double *vtX = malloc(sizeof(double) * 3 * N);
    ctx_interp(c, vt, 3, c->X, vtX);
    double *GX = malloc(sizeof(double) * 3 * N);
    double *mX = malloc(sizeof(double) * N);
    for (long p = 0; p < N; p++) mt[p] = 0.0;
    for (int j = 0; j < c->nt; j++) {
        ctx_interp(c, mt + (long)j * N, 1, c->X, mX);
        ctx_interp(c, c->G + (long)j * 3 * N, 3, c->X, GX);
        const double *G1 = c->G + (long)(j + 1) * 3 * N;
        for (long p = 0; p < N; p++) {
            double s0 = 0.0, s1 = 0.0;
            for (int d = 0; d < 3; d++) {
                s0 += vtX[d * N + p] * GX[d * N + p];
                s1 += vt[d * N + p] * G1[d * N + p];
            }
            mt[(long)(j + 1) * N + p] = mX[p] - 0.5 * dt * (s0 + s1);
        }
    }
    free(mX);
    free(GX);
    free(vtX);
}

/* Gauss-Newton matvec (eq. matvec): H v~ = beta A v~ + K int lam~ grad m dt,
 * lam~ from the incremental adjoint (eq. incadj) with final value -m~(1) */
void or_ctx_matvec(const or_ctx *c, const double *vt, double *hvt)
{
    long N = c->N;
    int nt = c->nt;
    double *mt = malloc(sizeof(double) * (nt + 1) * N);
    or_ctx_inc_state(c, vt, mt);
    double *phi = malloc(sizeof(double) * N);
    for (long p = 0; p < N; p++) phi[p] = -mt[(long)nt * N + p];
    double *lam = malloc(sizeof(double) * (nt + 1) * N);
    or_ctx_adjoint(c, phi, lam);
    double *b = malloc(sizeof(double) * 3 * N);
    or_ctx_body_force(c, lam, b);
    assemble(c, vt, b, hvt);
    free(b);
    free(lam);
    free(phi);
    free(mt);
}

/* Read back one precomputed array.  what: 0 X, 1 Xa (3N each), 2 m_j (N),
 * 3 grad m_j (3N), 4 div v (N), 5 div v at Xa (N), 6 v (3N). */
void or_ctx_get(const or_ctx *c, int what, int j, double *out)
{
    long N = c->N;
    switch (what) {
    case 0: memcpy(out, c->X, sizeof(double) * 3 * N); break;
    case 1: memcpy(out, c->Xa, sizeof(double) * 3 * N); break;
    case 2: memcpy(out, c->m + (long)j * N, sizeof(double) * N); break;
    case 3: memcpy(out, c->G + (long)j * 3 * N, sizeof(double) * 3 * N); break;
    case 4: memcpy(out, c->delta, sizeof(double) * N); break;
    case 5: memcpy(out, c->delta_a, sizeof(double) * N); break;
    case 6: memcpy(out, c->v, sizeof(double) * 3 * N); break;
    default: break;
    }
}

/* ------------------------------------------------------------------------ */
/* PCG and Gauss-Newton (eq. iter, Algorithm "GNK", preconditioner InvA)    */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* Zero-velocity Hessian preconditioner InvH0 (Section 2 "Preconditioning", */
/* eq. h0-pc, Algorithm "PC", first function)                               */
/* ------------------------------------------------------------------------ */

/* beta inside H0: the problem's beta, bounded below by 5e-2 */
static double h0_beta(const or_ctx *c) { return c->beta < 5e-2 ? 5e-2 : c->beta; }

/* out = H0 s = beta0 A s + grad m (grad m . s) with m the deformed template
 * m(1) = m_{N_t} at the current velocity (the paper refreshes m0 in H0 with
 * the template transported by the current iterate) and beta0 = h0_beta. */
/* out = beta0 A s + G (G . s) on an n[0] x n[1] x n[2] grid */
static void h0_apply_grid(const double *G, const int n[3], int reg, double b0, const double *s,
                          double *out)
{
    long N = (long)n[0] * n[1] * n[2];
    or_reg_apply(s, out, 3, n[0], n[1], n[2], reg);
    for (long p = 0; p < N; p++) {
        double gs = G[p] * s[p] + G[N + p] * s[N + p] + G[2 * N + p] * s[2 * N + p];
        for (int d = 0; d < 3; d++) out[d * N + p] = b0 * out[d * N + p] + G[d * N + p] * gs;
    }
}

void or_ctx_h0_apply(const or_ctx *c, const double *s, double *out)
{
    h0_apply_grid(c->G + (long)c->nt * 3 * c->N, c->n, c->reg, h0_beta(c), s, out);
}

/* s ~= H0^{-1} r: PCG on H0 s = r, preconditioned by (beta0 A)^{-1}, started
 * from s = (beta0 A)^{-1} r; stops when ||r - H0 s|| <= tol ||r|| (the
 * unweighted L2 norm, as the outer PCG), after max_it iterations, or when
 * <p, H0 p> <= 0.  Returns the iterations taken. */
/* PCG on H0 s = r over an n-grid (G its grad m, cell volume h3), from the
 * start s0 given in s, preconditioned by (beta0 A)^{-1}; the stopping rule of
 * or_ctx_invh0.  Returns the iterations. */
static int h0_pcg_grid(const double *G, const int n[3], int reg, double b0, double h3,
                       const double *r, double tol, int max_it, double *s)
{
    long M = 3L * n[0] * n[1] * n[2];
    double *ri = malloc(sizeof(double) * M);
    double *zi = malloc(sizeof(double) * M);
    double *pi = malloc(sizeof(double) * M);
    double *qi = malloc(sizeof(double) * M);
    double rn0 = sqrt(or_inner(r, r, M, h3));
    int it = 0;
    if (rn0 > 0.0) {
        h0_apply_grid(G, n, reg, b0, s, qi);
        for (long i = 0; i < M; i++) ri[i] = r[i] - qi[i];
        double rn = sqrt(or_inner(ri, ri, M, h3));
        if (rn > tol * rn0) {
            or_reg_inverse(ri, zi, 3, n[0], n[1], n[2], reg, b0);
            memcpy(pi, zi, sizeof(double) * M);
            double rz = or_inner(ri, zi, M, h3);
            while (it < max_it) {
                h0_apply_grid(G, n, reg, b0, pi, qi);
                it++;
                double kappa = or_inner(pi, qi, M, h3);
                if (!(kappa > 0.0)) break;
                double alpha = rz / kappa;
                for (long i = 0; i < M; i++) {
                    s[i] += alpha * pi[i];
                    ri[i] -= alpha * qi[i];
                }
                rn = sqrt(or_inner(ri, ri, M, h3));
                if (rn <= tol * rn0) break;
                or_reg_inverse(ri, zi, 3, n[0], n[1], n[2], reg, b0);
                double rz_new = or_inner(ri, zi, M, h3);
                double bet = rz_new / rz;
                rz = rz_new;
                for (long i = 0; i < M; i++) pi[i] = zi[i] + bet * pi[i];
            }
        }
    }
    free(ri); free(zi); free(pi); free(qi);
    return it;
}

int or_ctx_invh0(const or_ctx *c, const double *r, double tol, int max_it, double *s)
{
    double b0 = h0_beta(c);
    or_reg_inverse(r, s, 3, c->n[0], c->n[1], c->n[2], c->reg, b0);
    return h0_pcg_grid(c->G + (long)c->nt * 3 * c->N, c->n, c->reg, b0, c->h3, r, tol, max_it, s);
}

/* ------------------------------------------------------------------------ */
/* Two-level variant 2LInvH0 (Section 2 "Preconditioning", Algorithm "PC", */
/* second function): H0 inverted on a grid of half the resolution.          */
/* ------------------------------------------------------------------------ */

/* Spectral restriction of ncomp fields from the fine grid nf to the coarse
 * grid nc = nf/2: the coarse field keeps the fine Fourier coefficients of
 * the wavenumbers |k_d| < nc_d/2 (the coarse Nyquist modes are dropped), so a
 * band-limited field restricts to its samples on the coarse grid. */
void or_restrict(const double *f, double *out, int ncomp, int n1, int n2, int n3)
{
    int nf[3] = {n1, n2, n3}, nc[3] = {n1 / 2, n2 / 2, n3 / 2};
    long Nf = (long)n1 * n2 * n3, Nc = (long)nc[0] * nc[1] * nc[2];
    for (int c = 0; c < ncomp; c++) {
        cplx *F = forward_real(f + c * Nf, nf);
        cplx *C = malloc(sizeof(cplx) * (size_t)Nc);
        for (long q = 0; q < Nc; q++) {
            int l[3], lf[3], keep = 1;
            spectral_index(q, nc, l);
            for (int d = 0; d < 3; d++) {
                int k = (int)wavenumber(l[d], nc[d]);
                if (2 * abs(k) == nc[d]) keep = 0;
                lf[d] = (k + nf[d]) % nf[d];
            }
            C[q] = keep ? F[((long)lf[0] * nf[1] + lf[1]) * nf[2] + lf[2]] * ((double)Nc / (double)Nf) : 0.0;
        }
        inverse_real(C, out + c * Nc, nc);
        free(C);
        free(F);
    }
}

/* Spectral prolongation (zero padding) of ncomp coarse fields on nc to the
 * fine grid 2 nc: the coarse coefficients of |k_d| < nc_d/2 move to the same
 * wavenumbers of the fine spectrum, every other fine coefficient is zero. */
void or_prolong(const double *f, double *out, int ncomp, int n1c, int n2c, int n3c)
{
    int nc[3] = {n1c, n2c, n3c}, nf[3] = {2 * n1c, 2 * n2c, 2 * n3c};
    long Nc = (long)n1c * n2c * n3c, Nf = 8 * Nc;
    for (int c = 0; c < ncomp; c++) {
        cplx *C = forward_real(f + c * Nc, nc);
        cplx *F = calloc((size_t)Nf, sizeof(cplx));
        for (long q = 0; q < Nc; q++) {
            int l[3], lf[3], keep = 1;
            spectral_index(q, nc, l);
            for (int d = 0; d < 3; d++) {
                int k = (int)wavenumber(l[d], nc[d]);
                if (2 * abs(k) == nc[d]) keep = 0;
                lf[d] = (k + nf[d]) % nf[d];
            }
            if (keep) F[((long)lf[0] * nf[1] + lf[1]) * nf[2] + lf[2]] = C[q] * ((double)Nf / (double)Nc);
        }
        inverse_real(F, out + c * Nf, nf);
        free(F);
        free(C);
    }
}

/* s ~= 2LInvH0(r), the steps of Algorithm "PC" (second function):
 *   s_f = (beta0 A)^{-1} r;  s_c = Restrict(s_f);
 *   s_c <- PCG on H0_c s_c = Restrict(r) from s_c, preconditioned by
 *          (beta0 A_c)^{-1}, H0_c built from Restrict(grad m(1)), relative
 *          tolerance tol, at most max_it iterations;
 *   s_f = Prolong(s_c) + HighPass(s_f),  HighPass(f) = f - Prolong(Restrict(f)).
 * The fine grid must halve to a valid grid.  Returns the coarse iterations. */
int or_ctx_2linvh0(const or_ctx *c, const double *r, double tol, int max_it, double *s)
{
    int nc[3] = {c->n[0] / 2, c->n[1] / 2, c->n[2] / 2};
    long Mf = 3 * c->N, Mc = 3L * nc[0] * nc[1] * nc[2];
    double b0 = h0_beta(c), h3c = 8.0 * c->h3;
    double *sc = malloc(sizeof(double) * Mc);
    double *rc = malloc(sizeof(double) * Mc);
    double *Gc = malloc(sizeof(double) * Mc);
    double *lo = malloc(sizeof(double) * Mf);
    or_reg_inverse(r, s, 3, c->n[0], c->n[1], c->n[2], c->reg, b0);
    or_restrict(s, sc, 3, c->n[0], c->n[1], c->n[2]);
    or_restrict(r, rc, 3, c->n[0], c->n[1], c->n[2]);
    or_restrict(c->G + (long)c->nt * 3 * c->N, Gc, 3, c->n[0], c->n[1], c->n[2]);
    /* the high-pass part of s_f: s_f - Prolong(Restrict(s_f)) */
    or_prolong(sc, lo, 3, nc[0], nc[1], nc[2]);
    for (long i = 0; i < Mf; i++) s[i] -= lo[i];
    int it = h0_pcg_grid(Gc, nc, c->reg, b0, h3c, rc, tol, max_it, sc);
    or_prolong(sc, lo, 3, nc[0], nc[1], nc[2]);
    for (long i = 0; i < Mf; i++) s[i] += lo[i];
    free(sc); free(rc); free(Gc); free(lo);
    return it;
}

/* the preconditioner M^{-1}: pc 0 = InvA, (beta A)^{-1}; pc 1 = InvH0, pc 2
 * = 2LInvH0, with the inner tolerance tol_h0 and at most max_inner inner
 * iterations.
 * Returns the inner iterations. */
static int precondition(const or_ctx *c, const double *r, double *z, int pc, double tol_h0,
                        int max_inner)
{
    if (pc == 1) return or_ctx_invh0(c, r, tol_h0, max_inner, z);
    if (pc == 2) return or_ctx_2linvh0(c, r, tol_h0, max_inner, z);
    or_reg_inverse(r, z, 3, c->n[0], c->n[1], c->n[2], c->reg, c->beta);
    return 0;
}

/* Preconditioned CG for H x = rhs, x0 = 0, M^{-1} from precondition() (InvA
 * or InvH0 with the inner tolerance eps_h0 * rtol, Algorithm "PC").
 * Stops when ||r|| <= rtol ||r0||, after max_it matvecs, or when
 * <p, H p> <= 0 (then the current x; at the first iteration M^{-1} r0).
 * info: [0] iterations (matvecs), [1] ||r||/||r0||, [2] flags
 * (1 negative curvature, 2 non-finite), [3] ||r0||, [4] inner iterations of
 * the preconditioner (summed).  hist (may be NULL, max_it entries): after
 * iteration k + 1, hist[k] = ||r|| / ||r0|| (the current value when the
 * iteration stopped at the curvature test).  Returns flags. */
int or_ctx_pcg_hist(const or_ctx *c, const double *rhs, int max_it, double rtol, int pc,
                    double eps_h0, int max_inner, double *x, double *info, double *hist)
{
    long M = 3 * c->N;
    double h3 = c->h3, tol_h0 = eps_h0 * rtol;
    double *r = malloc(sizeof(double) * M);
    double *z = malloc(sizeof(double) * M);
    double *p = malloc(sizeof(double) * M);
    double *q = malloc(sizeof(double) * M);
    for (long i = 0; i < M; i++) {
        x[i] = 0.0;
        r[i] = rhs[i];
    }
    double r0 = sqrt(or_inner(r, r, M, h3));
    int it = 0, flags = 0, inner = 0;
    double rn = r0;
    if (r0 == 0.0) {
        info[0] = 0; info[1] = 0.0; info[2] = 0; info[3] = 0.0; info[4] = 0;
        free(r); free(z); free(p); free(q);
        return 0;
    }
    inner += precondition(c, r, z, pc, tol_h0, max_inner);
    memcpy(p, z, sizeof(double) * M);
    double rz = or_inner(r, z, M, h3);
    while (it < max_it) {
        or_ctx_matvec(c, p, q);
        it++;
        if (hist) hist[it - 1] = rn / r0;
        double kappa = or_inner(p, q, M, h3);
        if (!isfinite(kappa)) {
            flags |= 2;
            break;
        }
        if (kappa <= 0.0) {
            flags |= 1;
            if (it == 1) memcpy(x, z, sizeof(double) * M);  /* z = M^{-1} r0 */
            break;
        }
        double alpha = rz / kappa;
        for (long i = 0; i < M; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        rn = sqrt(or_inner(r, r, M, h3));
        if (hist) hist[it - 1] = rn / r0;
        if (rn <= rtol * r0) break;
        inner += precondition(c, r, z, pc, tol_h0, max_inner);
        double rz_new = or_inner(r, z, M, h3);
        double bet = rz_new / rz;
        rz = rz_new;
        for (long i = 0; i < M; i++) p[i] = z[i] + bet * p[i];
    }
    info[0] = it;
    info[1] = rn / r0;
    info[2] = flags;
    info[3] = r0;
    info[4] = inner;
    free(r); free(z); free(p); free(q);
    return flags;
}

int or_ctx_pcg_pc(const or_ctx *c, const double *rhs, int max_it, double rtol, int pc,
                  double eps_h0, int max_inner, double *x, double *info)
{
    return or_ctx_pcg_hist(c, rhs, max_it, rtol, pc, eps_h0, max_inner, x, info, NULL);
}

/* PCG with M^{-1} = (beta A)^{-1} (preconditioner InvA); info [0..3] */
int or_ctx_pcg(const or_ctx *c, const double *rhs, int max_it, double rtol, double *x,
               double *info)
{
    double inf5[5];
    int flags = or_ctx_pcg_pc(c, rhs, max_it, rtol, 0, 0.0, 0, x, inf5);
    for (int k = 0; k < 4; k++) info[k] = inf5[k];
    return flags;
}

/* One Gauss-Newton iteration at the current velocity:
 * g, J; eps_K = min(sqrt(||g||/||g0||), 0.5) when rtol <= 0;
 * PCG on H v~ = -g; Armijo: alpha = 1, accept when
 * J(v + alpha v~) <= J(v) + 1e-4 alpha <g, v~>, else halve (10 tries);
 * then v <- v + alpha v~ and the context is refreshed.
 * v_out receives the new velocity.  info: [0] pcg its, [1] rel res, [2] flags,
 * [3] alpha (0 if the search failed), [4] J before, [5] J after,
 * [6] ||g||/||g0||, [7] ||g||, [8] inner preconditioner iterations. */
int or_ctx_gn_iterate_pc(or_ctx *c, int max_pcg, double rtol, int pc, double eps_h0, int max_inner,
                         double *v_out, double *info)
{
    long M = 3 * c->N;
    double *g = malloc(sizeof(double) * M);
    double *mg = malloc(sizeof(double) * M);
    double *vt = malloc(sizeof(double) * M);
    double *v0 = malloc(sizeof(double) * M);
    double *vn = malloc(sizeof(double) * M);
    memcpy(v0, c->v, sizeof(double) * M);
    or_ctx_gradient(c, g);
    double gnorm = sqrt(or_inner(g, g, M, c->h3));
    double grel = c->g0norm > 0.0 ? gnorm / c->g0norm : 1.0;
    double J0[3];
    or_ctx_objective(c, J0);
    double tol = rtol > 0.0 ? rtol : fmin(sqrt(grel), 0.5);
    for (long i = 0; i < M; i++) mg[i] = -g[i];
    double pinfo[5];
    int flags = or_ctx_pcg_pc(c, mg, max_pcg, tol, pc, eps_h0, max_inner, vt, pinfo);
    double gv = or_inner(g, vt, M, c->h3);
    double alpha = 1.0, Jn[3] = {J0[0], J0[1], J0[2]};
    int ok = 0;
    for (int tries = 0; tries < 10; tries++) {
        for (long i = 0; i < M; i++) vn[i] = v0[i] + alpha * vt[i];
        or_ctx_set_velocity(c, vn);
        or_ctx_objective(c, Jn);
        if (Jn[0] <= J0[0] + 1e-4 * alpha * gv) {
            ok = 1;
            break;
        }
        alpha *= 0.5;
    }
    if (!ok) {
        or_ctx_set_velocity(c, v0);
        memcpy(vn, v0, sizeof(double) * M);
        Jn[0] = J0[0];
        alpha = 0.0;
    }
    memcpy(v_out, vn, sizeof(double) * M);
    info[0] = pinfo[0];
    info[1] = pinfo[1];
    info[2] = flags;
    info[3] = alpha;
    info[4] = J0[0];
    info[5] = Jn[0];
    info[6] = grel;
    info[7] = gnorm;
    info[8] = pinfo[4];
    free(g); free(mg); free(vt); free(v0); free(vn);
    return flags;
}

/* the Gauss-Newton iteration with PCG preconditioned by InvA; info [0..7] */
int or_ctx_gn_iterate(or_ctx *c, int max_pcg, double rtol, double *v_out, double *info)
{
    double inf9[9];
    int flags = or_ctx_gn_iterate_pc(c, max_pcg, rtol, 0, 0.0, 0, v_out, inf9);
    for (int k = 0; k < 8; k++) info[k] = inf9[k];
    return flags;
}

/* ------------------------------------------------------------------------ */
/* Transport map and its vector-Jacobian product (differentiable form)      */
/* ------------------------------------------------------------------------ */

/* m(1) and all m_j for template m0 under the context's velocity */
void or_ctx_transport(const or_ctx *c, const double *m0, double *m_all)
{
    solve_state(c, m0, m_all);
}

/* For a loss L(m(1)) with dL/dm(1) = gout: lam = adjoint sweep with final
 * value gout; dL/dm0 = lam_0; dL/dv = -int lam grad m dt.  The gradients of
 * the transported m0 are recomputed from m0 here. */
void or_ctx_transport_vjp(const or_ctx *c, const double *m0, const double *gout,
                          double *grad_m0, double *grad_v)
{
    long N = c->N;
    int nt = c->nt;
    or_ctx tmp = *c;
    tmp.m = malloc(sizeof(double) * (nt + 1) * N);
    tmp.G = malloc(sizeof(double) * (nt + 1) * 3 * N);
    solve_state(&tmp, m0, tmp.m);
    for (int j = 0; j <= nt; j++) ctx_grad(c, tmp.m + j * N, tmp.G + (long)j * 3 * N);
    double *lam = malloc(sizeof(double) * (nt + 1) * N);
    or_ctx_adjoint(&tmp, gout, lam);
    memcpy(grad_m0, lam, sizeof(double) * N);
    or_ctx_body_force(&tmp, lam, grad_v);
    for (long i = 0; i < 3 * N; i++) grad_v[i] = -grad_v[i];
    free(lam);
    free(tmp.m);
    free(tmp.G);
}
