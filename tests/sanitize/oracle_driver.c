/* Runs the FP64 oracle through one gradient, matvec, PCG (InvA and InvH0),
 * Gauss-Newton iteration, transport VJP and the standalone operators, on a
 * small grid (naive DFT) and on one above 32 per axis (the mixed-radix FFT),
 * so that a build with AddressSanitizer and UndefinedBehaviorSanitizer checks
 * every host memory access and integer operation of those paths.  Exit
 * status 0 when every result is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct or_ctx or_ctx;
or_ctx *or_ctx_create(int n1, int n2, int n3, int nt, int reg, double beta, int leray);
void or_ctx_destroy(or_ctx *c);
void or_ctx_set_images(or_ctx *c, const double *m0, const double *m1);
void or_ctx_set_velocity(or_ctx *c, const double *v);
void or_ctx_gradient(or_ctx *c, double *g);
void or_ctx_matvec(const or_ctx *c, const double *vt, double *hvt);
void or_ctx_objective(const or_ctx *c, double out[3]);
void or_ctx_set_fd8(or_ctx *c, int on);
void or_ctx_set_ip_order(or_ctx *c, int order);
int or_ctx_pcg_pc(const or_ctx *c, const double *rhs, int max_it, double rtol, int pc, double eps_h0,
                  int max_inner, double *x, double *info);
int or_ctx_gn_iterate_pc(or_ctx *c, int max_pcg, double rtol, int pc, double eps_h0, int max_inner,
                         double *v_out, double *info);
void or_ctx_transport(const or_ctx *c, const double *m0, double *m_all);
void or_ctx_transport_vjp(const or_ctx *c, const double *m0, const double *gout, double *gm0, double *gv);
void or_leray(const double *v, double *out, int n1, int n2, int n3);
void or_restrict(const double *f, double *out, int ncomp, int n1, int n2, int n3);

static int all_finite(const double *a, long n)
{
    for (long i = 0; i < n; i++)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int run(int n1, int n2, int n3, int nt, int reg, int leray, int fd8, int ip)
{
    const long N = (long)n1 * n2 * n3, M = 3 * N;
    const double tp = 6.283185307179586;
    double *m0 = malloc(sizeof(double) * N), *m1 = malloc(sizeof(double) * N);
    double *v = malloc(sizeof(double) * M), *vt = malloc(sizeof(double) * M);
    double *g = malloc(sizeof(double) * M), *h = malloc(sizeof(double) * M), *x = malloc(sizeof(double) * M);
    double *mall = malloc(sizeof(double) * (nt + 1) * N), *gm0 = malloc(sizeof(double) * N);
    double *r = malloc(sizeof(double) * M / 8 + 8);
    for (int i = 0; i < n1; i++)
        for (int j = 0; j < n2; j++)
            for (int k = 0; k < n3; k++) {
                const long p = ((long)i * n2 + j) * n3 + k;
                const double a = tp * i / n1, b = tp * j / n2, c = tp * k / n3;
                m0[p] = sin(a) * sin(a) * cos(b) + 0.3 * sin(c + b);
                m1[p] = sin(a + 0.2) * sin(a + 0.2) * cos(b) + 0.3 * sin(c + b - 0.1);
                v[p] = 0.2 * sin(b + c);
                v[N + p] = 0.3 * cos(a - c);
                v[2 * N + p] = 0.1 * sin(a + b);
                vt[p] = cos(c);
                vt[N + p] = sin(a);
                vt[2 * N + p] = cos(a + b + c);
            }
    or_ctx *c = or_ctx_create(n1, n2, n3, nt, reg, 1e-2, leray);
    or_ctx_set_fd8(c, fd8);
    or_ctx_set_ip_order(c, ip);
    or_ctx_set_images(c, m0, m1);
    or_ctx_set_velocity(c, v);
    double J[3], info[9];
    or_ctx_objective(c, J);
    or_ctx_gradient(c, g);
    or_ctx_matvec(c, vt, h);
    int ok = all_finite(g, M) && all_finite(h, M) && isfinite(J[0]);
    for (int k = 0; k < M; k++) g[k] = -g[k];
    or_ctx_pcg_pc(c, g, 3, 1e-12, 0, 0.0, 0, x, info);
    ok = ok && all_finite(x, M);
    or_ctx_pcg_pc(c, g, 2, 1e-12, 1, 1e-3, 3, x, info);
    ok = ok && all_finite(x, M);
    if (n1 % 4 == 0 && n2 % 4 == 0 && n3 % 4 == 0 && n1 >= 16 && n2 >= 16 && n3 >= 16) {
        or_ctx_pcg_pc(c, g, 2, 1e-12, 2, 1e-3, 3, x, info);
        ok = ok && all_finite(x, M);
        or_restrict(m0, r, 1, n1, n2, n3);
        ok = ok && all_finite(r, N / 8);
    }
    or_ctx_transport(c, m0, mall);
    or_ctx_transport_vjp(c, m0, m1, gm0, x);
    ok = ok && all_finite(mall, (nt + 1) * N) && all_finite(gm0, N) && all_finite(x, M);
    or_leray(v, x, n1, n2, n3);
    ok = ok && all_finite(x, M);
    or_ctx_gn_iterate_pc(c, 2, 0.0, 0, 1e-3, 3, x, info);
    ok = ok && all_finite(x, M);
    or_ctx_destroy(c);
    free(m0); free(m1); free(v); free(vt); free(g); free(h); free(x); free(mall); free(gm0); free(r);
    return ok;
}

int main(void)
{
    int ok = run(8, 12, 10, 2, 1, 0, 0, 3);
    ok = ok && run(16, 16, 20, 3, 2, 1, 0, 3);
    ok = ok && run(8, 10, 12, 2, 2, 0, 1, 1);
    ok = ok && run(36, 8, 40, 1, 2, 1, 0, 3);  /* lines above 32: the mixed-radix FFT */
    printf(ok ? "oracle sanitizer run: ok\n" : "oracle sanitizer run: non-finite result\n");
    return ok ? 0 : 1;
}
