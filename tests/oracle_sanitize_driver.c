/* Drives every oracle entry point on small deterministic inputs, for a
 * build of the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitizers.py compiles and runs it).  Exit status 0 when
 * every call returns its expected code; a sanitizer report aborts. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_elementwise(int m, int op, int64_t count, const double *a, const double *b, double *out);
int orc_norm2(int m, int64_t count, const double *x, double *out);
int orc_convolve(int m, int d, int64_t count, const double *x, const double *y, double *z);
int orc_eval_diff(int m, int d, int N, int n, int M, int dc, const int32_t *eq_ptr,
                  const int32_t *term_ptr, const int32_t *factors, const double *coef,
                  const double *x, double *f, double *A);
int orc_qr(int m, int N, int n, const double *A0, double *QR, double *vdiag, double *beta,
           int32_t *status);
int orc_series_solve(int m, int N, int n, int d, const double *QR, const double *vdiag,
                     const double *beta, const double *A, const double *b, double *dx,
                     int32_t *status);
int orc_newton_step(int m, int d, int N, int n, int M, int dc, const int32_t *eq_ptr,
                    const int32_t *term_ptr, const int32_t *factors, const double *coef,
                    double *x, double *dx_norm, int32_t *status);
int orc_newton_adjoint(int m, int d, int N, int n, int M, int dc, const int32_t *eq_ptr,
                       const int32_t *term_ptr, const int32_t *factors, const double *coef,
                       const double *x, const double *grad_x, double *grad_coef,
                       int32_t *status);

static uint64_t lcg = 12345;
/* a double in [-1, 1) away from zero, as the leading limb; lower limbs 0 */
static double rnd(void) {
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    double u = (double)(lcg >> 11) / 9007199254740992.0;
    return u < 0.5 ? -0.25 - u : u;
}

/* planes of `count` complex numbers with m limbs: limb 0 random, rest 0 */
static double *cplanes(int m, int64_t count) {
    double *p = calloc((size_t)2 * m * count, sizeof(double));
    for (int64_t e = 0; e < count; ++e) {
        p[e] = rnd();
        p[(int64_t)m * count + e] = rnd();
    }
    return p;
}

static int fails = 0;
static void expect(int got, int want, const char *what, int m) {
    if (got != want) {
        fprintf(stderr, "%s (m=%d): returned %d, expected %d\n", what, m, got, want);
        ++fails;
    }
}

int main(void) {
    static const int ms[] = {1, 2, 3, 4, 5, 8, 10};
    /* 3 equations in 3 unknowns (Section 4 form): terms with repeated
     * factors, a constant term and a t-term in each equation */
    const int N = 3, n = 3, dc = 1;
    const int32_t eq_ptr[] = {0, 4, 8, 12};
    const int32_t term_ptr[] = {0, 2, 3, 3, 3, 6, 7, 7, 7, 8, 10, 10, 10};
    const int32_t factors[] = {0, 1, 2, 0, 0, 2, 1, 0, 1, 2};
    const int M = 12;
    for (size_t q = 0; q < sizeof ms / sizeof ms[0]; ++q) {
        const int m = ms[q], d = 6, L = d + 1;
        const int64_t cnt = 37;
        double *a = cplanes(m, cnt), *b = cplanes(m, cnt), *o = calloc((size_t)2 * m * cnt, 8);
        for (int op = 0; op <= 11; ++op) {
            /* real operations read real planes (m, count): the first half */
            expect(orc_elementwise(m, op, cnt, a, b, o), 0, "orc_elementwise", m);
        }
        expect(orc_elementwise(m, 99, cnt, a, b, o), 2, "orc_elementwise bad op", m);
        double nrm[10];
        expect(orc_norm2(m, cnt, a, nrm), 0, "orc_norm2", m);
        double *xs = cplanes(m, 5 * (int64_t)L), *ys = cplanes(m, 5 * (int64_t)L);
        double *zs = calloc((size_t)2 * m * 5 * L, 8);
        expect(orc_convolve(m, d, 5, xs, ys, zs), 0, "orc_convolve", m);
        double *coef = cplanes(m, (int64_t)M * (dc + 1));
        double *x = cplanes(m, (int64_t)L * n);
        double *f = calloc((size_t)2 * m * L * N, 8), *A = calloc((size_t)2 * m * L * N * n, 8);
        expect(orc_eval_diff(m, d, N, n, M, dc, eq_ptr, term_ptr, factors, coef, x, f, A), 0,
               "orc_eval_diff", m);
        /* QR and the staggered solve of the Jacobian series just formed */
        double *A0 = calloc((size_t)2 * m * N * n, 8), *QR = calloc((size_t)2 * m * N * n, 8);
        for (int p = 0; p < 2 * m; ++p)
            memcpy(A0 + (size_t)p * N * n, A + (size_t)p * L * N * n, sizeof(double) * N * n);
        double *vd = calloc((size_t)2 * m * n, 8), *bet = calloc((size_t)m * n, 8);
        int32_t st = 0;
        expect(orc_qr(m, N, n, A0, QR, vd, bet, &st), 0, "orc_qr", m);
        double *dx = calloc((size_t)2 * m * L * n, 8);
        expect(orc_series_solve(m, N, n, d, QR, vd, bet, A, f, dx, &st), 0, "orc_series_solve",
               m);
        double dxn[20];
        expect(orc_newton_step(m, d, N, n, M, dc, eq_ptr, term_ptr, factors, coef, x, dxn, &st),
               0, "orc_newton_step", m);
        double *gx = cplanes(m, (int64_t)L * n);
        double *g = calloc((size_t)2 * 2 * M * (dc + 1), 8);
        expect(orc_newton_adjoint(m, d, N, n, M, dc, eq_ptr, term_ptr, factors, coef, x, gx, g,
                                  &st),
               0, "orc_newton_adjoint", m);
        /* argument errors */
        expect(orc_qr(m, 2, 3, A0, QR, vd, bet, &st), 1, "orc_qr N < n", m);
        expect(orc_convolve(m, -1, 5, xs, ys, zs), 1, "orc_convolve d < 0", m);
        free(a); free(b); free(o); free(xs); free(ys); free(zs); free(coef); free(x); free(f);
        free(A); free(A0); free(QR); free(vd); free(bet); free(dx); free(gx); free(g);
    }
    expect(orc_norm2(6, 4, NULL, NULL), 1, "orc_norm2 m = 6", 6);
    if (fails) return 1;
    printf("oracle entry points clean under the sanitizers\n");
    return 0;
}
