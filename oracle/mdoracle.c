/*
 * Oracle: a plain, slow CPU implementation of one Newton step on truncated
 * power series in complex multiple-double arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP path: no headers, helpers or tables.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (explicit
 * fma() calls only; no contraction), IEEE binary64, round to nearest even.
 *
 * Paper: J. Verschelde, "Parallel Software to Offset the Cost of Higher
 * Precision" (arXiv:2012.06607).  Citations name its sections, equations,
 * tables and figures.
 *
 * Numbers (Section 2): a multiple double with m limbs is an unevaluated sum
 * x_0 + x_1 + ... + x_{m-1} of hardware doubles, limb 0 most significant.
 * The paper takes its arithmetic from QDlib (m = 2, 4) and CAMPARY-generated
 * code (m = 3, 5, 8, 10); neither source is used here.  The algorithms below
 * are written from the error-free transformations the section cites
 * (Knuth's two-sum, Dekker's fast two-sum, the fma two-product) and are
 * the reading this project fixes for every m (the same sequence of hardware
 * operations runs on the GPU, so single operations agree bit for bit):
 *   m = 1  plain double arithmetic;
 *   m = 2  double-double: the accurate ("IEEE") addition of Hida, Li and
 *          Bailey, whose operation count is exactly Table 1's double double
 *          add row (8 additions, 12 subtractions), and the fma product;
 *   m >= 3 addition: level i holds a_i, b_i and the errors carried from
 *          level i-1, summed by a two-sum cascade whose errors go to level
 *          i+1; the last level (m-1) is summed in plain arithmetic (its
 *          rounding errors lie below the last limb), then the m level sums
 *          are renormalised; multiplication: the partial products a_i b_j
 *          with i + j < m-1 as exact two-products, summed level by level
 *          with two-sum cascades whose errors are carried to the next level,
 *          the products of level m-1 and the carries into it summed in
 *          plain arithmetic, then renormalised;
 *   division: long division with m+1 quotient digits, each one hardware
 *          division (Table 1's "/" column is m+1 for every m);
 *   square root: Newton iteration for 1/sqrt(a) from the hardware value,
 *          ceil(log2 m)+1 steps, then sqrt(a) = a * (1/sqrt(a)).
 * Multiple double times double: a_i b = p_i + q_i exactly for i < m-1 and
 * a plain product at i = m-1; level i holds p_i, q_{i-1} and the carries,
 * summed as in the addition.
 * Renormalisation of K >= m terms, one per level: a bottom-up two-sum
 * sweep (error free), then a top-down two-sum sweep that emits limbs
 * 0..m-2, the last limb collecting the rest.
 *
 * Complex arithmetic: (a+bi)(c+di) = (ac - bd) + (ad + bc)i with four real
 * products; x/y = (x conj(y)) / |y|^2.
 *
 * Layout of every array argument: planes (2, m, S...) contiguous float64;
 * element e of a tensor with E elements has real limb l at p[l*E + e] and
 * imaginary limb l at p[(m+l)*E + e].  Real tensors (beta, norms) are
 * planes (m, S...).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MDMAX 10
#define TERMS_MAX 256

/* ------------------------------------------------------------------------ */
/* operation counters: hardware operations by kind, and top-level
 * multiple-double operations (the units of Table 1)                          */

enum { C_ADD, C_SUB, C_MUL, C_DIV, C_FMA, C_SQRT, C_MDADD, C_MDMUL, C_MDDIV,
       C_MDMULD, C_NCOUNT };
static _Thread_local int64_t CNT[C_NCOUNT]; /* per thread: callers may run the oracle on several threads */
static _Thread_local int depth; /* > 0 while inside a multiple-double division */

void orc_reset_counters(void) { memset(CNT, 0, sizeof CNT); }
void orc_get_counters(int64_t *out) { memcpy(out, CNT, sizeof CNT); }

static double hadd(double a, double b) { CNT[C_ADD]++; return a + b; }
static double hsub(double a, double b) { CNT[C_SUB]++; return a - b; }
static double hmul(double a, double b) { CNT[C_MUL]++; return a * b; }
static double hdiv(double a, double b) { CNT[C_DIV]++; return a / b; }
static double hfma(double a, double b, double c) { CNT[C_FMA]++; return fma(a, b, c); }
static double hsqrt(double a) { CNT[C_SQRT]++; return sqrt(a); }

/* ------------------------------------------------------------------------ */
/* error-free transformations (Section 2; Rump 2010, Handbook ch. 14)         */

/* Knuth: s + e = a + b exactly, s = fl(a + b). */
static void two_sum(double a, double b, double *s, double *e)
{
    double ss = hadd(a, b);
    double bb = hsub(ss, a);
    double ea = hsub(a, hsub(ss, bb));
    double eb = hsub(b, bb);
    *s = ss;
    *e = hadd(ea, eb);
}

/* Dekker: s + e = a + b exactly when |a| >= |b|. */
static void fast_two_sum(double a, double b, double *s, double *e)
{
    double ss = hadd(a, b);
    *e = hsub(b, hsub(ss, a));
    *s = ss;
}

/* p + e = a * b exactly (fma). */
static void two_prod(double a, double b, double *p, double *e)
{
    double pp = hmul(a, b);
    *e = hfma(a, b, -pp);
    *p = pp;
}

/* ------------------------------------------------------------------------ */
/* real multiple doubles                                                       */

typedef struct { double v[MDMAX]; } md_t;

static md_t md_zero(void) { md_t z; memset(&z, 0, sizeof z); return z; }

static md_t md_from_d(int m, double a)
{
    md_t z = md_zero();
    (void)m;
    z.v[0] = a;
    return z;
}

static md_t md_neg(int m, md_t a)
{
    for (int i = 0; i < m; ++i) a.v[i] = -a.v[i];
    return a;
}

/* K terms -> m limbs (K >= m). */
static md_t renorm(int m, const double *x, int K)
{
    double t[TERMS_MAX];
    md_t y = md_zero();
    double s = x[K - 1];
    for (int i = K - 2; i >= 0; --i) two_sum(x[i], s, &s, &t[i + 1]);
    t[0] = s;
    double e = t[0];
    for (int i = 0; i < m - 1; ++i) two_sum(e, t[i + 1], &y.v[i], &e);
    if (K > m) {
        double tail = t[K - 1];
        for (int i = K - 2; i >= m; --i) tail = hadd(tail, t[i]);
        e = hadd(e, tail);
    }
    y.v[m - 1] = e;
    return y;
}

/* plain left-to-right sum of n terms */
static double plain_sum(const double *x, int n)
{
    double s = x[0];
    for (int i = 1; i < n; ++i) s = hadd(s, x[i]);
    return s;
}

static md_t add_(int m, md_t a, md_t b)
{
    md_t z = md_zero();
    if (m == 1) {
        z.v[0] = hadd(a.v[0], b.v[0]);
        return z;
    }
    if (m == 2) {
        double s, e, t, f;
        two_sum(a.v[0], b.v[0], &s, &e);
        two_sum(a.v[1], b.v[1], &t, &f);
        e = hadd(e, t);
        fast_two_sum(s, e, &s, &e);
        e = hadd(e, f);
        fast_two_sum(s, e, &s, &e);
        z.v[0] = s;
        z.v[1] = e;
        return z;
    }
    /* level i holds a_i, b_i and the errors carried from level i-1; the last
       level is summed in plain arithmetic (its rounding errors lie below
       the last limb) */
    double carry[MDMAX + 1], c[MDMAX + 1];
    int nc = 0;
    for (int i = 0; i < m; ++i) {
        double terms[MDMAX + 2];
        int nt = 0;
        terms[nt++] = a.v[i];
        terms[nt++] = b.v[i];
        for (int q = 0; q < nc; ++q) terms[nt++] = carry[q];
        if (i == m - 1) {
            c[i] = plain_sum(terms, nt);
            break;
        }
        double s = terms[0];
        nc = 0;
        for (int q = 1; q < nt; ++q) two_sum(s, terms[q], &s, &carry[nc++]);
        c[i] = s;
    }
    return renorm(m, c, m);
}

static md_t mul_(int m, md_t a, md_t b)
{
    md_t z = md_zero();
    if (m == 1) {
        z.v[0] = hmul(a.v[0], b.v[0]);
        return z;
    }
    if (m == 2) {
        double p, e;
        two_prod(a.v[0], b.v[0], &p, &e);
        double t1 = hmul(a.v[0], b.v[1]);
        double t2 = hmul(a.v[1], b.v[0]);
        t1 = hadd(t1, t2);
        e = hadd(e, t1);
        fast_two_sum(p, e, &p, &e);
        z.v[0] = p;
        z.v[1] = e;
        return z;
    }
    /* level k: the products a_i b_{k-i}, the low parts of level k-1's
       products and the carries of level k-1; the last level takes plain
       products and a plain sum (its rounding errors lie below the last
       limb) */
    double carry[TERMS_MAX], lo[MDMAX + 1], c[MDMAX + 1];
    int nc = 0, nlo = 0;
    for (int k = 0; k < m; ++k) {
        double terms[TERMS_MAX], newlo[MDMAX + 1];
        int nt = 0;
        if (k == m - 1) {
            for (int i = 0; i <= k; ++i) terms[nt++] = hmul(a.v[i], b.v[k - i]);
            for (int i = 0; i < nlo; ++i) terms[nt++] = lo[i];
            for (int i = 0; i < nc; ++i) terms[nt++] = carry[i];
            c[k] = plain_sum(terms, nt);
            break;
        }
        for (int i = 0; i <= k; ++i) two_prod(a.v[i], b.v[k - i], &terms[nt++], &newlo[i]);
        for (int i = 0; i < nlo; ++i) terms[nt++] = lo[i];
        for (int i = 0; i < nc; ++i) terms[nt++] = carry[i];
        double s = terms[0];
        nc = 0;
        for (int i = 1; i < nt; ++i) two_sum(s, terms[i], &s, &carry[nc++]);
        c[k] = s;
        for (int i = 0; i <= k; ++i) lo[i] = newlo[i];
        nlo = k + 1;
    }
    return renorm(m, c, m);
}

/* multiple double times hardware double */
static md_t muld_(int m, md_t a, double b)
{
    md_t z = md_zero();
    if (m == 1) {
        z.v[0] = hmul(a.v[0], b);
        return z;
    }
    /* level i holds p_i, q_{i-1} (a_i b = p_i + q_i exactly) and the
       carries; the last level takes a plain product and a plain sum */
    double p[MDMAX], q[MDMAX], carry[MDMAX + 1], c[MDMAX + 1];
    for (int i = 0; i < m - 1; ++i) two_prod(a.v[i], b, &p[i], &q[i]);
    p[m - 1] = hmul(a.v[m - 1], b);
    c[0] = p[0];
    int nc = 0;
    for (int i = 1; i < m; ++i) {
        double terms[MDMAX + 2];
        int nt = 0;
        terms[nt++] = p[i];
        terms[nt++] = q[i - 1];
        for (int r = 0; r < nc; ++r) terms[nt++] = carry[r];
        if (i == m - 1) {
            c[i] = plain_sum(terms, nt);
            break;
        }
        double s = terms[0];
        nc = 0;
        for (int r = 1; r < nt; ++r) two_sum(s, terms[r], &s, &carry[nc++]);
        c[i] = s;
    }
    return renorm(m, c, m);
}

static md_t div_(int m, md_t a, md_t b)
{
    md_t z = md_zero();
    if (m == 1) {
        z.v[0] = hdiv(a.v[0], b.v[0]);
        return z;
    }
    double q[MDMAX + 1];
    md_t r = a;
    for (int i = 0; i <= m; ++i) {
        q[i] = hdiv(r.v[0], b.v[0]);
        if (i < m) r = add_(m, r, md_neg(m, muld_(m, b, q[i])));
    }
    return renorm(m, q, m + 1);
}

/* counted top-level operations */
static md_t md_add(int m, md_t a, md_t b) { if (!depth) CNT[C_MDADD]++; return add_(m, a, b); }
static md_t md_sub(int m, md_t a, md_t b) { return md_add(m, a, md_neg(m, b)); }
static md_t md_mul(int m, md_t a, md_t b) { if (!depth) CNT[C_MDMUL]++; return mul_(m, a, b); }
static md_t md_muld(int m, md_t a, double b) { if (!depth) CNT[C_MDMULD]++; return muld_(m, a, b); }
static md_t md_div(int m, md_t a, md_t b)
{
    if (!depth) CNT[C_MDDIV]++;
    depth++;
    md_t z = div_(m, a, b);
    depth--;
    return z;
}

static int rsqrt_iterations(int m)
{
    int it = 1, p = 1;
    while (p < m) { p *= 2; it++; }
    return it; /* ceil(log2 m) + 1 */
}

/* 1/sqrt(a): y <- y + y (1 - a y^2) / 2 from the hardware value */
static md_t md_rsqrt(int m, md_t a)
{
    double y0 = hdiv(1.0, hsqrt(a.v[0]));
    md_t y = md_from_d(m, y0);
    if (m == 1) return y;
    md_t one = md_from_d(m, 1.0);
    int nit = rsqrt_iterations(m);
    for (int it = 0; it < nit; ++it) {
        md_t t = md_mul(m, y, y);
        t = md_mul(m, a, t);
        t = md_sub(m, one, t);
        t = md_mul(m, y, t);
        for (int i = 0; i < m; ++i) t.v[i] = hmul(t.v[i], 0.5);
        y = md_add(m, y, t);
    }
    return y;
}

static md_t md_sqrt(int m, md_t a)
{
    if (m == 1) return md_from_d(m, hsqrt(a.v[0]));
    md_t y = md_rsqrt(m, a);
    md_t s = md_mul(m, a, y);
    if (a.v[0] == 0.0) s = md_zero();
    return s;
}

/* a < b on the values, for normalised expansions (sign of a - b) */
static int md_less(int m, md_t a, md_t b)
{
    md_t d = add_(m, a, md_neg(m, b));
    for (int i = 0; i < m; ++i) {
        if (d.v[i] < 0.0) return 1;
        if (d.v[i] > 0.0) return 0;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* complex multiple doubles                                                    */

typedef struct { md_t re, im; } cmd_t;

static cmd_t c_zero(void) { cmd_t z; z.re = md_zero(); z.im = md_zero(); return z; }
static cmd_t c_conj(int m, cmd_t a) { a.im = md_neg(m, a.im); return a; }
static cmd_t c_neg(int m, cmd_t a) { a.re = md_neg(m, a.re); a.im = md_neg(m, a.im); return a; }

static cmd_t c_add(int m, cmd_t a, cmd_t b)
{
    cmd_t z;
    z.re = md_add(m, a.re, b.re);
    z.im = md_add(m, a.im, b.im);
    return z;
}

static cmd_t c_sub(int m, cmd_t a, cmd_t b) { return c_add(m, a, c_neg(m, b)); }

static cmd_t c_mul(int m, cmd_t a, cmd_t b)
{
    md_t p1 = md_mul(m, a.re, b.re);
    md_t p2 = md_mul(m, a.im, b.im);
    md_t p3 = md_mul(m, a.re, b.im);
    md_t p4 = md_mul(m, a.im, b.re);
    cmd_t z;
    z.re = md_add(m, p1, md_neg(m, p2));
    z.im = md_add(m, p3, p4);
    return z;
}

/* complex times real */
static cmd_t c_mulr(int m, cmd_t a, md_t r)
{
    cmd_t z;
    z.re = md_mul(m, a.re, r);
    z.im = md_mul(m, a.im, r);
    return z;
}

static md_t c_abs2(int m, cmd_t a)
{
    md_t p1 = md_mul(m, a.re, a.re);
    md_t p2 = md_mul(m, a.im, a.im);
    return md_add(m, p1, p2);
}

static cmd_t c_div(int m, cmd_t a, cmd_t b)
{
    md_t den = c_abs2(m, b);
    cmd_t num = c_mul(m, a, c_conj(m, b));
    cmd_t z;
    z.re = md_div(m, num.re, den);
    z.im = md_div(m, num.im, den);
    return z;
}

/* ------------------------------------------------------------------------ */
/* plane access                                                                */

static cmd_t cload(int m, const double *p, int64_t E, int64_t e)
{
    cmd_t z = c_zero();
    for (int l = 0; l < m; ++l) {
        z.re.v[l] = p[(int64_t)l * E + e];
        z.im.v[l] = p[(int64_t)(m + l) * E + e];
    }
    return z;
}

static void cstore(int m, double *p, int64_t E, int64_t e, cmd_t z)
{
    for (int l = 0; l < m; ++l) {
        p[(int64_t)l * E + e] = z.re.v[l];
        p[(int64_t)(m + l) * E + e] = z.im.v[l];
    }
}

static md_t rload(int m, const double *p, int64_t E, int64_t e)
{
    md_t z = md_zero();
    for (int l = 0; l < m; ++l) z.v[l] = p[(int64_t)l * E + e];
    return z;
}

static void rstore(int m, double *p, int64_t E, int64_t e, md_t z)
{
    for (int l = 0; l < m; ++l) p[(int64_t)l * E + e] = z.v[l];
}

static int valid_m(int m)
{
    return m == 1 || m == 2 || m == 3 || m == 4 || m == 5 || m == 8 || m == 10;
}

/* ------------------------------------------------------------------------ */
/* single operations (one per element), for operation-level parity           */

enum { OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_SQRT, OP_RSQRT, OP_MULD,
       OP_CADD, OP_CSUB, OP_CMUL, OP_CDIV, OP_CABS2 };

/* Real ops read planes (m, count) (b's leading limb for OP_MULD) and write
 * (m, count); complex ops read and write (2, m, count); OP_CABS2 writes
 * (m, count). */
int orc_elementwise(int m, int op, int64_t count, const double *a, const double *b,
                    double *out)
{
    if (!valid_m(m) || count < 0) return 1;
    for (int64_t e = 0; e < count; ++e) {
        if (op <= OP_MULD) {
            md_t x = rload(m, a, count, e), y = md_zero(), z;
            if (op != OP_SQRT && op != OP_RSQRT) y = rload(m, b, count, e);
            switch (op) {
            case OP_ADD: z = md_add(m, x, y); break;
            case OP_SUB: z = md_sub(m, x, y); break;
            case OP_MUL: z = md_mul(m, x, y); break;
            case OP_DIV: z = md_div(m, x, y); break;
            case OP_SQRT: z = md_sqrt(m, x); break;
            case OP_RSQRT: z = md_rsqrt(m, x); break;
            default: z = md_muld(m, x, y.v[0]); break;
            }
            rstore(m, out, count, e, z);
        } else {
            cmd_t x = cload(m, a, count, e), y = c_zero(), z;
            if (op != OP_CABS2) y = cload(m, b, count, e);
            switch (op) {
            case OP_CADD: z = c_add(m, x, y); break;
            case OP_CSUB: z = c_sub(m, x, y); break;
            case OP_CMUL: z = c_mul(m, x, y); break;
            case OP_CDIV: z = c_div(m, x, y); break;
            case OP_CABS2: rstore(m, out, count, e, c_abs2(m, x)); continue;
            default: return 2;
            }
            cstore(m, out, count, e, z);
        }
    }
    return 0;
}

/* Section 2 example: the 2-norm sqrt(sum |x_j|^2) of a complex vector,
 * summed in index order.  out: planes (m, 1). */
int orc_norm2(int m, int64_t count, const double *x, double *out)
{
    if (!valid_m(m) || count < 1) return 1;
    md_t s = c_abs2(m, cload(m, x, count, 0));
    for (int64_t e = 1; e < count; ++e) s = md_add(m, s, c_abs2(m, cload(m, x, count, e)));
    rstore(m, out, 1, 0, md_sqrt(m, s));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* truncated power series (Section 3)                                          */

/* Product of x (degree dx <= d, coefficient i at element xb + i*xs of a
 * tensor with xE elements) and y (degree d) truncated at degree d:
 * z_k = x_0 y_k + x_1 y_{k-1} + ... + x_{min(k,dx)} y_{k-min(k,dx)}, each z_k
 * started from its first product; with dx = d this is (d+2)(d+1)/2
 * multiplications and (d+1)d/2 additions (Section 3). */
static void series_mul(int m, int d, int dx, const double *x, int64_t xE, int64_t xb,
                       int64_t xs, const double *y, int64_t yE, int64_t yb, int64_t ys,
                       cmd_t *z)
{
    for (int k = 0; k <= d; ++k) {
        cmd_t acc = c_mul(m, cload(m, x, xE, xb), cload(m, y, yE, yb + (int64_t)k * ys));
        int top = k < dx ? k : dx;
        for (int i = 1; i <= top; ++i)
            acc = c_add(m, acc, c_mul(m, cload(m, x, xE, xb + (int64_t)i * xs),
                                      cload(m, y, yE, yb + (int64_t)(k - i) * ys)));
        z[k] = acc;
    }
}

/* z[c] = x[c] * y[c] mod t^{d+1}; planes (2, m, count, d+1). */
int orc_convolve(int m, int d, int64_t count, const double *x, const double *y, double *z)
{
    if (!valid_m(m) || d < 0 || count < 0) return 1;
    int64_t E = count * (d + 1);
    cmd_t *buf = malloc(sizeof(cmd_t) * (size_t)(d + 1));
    if (!buf) return 3;
    for (int64_t c = 0; c < count; ++c) {
        series_mul(m, d, d, x, E, c * (d + 1), 1, y, E, c * (d + 1), 1, buf);
        for (int k = 0; k <= d; ++k) cstore(m, z, E, c * (d + 1) + k, buf[k]);
    }
    free(buf);
    return 0;
}

/*
 * z[c] = x[c] / y[c] mod t^{d+1} (Section 3: a series with a nonzero
 * constant term has an inverse, and series divide like numbers).  From
 * x(t) = y(t) z(t): z_0 = x_0 / y_0 and, for k = 1..d,
 * z_k = (x_k - (y_1 z_{k-1} + y_2 z_{k-2} + ... + y_k z_0)) / y_0,
 * the products added in increasing i.  A zero y_0 sets ST_SINGULAR (the
 * quotient is then not defined; its coefficients are whatever the
 * divisions give).  Planes (2, m, count, d+1).
 */
int orc_series_divide(int m, int d, int64_t count, const double *x, const double *y, double *z,
                      int32_t *status)
{
    if (!valid_m(m) || d < 0 || count < 0) return 1;
    int64_t E = count * (d + 1);
    cmd_t *zc = malloc(sizeof(cmd_t) * (size_t)(d + 1));
    if (!zc) return 3;
    int32_t st = 0;
    for (int64_t c = 0; c < count; ++c) {
        int64_t b = c * (d + 1);
        cmd_t y0 = cload(m, y, E, b);
        if (y0.re.v[0] == 0.0 && y0.im.v[0] == 0.0) st |= 1;
        for (int k = 0; k <= d; ++k) {
            cmd_t r = cload(m, x, E, b + k);
            if (k > 0) {
                cmd_t s = c_mul(m, cload(m, y, E, b + 1), zc[k - 1]);
                for (int i = 2; i <= k; ++i) s = c_add(m, s, c_mul(m, cload(m, y, E, b + i), zc[k - i]));
                r = c_sub(m, r, s);
            }
            zc[k] = c_div(m, r, y0);
            cstore(m, z, E, b + k, zc[k]);
        }
    }
    free(zc);
    if (status) *status = st;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* evaluation and reverse-mode differentiation (Section 4)                    */

/* a series held in the oracle's own memory */
typedef struct { cmd_t *c; } ser_t;

static void ser_mul_mem(int m, int d, int dx, const cmd_t *x, const cmd_t *y, cmd_t *z)
{
    for (int k = 0; k <= d; ++k) {
        cmd_t acc = c_mul(m, x[0], y[k]);
        int top = k < dx ? k : dx;
        for (int i = 1; i <= top; ++i) acc = c_add(m, acc, c_mul(m, x[i], y[k - i]));
        z[k] = acc;
    }
}

/*
 * f(x(t)) and A(t) = df/dx(x(t)) for a system whose terms are c(t) x^a.
 * For a term with factor list v_1..v_D (variables with repetition, sorted)
 * the forward products P_j = v_1 ... v_j, backward products
 * Q_j = v_j ... v_D and cross products C_j = P_{j-1} Q_{j+1} give the value
 * P_D and every partial derivative: d/dx_l of x^a is a_l C_{j*}, j* the
 * first position of x_l (reverse-mode differentiation, Section 4: all
 * partials for a small multiple of the cost of the value).  Value and
 * derivatives are multiplied by the coefficient series c(t) (degree dc),
 * then added into f_i and A_{i,l} in term order, from zero.
 * x: planes (2, m, d+1, n); coef: (2, m, M, dc+1);
 * f: (2, m, d+1, N); A: (2, m, d+1, N, n).
 */
int orc_eval_diff(int m, int d, int N, int n, int M, int dc, const int32_t *eq_ptr,
                  const int32_t *term_ptr, const int32_t *factors, const double *coef,
                  const double *x, double *f, double *A)
{
    if (!valid_m(m) || d < 0 || N < 1 || n < 1 || dc < 0) return 1;
    int L = d + 1;
    int64_t xE = (int64_t)L * n, cE = (int64_t)M * (dc + 1);
    int64_t fE = (int64_t)L * N, AE = (int64_t)L * N * n;
    int maxD = 0;
    for (int j = 0; j < M; ++j)
        if (term_ptr[j + 1] - term_ptr[j] > maxD) maxD = term_ptr[j + 1] - term_ptr[j];
    int nser = 3 * (maxD + 2) + 4;
    cmd_t *mem = malloc(sizeof(cmd_t) * (size_t)L * (size_t)nser);
    if (!mem) return 3;
    /* views: X[v] copies of x_v, P[j], Q[j], C[j], val, der, cs */
    cmd_t *cs = mem, *val = mem + L, *der = mem + 2 * L;
    cmd_t *P = mem + 3 * L;                      /* P[j] at P + j*L, j = 1..maxD */
    cmd_t *Q = P + (size_t)(maxD + 2) * L;       /* Q[j] */
    cmd_t *C = Q + (size_t)(maxD + 2) * L;       /* C[j] */
    cmd_t *fi = malloc(sizeof(cmd_t) * (size_t)L);
    cmd_t *Ai = malloc(sizeof(cmd_t) * (size_t)L * (size_t)n);
    if (!fi || !Ai) { free(mem); free(fi); free(Ai); return 3; }

    for (int i = 0; i < N; ++i) {
        for (int k = 0; k < L; ++k) fi[k] = c_zero();
        for (int k = 0; k < L * n; ++k) Ai[k] = c_zero();
        for (int j = eq_ptr[i]; j < eq_ptr[i + 1]; ++j) {
            const int32_t *v = factors + term_ptr[j];
            int D = term_ptr[j + 1] - term_ptr[j];
            /* coefficient series, zero beyond degree dc */
            for (int k = 0; k < L; ++k) cs[k] = k <= dc ? cload(m, coef, cE, (int64_t)j * (dc + 1) + k) : c_zero();
            int dcu = dc < d ? dc : d;
            if (D == 0) {
                for (int k = 0; k < L; ++k) val[k] = cs[k];
            } else {
                /* P_1 = x_{v_1}, P_j = P_{j-1} * x_{v_j} */
                for (int k = 0; k < L; ++k) P[1 * L + k] = cload(m, x, xE, (int64_t)k * n + v[0]);
                for (int jj = 2; jj <= D; ++jj) {
                    cmd_t *xv = C; /* scratch: the factor series */
                    for (int k = 0; k < L; ++k) xv[k] = cload(m, x, xE, (int64_t)k * n + v[jj - 1]);
                    ser_mul_mem(m, d, d, P + (size_t)(jj - 1) * L, xv, P + (size_t)jj * L);
                }
                /* Q_D = x_{v_D}, Q_j = x_{v_j} * Q_{j+1} for j = D-1 .. 2 */
                for (int k = 0; k < L; ++k) Q[(size_t)D * L + k] = cload(m, x, xE, (int64_t)k * n + v[D - 1]);
                for (int jj = D - 1; jj >= 2; --jj) {
                    cmd_t *xv = C;
                    for (int k = 0; k < L; ++k) xv[k] = cload(m, x, xE, (int64_t)k * n + v[jj - 1]);
                    ser_mul_mem(m, d, d, xv, Q + (size_t)(jj + 1) * L, Q + (size_t)jj * L);
                }
                /* value = c * P_D */
                ser_mul_mem(m, d, dcu, cs, P + (size_t)D * L, val);
            }
            for (int k = 0; k < L; ++k) fi[k] = c_add(m, fi[k], val[k]);
            /* derivatives, one per distinct variable at its first position */
            for (int jj = 1; jj <= D; ++jj) {
                if (jj > 1 && v[jj - 1] == v[jj - 2]) continue;
                int a = 0;
                for (int q = 0; q < D; ++q) a += (v[q] == v[jj - 1]);
                if (D == 1) {
                    for (int k = 0; k < L; ++k) der[k] = cs[k];
                } else {
                    const cmd_t *cross;
                    if (jj == 1) cross = Q + 2 * (size_t)L;
                    else if (jj == D) cross = P + (size_t)(D - 1) * L;
                    else {
                        ser_mul_mem(m, d, d, P + (size_t)(jj - 1) * L, Q + (size_t)(jj + 1) * L, C + L);
                        cross = C + L;
                    }
                    ser_mul_mem(m, d, dcu, cs, cross, der);
                }
                if (a > 1)
                    for (int k = 0; k < L; ++k) {
                        der[k].re = md_muld(m, der[k].re, (double)a);
                        der[k].im = md_muld(m, der[k].im, (double)a);
                    }
                int l = v[jj - 1];
                for (int k = 0; k < L; ++k) Ai[(size_t)k * n + l] = c_add(m, Ai[(size_t)k * n + l], der[k]);
            }
        }
        for (int k = 0; k < L; ++k) {
            cstore(m, f, fE, (int64_t)k * N + i, fi[k]);
            for (int l = 0; l < n; ++l) cstore(m, A, AE, ((int64_t)k * N + i) * n + l, Ai[(size_t)k * n + l]);
        }
    }
    free(mem);
    free(fi);
    free(Ai);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Householder QR (Section 4: the linear systems are solved with QR)         */

#define ST_SINGULAR 1
#define ST_NONFINITE 2

/*
 * A0 = Q R with Q = H_0 H_1 ... H_{n-1}, H_j = I - beta_j v_j v_j^H acting on
 * rows j..N-1.  For column j with entries x = A[j:N, j], alpha = x_0:
 *   sigma = sqrt(sum |x_i|^2), phi = alpha/|alpha| (1 when alpha = 0),
 *   v = (phi (|alpha| + sigma), x_1, ..., x_{N-j-1}),
 *   beta = 1/(sigma (sigma + |alpha|)), R_jj = -phi sigma,
 * and every later column l gets A[:, l] -= beta (v^H A[:, l]) v.
 * QR: planes (2, m, N, n) with R on and above the diagonal and the reflector
 * tails below it; vdiag: (2, m, n) reflector heads; beta: (m, n).
 * A zero column sets ST_SINGULAR (beta = 0, R_jj = 0).
 */
int orc_qr(int m, int N, int n, const double *A0, double *QR, double *vdiag, double *beta,
           int32_t *status)
{
    if (!valid_m(m) || n < 1 || N < n) return 1;
    int64_t E = (int64_t)N * n;
    cmd_t *a = malloc(sizeof(cmd_t) * (size_t)E);
    if (!a) return 3;
    for (int64_t e = 0; e < E; ++e) a[e] = cload(m, A0, E, e);
    *status = 0;
    for (int j = 0; j < n; ++j) {
        cmd_t alpha = a[(size_t)j * n + j];
        md_t s2 = c_abs2(m, alpha);
        md_t a2 = s2;
        for (int i = j + 1; i < N; ++i) s2 = md_add(m, s2, c_abs2(m, a[(size_t)i * n + j]));
        md_t sigma = md_sqrt(m, s2);
        md_t aabs = md_sqrt(m, a2);
        cmd_t phi = c_zero();
        phi.re = md_from_d(m, 1.0);
        if (aabs.v[0] != 0.0) {
            phi.re = md_div(m, alpha.re, aabs);
            phi.im = md_div(m, alpha.im, aabs);
        }
        md_t bet = md_zero();
        cmd_t v0 = c_zero(), rjj = c_zero();
        if (sigma.v[0] == 0.0) {
            *status |= ST_SINGULAR;
        } else {
            md_t sp = md_add(m, aabs, sigma);
            v0 = c_mulr(m, phi, sp);
            bet = md_div(m, md_from_d(m, 1.0), md_mul(m, sigma, sp));
            rjj = c_neg(m, c_mulr(m, phi, sigma));
        }
        /* trailing columns */
        for (int l = j + 1; l < n; ++l) {
            cmd_t w = c_mul(m, c_conj(m, v0), a[(size_t)j * n + l]);
            for (int i = j + 1; i < N; ++i)
                w = c_add(m, w, c_mul(m, c_conj(m, a[(size_t)i * n + j]), a[(size_t)i * n + l]));
            cmd_t bw = c_mulr(m, w, bet);
            a[(size_t)j * n + l] = c_sub(m, a[(size_t)j * n + l], c_mul(m, bw, v0));
            for (int i = j + 1; i < N; ++i)
                a[(size_t)i * n + l] = c_sub(m, a[(size_t)i * n + l], c_mul(m, bw, a[(size_t)i * n + j]));
        }
        a[(size_t)j * n + j] = rjj;
        cstore(m, vdiag, n, j, v0);
        rstore(m, beta, n, j, bet);
    }
    for (int64_t e = 0; e < E; ++e) {
        cstore(m, QR, E, e, a[e]);
        for (int l = 0; l < m; ++l)
            if (!isfinite(a[e].re.v[l]) || !isfinite(a[e].im.v[l])) *status |= ST_NONFINITE;
    }
    free(a);
    return 0;
}

/* y <- Q^H y: apply H_0, H_1, ..., H_{n-1} in that order (y has N entries) */
static void apply_qh(int m, int N, int n, const cmd_t *qr, const cmd_t *vd, const md_t *bet,
                     cmd_t *y)
{
    for (int j = 0; j < n; ++j) {
        cmd_t w = c_mul(m, c_conj(m, vd[j]), y[j]);
        for (int i = j + 1; i < N; ++i) w = c_add(m, w, c_mul(m, c_conj(m, qr[(size_t)i * n + j]), y[i]));
        cmd_t bw = c_mulr(m, w, bet[j]);
        y[j] = c_sub(m, y[j], c_mul(m, bw, vd[j]));
        for (int i = j + 1; i < N; ++i) y[i] = c_sub(m, y[i], c_mul(m, bw, qr[(size_t)i * n + j]));
    }
}

/* R z = y[0:n] by back substitution, row i from n-1 down to 0 */
static void back_sub(int m, int n, const cmd_t *qr, const cmd_t *y, cmd_t *z)
{
    for (int i = n - 1; i >= 0; --i) {
        cmd_t s = y[i];
        for (int l = i + 1; l < n; ++l) s = c_sub(m, s, c_mul(m, qr[(size_t)i * n + l], z[l]));
        z[i] = c_div(m, s, qr[(size_t)i * n + i]);
    }
}

/*
 * The linearised system A(t) dx(t) = b(t) is the block lower triangular
 * Toeplitz system of Section 4; forward substitution solves
 * A_0 dx_k = b_k - A_1 dx_{k-1} - ... - A_k dx_0 for k = 0..d with the one
 * QR factorisation of A_0 (least squares in the first n rows of Q^H r_k when
 * N > n).  After dx_k is found the right hand sides of the later stages are
 * updated: r_{k+j} -= A_j dx_k, j = 1..d-k (one job per update in the
 * paper's job queue, Section 5).
 * A: planes (2, m, d+1, N, n) (the A_0 slot is not read); b: (2, m, d+1, N);
 * dx: (2, m, d+1, n).
 */
int orc_series_solve(int m, int N, int n, int d, const double *QR, const double *vdiag,
                     const double *beta, const double *A, const double *b, double *dx,
                     int32_t *status)
{
    if (!valid_m(m) || n < 1 || N < n || d < 0) return 1;
    int L = d + 1;
    int64_t E = (int64_t)N * n, AE = (int64_t)L * N * n, bE = (int64_t)L * N, xE = (int64_t)L * n;
    cmd_t *qr = malloc(sizeof(cmd_t) * (size_t)E);
    cmd_t *vd = malloc(sizeof(cmd_t) * (size_t)n);
    md_t *bet = malloc(sizeof(md_t) * (size_t)n);
    cmd_t *r = malloc(sizeof(cmd_t) * (size_t)bE);
    cmd_t *y = malloc(sizeof(cmd_t) * (size_t)N);
    cmd_t *z = malloc(sizeof(cmd_t) * (size_t)n);
    if (!qr || !vd || !bet || !r || !y || !z) {
        free(qr); free(vd); free(bet); free(r); free(y); free(z);
        return 3;
    }
    for (int64_t e = 0; e < E; ++e) qr[e] = cload(m, QR, E, e);
    for (int j = 0; j < n; ++j) { vd[j] = cload(m, vdiag, n, j); bet[j] = rload(m, beta, n, j); }
    for (int64_t e = 0; e < bE; ++e) r[e] = cload(m, b, bE, e);
    *status = 0;
    for (int k = 0; k <= d; ++k) {
        for (int i = 0; i < N; ++i) y[i] = r[(size_t)k * N + i];
        apply_qh(m, N, n, qr, vd, bet, y);
        back_sub(m, n, qr, y, z);
        for (int l = 0; l < n; ++l) {
            cstore(m, dx, xE, (int64_t)k * n + l, z[l]);
            for (int q = 0; q < m; ++q)
                if (!isfinite(z[l].re.v[q]) || !isfinite(z[l].im.v[q])) *status |= ST_NONFINITE;
        }
        for (int j = 1; j <= d - k; ++j)
            for (int i = 0; i < N; ++i) {
                int64_t row = ((int64_t)j * N + i) * n;
                cmd_t t = c_mul(m, cload(m, A, AE, row), z[0]);
                for (int l = 1; l < n; ++l) t = c_add(m, t, c_mul(m, cload(m, A, AE, row + l), z[l]));
                r[(size_t)(k + j) * N + i] = c_sub(m, r[(size_t)(k + j) * N + i], t);
            }
    }
    free(qr); free(vd); free(bet); free(r); free(y); free(z);
    return 0;
}

/*
 * One Newton step (Section 4): evaluate and differentiate f at x(t),
 * b = -f, solve A(t) dx(t) = b(t) with one QR of A_0 and the staggered
 * substitution, x(t) += dx(t).
 * dx_norm: planes (m, 2): [max_i |dx_{d,i}|, max_{k,i} |dx_{k,i}|] (the
 * modulus of the update to the last coefficient, Section 6, and the largest
 * update over all coefficients).
 */
int orc_newton_step(int m, int d, int N, int n, int M, int dc, const int32_t *eq_ptr,
                    const int32_t *term_ptr, const int32_t *factors, const double *coef,
                    double *x, double *dx_norm, int32_t *status)
{
    if (!valid_m(m) || d < 0 || n < 1 || N < n) return 1;
    int L = d + 1;
    size_t fsz = (size_t)2 * m * L * N, Asz = (size_t)2 * m * L * N * n, A0sz = (size_t)2 * m * N * n;
    double *f = malloc(sizeof(double) * fsz);
    double *A = malloc(sizeof(double) * Asz);
    double *A0 = malloc(sizeof(double) * A0sz);
    double *QR = malloc(sizeof(double) * A0sz);
    double *vd = malloc(sizeof(double) * (size_t)2 * m * n);
    double *bet = malloc(sizeof(double) * (size_t)m * n);
    double *dx = malloc(sizeof(double) * (size_t)2 * m * L * n);
    if (!f || !A || !A0 || !QR || !vd || !bet || !dx) {
        free(f); free(A); free(A0); free(QR); free(vd); free(bet); free(dx);
        return 3;
    }
    int rc = orc_eval_diff(m, d, N, n, M, dc, eq_ptr, term_ptr, factors, coef, x, f, A);
    if (rc) {
        free(f); free(A); free(A0); free(QR); free(vd); free(bet); free(dx);
        return rc;
    }
    for (size_t q = 0; q < fsz; ++q) f[q] = -f[q]; /* b = -f (exact) */
    int64_t AE = (int64_t)L * N * n, E0 = (int64_t)N * n;
    for (int p = 0; p < 2 * m; ++p)
        memcpy(A0 + (size_t)p * E0, A + (size_t)p * AE, sizeof(double) * (size_t)E0);
    int32_t st1 = 0, st2 = 0;
    orc_qr(m, N, n, A0, QR, vd, bet, &st1);
    orc_series_solve(m, N, n, d, QR, vd, bet, A, f, dx, &st2);
    *status = st1 | st2;
    int64_t xE = (int64_t)L * n;
    md_t best_d = md_zero(), best_all = md_zero();
    for (int k = 0; k <= d; ++k)
        for (int l = 0; l < n; ++l) {
            int64_t e = (int64_t)k * n + l;
            cmd_t u = cload(m, dx, xE, e);
            cstore(m, x, xE, e, c_add(m, cload(m, x, xE, e), u));
            md_t a2 = c_abs2(m, u);
            if (md_less(m, best_all, a2)) best_all = a2;
            if (k == d && md_less(m, best_d, a2)) best_d = a2;
        }
    rstore(m, dx_norm, 2, 0, md_sqrt(m, best_d));
    rstore(m, dx_norm, 2, 1, md_sqrt(m, best_all));
    free(f); free(A); free(A0); free(QR); free(vd); free(bet); free(dx);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* adjoint of the converged series solution                                   */

/* z <- Q z with Q = H_0 H_1 ... H_{n-1}: apply H_{n-1} first (z has N entries) */
static void apply_q(int m, int N, int n, const cmd_t *qr, const cmd_t *vd, const md_t *bet,
                    cmd_t *z)
{
    for (int j = n - 1; j >= 0; --j) {
        cmd_t w = c_mul(m, c_conj(m, vd[j]), z[j]);
        for (int i = j + 1; i < N; ++i) w = c_add(m, w, c_mul(m, c_conj(m, qr[(size_t)i * n + j]), z[i]));
        cmd_t bw = c_mulr(m, w, bet[j]);
        z[j] = c_sub(m, z[j], c_mul(m, bw, vd[j]));
        for (int i = j + 1; i < N; ++i) z[i] = c_sub(m, z[i], c_mul(m, bw, qr[(size_t)i * n + j]));
    }
}

/*
 * Gradient of a real loss through the converged series solution x(t) of
 * f(x(t); c) = 0 mod t^{d+1} (Section 4's system, solved by the Newton
 * steps), with respect to every coefficient of the system.
 * The Jacobian of the truncated system in the series coefficients of x is
 * the block lower triangular Toeplitz matrix T(A) of Section 4, so for the
 * upstream gradient G (G = dL/dRe x + i dL/dIm x, planes (2, m, d+1, n))
 * the coefficient gradient is -B^H lambda with T(A)^H lambda = G, B the
 * derivative of the truncated system in the coefficients.  T(A)^H is block
 * upper triangular: for k = d down to 0,
 *   A_0^H lambda_k = G_k - sum_{j=1}^{d-k} A_j^H lambda_{k+j},
 * solved with the QR factors: R^H y = rhs (forward substitution), then
 * lambda_k = Q (y, 0).  A coefficient c_{tau,j} (degree j of the coefficient
 * series of term tau in equation i) enters f_i through c_tau(t) x^a(t), so
 *   grad c_{tau,j} = - sum_{k=j}^{d} conj(m_{tau,k-j}) lambda_{k,i},
 * m_tau = x^a (1 for a constant term), by forward products.
 * x: the converged series (2, m, d+1, n); grad_coef: planes (2, 2, M, dc+1),
 * the gradient's first two limbs (double double).
 */
int orc_newton_adjoint(int m, int d, int N, int n, int M, int dc, const int32_t *eq_ptr,
                       const int32_t *term_ptr, const int32_t *factors, const double *coef,
                       const double *x, const double *grad_x, double *grad_coef, int32_t *status)
{
    if (!valid_m(m) || d < 0 || n < 1 || N < n || dc < 0) return 1;
    int L = d + 1;
    size_t fsz = (size_t)2 * m * L * N, Asz = (size_t)2 * m * L * N * n, A0sz = (size_t)2 * m * N * n;
    double *f = malloc(sizeof(double) * fsz);
    double *A = malloc(sizeof(double) * Asz);
    double *A0 = malloc(sizeof(double) * A0sz);
    double *QR = malloc(sizeof(double) * A0sz);
    double *vdp = malloc(sizeof(double) * (size_t)2 * m * n);
    double *betp = malloc(sizeof(double) * (size_t)m * n);
    cmd_t *qr = malloc(sizeof(cmd_t) * (size_t)N * n);
    cmd_t *vd = malloc(sizeof(cmd_t) * (size_t)n);
    md_t *bet = malloc(sizeof(md_t) * (size_t)n);
    cmd_t *rhs = malloc(sizeof(cmd_t) * (size_t)L * n);
    cmd_t *lam = malloc(sizeof(cmd_t) * (size_t)L * N);
    cmd_t *y = malloc(sizeof(cmd_t) * (size_t)N);
    cmd_t *ser = malloc(sizeof(cmd_t) * (size_t)L * 3);
    int rc = 3;
    if (!f || !A || !A0 || !QR || !vdp || !betp || !qr || !vd || !bet || !rhs || !lam || !y || !ser)
        goto done;
    rc = orc_eval_diff(m, d, N, n, M, dc, eq_ptr, term_ptr, factors, coef, x, f, A);
    if (rc) goto done;
    int64_t AE = (int64_t)L * N * n, E0 = (int64_t)N * n, xE = (int64_t)L * n;
    for (int p = 0; p < 2 * m; ++p)
        memcpy(A0 + (size_t)p * E0, A + (size_t)p * AE, sizeof(double) * (size_t)E0);
    int32_t st = 0;
    orc_qr(m, N, n, A0, QR, vdp, betp, &st);
    *status = st;
    for (int64_t e = 0; e < E0; ++e) qr[e] = cload(m, QR, E0, e);
    for (int j = 0; j < n; ++j) { vd[j] = cload(m, vdp, n, j); bet[j] = rload(m, betp, n, j); }
    for (int64_t e = 0; e < xE; ++e) rhs[e] = cload(m, grad_x, xE, e);
    for (int k = d; k >= 0; --k) {
        /* R^H y = rhs_k, R^H lower triangular with (R^H)_{il} = conj(R_li) */
        for (int i = 0; i < n; ++i) {
            cmd_t s = rhs[(size_t)k * n + i];
            for (int l = 0; l < i; ++l)
                s = c_sub(m, s, c_mul(m, c_conj(m, qr[(size_t)l * n + i]), y[l]));
            y[i] = c_div(m, s, c_conj(m, qr[(size_t)i * n + i]));
        }
        for (int i = n; i < N; ++i) y[i] = c_zero();
        apply_q(m, N, n, qr, vd, bet, y);
        for (int i = 0; i < N; ++i) lam[(size_t)k * N + i] = y[i];
        /* rhs_{k-j} -= A_j^H lambda_k, j = 1..k */
        for (int j = 1; j <= k; ++j)
            for (int c = 0; c < n; ++c) {
                int64_t base = (int64_t)j * N * n;
                cmd_t t = c_mul(m, c_conj(m, cload(m, A, AE, base + c)), lam[(size_t)k * N]);
                for (int i = 1; i < N; ++i)
                    t = c_add(m, t, c_mul(m, c_conj(m, cload(m, A, AE, base + (int64_t)i * n + c)),
                                          lam[(size_t)k * N + i]));
                rhs[(size_t)(k - j) * n + c] = c_sub(m, rhs[(size_t)(k - j) * n + c], t);
            }
    }
    /* monomial series and the contraction with lambda */
    int64_t cE = (int64_t)M * (dc + 1), gE = cE;
    for (int i = 0; i < N; ++i)
        for (int tau = eq_ptr[i]; tau < eq_ptr[i + 1]; ++tau) {
            const int32_t *v = factors + term_ptr[tau];
            int D = term_ptr[tau + 1] - term_ptr[tau];
            cmd_t *mono = ser, *xv = ser + L, *tmp = ser + 2 * L;
            for (int k = 0; k < L; ++k) mono[k] = c_zero();
            mono[0].re = md_from_d(m, 1.0);
            if (D >= 1)
                for (int k = 0; k < L; ++k) mono[k] = cload(m, x, xE, (int64_t)k * n + v[0]);
            for (int q = 1; q < D; ++q) {
                for (int k = 0; k < L; ++k) xv[k] = cload(m, x, xE, (int64_t)k * n + v[q]);
                ser_mul_mem(m, d, d, mono, xv, tmp);
                for (int k = 0; k < L; ++k) mono[k] = tmp[k];
            }
            for (int j = 0; j <= dc; ++j) {
                cmd_t g = c_zero();
                if (j <= d) {
                    g = c_mul(m, c_conj(m, mono[0]), lam[(size_t)j * N + i]);
                    for (int k = j + 1; k <= d; ++k)
                        g = c_add(m, g, c_mul(m, c_conj(m, mono[k - j]), lam[(size_t)k * N + i]));
                }
                g = c_neg(m, g);
                for (int l = 0; l < 2; ++l) {
                    grad_coef[(int64_t)l * gE + (int64_t)tau * (dc + 1) + j] = l < m ? g.re.v[l] : 0.0;
                    grad_coef[(int64_t)(2 + l) * gE + (int64_t)tau * (dc + 1) + j] = l < m ? g.im.v[l] : 0.0;
                }
            }
        }
    rc = 0;
done:
    free(f); free(A); free(A0); free(QR); free(vdp); free(betp); free(qr); free(vd); free(bet);
    free(rhs); free(lam); free(y); free(ser);
    return rc;
}
