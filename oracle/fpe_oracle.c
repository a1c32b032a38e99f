/*
 * FPE oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU reference for the evaluation phase of the Fast Polynomial
 * Evaluator (FPE) of Anton, Mihalache and Vigneron, "Fast evaluation of real
 * and complex polynomials" (arXiv 2211.06320).  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library; the
 * product library shares no code with it and never calls it.
 *
 * What it computes, and where the paper defines it:
 *   ora_scale         s(z) = 1 + floor(log2 |z|), s(0) = -inf         Section 2.3, eq. (dsz)
 *   ora_precondition  sort s(a_k) decreasingly (ties by increasing k),  Algorithm A_p (preconditioning);
 *                     build the concave cover by the incremental        Section 5.1 (lemma on E_n);
 *                     construction E_0, E_1, ..., list the good set     eq. (threshold)
 *                     G_p = { k : s(a_k) >= Ehat(k) - p - s(d) - 3 }
 *   ora_eval          lambda = log2|z|, k_lambda = argmax(Ehat+lambda Id),  Algorithm A_p (evaluation);
 *                     N = Ehat(k_lambda) + lambda k_lambda, the window   eqs. (defLambda), (defN), (def:LRN),
 *                     [l, r], and Q_lambda(z) = sum over G_p in [l, r]  (reducedQlambda)
 *   ora_horner        P(z) = sum_k a_k z^k by compensated Horner        Section 4.1 (the plain definition);
 *                     (error-free transforms), unbounded exponent       compensated Horner is cited in Section 1
 *   ora_eval_fp64     the same Q_lambda(z), window sum in plain FP64     Algorithm A_p at p = 53 (CPU timing)
 *                     (z^l by binary powering, Horner over the window)   Section 5.2
 *   ora_level_sets    N, x_L, x_R of eq. (def:LRN) for given lambdas     eqs. (defN), (def:LRN)
 *   ora_absum         D(z) = sum_k |a_k| |z|^k                          tolerance scale of the parity metric
 *   ora_eval_deriv    Q'_lambda(z) = sum over the same kept terms of    derivative of eq. (reducedQlambda);
 *                     k a_k z^(k-1)                                      Newton's method, Section 7.2
 *   ora_adjoint_coef  grad_a[k] = sum over the points keeping k of      reverse mode of eq. (reducedQlambda)
 *                     g_j conj(z_j)^k                                    (linear in a; kept set held fixed)
 *   ora_cancel_bound  max(0, floor(N) + 1 - s(v)) >= c, the cancelled   Theorem equivAlgo, eq. (def_prec_loss);
 *                     bits of a value v standing for P(z)                eq. (shear), Section 4.2
 *
 * Precision: every decision that yields an integer (scales, hull, G_p, the
 * argmax, the window ends) is taken in exact integer arithmetic or in FP64,
 * the precision of the method's target (p = 53).  The value sum of ora_eval is
 * accumulated in double-double with a separate 64-bit binary exponent so that
 * the oracle's own rounding stays far below the parity tolerance and no
 * intermediate overflows (the paper's number model has unbounded exponents,
 * Section 2.2).
 *
 * Readings of the paper (where it is silent or ambiguous):
 *   - p counts the bits of an FP64 significand: p = 53 for FP64, 24 for FP32.
 *   - the threshold offset is T = p + s(d) + 3 with d the degree of the
 *     polynomial after removing leading/trailing zero coefficients (Section 4.3
 *     assumes a_0 != 0 and a_d != 0); s(d) is taken for max(d, 1).
 *   - the concave cover is taken of the integer scales s(a_k); collinear
 *     points are not kept as vertices; zero coefficients are never good.
 *   - k_lambda is the leftmost maximiser; the window ends are
 *     l = ceil(x_L - eta), r = floor(x_R + eta), eta = 2^-20, clamped to the
 *     trimmed index range (a superset only adds accuracy).
 *   - P(0) = a_0; a non-finite z yields NaN.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -pthread (contraction must be
 * off: the error-free transforms below rely on separately rounded operations).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_NEG_INF INT64_MIN
#define ORA_ETA 0x1p-20

/* ------------------------------------------------------------------------- */
/* Scale of a complex number, exactly (Section 2.3, eq. (dsz), eq. (sz)).     */
/* s(x + iy) is max(s(x), s(y)) or one more; it is one more iff               */
/* x^2 + y^2 >= 4^m with m = max(s(x), s(y)).  Decided with 128-bit integers   */
/* on the 53-bit significands, so the answer is exact for every double.        */
/* ------------------------------------------------------------------------- */
int64_t ora_scale1(double x, double y)
{
    if (x == 0.0 && y == 0.0) return ORA_NEG_INF;
    int ex = INT32_MIN, ey = INT32_MIN;
    double fx = 0.0, fy = 0.0;
    if (x != 0.0) fx = frexp(fabs(x), &ex);   /* |x| = fx 2^ex, fx in [1/2, 1): s(x) = ex */
    if (y != 0.0) fy = frexp(fabs(y), &ey);
    int m = ex > ey ? ex : ey;
    /* integer significands: |x| = X 2^(ex - 53) */
    unsigned __int128 X = (unsigned __int128)(uint64_t)ldexp(fx, 53);
    unsigned __int128 Y = (unsigned __int128)(uint64_t)ldexp(fy, 53);
    unsigned __int128 A = X * X, B = Y * Y;        /* each < 2^106 */
    unsigned __int128 sum = 0;
    if (x != 0.0) { int sh = 2 * (m - ex); if (sh < 128) sum += A >> sh; }   /* sh >= 0 */
    if (y != 0.0) { int sh = 2 * (m - ey); if (sh < 128) sum += B >> sh; }
    /* x^2 + y^2 >= 4^m  <=>  X^2 4^(ex-m) + Y^2 4^(ey-m) >= 2^106; the floor of
       the smaller term does not change the comparison because the larger term
       and 2^106 are integers. */
    unsigned __int128 two106 = (unsigned __int128)1 << 106;
    return sum >= two106 ? (int64_t)m + 1 : (int64_t)m;
}

void ora_scale(const double *c, int64_t n, int64_t *s)
{
    for (int64_t k = 0; k < n; ++k) s[k] = ora_scale1(c[2 * k], c[2 * k + 1]);
}

static int64_t bitlen(int64_t v) /* s(v) = 1 + floor(log2 v) for an integer v >= 1 */
{
    int64_t b = 0;
    while (v > 0) { ++b; v >>= 1; }
    return b;
}

/* ------------------------------------------------------------------------- */
/* Preconditioning (Algorithm A_p, first block; Section 5.1).                 */
/* ------------------------------------------------------------------------- */
typedef struct ora_plan {
    int64_t d;          /* degree as given (d + 1 coefficients) */
    int64_t v, dt;      /* first and last nonzero index; -1 if P == 0 */
    int32_t p;
    int64_t T;          /* p + s(max(dt - v, 1)) + 3 */
    int64_t nh;         /* number of vertices of the concave cover */
    int64_t *hk, *hs;   /* vertices (k_i, s(a_{k_i})), increasing k */
    int64_t *s;         /* s(a_k), ORA_NEG_INF for a zero coefficient */
    uint8_t *good;      /* G_p indicator, d + 1 entries */
    int64_t ngood;
    double *coef;       /* copy of the coefficients, interleaved re, im */
} ora_plan;

typedef struct { int64_t k, s; } ora_pt;

static int ora_cmp_pts(const void *pa, const void *pb)
{
    const ora_pt *a = pa, *b = pb;
    if (a->s != b->s) return a->s > b->s ? -1 : 1;   /* decreasing scale */
    return a->k < b->k ? -1 : (a->k > b->k);           /* ties: increasing k */
}

/* v0 stays a vertex between a (left) and b (right) iff the slope a->v0 is
   strictly larger than the slope v0->b (concavity, collinear points dropped). */
static int strictly_above(int64_t ak, int64_t as, int64_t vk, int64_t vs, int64_t bk, int64_t bs)
{
    /* (vs - as)/(vk - ak) > (bs - vs)/(bk - vk), denominators positive */
    __int128 lhs = (__int128)(vs - as) * (bk - vk);
    __int128 rhs = (__int128)(bs - vs) * (vk - ak);
    return lhs > rhs;
}

void ora_plan_free(ora_plan *P)
{
    if (!P) return;
    free(P->hk); free(P->hs); free(P->s); free(P->good); free(P->coef); free(P);
}

/* T_fixed < 0: T = p + s(d_eff) + 3 as in the algorithm; T_fixed >= 0 sets the
   threshold offset directly (the worked example of Section 4.2 uses p alone). */
static ora_plan *ora_precondition_impl(const double *coef, int64_t d, int32_t p, int64_t T_fixed)
{
    ora_plan *P = calloc(1, sizeof *P);
    if (!P) return NULL;
    P->d = d; P->p = p; P->v = -1; P->dt = -1;
    P->s = malloc(sizeof(int64_t) * (size_t)(d + 1));
    P->good = calloc((size_t)(d + 1), 1);
    P->coef = malloc(sizeof(double) * 2 * (size_t)(d + 1));
    P->hk = malloc(sizeof(int64_t) * (size_t)(d + 1));
    P->hs = malloc(sizeof(int64_t) * (size_t)(d + 1));
    if (!P->s || !P->good || !P->coef || !P->hk || !P->hs) { ora_plan_free(P); return NULL; }
    memcpy(P->coef, coef, sizeof(double) * 2 * (size_t)(d + 1));

    /* Algorithm A_p, preconditioning: compute and sort s(a_k) */
    ora_scale(coef, d + 1, P->s);
    int64_t nz = 0;
    for (int64_t k = 0; k <= d; ++k) if (P->s[k] != ORA_NEG_INF) ++nz;
    if (nz == 0) { P->nh = 0; P->T = 0; return P; }   /* P == 0 */
    ora_pt *pts = malloc(sizeof(ora_pt) * (size_t)nz);
    int64_t j = 0;
    for (int64_t k = 0; k <= d; ++k)
        if (P->s[k] != ORA_NEG_INF) { pts[j].k = k; pts[j].s = P->s[k]; ++j; }
    qsort(pts, (size_t)nz, sizeof(ora_pt), ora_cmp_pts);

    /* Algorithm A_p, preconditioning: the concave cover, by the incremental construction of the
       lemma in Section 5.1.  E_n covers [l_n, r_n], the hull of the first n+1
       sorted abscissae.  A new point strictly inside (l_n, r_n) lies under E_n
       (its scale is <= every earlier one); a point left of l_n (right of r_n)
       extends E_n on that side after dropping the vertices that would break
       concavity.  Vertices live in a deque stored in buf[lo..hi]. */
    int64_t cap = 2 * nz + 2;
    ora_pt *buf = malloc(sizeof(ora_pt) * (size_t)cap);
    int64_t lo = nz + 1, hi = nz + 1;     /* buf[lo..hi] inclusive */
    buf[lo] = pts[0];
    for (int64_t n = 1; n < nz; ++n) {
        ora_pt q = pts[n];
        if (q.k > buf[lo].k && q.k < buf[hi].k) continue;   /* E_{n+1} = E_n */
        if (q.k < buf[lo].k) {
            while (hi - lo >= 1 && !strictly_above(q.k, q.s, buf[lo].k, buf[lo].s, buf[lo + 1].k, buf[lo + 1].s))
                ++lo;
            buf[--lo] = q;
        } else {
            while (hi - lo >= 1 && !strictly_above(buf[hi - 1].k, buf[hi - 1].s, buf[hi].k, buf[hi].s, q.k, q.s))
                --hi;
            buf[++hi] = q;
        }
    }
    P->nh = hi - lo + 1;
    for (int64_t i = 0; i < P->nh; ++i) { P->hk[i] = buf[lo + i].k; P->hs[i] = buf[lo + i].s; }
    free(buf); free(pts);
    P->v = P->hk[0];
    P->dt = P->hk[P->nh - 1];

    /* Algorithm A_p, preconditioning: the good set, s(a_k) >= Ehat(k) - T, exactly, with Ehat(k) linear
       between consecutive vertices. */
    int64_t deff = P->dt - P->v;
    P->T = T_fixed >= 0 ? T_fixed : (int64_t)p + bitlen(deff > 1 ? deff : 1) + 3;
    int64_t seg = 0;
    for (int64_t k = P->v; k <= P->dt; ++k) {
        if (P->s[k] == ORA_NEG_INF) continue;
        while (seg + 1 < P->nh - 1 && P->hk[seg + 1] < k) ++seg;
        int64_t ok;
        if (P->nh == 1) ok = 1;
        else {
            /* k lies on the segment [k0, k1] of the cover */
            int64_t k0 = P->hk[seg], k1 = P->hk[seg + 1], e0 = P->hs[seg], e1 = P->hs[seg + 1];
            /* s_k >= e0 + (e1 - e0)(k - k0)/(k1 - k0) - T, cleared of the denominator */
            ok = (__int128)(P->s[k] + P->T - e0) * (k1 - k0) >= (__int128)(e1 - e0) * (k - k0);
        }
        if (ok) { P->good[k] = 1; ++P->ngood; }
    }
    return P;
}

ora_plan *ora_precondition(const double *coef, int64_t d, int32_t p)
{
    return ora_precondition_impl(coef, d, p, -1);
}

ora_plan *ora_precondition_offset(const double *coef, int64_t d, int64_t T)
{
    return ora_precondition_impl(coef, d, 0, T);
}

void ora_plan_info(const ora_plan *P, int64_t *out /* 7 */)
{
    out[0] = P->d; out[1] = P->v; out[2] = P->dt; out[3] = P->nh;
    out[4] = P->ngood; out[5] = P->T; out[6] = P->p;
}

void ora_plan_hull(const ora_plan *P, int64_t *hk, int64_t *hs)
{
    for (int64_t i = 0; i < P->nh; ++i) { hk[i] = P->hk[i]; hs[i] = P->hs[i]; }
}

void ora_plan_good(const ora_plan *P, uint8_t *good)
{
    memcpy(good, P->good, (size_t)(P->d + 1));
}

void ora_plan_scales(const ora_plan *P, int64_t *s)
{
    memcpy(s, P->s, sizeof(int64_t) * (size_t)(P->d + 1));
}

/* ------------------------------------------------------------------------- */
/* Double-double numbers and complex numbers with a separate exponent.        */
/* ------------------------------------------------------------------------- */
typedef struct { double hi, lo; } dd_t;

static dd_t two_sum(double a, double b)
{
    double s = a + b, bb = s - a;
    dd_t r = { s, (a - (s - bb)) + (b - bb) };
    return r;
}
static dd_t fast_two_sum(double a, double b)   /* |a| >= |b| or a == 0 */
{
    double s = a + b;
    dd_t r = { s, b - (s - a) };
    return r;
}
static dd_t two_prod(double a, double b)
{
    double p = a * b;
    dd_t r = { p, fma(a, b, -p) };
    return r;
}
static dd_t dd_add(dd_t a, dd_t b)
{
    dd_t s = two_sum(a.hi, b.hi), t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}
static dd_t dd_neg(dd_t a) { dd_t r = { -a.hi, -a.lo }; return r; }
static dd_t dd_mul(dd_t a, dd_t b)
{
    dd_t p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return fast_two_sum(p.hi, p.lo);
}
static dd_t dd_ldexp(dd_t a, int64_t e)
{
    if (e < -3000) { dd_t z = { 0.0, 0.0 }; return z; }
    if (e > 3000) e = 3000;
    dd_t r = { ldexp(a.hi, (int)e), ldexp(a.lo, (int)e) };
    return r;
}

/* value = (re + i im) * 2^e; normalised so that max(|re.hi|, |im.hi|) is in
   [1/2, 1), or everything zero with e = 0. */
typedef struct { dd_t re, im; int64_t e; } xc_t;

static xc_t xc_norm(xc_t x)
{
    double m = fmax(fabs(x.re.hi), fabs(x.im.hi));
    if (m == 0.0) {
        /* a zero high part with a nonzero low part cannot occur after the
           renormalising operations above; treat as zero */
        xc_t z = { { 0, 0 }, { 0, 0 }, 0 };
        return z;
    }
    int k;
    frexp(m, &k);
    x.re = dd_ldexp(x.re, -k);
    x.im = dd_ldexp(x.im, -k);
    x.e += k;
    return x;
}
static xc_t xc_from(double re, double im)
{
    xc_t x = { { re, 0 }, { im, 0 }, 0 };
    return xc_norm(x);
}
static int xc_is_zero(xc_t x) { return x.re.hi == 0.0 && x.im.hi == 0.0; }
static xc_t xc_mul(xc_t a, xc_t b)
{
    xc_t r;
    r.re = dd_add(dd_mul(a.re, b.re), dd_neg(dd_mul(a.im, b.im)));
    r.im = dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re));
    r.e = a.e + b.e;
    return xc_norm(r);
}
static xc_t xc_add(xc_t a, xc_t b)
{
    if (xc_is_zero(a)) return b;
    if (xc_is_zero(b)) return a;
    if (a.e < b.e) { xc_t t = a; a = b; b = t; }
    int64_t sh = b.e - a.e;                  /* <= 0 */
    xc_t r;
    r.re = dd_add(a.re, dd_ldexp(b.re, sh));
    r.im = dd_add(a.im, dd_ldexp(b.im, sh));
    r.e = a.e;
    return xc_norm(r);
}
/* z^n by binary powering (Section 5.2: z^l in 2 log2 l multiplications) */
static xc_t xc_pow(xc_t z, int64_t n)
{
    xc_t r = xc_from(1.0, 0.0), b = z;
    while (n > 0) {
        if (n & 1) r = xc_mul(r, b);
        n >>= 1;
        if (n) b = xc_mul(b, b);
    }
    return r;
}
/* rounds to a (double complex mantissa, exponent) pair, normalised as above */
static void xc_out(xc_t x, double *m, int64_t *e)
{
    double re = x.re.hi + x.re.lo, im = x.im.hi + x.im.lo;
    double mx = fmax(fabs(re), fabs(im));
    if (mx == 0.0) { m[0] = 0.0; m[1] = 0.0; *e = 0; return; }
    int k;
    frexp(mx, &k);
    m[0] = ldexp(re, -k); m[1] = ldexp(im, -k); *e = x.e + k;
}

/* real nonnegative numbers with a separate exponent: value = m 2^e */
typedef struct { double m; int64_t e; } xr_t;
static xr_t xr_norm(xr_t x)
{
    if (x.m == 0.0) { x.e = 0; return x; }
    int k;
    frexp(x.m, &k);
    x.m = ldexp(x.m, -k);
    x.e += k;
    return x;
}
static xr_t xr_add(xr_t a, xr_t b)
{
    if (a.m == 0.0) return b;
    if (b.m == 0.0) return a;
    if (a.e < b.e) { xr_t t = a; a = b; b = t; }
    int64_t sh = b.e - a.e;
    xr_t r = { a.m + (sh < -2000 ? 0.0 : ldexp(b.m, (int)sh)), a.e };
    return xr_norm(r);
}

/* lambda = log2|z| in FP64 (the precision of the method's target). */
static double ora_log2abs(double x, double y)
{
    int k;
    double mx = fmax(fabs(x), fabs(y));
    frexp(mx, &k);
    return (double)k + log2(hypot(ldexp(x, -k), ldexp(y, -k)));
}

/* ------------------------------------------------------------------------- */
/* Evaluation of one point (Algorithm A_p, second block; Section 5.2).        */
/* ------------------------------------------------------------------------- */
/* evaluation for one lambda: k_lambda = argmax(Ehat + lambda Id), N (eq. defN)
   and the real ends x_L <= x_R of the level set {x : Ehat(x) + lambda x >= N - T}
   (eq. def:LRN); returns N.  P must have at least one cover vertex.  dlev
   moves the level to N - T + dlev (0 in the method; tests move it by the size
   of its rounding). */
static double ora_level_set(const ora_plan *P, double lam, double dlev, double *xLo, double *xRo)
{
    /* k_lambda = argmax(Ehat + lambda Id); the maximum of a concave
       piecewise-linear function is at a vertex; scan them all, keep the
       leftmost maximiser. */
    int64_t nh = P->nh, istar = 0;
    double *F = malloc(sizeof(double) * (size_t)nh);
    for (int64_t i = 0; i < nh; ++i) {
        F[i] = (double)P->hs[i] + lam * (double)P->hk[i];
        if (F[i] > F[istar]) istar = i;
    }
    /* N = Ehat(k_lambda) + lambda k_lambda (eq. defN) */
    double N = F[istar];
    /* the window at the level N - p - s(d) - 3 (eq. def:LRN); the level set of
       the concave function is an interval [x_L, x_R]. */
    double L = N - (double)P->T + dlev;
    double xL, xR;
    if (F[0] >= L) xL = (double)P->hk[0];
    else {
        int64_t i = istar;
        while (F[i - 1] >= L) --i;      /* F[i-1] < L <= F[i] */
        xL = (double)P->hk[i - 1] + (L - F[i - 1]) * (double)(P->hk[i] - P->hk[i - 1]) / (F[i] - F[i - 1]);
    }
    if (F[nh - 1] >= L) xR = (double)P->hk[nh - 1];
    else {
        int64_t i = istar;
        while (F[i + 1] >= L) ++i;      /* F[i] >= L > F[i+1] */
        xR = (double)P->hk[i] + (F[i] - L) * (double)(P->hk[i + 1] - P->hk[i]) / (F[i] - F[i + 1]);
    }
    free(F);
    *xLo = xL;
    *xRo = xR;
    return N;
}

/* N, x_L and x_R (as ora_level_set) for n given values of lambda and level
   offsets dlev (NULL: 0); NaN for a plan with no vertex.  Tests use it to find
   the points whose window ends would move under perturbations of lambda and
   of the level of the size of their rounding. */
void ora_level_sets(const ora_plan *P, const double *lam, const double *dlev, int64_t n, double *N, double *xL,
                    double *xR)
{
    for (int64_t j = 0; j < n; ++j) {
        if (P->nh == 0 || !isfinite(lam[j])) { N[j] = xL[j] = xR[j] = NAN; continue; }
        N[j] = ora_level_set(P, lam[j], dlev ? dlev[j] : 0.0, xL + j, xR + j);
    }
}

typedef struct {
    double m[2]; int64_t e;     /* Q_lambda(z) = (m0 + i m1) 2^e */
    double md[2]; int64_t de;   /* Q'_lambda(z) = sum over the kept terms of k a_k z^(k-1) */
    double ddm; int64_t dde;    /* sum over the window of |k a_k| |z|^(k-1) (its scale) */
    int64_t l, r;               /* window; l > r when empty */
    int64_t terms;              /* #(G_p within [l, r]) */
    double dwin_m; int64_t dwin_e;   /* sum over [l, r] of |a_k||z|^k */
    double lambda, N;
} ora_res;

static void ora_eval1(const ora_plan *P, double zr, double zi, int deriv, ora_res *o)
{
    memset(o, 0, sizeof *o);
    o->l = 0; o->r = -1;
    if (!isfinite(zr) || !isfinite(zi)) {
        o->m[0] = o->m[1] = NAN; o->lambda = NAN; o->N = NAN;
        o->md[0] = o->md[1] = NAN;
        return;
    }
    if (P->nh == 0) return;                          /* P == 0 */
    const double *a = P->coef;
    if (zr == 0.0 && zi == 0.0) {                    /* P(0) = a_0 */
        o->l = 0; o->r = 0; o->lambda = -INFINITY; o->N = -INFINITY;
        if (P->v == 0) {
            xc_out(xc_from(a[0], a[1]), o->m, &o->e);
            o->terms = P->good[0];
            xr_t ab = xr_norm((xr_t){ hypot(a[0], a[1]), 0 });
            o->dwin_m = ab.m; o->dwin_e = ab.e;
        }
        return;
    }
    /* evaluation: lambda = log2|z| (eq. defLambda) */
    double lam = ora_log2abs(zr, zi);
    o->lambda = lam;
    /* evaluation: k_lambda, N (eq. defN) and the level set [x_L, x_R] of
       eq. (def:LRN) */
    double xL, xR;
    double N = ora_level_set(P, lam, 0.0, &xL, &xR);
    o->N = N;
    int64_t l = (int64_t)ceil(xL - ORA_ETA), r = (int64_t)floor(xR + ORA_ETA);
    if (l < P->v) l = P->v;
    if (r > P->dt) r = P->dt;
    o->l = l; o->r = r;

    /* evaluation: Q_lambda(z) = sum over G_p within [l, r] of a_k z^k; z^l by binary
       powering, then the terms one by one with the running power z^k. */
    xc_t z = xc_from(zr, zi);
    xc_t pw = xc_pow(z, l);
    xc_t S = xc_from(0.0, 0.0);
    xr_t D = { 0.0, 0 };
    int64_t U = 0;
    for (int64_t k = l; k <= r; ++k) {
        double ar = a[2 * k], ai = a[2 * k + 1];
        if (ar != 0.0 || ai != 0.0) {
            double pabs = hypot(pw.re.hi, pw.im.hi);
            D = xr_add(D, xr_norm((xr_t){ hypot(ar, ai) * pabs, pw.e }));
        }
        if (P->good[k]) {
            S = xc_add(S, xc_mul(xc_from(ar, ai), pw));
            ++U;
        }
        if (k < r) pw = xc_mul(pw, z);
    }
    xc_out(S, o->m, &o->e);
    o->terms = U;
    o->dwin_m = D.m; o->dwin_e = D.e;

    /* derivative of the kept terms (the same window and good set):
       Q' = sum of k a_k z^(k-1), with the running power z^(k-1); and its scale
       sum of |k a_k| |z|^(k-1) over the window */
    if (deriv) {
        int64_t k0 = l < 1 ? 1 : l;
        xc_t pd = xc_pow(z, k0 - 1);
        xc_t Sd = xc_from(0.0, 0.0);
        xr_t Dd = { 0.0, 0 };
        for (int64_t k = k0; k <= r; ++k) {
            double ar = a[2 * k], ai = a[2 * k + 1];
            if (ar != 0.0 || ai != 0.0) {
                double pabs = hypot(pd.re.hi, pd.im.hi);
                Dd = xr_add(Dd, xr_norm((xr_t){ hypot(ar, ai) * (double)k * pabs, pd.e }));
            }
            if (P->good[k]) Sd = xc_add(Sd, xc_mul(xc_mul(xc_from(ar, ai), xc_from((double)k, 0.0)), pd));
            if (k < r) pd = xc_mul(pd, z);
        }
        xc_out(Sd, o->md, &o->de);
        o->ddm = Dd.m; o->dde = Dd.e;
    }
}

/* ------------------------------------------------------------------------- */
/* Compensated Horner for the full polynomial, with an unbounded exponent.    */
/* State: value = (h + c) 2^E with h the FP64 Horner value and c the running   */
/* sum of the exact rounding errors of each step (error-free transforms:       */
/* TwoSum, and TwoProd through fma), propagated by c <- c z + err.             */
/* z = zm 2^ze with max(|Re zm|, |Im zm|) in [1/2, 1); the factor 2^ze is      */
/* moved into E, so every step multiplies by zm only and adds a_k 2^-E.        */
/* ------------------------------------------------------------------------- */
static int max_exp(double re, double im)
{
    double m = fmax(fabs(re), fabs(im));
    int k;
    frexp(m, &k);
    return k;
}

static void ora_horner1(const double *a, int64_t d, double zr, double zi,
                        double *mo, int64_t *eo)
{
    if (!isfinite(zr) || !isfinite(zi)) { mo[0] = mo[1] = NAN; *eo = 0; return; }
    int64_t top = d;
    while (top >= 0 && a[2 * top] == 0.0 && a[2 * top + 1] == 0.0) --top;
    if (top < 0) { mo[0] = mo[1] = 0.0; *eo = 0; return; }
    if (zr == 0.0 && zi == 0.0) {
        xc_out(xc_from(a[0], a[1]), mo, eo);
        return;
    }
    int ze = max_exp(zr, zi);
    double wr = ldexp(zr, -ze), wi = ldexp(zi, -ze);
    /* start at the leading coefficient, scaled to a unit exponent */
    int64_t E = max_exp(a[2 * top], a[2 * top + 1]);
    double hr = ldexp(a[2 * top], (int)-E), hi = ldexp(a[2 * top + 1], (int)-E);
    double cr = 0.0, ci = 0.0;
    for (int64_t k = top - 1; k >= 0; --k) {
        E += ze;                                   /* h z = (h zm) 2^(E + ze) */
        double ar = a[2 * k], ai = a[2 * k + 1];
        if (ar != 0.0 || ai != 0.0) {
            /* keep the coefficient representable in the current scale: if it
               dominates by far, rebase the state onto its exponent */
            int64_t ea = max_exp(ar, ai);
            if (ea - E > 600) {
                int64_t sh = E - ea;               /* < -600: the old state is tiny */
                hr = sh < -1500 ? 0.0 : ldexp(hr, (int)sh); hi = sh < -1500 ? 0.0 : ldexp(hi, (int)sh);
                cr = sh < -1500 ? 0.0 : ldexp(cr, (int)sh); ci = sh < -1500 ? 0.0 : ldexp(ci, (int)sh);
                E = ea;
            }
        }
        int64_t sa = -E;
        double br = (ar == 0.0 || sa < -1500) ? 0.0 : ldexp(ar, (int)(sa > 1500 ? 1500 : sa));
        double bi = (ai == 0.0 || sa < -1500) ? 0.0 : ldexp(ai, (int)(sa > 1500 ? 1500 : sa));
        /* [p, pi] = TwoProd for the four real products of h * zm */
        dd_t p1 = two_prod(hr, wr), p2 = two_prod(hi, wi);
        dd_t p3 = two_prod(hr, wi), p4 = two_prod(hi, wr);
        dd_t sr = two_sum(p1.hi, -p2.hi), si = two_sum(p3.hi, p4.hi);
        dd_t tr = two_sum(sr.hi, br), ti = two_sum(si.hi, bi);
        double er = p1.lo - p2.lo + sr.lo + tr.lo;
        double ei = p3.lo + p4.lo + si.lo + ti.lo;
        double ncr = cr * wr - ci * wi + er;
        double nci = cr * wi + ci * wr + ei;
        hr = tr.hi; hi = ti.hi; cr = ncr; ci = nci;
        /* renormalise the state by an exact power of two */
        double mh = fmax(fabs(hr), fabs(hi));
        if (mh > 0x1p200 || (mh < 0x1p-200 && mh > 0.0)) {
            int kk;
            frexp(mh, &kk);
            hr = ldexp(hr, -kk); hi = ldexp(hi, -kk);
            cr = ldexp(cr, -kk); ci = ldexp(ci, -kk);
            E += kk;
        } else if (mh == 0.0) {
            double mc = fmax(fabs(cr), fabs(ci));
            if (mc > 0.0) {
                int kk;
                frexp(mc, &kk);
                cr = ldexp(cr, -kk); ci = ldexp(ci, -kk);
                E += kk;
            }
        }
    }
    /* result h + c, rounded once */
    dd_t rr = two_sum(hr, cr), ri = two_sum(hi, ci);
    xc_t x = { rr, ri, E };
    x = xc_norm(x);
    xc_out(x, mo, eo);
}

/* D(z) = sum_k |a_k| |z|^k, with an unbounded exponent (tolerance scale). */
static void ora_absum1(const double *a, int64_t d, double zr, double zi, double *dm, int64_t *de)
{
    xr_t z = xr_norm((xr_t){ 0.0, 0 });
    {
        int k;
        double mx = fmax(fabs(zr), fabs(zi));
        if (mx == 0.0) { xr_t a0 = xr_norm((xr_t){ hypot(a[0], a[1]), 0 }); *dm = a0.m; *de = a0.e; return; }
        frexp(mx, &k);
        z.m = hypot(ldexp(zr, -k), ldexp(zi, -k)); z.e = k;
        z = xr_norm(z);
    }
    xr_t pw = { 0.5, 1 }, S = { 0.0, 0 };   /* pw = |z|^k, starting at 1 */
    for (int64_t k = 0; k <= d; ++k) {
        double ab = hypot(a[2 * k], a[2 * k + 1]);
        if (ab != 0.0) S = xr_add(S, xr_norm((xr_t){ ab * pw.m, pw.e }));
        pw = xr_norm((xr_t){ pw.m * z.m, pw.e + z.e });
    }
    *dm = S.m; *de = S.e;
}

/* ------------------------------------------------------------------------- */
/* The evaluation with its window sum in plain FP64 (Algorithm A_p, second    */
/* block, at the precision of the method's target): lambda, N and [l, r] as   */
/* in ora_eval1, z^l by binary powering (Section 5.2) with a separate binary  */
/* exponent, then Horner's rule over the window with the terms outside G_p    */
/* skipped, on the coefficients scaled by 2^-c, c = floor(N - lambda l), so   */
/* that every kept term a_k z^(k-l) 2^-c is below 4 in modulus (eq. shear).   */
/* The CPU baseline times this form; its values are pinned against exact      */
/* rationals.  The Horner partials stay in the FP64 range while |lambda| W    */
/* and the spread of the cover over the window stay below about 900 bits.     */
/* ------------------------------------------------------------------------- */
static void ora_cmul_norm(double *xr, double *xi, int64_t *xe, double yr, double yi, int64_t ye)
{
    double r = *xr * yr - *xi * yi, i = *xr * yi + *xi * yr;
    double mx = fmax(fabs(r), fabs(i));
    int k = 0;
    if (mx != 0.0) frexp(mx, &k);
    *xr = ldexp(r, -k);
    *xi = ldexp(i, -k);
    *xe += ye + k;
}

static void ora_eval1_fp64(const ora_plan *P, double zr, double zi, double *m, int64_t *e)
{
    m[0] = m[1] = 0.0;
    *e = 0;
    if (!isfinite(zr) || !isfinite(zi)) { m[0] = m[1] = NAN; return; }
    if (P->nh == 0) return;                          /* P == 0 */
    const double *a = P->coef;
    if (zr == 0.0 && zi == 0.0) {                    /* P(0) = a_0 */
        if (P->v == 0) xc_out(xc_from(a[0], a[1]), m, e);
        return;
    }
    double lam = ora_log2abs(zr, zi);
    double xL, xR;
    double N = ora_level_set(P, lam, 0.0, &xL, &xR);
    int64_t l = (int64_t)ceil(xL - ORA_ETA), r = (int64_t)floor(xR + ORA_ETA);
    if (l < P->v) l = P->v;
    if (r > P->dt) r = P->dt;
    /* z^l = (pr + i pi) 2^pe by right-to-left binary powering of w = z 2^-ez */
    int ez = max_exp(zr, zi);
    double wr = ldexp(zr, -ez), wi = ldexp(zi, -ez);
    double pr = 1.0, pi = 0.0, br = wr, bi = wi;
    int64_t pe = 0, be = 0;
    for (int64_t n = l; n > 0; n >>= 1) {
        if (n & 1) ora_cmul_norm(&pr, &pi, &pe, br, bi, be);
        if (n > 1) ora_cmul_norm(&br, &bi, &be, br, bi, be);
    }
    pe += l * (int64_t)ez;
    /* Horner's rule over the window on a_k 2^-c */
    int64_t c = (int64_t)floor(N - lam * (double)l);
    int exact_scale = c > -1000 && c < 1000;
    double sc = exact_scale ? ldexp(1.0, (int)-c) : 0.0;
    double hr = 0.0, hi = 0.0;
    for (int64_t k = r; k >= l; --k) {
        double tr = hr * zr - hi * zi, ti = hr * zi + hi * zr;
        if (P->good[k]) {
            if (exact_scale) { tr += a[2 * k] * sc; ti += a[2 * k + 1] * sc; }
            else { tr += ldexp(a[2 * k], (int)-c); ti += ldexp(a[2 * k + 1], (int)-c); }
        }
        hr = tr;
        hi = ti;
    }
    double qr = hr * pr - hi * pi, qi = hr * pi + hi * pr;
    double mx = fmax(fabs(qr), fabs(qi));
    if (mx == 0.0) return;
    int k;
    frexp(mx, &k);
    m[0] = ldexp(qr, -k);
    m[1] = ldexp(qi, -k);
    *e = pe + c + k;
}

/* ------------------------------------------------------------------------- */
/* Batch drivers (points are independent; threads split the point range).    */
/* ------------------------------------------------------------------------- */
typedef struct {
    int kind;                  /* 0 = eval, 1 = horner, 2 = absum, 3 = eval, FP64 window sum */
    const ora_plan *P;
    const double *coef; int64_t d;
    const double *z; int64_t i0, i1;
    double *m; int64_t *e, *l, *r, *terms;
    double *dwin_m; int64_t *dwin_e; double *lambda, *N;
    double *md; int64_t *de; double *ddm; int64_t *dde;   /* derivative (eval only) */
} ora_job;

static void *ora_worker(void *arg)
{
    ora_job *J = arg;
    for (int64_t i = J->i0; i < J->i1; ++i) {
        double zr = J->z[2 * i], zi = J->z[2 * i + 1];
        if (J->kind == 0) {
            ora_res o;
            ora_eval1(J->P, zr, zi, J->md != NULL, &o);
            J->m[2 * i] = o.m[0]; J->m[2 * i + 1] = o.m[1]; J->e[i] = o.e;
            if (J->md) {
                J->md[2 * i] = o.md[0]; J->md[2 * i + 1] = o.md[1]; J->de[i] = o.de;
                J->ddm[i] = o.ddm; J->dde[i] = o.dde;
            }
            if (J->l) J->l[i] = o.l;
            if (J->r) J->r[i] = o.r;
            if (J->terms) J->terms[i] = o.terms;
            if (J->dwin_m) J->dwin_m[i] = o.dwin_m;
            if (J->dwin_e) J->dwin_e[i] = o.dwin_e;
            if (J->lambda) J->lambda[i] = o.lambda;
            if (J->N) J->N[i] = o.N;
        } else if (J->kind == 1) {
            ora_horner1(J->coef, J->d, zr, zi, J->m + 2 * i, J->e + i);
        } else if (J->kind == 3) {
            ora_eval1_fp64(J->P, zr, zi, J->m + 2 * i, J->e + i);
        } else {
            ora_absum1(J->coef, J->d, zr, zi, J->m + i, J->e + i);
        }
    }
    return NULL;
}

static void ora_run(ora_job base, int64_t n, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (n < 64) nthreads = 1;
    pthread_t th[256];
    ora_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = base;
        jobs[t].i0 = n * t / nthreads;
        jobs[t].i1 = n * (t + 1) / nthreads;
    }
    if (nthreads == 1) { ora_worker(&jobs[0]); return; }
    int started[256] = { 0 };
    for (int t = 0; t < nthreads; ++t)
        started[t] = pthread_create(&th[t], NULL, ora_worker, &jobs[t]) == 0;
    for (int t = 0; t < nthreads; ++t) {
        if (started[t]) pthread_join(th[t], NULL);
        else ora_worker(&jobs[t]);
    }
}

void ora_eval(const ora_plan *P, const double *z, int64_t n, double *m, int64_t *e,
              int64_t *l, int64_t *r, int64_t *terms, double *dwin_m, int64_t *dwin_e,
              double *lambda, double *N, int nthreads)
{
    ora_job J = { 0, P, NULL, 0, z, 0, 0, m, e, l, r, terms, dwin_m, dwin_e, lambda, N, NULL, NULL, NULL, NULL };
    ora_run(J, n, nthreads);
}

/* Q and Q' (the derivative of the kept terms), with the scale of each */
void ora_eval_deriv(const ora_plan *P, const double *z, int64_t n, double *m, int64_t *e,
                    double *dwin_m, int64_t *dwin_e, double *md, int64_t *de, double *ddm, int64_t *dde,
                    int nthreads)
{
    ora_job J = { 0, P, NULL, 0, z, 0, 0, m, e, NULL, NULL, NULL, dwin_m, dwin_e, NULL, NULL, md, de, ddm, dde };
    ora_run(J, n, nthreads);
}

/* Q_lambda(z) with the window sum in plain FP64 (ora_eval1_fp64) */
void ora_eval_fp64(const ora_plan *P, const double *z, int64_t n, double *m, int64_t *e, int nthreads)
{
    ora_job J = { 3, P, NULL, 0, z, 0, 0, m, e, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL };
    ora_run(J, n, nthreads);
}

void ora_horner(const double *coef, int64_t d, const double *z, int64_t n,
                double *m, int64_t *e, int nthreads)
{
    ora_job J = { 1, NULL, coef, d, z, 0, 0, m, e, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL };
    ora_run(J, n, nthreads);
}

void ora_absum(const double *coef, int64_t d, const double *z, int64_t n,
               double *dm, int64_t *de, int nthreads)
{
    ora_job J = { 2, NULL, coef, d, z, 0, 0, dm, de, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL };
    ora_run(J, n, nthreads);
}

/* ------------------------------------------------------------------------- */
/* Cancelled bits (Theorem equivAlgo, eq. (def_prec_loss), Section 4.3):      */
/* c = 0 when |P(z)| >= M, else s(M) - s(P(z)), with M = max_j |a_j z^j|.     */
/* By eq. (shear) (Section 4.2) s(a_j z^j) <= s(a_j) + j lambda + 1, and       */
/* s(a_j) <= Ehat(j), so s(M) <= N + 1 and, s(M) being an integer,            */
/* s(M) <= floor(N) + 1.  The reported count is the upper bound               */
/* max(0, floor(N) + 1 - s(v)) for a value v = m 2^e standing for P(z) (the    */
/* value the method returned); with the exact c it satisfies                   */
/* c <= bound <= c + 2 when v = P(z), since s(M) >= N - 1 (the term at the     */
/* vertex k_lambda).  Points without a window report 0: z = 0 (P(0) = a_0,     */
/* so |P| >= M), P == 0, and a non-finite z.  v = 0 (every bit cancelled)      */
/* reports INT32_MAX.  N is the oracle's FP64 N of ora_eval.                   */
/* ------------------------------------------------------------------------- */
void ora_cancel_bound(const ora_plan *P, const double *z, const double *N, const double *m,
                      const int64_t *e, int64_t n, int32_t *out)
{
    for (int64_t j = 0; j < n; ++j) {
        const double zr = z[2 * j], zi = z[2 * j + 1];
        if (P->nh == 0 || !isfinite(zr) || !isfinite(zi) || (zr == 0.0 && zi == 0.0)) {
            out[j] = 0;
            continue;
        }
        const int64_t sv = ora_scale1(m[2 * j], m[2 * j + 1]);
        if (sv == ORA_NEG_INF) { out[j] = INT32_MAX; continue; }
        const int64_t c = (int64_t)floor(N[j]) + 1 - (sv + e[j]);
        out[j] = c > 0 ? (int32_t)(c < INT32_MAX ? c : INT32_MAX) : 0;
    }
}

/* ------------------------------------------------------------------------- */
/* Reverse mode of the evaluation with respect to the coefficients.          */
/* Q_lambda(z) (eq. reducedQlambda) is linear in a: its partial derivative    */
/* in a_k is z^k for the kept k (G_p within [l, r], held fixed) and 0         */
/* otherwise.  With upstream gradients g_j and the convention of complex      */
/* reverse mode (gradient = upstream gradient times the conjugate             */
/* derivative), grad_a[k] = sum over the points j keeping k of                */
/* g_j conj(z_j)^k, and its scale sum of |g_j| |z_j|^k over the same terms.    */
/* One thread: the points are summed in input order into double-double        */
/* accumulators with a separate exponent.                                     */
/* ------------------------------------------------------------------------- */
void ora_adjoint_coef(const ora_plan *P, const double *z, const double *g, int64_t n, int64_t d,
                      double *ga_m, int64_t *ga_e, double *sc_m, int64_t *sc_e)
{
    xc_t *acc = malloc(sizeof(xc_t) * (size_t)(d + 1));
    xr_t *sc = malloc(sizeof(xr_t) * (size_t)(d + 1));
    for (int64_t k = 0; k <= d; ++k) { acc[k] = xc_from(0.0, 0.0); sc[k] = (xr_t){ 0.0, 0 }; }
    for (int64_t j = 0; j < n; ++j) {
        double zr = z[2 * j], zi = z[2 * j + 1];
        ora_res o;
        ora_eval1(P, zr, zi, 0, &o);               /* the window [l, r] of this point */
        if (!isfinite(zr) || !isfinite(zi) || o.l > o.r) continue;
        xc_t gj = xc_from(g[2 * j], g[2 * j + 1]);
        double gabs = hypot(g[2 * j], g[2 * j + 1]);
        xc_t zc = xc_from(zr, -zi);                /* conj(z) */
        xc_t pw = xc_pow(zc, o.l);                 /* conj(z)^l, then one product per k */
        for (int64_t k = o.l; k <= o.r; ++k) {
            if (P->good[k]) {
                acc[k] = xc_add(acc[k], xc_mul(gj, pw));
                sc[k] = xr_add(sc[k], xr_norm((xr_t){ gabs * hypot(pw.re.hi, pw.im.hi), pw.e }));
            }
            if (k < o.r) pw = xc_mul(pw, zc);
        }
    }
    for (int64_t k = 0; k <= d; ++k) {
        xc_out(acc[k], ga_m + 2 * k, ga_e + k);
        sc_m[k] = sc[k].m; sc_e[k] = sc[k].e;
    }
    free(acc);
    free(sc);
}
