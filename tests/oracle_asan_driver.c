/* Runs every entry point of the oracle (oracle/fpe_oracle.c, compiled into this
 * program) on small seeded inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host.  Test infrastructure only; prints one
 * line per case and "ok" at the end. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct ora_plan ora_plan;
int64_t ora_scale1(double x, double y);
ora_plan *ora_precondition(const double *coef, int64_t d, int32_t p);
ora_plan *ora_precondition_offset(const double *coef, int64_t d, int64_t T);
void ora_plan_free(ora_plan *P);
void ora_plan_info(const ora_plan *P, int64_t *out);
void ora_plan_hull(const ora_plan *P, int64_t *hk, int64_t *hs);
void ora_plan_good(const ora_plan *P, uint8_t *good);
void ora_plan_scales(const ora_plan *P, int64_t *s);
void ora_eval(const ora_plan *P, const double *z, int64_t n, double *m, int64_t *e, int64_t *l, int64_t *r,
              int64_t *terms, double *dwin_m, int64_t *dwin_e, double *lambda, double *N, int nthreads);
void ora_eval_deriv(const ora_plan *P, const double *z, int64_t n, double *m, int64_t *e, double *dwin_m,
                    int64_t *dwin_e, double *md, int64_t *de, double *ddm, int64_t *dde, int nthreads);
void ora_eval_fp64(const ora_plan *P, const double *z, int64_t n, double *m, int64_t *e, int nthreads);
void ora_level_sets(const ora_plan *P, const double *lam, const double *dlev, int64_t n, double *N, double *xL,
                    double *xR);
void ora_horner(const double *coef, int64_t d, const double *z, int64_t n, double *m, int64_t *e, int nthreads);
void ora_absum(const double *coef, int64_t d, const double *z, int64_t n, double *dm, int64_t *de, int nthreads);
void ora_cancel_bound(const ora_plan *P, const double *z, const double *N, const double *m, const int64_t *e,
                      int64_t n, int32_t *out);
void ora_adjoint_coef(const ora_plan *P, const double *z, const double *g, int64_t n, int64_t d, double *ga_m,
                      int64_t *ga_e, double *sc_m, int64_t *sc_e);

static uint64_t rng_state = 88172645463325252ull;
static double urand(void) /* xorshift64, uniform in [0, 1) */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * 0x1p-53;
}

static void run_case(const double *c, int64_t d, int32_t p, int nthreads)
{
    enum { NZ = 97 };
    double z[2 * NZ], g[2 * NZ];
    for (int j = 0; j < NZ; ++j) {
        double r = ldexp(1.0, (int)(urand() * 8) - 4) * (0.5 + urand()), t = 6.283185307179586 * urand();
        z[2 * j] = r * cos(t);
        z[2 * j + 1] = r * sin(t);
        g[2 * j] = urand() - 0.5;
        g[2 * j + 1] = urand() - 0.5;
    }
    z[0] = z[1] = 0.0;                 /* z = 0 */
    z[2] = NAN;                        /* a non-finite point */
    z[4] = 1.0; z[5] = 0.0;
    ora_plan *P = ora_precondition(c, d, p);
    int64_t info[7];
    ora_plan_info(P, info);
    int64_t *hk = malloc(sizeof(int64_t) * (size_t)(info[3] + 1)), *hs = malloc(sizeof(int64_t) * (size_t)(info[3] + 1));
    ora_plan_hull(P, hk, hs);
    uint8_t *good = malloc((size_t)d + 1);
    ora_plan_good(P, good);
    int64_t *sc = malloc(sizeof(int64_t) * (size_t)(d + 1));
    ora_plan_scales(P, sc);
    double m[2 * NZ], dm[NZ], lam[NZ], N[NZ], md[2 * NZ], ddm[NZ], xl[NZ], xr[NZ], N2[NZ];
    int64_t e[NZ], l[NZ], r[NZ], t[NZ], de[NZ], ed[NZ], dde[NZ];
    int32_t bits[NZ];
    ora_eval(P, z, NZ, m, e, l, r, t, dm, de, lam, N, nthreads);
    ora_eval_deriv(P, z, NZ, m, e, dm, de, md, ed, ddm, dde, nthreads);
    ora_eval_fp64(P, z, NZ, m, e, nthreads);
    ora_level_sets(P, lam, NULL, NZ, N2, xl, xr);
    ora_level_sets(P, lam, ddm, NZ, N2, xl, xr);
    ora_cancel_bound(P, z, N, m, e, NZ, bits);
    double *ga = malloc(sizeof(double) * 2 * (size_t)(d + 1)), *gs = malloc(sizeof(double) * (size_t)(d + 1));
    int64_t *gae = malloc(sizeof(int64_t) * (size_t)(d + 1)), *gse = malloc(sizeof(int64_t) * (size_t)(d + 1));
    ora_adjoint_coef(P, z, g, NZ, d, ga, gae, gs, gse);
    ora_horner(c, d, z, NZ, m, e, nthreads);
    ora_absum(c, d, z, NZ, dm, de, nthreads);
    ora_plan_free(P);
    P = ora_precondition_offset(c, d, 6);
    ora_eval(P, z, NZ, m, e, l, r, t, dm, de, lam, N, 1);
    ora_plan_free(P);
    printf("d=%lld p=%d vertices=%lld good=%lld\n", (long long)d, p, (long long)info[3], (long long)info[4]);
    free(hk); free(hs); free(good); free(sc); free(ga); free(gs); free(gae); free(gse);
}

int main(void)
{
    for (int it = 0; it < 24; ++it) {
        int64_t d = it < 4 ? it : (int64_t)(urand() * 3000);
        double *c = malloc(sizeof(double) * 2 * (size_t)(d + 1));
        for (int64_t k = 0; k <= d; ++k) {
            double s = ldexp(1.0, it % 3 == 0 ? 0 : (int)(urand() * 200) - 100);
            c[2 * k] = s * (urand() - 0.5);
            c[2 * k + 1] = s * (urand() - 0.5);
            if (it % 4 == 1 && urand() < 0.6) c[2 * k] = c[2 * k + 1] = 0.0;
        }
        if (it == 2) for (int64_t k = 0; k <= d; ++k) c[2 * k] = c[2 * k + 1] = 0.0;   /* P == 0 */
        run_case(c, d, it % 2 ? 24 : 53, 1 + it % 3);
        free(c);
    }
    printf("ok\n");
    return 0;
}
