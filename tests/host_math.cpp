// Host build of the library's double-double helpers (the kernels call the same
// inline functions), exported for tests/test_host_math.py.
#include "../paper_2211_06320_amd/csrc/fpe_internal.h"

extern "C" void hm_cpow(double wr, double wi, int n, double *pr, double *pi, long long *E) {
    long long e = 0;
    fpe::cpow_dd(wr, wi, n, *pr, *pi, e);
    *E = e;
}

// one complex double-double square or product by a complex double, unrounded
extern "C" void hm_cdd_sqr(const double *x, double *out) {
    const fpe::CDD r = fpe::cdd_sqr({x[0], x[1], x[2], x[3]});
    out[0] = r.rh; out[1] = r.rl; out[2] = r.ih; out[3] = r.il;
}

extern "C" void hm_cdd_mul_d(const double *x, double wr, double wi, double *out) {
    const fpe::CDD r = fpe::cdd_mul_d({x[0], x[1], x[2], x[3]}, wr, wi);
    out[0] = r.rh; out[1] = r.rl; out[2] = r.ih; out[3] = r.il;
}

// w^(c C) by the chained recipe of the window kernel
extern "C" void hm_chunk_start(double wr, double wi, int c, int C, double *pr, double *pi, long long *E) {
    double zcr, zci;
    long long zce = 0;
    fpe::cpow_dd(wr, wi, C, zcr, zci, zce);
    long long e = 0;
    fpe::cpow_chunk_start(wr, wi, c, C, zcr, zci, zce, *pr, *pi, e);
    *E = e;
}

// the renormalisation: low words folded into the high ones, then a power-of-two scaling
extern "C" void hm_cdd_renorm(const double *x, double *out, long long *E) {
    fpe::CDD r = {x[0], x[1], x[2], x[3]};
    long long e = 0;
    fpe::cdd_renorm(r, e);
    out[0] = r.rh; out[1] = r.rl; out[2] = r.ih; out[3] = r.il;
    *E = e;
}
