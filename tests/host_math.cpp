// Host build of the library's double-double helpers (the kernels call the same
// inline functions), exported for tests/test_host_math.py.
#include "../paper_2211_06320_amd/csrc/fpe_internal.h"

extern "C" void hm_cpow(double wr, double wi, int n, double *pr, double *pi, long long *E) {
    long long e = 0;
    fpe::cpow_dd(wr, wi, n, *pr, *pi, e);
    *E = e;
}
