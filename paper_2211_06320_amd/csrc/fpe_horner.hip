// Same-GPU baseline: Horner's rule on the full polynomial, one lane per point.
//
// Every lane runs h <- h z + a_k for k = d .. 0; the coefficient index is
// wave-uniform, so each coefficient is one scalar load shared by the wavefront.
// |P(z)| leaves the FP64 range for many points at large d, so the running value
// is rescaled by an exact power of two whenever it grows past 2^400; later
// coefficients are multiplied by the same factor (they underflow harmlessly
// once the running value dwarfs them).  The check runs every 4 steps, which is
// safe while |z| < 2^150; the rare lanes with a larger |z| take a slow path that
// renormalises after every step.
#include "fpe_internal.h"

namespace fpe {
namespace {

__device__ __forceinline__ void normalise_out(double re, double im, long long E, double2 &m, long long &e) {
    double mx = fmax(fabs(re), fabs(im));
    if (mx == 0.0) { m = make_double2(0.0, 0.0); e = 0; return; }
    int k = exp_of(mx);
    m = make_double2(ldexp(re, -k), ldexp(im, -k));
    e = E + k;
}

// Horner with a renormalisation after every step: h = (hr + i hi) 2^E.
__device__ void horner_slow(const double2 *__restrict__ cf, int d, double zr, double zi,
                            double &hr, double &hi, long long &E) {
    const int ez = exp_of(fmax(fabs(zr), fabs(zi)));
    const double wr = ldexp(zr, -ez), wi = ldexp(zi, -ez);
    hr = 0.0; hi = 0.0; E = 0;
    for (int k = d; k >= 0; --k) {
        // h z = (h w) 2^(E + ez)
        double pr = fma(hr, wr, -hi * wi), pi = fma(hr, wi, hi * wr);
        long long Ep = E + ez;
        double2 a = cf[k];
        double ma = fmax(fabs(a.x), fabs(a.y)), mp = fmax(fabs(pr), fabs(pi));
        long long ea = ma > 0.0 ? exp_of(ma) : LLONG_MIN / 4;
        long long ep = mp > 0.0 ? Ep + exp_of(mp) : LLONG_MIN / 4;
        long long Et = ea > ep ? ea : ep;          // exponent of the larger term
        if (Et == LLONG_MIN / 4) { hr = 0.0; hi = 0.0; E = 0; continue; }
        long long sp = Ep - Et, sa = -Et;
        sp = sp < -2200 ? -2200 : sp;
        sa = sa < -2200 ? -2200 : (sa > 2200 ? 2200 : sa);
        hr = ldexp(pr, (int)sp) + ldexp(a.x, (int)sa);
        hi = ldexp(pi, (int)sp) + ldexp(a.y, (int)sa);
        E = Et;
    }
}

__global__ __launch_bounds__(256) void k_horner(const double2 *__restrict__ cf, int d,
                                                const double2 *__restrict__ z, int n,
                                                double2 *__restrict__ m_out, long long *__restrict__ e_out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = j < n;
    double2 zz = in ? z[j] : make_double2(0.0, 0.0);
    const bool bad = !isfinite(zz.x) || !isfinite(zz.y);
    const bool huge = !bad && fmax(fabs(zz.x), fabs(zz.y)) > 0x1p150;
    const double zr = (bad || huge) ? 0.0 : zz.x, zi = (bad || huge) ? 0.0 : zz.y;
    double hr = 0.0, hi = 0.0, sig = 1.0;
    long long E = 0;
    int k = d;
    for (; k >= 3; k -= 4) {
        double2 a0 = cf[k], a1 = cf[k - 1], a2 = cf[k - 2], a3 = cf[k - 3];
#define HB(A)                                                           \
        {                                                               \
            double nr = fma(hr, zr, fma(-hi, zi, (A).x * sig));        \
            double ni = fma(hr, zi, fma(hi, zr, (A).y * sig));         \
            hr = nr; hi = ni;                                           \
        }
        HB(a0) HB(a1) HB(a2) HB(a3)
        if (fmax(fabs(hr), fabs(hi)) > 0x1p400) {
            hr = ldexp(hr, -400); hi = ldexp(hi, -400);
            sig = ldexp(sig, -400);
            E += 400;
        }
    }
    for (; k >= 0; --k) { double2 a = cf[k]; HB(a) }
#undef HB
    if (!in) return;
    if (huge) horner_slow(cf, d, zz.x, zz.y, hr, hi, E);
    double2 m;
    long long e;
    if (bad) { m = make_double2(__builtin_nan(""), __builtin_nan("")); e = 0; }
    else normalise_out(hr, hi, E, m, e);
    m_out[j] = m;
    e_out[j] = e;
}

}  // namespace
}  // namespace fpe

using namespace fpe;

extern "C" fpe_status fpe_horner_eval(const double *coef_dev, int64_t d, const double *z_dev, int64_t n,
                                      double *m_dev, int64_t *e_dev, hipStream_t stream) {
    if (d < 0 || d >= INT32_MAX - 2 || n < 0 || n >= INT32_MAX) return fail(FPE_ERR_INVALID_ARG, "size out of range");
    if (n == 0) { set_error(""); return FPE_OK; }
    if (!coef_dev || !z_dev || !m_dev || !e_dev) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(coef_dev) % 16 != 0 || reinterpret_cast<uintptr_t>(z_dev) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(m_dev) % 16 != 0)
        return fail(FPE_ERR_INVALID_ARG, "misaligned buffer");
    const unsigned blocks = (unsigned)((n + 255) / 256);
    k_horner<<<blocks, 256, 0, stream>>>(reinterpret_cast<const double2 *>(coef_dev), (int)d,
                                         reinterpret_cast<const double2 *>(z_dev), (int)n,
                                         reinterpret_cast<double2 *>(m_dev), reinterpret_cast<long long *>(e_dev));
    FPE_HIP_CHECK(hipGetLastError());
    set_error("");
    return FPE_OK;
}
