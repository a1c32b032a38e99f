// Internal declarations of the FPE library: plan layout, workspace layout and
// device helpers shared by the kernels.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fpe.h"

namespace fpe {

constexpr int kWave = 64;                 // CDNA wavefront width
constexpr int kHullLds = 512;             // cover vertices staged in LDS by the plan kernel
constexpr double kEta = 0x1p-20;          // widening of the window ends before ceil/floor
constexpr int kChunk = 512;               // default coefficient chunk length C of the window kernel
constexpr int kChunkMin = 256;            // shortest chunk an evaluation may use (sizes the fixed point)
constexpr int kChunkMax = 2048;
constexpr int32_t kNegInfScale = INT32_MIN;

// Device view of a preconditioned polynomial.  All pointers point into the
// caller's precondition workspace.
struct DevPlan {
    const double2 *coef;      // a_k for k in G_p, 0 elsewhere; k = 0 .. dt
    const int32_t *gprefix;   // gprefix[k] = #(G_p within [0, k)); k = 0 .. dt + 1
    const int32_t *gidx;      // G_p as a list: its indices in increasing order (|G_p| entries)
    const double2 *gcoef;     //   and their coefficients, as in coef
    const double *hull_k;     // cover vertices: abscissae k_i (exact in double)
    const double *hull_s;     // cover vertices: s(a_{k_i})
    int32_t nh;               // number of vertices; 0 when P == 0
    int32_t v, dt;            // first and last nonzero index
    int32_t T;                // threshold offset p + s(dt - v) + 3
    int32_t chunk;            // coefficient chunk length C of the window kernel
    int32_t fix_shift;        // scale of the fixed-point chunk accumulators (high word)
    int32_t fix_lo;           // extra bits of their low word
    int32_t coef_shift;       // coef holds a_k 2^-coef_shift (keeps window sums in range)
    double2 a0;               // a_0, returned at z = 0
    // FP32 window sums (FPE_PRECONDITION_FP32), else both NULL: coef32[k] =
    // coef[k] 2^-sig32[c] as FP32, c = k / chunk; sig32[c] = kNoFp32 where a
    // chunk's tiles stay in FP64
    const float2 *coef32;
    const int32_t *sig32;
    int32_t f32comp;          // FP32 blocks by the compensated recurrence (FPE_PRECONDITION_FP32_COMPENSATED)
};
constexpr int32_t kNoFp32 = INT32_MIN;

// What the window kernel needs of one point: z, its window [l, r] and its
// input index j (-1 for a batch's padding).  The sort moves these 32 bytes; the
// reference exponent eref (every kept term is below 2^eref in magnitude) stays
// in input order, read only for windows that span several chunks.
struct __align__(16) PointRec {
    double2 z;
    int32_t l, r;
    int32_t j, pad;
};

// Workspace of one evaluation of n points, carved from the caller's buffer.
struct EvalWs {
    int2 *lr;                     // per point, input order: its window [l, r] (l > r: finished)
    int32_t *keyrank;             // per point, input order: lambda bin x (points per sort block) + rank
    PointRec *srec;               // records sorted by lambda bin
    long long *eref;              // per point, input order: the reference exponent
    int32_t *table, *tscan;       // (sort block x bin) counts, and their bin-major scan
    int32_t *bin_sum, *bin_off;   // per table-scan segment (tab_ib bins)
    int32_t *glo, *ghi;           // per group of kWave sorted points: union window,
    int32_t *gml;                 //   largest window start,
    int32_t *gcost, *gcum;        //   work of its tiles and its prefix within its k_groups workgroup
    int4 *split;                  // groups owned by a few window wavefronts (ctl[8] of them): group,
                                  //   first and last owner
    int4 *lgroups;                // groups owned by many (ctl[9] of them): group, first and last owner,
    long long *lacc;              //   per such group 64 lanes x kSlotWords: the sum of its slots
    int32_t *lcnt;                //   and the pieces of its owners summed so far
    int32_t *gblk_sum, *gblk_pre; // per k_groups workgroup: total work and (many groups) its scan
    int32_t *gseg_sum, *gseg_off; //   per 4096-entry segment of that scan
    int2 *wstart;                 // per window wavefront: first tile (group, chunk); n_waves + 1
    long long *slots;             // per window wavefront, 2 x kSlotWords x 64 lanes: fixed-point partials
    int32_t *ctl;                 // [0] total tile work, [5] points in the count table, [8] [9] split groups
    int64_t n, n_groups, n_sort_blocks, n_waves;
    int32_t cost_shift;           // tile work is counted in units of (16 << cost_shift) steps
    int32_t tab_ib;               // bins per table-scan segment
    // a batch of polynomials (else NULL / -1): the plan of each group, and the
    // number of sorted slots (every polynomial's points padded to whole groups
    // with records that have no window)
    const DevPlan *plans;
    const int32_t *gpoly;
    int64_t n_slots;
    int32_t chunk;                // coefficient chunk length C of the tiles (a power of two)
    // sparse window sums (the list of G_p with gaps jumped by powers of z):
    // per group the share of its union window's Horner steps its tiles cost,
    // in 1/256 (256 for dense window sums)
    int32_t sparse;
    int32_t *gdens;
    // the reverse mode's exact accumulators of grad_a, one per coefficient
    // index up to dt (absent from a layout sized for the values alone)
    int32_t *aexp, *aflag;
    long long *aacc;
    int64_t n_acc;
};

// The reverse mode's accumulators, as kernel arguments: per coefficient index
// the exponent of the fixed-point scale, a non-finite flag, and four words
// (integer and fraction words of the real, then of the imaginary part).
struct AdjAcc {
    int32_t *aexp, *aflag;
    long long *acc;
};

// tight: the per-wavefront tables sized for this kind of tile kernel alone (by
// default one workspace serves every tile kernel)
size_t eval_workspace_bytes(const DevPlan &P, int64_t n, EvalWs *ws, void *base, int kind,
                            int64_t batch_groups = -1, int chunk = kChunk, bool tight = false);

// Read-only tables are read through the constant address space in device code:
// a wave-uniform index then becomes a scalar load, one per wavefront, broadcast
// to its 64 lanes.  (The host pass only parses kernel bodies.)
#if defined(__HIP_DEVICE_COMPILE__)
#define FPE_CONST_AS __attribute__((address_space(4)))
#else
#define FPE_CONST_AS
#endif
typedef const FPE_CONST_AS double *const_table_t;
typedef const FPE_CONST_AS float *const_table32_t;

// ---------------------------------------------------------------- device math
// The error-free transforms below (TwoSum, TwoProd through fma) rely on every
// product and sum being rounded separately: contracting a*b + c into one fma
// would silently drop the low words.  Explicit fma() calls are unaffected.
#define FPE_NO_CONTRACT _Pragma("clang fp contract(off)")

struct dd2 { double hi, lo; };

__host__ __device__ __forceinline__ dd2 two_sum(double a, double b) {
    FPE_NO_CONTRACT
    double s = a + b;
    double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

__host__ __device__ __forceinline__ dd2 fast_two_sum(double a, double b) {
    FPE_NO_CONTRACT
    double s = a + b;
    return {s, b - (s - a)};
}

// frexp-style exponent: x = f 2^k with |f| in [1/2, 1); x != 0 and finite
__host__ __device__ __forceinline__ int exp_of(double x) { return ilogb(x) + 1; }

// s(x + iy) exactly.  With a = max(|x|, |y|) = A 2^(m-53), b = min = B 2^(mb-53),
// A, B < 2^53 integers and m = exponent of a (so s(a) = m), s(z) = m + 1 iff
// x^2 + y^2 >= 4^m iff A^2 + B^2 4^(mb-m) >= 2^106.  The 106-bit squares are
// formed from 64-bit halves; the floor of the shifted smaller square cannot
// change the comparison because A^2 and 2^106 are integers.
__device__ __forceinline__ int32_t scale_exact(double x, double y) {
    double ax = fabs(x), ay = fabs(y);
    double a = fmax(ax, ay), b = fmin(ax, ay);
    if (a == 0.0) return kNegInfScale;
    int m = exp_of(a);
    unsigned long long A = (unsigned long long)ldexp(a, 53 - m);
    unsigned long long ahi = __umul64hi(A, A), alo = A * A;
    unsigned long long bhi = 0, blo = 0;
    if (b != 0.0) {
        int mb = exp_of(b);
        int sh = 2 * (m - mb);
        if (sh < 128) {
            unsigned long long B = (unsigned long long)ldexp(b, 53 - mb);
            unsigned long long h = __umul64hi(B, B), l = B * B;
            if (sh >= 64) { l = h >> (sh - 64); h = 0; }
            else if (sh > 0) { l = (l >> sh) | (h << (64 - sh)); h >>= sh; }
            bhi = h; blo = l;
        }
    }
    unsigned long long lo = alo + blo;
    unsigned long long hi = ahi + bhi + (lo < alo ? 1ull : 0ull);
    // 2^106 = bit 42 of the high word
    return (hi >= (1ull << 42)) ? m + 1 : m;
}

// complex double-double with a separate binary exponent
struct CDD { double rh, rl, ih, il; };

// Scales x by a power of two so that max(|Re|, |Im|) of its high words lies in
// [1/2, 1) and adds the power to E; the low words are folded into the high
// ones first (the products below leave them unnormalised).
__host__ __device__ __forceinline__ void cdd_renorm(CDD &x, long long &E) {
    FPE_NO_CONTRACT
    const dd2 r = two_sum(x.rh, x.rl), i = two_sum(x.ih, x.il);
    double m = fmax(fabs(r.hi), fabs(i.hi));
    int k = exp_of(m);
    x.rh = ldexp(r.hi, -k); x.rl = ldexp(r.lo, -k);
    x.ih = ldexp(i.hi, -k); x.il = ldexp(i.lo, -k);
    E += k;
}

// x^2 for a complex double-double x = (rh + rl) + i (ih + il).  The products
// of high words are split exactly (TwoProd through fma) and the real part's
// difference of squares by TwoSum; the cross terms with one low word are added
// to the low words, the products of two low words dropped.  The low words are
// left unnormalised: relative to |x|, each squaring at most doubles their size
// and adds 2^-51, so j squarings after a renormalisation they stay below
// 2^(j - 50) |x|, and the dropped terms below 2^(2 j - 100) |x|^2.
__host__ __device__ __forceinline__ CDD cdd_sqr(const CDD &x) {
    FPE_NO_CONTRACT
    const double rh2 = x.rh + x.rh;                  // exact
    double p1 = x.rh * x.rh;
    double e1 = fma(x.rh, x.rh, -p1);
    e1 = fma(rh2, x.rl, e1);
    double p2 = x.ih * x.ih;
    double e2 = fma(x.ih, x.ih, -p2);
    e2 = fma(x.ih + x.ih, x.il, e2);
    dd2 s = two_sum(p1, -p2);
    // 2 rh ih: (2 rh) ih, and 2 (rh il + rl ih)
    double q = rh2 * x.ih;
    double eq = fma(rh2, x.ih, -q);
    eq = fma(rh2, x.il, eq);
    eq = fma(x.rl + x.rl, x.ih, eq);
    return {s.hi, s.lo + (e1 - e2), q, eq};
}

// x * w for a complex double-double x and a complex double w (low words as in
// cdd_sqr: the product by w, |w| < 2^(1/2), leaves their size relative to |x|)
__host__ __device__ __forceinline__ CDD cdd_mul_d(const CDD &x, double wr, double wi) {
    FPE_NO_CONTRACT
    double p1 = x.rh * wr, e1 = fma(x.rh, wr, -p1);
    e1 = fma(x.rl, wr, e1);
    double p2 = x.ih * wi, e2 = fma(x.ih, wi, -p2);
    e2 = fma(x.il, wi, e2);
    dd2 s = two_sum(p1, -p2);
    double p3 = x.rh * wi, e3 = fma(x.rh, wi, -p3);
    e3 = fma(x.rl, wi, e3);
    double p4 = x.ih * wr, e4 = fma(x.ih, wr, -p4);
    e4 = fma(x.il, wr, e4);
    dd2 t = two_sum(p3, p4);
    return {s.hi, s.lo + (e1 - e2), t.hi, t.lo + (e3 + e4)};
}

// w^n (n >= 0) for |Re w|, |Im w| < 1 with max in [1/2, 1): left-to-right binary
// powering in double-double, renormalised every fourth bit and after the last
// (from a renormalised value, whose modulus is in [1/2, 2^(1/2)), four
// squarings with products by w keep the modulus within [2^-31, 2^8], far from
// the FP64 range limits).  Returns the renormalised, rounded mantissa and adds
// the binary exponent to E.  Each squaring drops at most 2^-92 |x|^2 (four
// squarings after a renormalisation) and later squarings double a relative
// error, so after k squarings the relative error is below 2^(k - 92) before
// the final rounding: below 2^-62 for n < 2^31.
__host__ __device__ __forceinline__ void cpow_dd(double wr, double wi, int n, double &pr, double &pi,
                                        long long &E) {
    if (n == 0) { pr = 1.0; pi = 0.0; return; }
    CDD x = {wr, 0.0, wi, 0.0};
    long long ex = 0;                 // x stands for (its mantissa) 2^ex
    int top = 31 - __builtin_clz((unsigned)n);
    for (int b = top - 1; b >= 0; --b) {
        x = cdd_sqr(x);
        ex *= 2;                      // squaring doubles the exponent
        if ((n >> b) & 1) x = cdd_mul_d(x, wr, wi);
        if ((b & 3) == 0) cdd_renorm(x, ex);
    }
    E += ex;
    pr = x.rh + x.rl;
    pi = x.ih + x.il;
}

// x <- x y for complex doubles x = (xr + i xi) 2^xe and y = (yr + i yi) 2^ye,
// both with max(|re|, |im|) in [1/2, 1), renormalised the same way; about two
// roundings per component.
__host__ __device__ __forceinline__ void cmul_renorm(double &xr, double &xi, long long &xe, double yr, double yi,
                                                     long long ye) {
    FPE_NO_CONTRACT
    const double r = fma(xr, yr, -(xi * yi));
    const double i = fma(xr, yi, xi * yr);
    const int k = exp_of(fmax(fabs(r), fabs(i)));
    xr = ldexp(r, -k);
    xi = ldexp(i, -k);
    xe += ye + k;
}

// w^(c C) by a fixed recipe, so that every caller gets the same bits: the
// anchor w^(m C), m = c - c mod kAnchor, by cpow_dd, then (c mod kAnchor)
// products by w^C (itself from cpow_dd), each rounded to double.  Relative
// error below (3 kAnchor) 2^-53.
constexpr int kAnchor = 8;

__host__ __device__ __forceinline__ void cpow_chunk_start(double wr, double wi, int c, int C, double zcr, double zci,
                                                          long long zce, double &xr, double &xi, long long &xe) {
    const int m = c - c % kAnchor;
    xe = 0;
    cpow_dd(wr, wi, m * C, xr, xi, xe);
    for (int j = m; j < c; ++j) cmul_renorm(xr, xi, xe, zcr, zci, zce);
}

}  // namespace fpe

// Host-side plan handle (the ABI's opaque fpe_plan_s).
struct fpe_plan_s {
    fpe::DevPlan dev;
    int64_t d, v, dt, nh, ngood, T, p, smax, smin_good;
    const int32_t *good_dev = nullptr;   // d + 1 flags of G_p, in the plan's workspace
    int device;
    int32_t chunk_sel = 0;           // chunk length chosen by fpe_autotune or set; 0: cached choice or default
    int32_t mode_sel = 0;            // window-sum form chosen or set (FPE_WINDOW_*); 0: cached choice or default
    int32_t adjoint_mode = 0;        // FPE_ADJOINT_EXACT (0) or FPE_ADJOINT_ATOMIC
};

namespace fpe {
void set_error(const std::string &msg);
fpe_status fail(fpe_status s, const std::string &msg);
fpe_status hip_fail(hipError_t e, const char *what);
}  // namespace fpe

#define FPE_HIP_CHECK(call)                                                 \
    do {                                                                    \
        hipError_t _e = (call);                                             \
        if (_e != hipSuccess) return ::fpe::hip_fail(_e, #call);            \
    } while (0)
