// Preconditioning (Algorithm A_p, first block; Section 5.1 of arXiv 2211.06320),
// on the GPU, with one host synchronisation at the end.  Its two parts are
// split as Remark partialpreproc (Section 5.1) allows: the concave cover does
// not depend on p, only the good set G_p does.
//
// The cover (fpe_cover_build, or the first part of fpe_precondition):
//   k_pre_init    the candidate table and the counters
//   k_pre_scale   s(a_k) = 1 + floor(log2|a_k|) of every coefficient (Section 2.3,
//                 eq. dsz), decided exactly with 64-bit integer arithmetic on the
//                 significands; per value of s, the least and the largest index
//                 holding it.  Only those can be vertices of the concave cover:
//                 the points of one height between them lie on a level segment.
//   k_pre_hull    one workgroup: the candidates sorted by index (bitonic sort in
//                 LDS), the cover by Andrew's monotone chain (the same function
//                 as the paper's sorted incremental construction)
// The good set and the tables for a precision p (fpe_plan_from_cover, or the
// second part of fpe_precondition):
//   k_plan_init   the plan's counters
//   k_pre_good    T = p + s(d') + 3; G_p = { k : s(a_k) >= Ehat(k) - T } (eq.
//                 threshold) in exact integer arithmetic, counted per workgroup,
//                 and the least good s; the plan's copy of the cover
//   k_pre_scan    the workgroups' offsets, |G_p|, the shift of the table
//   k_pre_table   prefix counts of G_p, the masked, shifted coefficient table and
//                 G_p as a list
//   k_pre_sig32   (FP32 plans) per chunk, the scale of the FP32 table
//   k_mask32      (FP32 plans) the FP32 table
// Polynomials of at most kFusedMax coefficients (alone, or many at once in
// fpe_precondition_batched) take k_pre_fused instead: one workgroup per
// polynomial runs every step above in turn, with the candidates, their sort and
// the cover in LDS.  Both forms compute the same plan bit for bit: the cover is
// the unique upper concave majorant of distinct candidate indices, and every
// later quantity is exact integer arithmetic or the same FP64 operations.
#include <algorithm>
#include <climits>
#include <cstring>
#include <memory>

#include "fpe_internal.h"

namespace fpe {
namespace {

constexpr size_t kAlign = 256;
constexpr int kSOff = 1080;                 // table index of a scale: s + kSOff
constexpr int kSBins = 2112;                // covers s in [-1074, 1025], every finite nonzero double
constexpr int kMaxCand = 2 * kSBins;        // candidates (and cover vertices) at most
constexpr int kSortCap = 8192;              // the candidate sort pads to a power of two
constexpr int kPreThreads = 1024;
constexpr int kPrePer = 8;                  // coefficients per thread in the per-coefficient kernels
constexpr int kPreBlock = kPreThreads * kPrePer;

// counters and results read back by the host (int64)
enum Info {
    kNonFinite = 0, kV, kDt, kNh, kNGood, kT, kSMax, kSMinGood, kShift, kUnsupported,
    kA0Re, kA0Im,              // a_0 (its bits), returned at z = 0
    kInfoLen = 16
};

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// The cover of one polynomial (p-independent): its vertices, the counters
// kNonFinite, kV, kDt, kNh, kSMax of info, and the candidate table.
struct CoverWs {
    double *hull_k;    // cover vertices (at most hull_cap)
    double *hull_s;
    long long *info;   // kInfoLen
    int32_t *cmin;     // kSBins: least index of each scale (INT_MAX: none)
    int32_t *cmax;     // kSBins: largest index of each scale
};

// A plan's tables (the plan's workspace).
struct PlanWs {
    int32_t *good;     // d + 1: k in G_p
    double2 *coef;     // d + 1: a_k 2^-shift for k in G_p, else 0
    int32_t *gprefix;  // d + 2
    int32_t *gidx;     // |G_p| <= d + 1: the indices of G_p in increasing order
    double2 *gcoef;    //   and their coefficients a_k 2^-shift (the sparse window sum's list)
    double *hull_k;    // the plan's copy of the cover vertices
    double *hull_s;
    long long *info;   // kInfoLen
    int32_t *ictl;     // [0] least good s
    int32_t *blk_sum;  // per kPreBlock coefficients: |G_p| there
    int32_t *blk_off;  //   and its exclusive prefix
    float2 *coef32;    // d + 1 (FP32 plans): coef 2^-sig32[chunk] as FP32
    int32_t *sig32;    // chunks (FP32 plans)
};

__host__ __device__ int64_t n_chunks(int64_t d) { return d / kChunk + 1; }
int64_t n_blocks(int64_t n1) { return (n1 + kPreBlock - 1) / kPreBlock; }
int64_t hull_cap(int64_t n1) { return std::min<int64_t>(n1, kMaxCand); }

template <class Take>
PlanWs plan_layout(int64_t d, uint32_t pflags, Take &&take) {
    const int64_t n1 = d + 1, nb = n_blocks(n1);
    PlanWs x;
    x.good = (int32_t *)take(sizeof(int32_t) * n1);
    x.coef = (double2 *)take(sizeof(double2) * n1);
    x.gprefix = (int32_t *)take(sizeof(int32_t) * (n1 + 1));
    x.gidx = (int32_t *)take(sizeof(int32_t) * n1);
    x.gcoef = (double2 *)take(sizeof(double2) * n1);
    x.hull_k = (double *)take(sizeof(double) * hull_cap(n1));
    x.hull_s = (double *)take(sizeof(double) * hull_cap(n1));
    x.info = (long long *)take(sizeof(long long) * kInfoLen);
    x.ictl = (int32_t *)take(sizeof(int32_t) * 16);
    x.blk_sum = (int32_t *)take(sizeof(int32_t) * nb);
    x.blk_off = (int32_t *)take(sizeof(int32_t) * nb);
    x.coef32 = nullptr;
    x.sig32 = nullptr;
    if (pflags & FPE_PRECONDITION_FP32) {
        x.coef32 = (float2 *)take(sizeof(float2) * n1);
        x.sig32 = (int32_t *)take(sizeof(int32_t) * n_chunks(d));
    }
    return x;
}

// the candidate table and counters of a cover; with own_hull, its vertices too
template <class Take>
CoverWs cover_layout(int64_t d, bool own_hull, Take &&take) {
    const int64_t n1 = d + 1;
    CoverWs c;
    c.hull_k = own_hull ? (double *)take(sizeof(double) * hull_cap(n1)) : nullptr;
    c.hull_s = own_hull ? (double *)take(sizeof(double) * hull_cap(n1)) : nullptr;
    c.info = (long long *)take(sizeof(long long) * kInfoLen);
    c.cmin = (int32_t *)take(sizeof(int32_t) * kSBins);
    c.cmax = (int32_t *)take(sizeof(int32_t) * kSBins);
    return c;
}

struct Carver {
    char *b;
    size_t off = 0;
    void *operator()(size_t bytes) { char *p = b ? b + off : nullptr; off = align_up(off + bytes); return p; }
};

// fpe_precondition's workspace: a plan and the scratch of its cover, whose
// vertices are the plan's own
size_t pre_layout(int64_t d, uint32_t pflags, PlanWs *w, CoverWs *c, void *base) {
    Carver take{static_cast<char *>(base)};
    PlanWs x = plan_layout(d, pflags, take);
    CoverWs y = cover_layout(d, false, take);
    y.hull_k = x.hull_k;
    y.hull_s = x.hull_s;
    if (w) *w = x;
    if (c) *c = y;
    return take.off;
}

__device__ __forceinline__ int64_t bitlen_d(int64_t v) {
    int64_t b = 0;
    while (v > 0) { ++b; v >>= 1; }
    return b;
}

__global__ __launch_bounds__(256) void k_pre_init(CoverWs W) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < kSBins) { W.cmin[i] = INT_MAX; W.cmax[i] = INT_MIN; }
    if (i < kInfoLen) W.info[i] = 0;
}

__global__ __launch_bounds__(64) void k_plan_init(PlanWs W) {
    const int i = threadIdx.x;
    if (i < kInfoLen) W.info[i] = 0;
    if (i < 16) W.ictl[i] = i == 0 ? INT_MAX : 0;
}

__global__ __launch_bounds__(kPreThreads) void k_pre_scale(const double2 *__restrict__ coef, int64_t n1, CoverWs W) {
    __shared__ int32_t lmin[kSBins], lmax[kSBins];
    const int t = threadIdx.x;
    for (int i = t; i < kSBins; i += kPreThreads) { lmin[i] = INT_MAX; lmax[i] = INT_MIN; }
    __syncthreads();
    bool bad = false;
    for (int q = 0; q < kPrePer; ++q) {
        const int64_t k = (int64_t)blockIdx.x * kPreBlock + (int64_t)q * kPreThreads + t;
        if (k >= n1) break;
        const double2 a = coef[k];
        int32_t s = kNegInfScale;
        if (!isfinite(a.x) || !isfinite(a.y)) bad = true;
        else s = scale_exact(a.x, a.y);
        if (s != kNegInfScale) {
            atomicMin(&lmin[s + kSOff], (int32_t)k);
            atomicMax(&lmax[s + kSOff], (int32_t)k);
        }
    }
    if (__any(bad) && (t % kWave) == 0) atomicOr((unsigned long long *)&W.info[kNonFinite], 1ull);
    __syncthreads();
    for (int i = t; i < kSBins; i += kPreThreads) {
        if (lmin[i] != INT_MAX) {
            atomicMin(&W.cmin[i], lmin[i]);
            atomicMax(&W.cmax[i], lmax[i]);
        }
    }
}

// The candidates (index, scale) sorted by index, then the upper concave cover
// by the monotone chain, scanning the indices upwards and popping the last
// vertex while the turn it makes is not strictly clockwise (collinear vertices
// are dropped).  The chain runs in place: its stack occupies a prefix of the
// sorted candidates.
// The monotone chain over n candidates (ck: index, cb: scale + kSOff) sorted
// by index, in place; returns the number of vertices and sets smax, the
// largest candidate scale.  One thread.
__device__ int monotone_chain(int32_t *ck, int16_t *cb, int n, int &smax) {
    int h = 0;
    smax = INT_MIN;
    for (int i = 0; i < n; ++i) {
        const int64_t k = ck[i], s = (int64_t)cb[i] - kSOff;
        smax = max(smax, (int)s);
        while (h >= 2) {
            const int64_t ax = ck[h - 2], ay = (int64_t)cb[h - 2] - kSOff;
            const int64_t bx = ck[h - 1], by = (int64_t)cb[h - 1] - kSOff;
            const int64_t cross = (bx - ax) * (s - ay) - (by - ay) * (k - ax);
            if (cross >= 0) --h; else break;
        }
        ck[h] = (int32_t)k;
        cb[h] = (int16_t)(s + kSOff);
        ++h;
    }
    return h;
}

// bitonic sort of np2 (a power of two) entries of ck (keys) and cb, by the
// whole workgroup of kPreThreads threads
__device__ void bitonic_sort(int32_t *ck, int16_t *cb, int np2) {
    const int t = threadIdx.x;
    for (int k = 2; k <= np2; k <<= 1) {
        for (int h = k >> 1; h > 0; h >>= 1) {
            for (int i = t; i < np2; i += kPreThreads) {
                const int o = i ^ h;
                if (o > i) {
                    const int32_t a = ck[i], b = ck[o];
                    if ((a > b) == ((i & k) == 0)) {
                        ck[i] = b; ck[o] = a;
                        const int16_t x = cb[i]; cb[i] = cb[o]; cb[o] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kPreThreads) void k_pre_hull(CoverWs W) {
    __shared__ int32_t ck[kSortCap];
    __shared__ int16_t cb[kSortCap];
    __shared__ int32_t cnt;
    const int t = threadIdx.x;
    if (t == 0) cnt = 0;
    __syncthreads();
    for (int b = t; b < kSBins; b += kPreThreads) {
        const int32_t lo = W.cmin[b];
        if (lo != INT_MAX) {
            const int32_t hi = W.cmax[b];
            const int i = atomicAdd(&cnt, hi != lo ? 2 : 1);
            ck[i] = lo;
            cb[i] = (int16_t)b;
            if (hi != lo) { ck[i + 1] = hi; cb[i + 1] = (int16_t)b; }
        }
    }
    __syncthreads();
    const int n = cnt;
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (int i = n + t; i < np2; i += kPreThreads) { ck[i] = INT_MAX; cb[i] = 0; }
    __syncthreads();
    bitonic_sort(ck, cb, np2);
    if (t == 0) {
        int smax = INT_MIN;
        const int h = monotone_chain(ck, cb, n, smax);
        if (n > 0) {
            W.info[kV] = ck[0];
            W.info[kDt] = ck[h - 1];
            W.info[kNh] = h;
            W.info[kSMax] = smax;
        } else {
            W.info[kV] = -1;
            W.info[kDt] = -1;
            W.info[kNh] = 0;
        }
        cnt = h;
    }
    __syncthreads();
    for (int i = t; i < cnt; i += kPreThreads) {
        W.hull_k[i] = (double)ck[i];
        W.hull_s[i] = (double)((int)cb[i] - kSOff);
    }
}

// the cover segment [k_i, k_{i+1}] holding k (vertices in increasing index; nh >= 2)
__device__ __forceinline__ int cover_segment(const double *hk, int nh, double k) {
    int lo = 0, hi = nh - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (hk[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// T = p + s(d') + 3 for the cover's trimmed degree d' - v (eq. threshold)
__device__ __forceinline__ int64_t threshold_T(int32_t p_bits, const long long *cinfo) {
    const int64_t deff = cinfo[kDt] - cinfo[kV];
    return p_bits + bitlen_d(deff > 1 ? deff : 1) + 3;
}

// k in G_p: s >= Ehat(k) - T with Ehat(k) = s0 + (s1 - s0)(k - k0)/(k1 - k0) on
// the cover segment [k0, k1] holding k, decided in exact integer arithmetic
template <class HK, class HS>
__device__ __forceinline__ int is_good(int32_t s, int64_t k, HK hk, HS hs, int nh, int64_t T) {
    if (s == kNegInfScale || nh == 0) return 0;
    if (nh == 1) return 1;
    int lo = 0, hi = nh - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)hk[mid] <= k) lo = mid; else hi = mid - 1;
    }
    const int64_t k0 = (int64_t)hk[lo], k1 = (int64_t)hk[lo + 1];
    const int64_t s0 = (int64_t)hs[lo], s1 = (int64_t)hs[lo + 1];
    return ((int64_t)s + T - s0) * (k1 - k0) >= (s1 - s0) * (k - k0) ? 1 : 0;
}

// s(a_k), kNegInfScale for a_k = 0 (and for a non-finite a_k, which fails the
// plan; it then only has to stay harmless)
__device__ __forceinline__ int32_t coef_scale(const double2 *__restrict__ coef, int64_t k) {
    const double2 a = coef[k];
    if (!isfinite(a.x) || !isfinite(a.y)) return kNegInfScale;
    return scale_exact(a.x, a.y);
}

// G_p flags and counts per workgroup; workgroup 0 also writes the plan's copy
// of the cover (when the plan does not share the cover's vertices) and its
// counters
__global__ __launch_bounds__(kPreThreads) void k_pre_good(const double2 *__restrict__ coef, int64_t n1, CoverWs C,
                                                          PlanWs W, int32_t p_bits) {
    __shared__ double s_k[kHullLds], s_s[kHullLds];
    __shared__ int32_t s_cnt[kPreThreads / kWave], s_min[kPreThreads / kWave];
    const int t = threadIdx.x;
    const int nh = (int)C.info[kNh];
    const int64_t T = nh > 0 ? threshold_T(p_bits, C.info) : 0;
    if (blockIdx.x == 0) {
        if (W.hull_k != C.hull_k)
            for (int i = t; i < nh; i += kPreThreads) { W.hull_k[i] = C.hull_k[i]; W.hull_s[i] = C.hull_s[i]; }
        if (t == 0) {
            for (int i : {(int)kNonFinite, (int)kV, (int)kDt, (int)kNh, (int)kSMax}) W.info[i] = C.info[i];
            W.info[kT] = T;
            W.info[kA0Re] = __double_as_longlong(coef[0].x);
            W.info[kA0Im] = __double_as_longlong(coef[0].y);
        }
    }
    const bool in_lds = nh <= kHullLds;
    if (in_lds)
        for (int i = t; i < nh; i += kPreThreads) { s_k[i] = C.hull_k[i]; s_s[i] = C.hull_s[i]; }
    __syncthreads();
    const double *hk = in_lds ? s_k : C.hull_k;
    const double *hs = in_lds ? s_s : C.hull_s;
    int cnt = 0, smin = INT_MAX;
    for (int q = 0; q < kPrePer; ++q) {
        const int64_t k = (int64_t)blockIdx.x * kPreBlock + (int64_t)q * kPreThreads + t;
        if (k >= n1) break;
        const int32_t s = coef_scale(coef, k);
        const int g = is_good(s, k, hk, hs, nh, T);
        W.good[k] = g;
        cnt += g;
        if (g) smin = min(smin, (int)s);
    }
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o, kWave);
        smin = min(smin, __shfl_xor(smin, o, kWave));
    }
    if (t % kWave == 0) { s_cnt[t / kWave] = cnt; s_min[t / kWave] = smin; }
    __syncthreads();
    if (t == 0) {
        int c = 0, m = INT_MAX;
        for (int i = 0; i < kPreThreads / kWave; ++i) { c += s_cnt[i]; m = min(m, s_min[i]); }
        W.blk_sum[blockIdx.x] = c;
        if (m != INT_MAX) atomicMin(&W.ictl[0], m);
    }
}

// one workgroup: exclusive prefix of the workgroup counts, |G_p|, and the table
// shift: the window sum holds a_k z^(k - lo) in FP64, whose terms span
// [smin - T, smax + T] binary orders after a shift of the coefficients by
// 2^-shift, which must fit the FP64 exponent range with margin
// the table shift and the range check of the good scales
__device__ __forceinline__ void table_shift(long long smax, long long smin, long long T, long long *info) {
    const long long shift = (smax + smin) / 2;
    const long long half = 1022 - T - 64;
    info[kShift] = shift;
    info[kUnsupported] = (smax - shift > half || shift - smin > half) ? 1 : 0;
}

__global__ __launch_bounds__(kPreThreads) void k_pre_scan(int64_t nb, PlanWs W) {
    __shared__ int32_t part[kPreThreads];
    const int t = threadIdx.x;
    const int64_t per = (nb + kPreThreads - 1) / kPreThreads;
    const int64_t b0 = std::min<int64_t>((int64_t)t * per, nb), b1 = std::min<int64_t>(b0 + per, nb);
    int32_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += W.blk_sum[b];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int32_t acc = 0;
        for (int i = 0; i < kPreThreads; ++i) { const int32_t x = part[i]; part[i] = acc; acc += x; }
        W.info[kNGood] = acc;
        const long long smin = W.ictl[0];
        W.info[kSMinGood] = acc > 0 ? smin : 0;
        if (acc > 0) table_shift(W.info[kSMax], smin, W.info[kT], W.info);
    }
    __syncthreads();
    int32_t acc = part[t];
    for (int64_t b = b0; b < b1; ++b) { W.blk_off[b] = acc; acc += W.blk_sum[b]; }
}

// prefix counts of G_p (gprefix[k] = #(G_p within [0, k))), the masked,
// shifted coefficient table, and G_p as a list (index, shifted coefficient)
__global__ __launch_bounds__(kPreThreads) void k_pre_table(const double2 *__restrict__ coef, int64_t n1, PlanWs W) {
    __shared__ int32_t s_wave[kPreThreads / kWave];
    const int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    const int shift = (int)W.info[kShift];
    // this thread's kPrePer consecutive coefficients
    const int64_t k0 = (int64_t)blockIdx.x * kPreBlock + (int64_t)t * kPrePer;
    int32_t g[kPrePer];
    int32_t own = 0;
#pragma unroll
    for (int q = 0; q < kPrePer; ++q) {
        const int64_t k = k0 + q;
        g[q] = k < n1 ? W.good[k] : 0;
        own += g[q];
    }
    // exclusive prefix of own over the workgroup
    int32_t x = own;
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) s_wave[wv] = x;
    __syncthreads();
    if (t == 0) {
        int32_t acc = 0;
        for (int i = 0; i < kPreThreads / kWave; ++i) { const int32_t v = s_wave[i]; s_wave[i] = acc; acc += v; }
    }
    __syncthreads();
    int32_t pre = W.blk_off[blockIdx.x] + s_wave[wv] + x - own;
#pragma unroll
    for (int q = 0; q < kPrePer; ++q) {
        const int64_t k = k0 + q;
        if (k < n1) {
            W.gprefix[k] = pre;
            double2 o = make_double2(0.0, 0.0);
            if (g[q]) {
                const double2 a = coef[k];
                o = make_double2(ldexp(a.x, -shift), ldexp(a.y, -shift));
                W.gidx[pre] = (int32_t)k;
                W.gcoef[pre] = o;
            }
            pre += g[q];
            W.coef[k] = o;
            if (k == n1 - 1) W.gprefix[n1] = pre;
        }
    }
}

// FP32 plans, per chunk of kChunk coefficients: sigma = the largest good scale
// (FP32 entries below 1 in modulus); FP32 only if every good entry stays a
// normal FP32 number with margin (sigma - least good s <= 120) and the cover
// drops by at most 99 within the chunk (then a block partial of any point
// that matters stays above the FP32 range floor).  sig32 = sigma - shift.
template <class HK, class HS>
__device__ __forceinline__ double cover_at(HK hk, HS hs, int nh, int64_t k) {
    if (nh == 1) return (double)hs[0];
    int lo = 0, hi = nh - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((double)hk[mid] <= (double)k) lo = mid; else hi = mid - 1;
    }
    const double k0 = (double)hk[lo], k1 = (double)hk[lo + 1];
    const double s0 = (double)hs[lo], s1 = (double)hs[lo + 1];
    return s0 + (s1 - s0) * ((double)k - k0) / (k1 - k0);
}

// sig32 of chunk [a, b] (inside the trimmed range) from the largest and the
// least good scale there
template <class HK, class HS>
__device__ __forceinline__ int32_t chunk_sig32(int gmax, int gmin, HK hk, HS hs, int nh, int64_t a, int64_t b,
                                               long long shift) {
    if (gmax == INT_MIN) return 0;                        // no good coefficient: entries 0
    const double emin = fmin(cover_at(hk, hs, nh, a), cover_at(hk, hs, nh, b));
    return ((int64_t)gmax - gmin <= 120 && (double)gmax - emin <= 99.0) ? (int32_t)(gmax - shift) : kNoFp32;
}

__global__ __launch_bounds__(256) void k_pre_sig32(const double2 *__restrict__ coef, PlanWs W) {
    __shared__ int32_t s_max[256 / kWave], s_min[256 / kWave];
    const int64_t c = blockIdx.x;
    const int t = threadIdx.x;
    const int nh = (int)W.info[kNh];
    if (nh == 0) {
        if (t == 0) W.sig32[c] = kNoFp32;
        return;
    }
    const int64_t v = W.info[kV], dt = W.info[kDt];
    const int64_t a = std::max<int64_t>(c * kChunk, v), b = std::min<int64_t>(c * kChunk + kChunk - 1, dt);
    if (a > b) {                                           // no coefficient of the trimmed range
        if (t == 0) W.sig32[c] = 0;
        return;
    }
    int gmax = INT_MIN, gmin = INT_MAX;
    for (int64_t k = a + t; k <= b; k += 256)
        if (W.good[k]) { const int32_t sk = coef_scale(coef, k); gmax = max(gmax, sk); gmin = min(gmin, sk); }
    for (int o = 32; o > 0; o >>= 1) {
        gmax = max(gmax, __shfl_xor(gmax, o, kWave));
        gmin = min(gmin, __shfl_xor(gmin, o, kWave));
    }
    if (t % kWave == 0) { s_max[t / kWave] = gmax; s_min[t / kWave] = gmin; }
    __syncthreads();
    if (t == 0) {
        for (int i = 0; i < 256 / kWave; ++i) { gmax = max(gmax, s_max[i]); gmin = min(gmin, s_min[i]); }
        W.sig32[c] = chunk_sig32(gmax, gmin, (const double *)W.hull_k, (const double *)W.hull_s, nh, a, b,
                                 W.info[kShift]);
    }
}

// the FP32 table: coef32[k] = coef[k] 2^-sig32[k / C] rounded to FP32 (0 in
// chunks that stay in FP64)
__global__ void k_mask32(const double2 *__restrict__ coef, const int32_t *__restrict__ sig32, int64_t n,
                         float2 *__restrict__ out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t sg = sig32[k / kChunk];
    float2 o = make_float2(0.0f, 0.0f);
    if (sg != kNoFp32) {
        const double2 a = coef[k];
        o = make_float2((float)ldexp(a.x, -sg), (float)ldexp(a.y, -sg));
    }
    out[k] = o;
}

// ---- one workgroup per polynomial (small polynomials, batches)
constexpr int64_t kFusedMax = (int64_t)1 << 17;   // coefficients of a polynomial k_pre_fused takes

struct PreJob {
    const double2 *coef;
    int64_t n1;
    PlanWs W;
};

// the cover as k_pre_fused holds it in LDS: index and scale + kSOff
struct LdsK { const int32_t *p; __device__ int64_t operator[](int i) const { return p[i]; } };
struct LdsS { const int16_t *p; __device__ int64_t operator[](int i) const { return (int64_t)p[i] - kSOff; } };

// exclusive prefix of own over the workgroup (s_wave: kPreThreads / kWave
// entries of LDS); returns it and sets total
__device__ __forceinline__ int32_t block_excl(int32_t own, int32_t *s_wave, int32_t &total) {
    const int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    int32_t x = own;
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) s_wave[wv] = x;
    __syncthreads();
    int32_t before = 0, tot = 0;
    for (int i = 0; i < kPreThreads / kWave; ++i) {
        const int32_t v = s_wave[i];
        if (i < wv) before += v;
        tot += v;
    }
    __syncthreads();
    total = tot;
    return before + x - own;
}

// Every step of the preconditioning for one polynomial per workgroup (jobs,
// or `single` when jobs is NULL): the scales' extreme indices in LDS, the
// candidates sorted in LDS, the monotone chain, G_p, the prefix counts and
// tables (the good test is recomputed where it is needed again, rather than
// read back), and for FP32 plans the FP32 table.  The same arithmetic as the
// per-coefficient kernels, so the same plan bit for bit.
__global__ __launch_bounds__(kPreThreads) void k_pre_fused(const PreJob *__restrict__ jobs, PreJob single,
                                                           int32_t p_bits, int32_t fp32) {
    __shared__ int32_t ck[kSortCap];
    __shared__ int16_t cb[kSortCap];
    __shared__ int32_t s_wave[kPreThreads / kWave], s_min[kPreThreads / kWave];
    __shared__ int32_t s_cnt, s_bad, s_nh, s_smax;
    const PreJob J = jobs ? jobs[blockIdx.x] : single;
    const double2 *__restrict__ coef = J.coef;
    const int64_t n1 = J.n1;
    const PlanWs &W = J.W;
    const int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    // per scale value, its least and largest index (the candidates), in the
    // first 2 kSBins entries of ck
    int32_t *lmin = ck, *lmax = ck + kSBins;
    for (int i = t; i < kSBins; i += kPreThreads) { lmin[i] = INT_MAX; lmax[i] = INT_MIN; }
    if (t == 0) { s_cnt = 0; s_bad = 0; }
    __syncthreads();
    bool bad = false;
    for (int64_t k = t; k < n1; k += kPreThreads) {
        const double2 a = coef[k];
        if (!isfinite(a.x) || !isfinite(a.y)) { bad = true; continue; }
        const int32_t s = scale_exact(a.x, a.y);
        if (s != kNegInfScale) {
            atomicMin(&lmin[s + kSOff], (int32_t)k);
            atomicMax(&lmax[s + kSOff], (int32_t)k);
        }
    }
    if (bad) s_bad = 1;
    __syncthreads();
    // the candidates of this thread's bins, held until every bin is read
    constexpr int kBinsPer = (kSBins + kPreThreads - 1) / kPreThreads;
    int32_t qlo[kBinsPer], qhi[kBinsPer];
    int nq = 0;
#pragma unroll
    for (int r = 0; r < kBinsPer; ++r) {
        const int b = t + r * kPreThreads;
        qlo[r] = b < kSBins ? lmin[b] : INT_MAX;
        qhi[r] = b < kSBins ? lmax[b] : INT_MIN;
        nq += qlo[r] == INT_MAX ? 0 : (qhi[r] != qlo[r] ? 2 : 1);
    }
    __syncthreads();
    int pos = nq ? atomicAdd(&s_cnt, nq) : 0;
#pragma unroll
    for (int r = 0; r < kBinsPer; ++r) {
        if (qlo[r] != INT_MAX) {
            const int16_t b = (int16_t)(t + r * kPreThreads);
            ck[pos] = qlo[r]; cb[pos] = b; ++pos;
            if (qhi[r] != qlo[r]) { ck[pos] = qhi[r]; cb[pos] = b; ++pos; }
        }
    }
    __syncthreads();
    const int n = s_cnt;
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (int i = n + t; i < np2; i += kPreThreads) { ck[i] = INT_MAX; cb[i] = 0; }
    __syncthreads();
    bitonic_sort(ck, cb, np2);
    if (t == 0) {
        int smax = INT_MIN;
        s_nh = n > 0 ? monotone_chain(ck, cb, n, smax) : 0;
        s_smax = smax;
    }
    __syncthreads();
    const int nh = s_nh;
    const LdsK hk{ck};
    const LdsS hs{cb};
    const int64_t v = nh > 0 ? ck[0] : -1, dt = nh > 0 ? ck[nh - 1] : -1;
    int64_t T = 0;
    if (nh > 0) {
        const int64_t deff = dt - v;
        T = p_bits + bitlen_d(deff > 1 ? deff : 1) + 3;
    }
    for (int i = t; i < nh; i += kPreThreads) {
        W.hull_k[i] = (double)ck[i];
        W.hull_s[i] = (double)((int)cb[i] - kSOff);
    }
    // G_p: flags, count, least good scale
    int cnt = 0, smin = INT_MAX;
    for (int64_t k = t; k < n1; k += kPreThreads) {
        const int32_t s = coef_scale(coef, k);
        const int g = is_good(s, k, hk, hs, nh, T);
        W.good[k] = g;
        cnt += g;
        if (g) smin = min(smin, (int)s);
    }
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o, kWave);
        smin = min(smin, __shfl_xor(smin, o, kWave));
    }
    if (lane == 0) { s_wave[wv] = cnt; s_min[wv] = smin; }
    __syncthreads();
    int32_t ngood = 0, sming = INT_MAX;
    for (int i = 0; i < kPreThreads / kWave; ++i) { ngood += s_wave[i]; sming = min(sming, s_min[i]); }
    __syncthreads();
    long long sh_info[2] = {0, 0};                     // kShift, kUnsupported
    if (ngood > 0) {
        long long tmp[kInfoLen];
        table_shift(s_smax, sming, T, tmp);
        sh_info[0] = tmp[kShift];
        sh_info[1] = tmp[kUnsupported];
    }
    const int shift = (int)sh_info[0];
    // prefix counts, the masked table and the list, kPreBlock coefficients at a time
    int32_t carry = 0;
    for (int64_t base = 0; base < n1; base += kPreBlock) {
        const int64_t k0 = base + (int64_t)t * kPrePer;
        int32_t g[kPrePer];
        int32_t own = 0;
#pragma unroll
        for (int q = 0; q < kPrePer; ++q) {
            const int64_t k = k0 + q;
            g[q] = k < n1 ? is_good(coef_scale(coef, k), k, hk, hs, nh, T) : 0;
            own += g[q];
        }
        int32_t total = 0;
        int32_t pre = carry + block_excl(own, s_wave, total);
#pragma unroll
        for (int q = 0; q < kPrePer; ++q) {
            const int64_t k = k0 + q;
            if (k < n1) {
                W.gprefix[k] = pre;
                double2 o = make_double2(0.0, 0.0);
                if (g[q]) {
                    const double2 a = coef[k];
                    o = make_double2(ldexp(a.x, -shift), ldexp(a.y, -shift));
                    W.gidx[pre] = (int32_t)k;
                    W.gcoef[pre] = o;
                }
                pre += g[q];
                W.coef[k] = o;
            }
        }
        carry += total;
    }
    if (t == 0) W.gprefix[n1] = carry;
    // FP32 plans: a wavefront per chunk of kChunk coefficients
    if (fp32) {
        const int64_t nc = n_chunks(n1 - 1);
        for (int64_t c = wv; c < nc; c += kPreThreads / kWave) {
            int32_t sg = kNoFp32;
            if (nh > 0) {
                const int64_t a = max(c * kChunk, v), b = min(c * kChunk + kChunk - 1, dt);
                if (a > b) {
                    sg = 0;
                } else {
                    int gmax = INT_MIN, gmin = INT_MAX;
                    for (int64_t k = a + lane; k <= b; k += kWave) {
                        const int32_t sk = coef_scale(coef, k);
                        if (is_good(sk, k, hk, hs, nh, T)) { gmax = max(gmax, sk); gmin = min(gmin, sk); }
                    }
                    for (int o = 32; o > 0; o >>= 1) {
                        gmax = max(gmax, __shfl_xor(gmax, o, kWave));
                        gmin = min(gmin, __shfl_xor(gmin, o, kWave));
                    }
                    sg = chunk_sig32(gmax, gmin, hk, hs, nh, a, b, shift);
                }
            }
            if (lane == 0) W.sig32[c] = sg;
            const int64_t e = min(c * kChunk + kChunk, n1);
            for (int64_t k = c * kChunk + lane; k < e; k += kWave) {
                float2 o = make_float2(0.0f, 0.0f);
                if (sg != kNoFp32 && is_good(coef_scale(coef, k), k, hk, hs, nh, T)) {
                    const double2 a = coef[k];
                    const double ox = ldexp(a.x, -shift), oy = ldexp(a.y, -shift);
                    o = make_float2((float)ldexp(ox, -sg), (float)ldexp(oy, -sg));
                }
                W.coef32[k] = o;
            }
        }
    }
    if (t == 0) {
        long long *info = W.info;
        for (int i = 0; i < kInfoLen; ++i) info[i] = 0;
        info[kNonFinite] = s_bad;
        info[kV] = v;
        info[kDt] = dt;
        info[kNh] = nh;
        if (n > 0) info[kSMax] = s_smax;
        info[kT] = T;
        info[kNGood] = ngood;
        info[kSMinGood] = ngood > 0 ? sming : 0;
        info[kShift] = sh_info[0];
        info[kUnsupported] = sh_info[1];
        info[kA0Re] = __double_as_longlong(coef[0].x);
        info[kA0Im] = __double_as_longlong(coef[0].y);
    }
}

int64_t bitlen(int64_t v) {
    int64_t b = 0;
    while (v > 0) { ++b; v >>= 1; }
    return b;
}

// the kernels of the good set and the tables (the second part), given the cover
void launch_plan_part(const double2 *coef, int64_t n1, const CoverWs &C, const PlanWs &W, int32_t p_bits, bool fp32,
                      hipStream_t stream) {
    const int64_t nb = n_blocks(n1);
    k_plan_init<<<1, 64, 0, stream>>>(W);
    k_pre_good<<<(unsigned)nb, kPreThreads, 0, stream>>>(coef, n1, C, W, p_bits);
    k_pre_scan<<<1, kPreThreads, 0, stream>>>(nb, W);
    k_pre_table<<<(unsigned)nb, kPreThreads, 0, stream>>>(coef, n1, W);
    if (fp32) {
        k_pre_sig32<<<(unsigned)n_chunks(n1 - 1), 256, 0, stream>>>(coef, W);
        k_mask32<<<(unsigned)((n1 + 255) / 256), 256, 0, stream>>>(W.coef, W.sig32, n1, W.coef32);
    }
}

// the kernels of the cover (the first part)
void launch_cover_part(const double2 *coef, int64_t n1, const CoverWs &C, hipStream_t stream) {
    k_pre_init<<<(kSBins + 255) / 256, 256, 0, stream>>>(C);
    k_pre_scale<<<(unsigned)n_blocks(n1), kPreThreads, 0, stream>>>(coef, n1, C);
    k_pre_hull<<<1, kPreThreads, 0, stream>>>(C);
}

fpe_status check_precondition_args(int64_t d, int32_t p_bits, uint32_t flags) {
    if (d < 0 || d >= INT32_MAX - 2) return fail(FPE_ERR_INVALID_ARG, "degree out of range");
    if (p_bits < 1 || p_bits > 53) return fail(FPE_ERR_PRECISION, "p_bits must be in 1..53");
    if (flags & ~(uint32_t)(FPE_PRECONDITION_FP32 | FPE_PRECONDITION_FP32_COMPENSATED))
        return fail(FPE_ERR_INVALID_ARG, "unknown flag");
    if ((flags & FPE_PRECONDITION_FP32_COMPENSATED) && !(flags & FPE_PRECONDITION_FP32))
        return fail(FPE_ERR_INVALID_ARG, "FPE_PRECONDITION_FP32_COMPENSATED needs FPE_PRECONDITION_FP32");
    if ((flags & FPE_PRECONDITION_FP32) && p_bits > 24)
        return fail(FPE_ERR_PRECISION, "FP32 window sums need p_bits <= 24");
    return FPE_OK;
}

// the host handle of a plan from its tables and the counters read back
fpe_status make_plan(const long long *info, const PlanWs &w, int64_t d, int32_t p_bits, uint32_t flags, int device,
                     fpe_plan_t *out_plan) {
    const bool fp32 = (flags & FPE_PRECONDITION_FP32) != 0;
    if (info[kNonFinite]) return fail(FPE_ERR_NONFINITE, "a coefficient is NaN or infinite");
    if (info[kUnsupported])
        return fail(FPE_ERR_UNSUPPORTED, "good coefficients span too many binary orders for FP64 windows");
    std::unique_ptr<fpe_plan_s> plan(new fpe_plan_s());
    plan->d = d;
    plan->p = p_bits;
    plan->device = device;
    plan->nh = info[kNh];
    if (plan->nh == 0) {   // P == 0
        plan->v = -1; plan->dt = -1; plan->ngood = 0; plan->T = 0; plan->smax = 0; plan->smin_good = 0;
    } else {
        plan->v = info[kV]; plan->dt = info[kDt]; plan->ngood = info[kNGood]; plan->T = info[kT];
        plan->smax = info[kSMax]; plan->smin_good = info[kSMinGood];
    }
    plan->good_dev = w.good;

    DevPlan &P = plan->dev;
    P.coef = w.coef;
    P.gprefix = w.gprefix;
    P.gidx = w.gidx;
    P.gcoef = w.gcoef;
    P.hull_k = w.hull_k;
    P.hull_s = w.hull_s;
    P.nh = (int32_t)plan->nh;
    P.v = (int32_t)plan->v;
    P.dt = (int32_t)plan->dt;
    P.T = (int32_t)plan->T;
    P.chunk = kChunk;
    // fixed-point accumulators of windows spanning several chunks: the high
    // word holds value 2^(fix_shift - eref), whose sum over a window is below
    // W / 4 < 2^(bitlen(W) - 2); the low word holds fix_lo more bits of each
    // partial and its sum over at most `chunks` partials stays below 2^62
    // (counted for the shortest chunk an evaluation may choose)
    const int64_t wmax = std::max<int64_t>(plan->dt - plan->v + 1, 1);
    const int64_t chunks = std::max<int64_t>(plan->dt / kChunkMin - plan->v / kChunkMin + 1, 1);
    P.fix_shift = (int32_t)(60 - bitlen(wmax));
    P.fix_lo = (int32_t)std::min<int64_t>(44, 62 - bitlen(chunks));
    P.coef_shift = plan->ngood > 0 ? (int32_t)info[kShift] : 0;
    double a0r, a0i;
    std::memcpy(&a0r, &info[kA0Re], sizeof(double));
    std::memcpy(&a0i, &info[kA0Im], sizeof(double));
    P.a0 = make_double2(a0r, a0i);
    P.coef32 = fp32 ? w.coef32 : nullptr;
    P.sig32 = fp32 ? w.sig32 : nullptr;
    P.f32comp = fp32 && (flags & FPE_PRECONDITION_FP32_COMPENSATED) ? 1 : 0;
    *out_plan = plan.release();
    return FPE_OK;
}

}  // namespace
}  // namespace fpe

// Host handle of a cover (fpe_cover_build): the device view and its summary.
struct fpe_cover_s {
    fpe::CoverWs dev;
    int64_t d, v, dt, nh, smax;
    int device;
};

using namespace fpe;

extern "C" fpe_status fpe_precondition_workspace_size(int64_t d, int32_t p_bits, uint32_t flags,
                                                      size_t *bytes) {
    if (!bytes) return fail(FPE_ERR_INVALID_ARG, "bytes is NULL");
    fpe_status st = check_precondition_args(d, p_bits, flags);
    if (st != FPE_OK) return st;
    *bytes = pre_layout(d, flags, nullptr, nullptr, nullptr);
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_precondition(const double *coef_dev, int64_t d, int32_t p_bits,
                                       uint32_t flags, void *workspace_dev, size_t workspace_bytes,
                                       hipStream_t stream, fpe_plan_t *out_plan) {
    if (!coef_dev || !workspace_dev || !out_plan) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    *out_plan = nullptr;
    size_t need = 0;
    fpe_status st = fpe_precondition_workspace_size(d, p_bits, flags, &need);
    if (st != FPE_OK) return st;
    if (workspace_bytes < need)
        return fail(FPE_ERR_WORKSPACE, "precondition workspace too small: need " + std::to_string(need));
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0 ||
        reinterpret_cast<uintptr_t>(coef_dev) % 16 != 0)
        return fail(FPE_ERR_INVALID_ARG, "workspace must be 256-byte aligned, coefficients 16-byte aligned");

    PlanWs w;
    CoverWs c;
    pre_layout(d, flags, &w, &c, workspace_dev);
    const int64_t n1 = d + 1;
    const double2 *coef = reinterpret_cast<const double2 *>(coef_dev);
    const bool fp32 = (flags & FPE_PRECONDITION_FP32) != 0;
    if (n1 <= kFusedMax) {
        k_pre_fused<<<1, kPreThreads, 0, stream>>>(nullptr, PreJob{coef, n1, w}, p_bits, fp32 ? 1 : 0);
    } else {
        launch_cover_part(coef, n1, c, stream);
        launch_plan_part(coef, n1, c, w, p_bits, fp32, stream);
    }
    FPE_HIP_CHECK(hipGetLastError());
    long long info[kInfoLen];
    FPE_HIP_CHECK(hipMemcpyAsync(info, w.info, sizeof(info), hipMemcpyDeviceToHost, stream));
    FPE_HIP_CHECK(hipStreamSynchronize(stream));
    int device = 0;
    FPE_HIP_CHECK(hipGetDevice(&device));
    st = make_plan(info, w, d, p_bits, flags, device, out_plan);
    if (st == FPE_OK) set_error("");
    return st;
}

// ---- the two parts apart (Remark partialpreproc, Section 5.1)
extern "C" fpe_status fpe_cover_workspace_size(int64_t d, size_t *bytes) {
    if (!bytes) return fail(FPE_ERR_INVALID_ARG, "bytes is NULL");
    if (d < 0 || d >= INT32_MAX - 2) return fail(FPE_ERR_INVALID_ARG, "degree out of range");
    Carver take{nullptr};
    cover_layout(d, true, take);
    *bytes = take.off;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_cover_build(const double *coef_dev, int64_t d, void *workspace_dev, size_t workspace_bytes,
                                      hipStream_t stream, fpe_cover_t *out_cover) {
    if (!coef_dev || !workspace_dev || !out_cover) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    *out_cover = nullptr;
    size_t need = 0;
    fpe_status st = fpe_cover_workspace_size(d, &need);
    if (st != FPE_OK) return st;
    if (workspace_bytes < need)
        return fail(FPE_ERR_WORKSPACE, "cover workspace too small: need " + std::to_string(need));
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0 ||
        reinterpret_cast<uintptr_t>(coef_dev) % 16 != 0)
        return fail(FPE_ERR_INVALID_ARG, "workspace must be 256-byte aligned, coefficients 16-byte aligned");
    Carver take{static_cast<char *>(workspace_dev)};
    const CoverWs c = cover_layout(d, true, take);
    launch_cover_part(reinterpret_cast<const double2 *>(coef_dev), d + 1, c, stream);
    FPE_HIP_CHECK(hipGetLastError());
    long long info[kInfoLen];
    FPE_HIP_CHECK(hipMemcpyAsync(info, c.info, sizeof(info), hipMemcpyDeviceToHost, stream));
    FPE_HIP_CHECK(hipStreamSynchronize(stream));
    if (info[kNonFinite]) return fail(FPE_ERR_NONFINITE, "a coefficient is NaN or infinite");
    std::unique_ptr<fpe_cover_s> cv(new fpe_cover_s());
    cv->dev = c;
    cv->d = d;
    cv->nh = info[kNh];
    cv->v = cv->nh > 0 ? info[kV] : -1;
    cv->dt = cv->nh > 0 ? info[kDt] : -1;
    cv->smax = cv->nh > 0 ? info[kSMax] : 0;
    FPE_HIP_CHECK(hipGetDevice(&cv->device));
    *out_cover = cv.release();
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_cover_info(fpe_cover_t cover, int64_t *info_host) {
    if (!cover || !info_host) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    info_host[0] = cover->d; info_host[1] = cover->v; info_host[2] = cover->dt; info_host[3] = cover->nh;
    info_host[4] = cover->smax;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_cover_destroy(fpe_cover_t cover) {
    delete cover;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_plan_from_cover_workspace_size(fpe_cover_t cover, int32_t p_bits, uint32_t flags,
                                                         size_t *bytes) {
    if (!cover || !bytes) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    fpe_status st = check_precondition_args(cover->d, p_bits, flags);
    if (st != FPE_OK) return st;
    Carver take{nullptr};
    plan_layout(cover->d, flags, take);
    *bytes = take.off;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_plan_from_cover(fpe_cover_t cover, const double *coef_dev, int32_t p_bits, uint32_t flags,
                                          void *workspace_dev, size_t workspace_bytes, hipStream_t stream,
                                          fpe_plan_t *out_plan) {
    if (!cover || !coef_dev || !workspace_dev || !out_plan) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    *out_plan = nullptr;
    size_t need = 0;
    fpe_status st = fpe_plan_from_cover_workspace_size(cover, p_bits, flags, &need);
    if (st != FPE_OK) return st;
    if (workspace_bytes < need)
        return fail(FPE_ERR_WORKSPACE, "plan workspace too small: need " + std::to_string(need));
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0 ||
        reinterpret_cast<uintptr_t>(coef_dev) % 16 != 0)
        return fail(FPE_ERR_INVALID_ARG, "workspace must be 256-byte aligned, coefficients 16-byte aligned");
    int device = 0;
    FPE_HIP_CHECK(hipGetDevice(&device));
    if (device != cover->device) return fail(FPE_ERR_INVALID_ARG, "the cover lives on another device");
    Carver take{static_cast<char *>(workspace_dev)};
    const PlanWs w = plan_layout(cover->d, flags, take);
    const bool fp32 = (flags & FPE_PRECONDITION_FP32) != 0;
    launch_plan_part(reinterpret_cast<const double2 *>(coef_dev), cover->d + 1, cover->dev, w, p_bits, fp32, stream);
    FPE_HIP_CHECK(hipGetLastError());
    long long info[kInfoLen];
    FPE_HIP_CHECK(hipMemcpyAsync(info, w.info, sizeof(info), hipMemcpyDeviceToHost, stream));
    FPE_HIP_CHECK(hipStreamSynchronize(stream));
    st = make_plan(info, w, cover->d, p_bits, flags, device, out_plan);
    if (st == FPE_OK) set_error("");
    return st;
}

// ---- many polynomials at once
namespace {
struct BatchPreLayout {
    size_t jobs, infos, total;
    std::vector<size_t> plan_off;     // per polynomial: its plan (and cover scratch when large)
};

fpe_status batch_pre_layout(int32_t n_poly, const int64_t *offs, uint32_t flags, BatchPreLayout *L) {
    if (n_poly < 1) return fail(FPE_ERR_INVALID_ARG, "n_poly must be >= 1");
    if (!offs) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    if (offs[0] != 0) return fail(FPE_ERR_INVALID_ARG, "coef_offsets[0] must be 0");
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L->jobs = take(sizeof(PreJob) * (size_t)n_poly);
    L->infos = take(sizeof(long long) * kInfoLen * (size_t)n_poly);
    L->plan_off.resize(n_poly);
    for (int32_t i = 0; i < n_poly; ++i) {
        const int64_t n1 = offs[i + 1] - offs[i];
        if (n1 < 1) return fail(FPE_ERR_INVALID_ARG, "every polynomial needs at least one coefficient");
        if (n1 - 1 >= INT32_MAX - 2) return fail(FPE_ERR_INVALID_ARG, "degree out of range");
        Carver c{nullptr};
        plan_layout(n1 - 1, flags, c);
        if (n1 > kFusedMax) cover_layout(n1 - 1, false, c);
        L->plan_off[i] = take(c.off);
    }
    L->total = off;
    return FPE_OK;
}
}  // namespace

extern "C" fpe_status fpe_precondition_batched_workspace_size(int32_t n_poly, const int64_t *coef_offsets_host,
                                                              int32_t p_bits, uint32_t flags, size_t *bytes) {
    if (!bytes) return fail(FPE_ERR_INVALID_ARG, "bytes is NULL");
    fpe_status st = check_precondition_args(0, p_bits, flags);
    if (st != FPE_OK) return st;
    BatchPreLayout L;
    st = batch_pre_layout(n_poly, coef_offsets_host, flags, &L);
    if (st != FPE_OK) return st;
    *bytes = L.total;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_precondition_batched(const double *coef_dev, const int64_t *coef_offsets_host,
                                               int32_t n_poly, int32_t p_bits, uint32_t flags, void *workspace_dev,
                                               size_t workspace_bytes, hipStream_t stream, fpe_plan_t *plans_out) {
    if (!coef_dev || !workspace_dev || !plans_out) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    fpe_status st = check_precondition_args(0, p_bits, flags);
    if (st != FPE_OK) return st;
    BatchPreLayout L;
    st = batch_pre_layout(n_poly, coef_offsets_host, flags, &L);
    if (st != FPE_OK) return st;
    for (int32_t i = 0; i < n_poly; ++i) plans_out[i] = nullptr;
    if (workspace_bytes < L.total)
        return fail(FPE_ERR_WORKSPACE, "batched precondition workspace too small: need " + std::to_string(L.total));
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0 ||
        reinterpret_cast<uintptr_t>(coef_dev) % 16 != 0)
        return fail(FPE_ERR_INVALID_ARG, "workspace must be 256-byte aligned, coefficients 16-byte aligned");
    char *base = static_cast<char *>(workspace_dev);
    const double2 *coef = reinterpret_cast<const double2 *>(coef_dev);
    long long *infos = reinterpret_cast<long long *>(base + L.infos);
    const bool fp32 = (flags & FPE_PRECONDITION_FP32) != 0;
    std::vector<PreJob> jobs;
    std::vector<PlanWs> ws(n_poly);
    jobs.reserve(n_poly);
    for (int32_t i = 0; i < n_poly; ++i) {
        const int64_t n1 = coef_offsets_host[i + 1] - coef_offsets_host[i];
        Carver c{base + L.plan_off[i]};
        ws[i] = plan_layout(n1 - 1, flags, c);
        ws[i].info = infos + (size_t)i * kInfoLen;     // every counter block in one run, read back at once
        const double2 *ci = coef + coef_offsets_host[i];
        if (n1 <= kFusedMax) {
            jobs.push_back(PreJob{ci, n1, ws[i]});
        } else {
            CoverWs cv = cover_layout(n1 - 1, false, c);
            cv.hull_k = ws[i].hull_k;
            cv.hull_s = ws[i].hull_s;
            launch_cover_part(ci, n1, cv, stream);
            launch_plan_part(ci, n1, cv, ws[i], p_bits, fp32, stream);
        }
    }
    if (!jobs.empty()) {
        PreJob *jd = reinterpret_cast<PreJob *>(base + L.jobs);
        FPE_HIP_CHECK(hipMemcpyAsync(jd, jobs.data(), sizeof(PreJob) * jobs.size(), hipMemcpyHostToDevice, stream));
        k_pre_fused<<<(unsigned)jobs.size(), kPreThreads, 0, stream>>>(jd, jobs[0], p_bits, fp32 ? 1 : 0);
    }
    FPE_HIP_CHECK(hipGetLastError());
    std::vector<long long> info((size_t)n_poly * kInfoLen);
    FPE_HIP_CHECK(hipMemcpyAsync(info.data(), infos, sizeof(long long) * info.size(), hipMemcpyDeviceToHost, stream));
    FPE_HIP_CHECK(hipStreamSynchronize(stream));
    int device = 0;
    FPE_HIP_CHECK(hipGetDevice(&device));
    for (int32_t i = 0; i < n_poly; ++i) {
        const int64_t d = coef_offsets_host[i + 1] - coef_offsets_host[i] - 1;
        st = make_plan(&info[(size_t)i * kInfoLen], ws[i], d, p_bits, flags, device, &plans_out[i]);
        if (st != FPE_OK) {
            const std::string msg = "polynomial " + std::to_string(i) + ": " + fpe_last_error();
            for (int32_t j = 0; j < i; ++j) { delete plans_out[j]; plans_out[j] = nullptr; }
            return fail(st, msg);
        }
    }
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_plan_info(fpe_plan_t plan, int64_t *info) {
    if (!plan || !info) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    info[0] = plan->d; info[1] = plan->v; info[2] = plan->dt; info[3] = plan->nh;
    info[4] = plan->ngood; info[5] = plan->T; info[6] = plan->p; info[7] = plan->dev.chunk;
    info[8] = plan->smax; info[9] = plan->smin_good;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_plan_export(fpe_plan_t plan, int64_t *hull_k, int64_t *hull_s,
                                      int64_t hull_cap, uint8_t *good) {
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    if ((hull_k || hull_s) && hull_cap < plan->nh) return fail(FPE_ERR_INVALID_ARG, "hull_cap too small");
    if ((hull_k || hull_s) && plan->nh > 0) {
        std::vector<double> hk(plan->nh), hs(plan->nh);
        FPE_HIP_CHECK(hipMemcpy(hk.data(), plan->dev.hull_k, sizeof(double) * hk.size(), hipMemcpyDeviceToHost));
        FPE_HIP_CHECK(hipMemcpy(hs.data(), plan->dev.hull_s, sizeof(double) * hs.size(), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < plan->nh; ++i) {
            if (hull_k) hull_k[i] = (int64_t)hk[i];
            if (hull_s) hull_s[i] = (int64_t)hs[i];
        }
    }
    if (good) {
        std::vector<int32_t> g(plan->d + 1);
        FPE_HIP_CHECK(hipMemcpy(g.data(), plan->good_dev, sizeof(int32_t) * g.size(), hipMemcpyDeviceToHost));
        for (size_t k = 0; k < g.size(); ++k) good[k] = (uint8_t)(g[k] != 0);
    }
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_plan_destroy(fpe_plan_t plan) {
    delete plan;
    set_error("");
    return FPE_OK;
}
