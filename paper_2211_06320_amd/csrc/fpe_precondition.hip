// Preconditioning (Algorithm A_p, first block; Section 5.1 of arXiv 2211.06320),
// on the GPU, with one host synchronisation at the end:
//
//   k_pre_init    the candidate table and the counters
//   k_pre_scale   s(a_k) = 1 + floor(log2|a_k|) of every coefficient (Section 2.3,
//                 eq. dsz), decided exactly with 64-bit integer arithmetic on the
//                 significands; per value of s, the least and the largest index
//                 holding it.  Only those can be vertices of the concave cover:
//                 the points of one height between them lie on a level segment.
//   k_pre_hull    one workgroup: the candidates sorted by index (bitonic sort in
//                 LDS), the cover by Andrew's monotone chain (the same function
//                 as the paper's sorted incremental construction), T = p + s(d') + 3
//   k_pre_good    G_p = { k : s(a_k) >= Ehat(k) - T } (eq. threshold) in exact
//                 integer arithmetic, counted per workgroup, and the least good s
//   k_pre_scan    the workgroups' offsets, |G_p|, the shift of the table
//   k_pre_table   prefix counts of G_p and the masked, shifted coefficient table
//   k_pre_sig32   (FP32 plans) per chunk, the scale of the FP32 table
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
    kNonFinite = 0, kV, kDt, kNh, kNGood, kT, kSMax, kSMinGood, kShift, kUnsupported, kInfoLen = 16
};

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct PreWs {
    int32_t *scales;   // d + 1: s(a_k), kNegInfScale for a_k = 0
    int32_t *good;     // d + 1: k in G_p
    double2 *coef;     // d + 1: a_k 2^-shift for k in G_p, else 0
    int32_t *gprefix;  // d + 2
    double *hull_k;    // cover vertices
    double *hull_s;
    long long *info;   // kInfoLen
    int32_t *ictl;     // [0] least good s
    int32_t *cmin;     // kSBins: least index of each scale (INT_MAX: none)
    int32_t *cmax;     // kSBins: largest index of each scale
    int32_t *blk_sum;  // per kPreBlock coefficients: |G_p| there
    int32_t *blk_off;  //   and its exclusive prefix
    float2 *coef32;    // d + 1 (FP32 plans): coef 2^-sig32[chunk] as FP32
    int32_t *sig32;    // chunks (FP32 plans)
};

int64_t n_chunks(int64_t d) { return d / kChunk + 1; }
int64_t n_blocks(int64_t n1) { return (n1 + kPreBlock - 1) / kPreBlock; }
int64_t hull_cap(int64_t n1) { return std::min<int64_t>(n1, kMaxCand); }

size_t pre_layout(int64_t d, uint32_t pflags, PreWs *w, void *base) {
    size_t off = 0;
    char *b = static_cast<char *>(base);
    auto take = [&](size_t bytes) { char *p = b ? b + off : nullptr; off = align_up(off + bytes); return p; };
    const int64_t n1 = d + 1, nb = n_blocks(n1);
    PreWs x;
    x.scales = (int32_t *)take(sizeof(int32_t) * n1);
    x.good = (int32_t *)take(sizeof(int32_t) * n1);
    x.coef = (double2 *)take(sizeof(double2) * n1);
    x.gprefix = (int32_t *)take(sizeof(int32_t) * (n1 + 1));
    x.hull_k = (double *)take(sizeof(double) * hull_cap(n1));
    x.hull_s = (double *)take(sizeof(double) * hull_cap(n1));
    x.info = (long long *)take(sizeof(long long) * kInfoLen);
    x.ictl = (int32_t *)take(sizeof(int32_t) * 16);
    x.cmin = (int32_t *)take(sizeof(int32_t) * kSBins);
    x.cmax = (int32_t *)take(sizeof(int32_t) * kSBins);
    x.blk_sum = (int32_t *)take(sizeof(int32_t) * nb);
    x.blk_off = (int32_t *)take(sizeof(int32_t) * nb);
    x.coef32 = nullptr;
    x.sig32 = nullptr;
    if (pflags & FPE_PRECONDITION_FP32) {
        x.coef32 = (float2 *)take(sizeof(float2) * n1);
        x.sig32 = (int32_t *)take(sizeof(int32_t) * n_chunks(d));
    }
    if (w) *w = x;
    return off;
}

__device__ __forceinline__ int64_t bitlen_d(int64_t v) {
    int64_t b = 0;
    while (v > 0) { ++b; v >>= 1; }
    return b;
}

__global__ __launch_bounds__(256) void k_pre_init(PreWs W) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < kSBins) { W.cmin[i] = INT_MAX; W.cmax[i] = INT_MIN; }
    if (i < kInfoLen) W.info[i] = 0;
    if (i < 16) W.ictl[i] = i == 0 ? INT_MAX : 0;
}

__global__ __launch_bounds__(kPreThreads) void k_pre_scale(const double2 *__restrict__ coef, int64_t n1, PreWs W) {
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
        W.scales[k] = s;
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
__global__ __launch_bounds__(kPreThreads) void k_pre_hull(PreWs W, int32_t p_bits) {
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
    if (t == 0) {
        int h = 0;
        int smax = INT_MIN;
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
        if (n > 0) {
            const int64_t v = ck[0], dt = ck[h - 1];
            const int64_t deff = dt - v;
            W.info[kV] = v;
            W.info[kDt] = dt;
            W.info[kNh] = h;
            W.info[kSMax] = smax;
            W.info[kT] = p_bits + bitlen_d(deff > 1 ? deff : 1) + 3;
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

__global__ __launch_bounds__(kPreThreads) void k_pre_good(int64_t n1, PreWs W) {
    __shared__ double s_k[kHullLds], s_s[kHullLds];
    __shared__ int32_t s_cnt[kPreThreads / kWave], s_min[kPreThreads / kWave];
    const int t = threadIdx.x;
    const int nh = (int)W.info[kNh];
    const int64_t T = W.info[kT];
    const bool in_lds = nh <= kHullLds;
    if (in_lds)
        for (int i = t; i < nh; i += kPreThreads) { s_k[i] = W.hull_k[i]; s_s[i] = W.hull_s[i]; }
    __syncthreads();
    const double *hk = in_lds ? s_k : W.hull_k;
    const double *hs = in_lds ? s_s : W.hull_s;
    int cnt = 0, smin = INT_MAX;
    for (int q = 0; q < kPrePer; ++q) {
        const int64_t k = (int64_t)blockIdx.x * kPreBlock + (int64_t)q * kPreThreads + t;
        if (k >= n1) break;
        const int32_t s = W.scales[k];
        int g = 0;
        if (s != kNegInfScale && nh > 0) {
            if (nh == 1) {
                g = 1;
            } else {
                const int i = cover_segment(hk, nh, (double)k);
                const int64_t k0 = (int64_t)hk[i], k1 = (int64_t)hk[i + 1];
                const int64_t s0 = (int64_t)hs[i], s1 = (int64_t)hs[i + 1];
                // s >= Ehat(k) - T with Ehat(k) = s0 + (s1 - s0)(k - k0)/(k1 - k0)
                g = ((int64_t)s + T - s0) * (k1 - k0) >= (s1 - s0) * (k - k0) ? 1 : 0;
            }
        }
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
__global__ __launch_bounds__(kPreThreads) void k_pre_scan(int64_t nb, PreWs W) {
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
        if (acc > 0) {
            const long long smax = W.info[kSMax], T = W.info[kT];
            const long long shift = (smax + smin) / 2;
            const long long half = 1022 - T - 64;
            W.info[kShift] = shift;
            W.info[kUnsupported] = (smax - shift > half || shift - smin > half) ? 1 : 0;
        }
    }
    __syncthreads();
    int32_t acc = part[t];
    for (int64_t b = b0; b < b1; ++b) { W.blk_off[b] = acc; acc += W.blk_sum[b]; }
}

// prefix counts of G_p (gprefix[k] = #(G_p within [0, k))) and the masked,
// shifted coefficient table
__global__ __launch_bounds__(kPreThreads) void k_pre_table(const double2 *__restrict__ coef, int64_t n1, PreWs W) {
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
            pre += g[q];
            double2 o = make_double2(0.0, 0.0);
            if (g[q]) {
                const double2 a = coef[k];
                o = make_double2(ldexp(a.x, -shift), ldexp(a.y, -shift));
            }
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
__device__ __forceinline__ double cover_at(const double *hk, const double *hs, int nh, int64_t k) {
    if (nh == 1) return hs[0];
    const int i = cover_segment(hk, nh, (double)k);
    const double k0 = hk[i], k1 = hk[i + 1];
    return hs[i] + (hs[i + 1] - hs[i]) * ((double)k - k0) / (k1 - k0);
}

__global__ __launch_bounds__(256) void k_pre_sig32(PreWs W) {
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
        if (W.good[k]) { gmax = max(gmax, W.scales[k]); gmin = min(gmin, W.scales[k]); }
    for (int o = 32; o > 0; o >>= 1) {
        gmax = max(gmax, __shfl_xor(gmax, o, kWave));
        gmin = min(gmin, __shfl_xor(gmin, o, kWave));
    }
    if (t % kWave == 0) { s_max[t / kWave] = gmax; s_min[t / kWave] = gmin; }
    __syncthreads();
    if (t == 0) {
        for (int i = 0; i < 256 / kWave; ++i) { gmax = max(gmax, s_max[i]); gmin = min(gmin, s_min[i]); }
        int32_t sg = 0;                                    // no good coefficient: entries 0
        if (gmax != INT_MIN) {
            const double emin = fmin(cover_at(W.hull_k, W.hull_s, nh, a), cover_at(W.hull_k, W.hull_s, nh, b));
            sg = ((int64_t)gmax - gmin <= 120 && (double)gmax - emin <= 99.0) ? (int32_t)(gmax - W.info[kShift])
                                                                              : kNoFp32;
        }
        W.sig32[c] = sg;
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

int64_t bitlen(int64_t v) {
    int64_t b = 0;
    while (v > 0) { ++b; v >>= 1; }
    return b;
}

}  // namespace
}  // namespace fpe

using namespace fpe;

extern "C" fpe_status fpe_precondition_workspace_size(int64_t d, int32_t p_bits, uint32_t flags,
                                                      size_t *bytes) {
    if (!bytes) return fail(FPE_ERR_INVALID_ARG, "bytes is NULL");
    if (d < 0 || d >= INT32_MAX - 2) return fail(FPE_ERR_INVALID_ARG, "degree out of range");
    if (p_bits < 1 || p_bits > 53) return fail(FPE_ERR_PRECISION, "p_bits must be in 1..53");
    if (flags & ~(uint32_t)FPE_PRECONDITION_FP32) return fail(FPE_ERR_INVALID_ARG, "unknown flag");
    if ((flags & FPE_PRECONDITION_FP32) && p_bits > 24)
        return fail(FPE_ERR_PRECISION, "FP32 window sums need p_bits <= 24");
    *bytes = pre_layout(d, flags, nullptr, nullptr);
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

    PreWs w;
    pre_layout(d, flags, &w, workspace_dev);
    const int64_t n1 = d + 1, nb = n_blocks(n1);
    const double2 *coef = reinterpret_cast<const double2 *>(coef_dev);
    const bool fp32 = (flags & FPE_PRECONDITION_FP32) != 0;

    k_pre_init<<<(kSBins + 255) / 256, 256, 0, stream>>>(w);
    k_pre_scale<<<(unsigned)nb, kPreThreads, 0, stream>>>(coef, n1, w);
    k_pre_hull<<<1, kPreThreads, 0, stream>>>(w, p_bits);
    k_pre_good<<<(unsigned)nb, kPreThreads, 0, stream>>>(n1, w);
    k_pre_scan<<<1, kPreThreads, 0, stream>>>(nb, w);
    k_pre_table<<<(unsigned)nb, kPreThreads, 0, stream>>>(coef, n1, w);
    if (fp32) {
        k_pre_sig32<<<(unsigned)n_chunks(d), 256, 0, stream>>>(w);
        k_mask32<<<(unsigned)((n1 + 255) / 256), 256, 0, stream>>>(w.coef, w.sig32, n1, w.coef32);
    }
    FPE_HIP_CHECK(hipGetLastError());
    long long info[kInfoLen];
    const int64_t cap = hull_cap(n1);
    std::vector<double> hk(cap), hs(cap);
    double2 a0 = {0.0, 0.0};
    FPE_HIP_CHECK(hipMemcpyAsync(info, w.info, sizeof(info), hipMemcpyDeviceToHost, stream));
    FPE_HIP_CHECK(hipMemcpyAsync(hk.data(), w.hull_k, sizeof(double) * cap, hipMemcpyDeviceToHost, stream));
    FPE_HIP_CHECK(hipMemcpyAsync(hs.data(), w.hull_s, sizeof(double) * cap, hipMemcpyDeviceToHost, stream));
    FPE_HIP_CHECK(hipMemcpyAsync(&a0, coef, sizeof(double2), hipMemcpyDeviceToHost, stream));
    FPE_HIP_CHECK(hipStreamSynchronize(stream));
    if (info[kNonFinite]) return fail(FPE_ERR_NONFINITE, "a coefficient is NaN or infinite");
    if (info[kUnsupported])
        return fail(FPE_ERR_UNSUPPORTED, "good coefficients span too many binary orders for FP64 windows");

    std::unique_ptr<fpe_plan_s> plan(new fpe_plan_s());
    plan->d = d;
    plan->p = p_bits;
    FPE_HIP_CHECK(hipGetDevice(&plan->device));
    plan->nh = info[kNh];
    if (plan->nh == 0) {   // P == 0
        plan->v = -1; plan->dt = -1; plan->ngood = 0; plan->T = 0; plan->smax = 0; plan->smin_good = 0;
    } else {
        plan->v = info[kV]; plan->dt = info[kDt]; plan->ngood = info[kNGood]; plan->T = info[kT];
        plan->smax = info[kSMax]; plan->smin_good = info[kSMinGood];
        for (int64_t i = 0; i < plan->nh; ++i) {
            plan->hull_k.push_back((int64_t)hk[i]);
            plan->hull_s.push_back((int64_t)hs[i]);
        }
    }
    plan->good_dev = w.good;

    DevPlan &P = plan->dev;
    P.coef = w.coef;
    P.gprefix = w.gprefix;
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
    P.a0 = a0;
    P.coef32 = fp32 ? w.coef32 : nullptr;
    P.sig32 = fp32 ? w.sig32 : nullptr;
    *out_plan = plan.release();
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
    for (int64_t i = 0; i < plan->nh; ++i) {
        if (hull_k) hull_k[i] = plan->hull_k[i];
        if (hull_s) hull_s[i] = plan->hull_s[i];
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
