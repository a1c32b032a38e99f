// Preconditioning (Algorithm A_p, first block; Section 5.1 of arXiv 2211.06320).
//
// Device: the scale s(a_k) = 1 + floor(log2|a_k|) of every coefficient
// (Section 2.3, eq. dsz), decided exactly with 64-bit integer arithmetic on the
// significands, and the masked/scaled coefficient table.
// Host: the concave cover of k -> s(a_k) by Andrew's monotone chain over the
// abscissae (O(d), same function as the paper's sorted incremental
// construction), and the good set G_p = { k : s(a_k) >= Ehat(k) - T } (eq.
// threshold) decided in exact integer arithmetic.
#include <algorithm>
#include <cstring>
#include <memory>

#include "fpe_internal.h"

namespace fpe {
namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct PreWs {
    int32_t *scales;   // d + 1: s(a_k); later reused for the good flags
    double2 *coef;     // d + 1: a_k 2^-shift for k in G_p, else 0
    int32_t *gprefix;  // d + 2
    double *hull_k;    // d + 1
    double *hull_s;    // d + 1
    int32_t *flags;    // [0] non-finite coefficient seen
    float2 *coef32;    // d + 1 (FP32 plans): coef 2^-sig32[chunk] as FP32
    int32_t *sig32;    // chunks (FP32 plans)
};

int64_t n_chunks(int64_t d) { return d / kChunk + 1; }

size_t pre_layout(int64_t d, uint32_t pflags, PreWs *w, void *base) {
    size_t off = 0;
    char *b = static_cast<char *>(base);
    auto take = [&](size_t bytes) { char *p = b ? b + off : nullptr; off = align_up(off + bytes); return p; };
    int64_t n1 = d + 1;
    int32_t *scales = (int32_t *)take(sizeof(int32_t) * n1);
    double2 *coef = (double2 *)take(sizeof(double2) * n1);
    int32_t *gprefix = (int32_t *)take(sizeof(int32_t) * (n1 + 1));
    double *hk = (double *)take(sizeof(double) * n1);
    double *hs = (double *)take(sizeof(double) * n1);
    int32_t *flags = (int32_t *)take(sizeof(int32_t) * 64);
    float2 *coef32 = nullptr;
    int32_t *sig32 = nullptr;
    if (pflags & FPE_PRECONDITION_FP32) {
        coef32 = (float2 *)take(sizeof(float2) * n1);
        sig32 = (int32_t *)take(sizeof(int32_t) * n_chunks(d));
    }
    if (w) *w = {scales, coef, gprefix, hk, hs, flags, coef32, sig32};
    return off;
}

// s(x + iy) exactly.  With a = max(|x|, |y|) = A 2^(m-53), b = min = B 2^(mb-53),
// A, B < 2^53 integers and m = exponent of a (so s(a) = m), s(z) = m + 1 iff
// x^2 + y^2 >= 4^m iff A^2 + B^2 4^(mb-m) >= 2^106.  The 106-bit squares are
// formed from 64-bit halves; the floor of the shifted smaller square cannot
// change the comparison because A^2 and 2^106 are integers.
__device__ int32_t scale_exact(double x, double y) {
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

__global__ void k_scale(const double2 *__restrict__ coef, int64_t n, int32_t *__restrict__ s,
                        int32_t *__restrict__ flags) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double2 a = coef[k];
    if (!isfinite(a.x) || !isfinite(a.y)) {
        flags[0] = 1;
        s[k] = kNegInfScale;
        return;
    }
    s[k] = scale_exact(a.x, a.y);
}

__global__ void k_mask(const double2 *__restrict__ coef, const int32_t *__restrict__ good,
                       int64_t n, int shift, double2 *__restrict__ out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double2 a = coef[k];
    double2 o = {0.0, 0.0};
    if (good[k]) { o.x = ldexp(a.x, -shift); o.y = ldexp(a.y, -shift); }
    out[k] = o;
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
    const int64_t n1 = d + 1;
    const double2 *coef = reinterpret_cast<const double2 *>(coef_dev);
    const int threads = 256;
    const unsigned blocks = (unsigned)((n1 + threads - 1) / threads);

    FPE_HIP_CHECK(hipMemsetAsync(w.flags, 0, sizeof(int32_t) * 64, stream));
    k_scale<<<blocks, threads, 0, stream>>>(coef, n1, w.scales, w.flags);
    FPE_HIP_CHECK(hipGetLastError());
    std::vector<int32_t> s(n1);
    int32_t hflags[64];
    FPE_HIP_CHECK(hipMemcpyAsync(s.data(), w.scales, sizeof(int32_t) * n1, hipMemcpyDeviceToHost, stream));
    FPE_HIP_CHECK(hipMemcpyAsync(hflags, w.flags, sizeof(hflags), hipMemcpyDeviceToHost, stream));
    double2 a0 = {0.0, 0.0};
    FPE_HIP_CHECK(hipMemcpyAsync(&a0, coef, sizeof(double2), hipMemcpyDeviceToHost, stream));
    FPE_HIP_CHECK(hipStreamSynchronize(stream));
    if (hflags[0]) return fail(FPE_ERR_NONFINITE, "a coefficient is NaN or infinite");

    std::unique_ptr<fpe_plan_s> plan(new fpe_plan_s());
    plan->d = d;
    plan->p = p_bits;
    plan->good.assign(n1, 0);
    FPE_HIP_CHECK(hipGetDevice(&plan->device));

    // trimmed range [v, dt]
    int64_t v = 0;
    while (v < n1 && s[v] == kNegInfScale) ++v;
    int64_t dt = n1 - 1;
    while (dt >= v && s[dt] == kNegInfScale) --dt;

    std::vector<int32_t> goodflag(n1, 0);
    std::vector<int32_t> prefix(n1 + 1, 0);
    std::vector<double> hk, hs;
    std::vector<int32_t> sig32;
    int64_t shift = 0;
    if (v >= n1) {  // P == 0
        plan->v = -1; plan->dt = -1; plan->nh = 0; plan->ngood = 0; plan->T = 0;
        plan->smax = 0; plan->smin_good = 0;
    } else {
        // Andrew's monotone chain: upper hull of (k, s_k) over nonzero a_k,
        // scanning k upwards; a point is popped while the last turn is not
        // strictly clockwise (collinear vertices are dropped).
        std::vector<int64_t> ck, cs;
        for (int64_t k = v; k <= dt; ++k) {
            if (s[k] == kNegInfScale) continue;
            int64_t sk = s[k];
            while (ck.size() >= 2) {
                size_t t = ck.size();
                int64_t ax = ck[t - 2], ay = cs[t - 2], bx = ck[t - 1], by = cs[t - 1];
                int64_t cross = (bx - ax) * (sk - ay) - (by - ay) * (k - ax);
                if (cross >= 0) { ck.pop_back(); cs.pop_back(); } else break;
            }
            ck.push_back(k);
            cs.push_back(sk);
        }
        const int64_t deff = dt - v;
        const int64_t T = p_bits + bitlen(deff > 1 ? deff : 1) + 3;
        // good set: on the segment [k_i, k_{i+1}], Ehat(k) = s_i + (s_{i+1} - s_i)(k - k_i)/(k_{i+1} - k_i)
        int64_t ngood = 0, smax = INT64_MIN, smin = INT64_MAX;
        size_t seg = 0;
        for (int64_t k = v; k <= dt; ++k) {
            if (s[k] == kNegInfScale) continue;
            bool g;
            if (ck.size() == 1) {
                g = true;
            } else {
                while (seg + 2 < ck.size() && ck[seg + 1] < k) ++seg;
                int64_t k0 = ck[seg], k1 = ck[seg + 1], s0 = cs[seg], s1 = cs[seg + 1];
                g = (s[k] + T - s0) * (k1 - k0) >= (s1 - s0) * (k - k0);
            }
            if (g) {
                goodflag[k] = 1;
                ++ngood;
                smin = std::min<int64_t>(smin, s[k]);
            }
            smax = std::max<int64_t>(smax, s[k]);
        }
        // the window sum holds a_k z^(k - lo) in FP64: its terms span
        // [smin - T, smax + T] binary orders after a shift of the coefficients
        // by 2^-shift, which must fit the FP64 exponent range with margin
        shift = (smax + smin) / 2;
        const int64_t half = 1022 - T - 64;
        if (smax - shift > half || shift - smin > half) {
            return fail(FPE_ERR_UNSUPPORTED, "good coefficients span too many binary orders for FP64 windows");
        }
        for (int64_t k = 0; k < n1; ++k) prefix[k + 1] = prefix[k] + goodflag[k];
        if (flags & FPE_PRECONDITION_FP32) {
            // per chunk: sigma = the largest good scale (FP32 entries below 1 in
            // modulus), FP32 only if every good entry stays a normal FP32
            // number with margin (sigma - min good s <= 120) and the cover drops
            // by at most 99 within the chunk (then a block partial of any point
            // that matters stays above the FP32 range floor)
            const int64_t nch = n_chunks(d);
            sig32.assign(nch, kNoFp32);
            auto ehat = [&](int64_t k) {        // the cover at k in [v, dt]
                if (ck.size() == 1) return (double)cs[0];
                size_t i = std::upper_bound(ck.begin(), ck.end(), k) - ck.begin();
                if (i == 0) i = 1;
                if (i >= ck.size()) i = ck.size() - 1;
                const double k0 = (double)ck[i - 1], k1 = (double)ck[i];
                return (double)cs[i - 1] + (double)(cs[i] - cs[i - 1]) * ((double)k - k0) / (k1 - k0);
            };
            for (int64_t c = 0; c < nch; ++c) {
                const int64_t a = std::max<int64_t>(c * kChunk, v), b = std::min<int64_t>(c * kChunk + kChunk - 1, dt);
                if (a > b) { sig32[c] = 0; continue; }          // no coefficient of the trimmed range
                int64_t gmax = INT64_MIN, gmin = INT64_MAX;
                for (int64_t k = a; k <= b; ++k)
                    if (goodflag[k]) { gmax = std::max<int64_t>(gmax, s[k]); gmin = std::min<int64_t>(gmin, s[k]); }
                if (gmax == INT64_MIN) { sig32[c] = 0; continue; }   // no good coefficient: entries 0
                const double emin = std::min(ehat(a), ehat(b));      // concave: least at an end
                if (gmax - gmin <= 120 && (double)gmax - emin <= 99.0) sig32[c] = (int32_t)(gmax - shift);
            }
        }
        hk.assign(ck.begin(), ck.end());
        hs.assign(cs.begin(), cs.end());
        plan->v = v; plan->dt = dt; plan->nh = (int64_t)ck.size(); plan->ngood = ngood; plan->T = T;
        plan->smax = smax; plan->smin_good = smin;
        plan->hull_k = ck; plan->hull_s = cs;
        for (int64_t k = 0; k < n1; ++k) plan->good[k] = (uint8_t)goodflag[k];
    }

    if (plan->nh > 0) {
        FPE_HIP_CHECK(hipMemcpyAsync(w.hull_k, hk.data(), sizeof(double) * hk.size(), hipMemcpyHostToDevice, stream));
        FPE_HIP_CHECK(hipMemcpyAsync(w.hull_s, hs.data(), sizeof(double) * hs.size(), hipMemcpyHostToDevice, stream));
    }
    FPE_HIP_CHECK(hipMemcpyAsync(w.gprefix, prefix.data(), sizeof(int32_t) * (n1 + 1), hipMemcpyHostToDevice, stream));
    FPE_HIP_CHECK(hipMemcpyAsync(w.scales, goodflag.data(), sizeof(int32_t) * n1, hipMemcpyHostToDevice, stream));
    k_mask<<<blocks, threads, 0, stream>>>(coef, w.scales, n1, (int)shift, w.coef);
    FPE_HIP_CHECK(hipGetLastError());
    if (flags & FPE_PRECONDITION_FP32) {
        if (sig32.empty()) sig32.assign(n_chunks(d), kNoFp32);      // P == 0
        FPE_HIP_CHECK(hipMemcpyAsync(w.sig32, sig32.data(), sizeof(int32_t) * sig32.size(), hipMemcpyHostToDevice,
                                     stream));
        k_mask32<<<blocks, threads, 0, stream>>>(w.coef, w.sig32, n1, w.coef32);
        FPE_HIP_CHECK(hipGetLastError());
    }
    FPE_HIP_CHECK(hipStreamSynchronize(stream));

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
    const int64_t wmax = std::max<int64_t>(plan->dt - plan->v + 1, 1);
    // (counted for the shortest chunk an evaluation may choose)
    const int64_t chunks = std::max<int64_t>(plan->dt / kChunkMin - plan->v / kChunkMin + 1, 1);
    P.fix_shift = (int32_t)(60 - bitlen(wmax));
    P.fix_lo = (int32_t)std::min<int64_t>(44, 62 - bitlen(chunks));
    P.coef_shift = (int32_t)shift;
    P.a0 = a0;
    P.coef32 = (flags & FPE_PRECONDITION_FP32) ? w.coef32 : nullptr;
    P.sig32 = (flags & FPE_PRECONDITION_FP32) ? w.sig32 : nullptr;
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
    if (good) std::memcpy(good, plan->good.data(), plan->good.size());
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_plan_destroy(fpe_plan_t plan) {
    delete plan;
    set_error("");
    return FPE_OK;
}
