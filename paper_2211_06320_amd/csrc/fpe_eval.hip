// Evaluation phase (Algorithm A_p, second block; Section 5.2 of arXiv 2211.06320)
// on gfx950.
//
// One evaluation is a chain of short kernels on one stream:
//   k_clear      zero the bin histogram and the control words
//   k_plan       per point: lambda = log2|z| (eq. defLambda), k_lambda and
//                N = max(Ehat + lambda Id) (eq. defN) by binary search over the
//                cover vertices staged in LDS, the window [l, r] (eq. def:LRN) by
//                two binary searches and a linear solve, the term count, and a
//                lambda bin for the sort
//   k_scan_bins  exclusive scan of the bin histogram (one workgroup)
//   k_scatter    counting-sort scatter: points ordered by lambda bin
//   k_groups     per group of 64 consecutive sorted points (one wavefront):
//                the union of their windows and its number of C-term chunks
//   k_scan_groups, k_tiles   the list of (group, chunk) tiles
//   k_window     persistent: one wavefront per tile.  Its 64 lanes share the
//                coefficient stream (wave-uniform index, scalar loads) and each
//                runs Horner's rule over its own part of the chunk; lanes whose
//                window is shorter are masked only at the ragged ends.  Then
//                z^lo by double-double binary powering with an exact exponent,
//                and either the final value or an exact fixed-point partial.
//   k_finalize   points whose window spans several chunks: fixed-point sum to
//                (mantissa, exponent)
//
// The paper sorts points by |z| only as a suggestion (Section 1 and Section 8.1,
// on parallelisation); here the sort is what lets a wavefront read one
// coefficient per step for all of its lanes.
#include <climits>
#include <utility>
#include <vector>

#include "fpe_internal.h"

namespace fpe {
namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// lambda bin: a monotone map of lambda onto [0, kBuckets), finest near 0 where
// windows are longest (bin width about 3.8e-5 in lambda there, 1.5e-3 at
// |lambda| = 5); |lambda| <= 1075 + 31 keeps asinh(8 lambda) below 9.8
__device__ __forceinline__ uint32_t lambda_bin(double lam) {
    double t = asinh(8.0 * lam) * (1.0 / 20.0) + 0.5;
    int b = (int)(t * (double)kBuckets);
    b = b < 0 ? 0 : (b >= kBuckets ? kBuckets - 1 : b);
    return (uint32_t)b;
}

__device__ __forceinline__ void normalise(double re, double im, long long E, double2 &m, long long &e) {
    double mx = fmax(fabs(re), fabs(im));
    if (mx == 0.0) { m = make_double2(0.0, 0.0); e = 0; return; }
    int k = exp_of(mx);
    m = make_double2(ldexp(re, -k), ldexp(im, -k));
    e = E + k;
}

__global__ void k_clear(EvalWs W) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= kBuckets) W.hist[i] = 0;
    if (i < 64) W.ctl[i] = 0;
}

__global__ __launch_bounds__(256) void k_plan(DevPlan P, const double2 *__restrict__ z, int n,
                                              double2 *__restrict__ m_out, long long *__restrict__ e_out,
                                              int32_t *__restrict__ terms, long long *__restrict__ win,
                                              EvalWs W) {
    __shared__ double s_k[kHullLds];
    __shared__ double s_s[kHullLds];
    const bool in_lds = P.nh <= kHullLds;
    if (in_lds)
        for (int i = threadIdx.x; i < P.nh; i += blockDim.x) { s_k[i] = P.hull_k[i]; s_s[i] = P.hull_s[i]; }
    __syncthreads();
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double *hk = in_lds ? s_k : P.hull_k;
    const double *hs = in_lds ? s_s : P.hull_s;

    const double2 zz = z[j];
    int32_t l = 1, r = 0, cnt = 0;
    long long wl = 0, wr = -1, er = 0;
    uint32_t key = kBuckets;
    bool done = true;
    double2 mo = make_double2(0.0, 0.0);
    long long eo = 0;
    if (!isfinite(zz.x) || !isfinite(zz.y)) {
        mo = make_double2(__builtin_nan(""), __builtin_nan(""));
    } else if (P.nh == 0) {
        // P == 0
    } else if (zz.x == 0.0 && zz.y == 0.0) {
        wl = 0; wr = 0;                                   // P(0) = a_0
        if (P.v == 0) { normalise(P.a0.x, P.a0.y, 0, mo, eo); cnt = 1; }
    } else {
        done = false;
        const int ez = exp_of(fmax(fabs(zz.x), fabs(zz.y)));
        const double xr = ldexp(zz.x, -ez), xi = ldexp(zz.y, -ez);
        const double lam = (double)ez + 0.5 * log2(fma(xr, xr, xi * xi));
        const int nh = P.nh;
        // k_lambda: Ehat + lambda Id is concave, so its vertex values rise then
        // fall; the leftmost maximiser is the first i whose next value is not larger
        int lo = 0, hi = nh - 1;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            double dF = (hs[mid + 1] - hs[mid]) + lam * (hk[mid + 1] - hk[mid]);
            if (dF <= 0.0) hi = mid; else lo = mid + 1;
        }
        const int is = lo;
        const double N = fma(lam, hk[is], hs[is]);
        const double L = N - (double)P.T;
        // left end: the crossing of the level L on the rising branch [0, is]
        double xL;
        if (fma(lam, hk[0], hs[0]) >= L) {
            xL = hk[0];
        } else {
            int a = 0, b = is;                              // F(a) < L <= F(b)
            while (b - a > 1) {
                int mid = (a + b) >> 1;
                if (fma(lam, hk[mid], hs[mid]) < L) a = mid; else b = mid;
            }
            double Fa = fma(lam, hk[a], hs[a]), Fb = fma(lam, hk[b], hs[b]);
            xL = hk[a] + (L - Fa) * (hk[b] - hk[a]) / (Fb - Fa);
        }
        // right end: the crossing on the falling branch [is, nh - 1]
        double xR;
        if (fma(lam, hk[nh - 1], hs[nh - 1]) >= L) {
            xR = hk[nh - 1];
        } else {
            int a = is, b = nh - 1;                         // F(a) >= L > F(b)
            while (b - a > 1) {
                int mid = (a + b) >> 1;
                if (fma(lam, hk[mid], hs[mid]) >= L) a = mid; else b = mid;
            }
            double Fa = fma(lam, hk[a], hs[a]), Fb = fma(lam, hk[b], hs[b]);
            xR = hk[a] + (Fa - L) * (hk[b] - hk[a]) / (Fa - Fb);
        }
        double cl = ceil(xL - kEta), cr = floor(xR + kEta);
        l = (int32_t)fmax(cl, (double)P.v);
        r = (int32_t)fmin(cr, (double)P.dt);
        wl = l; wr = r;
        cnt = P.gprefix[r + 1] - P.gprefix[l];
        er = (long long)floor(N) + 2;
        key = lambda_bin(lam);
        if (l / P.chunk != r / P.chunk) {
            unsigned long long *a = W.acc + 4 * (size_t)j;
            a[0] = 0; a[1] = 0; a[2] = 0; a[3] = 0;
        }
    }
    if (done) { m_out[j] = mo; e_out[j] = eo; }
    if (terms) terms[j] = cnt;
    if (win) { win[2 * (size_t)j] = wl; win[2 * (size_t)j + 1] = wr; }
    W.ell[j] = done ? 1 : l;
    W.rr[j] = done ? 0 : r;
    W.eref[j] = er;
    W.key[j] = key;
    atomicAdd(&W.hist[key], 1);
}

// exclusive scan of `count` ints in one workgroup of 1024 threads
__device__ void block_exclusive_scan(const int32_t *in, int32_t *out, int count, int32_t *total) {
    __shared__ int32_t part[1024];
    const int t = threadIdx.x, T = blockDim.x;
    const int per = (count + T - 1) / T;
    const int b = t * per, e = min(count, b + per);
    int32_t s = 0;
    for (int i = b; i < e; ++i) s += in[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {
        int32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - s;   // exclusive prefix of this thread's segment
    for (int i = b; i < e; ++i) { int32_t x = in[i]; out[i] = run; run += x; }
    if (t == T - 1 && total) *total = part[t];
}

__global__ __launch_bounds__(1024) void k_scan_bins(EvalWs W) {
    __shared__ int32_t tot;
    block_exclusive_scan(W.hist, W.cursor, kBuckets + 1, threadIdx.x == blockDim.x - 1 ? &tot : nullptr);
    __syncthreads();
    if (threadIdx.x == 0) W.ctl[2] = W.cursor[kBuckets];   // points with a window
}

__global__ __launch_bounds__(256) void k_scatter(EvalWs W, int n) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int pos = atomicAdd(&W.cursor[W.key[j]], 1);
    W.perm[pos] = j;
}

__global__ __launch_bounds__(256) void k_groups(DevPlan P, EvalWs W) {
    const int g = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    if (g >= W.n_groups) return;
    const int nvalid = W.ctl[2];
    const int idx = g * kWave + lane;
    int l = INT_MAX, r = INT_MIN;
    if (idx < nvalid) { int j = W.perm[idx]; l = W.ell[j]; r = W.rr[j]; }
    const int lo = wave_min(l), hi = wave_max(r);
    if (lane == 0) {
        W.glo[g] = lo;
        W.ghi[g] = hi;
        W.gtiles[g] = hi >= lo ? hi / P.chunk - lo / P.chunk + 1 : 0;
    }
}

__global__ __launch_bounds__(1024) void k_scan_groups(EvalWs W) {
    __shared__ int32_t tot;
    block_exclusive_scan(W.gtiles, W.goff, (int)W.n_groups, threadIdx.x == blockDim.x - 1 ? &tot : nullptr);
    __syncthreads();
    if (threadIdx.x == 0) {
        W.goff[W.n_groups] = tot;
        W.ctl[0] = tot;     // tiles
        W.ctl[1] = 0;       // tile cursor of k_window
    }
}

__global__ __launch_bounds__(256) void k_tiles(DevPlan P, EvalWs W) {
    const int g = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    if (g >= W.n_groups) return;
    const int cnt = W.gtiles[g], base = W.goff[g], c0 = W.glo[g] / P.chunk;
    for (int i = lane; i < cnt; i += kWave) W.tiles[base + i] = make_int2(g, c0 + i);
}

// one Horner step acc <- acc z + a_K (4 FMAs); a_K read from the table cf
#define HSTEP(K)                                              \
    do {                                                      \
        const double ar_ = cf[2 * (K)], ai_ = cf[2 * (K) + 1]; \
        double nr_ = fma(hr, zr, fma(-hi_, zi, ar_));         \
        double ni_ = fma(hr, zi, fma(hi_, zr, ai_));          \
        hr = nr_; hi_ = ni_;                                  \
    } while (0)

__global__ __launch_bounds__(256) void k_window(DevPlan P, const double2 *__restrict__ z,
                                                double2 *__restrict__ m_out, long long *__restrict__ e_out,
                                                EvalWs W) {
    const int lane = threadIdx.x % kWave;
    const int total = W.ctl[0];
    const int nvalid = W.ctl[2];
    const int C = P.chunk;
    // the coefficient table is read-only for the whole evaluation: wave-uniform
    // indices into it become scalar loads
    const_table_t cf = (const_table_t)P.coef;
    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(&W.ctl[1], 1);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, kWave));
        if (t >= total) break;
        const int2 gc = W.tiles[t];
        const int g = __builtin_amdgcn_readfirstlane(gc.x);
        const int c = __builtin_amdgcn_readfirstlane(gc.y);
        const int idx = g * kWave + lane;
        const bool valid = idx < nvalid;
        const int j = valid ? W.perm[idx] : 0;
        const int l = valid ? W.ell[j] : 1, r = valid ? W.rr[j] : 0;
        const int c0 = c * C, c1 = c0 + C - 1;
        const int lo = max(l, c0), hi = min(r, c1);
        const bool act = valid && lo <= hi;
        const int Khi = __builtin_amdgcn_readfirstlane(wave_max(act ? hi : INT_MIN));
        const int Klo = __builtin_amdgcn_readfirstlane(wave_min(act ? lo : INT_MAX));
        const int Ahi = __builtin_amdgcn_readfirstlane(wave_min(act ? hi : INT_MAX));
        const int Alo = __builtin_amdgcn_readfirstlane(wave_max(act ? lo : INT_MIN));
        // the union of the lanes' windows may have a gap at this chunk
        if (Khi < Klo) continue;
        const double2 zz = act ? z[j] : make_double2(0.0, 0.0);
        const double zr = zz.x, zi = zz.y;
        double hr = 0.0, hi_ = 0.0;
        if (Ahi >= Alo) {
            // ragged top: lanes start at their own hi
            for (int k = Khi; k > Ahi; --k) { if (k <= hi) HSTEP(k); }
            // common part: every active lane steps; wave-uniform coefficient
            int k = Ahi;
            for (; k - 3 >= Alo; k -= 4) {
                HSTEP(k); HSTEP(k - 1); HSTEP(k - 2); HSTEP(k - 3);
            }
            for (; k >= Alo; --k) HSTEP(k);
            // ragged bottom: lanes stop at their own lo
            for (int k2 = Alo - 1; k2 >= Klo; --k2) { if (k2 >= lo) HSTEP(k2); }
        } else {
            for (int k = Khi; k >= Klo; --k) { if (k >= lo && k <= hi) HSTEP(k); }
        }
        if (!act) continue;
        // multiply by z^lo: z = w 2^ez with max(|Re w|, |Im w|) in [1/2, 1)
        long long E = P.coef_shift;
        double pr = 1.0, pi = 0.0;
        if (lo > 0) {
            const int ez = exp_of(fmax(fabs(zr), fabs(zi)));
            cpow_dd(ldexp(zr, -ez), ldexp(zi, -ez), lo, pr, pi, E);
            E += (long long)lo * ez;
        }
        const double qr = fma(hr, pr, -hi_ * pi);
        const double qi = fma(hr, pi, hi_ * pr);
        if (l / C == r / C) {
            double2 m;
            long long e;
            normalise(qr, qi, E, m, e);
            m_out[j] = m;
            e_out[j] = e;
        } else {
            // exact fixed-point partial: value 2^-(eref) * 2^fix_shift, split in a
            // high word (integer part) and a low word (kFixLoBits more bits)
            long long sh = E - W.eref[j] + P.fix_shift;
            sh = sh < -2200 ? -2200 : (sh > 200 ? 200 : sh);
            const double xr = ldexp(qr, (int)sh), xi = ldexp(qi, (int)sh);
            const double hr0 = trunc(xr), hi0 = trunc(xi);
            const long long ihr = (long long)hr0, ihi = (long long)hi0;
            const long long ilr = (long long)rint(ldexp(xr - hr0, kFixLoBits));
            const long long ili = (long long)rint(ldexp(xi - hi0, kFixLoBits));
            unsigned long long *a = W.acc + 4 * (size_t)j;
            atomicAdd(a + 0, (unsigned long long)ihr);
            atomicAdd(a + 1, (unsigned long long)ilr);
            atomicAdd(a + 2, (unsigned long long)ihi);
            atomicAdd(a + 3, (unsigned long long)ili);
        }
    }
}

__global__ __launch_bounds__(256) void k_finalize(DevPlan P, int n, double2 *__restrict__ m_out,
                                                  long long *__restrict__ e_out, EvalWs W) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int l = W.ell[j], r = W.rr[j];
    if (l > r || l / P.chunk == r / P.chunk) return;
    const unsigned long long *a = W.acc + 4 * (size_t)j;
    const int f = P.fix_shift;
    const double vr = ldexp((double)(long long)a[0], -f) + ldexp((double)(long long)a[1], -f - kFixLoBits);
    const double vi = ldexp((double)(long long)a[2], -f) + ldexp((double)(long long)a[3], -f - kFixLoBits);
    double2 m;
    long long e;
    normalise(vr, vi, W.eref[j], m, e);
    m_out[j] = m;
    e_out[j] = e;
}

int g_num_cu = 0;

// instrumentation: event pairs around k_window
struct ProfileState {
    bool on = false;
    std::vector<hipEvent_t> pool;     // free events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};
ProfileState g_prof;

hipError_t prof_event(hipEvent_t *ev) {
    if (!g_prof.pool.empty()) { *ev = g_prof.pool.back(); g_prof.pool.pop_back(); return hipSuccess; }
    return hipEventCreate(ev);
}

}  // namespace

size_t eval_workspace_bytes(const DevPlan &P, int64_t n, EvalWs *ws, void *base) {
    size_t off = 0;
    char *b = static_cast<char *>(base);
    auto take = [&](size_t bytes) { char *p = b ? b + off : nullptr; off = align_up(off + bytes); return p; };
    const int64_t G = (n + kWave - 1) / kWave;
    int64_t chunks = 0;
    if (P.nh > 0) chunks = (int64_t)P.dt / P.chunk - (int64_t)P.v / P.chunk + 1;
    const int64_t cap = G * chunks;
    EvalWs w;
    w.ell = (int32_t *)take(sizeof(int32_t) * n);
    w.rr = (int32_t *)take(sizeof(int32_t) * n);
    w.eref = (long long *)take(sizeof(long long) * n);
    w.key = (uint32_t *)take(sizeof(uint32_t) * n);
    w.perm = (int32_t *)take(sizeof(int32_t) * n);
    w.acc = (unsigned long long *)take(sizeof(unsigned long long) * 4 * n);
    w.hist = (int32_t *)take(sizeof(int32_t) * (kBuckets + 1));
    w.cursor = (int32_t *)take(sizeof(int32_t) * (kBuckets + 1));
    w.glo = (int32_t *)take(sizeof(int32_t) * G);
    w.ghi = (int32_t *)take(sizeof(int32_t) * G);
    w.gtiles = (int32_t *)take(sizeof(int32_t) * G);
    w.goff = (int32_t *)take(sizeof(int32_t) * (G + 1));
    w.tiles = (int2 *)take(sizeof(int2) * (cap > 0 ? cap : 1));
    w.ctl = (int32_t *)take(sizeof(int32_t) * 64);
    w.n = n;
    w.n_groups = G;
    w.tile_cap = cap;
    if (ws) *ws = w;
    return off;
}

}  // namespace fpe

using namespace fpe;

extern "C" fpe_status fpe_eval_workspace_size(fpe_plan_t plan, int64_t n, size_t *bytes) {
    if (!plan || !bytes) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    if (n < 0 || n >= INT32_MAX) return fail(FPE_ERR_INVALID_ARG, "n out of range");
    const int64_t G = (n + kWave - 1) / kWave;
    int64_t chunks = plan->nh > 0 ? plan->dev.dt / plan->dev.chunk - plan->dev.v / plan->dev.chunk + 1 : 0;
    if (G * chunks >= INT32_MAX) return fail(FPE_ERR_UNSUPPORTED, "too many (point group, chunk) tiles");
    *bytes = eval_workspace_bytes(plan->dev, n, nullptr, nullptr);
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_eval(fpe_plan_t plan, const double *z_dev, int64_t n, double *m_dev,
                               int64_t *e_dev, int32_t *terms_dev, int64_t *window_dev,
                               void *workspace_dev, size_t workspace_bytes, hipStream_t stream) {
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    size_t need = 0;
    fpe_status st = fpe_eval_workspace_size(plan, n, &need);
    if (st != FPE_OK) return st;
    if (n == 0) { set_error(""); return FPE_OK; }
    if (!z_dev || !m_dev || !e_dev || !workspace_dev) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    if (workspace_bytes < need)
        return fail(FPE_ERR_WORKSPACE, "eval workspace too small: need " + std::to_string(need));
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0 || reinterpret_cast<uintptr_t>(z_dev) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(m_dev) % 16 != 0)
        return fail(FPE_ERR_INVALID_ARG, "misaligned buffer");
    EvalWs W;
    eval_workspace_bytes(plan->dev, n, &W, workspace_dev);
    const DevPlan &P = plan->dev;
    const double2 *z = reinterpret_cast<const double2 *>(z_dev);
    double2 *m = reinterpret_cast<double2 *>(m_dev);
    long long *e = reinterpret_cast<long long *>(e_dev);
    long long *win = reinterpret_cast<long long *>(window_dev);
    const int ni = (int)n;
    const unsigned pb = (unsigned)((n + 255) / 256);
    const unsigned gb = (unsigned)((W.n_groups + 3) / 4);

    if (g_num_cu == 0) {
        int dev = 0;
        FPE_HIP_CHECK(hipGetDevice(&dev));
        FPE_HIP_CHECK(hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev));
        if (g_num_cu <= 0) g_num_cu = 256;
    }
    k_clear<<<(kBuckets + 1 + 255) / 256, 256, 0, stream>>>(W);
    k_plan<<<pb, 256, 0, stream>>>(P, z, ni, m, e, terms_dev, win, W);
    if (P.nh > 0) {
        k_scan_bins<<<1, 1024, 0, stream>>>(W);
        k_scatter<<<pb, 256, 0, stream>>>(W, ni);
        k_groups<<<gb, 256, 0, stream>>>(P, W);
        k_scan_groups<<<1, 1024, 0, stream>>>(W);
        k_tiles<<<gb, 256, 0, stream>>>(P, W);
        const int64_t want = (W.tile_cap + 3) / 4;
        const unsigned wb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)g_num_cu * 8));
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (g_prof.on) {
            FPE_HIP_CHECK(prof_event(&ev0));
            FPE_HIP_CHECK(prof_event(&ev1));
            FPE_HIP_CHECK(hipEventRecord(ev0, stream));
        }
        k_window<<<wb, 256, 0, stream>>>(P, z, m, e, W);
        if (g_prof.on) {
            FPE_HIP_CHECK(hipEventRecord(ev1, stream));
            g_prof.pending.emplace_back(ev0, ev1);
        }
        k_finalize<<<pb, 256, 0, stream>>>(P, ni, m, e, W);
    }
    FPE_HIP_CHECK(hipGetLastError());
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_profile_enable(int32_t on) {
    g_prof.on = on != 0;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_profile_read(double *window_ms, int64_t *launches) {
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto &pr : g_prof.pending) {
        FPE_HIP_CHECK(hipEventSynchronize(pr.second));
        float ms = 0.0f;
        FPE_HIP_CHECK(hipEventElapsedTime(&ms, pr.first, pr.second));
        tot += ms;
        ++cnt;
        g_prof.pool.push_back(pr.first);
        g_prof.pool.push_back(pr.second);
    }
    g_prof.pending.clear();
    if (window_ms) *window_ms = tot;
    if (launches) *launches = cnt;
    set_error("");
    return FPE_OK;
}
