// Evaluation phase (Algorithm A_p, second block; Section 5.2 of arXiv 2211.06320)
// on gfx950.
//
// One evaluation is a chain of short kernels on one stream; device-scope
// atomics serve only list counters and the integer accumulators of the few
// long split groups (exact sums, so their order does not matter):
//
//   k_bounds     per point: lambda = log2|z| (eq. defLambda), k_lambda and
//                N = max(Ehat + lambda Id) (eq. defN) by binary search over the
//                cover vertices staged in LDS, the window [l, r] (eq. def:LRN) by
//                two binary searches and a linear solve, the term count, a
//                reference exponent and a lambda bin (the window and the
//                exponent written in input order); per sort block of 2048 points, LDS counters
//                give each point its rank within its bin and the block's row of
//                the (block x bin) count table
//   k_scan_table exclusive scan of the count table in bin-major order
//   k_scatter    counting-sort scatter into lambda-bin order, one thread per
//                point: a 32-byte record {z, window, input index} per point
//   k_groups     per group of 64 consecutive sorted points (one wavefront):
//                the union of their windows and the work of its C-term chunks
//   k_scan_seg, k_partition   an equal-work partition of the (group, chunk)
//                tiles over the window kernel's wavefronts, and the lists of
//                groups split across wavefronts (few owners / many owners)
//   k_window     every wavefront runs its contiguous range of tiles.  The 64
//                lanes of a tile share the coefficient stream (wave-uniform
//                index, scalar loads two batches in flight) and each runs
//                Horner's rule over its own part of the chunk; lanes whose
//                window is shorter are masked only at the ragged ends.  Then
//                z^lo by double-double binary powering with an exact exponent.
//                A window inside one chunk is written out at once; the chunk
//                partials of longer windows are summed exactly in fixed point,
//                in LDS while the wavefront stays on the group, in the
//                wavefront's slots otherwise
//   k_finalize   windows of groups split across wavefronts: the sum of the
//                wavefronts' fixed-point partials, to (mantissa, exponent); a
//                wavefront per group with a few owners, 32-owner pieces with
//                atomic accumulation for groups with many
//
// fpe_cancelled_bits (k_cancel) reports, per point and for a value standing
// for P(z), an upper bound of the cancelled bits c of eq. (def_prec_loss).
//
// Every chunk partial is computed the same way whichever wavefront runs it and
// fixed-point sums are exact, so FP64 results do not depend on the partition or
// on which points share a wavefront.  (With an FP32 table, which part of a tile
// runs FP32 blocks depends on the tile's other lanes, so those last bits vary
// with the order the sort leaves open, within the FP32 bound.)  The paper only
// suggests ordering points by |z| and evaluating points of similar size
// together (Section 1; Section 8.1 on parallelisation); here the order is what
// lets a wavefront read one coefficient per step for all of its lanes.
#include <algorithm>
#include <climits>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "fpe_internal.h"

namespace fpe {
namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr int kBins = 2048;            // lambda bins; bin kBins holds finished points
constexpr int kBoundsThreads = 1024;
constexpr int kPerThread = 2;          // points per k_bounds thread
constexpr int kSortPoints = kBoundsThreads * kPerThread;   // points per sort block (one k_bounds block)
constexpr int kSeg = 4096;             // scan segment

// lambda bin: a monotone map of lambda onto [0, kBins), finest near 0 where the
// windows of a flat cover are longest and vary fastest (a sort by this key loses
// less than 1 % of lane efficiency against an exact sort by lambda on the
// uniform and wide-range workloads); |lambda| <= 1106 keeps asinh below 14.6
__device__ __forceinline__ int lambda_bin(double lam) {
    // asinh in FP32 (the key only orders points; rounding that breaks ties
    // differently changes which points share a wavefront, not any result)
    const float x = (float)(1024.0 * lam), ax = fabsf(x);
    const float a = __logf(ax + __fsqrt_rn(fmaf(ax, ax, 1.0f)));
    const float t = copysignf(a, x) * (1.0f / 34.0f) + 0.5f;
    const int b = (int)(t * (float)kBins);
    return b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
}

__device__ __forceinline__ void normalise(double re, double im, long long E, double2 &m, long long &e) {
    double mx = fmax(fabs(re), fabs(im));
    if (mx == 0.0) { m = make_double2(0.0, 0.0); e = 0; return; }
    int k = exp_of(mx);
    m = make_double2(ldexp(re, -k), ldexp(im, -k));
    e = E + k;
}

// The smallest / largest value over the 64 lanes, in every lane: the gfx950
// half swaps (v_permlane32_swap: lanes 32..63 of one operand with lanes 0..31
// of the other; v_permlane16_swap: odd rows with even rows) leave in each row
// the extremes over lanes i, i + 16, i + 32, i + 48, and DPP row shifts take
// the row's extreme into its lane 15 (no LDS crossbar round trips).  Every
// lane of the wavefront must be active.
template <bool MAX>
__device__ __forceinline__ int wave_ext(int v) {
    auto ext = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    v = ext((int)r[0], (int)r[1]);
    r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    v = ext((int)r[0], (int)r[1]);
    constexpr int id = MAX ? INT_MIN : INT_MAX;
    v = ext(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = ext(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = ext(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = ext(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false));   // row_shr:8
    return __builtin_amdgcn_readlane(v, 15);
}
__device__ __forceinline__ int wave_min(int v) { return wave_ext<false>(v); }
__device__ __forceinline__ int wave_max(int v) { return wave_ext<true>(v); }

// global exclusive prefix of the finished-points bin = number of points with a window
__device__ __forceinline__ int valid_points(const EvalWs &W) {
    if (W.n_slots >= 0) return (int)W.n_slots;      // a batch: every slot, padding included
    const int64_t idx = (int64_t)kBins * W.n_sort_blocks;
    return W.tscan[idx] + W.bin_off[kBins / W.tab_ib];
}

// Per point: lambda = log2|z| (eq. defLambda), k_lambda and N = max(Ehat +
// lambda Id) (eq. defN) by binary search over the cover vertices, the window
// [l, r] (eq. def:LRN) by two binary searches and a linear solve, the reference
// exponent and the lambda bin.  Points with no window (z = 0, a non-finite z,
// P == 0) get their value here and the bin kBins.  Returns the bin.
// lambda = log2|z| (eq. defLambda) for a finite nonzero z: |z| = |w| 2^ez with
// max(|Re w|, |Im w|) in [1/2, 1) (an exact rescaling), so no square overflows
__device__ __forceinline__ double log2_abs(double2 zz) {
    const int ez = exp_of(fmax(fabs(zz.x), fabs(zz.y)));
    const double xr = ldexp(zz.x, -ez), xi = ldexp(zz.y, -ez);
    return (double)ez + 0.5 * log2(fma(xr, xr, xi * xi));
}

// k_lambda (eq. defN): Ehat + lambda Id is concave, so its vertex values rise
// then fall; the leftmost maximiser is the first vertex whose next value is
// not larger (binary search over the nh >= 1 cover vertices)
template <class HP>
__device__ __forceinline__ int cover_argmax(int nh, HP hk, HP hs, double lam) {
    int lo = 0, hi = nh - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        double dF = (hs[mid + 1] - hs[mid]) + lam * (hk[mid + 1] - hk[mid]);
        if (dF <= 0.0) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// The cover vertices (hk, hs) are read through an LDS-typed pointer when they
// fit in LDS (ds_read, one short wait per search step) and through a global
// pointer otherwise; through a generic pointer every search step would be a
// flat load, waiting on both the memory and the LDS counter.
#if defined(__HIP_DEVICE_COMPILE__)
#define FPE_LDS_AS __attribute__((address_space(3)))
#else
#define FPE_LDS_AS
#endif
typedef const FPE_LDS_AS double *lds_table_t;

template <class HP>
__device__ __forceinline__ int bounds_point(const DevPlan &P, HP hk, HP hs,
                                            const double2 *__restrict__ z, int j, double2 *__restrict__ m_out,
                                            long long *__restrict__ e_out, double2 *__restrict__ md_out,
                                            long long *__restrict__ ed_out, int32_t *__restrict__ terms,
                                            long long *__restrict__ win, const EvalWs &W) {
    const int nh = P.nh;
    const double2 zz = z[j];
    int32_t l = 1, r = 0, cnt = 0;                     // l > r: no window for the window kernel
    long long wl = 0, wr = -1, er = 0;                 // reported window
    int key = kBins;
    bool done = true;
    double2 mo = make_double2(0.0, 0.0);
    long long eo = 0;
    if (!isfinite(zz.x) || !isfinite(zz.y)) {
        mo = make_double2(__builtin_nan(""), __builtin_nan(""));
    } else if (nh == 0) {
        // P == 0
    } else if (zz.x == 0.0 && zz.y == 0.0) {
        wl = 0; wr = 0;                                // P(0) = a_0
        if (P.v == 0) { normalise(P.a0.x, P.a0.y, 0, mo, eo); cnt = 1; }
    } else {
        done = false;
        const double lam = log2_abs(zz);
        const int is = cover_argmax(nh, hk, hs, lam);
        const double N = fma(lam, hk[is], hs[is]);
        const double L = N - (double)P.T;
        // left end: the crossing of the level L on the rising branch [0, is]
        double xL;
        if (fma(lam, hk[0], hs[0]) >= L) {
            xL = hk[0];
        } else {
            int a = 0, c = is;                          // F(a) < L <= F(c)
            while (c - a > 1) {
                int mid = (a + c) >> 1;
                if (fma(lam, hk[mid], hs[mid]) < L) a = mid; else c = mid;
            }
            double Fa = fma(lam, hk[a], hs[a]), Fc = fma(lam, hk[c], hs[c]);
            xL = hk[a] + (L - Fa) * (hk[c] - hk[a]) / (Fc - Fa);
        }
        // right end: the crossing on the falling branch [is, nh - 1]
        double xR;
        if (fma(lam, hk[nh - 1], hs[nh - 1]) >= L) {
            xR = hk[nh - 1];
        } else {
            int a = is, c = nh - 1;                     // F(a) >= L > F(c)
            while (c - a > 1) {
                int mid = (a + c) >> 1;
                if (fma(lam, hk[mid], hs[mid]) >= L) a = mid; else c = mid;
            }
            double Fa = fma(lam, hk[a], hs[a]), Fc = fma(lam, hk[c], hs[c]);
            xR = hk[a] + (Fa - L) * (hk[c] - hk[a]) / (Fa - Fc);
        }
        l = (int32_t)fmax(ceil(xL - kEta), (double)P.v);
        r = (int32_t)fmin(floor(xR + kEta), (double)P.dt);
        wl = l; wr = r;
        if (terms) cnt = P.gprefix[r + 1] - P.gprefix[l];
        er = (long long)floor(N) + 2;
        key = lambda_bin(lam);
    }
    if (done && m_out) {
        m_out[j] = mo;
        e_out[j] = eo;
        // the kept terms of a finished point are at most a_0: derivative 0
        // (NaN for a non-finite z)
        if (md_out) { md_out[j] = mo.x != mo.x ? mo : make_double2(0.0, 0.0); ed_out[j] = 0; }
    }
    if (terms) terms[j] = cnt;
    if (win) { win[2 * (size_t)j] = wl; win[2 * (size_t)j + 1] = wr; }
    W.lr[j] = make_int2(l, r);
    W.eref[j] = er;
    return key;
}

// the record the window kernel reads for point j, built where the sort moves
// it: z from the caller's points, the window from k_bounds
__device__ __forceinline__ PointRec point_rec(const double2 *__restrict__ z, const EvalWs &W, int j) {
    PointRec rc;
    rc.z = z[j];
    const int2 lr = W.lr[j];
    rc.l = lr.x;
    rc.r = lr.y;
    rc.j = j;
    rc.pad = 0;
    return rc;
}

// One sort block of kSortPoints consecutive points per workgroup: the points'
// bounds and bins, each point's rank among the block's points of its bin (LDS
// counters), and the block's bin counts, written as one row of the
// (block x bin) count table.
__global__ __launch_bounds__(kBoundsThreads) void k_bounds(DevPlan P, const double2 *__restrict__ z, int n,
                                                           double2 *__restrict__ m_out,
                                                           long long *__restrict__ e_out,
                                                           double2 *__restrict__ md_out,
                                                           long long *__restrict__ ed_out,
                                                           int32_t *__restrict__ terms,
                                                           long long *__restrict__ win, EvalWs W) {
    __shared__ double s_k[kHullLds];
    __shared__ double s_s[kHullLds];
    __shared__ int32_t hist[kBins + 1];
    const int t = threadIdx.x, b = blockIdx.x;
    if (b == 0 && t < 64) W.ctl[t] = 0;               // totals and counters of the later kernels
    const bool in_lds = P.nh <= kHullLds;
    if (in_lds)
        for (int i = t; i < P.nh; i += kBoundsThreads) { s_k[i] = P.hull_k[i]; s_s[i] = P.hull_s[i]; }
    for (int i = t; i <= kBins; i += kBoundsThreads) hist[i] = 0;
    __syncthreads();
    auto run = [&](auto hk, auto hs) {
#pragma unroll
        for (int it = 0; it < kPerThread; ++it) {
            const int j = b * kSortPoints + it * kBoundsThreads + t;
            if (j < n) {
                const int key = bounds_point(P, hk, hs, z, j, m_out, e_out, md_out, ed_out, terms, win, W);
                const int rank = atomicAdd(&hist[key], 1);  // LDS
                W.keyrank[j] = key * kSortPoints + rank;
            }
        }
    };
    if (in_lds) run((lds_table_t)s_k, (lds_table_t)s_s);
    else run((const double *)P.hull_k, (const double *)P.hull_s);
    __syncthreads();
    for (int i = t; i <= kBins; i += kBoundsThreads) W.table[(size_t)b * (kBins + 1) + i] = hist[i];
}

// Exclusive scan of int32 values in segments of kSeg = 4096 (1024 threads x 4).
// Every block scans its segment and writes the segment-local exclusive prefix
// to out and the segment total to seg_sum; k_scan_sums then scans the totals
// into seg_off.  A global prefix is out[i] + seg_off[i / kSeg].
// v: this thread's 4 consecutive values (zero past n); out: the segment's output.
__device__ int32_t block_scan4(const int32_t v[4], int32_t *out, int n, int32_t carry) {
    __shared__ int32_t wsum[16];
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const int i0 = 4 * t;
    const int32_t s1 = v[0] + v[1], s2 = s1 + v[2], tot = s2 + v[3];
    int32_t x = tot;
    for (int o = 1; o < kWave; o <<= 1) {
        int32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[wave] = x;
    __syncthreads();
    if (wave == 0) {
        int32_t w = lane < 16 ? wsum[lane] : 0;
        for (int o = 1; o < 16; o <<= 1) {
            int32_t y = __shfl_up(w, o, kWave);
            if (lane >= o) w += y;
        }
        if (lane < 16) wsum[lane] = w;
    }
    __syncthreads();
    const int32_t excl = carry + (wave ? wsum[wave - 1] : 0) + x - tot;
    const int32_t pre[4] = {excl, excl + v[0], excl + s1, excl + s2};
    for (int k = 0; k < 4; ++k)
        if (i0 + k < n) out[i0 + k] = pre[k];
    const int32_t block_total = wsum[15];
    __syncthreads();
    return block_total;
}

__device__ __forceinline__ void load4(const int32_t *in, int n, int32_t v[4]) {
    const int i0 = 4 * threadIdx.x;
    if (i0 + 3 < n && ((reinterpret_cast<uintptr_t>(in) & 15) == 0)) {
        const int4 q = reinterpret_cast<const int4 *>(in)[threadIdx.x];
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
        for (int k = 0; k < 4; ++k) v[k] = (i0 + k < n) ? in[i0 + k] : 0;
    }
}

__global__ __launch_bounds__(1024) void k_scan_seg(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                   int64_t count, int32_t *__restrict__ seg_sum) {
    const int64_t base = (int64_t)blockIdx.x * kSeg;
    const int n = (int)min((int64_t)kSeg, count - base);
    int32_t v[4];
    load4(in + base, n, v);
    const int32_t tot = block_scan4(v, out + base, n, 0);
    if (threadIdx.x == 0) seg_sum[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the nseg segment totals into seg_off, and
// the grand total.  (A separate launch rather than a last-workgroup ticket: a
// device-scope fence between workgroups would have to write back the L2 of
// each XCD.)
__global__ __launch_bounds__(1024) void k_scan_sums(const int32_t *__restrict__ seg_sum, int nseg,
                                                    int32_t *__restrict__ seg_off, int32_t *__restrict__ total) {
    int32_t carry = 0;
    for (int s0 = 0; s0 < nseg; s0 += kSeg) {
        int32_t v[4];
        load4(seg_sum + s0, min(kSeg, nseg - s0), v);
        carry += block_scan4(v, seg_off + s0, min(kSeg, nseg - s0), carry);
    }
    if (threadIdx.x == 0) *total = carry;
}

// The count table is stored by block (row b holds the block's kBins + 1 bin
// counts) and scanned in bin-major order, entry (bin i, block b) at position
// i NB + b: all points of bin 0, block by block, then bin 1, ...  Workgroup s
// scans the bins [s Ib, (s + 1) Ib), Ib = max(1, kSeg / NB): it reads each
// block row's Ib counts as one piece (coalesced) into LDS in bin-major order,
// in passes of at most kSeg entries (several only when NB > kSeg).  A global
// prefix is tscan[i NB + b] + bin_off[i / Ib].
__global__ __launch_bounds__(1024) void k_scan_table(EvalWs W) {
    __shared__ int32_t tile[kSeg];
    const int NB = (int)W.n_sort_blocks, K1 = kBins + 1, Ib = W.tab_ib;
    const int i0 = blockIdx.x * Ib, ni = min(Ib, K1 - i0);
    const int rows = kSeg / ni;                        // block rows per pass
    int32_t carry = 0;
    for (int b0 = 0; b0 < NB; b0 += rows) {
        const int nb = min(rows, NB - b0), cnt = ni * nb;
        for (int idx = threadIdx.x; idx < cnt; idx += 1024) {
            const int b = idx / ni, ii = idx % ni;
            tile[ii * nb + b] = W.table[(size_t)(b0 + b) * K1 + i0 + ii];
        }
        __syncthreads();
        int32_t v[4];
        for (int k = 0; k < 4; ++k) v[k] = 4 * (int)threadIdx.x + k < cnt ? tile[4 * threadIdx.x + k] : 0;
        // one pass covers whole bins (nb == NB) or one bin (ni == 1): contiguous output
        carry += block_scan4(v, W.tscan + (size_t)i0 * NB + b0, cnt, carry);
    }
    if (threadIdx.x == 0) W.bin_sum[blockIdx.x] = carry;
}

// Counting-sort scatter of the point records, one thread per point: the
// position is the bin-major prefix of the point's (bin, sort block) entry plus
// its rank within that entry.  Each workgroup first scans the table-scan
// segment totals in LDS (at most kBins + 1 of them); workgroup 0 also stores
// them, and their sum, for the later kernels.  Points of a bin that share a
// sort block land in an unspecified order; FP64 results do not depend on it.
__global__ __launch_bounds__(1024) void k_scatter(int n, const double2 *__restrict__ z, EvalWs W) {
    __shared__ int32_t s_boff[kSeg];
    const int nseg = (kBins + 1 + W.tab_ib - 1) / W.tab_ib;
    {
        int32_t v[4];
        load4(W.bin_sum, nseg, v);
        const int32_t tot = block_scan4(v, s_boff, nseg, 0);
        if (blockIdx.x == 0) {
            for (int i = threadIdx.x; i < nseg; i += 1024) W.bin_off[i] = s_boff[i];
            if (threadIdx.x == 0) W.ctl[5] = tot;
        }
        __syncthreads();
    }
    const int j = blockIdx.x * 1024 + threadIdx.x;
    if (j >= n) return;
    const int kr = W.keyrank[j];
    const int key = kr / kSortPoints, rank = kr % kSortPoints;
    if (key == kBins) return;                          // finished points are not sorted
    const int64_t idx = (int64_t)key * W.n_sort_blocks + j / kSortPoints;
    const int pos = W.tscan[idx] + s_boff[key / W.tab_ib] + rank;
    W.srec[pos] = point_rec(z, W, j);
}

// Work of the (group, chunk) tiles, in Horner steps, counted in units of
// (16 << cost_shift) steps.  A tile costs its steps plus a fixed part by kind,
// plus a full binary powering where some window of the group starts in the
// chunk (at most the chunks up to the group's largest window start), at
// kPowSteps steps per bit of the exponent.  The fixed parts: every tile
// kTileSteps (the coefficient batches, the output); the first tile of a group
// spanning several chunks kFirstSteps more (fixed-point partials); its last
// tile kLastSteps more and its middle tiles kMidSteps + C/8 more (the chained
// power, the partials and the LDS state of the continuing lanes, and a middle
// tile's Horner steps running with every lane active); a tile the windows
// continue into kAnchorBitSteps per bit of the group's last index more (the
// anchors of the chained power every kAnchor chunks, spread over the tiles).
// The weights were fitted to the time of every tile of the window kernel
// measured on gfx950 (start and end clocks per tile, against its Horner
// steps, powering bits and kind, with one contention factor per interval of
// the kernel's span shared by all tiles in it): the steps of one wavefront
// are the unit, and the fit explains 89-96 % of the tiles' variance.  Middle
// tiles cost one of two amounts, before and after the last window start,
// which lets the partition locate a tile in O(1).
constexpr int kCostUnit = 16;
constexpr int kPowSteps = 20;
constexpr int kTileSteps = 40;
constexpr int kFirstSteps = 50;
constexpr int kLastSteps = 100;
constexpr int kMidSteps = 143;
constexpr int kAnchorBitSteps = 4;

struct GroupCost {
    int clo, chi;              // first and last chunk of the group's union window
    int first, last;           // cost of its first and last tiles (first: the whole group if clo == chi)
    int ns, cs;                // the next ns middle tiles (a window may start there) cost cs each,
    int cn;                    //   the other middle tiles cn each
};

__device__ __forceinline__ int cost_units(int steps, int shift) {
    const int lg = 4 + shift;                          // kCostUnit = 16 = 2^4
    return (steps + (1 << lg) - 1) >> lg;
}

__device__ __forceinline__ int bit_length(int x) { return x > 0 ? 32 - __clz(x) : 0; }

// the Horner steps of a tile part of len coefficients: all of them for a dense
// window sum, the share dens / 256 for a sparse one
__device__ __forceinline__ int tile_steps(int len, int dens) {
    return dens >= 256 ? len : (int)(((long long)len * dens + 255) >> 8);
}

// glo, ghi: the group's union window; gml: its largest window start; dens: the
// share of the union window's Horner steps the tiles run (256: dense)
__device__ __forceinline__ GroupCost group_cost(int glo, int ghi, int gml, int C, int shift, int dens) {
    GroupCost gc;
    gc.clo = glo / C;
    gc.chi = ghi / C;
    const int cl = gml / C;
    const int pow_start = kPowSteps * bit_length(gml);
    const int anchor = kAnchorBitSteps * bit_length(ghi);
    if (gc.chi == gc.clo) {
        gc.first = gc.last = cost_units(tile_steps(ghi - glo + 1, dens) + kTileSteps + pow_start, shift);
        gc.ns = 0;
        gc.cs = gc.cn = 1;
        return gc;
    }
    gc.first = cost_units(tile_steps(gc.clo * C + C - glo, dens) + kTileSteps + kFirstSteps + pow_start, shift);
    gc.last = cost_units(tile_steps(ghi - gc.chi * C + 1, dens) + kTileSteps + kLastSteps + anchor +
                             (gc.chi <= cl ? pow_start : 0),
                         shift);
    gc.ns = max(0, min(cl, gc.chi - 1) - gc.clo);
    const int mid = tile_steps(C + C / 8, dens) + kTileSteps + kMidSteps + anchor;
    gc.cs = cost_units(mid + pow_start, shift);
    gc.cn = cost_units(mid, shift);
    return gc;
}

__device__ __forceinline__ long long group_total(const GroupCost &gc) {
    if (gc.chi == gc.clo) return gc.first;
    const long long nn = gc.chi - gc.clo - 1 - gc.ns;
    return (long long)gc.first + gc.last + (long long)gc.ns * gc.cs + nn * gc.cn;
}

constexpr int kGroupsPerBlock = 1024 / kWave;
constexpr int kSparseSteps = 5;        // cost of one entry of a sparse window sum, in Horner steps

// ---- many polynomials in one evaluation (fpe_eval_batched)
constexpr int kBatchMaxPoints = 4096;   // points of one polynomial of a batch (sorted by one workgroup)
constexpr int kBatchThreads = 256;
constexpr int kBatchScanPer = (kBins + 1 + kBatchThreads - 1) / kBatchThreads;   // bins per thread in the scan

// One workgroup per polynomial of a batch: the bounds of its points (as in
// k_bounds, with its own cover in LDS), their order by lambda bin (a counting
// sort in LDS: a point's rank within its bin from an LDS counter, then a scan
// of the bin counts; finished points have the bin kBins and come last; the
// order within a bin is free, since FP64 results do not depend on which points
// share a wavefront) and its slots of the sorted records: the records in that
// order, then records without a window up to a whole number of groups, so
// that no group mixes two polynomials.
__global__ __launch_bounds__(kBatchThreads) void k_bbounds(const DevPlan *__restrict__ plans,
                                                           const long long *__restrict__ pstart,
                                                           const int32_t *__restrict__ gstart,
                                                           const double2 *__restrict__ z, double2 *__restrict__ m_out,
                                                           long long *__restrict__ e_out, int32_t *__restrict__ terms,
                                                           EvalWs W) {
    __shared__ double s_k[kHullLds];
    __shared__ double s_s[kHullLds];
    __shared__ int32_t s_bin[kBins + 1];              // bin counts, then their exclusive prefix
    __shared__ int32_t s_kr[kBatchMaxPoints];         // per point: bin x kBatchMaxPoints + rank in the bin
    __shared__ int32_t s_wsum[kBatchThreads / kWave];
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const int pidx = blockIdx.x;
    if (pidx == 0 && t < 64) W.ctl[t] = 0;            // totals and counters of the later kernels
    const DevPlan P = plans[pidx];
    const long long p0 = pstart[pidx];
    const int m = (int)(pstart[pidx + 1] - p0);
    const int g0 = gstart[pidx], ng = gstart[pidx + 1] - g0;
    const bool in_lds = P.nh <= kHullLds;
    if (in_lds)
        for (int i = t; i < P.nh; i += kBatchThreads) { s_k[i] = P.hull_k[i]; s_s[i] = P.hull_s[i]; }
    for (int i = t; i <= kBins; i += kBatchThreads) s_bin[i] = 0;
    __syncthreads();
    auto run = [&](auto hk, auto hs) {
        for (int j = t; j < m; j += kBatchThreads) {
            const int key = bounds_point(P, hk, hs, z, (int)(p0 + j), m_out, e_out, nullptr, nullptr, terms, nullptr, W);
            s_kr[j] = key * kBatchMaxPoints + atomicAdd(&s_bin[key], 1);   // LDS
        }
    };
    if (in_lds) run((lds_table_t)s_k, (lds_table_t)s_s);
    else run((const double *)P.hull_k, (const double *)P.hull_s);
    __syncthreads();
    // exclusive prefix of the bin counts: a run of consecutive bins per thread
    {
        const int i0 = t * kBatchScanPer;
        int v[kBatchScanPer];
        int sum = 0;
#pragma unroll
        for (int k = 0; k < kBatchScanPer; ++k) {
            v[k] = i0 + k <= kBins ? s_bin[i0 + k] : 0;
            sum += v[k];
        }
        int incl = sum;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int x = __shfl_up(incl, d);
            if (lane >= d) incl += x;
        }
        if (lane == kWave - 1) s_wsum[wave] = incl;
        __syncthreads();
        int run_ = incl - sum;
        for (int r = 0; r < wave; ++r) run_ += s_wsum[r];
#pragma unroll
        for (int k = 0; k < kBatchScanPer; ++k) {
            if (i0 + k <= kBins) s_bin[i0 + k] = run_;
            run_ += v[k];
        }
    }
    __syncthreads();
    // the records in bin order (each thread moves the points it bounded), then
    // records without a window up to whole groups
    for (int j = t; j < m; j += kBatchThreads) {
        const int kr = s_kr[j];
        const size_t dst = (size_t)g0 * kWave + s_bin[kr / kBatchMaxPoints] + kr % kBatchMaxPoints;
        W.srec[dst] = point_rec(z, W, (int)(p0 + j));
    }
    for (int q = m + t; q < ng * kWave; q += kBatchThreads) {
        const size_t dst = (size_t)g0 * kWave + q;
        PointRec rc;
        rc.z = make_double2(0.0, 0.0);
        rc.l = 1;
        rc.r = 0;
        rc.j = -1;
        rc.pad = 0;
        W.srec[dst] = rc;
    }
}

// One wavefront per group of 64 sorted points: the union window, the largest
// window start and the tile cost; then, per workgroup of kGroupsPerBlock
// groups, the exclusive prefix of the costs (gcum) and their total (gblk_sum).
__global__ __launch_bounds__(1024) void k_groups(DevPlan P, EvalWs W) {
    __shared__ int32_t s_cost[kGroupsPerBlock];
    const int gw = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int g = blockIdx.x * kGroupsPerBlock + gw;
    int cost = 0;
    if (g < W.n_groups) {
        const int nvalid = valid_points(W);
        const int idx = g * kWave + lane;
        int l = INT_MAX, r = INT_MIN;
        // records without a window (a batch's padding and finished points) do not count
        if (idx < nvalid) { const PointRec &rc = W.srec[idx]; if (rc.l <= rc.r) { l = rc.l; r = rc.r; } }
        const int lo = wave_min(l), hi = wave_max(r), ml = wave_max(l != INT_MAX ? l : INT_MIN);
        int dens = 256;
        if (W.sparse && hi >= lo) {
            // a sparse window sum runs about kSparseSteps Horner steps per
            // index of G_p in the union window
            const long long u = (long long)P.gprefix[hi + 1] - P.gprefix[lo];
            const long long w = (long long)hi - lo + 1;
            dens = (int)min(256LL, max(1LL, (u * kSparseSteps * 256 + w - 1) / w));
        }
        cost = hi >= lo ? (int)group_total(group_cost(lo, hi, ml, W.chunk, W.cost_shift, dens)) : 0;
        if (lane == 0) {
            W.glo[g] = lo;
            W.ghi[g] = hi;
            W.gml[g] = ml;
            W.gcost[g] = cost;
            W.gdens[g] = dens;
        }
    }
    if (lane == 0) s_cost[gw] = cost;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int k = 0; k < kGroupsPerBlock; ++k) {
            const int gg = blockIdx.x * kGroupsPerBlock + k;
            if (gg < W.n_groups) W.gcum[gg] = acc;
            acc += s_cost[k];
        }
        W.gblk_sum[blockIdx.x] = acc;
    }
}

// Equal-work partition of the tiles over the window kernel's wavefronts.  The
// tiles, in (group, chunk) order, cover consecutive intervals of a cost axis of
// length `total`; wavefront w owns the tiles whose interval starts in
// [s_w, s_{w+1}), s_w = ceil(w total / NW), so its work is total / NW up to one
// tile, and the owner of a tile starting at a is floor(a NW / total).  A group
// starts at gcum[g] (its offset inside its k_groups workgroup) plus the
// exclusive prefix of the workgroup totals: scanned here in LDS when there are
// at most kPartLds workgroups, otherwise by k_scan_seg and k_scan_sums
// beforehand.

// floor(a / b) for 0 <= a < 2^62, 0 < b < 2^31 (quotients here fit in int32):
// a double quotient, corrected exactly
__device__ __forceinline__ long long div_floor(long long a, long long b) {
    long long q = (long long)((double)a / (double)b);
    while (q * b > a) --q;
    while ((q + 1) * b <= a) ++q;
    return q;
}

constexpr int kPartLds = 8192;

struct BlockOffsets {
    const int32_t *lds;        // exclusive prefix per k_groups workgroup (few workgroups)
    const int32_t *pre, *seg;  // segment-local prefix and segment offsets (many)
    __device__ long long at(int b) const {
        return lds ? (long long)lds[b] : (long long)pre[b] + seg[b / kSeg];
    }
};

// the first tile of wavefront w, whose start s lies in group g's interval
// [A, B) of the cost axis: (g, c) if a tile of g starts exactly at s, else
// (g, c + 1) for the tile after the one holding s, or (g + 1, -1) for "the
// first tile of the first group with tiles after g"
__device__ __forceinline__ int2 wave_start(const GroupCost &gc, int g, long long A, long long B, long long s) {
    int c;
    long long a;
    if (s < A + gc.first || gc.chi == gc.clo) { c = gc.clo; a = A; }
    else if (s >= B - gc.last) { c = gc.chi; a = B - gc.last; }
    else {
        const long long x = s - A - gc.first, xs = (long long)gc.ns * gc.cs;
        if (x < xs) {
            const long long q = div_floor(x, gc.cs);
            c = gc.clo + 1 + (int)q;
            a = A + gc.first + q * gc.cs;
        } else {
            const long long q = div_floor(x - xs, gc.cn);
            c = gc.clo + 1 + gc.ns + (int)q;
            a = A + gc.first + xs + q * gc.cn;
        }
    }
    if (a == s) return make_int2(g, c);
    if (c < gc.chi) return make_int2(g, c + 1);
    return make_int2(g + 1, -1);
}

// threads [0, G): per group, the owners of its first and last tiles; threads
// [G, G + NW]: per wavefront, its first tile as (group, chunk), or (group, -1)
// for "the first tile of the first group with tiles at or after this one";
// (G, 0) past the end of the work and for the sentinel w = NW
// fixed-point words per lane and window-wavefront slot: the sums of Q, then of Q'
constexpr int kSlotWords = 8;

// slot s of the window wavefronts (two per wavefront), stored by word pair:
// pair q (words 2q and 2q + 1) of the 64 lanes lies at [q 64, q 64 + 64), so
// a wavefront writes and reads each pair as one contiguous 1 KB run
__device__ __forceinline__ longlong2 *slot_pairs(const EvalWs &W, size_t s) {
    return reinterpret_cast<longlong2 *>(W.slots + s * kWave * kSlotWords);
}

// Split groups whose windows span more than kFinalShort + 1 window wavefronts
// are long groups: the finalize kernel cuts their owners into pieces of
// kLongPiece and spreads the pieces over its grid.  Owner ranges of two groups
// share at most one wavefront, so an evaluation over n_waves wavefronts has
// fewer than long_cap(n_waves) long groups.
constexpr int kFinalShort = 8;
constexpr int kLongPiece = 32;
constexpr int kLongLds = 2048;        // long groups the finalize kernel holds in LDS
__host__ __device__ inline int long_cap(int64_t n_waves) { return (int)(n_waves / kFinalShort + 1); }
// pieces of a long group (group, first owner, last owner)
__device__ __forceinline__ int long_pieces(int4 v) { return (v.z - v.y + kLongPiece) / kLongPiece; }

// window wavefront w's first tile (its share of the work starts at
// ceil(w total / NW)), and the split-group list entry of the group it starts in
__device__ __forceinline__ void partition_wave(const EvalWs &W, const BlockOffsets &bo, long long total, int nblk,
                                               int w) {
    const int G = (int)W.n_groups, NW = (int)W.n_waves, C = W.chunk;
    const long long sw = total > 0 ? div_floor((long long)w * total + NW - 1, NW) : 0;
    if (w == NW || total == 0 || sw >= total) { W.wstart[w] = make_int2(G, 0); return; }
    // the last group starting at or before s_w: first its k_groups workgroup,
    // then among that workgroup's groups
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bo.at(mid) <= sw) lo = mid; else hi = mid - 1;
    }
    const long long base = bo.at(lo);
    // offsets inside a workgroup do not decrease: g is g0 plus the number of
    // the workgroup's later groups starting at or before s_w (independent
    // loads, one memory latency instead of one per group: the indices are
    // clamped rather than the loads guarded, which the compiler would turn
    // into one branch and one wait per load)
    const int g0 = lo * kGroupsPerBlock, ng = min(G - g0, kGroupsPerBlock);
    int32_t cum[kGroupsPerBlock];
#pragma unroll
    for (int k = 1; k < kGroupsPerBlock; ++k) cum[k] = W.gcum[g0 + min(k, ng - 1)];
    int g = g0;
#pragma unroll
    for (int k = 1; k < kGroupsPerBlock; ++k) g += (k < ng && base + cum[k] <= sw) ? 1 : 0;
    const long long A = base + W.gcum[g], B = A + W.gcost[g];
    if (sw >= B) { W.wstart[w] = make_int2(g + 1, -1); return; }
    const GroupCost gc = group_cost(W.glo[g], W.ghi[g], W.gml[g], C, W.cost_shift, W.gdens[g]);
    const int2 st = wave_start(gc, g, A, B, sw);
    W.wstart[w] = st;
    // w starts inside g and g's first tile belongs to w - 1: g is split, and
    // w is its second owner (this identifies each split group once); long
    // groups have their own list
    if (st.x == g && div_floor(A * NW, total) == w - 1) {
        const int wy = (int)div_floor((B - gc.last) * NW, total);
        if (wy - (w - 1) < kFinalShort) W.split[atomicAdd(W.ctl + 8, 1)] = make_int4(g, w - 1, wy, 0);
    }
}

__global__ __launch_bounds__(1024) void k_partition(DevPlan P, EvalWs W) {
    __shared__ int32_t s_off[kPartLds];
    __shared__ int s_nl;                       // long groups found by this workgroup
    __shared__ int s_li[1024];                 //   and their list indices
    const int G = (int)W.n_groups, NW = (int)W.n_waves, C = W.chunk;
    const int nblk = (G + kGroupsPerBlock - 1) / kGroupsPerBlock;
    BlockOffsets bo{nullptr, W.gblk_pre, W.gseg_off};
    long long total;
    if (threadIdx.x == 0) s_nl = 0;
    if (nblk <= kPartLds) {
        int32_t carry = 0;
        for (int s0 = 0; s0 < nblk; s0 += kSeg) {
            int32_t v[4];
            load4(W.gblk_sum + s0, min(kSeg, nblk - s0), v);
            carry += block_scan4(v, s_off + s0, min(kSeg, nblk - s0), carry);
        }
        bo.lds = s_off;
        total = carry;
    } else {
        total = W.ctl[0];
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < G) {
        // group g's owners: the wavefronts whose shares hold its first and its
        // last tile's start
        const int g = (int)i;
        const int cost = W.gcost[g];
        if (cost != 0 && total != 0) {
            const GroupCost gc = group_cost(W.glo[g], W.ghi[g], W.gml[g], C, W.cost_shift, W.gdens[g]);
            const long long A = W.gcum[g] + bo.at(g / kGroupsPerBlock), B = A + cost;
            const int2 gw = make_int2((int)div_floor(A * NW, total), (int)div_floor((B - gc.last) * NW, total));
            if (gw.y - gw.x >= kFinalShort) {
                const int li = atomicAdd(W.ctl + 9, 1);
                const int4 lg = make_int4(g, gw.x, gw.y, 0);
                W.lgroups[li] = lg;
                // only a group summed in several pieces uses an accumulator
                if (long_pieces(lg) > 1) s_li[atomicAdd(&s_nl, 1)] = li;
            }
        }
    } else if (i <= (int64_t)G + NW) {
        partition_wave(W, bo, total, nblk, (int)(i - G));
    }
    __syncthreads();
    // the finalize kernel's accumulators and piece count of each long group
    // of several pieces found here start at zero
    const int nl = s_nl;
    for (int k = threadIdx.x; k < nl * (kWave * kSlotWords / 2); k += blockDim.x) {
        const int li = s_li[k / (kWave * kSlotWords / 2)];
        reinterpret_cast<longlong2 *>(W.lacc + (size_t)li * kWave * kSlotWords)[k % (kWave * kSlotWords / 2)] =
            make_longlong2(0, 0);
    }
    if (threadIdx.x < nl) W.lcnt[s_li[threadIdx.x]] = 0;
}

// (g, c) with c < 0: the first tile of the first group at or after g with tiles
__device__ __forceinline__ void resolve_tile(const EvalWs &W, int C, int &g, int &c) {
    const int G = (int)W.n_groups;
    if (c >= 0) return;
    while (g < G && W.gcost[g] == 0) ++g;
    c = g < G ? W.glo[g] / C : 0;
}

// One Horner step acc <- acc z + a, a = (ar, ai) wave-uniform:
//   hr' = hr zr + (ar - hi zi),  hi' = hi zr + (ai + hr zi)
// four VOP3 FMAs whose addends are read straight from scalar registers, updating
// the accumulator in place (written out because the compiler otherwise copies
// half of the addends into vector registers, and the accumulator between
// masked steps).
__device__ __forceinline__ void horner_step(double &hr, double &hi, double zr, double zi, double ar, double ai) {
    double tr, ti;
    asm volatile("v_fma_f64 %2, -%1, %4, %6\n\t"
                 "v_fma_f64 %3, %0, %4, %7\n\t"
                 "v_fma_f64 %0, %0, %5, %2\n\t"
                 "v_fma_f64 %1, %1, %5, %3"
                 : "+v"(hr), "+v"(hi), "=&v"(tr), "=&v"(ti)
                 : "v"(zi), "v"(zr), "s"(ar), "s"(ai));
}

constexpr int kBatch = 4;   // coefficients per scalar-load batch (64 bytes, one s_load_dwordx16)

__device__ __forceinline__ void load_batch(double *dst, const_table_t p) {
#pragma unroll
    for (int q = 0; q < 2 * kBatch; ++q) dst[q] = p[q];
}

// s_waitcnt lgkmcnt(0) (vmcnt and expcnt left at their maxima)
__device__ __forceinline__ void wait_scalar_loads() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// The running Horner value of a lane, and with D its derivative in z:
//   H' <- H' z + H (the old H), then H <- H z + a_k
template <bool D> struct Acc { double hr = 0.0, hi = 0.0; };
template <> struct Acc<true> { double hr = 0.0, hi = 0.0, dr = 0.0, di = 0.0; };

template <bool D>
__device__ __forceinline__ void acc_step(Acc<D> &a, double zr, double zi, double ar, double ai) {
    if constexpr (D) {
        FPE_NO_CONTRACT
        const double tr = fma(-a.di, zi, a.hr), ti = fma(a.dr, zi, a.hi);
        a.dr = fma(a.dr, zr, tr);
        a.di = fma(a.di, zr, ti);
    }
    horner_step(a.hr, a.hi, zr, zi, ar, ai);
}

// Which lanes take the step of coefficient k in a tile where lane i covers
// [lo_i, hi_i]: all of them (the common part), those that have started
// (k <= hi_i, the ragged top), those that have not finished (k >= lo_i, the
// ragged bottom), or both tests.
enum StepMask { kAll = 0, kTop = 1, kBottom = 2, kBoth = 3 };

template <int M, bool D>
__device__ __forceinline__ void masked_step(Acc<D> &a, double zr, double zi, double ar, double ai, int k, int lo,
                                            int hi) {
    if ((M & kTop) && k > hi) return;
    if ((M & kBottom) && k < lo) return;
    acc_step(a, zr, zi, ar, ai);
}

template <int M, bool D>
__device__ __forceinline__ void batch_steps(Acc<D> &a, double zr, double zi, const double *X, int kbase, int lo,
                                            int hi) {
#pragma unroll
    for (int s2 = kBatch - 1; s2 >= 0; --s2) masked_step<M>(a, zr, zi, X[2 * s2], X[2 * s2 + 1], kbase + s2, lo, hi);
}

// Horner steps for k = kfrom, kfrom - 1, ..., kto (none if kfrom < kto); kfrom
// and kto are wave-uniform.  Coefficients come in batches of kBatch (one 64-byte
// scalar load each), one batch ahead.  Scalar loads may return out of order, so
// a wait for one batch waits for every batch in flight: each batch starts with
// an unconditional wait for itself (nothing else is in flight then), requests
// the next batch, and runs its steps, which need no further wait even when
// they are masked.
template <int M, bool D>
__device__ __forceinline__ void run_steps(Acc<D> &a, double zr, double zi, const_table_t cf, int kfrom, int kto,
                                          int lo, int hi) {
    if (kfrom < kto) return;
    const int nb = (kfrom - kto + 1) / kBatch;
    int k = kfrom;
    if (nb > 0) {
        // batch b holds a_{kb}, ..., a_{kb + kBatch - 1}, kb = kfrom - kBatch (b + 1) + 1
        const_table_t base = cf + 2 * (kfrom - kBatch + 1);
        const int kb0 = kfrom - kBatch + 1;
        double A[2 * kBatch], B[2 * kBatch];
        load_batch(A, base);
        int bi = 0;
        for (; bi + 2 <= nb; bi += 2) {
            wait_scalar_loads();
            __builtin_amdgcn_sched_barrier(0);
            load_batch(B, base - 2 * kBatch * (bi + 1));
            __builtin_amdgcn_sched_barrier(0);
            batch_steps<M>(a, zr, zi, A, kb0 - kBatch * bi, lo, hi);
            wait_scalar_loads();
            __builtin_amdgcn_sched_barrier(0);
            if (bi + 2 < nb) load_batch(A, base - 2 * kBatch * (bi + 2));
            __builtin_amdgcn_sched_barrier(0);
            batch_steps<M>(a, zr, zi, B, kb0 - kBatch * (bi + 1), lo, hi);
        }
        if (bi < nb) {
            wait_scalar_loads();
            batch_steps<M>(a, zr, zi, A, kb0 - kBatch * bi, lo, hi);
        }
        k -= kBatch * nb;
    }
    for (; k >= kto; --k) masked_step<M>(a, zr, zi, cf[2 * k], cf[2 * k + 1], k, lo, hi);
}

// ---- FP32 window sums (plans with FP32 tables)
constexpr int kBlock32 = 8;   // coefficients per FP32 block: one 64-byte scalar load of float2

// one FP32 Horner step h <- h z + a (four FMAs, each rounded to FP32)
__device__ __forceinline__ void step32(float &hr, float &hi, float zr, float zi, float ar, float ai) {
    const float tr = fmaf(-hi, zi, ar), ti = fmaf(hr, zi, ai);
    hr = fmaf(hr, zr, tr);
    hi = fmaf(hi, zr, ti);
}

// TwoSum in FP32: s + e = a + b exactly
__device__ __forceinline__ void two_sum_f(float a, float b, float &s, float &e) {
    FPE_NO_CONTRACT
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// One compensated FP32 Horner step (s, c) <- (s, c) z + a, z = zh + zl: the
// products s zh split exactly by TwoProd (fmaf), the two additions of each
// component by TwoSum, and the lost parts (product and sum errors, s zl) carried
// in the correction c, itself advanced by c zh.  s + c is the sum with a
// relative error of a few units of 2^-48 per step, far below the rounding of
// the FP32 coefficients (2^-24) that bounds the form's accuracy.
__device__ __forceinline__ void step32c(float &sr, float &si, float &cr, float &ci, float zhr, float zhi, float zlr,
                                        float zli, float ar, float ai) {
    FPE_NO_CONTRACT
    const float p1 = sr * zhr, q1 = fmaf(sr, zhr, -p1);
    const float p2 = si * zhi, q2 = fmaf(si, zhi, -p2);
    const float p3 = sr * zhi, q3 = fmaf(sr, zhi, -p3);
    const float p4 = si * zhr, q4 = fmaf(si, zhr, -p4);
    float t1, e1, nr, e2, t2, e3, ni, e4;
    two_sum_f(p1, -p2, t1, e1);
    two_sum_f(t1, ar, nr, e2);
    two_sum_f(p3, p4, t2, e3);
    two_sum_f(t2, ai, ni, e4);
    const float er = ((q1 - q2) + (e1 + e2)) + fmaf(sr, zlr, -(si * zli));
    const float ei = ((q3 + q4) + (e3 + e4)) + fmaf(sr, zli, si * zlr);
    const float ncr = fmaf(cr, zhr, fmaf(-ci, zhi, er));
    ci = fmaf(cr, zhi, fmaf(ci, zhr, ei));
    cr = ncr;
    sr = nr;
    si = ni;
}

// z in the forms the FP32 blocks use: FP32 z (and its rounding error, for the
// compensated form), and z^8 and 8 z^7 in FP64 for the block accumulation
struct Z32 { float r, i, lr, li; double z8r, z8i, z7r, z7i; };

__device__ __forceinline__ Z32 make_z32(double zr, double zi) {
    FPE_NO_CONTRACT
    Z32 q;
    q.r = (float)zr;
    q.i = (float)zi;
    q.lr = (float)(zr - (double)q.r);
    q.li = (float)(zi - (double)q.i);
    const double z2r = fma(zr, zr, -(zi * zi)), z2i = 2.0 * zr * zi;
    const double z3r = fma(z2r, zr, -(z2i * zi)), z3i = fma(z2r, zi, z2i * zr);
    const double z4r = fma(z2r, z2r, -(z2i * z2i)), z4i = 2.0 * z2r * z2i;
    q.z8r = fma(z4r, z4r, -(z4i * z4i));
    q.z8i = 2.0 * z4r * z4i;
    q.z7r = 8.0 * fma(z4r, z3r, -(z4i * z3i));
    q.z7i = 8.0 * fma(z4r, z3i, z4i * z3r);
    return q;
}

// the FP32 recurrence of one block of L coefficients from A (a_{kt - L + 1}
// .. a_{kt}, interleaved), from the top; with MASKED, lanes above their part
// add 0 (their recurrence stays 0 until the part starts), without it every
// lane takes every step and the coefficients stay wave-uniform operands.
// Returns the block's sum h (and with D its derivative d) as doubles.
template <bool D, bool COMP, int L, bool MASKED>
__device__ __forceinline__ void block32(const float *A, int kt, int hi, const Z32 &z, double &br,
                                        double &bi, double &dr, double &di) {
    float hr = 0.0f, hh = 0.0f, cr = 0.0f, ch = 0.0f, gr = 0.0f, gh = 0.0f;
#pragma unroll
    for (int s2 = L - 1; s2 >= 0; --s2) {
        const bool on = !MASKED || kt - (L - 1 - s2) <= hi;
        const float ar = on ? A[2 * s2] : 0.0f, ai = on ? A[2 * s2 + 1] : 0.0f;
        if constexpr (D) {
            const float tr = fmaf(-gh, z.i, hr), ti = fmaf(gr, z.i, hh);
            gr = fmaf(gr, z.r, tr);
            gh = fmaf(gh, z.r, ti);
        }
        if constexpr (COMP) step32c(hr, hh, cr, ch, z.r, z.i, z.lr, z.li, ar, ai);
        else step32(hr, hh, z.r, z.i, ar, ai);
    }
    br = COMP ? (double)hr + (double)cr : (double)hr;
    bi = COMP ? (double)hh + (double)ch : (double)hh;
    dr = (double)gr;
    di = (double)gh;
}

// H = sum over k = kto .. min(hi, kfrom) of a_k z^(k - kto) (and with D its
// derivative in z), for the common and top parts [kto, kfrom] of a tile (every
// active lane has lo <= kto): the FP32 table in blocks of kBlock32
// coefficients from the top, each block by an FP32 Horner recurrence in z
// (plain, or with COMP compensated: TwoSum/TwoProd error terms carried in a
// correction), and the block partials by an FP64 Horner recurrence in z^8
// (H' <- H' z^8 + 8 z^7 H + block's derivative).  ktop: above it every lane
// takes every step.  Returns H in the FP64 table's scale (times 2^sg).
template <bool D, bool COMP>
__device__ __forceinline__ void run_f32(Acc<D> &acc, const Z32 &z, const_table32_t c32, int sg, int kfrom, int kto,
                                        int ktop, int hi) {
    FPE_NO_CONTRACT
    const int len = kfrom - kto + 1;
    const int l0 = len % kBlock32;
    double Hr = 0.0, Hi = 0.0, Dr = 0.0, Di = 0.0;
    int k = kfrom;
    if (l0 > 0) {                              // the short block at the top: H starts there
        float hr = 0.0f, hh = 0.0f, cr = 0.0f, ch = 0.0f, gr = 0.0f, gh = 0.0f;
        for (int j = 0; j < l0; ++j) {
            const int kk = k - j;
            const bool on = kk <= hi;
            const float ar = on ? c32[2 * kk] : 0.0f, ai = on ? c32[2 * kk + 1] : 0.0f;
            if constexpr (D) {
                const float tr = fmaf(-gh, z.i, hr), ti = fmaf(gr, z.i, hh);
                gr = fmaf(gr, z.r, tr);
                gh = fmaf(gh, z.r, ti);
            }
            if constexpr (COMP) step32c(hr, hh, cr, ch, z.r, z.i, z.lr, z.li, ar, ai);
            else step32(hr, hh, z.r, z.i, ar, ai);
        }
        Hr = COMP ? (double)hr + (double)cr : (double)hr;
        Hi = COMP ? (double)hh + (double)ch : (double)hh;
        Dr = (double)gr;
        Di = (double)gh;
        k -= l0;
    }
    for (; k >= kto; k -= kBlock32) {          // full blocks [k - 7, k]
        const_table32_t p = c32 + 2 * (k - kBlock32 + 1);
        float A[2 * kBlock32];
#pragma unroll
        for (int q = 0; q < 2 * kBlock32; ++q) A[q] = p[q];
        double br, bi, dr, di;
        if (k > ktop) block32<D, COMP, kBlock32, true>(A, k, hi, z, br, bi, dr, di);
        else block32<D, COMP, kBlock32, false>(A, k, hi, z, br, bi, dr, di);
        if constexpr (D) {
            const double nr = fma(Dr, z.z8r, fma(-Di, z.z8i, fma(Hr, z.z7r, fma(-Hi, z.z7i, dr))));
            Di = fma(Dr, z.z8i, fma(Di, z.z8r, fma(Hr, z.z7i, fma(Hi, z.z7r, di))));
            Dr = nr;
        }
        const double nr = fma(Hr, z.z8r, fma(-Hi, z.z8i, br));
        Hi = fma(Hr, z.z8i, fma(Hi, z.z8r, bi));
        Hr = nr;
    }
    acc.hr = ldexp(Hr, sg);
    acc.hi = ldexp(Hi, sg);
    if constexpr (D) {
        acc.dr = ldexp(Dr, sg);
        acc.di = ldexp(Di, sg);
    }
}

constexpr int kWindowThreads = 256;
constexpr int kWindowWaves = kWindowThreads / kWave;

// State of the chained powers of one segment (see tile_power).
struct PowState {
    int chain_c = -1;          // chunk of the chained power; -1: none
    bool have_zc = false;      // w^C is in LDS
    bool xv = false;           // this lane's chained power is w^(chain_c C)
};

// z^lo for the lanes of tile (g, c), as (pr + i pi) 2^pe times 2^(lo ez):
// w^l by binary powering for lanes whose window starts in this chunk (lo = l),
// the chained w^(c C) for lanes that started earlier (lo = c C), advanced by one
// product per chunk from the anchor w^(m C), m = c - c mod kAnchor, by
// cpow_chunk_start's recipe, so that every wavefront gets the same bits for the
// same chunk.  s_ch / s_che hold per thread the chained power and w^C.
__device__ __forceinline__ void tile_power(PowState &ps, int l, int lo, bool act, int c, int C, double wr, double wi,
                                           double (*s_ch)[kWindowThreads], long long (*s_che)[kWindowThreads], int t,
                                           double &pr, double &pi, long long &pe) {
    const int c0 = c * C;
    const bool cont = act && l < c0;
    pr = 1.0; pi = 0.0; pe = 0;
    const bool any_cont = __ballot(cont) != 0;
    // a continuing lane advances its chained power by one product if it holds
    // w^((c - 1) C) and c is not an anchor; otherwise it starts from the anchor
    const bool step_ok = ps.chain_c >= 0 && ps.chain_c == c - 1 && c % kAnchor != 0;
    const bool use_chain = cont && ps.xv && step_ok;
    const bool need_anchor = cont && !use_chain;
    // at most two rounds of one binary powering each (one call site keeps the
    // register footprint down): round 0, once per segment, w^C; round 1, the
    // anchors of continuing lanes that need them and w^lo of lanes whose window
    // starts in this chunk
    const bool need1 = __ballot(need_anchor || (!cont && act && lo > 0)) != 0;
    const int rd_end = need1 ? 1 : 0;
#pragma nounroll
    for (int rd = (any_cont && !ps.have_zc) ? 0 : 1; rd <= rd_end; ++rd) {
        const int n = rd == 0 ? C : (need_anchor ? (c - c % kAnchor) * C : (!cont && act ? lo : 0));
        double qr_, qi_;
        long long qe = 0;
        cpow_dd(wr, wi, n, qr_, qi_, qe);
        if (rd == 0) {
            s_ch[2][t] = qr_; s_ch[3][t] = qi_; s_che[1][t] = qe;
        } else {
            pr = qr_; pi = qi_; pe = qe;
        }
    }
    if (any_cont) {
        ps.have_zc = true;
        if (cont) {
            const double zcr = s_ch[2][t], zci = s_ch[3][t];
            const long long zce = s_che[1][t];
            double xr, xi;
            long long xe;
            int j0;
            if (use_chain) { xr = s_ch[0][t]; xi = s_ch[1][t]; xe = s_che[0][t]; j0 = c - 1; }
            else { xr = pr; xi = pi; xe = pe; j0 = c - c % kAnchor; }
            for (int j = j0; j < c; ++j) cmul_renorm(xr, xi, xe, zcr, zci, zce);
            s_ch[0][t] = xr; s_ch[1][t] = xi; s_che[0][t] = xe;
            pr = xr; pi = xi; pe = xe;
        }
        ps.xv = cont;
        ps.chain_c = c;
    }
}

// reference exponent of the derivative's terms k a_k z^(k-1): each is below
// r 2^(N - lambda), and with lambda >= ez - 1 (z = w 2^ez) and eref = floor(N) + 2,
// eref + 1 - ez + bitlen(r) bounds floor(N - lambda) + 2 + bitlen(r) from above
__device__ __forceinline__ long long deriv_eref(long long eref, int ez, int r) {
    return eref + 1 - ez + (32 - __clz(r > 0 ? r : 1));
}

// fixed-point form of a partial value (qr + i qi) 2^E relative to 2^eref: a
// high word (integer part of value 2^(fix_shift - eref)) and a low word
// (fix_lo more bits), summed exactly across chunks
// The fields of a polynomial's plan that the tile kernels read per group: of the
// kernel's plan, or in a batch of the group's own plan (scalar loads).
typedef const FPE_CONST_AS int32_t *const_itable_t;
struct SegPlan {
    const_table_t cf;
    const_table32_t c32;
    const_itable_t sig32;
    int coef_shift, fix_shift, fix_lo;
    const_itable_t gprefix, gidx;    // G_p as prefix counts and as a list (sparse window sums)
    const_table_t gcoef;
    int f32comp;                     // FP32 blocks compensated (TwoSum/TwoProd)
};
typedef const FPE_CONST_AS DevPlan *const_plans_t;

template <bool B>
__device__ __forceinline__ SegPlan group_plan(const DevPlan &P, const EvalWs &W, int g) {
    if constexpr (B) {
        const int gp = __builtin_amdgcn_readfirstlane(W.gpoly[g]);
        const_plans_t pl = (const_plans_t)W.plans;
        return {(const_table_t)pl[gp].coef, (const_table32_t)pl[gp].coef32, (const_itable_t)pl[gp].sig32,
                pl[gp].coef_shift, pl[gp].fix_shift, pl[gp].fix_lo, (const_itable_t)pl[gp].gprefix,
                (const_itable_t)pl[gp].gidx, (const_table_t)pl[gp].gcoef, pl[gp].f32comp};
    } else {
        return {(const_table_t)P.coef, (const_table32_t)P.coef32, (const_itable_t)P.sig32,
                P.coef_shift, P.fix_shift, P.fix_lo, (const_itable_t)P.gprefix, (const_itable_t)P.gidx,
                (const_table_t)P.gcoef, P.f32comp};
    }
}

// ---- sparse window sums: Horner's rule over the list of G_p, each gap between
// two consecutive indices jumped by powers of z (the precomputed powers of the
// paper's implementation notes, Section 8.2, for lacunary windows).  A gap
// inside a chunk is below kChunkMax = 2^11, so z^(2^j), j < 11, suffice.
constexpr int kGapBits = 11;
constexpr int kSparseRun = 16;        // list entries of a run, at least (see sparse_tile)
constexpr int kSparseRunShift = 8;    // a run ends only between blocks of 2^8 indices

// z^(2^j) = (tr[j] + i ti[j]) 2^f[j] for j < nb, with max(|tr|, |ti|) in
// [1/2, 1] (rounded once from complex double-double squarings: relative error
// one rounding); t_0 = w 2^ez = z exactly
struct GapPowers { double tr[kGapBits], ti[kGapBits]; int f[kGapBits]; };

__device__ __forceinline__ void gap_powers(double wr, double wi, int ez, int nb, GapPowers &T) {
    T.tr[0] = wr;
    T.ti[0] = wi;
    T.f[0] = ez;
    CDD x = {wr, 0.0, wi, 0.0};
    long long ex = 0;
#pragma unroll
    for (int j = 1; j < kGapBits; ++j) {
        if (j < nb) {
            FPE_NO_CONTRACT
            x = cdd_sqr(x);
            ex *= 2;
            cdd_renorm(x, ex);
            T.tr[j] = x.rh + x.rl;
            T.ti[j] = x.ih + x.il;
            T.f[j] = (int)(ex + (long long)ez * (1LL << j));
        } else {
            T.tr[j] = 0.0;
            T.ti[j] = 0.0;
            T.f[j] = 0;
        }
    }
}

// (hr + i hi) 2^E <- (hr + i hi) 2^E z^(2^j)
__device__ __forceinline__ void gap_mul(double &hr, double &hi, int &E, const GapPowers &T, int j) {
    const double nr = fma(hr, T.tr[j], -(hi * T.ti[j]));
    hi = fma(hr, T.ti[j], hi * T.tr[j]);
    hr = nr;
    E += T.f[j];
}

// One entry (k, a_k) of a sparse window sum for this lane: the gap from the
// previous entry taken (z^gap by the binary digits of the wave-uniform gap),
// then a_k 2^-e where k lies in the lane's part [lo, hi].  Returns whether the
// lane ends its run before taking k (see sparse_tile).
__device__ __forceinline__ bool sparse_entry(const GapPowers &T, int k, double ar, double ai, int kprev, int lo,
                                             int hi, bool act, double &hr, double &hi_, int &e, int &kl, int &cnt) {
    const bool in = act && k >= lo && k <= hi;
    const bool mul = in && kl >= 0;
    // a run ends where it has kSparseRun entries and the next one lies in
    // another block of 2^kSparseRunShift indices than its last (a test on the
    // lane's own entries, so the runs do not depend on the other lanes)
    const bool brk = mul && cnt >= kSparseRun && (k >> kSparseRunShift) != (kl >> kSparseRunShift);
    if (brk) return true;
    const int gap = kprev - k;
    if (__ballot(mul) != 0) {
#pragma unroll
        for (int j = 0; j < kGapBits; ++j) {
            if ((gap >> j) == 0) break;
            if ((gap >> j) & 1)
                if (mul) gap_mul(hr, hi_, e, T, j);
        }
    }
    if (in) {
        hr += ldexp(ar, -e);
        hi_ += ldexp(ai, -e);
        kl = k;
        ++cnt;
    }
    return false;
}

// the running sum's mantissa folded into E (exact: a power of two moves)
__device__ __forceinline__ void sparse_renorm(double &Hr, double &Hi, int &E) {
    const double mx = fmax(fabs(Hr), fabs(Hi));
    if (mx != 0.0) {
        const int ex = exp_of(mx);
        Hr = ldexp(Hr, -ex);
        Hi = ldexp(Hi, -ex);
        E += ex;
    }
}

constexpr int kSpBatch = 4;   // list entries per scalar-load batch (16 B of indices, 64 B of coefficients)

__device__ __forceinline__ void load_entries(int *K, double *A, const_itable_t gidx, const_table_t gcoef, int i0) {
#pragma unroll
    for (int q = 0; q < kSpBatch; ++q) K[q] = gidx[i0 + q];
#pragma unroll
    for (int q = 0; q < 2 * kSpBatch; ++q) A[q] = gcoef[2 * i0 + q];
}

// Ends a run of a sparse window sum (lanes with go): the run's sum
// (hr + i hi) 2^e, relative to the lowest index kl it took, carried down to lo
// (z^(kl - lo) by the binary digits of kl - lo < 2^nb) and added to the tile's
// sum (Hr + i Hi) 2^E; the run restarts empty.
__device__ __forceinline__ void sparse_flush(const GapPowers &T, int nb, int lo, bool go, double &hr, double &hi,
                                             int &e, int &kl, int &cnt, double &Hr, double &Hi, int &E) {
    if (!go) return;
    if (kl >= 0) {
        const int g2 = kl - lo;
#pragma unroll
        for (int j = 0; j < kGapBits; ++j)
            if (j < nb && ((g2 >> j) & 1)) gap_mul(hr, hi, e, T, j);
        if (Hr == 0.0 && Hi == 0.0) {
            Hr = hr; Hi = hi; E = e;
        } else {
            // both sums are renormalised: the sum of the tile's terms stays
            // within the window's range, and a part below 2^-2000 of it is lost
            const int sh = max(-2100, min(2100, e - E));
            Hr += ldexp(hr, sh);
            Hi += ldexp(hi, sh);
        }
        sparse_renorm(Hr, Hi, E);
    }
    hr = 0.0;
    hi = 0.0;
    e = 0;
    kl = -1;
    cnt = 0;
}

// The sparse form of one tile: H 2^E = sum over k in G_p within this lane's
// part [lo, hi] of the chunk of a_k z^(k - lo).  The indices of G_p within
// the tile's union part [Klo, Khi] are wave-uniform: their list entries come
// through the scalar cache in batches of kSpBatch, two batches in flight (as
// the dense steps' coefficients), from the top.  A lane takes the entries
// inside its part: z^gap between two of them by the binary digits of the gap
// (a product by z^(2^j) per digit), then the coefficient scaled by 2^-e.  The
// running sum keeps its binary exponent e apart (renormalised after every
// batch: exact), so no power of z need fit the double range on its own.  The
// rounded powers z^(2^j) are reused along the recurrence, so their rounding
// errors add up: a lane's entries are cut into runs (at least kSparseRun
// entries, ending at a block boundary of 2^kSparseRunShift indices, decided
// on the lane's own entries), each carried down to lo and added to the
// tile's sum, so a term passes through at most about kSparseRun + 2^8 gaps
// and one carry whatever the chunk length, and each lane's arithmetic does not
// depend on the other lanes.
__device__ __forceinline__ void sparse_tile(const SegPlan &S, const GapPowers &T, int nb, int Klo, int Khi, int lo,
                                            int hi, bool act, double &Hr, double &Hi, int &E) {
    Hr = 0.0;
    Hi = 0.0;
    E = 0;
    double hr_ = 0.0, hi_ = 0.0;                  // the current run
    int e_ = 0;
    int kl = -1;                                   // the lowest index this lane took in the run
    int cnt = 0;                                   //   and the entries it took
    const int pa = __builtin_amdgcn_readfirstlane(S.gprefix[Klo]);
    const int pb = __builtin_amdgcn_readfirstlane(S.gprefix[Khi + 1]);
    if (pb <= pa) return;
    int kprev = Khi + 1;                           // the first entry takes no gap (kl < 0 everywhere)
    const int nfull = (pb - pa) / kSpBatch;
    if (nfull > 0) {
        // batch b holds the entries [pb - kSpBatch (b + 1), pb - kSpBatch b)
        int KA[kSpBatch], KB[kSpBatch];
        double AA[2 * kSpBatch], AB[2 * kSpBatch];
        load_entries(KA, AA, S.gidx, S.gcoef, pb - kSpBatch);
        for (int bi = 0; bi < nfull; bi += 2) {
            wait_scalar_loads();
            __builtin_amdgcn_sched_barrier(0);
            if (bi + 1 < nfull) load_entries(KB, AB, S.gidx, S.gcoef, pb - kSpBatch * (bi + 2));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = kSpBatch - 1; q >= 0; --q) {
                const bool brk = sparse_entry(T, KA[q], AA[2 * q], AA[2 * q + 1], kprev, lo, hi, act, hr_, hi_, e_,
                                              kl, cnt);
                if (__ballot(brk) != 0) {
                    sparse_flush(T, nb, lo, brk, hr_, hi_, e_, kl, cnt, Hr, Hi, E);
                    sparse_entry(T, KA[q], AA[2 * q], AA[2 * q + 1], kprev, lo, hi, act && brk, hr_, hi_, e_,
                                 kl, cnt);
                }
                kprev = KA[q];
            }
            sparse_renorm(hr_, hi_, e_);
            if (bi + 1 < nfull) {
                wait_scalar_loads();
                __builtin_amdgcn_sched_barrier(0);
                if (bi + 2 < nfull) load_entries(KA, AA, S.gidx, S.gcoef, pb - kSpBatch * (bi + 3));
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = kSpBatch - 1; q >= 0; --q) {
                    const bool brk = sparse_entry(T, KB[q], AB[2 * q], AB[2 * q + 1], kprev, lo, hi, act, hr_, hi_, e_,
                                                  kl, cnt);
                    if (__ballot(brk) != 0) {
                        sparse_flush(T, nb, lo, brk, hr_, hi_, e_, kl, cnt, Hr, Hi, E);
                        sparse_entry(T, KB[q], AB[2 * q], AB[2 * q + 1], kprev, lo, hi, act && brk, hr_, hi_, e_,
                                     kl, cnt);
                    }
                    kprev = KB[q];
                }
                sparse_renorm(hr_, hi_, e_);
            }
        }
    }
    // the lowest (pb - pa) mod kSpBatch entries one by one
    for (int i = pb - kSpBatch * nfull - 1; i >= pa; --i) {
        const int k = S.gidx[i];
        const double ar = S.gcoef[2 * i], ai = S.gcoef[2 * i + 1];
        const bool brk = sparse_entry(T, k, ar, ai, kprev, lo, hi, act, hr_, hi_, e_, kl, cnt);
        if (__ballot(brk) != 0) {
            sparse_flush(T, nb, lo, brk, hr_, hi_, e_, kl, cnt, Hr, Hi, E);
            sparse_entry(T, k, ar, ai, kprev, lo, hi, act && brk, hr_, hi_, e_, kl, cnt);
        }
        kprev = k;
    }
    sparse_flush(T, nb, lo, true, hr_, hi_, e_, kl, cnt, Hr, Hi, E);
}

__device__ __forceinline__ void fix_add(const SegPlan &P, double qr, double qi, long long E, long long eref,
                                        long long &a0, long long &a1, long long &a2, long long &a3) {
    // (qr, qi) is not normalised: the table holds a_k 2^-coef_shift, so a
    // partial of small terms under a large coef_shift has a mantissa far below
    // 1 and needs a shift of up to about the coefficients' scale range (at most
    // 2 (958 - T)).  The window bound keeps the result below 2^(fix_shift +
    // bitlen(W) - 2) <= 2^58; the clamp only keeps ldexp's argument in range.
    long long sh = E - eref + P.fix_shift;
    sh = sh < -2200 ? -2200 : (sh > 2200 ? 2200 : sh);
    const double xr = ldexp(qr, (int)sh), xi = ldexp(qi, (int)sh);
    const double hr0 = trunc(xr), hi0 = trunc(xi);
    a0 += (long long)hr0;
    a1 += (long long)rint(ldexp(xr - hr0, P.fix_lo));
    a2 += (long long)hi0;
    a3 += (long long)rint(ldexp(xi - hi0, P.fix_lo));
}

__device__ __forceinline__ void fix_out(int fix_shift, int fix_lo, long long a0, long long a1, long long a2, long long a3,
                                        long long eref, double2 &m, long long &e) {
    const int f = fix_shift;
    const double vr = ldexp((double)a0, -f) + ldexp((double)a1, -f - fix_lo);
    const double vi = ldexp((double)a2, -f) + ldexp((double)a3, -f - fix_lo);
    normalise(vr, vi, eref, m, e);
}

// With D, the same pass also sums the derivative of the kept terms,
// Q'(z) = sum k a_k z^(k-1) over G_p within [l, r], into (md_out, ed_out).
// With SP, each tile runs the sparse form (sparse_tile) instead of Horner's
// rule over every index.  With FC, the FP32 blocks of plans that ask for it
// run the compensated recurrence (a variant of its own: its registers would
// otherwise spill in the FP64 kernel).
template <bool D, bool B, bool SP = false, bool FC = false>
__global__ __launch_bounds__(kWindowThreads) __attribute__((amdgpu_waves_per_eu(SP || FC ? 4 : (D ? 5 : 6))))
void k_window(DevPlan P, double2 *__restrict__ m_out,
                                                           long long *__restrict__ e_out,
                                                           double2 *__restrict__ md_out,
                                                           long long *__restrict__ ed_out, EvalWs W) {
    constexpr int kAccWords = D ? 8 : 4;
    const int lane = threadIdx.x % kWave;
    const int w = blockIdx.x * kWindowWaves + threadIdx.x / kWave;
    // per lane: the chained w^(c C) and w^C, and the fixed-point sums of the
    // segment (kept here, not in registers: they are touched once per tile)
    __shared__ double s_ch[4][kWindowThreads];
    __shared__ long long s_che[2][kWindowThreads];
    __shared__ long long s_acc[kAccWords][kWindowThreads];   // fixed-point sums of the segment
    __shared__ long long s_eref[kWindowThreads];              // eref of a lane whose window spans chunks
    if (w >= W.n_waves) return;
    const int nvalid = valid_points(W);
    const int G = (int)W.n_groups;
    const int C = W.chunk;
    int g, c, ge, ce;
    {
        const int2 st = W.wstart[w], en = W.wstart[w + 1];
        g = __builtin_amdgcn_readfirstlane(st.x);
        c = __builtin_amdgcn_readfirstlane(st.y);
        ge = __builtin_amdgcn_readfirstlane(en.x);
        ce = __builtin_amdgcn_readfirstlane(en.y);
    }
    resolve_tile(W, C, g, c);
    resolve_tile(W, C, ge, ce);
    // a wavefront may own no tile (a tile's work can exceed one share) and yet
    // lie inside a split group's owner range, where the finalize kernel reads
    // its slot 0; every other slot that kernel reads is written below
    if (g == ge && c == ce) {
        longlong2 *s0 = slot_pairs(W, 2 * (size_t)w);
        for (int q = 0; q < kAccWords / 2; ++q) s0[q * kWave + lane] = make_longlong2(0, 0);
    }
    // one pass per group segment: the consecutive tiles of one group this
    // wavefront owns
    while (g < G && !(g == ge && c == ce)) {
        const int glo = __builtin_amdgcn_readfirstlane(W.glo[g]);
        const int ghi = __builtin_amdgcn_readfirstlane(W.ghi[g]);
        const int clo = glo / C, chi = ghi / C;
        // the coefficient tables are read-only for the whole evaluation:
        // wave-uniform indices into them become scalar loads
        const SegPlan S = group_plan<B>(P, W, g);
        const_table_t cf = S.cf;
        const int seg_c0 = c;
        const int idx = g * kWave + lane;
        const bool valid = idx < nvalid;
        PointRec rc;
        if (valid) rc = W.srec[idx];
        else { rc.z = make_double2(0.0, 0.0); rc.l = 1; rc.r = 0; rc.j = -1; rc.pad = 0; }
        const int l = rc.l, r = rc.r;
        const bool multi = valid && (l / C != r / C);
        if (multi) s_eref[threadIdx.x] = W.eref[rc.j];
        // z = w 2^ez with max(|Re w|, |Im w|) in [1/2, 1) (a stand-in for lanes
        // without a point); z itself is rebuilt exactly from w when needed
        const int ez = valid ? exp_of(fmax(fabs(rc.z.x), fabs(rc.z.y))) : 0;
        const double wr = valid ? ldexp(rc.z.x, -ez) : 0.5, wi = valid ? ldexp(rc.z.y, -ez) : 0.0;
        PowState pw;                                      // chained powers of this segment
        for (int k = 0; k < kAccWords; ++k) s_acc[k][threadIdx.x] = 0;
        // FP32 tiles: z in FP32 (|z| in [2^-12, 2^12]) and z^8, 8 z^7 in FP64
        const bool z32ok = !valid || (ez >= -11 && ez <= 12);
        GapPowers gp;
        const int gbits = bit_length(C - 1);
        if constexpr (SP) gap_powers(wr, wi, ez, gbits, gp);
        Z32 z32 = {};
        if (!SP && S.c32) z32 = make_z32(ldexp(wr, ez), ldexp(wi, ez));
        for (;;) {
            // ---- tile (g, c): this lane's part [lo, hi] of chunk c
            const int c0 = c * C, c1 = c0 + C - 1;
            const int lo = max(l, c0), hi = min(r, c1);
            const bool act = valid && lo <= hi;
            const int Khi = __builtin_amdgcn_readfirstlane(wave_max(act ? hi : INT_MIN));
            const int Klo = __builtin_amdgcn_readfirstlane(wave_min(act ? lo : INT_MAX));
            const int Ahi = __builtin_amdgcn_readfirstlane(wave_min(act ? hi : INT_MAX));
            const int Alo = __builtin_amdgcn_readfirstlane(wave_max(act ? lo : INT_MIN));
            if (Khi >= Klo) {
                // z^lo first: w^l by binary powering where the window starts in this
                // chunk, the chained w^(c C) where it started earlier
                const int t = threadIdx.x;
                double pr, pi;
                long long pe;
                tile_power(pw, l, lo, act, c, C, wr, wi, s_ch, s_che, t, pr, pi, pe);
                Acc<D> acc;
                int es = 0;                       // binary exponent of a sparse tile's sum
                const double zr = ldexp(wr, ez), zi = ldexp(wi, ez);
                // FP32 for the common and top parts where the chunk and every
                // active lane's |z| allow it, then the ragged bottom in FP64
                bool f32 = SP;
                if constexpr (SP) {
                    sparse_tile(S, gp, gbits, Klo, Khi, lo, hi, act, acc.hr, acc.hi, es);
                } else {
                    if (S.c32 && C == kChunk && Ahi >= Alo) {
                        const int sg = __builtin_amdgcn_readfirstlane(S.sig32[c]);
                        f32 = sg != kNoFp32 && __ballot(act && !z32ok) == 0;
                        if (f32) {
                            // the compensated form sums values; a derivative
                            // pass runs the plain FP32 blocks for Q and Q'
                            bool comp = false;
                            if constexpr (FC && !D) {
                                comp = S.f32comp != 0;
                                if (comp) run_f32<D, true>(acc, z32, S.c32, sg, Khi, Alo, Ahi, hi);
                            }
                            if (!comp) run_f32<D, false>(acc, z32, S.c32, sg, Khi, Alo, Ahi, hi);
                            run_steps<kBottom>(acc, zr, zi, cf, Alo - 1, Klo, lo, hi);
                        }
                    }
                }
                if (!f32) {
                    if (Ahi >= Alo) {
                        run_steps<kTop>(acc, zr, zi, cf, Khi, Ahi + 1, lo, hi);
                        run_steps<kAll>(acc, zr, zi, cf, Ahi, Alo, lo, hi);
                        run_steps<kBottom>(acc, zr, zi, cf, Alo - 1, Klo, lo, hi);
                    } else {
                        run_steps<kBoth>(acc, zr, zi, cf, Khi, Klo, lo, hi);
                    }
                }
                if (act) {
                    // times z^lo = (pr + i pi) 2^(pe + lo ez)
                    const long long E = S.coef_shift + pe + (long long)lo * ez + es;
                    const double qr = fma(acc.hr, pr, -acc.hi * pi);
                    const double qi = fma(acc.hr, pi, acc.hi * pr);
                    double dqr = 0.0, dqi = 0.0;
                    if constexpr (D) {
                        // d/dz (z^lo H) = z^lo (lo H + z H') / z, and 1/z = conj(w) / |w|^2 2^-ez
                        FPE_NO_CONTRACT
                        const double ur = fma((double)lo, acc.hr, fma(zr, acc.dr, -zi * acc.di));
                        const double ui = fma((double)lo, acc.hi, fma(zr, acc.di, zi * acc.dr));
                        const double inv = 1.0 / fma(wr, wr, wi * wi);
                        const double vr = fma(ur, wr, ui * wi) * inv, vi = fma(ui, wr, -ur * wi) * inv;
                        dqr = fma(vr, pr, -vi * pi);
                        dqi = fma(vr, pi, vi * pr);
                    }
                    if (!multi) {
                        double2 m;
                        long long e;
                        normalise(qr, qi, E, m, e);
                        const int j = W.srec[idx].j;
                        m_out[j] = m;
                        e_out[j] = e;
                        if constexpr (D) {
                            normalise(dqr, dqi, E - ez, m, e);
                            md_out[j] = m;
                            ed_out[j] = e;
                        }
                    } else {
                        const long long eref = s_eref[t];
                        fix_add(S, qr, qi, E, eref, s_acc[0][t], s_acc[1][t], s_acc[2][t], s_acc[3][t]);
                        if constexpr (D)
                            fix_add(S, dqr, dqi, E - ez, deriv_eref(eref, ez, r), s_acc[4][t], s_acc[5][t],
                                    s_acc[6][t], s_acc[7][t]);
                    }
                }
            }
            // ---- next tile of this segment, if this wavefront owns it
            if (c == chi || (g == ge && c + 1 == ce)) break;
            ++c;
        }
        // ---- end of the segment: a group done entirely here is written out; a
        // part of a group leaves its fixed-point sums in this wavefront's slot 0
        // if earlier wavefronts own the group's first tiles, and in slot 1 if
        // later ones own its last tiles (a middle owner writes both; only the
        // first segment can start inside a group, only the last can end inside
        // one, so no slot is written twice)
        if (multi) {
            const int t = threadIdx.x;
            if (seg_c0 == clo && c == chi) {
                double2 m;
                long long e;
                const long long eref = s_eref[t];
                fix_out(S.fix_shift, S.fix_lo, s_acc[0][t], s_acc[1][t], s_acc[2][t], s_acc[3][t], eref, m, e);
                const int j = W.srec[idx].j;
                m_out[j] = m;
                e_out[j] = e;
                if constexpr (D) {
                    fix_out(S.fix_shift, S.fix_lo, s_acc[4][t], s_acc[5][t], s_acc[6][t], s_acc[7][t], deriv_eref(eref, ez, r), m, e);
                    md_out[j] = m;
                    ed_out[j] = e;
                }
            } else {
                if (seg_c0 != clo) {
                    longlong2 *sl = slot_pairs(W, 2 * (size_t)w);
                    for (int q = 0; q < kAccWords / 2; ++q)
                        sl[q * kWave + lane] = make_longlong2(s_acc[2 * q][t], s_acc[2 * q + 1][t]);
                }
                if (c != chi) {
                    longlong2 *sl = slot_pairs(W, 2 * (size_t)w + 1);
                    for (int q = 0; q < kAccWords / 2; ++q)
                        sl[q * kWave + lane] = make_longlong2(s_acc[2 * q][t], s_acc[2 * q + 1][t]);
                }
            }
        }
        if (c < chi) { ++c; }
        else { ++g; c = -1; resolve_tile(W, C, g, c); }
    }
}

// Points whose window spans several chunks, in groups split across
// wavefronts: the sum of the fixed-point partials the owning wavefronts left
// in their slots (integer sums: the order does not matter).  The first owner
// holds the group in its slot 1, every later owner in its slot 0.  Work items
// of the grid's wavefronts: the short split groups k_partition listed (one
// wavefront sums all owners), then the pieces of the long groups (a wavefront
// sums kLongPiece owners; a group of several pieces adds them to its
// accumulator with device-scope atomics, and the piece that arrives last
// writes the outputs).  A long group's slots, up to one per window
// wavefront, are so read by many compute units at once.
constexpr int kFinalThreads = 256;
constexpr int kFinalBlocks = 4096;    // workgroups of the finalize grid, at most
constexpr int kLongPer = kLongLds / kFinalThreads;   // long groups per thread in the piece scan

// the outputs of one point of a split group from its summed partials
template <bool D, bool B>
__device__ __forceinline__ void final_out(const DevPlan &P, const EvalWs &W, int g, const PointRec &rc,
                                          int j, long long eref, const long long *a, double2 *__restrict__ m_out,
                                          long long *__restrict__ e_out, double2 *__restrict__ md_out,
                                          long long *__restrict__ ed_out) {
    double2 m;
    long long e;
    int fs = P.fix_shift, fl = P.fix_lo;
    if constexpr (B) {
        const DevPlan &Q = W.plans[W.gpoly[g]];
        fs = Q.fix_shift;
        fl = Q.fix_lo;
    }
    fix_out(fs, fl, a[0], a[1], a[2], a[3], eref, m, e);
    m_out[j] = m;
    e_out[j] = e;
    if constexpr (D) {
        const int ez = exp_of(fmax(fabs(rc.z.x), fabs(rc.z.y)));
        fix_out(fs, fl, a[4], a[5], a[6], a[7], deriv_eref(eref, ez, rc.r), m, e);
        md_out[j] = m;
        ed_out[j] = e;
    }
}

// adds the slots of owners w0 .. min(w0 + kU - 1, wy) of a group whose first
// owner is wx to a; the loads are all issued before the first sum
template <int kAccWords, int kU>
__device__ __forceinline__ void add_slots(const EvalWs &W, int wx, int wy, int w0, int lane, long long *a) {
    longlong2 x[kU][kAccWords / 2];
    const uint32_t loff = (uint32_t)lane * sizeof(longlong2);   // one lane offset for every slot
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int w = __builtin_amdgcn_readfirstlane(w0 + u);   // the same for the whole wavefront
        if (w <= wy) {
            const char *sb = reinterpret_cast<const char *>(slot_pairs(W, 2 * (size_t)w + (w == wx ? 1 : 0)));
#pragma unroll
            for (int k = 0; k < kAccWords / 2; ++k)
                x[u][k] = *reinterpret_cast<const longlong2 *>(sb + loff + k * kWave * sizeof(longlong2));
        } else {
#pragma unroll
            for (int k = 0; k < kAccWords / 2; ++k) x[u][k] = make_longlong2(0, 0);
        }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
        for (int k = 0; k < kAccWords / 2; ++k) {
            a[2 * k] += x[u][k].x;
            a[2 * k + 1] += x[u][k].y;
        }
}

template <bool D, bool B>
__global__ __launch_bounds__(kFinalThreads, D ? 4 : 7) void k_finalize(DevPlan P, double2 *__restrict__ m_out,
                                                            long long *__restrict__ e_out,
                                                            double2 *__restrict__ md_out,
                                                            long long *__restrict__ ed_out, EvalWs W) {
    constexpr int kAccWords = D ? 8 : 4;
    constexpr int nq = kFinalThreads / kWave;
    __shared__ int s_pre[kLongLds];           // inclusive prefix of the long groups' pieces
    __shared__ int s_wsum[nq];
    const int lane = threadIdx.x % kWave, q = threadIdx.x / kWave;
    const int nsplit = W.ctl[8], nlong = W.ctl[9];
    const int nvalid = valid_points(W);
    int npieces = 0;
    if (nlong > 0) {                                   // the same for every thread
        const int i0 = threadIdx.x * kLongPer;
        int cnt[kLongPer] = {};
        int sum = 0;
        if (i0 < nlong) {
            // clamped indices, all loads issued before the first use
            int4 lg[kLongPer];
#pragma unroll
            for (int e = 0; e < kLongPer; ++e) lg[e] = W.lgroups[min(i0 + e, nlong - 1)];
#pragma unroll
            for (int e = 0; e < kLongPer; ++e) {
                cnt[e] = i0 + e < nlong ? long_pieces(lg[e]) : 0;
                sum += cnt[e];
            }
        }
        int incl = sum;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int t = __shfl_up(incl, d);
            if (lane >= d) incl += t;
        }
        if (lane == kWave - 1) s_wsum[q] = incl;
        __syncthreads();
        int run = incl - sum;
        for (int r = 0; r < nq; ++r) {
            const int ws = s_wsum[r];
            if (r < q) run += ws;
            npieces += ws;
        }
#pragma unroll
        for (int e = 0; e < kLongPer; ++e) {
            run += cnt[e];
            if (i0 + e < nlong) s_pre[i0 + e] = run;
        }
        __syncthreads();
    }
    // work items in wavefront order q * gridDim.x + blockIdx.x: neighbouring
    // items go to different workgroups
    const int nwork = nsplit + npieces;
    for (int u = q * (int)gridDim.x + (int)blockIdx.x; u < nwork; u += (int)gridDim.x * nq) {
        // the owners [wa, wb] this item sums, of group g whose first owner is wx
        int g, wx, wa, wb, li = -1, np = 0;
        if (u < nsplit) {
            const int4 sp = W.split[u];
            g = sp.x;
            wx = wa = sp.y;
            wb = sp.z;
        } else {
            const int pid = u - nsplit;
            int lo = 0, hi = nlong - 1;                // the first long group with s_pre > pid
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_pre[mid] > pid) hi = mid; else lo = mid + 1;
            }
            li = lo;
            const int first = li > 0 ? s_pre[li - 1] : 0;
            np = s_pre[li] - first;
            const int4 lg = W.lgroups[li];             // group, first and last owner
            g = lg.x;
            wx = lg.y;
            wa = lg.y + (pid - first) * kLongPiece;
            wb = min(lg.z, wa + kLongPiece - 1);
        }
        const int p = g * kWave + lane;
        PointRec rc;
        int j = 0;
        long long eref = 0;
        if (p < nvalid) {                              // requested with the slots
            rc = W.srec[p];
            j = rc.j;
            if (j >= 0) eref = W.eref[j];
        }
        long long a[kAccWords] = {};
        for (int w0 = wa; w0 <= wb; w0 += 4) add_slots<kAccWords, 4>(W, wx, wb, w0, lane, a);
        bool last = true;
        if (np > 1) {
            // one of several pieces of a long group: its sums go to the
            // group's accumulator; the piece that arrives last writes the
            // outputs (a group of one piece writes them at once)
            unsigned long long *acc =
                reinterpret_cast<unsigned long long *>(W.lacc) + ((size_t)li * kWave + lane) * kSlotWords;
#pragma unroll
            for (int t = 0; t < kAccWords; ++t) atomicAdd(acc + t, (unsigned long long)a[t]);
            __threadfence();                           // the sums before the count
            int done = 0;
            if (lane == 0) done = atomicAdd(W.lcnt + li, 1);
            last = __shfl(done, 0) == np - 1;
            if (last) {                                // every other piece has added its sums
                __threadfence();
#pragma unroll
                for (int t = 0; t < kAccWords; ++t)
                    a[t] = (long long)__hip_atomic_load(acc + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (last && p < nvalid && rc.l / W.chunk != rc.r / W.chunk)
            final_out<D, B>(P, W, g, rc, j, eref, a, m_out, e_out, md_out, ed_out);
    }
}

// Adjoint of the window sums with respect to the coefficients: for upstream
// gradients gin_j (per point, input order), grad_a[k] += sum over the points j
// whose kept terms include k (k in G_p within [l_j, r_j]) of gin_j conj(z_j)^k
// (the convention of complex autograd: the gradient of a holomorphic map is
// the upstream gradient times the conjugate derivative, here d Q / d a_k = z^k).
// Same tiles and partition as k_window: each lane starts from gin conj(z^lo)
// (z^lo by tile_power) and multiplies by conj(z) per step, mantissa and
// exponent apart, so that a term is rounded to the double range only when it
// is emitted; the 64 lanes' terms of four consecutive k at a time are summed
// across the wavefront by a reduce-scatter (a fixed order).
//
// The sums over wavefronts are exact, so grad_a does not depend on the order
// in which tiles finish.  Two passes over the tiles: with BOUND, each term's
// magnitude is bounded from above, |gin conj(z)^k| < 2^(e + 1 + k lambda),
// lambda = log2|z| and e the exponent of gin (no products, no powering), and
// per k the largest bound, plus two, goes to aexp[k] (integer atomicMax).
// Then every term goes to fixed point relative to 2^aexp[k]: v 2^(S -
// aexp[k]) split into an integer part and S fraction bits, two int64 words per
// component, summed over the wavefront and added with integer atomics, all
// exact: grad_a depends neither on the order of the additions nor on which
// points share a wavefront.  A term stays below 2^(S - 2) in these units and
// an index gathers at most n terms, so S = min(47, 62 - bitlen(n)) keeps every
// word below 2^62 and a wavefront's sums exact in FP64; the fraction word
// rounds each term to 2^(aexp[k] - 2 S), below 2^-70 of the largest term for
// n up to 2^24.  A non-finite term sets
// aflag[k] (the output is then NaN).  k_adj_out turns the words into grad_a.
constexpr int kRenormSteps = 256;   // products by conj(w) between two folds of the term mantissa

// ---- cross-lane sums for four indices at a time, without the LDS crossbar:
// the gfx950 half swaps v_permlane32_swap (lanes 32..63 of the first operand
// with lanes 0..31 of the second) and v_permlane16_swap (odd rows of the first
// with even rows of the second) bring index r's values into row r (lanes
// 16 r .. 16 r + 15), and DPP row shifts sum each row into its lane 15.
template <class F>
__device__ __forceinline__ void swap32(F &a, F &b);
template <>
__device__ __forceinline__ void swap32<int>(int &a, int &b) {
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)a, (unsigned)b, false, false);
    a = (int)r[0];
    b = (int)r[1];
}
template <>
__device__ __forceinline__ void swap32<double>(double &a, double &b) {
    const long long A = __double_as_longlong(a), B = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)A, (unsigned)B, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(A >> 32), (unsigned)(B >> 32), false, false);
    a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
    b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}
template <class F>
__device__ __forceinline__ void swap16(F &a, F &b);
template <>
__device__ __forceinline__ void swap16<int>(int &a, int &b) {
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)a, (unsigned)b, false, false);
    a = (int)r[0];
    b = (int)r[1];
}
template <>
__device__ __forceinline__ void swap16<double>(double &a, double &b) {
    const long long A = __double_as_longlong(a), B = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)A, (unsigned)B, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(A >> 32), (unsigned)(B >> 32), false, false);
    a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
    b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

// x from lane i - n of the same row (lanes before the row's n-th: 0.0)
template <int N>
__device__ __forceinline__ double row_shr(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x110 + N, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x110 + N, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int N>
__device__ __forceinline__ int row_shr_max(int x) {
    return max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x110 + N, 0xf, 0xf, false));
}

// per lane four values v[0..3] (one per index): returns in lane 16 r + 15 the
// sum (ADD) or the largest value over the 64 lanes of index r
template <class F, bool ADD>
__device__ __forceinline__ F reduce4(F v0, F v1, F v2, F v3) {
    swap32(v0, v2);
    swap32(v1, v3);
    F a = ADD ? v0 + v2 : max(v0, v2), b = ADD ? v1 + v3 : max(v1, v3);   // rows 0, 1: indices 0, 1; rows 2, 3: 2, 3
    swap16(a, b);
    F x = ADD ? a + b : max(a, b);                                         // row r: index r
    if constexpr (ADD) {
        x += row_shr<1>(x);
        x += row_shr<2>(x);
        x += row_shr<4>(x);
        x += row_shr<8>(x);
    } else {
        x = row_shr_max<1>(x);
        x = row_shr_max<2>(x);
        x = row_shr_max<4>(x);
        x = row_shr_max<8>(x);
    }
    return x;
}

// which of k0 .. k0 + 3 (at most khi) are in G_p (the nonzero entries of the
// masked table), as 4 bits: wave-uniform indices, so scalar loads, issued at
// the top of a step and waited for only where the sums are added
__device__ __forceinline__ int gp_mask4(const DevPlan &P, int k0, int khi) {
    const_table_t cf = (const_table_t)P.coef;
    int m = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = min(k0 + j, khi);
        const double re = cf[2 * k], im = cf[2 * k + 1];
        if (k0 + j <= khi && (re != 0.0 || im != 0.0)) m |= 1 << j;
    }
    return m;
}

// the exponent bound of a wavefront term (clamped far outside the FP64 range)
__device__ __forceinline__ int term_bound(double gam, double lam, int k) {
    const double b = ceil(fma((double)k, lam, gam));
    return (int)fmin(4000.0, fmax(-4000.0, b)) + 2;
}

// v 2^sh in fixed point: its integer part h and S fraction bits l, both
// integers held exactly in doubles (|h| < 2^(S - 2), |l| <= 2^S with S <= 47,
// so sums of 64 of them stay exact in FP64); l is rounded when v 2^sh has bits
// below 2^-S
__device__ __forceinline__ void to_fixed(double v, int sh, int S, double &h, double &l) {
    const double x = ldexp(v, sh);
    h = trunc(x);
    l = rint(ldexp(x - h, S));
}

// the passes of k_adjoint and k_adj_zero: the bounds, the exact sums, or (the
// atomic mode) the wavefront sums added to grad_a with FP64 atomics
enum AdjPass { kAdjBound = 0, kAdjExact = 1, kAdjAtomic = 2 };

template <int MODE>
__global__ __launch_bounds__(kWindowThreads) void k_adjoint(DevPlan P, const double2 *__restrict__ gin,
                                                            const long long *__restrict__ gexp, AdjAcc A, int S,
                                                            double2 *__restrict__ grad_a, EvalWs W) {
    constexpr bool BOUND = MODE == kAdjBound;
    const int lane = threadIdx.x % kWave;
    const int w = blockIdx.x * kWindowWaves + threadIdx.x / kWave;
    __shared__ double s_ch[4][kWindowThreads];
    __shared__ long long s_che[2][kWindowThreads];
    if (w >= W.n_waves) return;
    const int nvalid = valid_points(W);
    const int G = (int)W.n_groups;
    const int C = W.chunk;
    int g, c, ge, ce;
    {
        const int2 st = W.wstart[w], en = W.wstart[w + 1];
        g = __builtin_amdgcn_readfirstlane(st.x);
        c = __builtin_amdgcn_readfirstlane(st.y);
        ge = __builtin_amdgcn_readfirstlane(en.x);
        ce = __builtin_amdgcn_readfirstlane(en.y);
    }
    resolve_tile(W, C, g, c);
    resolve_tile(W, C, ge, ce);
    while (g < G && !(g == ge && c == ce)) {
        const int ghi = __builtin_amdgcn_readfirstlane(W.ghi[g]);
        const int chi = ghi / C;
        const int idx = g * kWave + lane;
        const bool valid = idx < nvalid;
        PointRec rc;
        if (valid) rc = W.srec[idx];
        else { rc.z = make_double2(0.0, 0.0); rc.l = 1; rc.r = 0; rc.j = -1; rc.pad = 0; }
        const int l = rc.l, r = rc.r;
        const int ez = valid ? exp_of(fmax(fabs(rc.z.x), fabs(rc.z.y))) : 0;
        const double wr = valid ? ldexp(rc.z.x, -ez) : 0.5, wi = valid ? ldexp(rc.z.y, -ez) : 0.0;
        // g = (gr + i gi) 2^eg with max(|gr|, |gi|) in [1/2, 1) (0 for no point)
        double gr = 0.0, gi = 0.0;
        int eg = 0;
        if (valid) {
            const double2 gj = gin[rc.j];
            const double gm = fmax(fabs(gj.x), fabs(gj.y));
            if (gm != 0.0 && isfinite(gm)) { eg = exp_of(gm); gr = ldexp(gj.x, -eg); gi = ldexp(gj.y, -eg); }
            else { gr = gj.x; gi = gj.y; }
            // upstream gradients given as g 2^-gexp: the exponent joins E below
            if (gexp) {
                long long x = (long long)eg - gexp[rc.j];
                eg = (int)(x < -1000000000LL ? -1000000000LL : (x > 1000000000LL ? 1000000000LL : x));
            }
        }
        // BOUND: |g| < 2^(eg + 1/2) for a finite nonzero g (no term otherwise)
        const bool gterm = valid && (gr != 0.0 || gi != 0.0);
        const double gam = (double)eg + 1.0;
        const double lam = valid ? log2_abs(rc.z) : 0.0;
        PowState pw;
        for (;;) {
            const int c0 = c * C, c1 = c0 + C - 1;
            const int lo = max(l, c0), hi = min(r, c1);
            const bool act = valid && lo <= hi;
            const int Khi = __builtin_amdgcn_readfirstlane(wave_max(act ? hi : INT_MIN));
            const int Klo = __builtin_amdgcn_readfirstlane(wave_min(act ? lo : INT_MAX));
            if (BOUND && Khi >= Klo) {
                // the largest bound per k
                for (int k0 = Klo; k0 <= Khi; k0 += 4) {
                    const int gm = gp_mask4(P, k0, Khi);
                    int e[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int k = k0 + j;
                        e[j] = (gterm && act && k >= lo && k <= hi) ? term_bound(gam, lam, k) : INT_MIN;
                    }
                    const int x = reduce4<int, false>(e[0], e[1], e[2], e[3]);
                    const int k = k0 + (lane >> 4);
                    // (a read of the current bound before the atomic, to skip
                    // it where the bound is reached, measured slower: the
                    // read's latency is exposed at every step)
                    if ((lane & 15) == 15 && ((gm >> (lane >> 4)) & 1) && x != INT_MIN) atomicMax(A.aexp + k, x);
                }
            }
            if (!BOUND && Khi >= Klo) {
                const int t = threadIdx.x;
                double pr, pi;
                long long pe;
                tile_power(pw, l, lo, act, c, C, wr, wi, s_ch, s_che, t, pr, pi, pe);
                // term k = (tr + i ti) 2^E: the mantissa g conj(w^k) and the
                // exponent eg + pe + k ez apart; only the emitted term is scaled
                // (and may saturate or flush).  |w| lies in [1/2, 2^(1/2)), so
                // the mantissa is folded into E every kRenormSteps products
                // (within [2^-258, 2^129] of its start between two folds, for
                // any chunk length)
                double tr = fma(gr, pr, gi * pi);
                double ti = fma(gi, pr, -gr * pi);
                long long E = (long long)eg + pe + (long long)lo * ez;
                // four indices at a time: each lane's four terms, then their
                // sums over the wavefront (reduce4)
                for (int k0 = Klo; k0 <= Khi; k0 += 4) {
                    if (((k0 - Klo) & (kRenormSteps - 1)) == 0 && k0 != Klo) {
                        // exact: a power of two moves from the mantissa to E
                        const double mx = fmax(fabs(tr), fabs(ti));
                        if (mx != 0.0 && isfinite(mx)) {
                            const int ex = exp_of(mx);
                            tr = ldexp(tr, -ex);
                            ti = ldexp(ti, -ex);
                            E += ex;
                        }
                    }
                    const int gm = gp_mask4(P, k0, Khi);
                    if constexpr (MODE == kAdjAtomic) {
                        // the terms as they are, their wavefront sums (fixed
                        // order) added to grad_a with FP64 atomics
                        double vr[4], vi[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int k = k0 + j;
                            vr[j] = 0.0;
                            vi[j] = 0.0;
                            if (act && k >= lo && k <= hi) {
                                const int sh = (int)(E < -2200 ? -2200 : (E > 2200 ? 2200 : E));
                                vr[j] = ldexp(tr, sh);
                                vi[j] = ldexp(ti, sh);
                                const double nr = fma(tr, wr, ti * wi);       // times conj(w)
                                ti = fma(ti, wr, -tr * wi);
                                tr = nr;
                                E += ez;
                            }
                        }
                        const double xr = reduce4<double, true>(vr[0], vr[1], vr[2], vr[3]);
                        const double xi = reduce4<double, true>(vi[0], vi[1], vi[2], vi[3]);
                        const int k = k0 + (lane >> 4);
                        if ((lane & 15) == 15 && ((gm >> (lane >> 4)) & 1) && (xr != 0.0 || xi != 0.0)) {
                            atomicAdd(&grad_a[k].x, xr);
                            atomicAdd(&grad_a[k].y, xi);
                        }
                        continue;
                    }
                    // each term to fixed point relative to its index's scale
                    // 2^aexp[k] (four words: integer and fraction parts of
                    // Re and Im), so that every sum below is exact
                    int ek[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        ek[j] = k0 + j <= Khi ? __builtin_amdgcn_readfirstlane(A.aexp[k0 + j]) : 0;
                    double wv[4][4];
                    int bad = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int k = k0 + j;
                        wv[j][0] = wv[j][1] = wv[j][2] = wv[j][3] = 0.0;
                        if (act && k >= lo && k <= hi) {
                            const int sh = (int)(E < -2200 ? -2200 : (E > 2200 ? 2200 : E));
                            const double vr = ldexp(tr, sh), vi = ldexp(ti, sh);
                            if (!isfinite(vr) || !isfinite(vi)) {
                                bad |= 1 << j;
                            } else if (vr != 0.0 || vi != 0.0) {
                                const int fs = max(-2200, min(2200, S - ek[j]));
                                to_fixed(vr, fs, S, wv[j][0], wv[j][1]);
                                to_fixed(vi, fs, S, wv[j][2], wv[j][3]);
                            }
                            const double nr = fma(tr, wr, ti * wi);       // times conj(w)
                            ti = fma(ti, wr, -tr * wi);
                            tr = nr;
                            E += ez;
                        }
                    }
                    // the 64 lanes' words per index (sums of integers below
                    // 2^53: exact in any order)
                    double x[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) x[q] = reduce4<double, true>(wv[0][q], wv[1][q], wv[2][q], wv[3][q]);
                    const int k = k0 + (lane >> 4);
                    // only terms of G_p: their coefficients are the nonzero
                    // entries of the masked table
                    if ((lane & 15) == 15 && ((gm >> (lane >> 4)) & 1) &&
                        (x[0] != 0.0 || x[1] != 0.0 || x[2] != 0.0 || x[3] != 0.0)) {
                        unsigned long long *wd = reinterpret_cast<unsigned long long *>(A.acc + 4 * (size_t)k);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (x[q] != 0.0) atomicAdd(wd + q, (unsigned long long)(long long)x[q]);
                    }
                    // a non-finite term makes its index NaN
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (__ballot((bad >> j) & 1) != 0 && lane == 0 && ((gm >> j) & 1)) atomicOr(A.aflag + k0 + j, 1);
                    }
                }
            }
            if (c == chi || (g == ge && c + 1 == ce)) break;
            ++c;
        }
        if (c < chi) { ++c; }
        else { ++g; c = -1; resolve_tile(W, C, g, c); }
    }
}

__global__ __launch_bounds__(256) void k_zero2(double2 *__restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = make_double2(0.0, 0.0);
}

// grad_a's accumulators start empty: no bound, no flag, zero words
__global__ __launch_bounds__(256) void k_adj_init(AdjAcc A, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    A.aexp[i] = INT_MIN;
    A.aflag[i] = 0;
    longlong2 *w = reinterpret_cast<longlong2 *>(A.acc + 4 * i);
    w[0] = make_longlong2(0, 0);
    w[1] = make_longlong2(0, 0);
}

// The points z = 0 (no window; their kept term is a_0 alone when a_0 != 0):
// grad_a[0] += gin 2^-gexp.  With BOUND, aexp[0] rises to the terms' bound;
// then each term goes to fixed point like k_adjoint's, and each workgroup adds
// the integer sum of its points' words (exact).
template <int MODE>
__global__ __launch_bounds__(256) void k_adj_zero(DevPlan P, const double2 *__restrict__ z, int n,
                                                  const double2 *__restrict__ gin, const long long *__restrict__ gexp,
                                                  AdjAcc A, int S, double2 *__restrict__ grad_a) {
    constexpr bool BOUND = MODE == kAdjBound;
    __shared__ long long s_w[4][256];
    __shared__ int s_e[256];
    __shared__ double s_d[2][256];
    const int t = threadIdx.x, j = blockIdx.x * 256 + t;
    double vr = 0.0, vi = 0.0;
    bool term = false;
    if (j < n && P.nh > 0 && P.v == 0) {
        const double2 zz = z[j];
        if (zz.x == 0.0 && zz.y == 0.0) {
            const double2 g = gin[j];
            const long long gx = gexp ? gexp[j] : 0;
            const int sh = (int)(gx > 2200 ? 2200 : (gx < -2200 ? -2200 : gx));
            vr = ldexp(g.x, -sh);
            vi = ldexp(g.y, -sh);
            term = vr != 0.0 || vi != 0.0;
        }
    }
    const double m = fmax(fabs(vr), fabs(vi));
    if (BOUND) {
        // |v| < 2^(exp_of(m) + 1/2): the same margin as term_bound
        s_e[t] = term && isfinite(m) ? exp_of(m) + 3 : INT_MIN;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) s_e[t] = max(s_e[t], s_e[t + o]);
            __syncthreads();
        }
        if (t == 0 && s_e[0] != INT_MIN) atomicMax(A.aexp, s_e[0]);
        return;
    }
    if constexpr (MODE == kAdjAtomic) {
        s_d[0][t] = vr;
        s_d[1][t] = vi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) { s_d[0][t] += s_d[0][t + o]; s_d[1][t] += s_d[1][t + o]; }
            __syncthreads();
        }
        if (t == 0 && (s_d[0][0] != 0.0 || s_d[1][0] != 0.0)) {
            atomicAdd(&grad_a[0].x, s_d[0][0]);
            atomicAdd(&grad_a[0].y, s_d[1][0]);
        }
        return;
    }
    double w[4] = {0.0, 0.0, 0.0, 0.0};
    const bool bad = term && !isfinite(m);
    if (term && !bad) {
        const int fs = max(-2200, min(2200, S - A.aexp[0]));
        to_fixed(vr, fs, S, w[0], w[1]);
        to_fixed(vi, fs, S, w[2], w[3]);
    }
    for (int q = 0; q < 4; ++q) s_w[q][t] = (long long)w[q];
    if (__syncthreads_or(bad) && t == 0) atomicOr(A.aflag, 1);
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o)
            for (int q = 0; q < 4; ++q) s_w[q][t] += s_w[q][t + o];
        __syncthreads();
    }
    if (t == 0) {
        unsigned long long *wd = reinterpret_cast<unsigned long long *>(A.acc);
        for (int q = 0; q < 4; ++q)
            if (s_w[q][0] != 0) atomicAdd(wd + q, (unsigned long long)s_w[q][0]);
    }
}

// one component of grad_a[k] from its two words: (h 2^S + l) 2^(aexp - 2 S)
__device__ __forceinline__ double fixed_value(long long h, long long l, int S, int E) {
    const long long t = h + (l >> S);                  // l = (l >> S) 2^S + r, 0 <= r < 2^S
    const long long r = l - ((l >> S) << S);
    const double v = fma((double)t, ldexp(1.0, S), (double)r);
    return ldexp(v, max(-2200, min(2200, E - 2 * S)));
}

__global__ __launch_bounds__(256) void k_adj_out(AdjAcc A, int64_t nacc, int64_t n, int S,
                                                 double2 *__restrict__ grad_a) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    double2 v = make_double2(0.0, 0.0);
    if (k < nacc) {
        const int E = A.aexp[k];
        if (A.aflag[k]) {
            v = make_double2(__builtin_nan(""), __builtin_nan(""));
        } else if (E != INT_MIN) {
            const long long *w = A.acc + 4 * k;
            v = make_double2(fixed_value(w[0], w[1], S, E), fixed_value(w[2], w[3], S, E));
        }
    }
    grad_a[k] = v;
}

// Per point: the gradient with respect to z, gin conj(Q'(z)) with Q' = md 2^ed
// (NaN for a non-finite z).
__global__ __launch_bounds__(256) void k_grad_z(const double2 *__restrict__ z, int n,
                                                const double2 *__restrict__ gin, const long long *__restrict__ gexp,
                                                const double2 *__restrict__ md, const long long *__restrict__ ed,
                                                double2 *__restrict__ grad_z) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double2 zz = z[j];
    double2 g = gin[j];
    const long long gx = gexp ? gexp[j] : 0;
    if (!isfinite(zz.x) || !isfinite(zz.y)) {
        grad_z[j] = make_double2(__builtin_nan(""), __builtin_nan(""));
    } else {
        const double2 b = md[j];
        long long sh = ed[j] - gx;
        sh = sh < -2200 ? -2200 : (sh > 2200 ? 2200 : sh);
        grad_z[j] = make_double2(ldexp(fma(g.x, b.x, g.y * b.y), (int)sh), ldexp(fma(g.y, b.x, -g.x * b.y), (int)sh));
    }
}

int g_num_cu = 0;
// the kernels that run the (group, chunk) tiles: values, values and
// derivatives, adjoint
enum TileKernel {
    kTileValue = 0, kTileDeriv = 1, kTileAdjoint = 2, kTileBatch = 3, kTileSparse = 4, kTileComp = 5, kTileBatchComp = 6,
    kTileKinds = 7
};
int g_window_blocks_per_cu[kTileKinds] = {};
int g_final_blocks_per_cu[3] = {0, 0, 0};   // k_finalize: values, derivatives, batch

// wavefronts of a tile kernel: as many as are resident at once on the device
// (the partition hands each one an equal share, so none may wait for a second
// round)
int64_t window_waves(int kind) {
    const int b = g_window_blocks_per_cu[kind];
    return (int64_t)(g_num_cu > 0 ? g_num_cu : 256) * (b > 0 ? b : 1) * kWindowWaves;
}

// finalize workgroups: as many as are resident at once (a long group's
// workgroup must not wait for a later round), at most one per split group
unsigned final_blocks(int kind, int64_t n_waves) {
    const int b = g_final_blocks_per_cu[kind];
    const int64_t res = (int64_t)(g_num_cu > 0 ? g_num_cu : 256) * (b > 0 ? b : 1);
    const int64_t need = (n_waves + kFinalThreads / kWave - 1) / (kFinalThreads / kWave);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>({need, res, kFinalBlocks}));
}

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

// compute units and resident window workgroups per compute unit (once per process)
hipError_t device_setup() {
    if (g_num_cu > 0) return hipSuccess;
    int dev = 0, ncu = 0, nb[kTileKinds] = {};
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const void *kern[kTileKinds] = {reinterpret_cast<const void *>(k_window<false, false>),
                                    reinterpret_cast<const void *>(k_window<true, false>),
                                    reinterpret_cast<const void *>(k_adjoint<kAdjExact>),
                                    reinterpret_cast<const void *>(k_window<false, true>),
                                    reinterpret_cast<const void *>(k_window<false, false, true>),
                                    reinterpret_cast<const void *>(k_window<false, false, false, true>),
                                    reinterpret_cast<const void *>(k_window<false, true, false, true>)};
    for (int i = 0; i < kTileKinds && e == hipSuccess; ++i)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb[i], kern[i], kWindowThreads, 0);
    if (e != hipSuccess) return e;
    for (int i = 0; i < kTileKinds; ++i) g_window_blocks_per_cu[i] = nb[i] > 0 ? nb[i] : 1;
    const void *fin[3] = {reinterpret_cast<const void *>(k_finalize<false, false>),
                          reinterpret_cast<const void *>(k_finalize<true, false>),
                          reinterpret_cast<const void *>(k_finalize<false, true>)};
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
        int f = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&f, fin[i], kFinalThreads, 0);
        g_final_blocks_per_cu[i] = f > 0 ? f : 1;
    }
    if (e != hipSuccess) return e;
    g_num_cu = ncu > 0 ? ncu : 256;
    return hipSuccess;
}

// One Newton step per point, z - Q / Q' with Q = m 2^e and Q' = md 2^ed: the
// mantissa quotient times 2^(e - ed); Q' = 0 or a non-finite input gives NaN.
__global__ __launch_bounds__(256) void k_newton(const double2 *__restrict__ z, int n, const double2 *__restrict__ m,
                                                const long long *__restrict__ e, const double2 *__restrict__ md,
                                                const long long *__restrict__ ed, double2 *__restrict__ z_out) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double2 zz = z[j], a = m[j], b = md[j];
    const double den = fma(b.x, b.x, b.y * b.y);
    if (!(den > 0.0) || !isfinite(zz.x) || !isfinite(zz.y) || a.x != a.x) {
        z_out[j] = make_double2(__builtin_nan(""), __builtin_nan(""));
        return;
    }
    long long sh = e[j] - ed[j];
    sh = sh < -2200 ? -2200 : (sh > 2200 ? 2200 : sh);
    const double qr = ldexp(fma(a.x, b.x, a.y * b.y) / den, (int)sh);
    const double qi = ldexp(fma(a.y, b.x, -a.x * b.y) / den, (int)sh);
    z_out[j] = make_double2(zz.x - qr, zz.y - qi);
}

// Upper bound of the cancelled bits c of eq. (def_prec_loss) (Theorem
// equivAlgo): every term has s(a_k z^k) <= s(a_k) + k lambda + 1 (eq. shear)
// <= Ehat(k) + k lambda + 1 <= N + 1, so s(M) <= floor(N) + 1 for
// M = max_k |a_k z^k|, and c <= max(0, floor(N) + 1 - s(v)) for the value
// v = m 2^e standing for P(z).  lambda and N as k_bounds computes them, s(v)
// exactly.  0 where the point has no window (z = 0, where P(0) = a_0 and
// |P| >= M; a non-finite z; P == 0); INT32_MAX where v = 0.
constexpr int kCancelThreads = 1024;
constexpr int kCancelPer = 2;                   // points per thread

__global__ __launch_bounds__(kCancelThreads) void k_cancel(DevPlan P, const double2 *__restrict__ z, int n,
                                                           const double2 *__restrict__ m,
                                                           const long long *__restrict__ e,
                                                           int32_t *__restrict__ out) {
    __shared__ double s_k[kHullLds];
    __shared__ double s_s[kHullLds];
    const int t = threadIdx.x;
    const bool in_lds = P.nh <= kHullLds;
    if (in_lds)
        for (int i = t; i < P.nh; i += kCancelThreads) { s_k[i] = P.hull_k[i]; s_s[i] = P.hull_s[i]; }
    __syncthreads();
    auto run = [&](auto hk, auto hs) {
#pragma unroll
        for (int it = 0; it < kCancelPer; ++it) {
            const int j = (blockIdx.x * kCancelPer + it) * kCancelThreads + t;
            if (j >= n) continue;
            const double2 zz = z[j];
            int32_t c = 0;
            if (P.nh > 0 && isfinite(zz.x) && isfinite(zz.y) && (zz.x != 0.0 || zz.y != 0.0)) {
                const double2 v = m[j];
                const int32_t sv = scale_exact(v.x, v.y);
                if (sv == kNegInfScale) {
                    c = INT32_MAX;
                } else {
                    const double lam = log2_abs(zz);
                    const int is = cover_argmax(P.nh, hk, hs, lam);
                    const double N = fma(lam, hk[is], hs[is]);
                    const long long b = (long long)floor(N) + 1 - ((long long)sv + e[j]);
                    c = b <= 0 ? 0 : (b >= INT32_MAX ? INT32_MAX : (int32_t)b);
                }
            }
            out[j] = c;
        }
    };
    if (in_lds) run((lds_table_t)s_k, (lds_table_t)s_s);
    else run((const double *)P.hull_k, (const double *)P.hull_s);
}

}  // namespace

// Smallest cost unit shift for which the total tile work of n points fits the
// int32 scans: at most G groups x (chunks x (C / u + powering overhead) + the
// per-group part), u = 16 << shift; -1 if none does.
int cost_shift_for_chunks(int64_t G, int64_t chunks, int chunk);

int cost_shift_for(const DevPlan &P, int64_t n, int C) {
    const int64_t G = (n + kWave - 1) / kWave;
    const int64_t chunks = P.nh > 0 ? (int64_t)P.dt / C - (int64_t)P.v / C + 1 : 0;
    return cost_shift_for_chunks(G, chunks, C);
}

int cost_shift_for_chunks(int64_t G, int64_t chunks, int chunk) {
    for (int sh = 0; sh <= 20; ++sh) {
        const int64_t u = (int64_t)kCostUnit << sh;
        auto units = [u](int64_t steps) { return (steps + u - 1) / u; };
        const int64_t per_tile = units(chunk + chunk / 8 + kTileSteps + kFirstSteps + kLastSteps + kMidSteps +
                                       (kPowSteps + kAnchorBitSteps) * 31);
        const int64_t bound = G * chunks * per_tile;
        if (bound < INT32_MAX) return sh;
    }
    return -1;
}

size_t eval_workspace_bytes(const DevPlan &P, int64_t n, EvalWs *ws, void *base, int kind, int64_t batch_groups,
                            int chunk, bool tight) {
    size_t off = 0;
    char *b = static_cast<char *>(base);
    auto take = [&](size_t bytes) { char *p = b ? b + off : nullptr; off = align_up(off + bytes); return p; };
    // a batch sorts each polynomial's points in its own whole groups (no sort table)
    const bool batch = batch_groups >= 0;
    const int64_t G = batch ? batch_groups : (n + kWave - 1) / kWave;
    const int64_t nslot = batch ? G * kWave : n;
    const int64_t NB = batch ? 0 : (n + kSortPoints - 1) / kSortPoints;
    const int64_t tlen = (int64_t)(kBins + 1) * NB;
    const int tab_ib = NB <= kSeg ? (int)(kSeg / (NB > 0 ? NB : 1)) : 1;
    const int64_t nblk_g = (G + kGroupsPerBlock - 1) / kGroupsPerBlock;
    const int64_t nseg_t = (kBins + 1 + tab_ib - 1) / tab_ib, nseg_g = (nblk_g + kSeg - 1) / kSeg;
    EvalWs w;
    w.lr = (int2 *)take(sizeof(int2) * (n > 0 ? n : 1));
    w.keyrank = (int32_t *)take(sizeof(int32_t) * n);
    w.srec = (PointRec *)take(sizeof(PointRec) * nslot);
    w.eref = (long long *)take(sizeof(long long) * (n > 0 ? n : 1));
    w.table = (int32_t *)take(sizeof(int32_t) * (tlen > 0 ? tlen : 1));
    w.tscan = (int32_t *)take(sizeof(int32_t) * (tlen > 0 ? tlen : 1));
    w.bin_sum = (int32_t *)take(sizeof(int32_t) * (nseg_t > 0 ? nseg_t : 1));
    w.bin_off = (int32_t *)take(sizeof(int32_t) * (nseg_t > 0 ? nseg_t : 1));
    w.glo = (int32_t *)take(sizeof(int32_t) * (G > 0 ? G : 1));
    w.gml = (int32_t *)take(sizeof(int32_t) * (G > 0 ? G : 1));
    w.ghi = (int32_t *)take(sizeof(int32_t) * (G > 0 ? G : 1));
    w.gcost = (int32_t *)take(sizeof(int32_t) * (G > 0 ? G : 1));
    w.gcum = (int32_t *)take(sizeof(int32_t) * (G > 0 ? G : 1));
    w.gdens = (int32_t *)take(sizeof(int32_t) * (G > 0 ? G : 1));
    w.gblk_sum = (int32_t *)take(sizeof(int32_t) * (nblk_g > 0 ? nblk_g : 1));
    w.gblk_pre = (int32_t *)take(sizeof(int32_t) * (nblk_g > 0 ? nblk_g : 1));
    w.gseg_sum = (int32_t *)take(sizeof(int32_t) * (nseg_g > 0 ? nseg_g : 1));
    w.gseg_off = (int32_t *)take(sizeof(int32_t) * (nseg_g > 0 ? nseg_g : 1));
    w.split = (int4 *)take(sizeof(int4) * (G > 0 ? G : 1));
    // as many window wavefronts as are resident, but no more than four per
    // group: a small evaluation then spreads its few tiles over few wavefronts
    w.n_waves = std::min<int64_t>(window_waves(kind), std::max<int64_t>(4 * G, 1));
    // the finalize kernel holds the long groups in LDS
    w.n_waves = std::min<int64_t>(w.n_waves, (int64_t)(kLongLds - 1) * kFinalShort);
    // one workspace serves every tile kernel, unless sized for this kind alone
    const int64_t nw_max = tight ? w.n_waves
                                 : std::max({window_waves(kTileValue), window_waves(kTileDeriv),
                                             window_waves(kTileAdjoint), window_waves(kTileBatch),
                                             window_waves(kTileSparse), window_waves(kTileComp),
                                             window_waves(kTileBatchComp)});
    w.wstart = (int2 *)take(sizeof(int2) * (nw_max + 1));
    w.slots = (long long *)take(sizeof(long long) * kSlotWords * kWave * 2 * nw_max);
    const int64_t nlong = long_cap(nw_max);
    w.lgroups = (int4 *)take(sizeof(int4) * nlong);
    w.lacc = (long long *)take(sizeof(long long) * kSlotWords * kWave * nlong);
    w.lcnt = (int32_t *)take(sizeof(int32_t) * nlong);
    w.ctl = (int32_t *)take(sizeof(int32_t) * 64);
    // the reverse mode's accumulators (a layout for the values alone has none)
    w.n_acc = (!tight || kind == kTileAdjoint) ? std::max<int64_t>((int64_t)P.dt + 1, 1) : 0;
    w.aexp = (int32_t *)take(sizeof(int32_t) * std::max<int64_t>(w.n_acc, 1));
    w.aflag = (int32_t *)take(sizeof(int32_t) * std::max<int64_t>(w.n_acc, 1));
    w.aacc = (long long *)take(sizeof(long long) * 4 * std::max<int64_t>(w.n_acc, 1));
    w.n = n;
    w.tab_ib = tab_ib;
    w.cost_shift = cost_shift_for(P, n, chunk);
    w.chunk = chunk;
    w.n_groups = G;
    w.n_sort_blocks = NB;
    w.plans = nullptr;
    w.gpoly = nullptr;
    w.n_slots = batch ? nslot : -1;
    w.sparse = kind == kTileSparse ? 1 : 0;
    if (ws) *ws = w;
    return off;
}

}  // namespace fpe

using namespace fpe;

// ---------------------------------------------------------------- tile schedule
// The chunk length C of the (group, chunk) tiles and the form of the window
// sums (dense: Horner's rule over every index with bad coefficients masked;
// sparse: over the list of G_p with gaps jumped by powers of z): the ones
// fpe_autotune chose or fpe_plan_set_chunk / fpe_plan_set_window_mode set for
// this plan, else the ones tuned earlier in this process for the same
// (degree, points, |G_p|, FP32, batch) bucket, else C = kChunk and the dense
// form (the density of G_p inside the windows, which decides, is only known by
// evaluating: the wide-range workloads hold G_p on 1/267 of the indices but on
// 1/13 of their windows' indices, where the dense form is faster).  FP32
// plans keep kChunk and the dense form (their FP32 table is scaled per kChunk
// coefficients); derivatives and the reverse mode always run the dense form.
namespace {
typedef std::tuple<int, int, int, int, int> TuneKey;
struct TileChoice { int chunk; bool sparse; };
std::map<TuneKey, TileChoice> g_tuned;
std::mutex g_tuned_mu;

int bucket(int64_t x) {
    int b = 0;
    while (x > 0) { ++b; x >>= 1; }
    return b;
}

TuneKey tune_key(int64_t d, int64_t n, int64_t ngood, bool fp32, bool batch) {
    return {bucket(d), bucket(n), bucket(ngood), fp32 ? 1 : 0, batch ? 1 : 0};
}

bool cached_choice(const TuneKey &key, TileChoice *c) {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    auto it = g_tuned.find(key);
    if (it == g_tuned.end()) return false;
    *c = it->second;
    return true;
}

int cached_chunk(const TuneKey &key) {
    TileChoice c;
    return cached_choice(key, &c) ? c.chunk : kChunk;
}

bool valid_chunk(int c) { return c >= kChunkMin && c <= kChunkMax && (c & (c - 1)) == 0; }

TileChoice plan_choice(const fpe_plan_s *plan, int64_t n) {
    if (plan->dev.coef32) return {kChunk, false};
    TileChoice c;
    if (!cached_choice(tune_key(plan->d, n, plan->ngood, false, false), &c)) c = {kChunk, false};
    if (plan->chunk_sel) c.chunk = plan->chunk_sel;
    if (plan->mode_sel) c.sparse = plan->mode_sel == FPE_WINDOW_SPARSE;
    return c;
}

int plan_chunk(const fpe_plan_s *plan, int64_t n) { return plan_choice(plan, n).chunk; }
}  // namespace

extern "C" fpe_status fpe_eval_workspace_size(fpe_plan_t plan, int64_t n, size_t *bytes) {
    if (!plan || !bytes) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    if (n < 0 || n >= INT32_MAX) return fail(FPE_ERR_INVALID_ARG, "n out of range");
    if (cost_shift_for(plan->dev, n, kChunkMin) < 0)
        return fail(FPE_ERR_UNSUPPORTED, "too many (point group, chunk) tiles");
    FPE_HIP_CHECK(device_setup());
    *bytes = eval_workspace_bytes(plan->dev, n, nullptr, nullptr, kTileValue);
    set_error("");
    return FPE_OK;
}

// The kernels before the tile kernel: bounds, sort, groups, partition.
// From the sorted records: group windows and costs, their scan, the partition.
static void launch_groups(const DevPlan &P, const EvalWs &W, int nblk_g, hipStream_t stream) {
    k_groups<<<(unsigned)nblk_g, 1024, 0, stream>>>(P, W);
    if (nblk_g > kPartLds) {
        const int nseg = (nblk_g + kSeg - 1) / kSeg;
        k_scan_seg<<<(unsigned)nseg, 1024, 0, stream>>>(W.gblk_sum, W.gblk_pre, nblk_g, W.gseg_sum);
        k_scan_sums<<<1, 1024, 0, stream>>>(W.gseg_sum, nseg, W.gseg_off, W.ctl + 0);
    }
    k_partition<<<(unsigned)((W.n_groups + W.n_waves + 1 + 1023) / 1024), 1024, 0, stream>>>(P, W);
}

static hipError_t launch_front(const DevPlan &P, const double2 *z, int ni, double2 *m, long long *e, double2 *md,
                               long long *ed, int32_t *terms, long long *win, const EvalWs &W, hipStream_t stream) {
    const unsigned sb = (unsigned)W.n_sort_blocks;
    const unsigned pb = (unsigned)((ni + 1023) / 1024);
    const int nblk_g = (int)((W.n_groups + kGroupsPerBlock - 1) / kGroupsPerBlock);
    k_bounds<<<sb, kBoundsThreads, 0, stream>>>(P, z, ni, m, e, md, ed, terms, win, W);
    if (P.nh > 0) {
        const int nseg_t = (kBins + 1 + W.tab_ib - 1) / W.tab_ib;
        k_scan_table<<<(unsigned)nseg_t, 1024, 0, stream>>>(W);
        k_scatter<<<pb, 1024, 0, stream>>>(ni, z, W);
        launch_groups(P, W, nblk_g, stream);
    }
    return hipGetLastError();
}

// tight: the workspace is laid out for this evaluation alone (the layout the
// no-allocation entry point uses); otherwise as fpe_eval_workspace_size says.
// With tight, no profiling events are recorded (creating one may allocate).
static fpe_status eval_impl(fpe_plan_t plan, const double *z_dev, int64_t n, double *m_dev, int64_t *e_dev,
                            double *md_dev, int64_t *ed_dev, int32_t *terms_dev, int64_t *window_dev,
                            void *workspace_dev, size_t workspace_bytes, hipStream_t stream, bool tight = false) {
    const bool deriv = md_dev != nullptr;
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    size_t need = 0;
    fpe_status st = fpe_eval_workspace_size(plan, n, &need);
    if (st != FPE_OK) return st;
    const TileChoice tc = plan_choice(plan, n);
    const bool sparse = !deriv && tc.sparse;
    const bool comp = !deriv && plan->dev.f32comp;
    const int kind = sparse ? kTileSparse : (deriv ? kTileDeriv : (comp ? kTileComp : kTileValue));
    if (tight) need = eval_workspace_bytes(plan->dev, n, nullptr, nullptr, kind, -1, tc.chunk, true);
    if (n == 0) { set_error(""); return FPE_OK; }
    if (!z_dev || !m_dev || !e_dev || !workspace_dev || (deriv && !ed_dev))
        return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    if (workspace_bytes < need)
        return fail(FPE_ERR_WORKSPACE, "eval workspace too small: need " + std::to_string(need));
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0 || reinterpret_cast<uintptr_t>(z_dev) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(m_dev) % 16 != 0 || reinterpret_cast<uintptr_t>(md_dev) % 16 != 0)
        return fail(FPE_ERR_INVALID_ARG, "misaligned buffer");
    EvalWs W;
    eval_workspace_bytes(plan->dev, n, &W, workspace_dev, kind, -1, tc.chunk, tight);
    const bool prof = g_prof.on && !tight;
    const DevPlan &P = plan->dev;
    const double2 *z = reinterpret_cast<const double2 *>(z_dev);
    double2 *m = reinterpret_cast<double2 *>(m_dev);
    long long *e = reinterpret_cast<long long *>(e_dev);
    double2 *md = reinterpret_cast<double2 *>(md_dev);
    long long *ed = reinterpret_cast<long long *>(ed_dev);
    long long *win = reinterpret_cast<long long *>(window_dev);
    const int ni = (int)n;

    FPE_HIP_CHECK(device_setup());
    FPE_HIP_CHECK(launch_front(P, z, ni, m, e, md, ed, terms_dev, win, W, stream));
    if (P.nh > 0) {
        const unsigned wb = (unsigned)((W.n_waves + kWindowWaves - 1) / kWindowWaves);
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (prof) {
            FPE_HIP_CHECK(prof_event(&ev0));
            FPE_HIP_CHECK(prof_event(&ev1));
            FPE_HIP_CHECK(hipEventRecord(ev0, stream));
        }
        if (deriv) k_window<true, false><<<wb, kWindowThreads, 0, stream>>>(P, m, e, md, ed, W);
        else if (sparse) k_window<false, false, true><<<wb, kWindowThreads, 0, stream>>>(P, m, e, nullptr, nullptr, W);
        else if (comp) k_window<false, false, false, true><<<wb, kWindowThreads, 0, stream>>>(P, m, e, nullptr, nullptr, W);
        else k_window<false, false><<<wb, kWindowThreads, 0, stream>>>(P, m, e, nullptr, nullptr, W);
        if (prof) {
            FPE_HIP_CHECK(hipEventRecord(ev1, stream));
            g_prof.pending.emplace_back(ev0, ev1);
        }
        if (W.n_waves > 1) {
            const unsigned fb = final_blocks(deriv ? 1 : 0, W.n_waves);
            if (deriv) k_finalize<true, false><<<fb, kFinalThreads, 0, stream>>>(P, m, e, md, ed, W);
            else k_finalize<false, false><<<fb, kFinalThreads, 0, stream>>>(P, m, e, nullptr, nullptr, W);
        }
    }
    FPE_HIP_CHECK(hipGetLastError());
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_eval(fpe_plan_t plan, const double *z_dev, int64_t n, double *m_dev, int64_t *e_dev,
                               int32_t *terms_dev, int64_t *window_dev, void *workspace_dev, size_t workspace_bytes,
                               hipStream_t stream) {
    return eval_impl(plan, z_dev, n, m_dev, e_dev, nullptr, nullptr, terms_dev, window_dev, workspace_dev,
                     workspace_bytes, stream);
}

extern "C" fpe_status fpe_eval_deriv(fpe_plan_t plan, const double *z_dev, int64_t n, double *m_dev,
                                     int64_t *e_dev, double *md_dev, int64_t *ed_dev, void *workspace_dev,
                                     size_t workspace_bytes, hipStream_t stream) {
    if (n > 0 && (!md_dev || !ed_dev)) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    return eval_impl(plan, z_dev, n, m_dev, e_dev, md_dev, ed_dev, nullptr, nullptr, workspace_dev,
                     workspace_bytes, stream);
}

// ---------------------------------------------------------------- no allocation
// fpe_eval_noalloc: fpe_eval with its workspace in a static device array of
// kScratchBytes instead of a caller buffer.  Each device the library runs on
// holds its own copy of the array from the module's load to the end of the
// process; its address on a device comes from hipGetSymbolAddress once, on the
// first call with that device current (the name `scratch` in host code is a
// host-side stand-in, never a device address).  The evaluation writes every
// word of the workspace it later reads (k_bounds clears the counters,
// k_partition the long groups' accumulators), so nothing needs clearing
// between calls; calls that overlap on one device share the array and race.
constexpr size_t kScratchBytes = (size_t)96 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void *g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

fpe_status scratch_address(void **out) {
    int dev = 0;
    FPE_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FPE_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256 != 0)
            return fail(FPE_ERR_HIP, "static scratch array has no aligned device address");
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return FPE_OK;
}
}  // namespace

extern "C" fpe_status fpe_eval_noalloc(fpe_plan_t plan, const double *z_dev, int64_t n, double *m_dev,
                                       int64_t *e_dev, int32_t *terms_dev, int64_t *window_dev,
                                       hipStream_t stream) {
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    if (n < 0 || n >= INT32_MAX) return fail(FPE_ERR_INVALID_ARG, "n out of range");
    if (n == 0) { set_error(""); return FPE_OK; }
    FPE_HIP_CHECK(device_setup());
    if (cost_shift_for(plan->dev, n, kChunkMin) < 0)
        return fail(FPE_ERR_UNSUPPORTED, "too many (point group, chunk) tiles");
    const TileChoice tc = plan_choice(plan, n);
    const size_t need = eval_workspace_bytes(plan->dev, n, nullptr, nullptr, tc.sparse ? kTileSparse : kTileValue, -1,
                                             tc.chunk, true);
    if (need > kScratchBytes)
        return fail(FPE_ERR_WORKSPACE, "fpe_eval_noalloc: " + std::to_string(n) + " points need " +
                                           std::to_string(need) + " bytes of workspace, above the static " +
                                           std::to_string(kScratchBytes) + "-byte scratch (use fpe_eval)");
    void *ws = nullptr;
    fpe_status st = scratch_address(&ws);
    if (st != FPE_OK) return st;
    return eval_impl(plan, z_dev, n, m_dev, e_dev, nullptr, nullptr, terms_dev, window_dev, ws, kScratchBytes,
                     stream, true);
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

extern "C" fpe_status fpe_newton_step(fpe_plan_t plan, const double *z_dev, int64_t n, double *m_dev,
                                      int64_t *e_dev, double *md_dev, int64_t *ed_dev, double *z_out_dev,
                                      void *workspace_dev, size_t workspace_bytes, hipStream_t stream) {
    if (!z_out_dev && n > 0) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(z_out_dev) % 16 != 0) return fail(FPE_ERR_INVALID_ARG, "misaligned buffer");
    fpe_status st = fpe_eval_deriv(plan, z_dev, n, m_dev, e_dev, md_dev, ed_dev, workspace_dev, workspace_bytes,
                                   stream);
    if (st != FPE_OK || n == 0) return st;
    k_newton<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(
        reinterpret_cast<const double2 *>(z_dev), (int)n, reinterpret_cast<const double2 *>(m_dev),
        reinterpret_cast<const long long *>(e_dev), reinterpret_cast<const double2 *>(md_dev),
        reinterpret_cast<const long long *>(ed_dev), reinterpret_cast<double2 *>(z_out_dev));
    FPE_HIP_CHECK(hipGetLastError());
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_cancelled_bits(fpe_plan_t plan, const double *z_dev, int64_t n, const double *m_dev,
                                         const int64_t *e_dev, int32_t *bits_dev, hipStream_t stream) {
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    if (n < 0 || n >= INT32_MAX) return fail(FPE_ERR_INVALID_ARG, "n out of range");
    if (n == 0) { set_error(""); return FPE_OK; }
    if (!z_dev || !m_dev || !e_dev || !bits_dev) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(z_dev) % 16 != 0 || reinterpret_cast<uintptr_t>(m_dev) % 16 != 0)
        return fail(FPE_ERR_INVALID_ARG, "misaligned buffer");
    const int64_t per = (int64_t)kCancelThreads * kCancelPer;
    k_cancel<<<(unsigned)((n + per - 1) / per), kCancelThreads, 0, stream>>>(
        plan->dev, reinterpret_cast<const double2 *>(z_dev), (int)n, reinterpret_cast<const double2 *>(m_dev),
        reinterpret_cast<const long long *>(e_dev), bits_dev);
    FPE_HIP_CHECK(hipGetLastError());
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_eval_adjoint(fpe_plan_t plan, const double *z_dev, int64_t n, const double *g_dev,
                                       const int64_t *g_exp_dev, const double *md_dev, const int64_t *ed_dev,
                                       double *grad_a_dev,
                                       double *grad_z_dev, void *workspace_dev, size_t workspace_bytes,
                                       hipStream_t stream) {
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    size_t need = 0;
    fpe_status st = fpe_eval_workspace_size(plan, n, &need);
    if (st != FPE_OK) return st;
    if (n > 0 && (!z_dev || !g_dev || !workspace_dev || (grad_z_dev && (!md_dev || !ed_dev))))
        return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    if (n > 0 && workspace_bytes < need)
        return fail(FPE_ERR_WORKSPACE, "eval workspace too small: need " + std::to_string(need));
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0 || reinterpret_cast<uintptr_t>(z_dev) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(g_dev) % 16 != 0 || reinterpret_cast<uintptr_t>(grad_a_dev) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(grad_z_dev) % 16 != 0 || reinterpret_cast<uintptr_t>(md_dev) % 16 != 0)
        return fail(FPE_ERR_INVALID_ARG, "misaligned buffer");
    const DevPlan &P = plan->dev;
    const int64_t na = plan->d + 1;
    double2 *ga = reinterpret_cast<double2 *>(grad_a_dev);
    FPE_HIP_CHECK(device_setup());
    EvalWs W;
    eval_workspace_bytes(P, n, &W, workspace_dev, kTileAdjoint, -1, plan_chunk(plan, n));
    const AdjAcc A{W.aexp, W.aflag, W.aacc};
    // fraction bits of the fixed point: an index gathers at most one term per
    // point, each below 2^(S - 2) in units of its scale, so n 2^S <= 2^62;
    // and S <= 47 keeps a wavefront's sums of 64 terms exact in FP64
    int S = 62;
    for (int64_t cnt = n; cnt > 0; cnt >>= 1) --S;
    S = std::min(S, 47);
    const double2 *z = reinterpret_cast<const double2 *>(z_dev);
    const double2 *g = reinterpret_cast<const double2 *>(g_dev);
    const long long *gx = reinterpret_cast<const long long *>(g_exp_dev);
    const int ni = (int)n;
    const unsigned pb = (unsigned)((n + 255) / 256);
    if (ga && plan->adjoint_mode == FPE_ADJOINT_ATOMIC) {
        k_zero2<<<(unsigned)((na + 255) / 256), 256, 0, stream>>>(ga, na);
        if (n > 0) {
            FPE_HIP_CHECK(launch_front(P, z, ni, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, W, stream));
            const unsigned wb = (unsigned)((W.n_waves + kWindowWaves - 1) / kWindowWaves);
            if (P.nh > 0) k_adjoint<kAdjAtomic><<<wb, kWindowThreads, 0, stream>>>(P, g, gx, A, S, ga, W);
            k_adj_zero<kAdjAtomic><<<pb, 256, 0, stream>>>(P, z, ni, g, gx, A, S, ga);
        }
    } else if (ga) {
        // (with no points the workspace may be absent: grad_a is only zeroed)
        if (n > 0) {
            k_adj_init<<<(unsigned)((W.n_acc + 255) / 256), 256, 0, stream>>>(A, W.n_acc);
            FPE_HIP_CHECK(launch_front(P, z, ni, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, W, stream));
            const unsigned wb = (unsigned)((W.n_waves + kWindowWaves - 1) / kWindowWaves);
            if (P.nh > 0) k_adjoint<kAdjBound><<<wb, kWindowThreads, 0, stream>>>(P, g, gx, A, S, ga, W);
            k_adj_zero<kAdjBound><<<pb, 256, 0, stream>>>(P, z, ni, g, gx, A, S, ga);
            if (P.nh > 0) k_adjoint<kAdjExact><<<wb, kWindowThreads, 0, stream>>>(P, g, gx, A, S, ga, W);
            k_adj_zero<kAdjExact><<<pb, 256, 0, stream>>>(P, z, ni, g, gx, A, S, ga);
        }
        k_adj_out<<<(unsigned)((na + 255) / 256), 256, 0, stream>>>(A, n > 0 ? W.n_acc : 0, na, S, ga);
    }
    if (n > 0 && grad_z_dev)
        k_grad_z<<<pb, 256, 0, stream>>>(z, ni, g, gx, reinterpret_cast<const double2 *>(md_dev),
                                         reinterpret_cast<const long long *>(ed_dev),
                                         reinterpret_cast<double2 *>(grad_z_dev));
    FPE_HIP_CHECK(hipGetLastError());
    set_error("");
    return FPE_OK;
}

// ---------------------------------------------------------------- batches
struct fpe_batch_s {
    int32_t n_poly;
    int64_t n_points, n_groups;
    DevPlan rep;                   // the first plan (every plan has the same chunk length)
    const DevPlan *plans_dev;      // per polynomial, in the batch workspace
    const long long *pstart_dev;   // n_poly + 1 point offsets
    const int32_t *gstart_dev;     // n_poly + 1 group offsets
    const int32_t *gpoly_dev;      // per group: its polynomial
    int32_t cost_shift;
    int device;
    int64_t max_span;              // the longest trimmed coefficient range of its plans
    int64_t mean_degree;
    bool any_fp32;
    bool any_f32comp;              // some plan asks for compensated FP32 blocks
    int32_t chunk_sel = 0;         // chosen by fpe_batch_autotune or set; 0: cached choice or default
};

namespace {

int batch_chunk(const fpe_batch_s *b) {
    if (b->any_fp32) return kChunk;
    if (b->chunk_sel) return b->chunk_sel;
    return cached_chunk(tune_key(b->mean_degree, b->n_points, 0, false, true));
}

struct BatchLayout { size_t plans, pstart, gstart, gpoly, total; };

BatchLayout batch_layout(int64_t n_poly, int64_t n_groups) {
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.plans = take(sizeof(DevPlan) * (size_t)n_poly);
    L.pstart = take(sizeof(long long) * (size_t)(n_poly + 1));
    L.gstart = take(sizeof(int32_t) * (size_t)(n_poly + 1));
    L.gpoly = take(sizeof(int32_t) * (size_t)(n_groups > 0 ? n_groups : 1));
    L.total = off;
    return L;
}

// checks the point offsets and counts the groups
fpe_status batch_groups(int32_t n_poly, const int64_t *z_offsets, int64_t *n_groups) {
    if (n_poly < 1) return fail(FPE_ERR_INVALID_ARG, "n_poly must be >= 1");
    if (!z_offsets) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    if (z_offsets[0] != 0) return fail(FPE_ERR_INVALID_ARG, "z_offsets[0] must be 0");
    int64_t g = 0;
    for (int32_t i = 0; i < n_poly; ++i) {
        const int64_t m = z_offsets[i + 1] - z_offsets[i];
        if (m < 0) return fail(FPE_ERR_INVALID_ARG, "z_offsets must be non-decreasing");
        if (m > kBatchMaxPoints)
            return fail(FPE_ERR_UNSUPPORTED, "a polynomial of a batch has more than " +
                                                 std::to_string(kBatchMaxPoints) + " points (use fpe_eval)");
        g += (m + kWave - 1) / kWave;
    }
    if (z_offsets[n_poly] >= INT32_MAX || g * kWave >= INT32_MAX)
        return fail(FPE_ERR_INVALID_ARG, "too many points");
    *n_groups = g;
    return FPE_OK;
}

}  // namespace

extern "C" fpe_status fpe_batch_workspace_size(int32_t n_poly, const int64_t *z_offsets, size_t *bytes) {
    if (!bytes) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    int64_t g = 0;
    fpe_status st = batch_groups(n_poly, z_offsets, &g);
    if (st != FPE_OK) return st;
    *bytes = batch_layout(n_poly, g).total;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_batch_create(const fpe_plan_t *plans, int32_t n_poly, const int64_t *z_offsets,
                                       void *workspace_dev, size_t workspace_bytes, hipStream_t stream,
                                       fpe_batch_t *out_batch) {
    if (!plans || !out_batch || !workspace_dev) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    *out_batch = nullptr;
    int64_t G = 0;
    fpe_status st = batch_groups(n_poly, z_offsets, &G);
    if (st != FPE_OK) return st;
    const BatchLayout L = batch_layout(n_poly, G);
    if (workspace_bytes < L.total)
        return fail(FPE_ERR_WORKSPACE, "batch workspace too small: need " + std::to_string(L.total));
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0)
        return fail(FPE_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    std::vector<DevPlan> hp(n_poly);
    std::vector<long long> ps(n_poly + 1);
    std::vector<int32_t> gs(n_poly + 1), gp((size_t)(G > 0 ? G : 1), 0);
    int64_t chunks_max = 1, span_max = 1, deg_sum = 0;
    bool any_fp32 = false, any_f32comp = false;
    gs[0] = 0;
    for (int32_t i = 0; i < n_poly; ++i) {
        if (!plans[i]) return fail(FPE_ERR_INVALID_ARG, "NULL plan in the batch");
        if (plans[i]->device != plans[0]->device) return fail(FPE_ERR_INVALID_ARG, "plans on different devices");
        hp[i] = plans[i]->dev;
        const DevPlan &Q = hp[i];
        if (Q.nh > 0) {
            chunks_max = std::max<int64_t>(chunks_max, (int64_t)Q.dt / kChunkMin - (int64_t)Q.v / kChunkMin + 1);
            span_max = std::max<int64_t>(span_max, (int64_t)Q.dt - Q.v + 1);
        }
        deg_sum += plans[i]->d;
        any_fp32 = any_fp32 || Q.coef32 != nullptr;
        any_f32comp = any_f32comp || Q.f32comp != 0;
        ps[i] = z_offsets[i];
        const int32_t ng = (int32_t)((z_offsets[i + 1] - z_offsets[i] + kWave - 1) / kWave);
        gs[i + 1] = gs[i] + ng;
        for (int32_t k = gs[i]; k < gs[i + 1]; ++k) gp[k] = i;
    }
    ps[n_poly] = z_offsets[n_poly];
    const int cs = cost_shift_for_chunks(G, chunks_max, kChunkMin);
    if (cs < 0) return fail(FPE_ERR_UNSUPPORTED, "too many (point group, chunk) tiles");
    char *b = static_cast<char *>(workspace_dev);
    FPE_HIP_CHECK(hipMemcpyAsync(b + L.plans, hp.data(), sizeof(DevPlan) * hp.size(), hipMemcpyHostToDevice, stream));
    FPE_HIP_CHECK(hipMemcpyAsync(b + L.pstart, ps.data(), sizeof(long long) * ps.size(), hipMemcpyHostToDevice, stream));
    FPE_HIP_CHECK(hipMemcpyAsync(b + L.gstart, gs.data(), sizeof(int32_t) * gs.size(), hipMemcpyHostToDevice, stream));
    FPE_HIP_CHECK(hipMemcpyAsync(b + L.gpoly, gp.data(), sizeof(int32_t) * gp.size(), hipMemcpyHostToDevice, stream));
    FPE_HIP_CHECK(hipStreamSynchronize(stream));
    std::unique_ptr<fpe_batch_s> bt(new fpe_batch_s());
    bt->n_poly = n_poly;
    bt->n_points = z_offsets[n_poly];
    bt->n_groups = G;
    bt->rep = hp[0];
    bt->plans_dev = reinterpret_cast<const DevPlan *>(b + L.plans);
    bt->pstart_dev = reinterpret_cast<const long long *>(b + L.pstart);
    bt->gstart_dev = reinterpret_cast<const int32_t *>(b + L.gstart);
    bt->gpoly_dev = reinterpret_cast<const int32_t *>(b + L.gpoly);
    bt->cost_shift = cs;
    bt->device = plans[0]->device;
    bt->max_span = span_max;
    bt->mean_degree = deg_sum / n_poly;
    bt->any_fp32 = any_fp32;
    bt->any_f32comp = any_f32comp;
    *out_batch = bt.release();
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_batch_destroy(fpe_batch_t batch) {
    delete batch;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_eval_batched_workspace_size(fpe_batch_t batch, size_t *bytes) {
    if (!batch || !bytes) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    FPE_HIP_CHECK(device_setup());       // the resident wavefronts size the partition's tables
    *bytes = eval_workspace_bytes(batch->rep, batch->n_points, nullptr, nullptr,
                                  batch->any_f32comp ? kTileBatchComp : kTileBatch, batch->n_groups);
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_eval_batched(fpe_batch_t batch, const double *z_dev, double *m_dev, int64_t *e_dev,
                                       int32_t *terms_dev, void *workspace_dev, size_t workspace_bytes,
                                       hipStream_t stream) {
    if (!batch) return fail(FPE_ERR_INVALID_ARG, "NULL batch");
    const int64_t n = batch->n_points;
    if (n == 0) { set_error(""); return FPE_OK; }
    if (!z_dev || !m_dev || !e_dev || !workspace_dev) return fail(FPE_ERR_INVALID_ARG, "NULL pointer");
    FPE_HIP_CHECK(device_setup());
    size_t need = 0;
    fpe_status st = fpe_eval_batched_workspace_size(batch, &need);
    if (st != FPE_OK) return st;
    if (workspace_bytes < need)
        return fail(FPE_ERR_WORKSPACE, "eval workspace too small: need " + std::to_string(need));
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0 || reinterpret_cast<uintptr_t>(z_dev) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(m_dev) % 16 != 0)
        return fail(FPE_ERR_INVALID_ARG, "misaligned buffer");
    EvalWs W;
    const int C = batch_chunk(batch);
    eval_workspace_bytes(batch->rep, n, &W, workspace_dev, batch->any_f32comp ? kTileBatchComp : kTileBatch,
                         batch->n_groups, C);
    W.plans = batch->plans_dev;
    W.gpoly = batch->gpoly_dev;
    W.cost_shift = cost_shift_for_chunks(batch->n_groups, batch->max_span / C + 2, C);
    const DevPlan &P = batch->rep;
    const double2 *z = reinterpret_cast<const double2 *>(z_dev);
    double2 *m = reinterpret_cast<double2 *>(m_dev);
    long long *e = reinterpret_cast<long long *>(e_dev);
    k_bbounds<<<(unsigned)batch->n_poly, kBatchThreads, 0, stream>>>(batch->plans_dev, batch->pstart_dev,
                                                                      batch->gstart_dev, z, m, e, terms_dev, W);
    if (W.n_groups > 0) {
        const int nblk_g = (int)((W.n_groups + kGroupsPerBlock - 1) / kGroupsPerBlock);
        launch_groups(P, W, nblk_g, stream);
        const unsigned wb = (unsigned)((W.n_waves + kWindowWaves - 1) / kWindowWaves);
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (g_prof.on) {
            FPE_HIP_CHECK(prof_event(&ev0));
            FPE_HIP_CHECK(prof_event(&ev1));
            FPE_HIP_CHECK(hipEventRecord(ev0, stream));
        }
        if (batch->any_f32comp)
            k_window<false, true, false, true><<<wb, kWindowThreads, 0, stream>>>(P, m, e, nullptr, nullptr, W);
        else
            k_window<false, true><<<wb, kWindowThreads, 0, stream>>>(P, m, e, nullptr, nullptr, W);
        if (g_prof.on) {
            FPE_HIP_CHECK(hipEventRecord(ev1, stream));
            g_prof.pending.emplace_back(ev0, ev1);
        }
        if (W.n_waves > 1) {
            const unsigned fb = final_blocks(2, W.n_waves);
            k_finalize<false, true><<<fb, kFinalThreads, 0, stream>>>(P, m, e, nullptr, nullptr, W);
        }
    }
    FPE_HIP_CHECK(hipGetLastError());
    set_error("");
    return FPE_OK;
}

// ---------------------------------------------------------------- autotuning
namespace {

const int kChunkCandidates[] = {256, 512, 1024, 2048};

// average time of three calls of f on the stream, after one untimed call
template <class F>
fpe_status time_calls(F &&f, hipStream_t stream, float *ms) {
    fpe_status st = f();
    if (st != FPE_OK) return st;
    hipEvent_t a = nullptr, b = nullptr;
    FPE_HIP_CHECK(hipEventCreate(&a));
    FPE_HIP_CHECK(hipEventCreate(&b));
    FPE_HIP_CHECK(hipEventRecord(a, stream));
    for (int r = 0; r < 3 && st == FPE_OK; ++r) st = f();
    FPE_HIP_CHECK(hipEventRecord(b, stream));
    FPE_HIP_CHECK(hipEventSynchronize(b));
    float t = 0.0f;
    FPE_HIP_CHECK(hipEventElapsedTime(&t, a, b));
    FPE_HIP_CHECK(hipEventDestroy(a));
    FPE_HIP_CHECK(hipEventDestroy(b));
    *ms = t / 3.0f;
    return st;
}

}  // namespace

extern "C" fpe_status fpe_plan_set_chunk(fpe_plan_t plan, int32_t chunk) {
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    if (chunk != 0 && !valid_chunk(chunk)) return fail(FPE_ERR_INVALID_ARG, "chunk must be 0 or a power of two in [256, 2048]");
    if (chunk != 0 && chunk != kChunk && plan->dev.coef32)
        return fail(FPE_ERR_UNSUPPORTED, "FP32 plans use the chunk length 512");
    plan->chunk_sel = chunk;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_plan_set_window_mode(fpe_plan_t plan, int32_t mode) {
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    if (mode != FPE_WINDOW_AUTO && mode != FPE_WINDOW_DENSE && mode != FPE_WINDOW_SPARSE)
        return fail(FPE_ERR_INVALID_ARG, "mode must be FPE_WINDOW_AUTO, FPE_WINDOW_DENSE or FPE_WINDOW_SPARSE");
    if (mode == FPE_WINDOW_SPARSE && plan->dev.coef32)
        return fail(FPE_ERR_UNSUPPORTED, "FP32 plans sum their windows in the dense form");
    plan->mode_sel = mode;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_plan_set_adjoint_mode(fpe_plan_t plan, int32_t mode) {
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    if (mode != FPE_ADJOINT_EXACT && mode != FPE_ADJOINT_ATOMIC) return fail(FPE_ERR_INVALID_ARG, "unknown adjoint mode");
    plan->adjoint_mode = mode;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_plan_tile_choice(fpe_plan_t plan, int64_t n, int32_t *chunk_out, int32_t *mode_out) {
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    if (n < 0) return fail(FPE_ERR_INVALID_ARG, "n out of range");
    const TileChoice c = plan_choice(plan, n);
    if (chunk_out) *chunk_out = c.chunk;
    if (mode_out) *mode_out = c.sparse ? FPE_WINDOW_SPARSE : FPE_WINDOW_DENSE;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_autotune(fpe_plan_t plan, const double *z_dev, int64_t n, double *m_dev, int64_t *e_dev,
                                   void *workspace_dev, size_t workspace_bytes, hipStream_t stream,
                                   int32_t *chunk_out) {
    if (!plan) return fail(FPE_ERR_INVALID_ARG, "NULL plan");
    const bool fp32 = plan->dev.coef32 != nullptr;
    int best = kChunk;
    bool best_sparse = false;
    float best_ms = -1.0f;
    if (!fp32 && n > 0) {
        for (int mode : {FPE_WINDOW_DENSE, FPE_WINDOW_SPARSE}) {
            for (int C : kChunkCandidates) {
                plan->chunk_sel = C;
                plan->mode_sel = mode;
                float ms = 0.0f;
                fpe_status st = time_calls([&] {
                    return fpe_eval(plan, z_dev, n, m_dev, e_dev, nullptr, nullptr, workspace_dev, workspace_bytes,
                                    stream);
                }, stream, &ms);
                if (st != FPE_OK) { plan->chunk_sel = 0; plan->mode_sel = 0; return st; }
                if (best_ms < 0.0f || ms < best_ms) { best_ms = ms; best = C; best_sparse = mode == FPE_WINDOW_SPARSE; }
            }
        }
        std::lock_guard<std::mutex> lk(g_tuned_mu);
        g_tuned[tune_key(plan->d, n, plan->ngood, false, false)] = {best, best_sparse};
    }
    plan->chunk_sel = fp32 ? 0 : best;
    plan->mode_sel = fp32 ? 0 : (best_sparse ? FPE_WINDOW_SPARSE : FPE_WINDOW_DENSE);
    if (chunk_out) *chunk_out = best;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_batch_set_chunk(fpe_batch_t batch, int32_t chunk) {
    if (!batch) return fail(FPE_ERR_INVALID_ARG, "NULL batch");
    if (chunk != 0 && !valid_chunk(chunk)) return fail(FPE_ERR_INVALID_ARG, "chunk must be 0 or a power of two in [256, 2048]");
    if (chunk != 0 && chunk != kChunk && batch->any_fp32)
        return fail(FPE_ERR_UNSUPPORTED, "batches with FP32 plans use the chunk length 512");
    batch->chunk_sel = chunk;
    set_error("");
    return FPE_OK;
}

extern "C" fpe_status fpe_batch_autotune(fpe_batch_t batch, const double *z_dev, double *m_dev, int64_t *e_dev,
                                         void *workspace_dev, size_t workspace_bytes, hipStream_t stream,
                                         int32_t *chunk_out) {
    if (!batch) return fail(FPE_ERR_INVALID_ARG, "NULL batch");
    int best = kChunk;
    float best_ms = -1.0f;
    if (!batch->any_fp32 && batch->n_points > 0) {
        for (int C : kChunkCandidates) {
            batch->chunk_sel = C;
            float ms = 0.0f;
            fpe_status st = time_calls([&] {
                return fpe_eval_batched(batch, z_dev, m_dev, e_dev, nullptr, workspace_dev, workspace_bytes, stream);
            }, stream, &ms);
            if (st != FPE_OK) { batch->chunk_sel = 0; return st; }
            if (best_ms < 0.0f || ms < best_ms) { best_ms = ms; best = C; }
        }
        std::lock_guard<std::mutex> lk(g_tuned_mu);
        g_tuned[tune_key(batch->mean_degree, batch->n_points, 0, false, true)] = {best, false};
    }
    batch->chunk_sel = batch->any_fp32 ? 0 : best;
    if (chunk_out) *chunk_out = best;
    set_error("");
    return FPE_OK;
}
