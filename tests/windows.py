"""Exact comparison of window ends and term counts with the oracle.

The window [l, r] of a point (eq. def:LRN) is an integer decided in FP64 on
both sides: lambda = log2|z|, the vertex values Ehat(k_i) + lambda k_i, their
maximum N and the crossings x_L, x_R of the level N - T.  The two sides round
lambda and these values differently, so a window end may differ only where the
exact crossing sits within that rounding of the point where ceil(x_L - eta)
(or floor(x_R + eta)) jumps.  Those points are found from the oracle's own level
sets: both crossings grow with lambda, x_L grows and x_R shrinks with the level,
so moving lambda by +-dlam, the level by +-dlev and each crossing by the
rounding of its formula brackets each end.
Everywhere else the ends must be equal, and on every point the term count must
be #(G_p within the returned window), from the oracle's good set.
"""
from __future__ import annotations

import numpy as np

ETA = 2.0 ** -20


def _crossings(P, lam, dlev, sx):
    """x_L, x_R at the given lambda and level offset, each moved by sx times
    2^-44 max(1, |x|) (the rounding of the crossing's own formula)."""
    _, xl, xr = P.level_sets(lam, dlev)
    with np.errstate(invalid="ignore"):
        xl = xl + sx * 2.0 ** -44 * np.maximum(1.0, np.abs(xl))
        xr = xr + sx * 2.0 ** -44 * np.maximum(1.0, np.abs(xr))
    return xl, xr


def ambiguous_ends(P, ref):
    """Per point the range [lmin, lmax] x [rmin, rmax] that rounding allows:
    of lambda (2^-48 max(1, |lambda|), eight times the error of either side's
    FP64 log2), of the level (2^-46 (|N| + T + 1)) and of the crossing formula
    (2^-44 max(1, |x|)); NaN rows for points without a lambda (z = 0, a
    non-finite z, P == 0)."""
    info = P.info()
    lam = np.asarray(ref["lambda"], np.float64)
    ok = np.isfinite(lam)
    lam_f = np.where(ok, lam, 0.0)
    N = np.where(ok, np.asarray(ref["N"], np.float64), 0.0)
    dlam = 2.0 ** -48 * np.maximum(1.0, np.abs(lam_f))
    dlev = 2.0 ** -46 * (np.abs(N) + info.T + 1.0)
    xl_lo, xr_lo = _crossings(P, lam_f - dlam, -dlev, -1.0)    # smallest x_L
    xl_hi, _ = _crossings(P, lam_f + dlam, dlev, 1.0)          # largest x_L
    _, xr_lo = _crossings(P, lam_f - dlam, dlev, -1.0)         # smallest x_R
    _, xr_hi = _crossings(P, lam_f + dlam, -dlev, 1.0)         # largest x_R
    with np.errstate(invalid="ignore"):
        lmin = np.maximum(np.ceil(xl_lo - ETA), info.v)
        lmax = np.maximum(np.ceil(xl_hi - ETA), info.v)
        rmin = np.minimum(np.floor(xr_lo + ETA), info.dt)
        rmax = np.minimum(np.floor(xr_hi + ETA), info.dt)
    out = np.stack([lmin, lmax, rmin, rmax], axis=1)
    out[~ok] = np.nan
    return out


def good_prefix(good):
    g = np.asarray(good, np.int64)
    return np.concatenate([[0], np.cumsum(g)])


def check_windows(P, ref, w, terms=None, good=None, idx=None, say=None):
    """GPU windows w [n, 2] (and term counts) against the oracle plan P and its
    eval result ref, both over the same points (idx: the GPU rows of ref's
    points).  Returns the number of points whose ends may differ by rounding."""
    w = np.asarray(w if idx is None else w[idx])
    l_ref, r_ref = np.asarray(ref["l"]), np.asarray(ref["r"])
    amb = ambiguous_ends(P, ref)
    ok = np.isfinite(amb[:, 0])
    # points without a lambda: exact
    assert np.array_equal(w[~ok, 0], l_ref[~ok]) and np.array_equal(w[~ok, 1], r_ref[~ok])
    a = amb[ok]
    la, ra = w[ok, 0], w[ok, 1]
    # the oracle itself lies in its bracket (a check of the bracket)
    assert ((a[:, 0] <= l_ref[ok]) & (l_ref[ok] <= a[:, 1])).all()
    assert ((a[:, 2] <= r_ref[ok]) & (r_ref[ok] <= a[:, 3])).all()
    # the GPU within the bracket everywhere, equal where the bracket is one index
    assert ((a[:, 0] <= la) & (la <= a[:, 1])).all(), "a left end outside its rounding bracket"
    assert ((a[:, 2] <= ra) & (ra <= a[:, 3])).all(), "a right end outside its rounding bracket"
    tight_l = a[:, 0] == a[:, 1]
    tight_r = a[:, 2] == a[:, 3]
    assert np.array_equal(la[tight_l], l_ref[ok][tight_l]), "left ends differ"
    assert np.array_equal(ra[tight_r], r_ref[ok][tight_r]), "right ends differ"
    n_amb = int((~tight_l | ~tight_r).sum())
    n_diff = int(((la != l_ref[ok]) | (ra != r_ref[ok])).sum())
    if terms is not None:
        t = np.asarray(terms if idx is None else terms[idx]).astype(np.int64)
        pre = good_prefix(P.good() if good is None else good)
        empty = w[:, 0] > w[:, 1]
        want = np.where(empty, 0, pre[np.clip(w[:, 1] + 1, 0, len(pre) - 1)] - pre[np.clip(w[:, 0], 0, len(pre) - 1)])
        # z = 0 keeps a_0 alone (when it is good)
        assert np.array_equal(t, want), "term counts differ from #(G_p within the window)"
    if say is not None:
        say(f"  windows: {len(w)} points, {n_amb} within rounding of a jump, {n_diff} differing")
    return n_amb
