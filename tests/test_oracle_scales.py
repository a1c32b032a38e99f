"""Pins of the oracle's tolerance scales and of its plain-FP64 window sum.

Every parity test divides an error by a scale the oracle returns:
  absum       D(z) = sum_k |a_k| |z|^k                 (the parity metric's denominator)
  dwin        sum over the window [l, r] of |a_k| |z|^k (the same, restricted to the window)
  ddwin       sum over the window of |k a_k| |z|^(k-1)  (the derivative's scale)
  ga_scale    sum over the points keeping k of |g_j| |z_j|^k   (the adjoint's scale)
Each is checked here against something other than the oracle: high-precision
sums (mpmath at 200 bits, or 64-bit-mantissa long doubles for a million terms)
over the definition, and closed forms of the geometric series.  A scale off by
a factor 2, a skipped k = 0 or a power |z|^(k-1) in place of |z|^k fails them.

The plain-FP64 window sum (eval_fp64, the form the CPU baseline times) is
pinned against exact rationals over the kept terms.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np
import pytest

import oracle
from exact import exact_sum_subset, to_complex
from paper_2211_06320_amd import workloads

mpmath.mp.prec = 200


def _random_polys(rng, count):
    out = []
    for i in range(count):
        d = int(rng.integers(1, 30))
        kind = i % 4
        if kind == 0:
            c = rng.uniform(-1, 1, d + 1) + 1j * rng.uniform(-1, 1, d + 1)
        elif kind == 1:
            c = np.exp2(rng.normal(0, 20, d + 1)) * np.exp(1j * rng.uniform(0, 2 * np.pi, d + 1))
        elif kind == 2:
            c = rng.uniform(-1, 1, d + 1) + 1j * rng.uniform(-1, 1, d + 1)
            c[rng.random(d + 1) < 0.4] = 0
            c[0] = 0.75 - 0.5j             # a_0 present: a skipped k = 0 shows
        else:
            c = rng.integers(-9, 9, d + 1) + 1j * rng.integers(-9, 9, d + 1)
        out.append(np.asarray(c, np.complex128))
    return out


def _points(rng, n):
    z = list(workloads.spherical_points(n, int(rng.integers(1 << 30))))
    z += [0.3 - 0.1j, 2.5 + 1j, 1.0 + 0j, -0.999 + 0.02j, 1e-5 + 0j]
    return np.array(z, np.complex128)


def _mp_abs(c):
    return mpmath.sqrt(mpmath.mpf(c.real) ** 2 + mpmath.mpf(c.imag) ** 2)


def _mp_val(m, e):
    return mpmath.ldexp(mpmath.mpf(float(m)), int(e))


def _rel(got, want):
    if want == 0:
        return 0.0 if got == 0 else math.inf
    return float(abs(got - want) / want)


def test_absum_definition_mpmath():
    """absum = sum_k |a_k| |z|^k, at 200 bits, relative error <= 2^-45 (a few
    roundings per term; the sum has positive terms only)."""
    rng = np.random.default_rng(601)
    worst = 0.0
    for c in _random_polys(rng, 40):
        z = _points(rng, 6)
        dm, de = oracle.absum(c, z)
        for j, zj in enumerate(z):
            r = _mp_abs(zj)
            want = mpmath.fsum(_mp_abs(a) * r ** k for k, a in enumerate(c) if a != 0)
            worst = max(worst, _rel(_mp_val(dm[j], de[j]), want))
    assert worst <= 2.0 ** -45, worst


@pytest.mark.parametrize("d", [20, 64, 1000])
def test_absum_geometric_closed_form(d):
    """a_k = 1: D = (|z|^(d+1) - 1) / (|z| - 1) (and d + 1 at |z| = 1)."""
    rng = np.random.default_rng(602 + d)
    c = np.ones(d + 1, np.complex128)
    z = np.concatenate([workloads.spherical_points(20, 603 + d), [1.0 + 0j, 1j, 0.5 + 0j, 1.01 + 0.0j]])
    dm, de = oracle.absum(c, z)
    for j, zj in enumerate(z):
        r = _mp_abs(zj)
        want = mpmath.mpf(d + 1) if r == 1 else (r ** (d + 1) - 1) / (r - 1)
        assert _rel(_mp_val(dm[j], de[j]), want) <= (d + 2) * 2.0 ** -50, (d, zj)
    # planted mistakes (applied here to the oracle's output, not in the oracle):
    # each moves some point of this set far outside the tolerance
    worst = {"x2": 0.0, "no_k0": 0.0, "pow_k-1": 0.0}
    for j, zj in enumerate(z):
        r = _mp_abs(zj)
        if r == 1:
            continue
        want = (r ** (d + 1) - 1) / (r - 1)
        got = _mp_val(dm[j], de[j])
        worst["x2"] = max(worst["x2"], _rel(2 * got, want))
        worst["no_k0"] = max(worst["no_k0"], _rel(got - 1, want))
        worst["pow_k-1"] = max(worst["pow_k-1"], _rel(got / r, want))
    assert min(worst.values()) > 1000 * (d + 2) * 2.0 ** -50, worst


def test_absum_degree_1e6_long_double():
    """The headline polynomial (d = 10^6, Re, Im of a_k uniform): D at ten
    spherical points against a long-double sum in the log domain (each term
    exp(ln|a_k| + k ln|z| - M), M the largest exponent; relative error of a
    term below 10^6 |ln|z|| 2^-63 ~ 10^-13).  The oracle forms |z|^k by k
    rounded products, so its D carries a relative error up to (d + 2) 2^-52
    (2 10^-10 here; harmless in a denominator), which is the bound checked."""
    wl = workloads.workload("uniform_d1e6", n_points=10)
    c = wl.coeffs
    ld = np.longdouble
    la = np.log(np.hypot(c.real.astype(ld), c.imag.astype(ld)))
    k = np.arange(wl.degree + 1, dtype=ld)
    dm, de = oracle.absum(c, wl.points)
    for j, zj in enumerate(wl.points):
        lr = np.log(np.hypot(ld(zj.real), ld(zj.imag)))
        x = la + k * lr
        M = x.max()
        S = np.sum(np.exp(x - M))
        got = np.log(ld(dm[j])) + ld(int(de[j])) * np.log(ld(2)) - M
        assert abs(float(got - np.log(S))) <= (wl.degree + 2) * 2.0 ** -52, (j, zj)


def test_window_scale_definition_mpmath():
    """dwin = sum over the oracle's window [l, r] of |a_k| |z|^k (every nonzero
    a_k of the window, good or not), at 200 bits; it never exceeds absum, and
    equals it where the window is the whole index range."""
    rng = np.random.default_rng(604)
    worst = 0.0
    full = 0
    for c in _random_polys(rng, 40):
        z = _points(rng, 6)
        for p in (53, 8):
            P = oracle.precondition(c, p)
            r = P.eval(z)
            am, ae = oracle.absum(c, z)
            info = P.info()
            for j, zj in enumerate(z):
                if info.n_hull == 0 or r["l"][j] > r["r"][j]:
                    continue
                rz = _mp_abs(zj)
                want = mpmath.fsum(_mp_abs(c[k]) * rz ** k for k in range(r["l"][j], r["r"][j] + 1) if c[k] != 0)
                got = _mp_val(r["dwin_m"][j], r["dwin_e"][j])
                worst = max(worst, _rel(got, want))
                tot = _mp_val(am[j], ae[j])
                assert got <= tot * (1 + 2.0 ** -40)
                if r["l"][j] <= info.v and r["r"][j] >= info.dt:
                    assert _rel(got, tot) <= 2.0 ** -44
                    full += 1
    assert worst <= 2.0 ** -45, worst
    assert full > 50


@pytest.mark.parametrize("d", [20, 64, 1000])
def test_window_scale_geometric_closed_form(d):
    """a_k = 1 (flat cover): the window is [0, min(d, floor(T/|lambda|))] for
    |z| < 1 and [max(0, d - floor(T/lambda)), d] for |z| > 1 (eq. def:LRN), and
    dwin = (|z|^(r+1) - |z|^l) / (|z| - 1) over it."""
    c = np.ones(d + 1, np.complex128)
    P = oracle.precondition(c, 53)
    z = workloads.spherical_points(40, 605 + d)
    r = P.eval(z)
    for j, zj in enumerate(z):
        rz = _mp_abs(zj)
        l, rr = int(r["l"][j]), int(r["r"][j])
        want = (rz ** (rr + 1) - rz ** l) / (rz - 1)
        assert _rel(_mp_val(r["dwin_m"][j], r["dwin_e"][j]), want) <= (d + 2) * 2.0 ** -50, (d, zj)


def test_derivative_scale_definition_and_closed_form():
    """ddwin = sum over the window of |k a_k| |z|^(k-1) (k >= 1), at 200 bits;
    for a_k = 1 with the whole window kept, sum_{k=1}^d k r^(k-1), the
    derivative of (r^(d+1) - 1) / (r - 1)."""
    rng = np.random.default_rng(606)
    worst = 0.0
    for c in _random_polys(rng, 30):
        z = _points(rng, 5)
        P = oracle.precondition(c, 53)
        r = P.eval(z)
        dv = P.eval_deriv(z)
        for j, zj in enumerate(z):
            if r["l"][j] > r["r"][j]:
                continue
            rz = _mp_abs(zj)
            want = mpmath.fsum(k * _mp_abs(c[k]) * rz ** (k - 1)
                               for k in range(max(1, r["l"][j]), r["r"][j] + 1) if c[k] != 0)
            got = _mp_val(dv["ddwin_m"][j], dv["ddwin_e"][j])
            if want == 0:
                assert got == 0
                continue
            worst = max(worst, _rel(got, want))
    assert worst <= 2.0 ** -45, worst
    d = 40
    c = np.ones(d + 1, np.complex128)
    P = oracle.precondition(c, 53)
    z = 2.0 ** np.random.default_rng(607).uniform(-0.05, 0.05, 10) * np.exp(1j * np.arange(10))
    r = P.eval(z)
    assert (r["l"] == 0).all() and (r["r"] == d).all()
    dv = P.eval_deriv(z)
    for j, zj in enumerate(z):
        x = _mp_abs(zj)
        want = mpmath.diff(lambda t: (t ** (d + 1) - 1) / (t - 1), x)
        assert _rel(_mp_val(dv["ddwin_m"][j], dv["ddwin_e"][j]), want) <= 2.0 ** -40


def test_adjoint_scale_definition_mpmath():
    """ga_scale[k] = sum over the points j whose kept terms include k (k in G_p
    within the oracle's window [l_j, r_j]) of |g_j| |z_j|^k, at 200 bits;
    zero where no point keeps k.  gz_scale_j = |g_j| ddwin_j."""
    rng = np.random.default_rng(608)
    worst = 0.0
    for c in _random_polys(rng, 25):
        d = len(c) - 1
        z = _points(rng, 6)
        g = rng.normal(size=len(z)) + 1j * rng.normal(size=len(z))
        P = oracle.precondition(c, 53)
        r = P.eval(z)
        good = P.good()
        adj = P.adjoint(z, g)
        for k in range(d + 1):
            want = mpmath.fsum(_mp_abs(g[j]) * _mp_abs(z[j]) ** k for j in range(len(z))
                               if good[k] and r["l"][j] <= k <= r["r"][j])
            got = _mp_val(adj["ga_scale_m"][k], adj["ga_scale_e"][k])
            if want == 0:
                assert got == 0
                continue
            worst = max(worst, _rel(got, want))
        dv = P.eval_deriv(z)
        for j in range(len(z)):
            want = _mp_abs(g[j]) * _mp_val(dv["ddwin_m"][j], dv["ddwin_e"][j])
            got = _mp_val(adj["gz_scale_m"][j], adj["gz_scale_e"][j])
            assert _rel(got, want) <= 2.0 ** -50 or want == got
    assert worst <= 2.0 ** -45, worst


def test_adjoint_scale_geometric_closed_form():
    """a_k = 1, every term kept: sum_k ga_scale[k] = sum_j |g_j| (r_j^(d+1) - 1) / (r_j - 1)."""
    rng = np.random.default_rng(609)
    for d in (8, 33, 200):
        c = np.ones(d + 1, np.complex128)
        P = oracle.precondition(c, 53)
        z = 2.0 ** rng.uniform(-0.02, 0.02, 7) * np.exp(1j * rng.uniform(0, 6, 7))
        r = P.eval(z)
        assert (r["l"] == 0).all() and (r["r"] == d).all()
        g = rng.normal(size=7) + 1j * rng.normal(size=7)
        adj = P.adjoint(z, g)
        got = mpmath.fsum(_mp_val(m, e) for m, e in zip(adj["ga_scale_m"], adj["ga_scale_e"]))
        want = mpmath.fsum(_mp_abs(gj) * ((_mp_abs(zj) ** (d + 1) - 1) / (_mp_abs(zj) - 1)) for gj, zj in zip(g, z))
        assert _rel(got, want) <= (d + 2) * 2.0 ** -48, d
        assert _rel(_mp_val(adj["ga_scale_m"][0], adj["ga_scale_e"][0]), mpmath.fsum(_mp_abs(x) for x in g)) <= 2.0 ** -50


def test_eval_fp64_exact_rational():
    """The plain-FP64 window sum against the exact sum over the kept terms:
    |FP64 - exact| <= (4 W + 8) 2^-53 dwin (Horner's rule: a few roundings per
    step, each relative to the partial, bounded by the window's scale)."""
    rng = np.random.default_rng(610)
    checked = 0
    for c in _random_polys(rng, 40):
        z = _points(rng, 6)
        P = oracle.precondition(c, 53)
        r = P.eval(z)
        fm, fe = P.eval_fp64(z)
        good = P.good()
        for j, zj in enumerate(z):
            if r["l"][j] > r["r"][j]:
                assert fm[j] == 0 and fe[j] == 0
                continue
            ks = [k for k in range(r["l"][j], r["r"][j] + 1) if good[k]]
            ex = exact_sum_subset(c, zj, ks)
            D = math.ldexp(r["dwin_m"][j], 0)
            sh = -int(r["dwin_e"][j])
            exv = to_complex(ex, sh)
            got = math.ldexp(fm[j].real, int(fe[j]) + sh) + 1j * math.ldexp(fm[j].imag, int(fe[j]) + sh)
            W = r["r"][j] - r["l"][j] + 1
            assert abs(got - exv) <= (4 * W + 8) * 2.0 ** -53 * D, (c, zj)
            checked += 1
    assert checked > 200
    # special points
    P = oracle.precondition(np.array([3 + 4j, 1, 2], complex), 53)
    fm, fe = P.eval_fp64(np.array([0, complex(np.nan, 0)], complex))
    assert fm[0] * 2.0 ** fe[0] == 3 + 4j and np.isnan(fm[1].real)


def test_level_sets_match_eval():
    """level_sets(lambda) gives the N and the window ends eval uses."""
    wl = workloads.workload("uniform_d1000")
    P = oracle.precondition(wl.coeffs, 53)
    r = P.eval(wl.points[:2000])
    N, xl, xr = P.level_sets(r["lambda"])
    assert np.array_equal(N, r["N"])
    info = P.info()
    l = np.maximum(np.ceil(xl - 2.0 ** -20), info.v).astype(np.int64)
    rr = np.minimum(np.floor(xr + 2.0 ** -20), info.dt).astype(np.int64)
    assert np.array_equal(l, r["l"]) and np.array_equal(rr, r["r"])
