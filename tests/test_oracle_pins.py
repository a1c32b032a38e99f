"""Pins of the oracle against what the paper and the mathematics fix.

Every check compares the oracle with something other than itself: values the
paper prints (tests/golden), exact rational brute force on tiny inputs, closed
forms (geometric series, z^d - 1 at roots of unity, Chebyshev T_d(cos t) =
cos(d t)), and the invariants the paper proves (window and error bounds, term
counts, the average-length bound of the theorem on correctness).
"""
from __future__ import annotations

import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from exact import (concave_majorant, cover_vertices, cplx_mul, exact_deriv_subset, exact_poly, exact_scale,
                   exact_scale_pair, exact_sum_subset, frac_abs_log2, to_complex)
from paper_2211_06320_amd import workloads

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = [int(v) for v in vals]
    return out


def bitlen(v: int) -> int:
    return int(v).bit_length()


# --------------------------------------------------------------------------- scale
def test_scale_paper_examples():
    """s(3+2i) = 2, s(3+3i) = 3 (Section 2.3, eq. sz)."""
    rows = []
    with open(os.path.join(GOLD, "scale_examples.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    for re, im, s in rows:
        assert oracle.lib().ora_scale1(re, im) == int(s)


def test_scale_powers_of_two_table():
    """|a_k| = 2^n gives s(a_k) = n + 1 (worked example's first table)."""
    g = read_golden("worked_example_d10.txt")
    c = np.array([2.0 ** n for n in g["exponents"]], complex)
    assert list(oracle.scale(c)) == g["scales"]


def _scale_edge_cases():
    rng = np.random.default_rng(5)
    vals = [(0.0, 1.0), (1.0, 0.0), (-1.0, 0.0), (0.5, 0.5), (2.0 ** -1074, 0.0),
            (0.0, -2.0 ** -1074), (2.0 ** -1022, 2.0 ** -1022), (1.7976931348623157e308, 0.0),
            (1.7976931348623157e308, 1.7976931348623157e308), (1 - 2.0 ** -53, 0.0),
            (math.sqrt(0.5), math.sqrt(0.5)), (np.nextafter(math.sqrt(0.5), 1), math.sqrt(0.5)),
            (0.6, 0.8), (np.nextafter(0.6, 1), 0.8), (np.nextafter(0.6, 0), 0.8),
            (3.0, 4.0), (np.nextafter(3.0, 0), 4.0), (1.0, 2.0 ** -60), (1 - 2.0 ** -53, 2.0 ** -26),
            (1 - 2.0 ** -53, 2.0 ** -27), (1 - 2.0 ** -53, 2.0 ** -26 + 2.0 ** -60)]
    for _ in range(300):
        e = int(rng.integers(-1070, 1020))
        vals.append((rng.uniform(-1, 1) * 2.0 ** e, rng.uniform(-1, 1) * 2.0 ** (e + int(rng.integers(-60, 3)))))
    # on the circle |z| = 2^m: x^2 + y^2 within an ulp or two of 4^m
    for _ in range(200):
        t = rng.uniform(0, 2 * math.pi)
        x, y = math.cos(t), math.sin(t)
        for dx in (-1, 0, 1):
            vals.append((float(np.nextafter(x, x + dx)) if dx else x, y))
    return vals


def test_scale_exact_bruteforce():
    """ora_scale agrees with the exact rational definition 4^(s-1) <= |z|^2 < 4^s."""
    for x, y in _scale_edge_cases():
        s = oracle.lib().ora_scale1(float(x), float(y))
        assert s == exact_scale(float(x), float(y)), (x, y)
    assert oracle.lib().ora_scale1(0.0, 0.0) == oracle.NEG_INF


def test_scale_lemma_product_bounds():
    """s(zz') - s(z) - s(z') in {-1, 0} (eq. sp) on exact products of small dyadics."""
    rng = np.random.default_rng(11)
    for _ in range(500):
        a = complex(int(rng.integers(-2**20, 2**20)), int(rng.integers(-2**20, 2**20))) * 2.0 ** int(rng.integers(-30, 30))
        b = complex(int(rng.integers(-2**20, 2**20)), int(rng.integers(-2**20, 2**20))) * 2.0 ** int(rng.integers(-30, 30))
        if a == 0 or b == 0:
            continue
        ab = a * b   # exact: 21-bit integers times powers of two
        assert Fr(ab.real) == Fr(a.real) * Fr(b.real) - Fr(a.imag) * Fr(b.imag)
        sa, sb, sab = (oracle.lib().ora_scale1(x.real, x.imag) for x in (a, b, ab))
        assert sab - sa - sb in (-1, 0)


# --------------------------------------------------------------------------- worked example
def test_worked_example_tables_and_sets():
    """Section 4.2: scale rows, Q_0 = {6,8,9}, Q_{-3} = {1,3,6,8,9}, bounds."""
    g = read_golden("worked_example_d10.txt")
    c = np.array([2.0 ** n for n in g["exponents"]], complex)
    p = g["p"][0]
    # the figures of Section 4.2 use the offset p alone (the remark there)
    P = oracle.precondition(c, offset=p)
    s = P.scales()
    assert list(s) == g["scales"]
    # s(a_k z^k) at |z| = 2^-3 (z = 1/8 makes every monomial a power of two)
    z = 0.125
    assert list(oracle.scale(c * z ** np.arange(11))) == g["scales_lambda_m3"]
    for lam, zpt, key in ((0, 1.0, "Q0"), (-3, 0.125, "Qm3")):
        r = P.eval(np.array([zpt + 0j]))
        assert r["lambda"][0] == lam
        N = r["N"][0]
        # the per-term rule the figures use: s(a_k) + k lambda >= N - p
        per_term = [k for k in range(11) if s[k] + k * lam >= N - p]
        assert per_term == g[key]
        # the algorithm's rule: G_p within [l, r].  It keeps every per-term
        # index, and may keep more (k = 4 at lambda = -3, which is in G_p)
        good = P.good()
        alg = [k for k in range(r["l"][0], r["r"][0] + 1) if good[k]]
        assert set(per_term) <= set(alg)
        assert r["terms"][0] == len(alg)
    # printed bounds: s(P - Q_0) <= 22 on |z| = 1, and |P - Q_{-3}| < 2^5 at |z| = 1/8
    for zpt, key, bound in ((1.0, "Q0", g["Q0_residual_scale_max"][0]),
                            (0.125, "Qm3", g["Qm3_residual_log2_bound"][0])):
        zc = complex(zpt)
        Pz = exact_poly(c, zc)
        Qz = exact_sum_subset(c, zc, g[key])
        res = (Pz[0] - Qz[0], Pz[1] - Qz[1])
        assert frac_abs_log2(res) < bound
    # s(Q_{-3}(z)) = 9 at z = 1/8 (positive real coefficients: no cancellation)
    Qz = exact_sum_subset(c, 0.125 + 0j, g["Qm3"])
    assert exact_scale(float(Qz[0]), float(Qz[1])) == g["Qm3_scale"][0]


def test_worked_example_algorithm_threshold():
    """With the algorithm's offset T = p + s(d) + 3 = 13 the windows widen (Section 4.3)."""
    g = read_golden("worked_example_d10.txt")
    c = np.array([2.0 ** n for n in g["exponents"]], complex)
    P = oracle.precondition(c, p=6)
    info = P.info()
    assert info.T == 6 + bitlen(10) + 3 == 13
    hk, hs = P.hull()
    Ehat = concave_majorant({k: int(v) for k, v in enumerate(g["scales"])})
    assert list(hk) == cover_vertices(Ehat)
    r = P.eval(np.array([1.0 + 0j, 0.125 + 0j]))
    good = P.good()
    sets = [[k for k in range(r["l"][i], r["r"][i] + 1) if good[k]] for i in range(2)]
    # the window superset contains the paper's kept sets
    assert set(g["Q0"]) <= set(sets[0]) and set(g["Qm3"]) <= set(sets[1])


# --------------------------------------------------------------------------- hull, G_p, windows
def _random_tiny_polys(rng, count=60):
    polys = []
    for i in range(count):
        d = int(rng.integers(1, 14))
        kind = i % 5
        if kind == 0:
            c = rng.uniform(-1, 1, d + 1) + 1j * rng.uniform(-1, 1, d + 1)
        elif kind == 1:
            g = rng.normal(0, 25, d + 1)
            c = np.exp2(g) * np.exp(1j * rng.uniform(0, 2 * np.pi, d + 1))
        elif kind == 2:   # zeros inside, at the ends, and wide scales
            g = rng.integers(-40, 40, d + 1)
            c = np.exp2(g.astype(float)) * np.exp(1j * rng.uniform(0, 2 * np.pi, d + 1))
            c[rng.random(d + 1) < 0.3] = 0
        elif kind == 3:   # integer scales on a concave profile (many vertices)
            k = np.arange(d + 1)
            c = np.exp2(np.floor(np.sqrt((k + 1) * (d + 1 - k)) * 3)) * (1 + 0j)
        else:             # dyadic integers: exact products
            c = rng.integers(-50, 50, d + 1) + 1j * rng.integers(-50, 50, d + 1)
        polys.append(np.asarray(c, np.complex128))
    return polys


def _tiny_points(rng, n=25):
    pts = list(workloads.spherical_points(n, int(rng.integers(1 << 30))))
    pts += [2.0 ** 40 + 0j, 2.0 ** -40 * (1 + 1j), 1.0 + 0j, -1.0 + 0j, 1j, 0.999 + 0.01j, 3 - 4j]
    return np.array(pts, np.complex128)


def test_hull_and_good_set_bruteforce():
    """Hull vertices = corners of the brute-force concave majorant; G_p = its definition."""
    rng = np.random.default_rng(2211)
    for c in _random_tiny_polys(rng):
        d = len(c) - 1
        for p in (1, 6, 24, 53):
            P = oracle.precondition(c, p)
            info = P.info()
            sc = {k: exact_scale(float(c[k].real), float(c[k].imag)) for k in range(d + 1)}
            sc = {k: v for k, v in sc.items() if v is not None}
            if not sc:
                assert info.n_hull == 0 and info.v == -1
                continue
            assert info.v == min(sc) and info.dt == max(sc)
            deff = max(sc) - min(sc)
            assert info.T == p + bitlen(max(deff, 1)) + 3
            Ehat = concave_majorant(sc)
            hk, hs = P.hull()
            assert list(hk) == cover_vertices(Ehat)
            assert all(Fr(int(s)) == Ehat[int(k)] for k, s in zip(hk, hs))
            good = P.good()
            for k in range(d + 1):
                want = k in sc and Fr(sc[k]) >= Ehat[k] - info.T
                assert bool(good[k]) == want, (k, p)


def test_windows_bruteforce():
    """[l, r] is the largest integer interval where Ehat(k) + lambda k >= N - T (eq. def:LRN)."""
    rng = np.random.default_rng(5)
    for c in _random_tiny_polys(rng, 40):
        P = oracle.precondition(c, 24)
        info = P.info()
        if info.n_hull == 0:
            continue
        sc = {k: v for k in range(len(c)) if (v := exact_scale(float(c[k].real), float(c[k].imag))) is not None}
        Ehat = concave_majorant(sc)
        z = _tiny_points(rng)
        r = P.eval(z)
        for i in range(len(z)):
            lam = Fr(float(r["lambda"][i]))
            vals = {k: Ehat[k] + lam * k for k in Ehat}
            N = max(vals.values())
            assert abs(float(N) - r["N"][i]) <= 1e-9 * max(1.0, abs(float(N)))
            inside = [k for k in Ehat if vals[k] >= N - info.T]
            assert inside == list(range(inside[0], inside[-1] + 1))   # an interval (concavity)
            # the oracle's window contains it and adds only eta-borderline indices
            assert r["l"][i] <= inside[0] and r["r"][i] >= inside[-1]
            for k in range(r["l"][i], r["r"][i] + 1):
                assert vals[k] >= N - info.T - Fr(1, 2 ** 18)
            # leftmost argmax
            kl = min(k for k in Ehat if vals[k] == N)
            assert N == Ehat[kl] + lam * kl


def test_lambda_accuracy():
    """lambda = log2|z| within a few units of 2^-53 max(1, |lambda|) (eq. defLambda).

    The error is absolute near |z| = 1 (log2 of 1 + delta), relative elsewhere; the
    window ends depend on lambda k, so this is the accuracy that matters."""
    import mpmath
    mpmath.mp.prec = 200
    z = np.concatenate([workloads.spherical_points(200, 3), [2.0 ** 900 + 0j, 2.0 ** -900 * (1 - 1j), 1e300 + 1e300j]])
    P = oracle.precondition(np.array([1, 1], complex), 53)
    lam = P.eval(z)["lambda"]
    for zi, li in zip(z, lam):
        want = mpmath.log(mpmath.sqrt(mpmath.mpf(zi.real) ** 2 + mpmath.mpf(zi.imag) ** 2), 2)
        assert abs(li - float(want)) <= 2.0 ** -50 * max(1.0, abs(float(want)))


# --------------------------------------------------------------------------- values
def _rel_to_D(val_m, val_e, exact_pair, D):
    """|val - exact| / D with everything brought to a common scale."""
    sh = -int(math.floor(math.log2(D))) if D > 0 else 0
    ex = to_complex(exact_pair, sh)
    got = math.ldexp(val_m.real, int(val_e) + sh) + 1j * math.ldexp(val_m.imag, int(val_e) + sh)
    return abs(got - ex) / math.ldexp(D, sh)


def test_values_exact_rational_tiny():
    """Compensated Horner and the FPE sum against exact rational P(z), plus the error bounds."""
    rng = np.random.default_rng(77)
    for c in _random_tiny_polys(rng, 40):
        d = len(c) - 1
        z = _tiny_points(rng, 12)
        hm, he = oracle.horner(c, z)
        for p in (53, 24):
            P = oracle.precondition(c, p)
            info = P.info()
            r = P.eval(z)
            for i, zi in enumerate(z):
                Pz = exact_poly(c, zi)
                # the tolerance scale D = sum |a_k||z|^k (a float suffices for a bound)
                logs = [math.log2(abs(a)) + k * math.log2(abs(zi)) for k, a in enumerate(c) if a != 0]
                if not logs:
                    assert r["m"][i] == 0 and hm[i] == 0
                    continue
                top = max(logs)
                D = sum(2.0 ** (x - top) for x in logs)   # D / 2^top
                Dfull = D * 2.0 ** 0  # keep scaled
                # compensated Horner: within 2^-52 |P| + tiny D
                sh = -int(math.floor(top))
                ex = to_complex(Pz, sh)
                got = math.ldexp(hm[i].real, int(he[i]) + sh) + 1j * math.ldexp(hm[i].imag, int(he[i]) + sh)
                Dsc = D * 2.0 ** (top + sh)
                assert abs(got - ex) <= 2.0 ** -52 * abs(ex) + 2.0 ** -90 * Dsc, (c, zi)
                if p != 53:
                    continue
                # FPE value: the exact sum over the kept terms, to double-double accuracy
                ks = [k for k in range(r["l"][i], r["r"][i] + 1) if P.good()[k]]
                Qz = exact_sum_subset(c, zi, ks)
                exq = to_complex(Qz, sh)
                gotq = math.ldexp(r["m"][i].real, int(r["e"][i]) + sh) + 1j * math.ldexp(r["m"][i].imag, int(r["e"][i]) + sh)
                assert abs(gotq - exq) <= 2.0 ** -52 * abs(exq) + 2.0 ** -90 * Dsc
                # error bound of Section 6: |P - Q| <= sum of dropped |a_k z^k| < d_eff 2^(N - T)
                res = (Pz[0] - Qz[0], Pz[1] - Qz[1])
                lres = frac_abs_log2(res)
                deff = info.dt - info.v
                assert lres < math.log2(max(deff, 1)) + r["N"][i] - info.T + 1e-9
                # term counts never exceed Horner's d + 1 (theorem on complexity)
                assert r["terms"][i] <= r["r"][i] - r["l"][i] + 1 <= d + 1


def test_target_relative_bound_with_cancellation():
    """|P - Q| <= 2^-(p-c)-2 |P| with c the cancelled bits (eqs. target, def_prec_loss)."""
    rng = np.random.default_rng(123)
    checked = 0
    for c in _random_tiny_polys(rng, 30):
        z = _tiny_points(rng, 10)
        for p in (8, 24):
            P = oracle.precondition(c, p)
            r = P.eval(z)
            for i, zi in enumerate(z):
                Pz = exact_poly(c, zi)
                lp = frac_abs_log2(Pz)
                if lp == -math.inf:
                    continue
                ks = [k for k in range(r["l"][i], r["r"][i] + 1) if P.good()[k]]
                Qz = exact_sum_subset(c, zi, ks)
                res = (Pz[0] - Qz[0], Pz[1] - Qz[1])
                lres = frac_abs_log2(res)
                if lres == -math.inf:
                    continue
                M = max(math.log2(abs(a)) + k * math.log2(abs(zi)) for k, a in enumerate(c) if a != 0)
                cbits = 0 if lp >= M else (math.floor(M) + 1) - (math.floor(lp) + 1)
                assert lres <= -(p - cbits) - 2 + lp + 1e-9
                checked += 1
    assert checked > 100


def _exact_c(coeffs, z, Pz):
    """The cancelled bits of eq. (def_prec_loss) exactly: 0 if |P(z)| >= M, else
    s(M) - s(P(z)), M = max_j |a_j z^j| (scales of exact complex rationals)."""
    zr = (Fr(float(z.real)), Fr(float(z.imag)))
    t = (Fr(1), Fr(0))
    sM = None
    best = Fr(0)
    for a in coeffs:
        term = cplx_mul((Fr(float(a.real)), Fr(float(a.imag))), t)
        q = term[0] ** 2 + term[1] ** 2
        if q > best:
            best, sM = q, exact_scale_pair(term)
        t = cplx_mul(t, zr)
    sP = exact_scale_pair(Pz)
    if Pz[0] ** 2 + Pz[1] ** 2 >= best:
        return 0
    return sM - sP


def _as_value(pair):
    """A nonzero complex rational as a double mantissa pair and a binary exponent."""
    shift = -int(math.floor(frac_abs_log2(pair)))
    return to_complex(pair, shift), -shift


def test_cancel_bound_brackets_exact_c():
    """max(0, floor(N) + 1 - s(P)) >= c, and <= c + 2 (eq. def_prec_loss with
    eq. shear: N - 1 <= s(M) <= floor(N) + 1), fed the exact P(z); exact rationals."""
    rng = np.random.default_rng(321)
    checked = tight = 0
    for c in _random_tiny_polys(rng, 40):
        z = _tiny_points(rng, 12)
        P = oracle.precondition(c, 53)
        r = P.eval(z)
        for i, zi in enumerate(z):
            if zi == 0:
                continue
            N = r["N"][i]
            if abs(N - round(N)) < 1e-9:        # FP64 N on an integer: floor undecided
                continue
            Pz = exact_poly(c, zi)
            if Pz[0] == 0 and Pz[1] == 0:
                continue
            m, e = _as_value(Pz)
            if exact_scale(m.real, m.imag) + e != exact_scale_pair(Pz):
                continue                          # rounding reached the next power of two
            cb = int(P.cancel_bound(np.array([zi]), [N], np.array([m]), [e])[0])
            ce = _exact_c(c, zi, Pz)
            assert ce <= cb <= ce + 2, (c, zi, ce, cb)
            tight += cb == ce
            checked += 1
    assert checked > 300 and tight > checked // 4


def test_cancel_bound_special_values():
    """P = 1 + z: P(-1) = 0 (every bit cancelled), P(0) = a_0 (c = 0), a non-finite
    z reports 0; z^d - 1 at rounded roots of unity: deep cancellation, bracketed
    by the exact c; P == 0 reports 0."""
    P = oracle.precondition(np.array([1, 1], complex), 53)
    z = np.array([-1 + 0j, 0j, np.nan + 0j, np.inf + 1j])
    r = P.eval(z)
    cb = P.cancel_bound(z, r["N"], r["m"], r["e"])
    assert cb[0] == 2 ** 31 - 1 and list(cb[1:]) == [0, 0, 0]
    d = 12
    c = np.zeros(d + 1, complex)
    c[0], c[d] = -1, 1
    P = oracle.precondition(c, 53)
    z = np.exp(2j * np.pi * np.array([1, 5, 7]) / d)
    r = P.eval(z)
    for i, zi in enumerate(z):
        Pz = exact_poly(c, zi)
        m, e = _as_value(Pz)
        cb = int(P.cancel_bound(np.array([zi]), [r["N"][i]], np.array([m]), [e])[0])
        ce = _exact_c(c, zi, Pz)
        assert ce > 40 and ce <= cb <= ce + 2
    Z = oracle.precondition(np.zeros(4, complex), 53)
    z = np.array([0.5 + 0.5j, 2.0 + 0j])
    r = Z.eval(z)
    assert list(Z.cancel_bound(z, r["N"], r["m"], r["e"])) == [0, 0]


def test_cancel_bound_in_error_bound():
    """The error bound of eq. (target) holds with the reported count in place of
    c (it is an upper bound of c): |P - Q| <= 2^-(p - bound) - 2 |P|."""
    rng = np.random.default_rng(77)
    checked = 0
    for c in _random_tiny_polys(rng, 30):
        z = _tiny_points(rng, 10)
        for p in (8, 24, 53):
            P = oracle.precondition(c, p)
            r = P.eval(z)
            cb = P.cancel_bound(z, r["N"], r["m"], r["e"])
            for i, zi in enumerate(z):
                Pz = exact_poly(c, zi)
                lp = frac_abs_log2(Pz)
                if lp == -math.inf or zi == 0 or cb[i] == 2 ** 31 - 1:
                    continue
                ks = [k for k in range(r["l"][i], r["r"][i] + 1) if P.good()[k]]
                Qz = exact_sum_subset(c, zi, ks)
                lres = frac_abs_log2((Pz[0] - Qz[0], Pz[1] - Qz[1]))
                if lres == -math.inf:
                    continue
                assert lres <= -(p - int(cb[i])) - 2 + lp + 1e-9
                checked += 1
    assert checked > 300


def test_geometric_series_closed_forms():
    """a_k = 1: flat cover, closed-form windows; value (z^(d+1) - 1)/(z - 1) exactly."""
    import mpmath
    mpmath.mp.prec = 400
    for d in (20, 64, 1000):
        c = np.ones(d + 1, complex)
        P = oracle.precondition(c, 53)
        info = P.info()
        assert info.n_hull == 2 and info.n_good == d + 1
        T = info.T
        z = np.concatenate([workloads.spherical_points(300, d), [1.0 + 0j, -1.0 + 0j]])
        r = P.eval(z)
        for i, zi in enumerate(z):
            lam = r["lambda"][i]
            if lam < 0:
                x = T / -lam
                if abs(x - round(x)) < 1e-6:
                    continue
                want = (0, min(d, math.floor(x)))
            elif lam > 0:
                x = T / lam
                if abs(x - round(x)) < 1e-6:
                    continue
                want = (max(0, d - math.floor(x)), d)
            else:
                want = (0, d)
            assert (r["l"][i], r["r"][i]) == want
        # values against the closed form with a wide window (T large: all terms kept
        # except those below 2^-150 of the largest)
        Pw = oracle.precondition(c, 150)
        rw = Pw.eval(z)
        for i, zi in enumerate(z):
            zm = mpmath.mpc(zi.real, zi.imag)
            if zi == 1:
                exact = mpmath.mpf(d + 1)
            else:
                exact = (zm ** (d + 1) - 1) / (zm - 1)
            got = mpmath.mpc(rw["m"][i].real, rw["m"][i].imag) * mpmath.mpf(2) ** int(rw["e"][i])
            D = sum(abs(zm) ** k for k in range(0, d + 1)) if d <= 64 else \
                (mpmath.mpf(d + 1) if abs(zm) == 1 else (abs(zm) ** (d + 1) - 1) / (abs(zm) - 1))
            # the output is rounded once to a double mantissa
            assert abs(got - exact) <= 2.0 ** -52 * abs(exact) + 2.0 ** -95 * D


def test_roots_of_unity():
    """z^d - 1: G_p = {0, d}; at |z| = 1 two terms; exact zeros at z = 1, -1 (d even), +-i (4 | d)."""
    for d in (8, 12, 64, 100):
        c = np.zeros(d + 1, complex)
        c[0], c[d] = -1, 1
        P = oracle.precondition(c, 53)
        assert list(np.nonzero(P.good())[0]) == [0, d]
        ang = 2 * np.pi * np.arange(d) / d
        z = np.cos(ang) + 1j * np.sin(ang)
        z[0] = 1.0
        z[d // 2] = -1.0
        if d % 4 == 0:
            z[d // 4] = 1j
            z[3 * d // 4] = -1j
        r = P.eval(z)
        for i, zi in enumerate(z):
            assert r["terms"][i] == 2 and (r["l"][i], r["r"][i]) == (0, d)
            ex = exact_poly(c, zi)   # z_fl^d - 1 exactly at the rounded root
            if zi in (1.0, -1.0, 1j, -1j):
                assert ex == (0, 0) and r["m"][i] == 0
            got = complex(math.ldexp(r["m"][i].real, int(r["e"][i])), math.ldexp(r["m"][i].imag, int(r["e"][i])))
            assert abs(got - to_complex(ex)) <= 2.0 ** -100 * 2 + 2.0 ** -52 * abs(to_complex(ex))


def test_chebyshev_closed_form():
    """T_d(cos t) = cos(d t): exact at the rounded x, and cos(d acos x) within rounding."""
    for d in (5, 16, 31):
        # coefficients of T_d by the three-term recurrence, exact small integers
        Tm, T = [1], [0, 1]
        for _ in range(d - 1):
            nxt = [0] + [2 * t for t in T]
            for k, v in enumerate(Tm):
                nxt[k] -= v
            Tm, T = T, nxt
        c = np.array(T if d >= 1 else Tm, dtype=complex)
        assert len(c) == d + 1
        th = np.linspace(0.05, 3.1, 40)
        x = np.cos(th).astype(complex)
        P = oracle.precondition(c, 53)
        r = P.eval(x)
        hm, he = oracle.horner(c, x)
        for i, xi in enumerate(x):
            exact = exact_poly(c, xi)
            D = float(sum(abs(ci) * abs(xi) ** k for k, ci in enumerate(c)))
            for m, e in ((r["m"][i], r["e"][i]), (hm[i], he[i])):
                got = complex(math.ldexp(m.real, int(e)), math.ldexp(m.imag, int(e)))
                assert abs(got - to_complex(exact)) <= 2.0 ** -52 * abs(to_complex(exact)) + 2.0 ** -60 * D
                # the closed form through acos of the rounded x
                assert abs(got.real - math.cos(d * math.acos(xi.real))) <= d * d * 2.0 ** -50 + 2.0 ** -44 * D


# --------------------------------------------------------------------------- P = 1 + z and averages
def test_one_plus_z_term_counts():
    """P = 1 + z (Section 4.1 example): both terms iff |lambda| <= T, with T = p + s(1) + 3."""
    for p in (1, 6, 53):
        P = oracle.precondition(np.array([1, 1], complex), p)
        T = P.info().T
        assert T == p + 4
        lam = np.array([-T - 0.5, -T + 0.5, -0.3, 0.0, 0.7, T - 0.5, T + 0.5])
        z = np.exp2(lam) * np.exp(1j * 0.3)
        r = P.eval(z)
        want = [1, 2, 2, 2, 2, 2, 1]
        assert list(r["terms"]) == want


def test_one_plus_z_sphere_average():
    """Sphere average of the term count of 1 + z is 1 + tanh(T ln 2) (Section 4.1 example)."""
    P = oracle.precondition(np.array([1, 1], complex), 1)
    T = P.info().T
    z = workloads.spherical_points(200_000, 99)
    U = P.eval(z)["terms"]
    want = 1 + math.tanh(T * math.log(2))
    se = math.sqrt(want * 0 + (want - 1) * (2 - want) / len(z))
    assert abs(U.mean() - want) < 5 * se + 1e-4


@pytest.mark.parametrize("family", ["uniform", "halfcircle"])
def test_average_window_bound(family):
    """avg over the sphere of #[l, r] < 1 + 1.9046 sqrt(d (p + s(d) + 3)) (theorem on
    correctness); the half-circle family (eq. halfcirclepoly) nearly saturates it."""
    d = 1000
    if family == "uniform":
        c = workloads.uniform_coeffs(d, 4)
    else:
        n = np.arange(d + 1)
        c = np.exp2(np.sqrt((n + 1.0) * (d + 1 - n))).astype(complex)
    P = oracle.precondition(c, 53)
    T = P.info().T
    z = workloads.spherical_points(20_000, 17)
    r = P.eval(z)
    W = (r["r"] - r["l"] + 1).astype(float)
    bound = 1 + 1.9046 * math.sqrt(d * T)
    assert W.mean() < bound
    if family == "halfcircle":
        # lower constant 1.3217 holds as d -> infinity; at d = 1000 expect the same order
        assert W.mean() > 0.8 * math.sqrt(d * T)


def test_shear_inequality():
    """|s(a_k) + k lambda - s(a_k z^k)| <= 1 (eq. shear), checked with exact scales."""
    rng = np.random.default_rng(8)
    for _ in range(300):
        a = complex(rng.uniform(-1, 1), rng.uniform(-1, 1)) * 2.0 ** int(rng.integers(-20, 20))
        zz = complex(rng.uniform(-1, 1), rng.uniform(-1, 1)) * 2.0 ** int(rng.integers(-3, 3))
        k = int(rng.integers(0, 12))
        prod = exact_sum_subset(np.array([0] * k + [a], complex), zz, [k])
        s_prod = None
        q = prod[0] ** 2 + prod[1] ** 2
        if q == 0:
            continue
        # exact scale of a rational: 4^(s-1) <= q < 4^s
        s_prod = math.floor(0.5 * (math.log2(q.numerator) - math.log2(q.denominator))) + 1
        while not (Fr(4) ** (s_prod - 1) <= q):
            s_prod -= 1
        while not (q < Fr(4) ** s_prod):
            s_prod += 1
        lam = math.log2(abs(zz))
        sa = oracle.lib().ora_scale1(a.real, a.imag)
        assert abs(sa + k * lam - s_prod) <= 1 + 1e-9


# --------------------------------------------------------------------------- edge cases
def test_edge_cases():
    # all-zero polynomial
    P = oracle.precondition(np.zeros(5, complex), 53)
    r = P.eval(np.array([0.3 + 0.1j, 0j]))
    assert (r["m"] == 0).all() and (r["terms"] == 0).all()
    # a_0 = 0 and a_d = 0: trimmed to [v, d']
    c = np.array([0, 0, 1 + 1j, 0.5, 2, 0, 0], complex)
    P = oracle.precondition(c, 53)
    info = P.info()
    assert (info.v, info.dt) == (2, 4) and info.T == 53 + bitlen(2) + 3
    z = np.array([0j, 0.5 + 0.25j, 3 - 1j])
    r = P.eval(z)
    assert r["m"][0] == 0 and r["terms"][0] == 0            # P(0) = a_0 = 0
    for i in (1, 2):
        ex = to_complex(exact_poly(c, z[i]))
        got = complex(math.ldexp(r["m"][i].real, int(r["e"][i])), math.ldexp(r["m"][i].imag, int(r["e"][i])))
        assert abs(got - ex) <= 2.0 ** -50 * abs(ex)
        assert 2 <= r["l"][i] <= r["r"][i] <= 4
    # monomial
    P = oracle.precondition(np.array([0, 0, 0, 2 - 1j], complex), 53)
    r = P.eval(np.array([1.5 + 0.5j]))
    assert r["terms"][0] == 1 and (r["l"][0], r["r"][0]) == (3, 3)
    got = complex(math.ldexp(r["m"][0].real, int(r["e"][0])), math.ldexp(r["m"][0].imag, int(r["e"][0])))
    assert abs(got - (2 - 1j) * (1.5 + 0.5j) ** 3) < 1e-14 * abs(got)
    # z = 0 gives a_0; non-finite z gives NaN
    P = oracle.precondition(np.array([3 + 4j, 1, 1], complex), 53)
    r = P.eval(np.array([0j, complex(np.inf, 0), complex(np.nan, 1)]))
    got = complex(math.ldexp(r["m"][0].real, int(r["e"][0])), math.ldexp(r["m"][0].imag, int(r["e"][0])))
    assert got == 3 + 4j and r["terms"][0] == 1
    assert np.isnan(r["m"][1:].real).all()


def test_huge_exponents_no_overflow():
    """Values far beyond the FP64 range come out as mantissa 2^e (Section 2.2 model)."""
    import mpmath
    mpmath.mp.prec = 300
    d = 5000
    c = workloads.uniform_coeffs(d, 1)
    z = np.array([2.0 + 0.5j, -1.7 + 0.1j, 0.3 - 0.2j])
    P = oracle.precondition(c, 53)
    r = P.eval(z)
    hm, he = oracle.horner(c, z)
    for i, zi in enumerate(z):
        zm = mpmath.mpc(zi.real, zi.imag)
        ex = mpmath.polyval([mpmath.mpc(a.real, a.imag) for a in c[::-1]], zm)
        D = sum(abs(mpmath.mpc(a.real, a.imag)) * abs(zm) ** k for k, a in enumerate(c))
        for m, e in ((r["m"][i], r["e"][i]), (hm[i], he[i])):
            got = mpmath.mpc(m.real, m.imag) * mpmath.mpf(2) ** int(e)
            assert abs(got - ex) / D < 2.0 ** -50
    assert he.max() > 1024   # beyond FP64


def test_derivative_exact_rational_tiny():
    """Q' (the derivative of the kept terms) against exact rationals over the same
    window and good set, and its scale sum |k a_k||z|^(k-1) against a float sum."""
    rng = np.random.default_rng(91)
    for c in _random_tiny_polys(rng, 25):
        z = _tiny_points(rng, 10)
        P = oracle.precondition(c, 53)
        r = P.eval(z)
        rd = P.eval_deriv(z)
        assert np.array_equal(rd["m"], r["m"]) and np.array_equal(rd["e"], r["e"])
        good = P.good()
        for i, zi in enumerate(z):
            ks = [k for k in range(r["l"][i], r["r"][i] + 1) if good[k] and k >= 1]
            terms = [(k, abs(c[k]) * k * abs(zi) ** (k - 1)) for k in range(max(r["l"][i], 1), r["r"][i] + 1)
                     if c[k] != 0]
            if not terms:
                assert rd["md"][i] == 0
                continue
            logs = [math.log2(t) for _, t in terms if t > 0]
            top = max(logs)
            sh = -int(math.floor(top))
            Dd = sum(2.0 ** (x - top) for x in logs) * 2.0 ** (top + sh)
            ex = to_complex(exact_deriv_subset(c, zi, ks), sh)
            got = math.ldexp(rd["md"][i].real, int(rd["ed"][i]) + sh) + 1j * math.ldexp(rd["md"][i].imag, int(rd["ed"][i]) + sh)
            assert abs(got - ex) <= 2.0 ** -52 * abs(ex) + 2.0 ** -90 * Dd, (c, zi)
            gotD = math.ldexp(rd["ddwin_m"][i], int(rd["ddwin_e"][i]) + sh)
            assert abs(gotD - Dd) <= 1e-12 * Dd


def test_derivative_geometric_series_closed_form():
    """a_k = 1: where the window keeps every term, Q' = P' =
    (d z^(d+1) - (d+1) z^d + 1) / (z - 1)^2, compared in exact rationals."""
    rng = np.random.default_rng(92)
    for d in (5, 17, 40):
        c = np.ones(d + 1, np.complex128)
        P = oracle.precondition(c, 53)
        zs = 2.0 ** rng.uniform(-0.05, 0.05, 8) * np.exp(1j * rng.uniform(0.3, 6.0, 8))
        rd = P.eval_deriv(zs)
        for i, zi in enumerate(zs):
            z = (Fr(float(zi.real)), Fr(float(zi.imag)))
            zd = (Fr(1), Fr(0))
            for _ in range(d):
                zd = cplx_mul(zd, z)                   # z^d
            zd1 = cplx_mul(zd, z)
            num = (d * zd1[0] - (d + 1) * zd[0] + 1, d * zd1[1] - (d + 1) * zd[1])
            zm1 = (z[0] - 1, z[1])
            den = cplx_mul(zm1, zm1)
            q = den[0] ** 2 + den[1] ** 2
            ex = ((num[0] * den[0] + num[1] * den[1]) / q, (num[1] * den[0] - num[0] * den[1]) / q)
            exc = to_complex(ex)
            got = rd["md"][i] * 2.0 ** rd["ed"][i]
            assert abs(got - exc) <= 2.0 ** -50 * d * d, (d, zi, got, exc)


def test_newton_step_paper_example():
    """P = z^64 + 1 at z = 10 (Section 7.2): the window keeps only z^64 (a_0 lies
    more than T bits below), so Q'/Q gives the step z / 64: 10 - N(10) = 0.15625."""
    c = np.zeros(65, np.complex128)
    c[0] = 1.0
    c[64] = 1.0
    P = oracle.precondition(c, 53)
    rd = P.eval_deriv(np.array([10.0 + 0j]))
    q = rd["m"][0] * 2.0 ** rd["e"][0]
    qd = rd["md"][0] * 2.0 ** rd["ed"][0]
    assert q == 10.0 ** 64 and qd == 64 * 10.0 ** 63
    step = (rd["m"][0] / rd["md"][0]) * 2.0 ** (int(rd["e"][0]) - int(rd["ed"][0]))
    assert 10.0 - (10.0 - step) == 0.15625


def _xc(m, e):
    """(complex mantissa, exponent) -> exact Fraction pair."""
    sc = Fr(2) ** int(e) if e >= 0 else Fr(1, 2 ** int(-e))
    return (Fr(float(m.real)) * sc, Fr(float(m.imag)) * sc)


def test_adjoint_duality_exact_rational_tiny():
    """Reverse mode against forward mode, exactly: for any direction delta,
    sum_k conj(grad_a[k]) delta_k equals sum_j conj(g_j) Q_j(delta), where
    Q_j(delta) is the exact rational sum of delta_k z_j^k over the kept terms of
    point j (same window and G_p).  A dropped conjugate, a wrong power or a
    missed term breaks the identity."""
    rng = np.random.default_rng(93)
    for c in _random_tiny_polys(rng, 30):
        z = _tiny_points(rng, 8)
        d = len(c) - 1
        P = oracle.precondition(c, 53)
        r = P.eval(z)
        good = P.good()
        g = rng.normal(size=len(z)) + 1j * rng.normal(size=len(z))
        delta = rng.normal(size=d + 1) + 1j * rng.normal(size=d + 1)
        adj = P.adjoint(z, g)
        lhs = (Fr(0), Fr(0))
        bound = Fr(0)
        for k in range(d + 1):
            gk = _xc(adj["ga_m"][k], adj["ga_e"][k])
            dk = (Fr(float(delta[k].real)), Fr(float(delta[k].imag)))
            t = cplx_mul((gk[0], -gk[1]), dk)
            lhs = (lhs[0] + t[0], lhs[1] + t[1])
            sk = Fr(float(adj["ga_scale_m"][k])) * (Fr(2) ** int(adj["ga_scale_e"][k]) if adj["ga_scale_e"][k] >= 0
                                                   else Fr(1, 2 ** int(-adj["ga_scale_e"][k])))
            # the oracle rounds each grad_a[k] once (double-double inside)
            bound += Fr(abs(delta[k])) * (Fr(2) ** -52 * (abs(gk[0]) + abs(gk[1])) + Fr(2) ** -95 * sk)
            if not good[k]:
                assert adj["ga_m"][k] == 0
        rhs = (Fr(0), Fr(0))
        for j, zj in enumerate(z):
            if not np.isfinite(zj) or r["l"][j] > r["r"][j]:
                continue
            ks = [k for k in range(r["l"][j], r["r"][j] + 1) if good[k]]
            q = exact_sum_subset(delta, zj, ks)
            t = cplx_mul((Fr(float(g[j].real)), -Fr(float(g[j].imag))), q)
            rhs = (rhs[0] + t[0], rhs[1] + t[1])
        diff = abs(lhs[0] - rhs[0]) + abs(lhs[1] - rhs[1])
        assert diff <= 2 * bound + Fr(1, 2 ** 1000), (c, float(diff), float(bound))


def test_adjoint_geometric_series_closed_form():
    """a_k = 1 with every term kept (|z| near 1, so the window is [0, d]):
    sum_k grad_a[k] = sum_j g_j (1 - w_j^(d+1)) / (1 - w_j), w_j = conj(z_j),
    and grad_a[0] = sum_j g_j, in exact rationals."""
    rng = np.random.default_rng(94)
    for d in (4, 15, 33):
        c = np.ones(d + 1, np.complex128)
        P = oracle.precondition(c, 53)
        z = 2.0 ** rng.uniform(-0.05, 0.05, 6) * np.exp(1j * rng.uniform(0.3, 6.0, 6))
        r = P.eval(z)
        assert (r["l"] == 0).all() and (r["r"] == d).all() and P.good().all()
        g = rng.normal(size=6) + 1j * rng.normal(size=6)
        adj = P.adjoint(z, g)
        tot = (Fr(0), Fr(0))
        for k in range(d + 1):
            gk = _xc(adj["ga_m"][k], adj["ga_e"][k])
            tot = (tot[0] + gk[0], tot[1] + gk[1])
        ex = (Fr(0), Fr(0))
        for j in range(6):
            w = (Fr(float(z[j].real)), -Fr(float(z[j].imag)))
            wp = (Fr(1), Fr(0))
            for _ in range(d + 1):
                wp = cplx_mul(wp, w)
            num = (1 - wp[0], -wp[1])
            den = (1 - w[0], -w[1])
            q = den[0] ** 2 + den[1] ** 2
            s = ((num[0] * den[0] + num[1] * den[1]) / q, (num[1] * den[0] - num[0] * den[1]) / q)
            t = cplx_mul((Fr(float(g[j].real)), Fr(float(g[j].imag))), s)
            ex = (ex[0] + t[0], ex[1] + t[1])
        err = abs(to_complex(tot) - to_complex(ex))
        assert err <= 2.0 ** -48 * (d + 1) * np.abs(g).sum(), (d, err)
        g0 = _xc(adj["ga_m"][0], adj["ga_e"][0])
        assert to_complex(g0) == complex(sum(Fr(float(x.real)) for x in g), sum(Fr(float(x.imag)) for x in g))


def _loss(P, z, cw):
    """L = Re sum_j conj(c_j) Q_j with c_j = cw_j 2^-e0_j (each point O(1))."""
    r = P.eval(z)
    tot = 0.0
    for j in range(len(z)):
        v = np.conj(cw[j][0]) * r["m"][j]
        tot += math.ldexp(v.real, int(r["e"][j] - cw[j][1]))
    return tot


def test_adjoint_central_differences():
    """Central differences of the oracle's own evaluation in Re and Im of a_k
    (kept k; the plan's hull and G_p unchanged by the step) and of z (window
    unchanged by the step) against its reverse mode, with the complex
    convention grad = dL/dRe + i dL/dIm for L = Re sum_j conj(c_j) Q_j."""
    rng = np.random.default_rng(95)
    checked_a = checked_z = 0
    for c in _random_tiny_polys(rng, 20):
        d = len(c) - 1
        P = oracle.precondition(c, 53)
        good = P.good()
        hk, hs = P.hull()
        z = np.array(list(workloads.spherical_points(6, int(rng.integers(1 << 30)))) + [0.9 + 0.3j], np.complex128)
        r0 = P.eval(z)
        cw = [(complex(rng.normal(), rng.normal()), int(r0["e"][j])) for j in range(len(z))]
        g = np.array([math.ldexp(1.0, -e) * w for w, e in cw], np.complex128)
        adj = P.adjoint(z, g)
        ga = np.array([math.ldexp(m.real, int(e)) + 1j * math.ldexp(m.imag, int(e))
                       for m, e in zip(adj["ga_m"], adj["ga_e"])])
        for k in [k for k in range(d + 1) if good[k]][:3]:
            h = 2.0 ** -20 * abs(c[k])
            vals = []
            for step in (h, -h, 1j * h, -1j * h):
                cp = c.copy()
                cp[k] += step
                Pp = oracle.precondition(cp, 53)
                hk2, hs2 = Pp.hull()
                if not (np.array_equal(Pp.good(), good) and np.array_equal(hk2, hk) and np.array_equal(hs2, hs)):
                    break
                vals.append(_loss(Pp, z, cw))
            if len(vals) < 4:
                continue
            fd = (vals[0] - vals[1]) / (2 * h) + 1j * (vals[2] - vals[3]) / (2 * h)
            scale = sum(abs(w) * math.ldexp(m, int(e - e0)) for (w, e0), m, e in
                        zip(cw, r0["dwin_m"], r0["dwin_e"]))
            assert abs(fd - ga[k]) <= 2.0 ** -30 * abs(ga[k]) + 2.0 ** -48 * scale / h, (k, fd, ga[k])
            checked_a += 1
        gz = adj["gz_m"] * np.exp2(adj["gz_e"].astype(float))
        for j, zj in enumerate(z):
            if not (0.25 < abs(zj) < 4):
                continue
            h = 1e-6 * abs(zj)
            vals, same = [], True
            for step in (h, -h, 1j * h, -1j * h):
                rp = P.eval(np.array([zj + step]))
                same &= rp["l"][0] == r0["l"][j] and rp["r"][0] == r0["r"][j]
                q = rp["m"][0] * 2.0 ** rp["e"][0]
                vals.append((np.conj(g[j]) * q).real)
            if not same:
                continue
            fd = (vals[0] - vals[1]) / (2 * h) + 1j * (vals[2] - vals[3]) / (2 * h)
            sc = abs(g[j]) * (math.ldexp(adj["gz_scale_m"][j] / abs(g[j]) if g[j] else 0.0, int(adj["gz_scale_e"][j]))
                              + math.ldexp(r0["dwin_m"][j], int(r0["dwin_e"][j])) / abs(zj))
            assert abs(fd - gz[j]) <= 1e-6 * sc, (j, zj, fd, gz[j])
            checked_z += 1
    assert checked_a >= 20 and checked_z >= 20, (checked_a, checked_z)
