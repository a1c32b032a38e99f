"""Exact (rational) arithmetic used to pin the oracle: brute force on tiny inputs.

Nothing here is shared with the HIP path.  Every double is an exact rational, so
Fraction arithmetic gives the true value of P(z) at the given (rounded) z, the
exact scale s(z) = 1 + floor(log2|z|) and the exact concave majorant of the
integer scales.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr


def exact_scale(x: float, y: float):
    """s(x + iy) = sigma with 4^(sigma-1) <= x^2 + y^2 < 4^sigma; None for zero."""
    if x == 0 and y == 0:
        return None
    q = Fr(x) ** 2 + Fr(y) ** 2
    # start near the float estimate, then walk to the exact answer
    m = max(math.frexp(abs(x))[1] if x else -10**9, math.frexp(abs(y))[1] if y else -10**9)
    sigma = m
    while not (Fr(4) ** (sigma - 1) <= q):
        sigma -= 1
    while not (q < Fr(4) ** sigma):
        sigma += 1
    assert Fr(4) ** (sigma - 1) <= q < Fr(4) ** sigma
    return sigma


def exact_scale_pair(pair):
    """s of a complex rational (re, im): sigma with 4^(sigma-1) <= |v|^2 < 4^sigma; None for zero."""
    q = pair[0] * pair[0] + pair[1] * pair[1]
    if q == 0:
        return None
    sigma = int(math.floor(0.5 * (math.log2(q.numerator) - math.log2(q.denominator)))) + 1
    while not (Fr(4) ** (sigma - 1) <= q):
        sigma -= 1
    while not (q < Fr(4) ** sigma):
        sigma += 1
    return sigma


def cplx_mul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def exact_poly(coeffs, z):
    """P(z) = sum_k a_k z^k exactly, returned as a pair of Fractions."""
    zr = (Fr(float(z.real)), Fr(float(z.imag)))
    acc = (Fr(0), Fr(0))
    for a in reversed(list(coeffs)):
        acc = cplx_mul(acc, zr)
        acc = (acc[0] + Fr(float(a.real)), acc[1] + Fr(float(a.imag)))
    return acc


def exact_sum_subset(coeffs, z, ks):
    """sum over k in ks of a_k z^k exactly."""
    zr = (Fr(float(z.real)), Fr(float(z.imag)))
    tot = (Fr(0), Fr(0))
    for k in ks:
        p = (Fr(1), Fr(0))
        for _ in range(k):
            p = cplx_mul(p, zr)
        a = coeffs[k]
        t = cplx_mul((Fr(float(a.real)), Fr(float(a.imag))), p)
        tot = (tot[0] + t[0], tot[1] + t[1])
    return tot


def to_complex(pair, shift: int = 0) -> complex:
    """Fraction pair times 2^shift, rounded to complex (shift keeps it in range)."""
    sc = Fr(2) ** shift if shift >= 0 else Fr(1, 2 ** (-shift))
    return complex(float(pair[0] * sc), float(pair[1] * sc))


def frac_abs_log2(pair) -> float:
    """log2 |pair| (float, for bounds)."""
    re, im = pair
    q = re * re + im * im
    if q == 0:
        return -math.inf
    # log2 of a Fraction without overflow
    return 0.5 * (math.log2(q.numerator) - math.log2(q.denominator))


def concave_majorant(scales: dict[int, int]):
    """Least concave majorant of k -> s_k over [min k, max k], at every integer k.

    Brute force over all pairs of data points: Ehat(k) = max over i <= k <= j of the
    linear interpolation between (i, s_i) and (j, s_j).  Returns {k: Fraction}.
    """
    ks = sorted(scales)
    lo, hi = ks[0], ks[-1]
    out = {}
    for k in range(lo, hi + 1):
        best = None
        for i in ks:
            if i > k:
                break
            for j in ks:
                if j < k:
                    continue
                if i == j:
                    val = Fr(scales[i])
                else:
                    val = Fr(scales[i]) + Fr(scales[j] - scales[i], j - i) * (k - i)
                if best is None or val > best:
                    best = val
        out[k] = best
    return out


def cover_vertices(Ehat: dict[int, Fr]):
    """Corners of a piecewise-linear function sampled at the integers."""
    ks = sorted(Ehat)
    if len(ks) == 1:
        return ks
    verts = [ks[0]]
    for k in ks[1:-1]:
        if Ehat[k] - Ehat[k - 1] != Ehat[k + 1] - Ehat[k]:
            verts.append(k)
    verts.append(ks[-1])
    return verts


def exact_deriv_subset(coeffs, z, ks):
    """sum over k in ks (k >= 1) of k a_k z^(k-1) exactly."""
    zr = (Fr(float(z.real)), Fr(float(z.imag)))
    tot = (Fr(0), Fr(0))
    for k in ks:
        if k == 0:
            continue
        p = (Fr(1), Fr(0))
        for _ in range(k - 1):
            p = cplx_mul(p, zr)
        a = coeffs[k]
        t = cplx_mul((Fr(float(a.real)) * k, Fr(float(a.imag)) * k), p)
        tot = (tot[0] + t[0], tot[1] + t[1])
    return tot
