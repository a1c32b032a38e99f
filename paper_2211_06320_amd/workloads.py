"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This module only draws random numbers; it holds none of the evaluation method's
arithmetic (no scale, hull, window or sum).  Both sides of every parity check read
the arrays produced here.

Point sets follow the measure the paper averages over (Section 5.2, the uniform
measure on the Riemann sphere, whose radial density is 2r dr / (1 + r^2)^2): a
uniform point on the unit sphere is projected stereographically onto C.  The
paper's own 10 084 "-sphere" points (Section 8.3) are not available; seeded
points with the same distribution stand in for them.

Coefficient families:
  * uniform: Re, Im i.i.d. uniform on [-1, 1] (the configurations at d = 1000,
    d = 10^6, the batched set and the adjoint set);
  * wide: |a_k| = 2^{g_k}, g_k ~ N(0, 40^2), argument uniform on [0, 2 pi);
  * sparse-wide: the wide family with only round(0.01 (d + 1)) nonzero
    coefficients at random positions.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 221106320


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def spherical_points(n: int, seed: int) -> np.ndarray:
    """n points uniform on the Riemann sphere, projected to C (complex128)."""
    rng = _rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # stereographic projection from the north pole; v_z == 1 has probability 0
    den = 1.0 - v[:, 2]
    den[den == 0.0] = np.finfo(np.float64).tiny
    return ((v[:, 0] + 1j * v[:, 1]) / den).astype(np.complex128)


def uniform_coeffs(d: int, seed: int) -> np.ndarray:
    """a_0..a_d with Re, Im i.i.d. uniform on [-1, 1] (complex128, a_0 first)."""
    rng = _rng(seed)
    re = rng.uniform(-1.0, 1.0, d + 1)
    im = rng.uniform(-1.0, 1.0, d + 1)
    return (re + 1j * im).astype(np.complex128)


def wide_coeffs(d: int, seed: int, sigma: float = 40.0) -> np.ndarray:
    """|a_k| = 2^{g_k}, g_k ~ N(0, sigma^2), argument uniform on [0, 2 pi)."""
    rng = _rng(seed)
    g = rng.normal(0.0, sigma, d + 1)
    th = rng.uniform(0.0, 2.0 * math.pi, d + 1)
    return (np.exp2(g) * np.exp(1j * th)).astype(np.complex128)


def sparse_wide_coeffs(d: int, seed: int, frac: float = 0.01, sigma: float = 40.0) -> np.ndarray:
    """The wide family with round(frac (d + 1)) nonzero coefficients at random positions."""
    rng = _rng(seed)
    dense = wide_coeffs(d, seed + 7, sigma)
    keep = int(round(frac * (d + 1)))
    pos = rng.choice(d + 1, size=keep, replace=False)
    out = np.zeros(d + 1, np.complex128)
    out[pos] = dense[pos]
    return out


@dataclass
class Workload:
    """One polynomial and one point set, with the seeds that produced them."""
    name: str
    coeffs: np.ndarray
    points: np.ndarray
    p_bits: int = 53
    meta: dict = field(default_factory=dict)

    @property
    def degree(self) -> int:
        return int(self.coeffs.shape[0]) - 1


def workload(name: str, *, n_points: int | None = None, degree: int | None = None) -> Workload:
    """Named workloads; n_points / degree override the sizes (the distributions stay).

    uniform_d1000      d = 1000,  10^4 spherical points (the small parity case)
    uniform_d1e6       d = 10^6,  10^6 spherical points (the headline throughput case)
    wide_d2p20         d = 2^20,  10^6 points, wide coefficients
    sparse_wide_d2p20  d = 2^20,  10^6 points, 1 % nonzero wide coefficients
    uniform_d2p18      d = 2^18,  2^20 points (the adjoint case)
    """
    table = {
        "uniform_d1000": (1, 1000, 10_000, uniform_coeffs),
        "uniform_d1e6": (2, 1_000_000, 1_000_000, uniform_coeffs),
        "wide_d2p20": (3, 1 << 20, 1_000_000, wide_coeffs),
        "sparse_wide_d2p20": (3, 1 << 20, 1_000_000, sparse_wide_coeffs),
        "uniform_d2p18": (5, 1 << 18, 1 << 20, uniform_coeffs),
    }
    if name not in table:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(table)}")
    cfg, d, n, gen = table[name]
    d = degree if degree is not None else d
    n = n_points if n_points is not None else n
    coeffs = gen(d, SEED_BASE + cfg)
    points = spherical_points(n, SEED_BASE + 100 + cfg)
    return Workload(name, coeffs, points, 53, {"cfg": cfg, "d": d, "n": n})


def batched_workload(n_poly: int = 4096, seed: int = SEED_BASE + 4,
                     d_min: int = 16, d_max: int = 65536,
                     m_min: int = 64, m_max: int = 1024):
    """Many independent polynomials of uneven degree, each with its own point set.

    Degrees are log-uniform on [d_min, d_max]; each polynomial gets a uniform random
    number of spherical points in [m_min, m_max].  Returns (list of coefficient
    arrays, list of point arrays).
    """
    rng = _rng(seed)
    degs = np.floor(np.exp(rng.uniform(math.log(d_min), math.log(d_max), n_poly))).astype(np.int64)
    counts = rng.integers(m_min, m_max + 1, n_poly)
    coeffs, points = [], []
    for i in range(n_poly):
        coeffs.append(uniform_coeffs(int(degs[i]), seed * 7919 + i))
        points.append(spherical_points(int(counts[i]), seed * 104729 + i))
    return coeffs, points
