"""The seeded generators draw what the paper's workloads describe."""
import math

import numpy as np
from scipy import stats

from paper_2211_06320_amd import workloads


def test_spherical_points_distribution():
    """|z| has CDF r^2/(1+r^2) (density 2r/(1+r^2)^2, Section 5.2); arg is uniform."""
    z = workloads.spherical_points(200_000, 1)
    r = np.abs(z)
    ks = stats.kstest(r ** 2 / (1 + r ** 2), "uniform")
    assert ks.pvalue > 1e-3
    ka = stats.kstest((np.angle(z) + math.pi) / (2 * math.pi), "uniform")
    assert ka.pvalue > 1e-3


def test_seeded_and_reproducible():
    a = workloads.workload("uniform_d1000")
    b = workloads.workload("uniform_d1000")
    assert np.array_equal(a.coeffs, b.coeffs) and np.array_equal(a.points, b.points)
    assert a.coeffs.shape == (1001,) and a.points.shape == (10_000,)
    assert np.abs(a.coeffs.real).max() <= 1 and np.abs(a.coeffs.imag).max() <= 1


def test_wide_and_sparse_families():
    c = workloads.wide_coeffs(1 << 16, 3)
    g = np.log2(np.abs(c))
    assert abs(g.std() - 40) < 1.0 and abs(g.mean()) < 1.0
    s = workloads.sparse_wide_coeffs(1 << 16, 3)
    assert np.count_nonzero(s) == round(0.01 * ((1 << 16) + 1))


def test_batched_workload_shapes():
    cs, ps = workloads.batched_workload(n_poly=64)
    degs = np.array([len(c) - 1 for c in cs])
    cnt = np.array([len(p) for p in ps])
    assert degs.min() >= 16 and degs.max() <= 65536
    assert cnt.min() >= 64 and cnt.max() <= 1024
