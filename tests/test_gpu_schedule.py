"""Tile schedules: every chunk length the tuner may pick gives results within
the tolerance of the oracle (2^-44 of the window scale), on windows that span
several chunks and windows that start mid-chunk; a batch with a chunk length
equals each plan's own evaluation with that length bit for bit; the autotuner
returns a candidate and leaves the plan evaluating correctly."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2211_06320_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 2.0 ** -44
CANDIDATES = (256, 512, 1024, 2048)


@pytest.fixture(scope="module")
def fpe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2211_06320_amd as m
    m.lib()
    return m


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.device("cuda:0"))


def say(msg):
    print(msg, flush=True)


def cases():
    rng = np.random.default_rng(31)
    c1 = workloads.uniform_coeffs(20_000, 21)
    z1 = 2.0 ** rng.uniform(-0.02, 0.02, 2000) * np.exp(1j * rng.uniform(0, 2 * np.pi, 2000))
    c2 = workloads.uniform_coeffs(60_000, 22)
    lam = np.concatenate([rng.uniform(0.002, 0.016, 500), -rng.uniform(0.002, 0.016, 500)])
    z2 = 2.0 ** lam * np.exp(1j * rng.uniform(0, 2 * np.pi, lam.size))
    wl = workloads.workload("uniform_d1000", n_points=3000)
    return [("near circle d=20000", c1, z1), ("sparse lambda d=60000", c2, z2), ("d=1000", wl.coeffs, wl.points)]


@pytest.mark.parametrize("chunk", CANDIDATES)
def test_every_chunk_length_matches_oracle(fpe, chunk):
    for label, c, z in cases():
        plan = fpe.precondition(to_dev(c), 53)
        plan.set_chunk(chunk)
        m, e = [x.cpu().numpy() for x in plan.eval(to_dev(z))]
        ref = oracle.precondition(c, 53).eval(z)
        err = oracle.scaled_error(m, e, ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"])
        say(f"  C={chunk} {label}: max scaled error {err.max():.3e}")
        assert err.max() <= TOL


def test_batch_chunk_lengths_bitwise(fpe):
    coeffs, points = workloads.batched_workload(n_poly=64, d_max=20000)
    plans = [fpe.precondition(to_dev(c), 53) for c in coeffs]
    offs = np.concatenate([[0], np.cumsum([len(z) for z in points])])
    batch = fpe.Batch(plans, offs)
    zall = to_dev(np.concatenate(points))
    for chunk in (256, 2048):
        batch.set_chunk(chunk)
        m, e = [x.cpu().numpy() for x in batch.eval(zall)]
        for i in range(0, 64, 7):
            plans[i].set_chunk(chunk)
            m1, e1 = [x.cpu().numpy() for x in plans[i].eval(to_dev(points[i]))]
            sl = slice(offs[i], offs[i + 1])
            assert np.array_equal(m[sl].view(np.float64), m1.view(np.float64)) and np.array_equal(e[sl], e1)


def test_autotune(fpe):
    label, c, z = cases()[0]
    plan = fpe.precondition(to_dev(c), 53)
    best = plan.autotune(to_dev(z))
    assert best in CANDIDATES
    m, e = [x.cpu().numpy() for x in plan.eval(to_dev(z))]
    ref = oracle.precondition(c, 53).eval(z)
    assert oracle.scaled_error(m, e, ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"]).max() <= TOL
    # an untuned plan of the same bucket takes the cached choice: same results as setting it
    plan2 = fpe.precondition(to_dev(c), 53)
    m2, e2 = [x.cpu().numpy() for x in plan2.eval(to_dev(z))]
    assert np.array_equal(m2.view(np.float64), m.view(np.float64)) and np.array_equal(e2, e)
    coeffs, points = workloads.batched_workload(n_poly=32, d_max=5000)
    b = fpe.Batch([fpe.precondition(to_dev(x), 53) for x in coeffs],
                  np.concatenate([[0], np.cumsum([len(p) for p in points])]))
    assert b.autotune(to_dev(np.concatenate(points))) in CANDIDATES
    say(f"  tuned chunk: plan {best}")


def test_fp32_plans_keep_512(fpe):
    plan = fpe.precondition(to_dev(workloads.uniform_coeffs(1000, 5)), 24, fp32=True)
    with pytest.raises(fpe.FPEError):
        plan.set_chunk(1024)
    plan.set_chunk(512)
    assert plan.autotune(to_dev(workloads.spherical_points(500, 6))) == 512
