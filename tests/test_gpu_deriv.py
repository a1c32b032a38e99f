"""Derivative through the same window (Q'), and Newton steps, on the HIP path
against the oracle.  Q from fpe_eval_deriv must equal fpe_eval's bit for bit
(each chunk partial is computed the same way whatever the partition); Q' must
satisfy |Q'_gpu - Q'_oracle| <= 2^-44 sum over the window of |k a_k||z|^(k-1)."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2211_06320_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 2.0 ** -44


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


def run(fpe, c, z):
    plan = fpe.precondition(to_dev(c), 53)
    zd = to_dev(z)
    m0, e0 = plan.eval(zd)
    m, e, md, ed = plan.eval_deriv(zd)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (m0, e0, m, e, md, ed)]


def check(fpe, c, z, sample=None, label=""):
    m0, e0, m, e, md, ed = run(fpe, c, z)
    assert np.array_equal(m0.view(np.float64), m.view(np.float64), equal_nan=True) and np.array_equal(e0, e)
    idx = np.arange(len(z)) if sample is None else np.random.default_rng(5).choice(len(z), sample, replace=False)
    ref = oracle.precondition(c, 53).eval_deriv(z[idx])
    finite = np.isfinite(z[idx].real) & np.isfinite(z[idx].imag)
    none = finite & (ref["ddwin_m"] == 0)          # no kept term of degree >= 1
    assert (md[idx][none] == 0).all() and (ed[idx][none] == 0).all()
    ok = finite & ~none
    err = oracle.scaled_error(md[idx][ok], ed[idx][ok], ref["md"][ok], ref["ed"][ok],
                              ref["ddwin_m"][ok], ref["ddwin_e"][ok])
    worst = float(err.max(initial=0.0))
    say(f"  {label}: max scaled error of Q' {worst:.3e} on {ok.sum()} points")
    assert worst <= TOL, (worst, math.log2(max(worst, 1e-300)))
    assert np.isnan(md[idx][~finite]).all()
    mx = np.maximum(np.abs(md.real), np.abs(md.imag))
    assert (((mx >= 0.5) & (mx < 1.0)) | (mx == 0) | np.isnan(mx)).all()


def test_deriv_small_all_points(fpe):
    wl = workloads.workload("uniform_d1000", n_points=3000)
    z = np.concatenate([wl.points, [0, np.nan, 1e-300, 1e300 + 1e300j, 1.0]])
    check(fpe, wl.coeffs, z, label="uniform d=1000")


def test_deriv_long_windows(fpe):
    d = 20_000
    c = workloads.uniform_coeffs(d, 21)
    rng = np.random.default_rng(3)
    z = 2.0 ** rng.uniform(-0.02, 0.02, 3000) * np.exp(1j * rng.uniform(0, 2 * np.pi, 3000))
    check(fpe, c, z, label="near the unit circle d=20000")


def test_deriv_window_starts_across_chunks(fpe):
    d = 60_000
    c = workloads.uniform_coeffs(d, 22)
    rng = np.random.default_rng(8)
    lam = np.concatenate([rng.uniform(0.002, 0.02, 768), -rng.uniform(0.002, 0.02, 768)])
    z = 2.0 ** lam * np.exp(1j * rng.uniform(0, 2 * np.pi, lam.size))
    check(fpe, c, z, label="sparse lambda d=60000")


@pytest.mark.parametrize("kind", ["wide", "sparse_wide"])
def test_deriv_wide_dynamic_range(fpe, kind):
    gen = workloads.wide_coeffs if kind == "wide" else workloads.sparse_wide_coeffs
    c = gen(1 << 16, 31)
    z = workloads.spherical_points(3000, 32)
    check(fpe, c, z, label=kind)


def test_deriv_extreme_scale_range(fpe):
    """Good coefficients over 1700 binary orders (scales on a concave parabola),
    windows across several chunks: the fixed-point shifts of Q and Q' partials
    span the coefficient table's range."""
    d = 20_000
    k = np.arange(d + 1)
    sc = 850 - np.round(1700 * ((2.0 * k / d) - 1) ** 2)
    c = np.exp2(sc - 0.5) * np.exp(1j * 0.37 * k)
    rng = np.random.default_rng(47)
    z = 2.0 ** rng.uniform(-0.2, 0.2, 1500) * np.exp(1j * rng.uniform(0, 2 * np.pi, 1500))
    check(fpe, c, z, label="scale range 1700")


def test_deriv_full_size(fpe):
    wl = workloads.workload("uniform_d1e6")
    check(fpe, wl.coeffs, wl.points, sample=400, label="d=1e6 sample")


def test_deriv_adjoint_workload_sample(fpe):
    """Q and Q' at all 2^20 points of the reverse-mode workload (d = 2^18),
    checked against the oracle on 400 sampled points."""
    wl = workloads.workload("uniform_d2p18")
    check(fpe, wl.coeffs, wl.points, sample=400, label="d=2^18, 2^20 points, sample")


def test_newton_paper_example(fpe):
    """z^64 + 1 at z = 10 (Section 7.2): the kept terms are z^64 alone, the step
    is z/64, so the new point is 9.84375 exactly."""
    c = np.zeros(65, np.complex128)
    c[0] = 1.0
    c[64] = 1.0
    plan = fpe.precondition(to_dev(c), 53)
    zn, m, e, md, ed = plan.newton_step(to_dev(np.array([10.0 + 0j, 0j, np.nan + 0j])))
    zn = zn.cpu().numpy()
    assert zn[0] == 9.84375 + 0j
    assert np.isnan(zn[1].real) and np.isnan(zn[2].real)      # Q' = 0 at 0; NaN input


def test_newton_steps_against_oracle(fpe):
    """z - Q/Q' from the GPU against the same quotient from the oracle's Q and Q'."""
    c = workloads.uniform_coeffs(5000, 41)
    z = workloads.spherical_points(4000, 42)
    plan = fpe.precondition(to_dev(c), 53)
    zn = plan.newton_step(to_dev(z))[0].cpu().numpy()
    ref = oracle.precondition(c, 53).eval_deriv(z)
    ok = ref["ddwin_m"] > 0
    q = (ref["m"][ok] / ref["md"][ok]) * np.exp2((ref["e"][ok] - ref["ed"][ok]).astype(np.float64))
    want = z[ok] - q
    scale = np.abs(z[ok]) + np.abs(q)
    err = np.abs(zn[ok] - want) / scale
    say(f"  newton: max relative difference {err.max():.3e}")
    assert err.max() <= 2.0 ** -40
