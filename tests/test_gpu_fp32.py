"""FP32 window sums (FPE_PRECONDITION_FP32, p = 24) on the HIP path against the
oracle at p = 24: max |FPE - oracle| / sum over the window of |a_k||z|^k
<= 2^-18, the bound stated for FP32.  The windows and term counts are those of
the p = 24 plan (the same as an FP64-arithmetic plan at p = 24).  Errors above
FP64 level on most points show that the FP32 path, not the FP64 fallback, ran.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2211_06320_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 2.0 ** -18


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


def check32(fpe, c, z, sample=None, label="", expect_fp32=True):
    plan = fpe.precondition(to_dev(c), 24, fp32=True)
    plan64 = fpe.precondition(to_dev(c), 24)
    zd = to_dev(z)
    m, e, t, w = [x.cpu().numpy() for x in plan.eval(zd, terms=True, window=True)]
    m64, e64, t64, w64 = [x.cpu().numpy() for x in plan64.eval(zd, terms=True, window=True)]
    assert np.array_equal(t, t64) and np.array_equal(w, w64)
    idx = np.arange(len(z)) if sample is None else np.random.default_rng(7).choice(len(z), sample, replace=False)
    ref = oracle.precondition(c, 24).eval(z[idx])
    fin = np.isfinite(z[idx].real) & np.isfinite(z[idx].imag)
    assert np.isnan(m[idx][~fin].real).all()
    err = oracle.scaled_error(m[idx][fin], e[idx][fin], ref["m"][fin], ref["e"][fin], ref["dwin_m"][fin],
                              ref["dwin_e"][fin])
    err64 = oracle.scaled_error(m64[idx][fin], e64[idx][fin], ref["m"][fin], ref["e"][fin], ref["dwin_m"][fin],
                                ref["dwin_e"][fin])
    worst = float(err.max(initial=0.0))
    frac32 = float(np.mean(err > 1e-12))
    say(f"  {label}: FP32 max scaled error {worst:.3e} (FP64 arithmetic {err64.max():.3e}); "
        f"{100 * frac32:.1f} % of points above 1e-12")
    assert worst <= TOL32, (worst, np.log2(worst))
    if expect_fp32:
        assert frac32 > 0.5
    mx = np.maximum(np.abs(m.real), np.abs(m.imag))
    assert (((mx >= 0.5) & (mx < 1.0)) | (mx == 0) | np.isnan(mx)).all()


def test_fp32_flag_validation(fpe):
    c = to_dev(workloads.uniform_coeffs(100, 1))
    with pytest.raises(Exception):
        fpe.precondition(c, 53, fp32=True)      # FP32 window sums need p <= 24
    fpe.precondition(c, 24, fp32=True)
    fpe.precondition(c, 12, fp32=True)


def test_fp32_small_all_points(fpe):
    wl = workloads.workload("uniform_d1000")
    z = np.concatenate([wl.points, [0, np.nan, 1e300 + 1e300j, 1.0, 2.0 ** 20, 2.0 ** -20]])
    check32(fpe, wl.coeffs, z, label="uniform d=1000")


def test_fp32_long_windows(fpe):
    c = workloads.uniform_coeffs(20_000, 21)
    rng = np.random.default_rng(3)
    z = 2.0 ** rng.uniform(-0.02, 0.02, 3000) * np.exp(1j * rng.uniform(0, 2 * np.pi, 3000))
    check32(fpe, c, z, label="near the unit circle d=20000")


def test_fp32_large_points_fall_back(fpe):
    """|z| beyond 2^12: those tiles run in FP64 (errors at FP64 level)."""
    c = workloads.uniform_coeffs(5000, 23)
    rng = np.random.default_rng(4)
    z = 2.0 ** rng.uniform(13, 40, 2000) * np.exp(1j * rng.uniform(0, 2 * np.pi, 2000))
    check32(fpe, c, z, label="|z| > 2^13", expect_fp32=False)


@pytest.mark.parametrize("name", ["wide_d2p20", "sparse_wide_d2p20"])
def test_fp32_wide_dynamic_range(fpe, name):
    wl = workloads.workload(name, n_points=20_000)
    check32(fpe, wl.coeffs, wl.points, sample=1500, label=name, expect_fp32=False)


def test_fp32_full_size_sample(fpe):
    wl = workloads.workload("uniform_d1e6")
    check32(fpe, wl.coeffs, wl.points, sample=400, label="d=1e6 sample")


# ---------------------------------------------------------------- Q' and Newton in FP32
def check32_deriv(fpe, c, z, label, sample=None):
    """FP32 plan: Q and Q' from fpe_eval_deriv against the oracle's (at p = 24,
    the same kept terms), each within 2^-18 of its window scale; Q equal to the
    same plan's fpe_eval up to the FP32 bound."""
    plan = fpe.precondition(to_dev(c), 24, fp32=True)
    zd = to_dev(z)
    m, e, md, ed = [x.cpu().numpy() for x in plan.eval_deriv(zd)]
    idx = np.arange(len(z)) if sample is None else np.random.default_rng(9).choice(len(z), sample, replace=False)
    ref = oracle.precondition(c, 24).eval_deriv(z[idx])
    fin = np.isfinite(z[idx].real) & np.isfinite(z[idx].imag)
    err = oracle.scaled_error(m[idx][fin], e[idx][fin], ref["m"][fin], ref["e"][fin], ref["dwin_m"][fin],
                              ref["dwin_e"][fin])
    none = fin & (ref["ddwin_m"] == 0)
    assert (md[idx][none] == 0).all()
    ok = fin & ~none
    errd = oracle.scaled_error(md[idx][ok], ed[idx][ok], ref["md"][ok], ref["ed"][ok], ref["ddwin_m"][ok],
                               ref["ddwin_e"][ok])
    frac32 = float(np.mean(errd > 1e-12))
    say(f"  {label}: FP32 Q max scaled error {err.max():.3e}, Q' {errd.max():.3e}; "
        f"{100 * frac32:.1f} % of Q' above 1e-12")
    assert err.max() <= TOL32 and errd.max() <= TOL32
    return frac32


def test_fp32_derivative(fpe):
    wl = workloads.workload("uniform_d1000", n_points=3000)
    z = np.concatenate([wl.points, [0, np.nan, 1.0, 2.0 ** -20]])
    assert check32_deriv(fpe, wl.coeffs, z, "uniform d=1000") > 0.5
    c = workloads.uniform_coeffs(20_000, 21)
    rng = np.random.default_rng(31)
    zz = 2.0 ** rng.uniform(-0.02, 0.02, 3000) * np.exp(1j * rng.uniform(0, 2 * np.pi, 3000))
    assert check32_deriv(fpe, c, zz, "near the unit circle d=20000") > 0.5


def test_fp32_derivative_adjoint_workload_sample(fpe):
    """d = 2^18, 2^20 spherical points (the reverse-mode workload) with an FP32
    plan at p = 24: Q and Q' on a seeded sample."""
    wl = workloads.workload("uniform_d2p18")
    check32_deriv(fpe, wl.coeffs, wl.points, "d=2^18, 2^20 points", sample=1500)


def test_fp32_newton_example(fpe):
    """P = z^64 + 1, p = 24, z = 10 (Section 7.2): P(10) = 10^64 + 1 and P'(10)
    are beyond the FP32 range, yet the Newton increment P/P' = 10/64 = 0.15625
    comes out of the FP32 plan (the values carry their binary exponents)."""
    c = np.zeros(65, complex)
    c[0] = 1.0
    c[64] = 1.0
    plan = fpe.precondition(to_dev(c), 24, fp32=True)
    z = to_dev(np.array([10.0 + 0j]))
    zn, m, e, md, ed = plan.newton_step(z)
    torch.cuda.synchronize()
    zn = complex(zn.cpu().numpy()[0])
    say(f"  z^64 + 1 at z = 10, FP32 plan: Newton step to {zn!r} (increment {10 - zn.real!r})")
    assert abs((10.0 - zn.real) - 0.15625) <= 0.15625 * 2.0 ** -20 and zn.imag == 0.0
    q = float(m.cpu().numpy()[0].real) * 2.0 ** int(e.cpu().numpy()[0])
    assert abs(q / 1e64 - 1.0) < 2.0 ** -20          # Q = 10^64 (a_0 is below the window)


# ---------------------------------------------------------------- the compensated FP32 form
def test_fp32_compensated_flags(fpe):
    c = to_dev(workloads.uniform_coeffs(100, 1))
    with pytest.raises(ValueError):
        fpe.precondition(c, 24, compensated=True)     # needs fp32
    fpe.precondition(c, 24, fp32=True, compensated=True)


@pytest.mark.parametrize("case", ["uniform_d1000", "near_circle_d20000", "wide_d2p20", "uniform_d1e6"])
def test_fp32_compensated(fpe, case):
    """FP32 blocks by the compensated recurrence (TwoSum/TwoProd): within 2^-18
    of the oracle at p = 24, at least as accurate as the plain FP32 blocks on
    the same points up to rounding, and computed in FP32 (errors above FP64
    level: the coefficients are FP32)."""
    if case == "uniform_d1000":
        wl = workloads.workload("uniform_d1000")
        c, z, sample = wl.coeffs, np.concatenate([wl.points, [0, np.nan, 1.0]]), None
    elif case == "near_circle_d20000":
        c = workloads.uniform_coeffs(20_000, 21)
        rng = np.random.default_rng(3)
        z = 2.0 ** rng.uniform(-0.02, 0.02, 3000) * np.exp(1j * rng.uniform(0, 2 * np.pi, 3000))
        sample = None
    elif case == "wide_d2p20":
        wl = workloads.workload("wide_d2p20", n_points=20_000)
        c, z, sample = wl.coeffs, wl.points, 1500
    else:
        wl = workloads.workload("uniform_d1e6")
        c, z, sample = wl.coeffs, wl.points, 400
    zd = to_dev(z)
    idx = np.arange(len(z)) if sample is None else np.random.default_rng(7).choice(len(z), sample, replace=False)
    ref = oracle.precondition(c, 24).eval(z[idx])
    fin = np.isfinite(z[idx].real) & np.isfinite(z[idx].imag)
    errs = {}
    for comp in (False, True):
        plan = fpe.precondition(to_dev(c), 24, fp32=True, compensated=comp)
        m, e = [x.cpu().numpy() for x in plan.eval(zd)]
        errs[comp] = oracle.scaled_error(m[idx][fin], e[idx][fin], ref["m"][fin], ref["e"][fin],
                                         ref["dwin_m"][fin], ref["dwin_e"][fin])
    say(f"  {case}: max scaled error plain FP32 blocks {errs[False].max():.3e}, "
        f"compensated {errs[True].max():.3e}")
    assert errs[True].max() <= TOL32
    assert errs[True].max() <= errs[False].max() * 1.01 + 1e-15
