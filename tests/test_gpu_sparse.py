"""The sparse form of the window sums (Horner's rule over the list of G_p, gaps
jumped by powers of z; Section 8.2's precomputed powers for lacunary windows)
against the oracle: the same kept terms as the dense form (windows and term
counts are decided before the window sum, so they are equal bit for bit), and
values within 2^-44 of sum |a_k||z|^k of the oracle's reference, for every
chunk length, on workloads whose windows are lacunary (wide dynamic range,
1 % nonzero), dense (every index good: gaps of 1) and at the extremes of the
coefficient scale range; special points and tiny polynomials; bitwise
independence of the partition; the full d = 2^20 wide-range workloads at
p = 53 and p = 24 on a seeded sample."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2211_06320_amd import workloads
from windows import check_windows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 2.0 ** -44
CHUNKS = (256, 512, 1024, 2048)


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


def run(plan, z, mode, chunk=None):
    plan.set_window_mode(mode)
    if chunk is not None:
        plan.set_chunk(chunk)
    assert plan.tile_choice(len(z))[1] == mode
    m, e, t, w = plan.eval(to_dev(z), terms=True, window=True)
    torch.cuda.synchronize()
    return m.cpu().numpy(), e.cpu().numpy(), t.cpu().numpy(), w.cpu().numpy()


def horner_error(m, e, c, z):
    hm, he = oracle.horner(c, z)
    dm, de = oracle.absum(c, z)
    err = oracle.scaled_error(m, e, hm, he, dm, de)
    finite = np.isfinite(z.real) & np.isfinite(z.imag)
    return float(err[finite].max(initial=0.0))


def cases():
    rng = np.random.default_rng(61)
    lam = rng.uniform(-0.05, 0.05, 1500)
    near = 2.0 ** lam * np.exp(1j * rng.uniform(0, 2 * np.pi, lam.size))
    d = 20_000
    k = np.arange(d + 1)
    sc = 850 - np.round(1700 * ((2.0 * k / d) - 1) ** 2)
    extreme = np.exp2(sc - 0.5) * np.exp(1j * 0.37 * k)
    lam2 = rng.uniform(-0.2, 0.2, 1500)
    z_ext = 2.0 ** lam2 * np.exp(1j * rng.uniform(0, 2 * np.pi, lam2.size))
    sph = workloads.spherical_points(3000, 62)
    return [
        ("wide d=2^16", workloads.wide_coeffs(1 << 16, 63), np.concatenate([sph, near])),
        ("sparse wide d=2^16", workloads.sparse_wide_coeffs(1 << 16, 64), np.concatenate([sph, near])),
        ("uniform d=20000 (gaps of 1)", workloads.uniform_coeffs(20_000, 65), np.concatenate([sph[:1000], near])),
        ("scale range 1700 d=20000", extreme, np.concatenate([z_ext, sph[:500]])),
    ]


@pytest.mark.parametrize("chunk", CHUNKS)
def test_sparse_matches_oracle_every_chunk(fpe, chunk):
    for label, c, z in cases():
        for p in (53, 24):
            plan = fpe.precondition(to_dev(c), p)
            m, e, t, w = run(plan, z, "sparse", chunk)
            md, ed, td, wd = run(plan, z, "dense", chunk)
            assert np.array_equal(t, td) and np.array_equal(w, wd)
            P = oracle.precondition(c, p)
            ref = P.eval(z)
            check_windows(P, ref, w, t)
            err = oracle.scaled_error(m, e, ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"])
            worst = float(err.max())
            say(f"  C={chunk} p={p} {label}: sparse max scaled error {worst:.3e} "
                f"(2^{math.log2(max(worst, 1e-300)):.1f}), mean terms {t.mean():.1f}, "
                f"mean window {(w[:, 1] - w[:, 0] + 1).mean():.0f}")
            assert worst <= TOL
            mx = np.maximum(np.abs(m.real), np.abs(m.imag))
            assert (((mx >= 0.5) & (mx < 1.0)) | ((mx == 0) & (e == 0))).all()


def test_sparse_against_full_horner(fpe):
    """Small lacunary polynomials: the sparse sum against compensated Horner of
    the full polynomial (the plain definition of P, within the tolerance)."""
    for label, c, z in cases()[:2]:
        plan = fpe.precondition(to_dev(c), 53)
        m, e, _, _ = run(plan, z[:1500], "sparse", 512)
        worst = horner_error(m, e, c, z[:1500])
        say(f"  {label}: max scaled error vs compensated Horner {worst:.3e}")
        assert worst <= TOL


def test_sparse_special_points_and_tiny_polynomials(fpe):
    c = np.array([3 + 4j, 1, -2j, 0.5], complex)
    z = np.array([0, complex(np.inf, 0), complex(np.nan, 1), 1e-300, 1e300, 0.5 - 0.25j], complex)
    plan = fpe.precondition(to_dev(c), 53)
    m, e, t, w = run(plan, z, "sparse")
    assert m[0] == (3 + 4j) / 8 and e[0] == 3 and t[0] == 1
    assert np.isnan(m[1:3].real).all() and (t[1:3] == 0).all()
    assert horner_error(m[3:], e[3:], c, z[3:]) <= TOL
    zz = np.concatenate([[0], workloads.spherical_points(700, 66)])
    for cc in (np.concatenate([[0, 0], workloads.wide_coeffs(300, 67), [0, 0]]),
               np.array([0, 0, 0, 2 - 1j], complex), np.array([3 - 1j], complex),
               np.array([1] + [0] * 999 + [1], complex),          # z^1000 + 1: one gap of 1000
               np.array([2.0 ** 40] + [0] * 4000 + [1, 0, 0, 1e-30], complex)):
        plan = fpe.precondition(to_dev(cc), 53)
        m, e, t, w = run(plan, zz, "sparse", 2048)
        P = oracle.precondition(cc, 53)
        check_windows(P, P.eval(zz), w, t)
        worst = horner_error(m, e, cc, zz)
        say(f"  d={len(cc) - 1}: max scaled error {worst:.3e}")
        assert worst <= TOL
    # the all-zero polynomial
    plan = fpe.precondition(to_dev(np.zeros(9, complex)), 53)
    m, e, t, _ = run(plan, zz, "sparse")
    assert (m == 0).all() and (e == 0).all() and (t == 0).all()


def test_sparse_bitwise_independent_of_partition(fpe):
    c = workloads.wide_coeffs(1 << 17, 68)
    z = workloads.spherical_points(30_000, 69)
    plan = fpe.precondition(to_dev(c), 53)
    plan.set_window_mode("sparse")
    zd = to_dev(z)
    m1, e1 = plan.eval(zd)
    m2, e2 = plan.eval(zd)
    perm = torch.randperm(len(z), device=zd.device)
    m3, e3 = plan.eval(zd[perm].contiguous())
    m4, e4 = plan.eval(zd[:20_000].contiguous())          # other groups, another partition
    torch.cuda.synchronize()
    inv = torch.argsort(perm)
    assert torch.equal(m1, m2) and torch.equal(e1, e2)
    assert torch.equal(m3[inv], m1) and torch.equal(e3[inv], e1)
    assert torch.equal(m4, m1[:20_000]) and torch.equal(e4, e1[:20_000])


def test_fp32_plans_refuse_sparse(fpe):
    plan = fpe.precondition(to_dev(workloads.wide_coeffs(5000, 70)), 24, fp32=True)
    with pytest.raises(fpe.FPEError) as ei:
        plan.set_window_mode("sparse")
    assert ei.value.status == 6
    assert plan.tile_choice(1000)[1] == "dense"


def test_autotune_chooses_a_form(fpe):
    wl = workloads.workload("sparse_wide_d2p20", n_points=200_000)
    plan = fpe.precondition(to_dev(wl.coeffs), 53)
    z = to_dev(wl.points)
    chunk = plan.autotune(z)
    c2, mode = plan.tile_choice(len(wl.points))
    say(f"  autotune sparse_wide d=2^20, 2e5 points: chunk {chunk}, {mode}")
    assert chunk == c2 and chunk in CHUNKS and mode in ("dense", "sparse")
    m, e = plan.eval(z)
    torch.cuda.synchronize()
    idx = np.random.default_rng(71).choice(len(wl.points), 2000, replace=False)
    ref = oracle.precondition(wl.coeffs, 53).eval(wl.points[idx])
    err = oracle.scaled_error(m.cpu().numpy()[idx], e.cpu().numpy()[idx], ref["m"], ref["e"], ref["dwin_m"],
                              ref["dwin_e"])
    assert err.max() <= TOL


@pytest.mark.parametrize("name", ["wide_d2p20", "sparse_wide_d2p20"])
@pytest.mark.parametrize("p", [53, 24])
def test_sparse_full_size(fpe, name, p):
    """d = 2^20, 10^6 spherical points, the sparse form at the default chunk:
    every point's window and term count equal to the dense form's; values on a
    seeded sample (with the longest windows) against the oracle's window sum at
    the same p (the same kept terms: the error of the summation alone)."""
    wl = workloads.workload(name)
    say(f"sparse {name} p={p} n={len(wl.points)}")
    plan = fpe.precondition(to_dev(wl.coeffs), p)
    m, e, t, w = run(plan, wl.points, "sparse", 0)
    _, _, td, wd = run(plan, wl.points, "dense", 0)
    assert np.array_equal(t, td) and np.array_equal(w, wd)
    rng = np.random.default_rng(3100 + p)
    idx = np.unique(np.concatenate([rng.choice(len(wl.points), 20000, replace=False),
                                    np.argsort(w[:, 0] - w[:, 1])[:50]]))
    ref = oracle.precondition(wl.coeffs, p).eval(wl.points[idx])
    err = oracle.scaled_error(m[idx], e[idx], ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"])
    say(f"  max scaled error on {len(idx)} points {err.max():.3e}; mean terms {t.mean():.1f}, "
        f"mean window {(w[:, 1] - w[:, 0] + 1).mean():.0f}")
    assert err.max() <= TOL
