"""Reverse mode (fpe_eval_adjoint) on the HIP path against the oracle, and the
autograd wrapper against central finite differences.

Tolerance of grad_a[k], relative to its scale S[k] = sum |g_j| |z_j|^k over the
same terms, derived from the kernel's arithmetic (u = 2^-53): the start power
z^lo is within 24 u normwise (chained chunk powers), the product with g adds
2 u, each of the at most C - 1 = 511 further products by conj(z) adds 2 u
(complex product with FMA); the terms are then summed exactly in fixed point
(each rounded to far below u of the largest term) and the sum rounded once:
u (2 C + 42).  grad_z is g times conj(Q'), Q' within 2^-44 of its scale:
2^-43 |g| sum |k a_k||z|^(k-1).  The exact sums make grad_a independent of
the order of the points and of the tiles: tests compare it bit for bit.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2211_06320_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53
CHUNK = 512


def tol_grad_a(chunk: int = CHUNK) -> float:
    return U * (2 * chunk + 42)


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


def scaled_g(c, z, seed, limit=1000):
    """Upstream gradients whose terms g_j conj(z_j)^k stay within the double
    range: g_j = (random) 2^-s_j with s_j the largest lambda_j k of the point's
    window; 0 where that needs |s_j| > limit."""
    rng = np.random.default_rng(seed)
    r = oracle.precondition(c, 53).eval(z)
    with np.errstate(divide="ignore", invalid="ignore"):
        lam = np.log2(np.abs(z))
        s = np.where(r["l"] <= r["r"], np.maximum(lam * r["l"], lam * r["r"]), 0.0)
    s = np.where(np.isfinite(s), np.ceil(s), 0.0)
    g = (rng.normal(size=len(z)) + 1j * rng.normal(size=len(z))) * np.exp2(-np.clip(s, -limit, limit))
    g[np.abs(s) > limit] = 0
    return g


def xval(m, e):
    e = np.clip(np.asarray(e, np.int64), -3000, 3000)
    with np.errstate(over="ignore"):
        return np.ldexp(np.asarray(m).real, e) + 1j * np.ldexp(np.asarray(m).imag, e)


def check(fpe, c, z, g, label, chunk=CHUNK):
    plan = fpe.precondition(to_dev(c), 53)
    plan.set_chunk(chunk)
    ga, gz = plan.adjoint(to_dev(z), to_dev(g))
    torch.cuda.synchronize()
    ga, gz = ga.cpu().numpy(), gz.cpu().numpy()
    ref = oracle.precondition(c, 53).adjoint(z, g)
    S = np.ldexp(ref["ga_scale_m"], np.clip(ref["ga_scale_e"], -3000, 3000))
    want = xval(ref["ga_m"], ref["ga_e"])
    zero = S == 0
    assert (ga[zero] == 0).all()
    ok = (S >= 2.0 ** -1000) & (S <= 2.0 ** 1000)
    err = np.abs(ga[ok] - want[ok]) / S[ok]
    tol = tol_grad_a(chunk)
    worst = float(err.max(initial=0.0))
    say(f"  {label}: grad_a max scaled error {worst:.3e} (tol {tol:.3e}) on {ok.sum()} coefficients")
    assert worst <= tol, (worst, math.log2(max(worst, 1e-300)))
    # grad_z
    fin = np.isfinite(z.real) & np.isfinite(z.imag)
    assert np.isnan(gz[~fin].real).all()
    gs = ref["gz_scale_m"][fin]
    zs = gs == 0
    assert (gz[fin][zs] == 0).all()
    errz = oracle.scaled_error(gz[fin][~zs], np.zeros((~zs).sum(), np.int64), ref["gz_m"][fin][~zs],
                               ref["gz_e"][fin][~zs], gs[~zs], ref["gz_scale_e"][fin][~zs])
    wz = float(errz.max(initial=0.0))
    say(f"  {label}: grad_z max scaled error {wz:.3e} on {(~zs).sum()} points")
    assert wz <= 2.0 ** -43
    return ga, gz


def test_adjoint_small(fpe):
    wl = workloads.workload("uniform_d1000", n_points=1500)
    rng = np.random.default_rng(61)
    lam = rng.uniform(-0.5, 0.9, 1500)
    near = 2.0 ** lam * np.exp(1j * rng.uniform(0, 2 * np.pi, 1500))
    z = np.concatenate([wl.points, near, [0, np.nan, 1e300 + 1e300j, 1.0, -1j]])
    g = scaled_g(wl.coeffs, z, 62)
    g[-5:] = [1 + 2j, 1, 0, 0.5, 0.25j]
    check(fpe, wl.coeffs, z, g, "uniform d=1000")


@pytest.mark.parametrize("chunk", [1024, 2048])
def test_adjoint_chunk_lengths_w_half(fpe, chunk):
    """Long chunks on points with max(|Re z|, |Im z|) just above 1, where the
    unit-scale mantissa w = z / 2 has |w| near 1/2: over a chunk of 2048 the
    term mantissa g conj(w)^k would fall by 2^-2048 without its folds into
    the exponent; for |z| > 1 those are the largest terms of grad_a."""
    d = 20_000
    c = workloads.uniform_coeffs(d, 23)
    rng = np.random.default_rng(67)
    th = rng.uniform(-0.05, 0.05, 2000) + rng.integers(0, 4, 2000) * (np.pi / 2)
    z = 2.0 ** rng.uniform(0.002, 0.004, 2000) * np.exp(1j * th)
    z = z[np.maximum(np.abs(z.real), np.abs(z.imag)) >= 1.0]
    r = oracle.precondition(c, 53).eval(z)
    assert ((r["r"] - r["l"]) >= chunk).sum() > 100
    check(fpe, c, z, scaled_g(c, z, 68), f"|z| just above 1, chunk {chunk}", chunk=chunk)


def test_adjoint_long_windows(fpe):
    d = 20_000
    c = workloads.uniform_coeffs(d, 21)
    rng = np.random.default_rng(63)
    z = 2.0 ** rng.uniform(-0.02, 0.02, 3000) * np.exp(1j * rng.uniform(0, 2 * np.pi, 3000))
    check(fpe, c, z, scaled_g(c, z, 64), "near the unit circle d=20000")


def test_adjoint_window_starts_across_chunks(fpe):
    d = 60_000
    c = workloads.uniform_coeffs(d, 22)
    rng = np.random.default_rng(8)
    lam = np.concatenate([rng.uniform(0.002, 0.016, 768), -rng.uniform(0.002, 0.016, 768)])
    z = 2.0 ** lam * np.exp(1j * rng.uniform(0, 2 * np.pi, lam.size))
    check(fpe, c, z, scaled_g(c, z, 65), "sparse lambda d=60000")


@pytest.mark.parametrize("kind", ["wide", "sparse_wide"])
def test_adjoint_wide_dynamic_range(fpe, kind):
    gen = workloads.wide_coeffs if kind == "wide" else workloads.sparse_wide_coeffs
    c = gen(1 << 16, 31)
    z = workloads.spherical_points(3000, 32)
    check(fpe, c, z, scaled_g(c, z, 66), kind)


def test_adjoint_extreme_scale_range(fpe):
    """Good coefficients over 1700 binary orders, windows across several chunks."""
    d = 20_000
    k = np.arange(d + 1)
    c = np.exp2(850 - np.round(1700 * ((2.0 * k / d) - 1) ** 2) - 0.5) * np.exp(1j * 0.37 * k)
    rng = np.random.default_rng(67)
    z = 2.0 ** rng.uniform(-0.2, 0.2, 1500) * np.exp(1j * rng.uniform(0, 2 * np.pi, 1500))
    check(fpe, c, z, scaled_g(c, z, 68), "scale range 1700")


def test_adjoint_full_size_sample(fpe):
    """d = 10^6 and its 10^6 points, in the launch configuration of the
    benchmark; g is nonzero on 96 sampled points (every other point adds exact
    zeros), so the oracle sums those points alone."""
    wl = workloads.workload("uniform_d1e6")
    rng = np.random.default_rng(67)
    lam = np.log2(np.abs(wl.points))
    inside = np.flatnonzero(lam < -0.01)
    near = np.flatnonzero((np.abs(lam) > 2e-4) & (np.abs(lam) < 1e-3))
    idx = np.concatenate([rng.choice(inside, 64, replace=False), rng.choice(near, 32, replace=False)])
    gs = scaled_g(wl.coeffs, wl.points[idx], 68)
    assert (gs != 0).all()
    g = np.zeros(len(wl.points), np.complex128)
    g[idx] = gs
    plan = fpe.precondition(to_dev(wl.coeffs), 53)
    ga, gz = plan.adjoint(to_dev(wl.points), to_dev(g))
    torch.cuda.synchronize()
    ga, gz = ga.cpu().numpy(), gz.cpu().numpy()
    ref = oracle.precondition(wl.coeffs, 53).adjoint(wl.points[idx], gs)
    S = np.ldexp(ref["ga_scale_m"], np.clip(ref["ga_scale_e"], -3000, 3000))
    want = xval(ref["ga_m"], ref["ga_e"])
    assert (ga[S == 0] == 0).all()
    ok = (S >= 2.0 ** -1000) & (S <= 2.0 ** 1000)
    err = np.abs(ga[ok] - want[ok]) / S[ok]
    say(f"  d=1e6: grad_a max scaled error {err.max():.3e} on {ok.sum()} coefficients")
    assert err.max() <= tol_grad_a()
    assert (gz[np.setdiff1d(np.arange(len(g)), idx)] == 0).all()


def test_adjoint_edge_cases(fpe):
    c = workloads.uniform_coeffs(300, 71)
    plan = fpe.precondition(to_dev(c), 53)
    # no points: grad_a is cleared
    ga, gz = plan.adjoint(to_dev(np.zeros(0, np.complex128)), to_dev(np.zeros(0, np.complex128)))
    assert (ga.cpu().numpy() == 0).all() and gz.numel() == 0
    # one side only, and agreement with the two-sided call
    z = workloads.spherical_points(500, 72)
    g = scaled_g(c, z, 73)
    ga2, gz2 = plan.adjoint(to_dev(z), to_dev(g))
    ga1, none = plan.adjoint(to_dev(z), to_dev(g), grad_z=False)
    none2, gz1 = plan.adjoint(to_dev(z), to_dev(g), grad_a=False)
    assert none is None and none2 is None
    assert np.array_equal(gz1.cpu().numpy(), gz2.cpu().numpy())
    assert np.array_equal(ga1.cpu().numpy(), ga2.cpu().numpy())
    # z = 0 contributes g to grad_a[0]; a_0 = 0 keeps nothing at 0
    ga0, gz0 = plan.adjoint(to_dev(np.zeros(3, np.complex128)), to_dev(np.array([1 + 1j, 2.0, -0.5j])))
    ga0 = ga0.cpu().numpy()
    assert ga0[0] == (1 + 1j) + 2.0 - 0.5j and (ga0[1:] == 0).all() and (gz0.cpu().numpy() == 0).all()
    c2 = c.copy()
    c2[0] = 0
    plan2 = fpe.precondition(to_dev(c2), 53)
    ga0, _ = plan2.adjoint(to_dev(np.zeros(2, np.complex128)), to_dev(np.array([1.0, 1.0 + 0j])))
    assert (ga0.cpu().numpy() == 0).all()
    # P == 0
    plan3 = fpe.precondition(to_dev(np.zeros(10, np.complex128)), 53)
    ga3, gz3 = plan3.adjoint(to_dev(z[:50]), to_dev(g[:50]))
    assert (ga3.cpu().numpy() == 0).all() and (gz3.cpu().numpy() == 0).all()
    # mismatched lengths are rejected
    with pytest.raises(Exception):
        plan.adjoint(to_dev(z), to_dev(g[:10]))


def test_autograd_gradcheck(fpe):
    """torch.autograd.gradcheck of the differentiable evaluation (both inputs
    complex) where the window keeps every term (d = 24, |z| near 1)."""
    rng = np.random.default_rng(81)
    c = to_dev(workloads.uniform_coeffs(24, 82)).requires_grad_(True)
    z = to_dev(2.0 ** rng.uniform(-0.05, 0.05, 6) * np.exp(1j * rng.uniform(0, 2 * np.pi, 6))).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, x: fpe.fpe_eval(a, x), (c, z), eps=1e-6, atol=1e-7, rtol=1e-5,
                                    nondet_tol=1e-12)


def test_autograd_central_differences_restricted_windows(fpe):
    """Windows that drop terms (d = 400, |lambda| up to 1/2): the loss
    L = Re sum_j conj(c_j) Q_j, backpropagated, against central differences of
    the GPU evaluation in Re and Im of kept coefficients (hull and G_p
    unchanged by the step, so Q is linear in them) and of the points (windows
    unchanged by the step)."""
    d = 400
    a = workloads.uniform_coeffs(d, 83)
    rng = np.random.default_rng(84)
    lam = rng.uniform(-0.5, 0.5, 24)
    zs = 2.0 ** lam * np.exp(1j * rng.uniform(0, 2 * np.pi, 24))
    r0 = oracle.precondition(a, 53).eval(zs)
    cw = (rng.normal(size=24) + 1j * rng.normal(size=24)) * np.exp2(-r0["e"].astype(float))

    def loss_np(av, zv):
        q = fpe.fpe_eval(to_dev(av), to_dev(zv)).cpu().numpy()
        return float(np.sum((np.conj(cw) * q).real))

    at = to_dev(a).requires_grad_(True)
    zt = to_dev(zs).requires_grad_(True)
    L = (torch.conj(to_dev(cw)) * fpe.fpe_eval(at, zt)).real.sum()
    L.backward()
    ga, gz = at.grad.cpu().numpy(), zt.grad.cpu().numpy()
    plan = fpe.precondition(to_dev(a), 53)
    hk, hs, good = plan.export()
    kept = np.flatnonzero(np.abs(ga) > 0)
    assert len(kept) > 50
    top = kept[np.argsort(-np.abs(ga[kept]))[:100]]
    assert not np.any(ga[~good])
    checked = 0
    for k in rng.choice(top, 12, replace=False):
        h = 2.0 ** -12 * abs(a[k])
        vals = []
        for step in (h, -h, 1j * h, -1j * h):
            ap = a.copy()
            ap[k] += step
            p2 = fpe.precondition(to_dev(ap), 53)
            hk2, hs2, good2 = p2.export()
            if not (np.array_equal(good2, good) and np.array_equal(hk2, hk) and np.array_equal(hs2, hs)):
                break
            vals.append(loss_np(ap, zs))
        if len(vals) < 4:
            continue
        fd = (vals[0] - vals[1]) / (2 * h) + 1j * (vals[2] - vals[3]) / (2 * h)
        assert abs(fd - ga[k]) <= 1e-9 * abs(ga[k]) + 1e-12 / h, (k, fd, ga[k])
        checked += 1
    assert checked >= 8
    _, _, _, win0 = plan.eval(to_dev(zs), window=True)
    win0 = win0.cpu().numpy()
    checked = 0
    for j in range(24):
        h = 1e-7 * abs(zs[j])
        vals, same = [], True
        for step in (h, -h, 1j * h, -1j * h):
            zp = zs.copy()
            zp[j] += step
            _, _, _, wp = plan.eval(to_dev(zp), window=True)
            same &= bool(np.array_equal(wp.cpu().numpy()[j], win0[j]))
            vals.append(loss_np(a, zp))
        if not same:
            continue
        fd = (vals[0] - vals[1]) / (2 * h) + 1j * (vals[2] - vals[3]) / (2 * h)
        assert abs(fd - gz[j]) <= 1e-6 * abs(gz[j]) + 1e-8 / abs(zs[j]), (j, fd, gz[j])
        checked += 1
    assert checked >= 16


# ---------------------------------------------------------------- normalised values through autograd
def test_adjoint_exponent_scaled_gradients(fpe):
    """g_exp: the reverse mode with upstream gradients g 2^-g_exp equals the one
    with the scaled gradients passed directly (where those are representable),
    to rounding."""
    c = workloads.uniform_coeffs(3000, 91)
    z = workloads.spherical_points(2000, 92)
    plan = fpe.precondition(to_dev(c), 53)
    zd = to_dev(z)
    m, e, md, ed = plan.eval_deriv(zd)
    ok = (e.abs() < 900)
    g = (2.0 * m)[ok].contiguous()
    ga1, gz1 = plan.adjoint(zd[ok].contiguous(), g, md[ok].contiguous(), ed[ok].contiguous(), g_exp=e[ok].contiguous())
    gs = g * torch.pow(2.0, -e[ok].to(torch.float64))
    ga2, gz2 = plan.adjoint(zd[ok].contiguous(), gs.contiguous(), md[ok].contiguous(), ed[ok].contiguous())
    torch.cuda.synchronize()
    sa = ga2.abs().max().item()
    assert (ga1 - ga2).abs().max().item() <= 1e-12 * sa
    assert ((gz1 - gz2).abs() <= 1e-12 * gz2.abs() + 1e-300).all()


def test_autograd_normalised_values_adjoint_workload(fpe):
    """d = 2^18 (the reverse-mode workload's polynomial), a seeded sample of its
    2^20 spherical points, many with |Q| beyond the double range: the loss
    L = sum_j |q_j|^2 on the normalised values Q_j = q_j 2^(e_j) (e constant)
    backpropagates through eval_scaled to finite gradients, which agree with
    central differences of the GPU evaluation in Re and Im of kept
    coefficients (G_p and the cover unchanged by the step) and of points (their
    windows unchanged)."""
    wl = workloads.workload("uniform_d2p18")
    rng = np.random.default_rng(93)
    idx = rng.choice(len(wl.points), 2048, replace=False)
    zs = wl.points[idx]
    a = wl.coeffs
    plan = fpe.precondition(to_dev(a), 53)
    at = to_dev(a).requires_grad_(True)
    zt = to_dev(zs).requires_grad_(True)
    q, e = fpe.eval_scaled(plan, at, zt)
    e0 = e.cpu().numpy()
    say(f"  {int((np.abs(e0) > 1023).sum())} of {len(zs)} points have |Q| beyond the double range")
    assert (np.abs(e0) > 1023).sum() > 100
    L = (q.real ** 2 + q.imag ** 2).sum()
    L.backward()
    ga, gz = at.grad.cpu().numpy(), zt.grad.cpu().numpy()
    assert np.isfinite(ga).all() and np.isfinite(gz).all()

    def loss_np(av, zv, pl=None):
        pl = pl or fpe.precondition(to_dev(av), 53)
        m, ee = pl.eval(to_dev(zv))
        m, ee = m.cpu().numpy(), ee.cpu().numpy()
        return float(np.sum(np.abs(m) ** 2 * np.exp2(2.0 * (ee - e0))))

    hk, hs, good = plan.export()
    kept = np.flatnonzero(np.abs(ga) > 0)
    top = kept[np.argsort(-np.abs(ga[kept]))[:200]]
    checked = 0
    for k in rng.choice(top, 10, replace=False):
        h = 2.0 ** -12 * abs(a[k])
        vals = []
        for step in (h, -h, 1j * h, -1j * h):
            ap = a.copy()
            ap[k] += step
            p2 = fpe.precondition(to_dev(ap), 53)
            hk2, hs2, good2 = p2.export()
            if not (np.array_equal(good2, good) and np.array_equal(hk2, hk) and np.array_equal(hs2, hs)):
                break
            vals.append(loss_np(ap, zs, p2))
        if len(vals) < 4:
            continue
        fd = (vals[0] - vals[1]) / (2 * h) + 1j * (vals[2] - vals[3]) / (2 * h)
        assert abs(fd - ga[k]) <= 1e-7 * abs(ga[k]) + 1e-9 / h, (k, fd, ga[k])
        checked += 1
    assert checked >= 6
    # point gradients by central differences of the one point's term
    # L_j = |Q_j|^2 2^(-2 e_j) (the other terms do not move).  The step is
    # h = t |z| / r with t = 1e-5 for the window [l, r]: truncation ~ t^2 / 6
    # and rounding ~ eps / t relative to the derivative scale
    # B_j = 2 |q_j| 2^(-e_j) (sum |k a_k| |z|^(k-1) + r sum |a_k| |z|^k / |z|)
    qn = q.detach().cpu().numpy()
    sample = rng.choice(len(zs), 24, replace=False)
    ref = oracle.precondition(a, 53).eval_deriv(zs[sample])
    checked, sharp = 0, 0
    for i, j in enumerate(sample):
        _, _, _, w0 = plan.eval(to_dev(zs[j:j + 1]), window=True)
        w0 = w0.cpu().numpy()[0]
        if w0[1] < w0[0]:
            continue
        r = max(int(w0[1]), 1)
        h = 1e-5 * abs(zs[j]) / r
        vals, same = [], True
        for step in (h, -h, 1j * h, -1j * h):
            m, ee, _, wp = plan.eval(to_dev(np.array([zs[j] + step])), window=True)
            same &= bool(np.array_equal(wp.cpu().numpy()[0], w0))
            vals.append(float(abs(m.cpu().numpy()[0]) ** 2 * np.exp2(2.0 * (float(ee.cpu().numpy()[0]) - e0[j]))))
        if not same:
            continue
        fd = (vals[0] - vals[1]) / (2 * h) + 1j * (vals[2] - vals[3]) / (2 * h)
        dscale = ref["ddwin_m"][i] * np.exp2(float(ref["ddwin_e"][i] - e0[j]))
        vscale = r * ref["dwin_m"][i] * np.exp2(float(ref["dwin_e"][i] - e0[j])) / abs(zs[j])
        bound = 2.0 * abs(qn[j]) * (dscale + vscale)
        assert abs(fd - gz[j]) <= 1e-6 * bound, (j, fd, gz[j], bound)
        checked += 1
        sharp += abs(gz[j]) >= 1e-2 * bound
    assert checked >= 16 and sharp >= 8, (checked, sharp)
    say(f"  checked {checked} points by central differences")


def test_autograd_normalised_values_full_size(fpe):
    """All 2^20 points of the reverse-mode workload through eval_scaled and
    backward: finite gradients, bit for bit those of the direct reverse-mode
    call with g = 2 q, g_exp = e."""
    wl = workloads.workload("uniform_d2p18")
    plan = fpe.precondition(to_dev(wl.coeffs), 53)
    at = to_dev(wl.coeffs).requires_grad_(True)
    zt = to_dev(wl.points).requires_grad_(True)
    q, e = fpe.eval_scaled(plan, at, zt)
    (q.real ** 2 + q.imag ** 2).sum().backward()
    ga, gz = at.grad, zt.grad
    m, e2, md, ed = plan.eval_deriv(to_dev(wl.points))
    ga2, gz2 = plan.adjoint(to_dev(wl.points), 2.0 * m, md, ed, g_exp=e2)
    torch.cuda.synchronize()
    assert torch.isfinite(ga).all() and torch.isfinite(gz).all()
    assert torch.equal(ga, ga2)
    assert torch.equal(gz, gz2)


def test_adjoint_exact_sums_bitwise(fpe):
    """grad_a is an exact sum of fixed-point terms: the same bits on a second
    call and with the points (and their g) in another order, which changes
    which points share a wavefront; and within tolerance of the oracle.  2^16
    points of the reverse-mode workload."""
    wl = workloads.workload("uniform_d2p18", n_points=1 << 16)
    rng = np.random.default_rng(101)
    g = scaled_g(wl.coeffs, wl.points, 102)
    plan = fpe.precondition(to_dev(wl.coeffs), 53)
    ga1, _ = plan.adjoint(to_dev(wl.points), to_dev(g), grad_z=False)
    ga2, _ = plan.adjoint(to_dev(wl.points), to_dev(g), grad_z=False)
    perm = rng.permutation(len(g))
    ga3, _ = plan.adjoint(to_dev(wl.points[perm]), to_dev(g[perm]), grad_z=False)
    torch.cuda.synchronize()
    a1, a2, a3 = ga1.cpu().numpy(), ga2.cpu().numpy(), ga3.cpu().numpy()
    assert np.array_equal(a1.view(np.uint64), a2.view(np.uint64))
    assert np.array_equal(a1.view(np.uint64), a3.view(np.uint64))
    ref = oracle.precondition(wl.coeffs, 53).adjoint(wl.points, g)
    S = np.ldexp(ref["ga_scale_m"], np.clip(ref["ga_scale_e"], -3000, 3000))
    want = xval(ref["ga_m"], ref["ga_e"])
    ok = (S >= 2.0 ** -1000) & (S <= 2.0 ** 1000)
    err = np.abs(a1[ok] - want[ok]) / S[ok]
    say(f"  exact sums: grad_a max scaled error {err.max():.3e} on {ok.sum()} coefficients")
    assert err.max() <= tol_grad_a()


def test_adjoint_atomic_mode(fpe):
    """The atomic mode (each wavefront's sums added to grad_a with FP64
    atomics): within u (2 C + 40 + W) of the oracle, W the wavefront partials
    an index can gather, and within that of the exact mode."""
    c = workloads.uniform_coeffs(1000, 61)
    z = workloads.spherical_points(3000, 62)
    g = scaled_g(c, z, 63)
    plan = fpe.precondition(to_dev(c), 53)
    ga_x, gz_x = plan.adjoint(to_dev(z), to_dev(g))
    plan.set_adjoint_mode("atomic")
    ga_a, gz_a = plan.adjoint(to_dev(z), to_dev(g))
    plan.set_adjoint_mode("exact")
    torch.cuda.synchronize()
    ga_x, ga_a = ga_x.cpu().numpy(), ga_a.cpu().numpy()
    assert np.array_equal(gz_x.cpu().numpy(), gz_a.cpu().numpy())
    ref = oracle.precondition(c, 53).adjoint(z, g)
    S = np.ldexp(ref["ga_scale_m"], np.clip(ref["ga_scale_e"], -3000, 3000))
    want = xval(ref["ga_m"], ref["ga_e"])
    ok = (S >= 2.0 ** -1000) & (S <= 2.0 ** 1000)
    tol = U * (2 * CHUNK + 40 + math.ceil(len(z) / 64))
    for label, ga in (("atomic", ga_a), ("exact", ga_x)):
        err = np.abs(ga[ok] - want[ok]) / S[ok]
        say(f"  {label} mode: grad_a max scaled error {err.max():.3e} (tol {tol:.3e})")
        assert err.max() <= tol
    assert (np.abs(ga_a[ok] - ga_x[ok]) / S[ok]).max() <= tol
    with pytest.raises(Exception):
        plan.set_adjoint_mode(7)
