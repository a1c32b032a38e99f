"""Many polynomials in one evaluation (fpe_eval_batched) against fpe_eval of
each plan alone (bit for bit with FP64 plans: every lane's chunk partials and
powers follow the same recipe whatever the grouping) and against the oracle
(max |FPE - oracle| / sum over the window of |a_k||z|^k <= 2^-44; <= 2^-18 for
FP32 plans at p = 24).  Also: the 4096-polynomial workload, the limits, and
replays of a captured HIP graph."""
from __future__ import annotations

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


def mixed_batch(seed):
    rng = np.random.default_rng(seed)
    coeffs, points = [], []
    counts = [0, 1, 63, 64, 65, 128, 700, 1000] + [int(x) for x in rng.integers(1, 400, 28)]
    for i, m in enumerate(counts):
        d = int(np.exp(rng.uniform(np.log(16), np.log(8000))))
        c = workloads.uniform_coeffs(d, 1000 + i) if i % 3 else workloads.wide_coeffs(d, 1000 + i, sigma=12.0)
        coeffs.append(c)
        z = workloads.spherical_points(m, 2000 + i)
        if i == 6:
            z[:4] = [0, np.nan, 1e300 + 1e300j, 1.0]
        points.append(z)
    coeffs.append(np.zeros(40, np.complex128))         # P == 0
    points.append(workloads.spherical_points(70, 77))
    return coeffs, points


def run_batch(fpe, coeffs, points, fp32=False, p=53):
    # the chunk length pinned on every plan and on the batch: bit-for-bit
    # agreement holds for equal chunk lengths, and an earlier autotune in the
    # process may have cached another choice for some plan's size bucket
    plans = [fpe.precondition(to_dev(c), p, fp32=fp32) for c in coeffs]
    for pl in plans:
        pl.set_chunk(512)
    offs = np.concatenate([[0], np.cumsum([len(z) for z in points])])
    batch = fpe.Batch(plans, offs)
    batch.set_chunk(512)
    zall = np.concatenate(points) if len(points) else np.zeros(0, np.complex128)
    m, e, t = batch.eval(to_dev(zall), terms=True)
    torch.cuda.synchronize()
    return plans, offs, zall, m.cpu().numpy(), e.cpu().numpy(), t.cpu().numpy()


def test_batched_matches_single_and_oracle(fpe):
    coeffs, points = mixed_batch(5)
    plans, offs, zall, m, e, t = run_batch(fpe, coeffs, points)
    worst = 0.0
    for i, (c, z) in enumerate(zip(coeffs, points)):
        if len(z) == 0:
            continue
        sl = slice(offs[i], offs[i + 1])
        m1, e1, t1, _ = plans[i].eval(to_dev(z), terms=True, window=True)
        assert np.array_equal(m[sl].view(np.float64), m1.cpu().numpy().view(np.float64), equal_nan=True), i
        assert np.array_equal(e[sl], e1.cpu().numpy()) and np.array_equal(t[sl], t1.cpu().numpy()), i
        ref = oracle.precondition(c, 53).eval(z)
        fin = np.isfinite(z.real) & np.isfinite(z.imag)
        err = oracle.scaled_error(m[sl][fin], e[sl][fin], ref["m"][fin], ref["e"][fin], ref["dwin_m"][fin],
                                  ref["dwin_e"][fin])
        worst = max(worst, float(err.max(initial=0.0)))
    say(f"  mixed batch of {len(coeffs)}: max scaled error {worst:.3e}")
    assert worst <= TOL


def test_batched_extreme_plans(fpe):
    """A batch whose polynomials include a 600-vertex cover (searched in global
    memory) and good coefficients over 1700 binary orders, beside ordinary ones:
    bit for bit the single-plan results, and within tolerance of the oracle."""
    i = np.arange(600)
    k = i * (i + 1) // 2
    many = np.zeros(k[-1] + 1, complex)
    many[k] = 1.5 * np.exp2(i - 1.0) * np.exp(1j * i)
    d = 20_000
    kk = np.arange(d + 1)
    wide = np.exp2(850 - np.round(1700 * ((2.0 * kk / d) - 1) ** 2) - 0.5) * np.exp(1j * 0.37 * kk)
    rng = np.random.default_rng(61)
    near = lambda n, s: 2.0 ** rng.uniform(-s, s, n) * np.exp(1j * rng.uniform(0, 2 * np.pi, n))
    coeffs = [workloads.uniform_coeffs(300, 5), many, wide, workloads.uniform_coeffs(2000, 6)]
    points = [workloads.spherical_points(200, 71), near(1500, 0.2), near(1500, 0.2), near(900, 0.01)]
    say("batch with a 600-vertex cover and a 1700-bit scale range")
    plans, offs, zall, m, e, t = run_batch(fpe, coeffs, points)
    worst = 0.0
    for j, (c, z) in enumerate(zip(coeffs, points)):
        sl = slice(offs[j], offs[j + 1])
        m1, e1, t1, _ = plans[j].eval(to_dev(z), terms=True, window=True)
        assert np.array_equal(m[sl].view(np.float64), m1.cpu().numpy().view(np.float64)), j
        assert np.array_equal(e[sl], e1.cpu().numpy()) and np.array_equal(t[sl], t1.cpu().numpy()), j
        ref = oracle.precondition(c, 53).eval(z)
        err = oracle.scaled_error(m[sl], e[sl], ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"])
        worst = max(worst, float(err.max(initial=0.0)))
    say(f"  max scaled error {worst:.3e}")
    assert worst <= TOL


def test_batched_workload_4096(fpe):
    coeffs, points = workloads.batched_workload()
    plans, offs, zall, m, e, t = run_batch(fpe, coeffs, points)
    rng = np.random.default_rng(9)
    worst = 0.0
    for i in rng.choice(len(coeffs), 48, replace=False):
        sl = slice(offs[i], offs[i + 1])
        m1, e1 = plans[i].eval(to_dev(points[i]))
        assert np.array_equal(m[sl].view(np.float64), m1.cpu().numpy().view(np.float64)), i
        assert np.array_equal(e[sl], e1.cpu().numpy()), i
    for i in rng.choice(len(coeffs), 12, replace=False):
        sl = slice(offs[i], offs[i + 1])
        ref = oracle.precondition(coeffs[i], 53).eval(points[i])
        err = oracle.scaled_error(m[sl], e[sl], ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"])
        worst = max(worst, float(err.max()))
    say(f"  4096 polynomials, {len(zall)} points: max scaled error on 12 sampled polynomials {worst:.3e}")
    assert worst <= TOL


def test_batched_workload_4096_fp32(fpe):
    """The 4096-polynomial workload with FP32 plans (p = 24): within 2^-18 of
    the oracle at p = 24 on 12 sampled polynomials."""
    coeffs, points = workloads.batched_workload()
    plans, offs, zall, m, e, t = run_batch(fpe, coeffs, points, fp32=True, p=24)
    rng = np.random.default_rng(19)
    worst = 0.0
    for i in rng.choice(len(coeffs), 12, replace=False):
        sl = slice(offs[i], offs[i + 1])
        ref = oracle.precondition(coeffs[i], 24).eval(points[i])
        err = oracle.scaled_error(m[sl], e[sl], ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"])
        worst = max(worst, float(err.max()))
    say(f"  4096 polynomials with FP32 plans: max scaled error on 12 sampled polynomials {worst:.3e}")
    assert worst <= 2.0 ** -18


def test_batched_limits(fpe):
    c = to_dev(workloads.uniform_coeffs(50, 3))
    p = fpe.precondition(c, 53)
    with pytest.raises(fpe.FPEError):
        fpe.Batch([p], [0, 4097])                       # more than 4096 points on one polynomial
    with pytest.raises(fpe.FPEError):
        fpe.Batch([p, p], [0, 10, 5])                   # decreasing offsets
    b = fpe.Batch([p, p], [0, 4096, 4096])              # the maximum, then none
    z = workloads.spherical_points(4096, 4)
    m, e = b.eval(to_dev(z))
    m1, e1 = p.eval(to_dev(z))
    assert np.array_equal(m.cpu().numpy(), m1.cpu().numpy()) and np.array_equal(e.cpu().numpy(), e1.cpu().numpy())


def test_batched_graph_replays(fpe):
    """Captured in a HIP graph (kernels only), replayed three times with eager
    work in between: every replay equals the eager result."""
    coeffs, points = mixed_batch(6)
    plans = [fpe.precondition(to_dev(c), 53) for c in coeffs]
    offs = np.concatenate([[0], np.cumsum([len(z) for z in points])])
    batch = fpe.Batch(plans, offs)
    z = to_dev(np.concatenate(points))
    n = z.shape[0]
    out = (torch.empty(n, dtype=torch.complex128, device=z.device), torch.empty(n, dtype=torch.int64, device=z.device))
    batch.eval(z, out=out)
    torch.cuda.synchronize()
    ref = (out[0].clone(), out[1].clone())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.eval(z, out=out)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.eval(z, out=out)
    for r in range(3):
        out[0].fill_(0)
        out[1].fill_(-1)
        plans[1].eval(z[:100])                          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        # bit for bit (the batch holds a NaN point, so NaN compares equal to NaN here)
        assert np.array_equal(out[0].cpu().numpy().view(np.float64), ref[0].cpu().numpy().view(np.float64),
                              equal_nan=True), r
        assert torch.equal(out[1], ref[1]), r


def test_batched_fp32_plans(fpe):
    coeffs, points = mixed_batch(7)
    plans, offs, zall, m, e, t = run_batch(fpe, coeffs, points, fp32=True, p=24)
    worst = 0.0
    for i, (c, z) in enumerate(zip(coeffs, points)):
        if len(z) == 0:
            continue
        sl = slice(offs[i], offs[i + 1])
        ref = oracle.precondition(c, 24).eval(z)
        fin = np.isfinite(z.real) & np.isfinite(z.imag)
        err = oracle.scaled_error(m[sl][fin], e[sl][fin], ref["m"][fin], ref["e"][fin], ref["dwin_m"][fin],
                                  ref["dwin_e"][fin])
        worst = max(worst, float(err.max(initial=0.0)))
    say(f"  FP32 batch: max scaled error {worst:.3e}")
    assert worst <= 2.0 ** -18
