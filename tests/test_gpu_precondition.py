"""Preconditioning forms against each other and against the oracle.

* The split form (Remark partialpreproc, Section 5.1): one cover, then plans
  for p = 53, 24 and 6 (and an FP32 plan at 24), each bit for bit the plan
  fpe_precondition builds (cover vertices, G_p, then the evaluation of the
  same points, compared bit for bit), and the cover's vertices the oracle's.
* The batched form: plans of many polynomials from one launch sequence, bit for
  bit those of fpe_precondition one at a time, including a polynomial above
  the one-workgroup limit (2^17 coefficients) inside the batch.
* The one-workgroup kernel and the per-coefficient kernels on either side of
  that limit: both plans equal the oracle's bit for bit.
* Errors: a non-finite coefficient in a batch fails the call and names the
  polynomial.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2211_06320_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def same_plan(a, b, z=None):
    """Same summary, cover and G_p, and the same values bit for bit.  FP32
    plans are evaluated one point per call: which tiles of a wavefront run in
    FP32 depends on the points sharing it, so only a lone point's value is a
    function of the plan alone."""
    ia, ib = a.info(), b.info()
    assert ia == ib, (ia, ib)
    ha, hb = a.export(), b.export()
    for x, y in zip(ha, hb):
        assert np.array_equal(x, y)
    if z is not None and ia.n_hull > 0:
        if a.fp32:
            for i in range(0, z.shape[0], max(1, z.shape[0] // 40)):
                ma, ea = a.eval(z[i:i + 1])
                mb, eb = b.eval(z[i:i + 1])
                assert torch.equal(ma, mb) and torch.equal(ea, eb)
        else:
            ma, ea = a.eval(z)
            mb, eb = b.eval(z)
            assert torch.equal(ma, mb) and torch.equal(ea, eb)
        torch.cuda.synchronize()


def oracle_plan_equal(plan, c, p):
    ref = oracle.precondition(c, p)
    ri, gi = ref.info(), plan.info()
    assert (gi.d, gi.v, gi.dt, gi.n_hull, gi.n_good, gi.T, gi.p) == \
        (ri.d, ri.v, ri.dt, ri.n_hull, ri.n_good, ri.T, ri.p)
    hk, hs, good = plan.export()
    rk, rs = ref.hull()
    assert np.array_equal(hk, rk) and np.array_equal(hs, rs)
    assert np.array_equal(good, ref.good())


def polys():
    w = workloads
    return {
        "uniform_d1000": w.uniform_coeffs(1000, 1),
        "wide_d4096": w.wide_coeffs(4096, 3),
        "sparse_wide_d8192": w.sparse_wide_coeffs(8192, 3),
        "zeros_at_ends": np.concatenate([[0, 0], w.uniform_coeffs(50, 9), [0, 0, 0]]),
        "constant": np.array([3 + 4j], complex),
        "all_zero": np.zeros(7, complex),
        "wide_d200000": w.wide_coeffs(200_000, 5),          # above the one-workgroup limit
    }


def test_split_preconditioning_matches_one_shot(fpe):
    z = to_dev(workloads.spherical_points(5000, 81))
    for name, c in polys().items():
        cd = to_dev(c)
        cover = fpe.Cover(cd)
        d, v, dt, nh, smax = cover.info()
        ref = oracle.precondition(c, 53)
        rk, _ = ref.hull()
        assert d == len(c) - 1 and nh == len(rk)
        for p, fp32 in ((53, False), (24, False), (6, False), (24, True)):
            say(f"  split {name} p={p} fp32={fp32}")
            a = cover.plan(p, fp32=fp32)
            b = fpe.precondition(cd, p, fp32=fp32)
            same_plan(a, b, z)
            oracle_plan_equal(a, c, p)
        del cover                       # plans keep their own copy of the cover
        torch.cuda.synchronize()


def test_batched_preconditioning_matches_one_at_a_time(fpe):
    cs = list(polys().values())
    rng = np.random.default_rng(82)
    for i in range(40):                 # many small ones of uneven degree
        d = int(np.exp(rng.uniform(np.log(16), np.log(65536))))
        cs.append(workloads.uniform_coeffs(d, 1000 + i) if i % 3 else workloads.wide_coeffs(d, 2000 + i))
    z = to_dev(workloads.spherical_points(3000, 83))
    for p, fp32 in ((53, False), (24, True)):
        plans = fpe.precondition_batched([to_dev(c) for c in cs], p, fp32=fp32)
        assert len(plans) == len(cs)
        say(f"  batch of {len(cs)} polynomials p={p} fp32={fp32}")
        for c, a in zip(cs, plans):
            b = fpe.precondition(to_dev(c), p, fp32=fp32)
            same_plan(a, b, z)
        for i in (0, 1, 2, 6, len(cs) - 1):
            oracle_plan_equal(plans[i], cs[i], p)


@pytest.mark.parametrize("n1", [(1 << 17) - 1, 1 << 17, (1 << 17) + 1])
def test_both_kernels_at_the_limit(fpe, n1):
    c = workloads.wide_coeffs(n1 - 1, 84)
    c[:3] = 0
    c[-2:] = 0
    for p in (53, 24):
        plan = fpe.precondition(to_dev(c), p)
        oracle_plan_equal(plan, c, p)


def test_batch_with_a_bad_coefficient_fails(fpe):
    cs = [workloads.uniform_coeffs(100, 1), workloads.uniform_coeffs(50, 2), workloads.uniform_coeffs(70, 3)]
    cs[1][7] = np.nan
    with pytest.raises(fpe.FPEError) as ei:
        fpe.precondition_batched([to_dev(c) for c in cs], 53)
    assert ei.value.status == 2 and "polynomial 1" in str(ei.value)
