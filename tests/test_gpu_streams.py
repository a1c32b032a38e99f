"""One plan (and one batch) evaluated on several HIP streams at once.

The binding caches one evaluation workspace per stream, so calls queued on
different streams may run concurrently: every result must equal the result of
the same evaluation on a single stream, bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

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


def test_plan_on_two_streams(fpe):
    w = workloads.workload("uniform_d1e6", n_points=200_000)
    plan = fpe.precondition(to_dev(w.coeffs), 53)
    z = to_dev(w.points)
    m0, e0 = plan.eval(z)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    cur = torch.cuda.current_stream()
    outs = []
    for s in streams:
        s.wait_stream(cur)
    for i in range(6):
        s = streams[i % 2]
        with torch.cuda.stream(s):
            out = (torch.empty_like(m0), torch.empty_like(e0))
        plan.eval(z, out=out, stream=s)
        outs.append(out)
    for s in streams:
        cur.wait_stream(s)
    torch.cuda.synchronize()
    assert len(plan._eval_ws) >= 3          # the current stream's and one per side stream
    for i, (m, e) in enumerate(outs):
        assert torch.equal(m, m0) and torch.equal(e, e0), i


def test_batch_on_two_streams(fpe):
    rng = np.random.default_rng(3)
    coeffs = [workloads.uniform_coeffs(int(d), 40 + i) for i, d in enumerate(rng.integers(50, 3000, 12))]
    points = [workloads.spherical_points(int(k), 80 + i) for i, k in enumerate(rng.integers(1, 600, 12))]
    plans = [fpe.precondition(to_dev(c), 53) for c in coeffs]
    offs = np.concatenate([[0], np.cumsum([len(p) for p in points])])
    batch = fpe.Batch(plans, offs)
    z = to_dev(np.concatenate(points))
    m0, e0 = batch.eval(z)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    cur = torch.cuda.current_stream()
    for s in streams:
        s.wait_stream(cur)
    outs = []
    for i in range(4):
        s = streams[i % 2]
        with torch.cuda.stream(s):
            out = (torch.empty_like(m0), torch.empty_like(e0))
        batch.eval(z, out=out, stream=s)
        outs.append(out)
    for s in streams:
        cur.wait_stream(s)
    torch.cuda.synchronize()
    for i, (m, e) in enumerate(outs):
        assert torch.equal(m, m0) and torch.equal(e, e0), i
