"""fpe_eval_noalloc (the entry point for callers that cannot allocate): through
the C ABI, two calls in a row on one plan, the second with fewer points, each
equal bit for bit to fpe_eval on the same points (the same kernels run with
the static scratch as workspace) and within 2^-44 of the oracle's window sum
on a sample; a size above the scratch's limit is refused before any launch;
torch's allocator sees no new memory during the calls."""
from __future__ import annotations

import ctypes
import gc

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


def test_noalloc_matches_fpe_eval_twice(fpe):
    w = workloads.workload("uniform_d1e6", degree=200_000, n_points=1 << 17)
    plan = fpe.precondition(to_dev(w.coeffs), 53)
    dev = torch.device("cuda:0")
    ref_plan = oracle.precondition(w.coeffs, 53)
    for n in (1 << 17, 5003):
        z = to_dev(w.points[:n])
        say(f"  fpe_eval_noalloc d={w.degree} n={n}")
        m0, e0, t0, w0 = plan.eval(z, terms=True, window=True)
        m = torch.full((n,), complex("nan"), dtype=torch.complex128, device=dev)
        e = torch.full((n,), -7, dtype=torch.int64, device=dev)
        t = torch.full((n,), -1, dtype=torch.int32, device=dev)
        win = torch.full((n, 2), -1, dtype=torch.int64, device=dev)
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        # no collection of earlier tests' tensors inside the measured region
        gc.collect()
        gc.disable()
        try:
            before = torch.cuda.memory_allocated()
            st = fpe.lib().fpe_eval_noalloc(plan._h, z.data_ptr(), n, m.data_ptr(), e.data_ptr(), t.data_ptr(),
                                            win.data_ptr(), stream)
            assert st == fpe.FPE_OK, fpe.lib().fpe_last_error()
            torch.cuda.synchronize()
            after = torch.cuda.memory_allocated()
        finally:
            gc.enable()
        assert after == before
        assert torch.equal(m, m0) and torch.equal(e, e0)
        assert torch.equal(t, t0) and torch.equal(win, w0)
        # a sample against the oracle's window sum at the same precision
        idx = np.random.default_rng(n).choice(n, size=min(n, 400), replace=False)
        ref = ref_plan.eval(w.points[idx])
        err = oracle.scaled_error(m.cpu().numpy()[idx], e.cpu().numpy()[idx], ref["m"], ref["e"],
                                  ref["dwin_m"], ref["dwin_e"])
        say(f"    bit-exact against fpe_eval; max scaled error {err.max():.3e} on {idx.size} points")
        assert err.max() <= TOL


def test_noalloc_refuses_sizes_above_its_scratch(fpe):
    c = workloads.uniform_coeffs(2000, 5)
    plan = fpe.precondition(to_dev(c), 53)
    n = 1 << 22           # 128 MiB of sorted records alone: refused on the host, nothing launched
    dev = torch.device("cuda:0")
    z = torch.ones(n, dtype=torch.complex128, device=dev)
    m = torch.empty(n, dtype=torch.complex128, device=dev)
    e = torch.empty(n, dtype=torch.int64, device=dev)
    st = fpe.lib().fpe_eval_noalloc(plan._h, z.data_ptr(), n, m.data_ptr(), e.data_ptr(), None, None,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 4, st    # FPE_ERR_WORKSPACE
    assert "scratch" in fpe.lib().fpe_last_error().decode()
    # a valid call on the same device still works afterwards
    z = to_dev(workloads.spherical_points(300, 9))
    m, e = plan.eval(z)
    m2 = torch.empty_like(m)
    e2 = torch.empty_like(e)
    plan.eval_noalloc(z, (m2, e2))
    torch.cuda.synchronize()
    assert torch.equal(m, m2) and torch.equal(e, e2)
