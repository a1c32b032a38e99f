"""The exact window comparison of tests/windows.py, on the CPU: the oracle's
own windows pass with no rounding exception on the benchmark workloads; a
window end moved by one index fails; points placed on a jump of the window
rule (x_R within 2^-40 of an integer + eta) are found and both neighbouring
ends accepted there."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2211_06320_amd import workloads
from windows import ambiguous_ends, check_windows


@pytest.mark.parametrize("name", ["uniform_d1000", "wide_d2p20", "sparse_wide_d2p20"])
def test_oracle_windows_pass_exactly(name):
    wl = workloads.workload(name, n_points=20000)
    P = oracle.precondition(wl.coeffs, 53)
    r = P.eval(wl.points)
    w = np.stack([r["l"], r["r"]], axis=1)
    assert check_windows(P, r, w, r["terms"]) == 0


def test_planted_off_by_one_fails():
    wl = workloads.workload("uniform_d1000", n_points=5000)
    P = oracle.precondition(wl.coeffs, 53)
    r = P.eval(wl.points)
    w = np.stack([r["l"], r["r"]], axis=1)
    rng = np.random.default_rng(5)
    for col, delta in ((0, 1), (0, -1), (1, 1), (1, -1)):
        ww = w.copy()
        # a point whose end can move and stay inside [v, d]
        inner = (ww[:, 0] > 0) if col == 0 else (ww[:, 1] < wl.degree)
        cand = np.flatnonzero((ww[:, 1] - ww[:, 0] > 2) & inner)
        j = rng.choice(cand)
        ww[j, col] += delta
        with pytest.raises(AssertionError):
            check_windows(P, r, ww, r["terms"])
    # a term count off by one
    t = r["terms"].copy()
    t[17] += 1
    with pytest.raises(AssertionError):
        check_windows(P, r, w, t)


def test_points_on_a_jump_are_bracketed():
    """a_k = 1, d = 5000, |z| < 1: x_R = T / |lambda| (flat cover, eq. def:LRN).
    Choosing |lambda| = T / (m + eta) puts x_R + eta on the integer m + 2 eta,
    away from a jump; T / (m - eta) puts x_R + eta on m itself, where the floor
    jumps: those points are flagged and r = m - 1 and r = m both pass."""
    d = 5000
    c = np.ones(d + 1, np.complex128)
    P = oracle.precondition(c, 53)
    T = P.info().T
    eta = 2.0 ** -20
    m = np.arange(300, 4000, 7).astype(float)
    on = -T / (m - eta)
    off = -T / (m + 0.5)
    lam = np.concatenate([on, off])
    z = np.exp2(lam) * np.exp(1j * np.linspace(0, 6, lam.size))
    r = P.eval(z)
    amb = ambiguous_ends(P, r)
    flagged = amb[:, 2] != amb[:, 3]
    assert flagged[: on.size].mean() > 0.9
    assert not flagged[on.size:].any()
    w = np.stack([r["l"], r["r"]], axis=1)
    for delta in (-1, 1):
        ww = w.copy()
        sel = np.flatnonzero(flagged)
        ww[sel, 1] = np.where(ww[sel, 1] == amb[sel, 2], amb[sel, 3], amb[sel, 2])
        pre = np.concatenate([[0], np.cumsum(P.good())])
        t = pre[ww[:, 1] + 1] - pre[ww[:, 0]]
        assert check_windows(P, r, ww, t) == flagged.sum()
