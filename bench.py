#!/usr/bin/env python3
"""Headline measurement: FPE evaluation throughput on one MI355X.

Workload: one complex polynomial of degree d = 10^6 with Re, Im of the
coefficients i.i.d. uniform on [-1, 1], evaluated at 10^6 points uniform on the
Riemann sphere (seeded, synthetic), FP64, p = 53.  A step is one fpe_eval call
over all points (the whole evaluation phase: plan, sort, window sums, combine),
with the plan and the points resident in HBM.  Preconditioning is timed
separately, as the paper does.  value and ms_per_step: K steps queued back to
back between two events, right after the W warm-up steps; ms_per_step_median:
K further steps with an event after each (and the window kernel's events).

Besides the metric, value and timing fields, the line carries:
  roofline      the window kernel (the dominant kernel) against the FP64 vector
                peak: algorithmic flops per launch / its average launch time
                from HIP events recorded around it on its stream; traffic is
                the HBM bytes per launch recorded with rocprofv3 counters in
                profiles/k_window_uniform_d1e6_traffic.txt, reported only while
                the window kernel's sources are the ones those counters measured
  cpu_baseline  the oracle (plain C) with its plain-FP64 window sum over every
                point, on the host's threads (at most 16) and on one thread;
                its double-double mode on a sample beside it
  horner_gpu    the same-GPU Horner baseline over all points
  two_streams   the same evaluations queued alternately on two HIP streams
                (one plan, a workspace per stream): throughput beside the
                one-stream headline value
  max_scaled_err  max |FPE - reference| / sum|a_k||z|^k on a seeded sample,
                the reference being the oracle's window sum at p = 116
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "evaluations/sec at d=1e6 (FPE vs GPU Horner), max rel err vs FP64 oracle"
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
PROFILE_EVERY = 4
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_window_uniform_d1e6_traffic.txt")
WINDOW_SOURCES = [os.path.join(ROOT, "paper_2211_06320_amd", "csrc", f) for f in ("fpe_eval.hip", "fpe_internal.h")]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_flops(terms, window) -> float:
    """Per point: 8 flops per kept term (one complex multiply-add, Section 5.2)
    plus 6 flops per complex multiplication of z^l by repeated squaring
    (2 log2 l multiplications, Section 8.2)."""
    import numpy as np
    U = terms.astype(np.float64)
    l = window[:, 0].astype(np.float64)
    mults = np.where(l >= 2, np.ceil(2.0 * np.log2(np.maximum(l, 1.0))), 0.0)
    return float(8.0 * U.sum() + 6.0 * mults.sum())


def window_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in WINDOW_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


VALU_PROFILE = os.path.join(ROOT, "profiles", "k_window_uniform_d1e6_valu_l2.txt")


def recorded_counters(workload: str, chunk: int):
    """The window kernel's FP64 VALU and L2 counters per launch from the
    committed rocprofv3 summary (executed FP64 TFLOP/s, VALU busy and
    utilisation, L2 hit rate), or None when it is missing, for another workload
    or chunk length, or for other kernel sources."""
    if workload != "uniform_d1e6" or not os.path.exists(VALU_PROFILE):
        return None
    kv = {}
    with open(VALU_PROFILE) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.split("#")[0].strip()
    if kv.get("window_sources_sha256") != window_sources_sha256():
        return None
    try:
        return {"executed_fp64_tflops": float(kv[f"executed_fp64_tflops_c{chunk}"]),
                "executed_frac": float(kv[f"executed_fp64_tflops_c{chunk}"]) / FP64_VECTOR_PEAK_TFLOPS,
                "valu_busy_percent": float(kv[f"valu_busy_percent_c{chunk}"]),
                "valu_utilisation_percent": float(kv[f"valu_utilisation_percent_c{chunk}"]),
                "l2_hit_rate": float(kv[f"l2_hit_rate_c{chunk}"]),
                "profile": os.path.relpath(VALU_PROFILE, ROOT)}
    except (KeyError, ValueError):
        return None


def recorded_traffic(workload: str, chunk: int):
    """HBM bytes per window-kernel launch from the committed counter summary, or
    None when it is missing, for another workload or chunk length, or for other
    kernel sources."""
    if workload != "uniform_d1e6" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    kv = {}
    with open(TRAFFIC_PROFILE) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("window_sources_sha256") != window_sources_sha256():
        return None
    try:
        return float(kv[f"traffic_bytes_per_launch_c{chunk}"])
    except (KeyError, ValueError):
        return None


def adjoint_leg(fpe, workloads, torch, dev, steps: int) -> dict:
    """Derivative, reverse mode and Newton at d = 2^18 with 2^20 points: the
    forward pass with Q' (fpe_eval_deriv), the backward pass (grad_a summed
    exactly in fixed point, and with FP64 atomics) of
    L = sum_j |Q_j|^2 4^(-e_j) (each point's |Q|^2 normalised by its detached
    exponent, so that no term overflows; upstream gradient 2 Q_j 4^(-e_j), passed
    as 2 m_j with the exponent -e_j applied inside the kernels) with
    respect to every a_k and z_j (fpe_eval_adjoint), and one Newton step on
    every point (fpe_newton_step)."""
    wl = workloads.workload("uniform_d2p18")
    c = torch.from_numpy(wl.coeffs).to(dev)
    z = torch.from_numpy(wl.points).to(dev)
    plan = fpe.precondition(c, 53)
    m, e, md, ed = plan.eval_deriv(z)
    g = 2.0 * m                       # upstream gradients 2 Q_j 4^-e_j = (2 m_j) 2^-e_j
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    n = len(wl.points)
    t_fwd = timed(lambda: plan.eval_deriv(z))
    t_bwd = timed(lambda: plan.adjoint(z, g, md, ed, g_exp=e))
    plan.set_adjoint_mode("atomic")
    t_bwd_atomic = timed(lambda: plan.adjoint(z, g, md, ed, g_exp=e))
    plan.set_adjoint_mode("exact")
    t_newton = timed(lambda: plan.newton_step(z))
    log(f"d=2^18, 2^20 points: forward with Q' {t_fwd:.3f} ms, backward {t_bwd:.3f} ms (exact sums; "
        f"{t_bwd_atomic:.3f} ms with FP64 atomics), Newton step {t_newton:.3f} ms")
    out = {"workload": wl.name, "d": wl.degree, "n_points": n, "unit": "points/s",
           "forward_with_derivative": {"ms": t_fwd, "value": n / (t_fwd * 1e-3)},
           "backward_grad_a_and_z": {"ms": t_bwd, "value": n / (t_bwd * 1e-3), "grad_a_sums": "exact"},
           "backward_grad_a_and_z_atomic": {"ms": t_bwd_atomic, "value": n / (t_bwd_atomic * 1e-3),
                                            "grad_a_sums": "FP64 atomics"},
           "newton_step": {"ms": t_newton, "value": n / (t_newton * 1e-3)}}
    # p = 24: FP32 blocks for Q and Q' (and the Newton step), beside FP64
    # arithmetic at the same p; errors of Q' against the oracle on a sample
    import numpy as np
    import oracle
    idx = np.random.default_rng(12349).choice(n, 1000, replace=False)
    ref = oracle.precondition(wl.coeffs, 24).eval_deriv(wl.points[idx])
    for label, fp32 in (("fp32_p24", True), ("fp64_arith_p24", False)):
        p24 = fpe.precondition(c, 24, fp32=fp32)
        tf = timed(lambda: p24.eval_deriv(z))
        tn = timed(lambda: p24.newton_step(z))
        _, _, md24, ed24 = p24.eval_deriv(z)
        torch.cuda.synchronize()
        mdn, edn = md24.cpu().numpy()[idx], ed24.cpu().numpy()[idx]
        ok = ref["ddwin_m"] > 0
        err = oracle.scaled_error(mdn[ok], edn[ok], ref["md"][ok], ref["ed"][ok], ref["ddwin_m"][ok],
                                  ref["ddwin_e"][ok])
        out[label] = {"forward_with_derivative_ms": tf, "newton_step_ms": tn,
                      "value_forward": n / (tf * 1e-3), "max_scaled_err_derivative": float(err.max())}
        log(f"  {label}: forward with Q' {tf:.3f} ms, Newton step {tn:.3f} ms, Q' max scaled error {err.max():.2e}")
    return out


def fp32_leg(fpe, workloads, oracle, np, torch, dev, steps: int, check: int) -> dict:
    """FP32 window sums at p = 24 (FPE_PRECONDITION_FP32: plain FP32 blocks of 8
    with FP64 accumulation, and with FPE_PRECONDITION_FP32_COMPENSATED the
    blocks by the compensated TwoSum/TwoProd recurrence) beside FP64 arithmetic
    at the same p, on the headline workload and the two wide-range workloads
    (d = 2^20): evaluations/s over all points and the max scaled error against
    the oracle at p = 24 on a seeded sample."""
    out = {}
    for name in ("uniform_d1e6", "wide_d2p20", "sparse_wide_d2p20"):
        wl = workloads.workload(name)
        c = torch.from_numpy(wl.coeffs).to(dev)
        z = torch.from_numpy(wl.points).to(dev)
        n = len(wl.points)
        idx = np.random.default_rng(12346).choice(n, min(check, n), replace=False)
        ref = oracle.precondition(wl.coeffs, 24).eval(wl.points[idx])
        row = {"d": wl.degree, "n_points": n}
        for label, fp32, comp in (("fp32", True, False), ("fp32_compensated", True, True),
                                  ("fp64_arith", False, False)):
            plan = fpe.precondition(c, 24, fp32=fp32, compensated=comp)
            mo = (torch.empty(n, dtype=torch.complex128, device=dev), torch.empty(n, dtype=torch.int64, device=dev))
            plan.eval(z, out=mo)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                plan.eval(z, out=mo)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / steps
            mm, ee = mo[0].cpu().numpy(), mo[1].cpu().numpy()
            err = oracle.scaled_error(mm[idx], ee[idx], ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"])
            row[label] = {"ms": ms, "value": n / (ms * 1e-3), "max_scaled_err": float(err.max())}
        log(f"p=24 {name}: FP32 {row['fp32']['ms']:.3f} ms (max err {row['fp32']['max_scaled_err']:.2e}), "
            f"FP32 compensated {row['fp32_compensated']['ms']:.3f} ms "
            f"(max err {row['fp32_compensated']['max_scaled_err']:.2e}), "
            f"FP64 arithmetic {row['fp64_arith']['ms']:.3f} ms (max err {row['fp64_arith']['max_scaled_err']:.2e})")
        out[name] = row
    out["unit"] = "evaluations/s"
    out["tolerance"] = 2.0 ** -18
    return out


def sparse_gap_digits(good, terms, window, np) -> float:
    """Sum over the points of the binary digits of the gaps between consecutive
    kept indices (a product by a power z^(2^j) per digit in the sparse form)."""
    g = np.flatnonzero(good)
    if g.size < 2:
        return 0.0
    cp = np.concatenate([[0], np.cumsum(np.bitwise_count(np.diff(g)).astype(np.int64))])
    pref = np.concatenate([[0], np.cumsum(good.astype(np.int64))])
    ok = window[:, 0] <= window[:, 1]
    pa = pref[window[ok, 0]]
    pb = pref[window[ok, 1] + 1]
    m = pb - pa >= 2
    return float((cp[pb[m] - 1] - cp[pa[m]]).sum())


def wide_leg(fpe, workloads, oracle, np, torch, dev, steps: int, check: int) -> dict:
    """d = 2^20 with |a_k| = 2^g, g ~ N(0, 40^2) (dense, and 1 % nonzero), 10^6
    points, FP64 at p = 53 and p = 24: the window sums in the dense form
    (Horner over every index, bad coefficients masked) and in the sparse form
    (Horner over the list of G_p, gaps jumped by powers of z), each at its
    fastest chunk length; evaluations/s, the window kernel's time and its
    algorithmic fraction of the FP64 peak (8 flops per kept term, 6 per
    product of z^l's powering and, in the sparse form, 6 per binary digit of
    each gap), and the max scaled error against the oracle at the same p on a
    seeded sample."""
    out = {}
    for name in ("wide_d2p20", "sparse_wide_d2p20"):
        wl = workloads.workload(name)
        c = torch.from_numpy(wl.coeffs).to(dev)
        z = torch.from_numpy(wl.points).to(dev)
        n = len(wl.points)
        idx = np.random.default_rng(12348).choice(n, min(check, n), replace=False)
        for p in (53, 24):
            plan = fpe.precondition(c, p)
            _, _, good = plan.export()
            _, _, t, w = plan.eval(z, terms=True, window=True)
            torch.cuda.synchronize()
            terms, window = t.cpu().numpy(), w.cpu().numpy()
            base = algorithmic_flops(terms, window)
            digits = sparse_gap_digits(good, terms, window, np)
            ref = oracle.precondition(wl.coeffs, p).eval(wl.points[idx])
            row = {"d": wl.degree, "n_points": n, "p_bits": p, "kept_terms": int(terms.sum()),
                   "window_indices": int((window[:, 1] - window[:, 0] + 1).clip(0).sum()), "gap_digits": digits}
            mo = (torch.empty(n, dtype=torch.complex128, device=dev), torch.empty(n, dtype=torch.int64, device=dev))
            for mode in ("dense", "sparse"):
                plan.set_window_mode(mode)
                best = None
                for C in (256, 512, 1024, 2048):
                    plan.set_chunk(C)
                    plan.eval(z, out=mo)
                    torch.cuda.synchronize()
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    for _ in range(3):
                        plan.eval(z, out=mo)
                    b.record()
                    torch.cuda.synchronize()
                    ms = a.elapsed_time(b) / 3
                    if best is None or ms < best[1]:
                        best = (C, ms)
                plan.set_chunk(best[0])
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(steps):
                    plan.eval(z, out=mo)
                b.record()
                torch.cuda.synchronize()
                ms = a.elapsed_time(b) / steps
                fpe.profile_read()
                fpe.profile_enable(True)
                for _ in range(3):
                    plan.eval(z, out=mo)
                torch.cuda.synchronize()
                fpe.profile_enable(False)
                wms, k = fpe.profile_read()
                wms /= max(k, 1)
                flops = base + (6.0 * digits if mode == "sparse" else 0.0)
                mm, ee = mo[0].cpu().numpy(), mo[1].cpu().numpy()
                err = oracle.scaled_error(mm[idx], ee[idx], ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"])
                row[mode] = {"chunk": best[0], "ms": ms, "value": n / (ms * 1e-3), "window_kernel_ms": wms,
                             "algorithmic_flops": flops,
                             "frac_fp64_peak": flops / (wms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                             "max_scaled_err": float(err.max())}
            log(f"{name} p={p}: dense {row['dense']['ms']:.3f} ms (window {row['dense']['window_kernel_ms']:.3f}, "
                f"C={row['dense']['chunk']}), sparse {row['sparse']['ms']:.3f} ms "
                f"(window {row['sparse']['window_kernel_ms']:.3f}, C={row['sparse']['chunk']}); kept terms "
                f"{row['kept_terms']:.3e} of {row['window_indices']:.3e} window indices; max err dense "
                f"{row['dense']['max_scaled_err']:.2e} sparse {row['sparse']['max_scaled_err']:.2e}")
            out[f"{name}_p{p}"] = row
    out["unit"] = "evaluations/s"
    out["tolerance"] = 2.0 ** -44
    return out


def batched_leg(fpe, workloads, oracle, np, torch, dev, steps: int) -> dict:
    """4096 polynomials, degrees log-uniform in [16, 65536], 64..1024 spherical
    points each (FP64, p = 53): preconditioning of every plan (timed apart),
    the batch's chunk length from the autotuner, then fpe_eval_batched over all
    points, eagerly and as a replayed HIP graph, beside one fpe_eval per
    polynomial in a loop."""
    coeffs, points = workloads.batched_workload()
    cdev = [torch.from_numpy(c).to(dev) for c in coeffs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop_plans = [fpe.precondition(c, 53) for c in cdev]
    torch.cuda.synchronize()
    pre_loop_ms = (time.perf_counter() - t0) * 1e3
    del loop_plans
    fpe.precondition_batched(cdev[:8], 53)          # warm-up of the batched kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans = fpe.precondition_batched(cdev, 53)
    torch.cuda.synchronize()
    pre_ms = (time.perf_counter() - t0) * 1e3
    offs = np.concatenate([[0], np.cumsum([len(z) for z in points])])
    batch = fpe.Batch(plans, offs)
    z = torch.from_numpy(np.concatenate(points)).to(dev)
    n = z.shape[0]
    chunk = batch.autotune(z)
    out = (torch.empty(n, dtype=torch.complex128, device=dev), torch.empty(n, dtype=torch.int64, device=dev))
    batch.eval(z, out=out)
    torch.cuda.synchronize()

    def timed(fn, k):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(k):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    eager_ms = timed(lambda: batch.eval(z, out=out), steps)
    # kept terms (one untimed call with term counts) and the window kernel's
    # own time (HIP events around its launches, a few eager calls)
    kept = int(batch.eval(z, terms=True)[2].sum().item())
    fpe.profile_read()
    fpe.profile_enable(True)
    for _ in range(3):
        batch.eval(z, out=out)
    torch.cuda.synchronize()
    fpe.profile_enable(False)
    win_ms, win_k = fpe.profile_read()
    win_ms = win_ms / max(win_k, 1)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.eval(z, out=out)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.eval(z, out=out)
    graph_ms = timed(g.replay, steps)
    zs = [z[offs[i]:offs[i + 1]] for i in range(len(plans))]
    loop_ms = timed(lambda: [p.eval(zz) for p, zz in zip(plans, zs)], 1)
    mm, ee = out[0].cpu().numpy(), out[1].cpu().numpy()
    rng = np.random.default_rng(12347)
    worst = 0.0
    for i in rng.choice(len(coeffs), 16, replace=False):
        ref = oracle.precondition(coeffs[i], 53).eval(points[i])
        sl = slice(offs[i], offs[i + 1])
        worst = max(worst, float(oracle.scaled_error(mm[sl], ee[sl], ref["m"], ref["e"], ref["dwin_m"],
                                                     ref["dwin_e"]).max()))
    # the same batch with FP32 plans at p = 24 (plain and compensated blocks)
    # beside FP64 arithmetic at p = 24
    fp32_rows = {}
    for label, fp32, comp in (("fp32_p24", True, False), ("fp32_compensated_p24", True, True),
                              ("fp64_arith_p24", False, False)):
        pl24 = fpe.precondition_batched(cdev, 24, fp32=fp32, compensated=comp)
        b24 = fpe.Batch(pl24, offs)
        o24 = (torch.empty(n, dtype=torch.complex128, device=dev), torch.empty(n, dtype=torch.int64, device=dev))
        b24.eval(z, out=o24)
        torch.cuda.synchronize()
        ms24 = timed(lambda: b24.eval(z, out=o24), steps)
        m24, e24 = o24[0].cpu().numpy(), o24[1].cpu().numpy()
        w24 = 0.0
        for i in np.random.default_rng(12350).choice(len(coeffs), 8, replace=False):
            ref = oracle.precondition(coeffs[i], 24).eval(points[i])
            sl = slice(offs[i], offs[i + 1])
            w24 = max(w24, float(oracle.scaled_error(m24[sl], e24[sl], ref["m"], ref["e"], ref["dwin_m"],
                                                     ref["dwin_e"]).max()))
        fp32_rows[label] = {"ms": ms24, "value": n / (ms24 * 1e-3), "max_scaled_err_8_polys": w24}
        log(f"  batch {label}: {ms24:.3f} ms, max scaled error (8 polynomials) {w24:.2e}")
        del b24, pl24
    log(f"batch of {len(plans)} polynomials, {n} points: eager {eager_ms:.3f} ms, graph replay {graph_ms:.3f} ms, "
        f"per-polynomial loop {loop_ms:.1f} ms (chunk {chunk}); preconditioning {pre_ms:.1f} ms batched, "
        f"{pre_loop_ms:.0f} ms one at a time; "
        f"max scaled error (16 polynomials) {worst:.2e}; {kept} kept terms, window kernel {win_ms:.3f} ms "
        f"({8 * kept / (win_ms * 1e-3) / 1e12:.2f} TFLOP/s in the kept terms' FMAs)")
    return {"workload": "batched_4096", "n_poly": len(plans), "n_points": n,
            "coefficients": int(sum(len(c) for c in coeffs)), "unit": "evaluations/s", "chunk": chunk,
            "eager": {"ms": eager_ms, "value": n / (eager_ms * 1e-3)},
            "graph_replay": {"ms": graph_ms, "value": n / (graph_ms * 1e-3)},
            "per_polynomial_loop": {"ms": loop_ms, "value": n / (loop_ms * 1e-3)},
            "precondition_ms": pre_ms, "precondition_one_at_a_time_ms": pre_loop_ms,
            "max_scaled_err_16_polys": worst,
            "p24": fp32_rows,
            "kept_terms": kept, "window_kernel_ms": win_ms,
            "window_tflops_kept_terms": 8 * kept / (win_ms * 1e-3) / 1e12}


def two_stream_leg(plan, z, out, n, torch, warmup: int, steps: int) -> dict:
    """The same evaluations queued alternately on two streams (the plan keeps
    one workspace per stream): one evaluation's latency-bound sort kernels and
    the window kernel's tail overlap the other's work."""
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    souts = []
    for s in streams:
        with torch.cuda.stream(s):
            souts.append((torch.empty_like(out[0]), torch.empty_like(out[1])))
    cur = torch.cuda.current_stream()

    def run(k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        for s in streams:
            s.wait_event(e0)
        for i in range(k):
            plan.eval(z, out=souts[i % 2], stream=streams[i % 2])
        for s in streams:
            cur.wait_stream(s)
        e1.record(cur)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    run(max(warmup, 2))
    ms = run(steps) / steps
    same = all(torch.equal(o[0], out[0]) and torch.equal(o[1], out[1]) for o in souts)
    log(f"two streams: {ms:.3f} ms per evaluation ({n / (ms * 1e-3):.3e} evals/s), results identical: {same}")
    return {"value": n / (ms * 1e-3), "unit": "evaluations/s", "ms_per_step": ms, "streams": 2, "steps": steps,
            "results_identical": bool(same)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform_d1e6")
    ap.add_argument("--horner-steps", type=int, default=2)
    ap.add_argument("--no-horner", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-f3", action="store_true", help="skip the derivative / adjoint / Newton leg")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 (p = 24) leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the 4096-polynomial leg")
    ap.add_argument("--no-wide", action="store_true", help="skip the d = 2^20 wide-range leg (dense and sparse)")
    ap.add_argument("--fp32-blocks", choices=["off", "plain", "compensated"], default="off",
                    help="headline at p = 24 with FP32 window blocks (plain or compensated) instead of FP64 at "
                         "p = 53 (for counter runs of the FP32 path)")
    ap.add_argument("--no-two-streams", action="store_true",
                    help="skip the two-stream measurement (kernel-statistics runs: no overlapping launches)")
    ap.add_argument("--chunk", type=int, default=0,
                    help="chunk length of the tiles (0: autotuned before the timed steps)")
    ap.add_argument("--cpu-sample", type=int, default=131072,
                    help="points of the double-double oracle timing")
    ap.add_argument("--check-sample", type=int, default=1000)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (a kernel of known traffic, "
                         "to scale hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only: the library evaluates on a single MI355X "
              f"(--gpus {args.gpus}, WORLD_SIZE {world} requested); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2211_06320_amd as fpe
    from paper_2211_06320_amd import workloads

    dev = torch.device("cuda:0")
    wl = workloads.workload(args.workload)
    n, d = len(wl.points), wl.degree
    log(f"workload {wl.name}: d={d}, n={n}")
    coeffs = torch.from_numpy(wl.coeffs).to(dev)
    z = torch.from_numpy(wl.points).to(dev)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    fp32 = args.fp32_blocks != "off"
    p_bits = 24 if fp32 else wl.p_bits
    plan = fpe.precondition(coeffs, p_bits, fp32=fp32, compensated=args.fp32_blocks == "compensated")
    torch.cuda.synchronize()
    pre_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info()
    log(f"precondition {pre_ms:.1f} ms: {info}")

    # the tile schedule: the autotuner's chunk length (or a given one), chosen
    # before the timed region like the preconditioning
    if args.chunk:
        plan.set_chunk(args.chunk)
        chunk = args.chunk
    else:
        chunk = plan.autotune(z)
    log(f"chunk length {chunk}")
    # one untimed pass for the algorithmic work counts (counted on the host
    # after the timed steps, so that the GPU does not idle between the warm-up
    # and the timed steps)
    m, e, terms, window = plan.eval(z, terms=True, window=True)
    out = (torch.empty(n, dtype=torch.complex128, device=dev), torch.empty(n, dtype=torch.int64, device=dev))

    for _ in range(args.warmup):
        plan.eval(z, out=out)
    torch.cuda.synchronize()
    if args.copy_calibration > 0:
        nb = args.copy_calibration << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nb} bytes device to device")
        del src, dst
    # the timed steps: K evaluations between two events, nothing else on the
    # stream (the headline value and ms_per_step)
    t0ev, t1ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0ev.record()
    for _ in range(args.steps):
        plan.eval(z, out=out)
    t1ev.record()
    torch.cuda.synchronize()
    total_ms = t0ev.elapsed_time(t1ev)
    # K more steps, instrumented: an event between consecutive steps (the step
    # durations, for the median) and the window kernel timed with an event pair
    # on every PROFILE_EVERY-th step (each pair adds a few microseconds of
    # stream serialisation, so these steps run slower than the timed ones)
    fpe.profile_read()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    evs[0].record()
    for i in range(args.steps):
        fpe.profile_enable(i % PROFILE_EVERY == 0)
        plan.eval(z, out=out)
        evs[i + 1].record()
    torch.cuda.synchronize()
    fpe.profile_enable(False)
    step_ms = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
    median_ms = step_ms[len(step_ms) // 2] if len(step_ms) % 2 else 0.5 * (step_ms[len(step_ms) // 2 - 1] +
                                                                             step_ms[len(step_ms) // 2])
    win_ms, launches = fpe.profile_read()
    ms_per_step = total_ms / args.steps
    value = n / (ms_per_step * 1e-3)
    win_avg_ms = win_ms / max(launches, 1)
    terms_np, window_np = terms.cpu().numpy(), window.cpu().numpy()
    flops = algorithmic_flops(terms_np, window_np)
    achieved = flops / (win_avg_ms * 1e-3) / 1e12
    # the committed counter summaries are for the FP64 window sums
    traffic = None if fp32 else recorded_traffic(wl.name, chunk)
    peak = FP32_VECTOR_PEAK_TFLOPS if fp32 else FP64_VECTOR_PEAK_TFLOPS
    log(f"eval {ms_per_step:.3f} ms/step ({value:.3e} evals/s); instrumented steps: median {median_ms:.3f} ms; "
        f"window kernel {win_avg_ms:.3f} ms, "
        f"{achieved:.2f} TFLOP/s algorithmic")

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "evaluations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_median": median_ms,
        "value_median": n / (median_ms * 1e-3),
        "median_from": "K further steps with an event after each (and the window kernel's event pairs)",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 blocks, f64 accumulation" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "d": d, "n_points": n, "p_bits": p_bits,
                   "fp32_blocks": args.fp32_blocks,
                   "coefficients": "Re, Im i.i.d. uniform[-1,1]", "points": "uniform on the Riemann sphere",
                   "parallelism": "single GPU", "chunk": chunk},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "kernel": "k_window", "kernel_ms": win_avg_ms,
                     "algorithmic_flops": flops, "kept_terms": int(terms_np.sum()),
                     "hbm_gbs": traffic / (win_avg_ms * 1e-3) / 1e9 if traffic else None,
                     "counters": None if fp32 else recorded_counters(wl.name, chunk),
                     "step_frac": flops / (ms_per_step * 1e-3) / 1e12 / peak},
        "precondition_ms": pre_ms,
        "mean_terms": float(terms_np.mean()),
    }

    # the same K evaluations queued alternately on two streams (the plan keeps
    # one workspace per stream): one evaluation's latency-bound sort kernels and
    # the window kernel's tail overlap the other's work; reported beside the
    # one-stream value, which stays the headline
    if not args.no_two_streams:
        res["two_streams"] = two_stream_leg(plan, z, out, n, torch, args.warmup, args.steps)

    # accuracy on a seeded sample, against the oracle's wide window sum
    import oracle
    mm, ee = out[0].cpu().numpy(), out[1].cpu().numpy()
    rng = np.random.default_rng(12345)
    idx = rng.choice(n, min(args.check_sample, n), replace=False)
    ref = oracle.precondition(wl.coeffs, 116).eval(wl.points[idx])
    err = oracle.scaled_error(mm[idx], ee[idx], ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"])
    res["max_scaled_err"] = float(err.max())
    res["check_sample"] = int(len(idx))
    log(f"max scaled error on {len(idx)} points: {err.max():.3e}")

    if not args.no_horner:
        hout = (torch.empty(n, dtype=torch.complex128, device=dev), torch.empty(n, dtype=torch.int64, device=dev))
        fpe.horner_eval(coeffs, z, out=hout)
        torch.cuda.synchronize()
        h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        h0.record()
        for _ in range(args.horner_steps):
            fpe.horner_eval(coeffs, z, out=hout)
        h1.record()
        torch.cuda.synchronize()
        hms = h0.elapsed_time(h1) / args.horner_steps
        hm, he = hout[0].cpu().numpy(), hout[1].cpu().numpy()
        herr = oracle.scaled_error(hm[idx], he[idx], ref["m"], ref["e"], ref["dwin_m"], ref["dwin_e"])
        res["horner_gpu"] = {"value": n / (hms * 1e-3), "unit": "evaluations/s", "ms_per_step": hms,
                             "max_scaled_err": float(herr.max()), "speedup_fpe": (n / (ms_per_step * 1e-3)) / (n / (hms * 1e-3))}
        log(f"horner {hms:.1f} ms/step, max scaled error {herr.max():.3e}")

    if not args.no_f3:
        res["adjoint_newton"] = adjoint_leg(fpe, workloads, torch, dev, args.steps)
    if not args.no_fp32:
        res["fp32_p24"] = fp32_leg(fpe, workloads, oracle, np, torch, dev, args.steps, args.check_sample)
    if not args.no_wide:
        res["wide_range"] = wide_leg(fpe, workloads, oracle, np, torch, dev, args.steps, args.check_sample)
    if not args.no_batched:
        res["batched"] = batched_leg(fpe, workloads, oracle, np, torch, dev, args.steps)

    if not args.no_cpu:
        # the oracle's plain-FP64 window sum (its plan in FP64, z^l by binary
        # powering, Horner's rule over the window) over every point, on the
        # host's threads (at most 16) and on one
        # thread; its double-double mode (the parity reference) on a sample
        threads = oracle.default_threads()
        cplan = oracle.precondition(wl.coeffs, wl.p_bits)
        t0 = time.perf_counter()
        cplan.eval_fp64(wl.points, nthreads=threads)
        dt = time.perf_counter() - t0
        t0 = time.perf_counter()
        cplan.eval_fp64(wl.points, nthreads=1)
        dt1 = time.perf_counter() - t0
        zs = wl.points[:args.cpu_sample]
        t0 = time.perf_counter()
        cplan.eval(zs, nthreads=threads)
        dtd = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": n / dt, "unit": "evaluations/s", "cores": threads, "kind": "oracle",
                               "sample": f"all {n} points of {wl.name}, p={wl.p_bits}: the oracle's plain-FP64 "
                                         f"window sum, {threads} threads, {dt:.2f} s wall",
                               "single_thread": {"value": n / dt1, "cores": 1, "seconds": dt1},
                               "double_double": {"value": len(zs) / dtd, "cores": threads, "points": len(zs),
                                                 "seconds": dtd}}
        log(f"cpu oracle (plain FP64) {n / dt:.3e} evals/s on {threads} threads, {n / dt1:.3e} on 1 thread; "
            f"double-double {len(zs) / dtd:.3e} evals/s on {threads} threads")

    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
