"""Benchmark harness of Sec. III: optimality gap, time-to-epsilon, and the
SBQA-versus-SBM comparison on the GPU library.

* optimality gap g = (E - E0) / |E0| of a returned energy E against the best
  known (or planted) energy E0;
* time-to-epsilon TT_eps = tau log(1 - p_target) / log(1 - p_success), tau the
  mean time of one solve and p_success the fraction of solves whose returned
  solution is within eps of E0;
* SBM baseline: the same number of trajectories evolved without the Trotter
  ring (R = 1, J_perp = 0), which reduces Eqs. 6-7 to the simulated
  bifurcation machine of Eq. 3.

A "solve" is one call of the library with `runs` repetitions of R replicas
(auto-tuned beta, alpha per repetition, Sec. II.B) that returns the best
solution over all of them; its time is the wall time of stepping and readout
with the instance already on the device (inputs resident in HBM).
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import _abi as sb


def optimality_gap(E, E0):
    """g = (E - E0) / |E0| (Sec. III); E0 must be non-zero."""
    return (np.asarray(E, dtype=np.float64) - E0) / abs(E0)


def tt_epsilon(tau, p_success, p_target=0.99):
    """Time-to-epsilon of a solver whose solves take tau and reach the target
    with probability p_success. One solve suffices when p_success >= p_target;
    inf when no solve reached it."""
    if not 0.0 < p_target < 1.0:
        raise ValueError("p_target must be in (0, 1)")
    if p_success <= 0.0:
        return math.inf
    if p_success >= p_target:
        return float(tau)
    return float(tau) * math.log(1.0 - p_target) / math.log(1.0 - p_success)


def solve(J=None, csr=None, h=None, R=16, runs=8, steps=1000, seed=0, sbm=False, **kw):
    """One solve. SBQA: `runs` repetitions of R replicas in a ring with the
    paper's J_perp schedule (Eq. 5, auto-tuned beta, alpha). SBM: the same
    R*runs trajectories with R = 1 and J_perp = 0. Returns a dict with the
    best energy over all repetitions, the per-repetition best energies and
    the solve time in seconds (stepping and readout)."""
    if sbm:
        R, runs = 1, R * runs
        kw = dict(kw, jp_kind=sb.JP_LINEAR, jp_start=0.0, jp_end=0.0)
    else:
        kw.setdefault("jp_kind", sb.JP_PAPER)
    ctx = sb.sbqa_create(J=J, csr=csr, h=h, R=R, runs=runs, steps=steps, seed=seed, **kw)
    try:
        sb.sbqa_sync(ctx)
        t0 = time.perf_counter()
        sb.sbqa_step(ctx, steps)
        E, spins = sb.sbqa_best(ctx)
        t = time.perf_counter() - t0
    finally:
        sb.sbqa_destroy(ctx)
    return {"best": float(np.min(E)), "per_run": E, "spins": spins[int(np.argmin(E))], "seconds": t}


def tte_study(E0, eps, steps_list, seeds, J=None, csr=None, h=None, R=16, runs=8, sbm=False,
              p_target=0.99, **kw):
    """[TT_eps] for each number of steps and each target gap in `eps`, over
    solves with the given seeds; the best over the step counts is reported
    per target, as the median TT_eps is minimised over steps in Sec. III."""
    eps = np.atleast_1d(np.asarray(eps, dtype=np.float64))
    rows = []
    for S in steps_list:
        res = [solve(J=J, csr=csr, h=h, R=R, runs=runs, steps=S, seed=sd, sbm=sbm, **kw) for sd in seeds]
        gaps = optimality_gap([r["best"] for r in res], E0)
        tau = float(np.mean([r["seconds"] for r in res]))
        p = [(float(np.mean(gaps <= e))) for e in eps]
        rows.append({"steps": int(S), "tau_s": tau, "gap_mean": float(np.mean(gaps)),
                     "gap_min": float(np.min(gaps)), "p_success": p,
                     "tte_s": [tt_epsilon(tau, pe, p_target) for pe in p]})
    best = []
    for q in range(eps.size):
        t = [r["tte_s"][q] for r in rows]
        k = int(np.argmin(t))
        best.append({"eps": float(eps[q]), "tte_s": t[k], "steps": rows[k]["steps"]})
    return {"sbm": bool(sbm), "rows": rows, "best": best}


def step_time(J=None, csr=None, h=None, R=16, runs=8, steps=200, sbm=False, **kw):
    """Device time per step (HIP events around `steps` steps on the
    context's stream, after a warm-up step), SBQA or SBM with the same number
    of trajectories."""
    import torch
    if sbm:
        R, runs = 1, R * runs
        kw = dict(kw, jp_kind=sb.JP_LINEAR, jp_start=0.0, jp_end=0.0)
    st = torch.cuda.Stream()
    ctx = sb.sbqa_create(J=J, csr=csr, h=h, R=R, runs=runs, steps=steps + 1, **kw)
    try:
        sb.sbqa_set_stream(ctx, st)
        sb.sbqa_step(ctx, 1)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        sb.sbqa_step(ctx, steps)
        b.record(st)
        b.synchronize()
        return a.elapsed_time(b) * 1e-3 / steps
    finally:
        sb.sbqa_destroy(ctx)
