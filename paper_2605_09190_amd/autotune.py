"""Autotuner for the batched encoder: correlation kernel per block size, the
form of the N = 16 level, and the schedule.

The library offers several BF16 correlation kernel families that produce
bit-identical keys (``aqmp_options.corr_variant``, per block size through
``corr_variant_levels``), two forms of the N = 16 level of the BF16 form (one
launch for the whole level, or a correlation and a select launch per MP
step) and three schedules.  Which is fastest depends on how many nodes each
level holds at each step, so the tuner measures them on the caller's own
workload:

1. every kernel family is run once per candidate with the library's
   per-launch HIP events (``aqmp_code_timing``): per block size N >= 32 the
   correlation time of the level, per N = 16 the whole level's time (step by
   step with that family, or as one launch), each the best of ``reps``
   encodes;
2. a candidate replaces the library default of a level only when it is
   faster by more than ``margin`` (so that timing noise does not flip it);
3. the schedules are then timed as graph replays with the chosen kernels,
   under the same rule against the batched schedule.

The choices change speed only: every kernel family computes the same keys,
and every schedule the same nodes.
"""
from __future__ import annotations

import time

# Kernel families worth timing per block size (the others map onto these).
CANDIDATES = {64: (6, 5, 1, 2, 3), 32: (6, 5, 1, 2, 3, 4), 16: (2, 5, 1, 3, 4)}
DEFAULT = {64: 6, 32: 6, 16: 2}


def choose(times: dict, default, margin: float):
    """The key of the smallest time if it beats ``default``'s by more than
    ``margin`` (relative), else ``default``.  Ties keep the earlier key."""
    if not times:
        return default
    best = min(times, key=lambda k: times[k])
    if default in times and times[best] >= times[default] * (1.0 - margin):
        return default
    return best


def _timed(A, dic, images, params, jobs, reps, **kw):
    """Per-level correlation and level times (ms), best of ``reps`` encodes."""
    import torch
    code = A.Code(dic, images, params, jobs, precision=A.PREC_BF16, schedule=A.SCHED_BATCHED, timing=True, **kw)
    try:
        best_corr = [float("inf")] * 7
        best_level = [float("inf")] * 7
        for _ in range(reps):
            code.reencode(images)
            torch.cuda.synchronize()
            t = code.timing()
            best_corr = [min(a, b) for a, b in zip(best_corr, t["corr_ms"])]
            best_level = [min(a, b) for a, b in zip(best_level, t["level_ms"])]
        return best_corr, best_level
    finally:
        code.free()


def _replay_ms(A, dic, images, params, jobs, steps, **kw):
    import torch
    code = A.Code(dic, images, params, jobs, precision=A.PREC_BF16, **kw)
    try:
        code.reencode(images)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            code.reencode(images)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3
    finally:
        code.free()


def tune(A, dic, images, params, jobs, reps: int = 3, steps: int = 5, margin: float = 0.03,
         schedules: bool = True) -> dict:
    """Measures the candidates on this workload (BF16 form) and returns
    ``dict(options=..., measured=...)``; ``options`` are keyword arguments for
    ``Code`` (``corr_variant_levels``, ``stepwise``, ``schedule``)."""
    levels = sorted({1 << l for p in params for l in range(p["n_min"].bit_length() - 1, p["n_max"].bit_length())},
                    reverse=True)
    measured = {"corr_ms": {}, "level16_ms": {}, "schedule_ms": {}}
    corr = {n: {} for n in (64, 32) if n in levels}
    lvl16 = {}
    for v in sorted({v for n in CANDIDATES for v in CANDIDATES[n]}):
        c_ms, l_ms = _timed(A, dic, images, params, jobs, reps, corr_variant=v, stepwise=True)
        for n in corr:
            if v in CANDIDATES[n] and c_ms[n.bit_length() - 1] > 0:
                corr[n][v] = c_ms[n.bit_length() - 1]
        if 16 in levels and v in CANDIDATES[16] and l_ms[4] > 0:
            lvl16[("step", v)] = l_ms[4]
    if 16 in levels:
        _, l_ms = _timed(A, dic, images, params, jobs, reps, stepwise=False)
        if l_ms[4] > 0:
            lvl16[("whole", 0)] = l_ms[4]
    per_n = {}
    for n, times in corr.items():
        measured["corr_ms"][str(n)] = {str(v): round(t, 4) for v, t in times.items()}
        v = choose(times, DEFAULT[n], margin)
        if v != DEFAULT[n]:
            per_n[n] = v
    stepwise = False
    if lvl16:
        measured["level16_ms"] = {f"{k[0]}{k[1] or ''}": round(t, 4) for k, t in lvl16.items()}
        form, v = choose(lvl16, ("whole", 0), margin)
        if form == "step":
            stepwise = True
            if v != DEFAULT[16]:
                per_n[16] = v
    schedule = A.SCHED_BATCHED
    if schedules and len(jobs) > 1:
        sched_ms = {}
        for s in (A.SCHED_BATCHED, A.SCHED_CONCURRENT):
            sched_ms[s] = _replay_ms(A, dic, images, params, jobs, steps, schedule=s, stepwise=stepwise,
                                     corr_variant_levels=per_n)
        measured["schedule_ms"] = {("batched" if s == A.SCHED_BATCHED else "concurrent"): round(t, 4)
                                   for s, t in sched_ms.items()}
        schedule = choose(sched_ms, A.SCHED_BATCHED, margin)
    return dict(options=dict(corr_variant_levels=per_n, stepwise=stepwise, schedule=schedule), measured=measured)
