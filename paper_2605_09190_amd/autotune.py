"""Autotuner for the batched encoder: correlation kernel per block size, the
node-tile range of the generated-atom correlation, the form of the N = 16
level, and the schedule.

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
3. where the generated-atom kernel runs (N = 32, 64), its node-tile range
   [lo, hi] (the kernel picks the node-tile width 32 MB, lo <= MB <= hi, from
   the active-node count of each step) is timed over a few candidate ranges
   under the same rule against the library's range;
4. the schedules are then timed as graph replays with the chosen kernels,
   under the same rule against the batched schedule.

The choices change speed only: every kernel family computes the same keys,
every node-tile width the same per-node keys, and every schedule the same
nodes.  With ``cache`` (a JSON file path) a result is stored under a key made
of the workload's shapes and parameters, the device name and a hash of the
library's kernel sources, and reused when the same key comes again.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

# Kernel families worth timing per block size (the others map onto these).
CANDIDATES = {64: (6, 2), 32: (6, 2), 16: (2, 3)}
DEFAULT = {64: 6, 32: 6, 16: 2}
# Node-tile ranges (lo, hi) of the generated-atom kernel worth timing.
TILE_CANDIDATES = {64: ((3, 7), (4, 7), (5, 7), (2, 7), (3, 5)), 32: ((1, 7), (2, 7), (3, 7), (1, 4), (2, 5))}
DEFAULT_TILE = {64: (3, 7), 32: (1, 7)}
GEN_VARIANT = 6
CACHE_VERSION = 1


def source_hash() -> str:
    """SHA-256 over the library's kernel and host sources (the built library
    when the sources are not next to it)."""
    here = os.path.dirname(os.path.abspath(__file__))
    csrc = os.path.join(here, "csrc")
    h = hashlib.sha256()
    if os.path.isdir(csrc):
        for name in sorted(os.listdir(csrc)):
            if name.endswith((".hip", ".h")):
                with open(os.path.join(csrc, name), "rb") as f:
                    h.update(name.encode() + b"\0" + f.read())
    else:
        with open(os.path.join(here, "libaqmp.so"), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def cache_key(images, params, jobs, device: str, src: str) -> str:
    """The workload's shapes, sample types, parameters and jobs, the device and
    the source hash, as one canonical string."""
    shapes = [[int(t.shape[0]), int(t.shape[1]), str(t.dtype)] for t in images]
    prm = [{k: (v if not isinstance(v, dict) else {str(a): b for a, b in sorted(v.items())})
            for k, v in sorted(p.items())} for p in params]
    return json.dumps(dict(v=CACHE_VERSION, shapes=shapes, params=prm, jobs=[list(map(int, j)) for j in jobs],
                           device=device, src=src), sort_keys=True)


def cache_load(path: str, key: str):
    try:
        with open(path) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def cache_store(path: str, key: str, entry: dict) -> None:
    data = {}
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data[key] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _options_to_json(opt: dict) -> dict:
    return dict(corr_variant_levels={str(k): v for k, v in opt["corr_variant_levels"].items()},
                corr_tile_levels={str(k): list(v) for k, v in opt["corr_tile_levels"].items()},
                stepwise=opt["stepwise"], schedule=opt["schedule"])


def _options_from_json(d: dict) -> dict:
    return dict(corr_variant_levels={int(k): int(v) for k, v in d["corr_variant_levels"].items()},
                corr_tile_levels={int(k): tuple(v) for k, v in d["corr_tile_levels"].items()},
                stepwise=bool(d["stepwise"]), schedule=int(d["schedule"]))


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
         schedules: bool = True, cache: str | None = None) -> dict:
    """Measures the candidates on this workload (BF16 form) and returns
    ``dict(options=..., measured=...)``; ``options`` are keyword arguments for
    ``Code`` (``corr_variant_levels``, ``corr_tile_levels``, ``stepwise``,
    ``schedule``).  With ``cache``, a stored result for the same key is
    returned instead (``cached`` True), and a new one is stored."""
    key = None
    if cache:
        import torch
        key = cache_key(images, params, jobs, torch.cuda.get_device_name(), source_hash())
        hit = cache_load(cache, key)
        if hit is not None:
            return dict(options=_options_from_json(hit["options"]), measured=hit["measured"], cached=True)
    res = _tune(A, dic, images, params, jobs, reps, steps, margin, schedules)
    if cache:
        cache_store(cache, key, dict(options=_options_to_json(res["options"]), measured=res["measured"],
                                     created=time.time()))
    res["cached"] = False
    return res


def _tune(A, dic, images, params, jobs, reps, steps, margin, schedules) -> dict:
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
    # node-tile range of the generated-atom kernel, where it runs
    per_tile = {}
    measured["tile_ms"] = {}
    for n in (64, 32):
        if n not in corr or per_n.get(n, DEFAULT[n]) != GEN_VARIANT:
            continue
        lg = n.bit_length() - 1
        times = {}
        for rng in TILE_CANDIDATES[n]:
            c_ms, _ = _timed(A, dic, images, params, jobs, reps, corr_variant_levels={**per_n, n: GEN_VARIANT},
                             stepwise=stepwise, corr_tile_levels={n: rng})
            if c_ms[lg] > 0:
                times[rng] = c_ms[lg]
        measured["tile_ms"][str(n)] = {f"{lo}-{hi}": round(t, 4) for (lo, hi), t in times.items()}
        rng = choose(times, DEFAULT_TILE[n], margin)
        if rng != DEFAULT_TILE[n]:
            per_tile[n] = rng
    schedule = A.SCHED_BATCHED
    if schedules and len(jobs) > 1:
        sched_ms = {}
        for s in (A.SCHED_BATCHED, A.SCHED_CONCURRENT):
            sched_ms[s] = _replay_ms(A, dic, images, params, jobs, steps, schedule=s, stepwise=stepwise,
                                     corr_variant_levels=per_n, corr_tile_levels=per_tile)
        measured["schedule_ms"] = {("batched" if s == A.SCHED_BATCHED else "concurrent"): round(t, 4)
                                   for s, t in sched_ms.items()}
        schedule = choose(sched_ms, A.SCHED_BATCHED, margin)
    return dict(options=dict(corr_variant_levels=per_n, corr_tile_levels=per_tile, stepwise=stepwise,
                             schedule=schedule), measured=measured)
