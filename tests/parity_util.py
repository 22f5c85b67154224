"""Node-by-node comparison of the GPU encoder's quadtree with the oracle's.

Rules (per node, in the oracle's iteration order):
* atom tie: the oracle's relative gap between its two best distinct atoms is
  below 1e-6 and the GPU chose another atom whose oracle correlation is within
  that window; the rest of the node and its subtree are then excluded;
* stop tie: the oracle's squared residual norm is within 1e-6 ||y||^2 of
  eps_N^2 where the two sides took a different stop or split decision;
  the node's subtree is excluded;
* everything else must be identical: visited node set, per-node atom index
  sequence, number of iterations and split decision;
* coefficients: |c_gpu - c_orc| / max(|c_orc|, 1e-3 ||y||) <= coef_tol.  For
  |c_orc| >= 1e-3 ||y|| this is the plain relative error; below it the bound
  is absolute, coef_tol * 1e-3 ||y||: late coefficients of a pursuit are small
  and carry the FP32 residual's rounding, about u32 ||y|| sqrt(t) / N.  The
  report counts the floored coefficients and gives the largest unfloored
  relative error and the largest error over ||y||.

The oracle side of large cases runs in a pool of worker processes (spawned,
not forked, so that no GPU state is copied), one top-level block per task:
top-level quadtrees are independent, so this is the same computation.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

from oracle import aqmp_oracle as O

GAP_TIE = 1e-6
STOP_TIE = 1e-6


@dataclass
class Report:
    nodes: int = 0
    iters: int = 0
    atom_ties: int = 0
    stop_ties: int = 0
    excluded_nodes: int = 0
    max_coef_err: float = 0.0
    max_coef_err_unfloored: float = 0.0
    max_coef_err_over_ynorm: float = 0.0
    floored_coefs: int = 0
    failures: list = field(default_factory=list)

    def ok(self) -> bool:
        return not self.failures

    def summary(self) -> str:
        return (f"nodes={self.nodes} iters={self.iters} atom_ties={self.atom_ties} stop_ties={self.stop_ties} "
                f"excluded={self.excluded_nodes} max_coef_err={self.max_coef_err:.3e} "
                f"unfloored={self.max_coef_err_unfloored:.3e} over_ynorm={self.max_coef_err_over_ynorm:.3e} "
                f"floored={self.floored_coefs} failures={len(self.failures)} {self.failures[:5]}")


def gpu_nodes_by_key(exp, job: int) -> dict:
    """{(x0, y0, n): (idx list, coef list, split flag, resid_sq)} of one job."""
    out = {}
    lv = exp.leaves
    sel = np.nonzero(lv["job"] == job)[0]
    for r in sel:
        rec = lv[r]
        o, na = int(rec["atom_off"]), int(rec["n_atoms"])
        out[(int(rec["x0"]), int(rec["y0"]), int(rec["n"]))] = (
            exp.atom_idx[o:o + na].tolist(), exp.coef[o:o + na].tolist(), bool(rec["flags"] & 1),
            float(rec["resid_sq"]))
    return out


def _is_near_tie_member(img, nd: O.Node, t: int, gpu_atom: int, families: int, solver: str = "mp") -> bool:
    """Replays the oracle's pursuit on the node up to step t and checks that the
    GPU's atom is within the 1e-6 relative window of the best |correlation|
    (MP: the rank-1 updates; OMP: the least-squares residual of the first t
    atoms)."""
    dic = O.get_dict(nd.n, families)
    img = O.pad_edge(np.asarray(img, dtype=np.float64), 64)   # nodes may lie in the padding
    y = O.unravel(img[nd.y0:nd.y0 + nd.n, nd.x0:nd.x0 + nd.n]).astype(np.float64)
    if solver == "omp":
        sel = list(nd.mp.idx[:t])
        r = y - dic.D[:, sel] @ np.linalg.lstsq(dic.D[:, sel], y, rcond=None)[0] if sel else y.copy()
    else:
        r = y.copy()
        for i, c in zip(nd.mp.idx[:t], nd.mp.coef[:t]):
            r = r - c * dic.D[:, i]
    c = np.abs(dic.Dt @ r)
    return c[gpu_atom] >= c.max() * (1.0 - GAP_TIE)


def compare_job(img, onodes: list, gpu: dict, coef_tol: float, n_max: int, families: int = O.DCT | O.HAAR,
                rep: Report | None = None, solver: str = "mp") -> Report:
    """Compares the oracle's visited nodes (one job; possibly a subset of top
    blocks) with the GPU's nodes of that job."""
    rep = rep or Report()
    okeys = {(nd.x0, nd.y0, nd.n): nd for nd in onodes}
    excluded: list[tuple[int, int, int]] = []

    def inside(key) -> bool:
        x, y, n = key
        for (ex, ey, en) in excluded:
            if ex <= x and x + n <= ex + en and ey <= y and y + n <= ey + en:
                return True
        return False

    for nd in onodes:            # depth-first order: parents before children
        key = (nd.x0, nd.y0, nd.n)
        if inside(key):
            rep.excluded_nodes += 1
            continue
        if key not in gpu:
            rep.failures.append(("missing node on GPU", key))
            continue
        g_idx, g_coef, g_split, g_e = gpu[key]
        rep.nodes += 1
        ynorm = float(np.sqrt(nd.norm2))
        o_idx, o_coef = nd.mp.idx, nd.mp.coef
        diverged = False
        for t in range(min(len(o_idx), len(g_idx))):
            if o_idx[t] != g_idx[t]:
                if nd.mp.gap[t] < GAP_TIE and _is_near_tie_member(img, nd, t, g_idx[t], families, solver):
                    rep.atom_ties += 1
                    excluded.append(key)
                else:
                    rep.failures.append(("atom mismatch", key, t, o_idx[t], g_idx[t], nd.mp.gap[t]))
                diverged = True
                break
            rep.iters += 1
            den = max(abs(o_coef[t]), 1e-3 * ynorm)
            err = abs(g_coef[t] - o_coef[t]) / den
            rep.max_coef_err = max(rep.max_coef_err, err)
            if abs(o_coef[t]) < 1e-3 * ynorm:
                rep.floored_coefs += 1
            if ynorm > 0:
                rep.max_coef_err_over_ynorm = max(rep.max_coef_err_over_ynorm, abs(g_coef[t] - o_coef[t]) / ynorm)
            if o_coef[t] != 0:
                rep.max_coef_err_unfloored = max(rep.max_coef_err_unfloored,
                                                 abs(g_coef[t] - o_coef[t]) / abs(o_coef[t]))
            if err > coef_tol:
                rep.failures.append(("coef", key, t, o_coef[t], g_coef[t], err))
        if diverged:
            continue
        stop_tie_window = STOP_TIE * nd.norm2
        if len(o_idx) != len(g_idx):
            t = min(len(o_idx), len(g_idx))
            if abs(nd.mp.e[t] - nd.eps2) <= stop_tie_window:
                rep.stop_ties += 1
                excluded.append(key)
            else:
                rep.failures.append(("iteration count", key, len(o_idx), len(g_idx)))
            continue
        if g_split != nd.split:
            if abs(nd.mp.e_final - nd.eps2) <= stop_tie_window:
                rep.stop_ties += 1
                excluded.append(key)
            else:
                rep.failures.append(("split", key, nd.split, g_split, nd.mp.e_final, nd.eps2))
            continue
    # GPU nodes inside the compared region that the oracle never visited
    tops = {(nd.x0, nd.y0) for nd in onodes if nd.n == n_max}
    for key in gpu:
        x, y, n = key
        if (x - x % n_max, y - y % n_max) in tops and key not in okeys and not inside(key):
            rep.failures.append(("extra node on GPU", key))
    return rep


def decode_region(img_shape, onodes, families=O.DCT | O.HAAR):
    return O.decode(onodes, img_shape[0], img_shape[1], families)


def _oracle_block_task(task):
    crop, x0, y0, params = task
    p = O.Params.from_dict(params)
    nodes = O.encode_block(crop, p, 0, 0, p.n_max)
    for nd in nodes:
        nd.x0 += x0
        nd.y0 += y0
    return nodes


def _pool_init():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def pool_size() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_jobs_parallel(jobs, procs: int | None = None, timeout: float = 900.0) -> list:
    """The oracle's visited nodes of several jobs, each given as
    (plane, params dict, top-level blocks or None for all), in the order
    ``O.encode_channel`` gives them.  One task per top-level block (the crop
    of the edge-padded plane), run in spawned worker processes with BLAS on
    one thread."""
    import multiprocessing as mp
    tasks, spans = [], []
    for img, params, blocks in jobs:
        p = O.Params.from_dict(params)
        pad = O.pad_edge(np.asarray(img, dtype=np.float64), p.n_max)
        if blocks is None:
            blocks = O.top_blocks(pad.shape[0], pad.shape[1], p.n_max)
        t0 = len(tasks)
        for (x0, y0) in blocks:
            tasks.append((pad[y0:y0 + p.n_max, x0:x0 + p.n_max].copy(), x0, y0, dict(params)))
        spans.append((t0, len(tasks)))
    procs = procs or pool_size()
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(procs, initializer=_pool_init) as pool:
            # a bounded wait: a pool whose workers cannot start fails instead of hanging
            res = pool.map_async(_oracle_block_task, tasks, chunksize=1).get(timeout)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return [[nd for r in res[a:b] for nd in r] for a, b in spans]


def psnr_region(ref, rec, blocks, n):
    """PSNR over the union of the given top-level blocks (peak 1)."""
    se, cnt = 0.0, 0
    for (x0, y0) in blocks:
        d = ref[y0:y0 + n, x0:x0 + n] - rec[y0:y0 + n, x0:x0 + n]
        se += float(np.sum(d * d))
        cnt += d.size
    mse = se / cnt
    return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)
