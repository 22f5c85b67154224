"""Hyperparameter search over the batched encoder (Section 2.4 and Section 3).

The paper tunes AQMP's hyperparameters with the Tree-structured Parzen
Estimator (and compares a random sampler), maximising SSIM and the
compression rate together and reporting Pareto fronts.  This module is that
loop, with the trials of a round encoded together: every (image, trial) pair
is one job of one batched encode, one captured graph on the GPU.  Each trial
is then scored by the SSIM of its reconstruction (GPU kernel) and by the
compression rate of its DEFLATE-compressed bitstream.

Search space (the hyperparameters this encoder takes, Section 2.4):
``tol`` (RMS tolerance, log-uniform), ``max_atoms`` (k, integer),
``n_min`` and ``n_max`` (categorical powers of two).

TPE (Bergstra et al.; the multi-objective form splits by non-dominated
rank): observations are split into a good fraction gamma and the rest; each
parameter gets a Parzen density for both groups (Gaussian kernels in the
parameter's own scale plus a uniform prior component; smoothed frequencies
for categorical values); candidates drawn from the good density are ranked
by log l(x) - log g(x), and a round takes the best distinct ones.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SPACE = dict(
    tol=("log", 0.005, 0.06),
    max_atoms=("int", 8, 64),
    n_min=("cat", (4, 8)),
    n_max=("cat", (32, 64)),
)


# ---------------------------------------------------------------------------
# Pareto utilities (both objectives maximised)
# ---------------------------------------------------------------------------

def dominates(a, b) -> bool:
    return all(x >= y for x, y in zip(a, b)) and any(x > y for x, y in zip(a, b))


def nondominated_ranks(objs) -> np.ndarray:
    """Rank 0 for the non-dominated points, 1 for those dominated only by
    rank-0 points, and so on."""
    n = len(objs)
    ranks = np.full(n, -1)
    left = set(range(n))
    r = 0
    while left:
        front = [i for i in left if not any(dominates(objs[j], objs[i]) for j in left if j != i)]
        for i in front:
            ranks[i] = r
        left -= set(front)
        r += 1
    return ranks


def pareto_front(objs) -> list[int]:
    ranks = nondominated_ranks(objs)
    return [i for i in range(len(objs)) if ranks[i] == 0]


def hypervolume_2d(objs, ref=(0.0, 0.0)) -> float:
    """Area dominated by the points and bounded below by ``ref``."""
    pts = sorted({(float(a), float(b)) for a, b in objs if a > ref[0] and b > ref[1]}, key=lambda p: -p[0])
    area, best_b = 0.0, ref[1]
    for a, b in pts:
        if b > best_b:
            area += (a - ref[0]) * (b - best_b)
            best_b = b
    return area


# ---------------------------------------------------------------------------
# Samplers
# ---------------------------------------------------------------------------

def _to_unit(name, v):
    kind = SPACE[name][0]
    if kind == "log":
        lo, hi = math.log(SPACE[name][1]), math.log(SPACE[name][2])
        return (math.log(v) - lo) / (hi - lo)
    lo, hi = SPACE[name][1] - 0.5, SPACE[name][2] + 0.5
    return (v - lo) / (hi - lo)


def _from_unit(name, u):
    kind = SPACE[name][0]
    u = min(max(u, 0.0), 1.0)
    if kind == "log":
        lo, hi = math.log(SPACE[name][1]), math.log(SPACE[name][2])
        return float(math.exp(lo + u * (hi - lo)))
    lo, hi = SPACE[name][1] - 0.5, SPACE[name][2] + 0.5
    return int(min(max(round(lo + u * (hi - lo)), SPACE[name][1]), SPACE[name][2]))


class Parzen:
    """Parzen density on [0, 1] (Gaussian kernels at the points plus one
    uniform prior component, truncated to the interval)."""

    def __init__(self, pts):
        self.mu = np.asarray(sorted(pts), dtype=np.float64)
        n = len(self.mu)
        if n:
            ext = np.concatenate([[0.0], self.mu, [1.0]])
            gaps = np.maximum(ext[1:-1] - ext[:-2], ext[2:] - ext[1:-1])
            self.sig = np.clip(gaps, 1.0 / min(100.0, n + 1.0), 1.0)
        else:
            self.sig = np.zeros(0)
        self.w = np.full(n + 1, 1.0 / (n + 1))    # last weight: the uniform prior

    def pdf(self, u) -> np.ndarray:
        u = np.atleast_1d(np.asarray(u, dtype=np.float64))
        out = np.full(u.shape, self.w[-1])
        for m, s, w in zip(self.mu, self.sig, self.w[:-1]):
            z = (_phi((1 - m) / s) - _phi((0 - m) / s))
            out += w * np.exp(-0.5 * ((u - m) / s) ** 2) / (s * math.sqrt(2 * math.pi) * z)
        return out

    def sample(self, rng, n) -> np.ndarray:
        comp = rng.choice(len(self.w), size=n, p=self.w)
        out = np.empty(n)
        for i, c in enumerate(comp):
            if c == len(self.mu):
                out[i] = rng.uniform()
            else:
                while True:                   # truncated normal by rejection
                    v = rng.normal(self.mu[c], self.sig[c])
                    if 0.0 <= v <= 1.0:
                        out[i] = v
                        break
        return out


def _phi(z):
    return 0.5 * (1.0 + math.erf(z / math.sqrt(2.0)))


@dataclass
class Trial:
    params: dict
    objectives: tuple | None = None


@dataclass
class RandomSampler:
    seed: int = 0
    trials: list = field(default_factory=list)

    def __post_init__(self):
        self.rng = np.random.default_rng(self.seed)

    def _draw(self):
        p = {}
        for name, spec in SPACE.items():
            if spec[0] == "cat":
                p[name] = int(self.rng.choice(spec[1]))
            else:
                p[name] = _from_unit(name, self.rng.uniform())
        return p

    def ask(self, n: int) -> list[dict]:
        return [self._draw() for _ in range(n)]

    def tell(self, params: dict, objectives) -> None:
        self.trials.append(Trial(dict(params), tuple(objectives)))


@dataclass
class TPESampler(RandomSampler):
    gamma: float = 0.25
    n_startup: int = 8
    n_candidates: int = 24

    def _split(self):
        objs = [t.objectives for t in self.trials]
        ranks = nondominated_ranks(objs)
        # within a rank, prefer the larger normalised objective sum
        o = np.asarray(objs, dtype=np.float64)
        span = np.where(o.max(0) > o.min(0), o.max(0) - o.min(0), 1.0)
        score = ((o - o.min(0)) / span).sum(1)
        order = sorted(range(len(objs)), key=lambda i: (ranks[i], -score[i]))
        n_good = max(1, int(math.ceil(self.gamma * len(objs))))
        good = [self.trials[i] for i in order[:n_good]]
        bad = [self.trials[i] for i in order[n_good:]]
        return good, bad

    def ask(self, n: int) -> list[dict]:
        if len(self.trials) < self.n_startup:
            return super().ask(n)
        good, bad = self._split()
        cands = [dict() for _ in range(n * self.n_candidates)]
        score = np.zeros(len(cands))
        for name, spec in SPACE.items():
            if spec[0] == "cat":
                vals = list(spec[1])
                cg = np.array([1.0 + sum(t.params[name] == v for t in good) for v in vals])
                cb = np.array([1.0 + sum(t.params[name] == v for t in bad) for v in vals])
                pg, pb = cg / cg.sum(), cb / cb.sum()
                pick = self.rng.choice(len(vals), size=len(cands), p=pg)
                for c, k in zip(cands, pick):
                    c[name] = int(vals[k])
                score += np.log(pg[pick]) - np.log(pb[pick])
            else:
                lg = Parzen([_to_unit(name, t.params[name]) for t in good])
                lb = Parzen([_to_unit(name, t.params[name]) for t in bad])
                u = lg.sample(self.rng, len(cands))
                for c, v in zip(cands, u):
                    c[name] = _from_unit(name, v)
                uq = np.array([_to_unit(name, c[name]) for c in cands])
                score += np.log(lg.pdf(uq)) - np.log(lb.pdf(uq))
        out, seen = [], set()
        for i in np.argsort(-score, kind="stable"):
            key = tuple(sorted(cands[i].items()))
            if key in seen:
                continue
            seen.add(key)
            out.append(cands[i])
            if len(out) == n:
                break
        while len(out) < n:
            out.append(self._draw())
        return out


# ---------------------------------------------------------------------------
# The search loop over the batched encoder
# ---------------------------------------------------------------------------

def evaluate(A, dic, images, trials, ssim_mode=None, level: int = 9) -> list[tuple]:
    """Encodes every (image, trial) pair as one job of one batched encode (BF16
    form, one graph) and returns per trial the mean SSIM of its
    reconstructions and the compression rate of its streams (total original
    bytes / total DEFLATE-compressed bytes over the images)."""
    import torch
    ssim_mode = A.SSIM_WINDOW7 if ssim_mode is None else ssim_mode
    params = [dict(tol=t["tol"], tol_mode="rms", max_atoms=t["max_atoms"], n_min=t["n_min"], n_max=t["n_max"])
              for t in trials]
    jobs = [(i, j) for j in range(len(trials)) for i in range(len(images))]
    code = A.Code(dic, images, params, jobs, precision=A.PREC_BF16, schedule=A.SCHED_BATCHED)
    out = []
    try:
        for j in range(len(trials)):
            ss, orig, comp = [], 0, 0
            for i, img in enumerate(images):
                job = j * len(images) + i
                rec = torch.empty_like(img)
                code.decode(job, rec)
                ss.append(A.ssim(img, rec, ssim_mode))
                comp += len(code.pack([job], level=level))
                orig += img.shape[0] * img.shape[1]
            out.append((float(np.mean(ss)), orig / comp))
    finally:
        code.free()
    return out


def run(A, dic, images, rounds: int, batch: int, sampler: str = "tpe", seed: int = 0, ssim_mode=None) -> dict:
    """`rounds` rounds of `batch` trials each; returns the trial history and
    the indices of its Pareto front (SSIM, CR)."""
    s = TPESampler(seed=seed, n_startup=2 * batch) if sampler == "tpe" else RandomSampler(seed=seed)
    hist = []
    for _ in range(rounds):
        trials = s.ask(batch)
        for t, o in zip(trials, evaluate(A, dic, images, trials, ssim_mode)):
            s.tell(t, o)
            hist.append((t, o))
    objs = [o for _, o in hist]
    return dict(history=hist, pareto=pareto_front(objs), hypervolume=hypervolume_2d(objs))
