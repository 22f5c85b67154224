"""Host logic of the hyperparameter search (Section 2.4): Pareto utilities,
Parzen densities, the samplers' ranges, and TPE beating random search on a
cheap synthetic two-objective problem."""
import math

import numpy as np
import pytest

from paper_2605_09190_amd import hpo


def test_nondominated_ranks_brute_force():
    rng = np.random.default_rng(0)
    pts = [tuple(p) for p in rng.uniform(size=(40, 2))]
    ranks = hpo.nondominated_ranks(pts)
    for i, p in enumerate(pts):
        doms = [j for j, q in enumerate(pts) if hpo.dominates(q, p)]
        # rank = 1 + the largest rank of a dominator (0 if none)
        assert ranks[i] == (0 if not doms else 1 + max(ranks[j] for j in doms))
    front = hpo.pareto_front(pts)
    assert all(not any(hpo.dominates(pts[j], pts[i]) for j in range(len(pts))) for i in front)


def test_hypervolume_known_values():
    assert hpo.hypervolume_2d([(1.0, 1.0)]) == 1.0
    assert math.isclose(hpo.hypervolume_2d([(1.0, 0.5), (0.5, 1.0)]), 0.75)
    assert math.isclose(hpo.hypervolume_2d([(1.0, 0.5), (0.5, 1.0), (0.4, 0.4)]), 0.75)


def test_parzen_is_a_density():
    rng = np.random.default_rng(1)
    for pts in ([], [0.2], list(rng.uniform(size=9))):
        pz = hpo.Parzen(pts)
        u = np.linspace(0, 1, 20001)
        assert abs(np.trapezoid(pz.pdf(u), u) - 1.0) < 1e-3
        s = pz.sample(rng, 200)
        assert ((0 <= s) & (s <= 1)).all()


def test_samplers_stay_in_the_space():
    for cls in (hpo.RandomSampler, hpo.TPESampler):
        s = cls(seed=3)
        for _ in range(5):
            for t in s.ask(6):
                assert 0.005 <= t["tol"] <= 0.06
                assert isinstance(t["max_atoms"], int) and 8 <= t["max_atoms"] <= 64
                assert t["n_min"] in (4, 8) and t["n_max"] in (32, 64)
                s.tell(t, (np.random.default_rng(0).uniform(), 1.0))


def _toy(p):
    """Two competing objectives with a known good region."""
    u = hpo._to_unit("tol", p["tol"])
    v = hpo._to_unit("max_atoms", p["max_atoms"])
    a = 1.0 - abs(u - 0.2) - 0.3 * abs(v - 0.8) + (0.1 if p["n_min"] == 8 else 0.0)
    b = 1.0 - abs(v - 0.7) - 0.3 * abs(u - 0.3) + (0.1 if p["n_max"] == 64 else 0.0)
    return (a, b)


def test_tpe_beats_random_on_a_toy_problem():
    hv = {"tpe": [], "random": []}
    for seed in range(4):
        for name, cls in (("tpe", hpo.TPESampler), ("random", hpo.RandomSampler)):
            s = cls(seed=seed) if name == "random" else cls(seed=seed, n_startup=8)
            objs = []
            for _ in range(8):
                for t in s.ask(6):
                    o = _toy(t)
                    s.tell(t, o)
                    objs.append(o)
            hv[name].append(hpo.hypervolume_2d(objs))
    assert np.mean(hv["tpe"]) > np.mean(hv["random"])
