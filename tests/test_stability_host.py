"""Host logic of the stability-envelope drivers, with the marches replaced by
a known threshold: gamma is stable iff gamma >= g*(nu, u_max).  Both searches
must bracket g* within their stated resolution, flag the edge cases, and (for
the batched search) put every point of a round into one march."""
import math

import pytest

from paper_0809_4730_amd import stability


def _threshold(nu, um):
    return 0.002 + 0.9 * um * (1.0 + 2.0 * nu)


@pytest.fixture
def fake(monkeypatch):
    calls = {"single": 0, "batch": []}

    def march(nu, um, gamma, **kw):
        calls["single"] += 1
        v = stability.STABLE if gamma >= _threshold(nu, um) else stability.UNSTABLE
        return v, 100

    def march_batch(points, **kw):
        calls["batch"].append(len(points))
        return [(stability.STABLE if g >= _threshold(nu, um) else stability.UNSTABLE, 100)
                for nu, um, g in points]

    monkeypatch.setattr(stability, "march", march)
    monkeypatch.setattr(stability, "march_batch", march_batch)
    return calls


def test_bisection_brackets_threshold(fake):
    for nu, um in ((0.01, 0.02), (0.1, 0.08), (0.002, 0.001)):
        g, n = stability.gamma_min(nu, um, lo=1e-3, hi=1.0, iters=8)
        t = _threshold(nu, um)
        assert t <= g <= t * 1e3 ** (2.0 ** -8)
        assert n == 10


def test_bisection_edges(fake, monkeypatch):
    g, n = stability.gamma_min(0.1, 2.0, lo=1e-3, hi=1.0)   # threshold above hi
    assert g == math.inf and n == 1
    g, n = stability.gamma_min(0.1, 1e-6, lo=0.01, hi=1.0)  # threshold below lo
    assert g == 0.01


def test_batched_search_brackets_threshold_in_few_marches(fake):
    nus, us = (0.002, 0.02, 0.1), (0.005, 0.05, 0.08)
    env = stability.envelope_batched(nus, us, lo=1e-3, hi=1.0, per_round=15, rounds=2)
    assert fake["batch"] == [9 * 17, 9 * 15]  # one march per round for all points
    res = 1e3 ** (1.0 / 16 ** 2)
    for e in env:
        t = _threshold(e["nu"], e["u_max"])
        assert t <= e["gamma_min"] <= t * res * (1 + 1e-12), (e, t)


def test_batched_search_edges(fake):
    env = stability.envelope_batched((0.1,), (2.0, 1e-7), lo=0.01, hi=1.0, per_round=7, rounds=3)
    assert env[0]["gamma_min"] == math.inf
    assert env[1]["gamma_min"] == 0.01
    assert fake["batch"] == [2 * 9]  # both decided in the first round
