"""Host logic of the stability-envelope drivers, with the marches replaced by
a known threshold: gamma is stable iff gamma >= g*(nu, u_max).  Both searches
must bracket g* within their stated resolution, flag the edge cases, and (for
the batched search) put every point of a round into one march."""
import math

import numpy as np
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


# ------------------------------------------------ precision-ladder host logic
class _FakeSim:
    """Stands in for Simulation in the host-side ladder logic: a march whose
    kinetic energy approaches 1 as 1 - exp(-t / tau), checked every 10 steps."""

    def __init__(self, name, log, tau=2000.0, reach=None, nonfinite_at=None):
        import types
        self.name, self.log, self.tau, self.reach, self.nonfinite_at = name, log, tau, reach, nonfinite_at
        self.t = 0
        self._params = types.SimpleNamespace(check_every=10)

    def step(self, n):
        self.t += n

    def history(self, k):
        import math
        bad = 1.0 if self.nonfinite_at is not None and self.t >= self.nonfinite_at else 0.0
        return np.array([[self.t, 0.0, 0.0, 1.0 - math.exp(-self.t / self.tau), 0.0, 0.0, bad, 0.0]])

    def convert_from(self, other):
        self.log.append(("convert", other.name, self.name))
        self.t = other.t

    def run_to_residual(self, tol, max_steps, poll_every):
        self.log.append(("residual", self.name, tol))
        if self.reach is None:
            self.t += max_steps
            return -1, 1.0
        self.t = max(self.t, self.reach)
        return self.t, tol / 2

    def run_to_energy_change(self, tol, max_steps, window):
        self.log.append(("energy", self.name, tol))
        e0 = None
        for _ in range(max_steps // window):
            self.step(window)
            e1 = self.history(1)[-1, 3]
            if e0 is not None and abs(e1 - e0) / e1 < tol:
                return self.t, abs(e1 - e0) / e1
            e0 = e1
        return -1, 1.0


def test_run_ladder_chains_rungs_and_stops_at_a_failed_one():
    import paper_0809_4730_amd as pkg
    log = []
    a, b, c = _FakeSim("a", log), _FakeSim("b", log, reach=30000), _FakeSim("c", log, reach=40000)
    n, per = pkg.run_ladder([(a, "energy", 1e-4), (b, "residual", 2e-7), (c, "residual", 1e-8)], 10 ** 6)
    assert n == 40000 and [k for k, _ in per] == [a.t, 30000, 40000]
    assert [e[0] for e in log] == ["energy", "convert", "residual", "convert", "residual"]
    assert log[1] == ("convert", "a", "b") and log[3] == ("convert", "b", "c")
    log.clear()
    a, b, c = _FakeSim("a", log, tau=200.0), _FakeSim("b", log), _FakeSim("c", log, reach=40000)
    n, per = pkg.run_ladder([(a, "energy", 1e-4), (b, "residual", 2e-7), (c, "residual", 1e-8)], 5000)
    assert n == -1 and len(per) == 2             # c never runs
    assert not any(e[0] == "convert" and e[2] == "c" for e in log)
    with pytest.raises(ValueError):
        pkg.run_ladder([(_FakeSim("x", []), "bogus", 1.0)], 10)
