"""Stability envelope of the preconditioned GLBE on body-force Poiseuille flow
(Sec. 5): the library's instability verdict checked against the oracle, and the
shape of the gamma_min(u_max) map."""
import math

import numpy as np
import pytest

from oracle import glbe
from paper_0809_4730_amd import stability
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

BC = ("periodic", "periodic", "wall")


def _oracle_blows_up(nu, u_max, gamma, steps, H=64, width=4):
    """True when the oracle march of the same channel has non-finite values or
    |u| above 1 (lattice units) within `steps` steps."""
    F = stability.poiseuille_force(nu, u_max, H)
    flow = glbe.Flow((width, width, H), BC, (F, 0.0, 0.0), gamma, glbe.rates(nu, gamma))
    with np.errstate(all="ignore"):
        while flow.t < steps:
            flow.step(min(50, steps - flow.t))
            u = flow.velocity()
            if not np.isfinite(u).all() or np.abs(u).max() > 1.0:
                return True
    return False


def _oracle_settles(nu, u_max, gamma, steps, H=64, width=4):
    """True when the oracle march stays finite and within 10 % of u_max."""
    F = stability.poiseuille_force(nu, u_max, H)
    flow = glbe.Flow((width, width, H), BC, (F, 0.0, 0.0), gamma, glbe.rates(nu, gamma))
    with np.errstate(all="ignore"):
        flow.step(steps)
        u = flow.velocity()
    return bool(np.isfinite(u).all() and np.abs(u).max() < 1.1 * u_max)


def test_verdicts_match_oracle():
    announce("stability verdicts: nu=0.02 u_max=0.05")
    v, n = stability.march(0.02, 0.05, 1.0, max_steps=3000)
    assert v == stability.STABLE
    assert _oracle_settles(0.02, 0.05, 1.0, 600)
    v, n = stability.march(0.02, 0.05, 1e-3, max_steps=3000)
    assert v == stability.UNSTABLE and n <= 3000
    assert _oracle_blows_up(0.02, 0.05, 1e-3, n)


def test_gamma_min_bracket_matches_oracle():
    """The bisection's bracket around gamma_min: the oracle blows up just below
    it and stays bounded at it, over the same number of steps."""
    nu, um = 0.02, 0.05
    gmin, runs = stability.gamma_min(nu, um, lo=1e-3, hi=1.0, iters=6, max_steps=4000)
    announce("gamma_min(nu=%g, u_max=%g) = %.4g after %d runs" % (nu, um, gmin, runs))
    assert 1e-3 < gmin < 1.0
    below = gmin / (1e3 ** (2.0 ** -6))
    v, n = stability.march(nu, um, below, max_steps=4000)
    assert v == stability.UNSTABLE
    assert _oracle_blows_up(nu, um, below, n)
    assert _oracle_settles(nu, um, gmin, min(n, 1000))


def test_envelope_rises_with_u_max():
    """At fixed viscosity a faster flow needs a larger gamma (less
    preconditioning) to stay stable."""
    nu = 0.02
    us = (0.005, 0.02, 0.08)
    step = 1e3 ** (2.0 ** -6)  # bisection resolution (factor)
    env = stability.envelope((nu,), us, lo=1e-3, hi=1.0, iters=6, max_steps=4000)
    announce("envelope nu=%g: %s" % (nu, [(e["u_max"], e["gamma_min"]) for e in env]))
    g = [e["gamma_min"] for e in env]
    assert all(math.isfinite(x) for x in g)
    for a, b in zip(g, g[1:]):
        assert b * step >= a
    assert g[-1] > 2.0 * g[0]


def test_envelope_rises_with_viscosity():
    """At fixed u_max the smallest stable gamma is larger for the more viscous
    fluid (stronger preconditioning is possible at low viscosity)."""
    g_lo, _ = stability.gamma_min(0.002, 0.05, lo=1e-3, hi=1.0, iters=6, max_steps=4000)
    g_hi, _ = stability.gamma_min(0.1, 0.05, lo=1e-3, hi=1.0, iters=6, max_steps=4000)
    announce("gamma_min(u_max=0.05): nu=0.002 -> %.4g, nu=0.1 -> %.4g" % (g_lo, g_hi))
    assert g_hi > 1.5 * g_lo


POINTS = [(0.02, 0.05, 1.0), (0.02, 0.05, 1e-3), (0.02, 0.05, 0.05), (0.02, 0.05, 0.02),
          (0.1, 0.02, 0.5), (0.1, 0.08, 0.03), (0.002, 0.005, 0.01), (0.002, 0.08, 0.02)]


def test_batched_verdicts_match_single_lattice_marches():
    """Members of one batched march reach the verdicts of separate marches of
    the same lattices (and a converged member at the same step)."""
    got = stability.march_batch(POINTS, max_steps=4000, tol=1e-9)
    announce("batched verdicts: %s" % got)
    for (nu, um, g), (v, step) in zip(POINTS, got):
        vs, ts = stability.march(nu, um, g, max_steps=4000, tol=1e-9)
        assert v == vs, (nu, um, g, v, vs)
        if v == stability.UNSTABLE:
            assert step <= ts
    assert {v for v, _ in got} == {stability.STABLE, stability.UNSTABLE}


def test_batched_envelope_matches_bisection():
    nus, us = (0.02, 0.1), (0.02, 0.05)
    env_b = stability.envelope_batched(nus, us, per_round=15, rounds=2, max_steps=4000)
    announce("batched envelope: %s" % [(e["nu"], e["u_max"], round(e["gamma_min"], 5)) for e in env_b])
    res_b = 1e3 ** (1.0 / 16 ** 2)
    res_s = 1e3 ** (2.0 ** -7)
    for e in env_b:
        g, _ = stability.gamma_min(e["nu"], e["u_max"], lo=1e-3, hi=1.0, iters=7, max_steps=4000)
        assert g / (res_b * res_s) <= e["gamma_min"] <= g * res_b * res_s, (e, g)
