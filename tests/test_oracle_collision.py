"""Pins for the oracle's collision: conservation, the rates it may ignore, and
its single-relaxation-time limit computed by an independent velocity-space route."""
import numpy as np
import pytest

from oracle import glbe
from oracle.lattice import E19, W19


def _random_state(rng, n, amp=1e-2):
    d = amp * rng.uniform(-1, 1, (19, n)) * W19[:, None]
    F = 1e-3 * rng.uniform(-1, 1, (3, n))
    return d, F


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("gamma", [1.0, 0.3, 0.05])
def test_collision_conserves_mass_and_adds_force_over_gamma(seed, gamma):
    """P3: sum_a (f~ - f) = 0 and sum_a (f~ - f) e_a = F / gamma for any state and rates."""
    rng = np.random.default_rng(seed)
    d, F = _random_state(rng, 64)
    s = rng.uniform(0.2, 1.9, 19)
    out = glbe.collide(d, F, gamma, s)
    dd = out - d
    assert np.max(np.abs(dd.sum(axis=0))) < 1e-16
    mom = E19.T.astype(float) @ dd
    assert np.allclose(mom, F / gamma, rtol=0, atol=1e-16)


def test_conserved_mode_rates_do_not_matter():
    """s0, s3, s5, s7 are not given by the paper; any value gives the same step."""
    rng = np.random.default_rng(7)
    d, F = _random_state(rng, 32)
    s = glbe.rates(0.1, 0.2)
    a = glbe.collide(d, F, 0.2, s)
    s2 = s.copy()
    for k in (0, 3, 5, 7):
        s2[k] = rng.uniform(0.1, 1.9)
    b = glbe.collide(d, F, 0.2, s2)
    assert np.max(np.abs(a - b)) < 1e-17


@pytest.mark.parametrize("gamma", [1.0, 0.25, 0.04])
@pytest.mark.parametrize("tau", [0.6, 1.0, 3.7])
def test_equal_rates_reduce_to_preconditioned_bgk(gamma, tau):
    """P4: with every s_k = 1/tau the GLBE step is the preconditioned SRT-LBE of
    Sec. 3.1, evaluated here directly in velocity space (no moment basis):
        f~ = f - (f - f^eq*)/tau + (1 - 1/(2 tau)) S*,
    f^eq* = w[rho + 3 e.j + (9/2 (e.j)^2 - 3/2 j.j)/(gamma rho)],
    S* = w[3 (e - u/gamma).F/gamma + 9 (e.u)(e.F)/gamma^2]."""
    rng = np.random.default_rng(11)
    d, F = _random_state(rng, 80, amp=5e-2)
    s = np.full(19, 1.0 / tau)
    out = glbe.collide(d, F, gamma, s)
    f = d + W19[:, None]
    rho = f.sum(0)
    e = E19.astype(float)
    j = e.T @ f + F / (2 * gamma)
    u = j / rho
    ej = e @ j
    feq = W19[:, None] * (rho + 3 * ej + (4.5 * ej ** 2 - 1.5 * (j * j).sum(0)) / (gamma * rho))
    eu = e @ u
    eF = e @ F
    Sst = W19[:, None] * (3 * (eF - (u * F).sum(0) / gamma) / gamma + 9 * eu * eF / gamma ** 2)
    ref = f - (f - feq) / tau + (1 - 0.5 / tau) * Sst
    assert np.allclose(out + W19[:, None], ref, rtol=0, atol=2e-15)


def test_rest_state_is_fixed_point():
    d = np.zeros((19, 10))
    F = np.zeros((3, 10))
    out = glbe.collide(d, F, 0.1, glbe.rates(0.1, 0.1))
    assert np.all(out == 0)


def test_streaming_permutes_and_conserves():
    """Pull streaming with bounce-back is a permutation of the population entries."""
    rng = np.random.default_rng(3)
    post = rng.standard_normal((19, 5, 4, 3))
    for bc in [("periodic",) * 3, ("periodic", "wall", "wall"), ("wall", "wall", "wall")]:
        f = glbe.stream(post, bc)
        assert np.allclose(np.sort(f.ravel()), np.sort(post.ravel()))
        assert abs(f.sum() - post.sum()) < 1e-12
