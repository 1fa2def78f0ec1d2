"""Sec. 3.1: the preconditioned SRT limiting form and the naive source term.

With every rate equal the GLBE is the preconditioned SRT-LBE; the consistent
source is T^-1 P_S T S (tested in test_oracle_lattice), while the naive
S* = S/gamma (eq. precondsourceincorrect) adds a spurious momentum term
d_j[(gamma - 1)/gamma^2 (tau* - 1/2)(F_i u_j + F_j u_i)].  That term vanishes
for unidirectional flows (duct, Hartmann) and is a pure gradient for a single
Fourier-mode forcing, so the steady-state check uses F = F0 (sin ky, sin 2kx, 0),
whose (F.grad)F has a curl.
"""
import numpy as np
import pytest

from oracle import glbe
from oracle.lattice import E19, W19


def test_naive_and_consistent_agree_at_gamma_one():
    rng = np.random.default_rng(0)
    d = 1e-2 * rng.uniform(-1, 1, (19, 30)) * W19[:, None]
    F = 1e-3 * rng.uniform(-1, 1, (3, 30))
    s = rng.uniform(0.3, 1.8, 19)
    a = glbe.collide(d, F, 1.0, s, source="precond")
    b = glbe.collide(d, F, 1.0, s, source="naive")
    assert np.array_equal(a, b)
    c = glbe.collide(d, F, 0.3, s, source="precond")
    e = glbe.collide(d, F, 0.3, s, source="naive")
    assert np.max(np.abs(c - e)) > 1e-8


@pytest.mark.parametrize("gamma", [0.5, 0.1])
def test_naive_srt_equals_velocity_space_form(gamma):
    """All rates 1/tau with the naive source equals the SRT-LBE with
    S* = w [3 (e - u).F + 9 (e.u)(e.F)] / gamma, computed in velocity space."""
    rng = np.random.default_rng(1)
    tau = 0.9
    d = 5e-2 * rng.uniform(-1, 1, (19, 50)) * W19[:, None]
    F = 1e-3 * rng.uniform(-1, 1, (3, 50))
    out = glbe.collide(d, F, gamma, np.full(19, 1.0 / tau), source="naive")
    f = d + W19[:, None]
    rho = f.sum(0)
    e = E19.astype(float)
    j = e.T @ f + F / (2 * gamma)
    u = j / rho
    ej, eu, eF = e @ j, e @ u, e @ F
    feq = W19[:, None] * (rho + 3 * ej + (4.5 * ej ** 2 - 1.5 * (j * j).sum(0)) / (gamma * rho))
    S_naive = W19[:, None] * (3 * (eF - (u * F).sum(0)) + 9 * eu * eF) / gamma
    ref = f - (f - feq) / tau + (1 - 0.5 / tau) * S_naive
    assert np.allclose(out + W19[:, None], ref, rtol=0, atol=2e-15)


def _rotational_forcing(L, F0):
    x = np.arange(L) + 0.5
    y = np.arange(L) + 0.5
    k = 2 * np.pi / L
    F = np.zeros((3, 1, L, L))
    F[0] = F0 * np.sin(k * y)[None, :, None]
    F[1] = F0 * np.sin(2 * k * x)[None, None, :]
    return F


def test_naive_source_error_scales_as_one_minus_gamma_over_gamma_squared():
    L, nu, F0 = 16, 0.1, 1e-5
    F = _rotational_forcing(L, F0)
    diffs = []
    gammas = (0.5, 0.2, 0.1)
    for g in gammas:
        us = {}
        for src in ("precond", "naive"):
            fl = glbe.Flow((L, L, 1), ("periodic",) * 3, F, g, glbe.rates(nu, g), source=src)
            assert fl.run_to(1e-12, 100000)
            us[src] = fl.velocity()
        diffs.append(np.linalg.norm(us["naive"] - us["precond"]) / np.linalg.norm(us["precond"]))
    scaled = [d / ((1 - g) / g ** 2) for d, g in zip(diffs, gammas)]
    assert diffs[0] < diffs[1] < diffs[2]
    assert max(scaled) / min(scaled) < 1.15, scaled
