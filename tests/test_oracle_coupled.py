"""Pins of the oracle's coupled flow/induction fields (Sec. 4: the velocity,
current and Lorentz force solved per node) through their defining relations,
checked on the returned values only:

* the velocity satisfies rho u = sum f e + F / (2 gamma) with the returned
  total force F (the hydrodynamic fields of Sec. 3, taken from the flow
  oracle's own `fields`), in a regime where the magnetic coupling changes u
  by order one, so that a wrong sign or a transposed matrix in the per-node
  solve fails;
* the Lorentz part of the returned force is J x B by numpy's cross product;
* with no induction populations (B = 0, Lambda = 0) the fields reduce exactly
  to the flow oracle's.

Planted mistakes (the per-node system with a sign flipped, the cross product
reversed) fail the first and second pins.
"""
import numpy as np
import pytest

from oracle import d2q9, glbe, mhd

PARAMS = dict(gamma=0.3, gamma_m=0.4, chi=0.05, eta=0.03)


def _inputs3(seed):
    rng = np.random.default_rng(seed)
    shp = (3, 4, 5)
    f = 1e-3 * rng.standard_normal((19,) + shp)
    g = 0.04 * rng.standard_normal((3, 7) + shp)
    g[1] += 0.05  # B_y of order 0.35: kappa |B|^2 / (2 gamma rho) of order one
    F = 1e-4 * rng.standard_normal((3,) + shp)
    return f, g, F


def _coupling(B, rho, p):
    tau = mhd.tau_m(p["eta"], p["gamma_m"])
    kappa = 2.0 / (p["gamma_m"] * tau * mhd.THETA_M)
    return kappa * (B * B).sum(axis=0) / (2.0 * p["gamma"] * rho)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_coupled_velocity_satisfies_its_defining_relation(seed):
    p = PARAMS
    f, g, F_ext = _inputs3(seed)
    rho, u, B, J, F = mhd.coupled_fields(f, g, F_ext, p["gamma"], p["gamma_m"], p["chi"], p["eta"])
    assert _coupling(B, rho, p).min() > 0.3  # the coupling is strong enough to matter
    _, rho_f, j0, _ = glbe.fields(f, np.zeros_like(F_ext), p["gamma"])
    assert np.allclose(rho, rho_f, rtol=0, atol=1e-15)
    lhs = rho * u
    rhs = j0 + F / (2.0 * p["gamma"])
    assert np.abs(lhs - rhs).max() < 1e-14 * np.abs(lhs).max()
    # the Lorentz part of the force, by numpy's cross product
    FL = np.moveaxis(np.cross(np.moveaxis(J, 0, -1), np.moveaxis(B, 0, -1)), -1, 0)
    assert np.abs((F - F_ext) - FL).max() < 1e-15


def test_coupled_fields_reduce_to_the_flow_fields_without_a_field():
    p = PARAMS
    f, g, F_ext = _inputs3(3)
    rho, u, B, J, F = mhd.coupled_fields(f, np.zeros_like(g), F_ext, p["gamma"], p["gamma_m"],
                                         p["chi"], p["eta"])
    _, rho_f, _, u_f = glbe.fields(f, F_ext, p["gamma"])
    assert np.array_equal(B, np.zeros_like(B)) and np.abs(J).max() == 0.0
    assert np.allclose(u, u_f, rtol=1e-15, atol=0) and np.array_equal(F, F_ext)
    assert np.allclose(rho, rho_f, rtol=0, atol=0)


def test_planted_sign_mistake_in_the_solve_fails_the_pin(monkeypatch):
    """The per-node system built with the identity's sign flipped (in the
    system matrix and in (u x B) x B = (u.B) B - |B|^2 u): the returned
    velocity no longer satisfies its defining relation."""
    p = PARAMS
    f, g, F_ext = _inputs3(4)
    real_eye = np.eye

    def wrong_eye(n, *a, **k):
        # the identity of the 3 x 3 system and of (u x B) x B, negated
        return -real_eye(n, *a, **k) if n == 3 else real_eye(n, *a, **k)

    monkeypatch.setattr(mhd.np, "eye", wrong_eye)
    rho, u, B, J, F = mhd.coupled_fields(f, g, F_ext, p["gamma"], p["gamma_m"], p["chi"], p["eta"])
    monkeypatch.undo()
    _, _, j0, _ = glbe.fields(f, np.zeros_like(F_ext), p["gamma"])
    lhs, rhs = rho * u, j0 + F / (2.0 * p["gamma"])
    assert np.abs(lhs - rhs).max() > 1e-6 * np.abs(lhs).max()


def test_planted_reversed_cross_product_fails_the_pin(monkeypatch):
    """The oracle's cross product reversed: its Lorentz force is no longer
    J x B."""
    p = PARAMS
    f, g, F_ext = _inputs3(5)
    real = mhd._cross
    monkeypatch.setattr(mhd, "_cross", lambda a, b: real(b, a))
    rho, u, B, J, F = mhd.coupled_fields(f, g, F_ext, p["gamma"], p["gamma_m"], p["chi"], p["eta"])
    monkeypatch.undo()
    FL = np.moveaxis(np.cross(np.moveaxis(J, 0, -1), np.moveaxis(B, 0, -1)), -1, 0)
    assert np.abs((F - F_ext) - FL).max() > 1e-6 * np.abs(FL).max()


@pytest.mark.parametrize("seed", [0, 1])
def test_coupled_velocity_2d_satisfies_its_defining_relation(seed):
    p = PARAMS
    rng = np.random.default_rng(10 + seed)
    shp = (5, 6)
    f = 1e-3 * rng.standard_normal((9,) + shp)
    g = 0.04 * rng.standard_normal((2, 5) + shp)
    g[1] += 0.07
    F_ext = 1e-4 * rng.standard_normal((2,) + shp)
    rho, u, B, J, F = d2q9.coupled_fields(f, g, F_ext, p["gamma"], p["gamma_m"], p["chi"], p["eta"])
    _, _, j0, _ = d2q9.fields(f, np.zeros_like(F_ext), p["gamma"])
    lhs, rhs = rho * u, j0 + F / (2.0 * p["gamma"])
    assert np.abs(lhs - rhs).max() < 1e-14 * np.abs(lhs).max()
    # J along z, B in the plane: J z x B = J (-B_y, B_x)
    Jv = np.stack([np.zeros_like(J), np.zeros_like(J), J], axis=-1)
    Bv = np.stack([B[0], B[1], np.zeros_like(J)], axis=-1)
    FL = np.moveaxis(np.cross(Jv, Bv), -1, 0)
    assert np.abs(FL[2]).max() == 0.0
    assert np.abs((F - F_ext) - FL[:2]).max() < 1e-15
    # without the field the 2D fields are the flow oracle's
    rho0_, u0_, B0_, J0_, F0_ = d2q9.coupled_fields(f, np.zeros_like(g), F_ext, p["gamma"],
                                                    p["gamma_m"], p["chi"], p["eta"])
    assert np.allclose(u0_, d2q9.fields(f, F_ext, p["gamma"])[3], rtol=1e-15, atol=0)
