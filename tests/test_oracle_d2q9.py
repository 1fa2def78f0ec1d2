"""Pins for the 2D oracle (D2Q9 GLBE with forcing, D2Q5 induction LKE).

Tables and moment lists: the basis applied to velocity-space expressions must
reproduce the printed D2Q9 lists exactly (rational arithmetic).  Flows: plane
Poiseuille (exact parabola in the fixed-Lambda mode), preconditioning's
steady-state invariance and step reduction, and 2D Hartmann flow against its
closed form with second-order convergence.
"""
import os
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import d2q9 as d
from oracle import glbe

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PER, WALL = glbe.PERIODIC, glbe.WALL


def _golden(name, skip_name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows[int(parts[0])] = " ".join(parts[2:] if skip_name else parts[1:])
    return [rows[k] for k in range(len(rows))]


def _eval(expr, **env):
    env["Fraction"] = Fraction
    return Fraction(eval(expr, {"__builtins__": {}}, env))


def _frac(rng, lo=-50, hi=50, den=97):
    return Fraction(rng.randint(lo, hi), den)


def _matvec(T, v):
    return [sum(T[k][a] * v[a] for a in range(len(v))) for k in range(len(T))]


def _gamma(rng):
    g = Fraction(rng.choice([1, 2, 5, 10, 37]), rng.choice([1, 3, 10, 100]))
    return 1 / g if g > 1 else g


# ------------------------------------------------------------ tables
def test_velocity_sets_and_weights():
    assert sorted((d.E9 ** 2).sum(1).tolist()) == [0] + [1] * 4 + [2] * 4
    assert np.all(d.E9[d.OPP9] == -d.E9) and np.all(d.E5[d.OPP5] == -d.E5)
    assert sum(d.W9_FRAC) == 1
    for i in range(2):
        for j in range(2):
            s2 = sum(d.W9_FRAC[a] * int(d.E9[a][i]) * int(d.E9[a][j]) for a in range(9))
            assert s2 == (Fraction(1, 3) if i == j else 0)
    # D2Q5: sum W = 1, sum W e_i e_j = theta_m delta_ij (Sec. 4, N_m = 3)
    assert d.W5.sum() == pytest.approx(1.0, abs=1e-15)
    M = np.einsum("a,ai,aj->ij", d.W5, d.E5.astype(float), d.E5.astype(float))
    assert np.allclose(M, d.THETA_M2 * np.eye(2), atol=1e-15)


def test_basis_orthogonal_integer_rows():
    for k in range(9):
        for a in range(9):
            assert d.T9_FRAC[k][a].denominator == 1
        for l in range(9):
            dot = sum(d.T9_FRAC[k][a] * d.T9_FRAC[l][a] for a in range(9))
            assert (dot == 0) == (k != l)
    norms = [sum(v * v for v in r) for r in d.T9_FRAC]
    assert norms == [9, 36, 36, 6, 12, 6, 12, 4, 4]
    assert np.allclose(d.T9_INV, d.T9.T / np.array([float(n) for n in norms])[None], atol=1e-15)


def test_rest_state_moments():
    eq = _golden("d2q9_equilibrium_moments.txt", True)
    want = [_eval(eq[k], rho=1, jx=0, jy=0, jj=0, g=1) for k in range(9)]
    assert _matvec(d.T9_FRAC, d.W9_FRAC) == want


# -------------------------------------------------------- equilibria
@pytest.mark.parametrize("seed", range(6))
def test_T_of_velocity_equilibrium_matches_printed(seed):
    """T f^eq* (velocity space, w[rho + 3 e.j + (9/2 (e.j)^2 - 3/2 j.j)/(gamma rho)])
    equals the printed preconditioned D2Q9 list exactly."""
    rng = random.Random(seed)
    eq = _golden("d2q9_equilibrium_moments.txt", True)
    rho = 1 + _frac(rng, -20, 20, 101)
    j = [_frac(rng), _frac(rng)]
    g = _gamma(rng)
    jj = j[0] ** 2 + j[1] ** 2
    feq = []
    for a, c in enumerate(d.E9):
        ej = int(c[0]) * j[0] + int(c[1]) * j[1]
        feq.append(d.W9_FRAC[a] * (rho + 3 * ej + (Fraction(9, 2) * ej * ej
                                                    - Fraction(3, 2) * jj) / (g * rho)))
    want = [_eval(eq[k], rho=rho, jx=j[0], jy=j[1], jj=jj, g=g) for k in range(9)]
    assert _matvec(d.T9_FRAC, feq) == want


@pytest.mark.parametrize("seed", range(3))
def test_oracle_equilibrium_function(seed):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.05 * rng.uniform(-1, 1, 30)
    j = 0.05 * rng.uniform(-1, 1, (2, 30))
    g = rng.choice([1.0, 0.3, 0.01])
    e = d.E9.astype(float)
    ej = e @ j
    feq = d.W9[:, None] * (rho + 3 * ej + (4.5 * ej ** 2 - 1.5 * (j * j).sum(0)) / (g * rho))
    assert np.allclose(d.meq_star(rho, j, g), d.T9 @ feq, rtol=0, atol=1e-13)
    dev = d.meq_star_dev(rho - 1.0, rho, j, g)
    assert np.allclose(dev + (d.T9 @ d.W9)[:, None], d.T9 @ feq, rtol=0, atol=1e-13)


# ----------------------------------------------------------- sources
def _velocity_source(F, u, g=Fraction(1)):
    """w [3 (e - u/g).F / g + 9 (e.u)(e.F)/g^2] (Sec. 2; Sec. 3.1 for g != 1)."""
    out = []
    for a, c in enumerate(d.E9):
        eF = int(c[0]) * F[0] + int(c[1]) * F[1]
        eu = int(c[0]) * u[0] + int(c[1]) * u[1]
        uF = u[0] * F[0] + u[1] * F[1]
        out.append(d.W9_FRAC[a] * (3 * (eF - uF / g) / g + 9 * eu * eF / g ** 2))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_preconditioned_sources_match_printed(seed):
    """The printed S^* list equals P_S T S (S the gamma = 1 velocity-space source),
    and T^-1 S^* equals the velocity-space S^* of Sec. 3.1, exactly."""
    rng = random.Random(50 + seed)
    src = _golden("d2q9_source_moments.txt", False)
    F = [_frac(rng), _frac(rng)]
    u = [_frac(rng), _frac(rng)]
    g = _gamma(rng)
    Fu = F[0] * u[0] + F[1] * u[1]
    printed = [_eval(src[k], Fx=F[0], Fy=F[1], ux=u[0], uy=u[1], Fu=Fu, g=g) for k in range(9)]
    mS = _matvec(d.T9_FRAC, _velocity_source(F, u))
    PS = [Fraction(1), 1 / g ** 2, 1 / g ** 2, 1 / g, 1 / g, 1 / g, 1 / g, 1 / g ** 2, 1 / g ** 2]
    assert [PS[k] * mS[k] for k in range(9)] == printed
    norms = [sum(v * v for v in r) for r in d.T9_FRAC]
    back = [sum(d.T9_FRAC[k][a] * printed[k] / norms[k] for k in range(9)) for a in range(9)]
    assert back == _velocity_source(F, u, g)
    # the oracle's float functions
    Ff = np.array([float(x) for x in F])
    uf = np.array([float(x) for x in u])
    assert np.allclose(d.source_precond_diag(float(g)) * d.source_moments(Ff, uf),
                       [float(x) for x in printed], rtol=1e-13, atol=1e-16)
    assert np.allclose(d.T9 @ d.velocity_source(Ff, uf), d.source_moments(Ff, uf), atol=1e-14)


def test_rates_match_printed():
    with open(os.path.join(GOLDEN, "d2q9_rates.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    nu, g = 0.05, 0.2
    s = d.rates(nu, g)
    for k, v in rows:
        want = 1.0 / (3 * nu / g + 0.5) if v == "shear" else float(v)
        assert s[int(k)] == pytest.approx(want, rel=1e-15)


# -------------------------------------------------------------- flows
def _poiseuille(H, nu, gamma, F, s, tol=1e-12):
    fl = d.Flow2D((2, H), (PER, WALL), (F, 0.0), gamma, s)
    assert fl.run_to(tol, 100000)
    f = d.stream(fl.post, fl.bc)
    return fl, d.fields(f, fl.F, gamma)


@pytest.mark.parametrize("gamma", [1.0, 0.2])
def test_poiseuille_exact_in_fixed_lambda_mode(gamma):
    """Halfway bounce-back with Lambda = 3/16 gives the parabola to rounding;
    another Lambda adds the known slip F (16 Lambda - 3)/(24 nu)."""
    H, nu, F = 12, 0.1, 1e-5
    y = np.arange(H) + 0.5
    for Lam in (3 / 16, 0.25):
        _, (_, _, j, _) = _poiseuille(H, nu, gamma, F, d.rates(nu, gamma, "lambda", Lam))
        exact = F * y * (H - y) / (2 * nu) + F * (16 * Lam - 3) / (24 * nu)
        assert np.max(np.abs(j[0][:, 0] - exact)) / exact.max() < 1e-9
        assert np.max(np.abs(j[1])) < 1e-12 * exact.max()


def test_preconditioning_keeps_steady_state_and_cuts_steps():
    H, nu, F = 12, 0.1, 1e-5
    out = []
    for gamma in (1.0, 0.1):
        fl, (_, _, j, _) = _poiseuille(H, nu, gamma, F, d.rates(nu, gamma, "lambda", 3 / 16),
                                       tol=1e-11)
        out.append((fl.t, j[0][:, 0]))
    assert np.max(np.abs(out[0][1] - out[1][1])) / out[0][1].max() < 1e-7
    assert out[0][0] > 5 * out[1][0]


def _hartmann2d(L, Ha=5.0, chi=0.0025, gamma=0.1, gamma_m=0.1, nu=0.1, eta=0.025, F=1e-5):
    B0 = Ha * np.sqrt(eta * nu) / L
    s = d.rates(nu, gamma, "lambda", 3 / 16)
    fl = d.MHDFlow2D((1, 2 * L), (PER, WALL), (F, 0.0), gamma, s, gamma_m, chi, eta, (0.0, B0))
    assert fl.run_to(1e-11, 60000)
    y = np.arange(2 * L) + 0.5 - L
    uex = F * L * L / (nu * Ha) * (np.cosh(Ha) - np.cosh(Ha * y / L)) / np.sinh(Ha)
    bex = chi * F * L / B0 * (np.sinh(Ha * y / L) / np.sinh(Ha) - y / L)
    u, b = fl.u[0][:, 0], fl.B[0][:, 0]
    return (np.sqrt(np.mean((u - uex) ** 2)) / uex.max(),
            np.sqrt(np.mean((b - bex) ** 2)) / np.abs(bex).max())


def test_hartmann_2d_closed_form_second_order():
    """2D Hartmann flow (Sec. 5) with D2Q9 + D2Q5 against the insulating-wall
    profiles u(y) and b_x(y); the error falls fourfold per doubling."""
    eu1, eb1 = _hartmann2d(8)
    eu2, eb2 = _hartmann2d(16)
    assert eu2 < 0.008 and eb2 < 0.01, (eu2, eb2)
    assert 3.5 < eu1 / eu2 < 4.5 and 3.5 < eb1 / eb2 < 4.5, (eu1, eu2, eb1, eb2)


def test_hartmann_2d_printed_current_sign_fails(monkeypatch):
    """Planted mistake (on the oracle): the printed contraction's sign makes the
    Lorentz force drive the flow instead of braking it."""
    monkeypatch.setattr(d, "CURRENT_SIGN", 1.0)
    with np.errstate(all="ignore"):
        L, Ha, nu, eta, F = 8, 5.0, 0.1, 0.025, 1e-5
        B0 = Ha * np.sqrt(eta * nu) / L
        fl = d.MHDFlow2D((1, 2 * L), (PER, WALL), (F, 0.0), 0.1, d.rates(nu, 0.1, "lambda", 3 / 16),
                         0.1, 0.0025, eta, (0.0, B0))
        ok = fl.run_to(1e-10, 1500)
        y = np.arange(2 * L) + 0.5 - L
        uex = F * L * L / (nu * Ha) * (np.cosh(Ha) - np.cosh(Ha * y / L)) / np.sinh(Ha)
        u = fl.u[0][:, 0]
    assert (not ok) or (not np.all(np.isfinite(u))) or np.max(np.abs(u - uex)) > 0.5 * uex.max()
