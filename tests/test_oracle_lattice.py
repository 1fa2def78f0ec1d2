"""Pins for the oracle's lattice tables, equilibria and sources.

Each check compares two routes that share nothing but the velocity set:
the moment basis T (built from row polynomials) applied to a velocity-space
expression, against the moment-space lists the paper prints (golden fixtures)
and against the oracle's own moment-space functions.  Exact rational
arithmetic where possible.
"""
import os
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import glbe
from oracle.lattice import (E19, E7, OPP19, OPP7, T19, T19_FRAC, T19_INV, W19, W19_FRAC,
                            W7, THETA_M)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_golden(name):
    rows, extra = {}, None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "PS":
                extra = parts[1:]
                continue
            k = int(parts[0])
            expr = " ".join(parts[2:]) if name.startswith("d3q19_equilibrium") else \
                " ".join(parts[1:])
            rows[k] = expr
    return [rows[k] for k in range(19)], extra


def _eval(expr, **env):
    env = dict(env)
    env["Fraction"] = Fraction
    return Fraction(eval(expr, {"__builtins__": {}}, env))


def _rand_frac(rng, lo=-50, hi=50, den=97):
    return Fraction(rng.randint(lo, hi), den)


def _feq_velocity(rho, j, g):
    """Velocity-space preconditioned equilibrium (Sec. 3.1), with the
    -3/2 u.u coefficient and the rho prefactor (reading of the printed -1/2)."""
    out = []
    jj = sum(x * x for x in j)
    for a, c in enumerate(E19):
        ej = sum(int(c[i]) * j[i] for i in range(3))
        out.append(W19_FRAC[a] * (rho + 3 * ej + (Fraction(9, 2) * ej * ej
                                                   - Fraction(3, 2) * jj) / (g * rho)))
    return out


def _matvec(T, v):
    return [sum(T[k][a] * v[a] for a in range(len(v))) for k in range(len(T))]


# ----------------------------------------------------------- basis / weights
def test_velocity_set_and_opposites():
    assert E19.shape == (19, 3) and len({tuple(v) for v in E19}) == 19
    n2 = (E19 ** 2).sum(axis=1)
    assert sorted(n2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert np.all(E19[OPP19] == -E19)
    assert np.all(E7[OPP7] == -E7)


def test_weights_isotropy():
    # sum w = 1, sum w c_i c_j = delta_ij / 3, fourth moment isotropic with c_s^4 = 1/9,
    # odd moments zero: what recovers Navier-Stokes; fixes w uniquely per shell.
    assert sum(W19_FRAC) == 1
    for i in range(3):
        for j in range(3):
            s2 = sum(W19_FRAC[a] * int(E19[a][i]) * int(E19[a][j]) for a in range(19))
            assert s2 == (Fraction(1, 3) if i == j else 0)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    s4 = sum(W19_FRAC[a] * int(E19[a][i]) * int(E19[a][j]) * int(E19[a][k])
                             * int(E19[a][l]) for a in range(19))
                    d = lambda p, q: 1 if p == q else 0
                    want = Fraction(d(i, j) * d(k, l) + d(i, k) * d(j, l) + d(i, l) * d(j, k), 9)
                    assert s4 == want
    assert abs(W19.sum() - 1) < 1e-15


def test_basis_orthogonal_with_integer_rows():
    n = len(T19_FRAC)
    for k in range(n):
        for a in range(19):
            assert T19_FRAC[k][a].denominator == 1
        for l in range(n):
            dot = sum(T19_FRAC[k][a] * T19_FRAC[l][a] for a in range(19))
            if k != l:
                assert dot == 0, (k, l)
    norms = [sum(v * v for v in r) for r in T19_FRAC]
    assert norms == [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]
    assert np.allclose(T19_INV, T19.T / np.array([float(x) for x in norms])[None, :], atol=1e-15)


def test_rest_state_moments():
    # T w rho0 = printed equilibrium at j = 0: (rho, -11 rho, 3 rho, 0, ...)
    eq, _ = _load_golden("d3q19_equilibrium_moments.txt")
    m = _matvec(T19_FRAC, W19_FRAC)
    want = [_eval(eq[k], rho=1, jx=0, jy=0, jz=0, jj=0, g=1) for k in range(19)]
    assert m == want


def test_d3q7_tables():
    assert W7.sum() == pytest.approx(1.0, abs=1e-15)
    # sum W e_i e_j = theta_m delta_ij (App. C identity)
    M = np.einsum("a,ai,aj->ij", W7, E7.astype(float), E7.astype(float))
    assert np.allclose(M, THETA_M * np.eye(3), atol=1e-15)


# ------------------------------------------------------------- equilibria
@pytest.mark.parametrize("seed", range(6))
def test_T_of_velocity_equilibrium_matches_printed_moments(seed):
    """P1: T f^eq*(velocity space) equals the printed moment list, exactly."""
    rng = random.Random(seed)
    eq, _ = _load_golden("d3q19_equilibrium_moments.txt")
    rho = 1 + _rand_frac(rng, -20, 20, 101)
    j = [_rand_frac(rng) for _ in range(3)]
    g = Fraction(rng.choice([1, 1, 2, 5, 10, 37]), rng.choice([1, 3, 10, 100]))
    if g > 1:
        g = 1 / g
    m = _matvec(T19_FRAC, _feq_velocity(rho, j, g))
    jj = sum(x * x for x in j)
    want = [_eval(eq[k], rho=rho, jx=j[0], jy=j[1], jz=j[2], jj=jj, g=g) for k in range(19)]
    assert m == want


@pytest.mark.parametrize("seed", range(4))
def test_oracle_equilibrium_moments_match_basis(seed):
    """The oracle's moment-space equilibria (full and deviation form) against
    T applied to the velocity-space equilibrium, in floating point."""
    rng = np.random.default_rng(seed)
    n = 50
    rho = 1 + 0.05 * rng.uniform(-1, 1, n)
    j = 0.05 * rng.uniform(-1, 1, (3, n))
    g = rng.choice([1.0, 0.5, 0.1, 0.01])
    w = W19[:, None]
    e = E19.astype(float)
    ej = e @ j
    jj = (j * j).sum(0)
    feq = w * (rho + 3 * ej + (4.5 * ej ** 2 - 1.5 * jj) / (g * rho))
    m = T19 @ feq
    assert np.allclose(glbe.meq_star_full(rho, j, g), m, rtol=0, atol=1e-13)
    dev = glbe.meq_star_dev(rho - 1.0, rho, j, g)
    rest = T19 @ W19
    assert np.allclose(dev + rest[:, None], m, rtol=0, atol=1e-13)


def test_printed_maxwellian_coefficient_reading():
    """G1: with the printed -1/(2 gamma) u.u the equilibrium does not carry the
    density (sum f^eq != rho); with -3/(2 gamma) and the rho prefactor it does."""
    rho, g = Fraction(11, 10), Fraction(1, 4)
    u = [Fraction(1, 50), Fraction(-1, 70), Fraction(1, 90)]
    uu = sum(x * x for x in u)
    printed = []
    for a, c in enumerate(E19):
        eu = sum(int(c[i]) * u[i] for i in range(3))
        printed.append(W19_FRAC[a] * (1 + 3 * eu + Fraction(9, 2) / g * eu * eu - Fraction(1, 2) / g * uu))
    assert sum(printed) != 1
    read = _feq_velocity(rho, [rho * x for x in u], g)
    assert sum(read) == rho


# ---------------------------------------------------------------- sources
@pytest.mark.parametrize("seed", range(6))
def test_T_of_velocity_source_matches_printed_moments(seed):
    """P2: T S (S_a = w[3(e-u) + 9(e.u)e].F, Sec. 2) equals App. A's list, exactly."""
    rng = random.Random(100 + seed)
    src, _ = _load_golden("d3q19_source_moments.txt")
    F = [_rand_frac(rng) for _ in range(3)]
    u = [_rand_frac(rng) for _ in range(3)]
    S = []
    for a, c in enumerate(E19):
        eF = sum(int(c[i]) * F[i] for i in range(3))
        eu = sum(int(c[i]) * u[i] for i in range(3))
        uF = sum(u[i] * F[i] for i in range(3))
        S.append(W19_FRAC[a] * (3 * (eF - uF) + 9 * eu * eF))
    m = _matvec(T19_FRAC, S)
    Fu = sum(F[i] * u[i] for i in range(3))
    env = dict(Fx=F[0], Fy=F[1], Fz=F[2], ux=u[0], uy=u[1], uz=u[2], Fu=Fu)
    want = [_eval(src[k], **env) for k in range(19)]
    assert m == want


@pytest.mark.parametrize("seed", range(6))
def test_preconditioned_source_inverse_matches_closed_form(seed):
    """P2: T^-1 P_S T S equals the velocity-space S* of Sec. 3.1
    (eq. precondsourcecorrect), exactly; P_S from the printed diagonal."""
    rng = random.Random(200 + seed)
    _, ps = _load_golden("d3q19_source_moments.txt")
    g = Fraction(rng.choice([1, 2, 3, 10, 20]), rng.choice([20, 30, 50]))
    PS = [Fraction(eval(t, {"__builtins__": {}}, {"g": g})) for t in ps]
    F = [_rand_frac(rng) for _ in range(3)]
    u = [_rand_frac(rng) for _ in range(3)]
    S, Sstar = [], []
    for a, c in enumerate(E19):
        eF = sum(int(c[i]) * F[i] for i in range(3))
        eu = sum(int(c[i]) * u[i] for i in range(3))
        uF = sum(u[i] * F[i] for i in range(3))
        S.append(W19_FRAC[a] * (3 * (eF - uF) + 9 * eu * eF))
        Sstar.append(W19_FRAC[a] * (3 * (eF - uF / g) / g + 9 * eu * eF / g ** 2))
    mS = _matvec(T19_FRAC, S)
    mS = [PS[k] * mS[k] for k in range(19)]
    norms = [sum(v * v for v in r) for r in T19_FRAC]
    back = [sum(T19_FRAC[k][a] * mS[k] / norms[k] for k in range(19)) for a in range(19)]
    assert back == Sstar


@pytest.mark.parametrize("seed", range(3))
def test_oracle_source_functions(seed):
    rng = np.random.default_rng(seed)
    F = rng.uniform(-1, 1, (3, 40))
    u = rng.uniform(-1, 1, (3, 40))
    assert np.allclose(T19 @ glbe.velocity_source(F, u), glbe.source_moments(F, u), atol=1e-13)
    _, ps = _load_golden("d3q19_source_moments.txt")
    g = 0.05
    PS = np.array([float(eval(t, {"__builtins__": {}}, {"g": g})) for t in ps])
    assert np.allclose(glbe.source_precond_diag(g), PS, rtol=1e-15)


def test_rates_match_printed():
    with open(os.path.join(GOLDEN, "d3q19_rates.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    nu, g = 0.131, 0.05
    s = glbe.rates(nu, g)
    for k, v in rows:
        want = 1.0 / (3 * nu / g + 0.5) if v == "shear" else float(v)
        assert s[int(k)] == pytest.approx(want, rel=1e-15)
