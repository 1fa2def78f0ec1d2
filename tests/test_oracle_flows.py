"""Pins of the oracle's full time march against closed forms and invariants.

* Plane Poiseuille between halfway bounce-back plates (Sec. 5): with the
  energy-flux and third-order rates tied so that
  Lambda = (3 nu/gamma)(1/s_q - 1/2) is fixed, the x-momentum is exactly
      j_x(z) = F z (H - z) / (2 nu) + F (16 Lambda - 3) / (24 nu),  z = k + 1/2,
  at every node and every gamma (the x-odd populations obey a linear
  recurrence there; Lambda = 3/16 gives the parabola u_max = F L^2 / (2 nu)
  with H = 2L, Sec. 5).
* Square duct with F_x = F0 sin(k y)(1 + cos(k z)/2): u.grad u = 0, so the
  Stokes solution is exact; second-order convergence.
* Hartmann flow (Sec. 5) against the textbook profiles for insulating walls;
  second-order convergence, independence of chi, gamma, gamma_m.
* Vector LKE: moment constraints of g^eq* (App. C), and the decay of a
  diffusing mode against the exact eigenvalue of the one-step amplification
  matrix.
"""
import numpy as np
import pytest

from oracle import glbe, mhd
from oracle.lattice import E7, Q7, THETA_M, W7

PER, WALL = glbe.PERIODIC, glbe.WALL


def _poiseuille(H, nu, gamma, F, s, tol=1e-15, max_steps=200000):
    fl = glbe.Flow((1, 1, H), (PER, PER, WALL), np.array([F, 0.0, 0.0]), gamma, s)
    assert fl.run_to(tol, max_steps)
    f = glbe.stream(fl.post, fl.bc)
    return fl, glbe.fields(f, fl.F, gamma)


@pytest.mark.parametrize("H,gamma,Lam", [(8, 1.0, 3 / 16), (8, 0.5, 0.5), (16, 0.1, 3 / 16),
                                         (16, 0.1, 1.0), (12, 0.25, 0.3)])
def test_poiseuille_exact_in_fixed_lambda_mode(H, gamma, Lam):
    nu, F = 0.1, 1e-6
    s = glbe.rates(nu, gamma, "lambda", Lam)
    fl, (drho, rho, j, u) = _poiseuille(H, nu, gamma, F, s)
    z = np.arange(H) + 0.5
    exact = F * z * (H - z) / (2 * nu) + F * (16 * Lam - 3) / (24 * nu)
    err = np.max(np.abs(j[0][:, 0, 0] - exact)) / np.max(exact)
    assert err < 1e-11, err
    assert np.max(np.abs(j[1])) < 1e-18 and np.max(np.abs(j[2])) < 1e-18


def test_poiseuille_paper_rates_error_linear_in_nu_over_gamma():
    """Sec. 5 (fig. Poiseuille_error): with the paper's fixed kinetic rates the
    centre-velocity error is linear in nu/gamma and small.  The signed error is
    affine in nu/gamma (the wall slip scales with 3 nu/gamma); in the paper's
    regime (nu/gamma >= 1) it grows with nu/gamma."""
    H, nu, F = 16, 0.1, 1e-6
    ratios, errs = [], []
    for gamma in (0.1, 0.05, 0.02):
        s = glbe.rates(nu, gamma)
        fl, (drho, rho, j, u) = _poiseuille(H, nu, gamma, F, s, tol=1e-12)
        z = np.arange(H) + 0.5
        par = F * z * (H - z) / (2 * nu)
        errs.append((j[0][H // 2, 0, 0] - par[H // 2]) / par[H // 2])
        ratios.append(nu / gamma)
    assert 0 < errs[0] < errs[1] < errs[2] < 0.05, errs
    slope1 = (errs[1] - errs[0]) / (ratios[1] - ratios[0])
    slope2 = (errs[2] - errs[1]) / (ratios[2] - ratios[1])
    assert abs(slope1 / slope2 - 1) < 0.02, (slope1, slope2)


def test_preconditioning_reduces_steps_to_steady_state():
    """P13 (qualitative, Sec. 5): steps to a 1e-10 residual fall roughly as 1/gamma."""
    H, nu, F = 16, 0.1, 1e-6
    steps = []
    for gamma in (1.0, 0.1):
        s = glbe.rates(nu, gamma, "lambda", 3 / 16)
        fl, _ = _poiseuille(H, nu, gamma, F, s, tol=1e-10)
        steps.append(fl.t)
    assert steps[0] > 5 * steps[1], steps


def test_mass_is_conserved():
    rng = np.random.default_rng(5)
    shape = (4, 5, 6)
    post = 1e-3 * rng.uniform(-1, 1, (19, 6, 5, 4))
    F = 1e-4 * rng.uniform(-1, 1, (3, 6, 5, 4))
    m0 = post.sum()
    fl = glbe.Flow(shape, (PER, WALL, WALL), F, 0.2, glbe.rates(0.05, 0.2), post=post)
    fl.step(200)
    assert abs(fl.post.sum() - m0) < 1e-14


def _duct_exact(n, nu, F0):
    L = n
    y = np.arange(n) + 0.5
    z = np.arange(n) + 0.5
    k = 2 * np.pi / L
    A = F0 / (nu * k * k)
    B = 0.5 * F0 / (nu * 2 * k * k)
    C = -(A + B) / np.cosh(k * L / 2)
    h = A + B * np.cos(k * z) + C * np.cosh(k * (z - L / 2))
    return np.sin(k * y)[None, :] * h[:, None]


def _duct_force(n, F0):
    y = np.arange(n) + 0.5
    z = np.arange(n) + 0.5
    F = np.zeros((3, n, n, 1))
    F[0] = (F0 * np.sin(2 * np.pi * y / n)[None, :]
            * (1 + 0.5 * np.cos(2 * np.pi * z / n))[:, None])[:, :, None]
    return F


def _duct(n, gamma, s, nu=0.131, F0=1e-5, tol=1e-11):
    fl = glbe.Flow((1, n, n), (PER, WALL, WALL), _duct_force(n, F0), gamma, s)
    assert fl.run_to(tol, 200000)
    return fl


def test_duct_second_order_convergence():
    nu, F0, gamma = 0.131, 1e-5, 0.1
    errs = []
    for n in (16, 32):
        fl = _duct(n, gamma, glbe.rates(nu, gamma, "lambda", 3 / 16), nu, F0)
        u = fl.velocity()[0][:, :, 0]
        ex = _duct_exact(n, nu, F0)
        errs.append(np.sqrt(np.mean((u - ex) ** 2)) / np.max(np.abs(ex)))
    assert errs[1] < 0.006
    assert 3.5 < errs[0] / errs[1] < 4.6, errs


def test_duct_flow_rate_vanishes_by_antisymmetry():
    nu, gamma = 0.131, 0.2
    fl = _duct(16, gamma, glbe.rates(nu, gamma), nu)
    q = fl.flow_rate()
    assert abs(q) < 1e-16


def test_steady_state_independent_of_gamma_in_fixed_lambda_mode():
    """P8: preconditioning changes the transient, not the steady state (App. B);
    in fixed-Lambda mode the discrete steady duct flow agrees across gamma to
    the compressibility level (here Ma ~ 2e-3, so ~1e-6 relative)."""
    nu, n = 0.131, 16
    us = []
    for gamma in (1.0, 0.25):
        fl = _duct(n, gamma, glbe.rates(nu, gamma, "lambda", 0.5), nu, tol=1e-12)
        us.append(fl.velocity()[0])
    rel = np.max(np.abs(us[0] - us[1])) / np.max(np.abs(us[0]))
    assert rel < 2e-5, rel


# ------------------------------------------------------------------- MHD ---
def _hartmann(L, Ha, chi, gamma, gamma_m, nu=0.1, eta=0.025, F=1e-5, tol=1e-11,
              max_steps=20000):
    B0 = Ha * np.sqrt(eta * nu) / L
    s = glbe.rates(nu, gamma, "lambda", 3 / 16)
    fl = mhd.MHDFlow((1, 2 * L, 1), (PER, WALL, PER), np.array([F, 0, 0]), gamma, s,
                     gamma_m, chi, eta, np.array([0, B0, 0]))
    ok = fl.run_to(tol, max_steps)
    y = np.arange(2 * L) + 0.5 - L
    uex = F * L * L / (nu * Ha) * (np.cosh(Ha) - np.cosh(Ha * y / L)) / np.sinh(Ha)
    bex = chi * F * L / B0 * (np.sinh(Ha * y / L) / np.sinh(Ha) - y / L)
    return ok, fl, fl.u[0][0, :, 0], fl.B[0][0, :, 0], uex, bex


def test_hartmann_second_order_convergence():
    eu, eb = [], []
    for L in (8, 16):
        ok, fl, u, b, uex, bex = _hartmann(L, 5.0, 0.0025, 0.1, 0.1)
        assert ok
        eu.append(np.sqrt(np.mean((u - uex) ** 2)) / np.max(uex))
        eb.append(np.sqrt(np.mean((b - bex) ** 2)) / np.max(np.abs(bex)))
    assert eu[1] < 0.007 and eb[1] < 0.009, (eu, eb)
    assert 3.5 < eu[0] / eu[1] < 4.5 and 3.5 < eb[0] / eb[1] < 4.5, (eu, eb)


def test_hartmann_velocity_independent_of_chi_and_field_proportional():
    ok1, _, u1, b1, _, _ = _hartmann(8, 5.0, 0.0025, 0.1, 0.1)
    ok2, _, u2, b2, _, _ = _hartmann(8, 5.0, 0.025, 0.1, 0.1)
    assert ok1 and ok2
    assert np.max(np.abs(u1 - u2)) / np.max(u1) < 1e-4
    assert np.max(np.abs(b1 / 0.0025 - b2 / 0.025)) / np.max(np.abs(b1 / 0.0025)) < 1e-3


def test_hartmann_steady_state_independent_of_preconditioning():
    _, _, u1, b1, _, _ = _hartmann(8, 10.0, 0.0025, 0.1, 0.1, tol=1e-12)
    _, _, u2, b2, _, _ = _hartmann(8, 10.0, 0.0025, 0.5, 0.25, tol=1e-12)
    assert np.max(np.abs(u1 - u2)) / np.max(u1) < 1e-4
    assert np.max(np.abs(b1 - b2)) / np.max(np.abs(b1)) < 1e-3


def _hartmann_extended(L, d, Ha=5.0, chi=0.0025, gamma=0.1, gamma_m=0.1, nu=0.1, eta=0.025,
                       F=1e-5, tol=1e-11):
    """Hartmann channel whose induction lattice extends d nodes beyond each wall
    (zero induced field at the outer boundary, u = 0 outside the fluid).

    Closed form (derived for this pin): outside the fluid the steady induction
    equation reduces to b'' = 0, so b is linear there and vanishes at the outer
    boundary; with the flux eta b' + B0 u = C continuous across the wall the
    current that returns through the outer layer gives
        u = U (1 - cosh(Ha y/L)/cosh Ha),
        U = (F L^2 / (nu Ha^2)) / (1 - (L/(L+d)) (1 - tanh(Ha)/Ha)),
        C = B0 Q / (2 (L + d)),  Q = 2 L U (1 - tanh(Ha)/Ha),
    and b/chi = [d C + C (y+L) - B0 U ((y+L) - (L/Ha)(sinh(Ha y/L) + sinh Ha)/cosh Ha)]/eta
    inside, continued linearly with slope C/eta outside.  d = 0 is the
    insulating-wall profile; d -> inf the perfectly conducting one."""
    B0 = Ha * np.sqrt(eta * nu) / L
    s = glbe.rates(nu, gamma, "lambda", 3 / 16)
    fl = mhd.MHDFlow((1, 2 * L + 2 * d, 1), (PER, WALL, PER), np.array([F, 0, 0]), gamma, s,
                     gamma_m, chi, eta, np.array([0, B0, 0]), pad=(0, d, 0))
    ok = fl.run_to(tol, 60000)
    T = np.tanh(Ha)
    U = F * L * L / (nu * Ha * Ha) / (1 - (L / (L + d)) * (1 - T / Ha))
    y = np.arange(2 * L) + 0.5 - L
    uex = U * (1 - np.cosh(Ha * y / L) / np.cosh(Ha))
    C = B0 * 2 * L * U * (1 - T / Ha) / (2 * (L + d))

    def b_in(z):
        return (d * C + C * (z + L)
                - B0 * U * ((z + L) - (L / Ha) * (np.sinh(Ha * z / L) + np.sinh(Ha)) / np.cosh(Ha))) / eta

    yy = np.arange(2 * L + 2 * d) + 0.5 - L - d
    b = np.where(yy > L, b_in(L) + (yy - L) * C / eta,
                 np.where(yy < -L, b_in(-L) + (yy + L) * C / eta, b_in(yy)))
    u = fl.u[0][0, :, 0]
    bb = fl.B[0][0, :, 0]
    eu = np.sqrt(np.mean((u - uex) ** 2)) / np.max(uex)
    eb = np.sqrt(np.mean((bb - chi * b) ** 2)) / np.max(np.abs(chi * b))
    return ok, eu, eb


def test_hartmann_extended_magnetic_domain_closed_form():
    """Extended induction lattice (Sec. 5, MHD cavity): the return current through
    the outer layer lowers the flow by the factor in the closed form; the error
    against it is second order."""
    ok1, eu1, eb1 = _hartmann_extended(8, 8)
    ok2, eu2, eb2 = _hartmann_extended(16, 16)
    assert ok1 and ok2
    assert eu2 < 0.002 and eb2 < 0.002, (eu2, eb2)
    assert 3.5 < eu1 / eu2 < 4.5 and 3.5 < eb1 / eb2 < 4.5, (eu1, eu2, eb1, eb2)


def test_printed_current_contraction_is_unstable(monkeypatch):
    """Planted mistake (on the oracle): contracting as printed flips the sign of
    J; the Lorentz force then feeds the flow and the march diverges."""
    monkeypatch.setattr(mhd, "CURRENT_SIGN", 1.0)
    with np.errstate(all="ignore"):
        ok, fl, u, b, uex, bex = _hartmann(8, 5.0, 0.0025, 0.1, 0.1, tol=1e-10, max_steps=1500)
    assert (not ok) or (not np.all(np.isfinite(u))) or np.max(np.abs(u - uex)) > 0.5 * np.max(uex)


def test_lke_equilibrium_moment_constraints():
    """App. C: sum_a g^eq = B, sum_a e_k g^eq_j = (chi/gamma_m)(u_k B_j - B_k u_j),
    sum_a e_j e_k g^eq_i = theta_m delta_jk B_i."""
    rng = np.random.default_rng(2)
    B = rng.uniform(-1, 1, (3, 20))
    u = rng.uniform(-1, 1, (3, 20))
    chi, gm = 0.3, 0.2
    geq = mhd.g_eq(B, u, chi, gm)
    assert np.allclose(geq.sum(axis=1), B, atol=1e-15)
    e = E7.astype(float)
    first = np.einsum("ak,jan->kjn", e, geq)
    want = chi / gm * (u[:, None, :] * B[None, :, :] - B[:, None, :] * u[None, :, :])
    assert np.allclose(first, want, atol=1e-14)
    second = np.einsum("aj,ak,ian->jkin", e, e, geq)
    want2 = THETA_M * np.eye(3)[:, :, None, None] * B[None, None, :, :]
    assert np.allclose(second, want2, atol=1e-15)


def test_lke_diffusion_decay_matches_amplification_eigenvalue():
    """With u = 0 a mode B_z ~ sin(k x) decays by the dominant eigenvalue of the
    7x7 one-step map P(k)(I - (I - W 1^T)/tau_m); to leading order
    1 - (eta/gamma_m) k^2 (the preconditioned induction equation, Sec. 4)."""
    nx, eta, gm = 32, 0.02, 0.25
    tau = mhd.tau_m(eta, gm)
    k = 2 * np.pi / nx
    P = np.diag(np.exp(-1j * k * E7[:, 0]))
    C = np.eye(Q7) - (np.eye(Q7) - np.outer(W7, np.ones(Q7))) / tau
    lam = np.linalg.eigvals(P @ C)
    lam_max = lam[np.argmax(np.abs(lam))].real
    x = np.arange(nx)
    g = np.zeros((3, Q7, 1, 1, nx))
    for a in range(Q7):
        g[2, a, 0, 0, :] = W7[a] * np.sin(k * x)
    u0 = np.zeros((3, 1, 1, nx))
    amps = []
    for n in range(400):
        g = mhd.stream_g(g, (PER, PER, PER), np.zeros(3))
        B = g.sum(axis=1)
        g = mhd.collide_g(g, B, u0, 1.0, gm, eta)
        amps.append((B[2, 0, 0, :] * np.sin(k * x)).sum())
    ratio = amps[-1] / amps[-2]
    assert abs(ratio - lam_max) < 1e-12
    assert abs((1 - lam_max) / ((eta / gm) * k * k) - 1) < 0.05


@pytest.mark.parametrize("gamma", [1.0, 0.2])
def test_couette_exact_with_moving_wall(gamma):
    """Link bounce-back with wall momentum (Sec. 5, cavity lid): plane Couette
    flow between a fixed and a moving plate is linear, and halfway bounce-back
    places both walls exactly, so j_x(z) = U z / H at every node and gamma."""
    H, U, nu = 8, 0.01, 0.1
    wu = np.zeros((6, 3))
    wu[5] = [U, 0.0, 0.0]
    fl = glbe.Flow((1, 1, H), (PER, PER, WALL), np.zeros(3), gamma, glbe.rates(nu, gamma),
                   wall_u=wu)
    assert fl.run_to(1e-14, 200000)
    f = glbe.stream(fl.post, fl.bc, wall_u=wu)
    _, _, j, _ = glbe.fields(f, fl.F, gamma)
    z = np.arange(H) + 0.5
    assert np.max(np.abs(j[0][:, 0, 0] - U * z / H)) < 1e-11 * U


def test_moving_wall_conserves_mass_when_tangential():
    """A tangentially moving wall adds no mass: the wall terms of a link pair cancel."""
    rng = np.random.default_rng(8)
    post = 1e-3 * rng.uniform(-1, 1, (19, 5, 4, 3))
    wu = np.zeros((6, 3))
    wu[5] = [0.02, -0.01, 0.0]
    wu[2] = [0.0, 0.0, 0.015]
    f = glbe.stream(post, (PER, WALL, WALL), wall_u=wu)
    assert abs(f.sum() - post.sum()) < 1e-15


def test_lke_keeps_total_flux_and_small_divergence():
    """Induction lattice (Sec. 4): in a periodic box the total flux sum B is
    conserved exactly (collision keeps sum_a g = B, streaming moves it), and a
    smooth flow started from a uniform field keeps the discrete divergence of B
    at truncation level, far below the curl of the induced field (the
    continuum equation carries div B unchanged, Sec. 4)."""
    L = 8
    shape = (L, L, L)
    bc = (PER, PER, PER)
    B0 = np.array([0.01, 0.02, 0.015])
    p = dict(gamma=1.0, s=glbe.rates(0.05, 1.0), gamma_m=1.0, chi=1.0, eta=0.05, B_wall=B0)
    k = 2 * np.pi / L
    z, y, x = np.meshgrid(*(np.arange(L) + 0.5,) * 3, indexing="ij")
    F = 1e-5 * np.stack([np.sin(k * y) * np.cos(k * z), np.sin(k * z) * np.cos(k * x),
                         np.sin(k * x) * np.cos(k * y)])
    f = np.zeros((19,) + x.shape)
    g = mhd.initial_g(shape, B0)
    for _ in range(16):
        f, g, u, B = mhd.step(f, g, F, p, bc)
    total = g.sum(axis=(1, 2, 3, 4))
    assert np.allclose(total, B0 * L ** 3, rtol=0, atol=1e-15 * L ** 3)

    def d(a, ax):
        return (np.roll(a, -1, ax) - np.roll(a, 1, ax)) / 2

    div = d(B[0], 2) + d(B[1], 1) + d(B[2], 0)
    curl = np.stack([d(B[2], 1) - d(B[1], 0), d(B[0], 0) - d(B[2], 2), d(B[1], 2) - d(B[0], 1)])
    assert np.abs(curl).max() > 1e-6
    assert np.abs(div).max() < 1e-3 * np.abs(curl).max()
