"""Stability envelope of the preconditioned GLBE (Sec. 5, the map of the
smallest usable preconditioning parameter against the maximum velocity of
body-force Poiseuille flow for several viscosities).

Each classification runs the library's time march on a small channel (walls
normal to z, periodic x and y; default 4 x 4 x 64) driven by the force that
gives the requested centre velocity of the analytic parabola,
F = 8 nu u_max / H^2, and reads the library's instability verdict
(non-finite values, or the residual exceeding 10^3 times its running minimum).
A run that reaches the residual tolerance, or survives max_steps without either
sign, is counted stable.  gamma_min bisects in log(gamma) assuming the stable
set is gamma >= gamma_min.
"""
import math

from . import LbmError, Simulation, default_rates

STABLE, UNSTABLE = "stable", "unstable"


def poiseuille_force(nu, u_max, H):
    """Force density that gives centre velocity u_max between walls H apart."""
    return 8.0 * nu * u_max / (H * H)


def march(nu, u_max, gamma, H=64, width=4, max_steps=20000, tol=1e-9, storage="f64",
          rates_mode="paper"):
    """(verdict, steps) for one (nu, u_max, gamma): steps is the step at which
    the run converged, blew up, or was stopped."""
    F = poiseuille_force(nu, u_max, H)
    sim = Simulation((width, width, H), ("periodic", "periodic", "wall"), gamma,
                     default_rates(nu, gamma, rates_mode), storage=storage, force=(F, 0.0, 0.0))
    try:
        sim.run_to_residual(tol, max_steps, poll_every=1000)
        return STABLE, sim.t
    except LbmError as e:
        if e.status == -4:
            return UNSTABLE, sim.t
        raise
    finally:
        sim.close()


def classify(nu, u_max, gamma, **kw):
    """STABLE or UNSTABLE for one (nu, u_max, gamma)."""
    return march(nu, u_max, gamma, **kw)[0]


def gamma_min(nu, u_max, lo=1e-3, hi=1.0, iters=8, **kw):
    """Smallest stable gamma in [lo, hi] to a factor (hi/lo)^(2^-iters).

    Returns (gamma_min, n_classified).  If hi itself is unstable returns
    (inf, n); if lo is stable returns (lo, n)."""
    n = 0
    if classify(nu, u_max, hi, **kw) == UNSTABLE:
        return math.inf, 1
    n += 1
    if classify(nu, u_max, lo, **kw) == STABLE:
        return lo, n + 1
    n += 1
    a, b = math.log(lo), math.log(hi)  # a unstable, b stable
    for _ in range(iters):
        m = 0.5 * (a + b)
        n += 1
        if classify(nu, u_max, math.exp(m), **kw) == STABLE:
            b = m
        else:
            a = m
    return math.exp(b), n


def envelope(nus, u_maxes, **kw):
    """[{nu, u_max, gamma_min, runs}] over the grid of viscosities and velocities."""
    out = []
    for nu in nus:
        for um in u_maxes:
            g, n = gamma_min(nu, um, **kw)
            out.append({"nu": nu, "u_max": um, "gamma_min": g, "runs": n})
    return out
