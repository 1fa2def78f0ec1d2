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

import numpy as np

from . import LbmError, Simulation, batch_run, default_rates

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


# ------------------------------------------------------------ batched ----
def march_batch(points, H=64, width=4, max_steps=20000, tol=1e-9, storage="f64",
                rates_mode="paper", launch=None):
    """Verdicts for many (nu, u_max, gamma) points in one batched march (one
    launch per step for all points).  Returns [(STABLE | UNSTABLE, step)]."""
    members = [(g, default_rates(nu, g, rates_mode), (poiseuille_force(nu, um, H), 0.0, 0.0))
               for nu, um, g in points]
    out = batch_run((width, width, H), ("periodic", "periodic", "wall"), members,
                    storage=storage, tol=tol, max_steps=max_steps, launch=launch)
    return [(UNSTABLE if v == "unstable" else STABLE, step) for v, step, _ in out]


def envelope_batched(nus, u_maxes, lo=1e-3, hi=1.0, per_round=15, rounds=2, **kw):
    """gamma_min for every (nu, u_max) by k-section in log(gamma): each round
    evaluates per_round gammas inside every point's bracket, all points and
    gammas in one batched march.  The first round also covers lo and hi.  After
    r rounds the bracket is (hi/lo)^(1/(per_round+1)^r) wide.  Returns the same
    records as envelope()."""
    keys = [(nu, um) for nu in nus for um in u_maxes]
    brk = {k: (np.log(lo), np.log(hi)) for k in keys}
    state = {k: None for k in keys}  # None: open; math.inf: hi unstable; lo: lo stable
    runs = {k: 0 for k in keys}
    for r in range(rounds):
        pts, owner = [], []
        for k in keys:
            if state[k] is not None:
                continue
            a, b = brk[k]
            if r == 0:
                grid = np.linspace(a, b, per_round + 2)
            else:
                grid = np.linspace(a, b, per_round + 2)[1:-1]
            for x in grid:
                pts.append((k[0], k[1], float(np.exp(x))))
                owner.append((k, x))
        if not pts:
            break
        verdicts = march_batch(pts, **kw)
        by_key = {}
        for (k, x), (v, _) in zip(owner, verdicts):
            by_key.setdefault(k, []).append((x, v))
            runs[k] += 1
        for k, lst in by_key.items():
            a, b = brk[k]
            if r == 0:
                if lst[-1][1] == UNSTABLE:      # hi itself unstable
                    state[k] = math.inf
                    continue
                if lst[0][1] == STABLE:         # lo already stable
                    state[k] = lo
                    continue
            lst = [(a, UNSTABLE)] + lst + [(b, STABLE)] if r > 0 else lst
            unstable = [x for x, v in lst if v == UNSTABLE]
            a_new = max(unstable)
            b_new = min(x for x, v in lst if v == STABLE and x > a_new)
            brk[k] = (a_new, b_new)
    out = []
    for k in keys:
        g = state[k] if state[k] is not None else float(np.exp(brk[k][1]))
        out.append({"nu": k[0], "u_max": k[1], "gamma_min": g, "runs": runs[k]})
    return out
