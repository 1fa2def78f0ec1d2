"""Two-dimensional variants: the preconditioned D2Q9 GLBE with forcing and the
preconditioned D2Q5 vector induction LKE.  Plain FP64 oracle (test
infrastructure only, like the rest of this package).

Paper passages followed:

* Sec. 2 (eq. velocityd2q9): the D2Q9 velocity set.
* Sec. 3: the preconditioned D2Q9 equilibrium moments (rho, e, e2, j_x, q_x,
  j_y, q_y, p_xx, p_xy), the preconditioned D2Q9 source moments, and the D2Q9
  rates (shear 1/s = 3 nu/gamma + 1/2 for p_xx and p_xy; kinetic 1.63, 1.14,
  1.92, 1.92 for e, e2, q_x, q_y).
* Sec. 4 (eq. velocityd2q5, eq. mageqmoment, eq. mrelaxationtime): D2Q5
  populations for the field, W0 = 1/N_m, W = 1/(2 N_m), theta_m = 1/N_m, N_m = 3.

Readings (the paper is silent or ambiguous here):

* Basis: the nine moments are named but the rows are not printed.  They are the
  orthogonal rows of the cited D2Q9 construction, written as polynomials in the
  velocity: 1, 3|c|^2 - 4, (9|c|^4 - 21|c|^2 + 8)/2, c_x, (3|c|^2 - 5) c_x, c_y,
  (3|c|^2 - 5) c_y, c_x^2 - c_y^2, c_x c_y.  Tests check that they reproduce the
  printed equilibria and source lists exactly.
* Weights 4/9, 1/9, 1/36: forced by the printed rest-state moments e = -2 rho,
  e2 = rho (sum w = 1, sum w |c|^2 = 2/3, sum w |c|^4 = 8/9).
* P_S for D2Q9 is read off the printed preconditioned source list: 1/gamma on
  j and q, 1/gamma^2 on e, e2, p_xx, p_xy.
* The paper also gives a bulk-viscosity formula for s_e; as in 3D the fixed
  kinetic value is used.
* In 2D the field is in-plane, B = (B_x, B_y), the current is out of plane,
  J_z = (curl B)_z / (mu chi), and the Lorentz force is J_z (-B_y, B_x).  The
  current is taken from the non-equilibrium first moment with the sign reading
  of the 3D oracle, and the flow/field loop is solved exactly per node (2x2).
* Walls: halfway bounce-back for f, anti-bounce-back with B = B0 for g.
"""
from fractions import Fraction

import numpy as np

from . import glbe

PERIODIC, WALL = glbe.PERIODIC, glbe.WALL
CURRENT_SIGN = -1.0

# ---------------------------------------------------------------- D2Q9 -----
# rest; axis; diagonals; opposite directions adjacent.
E9 = np.array([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1),
               (1, 1), (-1, -1), (1, -1), (-1, 1)], dtype=np.int64)
Q9 = 9
OPP9 = np.array([0, 2, 1, 4, 3, 6, 5, 8, 7])
W9_FRAC = [{0: Fraction(4, 9), 1: Fraction(1, 9), 2: Fraction(1, 36)}[int(c @ c)] for c in E9]
W9 = np.array([float(w) for w in W9_FRAC])


def _rows():
    def c2(x, y):
        return x * x + y * y
    return [
        ("rho", lambda x, y: 1),
        ("e", lambda x, y: 3 * c2(x, y) - 4),
        ("e2", lambda x, y: Fraction(9 * c2(x, y) ** 2 - 21 * c2(x, y) + 8, 2)),
        ("jx", lambda x, y: x),
        ("qx", lambda x, y: (3 * c2(x, y) - 5) * x),
        ("jy", lambda x, y: y),
        ("qy", lambda x, y: (3 * c2(x, y) - 5) * y),
        ("pxx", lambda x, y: x * x - y * y),
        ("pxy", lambda x, y: x * y),
    ]


MOMENT_NAMES9 = [n for n, _ in _rows()]
T9_FRAC = [[Fraction(p(int(c[0]), int(c[1]))) for c in E9] for _, p in _rows()]
T9 = np.array([[float(v) for v in r] for r in T9_FRAC])
T9_INV = np.linalg.inv(T9)

# ---------------------------------------------------------------- D2Q5 -----
E5 = np.array([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)], dtype=np.int64)
Q5 = 5
OPP5 = np.array([0, 2, 1, 4, 3])
N_M2 = 3
W5 = np.array([1.0 / N_M2] + [1.0 / (2 * N_M2)] * 4)
THETA_M2 = 1.0 / N_M2


def _embed(e):
    """2D velocities as 3D ones (c_z = 0) for the shared streaming routine."""
    return np.concatenate([e, np.zeros((len(e), 1), dtype=np.int64)], axis=1)


# ---------------------------------------------------------------- rates ----
def rates(nu, gamma, mode="paper", Lambda=None):
    """Preconditioned D2Q9 rates (Sec. 3): s_e = 1.63, s_e2 = 1.14,
    s_q = 1.92 (mode "paper"), s_pxx = s_pxy = 1/(3 nu/gamma + 1/2).

    mode="lambda": s_q from (3 nu/gamma)(1/s_q - 1/2) = Lambda (gamma-independent
    wall location of the halfway bounce-back).  Conserved modes are set to 1."""
    s = np.ones(Q9)
    s_nu = 1.0 / (3.0 * nu / gamma + 0.5)
    s[7] = s[8] = s_nu
    s[1], s[2] = 1.63, 1.14
    if mode == "paper":
        s[4] = s[6] = 1.92
    elif mode == "lambda":
        s[4] = s[6] = 1.0 / (Lambda * gamma / (3.0 * nu) + 0.5)
    else:
        raise ValueError(mode)
    return s


# --------------------------------------------------------------- moments ---
def fields(d, F, gamma, rho0=1.0):
    """rho = rho0 + sum d, j = sum f e + F/(2 gamma), u = j/rho.  d: (9, ...), F: (2, ...)."""
    drho = d.sum(axis=0)
    rho = rho0 + drho
    j = np.tensordot(E9.T.astype(float), d, axes=(1, 0)) + F / (2.0 * gamma)
    return drho, rho, j, j / rho


def meq_star(rho, j, gamma):
    """Preconditioned D2Q9 equilibrium moments (Sec. 3 list)."""
    jx, jy = j
    jj = (jx * jx + jy * jy) / (gamma * rho)
    out = [rho, -2.0 * rho + 3.0 * jj, rho - 3.0 * jj, jx, -jx, jy, -jy,
           (jx * jx - jy * jy) / (gamma * rho), jx * jy / (gamma * rho)]
    return np.stack([np.broadcast_to(v, np.shape(rho)) for v in out])


def meq_star_dev(drho, rho, j, gamma):
    """meq*(rho, j) - T w rho0 written out (T w rho0 = rho0 (1, -2, 1, 0, ...), the
    printed list at rest), so that deviations keep full precision."""
    jx, jy = j
    jj = (jx * jx + jy * jy) / (gamma * rho)
    out = [drho, -2.0 * drho + 3.0 * jj, drho - 3.0 * jj, jx, -jx, jy, -jy,
           (jx * jx - jy * jy) / (gamma * rho), jx * jy / (gamma * rho)]
    return np.stack([np.broadcast_to(v, np.shape(drho)) for v in out])


def source_moments(F, u):
    """Moments of the source term at gamma = 1 (the D2Q9 list of Sec. 3 with gamma = 1)."""
    Fx, Fy = F
    ux, uy = u
    Fu = Fx * ux + Fy * uy
    out = [0.0 * Fu, 6.0 * Fu, -6.0 * Fu, Fx, -Fx, Fy, -Fy,
           2.0 * (Fx * ux - Fy * uy), Fx * uy + Fy * ux]
    return np.stack([np.broadcast_to(v, np.shape(Fu)) for v in out])


def source_precond_diag(gamma):
    """P_S for D2Q9: S^* = P_S S^ (read off the printed preconditioned list)."""
    g1, g2 = 1.0 / gamma, 1.0 / gamma ** 2
    return np.array([1.0, g2, g2, g1, g1, g1, g1, g2, g2])


def velocity_source(F, u):
    """S_alpha = w [3 (e - u) + 9 (e.u) e] . F (Sec. 2), D2Q9."""
    e = E9.astype(float)
    eF = np.tensordot(e, F, axes=(1, 0))
    eu = np.tensordot(e, u, axes=(1, 0))
    uF = (u * F).sum(axis=0)
    w = W9.reshape((Q9,) + (1,) * (np.ndim(F) - 1))
    return w * (3.0 * (eF - uF) + 9.0 * eu * eF)


# ------------------------------------------------------------- collision ---
def collide(d, F, gamma, s, rho0=1.0):
    """One preconditioned D2Q9 collision with forcing (Sec. 3, eq. prelax_term):
    m~ = m - s (m - meq*) + (1 - s/2) P_S S^.  d: deviations f - w rho0; both m
    and meq* are taken relative to the rest state (T d and meq*_dev)."""
    drho, rho, j, u = fields(d, F, gamma, rho0)
    neq = np.tensordot(T9, d, axes=(1, 0)) - meq_star_dev(drho, rho, j, gamma)
    sk = np.asarray(s, dtype=float).reshape((Q9,) + (1,) * (d.ndim - 1))
    S = source_precond_diag(gamma).reshape(sk.shape) * source_moments(F, u)
    dm = -sk * neq + (1.0 - 0.5 * sk) * S
    return d + np.tensordot(T9_INV, dm, axes=(1, 0))


def stream(post, bc):
    """Pull streaming with periodic wrap / halfway bounce-back.  post: (9, ny, nx);
    bc: (bcx, bcy)."""
    out = glbe.stream(post[:, None], (bc[0], bc[1], PERIODIC), e=_embed(E9), opp=OPP9)
    return out[:, 0]


def step(post, F, gamma, s, bc, rho0=1.0):
    f = stream(post, bc)
    u = fields(f, F, gamma, rho0)[3]
    return collide(f, F, gamma, s, rho0), u


def step_nodes(post, F, gamma, s, bc, nodes, rho0=1.0):
    """One step evaluated only at the given nodes (for large-lattice parity):
    each population pulled from its upstream node (periodic wrap), or from the
    opposite direction at the node itself where the link crosses a wall
    (halfway bounce-back), then the collision at those nodes.  nodes: (n, 2)
    integer (x, y); post (9, ny, nx); F (2,) or (2, ny, nx).  Returns (9, n)."""
    nodes = np.asarray(nodes)
    ny, nx = post.shape[1:]
    n = len(nodes)
    nodes3 = np.stack([nodes[:, 0], nodes[:, 1], np.zeros(n, dtype=nodes.dtype)], axis=1)
    dims, bc3 = (nx, ny, 1), (bc[0], bc[1], PERIODIC)
    e3 = _embed(E9)
    x, y = nodes[:, 0], nodes[:, 1]
    f = np.empty((Q9, n))
    for a in range(Q9):
        src, bounce = glbe.upstream(nodes3, e3[a], dims, bc3)
        srcc = np.where(bounce[:, None], nodes3, src)
        f[a] = np.where(bounce, post[OPP9[a], y, x], post[a, srcc[:, 1], srcc[:, 0]])
    if np.ndim(F) == 3:
        Fn = np.asarray(F[:, y, x], dtype=np.float64)
    else:
        Fn = np.broadcast_to(np.asarray(F, dtype=float).reshape(2, 1), (2, n))
    return collide(f, Fn, gamma, s, rho0)


class Flow2D:
    """Time march of the D2Q9 GLBE, residual every check_every steps."""

    def __init__(self, shape_xy, bc, F, gamma, s, rho0=1.0):
        nx, ny = shape_xy
        F = np.asarray(F, dtype=float)
        if F.ndim == 1:
            F = np.broadcast_to(F.reshape(2, 1, 1), (2, ny, nx))
        self.F = np.array(F)
        self.bc, self.gamma, self.s, self.rho0 = tuple(bc), gamma, np.asarray(s, float), rho0
        self.post = np.zeros((Q9, ny, nx))
        self.t = 0
        self.u_snap = None
        self.history = []
        self.u = None

    def step(self, n=1, check_every=10):
        for _ in range(n):
            self.post, self.u = step(self.post, self.F, self.gamma, self.s, self.bc, self.rho0)
            self.t += 1
            if self.t % check_every == 0:
                if self.u_snap is not None:
                    self.history.append((self.t, glbe.residual(self.u, self.u_snap)))
                self.u_snap = self.u.copy()
        return self

    def run_to(self, tol, max_steps, check_every=10):
        while self.t < max_steps:
            self.step(check_every, check_every)
            if self.history and self.history[-1][1] < tol:
                return True
        return False


# ------------------------------------------------------ D2Q5 induction -----
def tau_m(eta, gamma_m):
    """tau_m* = eta/(gamma_m theta_m) + 1/2 with theta_m = 1/3 (Sec. 4)."""
    return eta / (gamma_m * THETA_M2) + 0.5


def g_eq(B, u, chi, gamma_m):
    """g^eq*_{a j} = W_a [B_j + (e_{a k}/theta_m)(chi/gamma_m)(u_k B_j - B_k u_j)],
    j, k in {x, y}.  B, u: (2, ...).  Returns (2, 5, ...)."""
    e = E5.astype(float)
    out = []
    for jc in range(2):
        rows = []
        for a in range(Q5):
            adv = 0.0 * B[0]
            for k in range(2):
                if e[a, k] != 0.0:
                    adv = adv + e[a, k] * (u[k] * B[jc] - B[k] * u[jc])
            rows.append(W5[a] * (B[jc] + adv * chi / (gamma_m * THETA_M2)))
        out.append(np.stack(rows))
    return np.stack(out)


def stream_g(post_g, bc, B_wall):
    """Pull streaming of g with anti-bounce-back g_a = -g~_opp + 2 W_a B_wall.
    post_g: (2, 5, ny, nx)."""
    out = np.empty_like(post_g)
    bc3 = (bc[0], bc[1], PERIODIC)
    shape = (1,) + post_g.shape[2:]
    for jc in range(2):
        for a in range(Q5):
            ex, ey = int(E5[a, 0]), int(E5[a, 1])
            out[jc, a] = np.roll(post_g[jc, a], shift=(ey, ex), axis=(0, 1))
            m = glbe._outside_masks(shape, (ex, ey, 0), bc3)[0]
            if m.any():
                out[jc, a][m] = -post_g[jc, OPP5[a]][m] + 2.0 * W5[a] * B_wall[jc]
    return out


def coupled_fields(f, g, F_ext, gamma, gamma_m, chi, eta, mu=1.0, rho0=1.0):
    """(rho, u, B, J_z, F) from pre-collision f (deviations) and g.

    J_z = a + kappa (u_x B_y - u_y B_x), a = CURRENT_SIGN (Lam_xy - Lam_yx)/(mu chi tau theta),
    Lam_kj = sum_a e_{a k} g_{a j}, kappa = 2/(mu gamma_m tau theta);
    u = (sum f e + (F_ext + J_z (-B_y, B_x))/(2 gamma))/rho, solved per node."""
    tau = tau_m(eta, gamma_m)
    e = E5.astype(float)
    B = g.sum(axis=1)
    Lam = np.einsum("ak,jab->kjb", e, g.reshape(2, Q5, -1)).reshape((2, 2) + g.shape[2:])
    a = CURRENT_SIGN * (Lam[0, 1] - Lam[1, 0]) / (mu * chi * tau * THETA_M2)
    kappa = -CURRENT_SIGN * 2.0 / (mu * gamma_m * tau * THETA_M2)
    drho = f.sum(axis=0)
    rho = rho0 + drho
    jf = np.tensordot(E9.T.astype(float), f, axes=(1, 0))
    perp = np.stack([-B[1], B[0]])                       # (-B_y, B_x)
    u0 = (jf + (F_ext + a * perp) / (2.0 * gamma)) / rho
    c = kappa / (2.0 * gamma * rho)
    # u = u0 + c (u . perp') perp with u_x B_y - u_y B_x = -(u . perp)
    shp = B.shape[1:]
    P = perp.reshape(2, -1)
    cf = np.broadcast_to(c, shp).reshape(-1)
    A = np.eye(2)[None] + cf[:, None, None] * np.einsum("in,ln->nil", P, P)
    u = np.linalg.solve(A, u0.reshape(2, -1).T[:, :, None])[:, :, 0].T.reshape((2,) + shp)
    J = a + kappa * (u[0] * B[1] - u[1] * B[0])
    return rho, u, B, J, F_ext + J * perp


def collide_g(g, B, u, chi, gamma_m, eta):
    return g - (g - g_eq(B, u, chi, gamma_m)) / tau_m(eta, gamma_m)


def mhd_step(post_f, post_g, F_ext, p, bc):
    """One coupled D2Q9 + D2Q5 step.  p: dict(gamma, s, gamma_m, chi, eta, B_wall, rho0, mu)."""
    rho0 = p.get("rho0", 1.0)
    f = stream(post_f, bc)
    g = stream_g(post_g, bc, p["B_wall"])
    rho, u, B, J, F = coupled_fields(f, g, F_ext, p["gamma"], p["gamma_m"], p["chi"], p["eta"],
                                     p.get("mu", 1.0), rho0)
    return collide(f, F, p["gamma"], p["s"], rho0), collide_g(g, B, u, p["chi"], p["gamma_m"],
                                                              p["eta"]), u, B


def initial_g(shape_xy, B0):
    nx, ny = shape_xy
    g = np.zeros((2, Q5, ny, nx))
    for jc in range(2):
        for a in range(Q5):
            g[jc, a] = W5[a] * B0[jc]
    return g


class MHDFlow2D:
    def __init__(self, shape_xy, bc, F_ext, gamma, s, gamma_m, chi, eta, B0, rho0=1.0, mu=1.0):
        nx, ny = shape_xy
        F_ext = np.asarray(F_ext, dtype=float)
        if F_ext.ndim == 1:
            F_ext = np.broadcast_to(F_ext.reshape(2, 1, 1), (2, ny, nx))
        self.F = np.array(F_ext)
        self.bc = tuple(bc)
        self.p = dict(gamma=gamma, s=np.asarray(s, float), gamma_m=gamma_m, chi=chi, eta=eta,
                      B_wall=np.asarray(B0, float), rho0=rho0, mu=mu)
        self.post_f = np.zeros((Q9, ny, nx))
        self.post_g = initial_g(shape_xy, B0)
        self.t = 0
        self.u_snap = None
        self.history = []
        self.u = self.B = None

    def step(self, n=1, check_every=10):
        for _ in range(n):
            self.post_f, self.post_g, self.u, self.B = mhd_step(self.post_f, self.post_g, self.F,
                                                                self.p, self.bc)
            self.t += 1
            if self.t % check_every == 0:
                if self.u_snap is not None:
                    self.history.append((self.t, glbe.residual(self.u, self.u_snap)))
                self.u_snap = self.u.copy()
        return self

    def run_to(self, tol, max_steps, check_every=10):
        while self.t < max_steps:
            self.step(check_every, check_every)
            if self.history and self.history[-1][1] < tol:
                return True
        return False
