"""Preconditioned GLBE with forcing (D3Q19), plain FP64 / complex128 oracle.

State convention.  The stored state is the post-collision population f~ of the
last completed step, held as the deviation from the rest state,
d(x) = f~(x) - w rho0.  One step is

    f(x)  = f~(x - e_alpha)            pull streaming, Sec. 2 (eq. streaming),
                                       halfway bounce-back f~_opp(x) when the
                                       link crosses a wall (Sec. 5, link bounce-back)
    f~(x) = f(x) + varpi*(x)           Sec. 3 (eqs. ppostcollision, prelax_term)

which is the paper's collide-then-stream sequence with the time level drawn
after the collision.  The deviation form is an exact rewrite: the rest state
w rho0 has moments T w rho0 = feq*(rho0, j=0) = rho0 (1, -11, 3, 0, ..., 0)
(tested), so m - meq* = T d - meq*_dev with meq*_dev defined below.
"""
import numpy as np

from .lattice import E19, OPP19, Q19, T19, T19_INV, W19

PERIODIC = "periodic"
WALL = "wall"


# ------------------------------------------------------------------ rates ---
def rates(nu, gamma, mode="paper", Lambda=None):
    """Preconditioned relaxation rates s*_k (Sec. 3, D3Q19 rates).

    Shear modes (9, 11, 13, 14, 15): 1/s = 3 nu / gamma + 1/2.
    Kinetic modes as the paper fixes them: s1 = 1.19, s2 = s10 = s12 = 1.4,
    s4 = s6 = s8 = 1.2, s16 = s17 = s18 = 1.98.  The paper also quotes a bulk
    viscosity formula for s1; the fixed value is used (reading: it is the
    value the runs used).  Conserved modes 0, 3, 5, 7 are not given; their value
    does not change the result (tested) and is set to 1.

    mode="lambda": the energy-flux and third-order modes (4, 6, 8, 16, 17, 18)
    are set to s_q with (3 nu / gamma)(1/s_q - 1/2) = Lambda, which makes the
    halfway bounce-back wall location independent of gamma.
    """
    s = np.ones(Q19)
    s_nu = 1.0 / (3.0 * nu / gamma + 0.5)
    for k in (9, 11, 13, 14, 15):
        s[k] = s_nu
    s[1] = 1.19
    for k in (2, 10, 12):
        s[k] = 1.4
    if mode == "paper":
        for k in (4, 6, 8):
            s[k] = 1.2
        for k in (16, 17, 18):
            s[k] = 1.98
    elif mode == "lambda":
        s_q = 1.0 / (Lambda * gamma / (3.0 * nu) + 0.5)
        for k in (4, 6, 8, 16, 17, 18):
            s[k] = s_q
    else:
        raise ValueError(mode)
    return s


# ----------------------------------------------------------------- fields ---
def fields(d, F, gamma, rho0=1.0):
    """rho = sum f, j = sum f e + F/(2 gamma), u = j / rho  (Sec. 3, eq. precondhydrofields).

    d: (19, ...) deviations f - w rho0 (sum_alpha w e_alpha = 0, so j needs no rho0 term).
    F: (3, ...) force.
    """
    drho = d.sum(axis=0)
    rho = rho0 + drho
    j = np.tensordot(E19.T.astype(float), d, axes=(1, 0)) + F / (2.0 * gamma)
    u = j / rho
    return drho, rho, j, u


# ------------------------------------------------------- moment equilibria ---
def meq_star_dev(drho, rho, j, gamma):
    """Preconditioned equilibrium moments (Sec. 3, D3Q19 list) minus those of the rest state.

    Only the nonlinear j_i j_k / rho terms carry 1/gamma.  The linear terms are
    written with drho = rho - rho0 so that the rest-state moments
    rho0 (1, -11, 3, 0, ...) are removed exactly.
    """
    jx, jy, jz = j
    jj = (jx * jx + jy * jy + jz * jz) / (gamma * rho)
    pxx3 = (3.0 * jx * jx - (jx * jx + jy * jy + jz * jz)) / (gamma * rho)
    pww = (jy * jy - jz * jz) / (gamma * rho)
    out = [
        drho,
        -11.0 * drho + 19.0 * jj,
        3.0 * drho - 5.5 * jj,
        jx, -2.0 / 3.0 * jx,
        jy, -2.0 / 3.0 * jy,
        jz, -2.0 / 3.0 * jz,
        pxx3, -0.5 * pxx3,
        pww, -0.5 * pww,
        jx * jy / (gamma * rho),
        jy * jz / (gamma * rho),
        jx * jz / (gamma * rho),
        0.0 * drho, 0.0 * drho, 0.0 * drho,
    ]
    return np.stack([np.broadcast_to(v, np.shape(drho)) for v in out])


def meq_star_full(rho, j, gamma):
    """Full preconditioned equilibrium moments (Sec. 3 list), used by the tests."""
    jx, jy, jz = j
    jj = (jx * jx + jy * jy + jz * jz) / (gamma * rho)
    pxx3 = (3.0 * jx * jx - (jx * jx + jy * jy + jz * jz)) / (gamma * rho)
    pww = (jy * jy - jz * jz) / (gamma * rho)
    out = [
        rho, -11.0 * rho + 19.0 * jj, 3.0 * rho - 5.5 * jj,
        jx, -2.0 / 3.0 * jx, jy, -2.0 / 3.0 * jy, jz, -2.0 / 3.0 * jz,
        pxx3, -0.5 * pxx3, pww, -0.5 * pww,
        jx * jy / (gamma * rho), jy * jz / (gamma * rho), jx * jz / (gamma * rho),
        0.0 * rho, 0.0 * rho, 0.0 * rho,
    ]
    return np.stack([np.broadcast_to(v, np.shape(rho)) for v in out])


# ---------------------------------------------------------------- sources ---
def source_moments(F, u):
    """Moment projections of the source term, S^ (App. A, D3Q19 list)."""
    Fx, Fy, Fz = F
    ux, uy, uz = u
    Fu = Fx * ux + Fy * uy + Fz * uz
    a = 2.0 * Fx * ux - Fy * uy - Fz * uz
    b = Fy * uy - Fz * uz
    z = 0.0 * Fu
    out = [
        z, 38.0 * Fu, -11.0 * Fu,
        Fx, -2.0 / 3.0 * Fx, Fy, -2.0 / 3.0 * Fy, Fz, -2.0 / 3.0 * Fz,
        2.0 * a, -a, 2.0 * b, -b,
        Fx * uy + Fy * ux, Fy * uz + Fz * uy, Fx * uz + Fz * ux,
        z, z, z,
    ]
    return np.stack([np.broadcast_to(v, np.shape(Fu)) for v in out])


def source_precond_diag(gamma):
    """P_S of Sec. 3 (eq. precondsourceterm), D3Q19: S^* = P_S S^."""
    g1, g2 = 1.0 / gamma, 1.0 / gamma ** 2
    return np.array([1.0, g2, g2] + [g1] * 6 + [g2] * 7 + [1.0, 1.0, 1.0])


def velocity_source(F, u):
    """Velocity-space source S_alpha = w [3 (e - u) + 9 (e.u) e] . F (Sec. 2)."""
    e = E19.astype(float)
    eF = np.tensordot(e, F, axes=(1, 0))
    eu = np.tensordot(e, u, axes=(1, 0))
    uF = (u * F).sum(axis=0)
    w = W19.reshape((Q19,) + (1,) * (np.ndim(F) - 1))
    return w * (3.0 * (eF - uF) + 9.0 * eu * eF)


# -------------------------------------------------------------- collision ---
def collide(d, F, gamma, s, rho0=1.0, source="precond"):
    """One preconditioned GLBE collision with forcing (Sec. 3, eq. prelax_term).

    d:  (19, ...) pre-collision deviations f - w rho0.
    F:  (3, ...) force.
    s:  (19,) rates s*_k.
    source: "precond" uses S^* = P_S S^ (eq. precondsourceterm); "naive" uses
        S^/gamma for every moment, i.e. S* = S/gamma in velocity space
        (eq. precondsourceincorrect), the form Sec. 3.1 warns against.
    Returns the post-collision deviations f~ - w rho0.
    """
    drho, rho, j, u = fields(d, F, gamma, rho0)
    m_dev = np.tensordot(T19, d, axes=(1, 0))          # T f - T w rho0
    neq = m_dev - meq_star_dev(drho, rho, j, gamma)    # f^ - f^eq*
    if source == "precond":
        P = source_precond_diag(gamma)
    elif source == "naive":
        P = np.full(Q19, 1.0 / gamma)
    else:
        raise ValueError(source)
    S_star = P.reshape((Q19,) + (1,) * (d.ndim - 1)) * source_moments(F, u)
    sk = np.asarray(s, dtype=float).reshape((Q19,) + (1,) * (d.ndim - 1))
    dm = -sk * neq + (1.0 - 0.5 * sk) * S_star
    return d + np.tensordot(T19_INV, dm, axes=(1, 0))


# -------------------------------------------------------------- streaming ---
def _outside_masks(shape, e, bc):
    """Boolean mask of nodes whose upstream neighbour x - e crosses a wall."""
    nz, ny, nx = shape
    mask = np.zeros(shape, dtype=bool)
    coords = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    # axis order in the array is (z, y, x); e is (ex, ey, ez); bc is (bcx, bcy, bcz)
    for axis_arr, comp, n in ((2, 0, nx), (1, 1, ny), (0, 2, nz)):
        if bc[comp] == WALL and e[comp] != 0:
            src = coords[axis_arr] - e[comp]
            mask |= (src < 0) | (src >= n)
    return mask


def _crossed_faces(shape, e, bc):
    """For each of the six faces (x-low, x-high, y-low, y-high, z-low, z-high),
    the mask of nodes whose link to x - e crosses that wall."""
    nz, ny, nx = shape
    coords = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    faces = []
    for axis_arr, comp, n in ((2, 0, nx), (1, 1, ny), (0, 2, nz)):
        src = coords[axis_arr] - e[comp]
        wall = bc[comp] == WALL and e[comp] != 0
        faces.append(wall & (src < 0))
        faces.append(wall & (src >= n))
    return faces


def stream(post, bc, e=E19, opp=OPP19, wall_u=None, rho0=1.0):
    """Pull streaming f_a(x) = f~_a(x - e_a), periodic wrap or halfway bounce-back.

    post: (Q, nz, ny, nx).  bc: (bcx, bcy, bcz), each PERIODIC or WALL.
    wall_u: optional (6, 3) velocities of the faces x-low, x-high, y-low, y-high,
    z-low, z-high.  A link bounced at a moving wall gains 6 w_a rho0 (e_a . u_w)
    (link bounce-back with wall momentum, Sec. 5, cavity); a link crossing two
    walls at an edge takes the mean of the two faces' terms (reading).
    """
    out = np.empty_like(post)
    shape = post.shape[1:]
    for a in range(len(e)):
        ex, ey, ez = (int(v) for v in e[a])
        out[a] = np.roll(post[a], shift=(ez, ey, ex), axis=(0, 1, 2))
        m = _outside_masks(shape, (ex, ey, ez), bc)
        if m.any():
            out[a][m] = post[opp[a]][m]
            if wall_u is not None and len(e) == Q19:
                faces = _crossed_faces(shape, (ex, ey, ez), bc)
                total = np.zeros(shape)
                count = np.zeros(shape)
                for f, mf in enumerate(faces):
                    term = 6.0 * W19[a] * rho0 * float(np.dot(E19[a], wall_u[f]))
                    total = total + np.where(mf, term, 0.0)
                    count = count + mf
                out[a][m] = out[a][m] + (total / np.maximum(count, 1))[m]
    return out


# ------------------------------------------------------------------- step ---
def step(post, F, gamma, s, bc, rho0=1.0, source="precond", wall_u=None):
    """One time step: stream, then collide.  Returns (new_post, u) where u is the
    velocity of the collision just performed (physical, with F/(2 gamma))."""
    f = stream(post, bc, wall_u=wall_u, rho0=rho0)
    _, _, _, u = fields(f, F, gamma, rho0)
    return collide(f, F, gamma, s, rho0, source), u


def flow_rate(post, F, gamma, bc, rho0=1.0):
    """Q = (1/n_x) sum_x j_x over all nodes, j from the streamed populations
    (including F/(2 gamma)); the mass flux through one cross-section."""
    f = stream(post, bc)
    _, _, j, _ = fields(f, F, gamma, rho0)
    return j[0].sum() / post.shape[3]


def residual(u_now, u_prev):
    """Relative L2 residual ||u(t) - u(t-10)||_2 / ||u(t)||_2 over all nodes and
    components (Sec. 5 defines the unnormalised norm; reading: relative, FP64)."""
    num = ((u_now - u_prev) ** 2).sum()
    den = (u_now ** 2).sum()
    return float(np.sqrt(num.real / den.real))


# -------------------------------------------------------- sampled nodes -----
def upstream(nodes, e, dims, bc):
    """Upstream node x - e of each node (n, 3) for pull streaming (Sec. 2,
    eq. streaming): wrapped on periodic axes; ``bounce`` marks the nodes whose
    link crosses a wall (halfway bounce-back, Sec. 5), whose source entries are
    then meaningless."""
    src = nodes - np.asarray(e)[None, :]
    bounce = np.zeros(len(nodes), dtype=bool)
    for c in range(3):
        if bc[c] == WALL:
            bounce |= (src[:, c] < 0) | (src[:, c] >= dims[c])
        else:
            src[:, c] %= dims[c]
    return src, bounce


def step_nodes(post, F, gamma, s, bc, nodes, rho0=1.0):
    """One step evaluated only at the given nodes (for large-grid parity).

    nodes: (n, 3) integer array of (x, y, z).  Returns (19, n) post-collision
    deviations at those nodes after one step from ``post``.
    """
    nodes = np.asarray(nodes)
    nz, ny, nx = post.shape[1:]
    dims = (nx, ny, nz)
    n = len(nodes)
    f = np.empty((Q19, n), dtype=post.dtype)
    for a in range(Q19):
        src, bounce = upstream(nodes, E19[a], dims, bc)
        own = post[OPP19[a], nodes[:, 2], nodes[:, 1], nodes[:, 0]]
        srcc = np.where(bounce[:, None], nodes, src)
        pulled = post[a, srcc[:, 2], srcc[:, 1], srcc[:, 0]]
        f[a] = np.where(bounce, own, pulled)
    Fn = F[:, nodes[:, 2], nodes[:, 1], nodes[:, 0]] if np.ndim(F) == 4 else \
        np.broadcast_to(np.asarray(F, dtype=float).reshape(3, 1), (3, n))
    return collide(f, Fn, gamma, s, rho0)


# ---------------------------------------------------------------- driver ----
class Flow:
    """Time-march the preconditioned GLBE to steady state (Sec. 5 procedure).

    The residual is evaluated every ``check_every`` (10) steps from the
    velocity of that step's collision.
    """

    def __init__(self, shape_xyz, bc, F, gamma, s, rho0=1.0, dtype=np.float64, post=None,
                 source="precond", wall_u=None):
        nx, ny, nz = shape_xyz
        self.source = source
        self.wall_u = None if wall_u is None else np.asarray(wall_u, dtype=float)
        self.bc = tuple(bc)
        self.gamma = gamma
        self.s = np.asarray(s, dtype=float)
        self.rho0 = rho0
        F = np.asarray(F)
        if F.ndim == 1:
            F = np.broadcast_to(F.reshape(3, 1, 1, 1), (3, nz, ny, nx))
        self.F = np.array(F, dtype=dtype)
        self.post = np.zeros((Q19, nz, ny, nx), dtype=dtype) if post is None \
            else np.array(post, dtype=dtype)
        self.t = 0
        self.u_snap = None
        self.history = []

    def step(self, n=1, check_every=10):
        for _ in range(n):
            self.post, u = step(self.post, self.F, self.gamma, self.s, self.bc, self.rho0,
                                self.source, self.wall_u)
            self.t += 1
            if self.t % check_every == 0:
                if self.u_snap is not None:
                    self.history.append((self.t, residual(u, self.u_snap)))
                self.u_snap = u.copy()
        return self

    def run_to(self, tol, max_steps, check_every=10):
        while self.t < max_steps:
            self.step(check_every, check_every)
            if self.history and self.history[-1][1] < tol:
                return True
        return False

    def velocity(self):
        f = stream(self.post, self.bc, wall_u=self.wall_u, rho0=self.rho0)
        return fields(f, self.F, self.gamma, self.rho0)[3]

    def flow_rate(self):
        return flow_rate(self.post, self.F, self.gamma, self.bc, self.rho0)
