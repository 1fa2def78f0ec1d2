"""Lattice tables for the oracle: D3Q19 (flow) and D3Q7 (magnetic induction).

Velocity sets follow the groupings of Sec. 2 (eq. velocityd3q19) and Sec. 4
(D3Q7 set).  Within each group the ordering is the oracle's own choice; results
do not depend on it.

The weights w_alpha are not printed in the paper.  They are fixed by the printed
rest-state equilibrium moments (App. A, D3Q19: e^eq = -11 rho and e2^eq = 3 rho at
j = 0), which require sum w = 1, sum w |c|^2 = 1 and sum w |c|^4 = 5/3; with
isotropy inside each shell this gives w0 = 1/3, w(axis) = 1/18, w(diagonal) = 1/36.

The moment basis T is named in App. A (rho, e, e2, j, q, 3p_xx, 3pi_xx, p_ww,
pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z) and taken from the orthogonal
Gram-Schmidt construction the paper cites (Sec. 2); it is not printed, so each
row is written here as its polynomial in the velocity components.  Tests check
that these rows reproduce the printed equilibria and sources exactly.
"""
from fractions import Fraction

import numpy as np

# ---------------------------------------------------------------- D3Q19 -----
# alpha = 0 rest; 1..6 axis; 7..18 face diagonals.  Opposite directions are
# stored next to each other (1/2, 3/4, ..., 17/18).
E19 = np.array([
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
], dtype=np.int64)
Q19 = 19


def opposite(e):
    """Index of -e_alpha for every alpha."""
    out = np.empty(len(e), dtype=np.int64)
    for a, v in enumerate(e):
        hits = [b for b, w in enumerate(e) if tuple(w) == tuple(-v)]
        assert len(hits) == 1
        out[a] = hits[0]
    return out


OPP19 = opposite(E19)


def _shell_weight(c, w0, w1, w2):
    n2 = int(np.dot(c, c))
    return {0: w0, 1: w1, 2: w2}[n2]


W19_FRAC = [_shell_weight(c, Fraction(1, 3), Fraction(1, 18), Fraction(1, 36)) for c in E19]
W19 = np.array([float(w) for w in W19_FRAC])


def _row_polys():
    """Row polynomials of the D3Q19 moment basis, in App. A order."""
    def c2(cx, cy, cz):
        return cx * cx + cy * cy + cz * cz
    return [
        ("rho", lambda x, y, z: 1),
        ("e", lambda x, y, z: 19 * c2(x, y, z) - 30),
        ("e2", lambda x, y, z: Fraction(21 * c2(x, y, z) ** 2 - 53 * c2(x, y, z) + 24, 2)),
        ("jx", lambda x, y, z: x),
        ("qx", lambda x, y, z: (5 * c2(x, y, z) - 9) * x),
        ("jy", lambda x, y, z: y),
        ("qy", lambda x, y, z: (5 * c2(x, y, z) - 9) * y),
        ("jz", lambda x, y, z: z),
        ("qz", lambda x, y, z: (5 * c2(x, y, z) - 9) * z),
        ("3pxx", lambda x, y, z: 3 * x * x - c2(x, y, z)),
        ("3pixx", lambda x, y, z: (3 * c2(x, y, z) - 5) * (3 * x * x - c2(x, y, z))),
        ("pww", lambda x, y, z: y * y - z * z),
        ("piww", lambda x, y, z: (3 * c2(x, y, z) - 5) * (y * y - z * z)),
        ("pxy", lambda x, y, z: x * y),
        ("pyz", lambda x, y, z: y * z),
        ("pxz", lambda x, y, z: x * z),
        ("mx", lambda x, y, z: (y * y - z * z) * x),
        ("my", lambda x, y, z: (z * z - x * x) * y),
        ("mz", lambda x, y, z: (x * x - y * y) * z),
    ]


MOMENT_NAMES = [n for n, _ in _row_polys()]


def moment_matrix_fraction():
    """T as a list of lists of Fractions (exact)."""
    rows = []
    for _, p in _row_polys():
        rows.append([Fraction(p(int(c[0]), int(c[1]), int(c[2]))) for c in E19])
    return rows


T19_FRAC = moment_matrix_fraction()
T19 = np.array([[float(v) for v in r] for r in T19_FRAC])
T19_INV = np.linalg.inv(T19)

# ----------------------------------------------------------------- D3Q7 -----
# Sec. 4: rest plus the six axis directions; W0 = 1/N_m, W_alpha = 1/(2 N_m),
# theta_m = 1/N_m with N_m = 4 in 3D.
E7 = np.array([
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
], dtype=np.int64)
Q7 = 7
OPP7 = opposite(E7)
N_M = 4
W7 = np.array([1.0 / N_M] + [1.0 / (2 * N_M)] * 6)
THETA_M = 1.0 / N_M
