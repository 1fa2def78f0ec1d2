"""Pins for the oracle's reference gradients of the flow rate.

The complex-step derivative, the dense transposed solve and central finite
differences are three independent routes to dQ/dF; they must agree."""
import numpy as np
import pytest

from oracle import adjoint, glbe

PER, WALL = glbe.PERIODIC, glbe.WALL
SHAPE = (2, 4, 4)        # (nx, ny, nz)
BC = (PER, WALL, WALL)


def _force():
    nx, ny, nz = SHAPE
    F = np.zeros((3, nz, ny, nx))
    y = np.arange(ny) + 0.5
    F[0] = 1e-5 * (1.0 + 0.3 * np.sin(2 * np.pi * y / ny))[None, :, None]
    return F


@pytest.fixture(scope="module")
def steady():
    gamma, nu = 0.5, 0.131
    s = glbe.rates(nu, gamma)
    fl = glbe.Flow(SHAPE, BC, _force(), gamma, s)
    assert fl.run_to(1e-14, 100000)
    grad, lam = adjoint.steady_gradient_dense(fl.post, fl.F, gamma, s, BC)
    return dict(gamma=gamma, s=s, fl=fl, grad=grad, lam=lam)


def test_dense_gradient_matches_complex_step(steady):
    rng = np.random.default_rng(0)
    for _ in range(2):
        v = rng.standard_normal(steady["fl"].F.shape)
        _, d, _ = adjoint.steady_directional(SHAPE, BC, _force(), v, steady["gamma"],
                                             steady["s"], tol=1e-14)
        assert abs(d - (steady["grad"] * v).sum()) < 1e-10 * np.abs(steady["grad"]).sum()


def test_complex_step_matches_central_differences(steady):
    """Smooth direction; eps = 1e-4 of the force scale; O(eps^2) agreement."""
    nx, ny, nz = SHAPE
    z = np.arange(nz) + 0.5
    v = np.zeros((3, nz, ny, nx))
    v[0] = 1e-5 * np.cos(np.pi * z / nz)[:, None, None]
    v[1] = 0.5e-5
    g, s = steady["gamma"], steady["s"]
    _, d, _ = adjoint.steady_directional(SHAPE, BC, _force(), v, g, s, tol=1e-14)
    eps = 1e-4
    qs = []
    for sgn in (1, -1):
        fl = glbe.Flow(SHAPE, BC, _force() + sgn * eps * v, g, s)
        assert fl.run_to(1e-15, 100000)
        qs.append(fl.flow_rate())
    fd = (qs[0] - qs[1]) / (2 * eps)
    assert abs(fd - d) < 1e-6 * abs(d), (fd, d)


def test_adjoint_state_satisfies_fixed_point(steady):
    """lam solves the bordered transposed system (checked by re-applying J_f^T)."""
    Jf, _ = adjoint.step_jacobians(steady["fl"].post, steady["fl"].F, steady["gamma"],
                                   steady["s"], BC)
    gp, _ = adjoint.flow_rate_gradients(steady["fl"].post, steady["fl"].F, steady["gamma"], BC)
    lam = steady["lam"].ravel()
    r = lam - Jf.T @ lam - gp
    # residual is a multiple of the mass direction only
    assert np.max(np.abs(r - r.mean())) < 1e-12 * np.max(np.abs(gp))
    assert abs(lam.sum()) < 1e-10 * np.abs(lam).sum()


def test_unrolled_gradient_matches_directional_and_fd():
    g, nu, n = 1.0, 0.131, 40
    s = glbe.rates(nu, g)
    shape = (1, 2, 4)
    nx, ny, nz = shape
    F = np.zeros((3, nz, ny, nx))
    F[0] = 1e-5
    grad = adjoint.unrolled_gradient(shape, BC, F, g, s, n)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(F.shape)
    _, d = adjoint.unrolled_directional(shape, BC, F, v, g, s, n)
    assert abs(d - (grad * v).sum()) < 1e-12 * np.abs(grad).sum()
    eps = 1e-3 * 1e-5
    qp = glbe.Flow(shape, BC, F + eps * v, g, s).step(n).flow_rate()
    qm = glbe.Flow(shape, BC, F - eps * v, g, s).step(n).flow_rate()
    assert abs((qp - qm) / (2 * eps) - d) < 1e-6 * abs(d)


def test_newton_fixed_point_matches_time_march(steady):
    """The steady state as a fixed point f = Phi(f): Newton's method with the
    dense Jacobian (complex step) and the mass row bordering the singular
    I - J_f, started from rest, reaches the time-marched state."""
    g, s, fl = steady["gamma"], steady["s"], steady["fl"]
    f = np.zeros_like(fl.post)
    n = f.size
    for _ in range(4):
        phi, _ = glbe.step(f, fl.F, g, s, BC)
        Jf, _ = adjoint.step_jacobians(f, fl.F, g, s, BC)
        A = np.zeros((n + 1, n + 1))
        A[:n, :n] = np.eye(n) - Jf
        A[:n, n] = 1.0
        A[n, :n] = 1.0
        d = np.linalg.solve(A, np.concatenate([(phi - f).ravel(), [0.0]]))[:n]
        f = f + d.reshape(f.shape)
    phi, _ = glbe.step(f, fl.F, g, s, BC)
    assert np.max(np.abs(phi - f)) < 1e-15 * np.max(np.abs(f)) + 1e-20
    assert np.max(np.abs(f - fl.post)) < 1e-9 * np.max(np.abs(fl.post))
