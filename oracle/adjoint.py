"""Gradients of the flow rate with respect to the force field, by complex step.

The paper has no adjoint; this module only supplies reference derivatives of
the oracle's own time march, obtained without any hand-derived transpose:

* complex-step directional derivatives: run the whole march in complex128 with
  F + i h v (h = 1e-30); <dQ/dF, v> = Im Q / h to machine precision (the march
  has no abs/max/comparison on state values);
* dense Jacobians of one step on tiny grids, one complex-step column per state
  or force entry, and the steady-state gradient from the dense linear solve
      (I - dPhi/df)^T lam = dQ/df,   dQ/dF = dQ/dF|_direct + (dPhi/dF)^T lam;
* the unrolled (transient) gradient after N steps from rest, one complex-step
  run per force component.

Q is the flow rate (1/n_x) sum_x j_x of the state (see glbe.flow_rate).
"""
import numpy as np

from . import glbe

H_CS = 1e-30


def steady_directional(shape_xyz, bc, F, v, gamma, s, tol=1e-12, max_steps=10 ** 6,
                       rho0=1.0):
    """(Q, <dQ/dF, v>) at the steady state, by complex step on the time march."""
    Fc = np.asarray(F, dtype=np.complex128) + 1j * H_CS * np.asarray(v, dtype=np.complex128)
    fl = glbe.Flow(shape_xyz, bc, Fc, gamma, s, rho0=rho0, dtype=np.complex128)
    ok = fl.run_to(tol, max_steps)
    if not ok:
        raise RuntimeError("complex-step march did not reach the tolerance")
    # Keep marching until the derivative part has settled as well.  The
    # linearised step has undamped period-2 (eigenvalue -1) modes on even
    # periodic lattices; a rough direction v excites them, so the derivative
    # of Q alternates between two values forever.  Their mean is the fixed
    # point of the linearised map (the steady sensitivity), so two consecutive
    # steps are averaged.
    def pair_mean():
        a = fl.flow_rate().imag
        fl.step(1, check_every=1 << 60)
        b = fl.flow_rate().imag
        return 0.5 * (a + b)

    d_prev = pair_mean()
    while fl.t < max_steps:
        fl.step(100, check_every=1 << 60)
        d = pair_mean()
        if abs(d - d_prev) <= 1e-13 * abs(d):
            break
        d_prev = d
    q = fl.flow_rate()
    return q.real, d / H_CS, fl


def unrolled_directional(shape_xyz, bc, F, v, gamma, s, n_steps, rho0=1.0):
    """(Q_N, <dQ_N/dF, v>) after n_steps from rest, by complex step."""
    Fc = np.asarray(F, dtype=np.complex128) + 1j * H_CS * np.asarray(v, dtype=np.complex128)
    fl = glbe.Flow(shape_xyz, bc, Fc, gamma, s, rho0=rho0, dtype=np.complex128)
    fl.step(n_steps)
    q = fl.flow_rate()
    return q.real, q.imag / H_CS


def unrolled_gradient(shape_xyz, bc, F, gamma, s, n_steps, rho0=1.0):
    """Full dQ_N/dF (3, nz, ny, nx), one complex-step march per force entry."""
    F = np.asarray(F, dtype=float)
    grad = np.zeros_like(F)
    it = np.nditer(F, flags=["multi_index"])
    for _ in it:
        v = np.zeros_like(F)
        v[it.multi_index] = 1.0
        grad[it.multi_index] = unrolled_directional(shape_xyz, bc, F, v, gamma, s, n_steps,
                                                    rho0)[1]
    return grad


def step_jacobians(post, F, gamma, s, bc, rho0=1.0):
    """Dense Jacobians of one step Phi(post; F) by complex step.

    Returns (J_f, J_F) with shapes (19N, 19N) and (19N, 3N); flattening is
    C order over (alpha, z, y, x) and (component, z, y, x).
    """
    post = np.asarray(post, dtype=float)
    F = np.asarray(F, dtype=float)
    nf, nF = post.size, F.size
    Jf = np.empty((nf, nf))
    JF = np.empty((nf, nF))
    for c in range(nf):
        p = post.astype(np.complex128).ravel()
        p[c] += 1j * H_CS
        out, _ = glbe.step(p.reshape(post.shape), F.astype(np.complex128), gamma, s, bc, rho0)
        Jf[:, c] = out.imag.ravel() / H_CS
    for c in range(nF):
        Fc = F.astype(np.complex128).ravel()
        Fc[c] += 1j * H_CS
        out, _ = glbe.step(post.astype(np.complex128), Fc.reshape(F.shape), gamma, s, bc, rho0)
        JF[:, c] = out.imag.ravel() / H_CS
    return Jf, JF


def flow_rate_gradients(post, F, gamma, bc, rho0=1.0):
    """(dQ/dpost, dQ/dF|direct) of Q = flow_rate(post, F), by complex step."""
    post = np.asarray(post, dtype=float)
    F = np.asarray(F, dtype=float)
    gp = np.empty(post.size)
    gF = np.empty(F.size)
    for c in range(post.size):
        p = post.astype(np.complex128).ravel()
        p[c] += 1j * H_CS
        gp[c] = glbe.flow_rate(p.reshape(post.shape), F, gamma, bc, rho0).imag / H_CS
    for c in range(F.size):
        Fc = F.astype(np.complex128).ravel()
        Fc[c] += 1j * H_CS
        gF[c] = glbe.flow_rate(post, Fc.reshape(F.shape), gamma, bc, rho0).imag / H_CS
    return gp, gF


def steady_gradient_dense(post_star, F, gamma, s, bc, rho0=1.0):
    """dQ/dF at a converged state from the dense transposed linear solve.

    The step conserves total mass (1^T J_f = 1^T, 1^T J_F = 0), so I - J_f is
    singular: the steady states form a one-parameter family labelled by the
    mass, and the march from rest stays on the member with the initial mass.
    The sensitivity is therefore taken at fixed mass: lam solves the bordered
    system
        (I - J_f)^T lam + c 1 = dQ/dpost,   1^T lam = 0,
    and dQ/dF = dQ/dF|_direct + J_F^T lam (independent of the 1-component of lam).
    Returns (grad, lam).
    """
    Jf, JF = step_jacobians(post_star, F, gamma, s, bc, rho0)
    gp, gF = flow_rate_gradients(post_star, F, gamma, bc, rho0)
    n = Jf.shape[0]
    A = np.zeros((n + 1, n + 1))
    A[:n, :n] = (np.eye(n) - Jf).T
    A[:n, n] = 1.0
    A[n, :n] = 1.0
    rhs = np.concatenate([gp, [0.0]])
    lam = np.linalg.solve(A, rhs)[:n]
    grad = gF + JF.T @ lam
    return grad.reshape(np.shape(F)), lam.reshape(np.shape(post_star))
