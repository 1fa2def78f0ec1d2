"""GPU discrete adjoint of the preconditioned GLBE step (d flow rate / d force).

Checked against the oracle's gradients (dense bordered transposed solve and
complex-step derivatives, which share nothing with the kernel's hand-written
transpose) and against central finite differences of the GPU's own forward
march.
"""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import glbe
from paper_0809_4730_amd import inputs
from tests.gpu_util import announce, rel

pytestmark = pytest.mark.gpu
PER, WALL = "periodic", "wall"


def _sim(shape, bc, gamma, s, storage, F):
    import torch

    import paper_0809_4730_amd as pkg
    dt = torch.float64 if storage == "f64" else torch.float32
    return pkg.Simulation(shape, bc, gamma, s, storage=storage,
                          force=torch.tensor(F, dtype=dt, device="cuda"))


def _tiny_force(shape):
    nx, ny, nz = shape
    F = np.zeros((3, nz, ny, nx))
    y = np.arange(ny) + 0.5
    F[0] = 1e-5 * (1.0 + 0.3 * np.sin(2 * np.pi * y / ny))[None, :, None]
    return F


@pytest.mark.parametrize("gamma", [0.5, 1.0])
def test_steady_adjoint_matches_dense_oracle(gamma):
    """End to end: the GPU marches to its own steady state (residual 1e-14)
    and linearises there.  Its state differs from the oracle's by the
    residual amplified by the flow's slowest relaxation time, and the gradient
    inherits that gap; hence 1e-9.  The 1e-12 comparison starts both from
    the oracle's state (test_gpu_headline)."""
    announce("steady adjoint tiny gamma=%g" % gamma)
    shape, bc = (2, 4, 4), (PER, WALL, WALL)
    s = glbe.rates(0.131, gamma)
    F = _tiny_force(shape)
    fl = glbe.Flow(shape, bc, F, gamma, s)
    assert fl.run_to(1e-14, 100000)
    ref, _ = oadj.steady_gradient_dense(fl.post, fl.F, gamma, s, bc)
    sim = _sim(shape, bc, gamma, s, "f64", F)
    steps, r = sim.run_to_residual(1e-14, 200000, poll_every=500)
    assert steps > 0
    sim.step(200)
    grad, iters, change = sim.adjoint_steady(tol=1e-13, max_iter=200000)
    assert change < 1e-13, change
    g = grad.cpu().numpy()
    assert rel(g, ref) < 1e-9, rel(g, ref)


def test_steady_adjoint_matches_oracle_complex_step():
    shape, bc = (4, 6, 6), (PER, WALL, WALL)
    gamma = 0.5
    s = glbe.rates(0.131, gamma)
    F = inputs.duct_force(shape)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(F.shape)
    _, d_ref, _ = oadj.steady_directional(shape, bc, F, v, gamma, s, tol=1e-14)
    sim = _sim(shape, bc, gamma, s, "f64", F)
    assert sim.run_to_residual(1e-14, 200000, poll_every=500)[0] > 0
    sim.step(200)
    grad, iters, change = sim.adjoint_steady(tol=1e-13, max_iter=200000)
    d = float((grad.cpu().numpy() * v).sum())
    assert abs(d - d_ref) < 1e-9 * np.abs(grad.cpu().numpy() * v).sum(), (d, d_ref)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-7), ("f32", 2e-3)])
def test_steady_adjoint_duct_vs_finite_differences(storage, tol):
    """32^3 duct (walls y, z), gamma = 1: <dQ/dF, v> for a smooth v against
    central differences of two FP64 forward marches to steady state."""
    import torch
    announce("steady adjoint duct32 %s" % storage)
    shape, bc, gamma = (32, 32, 32), (PER, WALL, WALL), 1.0
    s = glbe.rates(0.131, gamma)
    F = inputs.duct_force(shape)
    nx, ny, nz = shape
    y = np.arange(ny) + 0.5
    z = np.arange(nz) + 0.5
    v = np.zeros_like(F)
    v[0] = 1e-5 * (np.cos(np.pi * z / nz)[:, None] * (1 + 0.2 * np.sin(2 * np.pi * y / ny))[None, :])[:, :, None]
    v[1] = 3e-6 * np.sin(np.pi * y / ny)[None, :, None]
    ref = _sim(shape, bc, gamma, s, "f64", F)
    assert ref.run_to_residual(1e-10, 400000)[0] > 0
    if storage == "f64":
        sim = ref
    else:
        # FP32 storage cannot reach 1e-10 (its rounding floor is ~1e-7): march the
        # same number of steps as FP64 plus margin, then iterate the FP32 adjoint
        sim = _sim(shape, bc, gamma, s, storage, F)
        sim.step(ref.t + 2000)
    grad, iters, change = sim.adjoint_steady(tol=1e-10 if storage == "f64" else 1e-6,
                                             max_iter=2 * ref.t + 20000)
    d = float((grad.double().cpu().numpy() * v).sum())
    eps = 1e-2
    q = []
    for sg in (1, -1):
        simf = _sim(shape, bc, gamma, s, "f64", F + sg * eps * v)
        assert simf.run_to_residual(1e-12, 400000)[0] > 0
        simf.step(1000)
        q.append(simf.reductions()[1])
    fd = (q[0] - q[1]) / (2 * eps)
    assert abs(d - fd) < tol * abs(fd), (d, fd)


def test_steady_adjoint_duct128_vs_finite_differences():
    """The adjoint workload at full size and in the bench's configuration:
    128^3 duct, FP32 storage, gamma = 0.1.  <dQ/dF, v> against central
    differences of two FP64 forward marches to steady state."""
    import torch
    cfg = inputs.ADJOINT
    shape, bc, gamma = cfg["shape"], cfg["bc"], 0.1
    announce("steady adjoint duct128 fp32")
    s = glbe.rates(cfg["nu"], gamma)
    F = inputs.duct_force(shape, cfg["F0"])
    nx, ny, nz = shape
    y = np.arange(ny) + 0.5
    z = np.arange(nz) + 0.5
    v = np.zeros_like(F)
    v[0] = 1e-5 * ((1 + 0.3 * np.cos(np.pi * z / nz))[:, None] *
                   (1 + 0.2 * np.sin(2 * np.pi * y / ny))[None, :])[:, :, None]
    v[1] = 3e-6 * np.sin(np.pi * y / ny)[None, :, None]
    ref = _sim(shape, bc, gamma, s, "f64", F)
    assert ref.run_to_residual(1e-10, 400000, poll_every=1000)[0] > 0
    sim = _sim(shape, bc, gamma, s, "f32", F)
    sim.step(ref.t + 2000)
    grad, iters, change = sim.adjoint_steady(tol=1e-6, max_iter=2 * ref.t + 40000)
    d = float((grad.double().cpu().numpy() * v).sum())
    del ref, sim, grad
    torch.cuda.empty_cache()
    eps = 1e-2
    q = []
    for sg in (1, -1):
        simf = _sim(shape, bc, gamma, s, "f64", F + sg * eps * v)
        assert simf.run_to_residual(1e-12, 400000, poll_every=1000)[0] > 0
        simf.step(1000)
        q.append(simf.reductions()[1])
        del simf
        torch.cuda.empty_cache()
    fd = (q[0] - q[1]) / (2 * eps)
    assert abs(fd) > 0
    assert abs(d - fd) < 2e-3 * abs(fd), (d, fd)


def test_unrolled_adjoint_matches_oracle_elementwise():
    announce("unrolled adjoint tiny")
    shape, bc, gamma, n = (1, 2, 4), (PER, WALL, WALL), 1.0, 40
    s = glbe.rates(0.131, gamma)
    F = np.zeros((3, 4, 2, 1))
    F[0] = 1e-5
    F[1] = 2e-6
    ref = oadj.unrolled_gradient(shape, bc, F, gamma, s, n)
    grads = []
    for K in (1, 7, 40):
        sim = _sim(shape, bc, gamma, s, "f64", F)
        grads.append(sim.adjoint_unrolled(n, K).cpu().numpy())
        assert sim.t == n
    assert rel(grads[0], ref) < 1e-12, rel(grads[0], ref)
    # checkpoint spacing changes only where states are recomputed, not the result
    assert np.array_equal(grads[0], grads[1]) and np.array_equal(grads[0], grads[2])


def test_unrolled_adjoint_32cubed_2000_steps_vs_fd():
    """Checkpointed (every 45 steps) unrolled adjoint over 2000 steps on 32^3,
    FP32, against central differences of the FP64 forward march."""
    cfg = inputs.ADJOINT
    shape, bc = cfg["unrolled_shape"], cfg["bc"]
    gamma = cfg["gamma"]
    announce("unrolled adjoint 32^3 x 2000")
    s = glbe.rates(cfg["nu"], gamma)
    F = inputs.duct_force(shape, cfg["F0"])
    rng = np.random.default_rng(9)
    v = 1e-5 * rng.standard_normal(F.shape)
    sim = _sim(shape, bc, gamma, s, "f32", F)
    g32 = sim.adjoint_unrolled(cfg["unrolled_steps"], cfg["ckpt_every"]).double().cpu().numpy()
    sim64 = _sim(shape, bc, gamma, s, "f64", F)
    g64 = sim64.adjoint_unrolled(cfg["unrolled_steps"], cfg["ckpt_every"]).cpu().numpy()
    eps = 1e-1
    q = []
    for sg in (1, -1):
        simf = _sim(shape, bc, gamma, s, "f64", F + sg * eps * v)
        simf.step(cfg["unrolled_steps"])
        q.append(simf.reductions()[1])
    fd = (q[0] - q[1]) / (2 * eps)
    d64 = float((g64 * v).sum())
    d32 = float((g32 * v).sum())
    assert abs(d64 - fd) < 1e-8 * abs(fd), (d64, fd)
    assert abs(d32 - d64) < 1e-4 * abs(d64), (d32, d64)
    assert rel(g32, g64) < 1e-4


def test_autograd_flow_rate_matches_finite_differences():
    """torch.autograd over the library: Q(F) for the steady state and after a
    finite march; F.grad along a direction against central differences of Q."""
    import torch
    import paper_0809_4730_amd as pkg
    shape, bc, gamma = (6, 8, 8), ("periodic", "wall", "wall"), 0.5
    s = glbe.rates(0.131, gamma)
    F0 = torch.tensor(inputs.duct_force(shape, 1e-5), dtype=torch.float64, device="cuda")
    v = torch.tensor(inputs.random_force(shape, seed=9, amp=1e-5), dtype=torch.float64,
                     device="cuda")
    eps = 1e-2

    def steady(F):
        return pkg.steady_flow_rate(F, shape, bc, gamma, s, storage="f64", tol=1e-13,
                                    max_steps=200000, adj_tol=1e-11)

    def unrolled(F):
        return pkg.unrolled_flow_rate(F, shape, bc, gamma, s, 80, 9, storage="f64")

    for fn in (steady, unrolled):
        F = F0.clone().requires_grad_(True)
        q = fn(F)
        q.backward()
        d = float((F.grad * v).sum())
        with torch.no_grad():
            fd = (float(fn(F0 + eps * v)) - float(fn(F0 - eps * v))) / (2 * eps)
        announce("autograd %s: <dQ/dF, v> %.6e fd %.6e" % (fn.__name__, d, fd))
        assert abs(d - fd) < 1e-6 * abs(fd), (d, fd)
