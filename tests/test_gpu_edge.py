"""Degenerate and edge cases of the step on the GPU.

* The rest state (zero force, deviations zero, B = B0) is a fixed point, kept
  bit for bit in every storage type, for the flow, the coupled field and the 2D
  variants; its residual is zero, so a march to any tolerance stops at the
  second check.
* A single periodic node under a uniform force: every collision adds F/gamma to
  the momentum (the conserved-moment rule of Sec. 3), so after n steps
  j = n F/gamma exactly in FP64, and the mass does not change.
* A fully periodic lattice from a random state under a random force field:
  total mass constant, total momentum grown by n sum F / gamma.
* An unstable march reports the instability and keeps its state readable."""
import numpy as np
import pytest

from oracle import d2q9, glbe
from paper_0809_4730_amd import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu
PER, WALL = "periodic", "wall"


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "f16"])
def test_rest_state_is_kept_exactly(storage):
    import torch
    import paper_0809_4730_amd as pkg
    announce("rest state %s" % storage)
    sims = [pkg.Simulation((9, 7, 5), (PER, WALL, WALL), 0.1, glbe.rates(0.05, 0.1),
                           storage=storage),
            pkg.Simulation((17, 6, 1), (PER, WALL, PER), 0.1, d2q9.rates(0.05, 0.1),
                           storage=storage, lattice="d2q9")]
    if storage in ("f64", "f32"):
        sims.append(pkg.Simulation((6, 8, 5), (PER, WALL, PER), 0.2, glbe.rates(0.05, 0.2),
                                   storage=storage,
                                   mhd=dict(gamma_m=0.2, chi=0.05, eta=0.02, B0=(0.01, 0.03, -0.02))))
    for sim in sims:
        sim.step(33)
        st = sim.get_state()
        for t in (st if isinstance(st, tuple) else (st,)):
            assert int(torch.count_nonzero(t)) == 0
        steps, r = sim.run_to_residual(1e-12, 1000, poll_every=10)
        assert r == 0.0 and steps > 0
        mass, flow = sim.reductions()
        assert mass == 0.0 and flow == 0.0


@pytest.mark.parametrize("gamma", [1.0, 0.25])
def test_single_node_momentum_grows_by_force_over_gamma(gamma):
    import paper_0809_4730_amd as pkg
    announce("single node gamma=%g" % gamma)
    F = np.array([2.0 ** -20, -(2.0 ** -21), 3 * 2.0 ** -22])
    sim = pkg.Simulation((1, 1, 1), (PER, PER, PER), gamma, glbe.rates(0.1, gamma),
                         storage="f64", force=tuple(F))
    n = 37
    sim.step(n)
    rho, u, _ = sim.moments("f64")
    rho = float(rho.cpu().numpy().ravel()[0])
    u = u.cpu().numpy().reshape(3)
    j_raw = n * F / gamma
    # fields of the current state carry the half force of the next collision
    j = j_raw + F / (2 * gamma)
    assert rho == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(u * rho, j, rtol=1e-13, atol=0)
    f = sim.get_state().cpu().numpy().reshape(19)
    e = pkg.lattice_velocities(19).astype(float)
    assert np.allclose(e.T @ f, j_raw, rtol=1e-13, atol=0)


def test_unstable_march_reports_and_keeps_state():
    import torch
    import paper_0809_4730_amd as pkg
    announce("unstable march")
    nu, g = 0.02, 1e-3
    sim = pkg.Simulation((4, 4, 64), (PER, PER, WALL), g, glbe.rates(nu, g), storage="f64",
                         force=(8 * nu * 0.05 / 64 ** 2, 0.0, 0.0))
    with pytest.raises(pkg.LbmError) as ei:
        sim.run_to_residual(1e-9, 5000, poll_every=100)
    assert ei.value.status == -4
    st = sim.get_state()
    assert st.shape == (19, 64, 4, 4)
    h = sim.history(1000)
    assert (h[:, 6] > 0).any() or not np.isfinite(h[:, 1]).all() or h[:, 1].max() > 1e-2
    assert not bool(torch.isfinite(st).all()) or h[:, 1].max() > 1e-2


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_periodic_lattice_conserves_mass_and_gains_force_momentum(storage, tol):
    """On a fully periodic lattice streaming permutes the populations, so from
    any state the total mass stays where it is and the total momentum of the
    stored populations, sum e f, grows by exactly sum F / gamma per step (the
    collision conserves mass and adds the force's momentum, Sec. 3): a seeded
    random state and force field, 1 and 40 steps."""
    import torch

    import paper_0809_4730_amd as pkg
    from tests.gpu_util import perms
    announce("periodic conservation %s" % storage)
    shape, gamma = (16, 12, 10), 0.3
    bc = (PER, PER, PER)
    dt = torch.float64 if storage == "f64" else torch.float32
    ndt = np.float64 if storage == "f64" else np.float32
    d0 = inputs.random_deviations(shape, seed=61, amp=1e-3).astype(ndt)
    F = (inputs.random_force(shape, seed=61, amp=1e-5) + 1e-5).astype(ndt)
    sim = pkg.Simulation(shape, bc, gamma, glbe.rates(0.05, gamma), storage=storage,
                         force=torch.from_numpy(F).cuda())
    p19, _ = perms()
    sim.set_state(torch.from_numpy(np.ascontiguousarray(d0[p19])).cuda())
    e = pkg.lattice_velocities(19).astype(np.float64)        # library direction order
    f0 = d0[p19].astype(np.float64)
    m0 = f0.sum()
    P0 = np.tensordot(e.T, f0, axes=(1, 0)).reshape(3, -1).sum(axis=1)
    dP = F.astype(np.float64).reshape(3, -1).sum(axis=1) / gamma
    done = 0
    for n in (1, 40):
        sim.step(n - done)
        done = n
        f = sim.get_state().double().cpu().numpy()
        P = np.tensordot(e.T, f, axes=(1, 0)).reshape(3, -1).sum(axis=1)
        scale = np.abs(P0).max() + n * np.abs(dP).max()
        assert abs(f.sum() - m0) < tol * np.abs(f0).sum()
        assert np.abs(P - (P0 + n * dP)).max() < tol * scale, (P, P0 + n * dP)
    sim.close()
