"""GPU parity of the fused preconditioned GLBE step against the FP64 oracle.

Bars: FP64 storage matches the oracle to 1e-12 relative (per step and after
hundreds of steps from the same state); FP32 storage to FP32 rounding
(2e-6 relative per step); BF16/FP16 storage to one rounding of the stored
value (RNE) plus FP32 noise, elementwise.
"""
import numpy as np
import pytest

from oracle import glbe
from paper_0809_4730_amd import inputs
from tests.gpu_util import announce, from_gpu_f, rel, to_gpu_f

pytestmark = pytest.mark.gpu

PER, WALL = "periodic", "wall"
GRIDS = [
    ((8, 8, 8), (PER, PER, PER)),
    ((8, 6, 10), (PER, WALL, WALL)),
    ((5, 7, 9), (WALL, WALL, WALL)),
    ((1, 1, 12), (PER, PER, WALL)),
    ((33, 3, 4), (PER, WALL, PER)),      # ragged: N not a multiple of the workgroup
]


def _torch():
    import torch
    return torch


def _sim(shape, bc, gamma, s, storage, F=None, **kw):
    import paper_0809_4730_amd as pkg
    torch = _torch()
    if F is None:
        force = (0.0, 0.0, 0.0)
    elif np.ndim(F) == 1:
        force = tuple(F)
    else:
        dt = torch.float64 if storage == "f64" else torch.float32
        force = torch.tensor(F, dtype=dt, device="cuda")
    return pkg.Simulation(shape, bc, gamma, s, storage=storage, force=force, **kw)


@pytest.mark.parametrize("shape,bc", GRIDS)
@pytest.mark.parametrize("gamma", [1.0, 0.1])
def test_fp64_single_step_matches_oracle(shape, bc, gamma):
    torch = _torch()
    announce("fp64 single step %s %s gamma=%g" % (shape, bc, gamma))
    d0 = inputs.random_deviations(shape, seed=1, amp=1e-3)
    F = inputs.random_force(shape, seed=1, amp=1e-4)
    s = glbe.rates(0.05, gamma)
    sim = _sim(shape, bc, gamma, s, "f64", F)
    sim.set_state(to_gpu_f(d0, torch.float64))
    sim.step(1)
    out = from_gpu_f(sim.get_state())
    ref, _ = glbe.step(d0, F, gamma, s, bc)
    assert rel(out - d0, ref - d0) < 1e-13
    assert rel(out, ref) < 1e-14


@pytest.mark.parametrize("shape,bc", GRIDS[:3])
def test_fp64_many_steps_match_oracle(shape, bc):
    torch = _torch()
    announce("fp64 300 steps %s %s" % (shape, bc))
    gamma = 0.2
    d0 = inputs.random_deviations(shape, seed=2, amp=1e-3)
    F = inputs.random_force(shape, seed=2, amp=1e-5)
    s = glbe.rates(0.05, gamma, "lambda", 0.25)
    sim = _sim(shape, bc, gamma, s, "f64", F)
    sim.set_state(to_gpu_f(d0, torch.float64))
    sim.step(300)
    out = from_gpu_f(sim.get_state())
    ref = d0
    for _ in range(300):
        ref, _ = glbe.step(ref, F, gamma, s, bc)
    assert rel(out, ref) < 1e-12


# nx a multiple of 64: every wave lies in one x-row, and the step takes its y/z
# neighbours and wall flags as wave-uniform values (the row-aligned variants:
# through the row table when x is periodic, else per-face flags)
ROW_GRIDS = [
    ((64, 3, 4), (PER, WALL, WALL)),
    ((64, 1, 3), (PER, WALL, WALL)),   # ny = 1: every row touches both y faces
    ((128, 3, 1), (PER, PER, WALL)),   # nz = 1
    ((64, 2, 5), (PER, PER, PER)),
    ((64, 2, 3), (WALL, PER, WALL)),
    ((128, 2, 2), (WALL, WALL, PER)),
]


@pytest.mark.parametrize("shape,bc", ROW_GRIDS)
def test_row_aligned_lattices_match_oracle(shape, bc):
    """One step and 40 steps in FP64, and the residual history of the check
    steps, against the oracle on lattices that take the row-aligned variant."""
    torch = _torch()
    announce("row-aligned %s %s" % (shape, bc))
    gamma = 0.3
    d0 = inputs.random_deviations(shape, seed=4, amp=1e-3)
    F = inputs.random_force(shape, seed=4, amp=1e-5)
    s = glbe.rates(0.05, gamma)
    sim = _sim(shape, bc, gamma, s, "f64", F)
    sim.set_state(to_gpu_f(d0, torch.float64))
    sim.step(1)
    ref, _ = glbe.step(d0, F, gamma, s, bc)
    out = from_gpu_f(sim.get_state())
    assert rel(out - d0, ref - d0) < 1e-13
    sim.step(39)
    for _ in range(39):
        ref, _ = glbe.step(ref, F, gamma, s, bc)
    assert rel(from_gpu_f(sim.get_state()), ref) < 1e-12
    fl = glbe.Flow(shape, bc, F, gamma, s)
    sim2 = _sim(shape, bc, gamma, s, "f64", F)
    sim2.step(60)
    fl.step(60)
    steps = {int(h[0]): h for h in sim2.history()}
    # R compares velocities 10 steps apart: FP64 velocity differences of a few
    # units of 1e-16 |u| between the two operation orders give a few 1e-17 in R
    # (measured at most 6.3e-17); the relative part covers the state's drift
    for t, r in fl.history:
        assert abs(steps[t][1] - r) <= 1e-15 + 1e-12 * r


def test_uniform_force_equals_field_of_constants():
    torch = _torch()
    shape, bc = (8, 6, 10), (PER, WALL, WALL)
    d0 = inputs.random_deviations(shape, seed=3, amp=1e-3)
    F = np.array([1e-5, -2e-6, 3e-6])
    s = glbe.rates(0.1, 0.5)
    a = _sim(shape, bc, 0.5, s, "f64", F)
    b = _sim(shape, bc, 0.5, s, "f64", inputs.uniform_force(shape, F))
    for sim in (a, b):
        sim.set_state(to_gpu_f(d0, torch.float64))
        sim.step(7)
    assert torch.equal(a.get_state(), b.get_state())


@pytest.mark.parametrize("shape,bc", GRIDS[1:3])
def test_fp32_single_step(shape, bc):
    torch = _torch()
    announce("fp32 single step %s" % (shape,))
    d0 = inputs.random_deviations(shape, seed=4, amp=1e-3).astype(np.float32).astype(np.float64)
    F = inputs.random_force(shape, seed=4, amp=1e-4).astype(np.float32).astype(np.float64)
    s = glbe.rates(0.05, 0.1)
    sim = _sim(shape, bc, 0.1, s, "f32", F)
    sim.set_state(to_gpu_f(d0, torch.float32))
    sim.step(1)
    out = from_gpu_f(sim.get_state())
    ref, _ = glbe.step(d0, F, 0.1, s, bc)
    assert rel(out, ref) < 2e-6
    assert rel(out - d0, ref - d0) < 2e-5


@pytest.mark.parametrize("storage,ulp", [("bf16", 2.0 ** -8), ("f16", 2.0 ** -11)])
def test_reduced_precision_single_step(storage, ulp):
    torch = _torch()
    shape, bc = (8, 6, 10), (PER, WALL, WALL)
    announce("%s single step" % storage)
    tdt = torch.bfloat16 if storage == "bf16" else torch.float16
    d0 = inputs.random_deviations(shape, seed=5, amp=1e-3)
    d0 = torch.tensor(d0).to(tdt).double().numpy()     # what the storage can hold
    F = inputs.random_force(shape, seed=5, amp=1e-4).astype(np.float32).astype(np.float64)
    s = glbe.rates(0.05, 0.5)
    sim = _sim(shape, bc, 0.5, s, storage, F)
    sim.set_state(to_gpu_f(d0, tdt))
    sim.step(1)
    out = from_gpu_f(sim.get_state())
    ref, _ = glbe.step(d0, F, 0.5, s, bc)
    # one round-to-nearest-even of the FP32 result, elementwise
    tiny = 6e-8 if storage == "f16" else 1e-38
    assert np.all(np.abs(out - ref) <= ulp * np.abs(ref) + tiny + 1e-9 * np.abs(ref).max())
    # the stored values are exactly the RNE rounding of the oracle's value except
    # where FP32 vs FP64 differences straddle a rounding boundary
    ref_r = torch.tensor(ref).to(tdt).double().numpy()
    mism = np.mean(out != ref_r)
    assert mism < 0.01, mism


def test_residual_history_matches_oracle():
    torch = _torch()
    shape, bc = (1, 16, 16), (PER, WALL, WALL)
    gamma = 0.25
    s = glbe.rates(0.131, gamma)
    F = inputs.duct_force(shape)
    sim = _sim(shape, bc, gamma, s, "f64", F)
    sim.step(200)
    hist = sim.history()
    fl = glbe.Flow(shape, bc, F, gamma, s)
    fl.step(200)
    steps = {int(h[0]): h for h in hist}
    assert sorted(steps) == list(range(10, 201, 10))
    # R is a relative difference of velocities 10 steps apart: an FP64 state error
    # of ~1e-16 |u| shows up as ~1e-16 / R relative in R
    # R compares velocities 10 steps apart: FP64 velocity differences of a few
    # units of 1e-16 |u| between the two operation orders give a few 1e-17 in R
    # (measured at most 6.3e-17); the relative part covers the state's drift
    for t, r in fl.history:
        assert abs(steps[t][1] - r) <= 1e-15 + 1e-12 * r
    mass, q = sim.reductions()
    assert abs(mass) < 1e-14
    # the duct's flow rate vanishes by antisymmetry: compare on the scale of sum |j_x|
    _, _, j, _ = glbe.fields(glbe.stream(fl.post, bc), fl.F, gamma)
    scale = np.abs(j[0]).sum() / shape[0]
    assert abs(q - fl.flow_rate()) < 1e-13 * scale


def test_moments_match_oracle():
    torch = _torch()
    shape, bc = (8, 6, 10), (PER, WALL, WALL)
    d0 = inputs.random_deviations(shape, seed=6, amp=1e-3)
    F = inputs.random_force(shape, seed=6, amp=1e-4)
    sim = _sim(shape, bc, 0.3, glbe.rates(0.1, 0.3), "f64", F)
    sim.set_state(to_gpu_f(d0, torch.float64))
    rho, u, B = sim.moments("f64")
    drho, rho_o, j, u_o = glbe.fields(glbe.stream(d0, bc), F, 0.3)
    assert B is None
    assert rel(rho.cpu().numpy(), rho_o) < 1e-15
    assert rel(u.cpu().numpy(), u_o) < 1e-14
    mass, q = sim.reductions()
    assert abs(mass - drho.sum()) < 1e-15
    assert abs(q - j[0].sum() / shape[0]) < 1e-15


def test_mass_conserved_fp64_and_fp32():
    torch = _torch()
    shape, bc = (16, 12, 20), (PER, WALL, WALL)
    F = inputs.random_force(shape, seed=7, amp=1e-5)
    for storage, tol in (("f64", 1e-13), ("f32", 1e-4)):
        sim = _sim(shape, bc, 0.1, glbe.rates(0.05, 0.1), storage, F)
        sim.step(500)
        mass, _ = sim.reductions()
        assert abs(mass) < tol * shape[0] * shape[1] * shape[2] * 1e-3, (storage, mass)


def test_poiseuille_workload_matches_oracle_and_parabola():
    """Plane Poiseuille 8x8x32, FP64, gamma 1 and 0.1, to residual 1e-10: same
    crossing step and same state as the oracle (1x1x32 by homogeneity), and
    within the wall-slip error of the analytic parabola (Sec. 5)."""
    cfg = inputs.POISEUILLE
    H = cfg["shape"][2]
    for gamma in cfg["gammas"]:
        announce("poiseuille gamma=%g" % gamma)
        s = glbe.rates(cfg["nu"], gamma)
        sim = _sim(cfg["shape"], cfg["bc"], gamma, s, "f64", np.array(cfg["F"]))
        steps, r = sim.run_to_residual(cfg["tol"], 400000, poll_every=1000)
        assert steps > 0 and r < cfg["tol"]
        fl = glbe.Flow((1, 1, H), cfg["bc"], np.array(cfg["F"]), gamma, s)
        assert fl.run_to(cfg["tol"], 400000)
        assert fl.t == steps
        # bring the GPU run back to the crossing step
        sim2 = _sim(cfg["shape"], cfg["bc"], gamma, s, "f64", np.array(cfg["F"]))
        sim2.step(steps)
        _, u, _ = sim2.moments("f64")
        ug = u[0].cpu().numpy()
        assert np.ptp(ug, axis=(1, 2)).max() < 1e-17
        uo = fl.velocity()[0][:, 0, 0]
        assert rel(ug[:, 0, 0], uo) < 1e-12  # measured 3.7e-14 (gamma 1), 1.4e-15 (0.1)
        z = np.arange(H) + 0.5
        par = cfg["F"][0] * z * (H - z) / (2 * cfg["nu"])
        assert rel(ug[:, 0, 0], par) < 5e-3


def test_state_roundtrip_and_step_counter():
    torch = _torch()
    shape, bc = (8, 6, 10), (PER, WALL, WALL)
    sim = _sim(shape, bc, 0.5, glbe.rates(0.1, 0.5), "f32", np.array([1e-5, 0, 0]))
    sim.step(13)
    st = sim.get_state()
    assert sim.t == 13
    sim.step(5)
    a = sim.get_state()
    sim.set_state(st, step=13)
    sim.step(5)
    assert torch.equal(a, sim.get_state())
    assert sim.t == 18


def test_large_grid_sampled_nodes_fp32():
    """Full-size duct (256^3, FP32, bench launch configuration): one step from a
    seeded random state, checked at sampled nodes (all corners included)."""
    torch = _torch()
    cfg = inputs.DUCT256
    shape = cfg["shape"]
    announce("256^3 sampled parity")
    d0 = inputs.random_deviations(shape, seed=8, amp=1e-3, dtype=np.float32)
    F = inputs.duct_force(shape, cfg["F0"], dtype=np.float32)
    s = glbe.rates(cfg["nu"], cfg["gamma"])
    sim = _sim(shape, cfg["bc"], cfg["gamma"], s, "f32", F)
    sim.set_state(torch.from_numpy(d0).cuda())
    sim.step(1)
    out = sim.get_state()
    nodes = inputs.random_nodes(shape, 4000, seed=8)
    ref = glbe.step_nodes(d0.astype(np.float64), F.astype(np.float64), cfg["gamma"], s,
                          cfg["bc"], nodes)
    idx = torch.tensor(nodes, device="cuda")
    got = out[:, idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()
    assert rel(got, ref) < 2e-6
    del sim, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_naive_source_mode_matches_oracle(storage):
    """Sec. 3.1 negative control (S* = S/gamma): same parity bar as the paper's form."""
    torch = _torch()
    shape, bc = (8, 6, 10), (PER, WALL, WALL)
    gamma = 0.2
    d0 = inputs.random_deviations(shape, seed=21, amp=1e-3)
    F = inputs.random_force(shape, seed=21, amp=1e-4)
    if storage == "f32":
        d0 = d0.astype(np.float32).astype(np.float64)
        F = F.astype(np.float32).astype(np.float64)
    s = glbe.rates(0.05, gamma)
    sim = _sim(shape, bc, gamma, s, storage, F, source="naive")
    sim.set_state(to_gpu_f(d0, torch.float64 if storage == "f64" else torch.float32))
    sim.step(5)
    out = from_gpu_f(sim.get_state())
    ref = d0
    for _ in range(5):
        ref, _ = glbe.step(ref, F, gamma, s, bc, source="naive")
    assert rel(out, ref) < (1e-13 if storage == "f64" else 5e-6)
    cons = d0
    for _ in range(5):
        cons, _ = glbe.step(cons, F, gamma, s, bc)
    assert rel(cons, ref) > 1e-6


@pytest.mark.parametrize("shape", [(5, 7, 9), (64, 3, 4)])
def test_moving_walls_match_oracle(shape):
    """Every face moving with its own velocity (edges and corners take the mean
    of the crossed faces' wall terms): FP64 steps against the oracle (nx = 64:
    the row-aligned variant)."""
    torch = _torch()
    bc = (WALL, WALL, WALL)
    rng = np.random.default_rng(31)
    wu = 0.01 * rng.uniform(-1, 1, (6, 3))
    d0 = inputs.random_deviations(shape, seed=31, amp=1e-3)
    F = inputs.random_force(shape, seed=31, amp=1e-5)
    s = glbe.rates(0.05, 0.3)
    sim = _sim(shape, bc, 0.3, s, "f64", F, wall_u=wu)
    sim.set_state(to_gpu_f(d0, torch.float64))
    sim.step(20)
    out = from_gpu_f(sim.get_state())
    ref = d0
    for _ in range(20):
        ref, _ = glbe.step(ref, F, 0.3, s, bc, wall_u=wu)
    assert rel(out, ref) < 1e-12
    _, u, _ = sim.moments("f64")
    uo = glbe.fields(glbe.stream(ref, bc, wall_u=wu), F, 0.3)[3]
    assert rel(u.cpu().numpy(), uo) < 1e-12


def test_lid_driven_cavity_preconditioning():
    """32^3 lid-driven cube (Sec. 5), Re = 100 (U0 = 0.0235, nu = 0.0075), FP64:
    gamma = 0.1 reaches the steady state in fewer steps and agrees with gamma = 1
    to the compressibility / slip level."""
    shape, bc = (32, 32, 32), (WALL, WALL, WALL)
    wu = np.zeros((6, 3))
    wu[5] = [0.0235, 0.0, 0.0]
    res = {}
    for gamma in (1.0, 0.1):
        announce("cavity gamma=%g" % gamma)
        sim = _sim(shape, bc, gamma, glbe.rates(0.0075, gamma), "f64", np.zeros(3), wall_u=wu)
        steps, r = sim.run_to_residual(1e-8, 400000, poll_every=500)
        assert steps > 0, r
        _, u, _ = sim.moments("f64")
        res[gamma] = (steps, u.cpu().numpy())
        mass, _ = sim.reductions()
        assert abs(mass) < 1e-10
    announce("cavity steps gamma=1: %d, gamma=0.1: %d, rel diff %.3e"
             % (res[1.0][0], res[0.1][0], rel(res[0.1][1], res[1.0][1])))
    assert res[1.0][0] > 3 * res[0.1][0]
    assert rel(res[0.1][1], res[1.0][1]) < 0.05


def test_paper_low_viscosity_poiseuille():
    """The paper's low-viscosity Poiseuille case (gap 64, nu = 0.001,
    u_max = 0.00051, Re = 32.6), FP64 to 1e-8: the parabola, and roughly
    tenfold fewer steps per tenfold smaller gamma (51,430 at gamma = 0.01,
    6,070 at 0.001; 3.2 million at gamma = 1, not run here)."""
    import paper_0809_4730_amd as pkg
    from paper_0809_4730_amd import stability
    announce("paper poiseuille nu=0.001")
    nu, umax, H = 0.001, 0.00051, 64
    F = stability.poiseuille_force(nu, umax, H)
    z = np.arange(H) + 0.5
    exact = umax * (1.0 - ((z - H / 2) / (H / 2)) ** 2)
    n = {}
    for g in (0.01, 0.001):
        sim = pkg.Simulation((4, 4, H), (PER, PER, WALL), g, pkg.default_rates(nu, g),
                             storage="f64", force=(F, 0.0, 0.0))
        n[g], _ = sim.run_to_residual(1e-8, 200000, poll_every=1000)
        assert n[g] > 0
        _, u, _ = sim.moments("f64")
        assert rel(u[0].cpu().numpy()[:, 0, 0], exact) < 1e-3
    assert 5 * n[0.001] < n[0.01]


def test_duct_steady_state_agrees_across_gamma():
    """Preconditioning changes the transient, not the steady state, up to the
    compressibility error (App. B).  The 64^3 duct (C1 force, nu = 0.131,
    Ma ~ 0.01), FP64 to a residual of 1e-10 at gamma = 1, 0.5, 0.1, 0.05: with
    the energy-flux and third-order rates tied to a fixed Lambda = 3/16 (so
    that the wall slip does not change with gamma) the steady velocity agrees
    with gamma = 1 to within Ma^2 / gamma, the order of the preconditioned
    equilibrium's nonlinear terms (measured: 1.2e-7, 1.6e-5, 1.3e-4); with the
    paper's fixed s_q the slip moves with nu/gamma and the states differ by
    less than 1% (measured: 3.6e-4, 3.3e-3, 6.8e-3)."""
    import torch

    import paper_0809_4730_amd as pkg
    shape, bc, nu = (64, 64, 64), (PER, WALL, WALL), 0.131
    F = torch.tensor(inputs.duct_force(shape, 1e-5), dtype=torch.float64, device="cuda")
    for mode in ("lambda", "paper"):
        ref = None
        for gamma in (1.0, 0.5, 0.1, 0.05):
            announce("duct steady state, %s rates, gamma=%g" % (mode, gamma))
            sim = pkg.Simulation(shape, bc, gamma, pkg.default_rates(nu, gamma, mode, 3 / 16),
                                 storage="f64", force=F)
            steps, r = sim.run_to_residual(1e-10, 400000, poll_every=500)
            assert steps > 0, r
            _, u, _ = sim.moments("f64")
            u = u.cpu().numpy()
            sim.close()
            if ref is None:
                ref = u
                ma = float(np.abs(u[0]).max()) * np.sqrt(3.0)
                assert 0.005 < ma < 0.02
                continue
            d = rel(u, ref)
            announce("  rel diff vs gamma = 1: %.3e (Ma^2/gamma %.3e)" % (d, ma * ma / gamma))
            if mode == "lambda":
                assert d < ma * ma / gamma
            else:
                assert d < 1e-2
