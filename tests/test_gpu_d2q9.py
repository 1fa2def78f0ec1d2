"""GPU parity of the two-dimensional variants (D2Q9 flow, D2Q5 induction)
against the 2D oracle: single and repeated steps in FP64 (1e-12), FP32 and
16-bit storage, fields, residual history, and the Poiseuille and Hartmann
workloads against their closed forms."""
import numpy as np
import pytest

from oracle import d2q9 as d
from paper_0809_4730_amd import inputs
from tests.gpu_util import announce, rel

pytestmark = pytest.mark.gpu
PER, WALL = "periodic", "wall"


def _perm(q):
    import paper_0809_4730_amd as pkg
    e_lib = pkg.lattice_velocities(q)[:, :2]
    e_or = d.E9 if q == 9 else d.E5
    idx = {tuple(v): a for a, v in enumerate(e_or)}
    return np.array([idx[tuple(v)] for v in e_lib])


def _to_f(f, dtype):
    """Oracle (9, ny, nx) -> library state (9, 1, ny, nx)."""
    import torch
    p = _perm(9)
    return torch.tensor(np.ascontiguousarray(f[p][:, None]), dtype=torch.float64,
                        device="cuda").to(dtype)


def _from_f(t):
    import torch
    p = _perm(9)
    a = t.to(torch.float64).cpu().numpy()[:, 0]
    out = np.empty_like(a)
    out[p] = a
    return out


def _rest_g(shape, B0):
    nx, ny = shape
    return d.initial_g((nx, ny), B0)


def _to_g(g, dtype, B0):
    import torch
    p = _perm(5)
    dev = g - _rest_g((g.shape[3], g.shape[2]), B0)
    return torch.tensor(np.ascontiguousarray(dev[:, p][:, :, None]), dtype=torch.float64,
                        device="cuda").to(dtype)


def _from_g(t, B0):
    import torch
    p = _perm(5)
    a = t.to(torch.float64).cpu().numpy()[:, :, 0]
    out = np.empty_like(a)
    out[:, p] = a
    return out + _rest_g((a.shape[3], a.shape[2]), B0)


def _sim(shape, bc, gamma, s, storage, force, mhd=None, launch=None):
    import paper_0809_4730_amd as pkg
    nx, ny = shape
    return pkg.Simulation((nx, ny, 1), (bc[0], bc[1], PER), gamma, s, storage=storage, force=force,
                          mhd=mhd, lattice="d2q9", launch=launch)


def _field_force(shape, seed, amp=1e-5):
    nx, ny = shape
    return amp * np.random.default_rng(seed).uniform(-1, 1, (2, ny, nx))


def _lib_force(F, dtype):
    import torch
    F3 = np.concatenate([F, np.zeros_like(F[:1])])[:, None]
    return torch.tensor(F3, dtype=dtype, device="cuda")


GRIDS = [((7, 9), (PER, WALL)), ((5, 6), (WALL, WALL)), ((8, 4), (PER, PER)), ((300, 5), (PER, WALL))]


@pytest.mark.parametrize("shape,bc", GRIDS)
@pytest.mark.parametrize("nsteps", [1, 40])
def test_d2q9_fp64_matches_oracle(shape, bc, nsteps):
    import torch
    announce("d2q9 fp64 %s %s n=%d" % (shape, bc, nsteps))
    gamma = 0.3
    s = d.rates(0.05, gamma)
    nx, ny = shape
    f0 = inputs.random_deviations((nx, ny, 1), seed=31, amp=1e-3, q=9)[:, 0]
    F = _field_force(shape, 32)
    sim = _sim(shape, bc, gamma, s, "f64", _lib_force(F, torch.float64))
    sim.set_state(_to_f(f0, torch.float64))
    sim.step(nsteps)
    fo = f0
    for _ in range(nsteps):
        fo, u = d.step(fo, F, gamma, s, bc)
    assert rel(_from_f(sim.get_state()), fo) < 1e-12
    rho, ug, _ = sim.moments("f64")
    fs = d.stream(fo, bc)
    _, rho_o, _, u_o = d.fields(fs, F, gamma)
    ug = ug.cpu().numpy()[:, 0]
    assert rel(ug[:2], u_o) < 1e-12
    assert np.all(ug[2] == 0.0)
    assert rel(rho.cpu().numpy()[0], rho_o) < 1e-14


@pytest.mark.parametrize("storage,tol", [("f32", 2e-6), ("bf16", 1e-2), ("f16", 2e-3)])
def test_d2q9_reduced_precision_single_step(storage, tol):
    import torch
    shape, bc = (33, 17), (PER, WALL)
    gamma = 0.2
    s = d.rates(0.04, gamma)
    nx, ny = shape
    f0 = inputs.random_deviations((nx, ny, 1), seed=41, amp=1e-3, q=9)[:, 0]
    dt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[storage]
    f0 = _from_f(_to_f(f0, dt))  # values the storage holds exactly
    F = (2e-5, -1e-5)
    sim = _sim(shape, bc, gamma, s, storage, F)
    sim.set_state(_to_f(f0, dt))
    sim.step(1)
    fo, _ = d.step(f0, np.broadcast_to(np.array(F).reshape(2, 1, 1), (2, ny, nx)), gamma, s, bc)
    assert rel(_from_f(sim.get_state()), fo) < tol


def test_d2q9_residual_history_matches_oracle():
    import torch
    shape, bc = (16, 24), (PER, WALL)
    gamma, nu = 0.5, 0.1
    s = d.rates(nu, gamma)
    sim = _sim(shape, bc, gamma, s, "f64", (1e-5, 0.0))
    sim.step(200)
    h = sim.history(64)
    fl = d.Flow2D(shape, bc, (1e-5, 0.0), gamma, s)
    fl.step(200)
    ref = np.array([r for _, r in fl.history])
    # the library also records the first check (against a zero snapshot: 1)
    assert h[0, 1] == 1.0
    got = h[1:, 1]
    assert len(got) == len(ref)
    assert np.all(np.abs(got - ref) <= 1e-14 + 1e-8 * ref)
    mass, flow = sim.reductions()
    assert abs(mass) < 1e-12


def test_d2q9_poiseuille_workload_fp32():
    """Plane Poiseuille, 4 x 64, FP32 storage, gamma = 0.1, Lambda = 3/16: the
    steady profile is the parabola to FP32 accuracy."""
    nu, gamma, F, H = 0.1, 0.1, 1e-6, 64
    import paper_0809_4730_amd as pkg
    s = pkg.default_rates_d2q9(nu, gamma, "lambda", 3 / 16)
    assert np.allclose(s, d.rates(nu, gamma, "lambda", 3 / 16), rtol=1e-15)
    sim = _sim((4, H), (PER, WALL), gamma, s, "f32", (F, 0.0))
    steps, r = sim.run_to_residual(2e-7, 200000, poll_every=500)
    assert steps > 0
    sim.step(2000)
    _, u, _ = sim.moments("f64")
    u = u.cpu().numpy()[0, 0, :, 0]
    y = np.arange(H) + 0.5
    exact = F * y * (H - y) / (2 * nu)
    assert np.max(np.abs(u - exact)) / exact.max() < 1e-4


@pytest.mark.parametrize("shape,bc", [((6, 10), (PER, WALL)), ((5, 7), (WALL, WALL))])
@pytest.mark.parametrize("nsteps", [1, 40])
def test_d2q5_mhd_fp64_matches_oracle(shape, bc, nsteps):
    import torch
    announce("d2q5 mhd fp64 %s %s n=%d" % (shape, bc, nsteps))
    gamma, gm = 0.2, 0.3
    B0 = np.array([0.01, 0.03])
    p = dict(gamma_m=gm, chi=0.05, eta=0.02, B0=tuple(B0))
    s = d.rates(0.05, gamma)
    nx, ny = shape
    F = np.array([1e-5, -2e-6])
    f0 = inputs.random_deviations((nx, ny, 1), seed=51, amp=1e-3, q=9)[:, 0]
    g0 = d.initial_g(shape, B0) + inputs.random_deviations((nx, ny, 1), seed=52, amp=1e-4,
                                                            q=10).reshape(2, 5, ny, nx)
    sim = _sim(shape, bc, gamma, s, "f64", tuple(F), mhd=p)
    sim.set_state(_to_f(f0, torch.float64), _to_g(g0, torch.float64, B0))
    sim.step(nsteps)
    fg, gg = sim.get_state()
    pp = dict(gamma=gamma, s=s, gamma_m=gm, chi=p["chi"], eta=p["eta"], B_wall=B0)
    Ff = np.broadcast_to(F.reshape(2, 1, 1), (2, ny, nx))
    fo, go = f0, g0
    for _ in range(nsteps):
        fo, go, u, B = d.mhd_step(fo, go, Ff, pp, bc)
    assert rel(_from_f(fg), fo) < 1e-12
    assert rel(_from_g(gg, B0), go) < 1e-13
    rho_g, ug, Bg = sim.moments("f64")
    fs, gs = d.stream(fo, bc), d.stream_g(go, bc, B0)
    rho_o, u_o, B_o, _, _ = d.coupled_fields(fs, gs, Ff, gamma, gm, p["chi"], p["eta"])
    # u is a cancelling sum of populations much larger than it: the momentum
    # rho u is held to the 1e-12 bar against the populations it sums, u itself
    # to 1e-11 relative to u (measured up to 4.9e-13)
    mom_g = rho_g.cpu().numpy()[0] * ug.cpu().numpy()[:2, 0]
    assert np.linalg.norm(mom_g - rho_o * u_o) < 1e-12 * np.linalg.norm(fs)
    assert rel(ug.cpu().numpy()[:2, 0], u_o) < 1e-11
    assert rel(Bg.cpu().numpy()[:2, 0], B_o) < 1e-14
    assert np.all(Bg.cpu().numpy()[2] == 0.0)


def test_d2q5_hartmann_fp32_closed_form():
    """2D Hartmann flow (Ha = 10, Pm = 0.01, 2L = 32 between walls normal to y),
    FP32, gamma = gamma_m = 0.1: u and b_x against the insulating-wall profiles."""
    L, Ha, Pm, nu, eta, F = 16, 10.0, 0.01, 0.1, 0.025, 1e-5
    B0, chi = inputs.hartmann_parameters(Ha, Pm, 2 * L, nu, eta)
    import paper_0809_4730_amd as pkg
    s = pkg.default_rates_d2q9(nu, 0.1, "lambda", 3 / 16)
    sim = _sim((4, 2 * L), (PER, WALL), 0.1, s, "f32", (F, 0.0),
               mhd=dict(gamma_m=0.1, chi=chi, eta=eta, B0=(0.0, B0)))
    steps, _ = sim.run_to_residual(2e-7, 200000, poll_every=500)
    assert steps > 0
    sim.step(2000)
    _, u, B = sim.moments("f64")
    u = u.cpu().numpy()[0, 0, :, 0]
    b = B.cpu().numpy()[0, 0, :, 0]
    y = np.arange(2 * L) + 0.5 - L
    uex = F * L * L / (nu * Ha) * (np.cosh(Ha) - np.cosh(Ha * y / L)) / np.sinh(Ha)
    bex = chi * F * L / B0 * (np.sinh(Ha * y / L) / np.sinh(Ha) - y / L)
    eu = np.sqrt(np.mean((u - uex) ** 2)) / uex.max()
    eb = np.sqrt(np.mean((b - bex) ** 2)) / np.abs(bex).max()
    announce("d2q5 hartmann: steps %d eu %.3g eb %.3g" % (steps, eu, eb))
    # the oracle at the same resolution carries the same discretisation error
    # (2.3% and 1.5% here); the FP32 library must agree with it closely
    fl = d.MHDFlow2D((1, 2 * L), (PER, WALL), (F, 0.0), 0.1, s, 0.1, chi, eta, (0.0, B0))
    assert fl.run_to(1e-10, 60000)
    assert rel(u, fl.u[0][:, 0]) < 1e-4 and rel(b, fl.B[0][:, 0]) < 1e-3
    assert eu < 0.03 and eb < 0.025


@pytest.mark.parametrize("storage,mhd", [("f32", False), ("f64", False), ("bf16", False),
                                         ("f32", True)])
def test_wave_caps_and_store_forms_bitwise(storage, mhd):
    """The D2Q9 flow and coupled D2Q9 + D2Q5 steps under caps on the waves per
    SIMD and with both store forms, residual checks on: bit for bit."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("d2q9 wave caps %s mhd=%s" % (storage, mhd))
    nx, ny = 96, 37
    gamma = 0.3
    kw = dict(mhd=dict(gamma_m=0.4, chi=0.05, eta=0.03, B0=(0.01, 0.02))) if mhd else {}
    out = []
    for store, waves in (("cached", 8), ("streaming", 8), ("streaming", 6), ("cached", 4),
                         ("streaming", 3)):
        sim = pkg.Simulation((nx, ny, 1), (PER, WALL, PER), gamma, d.rates(0.05, gamma),
                             storage=storage, force=(1e-5, -2e-6), lattice="d2q9",
                             launch=dict(store=store, waves=waves), **kw)
        assert sim.launch["waves"] == waves
        sim.step(41)
        st = sim.get_state()
        out.append((st if torch.is_tensor(st) else torch.cat([st[0].reshape(-1), st[1].reshape(-1)]),
                    sim.history(8)))
    for a, b in zip(out[1:], out[:-1]):
        assert torch.equal(a[0], b[0])
        assert np.array_equal(a[1], b[1])


def test_d2q9_4096_launch_shape_one_step_at_sampled_nodes():
    """D2Q9 at 4096^2 (FP32, periodic x, walls in y) in the launch shape such a
    lattice gets (streaming stores, create-time XCD chunk, 6 waves per SIMD):
    one step from a seeded random state against the oracle's step from the same
    state at 4000 sampled nodes (corners included), 2e-6 relative."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("d2q9 4096^2 sampled nodes")
    nx = ny = 4096
    bc, gamma = (PER, WALL), 0.1
    s = d.rates(0.1, gamma)
    F = np.array([1e-5, -2e-6], dtype=np.float32).astype(np.float64)
    sim = _sim((nx, ny), bc, gamma, s, "f32", (F[0], F[1], 0.0))
    assert sim.launch["store"] == "streaming" and sim.launch["waves"] == 6
    rng = np.random.default_rng(71)
    f0 = (1e-3 * rng.uniform(-1.0, 1.0, (9, ny, nx))).astype(np.float32)
    sim.set_state(_to_f(f0.astype(np.float64), torch.float32))
    sim.step(1)
    out = sim.get_state()
    pick = np.random.default_rng(72).choice(nx * ny, 4000, replace=False)
    nodes = np.stack([pick % nx, pick // nx], axis=1)
    nodes[:4] = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)]
    idx = torch.tensor(nodes, device="cuda")
    got = out[:, 0, idx[:, 1], idx[:, 0]].double().cpu().numpy()
    sim.close()
    del sim, out
    torch.cuda.empty_cache()
    ref = d.step_nodes(f0, F, gamma, s, bc, nodes)[_perm(9)]
    assert rel(got, ref) < 2e-6


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_d2q9_4096_rest_plane_kept_bitwise(storage):
    """D2Q9 at 4096^2 with a uniform force (no field to keep in the last-level
    cache, so with FP32 storage the rest population's plane keeps cacheable
    loads and stores while the other planes stream; BF16 keeps its
    streaming stores and cacheable loads): three steps from a seeded state bit
    for bit equal to the same steps with every store cacheable.  The oracle
    comparison of this launch shape is the FP32 sampled-node test above."""
    import torch
    announce("d2q9 4096^2 %s, rest plane cached" % storage)
    nx = ny = 4096
    bc, gamma = (PER, WALL), 0.1
    s = d.rates(0.1, gamma)
    tdt = torch.float32 if storage == "f32" else torch.bfloat16
    rng = np.random.default_rng(73)
    f0 = _to_f(1e-3 * rng.uniform(-1.0, 1.0, (9, ny, nx)), tdt)
    outs = []
    for launch in (None, dict(store="cached")):
        sim = _sim((nx, ny), bc, gamma, s, storage, (1e-5, -2e-6, 0.0), launch=launch)
        if launch is None:
            assert sim.launch["store"] == "streaming"
        sim.set_state(f0)
        sim.step(1)
        outs.append(sim.get_state())
        sim.step(2)
        outs.append(sim.get_state())
        sim.close()
        del sim
    assert torch.equal(outs[0], outs[2]) and torch.equal(outs[1], outs[3])
    del outs
    torch.cuda.empty_cache()


def test_coupled_d2q9_4096_rest_plane_kept_bitwise():
    """The coupled D2Q9 + D2Q5 step at 4096^2, FP32, uniform force (the rest
    flow population's plane keeps cacheable loads and stores, the other flow
    planes and the induction planes stream): three steps bit for bit equal to
    the same steps with every store cacheable (and so every load cacheable)."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("coupled d2q9 4096^2 f32, rest plane cached")
    mhd = dict(gamma_m=0.4, chi=0.05, eta=0.03, B0=(0.01, 0.02))
    states = []
    for launch in (None, dict(store="cached")):
        sim = pkg.Simulation((4096, 4096, 1), (PER, WALL, PER), 0.3, d.rates(0.05, 0.3),
                             storage="f32", force=(1e-5, -2e-6), lattice="d2q9", launch=launch,
                             mhd=mhd)
        if launch is None:
            assert sim.launch["store"] == "streaming"
        sim.step(3)
        f, g = sim.get_state()
        states.append(torch.cat([f.reshape(-1), g.reshape(-1)]))
        sim.close()
        del sim
    assert torch.equal(states[0], states[1]) and bool(states[0].abs().max() > 0)
    del states
    torch.cuda.empty_cache()
