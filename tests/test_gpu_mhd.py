"""GPU parity of the coupled GLBE + D3Q7 induction LKE step (Sec. 4, 4.1).

FP64 storage matches the oracle to 1e-12 relative; FP32 to FP32 rounding; the
Hartmann workload (32x32x128, FP32, gamma = gamma_m = 0.1) reaches the textbook
profiles within the discretisation error of the oracle at the same resolution.
"""
import numpy as np
import pytest

from oracle import glbe, mhd
from oracle.lattice import W7
from paper_0809_4730_amd import inputs
from tests.gpu_util import announce, from_gpu_f, from_gpu_g, rel, to_gpu_f, to_gpu_g

pytestmark = pytest.mark.gpu
PER, WALL = "periodic", "wall"


def _mhd_sim(shape, bc, gamma, s, storage, F, p):
    import paper_0809_4730_amd as pkg
    return pkg.Simulation(shape, bc, gamma, s, storage=storage, force=tuple(F), mhd=p)


def _random_g(shape, seed, B0, amp=1e-4):
    nx, ny, nz = shape
    g = mhd.initial_g(shape, B0)
    g += inputs.random_deviations(shape, seed=seed, amp=amp, q=21).reshape(3, 7, nz, ny, nx)
    return g


@pytest.mark.parametrize("shape,bc", [((6, 8, 5), (PER, WALL, PER)),
                                      ((5, 6, 7), (WALL, WALL, WALL)),
                                      ((8, 4, 4), (PER, PER, PER)),
                                      # nx a multiple of 64: the row-aligned form
                                      ((64, 3, 4), (PER, WALL, WALL)),
                                      ((128, 2, 3), (WALL, WALL, PER))])
@pytest.mark.parametrize("nsteps", [1, 40])
def test_mhd_fp64_matches_oracle(shape, bc, nsteps):
    import torch
    announce("mhd fp64 %s %s n=%d" % (shape, bc, nsteps))
    gamma, gm = 0.2, 0.3
    B0 = np.array([0.01, 0.03, -0.02])
    p = dict(gamma_m=gm, chi=0.05, eta=0.02, B0=tuple(B0))
    s = glbe.rates(0.05, gamma)
    F = np.array([1e-5, 2e-6, -3e-6])
    f0 = inputs.random_deviations(shape, seed=11, amp=1e-3)
    g0 = _random_g(shape, 12, B0)
    sim = _mhd_sim(shape, bc, gamma, s, "f64", F, p)
    sim.set_state(to_gpu_f(f0, torch.float64), to_gpu_g(g0, torch.float64, B0))
    sim.step(nsteps)
    fg, gg = sim.get_state()
    fo, go = f0, g0
    pp = dict(gamma=gamma, s=s, gamma_m=gm, chi=p["chi"], eta=p["eta"], B_wall=B0)
    Ff = inputs.uniform_force(shape, F)
    for _ in range(nsteps):
        fo, go, u, B = mhd.step(fo, go, Ff, pp, bc)
    assert rel(from_gpu_f(fg), fo) < 1e-12
    assert rel(from_gpu_g(gg, B0), go) < 1e-13
    rho, ug, Bg = sim.moments("f64")
    # fields of the streamed current state, with the self-consistent Lorentz force
    f_s = glbe.stream(fo, bc)
    g_s = mhd.stream_g(go, bc, B0)
    rho_o, u_o, B_o, J_o, F_o = mhd.coupled_fields(f_s, g_s, Ff, gamma, gm, p["chi"], p["eta"])
    # u is a cancelling sum of populations much larger than it (after 40 steps
    # from a random state the velocity has decayed, the deviations have not):
    # the momentum rho u is held to the 1e-12 bar against the populations it
    # sums, u itself to 1e-11 relative to u (measured up to 2.3e-12, where the
    # states agree to 7.8e-14)
    mom_g = rho.cpu().numpy() * ug.cpu().numpy()
    assert np.linalg.norm(mom_g - rho_o * u_o) < 1e-12 * np.linalg.norm(f_s)
    assert rel(ug.cpu().numpy(), u_o) < 1e-11
    assert rel(Bg.cpu().numpy(), B_o) < 1e-14


@pytest.mark.parametrize("shape", [(6, 8, 5), (32, 32, 128)])
def test_mhd_fp32_single_step(shape):
    """One coupled FP32 step from a random state against the oracle, on a small
    lattice and at the Hartmann workload's full size (its launch shape)."""
    import torch
    announce("mhd fp32 single step %s" % (shape,))
    bc = (PER, WALL, PER)
    gamma, gm = 0.1, 0.1
    B0 = np.array([0.0, 0.03, 0.0])
    p = dict(gamma_m=gm, chi=0.01, eta=0.025, B0=tuple(B0))
    s = glbe.rates(0.1, gamma)
    F = np.array([1e-5, 0.0, 0.0])
    f0 = inputs.random_deviations(shape, seed=13, amp=1e-3).astype(np.float32).astype(np.float64)
    nx, ny, nz = shape
    # FP32 stores g - W B0: give both sides deviations that FP32 holds exactly
    dev = inputs.random_deviations(shape, seed=14, amp=1e-4, q=21).astype(np.float32)
    g0 = mhd.initial_g(shape, B0) + dev.astype(np.float64).reshape(3, 7, nz, ny, nx)
    sim = _mhd_sim(shape, bc, gamma, s, "f32", F, p)
    sim.set_state(to_gpu_f(f0, torch.float32), to_gpu_g(g0, torch.float32, B0))
    sim.step(1)
    fg, gg = sim.get_state()
    pp = dict(gamma=gamma, s=s, gamma_m=gm, chi=p["chi"], eta=p["eta"], B_wall=B0)
    fo, go, _, _ = mhd.step(f0, g0, inputs.uniform_force(shape, F), pp, bc)
    assert rel(from_gpu_f(fg), fo) < 2e-6
    assert rel(from_gpu_g(gg, B0), go) < 1e-6
    # the deviation from W B0 (what FP32 stores) is itself accurate
    from tests.gpu_util import _rest_g
    rest = _rest_g(go.shape, B0)
    assert rel(from_gpu_g(gg, B0) - rest, go - rest) < 1e-5


@pytest.mark.parametrize("Ha", [5.0, 10.0, 20.0])
@pytest.mark.parametrize("Pm", [0.01, 0.1])
def test_hartmann_workload(Ha, Pm):
    """32x32x128, walls normal to y (the applied-field direction), FP32,
    gamma = gamma_m = 0.1, to residual 1e-8; compared with the oracle on the
    same y-resolution (1x32x1 by homogeneity) and the closed forms."""
    cfg = inputs.HARTMANN
    announce("hartmann Ha=%g Pm=%g" % (Ha, Pm))
    ny = cfg["shape"][1]
    B0, chi = inputs.hartmann_parameters(Ha, Pm, ny, cfg["nu"], cfg["eta"])
    p = dict(gamma_m=cfg["gamma_m"], chi=chi, eta=cfg["eta"], B0=(0.0, B0, 0.0))
    s = glbe.rates(cfg["nu"], cfg["gamma"])
    sim = _mhd_sim(cfg["shape"], cfg["bc"], cfg["gamma"], s, "f32", cfg["F"], p)
    # FP32 storage stalls near a residual of 5e-8 at this Mach number (rounding of
    # the stored deviations), so the march goes to 2e-7 and then 2000 more steps
    steps, r = sim.run_to_residual(2e-7, 200000, poll_every=500)
    assert steps > 0, r
    sim.step(2000)
    _, u, B = sim.moments("f64")
    ug = u[0].cpu().numpy()
    bg = B[0].cpu().numpy()
    assert np.ptp(ug, axis=(0, 2)).max() < 1e-6 * np.abs(ug).max()
    ug, bg = ug[0, :, 0], bg[0, :, 0]
    L = ny / 2
    y = np.arange(ny) + 0.5 - L
    F = cfg["F"][0]
    uex = F * L * L / (cfg["nu"] * Ha) * (np.cosh(Ha) - np.cosh(Ha * y / L)) / np.sinh(Ha)
    bex = chi * F * L / B0 * (np.sinh(Ha * y / L) / np.sinh(Ha) - y / L)
    fl = mhd.MHDFlow((1, ny, 1), cfg["bc"], np.array(cfg["F"]), cfg["gamma"], s, cfg["gamma_m"],
                     chi, cfg["eta"], np.array([0.0, B0, 0.0]))
    assert fl.run_to(1e-10, 200000)
    uo, bo = fl.u[0][0, :, 0], fl.B[0][0, :, 0]
    assert rel(ug, uo) < 1e-4
    assert rel(bg, bo) < 1e-3
    # paper rates at gamma = 0.1 put the bounce-back slip at Lambda ~ 1, and the
    # Ha = 20 layer (L/Ha = 0.8 cells) is under-resolved: oracle errors are
    # 0.9 / 3.5 / 13 % in u and 1.2 / 2.4 / 5.5 % in b for Ha = 5 / 10 / 20
    tol = {5.0: 0.015, 10.0: 0.05, 20.0: 0.15}[Ha]
    assert rel(uo, uex) < tol and rel(bo, bex) < tol


def test_hartmann_fp64_steady_state_matches_oracle():
    """The Hartmann workload (32x32x128, Ha = 10, Pm = 0.01, gamma = gamma_m =
    0.1) in FP64 storage marched to R < 1e-8.  x and z are periodic and the
    flow is homogeneous along them, so the oracle marches one 1 x 32 x 1
    column (its residual equals the whole lattice's): both cross at the same
    step, and there the GPU's flow and induction populations at every (x, z)
    equal the oracle's column to 1e-12 relative (deviations from the rest
    state), its velocity and induced field likewise."""
    import torch
    announce("hartmann fp64 steady state against the oracle")
    cfg = inputs.HARTMANN
    shape, ny = cfg["shape"], cfg["shape"][1]
    gamma, gm = cfg["gamma"], cfg["gamma_m"]
    B0, chi = inputs.hartmann_parameters(10.0, 0.01, ny, cfg["nu"], cfg["eta"])
    B0v = np.array([0.0, B0, 0.0])
    p = dict(gamma_m=gm, chi=chi, eta=cfg["eta"], B0=tuple(B0v))
    s = glbe.rates(cfg["nu"], gamma)
    sim = _mhd_sim(shape, cfg["bc"], gamma, s, "f64", cfg["F"], p)
    steps, r = sim.run_to_residual(1e-8, 100000, poll_every=100)
    assert steps > 0 and r < 1e-8
    sim.close()
    col = (1, ny, 1)
    fl = mhd.MHDFlow(col, cfg["bc"], np.array(cfg["F"]), gamma, s, gm, chi, cfg["eta"], B0v)
    assert fl.run_to(1e-8, 100000)
    assert fl.t == steps
    sim = _mhd_sim(shape, cfg["bc"], gamma, s, "f64", cfg["F"], p)
    sim.step(steps)
    fg, gg = sim.get_state()
    f = from_gpu_f(fg)
    g = from_gpu_g(gg, B0v) - mhd.initial_g(shape, B0v)
    fo = np.broadcast_to(fl.post_f, f.shape)
    go = np.broadcast_to(fl.post_g - mhd.initial_g(col, B0v), g.shape)
    err_f, err_g = rel(f, fo), rel(g, go)
    _, ug, Bg = sim.moments("f64")
    Ff = inputs.uniform_force(col, np.array(cfg["F"]))
    f_s = glbe.stream(fl.post_f, cfg["bc"])
    g_s = mhd.stream_g(fl.post_g, cfg["bc"], B0v)
    _, u_o, B_o, _, _ = mhd.coupled_fields(f_s, g_s, Ff, gamma, gm, chi, cfg["eta"])
    ug, bg = ug.cpu().numpy(), Bg.cpu().numpy() - B0v.reshape(3, 1, 1, 1)
    err_u = rel(ug, np.broadcast_to(u_o, ug.shape))
    err_b = rel(bg, np.broadcast_to(B_o - B0v.reshape(3, 1, 1, 1), bg.shape))
    announce("step %d: f %.3e, g %.3e, u %.3e, b %.3e" % (steps, err_f, err_g, err_u, err_b))
    assert max(err_f, err_g, err_u, err_b) < 1e-12


def test_paper_hartmann_preconditioning_ordering():
    """The paper's (gamma, gamma_m) findings on its own Hartmann case (Re = 286,
    Ha = 71.6, Pm = 1e-6, nu = eta = 0.004, half-width 64), FP64 to 1e-8: at
    gamma = 0.05, gamma_m = gamma converges fastest, a smaller gamma_m is slower
    and gamma_m = 1 slowest; with gamma = 1, preconditioning only the induction
    equation is slower than preconditioning neither."""
    import paper_0809_4730_amd as pkg
    announce("paper hartmann (gamma, gamma_m) ordering")
    nu = eta = 0.004
    ny, Ha = 128, 71.6
    B0, chi = inputs.hartmann_parameters(Ha, 1e-6, ny, nu, eta)
    F = (286 * nu / (ny / 2)) * nu * Ha / (ny / 2) ** 2

    def steps(g, gm):
        sim = pkg.Simulation((4, ny, 4), (PER, WALL, PER), g, pkg.default_rates(nu, g),
                             storage="f64", force=(F, 0.0, 0.0),
                             mhd=dict(gamma_m=gm, chi=chi, eta=eta, B0=(0.0, B0, 0.0)))
        n, _ = sim.run_to_residual(1e-8, 1000000, poll_every=1000)
        assert n > 0
        return n
    s_eq, s_lo, s_mid, s_one = steps(0.05, 0.05), steps(0.05, 0.02), steps(0.05, 0.2), steps(0.05, 1.0)
    assert s_eq < s_lo < s_mid < s_one
    assert steps(1.0, 1.0) < steps(1.0, 0.2)
