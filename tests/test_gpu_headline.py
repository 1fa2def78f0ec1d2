"""The kernels the benchmark times, in the launch shapes it times them, against
the FP64 oracle; the store and launch forms bit for bit; the failure path of
the instability detector; the residual history within a bound computed from
the measured velocity differences; the binding on a side stream.

Parity bars (FP32 storage, FP32 collision): one step from a seeded random
state within 2e-6 relative of the oracle's FP64 step from the same
FP32-representable state (one FP32 rounding of each stored value is 6e-8 of
it; the collision's FP32 arithmetic adds a few more).  Over n steps the
rounding errors of the steps add at most: in the orthonormal moment basis the
collision scales every non-conserved moment by 1 - s_k with |1 - s_k| < 1
and streaming with bounce-back permutes values, so the linear part of the
step does not amplify an L2 error, and the nonlinear terms are O(Ma) smaller.
The bound after n steps is therefore n * 2e-6 * |d0| / |d_n|.
"""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import glbe
from paper_0809_4730_amd import inputs
from tests.gpu_util import announce, rel

pytestmark = pytest.mark.gpu
PER, WALL = "periodic", "wall"
STEP_TOL = 2e-6


def _duct_sim(shape, storage, gamma, **kw):
    import torch

    import paper_0809_4730_amd as pkg
    cfg = inputs.DUCT64
    dt = torch.float64 if storage == "f64" else torch.float32
    F = torch.tensor(inputs.duct_force(shape, cfg["F0"]), dtype=dt, device="cuda")
    return pkg.Simulation(shape, cfg["bc"], gamma, pkg.default_rates(cfg["nu"], gamma),
                          storage=storage, force=F, **kw)


def test_duct64_fp32_bench_kernel_one_and_fifty_steps():
    """The 64^3 FP32 duct at gamma = 0.1 in its default launch shape (row-aligned
    waves, one slab per XCD, cacheable stores, 32-bit offsets): 1 and 50 steps
    from a seeded random state against the oracle, node by node."""
    import torch
    announce("64^3 fp32 duct, bench launch shape, 1 + 49 steps")
    shape, gamma = (64, 64, 64), 0.1
    cfg = inputs.DUCT64
    sim = _duct_sim(shape, "f32", gamma)
    lp = sim.launch
    assert lp["store"] == "cached" and lp["offsets"] == "narrow"
    assert lp["xcd_chunk"] >= (64 ** 3 // 256 + 7) // 8  # one slab per XCD
    d0 = inputs.random_deviations(shape, seed=11, amp=1e-3, dtype=np.float32)
    F = inputs.duct_force(shape, cfg["F0"]).astype(np.float32).astype(np.float64)
    s = glbe.rates(cfg["nu"], gamma)
    sim.set_state(torch.from_numpy(d0).cuda())
    sim.step(1)
    out1 = sim.get_state().double().cpu().numpy()
    ref = d0.astype(np.float64)
    ref, _ = glbe.step(ref, F, gamma, s, cfg["bc"])
    assert rel(out1, ref) < STEP_TOL
    assert rel(out1 - d0, ref - d0) < 10 * STEP_TOL
    sim.step(49)
    for _ in range(49):
        ref, _ = glbe.step(ref, F, gamma, s, cfg["bc"])
    out50 = sim.get_state().double().cpu().numpy()
    bound = 50 * STEP_TOL * np.linalg.norm(d0) / np.linalg.norm(ref)
    err = rel(out50, ref)
    announce("50 steps: rel %.3e, bound %.3e" % (err, bound))
    assert err < bound


def test_duct64_fp64_steady_state_matches_oracle():
    """The 64^3 duct (its force, nu = 0.131) marched in FP64 storage at
    gamma = 0.05 to a residual of 1e-8 (the Sec. 5 stopping rule, checked every
    10 steps): the GPU crosses at the oracle's step, and at that step its
    state and velocity equal the oracle's to 1e-12 relative.  The oracle
    takes some 40 s for the 580 steps."""
    announce("64^3 fp64 duct, gamma 0.05, steady state against the oracle")
    shape, gamma, tol = (64, 64, 64), 0.05, 1e-8
    cfg = inputs.DUCT64
    sim = _duct_sim(shape, "f64", gamma)
    steps, r = sim.run_to_residual(tol, 20000, poll_every=100)
    assert steps > 0 and r < tol
    sim.close()
    fl = glbe.Flow(shape, cfg["bc"], inputs.duct_force(shape, cfg["F0"]), gamma,
                   glbe.rates(cfg["nu"], gamma))
    assert fl.run_to(tol, 20000)
    assert fl.t == steps
    sim = _duct_sim(shape, "f64", gamma)
    sim.step(steps)
    err_f = rel(sim.get_state().cpu().numpy(), fl.post)
    _, u, _ = sim.moments("f64")
    err_u = rel(u.cpu().numpy(), fl.velocity())
    announce("steady state at step %d: state rel %.3e, u rel %.3e" % (steps, err_f, err_u))
    assert err_f < 1e-12 and err_u < 1e-12


@pytest.mark.parametrize("storage,check", [("f32", False), ("f32", True), ("f64", False),
                                           ("bf16", False), ("f16", True)])
def test_duct256_bench_kernel_one_step(storage, check):
    """The 256^3 duct at gamma = 1 in the benchmark's launch shape for each
    storage type (create-time XCD chunk, streaming loads and stores, the
    library's cap on waves per SIMD): a seeded random state (rounded to the
    storage type on the host) loaded at step 18 (or 19), one plain (or
    residual-check) step, compared with the oracle's step from that same
    seeded state at 4000 sampled nodes, corners included.  Bars: FP64 1e-12,
    FP32 2e-6 relative; BF16 / FP16 one rounding of each stored value (nearest
    even) plus the FP32 collision's error, element by element, and the stored
    value equal to the oracle's rounded value at all but a few nodes where
    FP32 and FP64 straddle a rounding boundary."""
    import torch
    cfg = inputs.DUCT256
    shape = cfg["shape"]
    announce("256^3 %s, one %s step" % (storage, "check" if check else "plain"))
    sim = _duct_sim(shape, storage, cfg["gamma"])
    assert sim.launch["store"] == "streaming" and sim.launch["load"] == "streaming"
    assert sim.launch["waves"] == {"f32": 5, "f64": 3, "bf16": 6, "f16": 6}[storage]
    tdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16,
           "f16": torch.float16}[storage]
    d0 = torch.from_numpy(inputs.random_deviations(shape, seed=12, amp=1e-3)).to(tdt)
    n0 = 19 if check else 18  # step n0 + 1 is a check step when it is 20
    sim.set_state(d0.cuda(), step=n0)
    sim.step(1)
    out = sim.get_state()
    mid = d0.double().numpy()
    del d0
    nodes = inputs.random_nodes(shape, 4000, seed=12)
    F = inputs.duct_force(shape, cfg["F0"])
    if storage != "f64":
        F = F.astype(np.float32).astype(np.float64)
    s = glbe.rates(cfg["nu"], cfg["gamma"])
    ref = glbe.step_nodes(mid, F, cfg["gamma"], s, cfg["bc"], nodes)
    del mid
    idx = torch.tensor(nodes, device="cuda")
    got_t = out[:, idx[:, 2], idx[:, 1], idx[:, 0]]
    got = got_t.double().cpu().numpy()
    if storage == "f64":
        assert rel(got, ref) < 1e-12
    elif storage == "f32":
        assert rel(got, ref) < STEP_TOL
    else:
        # one unit of the format at the value (nearest even is within half of it),
        # FP16's subnormal spacing, and the FP32 collision's own error, bounded
        # by the FP32 bar at the largest value (it decides values near zero)
        ulp = 2.0 ** -8 if storage == "bf16" else 2.0 ** -11
        tiny = 6e-8 if storage == "f16" else 0.0
        assert np.all(np.abs(got - ref) <= ulp * np.abs(ref) + tiny + STEP_TOL * np.abs(ref).max())
        ref_r = torch.tensor(ref).to(tdt).double().numpy()
        assert np.mean(got != ref_r) < 0.01
    if check:
        # the first check after set_state: u(t - 10) counts as zero, so R = 1
        h = sim.history(4)
        assert int(h[-1, 0]) == 20 and abs(h[-1, 1] - 1.0) < 1e-12 and h[-1, 6] == 0
    sim.close()
    del sim, out, got_t
    torch.cuda.empty_cache()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_duct256_uniform_force_keeps_the_rest_plane(storage):
    """The 256^3 duct with a uniform force (no field to keep in the
    last-level cache, so the rest population's planes keep cacheable loads
    and stores while the others stream): one step from a seeded state
    against the oracle at 4000 sampled nodes (FP32 2e-6; BF16 one rounding
    plus the FP32 bar), and three steps bit for bit equal to the same steps
    with every load and store cacheable."""
    import torch

    import paper_0809_4730_amd as pkg
    cfg = inputs.DUCT256
    shape = cfg["shape"]
    announce("256^3 %s, uniform force, rest plane cached" % storage)
    F = (1e-6, 2e-7, 0.0)
    s = glbe.rates(cfg["nu"], cfg["gamma"])
    tdt = torch.float32 if storage == "f32" else torch.bfloat16
    d0 = torch.from_numpy(inputs.random_deviations(shape, seed=13, amp=1e-3)).to(tdt)
    outs = []
    for launch in (None, dict(load="cached", store="cached")):
        sim = pkg.Simulation(shape, cfg["bc"], cfg["gamma"], s, storage=storage, force=F,
                             launch=launch)
        if launch is None:
            assert sim.launch["load"] == "streaming" and sim.launch["store"] == "streaming"
        sim.set_state(d0.cuda())
        sim.step(1)
        outs.append(sim.get_state())
        sim.step(2)
        outs.append(sim.get_state())
        sim.close()
        del sim
    assert torch.equal(outs[0], outs[2]) and torch.equal(outs[1], outs[3])
    nodes = inputs.random_nodes(shape, 4000, seed=13)
    idx = torch.tensor(nodes, device="cuda")
    got = outs[0][:, idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()
    del outs
    torch.cuda.empty_cache()
    F32 = np.array(F, dtype=np.float32).astype(np.float64)
    ref = glbe.step_nodes(d0.double().numpy(), inputs.uniform_force(shape, F32), cfg["gamma"], s,
                          cfg["bc"], nodes)
    if storage == "f32":
        assert rel(got, ref) < STEP_TOL
    else:
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + STEP_TOL * np.abs(ref).max())


@pytest.mark.parametrize("force", ["uniform", "field"])
def test_coupled256_bench_kernel_one_step(force):
    """The coupled step at 256^3 in the benchmark's launch shape (FP32, walls
    normal to y and B0: the coupled workload's Hartmann setting Ha = 10,
    Pm = 0.01, gamma = gamma_m = 0.1; create-time XCD chunk, streaming loads
    and stores, row-aligned waves, 3 waves per SIMD), with the workload's
    uniform force and with a force field (201 MB, which keeps cacheable loads
    while the populations stream): one step from a seeded random state
    against the oracle's coupled step from the same state at 4000 sampled
    nodes, corners included.  Bars as for the FP32 coupled step on the
    Hartmann lattice: f 2e-6, g 1e-6 relative, g's deviation from W B0 (what
    FP32 stores) 1e-5."""
    import torch

    import paper_0809_4730_amd as pkg
    from oracle import mhd
    from tests.gpu_util import perms
    announce("256^3 coupled step, bench launch shape, %s force" % force)
    cfg = inputs.HARTMANN
    shape = (256, 256, 256)
    nx, ny, nz = shape
    B0, chi = inputs.hartmann_parameters(10.0, 0.01, cfg["shape"][1], cfg["nu"], cfg["eta"])
    B0v = np.array([0.0, B0, 0.0])
    gamma = 0.1
    s = glbe.rates(cfg["nu"], gamma)
    if force == "uniform":
        F = np.array(cfg["F"], dtype=np.float32).astype(np.float64)
        F_lib = tuple(F)
    else:
        F32 = inputs.duct_force(shape, 1e-5, dtype=np.float32)
        F_lib = torch.from_numpy(F32).cuda()
        F = F32.astype(np.float64)
        del F32
    sim = pkg.Simulation(shape, cfg["bc"], gamma, s, storage="f32", force=F_lib,
                         mhd=dict(gamma_m=0.1, chi=chi, eta=cfg["eta"], B0=tuple(B0v)))
    del F_lib
    assert sim.launch["waves"] == 3
    assert sim.launch["store"] == "streaming" and sim.launch["load"] == "streaming"
    p19, p7 = perms()
    f0 = inputs.random_deviations(shape, seed=31, amp=1e-3, dtype=np.float32)
    dev = inputs.random_deviations(shape, seed=32, amp=1e-4, q=21,
                                   dtype=np.float32).reshape(3, 7, nz, ny, nx)
    sim.set_state(torch.from_numpy(np.ascontiguousarray(f0[p19])).cuda(),
                  torch.from_numpy(np.ascontiguousarray(dev[:, p7])).cuda())
    sim.step(1)
    fg, gg = sim.get_state()
    nodes = inputs.random_nodes(shape, 4000, seed=31)
    idx = torch.tensor(nodes, device="cuda")
    got_f = fg[:, idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()
    got_g = gg[:, :, idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()
    sim.close()
    del sim, fg, gg
    torch.cuda.empty_cache()
    g0 = mhd.initial_g(shape, B0v)
    g0 += dev
    del dev
    p = dict(gamma=gamma, s=s, gamma_m=0.1, chi=chi, eta=cfg["eta"], B_wall=B0v)
    ref_f, ref_g = mhd.step_nodes(f0, g0, F, p, cfg["bc"], nodes)
    del g0, f0
    rest = mhd.initial_g((len(nodes), 1, 1), B0v)[:, :, 0, 0, :]
    assert rel(got_f, ref_f[p19]) < STEP_TOL
    assert rel(got_g + rest[:, p7], ref_g[:, p7]) < 1e-6
    assert rel(got_g, (ref_g - rest)[:, p7]) < 1e-5


@pytest.mark.parametrize("storage", ["f32", "f64", "bf16", "f32_mhd"])
def test_load_store_forms_bitwise_on_a_row_aligned_lattice(storage):
    """Cacheable and streaming stores, streaming loads with them, and caps on
    the waves per SIMD, on a row-aligned lattice (64 x 6 x 10: the row-aligned
    variant the benchmark's lattices take), residual checks on, flow and
    coupled steps: bit for bit."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("load/store forms, row-aligned 64x6x10 %s" % storage)
    shape, bc = (64, 6, 10), (PER, WALL, WALL)
    dt = torch.float64 if storage == "f64" else torch.float32
    F = torch.tensor(inputs.random_force(shape, seed=13, amp=1e-5), dtype=dt, device="cuda")
    kw = dict(mhd=dict(gamma_m=0.3, chi=0.05, eta=0.03, B0=(0.01, 0.02, -0.01))) \
        if storage.endswith("_mhd") else {}
    out = []
    for store, load, waves in (("cached", "cached", 8), ("streaming", "cached", 8),
                               ("streaming", "streaming", 8), ("streaming", "streaming", 5),
                               ("cached", "cached", 3)):
        sim = pkg.Simulation(shape, bc, 0.2, glbe.rates(0.05, 0.2), storage=storage.split("_")[0],
                             force=F, launch=dict(store=store, load=load, waves=waves), **kw)
        assert sim.launch["store"] == store and sim.launch["load"] == load
        assert sim.launch["waves"] == waves
        sim.step(33)
        st = sim.get_state()
        out.append((st if torch.is_tensor(st) else torch.cat([st[0].reshape(-1), st[1].reshape(-1)]),
                    sim.history(8)))
    for a, b in zip(out[1:], out[:-1]):
        assert torch.equal(a[0], b[0])
        assert np.array_equal(a[1], b[1])


def test_nonfinite_force_is_detected_and_a_checkpoint_recovers():
    """Failure path of the instability detector: a non-finite force value at
    one node (ordinary IEEE arithmetic; nothing traps) reaches the populations
    and the next residual check counts it, so lbm_residual and
    lbm_run_to_residual report LBM_EUNSTABLE; the state stays readable.  A
    checkpoint taken before, loaded into a context with a larger gamma, marches
    to the tolerance."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("non-finite force -> EUNSTABLE, recovery from a checkpoint")
    shape, bc = (16, 12, 10), (PER, WALL, WALL)
    F = torch.tensor(inputs.duct_force(shape, 1e-5), dtype=torch.float32, device="cuda")
    sim = pkg.Simulation(shape, bc, 0.1, glbe.rates(0.131, 0.1), storage="f32", force=F)
    sim.step(20)
    r, t = sim.residual()
    assert t == 20 and np.isfinite(r)
    ckpt = sim.get_state().clone()
    bad = F.clone()
    bad[0, 5, 6, 7] = float("nan")
    sim.set_force(bad)
    sim.step(10)
    with pytest.raises(pkg.LbmError) as e:
        sim.residual()
    assert e.value.status == -4
    h = sim.history(1)
    assert int(h[0, 0]) == 30 and h[0, 6] >= 1
    state = sim.get_state()
    assert not bool(torch.isfinite(state).all())
    with pytest.raises(pkg.LbmError) as e:
        sim.run_to_residual(1e-8, 100, poll_every=10)
    assert e.value.status == -4
    sim.close()
    rec = pkg.Simulation(shape, bc, 0.5, glbe.rates(0.131, 0.5), storage="f32", force=F)
    rec.set_state(ckpt, step=20)
    steps, r = rec.run_to_residual(1e-6, 40000, poll_every=500)
    assert steps > 20 and r < 1e-6
    assert bool(torch.isfinite(rec.get_state()).all())


@pytest.mark.parametrize("gamma", [0.5, 1.0])
def test_steady_adjoint_from_the_oracle_state_to_1e12(gamma):
    """FP64 steady adjoint on the 2 x 4 x 4 duct from exactly the oracle's
    converged state (loaded with set_state), iterated to a relative change of
    1e-15: equal to the oracle's dense bordered transposed solve at that same
    state to 1e-12."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("steady adjoint from the oracle state, gamma=%g" % gamma)
    shape, bc = (2, 4, 4), (PER, WALL, WALL)
    s = glbe.rates(0.131, gamma)
    nx, ny, nz = shape
    F = np.zeros((3, nz, ny, nx))
    y = np.arange(ny) + 0.5
    F[0] = 1e-5 * (1.0 + 0.3 * np.sin(2 * np.pi * y / ny))[None, :, None]
    fl = glbe.Flow(shape, bc, F, gamma, s)
    assert fl.run_to(1e-14, 100000)
    ref, _ = oadj.steady_gradient_dense(fl.post, fl.F, gamma, s, bc)
    sim = pkg.Simulation(shape, bc, gamma, s, storage="f64",
                         force=torch.tensor(F, dtype=torch.float64, device="cuda"))
    sim.set_state(torch.tensor(fl.post, dtype=torch.float64, device="cuda"), step=fl.t)
    grad, iters, change = sim.adjoint_steady(tol=1e-15, max_iter=400000)
    assert change < 1e-15, change
    err = rel(grad.cpu().numpy(), ref)
    announce("iters %d change %.2e rel %.3e" % (iters, change, err))
    assert err < 1e-12


def test_residual_history_within_the_measured_velocity_bound():
    """FP64 residual history of the 1 x 16 x 16 duct against the oracle's.  With
    a = u_t - u_(t-10) and b = u_t, R = |a|/|b|; the GPU's velocities differ from
    the oracle's by du_t (measured here with lbm_moments), so
        |R_gpu - R| <= (|du_t - du_(t-10)| + R |du_t|) / |b_gpu|
    plus the rounding of the two FP64 reductions (a few units of 1e-16 of R)."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("residual history bound")
    shape, bc, gamma = (1, 16, 16), (PER, WALL, WALL), 0.25
    s = glbe.rates(0.131, gamma)
    F = inputs.duct_force(shape)
    Ft = torch.tensor(F, dtype=torch.float64, device="cuda")
    sim = pkg.Simulation(shape, bc, gamma, s, storage="f64", force=Ft)
    probe = pkg.Simulation(shape, bc, gamma, s, storage="f64", force=Ft)
    post = np.zeros((19,) + F.shape[1:])
    u_or, u_gpu = {0: np.zeros((3,) + F.shape[1:])}, {0: np.zeros((3,) + F.shape[1:])}
    for t in range(1, 201):
        if t % 10 == 0:
            _, u, _ = probe.moments("f64")  # the velocity of collision t
            u_gpu[t] = u.cpu().numpy()
        probe.step(1)
        post, u = glbe.step(post, F, gamma, s, bc)
        if t % 10 == 0:
            u_or[t] = u
    sim.step(200)
    hist = {int(h[0]): h[1] for h in sim.history()}
    assert sorted(hist) == list(range(10, 201, 10))
    worst = 0.0
    for t in range(20, 201, 10):
        a = u_or[t] - u_or[t - 10]
        R = np.linalg.norm(a) / np.linalg.norm(u_or[t])
        d_t, d_p = u_gpu[t] - u_or[t], u_gpu[t - 10] - u_or[t - 10]
        b = np.linalg.norm(u_gpu[t])
        bound = (np.linalg.norm(d_t - d_p) + R * np.linalg.norm(d_t)) / b + 8e-16 * R + 1e-300
        worst = max(worst, abs(hist[t] - R) / bound)
        assert abs(hist[t] - R) <= bound, (t, hist[t], R, bound)
    announce("largest |dR| / bound: %.3f" % worst)


def test_binding_on_a_side_stream_matches_the_current_stream():
    """A Simulation on its own stream, fed and read from torch's current
    stream (set_state from a tensor computed just before, set_force, moments,
    get_state, adjoint): every result equals the same calls on the current
    stream."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("side stream")
    shape, bc = (16, 10, 12), (PER, WALL, WALL)
    s = glbe.rates(0.1, 0.4)

    def run(stream):
        F = torch.tensor(inputs.duct_force(shape, 1e-5), dtype=torch.float64, device="cuda")
        sim = pkg.Simulation(shape, bc, 0.4, s, storage="f64", force=F * 1.0, stream=stream)
        d0 = torch.tensor(inputs.random_deviations(shape, seed=14, amp=1e-4), device="cuda")
        sim.set_state(d0 * 0.5 + d0 * 0.5)  # a fresh temporary from the current stream
        sim.step(25)
        sim.set_force(F * 2.0)
        sim.step(25)
        rho, u, _ = sim.moments("f64")
        st = sim.get_state()
        grad = sim.adjoint_unrolled(20, 5)
        return [rho.clone(), u.clone(), st.clone(), grad.clone(), sim.history(8)]

    ref = run(None)
    side = torch.cuda.Stream()
    got = run(side)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        if torch.is_tensor(a):
            assert torch.equal(a, b)
        else:
            assert np.array_equal(a, b)


def test_bandwidth_probe_copies_exactly():
    """The calibration copies move the data they claim: the 16-byte copy
    reproduces 22 planes, the plane-pattern copies the first 19 of 22 planes
    and all 40, on a ragged node count."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("bandwidth probe copies")
    nodes = 3 * 256 + 40
    src = torch.arange(40 * nodes, dtype=torch.float32, device="cuda") * 0.5 - 7.0
    for pattern, planes, waves in ((0, 22, 8), (1, 19, 8), (2, 40, 8), (1, 19, 5), (0, 22, 3)):
        dst = torch.full_like(src, -1.0)
        nbytes = pkg.bandwidth_probe(pattern, src, dst, nodes, waves=waves)
        torch.cuda.synchronize()
        assert torch.equal(dst[:planes * nodes], src[:planes * nodes])
        assert bool((dst[planes * nodes:] == -1.0).all())
        assert nbytes == {0: 2 * 88 * nodes, 1: 164 * nodes, 2: 320 * nodes}[pattern]


def _pulled(planes, vel, shape, walls):
    """Expected gather of one set of direction planes (q, nz, ny, nx): each
    direction from its upstream node with periodic wrap, or from the opposite
    direction at the node itself where the link crosses a wall."""
    nx, ny, nz = shape
    q = len(vel)
    opp = [next(b for b in range(q) if all(vel[b] == -vel[a])) for a in range(q)]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.empty_like(planes)
    for a in range(q):
        ex, ey, ez = vel[a]
        sx, sy, sz = x - ex, y - ey, z - ez
        bounce = np.zeros(x.shape, dtype=bool)
        for w, c, n in ((walls[0], sx, nx), (walls[1], sy, ny), (walls[2], sz, nz)):
            if w:
                bounce |= (c < 0) | (c >= n)
        shifted = planes[a][sz % nz, sy % ny, sx % nx]
        out[a] = np.where(bounce, planes[opp[a]], shifted)
    return out


@pytest.mark.parametrize("shape,walls", [((64, 6, 5), (False, True, True)),
                                         ((128, 3, 4), (True, True, False)),
                                         ((64, 1, 7), (False, False, True))])
def test_bandwidth_probe_step_patterns_gather_as_the_steps(shape, walls):
    """The exact-pattern copies read every population where the step reads it
    (Sec. 2 eq. streaming, the D3Q7 lattice of Sec. 4): compared value by value
    with a gather computed here from the lattice velocity tables alone."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("bandwidth probe step patterns %s walls %s" % (shape, walls))
    nx, ny, nz = shape
    N = nx * ny * nz
    v19 = pkg.lattice_velocities(19)
    v7 = pkg.lattice_velocities(7)
    host = (np.arange(40 * N, dtype=np.float32) * 0.25 + 1.0).reshape(40, nz, ny, nx)
    src = torch.tensor(host.reshape(-1), device="cuda")
    want_f = _pulled(host[:19], v19, shape, walls)
    want_g = np.concatenate([_pulled(host[19 + 7 * j:26 + 7 * j], v7, shape, walls)
                             for j in range(3)])
    for pattern in (3, 4):
        for waves in (8, 5):
            dst = torch.full_like(src, -1.0)
            nbytes = pkg.bandwidth_probe(pattern, src, dst, shape, walls=walls, waves=waves)
            torch.cuda.synchronize()
            got = dst.cpu().numpy().reshape(40, nz, ny, nx)
            assert np.array_equal(got[:19], want_f)
            if pattern == 3:
                assert (got[19:] == -1.0).all()
                assert nbytes == 164 * N
            else:
                assert np.array_equal(got[19:], want_g)
                assert nbytes == 320 * N


def test_history_records_of_a_large_lattice_equal_direct_sums():
    """Above 4096 workgroups the checks' partial sums are reduced in two passes.
    On a 1.15 M-node FP64 lattice, three checks reduced in one flush equal the
    FP64 sums taken directly from the velocities of the collisions (moments of
    the state one step before each check) to 1e-13 relative: du2, u2, the mass
    drift and the flow rate."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("history of a 128x100x90 lattice (two-pass reduction)")
    shape, bc, gamma = (128, 100, 90), (PER, WALL, WALL), 0.5
    Ft = torch.tensor(inputs.duct_force(shape, 1e-5), dtype=torch.float64, device="cuda")
    s = glbe.rates(0.131, gamma)
    sim = pkg.Simulation(shape, bc, gamma, s, storage="f64", force=Ft)
    d0 = torch.tensor(inputs.random_deviations(shape, seed=15, amp=1e-4), device="cuda")
    sim.set_state(d0)
    want = {}
    u_prev = None
    for t in range(1, 31):
        if t % 10 == 0:
            rho, u, _ = sim.moments("f64")
            jx = u[0] * rho
            du = u if u_prev is None else u - u_prev
            want[t] = (float((du * du).sum()), float((u * u).sum()), float((rho - 1.0).sum()),
                       float(jx.sum()) / shape[0])
            u_prev = u.clone()
        sim.step(1)
    h = sim.history(3)
    assert [int(r[0]) for r in h] == [10, 20, 30]
    for r in h:
        du2, u2, mass, flow = want[int(r[0])]
        assert abs(r[2] - du2) <= 1e-13 * du2
        assert abs(r[3] - u2) <= 1e-13 * u2
        assert abs(r[4] - mass) <= 1e-13 * float((rho - 1.0).abs().sum())
        assert abs(r[5] - flow) <= 1e-13 * float((u[0] * rho).abs().sum()) / shape[0]
        assert r[6] == 0

