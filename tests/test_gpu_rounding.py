"""GPU parity of BF16 storage with stochastic rounding (rounding="stochastic").

The step computes in FP32 like the nearest-even form; only the store differs:
the stored bits are (FP32 bits + r) >> 16 with r the counter-based random bits
of oracle/rounding.py.  The oracle's FP64 step gives the value before rounding
to within FP32 error, so wherever that error cannot move the sum across a
multiple of 2^16 (almost every population) the stored BF16 bits are fixed by
the oracle alone and must match exactly; everywhere the result must be one of
the two BF16 neighbours of the exact value.
"""
import numpy as np
import pytest

from oracle import glbe, rounding
from paper_0809_4730_amd import inputs
from tests.gpu_util import announce, from_gpu_f, perms, rel, to_gpu_f

pytestmark = pytest.mark.gpu

PER, WALL = "periodic", "wall"


def _sim(shape, bc, gamma, s, storage, F, **kw):
    import torch

    import paper_0809_4730_amd as pkg
    force = torch.tensor(F, dtype=torch.float32, device="cuda")
    return pkg.Simulation(shape, bc, gamma, s, storage=storage, force=force, **kw)


def _bf16_exact(d):
    import torch
    return torch.tensor(d).to(torch.bfloat16).double().numpy()


def _check_bits(out, ref, r, eps):
    """out: stored BF16 values, ref: the oracle's FP64 values before rounding,
    r: the random bits, all (19, n) in the library's direction order; eps: a
    bound on |FP32 result - ref|.  Returns the decided fraction."""
    # decided elements: a shift of the FP32 bits by up to the margin cannot
    # change (bits + r) >> 16
    ref32 = ref.astype(np.float32)
    ulp32 = np.spacing(np.abs(ref32)).astype(np.float64)
    margin = np.ceil(2 * eps / ulp32) + 2        # 2x: the FP32 result may sit one binade lower
    low = (ref32.view(np.uint32).astype(np.int64) + r) & 0xFFFF
    decided = (low >= margin) & (low < 65536 - margin) & (np.abs(ref) > 2 * eps)
    want = rounding.stochastic_bf16(ref32, r)
    frac = decided.mean()
    mism = np.count_nonzero(out[decided] != want[decided])
    announce("decided %.4f of %d populations, mismatches %d" % (frac, out.size, mism))
    assert mism == 0
    # every element lies between the BF16 neighbours of the exact value
    # (truncation and rounding away from zero are both monotone in the value)
    ends = [rounding.stochastic_bf16((ref + sgn * eps).astype(np.float32), np.full_like(r, rr))
            for sgn in (-1, 1) for rr in (0, 0xFFFF)]
    lo, hi = np.minimum.reduce(ends), np.maximum.reduce(ends)
    assert np.all((out >= lo) & (out <= hi))
    return frac


@pytest.mark.parametrize("shape,bc,start,moving", [
    ((33, 6, 10), (PER, WALL, WALL), 0, False),        # ragged
    ((64, 5, 7), (WALL, WALL, PER), 1000, False),      # row-aligned lattice, later step number
    ((9, 8, 7), (WALL, WALL, WALL), 5, True),          # every face moving
])
def test_stochastic_step_bits_match_oracle(shape, bc, start, moving):
    import torch
    announce("bf16 stochastic single step %s start=%d moving=%s" % (shape, start, moving))
    seed, gamma = 0xC0FFEE, 0.5
    d0 = _bf16_exact(inputs.random_deviations(shape, seed=21, amp=1e-3))
    F = inputs.random_force(shape, seed=21, amp=1e-4).astype(np.float32).astype(np.float64)
    s = glbe.rates(0.05, gamma)
    wu = 0.01 * np.random.default_rng(21).uniform(-1, 1, (6, 3)) if moving else None
    sim = _sim(shape, bc, gamma, s, "bf16", F, rounding="stochastic", seed=seed, wall_u=wu)
    sim.set_state(to_gpu_f(d0, torch.bfloat16), step=start)
    sim.step(1)
    p19, _ = perms()
    out = from_gpu_f(sim.get_state())[p19].reshape(19, -1)      # library direction order
    ref, _ = glbe.step(d0, F, gamma, s, bc, wall_u=wu)
    ref = ref[p19].reshape(19, -1)
    r = rounding.random_bits(ref.shape[1], 19, start + 1, seed).astype(np.int64)
    # FP32 error of the collision, bounded on the FP32-storage form of this step
    sim32 = _sim(shape, bc, gamma, s, "f32", F, wall_u=wu)
    sim32.set_state(to_gpu_f(d0, torch.float32))
    sim32.step(1)
    err32 = np.abs(from_gpu_f(sim32.get_state())[p19].reshape(19, -1) - ref).max()
    eps = 1e-6 * np.abs(ref).max()
    announce("FP32 step error %.3e, bound used %.3e" % (err32, eps))
    assert err32 <= eps / 4, (err32, eps)
    assert _check_bits(out, ref, r, eps) > 0.9


@pytest.mark.parametrize("shape,bc,start", [
    ((33, 17), (PER, WALL), 0),
    ((70, 12), (WALL, WALL), 500),
])
def test_stochastic_d2q9_step_bits_match_oracle(shape, bc, start):
    """The D2Q9 step with BF16 stochastic rounding (directions 2k, 2k+1 for
    k = 0..4 in the library's D2Q9 order) against the 2D oracle."""
    import torch

    import paper_0809_4730_amd as pkg
    from oracle import d2q9
    announce("bf16 stochastic D2Q9 step %s start=%d" % (shape, start))
    seed, gamma = 31337, 0.2
    nx, ny = shape
    e_lib = pkg.lattice_velocities(9)[:, :2]
    pos = {tuple(v): a for a, v in enumerate(d2q9.E9)}
    p9 = np.array([pos[tuple(v)] for v in e_lib])           # library direction i = oracle p9[i]
    f0 = inputs.random_deviations((nx, ny, 1), seed=43, amp=1e-3, q=9)[:, 0]
    f0 = _bf16_exact(f0)
    F = (2e-5, -1e-5)
    Ff = np.broadcast_to(np.array(F).reshape(2, 1, 1), (2, ny, nx))
    s = d2q9.rates(0.04, gamma)

    def run(storage, dt, **kw):
        sim = pkg.Simulation((nx, ny, 1), (bc[0], bc[1], PER), gamma, s, storage=storage, force=F,
                             lattice="d2q9", **kw)
        sim.set_state(torch.tensor(np.ascontiguousarray(f0[p9][:, None])).to(dt).cuda(),
                      step=start)
        sim.step(1)
        return sim.get_state().double().cpu().numpy()[:, 0].reshape(9, -1)
    out = run("bf16", torch.bfloat16, rounding="stochastic", seed=seed)
    out32 = run("f32", torch.float32)
    ref = d2q9.step(f0, Ff, gamma, s, bc)[0][p9].reshape(9, -1)
    err32 = np.abs(out32 - ref).max()
    eps = 1e-6 * np.abs(ref).max()
    announce("FP32 step error %.3e, bound used %.3e" % (err32, eps))
    assert err32 <= eps / 4, (err32, eps)
    r = rounding.random_bits(nx * ny, 9, start + 1, seed).astype(np.int64)
    assert _check_bits(out, ref, r, eps) > 0.9


def test_stochastic_full_size_sampled_nodes():
    """256^3 duct in BF16 with stochastic rounding, in the launch shape such a
    lattice gets (streaming stores, create-time workgroup mapping, row-aligned
    addressing): one step from a seeded state, bits at 4000 sampled nodes."""
    import torch
    cfg = inputs.DUCT256
    shape, seed = cfg["shape"], 2024
    announce("256^3 bf16 stochastic sampled parity")
    d0 = torch.tensor(inputs.random_deviations(shape, seed=9, amp=1e-3, dtype=np.float32))
    d0 = d0.to(torch.bfloat16)
    F = inputs.duct_force(shape, cfg["F0"], dtype=np.float32)
    s = glbe.rates(cfg["nu"], cfg["gamma"])
    sim = _sim(shape, cfg["bc"], cfg["gamma"], s, "bf16", F.astype(np.float64),
               rounding="stochastic", seed=seed)
    p19, _ = perms()
    lib = torch.empty_like(d0)
    lib[:] = d0[torch.as_tensor(p19)]                 # library order holds oracle direction p19[i]
    sim.set_state(lib.cuda(), step=41)
    sim.step(1)
    out = sim.get_state()
    nodes = inputs.random_nodes(shape, 4000, seed=9)
    idx = torch.tensor(nodes, device="cuda")
    got = out[:, idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()     # library order
    del sim, out
    torch.cuda.empty_cache()
    ref = glbe.step_nodes(d0.double().numpy(), F.astype(np.float64), cfg["gamma"], s, cfg["bc"],
                          nodes)[p19]
    nx, ny, _ = shape
    lin = nodes[:, 0] + nx * (nodes[:, 1] + ny * nodes[:, 2])
    r = rounding.random_bits_at(lin, 19, 42, seed).astype(np.int64)
    assert _check_bits(got, ref, r, 1e-6 * np.abs(ref).max()) > 0.9


def test_stochastic_rounding_is_deterministic_per_seed_and_step():
    import torch
    announce("bf16 stochastic determinism")
    shape, bc, gamma = (16, 12, 10), (PER, WALL, WALL), 0.5
    d0 = _bf16_exact(inputs.random_deviations(shape, seed=22, amp=1e-3))
    F = inputs.random_force(shape, seed=22, amp=1e-4).astype(np.float32).astype(np.float64)
    s = glbe.rates(0.05, gamma)
    states = {}
    for key, seed, start in (("a", 5, 0), ("b", 5, 0), ("seed", 6, 0), ("step", 5, 1)):
        sim = _sim(shape, bc, gamma, s, "bf16", F, rounding="stochastic", seed=seed)
        sim.set_state(to_gpu_f(d0, torch.bfloat16), step=start)
        sim.step(20)
        states[key] = sim.get_state().view(torch.int16).cpu().numpy()
    assert np.array_equal(states["a"], states["b"])
    for k in ("seed", "step"):
        assert np.mean(states[k] != states["a"]) > 0.05, k


def test_stochastic_rounding_tracks_fp64_where_nearest_stalls():
    """The 64^3 duct marched from rest at gamma = 1 to the FP64 steady state
    (residual 1e-8, about 9000 steps): the per-step force increment of a
    population (~w 3 F0) is below half the BF16 spacing of the larger stored
    deviations, so nearest-even stores drop it and the flow stalls short of the
    FP64 state; stochastic rounding keeps every increment in expectation."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("bf16 stochastic vs nearest at the 64^3 duct steady state")
    cfg = inputs.DUCT64
    shape, gamma = (64, 64, 64), 1.0
    F = torch.tensor(inputs.duct_force(shape, cfg["F0"]), dtype=torch.float64, device="cuda")
    s = pkg.default_rates(cfg["nu"], gamma)
    ref = pkg.Simulation(shape, cfg["bc"], gamma, s, storage="f64", force=F)
    ref.run_to_residual(1e-8, 200000, poll_every=1000)
    n = ref.t
    u64 = ref.moments("f64")[1].cpu().numpy()
    errs = {}
    for key, kw in (("nearest", {}), ("stochastic", dict(rounding="stochastic", seed=1))):
        sim = pkg.Simulation(shape, cfg["bc"], gamma, s, storage="bf16", force=F.float(), **kw)
        sim.step(n)
        errs[key] = rel(sim.moments("f64")[1].cpu().numpy(), u64)
        announce("bf16 %s: u rel L2 vs FP64 = %.3e (step %d)" % (key, errs[key], n))
    assert errs["stochastic"] < 0.01
    assert errs["stochastic"] < errs["nearest"] / 3
