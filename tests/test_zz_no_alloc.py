"""lbm_reductions_noalloc (the entry point for callers that cannot allocate
device memory) against lbm_reductions on the same state: the same fields and
finalize kernels over the same node ranges, so the FP64 mass drift and flow
rate agree bit for bit.  Calls follow each other on one GPU with a smaller
lattice each time (the shared scratch keeps the last call's contents), and a
lattice beyond the scratch's capacity is rejected before any launch."""
import ctypes

import numpy as np
import pytest

from oracle import d2q9, glbe
from paper_0809_4730_amd import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu
PER, WALL = "periodic", "wall"


def _case(kind):
    import torch

    import paper_0809_4730_amd as pkg
    if kind == "d3q19_f64_field":
        shape, bc = (40, 30, 36), (PER, WALL, WALL)
        F = torch.tensor(inputs.random_force(shape, seed=21, amp=1e-4), device="cuda")
        sim = pkg.Simulation(shape, bc, 0.3, glbe.rates(0.1, 0.3), storage="f64", force=F)
        sim.set_state(torch.tensor(inputs.random_deviations(shape, seed=21, amp=1e-3),
                                   device="cuda"))
        sim.step(7)
    elif kind == "d3q19_f32_uniform":
        shape, bc = (16, 12, 10), (WALL, PER, WALL)
        sim = pkg.Simulation(shape, bc, 0.5, glbe.rates(0.1, 0.5), storage="f32",
                             force=(2e-5, -1e-5, 3e-6))
        d0 = inputs.random_deviations(shape, seed=22, amp=1e-3).astype(np.float32)
        sim.set_state(torch.from_numpy(d0).cuda())
        sim.step(9)
    elif kind == "d2q9_bf16_field":
        shape, bc = (24, 10, 1), (PER, WALL, PER)
        F = torch.tensor(inputs.random_force(shape, seed=23, amp=1e-4), dtype=torch.float32,
                         device="cuda")
        F[2] = 0.0
        sim = pkg.Simulation(shape, bc, 0.2, d2q9.rates(0.05, 0.2), storage="bf16", force=F,
                             lattice="d2q9")
        sim.step(13)
    else:
        raise ValueError(kind)
    return sim


@pytest.mark.parametrize("order", [("d3q19_f64_field", "d3q19_f32_uniform", "d2q9_bf16_field")])
def test_noalloc_reductions_equal_the_context_reductions(order):
    import torch
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    for kind in order:  # each lattice smaller than the one before
        announce("no-alloc reductions: %s" % kind)
        sim = _case(kind)
        want = sim.reductions()
        state = sim.get_state()
        for _ in range(2):  # twice on the same state: nothing carried over
            sim.reductions_noalloc(state, out)
            torch.cuda.synchronize()
            got = tuple(out.cpu().numpy())
            assert got == want, (kind, got, want)
        sim.close()


def test_noalloc_rejects_a_lattice_beyond_its_scratch():
    import torch

    import paper_0809_4730_amd as pkg
    lib = pkg.load_library()
    g = pkg._Grid()
    for a, (n, b) in enumerate(zip((512, 256, 256), (0, 1, 1))):
        g.n[a], g.bc[a] = n, b
    p = pkg._Params()
    p.storage, p.gamma, p.rho0, p.check_every, p.history_len = pkg.F32, 1.0, 1.0, 10, 16
    for k, v in enumerate(glbe.rates(0.131, 1.0)):
        p.s[k] = v
    state = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    st = lib.lbm_reductions_noalloc(ctypes.byref(g), ctypes.byref(p), state.data_ptr(), None,
                                    None, out.data_ptr())
    assert st == -2
    assert b"26841856" in lib.lbm_last_error(None)
    assert float(out.abs().sum()) == 0.0
