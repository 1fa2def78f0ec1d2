"""Step launches captured into a HIP graph (torch.cuda.graph on the library's
stream) and replayed: each replay advances the state exactly as the same
number of eager steps does, bit for bit.  Residual checks are off so that the
captured work is the step kernels alone; every replay is followed by eager work
and a device synchronisation before it is checked."""
import numpy as np
import pytest

from oracle import glbe
from paper_0809_4730_amd import inputs
from tests.gpu_util import announce, to_gpu_f

pytestmark = pytest.mark.gpu
PER, WALL = "periodic", "wall"
NO_CHECK = 1 << 30


@pytest.mark.parametrize("mhd", [False, True])
def test_replayed_step_graph_equals_eager_steps(mhd):
    import torch

    import paper_0809_4730_amd as pkg
    announce("graph replay of 10 steps, mhd=%s" % mhd)
    shape, bc, gamma = (64, 6, 10), (PER, WALL, WALL), 0.3
    s = glbe.rates(0.05, gamma)
    kw = dict(mhd=dict(gamma_m=0.4, chi=0.05, eta=0.03, B0=(0.01, 0.02, -0.01))) if mhd else {}
    d0 = to_gpu_f(inputs.random_deviations(shape, seed=51, amp=1e-3), torch.float32)
    side = torch.cuda.Stream()
    cap = pkg.Simulation(shape, bc, gamma, s, storage="f32", force=(1e-5, 0.0, 0.0),
                         check_every=NO_CHECK, stream=side, **kw)
    ref = pkg.Simulation(shape, bc, gamma, s, storage="f32", force=(1e-5, 0.0, 0.0),
                         check_every=NO_CHECK, **kw)
    if mhd:
        g0 = torch.zeros((3, 7) + (shape[2], shape[1], shape[0]), dtype=torch.float32,
                         device="cuda")
        cap.set_state(d0, g0)
        ref.set_state(d0, g0)
    else:
        cap.set_state(d0)
        ref.set_state(d0)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        cap.step(10)
    for _ in range(3):
        graph.replay()
        torch.cuda.synchronize()
        ref.step(10)
        torch.cuda.synchronize()
        a, b = cap.get_state(), ref.get_state()
        if mhd:
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        else:
            assert torch.equal(a, b)
        assert bool(torch.isfinite(a[0] if mhd else a).all())
    cap.close()
    ref.close()
