"""How step kernels are launched, checked against plain eager steps bit for bit.

* Step launches captured into a HIP graph (torch.cuda.graph on the library's
  stream) and replayed: each replay advances the state exactly as the same
  number of eager steps does.  Residual checks are off so that the captured
  work is the step kernels alone; every replay is followed by eager work and a
  device synchronisation before it is checked.
* Timed steps (HIP events attached to each step kernel's launch) compute what
  plain steps compute: states and residual histories."""
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


@pytest.mark.parametrize("case", ["flow", "flow_short_ring", "mhd", "d2q9"])
def test_timed_steps_compute_what_plain_steps_compute(case):
    """lbm_step_times (an event on each step kernel's launch) over 700 steps,
    more than one batch of its event pool, residual checks on: the state and
    the residual history equal those of 700 plain steps bit for bit, every
    step's duration is positive and finite, and the durations (each from the
    previous step kernel's end) sum to no more than the call's wall time;
    lbm_step_timed likewise.  With a ring of 6 history records the reduction
    of pending checks runs inside the timed calls every 60 steps."""
    import torch

    import paper_0809_4730_amd as pkg
    announce("timed steps, %s" % case)
    gamma = 0.3
    if case == "d2q9":
        shape, bc = (64, 37, 1), (PER, WALL, PER)
        kw = dict(lattice="d2q9")
        s = pkg.default_rates_d2q9(0.05, gamma)
        F = (1e-5, -2e-6, 0.0)
    else:
        shape, bc = (64, 6, 10), (PER, WALL, WALL)
        kw = dict(mhd=dict(gamma_m=0.4, chi=0.05, eta=0.03, B0=(0.01, 0.02, -0.01))) \
            if case == "mhd" else {}
        if case == "flow_short_ring":
            kw = dict(history_len=6)
        s = glbe.rates(0.05, gamma)
        F = (1e-5, 0.0, 0.0)
    sims = [pkg.Simulation(shape, bc, gamma, s, storage="f32", force=F, **kw) for _ in range(3)]
    t, wall_ms = sims[0].step_times(700)
    assert len(t) == 700 and np.all(np.isfinite(t)) and np.all(t > 0) and wall_ms > 0
    assert t.sum() / 1000.0 <= wall_ms * (1.0 + 1e-6)
    mean_us, wall2 = sims[1].step_timed(700)
    assert mean_us > 0 and wall2 > 0 and 700 * mean_us / 1000.0 <= wall2 * (1.0 + 1e-6)
    sims[2].step(700)
    torch.cuda.synchronize()
    states = [sim.get_state() for sim in sims]
    hists = [sim.history(100) for sim in sims]
    assert len(hists[2]) == (6 if case == "flow_short_ring" else 70)
    if case == "flow":
        # reads of up to 64 records go through the context's pinned staging
        # buffer, longer ones straight to pageable memory: the same records
        assert np.array_equal(sims[2].history(64), hists[2][-64:])
        assert np.array_equal(sims[2].history(1), hists[2][-1:])
    for st, h in zip(states[:2], hists[:2]):
        if case == "mhd":
            assert torch.equal(st[0], states[2][0]) and torch.equal(st[1], states[2][1])
        else:
            assert torch.equal(st, states[2])
        assert np.array_equal(h, hists[2])
    for sim in sims:
        sim.close()
