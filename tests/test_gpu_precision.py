"""Precision form: FP32 / BF16 / FP16 deviation storage with FP32 collision,
compared with the FP64 path (itself matched to the oracle in test_gpu_glbe).

The velocity error against FP64 is measured on the 64^3 duct at the FP64
steady state (residual 1e-8), and on the 256^3 duct after a fixed transient;
bounds follow from one rounding of the stored deviation per step (BF16 2^-9,
FP16 2^-12 relative; FP16 deviations below 2^-14 become subnormal).
"""
import numpy as np
import pytest

from paper_0809_4730_amd import inputs
from tests.gpu_util import announce, rel

pytestmark = pytest.mark.gpu

BOUNDS_STEADY = {"f32": 1e-5, "bf16": 0.05, "f16": 0.01}


def _sim(shape, storage, gamma, **kw):
    import torch

    import paper_0809_4730_amd as pkg
    cfg = inputs.DUCT64
    dt = torch.float64 if storage == "f64" else torch.float32
    F = torch.tensor(inputs.duct_force(shape, cfg["F0"]), dtype=dt, device="cuda")
    return pkg.Simulation(shape, cfg["bc"], gamma, pkg.default_rates(cfg["nu"], gamma),
                          storage=storage, force=F, **kw)


def test_precision_forms_at_steady_state_duct64():
    shape, gamma = (64, 64, 64), 0.1
    ref = _sim(shape, "f64", gamma)
    steps, r = ref.run_to_residual(1e-8, 200000, poll_every=1000)
    assert steps > 0
    n = ref.t
    _, u64, _ = ref.moments("f64")
    u64 = u64.cpu().numpy()
    out = {}
    for st in ("f32", "bf16", "f16"):
        sim = _sim(shape, st, gamma)
        sim.step(n)
        _, u, _ = sim.moments("f64")
        err = rel(u.cpu().numpy(), u64)
        mass, _ = sim.reductions()
        out[st] = (err, mass)
        announce("storage %s: u rel L2 vs FP64 = %.3e, mass drift %.3e (step %d)" % (st, err, mass, n))
    for st, (err, _) in out.items():
        assert err < BOUNDS_STEADY[st], (st, err)
    assert out["f32"][0] < out["f16"][0] < out["bf16"][0]


def test_precision_forms_transient_duct256():
    """256^3 duct: u after 300 steps from rest, per storage type, vs FP64."""
    import torch
    shape, gamma, n = (256, 256, 256), 1.0, 300
    us = {}
    for st in ("f64", "f32", "bf16", "f16"):
        sim = _sim(shape, st, gamma)
        sim.step(n)
        _, u, _ = sim.moments("f32")
        us[st] = u[0].double().cpu().numpy()
        del sim, u
        torch.cuda.empty_cache()
    for st in ("f32", "bf16", "f16"):
        err = rel(us[st], us["f64"])
        announce("256^3 storage %s: u_x rel L2 vs FP64 after %d steps = %.3e" % (st, n, err))
        assert err < {"f32": 1e-5, "bf16": 0.05, "f16": 0.02}[st]


def test_create_time_launch_shape_choice_keeps_the_rest_state():
    """256^3 FP32 (2.5 GB of populations): lbm_create times three workgroup
    mappings on the plain step, then restores the rest state.  The state is
    zero and the step counter 0 after create, and the first 12 steps (one
    residual check) agree bit for bit with a context whose mapping is fixed (no timing)."""
    import torch
    announce("create-time launch shape, 256^3")
    shape, gamma = (256, 256, 256), 1.0
    tuned = _sim(shape, "f32", gamma)
    assert tuned.t == 0
    assert int(torch.count_nonzero(tuned.get_state())) == 0
    tuned.step(12)
    a = tuned.get_state()
    h = tuned.history(4)
    del tuned
    torch.cuda.empty_cache()
    fixed = _sim(shape, "f32", gamma, launch=dict(xcd_chunk=2))
    fixed.step(12)
    assert torch.equal(a, fixed.get_state())
    assert np.array_equal(h, fixed.history(4))
    del fixed, a
    torch.cuda.empty_cache()
