"""Benchmark of the fused preconditioned GLBE step on one MI355X.

Headline workload: the square-duct flow on 256x256x256 (walls in y and z,
periodic x) with F_x = F0 sin(2 pi y/Ly)(1 + cos(2 pi z/Lz)/2), F0 = 1e-5,
nu = 0.131, gamma = 1 (at this size the force drives Ma ~ 0.16, too fast for
gamma < 1), FP32 deviation storage with FP32 collision, FP64 residual, mass
and flow rate every 10th step.  One step = one fused stream-collide launch
over all 16.8 M nodes.  Inputs (state, force field) are resident in HBM
before the timed region; nothing crosses PCIe inside it.

Prints ONE JSON line: MLUPS of the timed steps; the roofline of the plain
step kernel from a HIP event on every launch on the library's stream
(algorithmic bytes per launch / mean time from one step kernel's end to the
next one's); the same for BF16,
FP16 and FP64 storage at 256^3 and for the cache-resident 64^3 duct; wall
time to a residual of 1e-8 for gamma < 1 against plain FP64 gamma = 1
(64^3 duct gamma sweep, 128^3 preconditioning-and-precision ladders); and
the FP64 CPU oracle timed on the host.  --extras adds the longer studies.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MALL_BYTES = 256 * 1024 * 1024   # last-level cache (Infinity Cache) of the MI355X
# the step kernels, their launch (shape, wave cap, timing events) and the
# constants they are given: a change to any of these invalidates the counter
# traffic taken on them
KERNEL_SOURCES = ["paper_0809_4730_amd/csrc/kernels.hip", "paper_0809_4730_amd/csrc/collide.hpp",
                  "paper_0809_4730_amd/csrc/common.hpp", "paper_0809_4730_amd/csrc/stream.hpp",
                  "paper_0809_4730_amd/csrc/lattice.hpp", "paper_0809_4730_amd/csrc/lbm_capi.hip",
                  "paper_0809_4730_amd/csrc/launch.hpp", "paper_0809_4730_amd/csrc/ctx.hpp",
                  "paper_0809_4730_amd/csrc/args.hpp"]
STORAGE_BYTES = {"f32": 4, "f64": 8, "bf16": 2, "f16": 2}
METRIC = "MLUPS, % HBM roofline; wall time to 1e-8 residual, gamma<1 vs plain gamma=1"


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_node(storage_bytes, force_field, check_every, mhd=False):
    """Bytes one node update must move: each population read once and written
    once, the force field read once (compute type), and on a residual step the
    velocity snapshot (compute type) read and written, amortised over
    check_every steps."""
    cb = 8 if storage_bytes == 8 else 4
    b = 2 * 19 * storage_bytes
    if mhd:
        b += 2 * 21 * cb
    if force_field:
        b += 3 * cb
    b += 2 * 3 * cb / check_every
    return b


NO_CHECK = 1 << 30   # check_every that never fires: a march of the plain step kernel only


def make_sim(shape, storage, gamma, nu=0.131, F0=1e-5, bc=("periodic", "wall", "wall"),
             check_every=10, **kw):
    import torch

    import paper_0809_4730_amd as pkg
    from paper_0809_4730_amd import inputs
    dt = torch.float64 if storage == "f64" else torch.float32
    F = torch.tensor(inputs.duct_force(shape, F0), dtype=dt, device="cuda")
    s = pkg.default_rates(nu, gamma)
    return pkg.Simulation(shape, bc, gamma, s, storage=storage, force=F, check_every=check_every,
                          **kw)


def timed_steps(sim, steps, warmup):
    """W untimed steps, then exactly `steps` steps bracketed by device
    synchronisations, each step kernel's launch on the library's stream carrying
    a HIP event (a step's duration: from the previous step kernel's end to its
    own, the kernel and the dispatch gap before it); the timed region ends with the residual checks' partial sums
    reduced into the history and its last record read.  Returns (MLUPS,
    wall s, plain-kernel us list, check-kernel us list)."""
    import torch
    if warmup > 0:  # the first timed call also creates the library's event pool
        sim.step_times(1)
        sim.step(warmup - 1)
    torch.cuda.synchronize()
    t_first = sim.t + 1
    t0 = time.perf_counter()
    times, _ = sim.step_times(steps)
    sim.history(1)  # the residual checks' FP64 sums reduced and read back
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ce = sim._params.check_every
    plain = [float(us) for i, us in enumerate(times) if (t_first + i) % ce != 0]
    check = [float(us) for i, us in enumerate(times) if (t_first + i) % ce == 0]
    return sim.N * steps / wall / 1e6, wall, plain, check


def kernel_time_us(sim, launches, warmup=20):
    """Mean duration of the step kernel from two HIP events around `launches`
    back-to-back launches on the library's stream (sim built with NO_CHECK on
    torch's current stream, so every launch is the same kernel).  For kernels
    of a few microseconds this is the rate a march achieves; events around
    each launch would add their own gaps."""
    import torch
    assert sim._stream == torch.cuda.current_stream(sim.device)
    sim.step(warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(launches)
    e1.record()
    e1.synchronize()
    return 1000.0 * e0.elapsed_time(e1) / launches


def traffic_from_profiles(kernel_tag, khash):
    """HBM bytes per launch from the committed rocprofv3 counter summary, only if
    it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    e = d.get(kernel_tag)
    if not e or e.get("kernel_hash") != khash:
        return None
    return e.get("bytes_per_launch")


def population_bytes(shape, storage):
    n = shape[0] * shape[1] * shape[2]
    return 2 * 19 * STORAGE_BYTES[storage] * n


def step_roofline(shape, storage, gamma, steps, warmup, **kw):
    """One storage type on one duct: MLUPS over the timed steps (checks
    included) and the roofline of the plain step kernel."""
    import torch
    sim = make_sim(shape, storage, gamma, **kw)
    launch = sim.launch
    mlups, wall, plain, check = timed_steps(sim, steps, warmup)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    N = shape[0] * shape[1] * shape[2]
    us = statistics.fmean(plain)
    bpn = algorithmic_bytes_per_node(STORAGE_BYTES[storage], True, NO_CHECK)
    achieved = bpn * N / (us * 1e-6) / 1e9
    resident = population_bytes(shape, storage) <= MALL_BYTES
    return {"storage": storage, "MLUPS": round(mlups, 2), "wall_s": wall,
            "ms_per_step": 1000.0 * wall / steps, "kernel_us": round(us, 3),
            "kernel_us_min": round(min(plain), 3), "kernel_us_max": round(max(plain), 3),
            "check_kernel_us": round(statistics.fmean(check), 3) if check else None,
            "launches_timed": len(plain), "alg_bytes_per_node": bpn,
            "alg_bytes_per_launch": int(round(bpn * N)),
            "achieved_GBs": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
            "bound": "mall" if resident else "hbm", "launch": launch}


def timed_region(sim, steps, warmup):
    """(MLUPS, wall seconds) of `steps` full steps (residual checks included),
    bracketed by device synchronisations."""
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return sim.N * steps / wall / 1e6, wall


def small_duct_line(steps, warmup):
    """The 64^3 duct (FP32, gamma = 0.1): 43 MB of populations, resident in the
    256 MB last-level cache, so a cache rate ("bound": "mall").  MLUPS of
    `steps` steps with checks; the plain kernel from events around
    back-to-back launches (kernel_time_us)."""
    import torch
    shape = (64, 64, 64)
    sim = make_sim(shape, "f32", 0.1)
    launch = sim.launch
    mlups, wall = timed_region(sim, steps, warmup)
    sim.close()
    sim = make_sim(shape, "f32", 0.1, check_every=NO_CHECK)
    us = kernel_time_us(sim, steps)
    sim.close()
    torch.cuda.empty_cache()
    bpn = algorithmic_bytes_per_node(4, True, NO_CHECK)
    gbs = bpn * 64 ** 3 / (us * 1e-6) / 1e9
    return {"storage": "f32", "gamma": 0.1, "MLUPS": round(mlups, 2),
            "ms_per_step": round(1000.0 * wall / steps, 5), "kernel_us": round(us, 3),
            "alg_bytes_per_node": bpn, "achieved_GBs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "bound": "mall", "launch": launch}


def mhd256_line(steps, warmup):
    """The coupled step (D3Q19 flow + D3Q7 induction, Lorentz force) at HBM
    scale: 256^3 FP32, walls normal to y and to B0 (the Hartmann setting of the
    coupled workload, Ha = 10, Pm = 0.01, gamma = gamma_m = 0.1).  MLUPS of
    the timed steps and the plain kernel from per-launch HIP events."""
    import torch

    import paper_0809_4730_amd as pkg
    from paper_0809_4730_amd import inputs
    cfg = inputs.HARTMANN
    B0, chi = inputs.hartmann_parameters(10.0, 0.01, cfg["shape"][1], cfg["nu"], cfg["eta"])
    sim = pkg.Simulation((256, 256, 256), cfg["bc"], 0.1, pkg.default_rates(cfg["nu"], 0.1),
                         storage="f32", force=cfg["F"],
                         mhd=dict(gamma_m=0.1, chi=chi, eta=cfg["eta"], B0=(0.0, B0, 0.0)))
    launch = sim.launch
    mlups, wall, plain, check = timed_steps(sim, steps, warmup)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    us = statistics.fmean(plain)
    bpn = 2 * (19 + 21) * 4
    gbs = bpn * 256 ** 3 / (us * 1e-6) / 1e9
    return {"workload": "coupled flow + induction step, 256^3, FP32, uniform force",
            "MLUPS": round(mlups, 2), "kernel_us": round(us, 3),
            "check_kernel_us": round(statistics.fmean(check), 3) if check else None,
            "alg_bytes_per_node": bpn, "achieved_GBs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "bound": "hbm", "launch": launch}


def hbm_ceiling(shape=(256, 256, 256), reps=10):
    """What the HBM delivers on this GPU for five copies (lbm_bandwidth_probe)
    over the 256^3 lattice: a plain streaming copy of 16-byte vectors; copies
    with the FP32 flow step's plane pattern (22 FP32 planes read, 19 written
    per node) and the coupled step's (40 and 40), every plane read at the node
    itself; and copies with each step's exact memory traffic (the steps'
    neighbour, gather and store code without the arithmetic; walls as in the
    duct, y and z, and in the coupled workload, y).  XCD chunks of 2,
    streaming loads and stores; each with no cap on the waves per SIMD and
    with the steps' caps of 5 and 3.  Mean of `reps` back-to-back launches
    between two HIP events on the current stream, after two warm-up launches
    (like the steps' durations, the dispatch gaps included); the best of the
    caps is the ceiling."""
    import torch

    import paper_0809_4730_amd as pkg
    nodes = shape[0] * shape[1] * shape[2]
    src = torch.ones(40 * nodes, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {"nodes": nodes}
    for pattern, key, walls in ((0, "stream_copy", ()), (1, "step_pattern_copy", ()),
                                (2, "coupled_pattern_copy", ()),
                                (3, "step_exact_copy", (False, True, True)),
                                (4, "coupled_exact_copy", (False, True, False))):
        best = None
        for waves in (8, 5, 3):
            for _ in range(2):
                pkg.bandwidth_probe(pattern, src, dst, shape, walls=walls, waves=waves)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                nbytes = pkg.bandwidth_probe(pattern, src, dst, shape, walls=walls, waves=waves)
            e1.record()
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            e = {"bytes": nbytes, "waves": waves, "us": round(us, 2),
                 "GBs": round(nbytes / (us * 1e-6) / 1e9, 1)}
            out["%s_waves%d" % (key, waves)] = e
            if best is None or e["GBs"] > best["GBs"]:
                best = e
        out[key] = best
    del src, dst
    torch.cuda.empty_cache()
    return out


def copy_bandwidth_GBs(nbytes=4 << 30, reps=10):
    """Device-to-device copy (read + write) bandwidth of torch's copy kernel."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def _oracle_step_times(shape, bc, F, gamma, s, warm=3, timed=20):
    """Per-step wall times of the FP64 oracle march (3 warm-up steps first)."""
    from oracle import glbe
    fl = glbe.Flow(shape, bc, F, gamma, s)
    fl.step(warm)
    out = []
    for _ in range(timed):
        t0 = time.perf_counter()
        fl.step(1)
        out.append(time.perf_counter() - t0)
    return out


def cpu_baseline():
    """The FP64 oracle (numpy, dense 19x19 transform through BLAS) on the host:
    median of 20 steps after 3 warm-ups on a z-slab of the 256^3 duct
    (256 x 256 x 16 nodes, the force of the slab's planes; the full lattice is
    processed slab by slab, each slab with the same per-node work), and on the
    whole 64^3 duct.  value = slab MLUPS."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import glbe
    from paper_0809_4730_amd import inputs
    bc = ("periodic", "wall", "wall")
    s = glbe.rates(0.131, 1.0)
    slab = (256, 256, 16)
    F256 = inputs.duct_force((256, 256, 256))[:, :slab[2]]
    t_slab = statistics.median(_oracle_step_times(slab, bc, np.ascontiguousarray(F256), 1.0, s))
    s01 = glbe.rates(0.131, 0.1)
    t64 = statistics.median(_oracle_step_times((64, 64, 64), bc, inputs.duct_force((64, 64, 64)),
                                               0.1, s01))
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    n_slab = slab[0] * slab[1] * slab[2]
    return {"value": round(n_slab / t_slab / 1e6, 4), "unit": "MLUPS", "cores": int(threads),
            "kind": "oracle",
            "sample": "FP64 numpy oracle (dense 19x19 transform via BLAS), median of 20 steps "
                      "after 3 warm-ups on a 256x256x16 z-slab of the 256^3 duct at gamma=1 "
                      "(%.3f s per slab step; the 256^3 step is 16 such slabs, %.1f s)"
                      % (t_slab, 16 * t_slab),
            "os_cpu_count": os.cpu_count(), "blas_threads": int(threads),
            "duct64_MLUPS": round(64 ** 3 / t64 / 1e6, 4),
            "duct64_sample": "whole 64^3 duct, gamma=0.1, median of 20 steps after 3 warm-ups"}


def cpu_time_to_residual_poiseuille():
    """The FP64 oracle (numpy, on the host) marched to steady state on the plane
    Poiseuille 8x8x32 workload (nu = 0.1, residual 1e-10) at gamma = 1 and 0.1:
    the CPU-side time to steady state, next to the GPU's in the extras."""
    import numpy as np

    from oracle import glbe
    from paper_0809_4730_amd import inputs
    cfg = inputs.POISEUILLE
    rows = []
    for g in (1.0, 0.1):
        fl = glbe.Flow(cfg["shape"], cfg["bc"], np.array(cfg["F"]), g, glbe.rates(cfg["nu"], g))
        t0 = time.perf_counter()
        ok = fl.run_to(cfg["tol"], 100000)
        rows.append({"gamma": g, "steps": fl.t if ok else -1,
                     "wall_s": round(time.perf_counter() - t0, 2)})
    return {"kind": "oracle", "workload": "plane Poiseuille 8x8x32, FP64, residual 1e-10",
            "rows": rows}


def time_to_residual(shape, storage, gamma, tol, max_steps, make=None, poll=200, **kw):
    """Steps and wall time to a residual below tol; `make` builds the simulation
    (default: the duct of make_sim)."""
    import torch
    sim = make_sim(shape, storage, gamma, **kw) if make is None else make()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        steps, r = sim.run_to_residual(tol, max_steps, poll_every=poll)
        status = "ok" if steps > 0 else "not reached"
    except Exception as e:  # unstable
        steps, r, status = -1, float("nan"), "error: %s" % e
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h = sim.history(64)
    floor = float(h[:, 1].min()) if len(h) else float("nan")
    return {"gamma": gamma, "storage": storage, "steps": int(steps), "wall_s": round(wall, 4),
            "final_residual": r, "min_residual_seen": floor, "status": status, "steps_run": sim.t}


def time_to_residual_mixed(shape, gamma, tol, switch_tol, max_steps, poll=200):
    """Wall time to tol marching FP32 storage until switch_tol, then continuing
    the same state in FP64 storage (lbm_convert_state); both simulations are
    built before the clock starts."""
    import torch

    import paper_0809_4730_amd as pkg
    lo, hi = make_sim(shape, "f32", gamma), make_sim(shape, "f64", gamma)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        steps, r = pkg.run_to_residual_mixed(lo, hi, tol, switch_tol, max_steps, poll)
        status = "ok" if steps > 0 else "not reached"
    except Exception as e:  # unstable
        steps, r, status = -1, float("nan"), "error: %s" % e
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"gamma": gamma, "storage": "f32 then f64", "switch_at": switch_tol,
            "f32_steps": lo.t, "steps": int(steps), "wall_s": round(wall, 4),
            "final_residual": r, "status": status}


def extras(args):
    import numpy as np
    import torch

    import paper_0809_4730_amd as pkg
    from paper_0809_4730_amd import inputs
    out = {}
    # time to residual 1e-8 on the 64^3 duct: gamma sweep vs plain gamma = 1 (FP64 and FP32)
    tt = []
    for g in (1.0, 0.5, 0.1, 0.05, 0.02, 0.01):
        tt.append(time_to_residual((64, 64, 64), "f64", g, 1e-8, 400000))
    for g in (1.0, 0.5, 0.1, 0.05):
        e = time_to_residual((64, 64, 64), "f32", g, 1e-7, 400000)
        e["note"] = "FP32 storage stalls near 6e-8 at this Mach number; tol 1e-7"
        tt.append(e)
    out["time_to_residual_duct64"] = tt
    # the same to 1e-8 marching FP32 until 1e-6, then the same state in FP64
    tm = [time_to_residual_mixed((64, 64, 64), g, 1e-8, 1e-6, 400000) for g in (1.0, 0.5, 0.1, 0.05)]
    for e in tm:
        if tt[0]["steps"] > 0 and e["steps"] > 0:
            e["speedup_vs_f64_gamma1_wall"] = round(tt[0]["wall_s"] / e["wall_s"], 3)
    out["time_to_residual_duct64_mixed_f32_f64"] = tm
    # plane Poiseuille 8x8x32 (uniform force) to 1e-10, FP64
    pc = inputs.POISEUILLE

    def pois(g):
        return pkg.Simulation(pc["shape"], pc["bc"], g, pkg.default_rates(pc["nu"], g),
                              storage="f64", force=pc["F"])
    tp = [time_to_residual(None, "f64", g, 1e-10, 400000, make=lambda g=g: pois(g))
          for g in (1.0, 0.5, 0.1, 0.05)]
    for e in tp[1:]:
        if tp[0]["steps"] > 0 and e["steps"] > 0:
            e["step_ratio_vs_gamma1"] = round(tp[0]["steps"] / e["steps"], 3)
    out["time_to_residual_poiseuille8x8x32_tol1e-10"] = tp
    if not args.no_cpu:  # the oracle on the host, same workload (about a minute)
        out["cpu_oracle_time_to_residual_poiseuille8x8x32"] = cpu_time_to_residual_poiseuille()
    ref = tt[0]
    if ref["steps"] > 0:
        for e in tt[1:]:
            if e["steps"] > 0:
                e["speedup_vs_f64_gamma1_wall"] = round(ref["wall_s"] / e["wall_s"], 3)
                e["step_ratio_vs_f64_gamma1"] = round(ref["steps"] / e["steps"], 3)
    # 256^3 throughput with stochastic 16-bit stores (the nearest-even forms
    # are in the headline line)
    out["duct256_stochastic_rounding"] = [
        step_roofline((256, 256, 256), st, 1.0, args.big_steps, 10, rounding="stochastic")
        for st in ("bf16", "f16")]
    out["hbm_copy_GBs"] = round(copy_bandwidth_GBs(), 1)
    # coupled MHD step on the Hartmann workload
    cfg = inputs.HARTMANN
    B0, chi = inputs.hartmann_parameters(10.0, 0.01, cfg["shape"][1], cfg["nu"], cfg["eta"])
    mp = dict(gamma_m=cfg["gamma_m"], chi=chi, eta=cfg["eta"], B0=(0.0, B0, 0.0))

    def hart(g=cfg["gamma"], gm=cfg["gamma_m"]):
        mp2 = dict(mp, gamma_m=gm)
        return pkg.Simulation(cfg["shape"], cfg["bc"], g, pkg.default_rates(cfg["nu"], g),
                              storage="f32", force=cfg["F"], mhd=mp2)
    sim = hart()
    mlups, wall = timed_region(sim, 1000, 100)
    us = 1e6 * wall / 1000
    bpn = algorithmic_bytes_per_node(4, False, 10, mhd=True)
    out["hartmann_mhd_step"] = {"shape": cfg["shape"], "MLUPS": round(mlups, 1),
                                "kernel_us": round(us, 2), "alg_bytes_per_node": bpn,
                                "achieved_GBs": round(bpn * sim.N / (us * 1e-6) / 1e9, 1)}
    del sim
    # the coupled step at HBM scale: 256^3, FP32, walls normal to B0, plain kernel
    big = pkg.Simulation((256, 256, 256), cfg["bc"], 0.1, pkg.default_rates(cfg["nu"], 0.1),
                         storage="f32", force=cfg["F"], check_every=NO_CHECK, mhd=mp)
    us = kernel_time_us(big, 30, warmup=5)
    bpn = 2 * (19 + 21) * 4
    out["mhd_step_256"] = {"kernel_us": round(us, 2), "kernel_MLUPS": round(big.N / us, 1),
                           "alg_bytes_per_node": bpn,
                           "achieved_GBs": round(bpn * big.N / (us * 1e-6) / 1e9, 1),
                           "frac_hbm": round(bpn * big.N / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    big.close()
    del big
    torch.cuda.empty_cache()
    ttm = []
    for g, gm in ((1.0, 1.0), (0.1, 0.1), (0.1, 1.0), (1.0, 0.1), (0.1, 0.3), (0.3, 0.1)):
        e = time_to_residual(None, "f32", g, 2e-7, 400000, make=lambda g=g, gm=gm: hart(g, gm))
        e["gamma_m"] = gm
        ttm.append(e)
    out["time_to_residual_hartmann_Ha10_f32_tol2e-7"] = ttm
    out["precision_duct64"] = precision_table()
    out["adjoint"] = adjoint_extras()
    out.update(cavity_extras())
    out["naive_source_control"] = naive_source_extras()
    out["paper_poiseuille"] = paper_poiseuille_extras()
    out["paper_hartmann_Re286_Ha71.6"] = paper_hartmann_extras()
    out["d2q9"] = d2q9_extras()
    out["stability_envelope"] = stability_extras()
    return out


def naive_source_extras():
    """Sec. 3.1 negative control on the GPU: steady states of a two-mode forcing
    F = F0 (sin ky, sin 2kx, 0) on a periodic LxLx1 lattice (FP64, MRT rates,
    residual 1e-11) with the preconditioned source and with the naive S/gamma.
    The naive form departs from the consistent one in proportion to
    (1 - gamma)/gamma^2.  The consistent form's own gamma-dependence is the
    lattice's truncation error, which grows with tau* = 3 nu/gamma + 1/2 and
    falls as (k dx)^2: shown at L = 64 and 128 with the same velocity amplitude."""
    import numpy as np
    import torch

    import paper_0809_4730_amd as pkg
    nu, F64 = 0.1, 1e-6
    per = ("periodic",) * 3

    def steady(L, gamma, source):
        F0 = F64 * (64 / L) ** 2  # the same velocity amplitude at every L
        k = 2 * np.pi / L
        x = np.arange(L) + 0.5
        F = np.zeros((3, 1, L, L))
        F[0] = F0 * np.sin(k * x)[None, :, None]
        F[1] = F0 * np.sin(2 * k * x)[None, None, :]
        sim = pkg.Simulation((L, L, 1), per, gamma, pkg.default_rates(nu, gamma), storage="f64",
                             force=torch.tensor(F, dtype=torch.float64, device="cuda"),
                             source=source)
        steps, r = sim.run_to_residual(1e-11, 4000000, poll_every=2000)
        _, u, _ = sim.moments("f64")
        return u.cpu().numpy(), steps

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out = {"nu": nu, "F0_at_L64": F64, "F0": "F0_at_L64 (64/L)^2"}
    for L in (64, 128):
        u1, _ = steady(L, 1.0, "precond")
        rows = []
        for g in ((0.5, 0.2, 0.1) if L == 64 else (0.1,)):
            uc, nc = steady(L, g, "precond")
            un, nn = steady(L, g, "naive")
            d = rel(un, uc)
            rows.append({"gamma": g, "consistent_vs_gamma1": rel(uc, u1), "naive_vs_consistent": d,
                         "naive_vs_consistent_over_(1-g)/g^2": d / ((1 - g) / g ** 2),
                         "steps_consistent": nc, "steps_naive": nn})
        out["L%d" % L] = rows
    return out


def paper_poiseuille_extras():
    """The paper's plane Poiseuille cases (Sec. 5), gap 64 between halfway
    bounce-back walls, FP64, residual 1e-8: the low-viscosity case (nu = 0.001,
    u_max = 0.00051, Re = 32.6) for gamma = 1 ... 0.001, and the higher-Mach
    case (nu = 0.005, u_max = 0.0128, Re = 163.8) down to where it turns
    unstable: steps, wall time and the profile's error against the parabola."""
    import numpy as np
    import torch

    import paper_0809_4730_amd as pkg
    from paper_0809_4730_amd import stability
    H = 64
    z = np.arange(H) + 0.5

    def case(nu, umax, gammas):
        F = stability.poiseuille_force(nu, umax, H)
        exact = umax * (1.0 - ((z - H / 2) / (H / 2)) ** 2)
        rows = []
        for g in gammas:
            sim = pkg.Simulation((4, 4, H), ("periodic", "periodic", "wall"), g,
                                 pkg.default_rates(nu, g), storage="f64", force=(F, 0.0, 0.0))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                steps, r = sim.run_to_residual(1e-8, 6000000, poll_every=5000)
                status = "ok" if steps > 0 else "not reached"
            except pkg.LbmError as e:
                steps, status = -1, "unstable" if e.status == -4 else "error: %s" % e
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            e = {"gamma": g, "steps": int(steps), "wall_s": round(wall, 3), "status": status}
            if status == "ok":
                _, u, _ = sim.moments("f64")
                ux = u[0].cpu().numpy()[:, 0, 0]
                e["profile_rel_error"] = float(np.linalg.norm(ux - exact) / np.linalg.norm(exact))
            rows.append(e)
            sim.close()
        for e in rows[1:]:
            if e["steps"] > 0 and rows[0]["steps"] > 0:
                e["step_ratio_vs_gamma1"] = round(rows[0]["steps"] / e["steps"], 1)
                e["wall_ratio_vs_gamma1"] = round(rows[0]["wall_s"] / e["wall_s"], 1)
        return {"nu": nu, "u_max": umax, "gap": H, "Re": umax * H / nu, "rows": rows}
    return {"low_viscosity": case(0.001, 0.00051, (1.0, 0.1, 0.01, 0.001)),
            "higher_mach": case(0.005, 0.0128, (1.0, 0.5, 0.2, 0.1, 0.05, 0.02, 0.01, 0.005))}


def paper_hartmann_extras():
    """The paper's Hartmann case for the (gamma, gamma_m) study (Sec. 5):
    Re = 286, Ha = 71.6, Pm = 1e-6, nu = eta = 0.004, half-width L = 64 (128
    nodes between walls normal to y and the applied field), FP64, residual 1e-8:
    steps for gamma = 0.05 with several gamma_m, for gamma = 1, and for equal
    pairs; the centreline velocity against the Re = 286 target."""
    import torch

    import paper_0809_4730_amd as pkg
    from paper_0809_4730_amd import inputs
    nu = eta = 0.004
    ny, Ha, Pm = 128, 71.6, 1e-6
    B0, chi = inputs.hartmann_parameters(Ha, Pm, ny, nu, eta)
    uc = 286 * nu / (ny / 2)
    F = uc * nu * Ha / (ny / 2) ** 2  # flat-core Hartmann centreline u = F L^2 / (nu Ha)
    rows = []
    for g, gm in ((0.05, 1.0), (0.05, 0.2), (0.05, 0.05), (0.05, 0.02), (1.0, 1.0), (1.0, 0.2),
                  (1.0, 0.05), (0.2, 0.2), (0.1, 0.1), (0.02, 0.02)):
        sim = pkg.Simulation((4, ny, 4), ("periodic", "wall", "periodic"), g,
                             pkg.default_rates(nu, g), storage="f64", force=(F, 0.0, 0.0),
                             mhd=dict(gamma_m=gm, chi=chi, eta=eta, B0=(0.0, B0, 0.0)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            steps, r = sim.run_to_residual(1e-8, 2000000, poll_every=2000)
            status = "ok" if steps > 0 else "not reached"
        except pkg.LbmError as e:
            steps, status = -1, "error: %s" % e
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        _, u, _ = sim.moments("f64")
        rows.append({"gamma": g, "gamma_m": gm, "steps": int(steps), "wall_s": round(wall, 3),
                     "status": status,
                     "u_center_over_target": float(u[0, 0, ny // 2, 0].item()) / uc})
        sim.close()
    return {"Re": 286, "Ha": Ha, "Pm": Pm, "nu": nu, "eta": eta, "B0": B0, "chi": chi, "F": F,
            "rows": rows}


def stability_extras():
    """Stability map (Sec. 5): gamma_min for 3 viscosities x 4 velocities on
    4x4x64 FP64 channels (20,000 steps per march): sequential bisection (one
    lattice per launch, 9 marches per point) against the batched k-section (all
    points and 15 gammas per round in one launch per step, 2 rounds)."""
    import torch

    from paper_0809_4730_amd import stability
    nus, us = (0.002, 0.02, 0.1), (0.005, 0.02, 0.05, 0.08)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = stability.envelope(nus, us, lo=1e-3, hi=1.0, iters=7, max_steps=20000)
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    bat = stability.envelope_batched(nus, us, per_round=15, rounds=2, max_steps=20000)
    t_bat = time.perf_counter() - t0
    return {"sequential_s": round(t_seq, 3), "batched_s": round(t_bat, 3),
            "points": [{"nu": a["nu"], "u_max": a["u_max"], "gamma_min_bisection": round(a["gamma_min"], 5),
                        "gamma_min_batched": round(b["gamma_min"], 5)} for a, b in zip(seq, bat)]}


def d2q9_extras():
    """Two-dimensional variants: plain D2Q9 step throughput at 4096^2 per
    storage type (uniform force, periodic x, walls in y), the coupled
    D2Q9 + D2Q5 step at 2048^2 (FP32), and 2D Hartmann (Ha = 10, Pm = 0.01,
    2L = 128) steps to a residual of 2e-7 at gamma = gamma_m = 1 and 0.1."""
    import paper_0809_4730_amd as pkg
    from paper_0809_4730_amd import inputs
    nu = 0.1
    bc = ("periodic", "wall", "periodic")
    out = {"step_4096x4096": []}
    for st, nb in (("f32", 4), ("bf16", 2), ("f16", 2), ("f64", 8)):
        sim = pkg.Simulation((4096, 4096, 1), bc, 0.1, pkg.default_rates_d2q9(nu, 0.1),
                             storage=st, force=(1e-7, 0.0), check_every=NO_CHECK, lattice="d2q9")
        us = kernel_time_us(sim, 200)
        bpn = 2 * 9 * nb
        out["step_4096x4096"].append({"storage": st, "kernel_us": round(us, 2),
                                      "kernel_MLUPS": round(sim.N / us, 1),
                                      "alg_bytes_per_node": bpn,
                                      "achieved_GBs": round(bpn * sim.N / (us * 1e-6) / 1e9, 1)})
        sim.close()
    L, Ha, Pm, eta, F = 64, 10.0, 0.01, 0.025, 1e-5
    B0, chi = inputs.hartmann_parameters(Ha, Pm, 2 * L, nu, eta)

    def hart(g, n=(4, 2 * L, 1), ce=10):
        return pkg.Simulation(n, bc, g, pkg.default_rates_d2q9(nu, g, "lambda", 3 / 16),
                              storage="f32", force=(F, 0.0), check_every=ce, lattice="d2q9",
                              mhd=dict(gamma_m=g, chi=chi, eta=eta, B0=(0.0, B0)))
    sim = hart(0.1, (2048, 2048, 1), NO_CHECK)
    us = kernel_time_us(sim, 200)
    bpn = 2 * (9 + 10) * 4
    out["mhd_step_2048x2048_f32"] = {"kernel_us": round(us, 2), "kernel_MLUPS": round(sim.N / us, 1),
                                     "alg_bytes_per_node": bpn,
                                     "achieved_GBs": round(bpn * sim.N / (us * 1e-6) / 1e9, 1)}
    sim.close()
    out["hartmann2d_Ha10_tol2e-7"] = [
        time_to_residual(None, "f32", g, 2e-7, 400000, make=lambda g=g: hart(g)) for g in (1.0, 0.1)]
    return out


def cavity_extras():
    """Lid-driven cubic cavity, 64^3 fluid nodes, Re = 100 (U0 = 0.0235,
    nu = 0.015), FP32: steps and wall time to a residual of 1e-6 for each gamma,
    without field and with Ha = 45 (B0 parallel to the lid, normal to its motion;
    eta = 0.015, Pm = 5.625e-7, gamma_m = gamma) on an induction lattice that
    extends 16 nodes beyond each wall; plus the per-step time of both."""
    import numpy as np

    import paper_0809_4730_amd as pkg
    from paper_0809_4730_amd import inputs
    c = inputs.MHD_CAVITY
    W, pad, nu = c["W"], c["pad"], c["nu"]
    walls = ("wall", "wall", "wall")
    wall_u = np.zeros((6, 3))
    wall_u[5] = (c["U0"], 0.0, 0.0)
    B0, chi = inputs.cavity_field(c["Ha"], c["Pm"], W, nu, c["eta"])
    n = W + 2 * pad

    def plain(g):
        return pkg.Simulation((W, W, W), walls, g, pkg.default_rates(nu, g), storage="f32",
                              wall_u=wall_u)

    def magnetic(g):
        return pkg.Simulation((n, n, n), walls, g, pkg.default_rates(nu, g), storage="f32",
                              wall_u=wall_u,
                              mhd=dict(gamma_m=g, chi=chi, eta=c["eta"], B0=(0.0, B0, 0.0),
                                       pad=(pad, pad, pad)))
    out = {}
    for name, make in (("cavity64_Ha0", plain), ("cavity64_Ha45_ext16", magnetic)):
        rows = []
        for g in c["gammas"]:
            rows.append(time_to_residual(None, "f32", g, c["tol"], 400000, make=lambda g=g: make(g)))
        ref = rows[0]
        for e in rows[1:]:
            if ref["steps"] > 0 and e["steps"] > 0:
                e["step_ratio_vs_gamma1"] = round(ref["steps"] / e["steps"], 3)
                e["speedup_vs_gamma1_wall"] = round(ref["wall_s"] / e["wall_s"], 3)
        sim = make(0.1)
        mlups, wall = timed_region(sim, 500, 50)
        out[name] = {"time_to_residual_tol1e-6": rows, "lattice_nodes": sim.N,
                     "us_per_step": round(1e6 * wall / 500, 2), "MLUPS": round(mlups, 1)}
    # stability of the SRT limit (all rates equal to the shear rate, Sec. 3.1)
    # against the paper's MRT rates on the same cavity, without and with the
    # Ha = 45 field (gamma_m = gamma), at gamma = 1 and 0.1
    srt = []
    for field in (False, True):
        for g in (1.0, 0.1):
            for v in ((0.015, 0.05, 0.166) if not field else (0.015, 0.166)):
                for form in ("mrt", "srt"):
                    r = pkg.default_rates(v, g)
                    if form == "srt":
                        r = np.full(19, r[9])

                    def mk(r=r, g=g, v=v, field=field):
                        if not field:
                            return pkg.Simulation((W, W, W), walls, g, r, storage="f32",
                                                  wall_u=wall_u)
                        Bv, cv = inputs.cavity_field(c["Ha"], c["Pm"], W, v, c["eta"])
                        return pkg.Simulation((n, n, n), walls, g, r, storage="f32",
                                              wall_u=wall_u,
                                              mhd=dict(gamma_m=g, chi=cv, eta=c["eta"],
                                                       B0=(0.0, Bv, 0.0), pad=(pad, pad, pad)))
                    e = time_to_residual(None, "f32", g, c["tol"], 60000, make=mk)
                    srt.append({"field": "Ha45" if field else "none", "gamma": g, "nu": v,
                                "rates": form, "status": e["status"][:60], "steps": e["steps"],
                                "steps_run": e["steps_run"]})
    out["cavity64_srt_vs_mrt"] = srt
    return out


def precision_table():
    """Velocity error of each storage type against FP64 on the 64^3 duct at the
    FP64 steady state (residual 1e-8), gamma = 0.1."""
    import numpy as np
    import torch
    ref = make_sim((64, 64, 64), "f64", 0.1)
    ref.run_to_residual(1e-8, 200000, poll_every=200)
    n = ref.t
    _, u64, _ = ref.moments("f64")
    out = {"steps": n}
    for st in ("f32", "bf16", "bf16_sr", "f16", "f16_sr"):
        kw = {"rounding": "stochastic"} if st.endswith("_sr") else {}
        sim = make_sim((64, 64, 64), st.split("_")[0], 0.1, **kw)
        sim.step(n)
        _, u, _ = sim.moments("f64")
        err = float(torch.linalg.vector_norm(u - u64) / torch.linalg.vector_norm(u64))
        mass, _ = sim.reductions()
        floor = float(sim.history(64)[:, 1].min())
        out[st] = {"u_rel_L2_vs_f64": err, "mass_drift": mass, "residual_floor": floor}
    return out


def adjoint_extras():
    """Steady adjoint on the 128^3 duct (FP32) and the checkpointed unrolled
    adjoint over 2000 steps on 32^3: iteration counts and kernel rates."""
    import torch
    from paper_0809_4730_amd import inputs
    cfg = inputs.ADJOINT
    out = {}
    sim = make_sim(cfg["shape"], "f32", 0.1)
    t0 = time.perf_counter()
    steps, r = sim.run_to_residual(1e-7, 400000, poll_every=1000)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    grad, iters, change = sim.adjoint_steady(tol=1e-6, max_iter=400000)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    N = sim.N
    out["steady_128"] = {"gamma": 0.1, "forward_steps_to_1e-7": steps, "forward_s": round(t_fwd, 3),
                         "adjoint_iters": iters, "adjoint_change": change,
                         "adjoint_s": round(t_adj, 3),
                         "adjoint_MLUPS": round(N * iters / t_adj / 1e6, 1),
                         "grad_norm": float(torch.linalg.vector_norm(grad))}
    del sim, grad
    torch.cuda.empty_cache()
    sim = make_sim(cfg["unrolled_shape"], "f32", cfg["gamma"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = sim.adjoint_unrolled(cfg["unrolled_steps"], cfg["ckpt_every"])
    torch.cuda.synchronize()
    out["unrolled_32"] = {"steps": cfg["unrolled_steps"], "ckpt_every": cfg["ckpt_every"],
                          "wall_s": round(time.perf_counter() - t0, 3),
                          "grad_norm": float(torch.linalg.vector_norm(g))}
    return out


def precision_steady_256():
    """The precision form at full size: the 256^3 duct (C1 force, nu = 0.131,
    gamma = 1) marched in FP64 to a residual of 1e-8, then FP32, BF16 and FP16
    (nearest and stochastic rounding) storage marched the same number of steps;
    u against FP64 per storage type, and each one's residual floor."""
    import numpy as np
    import torch
    shape = (256, 256, 256)
    out = {"workload": "square duct 256^3, gamma = 1, nu = 0.131, C1 force"}
    ref = make_sim(shape, "f64", 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = -1
    while n < 0 and ref.t < 400000:  # in chunks, with a progress line each
        n, r = ref.run_to_residual(1e-8, 20000, poll_every=2000)
        print("f64 step %d residual %.3e" % (ref.t, r), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    out["f64"] = {"steps": int(n), "wall_s": round(time.perf_counter() - t0, 2), "residual": r}
    _, u_ref, _ = ref.moments("f64")
    u_ref = u_ref[0].cpu().numpy()
    ref.close()
    del ref
    torch.cuda.empty_cache()
    for key in ("f32", "bf16", "bf16_sr", "f16", "f16_sr"):
        st = key.split("_")[0]
        sim = make_sim(shape, st, 1.0, **({"rounding": "stochastic"} if key.endswith("_sr") else {}))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while sim.t < n:
            sim.step(min(20000, int(n) - sim.t))
            torch.cuda.synchronize()
            print("%s step %d" % (key, sim.t), file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        h = np.asarray(sim.history())
        _, u, _ = sim.moments("f64")
        ux = u[0].cpu().numpy()
        out[key] = {"steps": int(n), "wall_s": round(wall, 2),
                   "u_rel_L2_vs_f64": float(np.linalg.norm(ux - u_ref) / np.linalg.norm(u_ref)),
                   "residual_floor": float(h[:, 1].min()) if len(h) else None}
        sim.close()
        del sim, u
        torch.cuda.empty_cache()
    print(json.dumps({"probe": "precision256", **out}), flush=True)


def ladder_results(shape, ladders, window, workload):
    """Wall time to a residual of 1e-8 for precision ladders on the duct of
    make_sim, each rung continuing the previous rung's state on the device
    (lbm_convert_state).  ladders: (gamma, rungs) with rungs of (storage,
    criterion, tol).  A rung ends on the velocity residual R ("r") or, for
    16-bit storage, on the kinetic energy sum |u|^2 ("e"): its relative change
    over `window` steps, a global sum in which the rounding noise of the
    stored values averages out while R measures it (the duct's net flow rate
    is zero by symmetry, so it cannot serve).  A ladder's contexts are built
    before its clock starts; u of each final state against the first ladder's
    (FP64 alone at gamma = 1)."""
    import numpy as np
    import torch
    out = {"workload": workload, "ladders": []}

    def energy(sim):
        return float(sim.history(1)[-1, 3])

    u_ref = None
    for gamma, lad in ladders:
        name = "gamma %g: " % gamma + " -> ".join("%s(%s<%g)" % rung for rung in lad)
        sims = [make_sim(shape, k.split("_")[0], gamma,
                         **({"rounding": "stochastic"} if k.endswith("_sr") else {}))
                for k, _, _ in lad]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rungs, prev, ok = [], None, True
        for (k, crit, tol), sim in zip(lad, sims):
            if prev is not None:
                sim.convert_from(prev)
            t1 = time.perf_counter()
            done = False
            try:
                if crit == "r":
                    while not done and sim.t < 400000:  # in chunks, with a progress line each
                        n, r = sim.run_to_residual(tol, 20000, poll_every=window)
                        done = n > 0
                        print("%s: %s step %d R %.3e" % (name, k, sim.t, r), file=sys.stderr,
                              flush=True)
                else:
                    sim.step(window)
                    e0 = energy(sim)
                    while not done and sim.t < 400000:
                        sim.step(window)
                        e1 = energy(sim)
                        de = abs(e1 - e0) / max(abs(e1), 1e-300)
                        done = de < tol
                        e0 = e1
                        if sim.t % 10000 == 0 or done:
                            print("%s: %s step %d dE/E %.3e" % (name, k, sim.t, de),
                                  file=sys.stderr, flush=True)
            except Exception as ex:  # unstable
                print("%s: %s failed: %s" % (name, k, ex), file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            rungs.append({"storage": k,
                          "until": "%s < %g" % ({"r": "R", "e": "dE/E per %d" % window}[crit], tol),
                          "until_step": int(sim.t), "wall_s": round(time.perf_counter() - t1, 2)})
            if not done:
                ok = False
                break
            prev = sim
        wall = time.perf_counter() - t0
        e = {"ladder": name, "gamma": gamma, "reached": ok,
             "steps": int(sims[-1].t) if ok else -1, "wall_s": round(wall, 2), "rungs": rungs}
        if ok:
            _, u, _ = sims[-1].moments("f64")
            ux = u[0].cpu().numpy()
            if u_ref is None:
                u_ref = ux
            e["u_rel_L2_vs_first"] = float(np.linalg.norm(ux - u_ref) / np.linalg.norm(u_ref))
            del u
        for sim in sims:
            sim.close()
        del sims, prev
        torch.cuda.empty_cache()
        out["ladders"].append(e)
        print(json.dumps(e), file=sys.stderr, flush=True)
    base = out["ladders"][0]["wall_s"]
    for e in out["ladders"]:
        if e["reached"]:
            e["speedup_vs_first"] = round(base / e["wall_s"], 3)
    return out


def run_ladders(probe, shape, ladders, window, workload):
    print(json.dumps({"probe": probe, **ladder_results(shape, ladders, window, workload)}),
          flush=True)


LADDERS_128 = [
    (1.0, (("f64", "r", 1e-8),)),
    (0.1, (("f64", "r", 1e-8),)),
    (0.1, (("f32", "r", 2e-7), ("f64", "r", 1e-8))),
    (0.1, (("f16_sr", "e", 1e-5), ("f32", "r", 2e-7), ("f64", "r", 1e-8))),
]


def time_to_residual_block():
    """The metric's second half: wall time (and steps) to a residual of 1e-8
    with gamma < 1 and with reduced-precision storage, against plain FP64 at
    gamma = 1 on the same lattice.  The 256^3 headline lattice runs at
    gamma = 1 only (Ma ~ 0.16 there), so the gamma comparison is made on the
    64^3 duct (same force, Ma ~ 0.01) and on the 128^3 duct."""
    shape = (64, 64, 64)
    rows = [time_to_residual(shape, "f64", g, 1e-8, 400000) for g in (1.0, 0.5, 0.1, 0.05)]
    ref = rows[0]
    for e in rows[1:]:
        if ref["steps"] > 0 and e["steps"] > 0:
            e["step_ratio_vs_f64_gamma1"] = round(ref["steps"] / e["steps"], 2)
            e["wall_ratio_vs_f64_gamma1"] = round(ref["wall_s"] / e["wall_s"], 2)
    mixed = [time_to_residual_mixed(shape, g, 1e-8, 1e-6, 400000) for g in (1.0, 0.1)]
    for e in mixed:
        if ref["steps"] > 0 and e["steps"] > 0:
            e["wall_ratio_vs_f64_gamma1"] = round(ref["wall_s"] / e["wall_s"], 2)
    lad = ladder_results((128, 128, 128), LADDERS_128, 100,
                         "square duct 128^3, nu = 0.131, same force; residual 1e-8; 16-bit "
                         "rungs end on the relative change of sum |u|^2 per 100 steps")
    for e in lad["ladders"]:
        e["wall_ratio_vs_f64_gamma1"] = e.pop("speedup_vs_first", None)
        e["u_rel_L2_vs_f64_gamma1"] = e.pop("u_rel_L2_vs_first", None)
    return {"tol": 1e-8,
            "reference": "plain FP64 storage at gamma = 1 on the same GPU, lattice and force",
            "duct64_f64_gamma_sweep": rows,
            "duct64_f32_then_f64": mixed,
            "duct128_ladders": lad,
            "paper_context": "Sec. 5: for its low-viscosity plane Poiseuille case the paper "
                             "reports more than two orders of magnitude fewer steps at "
                             "gamma = 0.001 than at gamma = 1, and several-fold to one-two "
                             "orders of magnitude reductions across its problems; it gives "
                             "no wall times and no hardware (bench.py --extras runs that "
                             "case: paper_poiseuille)."}


def ladder_256():
    """The 256^3 duct of precision_steady_256 (gamma = 1): FP64 alone, FP32
    then FP64, and BF16 / FP16 rungs (nearest and stochastic rounding) before
    them, the 16-bit rungs ended on the energy change per 1000 steps."""
    r64, r32 = ("f64", "r", 1e-8), ("f32", "r", 2e-7)
    run_ladders("ladder256", (256, 256, 256), [
        (1.0, (r64,)),
        (1.0, (r32, r64)),
        (1.0, (("bf16_sr", "e", 1e-4), r32, r64)),
        (1.0, (("bf16_sr", "e", 1e-5), r32, r64)),
        (1.0, (("bf16", "e", 1e-4), r32, r64)),
        (1.0, (("f16_sr", "e", 1e-5), r32, r64)),
        (1.0, (("f16_sr", "e", 1e-6), r32, r64)),
    ], 1000, "square duct 256^3, gamma = 1, nu = 0.131, C1 force; residual 1e-8")


def ladder_128():
    """The 128^3 duct (C1 force, nu = 0.131): preconditioning and precision
    ladders together.  FP64 at gamma = 1 and 0.1, then at gamma = 0.1 FP32
    then FP64, and an FP16 rung with stochastic rounding before them (energy
    change per 100 steps: the preconditioned march settles in a few thousand
    steps)."""
    r64, r32 = ("f64", "r", 1e-8), ("f32", "r", 2e-7)
    run_ladders("ladder128", (128, 128, 128), [
        (1.0, (r64,)),
        (0.1, (r64,)),
        (0.1, (r32, r64)),
        (0.1, (("f16_sr", "e", 1e-5), r32, r64)),
        (0.1, (("f16_sr", "e", 1e-6), r32, r64)),
    ], 100, "square duct 128^3, nu = 0.131, C1 force; residual 1e-8")


def oracle_time_to_steady(budget_s=900.0):
    """The FP64 oracle (numpy, on the host) marched to R < 1e-8 where that is
    tractable: the 64^3 duct (nu = 0.131, its force) at gamma = 0.1, 0.05 and
    1, and the coupled Hartmann channel 32 x 32 x 128 (Ha = 10, Pm = 0.01,
    gamma = gamma_m = 0.1), each beside the FP64 GPU march of the same case,
    whose crossing step it must equal (both check the residual every 10 steps).
    The oracle's time for a case is estimated from three timed steps and the
    GPU's step count; a case that would not fit in what is left of budget_s is
    skipped and says so.  Progress goes to stderr every 500 steps."""
    import numpy as np

    import paper_0809_4730_amd as pkg
    from oracle import glbe, mhd
    from paper_0809_4730_amd import inputs
    tol = 1e-8
    d = inputs.DUCT64
    h = inputs.HARTMANN
    B0, chi = inputs.hartmann_parameters(10.0, 0.01, h["shape"][1], h["nu"], h["eta"])
    mag = dict(gamma_m=0.1, chi=chi, eta=h["eta"], B0=(0.0, B0, 0.0))

    def duct(g):
        F = inputs.duct_force(d["shape"], d["F0"])
        return ("64^3 duct, gamma %g" % g,
                lambda: make_sim(d["shape"], "f64", g, nu=d["nu"], F0=d["F0"], bc=d["bc"]),
                lambda: glbe.Flow(d["shape"], d["bc"], F, g, glbe.rates(d["nu"], g)),
                d["shape"])

    def hartmann():
        g = 0.1
        return ("Hartmann 32x32x128, Ha 10, Pm 0.01, gamma = gamma_m = 0.1",
                lambda: pkg.Simulation(h["shape"], h["bc"], g, pkg.default_rates(h["nu"], g),
                                       storage="f64", force=h["F"], mhd=mag),
                lambda: mhd.MHDFlow(h["shape"], h["bc"], np.array(h["F"]), g,
                                    glbe.rates(h["nu"], g), mag["gamma_m"], chi, h["eta"],
                                    mag["B0"]),
                h["shape"])

    t_start = time.perf_counter()
    cases = []
    for name, gpu, cpu, shape in (duct(0.1), duct(0.05), hartmann(), duct(1.0)):
        nodes = shape[0] * shape[1] * shape[2]
        ge = time_to_residual(None, "f64", None, tol, 400000, make=gpu)
        e = {"case": name, "gpu_steps": ge["steps"], "gpu_wall_s": ge["wall_s"]}
        fl = cpu()
        t0 = time.perf_counter()
        fl.step(3, check_every=10 ** 9)
        t_step = (time.perf_counter() - t0) / 3
        fl = cpu()
        est = t_step * ge["steps"]
        left = budget_s - (time.perf_counter() - t_start)
        e["oracle_s_per_step"] = round(t_step, 4)
        e["oracle_MLUPS"] = round(nodes / t_step / 1e6, 3)
        if ge["steps"] <= 0 or est > left:
            e["oracle"] = "skipped: estimated %.0f s, %.0f s of the budget left" % (est, left)
            cases.append(e)
            print(json.dumps(e), file=sys.stderr, flush=True)
            continue
        t0 = time.perf_counter()
        reached = False
        while not reached and fl.t < 400000:
            reached = fl.run_to(tol, fl.t + 500)
            print("%s: oracle step %d, R %.3e" % (name, fl.t, fl.history[-1][1] if fl.history
                                                  else float("nan")), file=sys.stderr, flush=True)
        e["oracle_steps"] = fl.t if reached else -1
        e["oracle_wall_s"] = round(time.perf_counter() - t0, 2)
        e["steps_equal"] = e["oracle_steps"] == ge["steps"]
        e["gpu_speedup_wall"] = round(e["oracle_wall_s"] / ge["wall_s"], 1)
        cases.append(e)
        print(json.dumps(e), file=sys.stderr, flush=True)
    from threadpoolctl import threadpool_info
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"probe": "oracle_steady", "tol": tol, "os_cpu_count": os.cpu_count(),
            "blas_threads": int(threads), "cases": cases}


def shard_shares(launches=40):
    """One GPU's share of the 256^3 lattice when it is split into z-slabs over
    k = 1, 2, 4, 8 GPUs: the plain step kernel on a 256 x 256 x (256/k) slab,
    z periodic standing in for the halo planes a neighbour would fill, in the
    slab's own automatic launch shape; FP32 flow step (walls in y) and FP32
    coupled step (the Hartmann setting).  Median of `launches` launches (a HIP
    event on each, timed end to end), after 5 warm-up steps."""
    import numpy as np
    import torch

    import paper_0809_4730_amd as pkg
    from paper_0809_4730_amd import inputs
    h = inputs.HARTMANN
    B0, chi = inputs.hartmann_parameters(10.0, 0.01, h["shape"][1], h["nu"], h["eta"])
    bc = ("periodic", "wall", "periodic")
    rows = []
    for k in (1, 2, 4, 8):
        shape = (256, 256, 256 // k)
        for kind in ("flow", "coupled"):
            if kind == "flow":
                sim = make_sim(shape, "f32", 1.0, bc=bc, check_every=NO_CHECK)
                bpn = 164
            else:
                sim = pkg.Simulation(shape, bc, 0.1, pkg.default_rates(h["nu"], 0.1), storage="f32",
                                     force=h["F"], check_every=NO_CHECK,
                                     mhd=dict(gamma_m=0.1, chi=chi, eta=h["eta"], B0=(0.0, B0, 0.0)))
                bpn = 320
            sim.step(5)
            t, _ = sim.step_times(launches)
            us = float(np.median(t))
            rows.append({"gpus": k, "slab": list(shape), "step": kind, "kernel_us": round(us, 2),
                         "alg_GBs": round(bpn * sim.N / (us * 1e-6) / 1e9, 1),
                         "launch": sim.launch})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            sim.close()
            del sim
            torch.cuda.empty_cache()
    return {"probe": "shares", "rows": rows}


def kernel_probe(name, launches, copy_probe, launch=None):
    """One JSON line for the profilers: `launches` plain launches of one
    kernel at its HBM-scale size (coupled step 256^3 FP32, steady adjoint
    128^3 FP32, D2Q9 step 4096^2 FP32), timed with HIP events, with its
    algorithmic bytes per launch; optionally the calibration copy."""
    import torch

    import paper_0809_4730_amd as pkg
    from paper_0809_4730_amd import inputs
    if name == "mhd256":
        cfg = inputs.HARTMANN
        B0, chi = inputs.hartmann_parameters(10.0, 0.01, cfg["shape"][1], cfg["nu"], cfg["eta"])
        sim = pkg.Simulation((256, 256, 256), cfg["bc"], 0.1, pkg.default_rates(cfg["nu"], 0.1),
                             storage="f32", force=cfg["F"], check_every=NO_CHECK, launch=launch,
                             mhd=dict(gamma_m=0.1, chi=chi, eta=cfg["eta"], B0=(0.0, B0, 0.0)))
        us = kernel_time_us(sim, launches, warmup=5)
        alg = 2 * (19 + 21) * 4 * sim.N
        kernel = "mhd_step<float, check=false, field=false> (256^3)"
    elif name == "adjoint128":
        cfg = inputs.ADJOINT
        sim = make_sim(cfg["shape"], "f32", 0.1)
        sim.step(200)
        sim.adjoint_steady(tol=1e-30, max_iter=20)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.adjoint_steady(tol=1e-30, max_iter=launches)
        torch.cuda.synchronize()
        us = 1e6 * (time.perf_counter() - t0) / launches
        alg = (3 * 19 * 4 + 12) * sim.N  # mu in/out and the forward state; force
        kernel = "adjoint_step<float> (128^3, iterations with their gradient checks)"
    elif name == "d2q9_4096":
        sim = pkg.Simulation((4096, 4096, 1), ("periodic", "wall", "periodic"), 0.1,
                             pkg.default_rates_d2q9(0.1, 0.1), storage="f32", force=(1e-7, 0.0),
                             check_every=NO_CHECK, lattice="d2q9", launch=launch)
        us = kernel_time_us(sim, launches, warmup=5)
        alg = 2 * 9 * 4 * sim.N
        kernel = "glbe2_step<float, check=false> (4096^2)"
    elif name == "hbm_ceiling":
        print(json.dumps({"probe": name, **hbm_ceiling(reps=launches)}), flush=True)
        return
    elif name == "oracle_steady":
        print(json.dumps(oracle_time_to_steady()), flush=True)
        return
    elif name == "shares":
        print(json.dumps(shard_shares(launches)), flush=True)
        return
    elif name == "precision256":
        precision_steady_256()
        return
    elif name == "ladder256":
        ladder_256()
        return
    elif name == "ladder128":
        ladder_128()
        return
    else:
        raise SystemExit("unknown probe %s" % name)
    sim.close()
    line = {"probe": name, "kernel": kernel, "launches": launches, "kernel_us": round(us, 3),
            "alg_bytes_per_launch": alg, "achieved_GBs": round(alg / (us * 1e-6) / 1e9, 1),
            "kernel_hash": kernel_hash()}
    if copy_probe:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = src.numel() * 4
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--big-steps", type=int, default=100)
    ap.add_argument("--extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttr", action="store_true", help="skip the time-to-residual block")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline workload alone (profiler runs)")
    ap.add_argument("--grid", type=int, default=256, help="cube edge of the duct (256 = headline)")
    ap.add_argument("--gamma", type=float, default=None,
                    help="preconditioning parameter (default: 1 at 256^3, 0.1 below)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "bf16", "f16"])
    ap.add_argument("--rounding", default="nearest", choices=["nearest", "stochastic"],
                    help="rounding of 16-bit stores (stochastic: bf16 / f16 only)")
    ap.add_argument("--xcd-chunk", type=int, default=0,
                    help="fix the XCD workgroup chunk (0: the library's create-time choice)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--probe", choices=["mhd256", "adjoint128", "d2q9_4096", "precision256",
                                        "ladder256", "ladder128", "hbm_ceiling", "oracle_steady",
                                        "shares"],
                    help="only one other measurement: another kernel at HBM scale (for the "
                         "profilers), or the 256^3 precision form at steady state")
    ap.add_argument("--launches", type=int, default=30)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library and this benchmark have no "
              "multi-GPU path (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    import paper_0809_4730_amd as pkg
    pkg.load_library()
    if args.probe:
        kernel_probe(args.probe, args.launches, args.copy_probe,
                     {"xcd_chunk": args.xcd_chunk} if args.xcd_chunk else None)
        return

    shape, storage = (args.grid,) * 3, args.storage
    gamma = args.gamma if args.gamma is not None else (1.0 if args.grid >= 256 else 0.1)
    if args.rounding == "stochastic" and storage not in ("bf16", "f16"):
        raise SystemExit("--rounding stochastic needs --storage bf16 or f16")
    kw = {"rounding": "stochastic"} if args.rounding == "stochastic" else {}
    if args.xcd_chunk:
        kw["launch"] = {"xcd_chunk": args.xcd_chunk}
    print("headline: duct %s %s gamma=%g, %d + %d steps" % (shape, storage, gamma, args.warmup,
                                                            args.steps), file=sys.stderr,
          flush=True)
    head = step_roofline(shape, storage, gamma, args.steps, args.warmup, **kw)
    khash = kernel_hash()
    tag = "glbe_step_%s%s_duct%d" % (storage, "_sr" if args.rounding == "stochastic" else "",
                                     args.grid)
    traffic = traffic_from_profiles(tag, khash)
    # the library keeps cacheable loads for a force field that fits in 80% of
    # the 256 MB last-level cache (documented at lbm_create); its bytes are then
    # served from that cache, and only the populations must cross HBM
    cb = 8 if storage == "f64" else 4
    N_nodes = shape[0] * shape[1] * shape[2]
    force_fits = 3 * cb * N_nodes <= 0.8 * MALL_BYTES
    force_policy = ("cacheable: the field (%d MB) fits in the last-level cache"
                    if force_fits else "streaming: the field (%d MB) exceeds the last-level cache") \
        % (3 * cb * N_nodes // 10 ** 6)
    pop_only_gbs = 2 * 19 * STORAGE_BYTES[storage] * N_nodes / (head["kernel_us"] * 1e-6) / 1e9
    line = {
        "metric": METRIC,
        "value": head["MLUPS"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": storage,
        "data": "synthetic",
        "config": {"workload": "square duct %dx%dx%d, D3Q19 preconditioned MRT-GLBE, "
                               "force F_x=F0 sin(2 pi y/Ly)(1+cos(2 pi z/Lz)/2), F0=1e-5, "
                               "nu=0.131, gamma=%g, %s deviation storage%s, FP32 collision, "
                               "FP64 residual, mass and flow rate every 10 steps"
                               % (shape + (gamma, storage.upper(),
                                           " (stochastic rounding)" if kw.get("rounding") else "")),
                   "grid": list(shape), "gamma": gamma, "storage": storage,
                   "rounding": args.rounding, "launch": head["launch"]},
        "roofline": {"bound": head["bound"], "achieved": head["achieved_GBs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": head["frac"],
                     "traffic": traffic,
                     "frac_counter_traffic": (round(traffic / (head["kernel_us"] * 1e-6) / 1e9
                                                    / HBM_PEAK_GBS, 4) if traffic else None),
                     "force_field_loads": force_policy,
                     "frac_populations_only": round(pop_only_gbs / HBM_PEAK_GBS, 4),
                     "traffic_source": "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of this kernel "
                                       "in profiles/traffic.json, used only when taken on the "
                                       "current kernel sources (kernel_hash), else null",
                     "kernel": "glbe_step<%s, check=false, field=true%s>"
                               % (storage, ", stochastic" if kw.get("rounding") else ""),
                     "timing": "HIP events on the dispatches of the timed steps "
                               "(hipExtLaunchKernel), on the library's stream; mean over the "
                               "%d plain launches of the time from the previous step "
                               "kernel's end to each one's end"
                               % head["launches_timed"],
                     "alg_bytes_per_node": head["alg_bytes_per_node"],
                     "alg_bytes_per_launch": head["alg_bytes_per_launch"],
                     "mean_kernel_us": head["kernel_us"],
                     "min_kernel_us": head["kernel_us_min"],
                     "max_kernel_us": head["kernel_us_max"],
                     "check_kernel_us": head["check_kernel_us"],
                     "kernel_hash": khash},
    }
    if args.copy_probe:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = src.numel() * 4
        del src, dst
    if not args.only_headline:
        print("hbm ceiling", file=sys.stderr, flush=True)
        ceil = hbm_ceiling()
        line["roofline"]["ceiling"] = ceil
        line["roofline"]["frac_of_step_pattern_copy"] = round(
            head["achieved_GBs"] / ceil["step_pattern_copy"]["GBs"], 4)
        line["roofline"]["frac_of_stream_copy"] = round(
            head["achieved_GBs"] / ceil["stream_copy"]["GBs"], 4)
        line["roofline"]["frac_of_exact_pattern_copy"] = round(
            head["achieved_GBs"] / ceil["step_exact_copy"]["GBs"], 4)
        per = []
        for st in [x for x in ("bf16", "f16", "f64") if x != storage]:
            print("storage %s" % st, file=sys.stderr, flush=True)
            e = step_roofline(shape, st, gamma, args.steps, args.warmup)
            e.pop("wall_s")
            per.append(e)
        line["other_storage"] = per
        print("64^3 duct (cache-resident)", file=sys.stderr, flush=True)
        line["duct64_f32_gamma0.1"] = small_duct_line(max(args.steps, 1000), args.warmup)
        print("coupled step 256^3", file=sys.stderr, flush=True)
        mhd = mhd256_line(args.steps, args.warmup)
        mhd["frac_of_coupled_pattern_copy"] = round(
            mhd["achieved_GBs"] / ceil["coupled_pattern_copy"]["GBs"], 4)
        mhd["frac_of_exact_pattern_copy"] = round(
            mhd["achieved_GBs"] / ceil["coupled_exact_copy"]["GBs"], 4)
        line["mhd256_f32"] = mhd
        if not args.no_ttr:
            print("time to residual", file=sys.stderr, flush=True)
            line["time_to_residual"] = time_to_residual_block()
    if not args.no_cpu:
        print("cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline()
    if args.extras:
        line["extras"] = extras(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
