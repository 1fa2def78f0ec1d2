"""MI355X-native preconditioned generalized lattice Boltzmann equation with forcing.

Thin Python binding of the C ABI in ``include/lbm_capi.h`` (``liblbm.so``,
hand-written HIP kernels for gfx950).  This module only marshals arguments:
every step of the computation runs in the library's kernels.  PyTorch supplies
device memory (the workspace and the caller's buffers) and the HIP stream.

The library must be built (``paper_0809_4730_amd.build.build()``); if it is
missing, loading fails with an error instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

__all__ = ["Simulation", "default_rates", "lattice_velocities", "LbmError", "library_path",
           "run_ladder",
           "load_library", "F64", "F32", "BF16", "F16", "PERIODIC", "WALL"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbm.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
PERIODIC, WALL = 0, 1
_DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}
_STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOWS", -3: "LBM_EHIP", -4: "LBM_EUNSTABLE",
           -5: "LBM_ESTATE", -6: "LBM_EUNSUPPORTED"}


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("bc", ctypes.c_int32 * 3)]


class _Launch(ctypes.Structure):
    _fields_ = [("xcd_chunk", ctypes.c_int32), ("store", ctypes.c_int32),
                ("offsets", ctypes.c_int32), ("load", ctypes.c_int32),
                ("waves", ctypes.c_int32)]


_STORES = {"auto": 0, "cached": 1, "streaming": 2}


def _launch(launch):
    """lbm_launch from None or dict(xcd_chunk=int, store="auto"|"cached"|"streaming",
    load="auto"|"cached"|"streaming", offsets="auto"|"wide", waves=0|3..8)."""
    out = _Launch()
    if launch:
        unknown = set(launch) - {"xcd_chunk", "store", "offsets", "load", "waves"}
        if unknown:
            raise ValueError("unknown launch keys %s" % sorted(unknown))
        out.xcd_chunk = int(launch.get("xcd_chunk", 0))
        out.store = _STORES[launch.get("store", "auto")]
        out.offsets = {"auto": 0, "wide": 1}[launch.get("offsets", "auto")]
        out.load = _STORES[launch.get("load", "auto")]
        out.waves = int(launch.get("waves", 0))
    return out


class _Params(ctypes.Structure):
    _fields_ = [
        ("storage", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("s", ctypes.c_double * 19),
        ("rho0", ctypes.c_double),
        ("force_mode", ctypes.c_int32),
        ("force_const", ctypes.c_double * 3),
        ("mhd", ctypes.c_int32),
        ("gamma_m", ctypes.c_double),
        ("chi", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("B0", ctypes.c_double * 3),
        ("check_every", ctypes.c_int32),
        ("history_len", ctypes.c_int32),
        ("source_mode", ctypes.c_int32),
        ("wall_u", (ctypes.c_double * 3) * 6),
        ("mag_pad", ctypes.c_int32 * 3),
        ("lattice", ctypes.c_int32),
        ("rounding", ctypes.c_int32),
        ("seed", ctypes.c_uint32),
        ("launch", _Launch),
    ]


class _Member(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("s", ctypes.c_double * 19),
                ("force", ctypes.c_double * 3)]


class _MemberResult(ctypes.Structure):
    _fields_ = [("verdict", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("step", ctypes.c_int64), ("residual", ctypes.c_double)]


class _Record(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("step", "residual", "du2", "u2", "mass", "flow", "nonfinite", "reserved")]


_lib = None


def library_path():
    return _LIB_PATH


def load_library():
    """Load liblbm.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError("liblbm.so is not built (expected at %s); run "
                           "paper_0809_4730_amd.build.build()" % _LIB_PATH)
    # torch first: it ships its own HIP runtime, and liblbm.so must bind to that
    # one.  Loaded the other way round the process maps two HIP/HSA runtimes and
    # the second one finds no device.
    _torch()
    lib = ctypes.CDLL(_LIB_PATH)
    c_int32, c_int64, c_double, c_size_t, c_void_p = (ctypes.c_int32, ctypes.c_int64,
                                                      ctypes.c_double, ctypes.c_size_t,
                                                      ctypes.c_void_p)
    P = ctypes.POINTER
    sig = {
        "lbm_default_rates": [c_double, c_double, c_int32, c_double, P(c_double)],
        "lbm_default_rates_d2q9": [c_double, c_double, c_int32, c_double, P(c_double)],
        "lbm_batch_workspace_bytes": [P(_Grid), c_int32, c_int32, P(c_size_t)],
        "lbm_batch_run": [P(_Grid), c_int32, c_double, c_int32, P(_Member), c_void_p, c_size_t,
                          c_void_p, c_double, c_int64, c_int32, c_int64, P(_Launch),
                          P(_MemberResult)],
        "lbm_lattice_velocities": [c_int32, P(c_int32)],
        "lbm_bandwidth_probe": [c_int32, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                c_int32, c_int32, c_void_p],
        "lbm_workspace_bytes": [P(_Grid), P(_Params), P(c_size_t)],
        "lbm_create": [P(_Grid), P(_Params), c_void_p, c_void_p, c_size_t, c_void_p, P(c_void_p)],
        "lbm_set_force": [c_void_p, c_void_p],
        "lbm_step": [c_void_p, c_int64],
        "lbm_step_timed": [c_void_p, c_int64, P(c_double), P(c_double)],
        "lbm_step_times": [c_void_p, c_int64, P(c_double), P(c_double)],
        "lbm_residual": [c_void_p, P(c_double), P(c_int64)],
        "lbm_history": [c_void_p, P(_Record), c_int64, P(c_int64)],
        "lbm_run_to_residual": [c_void_p, c_double, c_int64, c_int64, P(c_int64), P(c_double)],
        "lbm_run_to_energy_change": [c_void_p, c_double, c_int64, c_int64, P(c_int64),
                                     P(c_double)],
        "lbm_reductions": [c_void_p, P(c_double), P(c_double)],
        "lbm_reductions_noalloc": [P(_Grid), P(_Params), c_void_p, c_void_p, c_void_p, c_void_p],
        "lbm_moments": [c_void_p, c_int32, c_void_p, c_void_p, c_void_p],
        "lbm_state_bytes": [c_void_p, P(c_size_t)],
        "lbm_get_state": [c_void_p, c_void_p],
        "lbm_set_state": [c_void_p, c_void_p, c_int64],
        "lbm_get_step": [c_void_p, P(c_int64)],
        "lbm_get_launch": [c_void_p, P(_Launch)],
        "lbm_convert_state": [c_void_p, c_void_p],
        "lbm_adjoint_workspace_bytes": [c_void_p, c_int32, c_int64, c_int64, P(c_size_t)],
        "lbm_adjoint_steady": [c_void_p, c_void_p, c_size_t, c_double, c_int64, c_void_p,
                               P(c_int64), P(c_double)],
        "lbm_adjoint_unrolled": [c_void_p, c_void_p, c_size_t, c_int64, c_int64, c_void_p],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c_int32
    lib.lbm_destroy.argtypes = [c_void_p]
    lib.lbm_destroy.restype = None
    lib.lbm_last_error.argtypes = [c_void_p]
    lib.lbm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status, ctx=None):
    if status != 0:
        lib = load_library()
        raise LbmError(status, lib.lbm_last_error(ctx).decode())


def default_rates(nu, gamma, mode="paper", Lambda=1.0):
    """Preconditioned D3Q19 rates (see lbm_default_rates)."""
    lib = load_library()
    out = (ctypes.c_double * 19)()
    _check(lib.lbm_default_rates(nu, gamma, 0 if mode == "paper" else 1, Lambda, out))
    return np.array(list(out))


def default_rates_d2q9(nu, gamma, mode="paper", Lambda=1.0):
    """Preconditioned D2Q9 rates (see lbm_default_rates_d2q9)."""
    lib = load_library()
    out = (ctypes.c_double * 9)()
    _check(lib.lbm_default_rates_d2q9(nu, gamma, 0 if mode == "paper" else 1, Lambda, out))
    return np.array(list(out))


def lattice_velocities(q=19):
    lib = load_library()
    out = (ctypes.c_int32 * (3 * q))()
    _check(lib.lbm_lattice_velocities(q, out))
    return np.array(list(out), dtype=np.int64).reshape(q, 3)


def bandwidth_probe(pattern, src, dst, shape, walls=(False, False, False), xcd_chunk=2, waves=8,
                    stream=None):
    """Enqueue one calibration copy (lbm_bandwidth_probe) between two float32
    device tensors of at least 22 * nodes (patterns 2 and 4: 40 * nodes)
    elements on `stream` (default: the current stream).  shape: (nx, ny, nz),
    or a node count (a 1 x 1 lattice row) for patterns 0-2; walls: per axis,
    for patterns 3 and 4.  Returns the bytes it moves."""
    torch = _torch()
    lib = load_library()
    nx, ny, nz = (int(shape), 1, 1) if np.ndim(shape) == 0 else (int(v) for v in shape)
    nodes = nx * ny * nz
    planes = 40 if pattern in (2, 4) else 22
    if src.numel() < planes * nodes or dst.numel() < planes * nodes \
            or src.dtype != torch.float32 or dst.dtype != torch.float32:
        raise ValueError("src and dst must be float32 tensors of at least %d * nodes elements"
                         % planes)
    mask = sum(1 << i for i, w in enumerate(walls) if w)
    if stream is None:
        stream = torch.cuda.current_stream(src.device)
    _check(lib.lbm_bandwidth_probe(int(pattern), src.data_ptr(), dst.data_ptr(), nx, ny, nz, mask,
                                   int(xcd_chunk), int(waves), stream.cuda_stream))
    return {0: 2 * 88, 1: 164, 2: 320, 3: 164, 4: 320}[int(pattern)] * nodes


VERDICTS = {0: "undecided", 1: "converged", 2: "unstable"}


def batch_run(shape, bc, members, storage="f64", rho0=1.0, tol=1e-9, max_steps=20000,
              check_every=10, poll_every=1000, device="cuda", stream=None, launch=None):
    """March independent lattices of one grid together (lbm_batch_run).

    members: sequence of (gamma, rates[19], force[3]).  launch: None or
    dict(offsets="wide") (see Simulation).  Returns a list of (verdict, step,
    last residual), verdict one of VERDICTS' values."""
    torch = _torch()
    lib = load_library()
    g = _Grid()
    for a in range(3):
        g.n[a] = int(shape[a])
        g.bc[a] = WALL if bc[a] in ("wall", WALL) else PERIODIC
    st = _DTYPES[storage] if isinstance(storage, str) else int(storage)
    count = len(members)
    arr = (_Member * count)()
    for i, (gamma, s, force) in enumerate(members):
        arr[i].gamma = float(gamma)
        for k in range(19):
            arr[i].s[k] = float(s[k])
        for a in range(3):
            arr[i].force[a] = float(force[a])
    nbytes = ctypes.c_size_t()
    _check(lib.lbm_batch_workspace_bytes(ctypes.byref(g), st, count, ctypes.byref(nbytes)))
    dev = torch.device(device)
    raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
    ptr = raw.data_ptr() + (-raw.data_ptr()) % 256
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    cur = torch.cuda.current_stream(dev)
    if stream != cur:  # the workspace was allocated on the current stream
        stream.wait_stream(cur)
        raw.record_stream(stream)
    res = (_MemberResult * count)()
    lp = _launch(launch)
    _check(lib.lbm_batch_run(ctypes.byref(g), st, float(rho0), count, arr, ptr, nbytes.value,
                             stream.cuda_stream, float(tol), int(max_steps), int(check_every),
                             int(poll_every), ctypes.byref(lp), res))
    del raw
    return [(VERDICTS[r.verdict], r.step, r.residual) for r in res]


def _torch():
    import torch
    return torch


def _state_torch_dtype(storage):
    torch = _torch()
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}[storage]


def _compute_torch_dtype(storage):
    torch = _torch()
    return torch.float64 if storage == F64 else torch.float32


class Simulation:
    """One lattice on one GPU.

    shape: (nx, ny, nz), x the unit-stride axis.  bc: three of "periodic"/"wall".
    s: 19 preconditioned rates (default_rates).  storage: "f64", "f32", "bf16", "f16".
    force: a 3-vector (uniform) or a device tensor (3, nz, ny, nx) in the compute
    dtype (float64 for f64 storage, float32 otherwise).
    mhd: None or dict(gamma_m=, chi=, eta=, B0=(..), mu=1.0, pad=(0, 0, 0)); pad > 0
         extends the induction lattice beyond the fluid box (shape is then the
         induction lattice, the fluid box is pad nodes in from each wall face).
    source: "precond" (P_S, the paper's form) or "naive" (S/gamma, its negative control).
    wall_u: None or (6, 3) face velocities (x-low, x-high, y-low, y-high, z-low, z-high).
    rounding: "nearest" or "stochastic" (bf16/f16 storage, flow step without mhd): how
              stored populations are rounded; seed: the stochastic rounding seed.
    launch: None (the library's choice) or dict(xcd_chunk=n, store="cached"|"streaming",
            load="cached"|"streaming", offsets="wide", waves=3..8): the launch shape
            (lbm_launch; results do not depend on it).
    """

    def __init__(self, shape, bc, gamma, s, storage="f32", force=(0.0, 0.0, 0.0), rho0=1.0,
                 mhd=None, check_every=10, history_len=4096, device="cuda", stream=None,
                 source="precond", wall_u=None, lattice="d3q19", rounding="nearest", seed=0,
                 launch=None):
        torch = _torch()
        self._lib = load_library()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.shape = tuple(int(v) for v in shape)
        self.lattice = {"d3q19": 0, "d2q9": 1}[lattice]
        self.q, self.qg = (9, (2, 5)) if self.lattice == 1 else (19, (3, 7))
        self.storage = _DTYPES[storage] if isinstance(storage, str) else int(storage)
        self._grid = _Grid()
        for a in range(3):
            self._grid.n[a] = self.shape[a]
            b = bc[a]
            self._grid.bc[a] = (WALL if b in ("wall", WALL) else PERIODIC)
        p = _Params()
        p.lattice = self.lattice
        p.storage = self.storage
        if rounding not in ("nearest", "stochastic"):
            raise ValueError("rounding must be 'nearest' or 'stochastic'")
        p.rounding = 1 if rounding == "stochastic" else 0
        p.seed = int(seed) & 0xFFFFFFFF
        p.launch = _launch(launch)
        p.gamma = gamma
        for k in range(len(s)):
            p.s[k] = float(s[k])
        p.rho0 = rho0
        self._force_tensor = None
        if torch.is_tensor(force):
            p.force_mode = 1
            nx, ny, nz = self.shape
            want = (3, nz, ny, nx)
            if tuple(force.shape) != want:
                raise ValueError("force field must have shape %s" % (want,))
            if force.dtype != _compute_torch_dtype(self.storage) or force.device != self.device:
                raise ValueError("force field must be a %s tensor on %s"
                                 % (_compute_torch_dtype(self.storage), self.device))
            self._force_tensor = force.contiguous()
        else:
            p.force_mode = 0
            for a in range(len(force)):
                p.force_const[a] = float(force[a])
        if mhd:
            p.mhd = 1
            p.gamma_m = mhd["gamma_m"]
            p.chi = mhd["chi"]
            p.eta = mhd["eta"]
            p.mu = mhd.get("mu", 1.0)
            for a in range(len(mhd["B0"])):
                p.B0[a] = float(mhd["B0"][a])
            for a in range(3):
                p.mag_pad[a] = int(mhd.get("pad", (0, 0, 0))[a])
        p.check_every = check_every
        p.history_len = history_len
        p.source_mode = {"precond": 0, "naive": 1}[source]
        if wall_u is not None:
            for f in range(6):
                for a in range(3):
                    p.wall_u[f][a] = float(wall_u[f][a])
        self._params = p
        self.gamma = gamma
        nbytes = ctypes.c_size_t()
        _check(self._lib.lbm_workspace_bytes(ctypes.byref(self._grid), ctypes.byref(p),
                                             ctypes.byref(nbytes)))
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = raw.data_ptr()
        off = (-base) % 256
        self._ws_raw = raw
        self._ws_ptr = base + off
        self._ws_bytes = nbytes.value
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._stream = stream
        # the library works on `stream`: the caching allocator must not hand this
        # memory out again before that stream's work on it has finished
        raw.record_stream(stream)
        self._enter()  # the force field was written on the caller's stream
        ctx = ctypes.c_void_p()
        fptr = self._force_tensor.data_ptr() if self._force_tensor is not None else None
        _check(self._lib.lbm_create(ctypes.byref(self._grid), ctypes.byref(p), fptr,
                                    self._ws_ptr, self._ws_bytes, stream.cuda_stream,
                                    ctypes.byref(ctx)))
        self._ctx = ctx
        self._leave(self._force_tensor)

    # ------------------------------------------------------------- streams
    # The library enqueues its work on self._stream, while the caller's tensors
    # are produced and consumed on torch's current stream.  Before a call that
    # reads or writes caller memory the library stream waits for the current
    # one (_enter); after it the current stream waits for the library's work
    # and every caller tensor the library touched is recorded on the library
    # stream, so that the caching allocator does not reuse it before that work
    # has run (_leave).  With stream=None both are the same stream and nothing
    # is added.
    def _enter(self):
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur != self._stream:
            self._stream.wait_stream(cur)

    def _leave(self, *tensors):
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur != self._stream:
            for t in tensors:
                if t is not None:
                    t.record_stream(self._stream)
            cur.wait_stream(self._stream)

    # ----------------------------------------------------------- lifetime
    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, status):
        _check(status, self._ctx)

    @property
    def N(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    # ------------------------------------------------------------- march
    def step(self, n=1):
        self._c(self._lib.lbm_step(self._ctx, int(n)))
        return self

    def step_timed(self, n):
        us, ms = ctypes.c_double(), ctypes.c_double()
        self._c(self._lib.lbm_step_timed(self._ctx, int(n), ctypes.byref(us), ctypes.byref(ms)))
        return us.value, ms.value

    def step_times(self, n):
        """n steps, each step kernel's launch on the library's stream carrying a
        HIP event (lbm_step_times): (numpy array of n step durations in us, each
        from the previous step kernel's end to its own, wall time of the call in
        ms).  Step i of the call is step self.t + i + 1."""
        buf = (ctypes.c_double * int(n))()
        ms = ctypes.c_double()
        self._c(self._lib.lbm_step_times(self._ctx, int(n), buf, ctypes.byref(ms)))
        return np.frombuffer(buf, dtype=np.float64).copy(), ms.value

    def residual(self):
        r, t = ctypes.c_double(), ctypes.c_int64()
        self._c(self._lib.lbm_residual(self._ctx, ctypes.byref(r), ctypes.byref(t)))
        return r.value, t.value

    def history(self, max_records=None):
        cap = self._params.history_len if max_records is None else int(max_records)
        buf = (_Record * cap)()
        n = ctypes.c_int64()
        self._c(self._lib.lbm_history(self._ctx, buf, cap, ctypes.byref(n)))
        return np.array([[getattr(buf[i], k) for k, _ in _Record._fields_]
                         for i in range(n.value)]).reshape(n.value, 8)

    def run_to_residual(self, tol, max_steps, poll_every=2000):
        steps, r = ctypes.c_int64(), ctypes.c_double()
        self._c(self._lib.lbm_run_to_residual(self._ctx, tol, int(max_steps), int(poll_every),
                                              ctypes.byref(steps), ctypes.byref(r)))
        return steps.value, r.value

    def run_to_energy_change(self, tol, max_steps, window=1000):
        """lbm_run_to_energy_change: march until the relative change of the
        kinetic-energy sum |u|^2 over `window` steps falls below tol (a test
        the rounding noise of 16-bit storage does not hold up, unlike R).
        Returns (step of the record where it did, or -1; last change)."""
        step, change = ctypes.c_int64(), ctypes.c_double()
        self._c(self._lib.lbm_run_to_energy_change(self._ctx, float(tol), int(max_steps),
                                                   int(window), ctypes.byref(step),
                                                   ctypes.byref(change)))
        return step.value, change.value

    @property
    def launch(self):
        """The launch shape in use: dict(xcd_chunk=, store="cached"|"streaming",
        offsets="narrow"|"wide") (lbm_get_launch)."""
        lp = _Launch()
        self._c(self._lib.lbm_get_launch(self._ctx, ctypes.byref(lp)))
        pol = {1: "cached", 2: "streaming"}
        return {"xcd_chunk": lp.xcd_chunk, "store": pol[lp.store], "load": pol[lp.load],
                "offsets": {0: "narrow", 1: "wide"}[lp.offsets], "waves": lp.waves}

    @property
    def t(self):
        s = ctypes.c_int64()
        self._c(self._lib.lbm_get_step(self._ctx, ctypes.byref(s)))
        return s.value

    # ------------------------------------------------------------ fields
    def reductions(self):
        m, q = ctypes.c_double(), ctypes.c_double()
        self._c(self._lib.lbm_reductions(self._ctx, ctypes.byref(m), ctypes.byref(q)))
        return m.value, q.value

    def reductions_noalloc(self, state, out):
        """lbm_reductions_noalloc on this simulation's grid, parameters and force
        for a state tensor (the layout of get_state): writes (mass drift, flow
        rate) into the FP64 device tensor `out` (2 elements) on the library's
        stream; allocates nothing."""
        torch = _torch()
        if not (out.dtype == torch.float64 and out.numel() >= 2 and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 tensor of 2 elements")
        state = state.contiguous()
        self._enter()
        fptr = self._force_tensor.data_ptr() if self._force_tensor is not None else None
        _check(self._lib.lbm_reductions_noalloc(ctypes.byref(self._grid), ctypes.byref(self._params),
                                                state.data_ptr(), fptr, self._stream.cuda_stream,
                                                out.data_ptr()))
        self._leave(state, out)
        return out

    def moments(self, dtype="f64"):
        """(rho, u, B) device tensors of the current state; B is None without mhd."""
        torch = _torch()
        nx, ny, nz = self.shape
        td = torch.float64 if dtype == "f64" else torch.float32
        rho = torch.empty((nz, ny, nx), dtype=td, device=self.device)
        u = torch.empty((3, nz, ny, nx), dtype=td, device=self.device)
        B = torch.empty((3, nz, ny, nx), dtype=td, device=self.device) if self._params.mhd else None
        self._enter()
        self._c(self._lib.lbm_moments(self._ctx, F64 if dtype == "f64" else F32, rho.data_ptr(),
                                      u.data_ptr(), B.data_ptr() if B is not None else None))
        self._leave(rho, u, B)
        return rho, u, B

    def set_force(self, force):
        force = force.contiguous()
        self._force_tensor = force
        self._enter()
        self._c(self._lib.lbm_set_force(self._ctx, force.data_ptr()))
        self._leave(force)

    # ------------------------------------------------------------- state
    def get_state(self):
        """Populations (q, nz, ny, nx) in the storage dtype (q = 19, or 9 for
        D2Q9), plus (mhd) the magnetic populations (3, 7, nz, ny, nx) (D2Q5:
        (2, 5, ...)); both as deviations from the rest state (f - w rho0,
        g - W B0)."""
        torch = _torch()
        nx, ny, nz = self.shape
        q, (gj, ga) = self.q, self.qg
        f = torch.empty((q, nz, ny, nx), dtype=_state_torch_dtype(self.storage), device=self.device)
        self._enter()
        if self._params.mhd:
            blob = torch.empty((q + gj * ga) * self.N * f.element_size(),
                               dtype=torch.uint8, device=self.device)
            self._c(self._lib.lbm_get_state(self._ctx, blob.data_ptr()))
            self._leave(blob)
            nf = q * self.N * f.element_size()
            f = blob[:nf].view(f.dtype).reshape(q, nz, ny, nx)
            g = blob[nf:].view(f.dtype).reshape(gj, ga, nz, ny, nx)
            return f, g
        self._c(self._lib.lbm_get_state(self._ctx, f.data_ptr()))
        self._leave(f)
        return f

    def set_state(self, f, g=None, step=0):
        torch = _torch()
        if self._params.mhd:
            if g is None:
                raise ValueError("mhd state needs g")
            blob = torch.cat([f.contiguous().view(torch.uint8).reshape(-1),
                              g.contiguous().view(torch.uint8).reshape(-1)])
            self._enter()
            self._c(self._lib.lbm_set_state(self._ctx, blob.data_ptr(), int(step)))
            self._leave(blob)
            return
        f = f.contiguous()
        if f.dtype != _state_torch_dtype(self.storage):
            raise ValueError("state dtype must be %s" % _state_torch_dtype(self.storage))
        self._enter()
        self._c(self._lib.lbm_set_state(self._ctx, f.data_ptr(), int(step)))
        self._leave(f)

    def convert_from(self, other):
        """Continue `other`'s march here: its current state converted to this
        simulation's storage type (lbm_convert_state), with its step counter."""
        self._c(self._lib.lbm_convert_state(self._ctx, other._ctx))

    # ----------------------------------------------------------- adjoint
    def _adj_ws(self, mode, n_steps=0, ckpt_every=1):
        torch = _torch()
        nbytes = ctypes.c_size_t()
        self._c(self._lib.lbm_adjoint_workspace_bytes(self._ctx, mode, int(n_steps),
                                                      int(ckpt_every), ctypes.byref(nbytes)))
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        return raw, raw.data_ptr() + off, nbytes.value

    def adjoint_steady(self, tol=1e-8, max_iter=10 ** 6):
        """dQ/dF (3, nz, ny, nx) of the steady flow rate at the current state."""
        torch = _torch()
        raw, ptr, nbytes = self._adj_ws(0)
        nx, ny, nz = self.shape
        grad = torch.empty((3, nz, ny, nx), dtype=_compute_torch_dtype(self.storage),
                           device=self.device)
        iters, change = ctypes.c_int64(), ctypes.c_double()
        self._enter()
        self._c(self._lib.lbm_adjoint_steady(self._ctx, ptr, nbytes, tol, int(max_iter),
                                             grad.data_ptr(), ctypes.byref(iters),
                                             ctypes.byref(change)))
        self._leave(raw, grad)
        del raw
        return grad, iters.value, change.value

    def adjoint_unrolled(self, n_steps, ckpt_every):
        """Advance n_steps and return dQ_N/dF (3, nz, ny, nx)."""
        torch = _torch()
        raw, ptr, nbytes = self._adj_ws(1, n_steps, ckpt_every)
        nx, ny, nz = self.shape
        grad = torch.empty((3, nz, ny, nx), dtype=_compute_torch_dtype(self.storage),
                           device=self.device)
        self._enter()
        self._c(self._lib.lbm_adjoint_unrolled(self._ctx, ptr, nbytes, int(n_steps),
                                               int(ckpt_every), grad.data_ptr()))
        self._leave(raw, grad)
        del raw
        return grad


def run_to_residual_mixed(lo, hi, tol, switch_tol, max_steps, poll_every=200):
    """March `lo` (cheaper storage, e.g. FP32) until its residual falls below
    switch_tol, continue the same state in `hi` (e.g. FP64: lbm_convert_state)
    and march it to tol.  Both must describe the same lattice, force and
    parameters.  Returns (steps to tol or -1, final residual); the step count is
    the total over both."""
    n_lo, _ = lo.run_to_residual(switch_tol, max_steps, poll_every)
    hi.convert_from(lo)
    return hi.run_to_residual(tol, max_steps, poll_every)


def run_ladder(rungs, max_steps, poll_every=1000):
    """March one flow through a ladder of storage precisions: each rung is
    (simulation, criterion, tol) with criterion "residual" (run_to_residual)
    or "energy" (run_to_energy_change, for 16-bit rungs whose rounding noise
    holds R up); each rung continues the previous rung's state on the device
    (convert_from).  All simulations must describe the same lattice, force and
    parameters.  Returns (step at which the last rung met its tol, or -1 if a
    rung did not within max_steps of its own; [(step, value) per rung])."""
    out, prev = [], None
    for sim, crit, tol in rungs:
        if prev is not None:
            sim.convert_from(prev)
        if crit == "residual":
            n, v = sim.run_to_residual(tol, max_steps, poll_every)
        elif crit == "energy":
            n, v = sim.run_to_energy_change(tol, max_steps, poll_every)
        else:
            raise ValueError("criterion must be 'residual' or 'energy'")
        out.append((n, v))
        if n < 0:
            return -1, out
        prev = sim
    return out[-1][0], out


# ------------------------------------------------------------- autograd ----
def _autograd():
    torch = _torch()

    class SteadyFlowRate(torch.autograd.Function):
        """Q(F): steady flow rate (1/nx) sum j_x for the force field F
        (3, nz, ny, nx); the backward pass is the steady adjoint."""

        @staticmethod
        def forward(ctx, F, cfg):
            shape, bc, gamma, s, storage, tol, max_steps, adj_tol = cfg
            sim = Simulation(shape, bc, gamma, s, storage=storage, force=F.detach().contiguous())
            steps, r = sim.run_to_residual(tol, max_steps)
            if steps < 0:
                sim.close()
                raise RuntimeError("steady state not reached in %d steps (residual %g)"
                                   % (max_steps, r))
            _, q = sim.reductions()
            ctx.sim, ctx.adj_tol = sim, adj_tol
            return torch.tensor(q, dtype=torch.float64, device=F.device)

        @staticmethod
        def backward(ctx, gq):
            grad, _, _ = ctx.sim.adjoint_steady(tol=ctx.adj_tol)
            ctx.sim.close()
            return (gq.to(grad.dtype) * grad), None

    class UnrolledFlowRate(torch.autograd.Function):
        """Q_N(F): flow rate after n_steps from rest; the backward pass is the
        checkpointed adjoint of the march."""

        @staticmethod
        def forward(ctx, F, cfg):
            shape, bc, gamma, s, storage, n_steps, ckpt_every = cfg
            Fc = F.detach().contiguous()
            sim = Simulation(shape, bc, gamma, s, storage=storage, force=Fc)
            sim.step(n_steps)
            _, q = sim.reductions()
            sim.close()
            ctx.cfg, ctx.F = cfg, Fc
            return torch.tensor(q, dtype=torch.float64, device=F.device)

        @staticmethod
        def backward(ctx, gq):
            shape, bc, gamma, s, storage, n_steps, ckpt_every = ctx.cfg
            sim = Simulation(shape, bc, gamma, s, storage=storage, force=ctx.F)
            grad = sim.adjoint_unrolled(n_steps, ckpt_every)
            sim.close()
            return (gq.to(grad.dtype) * grad), None

    return SteadyFlowRate, UnrolledFlowRate


def steady_flow_rate(F, shape, bc, gamma, s, storage="f32", tol=1e-8, max_steps=10 ** 6,
                     adj_tol=1e-7):
    """Differentiable steady flow rate Q(F) (torch.autograd): F is a device tensor
    (3, nz, ny, nx) in the compute dtype; the gradient comes from the library's
    steady adjoint (lbm_adjoint_steady)."""
    SteadyFlowRate, _ = _autograd()
    return SteadyFlowRate.apply(F, (tuple(shape), tuple(bc), gamma, tuple(s), storage, tol,
                                    max_steps, adj_tol))


def unrolled_flow_rate(F, shape, bc, gamma, s, n_steps, ckpt_every, storage="f32"):
    """Differentiable flow rate after n_steps from rest (torch.autograd); the
    gradient comes from the checkpointed adjoint (lbm_adjoint_unrolled)."""
    _, UnrolledFlowRate = _autograd()
    return UnrolledFlowRate.apply(F, (tuple(shape), tuple(bc), gamma, tuple(s), storage,
                                      int(n_steps), int(ckpt_every)))
