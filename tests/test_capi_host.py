"""Host-side checks of the C ABI: the library builds and loads, exports every
entry point the header declares, and its validation and host helpers agree
with the paper (no kernel is launched here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import glbe
from oracle.lattice import E19, E7

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm_capi.h")


@pytest.fixture(scope="module")
def lib():
    import paper_0809_4730_amd as pkg
    if not os.path.exists(pkg.library_path()):
        from paper_0809_4730_amd import build
        build.build()
    return pkg.load_library()


def _declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_named_calls():
    names = _declared_symbols()
    for n in ("lbm_create", "lbm_step", "lbm_residual", "lbm_moments", "lbm_destroy",
              "lbm_reductions", "lbm_adjoint_steady", "lbm_adjoint_unrolled"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_symbols():
        assert hasattr(lib, name), name


def test_library_has_gfx950_code_only():
    import paper_0809_4730_amd as pkg
    blob = open(pkg.library_path(), "rb").read()
    assert b"gfx950" in blob
    for other in (b"gfx942", b"gfx90a", b"gfx1100"):
        assert other not in blob


@pytest.mark.parametrize("nu,gamma", [(0.1, 1.0), (0.131, 0.05), (0.004, 0.05)])
def test_default_rates_match_oracle(lib, nu, gamma):
    import paper_0809_4730_amd as pkg
    assert np.allclose(pkg.default_rates(nu, gamma), glbe.rates(nu, gamma), rtol=1e-15)
    assert np.allclose(pkg.default_rates(nu, gamma, "lambda", 0.3),
                       glbe.rates(nu, gamma, "lambda", 0.3), rtol=1e-15)


def test_lattice_velocities(lib):
    import paper_0809_4730_amd as pkg
    e19 = pkg.lattice_velocities(19)
    assert sorted(map(tuple, e19)) == sorted(map(tuple, E19))
    # opposite pairs are adjacent (the kernels rely on it)
    for a in range(1, 19, 2):
        assert tuple(e19[a]) == tuple(-e19[a + 1])
    e7 = pkg.lattice_velocities(7)
    assert sorted(map(tuple, e7)) == sorted(map(tuple, E7))


def _grid_params(pkg, **kw):
    g = pkg._Grid()
    for a, n in enumerate(kw.get("n", (8, 8, 8))):
        g.n[a] = n
        g.bc[a] = kw.get("bc", (0, 0, 1))[a]
    p = pkg._Params()
    p.storage = kw.get("storage", pkg.F32)
    p.gamma = kw.get("gamma", 0.5)
    for k, v in enumerate(glbe.rates(0.1, 0.5)):
        p.s[k] = v
    p.rho0 = 1.0
    p.force_mode = 0
    p.check_every = 10
    p.history_len = 16
    p.mhd = kw.get("mhd", 0)
    p.gamma_m, p.chi, p.eta, p.mu = 0.1, 0.01, 0.025, 1.0
    p.rounding = kw.get("rounding", 0)
    p.lattice = kw.get("lattice", 0)
    for k in ("xcd_chunk", "store", "offsets", "load", "waves"):
        setattr(p.launch, k, kw.get(k, 0))
    return g, p


@pytest.mark.parametrize("bad", [
    dict(gamma=0.0), dict(gamma=1.5), dict(n=(0, 4, 4)), dict(storage=7),
    dict(mhd=1, storage=2), dict(n=(2048, 2048, 1024)),
    # stochastic rounding: 16-bit storage and the flow step without mhd only
    dict(rounding=2, storage=2), dict(rounding=1, storage=1), dict(rounding=1, storage=0),
    dict(rounding=1, storage=2, mhd=1), dict(rounding=1, storage=0, lattice=1, n=(8, 8, 1)),
    # launch shape fields
    dict(xcd_chunk=-1), dict(store=3), dict(store=-1), dict(offsets=2), dict(load=3),
    dict(waves=2), dict(waves=9), dict(waves=-1),
])
def test_validation_rejects(lib, bad):
    import paper_0809_4730_amd as pkg
    g, p = _grid_params(pkg, **bad)
    nbytes = ctypes.c_size_t()
    st = lib.lbm_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nbytes))
    assert st == -1
    assert lib.lbm_last_error(None)


@pytest.mark.parametrize("storage", [2, 3])
@pytest.mark.parametrize("lattice,n", [(0, (8, 8, 8)), (1, (8, 8, 1))])
def test_validation_accepts_stochastic_16bit(lib, lattice, n, storage):
    import paper_0809_4730_amd as pkg
    g, p = _grid_params(pkg, rounding=1, storage=storage, lattice=lattice, n=n)
    p.seed = 0xFFFFFFFF
    nbytes = ctypes.c_size_t()
    assert lib.lbm_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nbytes)) == 0
    assert nbytes.value > 0


def test_rate_outside_interval_rejected(lib):
    import paper_0809_4730_amd as pkg
    g, p = _grid_params(pkg)
    p.s[9] = 2.0
    nbytes = ctypes.c_size_t()
    assert lib.lbm_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nbytes)) == -1
    assert b"s[9]" in lib.lbm_last_error(None)
    p.s[9] = 1.0
    p.s[3] = 5.0   # conserved moment: ignored
    assert lib.lbm_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nbytes)) == 0


def test_workspace_size_and_create_checks(lib):
    import paper_0809_4730_amd as pkg
    g, p = _grid_params(pkg, n=(64, 64, 64))
    nbytes = ctypes.c_size_t()
    assert lib.lbm_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nbytes)) == 0
    N = 64 ** 3
    # two FP32 population buffers, the FP32 velocity snapshot, and at most 16 MB
    # of per-check partial sums plus small records
    assert nbytes.value >= 2 * 19 * N * 4 + 3 * N * 4
    assert nbytes.value < 2 * 19 * N * 4 + 3 * N * 4 + (17 << 20)
    ctx = ctypes.c_void_p()
    # NULL workspace and misaligned workspace are rejected before any device call
    st = lib.lbm_create(ctypes.byref(g), ctypes.byref(p), None, None, nbytes.value, None,
                        ctypes.byref(ctx))
    assert st == -2 and not ctx.value
    st = lib.lbm_create(ctypes.byref(g), ctypes.byref(p), None, 0x1001, nbytes.value, None,
                        ctypes.byref(ctx))
    assert st == -2
    st = lib.lbm_create(ctypes.byref(g), ctypes.byref(p), None, 0x10000, nbytes.value - 1, None,
                        ctypes.byref(ctx))
    assert st == -2
    p.force_mode = 1
    st = lib.lbm_create(ctypes.byref(g), ctypes.byref(p), None, 0x10000, nbytes.value, None,
                        ctypes.byref(ctx))
    assert st == -1


def test_product_path_refuses_missing_library(monkeypatch, tmp_path):
    import paper_0809_4730_amd as pkg
    monkeypatch.setattr(pkg, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pkg, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        pkg.load_library()


def test_library_binds_to_torch_hip_runtime():
    """Loading liblbm.so maps exactly one HIP runtime (torch's), whatever was
    imported first; two runtimes in one process leave the second without a device."""
    import subprocess
    import sys
    code = ("import paper_0809_4730_amd as p; p.load_library(); "
            "m = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


@pytest.mark.parametrize("pad,mhd,bc,msg", [
    ((0, 2, 0), 0, (0, 1, 0), b"needs mhd"),
    ((2, 0, 0), 1, (0, 1, 0), b"wall axes"),
    ((0, 4, 0), 1, (0, 1, 0), b"no fluid"),
    ((0, -1, 0), 1, (0, 1, 0), b">= 0"),
])
def test_mag_pad_validation(lib, pad, mhd, bc, msg):
    import paper_0809_4730_amd as pkg
    g, p = _grid_params(pkg, n=(8, 8, 8), bc=bc, mhd=mhd, storage=pkg.F64)
    for a in range(3):
        p.mag_pad[a] = pad[a]
    nbytes = ctypes.c_size_t()
    assert lib.lbm_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nbytes)) == -1
    assert msg in lib.lbm_last_error(None)
    p.mag_pad[0], p.mag_pad[1], p.mag_pad[2] = 0, 3, 0
    p.mhd = 1
    g.bc[1] = 1
    assert lib.lbm_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nbytes)) == 0


@pytest.mark.parametrize("change,msg", [
    (dict(n=(8, 8, 2)), b"n[2] = 1"),
    (dict(B0z=0.1), b"B0[2]"),
    (dict(wall=True), b"moving walls"),
    (dict(lattice=2), b"lattice must be"),
])
def test_d2q9_validation(lib, change, msg):
    import paper_0809_4730_amd as pkg
    g, p = _grid_params(pkg, n=change.get("n", (8, 8, 1)), bc=(0, 1, 0), mhd=1, storage=pkg.F64)
    p.lattice = change.get("lattice", 1)
    for k, v in enumerate(pkg.default_rates_d2q9(0.1, 0.5)):
        p.s[k] = v
    for k in range(9, 19):
        p.s[k] = 5.0  # beyond the nine D2Q9 rates: ignored
    p.B0[2] = change.get("B0z", 0.0)
    if change.get("wall"):
        p.wall_u[3][0] = 0.01
    nbytes = ctypes.c_size_t()
    assert lib.lbm_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nbytes)) == -1
    assert msg in lib.lbm_last_error(None)


def test_d2q9_workspace_and_rates(lib):
    import paper_0809_4730_amd as pkg
    from oracle import d2q9
    g, p = _grid_params(pkg, n=(64, 32, 1), bc=(0, 1, 0), storage=pkg.F32)
    p.lattice = 1
    for k, v in enumerate(pkg.default_rates_d2q9(0.1, 0.5)):
        p.s[k] = v
    nbytes = ctypes.c_size_t()
    assert lib.lbm_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nbytes)) == 0
    N = 64 * 32
    assert nbytes.value >= 2 * 9 * N * 4 + 3 * N * 4
    assert nbytes.value < 2 * 19 * N * 4
    assert np.allclose(pkg.default_rates_d2q9(0.05, 0.2), d2q9.rates(0.05, 0.2), rtol=1e-15)
    assert np.allclose(pkg.default_rates_d2q9(0.05, 0.2, "lambda", 0.25),
                       d2q9.rates(0.05, 0.2, "lambda", 0.25), rtol=1e-15)
    e9 = pkg.lattice_velocities(9)
    assert sorted(map(tuple, e9[:, :2])) == sorted(map(tuple, d2q9.E9)) and not e9[:, 2].any()
    e5 = pkg.lattice_velocities(5)
    assert sorted(map(tuple, e5[:, :2])) == sorted(map(tuple, d2q9.E5))
    for a in range(1, 9, 2):
        assert tuple(e9[a]) == tuple(-e9[a + 1])


def test_batch_workspace_and_validation(lib):
    import paper_0809_4730_amd as pkg
    g = pkg._Grid()
    for a in range(3):
        g.n[a] = (4, 4, 64)[a]
        g.bc[a] = (0, 0, 1)[a]
    nbytes = ctypes.c_size_t()
    assert lib.lbm_batch_workspace_bytes(ctypes.byref(g), pkg.F64, 10, ctypes.byref(nbytes)) == 0
    # two population buffers and the snapshot per member (1024 nodes: 4 whole workgroups)
    assert nbytes.value >= 10 * 1024 * (2 * 19 * 8 + 3 * 8)
    assert lib.lbm_batch_workspace_bytes(ctypes.byref(g), 9, 10, ctypes.byref(nbytes)) == -1
    assert lib.lbm_batch_workspace_bytes(ctypes.byref(g), pkg.F64, 0, ctypes.byref(nbytes)) == -1
    members = (pkg._Member * 2)()
    for i in range(2):
        members[i].gamma = 0.5
        for k, v in enumerate(glbe.rates(0.1, 0.5)):
            members[i].s[k] = v
    members[1].s[9] = 2.5
    res = (pkg._MemberResult * 2)()
    st = lib.lbm_batch_run(ctypes.byref(g), pkg.F64, 1.0, 2, members, None, 0, None, 1e-9, 100, 10,
                           100, None, res)
    assert st == -1 and b"member 1" in lib.lbm_last_error(None)
    members[1].s[9] = 1.0
    bad = pkg._Launch()
    bad.offsets = 2
    st = lib.lbm_batch_run(ctypes.byref(g), pkg.F64, 1.0, 2, members, None, 0, None, 1e-9, 100, 10,
                           100, ctypes.byref(bad), res)
    assert st == -1 and b"offsets" in lib.lbm_last_error(None)
    st = lib.lbm_batch_run(ctypes.byref(g), pkg.F64, 1.0, 2, members, None, 0, None, 1e-9, 100, 10,
                           100, None, res)
    assert st == -2  # no workspace: rejected before any device call


@pytest.mark.parametrize("args,msg", [
    ((5, 16, 32, 64, 4, 4, 0, 2, 8), b"pattern"),
    ((1, 0, 32, 64, 4, 4, 0, 2, 8), b"non-null"),
    ((1, 16, 32, 0, 4, 4, 0, 2, 8), b"nx, ny, nz"),
    ((1, 16, 32, 1 << 12, 1 << 12, 1 << 8, 0, 2, 8), b"nodes"),
    ((1, 20, 32, 64, 4, 4, 0, 2, 8), b"aligned"),
    ((1, 16, 32, 64, 4, 4, 0, 2, 2), b"waves"),
    ((3, 16, 32, 64, 4, 4, 8, 2, 8), b"walls"),
    ((1, 16, 32, 64, 4, 4, 0, 0, 8), b"xcd_chunk"),
    ((3, 16, 32, 96, 4, 4, 0, 2, 8), b"multiple of 64"),
    ((4, 16, 32, 1024, 1024, 64, 0, 2, 8), b"2^32"),
])
def test_bandwidth_probe_validation(lib, args, msg):
    """Every rejected argument is caught before a launch (the pointers here
    are never dereferenced)."""
    pattern, src, dst, nx, ny, nz, walls, chunk, waves = args
    st = lib.lbm_bandwidth_probe(pattern, ctypes.c_void_p(src), ctypes.c_void_p(dst), nx, ny, nz,
                                 walls, chunk, waves, None)
    assert st == -1 and msg in lib.lbm_last_error(None), lib.lbm_last_error(None)


def test_ctypes_mirrors_match_the_c_header(tmp_path):
    """The binding's ctypes structures have the size and field offsets the C
    header gives them (compiled here as C99 by gcc)."""
    import shutil
    import subprocess

    import paper_0809_4730_amd as pkg
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    mirrors = {"lbm_grid": pkg._Grid, "lbm_params": pkg._Params, "lbm_record": pkg._Record,
               "lbm_launch": pkg._Launch,
               "lbm_member": pkg._Member, "lbm_member_result": pkg._MemberResult}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lbm_capi.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", include, str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.rsplit(" ", 1) for line in
               subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    for cname, py in mirrors.items():
        assert int(got["%s size" % cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got["%s.%s" % (cname, fname)]) == getattr(py, fname).offset, (cname, fname)
