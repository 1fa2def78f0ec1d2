"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
the library is built with both sanitizers on its host code only (the gfx950
device code is unchanged), and a C program built with the same sanitizers
drives the host-side paths -- rate tables, velocity sets, workspace sizes up to
lattices of nearly 2^31 nodes, argument validation of the entry points -- none
of which reaches a device call, so this runs without a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
# host-only sanitizer flags for hipcc: -Xarch_host before each one
HOST_SANITIZE = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                 "-Xarch_host -fno-sanitize-recover=undefined "
                 "-Xarch_host -fno-omit-frame-pointer").split()


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if not os.path.exists(CLANG) or not shutil.which("hipcc") and \
            not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("the ROCm toolchain is needed for the sanitized build")
    from paper_0809_4730_amd import build
    d = tmp_path_factory.mktemp("sanitized")
    lib = build.build(out=str(d / "liblbm_san.so"), extra_flags=HOST_SANITIZE)
    exe = str(d / "capi_host_check")
    cmd = [CLANG, "-std=c11", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "capi_host_check.c"),
           lib, "-Wl,-rpath," + str(d), "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_host_paths_are_clean_under_asan_and_ubsan(sanitized):
    env = dict(os.environ)
    # the HIP runtime keeps allocations to the end of the process
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sanitized], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
