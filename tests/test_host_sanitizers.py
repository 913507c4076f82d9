"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

1. The library
(not GPU): a build whose host objects carry both sanitizers (device code is
built as usual) runs tests/host_checks.cpp, the C ABI's device-free paths
(option validation, status strings, null-handle argument checks, mesh size
limits, the 3-D operators' argument checks).  The
instrumented build takes a few minutes, so the test runs only with
PF_SANITIZE=1 in the environment.
2. The 3-D kernels' host replay (every index the device grids compute),
quick enough for every run."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2209_07969_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(os.environ.get("PF_SANITIZE") != "1",
                    reason="set PF_SANITIZE=1 to build and run the sanitized host checks")
def test_c_abi_host_paths_under_asan_ubsan():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include")] + san
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for src in ("pf_solver.cpp", "pf_kernels.hip", "pf3d_kernels.hip"):
            obj = os.path.join(d, src + ".o")
            subprocess.run([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj], check=True)
            objs.append(obj)
        lib = os.path.join(d, "libphasefield_san.so")
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host",
                        "-fsanitize=address,undefined", *objs, "-o", lib], check=True)
        exe = os.path.join(d, "host_checks")
        subprocess.run([CLANG, "-std=c++17", "-g", "-fsanitize=address,undefined",
                        "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "host_checks.cpp"), "-L" + d,
                        "-lphasefield_san", "-Wl,-rpath," + d, "-o", exe], check=True)
        env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert out.returncode == 0, out.stdout + out.stderr
        assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr
        assert "host checks: ok" in out.stdout


def test_hex3d_replay_indices_under_asan_ubsan(tmp_path):
    """Every 3-D kernel's grid, replayed on the host with each array in a
    heap buffer of exactly its size, under AddressSanitizer: an index the
    device grid would compute outside a buffer is reported here, before any
    device run (tests/hex3d_asan_main.cpp).  Host-only build, a few seconds,
    so it is part of the default run."""
    if not os.path.exists(HIPCC):
        pytest.skip("ROCm compiler not found")
    exe = str(tmp_path / "hex3d_asan")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "--offload-host-only", "-O1",
                    "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address,undefined",
                    "-Xarch_host", "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "hex3d_asan_main.cpp"), "-o", exe], check=True)
    env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "AddressSanitizer" not in out.stderr and "runtime error" not in out.stderr
    assert "hex3d asan: ok" in out.stdout
