"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/host_fuzz/fuzz_mesh.cpp drives p1e_mesh_create / p1e_mesh_get_info /
p1e_workspace_bytes / p1e_material_constants with random valid and corrupted meshes of every
kind, linked against the host sources (p1e_api.cpp, p1e_tiles.cpp) compiled with g++ and the
sanitizers, and stand-ins for the kernel launchers (no GPU code is built or run). Any
sanitizer report or failed check fails the test.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2109_01158_amd", "csrc")
ROCM = "/opt/rocm"


@pytest.mark.timeout(600)
def test_mesh_setup_fuzz_under_sanitizers(tmp_path):
    if shutil.which("g++") is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("needs g++ and the HIP headers")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__",
             "-I" + os.path.join(ROCM, "include"), "-I" + CSRC, "-I" + os.path.join(ROOT, "include")]
    srcs = [os.path.join(CSRC, "p1e_api.cpp"), os.path.join(CSRC, "p1e_tiles.cpp"),
            os.path.join(HERE, "host_fuzz", "launcher_stubs.cpp"),
            os.path.join(HERE, "host_fuzz", "fuzz_mesh.cpp")]
    exe = str(tmp_path / "fuzz_mesh")
    subprocess.run(["g++"] + flags + srcs + ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
                                             "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, "1500"], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "0 failed checks" in out


@pytest.mark.timeout(300)
def test_admission_with_a_fake_executor(tmp_path):
    """The serving loop's admission bookkeeping (p1e_admission.h, as p1e_server_step uses it)
    under a fake executor: Poisson arrivals, log-uniform sizes, first-fit pool bytes and slots;
    invariants at every step, FIFO admission, and (one slot) the latency percentiles of the
    single-server queue recursion (tests/host_fuzz/sim_admission.cpp)."""
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = str(tmp_path / "sim_admission")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-I" + CSRC,
                    os.path.join(HERE, "host_fuzz", "sim_admission.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "0 failed checks" in out
