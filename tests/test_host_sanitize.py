"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): api.cpp (all host logic: planning, sizing, launch tables,
argument validation) is compiled with both sanitizers by the host compiler and
linked, with the library's other objects as built, into
tests/host_sanitize/driver.cpp, which exercises every host-only path of the
C-ABI.  The run must end with "ok" and no sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _objects():
    from paper_1511_07482_amd import build as kbuild
    objs = [os.path.join(BUILD, u + ".o") for u in kbuild.UNITS if u != "api.cpp"]
    if not all(os.path.exists(o) for o in objs):
        kbuild.build()
    return objs


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_code_under_asan_ubsan(tmp_path):
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    common = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
              f"-I{ROOT}/include"]
    api_o, drv_o, exe = tmp_path / "api.o", tmp_path / "driver.o", tmp_path / "kdefft_sanitize"
    subprocess.run(common + san + ["-ffp-contract=off", "-c", os.path.join(ROOT, "paper_1511_07482_amd", "csrc",
                                                                            "api.cpp"), "-o", str(api_o)],
                   check=True, capture_output=True, text=True)
    subprocess.run(common + san + ["-c", os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp"), "-o",
                                   str(drv_o)], check=True, capture_output=True, text=True)
    subprocess.run(["g++"] + san + [str(drv_o), str(api_o)] + _objects() +
                   [f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    # leaks are not checked (the HIP runtime keeps its state to process exit);
    # the sanitizer runtime need not come first among preloaded libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), p.stdout + p.stderr
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr
