"""The C-ABI host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

csrc/api.cpp and csrc/serve.cpp (the host side of the library: argument
checks, tile maps, arena, serving) are compiled with the sanitizers on their
host code only (hipcc, -Xarch_host), linked by the ROCm clang++ with the
kernel objects of the regular build and a driver (tests/sanitize/host_check.cpp) that calls the entry points needing no
GPU: random band and guarded tile maps with their invariants, argument
rejection, version, serving footprint.  The run must end with status 0 and
no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_02701_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2406_02701_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"   # the host compiler behind hipcc, whose sanitizer runtimes the objects need
KERNEL_OBJS = ["tiles.o", "factor.o", "solve.o", "order.o", "gemm.o", "laplace.o", "mala.o", "krylov.o"]
HOST_SAN = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer".split()
CXX_SAN = "-fsanitize=address,undefined -fno-omit-frame-pointer".split()


@pytest.mark.timeout(900)
def test_host_code_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc or the ROCm clang++ not available")
    objs = [os.path.join(BUILD, o) for o in KERNEL_OBJS]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("kernel objects not built (run __graft_entry__.build())")
    common = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}"]
    host = []
    for src in ("api.cpp", "serve.cpp"):
        out = str(tmp_path / (src + ".o"))
        r = subprocess.run([HIPCC, *common, *HOST_SAN, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        host.append(out)
    drv = str(tmp_path / "host_check.o")
    r = subprocess.run([CLANG, "-O1", "-g", "-std=c++17", *CXX_SAN, "-c",
                        os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"), "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "host_check")
    r = subprocess.run([CLANG, *CXX_SAN, drv, *host, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                        "-lrocprofiler-sdk-roctx", "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_sanitizer_flags_catch_a_planted_overflow(tmp_path):
    """The same compile and link flags report a heap overflow in a small
    host program (so a clean run above means the checks were active)."""
    if not os.path.exists(CLANG):
        pytest.skip("the ROCm clang++ is not available")
    src = tmp_path / "overflow.cpp"
    src.write_text("#include <vector>\nint main(int c, char**) { std::vector<int> v(4); return v.data()[3 + c]; }\n")
    exe = str(tmp_path / "overflow")
    r = subprocess.run([CLANG, "-O0", "-g", *CXX_SAN, str(src), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=60)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
