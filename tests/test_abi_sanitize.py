"""The C ABI layer (ttt_abi.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the host: ttt_abi.cpp is compiled with both
sanitizers for the host only and linked, with the kernels' objects (the
library build's own, when they are newer than every source), into
tests/abi_sanitize_driver.cpp, which drives argument validation, workspace
sizing and the empty-stream paths.  No GPU is touched."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_08542_amd", "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def hipcc():
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not found")


def test_abi_under_asan_ubsan(tmp_path):
    cc = hipcc()
    clang = os.path.join(os.path.dirname(os.path.realpath(cc)), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    base = ["-std=c++17", "-O1", "-fPIC", "-w"]
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    newest = max(os.path.getmtime(f) for f in glob.glob(os.path.join(CSRC, "*")))

    def kernel_obj(src):
        built = os.path.join(ROOT, "_build", os.path.basename(src) + ".o")
        if os.path.exists(built) and os.path.getmtime(built) >= newest:
            return built
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        from paper_2604_08542_amd.build import FLAGS
        subprocess.run([cc] + [f for f in FLAGS if f not in ("-Wall", "-Werror")] + ["-w", "-c", "-o", obj, src],
                       check=True, capture_output=True, timeout=600)
        return obj
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(kernel_obj, srcs))
    abi = str(tmp_path / "ttt_abi.o")
    r = subprocess.run([cc, "-x", "hip", "--cuda-host-only"] + base + SAN +
                       ["-c", "-o", abi, os.path.join(CSRC, "ttt_abi.cpp")], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    drv = str(tmp_path / "driver.o")
    r = subprocess.run([clang, "-std=c++17", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-c",
                        "-o", drv, os.path.join(ROOT, "tests", "abi_sanitize_driver.cpp")], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    exe = str(tmp_path / "abi_sanitize")
    r = subprocess.run([clang, "-fsanitize=address,undefined", "-o", exe, drv, abi] + objs +
                       ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    print(out)
    assert r.returncode == 0, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
    assert "0 failure(s)" in out
