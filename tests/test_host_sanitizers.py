"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
on the CPU: the HIP sources are built with the host compilation instrumented
(device code as usual; nothing is launched), and
tests/host_sanitizer_driver.c exercises the paths that run without a GPU:
argument checks, error messages, the build id and the tile cache's file
parser on valid, malformed and oversized input."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"

pytestmark = pytest.mark.slow


def _have_tools():
    return os.path.exists(HIPCC) and os.path.exists(CLANG)


@pytest.mark.skipif(not _have_tools(), reason="hipcc / ROCm clang missing")
def test_host_paths_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "libspring_ising_san.so"
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2305_07187_amd", "csrc", "*.hip")))
    # sanitizers on the host compilation only (each flag behind -Xarch_host)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    common = ["-std=c++17", "--offload-arch=gfx950", "-fPIC", "-I", os.path.join(ROOT, "include"),
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              '-DSI_BUILD_ID="0123456789abcdef"']
    objs, procs = [], []
    for src in srcs:
        obj = tmp_path / (os.path.basename(src) + ".o")
        objs.append(str(obj))
        procs.append(subprocess.Popen([HIPCC, "-O1", "-g", "-c"] + common + san + [src, "-o", str(obj)],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        out, err = p.communicate(timeout=900)
        assert p.returncode == 0, err[-3000:]
    r = subprocess.run([HIPCC, "-shared", "--offload-arch=gfx950"] + san + objs + ["-o", str(lib)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = tmp_path / "driver"
    cmd = [CLANG, "-O1", "-g", "-std=c99", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host_sanitizer_driver.c"), "-L", str(tmp_path),
           "-lspring_ising_san", "-L", "/opt/rocm/lib", "-lamdhip64",
           f"-Wl,-rpath,{tmp_path}", "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    work = tmp_path / "files"
    work.mkdir()
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe), str(work)], capture_output=True, text=True, timeout=300,
                       env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
