"""The benchmark's command-line contract and bookkeeping, on the CPU."""
import importlib.util
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_07187_amd", "csrc")


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)  # module level only: constants and functions
    return mod


def _tile_names():
    """Step-kernel names the tile tables of the HIP sources produce."""
    names = set()
    f32 = open(os.path.join(CSRC, "si_f32_gemm.h")).read()
    for m in re.finditer(r"X\((\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),"
                         r"\s*(\d+)\)", f32):
        _, bm, bn, wm, wn, mb, bk, st, ks = m.groups()
        names.add(f"step_f32_{bm}x{bn}_w{wm}x{wn}_mfma{mb}_k{bk}_s{st}_a{ks}")
    b16 = open(os.path.join(CSRC, "si_step_bf16.hip")).read()
    for m in re.finditer(r"X\((\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+)\)",
                         b16):
        _, bm, bn, wm, wn, bk, st, pp = m.groups()
        names.add(f"step_bf16_{bm}x{bn}_w{wm}x{wn}_k{bk}_s{st}" + ("" if pp == "0" else f"_p{pp}"))
    return names


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert p.stdout == ""
    assert "one GPU" in p.stderr


def test_traffic_entries_name_existing_kernels():
    # A counter-measured traffic entry is keyed by the kernel it was taken
    # on; an entry whose kernel no longer exists could never be reported.
    bench = _bench_module()
    names = _tile_names()
    assert len(names) > 40
    forms = {"fp32"} | set(bench.FORMS) | {"bf16x_hiloj"}
    for (kernel, form, n, r), value in bench.MEASURED_TRAFFIC_BYTES.items():
        assert kernel in names, kernel
        assert form in forms, form
        assert kernel.startswith("step_f32_") == (form == "fp32"), (kernel, form)
        assert n >= 1 and r >= 1 and value > 0
    # the headline kernel's entry is present
    assert any(k[1] == "fp32" and (k[2], k[3]) == (bench.N, bench.R)
               for k in bench.MEASURED_TRAFFIC_BYTES)


def test_default_workload_constants():
    bench = _bench_module()
    assert (bench.N, bench.R, bench.ITERS) == (2000, 1024, 10000)
    # published MI355X peaks: FP32 and BF16 dense matrix rates, HBM
    assert (bench.PEAK_FP32_MFMA_TFLOPS, bench.PEAK_BF16_MFMA_TFLOPS) == (157.3, 2500.0)
    assert bench.PEAK_HBM_GBS == 8000.0
