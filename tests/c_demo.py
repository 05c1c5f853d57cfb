"""Build tests/c_abi_demo.c, a C program that uses the library through its C
ABI only (HIP runtime for device memory, no Python or torch)."""
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_c_demo(out_path):
    """Compile and link the demo; returns (ok, message)."""
    from paper_2305_07187_amd import spring_ising as si
    if shutil.which("gcc") is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        return False, "gcc or the HIP headers are missing"
    if not os.path.exists(si.LIB_PATH):
        from paper_2305_07187_amd import build
        build.build(verbose=False)
    libdir = os.path.dirname(si.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-isystem", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c_abi_demo.c"), "-L", libdir, "-lspring_ising",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{libdir}",
           f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", str(out_path)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return r.returncode == 0, r.stderr
