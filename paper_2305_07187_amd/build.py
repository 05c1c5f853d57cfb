"""Build the HIP library libspring_ising.so in-tree for gfx950.

    python -m paper_2305_07187_amd.build

Every HIP source under csrc/ is compiled and linked into one shared library
next to this file.  Packed-FP32 instructions are disabled for all device
code (the target feature '-packed-fp32-ops').
"""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libspring_ising.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


BUILD_ID_MARKER = b"SI_BUILD_ID:"


def stamped_inputs(root: str = ROOT):
    """Files whose content determines the library: every HIP source and
    header under csrc/ and the C-ABI headers under include/."""
    pkg = os.path.join(root, os.path.basename(PKG))
    files = (glob.glob(os.path.join(pkg, "csrc", "*.hip")) + glob.glob(os.path.join(pkg, "csrc", "*.h"))
             + glob.glob(os.path.join(root, "include", "*.h")))
    return sorted(files, key=lambda f: os.path.relpath(f, root))


def source_hash(root: str = ROOT) -> str:
    """16 hex digits of SHA-256 over the stamped inputs (relative path and
    bytes of each) and the compiler flags (include path excluded, so the
    value does not depend on where the tree sits)."""
    h = hashlib.sha256()
    for f in stamped_inputs(root):
        h.update(os.path.relpath(f, root).encode() + b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    flags = [f for f in FLAGS if not f.startswith(ROOT)]
    h.update(" ".join(flags + [ARCH]).encode())
    return h.hexdigest()[:16]


def embedded_build_id(lib_path: str = LIB):
    """The build id stamped into a built library (read from the file, so the
    library need not be loaded), or None."""
    with open(lib_path, "rb") as fh:
        data = fh.read()
    k = data.find(BUILD_ID_MARKER)
    if k < 0:
        return None
    return data[k + len(BUILD_ID_MARKER):k + len(BUILD_ID_MARKER) + 16].decode("ascii", "replace")


class StaleLibraryError(RuntimeError):
    pass


def check_fresh(lib_path: str = LIB, root: str = ROOT) -> str:
    """Raise StaleLibraryError unless the library was built from the
    sources and flags now in the tree; return the build id."""
    want = source_hash(root)
    have = embedded_build_id(lib_path)
    if have != want:
        raise StaleLibraryError(
            f"{lib_path} was built from other sources (build id {have}, tree {want}): "
            "rebuild it with `python -m paper_2305_07187_amd.build`")
    return have


def build(verbose: bool = True, jobs: int = 8) -> str:
    """Compile each source to an object in parallel, then link the library."""
    srcs = sources()
    stamp = source_hash()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    t0 = time.time()
    procs = []
    objs = []
    for s in srcs:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(o)
        cmd = ([HIPCC] + [f for f in FLAGS if f != "-shared"] +
               [f'-DSI_BUILD_ID="{stamp}"', "-c", s, "-o", o])
        procs.append((s, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                               stderr=subprocess.STDOUT, text=True)))
        while sum(p.poll() is None for _, _, p in procs) >= jobs:
            time.sleep(0.05)
    failed = False
    for s, cmd, p in procs:
        out, _ = p.communicate()
        out = "\n".join(l for l in out.splitlines()
                        if "is not a recognized feature for this target" not in l)
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"compile failed: {' '.join(cmd)}\n{out}\n")
        elif out.strip() and verbose:
            sys.stderr.write(out + "\n")
    if failed:
        raise RuntimeError("HIP compilation failed")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} (build id {stamp}) from {len(srcs)} sources in "
              f"{time.time() - t0:.1f}s")
    return LIB


if __name__ == "__main__":
    build()
