"""The library carries a hash of the sources and flags it was built from;
loading refuses a library whose hash differs from the tree's (a stale
binary), so tests, smoke() and the benchmark never run old code."""
import os
import shutil

import pytest

from paper_2305_07187_amd import build


def _copy_tree(dst):
    pkg = os.path.basename(build.PKG)
    shutil.copytree(os.path.join(build.PKG, "csrc"), os.path.join(dst, pkg, "csrc"))
    shutil.copytree(os.path.join(build.ROOT, "include"), os.path.join(dst, "include"))


def _fake_library(path, build_id):
    # a file with the stamp where the build puts it (in the read-only data)
    with open(path, "wb") as fh:
        fh.write(b"\x7fELF" + b"\0" * 64 + build.BUILD_ID_MARKER + build_id.encode() + b"\0" * 8)


def test_hash_depends_on_sources_not_on_location(tmp_path):
    _copy_tree(str(tmp_path))
    assert build.source_hash(str(tmp_path)) == build.source_hash()
    assert len(build.source_hash()) == 16


def test_editing_a_source_makes_the_library_stale(tmp_path):
    root = str(tmp_path)
    _copy_tree(root)
    lib = os.path.join(root, "lib.so")
    _fake_library(lib, build.source_hash(root))
    assert build.check_fresh(lib, root) == build.source_hash(root)
    src = sorted(build.stamped_inputs(root))
    hip = [f for f in src if f.endswith("si_epilogue.h")][0]
    with open(hip, "a") as fh:
        fh.write("\n// edited\n")
    with pytest.raises(build.StaleLibraryError):
        build.check_fresh(lib, root)
    # an edited public header counts too
    _fake_library(lib, build.source_hash(root))
    with open(os.path.join(root, "include", "spring_ising.h"), "a") as fh:
        fh.write("\n")
    with pytest.raises(build.StaleLibraryError):
        build.check_fresh(lib, root)


def test_unstamped_library_is_refused(tmp_path):
    lib = str(tmp_path / "lib.so")
    with open(lib, "wb") as fh:
        fh.write(b"\x7fELF no stamp")
    with pytest.raises(build.StaleLibraryError):
        build.check_fresh(lib)


def test_built_library_matches_tree():
    if not os.path.exists(build.LIB):
        build.build(verbose=False)
    assert build.embedded_build_id(build.LIB) == build.source_hash()
    from paper_2305_07187_amd import spring_ising as si
    si.load_library()
    assert si.spring_ising_build_id() == build.source_hash()
