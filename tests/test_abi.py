"""C ABI checks that need no GPU: the header, the exported symbols, and the
synchronous argument errors of the entry points."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_2305_07187_amd import spring_ising as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _ensure_lib():
    if not os.path.exists(si.LIB_PATH):
        from paper_2305_07187_amd import build
        build.build(verbose=False)
    return si.load_library()


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(spring_ising_\w+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    lib = _ensure_lib()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    # and the binding mirrors every entry point
    for name in names:
        if name != "spring_ising_last_error":
            assert hasattr(si, name), name


@pytest.mark.parametrize("std,compiler", [("-std=c99", "gcc"), ("-std=c++17", "g++")])
def test_header_compiles_standalone(tmp_path, std, compiler):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} missing")
    src = tmp_path / ("t.c" if compiler == "gcc" else "t.cpp")
    src.write_text('#include "spring_ising.h"\nint main(void){ si_params p; si_info i; '
                   '(void)p; (void)i; return (int)sizeof(si_params) - 56; }\n')
    r = subprocess.run([compiler, std, "-Wall", "-Werror", "-pedantic", "-I",
                        os.path.join(ROOT, "include"), str(src), "-o", str(tmp_path / "t")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert subprocess.run([str(tmp_path / "t")]).returncode == 0  # struct size fixed at 56


def test_struct_layouts_match_binding():
    assert ctypes.sizeof(si.si_params) == 56
    assert ctypes.sizeof(si.si_info) == 4 * 12 + 8 + 64 + 4 * 4


def test_default_params_are_the_papers():
    _ensure_lib()
    p = si.spring_ising_default_params(10000)
    import numpy as np
    f = lambda x: float(np.float32(x))
    assert (p.k, p.m, p.dt) == (0.5, 1.0, f(0.2))
    assert (p.zeta_start, p.zeta_end) == (f(0.04), 0.5)
    assert (p.qmax, p.pmax) == (f(2 ** 0.5), 2.0)
    assert (p.total_steps, p.stair_len, p.order, p.wall, p.precision) == (10000, 1, 0, 0, 0)
    with pytest.raises(si.SpringIsingError) as e:
        si.spring_ising_default_params(0)
    assert e.value.status == si.SI_ERR_INVALID


def test_argument_errors_are_synchronous():
    lib = _ensure_lib()
    p = si.spring_ising_default_params(100)
    ctx = ctypes.c_void_p()
    bogus = ctypes.c_void_p(0x1000)
    cases = [
        (0, 8, bogus, bogus, "n=0"),
        (8, 0, bogus, bogus, "r=0"),
        (8, 8, None, bogus, "J and x0 are required"),
    ]
    for n, r, J, x0, msg in cases:
        st = lib.spring_ising_init(ctypes.byref(ctx), n, r, J, x0, None, ctypes.byref(p), None)
        assert st == si.SI_ERR_INVALID
        assert msg in si.last_error()
    bad = si.spring_ising_default_params(100)
    for field, val in [("m", 0.0), ("dt", -1.0), ("qmax", 0.0), ("pmax", float("nan")),
                       ("total_steps", 0), ("stair_len", 0), ("order", 7), ("wall", 3),
                       ("precision", 99), ("tile", 999)]:
        bad = si.spring_ising_default_params(100)
        setattr(bad, field, val)
        st = lib.spring_ising_init(ctypes.byref(ctx), 8, 8, bogus, bogus, None, ctypes.byref(bad), None)
        assert st == si.SI_ERR_INVALID, field
        assert "params" in si.last_error()
    # host (non-device) memory is rejected
    host = (ctypes.c_float * 64)()
    st = lib.spring_ising_init(ctypes.byref(ctx), 8, 8, ctypes.cast(host, ctypes.c_void_p),
                               ctypes.cast(host, ctypes.c_void_p), None, ctypes.byref(p), None)
    assert st == si.SI_ERR_INVALID and "device pointers" in si.last_error()
    assert not ctx.value


def test_null_context_calls():
    lib = _ensure_lib()
    assert lib.spring_ising_destroy(None) == si.SI_OK
    for fn, args in [("spring_ising_step", []), ("spring_ising_run", [1]),
                     ("spring_ising_energy", [None, None]), ("spring_ising_spins", [None]),
                     ("spring_ising_get_state", [None, None, None]),
                     ("spring_ising_set_state", [None, None, 0]),
                     ("spring_ising_set_schedule", [None, None]),
                     ("spring_ising_get_schedule", [None, None]),
                     ("spring_ising_set_field", [None])]:
        assert getattr(lib, fn)(None, *args) == si.SI_ERR_INVALID, fn
        assert "null context" in si.last_error()


def test_c_program_builds(tmp_path):
    # A C99 program built against include/ and the library alone (the GPU
    # tests run it).
    from c_demo import build_c_demo
    ok, msg = build_c_demo(tmp_path / "c_abi_demo")
    if not ok and "missing" in msg:
        pytest.skip(msg)
    assert ok, msg

