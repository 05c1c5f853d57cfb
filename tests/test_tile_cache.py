"""Tile cache file format and validation (host code of the library; no GPU
work).  The cache keys and the autotuner that fills it are exercised by the
GPU tests."""
import os

import numpy as np
import pytest

from paper_2305_07187_amd import spring_ising as si
from paper_2305_07187_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(si.LIB_PATH):
        build.build(verbose=False)
    return si.load_library()


def _write(path, lines):
    path.write_text("".join(l + "\n" for l in lines))
    return str(path)


def _header():
    return ["# spring_ising tile cache 1", "build " + si.spring_ising_build_id()]


def test_round_trip(lib, tmp_path):
    si.spring_ising_tile_cache_clear()
    empty = tmp_path / "empty.txt"
    si.spring_ising_tile_cache_save(str(empty))
    assert empty.read_text().splitlines() == _header()
    entries = ["0 0 11 0 1024 256 27 73.5", "0 1 11 0 1024 256 32 17.1",
               "1 5 19 12 64 256 2 905.25", "1 0 19 12 64 256 1 1650"]
    src = _write(tmp_path / "in.txt", _header() + entries)
    assert si.spring_ising_tile_cache_load(src) == 4
    out = tmp_path / "out.txt"
    si.spring_ising_tile_cache_save(str(out))
    lines = out.read_text().splitlines()
    assert lines[:2] == _header()
    # the time is stored as a float32: it reads back to the same float32
    f32 = lambda l: tuple(int(v) for v in l.split()[:7]) + (float(np.float32(l.split()[7])),)
    assert sorted(map(f32, lines[2:])) == sorted(map(f32, entries))
    # loading merges: a second file overrides one key, adds none
    assert si.spring_ising_tile_cache_load(
        _write(tmp_path / "in2.txt", _header() + ["0 0 11 0 1024 256 26 74"])) == 1
    si.spring_ising_tile_cache_save(str(out))
    lines = out.read_text().splitlines()[2:]
    assert len(lines) == 4 and f32("0 0 11 0 1024 256 26 74") in map(f32, lines)
    si.spring_ising_tile_cache_clear()
    si.spring_ising_tile_cache_save(str(out))
    assert out.read_text().splitlines() == _header()


@pytest.mark.parametrize("lines,status", [
    (["# not a cache", "build x"], "invalid"),
    (["# spring_ising tile cache 1"], "invalid"),
    (["# spring_ising tile cache 1", "build 0000000000000000"], "state"),
    (None, "invalid_entry"),
])
def test_rejected_files_load_nothing(lib, tmp_path, lines, status):
    si.spring_ising_tile_cache_clear()
    bad_entries = [
        "0 0 11 0 1024 256 99 1",      # no FP32 tile 99
        "0 5 11 0 1024 256 19 1",      # single contexts resolve the mixed form
        "1 0 19 12 64 256 3 1",        # batch tiles are 1 and 2
        "0 0 11 0 1000 256 27 1",      # R not a multiple of 64
        "2 0 11 0 1024 256 27 1",      # unknown kind
        "0 0 11 0 1024 256 27",        # missing field
        "0 0 11 0 1024 256 27 1 x",    # trailing field
    ]
    if lines is None:
        for k, entry in enumerate(bad_entries):
            path = _write(tmp_path / f"bad{k}.txt",
                          _header() + ["0 0 11 0 1024 256 27 73.5", entry])
            with pytest.raises(si.SpringIsingError) as e:
                si.spring_ising_tile_cache_load(path)
            assert e.value.status == si.SI_ERR_INVALID, entry
    else:
        path = _write(tmp_path / "bad.txt", lines)
        with pytest.raises(si.SpringIsingError) as e:
            si.spring_ising_tile_cache_load(path)
        assert e.value.status == (si.SI_ERR_STATE if status == "state" else si.SI_ERR_INVALID)
    out = tmp_path / "out.txt"
    si.spring_ising_tile_cache_save(str(out))
    assert out.read_text().splitlines() == _header()  # nothing was merged


def test_missing_files(lib, tmp_path):
    with pytest.raises(si.SpringIsingError) as e:
        si.spring_ising_tile_cache_load(str(tmp_path / "absent.txt"))
    assert e.value.status == si.SI_ERR_INVALID
    with pytest.raises(si.SpringIsingError) as e:
        si.spring_ising_tile_cache_save(str(tmp_path / "no_dir" / "x.txt"))
    assert e.value.status == si.SI_ERR_INVALID
