"""CPU-side checks of the HIP library: it loads, exports every symbol that
include/lbm81.h declares, and its host-only entry points (sizes, velocity
set) agree with an independent construction.  No device call is made here.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm81.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2409_05114_amd import lbm81
    if not os.path.exists(lbm81.LIB_PATH):
        pytest.fail("liblbm81.so is not built (run __graft_entry__.build())")
    return lbm81


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("lbm_create", "lbm_init", "lbm_step", "lbm_moments",
              "lbm_totals", "lbm_step_batch", "lbm_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(so, n)]
    assert not missing, missing


def test_library_has_gfx950_code_object(lib):
    data = open(lib.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_sizes(lib):
    def planes(n_sites, es):  # 81 planes, rounded up to 256 B, + 4352 B
        return 81 * ((n_sites * es + 255) // 256 * 256 + 4352)

    def tiles(nx, ny, nz, es):  # rows of min(nx, 64)-wide tiles, padded
        tw = min(nx, 64)
        return 2 * ny * nz * (-(-nx // 64)) * 81 * tw * es

    assert lib.lbm_population_bytes(32, 32, 32, "f64") == planes(2 * 32 ** 3, 8)
    assert lib.lbm_population_bytes(512, 512, 256, "f32") == \
        81 * 2 * 512 * 512 * 256 * 4 == tiles(512, 512, 256, 4)
    assert lib.lbm_population_bytes(48, 48, 48, "bf16") == planes(2 * 48 ** 3, 2)
    assert lib.lbm_population_bytes(48, 48, 48, "f32") == 81 * 2 * 48 ** 3 * 4
    # rows longer than 64 that 64 does not divide are padded to whole tiles
    assert lib.lbm_population_bytes(96, 4, 4, "f32") == 81 * 2 * 128 * 4 * 4 * 4
    assert lib.lbm_population_bytes(20, 12, 10, "f64") == planes(2 * 2400, 8)
    for st, es in (("f64", 8), ("f32", 4), ("f16", 2), ("bf16", 2)):
        assert lib.lbm_population_bytes(5, 6, 7, st) >= 81 * 2 * 210 * es
    assert lib.lbm_population_bytes(0, 4, 4, "f64") == 0
    assert lib.lbm_workspace_bytes(8, 8, 8) > 0
    lib_so = lib.library()
    assert lib_so.lbm_population_bytes(4, 4, 4, 7) == 0  # unknown storage
    assert lib.lbm_version() >= 1


def test_size_limits(lib):
    """Sites and row lengths are indexed with 32-bit integers: 2 nx ny nz <
    2^31 and nx <= 2^24.  The largest grids are accepted, with byte counts
    computed in 64 bits (1.4 TB for FP64 at 1024 x 1024 x 1023); one more
    site or one more cell along x is refused (size 0)."""
    def planes(n_sites, es):
        return 81 * ((n_sites * es + 255) // 256 * 256 + 4352)

    big = (1024, 1024, 1023)
    assert 2 * 1024 * 1024 * 1023 < 2 ** 31
    assert lib.lbm_population_bytes(*big, "f64") == planes(2 * 1024 * 1024 * 1023, 8)
    assert lib.lbm_population_bytes(*big, "f32") == 81 * 2 * 1024 * 1024 * 1023 * 4
    assert lib.lbm_population_bytes(1024, 1024, 1024, "f64") == 0
    assert lib.lbm_population_bytes(2 ** 24, 1, 1, "f16") == planes(2 ** 25, 2)
    assert lib.lbm_population_bytes(2 ** 24 + 1, 1, 1, "f16") == 0
    # the workspace (a fixed number of reduction partials and the flag
    # word) does not depend on the grid
    assert lib.lbm_workspace_bytes(*big) == lib.lbm_workspace_bytes(8, 8, 8) > 0


def test_status_strings(lib):
    so = lib.library()
    assert so.lbm_status_string(0) == b"ok"
    assert so.lbm_status_string(-4) == b"unrealizable state"
    assert so.lbm_status_string(12345) == b"unknown status"


def test_create_rejects_bad_arguments_without_touching_the_device(lib):
    so = lib.library()
    h = ctypes.c_void_p()
    # NULL buffers, zero size, unknown storage: refused before any HIP call
    assert so.lbm_create(8, 8, 8, 0, None, None, None, ctypes.byref(h)) == -1
    assert so.lbm_create(0, 8, 8, 0, None, None, None, ctypes.byref(h)) == -1
    assert so.lbm_create(8, 8, 8, 9, None, None, None, ctypes.byref(h)) == -1
    # misaligned pointers
    assert so.lbm_create(8, 8, 8, 0, ctypes.c_void_p(8), ctypes.c_void_p(256),
                         None, ctypes.byref(h)) == -1
    # a sweep of 2^32 lanes or more (one wavefront per row of 4 x):
    # refused by size, before the buffers are looked at
    so.lbm_last_error.restype = ctypes.c_char_p
    assert so.lbm_create(4, 8192, 8192, 0, None, None, None, ctypes.byref(h)) == -1
    assert b"2^32 lanes" in so.lbm_last_error()
    assert so.lbm_create(4, 8192, 4095, 0, None, None, None, ctypes.byref(h)) == -1
    assert b"device pointers" in so.lbm_last_error()
    assert so.lbm_step(None, 1, 0.8) == -1
    # warm-start buffer: 4 bytes per site; NULL simulation refused
    so.lbm_warm_bytes.restype = ctypes.c_size_t
    assert so.lbm_warm_bytes(8, 8, 8) == 4 * 2 * 8 * 8 * 8
    assert so.lbm_warm_bytes(0, 8, 8) == 0
    assert so.lbm_set_warm_start(None, None) == -1
    # placement probe: NULL simulation or result pointer refused
    ms = ctypes.c_float(1.0)
    assert so.lbm_probe_placement(None, 3, ctypes.byref(ms)) == -1
    assert ms.value == 1.0
    assert so.lbm_step_batch(None, None, None, 0, None) == 0
    # per-simulation step counts are required (sims, nsteps[], taus[], n)
    one = (ctypes.c_void_p * 1)(None)
    steps = (ctypes.c_int * 1)(1)
    taus = (ctypes.c_double * 1)(0.8)
    assert so.lbm_step_batch(one, None, taus, 1, None) == -1
    assert so.lbm_step_batch(one, steps, taus, 1, None) == -1  # NULL sim
    assert so.lbm_step_batch(one, steps, taus, 65, None) == -1  # n > max
    flags = (ctypes.c_uint * 1)(0)
    assert so.lbm_flags_batch(None, 0, None, None) == 0
    assert so.lbm_flags_batch(one, 1, None, None) == -1  # no host array
    assert so.lbm_flags_batch(one, 1, flags, None) == -1  # NULL sim
    assert so.lbm_flags_batch(one, 65, flags, None) == -1  # n > max


def test_velocity_set_matches_the_oracle_lattice(lib, oracle_mod):
    """The library builds its lattice at compile time from the weight table;
    the oracle builds its own.  Same 81 vectors, same weights."""
    c, w = lib.lbm_velocities()
    co, wo, th0 = oracle_mod.lattice()
    lib_map = {tuple((2 * v).astype(int)): wi for v, wi in zip(c, w)}
    or_map = {tuple((2 * v).astype(int)): wi for v, wi in zip(co, wo)}
    assert set(lib_map) == set(or_map)
    for k in lib_map:
        assert lib_map[k] == pytest.approx(or_map[k], rel=2e-16, abs=0)
    assert w.sum() == pytest.approx(1.0, abs=3e-16)
    # library order: 0 rest, d and d + 40 opposite
    assert np.all(c[0] == 0)
    assert np.all(c[1:41] == -c[41:81])
