"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
its host-side validation returns the documented status codes before any
device work (no compute call reaches the GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1209_4506_amd", "libhartree.so")
HEADER = os.path.join(ROOT, "include", "hartree.h")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhartree.so not built")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hartree_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 16
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_lists_every_symbol():
    import paper_1209_4506_amd.hartree as H

    assert sorted(H.EXPORTED) == declared_symbols()


def _create(lib, cell, dims, prec=1, opts=None):
    h = ctypes.c_void_p()
    cell = np.ascontiguousarray(cell, dtype=np.float64).reshape(9)
    dims = np.ascontiguousarray(dims, dtype=np.int32)
    lib.hartree_plan_create.restype = ctypes.c_int
    rc = lib.hartree_plan_create(ctypes.byref(h), cell.ctypes.data_as(ctypes.c_void_p),
                                 dims.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(prec), opts)
    return rc, h


def test_plan_validation(lib):
    lib.hartree_last_error.restype = ctypes.c_char_p
    cube = np.eye(3) * 10
    assert _create(lib, cube, (32, 32, 33))[0] == 2          # 33 = 3 * 11
    assert _create(lib, cube, (0, 4, 4))[0] == 2
    assert _create(lib, cube, (8192, 4, 4))[0] == 2
    assert b"dimension" in lib.hartree_last_error()
    assert _create(lib, np.zeros((3, 3)), (8, 8, 8))[0] == 3
    assert _create(lib, [[1, 0, 0], [2, 0, 0], [0, 0, 1]], (8, 8, 8))[0] == 3
    bad = cube.copy()
    bad[1, 1] = np.nan
    assert _create(lib, bad, (8, 8, 8))[0] == 3
    assert _create(lib, cube, (8, 8, 8), prec=7)[0] == 1
    rc, h = _create(lib, cube, (7, 14, 21))       # radix 7 is accepted
    assert rc == 0
    n = ctypes.c_size_t()
    assert lib.hartree_workspace_size(h, ctypes.byref(n)) == 0 and n.value > 0
    # compute calls without a bound workspace fail before touching the device
    vp = ctypes.c_void_p
    lib.hartree_solve.argtypes = [vp, vp, vp, vp, vp]
    assert lib.hartree_solve(h, vp(16), vp(32), None, None) == 5
    lib.hartree_energy.argtypes = [vp, vp, vp, vp]
    assert lib.hartree_energy(h, vp(16), vp(32), None) == 5
    lib.hartree_plan_destroy.argtypes = [vp]
    lib.hartree_plan_destroy(h)


def test_noalloc_size_limit(lib):
    """hartree_solve_noalloc refuses a plan larger than its device scratch
    (HARTREE_NOALLOC_BYTES) with HARTREE_ERR_WORKSPACE before any device call;
    argument errors come first."""
    vp = ctypes.c_void_p
    lib.hartree_solve_noalloc.argtypes = [vp, vp, vp, vp, vp]
    lib.hartree_last_error.restype = ctypes.c_char_p
    rc, h = _create(lib, np.eye(3) * 20.0, (256, 256, 256))
    assert rc == 0
    assert lib.hartree_solve_noalloc(h, vp(16), vp(32), None, None) == 5
    msg = lib.hartree_last_error()
    assert b"HARTREE_NOALLOC_BYTES" in msg and b"67108864" in msg
    assert lib.hartree_solve_noalloc(h, None, vp(32), None, None) == 1
    assert lib.hartree_solve_noalloc(h, vp(16), vp(16), None, None) == 1
    assert lib.hartree_solve_noalloc(None, vp(16), vp(32), None, None) == 1
    lib.hartree_plan_destroy.argtypes = [vp]
    lib.hartree_plan_destroy(h)


def test_batched_plan_offsets(lib):
    from paper_1209_4506_amd import inputs

    probs = inputs.batched24()
    cells = np.stack([p.cell for p in probs]).astype(np.float64)
    dims = np.array([p.dims for p in probs], dtype=np.int32)
    h = ctypes.c_void_p()
    vp = ctypes.c_void_p
    lib.hartree_plan_create_batched.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32, vp]
    rc = lib.hartree_plan_create_batched(ctypes.byref(h), len(probs), cells.ctypes.data_as(vp),
                                         dims.ctypes.data_as(vp), 1, None)
    assert rc == 0
    off = ctypes.c_int64()
    lib.hartree_plan_grid_offset.argtypes = [vp, ctypes.c_int32, vp]
    total = 0
    for i, p in enumerate(probs):
        assert lib.hartree_plan_grid_offset(h, i, ctypes.byref(off)) == 0
        assert off.value == total
        total += p.npoints
    assert lib.hartree_plan_grid_offset(h, len(probs), ctypes.byref(off)) == 0 and off.value == total
    assert lib.hartree_plan_grid_offset(h, len(probs) + 1, ctypes.byref(off)) == 1
    lib.hartree_plan_destroy.argtypes = [vp]
    lib.hartree_plan_destroy(h)


def _smooth(limit):
    out = []
    for n in range(1, limit + 1):
        m = n
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def test_every_smooth_length_gets_a_plan(lib):
    """Every 7-smooth axis length up to 4096 has a stage plan that fits the
    kernels, in both precisions; other lengths are refused."""
    vp = ctypes.c_void_p
    lib.hartree_plan_destroy.argtypes = [vp]
    cube = np.eye(3) * 10
    for prec in (0, 1):
        for n in _smooth(4096):
            rc, h = _create(lib, cube, (n, 1, 1), prec=prec)
            assert rc == 0, (n, prec, lib.hartree_last_error())
            lib.hartree_plan_destroy(h)
    for n in (11, 13, 22, 4097, 4099):
        assert _create(lib, cube, (1, n, 1))[0] == 2


def test_pass_config_validation(lib):
    """Pass shapes: get returns one (plan, p_log2) per problem and axis; set
    accepts the current choice and rejects ones that do not apply; tuning
    needs a bound workspace (host-side checks only)."""
    lib.hartree_last_error.restype = ctypes.c_char_p
    for fn in ("hartree_plan_get_config", "hartree_plan_set_config", "hartree_plan_tune"):
        getattr(lib, fn).restype = ctypes.c_int
    for prec in (0, 1):
        rc, h = _create(lib, np.diag([9.0, 10.0, 11.0]), (360, 60, 45), prec=prec)
        assert rc == 0
        cfg = (ctypes.c_int32 * 9)()
        assert lib.hartree_plan_get_config(h, cfg) == 0
        vals = list(cfg)
        assert all(0 <= vals[3 * x + 1] <= 8 for x in range(3))
        assert all(0 <= vals[3 * x + 2] <= 3 for x in range(2)) and vals[8] == 0
        assert lib.hartree_plan_set_config(h, cfg) == 0          # the current choice round-trips
        for idx, bad_value in ((1, 9),                           # 512 pencils per workgroup
                               (0, 10_000),                      # no such compiled plan
                               (6, vals[0] if vals[0] >= 0 else 0),  # the 360 plan on the length-45 axis
                               (2, 4),                           # pad beyond 3
                               (8, 1)):                          # a pad on the c axis
            bad = (ctypes.c_int32 * 9)(*vals)
            bad[idx] = bad_value
            assert lib.hartree_plan_set_config(h, bad) == 1, (idx, bad_value)
        assert b"does not apply" in lib.hartree_last_error()
        assert lib.hartree_plan_get_config(h, cfg) == 0
        assert list(cfg) == vals                                 # rejected choices change nothing
        assert lib.hartree_plan_tune(h, ctypes.c_void_p(1), 3, None) == 5   # no workspace bound
        lib.hartree_plan_destroy(h)


def test_compiled_plans_for_360_and_180(lib):
    """The compiled radix plans accepted for a length are exactly the table
    entries whose radices multiply to it: for 360 the 9 x 8 x 5 entry, the
    three radix-6 orders (10 x 6 x 6, 6 x 6 x 10, 6 x 10 x 6) and the two
    radix-12 first stages (12 x 5 x 6, 12 x 6 x 5), for 180 the 9 x 5 x 4
    entry and 10 x 6 x 3, 6 x 6 x 5.  Entries are only appended to
    the table, so these indices are stable (stored tuner choices use them).
    Host-side validation only (64 KiB of LDS assumed without a device)."""
    lib.hartree_plan_destroy.argtypes = [ctypes.c_void_p]
    for fn in ("hartree_plan_get_config", "hartree_plan_set_config"):
        getattr(lib, fn).restype = ctypes.c_int
    expect = {360: {20, 36, 37, 38, 44, 45}, 180: {11, 39, 40}}
    for prec in (0, 1):
        for n, ids in expect.items():
            for x in range(3):
                dims = [12, 10, 14]
                dims[x] = n
                rc, h = _create(lib, np.diag([9.0, 10.0, 11.0]), tuple(dims), prec=prec)
                assert rc == 0
                cfg = (ctypes.c_int32 * 9)()
                assert lib.hartree_plan_get_config(h, cfg) == 0
                base = list(cfg)
                accepted = set()
                for pid in range(64):
                    for lp in range(7):
                        trial = (ctypes.c_int32 * 9)(*base)
                        trial[3 * x], trial[3 * x + 1], trial[3 * x + 2] = pid, lp, 0
                        if lib.hartree_plan_set_config(h, trial) == 0:
                            accepted.add(pid)
                            break
                assert accepted == ids, (prec, n, x, sorted(accepted))
                lib.hartree_plan_destroy(h)

