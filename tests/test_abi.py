"""The C ABI without a GPU: the library loads, exports every function the
header declares, and its host-side argument checks return the documented
error codes (host-only context, device = -1)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_0812_0244_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vdwnl.h")

E = dict(OK=0, ARG=-1, SIZE=-2, NOMEM=-3, TABLE=-4, KRANGE=-5, STATE=-6, HIP=-7)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vdwnl_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = B.load_library()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
        assert name in B.SIGNATURES, name


def test_error_codes_match_header():
    text = open(HEADER).read()
    for key, code in E.items():
        if key == "SIZE":
            key = "UNSUPPORTED_SIZE"
        assert re.search(r"VDWNL_E_%s\s*=\s*%d" % (key, code), text) or key == "OK"
    lib = B.load_library()
    assert lib.vdwnl_strerror(0) == b"ok"
    assert lib.vdwnl_strerror(-2) == b"unsupported grid size"
    assert lib.vdwnl_strerror(-8) == b"invalid density (negative, NaN or infinite)"


def _host_ctx():
    lib = B.load_library()
    h = ctypes.c_void_p()
    assert lib.vdwnl_create(ctypes.byref(h), -1) == 0
    return lib, h


def _set_grid(lib, h, shape, cell=(10.0, 10.0, 10.0), gm=0, prec=32):
    s = np.array(shape, dtype=np.int32)
    c = np.array(cell, dtype=np.float64)
    return lib.vdwnl_set_grid(h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), gm, prec)


@pytest.mark.parametrize("shape,code", [((24, 24, 24), 0), ((96, 96, 96), 0), ((160, 160, 320), 0),
                                        ((12, 30, 50), 0), ((14, 24, 24), -2), ((24, 24, 3), -2),
                                        ((256, 24, 24), -2), ((24, 24, 512), -2), ((15, 15, 16), -2)])
def test_grid_validation(shape, code):
    lib, h = _host_ctx()
    assert _set_grid(lib, h, shape) == code
    lib.vdwnl_destroy(h)


def test_bad_arguments():
    lib, h = _host_ctx()
    assert _set_grid(lib, h, (24, 24, 24), cell=(10.0, -1.0, 10.0)) == E["ARG"]
    assert _set_grid(lib, h, (24, 24, 24), prec=16) == E["ARG"]
    assert _set_grid(lib, h, (24, 24, 24), gm=5) == E["ARG"]
    assert _set_grid(lib, h, (24, 24, 24), gm=-1) == E["ARG"]
    for gm in (1, 2, 3, 4):          # central differences, m points a side
        assert _set_grid(lib, h, (24, 24, 24), gm=gm) == 0
    assert lib.vdwnl_set_grid(None, None, None, 0, 32) == E["ARG"]
    assert lib.vdwnl_energy_potential(None, None, None, None, None) == E["ARG"]
    # evaluation on a host-only context
    assert _set_grid(lib, h, (24, 24, 24)) == 0
    Eo = np.zeros(2)
    rc = lib.vdwnl_energy_potential(h, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                    Eo.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
    assert rc == E["STATE"]
    lib.vdwnl_destroy(h)


def _table(nq=20, nk=64, dk=0.5, sym=True, qlast=5.0):
    q = np.linspace(0.05, qlast, nq)
    phi = np.random.default_rng(0).normal(size=(nq, nq, nk))
    if sym:
        phi = phi + phi.transpose(1, 0, 2)
    return q, phi, dk


def _set_table(lib, h, q, phi, dk, qc=5.0, mc=12):
    q = np.ascontiguousarray(q)
    phi = np.ascontiguousarray(phi)
    dp = ctypes.POINTER(ctypes.c_double)
    return lib.vdwnl_set_kernel_table(h, q.size, q.ctypes.data_as(dp), qc, mc, phi.shape[-1], dk,
                                      phi.ctypes.data_as(dp), 0.04)


def test_table_validation():
    lib, h = _host_ctx()
    q, phi, dk = _table()
    assert _set_table(lib, h, q, phi, dk) == 0
    assert _set_table(lib, h, *_table(sym=False)) == E["TABLE"]
    assert _set_table(lib, h, *_table(nq=12)) == E["TABLE"]
    assert _set_table(lib, h, *_table(qlast=4.0)) == E["TABLE"]
    qbad = q.copy()
    qbad[5] = qbad[4]
    assert _set_table(lib, h, qbad, phi, dk) == E["TABLE"]
    assert _set_table(lib, h, q, phi, dk, mc=0) == E["TABLE"]
    lib.vdwnl_destroy(h)


def test_kernel_table_range_checked_against_grid():
    """max |G| of a 96^3 grid in a 20 bohr cell is 26.1 bohr^-1: a table to
    k = 31.5 covers it, one to k = 15.5 does not."""
    lib, h = _host_ctx()
    assert _set_grid(lib, h, (96, 96, 96), cell=(20.0, 20.0, 20.0)) == 0
    q, phi, _ = _table(nk=64)
    assert _set_table(lib, h, q, phi, 0.5) == 0
    assert _set_table(lib, h, q, phi, 0.25) == E["KRANGE"]
    lib.vdwnl_destroy(h)


def test_binding_fails_loudly_without_library(tmp_path):
    saved = B._lib
    B._lib = None
    try:
        with pytest.raises(RuntimeError):
            B.load_library(str(tmp_path / "missing.so"))
    finally:
        B._lib = saved


def test_lattice_planning_checks():
    """Cells given by their vectors: a triclinic cell plans, a singular or
    non-finite one is rejected; a diagonal matrix plans like the lengths."""
    lib, h = _host_ctx()
    s = np.array([20, 18, 24], dtype=np.int32)
    ip = ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)

    def plan(cell):
        c = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(-1))
        return lib.vdwnl_set_grids_lattice(h, 1, s.ctypes.data_as(ip), c.ctypes.data_as(dp), 0, 32)

    tri = np.array([[8.0, 0.0, 0.0], [3.05, 6.85, 0.0], [-2.2, 1.9, 7.9]])
    assert plan(tri) == 0
    assert plan(np.diag([8.0, 9.0, 10.0])) == 0
    flat = tri.copy()
    flat[2] = flat[0] + flat[1]                  # a_3 in the plane of a_1, a_2
    assert plan(flat) == E["ARG"]
    nan = tri.copy()
    nan[1, 2] = np.nan
    assert plan(nan) == E["ARG"]
    assert lib.vdwnl_set_grids_lattice(h, 1, s.ctypes.data_as(ip), None, 0, 32) == E["ARG"]
    lib.vdwnl_destroy(h)


def test_functional_mode_checks():
    """vdwnl_set_functional takes the two documented values only; the
    semilocal energies exist only after an evaluation of the whole functional
    (a host-only context never evaluates)."""
    lib, h = _host_ctx()
    assert lib.vdwnl_set_functional(h, B.FUNCTIONAL_VDW_DF) == 0
    assert lib.vdwnl_set_functional(h, B.FUNCTIONAL_NONLOCAL) == 0
    assert lib.vdwnl_set_functional(h, 2) == E["ARG"]
    assert lib.vdwnl_set_functional(h, -1) == E["ARG"]
    assert lib.vdwnl_set_functional(None, 1) == E["ARG"]
    assert _set_grid(lib, h, (24, 24, 24)) == 0
    out = np.zeros(2)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.vdwnl_semilocal_energies(h, 1, out.ctypes.data_as(dp)) == E["STATE"]
    assert lib.vdwnl_semilocal_energies(h, 1, None) == E["ARG"]
    lib.vdwnl_destroy(h)


def test_async_call_checks():
    """The asynchronous batched call rejects a null energy buffer and, on a
    host-only context, reports that there is no device."""
    lib, h = _host_ctx()
    assert _set_grid(lib, h, (24, 24, 24)) == 0
    vp = ctypes.c_void_p
    n = (vp * 1)(vp(16))
    v = (vp * 1)(vp(32))
    assert lib.vdwnl_energy_potential_batched_async(h, 1, n, v, None, None) == E["ARG"]
    assert lib.vdwnl_energy_potential_batched_async(h, 1, n, v, vp(64), None) == E["STATE"]
    assert lib.vdwnl_energy_potential_batched_async(None, 1, n, v, vp(64), None) == E["ARG"]
    lib.vdwnl_destroy(h)


def test_pass_lists_and_tiling_on_host():
    """Pass names, the pass order of each gradient mode, and the tile budgets
    (set, read back, range-checked) on a host-only context."""
    lib, h = _host_ctx()
    i32 = ctypes.c_int32
    names = [lib.vdwnl_pass_name(i).decode() for i in range(40)]
    assert "z_main" in names and "x_theta" in names and "fd_grad" in names
    assert lib.vdwnl_pass_name(-1) == b"" and lib.vdwnl_pass_name(1000) == b""
    for gm, n_pass in ((0, 11), (3, 7)):
        assert _set_grid(lib, h, (24, 24, 24), gm=gm) == 0
        kinds = (i32 * 32)()
        n = lib.vdwnl_pass_order(h, 32, kinds)
        assert n == n_pass
        order = [names[kinds[i]] for i in range(n)]
        assert order[0] == ("x_deriv" if gm == 0 else "fd_grad")
        assert "z_main" in order and order[-1] == ("z_div" if gm == 0 else "fd_div")
    b = (ctypes.c_int64 * 5)(32768, 32768, 16384, 49152, 24576)
    assert lib.vdwnl_set_tiling(h, 5, b) == 0
    out = (ctypes.c_int64 * 8)()
    assert lib.vdwnl_get_tiling(h, 8, out) == 5
    assert list(out)[:5] == [32768, 32768, 16384, 49152, 24576]
    assert lib.vdwnl_set_tiling(h, 4, b) == E["ARG"]
    bad = (ctypes.c_int64 * 5)(32768, 32768, 1024, 49152, 24576)
    assert lib.vdwnl_set_tiling(h, 5, bad) == E["ARG"]
    nb = ctypes.c_int32()
    ws = ctypes.c_int64()
    assert lib.vdwnl_info(h, ctypes.byref(nb), ctypes.byref(ws)) == 0 and nb.value == 1
    lib.vdwnl_destroy(h)


def test_log_qmesh_built_by_the_library():
    """The library's logarithmic q mesh: q_1 and q_c at the ends, increments
    growing by lambda (the paragraph before Eq. (qsat)), equal to the
    oracle's mesh; invalid arguments refused."""
    from oracle import kernel_table as kt
    for nq, q1, qc, lam in [(20, 0.05, 5.0, 1.17), (12, 0.1, 4.0, 1.3), (30, 0.02, 6.0, 1.05), (8, 0.5, 3.0, 1.0)]:
        q = B.log_qmesh(nq, q1, qc, lam)
        assert q[0] == q1 and q[-1] == qc and np.all(np.diff(q) > 0)
        d = np.diff(q)
        np.testing.assert_allclose(d[1:] / d[:-1], lam, rtol=1e-9)
        np.testing.assert_allclose(q, kt.log_qmesh(nq, q1, qc, lam), rtol=1e-14, atol=0)
    lib = B.load_library()
    out = np.zeros(4)
    p = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for args in [(1, 0.05, 5.0, 1.17), (4, 0.0, 5.0, 1.17), (4, 5.0, 5.0, 1.17), (4, 0.05, 5.0, 0.9),
                 (4, 0.05, float("nan"), 1.17)]:
        assert lib.vdwnl_log_qmesh(*args, p) == E["ARG"]
    assert lib.vdwnl_log_qmesh(4, 0.05, 5.0, 1.17, None) == E["ARG"]


def test_debug_stage_on_host_context():
    lib, h = _host_ctx()
    buf = np.zeros(16)
    p = buf.ctypes.data_as(ctypes.c_void_p)
    assert lib.vdwnl_debug_stage(None, 0, 0, p, None) == E["ARG"]
    assert lib.vdwnl_debug_stage(h, 0, 0, None, None) == E["ARG"]
    assert lib.vdwnl_debug_stage(h, 0, 7, p, None) == E["ARG"]
    assert lib.vdwnl_debug_stage(h, 0, 0, p, None) == E["STATE"]   # nothing evaluated
    lib.vdwnl_destroy(h)


def test_noalloc_entry_point_on_host_context():
    lib, h = _host_ctx()
    Eo = np.zeros(2)
    pe = Eo.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    buf = np.zeros(8)
    p = buf.ctypes.data_as(ctypes.c_void_p)
    assert lib.vdwnl_energy_potential_noalloc(None, p, p, pe, None) == E["ARG"]
    assert lib.vdwnl_energy_potential_noalloc(h, None, p, pe, None) == E["ARG"]
    assert lib.vdwnl_energy_potential_noalloc(h, p, p, pe, None) == E["STATE"]   # no plan
    assert _set_grid(lib, h, (24, 24, 24)) == 0
    assert lib.vdwnl_energy_potential_noalloc(h, p, p, pe, None) == E["STATE"]   # no table, host only
    lib.vdwnl_destroy(h)


def test_schedule_choice_arguments():
    lib, h = _host_ctx()
    v = ctypes.c_int32(-1)
    assert lib.vdwnl_set_schedule(h, 0, 1) == E["STATE"]          # no grid planned
    assert _set_grid(lib, h, (24, 24, 24)) == 0
    for what, val, code in [(0, 0, 0), (0, 1, 0), (0, 2, E["ARG"]), (7, 0, E["ARG"]), (0, -1, E["ARG"])]:
        assert lib.vdwnl_set_schedule(h, what, val) == code
    assert lib.vdwnl_get_schedule(h, 0, ctypes.byref(v)) == 0 and v.value == 1
    assert lib.vdwnl_get_schedule(h, 9, ctypes.byref(v)) == E["ARG"]
    assert lib.vdwnl_get_schedule(h, 0, None) == E["ARG"]
    lib.vdwnl_destroy(h)


def test_radix_orders_multiply_to_their_length():
    """Every radix order of every compile-time length class (and the runtime
    plan of other lengths) is a factorisation of the length into passes of
    2, 3, 4, 5, 8 and 16; the orders of a length are distinct; an order past
    a length's last takes its last."""
    for n, count in [(24, 1), (32, 2), (48, 2), (64, 4), (96, 3), (128, 6), (160, 2), (320, 2), (36, 1), (250, 1)]:
        seen = []
        for v in range(6):
            r = B.radix_order(n, v)
            assert np.prod(r) == n and all(x in (2, 3, 4, 5, 8, 16) for x in r), (n, v, r)
            if v < count:
                assert r not in seen
                seen.append(r)
            else:
                assert r == seen[-1]
    lib = B.load_library()
    out = (ctypes.c_int32 * 8)()
    assert lib.vdwnl_radix_order(14, 0, 8, out) == E["SIZE"]
    assert lib.vdwnl_radix_order(128, 6, 8, out) == E["ARG"]
    assert lib.vdwnl_radix_order(128, 4, 8, out) == 2 and list(out[:2]) == [16, 8]
    assert lib.vdwnl_radix_order(128, 0, 8, None) == E["ARG"]
    assert lib.vdwnl_radix_order(128, 2, 1, out) == 3 and out[0] == 2     # (count returned, one written)


def test_radix_schedule_arguments():
    lib, h = _host_ctx()
    v = ctypes.c_int32(-1)
    assert _set_grid(lib, h, (24, 24, 24)) == 0
    for what in range(1, 6):
        assert lib.vdwnl_set_schedule(h, what, 3) == 0
        assert lib.vdwnl_get_schedule(h, what, ctypes.byref(v)) == 0 and v.value == 3
        assert lib.vdwnl_set_schedule(h, what, 5) == 0
        assert lib.vdwnl_set_schedule(h, what, 6) == E["ARG"]
    assert lib.vdwnl_set_schedule(h, 6, 0) == E["ARG"]
    lib.vdwnl_destroy(h)
