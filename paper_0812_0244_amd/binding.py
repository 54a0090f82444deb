"""ctypes binding of libvdwnl.so: argument marshalling only.

Every step of the evaluation runs in the HIP kernels of the library.  The
binding fails loudly when the library has not been built; there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libvdwnl.so")

_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p

# name -> (restype, argtypes); every symbol that include/vdwnl.h declares
SIGNATURES = {
    "vdwnl_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int]),
    "vdwnl_destroy": (ctypes.c_int, [_vp]),
    "vdwnl_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "vdwnl_last_error": (ctypes.c_char_p, [_vp]),
    "vdwnl_set_grid": (ctypes.c_int, [_vp, _ip, _dp, _i32, _i32]),
    "vdwnl_set_grids": (ctypes.c_int, [_vp, _i32, _ip, _dp, _i32, _i32]),
    "vdwnl_set_grids_lattice": (ctypes.c_int, [_vp, _i32, _ip, _dp, _i32, _i32]),
    "vdwnl_set_kernel_table": (ctypes.c_int, [_vp, _i32, _dp, ctypes.c_double, _i32, _i32,
                                              ctypes.c_double, _dp, ctypes.c_double]),
    "vdwnl_energy_potential": (ctypes.c_int, [_vp, _vp, _vp, _dp, _vp]),
    "vdwnl_energy_potential_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _dp, _vp]),
    "vdwnl_energy_potential_batched": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_vp),
                                                      ctypes.POINTER(_vp), _dp, _vp]),
    "vdwnl_energy_potential_batched_async": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_vp),
                                                            ctypes.POINTER(_vp), _vp, _vp]),
    "vdwnl_debug_field": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp]),
    "vdwnl_debug_stage": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp]),
    "vdwnl_log_qmesh": (ctypes.c_int, [_i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]),
    "vdwnl_info": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_int64)]),
    "vdwnl_set_timing": (ctypes.c_int, [_vp, _i32]),
    "vdwnl_pass_times": (ctypes.c_int, [_vp, _i32, _dp, ctypes.POINTER(ctypes.c_int64)]),
    "vdwnl_pass_name": (ctypes.c_char_p, [_i32]),
    "vdwnl_pass_order": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i32)]),
    "vdwnl_build_kernel_table": (ctypes.c_int, [ctypes.c_int, _i32, _dp, ctypes.c_double, ctypes.c_double,
                                                _i32, ctypes.c_double, _dp, _dp]),
    "vdwnl_kernel_phi": (ctypes.c_int, [ctypes.c_int, _i32, _dp, _dp, _dp]),
    "vdwnl_set_graph": (ctypes.c_int, [_vp, _i32]),
    "vdwnl_set_functional": (ctypes.c_int, [_vp, _i32]),
    "vdwnl_semilocal_energies": (ctypes.c_int, [_vp, _i32, _dp]),
    "vdwnl_autotune": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i32, _vp]),
    "vdwnl_get_tiling": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_int64)]),
    "vdwnl_set_tiling": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_int64)]),
    "vdwnl_set_schedule": (ctypes.c_int, [_vp, _i32, _i32]),
    "vdwnl_get_schedule": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i32)]),
    "vdwnl_radix_order": (ctypes.c_int, [_i32, _i32, _i32, ctypes.POINTER(_i32)]),
}

_lib = None

FUNCTIONAL_NONLOCAL = 0
FUNCTIONAL_VDW_DF = 1
SCHEDULE_CONTRACTION = 0
CONTRACTION_VECTOR, CONTRACTION_MATRIX = 0, 1
RADIX_GROUPS = ("x", "y20", "yaux", "z", "zaux")     # schedule choices 1..5


def radix_order(n: int, order: int = 0):
    """The radix passes of the length-n transform in radix order `order`."""
    lib = load_library()
    r = (_i32 * 16)()
    k = lib.vdwnl_radix_order(int(n), int(order), 16, r)
    if k < 0:
        raise VdwNlError(k, "vdwnl_radix_order")
    return [int(r[i]) for i in range(k)]


class VdwNlError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_lib.vdwnl_strerror(code).decode() if _lib else "error", code, msg))
        self.code = code


def load_library(path: str = LIB_PATH):
    """Load libvdwnl.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: when torch is present its runtime
        # (same soname) must be loaded first, so the library binds to it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(path):
            raise RuntimeError("libvdwnl.so not built (%s); run __graft_entry__.build()" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


STAGE_THETA, STAGE_THETA_K, STAGE_U_K, STAGE_U, STAGE_GRAD = 0, 1, 2, 3, 4


def log_qmesh(nq: int = 20, q1: float = 0.05, qc: float = 5.0, lam: float = 1.17):
    """Logarithmic q mesh built by the library: (q_{a+1} - q_a) = lam (q_a - q_{a-1}),
    q_1 = q1, q_N = q_c."""
    lib = load_library()
    q = np.zeros(int(nq))
    rc = lib.vdwnl_log_qmesh(int(nq), float(q1), float(qc), float(lam), _as_ptr(q, ctypes.c_double))
    if rc != 0:
        raise VdwNlError(rc, "vdwnl_log_qmesh")
    return q


def kernel_phi(d1, d2, device: int = 0):
    """phi(d1, d2) of Eq. (Enl) evaluated on the GPU (host arrays in and out)."""
    lib = load_library()
    a = np.ascontiguousarray(np.broadcast_arrays(np.asarray(d1, float), np.asarray(d2, float))[0]).ravel()
    b = np.ascontiguousarray(np.broadcast_arrays(np.asarray(d1, float), np.asarray(d2, float))[1]).ravel()
    out = np.zeros(a.size)
    rc = lib.vdwnl_kernel_phi(int(device), a.size, _as_ptr(a, ctypes.c_double), _as_ptr(b, ctypes.c_double),
                              _as_ptr(out, ctypes.c_double))
    if rc != 0:
        raise VdwNlError(rc, "kernel_phi")
    return out


def build_kernel_table(device: int = 0, nq: int = 20, q1: float = 0.05, qc: float = 5.0, lam: float = 1.17,
                       mc: int = 12, d_s: float = 1.0, phi0: float = 0.5, nk: int = 6401, dk: float = 0.005):
    """The radial kernel table and C_s, computed by the library on the GPU."""
    lib = load_library()
    q = log_qmesh(nq, q1, qc, lam)
    phi = np.zeros((nq, nq, nk))
    cs = np.zeros(1)
    rc = lib.vdwnl_build_kernel_table(device, nq, _as_ptr(q, ctypes.c_double), d_s, phi0, nk, dk,
                                      _as_ptr(phi, ctypes.c_double), _as_ptr(cs, ctypes.c_double))
    if rc != 0:
        raise VdwNlError(rc, "vdwnl_build_kernel_table")
    return dict(qmesh=q, qc=qc, mc=mc, dk=dk, nk=nk, phi=phi, c_soft=float(cs[0]), ds=d_s, phi0=phi0)


def _as_ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class VdwNl:
    """One library context (same names as the C functions, without prefix)."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        h = _vp()
        rc = self.lib.vdwnl_create(ctypes.byref(h), int(device))
        if rc != 0:
            raise VdwNlError(rc, "vdwnl_create(device=%d): %s" % (device, self.lib.vdwnl_last_error(None).decode()))
        self.h = h
        self.ngrids = 0
        self.precision = None

    def _check(self, rc, what):
        if rc != 0:
            raise VdwNlError(rc, "%s: %s" % (what, self.lib.vdwnl_last_error(self.h).decode()))

    def close(self):
        if getattr(self, "h", None):
            self.lib.vdwnl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_grid(self, shape, cell, grad_mode: int = 0, precision: int = 32):
        """cell: three orthorhombic lengths or a 3 x 3 matrix of cell vectors (rows)."""
        if np.asarray(cell).shape != (3,):
            return self.set_grids([shape], [cell], grad_mode, precision)
        s = np.ascontiguousarray(shape, dtype=np.int32)
        c = np.ascontiguousarray(cell, dtype=np.float64)
        self._check(self.lib.vdwnl_set_grid(self.h, _as_ptr(s, ctypes.c_int32), _as_ptr(c, ctypes.c_double),
                                            grad_mode, precision), "set_grid")
        self.ngrids, self.precision = 1, precision

    def set_grids(self, shapes, cells, grad_mode: int = 0, precision: int = 32):
        """cells: per grid three orthorhombic lengths, or (any of them) a 3 x 3
        matrix of cell vectors (rows); a batch with any matrix is planned
        through vdwnl_set_grids_lattice."""
        s = np.ascontiguousarray(shapes, dtype=np.int32).reshape(-1, 3)
        cl = [np.asarray(c, dtype=np.float64) for c in cells]
        if all(c.shape == (3,) for c in cl):
            c = np.ascontiguousarray(np.stack(cl))
            rc = self.lib.vdwnl_set_grids(self.h, len(s), _as_ptr(s, ctypes.c_int32), _as_ptr(c, ctypes.c_double),
                                          grad_mode, precision)
        else:
            c = np.ascontiguousarray(np.stack([np.diag(x) if x.shape == (3,) else x.reshape(3, 3) for x in cl]))
            rc = self.lib.vdwnl_set_grids_lattice(self.h, len(s), _as_ptr(s, ctypes.c_int32),
                                                  _as_ptr(c, ctypes.c_double), grad_mode, precision)
        self._check(rc, "set_grids")
        self.ngrids, self.precision = len(s), precision

    def set_kernel_table(self, qmesh, q_c, m_c, dk, phi, c_soft):
        q = np.ascontiguousarray(qmesh, dtype=np.float64)
        p = np.ascontiguousarray(phi, dtype=np.float64)
        nq, nk = q.size, p.shape[-1]
        if p.shape != (nq, nq, nk):
            raise ValueError("phi must be [nq, nq, nk]")
        self._check(self.lib.vdwnl_set_kernel_table(self.h, nq, _as_ptr(q, ctypes.c_double), float(q_c), int(m_c),
                                                    nk, float(dk), _as_ptr(p, ctypes.c_double), float(c_soft)),
                    "set_kernel_table")

    def energy_potential(self, n_ptr: int, v_ptr: int, stream: int = 0):
        """Device pointers in, (E_k, Delta E) out; v written in place."""
        E = np.zeros(2)
        self._check(self.lib.vdwnl_energy_potential(self.h, _vp(n_ptr), _vp(v_ptr), _as_ptr(E, ctypes.c_double),
                                                    _vp(stream)), "energy_potential")
        return float(E[0]), float(E[1])

    def energy_potential_noalloc(self, n_ptr: int, v_ptr: int, stream: int = 0):
        """As energy_potential, through the entry point that allocates nothing
        (its device structures in the library's static scratch buffer)."""
        E = np.zeros(2)
        self._check(self.lib.vdwnl_energy_potential_noalloc(self.h, _vp(n_ptr), _vp(v_ptr),
                                                            _as_ptr(E, ctypes.c_double), _vp(stream)),
                    "energy_potential_noalloc")
        return float(E[0]), float(E[1])

    def energy_potential_batched(self, n_ptrs, v_ptrs, stream: int = 0):
        nb = len(n_ptrs)
        na = (_vp * nb)(*[_vp(p) for p in n_ptrs])
        va = (_vp * nb)(*[_vp(p) for p in v_ptrs])
        E = np.zeros((nb, 2))
        self._check(self.lib.vdwnl_energy_potential_batched(self.h, nb, na, va, _as_ptr(E, ctypes.c_double),
                                                            _vp(stream)), "energy_potential_batched")
        return E

    def energy_potential_batched_async(self, n_ptrs, v_ptrs, e_dev_ptr: int, stream: int = 0):
        """Enqueue one evaluation; (E_k, Delta E) per grid land in the device
        array at e_dev_ptr (double [nb, 2]) on the stream."""
        nb = len(n_ptrs)
        na = (_vp * nb)(*[_vp(p) for p in n_ptrs])
        va = (_vp * nb)(*[_vp(p) for p in v_ptrs])
        self._check(self.lib.vdwnl_energy_potential_batched_async(self.h, nb, na, va, _vp(e_dev_ptr), _vp(stream)),
                    "energy_potential_batched_async")

    def set_graph(self, on: bool = True):
        self._check(self.lib.vdwnl_set_graph(self.h, 1 if on else 0), "set_graph")

    def set_functional(self, functional: int):
        """FUNCTIONAL_NONLOCAL (E_c^nl, v_nl) or FUNCTIONAL_VDW_DF (the whole E_xc, v_xc)."""
        self._check(self.lib.vdwnl_set_functional(self.h, int(functional)), "set_functional")

    def semilocal_energies(self):
        """[nb, 2]: E_x^GGA and E_c^LDA of every grid of the last evaluation."""
        nb, _ = self.info()
        E = np.zeros((nb, 2))
        self._check(self.lib.vdwnl_semilocal_energies(self.h, nb, _as_ptr(E, ctypes.c_double)),
                    "semilocal_energies")
        return E

    def autotune(self, n_ptrs, v_ptrs, reps: int = 2, stream: int = 0):
        nb = len(n_ptrs)
        na = (_vp * nb)(*[_vp(p) for p in n_ptrs])
        va = (_vp * nb)(*[_vp(p) for p in v_ptrs])
        self._check(self.lib.vdwnl_autotune(self.h, nb, na, va, int(reps), _vp(stream)), "autotune")

    def set_tiling(self, budgets):
        """budgets: dict with keys x, y20, yaux, z, zaux (bytes), or a sequence of 5."""
        if isinstance(budgets, dict):
            budgets = [budgets[k] for k in ("x", "y20", "yaux", "z", "zaux")]
        b = (ctypes.c_int64 * 5)(*[int(x) for x in budgets])
        self._check(self.lib.vdwnl_set_tiling(self.h, 5, b), "set_tiling")

    def set_contraction(self, unit: int):
        """CONTRACTION_VECTOR or CONTRACTION_MATRIX (the per-k contraction's unit)."""
        self._check(self.lib.vdwnl_set_schedule(self.h, SCHEDULE_CONTRACTION, int(unit)), "set_schedule")

    def get_contraction(self) -> int:
        v = _i32()
        self._check(self.lib.vdwnl_get_schedule(self.h, SCHEDULE_CONTRACTION, ctypes.byref(v)), "get_schedule")
        return int(v.value)

    def set_radix_orders(self, orders):
        """orders: dict with keys x, y20, yaux, z, zaux (0..5), or a sequence of 5."""
        if isinstance(orders, dict):
            orders = [orders[k] for k in RADIX_GROUPS]
        for i, v in enumerate(orders):
            self._check(self.lib.vdwnl_set_schedule(self.h, 1 + i, int(v)), "set_schedule")

    def get_radix_orders(self):
        out = {}
        for i, k in enumerate(RADIX_GROUPS):
            v = _i32()
            self._check(self.lib.vdwnl_get_schedule(self.h, 1 + i, ctypes.byref(v)), "get_schedule")
            out[k] = int(v.value)
        return out

    def get_tiling(self):
        """LDS budget (bytes) per pass group: x, y20, yaux, z, zaux."""
        b = (ctypes.c_int64 * 8)()
        n = self.lib.vdwnl_get_tiling(self.h, 8, b)
        if n < 0:
            raise VdwNlError(n, "get_tiling")
        return dict(zip(("x", "y20", "yaux", "z", "zaux"), [int(b[i]) for i in range(n)]))

    def debug_field(self, inst: int, which: int, dst_ptr: int, stream: int = 0):
        self._check(self.lib.vdwnl_debug_field(self.h, inst, which, _vp(dst_ptr), _vp(stream)), "debug_field")

    def debug_stage(self, inst: int, stage: int, dst_ptr: int, stream: int = 0):
        """One stage (STAGE_THETA, STAGE_THETA_K, STAGE_U_K, STAGE_U, STAGE_GRAD) of grid
        inst, recomputed from the last evaluation's density, into dst."""
        self._check(self.lib.vdwnl_debug_stage(self.h, inst, stage, _vp(dst_ptr), _vp(stream)), "debug_stage")

    def set_timing(self, on: bool = True):
        self._check(self.lib.vdwnl_set_timing(self.h, 1 if on else 0), "set_timing")

    def pass_order(self):
        """Kinds of the passes the planned gradient mode launches, in order."""
        k = (_i32 * 32)()
        n = self.lib.vdwnl_pass_order(self.h, 32, k)
        if n < 0:
            raise VdwNlError(n, "pass_order")
        return [int(k[i]) for i in range(n)]

    def pass_times(self):
        """{pass name: (total ms, evaluations)} accumulated since set_timing(True),
        for the passes of the planned gradient mode in launch order, then the
        energy reduction."""
        ms = np.zeros(32)
        calls = ctypes.c_int64()
        nk = self.lib.vdwnl_pass_times(self.h, 32, _as_ptr(ms, ctypes.c_double), ctypes.byref(calls))
        if nk < 0:
            raise VdwNlError(nk, "pass_times")
        kinds = self.pass_order() + [nk - 1]
        return {self.lib.vdwnl_pass_name(i).decode(): (float(ms[i]), calls.value) for i in kinds}

    def info(self):
        n = _i32()
        b = ctypes.c_int64()
        self._check(self.lib.vdwnl_info(self.h, ctypes.byref(n), ctypes.byref(b)), "info")
        return n.value, b.value
