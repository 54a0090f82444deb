"""TEST INFRASTRUCTURE (oracle side): the brute-force real-space evaluation of
the nonlocal energy, for comparison with the factorised (FFT) evaluation.

Only tests/ may use this module; nothing on the HIP product path imports it.

Eq. (Enl) on the grid, with the soft kernel phi_s of Eq. (PhiSoft) in place
of phi (the factorised method approximates exactly this, and adds Delta E of
Eq. (DEnl) for the difference phi - phi_s):

    E_bf = 1/2 dOmega^2 sum_i sum_j sum_L n_i n_j phi_s(q_i r, q_j r),
    r = |r_j - r_i + L|, images L of the periodic cell,

with no interpolation in q (each pair uses its own q0 values).  Pairs with
r < rcut are summed; beyond rcut the continuum limit of the image sum,
(1/Omega) Int_{r > rcut} 4 pi r^2 phi_s(q_i r, q_j r) dr, is added from the
tail integral of phi_s tabulated along each ray.  phi_s(d1, d2) comes from a table over the
angle atan(d2/d1) in [0.5, 45] degrees (phi is symmetric) and log D,
D = |(d1, d2)| in [d_s, 200], built from the oracle's double integral
(kernel_table.phi) with cubic interpolation in both variables; below d_s the
soft polynomial (its coefficients per angle from the value and radial slope
of phi at d_s, as in the kernel table); beyond D = 200 the asymptote.

Parity unpinned: the paper gives no number for how closely the factorised
evaluation reproduces this sum.  The difference has two parts, the
interpolation in q of Eq. (phi) and the real-space sampling of the kernel on
the grid (the FFT evaluation integrates the band-limited interpolant); the
tests record it and check that it shrinks as the grid is refined.
"""
from __future__ import annotations

import ctypes
import hashlib
import os

import numpy as np

from . import functional as F
from . import kernel_table as kt

TH0_DEG, DTH_DEG, NTH = 0.5, 0.5, 90          # angles 0.5 .. 45 degrees
NU, DMAX = 300, 200.0                           # log D from log(d_s) to log(200)


def _fn():
    lib = kt._lib()
    f = lib.oracle_bf_energy
    dp = ctypes.POINTER(ctypes.c_double)
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_double,
                  ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                  ctypes.c_double, ctypes.c_double, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                  ctypes.c_double, dp]
    return f


def soft_table(ds: float = 1.0, phi0: float = 0.5):
    """phi_s on the (angle, log D) mesh, and the soft coefficients per angle."""
    key = hashlib.sha256(repr(("bf3", ds, phi0, TH0_DEG, DTH_DEG, NTH, NU, DMAX)).encode()).hexdigest()[:16]
    path = os.path.join(kt._CACHE, "bf_%s.npz" % key)
    if os.path.exists(path):
        z = np.load(path)
        return {k: z[k] for k in z.files}
    th = np.deg2rad(TH0_DEG + DTH_DEG * np.arange(NTH))
    u = np.log(ds) + np.arange(NU) * (np.log(DMAX / ds) / (NU - 1))
    D = np.exp(u)
    c, s = np.cos(th)[:, None], np.sin(th)[:, None]
    tab = kt.phi((D[None, :] * c).ravel(), (D[None, :] * s).ravel()).reshape(NTH, NU)
    # value and radial slope at d_s on each ray (centred difference), Eq. (PhiSoft)
    h = 1e-3 * ds
    pm = kt.phi(((ds - h) * c).ravel(), ((ds - h) * s).ravel())
    pp = kt.phi(((ds + h) * c).ravel(), ((ds + h) * s).ravel())
    f, fp = tab[:, 0], (pp - pm) / (2.0 * h)
    p4 = (fp * ds / 2.0 - (f - phi0)) / ds ** 4
    p2 = (2.0 * (f - phi0) - fp * ds / 2.0) / ds ** 2
    # tail integrals 4 pi Int_{D_m}^inf D^2 phi dD per ray: trapezoid in u = log D
    # (dD = D du) on the mesh with the Euler-Maclaurin end corrections
    # -du^2/12 [f'(end) - f'(start)] (fourth order), the r^-6 asymptote beyond DMAX
    f_u = 4.0 * np.pi * D[None, :] ** 3 * tab
    du = u[1] - u[0]
    seg = 0.5 * du * (f_u[:, 1:] + f_u[:, :-1])
    cum = np.zeros_like(tab)
    cum[:, :-1] = np.cumsum(seg[:, ::-1], axis=1)[:, ::-1]
    fp = np.gradient(f_u, du, axis=1, edge_order=2)
    cum += du * du / 12.0 * (fp - fp[:, -1:])
    coef = kt.C_ASYM / (np.cos(th) ** 2 * np.sin(th) ** 2)
    cum += (-4.0 * np.pi * coef / (3.0 * DMAX ** 3))[:, None]
    out = dict(tab=tab, p2=p2, p4=p4, cum=cum, u0=np.array(u[0]), du=np.array(du), ds=np.array(ds),
               phi0=np.array(phi0))
    os.makedirs(kt._CACHE, exist_ok=True)
    np.savez(path + ".tmp.npz", **out)
    os.replace(path + ".tmp.npz", path)
    return out


def energy(n, cell, table, rcut: float = 12.0, n_min: float = F.N_MIN):
    """E_bf (soft kernel, real space) and Delta E of the same density; returns
    dict(E_bf, dE, pair, self, tail).  The local correction Delta E is the
    method's own (Eq. DEnl), so E_bf + dE compares with E_k + dE."""
    n = np.ascontiguousarray(n, dtype=np.float64)
    grad = F.gradient(n, cell)
    loc = F.theta_fields(n, grad, table, n_min=n_min)
    q = np.ascontiguousarray(np.where(n >= n_min, loc["q0"], 1.0))
    nn = np.ascontiguousarray(np.where(n >= n_min, n, 0.0))
    st = soft_table(float(table.get("ds", 1.0)), float(table.get("phi0", 0.5)))
    cellv = np.ascontiguousarray(cell, dtype=np.float64)
    out = np.zeros(3)
    dp = kt._ptr
    rc = _fn()(n.shape[0], n.shape[1], n.shape[2], dp(cellv), dp(nn), dp(q), float(rcut),
               NTH, float(np.deg2rad(TH0_DEG)), float(np.deg2rad(DTH_DEG)), NU, float(st["u0"]), float(st["du"]),
               DMAX, dp(np.ascontiguousarray(st["tab"])), dp(np.ascontiguousarray(st["p2"])),
               dp(np.ascontiguousarray(st["p4"])), dp(np.ascontiguousarray(st["cum"])), float(st["ds"]),
               float(st["phi0"]), kt.C_ASYM, dp(out))
    if rc != 0:
        raise RuntimeError("oracle_bf_energy failed: %d" % rc)
    dvol = float(np.prod(cell)) / n.size
    half = 0.5 * dvol * dvol
    dE = dvol * float(np.sum(loc["e_delta"]))
    return dict(E_bf=half * out.sum(), dE=dE, pair=half * out[0], self=half * out[1], tail=half * out[2])


def phi_soft(d1, d2, ds: float = 1.0, phi0: float = 0.5):
    """phi_s(d1, d2) of Eq. (PhiSoft) from the table (any shapes, broadcast)."""
    a, b = np.broadcast_arrays(np.asarray(d1, dtype=np.float64), np.asarray(d2, dtype=np.float64))
    a = np.ascontiguousarray(a.ravel())
    b = np.ascontiguousarray(b.ravel())
    st = soft_table(ds, phi0)
    out = np.zeros(a.size)
    lib = kt._lib()
    f = lib.oracle_phi_soft
    dp = ctypes.POINTER(ctypes.c_double)
    f.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                  ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp, dp, ctypes.c_double,
                  ctypes.c_double, ctypes.c_double, dp]
    p = kt._ptr
    rc = f(a.size, p(a), p(b), NTH, float(np.deg2rad(TH0_DEG)), float(np.deg2rad(DTH_DEG)), NU, float(st["u0"]),
           float(st["du"]), DMAX, p(np.ascontiguousarray(st["tab"])), p(np.ascontiguousarray(st["p2"])),
           p(np.ascontiguousarray(st["p4"])), float(st["ds"]), float(st["phi0"]), kt.C_ASYM, p(out))
    if rc != 0:
        raise RuntimeError("oracle_phi_soft failed: %d" % rc)
    return out.reshape(np.broadcast(np.asarray(d1), np.asarray(d2)).shape)

