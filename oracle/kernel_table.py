"""Oracle: the vdW-DF kernel and its radial k-space table (FP64).

TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  The HIP product path never
imports, links or runs anything under ``oracle/``.

What it computes, in the paper's order:

* ``phi(d1, d2)``: the universal kernel of Eq. (Enl).  Its form is not in the
  paper; the reading used is Dion et al. (2004) (double integral over the
  plane-wave variables a, b; see ``dion_kernel.c``), validated against what
  the paper *does* state: phi integrates to zero over a uniform density
  and decays as r^-6 at large separation.
* ``soft``: the softened kernel of Eq. (PhiSoft): on each ray of fixed d2/d1,
  phi_s = phi0 + phi2 D^2 + phi4 D^4 for D = sqrt(d1^2 + d2^2) < d_s, with
  phi2, phi4 fixed by matching value and slope at D = d_s.
* ``c_soft``: the LDA-like correction constant of Eqs. (DEnl)/(Depsnl):
  Delta E = Int n^2 C_s / q0^3 with C_s = 1/2 Int_0^{d_s} 4 pi d^2
  [phi(d,d) - phi_s(d,d)] dd (the integrand vanishes beyond d = d_s/sqrt 2).
* ``kernel_table``: phi_ab(k) = 4 pi Int r^2 j0(k r) phi_s(q_a r, q_b r) dr on
  the radial mesh k_j = j dk, the transform that the text after Eq. (Eoffk)
  says is stored on a radial k mesh for interpolation.  With Q = |(q_a, q_b)|
  and D = Q r this is Q^-3 Psi(k/Q) where Psi(kappa) = 4 pi Int D^2
  j0(kappa D) Phi_ray(D) dD is the transform of the kernel along the ray.

Numerical choices (none of them affects GPU/oracle parity, which always
feeds the same table to both sides):

* a-integration: composite 6-point Gauss-Legendre, geometric panels from
  1e-5 up to 2 pi and panels of width pi/2 beyond, with a smooth cutoff of
  the oscillatory large-a tail; the upper limit grows with max(d1, d2)
  because the integrand settles into its oscillatory tail only for a >> d.
* along each ray, phi is sampled at log-spaced D in [d_s, X] and splined in
  log D (phi itself up to D = 10, log(-phi) beyond, where phi < 0); beyond
  X = min(20/min(cos, sin), 2000) the r^-6 asymptote -C/(d1^2 d2^2 (d1^2+d2^2)),
  C = 12 (4 pi/9)^3, is used and its transform is added in closed form
  (sine/cosine integrals).  The asymptote needs both d1 and d2 large: on the
  most skewed ray of the default mesh (q_b/q_a = 100) phi/asymptote is 1.038
  at d1 = 4, 1.0000 from d1 = 12 on, so X reaches d1 = 20 there (an end at
  D = 400 had left 1.2e-4 of that pair's largest table value at k = 0).
* radial transform: trapezoid rule on a uniform D mesh (step d_s/200, the
  soft-region boundary is a node).
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
import subprocess

import numpy as np
from scipy.interpolate import CubicSpline
from scipy.special import sici

GAMMA = 4.0 * np.pi / 9.0
C_ASYM = 12.0 * GAMMA ** 3  # r^-6 coefficient of phi at large d1, d2

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_CACHE = os.path.join(_HERE, "_cache")
_SO = os.path.join(_BUILD, "liboracle_dion.so")
_SRC = os.path.join(_HERE, "dion_kernel.c")

_dp = ctypes.POINTER(ctypes.c_double)


def build_c(force: bool = False) -> str:
    """Compile the oracle's plain-C helpers with gcc (FP64, OpenMP)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        _lib_handle = ctypes.CDLL(build_c())
        _lib_handle.oracle_dion_phi.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp, _dp]
        _lib_handle.oracle_radial_sine_sum.argtypes = [ctypes.c_int, ctypes.c_double, _dp,
                                                       ctypes.c_int, _dp, _dp]
    return _lib_handle


def _ptr(x):
    return x.ctypes.data_as(_dp)


# --------------------------------------------------------------------------
# phi(d1, d2)
# --------------------------------------------------------------------------

def _smooth_cutoff(a, a1, a2):
    """1 below a1, 0 above a2, C-infinity in between (exp(-1/t) smoothstep)."""
    t = np.clip((a - a1) / (a2 - a1), 0.0, 1.0)

    def f(u):
        return np.where(u > 0.0, np.exp(-1.0 / np.maximum(u, 1e-300)), 0.0)

    return 1.0 - f(t) / (f(t) + f(1.0 - t))


def a_mesh(n_wide: int, n_gl: int = 6, a_min: float = 1e-5, taper: float = 0.3):
    """Quadrature for Int_0^inf da: composite Gauss-Legendre on [0, A],
    A = 2 pi + n_wide pi/2, geometric panels below 2 pi, width pi/2 above.

    At large a the integrand is a trigonometric function of a times a smooth
    decaying factor, so the sharp cut at A is replaced by a smooth cutoff
    from taper*A to A; the truncation error then falls off much faster than
    the ~A^-2 of a sharp cut.
    """
    x, w = np.polynomial.legendre.leggauss(n_gl)
    edges = [0.0]
    e = a_min
    while e < 2.0 * np.pi:
        edges.append(e)
        e *= 2.0
    edges.append(2.0 * np.pi)
    for k in range(1, n_wide + 1):
        edges.append(2.0 * np.pi + k * np.pi / 2.0)
    nodes, weights = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        nodes.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        weights.append(0.5 * (hi - lo) * w)
    a = np.concatenate(nodes)
    wt = np.concatenate(weights)
    if taper is not None:
        wt = wt * _smooth_cutoff(a, taper * a[-1], a[-1])
    return a, wt


# (upper bound on max(d1, d2), number of pi/2 panels beyond 2 pi)
_BANDS = ((25.0, 100), (80.0, 250), (250.0, 700), (np.inf, 1100))
_meshes: dict = {}


def _mesh(n_wide):
    if n_wide not in _meshes:
        _meshes[n_wide] = a_mesh(n_wide)
    return _meshes[n_wide]


def phi(d1, d2, n_wide: int | None = None) -> np.ndarray:
    """The kernel phi(d1, d2) of Eq. (Enl) by direct double integration."""
    d1 = np.atleast_1d(np.asarray(d1, dtype=np.float64))
    d2 = np.atleast_1d(np.asarray(d2, dtype=np.float64))
    d1, d2 = np.broadcast_arrays(d1, d2)
    d1 = np.ascontiguousarray(d1.ravel())
    d2 = np.ascontiguousarray(d2.ravel())
    out = np.zeros(d1.size)
    m = np.maximum(d1, d2)
    lo = -np.inf
    bands = _BANDS if n_wide is None else ((np.inf, n_wide),)
    for bound, nw in bands:
        idx = np.nonzero((m > lo) & (m <= bound))[0]
        lo = bound
        if idx.size == 0:
            continue
        a, w = _mesh(nw)
        x1 = np.ascontiguousarray(d1[idx])
        x2 = np.ascontiguousarray(d2[idx])
        o = np.zeros(idx.size)
        rc = _lib().oracle_dion_phi(a.size, _ptr(a), _ptr(w), idx.size, _ptr(x1), _ptr(x2), _ptr(o))
        if rc != 0:
            raise RuntimeError("oracle_dion_phi failed: %d" % rc)
        out[idx] = o
    return out


def phi_asym(d1, d2):
    """Large-separation form of phi: -C / (d1^2 d2^2 (d1^2 + d2^2))."""
    d1 = np.asarray(d1, dtype=np.float64)
    d2 = np.asarray(d2, dtype=np.float64)
    return -C_ASYM / (d1 * d1 * d2 * d2 * (d1 * d1 + d2 * d2))


# --------------------------------------------------------------------------
# the soft kernel of Eq. (PhiSoft) along one ray
# --------------------------------------------------------------------------

class Ray:
    """phi_s along the ray d1 = D cos(theta), d2 = D sin(theta)."""

    D_SPLIT = 10.0  # phi < 0 on every ray beyond this D: spline log(-phi) there

    def __init__(self, cos_t: float, sin_t: float, ds: float, phi0: float):
        self.c, self.s = float(cos_t), float(sin_t)
        self.ds, self.phi0 = float(ds), float(phi0)
        cmin = min(self.c, self.s)
        self.X = min(20.0 / cmin, 2000.0)
        # value and slope at d_s (slope by a centred difference of the exact kernel)
        h = 1e-3 * ds
        p = phi(np.array([ds - h, ds, ds + h]) * self.c, np.array([ds - h, ds, ds + h]) * self.s)
        f, fp = p[1], (p[2] - p[0]) / (2.0 * h)
        self.phi_ds, self.dphi_ds = f, fp
        # Eq. (PhiSoft): phi0 + phi2 ds^2 + phi4 ds^4 = f ; 2 phi2 ds + 4 phi4 ds^3 = fp
        self.phi4 = (fp * ds / 2.0 - (f - phi0)) / ds ** 4
        self.phi2 = (2.0 * (f - phi0) - fp * ds / 2.0) / ds ** 2
        # samples of the exact kernel on [d_s, X]
        n1 = max(int(np.ceil(300 * np.log10(self.D_SPLIT / ds))), 8)
        Da = np.geomspace(ds, self.D_SPLIT, n1 + 1)
        n2 = max(int(np.ceil(60 * np.log10(self.X / self.D_SPLIT))), 4)
        Db = np.geomspace(self.D_SPLIT, self.X, n2 + 1)
        va = phi(Da * self.c, Da * self.s)
        vb = phi(Db * self.c, Db * self.s)
        if np.any(vb >= 0):
            raise RuntimeError("kernel not negative beyond D=%g on ray %g" % (self.D_SPLIT, self.s / self.c))
        self._spl_a = CubicSpline(np.log(Da), va, bc_type="not-a-knot")
        self._spl_b = CubicSpline(np.log(Db), np.log(-vb), bc_type="not-a-knot")
        self.asym_coef = C_ASYM / (self.c ** 2 * self.s ** 2)  # phi ~ -asym_coef / D^6

    def soft_poly(self, D):
        D2 = D * D
        return self.phi0 + self.phi2 * D2 + self.phi4 * D2 * D2

    def __call__(self, D):
        """phi_s on the ray (soft polynomial, splined exact kernel, asymptote)."""
        D = np.asarray(D, dtype=np.float64)
        out = np.empty_like(D)
        m0 = D < self.ds
        m1 = (~m0) & (D <= self.D_SPLIT)
        m2 = (D > self.D_SPLIT) & (D <= self.X)
        m3 = D > self.X
        out[m0] = self.soft_poly(D[m0])
        out[m1] = self._spl_a(np.log(D[m1]))
        out[m2] = -np.exp(self._spl_b(np.log(D[m2])))
        out[m3] = -self.asym_coef / D[m3] ** 6
        return out

    def monotone_soft(self) -> bool:
        """True when phi_s has no interior extremum on (0, d_s)."""
        return self.phi2 * (self.phi2 + 2.0 * self.phi4 * self.ds ** 2) > 0.0

    def transform(self, kappa: np.ndarray, step: float | None = None) -> np.ndarray:
        """Psi(kappa) = 4 pi Int_0^inf D^2 j0(kappa D) phi_s(D) dD."""
        kappa = np.ascontiguousarray(kappa, dtype=np.float64)
        dD = self.ds / 200.0 if step is None else step
        nd = int(round(self.X / dD)) + 1
        X = (nd - 1) * dD
        D = np.arange(nd) * dD
        g = np.ascontiguousarray(D * self(D))
        out = np.zeros(kappa.size)
        pos = kappa > 0
        if np.any(pos):
            kp = np.ascontiguousarray(kappa[pos])
            tmp = np.zeros(kp.size)
            rc = _lib().oracle_radial_sine_sum(nd, dD, _ptr(g), kp.size, _ptr(kp), _ptr(tmp))
            if rc != 0:
                raise RuntimeError("oracle_radial_sine_sum failed")
            out[pos] = 4.0 * np.pi * dD * tmp / kp
        if np.any(~pos):
            w = np.ones(nd)
            w[0] = w[-1] = 0.5
            out[~pos] = 4.0 * np.pi * dD * np.sum(w * D * g)
        out += _tail_transform(kappa, X, self.asym_coef)
        return out


def _tail_transform(kappa, X, coef):
    """4 pi Int_X^inf D^2 j0(kappa D) (-coef / D^6) dD in closed form.

    With t = kappa D this is -4 pi coef kappa^3 J5(kappa X), where
    J_n(x) = Int_x^inf sin t / t^n dt and K_n(x) = Int_x^inf cos t / t^n dt obey
    J_n = sin x / ((n-1) x^(n-1)) + K_{n-1} / (n-1),
    K_n = cos x / ((n-1) x^(n-1)) - J_{n-1} / (n-1),
    J_1 = pi/2 - Si(x), K_1 = -Ci(x).
    """
    kappa = np.asarray(kappa, dtype=np.float64)
    out = np.full(kappa.shape, -4.0 * np.pi * coef / (3.0 * X ** 3))
    pos = kappa > 0
    if np.any(pos):
        x = kappa[pos] * X
        si, ci = sici(x)
        J = np.pi / 2.0 - si
        K = -ci
        for n in range(2, 6):
            Jn = np.sin(x) / ((n - 1) * x ** (n - 1)) + K / (n - 1)
            Kn = np.cos(x) / ((n - 1) * x ** (n - 1)) - J / (n - 1)
            J, K = Jn, Kn
        out[pos] = -4.0 * np.pi * coef * kappa[pos] ** 3 * J
    return out


# --------------------------------------------------------------------------
# C_s of Eq. (Depsnl)
# --------------------------------------------------------------------------

def c_soft(ds: float, phi0: float) -> float:
    """C_s = 1/2 Int_0^{d_s/sqrt2} 4 pi d^2 [phi(d,d) - phi_s(d,d)] dd."""
    ray = Ray(np.sqrt(0.5), np.sqrt(0.5), ds, phi0)
    x, w = np.polynomial.legendre.leggauss(12)
    edges = [0.0] + list(np.geomspace(1e-6, ds / np.sqrt(2.0), 30))
    d, wt = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        d.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        wt.append(0.5 * (hi - lo) * w)
    d = np.concatenate(d)
    wt = np.concatenate(wt)
    hard = phi(d, d)
    soft = ray.soft_poly(np.sqrt(2.0) * d)
    return float(0.5 * np.sum(wt * 4.0 * np.pi * d * d * (hard - soft)))


# --------------------------------------------------------------------------
# the q mesh and the table
# --------------------------------------------------------------------------

def log_qmesh(nq: int = 20, q1: float = 0.05, qc: float = 5.0, lam: float = 1.17) -> np.ndarray:
    """q_a with (q_{a+1} - q_a) = lam (q_a - q_{a-1}), q_1 = q1, q_N = q_c."""
    steps = lam ** np.arange(nq - 1)
    delta1 = (qc - q1) / steps.sum()
    q = q1 + np.concatenate([[0.0], np.cumsum(delta1 * steps)])
    q[-1] = qc
    return q


DEFAULTS = dict(nq=20, q1=0.05, qc=5.0, lam=1.17, nk=6401, dk=0.005, ds=1.0, phi0=0.5)


def kernel_table(nq=20, q1=0.05, qc=5.0, lam=1.17, nk=6401, dk=0.005, ds=1.0, phi0=0.5,
                 cache: bool = True) -> dict:
    """phi_ab(k_j) on k_j = j dk for the log q mesh, plus C_s.

    Returns a dict with ``qmesh`` [nq], ``phi`` [nq, nq, nk] (symmetric in a, b),
    ``dk``, ``nk``, ``c_soft``, ``ds``, ``phi0``.
    """
    params = dict(nq=nq, q1=q1, qc=qc, lam=lam, nk=nk, dk=dk, ds=ds, phi0=phi0, version=4)
    key = hashlib.sha256(json.dumps(params, sort_keys=True).encode()).hexdigest()[:16]
    path = os.path.join(_CACHE, "table_%s.npz" % key)
    if cache and os.path.exists(path):
        z = np.load(path)
        return {k: (z[k] if z[k].ndim else z[k].item()) for k in z.files}
    q = log_qmesh(nq, q1, qc, lam)
    k = np.arange(nk) * dk
    tab = np.zeros((nq, nq, nk))
    for a in range(nq):
        for b in range(a, nq):
            Q = np.hypot(q[a], q[b])
            ray = Ray(q[a] / Q, q[b] / Q, ds, phi0)
            if not ray.monotone_soft():
                raise RuntimeError("soft kernel has an interior extremum; raise phi0")
            tab[a, b] = tab[b, a] = ray.transform(k / Q) / Q ** 3
    out = dict(qmesh=q, phi=tab, dk=float(dk), nk=int(nk), c_soft=c_soft(ds, phi0),
               ds=float(ds), phi0=float(phi0), qc=float(qc))
    if cache:
        os.makedirs(_CACHE, exist_ok=True)
        tmp = path + ".tmp%d.npz" % os.getpid()
        np.savez(tmp, **out)
        os.replace(tmp, path)
    return out
