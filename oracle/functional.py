"""Oracle: the nonlocal correlation energy E_c^nl and potential v_nl of a
density on a periodic grid (a cell of any shape), plain FP64 NumPy/SciPy.

TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It shares no code with the
HIP product path and never imports it.

The steps follow the paper's order.  Readings of points the paper leaves
open are marked READING; each has a line in the design notes.

 O1  gradient of n.  grad_mode 0: spectral differentiation (READING: the
     Nyquist multiplier set to zero so the derivative matrix is real
     antisymmetric).  grad_mode m = 1..4: the paper's own choice, finite
     differences on the same grid (Sec. on the potential, around Eq. (Vi);
     READING: the central formula with m points on each side of every axis,
     order 2m, periodic)
 O2  LDA correlation energy per electron (READING: Perdew-Wang 1992,
     spin-unpolarised)
 O3  q0(n, |grad n|) (READING: the Dion et al. form
     q0 = k_F - (4 pi/3) eps_c + (-Z_ab/36) |grad n|^2 / (k_F n^2), Z_ab = -0.8491)
 O4  saturation q0 <- h(q0, q_c), Eqs. (qsat)/(Sat)
 O5  cubic-spline cardinal functions p_a(q) on the q mesh, Eq. (fofx) and
     the text after it (READING: natural end conditions; below q_1 the
     linear continuation of the spline)
 O6  theta_a(r) = n(r) p_a(q0(r)), after Eq. (Eoffk); points with
     n < n_min contribute nothing (READING)
 O7  forward transforms c_a(G) = FFT(theta_a)/N
 O8  u_a(G) = sum_b phi_ab(|G|) c_b(G), phi_ab(|G|) by a natural cubic
     spline of the radial k table
 O9  E_k = (Omega/2) sum_G w_G sum_a Re(c_a(G)^* u_a(G)), Eq. (Eoffk) with
     the complex conjugate (READING), w_G = 1 on the k3 = 0 and k3 = N3/2
     planes of the half spectrum and 2 elsewhere
 O10 u_a(r_i) = sum_G u_a(G) exp(i G.r_i), Eqs. (epsilon)/(epsofk):
     u_ai = (1/dOmega) dE_k/dtheta_ai
 O11 Delta E = dOmega sum_i C_s n_i^2 / q0_i^3, Eqs. (DEnl)/(Depsnl)
 O12 local derivatives dtheta/dn, dtheta/dgrad n (and of e_Delta)
 O13 v_loc = sum_a u_a dtheta_a/dn + de/dn;  w = sum_a u_a dtheta_a/dgrad n + de/dgrad n
 O14 v = v_loc - sum_c D_c w_c, Eq. (Vi): the sum over j of
     w_j . d(grad n_j)/dn_i is the transpose of the (antisymmetric)
     derivative operator applied to w.
 O15 (xc_energy_potential only) the semilocal terms of Eq. (Exc):
     E_x^GGA (READING: the Zhang-Yang revPBE exchange, i.e. the PBE
     enhancement factor with kappa = 1.245) and E_c^LDA (the Perdew-Wang
     1992 LDA of O2).  Their energy densities depend on n and |grad n|^2
     only, so their derivatives add to v_loc and w of O13 and pass through
     the same gradient adjoint O14, as the paper does for the semilocal
     terms (Sec. on the potential, around Eq. (Vi)).
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline

# Perdew-Wang 1992 paramagnetic correlation (READING for the LDA of q0)
PW_A, PW_ALPHA1 = 0.031091, 0.21370
PW_BETA = (7.5957, 3.5876, 1.6382, 0.49294)
Z_AB = -0.8491
N_MIN = 1e-30


# ---------------------------------------------------------------- O2
def pw92(n):
    """eps_c(n) and d eps_c / dn (Hartree)."""
    n = np.asarray(n, dtype=np.float64)
    rs = (3.0 / (4.0 * np.pi * n)) ** (1.0 / 3.0)
    b1, b2, b3, b4 = PW_BETA
    srs = np.sqrt(rs)
    P = b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs
    dP = 0.5 * b1 / srs + b2 + 1.5 * b3 * srs + 2.0 * b4 * rs
    L = np.log1p(1.0 / (2.0 * PW_A * P))
    eps = -2.0 * PW_A * (1.0 + PW_ALPHA1 * rs) * L
    deps_drs = (-2.0 * PW_A * PW_ALPHA1 * L
                + 2.0 * PW_A * (1.0 + PW_ALPHA1 * rs) * dP / (P * (2.0 * PW_A * P + 1.0)))
    drs_dn = -rs / (3.0 * n)
    return eps, deps_drs * drs_dn


# ---------------------------------------------------------------- O15
# revPBE exchange (READING): e_x = n eps_x^unif(n) F_x(s), eps_x^unif =
# -3 k_F / (4 pi), s^2 = sigma / (4 k_F^2 n^2),
# F_x = 1 + kappa - kappa / (1 + mu s^2 / kappa); mu = beta pi^2 / 3 of PBE
REVPBE_KAPPA = 1.245
PBE_MU = 0.066725 * np.pi ** 2 / 3.0


def exchange_gga(n, sigma):
    """e_x per volume and its partials with respect to n and sigma = |grad n|^2."""
    n = np.asarray(n, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    kf = (3.0 * np.pi * np.pi * n) ** (1.0 / 3.0)
    e_unif = -3.0 * kf * n / (4.0 * np.pi)                  # n eps_x^unif
    ds2_dsigma = 1.0 / (4.0 * kf * kf * n * n)
    s2 = sigma * ds2_dsigma
    den = 1.0 + PBE_MU * s2 / REVPBE_KAPPA
    fx = 1.0 + REVPBE_KAPPA - REVPBE_KAPPA / den
    dfx = PBE_MU / (den * den)                               # dF_x / ds^2
    # d e_unif/dn = (4/3) e_unif / n;  d s^2/dn = -(8/3) s^2 / n
    de_dn = (4.0 / 3.0) * e_unif / n * fx - (8.0 / 3.0) * e_unif * dfx * s2 / n
    de_ds = e_unif * dfx * ds2_dsigma
    return e_unif * fx, de_dn, de_ds


def correlation_lda(n):
    """e_c = n eps_c(n) per volume (O2) and de_c/dn."""
    eps, deps = pw92(n)
    return n * eps, eps + n * deps


# ---------------------------------------------------------------- O3
def q0_unsaturated(n, sigma):
    """q0 and its partials with respect to n and sigma = |grad n|^2."""
    n = np.asarray(n, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    kf = (3.0 * np.pi * np.pi * n) ** (1.0 / 3.0)
    eps, deps = pw92(n)
    zg = -Z_AB / 36.0
    q = kf - (4.0 * np.pi / 3.0) * eps + zg * sigma / (kf * n * n)
    dq_dn = kf / (3.0 * n) - (4.0 * np.pi / 3.0) * deps - (7.0 / 3.0) * zg * sigma / (kf * n ** 3)
    dq_ds = zg / (kf * n * n)
    return q, dq_dn, dq_ds


# ---------------------------------------------------------------- O4
def saturate(q, qc, mc):
    """h(q, q_c) of Eq. (Sat) and dh/dq."""
    y = np.asarray(q, dtype=np.float64) / qc
    S = np.zeros_like(y)
    dS = np.zeros_like(y)   # dS/dy = sum_{m=0}^{mc-1} y^m
    ym = np.ones_like(y)
    with np.errstate(over="ignore", invalid="ignore"):   # (huge y: S overflows and saturates below)
        for m in range(1, mc + 1):
            dS += ym
            ym = ym * y
            S += ym / m
    big = S > 700.0
    e = np.exp(-np.where(big, 0.0, S))
    h = np.where(big, qc, qc * (1.0 - e))
    dh = np.where(big, 0.0, e * dS)
    return h, dh


# ---------------------------------------------------------------- O5
class CardinalSplines:
    """p_a(q), p'_a(q): the natural cubic spline through unit data e_a."""

    def __init__(self, qmesh):
        self.q = np.asarray(qmesh, dtype=np.float64)
        self.nq = self.q.size
        self._spl = CubicSpline(self.q, np.eye(self.nq), bc_type="natural", extrapolate=True)
        self._d1 = self._spl.derivative(1)
        self._p1 = self._spl(self.q[0])
        self._dp1 = self._d1(self.q[0])

    def __call__(self, q):
        """(p [nq, ...], dp/dq [nq, ...]) for q of any shape."""
        q = np.asarray(q, dtype=np.float64)
        flat = q.ravel()
        p = self._spl(flat)              # [npts, nq]
        dp = self._d1(flat)
        low = flat < self.q[0]
        if np.any(low):                  # linear continuation below q_1
            p[low] = self._p1[None, :] + (flat[low] - self.q[0])[:, None] * self._dp1[None, :]
            dp[low] = self._dp1[None, :]
        return (p.T.reshape((self.nq,) + q.shape), dp.T.reshape((self.nq,) + q.shape))


# ---------------------------------------------------------------- cells
def lattice(cell):
    """Rows a_1, a_2, a_3 of the cell (bohr): three orthorhombic lengths or a
    3 x 3 matrix of cell vectors.  Grid point i sits at sum_c (i_c/N_c) a_c."""
    c = np.asarray(cell, dtype=np.float64)
    return np.diag(c) if c.shape == (3,) else c.reshape(3, 3)


def reciprocal(cell):
    """Rows b_1, b_2, b_3 with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(lattice(cell)).T


def volume(cell):
    return float(abs(np.linalg.det(lattice(cell))))


def _freqs(shape, half):
    """Integer frequencies m_c on the (half) FFT grid (Nyquist as -N/2, or
    +N/2 on the last axis of the half spectrum) and the Nyquist flags."""
    ms, nyq = [], []
    for c in range(3):
        npts = shape[c]
        if c == 2 and half:
            m = np.arange(npts // 2 + 1, dtype=np.float64)
        else:
            m = np.fft.fftfreq(npts, d=1.0 / npts)
        ms.append(m)
        nyq.append((npts % 2 == 0) & (np.abs(m) == npts // 2))
    return ms, nyq


# ---------------------------------------------------------------- O1 / O14
def wavevectors(shape, cell, half=True):
    """Cartesian components of G = sum_c m_c b_c on the (half) FFT grid, with
    a Nyquist index m_c taken as zero (the derivative along that lattice
    axis vanishes there, so the operator stays real antisymmetric)."""
    B = reciprocal(cell)
    ms, nyq = _freqs(shape, half)
    mz = [np.where(nq, 0.0, m) for m, nq in zip(ms, nyq)]
    M = np.meshgrid(*mz, indexing="ij")
    return [M[0] * B[0, x] + M[1] * B[1, x] + M[2] * B[2, x] for x in range(3)]


def gradient(n, cell):
    """grad n by spectral differentiation (3 x shape)."""
    shape = n.shape
    nh = np.fft.rfftn(n)
    g = wavevectors(shape, cell)
    return np.stack([np.fft.irfftn(1j * g[c] * nh, s=shape, axes=(0, 1, 2)) for c in range(3)])


def divergence(w, cell):
    """sum_c D_c w_c with the same derivative operator as ``gradient``."""
    shape = w.shape[1:]
    g = wavevectors(shape, cell)
    acc = np.zeros(tuple(shape[:2]) + (shape[2] // 2 + 1,), dtype=np.complex128)
    for c in range(3):
        acc += 1j * g[c] * np.fft.rfftn(w[c])
    return np.fft.irfftn(acc, s=shape, axes=(0, 1, 2))


def fd_weights(m):
    """Weights c_s (s = 1..m) of the central first-derivative formula
    f'(x) ~ sum_s c_s (f(x + s h) - f(x - s h)) / h.  Expanding the right side
    in a Taylor series, the coefficient of h^(2k-2) f^(2k-1)(x) is
    sum_s c_s 2 s^(2k-1) / (2k-1)!; the formula has order 2m when it is 1 for
    k = 1 and 0 for k = 2..m, an m x m linear system solved here."""
    s = np.arange(1, m + 1, dtype=np.float64)
    A = np.array([2.0 * s ** (2 * k - 1) for k in range(1, m + 1)])
    rhs = np.zeros(m)
    rhs[0] = 1.0
    return np.linalg.solve(A, rhs)


def _stencil(f, ax, m):
    """sum_s c_s (f_{i + s e_ax} - f_{i - s e_ax}) on the periodic grid (unit spacing)."""
    c = fd_weights(m)
    out = np.zeros_like(f)
    for s in range(1, m + 1):
        out += c[s - 1] * (np.roll(f, -s, axis=ax) - np.roll(f, s, axis=ax))
    return out


def fd_metric(shape, cell):
    """W[c][x] = N_c b_c,x / (2 pi): grad n = sum_c W[c] d n/d(i_c), the chain
    rule from the grid index along lattice axis c to Cartesian x (for an
    orthorhombic cell W = diag(1 / h_c))."""
    B = reciprocal(cell)
    return np.array([shape[c] * B[c] / (2.0 * np.pi) for c in range(3)])


def gradient_fd(n, cell, m):
    """grad n by the central differences of ``fd_weights(m)`` along the three
    lattice axes of the periodic grid, d_c n_i = sum_s c_s (n_{i + s e_c} -
    n_{i - s e_c}), combined into Cartesian components with ``fd_metric``
    (3 x shape)."""
    W = fd_metric(n.shape, cell)
    d = [_stencil(n, c, m) for c in range(3)]
    return np.stack([W[0, x] * d[0] + W[1, x] * d[1] + W[2, x] * d[2] for x in range(3)])


def divergence_fd(w, cell, m):
    """The adjoint of ``gradient_fd`` with the sign flipped: sum_c D_c q_c with
    q_c = sum_x W[c][x] w_x (D_c antisymmetric)."""
    W = fd_metric(w.shape[1:], cell)
    return sum(_stencil(W[c, 0] * w[0] + W[c, 1] * w[1] + W[c, 2] * w[2], c, m) for c in range(3))


def gmod_half(shape, cell):
    """|G| on the half spectrum, |G|^2 = sum_cd m_c m_d (b_c . b_d).  A Nyquist
    index stands for both signs +-N_c/2, which give different |G| in a
    non-orthogonal cell (READING): |G|^2 there is the mean over the two, i.e.
    the cross terms of that axis are dropped.  The multiplier then takes the
    same value at G and -G, as a real transform needs; in an orthorhombic
    cell nothing changes (no cross terms)."""
    B = reciprocal(cell)
    Mt = B @ B.T
    ms, nyq = _freqs(shape, True)
    m = np.meshgrid(*ms, indexing="ij")
    q = np.meshgrid(*[(~nq).astype(np.float64) for nq in nyq], indexing="ij")
    g2 = sum(Mt[c, c] * m[c] * m[c] for c in range(3))
    for c in range(3):
        for d in range(c + 1, 3):
            g2 = g2 + 2.0 * Mt[c, d] * m[c] * m[d] * q[c] * q[d]
    return np.sqrt(np.maximum(g2, 0.0))


def half_weights(shape):
    """w_G of the half spectrum: 1 on k3 = 0 and (N3 even) k3 = N3/2, else 2."""
    n3h = shape[2] // 2 + 1
    w = np.full(n3h, 2.0)
    w[0] = 1.0
    if shape[2] % 2 == 0:
        w[-1] = 1.0
    return w


# ---------------------------------------------------------------- O5/O6/O12
def theta_fields(n, grad, table, n_min=N_MIN):
    """theta_a, dtheta_a/dn, the scalar g_a with dtheta_a/dgrad n = g_a grad n,
    and e_Delta with its derivatives; every local quantity of the method."""
    n = np.asarray(n, dtype=np.float64)
    sigma = np.sum(grad * grad, axis=0)
    ok = n >= n_min
    ns = np.where(ok, n, 1.0)
    q_raw, dq_dn, dq_ds = q0_unsaturated(ns, np.where(ok, sigma, 0.0))
    q0, Q = saturate(q_raw, table["qc"], int(table.get("mc", 12)))
    spl = CardinalSplines(table["qmesh"])
    p, dp = spl(q0)
    theta = ns * p
    dtheta_dn = p + ns * dp * Q * dq_dn
    g = 2.0 * ns * dp * Q * dq_ds      # dtheta_a/dgrad n = g_a * grad n
    cs = table["c_soft"]
    e_delta = cs * ns * ns / q0 ** 3
    de_dn = 2.0 * cs * ns / q0 ** 3 - 3.0 * cs * ns * ns / q0 ** 4 * Q * dq_dn
    ge = -6.0 * cs * ns * ns / q0 ** 4 * Q * dq_ds
    z = ~ok
    for arr in (theta, dtheta_dn, g):
        arr[:, z] = 0.0
    for arr in (e_delta, de_dn, ge):
        arr[z] = 0.0
    return dict(q0=np.where(ok, q0, 0.0), theta=theta, dtheta_dn=dtheta_dn, g=g,
                e_delta=e_delta, de_dn=de_dn, ge=ge)


# ---------------------------------------------------------------- O8
_spline_cache: dict = {}


def _table_spline(table):
    """Natural cubic spline in k of every (a, b) column of the radial table."""
    key = id(table["phi"])
    hit = _spline_cache.get(key)
    if hit is None or hit[0] is not table["phi"]:
        nq, nk = table["phi"].shape[0], table["phi"].shape[2]
        k = np.arange(nk) * table["dk"]
        spl = CubicSpline(k, table["phi"].reshape(nq * nq, nk).T, bc_type="natural")
        hit = (table["phi"], spl, k[-1])
        _spline_cache.clear()
        _spline_cache[key] = hit
    return hit[1], hit[2]


def kernel_at(gmod, table):
    """phi_ab(|G|) [..., nq, nq] by a natural cubic spline of the radial table,
    evaluated once per distinct |G| value."""
    nq = table["phi"].shape[0]
    spl, kmax = _table_spline(table)
    if gmod.max() > kmax:
        raise ValueError("|G| beyond the radial kernel table")
    uniq, inv = np.unique(gmod.ravel(), return_inverse=True)
    vals = spl(uniq).reshape(uniq.size, nq, nq)
    return vals, inv.reshape(gmod.shape)


# ---------------------------------------------------------------- O1..O14
def energy_potential(n, cell, table, n_min=N_MIN, return_parts=False, grad_mode=0):
    """(E_k, Delta E, v) for the density n [N1, N2, N3] in the cell (bohr:
    three orthorhombic lengths or the 3 x 3 matrix of cell vectors);
    grad_mode 0: spectral gradient, m = 1..4: central differences of order 2m."""
    parts = _evaluate(n, cell, table, n_min, grad_mode, semilocal=False)
    if return_parts:
        return parts
    return parts["E_k"], parts["dE"], parts["v"]


def xc_energy_potential(n, cell, table, n_min=N_MIN, return_parts=False, grad_mode=0):
    """The whole functional of Eq. (Exc): (E_k, Delta E, E_x^GGA, E_c^LDA, v_xc)
    with v_xc = v_nl + v_x + v_c^LDA (O15); arguments as energy_potential."""
    parts = _evaluate(n, cell, table, n_min, grad_mode, semilocal=True)
    if return_parts:
        return parts
    return parts["E_k"], parts["dE"], parts["E_x"], parts["E_c"], parts["v"]


def _evaluate(n, cell, table, n_min, grad_mode, semilocal):
    n = np.asarray(n, dtype=np.float64)
    shape = n.shape
    N = n.size
    omega = volume(cell)
    dvol = omega / N
    if grad_mode not in (0, 1, 2, 3, 4):
        raise ValueError("grad_mode must be 0 (spectral) or 1..4 (central differences)")
    if grad_mode == 0:
        grad = gradient(n, cell)                               # O1
    else:
        grad = gradient_fd(n, cell, grad_mode)
    loc = theta_fields(n, grad, table, n_min)                  # O2-O6, O12
    theta = loc["theta"]
    nq = theta.shape[0]
    chat = np.stack([np.fft.rfftn(theta[a]) for a in range(nq)]) / N     # O7
    vals, shell = kernel_at(gmod_half(shape, cell), table)
    uhat = np.zeros_like(chat)
    for a in range(nq):                                        # O8
        for b in range(nq):
            uhat[a] += vals[:, a, b][shell] * chat[b]
    w = half_weights(shape)
    ek = 0.5 * omega * np.sum(w * np.sum(np.real(np.conj(chat) * uhat), axis=0))   # O9
    u = np.stack([np.fft.irfftn(uhat[a], s=shape, axes=(0, 1, 2)) * N for a in range(nq)])       # O10
    de = dvol * np.sum(loc["e_delta"])                         # O11
    v_loc = np.sum(u * loc["dtheta_dn"], axis=0) + loc["de_dn"]                  # O13
    gsc = np.sum(u * loc["g"], axis=0) + loc["ge"]
    sl = {}
    if semilocal:                                              # O15
        ok = n >= n_min
        ns = np.where(ok, n, 1.0)
        sigma = np.where(ok, np.sum(grad * grad, axis=0), 0.0)
        ex, dex_dn, dex_ds = exchange_gga(ns, sigma)
        ec, dec_dn = correlation_lda(ns)
        z = ~ok
        for arr in (ex, dex_dn, dex_ds, ec, dec_dn):
            arr[z] = 0.0
        v_loc = v_loc + dex_dn + dec_dn
        gsc = gsc + 2.0 * dex_ds                               # de/dgrad n = 2 de/dsigma grad n
        sl = dict(E_x=dvol * np.sum(ex), E_c=dvol * np.sum(ec))
    wvec = gsc[None] * grad
    if grad_mode == 0:
        v = v_loc - divergence(wvec, cell)                     # O14
    else:
        v = v_loc - divergence_fd(wvec, cell, grad_mode)
    return dict(E_k=ek, dE=de, v=v, u=u, chat=chat, uhat=uhat, grad=grad, v_loc=v_loc,
                w=wvec, **sl, **loc)
