"""Pins of the oracle's semilocal terms of Eq. (Exc), E_x^GGA (revPBE
exchange) and E_c^LDA, and of the whole functional's potential: the
uniform-gas closed forms (Dirac exchange energy and potential), the limits
of the enhancement factor, the exact uniform-coordinate scaling of GGA
exchange, additivity with the nonlocal part, and v_xc = (1/dOmega) dE_xc/dn_i
by central differences (Eq. (Vi))."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import functional as F


def _zero_table(table):
    t = dict(table)
    t["phi"] = np.zeros_like(table["phi"])
    t["c_soft"] = 0.0
    return t


def _fx(s):
    """F_x(s) as the ratio of e_x at gradient s to e_x at zero gradient."""
    n = 0.3
    kf = (3 * math.pi ** 2 * n) ** (1 / 3)
    sigma = 4 * kf * kf * n * n * np.asarray(s, dtype=float) ** 2
    e, _, _ = F.exchange_gga(np.full_like(sigma, n), sigma)
    e0, _, _ = F.exchange_gga(np.array([n]), np.array([0.0]))
    return e / e0[0]


@pytest.mark.parametrize("n0", [1e-3, 0.05, 3 / (4 * math.pi), 1.7])
def test_uniform_gas_closed_forms(table, n0):
    """Uniform density: E_x = Omega (-3/4)(3/pi)^(1/3) n^(4/3) and
    v_x = -(3/pi)^(1/3) n^(1/3) (Dirac); E_c = Omega n eps_c(n), and
    v_c = d(n eps_c)/dn, here by a central difference of the scalar n eps_c."""
    cell = (4.0, 5.0, 6.0)
    n = np.full((6, 8, 10), n0)
    ek, de, ex, ec, v = F.xc_energy_potential(n, cell, _zero_table(table))
    omega = 120.0
    assert ek == 0.0 and de == 0.0
    ex_ref = omega * (-0.75) * (3 / math.pi) ** (1 / 3) * n0 ** (4 / 3)
    assert abs(ex - ex_ref) < 1e-13 * abs(ex_ref)
    eps = F.pw92(np.array([n0]))[0][0]
    assert abs(ec - omega * n0 * eps) < 1e-13 * abs(ec)
    h = 1e-5 * n0
    f = lambda x: x * F.pw92(np.array([x]))[0][0]
    vc_ref = (f(n0 + h) - f(n0 - h)) / (2 * h)
    vx_ref = -(3 / math.pi) ** (1 / 3) * n0 ** (1 / 3)
    np.testing.assert_allclose(v, vx_ref + vc_ref, rtol=1e-8)


def test_enhancement_factor_limits():
    """F_x(0) = 1, F_x -> 1 + kappa = 2.245 (revPBE) as s grows, and
    (F_x - 1)/s^2 -> mu = 0.21951 (PBE) as s -> 0; F_x increases with s and
    stays below 1 + kappa."""
    assert _fx([0.0])[0] == 1.0
    assert abs(_fx([1e6])[0] - 2.245) < 1e-9
    small = _fx([1e-4])[0]
    assert abs((small - 1) / 1e-8 - 0.21951) < 1e-5
    s = np.linspace(0.0, 20.0, 401)
    f = _fx(s)
    assert np.all(np.diff(f) > 0) and np.all(f < 2.245)


def test_exchange_partials_by_differences():
    rng = np.random.default_rng(3)
    n = rng.uniform(1e-3, 2.0, 50)
    kf = (3 * math.pi ** 2 * n) ** (1 / 3)
    sigma = 4 * kf ** 2 * n ** 2 * rng.uniform(0.0, 3.0, 50) ** 2
    _, dn, ds = F.exchange_gga(n, sigma)
    h = 1e-6 * n
    fdn = (F.exchange_gga(n + h, sigma)[0] - F.exchange_gga(n - h, sigma)[0]) / (2 * h)
    hs = 1e-6 * np.maximum(sigma, 1e-6)
    fds = (F.exchange_gga(n, sigma + hs)[0] - F.exchange_gga(n, np.maximum(sigma - hs, 0.0))[0]) / (
        sigma + hs - np.maximum(sigma - hs, 0.0))
    np.testing.assert_allclose(dn, fdn, rtol=1e-7)
    np.testing.assert_allclose(ds, fds, rtol=1e-6)


@pytest.mark.parametrize("grad_mode,triclinic", [(0, False), (2, False), (0, True), (3, True)])
def test_exchange_uniform_scaling(table, grad_mode, triclinic):
    """n_lam(r) = lam^3 n(lam r) has E_x[n_lam] = lam E_x[n] exactly for GGA
    exchange (s is scale invariant).  On the grid: values times lam^3 on the
    cell shrunk by lam, the same grid shape."""
    if triclinic:
        L = W.triclinic_lattice((8.0, 7.5, 8.5), (78.0, 104.0, 66.0))
        rng = np.random.default_rng(2)
        n = W.density_on_lattice((12, 10, 14), L, W.random_atoms_lattice(rng, 3, L))
    else:
        wl = W.gauss24_coarse()
        L, n = np.diag(wl.cell), wl.density()
    t = _zero_table(table)
    ex = F.xc_energy_potential(n, L, t, grad_mode=grad_mode)[2]
    for lam in (0.7, 1.9):
        ex_l = F.xc_energy_potential(lam ** 3 * n, L / lam, t, grad_mode=grad_mode)[2]
        assert abs(ex_l - lam * ex) < 1e-12 * abs(ex)


@pytest.mark.parametrize("grad_mode", [0, 2])
def test_semilocal_terms_add(table, grad_mode):
    """E_k and Delta E are those of the nonlocal evaluation, and v_xc - v_nl is
    the potential of the semilocal terms alone (a zero kernel table)."""
    wl = W.gauss24_coarse()
    n = wl.density()
    ek, de, v = F.energy_potential(n, wl.cell, table, grad_mode=grad_mode)
    ek2, de2, ex, ec, vxc = F.xc_energy_potential(n, wl.cell, table, grad_mode=grad_mode)
    assert (ek, de) == (ek2, de2)
    _, _, ex0, ec0, vsl = F.xc_energy_potential(n, wl.cell, _zero_table(table), grad_mode=grad_mode)
    assert (ex, ec) == (ex0, ec0)
    np.testing.assert_allclose(vxc - v, vsl, rtol=0, atol=1e-12 * np.abs(vxc).max())


@pytest.mark.parametrize("grad_mode,triclinic", [(0, False), (2, False), (0, True)])
def test_xc_potential_is_gradient_of_energy(table, grad_mode, triclinic):
    """v_xc_i = (1/dOmega) dE_xc/dn_i by central differences (Eq. (Vi)) at points
    away from the density floor."""
    if triclinic:
        L = W.triclinic_lattice((8.0, 7.5, 8.5), (78.0, 104.0, 66.0))
        rng = np.random.default_rng(6)
        n = W.density_on_lattice((14, 12, 16), L, W.random_atoms_lattice(rng, 3, L))
    else:
        wl = W.gauss24_coarse()
        L, n = np.diag(wl.cell), wl.density()
    dvol = F.volume(L) / n.size

    def E(x):
        ek, de, ex, ec, v = F.xc_energy_potential(x, L, table, grad_mode=grad_mode)
        return ek + de + ex + ec, v

    _, v = E(n)
    rng = np.random.default_rng(11)
    cand = np.argwhere(n > 1e-2)
    for row in rng.choice(len(cand), 5, replace=False):
        i = tuple(cand[row])
        d = 1e-6 * n[i]
        n1 = n.copy()
        n1[i] += d
        n2 = n.copy()
        n2[i] -= d
        fd = (E(n1)[0] - E(n2)[0]) / (2 * d * dvol)
        assert abs(fd - v[i]) < 1e-5 * abs(v[i]) + 1e-8, (i, fd, v[i])
