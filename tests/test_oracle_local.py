"""Pins of the oracle's pointwise steps: spline basis, saturation, q0.

Each test checks the oracle against something other than itself: an
identity the paper states, a closed form, a textbook value, or a finite
difference.
"""
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import make_interp_spline

from oracle import functional as F
from oracle import kernel_table as kt

QMESH = kt.log_qmesh()


# ---------------------------------------------------------------- P1 (Eq. fofx)
def test_cardinal_property_and_partition_of_unity():
    spl = F.CardinalSplines(QMESH)
    p, dp = spl(QMESH)
    # p_a(q_b) = delta_ab: the interpolant of f_b = delta_ab (text after Eq. fofx)
    np.testing.assert_allclose(p, np.eye(QMESH.size), atol=1e-14)
    q = np.linspace(QMESH[0], QMESH[-1], 2001)
    p, dp = spl(q)
    # interpolating f = 1 and f = x with the same basis reproduces them exactly
    np.testing.assert_allclose(p.sum(axis=0), 1.0, atol=1e-13)
    np.testing.assert_allclose((QMESH[:, None] * p).sum(axis=0), q, atol=1e-13)
    np.testing.assert_allclose(dp.sum(axis=0), 0.0, atol=1e-12)
    np.testing.assert_allclose((QMESH[:, None] * dp).sum(axis=0), 1.0, atol=1e-12)


def test_cardinal_basis_equals_spline_interpolation():
    """sum_a f(q_a) p_a(x) is the natural cubic spline of f (independent
    B-spline construction), so p_a does not depend on f (Eq. fofx)."""
    spl = F.CardinalSplines(QMESH)
    f = np.sin(3.0 * QMESH) + QMESH ** 2
    ref = make_interp_spline(QMESH, f, k=3, bc_type="natural")
    x = np.linspace(QMESH[0], QMESH[-1], 777)
    p, dp = spl(x)
    np.testing.assert_allclose(f @ p, ref(x), atol=1e-12)
    np.testing.assert_allclose(f @ dp, ref.derivative()(x), atol=1e-10)


def test_cardinal_splines_are_c2_with_natural_ends():
    """Adjacent cubic pieces match in value, slope and curvature at every
    interior node (text after Eq. fofx); curvature vanishes at both ends."""
    spl = F.CardinalSplines(QMESH)
    c = spl._spl.c                       # c[k, j, a]: piece j, power 3-k
    h = np.diff(QMESH)[:, None]
    left_val = c[0, :-1] * h[:-1] ** 3 + c[1, :-1] * h[:-1] ** 2 + c[2, :-1] * h[:-1] + c[3, :-1]
    left_d1 = 3 * c[0, :-1] * h[:-1] ** 2 + 2 * c[1, :-1] * h[:-1] + c[2, :-1]
    left_d2 = 6 * c[0, :-1] * h[:-1] + 2 * c[1, :-1]
    scale = np.abs(c).max()
    np.testing.assert_allclose(left_val, c[3, 1:], atol=1e-12 * scale)
    np.testing.assert_allclose(left_d1, c[2, 1:], atol=1e-12 * scale)
    np.testing.assert_allclose(left_d2, 2 * c[1, 1:], atol=1e-11 * scale)
    last_d2 = 6 * c[0, -1] * h[-1] + 2 * c[1, -1]
    np.testing.assert_allclose(2 * c[1, 0], 0.0, atol=1e-11 * scale)
    np.testing.assert_allclose(last_d2, 0.0, atol=1e-11 * scale)


def test_spline_below_first_node_is_linear():
    spl = F.CardinalSplines(QMESH)
    x = np.array([0.0, 0.01, 0.03])
    p, dp = spl(x)
    p1, dp1 = spl(np.array([QMESH[0]]))
    np.testing.assert_allclose(p, p1 + (x - QMESH[0])[None, :] * dp1, atol=1e-15)


def test_log_mesh_ratio():
    """(q_{a+1} - q_a) = lambda (q_a - q_{a-1}) with lambda > 1, q_N = q_c."""
    d = np.diff(QMESH)
    np.testing.assert_allclose(d[1:] / d[:-1], 1.17, rtol=1e-12)
    assert QMESH[-1] == 5.0 and QMESH.size == 20


# ---------------------------------------------------------------- P2 (Eq. Sat)
def test_saturation_closed_forms():
    qc, mc = 5.0, 12
    # h(x) = x - O((x/xc)^(mc+1)) for x << xc
    x = np.array([0.05, 0.5, 1.0])
    h, dh = F.saturate(x, qc, mc)
    bound = qc * (x / qc) ** (mc + 1)
    assert np.all(np.abs(h - x) <= bound + 4 * np.finfo(float).eps * x)
    # at x = xc the series is the harmonic number H_12 = 86021/27720
    H12 = Fraction(0)
    for m in range(1, 13):
        H12 += Fraction(1, m)
    assert H12 == Fraction(86021, 27720)
    h, dh = F.saturate(np.array([qc]), qc, mc)
    np.testing.assert_allclose(h, qc * (1.0 - np.exp(-float(H12))), rtol=1e-15)
    np.testing.assert_allclose(dh, 12.0 * np.exp(-float(H12)), rtol=1e-14)
    # h -> xc for x -> infinity, monotone
    xs = np.linspace(0.0, 40.0, 4001)
    h, dh = F.saturate(xs, qc, mc)
    assert np.all(np.diff(h) >= 0.0) and np.all(h <= qc)
    assert h[-1] == qc and dh[-1] == 0.0


def test_saturation_infinite_series_limit():
    """With m_c -> infinity, sum y^m/m = -ln(1-y) and h(x) = x for x < x_c."""
    x = np.array([0.3, 1.7, 3.2])
    h, dh = F.saturate(x, 5.0, 400)
    np.testing.assert_allclose(h, x, rtol=1e-12)
    np.testing.assert_allclose(dh, 1.0, rtol=1e-10)


def test_saturation_derivative_fd():
    x = np.linspace(0.1, 12.0, 50)
    h, dh = F.saturate(x, 5.0, 12)
    e = 1e-6
    fd = (F.saturate(x + e, 5.0, 12)[0] - F.saturate(x - e, 5.0, 12)[0]) / (2 * e)
    np.testing.assert_allclose(dh, fd, rtol=1e-7, atol=1e-9)


# ---------------------------------------------------------------- P3 (q0)
def _golden_rows(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    return [line.split() for line in open(path) if line.strip() and not line.startswith("#")]


@pytest.mark.parametrize("rs,ref", [(float(a), float(b)) for a, b in _golden_rows("uniform_gas_correlation.txt")])
def test_pw92_uniform_gas_values(rs, ref):
    """Correlation energy per electron of the uniform gas (Ceperley-Alder data
    as parametrised by Perdew-Wang; tests/golden/uniform_gas_correlation.txt),
    Hartree, three significant digits."""
    n = 3.0 / (4.0 * np.pi * rs ** 3)
    eps, _ = F.pw92(np.array([n]))
    np.testing.assert_allclose(eps, ref, rtol=2.5e-3)


def test_pw92_high_density_slope():
    """eps_c -> A ln r_s + const, A = (1 - ln 2)/pi^2 (random-phase limit)."""
    rs = np.array([1e-7, 2e-7])
    n = 3.0 / (4.0 * np.pi * rs ** 3)
    eps, _ = F.pw92(n)
    slope = (eps[1] - eps[0]) / np.log(2.0)
    np.testing.assert_allclose(slope, (1.0 - np.log(2.0)) / np.pi ** 2, rtol=2e-3)


def test_q0_matches_exchange_correlation_route():
    """q0 = -(4 pi/3) [eps_c + eps_x (1 - Z_ab s^2 / 9)] with the Dirac
    exchange eps_x = -(3/4)(3/pi)^(1/3) n^(1/3) and s = |grad n| / (2 (3 pi^2)^(1/3) n^(4/3))."""
    rng = np.random.default_rng(7)
    n = 10.0 ** rng.uniform(-4, 0.5, 200)
    gabs = rng.uniform(0, 3.0, 200) * n
    q, _, _ = F.q0_unsaturated(n, gabs ** 2)
    eps_c, _ = F.pw92(n)
    eps_x = -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * n ** (1.0 / 3.0)
    s = gabs / (2.0 * (3.0 * np.pi ** 2) ** (1.0 / 3.0) * n ** (4.0 / 3.0))
    ref = -(4.0 * np.pi / 3.0) * (eps_c + eps_x * (1.0 - F.Z_AB * s * s / 9.0))
    np.testing.assert_allclose(q, ref, rtol=1e-12)


def test_q0_partials_fd():
    rng = np.random.default_rng(8)
    n = 10.0 ** rng.uniform(-4, 0.5, 100)
    sig = (rng.uniform(0, 3.0, 100) * n) ** 2
    q, qn, qs = F.q0_unsaturated(n, sig)
    e = 1e-6
    fdn = (F.q0_unsaturated(n * (1 + e), sig)[0] - F.q0_unsaturated(n * (1 - e), sig)[0]) / (2 * e * n)
    fds = (F.q0_unsaturated(n, sig + e * (1 + sig))[0] - F.q0_unsaturated(n, sig - e * (1 + sig))[0]) / (2 * e * (1 + sig))
    np.testing.assert_allclose(qn, fdn, rtol=1e-6)
    np.testing.assert_allclose(qs, fds, rtol=1e-6)
    _, dpw = F.pw92(n)
    fdp = (F.pw92(n * (1 + e))[0] - F.pw92(n * (1 - e))[0]) / (2 * e * n)
    np.testing.assert_allclose(dpw, fdp, rtol=1e-6)


def test_local_derivatives_fd(table):
    """dtheta/dn, dtheta/dgrad n and the e_Delta derivatives by central differences."""
    rng = np.random.default_rng(9)
    n = 10.0 ** rng.uniform(-3.5, 0.3, 60)
    g = rng.normal(size=(3, 60)) * n
    loc = F.theta_fields(n, g, table)
    e = 1e-6
    lp = F.theta_fields(n * (1 + e), g, table)
    lm = F.theta_fields(n * (1 - e), g, table)
    np.testing.assert_allclose(loc["dtheta_dn"], (lp["theta"] - lm["theta"]) / (2 * e * n), rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(loc["de_dn"], (lp["e_delta"] - lm["e_delta"]) / (2 * e * n), rtol=1e-5, atol=1e-12)
    for c in range(3):
        gp, gm = g.copy(), g.copy()
        h = 1e-5 * (np.abs(g[c]) + n)
        gp[c] += h
        gm[c] -= h
        lp = F.theta_fields(n, gp, table)
        lm = F.theta_fields(n, gm, table)
        np.testing.assert_allclose(loc["g"] * g[c], (lp["theta"] - lm["theta"]) / (2 * h), rtol=1e-5, atol=1e-9)
        np.testing.assert_allclose(loc["ge"] * g[c], (lp["e_delta"] - lm["e_delta"]) / (2 * h), rtol=1e-5, atol=1e-12)


def test_paper_parameters(table):
    """The table and the saturation use the interpolation and saturation
    parameters the paper prints (tests/golden/paper_parameters.txt)."""
    from oracle import kernel_table as kt
    par = {r[0]: float(r[1]) for r in _golden_rows("paper_parameters.txt")}
    q = kt.log_qmesh()
    assert len(q) == int(par["n_alpha"]) == table["qmesh"].size
    assert q[-1] == par["q_c"] == table["qc"]
    assert table["mc"] == int(par["m_c"])
    d = np.diff(q)                       # a logarithmic mesh: spacings grow by a constant factor > 1
    assert d[1] / d[0] > 1.0 and np.allclose(d[1:] / d[:-1], d[1] / d[0], rtol=1e-12)
