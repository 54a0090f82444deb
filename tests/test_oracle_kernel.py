"""Pins of the oracle's kernel phi(d1, d2), its soft form and the radial table.

The paper does not print the kernel; it states its properties: E_c^nl is
exactly zero for a constant density, it decays as r^-6, and phi diverges
logarithmically at d -> 0.  These tests hold the recalled kernel to them.
"""
import numpy as np
import pytest

from oracle import kernel_table as kt


def _gl_panels(edges, order=16):
    x, w = np.polynomial.legendre.leggauss(order)
    d, wt = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        d.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        wt.append(0.5 * (hi - lo) * w)
    return np.concatenate(d), np.concatenate(wt)


def test_kernel_integrates_to_zero_over_uniform_density():
    """E_c^nl = 0 for any constant density: Int_0^inf 4 pi d^2 phi(d,d) dd = 0.
    Numerical part to d = 25, exact r^-6 tail beyond."""
    X = 25.0
    d, wt = _gl_panels([0.0] + list(np.geomspace(1e-7, X, 60)))
    f = kt.phi(d, d)
    integral = np.sum(wt * 4 * np.pi * d * d * f) - 2 * np.pi * kt.C_ASYM / (3 * X ** 3)
    positive = np.sum(wt * 4 * np.pi * d * d * np.maximum(f, 0.0))
    assert positive > 1.0
    assert abs(integral) < 5e-8 * positive


@pytest.mark.parametrize("d1,d2,tol", [(20.0, 20.0, 1e-6), (25.0, 35.0, 1e-5), (30.0, 18.0, 1e-5)])
def test_kernel_r6_asymptote(d1, d2, tol):
    """phi -> -C / (d1^2 d2^2 (d1^2 + d2^2)), C = 12 (4 pi/9)^3 (the r^-6 law)."""
    np.testing.assert_allclose(kt.phi([d1], [d2]), kt.phi_asym(d1, d2), rtol=tol)


def test_kernel_symmetry_and_log_divergence():
    a = kt.phi([0.3, 2.0, 0.05, 7.0], [1.7, 0.5, 3.0, 0.9])
    b = kt.phi([1.7, 0.5, 3.0, 0.9], [0.3, 2.0, 0.05, 7.0])
    np.testing.assert_allclose(a, b, rtol=1e-13)
    # logarithmic divergence at d -> 0: phi(d) - phi(2d) tends to a constant
    d = np.array([1e-4, 2e-4, 4e-4, 8e-4])
    f = kt.phi(d, d)
    steps = f[:-1] - f[1:]
    assert np.all(steps > 0)
    np.testing.assert_allclose(steps[1:], steps[0], rtol=2e-2)


def test_soft_kernel_matches_value_and_slope():
    """Eq. (PhiSoft): phi_s and phi agree in value and slope at D = d_s on a ray."""
    q = kt.log_qmesh()
    for a, b in [(19, 19), (3, 11), (0, 19)]:
        Q = np.hypot(q[a], q[b])
        ray = kt.Ray(q[a] / Q, q[b] / Q, 1.0, 0.5)
        ds = ray.ds
        np.testing.assert_allclose(ray.soft_poly(ds), ray.phi_ds, rtol=1e-13)
        h = 1e-6
        slope_soft = (ray.soft_poly(ds) - ray.soft_poly(ds - h)) / h
        np.testing.assert_allclose(slope_soft, ray.dphi_ds, rtol=1e-5)
        exact = kt.phi([(ds + 1e-3) * ray.c, (ds - 1e-3) * ray.c], [(ds + 1e-3) * ray.s, (ds - 1e-3) * ray.s])
        np.testing.assert_allclose((exact[0] - exact[1]) / 2e-3, ray.dphi_ds, rtol=1e-6)
        assert ray.monotone_soft()


def test_table_symmetric_and_tied_to_c_soft(table):
    """phi_ab(k) = phi_ba(k); and since Int d^3r phi = 0 (constant density),
    phi_aa(k = 0) = Int d^3r phi_s(q_a r, q_a r) = -2 C_s / q_a^3 (Eq. Depsnl)."""
    phi = table["phi"]
    assert np.array_equal(phi, phi.transpose(1, 0, 2))
    q = table["qmesh"]
    np.testing.assert_allclose(np.diag(phi[:, :, 0]), -2 * table["c_soft"] / q ** 3, rtol=1e-6)


@pytest.mark.parametrize("a,b,kmax", [(12, 12, 3.1), (6, 14, 3.1), (0, 19, 1.3), (0, 12, 1.3), (3, 19, 1.3)])
def test_table_against_direct_radial_quadrature(table, a, b, kmax):
    """phi_ab(k) = 4 pi Int r^2 j0(kr) phi_s(q_a r, q_b r) dr by Gauss-Legendre
    on the exact kernel (no spline, no trapezoid) at a few k, on rays from the
    diagonal to the most skewed of the mesh (q_b/q_a = 1, 4.7, 100, 30, 24).
    On the skewed rays the kernel is sampled out to D = 400 (d2 = 400), where
    the geometric panels (width 27 there) resolve the oscillation of j0(kD)
    only up to k ~ 1.3; measured agreement there 3e-8 of |phi_ab(0)|."""
    q = table["qmesh"]
    Q = np.hypot(q[a], q[b])
    ray = kt.Ray(q[a] / Q, q[b] / Q, 1.0, 0.5)
    X = ray.X
    D, wt = _gl_panels([0.0, 0.25, 0.5, 0.75, 1.0] + list(np.geomspace(1.0, X, 90))[1:], 12)
    f = np.where(D < ray.ds, ray.soft_poly(D), kt.phi(D * ray.c, D * ray.s))
    ks = np.array([k for k in (0.0, 0.4, 1.3, 3.1) if k <= kmax])   # k values on the table mesh
    j = np.rint(ks / table["dk"]).astype(int)
    for jj in j:
        kap = jj * table["dk"] / Q
        j0 = np.sinc(kap * D / np.pi)
        psi = np.sum(wt * 4 * np.pi * D * D * j0 * f) + kt._tail_transform(np.array([kap]), X, ray.asym_coef)[0]
        ref = psi / Q ** 3
        scale = np.abs(table["phi"][a, b, 0])
        np.testing.assert_allclose(table["phi"][a, b, jj], ref, atol=2e-6 * scale)
