"""Pins of the oracle's finite-difference gradient (grad_mode m = 1..4), the
paper's own treatment of grad n (the potential section, around Eq. (Vi)):
weights against the published central-difference table, exactness and the
truncation constant on monomials, the order on a periodic sine, the adjoint
identity behind Eq. (Vi), v as the exact gradient of E, and the spectral
derivative as the limit of growing stencils.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import functional as F

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fornberg():
    """First-derivative central weights, Fornberg, Math. Comp. 51 (1988),
    Table 1 (tests/golden/fd_central_weights.txt)."""
    out = {}
    for line in open(os.path.join(GOLDEN, "fd_central_weights.txt")):
        if line.strip() and not line.startswith("#"):
            m, *ws = line.split()
            out[int(m)] = [Fraction(w) for w in ws]
    return out


FORNBERG = _fornberg()


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_weights_match_published_table(m):
    np.testing.assert_allclose(F.fd_weights(m), [float(x) for x in FORNBERG[m]], rtol=1e-13, atol=0)


def _line_field(shape, cell, ax, f):
    x = np.arange(shape[ax]) * (cell[ax] / shape[ax])
    sh = [1, 1, 1]
    sh[ax] = shape[ax]
    return np.broadcast_to(f(x).reshape(sh), shape).copy(), x


@pytest.mark.parametrize("m", [1, 2, 3, 4])
@pytest.mark.parametrize("ax", [0, 1, 2])
def test_monomials_exact_then_truncation_constant(m, ax):
    """Away from the periodic wrap the formula of order 2m differentiates x^p
    exactly for p <= 2m; for p = 2m + 1 its error is C_m h^(2m) p!, with
    C_m = (-1)^(m+1) (m!)^2 / (2m + 1)! (the leading term of the Taylor
    remainder of the central formula)."""
    shape, cell = (20, 22, 18), (2.0, 2.2, 1.8)
    h = cell[ax] / shape[ax]
    inner = slice(m, shape[ax] - m)
    for p in range(1, 2 * m + 2):
        n, x = _line_field(shape, cell, ax, lambda t: (t - 0.37) ** p)
        g = F.gradient_fd(n, cell, m)
        got = np.moveaxis(g[ax], ax, 0)[inner, 0, 0]
        want = p * (x[inner] - 0.37) ** (p - 1)
        others = [g[c] for c in range(3) if c != ax]
        assert all(np.all(o == 0.0) for o in others)
        if p <= 2 * m:
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * max(1.0, np.abs(want).max()))
        else:
            cm = (-1) ** (m + 1) * math.factorial(m) ** 2 / math.factorial(2 * m + 1)
            np.testing.assert_allclose(got - want, cm * h ** (2 * m) * math.factorial(p), rtol=1e-6)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_order_on_periodic_sine(m):
    """Halving h on sin(2 pi x / L) divides the error by about 2^(2m)."""
    errs = []
    for N in (32, 64):
        shape, cell = (N, 4, 4), (3.0, 1.0, 1.0)
        n, x = _line_field(shape, cell, 0, lambda t: np.sin(2 * np.pi * t / 3.0))
        g = F.gradient_fd(n, cell, m)[0][:, 0, 0]
        errs.append(np.abs(g - 2 * np.pi / 3.0 * np.cos(2 * np.pi * x / 3.0)).max())
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - 2 * m) < 0.1, (m, rate)


@pytest.mark.parametrize("m", [1, 3, 4])
def test_adjoint_identity(m):
    """<D n, w> = -<n, div w>: the derivative operator is antisymmetric, which
    turns the sum over j in Eq. (Vi) into minus the divergence."""
    rng = np.random.default_rng(3)
    shape, cell = (9, 10, 7), (3.0, 4.0, 2.5)
    n = rng.standard_normal(shape)
    w = rng.standard_normal((3,) + shape)
    lhs = np.sum(F.gradient_fd(n, cell, m) * w)
    rhs = -np.sum(n * F.divergence_fd(w, cell, m))
    assert abs(lhs - rhs) < 1e-12 * np.sum(np.abs(n)) * np.sum(np.abs(w))


def test_wrapping_stencil_on_short_axis():
    """An axis shorter than the stencil (N = 4 < 2 m + 1 for m = 4) folds the
    weights of coinciding neighbours together: a unit impulse picks up every
    weight that lands on each point."""
    m, N = 4, 4
    c = F.fd_weights(m)
    n = np.zeros((N, 4, 4))
    n[0, 0, 0] = 1.0
    g = F.gradient_fd(n, (1.0, 1.0, 1.0), m)[0][:, 0, 0] * (1.0 / N)
    want = np.zeros(N)
    for s in range(1, m + 1):
        want[(-s) % N] += c[s - 1]        # d_i gets c_s n_{i+s}: i + s = 0
        want[s % N] -= c[s - 1]
    np.testing.assert_allclose(g, want, atol=1e-15)


@pytest.mark.parametrize("m", [1, 3])
def test_potential_is_gradient_of_energy_fd(table, m):
    """Eq. (Vi) with finite differences: v_i = (1/dOmega) dE/dn_i, checked
    by central differences of E, Richardson-extrapolated from the steps
    h = 1e-3 n_i and 2h (the O(h^2) term cancels).  Most sampled points sit on
    the 1e-4 density floor, where a smaller step (1e-4 n_i) leaves a change of
    E only about 1e5 times its FP64 rounding."""
    wl = W.gauss24()
    n = wl.density()
    cell = wl.cell
    dvol = np.prod(cell) / n.size

    def E(x):
        ek, de, v = F.energy_potential(x, cell, table, grad_mode=m)
        return ek + de, v

    def central(i, d):
        n1 = n.copy()
        n1[i] += d
        n2 = n.copy()
        n2[i] -= d
        return (E(n1)[0] - E(n2)[0]) / (2 * d * dvol)

    _, v = E(n)
    rng = np.random.default_rng(7)
    for _ in range(6):
        i = tuple(rng.integers(0, 24, 3))
        d = 1e-3 * n[i]
        fd = (4.0 * central(i, d) - central(i, 2 * d)) / 3.0
        assert abs(fd - v[i]) < 1e-5 * abs(v[i]) + 1e-9, (i, fd, v[i])


def test_stencils_approach_spectral_gradient(table):
    """On a band-limited field the central formulas converge to the spectral
    derivative as the stencil grows, and so do E and v."""
    rng = np.random.default_rng(9)
    shape, cell = (16, 16, 16), (6.0, 6.0, 6.0)
    spec = np.zeros((16, 16, 9), dtype=complex)
    spec[:4, :4, :4] = rng.standard_normal((4, 4, 4)) + 1j * rng.standard_normal((4, 4, 4))
    f = np.fft.irfftn(spec, s=shape, axes=(0, 1, 2))
    gs = F.gradient(f, cell)
    errs = [np.abs(F.gradient_fd(f, cell, m) - gs).max() for m in (1, 2, 3, 4)]
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:])), errs
    wl = W.gauss24_coarse()
    n = wl.density()
    e_s, de_s, v_s = F.energy_potential(n, wl.cell, table)
    gaps = []
    for m in (1, 2, 3, 4):
        e, de, v = F.energy_potential(n, wl.cell, table, grad_mode=m)
        gaps.append(abs(e + de - e_s - de_s))
    assert all(b < a for a, b in zip(gaps, gaps[1:])), gaps


def test_grad_mode_checked(table):
    wl = W.gauss24_coarse()
    with pytest.raises(ValueError):
        F.energy_potential(wl.density(), wl.cell, table, grad_mode=5)
