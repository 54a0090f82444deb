"""Pins of the oracle's whole pipeline (transforms, contraction, energy,
potential) against closed forms, direct sums and derivative identities."""
import numpy as np
import pytest

import workloads as W
from oracle import functional as F


def _evaluate(n, cell, table):
    ek, de, v = F.energy_potential(n, cell, table)
    return ek + de, v


# ---------------------------------------------------------------- P6
def _uniform_density_for_q(q_target, table):
    lo, hi = 1e-8, 50.0
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        q, _, _ = F.q0_unsaturated(np.array([mid]), np.array([0.0]))
        qs, _ = F.saturate(q, table["qc"], table["mc"])
        if qs[0] < q_target:
            lo = mid
        else:
            hi = mid
    return np.sqrt(lo * hi)


@pytest.mark.parametrize("alpha", [6, 12, 17])
def test_uniform_density_on_a_mesh_node_gives_zero(table, alpha):
    """Constant n with q0 = q_alpha: only theta_alpha(G=0) survives, and
    E_k + Delta E = (Omega/2) n^2 [phi_aa(0) + 2 C_s / q_a^3] = 0 because the
    kernel integrates to zero over a uniform density."""
    q = table["qmesh"][alpha]
    n0 = _uniform_density_for_q(q, table)
    n = np.full((8, 8, 8), n0)
    ek, de, v = F.energy_potential(n, (5.0, 5.0, 5.0), table)
    assert abs(de) > 0
    assert abs(ek + de) < 1e-6 * abs(de)
    np.testing.assert_allclose(v, v.flat[0], rtol=1e-12)


def test_uniform_density_between_nodes_small(table):
    n0 = 0.5 * (_uniform_density_for_q(table["qmesh"][10], table)
                + _uniform_density_for_q(table["qmesh"][11], table))
    ek, de, _ = F.energy_potential(np.full((6, 6, 6), n0), (4.0, 4.0, 4.0), table)
    assert abs(ek + de) < 2e-2 * abs(de)


# ---------------------------------------------------------------- P7
def _gaussian_table(table, s):
    k = np.arange(table["nk"]) * table["dk"]
    f = np.pi ** 1.5 * s ** 3 * np.exp(-(k * s) ** 2 / 4.0)
    nq = table["qmesh"].size
    t = dict(table)
    t["phi"] = np.broadcast_to(f, (nq, nq, k.size)).copy()
    t["c_soft"] = 0.0
    return t


def test_constant_table_closed_form(table):
    """phi_ab(k) = f(k) for all a, b, f(r) = exp(-r^2/s^2): by the partition of
    unity E_k = 1/2 Int Int n n f and v = f * n, analytic for Gaussian atoms."""
    s = 1.0
    t = _gaussian_table(table, s)
    cell = (8.0, 8.0, 8.0)
    rng = np.random.default_rng(11)
    atoms = W.random_atoms(rng, 5, cell)
    n = W.density_on_grid((32, 32, 32), cell, atoms)
    ek, de, v = F.energy_potential(n, cell, t)
    assert de == 0.0
    n0, omega = W.FLOOR, np.prod(cell)
    A, w, R = atoms.amp, atoms.width, atoms.pos
    e = 0.5 * omega * n0 ** 2 * np.pi ** 1.5 * s ** 3 + n0 * np.sum(A * np.pi ** 3 * w ** 3 * s ** 3)
    L = np.array(cell)
    shifts = np.array([(i, j, k) for i in range(-2, 3) for j in range(-2, 3) for k in range(-2, 3)]) * L
    for a in range(len(A)):
        for b in range(len(A)):
            c2 = w[a] ** 2 + w[b] ** 2 + s ** 2
            d2 = np.sum((R[a] - R[b] + shifts) ** 2, axis=1)
            e += 0.5 * A[a] * A[b] * np.pi ** 3 * (w[a] * w[b] * s) ** 3 / c2 ** 1.5 * np.sum(np.exp(-d2 / c2))
    np.testing.assert_allclose(ek, e, rtol=1e-10)
    x = [np.arange(32) * cell[c] / 32 for c in range(3)]
    X = np.stack(np.meshgrid(*x, indexing="ij"), axis=-1)
    vref = np.full(n.shape, n0 * np.pi ** 1.5 * s ** 3)
    for b in range(len(A)):
        c2 = w[b] ** 2 + s ** 2
        pref = A[b] * (np.pi * w[b] ** 2 * s ** 2 / c2) ** 1.5
        for sh in shifts:
            d2 = np.sum((X - R[b] - sh) ** 2, axis=-1)
            vref += pref * np.exp(-d2 / c2)
    np.testing.assert_allclose(v, vref, rtol=0, atol=1e-10 * np.abs(vref).max())


# ---------------------------------------------------------------- P8
def test_fft_energy_equals_direct_double_sum(table):
    """E = 1/2 dOmega^2 sum_ij sum_ab theta_ai theta_bj K_ab(r_i - r_j) (Eq. Eofni)
    with the band-limited periodic kernel K_ab(r) = (1/Omega) sum_{G in box}
    phi_ab(|G|) cos(G.r), summed directly (no FFT); likewise u (Eq. epsilon)."""
    wl = W.gauss24_coarse()
    n = wl.density()
    cell = wl.cell
    shape = n.shape
    N = n.size
    omega = np.prod(cell)
    dvol = omega / N
    parts = F.energy_potential(n, cell, table, return_parts=True)
    theta = parts["theta"].reshape(20, N)
    m = [np.fft.fftfreq(shape[c], 1.0 / shape[c]) for c in range(3)]
    G = np.stack(np.meshgrid(*[2 * np.pi * m[c] / cell[c] for c in range(3)], indexing="ij"), -1).reshape(N, 3)
    idx = np.stack(np.meshgrid(*[np.arange(s) for s in shape], indexing="ij"), -1).reshape(N, 3)
    r = idx * (np.array(cell) / np.array(shape))
    vals, shell = F.kernel_at(np.linalg.norm(G, axis=1), table)
    phiG = vals[shell]                                   # [N_G, 20, 20]
    cosm = np.cos(r @ G.T)                               # [N_disp, N_G]
    K = (cosm @ phiG.reshape(N, 400)).reshape(N, 20, 20) / omega   # K[displacement]
    # displacement index of r_i - r_j
    E = 0.0
    u = np.zeros((20, N))
    for j in range(N):
        disp = (idx - idx[j]) % np.array(shape)
        d = (disp[:, 0] * shape[1] + disp[:, 1]) * shape[2] + disp[:, 2]
        Kj = K[d]                                        # [N_i, 20, 20]
        t_j = theta[:, j]
        contrib = np.einsum("iab,b->ai", Kj, t_j)        # sum_b K_ab(r_i - r_j) theta_bj
        u += contrib
    E = 0.5 * dvol ** 2 * np.sum(theta * u)
    u *= dvol
    np.testing.assert_allclose(E, parts["E_k"], rtol=1e-12)
    np.testing.assert_allclose(u, parts["u"].reshape(20, N), atol=1e-11 * np.abs(u).max())


# ---------------------------------------------------------------- P11
def test_potential_is_gradient_of_energy(table):
    """v_i = (1/dOmega) dE/dn_i (Eq. Vi) by central differences."""
    wl = W.gauss24()
    n = wl.density()
    cell = wl.cell
    dvol = np.prod(cell) / n.size
    _, v = _evaluate(n, cell, table)
    rng = np.random.default_rng(5)
    for _ in range(8):
        i = tuple(rng.integers(0, 24, 3))
        d = 1e-4 * n[i]
        n1 = n.copy()
        n1[i] += d
        n2 = n.copy()
        n2[i] -= d
        fd = (_evaluate(n1, cell, table)[0] - _evaluate(n2, cell, table)[0]) / (2 * d * dvol)
        assert abs(fd - v[i]) < 1e-5 * abs(v[i]) + 1e-9


# ---------------------------------------------------------------- P12 / P13
def test_translation_permutation_inversion(table):
    wl = W.gauss24_coarse()
    n = wl.density()
    cell = wl.cell
    e0, v0 = _evaluate(n, cell, table)
    e1, v1 = _evaluate(np.roll(n, (3, -5, 7), axis=(0, 1, 2)), cell, table)
    np.testing.assert_allclose(e1, e0, rtol=1e-13)
    np.testing.assert_allclose(v1, np.roll(v0, (3, -5, 7), axis=(0, 1, 2)), atol=1e-13 * np.abs(v0).max())
    e2, v2 = _evaluate(np.ascontiguousarray(n.transpose(2, 0, 1)), cell, table)
    np.testing.assert_allclose(e2, e0, rtol=1e-13)
    np.testing.assert_allclose(v2, v0.transpose(2, 0, 1), atol=1e-12 * np.abs(v0).max())
    ninv = np.roll(n[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))    # n(-r) on the grid
    e3, v3 = _evaluate(ninv, cell, table)
    np.testing.assert_allclose(e3, e0, rtol=1e-13)
    np.testing.assert_allclose(v3, np.roll(v0[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)), atol=1e-12 * np.abs(v0).max())


def test_parseval(table):
    """E_k in k space (Eq. Eoffk) = (dOmega/2) sum_i sum_a theta_ai u_ai in real space."""
    wl = W.gauss24()
    n = wl.density()
    p = F.energy_potential(n, wl.cell, table, return_parts=True)
    dvol = np.prod(wl.cell) / n.size
    np.testing.assert_allclose(p["E_k"], 0.5 * dvol * np.sum(p["theta"] * p["u"]), rtol=1e-13)


def test_low_density_points_are_excluded(table):
    """n < n_min: theta and its derivatives vanish there (design reading)."""
    wl = W.gauss24_coarse()
    n = wl.density()
    n[0, 0, :4] = 1e-40
    loc = F.theta_fields(n, F.gradient(n, wl.cell), table)
    assert np.all(loc["theta"][:, 0, 0, :4] == 0) and np.all(loc["e_delta"][0, 0, :4] == 0)
