"""Pins of the oracle on non-orthogonal cells (the cell as three cell
vectors): the closed form of the constant-table special case with images
over the general lattice, exact invariance under a rotation of the cell, the
orthorhombic special case, and v = (1/dOmega) dE/dn_i (Eq. (Vi)) by central
differences with either gradient."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import functional as F

SHAPE = (20, 18, 22)


def _cell_and_density(seed=3, natoms=3, shape=SHAPE, lengths=(8.0, 7.5, 8.5), angles=(78.0, 104.0, 66.0)):
    L = W.triclinic_lattice(lengths, angles)
    rng = np.random.default_rng(seed)
    atoms = W.random_atoms_lattice(rng, natoms, L)
    return L, atoms, W.density_on_lattice(shape, L, atoms)


def _rotation(ax, ay, az):
    cx, sx, cy, sy, cz, sz = math.cos(ax), math.sin(ax), math.cos(ay), math.sin(ay), math.cos(az), math.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def _gaussian_table(table, s):
    k = np.arange(table["nk"]) * table["dk"]
    f = np.pi ** 1.5 * s ** 3 * np.exp(-(k * s) ** 2 / 4.0)
    nq = table["qmesh"].size
    t = dict(table)
    t["phi"] = np.broadcast_to(f, (nq, nq, k.size)).copy()
    t["c_soft"] = 0.0
    return t


def test_reciprocal_vectors_and_volume():
    L = W.triclinic_lattice()
    B = F.reciprocal(L)
    np.testing.assert_allclose(L @ B.T, 2 * np.pi * np.eye(3), atol=1e-13)
    a, b, c = (np.linalg.norm(L[i]) for i in range(3))
    al, be, ga = (math.radians(x) for x in (80.0, 105.0, 70.0))
    # the textbook volume of a triclinic cell from its edges and angles
    vol = a * b * c * math.sqrt(1 - math.cos(al) ** 2 - math.cos(be) ** 2 - math.cos(ga) ** 2
                                + 2 * math.cos(al) * math.cos(be) * math.cos(ga))
    assert abs(F.volume(L) - vol) < 1e-12 * vol


def test_constant_table_closed_form_triclinic(table):
    """phi_ab(k) = f(k), f(r) = exp(-r^2/s^2): E_k = 1/2 Int Int n n f and
    v = f * n, analytic for Gaussian atoms with images over the lattice."""
    s = 1.0
    t = _gaussian_table(table, s)
    shape = (32, 30, 34)
    L, atoms, n = _cell_and_density(seed=11, natoms=4, shape=shape)
    ek, de, v = F.energy_potential(n, L, t)
    assert de == 0.0
    n0, omega = W.FLOOR, F.volume(L)
    A, w, R = atoms.amp, atoms.width, atoms.pos
    e = 0.5 * omega * n0 ** 2 * np.pi ** 1.5 * s ** 3 + n0 * np.sum(A * np.pi ** 3 * w ** 3 * s ** 3)
    ks = np.array([(i, j, k) for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4)], dtype=float)
    shifts = ks @ L
    for a in range(len(A)):
        for b in range(len(A)):
            c2 = w[a] ** 2 + w[b] ** 2 + s ** 2
            d2 = np.sum((R[a] - R[b] + shifts) ** 2, axis=1)
            e += 0.5 * A[a] * A[b] * np.pi ** 3 * (w[a] * w[b] * s) ** 3 / c2 ** 1.5 * np.sum(np.exp(-d2 / c2))
    np.testing.assert_allclose(ek, e, rtol=1e-9)
    u = [np.arange(shape[c]) / shape[c] for c in range(3)]
    X = np.stack(np.meshgrid(*u, indexing="ij"), axis=-1) @ L
    vref = np.full(n.shape, n0 * np.pi ** 1.5 * s ** 3)
    for b in range(len(A)):
        c2 = w[b] ** 2 + s ** 2
        pref = A[b] * (np.pi * w[b] ** 2 * s ** 2 / c2) ** 1.5
        for sh in shifts:
            d2 = np.sum((X - R[b] - sh) ** 2, axis=-1)
            vref += pref * np.exp(-d2 / c2)
    np.testing.assert_allclose(v, vref, rtol=0, atol=1e-9 * np.abs(vref).max())


@pytest.mark.parametrize("grad_mode", [0, 2])
def test_rotation_invariance(table, grad_mode):
    """Rotating the cell vectors rotates G and grad n alike: |G| and |grad n|
    and so E and v on the grid are unchanged."""
    L, _, n = _cell_and_density()
    Lr = L @ _rotation(0.3, -0.7, 1.1).T
    e0, d0, v0 = F.energy_potential(n, L, table, grad_mode=grad_mode)
    e1, d1, v1 = F.energy_potential(n, Lr, table, grad_mode=grad_mode)
    np.testing.assert_allclose([e1, d1], [e0, d0], rtol=1e-12)
    np.testing.assert_allclose(v1, v0, rtol=0, atol=1e-12 * np.abs(v0).max())


@pytest.mark.parametrize("grad_mode", [0, 3])
def test_orthorhombic_lattice_equals_lengths(table, grad_mode):
    wl = W.gauss24_coarse()
    n = wl.density()
    a = F.energy_potential(n, wl.cell, table, grad_mode=grad_mode)
    b = F.energy_potential(n, np.diag(wl.cell), table, grad_mode=grad_mode)
    np.testing.assert_allclose(a[:2], b[:2], rtol=1e-14)
    np.testing.assert_allclose(a[2], b[2], rtol=0, atol=1e-14 * np.abs(a[2]).max())


def test_nyquist_multiplier_is_symmetric():
    """|G| of the half spectrum equals |G| of -G (mod the grid) everywhere,
    Nyquist planes included, so the kernel multiplier is Hermitian."""
    L = W.triclinic_lattice()
    shape = (8, 6, 10)
    g = F.gmod_half(shape, L)
    B = F.reciprocal(L)
    for k1 in range(shape[0]):
        for k2 in range(shape[1]):
            for k3 in (0, shape[2] // 2):
                j1, j2 = (-k1) % shape[0], (-k2) % shape[1]
                assert abs(g[k1, k2, k3] - g[j1, j2, k3]) < 1e-12 * max(g[k1, k2, k3], 1.0)
    # off the Nyquist planes |G| is the plain norm of sum_c m_c b_c
    m = np.array([2, -1, 3], dtype=float)
    assert abs(g[2, shape[1] - 1, 3] - np.linalg.norm(m @ B)) < 1e-12


@pytest.mark.parametrize("grad_mode", [0, 2])
def test_potential_is_gradient_of_energy_triclinic(table, grad_mode):
    L, _, n = _cell_and_density(seed=5, natoms=3, shape=(16, 14, 18))
    dvol = F.volume(L) / n.size

    def E(x):
        ek, de, v = F.energy_potential(x, L, table, grad_mode=grad_mode)
        return ek + de, v

    _, v = E(n)
    # points away from the density floor, step d = 1e-6 n_i: E is strongly
    # curved in a single n_i with the spectral gradient (the central
    # difference's error there is about 2e4 (d/n_i)^2 relative, checked down
    # to d = 1e-6 n_i), and the energy difference at such points is still far
    # above the rounding of E
    rng = np.random.default_rng(8)
    cand = np.argwhere(n > 1e-2)
    for row in rng.choice(len(cand), 6, replace=False):
        i = tuple(cand[row])
        d = 1e-6 * n[i]
        n1 = n.copy()
        n1[i] += d
        n2 = n.copy()
        n2[i] -= d
        fd = (E(n1)[0] - E(n2)[0]) / (2 * d * dvol)
        assert abs(fd - v[i]) < 1e-5 * abs(v[i]) + 1e-9, (i, fd, v[i])
