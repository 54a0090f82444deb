"""Seeded synthetic densities for the vdW-DF nonlocal-correlation path.

This module holds no part of the method's arithmetic: it only builds
electron densities n(r) on periodic grids (orthorhombic, or general cells
given by their three cell vectors).  It is the one
module that both the oracle and the product path (tests, benchmark, the
force example) use for their inputs.

The paper's own workloads are self-consistent DFT densities of double-wall
carbon nanotubes; they are not reproducible here, so the densities are sums
of isotropic Gaussian "atoms" on a small floor:

    n(r) = n_floor + sum_A sum_L  A_A exp(-|r - R_A - L|^2 / w_A^2)

(L runs over the periodic images with every Cartesian component of
r - R_A - L below 8 w_A in magnitude; the omitted terms are < 1e-27 A_A).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLOOR = 1e-4           # e/bohr^3, the density floor of every workload
IMAGE_CUT = 8.0        # images within IMAGE_CUT * w per axis
BATCH_SIZES = (32, 48, 64, 96, 128)
BATCH_SPACING = 20.0 / 96.0   # bohr, constant grid spacing of the batched workload


@dataclass
class Atoms:
    amp: np.ndarray      # [natoms] e/bohr^3
    width: np.ndarray    # [natoms] bohr
    pos: np.ndarray      # [natoms, 3] bohr


@dataclass
class Workload:
    name: str
    shape: tuple
    cell: tuple          # orthorhombic cell lengths, bohr
    atoms: Atoms
    floor: float = FLOOR
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def npoints(self) -> int:
        return int(np.prod(self.shape))

    def density(self) -> np.ndarray:
        return density_on_grid(self.shape, self.cell, self.atoms, self.floor)


def random_atoms(rng: np.random.Generator, natoms: int, cell) -> Atoms:
    """Amplitudes U[0.5, 2], widths U[0.6, 1.2], centres uniform in the cell."""
    amp = rng.uniform(0.5, 2.0, natoms)
    width = rng.uniform(0.6, 1.2, natoms)
    pos = rng.uniform(0.0, 1.0, (natoms, 3)) * np.asarray(cell, dtype=np.float64)
    return Atoms(amp, width, pos)


def _axis_profile(npts: int, length: float, centre: float, width: float) -> np.ndarray:
    """sum over images of exp(-(x_i - centre - k L)^2 / w^2) on x_i = i L / npts."""
    x = np.arange(npts) * (length / npts)
    out = np.zeros(npts)
    kmax = int(math.ceil((IMAGE_CUT * width + length) / length)) + 1
    for k in range(-kmax, kmax + 1):
        dx = x - centre - k * length
        m = np.abs(dx) < IMAGE_CUT * width
        if np.any(m):
            out[m] += np.exp(-(dx[m] / width) ** 2)
    return out


def density_on_grid(shape, cell, atoms: Atoms, floor: float = FLOOR) -> np.ndarray:
    """n on the grid r_i = (i1 L1/N1, i2 L2/N2, i3 L3/N3), FP64, C order."""
    shape = tuple(int(s) for s in shape)
    n = np.full(shape, floor, dtype=np.float64)
    for a, w, r in zip(atoms.amp, atoms.width, atoms.pos):
        prof = [_axis_profile(shape[c], cell[c], r[c], w) for c in range(3)]
        idx = [np.nonzero(p)[0] for p in prof]
        sub = (a * prof[0][idx[0]][:, None, None] * prof[1][idx[1]][None, :, None]
               * prof[2][idx[2]][None, None, :])
        n[np.ix_(idx[0], idx[1], idx[2])] += sub
    return n


# --------------------------------------------------------------------------
# general (non-orthogonal) periodic cells
# --------------------------------------------------------------------------

def lattice_matrix(cell) -> np.ndarray:
    """3 x 3 matrix whose rows are the cell vectors a_1, a_2, a_3 (bohr):
    a general cell as given, or the diagonal of three orthorhombic lengths."""
    c = np.asarray(cell, dtype=np.float64)
    return np.diag(c) if c.shape == (3,) else c.reshape(3, 3).copy()


def random_atoms_lattice(rng: np.random.Generator, natoms: int, lattice) -> Atoms:
    """As ``random_atoms``, centres uniform in the cell spanned by the rows of
    ``lattice`` (fractional coordinates uniform in [0, 1))."""
    amp = rng.uniform(0.5, 2.0, natoms)
    width = rng.uniform(0.6, 1.2, natoms)
    frac = rng.uniform(0.0, 1.0, (natoms, 3))
    return Atoms(amp, width, frac @ lattice_matrix(lattice))


def density_on_lattice(shape, lattice, atoms: Atoms, floor: float = FLOOR) -> np.ndarray:
    """n on the grid r_i = sum_c (i_c / N_c) a_c of a general cell (rows of
    ``lattice``), FP64, C order.  Images L = sum_c k_c a_c are summed while a
    Gaussian can reach the cell within IMAGE_CUT widths (|k_c| up to the
    cut's extent along the reciprocal direction, plus one)."""
    shape = tuple(int(s) for s in shape)
    A = lattice_matrix(lattice)
    recip = np.linalg.inv(A).T                       # rows b_c / (2 pi)
    u = [np.arange(shape[c]) / shape[c] for c in range(3)]
    U = np.stack(np.meshgrid(*u, indexing="ij"), axis=-1)
    r = U @ A                                        # [N1, N2, N3, 3]
    n = np.full(shape, floor, dtype=np.float64)
    for a, w, pos in zip(atoms.amp, atoms.width, atoms.pos):
        kmax = [int(math.ceil(IMAGE_CUT * w * np.linalg.norm(recip[c]))) + 1 for c in range(3)]
        for k1 in range(-kmax[0], kmax[0] + 1):
            for k2 in range(-kmax[1], kmax[1] + 1):
                for k3 in range(-kmax[2], kmax[2] + 1):
                    d = r - (pos + k1 * A[0] + k2 * A[1] + k3 * A[2])
                    d2 = np.einsum("...i,...i->...", d, d)
                    m = d2 < (IMAGE_CUT * w) ** 2
                    if np.any(m):
                        n[m] += a * np.exp(-d2[m] / (w * w))
    return n


def triclinic_lattice(lengths=(10.0, 9.0, 11.0), angles_deg=(80.0, 105.0, 70.0)) -> np.ndarray:
    """Rows a_1, a_2, a_3 of the cell with the given edge lengths and the
    angles (alpha between a_2 and a_3, beta between a_1 and a_3, gamma
    between a_1 and a_2), a_1 along x and a_2 in the xy plane."""
    a, b, c = lengths
    al, be, ga = (math.radians(x) for x in angles_deg)
    a1 = np.array([a, 0.0, 0.0])
    a2 = np.array([b * math.cos(ga), b * math.sin(ga), 0.0])
    cx = c * math.cos(be)
    cy = c * (math.cos(al) - math.cos(be) * math.cos(ga)) / math.sin(ga)
    a3 = np.array([cx, cy, math.sqrt(c * c - cx * cx - cy * cy)])
    return np.stack([a1, a2, a3])


# --------------------------------------------------------------------------
# double-wall nanotube geometry
# --------------------------------------------------------------------------

def nanotube_atoms(n: int, m: int, acc: float):
    """One translational period of an (n, m) tube: (cylindrical angle, z) of
    every atom, the radius and the period length, by rolling up graphene.
    """
    a = math.sqrt(3.0) * acc
    a1 = np.array([a * math.sqrt(3.0) / 2.0, a / 2.0])
    a2 = np.array([a * math.sqrt(3.0) / 2.0, -a / 2.0])
    ch = n * a1 + m * a2
    dr = math.gcd(2 * m + n, 2 * n + m)
    t = ((2 * m + n) / dr) * a1 - ((2 * n + m) / dr) * a2
    basis = [np.zeros(2), (a1 + a2) / 3.0]
    span = 2 * (n + m + abs(2 * m + n) + abs(2 * n + m)) + 4
    pts = []
    for i in range(-span, span + 1):
        for j in range(-span, span + 1):
            for b in basis:
                p = i * a1 + j * a2 + b
                u = p @ ch / (ch @ ch)
                v = p @ t / (t @ t)
                if -1e-9 <= u < 1.0 - 1e-9 and -1e-9 <= v < 1.0 - 1e-9:
                    pts.append((2.0 * math.pi * u, v * np.linalg.norm(t)))
    radius = np.linalg.norm(ch) / (2.0 * math.pi)
    return np.array(pts), radius, float(np.linalg.norm(t))


def dwnt_workload() -> Workload:
    """(5,5)@(10,10) armchair double-wall tube, 160x160x320 grid, 30x30x60 bohr.

    C-C distance 2.68 bohr; axis along z through (15, 15); 13 axial periods
    (13 x 4.642 = 60.34 bohr) rescaled to exactly 60 bohr so the cell is
    seamless; 20 + 40 atoms per period, 780 atoms.  Each "carbon-like" atom
    carries 4 electrons in a Gaussian of width 1 bohr.
    """
    cell = (30.0, 30.0, 60.0)
    shape = (160, 160, 320)
    acc, nper, w = 2.68, 13, 1.0
    pos = []
    for (n, m) in ((5, 5), (10, 10)):
        cyl, radius, period = nanotube_atoms(n, m, acc)
        scale = cell[2] / (nper * period)
        for k in range(nper):
            for phi, z in cyl:
                pos.append((15.0 + radius * math.cos(phi), 15.0 + radius * math.sin(phi),
                            (z + k * period) * scale))
    pos = np.array(pos)
    amp = np.full(len(pos), 4.0 / (math.pi ** 1.5 * w ** 3))
    width = np.full(len(pos), w)
    return Workload("dwnt_5_5_at_10_10", shape, cell, Atoms(amp, width, pos), seed=3,
                    meta=dict(radii=(6.398, 12.796), atoms=len(pos)))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def gaussian_workload(name, npts, length, natoms, seed) -> Workload:
    rng = np.random.default_rng(seed)
    cell = (float(length),) * 3
    return Workload(name, (npts,) * 3, cell, random_atoms(rng, natoms, cell), seed=seed)


def gauss24() -> Workload:
    """Four Gaussian atoms in a 10-bohr cube on a 24^3 grid (small enough for
    the oracle to finish in seconds)."""
    return gaussian_workload("gauss4_24c_L10", 24, 10.0, 4, 1)


def gauss96() -> Workload:
    """64 Gaussian atoms in a 20-bohr cube on a 96^3 grid."""
    return gaussian_workload("gauss64_96c_L20", 96, 20.0, 64, 2)


def gauss128() -> Workload:
    """128 Gaussian atoms on a 128^3 grid at the batch's spacing (20/96 bohr)."""
    return gaussian_workload("gauss128_128c", 128, 128 * BATCH_SPACING, 128, 5)


def gauss24_coarse() -> Workload:
    """The atoms and cell of gauss24() on a 12^3 grid."""
    w = gauss24()
    return Workload("gauss4_12c_L10", (12, 12, 12), w.cell, w.atoms, seed=w.seed)


def batch_instances(count: int = 64, first_seed: int = 4000) -> list:
    """Member i: seed first_seed + i; edge N_i uniform in {32,48,64,96,128},
    cubic cell of side N_i * 20/96 bohr (constant spacing), 4..128 atoms."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(first_seed + i)
        npts = int(rng.choice(BATCH_SIZES))
        natoms = int(rng.integers(4, 129))
        length = npts * BATCH_SPACING
        cell = (length,) * 3
        out.append(Workload("batch%02d_%dc" % (i, npts), (npts,) * 3, cell,
                            random_atoms(rng, natoms, cell), seed=first_seed + i))
    return out


# --------------------------------------------------------------------------
# torch twin, differentiable in the atom centres (forces)
# --------------------------------------------------------------------------

def density_torch(shape, cell, amp, width, pos, floor: float = FLOOR):
    """Same density as ``density_on_grid`` with torch ops, differentiable in
    ``pos`` (a [natoms, 3] tensor); grid, dtype and device follow ``pos``."""
    import torch

    dev, dt = pos.device, pos.dtype
    n = torch.full(tuple(shape), floor, dtype=dt, device=dev)
    amp = torch.as_tensor(amp, dtype=dt, device=dev)
    width = torch.as_tensor(width, dtype=dt, device=dev)
    profiles = []
    for c in range(3):
        npts, length = int(shape[c]), float(cell[c])
        x = torch.arange(npts, dtype=dt, device=dev) * (length / npts)
        wmax = float(width.max())
        kmax = int(math.ceil((IMAGE_CUT * wmax + length) / length)) + 1
        ks = torch.arange(-kmax, kmax + 1, dtype=dt, device=dev) * length
        # dx[atom, image, i]
        dx = x[None, None, :] - pos[:, c, None, None] - ks[None, :, None]
        w = width[:, None, None]
        g = torch.exp(-(dx / w) ** 2) * (dx.abs() < IMAGE_CUT * w)
        profiles.append(g.sum(dim=1))   # [natoms, npts]
    for a in range(pos.shape[0]):
        n = n + amp[a] * profiles[0][a][:, None, None] * profiles[1][a][None, :, None] \
            * profiles[2][a][None, None, :]
    return n
