"""Every FFT length class of the HIP path against the oracle, on every axis.

The transforms of Eq. (Eoffk) (forward, N_a fields) and of Eq. (epsofk)
(inverse) run as compile-time radix plans for the lengths 24, 32, 48, 64,
96, 128, 160 and 320 and as a runtime Stockham plan for the others; each
plan has its own lanes-per-line and elements-per-lane layout, and each axis
its own pass (axis 3 fused with the local steps, axis 2 alone, axis 1 fused
with the contraction).  Each case here puts one length class on one axis
(the other two short, runtime-radix lengths) and compares E_k, Delta E and
v element by element with the FP64 oracle:

* FP64: relative 1e-10 in E_k and Delta E, max|dv| <= 1e-10 max|v|;
* FP32: relative 1e-6 in E, max|dv| <= 1e-5 Ha, the oracle evaluated on the
  same FP32-rounded density.

Axis 1 takes at most 204 points (one line of the fused axis-1 pass must fit
a tile), so 320 is tested there as a clean refusal.  A subset runs in
triclinic cells (the general-cell variant of the fused pass).  The full 128^3
density of the differentiation workload is compared at its real size too.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import functional as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LENS = (24, 32, 48, 64, 96, 128, 160, 320)
SHORT = (10, 12)
H = 0.2          # grid spacing (bohr): max |G| = pi sqrt(3) / H = 27.2 < 32


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def shape_for(axis, L):
    s = list(SHORT)
    s.insert(axis, L)
    return tuple(s)


def gpu_eval(n, cell, table, precision):
    from paper_0812_0244_amd import NonlocalCorrelation
    eng = NonlocalCorrelation(n.shape, cell, table, precision=precision, device=0)
    dt = torch.float64 if precision == 64 else torch.float32
    ek, de, v = eng.energy_potential(torch.from_numpy(n).to(device="cuda", dtype=dt))
    return ek, de, v.double().cpu().numpy()


def compare(n, cell, table, precision):
    ek_o, de_o, v_o = F.energy_potential(n, cell, table)
    ek, de, v = gpu_eval(n, cell, table, precision)
    vmax = np.abs(v_o).max()
    dv = np.abs(v - v_o).max()
    e, e_o = ek + de, ek_o + de_o
    say("  fp%d %s: E_k %.14e / %.14e  dE %.14e / %.14e  rel(E) %.2e  max|dv| %.2e (max|v| %.2e)"
        % (precision, n.shape, ek, ek_o, de, de_o, abs(e - e_o) / abs(e_o), dv, vmax))
    if precision == 64:
        assert abs(ek - ek_o) <= 1e-10 * abs(ek_o)
        assert abs(de - de_o) <= 1e-10 * abs(de_o)
        assert dv <= 1e-10 * vmax
    else:
        assert abs(e - e_o) <= 1e-6 * abs(e_o)
        assert dv <= 1e-5


def density(shape, cell, seed):
    vol = float(np.prod(cell))
    natoms = max(2, int(vol / 25.0))
    return W.density_on_grid(shape, cell, W.random_atoms(np.random.default_rng(seed), natoms, cell))


CASES = [(axis, L) for axis in range(3) for L in LENS if not (axis == 0 and L > 204)]


@pytest.mark.parametrize("axis,L", CASES)
def test_length_class_on_axis(table, axis, L):
    shape = shape_for(axis, L)
    cell = tuple(H * s for s in shape)
    say("  axis %d length %d: shape %s" % (axis + 1, L, shape))
    n = density(shape, cell, 7000 + 10 * L + axis)
    compare(n, cell, table, 64)
    compare(n.astype(np.float32).astype(np.float64), cell, table, 32)


def test_axis1_length_320_refused(table):
    from paper_0812_0244_amd import VdwNl, VdwNlError
    lib = VdwNl(0)
    with pytest.raises(VdwNlError) as ex:
        lib.set_grid((320, 10, 12), (64.0, 2.0, 2.4), 0, 32)
    assert ex.value.code == -2


@pytest.mark.parametrize("axis,L", [(0, 64), (1, 128), (2, 160), (2, 320), (0, 160), (1, 320)])
def test_length_class_on_axis_triclinic(table, axis, L):
    shape = shape_for(axis, L)
    h = 0.23
    lat = W.triclinic_lattice(tuple(h * s for s in shape), (85.0, 95.0, 80.0))
    rng = np.random.default_rng(9000 + L + axis)
    natoms = max(2, int(abs(np.linalg.det(lat)) / 25.0))
    n = W.density_on_lattice(shape, lat, W.random_atoms_lattice(rng, natoms, lat))
    say("  triclinic axis %d length %d: shape %s" % (axis + 1, L, shape))
    compare(n, lat, table, 64)
    compare(n.astype(np.float32).astype(np.float64), lat, table, 32)


def test_two_long_axes(table):
    """Long lengths on two axes at once (their passes meet in the same grid)."""
    for shape in [(128, 160, 12), (10, 128, 320), (160, 12, 128), (64, 96, 160)]:
        cell = tuple(H * s for s in shape)
        n = density(shape, cell, 7777 + sum(shape))
        compare(n, cell, table, 64)
        compare(n.astype(np.float32).astype(np.float64), cell, table, 32)


def test_differentiation_workload_128_cubed_against_oracle(table):
    """The 128^3 density of the differentiation workload (128 atoms) at full
    size, both precisions, against the oracle element by element."""
    wl = W.gauss128()
    n = wl.density()
    say("  128^3, %d atoms" % len(wl.atoms.amp))
    compare(n, wl.cell, table, 64)
    compare(n.astype(np.float32).astype(np.float64), wl.cell, table, 32)
