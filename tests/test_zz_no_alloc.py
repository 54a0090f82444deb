"""vdwnl_energy_potential_noalloc (the evaluation that allocates nothing,
its device structures in the library's static scratch buffer) against
vdwnl_energy_potential, through the C ABI.

Both run the same kernels on the same tiles, so E_k, Delta E and v must be
bitwise equal; the FP64 bar of the parity tests (1e-10 relative) is asserted
as well.  Two calls in a row on different grids, the second smaller, then the
first grid again (its tables copied back into the shared buffer), in both
precisions; a plan larger than the buffer is refused with the bytes it needs.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _context(shape, cell, table, precision, grad_mode=0):
    from paper_0812_0244_amd import VdwNl
    lib = VdwNl(0)
    lib.set_grid(shape, cell, grad_mode, precision)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    return lib


def _both(lib, n):
    v1 = torch.full_like(n, float("nan"))
    v2 = torch.full_like(n, float("nan"))
    E1 = lib.energy_potential(n.data_ptr(), v1.data_ptr())
    E2 = lib.energy_potential_noalloc(n.data_ptr(), v2.data_ptr())
    return E1, v1, E2, v2


def _check(E1, v1, E2, v2, tag):
    dv = float((v1.double() - v2.double()).abs().max())
    say("  %s: E_k %.15e / %.15e  dE %.15e / %.15e  max|dv| %.1e" % (tag, E1[0], E2[0], E1[1], E2[1], dv))
    assert abs(E2[0] - E1[0]) <= 1e-10 * abs(E1[0]) and abs(E2[1] - E1[1]) <= 1e-10 * abs(E1[1])
    assert dv <= 1e-10 * float(v1.double().abs().max())
    assert E1 == E2 and torch.equal(v1, v2)


@pytest.mark.parametrize("precision", [64, 32])
def test_noalloc_equals_energy_potential(table, precision):
    dt = torch.float64 if precision == 64 else torch.float32
    big = ((40, 36, 48), (8.0, 7.5, 10.0))
    small = ((24, 24, 24), (10.0, 10.0, 10.0))
    ctx, dens = [], []
    for i, (shape, cell) in enumerate((big, small)):
        d = W.density_on_grid(shape, cell, W.random_atoms(np.random.default_rng(40 + i), 5, cell))
        dens.append(torch.from_numpy(d).to("cuda", dt))
        ctx.append(_context(shape, cell, table, precision))
    # two calls in a row, the second on the smaller grid, then the first again
    for k in (0, 1, 0, 0):
        _check(*_both(ctx[k], dens[k]), "fp%d %s" % (precision, tuple(dens[k].shape)))


def test_noalloc_finite_differences_and_triclinic(table):
    wl = W.gauss24()
    n = torch.from_numpy(wl.density()).cuda()
    _check(*_both(_context(wl.shape, wl.cell, table, 64, grad_mode=3), n), "24^3 m=3")
    lat = W.triclinic_lattice((7.0, 6.5, 8.0), (80.0, 100.0, 75.0))
    shape = (20, 18, 24)
    d = W.density_on_lattice(shape, lat, W.random_atoms_lattice(np.random.default_rng(5), 4, lat))
    _check(*_both(_context(shape, lat, table, 64), torch.from_numpy(d).cuda()), "triclinic 20x18x24")


def test_noalloc_triclinic_packs_rows_to_fit(table):
    """A lone grid in a general cell whose full-matrix kernel rows would not
    fit the scratch array (48 x 45 x 45 FP32, edges 14.4, 14.2, 12.6 bohr,
    angles 78, 104, 66 degrees: about 48,600 shells, 74 MiB as full
    matrices, 39 MiB packed) keeps packed rows: the no-allocation call runs
    it and equals the allocating call bitwise."""
    shape = (48, 45, 45)
    lat = W.triclinic_lattice((14.4, 14.2, 12.6), (78.0, 104.0, 66.0))
    d = W.density_on_lattice(shape, lat, W.random_atoms_lattice(np.random.default_rng(7), 5, lat))
    n = torch.from_numpy(d.astype(np.float32)).cuda()
    _check(*_both(_context(shape, lat, table, 32), n), "triclinic 48x45x45 FP32")


def test_noalloc_allocates_no_device_memory(table):
    wl = W.gauss24()
    n = torch.from_numpy(wl.density()).cuda()
    v = torch.empty_like(n)
    lib = _context(wl.shape, wl.cell, table, 64)
    lib.energy_potential_noalloc(n.data_ptr(), v.data_ptr())
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        lib.energy_potential_noalloc(n.data_ptr(), v.data_ptr())
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    say("  free device memory before %d after %d" % (free0, free1))
    assert free1 == free0
    nb, ws = lib.info()
    assert ws == 0          # the context's own workspace was never allocated


def test_noalloc_refuses_what_does_not_fit(table):
    from paper_0812_0244_amd import VdwNl, VdwNlError
    lib = _context((128, 128, 128), (26.0, 26.0, 26.0), table, 32)
    n = torch.full((128, 128, 128), 0.01, dtype=torch.float32, device="cuda")
    v = torch.empty_like(n)
    with pytest.raises(VdwNlError) as ex:
        lib.energy_potential_noalloc(n.data_ptr(), v.data_ptr())
    assert ex.value.code == -2 and "bytes of device scratch" in str(ex.value)
    say("  %s" % ex.value)
    lib2 = VdwNl(0)
    lib2.set_grids([(24, 24, 24), (12, 12, 12)], [(10.0,) * 3, (5.0,) * 3], 0, 64)
    lib2.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    with pytest.raises(VdwNlError) as ex:
        lib2.energy_potential_noalloc(n.data_ptr(), v.data_ptr())
    assert ex.value.code == -6
