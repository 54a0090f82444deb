"""Densities outside the method's domain (the problem is posed for n >= 0):
a negative, NaN or infinite value is flagged by the theta pass as it reads
the density, the grid's energies come out NaN and the call reports
VDWNL_E_BAD_DENSITY; the other grids of a batch and the next evaluation are
unaffected."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

E_BAD = -8


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _lib(shapes, cells, table, prec, fd=0):
    from paper_0812_0244_amd import VdwNl
    lib = VdwNl(0)
    if len(shapes) == 1:
        lib.set_grid(shapes[0], cells[0], fd, prec)
    else:
        lib.set_grids(shapes, cells, fd, prec)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    return lib


def _density(shape, cell, seed):
    return W.density_on_grid(shape, cell, W.random_atoms(np.random.default_rng(seed), 4, cell))


@pytest.mark.parametrize("prec,fd", [(32, 0), (64, 0), (32, 3)])
def test_single_grid_bad_values(table, prec, fd):
    from paper_0812_0244_amd.binding import VdwNlError
    shape, cell = (24, 20, 16), (8.0, 7.0, 6.0)
    n = _density(shape, cell, 5)
    dt = torch.float32 if prec == 32 else torch.float64
    lib = _lib([shape], [cell], table, prec, fd)
    good = torch.from_numpy(n).to("cuda", dt)
    v = torch.empty_like(good)
    ref = lib.energy_potential(good.data_ptr(), v.data_ptr())
    vref = v.clone()
    for bad_value in (float("nan"), -1e-3, float("inf")):
        say("  precision %d fd %d: value %r" % (prec, fd, bad_value))
        bad = good.clone()
        bad[3, 5, 7] = bad_value
        with pytest.raises(VdwNlError) as ei:
            lib.energy_potential(bad.data_ptr(), v.data_ptr())
        assert ei.value.code == E_BAD
        # the raw call: NaN energies
        E = np.zeros(2)
        rc = lib.lib.vdwnl_energy_potential(lib.h, ctypes.c_void_p(bad.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                            E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
        assert rc == E_BAD and np.isnan(E).all()
        # the next evaluation starts clean and repeats the reference bitwise
        assert lib.energy_potential(good.data_ptr(), v.data_ptr()) == ref
        assert torch.equal(v, vref)
    # zero density is in the domain
    zero = good.clone()
    zero[3, 5, 7] = 0.0
    lib.energy_potential(zero.data_ptr(), v.data_ptr())


def test_batched_flags_only_the_bad_grid(table):
    from paper_0812_0244_amd.binding import VdwNlError
    shapes = [(16, 16, 16), (24, 24, 24), (20, 16, 24)]
    cells = [(6.0, 6.0, 6.0), (8.0, 8.0, 8.0), (7.0, 6.0, 8.0)]
    dens = [torch.from_numpy(_density(s, c, 40 + i)).to("cuda", torch.float32)
            for i, (s, c) in enumerate(zip(shapes, cells))]
    lib = _lib(shapes, cells, table, 32)
    vs = [torch.empty_like(x) for x in dens]
    ref = lib.energy_potential_batched([x.data_ptr() for x in dens], [x.data_ptr() for x in vs])
    bad = [x.clone() for x in dens]
    bad[1][0, 0, 0] = float("nan")
    nb = len(shapes)
    na = (ctypes.c_void_p * nb)(*[x.data_ptr() for x in bad])
    va = (ctypes.c_void_p * nb)(*[x.data_ptr() for x in vs])
    E = np.zeros((nb, 2))
    rc = lib.lib.vdwnl_energy_potential_batched(lib.h, nb, na, va, E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                None)
    say("  batched: rc %d, E %s" % (rc, E.tolist()))
    assert rc == E_BAD
    assert np.isnan(E[1]).all()
    assert np.array_equal(E[[0, 2]], ref[[0, 2]])
    # asynchronous: only the device energies tell
    E_dev = torch.zeros((nb, 2), dtype=torch.float64, device="cuda")
    lib.energy_potential_batched_async([x.data_ptr() for x in bad], [x.data_ptr() for x in vs], E_dev.data_ptr())
    torch.cuda.synchronize()
    Ed = E_dev.cpu().numpy()
    assert np.isnan(Ed[1]).all() and np.array_equal(Ed[[0, 2]], ref[[0, 2]])
    # clean again
    assert np.array_equal(lib.energy_potential_batched([x.data_ptr() for x in dens], [x.data_ptr() for x in vs]), ref)
    with pytest.raises(VdwNlError):
        lib.energy_potential_batched([x.data_ptr() for x in bad], [x.data_ptr() for x in vs])


def test_noalloc_entry_point_flags_bad_density(table):
    from paper_0812_0244_amd.binding import VdwNlError
    shape, cell = (16, 24, 20), (6.0, 8.0, 7.0)
    n = torch.from_numpy(_density(shape, cell, 9)).to("cuda", torch.float32)
    lib = _lib([shape], [cell], table, 32)
    v = torch.empty_like(n)
    ref = lib.energy_potential_noalloc(n.data_ptr(), v.data_ptr())
    bad = n.clone()
    bad[1, 2, 3] = -5.0
    with pytest.raises(VdwNlError) as ei:
        lib.energy_potential_noalloc(bad.data_ptr(), v.data_ptr())
    assert ei.value.code == E_BAD
    assert lib.energy_potential_noalloc(n.data_ptr(), v.data_ptr()) == ref
