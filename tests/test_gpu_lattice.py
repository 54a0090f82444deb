"""Parity of the HIP path with the FP64 oracle on cells of any shape (the cell
given by its three vectors), through the C ABI: triclinic cells with the
spectral and the finite-difference gradient, FP64 to rounding and FP32 at
the method's accuracy; a rotated cell gives the same E and v; a diagonal
cell matrix reproduces the orthorhombic call bitwise; a batch mixing cell
shapes equals its single-grid evaluations bitwise."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import functional as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP64_REL = 1e-10
FP32_EREL = 1e-6
FP32_DV = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _lattice_density(shape, seed=3, natoms=3, lengths=(8.0, 7.5, 8.5), angles=(78.0, 104.0, 66.0)):
    L = W.triclinic_lattice(lengths, angles)
    rng = np.random.default_rng(seed)
    return L, W.density_on_lattice(shape, L, W.random_atoms_lattice(rng, natoms, L))


def _rotation(ax, ay, az):
    cx, sx, cy, sy, cz, sz = math.cos(ax), math.sin(ax), math.cos(ay), math.sin(ay), math.cos(az), math.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def gpu_eval(n, cell, table, precision, m=0, debug=False):
    from paper_0812_0244_amd import NonlocalCorrelation
    say("  gpu eval shape=%s precision=%d grad_mode=%d" % (n.shape, precision, m))
    eng = NonlocalCorrelation(n.shape, cell, table, precision=precision, device=0, grad_mode=m)
    dt = torch.float64 if precision == 64 else torch.float32
    nt = torch.from_numpy(n).to(device="cuda", dtype=dt)    # (kept: the stage probe reruns on it)
    ek, de, v = eng.energy_potential(nt)
    out = dict(E_k=ek, dE=de, v=v.double().cpu().numpy())
    if debug:
        from paper_0812_0244_amd.binding import STAGE_GRAD
        g = torch.empty((3,) + n.shape, dtype=dt, device="cuda")
        eng.lib.debug_field(0, 0, g.data_ptr())
        vl = torch.empty(n.shape, dtype=dt, device="cuda")
        eng.lib.debug_field(0, 1, vl.data_ptr())
        out["field0"] = g.double().cpu().numpy()
        out["v_loc"] = vl.double().cpu().numpy()
        gr = torch.empty((3,) + n.shape, dtype=dt, device="cuda")
        eng.lib.debug_stage(0, STAGE_GRAD, gr.data_ptr())
        out["grad"] = gr.double().cpu().numpy()
    return out


def check(g, o, precision):
    vmax = np.abs(o["v"]).max()
    dv = np.abs(g["v"] - o["v"]).max()
    e_g, e_o = g["E_k"] + g["dE"], o["E_k"] + o["dE"]
    say("  E_k %.15e / %.15e  dE %.15e / %.15e  rel(E) %.2e  max|dv| %.2e (max|v| %.2e)"
        % (g["E_k"], o["E_k"], g["dE"], o["dE"], abs(e_g - e_o) / abs(e_o), dv, vmax))
    if precision == 64:
        assert abs(g["E_k"] - o["E_k"]) <= FP64_REL * abs(o["E_k"])
        assert abs(g["dE"] - o["dE"]) <= FP64_REL * abs(o["dE"])
        assert dv <= FP64_REL * vmax
    else:
        assert abs(e_g - e_o) <= FP32_EREL * abs(e_o)
        assert dv <= FP32_DV


def test_triclinic_fp64_spectral_with_intermediates(table):
    L, n = _lattice_density((20, 18, 24))
    o = F.energy_potential(n, L, table, return_parts=True)
    g = gpu_eval(n, L, table, 64, debug=True)
    np.testing.assert_allclose(g["grad"], o["grad"], rtol=0, atol=1e-12 * np.abs(o["grad"]).max())
    np.testing.assert_allclose(g["v_loc"], o["v_loc"], rtol=0, atol=1e-10 * np.abs(o["v_loc"]).max())
    # the buffer of grad n ends holding the lattice components of w
    q = np.einsum("cx,x...->c...", F.fd_metric(n.shape, L), o["w"])
    np.testing.assert_allclose(g["field0"], q, rtol=0, atol=1e-10 * np.abs(q).max())
    check(g, o, 64)


@pytest.mark.parametrize("m", [1, 2, 4])
def test_triclinic_fp64_finite_differences(table, m):
    """With finite differences the buffer of grad n ends holding the lattice
    components q_c = sum_x W[c][x] w_x of the vector field w."""
    L, n = _lattice_density((20, 18, 24), seed=4)
    o = F.energy_potential(n, L, table, return_parts=True, grad_mode=m)
    g = gpu_eval(n, L, table, 64, m, debug=True)
    Wm = F.fd_metric(n.shape, L)
    q = np.einsum("cx,x...->c...", Wm, o["w"])
    np.testing.assert_allclose(g["field0"], q, rtol=0, atol=1e-10 * np.abs(q).max())
    np.testing.assert_allclose(g["v_loc"], o["v_loc"], rtol=0, atol=1e-10 * np.abs(o["v_loc"]).max())
    check(g, o, 64)


@pytest.mark.parametrize("shape,angles,m", [
    ((15, 16, 18), (85.0, 95.0, 60.0), 0),     # odd edge: no Nyquist index on axis 1
    ((16, 20, 15), (70.0, 100.0, 120.0), 0),
    ((16, 20, 15), (70.0, 100.0, 120.0), 3),
    ((12, 12, 12), (90.0, 90.0, 120.0), 0),     # hexagonal
])
def test_general_cells_fp64(table, shape, angles, m):
    L, n = _lattice_density(shape, seed=sum(shape), angles=angles)
    o = F.energy_potential(n, L, table, return_parts=True, grad_mode=m)
    check(gpu_eval(n, L, table, 64, m), o, 64)


@pytest.mark.parametrize("m", [0, 3])
def test_triclinic_fp32(table, m):
    L, n = _lattice_density((40, 36, 48), seed=7, natoms=8, lengths=(12.0, 11.0, 13.0))   # max |G| 27.2
    n32 = n.astype(np.float32).astype(np.float64)
    o = F.energy_potential(n32, L, table, return_parts=True, grad_mode=m)
    check(gpu_eval(n32, L, table, 32, m), o, 32)


@pytest.mark.parametrize("m", [0, 2])
def test_rotated_cell_same_result(table, m):
    L, n = _lattice_density((20, 18, 24), seed=9)
    a = gpu_eval(n, L, table, 64, m)
    b = gpu_eval(n, L @ _rotation(0.3, -0.7, 1.1).T, table, 64, m)
    np.testing.assert_allclose([b["E_k"], b["dE"]], [a["E_k"], a["dE"]], rtol=1e-12)
    # (each FP64 evaluation's v carries rounding of about 3e-12 max|v| from the
    # gradient chain, measured against the oracle; the two differ by that much)
    np.testing.assert_allclose(b["v"], a["v"], rtol=0, atol=1e-11 * np.abs(a["v"]).max())


@pytest.mark.parametrize("precision", [32, 64])
def test_diagonal_lattice_equals_lengths_bitwise(table, precision):
    wl = W.gauss24()
    n = wl.density()
    for m in (0, 3):
        a = gpu_eval(n, wl.cell, table, precision, m)
        b = gpu_eval(n, np.diag(wl.cell), table, precision, m)
        assert (a["E_k"], a["dE"]) == (b["E_k"], b["dE"])
        assert np.array_equal(a["v"], b["v"])


def test_mixed_batch_equals_single(table):
    from paper_0812_0244_amd import VdwNl
    L1, n1 = _lattice_density((20, 18, 24), seed=21)
    L2, n2 = _lattice_density((16, 20, 15), seed=22, angles=(70.0, 100.0, 120.0))
    wl = W.gauss24()
    shapes = [n1.shape, wl.shape, n2.shape]
    cells = [L1, wl.cell, L2]
    dens = [n1, wl.density(), n2]
    for m in (0, 2):
        lib = VdwNl(0)
        lib.set_grids(shapes, cells, m, 64)
        lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
        n = [torch.from_numpy(d).to("cuda") for d in dens]
        v = [torch.empty_like(x) for x in n]
        E = lib.energy_potential_batched([x.data_ptr() for x in n], [x.data_ptr() for x in v])
        v2 = [torch.full_like(x, float("nan")) for x in n]
        assert np.array_equal(E, lib.energy_potential_batched([x.data_ptr() for x in n], [x.data_ptr() for x in v2]))
        assert all(torch.equal(a, b) for a, b in zip(v, v2))
        for i in range(3):
            s = gpu_eval(dens[i], cells[i], table, 64, m)
            assert (s["E_k"], s["dE"]) == (E[i, 0], E[i, 1])
            assert np.array_equal(s["v"], v[i].cpu().numpy())
            o = F.energy_potential(dens[i], cells[i], table, grad_mode=m, return_parts=True)
            check(s, o, 64)


@pytest.mark.parametrize("precision", [64, 32])
def test_packed_and_full_kernel_rows_agree(table, precision):
    """General cells keep each shell's kernel rows as full 20 x 20 matrices
    unless a single grid uses the table and its full matrices would not fit
    in the 256 MB Infinity Cache; then the packed upper triangle (half the
    bytes).  FP64: a 60^3 triclinic grid (edges 18.0, 18.9, 16.8 bohr, angles
    78, 104, 66 degrees) has about 1.08e5 shells (330 MB as full FP64
    matrices); FP32: a 72^3 grid (edges 21.6, 22.7, 20.2 bohr) about 1.87e5
    (285 MB as full FP32 matrices).  Alone each takes packed rows, twice in a
    batch full rows.  Both against the oracle at the bars of the precision
    (FP32 on the FP32-rounded input), and bitwise equal to each other (the
    same row values, only loaded differently)."""
    from paper_0812_0244_amd import VdwNl
    if precision == 64:
        L, n = _lattice_density((60, 60, 60), seed=31, natoms=6, lengths=(18.0, 18.9, 16.8))
        row_bytes = 3200
    else:
        L, n = _lattice_density((72, 72, 72), seed=32, natoms=8, lengths=(21.6, 22.7, 20.2))
        n = n.astype(np.float32).astype(np.float64)
        row_bytes = 1600
    nshell = len(np.unique(F.gmod_half(n.shape, L)))
    say("  distinct |G| shells: %d (full matrices %.0f MB)" % (nshell, nshell * row_bytes / 2 ** 20))
    assert nshell * row_bytes > 256 * 2 ** 20     # (the single-grid plan packs its rows)
    o = F.energy_potential(n, L, table, return_parts=True)
    single = gpu_eval(n, L, table, precision)
    check(single, o, precision)
    dt = torch.float64 if precision == 64 else torch.float32
    lib = VdwNl(0)
    lib.set_grids([n.shape, n.shape], [L, L], 0, precision)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    nt = [torch.from_numpy(n).to("cuda", dt), torch.from_numpy(n).to("cuda", dt)]
    v = [torch.empty_like(x) for x in nt]
    E = lib.energy_potential_batched([x.data_ptr() for x in nt], [x.data_ptr() for x in v])
    for i in range(2):
        say("  batch member %d: E_k %.15e dE %.15e (single %.15e %.15e)" % (i, E[i, 0], E[i, 1], single["E_k"], single["dE"]))
        assert (E[i, 0], E[i, 1]) == (single["E_k"], single["dE"])
        assert np.array_equal(v[i].double().cpu().numpy(), single["v"])
