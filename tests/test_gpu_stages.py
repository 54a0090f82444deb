"""The stages of the method one by one, through vdwnl_debug_stage.

Each stage of the HIP path is compared element by element with the same
quantity of the oracle:

* theta_a(r_i) = n_i p_a(q0_i) (the weighted densities, text after Eq. (Eoffk));
* c_a(G) = FFT(theta_a)/N, the forward transforms of Eq. (Eoffk);
* u_a(G) = sum_b phi_ab(|G|) c_b(G), the per-k contraction of Eq. (epsofk);
* u_a(r_i), the inverse transforms of Eq. (epsilon).

FP64 bars are relative to the largest magnitude of the quantity (1e-12);
FP32 runs take the FP32-rounded density, and their bars (a few 1e-6 of the
largest magnitude) follow from FP32 rounding of the local chain and of the
transforms.  A second set checks only the transforms: numpy's FFT of the
GPU's own theta against the GPU's spectra, and numpy's inverse FFT of the
GPU's u spectra against the GPU's u(r), for every compile-time length class
on every axis, so that a plan's error cannot hide behind the oracle's.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import functional as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NQ = 20


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def stages(dens, cells, table, precision, grad_mode=0, which=None):
    """Evaluate the batch once, then probe every stage of grid `which` (all
    grids when None); returns per grid {theta, chat, uhat, u} (FP64/complex128)."""
    from paper_0812_0244_amd import VdwNl
    from paper_0812_0244_amd.binding import STAGE_THETA, STAGE_THETA_K, STAGE_U, STAGE_U_K
    dt = torch.float64 if precision == 64 else torch.float32
    lib = VdwNl(0)
    lib.set_grids([d.shape for d in dens], cells, grad_mode, precision)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    ns = [torch.from_numpy(d).to("cuda", dt) for d in dens]
    vs = [torch.empty_like(x) for x in ns]
    lib.energy_potential_batched([x.data_ptr() for x in ns], [x.data_ptr() for x in vs])
    out = []
    for i, d in enumerate(dens):
        if which is not None and i != which:
            out.append(None)
            continue
        n1, n2, n3 = d.shape
        h = n3 // 2 + 1
        r = {}
        th = torch.empty((NQ,) + d.shape, dtype=dt, device="cuda")
        lib.debug_stage(i, STAGE_THETA, th.data_ptr())
        r["theta"] = th.double().cpu().numpy()
        for key, st in (("chat", STAGE_THETA_K), ("uhat", STAGE_U_K)):
            sp = torch.empty((n1, n2, h, NQ, 2), dtype=dt, device="cuda")
            lib.debug_stage(i, st, sp.data_ptr())
            a = sp.double().cpu().numpy()
            r[key] = np.moveaxis(a[..., 0] + 1j * a[..., 1], -1, 0)
        u = torch.empty((NQ,) + d.shape, dtype=dt, device="cuda")
        lib.debug_stage(i, STAGE_U, u.data_ptr())
        r["u"] = u.double().cpu().numpy()
        out.append(r)
    # the probes leave the caller's potential alone and the next evaluation
    # is unaffected: evaluate again and compare with the first result
    v2 = [torch.empty_like(x) for x in ns]
    lib.energy_potential_batched([x.data_ptr() for x in ns], [x.data_ptr() for x in v2])
    assert all(torch.equal(a, b) for a, b in zip(vs, v2))
    return out


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


BARS = {64: dict(theta=1e-12, chat=1e-12, uhat=1e-12, u=1e-12),
        32: dict(theta=4e-6, chat=4e-6, uhat=4e-6, u=8e-6)}


def check_against_oracle(g, o, precision, tag):
    errs = {k: rel(g[k], o[k]) for k in ("theta", "chat", "uhat", "u")}
    say("  %s fp%d: " % (tag, precision) + "  ".join("%s %.2e" % kv for kv in errs.items()))
    for k, e in errs.items():
        assert e <= BARS[precision][k], (k, e)


@pytest.mark.parametrize("precision", [64, 32])
def test_stages_c1(table, precision):
    wl = W.gauss24()
    n = wl.density()
    if precision == 32:
        n = n.astype(np.float32).astype(np.float64)
    o = F.energy_potential(n, wl.cell, table, return_parts=True)
    g = stages([n], [wl.cell], table, precision)[0]
    check_against_oracle(g, o, precision, "24^3")


@pytest.mark.parametrize("precision", [64, 32])
def test_stages_batch_members(table, precision):
    """A batch of uneven grids (ragged, non-cubic cells): every member's stages."""
    cases = [((20, 30, 18), (8.0, 11.0, 7.5)), ((12, 12, 12), (5.0, 5.0, 5.0)), ((32, 16, 48), (6.0, 3.0, 9.0))]
    dens, cells = [], []
    for i, (shape, cell) in enumerate(cases):
        d = W.density_on_grid(shape, cell, W.random_atoms(np.random.default_rng(300 + i), 5, cell))
        if precision == 32:
            d = d.astype(np.float32).astype(np.float64)
        dens.append(d)
        cells.append(cell)
    gs = stages(dens, cells, table, precision)
    for d, c, g in zip(dens, cells, gs):
        check_against_oracle(g, F.energy_potential(d, c, table, return_parts=True), precision, str(d.shape))


def test_stages_finite_differences_and_triclinic(table):
    wl = W.gauss24()
    n = wl.density()
    o = F.energy_potential(n, wl.cell, table, grad_mode=2, return_parts=True)
    check_against_oracle(stages([n], [wl.cell], table, 64, grad_mode=2)[0], o, 64, "24^3 m=2")
    lat = W.triclinic_lattice((7.0, 6.5, 8.0), (80.0, 100.0, 75.0))
    shape = (20, 18, 24)
    nt = W.density_on_lattice(shape, lat, W.random_atoms_lattice(np.random.default_rng(5), 4, lat))
    o = F.energy_potential(nt, lat, table, return_parts=True)
    check_against_oracle(stages([nt], [lat], table, 64)[0], o, 64, "triclinic 20x18x24")
    nt32 = nt.astype(np.float32).astype(np.float64)
    o = F.energy_potential(nt32, lat, table, return_parts=True)
    check_against_oracle(stages([nt32], [lat], table, 32)[0], o, 32, "triclinic 20x18x24")


LENS = (24, 32, 48, 64, 96, 128, 160, 320)
CASES = [(axis, L) for axis in range(3) for L in LENS if not (axis == 0 and L > 204)]


@pytest.mark.parametrize("axis,L", CASES)
def test_transforms_against_numpy_fft(table, axis, L):
    """Every compile-time plan on every axis, transforms only: numpy's rfftn of
    the GPU's theta equals the GPU's c (times N), numpy's irfftn of the GPU's
    u spectra equals the GPU's u(r) (divided by N)."""
    s = [10, 12]
    s.insert(axis, L)
    shape = tuple(s)
    cell = tuple(0.2 * x for x in shape)
    d = W.density_on_grid(shape, cell, W.random_atoms(np.random.default_rng(L + axis), 3, cell))
    for precision in (64, 32):
        dd = d if precision == 64 else d.astype(np.float32).astype(np.float64)
        g = stages([dd], [cell], table, precision)[0]
        N = d.size
        ref_c = np.stack([np.fft.rfftn(g["theta"][a]) for a in range(NQ)]) / N
        ref_u = np.stack([np.fft.irfftn(g["uhat"][a], s=shape) for a in range(NQ)]) * N
        ec, eu = rel(g["chat"], ref_c), rel(g["u"], ref_u)
        say("  axis %d L %d fp%d: forward %.2e  inverse %.2e" % (axis + 1, L, precision, ec, eu))
        bar = 1e-13 if precision == 64 else 2e-6
        assert ec <= bar and eu <= bar


def test_stage_probe_errors(table):
    from paper_0812_0244_amd import VdwNl, VdwNlError
    lib = VdwNl(0)
    lib.set_grid((12, 12, 12), (5.0, 5.0, 5.0), 0, 64)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    buf = torch.empty((NQ, 12, 12, 12), dtype=torch.float64, device="cuda")
    with pytest.raises(VdwNlError) as ex:          # no evaluation yet
        lib.debug_stage(0, 0, buf.data_ptr())
    assert ex.value.code == -6
    n = torch.full((12, 12, 12), 0.01, dtype=torch.float64, device="cuda")
    v = torch.empty_like(n)
    lib.energy_potential(n.data_ptr(), v.data_ptr())
    for inst, stage, code in [(1, 0, -6), (-1, 0, -6), (0, 5, -1), (0, -1, -1)]:
        with pytest.raises(VdwNlError) as ex:
            lib.debug_stage(inst, stage, buf.data_ptr())
        assert ex.value.code == code


@pytest.mark.parametrize("shape,cell,m", [((20, 18, 24), (9.0, 8.0, 10.0), 0), ((16, 20, 15), (7.0, 8.0, 6.0), 0),
                                          ((12, 10, 9), (6.0, 5.0, 4.5), 0), ((16, 20, 15), (7.0, 8.0, 6.0), 2)])
def test_gradient_stage_against_oracle(table, shape, cell, m):
    """grad n as the theta pass takes it: the spectral gradient (one-axis
    passes along the three grid axes, each multiplier i 2 pi m_c / N_c with
    the Nyquist index zero) or the central differences of order 2m, against
    the oracle's 3-D spectral gradient or its stencils; FP64 to 1e-12 of
    max |grad n|, FP32 (same rounded input) to 1e-6."""
    from paper_0812_0244_amd import VdwNl
    from paper_0812_0244_amd.binding import STAGE_GRAD
    rng = np.random.default_rng(sum(shape) + m)
    n = W.density_on_grid(shape, cell, W.random_atoms(rng, 5, cell))
    for prec in (64, 32):
        dt = torch.float64 if prec == 64 else torch.float32
        nin = n if prec == 64 else n.astype(np.float32).astype(np.float64)
        ref = F.gradient(nin, cell) if m == 0 else F.gradient_fd(nin, cell, m)
        lib = VdwNl(0)
        lib.set_grid(shape, cell, m, prec)
        lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
        nt = torch.from_numpy(nin).to("cuda", dt)
        v = torch.empty_like(nt)
        lib.energy_potential(nt.data_ptr(), v.data_ptr())
        g = torch.empty((3,) + shape, dtype=dt, device="cuda")
        lib.debug_stage(0, STAGE_GRAD, g.data_ptr())
        err = np.abs(g.double().cpu().numpy() - ref).max() / np.abs(ref).max()
        say("  %s m=%d FP%d: max |d grad| / max |grad| = %.2e" % (shape, m, prec, err))
        assert err <= (1e-12 if prec == 64 else 1e-6)
