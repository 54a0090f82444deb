"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 runs must agree with the oracle to rounding (relative 1e-10 in E and
in max|v|); FP32 runs to the accuracy the method is specified at: relative
energy error <= 1e-6 and max |dv| <= 1e-5 Ha.  An FP32 run receives the
density rounded to FP32, so the oracle evaluates that same rounded density:
v_nl is ill-conditioned in n where n sits on the 1e-4 floor (the gradient
term scales as 1/n), and the input rounding alone moves the FP64 oracle's v
by up to 4.6e-5 Ha on the 96^3 workload.  That figure is asserted too.
"""
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


def gpu_eval(n, cell, table, precision, debug=False):
    from paper_0812_0244_amd import NonlocalCorrelation
    say("  gpu eval shape=%s cell=%s precision=%d" % (n.shape, cell, precision))
    eng = NonlocalCorrelation(n.shape, cell, table, precision=precision, device=0)
    dt = torch.float64 if precision == 64 else torch.float32
    nt = torch.from_numpy(n).to(device="cuda", dtype=dt)
    ek, de, v = eng.energy_potential(nt)
    out = dict(E_k=ek, dE=de, v=v.double().cpu().numpy())
    if debug:
        from paper_0812_0244_amd.binding import STAGE_GRAD
        # after the evaluation: the lattice components q_c of w, and v_loc;
        # then the gradient passes again for grad n itself
        q = torch.empty((3,) + n.shape, dtype=dt, device="cuda")
        eng.lib.debug_field(0, 0, q.data_ptr())
        vl = torch.empty(n.shape, dtype=dt, device="cuda")
        eng.lib.debug_field(0, 1, vl.data_ptr())
        g = torch.empty((3,) + n.shape, dtype=dt, device="cuda")
        eng.lib.debug_stage(0, STAGE_GRAD, g.data_ptr())
        out["q"] = q.double().cpu().numpy()
        out["grad"] = g.double().cpu().numpy()
        out["v_loc"] = vl.double().cpu().numpy()
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


def test_c1_fp64_parity_with_intermediates(table):
    wl = W.gauss24()
    n = wl.density()
    o = F.energy_potential(n, wl.cell, table, return_parts=True)
    g = gpu_eval(n, wl.cell, table, 64, debug=True)
    np.testing.assert_allclose(g["grad"], o["grad"], rtol=0, atol=1e-12 * np.abs(o["grad"]).max())
    np.testing.assert_allclose(g["v_loc"], o["v_loc"], rtol=0, atol=1e-10 * np.abs(o["v_loc"]).max())
    # the divergence passes' input: q_c = sum_x W[c][x] w_x of the vector field of Eq. (Vi)
    q = np.einsum("cx,x...->c...", F.fd_metric(n.shape, wl.cell), o["w"])
    np.testing.assert_allclose(g["q"], q, rtol=0, atol=1e-10 * np.abs(q).max())
    check(g, o, 64)


def fp32_input(n):
    return n.astype(np.float32).astype(np.float64)


def test_c1_fp32_parity(table):
    wl = W.gauss24()
    n = fp32_input(wl.density())
    o = F.energy_potential(n, wl.cell, table, return_parts=True)
    check(gpu_eval(n, wl.cell, table, 32), o, 32)


@pytest.mark.parametrize("shape,cell,natoms", [
    ((12, 12, 12), (10.0, 10.0, 10.0), 4),
    ((20, 30, 18), (8.0, 11.0, 7.5), 6),
    ((32, 16, 48), (6.0, 3.0, 9.0), 5),
    ((40, 36, 50), (9.0, 8.0, 10.0), 9),
    ((6, 8, 10), (3.0, 4.0, 5.0), 2),
    ((16, 20, 15), (7.0, 8.0, 6.0), 4),       # odd N3: rows of odd length, odd i3 runs
    ((10, 12, 25), (5.0, 6.0, 9.0), 3),
])
def test_fp64_parity_ragged_shapes(table, shape, cell, natoms):
    rng = np.random.default_rng(sum(shape))
    n = W.density_on_grid(shape, cell, W.random_atoms(rng, natoms, cell))
    o = F.energy_potential(n, cell, table, return_parts=True)
    check(gpu_eval(n, cell, table, 64), o, 64)


def test_c2_fp64_and_fp32_parity(table):
    wl = W.gauss96()
    n = wl.density()
    o = F.energy_potential(n, wl.cell, table, return_parts=True)
    check(gpu_eval(n, wl.cell, table, 64), o, 64)
    n32 = fp32_input(n)
    o32 = F.energy_potential(n32, wl.cell, table, return_parts=True)
    g32 = gpu_eval(n32, wl.cell, table, 32)
    check(g32, o32, 32)
    # against the FP64-input oracle: energy to 1e-6, v limited by the input rounding
    e64 = o["E_k"] + o["dE"]
    assert abs(g32["E_k"] + g32["dE"] - e64) <= FP32_EREL * abs(e64)
    say("  FP32 run vs FP64-input oracle: max|dv| %.2e" % np.abs(g32["v"] - o["v"]).max())
    assert np.abs(g32["v"] - o["v"]).max() <= 1e-4


def test_constant_table_closed_form_on_gpu(table):
    """phi_ab(k) = f(k) for every pair: E_k = 1/2 Int Int n n f, v = f * n."""
    s = 1.0
    t = dict(table)
    k = np.arange(table["nk"]) * table["dk"]
    f = np.pi ** 1.5 * s ** 3 * np.exp(-(k * s) ** 2 / 4.0)
    t["phi"] = np.broadcast_to(f, (20, 20, k.size)).copy()
    t["c_soft"] = 0.0
    cell = (8.0, 8.0, 8.0)
    atoms = W.random_atoms(np.random.default_rng(11), 5, cell)
    n = W.density_on_grid((32, 32, 32), cell, atoms)
    o = F.energy_potential(n, cell, t, return_parts=True)
    g = gpu_eval(n, cell, t, 64)
    assert g["dE"] == 0.0
    np.testing.assert_allclose(g["E_k"], o["E_k"], rtol=1e-11)
    np.testing.assert_allclose(g["v"], o["v"], rtol=0, atol=1e-11 * np.abs(o["v"]).max())


def test_batched_equals_single(table):
    from paper_0812_0244_amd import VdwNl
    cases = [((24, 24, 24), (10.0, 10.0, 10.0)), ((12, 20, 16), (6.0, 9.0, 7.0)), ((32, 24, 20), (9.0, 7.0, 6.0))]
    dens = []
    for i, (shape, cell) in enumerate(cases):
        dens.append(W.density_on_grid(shape, cell, W.random_atoms(np.random.default_rng(100 + i), 5, cell)))
    for prec in (64, 32):
        dt = torch.float64 if prec == 64 else torch.float32
        say("  batched precision %d" % prec)
        lib = VdwNl(0)
        lib.set_grids([c[0] for c in cases], [c[1] for c in cases], 0, prec)
        lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
        ns = [torch.from_numpy(d).to("cuda", dt) for d in dens]
        vs = [torch.empty_like(x) for x in ns]
        E = lib.energy_potential_batched([x.data_ptr() for x in ns], [x.data_ptr() for x in vs])
        for i, (shape, cell) in enumerate(cases):
            g = gpu_eval(dens[i], cell, table, prec)
            assert E[i, 0] == g["E_k"] and E[i, 1] == g["dE"]
            assert np.array_equal(vs[i].double().cpu().numpy(), g["v"])


def test_repeat_runs_bitwise_identical(table):
    from paper_0812_0244_amd import NonlocalCorrelation
    wl = W.gauss24()
    n = torch.from_numpy(wl.density()).to("cuda", torch.float32)
    eng = NonlocalCorrelation(n.shape, wl.cell, table, precision=32)
    ref = eng.energy_potential(n)
    for _ in range(5):
        r = eng.energy_potential(n)
        assert r[0] == ref[0] and r[1] == ref[1]
        assert torch.equal(r[2], ref[2])


def test_uniform_density_on_node_gives_zero_on_gpu(table):
    """Constant density with q0 on a mesh node: E_k + Delta E = 0 (the kernel
    integrates to zero over a uniform density), on the GPU's G = 0 path."""
    from tests.test_oracle_pipeline import _uniform_density_for_q
    n0 = _uniform_density_for_q(table["qmesh"][12], table)
    n = np.full((16, 16, 16), n0)
    g = gpu_eval(n, (6.0, 6.0, 6.0), table, 64)
    assert abs(g["E_k"] + g["dE"]) < 1e-6 * abs(g["dE"])
    np.testing.assert_allclose(g["v"], g["v"].flat[0], rtol=1e-10)


def test_autograd_backward_is_dvol_times_v(table):
    from paper_0812_0244_amd import NonlocalCorrelation
    wl = W.gauss24()
    eng = NonlocalCorrelation(wl.shape, wl.cell, table, precision=64)
    n = torch.from_numpy(wl.density()).to("cuda").requires_grad_(True)
    E = eng(n)
    E.backward()
    _, _, v = eng.energy_potential(n.detach())
    assert torch.equal(n.grad, v * eng.dvol)


def test_contraction_units_agree_with_oracle(table):
    """The per-k contraction of Eqs. (Eoffk)/(epsofk) on the vector ALU and on
    the matrix cores (FP32): both against the oracle on the same rounded input
    (1e-6 relative E, 1e-5 Ha), and against each other; the probed u spectra
    too.  Single columns and column pairs (tile budgets 32 and 48 KB) on the
    96^3 workload, a ragged non-cubic grid."""
    from paper_0812_0244_amd import VdwNl
    from paper_0812_0244_amd.binding import CONTRACTION_MATRIX, CONTRACTION_VECTOR, STAGE_U_K
    cases = [(W.gauss96().density(), W.gauss96().cell, W.gauss96().shape),
             (None, (8.0, 11.0, 7.5), (20, 30, 18))]
    for n, cell, shape in cases:
        if n is None:
            n = W.density_on_grid(shape, cell, W.random_atoms(np.random.default_rng(77), 6, cell))
        n = fp32_input(n)
        o = F.energy_potential(n, cell, table, return_parts=True)
        nt = torch.from_numpy(n).to("cuda", torch.float32)
        res = {}
        for zb in (32768, 49152):
            for unit in (CONTRACTION_VECTOR, CONTRACTION_MATRIX):
                lib = VdwNl(0)
                lib.set_grid(shape, cell, 0, 32)
                lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
                lib.set_tiling([65536, 65536, 65536, zb, 65536])
                lib.set_contraction(unit)
                assert lib.get_contraction() == unit
                v = torch.empty_like(nt)
                ek, de = lib.energy_potential(nt.data_ptr(), v.data_ptr())
                uk = torch.empty((shape[0], shape[1], shape[2] // 2 + 1, 20, 2), dtype=torch.float32, device="cuda")
                lib.debug_stage(0, STAGE_U_K, uk.data_ptr())
                g = dict(E_k=ek, dE=de, v=v.double().cpu().numpy())
                say("  %s z budget %d unit %d" % (shape, zb, unit))
                check(g, o, 32)
                res[(zb, unit)] = (ek + de, g["v"], uk.double().cpu().numpy())
        base = res[(32768, CONTRACTION_VECTOR)]
        for key, r in res.items():
            assert abs(r[0] - base[0]) <= 1e-6 * abs(base[0])
            assert np.abs(r[1] - base[1]).max() <= 1e-5
            assert np.abs(r[2] - base[2]).max() <= 2e-6 * np.abs(base[2]).max()
