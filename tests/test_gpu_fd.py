"""Parity of the finite-difference gradient mode (grad_mode m = 1..4, the
paper's treatment of grad n around Eq. (Vi)) of the HIP path with the FP64
oracle, through the C ABI.

Same bars as the spectral mode: FP64 to rounding (relative 1e-10 in each
energy part and in max|v|), FP32 at relative energy error <= 1e-6 and
max|dv| <= 1e-5 Ha against the oracle of the FP32-rounded density.  The
intermediates are compared too: the vector field w of Eq. (Vi) (whose
lattice components q_c = sum_x W[c][x] w_x the library stores in place of
grad n in this mode) and v_loc.
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


def gpu_eval(n, cell, table, precision, m, debug=False):
    from paper_0812_0244_amd import NonlocalCorrelation
    say("  gpu eval shape=%s cell=%s precision=%d grad_mode=%d" % (n.shape, cell, precision, m))
    eng = NonlocalCorrelation(n.shape, cell, table, precision=precision, device=0, grad_mode=m)
    dt = torch.float64 if precision == 64 else torch.float32
    ek, de, v = eng.energy_potential(torch.from_numpy(n).to(device="cuda", dtype=dt))
    out = dict(E_k=ek, dE=de, v=v.double().cpu().numpy())
    if debug:
        w = torch.empty((3,) + n.shape, dtype=dt, device="cuda")
        eng.lib.debug_field(0, 0, w.data_ptr())
        vl = torch.empty(n.shape, dtype=dt, device="cuda")
        eng.lib.debug_field(0, 1, vl.data_ptr())
        out["w"] = w.double().cpu().numpy()
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


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_c1_fp64_fd_parity_with_intermediates(table, m):
    wl = W.gauss24()
    n = wl.density()
    o = F.energy_potential(n, wl.cell, table, return_parts=True, grad_mode=m)
    g = gpu_eval(n, wl.cell, table, 64, m, debug=True)
    np.testing.assert_allclose(g["v_loc"], o["v_loc"], rtol=0, atol=1e-10 * np.abs(o["v_loc"]).max())
    # the buffer holds the lattice components q_c = sum_x W[c][x] w_x of w
    q = np.einsum("cx,x...->c...", F.fd_metric(n.shape, wl.cell), o["w"])
    np.testing.assert_allclose(g["w"], q, rtol=0, atol=1e-10 * np.abs(q).max())
    check(g, o, 64)


@pytest.mark.parametrize("shape,cell,natoms,m", [
    ((4, 6, 8), (2.0, 3.0, 4.0), 1, 4),        # edges shorter than the stencil: folded weights
    ((12, 12, 12), (10.0, 10.0, 10.0), 4, 3),
    ((20, 30, 18), (8.0, 11.0, 7.5), 6, 2),
    ((32, 16, 48), (6.0, 3.0, 9.0), 5, 3),
    ((40, 36, 50), (9.0, 8.0, 10.0), 9, 4),
    ((6, 8, 10), (3.0, 4.0, 5.0), 2, 1),
])
def test_fp64_fd_parity_ragged_shapes(table, shape, cell, natoms, m):
    rng = np.random.default_rng(sum(shape) + m)
    n = W.density_on_grid(shape, cell, W.random_atoms(rng, natoms, cell))
    o = F.energy_potential(n, cell, table, return_parts=True, grad_mode=m)
    check(gpu_eval(n, cell, table, 64, m), o, 64)


def test_c2_fd_fp64_and_fp32_parity(table):
    wl = W.gauss96()
    n = wl.density()
    o = F.energy_potential(n, wl.cell, table, grad_mode=3, return_parts=True)
    check(gpu_eval(n, wl.cell, table, 64, 3), o, 64)
    n32 = n.astype(np.float32).astype(np.float64)
    o32 = F.energy_potential(n32, wl.cell, table, grad_mode=3, return_parts=True)
    check(gpu_eval(n32, wl.cell, table, 32, 3), o32, 32)


def test_fd_batched_equals_single_and_graph_replay(table):
    """A batch of uneven grids in FD mode: each member equals its own
    single-grid evaluation (bitwise: the same tiles), graph replays equal
    eager launches, and every FP64 member (128^3 and 32^3) matches the oracle."""
    from paper_0812_0244_amd import NonlocalCorrelation, VdwNl
    insts = W.batch_instances(4)
    n = [torch.from_numpy(w.density()).to("cuda", torch.float64) for w in insts]
    lib = VdwNl(0)
    lib.set_grids([w.shape for w in insts], [w.cell for w in insts], 3, 64)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    v = [torch.empty_like(x) for x in n]
    E = lib.energy_potential_batched([x.data_ptr() for x in n], [x.data_ptr() for x in v])
    for rep in range(2):
        v2 = [torch.full_like(x, float("nan")) for x in n]
        E2 = lib.energy_potential_batched([x.data_ptr() for x in n], [x.data_ptr() for x in v2])
        assert np.array_equal(E, E2)
        assert all(torch.equal(a, b) for a, b in zip(v, v2))
    lib.set_graph(False)
    v3 = [torch.empty_like(x) for x in n]
    assert np.array_equal(E, lib.energy_potential_batched([x.data_ptr() for x in n], [x.data_ptr() for x in v3]))
    assert all(torch.equal(a, b) for a, b in zip(v, v3))
    for i, w in enumerate(insts):
        say("  member %d shape %s" % (i, w.shape))
        eng = NonlocalCorrelation(w.shape, w.cell, table, precision=64, device=0, grad_mode=3)
        ek, de, vs = eng.energy_potential(n[i])
        assert (ek, de) == (E[i, 0], E[i, 1])
        assert torch.equal(vs, v[i])
        o = F.energy_potential(w.density(), w.cell, table, grad_mode=3, return_parts=True)
        check(dict(E_k=ek, dE=de, v=vs.cpu().numpy()), o, 64)


def test_fd_pass_order_and_timing(table):
    from paper_0812_0244_amd import VdwNl
    wl = W.gauss24()
    lib = VdwNl(0)
    lib.set_grid(wl.shape, wl.cell, 2, 32)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    n = torch.from_numpy(wl.density()).to("cuda", torch.float32)
    v = torch.empty_like(n)
    lib.set_timing(True)
    lib.energy_potential(n.data_ptr(), v.data_ptr())
    t = lib.pass_times()
    say("  passes %s" % list(t))
    assert list(t) == ["fd_grad", "x_theta", "y_20f", "z_main", "y_20i", "x_assemble", "fd_div", "reduce"]
    assert all(ms > 0 and calls == 1 for ms, calls in t.values())
