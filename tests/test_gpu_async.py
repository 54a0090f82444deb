"""The asynchronous batched call through the C ABI: the energies it leaves in
a device array equal the synchronous call's bitwise, v likewise; calls in a
row with other buffers each see their own; the semilocal energies of an
asynchronous evaluation of the whole functional are those of the
synchronous one."""
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


def _lib(table, insts, precision, graph=True):
    from paper_0812_0244_amd import VdwNl
    lib = VdwNl(0)
    lib.set_grids([w.shape for w in insts], [w.cell for w in insts], 0, precision)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    lib.set_graph(graph)
    return lib


@pytest.mark.parametrize("precision,graph", [(32, True), (64, True), (32, False)])
def test_async_equals_sync(table, precision, graph):
    insts = [W.gauss24()] + W.batch_instances(3)[:2]
    say("  async vs sync: %s precision=%d graph=%s" % ([w.shape for w in insts], precision, graph))
    dt = torch.float64 if precision == 64 else torch.float32
    n = [torch.from_numpy(w.density()).to("cuda", dt) for w in insts]
    lib = _lib(table, insts, precision, graph)
    v_s = [torch.empty_like(x) for x in n]
    E_s = lib.energy_potential_batched([x.data_ptr() for x in n], [x.data_ptr() for x in v_s])
    stream = torch.cuda.current_stream().cuda_stream
    v_a = [torch.full_like(x, float("nan")) for x in n]
    E_a = torch.full((len(n), 2), float("nan"), dtype=torch.float64, device="cuda")
    lib.energy_potential_batched_async([x.data_ptr() for x in n], [x.data_ptr() for x in v_a], E_a.data_ptr(), stream)
    torch.cuda.synchronize()
    assert np.array_equal(E_a.cpu().numpy(), E_s)
    assert all(torch.equal(a, b) for a, b in zip(v_a, v_s))


def test_async_calls_in_a_row(table):
    """Two asynchronous calls with other densities and buffers, then a
    synchronous one: each result is its own (the second call waits for the
    first to release the instance table)."""
    insts = W.batch_instances(4)[2:]
    lib = _lib(table, insts, 32)
    stream = torch.cuda.current_stream().cuda_stream
    n1 = [torch.from_numpy(w.density()).to("cuda", torch.float32) for w in insts]
    n2 = [x * 0.9 + 1e-4 for x in n1]
    ref = []
    for n in (n1, n2):
        v = [torch.empty_like(x) for x in n]
        ref.append((lib.energy_potential_batched([x.data_ptr() for x in n], [x.data_ptr() for x in v]), v))
    outs = []
    for n in (n1, n2):
        v = [torch.empty_like(x) for x in n]
        E = torch.empty((len(n), 2), dtype=torch.float64, device="cuda")
        lib.energy_potential_batched_async([x.data_ptr() for x in n], [x.data_ptr() for x in v], E.data_ptr(), stream)
        outs.append((E, v))
    torch.cuda.synchronize()
    for (E_ref, v_ref), (E, v) in zip(ref, outs):
        assert np.array_equal(E.cpu().numpy(), E_ref)
        assert all(torch.equal(a, b) for a, b in zip(v, v_ref))


def test_async_semilocal_energies(table):
    from paper_0812_0244_amd.binding import FUNCTIONAL_VDW_DF
    insts = [W.gauss24()]
    lib = _lib(table, insts, 64)
    lib.set_functional(FUNCTIONAL_VDW_DF)
    n = [torch.from_numpy(insts[0].density()).to("cuda")]
    v = [torch.empty_like(n[0])]
    lib.energy_potential_batched([n[0].data_ptr()], [v[0].data_ptr()])
    S_sync = lib.semilocal_energies()
    E = torch.empty((1, 2), dtype=torch.float64, device="cuda")
    lib.energy_potential_batched_async([n[0].data_ptr()], [v[0].data_ptr()], E.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream)
    assert np.array_equal(lib.semilocal_energies(), S_sync)
