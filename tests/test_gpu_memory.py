"""Device memory over re-planning.  A context keeps one workspace allocation
across plans (it is re-allocated only when a plan needs more, and freed when
the context is destroyed): device memory freed while a context held captured
graphs was not returned to the device on this runtime, so re-planning with
graph replay (tile budgets, tuning) lost one workspace per plan."""
import sys

import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_replanning_with_graphs_keeps_one_workspace(table):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0812_0244_amd import VdwNl
    insts = W.batch_instances(64)[:16]
    lib = VdwNl(0)
    lib.set_grids([w.shape for w in insts], [w.cell for w in insts], 0, 32)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    n = [torch.from_numpy(w.density()).to("cuda", torch.float32) for w in insts]
    v = [torch.empty_like(x) for x in n]
    nptr, vptr = [x.data_ptr() for x in n], [x.data_ptr() for x in v]

    def free_bytes():
        torch.cuda.synchronize()
        return torch.cuda.mem_get_info()[0]

    E0 = lib.energy_potential_batched(nptr, vptr)          # (graph captured)
    ws = lib.info()[1]
    f0 = free_bytes()
    for i in range(6):
        lib.set_tiling([65536, 49152 if i % 2 else 32768, 49152, 49152, 49152])
        E = lib.energy_potential_batched(nptr, vptr)
        E = lib.energy_potential_batched(nptr, vptr)        # (graph replay)
        assert abs(E[:, 0] - E0[:, 0]).max() <= 1e-12 * abs(E0[:, 0]).max()
    f1 = free_bytes()
    say("  workspace %.2f GB; free memory %.2f -> %.2f GB over six re-plans" % (ws / 2 ** 30, f0 / 2 ** 30, f1 / 2 ** 30))
    assert f0 - f1 < ws // 4


def test_contexts_reuse_workspaces(table):
    """Contexts created and destroyed one after another (each evaluating with
    graph replay) reuse the process's pooled workspace: device free memory
    drops by one workspace at most over five contexts."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0812_0244_amd import VdwNl
    insts = W.batch_instances(64)[:16]
    n = [torch.from_numpy(w.density()).to("cuda", torch.float32) for w in insts]
    v = [torch.empty_like(x) for x in n]
    nptr, vptr = [x.data_ptr() for x in n], [x.data_ptr() for x in v]

    def free_bytes():
        torch.cuda.synchronize()
        return torch.cuda.mem_get_info()[0]

    f0 = free_bytes()
    ws = 0
    E0 = None
    for _ in range(5):
        lib = VdwNl(0)
        lib.set_grids([w.shape for w in insts], [w.cell for w in insts], 0, 32)
        lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
        E = lib.energy_potential_batched(nptr, vptr)
        E = lib.energy_potential_batched(nptr, vptr)          # (graph replay)
        if E0 is None:
            E0 = E
        assert (E == E0).all()
        ws = lib.info()[1]
        del lib
    f1 = free_bytes()
    say("  workspace %.2f GB; free memory %.2f -> %.2f GB over five contexts" % (ws / 2 ** 30, f0 / 2 ** 30, f1 / 2 ** 30))
    assert f0 - f1 < ws + ws // 4
