"""Batched evaluation machinery on the GPU: graph replay and tile tuning.

Neither may change results: the graph replays the same launches (bitwise
equal to launching the passes one by one, also after the caller's buffers
change), and tile shapes only change how lines are grouped into workgroups
(v bitwise equal; the energy partial sums are grouped differently, so E
agrees to rounding).
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


def small_batch(k=5, precision=32):
    insts = W.batch_instances(k)
    dt = torch.float32 if precision == 32 else torch.float64
    n = [torch.from_numpy(w.density()).to("cuda", dt) for w in insts]
    return insts, n


def make_ctx(insts, table, precision=32):
    from paper_0812_0244_amd import VdwNl
    lib = VdwNl(0)
    lib.set_grids([w.shape for w in insts], [w.cell for w in insts], 0, precision)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    return lib


def run(lib, n, v):
    return lib.energy_potential_batched([x.data_ptr() for x in n], [x.data_ptr() for x in v])


@pytest.mark.parametrize("precision", [32, 64])
def test_graph_replay_equals_eager(table, precision):
    insts, n = small_batch(5, precision)
    say("  shapes %s precision %d" % ([w.shape for w in insts], precision))
    lib = make_ctx(insts, table, precision)
    eager = make_ctx(insts, table, precision)
    eager.set_graph(False)
    v_e = [torch.empty_like(x) for x in n]
    E_e = run(eager, n, v_e)
    # several replays; the second and third use other buffers (the graph reads
    # the pointers of each call), the densities permuted in content
    for rep in range(3):
        if rep == 0:
            nn = n
        else:
            nn = [x.clone() for x in n]
        v = [torch.full_like(x, float("nan")) for x in nn]
        E = run(lib, nn, v)
        assert np.array_equal(E, E_e), (rep, E, E_e)
        for a, b in zip(v, v_e):
            assert torch.equal(a, b)
    # eager work between replays, then one more replay
    _ = torch.randn(1000, device="cuda").sum().item()
    v = [torch.empty_like(x) for x in n]
    assert np.array_equal(run(lib, n, v), E_e)
    say("  graph replays bitwise equal to eager launches: E[0] = %.15e" % E_e[0].sum())


def test_autotune_keeps_results_and_is_cached(table):
    insts, n = small_batch(6, 32)
    lib = make_ctx(insts, table, 32)
    v0 = [torch.empty_like(x) for x in n]
    E0 = run(lib, n, v0)
    before = lib.get_tiling()
    lib.autotune([x.data_ptr() for x in n], [x.data_ptr() for x in v0], reps=1)
    after = lib.get_tiling()
    say("  LDS budgets before %s after %s" % (before, after))
    assert all(b in (16384, 24576, 32768, 49152, 65536, 98304, 131072) for b in after.values())
    say("  radix orders %s, contraction unit %d" % (lib.get_radix_orders(), lib.get_contraction()))
    v1 = [torch.empty_like(x) for x in n]
    E1 = run(lib, n, v1)
    # (other radix orders and contraction units round differently: FP32 bars)
    for a, b in zip(v0, v1):
        assert float((a.double() - b.double()).abs().max()) <= 1e-5
    np.testing.assert_allclose(E1, E0, rtol=1e-6, atol=0)
    # a new context planning the same grid list picks the tuned budgets up
    lib2 = make_ctx(insts, table, 32)
    assert lib2.get_tiling() == after
    assert lib2.get_radix_orders() == lib.get_radix_orders() and lib2.get_contraction() == lib.get_contraction()
    v2 = [torch.empty_like(x) for x in n]
    E2 = run(lib2, n, v2)
    assert np.array_equal(E2, E1)


def test_tuning_file_persists_across_processes(table, tmp_path, monkeypatch):
    """Tuned budgets land in the tuning file (a JSON object keyed by device
    architecture and plan) and a later process planning the same grid list
    takes its budgets from there: the entry is edited here, and a fresh
    process must plan with exactly the edited values."""
    import json
    import os
    import subprocess
    path = tmp_path / "tuning.json"
    monkeypatch.setenv("VDWNL_TUNE_CACHE", str(path))
    insts, n = small_batch(3, 32)
    lib = make_ctx(insts, table, 32)
    v = [torch.empty_like(x) for x in n]
    lib.autotune([x.data_ptr() for x in n], [x.data_ptr() for x in v], reps=1)
    entries = json.load(open(path))
    say("  tuning file: %s" % entries)
    assert len(entries) == 1
    key = next(iter(entries))
    # the five LDS budgets, the contraction unit, the five radix orders
    assert key.startswith("gfx") and entries[key][:5] == list(lib.get_tiling().values())
    assert entries[key][5] == lib.get_contraction()
    assert entries[key][6:] == list(lib.get_radix_orders().values())
    orders = [1, 5, 0, 4, 1]          # (orders 4 and 5: the two-pass radix-16 plans)
    json.dump({key: [24576] * 5 + [1 - entries[key][5]] + orders}, open(path, "w"))
    code = ("import sys, json; sys.path.insert(0, %r)\n"
            "import workloads as W\n"
            "from paper_0812_0244_amd import VdwNl\n"
            "insts = W.batch_instances(3)\n"
            "lib = VdwNl(0)\n"
            "lib.set_grids([w.shape for w in insts], [w.cell for w in insts], 0, 32)\n"
            "print(json.dumps([lib.get_tiling(), lib.get_contraction(), lib.get_radix_orders()]))\n"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                         env=dict(os.environ))
    assert out.returncode == 0, out.stderr
    got, unit, radix = json.loads(out.stdout.strip().splitlines()[-1])
    say("  budgets in the new process: %s, contraction unit %d, radix orders %s" % (got, unit, radix))
    assert list(got.values()) == [24576] * 5 and unit == 1 - entries[key][5] and list(radix.values()) == orders


def test_every_radix_order_against_oracle(table):
    """Every radix order of every compile-time length class, on every axis, in
    one batch of thin grids: each order (all five pass groups at once) in FP64
    against the oracle (1e-10) and in FP32 against the oracle on the same
    rounded input (1e-6 relative E, 1e-5 Ha)."""
    from oracle import functional as F
    from paper_0812_0244_amd import VdwNl
    shapes = []
    for L in (32, 48, 64, 96, 128, 160, 320):
        for axis in range(3):
            if axis == 0 and L > 204:
                continue
            sh = [10, 12]
            sh.insert(axis, L)
            shapes.append(tuple(sh))
    cells = [tuple(0.2 * x for x in sh) for sh in shapes]
    dens = [W.density_on_grid(sh, c, W.random_atoms(np.random.default_rng(500 + i), 3, c))
            for i, (sh, c) in enumerate(zip(shapes, cells))]
    for prec in (64, 32):
        dt = torch.float64 if prec == 64 else torch.float32
        ins = [d if prec == 64 else d.astype(np.float32).astype(np.float64) for d in dens]
        ref = [F.energy_potential(d, c, table) for d, c in zip(ins, cells)]
        lib = VdwNl(0)
        lib.set_grids(shapes, cells, 0, prec)
        lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
        ns = [torch.from_numpy(d).to("cuda", dt) for d in ins]
        for order in range(6):
            lib.set_radix_orders([order] * 5)
            vs = [torch.empty_like(x) for x in ns]
            E = lib.energy_potential_batched([x.data_ptr() for x in ns], [x.data_ptr() for x in vs])
            worst_e, worst_v = 0.0, 0.0
            for i, (ek, de, vo) in enumerate(ref):
                e_rel = abs(E[i].sum() - (ek + de)) / abs(ek + de)
                dv = float(np.abs(vs[i].double().cpu().numpy() - vo).max())
                worst_e = max(worst_e, e_rel)
                worst_v = max(worst_v, dv / np.abs(vo).max() if prec == 64 else dv)
                if prec == 64:
                    assert e_rel <= 1e-10 and dv <= 1e-10 * np.abs(vo).max(), (shapes[i], order, e_rel, dv)
                else:
                    assert e_rel <= 1e-6 and dv <= 1e-5, (shapes[i], order, e_rel, dv)
            say("  fp%d radix order %d: worst rel E %.2e, worst dv %.2e" % (prec, order, worst_e, worst_v))
