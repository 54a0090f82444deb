"""The full-size workloads, in the launch configuration the benchmark times.

At these sizes the oracle is not run on every output, so the checks are:
the oracle on one member of every edge length of the batch (up to 128^3),
every member's FP32 potential against the FP64 GPU path on the same
FP32-rounded input, properties that hold
at any size (v = dE/dn by central differences of FP64 energies, translation
invariance), and the forces of the differentiation workload against central
differences of the energy in the atom positions.
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


def engine(shape, cell, table, precision):
    from paper_0812_0244_amd import NonlocalCorrelation
    return NonlocalCorrelation(shape, cell, table, precision=precision)


def run(eng, n):
    ek, de, v = eng.energy_potential(n)
    return ek + de, v


def test_batched_workload_against_fp64_plain_and_oracle(table):
    from oracle import functional as F
    from paper_0812_0244_amd import VdwNl
    insts = W.batch_instances(64)
    dens = [w.density() for w in insts]
    lib = VdwNl(0)
    lib.set_grids([w.shape for w in insts], [w.cell for w in insts], 0, 32)
    lib.set_kernel_table(table["qmesh"], table["qc"], 12, table["dk"], table["phi"], table["c_soft"])
    n32 = [torch.from_numpy(d).to("cuda", torch.float32) for d in dens]
    v32 = [torch.empty_like(x) for x in n32]
    E32 = lib.energy_potential_batched([x.data_ptr() for x in n32], [x.data_ptr() for x in v32])
    worst, worst_dv = 0.0, 0.0
    checked_edges = set()
    for i, w in enumerate(insts):
        eng = engine(w.shape, w.cell, table, 64)
        e64, _ = run(eng, torch.from_numpy(dens[i]).cuda())
        rel = abs(E32[i].sum() - e64) / abs(e64)
        worst = max(worst, rel)
        assert rel <= 1e-6, (i, rel)
        # v of every member against the FP64 path on the same FP32-rounded input
        e64r, v64r = run(eng, n32[i].double())
        dv = float((v32[i].double() - v64r).abs().max())
        worst_dv = max(worst_dv, dv)
        assert dv <= 1e-5, (i, w.shape, dv)
        assert abs(E32[i].sum() - e64r) <= 1e-6 * abs(e64r)
        # the first member of every edge length against the oracle (same input)
        if w.shape[0] not in checked_edges:
            checked_edges.add(w.shape[0])
            n32h = n32[i].double().cpu().numpy()
            ek, de, vo = F.energy_potential(n32h, w.cell, table)
            dvo = np.abs(v32[i].double().cpu().numpy() - vo).max()
            say("  member %d (%d^3): E gpu32 %.12e oracle %.12e  max|dv| %.2e (gpu64 same input %.2e)"
                % (i, w.shape[0], E32[i].sum(), ek + de, dvo, dv))
            assert abs(E32[i].sum() - (ek + de)) <= 1e-6 * abs(ek + de)
            assert dvo <= 1e-5
            assert abs(e64r - (ek + de)) <= 1e-10 * abs(ek + de)
            assert float(np.abs(v64r.cpu().numpy() - vo).max()) <= 1e-10 * np.abs(vo).max()
    assert checked_edges == {32, 48, 64, 96, 128}
    say("  batched FP32 vs FP64 plain: worst relative energy difference %.2e, worst max|dv| "
        "(same input) %.2e Ha" % (worst, worst_dv))


def _directional_check(eng, n, cell, centre, dvol, eps=1e-4, width=1.5):
    """dE/d eps along n + eps f, f = n exp(-|r - centre|^2 / width^2) (a smooth,
    localized change of the density), against dOmega sum_i v_i f_i (Eq. Vi)."""
    _, v = run(eng, n)
    shape = n.shape
    axes = [torch.arange(shape[c], dtype=torch.float64, device=n.device) * (cell[c] / shape[c]) for c in range(3)]
    d2 = 0
    for c in range(3):
        dx = axes[c] - centre[c]
        dx = dx - cell[c] * torch.round(dx / cell[c])
        d2 = d2 + (dx ** 2).reshape([-1 if k == c else 1 for k in range(3)])
    f = n * torch.exp(-d2 / width ** 2)
    fd = (run(eng, n + eps * f)[0] - run(eng, n - eps * f)[0]) / (2 * eps)
    pred = dvol * float((v * f).sum())
    say("  directional derivative at %s: FD %.10e  dOmega sum v f %.10e" % (tuple(round(x, 2) for x in centre), fd, pred))
    assert abs(fd - pred) <= 1e-6 * abs(pred)


def test_dwnt_workload(table):
    wl = W.dwnt_workload()
    n = wl.density()
    say("  DWNT: %d atoms, %s grid" % (wl.meta["atoms"], wl.shape))
    e64eng = engine(wl.shape, wl.cell, table, 64)
    n64 = torch.from_numpy(n).cuda()
    e64, v64 = run(e64eng, n64)
    e32eng = engine(wl.shape, wl.cell, table, 32)
    n32 = n64.float()
    e32, v32 = run(e32eng, n32)
    e64r, v64r = run(e64eng, n32.double())     # FP64 path on the FP32-rounded input
    dv = float((v32.double() - v64r).abs().max())
    say("  E fp64 %.12e  fp32 %.12e  rel %.2e  max|dv| (same input) %.2e" % (e64, e32, abs(e32 - e64) / abs(e64), dv))
    assert abs(e32 - e64) <= 1e-6 * abs(e64)
    assert dv <= 1e-5
    # translation by a lattice vector of the grid
    et, vt = run(e64eng, torch.roll(n64, shifts=(7, -3, 11), dims=(0, 1, 2)))
    assert abs(et - e64) <= 1e-12 * abs(e64)
    assert torch.allclose(vt, torch.roll(v64, shifts=(7, -3, 11), dims=(0, 1, 2)), rtol=0, atol=1e-11)
    dvol = np.prod(wl.cell) / n.size
    # v is the gradient of E: directional derivatives along smooth bumps on
    # the two walls (a change of a single grid value rings through the
    # spectral gradient into the 1e-4 floor, where the gradient term is
    # 1/n-sensitive, and is not resolved by differences of FP64 energies)
    for centre in [(15.0 + 6.4, 15.0, 30.0), (15.0, 15.0 - 12.8, 11.0)]:
        _directional_check(e64eng, n64, wl.cell, centre, dvol)


def test_differentiation_workload_forces(table):
    """Forces F_A = -dE/dR_A through the torch density builder (autograd,
    backward = dOmega v) against central differences of FP64 energies with
    h = 1e-4 bohr; the FP32 path's forces against the FP64 ones."""
    wl = W.gauss128()
    say("  %d atoms, %s grid" % (len(wl.atoms.amp), wl.shape))
    pos = torch.tensor(wl.atoms.pos, dtype=torch.float64, device="cuda")
    e64 = engine(wl.shape, wl.cell, table, 64)
    e32 = engine(wl.shape, wl.cell, table, 32)

    def energy(p, eng):
        n = W.density_torch(wl.shape, wl.cell, wl.atoms.amp, wl.atoms.width, p)
        if eng.precision == 32:
            n = n.float()
        return eng(n)

    r = pos.clone().requires_grad_(True)
    E = energy(r, e64)
    E.backward()
    f64 = -r.grad.cpu().numpy()
    r32 = pos.clone().requires_grad_(True)
    energy(r32, e32).backward()
    f32 = -r32.grad.cpu().numpy()
    fscale = np.abs(f64).max()
    say("  max|F| %.3e  max|F32 - F64| %.3e" % (fscale, np.abs(f32 - f64).max()))
    assert np.abs(f32 - f64).max() <= 1e-4 * fscale + 1e-7
    h = 1e-4
    for a, c in [(0, 0), (17, 1), (63, 2), (127, 0)]:
        pp = pos.clone()
        pp[a, c] += h
        pm = pos.clone()
        pm[a, c] -= h
        with torch.no_grad():
            fd = -(float(energy(pp, e64)) - float(energy(pm, e64))) / (2 * h)
        say("  F[%d,%d] autograd %.10e  FD %.10e" % (a, c, f64[a, c], fd))
        assert abs(fd - f64[a, c]) <= 1e-5 * fscale + 1e-9


def test_forces_against_oracle_energy_differences(table):
    """F_A = -dE/dR_A: the autograd forces of the HIP path (backward =
    dOmega v, chained through the torch density builder) against central
    differences (h = 1e-4 bohr) of the FP64 oracle's energies E_k + Delta E
    on a 48^3 grid with six atoms, in FP64 (to 1e-6 of max|F|) and FP32 (to
    1e-4 of max|F|)."""
    from oracle import functional as F
    shape, L = (48, 48, 48), 48 * W.BATCH_SPACING
    cell = (L, L, L)
    atoms = W.random_atoms(np.random.default_rng(4848), 6, cell)
    pos = torch.tensor(atoms.pos, dtype=torch.float64, device="cuda")
    forces = {}
    for prec in (64, 32):
        eng = engine(shape, cell, table, prec)
        r = pos.clone().requires_grad_(True)
        n = W.density_torch(shape, cell, atoms.amp, atoms.width, r)
        if prec == 32:
            n = n.float()
        eng(n).backward()
        forces[prec] = -r.grad.cpu().numpy()
    fscale = np.abs(forces[64]).max()
    h = 1e-4

    def e_oracle(p):
        ek, de, _ = F.energy_potential(W.density_on_grid(shape, cell, W.Atoms(atoms.amp, atoms.width, p)), cell, table)
        return ek + de

    for a, c in [(0, 0), (1, 2), (3, 1), (5, 0), (5, 2)]:
        pp, pm = atoms.pos.copy(), atoms.pos.copy()
        pp[a, c] += h
        pm[a, c] -= h
        fd = -(e_oracle(pp) - e_oracle(pm)) / (2 * h)
        say("  F[%d,%d] oracle FD %.10e  gpu64 %.10e  gpu32 %.10e" % (a, c, fd, forces[64][a, c], forces[32][a, c]))
        assert abs(forces[64][a, c] - fd) <= 1e-6 * fscale
        assert abs(forces[32][a, c] - fd) <= 1e-4 * fscale
