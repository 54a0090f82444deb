#!/usr/bin/env python3
"""Throughput of the vdW-DF nonlocal correlation path on one MI355X.

Workload: the batched configuration -- 64 independent Gaussian-atom densities
with cubic grids drawn from {32, 48, 64, 96, 128}^3 (spacing 20/96 bohr,
4..128 atoms each, seeds 4000..4063), N_q = 20.  A step is one call of the
whole path (E_c^nl and v_nl of every density) with the densities already in
HBM; the FP32 batched call is the headline, the FP64 per-density ("plain")
evaluation of the same densities is timed beside it and the relative energy
difference between the two is reported.

Prints one JSON line (rank 0).  `--gpus N` with N > 1 exits: this build runs
on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def pass_bytes(name, shapes, s):
    """Algorithmic bytes one launch of a pass moves over all grids: what it
    must read and write given its inputs and outputs (spectra as N1 N2
    (N3/2+1) complex values; the gradient chain's spectra are FP64, the
    divergence chain's in the working precision)."""
    tot = 0
    for (n1, n2, n3) in shapes:
        N = n1 * n2 * n3
        NH = n1 * n2 * (n3 // 2 + 1)
        c, d = 2 * s, 16
        b = {
            "x_nfwd": N * s + NH * d,
            "y_1f": 2 * NH * d, "y_1i": 2 * NH * c,
            "z_grad": 4 * NH * d, "z_div": 4 * NH * c,
            "y_3i": 6 * NH * d, "y_3f": 6 * NH * c,
            "x_grad": 3 * NH * d + 3 * N * s,
            "x_theta": 4 * N * s + 20 * NH * c,
            "y_20f": 40 * NH * c, "z_main": 40 * NH * c, "y_20i": 40 * NH * c,
            "x_assemble": 20 * NH * c + 5 * N * s + 3 * NH * c,
            "x_final": NH * c + 2 * N * s,
            # finite-difference gradient mode
            "fd_grad": 4 * N * s,
            "x_assemble_fd": 20 * NH * c + 8 * N * s,
            "fd_div": 5 * N * s,
            "reduce": 0,
        }[name]
        tot += b
    return tot


def z_main_flops(shapes):
    """Algorithmic FP32 flops of one launch of the fused axis-1 pass over all
    grids: per half-spectrum k point the contraction (20 x 20 real matrix on
    a complex 20-vector: 1600 flops) and its share of the forward and inverse
    axis-1 FFTs of the 20 spectra (5 N1 log2 N1 flops per complex line)."""
    import math
    tot = 0.0
    for (n1, n2, n3) in shapes:
        tot += n1 * n2 * (n3 // 2 + 1) * (1600.0 + 2 * 20 * 5 * math.log2(n1))
    return tot


# FP32 vector arithmetic of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# (FMA) x 2.4 GHz without packed FP32 (which this build does not use); the
# published 157.3 TFLOP/s counts packed FP32
PEAK_FP32_VALU_TFS = 78.6


def measured_traffic(kernel, lds_budget_z):
    """HBM bytes per evaluation of `kernel` from the committed counter summary
    (profiles/<kernel>_batched64_fp32.md), if it was taken on the kernel
    sources as they are now and at the tile budget of this run; else None."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "%s_batched64_fp32.md" % kernel)
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_0812_0244_amd", "csrc")
    for f in ("common.hpp", "fft_lds.hpp", "fft_fast.hpp", "tile_io.hpp", "kernels.hip"):
        h.update(open(os.path.join(src, f), "rb").read())
    if rec.get("kernel_sources_sha256") != h.hexdigest():
        return None
    hit = rec.get("by_lds_budget_z", {}).get(str(lds_budget_z))
    return None if hit is None else float(hit["hbm_bytes_per_evaluation"])


def cpu_baseline(insts, dens, budget_s):
    """The FP64 oracle on the smallest densities of the batch, until about
    budget_s seconds of host work; grid points per second."""
    from oracle import functional as F
    from oracle import kernel_table as kt
    table = dict(kt.kernel_table())
    table["mc"] = 12
    order = sorted(range(len(insts)), key=lambda i: insts[i].npoints)
    done, pts, t_used = [], 0, 0.0
    F.energy_potential(dens[order[0]], insts[order[0]].cell, table)   # warm the table spline
    for i in order:
        t0 = time.perf_counter()
        F.energy_potential(dens[i], insts[i].cell, table)
        t_used += time.perf_counter() - t0
        pts += insts[i].npoints
        done.append(insts[i].shape[0])
        if t_used > budget_s:
            break
    sizes = {}
    for n in done:
        sizes[n] = sizes.get(n, 0) + 1
    sample = "%d of the 64 densities, smallest first (%s), FP64 NumPy oracle, %.1f s" % (
        len(done), ", ".join("%dx %d^3" % (v, k) for k, v in sorted(sizes.items())), t_used)
    return dict(value=pts / t_used, unit="grid-points/s", cores=1, kind="oracle", sample=sample)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--lds-budgets", type=str, default=None,
                    help="x,y20,yaux,z,zaux LDS budgets in bytes (fixes the tiles; no tuning)")
    ap.add_argument("--fd-mode", type=int, default=3,
                    help="finite-difference half-width of the second leg (0: skip that leg)")
    ap.add_argument("--lattice-leg", type=int, default=1,
                    help="1: also time the batch in triclinic cells (general-cell path); 0: skip")
    ap.add_argument("--xc-leg", type=int, default=1,
                    help="1: also time the batch with the whole functional of Eq. (Exc) "
                         "(semilocal terms added); 0: skip")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of 1 GiB (reference dispatch for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_0812_0244_amd.binding import VdwNl, build_kernel_table

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    insts = W.batch_instances(64)
    t0 = time.time()
    dens = [w.density() for w in insts]
    shapes = [w.shape for w in insts]
    cells = [w.cell for w in insts]
    total = sum(w.npoints for w in insts)
    log("densities built (%.1f s), %d grids, %d points" % (time.time() - t0, len(insts), total))
    t0 = time.time()
    table = build_kernel_table(0)
    log("kernel table built on the GPU (%.1f s)" % (time.time() - t0))

    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read, 1 GiB written
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 1 GiB device to device")

    # ---- FP32 batched (headline): tile tuning (setup), then graph replays
    lib = VdwNl(0)
    lib.set_grids(shapes, cells, 0, 32)
    lib.set_kernel_table(table["qmesh"], table["qc"], table["mc"], table["dk"], table["phi"], table["c_soft"])
    n32 = [torch.from_numpy(d).to("cuda", torch.float32) for d in dens]
    v32 = [torch.empty_like(x) for x in n32]
    nptr, vptr = [x.data_ptr() for x in n32], [x.data_ptr() for x in v32]
    stream = torch.cuda.current_stream().cuda_stream
    t0 = time.time()
    if args.lds_budgets:
        lib.set_tiling([int(x) for x in args.lds_budgets.split(",")])
    elif not args.no_autotune:
        lib.autotune(nptr, vptr, reps=5, stream=stream)
    tiling = lib.get_tiling()
    log("tile budgets %s (%.1f s)" % (tiling, time.time() - t0))
    for _ in range(args.warmup):
        lib.energy_potential_batched(nptr, vptr, stream)
    torch.cuda.synchronize()
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        E32 = lib.energy_potential_batched(nptr, vptr, stream)   # returns after the stream is done
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    med_ms = float(np.median(step_ms))
    log("fp32 batched (graph replay): %.3f ms/step, median %.3f" % (ms_step, med_ms))
    # the same steps again with a HIP event after every pass (passes launched
    # one by one on the same stream): per-pass durations
    lib.set_timing(True)
    for _ in range(args.steps):
        lib.energy_potential_batched(nptr, vptr, stream)
    torch.cuda.synchronize()
    passes = lib.pass_times()
    lib.set_timing(False)
    ev_ms = sum(v[0] for v in passes.values()) / args.steps
    log("fp32 batched (event-timed launches): %.3f ms/step of passes" % ev_ms)
    for k, (ms, calls) in passes.items():
        log("  pass %-10s %8.3f ms/step" % (k, ms / max(calls, 1)))

    # dominant pass and its roofline (bytes and time per step: the pass's
    # launches over every grid of the batch)
    dom = max((k for k in passes if k != "reduce"), key=lambda k: passes[k][0])
    dom_ms = passes[dom][0] / max(passes[dom][1], 1)
    dom_bytes = pass_bytes(dom, shapes, 4)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    path_bytes = sum(pass_bytes(k, shapes, 4) for k in passes)

    # ---- the same batch with the whole functional of Eq. (Exc): revPBE
    # exchange and LDA correlation added in the theta and assembly passes
    xc = None
    if args.xc_leg:
        from paper_0812_0244_amd.binding import FUNCTIONAL_NONLOCAL, FUNCTIONAL_VDW_DF
        lib.set_functional(FUNCTIONAL_VDW_DF)
        vxc = [torch.empty_like(x) for x in n32]             # (v32 keeps v_nl for the comparison below)
        vxptr = [x.data_ptr() for x in vxc]
        for _ in range(args.warmup):
            lib.energy_potential_batched(nptr, vxptr, stream)
        torch.cuda.synchronize()
        xc_ms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            Exc = lib.energy_potential_batched(nptr, vxptr, stream)
            xc_ms.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        xc_step = (time.perf_counter() - t0) * 1e3 / args.steps
        sl = lib.semilocal_energies()
        lib.set_functional(FUNCTIONAL_NONLOCAL)
        del vxc
        log("fp32 batched, whole functional (graph replay): %.3f ms/step, median %.3f"
            % (xc_step, float(np.median(xc_ms))))
        xc = {"functional": "E_x^GGA (revPBE) + E_c^LDA (PW92) + E_c^nl, v_xc",
              "ms_per_step": xc_step, "median_ms_per_step": float(np.median(xc_ms)),
              "value": total / (xc_step * 1e-3), "unit": "grid-points/s",
              "E_sum": float(Exc.sum()), "E_x_sum": float(sl[:, 0].sum()), "E_c_lda_sum": float(sl[:, 1].sum())}

    # ---- the same workload with the finite-difference gradient (the paper's
    # own choice; seven passes instead of fourteen), FP32 batched
    del lib
    fd = None
    if args.fd_mode > 0:
        lib = VdwNl(0)
        lib.set_grids(shapes, cells, args.fd_mode, 32)
        lib.set_kernel_table(table["qmesh"], table["qc"], table["mc"], table["dk"], table["phi"], table["c_soft"])
        vfd = [torch.empty_like(x) for x in n32]
        vfptr = [x.data_ptr() for x in vfd]
        if args.lds_budgets:
            lib.set_tiling([int(x) for x in args.lds_budgets.split(",")])
        elif not args.no_autotune:
            lib.autotune(nptr, vfptr, reps=5, stream=stream)
        fd_tiling = lib.get_tiling()
        for _ in range(args.warmup):
            lib.energy_potential_batched(nptr, vfptr, stream)
        torch.cuda.synchronize()
        fd_ms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            Efd = lib.energy_potential_batched(nptr, vfptr, stream)
            fd_ms.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        fd_step = (time.perf_counter() - t0) * 1e3 / args.steps
        lib.set_timing(True)
        for _ in range(args.steps):
            lib.energy_potential_batched(nptr, vfptr, stream)
        torch.cuda.synchronize()
        fd_passes = lib.pass_times()
        lib.set_timing(False)
        del lib
        log("fp32 batched, finite differences m=%d (graph replay): %.3f ms/step, median %.3f"
            % (args.fd_mode, fd_step, float(np.median(fd_ms))))
        for k, (ms, calls) in fd_passes.items():
            log("  pass %-14s %8.3f ms/step" % (k, ms / max(calls, 1)))
        fd_bytes = sum(pass_bytes(k, shapes, 4) for k in fd_passes)
        fd = {"grad_mode": args.fd_mode, "ms_per_step": fd_step, "median_ms_per_step": float(np.median(fd_ms)),
              "value": total / (fd_step * 1e-3), "unit": "grid-points/s", "lds_budgets": fd_tiling,
              "passes_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in fd_passes.items()},
              "path_algorithmic_bytes_per_step": fd_bytes,
              "path_frac": fd_bytes / (fd_step * 1e-3) / 1e9 / PEAK_HBM_GBS,
              "E_sum": float(Efd.sum())}

    # ---- the same grids (and grid values) in triclinic cells of the same edge
    # lengths: the general-cell path (every k point its own |G| shell)
    tri = None
    if args.lattice_leg:
        t0 = time.time()
        lats = [W.triclinic_lattice((c[0], c[1], c[2]), (85.0, 95.0, 80.0)) for c in cells]   # max |G| 28
        lib = VdwNl(0)
        lib.set_grids(shapes, lats, 0, 32)
        lib.set_kernel_table(table["qmesh"], table["qc"], table["mc"], table["dk"], table["phi"], table["c_soft"])
        vtr = [torch.empty_like(x) for x in n32]
        vtptr = [x.data_ptr() for x in vtr]
        # (the headline's tuned budgets: tuning re-plans, which here rebuilds
        # the large per-k-point kernel tables for every candidate)
        lib.set_tiling(tiling)
        tr_tiling = lib.get_tiling()
        for _ in range(args.warmup):
            lib.energy_potential_batched(nptr, vtptr, stream)
        torch.cuda.synchronize()
        setup_s = time.time() - t0
        tr_ms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            Etr = lib.energy_potential_batched(nptr, vtptr, stream)
            tr_ms.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        tr_step = (time.perf_counter() - t0) * 1e3 / args.steps
        lib.set_timing(True)
        for _ in range(args.steps):
            lib.energy_potential_batched(nptr, vtptr, stream)
        torch.cuda.synchronize()
        tr_passes = lib.pass_times()
        lib.set_timing(False)
        _, ws_bytes = lib.info()
        del lib
        log("fp32 batched, triclinic cells (graph replay): %.3f ms/step, median %.3f (setup %.1f s, workspace %.2f GB)"
            % (tr_step, float(np.median(tr_ms)), setup_s, ws_bytes / 1e9))
        for k, (ms, calls) in tr_passes.items():
            log("  pass %-14s %8.3f ms/step" % (k, ms / max(calls, 1)))
        tri = {"cells": "triclinic: the same edge lengths, angles (85, 95, 80) degrees; the same grid values",
               "ms_per_step": tr_step, "median_ms_per_step": float(np.median(tr_ms)),
               "value": total / (tr_step * 1e-3), "unit": "grid-points/s", "lds_budgets": tr_tiling,
               "workspace_bytes": ws_bytes,
               "passes_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in tr_passes.items()},
               "E_sum": float(Etr.sum())}

    # ---- FP64 plain: one context per density, evaluated one after another
    ctxs, n64, v64 = [], [], []
    for w, d in zip(insts, dens):
        c = VdwNl(0)
        c.set_grid(w.shape, w.cell, 0, 64)
        c.set_kernel_table(table["qmesh"], table["qc"], table["mc"], table["dk"], table["phi"], table["c_soft"])
        ctxs.append(c)
        n64.append(torch.from_numpy(d).to("cuda"))
        v64.append(torch.empty_like(n64[-1]))
    E64 = np.zeros((len(insts), 2))
    for i, c in enumerate(ctxs):
        E64[i] = c.energy_potential(n64[i].data_ptr(), v64[i].data_ptr(), stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.fp64_steps):
        for i, c in enumerate(ctxs):
            E64[i] = c.energy_potential(n64[i].data_ptr(), v64[i].data_ptr(), stream)
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) * 1e3 / args.fp64_steps
    e32 = E32.sum(axis=1)
    e64 = E64.sum(axis=1)
    max_rel = float(np.max(np.abs(e32 - e64) / np.abs(e64)))
    max_dv = max(float((v32[i].double() - v64[i]).abs().max()) for i in range(len(insts)))
    log("fp64 plain: %.3f ms/step; max rel E (fp32 batched vs fp64 plain) %.2e; max|dv| %.2e"
        % (ms64, max_rel, max_dv))
    del ctxs

    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.time()
        cpu = cpu_baseline(insts, dens, args.cpu_seconds)
        log("cpu baseline: %.3e pts/s (%.1f s)" % (cpu["value"], time.time() - t0))

    sizes = {}
    for s in shapes:
        sizes[str(s[0])] = sizes.get(str(s[0]), 0) + 1
    out = {
        "metric": "E_c^nl+v_nl grid-points/s (N_q=20), FP32 batched vs FP64 plain at 1e-6 rel E",
        "value": total / (ms_step * 1e-3),
        "unit": "grid-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "median_ms_per_step": med_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched: 64 Gaussian-atom densities, cubic grids from {32,48,64,96,128}^3 "
                        "(spacing 20/96 bohr, seeds 4000-4063), N_q=20, one call per step",
            "grids_by_edge": sizes,
            "total_points": total,
            "precision": "theta/u FFTs, contraction and divergence chain FP32; grad n chain and "
                         "reductions FP64",
            "launch": "one HIP graph per call (14 passes x FFT length classes), tile LDS budgets "
                      "tuned at setup",
            "lds_budgets": tiling,
        },
        "fp64_plain": {"ms_per_step": ms64, "value": total / (ms64 * 1e-3),
                       "max_rel_E_fp32_batched_vs_fp64_plain": max_rel, "max_abs_dv_Ha": max_dv},
        "passes_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in passes.items()},
        "event_timed_ms_per_step": ev_ms,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": measured_traffic(dom, tiling["z"]) if dom == "z_main" else None,
                     "algorithmic_bytes": dom_bytes,
                     "path_algorithmic_bytes_per_step": path_bytes,
                     "path_frac": path_bytes / (ms_step * 1e-3) / 1e9 / PEAK_HBM_GBS},
        # the same pass against the vector-ALU roofline (its counters show it
        # bound by instruction issue, not bandwidth)
        "roofline_valu": None if dom != "z_main" else {
            "bound": "alu", "kernel": dom, "unit": "TFLOP/s",
            "achieved": z_main_flops(shapes) / (dom_ms * 1e-3) / 1e12, "peak": PEAK_FP32_VALU_TFS,
            "frac": z_main_flops(shapes) / (dom_ms * 1e-3) / 1e12 / PEAK_FP32_VALU_TFS,
            "algorithmic_flops": z_main_flops(shapes)},
        "fd_gradient": fd,
        "triclinic_cells": tri,
        "whole_functional": xc,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
