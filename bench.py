"""Throughput of the MI355X immersed-boundary DNS time step.

One step = the whole hot path (RHS + AB2 predictor, outflow, immersed-boundary
forcing of the grid points and the flag, FFT/tridiagonal pressure projection,
CFL time step, flag sub-steps) over the paper-like workload: 12L x 6L x 6L on
768 x 384 x 384 cells (113M), Re 1000, passive grid of square bars
(M = 0.5L, d = 0.1L, about 3.0e5 solid points) and a 96 x 96 flag 6M
downstream, dt from CFL 0.5, plain FP64.  Inputs are seeded and synthetic
(uniform inflow plus Gaussian noise of amplitude 0.05) and resident in HBM
before the timed region.

Prints one JSON line.  --gpus above 1 is rejected: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Mcell-steps/s and HBM GB/s: plain FP64 vs FP32-mixed / batched, fixed accuracy")
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per cell of each FP64 kernel (compulsory reads + writes;
# half-spectrum complex arrays hold (ny/2+1)/ny of a complex per cell).
def kernel_bytes_per_cell(ny: int) -> dict:
    half = 16.0 * (ny // 2 + 1) / ny          # bytes of half spectrum per cell
    return {
        "predict": 7 * 8 + 6 * 8,            # u v w p H(3) in; H(3) u~(3) out
        "div_ffty": 3 * 8 + half,             # u~(3) in; spectrum out
        "fftz_fwd": 2 * half,
        "tri_x": 2 * half,
        "fftz_inv": 2 * half,
        "iffty": half + 8,                    # spectrum in; phi out
        "project": 5 * 8 + 4 * 8,             # u~(3) phi p in; u v w p out
    }


def max_divergence(u, v, w, h):
    """max |D u| over the cells of fields in the ABI's host layout (measurement only)."""
    d = (u[..., 1:] - u[..., :-1]) + (np.roll(v, -1, axis=1) - v) + (np.roll(w, -1, axis=0) - w)
    return float(np.max(np.abs(d))) / h


def cn_axis_ms(times: dict, steps: int) -> dict:
    """Per-step milliseconds of the Crank-Nicolson factors (z, y, x; three
    components each) from the per-kernel pass."""
    return {k: times[k][0] / steps for k in ("cn_z", "cn_y", "cn_x") if k in times}


def max_edge_strain(X, X0):
    """max |l/l0 - 1| over the flag's a-edges, b-edges and cell diagonals
    (X, X0: (ns, ns, 3) indexed [b, a]); the spring network's inextensibility."""
    out = 0.0
    for sl_p, sl_q in (((slice(None), slice(1, None)), (slice(None), slice(None, -1))),
                       ((slice(1, None), slice(None)), (slice(None, -1), slice(None))),
                       ((slice(1, None), slice(1, None)), (slice(None, -1), slice(None, -1)))):
        ln = np.linalg.norm(X[sl_p] - X[sl_q], axis=-1)
        l0 = np.linalg.norm(X0[sl_p] - X0[sl_q], axis=-1)
        out = max(out, float(np.max(np.abs(ln / l0 - 1.0))))
    return out


def make_workload(name: str):
    import synth
    if name in ("grid_flag_768x384x384_re1000", "default"):
        return synth.grid_flag_768_re1000()
    if name == "flag_64x32x32_re200":
        return synth.flag_64_re200()
    raise SystemExit(f"unknown workload {name}")


def batch_leg(ib, torch, ws_list, precision, steps, warmup, keep=False):
    """Run an ensemble through one batch (autotuned tiles, hipGraph replay)."""
    import synth
    runs = []
    for w in ws_list:
        noise = synth.ic_noise(w)
        runs.append(ib.create(ib.domain_from(w, precision=precision), noise, grid=w.grid, flag=w.flag))
    b = ib.Batch(runs)
    variant = b.autotune()
    b.use_graph(True)
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for r in runs:
        ib.sync(r.ctx)
    cells = sum(w.cells for w in ws_list)
    out = {"runs": len(ws_list), "cells": cells, "steps": steps,
           "value": round(cells * steps / wall / 1e6, 1), "ms_per_step": round(wall * 1e3 / steps, 4),
           "precision": "mixed" if precision else "fp64", "graph": True, "tile_variant": variant}
    if keep:
        return out, b, runs
    b.close()
    for r in runs:
        r.close()
    return out, None, None


def cpu_baseline(w, budget_s: float = 20.0) -> dict:
    """Time the oracle (as it stands) on a bounded sample of the workload.

    The oracle's fast form (oracle/fast.py: the fluid stages as plain C loops,
    OpenMP over the host's threads, the flag's spring network in numpy) steps
    the full workload -- the same mesh, bodies and seeded inputs -- for about
    budget_s after one warm-up step; the rate is cells / (mean time per step).
    """
    import synth
    from oracle import fast, geometry
    noise = synth.ic_noise(w)
    bars = geometry.grid_points_of(w) if w.grid is not None else None
    flag = None
    if w.flag is not None:
        f = w.flag
        flag = dict(X0=geometry.flag_lattice(f), length=f.length, rho=f.mass_ratio, beta=f.bending,
                    ks=f.stretch, le_bc=f.le_bc)
    C = fast.FastSolver(w, noise, bars, flag)
    del noise
    C.step(1)   # warm-up: first touch of the work arrays
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s or n < 2:
        C.step(1)
        n += 1
    t_step = (time.perf_counter() - t0) / n
    threads = fast.threads()
    return {"value": w.cells / t_step / 1e6, "unit": "Mcell-steps/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle (fluid stages as plain C loops over {threads} OpenMP threads, "
                       f"flag model in numpy): {n} steps of the full {w.name} workload "
                       f"({w.cells} cells, bars and flag) after one warm-up step, {t_step:.2f} s/step")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="grid_flag_768x384x384_re1000")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-eulerian", action="store_true")
    ap.add_argument("--no-cn", action="store_true")
    ap.add_argument("--no-mls", action="store_true")
    ap.add_argument("--no-paper-scheme", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain device copy of 1 GiB (calibrates HBM counters)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    import paper_2103_08246_amd as ib

    w = make_workload(args.workload)
    print(f"# workload {w.name}: {w.nx}x{w.ny}x{w.nz} = {w.cells} cells", file=sys.stderr, flush=True)
    noise = synth.ic_noise(w)

    def measure(precision, breakdown, eulerian=False, diffusion=0, mls=False):
        """Timed region: args.steps steps with HIP events around the predictor
        only (two per step).  breakdown: then as many steps again with events
        around every kernel, for the per-kernel table (not the value).
        eulerian: the grid forced at its nodes instead of as points; mls: the
        flag coupled at its tiling markers by MLS instead of at its nodes."""
        run = ib.create(ib.domain_from(w, precision=precision, diffusion=diffusion), noise,
                        grid=None if eulerian else w.grid, flag=w.flag,
                        grid_forcing=w.grid if eulerian else None, flag_mls=mls and w.flag is not None)
        # the flag's reference lattice as the library built it (rest lengths of the strain)
        run.X_ref = run.flag()[0] if w.flag is not None else None
        run.variant = ib.autotune(run.ctx)   # predictor tile shape, picked by timing
        run.step(args.warmup)
        ib.sync(run.ctx)
        stream = torch.cuda.current_stream()
        ib.enable_timing(run.ctx, ib.TIMING_PREDICT)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        run.step(args.steps)
        ev1.record(stream)
        ib.sync(run.ctx)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ib.enable_timing(run.ctx, ib.TIMING_OFF)
        times = {"timed_region": ib.kernel_times(run.ctx)}
        if breakdown:
            # the per-kernel pass also samples the virtual probes of Sec. III
            # (their kernel appears in the table; the timed region has none)
            pr = synth.probe_layout(w, 64)
            run.set_probes(pr["n_x"], pr["x0"], pr["dx"], pr["yc"], pr["zc"], pr["dyz"],
                           pr["n_lags"])
            run.probe_layout = pr
            ib.enable_timing(run.ctx, ib.TIMING_ALL)
            run.step(args.steps)
            ib.sync(run.ctx)
            ib.enable_timing(run.ctx, ib.TIMING_OFF)
            times["all"] = ib.kernel_times(run.ctx)
        return run, wall, ev0.elapsed_time(ev1), times

    run, wall, gpu_ms, times = measure(ib.FP64, True)
    print(f"# fp64: {wall * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    sc = ib.get_scalars(run.ctx)
    ms_per_step = wall * 1e3 / args.steps
    value = w.cells * args.steps / wall / 1e6

    # roofline of the dominant fluid kernel (largest share in the per-kernel
    # pass), its launch time from the events of the timed region
    bpc = kernel_bytes_per_cell(w.ny)
    dom = max((k for k in times["all"] if k in bpc), key=lambda k: times["all"][k][0])
    if dom not in times["timed_region"]:
        raise SystemExit(f"the timed region recorded no events around {dom}")
    avg_ms = times["timed_region"][dom][0] / times["timed_region"][dom][1]
    achieved = bpc[dom] * w.cells / (avg_ms * 1e-3) / 1e9
    # HBM bytes per launch from the committed counter runs, while they still
    # describe this kernel: same source file, and a record for the tile shape
    # the autotuner chose (the counter runs measure every shape it tries)
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"traffic_{dom}.json")
    if os.path.exists(tf):
        rec = json.load(open(tf))
        src = os.path.join(ROOT, "paper_2103_08246_amd", "csrc", f"k_{dom}.hip")
        same_src = os.path.exists(src) and hashlib.sha256(open(src, "rb").read()).hexdigest() == \
            rec.get("source_sha256")
        if same_src and rec.get("variant") == run.variant:
            traffic = rec.get("hbm_bytes_per_launch")
        elif same_src and str(run.variant) in rec.get("per_variant", {}):
            traffic = rec["per_variant"][str(run.variant)]["hbm_bytes_per_launch"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "algorithmic_bytes_per_launch": int(bpc[dom] * w.cells),
                "avg_launch_ms": round(avg_ms, 4)}
    breakdown = {k: round(v[0] / max(v[1], 1), 4) for k, v in sorted(times["all"].items(),
                 key=lambda kv: -kv[1][0])}
    step_bytes = sum(bpc.values()) * w.cells
    out = {"metric": METRIC, "value": round(value, 1), "unit": "Mcell-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": w.name, "cells": w.cells, "grid": [w.nx, w.ny, w.nz],
                      "re": w.re, "cfl": w.cfl, "solid_points": int(ib.get_grid_points(run.ctx)[1].size),
                      "flag_nodes": 0 if w.flag is None else w.flag.ns ** 2,
                      "precision": "fp64", "flag_substeps": sc["nsub"], "dt": sc["dt"],
                      "predict_variant": run.variant},
           "roofline": roofline,
           "step_hbm_gbs": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
           "gpu_event_ms_per_step": round(gpu_ms / args.steps, 4),
           "kernel_avg_ms": breakdown,
           "kernel_avg_ms_note": "separate pass of the same length with events around every kernel"}
    if w.flag is not None:
        out["flag_max_edge_strain"] = max_edge_strain(run.flag()[0], run.X_ref)
        out["flag_max_edge_strain_after_steps"] = args.warmup + 2 * args.steps
    rec = run.probe_stats()
    out["probes"] = {"probes": int(rec.shape[0]), "stations": run.probe_layout["n_x"],
                     "lags": run.probe_layout["n_lags"], "samples": int(rec[0, 0]),
                     "kernel_avg_ms": breakdown.get("probes"),
                     "note": "Sec. III probe stencil (M/2 streamwise, 2M/3 transverse), sampled "
                             "in the per-kernel pass only"}
    if not args.no_mixed:
        # the same workload with the FP32 RHS/predictor and IB transfer
        # (with the per-kernel pass too, so that both runs stand at the same step)
        run_m, wall_m, _, times_m = measure(ib.MIXED, True)
        print(f"# mixed: {wall_m * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
        a = run.fields()
        b = run_m.fields()
        num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(b[:3], a[:3]))
        den = sum(float(np.sum(y ** 2)) for y in a[:3])
        dmax = max_divergence(b[0], b[1], b[2], w.h)
        out["mixed"] = {"value": round(w.cells * args.steps / wall_m / 1e6, 1),
                        "ms_per_step": round(wall_m * 1e3 / args.steps, 4),
                        "speedup_vs_fp64": round(wall / wall_m, 3),
                        "vel_rel_l2_vs_fp64": (num / den) ** 0.5, "max_abs_div": dmax,
                        "after_steps": args.warmup + 2 * args.steps,
                        "predict_variant": run_m.variant,
                        "kernel_avg_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in
                                          sorted(times_m["all"].items(), key=lambda kv: -kv[1][0])}}
        run_m.close()
    if w.grid is not None and not args.no_eulerian:
        # the paper's own treatment of the fixed grid (Sec. II.B (i)): Eulerian
        # forcing at the velocity nodes instead of the delta points
        run_e, wall_e, _, times_e = measure(ib.FP64, True, eulerian=True)
        n_forced = sum(run_e.grid_forcing(c)[0].size for c in range(3))
        out["grid_eulerian"] = {"value": round(w.cells * args.steps / wall_e / 1e6, 1),
                                "ms_per_step": round(wall_e * 1e3 / args.steps, 4),
                                "forced_nodes": int(n_forced),
                                "kernel_avg_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in
                                                  sorted(times_e["all"].items(), key=lambda kv: -kv[1][0])
                                                  if k in ("grid_force", "flag_interp", "flag_spread",
                                                           "flag_bbox")},
                                "note": "FP64, grid forced at its velocity nodes, flag by delta markers"}
        print(f"# eulerian grid: {wall_e * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
        run_e.close()
    flag_keys = ("flag_markers", "flag_interp", "flag_node_load", "flag_bbox", "flag_spread", "flag_step")
    if w.flag is not None and not args.no_mls:
        # the paper's flag coupling (Sec. II.B (ii)): MLS transfer at the markers of
        # the adaptive tiling instead of the delta at the nodes
        run_l, wall_l, _, times_l = measure(ib.FP64, True, mls=True)
        a = run.fields()
        b = run_l.fields()
        out["flag_mls"] = {"value": round(w.cells * args.steps / wall_l / 1e6, 1),
                           "ms_per_step": round(wall_l * 1e3 / args.steps, 4),
                           "markers": int(run_l.n_markers), "nodes": int(w.flag.ns ** 2),
                           "kernel_avg_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in
                                             sorted(times_l["all"].items(), key=lambda kv: -kv[1][0])
                                             if k in flag_keys},
                           "node_coupling_kernel_avg_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in
                                                           sorted(times["all"].items(), key=lambda kv: -kv[1][0])
                                                           if k in flag_keys},
                           "vel_rel_l2_vs_nodes": (sum(float(np.sum((x - y) ** 2)) for x, y in zip(b[:3], a[:3]))
                                                   / sum(float(np.sum(y ** 2)) for y in a[:3])) ** 0.5,
                           "note": "FP64; grid by delta points, flag by MLS at its tiling markers"}
        print(f"# flag mls: {wall_l * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
        run_l.close()
    if w.flag is not None and w.grid is not None and not args.no_paper_scheme:
        # all three of the paper's choices together (Sec. II.B): Eulerian grid
        # forcing, MLS flag markers, Crank-Nicolson with approximate factorisation
        run_p, wall_p, _, times_p = measure(ib.FP64, False, eulerian=True, diffusion=ib.DIFFUSION_CN, mls=True)
        out["paper_scheme"] = {"value": round(w.cells * args.steps / wall_p / 1e6, 1),
                               "ms_per_step": round(wall_p * 1e3 / args.steps, 4),
                               "note": "FP64; Eulerian grid forcing + MLS flag markers + Crank-Nicolson "
                                       "with approximate factorisation"}
        print(f"# paper scheme: {wall_p * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
        run_p.close()
        if not args.no_mixed:
            run_pm, wall_pm, _, _ = measure(ib.MIXED, False, eulerian=True, diffusion=ib.DIFFUSION_CN, mls=True)
            out["paper_scheme"]["mixed"] = {"value": round(w.cells * args.steps / wall_pm / 1e6, 1),
                                            "ms_per_step": round(wall_pm * 1e3 / args.steps, 4),
                                            "speedup_vs_fp64": round(wall_p / wall_pm, 3)}
            print(f"# paper scheme mixed: {wall_pm * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
            run_pm.close()
    if not args.no_cn:
        # the paper's diffusion scheme (Sec. II.B): Crank-Nicolson with approximate
        # factorisation, same workload and CFL step
        run_c, wall_c, _, times_c = measure(ib.FP64, True, diffusion=ib.DIFFUSION_CN)
        a = run.fields()
        b = run_c.fields()
        per_axis = cn_axis_ms(times_c["all"], args.steps)
        sweep_ms = sum(per_axis.values())
        # algorithmic bytes of the factors per evolved node (u: (nx-1) ny nz,
        # v, w: nx ny nz): z and y one read and one write each, x the read of
        # the right-hand side and of u^n and the write of u~
        sweep_bytes = (16 + 16 + 24) * (3 * w.nx - 1) * w.ny * w.nz
        out["crank_nicolson"] = {
            "value": round(w.cells * args.steps / wall_c / 1e6, 1),
            "ms_per_step": round(wall_c * 1e3 / args.steps, 4),
            "cn_sweeps_ms": round(sweep_ms, 4),
            "cn_factor_ms": {k: round(v, 4) for k, v in per_axis.items()},
            "cn_sweeps_algorithmic_gbs": round(sweep_bytes / (sweep_ms * 1e-3) / 1e9, 1),
            "vel_rel_l2_vs_explicit": (sum(float(np.sum((x - y) ** 2)) for x, y in zip(b[:3], a[:3]))
                                       / sum(float(np.sum(y ** 2)) for y in a[:3])) ** 0.5,
            "note": "FP64; z, y, x factored solves per component, each one read and one write of the field "
                    "(z, y: the periodic factors' inverse as a short convolution, thread per line; x: a "
                    "wavefront per line, chunked elimination and cyclic reduction)"}
        print(f"# crank-nicolson: {wall_c * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
        if not args.no_mixed:
            # mixed form: FP32 right-hand side and increments between the sweeps
            run_cm, wall_cm, _, times_cm = measure(ib.MIXED, True, diffusion=ib.DIFFUSION_CN)
            bm = run_cm.fields()
            per_axis_m = cn_axis_ms(times_cm["all"], args.steps)
            sw_ms = sum(per_axis_m.values())
            out["crank_nicolson"]["mixed"] = {
                "value": round(w.cells * args.steps / wall_cm / 1e6, 1),
                "ms_per_step": round(wall_cm * 1e3 / args.steps, 4),
                "speedup_vs_fp64_cn": round(wall_c / wall_cm, 3),
                "cn_sweeps_ms": round(sw_ms, 4),
                "cn_factor_ms": {k: round(v, 4) for k, v in per_axis_m.items()},
                "vel_rel_l2_vs_fp64_cn": (sum(float(np.sum((x - y) ** 2)) for x, y in zip(bm[:3], b[:3]))
                                          / sum(float(np.sum(y ** 2)) for y in b[:3])) ** 0.5}
            print(f"# crank-nicolson mixed: {wall_cm * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
            run_cm.close()
        run_c.close()
    del noise
    run.close()
    if args.copy_calib:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_batch:
        import synth as _s
        ens24 = _s.ensemble_24()
        res, _, _ = batch_leg(ib, torch, ens24, ib.FP64, args.batch_steps, 3)
        res["workload"] = "ensemble 8x96x48x48 + 8x128x64x64 + 8x192x96x96, bars + 24x24 flags, Re 500"
        print(f"# batch24 fp64: {res['ms_per_step']} ms/step", file=sys.stderr, flush=True)
        out["batched"] = {"ensemble_24": res}
        ens6 = _s.ensemble_6_384()
        r64, b64, runs64 = batch_leg(ib, torch, ens6, ib.FP64, args.batch_steps, 3, keep=True)
        rmx, bmx, runsmx = batch_leg(ib, torch, ens6, ib.MIXED, args.batch_steps, 3, keep=True)
        errs, divs = [], []
        for ra, rb, w6 in zip(runs64, runsmx, ens6):
            a = ra.fields()
            c = rb.fields()
            num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(c[:3], a[:3]))
            den = sum(float(np.sum(y ** 2)) for y in a[:3])
            errs.append((num / den) ** 0.5)
            divs.append(max_divergence(c[0], c[1], c[2], w6.h))
        for bb, rr in ((b64, runs64), (bmx, runsmx)):
            bb.close()
            for r in rr:
                r.close()
        rmx["speedup_vs_fp64_batch"] = round(r64["ms_per_step"] / rmx["ms_per_step"], 3)
        rmx["vel_rel_l2_vs_fp64_max"] = max(errs)
        rmx["max_abs_div"] = max(divs)
        rmx["after_steps"] = args.batch_steps + 3
        for r in (r64, rmx):
            r["workload"] = "6 x 384x192x192, bars + 64x64 flags at 3..10 M, Re 1000"
        print(f"# batch6: fp64 {r64['ms_per_step']} / mixed {rmx['ms_per_step']} ms/step",
              file=sys.stderr, flush=True)
        out["batched"]["ensemble_6_384_fp64"] = r64
        out["batched"]["ensemble_6_384_mixed"] = rmx
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
