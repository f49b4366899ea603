"""Throughput of the Yin-Yang AC direction-splitting time step on one MI355X.

One step = the whole hot path: extrapolation, K Schwarz iterations (overlap
interpolation + walls; residual and three direction-split line sweeps for T,
u1 (r, theta, phi), u2 (r, theta, phi); FP64 pressure updates; norms) and
the post-step interpolation, on a synthetic convecting shell (conductive
temperature + seeded noise, hydrostatic pressure, u = 0) with every input
resident in HBM before the timed region.

Prints one JSON line (metric, value in Mcell-steps/s, per-kernel timing
from HIP events, the roofline of the dominant kernel, and the oracle's
CPU baseline on a bounded sample).
"""
import argparse
import math
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-steps/s, FP64 vs FP32-mixed at stated error; line-solve HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0

# distinct arrays (read + written) per launch of each kernel class, in
# compute-precision words (R) and FP64 words (D), per cell; classes merge
# the launches of several fields, so the figure is their mean.
# sweep: x in, y out (+ the advecting-velocity components its coefficients
# use); last sweep: x in, psi^k read and written.
_ADV = {  # (location, direction) -> extra u2* components read by the sweep
    ("c", 0): 1, ("c", 1): 1, ("c", 2): 1,
    ("r", 0): 1, ("r", 1): 1, ("r", 2): 1,
    ("t", 0): 1, ("t", 1): 2, ("t", 2): 1,
    ("p", 0): 1, ("p", 1): 1, ("p", 2): 3,
}
_ORDER = {"c": (0, 1, 2), "r": (1, 2, 0), "t": (2, 0, 1), "p": (0, 1, 2)}


def class_words():
    """{class: (R words per cell, D words per cell)} averaged over launches"""
    fields = ["c", "r", "t", "p", "r", "t", "p"]          # T, u1, u2
    sw = {0: [], 1: [], 2: []}
    swl = {0: [], 1: [], 2: []}
    for loc in fields:
        o = _ORDER[loc]
        for q in range(2):
            sw[o[q]].append(2 + _ADV[(loc, o[q])])
        swl[o[2]].append(3 + _ADV[(loc, o[2])])
    W = {}
    for d, name in enumerate("rtp"):
        W["sweep_" + name] = (float(np.mean(sw[d])), 0.0)
        W["sweep_" + name + "_last"] = (float(np.mean(swl[d])), 0.0)
    # the last phi sweep is timed apart for u_phi (sweep_p_last) and T
    W["sweep_p_last"] = (3.0 + _ADV[("p", 2)], 0.0)
    W["sweep_p_last_T"] = (3.0 + _ADV[("c", 2)], 0.0)
    # residuals: own levels n, k, *, u2* (3), write 1 (+ sources)
    W["residual_T"] = (7.0, 0.0)                          # Tn Tk T* w3 out
    W["residual_ur"] = (0.5 * (11 + 8), 0.5 * (1 + 3))    # s=1 / s=2 distinct arrays
    W["residual_ut"] = (0.5 * (12 + 9), 0.5 * (1 + 3))
    W["residual_up"] = (0.5 * (12 + 10), 0.5 * (1 + 3))
    W["pressure_1"] = (6.0, 3.0)
    W["pressure_2"] = (6.0, 5.0)
    W["step_start"] = (28.0, 4.0)                        # 14 read, 14 written; p1, p2 copied
    W["extrap"] = (21.0, 0.0)
    return W


KERNEL_SRC = os.path.join(ROOT, "paper_1905_02300_amd", "csrc", "yy_kernels.hip")
# residual class -> (unknown's tuning key, location index in the kernel name)
RES_CLASSES = {"residual_T": ("T", 0), "residual_ur": ("u_r", 1), "residual_ut": ("u_t", 2),
               "residual_up": ("u_p", 3)}


def kernel_source_sha():
    import hashlib
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def stored_traffic(cls, prec, tiles):
    """HBM bytes per launch of a kernel class from profiles/, or None when
    the record is missing or stale (taken with other kernel sources or
    another tile than this run's)"""
    if cls not in RES_CLASSES or not tiles:
        return None
    tile = json.loads(tiles).get("res." + RES_CLASSES[cls][0])
    tfile = os.path.join(ROOT, "profiles", "traffic_%s_%s_%s.json" % (cls, prec, tile))
    if not os.path.exists(tfile):
        return None
    with open(tfile) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_source_sha() or rec.get("tile") != tile:
        return None
    return rec.get("bytes_per_launch")


def copy_ceiling(gib=2, reps=20):
    """HBM rate of the library's plain streaming copy (every word read once
    and written once) over 2 GiB buffers: the practical ceiling of the
    step's streaming kernels, read + write bytes per second"""
    import torch
    from paper_1905_02300_amd import yy
    n = gib * (1 << 30) // 8
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        yy.stream_copy(b, a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        yy.stream_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(a, b))
    del a, b
    torch.cuda.empty_cache()
    return {"bytes": 2 * n * 8, "ms": ms, "gbs": 2 * n * 8 / ms / 1e6, "copy_exact": ok}


def traffic_summary(args):
    """Per-launch HBM bytes of the residual kernels of the timed step, from
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the
    counter reads for the step-start kernel, which streams 16 padded arrays
    in and 16 out with no reuse."""
    import re
    import sqlite3
    nr, nt, np_ = (int(v) for v in args.grid.split(","))
    wb = 8 if args.prec == "fp64" else 4
    pitch = -(-(np_ + 1 + 128 // wb) // (128 // wb)) * (128 // wb)
    # FP64: every array in compute precision; the step start reads 14 + 2
    # (p1, p2 in FP64) arrays and writes as many
    arr = 2 * (nr + 2) * (nt + 2) * pitch
    stream = 14 * arr * wb + 2 * arr * 8

    def rows(db, counter):
        cur = sqlite3.connect(db).cursor()
        return list(cur.execute("select dispatch_id, name, counter_value from pmc_events "
                                "where counter_name = ? order by dispatch_id", (counter,)))
    fetch, write = rows(args.traffic[0], "FETCH_SIZE"), rows(args.traffic[1], "WRITE_SIZE")
    rtype = "double" if args.prec == "fp64" else "float"

    def last(rs, pat, n):
        sel = [r for r in rs if re.search(pat, r[1])]
        return sel[-n:]
    cal_f = last(fetch, r"KExtrapCopy<%s>" % rtype, 1)
    cal_w = last(write, r"KExtrapCopy<%s>" % rtype, 1)
    ff = stream / (cal_f[0][2] * 1024.0)
    fw = stream / (cal_w[0][2] * 1024.0)
    W = class_words()
    tiles = json.loads(args.tiles) if args.tiles else {}
    sha = kernel_source_sha()
    cells = 2 * nr * nt * np_
    for cls, (key, L) in RES_CLASSES.items():
        n = 3 if L == 0 else 6
        pat = r"KResidual(Lds)?<%s, %d[,>]" % (rtype, L)
        f, w = last(fetch, pat, n), last(write, pat, n)
        names = sorted({r[1].split("(")[0] for r in f})
        fb = sum(r[2] for r in f) / len(f) * 1024.0 * ff
        wbytes = sum(r[2] for r in w) / len(w) * 1024.0 * fw
        r, dw = W[cls]
        alg = cells * (r * wb + dw * 8)
        rec = {"class": cls, "kernel": names, "tile": tiles.get("res." + key),
               "workload": f"{args.prec.upper()} 2x{nr}x{nt}x{np_}, K=3 (the timed step's launches averaged)",
               "bytes_per_launch": fb + wbytes, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wbytes,
               "alg_bytes_per_launch": alg, "ratio_to_algorithmic": (fb + wbytes) / alg, "dispatches": len(f),
               "fetch_factor": ff, "write_factor": fw,
               "calibration": "the step-start kernel reads 16 padded arrays (levels n and n-1 of T, u1, u2; "
                              "p1, p2) and writes 16, %d elements each" % arr,
               "commands": [
                   "rocprofv3 --pmc FETCH_SIZE --kernel-trace -d <fetch> -o fetch -- python3 bench.py "
                   "--steps 1 --warmup 0 --no-cpu --no-line --set-tiles '<tiles>'",
                   "rocprofv3 --pmc WRITE_SIZE --kernel-trace -d <write> -o write -- python3 bench.py "
                   "--steps 1 --warmup 0 --no-cpu --no-line --set-tiles '<tiles>'",
                   "python3 bench.py --traffic <fetch>/fetch_results.db <write>/write_results.db --tiles '<tiles>'"],
               "source_sha256": sha,
               "note": "counters in KiB per dispatch, scaled by the factors; FETCH_SIZE counts L2 misses to "
                       "the fabric, some of which the Infinity Cache serves; stale (ignored by bench.py) once "
                       "the kernel source or the tile changes"}
        out = os.path.join(ROOT, "profiles", "traffic_%s_%s_%s.json" % (cls, args.prec, rec["tile"]))
        with open(out, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps({cls: {"ratio": rec["ratio_to_algorithmic"], "kernel": names, "tile": rec["tile"]}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--grid", default="128,384,1152")
    ap.add_argument("--schwarz", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the line-solver tile autotuner")
    ap.add_argument("--no-line", action="store_true", help="skip the line-solve benchmark")
    ap.add_argument("--line-only", action="store_true", help="run only the line-solve benchmark")
    ap.add_argument("--line-tiles", default="",
                    help='with --line-only: time only these tiles, JSON {"fp64": {"r": tile, "t": tile, '
                         '"p": tile}, "fp32": {...}} (for profiling the chosen kernels alone)')
    ap.add_argument("--cpu-grid", default="40,120,360")
    ap.add_argument("--ensemble-modes", default="sequential_eager,graph_streams,graph_batched",
                    help="ensemble modes to time (comma list)")
    ap.add_argument("--ensemble", type=int, default=0,
                    help="batched ensemble of N shells (uneven sizes, seed 5), FP32-mixed, graph-captured")
    ap.add_argument("--mixed-error", type=int, default=0,
                    help="run FP64 and FP32-mixed side by side for N steps and report their difference")
    ap.add_argument("--paper-mms", action="store_true",
                    help="time and space convergence on the paper's manufactured solution with its wall data")
    ap.add_argument("--mms-taus", default="0.01,0.005,0.0025", help="time steps of the --paper-mms time study")
    ap.add_argument("--mms-delta", type=float, default=0.0,
                    help="overlap of the --paper-mms grids (radians; 0: one cell)")
    ap.add_argument("--mms-tf", type=float, default=1.0, help="final time of the --paper-mms time study")
    ap.add_argument("--mms-chi", type=float, default=4.0,
                    help="artificial-compressibility parameter chi of the --paper-mms runs")
    ap.add_argument("--mms-tol", type=float, default=1e-6,
                    help="Schwarz stop tolerance of the --paper-mms time study (the paper's 1e-6)")
    ap.add_argument("--mms-kmax", type=int, default=64, help="Schwarz iteration cap of the --paper-mms runs")
    ap.add_argument("--mms-mass-fix", action="store_true",
                    help="apply the mass-flux correction (Algorithm step 4) in the --paper-mms runs")
    ap.add_argument("--mms-ring", type=int, default=0,
                    help="rings of pressure cells exchanged between the patches (Algorithm step 7) "
                         "in the --paper-mms runs; 0: off")
    ap.add_argument("--mms-no-space", action="store_true", help="skip the --paper-mms space study")
    ap.add_argument("--parity-oracle", type=int, default=0,
                    help="run the first N steps of the workload (--grid, --prec fp64, autotuned tiles) on "
                         "the GPU and on the oracle and report their difference per field")
    ap.add_argument("--out", default="", help="also write the --parity-oracle record to this file")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="turn the rocprofv3 databases of two PMC runs of the default workload "
                         "(FETCH_SIZE, then WRITE_SIZE; --steps 1 --warmup 0 --no-cpu --no-line "
                         "--set-tiles) into profiles/traffic_<class>_<prec>_<tile>.json for the "
                         "residual classes")
    ap.add_argument("--tiles", default="", help="with --traffic: the tiles JSON of the profiled run")
    ap.add_argument("--set-tiles", default="", help="use these tiles (JSON) instead of the autotuner's")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.traffic:
        traffic_summary(args)
        return
    if args.mixed_error:
        mixed_error(args)
        return
    if args.paper_mms:
        paper_mms(args)
        return
    if args.parity_oracle:
        parity_oracle(args)
        return
    if args.ensemble:
        ensemble(args)
        return
    if args.line_only:
        fixed = json.loads(args.line_tiles) if args.line_tiles else None
        print(json.dumps({"metric": "line-solve HBM GB/s", "line_solve": line_solve_bench(fixed=fixed)}),
              flush=True)
        return

    import torch
    from paper_1905_02300_amd import inputs as I
    from paper_1905_02300_amd import yy

    assert torch.cuda.is_available(), "bench.py needs an MI355X"
    nr, nt, np_ = (int(x) for x in args.grid.split(","))
    pr, ra, dt, K = 1.0, 1e5, 2e-4, args.schwarz
    prec = yy.YY_FP64 if args.prec == "fp64" else yy.YY_FP32_MIXED
    grid = I.Grid(nr, nt, np_)
    sh = yy.Shell(nr, nt, np_, prec=prec)
    sh.set_params(pr=pr, ra=ra, dt=dt, chi=1.0, t_inner=1.0, t_outer=0.0)
    st = I.convection_state(grid, pr, ra, seed=3)
    for f in range(9):
        sh.set_field(f, 0, st[f])
        if f not in (I.P1, I.P2):
            sh.set_field(f, 1, st[f])
    del st
    stream = torch.cuda.current_stream()
    if args.set_tiles:
        sh.set_tuning(args.set_tiles)
        tiles = sh.tuning_json()
    else:
        tiles = sh.autotune() if not args.no_tune else None
    for _ in range(args.warmup):
        sh.step(K)
    torch.cuda.synchronize()
    sh.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sh.step(K)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = sh.profile_read(stream)
    sh.profile(False)
    norms = sh.norms()
    cells = grid.cells
    value = cells * args.steps / el / 1e6

    wbytes = 8 if prec == yy.YY_FP64 else 4
    W = class_words()
    kernels = {}
    for name, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        entry = {"ms_total": ms, "launches": cnt, "ms_avg": ms / cnt}
        if name in W:
            r, d = W[name]
            bytes_per = cells * (r * wbytes + d * 8)
            entry["alg_bytes"] = bytes_per
            entry["gbs"] = bytes_per / (ms / cnt * 1e-3) / 1e9
        kernels[name] = entry
    dom = max((k for k in kernels if "gbs" in kernels[k]), key=lambda k: kernels[k]["ms_total"])
    dk = kernels[dom]
    roofline = {"kernel": dom, "bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": None,
                "alg_bytes_per_launch": dk["alg_bytes"], "ms_avg": dk["ms_avg"]}
    roofline["traffic"] = stored_traffic(dom, args.prec, tiles)

    del sh
    torch.cuda.empty_cache()
    copy = copy_ceiling()
    roofline["copy_ceiling_gbs"] = copy["gbs"]
    roofline["frac_of_copy_ceiling"] = dk["gbs"] / copy["gbs"]
    line = None if args.no_line else line_solve_bench()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.cpu_grid, pr, ra, dt, K)
        if line is not None:
            line["cpu_baseline"] = line_solve_cpu()

    out = {
        "metric": METRIC, "value": value, "unit": "Mcell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == yy.YY_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"yinyang_ac_step_2x{nr}x{nt}x{np_}_{args.prec}_K{K}",
                   "cells": cells, "grid_per_patch": [nr, nt, np_], "schwarz_iterations": K,
                   "Pr": pr, "Ra": ra, "dt": dt, "parallelism": "single-gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hbm_copy": copy,
        "line_solve": line,
        "tiles": tiles,
        "kernels": kernels,
        "last_step_norms_k_last": {"div_u2": float(norms[-1, :, 9].max()),
                                   "dT": float(norms[-1, :, 0].max())},
    }
    print(json.dumps(out), flush=True)


def _paper_run(nr, nt, np_, tau, tf, delta, chi, tol=1e-6, kmax=64, keep=False, mass_fix=False, nring=0):
    """The manufactured solution of the paper's numerical tests (eq. Exact:
    R1=1, R2=2, Ra=Pr=1, the given chi, FP64, additive Schwarz) from its exact
    levels at t=0 and -tau, with its time-dependent wall data and forcing,
    Schwarz iterations until every increment norm < tol (the paper's stop
    test with its 1e-6); returns the l2 and max errors of u2, p2, T at tf."""
    import torch
    from paper_1905_02300_amd import inputs as I
    from paper_1905_02300_amd import yy
    pr, ra, kind = 1.0, 1.0, "paper"
    grid = I.Grid(nr, nt, np_, 1.0, 2.0, delta)
    sh = yy.Shell(nr, nt, np_, 1.0, 2.0, delta)
    sh.set_params(pr=pr, ra=ra, dt=tau, chi=chi, t_inner=0.0, t_outer=0.0)
    sh.set_mass_fix(1 if mass_fix else 0)
    sh.set_pressure_exchange(nring)
    dev = sh.ws.device
    wf = (I.T, I.U1R, I.U1T, I.U1P)
    walls = {f: torch.as_tensor(I.wall_parts(grid, f, kind), device=dev) for f in wf}
    parts = {f: [torch.as_tensor(x, device=dev) for x in I.forcing_parts(grid, f, pr, ra, kind=kind)]
             for f in wf}
    for lev, t in ((0, 0.0), (1, -tau)):
        st = I.mms_state(grid, t, kind=kind)
        for f in range(9):
            if lev == 1 and f in (I.P1, I.P2):
                continue
            sh.set_field(f, lev, st[f])
        a = I.time_factor(kind, t)[0]
        for f in wf:
            for side in (0, 1):
                sh.set_wall(f, lev, side, a * walls[f][side])
    nsteps = int(round(tf / tau))
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(nsteps):
        a, da = I.time_factor(kind, (s + 0.5) * tau)
        for f in wf:
            A, B, C = parts[f]
            sh.set_forcing(f, a * A + da * B + (a * a) * C)
        a1 = I.time_factor(kind, (s + 1) * tau)[0]
        for f in wf:
            for side in (0, 1):
                sh.set_wall(f, 2, side, a1 * walls[f][side])
        iters.append(sh.step_tol(kmax, tol))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    r, th, _ = grid.axes(I.T)
    vol = (r[None, :, None, None] ** 2 * np.sin(th)[None, None, :, None] * grid.dr * grid.dth * grid.dph)
    err = {}
    for f, name in ((I.U2R, "u_r"), (I.U2T, "u_theta"), (I.U2P, "u_phi"), (I.P2, "p"), (I.T, "T")):
        e = sh.get_field(f).cpu().numpy() - I.mms_fields(grid, tf, f, kind=kind)
        # midpoint l2 with the cell-centre volume of the nearest cell
        ec = e[:, :grid.nr, :grid.nt, :grid.np]
        err[name] = {"l2": float(np.sqrt(np.sum(vol * ec * ec))), "max": float(np.abs(e).max())}
    res = {"grid": [nr, nt, np_], "overlap": delta, "chi": chi, "tau": tau, "steps": nsteps, "rings": nring,
           "iterations": [min(iters), max(iters)],
           "mean_iterations": float(np.mean(iters)), "seconds": el,
           "mcell_steps_s": grid.cells * nsteps / el / 1e6, "errors": err}
    if keep:
        res["_fields"] = {f: sh.get_field(f).cpu().numpy() for f in (I.U2R, I.U2T, I.U2P, I.P2, I.T)}
        res["_vol"] = vol
    return res


def paper_mms(args):
    """Second workload: the paper's manufactured solution (eq. Exact) on the
    paper's grid 20x92x192 -- time convergence at Tf = 10 -- and a space
    convergence study (tau = 1e-3, Tf = 0.1) on 10x46x96, 20x92x192,
    40x184x384; prints the errors and the observed orders."""
    out = {"workload": "paper_mms_eq_exact_R1_1_R2_2", "tol": args.mms_tol, "kmax": args.mms_kmax,
           "mass_fix": bool(args.mms_mass_fix), "rings": args.mms_ring,
           "overlap": args.mms_delta,
           "chi": args.mms_chi, "time_tf": args.mms_tf, "time": [], "space": []}
    from paper_1905_02300_amd import yy

    def run(*a, keep=False, tol=1e-6):
        try:
            res = _paper_run(*a, tol=tol, kmax=args.mms_kmax, keep=keep, mass_fix=args.mms_mass_fix,
                             nring=args.mms_ring)
        except yy.YYError as e:
            res = {"grid": list(a[:3]), "tau": a[3], "overlap": a[5], "error": str(e)}
        print(json.dumps({k: v for k, v in res.items() if not k.startswith("_")}), file=sys.stderr, flush=True)
        return res

    taus = [float(x) for x in args.mms_taus.split(",")]
    out["time"] = [run(20, 92, 192, tau, args.mms_tf, args.mms_delta, args.mms_chi, keep=True, tol=args.mms_tol)
                   for tau in taus]
    # the time error alone: differences of successive runs at the final time
    # (the spatial error of the common grid cancels), l2 with cell volumes
    from paper_1905_02300_amd import inputs as I
    names = {I.U2R: "u_r", I.U2T: "u_theta", I.U2P: "u_phi", I.P2: "p", I.T: "T"}
    kept = [r for r in out["time"] if "_fields" in r]
    diffs = []
    for q in range(len(kept) - 1):
        a, b, vol = kept[q]["_fields"], kept[q + 1]["_fields"], kept[q]["_vol"]
        nr, nt, np_ = kept[q]["grid"]
        dq = {}
        for f, name in names.items():
            e = (a[f] - b[f])[:, :nr, :nt, :np_]
            dq[name] = float(np.sqrt(np.sum(vol * e * e)))
        diffs.append({"taus": [kept[q]["tau"], kept[q + 1]["tau"]], "l2_difference": dq})
    out["time_differences"] = diffs
    if len(diffs) >= 2:
        out["time_self_orders"] = {name: [math.log2(diffs[q]["l2_difference"][name] / diffs[q + 1]["l2_difference"][name])
                                          for q in range(len(diffs) - 1)] for name in names.values()}
    for r in out["time"]:
        r.pop("_fields", None)
        r.pop("_vol", None)
    out["space"] = [] if args.mms_no_space else [run(10 * m, 46 * m, 96 * m, 1e-3, 0.1, args.mms_delta, args.mms_chi)
                                                 for m in (1, 2, 4)]
    for key in ("time", "space"):
        runs = [r for r in out[key] if "errors" in r]
        if len(runs) < 2:
            continue
        out[key + "_orders"] = {
            name: [math.log2(runs[q]["errors"][name]["l2"] / runs[q + 1]["errors"][name]["l2"])
                   for q in range(len(runs) - 1)]
            for name in runs[0]["errors"]}
    print(json.dumps(out), flush=True)


def mixed_error(args):
    """FP32-mixed (FP32 stencils and sweeps; FP64 pressure, divergence and
    norms) against FP64 on the same grid and initial state after N steps:
    relative L2 (volume-free, over MAC points) and Linf errors of u, p, T,
    recorded at several step counts.  A third run, FP64 from the initial
    state rounded to FP32, separates the problem's own sensitivity to an
    eps32-sized perturbation of the data from the error the FP32 arithmetic
    injects every step.  T is also compared as its deviation from the
    conductive profile."""
    import torch
    from paper_1905_02300_amd import inputs as I
    from paper_1905_02300_amd import yy
    nr, nt, np_ = (int(x) for x in args.grid.split(","))
    pr, ra, dt, K = 1.0, 1e5, 2e-4, args.schwarz
    grid = I.Grid(nr, nt, np_)
    st = I.convection_state(grid, pr, ra, seed=3)
    st32 = {f: st[f].astype(np.float32).astype(np.float64) for f in st}
    tc = torch.as_tensor(I.conductive_T(grid), device="cuda")
    runs = (("fp64", yy.YY_FP64, st), ("fp32", yy.YY_FP32_MIXED, st), ("fp64_from_fp32_data", yy.YY_FP64, st32))
    shells, ms = {}, {}
    for name, prec, s0 in runs:
        sh = yy.Shell(nr, nt, np_, prec=prec)
        sh.set_params(pr=pr, ra=ra, dt=dt, chi=1.0, t_inner=1.0, t_outer=0.0)
        for f in range(9):
            sh.set_field(f, 0, s0[f])
            if f not in (I.P1, I.P2):
                sh.set_field(f, 1, s0[f])
        shells[name] = sh
    checkpoints = sorted({c for c in (1, 2, 5, 10, 20, 50, 100, args.mixed_error) if c <= args.mixed_error})
    names = ((I.U2R, "u_r"), (I.U2T, "u_theta"), (I.U2P, "u_phi"), (I.P2, "p"), (I.T, "T"))

    def diff(a_name, b_name):
        out = {}
        for f, nm in names:
            a = shells[a_name].get_field(f)
            b = shells[b_name].get_field(f)
            d = a - b
            out[nm] = {"l2_rel": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(b)),
                       "linf_rel": float(d.abs().max() / b.abs().max())}
        a = shells[a_name].get_field(I.T) - tc
        b = shells[b_name].get_field(I.T) - tc
        out["T_minus_conductive"] = {"l2_rel": float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)),
                                     "linf_rel": float((a - b).abs().max() / b.abs().max())}
        return out

    history = []
    done = 0
    for c in checkpoints:
        for name, sh in shells.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(c - done):
                sh.step(K)
            torch.cuda.synchronize()
            ms[name] = ms.get(name, 0.0) + (time.perf_counter() - t0) * 1e3
        done = c
        rec = {"steps": c, "fp32_mixed_vs_fp64": diff("fp32", "fp64"),
               "fp64_from_fp32_data_vs_fp64": diff("fp64_from_fp32_data", "fp64")}
        history.append(rec)
        print(json.dumps(rec), file=sys.stderr, flush=True)
    n = args.mixed_error
    print(json.dumps({"workload": f"fp32_mixed_vs_fp64_2x{nr}x{nt}x{np_}_K{K}", "steps": n,
                      "errors": history[-1]["fp32_mixed_vs_fp64"],
                      "fp64_from_fp32_data_vs_fp64": history[-1]["fp64_from_fp32_data_vs_fp64"],
                      "history": history,
                      "fp64_ms_per_step": ms["fp64"] / n, "fp32_mixed_ms_per_step": ms["fp32"] / n,
                      "fp32_mixed_speedup": ms["fp64"] / ms["fp32"],
                      "cells": grid.cells}), flush=True)


def ensemble(args):
    """N shells of uneven sizes (Nr in [16,64], Nt in [48,192], Np = 3 Nt,
    Ra log-uniform in [1e3, 1e6], seed 5), FP32-mixed, K Schwarz
    iterations, advanced together by the captured graphs; compared with the
    same shells stepped one after another without a graph."""
    import torch
    from paper_1905_02300_amd import inputs as I
    from paper_1905_02300_amd import yy
    shapes = I.ensemble_shapes(args.ensemble, seed=5)
    K, dt, pr = args.schwarz, 2e-4, 1.0
    ens = yy.Ensemble([s[:3] for s in shapes], prec=yy.YY_FP32_MIXED)
    cells = 0
    for q, (nr, nt, np_, ra) in enumerate(shapes):
        g = I.Grid(nr, nt, np_)
        cells += g.cells
        sh = ens.shells[q]
        sh.set_params(pr=pr, ra=ra, dt=dt, chi=1.0, t_inner=1.0, t_outer=0.0)
        st = I.convection_state(g, pr, ra, seed=1000 + q)
        for f in range(9):
            sh.set_field(f, 0, st[f])
            if f not in (I.P1, I.P2):
                sh.set_field(f, 1, st[f])
    t0 = time.perf_counter()
    tiles = ens.autotune()
    tune_s = time.perf_counter() - t0
    res = {}
    modes = args.ensemble_modes.split(",")
    for mode, graph in (("sequential_eager", 0), ("graph_streams", 2), ("graph_batched", 1)):
        if mode not in modes:
            continue
        for _ in range(max(args.warmup, 2)):
            ens.step(K, graph=graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ens.step(K, graph=graph)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[mode] = {"ms_per_step": el / args.steps * 1e3, "mcell_steps_s": cells * args.steps / el / 1e6}
        if graph == 1:
            b, n, m = ens.info()
            res[mode]["batched"] = b
            res[mode]["launches_per_step"] = n
            res[mode]["shell_launches_per_step"] = m
        print(json.dumps({mode: res[mode]}), file=sys.stderr, flush=True)
    if len(res) < 3:
        print(json.dumps({"workload": f"ensemble_{args.ensemble}_shells_seed5_fp32mixed_K{K}", **res}), flush=True)
        return
    best = res["graph_batched"]
    print(json.dumps({"metric": METRIC, "value": best["mcell_steps_s"], "unit": "Mcell-steps/s",
                      "workload": f"ensemble_{args.ensemble}_shells_seed5_fp32mixed_K{K}", "cells": cells,
                      "steps": args.steps, **res,
                      "batched_speedup_over_sequential": res["sequential_eager"]["ms_per_step"] / best["ms_per_step"],
                      "batched_speedup_over_stream_graph": res["graph_streams"]["ms_per_step"] / best["ms_per_step"],
                      "autotune_seconds": tune_s, "tiles": tiles,
                      "shells": [list(s[:3]) + [round(s[3], 1)] for s in shapes]}), flush=True)


_LINE_TILES_RT = ["t"] + ["m%dw%d%s" % (m, w, b) for m in (4, 6, 8, 12, 16) for w in (16, 32, 64)
                          for b in ("", "b")]
_LINE_TILES_P = ["l1", "l2", "l4", "v2", "v4", "v8"]


def line_solve_bench(nr=64, nt=192, np_=576, reps=20, nbuf=6, fixed=None):
    """The line-solve kernel alone: (I - tau/2 Pr D) y = x along r, theta,
    phi on both patches of a 2x64x192x576 grid (D = D_rr, Dhat_thth,
    Dhat_phph, and the true-metric D_thth, D_phph; tau = 1e-3, Pr = 1),
    FP64 and FP32, each with the fastest tile under these conditions.
    Algorithmic bytes per sweep: x read + y written = 2 words per cell.
    nbuf buffer pairs (> 1 GB in FP64) rotate so that the 256 MB
    last-level cache cannot hold the working set.  fixed: {prec: {dir:
    tile}} to time only these tiles (split metric), e.g. under a profiler."""
    import torch
    from paper_1905_02300_amd import inputs as I
    from paper_1905_02300_amd import yy
    g = I.Grid(nr, nt, np_)
    x0 = I.line_rhs(g, seed=2)
    out = {"grid": [nr, nt, np_], "cells": g.cells, "buffers": nbuf, "peak_gbs": HBM_PEAK_GBS}
    for name, prec, wb in (("fp64", yy.YY_FP64, 8), ("fp32", yy.YY_FP32_MIXED, 4)):
        sh = yy.Shell(nr, nt, np_, prec=prec)
        sh.set_params(pr=1.0, dt=1e-3)
        xs = [sh.to_internal(x0) for _ in range(nbuf)]
        ys = [sh.internal_tensor() for _ in range(nbuf)]
        def timed(d, metric, n):
            for q in range(nbuf):
                sh.sweep_diffusion(d, xs[q], ys[q], metric=metric)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for r in range(n):
                sh.sweep_diffusion(d, xs[r % nbuf], ys[r % nbuf], metric=metric)
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / n

        for metric, key in ((0, name), (1, name + "_true_metric")):
            if fixed is not None and (metric == 1 or name not in fixed):
                continue
            res = {}
            for d, dn in enumerate("rtp"):
                if metric == 1 and d == 0:
                    continue             # D_rr is the same in both metrics
                # the tile of this solve, chosen under the measurement's own
                # conditions (rotating buffers, out of the last-level cache)
                cands = _LINE_TILES_P if d == 2 else _LINE_TILES_RT
                if fixed is not None:
                    cands = [fixed[name][dn]]
                best = None
                for tile in cands:
                    sh.set_tuning('{"D.%s":"%s"}' % (dn, tile))
                    ms = timed(d, metric, 6) if len(cands) > 1 else 0.0
                    if best is None or ms < best[0]:
                        best = (ms, tile)
                sh.set_tuning('{"D.%s":"%s"}' % (dn, best[1]))
                ms = timed(d, metric, reps)
                gbs = 2 * wb * g.cells / (ms * 1e-3) / 1e9
                res[dn] = {"ms": ms, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS, "tile": best[1]}
            out[key] = res
        del xs, ys, sh
        torch.cuda.empty_cache()
    return out


def line_solve_cpu(nr=64, nt=192, np_=576):
    """The oracle's line solves (per-line Thomas in FP64 on the host cores)
    on the same 2x64x192x576 workload and right-hand side as the GPU
    line-solve benchmark: one sweep per direction, same 2-words-per-cell
    accounting."""
    from oracle import yyo
    from paper_1905_02300_amd import inputs as I
    g = I.Grid(nr, nt, np_)
    o = yyo.Shell(nr, nt, np_)
    o.set_params(pr=1.0, tau=1e-3)
    x = I.line_rhs(g, seed=2)
    res = {"kind": "oracle", "cores": yyo.omp_threads(), "unit": "GB/s"}
    for name, op in (("r", yyo.OP_DRR), ("t", yyo.OP_DTT_HAT), ("p", yyo.OP_DPP_HAT)):
        t0 = time.perf_counter()
        o.sweep_op(op, x)
        el = time.perf_counter() - t0
        res[name] = {"ms": el * 1e3, "gbs": 2 * 8 * g.cells / el / 1e9}
    o.close()
    return res


def parity_oracle(args):
    """The first N steps of the benchmark's workload on the GPU (FP64, the
    tiles the autotuner picks, as in the timed run) and on the oracle (all
    host threads; a progress line per Schwarz iteration), compared field by
    field: max |gpu - oracle| relative to the oracle's max, and the
    velocities' rounding floor of the cancelling buoyancy and hydrostatic
    pressure gradient (16 eps tau Pr Ra max|T| per correction)."""
    import torch
    from oracle import yyo
    from paper_1905_02300_amd import inputs as I
    from paper_1905_02300_amd import yy
    nr, nt, np_ = (int(x) for x in args.grid.split(","))
    pr, ra, dt, K, n = 1.0, 1e5, 2e-4, args.schwarz, args.parity_oracle
    grid = I.Grid(nr, nt, np_)
    st = I.convection_state(grid, pr, ra, seed=3)
    sh = yy.Shell(nr, nt, np_, prec=yy.YY_FP64)
    sh.set_params(pr=pr, ra=ra, dt=dt, chi=1.0, t_inner=1.0, t_outer=0.0)
    for f in range(9):
        sh.set_field(f, 0, st[f])
        if f not in (I.P1, I.P2):
            sh.set_field(f, 1, st[f])
    tiles = sh.autotune()
    for _ in range(n):
        sh.step(K)
    got = {f: sh.get_field(f).cpu().numpy() for f in range(9)}
    gn = sh.norms()
    del sh
    torch.cuda.empty_cache()
    print(f"gpu: {n} steps done", file=sys.stderr, flush=True)
    o = yyo.Shell(nr, nt, np_)
    o.set_verbose(True)
    o.set_params(pr=pr, ra=ra, tau=dt, chi=1.0, t_inner=1.0, t_outer=0.0)
    for f in range(9):
        o.set_field(f, 0, st[f])
        if f not in (I.P1, I.P2):
            o.set_field(f, 1, st[f])
    steps_s = []
    for s_ in range(n):
        t0 = time.perf_counter()
        o.step(K)
        steps_s.append(time.perf_counter() - t0)
        print(f"oracle: step {s_ + 1} done in {steps_s[-1]:.1f} s", file=sys.stderr, flush=True)
    M = pr * ra * float(np.max(np.abs(st[I.T])))
    floor = 16 * np.finfo(float).eps * dt * M * n * K
    fields = {}
    ok = True
    for f in range(9):
        b = o.get_field(f)
        err = float(np.max(np.abs(got[f] - b)))
        scale = float(np.max(np.abs(b)))
        lim = 1e-12 * scale + (0.0 if f in (I.T, I.P1, I.P2) else floor)
        fields[I.FIELD_NAMES[f]] = {"max_abs_diff": err, "max_abs_oracle": scale, "relative": err / scale,
                                    "bound": lim, "ok": bool(err <= lim)}
        ok = ok and bool(err <= lim)
    on = o.norms(K)
    out = {"workload": f"yinyang_ac_step_2x{nr}x{nt}x{np_}_fp64_K{K}", "steps": n, "Pr": pr, "Ra": ra, "dt": dt,
           "tiles": tiles, "fields": fields, "velocity_rounding_floor": floor, "all_within_bound": ok,
           "norms_max_relative_difference": float(np.max(np.abs(gn - on) / np.maximum(np.abs(on), 1e-300))),
           "oracle_seconds_per_step": steps_s, "oracle_threads": yyo.omp_threads(),
           "oracle_mcell_steps_s": grid.cells / float(np.mean(steps_s)) / 1e6,
           "command": "python3 bench.py --parity-oracle %d --grid %s --out %s" % (n, args.grid, args.out)}
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)


def cpu_baseline(grid_s, pr, ra, dt, K, nsteps=2, single_grid="20,60,180"):
    """The oracle as it stands, on the host cores: the first nsteps steps of
    the same workload (same physics, schedule and start) on a bounded grid,
    all host threads; and one step on a smaller grid on one thread."""
    from oracle import yyo
    from paper_1905_02300_amd import inputs as I

    def run(gs, steps):
        nr, nt, np_ = (int(x) for x in gs.split(","))
        grid = I.Grid(nr, nt, np_)
        o = yyo.Shell(nr, nt, np_)
        o.set_params(pr=pr, ra=ra, tau=dt, chi=1.0, t_inner=1.0, t_outer=0.0)
        st = I.convection_state(grid, pr, ra, seed=3)
        for f in range(9):
            o.set_field(f, 0, st[f])
            o.set_field(f, 1, st[f])
        del st
        t0 = time.perf_counter()
        for _ in range(steps):
            o.step(K)
        el = time.perf_counter() - t0
        o.close()
        return grid, el

    yyo.set_threads(0)
    grid, el = run(grid_s, nsteps)
    out = {"value": grid.cells * nsteps / el / 1e6, "unit": "Mcell-steps/s", "cores": yyo.omp_threads(),
           "kind": "oracle",
           "sample": f"the first {nsteps} steps (K={K}) of the same convecting-shell workload on a "
                     f"2x{grid.nr}x{grid.nt}x{grid.np} grid ({grid.cells} cells), {el:.1f} s wall"}
    yyo.set_threads(1)
    g1, e1 = run(single_grid, 1)
    yyo.set_threads(0)
    out["single_thread"] = {"value": g1.cells / e1 / 1e6, "unit": "Mcell-steps/s", "cores": 1,
                            "sample": f"one step (K={K}) on a 2x{g1.nr}x{g1.nt}x{g1.np} grid "
                                      f"({g1.cells} cells), {e1:.1f} s wall"}
    return out


if __name__ == "__main__":
    main()
