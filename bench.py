"""Benchmark: SCR+AMG solves/s at a 1e-8 relative residual, FP64 against mixed precision, on the
refined unified fluid+solid tube (lumen R=1 with 4 boundary-layer shells, wall 1.0-1.2, L=10;
69x69x306 = 1,456,866 nodes, 1,525,410 block rows with the interface pressure rows, 23.5M 4x4
blocks) plus its mesh-motion solve.  --workload cfg1 runs the 300,899-node tube, cfg4 the
4.0M-node Y-bifurcation.

One step = one Newton corrector's linear work on the GPU:
    amg_setup(SCR_SYSTEM)  (block split, S^, AMG(A), AMG(S^), sliced-ELL copies)
  + scr_solve              (FGMRES(P_SCR) to ||b - Kx|| <= 1e-8 ||b||)
  + mesh_motion_solve      (CG + AMG(L), 3 right-hand sides, tol 1e-8; the mesh hierarchy is
                            built once before the timed region, as the paper's Sec. 5.2.2 does)
Inputs are resident in HBM before the timed region.  Each step uses its own seeded RHS.  The FP64
pass (W warm-up steps, then K timed steps) gives `value`; the mixed pass (FP32 hierarchy and
V-cycle, FP64 Krylov; one warm-up step, then K timed steps) is reported beside it.  The first
step's right-hand side is the oracle reference's: the solutions of both passes are compared with
the oracle's refined solution there, velocity and pressure apart.
Outside the timed region the line also reports the numeric re-setup (amg_update: new values on
the same pattern, aggregates kept) as resetup_ms beside the full setup_ms, and the device assembly
of the tangent matrix from the tetrahedra (scr_assemble_tangent, at the workload's advective state)
as "assembly".
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["cfg1", "cfg2", "cfg4"], default="cfg2",
                    help="cfg2 (default): the refined unified tube (1,456,866 nodes); cfg1: the unified tube "
                         "(300,899 nodes); cfg4: Y-bifurcation (about 4.0M nodes, mixed headline)")
    ap.add_argument("--precond", choices=["scr", "simple", "simplec"], default="scr",
                    help="outer preconditioner: SCR (Algorithm 1), SIMPLE or SIMPLEC (Sec. 5.2.1)")
    ap.add_argument("--dt-sweep", action="store_true",
                    help="compare SCR and SIMPLE iterations and times on cfg1 at dt = 1e-5, 1e-4, 1e-3 (FP64)")
    ap.add_argument("--flow", action="store_true",
                    help="cfg1 with the advective Poiseuille state (u_max = 30 cm/s; nonsymmetric velocity block) "
                         "and the outlet resistance coupling (m = 1000) attached in every step")
    ap.add_argument("--precision", choices=["fp64", "mixed", "mixed32", "both", "all"], default=None,
                    help="default: both (fp64 then mixed) for cfg1 and cfg2, mixed for cfg4; mixed32 is mixed "
                         "with Algorithm 2's inner solve on FP32 vectors; all = fp64, mixed, mixed32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB elementwise copy (read 1 GiB, write 1 GiB) before the steps, "
                         "as the calibration kernel of the rocprofv3 FETCH_SIZE/WRITE_SIZE counters")
    ap.add_argument("--serve", action="store_true",
                    help="serving stream instead of the single-system step: seeded tube requests of random "
                         "geometry through the continuous-batching server (mixed precision)")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--load", type=float, default=0.8, help="Poisson arrival rate as a fraction of saturation")
    ap.add_argument("--stepper", action="store_true",
                    help="time steps of the device predictor multi-corrector (scr_step) on --workload cfg1/cfg2: "
                         "seeded body force, --steps steps of dt = 1e-3 then one of 5e-4 (a numeric re-setup)")
    ap.add_argument("--amg", action="append", default=[], metavar="KEY=VALUE",
                    help="override an scr_amg_opts field for every hierarchy (repeatable), e.g. --amg theta=0.04")
    ap.add_argument("--dump-levels", metavar="JSON", default=None,
                    help="write the hierarchy sizes (AMG(A), AMG(S^), AMG(L)) and the first step's V-cycle "
                         "counts to JSON (for --kernel-table)")
    ap.add_argument("--kernel-table", nargs=2, metavar=("TRACE_DIR", "LEVELS_JSON"), default=None,
                    help="CPU only: per-kernel table (time, algorithmic bytes, GB/s) from a rocprofv3 kernel trace "
                         "of a one-step FP64 run and its --dump-levels file")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) into profiles/ and exit")
    return ap.parse_args()


HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
FLOW_U_MAX = 30.0       # --flow: centreline speed of the advective state (cm/s)
FLOW_M = 1000.0         # --flow: outlet resistance coefficient of the coupling
# the files that define the profiled kernel and its data layout
KERNEL_SOURCES = ["paper_2206_06996_amd/csrc/sparse.hip", "paper_2206_06996_amd/csrc/common.h"]


def pmc_path(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"smooth_a0_{workload}_pmc.json")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def pmc_traffic(workload: str):
    """HBM bytes per launch of the profiled kernel from the committed rocprofv3 --pmc summary of
    the workload (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration, averaged over
    the variants in the proportion the timed steps launch them), or None when the kernel sources
    changed since the counters were taken."""
    path = pmc_path(workload)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("traffic_bytes_per_launch")


COPY_BYTES = 1 << 30   # calibration copy: 1 GiB read + 1 GiB written
# the timed family: level-0 smoother steps of AMG(A) with a matrix product (the first, middle and
# last Chebyshev steps; the zero-initial-guess step has no product and is not timed)
SMOOTH_RE = r"smooth_rl3_k<double, (true|false), (true|false), false>"


def _pmc_rows(d, counter):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") == counter:
                rows.append(r)
    return rows


def pmc_summary(fetch_dir, write_dir, workload):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the level-0 smoother steps (all variants with
    a matrix product, averaged over their dispatches as the live timing averages them) and of the
    calibration copy; the copy's known 1 GiB read and 1 GiB write give the counter scale."""
    import re
    out = {"kernel": SMOOTH_RE, "source_hash": kernel_source_hash(), "workload": f"{workload} fp64, 1 step"}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _pmc_rows(d, counter)
        sm = [float(r["Counter_Value"]) for r in rows if re.search(SMOOTH_RE, r["Kernel_Name"])]
        # the calibration copies: the first three large elementwise dispatches (they run before
        # anything else of that size; later large ones belong to the assembly check)
        big = sorted((r for r in rows if "elementwise" in r["Kernel_Name"]
                      and float(r["Counter_Value"]) > 0.25 * COPY_BYTES / 1024), key=lambda r: int(r["Dispatch_Id"]))
        cp = [float(r["Counter_Value"]) for r in big[:3]]
        if not sm or not cp:
            raise SystemExit(f"no {counter} rows for the smoother or the copy in {d}")
        scale = (COPY_BYTES / 1024.0) / float(np.median(cp))
        out[counter] = {"smoother_kib_per_dispatch_mean": float(np.mean(sm)), "dispatches": len(sm),
                        "copy_kib_per_dispatch_median": float(np.median(cp)), "copy_expected_kib": COPY_BYTES / 1024.0,
                        "scale": scale, "smoother_bytes_scaled": float(np.mean(sm)) * 1024.0 * scale}
    out["traffic_bytes_per_launch"] = out["FETCH_SIZE"]["smoother_bytes_scaled"] + out["WRITE_SIZE"]["smoother_bytes_scaled"]
    path = pmc_path(workload)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def amg_overrides(args):
    out = {}
    for kv in args.amg:
        k, v = kv.split("=", 1)
        out[k] = float(v) if any(c in v for c in ".e") else int(v)
    return out


def dump_levels(path, scr, h, hm, s, first_stats):
    """Sizes of every level of the three FP64 hierarchies and one step's V-cycle counts."""
    out = {"n_b": int(s.n_b), "nnzb": int(s.nnzb), "n_phys": int(s.n_phys), "nnzL": int(s.Lci.size), "hier": {}}
    for name, hh, which in (("A", h, 0), ("S", h, 1), ("L", hm, 2)):
        out["hier"][name] = [hh.hier_level_info(which, l) for l in range(hh.hier_levels(which))]
    if first_stats is not None:
        st, stm = first_stats
        out["step"] = {k: st[k] for k in ("outer_it", "its_A", "its_S", "its_I", "vcycles_A", "vcycles_S")}
        out["step"]["mesh_its"] = list(stm["mesh_its"])
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


def _kt_bytes(levels):
    """Grid size -> (algorithmic bytes, where) for every launch shape of the V-cycle, Krylov and
    product kernels: each stored matrix value and index once, each vector it must read or write
    once.  D^-1 is not counted (it follows from the diagonal block the smoother streams)."""
    from math import ceil
    H = levels["hier"]
    shapes = {}

    def add(key, grid, byts, where):
        shapes.setdefault(key, {}).setdefault(grid, (byts, where))

    def slice_grid(nr, b, wps):
        nsl = ceil(nr / (64 // b))
        spb = 1 if wps >= 4 else 4 // wps
        return ceil(nsl / spb) * spb * wps * 64
    for name, lv in H.items():
        for l, L in enumerate(lv):
            nr, b, k, nnz = L["nr"], L["b"], L["k"], L["nnzA"]
            last = l + 1 == len(lv)
            if last:
                n = L["ncoarse"]
                add("dense_mv_k<double>", ceil(n / 4) * 256, 8.0 * n * n + 16.0 * n, f"{name}{l} coarse")
                add("dense_mv3_k<double>", ceil(n / 4) * 256, 8.0 * n * n + 48.0 * n, f"{name}{l} coarse")
                continue
            for tn, tb in (("double", 8.0), ("float", 4.0)):     # FP64 and the mixed form's FP32 V-cycle
                mat = nnz * (b * b * tb + 4.0)
                vec = b * tb
                for rd in (0, 1):
                    for wd in (0, 1):
                        byts = mat + nr * (4.0 + vec * (3 + rd + wd))
                        zero = nr * (4.0 + vec * (2 + wd))
                        if b == 3 and l == 0:
                            g = ceil(ceil(nr / 64) / 4) * 256
                            add(f"smooth_rl3_k<{tn},{rd},{wd},0>", g, byts, f"{name}{l}")
                            add(f"smooth_rl3_k<{tn},0,{wd},1>", g, zero, f"{name}{l}")
                        for w in (1, 2, 4, 8, 16):
                            add(f"smooth_k<{tn},{b},{rd},{wd},0,{w}>", slice_grid(nr, b, w), byts, f"{name}{l}")
                            add(f"smooth_k<{tn},{b},0,{wd},1,{w}>", slice_grid(nr, b, w), zero, f"{name}{l}")
                            if b == 1:
                                add(f"smooth3_k<{tn},{rd},{wd},0,{w}>", slice_grid(nr, 1, w),
                                    nnz * (tb + 4.0) + nr * (4.0 + 3 * tb * (3 + rd + wd)), f"{name}{l}")
                                add(f"smooth3_k<{tn},0,{wd},1,{w}>", slice_grid(nr, 1, w), nr * (4.0 + 3 * tb * (2 + wd)),
                                    f"{name}{l}")
                # products with A_l (residual y = b - A x: x, b read, y written)
                for mode in (0, 1, 3):
                    nv = 2 if mode == 0 else 3
                    byts = mat + nr * (4.0 + vec * nv)
                    if b == 3 and l == 0:
                        add(f"sell_mv_rl3_k<{tn},3,{mode}>", ceil(ceil(nr / 64) / 4) * 256, byts, f"{name}{l} A")
                    for w in (1, 2, 4, 8, 16):
                        add(f"sell_mv_k<{tn},{b},{b},{mode},{w}>", slice_grid(nr, b, w), byts, f"{name}{l} A")
                        if b == 1:
                            add(f"sell_mv3_k<{tn},{mode},{w}>", slice_grid(nr, 1, w), nnz * (tb + 4.0) + nr * (4.0 + 3 * tb * nv),
                                f"{name}{l} A")
                # prolongation y += P x (P: nr x nc blocks b x k; x coarse, y read and written)
                nc, nnzp = L["nagg"], L["nnzP"]
                pbytes = nnzp * (b * k * tb + 4.0) + nc * k * tb + nr * (4.0 + 2 * b * tb)
                if b == 3 and l == 0:
                    add(f"sell_mv_rl3_k<{tn},{k},2>", ceil(ceil(nr / 64) / 4) * 256, pbytes, f"{name}{l} P")
                for w in (1, 2, 4, 8, 16):
                    add(f"sell_mv_k<{tn},{b},{k},2,{w}>", slice_grid(nr, b, w), pbytes, f"{name}{l} P")
                    if b == 1:
                        add(f"sell_mv3_k<{tn},2,{w}>", slice_grid(nr, 1, w),
                            nnzp * (tb + 4.0) + nc * 3 * tb + nr * (4.0 + 6 * tb), f"{name}{l} P")
                # restriction y = R x (R: nc x nr blocks k x b)
                rbytes = L["nnzR"] * (k * b * tb + 4.0) + nr * b * tb + nc * (4.0 + k * tb)
                add(f"bsrt_mv_k<{tn},{k},{b}>", ceil(nc / 4) * 256, rbytes, f"{name}{l} R")
                if b == 1:
                    add(f"bsrt_mv3_k<{tn}>", ceil(nc / 4) * 256, L["nnzR"] * (tb + 4.0) + nr * 3 * tb + nc * (4.0 + 3 * tb), f"{name}{l} R")
    nb, nnzb = levels["n_b"], levels["nnzb"]
    for mode in (0, 1):
        add(f"sell_mv_split4_k<{mode}>", ceil(ceil(nb / 16) / 4) * 256,
            nnzb * (16 * 8.0 + 4.0) + nb * (4.0 + 32.0 * (2 + mode)), "K")
    return shapes


def _kt_key(name):
    """Normalised template key of a demangled kernel name (booleans as 0/1, no spaces)."""
    import re
    m = re.match(r"(?:void )?scr::(?:\(anonymous namespace\)::)?([A-Za-z0-9_]+)(<[^()]*>)?", name)
    if not m:
        return None
    base, targs = m.group(1), (m.group(2) or "")
    targs = targs.replace(" ", "").replace("true", "1").replace("false", "0")
    return base + targs


def kernel_table(trace_dir, levels_json):
    import csv
    import glob
    levels = json.load(open(levels_json))
    shapes = _kt_bytes(levels)
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *kernel_trace.csv under {trace_dir}")
    agg = {}
    total_ns = 0.0
    for f in files:
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"]
            ns = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
            grid = int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0)
            total_ns += ns
            a = agg.setdefault(name, {"calls": 0, "ns": 0.0, "bytes": 0.0, "bytes_ns": 0.0, "where": set()})
            a["calls"] += 1
            a["ns"] += ns
            key = _kt_key(name)
            hit = shapes.get(key, {}).get(grid) if key else None
            if hit:
                a["bytes"] += hit[0]
                a["bytes_ns"] += ns
                a["where"].add(hit[1])
    rows = sorted(agg.items(), key=lambda kv: -kv[1]["ns"])
    print(f"Total kernel time {total_ns / 1e6:.1f} ms over {sum(a['calls'] for a in agg.values())} dispatches.\n")
    print("| total ms | % | calls | avg us | alg. bytes / call | GB/s | of 8 TB/s | levels | kernel |")
    print("|---:|---:|---:|---:|---:|---:|---:|---|---|")
    tb = tt = 0.0
    for name, a in rows[:25]:
        cov = a["bytes_ns"] / a["ns"] if a["ns"] else 0.0
        if a["bytes"] and cov > 0.999:
            gbs = a["bytes"] / a["ns"]
            b_call = f"{a['bytes'] / a['calls'] / 1e6:.1f} MB"
            rate, frac = f"{gbs:.0f}", f"{gbs / HBM_PEAK_GBS:.2f}"
        else:
            b_call, rate, frac = "-", "-", "-"
        short = name.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0][:70]
        print(f"| {a['ns'] / 1e6:.2f} | {100 * a['ns'] / total_ns:.1f} | {a['calls']} | {a['ns'] / a['calls'] / 1e3:.2f} | "
              f"{b_call} | {rate} | {frac} | {', '.join(sorted(a['where']))[:40]} | `{short}` |")
    for name, a in agg.items():
        if a["bytes"] and a["bytes_ns"] >= 0.999 * a["ns"]:
            tb += a["bytes"]; tt += a["ns"]
    print(f"\nKernels with a byte count (every dispatch matched to a level): {tt / 1e6:.1f} ms of {total_ns / 1e6:.1f} ms "
          f"kernel time ({100 * tt / total_ns:.1f} %), {tb / 1e9:.2f} GB algorithmic, "
          f"{tb / tt:.0f} GB/s = {tb / tt / HBM_PEAK_GBS:.3f} of 8 TB/s.")


def load_reference(workload):
    """The oracle's reference run of the workload (oracle/<workload>_reference.json, written by
    oracle/reference_run.py), if it is complete; read as data only."""
    path = os.path.join(ROOT, "oracle", f"{workload}_reference.json")
    if not os.path.exists(path):
        return None
    ref = json.load(open(path))
    return ref if "xtv_sample" in ref else None


def field_errors_vs_reference(x, ref):
    """Sampled relative errors of the velocity and the pressure of x against the oracle's refined
    solution of the reference right-hand side (each field against its own norm)."""
    out = {}
    for f, name in (("v", "velocity"), ("p", "pressure")):
        idx = np.array(ref[f"x{f}_sample_idx"])
        r = np.array(ref[f"xt{f}_sample"])
        out[name] = float(np.linalg.norm(x[idx] - r) / np.linalg.norm(r))
    return out


def cpu_baseline(s, bm, args, ref):
    """The FP64 oracle on all host cores (OpenMP over independent rows, fixed-chunk dot products:
    the same results on any thread count), on a bounded sample of the same workload, run live:
    its full AMG setup of the SCR system, its full mesh-motion solve, two applications of
    Algorithm 2 (the matrix-free Schur product: an inner GMRES+AMG(A) solve to delta_I on a
    random vector) and three V-cycles of AMG(S^).  The solve time is estimated from the oracle's
    own operation counts for this workload's reference right-hand side (the reference file):
        calls_I x t(Alg. 2) + its_A x t(Alg. 2) / (its_I / calls_I) + its_S x t(V-cycle S^),
    i.e. every GMRES iteration on A is priced at the live per-iteration cost of the inner solves.
    The outer FGMRES and the Schur-level vector work are not counted (a lower bound on the
    oracle's time)."""
    import oracle
    st = ref["stats_1e-8"]
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    t_setup = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    for _ in range(2):
        o.apply("S", rng.uniform(-1, 1, s.n_b))
    t_s = (time.perf_counter() - t0) / 2
    x = rng.uniform(-1, 1, s.n_b)
    t0 = time.perf_counter()
    for _ in range(3):
        o.apply("VS", x)
    t_vs = (time.perf_counter() - t0) / 3
    del o
    m = oracle.Mesh(s.Lrp, s.Lci, s.Lval)
    t0 = time.perf_counter()
    m.solve(bm, tol=1e-8)
    t_mesh = time.perf_counter() - t0
    del m
    per_it = t_s / (st["its_I"] / st["calls_I"])
    t_solve = st["calls_I"] * t_s + st["its_A"] * per_it + st["its_S"] * t_vs
    total = t_setup + t_solve + t_mesh
    log(f"[bench] oracle sample ({threads} threads): setup {t_setup:.1f}s Alg.2 {t_s:.2f}s V-cycle S {t_vs:.3f}s "
        f"mesh {t_mesh:.1f}s -> step {total:.1f}s", args)
    full = ref["setup_s"] + ref["solve_1e-8_s"] + ref["mesh_solve_1e-8_s"]
    return {"value": round(1.0 / total, 6), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"live, {threads} threads: oracle AMG setup of the full {args.workload} SCR system "
                       f"({t_setup:.1f} s), full mesh-motion solve ({t_mesh:.1f} s), 2 applications of Algorithm 2 "
                       f"({t_s:.2f} s each, an inner GMRES+AMG(A) solve to 1e-3), 3 V-cycles of AMG(S^) "
                       f"({t_vs:.3f} s each); solve time = the oracle's own counts for this workload "
                       f"({st['calls_I']} Alg. 2 calls, {st['its_A']} A iterations, {st['its_S']} S iterations) x "
                       f"live unit times; outer FGMRES and Schur-level vector work excluded (a lower bound on "
                       f"oracle time)"),
            "step_s_estimate": round(total, 2),
            "full_run_reference": (f"oracle/{args.workload}_reference.json: one full oracle step (setup + solve to 1e-8 "
                                   f"+ mesh) took {full:.0f} s on {ref.get('omp_threads', '?')} threads when the "
                                   f"reference was written (another host)")}


def _serve_requests(n, seed):
    """Per request: length U[2,10], radius U[0.5,1.5], node count log-uniform in [20k, 400k],
    1-4 successive corrections; unit-rate exponential gaps (scaled by the arrival rate later)."""
    rng = np.random.default_rng(seed)
    return dict(L=rng.uniform(2.0, 10.0, n), R=rng.uniform(0.5, 1.5, n),
                N=np.exp(rng.uniform(math.log(2e4), math.log(4e5), n)), c=rng.integers(1, 5, n),
                gaps=rng.exponential(1.0, n))


def serve_bench(args):
    """Serving stream: a saturation pass (every request submitted at t = 0; its makespan gives the
    throughput) then a Poisson pass at args.load x that rate (request latency = arrival -> last
    correction done).  Inputs of every request are resident in HBM before either pass."""
    import threading
    from concurrent.futures import ThreadPoolExecutor

    import torch
    import synth
    import paper_2206_06996_amd.scr as scr

    spec = _serve_requests(args.requests, 0)
    n = args.requests

    def make(r):
        s = synth.generate(synth.tube_params(spec["N"][r], spec["R"][r], spec["L"][r]))
        mm = np.repeat(s.Lmask, 3)
        b = [synth.rhs(1_000_003 * (r + 1) + c, 4 * s.n_b, s.mask) for c in range(spec["c"][r])]
        bm = [synth.rhs(2_000_003 * (r + 1) + c, 3 * s.n_phys, mm) for c in range(spec["c"][r])]
        return s, b, bm

    t0 = time.time()
    gen = ThreadPoolExecutor(8)
    futs = [gen.submit(make, r) for r in range(n)]
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    reqs = []
    for r, f in enumerate(futs):
        s, b, bm = f.result()
        futs[r] = None
        reqs.append(dict(K=(dev(s.rp), dev(s.ci), dev(s.val.reshape(-1))), coords=dev(s.xyz.reshape(-1)),
                         L=(dev(s.Lrp), dev(s.Lci), dev(s.Lval)), b=[dev(v) for v in b], bm=[dev(v) for v in bm],
                         n_b=int(s.n_b), nnzb=int(s.nnzb), nodes=int(s.n_phys)))
        if (r + 1) % 32 == 0:
            log(f"[serve] generated {r + 1}/{n} requests ({time.time() - t0:.0f}s)", args)
    gen.shutdown()
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    ctx = scr.Context(0)
    ao = scr.amg_opts(precision=scr.SCR_MIXED)
    so = scr.solve_opts()
    n_rhs = int(sum(len(q["b"]) for q in reqs))
    log(f"[serve] {n} requests, {n_rhs} right-hand sides, nodes {min(q['nodes'] for q in reqs)}-"
        f"{max(q['nodes'] for q in reqs)}; budget {budget / 2**30:.1f} GiB, {args.slots} slots", args)

    def run(arrivals):
        srv = scr.Server(ctx, max_slots=args.slots, hbm_budget=budget, amg=ao, solve=so)
        outs = [([torch.zeros_like(v) for v in q["b"]], [torch.zeros_like(v) for v in q["bm"]]) for q in reqs]
        torch.cuda.synchronize()
        ids = [None] * n
        t_start = time.perf_counter()

        def feeder():
            for r in range(n):
                dt = t_start + arrivals[r] - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                q = reqs[r]
                ids[r] = srv.submit(q["K"], q["coords"], q["b"], outs[r][0], L=q["L"], bms=q["bm"], xms=outs[r][1])

        th = threading.Thread(target=feeder)
        th.start()
        res = []
        for r in range(n):
            while ids[r] is None:
                time.sleep(1e-4)
            res.append(srv.wait(ids[r]))
            if (r + 1) % 32 == 0:
                log(f"[serve] {r + 1}/{n} done ({time.perf_counter() - t_start:.1f}s)", args)
        th.join()
        max_active = srv.drain()
        makespan = time.perf_counter() - t_start
        srv.destroy()
        bad = [(r, x["status"], x["last"]["rel_res_true"]) for r, x in enumerate(res)
               if x["status"] != 0 or x["last"]["rel_res_true"] > so.tol]
        if bad:
            raise RuntimeError(f"serving: requests failed or missed the tolerance: {bad[:5]}")
        if args.requests <= 32 or arrivals.max() == 0:
            for r, x in enumerate(res):
                st = x["last"]
                log(f"[serve]   req {r:3d} nodes {reqs[r]['nodes']:6d} R {spec['R'][r]:.2f} L {spec['L'][r]:.2f} "
                    f"rhs {x['n_solves']} queue {x['queue_ms']:8.1f} setup {x['setup_ms']:7.1f} solve {x['solve_ms']:8.1f} ms "
                    f"outer {st['outer_it']} its_A {st['its_A']} its_S {st['its_S']} vA {st['vcycles_A']}", args)
        lat = np.array([x["latency_ms"] for x in res])
        per_rhs = np.array([x["solve_ms"] / x["n_solves"] for x in res])
        return dict(makespan_s=round(makespan, 3), solves_per_s=round(n_rhs / makespan, 4),
                    requests_per_s=round(n / makespan, 4), max_active=max_active,
                    p50_ms=round(float(np.percentile(lat, 50)), 1), p99_ms=round(float(np.percentile(lat, 99)), 1),
                    queue_p50_ms=round(float(np.percentile([x["queue_ms"] for x in res], 50)), 1),
                    per_rhs_p50_ms=round(float(np.percentile(per_rhs, 50)), 1),
                    per_rhs_p99_ms=round(float(np.percentile(per_rhs, 99)), 1),
                    outer_it_max=int(max(x["last"]["outer_it"] for x in res)),
                    max_rel_res=float(max(x["last"]["rel_res_true"] for x in res)))

    warm = reqs[0]
    h = scr.amg_setup(ctx, scr.SCR_SYSTEM, *warm["K"], warm["coords"], ao)
    scr.scr_solve(h, warm["b"][0], torch.zeros_like(warm["b"][0]), so)
    h.destroy()
    sat = run(np.zeros(n))
    log(f"[serve] saturation: {sat}", args)
    rate = args.load * sat["requests_per_s"]
    arrivals = np.cumsum(spec["gaps"]) / rate
    poi = run(arrivals)
    poi["arrival_rate_per_s"] = round(rate, 4)
    log(f"[serve] poisson: {poi}", args)
    ctx.destroy()
    out = {
        "metric": "SCR+AMG solves/s at 1e-8 rel. resid (FP64 vs mixed); p50/p99 solve latency",
        "value": sat["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": n, "warmup": 1,
        "ms_per_step": round(1e3 * sat["makespan_s"] / n_rhs, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic (seeded tube requests, seeded RHS)",
        "config": {"workload": f"serving stream: {n} unified tube requests (L U[2,10], R U[0.5,1.5], nodes "
                               f"log-U[20k,400k], 1-4 corrections each, {n_rhs} right-hand sides) + mesh motion",
                   "precision": "mixed", "tol": so.tol, "slots": args.slots},
        "saturation": sat, "poisson": poi, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def dt_sweep(args):
    """SCR against SIMPLE and SIMPLEC on the cfg1 tube as the time step grows (the paper's Sec. 6
    comparison of the two preconditioners over dt): outer iterations, block iterations and solve
    time per preconditioner, FP64, tol 1e-8, at most 200 outer iterations."""
    import torch
    import synth
    import paper_2206_06996_amd.scr as scr
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    ctx = scr.Context(0)
    rows = []
    for dt in (1e-5, 1e-4, 1e-3):
        s = synth.generate(synth.default_params(mode=0, m_core=12, n_bl=4, n_wall=4, nz=178, R=1.0, L=10.0, dt=dt))
        K = (dev(s.rp), dev(s.ci), dev(s.val.reshape(-1)))
        b = dev(synth.rhs(1000, 4 * s.n_b, s.mask))
        for name, diag, pc in (("SCR", 0, scr.SCR_PRECOND_SCR), ("SIMPLE", 0, scr.SCR_PRECOND_SIMPLE),
                               ("SIMPLEC", 1, scr.SCR_PRECOND_SIMPLE)):
            h = scr.amg_setup(ctx, scr.SCR_SYSTEM, *K, dev(s.xyz.reshape(-1)), scr.amg_opts(schur_diag=diag))
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = scr.scr_solve(h, b, x, scr.solve_opts(precond=pc, max_it=200))
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            h.destroy()
            row = dict(dt=dt, precond=name, converged=bool(st["converged"]), outer_it=st["outer_it"],
                       its_A=st["its_A"], its_S=st["its_S"], its_I=st["its_I"], solve_ms=round(1e3 * t, 1),
                       rel_res=st["rel_res_true"])
            log(f"[dt-sweep] {row}", args)
            rows.append(row)
    ctx.destroy()
    print(json.dumps({"metric": "SCR vs SIMPLE/SIMPLEC over the time step (outer iterations, solve ms)",
                      "unit": "iterations", "config": {"workload": "cfg1 tube, dt in {1e-5, 1e-4, 1e-3}",
                                                       "precision": "fp64", "tol": 1e-8, "max_it": 200},
                      "rows": rows}))


def stepper_bench(args):
    """Time steps of the segregated predictor multi-corrector (Sec. 3.5) on the device: each step
    assembles the residual at the intermediate states, solves the corrector systems (scr_solve) and
    the mesh motion (three-column CG), and updates every field; a new dt also re-assembles the four
    operator forms and re-sets the hierarchies up numerically."""
    import torch
    import synth
    import paper_2206_06996_amd.scr as scr
    prec = {"fp64": scr.SCR_FP64, "mixed": scr.SCR_MIXED}.get(args.precision or "fp64", scr.SCR_FP64)
    prm = {"cfg1": synth.cfg1_params, "cfg2": synth.cfg2_params}[args.workload]()
    s = synth.generate(prm, tets=True)
    free = synth.cfg1_params() if args.workload == "cfg1" else synth.cfg2_params()
    free.apply_bc = 0
    Lfull = synth.generate(free).Lval
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    solid = np.zeros(s.n_b, np.uint8)
    solid[s.tv[s.tsolid.astype(bool)].reshape(-1)] = 1
    ctx = scr.Context(0)
    a = scr.scr_assembler_create(ctx, dev(s.tv), dev(s.tp), dev(s.tsolid), dev(s.rp), dev(s.ci), dev(s.xyz),
                                 dev(s.mask), scr.tangent_params(**{k: getattr(prm, k) for k in (
                                     "rho_f", "mu_f", "rho_s", "E_s", "nu_s", "dt", "rho_inf", "terms",
                                     "vms_dt_coupling")}))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = scr.scr_stepper_create(ctx, a, dev(s.Lrp), dev(s.Lci), dev(s.Lval), dev(Lfull), dev(s.Lmask),
                                dev(s.blk_of_phys), dev(solid), dev(s.xyz.reshape(-1)), 1e-3,
                                amg=scr.amg_opts(precision=prec, **amg_overrides(args)))
    create_ms = 1e3 * (time.perf_counter() - t0)
    rows = []
    dts = [1e-3] * max(args.steps, 1) + [5e-4]
    for n, dt in enumerate(dts):
        f = dev(synth.rhs(3000 + n, 3 * s.n_b))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rc, gs = st.step(dt, f)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t1)
        row = dict(step=n, dt=dt, rc=rc, ms=round(ms, 1), **{k: gs[k] for k in (
            "correctors", "converged", "linear_its", "mesh_its", "resetups")}, res_ratio=gs["res"] / gs["res0"])
        log(f"[stepper] {row}", args)
        rows.append(row)
    st.destroy()
    a.destroy()
    ctx.destroy()
    plain = [r["ms"] for r in rows if not r["resetups"]]
    print(json.dumps({"metric": "predictor multi-corrector time steps per second (device scr_step)",
                      "value": round(1e3 / float(np.median(plain)), 4), "unit": "steps/s",
                      "config": {"workload": f"{args.workload} tube ({s.n_b:,} block rows, {s.n_tets:,} tetrahedra) "
                                             f"+ mesh motion ({s.n_phys:,} nodes)",
                                 "precision": args.precision or "fp64", "dt": "1e-3, then 5e-4"},
                      "create_ms": round(create_ms, 1), "rows": rows}))


def log(msg, args=None):
    if not (args and args.quiet):
        print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.kernel_table:
        kernel_table(*args.kernel_table)
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_bench(args)
        return
    if args.dt_sweep:
        dt_sweep(args)
        return
    if args.stepper:
        stepper_bench(args)
        return
    import torch
    import synth
    import paper_2206_06996_amd.scr as scr

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    t0 = time.time()
    if args.precision is None:
        args.precision = "mixed" if args.workload == "cfg4" else "both"
    prm = {"cfg1": synth.cfg1_params, "cfg2": synth.cfg2_params, "cfg4": synth.cfg4_params}[args.workload]()
    if args.flow:
        if args.workload != "cfg1":
            raise SystemExit("--flow runs on cfg1 only")
        prm.u_max = FLOW_U_MAX
    s = synth.generate(prm, tets=True)
    log(f"[bench] {args.workload} generated: n_b={s.n_b} nnzb={s.nnzb} nodes={s.n_phys} ({time.time() - t0:.1f}s)", args)
    if args.workload in ("cfg1", "cfg2"):
        sec = 2 * (prm.m_core + prm.n_bl + prm.n_wall) + 1
        workload = (f"{args.workload} unified fluid+solid tube {sec}x{sec}x{prm.nz + 1} ({s.n_phys:,} nodes, "
                    f"{s.n_b:,} block rows, {s.nnzb:,} 4x4 blocks) + mesh motion ({s.n_phys:,} x 3)")
        if args.flow:
            workload += (f"; advective Poiseuille state u_max = {FLOW_U_MAX:g} cm/s (Oseen VMS tangent, nonsymmetric A) "
                         f"and the outlet resistance coupling m = {FLOW_M:g} over {len(s.outlets[0][0])} outlet nodes")
    else:
        workload = (f"cfg4 Y-bifurcation, voxel mesh (parent R=1, daughters 0.7 at seeded angles, wall 1.2x; "
                    f"{s.n_phys:,} nodes, {s.n_b:,} block rows, {s.nnzb:,} 4x4 blocks) + mesh motion ({s.n_phys:,} x 3)")
    ref = None if (args.flow or args.precond != "scr") else load_reference(args.workload)
    if ref is not None and (ref["n_b"] != s.n_b or ref["nnzb"] != s.nnzb):
        ref = None
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    rp, ci, val, xyz = dev(s.rp), dev(s.ci), dev(s.val.reshape(-1)), dev(s.xyz.reshape(-1))
    Lrp, Lci, Lval = dev(s.Lrp), dev(s.Lci), dev(s.Lval)
    nsteps = args.warmup + args.steps
    B = [dev(synth.rhs(1000 + i, 4 * s.n_b, s.mask)) for i in range(nsteps)]
    BM = [dev(synth.rhs(2000 + i, 3 * s.n_phys, np.repeat(s.Lmask, 3))) for i in range(nsteps)]
    x = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
    xm = torch.zeros(3 * s.n_phys, dtype=torch.float64, device="cuda")
    ctx = scr.Context(0)
    if args.calibrate_copy:
        # three copies of 1 GiB (the counter calibration), then their rate: a plain stream on this card
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            torch.mul(src, 2.0, out=dst)
        e1.record()
        torch.cuda.synchronize()
        log(f"[bench] copy kernel: {2 * COPY_BYTES / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9:.0f} GB/s "
            f"(1 GiB read + 1 GiB written)", args)
        del src, dst
    precisions = {"both": ["fp64", "mixed"], "all": ["fp64", "mixed", "mixed32"]}.get(args.precision, [args.precision])
    pcode = {"fp64": scr.SCR_FP64, "mixed": scr.SCR_MIXED, "mixed32": scr.SCR_MIXED_FP32_INNER}
    results = {}
    x_first = {}
    for pi, prec in enumerate(precisions):
        ao = scr.amg_opts(precision=pcode[prec], schur_diag=1 if args.precond == "simplec" else 0, **amg_overrides(args))
        so = scr.solve_opts(precond=scr.SCR_PRECOND_SCR if args.precond == "scr" else scr.SCR_PRECOND_SIMPLE)
        hm = scr.amg_setup(ctx, scr.MESH_SYSTEM, Lrp, Lci, Lval, None, ao)
        # the first pass warms up W steps; the later passes one step (the device and the caches are warm)
        warm = args.warmup if pi == 0 else min(args.warmup, 1)
        lat, setup_ms, solve_ms, mesh_ms, destroy_ms, stats = [], [], [], [], [], []
        region = None
        for i in range(warm + args.steps):
            if i == warm:
                if not args.no_roofline:
                    ctx.profile(scr.SCR_PROF_SMOOTH_A0)
                    ctx.profile_read()
                torch.cuda.synchronize()
                region = time.perf_counter()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            h = scr.amg_setup(ctx, scr.SCR_SYSTEM, rp, ci, val, xyz, ao)
            if args.flow:
                scr.set_outlets(h, s.outlets, [FLOW_M])
            t1 = time.perf_counter()
            rc, st = scr.scr_solve(h, B[i], x, so)
            t2 = time.perf_counter()
            rcm, stm = scr.mesh_motion_solve(hm, BM[i], xm, so)
            t3 = time.perf_counter()
            h.destroy()
            torch.cuda.synchronize()
            te = time.perf_counter()
            if rc != 0 or rcm != 0:
                raise RuntimeError(f"step {i} {prec}: not converged (scr {rc}, mesh {rcm})")
            if i == 0:
                x_first[prec] = x.cpu().numpy()     # the reference right-hand side (seed 1000)
            if i >= warm:
                lat.append(te - ts); setup_ms.append((t1 - ts) * 1e3); solve_ms.append((t2 - t1) * 1e3)
                mesh_ms.append((t3 - t2) * 1e3); destroy_ms.append((te - t3) * 1e3)
                stats.append((st, stm))
            log(f"[bench] {prec} step {i}: setup {1e3 * (t1 - ts):.1f} ms solve {1e3 * (t2 - t1):.1f} ms "
                f"mesh {1e3 * (t3 - t2):.1f} ms free {1e3 * (te - t3):.1f} ms outer={st['outer_it']} its_A={st['its_A']} its_S={st['its_S']} "
                f"its_I={st['its_I']} vA={st['vcycles_A']} rel={st['rel_res_true']:.2e} mesh_its={stm['mesh_its']}",
                args)
        torch.cuda.synchronize()
        region = time.perf_counter() - region
        prof = None
        if not args.no_roofline:
            n, ms, by = ctx.profile_read()
            ctx.profile(scr.SCR_PROF_OFF)
            if n:
                prof = dict(launches=n, avg_us=1e3 * ms / n, bytes_per_launch=by / n, gbs=(by / n) / (ms / n * 1e-3) / 1e9)
        # numeric re-setup (outside the timed region): new values on the same pattern, aggregates kept
        h = scr.amg_setup(ctx, scr.SCR_SYSTEM, rp, ci, val, xyz, ao)
        upd_ms = []
        for _ in range(3):
            torch.cuda.synchronize()
            tu = time.perf_counter()
            scr.amg_update(h, rp, ci, val)
            upd_ms.append((time.perf_counter() - tu) * 1e3)
        peak = h.peak_bytes()
        fp = scr.footprint_estimate(scr.SCR_SYSTEM, s.n_b, s.nnzb, ao)
        if args.dump_levels and pi == 0:
            dump_levels(args.dump_levels, scr, h, hm, s, stats[0] if stats else None)
        h.destroy()
        log(f"[bench] {prec} amg_update: {' '.join(f'{v:.1f}' for v in upd_ms)} ms; handle peak {peak / 2**30:.2f} GiB, "
            f"footprint estimate {fp / 2**30:.2f} GiB", args)
        hm.destroy()
        results[prec] = dict(lat=lat, setup=setup_ms, solve=solve_ms, mesh=mesh_ms, destroy=destroy_ms, stats=stats, prof=prof,
                             region=region, update=upd_ms, warm=warm, peak=peak, footprint=fp)
    # device tangent assembly (outside the timed region): the same matrix from the tetrahedra
    asm_a = scr.scr_assembler_create(ctx, dev(s.tv), dev(s.tp), dev(s.tsolid), rp, ci, xyz, dev(s.mask),
                                     scr.tangent_params(**{k: getattr(prm, k) for k in (
                                         "rho_f", "mu_f", "rho_s", "E_s", "nu_s", "dt", "rho_inf", "terms",
                                         "vms_dt_coupling")}))
    u_adv = dev(s.uadv) if prm.u_max else None
    kval = torch.empty_like(val)
    asm_ms = []
    for _ in range(4):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        scr.scr_assemble_tangent(asm_a, u_adv, kval)
        asm_ms.append((time.perf_counter() - ta) * 1e3)
    asm_a.destroy()
    kdiff = float((kval - val).abs().max() / val.abs().max())
    del kval
    log(f"[bench] tangent assembly: {' '.join(f'{v:.2f}' for v in asm_ms)} ms, max |K_gpu - K| / max |K| = {kdiff:.1e}",
        args)
    main_prec = "fp64" if "fp64" in results else precisions[0]
    r = results[main_prec]
    total = r["region"]
    value = len(r["lat"]) / total
    out = {
        "metric": "SCR+AMG solves/s at 1e-8 rel. resid (FP64 vs mixed); p50/p99 solve latency",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / len(r["lat"]), 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32/f64",
        "data": "synthetic (seeded tube mesh, seeded RHS)",
        "config": {"workload": workload, "precision": main_prec, "tol": 1e-8, "precond": args.precond,
                   **({"amg": amg_overrides(args)} if args.amg else {})},
    }
    for prec, rr in results.items():
        lat = np.array(rr["lat"]) * 1e3
        st = [a for a, _ in rr["stats"]]
        out[prec] = {
            "solves_per_s": round(len(lat) / rr["region"], 4),
            "warmup_steps": rr["warm"],
            "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "setup_ms": round(float(np.median(rr["setup"])), 2),
            "resetup_ms": round(float(np.median(rr["update"])), 2),
            "scr_solve_ms": round(float(np.median(rr["solve"])), 2),
            "mesh_solve_ms": round(float(np.median(rr["mesh"])), 2),
            "handle_free_ms": round(float(np.median(rr["destroy"])), 2),
            "outer_it": int(np.median([a["outer_it"] for a in st])),
            "its_A": int(np.median([a["its_A"] for a in st])),
            "its_S": int(np.median([a["its_S"] for a in st])),
            "its_I": int(np.median([a["its_I"] for a in st])),
            "vcycles_A": int(np.median([a["vcycles_A"] for a in st])),
            "max_rel_res": float(max(a["rel_res_true"] for a in st)),
            "handle_peak_gib": round(rr["peak"] / 2**30, 3),
            "footprint_estimate_gib": round(rr["footprint"] / 2**30, 3),
        }
        if ref is not None:
            out[prec]["error_vs_oracle"] = field_errors_vs_reference(x_first[prec], ref)
        if rr["prof"]:
            out[prec]["smoother_l0_avg_us"] = round(rr["prof"]["avg_us"], 2)
            out[prec]["smoother_l0_GBps"] = round(rr["prof"]["gbs"], 1)
    if "fp64" in x_first and "mixed" in x_first:
        # velocity and pressure apart: the solution norm is dominated by the pressure
        xd, xm_ = x_first["fp64"].reshape(-1, 4), x_first["mixed"].reshape(-1, 4)
        out["mixed_vs_fp64_rel_diff"] = {
            "velocity": float(np.linalg.norm(xm_[:, :3] - xd[:, :3]) / np.linalg.norm(xd[:, :3])),
            "pressure": float(np.linalg.norm(xm_[:, 3] - xd[:, 3]) / np.linalg.norm(xd[:, 3]))}
    if ref is not None:
        out["oracle_reference"] = (f"oracle/{args.workload}_reference.json: the oracle's solution of the first step's "
                                   f"right-hand side refined to a {ref['tight_rel_res']:.1e} true residual; "
                                   f"error_vs_oracle = sampled relative error of each field (2,000 entries each)")
    out["assembly"] = {"ms": round(float(np.median(asm_ms[1:])), 3), "n_tets": int(s.n_tets),
                       "advective": bool(prm.u_max), "max_rel_diff_vs_input": kdiff}
    pr = r["prof"]
    if pr:
        traffic = pmc_traffic(args.workload) if (main_prec == "fp64" and not args.flow) else None
        out["roofline"] = {"bound": "hbm", "achieved": round(pr["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(pr["gbs"] / HBM_PEAK_GBS, 4),
                           "traffic": None if traffic is None else round(traffic / (pr["avg_us"] * 1e-6) / 1e9, 1),
                           "traffic_bytes_per_launch": traffic,
                           "kernel": ("smooth_rl3_k: fused Chebyshev step on level 0 of AMG(A) (3x3 %s blocks, "
                                      "block-row lanes)" % ("FP64" if main_prec == "fp64" else "FP32")),
                           "launches": pr["launches"], "avg_us": round(pr["avg_us"], 2),
                           "alg_bytes_per_launch": int(pr["bytes_per_launch"])}
    else:
        out["roofline"] = None
    out["cpu_baseline"] = None
    if not (args.no_cpu_baseline or ref is None or args.workload == "cfg4"):
        BM_host = synth.rhs(2000, 3 * s.n_phys, np.repeat(s.Lmask, 3))
        out["cpu_baseline"] = cpu_baseline(s, BM_host, args, ref)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
