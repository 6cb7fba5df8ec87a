"""Full FP64 oracle run on the unified tube workload (41x41x179 nodes): writes
oracle/cfg1_reference.json with

  * the oracle's own operation counts and phase times for one corrector step at the default
    settings (delta = 1e-8; RHS seed 1000 of the benchmark), used to scale the bounded
    CPU-baseline sample of bench.py;
  * 2,000 sampled entries (seeded indices) of the oracle solution at delta = 1e-8, and of the
    same solution refined towards 1e-11 (at most 8 more outer iterations from the 1e-8 one; the
    residual reached is recorded: rounding sets a floor near 1e-12 on these systems);
  * 2,000 sampled entries of the mesh-motion solution at tol 1e-12 for seed 2000.

The JSON is written after the delta = 1e-8 phase and again at the end.  Calls only oracle/ and
the input generator.  Run: python oracle/reference_run.py  (about 35 min on one core).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(ROOT, "oracle", "cfg1_reference.json")


def _write(out):
    with open(OUT + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(OUT + ".tmp", OUT)


def main():
    s = synth.generate(synth.cfg1_params())
    b = synth.rhs(1000, 4 * s.n_b, s.mask)
    bm = synth.rhs(2000, 3 * s.n_phys, np.repeat(s.Lmask, 3))
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(4 * s.n_b, 2000, replace=False))
    idm = np.sort(rng.choice(3 * s.n_phys, 2000, replace=False))
    out = {"workload": "cfg1", "n_b": int(s.n_b), "nnzb": int(s.nnzb), "n_phys": int(s.n_phys),
           "rhs_seed": 1000, "mesh_rhs_seed": 2000, "x_sample_idx": idx.tolist(), "xm_sample_idx": idm.tolist()}
    t = time.time()
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    out["setup_s"] = time.time() - t
    print("setup", out["setup_s"], flush=True)
    t = time.time()
    m = oracle.Mesh(s.Lrp, s.Lci, s.Lval)
    out["mesh_setup_s"] = time.time() - t
    t = time.time()
    xm8, rcm, its, rel = m.solve(bm, tol=1e-8)
    out["mesh_solve_1e-8_s"] = time.time() - t
    out["mesh_its_1e-8"] = [int(v) for v in its]
    xm12, rcm, its12, rel12 = m.solve(bm, tol=1e-12)
    out["mesh_its_1e-12"] = [int(v) for v in its12]
    out["xm_norm"] = float(np.linalg.norm(xm12))
    out["xm_sample"] = xm12[idm].tolist()
    print("mesh", out["mesh_setup_s"], out["mesh_solve_1e-8_s"], its, its12, flush=True)
    t = time.time()
    x8, rc, st = o.solve(b, oracle.solve_opts(tol=1e-8))
    out["solve_1e-8_s"] = time.time() - t
    out["stats_1e-8"] = st
    out["x8_norm"] = float(np.linalg.norm(x8))
    out["x8_sample"] = x8[idx].tolist()
    print("solve 1e-8", out["solve_1e-8_s"], st, flush=True)
    _write(out)
    t = time.time()
    xt, rc, stt = o.solve(b, oracle.solve_opts(tol=1e-11, max_it=8), x0=x8)
    out["solve_tight_s"] = time.time() - t
    out["stats_tight"] = stt
    out["tight_rel_res"] = float(np.linalg.norm(b - oracle.bsr_spmv(s.rp, s.ci, s.val, xt)) / np.linalg.norm(b))
    out["xt_norm"] = float(np.linalg.norm(xt))
    out["xt_sample"] = xt[idx].tolist()
    print("solve tight", out["solve_tight_s"], stt, out["tight_rel_res"], flush=True)
    _write(out)
    print("written", flush=True)


if __name__ == "__main__":
    main()
