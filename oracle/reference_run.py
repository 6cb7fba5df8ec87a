"""Full FP64 oracle run on the unified tube workload (41x41x179 nodes): writes
oracle/cfg1_reference.json with

  * the oracle's own operation counts and phase times for one corrector step at the default
    settings (delta = 1e-8; RHS seed 1000 of the benchmark), used to scale the bounded
    CPU-baseline sample of bench.py;
  * 2,000 sampled entries (seeded indices) of the oracle solution at delta = 1e-12 for RHS
    seed 1000, and of the mesh-motion solution at tol 1e-12 for seed 2000, used by the
    full-size GPU parity test.

Calls only oracle/ and the input generator.  Run: python oracle/reference_run.py  (~20-30 min).
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


def main():
    s = synth.generate(synth.cfg1_params())
    b = synth.rhs(1000, 4 * s.n_b, s.mask)
    bm = synth.rhs(2000, 3 * s.n_phys, np.repeat(s.Lmask, 3))
    out = {"workload": "cfg1", "n_b": int(s.n_b), "nnzb": int(s.nnzb), "n_phys": int(s.n_phys),
           "rhs_seed": 1000, "mesh_rhs_seed": 2000}
    t = time.time()
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    out["setup_s"] = time.time() - t
    print("setup", out["setup_s"], flush=True)
    t = time.time()
    x8, rc, st = o.solve(b, oracle.solve_opts(tol=1e-8))
    out["solve_1e-8_s"] = time.time() - t
    out["stats_1e-8"] = st
    print("solve 1e-8", out["solve_1e-8_s"], st, flush=True)
    t = time.time()
    m = oracle.Mesh(s.Lrp, s.Lci, s.Lval)
    out["mesh_setup_s"] = time.time() - t
    t = time.time()
    xm8, rcm, its, rel = m.solve(bm, tol=1e-8)
    out["mesh_solve_1e-8_s"] = time.time() - t
    out["mesh_its_1e-8"] = [int(v) for v in its]
    print("mesh", out["mesh_setup_s"], out["mesh_solve_1e-8_s"], its, flush=True)
    # reference solutions for sampled parity
    x12, rc, st12 = o.solve(b, oracle.solve_opts(tol=1e-12), x0=x8)
    xm12, rcm, _, _ = m.solve(bm, tol=1e-12)
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(4 * s.n_b, 2000, replace=False))
    idm = np.sort(rng.choice(3 * s.n_phys, 2000, replace=False))
    out["stats_1e-12"] = st12
    out["x_norm"] = float(np.linalg.norm(x12))
    out["x_sample_idx"] = idx.tolist()
    out["x_sample"] = x12[idx].tolist()
    out["xm_norm"] = float(np.linalg.norm(xm12))
    out["xm_sample_idx"] = idm.tolist()
    out["xm_sample"] = xm12[idm].tolist()
    with open(os.path.join(ROOT, "oracle", "cfg1_reference.json"), "w") as f:
        json.dump(out, f)
    print("written", flush=True)


if __name__ == "__main__":
    main()
