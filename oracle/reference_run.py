"""Full FP64 oracle run on a tube workload: writes oracle/<workload>_reference.json with

  * the oracle's own operation counts and phase times for one corrector step at the default
    settings (delta = 1e-8; RHS seed 1000 of the benchmark), used to scale the bounded
    CPU-baseline sample of bench.py;
  * sampled entries (seeded indices: 2,000 velocity and 2,000 pressure unknowns) of the oracle
    solution at delta = 1e-8, and of the same solution refined towards 1e-11 (at most 8 more outer
    iterations from the 1e-8 one; the residual reached is recorded: rounding sets a floor near
    1e-12 on these systems), with the velocity and pressure norms of both solutions;
  * 2,000 sampled entries of the mesh-motion solution at tol 1e-12 for seed 2000.

The JSON is written after each phase.  Calls only oracle/ and the input generator.  Threads:
OMP_NUM_THREADS (the results do not depend on it).
Run: python oracle/reference_run.py cfg1   (about 10 min on 8 cores; cfg2 about 2 h)
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


def _fields(x):
    x4 = x.reshape(-1, 4)
    return float(np.linalg.norm(x4[:, :3])), float(np.linalg.norm(x4[:, 3]))


def main(workload):
    out_path = os.path.join(ROOT, "oracle", f"{workload}_reference.json")

    def write(out):
        with open(out_path + ".tmp", "w") as f:
            json.dump(out, f)
        os.replace(out_path + ".tmp", out_path)

    prm = {"cfg1": synth.cfg1_params, "cfg2": synth.cfg2_params}[workload]()
    s = synth.generate(prm)
    b = synth.rhs(1000, 4 * s.n_b, s.mask)
    bm = synth.rhs(2000, 3 * s.n_phys, np.repeat(s.Lmask, 3))
    rng = np.random.default_rng(12345)
    nodes = rng.choice(s.n_b, 2000, replace=False)
    comps = rng.integers(0, 3, 2000)
    idx_v = np.sort(4 * nodes + comps)
    idx_p = np.sort(4 * rng.choice(s.n_b, 2000, replace=False) + 3)
    idm = np.sort(rng.choice(3 * s.n_phys, 2000, replace=False))
    out = {"workload": workload, "n_b": int(s.n_b), "nnzb": int(s.nnzb), "n_phys": int(s.n_phys),
           "omp_threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
           "rhs_seed": 1000, "mesh_rhs_seed": 2000, "xv_sample_idx": idx_v.tolist(), "xp_sample_idx": idx_p.tolist(),
           "xm_sample_idx": idm.tolist()}
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
    write(out)
    t = time.time()
    x8, rc, st = o.solve(b, oracle.solve_opts(tol=1e-8))
    out["solve_1e-8_s"] = time.time() - t
    out["stats_1e-8"] = st
    out["x8_norm_v"], out["x8_norm_p"] = _fields(x8)
    out["x8v_sample"] = x8[idx_v].tolist()
    out["x8p_sample"] = x8[idx_p].tolist()
    print("solve 1e-8", out["solve_1e-8_s"], st, flush=True)
    write(out)
    t = time.time()
    xt, rc, stt = o.solve(b, oracle.solve_opts(tol=1e-11, max_it=8), x0=x8)
    out["solve_tight_s"] = time.time() - t
    out["stats_tight"] = stt
    out["tight_rel_res"] = float(np.linalg.norm(b - oracle.bsr_spmv(s.rp, s.ci, s.val, xt)) / np.linalg.norm(b))
    out["xt_norm_v"], out["xt_norm_p"] = _fields(xt)
    out["xtv_sample"] = xt[idx_v].tolist()
    out["xtp_sample"] = xt[idx_p].tolist()
    # how far the 1e-8 solution is from the refined one, per field (over the whole vectors)
    d = (x8 - xt).reshape(-1, 4)
    out["x8_vs_xt_rel"] = {"velocity": float(np.linalg.norm(d[:, :3]) / out["xt_norm_v"]),
                           "pressure": float(np.linalg.norm(d[:, 3]) / out["xt_norm_p"])}
    print("solve tight", out["solve_tight_s"], stt, out["tight_rel_res"], out["x8_vs_xt_rel"], flush=True)
    write(out)
    print("written", out_path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "cfg1")
