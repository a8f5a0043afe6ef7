"""Write the oracle's converged solves of the benchmark workload (config 4:
128^3 cells, 6,291,456 unknowns) to tests/golden/oracle_solve_cfg4.json.

The oracle needs minutes per solve at this size (about 11 s of setup and
196 GMRES iterations), too long for a test run, so its results are stored here
once: per precision (FP64, and the FP32-apply mode that the mixed GPU form is
compared with) the iteration count, status, final relative residual, residual
history, hierarchy sizes, and the solution x as ||x||_2, eight projections
<w_k, x> on seeded N(0,1) vectors w_k, and x itself at 4,096 seeded indices.
A fingerprint of the generated inputs (CSR, labels, b) lets the GPU test check
that it regenerated the same system.  Calls only oracle/ and synth/.

Usage: python tests/golden/make_oracle_solutions.py  (both precisions run in
parallel, one process each; about 3 minutes and 10 GB of host memory).
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

CONFIG = 4
# the solver options of the benchmark: AMG V(1,1) F-relaxation at MGR level 1
OPTS = dict(frelax_amg_mask=2, frelax_amg_pre=1, frelax_amg_post=1)
TOL = 1e-8
N_SAMPLE = 4096
N_PROJ = 8
SAMPLE_SEED = 4096
PROJ_SEED0 = 1000
OUT = os.path.join(HERE, f"oracle_solve_cfg{CONFIG}.json")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def solve_one(precision):
    import numpy as np

    from oracle import oracle as O
    from synth import make_config, random_vector
    s = make_config(CONFIG)
    A = O.as_csr(s.indptr, s.indices, s.data)
    t0 = time.perf_counter()
    o = O.Oracle(A, s.labels, precision=precision, **OPTS)
    t1 = time.perf_counter()
    r = o.solve(s.b, TOL)
    t2 = time.perf_counter()
    o.close()
    x = r.x
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(s.n, N_SAMPLE, replace=False))
    proj = [float(np.dot(random_vector(s.n, PROJ_SEED0 + k), x)) for k in range(N_PROJ)]
    return dict(precision="fp64" if precision == 0 else "fp32_apply", status=int(r.status),
                iterations=int(r.iterations), rel_residual=float(r.rel_residual),
                history=[float(v) for v in r.history], level_n=[int(v) for v in r.level_n],
                level_nnz=[int(v) for v in r.level_nnz], x_norm=float(np.linalg.norm(x)), projections=proj,
                sample_index=[int(i) for i in idx], x_sample=[float(v) for v in x[idx]],
                rel_error_vs_x_true=float(np.linalg.norm(x - s.x_true) / np.linalg.norm(s.x_true)),
                host_setup_s=t1 - t0, host_solve_s=t2 - t1)


def main():
    from synth import CONFIGS, make_config
    s = make_config(CONFIG)
    fp = s.fingerprint()
    del s
    with mp.get_context("spawn").Pool(2) as pool:
        res = pool.map(solve_one, [0, 1])
    out = dict(config=CONFIG, workload=CONFIGS[CONFIG], options=OPTS, tol=TOL, input_sha256=fp,
               n_projections=N_PROJ, projection_seed0=PROJ_SEED0, sample_seed=SAMPLE_SEED,
               host_cpu=cpu_model(), host_threads_per_solve=1, fp64=res[0], fp32_apply=res[1])
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    for r in res:
        print(f"{r['precision']}: status {r['status']} iterations {r['iterations']} rel_res {r['rel_residual']:.3e} "
              f"setup {r['host_setup_s']:.1f} s solve {r['host_solve_s']:.1f} s")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
