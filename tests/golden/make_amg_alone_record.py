"""Write tests/golden/oracle_amg_alone_cfg4.json: AMG alone (GMRES(30), right-
preconditioned by the AMG V(2,2) cycle, at most 400 iterations) on the reduced
pressure system A_3 of the benchmark workload's hierarchy (config 4, 128^3), with
a seeded N(0,1) right-hand side.  A record of why the MGR iteration count grows
between 64^3 and 128^3: the coarse-grid AMG alone does not reach 1e-8 there.
Calls only oracle/ and synth/; about five minutes and 8 GB of host memory.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

OPTS = dict(frelax_amg_mask=2, frelax_amg_pre=1, frelax_amg_post=1)
RHS_SEED = 7


def main():
    import numpy as np

    from oracle import oracle as O
    from synth import make_config
    s = make_config(4)
    o = O.Oracle(O.as_csr(s.indptr, s.indices, s.data), s.labels, **OPTS)
    A3 = o.amg_level(0)["A"]
    o.close()
    rhs = np.random.default_rng(RHS_SEED).standard_normal(A3.shape[0])
    t = time.perf_counter()
    r = O.Oracle(A3, np.zeros(A3.shape[0], np.int32), block_size=1, max_iter=400).solve(rhs, 1e-8)
    out = dict(config=4, options=OPTS, rhs_seed=RHS_SEED, rows=int(A3.shape[0]), nnz=int(A3.indices.shape[0]),
               max_iter=400, tol=1e-8, status=int(r.status), iterations=int(r.iterations),
               rel_residual=float(r.rel_residual), history_every_30=[float(v) for v in r.history[29::30]],
               host_solve_s=time.perf_counter() - t, input_sha256=s.fingerprint())
    path = os.path.join(HERE, "oracle_amg_alone_cfg4.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"status {r.status} iterations {r.iterations} rel_res {r.rel_residual:.3e}; wrote {path}")


if __name__ == "__main__":
    main()
