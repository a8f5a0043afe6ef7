"""Benchmark: MGR-GMRES unknowns/s to a 1e-8 relative residual on one MI355X.

Workload (default): the 3D 128^3 NCP-shaped Jacobian (6,291,456 unknowns,
permeability contrast sigma = 2.0, 30 % two-phase cells in a seeded ball),
restart 30, tolerance 1e-8.  One step = one whole job from the CSR matrix
resident in HBM: mgr_setup (hierarchy built on the GPU) + mgr_solve.  The
FP64 form gives `value`; the mixed-precision form (FP32 hierarchy inside FP64
flexible GMRES) and the adjoint form (hierarchy on A^T + adjoint solve +
pattern scatter) are timed the same way and reported beside it.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MGR-GMRES unknowns/s to 1e-8 rel. residual, FP64 vs mixed; V-cycle % HBM peak"
HBM_PEAK_GBS = 8000.0
# Solver options after Section 6.2's phase-transition runs: non-injective R/P
# (eq. non_injective_rp) at every reduction, Jacobi F-relaxation at the first
# reduction, one AMG V(1,1)-cycle on A_FF at the second, AMG V(2,2) on the coarse
# grid.  Section 6.2 also puts an AMG V(1,1) at the last (constraint) reduction;
# here that F-block has a negative diagonal and only negative couplings, so its
# classical strength graph is empty and an AMG could not coarsen it: it keeps
# one Jacobi sweep.
SOLVER_OPTS = dict(frelax_amg_mask=2, frelax_amg_pre=1, frelax_amg_post=1)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_form(s, dev, form, steps, warmup, tol, timing=False):
    import numpy as np
    import torch

    from paper_1801_08464_amd.solver import MGRSolver

    rp = torch.as_tensor(s.indptr, device=dev)
    ci = torch.as_tensor(s.indices, device=dev)
    vals = torch.as_tensor(s.data, device=dev)
    lab = torch.as_tensor(s.labels, device=dev)
    if form == "adjoint":
        # dL/dx of L = sum of p over the observation cells
        g = np.zeros(s.n)
        g[3 * s.obs_cells] = 1.0
        rhs = torch.as_tensor(g, device=dev)
    else:
        rhs = torch.as_tensor(s.b, device=dev)
    kw = dict(precision="mixed" if form == "mixed" else "fp64", transpose=(form == "adjoint"), **SOLVER_OPTS)
    fwd_x = None
    if form == "adjoint":
        f = MGRSolver(rp, ci, vals, lab, **kw | dict(transpose=False))
        fwd_x, _ = f.solve(torch.as_tensor(s.b, device=dev), tol)
        f.close()

    def one_step(keep, timed):
        g = MGRSolver(rp, ci, vals, lab, **kw)
        if timed and timing:
            g.set_kernel_timing(True)
        x, info = g.solve(rhs, tol)
        if form == "adjoint":
            d = g.pattern_outer(x, fwd_x)
            keep.append(d)
        keep.append(g)
        return x, info

    for w in range(warmup):
        keep = []
        one_step(keep, False)
        torch.cuda.synchronize()
        for k in keep:
            if hasattr(k, "close"):
                k.close()
        log(f"{form}: warmup {w + 1}/{warmup} done")
    keep, infos = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        x, info = one_step(keep, True)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ktime = [k.kernel_time(0) for k in keep if hasattr(k, "kernel_time")] if timing else []
    vtime = [k.kernel_time(1) for k in keep if hasattr(k, "kernel_time")] if timing else []
    stime = [k.kernel_time(2) for k in keep if hasattr(k, "kernel_time")] if timing else []
    err = None
    x_host = None
    if form != "adjoint":
        xt = torch.as_tensor(s.x_true, device=dev)
        err = float(torch.linalg.norm(x - xt) / torch.linalg.norm(xt))
        x_host = x.cpu().numpy()
    for k in keep:
        if hasattr(k, "close"):
            k.close()
    del keep
    torch.cuda.empty_cache()
    info = infos[-1]
    log(f"{form}: {steps} steps in {dt:.3f}s, iterations {info.iterations}, rel_res {info.rel_residual:.2e}")
    out = dict(
        ms_per_step=1e3 * dt / steps,
        unknowns_per_s=s.n * steps / dt,
        setup_ms=info.setup_ms,
        solve_ms=info.solve_ms,
        solve_unknowns_per_s=s.n / (info.solve_ms * 1e-3),
        iterations=info.iterations,
        rel_residual=info.rel_residual,
        status=info.status,
        levels=info.level_n,
        level_nnz=info.level_nnz,
    )
    if err is not None:
        out["rel_error_vs_x_true"] = err
        out["_x"] = x_host
    def summary(rec):
        ms = sum(k[0] for k in rec)
        cnt = sum(k[1] for k in rec)
        byt = sum(k[2] for k in rec)
        return dict(total_ms=ms, launches=cnt, avg_us=1e3 * ms / max(cnt, 1), algorithmic_bytes=byt,
                    bytes_per_launch=byt / max(cnt, 1), achieved_GBs=byt / (ms * 1e-3) / 1e9 if ms > 0 else 0.0)

    if ktime:
        out["fine_kernel"] = summary(ktime)
    if stime:
        out["coarse_sweep"] = summary(stime)
    if vtime:
        v = summary(vtime)
        v["frac_of_hbm_peak"] = v["achieved_GBs"] / HBM_PEAK_GBS
        out["vcycle"] = v
    return out


FINE_RECORD = os.path.join(ROOT, "profiles", "k_csell_128cube_fp64_hbm_traffic.md")
FINE_SOURCE = os.path.join(ROOT, "paper_1801_08464_amd", "csrc", "k_fine.hip")
SWEEP_RECORD = os.path.join(ROOT, "profiles", "k_jag_stream_coarse_sweep_128cube_fp64_hbm_traffic.md")
SWEEP_SOURCE = os.path.join(ROOT, "paper_1801_08464_amd", "csrc", "k_solve.hip")


def measured_traffic(path, source, cfg):
    """HBM bytes per launch of a kernel from its rocprofv3 FETCH_SIZE and
    WRITE_SIZE record (calibrated against a plain copy), or None when the record
    is missing, is for another workload, or the kernel source has changed since."""
    import hashlib
    import re
    if not os.path.exists(path):
        return None, "no PMC record"
    txt = open(path).read()
    fields = dict(re.findall(r"^- (\w+): (\S+)", txt, re.M))
    src = hashlib.sha256(open(source, "rb").read()).hexdigest()
    if fields.get("source_sha256") != src:
        return None, "kernel changed since the PMC record"
    if fields.get("config") != str(cfg):
        return None, "PMC record is for another workload"
    return float(fields["hbm_bytes_per_launch"]), os.path.relpath(path, ROOT)


def roofline(rec, kernel, record, source, cfg):
    traffic, note = measured_traffic(record, source, cfg)
    return dict(bound="hbm", achieved=rec["achieved_GBs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=rec["achieved_GBs"] / HBM_PEAK_GBS, traffic=traffic, kernel=kernel, avg_us=rec["avg_us"],
                launches=rec["launches"], algorithmic_bytes_per_launch=rec["bytes_per_launch"],
                traffic_source=note)


def run_newton(dev, cfg, steps, warmup):
    """The semi-smooth Newton outer loop (Section 3.1) on the synthetic
    complementarity problem at config `cfg`'s grid, started from the solution of a
    smaller two-phase region (the previous state): one step = the whole Newton
    solve (residual, active set, Jacobian, MGR setup + solve per Newton step)."""
    import torch

    from paper_1801_08464_amd.newton import NCPNewton
    from synth import CONFIGS, make_ncp_problem
    p = CONFIGS[cfg]
    pr = make_ncp_problem(p["grid"], p["sigma"], p["region"], p["frac"], p["seed"])
    prev = make_ncp_problem(p["grid"], p["sigma"], p["region"], 0.8 * p["frac"], p["seed"])
    solver = NCPNewton(pr.l_indptr, pr.l_indices, pr.l_data, pr.henry, pr.f, device=dev)
    u0 = torch.as_tensor(prev.u_star, device=dev)
    for _ in range(warmup):
        solver.solve(u0=u0, **SOLVER_OPTS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = solver.solve(u0=u0, **SOLVER_OPTS)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    err = float(torch.linalg.norm(res.u - torch.as_tensor(pr.u_star, device=dev)) /
                torch.linalg.norm(torch.as_tensor(pr.u_star, device=dev)))
    log(f"newton: {len(res.steps) - 1} Newton steps, {dt * 1e3:.1f} ms per solve, error vs u* {err:.1e}")
    return dict(ms_per_step=1e3 * dt, unknowns_per_s=pr.n / dt, newton_steps=len(res.steps) - 1,
                converged=res.converged, rel_error_vs_u_star=err,
                linear_iterations=[s.lin_iterations for s in res.steps[1:]],
                values_only_updates=sum(1 for s in res.steps[1:] if s.values_only),
                active_cells=[s.nactive for s in res.steps],
                setup_ms=sum(s.setup_ms for s in res.steps), solve_ms=sum(s.solve_ms for s in res.steps),
                workload=f"config {cfg} grid {'x'.join(map(str, p['grid']))} ({pr.n} unknowns): semi-smooth Newton "
                         f"from the state of a two-phase region of {0.8 * p['frac']:.0%} to {p['frac']:.0%}; "
                         "step = the whole Newton solve")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def oracle_job(cfg, precision, out_prefix):
    """The oracle (plain C, one thread) on the benchmark's system, the whole job:
    setup, then GMRES to the tolerance.  Runs in a process of its own, started
    before the GPU forms; writes its timings and counts (JSON) and x (.npy)."""
    import numpy as np

    from oracle import oracle as O
    from synth import make_config
    s = make_config(cfg)
    A = O.as_csr(s.indptr, s.indices, s.data)
    log(f"oracle {precision}: n={s.n}, setup ...")
    t0 = time.perf_counter()
    o = O.Oracle(A, s.labels, precision=1 if precision == "fp32_apply" else 0, **SOLVER_OPTS)
    t1 = time.perf_counter()
    log(f"oracle {precision}: setup {t1 - t0:.1f} s, solving ...")
    r = o.solve(s.b, 1e-8)
    t2 = time.perf_counter()
    o.close()
    log(f"oracle {precision}: {r.iterations} iterations in {t2 - t1:.1f} s (status {r.status})")
    np.save(out_prefix + ".npy", r.x)
    with open(out_prefix + ".json", "w") as f:
        json.dump(dict(precision=precision, status=int(r.status), iterations=int(r.iterations),
                       rel_residual=float(r.rel_residual), setup_s=t1 - t0, solve_s=t2 - t1), f)


def start_oracle_jobs(cfg):
    import subprocess
    import tempfile
    tmp = tempfile.mkdtemp(prefix="mgr_bench_oracle_")
    jobs = {}
    for prec in ("fp64", "fp32_apply"):
        prefix = os.path.join(tmp, prec)
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-job", prec, "--config", str(cfg),
               "--oracle-out", prefix]
        jobs[prec] = (subprocess.Popen(cmd, env=dict(os.environ, OMP_NUM_THREADS="1")), prefix)
    return tmp, jobs


def finish_oracle_jobs(tmp, jobs):
    import shutil

    import numpy as np
    out = {}
    for prec, (proc, prefix) in jobs.items():
        rc = proc.wait()
        if rc != 0:
            raise RuntimeError(f"oracle job {prec} failed with status {rc}")
        with open(prefix + ".json") as f:
            rec = json.load(f)
        rec["x"] = np.load(prefix + ".npy")
        out[prec] = rec
    shutil.rmtree(tmp, ignore_errors=True)
    return out


def oracle_parity(s, dev, forms, orc):
    """Iterations against the oracle's (within one), and the solution error against
    the FP64 oracle's x: after exactly the oracle's number of iterations (tol = 0,
    the FP64 form) and, for information, of each form's own converged solve."""
    import numpy as np
    import torch

    from paper_1801_08464_amd.solver import MGRSolver
    xo = orc["fp64"]["x"]
    nxo = float(np.linalg.norm(xo))
    for form, key in (("fp64", "fp64"), ("mixed", "fp32_apply")):
        if form not in forms:
            continue
        f, rec = forms[form], orc[key]
        f["oracle"] = dict(mode="FP64" if key == "fp64" else "FP32 apply", iterations=rec["iterations"],
                           status=rec["status"], rel_residual=rec["rel_residual"])
        f["iterations_minus_oracle"] = f["iterations"] - rec["iterations"]
        f["converged_rel_error_vs_oracle"] = float(np.linalg.norm(f["_x"] - xo) / nxo)
    if "fp64" in forms:
        its = orc["fp64"]["iterations"]
        g = MGRSolver(torch.as_tensor(s.indptr, device=dev), torch.as_tensor(s.indices, device=dev),
                      torch.as_tensor(s.data, device=dev), torch.as_tensor(s.labels, device=dev),
                      max_iter=its, **SOLVER_OPTS)
        xm, im = g.solve(torch.as_tensor(s.b, device=dev), 0.0)
        g.close()
        err = float(np.linalg.norm(xm.cpu().numpy() - xo) / nxo)
        forms["fp64"]["rel_error_vs_oracle"] = err
        forms["fp64"]["rel_error_vs_oracle_mode"] = f"matched iterations ({im.iterations}, tol 0)"
        log(f"fp64: matched-iteration error vs the oracle {err:.2e} at {im.iterations} iterations")


def cpu_baseline(s, rec):
    """The oracle's whole job (setup + solve to 1e-8), measured on this host."""
    t = rec["setup_s"] + rec["solve_s"]
    return dict(value=s.n / t, unit="unknowns/s", cores=1, kind="oracle",
                sample=f"the whole oracle job on the same {'x'.join(map(str, s.grid))} system, measured (not "
                       f"scaled): setup {rec['setup_s']:.1f} s, then GMRES to 1e-8 in {rec['iterations']} iterations "
                       f"{rec['solve_s']:.1f} s, FP64, 1 thread (the FP32-apply oracle ran beside it in a process "
                       "of its own)",
                seconds=t, cpu=cpu_model())


# R/P and cycle variants of the MGR preconditioner (Section 4): each changes one
# choice of the default above
VARIANTS = {
    "default": {},
    "injective": dict(rp_type=1),                  # W_r = 0 (eq. injective_rp)
    "block_factorization": dict(rp_type=2),        # W_p = 0 (Section 4, last paragraph)
    "post_smoothing": dict(cycle_post=1),          # eq. MGR-post
    "f_sweeps_2": dict(f_sweeps=2),                # two F-relaxation sweeps per level
    "jacobi_frelax": dict(frelax_amg_mask=0),      # Jacobi F-relaxation at every level
}


def run_size_scaling(dev, configs, tol, forms_cfg, big_cfg):
    """Iterations and unknowns/s against problem size (the workloads of configs
    1-3, beside the main config's forms): each config's FP64 and mixed step with
    the benchmark's options, 2 timed steps after 1 warm-up."""
    from synth import CONFIGS, make_config
    rows = []
    for cfg in configs:
        s = make_config(cfg)
        for form in ("fp64", "mixed"):
            r = run_form(s, dev, form, 2, 1, tol)
            rows.append(dict(config=cfg, grid="x".join(map(str, CONFIGS[cfg]["grid"])), unknowns=s.n, form=form,
                             iterations=r["iterations"], ms_per_step=r["ms_per_step"], setup_ms=r["setup_ms"],
                             solve_ms=r["solve_ms"], unknowns_per_s=r["unknowns_per_s"]))
        del s
    for form in ("fp64", "mixed"):
        r = forms_cfg[form]
        rows.append(dict(config=big_cfg, grid="x".join(map(str, CONFIGS[big_cfg]["grid"])), unknowns=None, form=form,
                         iterations=r["iterations"], ms_per_step=r["ms_per_step"], setup_ms=r["setup_ms"],
                         solve_ms=r["solve_ms"], unknowns_per_s=r["unknowns_per_s"]))
    return rows


def run_variants(dev, configs, tol, warmup):
    import torch

    from paper_1801_08464_amd.solver import MGRSolver
    from synth import make_config
    rows = []
    for cfg in configs:
        s = make_config(cfg)
        rp, ci = torch.as_tensor(s.indptr, device=dev), torch.as_tensor(s.indices, device=dev)
        vals, lab = torch.as_tensor(s.data, device=dev), torch.as_tensor(s.labels, device=dev)
        b = torch.as_tensor(s.b, device=dev)
        for name, var in VARIANTS.items():
            for prec in ("fp64", "mixed"):
                opts = dict(SOLVER_OPTS) | var
                for w in range(warmup + 1):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    g = MGRSolver(rp, ci, vals, lab, precision=prec, **opts)
                    x, info = g.solve(b, tol)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    g.close()
                rows.append(dict(config=cfg, variant=name, precision=prec, options=var, status=info.status,
                                 iterations=info.iterations, rel_residual=info.rel_residual,
                                 setup_ms=info.setup_ms, solve_ms=info.solve_ms, step_ms=1e3 * dt,
                                 unknowns_per_s=s.n / dt))
                log(f"variant cfg {cfg} {name:20s} {prec:5s} status {info.status} its {info.iterations:4d} "
                    f"setup {info.setup_ms:7.1f} ms solve {info.solve_ms:8.1f} ms")
        del s, rp, ci, vals, lab, b
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--forms", default="fp64,mixed,adjoint,newton")
    ap.add_argument("--newton-config", type=int, default=3)
    ap.add_argument("--adjoint-config", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default=None,
                    help="comma-separated configs: time the R/P and cycle variants of the preconditioner "
                         "against the default on them (prints one JSON line with the table)")
    ap.add_argument("--oracle-job", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--oracle-out", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy kernel (calibrates FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.oracle_job:
        oracle_job(args.config, args.oracle_job, args.oracle_out)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from synth import CONFIGS, make_config
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.variants:
        cfgs = [int(c) for c in args.variants.split(",")]
        rows = run_variants(dev, cfgs, args.tol, args.warmup)
        print(json.dumps({"variants": rows, "tol": args.tol, "base_options": SOLVER_OPTS}))
        return
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # reads and writes exactly 512 MiB each
        torch.cuda.synchronize()
        del src, dst
    oracle_run = None
    if not args.no_cpu_baseline and "fp64" in args.forms.split(","):
        # the oracle's whole job runs on the host cores beside the GPU forms
        oracle_run = start_oracle_jobs(args.config)
    t = time.perf_counter()
    s = make_config(args.config)
    log(f"config {args.config}: n={s.n} nnz={s.nnz} generated in {time.perf_counter() - t:.1f}s")
    forms = {}
    for form in args.forms.split(","):
        if form == "adjoint":
            # the differentiable solve is specified on its own workload (48^3, 64 observation cells)
            s5 = make_config(args.adjoint_config)
            forms[form] = run_form(s5, dev, form, args.steps, args.warmup, args.tol)
            forms[form]["workload"] = f"config {args.adjoint_config}: {'x'.join(map(str, CONFIGS[args.adjoint_config]['grid']))} " \
                                      f"cells ({s5.n} unknowns); loss = sum of p over {len(s5.obs_cells)} cells; step = " \
                                      "setup on A^T + adjoint solve + pattern scatter"
            del s5
        elif form == "newton":
            forms[form] = run_newton(dev, args.newton_config, args.steps, args.warmup)
        else:
            forms[form] = run_form(s, dev, form, args.steps, args.warmup, args.tol, timing=True)
    main_form = forms.get("fp64") or next(iter(forms.values()))
    p = CONFIGS[args.config]
    fk = main_form.get("fine_kernel")
    cs = main_form.get("coarse_sweep")
    # the dominant kernel of a step: the l1-Jacobi sweep on the coarse-grid matrix
    # (three launches per iteration); the fine-level operator is reported beside it
    roof = roofline(cs, "k_jag_stream<double, int, 3, 4864>: l1-Jacobi sweep on the coarse-grid matrix "
                        "(AMG level 0 of the pressure system, row-block jagged copy)", SWEEP_RECORD, SWEEP_SOURCE,
                    args.config) if cs else None
    roof_fine = roofline(fk, "k_csell: level-0 sliced-ELL SpMV / residual (the GMRES operator)", FINE_RECORD,
                         FINE_SOURCE, args.config) if fk else None
    line = {
        "metric": METRIC,
        "value": main_form["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"config {args.config}: {'x'.join(map(str, p['grid']))} cells, 3 unknowns per cell "
                               f"({s.n} unknowns, {s.nnz} nonzeros), sigma {p['sigma']}, two-phase {p['frac']:.0%} "
                               f"{p['region']}; step = mgr_setup + mgr_solve to {args.tol:g}",
                   "restart": 30, "tol": args.tol, "seed": p["seed"]},
        "roofline": roof,
        "roofline_fine": roof_fine,
        "vcycle_hbm": {k: {"achieved_GBs": v["vcycle"]["achieved_GBs"], "frac": v["vcycle"]["frac_of_hbm_peak"],
                           "avg_us": v["vcycle"]["avg_us"], "bytes_per_apply": v["vcycle"]["bytes_per_launch"]}
                       for k, v in forms.items() if "vcycle" in v and k not in ("adjoint", "newton")},
        "forms": forms,
    }
    if "fp64" in forms and "mixed" in forms and args.config == 4:
        line["size_scaling"] = run_size_scaling(dev, (1, 2, 3), args.tol, forms, args.config)
        for r in line["size_scaling"]:
            if r["unknowns"] is None:
                r["unknowns"] = s.n
    if oracle_run is not None:
        log("waiting for the oracle ...")
        orc = finish_oracle_jobs(*oracle_run)
        oracle_parity(s, dev, forms, orc)
        line["cpu_baseline"] = cpu_baseline(s, orc["fp64"])
    for f in forms.values():
        f.pop("_x", None)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
