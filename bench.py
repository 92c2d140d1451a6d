"""Benchmark of the Lindblad master-equation / quantum-jump hot path on one MI355X.

Headline workload (one "step" = one full adaptive solve): the dissipative transverse-field Ising
chain, L = 8 (d = 256, Liouvillian 65,536 x 65,536 with 1,245,183 non-zeros), J = 1, h = 0.7,
gamma = 0.2, all spins up, t in [0, 10], <sigma_z^i> at 100 times, solved by the mixed-precision
CSR path (complex64 SpMV and stages, FP64 step control / error norm / trace / expectations) at the
loosest tolerance whose result stays within 1e-4 of a tight FP64 oracle solution.
``value`` = Liouvillian right-hand-side evaluations per second over the timed solves.

The same JSON line carries: the FP64 single-solve path on the same problem, the roofline of the
fused SpMV-stage kernel (live, HIP events) at this size and at an HBM-sized Liouvillian (L = 10),
the 512-cavity dense parameter sweep on the matrix cores (batched solves/s, TFLOP/s), the
quantum-jump ensemble (trajectories/s), the served request stream (p50/p99 latency), and the FP64
CPU oracle timed on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-extra] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
import paper_2504_21440_amd as qt  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_MATRIX_PEAK_TFLOPS = 157.3
METRIC = "Lindblad RHS evals/s + batched solves/s at 1e-4 error vs FP64; p50/p99 latency"
LADDER = [1e-4, 3e-5, 1e-5, 3e-6, 1e-6]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def sz_ops(L):
    import scipy.sparse as sp
    ops = []
    for i in range(L):
        diag = np.array([1.0 if ((s >> (L - 1 - i)) & 1) == 0 else -1.0 for s in range(2 ** L)])
        ops.append(sp.diags(diag.astype(complex), 0, format="csr"))
    return ops


def up_ket(L):
    v = np.zeros(2 ** L, complex)
    v[0] = 1
    return v


def load_golden(name):
    with open(os.path.join(ROOT, "tests", "golden", name + ".json")) as f:
        g = json.load(f)
    return np.array(g["expect_re"]) + 1j * np.array(g["expect_im"])


def spmv_bytes(n, nnz, val_bytes):
    """Algorithmic HBM bytes of one CSR SpMV: values + column indices, row pointers, x read, y write."""
    return nnz * (val_bytes + 4) + (n + 1) * 4 + 2 * n * val_bytes


def calibrate(ctx, L_obj, p, prec, ref, tol=1e-4):
    """Loosest rtol in the ladder (atol = rtol/100) whose solution is within tol of the tight reference."""
    tl = workloads.tlist(p["t_end"], p["nt"])
    chosen = None
    for rt in LADDER:
        ex, st, _ = qt.mesolve(ctx, L_obj, up_ket(p["L"]), tl, sz_ops(p["L"]),
                               options=qt.opts(abstol=rt / 100, reltol=rt, precision=prec))
        err = float(np.abs(ex - ref).max())
        log(f"  calibrate prec={prec} rtol={rt:g}: err={err:.2e} steps={st['n_accept']}")
        if err <= tol:
            chosen = (rt, err)
            break
    return chosen


def time_plan(plan, steps, warmup):
    for _ in range(warmup):
        plan.run()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run()
    dt = time.perf_counter() - t0
    return dt


def section_ising(ctx, steps, warmup):
    p = workloads.ising_single()
    H, cs = qt.model_ising(p["L"], p["J"], p["h"], p["gamma"])
    ref = load_golden("ising_l8_tight")
    tl = workloads.tlist(p["t_end"], p["nt"])
    out = {}
    for name, prec in [("mixed", qt.MIXED), ("fp64", qt.F64)]:
        Lo = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, prec)
        d, nnz, nbytes = Lo.info()
        cal = calibrate(ctx, Lo, p, prec, ref)
        rt, err = cal if cal else (1e-6, float("nan"))
        o = qt.opts(abstol=rt / 100, reltol=rt, precision=prec)
        plan = qt.MePlan(ctx, [(Lo, up_ket(p["L"]), tl, sz_ops(p["L"]))], o)
        dt = time_plan(plan, steps, warmup)
        ex, st, _ = plan.result(0)
        err = float(np.abs(ex - ref).max())
        n_rhs = st["n_rhs"]
        ms_stage = plan.time_rhs(reps=200)
        n = d * d
        vb = 8 if prec == qt.MIXED else 16
        b = spmv_bytes(n, nnz, vb)
        out[name] = {"rtol": rt, "atol": rt / 100, "max_err_vs_tight_fp64": err, "n_accept": st["n_accept"],
                     "n_reject": st["n_reject"], "n_rhs": n_rhs, "ms_per_solve": 1e3 * dt / steps,
                     "solves_per_s": steps / dt, "rhs_per_s": n_rhs * steps / dt,
                     "stage_kernel_ms": ms_stage, "spmv_bytes": b, "stage_kernel_GBs": b / (ms_stage * 1e-3) / 1e9,
                     "nnz": nnz, "n": n}
        log(f"ising L=8 {name}: {out[name]}")
        plan.close()
        Lo.close()
    return out


def section_hbm_spmv(ctx):
    """Fused SpMV-stage kernel on an HBM-sized Liouvillian (L = 10: 1,048,576 rows, 24.6 M nnz)."""
    out = {}
    H, cs = qt.model_ising(10, 1.0, 1.0, 0.1)
    tl = np.linspace(0, 0.1, 2)
    for name, prec, vb in [("mixed", qt.MIXED, 8), ("fp64", qt.F64, 16)]:
        Lo = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, prec)
        d, nnz, _ = Lo.info()
        plan = qt.MePlan(ctx, [(Lo, up_ket(10), tl, [])], qt.opts(precision=prec))
        ms = plan.time_rhs(reps=50)
        n = d * d
        b = spmv_bytes(n, nnz, vb)
        gbs = b / (ms * 1e-3) / 1e9
        out[name] = {"n": n, "nnz": nnz, "bytes_per_launch": b, "ms_per_launch": ms, "GBs": gbs,
                     "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
        log(f"HBM SpMV L=10 {name}: {out[name]}")
        plan.close()
        Lo.close()
    return out


def section_sweep(ctx, n=512, check=12):
    """512 driven Kerr cavities, N ~ U{10..80}, dense MFMA form, mixed precision, one launch set."""
    sweep = workloads.kerr_sweep(n=n)
    probs = []
    Ls = []
    for p in sweep:
        H, c = qt.model_kerr(p["N"], p["delta"], p["U"], p["F"], p["kappa"])
        Lo = qt.Liouvillian(ctx, H, c, qt.FORM_DENSE, qt.MIXED)
        Ls.append(Lo)
        rho0 = np.zeros((p["N"], p["N"]), complex)
        rho0[0, 0] = 1
        num = np.diag(np.arange(p["N"], dtype=float)).astype(complex)
        probs.append((Lo, rho0, workloads.tlist(p["t_end"], p["nt"]), [num]))
    o = qt.opts(abstol=1e-7, reltol=1e-5, precision=qt.MIXED)
    plan = qt.MePlan(ctx, probs, o)
    plan.run()
    t0 = time.perf_counter()
    plan.run()
    dt = time.perf_counter() - t0
    n_rhs = 0
    flops = 0.0
    res = []
    for i, p in enumerate(sweep):
        ex, st, _ = plan.result(i)
        res.append(ex)
        n_rhs += st["n_rhs"]
        flops += st["n_rhs"] * 24.0 * p["N"] ** 3
    kern_ms = plan.time_rhs(reps=1)
    out = {"instances": n, "solves_per_s": n / dt, "ms_per_batch": dt * 1e3, "rhs_per_s": n_rhs / dt,
           "dense_kernel_ms": kern_ms, "algorithmic_TFLOPs": flops / (kern_ms * 1e-3) / 1e12,
           "frac_of_fp32_matrix_peak": flops / (kern_ms * 1e-3) / 1e12 / FP32_MATRIX_PEAK_TFLOPS,
           "rtol": o.reltol, "atol": o.abstol}
    plan.close()
    return out, sweep, res


def cpu_oracle_baseline():
    import oracle
    from oracle import models as om
    p = workloads.ising_single()
    H, cs = om.ising(p["L"], p["J"], p["h"], p["gamma"])
    tl = workloads.tlist(p["t_end"], p["nt"])
    e_ops = [om.site_op(p["L"], i, om.sigmaz()) for i in range(p["L"])]
    t0 = time.perf_counter()
    ex, st, rc, _ = oracle.mesolve(H, cs, om.all_up_ket(p["L"]), tl, e_ops)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": st["n_rhs"] / dt, "unit": "RHS evals/s", "cores": threads, "kind": "oracle",
            "sample": f"one full FP64 solve of the L=8 chain (abstol 1e-8, reltol 1e-6): {st['n_rhs']} RHS in "
                      f"{dt:.1f} s", "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--skip-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (trajectories, sweep "
              "instances and served requests would shard by count across GPUs with one final FP64 "
              "all-reduce; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    log("context")
    ctx = qt.Context(0)
    ising = section_ising(ctx, args.steps, args.warmup)
    mixed = ising["mixed"]
    extra = {}
    if not args.skip_extra:
        log("hbm spmv")
        extra["spmv_hbm_L10"] = section_hbm_spmv(ctx)
        log("sweep")
        extra["kerr_sweep_512"], _, _ = section_sweep(ctx)
    rl = {"bound": "hbm", "achieved": mixed["stage_kernel_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
          "frac": mixed["stage_kernel_GBs"] / HBM_PEAK_GBS, "traffic": None,
          "kernel": "k_csr_stage<float,8,3> (fused SpMV + stage epilogue), L=8 Liouvillian (MALL-resident)"}
    line = {
        "metric": METRIC, "value": mixed["rhs_per_s"], "unit": "RHS evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mixed["ms_per_solve"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "dissipative TFIM chain L=8 mesolve, mixed precision, accuracy-matched to 1e-4",
                   "L": 8, "d": 256, "n": mixed["n"], "nnz": mixed["nnz"], "t_end": 10.0, "n_t": 100,
                   "rtol": mixed["rtol"], "atol": mixed["atol"], "parallelism": "single GPU"},
        "solves_per_s": mixed["solves_per_s"], "max_err_vs_fp64": mixed["max_err_vs_tight_fp64"],
        "fp64_single_solve": ising["fp64"], "mixed_detail": mixed,
        "roofline": rl,
    }
    line.update(extra)
    if not args.no_cpu:
        log("cpu oracle baseline")
        line["cpu_baseline"] = cpu_oracle_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
