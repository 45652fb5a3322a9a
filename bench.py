#!/usr/bin/env python3
"""Steady-state throughput benchmark on one MI355X.

Workload (default): the plain-FP64 batch of the 360,000-row operator -- N_c =
10, N_m = 60 (Hilbert dim 600), Delta = 1, g0 = 0.8, kappa = 0.4,
Gamma_m = 1e-3, n_th = 1, eight pump amplitudes E uniform in [0.1, 0.6]
(seeded); RCM, ILUT with drop tolerance 1e-6, GMRES(100) to a relative
residual of 1e-10.  One step is the whole method for the batch: device
assembly, RCM, ILUT factorisation, preconditioned GMRES and post-processing
(liouvillian_build -> rcm_permute -> ilu_factor -> gmres_solve -> rho).

Prints one JSON line: whole-job solves/s, the roofline of the dominant kernel
(the one with the largest total time: at this workload the device ILUT
factorisation, ahead of the triangular solves of the preconditioner) from HIP
events recorded on its launch stream over the timed region, and the oracle
timed on the host cores.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (description, params factory, opts)
    "batch360k": "N_c=10, N_m=60 (n=360,000), batch of 8 pump amplitudes, FP64, ILUT d=1e-6, GMRES(100), tol 1e-10; "
                 "one ILU factor (of the median-E item) preconditions the batch",
    "tiny1600": "N_c=4, N_m=10 (n=1,600), one solve, FP64, ILUT d=1e-5, GMRES(50), tol 1e-12",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name, fill):
    import workloads as W
    if name == "batch360k":
        opts = dict(drop_tol=W.BATCH_OPTS.drop_tol, fill_factor=fill or W.BATCH_OPTS.fill_factor,
                    m=W.BATCH_OPTS.restart, tol=W.BATCH_OPTS.tol, maxiter=W.BATCH_OPTS.maxiter,
                    share_factor=True)
        ps = W.batch_params()
        med = sorted(p.E for p in ps)[len(ps) // 2]
        ps.sort(key=lambda p: (abs(p.E - med), p.E))   # the shared factor is item 0's
        return ps, opts
    if name == "tiny1600":
        opts = dict(drop_tol=W.TINY_OPTS.drop_tol, fill_factor=fill or W.TINY_OPTS.fill_factor,
                    m=W.TINY_OPTS.restart, tol=W.TINY_OPTS.tol, maxiter=W.TINY_OPTS.maxiter)
        return [W.TINY], opts
    raise SystemExit(f"unknown workload {name}")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs, calibrated with a plain copy), or None
    when the summary is missing or the kernel source changed since."""
    import hashlib
    import re
    if kernel != "ilut":
        return None
    prof = os.path.join(ROOT, "profiles", "ilut_row_kernel_batch360k_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_1411_4356_amd", "csrc", "ilut_gpu.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m_t = re.search(r"ilut_traffic_bytes_per_launch:\s*(\d+)", text)
    m_s = re.search(r"ilut_source_sha256:\s*([0-9a-f]{64})", text)
    if not m_t or not m_s or m_s.group(1) != sha:
        return None
    return float(m_t.group(1))


def profile_query(lib, cls):
    launches, ms, nbytes = C.c_int64(), C.c_double(), C.c_double()
    lib.om_profile_query(cls.encode(), C.byref(launches), C.byref(ms), C.byref(nbytes))
    return launches.value, ms.value, nbytes.value


def matrix_free_comparison(P, lib, params, reps=50):
    """The product with the workload's permuted system matrix, stored (CSR
    SpMV) against matrix-free (stencil entries re-evaluated per row), on the
    same batch of vectors: HIP-event times and algorithmic bytes per launch,
    and the largest difference between the two results."""
    import torch
    A, _ = P.liouvillian_build(params)
    B, _, _ = P.rcm_permute(A)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.complex(torch.randn(B.batch * B.n, device="cuda", dtype=torch.float64, generator=g),
                      torch.randn(B.batch * B.n, device="cuda", dtype=torch.float64, generator=g))
    y0 = P.csr_spmv(B, x)
    y1 = P.liouvillian_apply(B, x)
    torch.cuda.synchronize()
    diff = float((y1 - y0).abs().max() / y0.abs().max())
    res = {}
    for cls, fn in (("spmv", lambda: P.csr_spmv(B, x, y0)), ("lapply", lambda: P.liouvillian_apply(B, x, y1))):
        torch.cuda.synchronize()
        lib.om_profile_enable(1)
        lib.om_profile_reset()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        lib.om_profile_enable(0)
        n, ms, nb = profile_query(lib, cls)
        res[cls] = {"avg_ms": ms / n, "GB/s": (nb / n) / (ms / n * 1e-3) / 1e9, "algorithmic_bytes": nb / n,
                    "launches": n}
    return {"csr_spmv": res["spmv"], "matrix_free": res["lapply"],
            "speedup": res["spmv"]["avg_ms"] / res["lapply"]["avg_ms"],
            "max_rel_diff": diff,
            "note": "one product of the batch with the RCM-permuted constrained matrix (complex128); bytes are "
                    "algorithmic: CSR nnz*20 + 4(n+1) + 32n per item, matrix-free 32n per item + 8n for the "
                    "permutation"}


def _oracle_solve_one(p, q):
    """Child process: the oracle's direct solve of one batch item."""
    import time as _t

    import numpy as np

    from oracle import direct, model
    t0 = _t.perf_counter()
    L = model.liouvillian(p)
    Lt, b, _ = model.constrained_system(L)
    x = direct.solve(Lt, b)
    q.put((_t.perf_counter() - t0, bool(np.isfinite(x).all())))


def cpu_baseline(params, opts, budget_s):
    """The oracle (Kronecker build + direct sparse LU of the constrained
    system, complex128, scipy/SuperLU) on the host, on batch items one after
    another until the budget is spent.  If not even one item finishes within
    the budget the reported value is an upper bound (1 / budget)."""
    import multiprocessing as mp

    # both oracle paths (dense LAPACK for small systems, SuperLU's supernodal
    # LU otherwise) run their dense kernels on the BLAS thread pool
    from oracle import direct as _direct
    how = "Kronecker build + scipy sparse LU (COLAMD, SuperLU)"
    if params[0].n <= _direct.DENSE_LIMIT:
        how = "Kronecker build + dense LU (LAPACK)"
    threads = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        pass
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    done = 0
    for p in params:
        left = budget_s - (time.perf_counter() - t0)
        if left <= 0:
            break
        q = ctx.Queue()
        proc = ctx.Process(target=_oracle_solve_one, args=(p, q))
        proc.start()
        proc.join(timeout=left)
        if proc.is_alive():
            proc.kill()
            proc.join()
            break
        dt, ok = q.get()
        if not ok:
            break
        done += 1
    dt = time.perf_counter() - t0
    if done == 0:
        return {"value": 1.0 / budget_s, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
                "bound": "upper",
                "sample": f"batch item 0 (n={params[0].n}): {how} did not finish "
                          f"within {budget_s:.0f} s; value is the upper bound 1/{budget_s:.0f} s"}
    return {"value": done / dt, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} of {len(params)} batch items (n={params[0].n}): {how} of the constrained system, "
                      f"{dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="batch360k", choices=sorted(WORKLOADS))
    ap.add_argument("--fill", type=float, default=None, help="ILUT fill limit p (default: workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison step")
    ap.add_argument("--no-matrix-free", action="store_true",
                    help="skip the comparison of the matrix-free product with the CSR SpMV")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--quiet", action="store_true", help="no library progress lines on stderr")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three plain device copies of 1 GiB (the reference dispatches that scale the "
                         "FETCH_SIZE / WRITE_SIZE byte counters) and exit")
    args = ap.parse_args()
    if not args.quiet:
        os.environ["OMSS_VERBOSE"] = "1"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (there is no multi-GPU "
              "path; the batch items would shard one or more per GPU).", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        a = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copied 3 x 1 GiB")
        return

    import paper_1411_4356_amd as P
    lib = P.lib()
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    torch.cuda.set_device(0)
    params, opts = make_workload(args.workload, args.fill)
    batch = len(params)
    log(f"workload {args.workload}: {WORKLOADS[args.workload]}; fill p = {opts['fill_factor']}; "
        f"E = {[round(p.E, 6) for p in params]}")

    def step():
        rho, info, res = P.steady_state(params, **opts)
        return info, res

    for w in range(args.warmup):
        info, _ = step()
        log(f"warmup {w}: {json.dumps(info['gmres'])}")
    torch.cuda.synchronize()
    lib.om_profile_enable(1)
    lib.om_profile_reset()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        info, res = step()
        infos.append((info, res))
        log(f"step {k}: build {info['t_build_s']:.3f}s rcm {info['t_rcm_s']:.3f}s factor {info['t_factor_s']:.3f}s "
            f"solve {info['t_solve_s']:.3f}s post {info['t_post_s']:.3f}s iters {info['gmres']['iters']} "
            f"relres {info['gmres']['relres_true']:.2e} fill {info['ilu']['fill']:.1f}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.om_profile_enable(0)
    elapsed = t1 - t0
    value = batch * args.steps / elapsed

    # kernel classes timed with HIP events on their launch streams; bytes are
    # algorithmic (what the operation must move), not measured traffic
    names = {"ilut": "ilut_row_kernel (device ILUT factorisation, one launch per factor)",
             "trsv": "trsv_coop_kernel (ILU apply, one triangular solve of the batch per launch)",
             "spmv": "spmv_kernel (CSR SpMV, batch)",
             "orth": "mdot/update kernels (CGS2 orthogonalisation)"}
    q = {k: profile_query(lib, k) for k in names}

    def rate(qq):
        n, ms, b = qq
        if n == 0 or ms <= 0:
            return None, None
        return (b / n) / ((ms / n) * 1e-3) / 1e9, ms / n

    dom = max(("ilut", "trsv"), key=lambda k: q[k][1])
    dom_gbs, dom_ms = rate(q[dom])
    solve_s = sum(i["t_solve_s"] for i, _ in infos) / len(infos)
    factor_s = sum(i["t_factor_s"] for i, _ in infos) / len(infos)
    last, lres = infos[-1]
    out = {
        "metric": "steady-state solves/s (whole method: build+RCM+ILUT+GMRES), FP64, 1e-10 relative residual",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "batch": batch,
                   "n": int(params[0].n), "drop_tol": opts["drop_tol"],
                   "fill_factor": opts["fill_factor"], "restart": opts["m"], "tol": opts["tol"]},
        "roofline": {"bound": "hbm", "kernel": names[dom],
                     "achieved": dom_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (dom_gbs / HBM_PEAK_GBS) if dom_gbs else None,
                     "traffic": measured_traffic(dom) if args.workload == "batch360k" and args.fill is None else None,
                     "avg_launch_ms": dom_ms, "launches": q[dom][0],
                     "algorithmic_bytes_per_launch": (q[dom][2] / q[dom][0]) if q[dom][0] else None},
        "kernels": {k: {"GB/s": rate(q[k])[0], "avg_ms": rate(q[k])[1], "launches": q[k][0],
                        "total_s": q[k][1] * 1e-3} for k in names},
        "phases_s": {k: last[k] for k in ("t_build_s", "t_rcm_s", "t_factor_s", "t_solve_s", "t_post_s")},
        "solve_phase_solves_per_s": batch / solve_s,
        "gmres": last["gmres"],
        "ilu": last["ilu"],
        "order": last["order"],
        "max_relres": float(max(lres["relres"])),
    }
    if not args.no_matrix_free:
        out["matrix_free_apply"] = matrix_free_comparison(P, lib, params)
    if not args.no_mixed:
        # the same step with complex64 SpMV and ILU application inside an FP64
        # GMRES-IR outer loop, to the same 1e-10 true relative residual
        log("mixed precision (GMRES-IR, complex64 inner solves) on the same workload")
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        _, minfo, mres = P.steady_state(params, precision="ir_c64", **opts)
        torch.cuda.synchronize()
        tm = time.perf_counter() - tm0
        log(f"mixed: factor {minfo['t_factor_s']:.3f}s solve {minfo['t_solve_s']:.3f}s outer "
            f"{minfo['gmres']['outer_iters']} iters {minfo['gmres']['iters']} relres {minfo['gmres']['relres_true']:.2e}")
        out["mixed_ir_c64"] = {
            "value": batch / tm, "unit": "solves/s", "ms_per_step": tm * 1e3,
            "t_factor_s": minfo["t_factor_s"], "t_solve_s": minfo["t_solve_s"],
            "solve_speedup_vs_fp64": solve_s / minfo["t_solve_s"] if minfo["t_solve_s"] > 0 else None,
            "outer_iters": minfo["gmres"]["outer_iters"], "inner_iters": minfo["gmres"]["iters"],
            "relres_true": minfo["gmres"]["relres_true"], "max_relres": float(max(mres["relres"])),
            "note": "same workload and factor arithmetic; the factor's schedules are also stored in complex64, "
                    "the residual, Hessenberg/Givens and normalisation stay FP64"}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(params, opts, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
