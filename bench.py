"""Benchmark: ROR-BK time to relative residual 1e-8 on one MI355X.

Workload: dense tall least-squares A 100000 x 2000 (U diag(s) V^T, s log-spaced
1..1e-8, cond 1e8), consistent b = A x_star, blocks of 64 rows, lambda 1e-4,
stop at ||b - A x|| / ||b|| < 1e-8 or after --steps outer iterations (the
workload's cap is 5000).  A step is one outer ROR-BK iteration: three sampled
block updates, the full residual pass with per-block norms and the stop test,
the top-K greedy selection and the greedy block update.

Other workloads (``--workload``): ``csr_200000`` (sparse square CSR, FP32
values for the inner passes), ``wide_2000x50000``, ``dense_2000x200``; the
paper's own protocol of 100 blocks (Section 3.1) on its dense random shapes,
``randn_60000x10000`` (Table 3, blocks of 600 rows) and ``unif_100000x10000``,
``unif_100000x15000``, ``unif_100000x20000`` (Table 5, blocks of 1000 rows),
all to relative residual 1e-6; and
``colform_200000x500`` (blocks of 2000 rows against 500 columns, solved in
the column form).

Timed: the mixed-precision solve (FP32 storage for the inner passes, FP64
outer residual and refinement; `value`) and the all-FP64 solve on the same
matrix, inputs resident in HBM.  The residual-pass kernel is timed with HIP
events inside the solve (RORBK_PROFILE).  The FP64 CPU oracle is timed on a
bounded sample of the same workload on the host cores (cpu_baseline), and the
GPU solves are compared with it over that sample.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time to rel. residual 1e-8 (s), mixed vs FP64 on GPU; "
          "residual-pass HBM GB/s")
PEAK_HBM_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_traffic(workload: str, mixed: str):
    """HBM bytes per launch of the residual kernel from the committed
    byte-counter summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy),
    used only if the counters were taken from the kernel source as it is now;
    otherwise None."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"k_resid_dense_{mixed}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    hs = re.search(r"kernel_source_sha256: ([0-9a-f]{64})", text)
    tb = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not hs or not tb:
        return None
    h = hashlib.sha256()
    for f in ("k_resid.hip", "rorbk_device.h"):
        with open(os.path.join(ROOT, "paper_2510_02156_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(tb.group(1)) if h.hexdigest() == hs.group(1) else None


def copy_calibration(mib: int):
    """A plain streaming copy (dst = -src) of known size: under a byte-counter
    profile, the counters it reads give the scale between counted and moved
    bytes on this part."""
    import torch
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        torch.neg(src, out=dst)   # one streaming elementwise kernel: reads and writes nbytes
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="tall_100000x2000")
    ap.add_argument("--mixed", default="f32", choices=["f32", "bf16"],
                    help="storage of the inner passes of the mixed solve")
    ap.add_argument("--inner", type=int, default=50, help="inner iterations per FP64 step")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-extra", action="store_true",
                    help="time only the mixed solve (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the "
                         "reference kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); "
              "this build has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_02156_amd as P
    from workloads import WORKLOADS, make, to_bf16_bits

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.time()
    w = make(args.workload)
    log(f"generated {args.workload} in {time.time() - t0:.1f}s")
    bh = w["b"]
    br, lam, tol, seed = w["block_rows"], w["lam"], w["tol"], w["seed"]
    b = torch.from_numpy(bh).to(dev)
    csr = w["format"] == "csr"
    if csr:
        if args.mixed != "f32":
            raise SystemExit("sparse storage is FP64 or FP32 only")
        m, n = w["m"], w["n"]
        nnz = len(w["val"])
        rowptr = torch.from_numpy(w["rowptr"]).to(dev)
        colidx = torch.from_numpy(w["colidx"]).to(dev)
        V64 = torch.from_numpy(w["val"]).to(dev)
        V32 = V64.float()
        torch.cuda.synchronize()
        t0 = time.time()
        s64 = P.Solver(None, br, lam, rowptr=rowptr, colidx=colidx, values=V64, shape=(m, n))
        torch.cuda.synchronize()
        t_setup64 = time.time() - t0
        t0 = time.time()
        smix = P.Solver(None, br, lam, rowptr=rowptr, colidx=colidx, values=V32, shape=(m, n),
                        A64=V64)
        torch.cuda.synchronize()
        t_setupmix = time.time() - t0
        oracle_A = w
    else:
        A64h = w["A"]
        m, n = A64h.shape
        nnz = m * n
        A64 = torch.from_numpy(A64h).to(dev)
        A32 = A64.float()
        Abf = torch.from_numpy(to_bf16_bits(A64h).view(np.int16)).view(torch.bfloat16).to(dev)
        torch.cuda.synchronize()
        t0 = time.time()
        s64 = P.Solver(A64, br, lam)
        torch.cuda.synchronize()
        t_setup64 = time.time() - t0
        Amix = A32 if args.mixed == "f32" else Abf
        t0 = time.time()
        smix = P.Solver(Amix, br, lam, A64=A64)
        torch.cuda.synchronize()
        t_setupmix = time.time() - t0
        oracle_A = A64h
    smix.set_refine(args.inner, 1e-4)
    log(f"setup: fp64 {t_setup64:.3f}s, mixed-{args.mixed} {t_setupmix:.3f}s "
        f"(k={s64.k}, K={s64.K})")

    K = args.steps

    def resid_bytes(es, xs):
        """Algorithmic bytes of one residual pass: the matrix once (values, and
        for CSR the column indices and row offsets), x once, the products written."""
        if csr:
            return nnz * (es + 4) + (m + 1) * 8 + n * xs + m * 8
        return m * n * es + n * xs + m * 8

    def run(sol, refine, iters, profile=False):
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, info = sol.solve(b, x, seed=seed, tol=tol, max_iters=iters, refine=refine,
                            profile=profile)
        torch.cuda.synchronize()
        return x, info, time.perf_counter() - t

    # warmup
    run(smix, True, args.warmup)
    if not args.skip_extra:
        run(s64, False, args.warmup)
    # timed: mixed (value), then FP64
    xm, im, tm = run(smix, True, K, profile=True)
    prof_m = smix.profile()
    marks = [i for i in (1, 10, 100, 500, 1000, 2000, 3000, 4000, 5000, K) if i <= K]

    def curve(sol):
        h = sol.record()["rrn"]
        return {str(i): float(h[i - 1]) for i in sorted(set(marks)) if i <= len(h)}

    curve_m = curve(smix)
    log(f"mixed-{args.mixed}: {tm:.3f}s for {im['iters']} iters, rrn {im['rrn']:.3e}, "
        f"converged {im['converged']}, refine steps {im['n_refine']}")
    res = {}
    if not args.skip_extra:
        x64, i64, t64 = run(s64, False, K, profile=True)
        prof_64 = s64.profile()
        res["rrn_curve"] = {"mixed": curve_m, "fp64": curve(s64)}
        log(f"fp64: {t64:.3f}s for {i64['iters']} iters, rrn {i64['rrn']:.3e}")
        res["fp64"] = {"time_s": t64, "iters": i64["iters"], "rrn": i64["rrn"],
                       "converged": i64["converged"],
                       "resid_kernel_ms": prof_64["inner_ms"],
                       "resid_GBs": resid_bytes(8, 8) / (prof_64["inner_ms"] * 1e-3) / 1e9
                       if prof_64["inner_ms"] > 0 else None}
        res["speedup_mixed_vs_fp64"] = t64 / tm
        xs = w["xstar"]
        # the returned iterates measured by one FP64 residual pass each
        res["rrn_of_returned_x"] = {"mixed": float(s64.residual(b, xm)[2]),
                                    "fp64": float(s64.residual(b, x64)[2])}
        res["rel_err_to_xstar"] = {"mixed": float(np.linalg.norm(xm.cpu().numpy() - xs) / np.linalg.norm(xs)),
                                   "fp64": float(np.linalg.norm(x64.cpu().numpy() - xs) / np.linalg.norm(xs))}
        # Algorithm 3: flexible AB-GMRES with ROR-BK inner iterations (FP64),
        # against plain ROR-BK run for the same number of inner iterations
        outer, inner = 30, 20
        xg = torch.zeros(n, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xg, ig = s64.fabgmres(b, xg, seed=seed, tol=tol, max_outer=outer, inner_iters=inner,
                              eta=1e-2)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        _, i_eq, t_eq = run(s64, False, max(ig["inner_iters"], 1))
        res["fabgmres"] = {"time_s": tg, "outer": ig["outer"], "inner_iters": ig["inner_iters"],
                           "rrn": ig["rrn"], "max_outer": outer, "inner_per_outer": inner,
                           "eta": 1e-2,
                           "plain_rorbk_same_iters": {"time_s": t_eq, "rrn": i_eq["rrn"]}}
        log(f"fabgmres: {tg:.3f}s, {ig['outer']} outer / {ig['inner_iters']} inner, "
            f"rrn {ig['rrn']:.3e} (plain ROR-BK same iterations: rrn {i_eq['rrn']:.3e})")
        # Algorithm 2's starting iterate (one product pass over A in FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x0i, coef = s64.initial_solution(b)
        torch.cuda.synchronize()
        res["initial_solution"] = {"ms": (time.perf_counter() - t0) * 1e3, "coefficient": coef,
                                   "rrn_x0": float(s64.residual(b, x0i)[2])}
        if not csr:
            # the other 16-/32-bit storage beside the one timed as `value`
            other = "bf16" if args.mixed == "f32" else "f32"
            Aoth = Abf if other == "bf16" else A32
            soth = P.Solver(Aoth, br, lam, A64=A64)
            soth.set_refine(args.inner, 1e-4)
            run(soth, True, args.warmup)
            xo, io, to = run(soth, True, K, profile=True)
            po = soth.profile()
            eo = 2 if other == "bf16" else 4
            log(f"mixed-{other}: {to:.3f}s for {io['iters']} iters")
            res[f"mixed_{other}"] = {
                "time_s": to, "iters": io["iters"], "converged": io["converged"],
                "speedup_vs_fp64": t64 / to,
                "rrn_of_returned_x": float(s64.residual(b, xo)[2]),
                "rrn_curve": curve(soth),
                "resid_kernel_ms": po["inner_ms"],
                "resid_GBs": resid_bytes(eo, 4) / (po["inner_ms"] * 1e-3) / 1e9
                if po["inner_ms"] > 0 else None}
            soth.close()

    # roofline of the dominant kernel: the inner residual pass of the mixed solve
    es = 4 if args.mixed == "f32" else 2
    bytes_resid = resid_bytes(es, 4)
    ms = prof_m["inner_ms"]
    achieved = bytes_resid / (ms * 1e-3) / 1e9 if ms > 0 else None
    roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": (achieved / PEAK_HBM_GBS) if achieved else None,
            "traffic": None if csr else measured_traffic(args.workload, args.mixed),
            "kernel": (f"k_csr_spmv<{args.mixed}>" if csr else f"k_resid_dense<{args.mixed}>"),
            "bytes_per_launch": bytes_resid,
            "avg_launch_ms": ms, "launches_timed": prof_m["inner_n"]}

    # CPU baseline: the FP64 oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        t0 = time.time()
        Wo = O.proposal(O.cosine_rowsums(oracle_A, br), n)[1]     # the oracle's own proposal
        t_prop = time.time() - t0
        probe = O.solve(oracle_A, br, lam, bh, seed=seed, tol=tol, max_iters=3, W=Wo,
                        record=False)
        per = max(probe["t_iter_s"] / 3, 1e-4)
        N = int(min(2000, max(10, args.cpu_seconds / per)))
        log(f"oracle: setup {probe['t_setup_s']:.2f}s, {per * 1e3:.1f} ms/iter; sample {N} iters")
        ref = O.solve(oracle_A, br, lam, bh, seed=seed, tol=tol, max_iters=N, W=Wo, record=False)
        per = ref["t_iter_s"] / max(ref["iters"], 1)
        # the oracle follows the FP64 solve's trajectory, so it needs the same
        # number of iterations to the tolerance (or the cap)
        need = i64["iters"] if not args.skip_extra else im["iters"]
        cpu = {"value": per * need, "unit": "s", "cores": O.num_threads(), "kind": "oracle",
               "sample": (f"FP64 oracle setup once (proposal {t_prop:.2f}s + block factors "
                          f"{ref['t_setup_s']:.2f}s, not counted) + "
                          f"{ref['iters']} outer iterations on the full {m}x{n} system; "
                          f"per-iteration time x {need} iterations (the FP64 solve's count "
                          f"to the tolerance or the cap)"),
               "iters_per_s": 1.0 / per}
        # GPU solves against the oracle over the same N iterations
        xg64, _, _ = run(s64, False, N)
        xgm, _, _ = run(smix, True, N)
        nr = np.linalg.norm(ref["x"])
        res["error_vs_oracle"] = {
            "iters": N,
            "fp64_rel": float(np.linalg.norm(xg64.cpu().numpy() - ref["x"]) / nr),
            f"mixed_{args.mixed}_rel": float(np.linalg.norm(xgm.cpu().numpy() - ref["x"]) / nr)}
        log(f"error vs oracle after {N} iters: {res['error_vs_oracle']}")

    out = {
        "metric": METRIC,
        "value": tm,
        "unit": "s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": tm / max(im["iters"], 1) * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.mixed}+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "nnz": nnz, "block_rows": br,
                   "lambda": lam, "cond": WORKLOADS[args.workload].get("cond"), "tol": tol,
                   "cap_iters": K,
                   "mixed": f"{args.mixed} storage inner passes, FP64 refinement every "
                            f"{args.inner} inner iterations",
                   "parallelism": "single GPU"},
        "reached_tol": bool(im["converged"]),
        "iters": im["iters"],
        "rrn_at_end": im["rrn"],
        "iters_per_s": im["iters"] / tm,
        "setup_s": {"fp64": t_setup64, "mixed": t_setupmix},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(res)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
