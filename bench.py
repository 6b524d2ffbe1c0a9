"""Throughput benchmark of the TSQR hot path on one MI355X.

Default workload (--workload single): one pass of the single-matrix path over
a 1,048,576 x 64 FP64 matrix (iid N(0,1), seed 0) split into 4096-row
domains with a binary tree:
    partition + leaf QR + tree + sign normalisation   (tsqr_factor, keep Q)
    thin Q                                             (tsqr_form_q)
    least squares for one right-hand side              (tsqr_lsq_solve)
The metric is useful Gflop/s: (2mn^2 - 2n^3/3) for R, the same again for Q
(Table 2 of the paper counts Q + R as twice R), plus 4mn + n^2 for the
solve.  Inputs are resident in HBM before the timed region.

Other workloads, one JSON line each:
  --workload mixed  4,194,304 x 128, A = U diag(s) V^T with s log-spaced
                    from 1 to 1e-6; factor + least squares (b ~ N(0,1) and a
                    consistent b), mixed precision beside FP64, with the
                    backward error of every solution;
  --workload batch  512 matrices, m ~ U[1000, 200000], n in {8,16,32,64},
                    odd ones mixed, one b each: autotuned plan, one captured
                    graph per run, beside 512 sequential single calls;
  --workload serve  a seeded Poisson stream of least-squares requests
                    (m log-uniform in 2^10..2^21, n in {16..256}, 1-8 RHS,
                    10 % at kappa 1e6, 25 % repeated matrices) through the
                    request server: saturated throughput, then p50/p99
                    latency at 0.5, 0.8 and 0.95 of it;
  --workload sweep  the single-matrix path at m = 2^20 for n in {8, 16, 32, 64};
  --workload orth   a block Krylov loop: TSQR-based block orthogonalisation;
  --workload tslu   LU with tournament pivoting of 1,048,576 x 64 (TSLU);
  --workload wide   262,144 x 1,024 in 64-column panels (factor + solve);
  --workload chol   8,192 x 8,192 Cholesky of an SPD Gram matrix, beside
                    torch.linalg.cholesky;
  --workload calu   4,096 x 4,096 LU with tournament-pivoted panels (CALU),
                    beside torch.linalg.lu_factor;
  --workload copy   a plain 1 GiB device copy (calibrates HBM counters).
The default run also appends compact records of these workloads.

--gpus N > 1 is refused: the library factors on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_PEAK_TFS = 78.6           # MI355X FP64 vector = matrix, published


def flops_step(m: int, n: int, k: int) -> float:
    f_r = 2.0 * m * n * n - 2.0 * n ** 3 / 3.0
    return 2.0 * f_r + 4.0 * m * n * k + n * n * k


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(m: int, n: int, mb: int, passes: int, samples: int = 3):
    """The FP64 CPU oracle on the same workload, on the host cores; test
    infrastructure only.  `samples` timed samples of `passes` full passes
    each (factor + thin Q + 1-RHS solve); the median sample is the value."""
    import numpy as np
    import oracle
    import synth
    A = synth.config_large(m, n, seed=0)
    b = synth.config_large_rhs(m, seed=1)
    rates, walls = [], []
    for _ in range(samples):
        t0 = time.perf_counter()
        for _ in range(passes):
            f = oracle.TSQR(A, mb=mb)
            f.form_q()
            f.lsq(b)
        dt = time.perf_counter() - t0
        walls.append(dt)
        rates.append(flops_step(m, n, 1) * passes / dt / 1e9)
    return {
        "value": round(float(np.median(rates)), 3),
        "unit": "Gflop/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "cpu_model": host_cpu_model(),
        "host_cpus": os.cpu_count(),
        "samples_gflops": [round(r, 3) for r in rates],
        "sample": f"median of {samples} samples, each {passes} full passes (factor + thin Q + 1-RHS "
                  f"solve) of the {m}x{n} matrix ({', '.join(f'{w:.1f}' for w in walls)} s wall)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="single",
                    choices=["single", "mixed", "batch", "serve", "sweep", "orth", "tslu", "wide", "chol", "calu", "copy"])
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--m", type=int, default=1 << 20)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--row-block", type=int, default=4096)
    ap.add_argument("--domains", type=int, default=0,
                    help="single workload: load-balanced partition into this many domains (-1: one per "
                         "resident leaf workgroup) instead of --row-block")
    ap.add_argument("--tree", default="binary", choices=["binary", "quad", "flat", "xcd"],
                    help="single workload: reduction tree (xcd: each XCD's domains first)")
    ap.add_argument("--cpu-passes", type=int, default=7)
    ap.add_argument("--no-sub", action="store_true",
                    help="single workload: leave out the compact mixed / batch / serve / n-sweep records")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--separate-calls", action="store_true",
                    help="single workload: tsqr_factor, tsqr_form_q and tsqr_lsq_solve as three calls "
                         "(the thin Q and the solve on two streams) instead of one tsqr_factor_solve")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this library factors on one GPU; sharding the rows "
              "over several GPUs (one more combine level across them) is not implemented", file=sys.stderr)
        sys.exit(2)
    {"single": run_single, "mixed": run_mixed, "batch": run_batch, "serve": run_serve,
     "sweep": run_sweep, "orth": run_orth, "tslu": run_tslu, "wide": run_wide, "chol": run_chol, "calu": run_calu, "copy": run_copy}[args.workload](args)


def counter_record(kernel: str, m: int, n: int, mb: int, tree: str, kind: str):
    """The committed counter record profiles/<kernel>_<m>x<n>_<kind>.json of
    this kernel and workload (row block 4096, binary tree), or None when there
    is none or the kernel's sources changed since its counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{m}x{n}_{kind}.json")
    if not os.path.exists(path) or mb != 4096 or tree != "binary":
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec


def counted_traffic(kernel: str, m: int, n: int, mb: int, tree: str):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, scaled by a plain
    copy) from the kernel's counter record, or None."""
    rec = counter_record(kernel, m, n, mb, tree, "hbm")
    return rec["traffic_bytes_per_launch"] if rec else None


def run_single(args):
    line = measure_single(args, args.m, args.n, args.row_block, args.steps, args.warmup, domains=args.domains)
    if not args.no_sub:
        line["sub_records"] = sub_records(args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.m, args.n, args.row_block, args.cpu_passes)
    print(json.dumps(line), flush=True)


def measure_single(args, m, n, mb, steps, warmup, domains=0):
    """One tsqr_factor_solve (factor + thin Q + 1-RHS solve) per step on an
    m x n N(0,1) matrix; returns the record of the timed loop.  domains != 0:
    the load-balanced partition (opts.domains) instead of mb-row domains."""
    import torch
    import paper_0912_2572_amd as tl
    import synth

    dev = torch.device("cuda:0")
    A = torch.as_tensor(synth.config_large(m, n, seed=0)).t().contiguous().t().to(dev)
    b = torch.as_tensor(synth.config_large_rhs(m, seed=1)).to(dev)
    tree_name = getattr(args, "tree", "binary")
    tree = {"binary": tl.TREE_BINARY, "quad": tl.TREE_QUAD, "flat": tl.TREE_FLAT,
            "xcd": tl.TREE_XCD}[tree_name]
    if domains:
        mb = 0
    o = tl.opts(row_block=mb, tree=tree, keep_q=True, lsq_max_rhs=1, domains=domains)
    work = torch.empty(tl.workspace_bytes(m, n, o), dtype=torch.uint8, device=dev)
    Q = tl.empty_colmajor(m, n, device=dev)
    X = tl.empty_colmajor(n, 1, device=dev)
    res = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    Bcol = b.reshape(-1, 1)
    P, chunk, _ = tl.plan_info(m, n, o)

    # one tsqr_factor_solve call per step: the solve's leaf pass of Q^T b
    # runs on the library's second stream beside the tree factorization, its
    # tree pass beside the thin Q.  --separate-calls: the three calls, the
    # thin Q and the solve on two streams after the factor (FP64, n <= 64:
    # they only read the factor and use disjoint workspace blocks), joined
    # before the next step's factor overwrites the workspace
    side = torch.cuda.Stream()

    overlap = n <= 64

    def step():
        if not args.separate_calls:
            f, _, _, _ = tl.factor_solve(A, Bcol, o, work=work, X=X, resid=res, info=info, Q=Q)
            return f
        main = torch.cuda.current_stream()
        f = tl.Factors(A, o, work=work)
        if overlap:
            side.wait_stream(main)
            with torch.cuda.stream(side):
                f.form_q(Q)
        else:
            f.form_q(Q)
        f.lsq(Bcol, X=X, resid=res, info=info)
        if overlap:
            main.wait_stream(side)
        return f

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # per-kernel breakdown from an untimed pass with every launch bracketed
    # by events; the timed loop then carries events around the dominant
    # kernel only (an event pair per launch of ~35 kernels costs ~0.2 ms)
    prof_steps = min(steps, 3)
    tl.prof_enable(True)
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    kern_all = tl.prof_query()
    tl.prof_enable(False)
    dom_name = max(kern_all.items(), key=lambda kv: kv[1][1])[0]
    tl.prof_enable(True)
    tl.prof_only(dom_name)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    kern = tl.prof_query()
    tl.prof_only(None)
    tl.prof_enable(False)
    assert int(info.item()) == 0

    fl = flops_step(m, n, 1)
    value = fl / (ms * 1e-3) / 1e9
    # dominant kernel, timed in the timed loop, and its algorithmic traffic per launch
    dom_cnt, dom_ms = kern[dom_name]
    avg_s = dom_ms / dom_cnt * 1e-3
    e = 8
    alg_bytes = {
        # read A, write V, one n x n T per domain
        "leaf_factor": 8.0 * m * n + e * m * n + 8.0 * P * n * n,
        # read V, write Q (the thin-Q leaf pass)
        "leaf_apply_q": e * m * n + 8.0 * m * n,
        # read V, read and write B (k = 1)
        "leaf_apply_qt": e * m * n + 16.0 * m,
    }
    ab = alg_bytes.get(dom_name)
    roof = None
    if ab is not None:
        gbs = ab / avg_s / 1e9
        roof = {"kernel": dom_name, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                "traffic": counted_traffic(dom_name, m, n, mb, tree_name),
                "avg_launch_us": round(avg_s * 1e6, 2), "alg_bytes_per_launch": ab}
        util = counter_record(dom_name, m, n, mb, tree_name, "util")
        if util:
            # matrix-core and vector-ALU use of the same kernel from its
            # committed SQ counter record (fractions of the FP64 peak)
            roof.update({k: util[k] for k in ("mfma_util", "valu_fp64_frac", "valu_issue_busy")})
    line = {
        "metric": "TSQR Gflop/s (factor + thin Q + LSQ), FP64",
        "value": round(value, 2),
        "unit": "Gflop/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic iid N(0,1), seed 0",
        "config": {"workload": f"tsqr_factor_formq_lsq {m}x{n}", "m": m, "n": n,
                   "row_block": mb if not domains else None,
                   "partition": "balanced" if domains else "row_block",
                   "domains": P, "chunk_rows": chunk, "tree": tree_name, "rhs": 1,
                   "parallelism": "single GPU",
                   "streams": ("one tsqr_factor_solve call: the solve's leaf pass beside the tree, its tree "
                               "pass beside the thin Q" if not args.separate_calls else
                               "thin Q and the solve overlap on two streams after the factor") if overlap
                   else "one stream"},
        "kernels_ms_per_step": {k: round(v[1] / prof_steps, 4) for k, v in kern_all.items()},
        "kernels_ms_note": "per-kernel times from an untimed pass with every launch timed; kernels on "
                           "the two streams overlap, so they do not add up to ms_per_step",
        "roofline": roof,
    }
    return line


def run_sweep(args):
    print(json.dumps(sweep_n(args, steps=args.steps, warmup=args.warmup)), flush=True)


def sweep_n(args, steps, warmup):
    """The single-matrix path at m = 2^20 for n in {8, 16, 32, 64} (the
    HBM-bound range of the factorization, n <= 64)."""
    out = {}
    for n in (8, 16, 32, 64):
        r = measure_single(args, 1 << 20, n, 4096, steps, warmup)
        rf = r["roofline"] or {}
        out[str(n)] = {"ms_per_step": r["ms_per_step"], "gflops": r["value"],
                       "dominant_kernel": rf.get("kernel"), "dominant_frac_hbm": rf.get("frac"),
                       "dominant_avg_us": rf.get("avg_launch_us"),
                       "leaf_ms": r["kernels_ms_per_step"].get("leaf_factor")}
    return {"metric": "TSQR Gflop/s (factor + thin Q + LSQ), FP64, n sweep at m = 2^20", "unit": "Gflop/s",
            "steps": steps, "warmup": warmup, "by_n": out}


def sub_records(args):
    """Compact records of the rest of the headline metric (mixed vs FP64 at
    kappa 1e6, the batch, the server) and the n sweep, so that one default
    run carries all of it."""
    t0 = time.perf_counter()
    mx = measure_mixed(args, steps=3, warmup=1)
    t1 = time.perf_counter()
    bt = measure_batch(args, steps=3, warmup=1)
    t2 = time.perf_counter()
    sv = measure_serve(args, requests=200, loads=(0.8,), mixed_pass=True)
    t3 = time.perf_counter()
    sw = sweep_n(args, steps=10, warmup=2)
    t4 = time.perf_counter()
    ob = measure_orth(args, steps=3, warmup=1)
    t5 = time.perf_counter()
    lu = measure_tslu(args, steps=5, warmup=1)
    t5b = time.perf_counter()
    wd = measure_wide(args, steps=3, warmup=1, domains=-1)
    t5c = time.perf_counter()
    ch = measure_chol(args, steps=5, warmup=1)
    t5d = time.perf_counter()
    cl = measure_calu(args, steps=3, warmup=1)
    t5e = time.perf_counter()
    # a row count where 4096-row domains (293 of them) leave a second, mostly
    # idle wave of leaf workgroups on the 256 compute units, against the
    # load-balanced partition (one domain of 18-19 chunks per unit)
    mr = 1_200_000
    uni = measure_single(args, mr, 64, 4096, 10, 2)
    bal = measure_single(args, mr, 64, 0, 10, 2, domains=-1)
    t6 = time.perf_counter()
    return {
        "balanced_domains": {
            "workload": f"tsqr_factor_formq_lsq {mr}x64",
            "row_block_4096": {"domains": uni["config"]["domains"], "ms_per_step": uni["ms_per_step"],
                               "gflops": uni["value"],
                               "leaf_ms": uni["kernels_ms_per_step"].get("leaf_factor")},
            "balanced": {"domains": bal["config"]["domains"], "ms_per_step": bal["ms_per_step"],
                         "gflops": bal["value"], "leaf_ms": bal["kernels_ms_per_step"].get("leaf_factor")},
            "speedup": round(uni["ms_per_step"] / bal["ms_per_step"], 3), "wall_s": round(t6 - t5e, 1)},
        "mixed_kappa1e6": {
            "workload": mx["config"]["workload"],
            "f64_ms": round(mx["f64"]["ms"], 3), "mixed_ms": round(mx["mixed"]["ms"], 3),
            "speedup_mixed_over_f64": mx["speedup_mixed_over_f64"],
            "mixed_sweeps": mx["mixed"]["sweeps"],
            "mixed_routed_ms": round(mx["mixed_routed"]["ms"], 3),
            "mixed_routed_kappa_estimate": mx["mixed_routed"]["kappa_estimate"],
            "eta_mixed_routed": mx["mixed_routed"]["eta"],
            "eta_f64": mx["f64"]["eta"], "eta_mixed": mx["mixed"]["eta"],
            "mixed_info": mx["mixed"]["info"], "wall_s": round(t1 - t0, 1)},
        "batch_512": {
            "ms_per_run": bt["ms_per_step"], "solves_per_s": bt["solves_per_s"], "gflops": bt["value"],
            "roofline_frac_hbm": bt["roofline"]["frac"], "speedup_vs_sequential": bt["speedup_vs_sequential"],
            "sampled_eta_max": bt["sampled_eta_max"], "wall_s": round(t2 - t1, 1)},
        "serve_200": {
            "f64_saturated_solves_per_s": round(sv["saturated"]["solves_per_s"], 2),
            "f64_p50_ms_at_0.8": round(sv["poisson"]["0.8"]["p50_ms"], 2),
            "f64_p99_ms_at_0.8": round(sv["poisson"]["0.8"]["p99_ms"], 2),
            "mixed_saturated_solves_per_s": round(sv["mixed_saturated"]["solves_per_s"], 2),
            "mixed_p50_ms_saturated": round(sv["mixed_saturated"]["p50_ms"], 2),
            "mixed_p99_ms_saturated": round(sv["mixed_saturated"]["p99_ms"], 2),
            "sampled_eta_max": sv["sampled_eta_max"], "wall_s": round(t3 - t2, 1)},
        "n_sweep_m2p20": {**sw["by_n"], "wall_s": round(t4 - t3, 1)},
        "tslu_1048576x64": {
            "ms": lu["ms_per_step"], "gflops": lu["value"], "leaf_ms": lu["leaf_ms"],
            "rel_residual": lu["rel_residual_A_minus_LU"], "max_abs_L": lu["max_abs_L"],
            "wall_s": round(t5b - t5, 1)},
        "panels_262144x1024": {
            "ms": wd["ms_per_step"], "gflops": wd["value"], "eta": wd["eta"], "info": wd["info"],
            "domains": wd["config"]["domains"],
            "trailing_update_ms": wd["kernels_ms_per_step"].get("leaf_apply_qt"),
            "wall_s": round(t5c - t5b, 1)},
        "cholesky_8192": {
            "ms": ch["ms_per_step"], "gflops": ch["value"], "info": ch["info"],
            "torch_linalg_cholesky_ms": ch["torch_linalg_cholesky_ms"], "speedup_vs_torch": ch["speedup_vs_torch"],
            "syrk_ms": ch["kernels_ms_per_step"].get("chol_syrk"), "syrk_tflops": ch["syrk_tflops"],
            "panel_ms": ch["kernels_ms_per_step"].get("chol_panel"),
            "sampled_backward_error": ch["sampled_backward_error"], "wall_s": round(t5d - t5c, 1)},
        "calu_4096": {
            "ms": cl["ms_per_step"], "gflops": cl["value"], "info": cl["info"],
            "torch_linalg_lu_factor_ms": cl["torch_linalg_lu_factor_ms"], "speedup_vs_torch": cl["speedup_vs_torch"],
            "tslu_ms": round(sum(v for k, v in cl["kernels_ms_per_step"].items() if k.startswith("tslu")), 3),
            "update_ms": cl["kernels_ms_per_step"].get("calu_update"),
            "rel_residual": cl["rel_residual_PA_minus_LU"], "max_abs_L": cl["max_abs_L"],
            "wall_s": round(t5e - t5d, 1)},
        "block_krylov_orth": {
            "workload": ob["config"]["workload"], "ms_per_loop": ob["ms_per_step"], "gflops": ob["value"],
            "roofline_frac_hbm": ob["roofline"]["frac"], "proj_update_gbs": ob["proj_update_gbs"],
            "basis_orthogonality_fro": ob["basis_orthogonality_fro"], "wall_s": round(t5 - t4, 1)},
    }


def _eta(A, x, b):
    """Backward-error proxy ||A^T (b - A x)|| / (||A||_F (||A||_F ||x|| + ||b||)), FP64 on the GPU."""
    import torch
    r = b - A @ x
    nA = torch.linalg.norm(A)
    return float(torch.linalg.norm(A.t() @ r) / (nA * (nA * torch.linalg.norm(x) + torch.linalg.norm(b))))


def run_mixed(args):
    print(json.dumps(measure_mixed(args, args.steps, args.warmup)), flush=True)


def measure_mixed(args, steps, warmup):
    """Config with kappa = 1e6: FP64 path vs mixed path, factor + 2-RHS solve."""
    import torch
    import paper_0912_2572_amd as tl
    import synth
    m, n = 4194304, 128
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    G1 = torch.randn((n, m), generator=g, device=dev, dtype=torch.float64).t()
    G2 = torch.randn((n, n), generator=g, device=dev, dtype=torch.float64)
    U, _ = torch.linalg.qr(G1)
    V, _ = torch.linalg.qr(G2)
    s = torch.as_tensor(synth.log_spaced_spectrum(n, -6.0), device=dev)
    A = ((U * s) @ V.t()).t().contiguous().t()
    del G1, U
    b = torch.randn(m, generator=g, device=dev, dtype=torch.float64)
    xt = torch.randn(n, generator=g, device=dev, dtype=torch.float64)
    bc = A @ xt
    B = torch.stack([b, bc], dim=1).t().contiguous().t()
    flops = 2.0 * m * n * n - 2.0 * n ** 3 / 3.0 + 2 * (4.0 * m * n + n * n)
    out = {}
    # "mixed_routed": the mixed path with route_kappa 1e4, which finds
    # kappa_1(R) ~ 1e6 and solves in FP64 instead of refining
    for name, prec, route in (("f64", tl.F64, 0.0), ("mixed", tl.MIXED, 0.0), ("mixed_routed", tl.MIXED, 1e4)):
        o = tl.opts(row_block=4096, prec=prec, lsq_max_rhs=2, route_kappa=route)
        work = torch.empty(tl.workspace_bytes(m, n, o), dtype=torch.uint8, device=dev)
        X = tl.empty_colmajor(n, 2, device=dev)
        res = torch.empty(2, dtype=torch.float64, device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)

        def step():
            f = tl.Factors(A, o, work=work)
            f.lsq(B, A=A, X=X, resid=res, info=info)
            return f
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            f = step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        sweeps = f.last_refine_iters()
        # per-kernel breakdown from one more, untimed step with every launch timed
        tl.prof_enable(True)
        step()
        torch.cuda.synchronize()
        kern = tl.prof_query()
        tl.prof_enable(False)
        e1 = [_eta(A, X[:, c], B[:, c]) for c in range(2)]
        rprec, rkappa = f.route_info()
        out[name] = {"ms": ms, "gflops": flops / (ms * 1e-3) / 1e9, "eta": e1, "sweeps": sweeps,
                     "info": int(info.item()), "x": X.clone(),
                     "routed_to_f64": bool(prec == tl.MIXED and rprec == tl.F64),
                     "kappa_estimate": rkappa,
                     "kernels_ms_per_step": {k: round(v[1], 4) for k, v in kern.items()}}
        del work
    xf, xm = out["f64"]["x"], out["mixed"]["x"]
    e2 = [float(torch.linalg.norm(xm[:, c] - xf[:, c]) / torch.linalg.norm(xf[:, c])) for c in range(2)]
    e_true = float(torch.linalg.norm(xm[:, 1] - xt) / torch.linalg.norm(xt))
    line = {
        "metric": "TSQR least squares Gflop/s (factor + 2-RHS solve), mixed vs FP64 at kappa 1e6",
        "value": round(out["mixed"]["gflops"], 2),
        "unit": "Gflop/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(out["mixed"]["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic U diag(s) V^T, U, V from QR of torch N(0,1) draws (Philox, seed 0)",
        "config": {"workload": f"tsqr_lsq_conditioned {m}x{n}", "m": m, "n": n, "row_block": 4096,
                   "tree": "binary", "rhs": 2, "kappa": 1e6},
        "f64": {k: v for k, v in out["f64"].items() if k != "x"},
        "mixed": {k: v for k, v in out["mixed"].items() if k != "x"},
        "mixed_routed": {k: v for k, v in out["mixed_routed"].items() if k != "x"},
        "mixed_vs_f64_rel_x": e2,
        "mixed_consistent_rhs_rel_err_x_true": e_true,
        "speedup_mixed_over_f64": round(out["f64"]["ms"] / out["mixed"]["ms"], 3),
    }
    del A, B, bc
    torch.cuda.empty_cache()
    return line


def run_batch(args):
    print(json.dumps(measure_batch(args, args.steps, args.warmup)), flush=True)


def measure_batch(args, steps, warmup):
    """512 independent least-squares problems through the batched path."""
    import numpy as np
    import torch
    import paper_0912_2572_amd as tl
    import synth
    dev = torch.device("cuda:0")
    shapes = synth.batch_shapes(512, seed=0)
    precs = [j % 2 for j in range(len(shapes))]
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    As, bs = [], []
    for m, n in shapes:
        As.append(torch.randn((n, m), generator=g, device=dev, dtype=torch.float64).t())
        bs.append(torch.randn(m, generator=g, device=dev, dtype=torch.float64))
    torch.cuda.synchronize()
    # the table depends only on the (n class, precision) classes, so it is
    # tuned on every 3rd matrix of the batch (both precisions)
    t0 = time.perf_counter()
    table = tl.autotune(As[::3], bs[::3], precs[::3], reps=1)
    tune_s = time.perf_counter() - t0
    B = tl.Batch(As, bs, precs, tune=table, refine_sweeps=4)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(max(warmup, 1)):
            B.run(use_graph=True, stream=stream)
        stream.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(steps):
            B.run(use_graph=True, stream=stream)
        ev1.record(stream)
    stream.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    # per-kernel breakdown of one run with plain launches (HIP events per launch)
    tl.prof_enable(True)
    B.run(use_graph=False)
    torch.cuda.synchronize()
    kern = tl.prof_query()
    tl.prof_enable(False)
    flops = sum(2.0 * m * n * n - 2.0 * n ** 3 / 3.0 + 4.0 * m * n + n * n for m, n in shapes)
    # algorithmic HBM bytes of one run: read A, write V (e = 8 or 4), read V
    # and b for Q^T b; the mixed matrices' refinement sweeps are not counted
    alg = sum(8.0 * m * n + 2 * (8 if p == 0 else 4) * m * n + 16.0 * m
              for (m, n), p in zip(shapes, precs))
    eta = []
    infos = 0
    for i in range(0, len(shapes), 16):
        infos += int(B.info(i).item() != 0)
        eta.append(_eta(As[i], B.x(i), bs[i]))
    # the launch-bound baseline: the same problems as 512 sequential single calls
    fs = []
    work = None

    def seq():
        nonlocal work
        for i, (m, n) in enumerate(shapes):
            mb, tree, P = B.plan(i)
            o = tl.opts(row_block=mb, tree=tree, prec=precs[i], lsq_max_rhs=1)
            need = tl.workspace_bytes(m, n, o)
            if work is None or work.numel() < need:
                work = torch.empty(max(need, 1 << 30), dtype=torch.uint8, device=dev)
            f = tl.Factors(As[i], o, work=work)
            f.lsq(bs[i].reshape(-1, 1), A=As[i])
    seq()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq()
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3
    line = {
        "metric": "batched TSQR + least squares Gflop/s (512 matrices, half mixed)",
        "value": round(flops / (ms * 1e-3) / 1e9, 2),
        "unit": "Gflop/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic iid N(0,1), torch Philox seed 1; shapes from numpy PCG64 seed 0",
        "config": {"workload": "tsqr_batch_512", "count": len(shapes),
                   "total_rows": int(sum(m for m, n in shapes)),
                   "mixed": int(sum(precs)), "graph_launches": B.launches(), "refine_sweeps": 4},
        "roofline": {"bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "alg_bytes_per_run": alg, "kernel": "whole graph"},
        "solves_per_s": round(len(shapes) / (ms * 1e-3), 1),
        "sequential_single_calls_ms": round(seq_ms, 3),
        "speedup_vs_sequential": round(seq_ms / ms, 2),
        "kernels_ms_plain_run": {k: round(v[1], 3) for k, v in kern.items()},
        "autotune_s": round(tune_s, 2),
        "autotune_sample": "every 3rd matrix (171)",
        "tune_table": table,
        "sampled_eta_max": max(eta),
        "sampled_info_nonzero": infos,
    }
    del B, As, bs, work
    torch.cuda.empty_cache()
    return line


def run_serve(args):
    print(json.dumps(measure_serve(args, args.requests, loads=(0.5, 0.8, 0.95), mixed_pass=True)), flush=True)


def measure_serve(args, requests, loads, mixed_pass):
    """Least-squares serving: closed-loop saturation, then Poisson arrivals
    at the given fractions of it; with mixed_pass, a saturated pass of a
    mixed-precision server over the same stream."""
    import numpy as np
    import torch
    import paper_0912_2572_amd as tl
    import synth
    dev = torch.device("cuda:0")
    reqs = synth.serving_stream(requests, seed=0)
    # host data: windows of one pinned pool of N(0,1) values (drawn on the
    # device from torch's Philox generator, seed 0, then copied); requests at
    # kappa 1e6 get their own scaled copy G diag(s) / sqrt(m)
    max_mn = max(r["m"] * r["n"] for r in reqs)
    max_mk = max(r["m"] * r["k"] for r in reqs)
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    poolA = torch.empty(max_mn + 4096, dtype=torch.float64, pin_memory=True)
    poolA.copy_(torch.randn(max_mn + 4096, generator=g, device=dev, dtype=torch.float64))
    poolB = torch.empty(max_mk + 4096, dtype=torch.float64, pin_memory=True)
    poolB.copy_(torch.randn(max_mk + 4096, generator=g, device=dev, dtype=torch.float64))
    rng = np.random.default_rng(7)
    mats = {}
    for r in reqs:
        mid = r["matrix_id"]
        if mid in mats:
            continue
        m, n = r["m"], r["n"]
        off = int(rng.integers(0, 4096))
        A = poolA[off:off + m * n].view(n, m).t()
        if r["ill"]:
            s = torch.as_tensor(synth.log_spaced_spectrum(n, -6.0), device=dev)
            Ad = A.to(dev) * s / float(np.sqrt(m))
            A = torch.empty((n, m), dtype=torch.float64, pin_memory=True).t()
            A.copy_(Ad)
            del Ad
        mats[mid] = A
    Bs = {}
    for r in reqs:
        off = int(rng.integers(0, 4096))
        Bs[r["id"]] = poolB[off:off + r["m"] * r["k"]].view(r["k"], r["m"]).t()
    outs = {r["id"]: (torch.zeros((r["k"], r["n"]), dtype=torch.float64, pin_memory=True).t(),
                      torch.zeros(r["k"], dtype=torch.float64, pin_memory=True),
                      torch.zeros(1, dtype=torch.int32, pin_memory=True)) for r in reqs}
    budget = 64 << 30
    flops = sum(2.0 * r["m"] * r["n"] ** 2 - 2.0 * r["n"] ** 3 / 3.0 + 4.0 * r["m"] * r["n"] * r["k"]
                for r in reqs)

    def one_pass(rate, prec=tl.F64):
        S = tl.Server(hbm_budget=budget, streams=4, max_inflight=8, cache=True, prec=prec)
        t0 = tl.server_now()
        arrive = []
        t = 0.0
        for r in reqs:
            t += r["gap"] / rate if rate else 0.0
            arrive.append(t0 + t)
        tickets = []
        i = 0
        while i < len(reqs) or S.progress() > 0:
            now = tl.server_now()
            while i < len(reqs) and arrive[i] <= now:
                r = reqs[i]
                X, res, info = outs[r["id"]]
                tickets.append(S.submit(r["matrix_id"], mats[r["matrix_id"]], Bs[r["id"]], X, res, info))
                i += 1
            if i < len(reqs):
                S.progress()
            else:
                S.progress(wait=True)
        lat = []
        t_end = 0.0
        for j, tk in enumerate(tickets):
            assert S.status(tk) == 1
            _, _, td = S.times(tk)
            lat.append(td - arrive[j])
            t_end = max(t_end, td)
        st = S.stats()
        S.close()
        span = t_end - t0
        return {"solves_per_s": len(reqs) / span, "rhs_solves_per_s": sum(r["k"] for r in reqs) / span,
                "gflops": flops / span / 1e9, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "makespan_s": span,
                "cache_hits": st["cache_hits"], "evictions": st["evictions"],
                "mean_admitted_gb": st["byte_seconds"] / max(span, 1e-9) / 1e9,
                "peak_admitted_gb": st["bytes_peak"] / 1e9}

    one_pass(0.0)                       # warm-up (kernels, allocator)
    sat = one_pass(0.0)
    mu = sat["solves_per_s"]
    by_load = {}
    for frac in loads:
        by_load[str(frac)] = one_pass(frac * mu)
    mixed_sat = None
    if mixed_pass:
        one_pass(0.0, tl.MIXED)
        mixed_sat = one_pass(0.0, tl.MIXED)
    # accuracy: backward error of a sample of results (FP64, on the device)
    worst = 0.0
    for r in reqs[:: max(1, len(reqs) // 12)]:
        A = mats[r["matrix_id"]].to(dev)
        X = outs[r["id"]][0].to(dev)
        B = Bs[r["id"]].to(dev)
        for c in range(r["k"]):
            worst = max(worst, _eta(A, X[:, c], B[:, c]))
        assert int(outs[r["id"]][2][0]) == 0
    line = {
        "metric": "least-squares serving solves/s (saturated) with p50/p99 latency",
        "value": round(mu, 2), "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(sat["makespan_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "seeded Poisson request stream; A, B windows of a pinned N(0,1) pool (torch Philox seed 0)",
        "config": {"workload": f"tsqr_serve_{len(reqs)}_requests", "requests": len(reqs),
                   "hbm_budget_gb": budget / 2 ** 30, "streams": 4, "max_inflight": 8,
                   "mean_m": float(np.mean([r["m"] for r in reqs])),
                   "ill_share": float(np.mean([r["ill"] for r in reqs])),
                   "repeat_share": float(np.mean([r["matrix_id"] != r["id"] for r in reqs]))},
        "saturated": sat,
        "poisson": by_load,
        "mixed_saturated": mixed_sat,
        "sampled_eta_max": worst,
    }
    return line


def run_tslu(args):
    print(json.dumps(measure_tslu(args, args.steps, args.warmup)), flush=True)


def measure_tslu(args, steps, warmup, m=1 << 20, b=64):
    """TSLU (LU with tournament pivoting over the TSQR partition and binary
    tree) of an m x b N(0,1) matrix with 4096-row domains; useful flops
    m b^2 - b^3/3 (the LU of the panel)."""
    import torch
    import paper_0912_2572_amd as tl
    import synth
    dev = torch.device("cuda:0")
    A = torch.as_tensor(synth.config_large(m, b, seed=0)).t().contiguous().t().to(dev)
    o = tl.opts(row_block=4096)
    work = torch.empty(tl.lib().tsqr_tslu_workspace_bytes(m, b, ctypes_ref(o)), dtype=torch.uint8, device=dev)
    L = tl.empty_colmajor(m, b, device=dev)
    U = tl.empty_colmajor(b, b, device=dev)

    def step():
        return tl.tslu(A, o, work=work, L=L, U=U)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    tl.prof_enable(True)
    step()
    torch.cuda.synchronize()
    kern = tl.prof_query()
    tl.prof_enable(False)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        ipiv, _, _, info = step()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    flops = m * b * b - b ** 3 / 3.0
    res = float(torch.linalg.norm(A - L @ U) / torch.linalg.norm(A))
    lmax = float(L.abs().max())
    leaf_ms = kern.get("tslu_leaf", (1, 0.0))[1]
    return {"metric": "TSLU Gflop/s (LU with tournament pivoting)", "value": round(flops / (ms * 1e-3) / 1e9, 2),
            "unit": "Gflop/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "dtype": "f64", "data": "synthetic iid N(0,1), seed 0",
            "config": {"workload": f"tsqr_tslu {m}x{b}", "m": m, "b": b, "row_block": 4096, "tree": "binary",
                       "stack_rows": 256},
            "info": int(info.item()), "rel_residual_A_minus_LU": res, "max_abs_L": lmax,
            "kernels_ms_per_step": {k: round(v[1], 4) for k, v in kern.items()},
            "leaf_ms": round(leaf_ms, 4)}


def run_chol(args):
    print(json.dumps(measure_chol(args, args.steps, args.warmup)), flush=True)


def chol_update_flops(n, outer=256):
    """Flops of the 256-column block columns' trailing updates (the lower
    triangle of each trailing matrix, 2 K flops per entry)."""
    f = 0.0
    for j in range(0, n, outer):
        jend = min(j + outer, n)
        t = n - jend
        f += 2.0 * (jend - j) * t * (t + 1) / 2.0
    return f


def measure_chol(args, steps, warmup, n=8192):
    """In-place Cholesky of an n x n SPD Gram matrix G G^T / 2n (G iid
    N(0,1), n x 2n); useful flops n^3/3.  torch.linalg.cholesky on the same
    matrix is timed beside it for context.  Each step restores A by a device
    copy outside the timed interval."""
    import numpy as np
    import torch
    import paper_0912_2572_amd as tl
    import synth
    dev = torch.device("cuda:0")
    g = torch.as_tensor(synth.spd_gram_factor(n, seed=0)).to(dev)
    A0 = (g @ g.t()) / (2 * n)
    A0 = (0.5 * (A0 + A0.t())).t().contiguous().t()
    del g
    A = torch.empty_like(A0).t().contiguous().t()
    info = torch.empty(1, dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream()

    def step():
        A.copy_(A0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        tl.cholesky(A, info)
        e1.record(st)
        return e0, e1
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    tl.prof_enable(True)
    step()
    torch.cuda.synchronize()
    kern = tl.prof_query()
    tl.prof_enable(False)
    evs = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in evs) / steps
    flops = n ** 3 / 3.0
    L = torch.tril(A)
    rng = np.random.default_rng(1)
    ii = torch.as_tensor(rng.integers(0, n, 2000), device=dev)
    jj = torch.as_tensor(rng.integers(0, n, 2000), device=dev)
    rec = (L[ii] * L[jj]).sum(dim=1)
    back = float(((rec - A0[ii, jj]).abs() / (L[ii].abs() * L[jj].abs()).sum(dim=1)).max())
    # torch's own Cholesky (rocSOLVER) on the same matrix, for context
    for _ in range(warmup):
        torch.linalg.cholesky(A0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        Lt = torch.linalg.cholesky(A0)
    e1.record()
    torch.cuda.synchronize()
    torch_ms = e0.elapsed_time(e1) / steps
    diff = float((Lt - L).abs().max() / L.abs().max())
    syrk_ms = kern.get("chol_syrk", (1, 0.0))[1]
    syrk_tf = chol_update_flops(n) / (syrk_ms * 1e-3) / 1e12 if syrk_ms > 0 else None
    return {"metric": "Cholesky Gflop/s (n^3/3 useful flops)", "value": round(flops / (ms * 1e-3) / 1e9, 2),
            "unit": "Gflop/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "dtype": "f64", "data": "synthetic SPD Gram G G^T/2n, G iid N(0,1), seed 0",
            "config": {"workload": f"tsqr_cholesky {n}x{n}", "n": n, "block_column": 256, "panel": 64},
            "info": int(info.item()), "sampled_backward_error": back, "max_rel_diff_vs_torch": diff,
            "torch_linalg_cholesky_ms": round(torch_ms, 4),
            "speedup_vs_torch": round(torch_ms / ms, 3),
            "kernels_ms_per_step": {k: round(v[1], 4) for k, v in kern.items()},
            "launches": {k: v[0] for k, v in kern.items()},
            "syrk_tflops": None if syrk_tf is None else round(syrk_tf, 2),
            "syrk_frac_fp64_mfma_peak": None if syrk_tf is None else round(syrk_tf / 78.6, 4)}


def run_calu(args):
    print(json.dumps(measure_calu(args, args.steps, args.warmup)), flush=True)


def measure_calu(args, steps, warmup, n=4096, row_block=256):
    """CALU (LU with tournament-pivoted 64-column panels) of an n x n N(0,1)
    matrix; each panel's TSLU uses row_block-row domains and the binary
    tree.  Useful flops 2n^3/3.  torch.linalg.lu_factor (partial pivoting)
    on the same matrix is timed beside it for context.  Each step restores
    A by a device copy outside the timed interval."""
    import torch
    import paper_0912_2572_amd as tl
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    A0 = torch.randn((n, n), generator=g, device=dev, dtype=torch.float64).t()
    A = torch.empty((n, n), device=dev, dtype=torch.float64).t()
    o = tl.opts(row_block=row_block)
    work = torch.empty(tl.lib().tsqr_calu_workspace_bytes(n, n, ctypes_ref(o)), dtype=torch.uint8, device=dev)
    ipiv = torch.empty(n, dtype=torch.int64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream()

    def step():
        A.copy_(A0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        tl.calu(A, o, work=work, ipiv=ipiv, info=info)
        e1.record(st)
        return e0, e1
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    tl.prof_enable(True)
    step()
    torch.cuda.synchronize()
    kern = tl.prof_query()
    tl.prof_enable(False)
    evs = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in evs) / steps
    # P A = L U on the device
    L = torch.tril(A, -1) + torch.eye(n, device=dev, dtype=torch.float64)
    U = torch.triu(A)
    perm = list(range(n))
    for i, p in enumerate(ipiv.cpu().tolist()):
        perm[i], perm[p] = perm[p], perm[i]
    res = float(torch.linalg.norm(A0[torch.as_tensor(perm, device=dev)] - L @ U) / torch.linalg.norm(A0))
    lmax = float(L.abs().max())
    for _ in range(warmup):
        torch.linalg.lu_factor(A0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        torch.linalg.lu_factor(A0)
    e1.record()
    torch.cuda.synchronize()
    torch_ms = e0.elapsed_time(e1) / steps
    flops = 2.0 * n ** 3 / 3.0
    return {"metric": "CALU Gflop/s (2n^3/3 useful flops)", "value": round(flops / (ms * 1e-3) / 1e9, 2),
            "unit": "Gflop/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "dtype": "f64", "data": "synthetic iid N(0,1), torch Philox seed 5",
            "config": {"workload": f"tsqr_calu {n}x{n}", "n": n, "panel": 64, "row_block": row_block,
                       "tree": "binary", "stack_rows": 256},
            "info": int(info.item()), "rel_residual_PA_minus_LU": res, "max_abs_L": lmax,
            "torch_linalg_lu_factor_ms": round(torch_ms, 4), "speedup_vs_torch": round(torch_ms / ms, 3),
            "kernels_ms_per_step": {k: round(v[1], 4) for k, v in kern.items()}}


def run_wide(args):
    print(json.dumps(measure_wide(args, args.steps, args.warmup, domains=args.domains)), flush=True)


def measure_wide(args, steps, warmup, m=262144, n=1024, domains=0):
    """Wider than 64 columns: FP64 factor + 1-RHS least squares of an m x n
    N(0,1) matrix in 64-column panels (each a TSQR of the rows below the
    previous ones, its Q^T applied to the columns to its right); useful
    flops 2mn^2 - 2n^3/3 (R) + 4mn + n^2 (the solve)."""
    import torch
    import paper_0912_2572_amd as tl
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    A = torch.randn((n, m), generator=g, device=dev, dtype=torch.float64).t()
    b = torch.randn((m, 1), generator=g, device=dev, dtype=torch.float64)
    o = tl.opts(row_block=0 if domains else 4096, lsq_max_rhs=1, domains=domains)
    work = torch.empty(tl.workspace_bytes(m, n, o), dtype=torch.uint8, device=dev)
    X = tl.empty_colmajor(n, 1, device=dev)
    res = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)

    def step():
        f, _, _, _ = tl.factor_solve(A, b, o, work=work, X=X, resid=res, info=info)
        return f
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    tl.prof_enable(True)
    step()
    torch.cuda.synchronize()
    kern = tl.prof_query()
    tl.prof_enable(False)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    fl = 2.0 * m * n * n - 2.0 * n ** 3 / 3.0 + 4.0 * m * n + n * n
    eta = _eta(A, X[:, 0], b[:, 0])
    return {"metric": "TSQR/CAQR Gflop/s (factor + LSQ), FP64, 64-column panels", "value": round(fl / (ms * 1e-3) / 1e9, 2),
            "unit": "Gflop/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "dtype": "f64", "data": "synthetic N(0,1), torch Philox seed 3",
            "config": {"workload": f"tsqr_panels_lsq {m}x{n}", "m": m, "n": n,
                       "row_block": None if domains else 4096, "domains": tl.plan_info(m, n, o)[0],
                       "partition": "balanced" if domains else "row_block", "panels": n // 64},
            "info": int(info.item()), "eta": eta,
            "kernels_ms_per_step": {k: round(v[1], 4) for k, v in kern.items()}}


def run_orth(args):
    print(json.dumps(measure_orth(args, steps=args.steps, warmup=args.warmup)), flush=True)


def measure_orth(args, steps, warmup, m=1 << 20, b=16, nblocks=16):
    """Block orthogonalisation inside a block Krylov loop: a basis of
    `nblocks` blocks of b columns for a diagonal operator D, each new block
    D Q_j orthogonalised against all previous ones (two block Gram-Schmidt
    passes, then TSQR and the thin Q).  One step is the whole loop."""
    import torch
    import paper_0912_2572_amd as tl
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(2)
    W0 = torch.randn((b, m), generator=g, device=dev, dtype=torch.float64).t()
    d = torch.linspace(1.0, 2.0, m, device=dev, dtype=torch.float64)
    Vg = tl.empty_colmajor(m, nblocks * b, device=dev)
    o = tl.opts(row_block=4096)
    work = torch.empty(tl.lib().tsqr_block_orth_workspace_bytes(m, (nblocks - 1) * b, b, ctypes_ref(o)),
                       dtype=torch.uint8, device=dev)
    Hs = [tl.empty_colmajor(max(j * b, 1), b, device=dev) for j in range(nblocks)]
    Rs = [tl.empty_colmajor(b, b, device=dev) for _ in range(nblocks)]

    def step():
        for j in range(nblocks):
            Wj = Vg[:, j * b:(j + 1) * b]
            if j == 0:
                Wj.copy_(W0)
                tl.block_orth(None, Wj, o, R=Rs[j], work=work)
            else:
                torch.mul(Vg[:, (j - 1) * b:j * b], d[:, None], out=Wj)
                tl.block_orth(Vg[:, :j * b], Wj, o, H=Hs[j], R=Rs[j], work=work)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    tl.prof_enable(True)
    step()
    torch.cuda.synchronize()
    kern = tl.prof_query()
    tl.prof_enable(False)
    G = Vg.t() @ Vg
    orth_err = float(torch.linalg.norm(G - torch.eye(nblocks * b, device=dev, dtype=torch.float64)))
    # useful flops: four block products per block (2 m nv b each) and TSQR +
    # thin Q of the m x b block (2 (2 m b^2 - 2 b^3 / 3))
    flops = sum(4 * 2.0 * m * (j * b) * b + 2 * (2.0 * m * b * b - 2.0 * b ** 3 / 3.0) for j in range(nblocks))
    # algorithmic HBM bytes: V read four times, W read/written by the
    # projections, the block read by TSQR, V and Q written by TSQR
    alg = sum(4 * 8.0 * m * j * b + 6 * 8.0 * m * b + 3 * 8.0 * m * b for j in range(nblocks))
    upd_cnt, upd_ms = kern.get("orth_proj_update", (0, 0.0))
    upd_bytes = sum(2 * (8.0 * m * j * b + 16.0 * m * b) for j in range(1, nblocks))
    line = {
        "metric": "block orthogonalisation (block Gram-Schmidt x2 + TSQR) Gflop/s in a block Krylov loop",
        "value": round(flops / (ms * 1e-3) / 1e9, 2), "unit": "Gflop/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic: first block N(0,1) (torch Philox seed 2), operator diag(linspace(1, 2, m))",
        "config": {"workload": f"tsqr_block_krylov {m}x({nblocks}x{b})", "m": m, "b": b, "blocks": nblocks},
        "roofline": {"kernel": "whole loop", "bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_step": alg},
        "proj_update_gbs": round(upd_bytes / (upd_ms * 1e-3) / 1e9, 1) if upd_ms else None,
        "kernels_ms_per_step": {k: round(v[1], 4) for k, v in kern.items()},
        "basis_orthogonality_fro": orth_err,
    }
    del Vg, work
    torch.cuda.empty_cache()
    return line


def ctypes_ref(o):
    import ctypes
    return ctypes.byref(o)


def run_copy(args):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    nbytes = 1 << 30
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(args.warmup + args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
                      "launches": args.warmup + args.steps}), flush=True)


if __name__ == "__main__":
    main()
