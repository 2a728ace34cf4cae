"""Benchmark: preconditioned GP log-likelihood + gradient evaluations per second.

One step = one full gp_mll_grad call (preconditioner build, probes, batched
preconditioned CG with on-the-fly K_hat tiles, Lanczos quadrature, derivative
sweep and preconditioner terms) on the n = 100,000, d = 16 RBF-ARD workload
(rank-100 pivoted Cholesky, 64 probes, CG tolerance 1e-6), inputs resident in
HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64] [--no-cpu] [--no-batch]

The headline runs the K_hat V tiles in split BF16 (BF16X3: hi + lo halves, three
products, FP32 accumulation), the configuration the metric is quoted on.  Beside it
the line reports the FP16X3 and FP64 tile precisions on the same workload (FP16X3
tiles run at the same speed, and their finer split needs the FP64 iteration count),
the randomized Nystrom and random Fourier feature preconditioners at the same rank,
posterior prediction at 256 test points (gp_predict) and the 64-problem ragged batch
(gp_batch_mll_grad) as extra fields.
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

METRIC = "log-lik+grad evals/sec at n=100k (split-prec vs FP64 GPU); K̂·V MFMA util"
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 MFMA
PEAK_FP64_TFLOPS = 78.6


# Counter readings of the split-precision tile kernel on this workload, per launch,
# for each kernel instance (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch, over `bench.py --tiles-only --tile-precision P`), each scaled by what the
# same counter reads for a 1 GiB elementwise copy, and the MFMA counters of the same
# launches.  Instance "v3" takes three-piece search directions (BF16x3, the first
# V3_ITERS CG iterations), "v2" two-piece ones.  They describe the kernel source whose
# hash is given, launched on the given grid; once either changes they are stale and
# are not reported.
V3_ITERS = 16          # the library's kBf16V3Iters
TILE_COUNTERS = {
    "fp16x3": {
        "kernel_source_sha256_16": "4db75bbb45375324",
        "grid": [391, 5],
        "v2": {"fetch_kib": 280408.0, "fetch_scale": 1048576.0 / 524304.0,
               "write_kib": 143761.0, "write_scale": 1.0,
               "mfma_insts": 3.131e8, "mfma_busy_cycles": 5.0096e9, "gui_active_per_xcd": 7.47607e7 / 8},
    },
    "bf16x3": {
        "kernel_source_sha256_16": "4db75bbb45375324",
        "grid": [391, 5],
        "v3": {"fetch_kib": 363819.0, "fetch_scale": 1048576.0 / 524310.0,
               "write_kib": 141717.0, "write_scale": 1.0,
               "mfma_insts": 3.91375e8, "mfma_busy_cycles": 6.26201e9, "gui_active_per_xcd": 8.71291e7 / 8},
        "v2": {"fetch_kib": 280158.0, "fetch_scale": 1048576.0 / 524310.0,
               "write_kib": 141916.0, "write_scale": 1.0,
               "mfma_insts": 3.131e8, "mfma_busy_cycles": 5.0096e9, "gui_active_per_xcd": 7.47617e7 / 8},
    },
}


def tile_launch_mix(precision, reps):
    """Launches per kernel instance among `reps` full-width CG products."""
    if precision == "bf16x3":
        n3 = min(reps, V3_ITERS)
        return {"v3": n3, "v2": reps - n3}
    return {"v2": reps}


def tile_source_text(khat: str) -> str:
    """k_khat.hip without its part-0 sections (the staging and reduction kernels,
    compiled as a translation unit of their own, not the tile kernels)."""
    import re
    return re.sub(r"#if GPMLL_KHAT_PART == 0\n.*?#endif  // part 0\n", "", khat, flags=re.S)


def bf16_tile_source_hash():
    """First 16 hex digits of the SHA-256 of the split-precision tile kernel's sources:
    k_khat.hip without its part-0 sections, then the shared header gpmll_impl.h."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2107_00243_amd", "csrc")
    h = hashlib.sha256()
    h.update(tile_source_text(open(os.path.join(csrc, "k_khat.hip")).read()).encode())
    h.update(open(os.path.join(csrc, "gpmll_impl.h"), "rb").read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def tile_flops(n, d, t):
    """Algorithmic flops of one K_hat V product: 2 n^2 (d + t) (distance and tile x V
    contractions) plus n^2 kernel-map evaluations counted as one flop each."""
    return 2.0 * n * n * (d + t) + float(n) * n


def run_gpu(pr, precision, steps, warmup, sync_every=1, timed=True):
    import torch
    from paper_2107_00243_amd import binding as B
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    opt = B.make_options(precision, pr.num_probes, pr.max_iters, pr.tol, pr.probe_seed, 0, sync_every)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, pr.rank))
    logp = torch.zeros(1, dtype=torch.float64, device=dev)
    grad = torch.zeros(len(pr.theta), dtype=torch.float64, device=dev)
    st = B.Stats(pr.num_probes, pr.rank)
    # one evaluation with statistics (untimed) for iteration counts and accuracy
    B.gp_mll_grad(prob, pr.theta, opt, pr.rank, None, ws, logp, grad, st)
    torch.cuda.synchronize()
    info = {"logp": float(logp.cpu()[0]), "grad": grad.cpu().numpy(), "iters_max": int(st.iters_max),
            "iters_mean": float(np.mean(st.col_iters)), "iters_y": int(st.col_iters[0]),
            "flags": int(st.flags), "rank": int(st.rank_achieved), "datafit": float(st.datafit),
            "logdet": float(st.logdet_estimate)}
    if not timed:
        del ws
        torch.cuda.empty_cache()
        return info
    for _ in range(warmup):
        B.gp_mll_grad(prob, pr.theta, opt, pr.rank, None, ws, logp, grad)
    torch.cuda.synchronize()
    log(f"[bench] {precision}: timing {steps} steps")
    t0 = time.perf_counter()
    for _ in range(steps):
        B.gp_mll_grad(prob, pr.theta, opt, pr.rank, None, ws, logp, grad)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info["ms_per_step"] = 1e3 * dt / steps
    info["evals_per_s"] = steps / dt
    # tile-kernel duration in the same launch configuration, HIP events on the stream:
    # the full-width launches of one evaluation (every CG iteration but the last,
    # which finishes a few straggling columns), in the order CG issues them; with
    # BF16x3 tiles the first 16 take three-piece search directions
    reps = max(1, info["iters_max"] - 1)
    ms, grid = B.gp_khat_profile(prob, pr.theta, opt, reps, ws)
    info["tile_ms"] = ms
    info["tile_launches_timed"] = reps
    info["tile_grid"] = list(grid)
    del ws
    torch.cuda.empty_cache()
    return info


def run_batched(steps, warmup, precision=None, sync_every=1):
    """The 64-problem ragged batch (n_b ~ U{500..8000}, d 4, RBF, rank 20, 16 probes,
    FP64 tiles unless precision is given): one gp_batch_mll_grad call evaluates log p
    and the gradient of all 64 problems."""
    import torch
    import synthgp
    from paper_2107_00243_amd import binding as B
    probs = synthgp.batched_rbf_64()
    pr0 = probs[0]
    dev = torch.device("cuda:0")
    X = torch.tensor(np.concatenate([p.X for p in probs]), device=dev)
    y = torch.tensor(np.concatenate([p.y for p in probs]), device=dev)
    bt = B.Batch(X, y, [p.n for p in probs], pr0.kernel, pr0.ard)
    prec = precision or pr0.precision
    opt = B.make_options(prec, pr0.num_probes, pr0.max_iters, pr0.tol, pr0.probe_seed, 0, sync_every)
    ws = B.alloc_workspace(B.gp_batch_workspace_size(bt, opt, pr0.rank))
    theta = np.stack([p.theta for p in probs])
    nb, P = len(probs), len(pr0.theta)
    logp = torch.zeros(nb, dtype=torch.float64, device=dev)
    grad = torch.zeros(nb * P, dtype=torch.float64, device=dev)
    st = B.BatchStats(nb)
    B.gp_batch_mll_grad(bt, theta, opt, pr0.rank, ws, logp, grad, st)
    for _ in range(warmup):
        B.gp_batch_mll_grad(bt, theta, opt, pr0.rank, ws, logp, grad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        B.gp_batch_mll_grad(bt, theta, opt, pr0.rank, ws, logp, grad)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    n = np.array([p.n for p in probs], dtype=np.float64)
    pair_iters = float(np.sum(n * n * st.iters))
    return {"value": 1.0 / dt, "unit": "batch evals/s (64 problems, log p + gradient each)",
            "problems_per_s": nb / dt, "ms_per_batch": 1e3 * dt, "steps": steps, "precision": prec,
            "sync_every": sync_every,
            "logp": logp.cpu().numpy().tolist(), "grad": grad.cpu().numpy().reshape(nb, P).tolist(),
            "problems": nb, "n_min": int(n.min()), "n_max": int(n.max()), "sum_n": int(n.sum()),
            "cg_iters_max": int(st.iters_max), "cg_iters_median": float(np.median(st.iters)),
            "kernel_pair_evaluations_in_cg": pair_iters,
            "flags_any": int(st.flags_any)}


def run_preconditioners(pr, steps, ref):
    """The other diagonal-plus-low-rank preconditioners of Table 1 on the headline
    workload at the same rank and tile precision (BF16x3): randomized Nystrom on
    uniform landmarks and random Fourier features.  A step is the preconditioner
    build plus one gp_mll_grad with that handle.  `ref` is the pivoted-Cholesky
    run, whose log p the estimates are compared with (both are stochastic
    estimates of the same quantity)."""
    import torch
    import synthgp
    from paper_2107_00243_amd import binding as B
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    opt = B.make_options("bf16x3", pr.num_probes, pr.max_iters, pr.tol, pr.probe_seed, 0, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, pr.rank))
    logp = torch.zeros(1, dtype=torch.float64, device=dev)
    grad = torch.zeros(len(pr.theta), dtype=torch.float64, device=dev)
    S = synthgp.uniform_landmarks(pr.n, pr.rank, seed=1)
    Wd = torch.tensor(synthgp.spectral_frequencies(pr.kernel, pr.rank // 2, pr.d, seed=1), device=dev)
    builders = {
        "nystrom_uniform_landmarks": lambda: B.gp_precond_build_nystrom(prob, pr.theta, pr.rank, S, ws),
        "random_fourier_features": lambda: B.gp_precond_build_rff(prob, pr.theta, pr.rank, Wd, ws),
    }
    out = {}
    for name, build in builders.items():
        st = B.Stats(pr.num_probes, pr.rank)
        h = build()
        B.gp_mll_grad(prob, pr.theta, opt, pr.rank, h, ws, logp, grad, st)
        B.gp_precond_free(h)
        torch.cuda.synchronize()
        lp = float(logp.cpu()[0])
        t0 = time.perf_counter()
        for _ in range(steps):
            h = build()
            B.gp_mll_grad(prob, pr.theta, opt, pr.rank, h, ws, logp, grad)
            B.gp_precond_free(h)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[name] = {"evals_per_s": 1.0 / dt, "ms_per_step": 1e3 * dt, "steps": steps,
                     "cg_iters_max": int(st.iters_max), "cg_iters_mean": float(np.mean(st.col_iters)),
                     "flags": int(st.flags), "logp": lp,
                     "rel_logp_vs_pivoted_cholesky": abs(lp - ref["logp"]) / abs(ref["logp"])}
        log(f"[bench] {name}: {1e3 * dt:.1f} ms/eval, iters {st.iters_max}")
    out["pivoted_cholesky"] = {"evals_per_s": ref["evals_per_s"], "cg_iters_max": ref["iters_max"],
                               "cg_iters_mean": ref["iters_mean"], "logp": ref["logp"]}
    del ws
    torch.cuda.empty_cache()
    return out


def run_predict(pr, nstar=256):
    """Posterior mean and latent variance at nstar test points drawn like the
    training inputs (gp_predict, BF16x3 tiles, chunks of 64 test points per CG
    call); the FP64-tile run of the same call gives the accuracy."""
    import torch
    from paper_2107_00243_amd import binding as B
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    Xs = torch.tensor(np.random.default_rng(7).uniform(0.0, 1.0, size=(nstar, pr.d)), device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    out = {}
    for prec in ("bf16x3", "fp64"):
        opt = B.make_options(prec, pr.num_probes, pr.max_iters, pr.tol, pr.probe_seed, 0, 1)
        ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, pr.rank))
        mean = torch.zeros(nstar, dtype=torch.float64, device=dev)
        var = torch.zeros(nstar, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.gp_predict(prob, pr.theta, opt, pr.rank, None, Xs, ws, mean, var)
        torch.cuda.synchronize()
        out[prec] = (time.perf_counter() - t0, mean.cpu().numpy(), var.cpu().numpy())
        del ws
        torch.cuda.empty_cache()
    dt, mb, vb = out["bf16x3"]
    _, m64, v64 = out["fp64"]
    return {"test_points": nstar, "seconds": dt, "test_points_per_s": nstar / dt, "precision": "bf16x3",
            "fp64_seconds": out["fp64"][0],
            "mean_err_vs_fp64": float(np.max(np.abs(mb - m64)) / np.max(np.abs(m64))),
            "var_err_vs_fp64_of_s": float(np.max(np.abs(vb - v64)) / pr.theta[-2])}


def tiles_only(pr, precision="bf16x3", reps=32, copy_bytes=1 << 30):
    """The tile kernel of one split precision alone in the bench's launch
    configuration (`reps` launches as CG iterations 0 .. reps-1 issue them: with
    BF16x3 tiles 16 with three-piece search directions, then two-piece ones), then
    a plain elementwise copy of copy_bytes (read copy_bytes, write copy_bytes) whose
    counter readings calibrate the HBM byte counters."""
    import torch
    from paper_2107_00243_amd import binding as B
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    opt = B.make_options(precision, pr.num_probes, pr.max_iters, pr.tol, pr.probe_seed, 0, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, pr.rank))
    ms, grid = B.gp_khat_profile(prob, pr.theta, opt, reps, ws)
    a = torch.ones(copy_bytes // 4, dtype=torch.float32, device=dev)
    c = torch.empty_like(a)
    torch.mul(a, 1.0, out=c)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    torch.mul(a, 1.0, out=c)
    e1.record()
    torch.cuda.synchronize()
    return {"precision": precision, "tile_ms": ms, "tile_grid": list(grid), "reps": reps,
            "copy_bytes_read": copy_bytes,
            "copy_bytes_written": copy_bytes, "copy_ms": e0.elapsed_time(e1)}


def cpu_baseline(pr, iters, budget_s=12.0):
    """The CPU oracle timed on a bounded sample of one evaluation of the same
    workload: its matrix-free K_hat V (plain-C direct differences, FP64, all host
    threads) on a block of rows, and its derivative contraction over M = A C^T on a
    block of rows, each scaled to all n rows; one evaluation is `iters` products
    plus one contraction (the preconditioner, probes and quadrature are
    negligible beside them)."""
    from oracle import gp_oracle as go
    n = pr.n
    t = 1 + pr.num_probes
    rng = np.random.default_rng(0)
    V = rng.standard_normal((n, t))
    w0 = time.perf_counter()
    go.khat_matvec(pr.X, pr.theta, pr.kernel, pr.ard, V, rows=np.arange(256), native=True)
    w = time.perf_counter() - w0
    rows = int(min(n, max(256, 256 * 0.6 * budget_s / max(w, 1e-3))))
    c0, w0 = time.process_time(), time.perf_counter()
    go.khat_matvec(pr.X, pr.theta, pr.kernel, pr.ard, V, rows=np.arange(rows), native=True)
    wall_mv = time.perf_counter() - w0
    cpu = time.process_time() - c0
    A, C = V, rng.standard_normal((n, t))
    w0 = time.perf_counter()
    go.dkhat_contract_lowrank(pr.X, pr.theta, pr.kernel, pr.ard, A, C, row_range=(0, 64))
    w = time.perf_counter() - w0
    drows = int(min(n, max(64, 64 * 0.4 * budget_s / max(w, 1e-3))))
    w0 = time.perf_counter()
    go.dkhat_contract_lowrank(pr.X, pr.theta, pr.kernel, pr.ard, A, C, row_range=(0, drows))
    wall_dk = time.perf_counter() - w0
    per_eval = iters * wall_mv * n / rows + wall_dk * n / drows
    return {"value": 1.0 / per_eval, "unit": "evals/s", "cores": max(1, int(round(cpu / wall_mv))),
            "kind": "oracle",
            "sample": f"oracle matrix-free K_hat V on {rows} of {n} rows x {t} rhs ({wall_mv:.1f} s) and its "
                      f"derivative contraction on {drows} rows ({wall_dk:.1f} s), scaled to n rows and to "
                      f"{iters} products + 1 contraction per evaluation",
            "host_cpus": os.cpu_count()}


def tile_roofline(n, d, t, run, precision):
    """Roofline of the split-precision tile kernel from the run's HIP-event launch
    time; traffic and MFMA counters only while the recorded readings still match
    the kernel source and grid."""
    flops = tile_flops(n, d, t)
    achieved = flops / (run["tile_ms"] * 1e-3) / 1e12
    name = {"fp16x3": "k_khat_bf16<0, 2, 4, 4, true, 1, 2> (K_hat V tile, FP16x3: 4 MFMA column tiles + 1 VALU "
                      "column)",
            "bf16x3": "k_khat_bf16<0, 2, 4, 4, false, 1, 3|2> (K_hat V tile, BF16x3: 4 MFMA column tiles + 1 VALU "
                      "column; search directions in 3 BF16 pieces for the first 16 CG iterations, then 2)"
            }[precision]
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None, "kernel": name,
            "launch_grid": run["tile_grid"], "algorithmic_flops_per_launch": flops, "avg_launch_ms": run["tile_ms"],
            "launches_averaged": run.get("tile_launches_timed")}
    tc = TILE_COUNTERS.get(precision)
    reps = run.get("tile_launches_timed") or 0
    mix = {k: c for k, c in tile_launch_mix(precision, reps).items() if c > 0}
    if (tc is not None and n == 100000 and reps > 0 and bf16_tile_source_hash() == tc["kernel_source_sha256_16"]
            and list(run["tile_grid"]) == tc["grid"] and all(k in tc for k in mix)):
        # launch-weighted means over the instances the timed launches used
        def mean(f):
            return sum(c * f(tc[k]) for k, c in mix.items()) / reps
        roof["traffic"] = 1024.0 * mean(lambda r: r["fetch_kib"] * r["fetch_scale"] + r["write_kib"] * r["write_scale"])
        roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        roof["traffic_gbps"] = roof["traffic"] / (run["tile_ms"] * 1e-3) / 1e9
        issued = mean(lambda r: r["mfma_insts"]) * 16384.0
        roof["issued_mfma_flops_per_launch"] = issued
        roof["issued_mfma_frac_of_peak"] = issued / (run["tile_ms"] * 1e-3) / 1e12 / PEAK_BF16_TFLOPS
        roof["mfma_busy_frac"] = (sum(c * tc[k]["mfma_busy_cycles"] for k, c in mix.items())
                                  / sum(c * tc[k]["gui_active_per_xcd"] * 1024 for k, c in mix.items()))
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem ragged batch")
    ap.add_argument("--batch-only", action="store_true", help="only the 64-problem ragged batch (one JSON line)")
    ap.add_argument("--batch-sync-every", type=int, default=1,
                    help="host convergence poll every q CG iterations in --batch-only (0: none)")
    ap.add_argument("--batch-precision", default=None, help="tile precision of --batch-only")
    ap.add_argument("--no-precond", action="store_true",
                    help="skip the Nystrom / RFF preconditioner and posterior prediction legs")
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--tiles-only", action="store_true",
                    help="only the split-precision tile kernel (10 launches) and a 1 GiB elementwise copy, "
                         "for counters")
    ap.add_argument("--tile-precision", default="bf16x3", choices=["bf16x3", "fp16x3"],
                    help="tile precision of --tiles-only")
    ap.add_argument("--tiles-workload", default="rbf_ard_100k", choices=["rbf_ard_100k", "gmm_matern32_300k"],
                    help="workload of --tiles-only")
    ap.add_argument("--table-s1", action="store_true",
                    help="only the Table S1 experiment (bias and variance, 25 repetitions; one JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(the whole problem sits on one GPU); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synthgp
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.table_s1:
        print(json.dumps(table_s1()))
        return
    if args.batch_only:
        r = run_batched(args.steps, args.warmup, args.batch_precision, args.batch_sync_every)
        r.pop("logp")
        r.pop("grad")
        print(json.dumps(r))
        return
    pr = synthgp.rbf_ard_100k(n=args.n)
    n, d, t = pr.n, pr.d, 1 + pr.num_probes
    log(f"[bench] workload rbf_ard_100k n={n} d={d} t={t} rank={pr.rank}")
    if args.tiles_only:
        if args.tiles_workload != "rbf_ard_100k":
            pr = getattr(synthgp, args.tiles_workload)()
            log(f"[bench] tiles of {pr.name} n={pr.n} d={pr.d} {pr.kernel}")
        r = tiles_only(pr, args.tile_precision)
        r["workload"] = pr.name
        print(json.dumps(r))
        return

    # headline: BF16X3 tiles; FP16X3 beside it (same tile kernel speed, fewer CG iterations)
    bf = run_gpu(pr, "bf16x3", args.steps, args.warmup)
    log(f"[bench] bf16x3: {bf['ms_per_step']:.2f} ms/eval, iters {bf['iters_max']}, tile {bf['tile_ms']:.3f} ms")
    h16 = run_gpu(pr, "fp16x3", args.steps, args.warmup)
    log(f"[bench] fp16x3: {h16['ms_per_step']:.2f} ms/eval, iters {h16['iters_max']}, tile {h16['tile_ms']:.3f} ms")
    out_fp64 = None
    if not args.no_fp64:
        f64 = run_gpu(pr, "fp64", args.fp64_steps, 0)
        log(f"[bench] fp64: {f64['ms_per_step']:.2f} ms/eval, iters {f64['iters_max']}, tile {f64['tile_ms']:.3f} ms")
        out_fp64 = {
            "value": f64["evals_per_s"], "ms_per_step": f64["ms_per_step"], "iters_max": f64["iters_max"],
            "tile_ms": f64["tile_ms"], "tile_tflops": tile_flops(n, d, t) / (f64["tile_ms"] * 1e-3) / 1e12,
            "tile_frac_fp64_peak": tile_flops(n, d, t) / (f64["tile_ms"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "ms_per_cg_iteration": f64["ms_per_step"] / max(1, f64["iters_max"]),
        }
    roofline = tile_roofline(n, d, t, bf, "bf16x3")
    pred = None
    if not args.no_precond:
        log("[bench] posterior prediction at 256 test points")
        pred = run_predict(pr)
        log(f"[bench] predict: {pred['seconds']:.2f} s for {pred['test_points']} test points")
    precs = None
    if not args.no_precond:
        log("[bench] other preconditioners of Table 1 (BF16x3)")
        precs = run_preconditioners(pr, 2, bf)
    batched = None
    if not args.no_batch:
        log("[bench] 64-problem ragged batch")
        batched = run_batched(2, 1, sync_every=8)
        log(f"[bench] batch: {batched['ms_per_batch']:.1f} ms per call, iters max {batched['cg_iters_max']}")
        # FP32 tiles on the same batch: faster, and how far from the FP64-tile results
        b32 = run_batched(1, 0, "fp32", sync_every=8)
        lp64, lp32 = np.array(batched.pop("logp")), np.array(b32.pop("logp"))
        g64, g32 = np.array(batched.pop("grad")), np.array(b32.pop("grad"))
        relg = np.linalg.norm(g32 - g64, axis=1) / np.linalg.norm(g64, axis=1)
        batched["fp32_tiles"] = {"ms_per_batch": b32["ms_per_batch"], "cg_iters_max": b32["cg_iters_max"],
                                 "max_rel_logp_vs_fp64": float(np.max(np.abs(lp32 - lp64) / np.abs(lp64))),
                                 "max_rel_grad_vs_fp64": float(relg.max()),
                                 "problems_within_1e-2_grad": int(np.sum(relg < 1e-2))}
        log(f"[bench] batch fp32: {b32['ms_per_batch']:.1f} ms per call")
    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle sample")
        cpu = cpu_baseline(pr, bf["iters_max"])
    rec = {
        "metric": METRIC, "value": bf["evals_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": bf["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"rbf_ard_100k: n={n}, d={d}, RBF ARD ls~LogU[0.1,1], sigma2=1e-3, "
                               f"rank {pr.rank} pivoted Cholesky, {pr.num_probes} probes, CG tol {pr.tol}, "
                               f"BF16x3 tiles (split BF16, FP32 accumulation), FP64 recurrences",
                   "n": n, "d": d, "num_probes": pr.num_probes, "rank": pr.rank, "precision": "bf16x3",
                   "cg_iters_max": bf["iters_max"], "cg_iters_mean": bf["iters_mean"],
                   "cg_iters_y_column": bf["iters_y"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64_gpu": out_fp64,
        "speedup_vs_fp64_gpu": (bf["evals_per_s"] / out_fp64["value"]) if out_fp64 else None,
        # the same comparison at equal iteration count: evaluation time per CG iteration
        # (the longest column's count), which also carries the fixed per-evaluation work
        "ms_per_cg_iteration": bf["ms_per_step"] / max(1, bf["iters_max"]),
        "speedup_vs_fp64_gpu_per_iteration": ((out_fp64["ms_per_cg_iteration"]
                                               / (bf["ms_per_step"] / max(1, bf["iters_max"])))
                                              if out_fp64 else None),
        "fp16x3_gpu": {"value": h16["evals_per_s"], "ms_per_step": h16["ms_per_step"],
                       "iters_max": h16["iters_max"], "iters_mean": h16["iters_mean"], "tile_ms": h16["tile_ms"],
                       "tile_tflops": tile_flops(n, d, t) / (h16["tile_ms"] * 1e-3) / 1e12,
                       "speedup_vs_fp64_gpu": (h16["evals_per_s"] / out_fp64["value"]) if out_fp64 else None,
                       "ms_per_cg_iteration": h16["ms_per_step"] / max(1, h16["iters_max"]),
                       "roofline": tile_roofline(n, d, t, h16, "fp16x3")},
        "batched_rbf_64": batched,
        "preconditioners_bf16x3": precs,
        "predict": pred,
    }
    if out_fp64 is not None:
        rec["accuracy_vs_fp64_gpu"] = {
            "rel_logp": abs(bf["logp"] - f64["logp"]) / abs(f64["logp"]),
            "rel_grad": float(np.linalg.norm(bf["grad"] - f64["grad"]) / np.linalg.norm(f64["grad"])),
        }
        rec["fp16x3_gpu"]["accuracy_vs_fp64_gpu"] = {
            "rel_logp": abs(h16["logp"] - f64["logp"]) / abs(f64["logp"]),
            "rel_grad": float(np.linalg.norm(h16["grad"] - f64["grad"]) / np.linalg.norm(f64["grad"])),
        }
    log("[bench] errors against the oracle references")
    rec["accuracy_vs_oracle"] = reference_errors((bf["logp"], bf["grad"]))
    rec["env"] = run_environment()
    print(json.dumps(rec))


GOLDEN = os.path.join(ROOT, "tests", "golden")


def _golden(name):
    path = os.path.join(GOLDEN, name)
    return json.load(open(path)) if os.path.exists(path) else None


def _relerr(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def reference_errors(headline=None):
    """Errors of the GPU estimate against the CPU oracle's stored references
    (tests/golden/oracle_<workload>.json, written by tests/golden/make_full_size.py):
    the same-probe estimate of Algorithms 1 and 2 on every workload, and the exact
    Eq. (1) / Eq. (2) targets where a dense factor fits (n <= 20,000).  The
    n = 100,000 headline takes its own run's numbers (headline = (logp, grad))."""
    import synthgp
    out = {}
    for workload, precision in (("plain_rbf_1000", "fp64"), ("matern52_ard_20k", "fp32"),
                                ("rbf_ard_100k", "bf16x3")):
        ref = _golden(f"oracle_{workload}.json")
        if ref is None:
            continue
        if workload == "rbf_ard_100k":
            if headline is None:
                continue
            lp, g, st = headline[0], headline[1], None
        else:
            pr = getattr(synthgp, workload)()
            r = run_gpu(pr, precision, 0, 0, timed=False)
            lp, g, st = r["logp"], r["grad"], r
        est = ref["estimate"]
        e = {"precision": precision, "same_probe_rel_logp": abs(lp - est["logp"]) / abs(est["logp"]),
             "same_probe_rel_grad": _relerr(g, est["grad"])}
        ex = ref.get("exact")
        if ex is not None and st is not None:
            e.update({"exact_rel_logp": abs(lp - ex["logp"]) / abs(ex["logp"]),
                      "exact_rel_datafit": abs(st["datafit"] - ex["datafit"]) / abs(ex["datafit"]),
                      "exact_rel_logdet": abs(st["logdet"] - ex["logdet"]) / abs(ex["logdet"]),
                      "exact_rel_grad": _relerr(g, ex["grad"])})
        else:
            e["exact"] = "out of reach (a dense factor of K_hat needs n^2 doubles)"
        out[workload] = e
    return out


def table_s1(reps=25):
    """Table S1 (supplement, synthetic data) on the GPU: relative bias and variance
    of log p and of its outputscale, lengthscale and noise derivatives over `reps`
    probe seeds, preconditioner rank 0 and 128 with 128 probes, FP64 tiles, for the
    three kernels and d = 1, 2, 3 (exact targets stored by
    tests/golden/make_table_s1.py)."""
    import synthgp
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from test_gpu_trends import COLUMNS, table_s1_errors
    exact = _golden("table_s1_exact.json")["problems"]
    rows = []
    for kernel in synthgp.TABLE_S1_KERNELS:
        for d in (1, 2, 3):
            pr = synthgp.table_s1(kernel, d)
            for rank in (0, 128):
                t0 = time.perf_counter()
                e, iters, flags = table_s1_errors(pr, exact[pr.name], rank, reps)
                row = {"kernel": kernel, "d": d, "precond_rank": rank, "probes": pr.num_probes, "reps": reps,
                       "cg_iters_max": iters, "flags": flags}
                for c, b, v in zip(COLUMNS, np.abs(e.mean(axis=0)), e.var(axis=0)):
                    row[c] = {"bias": float(b), "var": float(v)}
                rows.append(row)
                log(f"[bench] Table S1 {kernel} d={d} rank {rank}: " + "  ".join(
                    f"{c} {row[c]['bias']:.0e}/{row[c]['var']:.0e}" for c in COLUMNS)
                    + f"  ({time.perf_counter() - t0:.1f} s)")
    return {"experiment": "Table S1: n=10000 N(0,I_d), sigma2=1e-2, 128 probes, rank 0 vs 128, FP64 tiles",
            "rows": rows}


def run_environment():
    """GPU, HIP and host CPU the numbers were taken on."""
    import platform
    import torch
    cpu = platform.processor()
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), cpu)
    except OSError:
        pass
    return {"gpu": torch.cuda.get_device_name(0), "hip": torch.version.hip, "torch": torch.__version__,
            "host_cpu": cpu, "host_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()
