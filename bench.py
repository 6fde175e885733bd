#!/usr/bin/env python3
"""Benchmark of the Lippmann-Schwinger Nystrom hot path on one MI355X.

Workload: the two-material disk (inclusion |x| < 0.5 with n = 3, annulus 0.5 < |x| < 1 with
n = 1 + 0.5 exp(-|x|^2)), k = 20, O-grid/annulus mesh with 15 inner cells (N = 58 500 nodes),
one plane wave along +x.  One step = one FP64 GMRES solve (no restart, x0 = 0) of L u = b to a
relative residual of 1e-8, every operator application being the far-field Green's sum over all
N(N-1) node pairs plus the sparse correction.

Reported: Green interactions per second over the timed solves (value), the time to a 1e-8
residual (ms_per_step), the far-sum kernel's roofline position (average launch duration from
HIP events the library records around each launch on the caller's stream), and the oracle's
own throughput on a bounded sample of the same far sum on the host cores.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 operations of the far-sum kernel per (target, source) pair on its z >= 12 branch
# (the smaller-argument branches do more): coordinates and k^2 r^2 (6), inverse fourth root
# Halley step (9), 1/z, z, 1/z^2 (3), modulus and phase polynomials (34), modulus scaling (1),
# reduction modulo pi, sign and sine/cosine (49), and 8 per right-hand side for the complex
# multiply-accumulate.  FMA counts as 2.
FLOPS_PER_PAIR_BASE = 102
FLOPS_PER_PAIR_PER_RHS = 8
PEAK_FP64_TFLOPS = 78.6       # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
# HBM bytes per far-kernel launch in this workload, from two rocprofv3 counter passes
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors that make a 1 GiB copy read 1 GiB and write
# 1 GiB; profiles/far_fp64_two_material_N58500_hbm_counters.md), valid for the kernel sources
# with this digest only: after any change to them the field is reported as null.
FAR_TRAFFIC_BYTES = 37_603_000 + 134_780_000
FAR_TRAFFIC_SOURCES = ("apply.hip", "hankel.h", "hankel_tables.h")
FAR_TRAFFIC_DIGEST = "13b4ecaf968990a5"


def far_traffic():
    import hashlib
    h = hashlib.sha256()
    for f in FAR_TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_17615_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return FAR_TRAFFIC_BYTES if h.hexdigest()[:16] == FAR_TRAFFIC_DIGEST else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _oracle_rows(args):
    """Worker: the oracle's punctured far sum for a block of target rows (host only)."""
    x, y, w, k, f, rows = args
    from oracle import green
    green.far_rows(x, y, w, k, f, rows)
    return len(rows)


def cpu_baseline(prob, rows_total=1024, workers=None):
    """Oracle far sum on a seeded sample of target rows, split over host processes."""
    import multiprocessing as mp

    import numpy as np

    from workloads import problems as P
    workers = workers or max(1, min(os.cpu_count() or 1, 16))
    n = prob.n_nodes
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(n, rows_total, replace=False))
    f = prob.m * P.random_vectors(n, 1, 0)[0]
    chunks = np.array_split(rows, workers * 4)
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_rows, [(prob.mesh.x, prob.mesh.y, prob.mesh.w, prob.k, f, c[:2]) for c in chunks[:workers]])
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_rows, [(prob.mesh.x, prob.mesh.y, prob.mesh.w, prob.k, f, c) for c in chunks]))
        dt = time.perf_counter() - t0
    gis = done * (n - 1) / dt / 1e9
    return {"value": gis, "unit": "GI/s", "cores": workers, "kind": "oracle",
            "sample": f"punctured Green's far sum (SciPy AMOS H0) for {done} seeded target rows x {n - 1} "
                      f"sources of the same workload ({done * (n - 1):.3g} interactions, {dt:.2f} s wall); "
                      f"the sparse correction rows (10 per subdomain and row) are excluded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="first run one elementwise kernel that reads and writes BYTES each "
                         "(calibrates a profiler's HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is described "
              f"in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    from workloads import problems as P
    prob = P.config2()
    n = prob.n_nodes

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle far sum on a row sample")
        cpu = cpu_baseline(prob)
        log(f"cpu baseline: {cpu['value']:.4f} GI/s on {cpu['cores']} processes")

    import torch

    import paper_2608_17615_amd as lsg
    if args.copy_probe:
        src = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy probe: read and wrote {src.numel() * 8} bytes")
        del src, dst
    log(f"setup: N={n}")
    t0 = time.perf_counter()
    op = lsg.Operator(lsg.Scatterer.from_mesh(prob.mesh, prob.m, prob.k))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup done in {setup_s:.2f} s (nnz {op.correction_nnz()})")
    b = torch.tensor(prob.incident(), device="cuda")

    for w in range(args.warmup):
        x, info = op.solve(b, tol=args.tol, maxit=args.maxit)
        log(f"warmup {w}: {info['iters']} iterations, {info['seconds']:.3f} s")
    torch.cuda.synchronize()
    op.profile(True)
    op.profile(reset=True)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        x, info = op.solve(b, tol=args.tol, maxit=args.maxit)
        infos.append(info)
        log(f"step {s}: {int(info['iters'][0])} iterations, relres {info['relres'][0]:.3e}, {info['seconds']:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = op.profile(reset=True)
    op.profile(False)

    n_apply = sum(int(i["n_apply_fp64"]) for i in infos)
    pairs = n * (n - 1)
    gis = n_apply * pairs / elapsed / 1e9
    far_avg_s = prof["far_ms"] / max(prof["far_launches"], 1) / 1e3
    flops = pairs * (FLOPS_PER_PAIR_BASE + FLOPS_PER_PAIR_PER_RHS * 1)
    achieved = flops / far_avg_s / 1e12
    out = {
        "metric": "Green interactions/s + time to 1e-8 residual, batched/mixed vs FP64 plain",
        "value": gis,
        "unit": "GI/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"two-material disk, k=20, N={n}, one plane wave, FP64 GMRES (no restart) "
                               f"to relative residual {args.tol:g}",
                   "n_nodes": n, "k": prob.k, "nrhs": 1, "tol": args.tol,
                   "iterations": int(infos[-1]["iters"][0]), "applies_per_solve": n_apply // args.steps,
                   "final_relres": float(infos[-1]["relres"][0]), "setup_s": setup_s,
                   "far_kernel_ms_avg": far_avg_s * 1e3,
                   "apply_ms_avg": prof["apply_ms"] / max(prof["apply_calls"], 1)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": far_traffic()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
