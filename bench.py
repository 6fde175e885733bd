#!/usr/bin/env python3
"""Benchmark of the Lippmann-Schwinger Nystrom hot path on one MI355X.

Default workload (c3): the unit disk with n = 2, k = 40, O-grid mesh with 35 cells per side of
the central square (N = 122 500 nodes), 64 plane waves at evenly spaced angles as one right-hand
side block.  Form pcm: flexible GMRES (no restart within a pass, x0 = 0), right-preconditioned by
the paper's P = I + T_C^Q (S - I) T_Q^C with the library's sparsifying S^(C) on a grid of
k h = 0.3, raised to 1.5 mean node spacings (k h = 0.304, 270 x 270 nodes), in mixed-precision
refinement passes: every Arnoldi application uses the split-FP16 matrix-core Green's tiles (FP64
for the pairs with k r < 1, the correction, Arnoldi and residuals), and each pass starts from the
FP64 residual, until that meets the tolerance.  One step =
one solve of all 64 waves to a relative residual of 1e-8 in every column; every operator
application is the far-field Green's sum over all N(N-1) node pairs plus the sparse correction.
After the timed steps, untimed reference solves of one column by the plain FP64 kernel (one
right-hand side at a time; with and without the preconditioner) give the time to 1e-8 of the
plain form, extrapolated to 64 columns, and the speedups.

Other workloads (--workload, one JSON line each):
  c1  unit disk, n^2 = 2, k = 2 pi, N = 2 500, one plane wave (plain FP64);
  c2  two-material disk (inclusion |x| < 0.5 with n = 3, annulus with n = 1 + 0.5 exp(-|x|^2)),
      k = 20, N = 58 500, one plane wave, plain FP64 GMRES (form p64);
  c4  16 seeded scatterers of uneven size in one handle, 8 directions each, each with its own
      preconditioner (form pcm by default);
  c5  two-material disk at k = 40, N = 114 660, 16 directions: far-field misfit and its contrast
      gradient through the forward and adjoint solves;
  field  the scattered field (eq. field_recovery) of 16 plane waves on the c3 mesh at the exterior
      points of a Cartesian grid over the enclosing square.
Forms: p64 = FP64 VALU kernel, one right-hand side at a time (columns beyond --cols are
extrapolated from the timed ones, and the line says so); b64 = all right-hand sides together on
FP64 matrix-core tiles; bm = all together, mixed-precision matrix-core tiles inside FP64 GMRES
(relaxed; split-FP16 tiles for a single scatterer's 64-column groups, FP32 tiles otherwise);
pc / pcm = b64 / bm with the library's sparsifying preconditioner.

Reported: Green interactions per second over the timed work (value), the time to a 1e-8
residual (ms_per_step), the dominant kernel's roofline position (average launch duration from
HIP events the library records around each launch on the caller's stream), and the oracle's
own throughput on a bounded sample of the same far sum on the host cores.

Usage: python bench.py [--workload c3] [--form pcm] [--steps K] [--warmup W] [--gpus 1]
                       [--no-cpu-baseline] [--no-compare] [--check-orth]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Green interactions/s + time to 1e-8 residual, batched/mixed vs FP64 plain"

# FP64 operations per (target, source) pair of the far-sum kernel, by the argument range the
# pair falls in, counted on the gfx950 assembly of its loop body (add and multiply 1, FMA 2):
# coordinates and k^2 r^2 (6), inverse fourth root and 1/z (10), modulus and phase polynomials
# (far 34, z in [5, 12) 47, z in [2, 5) 61), e^{i theta} by the reduction modulo pi/256, the table
# entry's rotation by the short series of the remainder and the modulus (29); the
# small-argument series is 66 after the coordinates.  Each right-hand side adds 8 (complex
# multiply-accumulate).  The per-pair figure of a workload weights the ranges by the measured
# distribution of z = k |y_j - y_n| over a seeded sample of target rows.
FLOPS_RANGE = {"small": 72, "mid1": 106, "mid2": 92, "far": 79}
FLOPS_PER_RHS = 8
Z_BOUNDS = (2.0, 5.0, 12.0)
# The split-FP16 tile kernel (far_tile_h_kernel), counted the same way on its loop body: per pair,
# coordinates and k^2 r^2 in FP64 (6), z^(-1/2) and the tail (z, the FP64 Newton step for z, the
# phase in turns from polynomials that return turns, sine, cosine, modulus: 17), the modulus-phase
# polynomials (far z >= 8: 15, z in [1, 8): 38), or the FP64 small-argument series for z < 1 (69
# after the coordinates); plus 2 for the hi/lo splits of Re G and Im G.  The contraction runs on
# the matrix cores.
FLOPS_H16_RANGE = {"small": 75, "mid": 61, "far": 38}
FLOPS_H16_SPLIT = 2
Z_BOUNDS_H16 = (1.0, 8.0)
# VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz, for FP64 and for unpacked FP32 (the
# build turns the packed FP32 instructions off, so FP32 work issues at the FP64 rate)
PEAK_FP64_TFLOPS = 78.6
PEAK_VALU_TFLOPS = 78.6
PEAK_FP32_MFMA_TFLOPS = 157.3
# HBM bytes per launch of the single right-hand-side far sum at the two-material workload (N =
# 58 500), from two rocprofv3 counter passes (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors that
# make a 1 GiB copy read 1 GiB and write 1 GiB; profiles/far_fp64_sym_two_material_N58500_counters.md),
# valid for the kernel sources with this digest only: after any change to them the field is null.
FAR_TRAFFIC_BYTES = 73_242_000 + 214_344_000
FAR_TRAFFIC_SOURCES = ("apply.hip", "hankel.h", "hankel_tables.h")
FAR_TRAFFIC_DIGEST = "b8817d7cdd27a686"


# The same for the split-FP16 tile kernel at the default workload (unit disk, N = 122 500, 64
# plane waves): FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 per launch, averaged over the 17 launches of one
# solve (profiles/far_tile_h_disk_N122500_B64_counters.md); most of it is the 34 source splits'
# FP32 partial sums (34 x 64 x 122 500 x 8 B written, read back by the epilogue).
H16_TRAFFIC_BYTES = 1_339_250_000 + 2_191_376_000
H16_TRAFFIC_SOURCES = ("mfma.hip", "hankel.h", "hankel_tables.h")
H16_TRAFFIC_DIGEST = "4f64bbed0468337b"


def _digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2608_17615_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def far_traffic():
    return FAR_TRAFFIC_BYTES if _digest(FAR_TRAFFIC_SOURCES) == FAR_TRAFFIC_DIGEST else None


def h16_traffic():
    return H16_TRAFFIC_BYTES if _digest(H16_TRAFFIC_SOURCES) == H16_TRAFFIC_DIGEST else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def z_fractions(meshes_k, rows=256, seed=0, bounds=Z_BOUNDS, names=("small", "mid1", "mid2", "far")):
    """Fractions of node pairs in a far kernel's argument ranges (seeded row sample),
    weighted by each scatterer's pair count."""
    import numpy as np
    rng = np.random.default_rng(seed)
    acc = np.zeros(len(bounds) + 1)
    for mesh, k in meshes_k:
        n = mesh.x.size
        sel = rng.choice(n, min(rows, n), replace=False)
        cnt = np.zeros(len(bounds) + 1)
        for r in sel:
            z = np.hypot(mesh.x - mesh.x[r], mesh.y - mesh.y[r]) * k
            z[r] = -1.0
            z = z[z >= 0]
            cnt += np.histogram(z, bins=[0.0, *bounds, np.inf])[0]
        acc += cnt / cnt.sum() * float(n) * (n - 1)
    f = acc / acc.sum()
    return dict(zip(names, (float(v) for v in f)))


def flops_per_pair_h16(meshes_k):
    f = z_fractions(meshes_k, bounds=Z_BOUNDS_H16, names=("small", "mid", "far"))
    return sum(f[r] * FLOPS_H16_RANGE[r] for r in FLOPS_H16_RANGE) + FLOPS_H16_SPLIT, f


def flops_per_pair(frac, nrhs=1):
    return sum(frac[r] * FLOPS_RANGE[r] for r in FLOPS_RANGE) + FLOPS_PER_RHS * nrhs


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
    # the host cores this process may use, at most 16 (one GPU's share of the box)
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = workers or max(1, min(avail, 16))
    n = prob.n_nodes
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(n, min(rows_total, n), replace=False))
    f = prob.m * P.random_vectors(n, 1, 0)[0]
    chunks = np.array_split(rows, workers * 4)
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_rows, [(prob.mesh.x, prob.mesh.y, prob.mesh.w, prob.k, f, c[:2]) for c in chunks[:workers]])
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_rows, [(prob.mesh.x, prob.mesh.y, prob.mesh.w, prob.k, f, c) for c in chunks]))
        dt = time.perf_counter() - t0
    gis = done * (n - 1) / dt / 1e9
    return {"value": gis, "unit": "GI/s", "cores": workers, "kind": "oracle", "host_cpu_count": os.cpu_count(),
            "host_cpus_available": avail,
            "sample": f"punctured Green's far sum (SciPy AMOS H0), one right-hand side, for {done} seeded "
                      f"target rows x {n - 1} sources of the {prob.name} mesh ({done * (n - 1):.3g} "
                      f"interactions, {dt:.2f} s wall); the sparse correction rows (10 per subdomain and "
                      f"row) are excluded"}


def line(value, ms, steps, warmup, dtype, config, roofline, cpu):
    return {"metric": METRIC, "value": value, "unit": "GI/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config, "roofline": roofline, "cpu_baseline": cpu}


def roofline_valu(flops_pair, pairs, far_s, traffic=None):
    achieved = flops_pair * pairs / far_s / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic}


def roofline_mfma(pair_rhs, far_s, single):
    peak = PEAK_FP32_MFMA_TFLOPS if single else PEAK_FP64_TFLOPS
    achieved = FLOPS_PER_RHS * pair_rhs / far_s / 1e12
    return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": None}


def roofline_h16(pair_rhs, nrhs, far_s, meshes_k):
    """The split-FP16 tiles are bound by the Green's evaluation on the VALU (one per pair and
    64-column group; the contraction overlaps on the matrix cores): VALU flops per pair counted on
    the kernel's assembly, weighted by the pairs' z ranges, against the VALU peak."""
    fpp, frac = flops_per_pair_h16(meshes_k)
    groups = -(-nrhs // 64)
    pairs = pair_rhs / nrhs * groups
    achieved = fpp * pairs / far_s / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_VALU_TFLOPS, "traffic": h16_traffic() if nrhs == 64 else None}, fpp, frac


class Timer:
    """Wall time of GPU work between two device synchronisations, plus the library's far-kernel
    launch statistics over the same interval."""

    def __init__(self, op):
        self.op = op

    def __enter__(self):
        import torch
        torch.cuda.synchronize()
        self.op.profile(True)
        self.op.profile(reset=True)
        self.t0 = time.perf_counter()
        return self

    def __exit__(self, *exc):
        import torch
        torch.cuda.synchronize()
        self.seconds = time.perf_counter() - self.t0
        self.prof = self.op.profile(reset=True)
        self.op.profile(False)
        self.far_avg_s = self.prof["far_ms"] / max(self.prof["far_launches"], 1) / 1e3


# ---------------------------------------------------------------- c2 (default) and c1
def run_plain(args, prob, label):
    import torch

    import paper_2608_17615_amd as lsg
    n = prob.n_nodes
    log(f"setup: {prob.name}, N={n}")
    t0 = time.perf_counter()
    op = lsg.Operator(lsg.Scatterer.from_mesh(prob.mesh, prob.m, prob.k))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup done in {setup_s:.2f} s (nnz {op.correction_nnz()})")
    b = torch.tensor(prob.incident(), device="cuda")
    for w in range(args.warmup):
        x, info = op.solve(b, tol=args.tol, maxit=args.maxit)
        log(f"warmup {w}: {int(info['iters'][0])} iterations, {info['seconds']:.3f} s")
    infos = []
    with Timer(op) as t:
        for s in range(args.steps):
            x, info = op.solve(b, tol=args.tol, maxit=args.maxit)
            infos.append(info)
            log(f"step {s}: {int(info['iters'][0])} iterations, relres {info['relres'][0]:.3e}, "
                f"{info['seconds']:.3f} s")
    n_apply = sum(int(i["n_apply_fp64"]) for i in infos)
    pairs = n * (n - 1)
    frac = z_fractions([(prob.mesh, prob.k)])
    fpp = flops_per_pair(frac, 1)
    # the single right-hand-side sum evaluates each unordered pair once (blocks of 256 on the
    # diagonal in both orders) and does two complex multiply-adds per evaluation: executed flops
    # per launch, against which the roofline is taken; the ordered-pair count (every ordered pair
    # at the plain sum's flops) gives the effective rate
    blk = 256
    nb = -(-n // blk)
    evals = n * (n - 1) // 2 + nb * blk * (blk - 1) // 2
    executed = (fpp + FLOPS_PER_RHS) * evals
    cfg = {"workload": f"{label}, N={n}, one plane wave, FP64 GMRES (no restart) to relative residual "
                       f"{args.tol:g}",
           "n_nodes": n, "k": prob.k, "nrhs": 1, "tol": args.tol, "iterations": int(infos[-1]["iters"][0]),
           "applies_per_solve": n_apply // args.steps, "final_relres": float(infos[-1]["relres"][0]),
           "setup_s": setup_s, "far_kernel_ms_avg": t.far_avg_s * 1e3,
           "apply_ms_avg": t.prof["apply_ms"] / max(t.prof["apply_calls"], 1),
           "flops_per_pair": fpp, "z_range_fractions": frac,
           "hankel_evaluations_per_ordered_pair": evals / pairs,
           "executed_flops_per_launch": executed,
           "effective_tflops_ordered_pair_count": fpp * pairs / t.far_avg_s / 1e12,
           **orth_check(op, b, "p64", args)}
    roof = {"bound": "alu", "achieved": executed / t.far_avg_s / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": executed / t.far_avg_s / 1e12 / PEAK_FP64_TFLOPS,
            "traffic": far_traffic() if args.workload == "c2" else None}
    return line(n_apply * pairs / t.seconds / 1e9, t.seconds / args.steps * 1e3, args.steps, args.warmup, "f64", cfg,
                roof, None)


# ---------------------------------------------------------------- batched forms (c3, c4, c5)
def solve_form(op, b, form, args, adjoint=False):
    """Solve with one form; returns (x, seconds, FP64 applies, mixed applies, timer, per-column
    iterations, columns solved)."""
    import numpy as np
    import torch
    B = b.shape[0]
    if form == "p64":
        cols = min(B, args.cols)
        xs, its, applies = [], [], 0
        with Timer(op) as t:
            for c in range(cols):
                x, info = op.solve(b[c:c + 1], tol=args.tol, maxit=args.maxit, adjoint=adjoint,
                                   restart=args.restart)
                xs.append(x)
                its.append(int(info["iters"][0]))
                applies += int(info["n_apply_fp64"])
                log(f"  column {c}: {its[-1]} iterations, relres {info['relres'][0]:.2e}, {info['seconds']:.2f} s")
        return torch.cat(xs), t.seconds, applies, 0, t, its, cols
    if form in ("pc", "pcm"):
        # right preconditioner P = I + T_C^Q (S - I) T_Q^C with the library's S^(C) on every
        # scatterer (P^H for the adjoint system)
        with Timer(op) as t:
            x, info = op.solve_precond(b, None, tol=args.tol, maxit=args.maxit, restart=args.restart,
                                       adjoint=adjoint, precision="mixed" if form == "pcm" else "fp64",
                                       inner_tol=args.relax, scheme=args.scheme)
        its = [int(v) for v in info["iters"]]
        log(f"  preconditioned: max {max(its)} iterations, max relres {np.max(info['relres']):.2e}, applies "
            f"{info['n_apply_fp64']}+{info['n_apply_mixed']}, {info['seconds']:.2f} s")
        return x, t.seconds, int(info["n_apply_fp64"]), int(info["n_apply_mixed"]), t, its, B
    prec = "mixed" if form == "bm" else "fp64"
    batch = args.batch or B
    xs, its, a64, amx = [], [], 0, 0
    with Timer(op) as t:
        for c0 in range(0, B, batch):
            x, info = op.solve(b[c0:c0 + batch], tol=args.tol, maxit=args.maxit, precision=prec, adjoint=adjoint,
                               restart=args.restart, inner_maxit=args.inner if form == "bm" else 0,
                               inner_tol=args.relax if form == "bm" else 0.0,
                               scheme=args.scheme if form == "bm" else "relaxed")
            xs.append(x)
            its += [int(v) for v in info["iters"]]
            a64 += int(info["n_apply_fp64"])
            amx += int(info["n_apply_mixed"])
            log(f"  columns {c0}..{c0 + x.shape[0] - 1}: max {int(np.max(info['iters']))} iterations, "
                f"max relres {np.max(info['relres']):.2e}, applies {info['n_apply_fp64']}+"
                f"{info['n_apply_mixed']}, second Gram-Schmidt passes {info['n_reorth']}, {info['seconds']:.2f} s")
    return torch.cat(xs), t.seconds, a64, amx, t, its, B


# a scatterer gets the Cartesian preconditioner only when its quadrature nodes resolve the wave
# inside it: k sqrt(max n) times the mean node spacing sqrt(area / N) at most this (about 8 nodes per
# interior wavelength); on coarser meshes the Nystrom system is far from the continuous operator the
# Cartesian system approximates, and the preconditioned iteration stagnates
MAX_RESOLUTION = 0.75


# grid spacing of the Cartesian preconditioner at least this many mean node spacings
MIN_CELL = 1.5


def resolution(p):
    """k sqrt(max n) x mean node spacing of a problem (n = 1 - m at the nodes)."""
    import numpy as np
    n_max = float(np.max(np.real(1.0 - np.asarray(p.m))))
    return p.k * np.sqrt(max(n_max, 1.0)) * np.sqrt(p.mesh.w.sum() / p.n_nodes)


def setup_precond(op, probs, kh):
    """The library's sparsifying preconditioner S^(C) (ls_sparsify_setup) for every scatterer whose
    mesh resolves its interior wave, on a grid of spacing kh / k over it; returns a summary for the
    bench line."""
    import numpy as np
    import torch

    from workloads import problems as P
    t0 = time.perf_counter()
    nodes, lu_res, sv, skipped, grids, khs = 0, 0.0, [], [], [], []
    for s, p in enumerate(probs):
        if p.m_at is None:
            raise SystemExit("the preconditioned forms need the contrast off the nodes")
        if resolution(p) > MAX_RESOLUTION:
            skipped.append(s)
            continue
        # at least MIN_CELL node spacings per grid cell, so that T_Q^C sees nodes in most cells
        spacing = float(np.sqrt(p.mesh.w.sum() / p.n_nodes))
        kh_s = max(kh, MIN_CELL * spacing * p.k)
        g = P.cartesian_grid(p, kh_s)
        info = op.sparsify_setup(*g, P.grid_contrast(p, g), s=s)
        nodes += g[3] * g[4]
        grids.append([g[3], g[4]])
        khs.append(round(kh_s, 4))
        lu_res = max(lu_res, info["lu_residual"])
        sv.append(info["sv_ratio"])
    torch.cuda.synchronize()
    out = {"S": "sparsifying (C^(C))^-1 A, first-order V^(C), block LU by grid rows (library)", "k_h": kh,
           "k_h_used": khs, "grids": grids,
           "grid_nodes": nodes, "build_s": time.perf_counter() - t0, "lu_residual_max": lu_res,
           "stencil_sv_ratio_min": min(sv), "unpreconditioned_scatterers": skipped,
           "max_resolution": MAX_RESOLUTION, "min_cell_node_spacings": MIN_CELL}
    if skipped:
        log(f"preconditioner: scatterers {skipped} left unpreconditioned (under-resolved interior wave)")
    log(f"preconditioner: {nodes} grid nodes, built in {out['build_s']:.2f} s, LU residual {lu_res:.1e}")
    return out


def dominant_tiles(prof):
    """The tile kernel family ("h16" split-FP16, "f32" or "f64") with the largest share of far-sum
    time in a profile, with its launches, milliseconds and pair-RHS interactions."""
    ms16, n16, p16 = prof["far_ms_h16"], prof["far_launches_h16"], prof["pair_rhs_h16"]
    ms32, n32, p32 = (prof["far_ms_mixed"] - ms16, prof["far_launches_mixed"] - n16,
                      prof["pair_rhs_mixed"] - p16)
    ms64, n64, p64 = (prof["far_ms"] - prof["far_ms_mixed"], prof["far_launches"] - prof["far_launches_mixed"],
                      prof["pair_rhs"] - prof["pair_rhs_mixed"])
    return max([("h16", n16, ms16, p16), ("f32", n32, ms32, p32), ("f64", n64, ms64, p64)], key=lambda t: t[2])


TILE_KERNEL = {"h16": "far_tile_h_kernel", "f32": "far_tile_kernel<float>", "f64": "far_tile_kernel<double>"}


def tiles_roofline(prof, nrhs, meshes_k):
    """roofline entry and kernel record of the dominant tile kernel of a profile"""
    kind, nl, ms, pr = dominant_tiles(prof)
    extra = {}
    if kind == "h16":
        roof, fpp, zf = roofline_h16(pr, nrhs, ms / 1e3, meshes_k)
        extra = {"valu_flops_per_pair": fpp, "z_ranges": zf,
                 "matrix_core_tflops": FLOPS_PER_RHS * pr / (ms / 1e3) / 1e12}
    else:
        roof = roofline_mfma(pr, ms / 1e3, kind == "f32")
    kern = {"kernel": TILE_KERNEL[kind], "launches": nl, "ms_avg": ms / max(nl, 1), **extra}
    return kind, roof, kern, ms


def orth_check(op, b, form, args):
    """--check-orth (untimed): column 0 solved again by the timed form with the loss of
    orthogonality of its Krylov basis measured, max |<v_i, v_j> - delta_ij| over the normalized
    basis vectors (each scatterer's own basis)."""
    import numpy as np
    if not args.check_orth:
        return {}
    kw = dict(tol=args.tol, maxit=args.maxit, restart=args.restart, check_orth=True)
    if form in ("pc", "pcm"):
        _, info = op.solve_precond(b[:1], None, precision="mixed" if form == "pcm" else "fp64",
                                   inner_tol=args.relax, scheme=args.scheme, **kw)
    elif form in ("b64", "bm"):
        _, info = op.solve(b[:1], precision="mixed" if form == "bm" else "fp64",
                           inner_maxit=args.inner if form == "bm" else 0,
                           inner_tol=args.relax if form == "bm" else 0.0,
                           scheme=args.scheme if form == "bm" else "relaxed", **kw)
    else:
        _, info = op.solve(b[:1], **kw)
    it = int(np.max(info["iters"]))
    log(f"  orthogonality check (column 0): {it} steps, loss {info['orth_loss']:.2e}")
    return {"orth_loss": float(info["orth_loss"]), "orth_check_steps": it}


def reference_column(op, b, args, precond):
    """Untimed reference: one column solved alone (the FP64 VALU kernel, one right-hand side at a
    time), with or without the library's preconditioner; returns (seconds, iterations, GI/s)."""
    with Timer(op) as t:
        if precond:
            _, info = op.solve_precond(b[:1], None, tol=args.tol, maxit=args.maxit, restart=args.restart)
        else:
            _, info = op.solve(b[:1], tol=args.tol, maxit=args.maxit, restart=args.restart)
    it = int(info["iters"][0])
    log(f"  reference column ({'preconditioned' if precond else 'plain'} P64): {it} iterations, "
        f"relres {info['relres'][0]:.2e}, {t.seconds:.2f} s")
    return t.seconds, it, t.prof["pair_rhs"] / t.seconds / 1e9


def run_batched(args, probs, label, B):
    """c3 / c4: solve L u = b for B plane waves per scatterer with one form; a step is one solve
    of the whole block."""
    import numpy as np
    import torch

    import paper_2608_17615_amd as lsg
    form = args.form
    log(f"setup: {label}, {len(probs)} scatterer(s), N = {sum(p.n_nodes for p in probs)}")
    t0 = time.perf_counter()
    op = lsg.Operator([lsg.Scatterer.from_mesh(p.mesh, p.m, p.k) for p in probs])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup done in {setup_s:.2f} s")
    n = op.n
    b = torch.tensor(np.concatenate([p.incident() for p in probs], axis=1), device="cuda")
    tune = None
    pre = None
    if form in ("pc", "pcm"):
        pre = setup_precond(op, probs, args.kh)
    if form in ("bm", "pcm") and len(probs) > 1:
        tune = op.autotune(B, precision="mixed")
        log(f"autotune: {tune}")
    steps = 1 if form == "p64" else args.steps
    warm = 0 if form == "p64" else args.warmup
    for w in range(warm):
        solve_form(op, b, form, args)
        log(f"warmup {w} done")
    runs = []
    for st in range(steps):
        runs.append(solve_form(op, b, form, args))
        log(f"step {st}: {runs[-1][1]:.3f} s")
    x, _, a64, amx, t, its, cols = runs[-1]
    secs = sum(r[1] for r in runs)
    pair_rhs = sum(r[4].prof["pair_rhs"] for r in runs)
    pairs = sum(p.n_nodes * (p.n_nodes - 1) for p in probs)
    frac = z_fractions([(p.mesh, p.k) for p in probs])
    # interactions the far sums evaluated (the library leaves out scatterers whose systems have
    # all finished, so this is not applications x pairs for several scatterers)
    value = pair_rhs / secs / 1e9
    if form == "p64":
        # every column is its own solve: scale the timed columns to all B
        step_s = secs * B / cols
        roof = roofline_valu(flops_per_pair(frac, 1), pairs, t.far_avg_s)
        dtype = "f64"
        kern = {"kernel": "far_fp64_kernel", "launches": t.prof["far_launches"], "ms_avg": t.far_avg_s * 1e3}
    else:
        step_s = secs / steps
        prof = {k: sum(r[4].prof[k] for r in runs) for k in runs[-1][4].prof}
        kind, roof, kern, ms = tiles_roofline(prof, B, [(p.mesh, p.k) for p in probs])
        dtype = {"h16": "f16x2-mfma+f64", "f32": "f32-mfma+f64", "f64": "f64"}[kind]
        kern["share_of_step"] = ms / 1e3 / secs
        if len(probs) > 1 and kind != "h16":
            kern["kernel"] = kern["kernel"].replace("far_tile_kernel", "far_tile_persistent")
    # true FP64 residual of the returned solution, per column and per (scatterer, column) system
    r = b[:x.shape[0]] - op.apply(x)
    relres = (torch.linalg.norm(r, dim=1) / torch.linalg.norm(b[:x.shape[0]], dim=1)).cpu().numpy()
    per_scat = None
    if len(probs) > 1:
        per_scat = []
        for s_, p in enumerate(probs):
            o0, o1 = op.offsets[s_], op.offsets[s_] + p.n_nodes
            rs = (torch.linalg.norm(r[:, o0:o1], dim=1) / torch.linalg.norm(b[:x.shape[0], o0:o1], dim=1)).max()
            per_scat.append({"name": p.name, "N": p.n_nodes, "k": p.k, "resolution": resolution(p),
                             "relres_max": float(rs.item())})
        conv = sum(1 for q in per_scat if q["relres_max"] <= args.tol * 1.01)
        log(f"  scatterers converged to {args.tol:g}: {conv} of {len(probs)}")
    check = None
    if form in ("bm", "pcm"):
        # untimed: distance of the mixed-precision solution's first column from an FP64 solve of it
        if form == "pcm":
            x64, _ = op.solve_precond(b[:1], None, tol=args.tol, maxit=args.maxit)
        else:
            x64, _ = op.solve(b[:1], tol=args.tol, maxit=args.maxit, restart=args.restart)
        check = float(((x[:1] - x64).abs().max() / x64.abs().max()).item())
        log(f"first column against FP64 GMRES: {check:.2e}")
    compare = None
    if args.compare and form != "p64" and len(probs) == 1:
        p_s, p_it, p_gis = reference_column(op, b, args, False)
        compare = {"p64_plain_column_s": p_s, "p64_plain_iterations": p_it, "p64_plain_gis": p_gis,
                   "p64_plain_time_to_tol_s": p_s * B, "extrapolated": True}
        if pre is not None:
            c_s, c_it, c_gis = reference_column(op, b, args, True)
            compare.update({"p64_precond_column_s": c_s, "p64_precond_iterations": c_it,
                            "p64_precond_time_to_tol_s": c_s * B})
            compare["speedup_vs_p64_precond"] = c_s * B / step_s
        compare["speedup_vs_p64_plain"] = p_s * B / step_s
    cfg = {"workload": label, "form": form, "n_nodes": n, "scatterers": len(probs), "nrhs": B, "tol": args.tol,
           "step": "one solve of every right-hand side to the tolerance (true FP64 residual)",
           "restart": args.restart, "inner": args.inner, "relax": args.relax, "scheme": args.scheme, "batch": args.batch or B,
           "columns_timed": cols, "time_to_tol_s": step_s, "extrapolated": cols < B,
           "iterations_max": int(max(its)), "iterations_mean": float(np.mean(its)),
           "applies_fp64": a64, "applies_mixed": amx, "final_fp64_relres_max": float(relres.max()),
           "setup_s": setup_s, "dominant_kernel": kern, "z_range_fractions": frac,
           "autotune": tune, "error_vs_fp64_column0": check, "preconditioner": pre, "compare": compare,
           "per_scatterer": per_scat, **orth_check(op, b, form, args)}
    return line(value, step_s * 1e3, steps, warm, dtype, cfg, roof, None), x


def run_gradient(args, prob, label, B):
    """c5: J(m) = 1/2 sum |u_inf - data|^2 at 128 receivers and dJ/dm by the adjoint solve."""
    import torch

    import paper_2608_17615_amd as lsg
    from workloads import problems as P
    form = args.form
    log(f"setup: {label}, N = {prob.n_nodes}")
    t0 = time.perf_counter()
    op = lsg.Operator(lsg.Scatterer.from_mesh(prob.mesh, prob.m, prob.k))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    n = op.n
    b = torch.tensor(prob.incident(), device="cuda")
    thetas = P.receivers(128)
    pre = setup_precond(op, [prob], args.kh) if form in ("pc", "pcm") else None
    # synthetic data: far field of the seeded contrast perturbation (input generation, untimed)
    m0 = torch.tensor(prob.m, device="cuda").to(torch.complex128)
    dm = torch.tensor(P.contrast_perturbation(prob.mesh), device="cuda").to(torch.complex128)
    cols = B if form != "p64" else min(B, args.cols)
    op.set_contrast(m0 + dm)
    ud, _ = op.solve(b[:cols], tol=args.tol, maxit=args.maxit, precision="mixed", restart=args.restart)
    data, _, _ = op.farfield(ud, thetas)
    op.set_contrast(m0)
    log("data synthesised")
    fwd = solve_form(op, b[:cols], form, args)
    u = fwd[0]
    _, res, J = op.farfield(u, thetas, data)
    a, rhs = op.farfield_adjoint(res, thetas)
    adj = solve_form(op, rhs, form, args, adjoint=True)
    lam = adj[0]
    g = op.grad_contrast(u, lam, a)
    torch.cuda.synchronize()
    secs = fwd[1] + adj[1]
    pairs = n * (n - 1)
    frac = z_fractions([(prob.mesh, prob.k)])
    value = (fwd[4].prof["pair_rhs"] + adj[4].prof["pair_rhs"]) / secs / 1e9
    if form == "p64":
        total_s = secs * B / cols
        roof = roofline_valu(flops_per_pair(frac, 1), pairs, fwd[4].far_avg_s)
        dtype = "f64"
    else:
        total_s = secs
        prof = {k: fwd[4].prof[k] + adj[4].prof[k] for k in fwd[4].prof}
        kind, roof, _, _ = tiles_roofline(prof, B, [(prob.mesh, prob.k)])
        dtype = {"h16": "f16x2-mfma+f64", "f32": "f32-mfma+f64", "f64": "f64"}[kind]
    check = None
    if form == "bm":
        # untimed: the same misfit and gradient through FP64 solves (batched FP64 tiles)
        u64 = solve_form(op, b[:cols], "b64", args)[0]
        _, res64, J64 = op.farfield(u64, thetas, data)
        a64_, rhs64 = op.farfield_adjoint(res64, thetas)
        lam64 = solve_form(op, rhs64, "b64", args, adjoint=True)[0]
        g64 = op.grad_contrast(u64, lam64, a64_)
        check = {"misfit": abs(J - J64) / abs(J64),
                 "gradient": float(((g - g64).abs().max() / g64.abs().max()).item())}
        log(f"against FP64 solves: misfit {check['misfit']:.2e}, gradient {check['gradient']:.2e}")
    cfg = {"workload": label, "form": form, "n_nodes": n, "nrhs": B, "receivers": 128, "tol": args.tol,
           "restart": args.restart, "columns_timed": cols, "time_to_tol_s": total_s, "extrapolated": cols < B,
           "forward_s": fwd[1], "adjoint_s": adj[1], "iterations_forward_max": int(max(fwd[5])),
           "iterations_adjoint_max": int(max(adj[5])), "misfit_J": J,
           "grad_norm": float(torch.linalg.norm(g).item()), "setup_s": setup_s, "z_range_fractions": frac,
           "error_vs_fp64": check, "preconditioner": pre}
    return line(value, total_s * 1e3, 1, 0, dtype, cfg, roof, None), g


def run_field(args, prob, label, B):
    """Field recovery: the scattered field of B plane waves at the exterior points of a Cartesian
    grid over the enclosing square (the paper's exterior measurement set)."""
    import numpy as np
    import torch

    import paper_2608_17615_amd as lsg
    log(f"setup: {label}, N = {prob.n_nodes}")
    op = lsg.Operator(lsg.Scatterer.from_mesh(prob.mesh, prob.m, prob.k))
    n = op.n
    g = np.linspace(-1.5, 1.5, args.grid)
    X, Y = np.meshgrid(g, g)
    keep = np.hypot(X, Y) > 1.0 + 1.0 / args.grid
    tx, ty = X[keep], Y[keep]
    nt = tx.size
    u = torch.tensor(prob.incident()[:B], device="cuda")
    op.field(u, tx[:64], ty[:64])   # warm-up
    with Timer(op) as t:
        out = op.field(u, tx, ty)
    pairs = n * nt
    # per-pair flops weighted by the distribution of k |x_t - y_n|
    rng = np.random.default_rng(0)
    sel = rng.choice(nt, min(256, nt), replace=False)
    cnt = np.zeros(4)
    for r in sel:
        z = np.hypot(prob.mesh.x - tx[r], prob.mesh.y - ty[r]) * prob.k
        cnt += np.histogram(z, bins=[0.0, *Z_BOUNDS, np.inf])[0]
    frac = dict(zip(("small", "mid1", "mid2", "far"), (float(v) for v in cnt / cnt.sum())))
    fpp = flops_per_pair(frac, B)
    cfg = {"workload": f"{label}: scattered field of {B} plane waves at {nt} exterior points of a "
                       f"{args.grid} x {args.grid} grid on [-1.5, 1.5]^2", "form": "field", "n_nodes": n,
           "targets": nt, "nrhs": B, "time_s": t.seconds, "far_kernel_ms": t.far_avg_s * 1e3,
           "assembly_and_other_s": t.seconds - t.far_avg_s, "flops_per_pair": fpp, "z_range_fractions": frac,
           "finite": bool(torch.isfinite(out).all().item())}
    return line(pairs * B / t.seconds / 1e9, t.seconds * 1e3, 1, 0, "f64", cfg,
                roofline_valu(fpp, pairs, t.far_avg_s), None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5", "field"])
    ap.add_argument("--grid", type=int, default=256, help="field: points per side of the Cartesian grid")
    ap.add_argument("--form", default=None, choices=["p64", "b64", "bm", "pc", "pcm"],
                    help="p64: FP64 VALU kernel, one right-hand side at a time; b64: FP64 matrix-core tiles; "
                         "bm: FP32 matrix-core tiles in relaxed FP64 GMRES; pc: FP64 GMRES right-preconditioned "
                         "by P = I + T_C^Q (S - I) T_Q^C with the library's sparsifying S^(C); pcm: pc with "
                         "mixed precision (default for c3, c4, c5)")
    ap.add_argument("--kh", type=float, default=0.3,
                    help="pc, pcm: k times the Cartesian grid spacing (at least 1.5 mean node spacings)")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=None, help="GMRES steps at most (default 2000; c4: 1500)")
    ap.add_argument("--restart", type=int, default=0, help="GMRES restart length (0 = none)")
    ap.add_argument("--cols", type=int, default=1, help="p64: columns solved and timed (the rest extrapolated)")
    ap.add_argument("--batch", type=int, default=0, help="b64/bm: right-hand sides per solve (0 = all)")
    ap.add_argument("--inner", type=int, default=0,
                    help="bm: > 0 selects flexible GMRES with this many inner mixed-precision steps")
    ap.add_argument("--relax", type=float, default=None,
                    help="bm, pcm: accuracy granted to the mixed operator (relaxed GMRES) or inner tolerance "
                         "(flexible); 0 = the library default (default: 1e-6 for pcm, the library's for bm)")
    ap.add_argument("--scheme", default=None, choices=["relaxed", "passes"],
                    help="bm, pcm: relaxed GMRES (FP64 applications until the residual allows the mixed "
                         "operator) or mixed-precision refinement passes (default: passes for pcm, relaxed "
                         "for bm)")
    ap.add_argument("--no-compare", dest="compare", action="store_false",
                    help="c3: skip the untimed one-column P64 reference solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check-orth", action="store_true",
                    help="after the timed steps, solve column 0 again with the Krylov basis's loss of "
                         "orthogonality measured (orth_loss in the line's config)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); a multi-GPU layout (target rows, or "
              f"whole scatterers, per GPU) is not built", file=sys.stderr)
        sys.exit(2)

    from workloads import problems as P
    wl = args.workload
    if wl == "c1":
        probs, label = [P.config1()], "unit disk, n^2 = 2, k = 2 pi"
    elif wl == "c2":
        probs, label = [P.config2()], "two-material disk, k=20"
    elif wl == "c3":
        probs, label = [P.config3()], "unit disk, n^2 = 2, k = 40, 64 plane waves"
    elif wl == "c4":
        probs, label = P.config4(), "16 seeded disks and ellipses, k in [5, 40], 8 plane waves each"
    elif wl == "c5":
        probs, label = [P.config5()], "two-material disk, k = 40, 16 plane waves, 128 receivers"
    else:
        probs, label = [P.config3(B=16)], "unit disk, n^2 = 2, k = 40, N = 122500"
    form = args.form or ("p64" if wl in ("c1", "c2", "field") else "pcm")
    args.form = form
    if args.maxit is None:
        args.maxit = 1500 if wl == "c4" else 2000
    if args.scheme is None:
        # refinement passes (every Arnoldi application mixed) pay where the mixed tiles are much
        # faster than the FP64 ones (c3: split-FP16 at 64 columns, 1.07 s against 1.43 s relaxed);
        # at 16 columns (c5) the FP32 tiles are only twice as fast and the passes' extra steps cost
        # more than they save (3.41 s against 2.33 s relaxed); c4's slowest scatterers need
        # hundreds of steps, which the relaxed scheme keeps in one Krylov space
        args.scheme = "passes" if form == "pcm" and wl == "c3" else "relaxed"
    if args.relax is None:
        args.relax = 0.0
    if wl in ("c1", "c2") and form != "p64":
        ap.error("c1 and c2 are plain FP64 single-wave solves (form p64)")

    cpu = None
    if not args.no_cpu_baseline:
        big = max(probs, key=lambda p: p.n_nodes)
        log(f"cpu baseline: oracle far sum on a row sample of {big.name}")
        cpu = cpu_baseline(big)
        log(f"cpu baseline: {cpu['value']:.4f} GI/s on {cpu['cores']} processes")

    if wl == "field":
        out = run_field(args, probs[0], label, 16)
    elif wl in ("c1", "c2"):
        out = run_plain(args, probs[0], label)
    elif wl in ("c3", "c4"):
        out, _ = run_batched(args, probs, label, probs[0].directions.size)
    else:
        out, _ = run_gradient(args, probs[0], label, probs[0].directions.size)
    out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
