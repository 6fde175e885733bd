#!/usr/bin/env python3
"""Benchmark of the Lippmann-Schwinger Nystrom hot path on one MI355X.

Default workload (c2): the two-material disk (inclusion |x| < 0.5 with n = 3, annulus
0.5 < |x| < 1 with n = 1 + 0.5 exp(-|x|^2)), k = 20, O-grid/annulus mesh with 15 inner cells
(N = 58 500 nodes), one plane wave along +x.  One step = one FP64 GMRES solve (no restart,
x0 = 0) of L u = b to a relative residual of 1e-8, every operator application being the
far-field Green's sum over all N(N-1) node pairs plus the sparse correction.

Other workloads (--workload, one JSON line each):
  c1  unit disk, n^2 = 2, k = 2 pi, N = 2 500, one plane wave (plain FP64);
  c3  unit disk, n^2 = 2, k = 40, N = 122 500, 64 directions, forms p64 / b64 / bm;
  c4  16 seeded scatterers of uneven size in one handle, 8 directions each, forms p64 / bm;
  c5  two-material disk at k = 40, N = 114 660, 16 directions: far-field misfit and its contrast
      gradient through the forward and adjoint solves, forms p64 / b64 / bm;
  field  the scattered field (eq. field_recovery) of 16 plane waves on the c3 mesh at the exterior
      points of a Cartesian grid over the enclosing square.
Forms: p64 = FP64 VALU kernel, one right-hand side at a time (columns beyond --cols are
extrapolated from the timed ones, and the line says so); b64 = all right-hand sides together on
FP64 matrix-core tiles; bm = all together, FP32 matrix-core tiles inside FP64 GMRES (relaxed).

Reported: Green interactions per second over the timed work (value), the time to a 1e-8
residual (ms_per_step), the dominant kernel's roofline position (average launch duration from
HIP events the library records around each launch on the caller's stream), and the oracle's
own throughput on a bounded sample of the same far sum on the host cores.

Usage: python bench.py [--workload c2] [--form p64] [--steps K] [--warmup W] [--gpus 1]
                       [--no-cpu-baseline]
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
PEAK_FP64_TFLOPS = 78.6       # vector and matrix: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP32_MFMA_TFLOPS = 157.3
# HBM bytes per far-kernel launch in the default workload, from two rocprofv3 counter passes
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors that make a 1 GiB copy read 1 GiB and write
# 1 GiB; profiles/far_fp64_two_material_N58500_hbm_counters.md), valid for the kernel sources
# with this digest only: after any change to them the field is reported as null.
FAR_TRAFFIC_BYTES = 37_694_000 + 134_784_000
FAR_TRAFFIC_SOURCES = ("apply.hip", "hankel.h", "hankel_tables.h")
FAR_TRAFFIC_DIGEST = "57aa3428bd671f22"


def far_traffic():
    import hashlib
    h = hashlib.sha256()
    for f in FAR_TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_17615_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return FAR_TRAFFIC_BYTES if h.hexdigest()[:16] == FAR_TRAFFIC_DIGEST else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def z_fractions(meshes_k, rows=256, seed=0):
    """Fractions of node pairs in the far kernel's argument ranges (seeded row sample),
    weighted by each scatterer's pair count."""
    import numpy as np
    rng = np.random.default_rng(seed)
    acc = np.zeros(4)
    for mesh, k in meshes_k:
        n = mesh.x.size
        sel = rng.choice(n, min(rows, n), replace=False)
        cnt = np.zeros(4)
        for r in sel:
            z = np.hypot(mesh.x - mesh.x[r], mesh.y - mesh.y[r]) * k
            z[r] = -1.0
            z = z[z >= 0]
            cnt += np.histogram(z, bins=[0.0, *Z_BOUNDS, np.inf])[0]
        acc += cnt / cnt.sum() * float(n) * (n - 1)
    f = acc / acc.sum()
    return dict(zip(("small", "mid1", "mid2", "far"), (float(v) for v in f)))


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
    workers = workers or max(1, min(os.cpu_count() or 1, 16))
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
    return {"value": gis, "unit": "GI/s", "cores": workers, "kind": "oracle",
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


def far_kernel_avg(op, x, precision, reps=5):
    """Average far-kernel launch time of reps applications (the dominant kernel of a form)."""
    op.apply(x, precision=precision)
    with Timer(op) as t:
        for _ in range(reps):
            op.apply(x, precision=precision)
    return t.far_avg_s


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
    cfg = {"workload": f"{label}, N={n}, one plane wave, FP64 GMRES (no restart) to relative residual "
                       f"{args.tol:g}",
           "n_nodes": n, "k": prob.k, "nrhs": 1, "tol": args.tol, "iterations": int(infos[-1]["iters"][0]),
           "applies_per_solve": n_apply // args.steps, "final_relres": float(infos[-1]["relres"][0]),
           "setup_s": setup_s, "far_kernel_ms_avg": t.far_avg_s * 1e3,
           "apply_ms_avg": t.prof["apply_ms"] / max(t.prof["apply_calls"], 1),
           "flops_per_pair": fpp, "z_range_fractions": frac}
    traffic = far_traffic() if args.workload == "c2" else None
    return line(n_apply * pairs / t.seconds / 1e9, t.seconds / args.steps * 1e3, args.steps, args.warmup, "f64", cfg,
                roofline_valu(fpp, pairs, t.far_avg_s, traffic), None)


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
        # the adjoint system takes P^H = I + T_C^Q (D^-1 S^H D - I) T_Q^C (D: ls_transfer_colsums)
        S = args._cartesian_S
        if isinstance(S, tuple):
            # block LU appliers of S and S^H (BlockSparsifier)
            if adjoint:
                d = torch.tensor(op.transfer_colsums(), device="cuda")
                apply = lambda v: S[1](v * d) / d
            else:
                apply = S[0]
        else:
            ST = S
            if adjoint:
                if getattr(args, "_cartesian_S_adj", None) is None:
                    d = torch.tensor(op.transfer_colsums(), device="cuda")
                    args._cartesian_S_adj = (d[:, None] * ST.conj().T / d[None, :]).contiguous()
                ST = args._cartesian_S_adj
            apply = lambda v: v @ ST
        with Timer(op) as t:
            x, info = op.solve_precond(b, apply, tol=args.tol, maxit=args.maxit, restart=args.restart,
                                       adjoint=adjoint, precision="mixed" if form == "pcm" else "fp64",
                                       inner_tol=args.relax)
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
                               inner_tol=args.relax if form == "bm" else 0.0)
            xs.append(x)
            its += [int(v) for v in info["iters"]]
            a64 += int(info["n_apply_fp64"])
            amx += int(info["n_apply_mixed"])
            log(f"  columns {c0}..{c0 + x.shape[0] - 1}: max {int(np.max(info['iters']))} iterations, "
                f"max relres {np.max(info['relres']):.2e}, applies {info['n_apply_fp64']}+"
                f"{info['n_apply_mixed']}, second Gram-Schmidt passes {info['n_reorth']}, {info['seconds']:.2f} s")
    return torch.cat(xs), t.seconds, a64, amx, t, its, B


def cartesian_grid(prob, kh, pad=0.02):
    """(x0, y0, h, nx, ny) of the Cartesian grid of spacing kh / k over the scatterer's nodes."""
    import math
    h = kh / prob.k
    x, y = prob.mesh.x, prob.mesh.y
    x0, y0 = x.min() - pad, y.min() - pad
    nx = int(math.ceil((x.max() + pad - x0) / h)) + 1
    ny = int(math.ceil((y.max() + pad - y0) / h)) + 1
    return x0, y0, h, nx, ny


def cell_self_term(k, h):
    """Integral of G over the disk of area h^2 centred on the node: (-1 + (i pi/2) k a H1(k a)) / k^2."""
    import math

    from scipy.special import hankel1
    a = h / math.sqrt(math.pi)
    return (-1 + 0.5j * math.pi * a * k * complex(hankel1(1, k * a))) / k ** 2


STENCIL_OFFSETS = [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def sparsifying_stencil(x0, y0, h, nx, ny, k, m):
    """The pieces of the sparsifying preconditioner (paper, Section 4, eqs. sparsifying_min and
    LC_def) for the first-order Cartesian system L^(C) = I + k^2 V^(C) M^(C) on the grid
    (x0 + ix h, y0 + iy h): V^(C) is h^2 G off the diagonal (the library's host Green's
    evaluation) and the cell's own term on it, m the contrast at the grid nodes.  A row's weights
    are the smallest left singular vector of V^(C)(N(j), N(j)^c) over its 3 x 3 neighbourhood
    within the grid: the central node's serve every row with all 9 neighbours (the grid is
    uniform), and each edge and corner row gets its own on its 6 or 4.  C^(C) is A L^(C)
    restricted to the 3 x 3 pattern, which needs V^(C) only at the 25 offsets of at most two
    steps.  Returns (W, E, ratio): W[j, o] = A[j, j + o] and E[j, o] = C^(C)[j, j + o] for the 9
    offsets o of STENCIL_OFFSETS (0 where j + o is off the grid), and the central stencil's
    smallest / largest singular value."""
    import numpy as np

    import paper_2608_17615_amd as lsg
    nc = nx * ny
    iy, ix = np.divmod(np.arange(nc), nx)
    vself = cell_self_term(k, h)

    def vgrid(dx, dy):
        """V^(C) between nodes dx, dy steps apart (arrays)."""
        d2 = np.asarray(dx * dx + dy * dy, dtype=np.float64)
        out = h * h * lsg.eval_green_host((k * h) ** 2 * np.where(d2 > 0, d2, 1.0))
        return np.where(d2 > 0, out, vself)

    offs = STENCIL_OFFSETS
    rows = np.arange(nc)

    def shift(dx, dy):
        ok = (ix + dx >= 0) & (ix + dx < nx) & (iy + dy >= 0) & (iy + dy < ny)
        return ok, rows + dy * nx + dx

    def weights(j):
        """Smallest left singular vector over row j's neighbours (-> 9 slots, 0 where missing)."""
        have = [o for o in range(9) if 0 <= ix[j] + offs[o][0] < nx and 0 <= iy[j] + offs[o][1] < ny]
        nb = np.array([j + offs[o][1] * nx + offs[o][0] for o in have])
        rest = np.setdiff1d(rows, nb)
        B = vgrid(ix[rest][None, :] - ix[nb][:, None], iy[rest][None, :] - iy[nb][:, None])
        U, sig, _ = np.linalg.svd(B, full_matrices=False)
        w = np.zeros(9, dtype=np.complex128)
        w[have] = U[:, -1].conj()
        return w, sig[-1] / sig[0]

    v, ratio = weights((ny // 2) * nx + nx // 2)
    W = np.tile(v, (nc, 1))
    for j in np.nonzero((ix == 0) | (ix == nx - 1) | (iy == 0) | (iy == ny - 1))[0]:
        W[j] = weights(j)[0]
    m = np.asarray(m, dtype=np.complex128)
    E = np.zeros((nc, 9), dtype=np.complex128)
    for o, (dxl, dyl) in enumerate(offs):
        okl, _ = shift(dxl, dyl)
        W[~okl, o] = 0.0
        for o2, (dx2, dy2) in enumerate(offs):
            ok2, j2 = shift(dx2, dy2)
            ok = okl & ok2
            same = o == o2
            # L^(C)[l, j2] = [l == j2] + k^2 V^(C)(z_l - z_j2) m(z_j2)
            lval = (1.0 if same else 0.0) + k * k * vgrid(dxl - dx2, dyl - dy2) * m[j2[ok]]
            E[ok, o2] += W[ok, o] * lval
    return W, E, float(ratio)


def stencil_to_dense(X, nx, ny):
    """The (nx ny)^2 matrix with X[j, o] at (j, j + o)."""
    import numpy as np
    nc = nx * ny
    iy, ix = np.divmod(np.arange(nc), nx)
    M = np.zeros((nc, nc), dtype=np.complex128)
    for o, (dx, dy) in enumerate(STENCIL_OFFSETS):
        ok = (ix + dx >= 0) & (ix + dx < nx) & (iy + dy >= 0) & (iy + dy < ny)
        j = np.nonzero(ok)[0]
        M[j, j + dy * nx + dx] = X[j, o]
    return M


def sparsifying_S(x0, y0, h, nx, ny, k, m):
    """S^(C) = (C^(C))^-1 A as a dense (nx ny)^2 array (host LAPACK), with the central stencil's
    singular-value ratio (sparsifying_stencil)."""
    import numpy as np
    W, E, ratio = sparsifying_stencil(x0, y0, h, nx, ny, k, m)
    return np.linalg.solve(stencil_to_dense(E, nx, ny), stencil_to_dense(W, nx, ny)), ratio


class BlockSparsifier:
    """S^(C) = (C^(C))^-1 A (or its adjoint A^H (C^(C))^-H) applied without forming it.  With the
    grid numbered row by row, C^(C) is block tridiagonal in blocks of one grid row (nx x nx):
    block LU on the host at setup (Sigma_0 = D_0, Sigma_i = D_i - L_i Sigma_{i-1}^-1 U_{i-1}, no
    pivoting across blocks), then per application two sweeps of ny small matrix products on the
    device and one 9-point stencil for A.  Memory 3 ny nx^2 complex values instead of (nx ny)^2."""

    def __init__(self, W, E, nx, ny, device, adjoint=False):
        import numpy as np
        import torch
        self.nx, self.ny, self.adjoint = nx, ny, adjoint
        Eb = E.reshape(ny, nx, 9)
        ar = np.arange(nx)

        def block(i, dy):
            """The block of C^(C) at block row i, column block i + dy."""
            out = np.zeros((nx, nx), dtype=np.complex128)
            for o, (dx, ody) in enumerate(STENCIL_OFFSETS):
                if ody != dy:
                    continue
                ok = (ar + dx >= 0) & (ar + dx < nx)
                out[ar[ok], ar[ok] + dx] = Eb[i, ar[ok], o]
            return out

        D = [block(i, 0) for i in range(ny)]
        Lo = [block(i, -1) for i in range(ny)]    # block (i, i - 1)
        Up = [block(i, 1) for i in range(ny)]     # block (i, i + 1)
        if adjoint:
            # C^H: block (i, i) = D_i^H, (i, i - 1) = U_{i-1}^H, (i, i + 1) = L_{i+1}^H
            D, Lo, Up = ([d.conj().T for d in D], [np.zeros((nx, nx))] + [Up[i - 1].conj().T for i in range(1, ny)],
                         [Lo[i + 1].conj().T for i in range(ny - 1)] + [np.zeros((nx, nx))])
        G, M = [np.linalg.inv(D[0])], [np.zeros((nx, nx), dtype=np.complex128)]
        for i in range(1, ny):
            Mi = Lo[i] @ G[i - 1]
            M.append(Mi)
            G.append(np.linalg.inv(D[i] - Mi @ Up[i - 1]))
        # row-major right-hand sides (B, nx) multiply the transposes from the right
        t = lambda xs: torch.tensor(np.stack([x.T for x in xs]), device=device)
        self.Gt, self.Mt, self.Ut = t(G), t(M), t(Up)
        Wg = W.reshape(ny, nx, 9)
        self.W = torch.tensor(np.ascontiguousarray(np.moveaxis(Wg, 2, 0)), device=device)   # (9, ny, nx)

    def _stencil(self, c):
        """A c, or A^H c for the adjoint, on (B, ny, nx) grid arrays."""
        import torch
        nx, ny = self.nx, self.ny
        out = torch.zeros_like(c)
        if not self.adjoint:
            cp = torch.nn.functional.pad(c, (1, 1, 1, 1))
            for o, (dx, dy) in enumerate(STENCIL_OFFSETS):
                out += self.W[o] * cp[:, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
        else:
            # (A^H c)[l] = sum_o conj(W[l - o, o]) c[l - o]
            for o, (dx, dy) in enumerate(STENCIL_OFFSETS):
                t = torch.nn.functional.pad(self.W[o].conj() * c, (1, 1, 1, 1))
                out += t[:, 1 - dy:1 - dy + ny, 1 - dx:1 - dx + nx]
        return out

    def _solve(self, y):
        """(C^(C))^-1 y (or ^-H), y of shape (B, ny, nx)."""
        import torch
        z = [y[:, 0]]
        for i in range(1, self.ny):
            z.append(y[:, i] - z[-1] @ self.Mt[i])
        x = [None] * self.ny
        x[-1] = z[-1] @ self.Gt[-1]
        for i in range(self.ny - 2, -1, -1):
            x[i] = (z[i] - x[i + 1] @ self.Ut[i]) @ self.Gt[i]
        return torch.stack(x, dim=1)

    def __call__(self, v):
        """S^(C) v (or S^(C)^H v) for row-major grid vectors v of shape (B, nx ny)."""
        B = v.shape[0]
        c = v.reshape(B, self.ny, self.nx)
        if not self.adjoint:
            out = self._solve(self._stencil(c))
        else:
            out = self._stencil(self._solve(c))
        return out.reshape(B, self.nx * self.ny)


def cartesian_inverse(op, prob, kh, kind="inverse"):
    """The caller's S for the preconditioned form, on a grid of spacing kh / k.  kind "inverse":
    the dense inverse of a first-order Cartesian discretization of L (off-diagonal h^2 G(z_i, z_j)
    from the library's own Green's evaluation, the cell's own term integrated over the disk of the
    cell's area, the medium's contrast at the grid nodes), inverted by host LAPACK.  kind
    "sparsify": the sparsifying preconditioner S^(C) = (C^(C))^-1 A of the same discretization
    (sparsifying_S), applied as a dense matrix; "sparsify-lu": the same S applied through the block
    LU of C^(C) (BlockSparsifier).  Registers the grid with the operator and returns (S^T on the
    device, or the pair of appliers of S and S^H, grid size, seconds)."""
    import numpy as np
    import torch

    import paper_2608_17615_amd as lsg
    t0 = time.perf_counter()
    k = prob.k
    x0, y0, h, nx, ny = cartesian_grid(prob, kh)
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    if kind == "sparsify":
        S, ratio = sparsifying_S(x0, y0, h, nx, ny, k, prob.m_at(x0 + ix * h, y0 + iy * h))
        log(f"stencil: smallest / largest singular value {ratio:.2e}")
        ST = torch.tensor(S.T.copy(), device="cuda")
        del S
        op.set_grid(x0, y0, h, nx, ny)
        torch.cuda.synchronize()
        return ST, nx * ny, time.perf_counter() - t0
    if kind == "sparsify-lu":
        W, E, ratio = sparsifying_stencil(x0, y0, h, nx, ny, k, prob.m_at(x0 + ix * h, y0 + iy * h))
        log(f"stencil: smallest / largest singular value {ratio:.2e}")
        appliers = (BlockSparsifier(W, E, nx, ny, "cuda"), BlockSparsifier(W, E, nx, ny, "cuda", adjoint=True))
        op.set_grid(x0, y0, h, nx, ny)
        torch.cuda.synchronize()
        return appliers, nx * ny, time.perf_counter() - t0
    zx = torch.tensor(x0 + ix * h, device="cuda")
    zy = torch.tensor(y0 + iy * h, device="cuda")
    z2 = (k * k) * ((zx[:, None] - zx[None, :]) ** 2 + (zy[:, None] - zy[None, :]) ** 2)
    z2.fill_diagonal_(1.0)
    L = lsg.eval_green(z2)
    del z2
    L.mul_(h * h)
    L.diagonal().fill_(cell_self_term(k, h))
    m = torch.tensor(np.asarray(prob.m_at(x0 + ix * h, y0 + iy * h), dtype=np.complex128), device="cuda")
    L.mul_((k * k) * m[None, :])
    L.diagonal().add_(1.0)
    Lh = L.cpu().numpy()
    del L
    torch.cuda.empty_cache()
    ST = torch.tensor(np.linalg.inv(Lh).T.copy(), device="cuda")
    op.set_grid(x0, y0, h, nx, ny)
    torch.cuda.synchronize()
    return ST, nx * ny, time.perf_counter() - t0


def run_batched(args, probs, label, B):
    """c3 / c4: solve L u = b for B plane waves per scatterer with one form."""
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
        if len(probs) != 1 or probs[0].m_at is None:
            raise SystemExit("--form pc needs one scatterer whose contrast is known off the nodes")
        args._cartesian_S, nc, pre_s = cartesian_inverse(op, probs[0], args.kh, args.precond)
        pre = {"S": args.precond, "k_h": args.kh, "grid_nodes": nc, "build_s": pre_s}
        log(f"Cartesian S: {nc} grid nodes, built in {pre_s:.1f} s")
    if form == "bm" and len(probs) > 1:
        tune = op.autotune(B, precision="mixed")
        log(f"autotune: {tune}")
    x, secs, a64, amx, t, its, cols = solve_form(op, b, form, args)
    pairs = sum(p.n_nodes * (p.n_nodes - 1) for p in probs)
    frac = z_fractions([(p.mesh, p.k) for p in probs])
    # interactions the far sums evaluated (the library leaves out scatterers whose systems have
    # all finished, so this is not applications x pairs for several scatterers)
    value = t.prof["pair_rhs"] / secs / 1e9
    if form == "p64":
        # every column is its own solve: scale the timed columns to all B
        total_s = secs * B / cols
        roof = roofline_valu(flops_per_pair(frac, 1), pairs, t.far_avg_s)
        dtype = "f64"
    else:
        total_s = secs
        single = form == "bm"
        roof = roofline_mfma(pairs * B, far_kernel_avg(op, b, "mixed" if single else "fp64"), single)
        dtype = "f32-mfma+f64" if form in ("bm", "pcm") else "f64"
    # true FP64 residual of the returned solution
    r = b[:x.shape[0]] - op.apply(x)
    relres = (torch.linalg.norm(r, dim=1) / torch.linalg.norm(b[:x.shape[0]], dim=1)).cpu().numpy()
    check = None
    if form == "bm":
        # untimed: distance of the mixed-precision solution's first column from an FP64 solve of it
        x64, _ = op.solve(b[:1], tol=args.tol, maxit=args.maxit, restart=args.restart)
        check = float(((x[:1] - x64).abs().max() / x64.abs().max()).item())
        log(f"first column against FP64 GMRES: {check:.2e}")
    cfg = {"workload": label, "form": form, "n_nodes": n, "scatterers": len(probs), "nrhs": B, "tol": args.tol,
           "restart": args.restart, "inner": args.inner, "relax": args.relax, "batch": args.batch or B,
           "columns_timed": cols,
           "time_to_tol_s": total_s, "extrapolated": cols < B,
           "iterations_max": int(max(its)), "iterations_mean": float(np.mean(its)),
           "applies_fp64": a64, "applies_mixed": amx, "final_fp64_relres_max": float(relres.max()),
           "setup_s": setup_s, "far_kernel_ms_avg": t.far_avg_s * 1e3, "z_range_fractions": frac,
           "autotune": tune, "error_vs_fp64_column0": check, "preconditioner": pre}
    return line(value, total_s * 1e3, 1, 0, dtype, cfg, roof, None), x


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
    pre = None
    if form in ("pc", "pcm"):
        if prob.m_at is None:
            raise SystemExit("--form pc needs a scatterer whose contrast is known off the nodes")
        args._cartesian_S, nc, pre_s = cartesian_inverse(op, prob, args.kh, args.precond)
        pre = {"S": args.precond, "k_h": args.kh, "grid_nodes": nc, "build_s": pre_s}
        log(f"Cartesian S: {nc} grid nodes, built in {pre_s:.1f} s")
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
        single = form == "bm"
        roof = roofline_mfma(pairs * B, far_kernel_avg(op, b, "mixed" if single else "fp64"), single)
        dtype = "f32-mfma+f64" if form in ("bm", "pcm") else "f64"
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
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "field"])
    ap.add_argument("--grid", type=int, default=256, help="field: points per side of the Cartesian grid")
    ap.add_argument("--form", default=None, choices=["p64", "b64", "bm", "pc", "pcm"],
                    help="pc: FP64 GMRES right-preconditioned by P = I + T_C^Q (S - I) T_Q^C with a dense "
                         "first-order Cartesian inverse as S (c3, c5); pcm: the same with relaxed mixed "
                         "precision")
    ap.add_argument("--kh", type=float, default=0.8, help="pc: k times the Cartesian grid spacing")
    ap.add_argument("--precond", default="inverse", choices=["inverse", "sparsify", "sparsify-lu"],
                    help="pc: S is the dense inverse of the first-order Cartesian system (inverse), the "
                         "sparsifying preconditioner (C^(C))^-1 A of the same system as a dense matrix "
                         "(sparsify), or the same applied through a block LU of C^(C) (sparsify-lu)")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=2000)
    ap.add_argument("--restart", type=int, default=0, help="GMRES restart length (0 = none)")
    ap.add_argument("--cols", type=int, default=1, help="p64: columns solved and timed (the rest extrapolated)")
    ap.add_argument("--batch", type=int, default=0, help="b64/bm: right-hand sides per solve (0 = all)")
    ap.add_argument("--inner", type=int, default=0,
                    help="bm: > 0 selects flexible GMRES with this many inner mixed-precision steps")
    ap.add_argument("--relax", type=float, default=0.0,
                    help="bm: accuracy granted to the mixed operator (relaxed GMRES) or inner tolerance "
                         "(flexible); 0 = the library default")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="first run one elementwise kernel that reads and writes BYTES each "
                         "(calibrates a profiler's HBM byte counters)")
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
    form = args.form or ("p64" if wl in ("c1", "c2", "field") else "bm")
    args.form = form
    if wl in ("c1", "c2") and form != "p64":
        ap.error("c1 and c2 are plain FP64 single-wave solves (form p64)")

    cpu = None
    if not args.no_cpu_baseline:
        big = max(probs, key=lambda p: p.n_nodes)
        log(f"cpu baseline: oracle far sum on a row sample of {big.name}")
        cpu = cpu_baseline(big)
        log(f"cpu baseline: {cpu['value']:.4f} GI/s on {cpu['cores']} processes")

    import torch
    if args.copy_probe:
        src = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy probe: read and wrote {src.numel() * 8} bytes")
        del src, dst

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
