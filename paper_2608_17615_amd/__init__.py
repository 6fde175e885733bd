"""MI355X (gfx950) Lippmann-Schwinger Nystrom operator: Python binding of libls.so.

Argument marshalling only: every step of the operator, the solver and the gradient runs in
the HIP library.  torch supplies device memory and the current stream.  The library must be
built (``python -m paper_2608_17615_amd.build``); importing the compute entry points without
it raises, there is no CPU fallback.

The mathematics (paper, Sections 2-3): L u = u + k^2 (G~ W + C)(m u) at the quadrature nodes,
with m = 1 - n the contrast, G~ the punctured Green's matrix, W the weights and C the sparse
density-interpolation correction; see include/ls.h for the full statement of every call.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libls.so")

LS_OK, LS_NOT_CONVERGED, LS_ERR_ARG = 0, 1, -1
FP64, MIXED = 0, 1
_PREC = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}
_SCHEME = {"relaxed": 0, "passes": 1}
CIRCLE, ELLIPSE = 0, 1

_lib = None


class LSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class _Curve(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("orientation", ctypes.c_int32), ("subdomain", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double)]


class _Scatterer(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_elems", ctypes.c_int32), ("nq", ctypes.c_int32),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("elem_subdomain", ctypes.c_void_p), ("m", ctypes.c_void_p), ("k", ctypes.c_double),
                ("n_curves", ctypes.c_int32), ("pad_", ctypes.c_int32), ("curves", ctypes.c_void_p)]


class _Profile(ctypes.Structure):
    _fields_ = [("far_launches", ctypes.c_int64), ("far_ms", ctypes.c_double), ("apply_calls", ctypes.c_int64),
                ("apply_ms", ctypes.c_double), ("pair_rhs", ctypes.c_double),
                ("far_launches_mixed", ctypes.c_int64), ("far_ms_mixed", ctypes.c_double),
                ("pair_rhs_mixed", ctypes.c_double), ("far_launches_h16", ctypes.c_int64),
                ("far_ms_h16", ctypes.c_double), ("pair_rhs_h16", ctypes.c_double)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("mt", ctypes.c_int32), ("split_len", ctypes.c_int32), ("far_ms", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("source_split", ctypes.c_int32), ("rhs_chunk", ctypes.c_int32),
                ("targets_per_lane", ctypes.c_int32), ("mixed_tile", ctypes.c_int32),
                ("n_threads_host", ctypes.c_int32), ("fp64_matrix", ctypes.c_int32),
                ("mixed_fp16", ctypes.c_int32), ("mixed_near", ctypes.c_int32)]


class _SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("adjoint", ctypes.c_int32), ("x0_given", ctypes.c_int32),
                ("inner_maxit", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("mixed_scheme", ctypes.c_int32), ("check_orth", ctypes.c_int32)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_void_p), ("relres", ctypes.c_void_p), ("n_apply_fp64", ctypes.c_int64),
                ("n_apply_mixed", ctypes.c_int64), ("seconds", ctypes.c_double), ("n_reorth", ctypes.c_int64),
                ("orth_loss", ctypes.c_double)]


def lib():
    """The loaded libls.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2608_17615_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.ls_setup.argtypes = [vp, i32, vp, vp]
        L.ls_setup_from_csr.argtypes = [vp, vp, vp, vp, vp, vp]
        L.ls_apply.argtypes = [vp, vp, vp, i32, i64, i32, vp]
        L.ls_apply_adjoint.argtypes = [vp, vp, vp, i32, i64, i32, vp]
        L.ls_reserve.argtypes = [vp, i32, i32]
        L.ls_apply_noalloc.argtypes = [vp, vp, vp, i32, i64, i32, vp]
        L.ls_device_allocations.argtypes = []
        L.ls_device_allocations.restype = i64
        L.ls_solve_gmres.argtypes = [vp, vp, vp, i32, i64, vp, vp, vp]
        L.ls_grad_contrast.argtypes = [vp, vp, vp, vp, i32, i64, vp, vp]
        L.ls_num_nodes.argtypes = [vp]
        L.ls_num_nodes.restype = i64
        L.ls_num_scatterers.argtypes = [vp]
        L.ls_scatterer_offset.argtypes = [vp, i32]
        L.ls_scatterer_offset.restype = i64
        L.ls_correction_nnz.argtypes = [vp, i32]
        L.ls_correction_nnz.restype = i64
        L.ls_near_pairs.argtypes = [vp, i32]
        L.ls_near_pairs.restype = i64
        L.ls_export_correction.argtypes = [vp, i32, vp, vp, vp]
        L.ls_eval_green.argtypes = [vp, vp, i64, i32, vp]
        L.ls_eval_green_host.argtypes = [vp, vp, i64]
        L.ls_farfield.argtypes = [vp, i32, vp, i32, i64, vp, i32, vp, vp, vp, vp, vp]
        L.ls_farfield_adjoint.argtypes = [vp, i32, vp, i32, i64, vp, i32, vp, vp, vp]
        L.ls_field.argtypes = [vp, i32, vp, vp, i64, vp, i32, i64, vp, vp]
        L.ls_set_contrast.argtypes = [vp, vp, vp]
        L.ls_transfer_setup.argtypes = [vp, i32, vp]
        L.ls_quad_to_cart.argtypes = [vp, i32, vp, i64, vp, i64, i32, vp]
        L.ls_transfer_colsums.argtypes = [vp, i32, vp]
        L.ls_cart_to_quad.argtypes = [vp, i32, vp, i64, vp, i64, i32, vp]
        L.ls_precond_finish.argtypes = [vp, i32, vp, i64, vp, vp, i64, vp, i32, vp]
        L.ls_solve_gmres_precond.argtypes = [vp, vp, vp, i32, i64, vp, i32, _GridOp, vp, vp, vp, i64, vp, vp]
        L.ls_sparsify_setup.argtypes = [vp, i32, vp, vp, vp]
        L.ls_sparsify_apply.argtypes = [vp, i32, vp, i64, vp, i32, i32, vp]
        L.ls_sparsify_stencil_host.argtypes = [vp, dbl, vp, vp, vp, vp]
        L.ls_autotune.argtypes = [vp, i32, i32, vp, vp]
        L.ls_set_tile_shape.argtypes = [vp, i32, i32, i32]
        L.ls_profile_enable.argtypes = [vp, i32]
        L.ls_profile_query.argtypes = [vp, vp, i32]
        L.ls_destroy.argtypes = [vp]
        L.ls_destroy.restype = None
        L.ls_status_str.argtypes = [i32]
        L.ls_status_str.restype = ctypes.c_char_p
        L.ls_last_error.argtypes = [vp]
        L.ls_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status, handle=None):
    if status < 0:
        L = lib()
        raise LSError(status, (L.ls_last_error(handle) or b"").decode() or L.ls_status_str(status).decode())
    return status


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_GridOp = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                           ctypes.c_void_p, ctypes.c_void_p)


class _Grid(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("h", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


class _SparsifyInfo(ctypes.Structure):
    _fields_ = [("build_seconds", ctypes.c_double), ("sv_ratio", ctypes.c_double),
                ("lu_residual", ctypes.c_double), ("device_bytes", ctypes.c_int64)]


@dataclass
class Scatterer:
    """Host description of one scatterer (all arrays in the caller's node order)."""
    x: np.ndarray
    y: np.ndarray
    w: np.ndarray
    elem_subdomain: np.ndarray
    m: np.ndarray          # contrast 1 - n at the nodes (real or complex)
    k: float
    curves: list           # objects with kind ('circle'/'ellipse'), cx, cy, a, b, orientation, subdomain

    @classmethod
    def from_mesh(cls, mesh, m, k):
        return cls(mesh.x, mesh.y, mesh.w, mesh.elem_subdomain, m, k, list(mesh.curves))

    def _struct(self):
        keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a.ctypes.data

        m = np.asarray(self.m)
        mc = np.ascontiguousarray(m.astype(np.complex128)).view(np.float64)
        n = int(np.asarray(self.x).size)
        curves = (_Curve * max(1, len(self.curves)))()
        for i, c in enumerate(self.curves):
            kind = c.kind if isinstance(c.kind, int) else {"circle": CIRCLE, "ellipse": ELLIPSE}[c.kind]
            curves[i] = _Curve(kind, int(c.orientation), int(c.subdomain), 0, float(c.cx), float(c.cy),
                               float(c.a), float(c.b))
        keep.append(curves)
        s = _Scatterer(n, n // 10, 10, arr(self.x, np.float64), arr(self.y, np.float64), arr(self.w, np.float64),
                       arr(self.elem_subdomain, np.int32), arr(mc, np.float64), float(self.k),
                       len(self.curves), 0, ctypes.cast(curves, ctypes.c_void_p))
        return s, keep


def _options(source_split=0, rhs_chunk=0, targets_per_lane=0, mixed_tile=0, n_threads_host=0, fp64_matrix=0,
             mixed_fp16=0, mixed_near=0):
    return _Options(source_split, rhs_chunk, targets_per_lane, mixed_tile, n_threads_host, fp64_matrix, mixed_fp16,
                    mixed_near)


class Operator:
    """L = I + k^2 (G~ W + C) M for one or several scatterers, resident on the current GPU."""

    def __init__(self, scatterers, correction=None, **options):
        if isinstance(scatterers, Scatterer):
            scatterers = [scatterers]
        L = lib()
        self._h = ctypes.c_void_p()
        opts = _options(**options)
        structs = [s._struct() for s in scatterers]
        if correction is not None:
            if len(structs) != 1:
                raise ValueError("a supplied correction needs exactly one scatterer")
            rowptr, col, val = correction
            rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
            col = np.ascontiguousarray(col, dtype=np.int32)
            val = np.ascontiguousarray(np.asarray(val, dtype=np.complex128)).view(np.float64)
            _check(L.ls_setup_from_csr(ctypes.byref(structs[0][0]), rowptr.ctypes.data, col.ctypes.data,
                                       val.ctypes.data, ctypes.byref(opts), ctypes.byref(self._h)))
        else:
            arr = (_Scatterer * len(structs))(*[s for s, _ in structs])
            _check(L.ls_setup(arr, len(structs), ctypes.byref(opts), ctypes.byref(self._h)))
        self.n = int(L.ls_num_nodes(self._h))
        self.n_scatterers = int(L.ls_num_scatterers(self._h))
        self.offsets = [int(L.ls_scatterer_offset(self._h, i)) for i in range(self.n_scatterers)]

    def close(self):
        if self._h:
            lib().ls_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _cols(self, x):
        import torch
        if x.dtype != torch.complex128 or not x.is_cuda:
            raise TypeError("vectors must be complex128 CUDA tensors")
        x2 = x.reshape(1, -1) if x.dim() == 1 else x
        if x2.dim() != 2 or x2.shape[-1] != self.n:
            raise ValueError(f"expected a (B, {self.n}) tensor")
        return x2.contiguous()

    def apply(self, x, precision="fp64", adjoint=False, out=None):
        import torch
        x2 = self._cols(x)
        if out is not None and not (out.is_contiguous() and out.shape == x2.shape and out.dtype == x2.dtype):
            raise ValueError("out must be a contiguous tensor shaped like x")
        y = torch.empty_like(x2) if out is None else out
        self.reserve(x2.shape[0], precision)
        fn = lib().ls_apply_adjoint if adjoint else lib().ls_apply
        _check(fn(self._h, x2.data_ptr(), y.data_ptr(), x2.shape[0], self.n, _PREC[precision], _stream()), self._h)
        return y.reshape(x.shape)

    def reserve(self, nrhs, precision="fp64"):
        """Grow the application workspace for nrhs columns (ls_reserve); apply() calls it itself."""
        _check(lib().ls_reserve(self._h, int(nrhs), _PREC[precision]), self._h)

    def apply_noalloc(self, x, out, precision="fp64"):
        """y = L x through ls_apply_noalloc (the library's fixed workspace; nothing allocated)."""
        x2 = self._cols(x)
        if not (out.is_contiguous() and out.shape == x2.shape and out.dtype == x2.dtype):
            raise ValueError("out must be a contiguous tensor shaped like x")
        _check(lib().ls_apply_noalloc(self._h, x2.data_ptr(), out.data_ptr(), x2.shape[0], self.n, _PREC[precision],
                                      _stream()), self._h)
        return out

    def apply_raw(self, x, out, precision="fp64", adjoint=False):
        """ls_apply (or ls_apply_adjoint) alone, without reserving: fails if the workspace is too small."""
        x2, y = self._cols(x), out
        fn = lib().ls_apply_adjoint if adjoint else lib().ls_apply
        _check(fn(self._h, x2.data_ptr(), y.data_ptr(), x2.shape[0], self.n, _PREC[precision], _stream()), self._h)
        return y

    def apply_adjoint(self, x, precision="fp64", out=None):
        return self.apply(x, precision, adjoint=True, out=out)

    def solve(self, b, tol=1e-8, maxit=1000, precision="fp64", adjoint=False, x0=None, inner_tol=0.0,
              inner_maxit=0, restart=0, scheme="relaxed", check_orth=False):
        """Solve L x = b (or L^H x = b) by GMRES (restart = 0: none); returns (x, info dict).
        precision="mixed": scheme "relaxed" (or flexible with inner_maxit > 0) or "passes"
        (mixed-precision refinement passes), see ls_solve_opts.  check_orth: also measure the
        Krylov basis's loss of orthogonality (info["orth_loss"])."""
        import torch
        b2 = self._cols(b)
        if x0 is not None:
            x = self._cols(x0).clone()
        else:
            x = torch.zeros_like(b2)
        B = b2.shape[0]
        iters = np.zeros(B, dtype=np.int32)
        relres = np.zeros(B, dtype=np.float64)
        o = _SolveOpts(float(tol), int(maxit), int(restart), _PREC[precision], int(bool(adjoint)), int(x0 is not None),
                       int(inner_maxit), float(inner_tol), _SCHEME[scheme], int(bool(check_orth)))
        info = _SolveInfo(iters.ctypes.data, relres.ctypes.data, 0, 0, 0.0, 0, 0.0)
        st = _check(lib().ls_solve_gmres(self._h, b2.data_ptr(), x.data_ptr(), B, self.n, ctypes.byref(o),
                                         ctypes.byref(info), _stream()), self._h)
        return x.reshape(b.shape), {"converged": st == LS_OK, "iters": iters, "relres": relres,
                                    "n_apply_fp64": info.n_apply_fp64, "n_apply_mixed": info.n_apply_mixed,
                                    "seconds": info.seconds, "n_reorth": info.n_reorth,
                                    "orth_loss": info.orth_loss}

    def grad_contrast(self, u, lam, a):
        import torch
        u2, l2, a2 = self._cols(u), self._cols(lam), self._cols(a)
        g = torch.empty(self.n, dtype=torch.float64, device=u2.device)
        _check(lib().ls_grad_contrast(self._h, u2.data_ptr(), l2.data_ptr(), a2.data_ptr(), u2.shape[0], self.n,
                                      g.data_ptr(), _stream()), self._h)
        return g

    def set_contrast(self, m):
        """Replace the contrast (CUDA tensor of all nodes, real or complex); C is kept."""
        import torch
        mc = m.to(torch.complex128).contiguous()
        if mc.numel() != self.n or not mc.is_cuda:
            raise ValueError(f"expected a CUDA tensor with {self.n} entries")
        _check(lib().ls_set_contrast(self._h, mc.data_ptr(), _stream()), self._h)
        self._m_keep = mc

    def farfield(self, u, thetas, data=None, s=0):
        """Far-field pattern of scatterer s at angles thetas; with data also the residual and
        the misfit 1/2 sum |uinf - data|^2.  Returns (uinf, res or None, J or None)."""
        import torch
        u2 = self._cols(u)
        th = np.ascontiguousarray(thetas, dtype=np.float64)
        B, R = u2.shape[0], th.size
        uinf = torch.empty((B, R), dtype=torch.complex128, device=u2.device)
        res = J = None
        dptr = None
        if data is not None:
            data = data.to(torch.complex128).reshape(B, R).contiguous()
            res = torch.empty_like(uinf)
            dptr = data.data_ptr()
            Jh = ctypes.c_double()
        _check(lib().ls_farfield(self._h, s, u2.data_ptr(), B, self.n, th.ctypes.data, R, dptr, uinf.data_ptr(),
                                 res.data_ptr() if res is not None else None,
                                 ctypes.byref(Jh) if data is not None else None, _stream()), self._h)
        if data is not None:
            J = Jh.value
        return uinf, res, J

    def field(self, u, tx, ty, s=0):
        """Scattered field -k^2 V~[m u] of scatterer s at points (tx, ty) outside it (host
        arrays); u: (B, N) nodal solution.  Returns a (B, T) complex128 CUDA tensor."""
        import torch
        u2 = self._cols(u)
        tx = np.ascontiguousarray(tx, dtype=np.float64).ravel()
        ty = np.ascontiguousarray(ty, dtype=np.float64).ravel()
        if tx.size != ty.size:
            raise ValueError("tx and ty differ in length")
        out = torch.empty((u2.shape[0], tx.size), dtype=torch.complex128, device=u2.device)
        _check(lib().ls_field(self._h, s, tx.ctypes.data, ty.ctypes.data, tx.size, u2.data_ptr(), u2.shape[0],
                              self.n, out.data_ptr(), _stream()), self._h)
        return out

    def set_grid(self, x0, y0, h, nx, ny, s=0):
        """Cartesian grid of the transfer operators of scatterer s (node (ix, iy) at
        (x0 + ix h, y0 + iy h), numbered iy nx + ix); see ls_transfer_setup."""
        g = _Grid(float(x0), float(y0), float(h), int(nx), int(ny))
        _check(lib().ls_transfer_setup(self._h, s, ctypes.byref(g)), self._h)
        self._grids = getattr(self, "_grids", {})
        self._grids[s] = int(nx) * int(ny)

    def _grid_n(self, s):
        n = getattr(self, "_grids", {}).get(s)
        if n is None:
            raise LSError(LS_ERR_ARG, "no grid for this scatterer (set_grid)")
        return n

    def transfer_colsums(self, s=0):
        """D of eq. D_def (column sums of T_C^Q, 1 where zero) for scatterer s's grid, host array."""
        d = np.empty(self._grid_n(s), dtype=np.float64)
        _check(lib().ls_transfer_colsums(self._h, s, d.ctypes.data), self._h)
        return d

    def quad_to_cart(self, x, s=0):
        """T_Q^C x: grid values (B, nx ny) from the node values of scatterer s in x (B, N)."""
        import torch
        x2 = self._cols(x)
        c = torch.empty((x2.shape[0], self._grid_n(s)), dtype=torch.complex128, device=x2.device)
        _check(lib().ls_quad_to_cart(self._h, s, x2.data_ptr(), self.n, c.data_ptr(), c.shape[1], x2.shape[0],
                                     _stream()), self._h)
        return c

    def cart_to_quad(self, c, s=0):
        """T_C^Q c on scatterer s's nodes: (B, N), zero on the other scatterers."""
        import torch
        c = c.to(torch.complex128).contiguous()
        if c.dim() == 1:
            c = c[None, :]
        if c.shape[1] != self._grid_n(s):
            raise ValueError("grid vectors must have nx ny entries")
        y = torch.zeros((c.shape[0], self.n), dtype=torch.complex128, device=c.device)
        _check(lib().ls_cart_to_quad(self._h, s, c.data_ptr(), c.shape[1], y.data_ptr(), self.n, c.shape[0],
                                     _stream()), self._h)
        return y

    def precondition(self, x, S, s=0):
        """P x = x + T_C^Q (S - I) T_Q^C x on scatterer s (eq. preconditioner_factored), for a
        Cartesian approximate inverse S given as a callable on (B, nx ny) CUDA tensors; the other
        scatterers' entries of x are returned unchanged."""
        import torch
        x2 = self._cols(x)
        c = self.quad_to_cart(x2, s)
        sc = S(c).to(torch.complex128).contiguous()
        if sc.shape != c.shape:
            raise ValueError("S must return a grid vector of the shape it was given")
        y = x2.clone()
        _check(lib().ls_precond_finish(self._h, s, x2.data_ptr(), self.n, c.data_ptr(), sc.data_ptr(), c.shape[1],
                                       y.data_ptr(), x2.shape[0], _stream()), self._h)
        return y.reshape(x.shape)

    def sparsify_setup(self, x0, y0, h, nx, ny, m_grid, s=0):
        """Build the library's sparsifying preconditioner S^(C) of scatterer s on the grid
        (x0 + ix h, y0 + iy h) with the contrast m_grid (nx ny values in grid order, 0 outside the
        scatterer); also sets the transfer grid.  Returns the build info (see ls_sparsify_setup)."""
        g = _Grid(float(x0), float(y0), float(h), int(nx), int(ny))
        m = np.ascontiguousarray(np.asarray(m_grid, dtype=np.complex128).ravel())
        if m.size != int(nx) * int(ny):
            raise ValueError("m_grid must have nx ny entries")
        info = _SparsifyInfo()
        _check(lib().ls_sparsify_setup(self._h, s, ctypes.byref(g), m.ctypes.data, ctypes.byref(info)), self._h)
        self._grids = getattr(self, "_grids", {})
        self._grids[s] = int(nx) * int(ny)
        self._sparsified = getattr(self, "_sparsified", set()) | {s}
        return {"build_seconds": info.build_seconds, "sv_ratio": info.sv_ratio, "lu_residual": info.lu_residual,
                "device_bytes": info.device_bytes}

    def sparsify_apply(self, c, s=0, adjoint=False):
        """S^(C) c (or its adjoint) for grid vectors c of shape (B, nx ny) (complex128 CUDA)."""
        import torch
        c = c.to(torch.complex128).contiguous()
        if c.dim() == 1:
            c = c[None, :]
        if c.shape[1] != self._grid_n(s):
            raise ValueError("grid vectors must have nx ny entries")
        out = torch.empty_like(c)
        _check(lib().ls_sparsify_apply(self._h, s, c.data_ptr(), c.shape[1], out.data_ptr(), c.shape[0],
                                       int(bool(adjoint)), _stream()), self._h)
        return out

    def solve_precond(self, b, S=None, s=0, tol=1e-8, maxit=1000, restart=0, adjoint=False, precision="fp64",
                      inner_tol=0.0, scheme="relaxed", check_orth=False):
        """GMRES preconditioned on the right by P = I + T_C^Q (S - I) T_Q^C.  S=None: the library's
        sparsifying S^(C) on every scatterer that has one (sparsify_setup; s is ignored).  Otherwise S
        is a callable on (B, nx ny) CUDA tensors for scatterer s (set_grid first).  precision="mixed"
        relaxes the operator applications to the mixed-precision tiles late in the iteration (or runs
        refinement passes, scheme="passes").  check_orth as in solve.  Returns (x, info)."""
        import torch
        b2 = self._cols(b)
        B = b2.shape[0]
        if S is None:
            x = torch.zeros_like(b2)
            iters = np.zeros(B, dtype=np.int32)
            relres = np.zeros(B, dtype=np.float64)
            o = _SolveOpts(float(tol), int(maxit), int(restart), _PREC[precision], int(bool(adjoint)), 0, 0,
                           float(inner_tol), _SCHEME[scheme], int(bool(check_orth)))
            info = _SolveInfo(iters.ctypes.data, relres.ctypes.data, 0, 0, 0.0, 0, 0.0)
            st = _check(lib().ls_solve_gmres_precond(self._h, b2.data_ptr(), x.data_ptr(), B, self.n, ctypes.byref(o),
                                                     -1, _GridOp(), None, None, None, 0, ctypes.byref(info),
                                                     _stream()), self._h)
            return x.reshape(b.shape), {"converged": st == LS_OK, "iters": iters, "relres": relres,
                                        "n_apply_fp64": info.n_apply_fp64, "n_apply_mixed": info.n_apply_mixed,
                                        "seconds": info.seconds, "n_reorth": info.n_reorth,
                                        "orth_loss": info.orth_loss}
        nc = self._grid_n(s)
        c = torch.empty((B, nc), dtype=torch.complex128, device=b2.device)
        sc = torch.empty_like(c)
        failed = []

        def cb(cp, scp, nrhs, ldc, user, stream):
            try:
                out = S(c)
                if out.shape != c.shape:
                    raise ValueError("S must return a grid vector of the shape it was given")
                sc.copy_(out)
                return LS_OK
            except Exception as e:   # reported after the library returns
                failed.append(e)
                return LS_ERR_ARG

        fn = _GridOp(cb)
        x = torch.zeros_like(b2)
        iters = np.zeros(B, dtype=np.int32)
        relres = np.zeros(B, dtype=np.float64)
        o = _SolveOpts(float(tol), int(maxit), int(restart), _PREC[precision], int(bool(adjoint)), 0, 0,
                       float(inner_tol), _SCHEME[scheme], int(bool(check_orth)))
        info = _SolveInfo(iters.ctypes.data, relres.ctypes.data, 0, 0, 0.0, 0, 0.0)
        st = lib().ls_solve_gmres_precond(self._h, b2.data_ptr(), x.data_ptr(), B, self.n, ctypes.byref(o), s, fn,
                                          None, c.data_ptr(), sc.data_ptr(), nc, ctypes.byref(info), _stream())
        if failed:
            raise failed[0]
        _check(st, self._h)
        return x.reshape(b.shape), {"converged": st == LS_OK, "iters": iters, "relres": relres,
                                    "n_apply_fp64": info.n_apply_fp64, "n_apply_mixed": info.n_apply_mixed,
                                    "seconds": info.seconds, "n_reorth": info.n_reorth, "orth_loss": info.orth_loss}

    def farfield_adjoint(self, res, thetas, s=0):
        """(a, rhs) with a = A^H res and rhs = conj(m) a on scatterer s (zero elsewhere)."""
        import torch
        th = np.ascontiguousarray(thetas, dtype=np.float64)
        res = res.to(torch.complex128).contiguous()
        B = res.shape[0]
        a = torch.zeros((B, self.n), dtype=torch.complex128, device=res.device)
        rhs = torch.zeros_like(a)
        _check(lib().ls_farfield_adjoint(self._h, s, res.data_ptr(), B, self.n, th.ctypes.data, th.size,
                                         a.data_ptr(), rhs.data_ptr(), _stream()), self._h)
        return a, rhs

    def autotune(self, nrhs, precision="mixed", cache=None):
        """Pick the batched tile shape for nrhs right-hand sides by timing candidates on this
        handle's geometry (see ls_autotune).  With cache (a JSON path) the choice is read from /
        written to a table keyed by GPU architecture, size bucket, scatterer count, nrhs and
        precision.  Returns (mt, split_len, far_ms or None when taken from the cache)."""
        import json
        import math

        import torch
        arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
        key = f"{arch}|n2^{int(math.log2(max(self.n, 1)))}|s{self.n_scatterers}|b{nrhs}|{precision}"
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            mt, sl = table[key]
            _check(lib().ls_set_tile_shape(self._h, _PREC[precision], mt, sl), self._h)
            return mt, sl, None
        r = _TuneResult()
        _check(lib().ls_autotune(self._h, int(nrhs), _PREC[precision], ctypes.byref(r), _stream()), self._h)
        if cache:
            table[key] = [r.mt, r.split_len]
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return r.mt, r.split_len, r.far_ms

    def set_tile_shape(self, mt, split_len, precision="mixed"):
        _check(lib().ls_set_tile_shape(self._h, _PREC[precision], int(mt), int(split_len)), self._h)

    def profile(self, enable=None, reset=False):
        """Turn kernel timing on/off (enable=True/False) or read the totals (enable=None)."""
        if enable is not None:
            _check(lib().ls_profile_enable(self._h, int(bool(enable))), self._h)
            return None
        p = _Profile()
        _check(lib().ls_profile_query(self._h, ctypes.byref(p), int(bool(reset))), self._h)
        return {"far_launches": p.far_launches, "far_ms": p.far_ms, "apply_calls": p.apply_calls,
                "apply_ms": p.apply_ms, "pair_rhs": p.pair_rhs, "far_launches_mixed": p.far_launches_mixed,
                "far_ms_mixed": p.far_ms_mixed, "pair_rhs_mixed": p.pair_rhs_mixed,
                "far_launches_h16": p.far_launches_h16, "far_ms_h16": p.far_ms_h16,
                "pair_rhs_h16": p.pair_rhs_h16}

    def correction_nnz(self, s=0):
        return int(lib().ls_correction_nnz(self._h, s))

    def near_pairs(self, s=0):
        """Pairs with z < 1 that mixed applications take in FP64 (0: in the mixed tiles)."""
        return int(lib().ls_near_pairs(self._h, s))

    def export_correction(self, s=0):
        """Scatterer s's correction C as (rowptr, col, val) in the caller's node order."""
        L = lib()
        nnz = self.correction_nnz(s)
        n = (self.offsets[s + 1] if s + 1 < self.n_scatterers else self.n) - self.offsets[s]
        rowptr = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(max(nnz, 1), dtype=np.int32)
        val = np.zeros(max(nnz, 1), dtype=np.complex128)
        _check(L.ls_export_correction(self._h, s, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data), self._h)
        return rowptr, col[:nnz], val[:nnz]


def sparsify_stencil_host(h, nx, ny, k, m_grid):
    """The library's host construction of the sparsifying preconditioner's stencils on an nx x ny
    grid of spacing h: (W, E, sv_ratio) with W[j, o] = A[j, j + off(o)], E[j, o] = C^(C)[j, j + off(o)]
    (complex (nx ny, 9)), off(o) = (o % 3 - 1) + (o // 3 - 1) nx.  Needs no GPU."""
    g = _Grid(0.0, 0.0, float(h), int(nx), int(ny))
    m = np.ascontiguousarray(np.asarray(m_grid, dtype=np.complex128).ravel())
    nc = int(nx) * int(ny)
    if m.size != nc:
        raise ValueError("m_grid must have nx ny entries")
    W = np.empty((nc, 9), dtype=np.complex128)
    E = np.empty((nc, 9), dtype=np.complex128)
    r = ctypes.c_double()
    _check(lib().ls_sparsify_stencil_host(ctypes.byref(g), float(k), m.ctypes.data, W.ctypes.data, E.ctypes.data,
                                          ctypes.byref(r)))
    return W, E, r.value


def eval_green(z2, single=False):
    """G(z) = (i/4) H0^(1)(z) at z^2 values (float64 CUDA tensor) with the kernels' evaluation."""
    import torch
    z2 = z2.contiguous()
    g = torch.empty(z2.shape, dtype=torch.complex128, device=z2.device)
    _check(lib().ls_eval_green(z2.data_ptr(), g.data_ptr(), z2.numel(), int(bool(single)), _stream()))
    return g


def device_allocations():
    """Device allocations the library has made in this process (ls_device_allocations)."""
    return int(lib().ls_device_allocations())


def eval_green_host(z2):
    """Same evaluation compiled for the host CPU (numpy in, numpy complex128 out)."""
    z2 = np.ascontiguousarray(z2, dtype=np.float64)
    g = np.empty(z2.shape, dtype=np.complex128)
    _check(lib().ls_eval_green_host(z2.ctypes.data, g.ctypes.data, z2.size))
    return g


def _autograd():
    import torch

    class FarFieldMisfit(torch.autograd.Function):
        """J(m) = 1/2 sum_{d,r} |u_inf,d(theta_r) - data_{d,r}|^2 with L(m) u_d = b_d.

        forward: set the contrast, solve, far field and misfit; only the converged fields u and the
        far-field residual are kept (no Krylov vectors).  A forward or adjoint solve that misses
        tol within maxit raises LSError (status LS_NOT_CONVERGED) instead of returning a misfit or
        gradient of an unconverged field.  backward: a = A^H res, adjoint solve
        L^H lam = conj(m) a, grad_j = sum_d Re[conj(a_jd - k^2 (V^H lam_d)_j) u_jd].
        """

        @staticmethod
        def forward(ctx, m, op, b, data, thetas, tol, maxit, precision, adjoint_maxit):
            op.set_contrast(m)
            u, info = op.solve(b, tol=tol, maxit=maxit, precision=precision)
            if not info["converged"]:
                raise LSError(LS_NOT_CONVERGED, f"forward solve missed tol {tol:g} in {maxit} steps "
                                                f"(largest relative residual {float(np.max(info['relres'])):.2e})")
            _, res, J = op.farfield(u, thetas, data)
            ctx.op, ctx.thetas, ctx.tol, ctx.precision = op, thetas, tol, precision
            ctx.maxit = adjoint_maxit if adjoint_maxit is not None else maxit
            ctx.solve_info = info
            ctx.save_for_backward(m, u, res)
            return torch.tensor(J, dtype=torch.float64, device=m.device)

        @staticmethod
        def backward(ctx, gJ):
            m, u, res = ctx.saved_tensors
            op = ctx.op
            op.set_contrast(m)
            a, rhs = op.farfield_adjoint(res, ctx.thetas)
            lam, info = op.solve(rhs, tol=ctx.tol, maxit=ctx.maxit, precision=ctx.precision, adjoint=True)
            if not info["converged"]:
                raise LSError(LS_NOT_CONVERGED, f"adjoint solve missed tol {ctx.tol:g} in {ctx.maxit} steps "
                                                f"(largest relative residual {float(np.max(info['relres'])):.2e})")
            g = op.grad_contrast(u, lam, a)
            return gJ * g, None, None, None, None, None, None, None, None

    return FarFieldMisfit


def farfield_misfit(m, op, b, data, thetas, tol=1e-10, maxit=2000, precision="fp64", adjoint_maxit=None):
    """Differentiable far-field misfit J(m) (real contrast m as a float64 CUDA tensor); the adjoint
    solve of the backward pass takes adjoint_maxit steps at most (default: maxit)."""
    return _autograd().apply(m, op, b, data, thetas, tol, maxit, precision, adjoint_maxit)
