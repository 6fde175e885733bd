/* ls.h -- C ABI of the MI355X (gfx950) Lippmann-Schwinger Nystrom operator library (libls.so).
 *
 * Problem (paper, Section 2, eqs. Lippmann-Schwinger_Omega and contrast_def): the total field u
 * satisfies u + k^2 V[m u] = u_inc on the support Omega of the contrast m = 1 - n, with the
 * Green's function G(x, y) = (i/4) H0^(1)(k |x - y|).
 * Discretisation (Section 3, eqs. linear_system, nystrom_linear_system, linear_system_matrix):
 * at the N quadrature nodes y_j of a curved triangular mesh with weights w_j,
 *     L u = b,  L = I + k^2 V M,  V = G~ W + C,  M = diag(m(y_j)),  b_j = u_inc(y_j),
 * where (G~)_jn = G(y_j, y_n) for j != n and 0 for j = n, W = diag(w), and C is the sparse
 * near-singular correction of the density-interpolation (VDIM) scheme (eq. DIM_decomp): for each
 * subdomain l and node j it has 10 entries on one element of l,
 *     C_jn = E_l[L_n](y_j) - sum_{q in l, q != j} G(y_j, y_q) w_q L_n(y_q),
 * with L_n the cubic Lagrange basis of that element and E_l[P](x) = int_{Omega_l} G(x,y) P(y) dy.
 *
 * Conventions
 *   - Complex vectors are interleaved (re, im) doubles (the layout of torch.complex128).
 *   - Right-hand-side blocks are RHS-major: column c of a block starts at ptr + 2*c*ld doubles.
 *   - A handle may hold several independent scatterers; vectors are then the concatenation of
 *     the scatterers' node sets in the order given to ls_setup, and every column has that layout.
 *   - Vectors are always read and written in the caller's node order (the library reorders nodes
 *     internally for locality).
 *   - x, y, b, u, lam, a, grad arguments are DEVICE pointers owned by the caller; setup inputs
 *     are HOST pointers copied by the call.  All device work is enqueued on the given stream.
 *   - Every call validates its arguments before enqueuing anything and returns an ls_status;
 *     ls_last_error(h) gives a message for the last failure on h.  A handle must not be used by
 *     two host threads at once.
 */
#ifndef LS_H_
#define LS_H_

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LS_OK = 0,
  LS_NOT_CONVERGED = 1,     /* ls_solve_gmres: maxit reached; x holds the last iterate */
  LS_ERR_ARG = -1,          /* invalid argument (nothing was enqueued) */
  LS_ERR_HIP = -2,          /* a HIP runtime call failed */
  LS_ERR_ALLOC = -3,        /* device or host allocation failed */
  LS_ERR_BREAKDOWN = -4,    /* Krylov breakdown with a non-finite value */
  LS_ERR_NONFINITE = -5,    /* non-finite right-hand side or initial guess */
  LS_ERR_UNSUPPORTED = -6
} ls_status;

typedef enum {
  LS_FP64 = 0,   /* every operation in FP64 */
  LS_MIXED = 1   /* Green's tiles in FP32 (matrix cores), FP64 correction / small arguments */
} ls_precision;

enum { LS_CIRCLE = 0, LS_ELLIPSE = 1 };

/* A closed analytic boundary curve of one subdomain, parametrised by t in [0, 2 pi):
 * (cx + a cos t, cy + b sin t) (a = b for a circle).  orientation = +1 if the subdomain lies
 * inside the curve, -1 if it lies outside it (e.g. the inner circle of an annulus). */
typedef struct {
  int32_t kind;
  int32_t orientation;
  int32_t subdomain;
  int32_t pad_;
  double cx, cy, a, b;
} ls_curve;

/* One scatterer.  Nodes come in groups of nq = 10 per element (element e owns nodes 10e..10e+9);
 * elem_subdomain gives the subdomain (0..n_sub-1) of every element; the curves are the boundaries
 * of every subdomain (Section 3, eq. vol_pot_decomp).  m is the complex contrast 1 - n at the nodes
 * (interleaved, 2*n_nodes doubles).  All pointers are host pointers. */
typedef struct {
  int64_t n_nodes;
  int32_t n_elems;
  int32_t nq;
  const double *x, *y, *w;
  const int32_t *elem_subdomain;
  const double *m;
  double k;
  int32_t n_curves;
  int32_t pad_;
  const ls_curve *curves;
} ls_scatterer;

typedef struct {
  int32_t source_split;     /* far-sum source chunks per launch (0 = automatic); for one right-hand side and
                             * one target per lane, ceil(N / 256) chunks select the sum that evaluates each
                             * unordered pair once (automatic from N ~ 16 000 on) */
  int32_t rhs_chunk;        /* RHS per pass of the batched FP64 kernel (0 = automatic; 1, 4, 8, 16) */
  int32_t targets_per_lane; /* targets per lane in the FP64 far sum (0 = automatic; 1 or 2) */
  int32_t mixed_tile;       /* mixed-precision tile variant (0 = automatic / autotuned cache) */
  int32_t n_threads_host;   /* host threads for setup (0 = all) */
  int32_t fp64_matrix;      /* FP64 batched sum on the matrix cores: 0 = when nrhs >= 4, 1 = never, 2 = always */
  int32_t mixed_fp16;       /* LS_MIXED tiles on split FP16 (each operand a sum of two FP16 numbers, three FP16
                             * matrix-core products with FP32 accumulation per real product, one launch per
                             * scatterer) instead of FP32: 0 = for single-scatterer handles when nrhs rounds up
                             * to a multiple of 64, 1 = always, 2 = never */
  int32_t mixed_near;       /* LS_MIXED applications and the far sum's pairs with z = k |y_j - y_n| < 1 (the
                             * logarithmic part of G): 0 = left out of the mixed tiles and added by an FP64
                             * near launch (FP64 Green's values and contraction over per-tile source lists
                             * built at setup), unless they exceed 512 per node on average; 1 = in the mixed
                             * tiles like every other pair (G from the FP64 series, rounded to the tile
                             * precision) */
} ls_options;

typedef struct ls_ctx *ls_handle;

/* Build the operator for n_scatterers scatterers: sorts nodes, assembles the correction C
 * (exact polynomial potentials by Green's third identity on the boundary curves plus punctured
 * Green's sums on the GPU) and C^H, and uploads everything to the current HIP device.
 * Synchronous.  opt may be NULL. */
ls_status ls_setup(const ls_scatterer *s, int32_t n_scatterers, const ls_options *opt,
                   ls_handle *out);

/* Same as ls_setup for one scatterer, but with C supplied by the caller as a CSR matrix in the
 * caller's node order (rowptr[n_nodes+1], col[nnz], val[2*nnz] interleaved complex; host). */
ls_status ls_setup_from_csr(const ls_scatterer *s, const int64_t *rowptr, const int32_t *col,
                            const double *val, const ls_options *opt, ls_handle *out);

/* y = L x for nrhs columns (x, y: device, complex, leading dimension ld >= total nodes).
 * Asynchronous on stream.  Allocates nothing: the handle's workspace must already hold what nrhs
 * columns in precision p need (ls_reserve), else LS_ERR_ARG and nothing is enqueued.  With several
 * scatterers on the matrix cores the call copies its launch tables to the device and waits for
 * that copy when nrhs or p differ from the previous such application. */
ls_status ls_apply(ls_handle h, const double *x, double *y, int32_t nrhs, int64_t ld,
                   ls_precision p, hipStream_t stream);

/* y = L^H x = x + k^2 conj(m) (W conj(G~) x + C^H x)  (exact adjoint of ls_apply in FP64); the
 * workspace rules of ls_apply apply. */
ls_status ls_apply_adjoint(ls_handle h, const double *x, double *y, int32_t nrhs, int64_t ld,
                           ls_precision p, hipStream_t stream);

/* Grow the handle's application workspace (and, with several scatterers, its launch tables) to
 * what ls_apply / ls_apply_adjoint need for nrhs columns in precision p; a no-op when it is large
 * enough.  Synchronous (waits for the device before replacing a workspace). */
ls_status ls_reserve(ls_handle h, int32_t nrhs, ls_precision p);

/* Number of device allocations the library has made in this process (all handles), for checking
 * that a sequence of calls allocated nothing. */
int64_t ls_device_allocations(void);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops or
 * harnesses that forbid hipMalloc): y = L x as ls_apply computes it, with every temporary taken
 * from the library's fixed per-GPU workspace of 64 MiB (a static device array that each GPU the
 * library runs on holds until the process ends).  Same arguments as ls_apply; the same result up
 * to the order of the floating-point sums over source splits (a scatterer whose sums need more
 * room than the workspace holds takes fewer splits; FP32 tiles then accumulate longer partial
 * sums).  Each scatterer takes its own launch.  Allocates nothing and never waits on the device.
 * Sizes whose workspace exceeds 64 MiB (about nrhs x nodes > 1.3e6 for the FP64 sum, less for the
 * tiles) are rejected with LS_ERR_ARG before anything is enqueued.  Every call on a GPU uses that
 * GPU's one workspace, whatever the handle or stream: calls that overlap in time on one GPU race
 * and must be ordered by the caller. */
ls_status ls_apply_noalloc(ls_handle h, const double *x, double *y, int32_t nrhs, int64_t ld, ls_precision p,
                           hipStream_t stream);

typedef struct {
  double tol;          /* relative residual ||b - L x||_2 / ||b||_2 per column */
  int32_t maxit;       /* outer iterations (Arnoldi steps) */
  int32_t restart;     /* 0 = no restart */
  int32_t prec;        /* ls_precision, see below */
  int32_t adjoint;     /* solve L^H x = b instead */
  int32_t x0_given;    /* use x as the initial guess */
  int32_t inner_maxit; /* LS_MIXED: > 0 selects flexible GMRES with this many inner steps */
  double inner_tol;    /* LS_MIXED: inner tolerance (flexible), granted operator accuracy (relaxed) or
                        * residual reduction per pass (mixed_scheme 1) */
  int32_t mixed_scheme;/* LS_MIXED: 0 = relaxed or flexible as below, 1 = refinement passes */
  int32_t check_orth;  /* nonzero: measure the Arnoldi basis's loss of orthogonality (one more pass of
                        * inner products per step over the basis, about the cost of the
                        * Gram-Schmidt pass itself), reported in ls_solve_info.orth_loss */
  /* LS_MIXED solves keep the Krylov basis, orthogonalisation and residuals in FP64.
   *   inner_maxit > 0: flexible GMRES; each outer direction is preconditioned by up to
   *                    inner_maxit steps of GMRES with the mixed operator (to inner_tol,
   *                    default 1e-12, i.e. exactly inner_maxit steps).
   *   inner_maxit = 0: relaxed GMRES; FP64 applications while the residual estimate exceeds
   *                    0.3 tol / inner_tol, mixed ones after, then FP64 refinement passes from
   *                    the true residual if tol was missed.  Default inner_tol 1e-4 (switch at
   *                    3e-5 for tol 1e-8): the mixed operator's error is below 1e-6 at N ~ 1e5,
   *                    but switching earlier (inner_tol 1e-5 or 3e-5) slowed the k = 40 disk
   *                    solve from 1 069 to 1 471-1 560 steps.
   *   mixed_scheme = 1: refinement passes; every Arnoldi application uses the mixed operator,
   *                    each pass is a GMRES cycle from the FP64 residual that stops once its
   *                    estimate has fallen by the factor inner_tol (default 1e-5) or below
   *                    0.3 tol, and passes repeat until the residual meets tol (one FP64
   *                    application per pass).  A pass whose FP64 starting residual r is small
   *                    (1e-5 ||r|| <= tol ||b|| / 2) closes on r - L_mixed dx, dx its correction
   *                    of x, formed from the Arnoldi basis (V Q^H g_m e_m, no operator
   *                    application), instead of a new FP64 residual.  That differs from b - L x
   *                    by the mixed far sum's error on dx, bounded by
   *                    1e-5 (||r|| + ||r - L_mixed dx|| + ||dx||) (50 times the mixed operators'
   *                    measured error), and a column counts as converged only if its updated
   *                    residual plus that bound meets tol.  inner_maxit is ignored.
   * With several scatterers in the handle, every (column, scatterer) pair is an independent
   * system with its own Krylov space and convergence test; iters reports the most steps any
   * scatterer of the column took, relres the residual over the whole column. */
} ls_solve_opts;

typedef struct {
  int32_t *iters;       /* [nrhs] host, may be NULL: Arnoldi steps per column */
  double *relres;       /* [nrhs] host, may be NULL: final true relative residual (FP64 apply; for
                         * refinement passes that closed on the residual update, the updated
                         * residual, within the bound given above of the FP64 one) */
  int64_t n_apply_fp64; /* FP64 operator applications (per column count summed) */
  int64_t n_apply_mixed;
  double seconds;
  int64_t n_reorth;     /* Arnoldi steps (summed over systems) that needed a second Gram-Schmidt pass */
  double orth_loss;     /* with check_orth: the largest |<v_i, v_j> - delta_ij| over the normalized
                         * basis vectors of the outer iteration (each system's own basis, every
                         * cycle), measured as each v_j is formed; 0 otherwise */
} ls_solve_info;

/* Solve L x = b (or L^H x = b) by GMRES without restart, x0 = 0 unless x0_given, each column
 * (and each scatterer of it) independently.  Synchronous.  Returns LS_NOT_CONVERGED if any
 * column missed tol.  The environment variable LS_PROGRESS=k prints a progress line to stderr
 * every k steps (flexible GMRES: every outer step). */
ls_status ls_solve_gmres(ls_handle h, const double *b, double *x, int32_t nrhs, int64_t ld,
                         const ls_solve_opts *o, ls_solve_info *info, hipStream_t stream);

/* grad_j (real, device, total nodes) = sum_d Re[conj(a_jd - k^2 (V^H lam_d)_j) u_jd]:
 * the gradient of a far-field misfit J = 1/2 sum_d ||A u_d - data_d||^2 with respect to real
 * nodal contrast values m_j, given the forward fields u (L u_d = b_d), the adjoint states lam
 * (L^H lam_d = conj(m) a_d) and a_d = A^H (A u_d - data_d), A the far-field map of ls_farfield.
 * It differentiates the Nystrom system L = I + k^2 V M of Section 3 (eqs. linear_system,
 * linear_system_matrix) through its exact adjoint, with the far-field pattern of the energy
 * balance of Section 5 (subsection on the energy balance, eq. dissipativity_identity); the paper
 * names inverse problems as the application this serves (Conclusion), without a gradient of its
 * own.  nrhs columns with leading dimension ld (device); grad is written, not accumulated. */
ls_status ls_grad_contrast(ls_handle h, const double *u, const double *lam, const double *a,
                           int32_t nrhs, int64_t ld, double *grad, hipStream_t stream);

/* Far field of scatterer s at R receiver angles thetas (host array):
 *   uinf[d*R + r] = -k^2 gamma sum_q w_q exp(-i k (cos t_r, sin t_r).y_q) m_q u_qd,
 *   gamma = exp(i pi/4)/sqrt(8 pi k)
 * (the far-field pattern of the scattered part of the representation formula, Section 2, in the
 * normalisation of the energy balance of Section 5).  u: device, nrhs columns with leading
 * dimension ld.  uinf: device, nrhs x R complex.  If data (device, nrhs x R) is given, res
 * (device, may be NULL) receives uinf - data and *misfit (host, may be NULL) the value
 * 1/2 sum |uinf - data|^2, in which case the call synchronises the stream. */
ls_status ls_farfield(ls_handle h, int32_t s, const double *u, int32_t nrhs, int64_t ld, const double *thetas,
                      int32_t R, const double *data, double *uinf, double *res, double *misfit,
                      hipStream_t stream);

/* Field recovery (Section 3, eq. field_recovery, the discrete representation formula of
 * Section 2): the scattered field u_s(x) = u(x) - u_inc(x) = -k^2 V~_Omega[m u](x) of scatterer s
 * at nt points x_t = (tx[t], ty[t]) outside it, for the nodal solution u:
 *   u_s(x_t) = -k^2 ( sum_n G(x_t, y_n) w_n m_n u_n + sum_c C_tc m_c u_c ),
 * with a correction row C_t per point built like the operator's (the VDIM map at a target that
 * is not a node: in every subdomain the element with the nearest centroid, and the exact
 * polynomial potential with the point outside).  tx, ty: host [nt] (any order).  u: device,
 * nrhs columns with leading dimension ld (all scatterers' layout; scatterer s's segment is
 * read).  out: device, nrhs x nt complex (row-major, leading dimension nt).  Points on or
 * inside a curve that encloses a subdomain of s are rejected with LS_ERR_ARG; non-finite
 * points with LS_ERR_NONFINITE.  Synchronous: the correction rows are assembled per call (host
 * threads and the GPU) in a workspace allocated and freed by the call. */
ls_status ls_field(ls_handle h, int32_t s, const double *tx, const double *ty, int64_t nt, const double *u,
                   int32_t nrhs, int64_t ld, double *out, hipStream_t stream);

/* Adjoint of the far-field map of scatterer s: a = A^H res and rhs = conj(m) a (the right-hand
 * side of the adjoint solve L^H lam = conj(m) a), each written for scatterer s's nodes of nrhs
 * columns with leading dimension ld (device; either may be NULL). */
ls_status ls_farfield_adjoint(ls_handle h, int32_t s, const double *res, int32_t nrhs, int64_t ld,
                              const double *thetas, int32_t R, double *a, double *rhs, hipStream_t stream);

/* Replace the contrast m = 1 - n of every scatterer (device, caller order, interleaved complex,
 * total nodes).  The correction C depends only on the geometry and k, so it is kept. */
ls_status ls_set_contrast(ls_handle h, const double *m, hipStream_t stream);

/* Batched matrix-core sum over several scatterers (handles with n_scatterers > 1 and either
 * LS_MIXED or the FP64 tiles): the tile shape is mt 16-target tiles per wavefront (FP32: 2 or 4,
 * FP64: 1 or 2) and split_len sources per work item.  ls_autotune times the candidate shapes on
 * this handle's own geometry for nrhs right-hand sides (far sum only, synchronous) and keeps the
 * fastest for later applications; ls_set_tile_shape sets one directly (e.g. from a cache).  The
 * candidate split lengths are 1024 .. 8192 in FP64 and 1024 or 2048 in FP32, whose partial sums
 * lose accuracy with length (default 2048 for both). */
typedef struct {
  int32_t mt;
  int32_t split_len;
  double far_ms;
} ls_tune_result;
ls_status ls_autotune(ls_handle h, int32_t nrhs, ls_precision p, ls_tune_result *out, hipStream_t stream);
ls_status ls_set_tile_shape(ls_handle h, ls_precision p, int32_t mt, int32_t split_len);

/* Transfer operators between scatterer s's nodes and a Cartesian grid, and the last step of
 * the preconditioner built from them (paper, Section 4).  The grid's node (ix, iy), 0 <= ix < nx,
 * 0 <= iy < ny, sits at (x0 + ix h, y0 + iy h) and is numbered j = iy nx + ix; grid vectors are
 * [nrhs][ldc] interleaved complex (device), ldc >= nx ny.  Node vectors x, y are the handle's
 * [nrhs][ld] vectors in caller order (ld >= total nodes); only scatterer s's segment is read or
 * written.  All three transfer calls are asynchronous on stream and allocate nothing. */
typedef struct {
  double x0, y0; /* grid origin */
  double h;      /* spacing > 0 */
  int32_t nx, ny;/* nodes per direction, >= 2 each, nx ny < 2^31 */
} ls_grid;

/* Builds T_C^Q (bilinear hat functions of the cell containing each node, eq. psi_def; a node on
 * a grid line takes the cell above/right of it, on the last line the one below/left) and
 * T_Q^C = D^-1 (T_C^Q)^T (Approach II, eqs. T_H^C_def and D_def; D_jj = 1 where no node reaches
 * j with a positive weight) for scatterer s, replacing an earlier grid.  Every node must lie in
 * [x0, x0 + (nx-1) h] x [y0, y0 + (ny-1) h], else LS_ERR_ARG.  Synchronous. */
ls_status ls_transfer_setup(ls_handle h, int32_t s, const ls_grid *g);
/* D of eq. D_def for scatterer s's grid: d[j] = column sum of T_C^Q (1 where it is zero), nx ny
 * doubles written to host memory.  With it, P^H = I + T_C^Q (D^-1 S^H D - I) T_Q^C, the right
 * preconditioner for the adjoint system when P is the one for L. */
ls_status ls_transfer_colsums(ls_handle h, int32_t s, double *d);
/* c = T_Q^C x (grid values from scatterer s's node values). */
ls_status ls_quad_to_cart(ls_handle h, int32_t s, const double *x, int64_t ld, double *c, int64_t ldc,
                          int32_t nrhs, hipStream_t stream);
/* y = T_C^Q c on scatterer s's nodes (the rest of y is left alone). */
ls_status ls_cart_to_quad(ls_handle h, int32_t s, const double *c, int64_t ldc, double *y, int64_t ld,
                          int32_t nrhs, hipStream_t stream);
/* y = x + T_C^Q (sc - c) on scatterer s's nodes: with c = T_Q^C x (ls_quad_to_cart) and sc = S c
 * for the caller's Cartesian approximate inverse S, this is y = P x with
 * P = I + T_C^Q (S - I) T_Q^C (eq. preconditioner_factored).  y may be x. */
ls_status ls_precond_finish(ls_handle h, int32_t s, const double *x, int64_t ld, const double *c, const double *sc,
                            int64_t ldc, double *y, int32_t nrhs, hipStream_t stream);

/* A Cartesian approximate inverse supplied by the caller: writes S c to sc for nrhs grid vectors
 * [nrhs][ldc] (device), stream-ordered on stream, and returns LS_OK (anything negative stops the
 * solve with that status). */
typedef ls_status (*ls_grid_op)(const double *c, double *sc, int32_t nrhs, int64_t ldc, void *user,
                                hipStream_t stream);

/* GMRES with the right preconditioner P = I + T_C^Q (S - I) T_Q^C (eq. preconditioner_factored):
 * flexible GMRES with z_j = P v_j, so S may be inexact or change between calls.  Two forms:
 *   s >= 0, S given: the caller's S on scatterer s (ls_transfer_setup first); the other
 *     scatterers' segments are not preconditioned.  c and sc are the caller's grid workspaces
 *     [nrhs][ldc] (device, ldc >= nx ny): the library writes T_Q^C v_j into c and calls
 *     S(c, sc, ...) once per step.  For an adjoint solve the caller's S must be the one for L^H.
 *   s = -1, S = NULL (c, sc, ldc, user ignored): the library's sparsifying S^(C) on every
 *     scatterer that has one (ls_sparsify_setup), each (column, scatterer) system preconditioned
 *     by its own scatterer's P; scatterers without one are not preconditioned.  Adjoint solves
 *     (o->adjoint) take P^H = I + T_C^Q (D^-1 S^H D - I) T_Q^C (D of eq. D_def), the
 *     preconditioner of L^H that corresponds to P.  The grid workspaces are the library's, one
 *     per scatterer.  With two or more scatterers still iterating, their preconditioner steps run
 *     side by side on three streams the handle creates on first use (default priority, on the
 *     current device, destroyed by ls_destroy); each waits on stream for the step's input and
 *     stream waits for all of them, so the call stays ordered on stream.
 * With o->prec = LS_MIXED the operator applications switch to the mixed precision once the
 * residual allows it, as in relaxed GMRES (o->inner_tol is the granted accuracy, default 1e-4),
 * followed by FP64 refinement; o->inner_maxit is ignored.  The relaxed cycle closes on its
 * Arnoldi-basis residual when that is within tol including the bound
 * 1e-5 (||L_mixed dm|| + ||dm||), dm = sum over its mixed steps of y_j z_j (y the cycle's
 * coefficients, z_j = P v_j), the most such steps can change the FP64 residual; otherwise it takes
 * the FP64 residual.  Everything else is as for ls_solve_gmres. */
ls_status ls_solve_gmres_precond(ls_handle h, const double *b, double *x, int32_t nrhs, int64_t ld,
                                 const ls_solve_opts *o, int32_t s, ls_grid_op S, void *user, double *c, double *sc,
                                 int64_t ldc, ls_solve_info *info, hipStream_t stream);

/* The sparsifying Cartesian preconditioner S^(C) = (C^(C))^-1 A of Section 4 (subsection
 * "Sparsifying preconditioner": eqs. LS_eq_on_cartesian_points, cart_neighbors_LS,
 * sparsifying_min, LC_def, S_minus_I) for scatterer s on the grid g, built by the library.
 *   Cartesian system: L^(C) = I + k^2 V^(C) M^(C), M^(C) = diag(m(z_j)) with m_grid the contrast
 *     m = 1 - n at the grid nodes (host, interleaved complex, nx ny values in grid order, 0 outside
 *     the scatterer), k the scatterer's wavenumber.  V^(C) is the first-order rule: h^2 G(z_i, z_j)
 *     off the diagonal, (-1 + (i pi/2) k a H1(k a)) / k^2 with a = h / sqrt(pi) on it (the
 *     paper's Duan-Rokhlin corrections are cited there, not given).
 *   A (eq. sparsifying_min): row j's weights on its 3 x 3 neighbourhood N(j) within the grid are
 *     the conjugate of the left singular vector of the smallest singular value of
 *     V^(C)(N(j), N(j)^c); rows with all 9 neighbours share the central node's weights, each edge
 *     and corner row has its own.  A row's weights are unique up to a unit factor, which S^(C)
 *     does not depend on.
 *   C^(C) (eq. LC_def): A L^(C) kept on the 3 x 3 pattern; factored by block LU with grid rows as
 *     blocks (no pivoting across blocks, partial pivoting inside; O(ny nx^3) host work, ny nx^2
 *     complex values twice on the device).
 * ls_sparsify_setup also sets the transfer grid of s (as ls_transfer_setup, replacing an earlier
 * grid and preconditioner).  Needs 3 <= nx <= 1536, ny >= 3.  Synchronous; LS_ERR_BREAKDOWN if a
 * diagonal block of the LU is singular.  info (host, may be NULL) receives the build time, the
 * central stencil's smallest / largest singular value, ||C x - y|| / ||y|| for a seeded y solved
 * through the factors, and the device bytes held. */
typedef struct {
  double build_seconds;
  double sv_ratio;
  double lu_residual;
  int64_t device_bytes;
} ls_sparsify_info;
ls_status ls_sparsify_setup(ls_handle h, int32_t s, const ls_grid *g, const double *m_grid, ls_sparsify_info *info);
/* sc = S^(C) c (adjoint = 0) or sc = (S^(C))^H c (adjoint != 0) for nrhs grid vectors [nrhs][ldc]
 * (device, c and sc distinct, ldc >= nx ny), asynchronous on stream.  The adjoint form may
 * allocate a grid workspace on its first use with a larger nrhs. */
ls_status ls_sparsify_apply(ls_handle h, int32_t s, const double *c, int64_t ldc, double *sc, int32_t nrhs,
                            int32_t adjoint, hipStream_t stream);
/* Host-only construction of A and C^(C) for the grid g (origin unused), wavenumber k and grid
 * contrast m_grid, as ls_sparsify_setup builds them: W[9 j + o] = A[j, j + off(o)] and
 * E[9 j + o] = C^(C)[j, j + off(o)] (interleaved complex, 9 nx ny values each; 0 where j + off(o)
 * is off the grid), off(o) = (o mod 3 - 1) + (o div 3 - 1) nx.  Needs no GPU. */
ls_status ls_sparsify_stencil_host(const ls_grid *g, double k, const double *m_grid, double *W, double *E,
                                   double *sv_ratio);

/* Introspection. */
int64_t ls_num_nodes(ls_handle h);                       /* total nodes */
int32_t ls_num_scatterers(ls_handle h);
int64_t ls_scatterer_offset(ls_handle h, int32_t s);     /* first node of scatterer s */
int64_t ls_correction_nnz(ls_handle h, int32_t s);
/* Ordered pairs (j, n), n != j, with z = k |y_j - y_n| < 1 of scatterer s that mixed-precision
 * applications take in FP64 (0: the mixed tiles keep them, see ls_options.mixed_near); -1 for a bad
 * argument. */
int64_t ls_near_pairs(ls_handle h, int32_t s);
/* Copy scatterer s's correction back in the caller's node order (host buffers of sizes
 * n_nodes+1, nnz, 2*nnz). */
ls_status ls_export_correction(ls_handle h, int32_t s, int64_t *rowptr, int32_t *col, double *val);

/* Diagnostic: G(z) = (i/4) H0^(1)(z) for n arguments given as z^2 (device in, device out,
 * interleaved complex) with the kernels' own FP64 evaluation, or FP32 when single != 0. */
ls_status ls_eval_green(const double *z2, double *g, int64_t n, int32_t single, hipStream_t stream);
/* Same evaluation compiled for the host CPU (host pointers), for checks without a GPU. */
ls_status ls_eval_green_host(const double *z2, double *g, int64_t n);

/* Kernel timing: when enabled, HIP events are recorded on the caller's stream around every
 * far-sum kernel launch and around every operator application; ls_profile_query synchronises
 * those events and returns the totals (milliseconds), optionally resetting them. */
typedef struct {
  int64_t far_launches;
  double far_ms;
  int64_t apply_calls;
  double apply_ms;
  double pair_rhs;      /* Green's interactions evaluated: sum over applications of
                         * N_s (N_s - 1) x right-hand sides over the scatterers computed */
  int64_t far_launches_mixed;  /* the part of the three figures above in mixed precision */
  double far_ms_mixed;
  double pair_rhs_mixed;
  int64_t far_launches_h16;    /* the part of the mixed figures due to split-FP16 tiles */
  double far_ms_h16;
  double pair_rhs_h16;
} ls_profile;
ls_status ls_profile_enable(ls_handle h, int32_t on);
ls_status ls_profile_query(ls_handle h, ls_profile *out, int32_t reset);

void ls_destroy(ls_handle h);
const char *ls_status_str(ls_status s);
const char *ls_last_error(ls_handle h);

#ifdef __cplusplus
}
#endif

#endif /* LS_H_ */
