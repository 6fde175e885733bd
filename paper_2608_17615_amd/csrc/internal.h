// Internal definitions shared by the library's translation units (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ls.h"

namespace lsk {

// One source of the single-RHS FP64 far sum: position and weighted density.
struct alignas(32) Src4 {
  double x, y, sr, si;
};

// Host geometry of one scatterer kept after setup (element frames, interpolation matrices,
// boundary curves); defined and used by setup.hip, for the correction rows of the operator and
// of field-recovery targets.
struct GeomData;

// Transfer operators between one scatterer's nodes and a Cartesian grid (transfer.hip): per
// node (internal order) the grid index of its cell's lower-left vertex and the four bilinear
// weights; T_Q^C = D^-1 (T_C^Q)^T as CSR over the grid nodes.  Device arrays are in ls_ctx::owned.
struct TransferData {
  double x0 = 0, y0 = 0, h = 0;
  int32_t nx = 0, ny = 0;
  int32_t *cell = nullptr;
  double4 *w = nullptr;             // weights of the vertices (ix, iy), (ix+1, iy), (ix, iy+1), (ix+1, iy+1)
  int64_t *rp = nullptr;            // [nx ny + 1]
  int32_t *col = nullptr;           // caller index of the node within the scatterer
  double *val = nullptr;
  std::vector<void *> bufs;         // the allocations above
  std::vector<double> colsum;       // D: column sums of T_C^Q per grid node (1 where zero), host
};

// The sparsifying Cartesian preconditioner S^(C) = (C^(C))^-1 A of one scatterer on its transfer
// grid (sparsify.hip): the stencil weights W of A and the entries E of C^(C) as [9][nx ny]
// (slot o = (dy + 1) 3 + (dx + 1)), the inverse diagonal blocks G_i of the block LU of C^(C)
// (grid rows as blocks) column-major (Gc) and row-major (Gr), and D, D^-1 of the transfer grid.
struct SparsifyData {
  int32_t nx = 0, ny = 0;
  double2 *W = nullptr, *E = nullptr, *Gc = nullptr, *Gr = nullptr;
  double *d = nullptr, *dinv = nullptr;
  double sv_ratio = 0, lu_residual = 0;
  int64_t bytes = 0;
  std::vector<void *> bufs;         // the allocations above
};

// One scatterer, all device arrays in the internal (sorted) node order.
struct Scat {
  int64_t n = 0, off = 0;     // nodes, offset in the concatenated caller vectors
  double k = 0;
  int32_t n_sub = 1;
  double *px = nullptr, *py = nullptr, *w = nullptr;
  double2 *pos = nullptr;     // (px, py) interleaved, read per source by the far sum
  double2 *m = nullptr;       // contrast
  int32_t *perm = nullptr;    // internal index -> caller index (within the scatterer)
  int64_t nnz = 0;
  int64_t *rp = nullptr, *rpH = nullptr;
  int32_t *ci = nullptr, *ciH = nullptr;
  double2 *cv = nullptr, *cvH = nullptr;
  // Mixed-precision applications and the far sum's pairs with z = k |y_j - y_n| < 1: unless the
  // options keep them in the mixed tiles, the tiles leave them out and an FP64 near launch adds
  // them, one wave per tile of 16 targets over the source intervals near_iv[near_rp[t] ..
  // near_rp[t + 1]) that hold every such source of the tile (intervals of 4-aligned [begin, end)).
  // near_ok is false without the lists, also when the pairs would exceed kNearPerNode per node on
  // average (a scatterer small against the wavelength).
  static constexpr int64_t kNearPerNode = 512;
  bool near_ok = false;
  int64_t near_pairs = 0;
  int32_t near_ntiles = 0;
  int32_t *near_rp = nullptr;
  int2 *near_iv = nullptr;
  std::vector<int32_t> perm_host;   // same as perm, on the host
  std::vector<double> w_host;       // the quadrature weights, internal order, on the host
  std::shared_ptr<GeomData> geom;
  std::shared_ptr<TransferData> tr; // set by ls_transfer_setup
  std::shared_ptr<SparsifyData> sp; // set by ls_sparsify_setup (dropped by a new transfer grid)
};

// One scatterer of a batched launch and one unit of its far-sum work.
struct BatchDesc {
  int n, split_len, excl;   // excl: leave the pairs with z < 1 out (the mixed correction adds them)
  double k2;
  const double2 *pos;
  const void *X;
  double2 *part;
};
struct WorkItem {
  int s, tblock, split, bgroup;
};

// Tile shape of the batched matrix-core sum: MT 16-target tiles per wavefront and the number of
// sources per work item; chosen by ls_autotune (0 = defaults).
struct TileTune {
  int mt = 0, split_len = 0;
  double ms = 0.0;
};

struct Workspace {
  void *ptr = nullptr;
  size_t bytes = 0;
};

// Host threads for setup work: opt.n_threads_host when set, else the CPUs this process may run on
// (its affinity mask), at most 16.
int host_threads(const ls_options &opt);

// Every device allocation of the library goes through dmalloc, which counts them (process-wide;
// ls_device_allocations reports the count).
void count_device_allocation();
template <class T>
hipError_t dmalloc(T **p, size_t bytes) {
  count_device_allocation();
  return hipMalloc((void **)p, bytes);
}

}  // namespace lsk

struct ls_ctx {
  std::vector<lsk::Scat> sc;
  bool prof = false;
  std::vector<hipEvent_t> ev_far, ev_apply;   // start/stop pairs, in launch order
  std::vector<char> ev_far_mixed;              // per far-sum launch: 0 FP64, 1 FP32 tiles, 2 split-FP16 tiles
  double prof_pairs = 0.0;                     // interactions evaluated while profiling
  double prof_pairs_mixed = 0.0;               // of which in mixed precision
  double prof_pairs_h16 = 0.0;                 // of which by split-FP16 tiles
  int64_t n_total = 0;
  int device = 0;
  ls_options opt{};
  std::string err;
  lsk::Workspace ws_apply, ws_solve, ws_ff, ws_grid;
  lsk::TileTune tune[2];                 // [single]
  void *batch_tables = nullptr;          // device BatchDesc[] + WorkItem[] + counter
  size_t batch_bytes = 0;
  long long batch_key = -1;              // configuration the cached tables describe
  // scatterers an operator application may leave out (empty: none).  Set only by the solver for
  // the duration of its own applications: the output segments of skipped scatterers are left
  // unwritten, and the solver never reads them (their systems have all finished).
  std::vector<char> scat_skip;
  std::vector<void *> owned;  // device allocations freed by ls_destroy
  // streams (default priority) on which the solver runs the preconditioners of several scatterers
  // side by side, with a fork event and one join event each; created on first use
  std::vector<hipStream_t> aux_streams;
  std::vector<hipEvent_t> aux_join;
  hipEvent_t aux_fork = nullptr;
};

namespace lsk {

// Forward: y = L x;  Adjoint: y = L^H x;  AdjointPotential: y = V^H x = W conj(G~) x + C^H x.
enum class Mode { Forward, Adjoint, AdjointPotential };

// krylov.hip: the right preconditioner P = I + T_C^Q (S - I) T_Q^C, either with the caller's S on
// scatterer s (s >= 0), or (s < 0) with the library's sparsifying S on every scatterer that has one
struct PrecondCb {
  int s = 0;
  ls_grid_op S = nullptr;
  void *user = nullptr;
  double2 *c = nullptr, *sc = nullptr;   // the caller's grid buffers
  int64_t ldc = 0;
};

// apply.hip
hipError_t launch_apply_fp64(const Scat &s, const double *x, double *y, int nrhs, int64_t ld,
                             Mode mode, int source_split, int rhs_chunk, int tpl, void *ws, hipStream_t st,
                             hipEvent_t far_start = nullptr, hipEvent_t far_stop = nullptr);
size_t apply_workspace_bytes(int64_t n, int nrhs, int source_split);
// source splits of the single right-hand-side sum that evaluates each unordered pair once (one per
// block of 256 sources); launch_apply_fp64 takes that kernel for nrhs = 1, one target per lane and
// exactly this many splits
int fp64_sym_splits(int64_t n);
hipError_t launch_epilogue(const Scat &s, const double2 *part, int nsplit, const double2 *f, const double *x,
                           double *y, int nrhs, int64_t ld, Mode mode, hipStream_t st);
// the same for the split-FP16 tiles, whose nsplit partial sums are FP32 ([split][rhs][n] float2,
// each column scaled by colinv[b] here, in FP64); near (may be null) is the FP64 near launch's
// partial [rhs][n], added after them
hipError_t launch_epilogue_h(const Scat &s, const float2 *parth, int nsplit, const double *colinv,
                             const double2 *near, const double2 *f, const double *x, double *y, int nrhs, int64_t ld,
                             Mode mode, hipStream_t st);
// mfma.hip: batched right-hand sides on the matrix cores (single = FP32 tiles)
int tile_ldx(int nrhs);
int tile_mt(int nrhs, bool single);
size_t tile_workspace_bytes(int64_t n, int nrhs, int nsplit);
int tile_source_split(int64_t n, int nrhs, bool single);
hipError_t launch_apply_tile(const Scat &s, const double *x, double *y, int nrhs, int64_t ld, Mode mode, bool single,
                             int nsplit, void *ws, hipStream_t st, hipEvent_t far_start, hipEvent_t far_stop);
// split-FP16 tiles (LS_MIXED with opt.mixed_fp16, one scatterer per launch)
size_t tile_h_workspace_bytes(int64_t n, int nrhs, int nsplit);
hipError_t launch_apply_tile_h(const Scat &s, const double *x, double *y, int nrhs, int64_t ld, Mode mode, int nsplit,
                               void *ws, hipStream_t st, hipEvent_t far_start, hipEvent_t far_stop);
size_t batch_workspace_bytes(const ls_ctx *h, int nrhs, bool single, int split_len);
hipError_t launch_apply_batch(ls_ctx *h, const double *x, double *y, int nrhs, int64_t ld, Mode mode, bool single,
                              int mt, int split_len, void *ws, hipStream_t st, hipEvent_t far_start,
                              hipEvent_t far_stop, bool far_only = false, bool may_alloc = true);
// device tables of the persistent launch for nrhs right-hand sides and every scatterer
hipError_t reserve_batch_tables(ls_ctx *h, int nrhs, bool single, int mt, int split_len);
int batch_default_split_len(const ls_ctx *h, bool single);
hipError_t launch_eval_green(const double *z2, double *g, int64_t n, int single, hipStream_t st);
void eval_green_host(const double *z2, double *g, int64_t n);

// api.hip: with may_grow false the application fails (LS_ERR_ARG) instead of enlarging the
// handle's workspace
ls_status apply_op(ls_ctx *h, const double *x, double *y, int nrhs, int64_t ld, Mode mode, ls_precision p,
                   hipStream_t st, bool may_grow = true);
ls_status setup_fail(ls_ctx *h, ls_status st, const char *msg);
// krylov.hip
ls_status solve_gmres(ls_ctx *h, const double *b, double *x, int nrhs, int64_t ld, const ls_solve_opts &o,
                      ls_solve_info *info, hipStream_t st, const PrecondCb *pc = nullptr);
ls_status grad_contrast(ls_ctx *h, const double *u, const double *lam, const double *a, int nrhs, int64_t ld,
                        double *grad, hipStream_t st);
void free_solve_ws(ls_ctx *h);
// farfield.hip
size_t farfield_workspace_bytes(int64_t n, int R, int nrhs);
hipError_t launch_farfield(const Scat &s, const double *u, int nrhs, int64_t ld, const double *th_dev, int R,
                           const double *data, double *uinf, double *res, void *ws, hipStream_t st);
hipError_t launch_farfield_adjoint(const Scat &s, const double *res, int nrhs, int64_t ld, const double *th_dev,
                                   int R, double *a, double *rhs, hipStream_t st);
hipError_t launch_set_contrast(const Scat &s, const double *m_caller, hipStream_t st);
int auto_source_split(int64_t n, int nrhs, int launches_per_split, int tpl);
// field recovery (setup.hip: geometry and target correction rows; apply.hip: the sums)
ls_status build_geometry(ls_ctx *h, Scat &sc, const ls_scatterer &s, const std::vector<int32_t> &eord);
ls_status field_correction(ls_ctx *h, const Scat &sc, int64_t nt, const double *tx, const double *ty,
                           hipStream_t st, std::vector<int64_t> &rp, std::vector<int32_t> &ci,
                           std::vector<double> &cv);
bool outside_scatterer(const Scat &sc, double x, double y);
const double *geom_x(const Scat &sc);   // host node positions, internal order (nullptr without geometry)
const double *geom_y(const Scat &sc);
int field_source_split(int64_t n, int64_t nt, int nrhs);
// transfer.hip: c = T_Q^C x, and y = x + T_C^Q (sc - c) (y = x outside scatterer s's segment is
// the caller's business); x, y [nrhs][ld] caller order, c, sc [nrhs][ldc]
hipError_t launch_quad_to_cart(const Scat &s, const double2 *x, int64_t ld, double2 *c, int64_t ldc, int nrhs,
                               hipStream_t st);
// sparsify.hip: sc = S c (adjoint: sc = S^H c, or D^-1 S^H D c with dscale; tmp [nrhs][ldt] is then
// needed); c and sc must not alias
hipError_t launch_sparsify(const SparsifyData &sp, const double2 *c, int64_t ldc, double2 *sc, int64_t ldo,
                           double2 *tmp, int64_t ldt, int nrhs, bool adjoint, bool dscale, hipStream_t st);
hipError_t launch_precond_finish(const Scat &s, const double2 *x, int64_t ld, const double2 *c, const double2 *sc,
                                 int64_t ldc, double2 *y, int nrhs, hipStream_t st);
size_t field_workspace_bytes(int64_t n, int nrhs, int64_t nt, int nsplit);
hipError_t launch_field(const Scat &s, const double *u, int nrhs, int64_t ld, int64_t nt, const double *tx,
                        const double *ty, const int64_t *rp, const int32_t *ci, const double2 *cv, int nsplit,
                        double *out, void *ws, hipStream_t st, hipEvent_t far_start = nullptr,
                        hipEvent_t far_stop = nullptr);

}  // namespace lsk
