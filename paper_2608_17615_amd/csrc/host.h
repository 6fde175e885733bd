// Host-only stages of the setup (no HIP calls): the correction rows' element search, exact
// polynomial potentials and interpolation solves, and the sparsifying preconditioner's stencils,
// block LU and host sweeps.  Declared for the library's translation units and for the host
// sanitizer check, which runs them without a GPU.
#pragma once
#include <complex>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace lsk {

// api.hip: element order (by subdomain, then along a Hilbert curve through the centroids)
std::vector<int32_t> element_order(const ls_scatterer &s);

// setup.hip (nodes: the targets are the scatterer's own nodes in internal order, else the
// external points tx, ty).  Er, Ei, S are [nt][nsub][10]; S complex interleaved.
void correction_potentials(const GeomData &g, int threads, int64_t nt, const double *tx, const double *ty,
                           bool nodes, std::vector<int32_t> &tau, std::vector<double> &Er, std::vector<double> &Ei);
void correction_solve(const GeomData &g, int threads, int64_t nt, const std::vector<int32_t> &tau,
                      const std::vector<double> &Er, const std::vector<double> &Ei, const std::vector<double> &S,
                      std::vector<int64_t> &rp, std::vector<int32_t> &ci, std::vector<double> &cv);

// sparsify.hip
void sparsify_stencil(int nx, int ny, double h, double k, const std::complex<double> *m, int threads,
                      std::vector<std::complex<double>> &W, std::vector<std::complex<double>> &E, double *ratio);
bool sparsify_factor(int nx, int ny, const std::vector<std::complex<double>> &E,
                     std::vector<std::vector<std::complex<double>>> &G, int threads);
void sparsify_solve_host(int nx, int ny, const std::vector<std::complex<double>> &E,
                         const std::vector<std::vector<std::complex<double>>> &G, const std::complex<double> *y,
                         std::complex<double> *x);

}  // namespace lsk
