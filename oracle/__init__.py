"""Oracle: a plain, slow, FP64 CPU implementation of the discretized Lippmann-Schwinger
operator, written from the paper (Sections 2 and 3) for testing only.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.  It
shares no code with the GPU library: it never imports ``paper_2608_17615_amd`` and the
library never imports it.  Inputs (meshes, contrast, incident fields, seeded vectors)
come from ``workloads``, which holds none of the method's arithmetic.

Modules
  bessel    H0, H1 (SciPy AMOS Hankel)                          -- Section 2, G(x,y)
  green     punctured Nystrom far sum (dense or by target rows) -- Section 3, eq. DIM_map
  vdim      exact polynomial potentials and the correction C   -- Section 3, eq. DIM_decomp
  operator  L = I + k^2 (G~W + C) M and its adjoint             -- eqs. linear_system_matrix
  krylov    dense LU and GMRES without restart                  -- Section 6 setup
  mie       Fourier-Bessel series for one- and two-layer disks  -- Section 6.1
  farfield  far-field pattern, misfit and its adjoint gradient  -- Section 5, eq. dissipativity_identity
  field     the field at exterior points                        -- eq. field_recovery
  transfer  grid <-> node transfers and the preconditioner P    -- Section 4, eq. preconditioner_factored
  sparsify  the sparsifying Cartesian preconditioner S^(C)      -- Section 4, eqs. sparsifying_min, LC_def

Every function is pinned by a test in tests/test_oracle_*.py against something other
than itself (closed forms, an addition-theorem evaluation, brute-force quadrature,
Fourier-Bessel series, finite differences).  None is "parity unpinned".
"""
