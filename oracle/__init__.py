"""FP64 CPU reference implementation of the AIM operator, solve and RCS.

TEST INFRASTRUCTURE ONLY. This package is the independent oracle against
which the GPU library is checked. Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the library never does, and
the library shares no code, tables or helpers with it. Inputs come from the
separate ``workloads`` package, which holds no arithmetic of the method.

Everything here is plain NumPy/SciPy in float64/complex128, written for
readability rather than speed. Each module states the passage of the paper
(Wei & Yilmaz, "A Hybrid Parallelization of AIM for Multi-Core Clusters")
or the standard literature it follows. The paper defers the definition of
AIM itself to its references; where it is silent the module names the reading
taken.

Modules
  constants    physical constants and wavenumber
  quadrature   7-point (degree 5) triangle rule
  rwg          RWG basis table from a triangle mesh
  potentials   closed-form 1/R and (r'-r)/R triangle integrals
  mom          EFIE Galerkin moment matrix with singularity extraction
  excitation   plane-wave right-hand side
  aim          grid, stencils, projection, grid Green's function, near zone,
               direct-summation and FFT forms of the AIM product
  gmres        restarted GMRES with right Jacobi preconditioning
  farfield     scattered far field, bistatic RCS, err_theta_theta (eq. 1)
  mie          Mie series for a PEC sphere
"""
