/*
 * aim.h - C ABI of the MI355X adaptive-integral-method (AIM) library.
 *
 * The library solves time-harmonic scattering from perfectly conducting
 * (PEC) surfaces with the EFIE method of moments on RWG basis functions,
 * accelerated by AIM: the paper (Wei & Yilmaz, "A Hybrid Parallelization of
 * AIM for Multi-Core Clusters", Sections 2.1-2.2) benchmarks PEC plates and
 * spheres meshed with triangles at ~lambda/9, lit by an x-polarised plane
 * wave travelling toward -z, and measures the bistatic RCS sigma_theta_theta
 * against a reference through err_theta_theta (its eq. 1). Each iteration of
 * its diagonally preconditioned iterative solve applies the AIM product:
 * projection onto a regular grid, an FFT propagation step on the doubled
 * (zero-padded) grid, interpolation back, and the near-zone correction
 * (Section 4.1 and its footnote on pruning the zero-padded FFTs).
 *
 * Conventions for every entry point:
 *  - Every call returns aim_status; no C++ exception crosses the ABI. On a
 *    non-OK status aim_last_error() returns a message for the calling thread.
 *  - "device" pointers are HIP device allocations on the current device (for
 *    example torch tensors); "host" pointers are ordinary process memory.
 *  - Complex numbers are interleaved (re, im): c64 = 2 x float, c128 =
 *    2 x double. Multi-RHS vectors are column-major [sum_N][nrhs] with
 *    leading dimension sum_N (each right-hand side contiguous).
 *  - hip_stream is a hipStream_t (NULL = the null stream). Calls that say
 *    "asynchronous" only enqueue work on it; the others synchronise it.
 *  - A plan is not thread-safe; distinct plans are independent.
 *  - Units: SI (metres, hertz, square metres); angles in radians.
 *  - Time convention exp(+j w t); G(R) = exp(-j k R) / (4 pi R).
 */
#ifndef AIM_H
#define AIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AIM_OK = 0,
  AIM_ERR_ARG = -1,    /* invalid argument (NULL pointer, size, parameter) */
  AIM_ERR_MESH = -2,   /* invalid mesh: index out of range, degenerate
                          triangle, edge shared by more than two triangles */
  AIM_ERR_HIP = -3,    /* a HIP runtime call or kernel launch failed */
  AIM_ERR_NOMEM = -4,  /* the allocator returned NULL */
  AIM_ERR_NOCONV = -5, /* GMRES reached max_iter before the tolerance */
  AIM_ERR_STATE = -6   /* call not valid for this plan (e.g. FP32 data absent) */
} aim_status;

/* Arithmetic of the AIM product.
 * AIM_FP64:  projection, FFTs, Green's-function multiply, interpolation and
 *            near correction in complex double.
 * AIM_MIXED: the same steps in complex float (operator data rounded from the
 *            FP64 set-up); the solver keeps FP64 Krylov vectors and an FP64
 *            outer residual (iterative refinement). */
typedef enum { AIM_FP64 = 0, AIM_MIXED = 1, AIM_MIXED_IO64 = 2 } aim_precision;
/* AIM_MIXED_IO64: the AIM_MIXED arithmetic on c128 input/output vectors,
 * narrowed and widened in registers (how the solver applies the c64 operator
 * to its FP64 Krylov vectors). Accepted by aim_matvec and aim_matvec_timed. */

/* A PEC triangle surface (paper Section 2.1). Host memory, copied by
 * aim_setup/aim_host_plan; the caller may free it afterwards.
 * verts: nv x 3 doubles (metres); tris: nt x 3 int32 vertex indices (0-based;
 * closed surfaces consistently oriented). freq_hz > 0. */
typedef struct {
  int64_t nv;
  const double *verts;
  int64_t nt;
  const int32_t *tris;
  double freq_hz;
} aim_mesh;

/* AIM parameters (paper Section 2.2 sets the moment-matching order and the
 * near-zone size gamma; grid spacing is chosen empirically there).
 * h_lambda            grid spacing in wavelengths (> 0), e.g. 0.1
 * order               stencil order M in 1..5: (M+1)^3 nodes, moments matched
 *                     up to order M in each coordinate, e.g. 2 (the paper
 *                     matches up to fifth order for its reference solutions,
 *                     Section 2.2); other values give AIM_ERR_ARG
 * near_radius_lambda  near zone: basis pairs whose centres are within this
 *                     distance (wavelengths, >= 0), e.g. 0.3 (= 3 h)
 * fft_min_pad         0: FFT length per dimension = smallest supported
 *                     length >= 2 N_d - 1; otherwise a lower bound on it
 * flags               AIM_FLAG_* below
 * tuning              kernel variants the set-up would otherwise pick by
 *                     timing (for tests and measurements; 0 = pick all):
 *                     bits 0-7  field groups the forward y, x and inverse y
 *                               passes are pipelined over (aim_info.xy_groups):
 *                               0 (pick), 1, 2 or 4;
 *                     bits 8-15 tile rows of the x and strided y passes
 *                               (aim_info.tile_bytes): 0 (pick), 1 (128-byte
 *                               rows), 2 (64-byte rows);
 *                     bits 16-23 right-hand sides per mesh that the set-up
 *                               times the variants with, 0 (= 1) to 64: the
 *                               fastest variant depends on it (the passes
 *                               of many right-hand sides stream grids
 *                               larger than the GPU's last-level cache),
 *                               so a caller that will apply the operator to
 *                               R right-hand sides at a time passes R;
 *                     other values give AIM_ERR_ARG
 * cfie_alpha          with AIM_FLAG_CFIE: the combination parameter alpha in
 *                     [0, 1] of alpha EFIE + (1 - alpha) eta MFIE (the paper
 *                     uses 0.6 for its closed scatterers, Section 2.2);
 *                     ignored otherwise
 * quad_points         points of the triangle quadrature of the projection,
 *                     the near-zone fill, the excitation and the far field:
 *                     7 (the paper's rule, Section 2.2; degree 5) or 0 (the
 *                     same); other values give AIM_ERR_ARG */
typedef struct {
  double h_lambda;
  int32_t order;
  int32_t fft_min_pad;
  double near_radius_lambda;
  int32_t flags;
  int32_t tuning;
  double cfie_alpha;
  int32_t quad_points;
  int32_t reserved;
} aim_params;

#define AIM_FLAG_NO_MIXED 1 /* keep only FP64 operator data (AIM_MIXED -> AIM_ERR_STATE) */
/* Combined-field equation instead of the EFIE (Section 2.2): Galerkin-tested
 * alpha EFIE + (1 - alpha) eta MFIE, with MFIE J/2 - n x PV int grad G x J dS'
 * = n x H_inc and n the outward normal, (v1 - v0) x (v2 - v0) of each
 * triangle. Every mesh must be closed (every edge shared by two triangles)
 * and consistently oriented with positive enclosed volume, else AIM_ERR_MESH;
 * alpha outside [0, 1] gives AIM_ERR_ARG. The product, the solve (its
 * right-hand side V = alpha <f, E_inc> + (1 - alpha) <f, n x (k_hat x E_inc)>)
 * and the Jacobi preconditioner then use the combined operator. */
#define AIM_FLAG_CFIE 2
/* As the paper does for a mixed set of scatterers (Section 2.2: EFIE for the
 * open plate, CFIE for the closed bodies): the combined field with
 * cfie_alpha on every mesh that is closed, consistently oriented and of
 * positive volume, the EFIE on the others (no mesh is refused for it). */
#define AIM_FLAG_CFIE_CLOSED 4

/* Device memory provider. alloc returns device memory of >= bytes (NULL on
 * failure), ordered on `stream`; free releases it. Passing NULL for the
 * allocator uses hipMalloc/hipFree. The allocator must outlive the plan. */
typedef struct {
  void *ctx;
  void *(*alloc)(void *ctx, size_t bytes, void *stream);
  void (*free)(void *ctx, void *p, void *stream);
} aim_allocator;

/* Plane wave arriving from direction r_hat(theta, phi), i.e. travelling along
 * -r_hat, unit amplitude, polarised along theta_hat (pol 0) or phi_hat
 * (pol 1) at (theta, phi). The paper's x-polarised wave toward -z is
 * {0, 0, 0}. */
typedef struct {
  double theta;
  double phi;
  int32_t pol;
  int32_t reserved;
} aim_planewave;

#define AIM_MAX_MESH 16

/* Sizes of a plan (per mesh and totals). bytes_* are the algorithmic HBM
 * bytes of one single-RHS product in each precision: operator data read once,
 * vectors read/written once, grid traffic of the pruned pass structure used
 * (with fused_projection, the projected grid is never stored). */
/* set-up phases timed in aim_info.setup_ms */
#define AIM_NSETUP 5
#define AIM_SETUP_HOST_PLAN 0
#define AIM_SETUP_PROJECTION 1
#define AIM_SETUP_GREEN 2
#define AIM_SETUP_NEAR_FILL 3
#define AIM_SETUP_TUNE 4

typedef struct {
  int32_t nmesh;
  int32_t order;
  int64_t n_total;                      /* sum of unknowns */
  int64_t nnz_total;                    /* near-zone nonzeros */
  int64_t n[AIM_MAX_MESH];              /* unknowns (interior edges) */
  int64_t offset[AIM_MAX_MESH];         /* first row of each mesh */
  int64_t nnz[AIM_MAX_MESH];
  int32_t grid[AIM_MAX_MESH][3];        /* N_x, N_y, N_z */
  int32_t pad[AIM_MAX_MESH][3];         /* FFT lengths P_x, P_y, P_z */
  double h[AIM_MAX_MESH];               /* grid spacing, metres */
  double x0[AIM_MAX_MESH][3];           /* coordinate of grid node 0 */
  double k[AIM_MAX_MESH];               /* wavenumber, 1/m */
  double bytes_fp64[AIM_MAX_MESH];
  double bytes_mixed[AIM_MAX_MESH];
  int32_t fused_projection[AIM_MAX_MESH][2]; /* [mesh][0 FP64, 1 mixed]: 1 if the projection
                                               runs inside the forward z pass (chosen by
                                               timing at set-up) */
  int32_t planar_z[AIM_MAX_MESH];       /* z index of the one grid plane that holds every
                                           projection weight (a flat scatterer lying in a
                                           grid plane), else -1; the propagation then runs
                                           on that plane alone with the 2-D spectrum */
  double device_bytes;                  /* device memory held by the plan */
  double setup_ms[AIM_MAX_MESH][AIM_NSETUP]; /* wall time of each set-up phase, ms: host plan
                                               (mesh checks, RWG table, grid, anchors, near-zone
                                               pattern), projection weights, Green's spectrum,
                                               near-zone fill (FP64 quadrature of Z^MOM - Z^grid),
                                               variant tuning (paper Section 2.4, Fig. 4, times
                                               the matrix fill) */
  double cfie_alpha[AIM_MAX_MESH];      /* combined-field parameter of each mesh, or -1 where
                                           the mesh uses the EFIE */
  int64_t occ_nodes[AIM_MAX_MESH];      /* grid nodes with a non-zero projection weight (the
                                           only nodes the projection writes and the
                                           interpolation reads; plane nodes for planar_z >= 0) */
  int64_t occ_lines[AIM_MAX_MESH];      /* z lines (x, y) holding such a node (the only lines
                                           the z passes transform) */
  int32_t gather_npw[AIM_MAX_MESH][2];  /* [mesh][0 FP64, 1 mixed]: occupied nodes per wave of
                                           the projection gather (chosen by timing at set-up) */
  int32_t xy_groups[AIM_MAX_MESH][2];   /* [mesh][0 FP64, 1 mixed]: field groups over which the
                                           forward y, x and inverse y passes run pipelined, the
                                           x pass of one group beside the y passes of others in
                                           one launch (1: one pass after the other; chosen by
                                           timing at set-up) */
  int32_t tile_bytes[AIM_MAX_MESH][2][2]; /* [mesh][0 FP64, 1 mixed][0 x pass, 1 strided y
                                           passes]: bytes of consecutive grid lines (128 or 64)
                                           in one work-group's tile (chosen by timing at
                                           set-up) */
} aim_info;

/* GMRES options. restart m (<= 200), relative-residual tolerance on
 * ||b - A x|| / ||b|| (evaluated with the FP64 operator), iteration cap
 * (inner iterations summed over restarts and refinement steps). */
typedef struct {
  double tol;
  int32_t restart;
  int32_t max_iter;
  int32_t warm_start; /* 1: x_io holds the initial guess */
  int32_t flags;      /* AIM_SOLVE_* below */
} aim_solve_opts;

/* The Arnoldi steps between two convergence polls (8 iterations) are
 * captured once into a HIP graph and replayed on later restart cycles and
 * later solves of the same shape (right-hand sides, restart); results are
 * bitwise those of direct launches. This flag launches every kernel
 * directly instead. */
#define AIM_SOLVE_NO_GRAPH 1

/* Results of aim_gmres_solve for one system (one mesh lit by one wave).
 * Every system of a call advances in lock-step through shared batched
 * products, so the product counts and the time are those of the whole call;
 * the iterations, residual and convergence are the system's own. */
typedef struct {
  int32_t iterations;      /* inner GMRES iterations this system took part in
                              (summed over restarts and refinement steps) */
  int32_t converged;       /* 1 if this system's FP64 residual met tol */
  int32_t matvec_low;      /* batched products in the requested precision */
  int32_t matvec_fp64;     /* batched FP64 residual products */
  double residual;         /* this system's final ||b - A64 x|| / ||b|| */
  double seconds;          /* wall time of the whole solve call */
} aim_solve_stats;

typedef struct aim_plan aim_plan;
typedef struct aim_host_plan aim_host_plan;

/* ---- set-up ------------------------------------------------------------ */

/* Builds the operator for nmesh (1..AIM_MAX_MESH) scatterers: host planning
 * (mesh validation, RWG table, grid, stencil anchors, near-zone pattern),
 * then on the GPU the projection weights, the spectrum of the grid Green's
 * function, and the FP64 near-zone matrix Z^MOM - Z^grid with singularity
 * extraction on touching triangle pairs; finally it times the alternative
 * kernel variants of each mesh and keeps the faster (results do not depend
 * on the choice beyond rounding). Unknowns of mesh i occupy rows
 * offset[i] .. offset[i]+n[i]-1. Synchronises hip_stream. On failure *out is
 * NULL and nothing leaks. */
aim_status aim_setup(const aim_mesh *meshes, int32_t nmesh, const aim_params *p,
                     const aim_allocator *alloc, void *hip_stream, aim_plan **out);

aim_status aim_plan_info(const aim_plan *plan, aim_info *out);

/* Frees all device memory of the plan through its allocator. NULL-safe. */
void aim_destroy(aim_plan *plan);

/* ---- hot path ---------------------------------------------------------- */

/* y = Z^AIM x for nrhs right-hand sides (asynchronous). x, y: device,
 * column-major [n_total][nrhs]; c128 for AIM_FP64, c64 for AIM_MIXED.
 * x and y must not overlap. */
aim_status aim_matvec(aim_plan *plan, aim_precision prec, int32_t nrhs,
                      const void *x, void *y, void *hip_stream);

/* Runs nrep products y = Z^AIM x back to back on hip_stream with HIP events
 * between the kernels of every product, then synchronises. x, y as for
 * aim_matvec (c128 for AIM_FP64 and AIM_MIXED_IO64, c64 for AIM_MIXED).
 * stage_ms (host, AIM_NSTAGE doubles, may be NULL) receives the summed event
 * time of each step over all repetitions and meshes:
 *   0 projection (grid clear + anterpolation), 1 forward z pass,
 *   2 forward y pass, 3 x pass with the Green's spectrum multiply,
 *   4 inverse y pass, 5 inverse z pass, 6 interpolation + near correction;
 * total_ms (host, may be NULL) the event time from the first to the last
 * kernel. */
#define AIM_NSTAGE 7
aim_status aim_matvec_timed(aim_plan *plan, aim_precision prec, int32_t nrhs, const void *x,
                            void *y, int32_t nrep, double *stage_ms, double *total_ms,
                            void *hip_stream);

/* Measures the product as a HIP graph: runs one product directly (so that
 * every work buffer exists), captures nrep products y = Z^AIM x back to back
 * into one graph, launches it once untimed, then nlaunch times with HIP
 * events around each launch, and synchronises. launch_ms (host, nlaunch
 * doubles) receives each launch's event time for all nrep products. x, y as
 * for aim_matvec_timed. */
aim_status aim_matvec_graph_timed(aim_plan *plan, aim_precision prec, int32_t nrhs,
                                  const void *x, void *y, int32_t nrep, int32_t nlaunch,
                                  double *launch_ms, void *hip_stream);

/* Solves Z^AIM x = b for nrhs_per_mesh plane waves on every mesh of the plan
 * (waves: host, nrhs_per_mesh entries, the same set for every mesh) with
 * restarted GMRES, right Jacobi preconditioning D = diag(Z^MOM), FP64
 * (classical Gram-Schmidt, twice) Arnoldi and, for AIM_MIXED, an FP64 outer
 * refinement loop r = b - A64 x around inner solves with the c64 operator
 * (at most 20 refinement steps; an inner solve ends at its target or where
 * the c64 operator's rounding stops its true residual from falling).
 * x_io: device c128 [n_total][nrhs_per_mesh]. stats: host
 * [nmesh][nrhs_per_mesh] (entry mesh * nrhs_per_mesh + wave) or NULL.
 * Synchronises.
 * Returns AIM_ERR_NOCONV if some right-hand side missed tol (x_io then holds
 * the last iterate). A zero right-hand side gives x = 0. */
aim_status aim_gmres_solve(aim_plan *plan, aim_precision prec, int32_t nrhs_per_mesh,
                           const aim_planewave *waves, const aim_solve_opts *opts,
                           void *x_io, aim_solve_stats *stats, void *hip_stream);

/* Plane-wave right-hand sides V_m = <f_m, E_inc> in FP64 (asynchronous).
 * b: device c128 [n_total][nwaves]. */
aim_status aim_excitation(aim_plan *plan, int32_t nwaves, const aim_planewave *waves,
                          void *b, void *hip_stream);

/* Bistatic sigma_theta_theta (m^2) of the currents x (device c128
 * [n_total][nrhs]) on the grid theta[ntheta] x phi[nphi] (host, radians), in
 * FP64: sigma = (k eta)^2 / (4 pi) |theta_hat . N|^2 with
 * N = sum_n I_n int f_n exp(+j k r_hat . r') dS'. sigma_tt: host
 * [nmesh][nrhs][ntheta][nphi]. Synchronises. */
aim_status aim_rcs(aim_plan *plan, int32_t nrhs, const void *x, int32_t ntheta,
                   const double *theta, int32_t nphi, const double *phi,
                   double *sigma_tt, void *hip_stream);

/* aim_rcs without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid it): the same sigma_theta_theta, with theta, phi and sigma_tt in
 * device memory (theta[ntheta], phi[nphi] radians; sigma_tt [nmesh][nrhs]
 * [ntheta][nphi], m^2) and x as for aim_rcs; asynchronous on hip_stream, on
 * the plan's device (else AIM_ERR_ARG). Each quadrature point's current is
 * formed inside the kernel, and the partial sums over point chunks live in a
 * fixed array of 1,048,576 complex doubles (16 MiB) that the library holds on
 * each GPU it runs on until the process ends: ntheta * nphi * nrhs above
 * that gives AIM_ERR_ARG. Every call on a GPU shares that GPU's array (each
 * call writes every partial it reads, so nothing needs clearing), so calls
 * that overlap in time on one GPU, on different streams or threads, race;
 * calls ordered on one stream do not. */
aim_status aim_rcs_noalloc(aim_plan *plan, int32_t nrhs, const void *x, int32_t ntheta,
                           const double *theta, int32_t nphi, const double *phi,
                           double *sigma_tt, void *hip_stream);

/* ---- host-only planning (no GPU needed) -------------------------------- */

/* Runs only the host phase of aim_setup for one mesh: validation, RWG table,
 * grid plan, anchors, near-zone CSR pattern. */
aim_status aim_host_plan_build(const aim_mesh *mesh, const aim_params *p, aim_host_plan **out);

/* Copies the host plan out (any pointer may be NULL to skip it).
 * rwg:      [n][6] int32: edge vertex lo, hi, T+, T-, free vertex of T+, of T-
 * anchors:  [n][3] int32 lowest stencil corner per dimension
 * rowptr:   [n+1] int64, cols: [nnz] int32 (columns ascending per row)
 * grid:     [3] int32 nodes, pad: [3] int32 FFT lengths, x0h: [4] double
 *           (x0, y0, z0, h). */
aim_status aim_host_plan_export(const aim_host_plan *hp, int64_t *n, int64_t *nnz,
                                int32_t *rwg, int32_t *anchors, int64_t *rowptr,
                                int32_t *cols, int32_t *grid, int32_t *pad, double *x0h);

void aim_host_plan_destroy(aim_host_plan *hp);

/* ---- inspection (tests) ------------------------------------------------ */

/* Copies internal operator data of mesh `mesh` to host memory (synchronises):
 *  AIM_DATA_LAMBDA64  [n][4][(M+1)^3] double  projection weights (q = x,y,z,div)
 *  AIM_DATA_NEAR64    [nnz] c128              Z^near values (CSR order)
 *  AIM_DATA_ZDIAG64   [n] c128                diag of Z^MOM
 *  AIM_DATA_GHAT64    [Hx][Hy][Hz] c128       Green's spectrum octant,
 *                     H_d = P_d/2 + 1, scaled by 1/(P_x P_y P_z)
 *  AIM_DATA_CURL64    [n][3][(M+1)^3] double  curl weights of the combined
 *                     field (AIM_FLAG_CFIE plans only): int (t_n x grad l_u)_e
 *                     with t_n = f_n x n
 * `bytes` must equal the size of the item. */
#define AIM_DATA_LAMBDA64 1
#define AIM_DATA_NEAR64 2
#define AIM_DATA_ZDIAG64 3
#define AIM_DATA_GHAT64 4
#define AIM_DATA_CURL64 5
aim_status aim_export(const aim_plan *plan, int32_t mesh, int32_t what, void *host_dst,
                      size_t bytes);

/* Runs only the far (grid) part of the product for one precision, stopping
 * after `stage` (asynchronous): 1 = projection (grids [4 nrhs][Nx][Ny][Nz]),
 * 2 = forward z pass, 3 = forward y pass, 4 = Green's multiply pass,
 * 5 = inverse y pass, 6 = inverse z pass, and copies the resulting grid
 * buffer (device, same precision as x) to `grid_out` (device, sized for the
 * stage: [4 nrhs] x {NxNyNz, NxNyPz, NxPyPz, NxPyPz, NxNyPz, NxNyNz}). */
aim_status aim_debug_far_stage(aim_plan *plan, aim_precision prec, int32_t mesh, int32_t nrhs,
                               const void *x, int32_t stage, void *grid_out, void *hip_stream);

/* Runs the product's own far passes for one precision (the pruned and, for
 * a scatterer in one grid plane, in-plane passes that aim_matvec launches;
 * asynchronous) and copies the grid left after `stage` to grid_out (device,
 * same precision as x) in the plain layout [4 nrhs][A][Z]:
 *   3-D path:   1 (A, Z) = (Nx Ny, Nz), 2 and 5 (Nx Ny, Pz), 3 and 4 (Nx Py, Pz),
 *               6 (Nx Ny, Nz);
 *   plane path: 1 and 6 (Nx, Ny), 3 and 4 (Nx, Py) (aim_info.planar_z >= 0; it
 *               has no z passes, so stages 2 and 5 give AIM_ERR_ARG).
 * The product computes only what its next step reads, so only these elements
 * are defined: stages 1-4 all; stage 5 the rows y inside each plane x's range
 * of occupied z lines (3-D path); stage 6 the occupied z lines over their
 * occupied z range (3-D path), every element (plane path). A z line (x, y)
 * is occupied when it holds a node with a non-zero projection (or curl)
 * weight, and its occupied range runs from its first to its last such node.
 * Stages 1-3 stop after that stage; stages 4-6 run the whole far part. */
aim_status aim_debug_product_stage(aim_plan *plan, aim_precision prec, int32_t mesh,
                                   int32_t nrhs, const void *x, int32_t stage, void *grid_out,
                                   void *hip_stream);

const char *aim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AIM_H */
