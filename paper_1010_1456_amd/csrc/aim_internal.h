// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/aim.h"

namespace aim {

constexpr double kC0 = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;
constexpr double kEta0 = kMu0 * kC0;

// Status-carrying exception used inside the library; converted to
// aim_status at the ABI.
struct Error : std::runtime_error {
  aim_status status;
  Error(aim_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

void hip_check(hipError_t e, const char *what, const char *file, int line);
#define HIPCHECK(x) ::aim::hip_check((x), #x, __FILE__, __LINE__)
#define LAUNCHCHECK() ::aim::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// ---------------------------------------------------------------------------
// FFT plans: length P factored into stages of supported radices.
constexpr int kMaxStages = 4;
struct FftPlan {
  int P = 0;
  int ns = 0;
  int r[kMaxStages] = {0, 0, 0, 0};
};
bool fft_plan_for(int P, FftPlan *out);  // false if P has no supported factorisation
int fft_length_at_least(int lo);        // smallest supported length >= lo
// true if the projection has a kernel fused with the forward pass of length
// pl.P (all butterflies of 4 lines fit one work-group)
inline bool fft_anterp_fused(const FftPlan &pl) {
  int m = 0;
  for (int s = 0; s < pl.ns; ++s) m = pl.P / pl.r[s] > m ? pl.P / pl.r[s] : m;
  return 4 * m <= 1024;
}

// ---------------------------------------------------------------------------
// Host plan of one mesh (no GPU involved).
struct HostPlan {
  int64_t nv = 0, nt = 0, n = 0, nnz = 0;
  double freq = 0, lam = 0, k = 0, h = 0, r_near = 0;
  int order = 2, K = 27;
  // formulation: the combined field (alpha EFIE + (1 - alpha) eta MFIE) on
  // this mesh, else the EFIE (alpha = 1)
  bool cfie = false;
  double alpha = 1.0;
  std::vector<double> verts;     // nv*3
  std::vector<int32_t> tris;     // nt*3
  std::vector<double> area;      // nt
  // RWG table, per unknown
  std::vector<int32_t> e_lo, e_hi, tp, tm, vp, vm;
  std::vector<double> len;       // edge length
  std::vector<double> centre;    // n*3
  // grid
  int grid[3] = {0, 0, 0};
  int pad[3] = {0, 0, 0};
  double x0[3] = {0, 0, 0};
  std::vector<int32_t> anchor;   // n*3
  // near zone CSR
  std::vector<int64_t> rowptr;   // n+1
  std::vector<int32_t> cols;     // nnz
};

void host_plan_build(const aim_mesh &m, const aim_params &p, HostPlan *hp);

// ---------------------------------------------------------------------------
// Device-side data of one mesh.
template <typename T>
struct vec2_of;
template <>
struct vec2_of<float> {
  using type = float2;
};
template <>
struct vec2_of<double> {
  using type = double2;
};
// interleaved complex value of real type T (float2 / double2)
template <typename T>
using cx = typename vec2_of<T>::type;

// kz run length of the blocked grid between the y passes and the x pass:
// 128 bytes of complex values
template <typename T>
constexpr int kGridBlock = 128 / (int)sizeof(cx<T>);
// fewer padded kz than one such run (a flat scatterer): the grid between the
// passes is kept kz-outer instead, [F][Pz][Nx][Ny] and [F][Pz][Nx][Py]
template <typename T>
constexpr bool thin_layout(int Pz) {
  return Pz < kGridBlock<T>;
}

// streams a multi-mesh product spreads its meshes over
constexpr int kMaxLanes = 4;

struct MeshDev {
  HostPlan hp;
  int64_t offset = 0;
  int lane = 0;  // stream lane of this mesh's product (multi-mesh plans)
  FftPlan plan[3];
  int H[3] = {0, 0, 0};       // octant extents P_d/2 + 1
  // geometry
  double *verts = nullptr;    // nv*3
  int32_t *tris = nullptr;    // nt*3
  double *area = nullptr;     // nt
  int32_t *rwg = nullptr;     // n*4: T+, T-, v+, v-
  double *len = nullptr;      // n
  int32_t *anchor_lin = nullptr;  // n: linear index of the stencil corner
  // operator
  double *lam64 = nullptr;    // n*4*K
  float *lam32 = nullptr;
  int32_t *rowptr = nullptr;  // n+1
  int32_t *cols = nullptr;    // nnz
  double2 *near64 = nullptr;  // nnz
  float2 *near32 = nullptr;
  double2 *zdiag = nullptr;   // n (diag of Z^MOM)
  double2 *ghat64 = nullptr;  // H0*H1*H2
  float2 *ghat32 = nullptr;
  double2 *tw64[3] = {nullptr, nullptr, nullptr};  // twiddles exp(-2 pi i e / P_d)
  float2 *tw32[3] = {nullptr, nullptr, nullptr};
  int32_t *stencil_off = nullptr;  // K linear offsets
  // projection transposed to grid-node order (entries with a non-zero
  // weight only): entries of node v are node_ptr[v] .. node_ptr[v+1]-1, each
  // with its basis index and its 4 weights (x, y, z, div)
  int64_t n_entries = 0;
  int32_t *node_ptr = nullptr;  // V0 + 1
  // the nodes with at least one entry (occupied: on the scatterer's stencils)
  // and their entry ranges, occ_ptr[i] .. occ_ptr[i + 1] - 1
  int64_t n_occ = 0;
  int32_t *occ = nullptr;      // n_occ node indices, increasing
  int32_t *occ_ptr = nullptr;  // n_occ + 1
  // the z lines (x Ny + y) holding an occupied node: the interpolation reads
  // the propagated fields on these lines only, so the inverse z pass skips
  // the others
  int64_t n_occ_lines = 0;
  int32_t *occ_lines = nullptr;
  // per x: the y range [lo, hi) of the occupied z lines (x, y); the y passes
  // read (forward) and write (inverse) only these rows
  int32_t *occ_yrange = nullptr;  // 2 Nx
  // per occupied z line: the z range [lo, hi) of its occupied nodes (the z
  // passes read and write only these elements of the grid side)
  int32_t *occ_zrange = nullptr;  // 4 n_occ_lines: {lo, g0, g1, hi} per occupied line
  int32_t *ent_col = nullptr;   // n_entries
  double *lamT64 = nullptr;     // n_entries * 4
  float *lamT32 = nullptr;      // n_entries * 4
  // tuned variants, per precision [0 = FP64, 1 = FP32]: projection fused with
  // the forward z pass (1) or two launches (0)
  int fuse_proj[2] = {0, 0};
  // z index of the one grid plane holding every projection weight, or -1.
  // Then the sources, and the fields the interpolation weighs, live on that
  // plane only, and the propagation is the 2-D convolution on it with the
  // spectrum of g(x, y, 0): the 3-D spectrum summed over kz (octant H0 x H1)
  int planar_z = -1;
  double2 *ghat2d64 = nullptr;
  float2 *ghat2d32 = nullptr;
  // the projection restricted to that plane (plane node p = x Ny + y):
  // node-ordered entries (ent_col, lamT shared), in-plane stencils of
  // (M+1)^2 weights, plane-linear anchors and stencil offsets
  int32_t *plane_node_ptr = nullptr;  // Nx Ny + 1
  int64_t n_plane_occ = 0;            // occupied plane nodes and their entry ranges
  int32_t *plane_occ = nullptr;
  int32_t *plane_occ_ptr = nullptr;
  double *plane_lam64 = nullptr;      // n * 4 * (M+1)^2
  float *plane_lam32 = nullptr;
  int32_t *plane_anchor = nullptr;    // n
  int32_t *plane_soff = nullptr;      // (M+1)^2
  int plane_K = 0;                    // (M+1)^2
  // occupied nodes per wave of the projection gather, per precision [FP64,
  // FP32]: chosen by timing at set-up among 8, 16, 32
  int gather_npw[2] = {16, 16};
  // field groups of the pipelined y / x / y passes per precision (1: the
  // three passes one after the other), chosen by timing at set-up
  int xy_groups[2] = {1, 1};
  // bytes of consecutive lines per work-group tile (128 or 64) of the x pass
  // and of the strided y passes, per precision; chosen by timing at set-up
  int x_row[2] = {128, 128};
  int y_row[2] = {128, 128};
  double setup_ms[AIM_NSETUP] = {0, 0, 0, 0, 0};  // wall time per set-up phase
  // combined field only: curl weights W[n][e][u] = int (t_n x grad l_u)_e,
  // t_n = f_n x n (the MFIE part is interpolated from the vector potential's
  // grids with them)
  double *curl64 = nullptr;  // n*3*K
  float *curl32 = nullptr;
  // per triangle and local vertex i: (basis << 1 | side) of the basis whose
  // free vertex is vertex i (side 1 on T-), or -1 (far field, RCS)
  int32_t *tri_basis = nullptr;  // nt*3
  // projected source grids per precision [4 nrhs][V0] (the plane's [4 nrhs]
  // [Nx Ny] for a planar scatterer): zero once when allocated, after which the
  // projection writes the occupied nodes only (the same nodes every product)
  void *src[2] = {nullptr, nullptr};
  size_t src_bytes[2] = {0, 0};
  // field layout the source grid was last written in (0 none, 1 the 3-D grid
  // [4 nrhs][V0], 2 the plane [4 nrhs][Nx Ny]): the zero nodes of one layout
  // are not those of the other, so a change of layout clears the buffer
  int src_layout[2] = {0, 0};
  // forward z transforms of those grids per precision [4 nrhs][Nx Ny][Pzs]
  // (kz-blocked grids only): zero once, after which the forward z pass
  // writes the occupied z lines only
  void *fz[2] = {nullptr, nullptr};
  size_t fz_bytes[2] = {0, 0};
};

// milliseconds since an arbitrary epoch (steady clock)
double wall_ms();

struct Plan;

// Device memory through the plan's allocator.
void *dev_alloc(Plan *pl, size_t bytes);
void dev_free(Plan *pl, void *p);

struct Plan {
  int device = 0;  // HIP device the plan was set up on
  aim_allocator alloc{};
  bool own_alloc = true;
  hipStream_t setup_stream = nullptr;
  aim_params params{};
  bool mixed = true;
  int nmesh = 0;
  int64_t n_total = 0;
  std::vector<MeshDev> mesh;
  std::vector<std::pair<void *, size_t>> live;  // allocations (for destroy/info)
  double device_bytes = 0;
  // grid work buffers per lane and precision, grown on demand
  void *work[kMaxLanes][2][3] = {};
  size_t work_bytes[kMaxLanes][2][3] = {};
  // lanes of a multi-mesh product: the meshes are dealt to nlanes streams
  // (lane 0 is the caller's stream, lanes 1.. the plan's own, default
  // priority), each with its own work buffers, so that the members' products
  // overlap; fork / join events order them with the caller's stream
  int nlanes = 1;
  hipStream_t lane_stream[kMaxLanes] = {};
  hipEvent_t lane_fork = nullptr;
  hipEvent_t lane_join[kMaxLanes] = {};
  uint64_t work_gen = 0;  // bumped whenever a grid work buffer moves (invalidates solve graphs)
  // solver buffers, stream and captured graphs, kept across solves (solver.hip)
  struct SolverState *solver = nullptr;
};
// releases the solver state (graphs, stream, buffers) of a plan
void solver_release(Plan *pl);

// set-up kernels (setup_kernels.hip)
void setup_mesh_device(Plan *pl, MeshDev &md, hipStream_t s);
// times the alternative kernel variants of one mesh and keeps the faster
void autotune_mesh(Plan *pl, MeshDev &md, hipStream_t s);

namespace fftk {
struct LineMap;
struct ContigMap;
}

// FFT passes (fft_*.hip); one overload per precision, dispatching on pl.P
#define AIM_DECLARE_FFT(V)                                                                       \
  void fft_pass_contig(const V *in, V *out, const FftPlan &pl, int n_in, int n_out,              \
                       int64_t lines, const fftk::ContigMap &imap, const fftk::ContigMap &omap,  \
                       bool inverse, const V *tw, hipStream_t s);                                \
  void fft_pass_strided(const V *in, V *out, const FftPlan &pl, int n_in, int n_out,             \
                        int64_t outer, int64_t inner, const fftk::LineMap &imap,                 \
                        const fftk::LineMap &omap, bool inverse, const V *tw, int row_bytes,     \
                        hipStream_t s);                                                          \
  void fft_mid_pass(V *data, const FftPlan &pl, int n_x, int nfield, int Py, int Pz, int Hx,     \
                    int Hy, int Hz, const V *ghat, const V *tw, int blk, int64_t fstride,        \
                    int row_bytes, hipStream_t s);
AIM_DECLARE_FFT(float2)
AIM_DECLARE_FFT(double2)
#undef AIM_DECLARE_FFT

// the y, x and y passes of the kz-blocked layout pipelined over G field
// groups in G + 2 launches (fft_xy_*.hip); false if the lengths have no
// pipelined kernel (then nothing is launched)
bool xy_pipeline_available(const FftPlan &plx, const FftPlan &ply);
#define AIM_DECLARE_XY(V)                                                                         \
  void fft_xy_pipeline(const V *gz, V *g2, V *g1, const FftPlan &pl, int Nx, int Ny, int F,       \
                       int G, int Py, int Pz, int Hy, int Hz, const V *ghat, const V *twx,        \
                       const V *twy, int blk, int64_t V2, const fftk::LineMap &m1y,               \
                       const fftk::LineMap &m2, hipStream_t s);
AIM_DECLARE_XY(float2)
AIM_DECLARE_XY(double2)
#undef AIM_DECLARE_XY

// anterpolation fused with the forward z pass (fft_anterp_*.hip): x (c64 or
// c128) -> forward z transforms of the 4 source fields, [4 nrhs][nlines][out_ls]
#define AIM_DECLARE_ANTERP(VX, T, V)                                                             \
  bool anterp_fftz(const VX *x, int64_t ldx, int nrhs, const int32_t *node_ptr,                  \
                   const int32_t *ent_col, const T *lamT, int Nz, int64_t nlines, V *out,        \
                   int64_t out_ls, int64_t out_fstride, const V *tw, const FftPlan &pl,          \
                   hipStream_t s);
AIM_DECLARE_ANTERP(float2, float, float2)
AIM_DECLARE_ANTERP(double2, float, float2)
AIM_DECLARE_ANTERP(double2, double, double2)
#undef AIM_DECLARE_ANTERP

// Where the product left the grid after one of its stages (inspection):
// element (f, a, z) of the plain [F][A][Z] view is p[f fs + a as + z zs]
// (kind 1), or the kz-blocked grid [F][Z/blk][Nx][Py][blk] with fstride
// between fields and A = Nx Py (kind 2); kind 0: no such stage.
struct StageView {
  const void *p = nullptr;
  int kind = 0;
  int64_t F = 0, A = 0, Z = 0, fs = 0, as = 0, zs = 0;
  int Nx = 0, Py = 0, blk = 0;
  int64_t fstride = 0;
};

// matvec (matvec.hip)
// `ev` (optional) receives an event record before the first kernel and after
// each stage: ev[0] .. ev[AIM_NSTAGE]. `full3d` (inspection): the 3-D passes
// also for a scatterer in one grid plane. `views` (optional, AIM_NSTAGE
// entries, index = stage): where the product's own passes left each stage's
// output.
template <typename T, typename TX>
void far_stages(Plan *pl, MeshDev &md, int nrhs, const cx<TX> *x, int64_t ldx, int stop_stage,
                hipStream_t s, hipEvent_t *ev = nullptr, bool full3d = false,
                StageView *views = nullptr);
// copies a stage's output as recorded in `v` to out in the plain [F][A][Z] layout
template <typename T>
void copy_stage_view(const StageView &v, void *out, hipStream_t s);
template <typename T, typename TX, typename TY>
void matvec_mesh(Plan *pl, MeshDev &md, int nrhs, const cx<TX> *x, int64_t ldx, cx<TY> *y,
                 int64_t ldy, hipStream_t s, hipEvent_t *ev = nullptr);
void *work_buffer(Plan *pl, int lane, int prec, int which, size_t bytes, hipStream_t s);
// y = Z x over every mesh of the plan (x, y: [n_total][nrhs], leading
// dimension n_total; c128 for AIM_FP64 and AIM_MIXED_IO64, c64 for
// AIM_MIXED): the meshes' products run on their lanes, forked from and
// joined back to s; with `ev` (one event set of AIM_NSTAGE + 1 per mesh) they
// run one after the other on s instead, each event set recording its stages
// `mesh_on` (optional, one flag per mesh): meshes flagged 0 are skipped (their
// rows of y are left as they are)
void matvec_plan(Plan *pl, aim_precision prec, int nrhs, const void *x, void *y, hipStream_t s,
                 hipEvent_t *ev = nullptr, const std::vector<char> *mesh_on = nullptr);
// deals the meshes to lanes (longest product first to the least loaded lane)
// and creates the lanes' streams and events
void assign_lanes(Plan *pl, const std::vector<double> &cost);
void release_lanes(Plan *pl);
// copies the grid buffer after far stage `stage` to out in plain layout
template <typename T>
void copy_far_stage(Plan *pl, MeshDev &md, int nrhs, int stage, void *out, hipStream_t s);

// excitation / rcs (setup_kernels.hip, rcs.hip)
void excitation_mesh(Plan *pl, MeshDev &md, int nw, const aim_planewave *w, double2 *b, int64_t ldb,
                     hipStream_t s);
void rcs_mesh(Plan *pl, MeshDev &md, int nrhs, const double2 *x, int64_t ldx, int ntheta,
              const double *theta, int nphi, const double *phi, double *sigma, hipStream_t s);
// the triangle -> basis table of the far field (set-up)
void rcs_prepare_mesh(Plan *pl, MeshDev &md, hipStream_t s);
// address of the current device's fixed RCS scratch array, looked up once per
// device (set-up)
void rcs_scratch_init();
// elements (double2) of that array, and the current device's address of it
constexpr int64_t kRcsScratchElems = int64_t(1) << 20;
void *rcs_scratch_ptr(int device);
// the RCS without allocation: device directions and output, partial sums in
// the fixed scratch array (asynchronous)
void rcs_mesh_noalloc(MeshDev &md, int nrhs, const double2 *x, int64_t ldx, int ntheta,
                      const double *theta, int nphi, const double *phi, double *sigma,
                      double2 *part, hipStream_t s);

// solver (solver.hip)
aim_status gmres_solve(Plan *pl, aim_precision prec, int nrhs, const aim_planewave *waves,
                       const aim_solve_opts &o, double2 *x, aim_solve_stats *st, hipStream_t s);

}  // namespace aim
