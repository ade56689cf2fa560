// C ABI entry points (include/aim.h): argument checks, plan lifetime,
// per-mesh dispatch and error translation.
#include <chrono>
#include <cstring>
#include <memory>

#include "aim_internal.h"

namespace aim {

static thread_local std::string g_last_error;

void hip_check(hipError_t e, const char *what, const char *file, int line) {
  if (e != hipSuccess)
    throw Error(AIM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e) + " (" + file + ":" +
                                 std::to_string(line) + ")");
}

double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

void *dev_alloc(Plan *pl, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void *p = nullptr;
  if (pl->own_alloc) {
    if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  } else {
    p = pl->alloc.alloc(pl->alloc.ctx, bytes, (void *)pl->setup_stream);
  }
  if (!p) throw Error(AIM_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  pl->live.emplace_back(p, bytes);
  pl->device_bytes += (double)bytes;
  return p;
}

void dev_free(Plan *pl, void *p) {
  if (!p) return;
  // The buffer may still be read by kernels on any stream the library used
  // (the caller's or the solver's), while the allocator may hand it out again
  // at once on the stream it was obtained on: finish all work first. Frees
  // happen on growth, at the end of a solve or RCS call and at destroy only.
  HIPCHECK(hipDeviceSynchronize());
  for (size_t i = 0; i < pl->live.size(); ++i)
    if (pl->live[i].first == p) {
      pl->device_bytes -= (double)pl->live[i].second;
      pl->live.erase(pl->live.begin() + i);
      break;
    }
  if (pl->own_alloc)
    (void)hipFree(p);
  else
    pl->alloc.free(pl->alloc.ctx, p, (void *)pl->setup_stream);
}

static void free_all(Plan *pl) {
  if (!pl) return;
  (void)hipDeviceSynchronize();  // no kernel may still read what is freed
  for (auto &a : pl->live) {
    if (pl->own_alloc)
      (void)hipFree(a.first);
    else
      pl->alloc.free(pl->alloc.ctx, a.first, (void *)pl->setup_stream);
  }
  pl->live.clear();
}

static aim_status fail(aim_status s, const std::string &m) {
  g_last_error = m;
  return s;
}

template <class F>
static aim_status guarded(F &&f) {
  try {
    f();
    return AIM_OK;
  } catch (const Error &e) {
    return fail(e.status, e.what());
  } catch (const std::bad_alloc &) {
    return fail(AIM_ERR_NOMEM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(AIM_ERR_ARG, e.what());
  }
}

// algorithmic bytes of one single-RHS product (see the design notes): vectors
// read twice and written once, projection read twice, near CSR read once,
// spectrum octant once, grid traffic of the pruned passes.
static double model_bytes(const MeshDev &md, int sc, int sr) {
  const HostPlan &h = md.hp;
  const double n = (double)h.n, K = (double)h.K, nnz = (double)h.nnz;
  const double Nx = h.grid[0], Ny = h.grid[1], Nz = h.grid[2];
  const double Py = h.pad[1], Pz = h.pad[2];
  const double vec = 3.0 * n * sc;
  const double lam = 2.0 * n * (4.0 * K * sr + 4.0);
  const double nearb = nnz * (sc + 4.0) + 4.0 * (n + 1.0);
  const double ghat = (double)md.H[0] * md.H[1] * md.H[2] * sc;
  const double V0 = Nx * Ny * Nz, V1 = Nx * Ny * Pz, V2 = Nx * Py * Pz;
  // per field: [projection write V0; z read V0] + z write V1; y: V1 + V2; x: 2 V2;
  // inverse y: V2 + V1; inverse z: V1 + V0; interpolation read V0
  if (md.planar_z >= 0) {  // all on the scatterer's plane: per field projection Nx Ny, y
                           // passes 2 (Nx Ny + Nx Py), x 2 Nx Py, interpolation Nx Ny;
                           // in-plane stencils; the 2-D spectrum
    const double K2 = (double)md.plane_K;
    const double lam2 = 2.0 * n * (4.0 * K2 * sr + 4.0);
    const double grid = 4.0 * sc * (4.0 * Nx * Ny + 4.0 * Nx * Py);
    return vec + lam2 + nearb + (double)md.H[0] * md.H[1] * sc + grid;
  }
  const double v0_terms = md.fuse_proj[sc == 16 ? 0 : 1] ? 2.0 : 4.0;
  const double grid = 4.0 * sc * (v0_terms * V0 + 4.0 * V1 + 4.0 * V2);
  const double curl = md.curl64 ? 3.0 * n * K * sr : 0.0;  // combined field: interpolation only
  return vec + lam + curl + nearb + ghat + grid;
}

}  // namespace aim

using namespace aim;

struct aim_plan : Plan {};
struct aim_host_plan : HostPlan {};

extern "C" {

const char *aim_last_error(void) { return g_last_error.c_str(); }

aim_status aim_host_plan_build(const aim_mesh *mesh, const aim_params *p, aim_host_plan **out) {
  if (!out) return fail(AIM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!mesh || !p) return fail(AIM_ERR_ARG, "NULL mesh or params");
  std::unique_ptr<aim_host_plan> hp(new aim_host_plan());
  aim_status st = guarded([&] { host_plan_build(*mesh, *p, hp.get()); });
  if (st == AIM_OK) *out = hp.release();
  return st;
}

aim_status aim_host_plan_export(const aim_host_plan *hp, int64_t *n, int64_t *nnz, int32_t *rwg,
                                int32_t *anchors, int64_t *rowptr, int32_t *cols, int32_t *grid,
                                int32_t *pad, double *x0h) {
  if (!hp) return fail(AIM_ERR_ARG, "NULL host plan");
  if (n) *n = hp->n;
  if (nnz) *nnz = hp->nnz;
  if (rwg)
    for (int64_t i = 0; i < hp->n; ++i) {
      rwg[6 * i] = hp->e_lo[i];
      rwg[6 * i + 1] = hp->e_hi[i];
      rwg[6 * i + 2] = hp->tp[i];
      rwg[6 * i + 3] = hp->tm[i];
      rwg[6 * i + 4] = hp->vp[i];
      rwg[6 * i + 5] = hp->vm[i];
    }
  if (anchors) std::memcpy(anchors, hp->anchor.data(), sizeof(int32_t) * hp->anchor.size());
  if (rowptr) std::memcpy(rowptr, hp->rowptr.data(), sizeof(int64_t) * hp->rowptr.size());
  if (cols) std::memcpy(cols, hp->cols.data(), sizeof(int32_t) * hp->cols.size());
  if (grid)
    for (int c = 0; c < 3; ++c) grid[c] = hp->grid[c];
  if (pad)
    for (int c = 0; c < 3; ++c) pad[c] = hp->pad[c];
  if (x0h) {
    for (int c = 0; c < 3; ++c) x0h[c] = hp->x0[c];
    x0h[3] = hp->h;
  }
  return AIM_OK;
}

void aim_host_plan_destroy(aim_host_plan *hp) { delete hp; }

aim_status aim_setup(const aim_mesh *meshes, int32_t nmesh, const aim_params *p,
                     const aim_allocator *alloc, void *hip_stream, aim_plan **out) {
  if (!out) return fail(AIM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!meshes || !p) return fail(AIM_ERR_ARG, "NULL meshes or params");
  if (nmesh < 1 || nmesh > AIM_MAX_MESH) return fail(AIM_ERR_ARG, "nmesh out of range");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(AIM_ERR_ARG, "incomplete allocator");
  {
    const int g = p->tuning & 0xff, t = (p->tuning >> 8) & 0xff, r = (p->tuning >> 16) & 0xff;
    if ((p->tuning >> 24) != 0 || (g != 0 && g != 1 && g != 2 && g != 4) || t > 2 || r > 64)
      return fail(AIM_ERR_ARG,
                  "tuning: pipeline groups 0, 1, 2 or 4; tile rows 0, 1 or 2; right-hand sides "
                  "0 to 64");
  }
  std::unique_ptr<aim_plan> pl(new aim_plan());
  if (alloc) {
    pl->alloc = *alloc;
    pl->own_alloc = false;
  }
  pl->setup_stream = (hipStream_t)hip_stream;
  pl->params = *p;
  pl->mixed = !(p->flags & AIM_FLAG_NO_MIXED);
  pl->nmesh = nmesh;
  pl->mesh.resize(nmesh);
  aim_status st = guarded([&] {
    HIPCHECK(hipGetDevice(&pl->device));
    rcs_scratch_init();  // the device address of the allocation-free RCS's fixed array
    int64_t off = 0;
    for (int i = 0; i < nmesh; ++i) {
      const double t0 = wall_ms();
      host_plan_build(meshes[i], *p, &pl->mesh[i].hp);
      pl->mesh[i].setup_ms[AIM_SETUP_HOST_PLAN] = wall_ms() - t0;
      pl->mesh[i].offset = off;
      off += pl->mesh[i].hp.n;
    }
    pl->n_total = off;
    if (off > INT32_MAX) throw Error(AIM_ERR_ARG, "too many unknowns");
    for (int i = 0; i < nmesh; ++i) setup_mesh_device(pl.get(), pl->mesh[i], pl->setup_stream);
    std::vector<double> cost(nmesh);
    for (int i = 0; i < nmesh; ++i) cost[i] = model_bytes(pl->mesh[i], 8, 4);
    assign_lanes(pl.get(), cost);
    for (int i = 0; i < nmesh; ++i) {
      const double t0 = wall_ms();
      autotune_mesh(pl.get(), pl->mesh[i], pl->setup_stream);
      HIPCHECK(hipStreamSynchronize(pl->setup_stream));
      pl->mesh[i].setup_ms[AIM_SETUP_TUNE] = wall_ms() - t0;
    }
    HIPCHECK(hipStreamSynchronize(pl->setup_stream));
  });
  if (st != AIM_OK) {
    release_lanes(pl.get());
    free_all(pl.get());
    return st;
  }
  *out = pl.release();
  return AIM_OK;
}

aim_status aim_plan_info(const aim_plan *plan, aim_info *out) {
  if (!plan || !out) return fail(AIM_ERR_ARG, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->nmesh = plan->nmesh;
  out->order = plan->params.order;
  out->n_total = plan->n_total;
  for (int i = 0; i < plan->nmesh; ++i) {
    const MeshDev &md = plan->mesh[i];
    out->n[i] = md.hp.n;
    out->offset[i] = md.offset;
    out->nnz[i] = md.hp.nnz;
    out->nnz_total += md.hp.nnz;
    for (int c = 0; c < 3; ++c) {
      out->grid[i][c] = md.hp.grid[c];
      out->pad[i][c] = md.hp.pad[c];
      out->x0[i][c] = md.hp.x0[c];
    }
    out->h[i] = md.hp.h;
    out->k[i] = md.hp.k;
    out->bytes_fp64[i] = model_bytes(md, 16, 8);
    out->bytes_mixed[i] = model_bytes(md, 8, 4);
    out->fused_projection[i][0] = md.fuse_proj[0];
    out->fused_projection[i][1] = md.fuse_proj[1];
    out->planar_z[i] = md.planar_z;
    out->cfie_alpha[i] = md.hp.cfie ? md.hp.alpha : -1.0;
    out->occ_nodes[i] = md.planar_z >= 0 ? md.n_plane_occ : md.n_occ;
    out->occ_lines[i] = md.n_occ_lines;
    out->gather_npw[i][0] = md.gather_npw[0];
    out->gather_npw[i][1] = md.gather_npw[1];
    out->xy_groups[i][0] = md.xy_groups[0];
    out->xy_groups[i][1] = md.xy_groups[1];
    for (int q = 0; q < 2; ++q) {
      out->tile_bytes[i][q][0] = md.x_row[q];
      out->tile_bytes[i][q][1] = md.y_row[q];
    }
    for (int j = 0; j < AIM_NSETUP; ++j) out->setup_ms[i][j] = md.setup_ms[j];
  }
  out->device_bytes = plan->device_bytes;
  return AIM_OK;
}

void aim_destroy(aim_plan *plan) {
  if (!plan) return;
  solver_release(plan);
  release_lanes(plan);
  free_all(plan);
  delete plan;
}

static aim_status matvec_check(aim_plan *plan, aim_precision prec, int32_t nrhs, const void *x,
                               void *y) {
  if (!plan || !x || !y) return fail(AIM_ERR_ARG, "NULL argument");
  if (nrhs < 1) return fail(AIM_ERR_ARG, "nrhs must be >= 1");
  if (prec != AIM_FP64 && prec != AIM_MIXED && prec != AIM_MIXED_IO64)
    return fail(AIM_ERR_ARG, "bad precision");
  if (prec != AIM_FP64 && !plan->mixed) return fail(AIM_ERR_STATE, "plan has no FP32 data");
  return AIM_OK;
}

static void matvec_all(aim_plan *plan, aim_precision prec, int32_t nrhs, const void *x, void *y,
                       hipStream_t s) {
  matvec_plan(plan, prec, nrhs, x, y, s);
}

aim_status aim_matvec(aim_plan *plan, aim_precision prec, int32_t nrhs, const void *x, void *y,
                      void *hip_stream) {
  aim_status st = matvec_check(plan, prec, nrhs, x, y);
  if (st != AIM_OK) return st;
  return guarded([&] { matvec_all(plan, prec, nrhs, x, y, (hipStream_t)hip_stream); });
}

aim_status aim_matvec_timed(aim_plan *plan, aim_precision prec, int32_t nrhs, const void *x,
                            void *y, int32_t nrep, double *stage_ms, double *total_ms,
                            void *hip_stream) {
  aim_status st = matvec_check(plan, prec, nrhs, x, y);
  if (st != AIM_OK) return st;
  if (nrep < 1) return fail(AIM_ERR_ARG, "nrep must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  // one event set per (repetition, mesh) so that no event is re-recorded
  // before it has been read
  const int nm = plan->nmesh;
  std::vector<hipEvent_t> ev((size_t)nrep * nm * (AIM_NSTAGE + 1), nullptr);
  aim_status r = guarded([&] {
    for (auto &e : ev) HIPCHECK(hipEventCreate(&e));
    for (int rep = 0; rep < nrep; ++rep)
      matvec_plan(plan, prec, nrhs, x, y, s, &ev[(size_t)rep * nm * (AIM_NSTAGE + 1)]);
    HIPCHECK(hipStreamSynchronize(s));
    double acc[AIM_NSTAGE] = {0};
    for (size_t g = 0; g < (size_t)nrep * nm; ++g)
      for (int i = 0; i < AIM_NSTAGE; ++i) {
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, ev[g * (AIM_NSTAGE + 1) + i], ev[g * (AIM_NSTAGE + 1) + i + 1]));
        acc[i] += ms;
      }
    if (stage_ms)
      for (int i = 0; i < AIM_NSTAGE; ++i) stage_ms[i] = acc[i];
    if (total_ms) {
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, ev.front(), ev.back()));
      *total_ms = ms;
    }
  });
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
  return r;
}

aim_status aim_matvec_graph_timed(aim_plan *plan, aim_precision prec, int32_t nrhs, const void *x,
                                  void *y, int32_t nrep, int32_t nlaunch, double *launch_ms,
                                  void *hip_stream) {
  aim_status st = matvec_check(plan, prec, nrhs, x, y);
  if (st != AIM_OK) return st;
  if (nrep < 1 || nlaunch < 1 || !launch_ms) return fail(AIM_ERR_ARG, "bad repetition arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  hipStream_t cs = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  aim_status r = guarded([&] {
    // one direct product first: work buffers exist before the capture
    matvec_all(plan, prec, nrhs, x, y, s);
    HIPCHECK(hipStreamSynchronize(s));
    HIPCHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    HIPCHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      for (int i = 0; i < nrep; ++i) matvec_all(plan, prec, nrhs, x, y, cs);
    } catch (...) {
      (void)hipStreamEndCapture(cs, &g);
      throw;
    }
    HIPCHECK(hipStreamEndCapture(cs, &g));
    HIPCHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    HIPCHECK(hipGraphLaunch(ex, cs));  // first launch uploads the graph (untimed)
    HIPCHECK(hipStreamSynchronize(cs));
    for (int l = 0; l < nlaunch; ++l) {
      HIPCHECK(hipEventRecord(e0, cs));
      HIPCHECK(hipGraphLaunch(ex, cs));
      HIPCHECK(hipEventRecord(e1, cs));
      HIPCHECK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
      launch_ms[l] = ms;
    }
  });
  if (ex) (void)hipGraphExecDestroy(ex);
  if (g) (void)hipGraphDestroy(g);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (cs) {
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
  }
  return r;
}

aim_status aim_excitation(aim_plan *plan, int32_t nwaves, const aim_planewave *waves, void *b,
                          void *hip_stream) {
  if (!plan || !waves || !b || nwaves < 1) return fail(AIM_ERR_ARG, "bad argument");
  hipStream_t s = (hipStream_t)hip_stream;
  return guarded([&] {
    for (auto &md : plan->mesh)
      excitation_mesh(plan, md, nwaves, waves, (double2 *)b + md.offset, plan->n_total, s);
  });
}

aim_status aim_gmres_solve(aim_plan *plan, aim_precision prec, int32_t nrhs_per_mesh,
                           const aim_planewave *waves, const aim_solve_opts *opts, void *x_io,
                           aim_solve_stats *stats, void *hip_stream) {
  if (!plan || !waves || !opts || !x_io || nrhs_per_mesh < 1) return fail(AIM_ERR_ARG, "bad argument");
  if (!(opts->tol > 0) || opts->restart < 1 || opts->restart > 200 || opts->max_iter < 1)
    return fail(AIM_ERR_ARG, "bad solver options");
  if (prec == AIM_MIXED && !plan->mixed) return fail(AIM_ERR_STATE, "plan has no FP32 data");
  aim_status result = AIM_OK;
  aim_status st = guarded([&] {
    result = gmres_solve(plan, prec, nrhs_per_mesh, waves, *opts, (double2 *)x_io, stats,
                         (hipStream_t)hip_stream);
  });
  if (st != AIM_OK) return st;
  if (result == AIM_ERR_NOCONV) g_last_error = "GMRES did not reach the tolerance";
  return result;
}

aim_status aim_rcs(aim_plan *plan, int32_t nrhs, const void *x, int32_t ntheta, const double *theta,
                   int32_t nphi, const double *phi, double *sigma_tt, void *hip_stream) {
  if (!plan || !x || !theta || !phi || !sigma_tt || nrhs < 1 || ntheta < 1 || nphi < 1)
    return fail(AIM_ERR_ARG, "bad argument");
  return guarded([&] {
    const int64_t per = (int64_t)nrhs * ntheta * nphi;
    for (int i = 0; i < plan->nmesh; ++i) {
      MeshDev &md = plan->mesh[i];
      rcs_mesh(plan, md, nrhs, (const double2 *)x + md.offset, plan->n_total, ntheta, theta, nphi,
               phi, sigma_tt + i * per, (hipStream_t)hip_stream);
    }
  });
}

aim_status aim_rcs_noalloc(aim_plan *plan, int32_t nrhs, const void *x, int32_t ntheta,
                           const double *theta, int32_t nphi, const double *phi, double *sigma_tt,
                           void *hip_stream) {
  if (!plan || !x || !theta || !phi || !sigma_tt || nrhs < 1 || ntheta < 1 || nphi < 1)
    return fail(AIM_ERR_ARG, "bad argument");
  return guarded([&] {
    int dev = -1;
    HIPCHECK(hipGetDevice(&dev));
    if (dev != plan->device)
      throw Error(AIM_ERR_ARG, "aim_rcs_noalloc: the plan's device is not the current device");
    double2 *part = (double2 *)rcs_scratch_ptr(plan->device);
    if (!part) throw Error(AIM_ERR_STATE, "aim_rcs_noalloc: scratch address not initialised");
    const int64_t per = (int64_t)nrhs * ntheta * nphi;
    for (int i = 0; i < plan->nmesh; ++i) {
      MeshDev &md = plan->mesh[i];
      rcs_mesh_noalloc(md, nrhs, (const double2 *)x + md.offset, plan->n_total, ntheta, theta,
                       nphi, phi, sigma_tt + i * per, part, (hipStream_t)hip_stream);
    }
  });
}

aim_status aim_export(const aim_plan *plan, int32_t mesh, int32_t what, void *host_dst,
                      size_t bytes) {
  if (!plan || !host_dst || mesh < 0 || mesh >= plan->nmesh) return fail(AIM_ERR_ARG, "bad argument");
  const MeshDev &md = plan->mesh[mesh];
  const void *src = nullptr;
  size_t need = 0;
  switch (what) {
    case AIM_DATA_LAMBDA64:
      src = md.lam64;
      need = sizeof(double) * md.hp.n * 4 * md.hp.K;
      break;
    case AIM_DATA_NEAR64:
      src = md.near64;
      need = sizeof(double2) * md.hp.nnz;
      break;
    case AIM_DATA_ZDIAG64:
      src = md.zdiag;
      need = sizeof(double2) * md.hp.n;
      break;
    case AIM_DATA_GHAT64:
      src = md.ghat64;
      need = sizeof(double2) * md.H[0] * md.H[1] * md.H[2];
      break;
    case AIM_DATA_CURL64:
      if (!md.curl64) return fail(AIM_ERR_STATE, "the plan has no curl weights (not a CFIE plan)");
      src = md.curl64;
      need = sizeof(double) * md.hp.n * 3 * md.hp.K;
      break;
    default:
      return fail(AIM_ERR_ARG, "unknown export item");
  }
  if (bytes != need) return fail(AIM_ERR_ARG, "export size mismatch: need " + std::to_string(need));
  return guarded([&] {
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipMemcpy(host_dst, src, need, hipMemcpyDeviceToHost));
  });
}

aim_status aim_debug_far_stage(aim_plan *plan, aim_precision prec, int32_t mesh, int32_t nrhs,
                               const void *x, int32_t stage, void *grid_out, void *hip_stream) {
  if (!plan || !x || !grid_out || mesh < 0 || mesh >= plan->nmesh || nrhs < 1 || stage < 1 ||
      stage > 6)
    return fail(AIM_ERR_ARG, "bad argument");
  if (prec != AIM_FP64 && prec != AIM_MIXED) return fail(AIM_ERR_ARG, "bad precision");
  if (prec == AIM_MIXED && !plan->mixed) return fail(AIM_ERR_STATE, "plan has no FP32 data");
  hipStream_t s = (hipStream_t)hip_stream;
  return guarded([&] {
    MeshDev &md = plan->mesh[mesh];
    if (prec == AIM_FP64) {
      far_stages<double, double>(plan, md, nrhs, (const double2 *)x + md.offset, plan->n_total,
                                 stage, s, nullptr, true);
      copy_far_stage<double>(plan, md, nrhs, stage, grid_out, s);
    } else {
      far_stages<float, float>(plan, md, nrhs, (const float2 *)x + md.offset, plan->n_total, stage,
                               s, nullptr, true);
      copy_far_stage<float>(plan, md, nrhs, stage, grid_out, s);
    }
  });
}

aim_status aim_debug_product_stage(aim_plan *plan, aim_precision prec, int32_t mesh, int32_t nrhs,
                                   const void *x, int32_t stage, void *grid_out,
                                   void *hip_stream) {
  if (!plan || !x || !grid_out || mesh < 0 || mesh >= plan->nmesh || nrhs < 1 || stage < 1 ||
      stage > 6)
    return fail(AIM_ERR_ARG, "bad argument");
  if (prec != AIM_FP64 && prec != AIM_MIXED) return fail(AIM_ERR_ARG, "bad precision");
  if (prec == AIM_MIXED && !plan->mixed) return fail(AIM_ERR_STATE, "plan has no FP32 data");
  hipStream_t s = (hipStream_t)hip_stream;
  return guarded([&] {
    MeshDev &md = plan->mesh[mesh];
    // stages 1-3 stop there (the x pass overwrites stage 3's grid in place);
    // stages 4-6 run the product's whole far part, whose later passes leave
    // those grids in place
    const int stop = stage <= 3 ? stage : 6;
    StageView v[AIM_NSTAGE];
    if (prec == AIM_FP64) {
      far_stages<double, double>(plan, md, nrhs, (const double2 *)x + md.offset, plan->n_total,
                                 stop, s, nullptr, false, v);
      copy_stage_view<double>(v[stage], grid_out, s);
    } else {
      far_stages<float, float>(plan, md, nrhs, (const float2 *)x + md.offset, plan->n_total, stop,
                               s, nullptr, false, v);
      copy_stage_view<float>(v[stage], grid_out, s);
    }
  });
}

}  // extern "C"
