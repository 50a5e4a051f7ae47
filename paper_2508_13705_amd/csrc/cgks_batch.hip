// Batched execution: many independent grids of one dimension and precision
// advance together, one launch per phase of the step (Sec. 2.2) for the whole
// batch.  Every launch is a persistent grid of a fixed size that walks a
// device-resident job table: item k of a phase maps to (job, tile) through a
// per-phase prefix sum of the jobs' tile counts, and the tile is computed by
// the same device body the single-grid kernels use (cgks_internal.hpp), with
// the job's own tile coordinates and tile count.  A job therefore takes the
// same arithmetic, the same speed partials and the same time steps alone or
// in a batch.
//
// The launch grid and every kernel argument are fixed for the life of the
// batch (the table is read from device memory), so a hipGraph captured once
// stays valid while jobs are added and retired: cgks_batch_commit uploads the
// table outside the graph, the step itself does no copies and no memsets.
#define CGKS_UNIT batched
#include "cgks_internal.hpp"

#include <algorithm>
#include <chrono>

#include "cgks_batch.hpp"

namespace {

__global__ __launch_bounds__(256) void kb_dt(const BTab* tab) {
  const int n = tab->njobs;
  for (int j = blockIdx.x; j < n; j += gridDim.x) {
    const BJob J = tab->jobs[j];
    dt_block(J.B.hdr, J.B.part, J.sbc, J.dt_fixed, J.cfl, J.t_end, J.h, J.C.mu, J.viscous, J.max_steps,
             tab->stat + J.slot);
  }
}

// Strength commit and ghost faces (both directions), then ghost cells of W^n
// (ST: slope storage type of the batch's precision).
template <typename ST>
__global__ __launch_bounds__(256) void kb_prep(const BTab* tab, int remap) {
  for_items<true, true>(tab, PH_PREP, remap, [&](const BJob& J, int k) {
    if (!J.B.hdr->active) return;
    if (k < J.nsx) {
      bc_sigma_at(J.g, J.B.bct, bc_time(J.B.hdr, 1), 0, J.B.sxn, J.B.sxo, J.B.syn, J.B.syo,
                  (k % J.ax) * 256 + threadIdx.x, k / J.ax);
      return;
    }
    k -= J.nsx;
    if (k < J.nsy) {
      bc_sigma_at(J.g, J.B.bct, bc_time(J.B.hdr, 1), 1, J.B.sxn, J.B.sxo, J.B.syn, J.B.syo,
                  (k % J.ay) * 256 + threadIdx.x, k / J.ay);
      return;
    }
    k -= J.nsy;
    int I, Jr;
    GhostItems(J.g).at(J.g, k, I, Jr);
    bc_state_at<ST>(J.g, J.B.bct, bc_time(J.B.hdr, 1), J.B.U, I, Jr);
  });
}

// Ghost cells of the stage state W*.
template <typename ST>
__global__ __launch_bounds__(256) void kb_bcs(const BTab* tab, int remap) {
  for_items<true, true>(tab, PH_BCS, remap, [&](const BJob& J, int k) {
    if (!J.B.hdr->active) return;
    int I, Jr;
    GhostItems(J.g).at(J.g, k, I, Jr);
    bc_state_at<ST>(J.g, J.B.bct, bc_time(J.B.hdr, 2), J.B.S, I, Jr);
  });
}


// Kernel slots of the persistent launches (grid sizes are per slot).
enum Kern { K_DT = 0, K_PREP, K_BCS, K_LINES, K_FACE, K_S1D, NK };

}  // namespace

struct cgks_batch {
  int dim = 0, precision = 0, cap = 0;
  size_t budget = 0, used = 0;
  int ncu = 0;
  int occ[NK] = {};          // resident blocks per CU of each kernel slot (current shapes)
  int occ_face[kFaceTiles] = {}, occ_lines[kLineTiles] = {};   // per tile shape
  cgks_batch_tuning tune{};  // persistent-grid multiplier and XCD remap in use
  int grid[NK] = {};
  std::vector<BJob> slots;
  std::vector<char> busy, fresh;
  std::vector<size_t> bytes;
  std::vector<JobStat> init_stat;
  std::vector<int> order;    // table order -> slot
  // device: one allocation holding the table header, jobs, prefix sums and progress records
  void* dmem = nullptr;
  BTab* dtab = nullptr;
  BJob* djobs = nullptr;
  int* dpre = nullptr;
  JobStat* dstat = nullptr;
  JobStat* hstat = nullptr;  // pinned host copy of the progress records (cgks_batch_poll)
  size_t off_stat = 0, table_bytes = 0;
  std::vector<unsigned char> staging;
  S1Item* dimap = nullptr;    // device item map of a 1-D batch (BTab::imap)
  size_t icap = 0;            // its capacity in items
  std::vector<S1Item> himap;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_steps = 0;
  bool committed = false;
};

namespace {

void set_grids(cgks_batch* b) {
  b->occ[K_FACE] = b->occ_face[b->tune.face_tile];
  b->occ[K_LINES] = b->occ_lines[b->tune.line_tile];
  for (int k = 0; k < NK; ++k) {
    int g = b->ncu * std::max(1, b->occ[k]) * std::max(1, b->tune.grid_mult);
    b->grid[k] = (g + 7) & ~7;   // a multiple of 8 (one share per XCD)
  }
  b->grid[K_DT] = std::min(b->grid[K_DT], std::max(8, b->cap));
}

// Dynamic LDS limit of the batched face kernels and the scratch check of
// every batched kernel (none may use scratch).
template <int DIR, int STAGE, typename T, int M, int V>
cgks_status prepare_bface() {
  const void* f = (const void*)kb_face<DIR, STAGE, T, M, V>;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kb_face_lds<DIR, STAGE, T, M, V>());
  if (e != hipSuccess) return fail(CGKS_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  return check_private(f, 0, "batched face kernel");
}

template <typename T, int M, int V>
cgks_status prepare_bfaces() {
  cgks_status s;
  if ((s = prepare_bface<0, 1, T, M, V>()) != CGKS_OK) return s;
  if ((s = prepare_bface<1, 1, T, M, V>()) != CGKS_OK) return s;
  if ((s = prepare_bface<0, 2, T, M, V>()) != CGKS_OK) return s;
  return prepare_bface<1, 2, T, M, V>();
}

template <typename T, int V>
cgks_status prepare_bshape() {
  cgks_status s;
  if ((s = prepare_bfaces<T, 2, V>()) != CGKS_OK) return s;
  if ((s = prepare_bfaces<T, 3, V>()) != CGKS_OK) return s;
  return prepare_bfaces<T, 4, V>();
}

template <typename T>
cgks_status prepare_batch() {
  cgks_status s;
  if constexpr (sizeof(T) == 4) {
    if ((s = cgks_bf32::prepare()) != CGKS_OK) return s;
  } else {
    if ((s = prepare_bshape<T, 0>()) != CGKS_OK) return s;
    if ((s = prepare_bshape<T, 1>()) != CGKS_OK) return s;
    if ((s = prepare_bshape<T, 2>()) != CGKS_OK) return s;
  }
  const void* k[] = {(const void*)kb_dt, (const void*)kb_prep<T>, (const void*)kb_bcs<T>};
  for (const void* f : k)
    if ((s = check_private(f, 0, "batched kernel")) != CGKS_OK) return s;
  if constexpr (sizeof(T) == 8) {   // FP32: checked by cgks_bf32::prepare
    const void* k2[] = {(const void*)kb_lines<0, T>, (const void*)kb_lines<1, T>, (const void*)kb_stage1d<1, T>,
                        (const void*)kb_stage1d<2, T>};
    for (const void* f : k2)
      if ((s = check_private(f, 0, "batched kernel")) != CGKS_OK) return s;
  }
  return CGKS_OK;
}

template <typename T>
hipError_t occupancy(cgks_batch* b) {
  hipError_t e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->occ[K_DT], kb_dt, 256, 0))) return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->occ[K_PREP], kb_prep<T>, 256, 0))) return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->occ[K_BCS], kb_bcs<T>, 256, 0))) return e;
  if constexpr (sizeof(T) == 4) {
    return cgks_bf32::occupancy(b->occ_face, b->occ_lines, &b->occ[K_S1D]);
  } else {
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->occ_lines[0], kb_lines<0, T>, 256, 0))) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->occ_lines[1], kb_lines<1, T>, 256, 0))) return e;
    // the face grid serves every order: size it by the order that fits the
    // fewest blocks (the largest LDS tile)
    auto face_occ = [&](const void* f2, size_t l2, const void* f3, size_t l3, const void* f4, size_t l4, int* out) {
      int a = 0, c = 0, d = 0;
      hipError_t r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, f2, 256, l2);
      if (r == hipSuccess) r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, f3, 256, l3);
      if (r == hipSuccess) r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&d, f4, 256, l4);
      *out = std::min(a, std::min(c, d));
      return r;
    };
    if ((e = face_occ((const void*)kb_face<1, 2, T, 2, 0>, Lds<2, T, 0>::total, (const void*)kb_face<1, 2, T, 3, 0>,
                      Lds<3, T, 0>::total, (const void*)kb_face<1, 2, T, 4, 0>, Lds<4, T, 0>::total, &b->occ_face[0])))
      return e;
    if ((e = face_occ((const void*)kb_face<1, 2, T, 2, 1>, Lds<2, T, 1>::total, (const void*)kb_face<1, 2, T, 3, 1>,
                      Lds<3, T, 1>::total, (const void*)kb_face<1, 2, T, 4, 1>, Lds<4, T, 1>::total, &b->occ_face[1])))
      return e;
    if ((e = face_occ((const void*)kb_face<1, 2, T, 2, 2>, Lds<2, T, 2>::total, (const void*)kb_face<1, 2, T, 3, 2>,
                      Lds<3, T, 2>::total, (const void*)kb_face<1, 2, T, 4, 2>, Lds<4, T, 2>::total, &b->occ_face[2])))
      return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->occ[K_S1D], kb_stage1d<2, T>, 256, 0);
  }
}

// The face kernels of one direction, stage and tile shape, one launch per order.
template <int DIR, int STAGE, typename T, int V>
void launch_faces_v(int gf, hipStream_t st, const BTab* t, int r) {
  constexpr size_t l2 = Lds<2, T, V>::total, l3 = Lds<3, T, V>::total, l4 = Lds<4, T, V>::total;
  hipLaunchKernelGGL((kb_face<DIR, STAGE, T, 2, V>), dim3(gf), dim3(256), l2, st, t, r);
  hipLaunchKernelGGL((kb_face<DIR, STAGE, T, 3, V>), dim3(gf), dim3(256), l3, st, t, r);
  hipLaunchKernelGGL((kb_face<DIR, STAGE, T, 4, V>), dim3(gf), dim3(256), l4, st, t, r);
}

// FP32: each kernel's own persistent grid (its waves per SIMD differ by
// direction, stage and order), from the CU count and the grid multiplier
template <int DIR, int STAGE, typename T>
void launch_faces(const cgks_batch* b, int v, int gf, hipStream_t st, const BTab* t, int r) {
  if constexpr (sizeof(T) == 4) {
    cgks_bf32::launch_faces(DIR, STAGE, v, b->ncu, std::max(1, b->tune.grid_mult), st, t, r);
  } else {
    switch (v) {
      case 1: launch_faces_v<DIR, STAGE, T, 1>(gf, st, t, r); break;
      case 2: launch_faces_v<DIR, STAGE, T, 2>(gf, st, t, r); break;
      default: launch_faces_v<DIR, STAGE, T, 0>(gf, st, t, r); break;
    }
  }
}

template <typename T>
void launch_lines(int lw, int gl, hipStream_t st, const BTab* t, int stage, int r) {
  if constexpr (sizeof(T) == 4) {
    cgks_bf32::launch_lines(lw, gl, st, t, stage, r);
  } else {
    if (lw == 1) hipLaunchKernelGGL((kb_lines<1, T>), dim3(gl), dim3(256), 0, st, t, stage, r);
    else hipLaunchKernelGGL((kb_lines<0, T>), dim3(gl), dim3(256), 0, st, t, stage, r);
  }
}

template <typename T>
void launch_stage1d(int stage, int gs, hipStream_t st, const BTab* t, int r) {
  if constexpr (sizeof(T) == 4) {
    cgks_bf32::launch_stage1d(stage, gs, st, t, r);
  } else {
    if (stage == 1) hipLaunchKernelGGL((kb_stage1d<1, T>), dim3(gs), dim3(256), 0, st, t, r);
    else hipLaunchKernelGGL((kb_stage1d<2, T>), dim3(gs), dim3(256), 0, st, t, r);
  }
}

template <typename T>
hipError_t enqueue_batch_step(const cgks_batch* b, hipStream_t st) {
  const BTab* t = b->dtab;
  const int r = b->tune.xcd_remap ? 1 : 0;
  hipLaunchKernelGGL(kb_dt, dim3(b->grid[K_DT]), dim3(256), 0, st, t);
  hipLaunchKernelGGL(kb_prep<T>, dim3(b->grid[K_PREP]), dim3(256), 0, st, t, r);
  if (b->dim == 1) {
    launch_stage1d<T>(1, b->grid[K_S1D], st, t, r);
    hipLaunchKernelGGL(kb_bcs<T>, dim3(b->grid[K_BCS]), dim3(256), 0, st, t, r);
    launch_stage1d<T>(2, b->grid[K_S1D], st, t, r);
    return hipGetLastError();
  }
  const int gf = b->grid[K_FACE], gl = b->grid[K_LINES];
  const int v = b->tune.face_tile, lw = b->tune.line_tile;
  // every order is launched (a phase without jobs of that order ends at
  // once), so a captured step serves any later mix of orders
  launch_lines<T>(lw, gl, st, t, 1, r);
  launch_faces<0, 1, T>(b, v, gf, st, t, r);
  launch_faces<1, 1, T>(b, v, gf, st, t, r);
  hipLaunchKernelGGL(kb_bcs<T>, dim3(b->grid[K_BCS]), dim3(256), 0, st, t, r);
  launch_lines<T>(lw, gl, st, t, 2, r);
  launch_faces<0, 2, T>(b, v, gf, st, t, r);
  launch_faces<1, 2, T>(b, v, gf, st, t, r);
  return hipGetLastError();
}

hipError_t enqueue_steps(const cgks_batch* b, int n, hipStream_t st) {
  for (int k = 0; k < n; ++k) {
    hipError_t e = b->precision == CGKS_FP64 ? enqueue_batch_step<double>(b, st) : enqueue_batch_step<float>(b, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void drop_graph(cgks_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->graph_steps = 0;
}

// Tile counts of one job for every phase, for the batch's tile shapes.
void fill_counts(BJob& J, int face_tile, int line_tile) {
  const Geo& g = J.g;
  J.ax = (g.NX + 1 + 255) / 256;
  J.nsx = J.ax * g.NY;
  J.ay = g.dim == 2 ? (g.NY + 1 + 255) / 256 : 0;
  J.nsy = g.dim == 2 ? J.ay * g.NX : 0;
  J.ns = GhostItems(g).count(g);
  J.ltx = (g.NX + line_tile_x(line_tile) - 1) / line_tile_x(line_tile);
  J.lty = (g.NY + line_tile_y(line_tile) - 1) / line_tile_y(line_tile);
  if (g.dim == 2) {
    const int NF = tile_nf(face_tile), NT = tile_nt(face_tile, J.M);
    J.fnb[0][0] = face_tiles_n(g.nx, NF);
    J.fnb[0][1] = face_tiles_t(g.ny, NT);
    J.fnb[1][0] = face_tiles_n(g.ny, NF);
    J.fnb[1][1] = face_tiles_t(g.nx, NT);
    J.nseg = 0;
  } else {
    J.fnb[0][0] = J.fnb[0][1] = J.fnb[1][0] = J.fnb[1][1] = 0;
    J.nseg = (g.nx + S1_CELLS - 1) / S1_CELLS;
  }
}

long long items(const BJob& J, int ph) {
  switch (ph) {
    case PH_DT: return 1;
    case PH_PREP: return (long long)J.nsx + J.nsy + J.ns;
    case PH_BCS: return J.ns;
    case PH_LINES: return J.g.dim == 2 ? (long long)J.ltx * J.lty : 0;
    case PH_FX2: case PH_FX3: case PH_FX4:
      return J.M == 2 + (ph - PH_FX2) ? (long long)J.fnb[0][0] * J.fnb[0][1] : 0;
    case PH_FY2: case PH_FY3: case PH_FY4:
      return J.M == 2 + (ph - PH_FY2) ? (long long)J.fnb[1][0] * J.fnb[1][1] : 0;
    case PH_S1D: return J.nseg;
  }
  return 0;
}

}  // namespace

extern "C" {

cgks_status cgks_batch_create(int dim, int precision, int max_jobs, size_t hbm_budget_bytes, cgks_batch** out) {
  if (!out) return fail(CGKS_EINVAL, "NULL argument");
  *out = nullptr;
  if (dim != 1 && dim != 2) return fail(CGKS_EINVAL, "dim must be 1 or 2");
  if (precision != CGKS_FP64 && precision != CGKS_FP32_FLUX) return fail(CGKS_EINVAL, "unknown precision");
  if (max_jobs < 1 || max_jobs > (1 << 20)) return fail(CGKS_EINVAL, "max_jobs must lie in [1, 2^20]");
  cgks_batch* b = new (std::nothrow) cgks_batch;
  if (!b) return fail(CGKS_ENOMEM, "batch allocation");
  b->dim = dim;
  b->precision = precision;
  b->cap = max_jobs;
  b->budget = hbm_budget_bytes;
  b->tune.grid_mult = 1;
  b->tune.xcd_remap = 1;
  try {
    b->slots.resize(max_jobs);
    b->busy.assign(max_jobs, 0);
    b->fresh.assign(max_jobs, 0);
    b->bytes.assign(max_jobs, 0);
    b->init_stat.resize(max_jobs);
  } catch (...) {
    delete b;
    return fail(CGKS_ENOMEM, "batch host tables");
  }
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_jobs = up(sizeof(BTab));
  const size_t o_pre = o_jobs + up(sizeof(BJob) * max_jobs);
  b->off_stat = o_pre + up(sizeof(int) * NPH * (size_t)(max_jobs + 1));
  b->table_bytes = b->off_stat;
  const size_t total = b->off_stat + up(sizeof(JobStat) * max_jobs);
  hipError_t e = hipMalloc(&b->dmem, total);
  if (e == hipSuccess) e = hipMemset(b->dmem, 0, total);
  int dev = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) {
    // kernel attributes (dynamic LDS, scratch check) before the occupancy query
    const cgks_status ps = precision == CGKS_FP64 ? prepare_batch<double>() : prepare_batch<float>();
    if (ps != CGKS_OK) {
      hipFree(b->dmem);
      delete b;
      return ps;
    }
    e = precision == CGKS_FP64 ? occupancy<double>(b) : occupancy<float>(b);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->hstat, sizeof(JobStat) * max_jobs, hipHostMallocDefault);
  if (e != hipSuccess) {
    if (b->cap_stream) hipStreamDestroy(b->cap_stream);
    if (b->dmem) hipFree(b->dmem);
    delete b;
    return fail(CGKS_EHIP, std::string("batch create: ") + hipGetErrorString(e));
  }
  unsigned char* base = (unsigned char*)b->dmem;
  b->dtab = (BTab*)base;
  b->djobs = (BJob*)(base + o_jobs);
  b->dpre = (int*)(base + o_pre);
  b->dstat = (JobStat*)(base + b->off_stat);
  try {
    b->staging.assign(b->table_bytes, 0);
  } catch (...) {
    hipHostFree(b->hstat);
    hipStreamDestroy(b->cap_stream);
    hipFree(b->dmem);
    delete b;
    return fail(CGKS_ENOMEM, "batch staging");
  }
  set_grids(b);
  *out = b;
  return CGKS_OK;
}

cgks_status cgks_batch_destroy(cgks_batch* b) {
  if (!b) return CGKS_OK;
  drop_graph(b);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  if (b->hstat) hipHostFree(b->hstat);
  if (b->dmem) hipFree(b->dmem);
  if (b->dimap) hipFree(b->dimap);
  delete b;
  return CGKS_OK;
}

cgks_status cgks_batch_add(cgks_batch* b, const cgks_plan* p, void* d_state, void* d_work, long long max_steps,
                           double dt, double cfl, double t_end, int* slot) {
  if (!b || !p || !d_state || !d_work || !slot) return fail(CGKS_EINVAL, "NULL argument");
  *slot = -1;
  if (p->g.dim != b->dim) return fail(CGKS_EINVAL, "plan dimension differs from the batch");
  if (p->precision != b->precision) return fail(CGKS_EINVAL, "plan precision differs from the batch");
  if (p->C.prandtl != 1.0) return fail(CGKS_EINVAL, "batched kernels take Prandtl number 1 only");
  if (!(dt > 0.0) && !(cfl > 0.0 && cfl <= 1.0)) return fail(CGKS_EINVAL, "cfl must lie in (0, 1]");
  if (max_steps < 0) return fail(CGKS_EINVAL, "max_steps must be >= 0");
  if (max_steps == 0 && !(t_end > 0.0)) return fail(CGKS_EINVAL, "a batched job needs max_steps or t_end");
  const size_t need = (p->state_words + p->work_words) * sizeof(double);
  if (b->budget && b->used + need > b->budget) return fail(CGKS_EBUDGET, "job does not fit the HBM budget");
  int s = -1;
  for (int k = 0; k < b->cap; ++k)
    if (!b->busy[k]) { s = k; break; }
  if (s < 0) return fail(CGKS_EBUDGET, "no free job slot");
  Bufs B = bufs(p, d_state, d_work);
  Header hh;
  HIP_TRY(hipMemcpy(&hh, B.hdr, sizeof(hh), hipMemcpyDeviceToHost));
  if (hh.magic != kMagic) return fail(CGKS_ESTATE, "work buffer was not initialised by cgks_init_state");
  BJob& J = b->slots[s];
  memset(&J, 0, sizeof(J));
  J.g = p->g;
  J.C = p->C;
  J.B = B;
  J.dt_fixed = dt;
  J.cfl = cfl;
  J.t_end = t_end;
  J.h = p->g.dim == 2 ? fmin(p->dx, p->dy) : p->dx;
  J.sbc = p->bct.smax;
  J.max_steps = max_steps;
  J.viscous = p->C.tau_model == CGKS_TAU_VISCOUS ? 1 : 0;
  J.M = p->g.m;
  J.slot = s;
  fill_counts(J, b->tune.face_tile, b->tune.line_tile);
  JobStat& is = b->init_stat[s];
  is.t = hh.t;
  is.dt = hh.dt;
  is.steps = (long long)hh.steps;
  is.status = hh.nonphysical ? 2 : 0;
  is.active = 1;
  b->busy[s] = 1;
  b->fresh[s] = 1;
  b->bytes[s] = need;
  b->used += need;
  b->committed = false;
  *slot = s;
  return CGKS_OK;
}

cgks_status cgks_batch_remove(cgks_batch* b, int slot) {
  if (!b) return fail(CGKS_EINVAL, "NULL batch");
  if (slot < 0 || slot >= b->cap || !b->busy[slot]) return fail(CGKS_EINVAL, "no job in that slot");
  b->busy[slot] = 0;
  b->fresh[slot] = 0;
  b->used -= b->bytes[slot];
  b->bytes[slot] = 0;
  b->committed = false;
  return CGKS_OK;
}

cgks_status cgks_batch_commit(cgks_batch* b, void* stream) {
  if (!b) return fail(CGKS_EINVAL, "NULL batch");
  hipStream_t st = (hipStream_t)stream;
  // table order: slot order (the persistent loop strides over all items)
  b->order.clear();
  for (int k = 0; k < b->cap; ++k)
    if (b->busy[k]) b->order.push_back(k);
  const int n = (int)b->order.size();
  unsigned char* base = b->staging.data();
  BTab* T = (BTab*)base;
  memset(T, 0, sizeof(BTab));
  const size_t o_jobs = (unsigned char*)b->djobs - (unsigned char*)b->dmem;
  const size_t o_pre = (unsigned char*)b->dpre - (unsigned char*)b->dmem;
  BJob* jobs = (BJob*)(base + o_jobs);
  int* pre = (int*)(base + o_pre);
  T->njobs = n;
  T->cap = b->cap;
  T->jobs = b->djobs;
  T->pre = b->dpre;
  T->stat = b->dstat;
  for (int ph = 0; ph < NPH; ++ph) {
    int* P = pre + (size_t)ph * (b->cap + 1);
    long long acc = 0;
    for (int k = 0; k < n; ++k) {
      P[k] = (int)acc;
      acc += items(b->slots[b->order[k]], ph);
    }
    P[n] = (int)acc;
    if (acc >= (1ll << 31)) return fail(CGKS_EINVAL, "batch too large for 32-bit item indices");
    T->total[ph] = (int)acc;
  }
  for (int k = 0; k < n; ++k) jobs[k] = b->slots[b->order[k]];
  // 1-D: the (job, index) of every item of the item phases, in the device
  // map (grown when the batch outgrows it; the graph reads the map's address
  // from the table, so it stays valid)
  T->imap = nullptr;
  if (b->dim == 1) {
    const int phs[] = {PH_PREP, PH_BCS, PH_S1D};
    size_t tot = 0;
    for (int ph : phs) {
      T->ioff[ph] = (int)tot;
      tot += (size_t)T->total[ph];
    }
    if (tot >= (1ull << 31)) return fail(CGKS_EINVAL, "batch too large for 32-bit item indices");
    if (tot > b->icap) {
      const size_t cap = tot + tot / 4 + 1024;
      HIP_TRY(hipStreamSynchronize(st));   // no launch in flight reads the old map
      if (b->dimap) HIP_TRY(hipFree(b->dimap));
      b->dimap = nullptr;
      b->icap = 0;
      HIP_TRY(hipMalloc((void**)&b->dimap, cap * sizeof(S1Item)));
      b->icap = cap;
    }
    try {
      b->himap.resize(tot);
    } catch (...) {
      return fail(CGKS_ENOMEM, "batch item map");
    }
    for (int ph : phs) {
      const int* P = pre + (size_t)ph * (b->cap + 1);
      S1Item* M = b->himap.data() + T->ioff[ph];
      for (int k = 0; k < n; ++k)
        for (int q = P[k]; q < P[k + 1]; ++q) M[q] = S1Item{k, q - P[k]};
    }
    if (tot) HIP_TRY(hipMemcpyAsync(b->dimap, b->himap.data(), tot * sizeof(S1Item), hipMemcpyHostToDevice, st));
    T->imap = b->dimap;
  }
  // the host staging buffer is reused by the next commit: copy and wait
  HIP_TRY(hipMemcpyAsync(b->dmem, base, sizeof(BTab), hipMemcpyHostToDevice, st));
  if (n) HIP_TRY(hipMemcpyAsync(b->djobs, jobs, sizeof(BJob) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(b->dpre, pre, sizeof(int) * NPH * (size_t)(b->cap + 1), hipMemcpyHostToDevice, st));
  for (int k = 0; k < b->cap; ++k)
    if (b->fresh[k]) {
      HIP_TRY(hipMemcpyAsync(b->dstat + k, &b->init_stat[k], sizeof(JobStat), hipMemcpyHostToDevice, st));
      b->fresh[k] = 0;
    }
  HIP_TRY(hipStreamSynchronize(st));
  b->committed = true;
  return CGKS_OK;
}

cgks_status cgks_batch_step(cgks_batch* b, int nsteps, void* stream) {
  if (!b) return fail(CGKS_EINVAL, "NULL batch");
  if (!b->committed) return fail(CGKS_ESTATE, "batch changed since the last cgks_batch_commit");
  if (nsteps < 0) return fail(CGKS_EINVAL, "nsteps must be >= 0");
  HIP_TRY(enqueue_steps(b, nsteps, (hipStream_t)stream));
  return CGKS_OK;
}

cgks_status cgks_batch_capture(cgks_batch* b, int nsteps) {
  if (!b) return fail(CGKS_EINVAL, "NULL batch");
  if (nsteps < 1) return fail(CGKS_EINVAL, "nsteps must be >= 1");
  drop_graph(b);
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_steps(b, nsteps, b->cap_stream);
  hipError_t e2 = hipStreamEndCapture(b->cap_stream, &graph);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  if (graph) hipGraphDestroy(graph);
  if (e != hipSuccess) {
    b->exec = nullptr;
    return fail(CGKS_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  b->graph_steps = nsteps;
  return CGKS_OK;
}

cgks_status cgks_batch_launch(cgks_batch* b, void* stream) {
  if (!b) return fail(CGKS_EINVAL, "NULL batch");
  if (!b->exec) return fail(CGKS_ESTATE, "no captured graph (cgks_batch_capture)");
  if (!b->committed) return fail(CGKS_ESTATE, "batch changed since the last cgks_batch_commit");
  HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
  return CGKS_OK;
}

cgks_status cgks_batch_poll(cgks_batch* b, cgks_job_status* out, void* stream) {
  if (!b || !out) return fail(CGKS_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  // into pinned memory (a copy into pageable memory goes through a staging buffer)
  const JobStat* hs = b->hstat;
  HIP_TRY(hipMemcpyAsync(b->hstat, b->dstat, sizeof(JobStat) * b->cap, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int k = 0; k < b->cap; ++k) {
    out[k].in_use = b->busy[k];
    if (!b->busy[k]) {
      out[k].t = 0.0; out[k].dt = 0.0; out[k].steps = 0; out[k].status = 0;
      continue;
    }
    const JobStat& s = b->fresh[k] ? b->init_stat[k] : hs[k];
    out[k].t = s.t;
    out[k].dt = s.dt;
    out[k].steps = s.steps;
    out[k].status = s.status;
  }
  return CGKS_OK;
}

cgks_status cgks_batch_info(const cgks_batch* b, int* njobs, size_t* bytes_used, size_t* table_bytes,
                            int* grid_face) {
  if (!b) return fail(CGKS_EINVAL, "NULL batch");
  int n = 0;
  for (int k = 0; k < b->cap; ++k) n += b->busy[k];
  if (njobs) *njobs = n;
  if (bytes_used) *bytes_used = b->used;
  if (table_bytes) *table_bytes = b->off_stat + sizeof(JobStat) * b->cap;
  if (grid_face) *grid_face = b->dim == 2 ? b->grid[K_FACE] : b->grid[K_S1D];
  return CGKS_OK;
}

cgks_status cgks_batch_set_tuning(cgks_batch* b, const cgks_batch_tuning* t) {
  if (!b || !t) return fail(CGKS_EINVAL, "NULL argument");
  if (t->grid_mult < 1 || t->grid_mult > 16) return fail(CGKS_EINVAL, "grid_mult must lie in [1, 16]");
  if (t->face_tile < 0 || t->face_tile >= kFaceTiles) return fail(CGKS_EINVAL, "face_tile must lie in [0, 2]");
  if (t->line_tile < 0 || t->line_tile >= kLineTiles) return fail(CGKS_EINVAL, "line_tile must lie in [0, 1]");
  const bool reshape = t->face_tile != b->tune.face_tile || t->line_tile != b->tune.line_tile;
  b->tune.grid_mult = t->grid_mult;
  b->tune.xcd_remap = t->xcd_remap ? 1 : 0;
  b->tune.face_tile = t->face_tile;
  b->tune.line_tile = t->line_tile;
  b->tune.ms_per_step = t->ms_per_step;
  if (reshape) {
    // the jobs' tile counts follow the shapes: the table must be uploaded again
    for (int k = 0; k < b->cap; ++k)
      if (b->busy[k]) fill_counts(b->slots[k], b->tune.face_tile, b->tune.line_tile);
    b->committed = false;
  }
  set_grids(b);
  drop_graph(b);   // launch shapes are baked into a captured graph
  return CGKS_OK;
}

cgks_status cgks_batch_get_tuning(const cgks_batch* b, cgks_batch_tuning* t) {
  if (!b || !t) return fail(CGKS_EINVAL, "NULL argument");
  *t = b->tune;
  return CGKS_OK;
}

// Times `steps_per_trial` real steps of the committed jobs under each
// candidate and keeps the fastest: first the tile shapes of the face and
// Step 1 kernels (2-D batches; the table is uploaded again for each), with
// the current grid multiplier and remap, then the grid multiplier and remap
// with the chosen shapes.  Every candidate computes the same result, so the
// trial steps advance the jobs as ordinary steps do.
cgks_status cgks_batch_tune(cgks_batch* b, int steps_per_trial, void* stream, cgks_batch_tuning* chosen) {
  if (!b) return fail(CGKS_EINVAL, "NULL batch");
  if (!b->committed) return fail(CGKS_ESTATE, "batch changed since the last cgks_batch_commit");
  if (steps_per_trial < 1) return fail(CGKS_EINVAL, "steps_per_trial must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  cgks_batch_tuning best = b->tune;
  best.ms_per_step = -1.0f;
  hipError_t e = hipSuccess;
  cgks_status cs = CGKS_OK;
  auto trial = [&](const cgks_batch_tuning& c) {
    cgks_batch_tuning t = c;
    if ((cs = cgks_batch_set_tuning(b, &t)) != CGKS_OK) return;
    if (!b->committed && (cs = cgks_batch_commit(b, stream)) != CGKS_OK) return;
    if ((e = hipEventRecord(e0, st)) != hipSuccess) return;
    if ((e = enqueue_steps(b, steps_per_trial, st)) != hipSuccess) return;
    if ((e = hipEventRecord(e1, st)) != hipSuccess) return;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return;
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return;
    t.ms_per_step = ms / steps_per_trial;
    if (best.ms_per_step < 0.0f || t.ms_per_step < best.ms_per_step) best = t;
  };
  const cgks_batch_tuning start = b->tune;
  if (b->dim == 2)
    for (int v = 0; v < kFaceTiles && e == hipSuccess && cs == CGKS_OK; ++v)
      for (int lw = 0; lw < kLineTiles && e == hipSuccess && cs == CGKS_OK; ++lw) {
        cgks_batch_tuning c = start;
        c.face_tile = v;
        c.line_tile = lw;
        trial(c);
      }
  const int mults[] = {1, 2, 4};
  const int fv = b->dim == 2 ? best.face_tile : start.face_tile, flw = b->dim == 2 ? best.line_tile : start.line_tile;
  for (int remap = 0; remap < 2 && e == hipSuccess && cs == CGKS_OK; ++remap)
    for (int mi = 0; mi < 3 && e == hipSuccess && cs == CGKS_OK; ++mi) {
      cgks_batch_tuning c{};
      c.grid_mult = mults[mi];
      c.xcd_remap = remap;
      c.face_tile = fv;
      c.line_tile = flw;
      trial(c);
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (cs != CGKS_OK) return cs;
  if (e != hipSuccess) return fail(CGKS_EHIP, std::string("tune: ") + hipGetErrorString(e));
  cgks_batch_tuning keep = best;
  if ((cs = cgks_batch_set_tuning(b, &keep)) != CGKS_OK) return cs;
  if (!b->committed && (cs = cgks_batch_commit(b, stream)) != CGKS_OK) return cs;
  b->tune.ms_per_step = best.ms_per_step;
  if (chosen) *chosen = b->tune;
  return CGKS_OK;
}

}  // extern "C"
