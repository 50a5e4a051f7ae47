// libcgks.so: single-grid kernels and the plan/state C ABI of the ASE-DFF
// compact gas-kinetic scheme on one MI355X (gfx950).  The C ABI is declared in
// include/cgks.h; the batched kernels live in cgks_batch.hip, the shared types
// and per-tile device bodies in cgks_internal.hpp.
#define CGKS_UNIT single
#include "cgks_internal.hpp"

thread_local std::string cgks_g_err;

#include <mutex>

// Scratch of cgks_conservation_sums_static: the block partials of the
// conservation-sum reduction (double-double, [variable][block]), for callers
// that cannot allocate.  Each device holds its own copy for the life of the
// process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name is a host-side
// stand-in).  Every call on one device shares it.
constexpr int kStaticSumBlocks = 4096;   // grids up to 4096 * SUM_CHUNK = 2^26 interior cells
static __device__ __align__(256) double scratch[(size_t)kStaticSumBlocks * 4 * 2];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device, once resolved
}  // namespace

namespace {

// ---------------------------------------------------------------------------
// single-grid kernels: one launch per phase, one block per tile
// ---------------------------------------------------------------------------
// Strengths of the first step from the piecewise-constant states.
__global__ void k_init_sigma(Geo g, int which, double gam, const double* U, double* sxn, double* syn) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  const int D = g.dim;
  if (which == 0) {
    if (a > g.nx || b >= (D == 2 ? g.ny : 1)) return;
    double Wl[4], Wr[4];
    for (int v = 0; v < g.nv; ++v) { Wl[v] = U[g.avg(v, a - 1, b)]; Wr[v] = U[g.avg(v, a, b)]; }
    sxn[g.sgx(b, a)] = sigma_pair(Wl, Wr, D, gam);
  } else {
    if (a > g.ny || b >= g.nx) return;
    const int perm[4] = {0, 2, 1, 3};
    double Wl[4], Wr[4];
    for (int v = 0; v < 4; ++v) { Wl[perm[v]] = U[g.avg(v, b, a - 1)]; Wr[perm[v]] = U[g.avg(v, b, a)]; }
    syn[g.sgy(b, a)] = sigma_pair(Wl, Wr, 2, gam);
  }
}

// code: the time the ghosts are for (bc_time); ST: slope storage type
template <typename ST>
__global__ void k_bc_state(Geo g, const BcTable* T, const Header* hdr, int code, double* U) {
  int I, Jr;
  GhostItems(g).at(g, blockIdx.x, I, Jr);
  bc_state_at<ST>(g, T, bc_time(hdr, code), U, I, Jr);
}

__global__ void k_bc_sigma(Geo g, const BcTable* T, const Header* hdr, int which, const double* sxn, double* sxo,
                           const double* syn, double* syo) {
  bc_sigma_at(g, T, bc_time(hdr, 1), which, sxn, sxo, syn, syo, blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y);
}

__global__ void k_dt(Header* hdr, const double* part, double sbc, double dt_fixed, double cfl, double t_end, double h, double mu,
                     int viscous) {
  dt_block(hdr, part, sbc, dt_fixed, cfl, t_end, h, mu, viscous, 0, nullptr);
}

// Block (x, y) of a 2-D grid as the dispatcher orders it (x fastest) goes to
// XCD b mod 8, b = y * gridDim.x + x.  The kernels below work on the logical
// block xcd_block(b) instead: each XCD takes one contiguous run of logical
// blocks (a band of rows or tiles), so the halos that neighbouring blocks
// share are fetched into one L2.  A bijection for any block count.
__device__ __forceinline__ int xcd_block(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

template <int M, typename ST>
__global__ __launch_bounds__(256) void k_lines(Geo g, Consts C, const double* U, const double* sxo,
                                               const double* syo, double* lvx, double* lvy, Header* hdr) {
  __shared__ double sm[LinesLds<0>::total];
  if (!hdr->active) return;
  const int lb = xcd_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  lines_tile<M, ST>(g, C, U, sxo, syo, lvx, lvy, hdr, lb % gridDim.x, lb / gridDim.x, sm);
}

// Grid (tiles along the normal, tiles along the tangential).  x-face tiles
// are taken normal-first and y-face tiles tangential-first: either way the
// tiles that run together are neighbours along x, the contiguous direction,
// and share their cache lines in L2 (a y-face tile spans only NT + 2 cells
// along x).
// FP32 kernels: the LDS layout of their own direction, for their wave count
// (FP64 keeps the shared layout)
template <typename T, int DIR, int STAGE>
constexpr int kOwnW = sizeof(T) == 4 ? FaceWaves<T, DIR, STAGE>::value : 0;

template <int DIR, int STAGE, int M, typename T, bool PR>
__global__ __launch_bounds__(256, (FaceWaves<T, DIR, STAGE>::value)) void k_face2d(Geo g, Consts C, Bufs B) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lb = xcd_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int bx = DIR == 0 ? lb % gridDim.x : lb / gridDim.y;
  const int by = DIR == 0 ? lb / gridDim.x : lb % gridDim.y;
  face2d_tile<DIR, STAGE, M, T, PR, 32, false, 0, true, kOwnW<T, DIR, STAGE>>(g, C, B, smem, bx, by, gridDim.x, gridDim.y);
}

template <int STAGE, typename T, bool PR>
__global__ __launch_bounds__(256) void k_stage1d(Geo g, Consts C, Bufs B) {
  if constexpr (sizeof(T) == 4) {   // inputs copied into LDS by DMA
    __shared__ S1In<T> in;
    __shared__ S1Acc<T> acc;
    __shared__ S1Mid<T, STAGE> mid;
    s1_issue_in<STAGE, T>(g, B, blockIdx.x, &in, threadIdx.x);
    s1_landed();
    stage1d_seg_lds<STAGE, T, PR>(g, C, B, &in, &acc, &mid, blockIdx.x, gridDim.x);
  } else {                           // inputs through registers
    __shared__ double res[256][12];
    __shared__ __align__(16) unsigned char sm[Lds1D<T>::total];
    stage1d_seg<STAGE, T, PR>(g, C, B, res, sm, blockIdx.x, gridDim.x);
  }
}

__global__ __launch_bounds__(256) void k_sum1(Geo g, const double* U, DD* part, int nblk) {
  sums_pass1(g, U, part, nblk, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_sum2(int nv, const DD* part, int nblk, double* out) {
  sums_pass2(nv, part, nblk, out);
}

__global__ __launch_bounds__(256) void k_reduce(Geo g, double gam, const double* U, Bufs B) {
  Header* hdr = B.hdr;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  bool valid = i < g.nx;
  double s = 0.0, r = 1.0;
  if (valid) {
    double W[4];
    for (int v = 0; v < g.nv; ++v) W[v] = U[g.avg(v, i, j)];
    r = W[0];
    if (!cell_speed(W, g.dim, gam, s)) {
      atomicAdd(&hdr->nonphysical, 1ull);
      valid = false;
    }
  }
  reduce_speed(B, s, r, valid, blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
// Optional per-launch event marks (cgks_step_timed): mark k is recorded on
// the launch stream after launch k-1 and before launch k.
struct Marks {
  hipEvent_t ev[17];
  int n = 0;
  void tick(hipStream_t st) {
    if (n < 17) hipEventRecord(ev[n++], st);
  }
};
static inline void tick(Marks* mk, hipStream_t st) {
  if (mk) mk->tick(st);
}
hipError_t launch_bc_state(const cgks_plan* p, const Bufs& b, double* U, int code, hipStream_t st,
                           Marks* mk = nullptr) {
  const Geo& g = p->g;
  const dim3 grid(GhostItems(g).count(g));   // the segments that hold ghost cells
  if (p->precision == CGKS_FP64) hipLaunchKernelGGL(k_bc_state<double>, grid, dim3(256), 0, st, g, b.bct, b.hdr, code, U);
  else hipLaunchKernelGGL(k_bc_state<float>, grid, dim3(256), 0, st, g, b.bct, b.hdr, code, U);
  tick(mk, st);
  return hipGetLastError();
}

hipError_t launch_bc_sigma(const cgks_plan* p, const Bufs& b, hipStream_t st, Marks* mk = nullptr) {
  const Geo& g = p->g;
  dim3 gx((g.NX + 1 + 255) / 256, g.NY);
  hipLaunchKernelGGL(k_bc_sigma, gx, dim3(256), 0, st, g, b.bct, b.hdr, 0, b.sxn, b.sxo, b.syn, b.syo);
  if (g.dim == 2) {
    dim3 gy((g.NY + 1 + 255) / 256, g.NX);
    hipLaunchKernelGGL(k_bc_sigma, gy, dim3(256), 0, st, g, b.bct, b.hdr, 1, b.sxn, b.sxo, b.syn, b.syo);
  }
  tick(mk, st);
  return hipGetLastError();
}

template <int M, typename T, bool PR>
hipError_t launch_stage2d(const cgks_plan* p, const Bufs& b, int stage, hipStream_t st, Marks* mk) {
  const Geo& g = p->g;
  using TL = Tile<M>;
  const double* Uin = stage == 1 ? b.U : b.S;
  {
    dim3 grid((g.NX + LT_X - 1) / LT_X, (g.NY + LT_Y - 1) / LT_Y);
    hipLaunchKernelGGL((k_lines<M, T>), grid, dim3(256), 0, st, g, p->C, Uin, b.sxo, b.syo, b.lvx, b.lvy, b.hdr);
    tick(mk, st);
  }
  constexpr size_t lx1 = FaceLds<0, M, T, 0, kOwnW<T, 0, 1>>::total, ly1 = FaceLds<1, M, T, 0, kOwnW<T, 1, 1>>::total;
  constexpr size_t lx2 = FaceLds<0, M, T, 0, kOwnW<T, 0, 2>>::total, ly2 = FaceLds<1, M, T, 0, kOwnW<T, 1, 2>>::total;
  dim3 gx((g.nx + TL::NF - 2) / (TL::NF - 1), (g.ny + TL::NT - 1) / TL::NT);
  dim3 gy((g.ny + TL::NF - 2) / (TL::NF - 1), (g.nx + TL::NT - 1) / TL::NT);
  if (stage == 1) {
    hipLaunchKernelGGL((k_face2d<0, 1, M, T, PR>), gx, dim3(256), lx1, st, g, p->C, b);
    tick(mk, st);
    hipLaunchKernelGGL((k_face2d<1, 1, M, T, PR>), gy, dim3(256), ly1, st, g, p->C, b);
    tick(mk, st);
  } else {
    hipLaunchKernelGGL((k_face2d<0, 2, M, T, PR>), gx, dim3(256), lx2, st, g, p->C, b);
    tick(mk, st);
    hipLaunchKernelGGL((k_face2d<1, 2, M, T, PR>), gy, dim3(256), ly2, st, g, p->C, b);
    tick(mk, st);
  }
  return hipGetLastError();
}

template <typename T, bool PR>
hipError_t launch_stage_pr(const cgks_plan* p, const Bufs& b, int stage, hipStream_t st, Marks* mk) {
  const Geo& g = p->g;
  if (g.dim == 1) {
    dim3 grid((g.nx + S1_CELLS - 1) / S1_CELLS);
    if (stage == 1) hipLaunchKernelGGL((k_stage1d<1, T, PR>), grid, dim3(256), 0, st, g, p->C, b);
    else hipLaunchKernelGGL((k_stage1d<2, T, PR>), grid, dim3(256), 0, st, g, p->C, b);
    tick(mk, st);
    return hipGetLastError();
  }
  switch (g.m) {
    case 2: return launch_stage2d<2, T, PR>(p, b, stage, st, mk);
    case 3: return launch_stage2d<3, T, PR>(p, b, stage, st, mk);
    default: return launch_stage2d<4, T, PR>(p, b, stage, st, mk);
  }
}

template <typename T>
hipError_t launch_stage(const cgks_plan* p, const Bufs& b, int stage, hipStream_t st, Marks* mk) {
  return p->C.prandtl != 1.0 ? launch_stage_pr<T, true>(p, b, stage, st, mk)
                             : launch_stage_pr<T, false>(p, b, stage, st, mk);
}

// One step: dt, strengths, ghosts, stage 1, ghosts of U*, stage 2.
hipError_t enqueue_step(const cgks_plan* p, const Bufs& b, double dt, double cfl, double t_end, hipStream_t st,
                        Marks* mk) {
  const Geo& g = p->g;
  const double h = g.dim == 2 ? fmin(p->dx, p->dy) : p->dx;
  tick(mk, st);
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(256), 0, st, b.hdr, b.part, p->bct.smax, dt, cfl, t_end, h, p->C.mu,
                     p->C.tau_model == CGKS_TAU_VISCOUS ? 1 : 0);
  tick(mk, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_bc_sigma(p, b, st, mk)) != hipSuccess) return e;
  if ((e = launch_bc_state(p, b, b.U, 1, st, mk)) != hipSuccess) return e;
  e = p->precision == CGKS_FP64 ? launch_stage<double>(p, b, 1, st, mk) : launch_stage<float>(p, b, 1, st, mk);
  if (e != hipSuccess) return e;
  if ((e = launch_bc_state(p, b, b.S, 2, st, mk)) != hipSuccess) return e;
  return p->precision == CGKS_FP64 ? launch_stage<double>(p, b, 2, st, mk) : launch_stage<float>(p, b, 2, st, mk);
}

const char* kKernels1d[] = {"dt", "bc_sigma", "bc_state", "stage1_1d", "bc_state", "stage2_1d"};
const char* kKernels2d[] = {"dt", "bc_sigma", "bc_state", "lines", "face_x_stage1", "face_y_stage1",
                            "bc_state", "lines", "face_x_stage2", "face_y_stage2"};

// Face kernels of one order and precision: dynamic LDS limit and the scratch
// check (no scratch).
template <int DIR, int STAGE, int M, typename T, bool PR>
cgks_status prepare_face() {
  const void* f = (const void*)k_face2d<DIR, STAGE, M, T, PR>;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)FaceLds<DIR, M, T, 0, kOwnW<T, DIR, STAGE>>::total);
  if (e != hipSuccess) return fail(CGKS_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  return check_private(f, 0, "face kernel");
}

template <int M, typename T, bool PR>
cgks_status prepare_faces_pr() {
  cgks_status s;
  if ((s = prepare_face<0, 1, M, T, PR>()) != CGKS_OK) return s;
  if ((s = prepare_face<1, 1, M, T, PR>()) != CGKS_OK) return s;
  if ((s = prepare_face<0, 2, M, T, PR>()) != CGKS_OK) return s;
  if ((s = prepare_face<1, 2, M, T, PR>()) != CGKS_OK) return s;
  return check_private((const void*)k_lines<M, T>, 0, "line kernel");
}

template <int M, typename T>
cgks_status prepare_faces() {
  cgks_status s = prepare_faces_pr<M, T, false>();
  return s != CGKS_OK ? s : prepare_faces_pr<M, T, true>();
}

template <typename T>
cgks_status prepare_1d() {
  cgks_status s;
  if ((s = check_private((const void*)k_stage1d<1, T, false>, 0, "1-D stage kernel")) != CGKS_OK) return s;
  if ((s = check_private((const void*)k_stage1d<2, T, false>, 0, "1-D stage kernel")) != CGKS_OK) return s;
  if ((s = check_private((const void*)k_stage1d<1, T, true>, 0, "1-D stage kernel")) != CGKS_OK) return s;
  return check_private((const void*)k_stage1d<2, T, true>, 0, "1-D stage kernel");
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* cgks_status_string(cgks_status s) {
  switch (s) {
    case CGKS_OK: return "ok";
    case CGKS_EINVAL: return "invalid argument";
    case CGKS_ENOMEM: return "out of host memory";
    case CGKS_EHIP: return "HIP runtime error";
    case CGKS_ENONPHYSICAL: return "nonphysical state";
    case CGKS_ESTATE: return "work buffer holds no initialised state";
    case CGKS_EBUDGET: return "over budget";
  }
  return "unknown status";
}

const char* cgks_last_error(void) { return cgks_g_err.c_str(); }

cgks_status cgks_plan_create(const cgks_grid_desc* gd, const cgks_scheme_desc* sd, cgks_plan** out) {
  if (!gd || !sd || !out) return fail(CGKS_EINVAL, "NULL argument");
  *out = nullptr;
  if (gd->dim != 1 && gd->dim != 2) return fail(CGKS_EINVAL, "dim must be 1 or 2");
  if (sd->order != 5 && sd->order != 7 && sd->order != 9) return fail(CGKS_EINVAL, "order must be 5, 7 or 9");
  if (!(sd->gamma > 1.0)) return fail(CGKS_EINVAL, "gamma must exceed 1");
  if (gd->nx < 5 || (gd->dim == 2 && gd->ny < 5)) return fail(CGKS_EINVAL, "need at least 5 cells per direction");
  if (gd->dim == 1 && gd->ny != 1) return fail(CGKS_EINVAL, "1-D grids need ny = 1");
  if (!(gd->x1 > gd->x0) || (gd->dim == 2 && !(gd->y1 > gd->y0))) return fail(CGKS_EINVAL, "empty domain");
  for (int k = 0; k < (gd->dim == 2 ? 4 : 2); ++k) {
    const int b = gd->bc[k];
    if (b < CGKS_BC_PERIODIC || b > CGKS_BC_SEGMENTED) return fail(CGKS_EINVAL, "unknown boundary condition");
    if (b != CGKS_BC_INFLOW && b != CGKS_BC_SEGMENTED) continue;
    const cgks_bc_side& S = gd->side[k];
    const int ns = b == CGKS_BC_INFLOW ? 1 : S.nseg;
    if (ns < 1 || ns > CGKS_MAX_SEGMENTS) return fail(CGKS_EINVAL, "a segmented side needs 1 to 3 segments");
    for (int q = 0; q < ns; ++q) {
      const int ty = b == CGKS_BC_INFLOW ? CGKS_BC_INFLOW : S.type[q];
      if (ty < CGKS_BC_TRANSMISSIVE || ty > CGKS_BC_INFLOW) return fail(CGKS_EINVAL, "unknown segment kind");
      if (ty == CGKS_BC_INFLOW) {
        const double* w = S.prim[q];
        const double rho = w[0], pr = gd->dim == 2 ? w[3] : w[2];
        for (int v = 0; v < 4; ++v)
          if (!std::isfinite(w[v])) return fail(CGKS_EINVAL, "prescribed state must be finite");
        if (!(rho > 0.0) || !(pr > 0.0)) return fail(CGKS_EINVAL, "prescribed state needs rho > 0 and p > 0");
      }
    }
    for (int q = 0; q + 1 < ns; ++q)
      if (!std::isfinite(S.end0[q]) || !std::isfinite(S.speed[q])) return fail(CGKS_EINVAL, "segment ends must be finite");
  }
  if ((gd->bc[0] == CGKS_BC_PERIODIC) != (gd->bc[1] == CGKS_BC_PERIODIC))
    return fail(CGKS_EINVAL, "periodic x needs both ends periodic");
  if (gd->dim == 2 && (gd->bc[2] == CGKS_BC_PERIODIC) != (gd->bc[3] == CGKS_BC_PERIODIC))
    return fail(CGKS_EINVAL, "periodic y needs both ends periodic");
  if (sd->tau_model < 0 || sd->tau_model > 2) return fail(CGKS_EINVAL, "unknown tau model");
  if (!(sd->prandtl > 0.0)) return fail(CGKS_EINVAL, "prandtl must be > 0");
  if (sd->tau_model == CGKS_TAU_VISCOUS && !(sd->mu >= 0.0)) return fail(CGKS_EINVAL, "mu must be >= 0");
  if (!(sd->sigma_thres > 0.0)) return fail(CGKS_EINVAL, "sigma_thres must be > 0");
  if (!(sd->gamma_hi > 0.0 && sd->gamma_hi < 1.0 && sd->gamma_lo > 0.0 && sd->gamma_lo < 1.0))
    return fail(CGKS_EINVAL, "linear weights must lie in (0, 1)");
  if (sd->precision != CGKS_FP64 && sd->precision != CGKS_FP32_FLUX) return fail(CGKS_EINVAL, "unknown precision");
  if (sd->reading_flags & ~(CGKS_READ_A3_GAMMA1_LO | CGKS_READ_A5_UNSCALED_BETA | CGKS_READ_A10_SIGMA0_ZERO))
    return fail(CGKS_EINVAL, "unknown reading flag");
  if (gd->nx > (1 << 24) || gd->ny > (1 << 24)) return fail(CGKS_EINVAL, "grid too large");

  cgks_plan* p = new (std::nothrow) cgks_plan;
  if (!p) return fail(CGKS_ENOMEM, "plan allocation");
  memset(p, 0, sizeof(*p));
  Geo& g = p->g;
  g.dim = gd->dim;
  g.nx = gd->nx;
  g.ny = gd->dim == 2 ? gd->ny : 1;
  g.NX = g.nx + 2 * H;
  g.NY = gd->dim == 2 ? g.ny + 2 * H : 1;
  g.m = gd->dim == 2 ? (sd->order == 5 ? 2 : (sd->order == 7 ? 3 : 4)) : 1;
  g.nv = gd->dim + 2;
  for (int k = 0; k < 4; ++k) g.bc[k] = (k < 2 || gd->dim == 2) ? gd->bc[k] : CGKS_BC_PERIODIC;
  g.cells = (size_t)g.NX * g.NY;
  p->dx = (gd->x1 - gd->x0) / gd->nx;
  p->dy = gd->dim == 2 ? (gd->y1 - gd->y0) / gd->ny : 1.0;
  // sides with a prescribed state or segments: one table (kernels see code
  // SEGMENTED); prescribed states in conservative variables
  p->bct.x0 = gd->x0;
  p->bct.y0 = gd->dim == 2 ? gd->y0 : 0.0;
  p->bct.dx = p->dx;
  p->bct.dy = p->dy;
  for (int k = 0; k < 4; ++k) {
    if (g.bc[k] != CGKS_BC_INFLOW && g.bc[k] != CGKS_BC_SEGMENTED) continue;
    const cgks_bc_side& S = gd->side[k];
    BcSide& T = p->bct.side[k];
    T.nseg = g.bc[k] == CGKS_BC_INFLOW ? 1 : S.nseg;
    for (int q = 0; q < T.nseg; ++q) {
      T.type[q] = g.bc[k] == CGKS_BC_INFLOW ? CGKS_BC_INFLOW : S.type[q];
      if (T.type[q] != CGKS_BC_INFLOW) continue;
      const double* w = S.prim[q];
      const double gm1 = sd->gamma - 1.0;
      if (gd->dim == 2) {
        T.cons[q][0] = w[0];
        T.cons[q][1] = w[0] * w[1];
        T.cons[q][2] = w[0] * w[2];
        T.cons[q][3] = w[3] / gm1 + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2]);
      } else {
        T.cons[q][0] = w[0];
        T.cons[q][1] = w[0] * w[1];
        T.cons[q][2] = w[2] / gm1 + 0.5 * w[0] * w[1] * w[1];
      }
    }
    for (int q = 0; q < T.nseg; ++q) {
      if (T.type[q] != CGKS_BC_INFLOW) continue;
      const double* w = S.prim[q];
      const double u = w[1], v = gd->dim == 2 ? w[2] : 0.0, pr = gd->dim == 2 ? w[3] : w[2];
      const double sp = sqrt(u * u + v * v) + sqrt(sd->gamma * pr / w[0]);
      if (sp > p->bct.smax) p->bct.smax = sp;
    }
    for (int q = 0; q + 1 < T.nseg; ++q) {
      T.end0[q] = S.end0[q];
      T.speed[q] = S.speed[q];
    }
    g.bc[k] = CGKS_BC_SEGMENTED;
  }
  Consts& C = p->C;
  C.gamma = sd->gamma;
  C.Kd = 2.0 / (sd->gamma - 1.0);
  C.iKd = 1.0 / C.Kd;
  C.c1 = sd->c1;
  C.c2 = sd->c2;
  C.mu = sd->mu;
  C.prandtl = sd->prandtl;
  C.prfac = 1.0 / sd->prandtl - 1.0;
  C.thres = sd->sigma_thres;
  C.ghi = sd->gamma_hi;
  C.glo = sd->gamma_lo;
  C.eps = sd->weno_eps;
  static_assert(RF_A3_GAMMA1_LO == CGKS_READ_A3_GAMMA1_LO && RF_A5_UNSCALED_BETA == CGKS_READ_A5_UNSCALED_BETA &&
                RF_A10_SIGMA0_ZERO == CGKS_READ_A10_SIGMA0_ZERO, "reading flags");
  C.rflags = sd->reading_flags;
  {
    const double gH = sd->gamma_hi, gL = sd->gamma_lo, share = (1.0 - gH) * (1.0 - gL) / 2.0;
    C.gw[0] = share;
    C.gw[1] = (sd->reading_flags & CGKS_READ_A3_GAMMA1_LO) ? (1.0 - gH) * gL : share;
    C.gw[2] = (sd->reading_flags & CGKS_READ_A3_GAMMA1_LO) ? share : (1.0 - gH) * gL;
  }
  // near-tie band of the cascade decisions: the strengths entering A carry
  // the rounding of the flux arithmetic (FP64, or FP32 in the FP32-flux
  // variant), summed over up to 12 weighted faces
  C.tie = sd->sigma_thres * (sd->precision == CGKS_FP64 ? 1e-12 : 1e-5);
  C.dx = p->dx;
  C.idx = 1.0 / p->dx;
  C.idx2 = 1.0 / (p->dx * p->dx);
  C.idy = 1.0 / p->dy;
  C.idy2 = 1.0 / (p->dy * p->dy);
  C.dy = p->dy;
  C.tau_model = sd->tau_model;
  C.order = sd->order;
  C.m = gd->dim == 2 ? g.m : 1;
  p->precision = sd->precision;
  const size_t nv = g.nv, m = g.m, cells = g.cells;
  // averages in double, slopes and line values in the working precision
  const size_t esz = sd->precision == CGKS_FP64 ? sizeof(double) : sizeof(float);
  auto words = [](size_t bytes) { return (bytes + sizeof(double) - 1) / sizeof(double); };
  p->state_words = g.avg_words() + words(g.slope_elems() * esz);
  p->sig_x_words = (size_t)g.NY * (g.NX + 1);
  p->sig_y_words = g.dim == 2 ? (size_t)g.NX * (g.NY + 1) : 0;
  auto up = [](size_t w) { return (w + 31) & ~(size_t)31; };  // 256-byte aligned sections
  size_t o = 0;
  p->off_S = o; o += up(p->state_words);
  p->off_A = o; o += up(p->state_words);
  p->off_sxo = o; o += up(p->sig_x_words);
  p->off_sxn = o; o += up(p->sig_x_words);
  p->off_syo = o; o += up(p->sig_y_words);
  p->off_syn = o; o += up(p->sig_y_words);
  p->off_lvx = o; o += g.dim == 2 ? up(words(nv * m * cells * esz)) : 0;
  p->off_lvy = o; o += g.dim == 2 ? up(words(nv * m * cells * esz)) : 0;
  {
    // partials: the initial reduction grid, the 1-D stage grid, the 2-D y-face grid
    size_t a = (size_t)((g.nx + 255) / 256) * (g.dim == 2 ? g.ny : 1);
    size_t b1 = (size_t)((g.nx + S1_CELLS - 1) / S1_CELLS);
    size_t c = 0;
    if (g.dim == 2)   // y-face tiles of every tile shape (the batched kernels may take any)
      for (int v = 0; v < kFaceTiles; ++v) {
        const size_t t = (size_t)face_tiles_n(g.ny, tile_nf(v)) * face_tiles_t(g.nx, tile_nt(v, g.m));
        if (t > c) c = t;
      }
    p->max_parts = a > b1 ? (a > c ? a : c) : (b1 > c ? b1 : c);
  }
  p->off_part = o; o += up(2 * p->max_parts);
  p->off_hdr = o; o += 32;
  p->off_bct = o; o += up((sizeof(BcTable) + 7) / 8);
  {
    const long long nint = (long long)g.nx * g.ny;
    p->sum_blocks = (int)((nint + SUM_CHUNK - 1) / SUM_CHUNK);
    p->off_sum = o; o += up((size_t)p->sum_blocks * nv * 2);
  }
  p->work_words = o;
  *out = p;
  return CGKS_OK;
}

cgks_status cgks_plan_sizes(const cgks_plan* p, size_t* state_bytes, size_t* work_bytes) {
  if (!p) return fail(CGKS_EINVAL, "NULL plan");
  if (state_bytes) *state_bytes = p->state_words * sizeof(double);
  if (work_bytes) *work_bytes = p->work_words * sizeof(double);
  return CGKS_OK;
}

cgks_status cgks_plan_destroy(cgks_plan* p) {
  delete p;
  return CGKS_OK;
}

static cgks_status ensure_lds(const cgks_plan* p) {
  const bool d = p->precision == CGKS_FP64;
  if (p->g.dim != 2) return d ? prepare_1d<double>() : prepare_1d<float>();
  if (d) return p->g.m == 2 ? prepare_faces<2, double>() : (p->g.m == 3 ? prepare_faces<3, double>() : prepare_faces<4, double>());
  return p->g.m == 2 ? prepare_faces<2, float>() : (p->g.m == 3 ? prepare_faces<3, float>() : prepare_faces<4, float>());
}

cgks_status cgks_init_state(const cgks_plan* p, void* d_state, void* d_work, const double* h_avg,
                            const double* h_slope_x, const double* h_slope_y, const double* h_sigma_x,
                            const double* h_sigma_y, double t0, void* stream) {
  if (!p || !d_state || !d_work || !h_avg || !h_slope_x) return fail(CGKS_EINVAL, "NULL argument");
  const Geo& g = p->g;
  if (g.dim == 2 && !h_slope_y) return fail(CGKS_EINVAL, "2-D needs h_slope_y");
  if (g.dim == 2 && ((h_sigma_x == nullptr) != (h_sigma_y == nullptr)))
    return fail(CGKS_EINVAL, "give both strength arrays or neither");
  cgks_status cs = ensure_lds(p);
  if (cs != CGKS_OK) return cs;
  hipStream_t st = (hipStream_t)stream;
  const int nx = g.nx, ny = g.ny, m = g.m, nv = g.nv;
  std::vector<double> hs;
  try {
    hs.assign(p->state_words, 0.0);
  } catch (...) {
    return fail(CGKS_ENOMEM, "staging buffer");
  }
  // slopes in the storage type of the plan (rounded to float in the FP32-flux variant)
  const bool f64 = p->precision == CGKS_FP64;
  auto put_slope = [&](size_t k, double val) {
    if (f64) slopes<double>(hs.data(), g)[k] = val;
    else slopes<float>(hs.data(), g)[k] = (float)val;
  };
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        hs[g.avg(v, i, j)] = h_avg[((size_t)v * ny + j) * nx + i];
        for (int l = 0; l < m; ++l) {
          put_slope(g.sx(v, l, i, j), h_slope_x[(((size_t)v * m + l) * ny + j) * nx + i]);
          if (g.dim == 2) put_slope(g.sy(v, l, i, j), h_slope_y[(((size_t)v * m + l) * ny + j) * nx + i]);
        }
      }
  Bufs b = bufs(p, d_state, d_work);
  HIP_TRY(hipMemsetAsync(d_work, 0, p->work_words * sizeof(double), st));
  HIP_TRY(hipMemcpyAsync(d_state, hs.data(), p->state_words * sizeof(double), hipMemcpyHostToDevice, st));
  Header hh;
  memset(&hh, 0, sizeof(hh));
  hh.t = t0;
  hh.rmin_bits = 0x7ff0000000000000ull;
  hh.magic = kMagic;
  hh.active = 1;
  HIP_TRY(hipMemcpyAsync(b.hdr, &hh, sizeof(hh), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync((void*)b.bct, &p->bct, sizeof(BcTable), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_bc_state(p, b, b.U, 0, st));
  if (h_sigma_x) {
    std::vector<double> sx(p->sig_x_words, 0.0), sy(p->sig_y_words, 0.0);
    for (int j = 0; j < ny; ++j)
      for (int F = 0; F <= nx; ++F) sx[g.sgx(j, F)] = h_sigma_x[(size_t)j * (nx + 1) + F];
    if (g.dim == 2)
      for (int G = 0; G <= ny; ++G)
        for (int i = 0; i < nx; ++i) sy[g.sgy(i, G)] = h_sigma_y[(size_t)G * nx + i];
    HIP_TRY(hipMemcpyAsync(b.sxn, sx.data(), sx.size() * sizeof(double), hipMemcpyHostToDevice, st));
    if (g.dim == 2)
      HIP_TRY(hipMemcpyAsync(b.syn, sy.data(), sy.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  } else if (p->C.rflags & CGKS_READ_A10_SIGMA0_ZERO) {
    // first-step strengths zero: the work buffer was cleared above
  } else {
    dim3 gx((nx + 1 + 255) / 256, g.dim == 2 ? ny : 1);
    hipLaunchKernelGGL(k_init_sigma, gx, dim3(256), 0, st, g, 0, p->C.gamma, b.U, b.sxn, b.syn);
    if (g.dim == 2) {
      dim3 gy((ny + 1 + 255) / 256, nx);
      hipLaunchKernelGGL(k_init_sigma, gy, dim3(256), 0, st, g, 1, p->C.gamma, b.U, b.sxn, b.syn);
    }
    HIP_TRY(hipGetLastError());
  }
  {
    dim3 grid((nx + 255) / 256, g.dim == 2 ? ny : 1);
    hipLaunchKernelGGL(k_reduce, grid, dim3(256), 0, st, g, p->C.gamma, b.U, b);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(st));
  return CGKS_OK;
}

cgks_status cgks_step(const cgks_plan* p, void* d_state, void* d_work, double dt, double cfl, double t_end,
                      void* stream) {
  if (!p || !d_state || !d_work) return fail(CGKS_EINVAL, "NULL argument");
  if (!(dt > 0.0) && !(cfl > 0.0 && cfl <= 1.0)) return fail(CGKS_EINVAL, "cfl must lie in (0, 1]");
  Bufs b = bufs(p, d_state, d_work);
  HIP_TRY(enqueue_step(p, b, dt, cfl, t_end, (hipStream_t)stream, nullptr));
  return CGKS_OK;
}

cgks_status cgks_step_timed(const cgks_plan* p, void* d_state, void* d_work, double dt, double cfl, double t_end,
                            void* stream, double* kernel_ms, int* count) {
  if (!p || !d_state || !d_work || !kernel_ms || !count) return fail(CGKS_EINVAL, "NULL argument");
  if (!(dt > 0.0) && !(cfl > 0.0 && cfl <= 1.0)) return fail(CGKS_EINVAL, "cfl must lie in (0, 1]");
  hipStream_t st = (hipStream_t)stream;
  Marks mk;
  for (int k = 0; k < 17; ++k) HIP_TRY(hipEventCreate(&mk.ev[k]));
  Bufs b = bufs(p, d_state, d_work);
  hipError_t e = enqueue_step(p, b, dt, cfl, t_end, st, &mk);
  if (e == hipSuccess) e = hipEventSynchronize(mk.ev[mk.n - 1]);
  const int n = mk.n - 1;
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, mk.ev[k], mk.ev[k + 1]);
    kernel_ms[k] = ms;
  }
  for (int k = 0; k < 17; ++k) hipEventDestroy(mk.ev[k]);
  if (e != hipSuccess) return fail(CGKS_EHIP, std::string("timed step: ") + hipGetErrorString(e));
  *count = n;
  return CGKS_OK;
}

const char* cgks_kernel_name(const cgks_plan* p, int index) {
  if (!p || index < 0) return "";
  if (p->g.dim == 1) return index < 6 ? kKernels1d[index] : "";
  return index < 10 ? kKernels2d[index] : "";
}

cgks_status cgks_read_state(const cgks_plan* p, const void* d_state, const void* d_work, double* h_avg,
                            double* h_grad_x, double* h_grad_y, double* h_slope_x, double* h_slope_y,
                            double* h_sigma_x, double* h_sigma_y, double* h_time, long long* h_steps,
                            void* stream) {
  if (!p || !d_state || !d_work) return fail(CGKS_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const Geo& g = p->g;
  Bufs b = bufs(p, (void*)d_state, (void*)d_work);
  std::vector<double> hs(p->state_words), sx(p->sig_x_words), sy(p->sig_y_words);
  Header hh;
  HIP_TRY(hipMemcpyAsync(hs.data(), d_state, p->state_words * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(sx.data(), b.sxn, sx.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  if (g.dim == 2) HIP_TRY(hipMemcpyAsync(sy.data(), b.syn, sy.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&hh, b.hdr, sizeof(hh), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hh.magic != kMagic) return fail(CGKS_ESTATE, "work buffer was not initialised by cgks_init_state");
  const int nx = g.nx, ny = g.ny, m = g.m, nv = g.nv;
  const bool f64 = p->precision == CGKS_FP64;
  auto slope = [&](size_t k) -> double {
    return f64 ? slopes<double>(hs.data(), g)[k] : (double)slopes<float>(hs.data(), g)[k];
  };
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        if (h_avg) h_avg[((size_t)v * ny + j) * nx + i] = hs[g.avg(v, i, j)];
        for (int l = 0; l < m; ++l) {
          if (h_slope_x) h_slope_x[(((size_t)v * m + l) * ny + j) * nx + i] = slope(g.sx(v, l, i, j));
          if (g.dim == 2 && h_slope_y) h_slope_y[(((size_t)v * m + l) * ny + j) * nx + i] = slope(g.sy(v, l, i, j));
        }
        // cell-averaged gradients: Gauss-weighted means of the line slopes
        // (1-D: the stored slope itself)
        double gxs = 0.0, gys = 0.0;
        for (int l = 0; l < m; ++l) {
          const double w = g.dim == 2 ? kGw[m][l] : 1.0;
          gxs += w * slope(g.sx(v, l, i, j));
          if (g.dim == 2) gys += w * slope(g.sy(v, l, i, j));
        }
        if (h_grad_x) h_grad_x[((size_t)v * ny + j) * nx + i] = gxs;
        if (h_grad_y && g.dim == 2) h_grad_y[((size_t)v * ny + j) * nx + i] = gys;
      }
  if (h_sigma_x)
    for (int j = 0; j < ny; ++j)
      for (int F = 0; F <= nx; ++F) h_sigma_x[(size_t)j * (nx + 1) + F] = sx[g.sgx(j, F)];
  if (h_sigma_y && g.dim == 2)
    for (int G = 0; G <= ny; ++G)
      for (int i = 0; i < nx; ++i) h_sigma_y[(size_t)G * nx + i] = sy[g.sgy(i, G)];
  if (h_time) *h_time = hh.t;
  if (h_steps) *h_steps = (long long)hh.steps;
  if (hh.nonphysical) return fail(CGKS_ENONPHYSICAL, "nonphysical cell average");
  return CGKS_OK;
}

cgks_status cgks_query_health(const cgks_plan* p, const void* d_work, cgks_health* out, void* stream) {
  if (!p || !d_work || !out) return fail(CGKS_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  Header hh;
  const double* w = (const double*)d_work;
  HIP_TRY(hipMemcpyAsync(&hh, w + p->off_hdr, sizeof(hh), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hh.magic != kMagic) return fail(CGKS_ESTATE, "work buffer was not initialised by cgks_init_state");
  out->nonphysical = (long long)hh.nonphysical;
  out->fallbacks = (long long)hh.fallbacks;
  out->steps = (long long)hh.steps;
  // the device counts the branches below the scheme's order; the full
  // order's count is the rest of the reconstructions taken
  const Geo& g = p->g;
  const long long per_stage =
      g.dim == 2 ? 2ll * g.nx * g.ny * (1 + g.m) : (long long)g.nx + 2;
  out->recon_total = out->steps * 2 * per_stage;
  const long long ao = (long long)hh.rec_ao, l5 = (long long)hh.rec_lin5, l7 = (long long)hh.rec_lin7;
  const int order = p->C.order;
  out->ao_branch = ao;
  out->linear[0] = order == 5 ? out->recon_total - ao : l5;
  out->linear[1] = order == 7 ? out->recon_total - ao - l5 : (order == 9 ? l7 : 0);
  out->linear[2] = order == 9 ? out->recon_total - ao - l5 - l7 : 0;
  out->dff_lt1 = ao + (order > 5 ? l5 : 0) + (order > 7 ? l7 : 0);
  out->near_ties = (long long)hh.ties;
  if (hh.nonphysical) return fail(CGKS_ENONPHYSICAL, "nonphysical cell average");
  return CGKS_OK;
}

cgks_status cgks_conservation_sums_static(const cgks_plan* p, const void* d_state, double* d_sums, void* stream) {
  if (!p || !d_state || !d_sums) return fail(CGKS_EINVAL, "NULL argument");
  if (p->sum_blocks > kStaticSumBlocks)
    return fail(CGKS_EINVAL, "grid too large for the static scratch: at most " +
                                 std::to_string((long long)kStaticSumBlocks * SUM_CHUNK) + " interior cells");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CGKS_EINVAL, "device index out of range");
  void* ptr = nullptr;
  {
    // resolved once per device, with that device current
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* q = nullptr;
      HIP_TRY(hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)));
      if (!q) return fail(CGKS_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
      g_scratch_ptr[dev] = q;
    }
    ptr = g_scratch_ptr[dev];
  }
  // pass 1 writes every partial pass 2 reads: nothing needs clearing
  hipStream_t st = (hipStream_t)stream;
  DD* part = (DD*)ptr;
  hipLaunchKernelGGL(k_sum1, dim3(p->sum_blocks), dim3(256), 0, st, p->g, (const double*)d_state, part,
                     p->sum_blocks);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, st, p->g.nv, (const DD*)part, p->sum_blocks, d_sums);
  HIP_TRY(hipGetLastError());
  return CGKS_OK;
}

cgks_status cgks_conservation_sums(const cgks_plan* p, const void* d_state, void* d_work, double* d_sums,
                                   void* stream) {
  if (!p || !d_state || !d_work || !d_sums) return fail(CGKS_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  DD* part = (DD*)((double*)d_work + p->off_sum);
  hipLaunchKernelGGL(k_sum1, dim3(p->sum_blocks), dim3(256), 0, st, p->g, (const double*)d_state, part,
                     p->sum_blocks);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, st, p->g.nv, (const DD*)part, p->sum_blocks, d_sums);
  HIP_TRY(hipGetLastError());
  return CGKS_OK;
}

}  // extern "C"
