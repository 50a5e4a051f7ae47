// Internal header of libcgks.so: the types (header record, geometry, buffer
// set, plan) and the per-tile device bodies shared by the single-grid kernels
// (cgks.hip) and the batched persistent kernels (cgks_batch.hip).
//
// Data layout (FP64, structure of arrays, ghost halo of H = 3 cells):
//   state  = [avg: nv][NY][NX] [sx: nv][m][NY][NX] [sy: nv][m][NY][NX] (2-D)
//            1-D: NY = 1, m = 1, no sy.  Cell (i, j) sits at (j+H)*NX + i+H.
//   work   = [stage state U*][accumulator][sigx old/new][sigy old/new]
//            [line values LVx, LVy: nv][m][NY][NX] (2-D)][header]
//   sigx: [NY][NX+1], face F of row j at (j+H)*(NX+1) + F+H (1-D: one row)
//   sigy: [NX][NY+1], face G of column i at (i+H)*(NY+1) + G+H
//
// One step (Sec. 2.2): dt -> strengths commit + ghosts -> stage 1 (Eq. 2.21,
// slopes from W(dt/2)) -> ghosts of U* -> stage 2 (Eq. 2.22, 2.23; slopes from
// Eq. 2.25, 2.29, 2.30).  The stage-1 kernels also write the accumulator
//   Acc = W^n - (1/h) sum_l w_l [(8/3) F(dt/2) - (1/3) F(dt)],
//   Acc_slope = [-(4/3) W(0) + (8/3) W(dt/2) - (1/3) W(dt)] / h,
// so that stage 2 adds (4/3)[F*(dt) - 2 F*(dt/2)] and (4/3)[W*(0) - 2 W*(dt/2) + W*(dt)],
// which is Eq. 2.19-2.23 and 2.25/2.29 combined.
#pragma once
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/cgks.h"
#include "cgks_device.hpp"

using namespace cgks;

#define H 3

// Message of the last failing call on this thread (defined in cgks.hip).
extern thread_local std::string cgks_g_err;

namespace {

inline cgks_status fail(cgks_status s, const std::string& msg) {
  cgks_g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(CGKS_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// Scratch (private) bytes per thread a hot kernel may use.  FP64 face kernels
// compiled for two waves per SIMD spilled about 350 bytes per thread and then
// produced wrong, run-dependent results on gfx950, while the same source
// without spills is exact; every hot kernel is therefore built to keep its
// state in registers, and the library checks the built kernels before first
// use and refuses to run them otherwise (no hot kernel may use scratch).
inline cgks_status check_private(const void* kernel, size_t limit, const char* what) {
  hipFuncAttributes a;
  hipError_t e = hipFuncGetAttributes(&a, kernel);
  if (e != hipSuccess) return fail(CGKS_EHIP, std::string("hipFuncGetAttributes: ") + hipGetErrorString(e));
  if (a.localSizeBytes > limit)
    return fail(CGKS_EHIP, std::string(what) + " uses " + std::to_string(a.localSizeBytes) +
                               " bytes of scratch per thread (limit " + std::to_string(limit) + "): rebuild");
  return CGKS_OK;
}

struct Header {
  double t;
  double dt;
  double tn;       // start time of the current step (t before its dt was added)
  unsigned long long smax_bits;
  unsigned long long rmin_bits;
  unsigned long long steps;
  unsigned long long nonphysical;
  unsigned long long fallbacks;
  unsigned long long magic;
  int active;
  int nparts;      // per-block speed partials written by the last reduction
  // reconstructions (cell, line) by cascade branch below the scheme's order:
  // AO(5,3), linear 5th order (orders 7, 9), linear 7th order (order 9);
  // and cascade decisions taken within the tie band of the threshold
  unsigned long long rec_ao, rec_lin5, rec_lin7, ties;
  int pad[6];
};
static_assert(sizeof(Header) <= 256, "header");

// Segmented sides (and prescribed states), as the plan normalises them:
// segment k < nseg - 1 holds the ghost cells whose centre along the side is
// below end0[k] + speed[k] t; cons is a prescribed state in conservative
// variables.  Kept in the work buffer, so a job carries its own copy.
struct BcSide {
  int nseg;
  int type[3];
  double cons[3][4];
  double end0[3], speed[3];
};
struct BcTable {
  double x0, y0, dx, dy;   // cell centres: x0 + (i + 1/2) dx, y0 + (j + 1/2) dy
  double smax;             // largest |U| + c of the prescribed states (0: none)
  BcSide side[4];
};

// Per-job progress record of a batch, written by the dt phase each step.
struct JobStat {
  double t;
  double dt;
  long long steps;
  int status;   // 0 running, 1 finished (t_end or step limit), 2 nonphysical
  int active;
};
constexpr unsigned long long kMagic = 0x43474b5331ull;

// Geometry passed by value to every kernel.
struct Geo {
  int dim, nx, ny, NX, NY, m, nv;
  int bc[4];
  size_t cells;
  __host__ __device__ size_t cell(int i, int j) const {
    return (size_t)(dim == 2 ? j + H : 0) * NX + (i + H);
  }
  __host__ __device__ size_t avg(int v, int i, int j) const { return (size_t)v * cells + cell(i, j); }
  // A state is nv planes of cell averages (double) followed by its slope
  // planes: x-slopes [v][l], then (2-D) y-slopes [v][l].  The slopes are
  // stored in the working precision of the plan (double, or float in the
  // FP32-flux variant); sx and sy index them from the slope base
  // (slopes<ST>(U, g)), not from the start of the state.
  __host__ __device__ size_t sx(int v, int l, int i, int j) const {
    return ((size_t)v * m + l) * cells + cell(i, j);
  }
  __host__ __device__ size_t sy(int v, int l, int i, int j) const {
    return (size_t)nv * m * cells + ((size_t)v * m + l) * cells + cell(i, j);
  }
  __host__ __device__ size_t avg_words() const { return (size_t)nv * cells; }
  __host__ __device__ size_t slope_elems() const { return (size_t)nv * m * cells * (dim == 2 ? 2 : 1); }
  __host__ __device__ size_t lv(int v, int l, int i, int j) const { return ((size_t)v * m + l) * cells + cell(i, j); }
  __host__ __device__ size_t sgx(int j, int F) const { return (size_t)(dim == 2 ? j + H : 0) * (NX + 1) + F + H; }
  __host__ __device__ size_t sgy(int i, int G) const { return (size_t)(i + H) * (NY + 1) + G + H; }
};

struct Bufs {
  double* U;      // state (W^n, then W^{n+1})
  double* S;      // stage state W*
  double* A;      // accumulator
  double* sxo;    // strengths in use (previous step)
  double* sxn;    // strengths computed in this step
  double* syo;
  double* syn;
  double* lvx;    // Step 1 line values (element type: the plan's working precision)
  double* lvy;
  double* part;   // per-block [max(|U|+c), min(rho)] of the last reduction
  Header* hdr;
  const BcTable* bct;
};

// Pointers into device memory typed as such.  Kernel arguments are known to
// point to global memory, pointers read from memory (the batched job table)
// are not; loads and stores through the latter would be FLAT instructions,
// which also count against the LDS counter, so every wait for an LDS read
// would wait for the global accesses in flight as well.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> glb(T* p) {
  return (gptr<T>)p;
}

// The slope planes of a state whose averages start at U (element type ST).
template <typename ST>
__host__ __device__ __forceinline__ ST* slopes(double* U, const Geo& g) {
  return (ST*)(U + g.avg_words());
}
template <typename ST>
__host__ __device__ __forceinline__ const ST* slopes(const double* U, const Geo& g) {
  return (const ST*)(U + g.avg_words());
}

}  // namespace

struct cgks_plan {
  Geo g;
  Consts C;
  int precision;
  double dx, dy;
  size_t state_words, sig_x_words, sig_y_words;
  size_t off_S, off_A, off_sxo, off_sxn, off_syo, off_syn, off_lvx, off_lvy, off_part, off_hdr, off_bct, off_sum,
      work_words;
  size_t max_parts;
  int sum_blocks;  // blocks of the conservation-sum reduction (its partials sit at off_sum)
  BcTable bct;     // copied into the work buffer by cgks_init_state
};

namespace {

Bufs bufs(const cgks_plan* p, void* d_state, void* d_work) {
  Bufs b;
  double* w = (double*)d_work;
  b.U = (double*)d_state;
  b.S = w + p->off_S;
  b.A = w + p->off_A;
  b.sxo = w + p->off_sxo;
  b.sxn = w + p->off_sxn;
  b.syo = w + p->off_syo;
  b.syn = w + p->off_syn;
  b.lvx = w + p->off_lvx;
  b.lvy = w + p->off_lvy;
  b.part = w + p->off_part;
  b.hdr = (Header*)(w + p->off_hdr);
  b.bct = (const BcTable*)(w + p->off_bct);
  return b;
}

// ---------------------------------------------------------------------------
// boundary conditions (ghost cells and ghost faces)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int src_cell(int k, int n, int lo, int hi, int& mir) {
  mir = 0;
  if (k < 0) {
    if (lo == CGKS_BC_PERIODIC) return k + n;
    mir = 1;
    return -k - 1;
  }
  if (k >= n) {
    if (hi == CGKS_BC_PERIODIC) return k - n;
    mir = 1;
    return 2 * n - 1 - k;
  }
  return k;
}

__device__ __forceinline__ int src_face(int F, int n, int lo, int hi) {
  if (F < 0) return lo == CGKS_BC_PERIODIC ? F + n : -F;
  if (F > n) return hi == CGKS_BC_PERIODIC ? F - n : 2 * n - F;
  return F;
}

// Ghost cells mirror interior cells (transmissive, reflective) or wrap
// (periodic).  Mirrored: averages copied, the slope normal to the mirror
// negated, slopes along Gauss lines crossing the mirror taken at the mirrored
// Gauss point; a reflective wall also makes the normal momentum odd.
// Time the ghosts are filled for: 0 the initial state (t), 1 the first stage
// and the strengths (the step's start), 2 the second stage (start + dt/2).
__device__ __forceinline__ double bc_time(const Header* hdr, int code) {
  return code == 0 ? hdr->t : (code == 1 ? hdr->tn : hdr->tn + 0.5 * hdr->dt);
}

// Kind of side s for the ghosts whose centre along the side is c, at time
// t; a prescribed state is returned through cons.
__device__ __forceinline__ int side_kind(const Geo& g, const BcTable* T, int s, double c, double t,
                                         const double*& cons) {
  // selected, not indexed: a runtime index into a kernel's private copy of
  // the grid descriptor would put that copy in scratch memory
  const int b = s == 0 ? g.bc[0] : (s == 1 ? g.bc[1] : (s == 2 ? g.bc[2] : g.bc[3]));
  if (b != CGKS_BC_SEGMENTED) return b;
  const BcSide& S = T->side[s];
  int k = 0;
  while (k < S.nseg - 1 && !(c < S.end0[k] + S.speed[k] * t)) ++k;
  cons = S.cons[k];
  return S.type[k];
}

// Sign a wall gives component v of a mirrored ghost (normal momentum: nv_n).
__device__ __forceinline__ double wall_sign(int kind, int v, int nv_n, int D) {
  if (kind == CGKS_BC_REFLECTIVE) return v == nv_n ? -1.0 : 1.0;
  if (kind == CGKS_BC_NOSLIP) return (v >= 1 && v <= D) ? -1.0 : 1.0;
  return 1.0;
}

// Items of the ghost-cell fill: the 256-cell segments of the padded rows that
// hold ghost cells.  Every segment of the 2-D ghost rows (gr of them); of the
// other rows segment 0 and the segments r0..as-1 of the right-hand ghosts,
// which can straddle a segment boundary (sg segments per row).
struct GhostItems {
  int as, gr, r0, sg;
  __host__ __device__ explicit GhostItems(const Geo& g)
      : as((g.NX + 255) / 256), gr(g.dim == 2 ? 2 * H : 0), r0((g.NX - H) / 256 > 1 ? (g.NX - H) / 256 : 1),
        sg(as == 1 ? 1 : 1 + (as - r0)) {}
  __host__ __device__ int count(const Geo& g) const { return gr * as + (g.NY - gr) * sg; }
  // item k -> padded row Jr and the padded column I of this thread
  __device__ void at(const Geo& g, int k, int& I, int& Jr) const {
    int seg;
    if (k < gr * as) {
      const int q = k / as;
      Jr = q < H ? q : g.NY - 2 * H + q;
      seg = k % as;
    } else {
      k -= gr * as;
      const int idx = k % sg;
      Jr = (gr ? H : 0) + k / sg;
      seg = idx == 0 ? 0 : r0 + idx - 1;
    }
    I = seg * 256 + (int)threadIdx.x;
  }
};

// Ghost cell (I, J) (padded indices) at time tb.  A ghost row of a y-side
// takes that side's rule at the column's centre; its source cell, or an
// x-ghost of an interior row, takes the x-side rule at the row's centre
// (corners compose both).  Mirrored ghosts copy the averages, negate the
// normal slope and reverse the order of the tangential line slopes; walls
// add their momentum signs.  A prescribed state gives that state and zero
// slopes.
template <typename ST>
__device__ __forceinline__ void bc_state_at(const Geo& g, const BcTable* T, double tb, double* U, int I, int J) {
  if (I >= g.NX) return;
  const int i = I - H, j = (g.dim == 2) ? J - H : 0;
  const bool gx = (i < 0 || i >= g.nx), gy = (g.dim == 2) && (j < 0 || j >= g.ny);
  if (!gx && !gy) return;
  const double* cons = nullptr;
  int my = 0, sj = j, ky = CGKS_BC_PERIODIC;
  if (gy) {
    ky = side_kind(g, T, j < 0 ? 2 : 3, T->x0 + (i + 0.5) * T->dx, tb, cons);
    if (ky != CGKS_BC_INFLOW) sj = src_cell(j, g.ny, g.bc[2], g.bc[3], my);
  }
  int mx = 0, si = i, kx = CGKS_BC_PERIODIC;
  if (ky != CGKS_BC_INFLOW && gx) {
    kx = side_kind(g, T, i < 0 ? 0 : 1, g.dim == 2 ? T->y0 + (sj + 0.5) * T->dy : 0.0, tb, cons);
    if (kx != CGKS_BC_INFLOW) si = src_cell(i, g.nx, g.bc[0], g.bc[1], mx);
  }
  const bool fixed = ky == CGKS_BC_INFLOW || kx == CGKS_BC_INFLOW;
  ST* S = slopes<ST>(U, g);
  for (int v = 0; v < g.nv; ++v) {
    const double odd = (mx ? wall_sign(kx, v, 1, g.dim) : 1.0) * (my ? wall_sign(ky, v, 2, g.dim) : 1.0);
    if (fixed) {   // a prescribed state, seen through a y-mirror when the x-side prescribes it
      U[g.avg(v, i, j)] = odd * cons[v];
      for (int l = 0; l < g.m; ++l) {
        S[g.sx(v, l, i, j)] = ST(0);
        if (g.dim == 2) S[g.sy(v, l, i, j)] = ST(0);
      }
      continue;
    }
    U[g.avg(v, i, j)] = odd * U[g.avg(v, si, sj)];
    // the signs are +-1: the products are exact in either storage type
    for (int l = 0; l < g.m; ++l) {
      const int lx = my ? g.m - 1 - l : l;   // x-slope lines are horizontal: mirrored by a y-mirror
      S[g.sx(v, l, i, j)] = ST(mx ? -odd : odd) * S[g.sx(v, lx, si, sj)];
      if (g.dim == 2) {
        const int ly = mx ? g.m - 1 - l : l;
        S[g.sy(v, l, i, j)] = ST(my ? -odd : odd) * S[g.sy(v, ly, si, sj)];
      }
    }
  }
}


// Commit the strengths computed in the previous step (new -> old) and fill
// the ghost faces and ghost rows/columns of the old set at time tb.  Faces
// beyond a prescribed state are zero (its ghosts are uniform); in a ghost row
// (column) a face is judged by the cell that starts at it.
__device__ __forceinline__ void bc_sigma_at(const Geo& g, const BcTable* T, double tb, int which,
                                            const double* sxn, double* sxo, const double* syn, double* syo,
                                            int a, int b) {
  const double* cons = nullptr;
  if (which == 0) {
    // x-faces: a = F + H in [0, NX], b = row J
    if (a > g.NX) return;
    const int F = a - H, j = (g.dim == 2) ? b - H : 0;
    int my = 0, sj = j;
    if (g.dim == 2 && (j < 0 || j >= g.ny)) {
      if (side_kind(g, T, j < 0 ? 2 : 3, T->x0 + (F + 0.5) * T->dx, tb, cons) == CGKS_BC_INFLOW) {
        sxo[g.sgx(j, F)] = 0.0;
        return;
      }
      sj = src_cell(j, g.ny, g.bc[2], g.bc[3], my);
    }
    int sF = F;
    if (F < 0 || F > g.nx) {
      if (side_kind(g, T, F < 0 ? 0 : 1, g.dim == 2 ? T->y0 + (sj + 0.5) * T->dy : 0.0, tb, cons) ==
          CGKS_BC_INFLOW) {
        sxo[g.sgx(j, F)] = 0.0;
        return;
      }
      sF = src_face(F, g.nx, g.bc[0], g.bc[1]);
    }
    sxo[g.sgx(j, F)] = sxn[g.sgx(sj, sF)];
  } else {
    // y-faces: a = G + H in [0, NY], b = column I
    if (a > g.NY) return;
    const int G = a - H, i = b - H;
    int mx = 0, si = i;
    if (i < 0 || i >= g.nx) {
      if (side_kind(g, T, i < 0 ? 0 : 1, T->y0 + (G + 0.5) * T->dy, tb, cons) == CGKS_BC_INFLOW) {
        syo[g.sgy(i, G)] = 0.0;
        return;
      }
      si = src_cell(i, g.nx, g.bc[0], g.bc[1], mx);
    }
    int sG = G;
    if (G < 0 || G > g.ny) {
      if (side_kind(g, T, G < 0 ? 2 : 3, T->x0 + (si + 0.5) * T->dx, tb, cons) == CGKS_BC_INFLOW) {
        syo[g.sgy(i, G)] = 0.0;
        return;
      }
      sG = src_face(G, g.ny, g.bc[2], g.bc[3]);
    }
    syo[g.sgy(i, G)] = syn[g.sgy(si, sG)];
  }
}


__device__ __forceinline__ double sigma_pair(const double* Wl, const double* Wr, int D, double gam) {
  auto pr = [&](const double* W) {
    double ke = 0.5 * W[1] * W[1] / W[0];
    if (D == 2) ke += 0.5 * W[2] * W[2] / W[0];
    return (gam - 1.0) * (W[D + 1] - ke);
  };
  const double pl = pr(Wl), pp = pr(Wr);
  const double cl = sqrt(gam * pl / Wl[0]), cr = sqrt(gam * pp / Wr[0]);
  const double dp = fabs(pl - pp);
  const double mn = Wl[1] / Wl[0] / cl - Wr[1] / Wr[0] / cr;
  const double mt = (D == 2) ? Wl[2] / Wl[0] / cl - Wr[2] / Wr[0] / cr : 0.0;
  return dp / pl + dp / pp + mn * mn + mt * mt;
}


// ---------------------------------------------------------------------------
// Health tally of a tile's reconstructions.  Each wave counts, by ballot, the
// reconstructions it owns that took a cascade branch below the scheme's
// order, and the near ties, into LDS; one thread then adds the tile's
// nonzero counts to the header.  Reconstructions of the full order are not
// counted: their number follows from the reconstructions per step, so
// smooth tiles issue no global atomics.  Every tile reconstructs its halo
// cells too; only the cells and lines the tile updates are its own, so each
// reconstruction of the grid is counted once.
// ---------------------------------------------------------------------------
struct Tally {
  unsigned int c[4];   // AO(5,3), linear 5, linear 7, near ties
};

// before the first tally_add of a tile, separated from it by a barrier
__device__ __forceinline__ void tally_zero(Tally& t, int tid) {
  if (tid < 4) t.c[tid] = 0u;
}

// called by every lane of the block (ballots are per wave)
__device__ __forceinline__ void tally_add(Tally& t, bool own, int branch, bool tie, int order, int tid) {
  const unsigned long long m0 = __ballot(own && branch == 0);
  const unsigned long long m5 = __ballot(own && branch == 5 && order > 5);
  const unsigned long long m7 = __ballot(own && branch == 7 && order > 7);
  const unsigned long long mt = __ballot(own && tie);
  if ((tid & 63) == 0) {
    if (m0) atomicAdd(&t.c[0], (unsigned int)__popcll(m0));
    if (m5) atomicAdd(&t.c[1], (unsigned int)__popcll(m5));
    if (m7) atomicAdd(&t.c[2], (unsigned int)__popcll(m7));
    if (mt) atomicAdd(&t.c[3], (unsigned int)__popcll(mt));
  }
}

// after a barrier that follows the last tally_add of the tile
__device__ __forceinline__ void tally_flush(const Tally& t, Header* hdr, int tid) {
  if (tid == 0) {
    const unsigned int a = t.c[0], b = t.c[1], c = t.c[2], d = t.c[3];
    if (a) atomicAdd(&hdr->rec_ao, (unsigned long long)a);
    if (b) atomicAdd(&hdr->rec_lin5, (unsigned long long)b);
    if (c) atomicAdd(&hdr->rec_lin7, (unsigned long long)c);
    if (d) atomicAdd(&hdr->ties, (unsigned long long)d);
  }
}


// ---------------------------------------------------------------------------
// time step (Sec. 4): reduction of max(|U| + c) and min(rho), then dt
// ---------------------------------------------------------------------------
// Block-level max(|U| + c) and min(rho); thread 0 writes the block's partial
// (reduced by k_dt before the next step).  Called by every thread of the block.
struct SpeedRed {
  double v[2][4];   // per wave of a block of at most 256 threads
};
__device__ __forceinline__ void reduce_speed(const Bufs& B, double s, double r, bool valid, int bid, int nparts) {
  __shared__ SpeedRed red;
  double sm = valid ? s : 0.0;
  double rm = valid ? r : INFINITY;
  for (int off = 32; off > 0; off >>= 1) {
    sm = fmax(sm, __shfl_xor(sm, off, 64));
    rm = fmin(rm, __shfl_xor(rm, off, 64));
  }
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) { red.v[0][w] = sm; red.v[1][w] = rm; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < nw; ++k) { sm = fmax(sm, red.v[0][k]); rm = fmin(rm, red.v[1][k]); }
    const gptr<double> part = glb(B.part);
    part[2 * bid] = sm;
    part[2 * bid + 1] = rm;
    if (bid == 0) glb(B.hdr)->nparts = nparts;
  }
}

__device__ __forceinline__ bool cell_speed(const double* W, int D, double gam, double& s) {
  const double r = W[0];
  const double U = W[1] / r, V = (D == 2) ? W[2] / r : 0.0;
  const double p = (gam - 1.0) * (W[D + 1] - 0.5 * r * (U * U + V * V));
  const bool ok = (r > 0.0) && (p > 0.0) && isfinite(W[D + 1]);
  s = ok ? sqrt(U * U + V * V) + sqrt(gam * p / r) : 0.0;
  return ok;
}


// One block: reduce the speed partials, then dt, the active flag, time and
// step count; max_steps > 0 stops the run after that many steps.  The
// optional progress record gets t, dt, steps and the status.
// sbc: largest |U| + c of prescribed boundary states, which enter through
// the boundary faces every step and so bound the step like the cells do.
__device__ void dt_block(Header* hdr, const double* part, double sbc, double dt_fixed, double cfl, double t_end, double h,
                         double mu, int viscous, long long max_steps, JobStat* stat) {
  __shared__ double red[2][256];
  __syncthreads();
  const int np = hdr->nparts;
  // eight (speed, rate) pairs in flight per lane; max and min are exact, so
  // the order of the reduction does not matter
  constexpr int UR = 8;
  const int bd = blockDim.x;
  double smu[UR], rmu[UR];
#pragma unroll
  for (int u = 0; u < UR; ++u) { smu[u] = 0.0; rmu[u] = INFINITY; }
  int k = threadIdx.x;
  for (; k + (UR - 1) * bd < np; k += UR * bd) {
    double2 q[UR];
#pragma unroll
    for (int u = 0; u < UR; ++u) q[u] = ((const double2*)part)[k + u * bd];
#pragma unroll
    for (int u = 0; u < UR; ++u) { smu[u] = fmax(smu[u], q[u].x); rmu[u] = fmin(rmu[u], q[u].y); }
  }
  for (; k < np; k += bd) {
    const double2 q = ((const double2*)part)[k];
    smu[0] = fmax(smu[0], q.x);
    rmu[0] = fmin(rmu[0], q.y);
  }
  double sm = smu[0], rm = rmu[0];
#pragma unroll
  for (int u = 1; u < UR; ++u) { sm = fmax(sm, smu[u]); rm = fmin(rm, rmu[u]); }
  red[0][threadIdx.x] = sm;
  red[1][threadIdx.x] = rm;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
      red[1][threadIdx.x] = fmin(red[1][threadIdx.x], red[1][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double dt = dt_fixed;
  if (!(dt > 0.0)) {
    dt = cfl * h / fmax(red[0][0], sbc);
    if (viscous && mu > 0.0) {
      const double dv = cfl * h * h * red[1][0] / (4.0 * mu);
      if (dv < dt) dt = dv;
    }
  }
  int active = 1;
  if (hdr->nonphysical) { active = 0; dt = 0.0; }   // sticky: a nonphysical state stops the run
  else if (max_steps > 0 && (long long)hdr->steps >= max_steps) { active = 0; dt = 0.0; }
  else if (t_end > 0.0) {
    if (hdr->t >= t_end) { active = 0; dt = 0.0; }
    else if (hdr->t + dt > t_end) dt = t_end - hdr->t;
  }
  hdr->dt = dt;
  hdr->active = active;
  hdr->tn = hdr->t;   // the step's start: boundary data of its stages are taken at tn and tn + dt/2
  if (active) {
    hdr->t += dt;
    hdr->steps += 1;
  }
  if (stat) {
    // finished once no further step will be taken: the step enqueued now is
    // the last one when it reaches the step limit or t_end
    const bool last = (max_steps > 0 && (long long)hdr->steps >= max_steps) || (t_end > 0.0 && hdr->t >= t_end);
    stat->t = hdr->t;
    stat->dt = dt;
    stat->steps = (long long)hdr->steps;
    stat->status = hdr->nonphysical ? 2 : ((active && !last) ? 0 : 1);
    stat->active = active;
  }
}


// ---------------------------------------------------------------------------
// Conservation totals: sum over the interior cells of each conserved
// variable in a fixed order, with compensated (double-double) partial sums.
// Block b of the first pass takes the interior cells b*SUM_CHUNK .. (b+1)*
// SUM_CHUNK - 1 in row-major order, each thread every 256th of them in
// ascending order; the block's partials are combined by a fixed pairwise
// tree.  The second pass, one block, combines the block partials the same
// way.  The order depends only on the grid size, so results are bitwise
// reproducible.
// ---------------------------------------------------------------------------
constexpr int SUM_CHUNK = 256 * 64;   // interior cells per block of the first pass

struct DD {
  double hi, lo;
};
// error-free sum of two doubles (Knuth's TwoSum), then renormalised
__device__ __forceinline__ DD dd_add(DD a, DD b) {
  const double s = a.hi + b.hi;
  const double bb = s - a.hi;
  const double e = (a.hi - (s - bb)) + (b.hi - bb);
  const double lo = e + a.lo + b.lo;
  const double hi = s + lo;
  return DD{hi, lo - (hi - s)};
}

// 256 threads; part[v * nblk + b] receives block b's partial of variable v
__device__ __forceinline__ void sums_pass1(const Geo& g, const double* U, DD* part, int nblk, int b) {
  __shared__ DD red[256];
  const gptr<const double> Ug = glb(U);
  const long long nint = (long long)g.nx * (g.dim == 2 ? g.ny : 1);
  const long long k0 = (long long)b * SUM_CHUNK;
  const long long k1 = k0 + SUM_CHUNK < nint ? k0 + SUM_CHUNK : nint;
  const int t = threadIdx.x;
  for (int v = 0; v < g.nv; ++v) {
    DD acc{0.0, 0.0};
    for (long long k = k0 + t; k < k1; k += 256) {
      const int i = (int)(k % g.nx), j = (int)(k / g.nx);
      acc = dd_add(acc, DD{Ug[g.avg(v, i, j)], 0.0});
    }
    red[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) red[t] = dd_add(red[t], red[t + w]);
      __syncthreads();
    }
    if (t == 0) part[(size_t)v * nblk + b] = red[0];
    __syncthreads();
  }
}

__device__ __forceinline__ void sums_pass2(int nv, const DD* part, int nblk, double* out) {
  __shared__ DD red[256];
  const int t = threadIdx.x;
  for (int v = 0; v < nv; ++v) {
    DD acc{0.0, 0.0};
    for (int k = t; k < nblk; k += 256) acc = dd_add(acc, part[(size_t)v * nblk + k]);
    red[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) red[t] = dd_add(red[t], red[t + w]);
      __syncthreads();
    }
    if (t == 0) out[v] = red[0].hi + red[0].lo;
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// 2-D Step 1 (Sec. 3.3): tangential ASE-DFF in each column (row) gives the
// line averages of the cell on the horizontal (vertical) Gauss lines.
// ---------------------------------------------------------------------------
// The thread index as a value the compiler cannot prove loop-invariant.  In
// the persistent batched kernels a tile body sits inside the job loop; with
// the plain index the compiler hoists every lane decomposition of the tile
// out of that loop and holds it in registers through all phases.  The empty
// asm statement emits no instruction.
__device__ __forceinline__ int tile_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
// tile_tid for a block of 256 threads, with the range the compiler knows of
// threadIdx.x there (without it, LDS addresses derived from the index lose
// their immediate offsets)
__device__ __forceinline__ int tile_tid256() {
  const int t = tile_tid();
  __builtin_assume(t >= 0 && t < 256);
  return t;
}

// a value the compiler must take as new at this point, so that it does not
// keep what it derived from the value earlier live until here
__device__ __forceinline__ double fresh(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Step 1 over a tile of LT_X x LT_Y cells (x fastest; block of 256 threads,
// one cell each) with its inputs staged in LDS: the cell averages on the
// tile and a border of two cells, the cell-averaged normal gradients (line
// slopes weighted by the Gauss weights) on the strips each stencil direction
// reads, and the strengths of the faces the cascades use.  Every input is
// loaded once per tile, and the gradient means are formed once per cell
// rather than once per use (with the same operations in the same order as
// forming them at each use, so the results do not depend on the tiling).
// Tile shapes (LW): 0 = 32 x 8 cells (the single-grid shape), 1 = 16 x 16
// (fewer halo cells along x, shorter rows); the batched path's autotuner
// picks one.  Results do not depend on the shape.
constexpr int kLineTiles = 2;
template <int LW = 0> struct LinesLds {
  static constexpr int X = LW == 0 ? 32 : 16, Y = LW == 0 ? 8 : 16;
  static constexpr int BX = X + 4, BY = Y + 4;
  static constexpr int NAVG = 4 * BY * BX;        // averages [v][BY][BX], cells (i0-2+xx, j0-2+yy)
  static constexpr int NGY = 4 * BY * X;          // y-gradient means [v][BY][X], cells (i0+xx, j0-2+yy)
  static constexpr int NGX = 4 * Y * BX;          // x-gradient means [v][Y][BX], cells (i0-2+xx, j0+yy)
  static constexpr int SYN = Y + 5, SXN = X + 5;
  static constexpr int NSY = X * SYN;             // y-face strengths [xx][gg], face j0-2+gg of column i0+xx
  static constexpr int NSX = Y * SXN;             // x-face strengths [yy][ff], face i0-2+ff of row j0+yy
  static constexpr int total = NAVG + NGY + NGX + NSY + NSX;   // doubles
  static_assert(X * Y == 256, "one cell per thread");
};
constexpr int LT_X = LinesLds<0>::X, LT_Y = LinesLds<0>::Y;   // the single-grid shape
inline int line_tile_x(int lw) { return lw == 0 ? 32 : 16; }
inline int line_tile_y(int lw) { return lw == 0 ? 8 : 16; }

// ST: storage type of the slopes and line values (the plan's working
// precision); the arithmetic is double in both variants.
template <int M, typename ST, bool PERSIST = false, int LW = 0>
__device__ __forceinline__ void lines_tile(const Geo& g, const Consts& C, const double* U, const double* sxo,
                                           const double* syo, double* lvx, double* lvy, Header* hdr, int bx,
                                           int by, double* sm) {
  using L = LinesLds<LW>;
  constexpr int LT_X = L::X, LT_Y = L::Y;
  __shared__ Tally tally;
  const gptr<const double> Ug = glb(U), sxg = glb(sxo), syg = glb(syo);
  const gptr<const ST> Sl = glb(slopes<ST>(U, g));
  const gptr<ST> lvxg = glb((ST*)lvx), lvyg = glb((ST*)lvy);
  double* avg = sm;
  double* gy = avg + L::NAVG;
  double* gx = gy + L::NGY;
  double* sy = gx + L::NGX;
  double* sx = sy + L::NSY;
  __syncthreads();   // a persistent caller's previous tile has finished with the LDS
  const int i0 = -H + bx * LT_X, j0 = -H + by * LT_Y;
  // persistent FP32 callers: the opaque index with its range (FP64 keeps
  // the unranged one, the code of its batched kernels as tested)
  const int tid = PERSIST ? (sizeof(ST) == 4 ? tile_tid256() : tile_tid()) : (int)threadIdx.x;
  tally_zero(tally, tid);
  auto ci = [&](int i) { return i < -H ? -H : (i > g.nx + H - 1 ? g.nx + H - 1 : i); };
  auto cj = [&](int j) { return j < -H ? -H : (j > g.ny + H - 1 ? g.ny + H - 1 : j); };
  double wq[4];
#pragma unroll
  for (int l = 0; l < M; ++l) wq[l] = kGw[M][l];
  // staging (entries outside the stored grid are clamped into it; no cell
  // that computes line values reads them).  Each array's loads are issued
  // together (fixed pass counts; lanes past the end load a valid entry and
  // store nothing), then written to LDS.
  constexpr int PA = (L::NAVG + 255) / 256, PGY = (L::NGY + 255) / 256, PGX = (L::NGX + 255) / 256;
  constexpr int PSY = (L::NSY + 255) / 256, PSX = (L::NSX + 255) / 256;
  {
    double ra[PA];
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int k = tid + 256 * p < L::NAVG ? tid + 256 * p : L::NAVG - 1;
      const int v = k / (L::BY * L::BX), xx = k % L::BX, yy = (k / L::BX) % L::BY;
      ra[p] = Ug[g.avg(v, ci(i0 - 2 + xx), cj(j0 - 2 + yy))];
    }
#pragma unroll
    for (int p = 0; p < PA; ++p)
      if (tid + 256 * p < L::NAVG) avg[tid + 256 * p] = ra[p];
  }
  {
    double ra[PGY][4];
#pragma unroll
    for (int p = 0; p < PGY; ++p) {
      const int k = tid + 256 * p < L::NGY ? tid + 256 * p : L::NGY - 1;
      const int v = k / (L::BY * LT_X), xx = k % LT_X, yy = (k / LT_X) % L::BY;
      const int i = ci(i0 + xx), j = cj(j0 - 2 + yy);
#pragma unroll
      for (int l = 0; l < M; ++l) ra[p][l] = double(Sl[g.sy(v, l, i, j)]);
    }
#pragma unroll
    for (int p = 0; p < PGY; ++p) {
      double a = 0.0;
#pragma unroll
      for (int l = 0; l < M; ++l) a += wq[l] * ra[p][l];
      if (tid + 256 * p < L::NGY) gy[tid + 256 * p] = a;
    }
  }
  {
    double ra[PGX][4];
    double rs[PSY], rt[PSX];
#pragma unroll
    for (int p = 0; p < PGX; ++p) {
      const int k = tid + 256 * p < L::NGX ? tid + 256 * p : L::NGX - 1;
      const int v = k / (LT_Y * L::BX), xx = k % L::BX, yy = (k / L::BX) % LT_Y;
      const int i = ci(i0 - 2 + xx), j = cj(j0 + yy);
#pragma unroll
      for (int l = 0; l < M; ++l) ra[p][l] = double(Sl[g.sx(v, l, i, j)]);
    }
#pragma unroll
    for (int p = 0; p < PSY; ++p) {   // faces contiguous in memory along gg
      const int k = tid + 256 * p < L::NSY ? tid + 256 * p : L::NSY - 1;
      const int gg = k % L::SYN, xx = k / L::SYN;
      const int G = j0 - 2 + gg;
      rs[p] = syg[g.sgy(ci(i0 + xx), G < -H ? -H : (G > g.ny + H ? g.ny + H : G))];
    }
#pragma unroll
    for (int p = 0; p < PSX; ++p) {
      const int k = tid + 256 * p < L::NSX ? tid + 256 * p : L::NSX - 1;
      const int ff = k % L::SXN, yy = k / L::SXN;
      const int F = i0 - 2 + ff;
      rt[p] = sxg[g.sgx(cj(j0 + yy), F < -H ? -H : (F > g.nx + H ? g.nx + H : F))];
    }
#pragma unroll
    for (int p = 0; p < PGX; ++p) {
      double a = 0.0;
#pragma unroll
      for (int l = 0; l < M; ++l) a += wq[l] * ra[p][l];
      if (tid + 256 * p < L::NGX) gx[tid + 256 * p] = a;
    }
#pragma unroll
    for (int p = 0; p < PSY; ++p)
      if (tid + 256 * p < L::NSY) sy[tid + 256 * p] = rs[p];
#pragma unroll
    for (int p = 0; p < PSX; ++p)
      if (tid + 256 * p < L::NSX) sx[tid + 256 * p] = rt[p];
  }
  __syncthreads();
  const int xx = tid % LT_X, yy = tid / LT_X;
  const int i = i0 + xx, j = j0 + yy;
  // the tile's own cells (health tally): interior cells of the tile
  const bool interior = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
  int brx = 9, bry = 9;
  bool tiex = false, tiey = false;
  // x-face line values: column i, rows j-2..j+2, needed for j in [-1, ny]
  if (i <= g.nx + 2 && j >= -1 && j <= g.ny) {
    double d[4][9], s[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) s[f] = sy[xx * L::SYN + yy + f];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int k = 0; k < 5; ++k) d[v][k] = avg[(v * L::BY + yy + k) * L::BX + xx + 2];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int o = k < 2 ? k - 2 : k - 1;
        d[v][5 + k] = C.dy * gy[(v * L::BY + yy + 2 + o) * LT_X + xx];
      }
    }
    const Cascade cs = cascade(s, C.order, C.thres, C.tie);
    brx = cs.branch;
    tiex = cs.tie;
    double out[4][4];
    recon_nodes<double, 4, M>(d, cs, C, out);
#pragma unroll
    for (int l = 0; l < M; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) lvxg[g.lv(v, l, i, j)] = ST(out[l][v]);
  }
  // y-face line values: row j, columns i-2..i+2, needed for i in [-1, nx]
  if (i >= -1 && i <= g.nx && j <= g.ny + 2) {
    double d[4][9], s[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) s[f] = sx[yy * L::SXN + xx + f];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int k = 0; k < 5; ++k) d[v][k] = avg[(v * L::BY + yy + 2) * L::BX + xx + k];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int o = k < 2 ? k - 2 : k - 1;
        d[v][5 + k] = C.dx * gx[(v * LT_Y + yy) * L::BX + xx + 2 + o];
      }
    }
    const Cascade cs = cascade(s, C.order, C.thres, C.tie);
    bry = cs.branch;
    tiey = cs.tie;
    double out[4][4];
    recon_nodes<double, 4, M>(d, cs, C, out);
#pragma unroll
    for (int l = 0; l < M; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) lvyg[g.lv(v, l, i, j)] = ST(out[l][v]);
  }
  tally_add(tally, interior, brx, tiex, C.order, tid);
  tally_add(tally, interior, bry, tiey, C.order, tid);
  __syncthreads();
  tally_flush(tally, hdr, tid);
}


// ---------------------------------------------------------------------------
// 2-D face kernel: Step 2 (normal ASE-DFF on every Gauss line), Step 3
// (tangential derivatives), Step 4 (flux), and the cell update of one
// direction.  DIR 0: x-faces (normal x), DIR 1: y-faces.
// ---------------------------------------------------------------------------
// Wave-uniform execution.  On gfx950, FP64 kernels that spill (to scratch,
// accumulation registers or SGPR lanes) gave wrong results where the lanes of
// a wave were partly inactive (loop tails, ragged tile edges), while the same
// source executed on the CPU is exact.  The heavy phases of the face tile and
// of the 1-D stage therefore run on all lanes: a lane without an item of its
// own recomputes a valid one and only its stores are masked.
// Tile shapes (V): 0 = 16 faces x NT lines (the single-grid shape), 1 = 32 x
// NT/2 (fewer seam faces computed twice, more halo lines), 2 = 8 x 2 NT
// (fewer halo lines, more seam faces).  The batched kernels take any of them
// (chosen by the batch autotuner); the arithmetic of every face and cell is
// the same in all of them.
constexpr int kFaceTiles = 3;
template <int M, int V = 0> struct Tile {
  static constexpr int NF = V == 1 ? 32 : (V == 2 ? 8 : 16);  // faces along the normal
  static constexpr int NT = V == 0 ? (M == 2 ? 8 : (M == 3 ? 5 : 4))
                          : (V == 1 ? (M == 2 ? 4 : 2) : (M == 2 ? 16 : (M == 3 ? 10 : 8)));  // lines
  static constexpr int NC = NF + 1;                           // reconstructed cells
  static constexpr int NR = NT + 2;                           // reconstructed lines
  static constexpr int RK1 = 17, RK2 = 8;                     // results per Gauss point (stage 1 / 2)
  static_assert(NF * NT * M <= 256, "one Gauss point per thread");
};
// tiles of one direction of an nn (normal) x nt (tangential) grid
__host__ __device__ inline int face_tiles_n(int nn, int nf) { return (nn + nf - 2) / (nf - 1); }
__host__ __device__ inline int face_tiles_t(int nt, int nlines) { return (nt + nlines - 1) / nlines; }
inline int tile_nf(int v) { return v == 1 ? 32 : (v == 2 ? 8 : 16); }
inline int tile_nt(int v, int m) {
  return v == 0 ? (m == 2 ? 8 : (m == 3 ? 5 : 4)) : (v == 1 ? (m == 2 ? 4 : 2) : (m == 2 ? 16 : (m == 3 ? 10 : 8)));
}

// LDS of a face tile, laid out by lifetime (barriers B1..B4 of the tile):
//   staging  Step 2 inputs: line values and h-scaled normal slopes of the
//            cells n = F0-3 .. F0+NF+1 on the NR lines (element type T),
//            then the normal strengths of faces F0-3 .. F0+NF+2 (double);
//            written before B1, read in Step 2 (before B2);
//   recon    Step 2 results: one record of RS = 8M + 1 elements per (line,
//            cell) -- the odd stride puts neighbouring lanes on different
//            banks; written in Step 2, read in Step 3 (before B3);
//   atab     tangential DFF factors of the Step 3 states; written before B1,
//            read in Step 3;
//   res      Gauss-point results, structure of arrays (component k of Gauss
//            point g at k * NB + g, so lane g of a wave writes consecutive
//            words); written after B3, read in the cell update (after B4);
//   fin      updated averages of the tile (y-faces), written after B4.
// recon | staging | atab, with res and then fin over recon and staging,
// which are dead once B3 has passed.
// smallest stride >= n with stride mod 32 = 16 (two lines of 16 lanes on
// disjoint bank halves), for the shapes whose strides were not enumerated
constexpr int stride16(int n) { return n + (48 - n % 32) % 32; }
template <int M, typename T, int V = 0, int D = -1, bool OCC3 = false> struct Lds {
  using TL = Tile<M, V>;
  static constexpr int RS = 8 * M + 1;
  // Step 2 records of (line r, cell c): x-faces row-major, r RW + c RS;
  // y-faces cell-major, c CS + r RS.  A group of lanes that the LDS serves
  // together (16 for 64-bit, 32 for 32-bit words) holds up to two lines and
  // 16 cells on x-faces, and several lines and cells on y-faces; the padded
  // strides RW and CS put every lane of such a group on its own bank in
  // Step 3 (found by enumerating strides against the lane layout).  The
  // second-derivative records (NT lines) use RW and cell stride CSD.
  // D: the records of one direction only (0 x-faces, 1 y-faces; -1 both,
  // for kernels that serve both from one LDS size).  OCC3: the tile runs
  // three blocks per CU; at M = 4 its records then stay unpadded, since the
  // padded stride would push the tile past a third of the LDS, and the
  // third block is worth more than the conflicts the padding removes.
  static constexpr bool PAD = V == 0 && !(OCC3 && M == 4);
  static constexpr int RW = PAD ? (M == 2 ? 304 : (M == 3 ? 432 : 592)) : (V == 0 ? TL::NC * RS : stride16(TL::NC * RS));
  static constexpr int CS = PAD ? (M == 2 ? 200 : (M == 3 ? 189 : 204)) : (TL::NR * RS) | 1;
  static constexpr int CSD = TL::NT * RS;
  static_assert(RW >= TL::NC * RS && CS >= TL::NR * RS, "records do not overlap");
  static constexpr int NCS = TL::NC + 4, NSG = TL::NC + 5;
  static constexpr int NSTV = 4 * M * TL::NR * NCS;   // per staged array
  static constexpr size_t a8(size_t x) { return (x + 7) / 8 * 8; }
  static constexpr size_t mx(size_t a, size_t b) { return a > b ? a : b; }
  static constexpr size_t XW = D == 1 ? 0 : (size_t)TL::NR * RW, YW = D == 0 ? 0 : (size_t)TL::NC * CS;
  static constexpr size_t XD = D == 1 ? 0 : (size_t)TL::NT * RW, YD = D == 0 ? 0 : (size_t)TL::NC * CSD;
  static constexpr size_t s2v = mx(XW, YW) * sizeof(T);
  static constexpr size_t s2d = s2v;
  static constexpr size_t s2dd = mx(XD, YD) * sizeof(T);
  static constexpr size_t recon = a8(s2v + s2d + s2dd);
  static constexpr size_t st_sg = a8(2 * NSTV * sizeof(T));          // offset of the strengths in staging
  static constexpr size_t staging = st_sg + (size_t)TL::NR * NSG * sizeof(double);
  static constexpr size_t res = (size_t)TL::NF * TL::NT * M * TL::RK1 * sizeof(double);
  static constexpr size_t fin = (size_t)(TL::NF - 1) * TL::NT * 4 * sizeof(double);
  static constexpr size_t off_staging = recon;
  static constexpr size_t off_res = 0;
  static constexpr size_t off_fin = res;
  static constexpr size_t body = recon + staging > res + fin ? recon + staging : res + fin;
  static constexpr size_t off_atab = a8(body);
  static constexpr size_t total = off_atab + (size_t)TL::NC * TL::NT * sizeof(T);
};

// Waves per SIMD the single-grid face kernels are compiled for, each without
// spilling to scratch: FP64 with the whole register file of one wave per
// SIMD; FP32 with a third of it (168 registers), three blocks sharing a CU.
// The library checks at start-up that no face kernel uses private memory.
template <typename T, int DIR = 0, int STAGE = 2> struct FaceWaves {
  static constexpr int value = sizeof(T) == 8 ? 1 : 3;
};
// LDS layout of a face tile.  OWNW = 0: the layout every direction shares;
// OWNW = w > 0: the kernel's own direction only, for a kernel compiled for w
// waves per SIMD (three: unpadded records where the padding would cost the
// third block)
template <int DIR, int M, typename T, int V, int OWNW>
using FaceLds = Lds<M, T, V, OWNW ? DIR : -1, OWNW == 3>;
// three FP32 tiles of the three-wave kernels, with their static LDS (the
// tally, and the speed reduction at stage 2) and the allocation rounded up
// to 1280 bytes, fit one CU (a tile of 53.5 KB runs three blocks per CU, one
// of 54.2 KB two)
constexpr size_t lds_alloc(size_t b) { return (b + 1279) / 1280 * 1280; }
template <int M> constexpr bool fits3() {
  return lds_alloc(FaceLds<0, M, float, 0, 3>::total + sizeof(Tally) + sizeof(SpeedRed)) <= 160 * 1024 / 3 &&
         lds_alloc(FaceLds<1, M, float, 0, 3>::total + sizeof(Tally) + sizeof(SpeedRed)) <= 160 * 1024 / 3;
}
static_assert(fits3<2>() && fits3<3>() && fits3<4>(), "FP32 three-wave face tiles fit three blocks per CU");

// Step 3 tangential-fit weights in the working precision (float copies of
// the tables for the FP32-flux variant: no conversion per use)
template <typename T, int K>
__device__ __forceinline__ T tanw(int m, int l, int k) {
  if (sizeof(T) == 4) return T(K == 1 ? kT1f[m][l][k] : kT2f[m][l][k]);
  return T(K == 1 ? kT1[m][l][k] : kT2[m][l][k]);
}

// One tile (bx, by) of nbx x nby; callable from a persistent loop (starts
// with a barrier so the LDS of the previous tile is free).  SU: staging passes
// whose loads are issued together (all of them where registers allow; the
// persistent batched kernels keep more per-job state live and take fewer).
// OWNW: the LDS layout (FaceLds); a kernel compiled for its own direction
// (OWNW > 0) also takes the health block's indices afresh.
template <int DIR, int STAGE, int M, typename T, bool PR, int SU = 32, bool PERSIST = false, int V = 0,
          bool UNROLL = false, int OWNW = 0>
__device__ void face2d_tile(const Geo& g, const Consts& C, const Bufs& B, unsigned char* smem, int bx, int by,
                            int nbx, int nby) {
  using TL = Tile<M, V>;
  using LD = FaceLds<DIR, M, T, V, OWNW>;
  constexpr int NF = TL::NF, NT = TL::NT, NC = TL::NC, NR = TL::NR;
  const gptr<const Header> hdr = glb((const Header*)B.hdr);
  __shared__ Tally tally;
  __syncthreads();
  if (!hdr->active) return;
  // persistent callers: an index the compiler cannot hoist out of their loop
  const int tx = PERSIST ? tile_tid256() : (int)threadIdx.x;
  tally_zero(tally, tx);
  const double dt = hdr->dt;
  T* s2v = (T*)smem;
  T* s2d = (T*)(smem + LD::s2v);
  T* s2dd = (T*)(smem + LD::s2v + LD::s2d);
  double* res = (double*)(smem + LD::off_res);     // over recon and staging, after B3
  double* fin = (double*)(smem + LD::off_fin);
  constexpr int RS = LD::RS;
  constexpr int NB = NF * NT * M;   // Gauss points of the tile
  auto I2 = [&](int r, int c, int l, int sd, int v) {     // value and normal-derivative records
    return (DIR == 0 ? r * LD::RW + c * RS : c * LD::CS + r * RS) + (l * 2 + sd) * 4 + v;
  };
  auto I2D = [&](int r, int c, int l, int sd, int v) {    // second-derivative records (r < NT)
    return (DIR == 0 ? r * LD::RW + c * RS : c * LD::CSD + r * RS) + (l * 2 + sd) * 4 + v;
  };
  // Gauss point (face f, line r, node l) -> its thread / result column
  auto gp = [&](int f, int r, int l) { return DIR == 0 ? f + NF * (r + NT * l) : r + NT * (f + NF * l); };

  const int nmax = DIR == 0 ? g.nx : g.ny;   // cells along the normal
  const int tmax = DIR == 0 ? g.ny : g.nx;   // cells along the tangential
  const int F0 = bx * (NF - 1);
  const int T0 = by * NT;
  const double hn = DIR == 0 ? C.dx : C.dy;
  const double ihn = DIR == 0 ? C.idx : C.idy, ihn2 = DIR == 0 ? C.idx2 : C.idy2;   // normal 1/h, 1/h^2
  const double iht = DIR == 0 ? C.idy : C.idx, iht2 = DIR == 0 ? C.idy2 : C.idx2;   // tangential
  const gptr<const double> Uin = glb((const double*)(STAGE == 1 ? B.U : B.S));
  const gptr<const T> LV = glb((const T*)(DIR == 0 ? B.lvx : B.lvy));
  const gptr<const double> sgN = glb((const double*)(DIR == 0 ? B.sxo : B.syo));   // normal-face strengths
  const gptr<const double> sgT = glb((const double*)(DIR == 0 ? B.syo : B.sxo));   // tangential-face strengths
  const gptr<double> Ug = glb(B.U), Sg = glb(B.S), Ag = glb(B.A);
  // slope planes of the state, stage state and accumulator (element type T)
  const gptr<T> UgS = glb(slopes<T>(B.U, g)), SgS = glb(slopes<T>(B.S, g)), AgS = glb(slopes<T>(B.A, g));
  const int gcomp[4] = {0, DIR == 0 ? 1 : 2, DIR == 0 ? 2 : 1, 3};
  auto gi = [&](int n, int t) { return DIR == 0 ? n : t; };
  auto gj = [&](int n, int t) { return DIR == 0 ? t : n; };
  auto sgn_idx = [&](int t, int face) { return DIR == 0 ? g.sgx(t, face) : g.sgy(t, face); };
  auto sgt_idx = [&](int n, int face) { return DIR == 0 ? g.sgy(n, face) : g.sgx(n, face); };

  // ---- Step 2 inputs to LDS: one batch of loads for the whole tile ----
  // Entries outside the stored grid (ghosts included) are clamped into it;
  // only items that no thread owns read them.  Every pass runs on all lanes
  // (wave-uniform); only the LDS stores are masked.
  constexpr int NCS = LD::NCS, NSG = LD::NSG, NSTV = LD::NSTV;
  T* stv = (T*)(smem + LD::off_staging);                    // [v][l][r][cc]
  T* sts = stv + NSTV;                                               // same shape
  double* stg = (double*)(smem + LD::off_staging + LD::st_sg);   // [r][ff]
  T* atab = (T*)(smem + LD::off_atab);                       // [c][r], r < NT
  auto clampi = [](int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); };
  {
    // a lane keeps one (line, cell) position of a staged plane; the passes
    // walk the planes (array, variable, Gauss line), PPP planes per pass
    constexpr int PL = NR * NCS, PPP = 256 / PL, NPL = 2 * 4 * M;
    static_assert(PPP >= 1, "a plane fits one pass");
    const int tid = tx;
    const int lp = tid / PL < PPP ? tid / PL : PPP - 1;   // lanes past the last plane slot repeat it
    const int e = tid % PL;
    const int cc = DIR == 0 ? e % NCS : e / NR, r = DIR == 0 ? e / NCS : e % NR;
    const bool slot = tid < PPP * PL;
    const int n = clampi(F0 - 3 + cc, -H, nmax + H - 1), t = clampi(T0 - 1 + r, -H, tmax + H - 1);
    const size_t cell = g.cell(gi(n, t), gj(n, t));
    const T hnT = T(hn);   // the slopes are staged h-scaled
    const gptr<const T> slope = glb(slopes<T>((const double*)(STAGE == 1 ? B.U : B.S), g)) +
                                (DIR == 0 ? 0 : (size_t)g.nv * g.m * g.cells);
#pragma unroll SU
    for (int p0 = 0; p0 < NPL; p0 += PPP) {
      const int pl = p0 + lp < NPL ? p0 + lp : NPL - 1;
      const int arr = pl / (4 * M), vl = pl % (4 * M), v = vl / M, l = vl % M;
      const size_t off = ((size_t)gcomp[v] * M + l) * g.cells + cell;
      const T val = arr == 0 ? LV[off] : hnT * slope[off];
      if (slot && p0 + lp < NPL) stv[arr * NSTV + (vl * NR + r) * NCS + cc] = val;
    }
  }
  {
    // normal strengths of the staged faces, and the tangential DFF factors of
    // the Step 3 states (cell F0-1+c, line T0+r): one item of each per lane
    static_assert(NR * NSG <= 256 && NC * NT <= 256, "one pass");
    const int it = tx;
    {
      const int k = it < NR * NSG ? it : 0;
      const int ff = DIR == 0 ? k % NSG : k / NR, r = DIR == 0 ? k / NSG : k % NR;
      const int face = clampi(F0 - 3 + ff, -H, nmax + H), t = clampi(T0 - 1 + r, -H, tmax + H - 1);
      const double sg = sgN[sgn_idx(t, face)];
      if (it < NR * NSG) stg[r * NSG + ff] = sg;
    }
    {
      const int k = it < NC * NT ? it : 0;
      const int c = DIR == 0 ? k % NC : k / NT, r = DIR == 0 ? k / NC : k % NT;
      const int ncell = clampi(F0 - 1 + c, -H, nmax + H - 1);
      double A = 0.0;
#pragma unroll
      for (int q = -1; q <= 2; ++q) A += sgT[sgt_idx(ncell, clampi(T0 + r + q, -H, tmax + H))];
      const T at = T(dff_of(A, C.thres));
      if (it < NC * NT) atab[c * NT + r] = at;
    }
  }
  __syncthreads();

  // ---- Step 2: normal reconstruction on each line, both faces of a cell ----
  // Every pass runs on all 256 lanes: a lane without an item of its own
  // recomputes a valid item of the tile (c = r = 1, l = 0) and stores nothing.
  constexpr int NA = NC * NR * M;
  // UNROLL (single-grid kernels): in a loop the compiler keeps the
  // stencils' FP64 constants in scalar registers across the passes and
  // spills them into vector lanes; unrolled, the FP64 step is 7% shorter.
  // The arithmetic is the same either way.
#pragma unroll(UNROLL ? (NA + 255) / 256 : 1)
  for (int base = 0; base < NA; base += 256) {
    const int it = base + tx;
    int c, r, l;
    if (DIR == 0) { c = it % NC; r = (it / NC) % NR; l = it / (NC * NR); }
    else { r = it % NR; c = (it / NR) % NC; l = it / (NC * NR); }
    const bool own = it < NA && F0 - 1 + c <= nmax && T0 - 1 + r <= tmax;   // n, t >= -1 by construction
    if (!own) { c = 1; r = 1; l = 0; }
    // cell n = F0-1+c sits at staged column c+2; face n-2+f at column c+f
    double s[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) s[f] = stg[r * NSG + c + f];
    const Cascade cs = cascade(s, C.order, C.thres, C.tie);
    // the tile's own reconstructions: the cells it updates on its own lines
    tally_add(tally, own && c >= 1 && c <= NF - 1 && F0 - 1 + c < nmax && r >= 1 && r <= NT && T0 - 1 + r < tmax,
              cs.branch, cs.tie, C.order, tx);
    T d[4][9];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T* pv = stv + ((v * M + l) * NR + r) * NCS + c;
      const T* ps = sts + ((v * M + l) * NR + r) * NCS + c;
#pragma unroll
      for (int k = 0; k < 5; ++k) d[v][k] = pv[k];
#pragma unroll
      for (int k = 0; k < 4; ++k) d[v][5 + k] = ps[k < 2 ? k : k + 1];   // cells n-2, n-1, n+1, n+2
    }
    T out[2][3][4];
    recon_faces<T, 4>(d, cs, C, out);
    const T ih = T(ihn), ih2 = T(ihn2);
    if (own) {
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          s2v[I2(r, c, l, sd, v)] = out[sd][0][v];
          s2d[I2(r, c, l, sd, v)] = out[sd][1][v] * ih;
          if (r >= 1 && r <= NT) s2dd[I2D(r - 1, c, l, sd, v)] = out[sd][2][v] * ih2;
        }
    }
  }
  __syncthreads();

  tally_flush(tally, B.hdr, tx);

  // ---- Steps 3-4 at every face Gauss point: one Gauss point per thread ----
  static_assert(NB <= 256, "one Gauss point per thread of a 256-thread block");
  // as in Step 2, lanes without a Gauss point of their own compute at face
  // f = 0 of line r = 0 (always inside the grid) and store nothing.  They
  // keep their wave's node index l; at M = 3 the lanes past the tile's last
  // Gauss point (NB < 256) have l = M, a node whose tangential-fit weights are
  // zero in the tables, and read only LDS of the tile
  const int it = tx;
  int f, r, l;
  if (DIR == 0) { f = it % NF; r = (it / NF) % NT; l = it / (NF * NT); }
  else { r = it % NT; f = (it / NT) % NF; l = it / (NF * NT); }
  // a wave holds one Gauss node when NF NT is a multiple of 64 (m = 2, 4):
  // l is then wave-uniform, and the tangential-fit weights of that node are
  // scalar loads
  if ((NF * NT) % 64 == 0) l = __builtin_amdgcn_readfirstlane(l);
  const bool own = it < NB && F0 + f <= nmax && T0 + r < tmax;
  if (!own) { f = 0; r = 0; }
  {
    const int nf = F0 + f, t = T0 + r;
    T Wk[2][6][4];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int c = sd == 0 ? f : f + 1;      // left state: cell nf-1 (its +1/2 face); right: cell nf
      const int ncell = nf - 1 + sd;
      const T at = atab[(f + sd) * NT + r];    // cell ncell = F0-1+(f+sd), line t
      const T it1 = at * T(iht), it2 = at * T(iht2);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Wk[sd][0][v] = s2v[I2(r + 1, c, l, sd, v)];
        Wk[sd][1][v] = s2d[I2(r + 1, c, l, sd, v)];
        Wk[sd][3][v] = s2dd[I2D(r, c, l, sd, v)];
        T a1 = 0, a2 = 0, ax = 0;
#pragma unroll
        for (int rr = 0; rr < 3; ++rr)
#pragma unroll
          for (int q = 0; q < M; ++q) {
            const T w1 = tanw<T, 1>(M, l, rr * M + q), w2 = tanw<T, 2>(M, l, rr * M + q);
            const T val = s2v[I2(r + rr, c, q, sd, v)];
            a1 += w1 * val;
            a2 += w2 * val;
            ax += w1 * s2d[I2(r + rr, c, q, sd, v)];
          }
        Wk[sd][2][v] = it1 * a1;
        Wk[sd][5][v] = it2 * a2;
        Wk[sd][4][v] = it1 * ax;
      }
      // first order from the cell average where the state is nonphysical
      if (!positive_state<T, 2>(Wk[sd][0])) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Wk[sd][0][v] = T(Uin[g.avg(gcomp[v], gi(ncell, t), gj(ncell, t))]);
#pragma unroll
          for (int dd = 1; dd < 6; ++dd) Wk[sd][dd][v] = T(0);
        }
        // counted once per face: the tile's last face is the next tile's first
        if (own && (f < NF - 1 || nf == nmax)) atomicAdd((unsigned long long*)&B.hdr->fallbacks, 1ull);
      }
    }
    __syncthreads();   // B3: the Step 2 records are read; the results may overwrite them
    FaceOut fo;
    gks_flux<T, 2, PR>(Wk[0], Wk[1], dt, C, fo);
    // results to LDS (global component order)
    double* rp = res + gp(f, r, l);   // component k at rp[k * NB]
    if (own) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gv = gcomp[v];
      if (STAGE == 1) {
        rp[gv * NB] = fo.Fh[v];
        rp[(4 + gv) * NB] = (8.0 / 3.0) * fo.Fh[v] - (1.0 / 3.0) * fo.F1[v];
        rp[(8 + gv) * NB] = fo.Wh[v];
        rp[(12 + gv) * NB] = -(4.0 / 3.0) * fo.W0[v] + (8.0 / 3.0) * fo.Wh[v] - (1.0 / 3.0) * fo.W1[v];
      } else {
        rp[gv * NB] = (4.0 / 3.0) * (fo.F1[v] - 2.0 * fo.Fh[v]);
        rp[(4 + gv) * NB] = (4.0 / 3.0) * (fo.W0[v] - 2.0 * fo.Wh[v] + fo.W1[v]);
      }
    }
    if (STAGE == 1) rp[16 * NB] = fo.sigma;
    }
  }
  __syncthreads();

  // ---- strengths of this step (stage 1): mean over the Gauss points ----
  if (STAGE == 1) {
    for (int it = tx; it < NF * NT; it += blockDim.x) {
      const int f = DIR == 0 ? it % NF : it / NT, r = DIR == 0 ? it / NF : it % NT;
      const int nf = F0 + f, t = T0 + r;
      if (nf > nmax || t >= tmax) continue;
      double s = 0.0;
      for (int l = 0; l < M; ++l) s += res[16 * NB + gp(f, r, l)];
      (DIR == 0 ? glb(B.sxn) : glb(B.syn))[sgn_idx(t, nf)] = s / M;
    }
  }

  // ---- cell update of this direction ----
  constexpr int NFT = (NF - 1) * NT;   // updated cells of the tile
  for (int it = tx; it < (NF - 1) * NT * 4; it += blockDim.x) {
    int ci, r, v;
    if (DIR == 0) { ci = it % (NF - 1); r = (it / (NF - 1)) % NT; v = it / ((NF - 1) * NT); }
    else { r = it % NT; ci = (it / NT) % (NF - 1); v = it / ((NF - 1) * NT); }
    const int n = F0 + ci, t = T0 + r;
    if (n >= nmax || t >= tmax) continue;
    const int i = gi(n, t), j = gj(n, t);
    // component k of node l at face n: ra(k, l); at face n+1: rb(k, l)
    auto ra = [&](int k, int l) { return res[k * NB + gp(ci, r, l)]; };
    auto rb = [&](int k, int l) { return res[k * NB + gp(ci + 1, r, l)]; };
    const size_t ia = g.avg(v, i, j);
    if (STAGE == 1) {
      double dF = 0.0, dA = 0.0;
      for (int l = 0; l < M; ++l) {
        const double w = kGw[M][l];
        dF += w * (rb(v, l) - ra(v, l));
        dA += w * (rb(4 + v, l) - ra(4 + v, l));
      }
      const double base = DIR == 0 ? Ug[ia] : Sg[ia];
      const double abase = DIR == 0 ? Ug[ia] : Ag[ia];
      const double snew = base - dF * ihn;
      Sg[ia] = snew;
      Ag[ia] = abase - dA * ihn;
      if (DIR == 1) fin[v * NFT + ci * NT + r] = snew;
      for (int l = 0; l < M; ++l) {
        const size_t is = DIR == 0 ? g.sx(v, l, i, j) : g.sy(v, l, i, j);
        SgS[is] = T((rb(8 + v, l) - ra(8 + v, l)) * ihn);
        AgS[is] = T((rb(12 + v, l) - ra(12 + v, l)) * ihn);
      }
    } else {
      // every load before the first store: U and A are distinct arrays, but
      // the compiler cannot know it and would otherwise wait for each load
      double aslope[M];
#pragma unroll
      for (int l = 0; l < M; ++l) aslope[l] = double(AgS[DIR == 0 ? g.sx(v, l, i, j) : g.sy(v, l, i, j)]);
      const double base = DIR == 0 ? Ag[ia] : Ug[ia];
      double dA = 0.0;
      for (int l = 0; l < M; ++l) dA += kGw[M][l] * (rb(v, l) - ra(v, l));
      const double unew = base - dA * ihn;
      Ug[ia] = unew;
      if (DIR == 1) fin[v * NFT + ci * NT + r] = unew;
#pragma unroll
      for (int l = 0; l < M; ++l) {
        const size_t is = DIR == 0 ? g.sx(v, l, i, j) : g.sy(v, l, i, j);
        UgS[is] = T(aslope[l] + (rb(4 + v, l) - ra(4 + v, l)) * ihn);
      }
    }
  }
  if (DIR == 1) {
    __syncthreads();
    // health and (stage 2) the speed reduction for the next time step.  In
    // the kernels of one direction (OWNW) the lane's cell indices and gamma
    // are taken afresh (tile_tid, fresh): shared with Step 3, what is derived
    // from them would stay live in registers through the flux
    const int it = OWNW ? tile_tid256() : tx;
    bool valid = false;
    double s = 0.0, rr = 1.0;
    if (it < (NF - 1) * NT) {
      const int r = it % NT, ci = it / NT;
      const int n = F0 + ci, t = T0 + r;
      if (n < nmax && t < tmax) {
        double W[4];
        for (int v = 0; v < 4; ++v) W[v] = fin[v * NFT + ci * NT + r];
        rr = W[0];
        valid = cell_speed(W, 2, OWNW ? fresh(C.gamma) : C.gamma, s);
        if (!valid) atomicAdd((unsigned long long*)&B.hdr->nonphysical, 1ull);
      }
    }
    if (STAGE == 2) reduce_speed(B, s, rr, valid, bx + nbx * by, nbx * nby);
  }
}


// ---------------------------------------------------------------------------
// 1-D stage.  A segment owns faces F0 .. F0+S1_FACES-1 and updates cells
// F0 .. F0+S1_FACES-2.  Its inputs (cell averages, slopes and face strengths
// with the stencil halo; in stage 2 also the accumulator of the updated
// cells) are loaded straight from memory into LDS, as stored, without passing
// through registers (global_load_lds).  Phases, separated by barriers: one
// thread per cell reconstructs both of its faces (cells F0-1 .. F0+S1_FACES-1,
// one per thread); one thread per face takes its two states and computes the
// flux; the update.  A persistent block issues the next segment's input loads
// into a second buffer before it reconstructs the current one, so their
// latency is hidden behind this segment's arithmetic.
// ---------------------------------------------------------------------------
constexpr int S1_FACES = 255;                  // faces per block
constexpr int S1_CELLS = S1_FACES - 1;         // updated cells per block
constexpr int S1_NS = S1_FACES + 5;            // staged cells F0-3 .. F0+S1_FACES+1
constexpr int S1_NG = S1_FACES + 6;            // staged faces F0-3 .. F0+S1_FACES+2

// One input buffer: averages (double) and slopes (storage type T) of the
// staged cells, strengths (double) of the staged faces.
template <typename T> struct S1In {
  double avg[3][S1_NS];
  T slo[3][S1_NS];
  double sig[S1_NG];
};
// Stage 2: the accumulator (averages, slopes) of the updated cells.
template <typename T> struct S1Acc {
  double avg[3][S1_CELLS];
  T slo[3][S1_CELLS];
};
// The reconstructions [cell][side][k][v] and, once every flux has read its
// two states, the flux results [face][12 or 6] in the same space.  A result
// row holds an odd number of doubles (13, 7): the 16 lanes that the LDS
// serves together in a 64-bit access then write and read consecutive faces
// on distinct banks (12 and 6 put four and two lanes on each).
template <typename T, int STAGE> union S1Mid {
  T rc[256][18];
  double res[256][STAGE == 1 ? 13 : 7];
};

// Copy n 4-byte words into LDS at dst (word w from the global address
// src(w)) without passing through registers.  Each wave takes every fourth
// chunk of 64 words; lane L of chunk j writes word 64 j + L.  Complete after
// s1_landed.
template <class F>
__device__ __forceinline__ void lds_copy(void* dst, int n, int tid, F&& src) {
  const int lane = tid & 63;
  for (int j = tid >> 6; j * 64 < n; j += 4) {
    const int w = j * 64 + lane;
    auto* d = (__attribute__((address_space(3))) void*)((unsigned*)dst + j * 64);
    if (w < n) __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src(w), d, 4, 0, 0);
  }
}

// Every load of the block into LDS has landed: each wave waits for its own
// memory operations, then the barrier covers the other waves'.
__device__ __forceinline__ void s1_landed() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// Issue the input loads of segment seg (entries outside the stored grid are
// clamped into it; no owned item reads them).  One copy per plane: word w of
// a plane of doubles is half w & 1 of entry w / 2.
template <int STAGE, typename T>
__device__ __forceinline__ void s1_issue_in(const Geo& g, const Bufs& B, int seg, S1In<T>* in, int tid) {
  const int F0 = seg * S1_CELLS;
  const double* U = STAGE == 1 ? B.U : B.S;
  const T* Us = slopes<T>(U, g);
  auto cellc = [&](int c) {
    const int x = F0 - 3 + c;
    return x < -H ? -H : (x > g.nx + H - 1 ? g.nx + H - 1 : x);
  };
  constexpr int WS = sizeof(T) / 4;   // words per slope
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const double* Uv = U + g.avg(v, 0, 0);
    lds_copy(&in->avg[v][0], 2 * S1_NS, tid,
             [&](int w) { return (const unsigned*)(Uv + cellc(w >> 1)) + (w & 1); });
    const T* Sv = Us + g.sx(v, 0, 0, 0);
    lds_copy(&in->slo[v][0], WS * S1_NS, tid,
             [&](int w) { return (const unsigned*)(Sv + cellc(w / WS)) + (w % WS); });
  }
  lds_copy(&in->sig[0], 2 * S1_NG, tid, [&](int w) {
    const int face = F0 - 3 + (w >> 1);
    return (const unsigned*)(B.sxo + g.sgx(0, face < -H ? -H : (face > g.nx + H ? g.nx + H : face))) + (w & 1);
  });
}

// Stage 2: issue the loads of the accumulator of the segment's updated cells.
template <typename T>
__device__ __forceinline__ void s1_issue_acc(const Geo& g, const Bufs& B, int seg, S1Acc<T>* acc, int tid) {
  const int F0 = seg * S1_CELLS;
  const T* As = slopes<T>(B.A, g);
  auto cellc = [&](int c) { const int x = F0 + c; return x > g.nx - 1 ? g.nx - 1 : x; };
  constexpr int WS = sizeof(T) / 4;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const double* Av = B.A + g.avg(v, 0, 0);
    lds_copy(&acc->avg[v][0], 2 * S1_CELLS, tid, [&](int w) { return (const unsigned*)(Av + cellc(w >> 1)) + (w & 1); });
    const T* Sv = As + g.sx(v, 0, 0, 0);
    lds_copy(&acc->slo[v][0], WS * S1_CELLS, tid, [&](int w) { return (const unsigned*)(Sv + cellc(w / WS)) + (w % WS); });
  }
}

// The arithmetic of segment seg, from its inputs in LDS (landed and made
// visible by a barrier).  Stage 2 issues the accumulator loads itself.
// PERSIST: called from a persistent loop (an index the compiler cannot hoist
// out of the loop, as in face2d_tile).
template <int STAGE, typename T, bool PR, bool PERSIST = false>
__device__ void stage1d_seg_lds(const Geo& g, const Consts& C, const Bufs& B, const S1In<T>* in, S1Acc<T>* acc,
                            S1Mid<T, STAGE>* mid, int seg, int nseg) {
  const gptr<const Header> hdr = glb((const Header*)B.hdr);
  if (!hdr->active) return;
  const double dt = hdr->dt;
  const int F0 = seg * S1_CELLS;
  const int t = PERSIST ? tile_tid256() : (int)threadIdx.x;
  const gptr<double> Ug = glb(B.U), Sg = glb(B.S), Ag = glb(B.A);
  const gptr<T> UgS = glb(slopes<T>(B.U, g)), SgS = glb(slopes<T>(B.S, g)), AgS = glb(slopes<T>(B.A, g));
  const double h = C.dx;
  __shared__ Tally tally;
  tally_zero(tally, t);
  __syncthreads();
  // ---- reconstruction: cell F0-1+t (staged index t+2), both faces ----
  {
    double s[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) s[q] = in->sig[t + q];           // faces cell-2 .. cell+3
    const Cascade cs = cascade(s, C.order, C.thres, C.tie);
    // own reconstructions: the cells the segment updates, and the ghost
    // cells -1 and nx beside the first and last boundary faces
    const int cell = F0 - 1 + t;
    tally_add(tally,
              (cell >= F0 && cell < F0 + S1_CELLS && cell < g.nx) || (cell == -1 && seg == 0) ||
                  (cell == g.nx && seg == nseg - 1),
              cs.branch, cs.tie, C.order, t);
    T d[3][9];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
#pragma unroll
      for (int k = 0; k < 5; ++k) d[v][k] = T(in->avg[v][t + k]);
#pragma unroll
      for (int k = 0; k < 4; ++k) d[v][5 + k] = T(h * double(in->slo[v][t + (k < 2 ? k : k + 1)]));   // cells -2, -1, +1, +2
    }
    T out[2][3][3];
    recon_faces<T, 3>(d, cs, C, out);
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int v = 0; v < 3; ++v) mid->rc[t][(sd * 3 + k) * 3 + v] = out[sd][k][v];
  }
  __syncthreads();
  tally_flush(tally, B.hdr, t);
  if (STAGE == 2) s1_issue_acc<T>(g, B, seg, acc, t);   // lands during the flux
  // ---- flux: face F0+f, one per thread (wave-uniform: lanes without a face
  // of their own compute the block's last face and store nothing) ----
  const int f = t;
  const int F = F0 + f;
  const bool own = f < S1_FACES && F <= g.nx;
  const int fc = own ? f : (g.nx - F0 < S1_FACES - 1 ? g.nx - F0 : S1_FACES - 1);
  const int Fc = F0 + fc;
  {
    T Wk[2][6][4];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int cell = Fc - 1 + sd;
      const int tc = fc + sd;                  // its reconstruction slot
      const int side = sd == 0 ? 0 : 1;   // left state: +1/2 face of cell F-1; right: -1/2 face of cell F
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int dd = 0; dd < 6; ++dd) Wk[sd][dd][v] = T(0);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        Wk[sd][0][v] = mid->rc[tc][(side * 3 + 0) * 3 + v];
        Wk[sd][1][v] = mid->rc[tc][(side * 3 + 1) * 3 + v] * T(C.idx);
        Wk[sd][3][v] = mid->rc[tc][(side * 3 + 2) * 3 + v] * T(C.idx2);
      }
      if (!positive_state<T, 1>(Wk[sd][0])) {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          Wk[sd][0][v] = T(in->avg[v][cell - (F0 - 3)]);
          Wk[sd][1][v] = T(0);
          Wk[sd][3][v] = T(0);
        }
        // counted once per face: the segment's last face is the next one's first
        if (own && (f < S1_CELLS || F == g.nx)) atomicAdd((unsigned long long*)&B.hdr->fallbacks, 1ull);
      }
    }
    __syncthreads();   // every flux has its two states: the results may overwrite them
    FaceOut fo;
    gks_flux<T, 1, PR>(Wk[0], Wk[1], dt, C, fo);
    if (own) {
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      if (STAGE == 1) {
        mid->res[f][v] = fo.Fh[v];
        mid->res[f][3 + v] = (8.0 / 3.0) * fo.Fh[v] - (1.0 / 3.0) * fo.F1[v];
        mid->res[f][6 + v] = fo.Wh[v];
        mid->res[f][9 + v] = -(4.0 / 3.0) * fo.W0[v] + (8.0 / 3.0) * fo.Wh[v] - (1.0 / 3.0) * fo.W1[v];
      } else {
        mid->res[f][v] = (4.0 / 3.0) * (fo.F1[v] - 2.0 * fo.Fh[v]);
        mid->res[f][3 + v] = (4.0 / 3.0) * (fo.W0[v] - 2.0 * fo.Wh[v] + fo.W1[v]);
      }
    }
    if (STAGE == 1) glb(B.sxn)[g.sgx(0, F)] = fo.sigma;
    }
  }
  if (STAGE == 2) s1_landed();   // the accumulator loads, and the results
  else __syncthreads();
  const int i = F0 + f;  // cell
  bool valid = false;
  double s = 0.0, rr = 1.0;
  if (f < S1_CELLS && i < g.nx) {
    const double ih = C.idx;
    double W[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const size_t ia = g.avg(v, i, 0), is = g.sx(v, 0, i, 0);
      const auto& r0 = mid->res[f];
      const auto& r1 = mid->res[f + 1];
      if (STAGE == 1) {
        const double u0 = in->avg[v][f + 3];   // the stage input: W^n of cell i
        W[v] = u0 - (r1[v] - r0[v]) * ih;
        Sg[ia] = W[v];
        Ag[ia] = u0 - (r1[3 + v] - r0[3 + v]) * ih;
        SgS[is] = T((r1[6 + v] - r0[6 + v]) * ih);
        AgS[is] = T((r1[9 + v] - r0[9 + v]) * ih);
      } else {
        W[v] = acc->avg[v][f] - (r1[v] - r0[v]) * ih;
        Ug[ia] = W[v];
        UgS[is] = T(double(acc->slo[v][f]) + (r1[3 + v] - r0[3 + v]) * ih);
      }
    }
    rr = W[0];
    valid = cell_speed(W, 1, C.gamma, s);
    if (!valid) atomicAdd((unsigned long long*)&B.hdr->nonphysical, 1ull);
  }
  if (STAGE == 2) reduce_speed(B, s, rr, valid, seg, nseg);
}

// The FP64 variant of the stage body: the inputs pass through registers
// (converted and h-scaled on the way) into LDS, the update reads its inputs
// from memory, and the flux results have an LDS area of their own.  Measured
// on the 4096-problem batch it is 9% faster in FP64 than the body above,
// whose inputs are copied by LDS DMA (one instruction per 4 bytes, so twice
// the instructions for doubles); in FP32 the body above is 15% faster (three
// waves per SIMD).  The two do the same arithmetic on the same values.
// LDS of a segment (bytes, for element type T): averages and h-scaled slopes
// [v][S1_NS] (T), strengths [S1_NG] (double), reconstructions [cell][side][k][v] (T)
template <typename T> struct Lds1D {
  static constexpr size_t avg = 0;
  static constexpr size_t slo = avg + 3 * S1_NS * sizeof(T);
  static constexpr size_t sig = (slo + 3 * S1_NS * sizeof(T) + 7) / 8 * 8;
  static constexpr size_t rec = sig + S1_NG * sizeof(double);
  static constexpr size_t total = rec + 256 * 18 * sizeof(T);
};

template <int STAGE, typename T, bool PR>
__device__ void stage1d_seg(const Geo& g, const Consts& C, const Bufs& B, double (*res)[12], unsigned char* sm,
                            int seg, int nseg) {
  const gptr<const Header> hdr = glb((const Header*)B.hdr);
  __syncthreads();
  if (!hdr->active) return;
  const double dt = hdr->dt;
  const int F0 = seg * S1_CELLS;
  const int t = threadIdx.x;
  const gptr<const double> Uin = glb((const double*)(STAGE == 1 ? B.U : B.S));
  const gptr<double> Ug = glb(B.U), Sg = glb(B.S), Ag = glb(B.A);
  // slope planes (element type T)
  const gptr<const T> UinS = glb(slopes<T>((const double*)(STAGE == 1 ? B.U : B.S), g));
  const gptr<T> UgS = glb(slopes<T>(B.U, g)), SgS = glb(slopes<T>(B.S, g)), AgS = glb(slopes<T>(B.A, g));
  const double h = C.dx;
  T* sa = (T*)(sm + Lds1D<T>::avg);
  T* ss = (T*)(sm + Lds1D<T>::slo);
  double* sg = (double*)(sm + Lds1D<T>::sig);
  T* rc = (T*)(sm + Lds1D<T>::rec);
  __shared__ Tally tally;
  tally_zero(tally, t);
  // ---- inputs: staged cell c at F0-3+c, face q at F0-3+q (clamped into the
  // stored grid; no owned item reads a clamped entry); all lanes load ----
  auto clampc = [&](int x) { return x < -H ? -H : (x > g.nx + H - 1 ? g.nx + H - 1 : x); };
#pragma unroll
  for (int base = 0; base < 3 * S1_NS; base += 256) {
    const int k = base + t < 3 * S1_NS ? base + t : 3 * S1_NS - 1;
    const int v = k / S1_NS, c = k % S1_NS;
    const int cell = clampc(F0 - 3 + c);
    const T a = T(Uin[g.avg(v, cell, 0)]);
    const T sl = T(h * double(UinS[g.sx(v, 0, cell, 0)]));
    if (base + t < 3 * S1_NS) { sa[v * S1_NS + c] = a; ss[v * S1_NS + c] = sl; }
  }
#pragma unroll
  for (int base = 0; base < S1_NG; base += 256) {
    const int q = base + t < S1_NG ? base + t : S1_NG - 1;
    const int face = F0 - 3 + q;
    const double sv = glb(B.sxo)[g.sgx(0, face < -H ? -H : (face > g.nx + H ? g.nx + H : face))];
    if (base + t < S1_NG) sg[q] = sv;
  }
  __syncthreads();
  // ---- reconstruction: cell F0-1+t (staged index t+2), both faces ----
  {
    double s[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) s[q] = sg[t + q];           // faces cell-2 .. cell+3
    const Cascade cs = cascade(s, C.order, C.thres, C.tie);
    // own reconstructions: the cells the segment updates, and the ghost
    // cells -1 and nx beside the first and last boundary faces
    const int cell = F0 - 1 + t;
    tally_add(tally,
              (cell >= F0 && cell < F0 + S1_CELLS && cell < g.nx) || (cell == -1 && seg == 0) ||
                  (cell == g.nx && seg == nseg - 1),
              cs.branch, cs.tie, C.order, t);
    T d[3][9];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
#pragma unroll
      for (int k = 0; k < 5; ++k) d[v][k] = sa[v * S1_NS + t + k];
#pragma unroll
      for (int k = 0; k < 4; ++k) d[v][5 + k] = ss[v * S1_NS + t + (k < 2 ? k : k + 1)];   // cells -2, -1, +1, +2
    }
    T out[2][3][3];
    recon_faces<T, 3>(d, cs, C, out);
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int v = 0; v < 3; ++v) rc[((t * 2 + sd) * 3 + k) * 3 + v] = out[sd][k][v];
  }
  __syncthreads();
  tally_flush(tally, B.hdr, t);
  // ---- flux: face F0+f, one per thread (wave-uniform: lanes without a face
  // of their own compute the block's last face and store nothing) ----
  const int f = t;
  const int F = F0 + f;
  const bool own = f < S1_FACES && F <= g.nx;
  const int fc = own ? f : (g.nx - F0 < S1_FACES - 1 ? g.nx - F0 : S1_FACES - 1);
  const int Fc = F0 + fc;
  {
    T Wk[2][6][4];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int cell = Fc - 1 + sd;
      const int tc = fc + sd;                  // its reconstruction slot
      const int side = sd == 0 ? 0 : 1;   // left state: +1/2 face of cell F-1; right: -1/2 face of cell F
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int dd = 0; dd < 6; ++dd) Wk[sd][dd][v] = T(0);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        Wk[sd][0][v] = rc[((tc * 2 + side) * 3 + 0) * 3 + v];
        Wk[sd][1][v] = rc[((tc * 2 + side) * 3 + 1) * 3 + v] * T(C.idx);
        Wk[sd][3][v] = rc[((tc * 2 + side) * 3 + 2) * 3 + v] * T(C.idx2);
      }
      if (!positive_state<T, 1>(Wk[sd][0])) {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          Wk[sd][0][v] = sa[v * S1_NS + cell - (F0 - 3)];
          Wk[sd][1][v] = T(0);
          Wk[sd][3][v] = T(0);
        }
        // counted once per face: the segment's last face is the next one's first
        if (own && (f < S1_CELLS || F == g.nx)) atomicAdd((unsigned long long*)&B.hdr->fallbacks, 1ull);
      }
    }
    FaceOut fo;
    gks_flux<T, 1, PR>(Wk[0], Wk[1], dt, C, fo);
    if (own) {
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      if (STAGE == 1) {
        res[f][v] = fo.Fh[v];
        res[f][3 + v] = (8.0 / 3.0) * fo.Fh[v] - (1.0 / 3.0) * fo.F1[v];
        res[f][6 + v] = fo.Wh[v];
        res[f][9 + v] = -(4.0 / 3.0) * fo.W0[v] + (8.0 / 3.0) * fo.Wh[v] - (1.0 / 3.0) * fo.W1[v];
      } else {
        res[f][v] = (4.0 / 3.0) * (fo.F1[v] - 2.0 * fo.Fh[v]);
        res[f][3 + v] = (4.0 / 3.0) * (fo.W0[v] - 2.0 * fo.Wh[v] + fo.W1[v]);
      }
    }
    if (STAGE == 1) glb(B.sxn)[g.sgx(0, F)] = fo.sigma;
    }
  }
  __syncthreads();
  const int i = F0 + f;  // cell
  bool valid = false;
  double s = 0.0, rr = 1.0;
  if (f < S1_CELLS && i < g.nx) {
    const double ih = C.idx;
    double W[3];
    // every load before the first store (the arrays are distinct, which the
    // compiler cannot know)
    double in0[3], in1[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      in0[v] = STAGE == 1 ? Ug[g.avg(v, i, 0)] : Ag[g.avg(v, i, 0)];
      in1[v] = STAGE == 1 ? 0.0 : double(AgS[g.sx(v, 0, i, 0)]);
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const size_t ia = g.avg(v, i, 0), is = g.sx(v, 0, i, 0);
      if (STAGE == 1) {
        const double u0 = in0[v];
        W[v] = u0 - (res[f + 1][v] - res[f][v]) * ih;
        Sg[ia] = W[v];
        Ag[ia] = u0 - (res[f + 1][3 + v] - res[f][3 + v]) * ih;
        SgS[is] = T((res[f + 1][6 + v] - res[f][6 + v]) * ih);
        AgS[is] = T((res[f + 1][9 + v] - res[f][9 + v]) * ih);
      } else {
        W[v] = in0[v] - (res[f + 1][v] - res[f][v]) * ih;
        Ug[ia] = W[v];
        UgS[is] = T(in1[v] + (res[f + 1][3 + v] - res[f][3 + v]) * ih);
      }
    }
    rr = W[0];
    valid = cell_speed(W, 1, C.gamma, s);
    if (!valid) atomicAdd((unsigned long long*)&B.hdr->nonphysical, 1ull);
  }
  if (STAGE == 2) reduce_speed(B, s, rr, valid, seg, nseg);
}

}  // namespace
