// libcgks.so: kernels and C ABI of the ASE-DFF compact gas-kinetic scheme on
// one MI355X (gfx950).  The C ABI is declared in include/cgks.h.
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

namespace {

thread_local std::string g_err;

cgks_status fail(cgks_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(CGKS_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

struct Header {
  double t;
  double dt;
  unsigned long long smax_bits;
  unsigned long long rmin_bits;
  unsigned long long steps;
  unsigned long long nonphysical;
  unsigned long long fallbacks;
  unsigned long long magic;
  int active;
  int nparts;      // per-block speed partials written by the last reduction
  int pad[14];
};
static_assert(sizeof(Header) <= 256, "header");
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
  __host__ __device__ size_t sx(int v, int l, int i, int j) const {
    return (size_t)nv * cells + ((size_t)v * m + l) * cells + cell(i, j);
  }
  __host__ __device__ size_t sy(int v, int l, int i, int j) const {
    return (size_t)nv * cells + (size_t)nv * m * cells + ((size_t)v * m + l) * cells + cell(i, j);
  }
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
  double* lvx;
  double* lvy;
  double* part;   // per-block [max(|U|+c), min(rho)] of the last reduction
  Header* hdr;
};

}  // namespace

struct cgks_plan {
  Geo g;
  Consts C;
  int precision;
  double dx, dy;
  size_t state_words, sig_x_words, sig_y_words;
  size_t off_S, off_A, off_sxo, off_sxn, off_syo, off_syn, off_lvx, off_lvy, off_part, off_hdr, work_words;
  size_t max_parts;
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
__global__ void k_bc_state(Geo g, double* U) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y;
  if (I >= g.NX) return;
  const int i = I - H, j = (g.dim == 2) ? J - H : 0;
  const bool gx = (i < 0 || i >= g.nx), gy = (g.dim == 2) && (j < 0 || j >= g.ny);
  if (!gx && !gy) return;
  int mx, my = 0;
  const int si = src_cell(i, g.nx, g.bc[0], g.bc[1], mx);
  const int sj = (g.dim == 2) ? src_cell(j, g.ny, g.bc[2], g.bc[3], my) : 0;
  const bool rx = mx && (g.bc[i < 0 ? 0 : 1] == CGKS_BC_REFLECTIVE);
  const bool ry = my && (g.bc[j < 0 ? 2 : 3] == CGKS_BC_REFLECTIVE);
  for (int v = 0; v < g.nv; ++v) {
    double odd = 1.0;
    if (rx && v == 1) odd = -odd;
    if (ry && v == 2) odd = -odd;
    U[g.avg(v, i, j)] = odd * U[g.avg(v, si, sj)];
    for (int l = 0; l < g.m; ++l) {
      const int lx = my ? g.m - 1 - l : l;   // x-slope lines are horizontal: mirrored by a y-mirror
      U[g.sx(v, l, i, j)] = (mx ? -odd : odd) * U[g.sx(v, lx, si, sj)];
      if (g.dim == 2) {
        const int ly = mx ? g.m - 1 - l : l;
        U[g.sy(v, l, i, j)] = (my ? -odd : odd) * U[g.sy(v, ly, si, sj)];
      }
    }
  }
}

// Commit the strengths computed in the previous step (new -> old) and fill
// the ghost faces and ghost rows/columns of the old set.
__global__ void k_bc_sigma(Geo g, int which, const double* sxn, double* sxo, const double* syn, double* syo) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (which == 0) {
    // x-faces: a = F + H in [0, NX], b = row J
    if (a > g.NX) return;
    const int F = a - H, j = (g.dim == 2) ? b - H : 0;
    int my = 0;
    const int sj = (g.dim == 2) ? src_cell(j, g.ny, g.bc[2], g.bc[3], my) : 0;
    const int sF = src_face(F, g.nx, g.bc[0], g.bc[1]);
    sxo[g.sgx(j, F)] = sxn[g.sgx(sj, sF)];
  } else {
    // y-faces: a = G + H in [0, NY], b = column I
    if (a > g.NY) return;
    const int G = a - H, i = b - H;
    int mx = 0;
    const int si = src_cell(i, g.nx, g.bc[0], g.bc[1], mx);
    const int sG = src_face(G, g.ny, g.bc[2], g.bc[3]);
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

// ---------------------------------------------------------------------------
// time step (Sec. 4): reduction of max(|U| + c) and min(rho), then dt
// ---------------------------------------------------------------------------
// Block-level max(|U| + c) and min(rho); thread 0 writes the block's partial
// (reduced by k_dt before the next step).  Called by every thread of the block.
__device__ __forceinline__ void reduce_speed(Bufs B, double s, double r, bool valid) {
  __shared__ double red[2][16];
  double sm = valid ? s : 0.0;
  double rm = valid ? r : INFINITY;
  for (int off = 32; off > 0; off >>= 1) {
    sm = fmax(sm, __shfl_xor(sm, off, 64));
    rm = fmin(rm, __shfl_xor(rm, off, 64));
  }
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) { red[0][w] = sm; red[1][w] = rm; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < nw; ++k) { sm = fmax(sm, red[0][k]); rm = fmin(rm, red[1][k]); }
    const int bid = blockIdx.x + gridDim.x * blockIdx.y;
    B.part[2 * bid] = sm;
    B.part[2 * bid + 1] = rm;
    if (bid == 0) B.hdr->nparts = gridDim.x * gridDim.y;
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

__global__ void k_reduce(Geo g, double gam, const double* U, Bufs B) {
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
  reduce_speed(B, s, r, valid);
}

__global__ void k_dt(Header* hdr, const double* part, double dt_fixed, double cfl, double t_end, double h, double mu,
                     int viscous) {
  __shared__ double red[2][256];
  const int np = hdr->nparts;
  double sm = 0.0, rm = INFINITY;
  for (int k = threadIdx.x; k < np; k += blockDim.x) {
    sm = fmax(sm, part[2 * k]);
    rm = fmin(rm, part[2 * k + 1]);
  }
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
    dt = cfl * h / red[0][0];
    if (viscous && mu > 0.0) {
      const double dv = cfl * h * h * red[1][0] / (4.0 * mu);
      if (dv < dt) dt = dv;
    }
  }
  int active = 1;
  if (hdr->nonphysical) { active = 0; dt = 0.0; }   // sticky: a nonphysical state stops the run
  else if (t_end > 0.0) {
    if (hdr->t >= t_end) { active = 0; dt = 0.0; }
    else if (hdr->t + dt > t_end) dt = t_end - hdr->t;
  }
  hdr->dt = dt;
  hdr->active = active;
  if (active) {
    hdr->t += dt;
    hdr->steps += 1;
  }
}

// ---------------------------------------------------------------------------
// 2-D Step 1 (Sec. 3.3): tangential ASE-DFF in each column (row) gives the
// line averages of the cell on the horizontal (vertical) Gauss lines.
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(256) void k_lines(Geo g, Consts C, const double* U, const double* sxo,
                                               const double* syo, double* lvx, double* lvy, const Header* hdr) {
  if (!hdr->active) return;
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x) - H;
  const int j = (int)blockIdx.y - H;
  if (i > g.nx + 2) return;
  double wq[4];
#pragma unroll
  for (int l = 0; l < M; ++l) wq[l] = kGw[M][l];
  // x-face line values: column i, rows j-2..j+2, needed for j in [-1, ny]
  if (j >= -1 && j <= g.ny) {
    double d[4][9], s[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) s[f] = syo[g.sgy(i, j - 2 + f)];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int k = 0; k < 5; ++k) d[v][k] = U[g.avg(v, i, j + k - 2)];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int o = k < 2 ? k - 2 : k - 1;
        double a = 0.0;
#pragma unroll
        for (int l = 0; l < M; ++l) a += wq[l] * U[g.sy(v, l, i, j + o)];
        d[v][5 + k] = C.dy * a;
      }
    }
    const Cascade cs = cascade(s, C.order, C.thres);
    double out[4][4];
    recon_nodes<double, 4>(d, cs, C, out);
#pragma unroll
    for (int l = 0; l < M; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) lvx[g.lv(v, l, i, j)] = out[l][v];
  }
  // y-face line values: row j, columns i-2..i+2, needed for i in [-1, nx]
  if (i >= -1 && i <= g.nx && j >= -3 && j <= g.ny + 2) {
    double d[4][9], s[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) s[f] = sxo[g.sgx(j, i - 2 + f)];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int k = 0; k < 5; ++k) d[v][k] = U[g.avg(v, i + k - 2, j)];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int o = k < 2 ? k - 2 : k - 1;
        double a = 0.0;
#pragma unroll
        for (int l = 0; l < M; ++l) a += wq[l] * U[g.sx(v, l, i + o, j)];
        d[v][5 + k] = C.dx * a;
      }
    }
    const Cascade cs = cascade(s, C.order, C.thres);
    double out[4][4];
    recon_nodes<double, 4>(d, cs, C, out);
#pragma unroll
    for (int l = 0; l < M; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) lvy[g.lv(v, l, i, j)] = out[l][v];
  }
}

// ---------------------------------------------------------------------------
// 2-D face kernel: Step 2 (normal ASE-DFF on every Gauss line), Step 3
// (tangential derivatives), Step 4 (flux), and the cell update of one
// direction.  DIR 0: x-faces (normal x), DIR 1: y-faces.
// ---------------------------------------------------------------------------
template <int M> struct Tile {
  static constexpr int NF = 16;                               // faces along the normal
  static constexpr int NT = M == 2 ? 8 : (M == 3 ? 5 : 4);    // lines along the tangential
  static constexpr int NC = NF + 1;                           // reconstructed cells
  static constexpr int NR = NT + 2;                           // reconstructed lines
  static constexpr int RK1 = 17, RK2 = 8;                     // results per Gauss point (stage 1 / 2)
};

template <int M, typename T> struct Lds {
  static constexpr size_t s2v = (size_t)Tile<M>::NR * Tile<M>::NC * M * 8 * sizeof(T);
  static constexpr size_t s2d = s2v;
  static constexpr size_t s2dd = (size_t)Tile<M>::NT * Tile<M>::NC * M * 8 * sizeof(T);
  static constexpr size_t recon = s2v + s2d + s2dd;
  static constexpr size_t res = (size_t)Tile<M>::NF * Tile<M>::NT * M * Tile<M>::RK1 * sizeof(double);
  static constexpr size_t main = recon > res ? recon : res;
  static constexpr size_t fin = (size_t)(Tile<M>::NF - 1) * Tile<M>::NT * 4 * sizeof(double);
  static constexpr size_t total = main + fin;
};

#ifndef CGKS_FACE_WAVES
#define CGKS_FACE_WAVES 2   // minimum waves per SIMD the face kernels are compiled for
#endif

template <int DIR, int STAGE, int M, typename T, bool PR>
__global__ __launch_bounds__(256, CGKS_FACE_WAVES) void k_face2d(Geo g, Consts C, Bufs B) {
  using TL = Tile<M>;
  constexpr int NF = TL::NF, NT = TL::NT, NC = TL::NC, NR = TL::NR;
  const Header* hdr = B.hdr;
  if (!hdr->active) return;
  const double dt = hdr->dt;
  extern __shared__ __align__(16) unsigned char smem[];
  T* s2v = (T*)smem;
  T* s2d = (T*)(smem + Lds<M, T>::s2v);
  T* s2dd = (T*)(smem + Lds<M, T>::s2v + Lds<M, T>::s2d);
  double* res = (double*)smem;
  double* fin = (double*)(smem + Lds<M, T>::main);
  auto I2 = [&](int r, int c, int l, int sd, int v) { return (((r * NC + c) * M + l) * 2 + sd) * 4 + v; };

  const int nmax = DIR == 0 ? g.nx : g.ny;   // cells along the normal
  const int tmax = DIR == 0 ? g.ny : g.nx;   // cells along the tangential
  const int F0 = blockIdx.x * (NF - 1);
  const int T0 = blockIdx.y * NT;
  const double hn = DIR == 0 ? C.dx : C.dy, ht = DIR == 0 ? C.dy : C.dx;
  const double* Uin = STAGE == 1 ? B.U : B.S;
  const double* LV = DIR == 0 ? B.lvx : B.lvy;
  const double* sgN = DIR == 0 ? B.sxo : B.syo;   // normal-face strengths
  const double* sgT = DIR == 0 ? B.syo : B.sxo;   // tangential-face strengths
  const int gcomp[4] = {0, DIR == 0 ? 1 : 2, DIR == 0 ? 2 : 1, 3};
  auto gi = [&](int n, int t) { return DIR == 0 ? n : t; };
  auto gj = [&](int n, int t) { return DIR == 0 ? t : n; };
  auto sN = [&](int v, int l, int n, int t) {  // normal slope on line l
    return DIR == 0 ? g.sx(v, l, gi(n, t), gj(n, t)) : g.sy(v, l, gi(n, t), gj(n, t));
  };
  auto sgn_idx = [&](int t, int face) { return DIR == 0 ? g.sgx(t, face) : g.sgy(t, face); };
  auto sgt_idx = [&](int n, int face) { return DIR == 0 ? g.sgy(n, face) : g.sgx(n, face); };

  // ---- Step 2: normal reconstruction on each line, both faces of a cell ----
  constexpr int NA = NC * NR * M;
  for (int it = threadIdx.x; it < NA; it += blockDim.x) {
    int c, r, l;
    if (DIR == 0) { c = it % NC; r = (it / NC) % NR; l = it / (NC * NR); }
    else { r = it % NR; c = (it / NR) % NC; l = it / (NC * NR); }
    const int n = F0 - 1 + c, t = T0 - 1 + r;
    if (n < -1 || n > nmax || t < -1 || t > tmax) continue;
    double s[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) s[f] = sgN[sgn_idx(t, n - 2 + f)];
    const Cascade cs = cascade(s, C.order, C.thres);
    T d[4][9];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gv = gcomp[v];
#pragma unroll
      for (int k = 0; k < 5; ++k) d[v][k] = T(LV[g.lv(gv, l, gi(n + k - 2, t), gj(n + k - 2, t))]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int o = k < 2 ? k - 2 : k - 1;
        d[v][5 + k] = T(hn * Uin[sN(gv, l, n + o, t)]);
      }
    }
    T out[2][3][4];
    recon_faces<T, 4>(d, cs, C, out);
    const T ih = T(1.0 / hn), ih2 = T(1.0 / (hn * hn));
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        s2v[I2(r, c, l, sd, v)] = out[sd][0][v];
        s2d[I2(r, c, l, sd, v)] = out[sd][1][v] * ih;
        if (r >= 1 && r <= NT) s2dd[I2(r - 1, c, l, sd, v)] = out[sd][2][v] * ih2;
      }
  }
  __syncthreads();

  // ---- Steps 3-4 at every face Gauss point ----
  constexpr int NB = NF * NT * M;
  FaceOut fo;
  bool have = false;
  int my_f = 0, my_r = 0, my_l = 0;
  for (int it = threadIdx.x; it < NB; it += blockDim.x) {  // NB <= 256: one pass
    int f, r, l;
    if (DIR == 0) { f = it % NF; r = (it / NF) % NT; l = it / (NF * NT); }
    else { r = it % NT; f = (it / NT) % NF; l = it / (NF * NT); }
    my_f = f; my_r = r; my_l = l;
    const int nf = F0 + f, t = T0 + r;
    if (nf > nmax || t >= tmax) continue;
    T Wk[2][6][4];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int c = sd == 0 ? f : f + 1;      // left state: cell nf-1 (its +1/2 face); right: cell nf
      const int ncell = nf - 1 + sd;
      double A = 0.0;
#pragma unroll
      for (int q = -1; q <= 2; ++q) A += sgT[sgt_idx(ncell, t + q)];
      const T at = T(dff_of(A, C.thres));
      const T it1 = at / T(ht), it2 = at / T(ht * ht);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Wk[sd][0][v] = s2v[I2(r + 1, c, l, sd, v)];
        Wk[sd][1][v] = s2d[I2(r + 1, c, l, sd, v)];
        Wk[sd][3][v] = s2dd[I2(r, c, l, sd, v)];
        T a1 = 0, a2 = 0, ax = 0;
#pragma unroll
        for (int rr = 0; rr < 3; ++rr)
#pragma unroll
          for (int q = 0; q < M; ++q) {
            const T w1 = T(kT1[M][l][rr * M + q]), w2 = T(kT2[M][l][rr * M + q]);
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
      T rho, U, V, p;
      primitive<T, 2>(Wk[sd][0], T(C.gamma - 1.0), rho, U, V, p);
      if (!(rho > T(0)) || !(p > T(0))) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Wk[sd][0][v] = T(Uin[g.avg(gcomp[v], gi(ncell, t), gj(ncell, t))]);
#pragma unroll
          for (int dd = 1; dd < 6; ++dd) Wk[sd][dd][v] = T(0);
        }
        atomicAdd((unsigned long long*)&B.hdr->fallbacks, 1ull);
      }
    }
    gks_flux<T, 2, PR>(Wk[0], Wk[1], dt, C, fo);
    have = true;
  }
  __syncthreads();
  // results to LDS (global component order)
  if (have) {
    double* rp = res + (((size_t)my_f * NT + my_r) * M + my_l) * (STAGE == 1 ? TL::RK1 : TL::RK2);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gv = gcomp[v];
      if (STAGE == 1) {
        rp[gv] = fo.Fh[v];
        rp[4 + gv] = (8.0 / 3.0) * fo.Fh[v] - (1.0 / 3.0) * fo.F1[v];
        rp[8 + gv] = fo.Wh[v];
        rp[12 + gv] = -(4.0 / 3.0) * fo.W0[v] + (8.0 / 3.0) * fo.Wh[v] - (1.0 / 3.0) * fo.W1[v];
      } else {
        rp[gv] = (4.0 / 3.0) * (fo.F1[v] - 2.0 * fo.Fh[v]);
        rp[4 + gv] = (4.0 / 3.0) * (fo.W0[v] - 2.0 * fo.Wh[v] + fo.W1[v]);
      }
    }
    if (STAGE == 1) rp[16] = fo.sigma;
  }
  __syncthreads();

  // ---- strengths of this step (stage 1): mean over the Gauss points ----
  if (STAGE == 1) {
    for (int it = threadIdx.x; it < NF * NT; it += blockDim.x) {
      const int f = DIR == 0 ? it % NF : it / NT, r = DIR == 0 ? it / NF : it % NT;
      const int nf = F0 + f, t = T0 + r;
      if (nf > nmax || t >= tmax) continue;
      double s = 0.0;
      for (int l = 0; l < M; ++l) s += res[(((size_t)f * NT + r) * M + l) * TL::RK1 + 16];
      (DIR == 0 ? B.sxn : B.syn)[sgn_idx(t, nf)] = s / M;
    }
  }

  // ---- cell update of this direction ----
  constexpr int RK = STAGE == 1 ? TL::RK1 : TL::RK2;
  const double ihn = 1.0 / hn;
  for (int it = threadIdx.x; it < (NF - 1) * NT * 4; it += blockDim.x) {
    int ci, r, v;
    if (DIR == 0) { ci = it % (NF - 1); r = (it / (NF - 1)) % NT; v = it / ((NF - 1) * NT); }
    else { r = it % NT; ci = (it / NT) % (NF - 1); v = it / ((NF - 1) * NT); }
    const int n = F0 + ci, t = T0 + r;
    if (n >= nmax || t >= tmax) continue;
    const int i = gi(n, t), j = gj(n, t);
    const double* ra = res + (((size_t)ci * NT + r) * M) * RK;        // face n
    const double* rb = res + (((size_t)(ci + 1) * NT + r) * M) * RK;  // face n+1
    const size_t ia = g.avg(v, i, j);
    if (STAGE == 1) {
      double dF = 0.0, dA = 0.0;
      for (int l = 0; l < M; ++l) {
        const double w = kGw[M][l];
        dF += w * (rb[l * RK + v] - ra[l * RK + v]);
        dA += w * (rb[l * RK + 4 + v] - ra[l * RK + 4 + v]);
      }
      const double base = DIR == 0 ? B.U[ia] : B.S[ia];
      const double abase = DIR == 0 ? B.U[ia] : B.A[ia];
      const double snew = base - dF * ihn;
      B.S[ia] = snew;
      B.A[ia] = abase - dA * ihn;
      if (DIR == 1) fin[((size_t)ci * NT + r) * 4 + v] = snew;
      for (int l = 0; l < M; ++l) {
        const size_t is = DIR == 0 ? g.sx(v, l, i, j) : g.sy(v, l, i, j);
        B.S[is] = (rb[l * RK + 8 + v] - ra[l * RK + 8 + v]) * ihn;
        B.A[is] = (rb[l * RK + 12 + v] - ra[l * RK + 12 + v]) * ihn;
      }
    } else {
      double dA = 0.0;
      for (int l = 0; l < M; ++l) dA += kGw[M][l] * (rb[l * RK + v] - ra[l * RK + v]);
      const double base = DIR == 0 ? B.A[ia] : B.U[ia];
      const double unew = base - dA * ihn;
      B.U[ia] = unew;
      if (DIR == 1) fin[((size_t)ci * NT + r) * 4 + v] = unew;
      for (int l = 0; l < M; ++l) {
        const size_t is = DIR == 0 ? g.sx(v, l, i, j) : g.sy(v, l, i, j);
        B.U[is] = B.A[is] + (rb[l * RK + 4 + v] - ra[l * RK + 4 + v]) * ihn;
      }
    }
  }
  if (DIR == 1) {
    __syncthreads();
    // health and (stage 2) the speed reduction for the next time step
    const int it = threadIdx.x;
    bool valid = false;
    double s = 0.0, rr = 1.0;
    if (it < (NF - 1) * NT) {
      const int r = it % NT, ci = it / NT;
      const int n = F0 + ci, t = T0 + r;
      if (n < nmax && t < tmax) {
        double W[4];
        for (int v = 0; v < 4; ++v) W[v] = fin[((size_t)ci * NT + r) * 4 + v];
        rr = W[0];
        valid = cell_speed(W, 2, C.gamma, s);
        if (!valid) atomicAdd((unsigned long long*)&B.hdr->nonphysical, 1ull);
      }
    }
    if (STAGE == 2) reduce_speed(B, s, rr, valid);
  }
}

// ---------------------------------------------------------------------------
// 1-D stage kernel: one thread per face; each reconstructs its two cells.
// A block owns faces F0..F0+255 and updates cells F0..F0+254.
// ---------------------------------------------------------------------------
template <int STAGE, typename T, bool PR>
__global__ __launch_bounds__(256) void k_stage1d(Geo g, Consts C, Bufs B) {
  const Header* hdr = B.hdr;
  if (!hdr->active) return;
  const double dt = hdr->dt;
  constexpr int NFB = 256;
  __shared__ double res[NFB][12];
  const int F0 = blockIdx.x * (NFB - 1);
  const int f = threadIdx.x;
  const int F = F0 + f;
  const double* Uin = STAGE == 1 ? B.U : B.S;
  const double h = C.dx;
  if (F <= g.nx) {
    T Wk[2][6][4];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int cell = F - 1 + sd;
      double s[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) s[q] = B.sxo[g.sgx(0, cell - 2 + q)];
      const Cascade cs = cascade(s, C.order, C.thres);
      T d[3][9];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
#pragma unroll
        for (int k = 0; k < 5; ++k) d[v][k] = T(Uin[g.avg(v, cell + k - 2, 0)]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int o = k < 2 ? k - 2 : k - 1;
          d[v][5 + k] = T(h * Uin[g.sx(v, 0, cell + o, 0)]);
        }
      }
      T out[2][3][3];
      recon_faces<T, 3>(d, cs, C, out);
      const int side = sd == 0 ? 0 : 1;   // left state: +1/2 face of cell F-1; right: -1/2 face of cell F
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int dd = 0; dd < 6; ++dd) Wk[sd][dd][v] = T(0);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        Wk[sd][0][v] = out[side][0][v];
        Wk[sd][1][v] = out[side][1][v] / T(h);
        Wk[sd][3][v] = out[side][2][v] / T(h * h);
      }
      T rho, U, V, p;
      primitive<T, 1>(Wk[sd][0], T(C.gamma - 1.0), rho, U, V, p);
      if (!(rho > T(0)) || !(p > T(0))) {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          Wk[sd][0][v] = T(Uin[g.avg(v, cell, 0)]);
          Wk[sd][1][v] = T(0);
          Wk[sd][3][v] = T(0);
        }
        atomicAdd((unsigned long long*)&B.hdr->fallbacks, 1ull);
      }
    }
    FaceOut fo;
    gks_flux<T, 1, PR>(Wk[0], Wk[1], dt, C, fo);
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
    if (STAGE == 1) B.sxn[g.sgx(0, F)] = fo.sigma;
  }
  __syncthreads();
  const int i = F0 + f;  // cell
  bool valid = false;
  double s = 0.0, rr = 1.0;
  if (f < NFB - 1 && i < g.nx) {
    const double ih = 1.0 / h;
    double W[3];
    for (int v = 0; v < 3; ++v) {
      const size_t ia = g.avg(v, i, 0), is = g.sx(v, 0, i, 0);
      if (STAGE == 1) {
        const double u0 = B.U[ia];
        W[v] = u0 - (res[f + 1][v] - res[f][v]) * ih;
        B.S[ia] = W[v];
        B.A[ia] = u0 - (res[f + 1][3 + v] - res[f][3 + v]) * ih;
        B.S[is] = (res[f + 1][6 + v] - res[f][6 + v]) * ih;
        B.A[is] = (res[f + 1][9 + v] - res[f][9 + v]) * ih;
      } else {
        W[v] = B.A[ia] - (res[f + 1][v] - res[f][v]) * ih;
        B.U[ia] = W[v];
        B.U[is] = B.A[is] + (res[f + 1][3 + v] - res[f][3 + v]) * ih;
      }
    }
    rr = W[0];
    valid = cell_speed(W, 1, C.gamma, s);
    if (!valid) atomicAdd((unsigned long long*)&B.hdr->nonphysical, 1ull);
  }
  if (STAGE == 2) reduce_speed(B, s, rr, valid);
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
hipError_t launch_bc_state(const cgks_plan* p, double* U, hipStream_t st, Marks* mk = nullptr) {
  const Geo& g = p->g;
  dim3 grid((g.NX + 255) / 256, g.NY);
  hipLaunchKernelGGL(k_bc_state, grid, dim3(256), 0, st, g, U);
  tick(mk, st);
  return hipGetLastError();
}

hipError_t launch_bc_sigma(const cgks_plan* p, const Bufs& b, hipStream_t st, Marks* mk = nullptr) {
  const Geo& g = p->g;
  dim3 gx((g.NX + 1 + 255) / 256, g.NY);
  hipLaunchKernelGGL(k_bc_sigma, gx, dim3(256), 0, st, g, 0, b.sxn, b.sxo, b.syn, b.syo);
  if (g.dim == 2) {
    dim3 gy((g.NY + 1 + 255) / 256, g.NX);
    hipLaunchKernelGGL(k_bc_sigma, gy, dim3(256), 0, st, g, 1, b.sxn, b.sxo, b.syn, b.syo);
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
    dim3 grid((g.NX + 255) / 256, g.NY);
    hipLaunchKernelGGL(k_lines<M>, grid, dim3(256), 0, st, g, p->C, Uin, b.sxo, b.syo, b.lvx, b.lvy, b.hdr);
    tick(mk, st);
  }
  const size_t lds = Lds<M, T>::total;
  dim3 gx((g.nx + TL::NF - 2) / (TL::NF - 1), (g.ny + TL::NT - 1) / TL::NT);
  dim3 gy((g.ny + TL::NF - 2) / (TL::NF - 1), (g.nx + TL::NT - 1) / TL::NT);
  if (stage == 1) {
    hipLaunchKernelGGL((k_face2d<0, 1, M, T, PR>), gx, dim3(256), lds, st, g, p->C, b);
    tick(mk, st);
    hipLaunchKernelGGL((k_face2d<1, 1, M, T, PR>), gy, dim3(256), lds, st, g, p->C, b);
    tick(mk, st);
  } else {
    hipLaunchKernelGGL((k_face2d<0, 2, M, T, PR>), gx, dim3(256), lds, st, g, p->C, b);
    tick(mk, st);
    hipLaunchKernelGGL((k_face2d<1, 2, M, T, PR>), gy, dim3(256), lds, st, g, p->C, b);
    tick(mk, st);
  }
  return hipGetLastError();
}

template <typename T, bool PR>
hipError_t launch_stage_pr(const cgks_plan* p, const Bufs& b, int stage, hipStream_t st, Marks* mk) {
  const Geo& g = p->g;
  if (g.dim == 1) {
    dim3 grid((g.nx + 254) / 255);
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
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(256), 0, st, b.hdr, b.part, dt, cfl, t_end, h, p->C.mu,
                     p->C.tau_model == CGKS_TAU_VISCOUS ? 1 : 0);
  tick(mk, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_bc_sigma(p, b, st, mk)) != hipSuccess) return e;
  if ((e = launch_bc_state(p, b.U, st, mk)) != hipSuccess) return e;
  e = p->precision == CGKS_FP64 ? launch_stage<double>(p, b, 1, st, mk) : launch_stage<float>(p, b, 1, st, mk);
  if (e != hipSuccess) return e;
  if ((e = launch_bc_state(p, b.S, st, mk)) != hipSuccess) return e;
  return p->precision == CGKS_FP64 ? launch_stage<double>(p, b, 2, st, mk) : launch_stage<float>(p, b, 2, st, mk);
}

const char* kKernels1d[] = {"dt", "bc_sigma", "bc_state", "stage1_1d", "bc_state", "stage2_1d"};
const char* kKernels2d[] = {"dt", "bc_sigma", "bc_state", "lines", "face_x_stage1", "face_y_stage1",
                            "bc_state", "lines", "face_x_stage2", "face_y_stage2"};

template <int M, typename T, bool PR>
hipError_t set_lds_attr_pr() {
  hipError_t e = hipSuccess;
  const int lds = (int)Lds<M, T>::total;
  e = hipFuncSetAttribute((const void*)k_face2d<0, 1, M, T, PR>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_face2d<1, 1, M, T, PR>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_face2d<0, 2, M, T, PR>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_face2d<1, 2, M, T, PR>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

template <int M, typename T>
hipError_t set_lds_attr() {
  hipError_t e = set_lds_attr_pr<M, T, false>();
  return e != hipSuccess ? e : set_lds_attr_pr<M, T, true>();
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

const char* cgks_last_error(void) { return g_err.c_str(); }

cgks_status cgks_plan_create(const cgks_grid_desc* gd, const cgks_scheme_desc* sd, cgks_plan** out) {
  if (!gd || !sd || !out) return fail(CGKS_EINVAL, "NULL argument");
  *out = nullptr;
  if (gd->dim != 1 && gd->dim != 2) return fail(CGKS_EINVAL, "dim must be 1 or 2");
  if (sd->order != 5 && sd->order != 7 && sd->order != 9) return fail(CGKS_EINVAL, "order must be 5, 7 or 9");
  if (!(sd->gamma > 1.0)) return fail(CGKS_EINVAL, "gamma must exceed 1");
  if (gd->nx < 5 || (gd->dim == 2 && gd->ny < 5)) return fail(CGKS_EINVAL, "need at least 5 cells per direction");
  if (gd->dim == 1 && gd->ny != 1) return fail(CGKS_EINVAL, "1-D grids need ny = 1");
  if (!(gd->x1 > gd->x0) || (gd->dim == 2 && !(gd->y1 > gd->y0))) return fail(CGKS_EINVAL, "empty domain");
  for (int k = 0; k < (gd->dim == 2 ? 4 : 2); ++k)
    if (gd->bc[k] < 0 || gd->bc[k] > 2) return fail(CGKS_EINVAL, "unknown boundary condition");
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
  Consts& C = p->C;
  C.gamma = sd->gamma;
  C.Kd = 2.0 / (sd->gamma - 1.0);
  C.c1 = sd->c1;
  C.c2 = sd->c2;
  C.mu = sd->mu;
  C.prandtl = sd->prandtl;
  C.thres = sd->sigma_thres;
  C.ghi = sd->gamma_hi;
  C.glo = sd->gamma_lo;
  C.eps = sd->weno_eps;
  C.dx = p->dx;
  C.dy = p->dy;
  C.tau_model = sd->tau_model;
  C.order = sd->order;
  C.m = gd->dim == 2 ? g.m : 1;
  p->precision = sd->precision;
  const size_t nv = g.nv, m = g.m, cells = g.cells;
  p->state_words = nv * cells * (g.dim == 2 ? 1 + 2 * m : 2);
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
  p->off_lvx = o; o += g.dim == 2 ? up(nv * m * cells) : 0;
  p->off_lvy = o; o += g.dim == 2 ? up(nv * m * cells) : 0;
  {
    // partials: the initial reduction grid, the 1-D stage grid, the 2-D y-face grid
    size_t a = (size_t)((g.nx + 255) / 256) * (g.dim == 2 ? g.ny : 1);
    size_t b1 = (size_t)((g.nx + 254) / 255);
    size_t c = 0;
    if (g.dim == 2) {
      const int NT = g.m == 2 ? 8 : (g.m == 3 ? 5 : 4);
      c = (size_t)((g.ny + 14) / 15) * ((g.nx + NT - 1) / NT);
    }
    p->max_parts = a > b1 ? (a > c ? a : c) : (b1 > c ? b1 : c);
  }
  p->off_part = o; o += up(2 * p->max_parts);
  p->off_hdr = o; o += 32;
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
  if (p->g.dim != 2) return CGKS_OK;
  hipError_t e;
  if (p->precision == CGKS_FP64) e = p->g.m == 2 ? set_lds_attr<2, double>() : (p->g.m == 3 ? set_lds_attr<3, double>() : set_lds_attr<4, double>());
  else e = p->g.m == 2 ? set_lds_attr<2, float>() : (p->g.m == 3 ? set_lds_attr<3, float>() : set_lds_attr<4, float>());
  if (e != hipSuccess) return fail(CGKS_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  return CGKS_OK;
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
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        hs[g.avg(v, i, j)] = h_avg[((size_t)v * ny + j) * nx + i];
        for (int l = 0; l < m; ++l) {
          hs[g.sx(v, l, i, j)] = h_slope_x[(((size_t)v * m + l) * ny + j) * nx + i];
          if (g.dim == 2) hs[g.sy(v, l, i, j)] = h_slope_y[(((size_t)v * m + l) * ny + j) * nx + i];
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
  HIP_TRY(launch_bc_state(p, b.U, st));
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
                            double* h_slope_x, double* h_slope_y, double* h_sigma_x, double* h_sigma_y,
                            double* h_time, long long* h_steps, void* stream) {
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
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        if (h_avg) h_avg[((size_t)v * ny + j) * nx + i] = hs[g.avg(v, i, j)];
        for (int l = 0; l < m; ++l) {
          if (h_slope_x) h_slope_x[(((size_t)v * m + l) * ny + j) * nx + i] = hs[g.sx(v, l, i, j)];
          if (g.dim == 2 && h_slope_y) h_slope_y[(((size_t)v * m + l) * ny + j) * nx + i] = hs[g.sy(v, l, i, j)];
        }
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
  if (hh.nonphysical) return fail(CGKS_ENONPHYSICAL, "nonphysical cell average");
  return CGKS_OK;
}

}  // extern "C"
