// Operation count of the HIP path's arithmetic per unit of work, for the
// roofline model: the device functions of cgks_device.hpp instantiated on
// the host with a counting scalar type.  Adds, subtracts and multiplies count
// 1 FLOP each (a fused multiply-add is 2), divisions 1 FLOP (also listed
// apart), square roots, exponentials and erfc are listed as transcendentals.
// The loops that live in the kernels themselves (Step 3 tangential fits,
// update, strengths) are counted by formula at the end.
//
// Build and run (host only):
//   hipcc -O1 -std=c++17 -x hip --offload-arch=gfx950 flop_count.cpp -o flop_count && ./flop_count
#include <cmath>
#include <cstdio>

struct Fl;
namespace fc {
long long add = 0, mul = 0, dv = 0, tr = 0;
}

struct Fl {
  double v;
  Fl() : v(0) {}
  Fl(double x) : v(x) {}
  explicit operator double() const { return v; }
};
static inline Fl operator+(Fl a, Fl b) { ++fc::add; return Fl(a.v + b.v); }
static inline Fl operator-(Fl a, Fl b) { ++fc::add; return Fl(a.v - b.v); }
static inline Fl operator*(Fl a, Fl b) { ++fc::mul; return Fl(a.v * b.v); }
static inline Fl operator/(Fl a, Fl b) { ++fc::dv; return Fl(a.v / b.v); }
static inline Fl operator-(Fl a) { return Fl(-a.v); }
static inline Fl& operator+=(Fl& a, Fl b) { a = a + b; return a; }
static inline Fl& operator-=(Fl& a, Fl b) { a = a - b; return a; }
static inline Fl& operator*=(Fl& a, Fl b) { a = a * b; return a; }
static inline bool operator>(Fl a, Fl b) { return a.v > b.v; }
static inline bool operator<(Fl a, Fl b) { return a.v < b.v; }
static inline Fl fabs(Fl a) { return Fl(std::fabs(a.v)); }

#define CGKS_HD
#include "cgks_device.hpp"

namespace cgks {
template <> Fl dev_erfc<Fl>(Fl x) { ++fc::tr; return Fl(std::erfc(x.v)); }
template <> Fl dev_exp<Fl>(Fl x) { ++fc::tr; return Fl(std::exp(x.v)); }
template <> Fl dev_sqrt<Fl>(Fl x) { ++fc::tr; return Fl(std::sqrt(x.v)); }
}  // namespace cgks

using namespace cgks;

static void reset() { fc::add = fc::mul = fc::dv = fc::tr = 0; }
static long long flops() { return fc::add + fc::mul + fc::dv; }

int main() {
  Consts C;
  C.gamma = 1.4; C.Kd = 5.0; C.iKd = 0.2; C.c1 = 0.05; C.c2 = 1.0; C.mu = 1e-4; C.thres = 1.0; C.ghi = 0.85; C.glo = 0.6;
  C.eps = 1e-8; C.dx = C.dy = 1.0 / 2048; C.tau_model = 2; C.order = 9; C.m = 4;
  C.idx = C.idy = 2048; C.idx2 = C.idy2 = 2048.0 * 2048.0;
  C.gw[0] = C.gw[1] = (1.0 - C.ghi) * (1.0 - C.glo) / 2.0; C.gw[2] = (1.0 - C.ghi) * C.glo; C.rflags = 0;
  // flux at one Gauss point (2-D and 1-D), smooth viscous state
  Fl Wl[6][4], Wr[6][4];
  const double W0[4] = {1.0, 0.2, -0.1, 2.5 + 0.025};
  for (int v = 0; v < 4; ++v) {
    Wl[0][v] = W0[v]; Wr[0][v] = W0[v] * 1.0001;
    for (int d = 1; d < 6; ++d) { Wl[d][v] = 0.01 * (d + v); Wr[d][v] = 0.011 * (d + v); }
  }
  FaceOut o;
  C.prandtl = 1.0;
  reset();
  gks_flux<Fl, 2, false>(Wl, Wr, 1e-4, C, o);
  printf("flux2d (Pr = 1) flops %lld\n", flops());
  C.prandtl = 0.72;
  C.prfac = 1.0 / C.prandtl - 1.0;
  reset();
  gks_flux<Fl, 2, true>(Wl, Wr, 1e-4, C, o);
  // the time combination in double: 2 flux integrals x 4 components x ~14 ops,
  // 3 interface values x 4 x ~8 ops, strength ~20, tau ~8
  const long long comb2 = 2 * 4 * 14 + 3 * 4 * 8 + 20 + 8;
  printf("flux2d (Pr fix) flops %lld (+%lld double-side) div %lld transcendental %lld\n", flops(), comb2, fc::dv, fc::tr);
  const long long flux2 = flops() + comb2;
  reset();
  C.m = 1;
  {
    Fl a[6][4], b[6][4];
    for (int v = 0; v < 3; ++v) for (int d = 0; d < 6; ++d) { a[d][v] = Wl[d][v]; b[d][v] = Wr[d][v]; }
    a[0][2] = b[0][2] = 2.52;
    gks_flux<Fl, 1>(a, b, 1e-4, C, o);
  }
  const long long comb1 = 2 * 3 * 14 + 3 * 3 * 8 + 16 + 8;
  printf("flux1d  flops %lld (+%lld) div %lld transcendental %lld\n", flops(), comb1, fc::dv, fc::tr);
  const long long flux1 = flops() + comb1;
  // reconstruction of one cell on one line: 4 components, faces (value, d, d2) and nodes
  C.m = 4;
  Fl d[4][9];
  for (int v = 0; v < 4; ++v) for (int s = 0; s < 9; ++s) d[v][s] = 1.0 + 0.01 * s + v;
  Fl out[2][3][4], nodes[4][4];
  Cascade lin; lin.branch = 9;
  Cascade ao; ao.branch = 0; ao.al[0] = 0.5; ao.al[1] = 0.6; ao.al[2] = 0.7; ao.al[3] = 0.8;
  reset(); recon_faces<Fl, 4>(d, lin, C, out); const long long rf9 = flops();
  reset(); recon_faces<Fl, 4>(d, ao, C, out); const long long rfao = flops();
  reset(); recon_nodes<Fl, 4, 4>(d, lin, C, nodes); const long long rn9 = flops();
  reset(); recon_nodes<Fl, 4, 4>(d, ao, C, nodes); const long long rnao = flops();
  printf("recon faces r9 %lld AO %lld; nodes(m=4) r9 %lld AO %lld  (4 components)\n", rf9, rfao, rn9, rnao);
  // per 2-D cell and stage with the linear 9th-order branch (smooth flow), m = 4:
  //  Step 1: one node evaluation per direction (+ tangential slope sums 2*4*4*m)
  //  Step 2: one face evaluation per line and direction (x m x 2), both faces
  //  Step 3: per face Gauss point and side: 4 components x 3m x (2+2+2) flops
  //  flux: one per face Gauss point owned by the cell (2 directions x m)
  //  update: per direction 4 components x (m x 4 + m x 4) ~ small
  const int m = 4;
  const long long s1 = 2 * (rn9 + 2 * 4 * 4 * m);
  const long long s2 = 2 * m * rf9;
  const long long s3 = 2 * m * 2 * 4 * 3 * m * 6;
  const long long fx = 2 * m * flux2;
  const long long up = 2 * 4 * (8 * m + 4);
  printf("2-D m=4 per cell-stage: step1 %lld step2 %lld step3 %lld flux %lld update %lld total %lld\n", s1, s2, s3,
         fx, up, s1 + s2 + s3 + fx + up);
  printf("2-D m=4 per cell-update (2 stages): %lld FLOP; face kernel share per launch-cell: %lld\n",
         2 * (s1 + s2 + s3 + fx + up), (s2 + s3 + fx + up) / 2);
  printf("per face Gauss point in the face kernel (step 2 share + step 3 + flux): %lld\n",
         (2 * rf9) / 2 + 2 * 4 * 3 * m * 6 + flux2);
  printf("1-D per cell-stage: 2 recon (3 comps) + flux: %lld\n", 2 * (rf9 * 3 / 4) + flux1);
  return 0;
}
