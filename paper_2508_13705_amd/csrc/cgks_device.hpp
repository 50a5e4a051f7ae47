// Device arithmetic of the ASE-DFF compact gas-kinetic scheme for gfx950:
// Maxwellian moments, micro-coefficients and the interface flux (Sec. 2.1,
// Eq. 2.6-2.8, 2.11-2.15), the discontinuity feedback factor (Eq. 3.1-3.4)
// and the adaptive-stencil-extension reconstruction (Eq. 3.5-3.19,
// Algorithm 1).  Templated on the arithmetic type T (double, or float for the
// FP32-flux variant) and the dimension D; time coefficients stay in double.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef CGKS_HD
#define CGKS_HD __host__ __device__
#endif

// Each translation unit of the library is its own device code object, and
// HIP exports every __constant__ table of a code object as a global symbol
// under its mangled name.  A per-unit inline namespace gives the tables of
// each unit distinct symbol names, so the loaded code objects cannot bind
// one another's tables.
#ifndef CGKS_UNIT
#define CGKS_UNIT unit
#endif

namespace cgks {
inline namespace CGKS_UNIT {

#include "cgks_tables.inc"

struct Consts {
  double gamma, Kd;          // Kd = 2/(gamma-1) = K + D (K internal degrees of freedom)
  double iKd;                // 1 / Kd
  double c1, c2, mu, prandtl;
  double prfac;              // 1/prandtl - 1: weight of the heat flux in the Prandtl fix
  double thres, ghi, glo, eps;
  double gw[3];              // linear weights of the sub-stencils S0, S1, S2 (AO(5,3), Eq. 3.12)
  double tie;                // |A - thres| <= tie: a cascade decision counted as a near tie
  double dx, dy;
  double idx, idy, idx2, idy2;   // 1/dx, 1/dy, 1/dx^2, 1/dy^2 (no divisions in the kernels)
  int tau_model, order, m;
  int rflags;                // alternative readings, a set of RF_* below
};
// bits of Consts::rflags, equal to the CGKS_READ_* flags of the C interface
enum : int { RF_A3_GAMMA1_LO = 1, RF_A5_UNSCALED_BETA = 2, RF_A10_SIGMA0_ZERO = 4 };

template <typename T> CGKS_HD T dev_erfc(T x);
template <> CGKS_HD __forceinline__ double dev_erfc<double>(double x) { return erfc(x); }
template <> CGKS_HD __forceinline__ float dev_erfc<float>(float x) { return erfcf(x); }
template <typename T> CGKS_HD T dev_exp(T x);
template <> CGKS_HD __forceinline__ double dev_exp<double>(double x) { return exp(x); }
template <> CGKS_HD __forceinline__ float dev_exp<float>(float x) { return expf(x); }
template <typename T> CGKS_HD T dev_sqrt(T x);
template <> CGKS_HD __forceinline__ double dev_sqrt<double>(double x) { return sqrt(x); }
template <> CGKS_HD __forceinline__ float dev_sqrt<float>(float x) { return sqrtf(x); }

// Reciprocal and reciprocal square root: in double the hardware reciprocal
// estimate refined by two Newton steps (within an ulp or two of 1/x; the
// arguments are positive normal numbers); the hardware approximations (1 ulp)
// in the FP32 flux variant.
template <typename T> CGKS_HD __forceinline__ T dev_rcp(T x) { return T(1) / x; }
template <> CGKS_HD __forceinline__ double dev_rcp<double>(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}
template <typename T> CGKS_HD __forceinline__ T dev_rsqrt(T x) { return T(1) / dev_sqrt<T>(x); }
// double: the hardware estimate refined by two Newton steps,
// y <- y (3 - x y^2) / 2 (positive normal arguments)
template <> CGKS_HD __forceinline__ double dev_rsqrt<double>(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  return y * fma(-hx * y, y, 1.5);
#else
  return 1.0 / sqrt(x);
#endif
}
template <> CGKS_HD __forceinline__ float dev_rcp<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
template <> CGKS_HD __forceinline__ float dev_rsqrt<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}

// ---------------------------------------------------------------------------
// Moments of a normalised Maxwellian: <u^n> (full space or one half space),
// <v^n> (full), <xi^2>, <xi^4>.  <u^(n+2)> = U <u^(n+1)> + (n+1)/(2 lam) <u^n>.
// ---------------------------------------------------------------------------
template <typename T> struct Mom {
  T u[7];
  T v[6];
  T x2, x4;
};

// A Maxwellian's constants shared by its moments and micro-coefficient
// solves: velocity, lam, h = 1/(2 lam), q = U^2 + V^2 + Kd h, c4 = 4 lam^2/Kd.
template <typename T> struct Frame {
  T U, V, lam, h, q, c4;
};

template <typename T, int D>
CGKS_HD __forceinline__ Frame<T> frame(T U, T V, T lam, T Kd, T iKd) {
  Frame<T> f;
  f.U = U;
  f.V = (D == 2) ? V : T(0);
  f.lam = lam;
  f.h = T(0.5) * dev_rcp<T>(lam);
  f.q = U * U + f.V * f.V + Kd * f.h;
  f.c4 = T(4) * lam * lam * iKd;
  return f;
}

template <typename T, int D>
CGKS_HD __forceinline__ void moments(const Frame<T>& f, T K, int region, Mom<T>& M) {
  const T U = f.U, h = f.h;
  if (region == 0) {
    M.u[0] = T(1);
    M.u[1] = U;
  } else {
    const T s = dev_sqrt<T>(f.lam);
    const T sg = T(region);
    M.u[0] = T(0.5) * dev_erfc<T>(-sg * s * U);
    // 1/(s sqrt(pi)) = rsqrt(lam) / sqrt(pi)
    M.u[1] = U * M.u[0] + sg * T(0.5 * 0.56418958354775628695) * dev_exp<T>(-f.lam * U * U) * dev_rsqrt<T>(f.lam);
  }
#pragma unroll
  for (int n = 2; n < 7; ++n) M.u[n] = U * M.u[n - 1] + T(n - 1) * h * M.u[n - 2];
  if (D == 2) {
    const T V = f.V;
    M.v[0] = T(1);
    M.v[1] = V;
#pragma unroll
    for (int n = 2; n < 6; ++n) M.v[n] = V * M.v[n - 1] + T(n - 1) * h * M.v[n - 2];
  }
  M.x2 = K * h;
  M.x4 = (K + T(2)) * h * M.x2;
}

// <a u^AL v^BE>, a = a0 + a1 u + a2 v + a3 (u^2+v^2+xi^2)/2 (2-D), or
// a0 + a1 u + a2 (u^2+xi^2)/2 (1-D)
template <typename T, int D, int AL, int BE>
CGKS_HD __forceinline__ T mS(const T* a, const Mom<T>& M) {
  if (D == 2) {
    const T g = M.u[AL] * M.v[BE];
    return a[0] * g + a[1] * M.u[AL + 1] * M.v[BE] + a[2] * M.u[AL] * M.v[BE + 1] +
           T(0.5) * a[3] * (M.u[AL + 2] * M.v[BE] + M.u[AL] * M.v[BE + 2] + g * M.x2);
  } else {
    return a[0] * M.u[AL] + a[1] * M.u[AL + 1] + T(0.5) * a[2] * (M.u[AL + 2] + M.u[AL] * M.x2);
  }
}

// <a u^AL v^BE xi^2>
template <typename T, int D, int AL, int BE>
CGKS_HD __forceinline__ T mSx(const T* a, const Mom<T>& M) {
  if (D == 2) {
    const T g = M.u[AL] * M.v[BE];
    return M.x2 * (a[0] * g + a[1] * M.u[AL + 1] * M.v[BE] + a[2] * M.u[AL] * M.v[BE + 1] +
                   T(0.5) * a[3] * (M.u[AL + 2] * M.v[BE] + M.u[AL] * M.v[BE + 2])) +
           T(0.5) * a[3] * g * M.x4;
  } else {
    return M.x2 * (a[0] * M.u[AL] + a[1] * M.u[AL + 1] + T(0.5) * a[2] * M.u[AL + 2]) +
           T(0.5) * a[2] * M.u[AL] * M.x4;
  }
}

// psi-moment vector <a u^AL v^BE psi> (normalised, no rho)
template <typename T, int D, int AL, int BE>
CGKS_HD __forceinline__ void mauv(const T* a, const Mom<T>& M, T* out) {
  if (D == 2) {
    out[0] = mS<T, D, AL, BE>(a, M);
    out[1] = mS<T, D, AL + 1, BE>(a, M);
    out[2] = mS<T, D, AL, BE + 1>(a, M);
    out[3] = T(0.5) * (mS<T, D, AL + 2, BE>(a, M) + mS<T, D, AL, BE + 2>(a, M) + mSx<T, D, AL, BE>(a, M));
  } else {
    out[0] = mS<T, D, AL, 0>(a, M);
    out[1] = mS<T, D, AL + 1, 0>(a, M);
    out[2] = T(0.5) * (mS<T, D, AL + 2, 0>(a, M) + mSx<T, D, AL, 0>(a, M));
  }
}

// The same moment vectors for a = 1: the terms of the general form with a
// zero coefficient are left out (they add exact zeros).
template <typename T, int D, int AL, int BE>
CGKS_HD __forceinline__ T mS1(const Mom<T>& M) {
  if (D == 2) return M.u[AL] * M.v[BE];
  return M.u[AL];
}

template <typename T, int D, int AL, int BE>
CGKS_HD __forceinline__ void mauv1(const Mom<T>& M, T* out) {
  if (D == 2) {
    const T g = mS1<T, D, AL, BE>(M);
    out[0] = g;
    out[1] = mS1<T, D, AL + 1, BE>(M);
    out[2] = mS1<T, D, AL, BE + 1>(M);
    out[3] = T(0.5) * (mS1<T, D, AL + 2, BE>(M) + mS1<T, D, AL, BE + 2>(M) + M.x2 * g);
  } else {
    out[0] = M.u[AL];
    out[1] = M.u[AL + 1];
    out[2] = T(0.5) * (M.u[AL + 2] + M.x2 * M.u[AL]);
  }
}

// Moment matrix of a weight w = u^AL v^BE: G[k][j] = <w psi_k psi_j> with
// psi = (1, u, v, (u^2+v^2+xi^2)/2) (1-D: (1, u, (u^2+xi^2)/2)), so that
// <a w psi> = G a for a = a0 + a1 u + a2 v + a3 (u^2+v^2+xi^2)/2: the same
// vector mauv gives, at a matrix-vector product per coefficient vector once
// G is built.  Symmetric; both halves are stored.
template <typename T> struct Gram {
  T g[4][4];
};

template <typename T, int D, int AL, int BE>
CGKS_HD __forceinline__ void gram(const Mom<T>& M, Gram<T>& G) {
  if (D == 2) {
    const T w00 = mS1<T, D, AL, BE>(M), u1 = mS1<T, D, AL + 1, BE>(M), v1 = mS1<T, D, AL, BE + 1>(M);
    const T u2 = mS1<T, D, AL + 2, BE>(M), v2 = mS1<T, D, AL, BE + 2>(M), uv = mS1<T, D, AL + 1, BE + 1>(M);
    const T e = T(0.5) * (u2 + v2 + M.x2 * w00);
    const T ue = T(0.5) * (mS1<T, D, AL + 3, BE>(M) + mS1<T, D, AL + 1, BE + 2>(M) + M.x2 * u1);
    const T ve = T(0.5) * (mS1<T, D, AL + 2, BE + 1>(M) + mS1<T, D, AL, BE + 3>(M) + M.x2 * v1);
    const T ee = T(0.25) * (mS1<T, D, AL + 4, BE>(M) + mS1<T, D, AL, BE + 4>(M) +
                            T(2) * mS1<T, D, AL + 2, BE + 2>(M) + T(2) * M.x2 * (u2 + v2) + M.x4 * w00);
    G.g[0][0] = w00; G.g[0][1] = u1;  G.g[0][2] = v1;  G.g[0][3] = e;
    G.g[1][0] = u1;  G.g[1][1] = u2;  G.g[1][2] = uv;  G.g[1][3] = ue;
    G.g[2][0] = v1;  G.g[2][1] = uv;  G.g[2][2] = v2;  G.g[2][3] = ve;
    G.g[3][0] = e;   G.g[3][1] = ue;  G.g[3][2] = ve;  G.g[3][3] = ee;
  } else {
    const T w00 = M.u[AL], u1 = M.u[AL + 1], u2 = M.u[AL + 2];
    const T e = T(0.5) * (u2 + M.x2 * w00);
    const T ue = T(0.5) * (M.u[AL + 3] + M.x2 * u1);
    const T ee = T(0.25) * (M.u[AL + 4] + T(2) * M.x2 * u2 + M.x4 * w00);
    G.g[0][0] = w00; G.g[0][1] = u1; G.g[0][2] = e;
    G.g[1][0] = u1;  G.g[1][1] = u2; G.g[1][2] = ue;
    G.g[2][0] = e;   G.g[2][1] = ue; G.g[2][2] = ee;
#pragma unroll
    for (int k = 0; k < 4; ++k) { G.g[3][k] = T(0); G.g[k][3] = T(0); }
  }
}

// out = G a (1-D: the three components; out[3] = 0)
template <typename T, int D>
CGKS_HD __forceinline__ void gmul(const Gram<T>& G, const T* a, T* out) {
  constexpr int NV = D + 2;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k >= NV) { out[k] = T(0); continue; }
    T s = G.g[k][0] * a[0];
#pragma unroll
    for (int j = 1; j < NV; ++j) s += G.g[k][j] * a[j];
    out[k] = s;
  }
}

// out += G a
template <typename T, int D>
CGKS_HD __forceinline__ void gmul_add(const Gram<T>& G, const T* a, T* out) {
  T t[4];
  gmul<T, D>(G, a, t);
#pragma unroll
  for (int k = 0; k < D + 2; ++k) out[k] += t[k];
}

// micro-coefficients a with <a psi> = b (normalised moments of g): closed-form
// inverse of the Maxwellian moment matrix, with the frame's constants.
template <typename T, int D>
CGKS_HD __forceinline__ void micro(const T* b, const Frame<T>& f, T* a) {
  const T U = f.U, tl = T(2) * f.lam;
  if (D == 2) {
    const T V = f.V;
    const T R2 = b[1] - U * b[0], R3 = b[2] - V * b[0], R4 = T(2) * b[3] - f.q * b[0];
    a[3] = f.c4 * (R4 - T(2) * U * R2 - T(2) * V * R3);
    a[2] = tl * R3 - V * a[3];
    a[1] = tl * R2 - U * a[3];
    a[0] = b[0] - U * a[1] - V * a[2] - T(0.5) * a[3] * f.q;
  } else {
    const T R2 = b[1] - U * b[0], R3 = T(2) * b[2] - f.q * b[0];
    a[2] = f.c4 * (R3 - T(2) * U * R2);
    a[1] = tl * R2 - U * a[2];
    a[0] = b[0] - U * a[1] - T(0.5) * a[2] * f.q;
    a[3] = T(0);
  }
}

// Raw moments of X = a u^AL v^BE that the heat flux needs:
// [X u^3, X u^2, X u, X, X u v^2, X u v, X v^2, X v, X u xi^2, X xi^2]
template <typename T, int D, int AL, int BE>
CGKS_HD __forceinline__ void qraw(const T* a, const Mom<T>& M, T* r) {
  r[0] = mS<T, D, AL + 3, BE>(a, M);
  r[1] = mS<T, D, AL + 2, BE>(a, M);
  r[2] = mS<T, D, AL + 1, BE>(a, M);
  r[3] = mS<T, D, AL, BE>(a, M);
  if (D == 2) {
    r[4] = mS<T, D, AL + 1, BE + 2>(a, M);
    r[5] = mS<T, D, AL + 1, BE + 1>(a, M);
    r[6] = mS<T, D, AL, BE + 2>(a, M);
    r[7] = mS<T, D, AL, BE + 1>(a, M);
  } else {
    r[4] = r[5] = r[6] = r[7] = T(0);
  }
  r[8] = mSx<T, D, AL + 1, BE>(a, M);
  r[9] = mSx<T, D, AL, BE>(a, M);
}

// Raw moments of X = u^AL v^BE (a = 1) that the heat flux needs, as qraw.
template <typename T, int D, int AL, int BE>
CGKS_HD __forceinline__ void qraw1(const Mom<T>& M, T* r) {
  r[0] = mS1<T, D, AL + 3, BE>(M);
  r[1] = mS1<T, D, AL + 2, BE>(M);
  r[2] = mS1<T, D, AL + 1, BE>(M);
  r[3] = mS1<T, D, AL, BE>(M);
  if (D == 2) {
    r[4] = mS1<T, D, AL + 1, BE + 2>(M);
    r[5] = mS1<T, D, AL + 1, BE + 1>(M);
    r[6] = mS1<T, D, AL, BE + 2>(M);
    r[7] = mS1<T, D, AL, BE + 1>(M);
  } else {
    r[4] = r[5] = r[6] = r[7] = T(0);
  }
  r[8] = M.x2 * r[2];
  r[9] = M.x2 * r[3];
}

// Heat-flux moments over the equilibrium g0 itself (full space, mean (U0,
// V0), variance s = 1/(2 lam0)), in closed form.  With c = u - U0,
// w = v - V0, E = (c^2 + w^2 + xi^2)/2, a polynomial
// a = a0 + a1 u + a2 v + a3 (u^2 + v^2 + xi^2)/2 reads A0 + B1 c + B2 w + a3 E
// with B1 = a1 + a3 U0 and A0 = a0 + a1 U0 + a2 V0 + a3 (U0^2 + V0^2)/2; the
// odd central moments of the Gaussian vanish, which leaves
//   <a c E> = B1 Q2,   <a u c E> = (U0 B1 + A0) Q2 + a3 Q3,   <a v c E> = V0 B1 Q2,
// Q2 = <c^2 E> = (Kd + 2) s^2 / 2 and Q3 = <c^2 E^2> = (Kd + 2)(Kd + 4) s^3 / 4
// (Kd = K + D; the same in 1-D, where a = a0 + a1 u + a2 (u^2 + xi^2)/2).
template <typename T, int D>
CGKS_HD __forceinline__ void heat_split(const T* a, T U0, T V0, T& B1, T& A0, T& a3) {
  a3 = D == 2 ? a[3] : a[2];
  const T a2 = D == 2 ? a[2] : T(0);
  B1 = a[1] + a3 * U0;
  A0 = a[0] + a[1] * U0 + a2 * V0 + T(0.5) * a3 * (U0 * U0 + V0 * V0);
}

// <X (u-U0)/2 ((u-U0)^2 + (v-V0)^2 + xi^2)> from the raw moments of X
template <typename T, int D>
CGKS_HD __forceinline__ T qcomb(const T* r, T U0, T V0) {
  T q = r[0] - T(3) * U0 * r[1] + T(3) * U0 * U0 * r[2] - U0 * U0 * U0 * r[3] + r[8] - U0 * r[9];
  if (D == 2) q += r[4] - T(2) * V0 * r[5] + V0 * V0 * r[2] - U0 * r[6] + T(2) * U0 * V0 * r[7] - U0 * V0 * V0 * r[3];
  return T(0.5) * q;
}

template <typename T, int D>
CGKS_HD __forceinline__ void primitive(const T* W, T gm1, T& rho, T& U, T& V, T& p) {
  rho = W[0];
  const T ir = dev_rcp<T>(rho);
  U = W[1] * ir;
  V = (D == 2) ? W[2] * ir : T(0);
  const T ke = T(0.5) * rho * (U * U + V * V);
  p = gm1 * (W[D + 1] - ke);
}

// rho > 0 and p > 0, without a division: p > 0 <=> rho E > |rho u|^2 / 2
template <typename T, int D>
CGKS_HD __forceinline__ bool positive_state(const T* W) {
  const T m2 = W[1] * W[1] + ((D == 2) ? W[2] * W[2] : T(0));
  return (W[0] > T(0)) && (W[0] * W[D + 1] - T(0.5) * m2 > T(0));
}

// Results of one Gauss point, in double.
struct FaceOut {
  double Fh[4], F1[4];     // time integrals of the flux over [0, dt/2] and [0, dt]
  double W0[4], Wh[4], W1[4];  // interface values at 0, dt/2, dt
  double sigma;            // discontinuity strength, Eq. 3.2
};

// Interface flux at one Gauss point (normal = local x).  Wk[d][v]: d = 0 value,
// 1 d/dn, 2 d/dt, 3 d2/dn2, 4 d2/dndt, 5 d2/dt2; components in the face frame
// (rho, rho u_n, [rho u_t,] rho E).  PR: apply the Prandtl-number fix of the
// energy flux, (1/Pr - 1) times the time-integrated heat flux in the frame of
// the equilibrium velocity (the standard gas-kinetic correction; not part of
// the paper).
template <typename T, int D, bool PR = false>
CGKS_HD void gks_flux(const T (&Wl)[6][4], const T (&Wr)[6][4], double dt, const Consts& C, FaceOut& o) {
  constexpr int NV = D + 2;
  const T gm1 = T(C.gamma - 1.0), Kd = T(C.Kd), iKd = T(C.iKd), K = T(C.Kd - D);
  T Q0[4] = {0, 0, 0, 0}, dQ[5][4], NF0[4] = {0, 0, 0, 0}, NF1[4] = {0, 0, 0, 0}, NW1[4] = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 5; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) dQ[q][v] = T(0);
  // per side: pressure, and the normal and tangential Mach numbers of
  // Eq. 3.2; the sum of the reciprocal pressures
  T pside[2], ma[2], mt[2], ipsum = T(0);
  T QR0[10], QR1[10];
  if (PR) {
#pragma unroll
    for (int k = 0; k < 10; ++k) QR0[k] = QR1[k] = T(0);
  }

#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const T(&Wk)[6][4] = side == 0 ? Wl : Wr;
    T rho, U, V, p;
    primitive<T, D>(Wk[0], gm1, rho, U, V, p);
    const T ip = dev_rcp<T>(p), ir = dev_rcp<T>(rho);
    const T lam = T(0.5) * rho * ip;
    pside[side] = p;
    ipsum += ip;
    const T ic = dev_rsqrt<T>(T(C.gamma) * p * ir);   // 1 / sound speed
    ma[side] = U * ic;
    mt[side] = V * ic;
    const Frame<T> fr = frame<T, D>(U, V, lam, Kd, iKd);
    Mom<T> M;
    moments<T, D>(fr, K, side == 0 ? 1 : -1, M);
    T t4[4];
    // <psi_k psi_j> over this half space: <psi> and <u psi> are its columns
    // 0 and 1, and <a psi> = G a for every derivative below
    Gram<T> G0;
    gram<T, D, 0, 0>(M, G0);
#pragma unroll
    for (int v = 0; v < NV; ++v) Q0[v] += rho * G0.g[v][0];
#pragma unroll
    for (int v = 0; v < NV; ++v) NF0[v] += rho * G0.g[v][1];
    if (PR) {
      T r10[10];
      qraw1<T, D, 0, 0>(M, r10);
#pragma unroll
      for (int k = 0; k < 10; ++k) QR0[k] += rho * r10[k];
    }
    // derivative sources: 1 n, 2 t, 3 nn, 4 nt, 5 tt (1-D: n, nn)
    constexpr int NDER = (D == 2) ? 5 : 2;
#pragma unroll
    for (int q = 0; q < NDER; ++q) {
      const int d = (D == 2) ? q + 1 : (q == 0 ? 1 : 3);
      T b[4], a[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = (v < NV) ? Wk[d][v] * ir : T(0);
      micro<T, D>(b, fr, a);
      gmul<T, D>(G0, a, t4);
#pragma unroll
      for (int v = 0; v < NV; ++v) dQ[q][v] += rho * t4[v];
      if (q == 0) {
        mauv<T, D, 2, 0>(a, M, t4);
#pragma unroll
        for (int v = 0; v < NV; ++v) NF1[v] += rho * t4[v];
        mauv<T, D, 1, 0>(a, M, t4);
#pragma unroll
        for (int v = 0; v < NV; ++v) NW1[v] += rho * t4[v];
        if (PR) {
          T r10[10];
          qraw<T, D, 1, 0>(a, M, r10);
#pragma unroll
          for (int k = 0; k < 10; ++k) QR1[k] += rho * r10[k];
        }
      }
      if (D == 2 && q == 1) {
        mauv<T, D, 1, 1>(a, M, t4);
#pragma unroll
        for (int v = 0; v < NV; ++v) NF1[v] += rho * t4[v];
        mauv<T, D, 0, 1>(a, M, t4);
#pragma unroll
        for (int v = 0; v < NV; ++v) NW1[v] += rho * t4[v];
        if (PR) {
          T r10[10];
          qraw<T, D, 0, 1>(a, M, r10);
#pragma unroll
          for (int k = 0; k < 10; ++k) QR1[k] += rho * r10[k];
        }
      }
    }
  }

  // equilibrium state at the interface (kinetic weighting, Eq. 2.7)
  T rho0, U0, V0, p0;
  primitive<T, D>(Q0, gm1, rho0, U0, V0, p0);
  const T lam0 = T(0.5) * rho0 * dev_rcp<T>(p0);
  const Frame<T> f0 = frame<T, D>(U0, V0, lam0, Kd, iKd);
  Mom<T> M0;
  moments<T, D>(f0, K, 0, M0);
  const T ir0 = dev_rcp<T>(rho0);
  T ab[5][4];
  constexpr int NDER = (D == 2) ? 5 : 2;
#pragma unroll
  for (int q = 0; q < NDER; ++q) {
    T b[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) b[v] = (v < NV) ? dQ[q][v] * ir0 : T(0);
    micro<T, D>(b, f0, ab[q]);
  }
  // ab index: 2-D 0 n, 1 t, 2 nn, 3 nt, 4 tt; 1-D 0 n, 1 nn
  const T* an = ab[0];
  const T* ann = (D == 2) ? ab[2] : ab[1];
  T bA[4], AT[4], b1[4], anT[4], atT[4], bTT[4], ATT[4];
  // moment matrices of g0 for the weights u, v, u^2, u v: each serves
  // several coefficient vectors below
  Gram<T> Gu, Gv;
  gram<T, D, 1, 0>(M0, Gu);
  if (D == 2) gram<T, D, 0, 1>(M0, Gv);
  // <an u + at v + A> = 0
  gmul<T, D>(Gu, an, bA);
  if (D == 2) gmul_add<T, D>(Gv, ab[1], bA);
#pragma unroll
  for (int v = 0; v < 4; ++v) bA[v] = -bA[v];
  micro<T, D>(bA, f0, AT);
  // <ann u + ant v + anT> = 0, <ant u + att v + atT> = 0
  gmul<T, D>(Gu, ann, b1);
  if (D == 2) gmul_add<T, D>(Gv, ab[3], b1);
#pragma unroll
  for (int v = 0; v < 4; ++v) b1[v] = -b1[v];
  micro<T, D>(b1, f0, anT);
  if (D == 2) {
    gmul<T, D>(Gu, ab[3], b1);
    gmul_add<T, D>(Gv, ab[4], b1);
#pragma unroll
    for (int v = 0; v < 4; ++v) b1[v] = -b1[v];
    micro<T, D>(b1, f0, atT);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) atT[v] = T(0);
  }
  // <anT u + atT v + ATT> = 0
  gmul<T, D>(Gu, anT, bTT);
  if (D == 2) gmul_add<T, D>(Gv, atT, bTT);
#pragma unroll
  for (int v = 0; v < 4; ++v) bTT[v] = -bTT[v];
  micro<T, D>(bTT, f0, ATT);

  // flux moments of the equilibrium part (normalised): <u psi> is column 0
  // of Gu; the u^2 and u v weights take matrices of their own
  T F0[4], FA[4], F1[4], Ft[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) F0[v] = v < NV ? Gu.g[v][0] : T(0);
  gmul<T, D>(Gu, AT, FA);
  gmul<T, D>(Gu, ATT, Ft);
  {
    Gram<T> Guu;
    gram<T, D, 2, 0>(M0, Guu);
    gmul<T, D>(Guu, an, F1);
    gmul_add<T, D>(Guu, anT, Ft);
  }
  if (D == 2) {
    Gram<T> Guv;
    gram<T, D, 1, 1>(M0, Guv);
    gmul_add<T, D>(Guv, ab[1], F1);
    gmul_add<T, D>(Guv, atT, Ft);
  }

  // heat-flux moments of the Prandtl fix
  T hA = T(0), hP1 = T(0), hPt = T(0), hN0 = T(0), hN1 = T(0);
  if (PR) {
    // terms over g0: closed forms (heat_split); terms over the half-space
    // initial states: raw moments, shifted to the frame of (U0, V0)
    const T s0 = f0.h;
    const T Q2 = T(0.5) * (Kd + T(2)) * s0 * s0;
    const T Q3 = T(0.25) * (Kd + T(2)) * (Kd + T(4)) * s0 * s0 * s0;
    T B1, A0, a3, B1t, A0t, a3t;
    heat_split<T, D>(AT, U0, V0, B1, A0, a3);
    hA = B1 * Q2;
    heat_split<T, D>(an, U0, V0, B1, A0, a3);
    hP1 = (U0 * B1 + A0) * Q2 + a3 * Q3;
    if (D == 2) {
      heat_split<T, D>(ab[1], U0, V0, B1t, A0t, a3t);
      hP1 += V0 * B1t * Q2;
    }
    heat_split<T, D>(anT, U0, V0, B1, A0, a3);
    hPt = (U0 * B1 + A0) * Q2 + a3 * Q3;
    heat_split<T, D>(ATT, U0, V0, B1, A0, a3);
    hPt += B1 * Q2;
    if (D == 2) {
      heat_split<T, D>(atT, U0, V0, B1t, A0t, a3t);
      hPt += V0 * B1t * Q2;
    }
    hN0 = qcomb<T, D>(QR0, U0, V0);
    hN1 = qcomb<T, D>(QR1, U0, V0);
  }

  // collision time (Sec. 4); the pressure jump in the working precision,
  // tau and its reciprocal in double (they enter the exponential weights)
  const T dpT = fabs(pside[0] - pside[1]);
  const double jump = double(dpT * dev_rcp<T>(pside[0] + pside[1]));
  double tau = 0.0;
  if (C.tau_model == 1) tau = C.c1 * dt + C.c2 * jump * dt;
  else if (C.tau_model == 2) tau = C.mu * double(dev_rcp<T>(p0)) + C.c2 * jump * dt;
  const double itau = tau > 0.0 ? dev_rcp<double>(tau) : 0.0;

  // time integrals (the flux keeps the terms up to first order in t of the
  // equilibrium part; interface values keep the full quadratic)
  const double r0 = double(rho0);
  double ex[2] = {0.0, 0.0};   // exp(-dt/(2 tau)), exp(-dt/tau); 0 when tau = 0
  double emh = 0.0;             // expm1(-dt/(2 tau))
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const double d = w == 0 ? 0.5 * dt : dt;
    double E0 = 0.0, E1 = 0.0;
    if (tau > 0.0) {
      // the full step's exponentials from the half step's: exp(-2x) =
      // exp(-x)^2 and expm1(-2x) = expm1(-x) (2 + expm1(-x)), free of
      // cancellation for small x
      double e, em;
      if (w == 0) {
        const double x = d * itau;
        e = exp(-x);
        em = expm1(-x);
        emh = em;
      } else {
        e = ex[0] * ex[0];
        em = emh * (2.0 + emh);
      }
      ex[w] = e;
      E0 = -tau * em;
      E1 = tau * tau - tau * (tau + d) * e;
    }
    double* Fo = w == 0 ? o.Fh : o.F1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (v >= NV) { Fo[v] = 0.0; continue; }
      const double f1 = double(F1[v]), fa = double(FA[v]);
      Fo[v] = r0 * (double(F0[v]) * (d - E0) + fa * 0.5 * d * d - tau * ((f1 + fa) * d + double(Ft[v]) * 0.5 * d * d) +
                    f1 * E1) +
              double(NF0[v]) * E0 - double(NF1[v]) * E1;
    }
    if (PR) {
      const double ha = double(hA), hp = double(hP1);
      const double q = r0 * (ha * 0.5 * d * d - tau * ((hp + ha) * d + double(hPt) * 0.5 * d * d) + hp * E1) +
                       double(hN0) * E0 - double(hN1) * E1;
      Fo[NV - 1] += C.prfac * q;
    }
  }
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    const double t = w == 0 ? 0.0 : (w == 1 ? 0.5 * dt : dt);
    const double e = w == 0 ? 1.0 : ex[w - 1];   // exp(-t/tau)
    double* Wo = w == 0 ? o.W0 : (w == 1 ? o.Wh : o.W1);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (v >= NV) { Wo[v] = 0.0; continue; }
      Wo[v] = double(Q0[v]) + r0 * double(bA[v]) * t * (1.0 - e) + 0.5 * r0 * double(bTT[v]) * t * t -
              t * e * double(NW1[v]);
    }
  }
  // discontinuity strength (Eq. 3.2), in the working precision
  {
    const T dn = ma[0] - ma[1];
    const T dtn = (D == 2) ? mt[0] - mt[1] : T(0);
    o.sigma = double(dpT * ipsum + dn * dn + dtn * dtn);
  }
}

// ---------------------------------------------------------------------------
// Discontinuity feedback factor and the stencil cascade (Eq. 3.3, 3.4,
// Algorithm 1).  s[f], f = 0..5: strengths of faces -5/2 .. +5/2 around the
// cell (face -5/2 at index 0).  eta = 2 on the faces of cells whose gradient
// the stencil uses.
// ---------------------------------------------------------------------------
struct Cascade {
  int branch;          // 0: AO(5,3); 5, 7, 9: linear stencil of that order
  bool tie;            // a decision taken with A within the tie band of the threshold
  double al[4];        // AO: DFF of S0, S1, S2 and of the 5th-order stencil
};

CGKS_HD __forceinline__ double dff_of(double A, double thres) { return (A < thres) ? 1.0 : thres / A; }

// tie: half-width of the band around the threshold in which a decision
// counts as a near tie (rounding of the strengths can move A across it).
// Only the decisions the cascade takes are judged; the DFF values
// themselves are continuous in A.
// A decision "DFF below 1" is taken as A > thres: for a positive threshold
// and a finite A it is the same test (thres / A rounds below 1 exactly when
// A > thres), without a division where the stencil is kept.
CGKS_HD __forceinline__ Cascade cascade(const double* s, int order, double thres, double tie) {
  Cascade c;
  const double A5 = 2.0 * s[1] + 2.0 * s[2] + 2.0 * s[3] + 2.0 * s[4];
  c.tie = fabs(A5 - thres) <= tie;
  if (A5 > thres) {
    c.branch = 0;
    c.al[0] = dff_of(2.0 * s[1] + 2.0 * s[2] + s[3], thres);
    c.al[1] = dff_of(s[2] + 2.0 * s[3] + 2.0 * s[4], thres);
    c.al[2] = dff_of(s[1] + s[2] + s[3] + s[4], thres);
    c.al[3] = thres / A5;
    return c;
  }
  if (order == 5) { c.branch = 5; return c; }
  const double A7 = s[0] + 2.0 * s[1] + 2.0 * s[2] + 2.0 * s[3] + 2.0 * s[4] + s[5];
  c.tie = c.tie || fabs(A7 - thres) <= tie;
  if (A7 > thres) { c.branch = 5; return c; }
  if (order == 7) { c.branch = 7; return c; }
  const double A9 = 2.0 * s[0] + 2.0 * s[1] + 2.0 * s[2] + 2.0 * s[3] + 2.0 * s[4] + 2.0 * s[5];
  c.tie = c.tie || fabs(A9 - thres) <= tie;
  c.branch = A9 > thres ? 7 : 9;
  return c;
}

// AO(5,3) with DFF-scaled members (Eq. 3.11-3.17, 3.19) collapsed into one
// quartic in xi: P = Q0 (1 - sum w_k al_k) + sum w_k al_k p_k, with
// w_3 = omega_3/g_3 and w_k = omega_k - omega_3 g_k/g_3.
template <typename T>
CGKS_HD __forceinline__ void ao_poly(const T* d, const Cascade& cs, const Consts& C, T* P) {
  T c0[3], c1[3], c2[3], c3[5];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T a = 0, b = 0, e = 0;
#pragma unroll
    for (int s = 0; s < 9; ++s) {
      a += T(kC_S0[k][s]) * d[s];
      b += T(kC_S1[k][s]) * d[s];
      e += T(kC_S2[k][s]) * d[s];
    }
    c0[k] = a; c1[k] = b; c2[k] = e;
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    T a = 0;
#pragma unroll
    for (int s = 0; s < 9; ++s) a += T(kC_R5[k][s]) * d[s];
    c3[k] = a;
  }
  // smoothness indicators (Eq. 3.13 in xi units) of the unscaled members
  const T b0 = c0[1] * c0[1] + T(13.0 / 3.0) * c0[2] * c0[2];
  const T b1 = c1[1] * c1[1] + T(13.0 / 3.0) * c1[2] * c1[2];
  const T b2 = c2[1] * c2[1] + T(13.0 / 3.0) * c2[2] * c2[2];
  const T q1 = c3[1], q2 = c3[2], q3 = c3[3], q4 = c3[4];
  const T b3 = q1 * q1 + (T(4) * q2 * q2 + T(6) * q1 * q3) * T(1.0 / 12) +
               (T(9) * q3 * q3 + T(16) * q2 * q4) * T(1.0 / 80) + T(16) * q4 * q4 * T(1.0 / 448) + T(4) * q2 * q2 +
               (T(36) * q3 * q3 + T(48) * q2 * q4) * T(1.0 / 12) + T(144) * q4 * q4 * T(1.0 / 80) + T(36) * q3 * q3 +
               T(48) * q4 * q4 + T(576) * q4 * q4;
  // the DFF scaling of a member scales its indicator by alpha^2 (the
  // alternative reading takes the indicators of the unscaled members)
  const T al0 = T(cs.al[0]), al1 = T(cs.al[1]), al2 = T(cs.al[2]), al3 = T(cs.al[3]);
  const bool unscaled = (C.rflags & RF_A5_UNSCALED_BETA) != 0;
  const T B0 = unscaled ? b0 : al0 * al0 * b0, B1 = unscaled ? b1 : al1 * al1 * b1;
  const T B2 = unscaled ? b2 : al2 * al2 * b2, B3 = unscaled ? b3 : al3 * al3 * b3;
  const T g3 = T(C.ghi), g0 = T(C.gw[0]), g1 = T(C.gw[1]), g2 = T(C.gw[2]);
  const T tz = (fabs(B3 - B0) + fabs(B3 - B1) + fabs(B3 - B2)) * T(1.0 / 3);
  const T eps = T(C.eps);
  T r;
  r = tz * dev_rcp<T>(B0 + eps); const T w0 = g0 * (T(1) + r * r);
  r = tz * dev_rcp<T>(B1 + eps); const T w1 = g1 * (T(1) + r * r);
  r = tz * dev_rcp<T>(B2 + eps); const T w2 = g2 * (T(1) + r * r);
  r = tz * dev_rcp<T>(B3 + eps); const T w3 = g3 * (T(1) + r * r);
  const T ws = dev_rcp<T>(w0 + w1 + w2 + w3);
  const T o0 = w0 * ws, o1 = w1 * ws, o2 = w2 * ws, o3 = w3 * ws;
  const T k3 = o3 * T(1.0 / C.ghi);
  const T k0 = (o0 - k3 * g0) * al0, k1 = (o1 - k3 * g1) * al1, k2 = (o2 - k3 * g2) * al2, kk3 = k3 * al3;
  P[0] = d[2] * (T(1) - k0 - k1 - k2 - kk3) + k0 * c0[0] + k1 * c1[0] + k2 * c2[0] + kk3 * c3[0];
  P[1] = k0 * c0[1] + k1 * c1[1] + k2 * c2[1] + kk3 * c3[1];
  P[2] = k0 * c0[2] + k1 * c1[2] + k2 * c2[2] + kk3 * c3[2];
  P[3] = kk3 * c3[3];
  P[4] = kk3 * c3[4];
}

template <typename T>
CGKS_HD __forceinline__ T poly4(const T* P, T x, int deriv) {
  if (deriv == 0) return P[0] + x * (P[1] + x * (P[2] + x * (P[3] + x * P[4])));
  if (deriv == 1) return P[1] + x * (T(2) * P[2] + x * (T(3) * P[3] + x * T(4) * P[4]));
  return T(2) * P[2] + x * (T(6) * P[3] + x * T(12) * P[4]);
}

// A linear stencil (5th, 7th or 9th order) at both faces: value, d, d2
template <typename T, int NVAR, int K>
CGKS_HD __forceinline__ void lin_faces(const T (&d)[NVAR][9], T (&out)[2][3][NVAR]) {
  constexpr const double(&F)[2][3][9] = K == 5 ? kF_R5 : (K == 7 ? kF_R7 : kF_R9);
#pragma unroll
  for (int v = 0; v < NVAR; ++v)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) {
        T a = 0;
#pragma unroll
        for (int s = 0; s < 9; ++s)
          if (F[sd][dd][s] != 0.0) a += T(F[sd][dd][s]) * d[v][s];
        out[sd][dd][v] = a;
      }
}

// value, d/dxi and d2/dxi2 at xi = +1/2 (side 0) and xi = -1/2 (side 1) of
// every component; d[v][9] are the stencil data of component v.
template <typename T, int NVAR>
CGKS_HD __forceinline__ void recon_faces(const T (&d)[NVAR][9], const Cascade& cs, const Consts& C,
                                            T (&out)[2][3][NVAR]) {
  switch (cs.branch) {
    case 0:
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        T P[5];
        ao_poly<T>(d[v], cs, C, P);
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
          out[0][dd][v] = poly4<T>(P, T(0.5), dd);
          out[1][dd][v] = poly4<T>(P, T(-0.5), dd);
        }
      }
      return;
    case 5: lin_faces<T, NVAR, 5>(d, out); return;
    case 7: lin_faces<T, NVAR, 7>(d, out); return;
    default: lin_faces<T, NVAR, 9>(d, out); return;
  }
}

// A linear stencil at the M Gauss points of the cell
template <typename T, int NVAR, int M, int K>
CGKS_HD __forceinline__ void lin_nodes(const T (&d)[NVAR][9], T (&out)[4][NVAR]) {
  constexpr const double(&N)[5][4][9] = K == 5 ? kN_R5 : (K == 7 ? kN_R7 : kN_R9);
#pragma unroll
  for (int v = 0; v < NVAR; ++v)
#pragma unroll
    for (int l = 0; l < M; ++l) {
      T a = 0;
#pragma unroll
      for (int s = 0; s < 9; ++s)
        if (N[M][l][s] != 0.0) a += T(N[M][l][s]) * d[v][s];
      out[l][v] = a;
    }
}

// values at the M Gauss points of the cell
template <typename T, int NVAR, int M>
CGKS_HD __forceinline__ void recon_nodes(const T (&d)[NVAR][9], const Cascade& cs, const Consts& C,
                                            T (&out)[4][NVAR]) {
  switch (cs.branch) {
    case 0:
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        T P[5];
        ao_poly<T>(d[v], cs, C, P);
#pragma unroll
        for (int l = 0; l < M; ++l) out[l][v] = poly4<T>(P, T(kGx[M][l]), 0);
      }
      return;
    case 5: lin_nodes<T, NVAR, M, 5>(d, out); return;
    case 7: lin_nodes<T, NVAR, M, 7>(d, out); return;
    default: lin_nodes<T, NVAR, M, 9>(d, out); return;
  }
}

}  // inline namespace CGKS_UNIT
}  // namespace cgks
