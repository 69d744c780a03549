// Device code of the per-stage residual: ghost fill, edge flux (non-uniform
// WENO5 on characteristic variables + numerical flux), vertex least-squares
// divergence with the fused SSP-RK3 stage update, CFL reduction.
#pragma once

#include <hip/hip_runtime.h>

// Per-item math is host+device so the host tests can check it on the CPU;
// memory access and scheduling live in the __global__ kernels only.
#define FDU_HD __host__ __device__ __forceinline__

namespace fdu {

struct Scheme {
  double gamma;   // ratio of specific heats
  double gm1;     // gamma - 1
  double eps;     // WENO epsilon
  double efrac;   // Harten entropy-fix width as a fraction of the Roe sound speed
  int power;      // WENO power (1 or 2)
  int riemann;    // 0 Roe + Harten, 1 Rusanov
  int positivity; // 1: a non-physical interpolated state falls back to its end vertex state
  int conservative;  // 1: interpolate conservative instead of characteristic variables
  int uniform;       // 1: standard WENO5 (equally spaced nodes) instead of NU-WENO5
};

// Outer stencil nodes (L3, L2, R2, R3) in units of the middle-edge length:
// the arc coordinates, or the equally spaced nodes of standard WENO5.
FDU_HD void weno_nodes(const double g[6], const Scheme& S, double x[4]) {
  if (S.uniform) {
    x[0] = -2.5; x[1] = -1.5; x[2] = 1.5; x[3] = 2.5;
  } else {
    x[0] = g[0]; x[1] = g[1]; x[2] = g[2]; x[3] = g[3];
  }
}

// ----------------------------------------------------------------------------
// State access: array of structures [n][4]; one 32-byte (double) or 16-byte
// (float) vector load per vertex.
__device__ __forceinline__ void load4(const double* __restrict__ w, int v, double q[4]) {
  const double2* p = reinterpret_cast<const double2*>(w + 4 * (size_t)v);
  double2 a = p[0], b = p[1];
  q[0] = a.x; q[1] = a.y; q[2] = b.x; q[3] = b.y;
}
__device__ __forceinline__ void load4(const float* __restrict__ w, int v, double q[4]) {
  float4 a = reinterpret_cast<const float4*>(w)[v];
  q[0] = a.x; q[1] = a.y; q[2] = a.z; q[3] = a.w;
}
__device__ __forceinline__ void store4(double* __restrict__ w, int v, const double q[4]) {
  double2* p = reinterpret_cast<double2*>(w + 4 * (size_t)v);
  p[0] = make_double2(q[0], q[1]);
  p[1] = make_double2(q[2], q[3]);
}
__device__ __forceinline__ void store4(float* __restrict__ w, int v, const double q[4]) {
  reinterpret_cast<float4*>(w)[v] = make_float4((float)q[0], (float)q[1], (float)q[2], (float)q[3]);
}


// Reciprocal: the hardware estimate (relative error ~5e-8 on gfx950) refined by
// one Newton step (~2e-15 relative, 10 ulp at most over a 2^20-sample sweep
// of 1e-3..1e3 magnitudes); used where the lean kernels divide.
__device__ __forceinline__ double frcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// Square root of x > 0 (normal range): the hardware reciprocal square root
// estimate r ~ (1 + d)/sqrt(x), then one Goldschmidt step (y = x r, h = r/2,
// e = 1/2 - y h; y += y e, h += h e: error O(d^2)) and one residual correction
// y += h (x - y^2) (error O(d^3) plus rounding).
__device__ __forceinline__ double fsqrt(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  double y = x * r, h = 0.5 * r;
  const double e = fma(-y, h, 0.5);
  y = fma(y, e, y);
  h = fma(h, e, h);
  return fma(fma(-y, y, x), h, y);
}

// 1/x: IEEE division, or (FR, device code) the refined hardware reciprocal.
template <bool FR>
FDU_HD double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (FR) return frcp(x);
#endif
  return 1.0 / x;
}

// sqrt(x): the library square root, or (FR, device code) fsqrt.
template <bool FR>
FDU_HD double root(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (FR) return fsqrt(x);
#endif
  return sqrt(x);
}

// Euler fluxes f, g of a conservative state (Sec. 2.1); FR: 1/rho from the
// refined hardware reciprocal.
template <bool FR = false>
FDU_HD void euler_fg(const double q[4], double gm1, double f[4], double g[4]) {
  const double ir = recip<FR>(q[0]);
  const double u = q[1] * ir, v = q[2] * ir;
  const double p = gm1 * (q[3] - 0.5 * (q[1] * u + q[2] * v));
  f[0] = q[1]; f[1] = q[1] * u + p; f[2] = q[1] * v; f[3] = (q[3] + p) * u;
  g[0] = q[2]; g[1] = q[2] * u;     g[2] = q[2] * v + p; g[3] = (q[3] + p) * v;
}

// Sum over aligned groups of LPV consecutive lanes (LPV = 2, 4, 8 or 16),
// every lane of a group receiving the group's sum: DPP lane permutations
// within a row of 16 lanes (mirror, half-row mirror, quad swaps), no LDS
// traffic.  The four steps pair disjoint lane sets, so each lane's value
// enters once.  All lanes of the wave must execute it.
__device__ __forceinline__ double dpp_add(double x, int ctrl_sel) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  switch (ctrl_sel) {
    case 0: lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false);   // row mirror
            hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false); break;
    case 1: lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);   // half-row mirror
            hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false); break;
    case 2: lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);    // quad_perm(2, 3, 0, 1)
            hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false); break;
    default: lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);   // quad_perm(1, 0, 3, 2)
             hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
  }
  return x + __hiloint2double(hi, lo);
}

template <int LPV>
__device__ __forceinline__ double group_sum(double x) {
  static_assert(LPV == 2 || LPV == 4 || LPV == 8 || LPV == 16, "group of 2, 4, 8 or 16 lanes");
  if (LPV >= 16) x = dpp_add(x, 0);
  if (LPV >= 8) x = dpp_add(x, 1);
  if (LPV >= 4) x = dpp_add(x, 2);
  return dpp_add(x, 3);
}

// Opaque copy of a value: the compiler cannot merge a computation on it with
// an earlier identical one, so recomputing (cheap) replaces keeping the
// earlier result live across the whole reverse sweep (registers).
FDU_HD double opaque(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(x));
#endif
  return x;
}
FDU_HD int opaque(int x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(x));
#endif
  return x;
}

// ----------------------------------------------------------------------------
// Non-uniform WENO5 midpoint interpolation (Appendix).  Coordinates are
// normalised by the middle-edge length, so x2 = -1/2 and x3 = +1/2 exactly and
// the smoothness-indicator interval is [-1/2, 1/2] with dx = 1.
struct WenoGeom {
  double I[3][3];   // sub-stencil interpolation weights at 0 (Lagrange basis values)
  double D1[3][3];  // first derivatives of the Lagrange basis at 0
  double D2[3][3];  // second derivatives of the Lagrange basis
  double C[3];      // optimal linear weights
};

// x0, x1, x4: the outer nodes (x2 = -1/2, x3 = 1/2).
FDU_HD void weno_geom(double x0, double x1, double x4, WenoGeom& G) {
  const double x2 = -0.5, x3 = 0.5;
  const double xs[5] = {x0, x1, x2, x3, x4};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double a = xs[k], b = xs[k + 1], c = xs[k + 2];
    const double ia = 1.0 / ((a - b) * (a - c));
    const double ib = 1.0 / ((b - a) * (b - c));
    const double ic = 1.0 / ((c - a) * (c - b));
    G.I[k][0] = b * c * ia;  G.I[k][1] = a * c * ib;  G.I[k][2] = a * b * ic;
    G.D1[k][0] = -(b + c) * ia;  G.D1[k][1] = -(a + c) * ib;  G.D1[k][2] = -(a + b) * ic;
    G.D2[k][0] = 2.0 * ia;  G.D2[k][1] = 2.0 * ib;  G.D2[k][2] = 2.0 * ic;
  }
  // linear weights: C0 and C2 from their closed forms, C1 = 1 - C0 - C2
  const double i40 = 1.0 / (x4 - x0);
  G.C[0] = x3 * x4 * i40 / (x3 - x0);
  G.C[2] = x0 * x1 * i40 / (x4 - x1);
  G.C[1] = 1.0 - G.C[0] - G.C[2];
}

// Nonlinear interpolant at 0 from values u[0..4] at the five nodes.
FDU_HD double weno_eval(const WenoGeom& G, const double u[5], double eps, int power) {
  double ut[3], b[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double u0 = u[k], u1 = u[k + 1], u2 = u[k + 2];
    ut[k] = G.I[k][0] * u0 + G.I[k][1] * u1 + G.I[k][2] * u2;
    const double d1 = G.D1[k][0] * u0 + G.D1[k][1] * u1 + G.D1[k][2] * u2;
    const double d2 = G.D2[k][0] * u0 + G.D2[k][1] * u1 + G.D2[k][2] * u2;
    // beta = int_{-1/2}^{1/2} (q'^2 + q''^2) dx = q'(0)^2 + (13/12) q''^2
    b[k] = d1 * d1 + (13.0 / 12.0) * d2 * d2 + eps;
    if (power == 2) b[k] *= b[k];
  }
  // omega_k proportional to C_k / b_k: multiply through by b0 b1 b2
  const double n0 = G.C[0] * b[1] * b[2];
  const double n1 = G.C[1] * b[0] * b[2];
  const double n2 = G.C[2] * b[0] * b[1];
  return (n0 * ut[0] + n1 * ut[1] + n2 * ut[2]) / (n0 + n1 + n2);
}

// ----------------------------------------------------------------------------
// Forward-mode dual numbers: value plus N directional derivatives.  The frame
// and flux functions below are templates on the scalar type; the adjoint's
// vertex kernel takes the Euler flux Jacobians with N = 4.
using ::fabs;
using ::sqrt;

template <int N>
struct Dual {
  double v;
  double d[N];
  FDU_HD Dual() {}
  FDU_HD Dual(double x) : v(x) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
};
template <int N>
FDU_HD Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N>
FDU_HD Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N>
FDU_HD Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N>
FDU_HD Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N>
FDU_HD Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; const double ib = 1.0 / b.v; r.v = a.v * ib;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int N> FDU_HD Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> FDU_HD Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> FDU_HD Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> FDU_HD Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N>
FDU_HD Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int N> FDU_HD Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> FDU_HD Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> FDU_HD Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N>
FDU_HD Dual<N> sqrt(const Dual<N>& a) {
  Dual<N> r; r.v = ::sqrt(a.v); const double h = 0.5 / r.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * h;
  return r;
}
template <int N>
FDU_HD Dual<N> fabs(const Dual<N>& a) { return a.v < 0.0 ? -a : a; }
FDU_HD double val(double x) { return x; }
template <int N> FDU_HD double val(const Dual<N>& x) { return x.v; }
template <bool FR, int N>
FDU_HD Dual<N> recip(const Dual<N>& x) { return 1.0 / x; }
template <bool FR, int N>
FDU_HD Dual<N> root(const Dual<N>& x) { return sqrt(x); }

// ----------------------------------------------------------------------------
// Eigenvectors of A_n = n_x df/dw + n_y dg/dw at a Roe-averaged state:
// columns (1, u - c n, H - c u_n), (1, u, q^2/2), (0, t, u_t), (1, u + c n, H + c u_n),
// t = (-n_y, n_x); the left eigenvectors in closed form.
template <class T>
struct FrameT {
  T u, v, H, c, un, ut, q2;
  double nx, ny;
};
using Frame = FrameT<double>;

template <class T, bool FR = false>
FDU_HD FrameT<T> roe_frame(const T a[4], const T b[4], double nx, double ny, double gm1) {
  FrameT<T> F;
  const T ra = root<FR>(a[0]), rb = root<FR>(b[0]);
  const T ia = recip<FR>(a[0]), ib = recip<FR>(b[0]);
  const T ua = a[1] * ia, va = a[2] * ia, ub = b[1] * ib, vb = b[2] * ib;
  const T pa = gm1 * (a[3] - 0.5 * (a[1] * ua + a[2] * va));
  const T pb = gm1 * (b[3] - 0.5 * (b[1] * ub + b[2] * vb));
  const T Ha = (a[3] + pa) * ia, Hb = (b[3] + pb) * ib;
  const T is = recip<FR>(ra + rb);
  F.u = (ra * ua + rb * ub) * is;
  F.v = (ra * va + rb * vb) * is;
  F.H = (ra * Ha + rb * Hb) * is;
  F.q2 = 0.5 * (F.u * F.u + F.v * F.v);
  F.c = root<FR>(gm1 * (F.H - F.q2));
  F.nx = nx;
  F.ny = ny;
  F.un = F.u * nx + F.v * ny;
  F.ut = F.v * nx - F.u * ny;
  return F;
}

// characteristic variables l_k . q
template <class T, bool FR = false>
FDU_HD void to_char(const FrameT<T>& F, double gm1, const T q[4], T o[4]) {
  const T ic = recip<FR>(F.c);
  const T b1 = gm1 * ic * ic, b2 = b1 * F.q2;
  const T mv = F.u * q[1] + F.v * q[2];                 // u . m
  const T nm = F.nx * q[1] + F.ny * q[2];               // n . m
  const T tm = F.nx * q[2] - F.ny * q[1];               // t . m
  const T core = b2 * q[0] - b1 * mv + b1 * q[3];       // b2 rho - b1 u.m + b1 rhoE
  o[0] = 0.5 * (core + (F.un * q[0] - nm) * ic);
  o[1] = q[0] - core;
  o[2] = tm - F.ut * q[0];
  o[3] = 0.5 * (core - (F.un * q[0] - nm) * ic);
}

// conservative variables sum_k a_k r_k
template <class T>
FDU_HD void from_char(const FrameT<T>& F, const T a[4], T q[4]) {
  const T s = a[0] + a[3], d = a[3] - a[0];
  q[0] = s + a[1];
  q[1] = F.u * (s + a[1]) + F.c * F.nx * d - F.ny * a[2];
  q[2] = F.v * (s + a[1]) + F.c * F.ny * d + F.nx * a[2];
  q[3] = F.H * s + F.c * F.un * d + F.q2 * a[1] + F.ut * a[2];
}

// rho > 0 and p > 0 (false for NaN as well); FR: the division-free test
// rho E - |m|^2 / 2 > 0, equivalent for rho > 0 (rounding aside)
template <bool FR = false>
FDU_HD bool physical(const double q[4], double gm1) {
  if (!(q[0] > 0.0)) return false;
  if (FR) return gm1 * (q[0] * q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2])) > 0.0;
  const double ir = 1.0 / q[0];
  const double u = q[1] * ir, v = q[2] * ir;
  const double p = gm1 * (q[3] - 0.5 * q[0] * (u * u + v * v));
  return p > 0.0;
}

template <class T, bool FR = false>
FDU_HD T harten(const T& l, const T& delta) {
  const T a = fabs(l);
  return val(a) < val(delta) ? (l * l + delta * delta) * recip<FR>(2.0 * delta) : a;
}

template <class T, bool FR = false>
FDU_HD void normal_flux(const T q[4], double nx, double ny, double gm1, T F[4], T& un, T& c2) {
  const T ir = recip<FR>(q[0]);
  const T u = q[1] * ir, v = q[2] * ir;
  const T p = gm1 * (q[3] - 0.5 * (q[1] * u + q[2] * v));
  un = u * nx + v * ny;
  F[0] = q[0] * un;
  F[1] = q[1] * un + p * nx;
  F[2] = q[2] * un + p * ny;
  F[3] = (q[3] + p) * un;
  c2 = (gm1 + 1.0) * p * ir;
}

// Numerical flux along the edge direction n from the midpoint states wl, wr.
template <class T, bool FR = false>
FDU_HD void riemann_flux(const T wl[4], const T wr[4], double nx, double ny, const Scheme& S,
                                             T out[4]) {
  T Fl[4], Fr[4], unl, unr, c2l, c2r;
  normal_flux<T, FR>(wl, nx, ny, S.gm1, Fl, unl, c2l);
  normal_flux<T, FR>(wr, nx, ny, S.gm1, Fr, unr, c2r);
  if (S.riemann == 1) {
    const T sl = fabs(unl) + root<FR>(c2l), sr = fabs(unr) + root<FR>(c2r);
    const T sm = val(sl) >= val(sr) ? sl : sr;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = 0.5 * (Fl[k] + Fr[k]) - 0.5 * sm * (wr[k] - wl[k]);
    return;
  }
  const FrameT<T> F = roe_frame<T, FR>(wl, wr, nx, ny, S.gm1);
  T dq[4], a[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) dq[k] = wr[k] - wl[k];
  to_char<T, FR>(F, S.gm1, dq, a);
  const T delta = S.efrac * F.c;
  a[0] = a[0] * harten<T, FR>(F.un - F.c, delta);
  a[1] = a[1] * harten<T, FR>(F.un, delta);
  a[2] = a[2] * harten<T, FR>(F.un, delta);
  a[3] = a[3] * harten<T, FR>(F.un + F.c, delta);
  T d[4];
  from_char(F, a, d);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = 0.5 * (Fl[k] + Fr[k]) - 0.5 * d[k];
}

// Numerical flux r_k of one edge from its six stencil states W (L3 L2 L1 R1 R2
// R3) and geometry g (s0/d, s1/d, s4/d, s5/d, n_x, n_y).
FDU_HD void edge_flux_one(const double W[6][4], const double g[6], const Scheme& S, double out[4]) {
  const double nx = g[4], ny = g[5];
  // characteristic frame at the Roe average of the edge's end states
  const Frame F = roe_frame<double>(W[2], W[3], nx, ny, S.gm1);
  double Cv[6][4];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    if (S.conservative) {
#pragma unroll
      for (int i = 0; i < 4; ++i) Cv[k][i] = W[k][i];
    } else {
      to_char(F, S.gm1, W[k], Cv[k]);
    }
  }

  // left state from (L3 L2 L1 R1 R2); right state from the mirror (R3 R2 R1 L1 L2)
  double x[4];
  weno_nodes(g, S, x);
  WenoGeom GL, GR;
  weno_geom(x[0], x[1], x[2], GL);
  weno_geom(-x[3], -x[2], -x[1], GR);
  double cl[4], cr[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double ul[5] = {Cv[0][c], Cv[1][c], Cv[2][c], Cv[3][c], Cv[4][c]};
    const double ur[5] = {Cv[5][c], Cv[4][c], Cv[3][c], Cv[2][c], Cv[1][c]};
    cl[c] = weno_eval(GL, ul, S.eps, S.power);
    cr[c] = weno_eval(GR, ur, S.eps, S.power);
  }
  double wl[4], wr[4];
  if (S.conservative) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      wl[k] = cl[k];
      wr[k] = cr[k];
    }
  } else {
    from_char(F, cl, wl);
    from_char(F, cr, wr);
  }
  if (S.positivity) {
    if (!physical(wl, S.gm1))
#pragma unroll
      for (int k = 0; k < 4; ++k) wl[k] = W[2][k];
    if (!physical(wr, S.gm1))
#pragma unroll
      for (int k = 0; k < 4; ++k) wr[k] = W[3][k];
  }
  riemann_flux<double>(wl, wr, nx, ny, S, out);
}

// Vertex blocks of the LDS-staged vertex kernels: at most kBlockVertices
// consecutive vertices and kBlockRows staged rows (32 bytes each) per block.
constexpr int kBlockVertices = 256;
constexpr int kBlockRows = 928;

// Packed stream ids of the block kernel (vertex variants 4-5).  For every
// real vertex and each of its 8 lanes, one 12-byte record holds the
// block-local ids of the lane's first-round entries: its 3 state-row slots,
// then its 6 flux-row slots (entry pb + lane + 8 s of the vertex's range),
// 10 bits each, three to a 32-bit word; slots past the range hold 0.  One
// coalesced load per lane replaces nine 16-bit gathers.
constexpr int kPackLPV = 8, kPackMV = 3, kPackME = 6;
static_assert(kBlockRows <= 1024, "local ids of a block must fit in 10 bits");
struct PackedIds {
  unsigned w[3];
};

// Map a hardware block index to a logical one so that each of the 8 XCDs
// (blocks are dealt to XCDs round robin) works on one contiguous range.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// ----------------------------------------------------------------------------
// Kernels.
template <class T>
__device__ __forceinline__ void ghost_state(const T* __restrict__ w, int g, const int* __restrict__ src,
                                            const signed char* __restrict__ refl,
                                            const double* __restrict__ gstate, double q[4]) {
  const int f = refl[g];
  if (f & 4) {          // Dirichlet: the given boundary state
    load4(gstate, g, q);
    return;
  }
  load4(w, src[g], q);  // mirror copy, reflecting walls negate the normal momentum
  if (f & 1) q[1] = -q[1];
  if (f & 2) q[2] = -q[2];
}

template <class T>
__global__ void __launch_bounds__(256) k_fill_ghosts(T* __restrict__ w, int nreal, int ng, const int* __restrict__ src,
                                                     const signed char* __restrict__ refl,
                                                     const double* __restrict__ gstate) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  double q[4];
  ghost_state<T>(w, g, src, refl, gstate, q);
  store4(w, nreal + g, q);
}

template <class T, class TG>
__device__ __forceinline__ void edge_item(const T* __restrict__ w, const int* __restrict__ sten,
                                          const TG* __restrict__ geo, double* __restrict__ r, int e,
                                          const Scheme& S) {
  int id[6];
  {
    const int2* sp = reinterpret_cast<const int2*>(sten + 6 * (size_t)e);
    int2 a = sp[0], b = sp[1], c = sp[2];
    id[0] = a.x; id[1] = a.y; id[2] = b.x; id[3] = b.y; id[4] = c.x; id[5] = c.y;
  }
  double W[6][4];
#pragma unroll
  for (int k = 0; k < 6; ++k) load4(w, id[k], W[k]);
  double g[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = (double)geo[6 * (size_t)e + k];
  double out[4];
  edge_flux_one(W, g, S, out);
  double2* rp = reinterpret_cast<double2*>(r + 4 * (size_t)e);
  rp[0] = make_double2(out[0], out[1]);
  rp[1] = make_double2(out[2], out[3]);
}

template <class T, class TG>
__global__ void __launch_bounds__(256) k_edge_flux(const T* __restrict__ w, const int* __restrict__ sten,
                                                   const TG* __restrict__ geo, double* __restrict__ r, int ne,
                                                   Scheme S) {
  const int e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (e < ne) edge_item<T, TG>(w, sten, geo, r, e, S);
}

// Vertex step.  LPV lanes cooperate on one vertex: each accumulates a strided
// share of the vertex terms wf (f_j - f_O) + wg (g_j - g_O) and of the edge
// terms we r_k; a butterfly over the LPV lanes reduces them, no atomics.
// mode 0: R = -div.  mode 1: out = a w_n + b (w_prev + dt (-div)), w_prev = w.
// Streaming loads of the stencil arrays (read once per launch); NT marks them
// non-temporal so they do not displace the gathered states and fluxes in cache.
template <bool NT, class X>
__device__ __forceinline__ X ldstream(const X* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// One vertex of the vertex step, computed by the LPV lanes (lane = 0..LPV-1)
// of its group; all LPV lanes must call it (butterfly reduction).
template <class T, class TW, int LPV, bool NT>
__device__ __forceinline__ void vertex_item(const T* __restrict__ w, const int* __restrict__ vptr,
                                            const int* __restrict__ vcol, const TW* __restrict__ wfg,
                                            const int* __restrict__ eptr, const int* __restrict__ ecol,
                                            const TW* __restrict__ we, const double* __restrict__ cO,
                                            const double* __restrict__ r, int nreal, double gm1, int mode,
                                            T* __restrict__ R, const T* __restrict__ wn, T* __restrict__ out,
                                            double a, double b, const double* __restrict__ dt_dev, int v, int lane) {
  const bool active = v < nreal;
  const int vv = active ? v : 0;
  double q0[4], f0[4], g0[4];
  load4(w, vv, q0);
  euler_fg(q0, gm1, f0, g0);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (active) {
    const int pe = vptr[v + 1];
    for (int p = vptr[v] + lane; p < pe; p += LPV) {
      const int j = ldstream<NT>(vcol + p);
      const double wf = (double)ldstream<NT>(wfg + 2 * (size_t)p), wg = (double)ldstream<NT>(wfg + 2 * (size_t)p + 1);
      double q[4], f[4], g[4];
      load4(w, j, q);
      euler_fg(q, gm1, f, g);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += wf * (f[k] - f0[k]) + wg * (g[k] - g0[k]);
    }
    const int qe = eptr[v + 1];
    for (int p = eptr[v] + lane; p < qe; p += LPV) {
      const int k = ldstream<NT>(ecol + p);
      const double c = (double)ldstream<NT>(we + p);
      const double2* rp = reinterpret_cast<const double2*>(r + 4 * (size_t)k);
      const double2 x = rp[0], y = rp[1];
      acc[0] += c * x.x; acc[1] += c * x.y; acc[2] += c * y.x; acc[3] += c * y.y;
    }
  }
#pragma unroll
  for (int m = LPV / 2; m >= 1; m >>= 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += __shfl_xor(acc[k], m, LPV);
  }
  if (!active || lane != 0) return;
  const double cx = cO[2 * (size_t)v], cy = cO[2 * (size_t)v + 1];
  double res[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) res[k] = -(acc[k] - (cx * f0[k] + cy * g0[k]));
  if (mode == 0) {
    store4(R, v, res);
  } else {
    const double dt = *dt_dev;
    double n[4] = {0.0, 0.0, 0.0, 0.0};
    if (a != 0.0) load4(wn, v, n);
    double o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = a * n[k] + b * (q0[k] + dt * res[k]);
    store4(out, v, o);
  }
}

template <class T, class TW, int LPV, bool NT = false>
__global__ void __launch_bounds__(256) k_vertex(const T* __restrict__ w, const int* __restrict__ vptr,
                                                const int* __restrict__ vcol, const TW* __restrict__ wfg,
                                                const int* __restrict__ eptr, const int* __restrict__ ecol,
                                                const TW* __restrict__ we, const double* __restrict__ cO,
                                                const double* __restrict__ r, int nreal, double gm1, int mode,
                                                T* __restrict__ R, const T* __restrict__ wn, T* __restrict__ out,
                                                double a, double b, const double* __restrict__ dt_dev) {
  const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  vertex_item<T, TW, LPV, NT>(w, vptr, vcol, wfg, eptr, ecol, we, cO, r, nreal, gm1, mode, R, wn, out, a, b, dt_dev,
                              t / LPV, t % LPV);
}

// ----------------------------------------------------------------------------
// Register-lean WENO: the same interpolants written with divided differences.
// For a sub-stencil with nodes (a, b, c) and values (ua, ub, uc):
//   d1 = (ub - ua)/(b - a), d2 = (uc - ub)/(c - b), q'' = 2 (d2 - d1)/(c - a),
//   q'(0) = d1 - (q''/2)(a + b),  q(0) = ua - d1 a + (q''/2) a b,
// so the interpolants need the inverse node gaps, inverse double gaps, the
// nodes and C_k instead of the 30 coefficients of a side.

// Both sides at once on the edge's six nodes, in the left side's coordinates
// s = (s0, s1, -1/2, 1/2, s4, s5).  The left side combines the quadratics on
// nodes (0,1,2), (1,2,3), (2,3,4), the right side those on (5,4,3), (4,3,2),
// (3,2,1): the middle two are the same polynomials for both sides, and their
// value at the midpoint and smoothness indicator (the integral over the middle
// interval of squared derivatives) do not change under the mirror, so four
// quadratics are evaluated instead of six.  The twelve gaps and gap products
// are positive and of moderate size (normalised by the middle-edge length), so
// their inverses come from one reciprocal of their product (prefix products,
// then one multiplication back per gap: 1/a_i = (1/(a_1..a_i)) (a_1..a_{i-1})).
struct WenoDD2 {
  double s0, s1, s4, s5;
  double ig[5];   // 1/(s_{m+1} - s_m), ig[2] = 1
  double ih[4];   // 1/(s_{m+2} - s_m)
  double CL[3], CR[3];
};

__device__ __forceinline__ void weno_dd_geom2(double s0, double s1, double s4, double s5, WenoDD2& G) {
  G.s0 = s0; G.s1 = s1; G.s4 = s4; G.s5 = s5;
  const double a[12] = {s1 - s0,  -0.5 - s1, s4 - 0.5, s5 - s4,   -0.5 - s0, 0.5 - s1,
                        s4 + 0.5, s5 - 0.5,  s4 - s0,  (0.5 - s0) * (s4 - s1), s5 - s1, (s5 + 0.5) * (s4 - s1)};
  double p[12];
  p[0] = a[0];
#pragma unroll
  for (int i = 1; i < 12; ++i) p[i] = p[i - 1] * a[i];
  double inv = frcp(p[11]), ia[12];
#pragma unroll
  for (int i = 11; i > 0; --i) {
    ia[i] = inv * p[i - 1];
    inv *= a[i];
  }
  ia[0] = inv;
  G.ig[0] = ia[0];
  G.ig[1] = ia[1];
  G.ig[2] = 1.0;
  G.ig[3] = ia[2];
  G.ig[4] = ia[3];
  G.ih[0] = ia[4];
  G.ih[1] = ia[5];
  G.ih[2] = ia[6];
  G.ih[3] = ia[7];
  // left (nodes s0..s4): C0 = s3 s4 / ((s4 - s0)(s3 - s0)), C2 = s0 s1 / ((s4 - s0)(s4 - s1)), s3 = 1/2;
  // right: the same with the mirrored nodes (-s5, -s4, -1/2, 1/2, -s1)
  const double tl = ia[8] * ia[9], tr = ia[10] * ia[11];
  G.CL[0] = 0.5 * s4 * (s4 - s1) * tl;
  G.CL[2] = s0 * s1 * (0.5 - s0) * tl;
  G.CL[1] = 1.0 - G.CL[0] - G.CL[2];
  G.CR[0] = -0.5 * s1 * (s4 - s1) * tr;
  G.CR[2] = s5 * s4 * (s5 + 0.5) * tr;
  G.CR[1] = 1.0 - G.CR[0] - G.CR[2];
}

// Left and right midpoint values of one component from the six node values.
template <int POW>
__device__ __forceinline__ void weno_dd_eval2(const WenoDD2& G, const double u[6], double eps, double& ul,
                                              double& ur) {
  const double xs[6] = {G.s0, G.s1, -0.5, 0.5, G.s4, G.s5};
  double dd[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) dd[m] = (u[m + 1] - u[m]) * G.ig[m];
  double ut[4], b[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double a = xs[k], bb = xs[k + 1];
    const double h2 = (dd[k + 1] - dd[k]) * G.ih[k];          // q''/2
    const double d1 = dd[k] - h2 * (a + bb);                   // q'(0)
    ut[k] = u[k] - dd[k] * a + h2 * a * bb;                    // q(0)
    b[k] = fma(d1, d1, fma((13.0 / 3.0) * h2, h2, eps));
    if (POW == 2) b[k] *= b[k];
  }
  {
    const double n0 = G.CL[0] * b[1] * b[2];
    const double n1 = G.CL[1] * b[0] * b[2];
    const double n2 = G.CL[2] * b[0] * b[1];
    ul = (n0 * ut[0] + n1 * ut[1] + n2 * ut[2]) * frcp(n0 + n1 + n2);
  }
  {
    // the right side's sub-stencils 0, 1, 2 are quadratics 3, 2, 1
    const double n0 = G.CR[0] * b[2] * b[1];
    const double n1 = G.CR[1] * b[3] * b[1];
    const double n2 = G.CR[2] * b[3] * b[2];
    ur = (n0 * ut[3] + n1 * ut[2] + n2 * ut[1]) * frcp(n0 + n1 + n2);
  }
}

// Edge flux, register-lean variant: both sides' WENO evaluated together (four
// quadratics per component), divided-difference interpolants, refined
// reciprocals and square roots.
template <class T, class TG, int POW>
__device__ __forceinline__ void edge_lean_body(const T* __restrict__ w, const int* __restrict__ sten,
                                               const TG* __restrict__ geo, double* __restrict__ r, int e,
                                               const Scheme& S) {
  int id[6];
  {
    const int2* sp = reinterpret_cast<const int2*>(sten + 6 * (size_t)e);
    int2 a = sp[0], b = sp[1], c = sp[2];
    id[0] = a.x; id[1] = a.y; id[2] = b.x; id[3] = b.y; id[4] = c.x; id[5] = c.y;
  }
  // all six states and the geometry are requested before any is used (a use
  // between two loads would make the compiler wait for the first)
  double Cv[6][4];
#pragma unroll
  for (int k = 0; k < 6; ++k) load4(w, id[k], Cv[k]);
  double g[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = (double)geo[6 * (size_t)e + k];
  const double nx = g[4], ny = g[5];
  const Frame F = roe_frame<double, true>(Cv[2], Cv[3], nx, ny, S.gm1);
  if (!S.conservative) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double q[4] = {Cv[k][0], Cv[k][1], Cv[k][2], Cv[k][3]};
      to_char<double, true>(F, S.gm1, q, Cv[k]);
    }
  }
  double x[4];
  weno_nodes(g, S, x);
  double cl[4], cr[4];
  {
    WenoDD2 G;
    weno_dd_geom2(x[0], x[1], x[2], x[3], G);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double u[6] = {Cv[0][c], Cv[1][c], Cv[2][c], Cv[3][c], Cv[4][c], Cv[5][c]};
      weno_dd_eval2<POW>(G, u, S.eps, cl[c], cr[c]);
    }
  }
  double wl[4], wr[4];
  if (S.conservative) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      wl[k] = cl[k];
      wr[k] = cr[k];
    }
  } else {
    from_char(F, cl, wl);
    from_char(F, cr, wr);
  }
  if (S.positivity) {
    // the end states are reloaded (rarely needed; not kept live in registers)
    if (!physical<true>(wl, S.gm1)) load4(w, opaque(id[2]), wl);
    if (!physical<true>(wr, S.gm1)) load4(w, opaque(id[3]), wr);
  }
  double out[4];
  riemann_flux<double, true>(wl, wr, nx, ny, S, out);
  double2* rp = reinterpret_cast<double2*>(r + 4 * (size_t)e);
  rp[0] = make_double2(out[0], out[1]);
  rp[1] = make_double2(out[2], out[3]);
}

// The WENO power is uniform over a launch: one branch instead of a select per
// smoothness indicator.
template <class T, class TG>
__device__ __forceinline__ void edge_lean_item(const T* __restrict__ w, const int* __restrict__ sten,
                                               const TG* __restrict__ geo, double* __restrict__ r, int e,
                                               const Scheme& S) {
  if (S.power == 2)
    edge_lean_body<T, TG, 2>(w, sten, geo, r, e, S);
  else
    edge_lean_body<T, TG, 1>(w, sten, geo, r, e, S);
}

template <class T, class TG>
__global__ void __launch_bounds__(256) k_edge_flux_lean(const T* __restrict__ w, const int* __restrict__ sten,
                                                             const TG* __restrict__ geo, double* __restrict__ r,
                                                             int ne, Scheme S) {
  const int e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (e < ne) edge_lean_item<T, TG>(w, sten, geo, r, e, S);
}

// Vertex step, software-pipelined: every lane first loads the ids and weights
// of up to MV vertex entries and ME edge entries, then issues all their gathers,
// then accumulates; entries beyond MV*LPV / ME*LPV go through a tail loop.
template <class T, class TW, int LPV, int MV, int ME>
__device__ __forceinline__ void vertex_pipe_item(const T* __restrict__ w, const int* __restrict__ vptr,
                                                 const int* __restrict__ vcol, const TW* __restrict__ wfg,
                                                 const int* __restrict__ eptr, const int* __restrict__ ecol,
                                                 const TW* __restrict__ we, const double* __restrict__ cO,
                                                 const double* __restrict__ r, int nreal, double gm1, int mode,
                                                 T* __restrict__ R, const T* __restrict__ wn, T* __restrict__ out,
                                                 double a, double b, const double* __restrict__ dt_dev, int v,
                                                 int lane) {
  const bool active = v < nreal;
  const int vv = active ? v : 0;
  // every load issued unconditionally at an in-range index (an idle thread
  // reads an empty range at row nreal, a slot past its range reads entry 0);
  // the predicates are applied where the values are used
  const int vc = active ? v : nreal, vc1 = active ? v + 1 : nreal;
  const int vb = vptr[vc], ve = vptr[vc1], eb = eptr[vc], ee = eptr[vc1];
  int jv[MV], ke[ME];
  double wf[MV], wg[MV], cw[ME];
#pragma unroll
  for (int s = 0; s < MV; ++s) {
    const int p = vb + lane + s * LPV;
    const size_t pc = p < ve ? p : 0;
    jv[s] = vcol[pc];
    wf[s] = (double)wfg[2 * pc];
    wg[s] = (double)wfg[2 * pc + 1];
  }
#pragma unroll
  for (int s = 0; s < ME; ++s) {
    const int p = eb + lane + s * LPV;
    const size_t pc = p < ee ? p : 0;
    ke[s] = ecol[pc];
    cw[s] = (double)we[pc];
  }
  double qv[MV][4], rv[ME][4];
#pragma unroll
  for (int s = 0; s < MV; ++s) load4(w, vb + lane + s * LPV < ve ? jv[s] : vv, qv[s]);
#pragma unroll
  for (int s = 0; s < ME; ++s) {
    const double2* rp = reinterpret_cast<const double2*>(r + 4 * (size_t)(eb + lane + s * LPV < ee ? ke[s] : 0));
    const double2 x = rp[0], y = rp[1];
    rv[s][0] = x.x; rv[s][1] = x.y; rv[s][2] = y.x; rv[s][3] = y.y;
  }
  double q0[4], f0[4], g0[4];
  load4(w, vv, q0);
  euler_fg(q0, gm1, f0, g0);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < MV; ++s) {
    if (vb + lane + s * LPV < ve) {
      double f[4], g[4];
      euler_fg(qv[s], gm1, f, g);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += wf[s] * (f[k] - f0[k]) + wg[s] * (g[k] - g0[k]);
    }
  }
#pragma unroll
  for (int s = 0; s < ME; ++s) {
    const double c = eb + lane + s * LPV < ee ? cw[s] : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += c * rv[s][k];
  }
  // tails (rare: stencils larger than the pipelined slots)
  for (int p = vb + lane + MV * LPV; p < ve; p += LPV) {
    const int j = vcol[p];
    const double af = (double)wfg[2 * (size_t)p], ag = (double)wfg[2 * (size_t)p + 1];
    double q[4], f[4], g[4];
    load4(w, j, q);
    euler_fg(q, gm1, f, g);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += af * (f[k] - f0[k]) + ag * (g[k] - g0[k]);
  }
  for (int p = eb + lane + ME * LPV; p < ee; p += LPV) {
    const int k = ecol[p];
    const double c = (double)we[p];
    const double2* rp = reinterpret_cast<const double2*>(r + 4 * (size_t)k);
    const double2 x = rp[0], y = rp[1];
    acc[0] += c * x.x; acc[1] += c * x.y; acc[2] += c * y.x; acc[3] += c * y.y;
  }
#pragma unroll
  for (int m = LPV / 2; m >= 1; m >>= 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += __shfl_xor(acc[k], m, LPV);
  }
  if (!active || lane != 0) return;
  const double cx = cO[2 * (size_t)v], cy = cO[2 * (size_t)v + 1];
  double res[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) res[k] = -(acc[k] - (cx * f0[k] + cy * g0[k]));
  if (mode == 0) {
    store4(R, v, res);
  } else {
    const double dt = *dt_dev;
    double n[4] = {0.0, 0.0, 0.0, 0.0};
    if (a != 0.0) load4(wn, v, n);
    double o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = a * n[k] + b * (q0[k] + dt * res[k]);
    store4(out, v, o);
  }
}

template <class T, class TW, int LPV, int MV, int ME>
__global__ void __launch_bounds__(256) k_vertex_pipe(const T* __restrict__ w, const int* __restrict__ vptr,
                                                     const int* __restrict__ vcol, const TW* __restrict__ wfg,
                                                     const int* __restrict__ eptr, const int* __restrict__ ecol,
                                                     const TW* __restrict__ we, const double* __restrict__ cO,
                                                     const double* __restrict__ r, int nreal, double gm1, int mode,
                                                     T* __restrict__ R, const T* __restrict__ wn, T* __restrict__ out,
                                                     double a, double b, const double* __restrict__ dt_dev) {
  const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  vertex_pipe_item<T, TW, LPV, MV, ME>(w, vptr, vcol, wfg, eptr, ecol, we, cO, r, nreal, gm1, mode, R, wn, out, a, b,
                                       dt_dev, t / LPV, t % LPV);
}

// Vertex step with the stencil halo staged in LDS.  The real vertices are cut
// (at set-up) into blocks of consecutive ids; for each block the sorted list of
// state rows and of flux rows its stencils read is stored with the block, and
// the stencil entries hold 16-bit positions in those lists.  A workgroup copies
// its block's rows into LDS (sorted ids: mostly contiguous loads, each row
// fetched once per block instead of once per stencil entry), then walks the
// block's vertices in rounds of 256 / LPV, LPV lanes per vertex, reading rows
// from LDS.  The stream loads (CSR pointers, local indices, weights) of the
// first round are issued before the staging barrier; with PF = 2 those of
// round r + 1 are issued before round r is computed.  WPE is the occupancy
// (waves per SIMD) the register allocation is held to.
template <class TW, int MV, int ME>
struct VertexFetch {
  int v, pb, pe, qb, qe;
  int jv[MV], ke[ME];
  double wf[MV], wg[MV], cw[ME];
};

template <class TW, int LPV, int MV, int ME>
__device__ __forceinline__ void vertex_fetch(VertexFetch<TW, MV, ME>& F, int v, int v1, int lane,
                                             const int* __restrict__ vptr, const unsigned short* __restrict__ lvcol,
                                             const TW* __restrict__ wfg, const int* __restrict__ eptr,
                                             const unsigned short* __restrict__ lecol, const TW* __restrict__ we) {
  // unconditional loads at in-range indices (past the block: an empty range;
  // past a range: entry 0), the predicates applied where the values are used
  F.v = v;
  const int vc = v < v1 ? v : v1, vc1 = v < v1 ? v + 1 : v1;
  F.pb = vptr[vc]; F.pe = vptr[vc1];
  F.qb = eptr[vc]; F.qe = eptr[vc1];
#pragma unroll
  for (int s = 0; s < MV; ++s) {
    const int p = F.pb + lane + s * LPV;
    const size_t pc = p < F.pe ? p : 0;
    F.jv[s] = (int)lvcol[pc];
    F.wf[s] = (double)wfg[2 * pc];
    F.wg[s] = (double)wfg[2 * pc + 1];
  }
#pragma unroll
  for (int s = 0; s < ME; ++s) {
    const int p = F.qb + lane + s * LPV;
    const size_t pc = p < F.qe ? p : 0;
    F.ke[s] = (int)lecol[pc];
    F.cw[s] = (double)we[pc];
  }
}

template <class T, class TW, int LPV, int MV, int ME>
__device__ __forceinline__ void vertex_lds_compute(const VertexFetch<TW, MV, ME>& F, int v0, int v1, int lane,
                                                   const double* __restrict__ Lv, const double* __restrict__ Le,
                                                   const T* __restrict__ w, const unsigned short* __restrict__ lvcol,
                                                   const TW* __restrict__ wfg, const unsigned short* __restrict__ lecol,
                                                   const TW* __restrict__ we, const double* __restrict__ cO, double gm1,
                                                   int mode, T* __restrict__ R, const T* __restrict__ wn,
                                                   T* __restrict__ out, double a, double b,
                                                   const double* __restrict__ dt_dev) {
  const int v = F.v;
  const bool active = v < v1;
  const int vv = active ? v : v0;
  double q0[4], f0[4], g0[4];
  load4(w, vv, q0);
  euler_fg<true>(q0, gm1, f0, g0);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < MV; ++s) {
    if (F.pb + lane + s * LPV < F.pe) {
      const double2* lp = reinterpret_cast<const double2*>(Lv + 4 * F.jv[s]);
      const double2 x = lp[0], y = lp[1];
      const double q[4] = {x.x, x.y, y.x, y.y};
      double f[4], g[4];
      euler_fg<true>(q, gm1, f, g);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += F.wf[s] * (f[k] - f0[k]) + F.wg[s] * (g[k] - g0[k]);
    }
  }
#pragma unroll
  for (int s = 0; s < ME; ++s) {
    if (F.qb + lane + s * LPV < F.qe) {
      const double2* lp = reinterpret_cast<const double2*>(Le + 4 * F.ke[s]);
      const double2 x = lp[0], y = lp[1];
      acc[0] += F.cw[s] * x.x; acc[1] += F.cw[s] * x.y; acc[2] += F.cw[s] * y.x; acc[3] += F.cw[s] * y.y;
    }
  }
  for (int p = F.pb + lane + MV * LPV; p < F.pe; p += LPV) {
    const double2* lp = reinterpret_cast<const double2*>(Lv + 4 * (int)lvcol[p]);
    const double2 x = lp[0], y = lp[1];
    const double q[4] = {x.x, x.y, y.x, y.y};
    const double af = (double)wfg[2 * (size_t)p], ag = (double)wfg[2 * (size_t)p + 1];
    double f[4], g[4];
    euler_fg<true>(q, gm1, f, g);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += af * (f[k] - f0[k]) + ag * (g[k] - g0[k]);
  }
  for (int p = F.qb + lane + ME * LPV; p < F.qe; p += LPV) {
    const double2* lp = reinterpret_cast<const double2*>(Le + 4 * (int)lecol[p]);
    const double2 x = lp[0], y = lp[1];
    const double c = (double)we[p];
    acc[0] += c * x.x; acc[1] += c * x.y; acc[2] += c * y.x; acc[3] += c * y.y;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = group_sum<LPV>(acc[k]);
  if (active && lane == 0) {
    const double cx = cO[2 * (size_t)v], cy = cO[2 * (size_t)v + 1];
    double res[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) res[k] = -(acc[k] - (cx * f0[k] + cy * g0[k]));
    if (mode == 0) {
      store4(R, v, res);
    } else {
      const double dt = *dt_dev;
      double n[4] = {0.0, 0.0, 0.0, 0.0};
      if (a != 0.0) load4(wn, v, n);
      double q[4];
      load4(w, opaque(v), q);   // reloaded rather than kept live through the loops
      double o[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) o[k] = a * n[k] + b * (q[k] + dt * res[k]);
      store4(out, v, o);
    }
  }
}

// One vertex block of the LDS-staged vertex step (the workgroup's 256 threads).
template <class T, class TW, int LPV, int MV, int ME, int PF>
__device__ __forceinline__ void vertex_lds_block(int bk, double* lds, const T* __restrict__ w,
                                                 const int* __restrict__ blk, const int* __restrict__ uvp,
                                                 const int* __restrict__ uv, const int* __restrict__ uep,
                                                 const int* __restrict__ ue, const int* __restrict__ vptr,
                                                 const unsigned short* __restrict__ lvcol,
                                                 const TW* __restrict__ wfg, const int* __restrict__ eptr,
                                                 const unsigned short* __restrict__ lecol,
                                                 const TW* __restrict__ we, const double* __restrict__ cO,
                                                 const double* __restrict__ r, double gm1, int mode,
                                                 T* __restrict__ R, const T* __restrict__ wn, T* __restrict__ out,
                                                 double a, double b, const double* __restrict__ dt_dev) {
  constexpr int VPR = 256 / LPV;    // vertices per round
  const int v0 = blk[bk], v1 = blk[bk + 1];
  const int a0 = uvp[bk], na = uvp[bk + 1] - a0;
  const int e0 = uep[bk], ne = uep[bk + 1] - e0;
  const int lane = threadIdx.x % LPV, sub = threadIdx.x / LPV;
  VertexFetch<TW, MV, ME> F;
  vertex_fetch<TW, LPV, MV, ME>(F, v0 + sub, v1, lane, vptr, lvcol, wfg, eptr, lecol, we);
  for (int i = threadIdx.x; i < na; i += blockDim.x) {
    double q[4];
    load4(w, uv[a0 + i], q);
    double2* d = reinterpret_cast<double2*>(lds + 4 * i);
    d[0] = make_double2(q[0], q[1]);
    d[1] = make_double2(q[2], q[3]);
  }
  for (int i = threadIdx.x; i < ne; i += blockDim.x) {
    const double2* sp = reinterpret_cast<const double2*>(r + 4 * (size_t)ue[e0 + i]);
    double2* d = reinterpret_cast<double2*>(lds + 4 * (na + i));
    d[0] = sp[0];
    d[1] = sp[1];
  }
  __syncthreads();
  const double* Lv = lds;
  const double* Le = lds + 4 * na;
  for (int vb = v0; vb < v1; vb += VPR) {
    if (PF == 2) {
      VertexFetch<TW, MV, ME> G;
      vertex_fetch<TW, LPV, MV, ME>(G, vb + VPR + sub, v1, lane, vptr, lvcol, wfg, eptr, lecol, we);
      vertex_lds_compute<T, TW, LPV, MV, ME>(F, v0, v1, lane, Lv, Le, w, lvcol, wfg, lecol, we, cO, gm1, mode, R, wn,
                                             out, a, b, dt_dev);
      F = G;
    } else {
      if (vb > v0) vertex_fetch<TW, LPV, MV, ME>(F, vb + sub, v1, lane, vptr, lvcol, wfg, eptr, lecol, we);
      vertex_lds_compute<T, TW, LPV, MV, ME>(F, v0, v1, lane, Lv, Le, w, lvcol, wfg, lecol, we, cO, gm1, mode, R, wn,
                                             out, a, b, dt_dev);
    }
  }
}

template <class T, class TW, int LPV, int MV, int ME, int PF, int WPE>
__global__ void __launch_bounds__(256, WPE) k_vertex_lds(const T* __restrict__ w, const int* __restrict__ blk,
                                                         const int* __restrict__ uvp, const int* __restrict__ uv,
                                                         const int* __restrict__ uep, const int* __restrict__ ue,
                                                         const int* __restrict__ vptr,
                                                         const unsigned short* __restrict__ lvcol,
                                                         const TW* __restrict__ wfg, const int* __restrict__ eptr,
                                                         const unsigned short* __restrict__ lecol,
                                                         const TW* __restrict__ we, const double* __restrict__ cO,
                                                         const double* __restrict__ r, double gm1, int mode,
                                                         T* __restrict__ R, const T* __restrict__ wn,
                                                         T* __restrict__ out, double a, double b,
                                                         const double* __restrict__ dt_dev) {
  extern __shared__ double lds[];   // [rows][4]: the block's state rows, then its flux rows
  const int bk = xcd_block(blockIdx.x, gridDim.x);
  vertex_lds_block<T, TW, LPV, MV, ME, PF>(bk, lds, w, blk, uvp, uv, uep, ue, vptr,
                                           lvcol, wfg, eptr, lecol, we, cO, r, gm1, mode, R, wn, out, a, b, dt_dev);
}

// Vertex step over the same vertex blocks with more of the block in LDS: the
// block's CSR pointers and its own state rows (consecutive in its state-row
// list, starting at own[block]) are staged with the halo, so the only global
// loads of a round are the stream of 16-bit local ids and weights (with
// PF = 2 issued before the previous round is computed: no pointer load sits in
// front of them), and the stage combine is done by lanes 0-3 of each vertex,
// one component each (8-byte loads and stores instead of 32-byte rows).  The
// arithmetic is that of k_vertex_lds with the same lanes, term for term.
// With PK the round's row positions stay in their packed words until used
// (3 registers instead of 9 while a prefetched round waits).
template <class TW, int MV, int ME, bool PK>
struct BlockFetch {
  int i, pb, pe, qb, qe;
  int jv[PK ? 1 : MV], ke[PK ? 1 : ME];
  unsigned pk[PK ? 3 : 1];
  double wf[MV], wg[MV], cw[ME];
  // row position of vertex slot s and of edge slot s (s known at compile time)
  __device__ __forceinline__ int vid(int s) const {
    if constexpr (PK) return (int)((pk[s / 3] >> (10 * (s % 3))) & 1023u);
    else return jv[s];
  }
  __device__ __forceinline__ int eid(int s) const {
    if constexpr (PK) return (int)((pk[(MV + s) / 3] >> (10 * ((MV + s) % 3))) & 1023u);
    else return ke[s];
  }
};

// The stream loads of one round.  Slots past a vertex's entry range load
// entry pb instead (always in range) and are skipped where they are used:
// loads under a branch make the compiler wait for every load in flight at the
// join, which would serialise the round's memory requests.
// With PK the ids come from the vertex's packed record (vrow: the vertex's
// row, in range also past the block) instead of the 16-bit id lists.
template <class TW, int LPV, int MV, int ME, bool PK>
__device__ __forceinline__ void block_fetch_slots(BlockFetch<TW, MV, ME, PK>& F, int lane,
                                                  const unsigned short* __restrict__ lvcol,
                                                  const TW* __restrict__ wfg, const unsigned short* __restrict__ lecol,
                                                  const TW* __restrict__ we, const PackedIds* __restrict__ pk,
                                                  int vrow) {
  if constexpr (PK) {
    static_assert(LPV == kPackLPV && MV == kPackMV && ME == kPackME, "layout of the packed ids");
    const PackedIds k = pk[(size_t)vrow * LPV + lane];
    F.pk[0] = k.w[0]; F.pk[1] = k.w[1]; F.pk[2] = k.w[2];
  }
#pragma unroll
  for (int s = 0; s < MV; ++s) {
    const int p = F.pb + lane + s * LPV;
    const size_t pc = p < F.pe ? p : F.pb;
    if constexpr (!PK) F.jv[s] = (int)lvcol[pc];
    F.wf[s] = (double)wfg[2 * pc];
    F.wg[s] = (double)wfg[2 * pc + 1];
  }
#pragma unroll
  for (int s = 0; s < ME; ++s) {
    const int p = F.qb + lane + s * LPV;
    const size_t pc = p < F.qe ? p : F.qb;
    if constexpr (!PK) F.ke[s] = (int)lecol[pc];
    F.cw[s] = (double)we[pc];
  }
}

template <class TW, int LPV, int MV, int ME, bool PK>
__device__ __forceinline__ void block_fetch(BlockFetch<TW, MV, ME, PK>& F, int i, int v0, int nb, int lane,
                                            const int* __restrict__ lp, const unsigned short* __restrict__ lvcol,
                                            const TW* __restrict__ wfg, const unsigned short* __restrict__ lecol,
                                            const TW* __restrict__ we, const PackedIds* __restrict__ pk) {
  F.i = i;
  const int ic = i < nb ? i : nb, ic1 = i < nb ? i + 1 : nb;   // past the block: an empty entry range
  F.pb = lp[ic]; F.pe = lp[ic1];
  F.qb = lp[nb + 1 + ic]; F.qe = lp[nb + 1 + ic1];
  block_fetch_slots<TW, LPV, MV, ME, PK>(F, lane, lvcol, wfg, lecol, we, pk, v0 + (i < nb ? i : 0));
}

__device__ __forceinline__ double pick4(const double x[4], int k) {
  return k == 0 ? x[0] : (k == 1 ? x[1] : (k == 2 ? x[2] : x[3]));
}

template <class T, class TW, int LPV, int MV, int ME, bool PK>
__device__ __forceinline__ void block_compute(const BlockFetch<TW, MV, ME, PK>& F, int v0, int nb, int o0, int lane,
                                              const double* __restrict__ Lv, const double* __restrict__ Le,
                                              const unsigned short* __restrict__ lvcol, const TW* __restrict__ wfg,
                                              const unsigned short* __restrict__ lecol, const TW* __restrict__ we,
                                              const double* __restrict__ cO, double gm1, int mode,
                                              T* __restrict__ R, const T* __restrict__ wn, T* __restrict__ out,
                                              double a, double b, const double* __restrict__ dt_dev) {
  const bool active = F.i < nb;
  const double* own = Lv + 4 * (o0 + (active ? F.i : 0));
  double q0[4], f0[4], g0[4];
  {
    const double2* lp = reinterpret_cast<const double2*>(own);
    const double2 x = lp[0], y = lp[1];
    q0[0] = x.x; q0[1] = x.y; q0[2] = y.x; q0[3] = y.y;
  }
  euler_fg<true>(q0, gm1, f0, g0);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < MV; ++s) {
    if (F.pb + lane + s * LPV < F.pe) {
      const double2* lp = reinterpret_cast<const double2*>(Lv + 4 * F.vid(s));
      const double2 x = lp[0], y = lp[1];
      const double q[4] = {x.x, x.y, y.x, y.y};
      double f[4], g[4];
      euler_fg<true>(q, gm1, f, g);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += F.wf[s] * (f[k] - f0[k]) + F.wg[s] * (g[k] - g0[k]);
    }
  }
#pragma unroll
  for (int s = 0; s < ME; ++s) {
    if (F.qb + lane + s * LPV < F.qe) {
      const double2* lp = reinterpret_cast<const double2*>(Le + 4 * F.eid(s));
      const double2 x = lp[0], y = lp[1];
      acc[0] += F.cw[s] * x.x; acc[1] += F.cw[s] * x.y; acc[2] += F.cw[s] * y.x; acc[3] += F.cw[s] * y.y;
    }
  }
  for (int p = F.pb + lane + MV * LPV; p < F.pe; p += LPV) {
    const double2* lp = reinterpret_cast<const double2*>(Lv + 4 * (int)lvcol[p]);
    const double2 x = lp[0], y = lp[1];
    const double q[4] = {x.x, x.y, y.x, y.y};
    const double af = (double)wfg[2 * (size_t)p], ag = (double)wfg[2 * (size_t)p + 1];
    double f[4], g[4];
    euler_fg<true>(q, gm1, f, g);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += af * (f[k] - f0[k]) + ag * (g[k] - g0[k]);
  }
  for (int p = F.qb + lane + ME * LPV; p < F.qe; p += LPV) {
    const double2* lp = reinterpret_cast<const double2*>(Le + 4 * (int)lecol[p]);
    const double2 x = lp[0], y = lp[1];
    const double c = (double)we[p];
    acc[0] += c * x.x; acc[1] += c * x.y; acc[2] += c * y.x; acc[3] += c * y.y;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = group_sum<LPV>(acc[k]);
  if (active && lane < 4) {
    const int k = lane;
    const size_t v = (size_t)(v0 + F.i);
    const double cx = cO[2 * v], cy = cO[2 * v + 1];
    const double res = -(pick4(acc, k) - (cx * pick4(f0, k) + cy * pick4(g0, k)));
    if (mode == 0) {
      R[4 * v + k] = (T)res;
    } else {
      const double dt = *dt_dev;
      const double n = a != 0.0 ? (double)wn[4 * v + k] : 0.0;
      out[4 * v + k] = (T)(a * n + b * (own[k] + dt * res));
    }
  }
}

template <class T, class TW, int LPV, int MV, int ME, int PF, bool PK>
__device__ __forceinline__ void vertex_block2(int bk, double* lds, const T* __restrict__ w, const int* __restrict__ blk,
                                              const int* __restrict__ own, const int* __restrict__ uvp,
                                              const int* __restrict__ uv, const int* __restrict__ uep,
                                              const int* __restrict__ ue, const int* __restrict__ vptr,
                                              const unsigned short* __restrict__ lvcol, const TW* __restrict__ wfg,
                                              const int* __restrict__ eptr, const unsigned short* __restrict__ lecol,
                                              const TW* __restrict__ we, const double* __restrict__ cO,
                                              const double* __restrict__ r, double gm1, int mode,
                                              T* __restrict__ R, const T* __restrict__ wn, T* __restrict__ out,
                                              double a, double b, const double* __restrict__ dt_dev,
                                              const PackedIds* __restrict__ pk) {
  constexpr int VPR = 256 / LPV;    // vertices per round
  const int v0 = blk[bk], nb = blk[bk + 1] - v0;
  const int a0 = uvp[bk], na = uvp[bk + 1] - a0;
  const int e0 = uep[bk], ne = uep[bk + 1] - e0;
  const int o0 = own[bk];
  const int lane = threadIdx.x % LPV, sub = threadIdx.x / LPV;
  int* lp = reinterpret_cast<int*>(lds + 4 * (na + ne));   // vptr[v0 .. v0 + nb], then eptr[v0 .. v0 + nb]
  // The first round's stream loads (pointers read from global memory here),
  // then every thread's share of the staged rows (at most RPT each) loaded
  // together before any is written to LDS: one memory round trip, not one per
  // row.
  BlockFetch<TW, MV, ME, PK> F;
  {
    const int ic = v0 + (sub < nb ? sub : nb), ic1 = v0 + (sub < nb ? sub + 1 : nb);   // past the block: empty
    F.i = sub;
    F.pb = vptr[ic]; F.pe = vptr[ic1];
    F.qb = eptr[ic]; F.qe = eptr[ic1];
    block_fetch_slots<TW, LPV, MV, ME, PK>(F, lane, lvcol, wfg, lecol, we, pk, v0 + (sub < nb ? sub : 0));
  }
  {
    // row i of the staging list: state row uv[a0 + i] (i < na) or flux row
    // ue[e0 + i - na]; threads past the list load row 0 of the state list
    // (in range) and do not store it
    constexpr int RPT = (kBlockRows + 255) / 256;   // rows per thread
    int src[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = threadIdx.x + 256 * k;
      src[k] = i < na ? uv[a0 + i] : (i < na + ne ? ue[e0 + i - na] : uv[a0]);
    }
    double q[RPT][4];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = threadIdx.x + 256 * k;
      if constexpr (sizeof(T) == sizeof(double)) {
        const double* row = (i < na || i >= na + ne) ? reinterpret_cast<const double*>(w) + 4 * (size_t)src[k]
                                                     : r + 4 * (size_t)src[k];
        const double2* sp = reinterpret_cast<const double2*>(row);
        const double2 x = sp[0], y = sp[1];
        q[k][0] = x.x; q[k][1] = x.y; q[k][2] = y.x; q[k][3] = y.y;
      } else {
        if (i < na) {
          load4(w, src[k], q[k]);
        } else if (i < na + ne) {
          const double2* sp = reinterpret_cast<const double2*>(r + 4 * (size_t)src[k]);
          const double2 x = sp[0], y = sp[1];
          q[k][0] = x.x; q[k][1] = x.y; q[k][2] = y.x; q[k][3] = y.y;
        }
      }
    }
    // pointer table entries threadIdx.x and (nb = 256 only) 256
    const int t0 = (int)threadIdx.x <= nb ? (int)threadIdx.x : nb;
    const int pv = vptr[v0 + t0], pe = eptr[v0 + t0];
    int pv2 = 0, pe2 = 0;
    if (threadIdx.x == 0 && nb >= 256) { pv2 = vptr[v0 + 256]; pe2 = eptr[v0 + 256]; }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < na + ne) {
        double2* d = reinterpret_cast<double2*>(lds + 4 * i);
        d[0] = make_double2(q[k][0], q[k][1]);
        d[1] = make_double2(q[k][2], q[k][3]);
      }
    }
    if ((int)threadIdx.x <= nb) { lp[threadIdx.x] = pv; lp[nb + 1 + threadIdx.x] = pe; }
    if (threadIdx.x == 0 && nb >= 256) { lp[256] = pv2; lp[nb + 257] = pe2; }
  }
  __syncthreads();
  const double* Lv = lds;
  const double* Le = lds + 4 * na;
  for (int ib = 0; ib < nb; ib += VPR) {
    if (PF == 2) {
      BlockFetch<TW, MV, ME, PK> G;
      block_fetch<TW, LPV, MV, ME, PK>(G, ib + VPR + sub, v0, nb, lane, lp, lvcol, wfg, lecol, we, pk);
      block_compute<T, TW, LPV, MV, ME, PK>(F, v0, nb, o0, lane, Lv, Le, lvcol, wfg, lecol, we, cO, gm1, mode, R, wn,
                                            out, a, b, dt_dev);
      F = G;
    } else {
      if (ib > 0) block_fetch<TW, LPV, MV, ME, PK>(F, ib + sub, v0, nb, lane, lp, lvcol, wfg, lecol, we, pk);
      block_compute<T, TW, LPV, MV, ME, PK>(F, v0, nb, o0, lane, Lv, Le, lvcol, wfg, lecol, we, cO, gm1, mode, R, wn,
                                            out, a, b, dt_dev);
    }
  }
}

template <class T, class TW, int LPV, int MV, int ME, int PF, int WPE, bool PK>
__global__ void __launch_bounds__(256, WPE) k_vertex_blk(const T* __restrict__ w, const int* __restrict__ blk,
                                                         const int* __restrict__ own, const int* __restrict__ uvp,
                                                         const int* __restrict__ uv, const int* __restrict__ uep,
                                                         const int* __restrict__ ue, const int* __restrict__ vptr,
                                                         const unsigned short* __restrict__ lvcol,
                                                         const TW* __restrict__ wfg, const int* __restrict__ eptr,
                                                         const unsigned short* __restrict__ lecol,
                                                         const TW* __restrict__ we, const double* __restrict__ cO,
                                                         const double* __restrict__ r, double gm1, int mode,
                                                         T* __restrict__ R, const T* __restrict__ wn,
                                                         T* __restrict__ out, double a, double b,
                                                         const double* __restrict__ dt_dev,
                                                         const PackedIds* __restrict__ pk) {
  extern __shared__ double lds[];   // [rows][4] state then flux rows, then the block's CSR pointers
  vertex_block2<T, TW, LPV, MV, ME, PF, PK>(xcd_block(blockIdx.x, gridDim.x), lds, w, blk, own, uvp, uv, uep, ue,
                                            vptr, lvcol, wfg, eptr, lecol, we, cO, r, gm1, mode, R, wn, out, a, b,
                                            dt_dev, pk);
}

// State check: counts real rows that are not finite or not physical
// (rho <= 0 or p <= 0) and keeps the smallest such row index.
template <class T>
__global__ void __launch_bounds__(256) k_check_state(const T* __restrict__ w, int nreal, double gm1,
                                                     unsigned long long* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nreal) return;
  double q[4];
  load4(w, v, q);
  const bool finite = isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3]);
  if (finite && physical(q, gm1)) return;
  atomicAdd(&out[0], 1ull);
  atomicMin(&out[1], (unsigned long long)v);
}

__global__ void k_check_reset(unsigned long long* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = 0ull;
    out[1] = ~0ull;
  }
}

// CFL time step: per-block minima of hmin_v / (|u_v| + c_v), then one block
// reduces them and writes cfl * min (two launches: a one-launch form in which
// the last block to arrive, elected by an atomic counter, reduces the minima
// measured 2.5 times slower on the 1025^2 workload).
template <class T>
__global__ void __launch_bounds__(256) k_cfl_partial(const T* __restrict__ w, const double* __restrict__ hmin, int nreal,
                                                     double gamma, double* __restrict__ part) {
  __shared__ double sm[256];
  double best = 1e300;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nreal; v += gridDim.x * blockDim.x) {
    double q[4];
    load4(w, v, q);
    const double ir = 1.0 / q[0];
    const double u = q[1] * ir, vv = q[2] * ir;
    const double p = (gamma - 1.0) * (q[3] - 0.5 * (q[1] * u + q[2] * vv));
    const double s = sqrt(u * u + vv * vv) + sqrt(gamma * p * ir);
    best = fmin(best, hmin[v] / s);
  }
  sm[threadIdx.x] = best;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void __launch_bounds__(256) k_cfl_final(const double* __restrict__ part, int n, double cfl,
                                                   double* __restrict__ dt) {
  __shared__ double sm[256];
  double best = 1e300;
  for (int i = threadIdx.x; i < n; i += blockDim.x) best = fmin(best, part[i]);
  sm[threadIdx.x] = best;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) dt[0] = cfl * sm[0];
}

}  // namespace fdu
