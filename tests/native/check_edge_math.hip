// Host check of the per-edge device math (compiled for the CPU; no GPU call):
// edge_vjp_one against central differences of edge_flux_one on random smooth
// six-point stencils, and against a forward-mode dual-number derivation of the
// same cotangents.  Prints the worst relative errors and exits non-zero if
// they exceed the tolerances (finite differences: command line; dual numbers:
// 1e-11).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "adjoint.hpp"

using namespace fdu;

using D8 = Dual<8>;

// Second, independent route to the same cotangents: the Riemann flux and the
// Roe-averaged frame differentiated with 8-direction forward-mode dual
// numbers (the library's reverse sweep is written out by hand).
void edge_vjp_dual(const double W[6][4], const double g[6], const double ob[4], const Scheme& S,
                         double Wb[6][4]) {
  const double nx = g[4], ny = g[5];
  // ---- forward recomputation
  const Frame F = roe_frame<double>(W[2], W[3], nx, ny, S.gm1);
  double Cv[6][4];
#pragma unroll
  for (int k = 0; k < 6; ++k) to_char(F, S.gm1, W[k], Cv[k]);
  WenoGeom GL, GR;
  weno_geom(g[0], g[1], g[2], GL);
  weno_geom(-g[3], -g[2], -g[1], GR);
  double cl[4], cr[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double ul[5] = {Cv[0][c], Cv[1][c], Cv[2][c], Cv[3][c], Cv[4][c]};
    const double ur[5] = {Cv[5][c], Cv[4][c], Cv[3][c], Cv[2][c], Cv[1][c]};
    cl[c] = weno_eval(GL, ul, S.eps, S.power);
    cr[c] = weno_eval(GR, ur, S.eps, S.power);
  }
  double wl[4], wr[4];
  from_char(F, cl, wl);
  from_char(F, cr, wr);
  bool fl = false, fr = false;
  if (S.positivity) {
    fl = !physical(wl, S.gm1);
    fr = !physical(wr, S.gm1);
    if (fl)
#pragma unroll
      for (int k = 0; k < 4; ++k) wl[k] = W[2][k];
    if (fr)
#pragma unroll
      for (int k = 0; k < 4; ++k) wr[k] = W[3][k];
  }

#pragma unroll
  for (int s = 0; s < 6; ++s)
#pragma unroll
    for (int k = 0; k < 4; ++k) Wb[s][k] = 0.0;

  // ---- Riemann flux: Jacobian by dual numbers over (wl, wr)
  double wlb[4], wrb[4];
  {
    D8 a[4], b[4], o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = D8(wl[k]);
      a[k].d[k] = 1.0;
      b[k] = D8(wr[k]);
      b[k].d[4 + k] = 1.0;
    }
    riemann_flux<D8>(a, b, nx, ny, S, o);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double sl = 0.0, sr = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        sl += ob[i] * o[i].d[k];
        sr += ob[i] * o[i].d[4 + k];
      }
      wlb[k] = sl;
      wrb[k] = sr;
    }
  }
  if (fl) {
#pragma unroll
    for (int k = 0; k < 4; ++k) Wb[2][k] += wlb[k];
  }
  if (fr) {
#pragma unroll
    for (int k = 0; k < 4; ++k) Wb[3][k] += wrb[k];
  }

  // ---- back-projection and WENO, at the fixed frame
  double clb[4] = {0.0, 0.0, 0.0, 0.0}, crb[4] = {0.0, 0.0, 0.0, 0.0};
  if (!fl) from_char_T(F, wlb, clb);
  if (!fr) from_char_T(F, wrb, crb);
  double Cb[6][4];
#pragma unroll
  for (int s = 0; s < 6; ++s)
#pragma unroll
    for (int k = 0; k < 4; ++k) Cb[s][k] = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double ul[5] = {Cv[0][c], Cv[1][c], Cv[2][c], Cv[3][c], Cv[4][c]};
    const double ur[5] = {Cv[5][c], Cv[4][c], Cv[3][c], Cv[2][c], Cv[1][c]};
    double ubl[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, ubr[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    weno_eval_T(GL, ul, S.eps, S.power, clb[c], ubl);
    weno_eval_T(GR, ur, S.eps, S.power, crb[c], ubr);
#pragma unroll
    for (int m = 0; m < 5; ++m) Cb[m][c] += ubl[m];
#pragma unroll
    for (int m = 0; m < 5; ++m) Cb[5 - m][c] += ubr[m];
  }
  // characteristic projection at the fixed frame
#pragma unroll
  for (int s = 0; s < 6; ++s) to_char_T_acc(F, S.gm1, Cb[s], Wb[s]);

  // ---- frame dependence on the end states (W[2], W[3]) by dual numbers
  {
    D8 a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = D8(W[2][k]);
      a[k].d[k] = 1.0;
      b[k] = D8(W[3][k]);
      b[k].d[4 + k] = 1.0;
    }
    const FrameT<D8> Fd = roe_frame<D8>(a, b, nx, ny, S.gm1);
    double fb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto acc = [&](const D8 o[4], const double cot[4]) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) t += cot[i] * o[i].d[j];
        fb[j] += t;
      }
    };
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      D8 q[4], o[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) q[k] = D8(W[s][k]);
      to_char<D8>(Fd, S.gm1, q, o);
      acc(o, Cb[s]);
    }
    if (!fl) {
      D8 q[4], o[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) q[k] = D8(cl[k]);
      from_char<D8>(Fd, q, o);
      acc(o, wlb);
    }
    if (!fr) {
      D8 q[4], o[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) q[k] = D8(cr[k]);
      from_char<D8>(Fd, q, o);
      acc(o, wrb);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Wb[2][k] += fb[k];
      Wb[3][k] += fb[4 + k];
    }
  }
}




int main(int argc, char** argv) {
  const double tol = argc > 1 ? std::atof(argv[1]) : 1e-7;
  const int positivity = argc > 2 ? std::atoi(argv[2]) : 1;
  const int power = argc > 3 ? std::atoi(argv[3]) : 1;
  const double eps = argc > 4 ? std::atof(argv[4]) : 1e-6;
  const int riemann = argc > 5 ? std::atoi(argv[5]) : 0;
  const int conservative = argc > 6 ? std::atoi(argv[6]) : 0;
  const int uniform = argc > 7 ? std::atoi(argv[7]) : 0;
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  Scheme S{1.4, 0.4, eps, 0.1, power, riemann, positivity, conservative, uniform};
  const bool dual_ok = !conservative && !uniform;   // the dual-number route covers the paper's scheme
  double worst = 0.0, worst_dual = 0.0;
  for (int trial = 0; trial < 200; ++trial) {
    double W[6][4], g[6];
    // smooth stencil data: a state plus a smooth variation along the stencil
    const double rho = 0.8 + 0.4 * U(rng), u = 0.6 * (U(rng) - 0.5), v = 0.6 * (U(rng) - 0.5), p = 0.7 + 0.6 * U(rng);
    const double sl[4] = {0.1 * (U(rng) - 0.5), 0.1 * (U(rng) - 0.5), 0.1 * (U(rng) - 0.5), 0.1 * (U(rng) - 0.5)};
    const double xs[6] = {-2.5 - 0.3 * U(rng), -1.5 - 0.3 * U(rng), -0.5, 0.5, 1.5 + 0.3 * U(rng), 2.5 + 0.3 * U(rng)};
    for (int s = 0; s < 6; ++s) {
      const double x = xs[s];
      const double r = rho * (1 + sl[0] * x + 0.02 * x * x), uu = u + sl[1] * x, vv = v + sl[2] * x,
                   pp = p * (1 + sl[3] * x);
      W[s][0] = r; W[s][1] = r * uu; W[s][2] = r * vv; W[s][3] = pp / 0.4 + 0.5 * r * (uu * uu + vv * vv);
    }
    const double a = 2 * M_PI * U(rng);
    g[0] = xs[0]; g[1] = xs[1]; g[2] = xs[4]; g[3] = xs[5]; g[4] = std::cos(a); g[5] = std::sin(a);
    double ob[4];
    for (int k = 0; k < 4; ++k) ob[k] = U(rng) - 0.5;
    double Wb[6][4];
    edge_vjp_one([&](int k, double q[4], bool) { for (int i = 0; i < 4; ++i) q[i] = W[k][i]; }, g, ob, S,
                 [&](int k, const double q[4]) { for (int i = 0; i < 4; ++i) Wb[k][i] = q[i]; });
    double scale = 0.0;
    for (int s = 0; s < 6; ++s)
      for (int k = 0; k < 4; ++k) scale = std::fmax(scale, std::fabs(Wb[s][k]));
    double Wd[6][4];
    edge_vjp_dual(W, g, ob, S, Wd);
    for (int s = 0; s < 6 && dual_ok; ++s)
      for (int k = 0; k < 4; ++k) {
        const double err = std::fabs(Wd[s][k] - Wb[s][k]) / scale;
        if (err > worst_dual) worst_dual = err;
        if (err > 1e-11 && trial < 3)
          std::printf("trial %d slot %d comp %d: vjp %.14e dual %.14e\n", trial, s, k, Wb[s][k], Wd[s][k]);
      }
    for (int s = 0; s < 6; ++s)
      for (int k = 0; k < 4; ++k) {
        const double h = 1e-6 * std::fmax(1.0, std::fabs(W[s][k]));
        double Wp[6][4], Wm[6][4], op[4], om[4];
        for (int i = 0; i < 6; ++i)
          for (int j = 0; j < 4; ++j) Wp[i][j] = Wm[i][j] = W[i][j];
        Wp[s][k] += h;
        Wm[s][k] -= h;
        edge_flux_one(Wp, g, S, op);
        edge_flux_one(Wm, g, S, om);
        double fd = 0.0;
        for (int i = 0; i < 4; ++i) fd += ob[i] * (op[i] - om[i]) / (2 * h);
        const double err = std::fabs(fd - Wb[s][k]) / scale;
        if (err > worst) worst = err;
        if (err > tol && trial < 3) std::printf("trial %d slot %d comp %d: vjp %.10e fd %.10e\n", trial, s, k, Wb[s][k], fd);
      }
  }
  std::printf("worst relative error: finite differences %.3e, dual numbers %.3e\n", worst, worst_dual);
  return worst <= tol && worst_dual <= 1e-11 ? 0 : 1;
}
