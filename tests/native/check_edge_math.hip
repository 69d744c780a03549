// Host check of the per-edge device math (compiled for the CPU; no GPU call):
// edge_vjp_one against central differences of edge_flux_one on random smooth
// six-point stencils.  Prints the worst relative error and exits non-zero if it
// exceeds the tolerance given on the command line.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "adjoint.hpp"

using namespace fdu;

int main(int argc, char** argv) {
  const double tol = argc > 1 ? std::atof(argv[1]) : 1e-7;
  const int positivity = argc > 2 ? std::atoi(argv[2]) : 1;
  const int power = argc > 3 ? std::atoi(argv[3]) : 1;
  const double eps = argc > 4 ? std::atof(argv[4]) : 1e-6;
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  Scheme S{1.4, 0.4, eps, 0.1, power, 0, positivity};
  double worst = 0.0;
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
    edge_vjp_one(W, g, ob, S, Wb);
    double scale = 0.0;
    for (int s = 0; s < 6; ++s)
      for (int k = 0; k < 4; ++k) scale = std::fmax(scale, std::fabs(Wb[s][k]));
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
  std::printf("worst relative error %.3e\n", worst);
  return worst <= tol ? 0 : 1;
}
