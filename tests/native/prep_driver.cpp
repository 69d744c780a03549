// Host driver for the mesh preprocessing (CPU only, no GPU): builds a jittered
// periodic triangulated lattice and a walled one with mirror ghosts, runs
// fdu_prep_build on both (RCM and Hilbert orders, degrees 3 and 5, with and
// without artificial edges) and checks the returned view.  Built with address
// and undefined-behaviour sanitizers by the test that runs it.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include <string>

#include "fdu.h"

// The library keeps its error text in the runtime translation unit (HIP);
// this host-only build supplies the same two functions.
namespace fdu {
static thread_local std::string g_error;
void set_last_error(const std::string& msg) { g_error = msg; }
}  // namespace fdu
extern "C" const char* fdu_last_error(void) { return fdu::g_error.c_str(); }

struct Lattice {
  std::vector<double> xy;
  std::vector<int32_t> edges, tris, gsrc;
  std::vector<int8_t> grefl;
  int64_t nv_total = 0, nv_real = 0;
};

static void add_quad(Lattice& L, int32_t a, int32_t b, int32_t c, int32_t d, bool main_diag) {
  // quad a=(i,j) b=(i+1,j) c=(i,j+1) d=(i+1,j+1)
  const int32_t t[2][3] = {{a, b, main_diag ? d : c}, {main_diag ? a : b, d, c}};
  for (auto& tr : t)
    for (int k = 0; k < 3; ++k) L.tris.push_back(tr[k]);
}

static void finish_edges(Lattice& L) {
  std::vector<std::pair<int32_t, int32_t>> e;
  for (size_t t = 0; t < L.tris.size(); t += 3)
    for (int k = 0; k < 3; ++k) {
      int32_t a = L.tris[t + k], b = L.tris[t + (k + 1) % 3];
      e.push_back({std::min(a, b), std::max(a, b)});
    }
  std::sort(e.begin(), e.end());
  e.erase(std::unique(e.begin(), e.end()), e.end());
  for (auto& p : e) {
    L.edges.push_back(p.first);
    L.edges.push_back(p.second);
  }
}

static Lattice periodic_lattice(int N, double jitter, unsigned seed) {
  Lattice L;
  std::mt19937 rng(seed);
  std::uniform_real_distribution<double> U(-jitter, jitter);
  const double h = 1.0 / N;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      L.xy.push_back(i * h + U(rng) * h);
      L.xy.push_back(j * h + U(rng) * h);
    }
  auto id = [&](int i, int j) { return (int32_t)(((i + N) % N) * N + (j + N) % N); };
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) add_quad(L, id(i, j), id(i + 1, j), id(i, j + 1), id(i + 1, j + 1), rng() & 1);
  L.nv_total = L.nv_real = (int64_t)N * N;
  finish_edges(L);
  return L;
}

// walled N x N lattice on [0,1]^2 with a G-deep mirror ghost layer (lattice of
// (N+2G)^2 points, the outer ones ghosts of their mirror images)
static Lattice walled_lattice(int N, int G, unsigned seed) {
  Lattice L;
  std::mt19937 rng(seed);
  const int M = N + 2 * G;
  const double h = 1.0 / (N - 1);
  std::vector<int32_t> ids((size_t)M * M);
  auto mirror = [&](int k) { return k < 0 ? -k : (k > N - 1 ? 2 * (N - 1) - k : k); };
  int32_t next_ghost = N * N;
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < M; ++b) {
      const int i = a - G, j = b - G;
      const bool real = i >= 0 && i < N && j >= 0 && j < N;
      ids[(size_t)a * M + b] = real ? i * N + j : next_ghost++;
    }
  L.nv_real = (int64_t)N * N;
  L.nv_total = next_ghost;
  L.xy.assign(2 * L.nv_total, 0.0);
  L.gsrc.assign(L.nv_total - L.nv_real, 0);
  L.grefl.assign(L.nv_total - L.nv_real, 0);
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < M; ++b) {
      const int i = a - G, j = b - G;
      const int32_t v = ids[(size_t)a * M + b];
      L.xy[2 * v] = i * h;
      L.xy[2 * v + 1] = j * h;
      if (v >= L.nv_real) {
        L.gsrc[v - L.nv_real] = mirror(i) * N + mirror(j);
        L.grefl[v - L.nv_real] = (int8_t)((j < 0 || j > N - 1) ? 2 : 0);
      }
    }
  for (int a = 0; a + 1 < M; ++a)
    for (int b = 0; b + 1 < M; ++b)
      add_quad(L, ids[(size_t)a * M + b], ids[(size_t)(a + 1) * M + b], ids[(size_t)a * M + b + 1],
               ids[(size_t)(a + 1) * M + b + 1], ((a + b) & 1) == 0);
  (void)rng;
  finish_edges(L);
  return L;
}

static int run(const Lattice& L, int periodic, int deg, int reorder, int artificial) {
  fdu_prep* p = nullptr;
  const int64_t ng = L.nv_total - L.nv_real;
  fdu_status st = fdu_prep_build(&p, L.nv_total, L.nv_real, L.xy.data(), (int64_t)L.edges.size() / 2,
                                 L.edges.data(), (int64_t)L.tris.size() / 3, L.tris.data(),
                                 ng ? L.gsrc.data() : nullptr, ng ? L.grefl.data() : nullptr, periodic, 1.0, 1.0,
                                 deg, 0, reorder, 2, artificial);
  if (st != FDU_OK) {
    std::printf("prep failed: %s\n", fdu_last_error());
    return 1;
  }
  fdu_prep_view v;
  if (fdu_prep_view_get(p, &v) != FDU_OK) return 1;
  int bad = 0;
  for (int64_t i = 0; i < v.nv_real; ++i) bad += v.vptr[i + 1] < v.vptr[i] || v.eptr[i + 1] < v.eptr[i];
  for (int64_t k = 0; k < v.nnz_v; ++k) bad += v.vcol[k] < 0 || v.vcol[k] >= v.nv_total;
  for (int64_t k = 0; k < v.nnz_e; ++k) bad += v.ecol[k] < 0 || v.ecol[k] >= v.ne_flux;
  for (int64_t k = 0; k < 6 * v.ne_flux; ++k) bad += v.sten6[k] < 0 || v.sten6[k] >= v.nv_total;
  std::printf("nv %lld flux edges %lld nnz %lld + %lld artificial %lld bad %d\n", (long long)v.nv_total,
              (long long)v.ne_flux, (long long)v.nnz_v, (long long)v.nnz_e, (long long)v.n_artificial, bad);
  fdu_prep_destroy(p);
  return bad != 0;
}

int main() {
  int fails = 0;
  const Lattice P = periodic_lattice(24, 0.15, 3);
  const Lattice W = walled_lattice(14, 4, 5);
  for (int reorder = 1; reorder <= 2; ++reorder) {
    fails += run(P, 1, 5, reorder, 0);
    fails += run(P, 1, 3, reorder, 1);
    fails += run(W, 0, 5, reorder, 0);
    fails += run(W, 0, 3, reorder, 1);
  }
  // invalid input is an error status, not a crash
  fdu_prep* p = nullptr;
  std::vector<int32_t> bad_edges(P.edges);
  bad_edges[0] = -1;
  if (fdu_prep_build(&p, P.nv_total, P.nv_real, P.xy.data(), (int64_t)bad_edges.size() / 2, bad_edges.data(),
                     (int64_t)P.tris.size() / 3, P.tris.data(), nullptr, nullptr, 1, 1.0, 1.0, 5, 0, 1, 2, 0) !=
      FDU_ERR_INVALID_ARG)
    ++fails;
  std::printf("%s\n", fails ? "FAIL" : "OK");
  return fails;
}
