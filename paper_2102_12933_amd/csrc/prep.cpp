// Host preprocessing of a static mesh for the residual kernels: divergence
// stencils and least-squares weights (Sec. 2.2.1-2.2.2), six-point edge
// stencils with Catmull-Rom arc-length coordinates (Sec. 2.3.1), vertex and
// edge ordering.  Runs once per mesh; the weights depend on geometry only.
#include <algorithm>
#include <climits>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <numeric>
#include <thread>

#include "fdu_internal.h"

namespace fdu {
namespace {

constexpr double kTieTol = 1e-12;       // cosines this close count as a tie
constexpr double kRankTol = 1e-10;      // pivoted |R_jj| / |R_00| at or below this: dependent column

template <class F>
void parallel_for(int64_t n, int nthreads, F&& body) {
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  nthreads = (int)std::min<int64_t>(nthreads, std::max<int64_t>(1, n / 64));
  if (nthreads <= 1) {
    body(0, n);
    return;
  }
  std::atomic<int64_t> next(0);
  const int64_t chunk = 256;
  std::vector<std::thread> pool;
  std::vector<std::exception_ptr> errs(nthreads);
  for (int t = 0; t < nthreads; ++t) {
    pool.emplace_back([&, t] {
      try {
        for (;;) {
          int64_t b = next.fetch_add(chunk);
          if (b >= n) break;
          body(b, std::min(n, b + chunk));
        }
      } catch (...) {
        errs[t] = std::current_exception();
      }
    });
  }
  for (auto& th : pool) th.join();
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
}

// Displacements with optional periodic wrap to the nearest image
// (mode 0: none, 1: both directions, 2: y only).
struct Space {
  const double* xy;
  int mode;
  double Lx, Ly;
  void d(int64_t a, int64_t b, double& dx, double& dy) const {
    dx = xy[2 * b] - xy[2 * a];
    dy = xy[2 * b + 1] - xy[2 * a + 1];
    if (mode == 1) dx -= Lx * std::nearbyint(dx / Lx);
    if (mode != 0) dy -= Ly * std::nearbyint(dy / Ly);
  }
};

// Gauss-Legendre rule on [0,1] by Newton iteration on P_n.
void gauss_legendre01(int n, double* u, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    u[i] = 0.5 * (x + 1.0);
    w[i] = 1.0 / ((1.0 - x * x) * dp * dp);   // (2 / ((1-x^2) P'^2)) / 2
  }
}

struct Hermite {
  double u[16], w[16];
  Hermite() { gauss_legendre01(16, u, w); }
  // length of H(t) = h00 P0 + h10 m0 + h01 P1 + h11 m1, t in [0,1]
  double length(const double P0[2], const double P1[2], const double m0[2], const double m1[2]) const {
    double L = 0.0;
    for (int q = 0; q < 16; ++q) {
      double t = u[q];
      double a = 6 * t * t - 6 * t, b = 3 * t * t - 4 * t + 1, c = -6 * t * t + 6 * t, e = 3 * t * t - 2 * t;
      double hx = a * P0[0] + b * m0[0] + c * P1[0] + e * m1[0];
      double hy = a * P0[1] + b * m0[1] + c * P1[1] + e * m1[1];
      L += w[q] * std::sqrt(hx * hx + hy * hy);
    }
    return L;
  }
};

struct Mesh {
  int64_t nv, nreal, ne, nt;
  Space sp;
  const int32_t* edges;
  const int32_t* tris;
  std::vector<int64_t> nb_ptr;   // vertex -> neighbours (ascending)
  std::vector<int32_t> nb_col;
  std::vector<int64_t> vt_ptr;   // vertex -> triangles
  std::vector<int32_t> vt_col;
  std::vector<int32_t> tri_edge; // [nt][3]
  std::vector<int32_t> v_edge;   // vertex -> incident edge ids, aligned with nb_col
  // artificial edges: ids ne .. ne + na - 1, appended to the edge list
  bool use_artificial = false;
  int64_t na = 0;
  std::vector<int32_t> all_edges;   // [ne + na][2] when artificial edges exist
  std::vector<int64_t> art_key;     // sorted (a * nv + b) of the artificial edges

  void build() {
    std::vector<int64_t> deg(nv, 0);
    for (int64_t e = 0; e < ne; ++e) {
      int32_t a = edges[2 * e], b = edges[2 * e + 1];
      if (a < 0 || b < 0 || a >= nv || b >= nv || a == b)
        throw Error(FDU_ERR_INVALID_ARG, "edge " + std::to_string(e) + " has an invalid end id");
      if (a > b) throw Error(FDU_ERR_INVALID_ARG, "edges must be stored with a < b");
      deg[a]++;
      deg[b]++;
    }
    nb_ptr.assign(nv + 1, 0);
    for (int64_t v = 0; v < nv; ++v) nb_ptr[v + 1] = nb_ptr[v] + deg[v];
    nb_col.resize(nb_ptr[nv]);
    v_edge.resize(nb_ptr[nv]);
    std::vector<int64_t> fill(nb_ptr.begin(), nb_ptr.end() - 1);
    for (int64_t e = 0; e < ne; ++e) {
      int32_t a = edges[2 * e], b = edges[2 * e + 1];
      nb_col[fill[a]] = b; v_edge[fill[a]++] = (int32_t)e;
      nb_col[fill[b]] = a; v_edge[fill[b]++] = (int32_t)e;
    }
    for (int64_t v = 0; v < nv; ++v) {
      int64_t s = nb_ptr[v], n = nb_ptr[v + 1] - s;
      std::vector<std::pair<int32_t, int32_t>> tmp(n);
      for (int64_t i = 0; i < n; ++i) tmp[i] = {nb_col[s + i], v_edge[s + i]};
      std::sort(tmp.begin(), tmp.end());
      for (int64_t i = 0; i < n; ++i) {
        if (i && tmp[i].first == tmp[i - 1].first) throw Error(FDU_ERR_INVALID_ARG, "duplicate edge");
        nb_col[s + i] = tmp[i].first;
        v_edge[s + i] = tmp[i].second;
      }
    }
    std::vector<int64_t> tdeg(nv, 0);
    for (int64_t t = 0; t < 3 * nt; ++t) {
      if (tris[t] < 0 || tris[t] >= nv) throw Error(FDU_ERR_INVALID_ARG, "triangle with an invalid vertex id");
      tdeg[tris[t]]++;
    }
    vt_ptr.assign(nv + 1, 0);
    for (int64_t v = 0; v < nv; ++v) vt_ptr[v + 1] = vt_ptr[v] + tdeg[v];
    vt_col.resize(vt_ptr[nv]);
    std::vector<int64_t> f2(vt_ptr.begin(), vt_ptr.end() - 1);
    for (int64_t t = 0; t < nt; ++t)
      for (int k = 0; k < 3; ++k) vt_col[f2[tris[3 * t + k]]++] = (int32_t)t;
    tri_edge.resize(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
      for (int k = 0; k < 3; ++k) {
        int32_t a = tris[3 * t + k], b = tris[3 * t + (k + 1) % 3];
        int32_t e = edge_between(a, b);
        if (e < 0) throw Error(FDU_ERR_INVALID_ARG, "a triangle side is not in the edge list");
        tri_edge[3 * t + k] = e;
      }
  }
  // Far vertex of the triangle across each ring edge of O (a triangle side at
  // O not touching O), when it is neither O nor a neighbour of O.
  void across_vertices(int32_t O, std::vector<int32_t>& out) const {
    out.clear();
    for (int64_t i = vt_ptr[O]; i < vt_ptr[O + 1]; ++i) {
      const int32_t t = vt_col[i];
      int32_t ab[2], n = 0;
      for (int k = 0; k < 3; ++k)
        if (tris[3 * t + k] != O && n < 2) ab[n++] = tris[3 * t + k];
      if (n != 2) continue;
      for (int64_t j = vt_ptr[ab[0]]; j < vt_ptr[ab[0] + 1]; ++j) {
        const int32_t u = vt_col[j];
        if (u == t) continue;
        int32_t K = -1;
        bool has_b = false;
        for (int k = 0; k < 3; ++k) {
          const int32_t x = tris[3 * u + k];
          if (x == ab[1]) has_b = true;
          else if (x != ab[0]) K = x;
        }
        if (!has_b || K < 0 || K == O || edge_between(O, K) >= 0) continue;
        if (std::find(out.begin(), out.end(), K) == out.end()) out.push_back(K);
      }
    }
  }
  int32_t artificial_id(int32_t a, int32_t b) const {
    const int64_t key = (int64_t)std::min(a, b) * nv + std::max(a, b);
    auto it = std::lower_bound(art_key.begin(), art_key.end(), key);
    if (it == art_key.end() || *it != key) return -1;
    return (int32_t)(ne + (it - art_key.begin()));
  }
  int32_t edge_between(int32_t a, int32_t b) const {
    const int32_t* beg = nb_col.data() + nb_ptr[a];
    const int32_t* end = nb_col.data() + nb_ptr[a + 1];
    const int32_t* it = std::lower_bound(beg, end, b);
    if (it == end || *it != b) return -1;
    return v_edge[it - nb_col.data()];
  }
};

// ---------------------------------------------------------------------------
// Six-point edge stencils.
int32_t continuation(const Mesh& m, int32_t cur, double px, double py, const int32_t* excl, int nex) {
  double cmax = -std::numeric_limits<double>::infinity();
  const double pn = std::sqrt(px * px + py * py);
  double cosv[64];
  int32_t ids[64];
  int nc = 0;
  for (int64_t i = m.nb_ptr[cur]; i < m.nb_ptr[cur + 1]; ++i) {
    int32_t q = m.nb_col[i];
    bool skip = false;
    for (int k = 0; k < nex; ++k) skip |= (q == excl[k]);
    if (skip) continue;
    double dx, dy;
    m.sp.d(cur, q, dx, dy);
    double c = (dx * px + dy * py) / (std::sqrt(dx * dx + dy * dy) * pn);
    if (nc >= 64) throw Error(FDU_ERR_INVALID_ARG, "vertex valence above 64");
    cosv[nc] = c;
    ids[nc++] = q;
    cmax = std::max(cmax, c);
  }
  if (nc == 0) throw Error(FDU_ERR_NUMERIC, "an edge has no admissible stencil continuation");
  for (int k = 0; k < nc; ++k)   // neighbours are ascending: the first near-maximum has the smallest id
    if (cosv[k] >= cmax - kTieTol) return ids[k];
  return ids[0];
}

void edge_stencil(const Mesh& m, const Hermite& H, int32_t e, int32_t st[6], double geo[6]) {
  const int32_t L1 = m.edges[2 * e], R1 = m.edges[2 * e + 1];   // L1 = smaller input id
  double dx, dy;
  m.sp.d(R1, L1, dx, dy);
  int32_t ex1[1] = {R1};
  const int32_t L2 = continuation(m, L1, dx, dy, ex1, 1);
  m.sp.d(L1, R1, dx, dy);
  int32_t ex2[1] = {L1};
  const int32_t R2 = continuation(m, R1, dx, dy, ex2, 1);
  m.sp.d(L1, L2, dx, dy);
  int32_t ex3[3] = {L1, R1, R2};
  const int32_t L3 = continuation(m, L2, dx, dy, ex3, 3);
  m.sp.d(R1, R2, dx, dy);
  int32_t ex4[3] = {R1, L1, L2};
  const int32_t R3 = continuation(m, R2, dx, dy, ex4, 3);
  st[0] = L3; st[1] = L2; st[2] = L1; st[3] = R1; st[4] = R2; st[5] = R3;
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j)
      if (st[i] == st[j]) throw Error(FDU_ERR_NUMERIC, "an edge stencil repeats a vertex");

  // unwrapped positions relative to L1
  double pR1[2], pL2[2], pL3[2], pR2[2], pR3[2], t[2];
  m.sp.d(L1, R1, pR1[0], pR1[1]);
  m.sp.d(L1, L2, pL2[0], pL2[1]);
  m.sp.d(L2, L3, dx, dy); pL3[0] = pL2[0] + dx; pL3[1] = pL2[1] + dy;
  m.sp.d(R1, R2, dx, dy); pR2[0] = pR1[0] + dx; pR2[1] = pR1[1] + dy;
  m.sp.d(R2, R3, dx, dy); pR3[0] = pR2[0] + dx; pR3[1] = pR2[1] + dy;
  const double d = std::sqrt(pR1[0] * pR1[0] + pR1[1] * pR1[1]);
  t[0] = pR1[0] / d;
  t[1] = pR1[1] / d;
  const double p0[2] = {0.0, 0.0};
  // curve leaving P1 along +-t through P2 and P3: Catmull-Rom tangent at P2,
  // one-sided tangent at P3, middle-edge direction (scaled by |P2-P1|) at P1
  auto side = [&](const double P1[2], const double P2[2], const double P3[2], double sgn, double& a, double& b) {
    const double l12 = std::sqrt((P2[0] - P1[0]) * (P2[0] - P1[0]) + (P2[1] - P1[1]) * (P2[1] - P1[1]));
    const double m1[2] = {sgn * l12 * t[0], sgn * l12 * t[1]};
    const double m2[2] = {0.5 * (P3[0] - P1[0]), 0.5 * (P3[1] - P1[1])};
    const double m3[2] = {P3[0] - P2[0], P3[1] - P2[1]};
    a = H.length(P1, P2, m1, m2);
    b = H.length(P2, P3, m2, m3);
  };
  double aL, bL, aR, bR;
  side(p0, pL2, pL3, -1.0, aL, bL);
  side(pR1, pR2, pR3, +1.0, aR, bR);
  const double s0 = -0.5 * d - aL - bL, s1 = -0.5 * d - aL, s4 = 0.5 * d + aR, s5 = 0.5 * d + aR + bR;
  geo[0] = s0 / d; geo[1] = s1 / d; geo[2] = s4 / d; geo[3] = s5 / d;
  geo[4] = t[0]; geo[5] = t[1];
}

// ---------------------------------------------------------------------------
// Divergence stencils and least-squares weights.
void divergence_stencil(const Mesh& m, int32_t O, int deg, int level, std::vector<int32_t>& V,
                        std::vector<int32_t>& E) {
  auto tri_edges_of = [&](int32_t J, std::vector<int32_t>& out) {
    for (int64_t i = m.vt_ptr[J]; i < m.vt_ptr[J + 1]; ++i) {
      int32_t t = m.vt_col[i];
      out.push_back(m.tri_edge[3 * t]);
      out.push_back(m.tri_edge[3 * t + 1]);
      out.push_back(m.tri_edge[3 * t + 2]);
    }
  };
  auto uniq = [](std::vector<int32_t>& x) {
    std::sort(x.begin(), x.end());
    x.erase(std::unique(x.begin(), x.end()), x.end());
  };
  auto two_level = [&]() {
    E.clear();
    tri_edges_of(O, E);
    for (int64_t i = m.nb_ptr[O]; i < m.nb_ptr[O + 1]; ++i) tri_edges_of(m.nb_col[i], E);
    uniq(E);
    V.clear();
    for (int32_t e : E) {
      if (m.edges[2 * e] != O) V.push_back(m.edges[2 * e]);
      if (m.edges[2 * e + 1] != O) V.push_back(m.edges[2 * e + 1]);
    }
    uniq(V);
  };
  if (level == 0) level = deg > 3 ? 2 : 1;
  if (level == 1) {
    V.assign(m.nb_col.begin() + m.nb_ptr[O], m.nb_col.begin() + m.nb_ptr[O + 1]);
    E.clear();
    tri_edges_of(O, E);
    uniq(E);
    const int64_t need = (int64_t)deg * (deg + 3) + 4;
    if ((int64_t)(2 * V.size() + E.size()) < need && m.use_artificial) {
      std::vector<int32_t> K;
      m.across_vertices(O, K);
      for (int32_t k : K) {
        const int32_t id = m.artificial_id(O, k);
        if (id < 0) throw Error(FDU_ERR_NUMERIC, "artificial edge missing from the list");
        V.push_back(k);
        E.push_back(id);
      }
      uniq(V);
      uniq(E);
    }
    if ((int64_t)(2 * V.size() + E.size()) < need) two_level();
  } else {
    two_level();
  }
}

// Minimum-norm weight row rho (length m) with A^T rho = e_0 + e_{M+1}
// (A: m x n column-major, overwritten).  Householder QR with column pivoting,
// A P = Q R; columns whose pivot |R_jj| falls below kRankTol |R_00| are
// treated as dependent (rank r), so exactly symmetric stencils still get the
// pseudo-inverse row.  With R11 the leading r x r block and y solving
// R11^T y = (P^T e)[0:r], rho = Q [y; 0].
void ls_row(double* A, int m, int n, int M, double* rho, double* tau, double* z, int* piv, double* cn) {
  for (int j = 0; j < n; ++j) piv[j] = j;
  int r = n;
  double r00 = 0.0;
  for (int j = 0; j < n; ++j) {
    // pivot: remaining column with the largest norm below row j
    int best = j;
    double bn = -1.0;
    for (int c = j; c < n; ++c) {
      const double* b = A + (int64_t)c * m;
      double s = 0.0;
      for (int i = j; i < m; ++i) s += b[i] * b[i];
      cn[c] = s;
      if (s > bn) { bn = s; best = c; }
    }
    if (best != j) {
      std::swap(piv[j], piv[best]);
      double* a = A + (int64_t)j * m;
      double* b = A + (int64_t)best * m;
      for (int i = 0; i < m; ++i) std::swap(a[i], b[i]);
    }
    double* a = A + (int64_t)j * m;
    double alpha = a[j], xn = 0.0;
    for (int i = j + 1; i < m; ++i) xn += a[i] * a[i];
    if (xn == 0.0) {
      tau[j] = 0.0;
    } else {
      double beta = -std::copysign(std::sqrt(alpha * alpha + xn), alpha);
      tau[j] = (beta - alpha) / beta;
      double sc = 1.0 / (alpha - beta);
      for (int i = j + 1; i < m; ++i) a[i] *= sc;
      a[j] = beta;
      for (int c = j + 1; c < n; ++c) {
        double* b = A + (int64_t)c * m;
        double s = b[j];
        for (int i = j + 1; i < m; ++i) s += a[i] * b[i];
        s *= tau[j];
        b[j] -= s;
        for (int i = j + 1; i < m; ++i) b[i] -= s * a[i];
      }
    }
    if (j == 0) r00 = std::fabs(a[0]);
    if (std::fabs(a[j]) <= kRankTol * r00) {
      r = j;
      break;
    }
  }
  if (r == 0) throw Error(FDU_ERR_NUMERIC, "zero least-squares matrix");
  // R11^T y = (P^T e)[0:r]; R_kj = A[j*m + k] for k <= j
  for (int j = 0; j < r; ++j) {
    double s = (piv[j] == 0 || piv[j] == M + 1) ? 1.0 : 0.0;
    for (int k = 0; k < j; ++k) s -= A[(int64_t)j * m + k] * z[k];
    z[j] = s / A[(int64_t)j * m + j];
  }
  // consistency of the dependent columns: R12^T y = (P^T e)[r:n]
  for (int j = r; j < n; ++j) {
    double s = 0.0;
    for (int k = 0; k < r; ++k) s += A[(int64_t)j * m + k] * z[k];
    const double want = (piv[j] == 0 || piv[j] == M + 1) ? 1.0 : 0.0;
    if (std::fabs(s - want) > 1e-8) throw Error(FDU_ERR_NUMERIC, "divergence not determined by the stencil");
  }
  // rho = Q [y; 0] = H_0 ... H_{r-1} [y; 0]
  for (int i = 0; i < m; ++i) rho[i] = i < r ? z[i] : 0.0;
  for (int j = r - 1; j >= 0; --j) {
    if (tau[j] == 0.0) continue;
    const double* v = A + (int64_t)j * m;
    double s = rho[j];
    for (int i = j + 1; i < m; ++i) s += v[i] * rho[i];
    s *= tau[j];
    rho[j] -= s;
    for (int i = j + 1; i < m; ++i) rho[i] -= s * v[i];
  }
}

struct VertexRow {
  std::vector<int32_t> V, E;
  std::vector<double> wf, wg, we;
};

void vertex_weights(const Mesh& m, int32_t O, int deg, int level, VertexRow& row, std::vector<double>& work) {
  divergence_stencil(m, O, deg, level, row.V, row.E);
  const int nV = (int)row.V.size(), nE = (int)row.E.size();
  const int M = deg * (deg + 3) / 2, n = 2 * M, mrows = 2 * nV + nE;
  if (mrows < n) throw Error(FDU_ERR_NUMERIC, "divergence stencil has too few conditions");
  // scale: mean length of the edges at O
  double hO = 0.0;
  for (int64_t i = m.nb_ptr[O]; i < m.nb_ptr[O + 1]; ++i) {
    double dx, dy;
    m.sp.d(O, m.nb_col[i], dx, dy);
    hO += std::sqrt(dx * dx + dy * dy);
  }
  hO /= (double)(m.nb_ptr[O + 1] - m.nb_ptr[O]);
  const double ih = 1.0 / hO;
  work.assign((size_t)mrows * n + mrows + 4 * n, 0.0);
  double* A = work.data();
  double* rho = A + (size_t)mrows * n;
  double* tau = rho + mrows;
  double* z = tau + n;
  double* cn = z + n;
  std::vector<int> piv(n);
  auto put = [&](int r, int col0, double x, double y, double scale) {
    int c = 0;
    for (int d = 1; d <= deg; ++d)
      for (int j = 0; j <= d; ++j, ++c) {
        double v = scale;
        for (int k = 0; k < d - j; ++k) v *= x;
        for (int k = 0; k < j; ++k) v *= y;
        A[(int64_t)(col0 + c) * mrows + r] = v;
      }
  };
  for (int i = 0; i < nV; ++i) {
    double dx, dy;
    m.sp.d(O, row.V[i], dx, dy);
    put(2 * i, 0, dx * ih, dy * ih, 1.0);
    put(2 * i + 1, M, dx * ih, dy * ih, 1.0);
  }
  for (int k = 0; k < nE; ++k) {
    const int32_t a = m.edges[2 * row.E[k]], b = m.edges[2 * row.E[k] + 1];
    double ax, ay, ex, ey;
    m.sp.d(O, a, ax, ay);
    m.sp.d(a, b, ex, ey);
    const double len = std::sqrt(ex * ex + ey * ey);
    const double mx = (ax + 0.5 * ex) * ih, my = (ay + 0.5 * ey) * ih;
    put(2 * nV + k, 0, mx, my, ex / len);
    put(2 * nV + k, M, mx, my, ey / len);
  }
  ls_row(A, mrows, n, M, rho, tau, z, piv.data(), cn);
  row.wf.resize(nV);
  row.wg.resize(nV);
  row.we.resize(nE);
  for (int i = 0; i < nV; ++i) {
    row.wf[i] = rho[2 * i] * ih;
    row.wg[i] = rho[2 * i + 1] * ih;
  }
  for (int k = 0; k < nE; ++k) row.we[k] = rho[2 * nV + k] * ih;
}

// Reverse Cuthill-McKee order of the real vertices (graph restricted to them).
std::vector<int32_t> rcm_order(const Mesh& m) {
  const int64_t n = m.nreal;
  std::vector<int32_t> deg(n, 0);
  for (int64_t v = 0; v < n; ++v)
    for (int64_t i = m.nb_ptr[v]; i < m.nb_ptr[v + 1]; ++i) deg[v] += m.nb_col[i] < n;
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<char> seen(n, 0);
  std::vector<int32_t> level(n, -1);
  auto bfs_far = [&](int32_t s) {  // last vertex of a BFS from s, smallest degree among the farthest
    std::vector<int32_t> q{s};
    std::fill(level.begin(), level.end(), -1);
    level[s] = 0;
    for (size_t h = 0; h < q.size(); ++h) {
      int32_t v = q[h];
      for (int64_t i = m.nb_ptr[v]; i < m.nb_ptr[v + 1]; ++i) {
        int32_t u = m.nb_col[i];
        if (u < n && level[u] < 0) { level[u] = level[v] + 1; q.push_back(u); }
      }
    }
    int32_t best = s, lv = level[q.back()];
    for (int32_t v : q)
      if (level[v] == lv && (deg[v] < deg[best] || level[best] != lv)) best = v;
    return std::make_pair(best, lv);
  };
  for (int64_t root = 0; root < n; ++root) {
    if (seen[root]) continue;
    // pseudo-peripheral start: repeat far-vertex searches while the depth grows
    int32_t s = (int32_t)root;
    auto r = bfs_far(s);
    for (int it = 0; it < 4; ++it) {
      auto r2 = bfs_far(r.first);
      if (r2.second <= r.second) break;
      s = r.first;
      r = r2;
    }
    s = r.first;
    size_t head = order.size();
    order.push_back(s);
    seen[s] = 1;
    std::vector<int32_t> nb;
    for (; head < order.size(); ++head) {
      int32_t v = order[head];
      nb.clear();
      for (int64_t i = m.nb_ptr[v]; i < m.nb_ptr[v + 1]; ++i) {
        int32_t u = m.nb_col[i];
        if (u < n && !seen[u]) { seen[u] = 1; nb.push_back(u); }
      }
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// Position of the cell (x, y) along the Hilbert curve that fills a 2^b x 2^b
// grid (the usual quadrant recursion: at each scale take the quadrant's rank in
// the curve's visiting order, then rotate/reflect the coordinates so the
// sub-square is traversed in the base orientation).
uint64_t hilbert_index(uint32_t x, uint32_t y, int b) {
  const uint32_t n = 1u << b;
  uint64_t d = 0;
  for (uint32_t s = n >> 1; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += (uint64_t)s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = n - 1 - x;
        y = n - 1 - y;
      }
      std::swap(x, y);
    }
  }
  return d;
}

// Real vertices in the order of the Hilbert curve through their coordinates
// (bounding box of the real vertices, 2^16 cells per side; ties by id): a run
// of consecutive ids is a compact patch of the mesh.
std::vector<int32_t> hilbert_order(const Mesh& m, const double* xy) {
  const int64_t n = m.nreal;
  double x0 = xy[0], x1 = xy[0], y0 = xy[1], y1 = xy[1];
  for (int64_t v = 0; v < n; ++v) {
    x0 = std::min(x0, xy[2 * v]); x1 = std::max(x1, xy[2 * v]);
    y0 = std::min(y0, xy[2 * v + 1]); y1 = std::max(y1, xy[2 * v + 1]);
  }
  const int b = 16;
  const double span = std::max(x1 - x0, y1 - y0);
  const double sc = span > 0 ? (double)((1u << b) - 1) / span : 0.0;
  std::vector<std::pair<uint64_t, int32_t>> key(n);
  for (int64_t v = 0; v < n; ++v) {
    const uint32_t qx = (uint32_t)std::lround((xy[2 * v] - x0) * sc);
    const uint32_t qy = (uint32_t)std::lround((xy[2 * v + 1] - y0) * sc);
    key[v] = {hilbert_index(qx, qy, b), (int32_t)v};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = key[i].second;
  return order;
}

}  // namespace
}  // namespace fdu

using namespace fdu;

extern "C" fdu_status fdu_prep_build(fdu_prep** out, int64_t nv_total, int64_t nv_real, const double* xy,
                                     int64_t ne, const int32_t* edges, int64_t nt, const int32_t* tris,
                                     const int32_t* ghost_src, const int8_t* ghost_refl, int periodic,
                                     double Lx, double Ly, int deg, int level, int reorder, int nthreads,
                                     int artificial) {
  return guard([&] {
    if (!out || !xy || !edges || !tris) throw Error(FDU_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (nv_total <= 0 || nv_real <= 0 || nv_real > nv_total || ne <= 0 || nt <= 0)
      throw Error(FDU_ERR_INVALID_ARG, "invalid mesh sizes");
    if (nv_total >= INT32_MAX || ne >= INT32_MAX) throw Error(FDU_ERR_INVALID_ARG, "mesh too large for 32-bit ids");
    if (deg < 1 || deg > 6) throw Error(FDU_ERR_INVALID_ARG, "deg must be in 1..6");
    if (level < 0 || level > 2) throw Error(FDU_ERR_INVALID_ARG, "level must be 0, 1 or 2");
    if (reorder < 0 || reorder > 2) throw Error(FDU_ERR_INVALID_ARG, "reorder must be 0, 1 or 2");
    if (periodic < 0 || periodic > 2) throw Error(FDU_ERR_INVALID_ARG, "periodic must be 0, 1 or 2");
    if (periodic && (!(Lx > 0) || !(Ly > 0))) throw Error(FDU_ERR_INVALID_ARG, "periodic box must be positive");
    const int64_t ng = nv_total - nv_real;
    if (ng > 0 && (!ghost_src || !ghost_refl)) throw Error(FDU_ERR_INVALID_ARG, "ghost arrays required");
    for (int64_t i = 0; i < ng; ++i)
      if (ghost_src[i] < 0 || ghost_src[i] >= nv_real) throw Error(FDU_ERR_INVALID_ARG, "ghost source must be a real vertex");
    for (int64_t i = 0; i < 2 * nv_total; ++i)
      if (!std::isfinite(xy[i])) throw Error(FDU_ERR_INVALID_ARG, "non-finite coordinate");

    Mesh m;
    m.nv = nv_total; m.nreal = nv_real; m.ne = ne; m.nt = nt;
    m.sp = Space{xy, periodic, Lx, Ly};
    m.edges = edges; m.tris = tris;
    m.build();
    if (artificial) {
      // artificial edges for the short one-level stencils (ids after the mesh's edges)
      const int lvl = level == 0 ? (deg > 3 ? 2 : 1) : level;
      std::vector<int64_t> keys;
      if (lvl == 1) {
        std::vector<int32_t> E, K;
        for (int64_t O = 0; O < nv_real; ++O) {
          E.clear();
          for (int64_t i = m.vt_ptr[O]; i < m.vt_ptr[O + 1]; ++i)
            for (int k = 0; k < 3; ++k) E.push_back(m.tri_edge[3 * m.vt_col[i] + k]);
          std::sort(E.begin(), E.end());
          E.erase(std::unique(E.begin(), E.end()), E.end());
          const int64_t cond = 2 * (m.nb_ptr[O + 1] - m.nb_ptr[O]) + (int64_t)E.size();
          if (cond >= (int64_t)deg * (deg + 3) + 4) continue;
          m.across_vertices((int32_t)O, K);
          for (int32_t k : K) keys.push_back(std::min<int64_t>(O, k) * nv_total + std::max<int64_t>(O, k));
        }
      }
      std::sort(keys.begin(), keys.end());
      keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
      if (ne + (int64_t)keys.size() >= INT32_MAX) throw Error(FDU_ERR_INVALID_ARG, "too many edges for 32-bit ids");
      m.art_key = keys;
      m.na = (int64_t)keys.size();
      m.all_edges.assign(edges, edges + 2 * ne);
      for (int64_t key : keys) {
        m.all_edges.push_back((int32_t)(key / nv_total));
        m.all_edges.push_back((int32_t)(key % nv_total));
      }
      m.edges = m.all_edges.data();
      m.use_artificial = true;
    }
    const int64_t ne_all = ne + m.na;

    auto P = new fdu_prep();
    std::unique_ptr<fdu_prep> hold(P);
    P->nv_total = nv_total;
    P->nv_real = nv_real;

    // vertex order: real vertices first (natural or RCM), ghosts after in input order
    std::vector<int32_t> perm(nv_total);
    if (reorder == 1 || reorder == 2) {
      std::vector<int32_t> o = reorder == 1 ? rcm_order(m) : hilbert_order(m, xy);
      std::copy(o.begin(), o.end(), perm.begin());
    } else {
      std::iota(perm.begin(), perm.begin() + nv_real, 0);
    }
    std::iota(perm.begin() + nv_real, perm.end(), (int32_t)nv_real);
    std::vector<int32_t> iperm(nv_total);
    for (int64_t i = 0; i < nv_total; ++i) iperm[perm[i]] = (int32_t)i;

    // least-squares rows of every real vertex (input numbering)
    std::vector<VertexRow> rows(nv_real);
    parallel_for(nv_real, nthreads, [&](int64_t b, int64_t e) {
      std::vector<double> work;
      for (int64_t v = b; v < e; ++v) vertex_weights(m, (int32_t)v, deg, level, rows[v], work);
    });

    // flux edges: every edge a divergence stencil uses, ordered by new end ids
    std::vector<char> need(ne_all, 0);
    for (auto& r : rows)
      for (int32_t e : r.E) need[e] = 1;
    std::vector<int32_t> fe;
    for (int64_t e = 0; e < ne_all; ++e)
      if (need[e]) fe.push_back((int32_t)e);
    auto key = [&](int32_t e) {
      int32_t a = iperm[m.edges[2 * e]], b = iperm[m.edges[2 * e + 1]];
      return std::make_pair(std::min(a, b), std::max(a, b));
    };
    std::sort(fe.begin(), fe.end(), [&](int32_t x, int32_t y) { return key(x) < key(y); });
    const int64_t nf = (int64_t)fe.size();
    std::vector<int32_t> floc(ne_all, -1);
    for (int64_t i = 0; i < nf; ++i) floc[fe[i]] = (int32_t)i;
    P->ne_flux = nf;
    P->flux_edge = fe;
    P->sten6.resize(6 * nf);
    P->geo.resize(6 * nf);
    Hermite H;
    parallel_for(nf, nthreads, [&](int64_t b, int64_t e) {
      for (int64_t i = b; i < e; ++i) {
        int32_t st[6];
        edge_stencil(m, H, fe[i], st, &P->geo[6 * i]);
        for (int k = 0; k < 6; ++k) P->sten6[6 * i + k] = iperm[st[k]];
      }
    });

    // CSR in the new numbering, entries sorted by column
    P->vptr.assign(nv_real + 1, 0);
    P->eptr.assign(nv_real + 1, 0);
    // accumulated in 64 bits: the library's CSR pointers are 32-bit offsets
    int64_t nvsum = 0, nesum = 0;
    for (int64_t i = 0; i < nv_real; ++i) {
      const VertexRow& r = rows[perm[i]];
      nvsum += (int64_t)r.V.size();
      nesum += (int64_t)r.E.size();
      if (nvsum > INT32_MAX || nesum > INT32_MAX)
        throw Error(FDU_ERR_INVALID_ARG, "stencils too large: more than 2^31 - 1 entries");
      P->vptr[i + 1] = (int32_t)nvsum;
      P->eptr[i + 1] = (int32_t)nesum;
    }
    P->nnz_v = P->vptr[nv_real];
    P->nnz_e = P->eptr[nv_real];
    P->vcol.resize(P->nnz_v);
    P->wfg.resize(2 * P->nnz_v);
    P->ecol.resize(P->nnz_e);
    P->we.resize(P->nnz_e);
    parallel_for(nv_real, nthreads, [&](int64_t b, int64_t e) {
      std::vector<std::pair<int32_t, int32_t>> idx;
      for (int64_t i = b; i < e; ++i) {
        const VertexRow& r = rows[perm[i]];
        idx.clear();
        for (size_t k = 0; k < r.V.size(); ++k) idx.push_back({iperm[r.V[k]], (int32_t)k});
        std::sort(idx.begin(), idx.end());
        for (size_t k = 0; k < idx.size(); ++k) {
          int64_t p = P->vptr[i] + k;
          P->vcol[p] = idx[k].first;
          P->wfg[2 * p] = r.wf[idx[k].second];
          P->wfg[2 * p + 1] = r.wg[idx[k].second];
        }
        idx.clear();
        for (size_t k = 0; k < r.E.size(); ++k) idx.push_back({floc[r.E[k]], (int32_t)k});
        std::sort(idx.begin(), idx.end());
        for (size_t k = 0; k < idx.size(); ++k) {
          int64_t p = P->eptr[i] + k;
          P->ecol[p] = idx[k].first;
          P->we[p] = r.we[idx[k].second];
        }
      }
    });

    // shortest incident edge of each real vertex (CFL)
    P->hmin.resize(nv_real);
    for (int64_t i = 0; i < nv_real; ++i) {
      int32_t v = perm[i];
      double h = std::numeric_limits<double>::infinity();
      for (int64_t k = m.nb_ptr[v]; k < m.nb_ptr[v + 1]; ++k) {
        double dx, dy;
        m.sp.d(v, m.nb_col[k], dx, dy);
        h = std::min(h, std::sqrt(dx * dx + dy * dy));
      }
      P->hmin[i] = h;
    }
    P->ghost_src.resize(ng);
    P->ghost_refl.resize(ng);
    for (int64_t g = 0; g < ng; ++g) {
      P->ghost_src[g] = iperm[ghost_src[g]];
      P->ghost_refl[g] = ghost_refl[g];
    }
    P->n_artificial = m.na;
    P->artificial.assign(m.all_edges.begin() + (m.na ? 2 * ne : 0), m.all_edges.end());
    P->perm = std::move(perm);
    P->iperm = std::move(iperm);
    *out = hold.release();
  });
}

extern "C" fdu_status fdu_prep_view_get(const fdu_prep* p, fdu_prep_view* v) {
  return guard([&] {
    if (!p || !v) throw Error(FDU_ERR_INVALID_ARG, "NULL argument");
    v->nv_total = p->nv_total;
    v->nv_real = p->nv_real;
    v->ne_flux = p->ne_flux;
    v->nnz_v = p->nnz_v;
    v->nnz_e = p->nnz_e;
    v->perm = p->perm.data();
    v->iperm = p->iperm.data();
    v->flux_edge = p->flux_edge.data();
    v->sten6 = p->sten6.data();
    v->geo = p->geo.data();
    v->vptr = p->vptr.data();
    v->vcol = p->vcol.data();
    v->wfg = p->wfg.data();
    v->eptr = p->eptr.data();
    v->ecol = p->ecol.data();
    v->we = p->we.data();
    v->hmin = p->hmin.data();
    v->ghost_src = p->ghost_src.data();
    v->ghost_refl = p->ghost_refl.data();
    v->n_artificial = p->n_artificial;
    v->artificial = p->artificial.data();
  });
}

extern "C" void fdu_prep_destroy(fdu_prep* p) { delete p; }
