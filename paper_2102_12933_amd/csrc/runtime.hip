// libfdu runtime: device buffers of one mesh instance, uploads with
// validation, kernel launches and the C ABI of include/fdu.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fdu_internal.h"
#include "kernels.hpp"
#include "adjoint.hpp"
#include "batch.hpp"

namespace fdu {

thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

#define FDU_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::fdu::Error(e_ == hipErrorOutOfMemory ? FDU_ERR_OOM : FDU_ERR_HIP,           \
                         std::string(#call) + ": " + hipGetErrorString(e_));              \
  } while (0)

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    FDU_HIP(hipMalloc(&p, count * sizeof(T)));
    n = count;
  }
  void upload(const T* h, size_t count) {
    alloc(count);
    if (count) FDU_HIP(hipMemcpy(p, h, count * sizeof(T), hipMemcpyHostToDevice));
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  ~DevBuf() { release(); }
};

}  // namespace fdu

using namespace fdu;

// Stage states of fdu_rk_step_static, for callers that cannot allocate: one
// file-scope device array, which every GPU the library runs on holds (its own
// copy) until the process ends.  Host code never uses the array's name as an
// address: the device address of each GPU's copy is taken once per device with
// hipGetSymbolAddress (fdu_create, with that device current) and kept in
// g_static_scratch.
constexpr size_t kStaticScratchBytes = size_t(80) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_scratch[kMaxDevices] = {};

// With `device` current: records the device address of its copy of the array.
void static_scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (device < 0 || device >= kMaxDevices) throw Error(FDU_ERR_UNSUPPORTED, "device index beyond 63");
  if (g_static_scratch[device]) return;
  void* p = nullptr;
  FDU_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error(FDU_ERR_HIP, "hipGetSymbolAddress returned no address for the static stage states");
  g_static_scratch[device] = p;
}

void* static_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_static_mu);
  return (device >= 0 && device < kMaxDevices) ? g_static_scratch[device] : nullptr;
}
}  // namespace

struct fdu_solver {
  int device = 0;
  fdu_precision prec = FDU_F64;
  fdu_params params{};
  int64_t nv_total = 0, nv_real = 0, ne_flux = 0, nnz_v = 0, nnz_e = 0, ng = 0;
  bool have_edges = false, have_vertices = false, finalized = false;
  // host copies (c_O needs the edge directions and weights; the adjoint's
  // transposed maps need the stencils)
  std::vector<double> h_geo, h_we, h_wfg, h_cO;
  std::vector<int32_t> h_eptr, h_ecol, h_vptr, h_vcol, h_sten, h_gsrc;
  std::vector<int8_t> h_grefl;
  // adjoint: transposed maps and work buffers (fdu_enable_adjoint)
  bool adjoint = false;
  DevBuf<int32_t> te_ptr, te_row, tv_ptr, tv_row, ts_ptr, ts_col, tg_ptr, tg_col;
  DevBuf<double> te_w, tv_wfg, sfg, rbar, slots, vtmp;
  DevBuf<float> te_w32, tv_wfg32;
  DevBuf<int32_t> sten, vptr, vcol, eptr, ecol, gsrc;
  DevBuf<int8_t> grefl;
  DevBuf<double> gstate;     // [ng][4] Dirichlet ghost states (rows of other ghosts unused)
  int64_t n_dirichlet = 0;
  DevBuf<double> geo, wfg, we, cO, hmin, flux, part;
  // meshes with ghosts: a state-sized copy that fdu_residual and
  // fdu_residual_vjp fill (real rows copied, ghost rows filled) so that the
  // caller's state stays read-only
  DevBuf<unsigned char> wcopy;
  DevBuf<double> dt_adj;     // fdu_rk_step_vjp: the step's dt on the device (adjoint set-up)
  DevBuf<unsigned long long> chk;   // fdu_check_state: count, first bad row
  DevBuf<float> geo32, wfg32, we32;
  int cfl_blocks = 0;
  // vertex blocks with their stencil halos (LDS-staged vertex variants)
  DevBuf<int32_t> vblk, vb_own, vb_uvp, vb_uv, vb_uep, vb_ue;
  DevBuf<uint16_t> vb_lvcol, vb_lecol;
  DevBuf<PackedIds> vb_pk;   // packed first-round ids per real vertex and lane (vertex variants 4-5)
  int n_vblocks = 0, vb_rows_max = 0;
  // live kernel timer (fdu_kernel_timer_start/stop): event pairs recorded
  // around each launch of the ghost, edge, vertex and CFL kernels
  bool timer_on = false;
  int timer_cap = 0, timer_mask = 0;
  int timer_n[4] = {0, 0, 0, 0};
  std::vector<hipEvent_t> timer_ev[4];
  ~fdu_solver() {
    for (auto& v : timer_ev)
      for (hipEvent_t e : v) (void)hipEventDestroy(e);
  }
  int edge_variant = 1;    // 0: k_edge_flux, 1: k_edge_flux_lean
  int vertex_variant = 4;  // 0-1: k_vertex (strided loops, 16 and 8 lanes), 2: k_vertex_pipe,
                           // 3: k_vertex_lds, 4-5: k_vertex_blk (packed first-round ids; 5: prefetch)
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int d) {
    FDU_HIP(hipGetDevice(&prev));
    if (prev != d) FDU_HIP(hipSetDevice(d));
  }
  ~DeviceGuard() {
    int cur;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

void need(bool c, const char* msg) {
  if (!c) throw Error(FDU_ERR_INVALID_ARG, msg);
}

void check_csr(const int32_t* ptr, int64_t n, const int32_t* col, int64_t ncol_max, const char* what, int64_t& nnz) {
  need(ptr && col, "NULL CSR array");
  need(ptr[0] == 0, "CSR pointer must start at 0");
  for (int64_t i = 0; i < n; ++i)
    if (ptr[i + 1] < ptr[i]) throw Error(FDU_ERR_INVALID_ARG, std::string(what) + ": CSR pointer not monotone");
  nnz = ptr[n];
  for (int64_t p = 0; p < nnz; ++p)
    if (col[p] < 0 || col[p] >= ncol_max) throw Error(FDU_ERR_INVALID_ARG, std::string(what) + ": column id out of range");
}

void check_finite(const double* x, int64_t n, const char* what) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) throw Error(FDU_ERR_INVALID_ARG, std::string(what) + ": non-finite value");
}

Scheme scheme_of(const fdu_solver* s) {
  Scheme S;
  S.gamma = s->params.gamma;
  S.gm1 = s->params.gamma - 1.0;
  S.eps = s->params.weno_eps;
  S.efrac = s->params.entropy_frac;
  S.power = s->params.weno_power;
  S.riemann = s->params.riemann;
  S.positivity = s->params.positivity;
  S.conservative = s->params.interpolation;
  S.uniform = s->params.uniform_weno;
  return S;
}

void ready(const fdu_solver* s) {
  if (!s) throw Error(FDU_ERR_INVALID_ARG, "NULL solver");
  if (!s->finalized) throw Error(FDU_ERR_STATE, "solver not finalized");
}

inline unsigned nblocks(int64_t nthreads) { return (unsigned)((nthreads + 255) / 256); }

void launch_check() { FDU_HIP(hipGetLastError()); }

// Records a start/stop event pair around `launch` when the solver's live timer
// is on and has room (never while the stream is being captured).
template <class F>
void timed_launch(fdu_solver* s, int phase, hipStream_t st, F&& launch) {
  bool rec = s->timer_on && ((s->timer_mask >> phase) & 1) && s->timer_n[phase] < s->timer_cap;
  if (rec) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    FDU_HIP(hipStreamIsCapturing(st, &cs));
    rec = cs == hipStreamCaptureStatusNone;
  }
  if (!rec) {
    launch();
    return;
  }
  const int i = s->timer_n[phase]++;
  FDU_HIP(hipEventRecord(s->timer_ev[phase][2 * i], st));
  launch();
  FDU_HIP(hipEventRecord(s->timer_ev[phase][2 * i + 1], st));
}

template <class T>
void fill_ghosts_t(fdu_solver* s, T* w, hipStream_t st) {
  if (s->ng == 0) return;
  timed_launch(s, 0, st, [&] {
    hipLaunchKernelGGL(k_fill_ghosts<T>, dim3(nblocks(s->ng)), dim3(256), 0, st, w, (int)s->nv_real, (int)s->ng,
                       s->gsrc.p, reinterpret_cast<const signed char*>(s->grefl.p), s->gstate.p);
  });
  launch_check();
}

constexpr int kEdgeVariants = 2;
constexpr int kVertexVariants = 6;

template <class T, class TG>
void edge_flux_launch(fdu_solver* s, const T* w, const TG* geo, double* r, hipStream_t st) {
  const Scheme S = scheme_of(s);
  const dim3 grid(nblocks(s->ne_flux)), block(256);
  if (s->edge_variant == 1)
    hipLaunchKernelGGL((k_edge_flux_lean<T, TG>), grid, block, 0, st, w, s->sten.p, geo, r, (int)s->ne_flux, S);
  else
    hipLaunchKernelGGL((k_edge_flux<T, TG>), grid, block, 0, st, w, s->sten.p, geo, r, (int)s->ne_flux, S);
}

template <class T>
void edge_flux_t(fdu_solver* s, const T* w, double* r, hipStream_t st) {
  if (s->ne_flux == 0) return;
  timed_launch(s, 1, st, [&] {
    if (s->prec == FDU_F64)
      edge_flux_launch<T, double>(s, w, s->geo.p, r, st);
    else
      edge_flux_launch<T, float>(s, w, s->geo32.p, r, st);
  });
  launch_check();
}

template <class T, class TW, int LPV, int MV, int ME>
void vertex_pipe_launch(fdu_solver* s, const T* w, const TW* wfg, const TW* we, int mode, T* R, const T* wn, T* out,
                        double a, double b, const double* dt, hipStream_t st) {
  const unsigned nb = nblocks(s->nv_real * LPV);
  hipLaunchKernelGGL((k_vertex_pipe<T, TW, LPV, MV, ME>), dim3(nb), dim3(256), 0, st, w, s->vptr.p, s->vcol.p, wfg,
                     s->eptr.p, s->ecol.p, we, s->cO.p, s->flux.p, (int)s->nv_real, s->params.gamma - 1.0, mode, R,
                     wn, out, a, b, dt);
}

template <class T, class TW, int LPV, int MV, int ME, int PF, int WPE>
void vertex_lds_launch(fdu_solver* s, const T* w, const TW* wfg, const TW* we, int mode, T* R, const T* wn, T* out,
                       double a, double b, const double* dt, hipStream_t st) {
  if (s->n_vblocks == 0) return;
  const size_t lds = (size_t)s->vb_rows_max * 4 * sizeof(double);
  hipLaunchKernelGGL((k_vertex_lds<T, TW, LPV, MV, ME, PF, WPE>), dim3(s->n_vblocks), dim3(256), lds, st, w, s->vblk.p,
                     s->vb_uvp.p, s->vb_uv.p, s->vb_uep.p, s->vb_ue.p, s->vptr.p, s->vb_lvcol.p, wfg, s->eptr.p,
                     s->vb_lecol.p, we, s->cO.p, s->flux.p, s->params.gamma - 1.0, mode, R, wn, out, a, b, dt);
}

template <class T, class TW, int LPV, int MV, int ME, int PF, int WPE, bool PK>
void vertex_blk_launch(fdu_solver* s, const T* w, const TW* wfg, const TW* we, int mode, T* R, const T* wn, T* out,
                       double a, double b, const double* dt, hipStream_t st) {
  if (s->n_vblocks == 0) return;
  // the kernel stages at most ceil(kBlockRows / 256) = 4 rows per thread and one pointer pair per thread (+1)
  if (s->vb_rows_max > kBlockRows || kBlockVertices > 256)
    throw Error(FDU_ERR_UNSUPPORTED, "vertex blocks exceed the staging capacity of vertex variants 4-5");
  if (PK && s->vb_pk.n != (size_t)s->nv_real * kPackLPV)
    throw Error(FDU_ERR_STATE, "packed vertex-block ids were not built");
  const size_t lds = (size_t)s->vb_rows_max * 4 * sizeof(double) + 2 * (kBlockVertices + 1) * sizeof(int);
  hipLaunchKernelGGL((k_vertex_blk<T, TW, LPV, MV, ME, PF, WPE, PK>), dim3(s->n_vblocks), dim3(256), lds, st, w,
                     s->vblk.p, s->vb_own.p, s->vb_uvp.p, s->vb_uv.p, s->vb_uep.p, s->vb_ue.p, s->vptr.p,
                     s->vb_lvcol.p, wfg, s->eptr.p, s->vb_lecol.p, we, s->cO.p, s->flux.p, s->params.gamma - 1.0, mode,
                     R, wn, out, a, b, dt, s->vb_pk.p);
}

template <class T, class TW, int LPV, bool NT>
void vertex_loop_launch(fdu_solver* s, const T* w, const TW* wfg, const TW* we, int mode, T* R, const T* wn, T* out,
                        double a, double b, const double* dt, hipStream_t st) {
  const unsigned nb = nblocks(s->nv_real * LPV);
  hipLaunchKernelGGL((k_vertex<T, TW, LPV, NT>), dim3(nb), dim3(256), 0, st, w, s->vptr.p, s->vcol.p, wfg, s->eptr.p,
                     s->ecol.p, we, s->cO.p, s->flux.p, (int)s->nv_real, s->params.gamma - 1.0, mode, R, wn, out, a, b,
                     dt);
}

template <class T, class TW>
void vertex_launch(fdu_solver* s, const T* w, const TW* wfg, const TW* we, int mode, T* R, const T* wn, T* out,
                   double a, double b, const double* dt, hipStream_t st) {
  switch (s->vertex_variant) {
    case 1: vertex_loop_launch<T, TW, 8, false>(s, w, wfg, we, mode, R, wn, out, a, b, dt, st); break;
    case 2: vertex_pipe_launch<T, TW, 8, 3, 6>(s, w, wfg, we, mode, R, wn, out, a, b, dt, st); break;
    case 3: vertex_lds_launch<T, TW, 8, 3, 6, 1, 5>(s, w, wfg, we, mode, R, wn, out, a, b, dt, st); break;
    case 4: vertex_blk_launch<T, TW, 8, 3, 6, 1, 5, true>(s, w, wfg, we, mode, R, wn, out, a, b, dt, st); break;
    case 5: vertex_blk_launch<T, TW, 8, 3, 6, 2, 4, true>(s, w, wfg, we, mode, R, wn, out, a, b, dt, st); break;
    default: vertex_loop_launch<T, TW, 16, false>(s, w, wfg, we, mode, R, wn, out, a, b, dt, st);
  }
}

template <class T>
void vertex_t(fdu_solver* s, const T* w, int mode, T* R, const T* wn, T* out, double a, double b, const double* dt,
              hipStream_t st) {
  timed_launch(s, 2, st, [&] {
    if (s->prec == FDU_F64)
      vertex_launch<T, double>(s, w, s->wfg.p, s->we.p, mode, R, wn, out, a, b, dt, st);
    else
      vertex_launch<T, float>(s, w, s->wfg32.p, s->we32.p, mode, R, wn, out, a, b, dt, st);
  });
  launch_check();
}

template <class T>
void cfl_t(fdu_solver* s, const T* w, double cfl, double* dt, hipStream_t st) {
  timed_launch(s, 3, st, [&] {
    hipLaunchKernelGGL(k_cfl_partial<T>, dim3(s->cfl_blocks), dim3(256), 0, st, w, s->hmin.p, (int)s->nv_real,
                       s->params.gamma, s->part.p);
    launch_check();
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(256), 0, st, s->part.p, s->cfl_blocks, cfl, dt);
  });
  launch_check();
}

// The state the residual reads: w itself when the mesh has no ghosts, else the
// solver's copy of w's real rows with the ghost rows filled (w is not written).
template <class T>
const T* ghosted_state(fdu_solver* s, const T* w, hipStream_t st) {
  if (s->ng == 0) return w;
  T* c = reinterpret_cast<T*>(s->wcopy.p);
  FDU_HIP(hipMemcpyAsync(c, w, 4 * sizeof(T) * (size_t)s->nv_real, hipMemcpyDeviceToDevice, st));
  fill_ghosts_t<T>(s, c, st);
  return c;
}

template <class T>
void residual_t(fdu_solver* s, const T* w, T* R, hipStream_t st) {
  const T* wg = ghosted_state<T>(s, w, st);
  edge_flux_t<T>(s, wg, s->flux.p, st);
  vertex_t<T>(s, wg, 0, R, nullptr, nullptr, 0.0, 0.0, nullptr, st);
}

const double kRK[3][2] = {{0.0, 1.0}, {0.75, 0.25}, {1.0 / 3.0, 2.0 / 3.0}};

template <class T>
void rk_stage_t(fdu_solver* s, int k, const T* wn, T* wprev, T* wout, const double* dt, hipStream_t st) {
  fill_ghosts_t<T>(s, wprev, st);
  edge_flux_t<T>(s, wprev, s->flux.p, st);
  vertex_t<T>(s, wprev, 1, nullptr, wn, wout, kRK[k][0], kRK[k][1], dt, st);
}

template <class T>
void rk_step_t(fdu_solver* s, T* w, T* scratch, double cfl, double* dt, hipStream_t st) {
  T* w1 = scratch;
  T* w2 = scratch + 4 * s->nv_total;
  if (cfl > 0) cfl_t<T>(s, w, cfl, dt, st);
  rk_stage_t<T>(s, 0, w, w, w1, dt, st);
  rk_stage_t<T>(s, 1, w, w1, w2, dt, st);
  rk_stage_t<T>(s, 2, w, w2, w, dt, st);
}

// Vertex blocks for the LDS-staged vertex kernels: consecutive real vertices
// are grouped greedily (at most kBlockVertices per block) while the union of
// the state rows and flux rows their stencils read stays within kBlockRows
// rows (32 bytes each in LDS); each block stores its sorted row lists (the state
// rows always include the block's own vertices, a consecutive run starting at
// position own[block]) and every stencil entry the 16-bit position of its row
// in its block's list.

void build_vertex_blocks(fdu_solver* s) {
  const int64_t n = s->nv_real;
  std::vector<int32_t> blk{0}, own, uvp{0}, uep{0}, uv, ue;
  std::vector<uint16_t> lvcol(s->nnz_v), lecol(s->nnz_e);
  std::vector<int32_t> mark_v(s->nv_total, -1), mark_e(s->ne_flux, -1), pos_v(s->nv_total), pos_e(s->ne_flux);
  std::vector<int32_t> cur_v, cur_e;
  int rows_max = 0;
  auto close = [&](int64_t vend) {
    const int64_t vbeg = blk.back();
    std::sort(cur_v.begin(), cur_v.end());
    std::sort(cur_e.begin(), cur_e.end());
    for (size_t i = 0; i < cur_v.size(); ++i) pos_v[cur_v[i]] = (int32_t)i;
    for (size_t i = 0; i < cur_e.size(); ++i) pos_e[cur_e[i]] = (int32_t)i;
    own.push_back(pos_v[vbeg]);   // the block's own rows: consecutive ids, so consecutive in the sorted list
    for (int64_t v = vbeg; v < vend; ++v) {
      for (int32_t p = s->h_vptr[v]; p < s->h_vptr[v + 1]; ++p) lvcol[p] = (uint16_t)pos_v[s->h_vcol[p]];
      for (int32_t p = s->h_eptr[v]; p < s->h_eptr[v + 1]; ++p) lecol[p] = (uint16_t)pos_e[s->h_ecol[p]];
    }
    uv.insert(uv.end(), cur_v.begin(), cur_v.end());
    ue.insert(ue.end(), cur_e.begin(), cur_e.end());
    rows_max = std::max(rows_max, (int)(cur_v.size() + cur_e.size()));
    blk.push_back((int32_t)vend);
    uvp.push_back((int32_t)uv.size());
    uep.push_back((int32_t)ue.size());
    cur_v.clear();
    cur_e.clear();
  };
  int32_t id = 0;   // block being filled (marks rows already in it)
  for (int64_t v = 0; v < n; ++v) {
    int add = mark_v[v] != id;
    for (int32_t p = s->h_vptr[v]; p < s->h_vptr[v + 1]; ++p) add += mark_v[s->h_vcol[p]] != id;
    for (int32_t p = s->h_eptr[v]; p < s->h_eptr[v + 1]; ++p) add += mark_e[s->h_ecol[p]] != id;
    const int64_t nvb = v - blk.back();
    if (nvb > 0 && (nvb >= kBlockVertices || (int64_t)(cur_v.size() + cur_e.size()) + add > kBlockRows)) {
      close(v);
      ++id;
    }
    if (mark_v[v] != id) { mark_v[v] = id; cur_v.push_back((int32_t)v); }
    for (int32_t p = s->h_vptr[v]; p < s->h_vptr[v + 1]; ++p) {
      const int32_t j = s->h_vcol[p];
      if (mark_v[j] != id) { mark_v[j] = id; cur_v.push_back(j); }
    }
    for (int32_t p = s->h_eptr[v]; p < s->h_eptr[v + 1]; ++p) {
      const int32_t k = s->h_ecol[p];
      if (mark_e[k] != id) { mark_e[k] = id; cur_e.push_back(k); }
    }
    if ((int64_t)(cur_v.size() + cur_e.size()) > 65535)
      throw Error(FDU_ERR_UNSUPPORTED, "a single vertex stencil exceeds the LDS block capacity");
  }
  if (n > blk.back()) close(n);
  s->vblk.upload(blk.data(), blk.size());
  s->vb_own.upload(own.data(), own.size());
  s->vb_uvp.upload(uvp.data(), uvp.size());
  s->vb_uv.upload(uv.data(), uv.size());
  s->vb_uep.upload(uep.data(), uep.size());
  s->vb_ue.upload(ue.data(), ue.size());
  s->vb_lvcol.upload(lvcol.data(), lvcol.size());
  s->vb_lecol.upload(lecol.data(), lecol.size());
  s->n_vblocks = (int)blk.size() - 1;
  s->vb_rows_max = rows_max;
  // packed first-round ids (10 bits each; built when every block fits the block kernel)
  if (rows_max <= kBlockRows) {
    std::vector<PackedIds> pk((size_t)n * kPackLPV);
    for (int64_t v = 0; v < n; ++v) {
      for (int l = 0; l < kPackLPV; ++l) {
        PackedIds& k = pk[(size_t)v * kPackLPV + l];
        k.w[0] = k.w[1] = k.w[2] = 0u;
        for (int j = 0; j < kPackMV + kPackME; ++j) {
          const bool vs = j < kPackMV;
          const int64_t p = (vs ? s->h_vptr[v] : s->h_eptr[v]) + l + (int64_t)kPackLPV * (vs ? j : j - kPackMV);
          const int64_t pe = vs ? s->h_vptr[v + 1] : s->h_eptr[v + 1];
          const unsigned id = p < pe ? (unsigned)(vs ? lvcol[p] : lecol[p]) : 0u;
          k.w[j / 3] |= id << (10 * (j % 3));
        }
      }
    }
    s->vb_pk.upload(pk.data(), pk.size());
  } else {
    s->vb_pk.release();
  }
}

// Transposed maps for the adjoint, built on the host from the uploaded
// stencils; entries of each list are in increasing order of their source index.
void build_adjoint(fdu_solver* s) {
  const int64_t nv = s->nv_total, nr = s->nv_real, ne = s->ne_flux, ng = s->ng;
  // CSR of the positions p grouped by keys[p] (negative keys are left out)
  auto csr = [](int64_t n, const std::vector<int32_t>& keys, std::vector<int32_t>& ptr, std::vector<int32_t>& ord) {
    ptr.assign(n + 1, 0);
    for (int32_t k : keys)
      if (k >= 0) ptr[k + 1]++;
    for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    ord.assign(ptr[n], 0);
    for (size_t p = 0; p < keys.size(); ++p)
      if (keys[p] >= 0) ord[fill[keys[p]]++] = (int32_t)p;
  };
  std::vector<int32_t> ptr, ord, rowof;
  // edge -> (vertex O, we_Ok)
  rowof.resize(s->h_ecol.size());
  for (int64_t v = 0; v < nr; ++v)
    for (int32_t p = s->h_eptr[v]; p < s->h_eptr[v + 1]; ++p) rowof[p] = (int32_t)v;
  csr(ne, s->h_ecol, ptr, ord);
  std::vector<int32_t> row(ord.size());
  std::vector<double> wv(ord.size());
  for (size_t i = 0; i < ord.size(); ++i) { row[i] = rowof[ord[i]]; wv[i] = s->h_we[ord[i]]; }
  s->te_ptr.upload(ptr.data(), ptr.size());
  s->te_row.upload(row.data(), row.size());
  // vertex j -> (vertex O, wf_Oj, wg_Oj)
  rowof.resize(s->h_vcol.size());
  for (int64_t v = 0; v < nr; ++v)
    for (int32_t p = s->h_vptr[v]; p < s->h_vptr[v + 1]; ++p) rowof[p] = (int32_t)v;
  csr(nv, s->h_vcol, ptr, ord);
  std::vector<int32_t> vrow(ord.size());
  std::vector<double> vw(2 * ord.size());
  for (size_t i = 0; i < ord.size(); ++i) {
    vrow[i] = rowof[ord[i]];
    vw[2 * i] = s->h_wfg[2 * (size_t)ord[i]];
    vw[2 * i + 1] = s->h_wfg[2 * (size_t)ord[i] + 1];
  }
  s->tv_ptr.upload(ptr.data(), ptr.size());
  s->tv_row.upload(vrow.data(), vrow.size());
  if (s->prec == FDU_F64) {
    s->te_w.upload(wv.data(), wv.size());
    s->tv_wfg.upload(vw.data(), vw.size());
  } else {
    std::vector<float> a(wv.begin(), wv.end()), b(vw.begin(), vw.end());
    s->te_w32.upload(a.data(), a.size());
    s->tv_wfg32.upload(b.data(), b.size());
  }
  // sf_O = sum_j wf_Oj + cx_O, sg_O likewise
  std::vector<double> sf(2 * nr, 0.0);
  for (int64_t v = 0; v < nr; ++v) {
    double a = s->h_cO[2 * v], b = s->h_cO[2 * v + 1];
    for (int32_t p = s->h_vptr[v]; p < s->h_vptr[v + 1]; ++p) {
      a += s->h_wfg[2 * (size_t)p];
      b += s->h_wfg[2 * (size_t)p + 1];
    }
    sf[2 * v] = a;
    sf[2 * v + 1] = b;
  }
  s->sfg.upload(sf.data(), sf.size());
  // vertex -> edge slots (e * 6 + position) that read it
  csr(nv, s->h_sten, ptr, ord);
  s->ts_ptr.upload(ptr.data(), ptr.size());
  s->ts_col.upload(ord.data(), ord.size());
  // real vertex -> ghosts copied from it (Dirichlet ghosts hold given states:
  // no dependence on the solution, so they are left out)
  std::vector<int32_t> gkey(s->h_gsrc);
  for (size_t g = 0; g < gkey.size(); ++g)
    if (s->h_grefl[g] & 4) gkey[g] = -1;
  csr(nr, gkey, ptr, ord);
  s->tg_ptr.upload(ptr.data(), ptr.size());
  if (ord.empty()) ord.push_back(0);
  s->tg_col.upload(ord.data(), ord.size());
  if (ng == 0 && s->grefl.n == 0) {
    int8_t z = 0;
    s->grefl.upload(&z, 1);
  }
  s->rbar.alloc(4 * ne);
  s->slots.alloc(24 * ne);
  s->vtmp.alloc(4 * nv);
  s->dt_adj.alloc(1);
  s->adjoint = true;
}

void ready_adjoint(const fdu_solver* s) {
  ready(s);
  if (!s->adjoint) throw Error(FDU_ERR_STATE, "adjoint not enabled (fdu_enable_adjoint)");
}

// out = alpha (dR/dw)^T Rbar + beta add (real rows of add; add may be null);
// ghost rows of out are zero.  w's ghost rows must be filled.
template <class T>
void residual_vjp_t(fdu_solver* s, const T* w, const T* Rbar, T* out, double alpha, const T* add, double beta,
                    hipStream_t st) {
  const Scheme S = scheme_of(s);
  const int ne = (int)s->ne_flux, nv = (int)s->nv_total, nr = (int)s->nv_real;
  constexpr int kLanes = 8;   // lanes per edge / vertex in the transposed gathers
  if (s->prec == FDU_F64) {
    hipLaunchKernelGGL((k_edge_cot<T, double, kLanes>), dim3(nblocks((int64_t)ne * kLanes)), dim3(256), 0, st,
                       s->te_ptr.p, s->te_row.p, s->te_w.p, Rbar, s->rbar.p, ne);
    hipLaunchKernelGGL((k_edge_vjp<T, double>), dim3(nblocks(ne)), dim3(256), 0, st, w, s->sten.p, s->geo.p,
                       s->rbar.p, s->slots.p, ne, S);
    hipLaunchKernelGGL((k_vertex_vjp<T, double, kLanes>), dim3(nblocks((int64_t)nv * kLanes)), dim3(256), 0, st, w,
                       Rbar, s->tv_ptr.p, s->tv_row.p, s->tv_wfg.p, s->sfg.p, s->ts_ptr.p, s->ts_col.p, s->slots.p,
                       nr, nv, S.gm1, s->vtmp.p);
  } else {
    hipLaunchKernelGGL((k_edge_cot<T, float, kLanes>), dim3(nblocks((int64_t)ne * kLanes)), dim3(256), 0, st,
                       s->te_ptr.p, s->te_row.p, s->te_w32.p, Rbar, s->rbar.p, ne);
    hipLaunchKernelGGL((k_edge_vjp<T, float>), dim3(nblocks(ne)), dim3(256), 0, st, w, s->sten.p, s->geo32.p,
                       s->rbar.p, s->slots.p, ne, S);
    hipLaunchKernelGGL((k_vertex_vjp<T, float, kLanes>), dim3(nblocks((int64_t)nv * kLanes)), dim3(256), 0, st, w,
                       Rbar, s->tv_ptr.p, s->tv_row.p, s->tv_wfg32.p, s->sfg.p, s->ts_ptr.p, s->ts_col.p, s->slots.p,
                       nr, nv, S.gm1, s->vtmp.p);
  }
  launch_check();
  hipLaunchKernelGGL(k_ghost_vjp<T>, dim3(nblocks(nv)), dim3(256), 0, st, s->vtmp.p, s->tg_ptr.p, s->tg_col.p,
                     reinterpret_cast<const signed char*>(s->grefl.p), nr, nv, alpha, add, beta, out);
  launch_check();
}

// Adjoint of stage k: given obar (cotangent of the stage output's real rows),
// wbar_prev := b_k obar + b_k dt (dR/dw_prev)^T obar and wbar_n += a_k obar.
template <class T>
void rk_stage_vjp_t(fdu_solver* s, int k, T* wprev, const T* obar, T* wbar_n, T* wbar_prev, double dt,
                    hipStream_t st) {
  const double a = kRK[k][0], b = kRK[k][1];
  fill_ghosts_t<T>(s, wprev, st);
  residual_vjp_t<T>(s, wprev, obar, wbar_prev, b * dt, obar, b, st);
  if (a != 0.0) {
    hipLaunchKernelGGL(k_axpy_real<T>, dim3(nblocks(s->nv_real)), dim3(256), 0, st, wbar_n, a, obar,
                       (int)s->nv_real);
    launch_check();
  }
}

// The stages of one SSP-RK3 step run backwards, given the step's stage
// states w_n, w1, w2 (ghost rows filled here); g2, g1: two work states.
template <class T>
void rk_step_vjp_rev_t(fdu_solver* s, T* wn, T* w1, T* w2, const T* wbar_np1, T* wbar_n, T* g2, T* g1, double dt,
                       hipStream_t st) {
  // wbar_n := 0 on every row; the 1/3 wbar_np1 term of the last stage is
  // added by that stage's adjoint (its a_2 axpy)
  hipLaunchKernelGGL(k_scale<T>, dim3(nblocks(s->nv_total)), dim3(256), 0, st, wbar_n, 0.0, wbar_np1,
                     (int)s->nv_total);
  launch_check();
  rk_stage_vjp_t<T>(s, 2, w2, wbar_np1, wbar_n, g2, dt, st);
  rk_stage_vjp_t<T>(s, 1, w1, g2, wbar_n, g1, dt, st);
  rk_stage_vjp_t<T>(s, 0, wn, g1, wbar_n, g2, dt, st);
  hipLaunchKernelGGL(k_axpy_real<T>, dim3(nblocks(s->nv_real)), dim3(256), 0, st, wbar_n, 1.0, g2, (int)s->nv_real);
  launch_check();
}

// Adjoint of one SSP-RK3 step at a fixed dt: recompute the stage states from
// w_n with the same dt (written to the device once, so the recomputed forward
// stages and the reverse sweep cannot use different values), then run the
// stages backwards.  scratch holds 4 states.
template <class T>
void rk_step_vjp_t(fdu_solver* s, T* wn, const T* wbar_np1, T* wbar_n, T* scratch, double dt, hipStream_t st) {
  const size_t S4 = 4 * (size_t)s->nv_total;
  T* w1 = scratch;
  T* w2 = scratch + S4;
  hipLaunchKernelGGL(k_set_value, dim3(1), dim3(64), 0, st, s->dt_adj.p, dt);
  launch_check();
  rk_stage_t<T>(s, 0, wn, wn, w1, s->dt_adj.p, st);
  rk_stage_t<T>(s, 1, wn, w1, w2, s->dt_adj.p, st);
  rk_step_vjp_rev_t<T>(s, wn, w1, w2, wbar_np1, wbar_n, scratch + 2 * S4, scratch + 3 * S4, dt, st);
}

}  // namespace

struct fdu_batch {
  int device = 0;
  int n = 0;
  std::vector<fdu_solver*> inst;
  Scheme S{};
  int schedule = 0;     // 0 fused persistent, 1 one launch per phase, 2 per-instance kernels
  BatchTiling tl{4, 8};
  int vmode = 0;        // vertex tiles: 0 loop/16 lanes, 1 loop/8 lanes, 2 pipelined/8 lanes, 3 LDS blocks
  int lds_rows = 0;     // vertex mode 3: largest vertex-block row list over the instances
  int grid = 0;         // blocks of the fused launch
  int total = 0, ctiles = 0;
  std::vector<int32_t> h_tb;
  DevBuf<BatchInst> dinst;
  DevBuf<int32_t> tb, tbc, err;
  DevBuf<uint32_t> ctr;
  DevBuf<unsigned long long> dtbits;
  DevBuf<double> dt;
  std::vector<BatchInst> h_inst;
  bool have_states = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~fdu_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

// Dynamic LDS of the vertex-block tiles (vertex mode 3): the largest block's
// staged rows plus its CSR pointer table.
size_t batch_lds_bytes(const fdu_batch* b) {
  return b->vmode == 3 ? (size_t)b->lds_rows * 4 * sizeof(double) + 2 * (kBlockVertices + 1) * sizeof(int) : 0;
}

// The fused kernel's dynamic LDS: the vertex-block rows (mode 3), then the
// tile table (3 n + 1 ints, 4-byte aligned after the rows).
size_t fused_lds_bytes(const fdu_batch* b) { return batch_lds_bytes(b) + (size_t)(3 * b->n + 1) * sizeof(int); }

void batch_tiles(fdu_batch* b) {
  const int n = b->n;
  const int per_v = b->tl.vp * (256 / (b->vmode == 0 ? 16 : 8));
  b->h_tb.assign(3 * n + 1, 0);
  int acc = 0;
  for (int p = 0; p < 3; ++p)
    for (int i = 0; i < n; ++i) {
      const fdu_solver* s = b->inst[i];
      b->h_tb[p * n + i] = acc;
      const int nt = p == 0 ? (int)((s->ng + 255) / 256)
                   : p == 1 ? (int)((s->ne_flux + 256 * b->tl.ept - 1) / (256 * b->tl.ept))
                   : b->vmode == 3 ? s->n_vblocks
                            : (int)((s->nv_real + per_v - 1) / per_v);
      acc += nt;
    }
  b->h_tb[3 * n] = acc;
  b->total = acc;
  b->lds_rows = 0;
  for (int i = 0; i < n; ++i) b->lds_rows = std::max(b->lds_rows, b->inst[i]->vb_rows_max);
  b->tb.upload(b->h_tb.data(), b->h_tb.size());
  std::vector<int32_t> tbc(n + 1, 0);
  for (int i = 0; i < n; ++i) tbc[i + 1] = tbc[i] + (int)((b->inst[i]->nv_real + 255) / 256);
  b->ctiles = tbc[n];
  b->tbc.upload(tbc.data(), tbc.size());
  int cus = 0, per_cu = 0;
  FDU_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
  if (b->vmode == 3)
    FDU_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_stage<1, 3, -1>, 256, fused_lds_bytes(b)));
  else
    FDU_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_stage<1, 2, -1>, 256, fused_lds_bytes(b)));
  b->grid = std::max(1, std::min(b->total, cus * std::max(1, per_cu)));
}

template <int EV, int VM, int PH>
void batch_stage_launch(fdu_batch* b, int k, hipStream_t st, unsigned grid) {
  const size_t lds = PH < 0 ? fused_lds_bytes(b) : 0;
  hipLaunchKernelGGL((k_batch_stage<EV, VM, PH>), dim3(grid), dim3(256), lds, st, b->dinst.p, b->n, b->tb.p, b->total,
                     b->ctr.p, b->S, k, kRK[k][0], kRK[k][1], b->dt.p, b->err.p, b->tl,
                     (int)(batch_lds_bytes(b) / sizeof(int)));
}

template <int EV, int VM>
void batch_stage_vm(fdu_batch* b, int k, hipStream_t st) {
  if (b->schedule == 0) {
    hipLaunchKernelGGL(k_batch_reset, dim3(nblocks(1 + 2 * b->n)), dim3(256), 0, st, b->ctr.p, 1 + 2 * b->n,
                       (unsigned long long*)nullptr, 0);
    batch_stage_launch<EV, VM, -1>(b, k, st, (unsigned)b->grid);
    return;
  }
  const int n = b->n;
  const int t0 = b->h_tb[n] - b->h_tb[0], t1 = b->h_tb[2 * n] - b->h_tb[n], t2 = b->h_tb[3 * n] - b->h_tb[2 * n];
  if (t0 > 0) batch_stage_launch<EV, VM, 0>(b, k, st, (unsigned)t0);
  if (t1 > 0) batch_stage_launch<EV, VM, 1>(b, k, st, (unsigned)t1);
  if (t2 > 0) {
    if (VM == 3)
      hipLaunchKernelGGL((k_batch_vertex_lds<8, 3, 6, 1, 5, true>), dim3(t2), dim3(256),
                         (size_t)b->lds_rows * 4 * sizeof(double) + 2 * (kBlockVertices + 1) * sizeof(int), st,
                         b->dinst.p, n, b->tb.p, b->S, k, kRK[k][0],
                         kRK[k][1], b->dt.p);
    else
      batch_stage_launch<EV, VM, 2>(b, k, st, (unsigned)t2);
  }
}

void batch_stage(fdu_batch* b, int k, hipStream_t st) {
  const int ev = b->inst[0]->edge_variant >= 1 ? 1 : 0;
  if (ev == 1) {
    if (b->vmode == 3) batch_stage_vm<1, 3>(b, k, st);
    else if (b->vmode == 2) batch_stage_vm<1, 2>(b, k, st);
    else if (b->vmode == 1) batch_stage_vm<1, 1>(b, k, st);
    else batch_stage_vm<1, 0>(b, k, st);
  } else {
    if (b->vmode == 3) batch_stage_vm<0, 3>(b, k, st);
    else if (b->vmode == 2) batch_stage_vm<0, 2>(b, k, st);
    else if (b->vmode == 1) batch_stage_vm<0, 1>(b, k, st);
    else batch_stage_vm<0, 0>(b, k, st);
  }
  launch_check();
}

void batch_cfl(fdu_batch* b, double cfl, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3(nblocks(b->n)), dim3(256), 0, st, b->ctr.p, 0, b->dtbits.p, b->n);
  hipLaunchKernelGGL(k_batch_cfl, dim3(std::min(b->ctiles, 4096)), dim3(256), 0, st, b->dinst.p, b->n, b->tbc.p,
                     b->ctiles, b->S.gamma, b->dtbits.p);
  hipLaunchKernelGGL(k_batch_dt, dim3(nblocks(b->n)), dim3(256), 0, st, b->dtbits.p, b->n, cfl, b->dt.p);
  launch_check();
}

void batch_step(fdu_batch* b, double cfl, hipStream_t st) {
  if (!b->have_states) throw Error(FDU_ERR_STATE, "set the instance states first (fdu_batch_set_states)");
  batch_cfl(b, cfl, st);
  if (b->schedule == 2) {
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < b->n; ++i) {
        fdu_solver* s = b->inst[i];
        const BatchInst& I = b->h_inst[i];
        double* wprev = k == 0 ? I.w : (k == 1 ? I.w1 : I.w2);
        double* wout = k == 0 ? I.w1 : (k == 1 ? I.w2 : I.w);
        rk_stage_t<double>(s, k, I.w, wprev, wout, b->dt.p + i, st);
      }
    return;
  }
  for (int k = 0; k < 3; ++k) batch_stage(b, k, st);
}

}  // namespace

extern "C" {

const char* fdu_last_error(void) { return g_last_error.c_str(); }

void fdu_default_params(fdu_params* p) {
  if (!p) return;
  p->gamma = 1.4;
  p->weno_eps = 1e-40;
  p->entropy_frac = 0.1;
  p->weno_power = 1;
  p->riemann = 0;
  p->positivity = 1;
  p->interpolation = 0;
  p->uniform_weno = 0;
}

fdu_status fdu_create(fdu_solver** out, int hip_device, fdu_precision prec, const fdu_params* params) {
  return guard([&] {
    need(out != nullptr, "NULL output pointer");
    *out = nullptr;
    need(prec == FDU_F64 || prec == FDU_F32, "unknown precision");
    int n = 0;
    FDU_HIP(hipGetDeviceCount(&n));
    need(hip_device >= 0 && hip_device < n, "no such HIP device");
    auto s = new fdu_solver();
    s->device = hip_device;
    s->prec = prec;
    if (params)
      s->params = *params;
    else
      fdu_default_params(&s->params);
    if (!(s->params.gamma > 1.0) || !(s->params.weno_eps > 0) || (s->params.weno_power != 1 && s->params.weno_power != 2) ||
        (s->params.riemann != 0 && s->params.riemann != 1) || !(s->params.entropy_frac >= 0) ||
        (s->params.positivity != 0 && s->params.positivity != 1) ||
        (s->params.interpolation != 0 && s->params.interpolation != 1) ||
        (s->params.uniform_weno != 0 && s->params.uniform_weno != 1)) {
      delete s;
      throw Error(FDU_ERR_INVALID_ARG, "invalid scheme parameters");
    }
    try {
      DeviceGuard dg(hip_device);
      static_scratch_init(hip_device);
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

void fdu_destroy(fdu_solver* s) {
  if (!s) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  delete s;
  (void)hipSetDevice(prev);
}

fdu_status fdu_upload_edge_stencils(fdu_solver* s, int64_t nv_total, int64_t nv_real, int64_t ne_flux,
                                    const int32_t* sten6, const double* geo) {
  return guard([&] {
    need(s && sten6 && geo, "NULL argument");
    need(nv_total > 0 && nv_real > 0 && nv_real <= nv_total && nv_total < INT32_MAX / 4, "invalid vertex counts");
    need(ne_flux > 0 && ne_flux < INT32_MAX / 6, "invalid edge count");
    for (int64_t i = 0; i < 6 * ne_flux; ++i)
      need(sten6[i] >= 0 && sten6[i] < nv_total, "edge stencil vertex id out of range");
    check_finite(geo, 6 * ne_flux, "edge geometry");
    DeviceGuard dg(s->device);
    s->finalized = false;
    s->nv_total = nv_total;
    s->nv_real = nv_real;
    s->ne_flux = ne_flux;
    s->ng = nv_total - nv_real;
    s->sten.upload(sten6, 6 * ne_flux);
    s->h_sten.assign(sten6, sten6 + 6 * ne_flux);
    s->h_geo.assign(geo, geo + 6 * ne_flux);
    s->adjoint = false;
    if (s->prec == FDU_F64) {
      s->geo.upload(geo, 6 * ne_flux);
    } else {
      std::vector<float> g32(geo, geo + 6 * ne_flux);
      s->geo32.upload(g32.data(), g32.size());
    }
    s->flux.alloc(4 * ne_flux);
    s->have_edges = true;
  });
}

fdu_status fdu_upload_vertex_stencils(fdu_solver* s, const int32_t* vptr, const int32_t* vcol, const double* wfg,
                                      const int32_t* eptr, const int32_t* ecol, const double* we, const double* hmin) {
  return guard([&] {
    need(s && wfg && we && hmin, "NULL argument");
    if (!s->have_edges) throw Error(FDU_ERR_STATE, "upload the edge stencils first");
    int64_t nnz_v, nnz_e;
    check_csr(vptr, s->nv_real, vcol, s->nv_total, "vertex stencil", nnz_v);
    check_csr(eptr, s->nv_real, ecol, s->ne_flux, "edge stencil", nnz_e);
    check_finite(wfg, 2 * nnz_v, "vertex weights");
    check_finite(we, nnz_e, "edge weights");
    for (int64_t i = 0; i < s->nv_real; ++i) need(hmin[i] > 0 && std::isfinite(hmin[i]), "hmin must be positive");
    DeviceGuard dg(s->device);
    s->finalized = false;
    s->nnz_v = nnz_v;
    s->nnz_e = nnz_e;
    s->vptr.upload(vptr, s->nv_real + 1);
    s->vcol.upload(vcol, nnz_v);
    s->eptr.upload(eptr, s->nv_real + 1);
    s->ecol.upload(ecol, nnz_e);
    s->hmin.upload(hmin, s->nv_real);
    if (s->prec == FDU_F64) {
      s->wfg.upload(wfg, 2 * nnz_v);
      s->we.upload(we, nnz_e);
    } else {
      std::vector<float> a(wfg, wfg + 2 * nnz_v), b(we, we + nnz_e);
      s->wfg32.upload(a.data(), a.size());
      s->we32.upload(b.data(), b.size());
    }
    s->h_eptr.assign(eptr, eptr + s->nv_real + 1);
    s->h_ecol.assign(ecol, ecol + nnz_e);
    s->h_we.assign(we, we + nnz_e);
    s->h_vptr.assign(vptr, vptr + s->nv_real + 1);
    s->h_vcol.assign(vcol, vcol + nnz_v);
    s->h_wfg.assign(wfg, wfg + 2 * nnz_v);
    if (s->prec == FDU_F32) {  // c_O and the adjoint must use the weights the kernels see
      for (auto& x : s->h_we) x = (double)(float)x;
      for (auto& x : s->h_wfg) x = (double)(float)x;
    }
    s->adjoint = false;
    s->have_vertices = true;
  });
}

fdu_status fdu_upload_ghosts(fdu_solver* s, int64_t ng, const int32_t* ghost_src, const int8_t* ghost_refl) {
  return guard([&] {
    need(s != nullptr, "NULL solver");
    if (!s->have_edges) throw Error(FDU_ERR_STATE, "upload the edge stencils first");
    need(ng == s->ng, "ghost count must equal nv_total - nv_real");
    if (ng == 0) return;
    need(ghost_src && ghost_refl, "NULL ghost arrays");
    int64_t nd = 0;
    for (int64_t i = 0; i < ng; ++i) {
      need(ghost_src[i] >= 0 && ghost_src[i] < s->nv_real, "ghost source must be a real vertex");
      const int f = ghost_refl[i];
      need((f & ~7) == 0 && !((f & 4) && (f & 3)), "ghost flags must be 0..3, or 4 (Dirichlet) alone");
      nd += (f & 4) != 0;
    }
    DeviceGuard dg(s->device);
    s->finalized = false;
    s->adjoint = false;
    s->n_dirichlet = nd;
    s->gstate.release();
    s->gsrc.upload(ghost_src, ng);
    s->grefl.upload(ghost_refl, ng);
    s->h_gsrc.assign(ghost_src, ghost_src + ng);
    s->h_grefl.assign(ghost_refl, ghost_refl + ng);
  });
}

fdu_status fdu_upload_ghost_states(fdu_solver* s, int64_t ng, const double* states) {
  return guard([&] {
    need(s != nullptr, "NULL solver");
    need(ng == s->ng && s->grefl.n == (size_t)ng, "upload the ghosts first; ng must equal their count");
    if (ng == 0) return;
    need(states != nullptr, "NULL states");
    for (int64_t g = 0; g < ng; ++g) {
      if (!(s->h_grefl[g] & 4)) continue;
      const double* q = states + 4 * g;
      for (int k = 0; k < 4; ++k) need(std::isfinite(q[k]), "non-finite Dirichlet state");
      need(q[0] > 0.0, "Dirichlet density must be positive");
    }
    DeviceGuard dg(s->device);
    if (s->gstate.n != (size_t)(4 * ng)) s->gstate.alloc(4 * ng);   // keep the address for captured graphs
    FDU_HIP(hipMemcpy(s->gstate.p, states, 4 * ng * sizeof(double), hipMemcpyHostToDevice));
  });
}

fdu_status fdu_upload_prep(fdu_solver* s, const fdu_prep* p) {
  fdu_status st;
  if (!s || !p) {
    set_last_error("NULL argument");
    return FDU_ERR_INVALID_ARG;
  }
  if ((st = fdu_upload_edge_stencils(s, p->nv_total, p->nv_real, p->ne_flux, p->sten6.data(), p->geo.data())) != FDU_OK)
    return st;
  if ((st = fdu_upload_vertex_stencils(s, p->vptr.data(), p->vcol.data(), p->wfg.data(), p->eptr.data(),
                                       p->ecol.data(), p->we.data(), p->hmin.data())) != FDU_OK)
    return st;
  return fdu_upload_ghosts(s, p->nv_total - p->nv_real, p->ghost_src.data(), p->ghost_refl.data());
}

fdu_status fdu_finalize(fdu_solver* s) {
  return guard([&] {
    need(s != nullptr, "NULL solver");
    if (!s->have_edges || !s->have_vertices) throw Error(FDU_ERR_STATE, "upload edge and vertex stencils first");
    if (s->ng > 0 && s->gsrc.n != (size_t)s->ng) throw Error(FDU_ERR_STATE, "upload the ghosts first");
    if (s->n_dirichlet > 0 && s->gstate.n != (size_t)(4 * s->ng))
      throw Error(FDU_ERR_STATE, "upload the Dirichlet ghost states first (fdu_upload_ghost_states)");
    DeviceGuard dg(s->device);
    std::vector<double> c(2 * s->nv_real, 0.0);
    for (int64_t v = 0; v < s->nv_real; ++v)
      for (int32_t p = s->h_eptr[v]; p < s->h_eptr[v + 1]; ++p) {
        const int32_t k = s->h_ecol[p];
        double nx = s->h_geo[6 * k + 4], ny = s->h_geo[6 * k + 5];
        if (s->prec == FDU_F32) {
          nx = (double)(float)nx;
          ny = (double)(float)ny;
        }
        c[2 * v] += s->h_we[p] * nx;
        c[2 * v + 1] += s->h_we[p] * ny;
      }
    s->cO.upload(c.data(), c.size());
    s->h_cO = c;
    s->cfl_blocks = (int)std::min<int64_t>(1024, (s->nv_real + 255) / 256);
    s->part.alloc(s->cfl_blocks);
    s->chk.alloc(2);
    if (s->ng > 0) s->wcopy.alloc(4 * (size_t)s->nv_total * (s->prec == FDU_F64 ? sizeof(double) : sizeof(float)));
    build_vertex_blocks(s);
    s->finalized = true;
  });
}

fdu_status fdu_sizes(const fdu_solver* s, int64_t* nv_total, int64_t* nv_real, int64_t* ne_flux, int64_t* nnz_v,
                     int64_t* nnz_e) {
  return guard([&] {
    need(s != nullptr, "NULL solver");
    if (nv_total) *nv_total = s->nv_total;
    if (nv_real) *nv_real = s->nv_real;
    if (ne_flux) *ne_flux = s->ne_flux;
    if (nnz_v) *nnz_v = s->nnz_v;
    if (nnz_e) *nnz_e = s->nnz_e;
  });
}

fdu_status fdu_check_state(fdu_solver* s, const void* w, int64_t* n_bad, int64_t* first_bad, void* stream) {
  return guard([&] {
    ready(s);
    need(w && n_bad && first_bad, "NULL argument");
    DeviceGuard dg(s->device);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_check_reset, dim3(1), dim3(64), 0, st, s->chk.p);
    if (s->prec == FDU_F64)
      hipLaunchKernelGGL(k_check_state<double>, dim3(nblocks(s->nv_real)), dim3(256), 0, st, (const double*)w,
                         (int)s->nv_real, s->params.gamma - 1.0, s->chk.p);
    else
      hipLaunchKernelGGL(k_check_state<float>, dim3(nblocks(s->nv_real)), dim3(256), 0, st, (const float*)w,
                         (int)s->nv_real, s->params.gamma - 1.0, s->chk.p);
    launch_check();
    unsigned long long h[2];
    FDU_HIP(hipMemcpyAsync(h, s->chk.p, sizeof(h), hipMemcpyDeviceToHost, st));
    FDU_HIP(hipStreamSynchronize(st));
    *n_bad = (int64_t)h[0];
    *first_bad = h[0] ? (int64_t)h[1] : -1;
  });
}

fdu_status fdu_vertex_block_info(const fdu_solver* s, int* n_blocks, int64_t* halo_rows, int* rows_max) {
  return guard([&] {
    ready(s);
    if (n_blocks) *n_blocks = s->n_vblocks;
    if (halo_rows) *halo_rows = (int64_t)s->vb_uv.n + (int64_t)s->vb_ue.n;
    if (rows_max) *rows_max = s->vb_rows_max;
  });
}

fdu_status fdu_fill_ghosts(fdu_solver* s, void* w, void* stream) {
  return guard([&] {
    ready(s);
    need(w != nullptr, "NULL state");
    DeviceGuard dg(s->device);
    if (s->prec == FDU_F64)
      fill_ghosts_t<double>(s, (double*)w, (hipStream_t)stream);
    else
      fill_ghosts_t<float>(s, (float*)w, (hipStream_t)stream);
  });
}

fdu_status fdu_edge_fluxes(fdu_solver* s, const void* w, double* r, void* stream) {
  return guard([&] {
    ready(s);
    need(w && r, "NULL argument");
    DeviceGuard dg(s->device);
    if (s->prec == FDU_F64)
      edge_flux_t<double>(s, (const double*)w, r, (hipStream_t)stream);
    else
      edge_flux_t<float>(s, (const float*)w, r, (hipStream_t)stream);
  });
}

fdu_status fdu_residual(fdu_solver* s, const void* w, void* R, void* stream) {
  return guard([&] {
    ready(s);
    need(w && R, "NULL argument");
    DeviceGuard dg(s->device);
    if (s->prec == FDU_F64)
      residual_t<double>(s, (const double*)w, (double*)R, (hipStream_t)stream);
    else
      residual_t<float>(s, (const float*)w, (float*)R, (hipStream_t)stream);
  });
}

fdu_status fdu_cfl_dt(fdu_solver* s, const void* w, double cfl, double* dt_dev, void* stream) {
  return guard([&] {
    ready(s);
    need(w && dt_dev, "NULL argument");
    need(cfl > 0 && std::isfinite(cfl), "cfl must be positive");
    DeviceGuard dg(s->device);
    if (s->prec == FDU_F64)
      cfl_t<double>(s, (const double*)w, cfl, dt_dev, (hipStream_t)stream);
    else
      cfl_t<float>(s, (const float*)w, cfl, dt_dev, (hipStream_t)stream);
  });
}

fdu_status fdu_rk_stage(fdu_solver* s, int k, const void* w_n, void* w_prev, void* w_out, const double* dt_dev,
                        void* stream) {
  return guard([&] {
    ready(s);
    need(k >= 0 && k <= 2, "stage must be 0, 1 or 2");
    need(w_prev && w_out && dt_dev && (k == 0 || w_n), "NULL argument");
    need(w_out != w_prev, "w_out must not alias w_prev (other vertices gather from it)");
    DeviceGuard dg(s->device);
    if (s->prec == FDU_F64)
      rk_stage_t<double>(s, k, (const double*)w_n, (double*)w_prev, (double*)w_out, dt_dev, (hipStream_t)stream);
    else
      rk_stage_t<float>(s, k, (const float*)w_n, (float*)w_prev, (float*)w_out, dt_dev, (hipStream_t)stream);
  });
}

fdu_status fdu_rk_step(fdu_solver* s, void* w, void* scratch, double cfl, double* dt_dev, void* stream) {
  return guard([&] {
    ready(s);
    need(w && scratch && dt_dev, "NULL argument");
    DeviceGuard dg(s->device);
    if (s->prec == FDU_F64)
      rk_step_t<double>(s, (double*)w, (double*)scratch, cfl, dt_dev, (hipStream_t)stream);
    else
      rk_step_t<float>(s, (float*)w, (float*)scratch, cfl, dt_dev, (hipStream_t)stream);
  });
}

fdu_status fdu_rk_step_static(fdu_solver* s, void* w, double cfl, double* dt_dev, void* stream) {
  return guard([&] {
    ready(s);
    need(w && dt_dev, "NULL argument");
    const size_t elem = s->prec == FDU_F64 ? sizeof(double) : sizeof(float);
    const size_t need_bytes = 2 * 4 * elem * (size_t)s->nv_total;
    if (need_bytes > kStaticScratchBytes)
      throw Error(FDU_ERR_INVALID_ARG, "fdu_rk_step_static: two stage states of " + std::to_string(s->nv_total) +
                                           " vertices need " + std::to_string(need_bytes) +
                                           " bytes, more than the static array's " +
                                           std::to_string(kStaticScratchBytes) + " (use fdu_rk_step)");
    void* st_buf = static_scratch(s->device);
    if (!st_buf) throw Error(FDU_ERR_STATE, "static stage states not set up on this device");
    DeviceGuard dg(s->device);
    if (s->prec == FDU_F64)
      rk_step_t<double>(s, (double*)w, (double*)st_buf, cfl, dt_dev, (hipStream_t)stream);
    else
      rk_step_t<float>(s, (float*)w, (float*)st_buf, cfl, dt_dev, (hipStream_t)stream);
  });
}

fdu_status fdu_enable_adjoint(fdu_solver* s) {
  return guard([&] {
    ready(s);
    DeviceGuard dg(s->device);
    build_adjoint(s);
  });
}

fdu_status fdu_residual_vjp(fdu_solver* s, const void* w, const void* Rbar, void* wbar, void* stream) {
  return guard([&] {
    ready_adjoint(s);
    need(w && Rbar && wbar, "NULL argument");
    need(wbar != w && wbar != Rbar, "wbar must not alias w or Rbar");
    DeviceGuard dg(s->device);
    hipStream_t st = (hipStream_t)stream;
    if (s->prec == FDU_F64)
      residual_vjp_t<double>(s, ghosted_state<double>(s, (const double*)w, st), (const double*)Rbar, (double*)wbar,
                             1.0, nullptr, 0.0, st);
    else
      residual_vjp_t<float>(s, ghosted_state<float>(s, (const float*)w, st), (const float*)Rbar, (float*)wbar, 1.0,
                            nullptr, 0.0, st);
  });
}

fdu_status fdu_rk_stage_vjp(fdu_solver* s, int k, void* w_prev, const void* obar, void* wbar_n, void* wbar_prev,
                            double dt, void* stream) {
  return guard([&] {
    ready_adjoint(s);
    need(k >= 0 && k <= 2, "stage must be 0, 1 or 2");
    need(w_prev && obar && wbar_prev && (k == 0 || wbar_n), "NULL argument");
    need(wbar_prev != obar && wbar_prev != w_prev && wbar_prev != wbar_n, "wbar_prev must not alias other arrays");
    need(std::isfinite(dt), "dt must be finite");
    DeviceGuard dg(s->device);
    if (s->prec == FDU_F64)
      rk_stage_vjp_t<double>(s, k, (double*)w_prev, (const double*)obar, (double*)wbar_n, (double*)wbar_prev, dt,
                             (hipStream_t)stream);
    else
      rk_stage_vjp_t<float>(s, k, (float*)w_prev, (const float*)obar, (float*)wbar_n, (float*)wbar_prev, dt,
                            (hipStream_t)stream);
  });
}

fdu_status fdu_rk_step_vjp(fdu_solver* s, void* w_n, const void* wbar_np1, void* wbar_n, void* scratch, double dt,
                           void* stream) {
  return guard([&] {
    ready_adjoint(s);
    need(w_n && wbar_np1 && wbar_n && scratch, "NULL argument");
    need(wbar_n != wbar_np1, "wbar_n must not alias wbar_np1");
    need(std::isfinite(dt), "dt must be finite");
    DeviceGuard dg(s->device);
    if (s->prec == FDU_F64)
      rk_step_vjp_t<double>(s, (double*)w_n, (const double*)wbar_np1, (double*)wbar_n, (double*)scratch, dt,
                            (hipStream_t)stream);
    else
      rk_step_vjp_t<float>(s, (float*)w_n, (const float*)wbar_np1, (float*)wbar_n, (float*)scratch, dt,
                           (hipStream_t)stream);
  });
}

fdu_status fdu_rk_step_vjp_stages(fdu_solver* s, void* w_n, void* w_1, void* w_2, const void* wbar_np1,
                                  void* wbar_n, void* scratch, double dt, void* stream) {
  return guard([&] {
    ready_adjoint(s);
    need(w_n && w_1 && w_2 && wbar_np1 && wbar_n && scratch, "NULL argument");
    need(wbar_n != wbar_np1, "wbar_n must not alias wbar_np1");
    need(w_n != w_1 && w_n != w_2 && w_1 != w_2, "the stage states must be distinct");
    need(wbar_n != w_n && wbar_n != w_1 && wbar_n != w_2, "wbar_n must not alias a stage state");
    need(std::isfinite(dt), "dt must be finite");
    DeviceGuard dg(s->device);
    const size_t S4 = 4 * (size_t)s->nv_total;
    if (s->prec == FDU_F64) {
      double* g = (double*)scratch;
      rk_step_vjp_rev_t<double>(s, (double*)w_n, (double*)w_1, (double*)w_2, (const double*)wbar_np1,
                                (double*)wbar_n, g, g + S4, dt, (hipStream_t)stream);
    } else {
      float* g = (float*)scratch;
      rk_step_vjp_rev_t<float>(s, (float*)w_n, (float*)w_1, (float*)w_2, (const float*)wbar_np1, (float*)wbar_n, g,
                               g + S4, dt, (hipStream_t)stream);
    }
  });
}

fdu_status fdu_set_variants(fdu_solver* s, int edge_variant, int vertex_variant) {
  return guard([&] {
    need(s != nullptr, "NULL solver");
    need(edge_variant >= 0 && edge_variant < kEdgeVariants, "edge variant out of range");
    need(vertex_variant >= 0 && vertex_variant < kVertexVariants, "vertex variant out of range");
    s->edge_variant = edge_variant;
    s->vertex_variant = vertex_variant;
  });
}

fdu_status fdu_get_variants(const fdu_solver* s, int* edge_variant, int* vertex_variant, int* n_edge, int* n_vertex) {
  return guard([&] {
    need(s != nullptr, "NULL solver");
    if (edge_variant) *edge_variant = s->edge_variant;
    if (vertex_variant) *vertex_variant = s->vertex_variant;
    if (n_edge) *n_edge = kEdgeVariants;
    if (n_vertex) *n_vertex = kVertexVariants;
  });
}

fdu_status fdu_batch_create(fdu_batch** out, fdu_solver* const* inst, int n) {
  return guard([&] {
    need(out && inst && n > 0, "invalid argument");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
      ready(inst[i]);
      need(inst[i]->prec == FDU_F64, "batched instances must be FP64");
      need(inst[i]->device == inst[0]->device, "batched instances must share a device");
      need(std::memcmp(&inst[i]->params, &inst[0]->params, sizeof(fdu_params)) == 0,
           "batched instances must share scheme parameters");
      need(inst[i]->edge_variant == inst[0]->edge_variant, "batched instances must share the edge variant");
    }
    DeviceGuard dg(inst[0]->device);
    std::unique_ptr<fdu_batch> b(new fdu_batch());
    b->device = inst[0]->device;
    b->n = n;
    b->inst.assign(inst, inst + n);
    b->S = scheme_of(inst[0]);
    b->ctr.alloc(1 + 2 * n);
    b->dtbits.alloc(n);
    b->dt.alloc(n);
    b->err.alloc(1);
    int zero = 0;
    FDU_HIP(hipMemcpy(b->err.p, &zero, sizeof(int), hipMemcpyHostToDevice));
    batch_tiles(b.get());
    *out = b.release();
  });
}

void fdu_batch_destroy(fdu_batch* b) {
  if (!b) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(b->device);
  delete b;
  (void)hipSetDevice(prev);
}

fdu_status fdu_batch_set_states(fdu_batch* b, void* const* w, void* const* scratch) {
  return guard([&] {
    need(b && w && scratch, "NULL argument");
    DeviceGuard dg(b->device);
    b->h_inst.resize(b->n);
    for (int i = 0; i < b->n; ++i) {
      need(w[i] && scratch[i], "NULL state or scratch");
      fdu_solver* s = b->inst[i];
      BatchInst& I = b->h_inst[i];
      I.sten = s->sten.p; I.geo = s->geo.p; I.vptr = s->vptr.p; I.vcol = s->vcol.p; I.wfg = s->wfg.p;
      I.eptr = s->eptr.p; I.ecol = s->ecol.p; I.we = s->we.p; I.cO = s->cO.p; I.hmin = s->hmin.p;
      I.gsrc = s->gsrc.p; I.grefl = reinterpret_cast<const signed char*>(s->grefl.p); I.flux = s->flux.p;
      I.gstate = s->gstate.p;
      I.vblk = s->vblk.p; I.vb_own = s->vb_own.p; I.vb_uvp = s->vb_uvp.p; I.vb_uv = s->vb_uv.p; I.vb_uep = s->vb_uep.p; I.vb_ue = s->vb_ue.p;
      I.vb_lvcol = s->vb_lvcol.p; I.vb_lecol = s->vb_lecol.p; I.vb_pk = s->vb_pk.p;
      I.w = (double*)w[i];
      I.w1 = (double*)scratch[i];
      I.w2 = (double*)scratch[i] + 4 * s->nv_total;
      I.nv_real = (int)s->nv_real; I.nv_total = (int)s->nv_total; I.ne = (int)s->ne_flux; I.ng = (int)s->ng;
    }
    b->dinst.upload(b->h_inst.data(), b->h_inst.size());
    b->have_states = true;
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  });
}

fdu_status fdu_batch_set_schedule(fdu_batch* b, int schedule, int edges_per_thread, int vertex_passes,
                                  int vertex_mode) {
  return guard([&] {
    need(b != nullptr, "NULL batch");
    need(schedule >= 0 && schedule <= 2, "schedule must be 0, 1 or 2");
    need(edges_per_thread >= 1 && edges_per_thread <= 64, "edges_per_thread out of range");
    need(vertex_passes >= 1 && vertex_passes <= 64, "vertex_passes out of range");
    need(vertex_mode >= 0 && vertex_mode <= 3, "vertex_mode must be 0, 1, 2 or 3");
    if (vertex_mode == 3)
      for (int i = 0; i < b->n; ++i)
        if (b->inst[i]->vb_rows_max > kBlockRows ||
            b->inst[i]->vb_pk.n != (size_t)b->inst[i]->nv_real * kPackLPV)
          throw Error(FDU_ERR_UNSUPPORTED, "vertex blocks exceed the staging capacity of vertex mode 3");
    DeviceGuard dg(b->device);
    b->schedule = schedule;
    b->tl.ept = edges_per_thread;
    b->tl.vp = vertex_passes;
    b->vmode = vertex_mode;
    batch_tiles(b);
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  });
}

fdu_status fdu_batch_step(fdu_batch* b, double cfl, void* stream) {
  return guard([&] {
    need(b != nullptr, "NULL batch");
    need(cfl > 0 && std::isfinite(cfl), "cfl must be positive");
    DeviceGuard dg(b->device);
    batch_step(b, cfl, (hipStream_t)stream);
  });
}

fdu_status fdu_batch_capture(fdu_batch* b, double cfl, int nsteps, void* stream) {
  return guard([&] {
    need(b != nullptr && stream != nullptr, "a non-default stream is required for capture");
    need(nsteps > 0 && cfl > 0 && std::isfinite(cfl), "invalid steps or cfl");
    if (!b->have_states) throw Error(FDU_ERR_STATE, "set the instance states first (fdu_batch_set_states)");
    DeviceGuard dg(b->device);
    hipStream_t st = (hipStream_t)stream;
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    FDU_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      for (int i = 0; i < nsteps; ++i) batch_step(b, cfl, st);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(st, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    FDU_HIP(hipStreamEndCapture(st, &b->graph));
    FDU_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  });
}

fdu_status fdu_batch_launch(fdu_batch* b, void* stream) {
  return guard([&] {
    need(b != nullptr, "NULL batch");
    if (!b->exec) throw Error(FDU_ERR_STATE, "nothing captured (fdu_batch_capture)");
    DeviceGuard dg(b->device);
    FDU_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
  });
}

fdu_status fdu_batch_status(fdu_batch* b, int* wait_timeouts, double* dt_host) {
  return guard([&] {
    need(b != nullptr, "NULL batch");
    DeviceGuard dg(b->device);
    FDU_HIP(hipDeviceSynchronize());
    if (wait_timeouts) FDU_HIP(hipMemcpy(wait_timeouts, b->err.p, sizeof(int), hipMemcpyDeviceToHost));
    if (dt_host) FDU_HIP(hipMemcpy(dt_host, b->dt.p, b->n * sizeof(double), hipMemcpyDeviceToHost));
  });
}

fdu_status fdu_batch_info(const fdu_batch* b, int* schedule, int* total_tiles, int* grid, int* edges_per_thread,
                          int* vertex_passes, int* vertex_mode) {
  return guard([&] {
    need(b != nullptr, "NULL batch");
    if (schedule) *schedule = b->schedule;
    if (total_tiles) *total_tiles = b->total;
    if (grid) *grid = b->grid;
    if (edges_per_thread) *edges_per_thread = b->tl.ept;
    if (vertex_passes) *vertex_passes = b->tl.vp;
    if (vertex_mode) *vertex_mode = b->vmode;
  });
}

fdu_status fdu_kernel_times(fdu_solver* s, void* w, void* scratch, int reps, double* avg_ms, void* stream) {
  return guard([&] {
    ready(s);
    need(w && scratch && avg_ms && reps > 0, "invalid argument");
    DeviceGuard dg(s->device);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    FDU_HIP(hipEventCreate(&e0));
    FDU_HIP(hipEventCreate(&e1));
    auto timed = [&](auto&& launch) {
      launch();  // warm
      FDU_HIP(hipEventRecord(e0, st));
      for (int i = 0; i < reps; ++i) launch();
      FDU_HIP(hipEventRecord(e1, st));
      FDU_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      FDU_HIP(hipEventElapsedTime(&ms, e0, e1));
      return (double)ms / reps;
    };
    double* dt = reinterpret_cast<double*>(scratch);  // the first 8 bytes of scratch hold dt, rows 1.. the output
    if (s->prec == FDU_F64) {
      double* W = (double*)w;
      double* out = (double*)scratch;
      avg_ms[0] = timed([&] { fill_ghosts_t<double>(s, W, st); });
      avg_ms[3] = timed([&] { cfl_t<double>(s, W, 0.5, dt, st); });
      avg_ms[1] = timed([&] { edge_flux_t<double>(s, W, s->flux.p, st); });
      avg_ms[2] = timed([&] { vertex_t<double>(s, W, 1, nullptr, W, out + 4, 0.75, 0.25, dt, st); });
    } else {
      float* W = (float*)w;
      float* out = (float*)scratch;
      avg_ms[0] = timed([&] { fill_ghosts_t<float>(s, W, st); });
      avg_ms[3] = timed([&] { cfl_t<float>(s, W, 0.5, dt, st); });
      avg_ms[1] = timed([&] { edge_flux_t<float>(s, W, s->flux.p, st); });
      avg_ms[2] = timed([&] { vertex_t<float>(s, W, 1, nullptr, W, out + 4, 0.75, 0.25, dt, st); });
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
}

fdu_status fdu_kernel_timer_start(fdu_solver* s, int capacity, int phases) {
  return guard([&] {
    ready(s);
    need(capacity > 0 && capacity <= (1 << 20), "capacity must be in [1, 2^20]");
    need(phases > 0 && phases <= 15, "phases must be a non-empty subset of bits 0-3");
    DeviceGuard dg(s->device);
    // timing-only events: no system-scope fence (cache writeback) at each record
    for (auto& v : s->timer_ev) {
      while ((int)v.size() < 2 * capacity) {
        hipEvent_t e;
        FDU_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        v.push_back(e);
      }
    }
    s->timer_cap = capacity;
    s->timer_mask = phases;
    for (int& n : s->timer_n) n = 0;
    s->timer_on = true;
  });
}

fdu_status fdu_kernel_timer_stop(fdu_solver* s, double* avg_ms, int* counts) {
  return guard([&] {
    if (!s) throw Error(FDU_ERR_INVALID_ARG, "NULL solver");
    need(avg_ms && counts, "invalid argument");
    need(s->timer_on, "kernel timer not started");
    DeviceGuard dg(s->device);
    s->timer_on = false;
    for (int ph = 0; ph < 4; ++ph) {
      const int n = s->timer_n[ph];
      double sum = 0.0;
      if (n > 0) FDU_HIP(hipEventSynchronize(s->timer_ev[ph][2 * n - 1]));
      for (int i = 0; i < n; ++i) {
        float ms = 0.f;
        FDU_HIP(hipEventElapsedTime(&ms, s->timer_ev[ph][2 * i], s->timer_ev[ph][2 * i + 1]));
        sum += ms;
      }
      counts[ph] = n;
      avg_ms[ph] = n > 0 ? sum / n : 0.0;
    }
  });
}

fdu_status fdu_autotune(fdu_solver* s, void* w, void* scratch, int reps, double* times_ms, void* stream) {
  return guard([&] {
    ready(s);
    need(w && scratch && times_ms && reps > 0, "invalid argument");
    const int e0 = s->edge_variant, v0 = s->vertex_variant;
    double best_e = 1e300, best_v = 1e300;
    int be = e0, bv = v0;
    for (int e = 0; e < kEdgeVariants; ++e) {
      s->edge_variant = e;
      double t[4];
      fdu_status st = fdu_kernel_times(s, w, scratch, reps, t, stream);
      if (st != FDU_OK) { s->edge_variant = e0; s->vertex_variant = v0; throw Error(st, fdu_last_error()); }
      times_ms[e] = t[1];
      if (t[1] < best_e) { best_e = t[1]; be = e; }
    }
    s->edge_variant = be;
    for (int v = 0; v < kVertexVariants; ++v) {
      s->vertex_variant = v;
      double t[4];
      fdu_status st = fdu_kernel_times(s, w, scratch, reps, t, stream);
      if (st != FDU_OK) { s->edge_variant = e0; s->vertex_variant = v0; throw Error(st, fdu_last_error()); }
      times_ms[kEdgeVariants + v] = t[2];
      if (t[2] < best_v) { best_v = t[2]; bv = v; }
    }
    s->vertex_variant = bv;
  });
}

}  // extern "C"
