// Many mesh instances advanced together: one persistent launch per Runge-Kutta
// stage covers every instance's ghost fill, edge fluxes and vertex step.
//
// Work is cut into tiles (ghost tiles, edge tiles, vertex tiles) laid out
// phase-major over instances; workgroups take tiles in ticket order from one
// counter.  An edge tile of instance i waits until i's ghost tiles are done, a
// vertex tile until i's edge tiles are done (per-instance completion
// counters, release/acquire at agent scope).  A tile only waits on tiles with
// smaller tickets, which were taken by workgroups already running, so the
// schedule needs no co-residency.  Every wait is bounded: on timeout an error
// flag is set and the tile proceeds, so every wave always reaches its exit.
#pragma once

#include "kernels.hpp"

namespace fdu {

struct BatchInst {
  const int* sten;
  const double* geo;
  const int* vptr;
  const int* vcol;
  const double* wfg;
  const int* eptr;
  const int* ecol;
  const double* we;
  const double* cO;
  const double* hmin;
  const int* gsrc;
  const signed char* grefl;
  const double* gstate;   // Dirichlet ghost states ([ng][4]) or null
  const int* vblk;   // vertex blocks of the LDS-staged vertex step
  const int* vb_own;
  const int* vb_uvp;
  const int* vb_uv;
  const int* vb_uep;
  const int* vb_ue;
  const unsigned short* vb_lvcol;
  const unsigned short* vb_lecol;
  const PackedIds* vb_pk;   // packed first-round ids of the block kernel
  double* flux;
  double* w;    // state (in/out)
  double* w1;   // stage buffers
  double* w2;
  int nv_real, nv_total, ne, ng;
};

constexpr unsigned kWaitLimit = 1u << 22;

// The instance table as the kernels read it: the same layout with every
// pointer typed as a global-memory pointer.  Read through BatchInst the
// pointers would be generic, and generic (flat) loads also count against the
// LDS wait counter, so every LDS wait in the kernels would wait for all memory
// loads in flight.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

struct BatchInstG {
  gptr<const int> sten;
  gptr<const double> geo;
  gptr<const int> vptr;
  gptr<const int> vcol;
  gptr<const double> wfg;
  gptr<const int> eptr;
  gptr<const int> ecol;
  gptr<const double> we;
  gptr<const double> cO;
  gptr<const double> hmin;
  gptr<const int> gsrc;
  gptr<const signed char> grefl;
  gptr<const double> gstate;
  gptr<const int> vblk;
  gptr<const int> vb_own;
  gptr<const int> vb_uvp;
  gptr<const int> vb_uv;
  gptr<const int> vb_uep;
  gptr<const int> vb_ue;
  gptr<const unsigned short> vb_lvcol;
  gptr<const unsigned short> vb_lecol;
  gptr<const PackedIds> vb_pk;
  gptr<double> flux;
  gptr<double> w;
  gptr<double> w1;
  gptr<double> w2;
  int nv_real, nv_total, ne, ng;
};
static_assert(sizeof(BatchInstG) == sizeof(BatchInst) && offsetof(BatchInstG, w2) == offsetof(BatchInst, w2) &&
                  offsetof(BatchInstG, ng) == offsetof(BatchInst, ng),
              "the two views of an instance must share their layout");

// Instance i of the table, its pointers derived from global-memory pointers.
__device__ __forceinline__ BatchInst global_view(const BatchInst* __restrict__ inst, int i) {
  const BatchInstG& G = reinterpret_cast<const BatchInstG*>(inst)[i];
  BatchInst I;
  I.sten = (const int*)G.sten; I.geo = (const double*)G.geo;
  I.vptr = (const int*)G.vptr; I.vcol = (const int*)G.vcol; I.wfg = (const double*)G.wfg;
  I.eptr = (const int*)G.eptr; I.ecol = (const int*)G.ecol; I.we = (const double*)G.we;
  I.cO = (const double*)G.cO; I.hmin = (const double*)G.hmin;
  I.gsrc = (const int*)G.gsrc; I.grefl = (const signed char*)G.grefl; I.gstate = (const double*)G.gstate;
  I.vblk = (const int*)G.vblk; I.vb_own = (const int*)G.vb_own; I.vb_uvp = (const int*)G.vb_uvp;
  I.vb_uv = (const int*)G.vb_uv; I.vb_uep = (const int*)G.vb_uep; I.vb_ue = (const int*)G.vb_ue;
  I.vb_lvcol = (const unsigned short*)G.vb_lvcol; I.vb_lecol = (const unsigned short*)G.vb_lecol;
  I.vb_pk = (const PackedIds*)G.vb_pk;
  I.flux = (double*)G.flux; I.w = (double*)G.w; I.w1 = (double*)G.w1; I.w2 = (double*)G.w2;
  I.nv_real = G.nv_real; I.nv_total = G.nv_total; I.ne = G.ne; I.ng = G.ng;
  return I;
}

__device__ __forceinline__ void wait_count(unsigned* c, unsigned target, int* err) {
  if (threadIdx.x == 0) {
    unsigned it = 0;
    while (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++it > kWaitLimit) {
        atomicOr(err, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void signal_count(unsigned* c) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// largest j in [0, m) with tb[j] <= t (tb non-decreasing, tb[0] = 0)
__device__ __forceinline__ int find_slot(const int* __restrict__ tb, int m, int t) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tb[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct BatchTiling {
  int ept;   // edges per thread in an edge tile (tile = 256 * ept edges)
  int vp;    // vertex passes per tile (tile = vp * 256 / LPV vertices)
};

__device__ __forceinline__ int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Vertex-tile modes: 0 = strided loops, 16 lanes per vertex; 1 = strided
// loops, 8 lanes; 2 = pipelined loads, 8 lanes (few registers live across
// the gathers, for the fused kernel, whose register budget the edge code sets);
// 3 = one vertex block per tile with its stencil halo staged in LDS (the block
// code of vertex variant 4; the kernel is launched with the largest block's
// LDS, which edge and ghost tiles leave unused).
template <int VM>
struct VertexMode {
  static constexpr int lpv = VM == 0 ? 16 : 8;
};

// PH < 0: fused schedule with dynamic tickets and dependency waits; PH 0/1/2:
// a kernel holding only that phase's code, one tile per block (no waits).
// In the fused kernel a workgroup runs many tiles one after the other; the
// tile table is copied to LDS once (at tb_off ints into the dynamic LDS, after
// the vertex-block rows of mode 3) and searched there.  (Taking the next
// ticket while a tile runs was measured slower: a reserved edge tile can hold
// back every vertex tile of its instance until the current tile ends.)
template <int EV, int VM, int PH>
__global__ void __launch_bounds__(256) k_batch_stage(const BatchInst* __restrict__ inst, int n,
                                                     const int* __restrict__ tb, int total, unsigned* ctr, Scheme S,
                                                     int k, double a, double b, const double* __restrict__ dt,
                                                     int* err, BatchTiling tl, int tb_off) {
  constexpr int LPV = VertexMode<VM>::lpv;
  constexpr int phase = PH;
  __shared__ int sh;
  extern __shared__ double lds[];   // vertex mode 3: the block's staged rows and CSR pointers
  int* stb = reinterpret_cast<int*>(lds) + tb_off;   // fused kernel: the tile table
  if (phase < 0)
    for (int i = threadIdx.x; i <= 3 * n; i += blockDim.x) stb[i] = tb[i];
  for (int iter = 0;; ++iter) {
    int t;
    if (phase < 0) {
      __syncthreads();   // the previous tile is done (its LDS rows read); the table is written
      if (threadIdx.x == 0) sh = (int)atomicAdd(&ctr[0], 1u);
      __syncthreads();
      t = sh;
    } else {
      if (iter > 0) return;
      t = tb[phase * n] + blockIdx.x;
      if (t >= tb[(phase + 1) * n]) return;
    }
    if (t >= total) return;
    int j, tj;
    if constexpr (PH < 0) {
      j = find_slot(stb, 3 * n, t);
      tj = stb[j];
    } else {
      j = find_slot(tb, 3 * n, t);
      tj = tb[j];
    }
    const int p = j / n, i = j - p * n, local = t - tj;
    const BatchInst I = global_view(inst, i);
    double* wprev = k == 0 ? I.w : (k == 1 ? I.w1 : I.w2);
    double* wout = k == 0 ? I.w1 : (k == 1 ? I.w2 : I.w);
    if (PH <= 0 && p == 0) {
      const int g = local * 256 + threadIdx.x;
      if (g < I.ng) {
        double q[4];
        ghost_state<double>(wprev, g, I.gsrc, I.grefl, I.gstate, q);
        store4(wprev, I.nv_real + g, q);
      }
      if (phase < 0) signal_count(&ctr[1 + i]);
    } else if ((PH < 0 || PH == 1) && p == 1) {
      if (phase < 0 && I.ng > 0) wait_count(&ctr[1 + i], (unsigned)ceil_div(I.ng, 256), err);
      for (int q = 0; q < tl.ept; ++q) {
        const int e = (local * tl.ept + q) * 256 + threadIdx.x;
        if (e < I.ne) {
          if (EV == 1)
            edge_lean_item<double, double>(wprev, I.sten, I.geo, I.flux, e, S);
          else
            edge_item<double, double>(wprev, I.sten, I.geo, I.flux, e, S);
        }
      }
      if (phase < 0) signal_count(&ctr[1 + n + i]);
    } else if ((PH < 0 || PH == 2) && p == 2) {
      if (phase < 0) wait_count(&ctr[1 + n + i], (unsigned)ceil_div(I.ne, 256 * tl.ept), err);
      if constexpr (VM == 3 && PH < 0) {
        vertex_block2<double, double, 8, 3, 6, 1, true>(local, lds, wprev, I.vblk, I.vb_own, I.vb_uvp, I.vb_uv,
                                                        I.vb_uep, I.vb_ue, I.vptr, I.vb_lvcol, I.wfg, I.eptr,
                                                        I.vb_lecol, I.we, I.cO, I.flux, S.gm1, 1, nullptr, I.w, wout,
                                                        a, b, dt + i, I.vb_pk);
        continue;
      }
      for (int q = 0; q < tl.vp; ++q) {
        const int tt = (local * tl.vp + q) * 256 + threadIdx.x;
        const int v = tt / LPV;
        if (VM == 2)
          vertex_pipe_item<double, double, 8, 3, 6>(wprev, I.vptr, I.vcol, I.wfg, I.eptr, I.ecol, I.we, I.cO, I.flux,
                                                    I.nv_real, S.gm1, 1, nullptr, I.w, wout, a, b, dt + i, v,
                                                    tt % LPV);
        else
          vertex_item<double, double, LPV, false>(wprev, I.vptr, I.vcol, I.wfg, I.eptr, I.ecol, I.we, I.cO, I.flux,
                                                  I.nv_real, S.gm1, 1, nullptr, I.w, wout, a, b, dt + i, v,
                                                  tt % LPV);
      }
    }
  }
}

// Vertex phase over all instances with the stencil halos staged in LDS: one
// workgroup per vertex block; tile t of the phase maps to (instance, block).
// The block kernel of vertex variant 4 (packed ids, 5 waves per SIMD).
template <int LPV, int MV, int ME, int PF, int WPE, bool PK>
__global__ void __launch_bounds__(256, WPE) k_batch_vertex_lds(const BatchInst* __restrict__ inst, int n,
                                                               const int* __restrict__ tb, Scheme S, int k, double a,
                                                               double b, const double* __restrict__ dt) {
  extern __shared__ double lds[];
  const int t = tb[2 * n] + blockIdx.x;
  if (t >= tb[3 * n]) return;
  const int j = find_slot(tb + 2 * n, n, t);
  const BatchInst I = global_view(inst, j);
  const double* wprev = k == 0 ? I.w : (k == 1 ? I.w1 : I.w2);
  double* wout = k == 0 ? I.w1 : (k == 1 ? I.w2 : I.w);
  vertex_block2<double, double, LPV, MV, ME, PF, PK>(t - tb[2 * n + j], lds, wprev, I.vblk, I.vb_own, I.vb_uvp,
                                                     I.vb_uv, I.vb_uep, I.vb_ue, I.vptr, I.vb_lvcol, I.wfg, I.eptr,
                                                     I.vb_lecol, I.we, I.cO, I.flux, S.gm1, 1, nullptr, I.w, wout, a, b,
                                                     dt + j, I.vb_pk);
}

// Per-instance CFL: block minima of hmin_v / (|u_v| + c_v) over 256-vertex
// tiles, combined per instance with an integer atomicMin on the bit patterns
// (positive doubles order like their bits, so the result is exact and
// independent of the order).
__global__ void __launch_bounds__(256) k_batch_cfl(const BatchInst* __restrict__ inst, int n,
                                                   const int* __restrict__ tbc, int total, double gamma,
                                                   unsigned long long* dtbits) {
  __shared__ double sm[256];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int i = find_slot(tbc, n, t);
    const BatchInst I = global_view(inst, i);
    const int v = (t - tbc[i]) * 256 + threadIdx.x;
    double best = 1e300;
    if (v < I.nv_real) {
      double q[4];
      load4(I.w, v, q);
      const double ir = 1.0 / q[0];
      const double u = q[1] * ir, vv = q[2] * ir;
      const double p = (gamma - 1.0) * (q[3] - 0.5 * (q[1] * u + q[2] * vv));
      best = I.hmin[v] / (sqrt(u * u + vv * vv) + sqrt(gamma * p * ir));
    }
    sm[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
      __syncthreads();
    }
    if (threadIdx.x == 0) atomicMin(&dtbits[i], (unsigned long long)__double_as_longlong(sm[0]));
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_batch_dt(const unsigned long long* __restrict__ dtbits, int n, double cfl,
                                                  double* __restrict__ dt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dt[i] = cfl * __longlong_as_double((long long)dtbits[i]);
}

// Zero the stage counters; optionally reset the CFL minima to +inf.
__global__ void __launch_bounds__(256) k_batch_reset(unsigned* ctr, int nctr, unsigned long long* dtbits, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nctr) ctr[i] = 0u;
  if (dtbits != nullptr && i < n) dtbits[i] = 0x7FF0000000000000ull;
}

}  // namespace fdu
