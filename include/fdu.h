/*
 * fdu.h: C ABI of the MI355X (gfx950) library for the per-Runge-Kutta-stage
 * residual of the unstructured-mesh finite-difference Euler scheme of
 * Zhen, Qu and Cai, "A Novel Finite Difference Method for Euler Equations in
 * 2D Unstructured Meshes".
 *
 * The residual of one stage is dw/dt = -(df/dx + dg/dy) at every real vertex
 * (2D Euler equations, Sec. 2.1: w = [rho, rho u, rho v, rho E],
 * p = (gamma-1) rho e), computed in two steps (abstract; Sec. 2.2, 2.3):
 *   edge step   for every edge a divergence stencil uses, non-uniform WENO5
 *               interpolation of characteristic variables at the edge midpoint
 *               along the edge's six-point curvilinear stencil (Sec. 2.3.1,
 *               Appendix), then the numerical flux projected on the edge
 *               direction, r_k;
 *   vertex step the least-squares divergence at vertex O as a weighted sum over
 *               the stencil's vertex fluxes and edge projections (Sec. 2.2.1,
 *               the weight row r_a1 + r_b2 of the pseudo-inverse), then the
 *               SSP-RK3 stage update (the third-order TVD Runge-Kutta scheme of
 *               Sec. 3).
 *
 * Conventions
 *   - Every call returns fdu_status; on failure fdu_last_error() gives a
 *     message (thread-local, valid until the next call on that thread).  No
 *     C++ exception crosses this boundary.
 *   - "host" pointers are read during the call only; the caller keeps
 *     ownership.  "device" pointers are caller-owned device memory on the
 *     solver's HIP device; the library never frees them.
 *   - Compute calls are asynchronous on the given hipStream_t (passed as
 *     void*; NULL = the default stream) and allocate nothing.  Set-up calls
 *     (create, prep, upload, finalize) are synchronous.
 *   - State layout: array of structures, vertex-major [nv_total][4] of
 *     double (FDU_F64) or float (FDU_F32 storage); real vertices occupy rows
 *     [0, nv_real), ghost vertices rows [nv_real, nv_total).  Residual and
 *     cotangent arrays are [nv_real][4] (residual) or [nv_total][4] (state
 *     cotangents).  Edge fluxes are [ne_flux][4] double.
 *   - Vertex and edge numbering inside the library is the prep's order
 *     (reverse Cuthill-McKee or Hilbert order of the real vertices when
 *     requested); the prep exposes the permutation so callers can map their
 *     arrays.
 */
#ifndef FDU_H
#define FDU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FDU_OK = 0,
  FDU_ERR_INVALID_ARG = 1, /* bad size, pointer, index or value */
  FDU_ERR_HIP = 2,         /* a HIP runtime call failed */
  FDU_ERR_OOM = 3,         /* device or host allocation failed */
  FDU_ERR_STATE = 4,       /* call out of order (e.g. compute before finalize) */
  FDU_ERR_UNSUPPORTED = 5, /* option not built */
  FDU_ERR_NUMERIC = 6      /* rank-deficient least-squares system, bad stencil */
} fdu_status;

typedef enum { FDU_F64 = 0, FDU_F32 = 1 } fdu_precision;

/* Scheme parameters.  Defaults (fdu_default_params): gamma 1.4 (Sec. 2.1),
 * WENO eps 1e-40 and power 1 (Appendix), Roe flux with Harten's entropy fix
 * delta = 0.1 * c_roe, positivity fallback on.
 * positivity (not in the paper): when an interpolated midpoint state has
 * rho <= 0 or p <= 0, that side of the edge uses its end vertex state.
 * interpolation and uniform_weno (default 0 and 0, the paper's scheme) are
 * ablation switches: interpolate the conservative variables directly (no
 * characteristic projection), and/or use the uniform WENO5 coefficients
 * whatever the node spacing along the stencil. */
typedef struct {
  double gamma;
  double weno_eps;
  double entropy_frac;
  int weno_power; /* 1 or 2 */
  int riemann;    /* 0 = Roe + Harten fix, 1 = Rusanov */
  int positivity; /* 0 or 1 */
  int interpolation; /* 0 = characteristic variables (Sec. 2.3.1), 1 = conservative variables */
  int uniform_weno;  /* 0 = NU-WENO5 on the arc coordinates (Appendix), 1 = standard WENO5 on
                        equally spaced nodes (the comparison of Sec. 2.3.2) */
} fdu_params;

const char* fdu_last_error(void);
void fdu_default_params(fdu_params* out);

/* ------------------------------------------------------------------------
 * Host preprocessing (once per static mesh, Sec. 2.2.1: the weights depend on
 * geometry only).  Builds, in C++ on the host:
 *   - the divergence stencil of every real vertex (one-level: neighbours and
 *     the edges of the incident triangles; two-level: the union of the
 *     one-level stencils of the vertex and its neighbours, Sec. 2.2.2; a
 *     one-level stencil with fewer than deg(deg+3)+4 conditions is promoted
 *     to two-level);
 *   - the least-squares weights by Householder QR with column pivoting of the
 *     scaled system (the row r_a1 + r_b2 of the pseudo-inverse A^+, divided by
 *     the scale h_O; pivots below 1e-10 of the first count as dependent, as in
 *     a pseudo-inverse that drops zero singular values, and FDU_ERR_NUMERIC is
 *     returned if the divergence is then not determined by the stencil);
 *   - the six-point stencil (L3 L2 L1 R1 R2 R3) of every edge those stencils
 *     use (L1 = smaller input id; each continuation is the neighbour that best
 *     continues the previous segment's direction, cosines within 1e-12 tie to
 *     the smaller input id) and its Catmull-Rom arc-length coordinates
 *     (Sec. 2.3.1), normalised by the edge length;
 *   - the vertex order (natural, reverse Cuthill-McKee or Hilbert order of
 *     the real vertices) and the flux-edge order (by smallest new end id).
 * Inputs (host, read only during the call):
 *   xy [nv_total][2] double; edges [ne][2] int32 (a < b); tris [nt][3] int32;
 *   ghost_src [ng] int32 (source real vertex of ghost nv_real+i),
 *   ghost_refl [ng] int8 (bit 0: negate m_x, bit 1: negate m_y, bit 2:
 *   Dirichlet ghost whose state is given, see fdu_upload_ghost_states); ng =
 *   nv_total - nv_real; periodic = 1 wraps displacements to the nearest image
 *   in the box Lx x Ly, 2 wraps y only (a channel with walls in x), 0 none.  deg = polynomial degree (3..6), level = 0 (automatic:
 *   one-level for deg <= 3, two-level otherwise), 1 or 2; reorder = 0 natural,
 *   1 reverse Cuthill-McKee, 2 Hilbert curve through the vertex coordinates.
 *   nthreads <= 0 uses all host cores.  artificial != 0 (Sec. 2.2.2): a real
 *   vertex whose one-level stencil has fewer than deg(deg+3)+4 conditions is
 *   joined by artificial edges to the far vertex of the triangle across each of
 *   its ring edges (when not yet a neighbour), and those vertices and edges join
 *   its one-level stencil (two-level only if still short).  Artificial edges get
 *   input edge ids ne, ne+1, ... in lexicographic order of their end ids; the
 *   neighbour graph used for two-level stencils and for 1D stencil continuation
 *   stays that of the input edges.
 * Errors: FDU_ERR_INVALID_ARG for inconsistent sizes or ids, FDU_ERR_NUMERIC
 * when an edge has no admissible stencil continuation or a least-squares
 * matrix is rank deficient.
 */
typedef struct fdu_prep fdu_prep;

typedef struct {
  int64_t nv_total, nv_real, ne_flux, nnz_v, nnz_e;
  /* arrays owned by the prep object, valid until fdu_prep_destroy */
  const int32_t* perm;       /* [nv_total] new id -> input id */
  const int32_t* iperm;      /* [nv_total] input id -> new id */
  const int32_t* flux_edge;  /* [ne_flux] input edge id of each flux edge */
  const int32_t* sten6;      /* [ne_flux][6] new vertex ids L3 L2 L1 R1 R2 R3 */
  const double* geo;         /* [ne_flux][6] s0/d, s1/d, s4/d, s5/d, n_x, n_y */
  const int32_t* vptr;       /* [nv_real+1] */
  const int32_t* vcol;       /* [nnz_v] new vertex ids */
  const double* wfg;         /* [nnz_v][2] (wf, wg) */
  const int32_t* eptr;       /* [nv_real+1] */
  const int32_t* ecol;       /* [nnz_e] flux-edge ids */
  const double* we;          /* [nnz_e] */
  const double* hmin;        /* [nv_real] shortest incident edge */
  const int32_t* ghost_src;  /* [ng] new ids of the ghost sources */
  const int8_t* ghost_refl;  /* [ng] */
  int64_t n_artificial;      /* artificial edges (input edge ids ne .. ne + n - 1) */
  const int32_t* artificial; /* [n_artificial][2] their input end ids (a < b) */
} fdu_prep_view;

fdu_status fdu_prep_build(fdu_prep** out, int64_t nv_total, int64_t nv_real, const double* xy,
                          int64_t ne, const int32_t* edges, int64_t nt, const int32_t* tris,
                          const int32_t* ghost_src, const int8_t* ghost_refl, int periodic,
                          double Lx, double Ly, int deg, int level, int reorder, int nthreads,
                          int artificial);
fdu_status fdu_prep_view_get(const fdu_prep* prep, fdu_prep_view* out);
void fdu_prep_destroy(fdu_prep* prep);

/* ------------------------------------------------------------------------
 * Solver: device-resident stencils and weights of one mesh instance.
 * CSR pointers (vptr, eptr) are 32-bit offsets: a solver holds at most
 * 2^31 - 1 vertex entries and as many edge entries (about 110 M real vertices
 * with two-level stencils of 19 vertices and 44 edges); the prep refuses
 * larger meshes with FDU_ERR_INVALID_ARG.
 * fdu_create selects hip_device and allocates nothing large.
 * fdu_upload_* copy host arrays (layouts as in fdu_prep_view, all in the
 * library's numbering) into library-owned device memory; they validate ids
 * and CSR monotonicity and reject non-finite weights (FDU_ERR_INVALID_ARG).
 * fdu_upload_prep uploads everything a prep built.  fdu_finalize derives
 * the per-vertex sums c_O = sum_k we_k n_k and must precede compute calls.
 * fdu_upload_ghost_states (Dirichlet boundaries, the paper's inflow/outflow
 * conditions): states [ng][4] (host, conservative variables, library ghost
 * order); the rows of ghosts flagged Dirichlet (bit 2) are the states those
 * ghosts take at every ghost fill, other rows are ignored.  Required before
 * fdu_finalize when Dirichlet ghosts exist; may be called again later to
 * change the boundary values (same device buffer, so captured graphs see the
 * new values).  Synchronous.  FDU_ERR_INVALID_ARG for a count mismatch or a
 * non-finite or non-positive-density Dirichlet row.  The adjoint treats
 * Dirichlet ghosts as constants.
 */
typedef struct fdu_solver fdu_solver;

fdu_status fdu_create(fdu_solver** out, int hip_device, fdu_precision prec, const fdu_params* params);
void fdu_destroy(fdu_solver* s);
fdu_status fdu_upload_edge_stencils(fdu_solver* s, int64_t nv_total, int64_t nv_real, int64_t ne_flux,
                                    const int32_t* sten6, const double* geo);
fdu_status fdu_upload_vertex_stencils(fdu_solver* s, const int32_t* vptr, const int32_t* vcol,
                                      const double* wfg, const int32_t* eptr, const int32_t* ecol,
                                      const double* we, const double* hmin);
fdu_status fdu_upload_ghosts(fdu_solver* s, int64_t ng, const int32_t* ghost_src, const int8_t* ghost_refl);
fdu_status fdu_upload_ghost_states(fdu_solver* s, int64_t ng, const double* states);
fdu_status fdu_upload_prep(fdu_solver* s, const fdu_prep* prep);
fdu_status fdu_finalize(fdu_solver* s);

/* Sizes of the uploaded problem. */
fdu_status fdu_sizes(const fdu_solver* s, int64_t* nv_total, int64_t* nv_real, int64_t* ne_flux,
                     int64_t* nnz_v, int64_t* nnz_e);

/* ------------------------------------------------------------------------
 * Compute calls (asynchronous on stream, no allocation).
 *
 * fdu_fill_ghosts (boundary conditions; Sec. 3.3 for the Dirichlet
 *   inflow/outflow states, walls are not in the paper): rows [nv_real,
 *   nv_total) of w (device, in/out) := their mirror sources with the flagged
 *   momentum components negated, or the given Dirichlet states.
 * fdu_edge_fluxes (Sec. 2.3.1 and the Appendix: the six-point curvilinear
 *   stencil, NU-WENO5 of the characteristic variables at the edge midpoint,
 *   then the numerical flux): r (device [ne_flux][4] double) := the flux
 *   projections along each flux edge from the state w (device, read only;
 *   its ghost rows must be filled).
 * fdu_residual (Sec. 2.2.1, the least-squares divergence as the weight row of
 *   the pseudo-inverse applied to the differenced vertex fluxes and the edge
 *   projections; dw/dt = -div, Sec. 2.1): R (device [nv_real][4]) := dw/dt at
 *   the real vertices for the state w (device [nv_total][4], read only: on
 *   meshes with ghosts the library copies w's real rows into a state buffer it
 *   allocated at fdu_finalize and fills that copy's ghost rows, so w's ghost
 *   rows are neither read nor written).  The edge fluxes go to the solver's
 *   flux buffer.
 * fdu_cfl_dt (Sec. 3.1 names the CFL number; the formula is this library's
 *   reading): dt_dev (device, one double) := cfl * min over real vertices of
 *   hmin_v / (|u_v| + c_v), hmin_v the shortest edge at v.
 * fdu_rk_stage (Sec. 3, the third-order TVD Runge-Kutta scheme, here the
 *   Shu-Osher SSP-RK3): stage k in {0,1,2} on the real rows:
 *   w_out = a_k w_n + b_k (w_prev + dt R(w_prev)), (a,b) = (0,1), (3/4,1/4),
 *   (1/3,2/3); dt read from dt_dev (device).  w_prev's ghost rows are filled
 *   in place (the only rows of w_prev written); w_out must not alias w_prev
 *   (other vertices gather from it) but may alias w_n (each vertex reads only
 *   its own row of w_n); w_n is unused at k = 0; w_out's ghost rows are not
 *   written.
 * fdu_rk_step (Sec. 3): one full SSP-RK3 step in place on w (device
 *   [nv_total][4]), using scratch (device, two states [2][nv_total][4]); if
 *   cfl > 0 the step first sets *dt_dev from the CFL condition, otherwise it
 *   reads *dt_dev.
 * Errors: FDU_ERR_STATE before fdu_finalize; FDU_ERR_INVALID_ARG for NULL
 * pointers or k out of range; FDU_ERR_HIP if a launch fails.
 */
fdu_status fdu_fill_ghosts(fdu_solver* s, void* w, void* stream);
fdu_status fdu_edge_fluxes(fdu_solver* s, const void* w, double* r, void* stream);
fdu_status fdu_residual(fdu_solver* s, const void* w, void* R, void* stream);
fdu_status fdu_cfl_dt(fdu_solver* s, const void* w, double cfl, double* dt_dev, void* stream);
fdu_status fdu_rk_stage(fdu_solver* s, int k, const void* w_n, void* w_prev, void* w_out,
                        const double* dt_dev, void* stream);
fdu_status fdu_rk_step(fdu_solver* s, void* w, void* scratch, double cfl, double* dt_dev, void* stream);

/* fdu_rk_step_static: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same step as fdu_rk_step (same kernels, same results bit for
 * bit) with the two stage states in a static device array of the library
 * instead of a caller workspace: w (device [nv_total][4], in/out), cfl and
 * dt_dev as for fdu_rk_step.  Allocates nothing and calls no allocating
 * routine.  The array holds 80 MiB (83,886,080 bytes) on every GPU the library
 * runs on, until the process ends: two states of up to 1,310,720 vertices
 * (nv_total) in FP64, 2,621,440 in FP32 storage; larger solvers get
 * FDU_ERR_INVALID_ARG (use fdu_rk_step).  Every call on one GPU uses that GPU's
 * array, so calls that overlap in time on one GPU (other streams, other
 * threads) race; calls in stream order do not (each stage state is written
 * before it is read within the call).  Errors as for fdu_rk_step. */
fdu_status fdu_rk_step_static(fdu_solver* s, void* w, double cfl, double* dt_dev, void* stream);

/* ------------------------------------------------------------------------
 * Adjoint (vector-Jacobian products) of the residual and of the SSP-RK3 stage
 * and step, for gradients through unrolled time stepping.
 * fdu_enable_adjoint (set-up, synchronous, after fdu_finalize): builds the
 *   transposed stencil maps on the host and allocates the work buffers
 *   (about 250 bytes per flux edge plus 32 per vertex).
 * fdu_residual_vjp: wbar (device [nv_total][4], state dtype) :=
 *   (dR/dw)^T Rbar for Rbar (device [nv_real][4]); ghost rows of wbar are zero
 *   (ghost states are copies of real ones and their cotangent is added to the
 *   source rows).  w is read only (its ghost rows are filled in the library's
 *   copy, as in fdu_residual); wbar must not alias w or Rbar.
 * fdu_rk_stage_vjp: adjoint of fdu_rk_stage k with the scalar dt:
 *   wbar_prev := b_k obar + b_k dt (dR/dw_prev)^T obar (ghost rows zero) and,
 *   for k > 0, wbar_n += a_k obar on the real rows.  obar is [nv_total][4]
 *   (real rows used).
 * fdu_rk_step_vjp: adjoint of one fdu_rk_step at the fixed time step dt (one
 *   value, written to a device scalar of the solver and used both for the
 *   recomputed forward stages and for the reverse sweep): recomputes the stage
 *   states from w_n (in/out: ghost rows filled) and writes
 *   wbar_n := (dw_{n+1}/dw_n)^T wbar_np1.  scratch: device, 4 states.
 * fdu_rk_step_vjp_stages: the same adjoint given the step's stage states
 *   w_1, w_2 (the two states fdu_rk_step leaves in its workspace, in that
 *   order, or fdu_rk_stage's outputs for k = 0, 1) instead of recomputing them:
 *   for checkpointed unrolling, whose segment recompute already produces
 *   them.  w_n, w_1, w_2 are in/out (ghost rows filled); scratch: device, 2
 *   states.  Equal to fdu_rk_step_vjp bit for bit when the stage states are
 *   the ones it would recompute.
 * Errors: FDU_ERR_STATE if the adjoint is not enabled; FDU_ERR_INVALID_ARG for
 * NULL or aliased arguments.  Asynchronous on stream; no allocation.
 */
fdu_status fdu_enable_adjoint(fdu_solver* s);
fdu_status fdu_residual_vjp(fdu_solver* s, const void* w, const void* Rbar, void* wbar, void* stream);
fdu_status fdu_rk_stage_vjp(fdu_solver* s, int k, void* w_prev, const void* obar, void* wbar_n, void* wbar_prev,
                            double dt, void* stream);
fdu_status fdu_rk_step_vjp_stages(fdu_solver* s, void* w_n, void* w_1, void* w_2, const void* wbar_np1,
                                  void* wbar_n, void* scratch, double dt, void* stream);
fdu_status fdu_rk_step_vjp(fdu_solver* s, void* w_n, const void* wbar_np1, void* wbar_n, void* scratch, double dt,
                           void* stream);

/* fdu_kernel_times: measurement aid.  Launches each kernel of a stage reps
 * times back to back on stream, bracketed by HIP events, and writes the mean
 * duration in milliseconds to avg_ms[0..3] = ghost fill, edge flux, vertex
 * step (RK stage form), CFL reduction.  w (device state, ghost rows filled) is
 * read and its ghost rows rewritten with the same values; scratch (device,
 * [nv_total+1][4], same dtype as w) receives the time step in its first 8
 * bytes and the stage output from row 1 on.  Synchronous: returns after the last launch.
 * The timed work equals the work of the corresponding compute calls. */
fdu_status fdu_kernel_times(fdu_solver* s, void* w, void* scratch, int reps, double* avg_ms, void* stream);

/* Live kernel timer: measurement aid for the ordinary compute calls.
 * fdu_kernel_timer_start: from now on every launch of the ghost-fill, edge-flux,
 * vertex and CFL kernels by this solver (fdu_fill_ghosts, fdu_edge_fluxes,
 * fdu_residual, fdu_cfl_dt, fdu_rk_stage, fdu_rk_step) whose kind is selected
 * by `phases` (bit 0 ghost fill, 1 edge flux, 2 vertex step, 3 CFL; 15 = all)
 * is bracketed by a pair of timing-only HIP events recorded on the stream of
 * that call, for the first `capacity` (1 .. 2^20) launches of each kind;
 * nothing is recorded while the stream is being captured into a graph.
 * Creates the events on first use (set-up, synchronous); the solver owns them
 * until fdu_destroy.
 * fdu_kernel_timer_stop: stops recording, waits for the last recorded event and
 * writes, for ghost fill, edge flux, vertex step and CFL reduction in that
 * order, the mean bracketed duration in milliseconds to avg_ms[0..3] and the
 * number of launches timed to counts[0..3] (0 and 0.0 when none).  Returns
 * FDU_ERR_INVALID_ARG when the timer is not running or a pointer is NULL.
 * The event records add a few microseconds per launch to the stream. */
fdu_status fdu_kernel_timer_start(fdu_solver* s, int capacity, int phases);
fdu_status fdu_kernel_timer_stop(fdu_solver* s, double* avg_ms, int* counts);

/* ------------------------------------------------------------------------
 * Batches: many FP64 instances (finalized solvers on one device with equal
 * scheme parameters and edge variant) advanced together.
 * fdu_batch_create: builds the tile tables (set-up, synchronous).
 * fdu_batch_set_states: per instance, w[i] (device [nv_total_i][4] double,
 *   in/out) and scratch[i] (device, two states); pointers are captured, so a
 *   later call re-binds them (and drops a captured graph).
 * fdu_batch_set_schedule: 0 = one persistent launch per stage for all
 *   instances (tiles in ticket order, per-instance completion counters,
 *   bounded dependency waits); 1 = one launch per phase (ghost, edge, vertex)
 *   for all instances, each phase its own kernel; 2 = every instance's own
 *   stage kernels in turn.  Tile shape: edges_per_thread (edge tile = 256 x
 *   that), vertex_passes and vertex_mode (0: strided loops, 16 lanes per
 *   vertex; 1: strided loops, 8 lanes; 2: pipelined loads, 8 lanes; vertex
 *   tile = passes x 256 / lanes; 3: one tile per vertex block of the
 *   instance with its stencil halo staged in LDS, the code of vertex variant
 *   4; in schedule 0 the persistent kernel carries the largest block's LDS).  Results equal
 *   the plain path's with vertex variant 0, 1, 2 and 3 (= 4, 5) respectively,
 *   bit for bit (the edge phase runs edge variant 0's code when the instances
 *   use edge variant 0, else variant 1's).
 * fdu_batch_step: one SSP-RK3 step of every instance with its own dt =
 *   cfl * min hmin/(|u|+c) (computed on the device), asynchronous on stream.
 * fdu_batch_capture: records nsteps steps on stream (not the default stream)
 *   into a HIP graph owned by the batch; fdu_batch_launch replays it.
 * fdu_batch_status: synchronizes the device; returns the dependency-wait
 *   timeout flag (0 = none) and copies the last per-instance dt to the host.
 * fdu_batch_info: current schedule, tile count, fused grid size, tile shape.
 */
typedef struct fdu_batch fdu_batch;
fdu_status fdu_batch_create(fdu_batch** out, fdu_solver* const* inst, int n);
void fdu_batch_destroy(fdu_batch* b);
fdu_status fdu_batch_set_states(fdu_batch* b, void* const* w, void* const* scratch);
fdu_status fdu_batch_set_schedule(fdu_batch* b, int schedule, int edges_per_thread, int vertex_passes,
                                  int vertex_mode);
fdu_status fdu_batch_step(fdu_batch* b, double cfl, void* stream);
fdu_status fdu_batch_capture(fdu_batch* b, double cfl, int nsteps, void* stream);
fdu_status fdu_batch_launch(fdu_batch* b, void* stream);
fdu_status fdu_batch_status(fdu_batch* b, int* wait_timeouts, double* dt_host);
fdu_status fdu_batch_info(const fdu_batch* b, int* schedule, int* total_tiles, int* grid, int* edges_per_thread,
                          int* vertex_passes, int* vertex_mode);

/* Kernel variants and autotuning.  Every variant computes the same residual
 * (the parity tests run each one); they differ in schedule and register use:
 *   edge:   0 = coefficient-form WENO, IEEE divisions; 1 = divided-difference
 *           WENO on the edge's six nodes, the two middle quadratics shared by
 *           both sides (four per component instead of six), refined
 *           reciprocals and square roots;
 *   vertex: 0, 1 = 16 and 8 lanes per vertex, strided loops over the CSR
 *           rows; 2 = 8 lanes per vertex, all index/weight loads issued before
 *           all gathers; 3 = 8 lanes per vertex over vertex blocks whose
 *           stencil halo (state and flux rows) is first staged in LDS, 16-bit
 *           block-local row indices (blocks are built at fdu_finalize; they
 *           are compact when the prep used the Hilbert order, reorder = 2);
 *           4, 5 = the blocks of variant 3 with their CSR pointers and own
 *           state rows also staged in LDS, the stage combine spread over 4
 *           lanes, and each lane's first-round row indices (3 state rows, 6
 *           flux rows) packed 10 bits each into one 12-byte record per vertex
 *           and lane, built at fdu_finalize: one load instead of nine 16-bit
 *           gathers, kept packed until each position is used (4: one round at
 *           a time, 5 waves per SIMD without spills; 5: the next round's loads
 *           issued before the current round is computed, 4 waves per SIMD).
 *           Variants 3, 4 and 5 sum the same terms in the same order (equal
 *           results bit for bit).
 * fdu_set_variants / fdu_get_variants select and report them (n_edge, n_vertex:
 * how many exist); a new solver starts with edge 1 and vertex 4.  fdu_autotune
 * times every edge variant and then every vertex variant on the given state
 * with fdu_kernel_times (reps launches each), writes the mean times (ms) to
 * times_ms[0 .. n_edge + n_vertex - 1] and keeps the fastest of each;
 * synchronous; w and scratch as for fdu_kernel_times. */
/* fdu_check_state: failure detection for long runs.  Counts the real rows of
 * w (device state, the solver's precision) that are not finite or not
 * physical (rho <= 0 or p <= 0), writes the count to *n_bad and the smallest
 * such row (library numbering) to *first_bad (-1 when none).  Runs on stream
 * and waits for it (not for use inside graph capture).  FDU_ERR_STATE before
 * fdu_finalize. */
fdu_status fdu_check_state(fdu_solver* s, const void* w, int64_t* n_bad, int64_t* first_bad, void* stream);

/* fdu_vertex_block_info: the vertex blocks built at fdu_finalize for the
 * LDS-staged vertex variants: their number, the total length of their row
 * lists (state rows + flux rows, with repeats across blocks) and the largest
 * list of one block (each row takes 32 bytes of LDS).  Any pointer may be
 * NULL.  FDU_ERR_STATE before fdu_finalize. */
fdu_status fdu_vertex_block_info(const fdu_solver* s, int* n_blocks, int64_t* halo_rows, int* rows_max);
fdu_status fdu_set_variants(fdu_solver* s, int edge_variant, int vertex_variant);
fdu_status fdu_get_variants(const fdu_solver* s, int* edge_variant, int* vertex_variant, int* n_edge, int* n_vertex);
fdu_status fdu_autotune(fdu_solver* s, void* w, void* scratch, int reps, double* times_ms, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FDU_H */
