"""Oracle: a plain, slow FP64 CPU implementation of the per-stage residual of the
unstructured-mesh finite-difference Euler scheme (Zhen, Qu, Cai, Sec. 2 and the
Appendix), used ONLY as test infrastructure.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU path
(``paper_2102_12933_amd``); the only common module is the seeded input
generator ``paper_2102_12933_amd.inputs`` (meshes and initial states, none of
the scheme's arithmetic).

Layout:
  geometry.py  adjacency, minimum image, 1D curvilinear stencils (Sec. 2.3.1),
               Catmull-Rom arc-length coordinates (Sec. 2.3.1, curve stencil figure)
  lsq.py       divergence stencils (Sec. 2.2.2) and least-squares weights (Sec. 2.2.1)
  nuweno.py    non-uniform WENO5 interpolation (Appendix, eqs. A1-A3, C_k, beta_k, omega_k)
  euler.py     Euler fluxes (Sec. 2.1), characteristic basis, Roe flux
  solver.py    residual, ghost fill, CFL time step, SSP-RK3 (Sec. 3), autograd VJP

Parity status of each function is stated in its docstring.  Readings of points
the paper leaves open are stated where they are used.  Functions whose result
depends on such a reading and that no paper-fixed fact pins are marked
"parity unpinned": the Catmull-Rom tangent magnitudes and arc-length rule, the
Roe flux with Harten's entropy fix (the paper names no Riemann solver for its
scheme), and the mirror-ghost wall treatment (the paper has no walls).
"""
