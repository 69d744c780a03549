// Adjoint (vector-Jacobian product) of the per-stage residual.
//
// Forward, per real vertex O (Sec. 2.2.1 differenced form):
//   R_O = -( sum_j [wf_Oj (f_j - f_O) + wg_Oj (g_j - g_O)] + sum_k we_Ok r_k )
//         + cx_O f_O + cy_O g_O,          c_O = sum_k we_Ok n_k,
// with f_j = f(w_j), g_j = g(w_j) and r_k the edge flux of edge k, a function
// of the six states of its stencil.  Given a cotangent Rbar on the real
// vertices, the adjoint is assembled without atomics from transposed maps:
//   rbar_k  = -sum_{O uses k} we_Ok Rbar_O                      (k_edge_cot)
//   slots   = (d r_k / d w_{stencil(k)})^T rbar_k, [ne][6][4]     (k_edge_vjp)
//   fbar_v  = -sum_{O uses v} wf_Ov Rbar_O + [v real] sf_v Rbar_v,
//   gbar_v  likewise, sf_v = sum_j wf_vj + cx_v,
//   wbar_v  = (df/dw)^T fbar_v + (dg/dw)^T gbar_v + sum of v's slots  (k_vertex_vjp)
//   ghosts  copy their mirror source: a ghost's cotangent goes to its source
//           with the same momentum signs; ghost rows end at zero  (k_ghost_vjp)
// The edge-flux reverse sweep is written out by hand: Riemann flux (Roe with
// Harten's fix, or Rusanov), back-projection, NU-WENO5 nonlinear weights,
// characteristic projection and the Roe-averaged frame they all depend on.
#pragma once

#include "kernels.hpp"

namespace fdu {

// a = R^T q (transpose of from_char at a fixed frame)
FDU_HD void from_char_T(const Frame& F, const double qb[4], double ab[4]) {
  ab[0] = qb[0] + qb[1] * (F.u - F.c * F.nx) + qb[2] * (F.v - F.c * F.ny) + qb[3] * (F.H - F.c * F.un);
  ab[1] = qb[0] + qb[1] * F.u + qb[2] * F.v + qb[3] * F.q2;
  ab[2] = -qb[1] * F.ny + qb[2] * F.nx + qb[3] * F.ut;
  ab[3] = qb[0] + qb[1] * (F.u + F.c * F.nx) + qb[2] * (F.v + F.c * F.ny) + qb[3] * (F.H + F.c * F.un);
}

// q += L^T o (transpose of to_char at a fixed frame)
FDU_HD void to_char_T_acc(const Frame& F, double gm1, const double ob[4], double qb[4]) {
  const double ic = recip<true>(F.c);
  const double b1 = gm1 * ic * ic, b2 = b1 * F.q2;
  const double coreb = 0.5 * ob[0] - ob[1] + 0.5 * ob[3];
  const double xb = 0.5 * (ob[0] - ob[3]) * ic;   // cotangent of (u_n rho - n.m)
  qb[0] += coreb * b2 + xb * F.un + ob[1] - ob[2] * F.ut;
  qb[1] += -coreb * b1 * F.u - xb * F.nx - ob[2] * F.ny;
  qb[2] += -coreb * b1 * F.v - xb * F.ny + ob[2] * F.nx;
  qb[3] += coreb * b1;
}

// Reverse of weno_eval: ub[m] += vb * d(value)/d(u[m]).
FDU_HD void weno_eval_T(const WenoGeom& G, const double u[5], double eps, int power, double vb,
                                            double ub[5]) {
  double ut[3], d1[3], d2[3], be[3], b[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double u0 = u[k], u1 = u[k + 1], u2 = u[k + 2];
    ut[k] = G.I[k][0] * u0 + G.I[k][1] * u1 + G.I[k][2] * u2;
    d1[k] = G.D1[k][0] * u0 + G.D1[k][1] * u1 + G.D1[k][2] * u2;
    d2[k] = G.D2[k][0] * u0 + G.D2[k][1] * u1 + G.D2[k][2] * u2;
    be[k] = d1[k] * d1[k] + (13.0 / 12.0) * d2[k] * d2[k] + eps;
    b[k] = power == 2 ? be[k] * be[k] : be[k];
  }
  const double n[3] = {G.C[0] * b[1] * b[2], G.C[1] * b[0] * b[2], G.C[2] * b[0] * b[1]};
  const double iS = 1.0 / (n[0] + n[1] + n[2]);
  const double value = (n[0] * ut[0] + n[1] * ut[1] + n[2] * ut[2]) * iS;
  double nb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) nb[k] = (ut[k] - value) * iS * vb;
  double bb[3];
  bb[0] = nb[1] * G.C[1] * b[2] + nb[2] * G.C[2] * b[1];
  bb[1] = nb[0] * G.C[0] * b[2] + nb[2] * G.C[2] * b[0];
  bb[2] = nb[0] * G.C[0] * b[1] + nb[1] * G.C[1] * b[0];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double betab = power == 2 ? bb[k] * 2.0 * be[k] : bb[k];
    const double d1b = betab * 2.0 * d1[k], d2b = betab * (13.0 / 6.0) * d2[k];
    const double utb = n[k] * iS * vb;
#pragma unroll
    for (int m = 0; m < 3; ++m) ub[k + m] += utb * G.I[k][m] + d1b * G.D1[k][m] + d2b * G.D2[k][m];
  }
}

// ---------------------------------------------------------------------------
// Reverse mode, written out by hand: every *_T function below takes the
// cotangent of a forward function's output and accumulates the cotangents of
// its inputs (the forward values are recomputed, nothing is stored).

// Cotangents of the characteristic frame's fields.
struct FrameBar {
  double u = 0.0, v = 0.0, H = 0.0, c = 0.0, un = 0.0, ut = 0.0, q2 = 0.0;
};

// Frame cotangents of o = to_char(F, q) for fixed q.
FDU_HD void to_char_frame_T(const Frame& F, double gm1, const double q[4], const double ob[4], FrameBar& Fb) {
  const double ic = recip<true>(F.c);
  const double b1 = gm1 * ic * ic;
  const double mv = F.u * q[1] + F.v * q[2];
  const double nm = F.nx * q[1] + F.ny * q[2];
  const double coreb = 0.5 * ob[0] - ob[1] + 0.5 * ob[3];   // core = b1 (q2 rho - u.m + rhoE)
  const double xb = 0.5 * (ob[0] - ob[3]);                  // x = (u_n rho - n.m) / c
  Fb.ut -= ob[2] * q[0];
  Fb.un += xb * ic * q[0];
  const double b1b = coreb * (F.q2 * q[0] - mv + q[3]);
  Fb.q2 += coreb * b1 * q[0];
  const double mvb = -coreb * b1;
  Fb.u += mvb * q[1];
  Fb.v += mvb * q[2];
  const double icb = xb * (F.un * q[0] - nm) + b1b * 2.0 * gm1 * ic;
  Fb.c -= icb * ic * ic;
}

// Frame cotangents of q = from_char(F, a) for fixed a.
FDU_HD void from_char_frame_T(const Frame& F, const double a[4], const double qb[4], FrameBar& Fb) {
  const double s = a[0] + a[3], d = a[3] - a[0];
  Fb.u += qb[1] * (s + a[1]);
  Fb.v += qb[2] * (s + a[1]);
  Fb.c += (qb[1] * F.nx + qb[2] * F.ny + qb[3] * F.un) * d;
  Fb.H += qb[3] * s;
  Fb.un += qb[3] * F.c * d;
  Fb.q2 += qb[3] * a[1];
  Fb.ut += qb[3] * a[2];
}

// One side of the Roe average: cotangents of its velocity (usb, vsb),
// enthalpy (Hsb) and sqrt(rho) (rsb) to the conservative state q.
// H_s = gamma E / rho - (gamma - 1) (u^2 + v^2) / 2.
FDU_HD void roe_side_T(const double q[4], double gm1, double usb, double vsb, double Hsb, double rsb, double qb[4]) {
  const double iq = recip<true>(q[0]);
  const double us = q[1] * iq, vs = q[2] * iq;
  const double gam = gm1 + 1.0;
  usb -= Hsb * gm1 * us;
  vsb -= Hsb * gm1 * vs;
  qb[0] += -Hsb * gam * q[3] * iq * iq - (usb * us + vsb * vs) * iq + rsb * 0.5 * recip<true>(root<true>(q[0]));
  qb[1] += usb * iq;
  qb[2] += vsb * iq;
  qb[3] += Hsb * gam * iq;
}

// Frame cotangents back to the two states the frame was averaged from.
FDU_HD void roe_frame_T(const Frame& F, const double a[4], const double b[4], double gm1, const FrameBar& Fb,
                        double ab[4], double bb[4]) {
  // derived fields: u_n, u_t, c, q2 -> (u, v, H)
  double Ub = Fb.u + Fb.un * F.nx - Fb.ut * F.ny;
  double Vb = Fb.v + Fb.un * F.ny + Fb.ut * F.nx;
  const double t = Fb.c * 0.5 * gm1 * recip<true>(F.c);   // c = sqrt(gm1 (H - q2))
  const double Hb = Fb.H + t;
  const double q2b = Fb.q2 - t;
  Ub += q2b * F.u;
  Vb += q2b * F.v;
  // (u, v, H) = (ra x_a + rb x_b) / (ra + rb)
  const double ra = root<true>(a[0]), rb = root<true>(b[0]), is = recip<true>(ra + rb);
  const double ia = recip<true>(a[0]), ib = recip<true>(b[0]);
  const double ua = a[1] * ia, va = a[2] * ia, ubs = b[1] * ib, vbs = b[2] * ib;
  const double Ha = (gm1 + 1.0) * a[3] * ia - 0.5 * gm1 * (ua * ua + va * va);
  const double Hbs = (gm1 + 1.0) * b[3] * ib - 0.5 * gm1 * (ubs * ubs + vbs * vbs);
  const double wa = ra * is, wb = rb * is;
  const double rab = (Ub * (ua - F.u) + Vb * (va - F.v) + Hb * (Ha - F.H)) * is;
  const double rbb = (Ub * (ubs - F.u) + Vb * (vbs - F.v) + Hb * (Hbs - F.H)) * is;
  roe_side_T(a, gm1, Ub * wa, Vb * wa, Hb * wa, rab, ab);
  roe_side_T(b, gm1, Ub * wb, Vb * wb, Hb * wb, rbb, bb);
}

// q cotangent of normal_flux(q): Fb on the flux, plus direct cotangents unb on
// u_n and pb on the pressure.
FDU_HD void normal_flux_T(const double q[4], double nx, double ny, double gm1, const double Fb[4], double unb,
                          double pb, double qb[4]) {
  const double ir = recip<true>(q[0]);
  const double u = q[1] * ir, v = q[2] * ir;
  const double p = gm1 * (q[3] - 0.5 * (q[1] * u + q[2] * v));
  const double un = u * nx + v * ny;
  unb += Fb[0] * q[0] + Fb[1] * q[1] + Fb[2] * q[2] + Fb[3] * (q[3] + p);
  pb += Fb[1] * nx + Fb[2] * ny + Fb[3] * un;
  qb[0] += Fb[0] * un - unb * un * ir + pb * gm1 * 0.5 * (u * u + v * v);
  qb[1] += Fb[1] * un + unb * nx * ir - pb * gm1 * u;
  qb[2] += Fb[2] * un + unb * ny * ir - pb * gm1 * v;
  qb[3] += Fb[3] * un + pb * gm1;
}

// Cotangents of the midpoint states (wl, wr) for the flux cotangent ob.
FDU_HD void riemann_flux_T(const double wl[4], const double wr[4], double nx, double ny, const Scheme& S,
                           const double ob[4], double wlb[4], double wrb[4]) {
  double hb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    hb[k] = 0.5 * ob[k];          // out = (Fl + Fr) / 2 - dissipation / 2
    wlb[k] = 0.0;
    wrb[k] = 0.0;
  }
  if (S.riemann == 1) {
    double Fl[4], Fr[4], unl, unr, c2l, c2r;
    normal_flux<double>(wl, nx, ny, S.gm1, Fl, unl, c2l);
    normal_flux<double>(wr, nx, ny, S.gm1, Fr, unr, c2r);
    const double cl = root<true>(c2l), cr = root<true>(c2r);
    const double sl = ::fabs(unl) + cl, sr = ::fabs(unr) + cr;
    const bool left = sl >= sr;
    const double sm = left ? sl : sr;
    double smb = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      smb -= 0.5 * ob[k] * (wr[k] - wl[k]);
      wlb[k] += 0.5 * sm * ob[k];
      wrb[k] -= 0.5 * sm * ob[k];
    }
    // s = |u_n| + sqrt(gamma p / rho) of the side that gave the maximum
    const double* q = left ? wl : wr;
    const double un = left ? unl : unr, c = left ? cl : cr, c2 = left ? c2l : c2r;
    const double zero[4] = {0.0, 0.0, 0.0, 0.0};
    const double c2b = smb * 0.5 * recip<true>(c);
    double qb[4] = {-c2b * c2 * recip<true>(q[0]), 0.0, 0.0, 0.0};
    normal_flux_T(q, nx, ny, S.gm1, zero, smb * (un < 0.0 ? -1.0 : 1.0), c2b * (S.gm1 + 1.0) * recip<true>(q[0]), qb);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (left) wlb[k] += qb[k]; else wrb[k] += qb[k];
    }
    normal_flux_T(wl, nx, ny, S.gm1, hb, 0.0, 0.0, wlb);
    normal_flux_T(wr, nx, ny, S.gm1, hb, 0.0, 0.0, wrb);
    return;
  }
  // Roe with Harten's fix: dissipation = from_char(F, h * to_char(F, wr - wl))
  const Frame F = roe_frame<double, true>(wl, wr, nx, ny, S.gm1);
  double dq[4], a[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) dq[k] = wr[k] - wl[k];
  to_char(F, S.gm1, dq, a);
  const double delta = S.efrac * F.c;
  const double lam[4] = {F.un - F.c, F.un, F.un, F.un + F.c};
  double h[4], ap[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    h[k] = harten<double>(lam[k], delta);
    ap[k] = a[k] * h[k];
  }
  double db[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) db[k] = -0.5 * ob[k];
  FrameBar Fb;
  double apb[4];
  from_char_T(F, db, apb);
  from_char_frame_T(F, ap, db, Fb);
  double ab[4], deltab = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ab[k] = apb[k] * h[k];
    const double hk = apb[k] * a[k];
    const double l = lam[k];
    double lb;
    if (::fabs(l) < delta) {         // h = (l^2 + delta^2) / (2 delta)
      lb = hk * l * recip<true>(delta);
      deltab += hk * (delta * delta - l * l) * recip<true>(2.0 * delta * delta);
    } else {                         // h = |l|
      lb = l < 0.0 ? -hk : hk;
    }
    Fb.un += lb;
    if (k == 0) Fb.c -= lb;
    if (k == 3) Fb.c += lb;
  }
  Fb.c += S.efrac * deltab;
  double dqb[4] = {0.0, 0.0, 0.0, 0.0};
  to_char_T_acc(F, S.gm1, ab, dqb);
  to_char_frame_T(F, S.gm1, dq, ab, Fb);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    wrb[k] += dqb[k];
    wlb[k] -= dqb[k];
  }
  roe_frame_T(F, wl, wr, S.gm1, Fb, wlb, wrb);
  normal_flux_T(wl, nx, ny, S.gm1, hb, 0.0, 0.0, wlb);
  normal_flux_T(wr, nx, ny, S.gm1, hb, 0.0, 0.0, wrb);
}

// Cotangents of the six stencil states of one edge for the flux cotangent ob
// (the reverse of edge_flux_one).  load(s, q, again) writes stencil state s
// to q; it is called a second time (again = true) near the end instead of
// keeping the states live.  store(s, q) receives the cotangent of state s.
template <class Load, class Store>
FDU_HD void edge_vjp_one(Load&& load, const double g[6], const double ob[4], const Scheme& S, Store&& store) {
  const double nx = g[4], ny = g[5];
  const bool cons = S.conservative != 0;
  double x[4];
  weno_nodes(g, S, x);
  // ---- forward recomputation
  double W2[4], W3[4];
  load(2, W2, false);
  load(3, W3, false);
  const Frame F = roe_frame<double, true>(W2, W3, nx, ny, S.gm1);
  double Cv[6][4];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double q[4];
    if (k == 2 || k == 3) {
#pragma unroll
      for (int i = 0; i < 4; ++i) q[i] = k == 2 ? W2[i] : W3[i];
    } else {
      load(k, q, false);
    }
    if (cons) {
#pragma unroll
      for (int i = 0; i < 4; ++i) Cv[k][i] = q[i];
    } else {
      to_char(F, S.gm1, q, Cv[k]);
    }
  }
  double cl[4], cr[4];
  {
    WenoGeom G;
    weno_geom(x[0], x[1], x[2], G);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double u[5] = {Cv[0][c], Cv[1][c], Cv[2][c], Cv[3][c], Cv[4][c]};
      cl[c] = weno_eval(G, u, S.eps, S.power);
    }
  }
  {
    WenoGeom G;
    weno_geom(-x[3], -x[2], -x[1], G);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double u[5] = {Cv[5][c], Cv[4][c], Cv[3][c], Cv[2][c], Cv[1][c]};
      cr[c] = weno_eval(G, u, S.eps, S.power);
    }
  }
  double wl[4], wr[4];
  if (cons) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      wl[k] = cl[k];
      wr[k] = cr[k];
    }
  } else {
    from_char(F, cl, wl);
    from_char(F, cr, wr);
  }
  bool fl = false, fr = false;
  if (S.positivity) {
    fl = !physical(wl, S.gm1);
    fr = !physical(wr, S.gm1);
    if (fl)
#pragma unroll
      for (int k = 0; k < 4; ++k) wl[k] = W2[k];
    if (fr)
#pragma unroll
      for (int k = 0; k < 4; ++k) wr[k] = W3[k];
  }

  // ---- Riemann flux
  double wlb[4], wrb[4];
  riemann_flux_T(wl, wr, nx, ny, S, ob, wlb, wrb);
  // ---- back-projection (or the fallback's copy of the end state)
  FrameBar Fb;
  double clb[4] = {0.0, 0.0, 0.0, 0.0}, crb[4] = {0.0, 0.0, 0.0, 0.0};
  double e2[4] = {0.0, 0.0, 0.0, 0.0}, e3[4] = {0.0, 0.0, 0.0, 0.0};   // direct cotangents of W2, W3
  if (fl) {
#pragma unroll
    for (int k = 0; k < 4; ++k) e2[k] = wlb[k];
  } else if (cons) {
#pragma unroll
    for (int k = 0; k < 4; ++k) clb[k] = wlb[k];
  } else {
    from_char_T(F, wlb, clb);
    from_char_frame_T(F, cl, wlb, Fb);
  }
  if (fr) {
#pragma unroll
    for (int k = 0; k < 4; ++k) e3[k] = wrb[k];
  } else if (cons) {
#pragma unroll
    for (int k = 0; k < 4; ++k) crb[k] = wrb[k];
  } else {
    from_char_T(F, wrb, crb);
    from_char_frame_T(F, cr, wrb, Fb);
  }
  // ---- NU-WENO5 along the stencil, one side at a time (geometry recomputed)
  double Cb[6][4];
#pragma unroll
  for (int s = 0; s < 6; ++s)
#pragma unroll
    for (int k = 0; k < 4; ++k) Cb[s][k] = 0.0;
  {
    WenoGeom G;
    weno_geom(opaque(x[0]), opaque(x[1]), opaque(x[2]), G);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double u[5] = {Cv[0][c], Cv[1][c], Cv[2][c], Cv[3][c], Cv[4][c]};
      double ub[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      weno_eval_T(G, u, S.eps, S.power, clb[c], ub);
#pragma unroll
      for (int m = 0; m < 5; ++m) Cb[m][c] += ub[m];
    }
  }
  {
    WenoGeom G;
    weno_geom(-opaque(x[3]), -opaque(x[2]), -opaque(x[1]), G);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double u[5] = {Cv[5][c], Cv[4][c], Cv[3][c], Cv[2][c], Cv[1][c]};
      double ub[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      weno_eval_T(G, u, S.eps, S.power, crb[c], ub);
#pragma unroll
      for (int m = 0; m < 5; ++m) Cb[5 - m][c] += ub[m];
    }
  }
  if (cons) {
    // interpolated variables are the states themselves
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      double wb[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) wb[k] = Cb[s][k] + (s == 2 ? e2[k] : 0.0) + (s == 3 ? e3[k] : 0.0);
      store(s, wb);
    }
    return;
  }
  // ---- characteristic projection: frame cotangents first (they need the
  // states, loaded again), then the states at the fixed frame
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    double q[4];
    load(s, q, true);
    to_char_frame_T(F, S.gm1, q, Cb[s], Fb);
  }
  {
    double q2[4], q3[4];
    load(2, q2, true);
    load(3, q3, true);
    roe_frame_T(F, q2, q3, S.gm1, Fb, e2, e3);
  }
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    double wb[4] = {0.0, 0.0, 0.0, 0.0};
    if (s == 2) {
#pragma unroll
      for (int k = 0; k < 4; ++k) wb[k] = e2[k];
    }
    if (s == 3) {
#pragma unroll
      for (int k = 0; k < 4; ++k) wb[k] = e3[k];
    }
    to_char_T_acc(F, S.gm1, Cb[s], wb);
    store(s, wb);
  }
}

// rbar_k = -sum_{O uses k} we_Ok Rbar_O (transposed edge CSR); LPV lanes per
// edge take strided shares of its ~44 entries and a butterfly sums them.
template <class T, class TW, int LPV>
__global__ void __launch_bounds__(256) k_edge_cot(const int* __restrict__ tptr, const int* __restrict__ trow,
                                                  const TW* __restrict__ tw, const T* __restrict__ Rbar,
                                                  double* __restrict__ rbar, int ne) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = t / LPV, lane = t % LPV;
  const bool active = k < ne;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  if (active) {
    // the first NS entries of each lane: indices, weights and rows requested
    // together (slots past the list read entry 0 and are not used), then the
    // rest one by one; the per-lane order of the sum is the list order
    constexpr int NS = 2;
    const int pb = tptr[k], pe = tptr[k + 1];
    int row[NS];
    double c[NS], q[NS][4];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int p = pb + lane + s * LPV;
      const int pc = p < pe ? p : 0;
      row[s] = trow[pc];
      c[s] = (double)tw[pc];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) load4(Rbar, row[s], q[s]);
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (pb + lane + s * LPV < pe)
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] -= c[s] * q[s][i];
    for (int p = pb + lane + NS * LPV; p < pe; p += LPV) {
      double qq[4];
      load4(Rbar, trow[p], qq);
      const double cc = (double)tw[p];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] -= cc * qq[i];
    }
  }
#pragma unroll
  for (int m = LPV / 2; m >= 1; m >>= 1)
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] += __shfl_xor(a[i], m, LPV);
  if (!active || lane != 0) return;
  double2* o = reinterpret_cast<double2*>(rbar + 4 * (size_t)k);
  o[0] = make_double2(a[0], a[1]);
  o[1] = make_double2(a[2], a[3]);
}

// Per flux edge: cotangents of its six stencil states, slots[e][s][4].
template <class T, class TG>
__global__ void __launch_bounds__(256, 2) k_edge_vjp(const T* __restrict__ w, const int* __restrict__ sten,
                                                  const TG* __restrict__ geo, const double* __restrict__ rbar,
                                                  double* __restrict__ slots, int ne, Scheme S) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int id[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) id[k] = sten[6 * (size_t)e + k];
  double g[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = (double)geo[6 * (size_t)e + k];
  double ob[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) ob[k] = rbar[4 * (size_t)e + k];
  double* out = slots + 24 * (size_t)e;
  edge_vjp_one([&](int s, double q[4], bool again) { load4(w, again ? opaque(id[s]) : id[s], q); }, g, ob, S,
               [&](int s, const double q[4]) {
                 double2* o = reinterpret_cast<double2*>(out + 4 * s);
                 o[0] = make_double2(q[0], q[1]);
                 o[1] = make_double2(q[2], q[3]);
               });
}

// Per vertex (real and ghost): flux-cotangent gathers over the transposed
// vertex CSR, the flux Jacobian transposes, and the edge slots that read it.
// LPV lanes per vertex share both gather loops; a butterfly sums them.
template <class T, class TW, int LPV>
__global__ void __launch_bounds__(256) k_vertex_vjp(const T* __restrict__ w, const T* __restrict__ Rbar,
                                                    const int* __restrict__ tptr, const int* __restrict__ trow,
                                                    const TW* __restrict__ twfg, const double* __restrict__ sfg,
                                                    const int* __restrict__ sptr, const int* __restrict__ scol,
                                                    const double* __restrict__ slots, int nreal, int nv,
                                                    double gm1, double* __restrict__ tmp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = t / LPV, lane = t % LPV;
  const bool active = v < nv;
  double fb[4] = {0.0, 0.0, 0.0, 0.0}, gb[4] = {0.0, 0.0, 0.0, 0.0}, sl[4] = {0.0, 0.0, 0.0, 0.0};
  if (active) {
    // as in k_edge_cot: the first NS entries of each lane's share of both
    // lists requested together, the rest one by one, list order per lane
    constexpr int NS = 3;
    const int pb = tptr[v], pe = tptr[v + 1], qb = sptr[v], qe = sptr[v + 1];
    int row[NS], col[NS];
    double a[NS], b[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int p = pb + lane + s * LPV, pc = p < pe ? p : 0;
      row[s] = trow[pc];
      a[s] = (double)twfg[2 * (size_t)pc];
      b[s] = (double)twfg[2 * (size_t)pc + 1];
      const int r = qb + lane + s * LPV;
      col[s] = scol[r < qe ? r : 0];
    }
    double q[NS][4], x[NS][4];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      load4(Rbar, row[s], q[s]);
      const double2* sp = reinterpret_cast<const double2*>(slots + 4 * (size_t)col[s]);
      const double2 x0 = sp[0], x1 = sp[1];
      x[s][0] = x0.x; x[s][1] = x0.y; x[s][2] = x1.x; x[s][3] = x1.y;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (pb + lane + s * LPV < pe)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          fb[i] -= a[s] * q[s][i];
          gb[i] -= b[s] * q[s][i];
        }
    for (int p = pb + lane + NS * LPV; p < pe; p += LPV) {
      double qq[4];
      load4(Rbar, trow[p], qq);
      const double aa = (double)twfg[2 * (size_t)p], bb = (double)twfg[2 * (size_t)p + 1];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        fb[i] -= aa * qq[i];
        gb[i] -= bb * qq[i];
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (qb + lane + s * LPV < qe) {
        sl[0] += x[s][0]; sl[1] += x[s][1]; sl[2] += x[s][2]; sl[3] += x[s][3];
      }
    for (int p = qb + lane + NS * LPV; p < qe; p += LPV) {
      const double2* sp = reinterpret_cast<const double2*>(slots + 4 * (size_t)scol[p]);
      const double2 x0 = sp[0], x1 = sp[1];
      sl[0] += x0.x; sl[1] += x0.y; sl[2] += x1.x; sl[3] += x1.y;
    }
  }
#pragma unroll
  for (int m = LPV / 2; m >= 1; m >>= 1)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      fb[i] += __shfl_xor(fb[i], m, LPV);
      gb[i] += __shfl_xor(gb[i], m, LPV);
      sl[i] += __shfl_xor(sl[i], m, LPV);
    }
  if (!active || lane != 0) return;
  if (v < nreal) {
    double q[4];
    load4(Rbar, v, q);
    const double a = sfg[2 * (size_t)v], b = sfg[2 * (size_t)v + 1];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      fb[i] += a * q[i];
      gb[i] += b * q[i];
    }
  }
  double wb[4] = {0.0, 0.0, 0.0, 0.0};
  {
    double q0[4];
    load4(w, v, q0);
    Dual<4> q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      q[k] = Dual<4>(q0[k]);
      q[k].d[k] = 1.0;
    }
    const Dual<4> ir = 1.0 / q[0];
    const Dual<4> u = q[1] * ir, vv = q[2] * ir;
    const Dual<4> p = gm1 * (q[3] - 0.5 * (q[1] * u + q[2] * vv));
    const Dual<4> f[4] = {q[1], q[1] * u + p, q[1] * vv, (q[3] + p) * u};
    const Dual<4> g[4] = {q[2], q[2] * u, q[2] * vv + p, (q[3] + p) * vv};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double t2 = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) t2 += fb[i] * f[i].d[k] + gb[i] * g[i].d[k];
      wb[k] = t2 + sl[k];
    }
  }
  double2* o = reinterpret_cast<double2*>(tmp + 4 * (size_t)v);
  o[0] = make_double2(wb[0], wb[1]);
  o[1] = make_double2(wb[2], wb[3]);
}

// Real rows: own cotangent plus those of the ghosts copied from them (with the
// ghost's momentum signs); ghost rows: zero.  out = alpha * result + beta * add
// (add may be null), the form the Runge-Kutta stage adjoint needs.
template <class T>
__global__ void __launch_bounds__(256) k_ghost_vjp(const double* __restrict__ tmp, const int* __restrict__ gptr,
                                                   const int* __restrict__ gcol, const signed char* __restrict__ refl,
                                                   int nreal, int nv, double alpha, const T* __restrict__ add,
                                                   double beta, T* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  if (v < nreal) {
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = tmp[4 * (size_t)v + k];
    for (int p = gptr[v]; p < gptr[v + 1]; ++p) {
      const int gi = gcol[p];
      const double* t = tmp + 4 * (size_t)(nreal + gi);
      const int f = refl[gi];
      a[0] += t[0];
      a[1] += (f & 1) ? -t[1] : t[1];
      a[2] += (f & 2) ? -t[2] : t[2];
      a[3] += t[3];
    }
  }
  double r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = alpha * a[k];
  if (add != nullptr && v < nreal) {
    double q[4];
    load4(add, v, q);
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] += beta * q[k];
  }
  store4(out, v, r);
}

// out[v] += a * x[v] on the real rows (ghost rows untouched)
template <class T>
__global__ void __launch_bounds__(256) k_axpy_real(T* __restrict__ out, double a, const T* __restrict__ x, int nreal) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nreal) return;
  double q[4], o[4];
  load4(x, v, q);
  load4(out, v, o);
#pragma unroll
  for (int k = 0; k < 4; ++k) o[k] += a * q[k];
  store4(out, v, o);
}

// out[v] = a * x[v] on all rows
// *p := x (one value; launched with one wave).
__global__ void k_set_value(double* __restrict__ p, double x) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = x;
}

template <class T>
__global__ void __launch_bounds__(256) k_scale(T* __restrict__ out, double a, const T* __restrict__ x, int nv) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double q[4];
  load4(x, v, q);
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] *= a;
  store4(out, v, q);
}

}  // namespace fdu
