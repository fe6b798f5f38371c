// Reverse-mode derivative of the facet term with respect to the own-side
// state, for the vector-Jacobian product of the residual.  Not in the paper;
// the function differentiated is facet_term (two-point flux of Sec. 4 and
// the matrix interface dissipation of Sec. 4.5) composed with node_from_u
// and node_powers.  One plain evaluation of the forward quantities followed
// by one backward sweep, instead of one dual-number pass per component.
#pragma once
#include <hip/hip_runtime.h>

#include "device_physics.hpp"

namespace sbp {

// E = exp_avg(a, b, ar, br) and its partial derivatives with respect to a
// and ar (b, br held fixed), on the same branch as exp_avg.
__device__ __forceinline__ void exp_avg_d(double a, double b, double ar, double br, const ExpAvgC<double> &C,
                                          double &E, double &dE_da, double &dE_dar) {
  const double s = a + b;
  const double eps = (a - b) * drcp(s);
  if (fabs(eps) <= 1e-2) {
    const double ia = drcp(a);
    const double dl = 0.5 * (b - a) * ia;
    // B(dl) = 1 + dl q(dl), q = sum_k bn[k] dl^k (Horner with derivative)
    double q = C.bn[8], qd = 0.0;
#pragma unroll
    for (int k = 7; k >= 0; --k) {
      qd = q + dl * qd;
      q = C.bn[k] + dl * q;
    }
    const double B = 1.0 + dl * q, dB = q + dl * qd;
    const double e2 = eps * eps;
    const double S = 1.0 + e2 * (C.c[0] + e2 * (C.c[1] + e2 * (C.c[2] + e2 * C.c[3])));
    const double dS = C.c[0] + e2 * (2.0 * C.c[1] + e2 * (3.0 * C.c[2] + e2 * 4.0 * C.c[3]));
    E = ar * ia * B * S;
    dE_dar = ia * B * S;
    const double ddl = -0.5 * b * ia * ia;
    const double de2 = 2.0 * eps * (2.0 * b / (s * s));
    dE_da = ar * (-ia * ia * B * S + ia * dB * ddl * S + ia * B * dS * de2);
    return;
  }
  const double dab = a - b;
  const double den = C.r * dab;
  E = (ar - br) / den;
  dE_dar = 1.0 / den;
  dE_da = -E / dab;
}

__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// out = d/du_k [mu . facet_term(node(u_k), v, a)]; k: node of u_k with powers,
// v: neighbour node with powers, a = B n (held fixed).
template <int D>
__device__ __forceinline__ void facet_grad_rev(const Node<D, double> &k, const Node<D, double> &v, const double *a,
                                               const double *mu, const GasC<double> &G, bool diss, double *out) {
  constexpr int NC = D + 2;
  // ---- forward: two-point flux
  const double P1k = k.P1, P1v = v.P1, P2k = k.P2, P2v = v.P2;
  double Ep, Ep_a, Ep_ar, Ez, Ez_a, Ez_ar;
  exp_avg_d(k.p, v.p, P2k, P2v, G.e2, Ep, Ep_a, Ep_ar);
  exp_avg_d(k.z1, v.z1, P1k, P1v, G.e1, Ez, Ez_a, Ez_ar);
  const double Dn = 0.5 * (P1k + P1v) * Ep;
  const double iD = drcp(Dn);
  double an = 0.0, Vav[D], Vav2 = 0.0, q2av = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    an += a[i] * 0.5 * (k.z1 * k.V[i] + v.z1 * v.V[i]);
    Vav[i] = 0.5 * (k.V[i] + v.V[i]);
    Vav2 += Vav[i] * Vav[i];
    q2av += 0.5 * (k.V[i] * k.V[i] + v.V[i] * v.V[i]);
  }
  const double mass = an * iD;
  const double pav = 0.5 * (k.p + v.p);
  const double X = G.ggm1 * 0.5 * (P2k + P2v) * Ez + Vav2 - 0.5 * q2av;
  // ---- backward: two-point flux
  const double muE = mu[NC - 1];
  double bmass = mu[0] + muE * X;
  double bpav = 0.0;
  double bV[D], bw[NC];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    bmass += mu[1 + j] * Vav[j];
    bpav += mu[1 + j] * a[j];
  }
  const double bX = muE * mass;
  double bP2 = bX * G.ggm1 * 0.5 * Ez;
  double bEz = bX * G.ggm1 * 0.5 * (P2k + P2v);
  const double ban = bmass * iD;
  double bDn = -bmass * mass * iD;
  double bz1 = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double bVav = mu[1 + i] * mass + 2.0 * Vav[i] * bX;
    bV[i] = 0.5 * bVav - 0.5 * bX * k.V[i] + ban * a[i] * 0.5 * k.z1;
    bz1 += ban * a[i] * 0.5 * k.V[i];
  }
  double bEp = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) bw[c] = 0.0;
  if (diss) {
    // ---- forward: matrix dissipation
    const double z1a = 0.5 * (k.z1 + v.z1);
    const double iz = 1.0 / z1a;
    const double rho_h = z1a * iD;
    double Vh[D], n[D], Vh2 = 0.0, B2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      Vh[i] = 0.5 * (k.z1 * k.V[i] + v.z1 * v.V[i]) * iz;
      Vh2 += Vh[i] * Vh[i];
      B2 += a[i] * a[i];
    }
    const double B = sqrt(B2), iB = 1.0 / B;
    double Vn = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      n[i] = a[i] * iB;
      Vn += Vh[i] * n[i];
    }
    const double theta = rho_h / (pav * Dn);
    const double eta = 1.0 / (z1a * Ez * Ep);
    const double ah = sqrt(G.g * pav / rho_h);
    const double Hh = ah * ah / G.gm1 + 0.5 * Vh2;
    double dw[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) dw[c] = k.w[c] - v.w[c];
    const double dwE = dw[NC - 1];
    double xdV = 0.0, ndV = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      xdV += Vh[i] * dw[1 + i];
      ndV += n[i] * dw[1 + i];
    }
    const double pm = dw[0] + xdV - ah * ndV + (Hh - ah * Vn) * dwE;
    const double pp = dw[0] + xdV + ah * ndV + (Hh + ah * Vn) * dwE;
    const double p0 = dw[0] + xdV + 0.5 * Vh2 * dwE;
    const double sa = theta / (2.0 * G.g);
    const double am = fabs(Vn - ah), ap = fabs(Vn + ah), a0 = fabs(Vn);
    const double cm = am * sa * pm, cp = ap * sa * pp, c0 = a0 * G.sfac * theta * p0;
    double q[D], tq[D], nq = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      q[i] = dw[1 + i] + dwE * Vh[i];
      nq += n[i] * q[i];
    }
    const double cs = a0 * eta;
    double VTq = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      tq[i] = q[i] - n[i] * nq;
      VTq += Vh[i] * tq[i];
    }
    // ---- backward: matrix dissipation, out += B/2 y
    const double hb = 0.5 * B;
    double by[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) by[c] = hb * mu[c];
    const double byE = by[NC - 1];
    double bcm = by[0] + byE * (Hh - ah * Vn);
    double bc0 = by[0] + byE * 0.5 * Vh2;
    double bcp = by[0] + byE * (Hh + ah * Vn);
    double bcs = byE * VTq;
    double bah = byE * Vn * (cp - cm);
    double bHh = byE * (cm + cp);
    double bVn = byE * ah * (cp - cm);
    double bVh2 = byE * 0.5 * c0;
    double bVh[D], btq[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double byi = by[1 + i];
      bcm += byi * (Vh[i] - ah * n[i]);
      bc0 += byi * Vh[i];
      bcp += byi * (Vh[i] + ah * n[i]);
      bcs += byi * tq[i];
      bah += byi * n[i] * (cp - cm);
      bVh[i] = byi * (cm + c0 + cp) + byE * cs * tq[i];
      btq[i] = cs * (byi + byE * Vh[i]);
    }
    // tq = q - n (n . q);  q = dw_V + dw_E Vh
    double bnq = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) bnq -= n[i] * btq[i];
    double bdw[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) bdw[c] = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double bq = btq[i] + n[i] * bnq;
      bdw[1 + i] += bq;
      bdw[NC - 1] += bq * Vh[i];
      bVh[i] += bq * dwE;
    }
    // cs = |Vn| eta;  c0 = |Vn| sfac theta p0;  c+- = |Vn +- ah| sa p+-
    const double s0 = sgn(Vn), sp = sgn(Vn + ah), sm = sgn(Vn - ah);
    const double beta_ = bcs * a0;
    bVn += bcs * eta * s0 + bc0 * G.sfac * theta * p0 * s0 + bcp * sp * sa * pp + bcm * sm * sa * pm;
    bah += bcp * sp * sa * pp - bcm * sm * sa * pm;
    double btheta = bc0 * a0 * G.sfac * p0;
    const double bsa = bcp * ap * pp + bcm * am * pm;
    const double bp0 = bc0 * a0 * G.sfac * theta;
    const double bpp = bcp * ap * sa;
    const double bpm = bcm * am * sa;
    btheta += bsa / (2.0 * G.g);
    // p0, p+, p-
    const double bxdV = bp0 + bpp + bpm;
    const double bndV = ah * (bpp - bpm);
    bdw[0] += bp0 + bpp + bpm;
    bVh2 += bp0 * 0.5 * dwE;
    bdw[NC - 1] += bp0 * 0.5 * Vh2 + bpp * (Hh + ah * Vn) + bpm * (Hh - ah * Vn);
    bah += bpp * (ndV + Vn * dwE) - bpm * (ndV + Vn * dwE);
    bHh += (bpp + bpm) * dwE;
    bVn += (bpp - bpm) * ah * dwE;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      bVh[i] += bxdV * dw[1 + i];
      bdw[1 + i] += bxdV * Vh[i] + bndV * n[i];
    }
    // Hh = ah^2/(g-1) + Vh2/2;  ah^2 = g pav / rho_h
    bah += bHh * 2.0 * ah / G.gm1;
    bVh2 += 0.5 * bHh;
    bpav += bah * G.g / (2.0 * ah * rho_h);
    double brho_h = -bah * ah / (2.0 * rho_h);
    // eta = 1/(z1a Ez Ep);  theta = rho_h / (pav Dn)
    double bz1a = -beta_ * eta * iz;
    bEz -= beta_ * eta / Ez;
    bEp -= beta_ * eta / Ep;
    brho_h += btheta / (pav * Dn);
    bpav -= btheta * theta / pav;
    bDn -= btheta * theta * iD;
    // Vn = Vh . n;  Vh2 = |Vh|^2;  Vh = {z1 V} / z1a
#pragma unroll
    for (int i = 0; i < D; ++i) {
      bVh[i] += bVn * n[i] + 2.0 * Vh[i] * bVh2;
      bz1 += bVh[i] * 0.5 * k.V[i] * iz;
      bV[i] += bVh[i] * 0.5 * k.z1 * iz;
      bz1a -= bVh[i] * Vh[i] * iz;
    }
    // rho_h = z1a / Dn;  z1a = (z1_k + z1_v)/2
    bz1a += brho_h * iD;
    bDn -= brho_h * rho_h * iD;
    bz1 += 0.5 * bz1a;
#pragma unroll
    for (int c = 0; c < NC; ++c) bw[c] = bdw[c];
  }
  // Dn = (P1_k + P1_v)/2 Ep;  Ep, Ez exponential averages
  double bP1 = bDn * 0.5 * Ep;
  bEp += bDn * 0.5 * (P1k + P1v);
  double bp = 0.5 * bpav + bEp * Ep_a;
  bP2 += bEp * Ep_ar;
  bz1 += bEz * Ez_a;
  bP1 += bEz * Ez_ar;
  // ---- backward through node_powers and node_from_u
  double blz1 = bP1 * G.r1 * P1k;
  double blp = bP2 * G.r2 * P2k;
  const double irho = drcp(k.rho);
  const double theta = k.p * irho;
  double q2 = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) q2 += k.V[i] * k.V[i];
  // w = z1 (wfirst theta - q2/2, V, -1)
  bz1 += bw[0] * (G.wfirst * theta - 0.5 * q2) - bw[NC - 1];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    bz1 += bw[1 + i] * k.V[i];
    bV[i] += bw[1 + i] * k.z1;
  }
  const double btheta = bw[0] * k.z1 * G.wfirst;
  double bq2 = -0.5 * bw[0] * k.z1;
  // z1 = exp(lz1), lz1 = lrho - lp + (lp - g lrho)/(alpha + gamma)
  blz1 += bz1 * k.z1;
  const double blrho = blz1 * (1.0 - G.g * G.inv_apg);
  blp += blz1 * (G.inv_apg - 1.0);
  double brho = blrho * irho - btheta * theta * irho;
  bp += blp / k.p + btheta * irho;
  // p = (gamma-1)(E - rho q2 / 2)
  out[NC - 1] = G.gm1 * bp;
  brho -= 0.5 * G.gm1 * q2 * bp;
  bq2 -= 0.5 * G.gm1 * k.rho * bp;
  // V = m / rho
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double bVi = bV[i] + 2.0 * k.V[i] * bq2;
    out[1 + i] = bVi * irho;
    brho -= bVi * k.V[i] * irho;
  }
  out[0] = brho;
}

}  // namespace sbp
