// Vector-Jacobian product ubar = (dr/du)^T lambda of the entropy-split
// residual (Euler terms, optional interface dissipation), FP64.  Not part of
// the paper; derived by differentiating Sec. 6.2 eq. weak form split.
//
// For element k with mu = H^-1 lambda, w = w(u), g_i = D_xi w:
//   volume     d/du [H^-1 sum_l M_l fhat_l]^T lambda = sum_l sum_i Lambda_il A_i^T (M_l^T mu)
//   non-cons.  d/du [-c_b sum_i A~_i(w) g_i]^T lambda
//                = -c_b (dW/dU) [ sum_i D_xi^T (A~_i lambda) + sum_i d/de A~_i(w + e g_i) lambda ]
//              (A~_i and dW/dU symmetric; the last term is a Hessian-vector
//               product, evaluated with dual numbers)
//   facets     each facet node receives the derivative of its own SAT and of
//              the matching neighbour's SAT with respect to its own state;
//              the neighbour's SAT is the negative of its own (antisymmetric
//              two-point flux and dissipation, opposite B n), so both are one
//              gradient of Phi(u_k, u_v) with cotangent lambda_k/H_k -
//              lambda_v/H_v (reverse mode, facet_adjoint.hpp), gathered
//              without atomics.
// The transposed operators enter as per-node-pair sums over the reference
// skew operators S_l (Q_l = S_l + E_l/2), as in the forward row-form kernels.
//
// On curved triangles the physical operators are written with the skew parts
// K_i = 1/2 sum_l (Lambda_il S_l + S_l Lambda_il) and a_i = sum_l Lambda_il E_l:
//   Q_xi = K_i + a_i/2,  Q_xi^T = -K_i + a_i/2,
//   M_xi^T mu = (1 - c_b) K_i mu + (1 + c_b)/2 a_i mu,
// so only the reference skew operators S_l enter, as per-node-pair sums.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dual.hpp"
#include "facet_adjoint.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace sbp {

namespace {

constexpr int kT = 256;

// (dW/dU) y as the derivative of w(u + e y)
template <int D>
__device__ __forceinline__ void dWdU_apply(const double *u, const double *y, const GasC<Dual<double>> &G, double *out) {
  constexpr int NC = D + 2;
  Dual<double> x[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) x[q] = Dual<double>(u[q], y[q]);
  Node<D, Dual<double>> n;
  node_from_u<D, Dual<double>>(x, G, n);
#pragma unroll
  for (int q = 0; q < NC; ++q) out[q] = n.w[q].d;
}

// 3D affine tetrahedra, row form: one lane per node row; per node pair (i, j)
//   Z_l += S_l[i][j] mu_j,  V_s += sum_l S_l[i][j] shat_l,j,  G_l += S_l[i][j] w_j
// (45 FMAs per pair; shat_l = s_l / h), then per node
//   M_l^T mu = (1 - c_b) Z_l + (1 + c_b)/2 E_l mu,
//   sum_l D_l^T s_l = -V_s + 1/2 sum_l E_l shat_l,   D_l w = h^-1 (G_l + E_l w / 2).
// At p = 3 (60 x 60 operators) S_l is read through the caches, as in the
// forward kernel.
template <int P> struct VTileV3 { static constexpr int EB = P == 1 ? 21 : (P == 2 ? 10 : 4); };

// W: waves per SIMD the register budget allows (1: up to 512 registers,
// 2: 256).  The built-in choice is W = 2 except at p = 1, where the cap
// spills (measured on MI355X, 196608 tetrahedra: with the cap p = 3 takes
// 5.04 instead of 5.77 ms, p = 1 0.87 instead of 0.60 ms).
template <int P> constexpr int vjp3_waves() { return P == 1 ? 1 : 2; }

template <int P, int W>
__global__ __launch_bounds__(kT, W) void k_vjp3v(KArgs<double> A) {
  constexpr int D = 3, NC = 5, NFAC = 4;
  constexpr int NP = Shape<3, P>::NP, NF = Shape<3, P>::NF, NFN = NFAC * NF;
  constexpr int EB = VTileV3<P>::EB;
  constexpr bool SG = P == 3;
  static_assert(EB * NP <= kT, "one node per lane");
  constexpr int NDS = NP * 25 + 4;  // per node: mu[5] shat_1..3[15] w[5]
  __shared__ double Ss[SG ? 1 : 3][SG ? 1 : NP][SG ? 1 : NP];
  __shared__ double nd[EB * NDS];
  __shared__ double gs[EB][10];
  const int tid = threadIdx.x;
  if constexpr (!SG)
    for (int x = tid; x < 3 * NP * NP; x += kT) (&Ss[0][0][0])[x] = A.op.S[x];
  const GasC<double> &G = A.G;
  const GasC<Dual<double>> GD = dual_gas(G);
  const double cb = G.cb, he = 0.5 * (1.0 + cb), hz = 1.0 - cb;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  const int e = tid / NP, i = tid % NP;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    if (!tile_on(A, e0, ne)) continue;  // hybrid scheme: no element of this form
    const int eg = e0 + e;
    const bool act = tid < ne * NP && elem_on(A, eg);
    __syncthreads();
    for (int x = tid; x < ne * 10; x += kT) gs[x / 10][x % 10] = A.geo[(size_t)(e0 + x / 10) * 10 + x % 10];
    __syncthreads();
    Node<D, double> n;
    const double *Lam = gs[act ? e : 0];
    const double J = Lam[9], iJ = drcp(J);
    const double h = A.op.h[i], ih = drcp(h), iH = iJ * ih;
    if (act) {
      double uu[NC], lm[NC];
      const int uo = A.uoff[eg];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        uu[c] = A.u[uo + c * NP + i];
        lm[c] = A.lam[uo + c * NP + i];
      }
      node_from_u<D, double>(uu, G, n);
      if (!n.ok) atomicOr(A.err, 1);
      double t[D][NC];
#pragma unroll
      for (int m = 0; m < D; ++m) jvp_flux<D, double>(n, G, m, lm, t[m]);
      double *v = nd + e * NDS + i * 25;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        v[c] = lm[c] * iH;
        v[20 + c] = n.w[c];
      }
#pragma unroll
      for (int l = 0; l < D; ++l)
#pragma unroll
        for (int c = 0; c < NC; ++c)
          v[5 + l * NC + c] = (Lam[0 * 3 + l] * t[0][c] + Lam[1 * 3 + l] * t[1][c] + Lam[2 * 3 + l] * t[2][c]) * iH;
    }
    __syncthreads();
    if (act) {
      double Z[D][NC], Vs[NC], Gw[D][NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        Vs[c] = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) Z[l][c] = Gw[l][c] = 0.0;
      }
#pragma unroll (P >= 3 ? 2 : 1)
      for (int j = 0; j < NP; ++j) {
        double s0, s1, s2;
        if constexpr (SG) {
          // row-wise reads: measured faster here than the transposed reads of
          // the forward kernels (196608 tetrahedra, p = 3: 4.96 against 5.13 ms)
          s0 = A.op.S[(0 * NP + i) * NP + j];
          s1 = A.op.S[(1 * NP + i) * NP + j];
          s2 = A.op.S[(2 * NP + i) * NP + j];
        } else {
          s0 = Ss[0][i][j];
          s1 = Ss[1][i][j];
          s2 = Ss[2][i][j];
        }
        const double *v = nd + e * NDS + j * 25;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          Z[0][c] += s0 * v[c];
          Z[1][c] += s1 * v[c];
          Z[2][c] += s2 * v[c];
          Vs[c] += s0 * v[5 + c];  // one FMA per product
          Vs[c] += s1 * v[10 + c];
          Vs[c] += s2 * v[15 + c];
          Gw[0][c] += s0 * v[20 + c];
          Gw[1][c] += s1 * v[20 + c];
          Gw[2][c] += s2 * v[20 + c];
        }
      }
      // this node's state and cotangent: re-read after the pair loop (from
      // L1/L2) rather than held in registers across it
      const int uo = A.uoff[eg];
      double uu[NC], lm[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        uu[c] = A.u[uo + c * NP + i];
        lm[c] = A.lam[uo + c * NP + i];
      }
      const double *v = nd + e * NDS + i * 25;
      double El[D], ak[D];
#pragma unroll
      for (int l = 0; l < D; ++l) El[l] = A.op.E[l * NP + i];
#pragma unroll
      for (int m = 0; m < D; ++m) ak[m] = Lam[m * 3 + 0] * El[0] + Lam[m * 3 + 1] * El[1] + Lam[m * 3 + 2] * El[2];
      double ub[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] = 0.0;
      // volume: sum_m A_m^T sum_l Lambda_ml (M_l^T mu)
#pragma unroll
      for (int l = 0; l < D; ++l)
#pragma unroll
        for (int c = 0; c < NC; ++c) Z[l][c] = hz * Z[l][c] + he * El[l] * v[c];
#pragma unroll
      for (int m = 0; m < D; ++m) {
        double zm[NC], o[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) zm[c] = Lam[m * 3 + 0] * Z[0][c] + Lam[m * 3 + 1] * Z[1][c] + Lam[m * 3 + 2] * Z[2][c];
        flux_jac_T<D, double>(n, G, uu[NC - 1], m, zm, o);
#pragma unroll
        for (int c = 0; c < NC; ++c) ub[c] += o[c];
      }
      // non-conservative: y = sum_l D_l^T s_l + sum_m d/de A~_m(w + e g_m) lambda,
      // s_l = J^-1 sum_m Lambda_ml A~_m lambda, g_m = J^-1 sum_l Lambda_ml D_l w
      double y[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) y[c] = -Vs[c] + 0.5 * (El[0] * v[5 + c] + El[1] * v[10 + c] + El[2] * v[15 + c]);
#pragma unroll
      for (int l = 0; l < D; ++l)
#pragma unroll
        for (int c = 0; c < NC; ++c) Gw[l][c] = (Gw[l][c] + 0.5 * El[l] * n.w[c]) * ih;
#pragma unroll
      for (int m = 0; m < D; ++m) {
        double gm[NC], du[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
          gm[c] = (Lam[m * 3 + 0] * Gw[0][c] + Lam[m * 3 + 1] * Gw[1][c] + Lam[m * 3 + 2] * Gw[2][c]) * iJ;
        dU_from_dW<D, double>(n, G, gm, du);
        Dual<double> xd[NC], lmd[NC], hv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          xd[c] = Dual<double>(uu[c], du[c]);
          lmd[c] = Dual<double>(lm[c]);
        }
        Node<D, Dual<double>> ndu;
        node_from_u<D, Dual<double>>(xd, GD, ndu);
        jvp_flux<D, Dual<double>>(ndu, GD, m, lmd, hv);
#pragma unroll
        for (int c = 0; c < NC; ++c) y[c] += hv[c].d;
      }
      double wy[NC];
      dWdU_apply<D>(uu, y, GD, wy);
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] -= cb * wy[c];
      // facet SATs: one gradient of this node's SAT with the combined
      // cotangent lambda_k/H_k - lambda_v/H_v (the neighbour's SAT is its negative)
      if (i < NFN) {
        const int off = A.nbr[(size_t)eg * NFN + i];
        double uv[NC], lv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          uv[c] = A.u[off + c * NP];
          lv[c] = A.lam[off + c * NP];
        }
        const int q = A.nbrq[(size_t)eg * NFN + i];
        const double Hv = A.Hn[(size_t)(q / NFN) * NP + q % NFN];
        double mu[NC], g1[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) mu[c] = v[c] - lv[c] / Hv;
        Node<D, double> nk = n, nv;
        node_powers<D, double>(G, nk);
        node_from_u<D, double>(uv, G, nv);
        node_powers<D, double>(G, nv);
        facet_grad_rev<D>(nk, nv, ak, mu, G, A.diss != 0, g1);
#pragma unroll
        for (int c = 0; c < NC; ++c) ub[c] -= g1[c];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) A.ubar[uo + c * NP + i] = ub[c];
    }
  }
}

// 2D curved triangles, row form (as the forward 2D kernel): one lane per node
// row; per node pair (i, j), with c_m = sum_l S_l[i][j] (Lambda_ml(i) + Lambda_ml(j)),
//   Z_m += c_m mu_j,  V_s += c_0 s_0,j + c_1 s_1,j,  X_m += c_m w_j
// (Z_m = 2 K_m mu, V_s = 2 sum_m K_m s_m, X_m = 2 K_m w), then the pointwise
// transposed-Jacobian, Hessian-vector and facet-derivative terms per node.
template <int P> struct VTileV2 { static constexpr int EB = P == 1 ? 42 : (P == 2 ? 25 : (P == 3 ? 14 : 11)); };

template <int P>
struct Vjp2 {
  static constexpr int D = 2, NC = 4, NFAC = 3;
  static constexpr int NP = Shape<2, P>::NP, NF = Shape<2, P>::NF, NFN = NFAC * NF;
  static constexpr int EB = VTileV2<P>::EB;
  static_assert(EB * NP <= kT, "one node per lane");
  static constexpr int NDS = NP * 20 + 4;  // padded element blocks (LDS banks)
  // S[k][j] = (S_0[j][k], S_1[j][k]): a row's two entries in one read, the
  // rows of consecutive lanes at consecutive addresses
  struct Lds {
    double2 S[NP][NP];
    double nd[EB * NDS];  // per node: mu[4] s_0[4] s_1[4] w[4] Lambda_00 _01 _10 _11
  };

  __device__ static __forceinline__ void load_ops(const KArgs<double> &A, Lds &L) {
    for (int x = threadIdx.x; x < NP * NP; x += kT) {
      const int j = x / NP, k = x % NP;
      L.S[k][j] = double2(A.op.S[x], A.op.S[NP * NP + x]);
    }
  }

  __device__ static __forceinline__ void tile(const KArgs<double> &A, Lds &L, int tl) {
    const int tid = threadIdx.x;
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    if (!tile_on(A, e0, ne)) return;  // hybrid scheme: no element of this form
    const int e = tid / NP, j = tid % NP, eg = e0 + e;
    const bool act = tid < ne * NP && elem_on(A, eg);
    const GasC<double> &G = A.G;
    const GasC<Dual<double>> GD = dual_gas(G);
    const double cb = G.cb, he = 0.5 * (1.0 + cb), hz = 0.5 * (1.0 - cb);
    double lam[4], H = 1.0;
    Node<D, double> n;
    if (act) {
      double uu[NC], lm[NC], s[D][NC];
      const double *g = A.geo + (size_t)eg * 12;
      double F[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const double d0 = A.op.dN[(0 * 6 + a) * NP + j], d1 = A.op.dN[(1 * 6 + a) * NP + j];
        F[0][0] += d0 * g[2 * a];
        F[0][1] += d1 * g[2 * a];
        F[1][0] += d0 * g[2 * a + 1];
        F[1][1] += d1 * g[2 * a + 1];
      }
      lam[0] = F[1][1];
      lam[1] = -F[1][0];
      lam[2] = -F[0][1];
      lam[3] = F[0][0];
      H = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * A.op.h[j];
      const int uo = A.uoff[eg];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        uu[c] = A.u[uo + c * NP + j];
        lm[c] = A.lam[uo + c * NP + j];
      }
      node_from_u<D, double>(uu, G, n);
      if (!n.ok) atomicOr(A.err, 1);
#pragma unroll
      for (int i = 0; i < D; ++i) jvp_flux<D, double>(n, G, i, lm, s[i]);
      const double iH = drcp(H);
      double *v = L.nd + e * NDS + j * 20;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        v[c] = lm[c] * iH;
        v[4 + c] = s[0][c] * iH;
        v[8 + c] = s[1][c] * iH;
        v[12 + c] = n.w[c];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) v[16 + q] = lam[q];
    }
    __syncthreads();
    if (act) {
      double Z0[NC], Z1[NC], Vs[NC], X0[NC], X1[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) Z0[c] = Z1[c] = Vs[c] = X0[c] = X1[c] = 0.0;
#pragma unroll 2
      for (int k = 0; k < NP; ++k) {
        const double2 sp = L.S[k][j];
        const double s0 = sp.x, s1 = sp.y;
        const double *v = L.nd + e * NDS + k * 20;
        const double c0 = s0 * (lam[0] + v[16]) + s1 * (lam[1] + v[17]);
        const double c1 = s0 * (lam[2] + v[18]) + s1 * (lam[3] + v[19]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          Z0[c] += c0 * v[c];
          Z1[c] += c1 * v[c];
          Vs[c] += c0 * v[4 + c];  // one FMA per product
          Vs[c] += c1 * v[8 + c];
          X0[c] += c0 * v[12 + c];
          X1[c] += c1 * v[12 + c];
        }
      }
      // this node's state, cotangent and s_i: re-read after the pair loop
      // (from L1/L2 and LDS) rather than held in registers across it
      const int uo = A.uoff[eg];
      const double *vo = L.nd + e * NDS + j * 20;  // lambda/H, s_0/H, s_1/H, w
      double uu[NC], lm[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        uu[c] = A.u[uo + c * NP + j];
        lm[c] = A.lam[uo + c * NP + j];
      }
      const double E0 = A.op.E[j], E1 = A.op.E[NP + j];
      double ak[D];
      ak[0] = lam[0] * E0 + lam[1] * E1;
      ak[1] = lam[2] * E0 + lam[3] * E1;
      const double iH = drcp(H);
      double ub[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] = 0.0;
      // volume: sum_i A_i^T z_i, z_i = (1 - c_b)/2 Z_i + (1 + c_b)/2 a_i mu
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double zi[NC], o[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) zi[c] = hz * (i == 0 ? Z0[c] : Z1[c]) + he * ak[i] * vo[c];
        flux_jac_T<D, double>(n, G, uu[NC - 1], i, zi, o);
#pragma unroll
        for (int c = 0; c < NC; ++c) ub[c] += o[c];
      }
      // non-conservative: y = sum_i Q_xi^T s_i + sum_i d/de A~_i(w + e g_i) lambda,
      // sum_i Q_xi^T s_i = -V_s/2 + 1/2 sum_i a_i s_i,  g_i = H^-1 (X_i + a_i w)/2
      double y[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) y[c] = -0.5 * Vs[c] + 0.5 * (ak[0] * vo[4 + c] + ak[1] * vo[8 + c]);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double gi[NC], du[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) gi[c] = 0.5 * iH * ((i == 0 ? X0[c] : X1[c]) + ak[i] * n.w[c]);
        dU_from_dW<D, double>(n, G, gi, du);
        Dual<double> xd[NC], lmd[NC], hv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          xd[c] = Dual<double>(uu[c], du[c]);
          lmd[c] = Dual<double>(lm[c]);
        }
        Node<D, Dual<double>> nd;
        node_from_u<D, Dual<double>>(xd, GD, nd);
        jvp_flux<D, Dual<double>>(nd, GD, i, lmd, hv);
#pragma unroll
        for (int c = 0; c < NC; ++c) y[c] += hv[c].d;
      }
      double wy[NC];
      dWdU_apply<D>(uu, y, GD, wy);
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] -= cb * wy[c];
      // facet SATs: one gradient of this node's SAT with the combined
      // cotangent lambda_k/H_k - lambda_v/H_v (the neighbour's SAT is its negative)
      if (j < NFN) {
        const int off = A.nbr[(size_t)eg * NFN + j];
        double uv[NC], lv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          uv[c] = A.u[off + c * NP];
          lv[c] = A.lam[off + c * NP];
        }
        const int q = A.nbrq[(size_t)eg * NFN + j];
        const double Hv = A.Hn[(size_t)(q / NFN) * NP + q % NFN];
        double mu[NC], g1[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) mu[c] = vo[c] - lv[c] / Hv;
        Node<D, double> nk = n, nv;
        node_powers<D, double>(G, nk);
        node_from_u<D, double>(uv, G, nv);
        node_powers<D, double>(G, nv);
        facet_grad_rev<D>(nk, nv, ak, mu, G, A.diss != 0, g1);
#pragma unroll
        for (int c = 0; c < NC; ++c) ub[c] -= g1[c];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) A.ubar[uo + c * NP + j] = ub[c];
    }
    __syncthreads();
  }
};

// W as for k_vjp3v; built-in W = 2 (measured on MI355X, 32768 triangles:
// p = 4 170 -> 136 us against W = 1)
template <int P, int W>
__global__ __launch_bounds__(kT, W) void k_vjp2(KArgs<double> A) {
  typedef Vjp2<P> K;
  __shared__ typename K::Lds lds;
  K::load_ops(A, lds);
  __syncthreads();
  const int ntiles = (A.n_elem + K::EB - 1) / K::EB;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) K::tile(A, lds, tl);
}

constexpr size_t vjp2_lds_max() {
  size_t m = sizeof(Vjp2<1>::Lds);
  m = m > sizeof(Vjp2<2>::Lds) ? m : sizeof(Vjp2<2>::Lds);
  m = m > sizeof(Vjp2<3>::Lds) ? m : sizeof(Vjp2<3>::Lds);
  m = m > sizeof(Vjp2<4>::Lds) ? m : sizeof(Vjp2<4>::Lds);
  return m;
}

// every degree class of a 2D mesh in one persistent launch (tiles in degree
// order; a workgroup restages S_l when its tile changes degree)
__global__ __launch_bounds__(kT) void k_vjp2_batch(Batch2<double> Bt) {
  __shared__ __align__(16) unsigned char raw[vjp2_lds_max()];
  int cur = -1;
  for (int g = blockIdx.x; g < Bt.g0[4]; g += gridDim.x) {
    const int q = g < Bt.g0[1] ? 0 : (g < Bt.g0[2] ? 1 : (g < Bt.g0[3] ? 2 : 3));
    if (q != cur) {
      __syncthreads();
      if (q == 0) Vjp2<1>::load_ops(batch_args(Bt, 0), *(Vjp2<1>::Lds *)raw);
      else if (q == 1) Vjp2<2>::load_ops(batch_args(Bt, 1), *(Vjp2<2>::Lds *)raw);
      else if (q == 2) Vjp2<3>::load_ops(batch_args(Bt, 2), *(Vjp2<3>::Lds *)raw);
      else Vjp2<4>::load_ops(batch_args(Bt, 3), *(Vjp2<4>::Lds *)raw);
      __syncthreads();
      cur = q;
    }
    if (q == 0) Vjp2<1>::tile(batch_args(Bt, 0), *(Vjp2<1>::Lds *)raw, g);
    else if (q == 1) Vjp2<2>::tile(batch_args(Bt, 1), *(Vjp2<2>::Lds *)raw, g - Bt.g0[1]);
    else if (q == 2) Vjp2<3>::tile(batch_args(Bt, 2), *(Vjp2<3>::Lds *)raw, g - Bt.g0[2]);
    else Vjp2<4>::tile(batch_args(Bt, 3), *(Vjp2<4>::Lds *)raw, g - Bt.g0[3]);
  }
}

}  // namespace

hipError_t launch_vjp2_batch(const KArgs<double> *const cls[4], const KArgs<double> *cls_dev, hipStream_t s, int grid) {
  Batch2<double> Bt{};
  Bt.g0[0] = 0;
  const int eb[4] = {VTileV2<1>::EB, VTileV2<2>::EB, VTileV2<3>::EB, VTileV2<4>::EB};
  const KArgs<double> *any = nullptr;
  for (int q = 0; q < 4; ++q) {
    const int ne = cls[q] ? cls[q]->n_elem : 0;
    if (cls[q]) any = cls[q];
    Bt.g0[q + 1] = Bt.g0[q] + (ne + eb[q] - 1) / eb[q];
  }
  if (Bt.g0[4] == 0 || !any) return hipSuccess;
  Bt.cls = cls_dev;
  Bt.u = any->u;
  Bt.eform = any->eform;
  Bt.lam = any->lam;
  Bt.ubar = any->ubar;
  const int nb = launch_grid(reinterpret_cast<const void *>(&k_vjp2_batch), Bt.g0[4], grid);
  hipLaunchKernelGGL(k_vjp2_batch, dim3(nb), dim3(kT), 0, s, Bt);
  return hipGetLastError();
}

int vjp_variants(int dim, int p) {
  (void)dim;
  (void)p;
  return 2;
}

// VJP on tetrahedra with quadratic maps (Assumption 1: p >= 2): the curved-
// triangle derivation (Vjp2) in 3D.  Per node the metric cofactors Lambda
// and J from the element's ten map nodes; per pair
// c_m = sum_l S_l[j][k] (Lambda_ml(j) + Lambda_ml(k)), and
// Z_m += c_m mu_k, V_s += sum_m c_m s_m,k, X_m += c_m w_k; then the volume
// term sum_i A_i^T ((1 - c_b)/2 Z_i + (1 + c_b)/2 a_i mu), the
// non-conservative terms and the facet adjoint as on curved triangles.  S_l
// through the caches (rows read transposed, S being stored exactly skew).
template <int P, int W>
__global__ __launch_bounds__(kT, W) void k_vjp3c(KArgs<double> A) {
  constexpr int D = 3, NC = 5, NFAC = 4;
  constexpr int NP = Shape<3, P>::NP, NF = Shape<3, P>::NF, NFN = NFAC * NF;
  constexpr int EB = VTileV3<P>::EB;
  static_assert(EB * NP <= kT, "one node per lane");
  constexpr int NV = 34;  // per node: mu[5] s_1..3[15] w[5] Lambda[9]
  constexpr int NDS = NP * NV;
  __shared__ double nd[EB * NDS];
  __shared__ double gs[EB][30];
  const int tid = threadIdx.x;
  const GasC<double> &G = A.G;
  const GasC<Dual<double>> GD = dual_gas(G);
  const double cb = G.cb, he = 0.5 * (1.0 + cb), hz = 0.5 * (1.0 - cb);
  const int ntiles = (A.n_elem + EB - 1) / EB;
  const int e = tid / NP, j = tid % NP;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    if (!tile_on(A, e0, ne)) continue;  // hybrid scheme: no element of this form
    const int eg = e0 + e;
    const bool act = tid < ne * NP && elem_on(A, eg);
    __syncthreads();
    for (int x = tid; x < ne * 30; x += kT) gs[x / 30][x % 30] = A.geo[(size_t)(e0 + x / 30) * 30 + x % 30];
    __syncthreads();
    double uu[NC], lm[NC], L[D][D], H = 1.0, s[D][NC];
    Node<D, double> n;
    if (act) {
      double F[D][D];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int l = 0; l < D; ++l) F[k][l] = 0.0;
      const double *g = gs[e];
#pragma unroll
      for (int a = 0; a < 10; ++a)
#pragma unroll
        for (int l = 0; l < D; ++l) {
          const double d = A.op.dN[(l * 10 + a) * NP + j];
#pragma unroll
          for (int k = 0; k < D; ++k) F[k][l] += d * g[a * 3 + k];
        }
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int l = 0; l < D; ++l) {
          const int k1 = (k + 1) % 3, k2 = (k + 2) % 3, l1 = (l + 1) % 3, l2 = (l + 2) % 3;
          L[k][l] = F[k1][l1] * F[k2][l2] - F[k1][l2] * F[k2][l1];
        }
      H = (F[0][0] * L[0][0] + F[0][1] * L[0][1] + F[0][2] * L[0][2]) * A.op.h[j];
      const int uo = A.uoff[eg];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        uu[c] = A.u[uo + c * NP + j];
        lm[c] = A.lam[uo + c * NP + j];
      }
      node_from_u<D, double>(uu, G, n);
      if (!n.ok) atomicOr(A.err, 1);
#pragma unroll
      for (int i = 0; i < D; ++i) jvp_flux<D, double>(n, G, i, lm, s[i]);
      const double iH = drcp(H);
      double *v = nd + e * NDS + j * NV;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        v[c] = lm[c] * iH;
#pragma unroll
        for (int i = 0; i < D; ++i) v[5 + i * NC + c] = s[i][c] * iH;
        v[20 + c] = n.w[c];
      }
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int l = 0; l < D; ++l) v[25 + k * 3 + l] = L[k][l];
    }
    __syncthreads();
    if (act) {
      double Z[D][NC], Vs[NC], X[D][NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        Vs[c] = 0.0;
#pragma unroll
        for (int m = 0; m < D; ++m) Z[m][c] = X[m][c] = 0.0;
      }
#pragma unroll (P >= 3 ? 2 : 1)
      for (int k = 0; k < NP; ++k) {
        const double s0 = -A.op.S[(0 * NP + k) * NP + j];
        const double s1 = -A.op.S[(1 * NP + k) * NP + j];
        const double s2 = -A.op.S[(2 * NP + k) * NP + j];
        const double *v = nd + e * NDS + k * NV;
        double cm[D];
#pragma unroll
        for (int m = 0; m < D; ++m)
          cm[m] = s0 * (L[m][0] + v[25 + m * 3 + 0]) + s1 * (L[m][1] + v[25 + m * 3 + 1]) +
                  s2 * (L[m][2] + v[25 + m * 3 + 2]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
#pragma unroll
          for (int m = 0; m < D; ++m) {
            Z[m][c] += cm[m] * v[c];  // one FMA per product
            Vs[c] += cm[m] * v[5 + m * NC + c];
            X[m][c] += cm[m] * v[20 + c];
          }
        }
      }
      double ak[D];
#pragma unroll
      for (int m = 0; m < D; ++m) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) t += L[m][l] * A.op.E[l * NP + j];
        ak[m] = t;
      }
      const double iH = drcp(H);
      double ub[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] = 0.0;
      // volume: sum_i A_i^T z_i, z_i = (1 - c_b)/2 Z_i + (1 + c_b)/2 a_i mu
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double zi[NC], o[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) zi[c] = hz * Z[i][c] + he * ak[i] * lm[c] * iH;
        flux_jac_T<D, double>(n, G, uu[NC - 1], i, zi, o);
#pragma unroll
        for (int c = 0; c < NC; ++c) ub[c] += o[c];
      }
      // non-conservative: y = sum_i Q_xi^T s_i + sum_i d/de A~_i(w + e g_i) lambda,
      // sum_i Q_xi^T s_i = -V_s/2 + 1/2 sum_i a_i s_i,  g_i = H^-1 (X_i + a_i w)/2
      double y[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) y[c] = -0.5 * Vs[c] + 0.5 * iH * (ak[0] * s[0][c] + ak[1] * s[1][c] + ak[2] * s[2][c]);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double gi[NC], du[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) gi[c] = 0.5 * iH * (X[i][c] + ak[i] * n.w[c]);
        dU_from_dW<D, double>(n, G, gi, du);
        Dual<double> xd[NC], lmd[NC], hv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          xd[c] = Dual<double>(uu[c], du[c]);
          lmd[c] = Dual<double>(lm[c]);
        }
        Node<D, Dual<double>> ndu;
        node_from_u<D, Dual<double>>(xd, GD, ndu);
        jvp_flux<D, Dual<double>>(ndu, GD, i, lmd, hv);
#pragma unroll
        for (int c = 0; c < NC; ++c) y[c] += hv[c].d;
      }
      double wy[NC];
      dWdU_apply<D>(uu, y, GD, wy);
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] -= cb * wy[c];
      // facet SATs: one gradient of this node's SAT with the combined
      // cotangent lambda_k/H_k - lambda_v/H_v (the neighbour's SAT is its negative)
      if (j < NFN) {
        const int off = A.nbr[(size_t)eg * NFN + j];
        double uv[NC], lv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          uv[c] = A.u[off + c * NP];
          lv[c] = A.lam[off + c * NP];
        }
        const int q = A.nbrq[(size_t)eg * NFN + j];
        const double Hv = A.Hn[(size_t)(q / NFN) * NP + q % NFN];
        double mu[NC], g1[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) mu[c] = lm[c] * iH - lv[c] / Hv;
        Node<D, double> nk = n, nv;
        node_powers<D, double>(G, nk);
        node_from_u<D, double>(uv, G, nv);
        node_powers<D, double>(G, nv);
        facet_grad_rev<D>(nk, nv, ak, mu, G, A.diss != 0, g1);
#pragma unroll
        for (int c = 0; c < NC; ++c) ub[c] -= g1[c];
      }
      const int uo = A.uoff[eg];
#pragma unroll
      for (int c = 0; c < NC; ++c) A.ubar[uo + c * NP + j] = ub[c];
    }
  }
}

// VJP of the Hadamard form (the comparator, eq. weak form 2pt; not in the
// paper).  With r_a = -H_a^-1 sum_{n != a} c_an . F*(u_a, u_n),
// c_an = sum_l S_l[a][n] (Lambda_.l(a) + Lambda_.l(n)), the two-point flux
// symmetric in its arguments and c_na = -c_an, the contributions of row a
// and of the other rows to u_a combine into one gradient per pair of a's own
// two-point flux with the cotangent lambda_a/H_a - lambda_n/H_n (as for the
// facet SATs):
//   ubar_a = -sum_{n != a} grad_{u_a}[c_an . F*(u_a, u_n)]^T (lambda_a/H_a - lambda_n/H_n)
// plus the facet SAT adjoint.  One lane per node row; node values (V, p, z1,
// the flux powers, lambda/H) and per-node metrics of the tile in LDS; S_l
// through the caches (rows read transposed, S being stored exactly skew).
// The kernel skips the elements of the other form (hybrid scheme).
template <int DIM, int P, bool CURVED>
__global__ __launch_bounds__(kT) void k_vjp_had(KArgs<double> A) {
  constexpr int D = DIM, NC = D + 2, NFAC = D + 1;
  constexpr int NP = Shape<DIM, P>::NP, NF = Shape<DIM, P>::NF, NFN = NFAC * NF;
  constexpr int EB = kT / NP;
  constexpr bool PN = DIM == 2 || CURVED;         // metrics per node
  constexpr int NM = D * D + 1;                   // Lambda (row i, col l), J
  constexpr int NG = DIM == 2 ? 12 : (CURVED ? 30 : 10);
  constexpr int NV = D + 4;                       // V, p, z1, P1, P2
  __shared__ double nd[NV + NC][EB][NP];           // ... and lambda / H
  __shared__ double met[PN ? NM : 1][EB][PN ? NP : 1];
  __shared__ double gs[EB][NG];
  const int tid = threadIdx.x;
  const int e = tid / NP, a = tid % NP;
  const GasC<double> &G = A.G;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    if (!tile_on(A, e0, ne)) continue;  // hybrid scheme: no element of this form
    const bool act = tid < ne * NP && elem_on(A, e0 + e);
    const int eg = e0 + e;
    __syncthreads();
    for (int x = tid; x < ne * NG; x += kT) gs[x / NG][x % NG] = A.geo[(size_t)(e0 + x / NG) * NG + x % NG];
    __syncthreads();
    Node<D, double> n;
    double lm[NC], L[D][D], H = 1.0, ak[D];
    if (act) {
      double J;
      if constexpr (DIM == 2) {
        const double *g = gs[e];
        double F[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const double d0 = A.op.dN[(0 * 6 + q) * NP + a], d1 = A.op.dN[(1 * 6 + q) * NP + a];
          F[0][0] += d0 * g[2 * q];
          F[0][1] += d1 * g[2 * q];
          F[1][0] += d0 * g[2 * q + 1];
          F[1][1] += d1 * g[2 * q + 1];
        }
        L[0][0] = F[1][1];
        L[0][1] = -F[1][0];
        L[1][0] = -F[0][1];
        L[1][1] = F[0][0];
        J = F[0][0] * F[1][1] - F[0][1] * F[1][0];
      } else if constexpr (CURVED) {
        double F[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 3; ++l) F[k][l] = 0.0;
#pragma unroll
        for (int q = 0; q < 10; ++q)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            const double d = A.op.dN[(l * 10 + q) * NP + a];
#pragma unroll
            for (int k = 0; k < 3; ++k) F[k][l] += d * gs[e][q * 3 + k];
          }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            const int k1 = (k + 1) % 3, k2 = (k + 2) % 3, l1 = (l + 1) % 3, l2 = (l + 2) % 3;
            L[k][l] = F[k1][l1] * F[k2][l2] - F[k1][l2] * F[k2][l1];
          }
        J = F[0][0] * L[0][0] + F[0][1] * L[0][1] + F[0][2] * L[0][2];
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 3; ++l) L[k][l] = gs[e][k * 3 + l];
        J = gs[e][9];
      }
      if constexpr (PN) {
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int l = 0; l < D; ++l) met[k * D + l][e][a] = L[k][l];
      }
      H = J * A.op.h[a];
      const int uo = A.uoff[eg];
      double uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        uu[c] = A.u[uo + c * NP + a];
        lm[c] = A.lam[uo + c * NP + a];
      }
      node_from_u<D, double>(uu, G, n);
      if (!n.ok) atomicOr(A.err, 1);
      node_powers<D, double>(G, n);
#pragma unroll
      for (int i = 0; i < D; ++i) nd[i][e][a] = n.V[i];
      nd[D][e][a] = n.p;
      nd[D + 1][e][a] = n.z1;
      nd[D + 2][e][a] = n.P1;
      nd[D + 3][e][a] = n.P2;
      const double iH = drcp(H);
#pragma unroll
      for (int c = 0; c < NC; ++c) nd[NV + c][e][a] = lm[c] * iH;
#pragma unroll
      for (int m = 0; m < D; ++m) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) t += L[m][l] * A.op.E[l * NP + a];
        ak[m] = t;
      }
    }
    __syncthreads();
    if (act) {
      double ub[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] = 0.0;
      for (int nn = 0; nn < NP; ++nn) {
        if (nn == a) continue;
        Node<D, double> b;
#pragma unroll
        for (int i = 0; i < D; ++i) b.V[i] = nd[i][e][nn];
        b.p = nd[D][e][nn];
        b.z1 = nd[D + 1][e][nn];
        b.P1 = nd[D + 2][e][nn];
        b.P2 = nd[D + 3][e][nn];
#pragma unroll
        for (int c = 0; c < NC; ++c) b.w[c] = 0.0;  // read only with dissipation
        double sl[D];
#pragma unroll
        for (int l = 0; l < D; ++l) sl[l] = -A.op.S[(l * NP + nn) * NP + a];  // S_l[a][nn]
        double cvec[D], mu[NC], g[NC];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          double t = 0.0;
#pragma unroll
          for (int l = 0; l < D; ++l) {
            const double lsum = PN ? L[i][l] + met[i * D + l][e][PN ? nn : 0] : 2.0 * L[i][l];
            t += sl[l] * lsum;
          }
          cvec[i] = t;
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) mu[c] = nd[NV + c][e][a] - nd[NV + c][e][nn];
        facet_grad_rev<D>(n, b, cvec, mu, G, false, g);
#pragma unroll
        for (int c = 0; c < NC; ++c) ub[c] -= g[c];
      }
      // facet SATs: as in the entropy-split VJP
      if (a < NFN) {
        const int off = A.nbr[(size_t)eg * NFN + a];
        double uv[NC], lv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          uv[c] = A.u[off + c * NP];
          lv[c] = A.lam[off + c * NP];
        }
        const int q = A.nbrq[(size_t)eg * NFN + a];
        const double Hv = A.Hn[(size_t)(q / NFN) * NP + q % NFN];
        double mu[NC], g1[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) mu[c] = lm[c] / H - lv[c] / Hv;
        Node<D, double> nv;
        node_from_u<D, double>(uv, G, nv);
        node_powers<D, double>(G, nv);
        facet_grad_rev<D>(n, nv, ak, mu, G, A.diss != 0, g1);
#pragma unroll
        for (int c = 0; c < NC; ++c) ub[c] -= g1[c];
      }
      const int uo = A.uoff[eg];
#pragma unroll
      for (int c = 0; c < NC; ++c) A.ubar[uo + c * NP + a] = ub[c];
    }
  }
}

namespace {

// kernel of a VJP slot: variant 0 the built-in register budget, 1 the other
const void *vjp_kernel(int dim, int p, int variant, int &eb) {
#define SBP_V2(PP)                                                                        \
  if (dim == 2 && p == PP) {                                                              \
    eb = VTileV2<PP>::EB;                                                                 \
    return variant == 1 ? reinterpret_cast<const void *>(&k_vjp2<PP, 1>)                 \
                        : reinterpret_cast<const void *>(&k_vjp2<PP, 2>);                 \
  }
  SBP_V2(1) SBP_V2(2) SBP_V2(3) SBP_V2(4)
#undef SBP_V2
#define SBP_V3(PP)                                                                        \
  if (dim == 3 && p == PP) {                                                              \
    eb = VTileV3<PP>::EB;                                                                 \
    return (vjp3_waves<PP>() == 2) != (variant == 1)                                      \
               ? reinterpret_cast<const void *>(&k_vjp3v<PP, 2>)                          \
               : reinterpret_cast<const void *>(&k_vjp3v<PP, 1>);                         \
  }
  SBP_V3(1) SBP_V3(2) SBP_V3(3)
#undef SBP_V3
  eb = 0;
  return nullptr;
}

// curved tetrahedra: built-in W = 1 (the per-node metrics and three
// accumulator sets need the larger register budget)
const void *vjp3c_kernel(int p, int variant, int &eb) {
  eb = p == 2 ? VTileV3<2>::EB : VTileV3<3>::EB;
  if (p == 2) return variant == 1 ? reinterpret_cast<const void *>(&k_vjp3c<2, 2>)
                                  : reinterpret_cast<const void *>(&k_vjp3c<2, 1>);
  if (p == 3) return variant == 1 ? reinterpret_cast<const void *>(&k_vjp3c<3, 2>)
                                  : reinterpret_cast<const void *>(&k_vjp3c<3, 1>);
  eb = 0;
  return nullptr;
}

// ---------------------------------------------------------------------------
// VJP of the Navier-Stokes terms (Sec. 5, eqs. sats visc, bo sats), added to
// the VJP of the Euler terms.  With mu = H^-1 lambda, Q_xi = K_i + a_i/2 the
// metric-averaged physical operators and y'_i = -1/2 H^-1 y_i, the viscous
// part of lambda^T r is
//   sum_i (Q_xi^T mu)^T F^V(i)(w, g)            g_j = D_xj w
//   - 1/2 sum_facet (w_k - w_v)^T s,            s = a . F^V(w, nu), nu_i = D_xi mu
//   - 1/2 sum_facet mu^T (q_k + q_v),           q = a . F^V(w, g) of each side
// (F^V(i) = sum_j K~_ij g_j is linear in the gradient; a_i = B n_i).  Its
// derivative: the cotangent of F^V(i) at a node is alpha_i = Q_xi^T mu plus,
// at facet nodes, a_i qbar with qbar = -1/2 (mu_k + mu_v) (each side's q
// enters both residuals); through the gradient, sum_j D_xj^T gbar_j with
// gbar_j = sum_i K~_ij^T alpha_i (viscous_flux_adjoint); through the node
// state at fixed gradients, dual numbers (the Hessian-vector terms, with the
// facet weight -1/2 a_i (w_k - w_v) on F^V(w, nu)); and through the jump
// w_k - w_v, -1/2 s_k + 1/2 s_v at the facet node.  nu is a function of
// lambda alone.  A pre-pass writes s and mu at every facet node so that each
// side reads the other's.
//
// Metrics per node, GM: 0 triangles (quadratic or affine map, 12 map-node
// coordinates), 1 affine tetrahedra (Lambda and J per element), 2
// tetrahedra with quadratic maps (30 map-node coordinates).  Every operator
// application is a metric-averaged node-pair sum over the reference skew
// operators (c_k(i, j) = sum_l S_l[i][j] (Lambda_kl(i) + Lambda_kl(j)),
// K_k at row i = 1/2 sum_j c_k(i, j)); one lane per node row.

template <int D, int NP, int GM>
__device__ __forceinline__ void vnode_metrics(const KArgs<double> &A, int eg, int i, double L[D][D], double &J) {
  if constexpr (GM == 0) {
    const double *g = A.geo + (size_t)eg * 12;
    double F[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const double d0 = A.op.dN[(0 * 6 + a) * NP + i], d1 = A.op.dN[(1 * 6 + a) * NP + i];
      F[0][0] += d0 * g[2 * a];
      F[0][1] += d1 * g[2 * a];
      F[1][0] += d0 * g[2 * a + 1];
      F[1][1] += d1 * g[2 * a + 1];
    }
    L[0][0] = F[1][1];
    L[0][1] = -F[1][0];
    L[D - 1][0] = -F[0][1];
    L[D - 1][D - 1] = F[0][0];
    J = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  } else if constexpr (GM == 1) {
    const double *g = A.geo + (size_t)eg * 10;
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int l = 0; l < D; ++l) L[k][l] = g[k * 3 + l];
    J = g[9];
  } else {
    const double *g = A.geo + (size_t)eg * 30;
    double F[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) F[k][l] = 0.0;
#pragma unroll
    for (int a = 0; a < 10; ++a)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const double d = A.op.dN[(l * 10 + a) * NP + i];
#pragma unroll
        for (int k = 0; k < 3; ++k) F[k][l] += d * g[a * 3 + k];
      }
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int l = 0; l < D; ++l) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3, l1 = (l + 1) % 3, l2 = (l + 2) % 3;
        L[k][l] = F[k1][l1] * F[k2][l2] - F[k1][l2] * F[k2][l1];
      }
    J = F[0][0] * L[0][0] + F[0][1] * L[0][1] + F[0][2] * L[0][D - 1];
  }
}

// c_k(i, j) for k < D from the skew operators (read transposed through the
// caches: S is stored exactly skew) and the metrics of rows i and j.
template <int D, int NP>
__device__ __forceinline__ void vpair_coef(const KArgs<double> &A, int i, int j, const double L[D][D],
                                           const double *Lj, double c[D]) {
  double sl[D];
#pragma unroll
  for (int l = 0; l < D; ++l) sl[l] = -A.op.S[(l * NP + j) * NP + i];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double t = 0.0;
#pragma unroll
    for (int l = 0; l < D; ++l) t += sl[l] * (L[k][l] + Lj[k * D + l]);
    c[k] = t;
  }
}

template <int D, int P, int GM>
__global__ __launch_bounds__(kT) void k_vjpv_pre(KArgs<double> A, double *sb) {
  constexpr int NC = D + 2, NFAC = D + 1;
  constexpr int NP = Shape<D, P>::NP, NF = Shape<D, P>::NF, NFN = NFAC * NF;
  constexpr int EB = kT / NP;
  constexpr int NV = NC + D * D + 1;  // mu, Lambda (odd stride in 3D)
  __shared__ double nd[EB * NP * NV];
  const int tid = threadIdx.x;
  const int e = tid / NP, i = tid % NP;
  const ViscC<double> Vc = A.V;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    const int eg = e0 + e;
    const bool act = e < ne;
    double L[D][D], J = 1.0, H = 1.0, mu[NC];
    Node<D, double> n;
    __syncthreads();
    if (act) {
      vnode_metrics<D, NP, GM>(A, eg, i, L, J);
      H = J * A.op.h[i];
      const int uo = A.uoff[eg];
      double uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        uu[c] = A.u[uo + c * NP + i];
        mu[c] = A.lam[uo + c * NP + i] / H;
      }
      node_from_u<D, double>(uu, A.G, n);
      double *v = nd + (e * NP + i) * NV;
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = mu[c];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int l = 0; l < D; ++l) v[NC + k * D + l] = L[k][l];
    }
    __syncthreads();
    if (act && i < NFN) {
      double X[D][NC];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) X[k][c] = 0.0;
#pragma unroll 1
      for (int j = 0; j < NP; ++j) {
        const double *v = nd + (e * NP + j) * NV;
        double ck[D];
        vpair_coef<D, NP>(A, i, j, L, v + NC, ck);
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c) X[k][c] += ck[k] * v[c];
      }
      double a[D], nu[D][NC], FV[D][NC];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) t += L[k][l] * A.op.E[l * NP + i];
        a[k] = t;
      }
      const double iH = drcp(H);
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) nu[k][c] = 0.5 * iH * (X[k][c] + a[k] * mu[c]);
      viscous_flux<D, double>(n, A.G, Vc, nu, FV);
      double *o = sb + ((size_t)eg * NFN + i) * 2 * NC;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) t += a[k] * FV[k][c];
        o[c] = t;
        o[NC + c] = mu[c];
      }
    }
  }
}

template <int D, int P, int GM>
__global__ __launch_bounds__(kT) void k_vjpv(KArgs<double> A, const double *sb) {
  constexpr int NC = D + 2, NFAC = D + 1;
  constexpr int NP = Shape<D, P>::NP, NF = Shape<D, P>::NF, NFN = NFAC * NF;
  constexpr int EB = kT / NP;
  // per node: w, mu, Lambda, z_1..z_D (z = H^-1 gbar)
  constexpr int OW = 0, OM = NC, OL = 2 * NC, OZ = 2 * NC + D * D;
  constexpr int NV = OZ + D * NC + 1;
  __shared__ double nd[EB * NP * NV];
  const int tid = threadIdx.x;
  const int e = tid / NP, i = tid % NP;
  const GasC<double> &G = A.G;
  const GasC<Dual<double>> GD = dual_gas(G);
  const ViscC<double> Vc = A.V;
  ViscC<Dual<double>> VD;
  VD.mu = Vc.mu;
  VD.kappa = Vc.kappa;
  VD.R = Vc.R;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    const int eg = e0 + e;
    const bool act = e < ne;
    double L[D][D], J = 1.0, H = 1.0, uu[NC], mu[NC];
    Node<D, double> n;
    __syncthreads();
    if (act) {
      vnode_metrics<D, NP, GM>(A, eg, i, L, J);
      H = J * A.op.h[i];
      const int uo = A.uoff[eg];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        uu[c] = A.u[uo + c * NP + i];
        mu[c] = A.lam[uo + c * NP + i] / H;
      }
      node_from_u<D, double>(uu, G, n);
      double *v = nd + (e * NP + i) * NV;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        v[OW + c] = n.w[c];
        v[OM + c] = mu[c];
      }
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int l = 0; l < D; ++l) v[OL + k * D + l] = L[k][l];
    }
    __syncthreads();
    double z[D][NC], wl[NC], ud[NC], a[D];
    if (act) {
      double Xw[D][NC], Xm[D][NC];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) Xw[k][c] = Xm[k][c] = 0.0;
#pragma unroll 1
      for (int j = 0; j < NP; ++j) {
        const double *v = nd + (e * NP + j) * NV;
        double ck[D];
        vpair_coef<D, NP>(A, i, j, L, v + OL, ck);
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            Xw[k][c] += ck[k] * v[OW + c];
            Xm[k][c] += ck[k] * v[OM + c];
          }
      }
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) t += L[k][l] * A.op.E[l * NP + i];
        a[k] = t;
      }
      const double iH = drcp(H);
      double g[D][NC], al[D][NC], nu[D][NC], ze[D][NC];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          g[k][c] = 0.5 * iH * (Xw[k][c] + a[k] * n.w[c]);
          al[k][c] = 0.5 * (a[k] * mu[c] - Xm[k][c]);
          nu[k][c] = 0.5 * iH * (Xm[k][c] + a[k] * mu[c]);
          ze[k][c] = 0.0;
        }
#pragma unroll
      for (int c = 0; c < NC; ++c) wl[c] = 0.0;
      const bool fac = i < NFN;
      if (fac) {
        const size_t fi = (size_t)eg * NFN + i;
        const int off = A.nbr[fi];
        double uv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) uv[c] = A.u[off + c * NP];
        Node<D, double> nv;
        node_from_u<D, double>(uv, G, nv);
        const double *sv = sb + (size_t)A.nbrq[fi] * 2 * NC;
        const double *sk = sb + fi * 2 * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double qb = -0.5 * (mu[c] + sv[NC + c]);
          const double dw = n.w[c] - nv.w[c];
#pragma unroll
          for (int k = 0; k < D; ++k) {
            al[k][c] += a[k] * qb;
            ze[k][c] = -0.5 * a[k] * dw;
          }
          wl[c] = 0.5 * (sv[c] - sk[c]);
        }
      }
      double gb[D][NC];
      viscous_flux_adjoint<D, double>(n, G, Vc, al, gb);
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) z[k][c] = iH * gb[k][c];
      // state derivative at fixed gradients (dual numbers, one pass per
      // component of u): alpha_i . F^V(i)(u; g) + facet -1/2 a_i dw . F^V(i)(u; nu)
#pragma unroll 1
      for (int q = 0; q < NC; ++q) {
        Dual<double> x[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = Dual<double>(uu[c], c == q ? 1.0 : 0.0);
        Node<D, Dual<double>> nq;
        node_from_u<D, Dual<double>>(x, GD, nq);
        Dual<double> gq[D][NC], F[D][NC];
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c) gq[k][c] = Dual<double>(g[k][c]);
        viscous_flux<D, Dual<double>>(nq, GD, VD, gq, F);
        double dphi = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c) dphi += al[k][c] * F[k][c].d;
        if (fac) {
#pragma unroll
          for (int k = 0; k < D; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) gq[k][c] = Dual<double>(nu[k][c]);
          viscous_flux<D, Dual<double>>(nq, GD, VD, gq, F);
#pragma unroll
          for (int k = 0; k < D; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) dphi += ze[k][c] * F[k][c].d;
        }
        ud[q] = dphi;
      }
      double *v = nd + (e * NP + i) * NV;
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) v[OZ + k * NC + c] = z[k][c];
    }
    __syncthreads();
    if (act) {
      // sum_j D_xj^T gbar_j = sum_j Q_xj^T z_j = -1/2 sum_n c_j(i, n) z_j,n + 1/2 sum_j a_j z_j,i
      double T[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) t += a[k] * z[k][c];
        T[c] = 0.5 * t;
      }
#pragma unroll 1
      for (int j = 0; j < NP; ++j) {
        const double *v = nd + (e * NP + j) * NV;
        double ck[D];
        vpair_coef<D, NP>(A, i, j, L, v + OL, ck);
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c) T[c] -= 0.5 * ck[k] * v[OZ + k * NC + c];
      }
      double wb[NC], du[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) wb[c] = T[c] + wl[c];
      dWdU_apply<D>(uu, wb, GD, du);
      const int uo = A.uoff[eg];
#pragma unroll
      for (int c = 0; c < NC; ++c) A.ubar[uo + c * NP + i] += du[c] + ud[c];
    }
  }
}

template <int D, int P, int GM>
hipError_t launch_vjpv_t(const KArgs<double> &A, double *sb, hipStream_t s) {
  constexpr int EB = kT / Shape<D, P>::NP;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  const void *f0 = reinterpret_cast<const void *>(&k_vjpv_pre<D, P, GM>);
  const void *f1 = reinterpret_cast<const void *>(&k_vjpv<D, P, GM>);
  KArgs<double> a = A;
  double *sp = sb;
  const double *cs = sb;
  void *args0[] = {&a, &sp};
  hipError_t e = hipLaunchKernel(f0, dim3(launch_grid(f0, ntiles, 1)), dim3(kT), args0, 0, s);
  if (e != hipSuccess) return e;
  void *args1[] = {&a, &cs};
  return hipLaunchKernel(f1, dim3(launch_grid(f1, ntiles, 1)), dim3(kT), args1, 0, s);
}

}  // namespace

hipError_t launch_vjp_hadamard(int dim, int p, const KArgs<double> &A, hipStream_t s) {
  if (A.n_elem <= 0) return hipSuccess;
  const void *fn = nullptr;
  int eb = 0;
#define SBP_VH(DD, PP, CC)                                                              \
  if (dim == DD && p == PP && (A.curved != 0) == CC) {                                   \
    fn = reinterpret_cast<const void *>(&k_vjp_had<DD, PP, CC>);                          \
    eb = kT / Shape<DD, PP>::NP;                                                          \
  }
  SBP_VH(2, 1, false) SBP_VH(2, 2, false) SBP_VH(2, 3, false) SBP_VH(2, 4, false)
  SBP_VH(3, 1, false) SBP_VH(3, 2, false) SBP_VH(3, 3, false) SBP_VH(3, 2, true) SBP_VH(3, 3, true)
#undef SBP_VH
  if (!fn) return hipErrorInvalidValue;
  const int nb = launch_grid(fn, (A.n_elem + eb - 1) / eb, 1);
  KArgs<double> a = A;
  void *args[] = {&a};
  return hipLaunchKernel(fn, dim3(nb), dim3(kT), args, 0, s);
}

hipError_t launch_vjp(int dim, int p, const KArgs<double> &A, hipStream_t s, LaunchCfg cfg) {
  if (A.n_elem <= 0) return hipSuccess;
  int eb = 0;
  const void *fn = A.curved ? (dim == 3 ? vjp3c_kernel(p, cfg.variant, eb) : nullptr)
                            : vjp_kernel(dim, p, cfg.variant, eb);
  if (!fn) return hipErrorInvalidValue;
  const int nb = launch_grid(fn, (A.n_elem + eb - 1) / eb, cfg.grid);
  KArgs<double> a = A;
  void *args[] = {&a};
  return hipLaunchKernel(fn, dim3(nb), dim3(kT), args, 0, s);
}

hipError_t launch_vjp_viscous(int dim, int p, const KArgs<double> &A, double *sbuf, hipStream_t s) {
  if (A.n_elem <= 0) return hipSuccess;
  if (dim == 2) {
    switch (p) {
      case 1: return launch_vjpv_t<2, 1, 0>(A, sbuf, s);
      case 2: return launch_vjpv_t<2, 2, 0>(A, sbuf, s);
      case 3: return launch_vjpv_t<2, 3, 0>(A, sbuf, s);
      case 4: return launch_vjpv_t<2, 4, 0>(A, sbuf, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (A.curved) {
    switch (p) {
      case 2: return launch_vjpv_t<3, 2, 2>(A, sbuf, s);
      case 3: return launch_vjpv_t<3, 3, 2>(A, sbuf, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (p) {
    case 1: return launch_vjpv_t<3, 1, 1>(A, sbuf, s);
    case 2: return launch_vjpv_t<3, 2, 1>(A, sbuf, s);
    case 3: return launch_vjpv_t<3, 3, 1>(A, sbuf, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sbp
