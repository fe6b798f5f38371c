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
//              lambda_v/H_v (dual numbers, one pass per component), gathered
//              without atomics.
// The transposed operators are applied as MFMA contractions like the forward
// kernel: [M_1^T; M_2^T; M_3^T] mu, [D_1^T D_2^T D_3^T] s, and D w.
//
// On curved triangles the physical operators are written with the skew parts
// K_i = 1/2 sum_l (Lambda_il S_l + S_l Lambda_il) and a_i = sum_l Lambda_il E_l:
//   Q_xi = K_i + a_i/2,  Q_xi^T = -K_i + a_i/2,
//   M_xi^T mu = (1 - c_b) K_i mu + (1 + c_b)/2 a_i mu,
// so only the reference skew operators S_l enter, as per-node-pair sums.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dual.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace sbp {

namespace {

constexpr int kT = 256;
constexpr int kW = kT / 64;

template <int P> struct VjpTile;
template <> struct VjpTile<1> { static constexpr int EB = 16; };
template <> struct VjpTile<2> { static constexpr int EB = 9; };
template <> struct VjpTile<3> { static constexpr int EB = 3; };

typedef double v4d __attribute__((ext_vector_type(4)));

// Same MFMA contraction as the forward kernels (f64 16x16x4; accumulator
// register i of lane l holds row l/16 + 4 i, column l%16).
template <int MP, int KP, int NCP>
__device__ __forceinline__ void gemm64(const double *__restrict__ At, const double *B, double *C) {
  constexpr int MT = MP / 16, NT = NCP / 16, NTILE = MT * NT;
  constexpr int TPW = (NTILE + kW - 1) / kW;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kr = lane >> 4;
  v4d acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = v4d{0, 0, 0, 0};
#pragma unroll 4
  for (int k = 0; k < KP; k += 4) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wave + t * kW;
      if (tile < NTILE) {
        const int mt = tile % MT, nt = tile / MT;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(At[(k + kr) * MP + mt * 16 + col],
                                                       B[(k + kr) * NCP + nt * 16 + col], acc[t], 0, 0, 0);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wave + t * kW;
    if (tile < NTILE) {
      const int mt = tile % MT, nt = tile / MT;
#pragma unroll
      for (int i = 0; i < 4; ++i) C[(mt * 16 + kr + 4 * i) * NCP + nt * 16 + col] = acc[t][i];
    }
  }
  __syncthreads();
}

// gradient of mu . Phi(u1, u2; a) with respect to u1, Phi = facet_term
// (two-point flux [+ dissipation]); one dual-number pass per component of
// u1, the neighbour state u2 evaluated once in plain arithmetic.
template <int D>
__device__ __forceinline__ void facet_grad(const double *u1, const double *u2, const double *a, const double *mu,
                                           const GasC<double> &G0, const GasC<Dual<double>> &G, bool diss,
                                           double *out) {
  constexpr int NC = D + 2;
  Dual<double> av[D];
#pragma unroll
  for (int i = 0; i < D; ++i) av[i] = Dual<double>(a[i]);
  Node<D, double> m2;
  node_from_u<D, double>(u2, G0, m2);
  node_powers<D, double>(G0, m2);
  Node<D, Dual<double>> n2;
  n2.rho = m2.rho;
#pragma unroll
  for (int i = 0; i < D; ++i) n2.V[i] = m2.V[i];
  n2.p = m2.p;
  n2.lrho = m2.lrho;
  n2.lp = m2.lp;
  n2.lz1 = m2.lz1;
  n2.z1 = m2.z1;
  n2.P1 = m2.P1;
  n2.P2 = m2.P2;
#pragma unroll
  for (int c = 0; c < NC; ++c) n2.w[c] = m2.w[c];
  n2.ok = m2.ok;
  for (int c = 0; c < NC; ++c) {
    Dual<double> x1[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) x1[q] = Dual<double>(u1[q], q == c ? 1.0 : 0.0);
    Node<D, Dual<double>> n1;
    node_from_u<D, Dual<double>>(x1, G, n1);
    node_powers<D, Dual<double>>(G, n1);
    Dual<double> ph[NC];
    facet_term<D, Dual<double>>(n1, n2, av, G, diss, ph);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NC; ++q) s += mu[q] * ph[q].d;
    out[c] = s;
  }
}

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

template <int P>
__global__ __launch_bounds__(kT) void k_vjp3(KArgs<double> A) {
  constexpr int D = 3, NC = 5, NFAC = 4;
  constexpr int NP = Shape<3, P>::NP, NF = Shape<3, P>::NF, NFN = NFAC * NF;
  constexpr int EB = VjpTile<P>::EB;
  constexpr int NCP = ru(EB * NC, 16);
  constexpr int K1P = ru(3 * NP, 4), M1P = ru(NP, 16);
  constexpr int K2P = ru(NP, 4), M2P = ru(3 * NP, 16);
  __shared__ double Bmu[K2P * NCP];
  __shared__ double Bw[K2P * NCP];
  __shared__ double Bs[K1P * NCP];
  __shared__ double Z[M2P * NCP];
  __shared__ double C2[M2P * NCP];
  __shared__ double Qo[M1P * NCP];
  __shared__ double us[EB * NC * NP];
  __shared__ double ls[EB * NC * NP];
  __shared__ double gs[EB * 10];
  __shared__ double hs[NP];
  __shared__ double Es[3 * NP];
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * EB;
  const int ne = min(EB, A.n_elem - e0);
  const GasC<double> &G = A.G;
  const GasC<Dual<double>> GD = dual_gas(G);
  for (int x = tid; x < EB * 10; x += kT) {
    const int e = x / 10;
    gs[x] = e < ne ? A.geo[(size_t)(e0 + e) * 10 + x % 10] : 0.0;
  }
  for (int x = tid; x < NP; x += kT) hs[x] = A.op.h[x];
  for (int x = tid; x < 3 * NP; x += kT) Es[x] = A.op.E[x];
  for (int x = tid; x < ne * NC * NP; x += kT) {
    const int e = x / (NC * NP);
    const int o = A.uoff[e0 + e] + x % (NC * NP);
    us[x] = A.u[o];
    ls[x] = A.lam[o];
  }
  for (int x = tid; x < K2P * NCP; x += kT) {
    Bmu[x] = 0.0;
    Bw[x] = 0.0;
  }
  for (int x = tid; x < K1P * NCP; x += kT) Bs[x] = 0.0;
  __syncthreads();
  for (int x = tid; x < ne * NP; x += kT) {
    const int e = x / NP, j = x % NP;
    double uu[NC], lm[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      uu[c] = us[(e * NC + c) * NP + j];
      lm[c] = ls[(e * NC + c) * NP + j];
    }
    Node<D, double> n;
    node_from_u<D, double>(uu, G, n);
    if (!n.ok) atomicOr(A.err, 1);
    const double *Lam = gs + e * 10;
    const double J = Lam[9], iJ = 1.0 / J;
    const double iH = 1.0 / (J * hs[j]);
    double t[D][NC];
#pragma unroll
    for (int i = 0; i < D; ++i) jvp_flux<D, double>(n, G, i, lm, t[i]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      Bmu[j * NCP + e * NC + c] = lm[c] * iH;
      Bw[j * NCP + e * NC + c] = n.w[c];
#pragma unroll
      for (int l = 0; l < D; ++l)
        Bs[(l * NP + j) * NCP + e * NC + c] =
            (Lam[0 * 3 + l] * t[0][c] + Lam[1 * 3 + l] * t[1][c] + Lam[2 * 3 + l] * t[2][c]) * iJ;
    }
  }
  __syncthreads();
  gemm64<M2P, K2P, NCP>(A.op.At6, Bmu, Z);   // z_l = M_l^T mu, rows l*NP + j
  gemm64<M2P, K2P, NCP>(A.op.At2, Bw, C2);   // D_l w
  gemm64<M1P, K1P, NCP>(A.op.At7, Bs, Qo);   // sum_l D_l^T s_l
  for (int x = tid; x < ne * NP; x += kT) {
    const int e = x / NP, j = x % NP;
    const int eg = e0 + e;
    double uu[NC], lm[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      uu[c] = us[(e * NC + c) * NP + j];
      lm[c] = ls[(e * NC + c) * NP + j];
    }
    Node<D, double> n;
    node_from_u<D, double>(uu, G, n);
    const double *Lam = gs + e * 10;
    const double J = Lam[9], iJ = 1.0 / J;
    const double H = J * hs[j];
    double ub[NC];
    // volume: sum_l sum_i Lambda_il A_i^T z_l
#pragma unroll
    for (int c = 0; c < NC; ++c) ub[c] = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double zi[NC], o[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) s += Lam[i * 3 + l] * Z[(l * NP + j) * NCP + e * NC + c];
        zi[c] = s;
      }
      flux_jac_T<D, double>(n, G, uu[NC - 1], i, zi, o);
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] += o[c];
    }
    // non-conservative: -c_b dW/dU [ sum_i D_xi^T (A~_i lambda) + HVP ]
    double y[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) y[c] = Qo[j * NCP + e * NC + c];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double gi[NC], du[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) s += Lam[i * 3 + l] * C2[(l * NP + j) * NCP + e * NC + c];
        gi[c] = s * iJ;
      }
      dU_from_dW<D, double>(n, G, gi, du);
      Dual<double> x[NC], lmd[NC], hv[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        x[c] = Dual<double>(uu[c], du[c]);
        lmd[c] = Dual<double>(lm[c]);
      }
      Node<D, Dual<double>> nd;
      node_from_u<D, Dual<double>>(x, GD, nd);
      jvp_flux<D, Dual<double>>(nd, GD, i, lmd, hv);
#pragma unroll
      for (int c = 0; c < NC; ++c) y[c] += hv[c].d;
    }
    double wy[NC];
    dWdU_apply<D>(uu, y, GD, wy);
#pragma unroll
    for (int c = 0; c < NC; ++c) ub[c] -= G.cb * wy[c];
    // facet SATs: own term and the neighbour's term at this node
    if (j < NFN) {
      const int off = A.nbr[(size_t)eg * NFN + j];
      double uv[NC], lv[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        uv[c] = A.u[off + c * NP];
        lv[c] = A.lam[off + c * NP];
      }
      double ak[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) s += Lam[i * 3 + l] * Es[l * NP + j];
        ak[i] = s;
      }
      // the neighbour's SAT is the negative of this node's (antisymmetric
      // two-point flux and dissipation, opposite B n), so both derivatives
      // are one gradient of Phi(u_k, u_v) with the cotangent
      // lambda_k / H_k - lambda_v / H_v
      const int q = A.nbrq[(size_t)eg * NFN + j];
      const double Hv = A.Hn[(size_t)(q / NFN) * NP + q % NFN];
      double mu[NC], g1[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) mu[c] = lm[c] / H - lv[c] / Hv;
      facet_grad<D>(uu, uv, ak, mu, G, GD, A.diss != 0, g1);
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] -= g1[c];
    }
    const int uo = A.uoff[eg];
#pragma unroll
    for (int c = 0; c < NC; ++c) A.ubar[uo + c * NP + j] = ub[c];
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
  struct Lds {
    double S[2][NP][NP];
    double nd[EB * NDS];  // per node: mu[4] s_0[4] s_1[4] w[4] Lambda_00 _01 _10 _11
  };

  __device__ static __forceinline__ void load_ops(const KArgs<double> &A, Lds &L) {
    for (int x = threadIdx.x; x < 2 * NP * NP; x += kT) (&L.S[0][0][0])[x] = A.op.S[x];
  }

  __device__ static __forceinline__ void tile(const KArgs<double> &A, Lds &L, int tl) {
    const int tid = threadIdx.x;
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    const bool act = tid < ne * NP;
    const int e = tid / NP, j = tid % NP, eg = e0 + e;
    const GasC<double> &G = A.G;
    const GasC<Dual<double>> GD = dual_gas(G);
    const double cb = G.cb, he = 0.5 * (1.0 + cb), hz = 0.5 * (1.0 - cb);
    double uu[NC], lm[NC], lam[4], H = 1.0, s[D][NC];
    Node<D, double> n;
    if (act) {
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
      const double iH = 1.0 / H;
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
#pragma unroll 1
      for (int k = 0; k < NP; ++k) {
        const double s0 = L.S[0][j][k], s1 = L.S[1][j][k];
        const double *v = L.nd + e * NDS + k * 20;
        const double c0 = s0 * (lam[0] + v[16]) + s1 * (lam[1] + v[17]);
        const double c1 = s0 * (lam[2] + v[18]) + s1 * (lam[3] + v[19]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          Z0[c] += c0 * v[c];
          Z1[c] += c1 * v[c];
          Vs[c] += c0 * v[4 + c] + c1 * v[8 + c];
          X0[c] += c0 * v[12 + c];
          X1[c] += c1 * v[12 + c];
        }
      }
      const double E0 = A.op.E[j], E1 = A.op.E[NP + j];
      double ak[D];
      ak[0] = lam[0] * E0 + lam[1] * E1;
      ak[1] = lam[2] * E0 + lam[3] * E1;
      const double iH = 1.0 / H;
      double ub[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] = 0.0;
      // volume: sum_i A_i^T z_i, z_i = (1 - c_b)/2 Z_i + (1 + c_b)/2 a_i mu
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double zi[NC], o[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) zi[c] = hz * (i == 0 ? Z0[c] : Z1[c]) + he * ak[i] * lm[c] * iH;
        flux_jac_T<D, double>(n, G, uu[NC - 1], i, zi, o);
#pragma unroll
        for (int c = 0; c < NC; ++c) ub[c] += o[c];
      }
      // non-conservative: y = sum_i Q_xi^T s_i + sum_i d/de A~_i(w + e g_i) lambda,
      // sum_i Q_xi^T s_i = -V_s/2 + 1/2 sum_i a_i s_i,  g_i = H^-1 (X_i + a_i w)/2
      double y[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) y[c] = -0.5 * Vs[c] + 0.5 * iH * (ak[0] * s[0][c] + ak[1] * s[1][c]);
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
        for (int c = 0; c < NC; ++c) mu[c] = lm[c] * iH - lv[c] / Hv;
        facet_grad<D>(uu, uv, ak, mu, G, GD, A.diss != 0, g1);
#pragma unroll
        for (int c = 0; c < NC; ++c) ub[c] -= g1[c];
      }
      const int uo = A.uoff[eg];
#pragma unroll
      for (int c = 0; c < NC; ++c) A.ubar[uo + c * NP + j] = ub[c];
    }
    __syncthreads();
  }
};

template <int P>
__global__ __launch_bounds__(kT) void k_vjp2(KArgs<double> A) {
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
      if (q == 0) Vjp2<1>::load_ops(Bt.c[0], *(Vjp2<1>::Lds *)raw);
      else if (q == 1) Vjp2<2>::load_ops(Bt.c[1], *(Vjp2<2>::Lds *)raw);
      else if (q == 2) Vjp2<3>::load_ops(Bt.c[2], *(Vjp2<3>::Lds *)raw);
      else Vjp2<4>::load_ops(Bt.c[3], *(Vjp2<4>::Lds *)raw);
      __syncthreads();
      cur = q;
    }
    if (q == 0) Vjp2<1>::tile(Bt.c[0], *(Vjp2<1>::Lds *)raw, g);
    else if (q == 1) Vjp2<2>::tile(Bt.c[1], *(Vjp2<2>::Lds *)raw, g - Bt.g0[1]);
    else if (q == 2) Vjp2<3>::tile(Bt.c[2], *(Vjp2<3>::Lds *)raw, g - Bt.g0[2]);
    else Vjp2<4>::tile(Bt.c[3], *(Vjp2<4>::Lds *)raw, g - Bt.g0[3]);
  }
}

}  // namespace

hipError_t launch_vjp2_batch(const KArgs<double> *const cls[4], hipStream_t s) {
  Batch2<double> Bt{};
  Bt.g0[0] = 0;
  const int eb[4] = {VTileV2<1>::EB, VTileV2<2>::EB, VTileV2<3>::EB, VTileV2<4>::EB};
  for (int q = 0; q < 4; ++q) {
    const int ne = cls[q] ? cls[q]->n_elem : 0;
    if (cls[q]) Bt.c[q] = *cls[q];
    Bt.g0[q + 1] = Bt.g0[q] + (ne + eb[q] - 1) / eb[q];
  }
  if (Bt.g0[4] == 0) return hipSuccess;
  const dim3 grid(std::min(Bt.g0[4], 2048));
  hipLaunchKernelGGL(k_vjp2_batch, grid, dim3(kT), 0, s, Bt);
  return hipGetLastError();
}

hipError_t launch_vjp(int dim, int p, const KArgs<double> &A, hipStream_t s) {
  dim3 block(kT);
  if (A.n_elem <= 0) return hipSuccess;
  if (dim == 2) {
    // persistent workgroups: at most about as many as 256 CUs keep resident
    const int eb = p == 1 ? VTileV2<1>::EB : (p == 2 ? VTileV2<2>::EB : (p == 3 ? VTileV2<3>::EB : VTileV2<4>::EB));
    const dim3 grid(std::min((A.n_elem + eb - 1) / eb, 2048));
    switch (p) {
      case 1: hipLaunchKernelGGL(k_vjp2<1>, grid, block, 0, s, A); break;
      case 2: hipLaunchKernelGGL(k_vjp2<2>, grid, block, 0, s, A); break;
      case 3: hipLaunchKernelGGL(k_vjp2<3>, grid, block, 0, s, A); break;
      case 4: hipLaunchKernelGGL(k_vjp2<4>, grid, block, 0, s, A); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (dim != 3) return hipErrorInvalidValue;
  switch (p) {
    case 1: hipLaunchKernelGGL(k_vjp3<1>, dim3((A.n_elem + VjpTile<1>::EB - 1) / VjpTile<1>::EB), block, 0, s, A); break;
    case 2: hipLaunchKernelGGL(k_vjp3<2>, dim3((A.n_elem + VjpTile<2>::EB - 1) / VjpTile<2>::EB), block, 0, s, A); break;
    case 3: hipLaunchKernelGGL(k_vjp3<3>, dim3((A.n_elem + VjpTile<3>::EB - 1) / VjpTile<3>::EB), block, 0, s, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sbp
