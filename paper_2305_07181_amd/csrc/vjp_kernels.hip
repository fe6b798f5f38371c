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
//   facets     each facet node receives the derivative of its own SAT with
//              respect to its own state and the derivative of the matching
//              neighbour's SAT with respect to this node's state (both by dual
//              numbers, one pass per component), gathered without atomics.
// The transposed operators are applied as MFMA contractions like the forward
// kernel: [M_1^T; M_2^T; M_3^T] mu, [D_1^T D_2^T D_3^T] s, and D w.
#include <hip/hip_runtime.h>

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

// gradient of lambda . Phi(u1, u2; a) with respect to u1 (which = 0) or u2
// (which = 1), Phi = facet_term (two-point flux [+ dissipation]).
template <int D>
__device__ __forceinline__ void facet_grad(const double *u1, const double *u2, const double *a, const double *lam,
                                           const GasC<Dual<double>> &G, bool diss, int which, double *out) {
  constexpr int NC = D + 2;
  Dual<double> av[D];
#pragma unroll
  for (int i = 0; i < D; ++i) av[i] = Dual<double>(a[i]);
  for (int c = 0; c < NC; ++c) {
    Dual<double> x1[NC], x2[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      x1[q] = Dual<double>(u1[q], (which == 0 && q == c) ? 1.0 : 0.0);
      x2[q] = Dual<double>(u2[q], (which == 1 && q == c) ? 1.0 : 0.0);
    }
    Node<D, Dual<double>> n1, n2;
    node_from_u<D, Dual<double>>(x1, G, n1);
    node_from_u<D, Dual<double>>(x2, G, n2);
    node_powers<D, Dual<double>>(G, n1);
    node_powers<D, Dual<double>>(G, n2);
    Dual<double> ph[NC];
    facet_term<D, Dual<double>>(n1, n2, av, G, diss, ph);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NC; ++q) s += lam[q] * ph[q].d;
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
      const int q = A.nbrq[(size_t)eg * NFN + j];
      const int vk = q / NFN, nn = q % NFN;
      const double *Lv = A.geo + (size_t)vk * 10;
      double av[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) s += Lv[i * 3 + l] * Es[l * NP + nn];
        av[i] = s;
      }
      const double Hv = A.Hn[(size_t)vk * NP + nn];
      double g1[NC], g2[NC];
      facet_grad<D>(uu, uv, ak, lm, GD, A.diss != 0, 0, g1);
      facet_grad<D>(uv, uu, av, lv, GD, A.diss != 0, 1, g2);
#pragma unroll
      for (int c = 0; c < NC; ++c) ub[c] -= g1[c] / H + g2[c] / Hv;
    }
    const int uo = A.uoff[eg];
#pragma unroll
    for (int c = 0; c < NC; ++c) A.ubar[uo + c * NP + j] = ub[c];
  }
}

}  // namespace

hipError_t launch_vjp(int dim, int p, const KArgs<double> &A, hipStream_t s) {
  if (dim != 3) return hipErrorInvalidValue;
  dim3 block(kT);
  switch (p) {
    case 1: hipLaunchKernelGGL(k_vjp3<1>, dim3((A.n_elem + VjpTile<1>::EB - 1) / VjpTile<1>::EB), block, 0, s, A); break;
    case 2: hipLaunchKernelGGL(k_vjp3<2>, dim3((A.n_elem + VjpTile<2>::EB - 1) / VjpTile<2>::EB), block, 0, s, A); break;
    case 3: hipLaunchKernelGGL(k_vjp3<3>, dim3((A.n_elem + VjpTile<3>::EB - 1) / VjpTile<3>::EB), block, 0, s, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sbp
