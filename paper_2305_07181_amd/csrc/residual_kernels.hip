// Residual kernels of the entropy-split SBP-SAT scheme for gfx950 (CDNA4).
//
// Every kernel is persistent: a workgroup (4 wave64) loops over tiles of
// elements of one degree class.  Per tile:
//   1. per node: primitives, entropy variables w, fluxes f^(i) (and their
//      contravariant combinations), written to LDS rows;
//   2. the volume term of Sec. 6.2, eq. weak form split, through the skew
//      parts S_l = Q_l - E_l/2 of the reference operators shared by the class:
//      - Euler terms (k_split2, k_split3v): per-node-pair sums on the vector
//        ALUs, one lane per node row (2D: R rows per lane), S_l in LDS or
//        read through the caches;
//      - Navier-Stokes terms (k_split3<..., true>): MFMA contractions with
//        columns = element x component (v_mfma_f64_16x16x4 / _f32_);
//   3. per node: H^-1 (volume) - c_b sum_i A~_i D_xi w with A~_i applied as a
//      directional derivative, then at facet nodes the entropy-conservative
//      SAT with the Sjogreen-Yee two-point flux (Sec. 4, eq. sats inv) and the
//      optional matrix interface dissipation (Sec. 4.5), the neighbour state
//      gathered through the precomputed face-node map; write r once;
//   4. FP64 partial of sum w^T H r per workgroup (deterministic).
// Each facet node belongs to exactly one facet, so every node's residual is
// written by exactly one thread (no atomics, no second pass).
//
// The Hadamard-form comparator (Sec. 6.2, eq. weak form 2pt, k_hadamard)
// gives each lane one node row and sums the two-point fluxes of that row in a
// fixed order (each pair evaluated from both of its rows), then shares the
// facet epilogue.  In the hybrid scheme (Sec. 4.4) each kernel skips the
// elements flagged for the other volume form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "kernels.hpp"
#include "launch.hpp"
#include "mfma.hpp"

namespace sbp {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ void block_sum_store(double v, double *out) {
  __shared__ double red[kWaves];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += red[w];
    if (out) out[blockIdx.x] = s;
  }
}

// Facet SAT (+ dissipation), store of r, entropy-rate accumulation.
template <int D, int NP, int NF, typename T>
__device__ __forceinline__ void finish_node(const KArgs<T> &A, int eg, int i, const Node<D, T> &n,
                                            T H, const T *avec, T *r, double &ent) {
  constexpr int NC = D + 2, NFAC = D + 1;
  const T iH = (T)1 / H;
  if (i < NFAC * NF) {
    const int off = A.nbr[(size_t)eg * NFAC * NF + i];
    T uv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) uv[c] = (T)A.u[off + c * NP];
    Node<D, T> nv;
    node_from_u<D, T>(uv, A.G, nv);
    if (!nv.ok) atomicOr(A.err, 1);
    node_powers<D, T>(A.G, nv);
    Node<D, T> nk = n;
    node_powers<D, T>(A.G, nk);
    T ft[NC];
    facet_term<D, T>(nk, nv, avec, A.G, A.diss != 0, ft);
#pragma unroll
    for (int c = 0; c < NC; ++c) r[c] -= ft[c] * iH;
  }
  const int uo = A.uoff[eg];
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    A.r[uo + c * NP + i] = r[c];
    s += (double)n.w[c] * (double)r[c];
  }
  ent += (double)H * s;
}

// ---------------------------------------------------------------------------
// Entropy split, 3D affine tetrahedra.  With Q_l = S_l + E_l/2 (S_l skew,
// E_l diagonal) every contraction uses the skew reference operators:
//   vol    = sum_l M_l fhat_l = (c_b - 1) sum_l S_l fhat_l + (c_b + 1)/2 sum_l E_l fhat_l,
//            fhat_l = sum_i Lambda_il f^(i)
//   D_xi w = J^-1 sum_l Lambda_il h^-1 (S_l w + E_l w / 2)
// With VISC (Navier-Stokes, Baumann-Oden SATs, Sec. 5):
//   sum_i D_xi F^V(i) - 1/2 H^-1 sum_j D_xj^T y_j
//     = H^-1 [ sum_l Q_l FVhat_l + sum_l Q_l^T y'_l ]
//     = H^-1 [ sum_l S_l (FVhat_l - y'_l) + 1/2 sum_l E_l (FVhat_l + y'_l) ]
//   with FVhat_l = sum_i Lambda_il F^V(i), y'_l = -1/2 H^-1 sum_j Lambda_jl y_j,
//   y_j = sum_i K~_ij^T (B n_i (w_k - w_v)) at facet nodes, plus the facet
//   flux jump -1/2 H^-1 (q_k + q_v), q = B n . F^V from the pre-pass.
//
// This contraction kernel serves the Navier-Stokes residual (VISC); the Euler
// terms alone run in the row form (k_split3v).  A workgroup takes a tile of
// CT column tiles (3 elements x 5 components per 16 columns); wave w owns row
// tile mt = w % MT of the operators (its A
// fragments of S_1, S_2, S_3 stay in registers for the whole persistent
// launch) and the column tiles t = w / MT (mod 4 / MT).
template <int P, typename T> struct Wave3;
template <> struct Wave3<1, double> { static constexpr int CT = 4; };
template <> struct Wave3<2, double> { static constexpr int CT = 2; };
template <> struct Wave3<3, double> { static constexpr int CT = 1; };
template <> struct Wave3<1, float> { static constexpr int CT = 8; };
template <> struct Wave3<2, float> { static constexpr int CT = 4; };
template <> struct Wave3<3, float> { static constexpr int CT = 2; };

template <int P, typename T, bool VISC>
__global__ __launch_bounds__(kThreads) void k_split3(KArgs<T> A) {
  constexpr int D = 3, NC = 5, NFAC = 4;
  constexpr int NP = Shape<3, P>::NP, NF = Shape<3, P>::NF, NFN = NFAC * NF;
  constexpr int KP = ru(NP, 4), MP = ru(NP, 16), MT = MP / 16, KS = KP / 4;
  constexpr int WPM = kWaves / MT;  // waves per row tile
  constexpr int CT = Wave3<P, T>::CT, EB = 3 * CT, NCOL = 16 * CT;
  constexpr int NG = VISC ? 5 : 4;  // output slots: S fhat, S_l w (3), [S z]
  constexpr int NPT = (EB * NP + kThreads - 1) / kThreads;
  static_assert(CT % WPM == 0, "column tiles must split evenly over the waves of a row tile");
  typedef typename MF<T>::v4 V4;
  constexpr int MR = KP > MP ? KP : MP;
  // inputs [fhat_1 fhat_2 fhat_3 w][node < KP][column] (VISC: later z_l in slots 0..2);
  // without VISC the outputs reuse this buffer (MR rows per slot)
  __shared__ T Bi[4][MR][NCOL];
  // outputs [S fhat | S_1 w | S_2 w | S_3 w | S z][row][column]
  __shared__ T Bo[VISC ? NG : 1][VISC ? MP : 1][VISC ? NCOL : 1];
  __shared__ T gs[EB][10];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kr = lane >> 4;
  const int mt = wave % MT;
  T(*Out)[MP][NCOL] = VISC ? reinterpret_cast<T(*)[MP][NCOL]>(&Bo[0][0][0])
                           : reinterpret_cast<T(*)[MP][NCOL]>(&Bi[0][0][0]);
  // A fragments of S_1, S_2, S_3 for row tile mt: lane holds S_l[mt*16 + col][4 ks + kr]
  T sf[3][KS];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int m = mt * 16 + col, k = 4 * ks + kr;
      sf[l][ks] = (m < NP && k < NP) ? A.op.S[(l * NP + m) * NP + k] : (T)0;
    }
  const T cb = A.G.cb;
  const T hv = cb - (T)1, he = (T)0.5 * (cb + (T)1);
  double ent = 0.0;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int e0 = tile * EB;
    const int ne = min(EB, A.n_elem - e0);
    __syncthreads();
    for (int x = tid; x < EB * 10; x += kThreads) {
      const int e = x / 10;
      gs[e][x % 10] = e < ne ? (T)A.geo[(size_t)(e0 + e) * 10 + x % 10] : (T)0;
    }
    // zero the inputs (padding rows and columns, ragged elements)
    for (int x = tid; x < 4 * MR * NCOL; x += kThreads) (&Bi[0][0][0])[x] = (T)0;
    __syncthreads();
    // pointwise: contravariant fluxes and entropy variables; node states kept
    // in registers for the later phases
    Node<D, T> nodes[NPT];
#pragma unroll
    for (int kq = 0; kq < NPT; ++kq) {
      const int x = tid + kq * kThreads;
      if (x >= ne * NP) break;
      const int e = x / NP, j = x % NP;
      const int cc = (e / 3) * 16 + (e % 3) * NC;
      const int uo = A.uoff[e0 + e];
      T uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + j];
      Node<D, T> &n = nodes[kq];
      node_from_u<D, T>(uu, A.G, n);
      if (!n.ok) atomicOr(A.err, 1);
      T f[D][NC];
#pragma unroll
      for (int i = 0; i < D; ++i) flux_i<D, T>(n, uu[NC - 1], i, f[i]);
      const T *Lam = gs[e];
#pragma unroll
      for (int l = 0; l < D; ++l)
#pragma unroll
        for (int c = 0; c < NC; ++c)
          Bi[l][j][cc + c] = Lam[0 * 3 + l] * f[0][c] + Lam[1 * 3 + l] * f[1][c] + Lam[2 * 3 + l] * f[2][c];
#pragma unroll
      for (int c = 0; c < NC; ++c) Bi[3][j][cc + c] = n.w[c];
    }
    __syncthreads();
    // skew contractions: S fhat (K = 3 KP) and S_l w (l = 1..3)
    {
      V4 acc[CT / WPM][4];
#pragma unroll
      for (int tt = 0; tt < CT / WPM; ++tt)
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[tt][g] = V4{0, 0, 0, 0};
#pragma unroll
      for (int tt = 0; tt < CT / WPM; ++tt) {
        const int cc = (wave / MT + tt * WPM) * 16 + col;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int k = 4 * ks + kr;
          const T b0 = Bi[0][k][cc], b1 = Bi[1][k][cc], b2 = Bi[2][k][cc], bw = Bi[3][k][cc];
          acc[tt][0] = MF<T>::mma(sf[0][ks], b0, acc[tt][0]);
          acc[tt][1] = MF<T>::mma(sf[0][ks], bw, acc[tt][1]);
          acc[tt][0] = MF<T>::mma(sf[1][ks], b1, acc[tt][0]);
          acc[tt][2] = MF<T>::mma(sf[1][ks], bw, acc[tt][2]);
          acc[tt][0] = MF<T>::mma(sf[2][ks], b2, acc[tt][0]);
          acc[tt][3] = MF<T>::mma(sf[2][ks], bw, acc[tt][3]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int tt = 0; tt < CT / WPM; ++tt) {
        const int cc = (wave / MT + tt * WPM) * 16 + col;
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) Out[g][mt * 16 + MF<T>::row(kr, ii)][cc] = acc[tt][g][ii];
      }
      __syncthreads();
    }
    T ev[NPT][NC];  // VISC: pointwise part 1/2 sum_l E_l (FVhat_l + y'_l)
    if constexpr (VISC) {
      for (int x = tid; x < 3 * MR * NCOL; x += kThreads) (&Bi[0][0][0])[x] = (T)0;
      __syncthreads();
#pragma unroll
      for (int kq = 0; kq < NPT; ++kq) {
        const int x = tid + kq * kThreads;
        if (x >= ne * NP) break;
        const int e = x / NP, i = x % NP;
        const int cc = (e / 3) * 16 + (e % 3) * NC;
        const Node<D, T> &n = nodes[kq];
        const T *Lam = gs[e];
        const T iJ = (T)1 / Lam[9], ih = (T)1 / (T)A.op.h[i];
        T El[D];
#pragma unroll
        for (int l = 0; l < D; ++l) El[l] = A.op.E[l * NP + i];
        T Dw[D][NC];  // D_xi_l w
#pragma unroll
        for (int l = 0; l < D; ++l)
#pragma unroll
          for (int c = 0; c < NC; ++c) Dw[l][c] = (Out[1 + l][i][cc + c] + (T)0.5 * El[l] * n.w[c]) * ih;
        T gW[D][NC], FV[D][NC];
#pragma unroll
        for (int dir = 0; dir < D; ++dir)
#pragma unroll
          for (int c = 0; c < NC; ++c)
            gW[dir][c] = (Lam[dir * 3 + 0] * Dw[0][c] + Lam[dir * 3 + 1] * Dw[1][c] + Lam[dir * 3 + 2] * Dw[2][c]) * iJ;
        viscous_flux<D, T>(n, A.G, A.V, gW, FV);
        T z[D][NC], yp[D][NC];
#pragma unroll
        for (int l = 0; l < D; ++l)
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            z[l][c] = Lam[0 * 3 + l] * FV[0][c] + Lam[1 * 3 + l] * FV[1][c] + Lam[2 * 3 + l] * FV[2][c];
            yp[l][c] = (T)0;
          }
        if (i < NFN) {
          const int off = A.nbr[(size_t)(e0 + e) * NFN + i];
          T uv[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) uv[c] = (T)A.u[off + c * NP];
          Node<D, T> nv;
          node_from_u<D, T>(uv, A.G, nv);
          T dw[NC], avec[D];
#pragma unroll
          for (int c = 0; c < NC; ++c) dw[c] = n.w[c] - nv.w[c];
#pragma unroll
          for (int dir = 0; dir < D; ++dir)
            avec[dir] = Lam[dir * 3 + 0] * El[0] + Lam[dir * 3 + 1] * El[1] + Lam[dir * 3 + 2] * El[2];
          T y[D][NC];
          viscous_adjoint_facet<D, T>(n, A.G, A.V, avec, dw, y);
          const T sc = (T)(-0.5) / (Lam[9] * (T)A.op.h[i]);
#pragma unroll
          for (int l = 0; l < D; ++l)
#pragma unroll
            for (int c = 0; c < NC; ++c)
              yp[l][c] = sc * (Lam[0 * 3 + l] * y[0][c] + Lam[1 * 3 + l] * y[1][c] + Lam[2 * 3 + l] * y[2][c]);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T s = 0;
#pragma unroll
          for (int l = 0; l < D; ++l) {
            Bi[l][i][cc + c] = z[l][c] - yp[l][c];
            s += El[l] * (z[l][c] + yp[l][c]);
          }
          ev[kq][c] = (T)0.5 * s;
        }
      }
      __syncthreads();
      V4 acc[CT / WPM];
#pragma unroll
      for (int tt = 0; tt < CT / WPM; ++tt) {
        const int cc = (wave / MT + tt * WPM) * 16 + col;
        acc[tt] = V4{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int k = 4 * ks + kr;
#pragma unroll
          for (int l = 0; l < 3; ++l) acc[tt] = MF<T>::mma(sf[l][ks], Bi[l][k][cc], acc[tt]);
        }
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) Out[4][mt * 16 + MF<T>::row(kr, ii)][cc] = acc[tt][ii];
      }
      __syncthreads();
    }
    // per node: combine, A~_i as directional derivatives, viscous terms, facet SATs
#pragma unroll
    for (int kq = 0; kq < NPT; ++kq) {
      const int x = tid + kq * kThreads;
      if (x >= ne * NP) break;
      const int e = x / NP, i = x % NP;
      const int cc = (e / 3) * 16 + (e % 3) * NC;
      const Node<D, T> &n = nodes[kq];
      const T *Lam = gs[e];
      const T J = Lam[9];
      const T iJ = (T)1 / J, ih = (T)1 / (T)A.op.h[i];
      const T H = J * (T)A.op.h[i];
      const T iH = (T)1 / H;
      T El[D];
#pragma unroll
      for (int l = 0; l < D; ++l) El[l] = A.op.E[l * NP + i];
      T avec[D];
#pragma unroll
      for (int dir = 0; dir < D; ++dir)
        avec[dir] = Lam[dir * 3 + 0] * El[0] + Lam[dir * 3 + 1] * El[1] + Lam[dir * 3 + 2] * El[2];
      // E part of the volume term: (c_b + 1)/2 sum_l E_l fhat_l = (c_b + 1)/2 sum_i a_i f^(i)
      T f[D][NC];
#pragma unroll
      for (int d = 0; d < D; ++d) flux_i<D, T>(n, (T)A.u[A.uoff[e0 + e] + (NC - 1) * NP + i], d, f[d]);
      T r[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c)
        r[c] = iH * (hv * Out[0][i][cc + c] + he * (avec[0] * f[0][c] + avec[1] * f[1][c] + avec[2] * f[2][c]));
      T Dw[D][NC];
#pragma unroll
      for (int l = 0; l < D; ++l)
#pragma unroll
        for (int c = 0; c < NC; ++c) Dw[l][c] = (Out[1 + l][i][cc + c] + (T)0.5 * El[l] * n.w[c]) * ih;
#pragma unroll
      for (int dir = 0; dir < D; ++dir) {
        T g[NC], t[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
          g[c] = (Lam[dir * 3 + 0] * Dw[0][c] + Lam[dir * 3 + 1] * Dw[1][c] + Lam[dir * 3 + 2] * Dw[2][c]) * iJ;
        jvp_flux<D, T>(n, A.G, dir, g, t);
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] -= cb * t[c];
      }
      if constexpr (VISC) {
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] += (Out[4][i][cc + c] + ev[kq][c]) * iH;
        if (i < NFN) {
          const T *qk = A.q + ((size_t)(e0 + e) * NFN + i) * NC;
          const T *qv = A.q + (size_t)A.nbrq[(size_t)(e0 + e) * NFN + i] * NC;
#pragma unroll
          for (int c = 0; c < NC; ++c) r[c] -= (T)0.5 * (qk[c] + qv[c]) * iH;
        }
      }
      finish_node<D, NP, NF, T>(A, e0 + e, i, n, H, avec, r, ent);
    }
  }
  block_sum_store(ent, A.ent_part);
}

// Entropy split on affine tetrahedra, row form on the vector ALUs (Euler
// terms): per node pair (i, j)
//   V_i   = sum_j sum_l S_l[i][j] fhat_l,j,   G_l,i = sum_j S_l[i][j] w_j
// (30 FMAs per pair), then vol = (c_b - 1) V + (c_b + 1)/2 sum_l E_l fhat_l and
// D_xi_l w = h^-1 (G_l + E_l w / 2).  One lane per node row; the skew
// operators in LDS for the persistent launch; the tile's fhat and w in LDS.
template <int P, typename T> struct VTile3;
template <typename T> struct VTile3<1, T> { static constexpr int EB = 21; };
template <typename T> struct VTile3<2, T> { static constexpr int EB = 10; };
template <typename T> struct VTile3<3, T> { static constexpr int EB = 4; };

// The 3D Euler split terms run in the row form.  At p = 3 in FP64 its three
// 60 x 60 skew operators would take 86 KB of LDS (one wave per SIMD); there
// the built-in choice reads them through the caches instead (measured on
// MI355X: 2.82 ms against 2.97 ms for the contraction form on 196608
// tetrahedra).  The autotuner may pick the other variant; the viscous
// pre-pass uses the built-in choice.
template <int P, typename T>
constexpr bool skew_from_cache3() {
  return P == 3 && sizeof(T) == 8;
}

template <int P, typename T, bool SG = false>
__global__ __launch_bounds__(kThreads, 2) void k_split3v(KArgs<T> A) {
  constexpr int D = 3, NC = 5;
  constexpr int NP = Shape<3, P>::NP, NF = Shape<3, P>::NF;
  constexpr int EB = VTile3<P, T>::EB;
  static_assert(EB * NP <= kThreads, "one node per lane");
  // SG: the skew operators are read through the caches instead of LDS
  __shared__ T Ss[SG ? 1 : 3][SG ? 1 : NP][SG ? 1 : NP];
  // per node: fhat_1[5] fhat_2[5] fhat_3[5] w[5]; element blocks padded so
  // that the elements sharing a wave read different LDS banks
  constexpr int NDS = NP * 20 + 4;
  __shared__ T nd[EB * NDS];
  __shared__ T gs[EB][10];
  const int tid = threadIdx.x;
  if constexpr (!SG)
    for (int x = tid; x < 3 * NP * NP; x += kThreads) (&Ss[0][0][0])[x] = A.op.S[x];
  const T cb = A.G.cb;
  const T hv = cb - (T)1, he = (T)0.5 * (cb + (T)1);
  double ent = 0.0;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  const int e = tid / NP, i = tid % NP;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    if (!tile_on(A, e0, ne)) continue;  // hybrid scheme: no element of this form
    const bool act = tid < ne * NP && elem_on(A, e0 + e);
    __syncthreads();
    for (int x = tid; x < ne * 10; x += kThreads) gs[x / 10][x % 10] = (T)A.geo[(size_t)(e0 + x / 10) * 10 + x % 10];
    __syncthreads();
    Node<D, T> n;
    T f[D][NC];
    if (act) {
      const int uo = A.uoff[e0 + e];
      T uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + i];
      node_from_u<D, T>(uu, A.G, n);
      if (!n.ok) atomicOr(A.err, 1);
#pragma unroll
      for (int m = 0; m < D; ++m) flux_i<D, T>(n, uu[NC - 1], m, f[m]);
      const T *Lam = gs[e];
      T *v = nd + e * NDS + i * 20;
#pragma unroll
      for (int l = 0; l < D; ++l)
#pragma unroll
        for (int c = 0; c < NC; ++c) v[l * NC + c] = Lam[0 * 3 + l] * f[0][c] + Lam[1 * 3 + l] * f[1][c] + Lam[2 * 3 + l] * f[2][c];
#pragma unroll
      for (int c = 0; c < NC; ++c) v[15 + c] = n.w[c];
    }
    __syncthreads();
    if (act) {
      T V[NC], G[D][NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        V[c] = (T)0;
#pragma unroll
        for (int l = 0; l < D; ++l) G[l][c] = (T)0;
      }
#pragma unroll 2
      for (int j = 0; j < NP; ++j) {
        T s0, s1, s2;
        if constexpr (SG) {
          // S_l is stored exactly skew (S^T = -S bitwise): S_l[i][j] is read
          // as -S_l[j][i], so consecutive rows i of a wave read consecutive
          // addresses (a few cache lines per load instead of one per lane)
          s0 = -A.op.S[(0 * NP + j) * NP + i];
          s1 = -A.op.S[(1 * NP + j) * NP + i];
          s2 = -A.op.S[(2 * NP + j) * NP + i];
        } else {
          s0 = Ss[0][i][j];
          s1 = Ss[1][i][j];
          s2 = Ss[2][i][j];
        }
        const T *v = nd + e * NDS + j * 20;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          V[c] += s0 * v[c];  // one FMA per product
          V[c] += s1 * v[5 + c];
          V[c] += s2 * v[10 + c];
          G[0][c] += s0 * v[15 + c];
          G[1][c] += s1 * v[15 + c];
          G[2][c] += s2 * v[15 + c];
        }
      }
      const T *Lam = gs[e];
      const T J = Lam[9], iJ = (T)1 / J;
      const T h = (T)A.op.h[i], ih = (T)1 / h;
      const T H = J * h, iH = (T)1 / H;
      T El[D];
#pragma unroll
      for (int l = 0; l < D; ++l) El[l] = A.op.E[l * NP + i];
      T avec[D];
#pragma unroll
      for (int dir = 0; dir < D; ++dir)
        avec[dir] = Lam[dir * 3 + 0] * El[0] + Lam[dir * 3 + 1] * El[1] + Lam[dir * 3 + 2] * El[2];
      T r[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c)
        r[c] = iH * (hv * V[c] + he * (avec[0] * f[0][c] + avec[1] * f[1][c] + avec[2] * f[2][c]));
      T Dw[D][NC];
#pragma unroll
      for (int l = 0; l < D; ++l)
#pragma unroll
        for (int c = 0; c < NC; ++c) Dw[l][c] = (G[l][c] + (T)0.5 * El[l] * n.w[c]) * ih;
#pragma unroll
      for (int dir = 0; dir < D; ++dir) {
        T g[NC], t[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
          g[c] = (Lam[dir * 3 + 0] * Dw[0][c] + Lam[dir * 3 + 1] * Dw[1][c] + Lam[dir * 3 + 2] * Dw[2][c]) * iJ;
        jvp_flux<D, T>(n, A.G, dir, g, t);
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] -= cb * t[c];
      }
      finish_node<D, NP, NF, T>(A, e0 + e, i, n, H, avec, r, ent);
    }
  }
  block_sum_store(ent, A.ent_part);
}

// Entropy split, tetrahedra with quadratic maps (Assumption 1: p >= 2).  At
// every node the metric cofactors Lambda_il = J dxi_l/dx_i and J follow from
// the element's ten map nodes and the map basis derivatives at the node.
// The node-pair sums take the metric average of the two nodes, as on curved
// triangles:
//   V_i    = sum_j sum_l S_l[i][j] sum_m (Lambda_ml(i) + Lambda_ml(j)) f^(m)_j
//   X_k,i  = sum_j sum_l S_l[i][j] (Lambda_kl(i) + Lambda_kl(j)) w_j
//   vol    = (c_b-1)/2 V + (c_b+1)/2 sum_m a_m f^(m),  a_m = sum_l Lambda_ml E_l
//   D_xk w = (X_k + a_k w) / (2 H),  H = J h.
// One lane per node row; node values of the tile (fluxes, w, Lambda) in LDS;
// the skew operators are read through the caches (rows read transposed, S
// being stored exactly skew).
template <int P, typename T>
__global__ __launch_bounds__(kThreads, 2) void k_split3c(KArgs<T> A) {
  constexpr int D = 3, NC = 5;
  constexpr int NP = Shape<3, P>::NP, NF = Shape<3, P>::NF;
  constexpr int EB = VTile3<P, T>::EB;
  static_assert(EB * NP <= kThreads, "one node per lane");
  // per node: f^(1)[5] f^(2)[5] f^(3)[5] w[5] Lambda[9] (odd stride: rows of
  // the lanes of a wave fall in different banks)
  constexpr int NV = 29;
  constexpr int NDS = NP * NV;
  __shared__ T nd[EB * NDS];
  __shared__ T gs[EB][30];
  const int tid = threadIdx.x;
  const T cb = A.G.cb;
  const T hv = (T)0.5 * (cb - (T)1), he = (T)0.5 * (cb + (T)1);
  double ent = 0.0;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  const int e = tid / NP, i = tid % NP;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    if (!tile_on(A, e0, ne)) continue;  // hybrid scheme: no element of this form
    const bool act = tid < ne * NP && elem_on(A, e0 + e);
    __syncthreads();
    for (int x = tid; x < ne * 30; x += kThreads) gs[x / 30][x % 30] = map_node<T>(A.geo + (size_t)(e0 + x / 30) * 30, x % 30, x % 3);
    __syncthreads();
    Node<D, T> n;
    T L[D][D], J = (T)1;
    if (act) {
      // F_kl = dx_k/dxi_l at node i; Lambda = cofactor matrix of F
      T F[D][D];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int l = 0; l < D; ++l) F[k][l] = (T)0;
      const T *g = gs[e];
#pragma unroll
      for (int a = 0; a < 10; ++a) {
#pragma unroll
        for (int l = 0; l < D; ++l) {
          const T d = A.op.dN[(l * 10 + a) * NP + i];
#pragma unroll
          for (int k = 0; k < D; ++k) F[k][l] += d * g[a * 3 + k];
        }
      }
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int l = 0; l < D; ++l) {
          const int k1 = (k + 1) % 3, k2 = (k + 2) % 3, l1 = (l + 1) % 3, l2 = (l + 2) % 3;
          L[k][l] = F[k1][l1] * F[k2][l2] - F[k1][l2] * F[k2][l1];
        }
      J = F[0][0] * L[0][0] + F[0][1] * L[0][1] + F[0][2] * L[0][2];
      const int uo = A.uoff[e0 + e];
      T uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + i];
      node_from_u<D, T>(uu, A.G, n);
      if (!n.ok) atomicOr(A.err, 1);
      // the fluxes go to LDS only (read back after the pair loop: fewer live
      // registers across it)
      T *v = nd + e * NDS + i * NV;
#pragma unroll
      for (int m = 0; m < D; ++m) flux_i<D, T>(n, uu[NC - 1], m, v + m * NC);
#pragma unroll
      for (int c = 0; c < NC; ++c) v[15 + c] = n.w[c];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int l = 0; l < D; ++l) v[20 + k * 3 + l] = L[k][l];
    }
    __syncthreads();
    if (act) {
      T V[NC], X[D][NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        V[c] = (T)0;
#pragma unroll
        for (int k = 0; k < D; ++k) X[k][c] = (T)0;
      }
#pragma unroll (P >= 3 ? 2 : 1)
      for (int j = 0; j < NP; ++j) {
        const T s0 = -A.op.S[(0 * NP + j) * NP + i];
        const T s1 = -A.op.S[(1 * NP + j) * NP + i];
        const T s2 = -A.op.S[(2 * NP + j) * NP + i];
        const T *v = nd + e * NDS + j * NV;
        T cm[D];
#pragma unroll
        for (int m = 0; m < D; ++m)
          cm[m] = s0 * (L[m][0] + v[20 + m * 3 + 0]) + s1 * (L[m][1] + v[20 + m * 3 + 1]) +
                  s2 * (L[m][2] + v[20 + m * 3 + 2]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          V[c] += cm[0] * v[c];  // one FMA per product
          V[c] += cm[1] * v[5 + c];
          V[c] += cm[2] * v[10 + c];
          X[0][c] += cm[0] * v[15 + c];
          X[1][c] += cm[1] * v[15 + c];
          X[2][c] += cm[2] * v[15 + c];
        }
      }
      const T H = J * (T)A.op.h[i], iH = (T)1 / H;
      T El[D], avec[D];
#pragma unroll
      for (int l = 0; l < D; ++l) El[l] = A.op.E[l * NP + i];
#pragma unroll
      for (int m = 0; m < D; ++m) avec[m] = L[m][0] * El[0] + L[m][1] * El[1] + L[m][2] * El[2];
      const T *fi = nd + e * NDS + i * NV;
      T r[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c)
        r[c] = iH * (hv * V[c] + he * (avec[0] * fi[c] + avec[1] * fi[NC + c] + avec[2] * fi[2 * NC + c]));
#pragma unroll
      for (int dir = 0; dir < D; ++dir) {
        T gg[NC], tt[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) gg[c] = (T)0.5 * iH * (X[dir][c] + avec[dir] * n.w[c]);
        jvp_flux<D, T>(n, A.G, dir, gg, tt);
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] -= cb * tt[c];
      }
      finish_node<D, NP, NF, T>(A, e0 + e, i, n, H, avec, r, ent);
    }
  }
  block_sum_store(ent, A.ent_part);
}

// Viscous facet-flux pre-pass, 3D affine: q = B n . F^V(w, grad w) at the
// facet nodes of every element, in the row form of k_split3v: one lane per
// facet node row i, G_l,i = sum_j S_l[i][j] w_j (15 FMAs per pair), then
// D_xi_l w = h^-1 (G_l + E_l w / 2) and grad w = J^-1 Lambda D_xi w.  Only the
// facet rows are formed; w of all nodes of the tile sits in LDS.
template <int P, typename T>
__global__ __launch_bounds__(kThreads) void k_visc_q3(KArgs<T> A) {
  constexpr int D = 3, NC = 5, NFAC = 4;
  constexpr int NP = Shape<3, P>::NP, NF = Shape<3, P>::NF, NFN = NFAC * NF;
  constexpr int EB = VTile3<P, T>::EB;
  constexpr bool SG = skew_from_cache3<P, T>();
  static_assert(EB * NP <= kThreads && EB * NFN <= kThreads, "one node per lane");
  constexpr int NDW = NP * NC + 4;  // padded element blocks of w
  __shared__ T Ss[SG ? 1 : 3][SG ? 1 : NP][SG ? 1 : NP];
  __shared__ T wd[EB * NDW];
  __shared__ T gs[EB][10];
  const int tid = threadIdx.x;
  if constexpr (!SG)
    for (int x = tid; x < 3 * NP * NP; x += kThreads) (&Ss[0][0][0])[x] = A.op.S[x];
  const int ntiles = (A.n_elem + EB - 1) / EB;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    __syncthreads();
    for (int x = tid; x < ne * 10; x += kThreads) gs[x / 10][x % 10] = (T)A.geo[(size_t)(e0 + x / 10) * 10 + x % 10];
    if (tid < ne * NP) {
      const int e = tid / NP, j = tid % NP;
      const int uo = A.uoff[e0 + e];
      T uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + j];
      Node<D, T> n;
      node_from_u<D, T>(uu, A.G, n);
#pragma unroll
      for (int c = 0; c < NC; ++c) wd[e * NDW + j * NC + c] = n.w[c];
    }
    __syncthreads();
    if (tid < ne * NFN) {
      const int e = tid / NFN, i = tid % NFN;
      T G[D][NC];
#pragma unroll
      for (int l = 0; l < D; ++l)
#pragma unroll
        for (int c = 0; c < NC; ++c) G[l][c] = (T)0;
#pragma unroll 2
      for (int j = 0; j < NP; ++j) {
        T s0, s1, s2;
        if constexpr (SG) {
          // S_l is stored exactly skew (S^T = -S bitwise): S_l[i][j] is read
          // as -S_l[j][i], so consecutive rows i of a wave read consecutive
          // addresses (a few cache lines per load instead of one per lane)
          s0 = -A.op.S[(0 * NP + j) * NP + i];
          s1 = -A.op.S[(1 * NP + j) * NP + i];
          s2 = -A.op.S[(2 * NP + j) * NP + i];
        } else {
          s0 = Ss[0][i][j];
          s1 = Ss[1][i][j];
          s2 = Ss[2][i][j];
        }
        const T *w = wd + e * NDW + j * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          G[0][c] += s0 * w[c];
          G[1][c] += s1 * w[c];
          G[2][c] += s2 * w[c];
        }
      }
      const int uo = A.uoff[e0 + e];
      T uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + i];
      Node<D, T> n;
      node_from_u<D, T>(uu, A.G, n);
      const T *Lam = gs[e];
      const T iJ = (T)1 / Lam[9];
      const T ih = (T)1 / (T)A.op.h[i];
      T El[D];
#pragma unroll
      for (int l = 0; l < D; ++l) El[l] = A.op.E[l * NP + i];
#pragma unroll
      for (int l = 0; l < D; ++l)
#pragma unroll
        for (int c = 0; c < NC; ++c) G[l][c] = (G[l][c] + (T)0.5 * El[l] * n.w[c]) * ih;
      T gW[D][NC], FV[D][NC];
#pragma unroll
      for (int dir = 0; dir < D; ++dir)
#pragma unroll
        for (int c = 0; c < NC; ++c)
          gW[dir][c] = (Lam[dir * 3 + 0] * G[0][c] + Lam[dir * 3 + 1] * G[1][c] + Lam[dir * 3 + 2] * G[2][c]) * iJ;
      viscous_flux<D, T>(n, A.G, A.V, gW, FV);
      T avec[D];
#pragma unroll
      for (int dir = 0; dir < D; ++dir)
        avec[dir] = Lam[dir * 3 + 0] * El[0] + Lam[dir * 3 + 1] * El[1] + Lam[dir * 3 + 2] * El[2];
#pragma unroll
      for (int c = 0; c < NC; ++c)
        A.qout[((size_t)(e0 + e) * NFN + i) * NC + c] = avec[0] * FV[0][c] + avec[1] * FV[1][c] + avec[2] * FV[2][c];
    }
  }
}

// ---------------------------------------------------------------------------
// Entropy split, 2D triangles with per-node metrics of a quadratic map.
//
// With Q_l = S_l + E_l/2 (S_l skew, E_l diagonal for diagonal-E operators)
// and M_l = c_b Q_l + Q_l^T = (c_b - 1) S_l + (c_b + 1)/2 E_l, the curved
// split terms
//   sum_i [c_b Q_xi + Q_xi^T] f^(i) = 1/2 sum_l [ sum_i Lambda_il o (M_l f^(i)) + M_l fhat_l ]
//   Q_xi w                           = 1/2 sum_l [ Lambda_il o (Q_l w) + Q_l (Lambda_il o w) ]
// become, with a_i = sum_l Lambda_il E_l (the facet B n_i, zero off the facets),
//   vol    = (c_b - 1)/2 V + (c_b + 1)/2 sum_m a_m f^(m)
//   Q_xi w = 1/2 X_i + 1/2 a_i w
// and, per node pair (i, j), onto the metric average Lambda(i) + Lambda(j):
//   V_i   = sum_j sum_l S_l[i][j] sum_m (Lambda_ml(i) + Lambda_ml(j)) f^(m)_j
//   X_k,i = sum_j sum_l S_l[i][j] (Lambda_kl(i) + Lambda_kl(j)) w_j
// (20 FMAs per pair).  On MI355X an FP64 MFMA has the throughput of the FP64
// vector ALUs, and the contraction form of the same terms issues about five
// times these flops (six column groups per direction for curved metrics,
// 16-row padding), so the pair sums run on the vector ALUs: R node rows per
// lane (rows k and k + n_p/2 for R = 2), the skew operators in LDS, the
// tile's node values (f^(0), f^(1), w, Lambda) in LDS rows of 16 values per
// node.  Every lane re-reads the 16 values of node j for each pair; with
// R = 2 each value read feeds two rows (half the LDS bytes per FMA, at two
// waves per SIMD instead of three for R = 1).
template <int P, typename T, int R, int EF = 0>
struct Split2 {
  static constexpr int D = 2, NC = 4, NFAC = 3;
  static constexpr int NP = Shape<2, P>::NP, NF = Shape<2, P>::NF;
  static_assert(NP % R == 0, "rows split evenly over the lanes of an element");
  static constexpr int L = NP / R;            // lanes per element
  static constexpr int EB = kThreads / L;     // elements per tile
  // node rows of 16 values; element blocks padded by 4 values so that the
  // rows of the elements sharing a wave fall in different LDS banks
  static constexpr int NDS = NP * 16 + 4;
  // S[j][i] = (S_0[i][j], S_1[i][j]): a row's two entries in one read, the
  // rows of consecutive lanes at consecutive addresses
  typedef HIP_vector_type<T, 2> T2;
  struct Lds {
    T2 S[NP][NP];
    __align__(16) T nd[EB * NDS];  // per node: f0[4] f1[4] w[4] Lambda_00 _01 _10 _11
  };

  __device__ static __forceinline__ void load_ops(const KArgs<T> &A, Lds &L_) {
    for (int x = threadIdx.x; x < NP * NP; x += kThreads) {
      const int i = x / NP, j = x % NP;
      L_.S[j][i] = T2(A.op.S[x], A.op.S[NP * NP + x]);
    }
  }

  // Residual of the elements [tile*EB, tile*EB + EB); ent accumulates w^T H r.
  // Call with the operators loaded (load_ops, then a barrier).
  __device__ static __forceinline__ void tile(const KArgs<T> &A, Lds &L_, int tl, double &ent) {
    const int tid = threadIdx.x;
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    if (!tile_on(A, e0, ne)) return;  // hybrid scheme: no element of this form
    const int e = tid / L, k = tid % L;
    const bool act = e < ne && elem_on(A, e0 + e);
    const T cb = A.G.cb;
    const T hv = (T)0.5 * (cb - (T)1), he = (T)0.5 * (cb + (T)1);
    Node<D, T> n[R];
    T lam[R][4];
    if (act) {
      const double *g = A.geo + (size_t)(e0 + e) * 12;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = k + q * L;
        T F[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          const T d0 = A.op.dN[(0 * 6 + a) * NP + i], d1 = A.op.dN[(1 * 6 + a) * NP + i];
          const T gx = map_node<T>(g, 2 * a, 0), gy = map_node<T>(g, 2 * a + 1, 1);
          F[0][0] += d0 * gx;
          F[0][1] += d1 * gx;
          F[1][0] += d0 * gy;
          F[1][1] += d1 * gy;
        }
        lam[q][0] = F[1][1];   // Lambda_00 = J dxi_0/dx_0
        lam[q][1] = -F[1][0];  // Lambda_01
        lam[q][2] = -F[0][1];  // Lambda_10
        lam[q][3] = F[0][0];   // Lambda_11
        const int uo = A.uoff[e0 + e];
        T uu[NC], f0[NC], f1[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + i];
        node_from_u<D, T>(uu, A.G, n[q]);
        if (!n[q].ok) atomicOr(A.err, 1);
        flux_i<D, T>(n[q], uu[NC - 1], 0, f0);
        flux_i<D, T>(n[q], uu[NC - 1], 1, f1);
        T *v = L_.nd + e * NDS + i * 16;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          v[c] = f0[c];
          v[4 + c] = f1[c];
          v[8 + c] = n[q].w[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) v[12 + c] = lam[q][c];
      }
    }
    __syncthreads();
    if (act) {
      T V[R][NC], X0[R][NC], X1[R][NC];
#pragma unroll
      for (int q = 0; q < R; ++q)
#pragma unroll
        for (int c = 0; c < NC; ++c) V[q][c] = X0[q][c] = X1[q][c] = (T)0;
#pragma unroll 2
      for (int j = 0; j < NP; ++j) {
        const T *v = L_.nd + e * NDS + j * 16;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = k + q * L;
          const T2 sp = L_.S[j][i];
          const T s0 = sp.x, s1 = sp.y;
          const T c0 = s0 * (lam[q][0] + v[12]) + s1 * (lam[q][1] + v[13]);
          const T c1 = s0 * (lam[q][2] + v[14]) + s1 * (lam[q][3] + v[15]);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            // one FMA per product (a sum of products added at once costs
            // a multiply, an FMA and an add)
            V[q][c] += c0 * v[c];
            V[q][c] += c1 * v[4 + c];
            X0[q][c] += c0 * v[8 + c];
            X1[q][c] += c1 * v[8 + c];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = k + q * L;
        const T *v = L_.nd + e * NDS + i * 16;
        const T E0 = A.op.E[i], E1 = A.op.E[NP + i];
        T avec[D];
        avec[0] = lam[q][0] * E0 + lam[q][1] * E1;
        avec[1] = lam[q][2] * E0 + lam[q][3] * E1;
        // J = F_00 F_11 - F_01 F_10 in terms of the cofactors
        const T J = lam[q][3] * lam[q][0] - lam[q][2] * lam[q][1];
        const T H = J * (T)A.op.h[i];
        const T iH = drcp(H);
        T r[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] = iH * (hv * V[q][c] + he * (avec[0] * v[c] + avec[1] * v[4 + c]));
#pragma unroll
        for (int dir = 0; dir < D; ++dir) {
          T gg[NC], tt[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c)
            gg[c] = (T)0.5 * iH * ((dir == 0 ? X0[q][c] : X1[q][c]) + avec[dir] * n[q].w[c]);
          jvp_flux<D, T>(n[q], A.G, dir, gg, tt);
#pragma unroll
          for (int c = 0; c < NC; ++c) r[c] -= cb * tt[c];
        }
        finish_node<D, NP, NF, T>(A, e0 + e, i, n[q], H, avec, r, ent);
      }
    }
    __syncthreads();
  }

  // The same residual with the facet SATs evaluated before the pair sums:
  // the neighbour index and state loads are issued with the element's own
  // loads at the start of the tile, so their latency overlaps the node work
  // instead of following the pair loop; only the facet term (n_c values per
  // row) and the node quantities of the combine stay live across the loop.
  // Neighbour data of one tile's facet rows, loaded ahead of the tile (EF 3):
  // face-node offsets and the neighbour states.
  struct Pref {
    int t;
    int nb[R];
    T uv[R][NC];
  };

  // Face-node offsets of tile tl for this lane's rows (-1: not a facet row).
  __device__ static __forceinline__ void pref_nb(const KArgs<T> &A, int tl, int nb[R]) {
    constexpr int NFN = NFAC * NF;
    const int e = threadIdx.x / L, k = threadIdx.x % L;
    const int e0 = tl * EB;
    const bool ok = tl >= 0 && e < min(EB, A.n_elem - e0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = k + q * L;
      nb[q] = (ok && i < NFN) ? A.nbr[(size_t)(e0 + e) * NFN + i] : -1;
    }
  }

  __device__ static __forceinline__ void pref_uv(const KArgs<T> &A, Pref &pf) {
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int c = 0; c < NC; ++c) pf.uv[q][c] = pf.nb[q] >= 0 ? (T)A.u[pf.nb[q] + c * NP] : (T)0;
  }

  __device__ static __forceinline__ void tile_early(const KArgs<T> &A, Lds &L_, int tl, double &ent,
                                                    Pref *pf = nullptr, int next = -1) {
    constexpr int NFN = NFAC * NF;
    const int tid = threadIdx.x;
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    // EF 3: the next tile's face-node offsets now, its neighbour states
    // during this tile's pair loop
    int nbn[R];
    if constexpr (EF == 3) pref_nb(A, next, nbn);
    if (!tile_on(A, e0, ne)) {  // hybrid scheme: no element of this form
      if constexpr (EF == 3) {
#pragma unroll
        for (int q = 0; q < R; ++q) pf->nb[q] = nbn[q];
        pref_uv(A, *pf);
        pf->t = next;
      }
      return;
    }
    const int e = tid / L, k = tid % L;
    const bool act = e < ne && elem_on(A, e0 + e);
    const T cb = A.G.cb;
    const T hv = (T)0.5 * (cb - (T)1), he = (T)0.5 * (cb + (T)1);
    Node<D, T> n[R];
    T lam[R][4];
    T ft[R][NC];
    T iWn[R], ith[R], ipk[R];  // 1/W_nc = -1/z1, rho/p and 1/p of the row's node
    if (act) {
      const int eg = e0 + e;
      T uu[R][NC], uv[R][NC];
      int nb[R];
      const double *g = A.geo + (size_t)eg * 12;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = k + q * L;
        T F[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          const T d0 = A.op.dN[(0 * 6 + a) * NP + i], d1 = A.op.dN[(1 * 6 + a) * NP + i];
          const T gx = map_node<T>(g, 2 * a, 0), gy = map_node<T>(g, 2 * a + 1, 1);
          F[0][0] += d0 * gx;
          F[0][1] += d1 * gx;
          F[1][0] += d0 * gy;
          F[1][1] += d1 * gy;
        }
        lam[q][0] = F[1][1];   // Lambda_00 = J dxi_0/dx_0
        lam[q][1] = -F[1][0];  // Lambda_01
        lam[q][2] = -F[0][1];  // Lambda_10
        lam[q][3] = F[0][0];   // Lambda_11
      }
      if constexpr (EF == 2) {
        // the state loads after the metric tables: the memory counter is
        // waited on in issue order, so the metrics need not wait for them;
        // the neighbour gathers go last (the node states need not wait for
        // them either)
        const int uo = A.u_dense ? A.u_base + eg * (NC * NP) : A.uoff[eg];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = k + q * L;
          nb[q] = i < NFN ? A.nbr[(size_t)eg * NFN + i] : -1;
#pragma unroll
          for (int c = 0; c < NC; ++c) uu[q][c] = (T)A.u[uo + c * NP + i];
        }
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
          for (int c = 0; c < NC; ++c) uv[q][c] = nb[q] >= 0 ? (T)A.u[nb[q] + c * NP] : uu[q][c];
      }
      if constexpr (EF == 3) {
        // the neighbour data came with the previous tile
        const int uo = A.u_dense ? A.u_base + eg * (NC * NP) : A.uoff[eg];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = k + q * L;
          nb[q] = pf->nb[q];
#pragma unroll
          for (int c = 0; c < NC; ++c) uu[q][c] = (T)A.u[uo + c * NP + i];
        }
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
          for (int c = 0; c < NC; ++c) uv[q][c] = nb[q] >= 0 ? pf->uv[q][c] : uu[q][c];
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = k + q * L;
        T f0[NC], f1[NC];
        node_from_u<D, T>(uu[q], A.G, n[q]);
        if (!n[q].ok) atomicOr(A.err, 1);
        iWn[q] = drcp(n[q].w[NC - 1]);
        ipk[q] = drcp(n[q].p);
        ith[q] = n[q].rho * ipk[q];
        flux_i<D, T>(n[q], uu[q][NC - 1], 0, f0);
        flux_i<D, T>(n[q], uu[q][NC - 1], 1, f1);
        T *v = L_.nd + e * NDS + i * 16;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          v[c] = f0[c];
          v[4 + c] = f1[c];
          v[8 + c] = n[q].w[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) v[12 + c] = lam[q][c];
      }
      {
        // every row evaluates its facet term without branching on whether it
        // is a facet node (interior rows pair with themselves and discard the
        // result), stage by stage across the rows: the rows' transcendental
        // chains are independent and interleave
        Node<D, T> nv[R], nk[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          nk[q] = n[q];
          node_powers<D, T>(A.G, nk[q]);
        }
        // the neighbour's powers follow from the node's by series when the
        // interface jump is small (a continuous state), else from its own
        // logarithms
#pragma unroll
        for (int q = 0; q < R; ++q) {
          if (!node_near<D, T>(uv[q], nk[q], n[q].irho, ipk[q], A.G, *A.jc, nv[q])) {
            node_from_u<D, T>(uv[q], A.G, nv[q]);
            node_powers<D, T>(A.G, nv[q]);
          }
          if (nb[q] >= 0 && !nv[q].ok) atomicOr(A.err, 1);
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = k + q * L;
          const T E0 = A.op.E[i], E1 = A.op.E[NP + i];
          T avec[D];
          avec[0] = lam[q][0] * E0 + lam[q][1] * E1;
          avec[1] = lam[q][2] * E0 + lam[q][3] * E1;
          T f[NC];
          facet_term_c<D, T>(nk[q], nv[q], avec, A.G, A.eac[0], A.eac[1], A.diss != 0, f, ipk[q], -iWn[q]);
#pragma unroll
          for (int c = 0; c < NC; ++c) ft[q][c] = nb[q] >= 0 ? f[c] : (T)0;
        }
      }
    }
    if constexpr (EF == 3) {
      // this tile's neighbour data is consumed: load the next tile's, to
      // arrive during the pair loop
#pragma unroll
      for (int q = 0; q < R; ++q) pf->nb[q] = nbn[q];
      pref_uv(A, *pf);
      pf->t = next;
    }
    __syncthreads();
    if (act) {
      T V[R][NC], X0[R][NC], X1[R][NC];
#pragma unroll
      for (int q = 0; q < R; ++q)
#pragma unroll
        for (int c = 0; c < NC; ++c) V[q][c] = X0[q][c] = X1[q][c] = (T)0;
#pragma unroll 2
      for (int j = 0; j < NP; ++j) {
        const T *v = L_.nd + e * NDS + j * 16;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = k + q * L;
          const T2 sp = L_.S[j][i];
          const T s0 = sp.x, s1 = sp.y;
          const T c0 = s0 * (lam[q][0] + v[12]) + s1 * (lam[q][1] + v[13]);
          const T c1 = s0 * (lam[q][2] + v[14]) + s1 * (lam[q][3] + v[15]);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            V[q][c] += c0 * v[c];
            V[q][c] += c1 * v[4 + c];
            X0[q][c] += c0 * v[8 + c];
            X1[q][c] += c1 * v[8 + c];
          }
        }
      }
      const int uo = A.u_dense ? A.u_base + (e0 + e) * (NC * NP) : A.uoff[e0 + e];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = k + q * L;
        const T *v = L_.nd + e * NDS + i * 16;
        const T E0 = A.op.E[i], E1 = A.op.E[NP + i];
        T avec[D];
        avec[0] = lam[q][0] * E0 + lam[q][1] * E1;
        avec[1] = lam[q][2] * E0 + lam[q][3] * E1;
        const T J = lam[q][3] * lam[q][0] - lam[q][2] * lam[q][1];
        const T H = J * (T)A.op.h[i];
        const T iH = drcp(H);
        T r[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] = iH * (hv * V[q][c] + he * (avec[0] * v[c] + avec[1] * v[4 + c]));
        {
          T gg[D][NC], tt[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            gg[0][c] = (T)0.5 * iH * (X0[q][c] + avec[0] * n[q].w[c]);
            gg[1][c] = (T)0.5 * iH * (X1[q][c] + avec[1] * n[q].w[c]);
          }
          jvp_flux_sum<D, T>(n[q], A.G, iWn[q], ith[q], gg, tt);
#pragma unroll
          for (int c = 0; c < NC; ++c) r[c] -= cb * tt[c];
        }
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          r[c] -= ft[q][c] * iH;
          A.r[uo + c * NP + i] = r[c];
          s += (double)n[q].w[c] * (double)r[c];
        }
        ent += (double)H * s;
      }
    }
    __syncthreads();
  }
};

// Rows per lane of the built-in 2D split variant; the autotuner may pick the other.
template <int P, typename T> constexpr int split2_rows() { return 2; }

template <int P, typename T, int R, int EF = 0>
__global__ __launch_bounds__(kThreads, R == 2 ? 2 : (P == 1 ? 2 : 3)) void k_split2(KArgs<T> A) {
  typedef Split2<P, T, R, EF> K;
  __shared__ typename K::Lds lds;
  // launch timing: the earliest workgroup start and the latest workgroup end
  // on the device's constant-rate clock
  if (A.tstamp && threadIdx.x == 0) atomicMin(&A.tstamp[0], (unsigned long long)wall_clock64());
  K::load_ops(A, lds);
  __syncthreads();
  double ent = 0.0;
  const int ntiles = (A.n_elem + K::EB - 1) / K::EB;
  if constexpr (EF == 3) {
    typename K::Pref pf;
    TileSeq ts(ntiles);
    pf.t = ts.t < ts.end ? ts.t : -1;
    K::pref_nb(A, pf.t, pf.nb);
    K::pref_uv(A, pf);
    for (; ts.t < ts.end; ts.t += ts.step)
      K::tile_early(A, lds, ts.t, ent, &pf, ts.t + ts.step < ts.end ? ts.t + ts.step : -1);
  } else {
    for (TileSeq ts(ntiles); ts.t < ts.end; ts.t += ts.step) {
      if constexpr (EF != 0)
        K::tile_early(A, lds, ts.t, ent);
      else
        K::tile(A, lds, ts.t, ent);
    }
  }
  block_sum_store(ent, A.ent_part);
  if (A.tstamp && threadIdx.x == 0) atomicMax(&A.tstamp[1], (unsigned long long)wall_clock64());
}

// All degree classes of a 2D mesh (batched problems) in one persistent
// launch; a workgroup restages the skew operators when its tile changes
// degree.
template <typename T>
constexpr size_t split2_lds_max() {
  size_t m = sizeof(typename Split2<1, T, split2_rows<1, T>()>::Lds);
  m = m > sizeof(typename Split2<2, T, split2_rows<2, T>()>::Lds) ? m : sizeof(typename Split2<2, T, split2_rows<2, T>()>::Lds);
  m = m > sizeof(typename Split2<3, T, split2_rows<3, T>()>::Lds) ? m : sizeof(typename Split2<3, T, split2_rows<3, T>()>::Lds);
  m = m > sizeof(typename Split2<4, T, split2_rows<4, T>()>::Lds) ? m : sizeof(typename Split2<4, T, split2_rows<4, T>()>::Lds);
  return m;
}

template <typename T>
__global__ __launch_bounds__(kThreads, sizeof(T) == 8 ? 2 : 3) void k_split2_batch(Batch2<T> Bt) {
  __shared__ __align__(16) unsigned char raw[split2_lds_max<T>()];
  if (Bt.tstamp && threadIdx.x == 0) atomicMin(&Bt.tstamp[0], (unsigned long long)wall_clock64());
  double ent = 0.0;
  int cur = -1;
  // Tile order: with a grid that is a multiple of the XCD count, each XCD
  // takes a contiguous share of every degree class (the facet neighbours of
  // its elements then mostly sit in its own L2), chains its shares from the
  // highest degree down (the costliest tiles first, the launch's tail made
  // of the cheapest), and its workgroups deal the chain round-robin, so the
  // work per workgroup is even to one tile whatever the classes cost.
  const bool xa = gridDim.x % kXcds == 0;
  const int nx = xa ? kXcds : 1, x = xa ? blockIdx.x % kXcds : 0;
  const int lg = gridDim.x / nx, lb = xa ? blockIdx.x / kXcds : blockIdx.x;
  int beg[4], len[4], total = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int n = Bt.g0[c + 1] - Bt.g0[c];
    const int per = (n + nx - 1) / nx;
    beg[c] = min(n, x * per);
    len[c] = min(n, beg[c] + per) - beg[c];
    total += len[c];
  }
  for (int pos = lb; pos < total; pos += lg) {
    // the class of chain position pos (pos < total, so one of the four)
    int q, t = pos;
    if (t < len[3]) {
      q = 3;
      t += beg[3];
    } else if ((t -= len[3]) < len[2]) {
      q = 2;
      t += beg[2];
    } else if ((t -= len[2]) < len[1]) {
      q = 1;
      t += beg[1];
    } else {
      t -= len[1];
      q = 0;
      t += beg[0];
    }
    const int g = Bt.g0[q] + t;
    if (q != cur) {
      __syncthreads();
      if (q == 0) Split2<1, T, split2_rows<1, T>()>::load_ops(batch_args(Bt, 0), *(typename Split2<1, T, split2_rows<1, T>()>::Lds *)raw);
      else if (q == 1) Split2<2, T, split2_rows<2, T>()>::load_ops(batch_args(Bt, 1), *(typename Split2<2, T, split2_rows<2, T>()>::Lds *)raw);
      else if (q == 2) Split2<3, T, split2_rows<3, T>()>::load_ops(batch_args(Bt, 2), *(typename Split2<3, T, split2_rows<3, T>()>::Lds *)raw);
      else Split2<4, T, split2_rows<4, T>()>::load_ops(batch_args(Bt, 3), *(typename Split2<4, T, split2_rows<4, T>()>::Lds *)raw);
      __syncthreads();
      cur = q;
    }
    if (q == 0) Split2<1, T, split2_rows<1, T>(), 2>::tile_early(batch_args(Bt, 0), *(typename Split2<1, T, split2_rows<1, T>(), 2>::Lds *)raw, g, ent);
    else if (q == 1) Split2<2, T, split2_rows<2, T>(), 2>::tile_early(batch_args(Bt, 1), *(typename Split2<2, T, split2_rows<2, T>(), 2>::Lds *)raw, g - Bt.g0[1], ent);
    else if (q == 2) Split2<3, T, split2_rows<3, T>(), 2>::tile_early(batch_args(Bt, 2), *(typename Split2<3, T, split2_rows<3, T>(), 2>::Lds *)raw, g - Bt.g0[2], ent);
    else Split2<4, T, split2_rows<4, T>(), 2>::tile_early(batch_args(Bt, 3), *(typename Split2<4, T, split2_rows<4, T>(), 2>::Lds *)raw, g - Bt.g0[3], ent);
  }
  block_sum_store(ent, Bt.ent_part);
  if (Bt.tstamp && threadIdx.x == 0) atomicMax(&Bt.tstamp[1], (unsigned long long)wall_clock64());
}

// ---------------------------------------------------------------------------
// Hadamard form (comparator): r_m = -H_m^-1 sum_{n != m} sum_l S_l[m][n]
//   sum_i (Lambda_il(m) + Lambda_il(n)) F*_i(u_m, u_n).
// One lane per node row: the lane sums the two-point fluxes of its row over
// all other nodes of the element (each pair is evaluated by both of its
// rows; no atomics, fixed order, no pair buffer).  The skew operators are
// staged in LDS once per persistent workgroup; node values (V, p, z1 and the
// flux powers) of the tile sit in LDS with the node index fastest.
template <int DIM, int P, typename T> struct HadTile;
template <> struct HadTile<2, 1, double> { static constexpr int EB = 42; };
template <> struct HadTile<2, 2, double> { static constexpr int EB = 25; };
template <> struct HadTile<2, 3, double> { static constexpr int EB = 14; };
template <> struct HadTile<2, 4, double> { static constexpr int EB = 11; };
template <> struct HadTile<3, 1, double> { static constexpr int EB = 21; };
template <> struct HadTile<3, 2, double> { static constexpr int EB = 20; };
template <> struct HadTile<3, 3, double> { static constexpr int EB = 8; };
template <> struct HadTile<2, 1, float> { static constexpr int EB = 42; };
template <> struct HadTile<2, 2, float> { static constexpr int EB = 25; };
template <> struct HadTile<2, 3, float> { static constexpr int EB = 14; };
template <> struct HadTile<2, 4, float> { static constexpr int EB = 11; };
template <> struct HadTile<3, 1, float> { static constexpr int EB = 21; };
template <> struct HadTile<3, 2, float> { static constexpr int EB = 20; };
template <> struct HadTile<3, 3, float> { static constexpr int EB = 8; };

// CURVED (3D): quadratic tetrahedral maps, metrics per node from the ten map
// nodes as in k_split3c, and the metric average of the two nodes per pair.
template <int DIM, int P, typename T, bool CURVED = false>
__global__ __launch_bounds__(kThreads) void k_hadamard(KArgs<T> A) {
  constexpr int D = DIM, NC = D + 2;
  constexpr int NP = Shape<DIM, P>::NP, NF = Shape<DIM, P>::NF;
  constexpr int EB = HadTile<DIM, P, T>::EB;
  constexpr int NV = D + 4;  // V, p, z1, P1, P2
  constexpr int NT = (EB * NP + kThreads - 1) / kThreads;
  constexpr bool PN = DIM == 2 || CURVED;  // metrics per node
  constexpr int NM = DIM == 2 ? 5 : (CURVED ? 10 : 1);
  __shared__ T Ss[D][NP][NP];
  __shared__ T nd[NV][EB][NP];
  // per node: 2D Lambda_00, _01, _10, _11, J; curved 3D Lambda (row i, col l), J
  __shared__ T met[NM][EB][PN ? NP : 1];
  __shared__ T gm[EB][CURVED ? 30 : 10];  // 3D: Lambda, J per element (affine) or the map nodes (curved)
  const int tid = threadIdx.x;
  for (int x = tid; x < D * NP * NP; x += kThreads) (&Ss[0][0][0])[x] = A.op.S[x];
  double ent = 0.0;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int e0 = tile * EB;
    const int ne = min(EB, A.n_elem - e0);
    if (!tile_on(A, e0, ne)) continue;  // hybrid scheme: no element of this form
    __syncthreads();
    if constexpr (DIM == 3) {
      constexpr int GS = CURVED ? 30 : 10;
      for (int x = tid; x < ne * GS; x += kThreads)
        gm[x / GS][x % GS] = CURVED ? map_node<T>(A.geo + (size_t)(e0 + x / GS) * GS, x % GS, x % 3)
                                    : (T)A.geo[(size_t)(e0 + x / GS) * GS + x % GS];
      if constexpr (CURVED) __syncthreads();  // the map nodes feed the per-node metrics below
    }
    Node<D, T> nodes[NT];
#pragma unroll
    for (int kq = 0; kq < NT; ++kq) {
      const int x = tid + kq * kThreads;
      if (x >= ne * NP) break;
      const int e = x / NP, j = x % NP;
      if (!elem_on(A, e0 + e)) continue;
      const int uo = A.uoff[e0 + e];
      T uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + j];
      Node<D, T> &n = nodes[kq];
      node_from_u<D, T>(uu, A.G, n);
      if (!n.ok) atomicOr(A.err, 1);
      node_powers<D, T>(A.G, n);
#pragma unroll
      for (int i = 0; i < D; ++i) nd[i][e][j] = n.V[i];
      nd[D][e][j] = n.p;
      nd[D + 1][e][j] = n.z1;
      nd[D + 2][e][j] = n.P1;
      nd[D + 3][e][j] = n.P2;
      if constexpr (DIM == 2) {
        const double *g = A.geo + (size_t)(e0 + e) * 12;
        T F[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          const T d0 = A.op.dN[(0 * 6 + a) * NP + j], d1 = A.op.dN[(1 * 6 + a) * NP + j];
          const T gx = map_node<T>(g, 2 * a, 0), gy = map_node<T>(g, 2 * a + 1, 1);
          F[0][0] += d0 * gx;
          F[0][1] += d1 * gx;
          F[1][0] += d0 * gy;
          F[1][1] += d1 * gy;
        }
        met[0][e][j] = F[1][1];
        met[1][e][j] = -F[1][0];
        met[2][e][j] = -F[0][1];
        met[3][e][j] = F[0][0];
        met[4][e][j] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
      } else if constexpr (CURVED) {
        T F[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 3; ++l) F[k][l] = (T)0;
#pragma unroll
        for (int q = 0; q < 10; ++q)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            const T d = A.op.dN[(l * 10 + q) * NP + j];
#pragma unroll
            for (int k = 0; k < 3; ++k) F[k][l] += d * gm[e][q * 3 + k];
          }
        T J = (T)0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            const int k1 = (k + 1) % 3, k2 = (k + 2) % 3, l1 = (l + 1) % 3, l2 = (l + 2) % 3;
            const T c = F[k1][l1] * F[k2][l2] - F[k1][l2] * F[k2][l1];
            met[k * 3 + l][e][j] = c;
            if (k == 0) J += F[0][l] * c;
          }
        met[9][e][j] = J;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < NT; ++kq) {
      const int x = tid + kq * kThreads;
      if (x >= ne * NP) break;
      const int e = x / NP, m = x % NP;
      if (!elem_on(A, e0 + e)) continue;
      const Node<D, T> &a = nodes[kq];
      T Lm[D][D], J;
      if constexpr (DIM == 2) {
#pragma unroll
        for (int q = 0; q < 4; ++q) Lm[q / 2][q % 2] = met[q][e][m];
        J = met[4][e][m];
      } else if constexpr (CURVED) {
#pragma unroll
        for (int q = 0; q < 9; ++q) Lm[q / 3][q % 3] = met[q][e][m];
        J = met[9][e][m];
      } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) Lm[q / 3][q % 3] = gm[e][q];
        J = gm[e][9];
      }
      T acc[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = (T)0;
      for (int nn = 0; nn < NP; ++nn) {
        if (nn == m) continue;
        Node<D, T> b;
#pragma unroll
        for (int i = 0; i < D; ++i) b.V[i] = nd[i][e][nn];
        b.p = nd[D][e][nn];
        b.z1 = nd[D + 1][e][nn];
        b.P1 = nd[D + 2][e][nn];
        b.P2 = nd[D + 3][e][nn];
        T cvec[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          T s = 0;
#pragma unroll
          for (int l = 0; l < D; ++l) {
            const T lsum = DIM == 2 ? Lm[i][l] + met[i * 2 + l][e][nn]
                                    : (CURVED ? Lm[i][l] + met[i * 3 + l][e][nn] : (T)2 * Lm[i][l]);
            s += Ss[l][m][nn] * lsum;
          }
          cvec[i] = s;
        }
        T out[NC];
        facet_term<D, T>(a, b, cvec, A.G, false, out);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += out[c];
      }
      const T H = J * (T)A.op.h[m];
      const T iH = (T)1 / H;
      T r[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) r[c] = -acc[c] * iH;
      T avec[D];
#pragma unroll
      for (int dir = 0; dir < D; ++dir) {
        T s = 0;
#pragma unroll
        for (int l = 0; l < D; ++l) s += Lm[dir][l] * (T)A.op.E[l * NP + m];
        avec[dir] = s;
      }
      finish_node<D, NP, NF, T>(A, e0 + e, m, a, H, avec, r, ent);
    }
  }
  block_sum_store(ent, A.ent_part);
}

// ---------------------------------------------------------------------------
// Navier-Stokes terms on triangles (affine or quadratic maps) and on
// tetrahedra with quadratic maps, in the row form of k_split2 / k_split3c.
// With D_xi = H^-1 Q_xi, Q_xi = K_i + a_i/2 (K_i the metric-averaged skew
// part, a_i = sum_l Lambda_il E_l) and the Baumann-Oden term
// y'_j = -1/2 H^-1 y_j at the facet nodes (y_j = sum_i K~_ij^T (B n_i (w_k -
// w_v)), Sec. 5, eq. bo sats):
//   sum_i D_xi F^V(i) - 1/2 H^-1 sum_j D_xj^T y_j
//     = H^-1 [ sum_i K_i (F^V(i) - y'_i) + 1/2 sum_i a_i (F^V(i) + y'_i) ],
// and per node pair K_i z_i at row m = 1/2 sum_n c_i(m, n) z_i,n with the
// metric-averaged coefficients c_i(m, n) = sum_l S_l[m][n] (Lambda_il(m) +
// Lambda_il(n)) of the Euler pair sums.  So the viscous residual is a second
// pass of node-pair sums over Z_i = F^V(i) - y'_i, after the first pass has
// given D_x w = (X + a w) / (2 H) at every node.  The facet flux jump
// -1/2 H^-1 (q_k + q_v), q = B n . F^V from each side's own gradient, reads
// the facet fluxes that the pre-pass (k_visc_q2 / k_visc_q3c) wrote.
//
// One lane per node row; per node in LDS: fluxes (then Z), w, Lambda.

// Pre-pass on triangles: q = B n . F^V at the facet nodes of every element.
template <int P, typename T>
__global__ __launch_bounds__(kThreads) void k_visc_q2(KArgs<T> A) {
  constexpr int D = 2, NC = 4, NFAC = 3;
  constexpr int NP = Shape<2, P>::NP, NF = Shape<2, P>::NF, NFN = NFAC * NF;
  constexpr int EB = kThreads / NP;
  constexpr int NV = 8;  // w[4], Lambda[4]
  constexpr int NDS = NP * NV + 2;
  __shared__ T nd[EB * NDS];
  const int tid = threadIdx.x;
  const int e = tid / NP, i = tid % NP;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    const bool act = e < ne;
    Node<D, T> n;
    T lam[4];
    __syncthreads();
    if (act) {
      const double *g = A.geo + (size_t)(e0 + e) * 12;
      T F[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const T d0 = A.op.dN[(0 * 6 + a) * NP + i], d1 = A.op.dN[(1 * 6 + a) * NP + i];
        const T gx = map_node<T>(g, 2 * a, 0), gy = map_node<T>(g, 2 * a + 1, 1);
        F[0][0] += d0 * gx;
        F[0][1] += d1 * gx;
        F[1][0] += d0 * gy;
        F[1][1] += d1 * gy;
      }
      lam[0] = F[1][1];
      lam[1] = -F[1][0];
      lam[2] = -F[0][1];
      lam[3] = F[0][0];
      const int uo = A.uoff[e0 + e];
      T uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + i];
      node_from_u<D, T>(uu, A.G, n);
      T *v = nd + e * NDS + i * NV;
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = n.w[c];
#pragma unroll
      for (int c = 0; c < 4; ++c) v[4 + c] = lam[c];
    }
    __syncthreads();
    if (act && i < NFN) {
      T X0[NC], X1[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) X0[c] = X1[c] = (T)0;
#pragma unroll 2
      for (int j = 0; j < NP; ++j) {
        // S_l is stored exactly skew: S_l[i][j] read as -S_l[j][i]
        const T s0 = -A.op.S[(0 * NP + j) * NP + i], s1 = -A.op.S[(1 * NP + j) * NP + i];
        const T *v = nd + e * NDS + j * NV;
        const T c0 = s0 * (lam[0] + v[4]) + s1 * (lam[1] + v[5]);
        const T c1 = s0 * (lam[2] + v[6]) + s1 * (lam[3] + v[7]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          X0[c] += c0 * v[c];
          X1[c] += c1 * v[c];
        }
      }
      const T E0 = A.op.E[i], E1 = A.op.E[NP + i];
      T avec[D];
      avec[0] = lam[0] * E0 + lam[1] * E1;
      avec[1] = lam[2] * E0 + lam[3] * E1;
      const T J = lam[3] * lam[0] - lam[2] * lam[1];
      const T iH = (T)1 / (J * (T)A.op.h[i]);
      T gW[D][NC], FV[D][NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        gW[0][c] = (T)0.5 * iH * (X0[c] + avec[0] * n.w[c]);
        gW[1][c] = (T)0.5 * iH * (X1[c] + avec[1] * n.w[c]);
      }
      viscous_flux<D, T>(n, A.G, A.V, gW, FV);
#pragma unroll
      for (int c = 0; c < NC; ++c)
        A.qout[((size_t)(e0 + e) * NFN + i) * NC + c] = avec[0] * FV[0][c] + avec[1] * FV[1][c];
    }
  }
}

// Entropy split with the Navier-Stokes terms on triangles.
template <int P, typename T>
__global__ __launch_bounds__(kThreads) void k_visc2(KArgs<T> A) {
  constexpr int D = 2, NC = 4, NFAC = 3;
  constexpr int NP = Shape<2, P>::NP, NF = Shape<2, P>::NF, NFN = NFAC * NF;
  constexpr int EB = kThreads / NP;
  constexpr int NDS = NP * 16 + 4;  // per node: f0[4] f1[4] (later Z_0, Z_1) w[4] Lambda[4]
  __shared__ __align__(16) T nd[EB * NDS];
  __shared__ T Ss[2][NP][NP];
  const int tid = threadIdx.x;
  for (int x = tid; x < 2 * NP * NP; x += kThreads) (&Ss[0][0][0])[x] = A.op.S[x];
  const T cb = A.G.cb;
  const T hv = (T)0.5 * (cb - (T)1), he = (T)0.5 * (cb + (T)1);
  const int e = tid / NP, i = tid % NP;
  double ent = 0.0;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    const bool act = e < ne;
    Node<D, T> n;
    T lam[4];
    __syncthreads();
    if (act) {
      const double *g = A.geo + (size_t)(e0 + e) * 12;
      T F[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const T d0 = A.op.dN[(0 * 6 + a) * NP + i], d1 = A.op.dN[(1 * 6 + a) * NP + i];
        const T gx = map_node<T>(g, 2 * a, 0), gy = map_node<T>(g, 2 * a + 1, 1);
        F[0][0] += d0 * gx;
        F[0][1] += d1 * gx;
        F[1][0] += d0 * gy;
        F[1][1] += d1 * gy;
      }
      lam[0] = F[1][1];
      lam[1] = -F[1][0];
      lam[2] = -F[0][1];
      lam[3] = F[0][0];
      const int uo = A.uoff[e0 + e];
      T uu[NC], f0[NC], f1[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + i];
      node_from_u<D, T>(uu, A.G, n);
      if (!n.ok) atomicOr(A.err, 1);
      flux_i<D, T>(n, uu[NC - 1], 0, f0);
      flux_i<D, T>(n, uu[NC - 1], 1, f1);
      T *v = nd + e * NDS + i * 16;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        v[c] = f0[c];
        v[4 + c] = f1[c];
        v[8 + c] = n.w[c];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) v[12 + c] = lam[c];
    }
    __syncthreads();
    T r[NC], Pv[NC], Z[D][NC];
    T H = (T)1, iH = (T)1, avec[D] = {(T)0, (T)0};
    if (act) {
      T V[NC], X0[NC], X1[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) V[c] = X0[c] = X1[c] = (T)0;
#pragma unroll 1
      for (int j = 0; j < NP; ++j) {
        const T *v = nd + e * NDS + j * 16;
        const T s0 = Ss[0][i][j], s1 = Ss[1][i][j];
        const T c0 = s0 * (lam[0] + v[12]) + s1 * (lam[1] + v[13]);
        const T c1 = s0 * (lam[2] + v[14]) + s1 * (lam[3] + v[15]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          V[c] += c0 * v[c];
          V[c] += c1 * v[4 + c];
          X0[c] += c0 * v[8 + c];
          X1[c] += c1 * v[8 + c];
        }
      }
      const T E0 = A.op.E[i], E1 = A.op.E[NP + i];
      avec[0] = lam[0] * E0 + lam[1] * E1;
      avec[1] = lam[2] * E0 + lam[3] * E1;
      const T J = lam[3] * lam[0] - lam[2] * lam[1];
      H = J * (T)A.op.h[i];
      iH = (T)1 / H;
      const T *vi = nd + e * NDS + i * 16;
#pragma unroll
      for (int c = 0; c < NC; ++c) r[c] = iH * (hv * V[c] + he * (avec[0] * vi[c] + avec[1] * vi[4 + c]));
      T gW[D][NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        gW[0][c] = (T)0.5 * iH * (X0[c] + avec[0] * n.w[c]);
        gW[1][c] = (T)0.5 * iH * (X1[c] + avec[1] * n.w[c]);
      }
#pragma unroll
      for (int dir = 0; dir < D; ++dir) {
        T tt[NC];
        jvp_flux<D, T>(n, A.G, dir, gW[dir], tt);
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] -= cb * tt[c];
      }
      T FV[D][NC], yp[D][NC];
      viscous_flux<D, T>(n, A.G, A.V, gW, FV);
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) yp[k][c] = (T)0;
      if (i < NFN) {
        const int off = A.nbr[(size_t)(e0 + e) * NFN + i];
        T uv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) uv[c] = (T)A.u[off + c * NP];
        Node<D, T> nv;
        node_from_u<D, T>(uv, A.G, nv);
        T dw[NC], y[D][NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) dw[c] = n.w[c] - nv.w[c];
        viscous_adjoint_facet<D, T>(n, A.G, A.V, avec, dw, y);
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c) yp[k][c] = (T)(-0.5) * iH * y[k][c];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        Z[0][c] = FV[0][c] - yp[0][c];
        Z[1][c] = FV[1][c] - yp[1][c];
        Pv[c] = (T)0.5 * (avec[0] * (FV[0][c] + yp[0][c]) + avec[1] * (FV[1][c] + yp[1][c]));
      }
    }
    __syncthreads();  // every lane is done with the fluxes of pass one
    if (act) {
      T *v = nd + e * NDS + i * 16;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        v[c] = Z[0][c];
        v[4 + c] = Z[1][c];
      }
    }
    __syncthreads();
    if (act) {
      T W[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) W[c] = (T)0;
#pragma unroll 1
      for (int j = 0; j < NP; ++j) {
        const T *v = nd + e * NDS + j * 16;
        const T s0 = Ss[0][i][j], s1 = Ss[1][i][j];
        const T c0 = s0 * (lam[0] + v[12]) + s1 * (lam[1] + v[13]);
        const T c1 = s0 * (lam[2] + v[14]) + s1 * (lam[3] + v[15]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          W[c] += c0 * v[c];
          W[c] += c1 * v[4 + c];
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) r[c] += iH * ((T)0.5 * W[c] + Pv[c]);
      if (i < NFN) {
        const T *qk = A.q + ((size_t)(e0 + e) * NFN + i) * NC;
        const T *qv = A.q + (size_t)A.nbrq[(size_t)(e0 + e) * NFN + i] * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] -= (T)0.5 * (qk[c] + qv[c]) * iH;
      }
      finish_node<D, NP, NF, T>(A, e0 + e, i, n, H, avec, r, ent);
    }
  }
  block_sum_store(ent, A.ent_part);
}

// Metric cofactors Lambda (L[k][l] = J dxi_l/dx_k) and J at node i of a
// tetrahedron with a quadratic map (ten map nodes g[a*3 + k]).
template <int NP, typename T>
__device__ __forceinline__ void curved3_metrics(const KArgs<T> &A, const T *g, int i, T L[3][3], T &J) {
  T F[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) F[k][l] = (T)0;
#pragma unroll
  for (int a = 0; a < 10; ++a) {
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const T d = A.op.dN[(l * 10 + a) * NP + i];
#pragma unroll
      for (int k = 0; k < 3; ++k) F[k][l] += d * g[a * 3 + k];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const int k1 = (k + 1) % 3, k2 = (k + 2) % 3, l1 = (l + 1) % 3, l2 = (l + 2) % 3;
      L[k][l] = F[k1][l1] * F[k2][l2] - F[k1][l2] * F[k2][l1];
    }
  J = F[0][0] * L[0][0] + F[0][1] * L[0][1] + F[0][2] * L[0][2];
}

// Pre-pass on tetrahedra with quadratic maps: q = B n . F^V at the facet nodes.
template <int P, typename T>
__global__ __launch_bounds__(kThreads) void k_visc_q3c(KArgs<T> A) {
  constexpr int D = 3, NC = 5, NFAC = 4;
  constexpr int NP = Shape<3, P>::NP, NF = Shape<3, P>::NF, NFN = NFAC * NF;
  constexpr int EB = VTile3<P, T>::EB;
  static_assert(EB * NP <= kThreads, "one node per lane");
  constexpr int NV = 15;  // w[5], Lambda[9], pad
  constexpr int NDS = NP * NV;
  __shared__ T nd[EB * NDS];
  __shared__ T gs[EB][30];
  const int tid = threadIdx.x;
  const int e = tid / NP, i = tid % NP;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    const bool act = tid < ne * NP;
    __syncthreads();
    for (int x = tid; x < ne * 30; x += kThreads) gs[x / 30][x % 30] = map_node<T>(A.geo + (size_t)(e0 + x / 30) * 30, x % 30, x % 3);
    __syncthreads();
    Node<D, T> n;
    T L[D][D], J = (T)1;
    if (act) {
      curved3_metrics<NP, T>(A, gs[e], i, L, J);
      const int uo = A.uoff[e0 + e];
      T uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + i];
      node_from_u<D, T>(uu, A.G, n);
      T *v = nd + e * NDS + i * NV;
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = n.w[c];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int l = 0; l < D; ++l) v[5 + k * 3 + l] = L[k][l];
    }
    __syncthreads();
    if (act && i < NFN) {
      T X[D][NC];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) X[k][c] = (T)0;
#pragma unroll 1
      for (int j = 0; j < NP; ++j) {
        const T s0 = -A.op.S[(0 * NP + j) * NP + i];
        const T s1 = -A.op.S[(1 * NP + j) * NP + i];
        const T s2 = -A.op.S[(2 * NP + j) * NP + i];
        const T *v = nd + e * NDS + j * NV;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const T ck = s0 * (L[k][0] + v[5 + k * 3 + 0]) + s1 * (L[k][1] + v[5 + k * 3 + 1]) +
                       s2 * (L[k][2] + v[5 + k * 3 + 2]);
#pragma unroll
          for (int c = 0; c < NC; ++c) X[k][c] += ck * v[c];
        }
      }
      T El[D], avec[D];
#pragma unroll
      for (int l = 0; l < D; ++l) El[l] = A.op.E[l * NP + i];
#pragma unroll
      for (int m = 0; m < D; ++m) avec[m] = L[m][0] * El[0] + L[m][1] * El[1] + L[m][2] * El[2];
      const T iH = (T)1 / (J * (T)A.op.h[i]);
      T gW[D][NC], FV[D][NC];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) gW[k][c] = (T)0.5 * iH * (X[k][c] + avec[k] * n.w[c]);
      viscous_flux<D, T>(n, A.G, A.V, gW, FV);
#pragma unroll
      for (int c = 0; c < NC; ++c)
        A.qout[((size_t)(e0 + e) * NFN + i) * NC + c] = avec[0] * FV[0][c] + avec[1] * FV[1][c] + avec[2] * FV[2][c];
    }
  }
}

// Entropy split with the Navier-Stokes terms on tetrahedra with quadratic maps.
template <int P, typename T>
__global__ __launch_bounds__(kThreads) void k_visc3c(KArgs<T> A) {
  constexpr int D = 3, NC = 5, NFAC = 4;
  constexpr int NP = Shape<3, P>::NP, NF = Shape<3, P>::NF, NFN = NFAC * NF;
  constexpr int EB = VTile3<P, T>::EB;
  static_assert(EB * NP <= kThreads, "one node per lane");
  constexpr int NV = 29;  // f^(1..3)[15] (later Z_1..Z_3), w[5], Lambda[9]
  constexpr int NDS = NP * NV;
  __shared__ T nd[EB * NDS];
  __shared__ T gs[EB][30];
  const int tid = threadIdx.x;
  const T cb = A.G.cb;
  const T hv = (T)0.5 * (cb - (T)1), he = (T)0.5 * (cb + (T)1);
  double ent = 0.0;
  const int ntiles = (A.n_elem + EB - 1) / EB;
  const int e = tid / NP, i = tid % NP;
  for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int e0 = tl * EB;
    const int ne = min(EB, A.n_elem - e0);
    const bool act = tid < ne * NP;
    __syncthreads();
    for (int x = tid; x < ne * 30; x += kThreads) gs[x / 30][x % 30] = map_node<T>(A.geo + (size_t)(e0 + x / 30) * 30, x % 30, x % 3);
    __syncthreads();
    Node<D, T> n;
    T L[D][D], J = (T)1;
    if (act) {
      curved3_metrics<NP, T>(A, gs[e], i, L, J);
      const int uo = A.uoff[e0 + e];
      T uu[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) uu[c] = (T)A.u[uo + c * NP + i];
      node_from_u<D, T>(uu, A.G, n);
      if (!n.ok) atomicOr(A.err, 1);
      T *v = nd + e * NDS + i * NV;
#pragma unroll
      for (int m = 0; m < D; ++m) flux_i<D, T>(n, uu[NC - 1], m, v + m * NC);
#pragma unroll
      for (int c = 0; c < NC; ++c) v[15 + c] = n.w[c];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int l = 0; l < D; ++l) v[20 + k * 3 + l] = L[k][l];
    }
    __syncthreads();
    T r[NC], Pv[NC], Z[D][NC];
    T H = (T)1, iH = (T)1, avec[D] = {(T)0, (T)0, (T)0};
    if (act) {
      T V[NC], X[D][NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        V[c] = (T)0;
#pragma unroll
        for (int k = 0; k < D; ++k) X[k][c] = (T)0;
      }
#pragma unroll 1
      for (int j = 0; j < NP; ++j) {
        const T s0 = -A.op.S[(0 * NP + j) * NP + i];
        const T s1 = -A.op.S[(1 * NP + j) * NP + i];
        const T s2 = -A.op.S[(2 * NP + j) * NP + i];
        const T *v = nd + e * NDS + j * NV;
        T cm[D];
#pragma unroll
        for (int m = 0; m < D; ++m)
          cm[m] = s0 * (L[m][0] + v[20 + m * 3 + 0]) + s1 * (L[m][1] + v[20 + m * 3 + 1]) +
                  s2 * (L[m][2] + v[20 + m * 3 + 2]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          V[c] += cm[0] * v[c];
          V[c] += cm[1] * v[5 + c];
          V[c] += cm[2] * v[10 + c];
          X[0][c] += cm[0] * v[15 + c];
          X[1][c] += cm[1] * v[15 + c];
          X[2][c] += cm[2] * v[15 + c];
        }
      }
      H = J * (T)A.op.h[i];
      iH = (T)1 / H;
      T El[D];
#pragma unroll
      for (int l = 0; l < D; ++l) El[l] = A.op.E[l * NP + i];
#pragma unroll
      for (int m = 0; m < D; ++m) avec[m] = L[m][0] * El[0] + L[m][1] * El[1] + L[m][2] * El[2];
      const T *fi = nd + e * NDS + i * NV;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        r[c] = iH * (hv * V[c] + he * (avec[0] * fi[c] + avec[1] * fi[NC + c] + avec[2] * fi[2 * NC + c]));
      T gW[D][NC];
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) gW[k][c] = (T)0.5 * iH * (X[k][c] + avec[k] * n.w[c]);
#pragma unroll
      for (int dir = 0; dir < D; ++dir) {
        T tt[NC];
        jvp_flux<D, T>(n, A.G, dir, gW[dir], tt);
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] -= cb * tt[c];
      }
      T FV[D][NC], yp[D][NC];
      viscous_flux<D, T>(n, A.G, A.V, gW, FV);
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) yp[k][c] = (T)0;
      if (i < NFN) {
        const int off = A.nbr[(size_t)(e0 + e) * NFN + i];
        T uv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) uv[c] = (T)A.u[off + c * NP];
        Node<D, T> nv;
        node_from_u<D, T>(uv, A.G, nv);
        T dw[NC], y[D][NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) dw[c] = n.w[c] - nv.w[c];
        viscous_adjoint_facet<D, T>(n, A.G, A.V, avec, dw, y);
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c) yp[k][c] = (T)(-0.5) * iH * y[k][c];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        T s = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          Z[k][c] = FV[k][c] - yp[k][c];
          s += avec[k] * (FV[k][c] + yp[k][c]);
        }
        Pv[c] = (T)0.5 * s;
      }
    }
    __syncthreads();  // every lane is done with the fluxes of pass one
    if (act) {
      T *v = nd + e * NDS + i * NV;
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) v[k * NC + c] = Z[k][c];
    }
    __syncthreads();
    if (act) {
      T W[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) W[c] = (T)0;
#pragma unroll 1
      for (int j = 0; j < NP; ++j) {
        const T s0 = -A.op.S[(0 * NP + j) * NP + i];
        const T s1 = -A.op.S[(1 * NP + j) * NP + i];
        const T s2 = -A.op.S[(2 * NP + j) * NP + i];
        const T *v = nd + e * NDS + j * NV;
        T cm[D];
#pragma unroll
        for (int m = 0; m < D; ++m)
          cm[m] = s0 * (L[m][0] + v[20 + m * 3 + 0]) + s1 * (L[m][1] + v[20 + m * 3 + 1]) +
                  s2 * (L[m][2] + v[20 + m * 3 + 2]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          W[c] += cm[0] * v[c];
          W[c] += cm[1] * v[5 + c];
          W[c] += cm[2] * v[10 + c];
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) r[c] += iH * ((T)0.5 * W[c] + Pv[c]);
      if (i < NFN) {
        const T *qk = A.q + ((size_t)(e0 + e) * NFN + i) * NC;
        const T *qv = A.q + (size_t)A.nbrq[(size_t)(e0 + e) * NFN + i] * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] -= (T)0.5 * (qk[c] + qv[c]) * iH;
      }
      finish_node<D, NP, NF, T>(A, e0 + e, i, n, H, avec, r, ent);
    }
  }
  block_sum_store(ent, A.ent_part);
}

// ---------------------------------------------------------------------------

struct KernelRef {
  const void *fn;
  int eb;  // elements per tile
};

// Kernel of a residual slot; form_eff 0: entropy split (Euler), 1: Hadamard,
// 2: entropy split with the Navier-Stokes terms, 3 and 4: entropy split and
// Hadamard on curved tetrahedra.
// Curved tetrahedra (form_eff 3): quadratic maps need p >= 2.
template <int P, typename T>
static KernelRef curved3_kernel() {
  if constexpr (P >= 2) return {reinterpret_cast<const void *>(&k_split3c<P, T>), VTile3<P, T>::EB};
  return {nullptr, 0};
}

template <int P, typename T>
static KernelRef curved3_hadamard_kernel() {
  if constexpr (P >= 2) return {reinterpret_cast<const void *>(&k_hadamard<3, P, T, true>), HadTile<3, P, T>::EB};
  return {nullptr, 0};
}

template <int P, typename T>
static KernelRef curved3_visc_kernel() {
  if constexpr (P >= 2) return {reinterpret_cast<const void *>(&k_visc3c<P, T>), VTile3<P, T>::EB};
  return {nullptr, 0};
}

template <typename T>
static KernelRef residual_kernel(int dim, int p, int form_eff, int variant) {
#define SBP_K2(PP)                                                                              \
  if (dim == 2 && p == PP) {                                                                    \
    if (form_eff == 1) return {reinterpret_cast<const void *>(&k_hadamard<2, PP, T>), HadTile<2, PP, T>::EB}; \
    if (form_eff == 2) return {reinterpret_cast<const void *>(&k_visc2<PP, T>), kThreads / Shape<2, PP>::NP}; \
    if (form_eff == 0) {                                                                        \
      /* variant 0 (built-in): FP64 facet SATs before the pair sums with the next */            \
      /* tile's neighbour states loaded ahead; FP32 SATs after the pair sums (fewer */           \
      /* registers, four waves per SIMD); 1: one row per lane, SATs first; 2: the other */     \
      if (variant == 1)                                                                         \
        return {reinterpret_cast<const void *>(&k_split2<PP, T, 1, 3>), Split2<PP, T, 1>::EB};  \
      if ((variant == 2) == (sizeof(T) == 8))                                                   \
        return {reinterpret_cast<const void *>(&k_split2<PP, T, 2, 0>), Split2<PP, T, 2>::EB};  \
      return {reinterpret_cast<const void *>(&k_split2<PP, T, 2, 3>), Split2<PP, T, 2>::EB};    \
    }                                                                                           \
    return {nullptr, 0};                                                                        \
  }
  SBP_K2(1) SBP_K2(2) SBP_K2(3) SBP_K2(4)
#undef SBP_K2
#define SBP_K3(PP)                                                                              \
  if (dim == 3 && p == PP) {                                                                    \
    if (form_eff == 1) return {reinterpret_cast<const void *>(&k_hadamard<3, PP, T>), HadTile<3, PP, T>::EB}; \
    if (form_eff == 2) return {reinterpret_cast<const void *>(&k_split3<PP, T, true>), 3 * Wave3<PP, T>::CT}; \
    if (form_eff == 3) return curved3_kernel<PP, T>();                                         \
    if (form_eff == 4) return curved3_hadamard_kernel<PP, T>();                                \
    if (form_eff == 5) return curved3_visc_kernel<PP, T>();                                    \
    const bool sg = skew_from_cache3<PP, T>() != (variant == 1);                                \
    return {sg ? reinterpret_cast<const void *>(&k_split3v<PP, T, true>)                        \
               : reinterpret_cast<const void *>(&k_split3v<PP, T, false>),                      \
            VTile3<PP, T>::EB};                                                                 \
  }
  SBP_K3(1) SBP_K3(2) SBP_K3(3)
#undef SBP_K3
  return {nullptr, 0};
}

int resident_blocks(const void *kernel) {
  static std::mutex mu;
  static std::map<std::pair<int, const void *>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(dev, kernel);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per = 0, cap = 1024;
  if (dev >= 0 && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kThreads, 0) == hipSuccess && cus > 0 && per > 0)
    cap = cus * per;
  cache[key] = cap;
  return cap;
}

int launch_grid(const void *kernel, int ntiles, int grid) {
  if (ntiles <= 0) return 0;
  // one workgroup per tile, rounded up to a multiple of the XCD count (the
  // kernels' TileSeq then gives each XCD a contiguous eighth of the tiles;
  // surplus workgroups find no tile)
  if (grid <= 0) return ntiles < kXcds ? ntiles : (ntiles + kXcds - 1) / kXcds * kXcds;
  const long long cap = (long long)grid * resident_blocks(kernel);
  return (int)std::min<long long>(ntiles, cap);
}

int residual_variants(int dim, int p, int precision, int form_eff) {
  (void)p;
  (void)precision;
  if (form_eff != 0) return 1;
  return dim == 2 ? 3 : 2;
}

int residual_blocks(int dim, int p, int precision, int form_eff, int n_elem, LaunchCfg cfg) {
  if (n_elem <= 0) return 0;
  const KernelRef k = precision == 0 ? residual_kernel<double>(dim, p, form_eff, cfg.variant)
                                     : residual_kernel<float>(dim, p, form_eff, cfg.variant);
  if (!k.fn) return 0;
  return launch_grid(k.fn, (n_elem + k.eb - 1) / k.eb, cfg.grid);
}

template <typename T>
static hipError_t launch_t(int dim, int p, int form, const KArgs<T> &A, hipStream_t s, LaunchCfg cfg) {
  if (A.visc && form != 0) return hipErrorInvalidValue;
  if (A.curved && dim != 3) return hipErrorInvalidValue;
  const int fe = A.visc ? (A.curved ? 5 : 2) : (A.curved ? (form == 0 ? 3 : 4) : form);
  const KernelRef k = residual_kernel<T>(dim, p, fe, cfg.variant);
  if (!k.fn || A.n_elem <= 0) return hipErrorInvalidValue;
  const int nb = launch_grid(k.fn, (A.n_elem + k.eb - 1) / k.eb, cfg.grid);
  KArgs<T> a = A;
  void *args[] = {&a};
  return hipLaunchKernel(k.fn, dim3(nb), dim3(kThreads), args, 0, s);
}

template <typename T>
static hipError_t launch_q(int dim, int p, const KArgs<T> &A, hipStream_t s) {
  if (A.n_elem <= 0) return hipErrorInvalidValue;
  const void *fn = nullptr;
  int eb = 0;
  if (dim == 2) {
    fn = p == 1 ? reinterpret_cast<const void *>(&k_visc_q2<1, T>)
       : p == 2 ? reinterpret_cast<const void *>(&k_visc_q2<2, T>)
       : p == 3 ? reinterpret_cast<const void *>(&k_visc_q2<3, T>)
       : p == 4 ? reinterpret_cast<const void *>(&k_visc_q2<4, T>) : nullptr;
    eb = p >= 1 && p <= 4 ? kThreads / (p == 1 ? Shape<2, 1>::NP : p == 2 ? Shape<2, 2>::NP
                                       : p == 3 ? Shape<2, 3>::NP : Shape<2, 4>::NP) : 0;
  } else if (A.curved) {
    fn = p == 2 ? reinterpret_cast<const void *>(&k_visc_q3c<2, T>)
       : p == 3 ? reinterpret_cast<const void *>(&k_visc_q3c<3, T>) : nullptr;
    eb = p == 2 ? VTile3<2, T>::EB : VTile3<3, T>::EB;
  } else {
    fn = p == 1 ? reinterpret_cast<const void *>(&k_visc_q3<1, T>)
       : p == 2 ? reinterpret_cast<const void *>(&k_visc_q3<2, T>)
       : p == 3 ? reinterpret_cast<const void *>(&k_visc_q3<3, T>) : nullptr;
    eb = p == 1 ? VTile3<1, T>::EB : (p == 2 ? VTile3<2, T>::EB : VTile3<3, T>::EB);
  }
  if (!fn) return hipErrorInvalidValue;
  const int nb = launch_grid(fn, (A.n_elem + eb - 1) / eb, 1);
  KArgs<T> a = A;
  void *args[] = {&a};
  return hipLaunchKernel(fn, dim3(nb), dim3(kThreads), args, 0, s);
}

hipError_t launch_visc_q(int dim, int p, const KArgs<double> &A, hipStream_t s) { return launch_q<double>(dim, p, A, s); }
hipError_t launch_visc_q(int dim, int p, const KArgs<float> &A, hipStream_t s) { return launch_q<float>(dim, p, A, s); }

template <typename T>
static int split2_ew(int p) {
  switch (p) {
    case 1: return Split2<1, T, split2_rows<1, T>()>::EB;
    case 2: return Split2<2, T, split2_rows<2, T>()>::EB;
    case 3: return Split2<3, T, split2_rows<3, T>()>::EB;
    default: return Split2<4, T, split2_rows<4, T>()>::EB;
  }
}

template <typename T>
static int batch_groups(const int n_elem_of_p[4], int g0[5]) {
  g0[0] = 0;
  for (int q = 0; q < 4; ++q) {
    const int ew = split2_ew<T>(q + 1);
    g0[q + 1] = g0[q] + (n_elem_of_p[q] + ew - 1) / ew;
  }
  return g0[4];
}

int residual2_batch_blocks(const int n_elem_of_p[4], int precision, int grid) {
  int g0[5];
  if (precision == 0)
    return launch_grid(reinterpret_cast<const void *>(&k_split2_batch<double>), batch_groups<double>(n_elem_of_p, g0), grid);
  return launch_grid(reinterpret_cast<const void *>(&k_split2_batch<float>), batch_groups<float>(n_elem_of_p, g0), grid);
}

template <typename T>
static hipError_t launch_batch2_t(const KArgs<T> *const cls[4], const KArgs<T> *cls_dev, double *ent_part,
                                  hipStream_t s, int grid) {
  Batch2<T> Bt{};
  int ne[4];
  const KArgs<T> *any = nullptr;
  for (int q = 0; q < 4; ++q) {
    ne[q] = cls[q] ? cls[q]->n_elem : 0;
    if (cls[q]) any = cls[q];
  }
  const int ng = batch_groups<T>(ne, Bt.g0);
  if (ng == 0 || !any) return hipSuccess;
  Bt.cls = cls_dev;
  Bt.u = any->u;
  Bt.r = any->r;
  Bt.eform = any->eform;
  Bt.ent_part = ent_part;
  Bt.tstamp = any->tstamp;
  const int nb = residual2_batch_blocks(ne, sizeof(T) == 8 ? 0 : 1, grid);
  hipLaunchKernelGGL((k_split2_batch<T>), dim3(nb), dim3(kThreads), 0, s, Bt);
  return hipGetLastError();
}

hipError_t launch_residual2_batch(const KArgs<double> *const cls[4], const KArgs<double> *cls_dev, double *ent_part,
                                  hipStream_t s, int grid) {
  return launch_batch2_t<double>(cls, cls_dev, ent_part, s, grid);
}
hipError_t launch_residual2_batch(const KArgs<float> *const cls[4], const KArgs<float> *cls_dev, double *ent_part,
                                  hipStream_t s, int grid) {
  return launch_batch2_t<float>(cls, cls_dev, ent_part, s, grid);
}

hipError_t launch_residual(int dim, int p, int form, const KArgs<double> &A, hipStream_t s, LaunchCfg cfg) {
  return launch_t<double>(dim, p, form, A, s, cfg);
}
hipError_t launch_residual(int dim, int p, int form, const KArgs<float> &A, hipStream_t s, LaunchCfg cfg) {
  return launch_t<float>(dim, p, form, A, s, cfg);
}

}  // namespace sbp
