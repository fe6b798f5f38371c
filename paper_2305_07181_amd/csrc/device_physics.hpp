// Pointwise device functions of the entropy-split scheme (HIP, gfx950).
//
// Paper references: fluxes and EOS (Sec. 2.2); Harten entropy and entropy
// variables (Sec. 2.4, Sec. 3); Sjogreen-Yee two-point flux with arithmetic
// and exponential averages (Sec. 4); matrix interface dissipation (Sec. 4.5).
//
// Computation route (differs from a dense-matrix formulation on purpose):
//   * A~_i g = dF^(i)/dW g is a forward-mode directional derivative through
//     the inverse map U(W) (temperature and W_nc formulas of Sec. 3);
//   * the dissipation X|Lambda|S X^T dw is applied column by column with the
//     shear part in tangent-free form |V.n| eta (0, T q, V.T q),
//     T = I - n n^T, q = dw_V + dw_E V (valid in 2D and 3D);
//   * all powers come from per-node logarithms: z1 = exp(ln rho - ln p +
//     (ln p - gamma ln rho)/(alpha+gamma)), z1^r1, p^r2 as exps.
#pragma once
#include <hip/hip_runtime.h>

namespace sbp {

// Constants of the exponential average {x^(r-1)}_e for one exponent r:
// odd-power series coefficients C(r, 2k+1)/r, k = 1..4, and the binomial
// coefficients of (1 + delta)^(r-1), powers 1..9.
template <typename T>
struct ExpAvgC {
  T r;
  T c[4];
  T bn[9];
};

template <typename T>
struct GasC {
  T g, gm1, a, cb;       // gamma, gamma-1, alpha, 1/(beta+1)
  T inv_apg;             // 1/(alpha+gamma)
  T r1, r2;              // -gamma/alpha, (1-gamma)/alpha
  T wfirst;              // -alpha/(gamma-1)
  T ja, jb_inv;          // (1-alpha-gamma)/(alpha+gamma), (alpha+gamma)/(1-gamma)
  T sfac;                // (gamma-1)(gamma+alpha)/(gamma alpha)
  T ggm1;                // gamma/(gamma-1)
  T gm1_a;               // (gamma-1)/alpha
  ExpAvgC<T> e1, e2;     // exponential averages of z1 (r1) and p (r2)
};

template <typename T>
__host__ ExpAvgC<T> make_exp_avg(double r) {
  ExpAvgC<T> C;
  C.r = (T)r;
  double c = (r - 1.0) * (r - 2.0) / 6.0;
  C.c[0] = (T)c;
  c *= (r - 3.0) * (r - 4.0) / 20.0;
  C.c[1] = (T)c;
  c *= (r - 5.0) * (r - 6.0) / 42.0;
  C.c[2] = (T)c;
  c *= (r - 7.0) * (r - 8.0) / 72.0;
  C.c[3] = (T)c;
  double b = 1.0;
  for (int k = 1; k <= 9; ++k) {
    b *= (r - 1.0 - (k - 1)) / k;
    C.bn[k - 1] = (T)b;
  }
  return C;
}

template <typename T>
__host__ GasC<T> make_gas(double gamma, double beta) {
  double alpha = -gamma - beta * (gamma - 1.0);
  GasC<T> G;
  G.g = (T)gamma;
  G.gm1 = (T)(gamma - 1.0);
  G.a = (T)alpha;
  G.cb = (T)(1.0 / (beta + 1.0));
  G.inv_apg = (T)(1.0 / (alpha + gamma));
  G.r1 = (T)(-gamma / alpha);
  G.r2 = (T)((1.0 - gamma) / alpha);
  G.wfirst = (T)(-alpha / (gamma - 1.0));
  G.ja = (T)((1.0 - alpha - gamma) / (alpha + gamma));
  G.jb_inv = (T)((alpha + gamma) / (1.0 - gamma));
  G.sfac = (T)((gamma - 1.0) * (gamma + alpha) / (gamma * alpha));
  G.ggm1 = (T)(gamma / (gamma - 1.0));
  G.gm1_a = (T)((gamma - 1.0) / alpha);
  G.e1 = make_exp_avg<T>(-gamma / alpha);
  G.e2 = make_exp_avg<T>((1.0 - gamma) / alpha);
  return G;
}

__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float dexp(float x) { return expf(x); }
__device__ __forceinline__ double dlog(double x) { return log(x); }
__device__ __forceinline__ float dlog(float x) { return logf(x); }
__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float dsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double dabs(double x) { return fabs(x); }
__device__ __forceinline__ float dabs(float x) { return fabsf(x); }

// 1/x of a nonzero finite FP64 value by Newton's iteration on f(r) = 1/r - x,
// r <- r + r (1 - x r), started from the hardware reciprocal estimate: each
// step squares the relative error, and two leave the result within about one
// unit in the last place.  Five dependent instructions in place of the
// correctly rounded division sequence (about ten); the residual's quotients
// of positive state quantities (1/rho, 1/p, 1/W_nc, 1/H, the averages'
// denominators) take it.  FP32 keeps its division.
__device__ __forceinline__ double drcp(double x) {
  const double r0 = __builtin_amdgcn_rcp(x);
  const double r1 = fma(r0, fma(-x, r0, 1.0), r0);
  return fma(r1, fma(-x, r1, 1.0), r1);
}
__device__ __forceinline__ float drcp(float x) { return 1.0f / x; }
// other arithmetic types (the dual numbers of the forward-mode derivatives)
template <typename T>
__device__ __forceinline__ T drcp(const T &x) { return (T)1 / x; }

// Node quantities shared by the volume and facet terms.
template <int D, typename T>
struct Node {
  T rho, V[D], p;
  T irho;       // 1/rho
  T lrho, lp, lz1;  // logarithms of rho, p, z1
  T z1;         // (rho/p)(p rho^-gamma)^(1/(alpha+gamma)) = -W_nc
  T P1, P2;     // z1^r1, p^r2 (powers entering the two-point flux averages)
  T w[D + 2];   // entropy variables
  bool ok;      // rho > 0 and p > 0 and finite
};

template <int D, typename T>
__device__ __forceinline__ void node_from_u(const T *u, const GasC<T> &G, Node<D, T> &n) {
  n.rho = u[0];
  T q2 = 0;
  T irho = drcp(n.rho);
  n.irho = irho;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    n.V[i] = u[1 + i] * irho;
    q2 += n.V[i] * n.V[i];
  }
  n.p = G.gm1 * (u[D + 1] - (T)0.5 * n.rho * q2);
  n.ok = (n.rho > (T)0) && (n.p > (T)0) && (n.rho < (T)1e300) && (n.p < (T)1e300);
  n.lrho = dlog(n.rho);
  n.lp = dlog(n.p);
  n.lz1 = n.lrho - n.lp + (n.lp - G.g * n.lrho) * G.inv_apg;
  n.z1 = dexp(n.lz1);
  n.P1 = (T)0;
  n.P2 = (T)0;
  T theta = n.p * irho;
  n.w[0] = n.z1 * (G.wfirst * theta - (T)0.5 * q2);
#pragma unroll
  for (int i = 0; i < D; ++i) n.w[1 + i] = n.z1 * n.V[i];
  n.w[D + 1] = -n.z1;
}

// Binomial coefficients C(e, k), k = 1..9, of (1 + x)^e for the exponents of
// the node powers: z1 = rho^ea p^eb (ln z1 = ea ln rho + eb ln p), z1^r1,
// p^r2.  Used to carry a node's powers over to a nearby state.
template <typename T>
struct JumpC {
  T ea[9], eb[9], r1[9], r2[9];
};

template <typename T>
__host__ JumpC<T> make_jump(double gamma, double beta) {
  const double alpha = -gamma - beta * (gamma - 1.0);
  const double inv_apg = 1.0 / (alpha + gamma);
  const double ex[4] = {1.0 - gamma * inv_apg, inv_apg - 1.0, -gamma / alpha, (1.0 - gamma) / alpha};
  JumpC<T> J;
  T *dst[4] = {J.ea, J.eb, J.r1, J.r2};
  for (int q = 0; q < 4; ++q) {
    double c = 1.0;
    for (int k = 1; k <= 9; ++k) {
      c *= (ex[q] - (k - 1)) / k;
      dst[q][k - 1] = (T)c;
    }
  }
  return J;
}

// (1 + x)^e by its binomial series to degree 9 (coefficients C(e, 1..9)).
template <typename T>
__device__ __forceinline__ T binom9(const T *C, T x) {
  T t = C[8];
#pragma unroll
  for (int k = 7; k >= 0; --k) t = C[k] + x * t;
  return (T)1 + x * t;
}

// Largest |rho_v/rho_k - 1| and |p_v/p_k - 1| for which node_near carries
// the powers over by series: the ratio of the z1 values then stays within
// about 0.022 (FP64) or 0.22 (FP32) of 1, where the degree-9 remainders are
// ~1e-19 and ~1e-9 of the value.
template <typename T>
__device__ __forceinline__ constexpr T near_max() {
  return sizeof(T) == 4 ? (T)0.05 : (T)0.005;
}

// The node state of conservative values u for the two-point flux (primitives,
// z1, z1^r1, p^r2, w; the logarithms are not set) when u is close to the
// node k with powers: z1 = z1_k (1 + dr)^ea (1 + dp)^eb, z1^r1 = z1_k^r1
// (z1 / z1_k)^r1, p^r2 = p_k^r2 (1 + dp)^r2 with dr = rho/rho_k - 1,
// dp = p/p_k - 1 -- no transcendental function.  irho_k = 1/rho_k,
// ip_k = 1/p_k.  Returns false, leaving the powers unset, when a ratio is
// outside the series' range (the caller then takes node_from_u and
// node_powers).
template <int D, typename T>
__device__ __forceinline__ bool node_near(const T *u, const Node<D, T> &k, T irho_k, T ip_k, const GasC<T> &G,
                                          const JumpC<T> &Jc, Node<D, T> &n) {
  n.rho = u[0];
  T q2 = 0;
  const T irho = drcp(n.rho);
  n.irho = irho;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    n.V[i] = u[1 + i] * irho;
    q2 += n.V[i] * n.V[i];
  }
  n.p = G.gm1 * (u[D + 1] - (T)0.5 * n.rho * q2);
  n.ok = (n.rho > (T)0) && (n.p > (T)0) && (n.rho < (T)1e300) && (n.p < (T)1e300);
  const T dr = n.rho * irho_k - (T)1, dp = n.p * ip_k - (T)1;
  if (!(dabs(dr) <= near_max<T>() && dabs(dp) <= near_max<T>())) return false;
  const T zr = binom9(Jc.ea, dr) * binom9(Jc.eb, dp);
  n.lrho = n.lp = n.lz1 = (T)0;
  n.z1 = k.z1 * zr;
  n.P1 = k.P1 * binom9(Jc.r1, zr - (T)1);
  n.P2 = k.P2 * binom9(Jc.r2, dp);
  const T theta = n.p * irho;
  n.w[0] = n.z1 * (G.wfirst * theta - (T)0.5 * q2);
#pragma unroll
  for (int i = 0; i < D; ++i) n.w[1 + i] = n.z1 * n.V[i];
  n.w[D + 1] = -n.z1;
  return true;
}

// z1^r1 and p^r2, needed only by the two-point flux at facet nodes and in the
// Hadamard volume term.
template <int D, typename T>
__device__ __forceinline__ void node_powers(const GasC<T> &G, Node<D, T> &n) {
  n.P1 = dexp(G.r1 * n.lz1);
  n.P2 = dexp(G.r2 * n.lp);
}

// F^(i) from primitives.
template <int D, typename T>
__device__ __forceinline__ void flux_i(const Node<D, T> &n, T E, int i, T *f) {
  T m = n.rho * n.V[i];
  f[0] = m;
#pragma unroll
  for (int j = 0; j < D; ++j) f[1 + j] = m * n.V[j] + (j == i ? n.p : (T)0);
  f[D + 1] = (E + n.p) * n.V[i];
}

// out = A~_i g = dF^(i)/dW [g] (forward-mode derivative through U(W)).
template <int D, typename T>
__device__ __forceinline__ void jvp_flux(const Node<D, T> &n, const GasC<T> &G, int i, const T *g, T *out) {
  const T Wn = n.w[D + 1];
  const T iWn = (T)1 / Wn;
  T dV[D];
  T q2 = 0, Vg = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    dV[k] = -(g[1 + k] + n.V[k] * g[D + 1]) * iWn;
    q2 += n.V[k] * n.V[k];
    Vg += n.V[k] * g[1 + k];
  }
  const T theta = n.p / n.rho;
  const T c1 = G.gm1_a * iWn;  // (gamma-1)/(alpha W_nc)
  const T dtheta = c1 * (g[0] + Vg) + (-theta + (T)0.5 * G.gm1_a * q2) * iWn * g[D + 1];
  // ln(-W_nc) = ja ln(theta) + jb ln(rho)
  const T drho = n.rho * (g[D + 1] * iWn - G.ja * dtheta / theta) * G.jb_inv;
  const T dp = theta * drho + n.rho * dtheta;
  T VdV = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) VdV += n.V[k] * dV[k];
  out[0] = drho * n.V[i] + n.rho * dV[i];
#pragma unroll
  for (int j = 0; j < D; ++j)
    out[1 + j] = drho * n.V[i] * n.V[j] + n.rho * (dV[i] * n.V[j] + n.V[i] * dV[j]) + (j == i ? dp : (T)0);
  const T ep = G.ggm1 * n.p + (T)0.5 * n.rho * q2;  // e + p
  out[D + 1] = dV[i] * ep + n.V[i] * (G.ggm1 * dp + (T)0.5 * q2 * drho + n.rho * VdV);
}

// sum_i A~_i g_i = sum_i dF^(i)/dW [g_i] for all D directions at once (the
// same derivative as jvp_flux), with the node's reciprocals iWn = 1/W_nc and
// itheta = rho/p given, so that no division is left per direction.
template <int D, typename T>
__device__ __forceinline__ void jvp_flux_sum(const Node<D, T> &n, const GasC<T> &G, T iWn, T itheta,
                                             const T (*g)[D + 2], T *out) {
  constexpr int NC = D + 2;
  T q2 = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) q2 += n.V[k] * n.V[k];
  const T theta = n.p * n.irho;
  const T c1 = G.gm1_a * iWn;  // (gamma-1)/(alpha W_nc)
  const T c2 = (-theta + (T)0.5 * G.gm1_a * q2) * iWn;
  const T ep = G.ggm1 * n.p + (T)0.5 * n.rho * q2;  // e + p
#pragma unroll
  for (int c = 0; c < NC; ++c) out[c] = (T)0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T *gi = g[i];
    T dV[D];
    T Vg = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      dV[k] = -(gi[1 + k] + n.V[k] * gi[NC - 1]) * iWn;
      Vg += n.V[k] * gi[1 + k];
    }
    const T dtheta = c1 * (gi[0] + Vg) + c2 * gi[NC - 1];
    const T drho = n.rho * (gi[NC - 1] * iWn - G.ja * dtheta * itheta) * G.jb_inv;
    const T dp = theta * drho + n.rho * dtheta;
    T VdV = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) VdV += n.V[k] * dV[k];
    out[0] += drho * n.V[i] + n.rho * dV[i];
#pragma unroll
    for (int j = 0; j < D; ++j)
      out[1 + j] += drho * n.V[i] * n.V[j] + n.rho * (dV[i] * n.V[j] + n.V[i] * dV[j]) + (j == i ? dp : (T)0);
    out[NC - 1] += dV[i] * ep + n.V[i] * (G.ggm1 * dp + (T)0.5 * q2 * drho + n.rho * VdV);
  }
}

// Largest |eps| = |a - b| / (a + b) for which the exponential average takes
// its series form.  The direct quotient loses about -log10|eps| digits to
// cancellation and the series' truncation error is about |eps|^10: 1e-2
// keeps both near 1e-14 in FP64; in FP32 the quotient would lose two of its
// seven digits there, so the series (still exact to ~1e-10 at 0.1) runs up
// to 0.1.
template <typename T>
__device__ __forceinline__ constexpr T exp_avg_series_max() {
  return sizeof(T) == 4 ? (T)0.1 : (T)1e-2;
}

// Exponential average {x^{r-1}}_e = (a^r - b^r) / (r (a - b)) from values
// a, b and their r-th powers; near a = b the series form
//   m^{r-1} [1 + sum_k C(r,2k+1)/r eps^{2k}],  m = (a+b)/2,  eps = (a-b)/(a+b),
// with m^{r-1} = (a^r / a) (1 + delta)^{r-1}, delta = (b - a)/(2a),
// the binomial series summed to delta^9 (FP64: |delta| < 0.0102, remainder
// < 1e-19; FP32: |delta| < 0.1, remainder < 1e-10).
template <typename T>
__device__ __forceinline__ T exp_avg_ia(T a, T b, T ar, T br, T ia, const ExpAvgC<T> &C) {
  const T s = a + b;
  const T eps = (a - b) * drcp(s);
  if (dabs(eps) <= exp_avg_series_max<T>()) {
    const T dl = (T)0.5 * (b - a) * ia;
    T bin = C.bn[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) bin = C.bn[k] + dl * bin;
    bin = (T)1 + dl * bin;
    const T e2 = eps * eps;
    return ar * ia * bin * ((T)1 + e2 * (C.c[0] + e2 * (C.c[1] + e2 * (C.c[2] + e2 * C.c[3]))));
  }
  return (ar - br) / (C.r * (a - b));
}

// The same with 1/a computed here.
template <typename T>
__device__ __forceinline__ T exp_avg(T a, T b, T ar, T br, const ExpAvgC<T> &C) {
  const T s = a + b;
  const T eps = (a - b) * drcp(s);
  if (dabs(eps) <= exp_avg_series_max<T>()) {
    const T ia = (T)1 / a;
    const T dl = (T)0.5 * (b - a) * ia;
    T bin = C.bn[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) bin = C.bn[k] + dl * bin;
    bin = (T)1 + dl * bin;
    const T e2 = eps * eps;
    return ar * ia * bin * ((T)1 + e2 * (C.c[0] + e2 * (C.c[1] + e2 * (C.c[2] + e2 * C.c[3]))));
  }
  return (ar - br) / (C.r * (a - b));
}

// Facet term at one facet node pair, own side k, neighbour v, area-normal
// a = B n (length B, direction the unit outward normal of k):
//   out = a . F*(u_k, u_v)  [+ 1/2 |a| X|Lambda|S X^T (w_k - w_v)]
// The residual receives -out / H_m.
template <int D, typename T>
__device__ __forceinline__ void facet_term_c(const Node<D, T> &k, const Node<D, T> &v, const T *a,
                                             const GasC<T> &G, const ExpAvgC<T> &C1, const ExpAvgC<T> &C2,
                                             bool diss, T *out, T ip_k, T iz1_k) {
  constexpr int NC = D + 2;
  const T P1k = k.P1, P1v = v.P1, P2k = k.P2, P2v = v.P2;
  // own-side reciprocals 1/p_k and 1/z1_k, if the caller has them
  const T Ep = ip_k != (T)0 ? exp_avg_ia(k.p, v.p, P2k, P2v, ip_k, C2) : exp_avg(k.p, v.p, P2k, P2v, C2);
  const T Ez = iz1_k != (T)0 ? exp_avg_ia(k.z1, v.z1, P1k, P1v, iz1_k, C1) : exp_avg(k.z1, v.z1, P1k, P1v, C1);
  const T Dn = (T)0.5 * (P1k + P1v) * Ep;
  const T iD = drcp(Dn);
  T an = 0;  // a . {z1 V} / D
  T Vav[D];
  T q2av = 0, Vav2 = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    an += a[i] * (T)0.5 * (k.z1 * k.V[i] + v.z1 * v.V[i]);
    Vav[i] = (T)0.5 * (k.V[i] + v.V[i]);
    Vav2 += Vav[i] * Vav[i];
    q2av += (T)0.5 * (k.V[i] * k.V[i] + v.V[i] * v.V[i]);
  }
  const T mass = an * iD;
  const T pav = (T)0.5 * (k.p + v.p);
  out[0] = mass;
#pragma unroll
  for (int j = 0; j < D; ++j) out[1 + j] = mass * Vav[j] + a[j] * pav;
  out[NC - 1] = mass * (G.ggm1 * (T)0.5 * (P2k + P2v) * Ez + Vav2 - (T)0.5 * q2av);
  if (!diss) return;
  // intermediate state (Sec. 4.5)
  const T z1a = (T)0.5 * (k.z1 + v.z1);
  const T rho_h = z1a * iD;
  T Vh[D];
  T Vh2 = 0, B2 = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    Vh[i] = (T)0.5 * (k.z1 * k.V[i] + v.z1 * v.V[i]) / z1a;
    Vh2 += Vh[i] * Vh[i];
    B2 += a[i] * a[i];
  }
  const T B = dsqrt(B2);
  const T iB = (T)1 / B;
  T n[D];
  T Vn = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    n[i] = a[i] * iB;
    Vn += Vh[i] * n[i];
  }
  const T theta = rho_h / (pav * Dn);
  const T eta = (T)1 / (z1a * Ez * Ep);
  const T ah = dsqrt(G.g * pav / rho_h);
  const T Hh = ah * ah / G.gm1 + (T)0.5 * Vh2;
  T dw[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) dw[c] = k.w[c] - v.w[c];
  // projections on the acoustic and entropy columns
  T xdV = 0, ndV = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    xdV += Vh[i] * dw[1 + i];
    ndV += n[i] * dw[1 + i];
  }
  const T pm = dw[0] + xdV - ah * ndV + (Hh - ah * Vn) * dw[NC - 1];   // x_-^T dw
  const T pp = dw[0] + xdV + ah * ndV + (Hh + ah * Vn) * dw[NC - 1];   // x_+^T dw
  const T p0 = dw[0] + xdV + (T)0.5 * Vh2 * dw[NC - 1];               // x_0^T dw
  const T sa = theta / ((T)2 * G.g);
  const T cm = dabs(Vn - ah) * sa * pm;
  const T cp = dabs(Vn + ah) * sa * pp;
  const T c0 = dabs(Vn) * G.sfac * theta * p0;
  // shear: |Vn| eta (0, T q, V.T q), q = dw_V + dw_E V
  T q[D];
  T nq = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    q[i] = dw[1 + i] + dw[NC - 1] * Vh[i];
    nq += n[i] * q[i];
  }
  const T cs = dabs(Vn) * eta;
  T y[NC];
  y[0] = cm + c0 + cp;
  T VTq = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T tq = q[i] - n[i] * nq;
    VTq += Vh[i] * tq;
    y[1 + i] = cm * (Vh[i] - ah * n[i]) + c0 * Vh[i] + cp * (Vh[i] + ah * n[i]) + cs * tq;
  }
  y[NC - 1] = cm * (Hh - ah * Vn) + c0 * (T)0.5 * Vh2 + cp * (Hh + ah * Vn) + cs * VTq;
  const T hb = (T)0.5 * B;
#pragma unroll
  for (int c = 0; c < NC; ++c) out[c] += hb * y[c];
}

// The same with the exponential-average constants of the gas block.
template <int D, typename T>
__device__ __forceinline__ void facet_term(const Node<D, T> &k, const Node<D, T> &v, const T *a,
                                           const GasC<T> &G, bool diss, T *out, T ip_k = (T)0, T iz1_k = (T)0) {
  facet_term_c<D, T>(k, v, a, G, G.e1, G.e2, diss, out, ip_k, iz1_k);
}

// Harten entropy S = beta rho (p rho^-gamma)^(1/(alpha+gamma)) in FP64.
__device__ __forceinline__ double entropy_harten(double rho, double p, double beta, double g, double inv_apg) {
  return beta * rho * exp((log(p) - g * log(rho)) * inv_apg);
}

}  // namespace sbp

namespace sbp {

// Viscous constants (Sec. 2.2): mu, kappa = mu gamma R / ((gamma-1) Pr), R.
template <typename T>
struct ViscC {
  T mu, kappa, R;
};

// dtheta/dW for theta = p/rho as a function of W (temperature formula of
// Sec. 3, derivatives through the chain rule): out[c] = d theta / d W_c.
template <int D, typename T>
__device__ __forceinline__ void dtheta_dW(const Node<D, T> &n, const GasC<T> &G, T *out) {
  const T iWn = (T)1 / n.w[D + 1];
  T q2 = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) q2 += n.V[k] * n.V[k];
  const T c1 = G.gm1_a * iWn;
  out[0] = c1;
#pragma unroll
  for (int k = 0; k < D; ++k) out[1 + k] = c1 * n.V[k];
  out[D + 1] = (-(n.p / n.rho) + (T)0.5 * G.gm1_a * q2) * iWn;
}

// Viscous flux F^{V(i)}, i = 0..D-1, from the entropy-variable gradient
// gW[j][c] = dW_c/dx_j:  dV/dx_j = -(gW_V + V gW_E)/W_nc,
// dT/dx_j = (dtheta/dW . gW_j)/R,  tau_ik = mu (dV_i/dx_k + dV_k/dx_i
// - 2/3 delta_ik div V),  F^V(i) = [0, tau_i., V.tau_i + kappa dT/dx_i].
template <int D, typename T>
__device__ __forceinline__ void viscous_flux(const Node<D, T> &n, const GasC<T> &G, const ViscC<T> &Vc,
                                             const T gW[D][D + 2], T FV[D][D + 2]) {
  constexpr int NC = D + 2;
  const T iWn = (T)1 / n.w[NC - 1];
  T dth[NC];
  dtheta_dW<D, T>(n, G, dth);
  T dV[D][D];  // dV[j][m] = d V_m / d x_j
  T dT[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    T s = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) s += dth[c] * gW[j][c];
    dT[j] = s / Vc.R;
#pragma unroll
    for (int m = 0; m < D; ++m) dV[j][m] = -(gW[j][1 + m] + n.V[m] * gW[j][NC - 1]) * iWn;
  }
  T div = 0;
#pragma unroll
  for (int m = 0; m < D; ++m) div += dV[m][m];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    FV[i][0] = 0;
    T e = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const T tau = Vc.mu * (dV[k][i] + dV[i][k] - (i == k ? (T)(2.0 / 3.0) * div : (T)0));
      FV[i][1 + k] = tau;
      e += n.V[k] * tau;
    }
    FV[i][NC - 1] = e + Vc.kappa * dT[i];
  }
}

// gbar_j = sum_i K~_ij^T z_i for j = 0..D-1: the adjoint of viscous_flux
// with respect to its gradient argument (F^V(i) = sum_j K~_ij dW/dx_j) for
// cotangents z_i of F^V(i).  Reverse sweep of viscous_flux:
//   tbar_ik = z_i,V_k + z_i,E V_k,  Tbar_i = kappa z_i,E,
//   dVbar_ji = mu (tbar_ij + tbar_ji) - 2/3 mu delta_ij sum_k tbar_kk,
//   gbar_j,V_m = -dVbar_jm / W_nc,  gbar_j,E = -sum_m V_m dVbar_jm / W_nc,
//   gbar_j += (dT/dW) Tbar_j / R.
template <int D, typename T>
__device__ __forceinline__ void viscous_flux_adjoint(const Node<D, T> &n, const GasC<T> &G, const ViscC<T> &Vc,
                                                     const T z[D][D + 2], T gbar[D][D + 2]) {
  constexpr int NC = D + 2;
  const T iWn = (T)1 / n.w[NC - 1];
  T dth[NC];
  dtheta_dW<D, T>(n, G, dth);
  T tb[D][D];
  T tr = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) tb[i][k] = z[i][1 + k] + z[i][NC - 1] * n.V[k];
#pragma unroll
  for (int i = 0; i < D; ++i) tr += tb[i][i];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    T dvb[D];
    T s = 0;
#pragma unroll
    for (int m = 0; m < D; ++m) {
      dvb[m] = Vc.mu * (tb[j][m] + tb[m][j] - (m == j ? (T)(2.0 / 3.0) * tr : (T)0));
      s += n.V[m] * dvb[m];
    }
    const T be = Vc.kappa * z[j][NC - 1] / Vc.R;
    gbar[j][0] = be * dth[0];
#pragma unroll
    for (int m = 0; m < D; ++m) gbar[j][1 + m] = -dvb[m] * iWn + be * dth[1 + m];
    gbar[j][NC - 1] = -s * iWn + be * dth[NC - 1];
  }
}

// y_j = sum_i K~_ij^T (a_i dw) for j = 0..D-1, where K~_ij g is the viscous
// flux F^V(i) produced by the gradient dW/dx_j = g alone.  With
// vt = dw_V + dw_E V and the gradient maps dV/dW, dT/dW:
//   alpha_j = mu [vt_j a + a_j vt - 2/3 (a.vt) e_j],  beta_j = kappa a_j dw_E,
//   y_j = (dV/dW)^T alpha_j + (dT/dW)^T beta_j.
template <int D, typename T>
__device__ __forceinline__ void viscous_adjoint_facet(const Node<D, T> &n, const GasC<T> &G, const ViscC<T> &Vc,
                                                      const T *a, const T *dw, T y[D][D + 2]) {
  constexpr int NC = D + 2;
  const T iWn = (T)1 / n.w[NC - 1];
  T dth[NC];
  dtheta_dW<D, T>(n, G, dth);
  T vt[D];
  T avt = 0;
#pragma unroll
  for (int m = 0; m < D; ++m) {
    vt[m] = dw[1 + m] + dw[NC - 1] * n.V[m];
    avt += a[m] * vt[m];
  }
#pragma unroll
  for (int j = 0; j < D; ++j) {
    T al[D];
    T alV = 0;
#pragma unroll
    for (int m = 0; m < D; ++m) {
      al[m] = Vc.mu * (vt[j] * a[m] + a[j] * vt[m] - (m == j ? (T)(2.0 / 3.0) * avt : (T)0));
      alV += al[m] * n.V[m];
    }
    const T be = Vc.kappa * a[j] * dw[NC - 1] / Vc.R;
    y[j][0] = be * dth[0];
#pragma unroll
    for (int m = 0; m < D; ++m) y[j][1 + m] = -al[m] * iWn + be * dth[1 + m];
    y[j][NC - 1] = -alV * iWn + be * dth[NC - 1];
  }
}

}  // namespace sbp

namespace sbp {

// dU = (dU/dW) g, the state perturbation produced by the entropy-variable
// perturbation g (same chain rule as jvp_flux).
template <int D, typename T>
__device__ __forceinline__ void dU_from_dW(const Node<D, T> &n, const GasC<T> &G, const T *g, T *dU) {
  const T iWn = (T)1 / n.w[D + 1];
  T dV[D];
  T q2 = 0, Vg = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    dV[k] = -(g[1 + k] + n.V[k] * g[D + 1]) * iWn;
    q2 += n.V[k] * n.V[k];
    Vg += n.V[k] * g[1 + k];
  }
  const T theta = n.p / n.rho;
  const T c1 = G.gm1_a * iWn;
  const T dtheta = c1 * (g[0] + Vg) + (-theta + (T)0.5 * G.gm1_a * q2) * iWn * g[D + 1];
  const T drho = n.rho * (g[D + 1] * iWn - G.ja * dtheta / theta) * G.jb_inv;
  const T dp = theta * drho + n.rho * dtheta;
  T VdV = 0;
  dU[0] = drho;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    dU[1 + k] = drho * n.V[k] + n.rho * dV[k];
    VdV += n.V[k] * dV[k];
  }
  dU[D + 1] = dp / G.gm1 + (T)0.5 * q2 * drho + n.rho * VdV;
}

// out = A_i^T z with A_i = dF^(i)/dU (Euler flux Jacobian, closed form).
template <int D, typename T>
__device__ __forceinline__ void flux_jac_T(const Node<D, T> &n, const GasC<T> &G, T E, int i, const T *z, T *out) {
  constexpr int NC = D + 2;
  T q2 = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) q2 += n.V[k] * n.V[k];
  const T Ht = (E + n.p) / n.rho;
  const T g1 = G.gm1;
  // column 0
  T s = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) s += z[1 + j] * (-n.V[i] * n.V[j] + (j == i ? (T)0.5 * g1 * q2 : (T)0));
  out[0] = s + z[NC - 1] * n.V[i] * ((T)0.5 * g1 * q2 - Ht);
  // columns 1+k
#pragma unroll
  for (int k = 0; k < D; ++k) {
    T t = (k == i ? z[0] : (T)0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T a = (k == i ? n.V[j] : (T)0) + (k == j ? n.V[i] : (T)0) - (j == i ? g1 * n.V[k] : (T)0);
      t += z[1 + j] * a;
    }
    t += z[NC - 1] * ((k == i ? Ht : (T)0) - g1 * n.V[i] * n.V[k]);
    out[1 + k] = t;
  }
  // column NC-1
  out[NC - 1] = z[1 + i] * g1 + z[NC - 1] * G.g * n.V[i];
}

}  // namespace sbp
