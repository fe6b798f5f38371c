// Time-integration kernels: relaxation RK4 stages, FP64 entropy sums, the
// relaxation root function, the time step and diagnostics (Sec. 6.1, 7.1),
// and the manufactured solution and source of the Navier-Stokes study (Sec. 7).
//
// All reductions are two-stage and deterministic: every workgroup writes one
// partial per quantity, a single workgroup combines the partials in a fixed
// order.  Entropy differences are summed node by node,
// H_m [s(u_m + g d_m) - s(u_m)], to avoid cancellation of two global sums.
#include <hip/hip_runtime.h>

#include <cmath>

#include "launch.hpp"

namespace sbp {

namespace {

constexpr int kT = kNodeThreads;

__device__ __forceinline__ double block_reduce_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

__device__ __forceinline__ double block_reduce_min(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = INFINITY;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmin(s, red[w]);
  return s;
}

// Harten entropy and entropy variables in FP64 from a conservative state.
template <int D>
__device__ __forceinline__ bool ent_state(const double *u, double g, double beta, double *S, double *w) {
  const double alpha = -g - beta * (g - 1.0);
  const double rho = u[0];
  double q2 = 0.0, V[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    V[i] = u[1 + i] / rho;
    q2 += V[i] * V[i];
  }
  const double p = (g - 1.0) * (u[D + 1] - 0.5 * rho * q2);
  const double phi = exp((log(p) - g * log(rho)) / (alpha + g));  // (p rho^-g)^(1/(a+g))
  *S = beta * rho * phi;
  if (w) {
    const double z1 = rho / p * phi;
    w[0] = z1 * (-alpha / (g - 1.0) * p / rho - 0.5 * q2);
#pragma unroll
    for (int i = 0; i < D; ++i) w[1 + i] = z1 * V[i];
    w[D + 1] = -z1;
  }
  return rho > 0.0 && p > 0.0;
}

template <int D>
__global__ __launch_bounds__(kT) void k_entropy_gap(NodeArgs A, double gam, double *part, const double *rk) {
  constexpr int NC = D + 2;
  __shared__ double red[kT / 64];
  // device relaxation solve: gamma from the device scalars, nothing to do
  // once the root is found (the partials are then not read)
  if (rk) {
    if (rk[RK_DONE] != 0.0) return;
    gam = rk[RK_G];
  }
  const int x = blockIdx.x * kT + threadIdx.x;
  double a = 0.0, b = 0.0, m = 0.0;
  if (x < A.n_elem * A.np) {
    const int e = x / A.np, j = x % A.np;
    const int base = A.uoff[e] + j;
    double u0[NC], u1[NC], dd[NC], w1[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      u0[c] = A.u[base + c * A.np];
      dd[c] = A.d[base + c * A.np];
      u1[c] = u0[c] + gam * dd[c];
    }
    double s0, s1;
    ent_state<D>(u0, A.gamma, A.beta, &s0, nullptr);
    ent_state<D>(u1, A.gamma, A.beta, &s1, w1);
    const double H = A.Hn[x];
    a = H * (s1 - s0);
    double wd = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) wd += w1[c] * dd[c];
    b = H * wd;
    m = H * fabs(s1);
  }
  const double sa = block_reduce_sum(a, red);
  const double sb = block_reduce_sum(b, red);
  const double sm = block_reduce_sum(m, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sa;
    part[A.pstride + blockIdx.x] = sb;
    part[2 * A.pstride + blockIdx.x] = sm;
  }
}

template <int D>
__global__ __launch_bounds__(kT) void k_diagnostics(NodeArgs A, double *part) {
  constexpr int NC = D + 2;
  __shared__ double red[kT / 64];
  const int x = blockIdx.x * kT + threadIdx.x;
  double v[NC + 2];
#pragma unroll
  for (int c = 0; c <= NC + 1; ++c) v[c] = 0.0;
  if (x < A.n_elem * A.np) {
    const int e = x / A.np, j = x % A.np;
    const int base = A.uoff[e] + j;
    double u0[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) u0[c] = A.u[base + c * A.np];
    double s;
    ent_state<D>(u0, A.gamma, A.beta, &s, nullptr);
    const double H = A.Hn[x];
    v[0] = H * s;
#pragma unroll
    for (int c = 0; c < NC; ++c) v[1 + c] = H * u0[c];
    // kinetic energy rho |V|^2 / 2 = |rho V|^2 / (2 rho)
    double m2 = 0.0;
#pragma unroll
    for (int i = 1; i <= D; ++i) m2 += u0[i] * u0[i];
    v[NC + 1] = H * (0.5 * m2 / u0[0]);
  }
#pragma unroll
  for (int c = 0; c <= NC + 1; ++c) {
    const double t = block_reduce_sum(v[c], red);
    if (threadIdx.x == 0) part[c * A.pstride + blockIdx.x] = t;
  }
}

// One thread per node computes |V| + a; the element minimum of
// hmin / lambda_max equals min over its nodes of hmin / (|V| + a).
template <int D>
__global__ __launch_bounds__(kT) void k_dt(NodeArgs A, double *part, const double *rk) {
  if (rk && rk[RK_DTIN] > 0.0) return;  // the step size is given
  constexpr int NC = D + 2;
  __shared__ double red[kT / 64];
  const int x = blockIdx.x * kT + threadIdx.x;
  double v = INFINITY;
  if (x < A.n_elem * A.np) {
    const int e = x / A.np, j = x % A.np;
    const int base = A.uoff[e] + j;
    double u0[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) u0[c] = A.u[base + c * A.np];
    const double rho = u0[0];
    double q2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) q2 += (u0[1 + i] / rho) * (u0[1 + i] / rho);
    const double p = (A.gamma - 1.0) * (u0[NC - 1] - 0.5 * rho * q2);
    const double lam = sqrt(q2) + sqrt(A.gamma * p / rho);
    v = A.hmin[e] / lam;
    if (!(v > 0.0)) v = 0.0;  // non-physical state: forces dt = 0, reported by the caller
  }
  const double m = block_reduce_min(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// Manufactured solution of the Navier-Stokes study (Sec. 7) at one node:
// with xi = pi (sum_i x_i - c t), g = d rho/dx_i = a pi cos xi (the same
// for every i), d rho/dt = -c g and, for the constant velocity, the total
// energy e = rho^2; the source du/dt + div F^I - div F^V is
//   mass      (d V0 - c) g
//   momentum  (V0 (d V0 - c) + dp/drho) g,   dp/drho = (gamma-1)(2 rho - d V0^2/2)
//   energy    (d V0 (2 rho + dp/drho) - 2 c rho) g + heat d a pi^2 sin xi
// (the stress vanishes; the heat flux kappa dT/dx_i with T = p/(rho R)
// linear in rho gives the last term).
template <int D>
__device__ __forceinline__ void mms_point(double sx, double gamma, const SrcArgs &P, double t, double *u, double *S) {
  const double xi = M_PI * (sx - P.c * t);
  double sn, cs;
  sincos(xi, &sn, &cs);
  const double rho = P.rho0 + P.a * sn;
  const double q2 = D * P.V0 * P.V0;
  if (u) {
    u[0] = rho;
#pragma unroll
    for (int i = 0; i < D; ++i) u[1 + i] = rho * P.V0;
    u[D + 1] = rho * rho;
  }
  if (S) {
    const double g = P.a * M_PI * cs;
    const double dp = (gamma - 1.0) * (2.0 * rho - 0.5 * q2);
    const double dv = D * P.V0 - P.c;
    S[0] = dv * g;
#pragma unroll
    for (int i = 0; i < D; ++i) S[1 + i] = (P.V0 * dv + dp) * g;
    S[D + 1] = (D * P.V0 * (2.0 * rho + dp) - 2.0 * P.c * rho) * g + P.heat * D * P.a * M_PI * M_PI * sn;
  }
}

// The 3D isentropic vortex of the accuracy study (Sec. 7.3), an exact Euler
// solution: with r^2 = x1^2 + (x2 - t)^2 and g = exp(1 - r^2),
// rho = (1 - 2/25 (gamma-1) g)^(1/(gamma-1)), V = (-2/5 (x2-t) g^(1/2),
// 1 + 2/5 x1 g^(1/2), 0), p = rho^gamma / gamma.
__device__ __forceinline__ void vortex3_point(const double *x, double t, double gamma, double *u) {
  const double y = x[1] - t;
  const double g = exp(1.0 - x[0] * x[0] - y * y), sg = sqrt(g);
  const double lr = log(1.0 - 0.08 * (gamma - 1.0) * g) / (gamma - 1.0);
  const double rho = exp(lr);
  const double V1 = -0.4 * y * sg, V2 = 1.0 + 0.4 * x[0] * sg;
  const double p = exp(gamma * lr) / gamma;
  u[0] = rho;
  u[1] = rho * V1;
  u[2] = rho * V2;
  u[3] = 0.0;
  u[4] = p / (gamma - 1.0) + 0.5 * rho * (V1 * V1 + V2 * V2);
}

// The 2D isentropic vortex of the accuracy study (Sec. 7.3): centre
// (xc + t, yc) advected by the free stream (1, 0), minimum-image distance in
// the periodic box, r^2 = dx^2 + dy^2, f = alpha/(2 pi) exp(1 - r^2):
// V = (1 - f dy, f dx), T = 1 - alpha^2 (gamma-1)/(16 gamma pi^2) exp(2(1 - r^2)),
// rho = T^(1/(gamma-1)), p = rho^gamma.
__device__ __forceinline__ void vortex2_point(const double *x, double t, const SrcArgs &P, double gamma, double *u) {
  double dx = x[0] - (P.xc + t), dy = x[1] - P.yc;
  dx -= P.px * rint(dx / P.px);
  dy -= P.py * rint(dy / P.py);
  const double e1 = exp(1.0 - dx * dx - dy * dy);
  const double T = 1.0 - P.alpha * P.alpha * (gamma - 1.0) / (16.0 * gamma * M_PI * M_PI) * e1 * e1;
  const double lr = log(T) / (gamma - 1.0);
  const double rho = exp(lr), p = exp(gamma * lr);
  const double f = P.alpha / (2.0 * M_PI) * e1;
  const double V0 = 1.0 - f * dy, V1 = f * dx;
  u[0] = rho;
  u[1] = rho * V0;
  u[2] = rho * V1;
  u[3] = p / (gamma - 1.0) + 0.5 * rho * (V0 * V0 + V1 * V1);
}

// the fields of the study selected by P.kind at the point x[D]
template <int D>
__device__ __forceinline__ void fields_at(const double *x, double t, const SrcArgs &P, double gamma, double *u) {
  if constexpr (D == 3) {
    if (P.kind == 2) {
      vortex3_point(x, t, gamma, u);
      return;
    }
  } else {
    if (P.kind == 3) {
      vortex2_point(x, t, P, gamma, u);
      return;
    }
  }
  double sx = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) sx += x[i];
  mms_point<D>(sx, gamma, P, t, u, nullptr);
}

// the source (S, manufactured solution) or the fields (u) at SBP node j of
// element e (either may be null; S only for the manufactured solution)
template <int D>
__device__ __forceinline__ void mms_node(const NodeArgs &A, const SrcArgs &P, int e, int j, double t, double *u,
                                         double *S) {
  const double *xn = A.xyz + (size_t)(A.uoff[e] / (D + 2)) * D + j;
  double x[D];
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = xn[i * A.np];
  if (u) fields_at<D>(x, t, P, A.gamma, u);
  if (S) {
    double sx = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) sx += x[i];
    mms_point<D>(sx, A.gamma, P, t, nullptr, S);
  }
}

template <int D, typename R>
__global__ __launch_bounds__(kT) void k_source_add(NodeArgs A, SrcArgs P, R *r, const double *t0, const double *dt,
                                                    double c, double *part) {
  constexpr int NC = D + 2;
  __shared__ double red[kT / 64];
  const int x = blockIdx.x * kT + threadIdx.x;
  double v = 0.0;
  if (x < A.n_elem * A.np) {
    const int e = x / A.np, j = x % A.np;
    const double t = dt ? t0[0] + c * dt[0] : t0[0];
    double S[NC];
    mms_node<D>(A, P, e, j, t, nullptr, S);
    const int base = A.uoff[e] + j;
#pragma unroll
    for (int k = 0; k < NC; ++k) r[base + k * A.np] = (R)((double)r[base + k * A.np] + S[k]);
    if (part) {
      double u0[NC], w[NC], s;
#pragma unroll
      for (int k = 0; k < NC; ++k) u0[k] = A.u[base + k * A.np];
      ent_state<D>(u0, A.gamma, A.beta, &s, w);
#pragma unroll
      for (int k = 0; k < NC; ++k) v += w[k] * S[k];
      v *= A.Hn[x];
    }
  }
  if (part) {
    const double sum = block_reduce_sum(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// The error of the grid studies (Sec. 7.3): per component sum over elements
// and points q of a degree-(3p+1) rule of w_q J_q (I u - u*)^2(x_q), with I
// the degree-p fit from the nodes to the points.  One thread per (element,
// point), grid-stride over the class.  tab: I [nq][np], w [nq] and, for
// quadratic maps, the map basis N [nq][NG] and its derivatives dN [D][nq][NG]
// at the points (NG = 6 map nodes in 2D, 10 in 3D; x_q and J_q from the
// element's map nodes geo[e][NG][D]); on affine tetrahedra the map is
// reproduced by I applied to the node coordinates and J is the element's
// constant (geo[e][9]).
template <int D>
__global__ __launch_bounds__(kT) void k_source_error_quad(NodeArgs A, SrcArgs P, double t, const double *tab, int nq,
                                                           const double *geo, int curved, double *part) {
  constexpr int NC = D + 2, NG = D == 2 ? 6 : 10;
  __shared__ double red[kT / 64];
  const double *I = tab, *W = tab + (size_t)nq * A.np;
  const double *N = W + nq, *dN = N + (size_t)nq * NG;
  double v[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) v[k] = 0.0;
  const long long total = (long long)A.n_elem * nq;
  for (long long idx = blockIdx.x * (long long)kT + threadIdx.x; idx < total; idx += (long long)gridDim.x * kT) {
    const int e = (int)(idx / nq), q = (int)(idx % nq);
    const int base = A.uoff[e];
    const double *Iq = I + (size_t)q * A.np;
    double uq[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) uq[k] = 0.0;
    for (int j = 0; j < A.np; ++j) {
      const double c = Iq[j];
#pragma unroll
      for (int k = 0; k < NC; ++k) uq[k] += c * A.u[base + k * A.np + j];
    }
    double x[D], J;
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = 0.0;
    if (D == 2 || curved) {
      const double *g = geo + (size_t)e * NG * D;
      double F[D][D];
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int l = 0; l < D; ++l) F[i][l] = 0.0;
      for (int a = 0; a < NG; ++a) {
        const double n = N[q * NG + a];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          x[i] += n * g[a * D + i];
#pragma unroll
          for (int l = 0; l < D; ++l) F[i][l] += dN[(l * nq + q) * NG + a] * g[a * D + i];
        }
      }
      if constexpr (D == 2)
        J = F[0][0] * F[1][1] - F[0][1] * F[1][0];
      else
        J = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
            F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
    } else {
      const double *xn = A.xyz + (size_t)(base / NC) * D;
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < A.np; ++j) x[i] += Iq[j] * xn[i * A.np + j];
      J = geo[(size_t)e * 10 + 9];
    }
    double ue[NC];
    fields_at<D>(x, t, P, A.gamma, ue);
    const double wj = W[q] * J;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const double d = uq[k] - ue[k];
      v[k] += wj * d * d;
    }
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const double sum = block_reduce_sum(v[k], red);
    if (threadIdx.x == 0) part[k * A.pstride + blockIdx.x] = sum;
  }
}

template <int D>
__global__ __launch_bounds__(kT) void k_source_state(NodeArgs A, SrcArgs P, double t, double *u) {
  constexpr int NC = D + 2;
  const int x = blockIdx.x * kT + threadIdx.x;
  if (x < A.n_elem * A.np) {
    const int e = x / A.np, j = x % A.np;
    double ue[NC];
    mms_node<D>(A, P, e, j, t, ue, nullptr);
    const int base = A.uoff[e] + j;
#pragma unroll
    for (int k = 0; k < NC; ++k) u[base + k * A.np] = ue[k];
  }
}

template <int D>
__global__ __launch_bounds__(kT) void k_source_error(NodeArgs A, SrcArgs P, double t, double *part) {
  constexpr int NC = D + 2;
  __shared__ double red[kT / 64];
  const int x = blockIdx.x * kT + threadIdx.x;
  double v[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) v[k] = 0.0;
  if (x < A.n_elem * A.np) {
    const int e = x / A.np, j = x % A.np;
    double ue[NC];
    mms_node<D>(A, P, e, j, t, ue, nullptr);
    const int base = A.uoff[e] + j;
    const double H = A.Hn[x];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const double d = A.u[base + k * A.np] - ue[k];
      v[k] = H * d * d;
    }
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const double sum = block_reduce_sum(v[k], red);
    if (threadIdx.x == 0) part[k * A.pstride + blockIdx.x] = sum;
  }
}

__global__ __launch_bounds__(kT) void k_reduce(const double *part, int nb, int op, double *out) {
  __shared__ double red[kT / 64];
  const int v = blockIdx.x;
  double acc = op == 0 ? 0.0 : INFINITY;
  for (int b = threadIdx.x; b < nb; b += kT) {
    const double x = part[(size_t)v * nb + b];
    acc = op == 0 ? acc + x : fmin(acc, x);
  }
  const double r = op == 0 ? block_reduce_sum(acc, red) : block_reduce_min(acc, red);
  if (threadIdx.x == 0) out[v] = r;
}

// y = x + a s z (x null: y = a s z), s = *scale if scale is not null, else 1
template <typename Z>
__global__ __launch_bounds__(kT) void k_axpy(double *y, const double *x, const Z *z, double a, const double *scale,
                                             long long n) {
  const double as = scale ? a * scale[0] : a;
  for (long long i = blockIdx.x * (long long)kT + threadIdx.x; i < n; i += (long long)gridDim.x * kT)
    y[i] = (x ? x[i] : 0.0) + as * (double)z[i];
}

template <typename Z>
__global__ __launch_bounds__(kT) void k_accum(double *y, const Z *z, double a, const double *scale, long long n) {
  const double as = scale ? a * scale[0] : a;
  for (long long i = blockIdx.x * (long long)kT + threadIdx.x; i < n; i += (long long)gridDim.x * kT)
    y[i] += as * (double)z[i];
}

// Relaxation solve on the device (Sec. 6.1, eq. rrk4 gamma_n): the scalars
// rk[RK_*] (see launch.hpp) hold dt, the stage entropy rates, gamma, the
// bracket and the state of the iteration.
__global__ void k_rrk_dt(const double *hmin_over_lam, double *rk) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double dt = rk[RK_DTIN] > 0.0 ? rk[RK_DTIN] : rk[RK_CFL] * hmin_over_lam[0];
  rk[RK_DT] = dt;
  rk[RK_BAD] = (dt > 0.0 && dt < INFINITY) ? 0.0 : 1.0;
}

// e = dt sum_i b_i w_i^T H r_i; gamma = 1 in the bracket [0.5, 1.5]
__global__ void k_rrk_init(double *rk) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  double e = 0.0;
  for (int i = 0; i < 4; ++i) e += rk[RK_DT] * b[i] * rk[RK_ENT + i];
  rk[RK_E] = e;
  rk[RK_G] = 1.0;
  rk[RK_LO] = 0.5;
  rk[RK_HI] = 1.5;
  rk[RK_DONE] = rk[RK_BAD] != 0.0 ? 3.0 : 0.0;
  rk[RK_IT] = 0.0;
  rk[RK_F] = 0.0;
}

// One Newton step on r(g) = sum H [s(u + g d) - s(u)] - g e from the reduced
// gap[3] = {sum H [s(u + g d) - s(u)], sum H w(u + g d).d, sum H |s(u + g d)|}:
// stop once |r| is at the rounding level of its evaluation (eps sum H |s|),
// DONE = 1, or once the step stalls, DONE = 2; the bracket follows the sign
// of r (r < 0 below the root); a step leaving it or a non-increasing r
// bisects instead.
__global__ void k_rrk_newton(const double *gap, double *rk) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (rk[RK_DONE] != 0.0) return;
  constexpr double eps = 2.220446049250313e-16;
  const double g = rk[RK_G], e = rk[RK_E];
  const double f = gap[0] - g * e, df = gap[1] - e;
  rk[RK_IT] += 1.0;
  rk[RK_F] = f;
  rk[RK_TOL] = eps * gap[2];
  if (fabs(f) <= eps * gap[2]) {
    rk[RK_DONE] = 1.0;
    return;
  }
  if (f < 0.0) rk[RK_LO] = g; else rk[RK_HI] = g;
  const double lo = rk[RK_LO], hi = rk[RK_HI];
  double gn = g - f / df;
  if (!(df > 0.0) || !(gn > lo && gn < hi)) gn = 0.5 * (lo + hi);
  if (gn == g || fabs(gn - g) <= eps * g || hi - lo <= 4.0 * eps * g) rk[RK_DONE] = 2.0;
  rk[RK_G] = gn;
}

// u += g d once the solve has ended inside the bracket and no kernel of the
// step has flagged a non-physical state (else u is left unchanged: for the
// host's safeguarded solve, or for the error return)
__global__ __launch_bounds__(kT) void k_rrk_update(double *u, const double *d, const double *rk, const int *err,
                                                   long long n) {
  const double done = rk[RK_DONE], g = rk[RK_G];
  if (!(done == 1.0 || done == 2.0) || !(g > 0.5 && g < 1.5) || *err != 0) return;
  for (long long i = blockIdx.x * (long long)kT + threadIdx.x; i < n; i += (long long)gridDim.x * kT)
    u[i] += g * d[i];
}

__global__ void k_scalar_set(double *out, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = v;
}

__global__ void k_scalar_combine(const double *in, const double *coef, int nk, double *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < nk; ++k) s += coef[k] * in[k];
    out[0] = s;
  }
}

int grid_for(long long n) {
  long long b = (n + kT - 1) / kT;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

hipError_t launch_entropy_gap(const NodeArgs &A, double g, double *part, hipStream_t s, const double *rk) {
  const int nb = node_blocks(A.n_elem, A.np);
  if (A.dim == 2)
    hipLaunchKernelGGL(k_entropy_gap<2>, dim3(nb), dim3(kT), 0, s, A, g, part, rk);
  else
    hipLaunchKernelGGL(k_entropy_gap<3>, dim3(nb), dim3(kT), 0, s, A, g, part, rk);
  return hipGetLastError();
}

hipError_t launch_diagnostics(const NodeArgs &A, double *part, hipStream_t s) {
  const int nb = node_blocks(A.n_elem, A.np);
  if (A.dim == 2)
    hipLaunchKernelGGL(k_diagnostics<2>, dim3(nb), dim3(kT), 0, s, A, part);
  else
    hipLaunchKernelGGL(k_diagnostics<3>, dim3(nb), dim3(kT), 0, s, A, part);
  return hipGetLastError();
}

hipError_t launch_dt(const NodeArgs &A, double *part, hipStream_t s, const double *rk) {
  const int nb = node_blocks(A.n_elem, A.np);
  if (A.dim == 2)
    hipLaunchKernelGGL(k_dt<2>, dim3(nb), dim3(kT), 0, s, A, part, rk);
  else
    hipLaunchKernelGGL(k_dt<3>, dim3(nb), dim3(kT), 0, s, A, part, rk);
  return hipGetLastError();
}

hipError_t launch_source_add(const NodeArgs &A, const SrcArgs &P, void *r, int r_f32, const double *t0,
                             const double *dt, double c, double *part, hipStream_t s) {
  const int nb = node_blocks(A.n_elem, A.np);
  if (A.dim == 2) {
    if (r_f32)
      hipLaunchKernelGGL((k_source_add<2, float>), dim3(nb), dim3(kT), 0, s, A, P, (float *)r, t0, dt, c, part);
    else
      hipLaunchKernelGGL((k_source_add<2, double>), dim3(nb), dim3(kT), 0, s, A, P, (double *)r, t0, dt, c, part);
  } else {
    if (r_f32)
      hipLaunchKernelGGL((k_source_add<3, float>), dim3(nb), dim3(kT), 0, s, A, P, (float *)r, t0, dt, c, part);
    else
      hipLaunchKernelGGL((k_source_add<3, double>), dim3(nb), dim3(kT), 0, s, A, P, (double *)r, t0, dt, c, part);
  }
  return hipGetLastError();
}

hipError_t launch_source_state(const NodeArgs &A, const SrcArgs &P, double t, double *u, hipStream_t s) {
  const int nb = node_blocks(A.n_elem, A.np);
  if (A.dim == 2)
    hipLaunchKernelGGL(k_source_state<2>, dim3(nb), dim3(kT), 0, s, A, P, t, u);
  else
    hipLaunchKernelGGL(k_source_state<3>, dim3(nb), dim3(kT), 0, s, A, P, t, u);
  return hipGetLastError();
}

hipError_t launch_source_error_quad(const NodeArgs &A, const SrcArgs &P, double t, const double *tab, int nq,
                                   const double *geo, int curved, double *part, hipStream_t s) {
  const int nb = node_blocks(A.n_elem, A.np);
  if (A.dim == 2)
    hipLaunchKernelGGL(k_source_error_quad<2>, dim3(nb), dim3(kT), 0, s, A, P, t, tab, nq, geo, curved, part);
  else
    hipLaunchKernelGGL(k_source_error_quad<3>, dim3(nb), dim3(kT), 0, s, A, P, t, tab, nq, geo, curved, part);
  return hipGetLastError();
}

hipError_t launch_source_error(const NodeArgs &A, const SrcArgs &P, double t, double *part, hipStream_t s) {
  const int nb = node_blocks(A.n_elem, A.np);
  if (A.dim == 2)
    hipLaunchKernelGGL(k_source_error<2>, dim3(nb), dim3(kT), 0, s, A, P, t, part);
  else
    hipLaunchKernelGGL(k_source_error<3>, dim3(nb), dim3(kT), 0, s, A, P, t, part);
  return hipGetLastError();
}

hipError_t launch_reduce(const double *part, int nb, int nv, int op, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(nv), dim3(kT), 0, s, part, nb, op, out);
  return hipGetLastError();
}

hipError_t launch_axpy(double *y, const double *x, const void *z, int z_f32, double a, long long n, hipStream_t s,
                       const double *scale) {
  if (z_f32)
    hipLaunchKernelGGL(k_axpy<float>, dim3(grid_for(n)), dim3(kT), 0, s, y, x, (const float *)z, a, scale, n);
  else
    hipLaunchKernelGGL(k_axpy<double>, dim3(grid_for(n)), dim3(kT), 0, s, y, x, (const double *)z, a, scale, n);
  return hipGetLastError();
}

hipError_t launch_accum(double *y, const void *z, int z_f32, double a, long long n, hipStream_t s,
                        const double *scale) {
  if (z_f32)
    hipLaunchKernelGGL(k_accum<float>, dim3(grid_for(n)), dim3(kT), 0, s, y, (const float *)z, a, scale, n);
  else
    hipLaunchKernelGGL(k_accum<double>, dim3(grid_for(n)), dim3(kT), 0, s, y, (const double *)z, a, scale, n);
  return hipGetLastError();
}

hipError_t launch_scalar_set(double *out, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_scalar_set, dim3(1), dim3(64), 0, s, out, v);
  return hipGetLastError();
}

hipError_t launch_scalar_combine(const double *in, const double *coef_dev, int nk, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_scalar_combine, dim3(1), dim3(64), 0, s, in, coef_dev, nk, out);
  return hipGetLastError();
}

hipError_t launch_rrk_dt(const double *hmin_over_lam, double *rk, hipStream_t s) {
  hipLaunchKernelGGL(k_rrk_dt, dim3(1), dim3(64), 0, s, hmin_over_lam, rk);
  return hipGetLastError();
}

hipError_t launch_rrk_init(double *rk, hipStream_t s) {
  hipLaunchKernelGGL(k_rrk_init, dim3(1), dim3(64), 0, s, rk);
  return hipGetLastError();
}

hipError_t launch_rrk_newton(const double *gap, double *rk, hipStream_t s) {
  hipLaunchKernelGGL(k_rrk_newton, dim3(1), dim3(64), 0, s, gap, rk);
  return hipGetLastError();
}

hipError_t launch_rrk_update(double *u, const double *d, const double *rk, const int *err, long long n,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_rrk_update, dim3(grid_for(n)), dim3(kT), 0, s, u, d, rk, err, n);
  return hipGetLastError();
}

}  // namespace sbp
