// Host-callable kernel launchers (implemented in the .hip translation units).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sbp {

// Launch shape of one kernel slot.  Every residual and VJP kernel is
// persistent (its workgroups loop over the element tiles), so any grid is
// correct; grid and kernel variant only change the speed and are picked by
// the autotuner (capi.cpp, sbp_autotune).
struct LaunchCfg {
  int variant = 0;  // 0: the built-in choice; 1: the alternative (see *_variants)
  int grid = 1;     // k > 0: k x (CUs x resident workgroups per CU), capped at
                    // one workgroup per tile; 0: one workgroup per tile
};
constexpr int kGridChoices[3] = {1, 2, 0};

// Workgroups that the device keeps resident for `kernel` (256 threads),
// cached per device and kernel; launch_grid applies LaunchCfg::grid.
int resident_blocks(const void *kernel);
int launch_grid(const void *kernel, int ntiles, int grid);

// Residual of one degree class (form 0: entropy split, 1: Hadamard; the
// Navier-Stokes terms are selected by A.visc).
hipError_t launch_residual(int dim, int p, int form, const KArgs<double> &A, hipStream_t s, LaunchCfg cfg = {});
hipError_t launch_residual(int dim, int p, int form, const KArgs<float> &A, hipStream_t s, LaunchCfg cfg = {});
// form_eff: 0 entropy split, 1 Hadamard, 2 entropy split with Navier-Stokes terms
int residual_blocks(int dim, int p, int precision, int form_eff, int n_elem, LaunchCfg cfg = {});
// kernel variants of a slot: 2D entropy split: one or two node rows per lane;
// 3D entropy split (Euler): skew operators in LDS or read through the caches;
// Hadamard and Navier-Stokes: one
int residual_variants(int dim, int p, int precision, int form_eff);
// 2D entropy split, every degree class in one persistent launch: cls[p-1] is
// the class of degree p or null.  Workgroups of the launch (partial sums):
int residual2_batch_blocks(const int n_elem_of_p[4], int precision, int grid = 1);
// cls_dev: the classes' argument blocks in device memory ([4], by degree;
// the per-call pointers u, r, eform are taken from cls)
hipError_t launch_residual2_batch(const KArgs<double> *const cls[4], const KArgs<double> *cls_dev, double *ent_part,
                                  hipStream_t s, int grid = 1);
hipError_t launch_residual2_batch(const KArgs<float> *const cls[4], const KArgs<float> *cls_dev, double *ent_part,
                                  hipStream_t s, int grid = 1);
// Viscous facet-flux pre-pass (3D): A.qout[(e*NFAC*NF + m)*n_c + c] = B n . F^V
hipError_t launch_visc_q(int dim, int p, const KArgs<double> &A, hipStream_t s);
hipError_t launch_visc_q(int dim, int p, const KArgs<float> &A, hipStream_t s);

// Vector-Jacobian product of the entropy-split residual (FP64, Euler terms).
// Variants: register budget of one or two waves per SIMD.
hipError_t launch_vjp(int dim, int p, const KArgs<double> &A, hipStream_t s, LaunchCfg cfg = {});
int vjp_variants(int dim, int p);
// VJP of the Hadamard form (A.curved selects the curved-tetrahedron kernel);
// elements of the other form are skipped (hybrid scheme, A.eform/A.form_id)
hipError_t launch_vjp_hadamard(int dim, int p, const KArgs<double> &A, hipStream_t s);
// 2D, every degree class in one persistent launch (cls[p-1] or null)
hipError_t launch_vjp2_batch(const KArgs<double> *const cls[4], const KArgs<double> *cls_dev, hipStream_t s,
                             int grid = 1);
// VJP of the Navier-Stokes terms, added to A.ubar (after the Euler terms'
// VJP): a pre-pass writes s = B n . F^V(w, D_x mu) and mu = H^-1 lambda at
// every facet node into sbuf ([n_elem][NFAC*NF][2 n_c] doubles), then the
// main kernel reads both sides' values
hipError_t launch_vjp_viscous(int dim, int p, const KArgs<double> &A, double *sbuf, hipStream_t s);

// Per-node pointwise work over one degree class.
struct NodeArgs {
  const double *u;     // state
  const double *d;     // direction (entropy gap) or null
  const int *uoff;     // [n_elem] element offsets into u
  const double *Hn;    // [n_elem*np] diagonal of H_k
  const double *hmin;  // [n_elem] minimum node distance (time step)
  int n_elem, np, dim;
  double gamma, beta;
  int pstride;         // stride between the partial-sum rows of one launch
  const double *xyz;   // node coordinates, element e at uoff[e]/n_c*dim, [dim][np]
};

// Manufactured solution of the Navier-Stokes study (Sec. 7):
// rho = rho0 + a sin(pi (sum_i x_i - c t)), V_i = V0,
// p = (gamma-1)(rho^2 - rho |V|^2/2); heat = kappa (gamma-1)/R when the heat
// flux is part of the equations (else 0).
struct SrcArgs {
  double rho0, a, c, V0;
  double heat;
  int kind;  // 1: the manufactured solution above; 2: the 3D isentropic vortex of
             // the accuracy study (an exact Euler solution, no source); 3: the 2D
             // isentropic vortex of the accuracy study (idem)
  double alpha, xc, yc;  // 2D vortex: strength and centre at t = 0
  double px, py;         // 2D vortex: box periods (minimum-image distance)
};
constexpr int kNodeThreads = 256;
inline int node_blocks(int n_elem, int np) { return (n_elem * np + kNodeThreads - 1) / kNodeThreads; }

// Device scalars of the relaxation RK step (indices into the handle's
// scalar array): the four stage entropy rates, dt, the requested dt (> 0) or
// the CFL number, e, gamma and its bracket, r(gamma), its rounding level,
// the solve's state (0 running, 1 |r| at rounding level, 2 stalled, 3 no
// valid dt), iterations, the total entropy before and after, a non-positive
// dt flag, the reduced entropy gap (3 values).
enum {
  RK_ENT = 0, RK_DT = 16, RK_DTIN = 22, RK_CFL = 23, RK_E = 24, RK_G = 25, RK_LO = 26, RK_HI = 27,
  RK_F = 28, RK_TOL = 29, RK_DONE = 30, RK_IT = 31, RK_S0 = 32, RK_S1 = 33, RK_BAD = 34, RK_GAP = 40,
  RK_TOTAL = 48
};

// part[v*pstride + b], v = 0,1,2: sum_nodes H [s(u + g d) - s(u)], sum_nodes H w(u + g d).d,
// sum_nodes H |s(u + g d)|; with rk non-null g = rk[RK_G], and nothing is
// done once rk[RK_DONE] != 0
hipError_t launch_entropy_gap(const NodeArgs &A, double g, double *part, hipStream_t s, const double *rk = nullptr);
// rk[RK_DT] = rk[RK_DTIN] > 0 ? rk[RK_DTIN] : rk[RK_CFL] * hmin_over_lam[0]; rk[RK_BAD] if not positive
hipError_t launch_rrk_dt(const double *hmin_over_lam, double *rk, hipStream_t s);
// e from the stage entropy rates, gamma = 1, bracket [0.5, 1.5]
hipError_t launch_rrk_init(double *rk, hipStream_t s);
// one safeguarded Newton step of the relaxation root from the reduced gap
hipError_t launch_rrk_newton(const double *gap, double *rk, hipStream_t s);
// u += gamma d if the device solve ended inside the bracket and *err == 0
hipError_t launch_rrk_update(double *u, const double *d, const double *rk, const int *err, long long n,
                             hipStream_t s);
// part[v*pstride + b], v = 0: sum H s(u); v = 1..n_c: sum H u_c
hipError_t launch_diagnostics(const NodeArgs &A, double *part, hipStream_t s);
// part[b] = min over the block's elements of hmin / max_nodes(|V| + a);
// nothing is done when rk is non-null and rk[RK_DTIN] > 0
hipError_t launch_dt(const NodeArgs &A, double *part, hipStream_t s, const double *rk = nullptr);
// r += S(x, t) at every node (S the manufactured source; r double or float),
// t = *t0 + c * *dt (dt null: t = *t0); part (may be null): per workgroup
// sum_nodes H w(u).S in FP64
hipError_t launch_source_add(const NodeArgs &A, const SrcArgs &P, void *r, int r_f32, const double *t0,
                             const double *dt, double c, double *part, hipStream_t s);
// u = the manufactured state at time t (FP64)
hipError_t launch_source_state(const NodeArgs &A, const SrcArgs &P, double t, double *u, hipStream_t s);
// part[c*pstride + b] = sum_nodes H (u_c - u*_c)^2 at time t
hipError_t launch_source_error(const NodeArgs &A, const SrcArgs &P, double t, double *part, hipStream_t s);
// part[c*pstride + b] = per component sum of w_q J_q (I u - u*)^2 over the
// elements and the points of the degree-(3p+1) error rule (tab: I [nq][np],
// w [nq], for quadratic maps (2D always; 3D when curved) N [nq][NG],
// dN [dim][nq][NG] of the map basis, NG = 6 or 10); launched with
// node_blocks(n_elem, np) workgroups like the other node kernels
hipError_t launch_source_error_quad(const NodeArgs &A, const SrcArgs &P, double t, const double *tab, int nq,
                                   const double *geo, int curved, double *part, hipStream_t s);
// out[v] = reduction over part[v*nb + b], b < nb (op 0: sum, 1: min); fixed order.
hipError_t launch_reduce(const double *part, int nb, int nv, int op, double *out, hipStream_t s);
// y = x + a s z (x null: y = a s z), z double or float (z_f32), n doubles,
// s = *scale (a device scalar read by the kernel) or 1 if scale is null
hipError_t launch_axpy(double *y, const double *x, const void *z, int z_f32, double a, long long n, hipStream_t s,
                       const double *scale = nullptr);
// y = y + a s z (accumulate), z double or float
hipError_t launch_accum(double *y, const void *z, int z_f32, double a, long long n, hipStream_t s,
                        const double *scale = nullptr);
// out[0] = v (device scalar written in stream order)
hipError_t launch_scalar_set(double *out, double v, hipStream_t s);
// out[slot] = sum_k coef_k * in[k] for k < nk (device scalars)
hipError_t launch_scalar_combine(const double *in, const double *coef_dev, int nk, double *out, hipStream_t s);

}  // namespace sbp
