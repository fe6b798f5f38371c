/*
 * sbp.h -- C ABI of the MI355X entropy-split SBP-SAT residual library.
 *
 * The library evaluates the semi-discrete residual du/dt = r(u) of the
 * entropy-split summation-by-parts discretization of the Euler and
 * compressible Navier-Stokes equations on periodic triangle and tetrahedral
 * meshes (Worku & Zingg, efficient form Sec. 6.2, eq. weak form split), and
 * advances it by relaxation RK4 (Sec. 6.1).  All compute runs in HIP kernels
 * for gfx950; the host part only prepares mesh tables.
 *
 * Conventions
 *   - Every call returns int: SBP_OK (0) or a negative SBP_E* code; nothing
 *     throws across the ABI.  sbp_last_error() gives a thread-local message.
 *   - State layout: for element e with n_p(e) SBP nodes and n_c = dim + 2
 *     components (rho, rho V_1..rho V_dim, e), the values of element e start
 *     at double offset node_off[e] * n_c and are stored component-major:
 *     u[node_off[e]*n_c + c*n_p(e) + j].  For a single-degree mesh this is a
 *     dense [n_elem][n_c][n_p] array.  node_off is reported by sbp_mesh_info.
 *   - Device pointers are caller-owned HIP device allocations; the library
 *     never frees them.  Host arrays passed to sbp_setup_mesh are borrowed for
 *     the duration of the call only.
 *   - hip_stream is a hipStream_t (NULL = default stream).  Residual calls are
 *     asynchronous on that stream; sbp_rrk_step synchronises it.
 *   - Device-detected non-physical states (rho <= 0, p <= 0 or NaN) raise a
 *     flag that the next synchronising call (sbp_rrk_step, sbp_mesh_info,
 *     sbp_check_device) reports as SBP_ENONPHYS.
 */
#ifndef SBP_H
#define SBP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbp_mesh sbp_mesh; /* opaque, owned by the library */

enum sbp_status {
  SBP_OK = 0,
  SBP_EINVAL = -1,   /* invalid argument (reported at once, nothing launched) */
  SBP_ENOMEM = -2,   /* device or host allocation failed */
  SBP_EDEVICE = -3,  /* HIP runtime error */
  SBP_ENOTSUP = -4,  /* combination not supported by this library */
  SBP_ENONPHYS = -5, /* rho <= 0, p <= 0 or NaN seen on the device */
  SBP_ERRK = -6      /* relaxation parameter not bracketed / not converged */
};

enum { SBP_FORM_SPLIT = 0, SBP_FORM_HADAMARD = 1 };
enum { SBP_FP64 = 0, SBP_FP32 = 1 };

/* Mesh description (paper Sec. 2.1: conforming elements, periodic domain).
 * Vertices on the periodic boundary may be duplicated; facets are matched by
 * their vertex centroids and facet nodes by coordinates modulo `period`.   */
typedef struct {
  int32_t dim;                 /* 2 = triangles, 3 = tetrahedra                  */
  int32_t n_vert, n_elem;
  const double *vert_xyz;      /* [n_vert][dim], host                             */
  const int32_t *elem_vert;    /* [n_elem][dim+1], positively oriented            */
  int32_t p_geom;              /* 1 affine; 2 quadratic map (3D: degrees p >= 2,
                                  Assumption 1)                                   */
  const double *geom_nodes;    /* 2D: [n_elem][6][2] P2 map nodes (v0,v1,v2,m01,m12,m20);
                                  3D: [n_elem][10][3] (v0..v3, m01,m12,m02,m03,m13,m23);
                                  NULL when p_geom == 1                           */
  const double *period;        /* [dim] periodic box lengths                      */
  const int32_t *elem_degree;  /* [n_elem] SBP degree p (2D: 1..4, 3D: 1..3),
                                  uniform inside each problem                     */
  const int32_t *problem_off;  /* [n_problems+1] element ranges of independent
                                  problems (facets never couple two problems),
                                  or NULL for one problem                         */
  int32_t n_problems;          /* >= 1                                            */
} sbp_mesh_desc;

/* Physical and scheme parameters. */
typedef struct {
  double gamma;        /* ratio of specific heats (Sec. 2.2: 7/5)                  */
  double beta;         /* split parameter; alpha = -gamma - beta (gamma-1)
                          (Sec. 2.4; Sec. 6.4 uses beta = 2.5)                     */
  int32_t form;        /* SBP_FORM_SPLIT or SBP_FORM_HADAMARD (Sec. 6.2)           */
  int32_t dissipation; /* 1: matrix interface dissipation (Sec. 4.5)              */
  int32_t viscous;     /* 1: Navier-Stokes terms with Baumann-Oden SATs (Sec. 5)   */
  int32_t heat_flux;   /* 1: include kappa grad T in the viscous flux             */
  double mu, Pr, R;    /* viscosity, Prandtl number, gas constant                  */
  int32_t precision;   /* SBP_FP64 or SBP_FP32 (residual kernels; reductions FP64) */
} sbp_physics;

typedef struct {
  int32_t dim, n_c;
  int32_t n_elem;
  int64_t n_nodes;           /* total SBP nodes, sum_e n_p(e)                     */
  const int64_t *node_off;   /* host array [n_elem+1] owned by the handle         */
  const int32_t *elem_np;    /* host array [n_elem]: n_p(e)                       */
  const double *node_xyz;    /* device array [n_nodes*dim], element e at
                                node_off[e]*dim, layout [dim][n_p(e)]             */
  const double *node_h;      /* device array [n_nodes]: diagonal of H_k           */
  double t;                  /* time held by the handle (advanced by RRK steps)   */
} sbp_info;

typedef struct {
  double gamma_n;        /* relaxation parameter                                 */
  double dt;             /* nominal step (the solution advanced by gamma_n dt)   */
  double t;              /* time after the step                                  */
  double entropy_before; /* 1^T H s(u_n)                                         */
  double entropy_after;  /* 1^T H s(u_{n+1})                                     */
  double entropy_rate_e; /* dt sum_i b_i w_i^T H r_i                             */
  int32_t newton_iters;  /* gamma root-solve iterations                          */
} sbp_rrk_report;

/* Build a mesh handle: reference operators (Def. 1), metrics, facet matching,
 * device tables.  `hip_stream` is used for the uploads.  Paper: Sec. 2.1.
 * Curved tetrahedra (p_geom 2 in 3D) need every degree >= 2 (Assumption 1:
 * p_geom <= floor(p/2) + 1), else SBP_EINVAL.  The viscous terms (Sec. 5)
 * need the entropy-split form (else SBP_ENOTSUP) and run on triangles and
 * tetrahedra, affine or curved. */
int sbp_setup_mesh(const sbp_mesh_desc *desc, const sbp_physics *phys,
                   void *hip_stream, sbp_mesh **out);

/* Query layout and device tables.  Also reports a pending device error. */
int sbp_mesh_info(sbp_mesh *mesh, sbp_info *out);

/* r = du/dt at state u (Sec. 6.2, eq. weak form split; Hadamard form eq. weak
 * form 2pt when phys.form == SBP_FORM_HADAMARD).  u_dev: doubles, r_dev:
 * doubles (FP64) or floats (FP32), both in the state layout above.  If
 * entropy_rate_dev != NULL the FP64 scalar sum_k w_k^T H_k r_k is written to
 * it.  Asynchronous on hip_stream. */
int sbp_residual(sbp_mesh *mesh, const void *u_dev, void *r_dev,
                 double *entropy_rate_dev, void *hip_stream);

/* The same residual as sbp_residual, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the call allocates nothing; its device scratch (the
 * entropy rate's per-workgroup partial sums, reduction scalars and, with the
 * manufactured source, the node partials) lives in one static device array of
 * 2^17 doubles (1 MiB) per GPU, held until the process ends.  Arguments,
 * layouts and results as for sbp_residual (bitwise the same values).
 * SBP_EINVAL when the mesh needs more scratch than the array holds (meshes of
 * up to about 10^5 workgroup tiles; the message gives both sizes).  Every call
 * on a GPU shares that GPU's array and leaves its contents behind: calls that
 * overlap on one GPU (other streams, other threads) race and must be ordered
 * by the caller.  Nothing in the array needs to start at zero.  The facet
 * viscous fluxes that the two kernels of a Navier-Stokes residual exchange
 * live in a buffer of the handle, allocated by sbp_setup_mesh, so calls on
 * one handle must not overlap either.  Not in the paper. */
int sbp_residual_noalloc(sbp_mesh *mesh, const void *u_dev, void *r_dev,
                         double *entropy_rate_dev, void *hip_stream);

/* ubar = (dr/du)^T lambda (vector-Jacobian product of sbp_residual).  Not in
 * the paper.  Layouts as for sbp_residual, all FP64 (also on FP32 meshes: the
 * VJP kernels compute in FP64).  Every residual the library evaluates: Euler
 * terms with or without dissipation in either volume form and with the
 * hybrid form flags, and the Navier-Stokes terms (viscous flux with heat
 * flux, Baumann-Oden SATs), on affine and curved elements.  Asynchronous on
 * hip_stream. */
int sbp_residual_vjp(sbp_mesh *mesh, const void *u_dev, const void *lambda_dev,
                     void *ubar_dev, void *hip_stream);

/* One relaxation RK4 step in place (Sec. 6.1, eqs. rrk4 gamma_n, rrk_update).
 * dt > 0: use it; dt <= 0: dt = cfl * min_k h_min,k / |lambda|_max,k
 * (Sec. 7.1).  rep may be NULL.  Synchronises hip_stream.
 * The relaxation parameter is the root near 1 of sum H [s(u + g d) - s(u)] -
 * g e, e = dt sum_i b_i w_i^T H r_i, found by Newton steps from g = 1
 * safeguarded by bisection on [0.5, 1.5].  The whole step (step size, the
 * four RK stages, up to 8 Newton steps on device scalars, the update and the
 * report's entropy sums) is one device sequence with no host round trip,
 * captured once per state pointer and report flag as a HIP graph on a
 * private stream of the handle and replayed on hip_stream (see
 * sbp_use_graphs); the host reads its scalars once at the end.  If those
 * Newton steps have not settled, the host continues the solve (u still
 * unchanged) and evaluates the bracket; SBP_ERRK if the root is not
 * bracketed there.  On any error u is left unchanged. */
int sbp_rrk_step(sbp_mesh *mesh, void *u_dev, double dt, double cfl,
                 sbp_rrk_report *rep, void *hip_stream);

/* Hybrid scheme (Sec. 4.4, Thm. switching hybrid): per element the volume
 * term of the entropy-split form (eq. weak form split) or of the Hadamard
 * form (eq. weak form 2pt), with the same SATs; entropy conservation holds for
 * any choice, and the elements on the Hadamard form conserve locally.
 * form_dev: device array of n_elem bytes in the element order of the mesh
 * description, 0 = entropy split, any nonzero byte = Hadamard; borrowed:
 * every later sbp_residual and sbp_rrk_step reads it, so the caller may
 * change its contents between calls (switching between time steps; a
 * captured RK stage graph reads the same array).  NULL returns every element
 * to phys.form.
 * SBP_ENOTSUP with the viscous terms.  sbp_residual_vjp follows the flags.
 * The FP64 entropy rate sums both launches. */
int sbp_set_volume_form(sbp_mesh *mesh, const uint8_t *form_dev);

/* Source terms of the manufactured-solution study (Sec. 7, manufactured
 * solution for the compressible Navier-Stokes equations): the fields
 *   rho = rho0 + a sin(pi (sum_i x_i - c t)),  V_i = V0 (every i),
 *   p = (gamma - 1) (rho^2 - rho |V|^2 / 2)
 * solve du/dt = r(u) + S(x, t) with S = du/dt + div F^I - div F^V of the
 * fields (the heat flux enters when phys.viscous and phys.heat_flux; the
 * stress vanishes for the constant velocity).
 * kind SBP_SOURCE_NS_MMS: every later sbp_residual adds S at the handle's
 * time (sbp_set_time), and sbp_rrk_step at each RK stage time t + c_i dt
 * (the entropy rates then include w^T H S).  params = {rho0, a, c, V0}
 * (host, read during the call), or NULL for the paper's {2, 0.1, 0.6, 1}.
 * kind SBP_SOURCE_VORTEX3D selects the 3D isentropic vortex of the accuracy
 * study (Sec. 7.3; r^2 = x1^2 + (x2 - t)^2, g = exp(1 - r^2),
 * rho = (1 - 2/25 (gamma-1) g)^(1/(gamma-1)), V = (-2/5 (x2-t) g^(1/2),
 * 1 + 2/5 x1 g^(1/2), 0), p = rho^gamma / gamma): an exact solution of the
 * Euler equations, so no source term is added; it only sets the fields of
 * sbp_source_state and sbp_source_error (3D meshes, params ignored; the
 * fields decay like exp(-r^2), so a box such as the paper's [-10,10]^3 is
 * periodic to rounding).
 * kind SBP_SOURCE_VORTEX2D selects the 2D isentropic vortex of the accuracy
 * study (Sec. 7.3): strength alpha, centre (xc + t, yc) advected by the free
 * stream (1, 0), minimum-image distance in the mesh's periodic box,
 * f = alpha/(2 pi) exp(1 - r^2), V = (1 - f dy, f dx),
 * T = 1 - alpha^2 (gamma-1)/(16 gamma pi^2) exp(2 (1 - r^2)),
 * rho = T^(1/(gamma-1)), p = rho^gamma; params = {alpha, xc, yc} or NULL for
 * the paper's {3, 5, 0}; no source term (2D meshes; SBP_EINVAL if the
 * temperature at the centre would not be positive).
 * kind SBP_SOURCE_NONE removes the source.  SBP_EINVAL for an unknown kind,
 * non-finite parameters, rho0 - |a| <= d V0^2 / 2 (the pressure would not
 * stay positive) or a box side that is not a multiple of 2 (the fields have
 * period 2 in every x_i). */
enum { SBP_SOURCE_NONE = 0, SBP_SOURCE_NS_MMS = 1, SBP_SOURCE_VORTEX3D = 2, SBP_SOURCE_VORTEX2D = 3 };
int sbp_set_source(sbp_mesh *mesh, int32_t kind, const double *params);

/* u_dev (FP64, state layout) = the fields of the source set by
 * sbp_set_source at the SBP nodes at time t.  SBP_EINVAL when no source is
 * set.  Asynchronous on hip_stream. */
int sbp_source_state(sbp_mesh *mesh, double t, void *u_dev, void *hip_stream);

/* Squared L2 error against the manufactured fields u* at time t, per
 * component c (n_c values in out_host):
 *   norm SBP_NORM_QUADRATURE (the grid studies, Sec. 7.3): the nodal values
 *     of each element are fitted by a polynomial of degree p (least squares
 *     weighted by the reference norm h, exact for degree p) and the squared
 *     error integrated with a collapsed Gauss-Legendre rule of degree 3p + 1
 *     on the element's map (affine or quadratic);
 *   norm SBP_NORM_NODAL: sum_k (u_k - u*_k)^T H_k (u_k - u*_k) at the nodes.
 * FP64; synchronises hip_stream.  The rule's device tables are built on the
 * first quadrature call.  SBP_EINVAL when no source is set or for an unknown
 * norm. */
enum { SBP_NORM_NODAL = 0, SBP_NORM_QUADRATURE = 1 };
int sbp_source_error(sbp_mesh *mesh, const void *u_dev, double t, int32_t norm, double *out_host,
                     void *hip_stream);

/* enable != 0 (default): sbp_rrk_step replays its captured stage graph;
 * enable == 0: the stages are launched one by one (for callers that capture
 * the stream themselves).  Not in the paper.  SBP_EINVAL for a null handle. */
int sbp_use_graphs(sbp_mesh *mesh, int enable);

/* One kernel slot tuned by sbp_autotune. */
typedef struct {
  int32_t kind;         /* 0: residual, 1: VJP                                    */
  int32_t p;            /* degree class; 0: all classes of a 2D mesh in one launch */
  int32_t variant;      /* chosen kernel variant (0: the built-in choice)         */
  int32_t grid;         /* chosen grid: k > 0 -> k x resident workgroups (at most
                           one per tile); 0 -> one workgroup per tile             */
  int32_t n_candidates; /* launch shapes timed                                    */
  double ms_builtin;    /* mean launch time of variant 0, grid 1                  */
  double ms_best;       /* mean launch time of the chosen shape                   */
} sbp_tune_slot;

typedef struct {
  int32_t n_slots;
  sbp_tune_slot slot[8];
} sbp_tune_report;

/* Autotuner (not in the paper): for every kernel slot of the handle (each
 * degree class of sbp_residual, or its single batched launch on a 2D mesh
 * with several degrees; likewise of sbp_residual_vjp when lambda_dev != NULL)
 * time each launch shape -- kernel variant (2D entropy split: one or two node
 * rows per lane, the next tile's neighbour data loaded ahead or not; 3D
 * entropy split: skew operators in LDS or read through the caches; VJP:
 * register budget of one or two waves per SIMD) times persistent grid (1x or 2x the resident workgroups, or
 * one workgroup per tile) -- on the state u_dev and keep the fastest for
 * later calls.  Results of all shapes agree up to the summation order of the
 * FP64 entropy rate.  Choices are remembered for the process per workload
 * (dimension, degree, precision, form, physics flags, element count, device);
 * handles set up later with the same workload start from them.  A captured
 * RRK stage graph is re-captured on the next sbp_rrk_step.  rep may be NULL.
 * Synchronises hip_stream; overwrites the handle's RK work buffers.
 * SBP_EINVAL for a null handle or state; SBP_EDEVICE if a launch fails. */
int sbp_autotune(sbp_mesh *mesh, const void *u_dev, const void *lambda_dev, sbp_tune_report *rep,
                 void *hip_stream);

/* Read or pin the launch shape of one kernel slot: kind 0 residual, 1 VJP;
 * p the degree class, or 0 for the batched launch of a 2D mesh with several
 * degrees; variant < the slot's variant count (entropy split without the
 * Navier-Stokes terms: 3 on triangles, 2 on tetrahedra; VJP: 2; otherwise 1);
 * grid 0..64 as in sbp_tune_slot.  Not in the paper.
 * SBP_EINVAL for a slot the handle does not have or a value out of range. */
int sbp_get_launch_shape(sbp_mesh *mesh, int32_t kind, int32_t p, int32_t *variant, int32_t *grid);
int sbp_set_launch_shape(sbp_mesh *mesh, int32_t kind, int32_t p, int32_t variant, int32_t grid);

/* Launch timing (not in the paper; for benchmarks and profilers) of the
 * entropy-split residual kernels on triangles (Euler terms; one launch per
 * degree class, or the one batched launch of a mesh of several degrees).
 * sbp_time_launches(mesh, capacity): from now on every sbp_residual call on
 * the handle records, per launch, the earliest workgroup start and the
 * latest workgroup end of the kernel on the device's constant-rate clock
 * (hipDeviceAttributeWallClockRate), in call order, until capacity launches
 * are recorded; the kernel writes them itself, so the stream carries no
 * extra packets.  capacity 0 stops the recording; any call discards earlier
 * records; allocates the record (2 x 8 bytes per launch) and synchronises
 * the device.  Other entry points (RK steps, the allocation-free residual,
 * the autotuner) are never timed.  SBP_EINVAL for a null handle or capacity
 * outside 0..65536; SBP_ENOTSUP (capacity > 0) for other meshes.
 * sbp_launch_times(mesh, ms_out, max, n_out): synchronises the device,
 * writes the first min(recorded, max) durations in milliseconds to ms_out
 * (host, caller-owned) and their count to *n_out, and clears the record
 * (recording continues). */
int sbp_time_launches(sbp_mesh *mesh, int32_t capacity);
int sbp_launch_times(sbp_mesh *mesh, double *ms_out, int32_t max, int32_t *n_out);

/* FP64 diagnostics on the device, results copied to host (synchronises):
 * out[0] = 1^T H s(u); out[1..n_c] = sum_k 1^T H_k u_k per component;
 * out[n_c + 1] = sum_k 1^T H_k (rho |V|^2 / 2), the kinetic energy whose
 * scaled form E_k = out[n_c + 1] / (rho_0 |Omega|) the viscous Taylor-Green
 * study follows (Sec. 7.5).  out_host holds n_c + 2 doubles, caller-owned;
 * u_dev is a state laid out as for sbp_residual.  Null arguments give
 * SBP_EINVAL. */
int sbp_diagnostics(sbp_mesh *mesh, const void *u_dev, double *out_host,
                    void *hip_stream);

/* Report (and clear) a pending device-side error flag. Synchronises. */
int sbp_check_device(sbp_mesh *mesh, void *hip_stream);

int sbp_set_time(sbp_mesh *mesh, double t);

int sbp_destroy_mesh(sbp_mesh *mesh);

const char *sbp_last_error(void);

/* Host-only query of the reference-element operator the library builds for
 * (dim, p) (Def. 1): n_p nodes, n_f nodes per facet.  Arrays (row-major):
 * nodes [n_p][dim], h [n_p], Q [dim][n_p][n_p], E [dim][n_p],
 * facet_nodes [dim+1][n_f], facet_w [dim+1][n_f].  Any pointer may be NULL.
 * No device is touched. */
int sbp_reference_operator(int32_t dim, int32_t p, int32_t *n_p, int32_t *n_f,
                           double *nodes, double *h, double *Q, double *E,
                           int32_t *facet_nodes, double *facet_w);

#ifdef __cplusplus
}
#endif
#endif /* SBP_H */
