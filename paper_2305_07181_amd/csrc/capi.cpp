// C ABI of the library (include/sbp.h): mesh setup on the host, device
// tables, residual dispatch, relaxation RK4 driver.
//
// Setup (Sec. 2.1): per element the map x(xi) (affine, or quadratic through
// the vertices and edge midpoints in 2D), metric cofactors Lambda_il =
// J dxi_l/dx_i, H_k = J H_ref, the minimum node distance h_min (Sec. 7.1);
// facets matched by vertex centroids modulo the period, facet nodes by
// coordinates modulo the period, stored as the u offset of the matching
// neighbour node (the face-node permutation, resolved once).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/sbp.h"
#include "launch.hpp"
#include "refops.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? SBP_ENOMEM : SBP_EDEVICE,                \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
};

struct DegreeClass {
  int p = 0, np = 0, nf = 0, n_elem = 0;
  std::vector<int> elems;  // global element ids
  int *d_uoff = nullptr;
  int u_dense = 0, u_base = 0;  // d_uoff[k] == u_base + k n_c n_p for every k
  int *d_gid = nullptr;   // mesh element id of each element of the class
  double *d_geo = nullptr;
  int *d_nbr = nullptr;
  double *d_Hn = nullptr;
  double *d_hmin = nullptr;
  void *d_ops = nullptr;  // both precisions
  sbp::OpTables<double> op64{};
  sbp::OpTables<float> op32{};
  int *d_nbrq = nullptr;  // viscous: neighbour q index per facet node
  void *d_q = nullptr;    // viscous: facet normal viscous fluxes
  double *d_vq = nullptr; // viscous VJP: s and mu at the facet nodes
  int part_off = 0;       // offset of this class in the residual partial buffer
  int res_blocks = 0;     // partial sums reserved: the largest grid of any launch shape
  int part_off_h = 0, res_blocks_h = 0;  // hybrid scheme: the Hadamard launch's partial sums
  sbp::LaunchCfg res_cfg, vjp_cfg;  // launch shapes (autotuner)
  int node_off_blk = 0;   // offset in the node partial buffers
  int node_blocks = 0;
  double *d_eq = nullptr;  // error rule of the grid studies (built on first use)
  int eq_nq = 0;
};

}  // namespace

struct sbp_mesh {
  int dim = 0, nc = 0, n_elem = 0;
  long long n_nodes = 0;
  long long n_dof = 0;  // doubles in a state vector
  std::vector<int64_t> node_off;
  std::vector<int> elem_np;
  sbp_physics phys{};
  std::vector<DegreeClass> cls;
  double *d_node_xyz = nullptr;
  double *d_node_h = nullptr;
  double *d_part = nullptr;   // residual partials (sum over classes of blocks)
  int part_total = 0;
  int batch_blocks = 0;       // 2D entropy split with several degree classes: one launch
  int batch_grid = 1, vjp_batch_grid = 1;  // grid choices of the batched launches (autotuner)
  const unsigned char *eform = nullptr;      // hybrid scheme: caller's per-element form flags
  double *d_npart = nullptr;  // node-kernel partials [(n_c+2) x node_total]
  int node_total = 0;
  double *d_scal = nullptr;   // device scalars
  void *d_eac = nullptr;      // exponential-average constants [2] per precision (FP64 then FP32)
  // 2D meshes of several degrees: the argument blocks of the degree classes
  // ([4] by degree, static fields) for the batched launches
  sbp::KArgs<double> *d_bcls64 = nullptr;
  sbp::KArgs<float> *d_bcls32 = nullptr;
  int *d_err = nullptr;
  double *d_y = nullptr, *d_d = nullptr;
  void *d_r = nullptr;        // RK stage residual
  double t = 0.0;
  double period[3] = {0.0, 0.0, 0.0};
  int curved3 = 0;            // tetrahedra with quadratic maps (per-node metrics)
  int src_kind = 0;           // SBP_SOURCE_*: source added to every residual
  sbp::SrcArgs src{};
  // RRK steps captured once as a HIP graph (per state pointer and report
  // mode), replayed on the caller's stream; captured on a private stream of
  // default priority
  int use_graphs = 1;
  // launch timing of sbp_residual (sbp_time_launches): per timed launch a
  // slot {earliest start, latest end} of device clock ticks, in call order
  unsigned long long *d_tstamp = nullptr;
  int t_cap = 0, t_n = 0;
  bool timing_call = false;   // set inside sbp_residual only (never under capture)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t rk_exec = nullptr;
  const void *rk_u = nullptr;
  int rk_rep = -1;
};

namespace {

// Kernel family of the residual: 0 entropy split, 1 Hadamard, 2 entropy
// split with the Navier-Stokes terms, 3 and 4 entropy split and Hadamard on
// curved tetrahedra, 5 entropy split with the Navier-Stokes terms on curved
// tetrahedra.
int curved_eff(const sbp_mesh *M, int form) {
  return M->curved3 ? (form == SBP_FORM_SPLIT ? 3 : 4) : form;
}
int form_eff_of(const sbp_mesh *M) {
  if (M->phys.viscous) return M->curved3 ? 5 : 2;
  return curved_eff(M, M->phys.form);
}

// device table of the pointwise constants read at their use: per precision
// (FP64 at 0, FP32 at kEacPrec) the exponential-average constants, then at
// kEacJump the binomial coefficients of the node powers
constexpr size_t kEacPrec = 1024, kEacJump = 512;

constexpr int SC_ENT = sbp::RK_ENT;  // 4 stage entropy rates
constexpr int SC_RED = 8;     // reduction outputs (up to 8)
constexpr int SC_DT = sbp::RK_DT;    // time step of the current RRK step
constexpr int SC_T = 17;      // time at the start of the current RRK step
constexpr int SC_TR = 18;     // time of a residual call (the handle's time)
constexpr int SC_SRC = 20;    // entropy rates of the residual and of the source (2)
constexpr int SC_TOTAL = sbp::RK_TOTAL;  // 22.. hold the device relaxation solve (sbp::RK_*)
static_assert(SC_SRC + 2 <= sbp::RK_DTIN && SC_T < SC_TR && SC_RED + 8 <= SC_DT, "scalar slots overlap");

// --------------------------------------------------------------------------
// geometry helpers
void p2_dbasis(double x, double y, double dN[2][6]) {
  const double l[3] = {1.0 - x - y, x, y};
  const double dl[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
  for (int k = 0; k < 2; ++k) {
    for (int a = 0; a < 3; ++a) dN[k][a] = (4.0 * l[a] - 1.0) * dl[a][k];
    const int pr[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    for (int q = 0; q < 3; ++q) {
      const int a = pr[q][0], b = pr[q][1];
      dN[k][3 + q] = 4.0 * (dl[a][k] * l[b] + l[a] * dl[b][k]);
    }
  }
}

// Quadratic tetrahedron: vertices 0..3, then the edge midpoints of the
// edges (0,1) (1,2) (0,2) (0,3) (1,3) (2,3); derivatives dN[l][a] = dN_a/dxi_l.
const int kP2TetEdges[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};

void p2t_basis(const double *xi, double N[10], double dN[3][10]) {
  const double l[4] = {1.0 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]};
  const double dl[4][3] = {{-1.0, -1.0, -1.0}, {1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  for (int a = 0; a < 4; ++a) {
    N[a] = l[a] * (2.0 * l[a] - 1.0);
    for (int k = 0; k < 3; ++k) dN[k][a] = (4.0 * l[a] - 1.0) * dl[a][k];
  }
  for (int q = 0; q < 6; ++q) {
    const int a = kP2TetEdges[q][0], b = kP2TetEdges[q][1];
    N[4 + q] = 4.0 * l[a] * l[b];
    for (int k = 0; k < 3; ++k) dN[k][4 + q] = 4.0 * (dl[a][k] * l[b] + l[a] * dl[b][k]);
  }
}

void p2_basis(double x, double y, double N[6]) {
  const double l0 = 1.0 - x - y, l1 = x, l2 = y;
  N[0] = l0 * (2 * l0 - 1);
  N[1] = l1 * (2 * l1 - 1);
  N[2] = l2 * (2 * l2 - 1);
  N[3] = 4 * l0 * l1;
  N[4] = 4 * l1 * l2;
  N[5] = 4 * l2 * l0;
}

struct KeyHash {
  size_t operator()(const std::array<long long, 4> &k) const {
    size_t h = 1469598103934665603ull;
    for (long long v : k) h = (h ^ (size_t)v) * 1099511628211ull;
    return h;
  }
};

template <typename T>
int upload(T *&dst, const std::vector<T> &src, hipStream_t s) {
  HIPCHK(hipMalloc((void **)&dst, std::max<size_t>(1, src.size()) * sizeof(T)));
  if (!src.empty()) HIPCHK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return SBP_OK;
}

// Operator tables of one class for precision T: skew parts S_l = Q_l - E_l/2,
// H and E diagonals, and (2D) the quadratic-map basis derivatives at the nodes.
template <typename T>
void build_tables(const sbp::RefOp &op, int dim, std::vector<T> &blob, size_t off[11]) {
  const int NP = op.np;
  auto Q = [&](int l, int i, int j) { return op.Q[((size_t)l * NP + i) * NP + j]; };
  auto align = [&](size_t n) { return (n + 63) / 64 * 64; };
  blob.clear();
  auto push = [&](const std::vector<double> &v) {
    size_t o = blob.size();
    blob.resize(align(o + v.size()), (T)0);
    for (size_t k = 0; k < v.size(); ++k) blob[o + k] = (T)v[k];
    return o;
  };
  std::vector<double> S((size_t)dim * NP * NP);
  for (int l = 0; l < dim; ++l)
    for (int m = 0; m < NP; ++m)
      for (int n = 0; n < NP; ++n)
        S[((size_t)l * NP + m) * NP + n] = Q(l, m, n) - (m == n ? 0.5 * op.E[(size_t)l * NP + m] : 0.0);
  off[4] = push(S);
  off[5] = push(op.h);
  off[6] = push(op.E);
  std::vector<double> dN;
  if (dim == 2) {
    dN.assign((size_t)2 * 6 * NP, 0.0);
    for (int j = 0; j < NP; ++j) {
      double d[2][6];
      p2_dbasis(op.nodes[2 * j], op.nodes[2 * j + 1], d);
      for (int k = 0; k < 2; ++k)
        for (int a = 0; a < 6; ++a) dN[((size_t)k * 6 + a) * NP + j] = d[k][a];
    }
  } else {
    // quadratic tetrahedral maps: [3][10][NP]
    dN.assign((size_t)3 * 10 * NP, 0.0);
    for (int j = 0; j < NP; ++j) {
      double n[10], d[3][10];
      p2t_basis(&op.nodes[(size_t)3 * j], n, d);
      for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 10; ++a) dN[((size_t)k * 10 + a) * NP + j] = d[k][a];
    }
  }
  off[7] = push(dN);
}

template <typename T>
sbp::OpTables<T> tables_at(const T *base, const size_t off[11], int dim) {
  sbp::OpTables<T> t{};
  t.S = base + off[4];
  t.h = base + off[5];
  t.E = base + off[6];
  t.dN = base + off[7];
  return t;
}

void apply_tuned(sbp_mesh *M);

template <typename T>
sbp::KArgs<T> kargs(sbp_mesh *M, DegreeClass &c, const double *u, void *r, const sbp::OpTables<T> &op);

int setup_impl(const sbp_mesh_desc *D, const sbp_physics *ph, hipStream_t s, sbp_mesh *M) {
  const int dim = D->dim;
  M->dim = dim;
  M->nc = dim + 2;
  M->n_elem = D->n_elem;
  M->phys = *ph;
  const int nv = dim + 1;
  const int ne = D->n_elem;
  std::vector<int> prob_of(ne, 0);
  if (D->problem_off) {
    for (int q = 0; q < D->n_problems; ++q) {
      if (D->problem_off[q] > D->problem_off[q + 1] || D->problem_off[q + 1] > ne)
        return fail(SBP_EINVAL, "problem_off not monotone within [0, n_elem]");
      for (int e = D->problem_off[q]; e < D->problem_off[q + 1]; ++e) prob_of[e] = q;
    }
    if (D->problem_off[0] != 0 || D->problem_off[D->n_problems] != ne)
      return fail(SBP_EINVAL, "problem_off must cover [0, n_elem]");
  }
  // degree per element, uniform per problem
  std::vector<int> deg(ne);
  for (int e = 0; e < ne; ++e) {
    deg[e] = D->elem_degree[e];
    if (dim == 2 && (deg[e] < 1 || deg[e] > 4)) return fail(SBP_ENOTSUP, "triangle degree must be 1..4");
    if (dim == 3 && (deg[e] < 1 || deg[e] > 3)) return fail(SBP_ENOTSUP, "tetrahedron degree must be 1..3");
    if (e > 0 && prob_of[e] == prob_of[e - 1] && deg[e] != deg[e - 1])
      return fail(SBP_EINVAL, "degree must be uniform inside a problem");
  }
  // layout
  M->node_off.assign(ne + 1, 0);
  M->elem_np.assign(ne, 0);
  for (int e = 0; e < ne; ++e) {
    const sbp::RefOp &op = sbp::reference_operator(dim, deg[e]);
    M->elem_np[e] = op.np;
    M->node_off[e + 1] = M->node_off[e] + op.np;
  }
  M->n_nodes = M->node_off[ne];
  M->n_dof = M->n_nodes * M->nc;
  if (M->n_dof >= (1ll << 31) - 1) return fail(SBP_ENOTSUP, "state larger than 2^31 doubles");
  // geometry on the host
  std::vector<double> xyz((size_t)M->n_nodes * dim);
  std::vector<double> Hn(M->n_nodes);
  std::vector<double> geo2, geo3;
  std::vector<double> hmin(ne);
  const double *P = D->period;
  for (int e = 0; e < ne; ++e) {
    const sbp::RefOp &op = sbp::reference_operator(dim, deg[e]);
    const int np = op.np;
    double g[6][3] = {};
    const int32_t *ev = D->elem_vert + (size_t)e * nv;
    for (int a = 0; a < nv; ++a) {
      if (ev[a] < 0 || ev[a] >= D->n_vert) return fail(SBP_EINVAL, "elem_vert out of range");
      for (int i = 0; i < dim; ++i) g[a][i] = D->vert_xyz[(size_t)ev[a] * dim + i];
    }
    double *xe = xyz.data() + (size_t)M->node_off[e] * dim;
    if (dim == 2) {
      double gn[6][2];
      if (D->p_geom == 2) {
        for (int a = 0; a < 6; ++a)
          for (int i = 0; i < 2; ++i) gn[a][i] = D->geom_nodes[((size_t)e * 6 + a) * 2 + i];
      } else {
        for (int a = 0; a < 3; ++a)
          for (int i = 0; i < 2; ++i) gn[a][i] = g[a][i];
        const int pr[3][2] = {{0, 1}, {1, 2}, {2, 0}};
        for (int q = 0; q < 3; ++q)
          for (int i = 0; i < 2; ++i) gn[3 + q][i] = 0.5 * (g[pr[q][0]][i] + g[pr[q][1]][i]);
      }
      for (int a = 0; a < 6; ++a)
        for (int i = 0; i < 2; ++i) geo2.push_back(gn[a][i]);
      for (int j = 0; j < np; ++j) {
        double N[6], dN[2][6];
        p2_basis(op.nodes[2 * j], op.nodes[2 * j + 1], N);
        p2_dbasis(op.nodes[2 * j], op.nodes[2 * j + 1], dN);
        double F[2][2] = {{0, 0}, {0, 0}}, x[2] = {0, 0};
        for (int a = 0; a < 6; ++a)
          for (int i = 0; i < 2; ++i) {
            x[i] += N[a] * gn[a][i];
            F[i][0] += dN[0][a] * gn[a][i];
            F[i][1] += dN[1][a] * gn[a][i];
          }
        const double J = F[0][0] * F[1][1] - F[0][1] * F[1][0];
        if (!(J > 0)) return fail(SBP_EINVAL, "non-positive Jacobian (element " + std::to_string(e) + ")");
        xe[0 * np + j] = x[0];
        xe[1 * np + j] = x[1];
        Hn[M->node_off[e] + j] = J * op.h[j];
      }
    } else if (D->p_geom == 2) {
      // quadratic map: metric cofactors and J at every node (geo: the ten map nodes)
      double gn[10][3];
      for (int a = 0; a < 10; ++a)
        for (int i = 0; i < 3; ++i) {
          gn[a][i] = D->geom_nodes[((size_t)e * 10 + a) * 3 + i];
          geo3.push_back(gn[a][i]);
        }
      for (int j = 0; j < np; ++j) {
        double N[10], dN[3][10], F[3][3] = {}, x[3] = {};
        p2t_basis(&op.nodes[(size_t)3 * j], N, dN);
        for (int a = 0; a < 10; ++a)
          for (int i = 0; i < 3; ++i) {
            x[i] += N[a] * gn[a][i];
            for (int l = 0; l < 3; ++l) F[i][l] += dN[l][a] * gn[a][i];
          }
        const double J = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                         F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                         F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
        if (!(J > 0)) return fail(SBP_EINVAL, "non-positive Jacobian (element " + std::to_string(e) + ")");
        for (int i = 0; i < 3; ++i) xe[i * np + j] = x[i];
        Hn[M->node_off[e] + j] = J * op.h[j];
      }
    } else {
      double F[3][3];
      for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l) F[i][l] = g[l + 1][i] - g[0][i];
      double C[3][3];  // cofactors
      for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l) {
          const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, l1 = (l + 1) % 3, l2 = (l + 2) % 3;
          C[i][l] = F[i1][l1] * F[i2][l2] - F[i1][l2] * F[i2][l1];
        }
      const double J = F[0][0] * C[0][0] + F[0][1] * C[0][1] + F[0][2] * C[0][2];
      if (!(J > 0)) return fail(SBP_EINVAL, "non-positive Jacobian (element " + std::to_string(e) + ")");
      for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l) geo3.push_back(C[i][l]);
      geo3.push_back(J);
      for (int j = 0; j < np; ++j) {
        for (int i = 0; i < 3; ++i) {
          double x = g[0][i];
          for (int l = 0; l < 3; ++l) x += F[i][l] * op.nodes[3 * j + l];
          xe[i * np + j] = x;
        }
        Hn[M->node_off[e] + j] = J * op.h[j];
      }
    }
    double hm = INFINITY;
    for (int a = 0; a < np; ++a)
      for (int b = a + 1; b < np; ++b) {
        double d2 = 0;
        for (int i = 0; i < dim; ++i) {
          const double d = xe[i * np + a] - xe[i * np + b];
          d2 += d * d;
        }
        hm = std::min(hm, std::sqrt(d2));
      }
    hmin[e] = hm;
  }
  // facet matching by centroid keys modulo the period, per problem
  std::unordered_map<std::array<long long, 4>, std::pair<int, int>, KeyHash> table;
  table.reserve((size_t)ne * nv);
  std::vector<int> nb_elem((size_t)ne * nv, -1), nb_fac((size_t)ne * nv, -1);
  const long long RES = 1ll << 22;
  for (int e = 0; e < ne; ++e)
    for (int f = 0; f < nv; ++f) {
      double c[3] = {0, 0, 0};
      for (int a = 0; a < nv; ++a) {
        if (a == f) continue;
        const int vtx = D->elem_vert[(size_t)e * nv + a];
        for (int i = 0; i < dim; ++i) c[i] += D->vert_xyz[(size_t)vtx * dim + i] / dim;
      }
      std::array<long long, 4> key{0, 0, 0, prob_of[e]};
      for (int i = 0; i < dim; ++i) {
        long long q = (long long)std::llround(c[i] / P[i] * (double)RES);
        key[i] = ((q % RES) + RES) % RES;
      }
      auto it = table.find(key);
      if (it == table.end()) {
        table.emplace(key, std::make_pair(e, f));
      } else {
        const int v = it->second.first, g2 = it->second.second;
        if (nb_elem[(size_t)v * nv + g2] >= 0) return fail(SBP_EINVAL, "facet shared by more than two elements");
        nb_elem[(size_t)e * nv + f] = v;
        nb_fac[(size_t)e * nv + f] = g2;
        nb_elem[(size_t)v * nv + g2] = e;
        nb_fac[(size_t)v * nv + g2] = f;
      }
    }
  for (size_t k = 0; k < nb_elem.size(); ++k)
    if (nb_elem[k] < 0) return fail(SBP_EINVAL, "unmatched facet (mesh not periodic/conforming)");
  // degree classes
  std::vector<int> class_of_p(5, -1);
  for (int e = 0; e < ne; ++e) {
    if (class_of_p[deg[e]] < 0) {
      class_of_p[deg[e]] = (int)M->cls.size();
      DegreeClass c;
      c.p = deg[e];
      const sbp::RefOp &op = sbp::reference_operator(dim, deg[e]);
      c.np = op.np;
      c.nf = op.nf;
      M->cls.push_back(c);
    }
    M->cls[class_of_p[deg[e]]].elems.push_back(e);
  }
  int part_total = 0, node_total = 0;
  const int prec = ph->precision;
  std::vector<int> local_of(ne, -1);
  for (auto &c : M->cls)
    for (size_t k = 0; k < c.elems.size(); ++k) local_of[c.elems[k]] = (int)k;
  M->curved3 = dim == 3 && D->p_geom == 2;
  const int form_eff = form_eff_of(M);
  for (auto &c : M->cls) {
    c.n_elem = (int)c.elems.size();
    const sbp::RefOp &op = sbp::reference_operator(dim, c.p);
    const int np = c.np, nf = c.nf;
    std::vector<int> uoff(c.n_elem), nbr((size_t)c.n_elem * nv * nf), nbrq((size_t)c.n_elem * nv * nf);
    std::vector<double> geo, hn((size_t)c.n_elem * np), hm(c.n_elem);
    const int gsz = dim == 2 ? 12 : (D->p_geom == 2 ? 30 : 10);
    for (int k = 0; k < c.n_elem; ++k) {
      const int e = c.elems[k];
      uoff[k] = (int)(M->node_off[e] * M->nc);
      const std::vector<double> &G = dim == 2 ? geo2 : geo3;
      geo.insert(geo.end(), G.begin() + (size_t)e * gsz, G.begin() + (size_t)(e + 1) * gsz);
      for (int j = 0; j < np; ++j) hn[(size_t)k * np + j] = Hn[M->node_off[e] + j];
      hm[k] = hmin[e];
      const double *xe = xyz.data() + (size_t)M->node_off[e] * dim;
      for (int f = 0; f < nv; ++f) {
        const int v = nb_elem[(size_t)e * nv + f], g2 = nb_fac[(size_t)e * nv + f];
        const double *xv = xyz.data() + (size_t)M->node_off[v] * dim;
        const int npv = M->elem_np[v];
        for (int j = 0; j < nf; ++j) {
          const int m = op.facet_nodes[(size_t)f * nf + j];
          int best = -1;
          double bd = INFINITY;
          for (int jj = 0; jj < nf; ++jj) {
            const int mv = op.facet_nodes[(size_t)g2 * nf + jj];
            double d2 = 0;
            for (int i = 0; i < dim; ++i) {
              double d = xe[i * np + m] - xv[i * npv + mv];
              d -= P[i] * std::nearbyint(d / P[i]);
              d2 += d * d;
            }
            if (d2 < bd) { bd = d2; best = mv; }
          }
          if (!(std::sqrt(bd) <= 1e-8 * std::max(hmin[e], 1.0)))
            return fail(SBP_EINVAL, "facet nodes do not match (element " + std::to_string(e) + ")");
          nbr[((size_t)k * nv + f) * nf + j] = (int)(M->node_off[v] * M->nc) + best;
          nbrq[((size_t)k * nv + f) * nf + j] = local_of[v] * nv * nf + best;
        }
      }
    }
    int rc;
    c.u_base = uoff.empty() ? 0 : uoff[0];
    c.u_dense = 1;
    for (int k = 0; k < c.n_elem; ++k)
      if (uoff[k] != c.u_base + k * M->nc * np) c.u_dense = 0;
    if ((rc = upload(c.d_uoff, uoff, s))) return rc;
    if ((rc = upload(c.d_gid, c.elems, s))) return rc;
    if ((rc = upload(c.d_geo, geo, s))) return rc;
    if ((rc = upload(c.d_nbr, nbr, s))) return rc;
    if ((rc = upload(c.d_Hn, hn, s))) return rc;
    if ((rc = upload(c.d_hmin, hm, s))) return rc;
    if ((rc = upload(c.d_nbrq, nbrq, s))) return rc;
    if (ph->viscous) {
      HIPCHK(hipMalloc(&c.d_q, sizeof(double) * (size_t)c.n_elem * nv * nf * M->nc));
      HIPCHK(hipMalloc((void **)&c.d_vq, sizeof(double) * (size_t)c.n_elem * nv * nf * 2 * M->nc));
    }
    std::vector<double> b64;
    std::vector<float> b32;
    size_t o64[11], o32[11];
    build_tables<double>(op, dim, b64, o64);
    build_tables<float>(op, dim, b32, o32);
    const size_t bytes64 = b64.size() * sizeof(double), bytes32 = b32.size() * sizeof(float);
    HIPCHK(hipMalloc(&c.d_ops, bytes64 + bytes32));
    HIPCHK(hipMemcpyAsync(c.d_ops, b64.data(), bytes64, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync((char *)c.d_ops + bytes64, b32.data(), bytes32, hipMemcpyHostToDevice, s));
    c.op64 = tables_at<double>((const double *)c.d_ops, o64, dim);
    c.op32 = tables_at<float>((const float *)((char *)c.d_ops + bytes64), o32, dim);
    c.res_blocks = 0;
    for (int pr = 0; pr < 2; ++pr)
      for (int v = 0; v < sbp::residual_variants(dim, c.p, pr, form_eff); ++v)
        c.res_blocks = std::max(c.res_blocks, sbp::residual_blocks(dim, c.p, pr, form_eff, c.n_elem, {v, 0}));
    c.part_off = part_total;
    part_total += c.res_blocks;
    c.node_blocks = sbp::node_blocks(c.n_elem, np);
    c.node_off_blk = node_total;
    node_total += c.node_blocks;
  }
  (void)prec;
  if (dim == 2 && form_eff == 0 && M->cls.size() > 1) {
    int ne_p[4] = {0, 0, 0, 0};
    for (auto &c : M->cls) ne_p[c.p - 1] = c.n_elem;
    M->batch_blocks = std::max(sbp::residual2_batch_blocks(ne_p, 0, 0), sbp::residual2_batch_blocks(ne_p, 1, 0));
    part_total = std::max(part_total, M->batch_blocks);
  }
  if (!ph->viscous)  // the hybrid scheme's second launch (the other volume form) per class
    for (auto &c : M->cls) {
      const int other = ph->form == SBP_FORM_SPLIT ? SBP_FORM_HADAMARD : SBP_FORM_SPLIT;
      c.res_blocks_h = 0;
      for (int pr = 0; pr < 2; ++pr)
        c.res_blocks_h = std::max(c.res_blocks_h, sbp::residual_blocks(dim, c.p, pr, curved_eff(M, other), c.n_elem, {0, 1}));
      c.part_off_h = part_total;
      part_total += c.res_blocks_h;
    }
  M->part_total = part_total;
  M->node_total = node_total;
  int rc;
  if ((rc = upload(M->d_node_xyz, xyz, s))) return rc;
  if ((rc = upload(M->d_node_h, Hn, s))) return rc;
  HIPCHK(hipMalloc((void **)&M->d_part, sizeof(double) * std::max(1, part_total)));
  HIPCHK(hipMalloc((void **)&M->d_npart, sizeof(double) * (M->nc + 2) * std::max(1, node_total)));
  {
    const sbp::GasC<double> g64 = sbp::make_gas<double>(ph->gamma, ph->beta);
    const sbp::GasC<float> g32 = sbp::make_gas<float>(ph->gamma, ph->beta);
    const sbp::ExpAvgC<double> e64[2] = {g64.e1, g64.e2};
    const sbp::ExpAvgC<float> e32[2] = {g32.e1, g32.e2};
    const sbp::JumpC<double> j64 = sbp::make_jump<double>(ph->gamma, ph->beta);
    const sbp::JumpC<float> j32 = sbp::make_jump<float>(ph->gamma, ph->beta);
    static_assert(sizeof(e64) <= kEacJump && sizeof(j64) <= kEacPrec - kEacJump, "constant table layout");
    HIPCHK(hipMalloc(&M->d_eac, 2 * kEacPrec));
    char *base = (char *)M->d_eac;
    HIPCHK(hipMemcpy(base, e64, sizeof(e64), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(base + kEacJump, &j64, sizeof(j64), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(base + kEacPrec, e32, sizeof(e32), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(base + kEacPrec + kEacJump, &j32, sizeof(j32), hipMemcpyHostToDevice));
  }
  HIPCHK(hipMalloc((void **)&M->d_scal, sizeof(double) * SC_TOTAL));
  HIPCHK(hipMemsetAsync(M->d_scal, 0, sizeof(double) * SC_TOTAL, s));
  HIPCHK(hipMalloc((void **)&M->d_err, sizeof(int)));
  HIPCHK(hipMemsetAsync(M->d_err, 0, sizeof(int), s));
  if (M->batch_blocks > 0 || (dim == 2 && M->cls.size() > 1)) {
    std::vector<sbp::KArgs<double>> b64(4);
    std::vector<sbp::KArgs<float>> b32(4);
    for (auto &c : M->cls) {
      b64[c.p - 1] = kargs<double>(M, c, nullptr, nullptr, c.op64);
      b32[c.p - 1] = kargs<float>(M, c, nullptr, nullptr, c.op32);
    }
    if ((rc = upload(M->d_bcls64, b64, s))) return rc;
    if ((rc = upload(M->d_bcls32, b32, s))) return rc;
  }
  HIPCHK(hipStreamSynchronize(s));
  apply_tuned(M);
  return SBP_OK;
}

sbp::NodeArgs node_args(const sbp_mesh *M, const DegreeClass &c, const double *u, const double *d) {
  sbp::NodeArgs A{};
  A.u = u;
  A.d = d;
  A.uoff = c.d_uoff;
  A.Hn = c.d_Hn;
  A.hmin = c.d_hmin;
  A.n_elem = c.n_elem;
  A.np = c.np;
  A.dim = M->dim;
  A.gamma = M->phys.gamma;
  A.beta = M->phys.beta;
  A.pstride = M->node_total;
  A.xyz = M->d_node_xyz;
  return A;
}

template <typename T>
sbp::KArgs<T> kargs(sbp_mesh *M, DegreeClass &c, const double *u, void *r, const sbp::OpTables<T> &op) {
  const sbp_physics &ph = M->phys;
  sbp::KArgs<T> A{};
  A.u = u;
  A.r = (T *)r;
  A.geo = c.d_geo;
  A.nbr = c.d_nbr;
  A.uoff = c.d_uoff;
  A.u_dense = c.u_dense;
  A.u_base = c.u_base;
  A.gid = c.d_gid;
  A.Hn = c.d_Hn;
  A.n_elem = c.n_elem;
  A.diss = ph.dissipation;
  A.op = op;
  A.G = sbp::make_gas<T>(ph.gamma, ph.beta);
  const char *eac = (const char *)M->d_eac + (sizeof(T) == 8 ? 0 : kEacPrec);
  A.eac = (const sbp::ExpAvgC<T> *)eac;
  A.jc = (const sbp::JumpC<T> *)(eac + kEacJump);
  A.ent_part = M->d_part + c.part_off;
  A.err = M->d_err;
  A.visc = ph.viscous;
  A.curved = M->curved3;
  A.nbrq = c.d_nbrq;
  if (ph.viscous) {
    A.V.mu = (T)ph.mu;
    A.V.R = (T)ph.R;
    A.V.kappa = ph.heat_flux ? (T)(ph.mu * ph.gamma * ph.R / ((ph.gamma - 1.0) * ph.Pr)) : (T)0;
    A.q = (const T *)c.d_q;
    A.qout = (T *)c.d_q;
  }
  return A;
}

// Device scratch of one residual evaluation: the per-workgroup partial sums
// of the entropy rate (part, M->part_total values), the reduction and time
// scalars (scal, SC_TOTAL values) and the node-kernel partials of the
// manufactured source's entropy rate (npart, M->node_total values).  The
// handle's own buffers serve sbp_residual and the RK stages; the static
// scratch array serves sbp_residual_noalloc.  Every value is written before
// it is read within one evaluation, so nothing needs clearing.
struct Work {
  double *part, *scal, *npart;
};
Work handle_work(const sbp_mesh *M) { return Work{M->d_part, M->d_scal, M->d_npart}; }
size_t work_doubles(const sbp_mesh *M) {
  return (size_t)std::max(1, M->part_total) + SC_TOTAL +
         (M->src_kind == SBP_SOURCE_NS_MMS ? (size_t)std::max(1, M->node_total) : 0);
}

int residual_core(sbp_mesh *M, const Work &W, const double *u, void *r, double *ent_dev, hipStream_t s) {
  const sbp_physics &ph = M->phys;
  if (ph.viscous) {
    for (auto &c : M->cls) {
      if (ph.precision == SBP_FP64)
        HIPCHK(sbp::launch_visc_q(M->dim, c.p, kargs<double>(M, c, u, r, c.op64), s));
      else
        HIPCHK(sbp::launch_visc_q(M->dim, c.p, kargs<float>(M, c, u, r, c.op32), s));
    }
  }
  // hybrid scheme (Sec. 4.4): the mesh's own form runs on the elements flagged
  // with it, the other form on the rest, each with the shared SATs; the second
  // launch keeps its partial sums apart
  const bool hyb = M->eform != nullptr;
  const int form_other = ph.form == SBP_FORM_SPLIT ? SBP_FORM_HADAMARD : SBP_FORM_SPLIT;
  auto other_launch = [&](DegreeClass &c) -> int {
    if (ph.precision == SBP_FP64) {
      sbp::KArgs<double> A = kargs<double>(M, c, u, r, c.op64);
      A.eform = M->eform;
      A.form_id = form_other;
      A.ent_part = W.part + c.part_off_h;
      HIPCHK(sbp::launch_residual(M->dim, c.p, form_other, A, s, sbp::LaunchCfg{0, 1}));
    } else {
      sbp::KArgs<float> A = kargs<float>(M, c, u, r, c.op32);
      A.eform = M->eform;
      A.form_id = form_other;
      A.ent_part = W.part + c.part_off_h;
      HIPCHK(sbp::launch_residual(M->dim, c.p, form_other, A, s, sbp::LaunchCfg{0, 1}));
    }
    return SBP_OK;
  };
  auto other_blocks = [&](const DegreeClass &c) {
    return sbp::residual_blocks(M->dim, c.p, ph.precision, curved_eff(M, form_other), c.n_elem, sbp::LaunchCfg{0, 1});
  };
  const int ncls = (int)M->cls.size();
  int rc;
  if (M->batch_blocks > 0 && ph.form == SBP_FORM_SPLIT && !ph.viscous) {
    // every degree class in one persistent launch
    sbp::KArgs<double> a64[4];
    sbp::KArgs<float> a32[4];
    const sbp::KArgs<double> *p64[4] = {nullptr, nullptr, nullptr, nullptr};
    const sbp::KArgs<float> *p32[4] = {nullptr, nullptr, nullptr, nullptr};
    // launch timing: one slot for the one launch
    unsigned long long *ts = nullptr;
    if (M->timing_call && M->t_n < M->t_cap) ts = M->d_tstamp + 2 * (size_t)M->t_n++;
    for (auto &c : M->cls) {
      if (ph.precision == SBP_FP64) {
        a64[c.p - 1] = kargs<double>(M, c, u, r, c.op64);
        a64[c.p - 1].eform = M->eform;
        a64[c.p - 1].tstamp = ts;
        p64[c.p - 1] = &a64[c.p - 1];
      } else {
        a32[c.p - 1] = kargs<float>(M, c, u, r, c.op32);
        a32[c.p - 1].eform = M->eform;
        a32[c.p - 1].tstamp = ts;
        p32[c.p - 1] = &a32[c.p - 1];
      }
    }
    if (ph.precision == SBP_FP64)
      HIPCHK(sbp::launch_residual2_batch(p64, M->d_bcls64, W.part, s, M->batch_grid));
    else
      HIPCHK(sbp::launch_residual2_batch(p32, M->d_bcls32, W.part, s, M->batch_grid));
    if (hyb)
      for (auto &c : M->cls)
        if ((rc = other_launch(c))) return rc;
    if (ent_dev) {
      int ne_p[4] = {0, 0, 0, 0};
      for (auto &c : M->cls) ne_p[c.p - 1] = c.n_elem;
      const int nb = sbp::residual2_batch_blocks(ne_p, ph.precision == SBP_FP64 ? 0 : 1, M->batch_grid);
      if (!hyb) {
        HIPCHK(sbp::launch_reduce(W.part, nb, 1, 0, ent_dev, s));
      } else {
        HIPCHK(sbp::launch_reduce(W.part, nb, 1, 0, W.scal + SC_RED, s));
        for (int ci = 0; ci < ncls; ++ci)
          HIPCHK(sbp::launch_reduce(W.part + M->cls[ci].part_off_h, other_blocks(M->cls[ci]), 1, 0,
                                    W.scal + SC_RED + 1 + ci, s));
        HIPCHK(sbp::launch_reduce(W.scal + SC_RED, 1 + ncls, 1, 0, ent_dev, s));
      }
    }
    return SBP_OK;
  }
  for (auto &c : M->cls) {
    // launch timing: the next free slot (the 2D entropy-split kernel records
    // its own start and end there)
    unsigned long long *ts = nullptr;
    if (M->timing_call && M->t_n < M->t_cap) ts = M->d_tstamp + 2 * (size_t)M->t_n++;
    if (ph.precision == SBP_FP64) {
      sbp::KArgs<double> A = kargs<double>(M, c, u, r, c.op64);
      A.ent_part = W.part + c.part_off;
      A.eform = M->eform;
      A.form_id = ph.form;
      A.tstamp = ts;
      HIPCHK(sbp::launch_residual(M->dim, c.p, ph.form, A, s, c.res_cfg));
    } else {
      sbp::KArgs<float> A = kargs<float>(M, c, u, r, c.op32);
      A.ent_part = W.part + c.part_off;
      A.eform = M->eform;
      A.form_id = ph.form;
      A.tstamp = ts;
      HIPCHK(sbp::launch_residual(M->dim, c.p, ph.form, A, s, c.res_cfg));
    }
    if (hyb && (rc = other_launch(c))) return rc;
  }
  if (ent_dev) {
    const int form_eff = form_eff_of(M);
    for (int ci = 0; ci < ncls; ++ci) {
      auto &c = M->cls[ci];
      const int nb = sbp::residual_blocks(M->dim, c.p, ph.precision, form_eff, c.n_elem, c.res_cfg);
      HIPCHK(sbp::launch_reduce(W.part + c.part_off, nb, 1, 0, W.scal + SC_RED + ci, s));
      if (hyb)
        HIPCHK(sbp::launch_reduce(W.part + c.part_off_h, other_blocks(c), 1, 0, W.scal + SC_RED + ncls + ci, s));
    }
    HIPCHK(sbp::launch_reduce(W.scal + SC_RED, hyb ? 2 * ncls : ncls, 1, 0, ent_dev, s));
  }
  return SBP_OK;
}

// The residual plus the manufactured source when one is set (Sec. 7), at
// time *t0 + c * *dt (the RK stage times; t0 null: the handle's time).  The
// entropy rate then sums w^T H r of both parts.
int residual_impl(sbp_mesh *M, const Work &W, const double *u, void *r, double *ent_dev, hipStream_t s,
                  const double *t0 = nullptr, const double *dt = nullptr, double c = 0.0) {
  // the vortices are exact Euler solutions: no source term
  if (M->src_kind != SBP_SOURCE_NS_MMS) return residual_core(M, W, u, r, ent_dev, s);
  int rc;
  if ((rc = residual_core(M, W, u, r, ent_dev ? W.scal + SC_SRC : nullptr, s))) return rc;
  if (!t0) {
    HIPCHK(sbp::launch_scalar_set(W.scal + SC_TR, M->t, s));
    t0 = W.scal + SC_TR;
    dt = nullptr;
  }
  const int f32 = M->phys.precision == SBP_FP32;
  for (auto &cl : M->cls) {
    sbp::NodeArgs A = node_args(M, cl, u, nullptr);
    HIPCHK(sbp::launch_source_add(A, M->src, r, f32, t0, dt, c, ent_dev ? W.npart + cl.node_off_blk : nullptr, s));
  }
  if (ent_dev) {
    HIPCHK(sbp::launch_reduce(W.npart, M->node_total, 1, 0, W.scal + SC_SRC + 1, s));
    HIPCHK(sbp::launch_reduce(W.scal + SC_SRC, 2, 1, 0, ent_dev, s));
  }
  return SBP_OK;
}

// Sum node-kernel partials of all classes; nv values.  Returns host values.
int reduce_nodes(sbp_mesh *M, int nv, int op, double *host, hipStream_t s) {
  HIPCHK(sbp::launch_reduce(M->d_npart, M->node_total, nv, op, M->d_scal + SC_RED, s));
  HIPCHK(hipMemcpyAsync(host, M->d_scal + SC_RED, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return SBP_OK;
}

int check_err(sbp_mesh *M, hipStream_t s) {
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, M->d_err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h) {
    HIPCHK(hipMemsetAsync(M->d_err, 0, sizeof(int), s));
    HIPCHK(hipStreamSynchronize(s));
    return fail(SBP_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or NaN) seen on the device");
  }
  return SBP_OK;
}

// out = { sum H [s(u + g d) - s(u)], sum H w(u + g d).d, sum H |s(u + g d)| }
int entropy_gap(sbp_mesh *M, const double *u, const double *d, double g, double out[3], hipStream_t s) {
  for (auto &c : M->cls) {
    sbp::NodeArgs A = node_args(M, c, u, d);
    HIPCHK(sbp::launch_entropy_gap(A, g, M->d_npart + c.node_off_blk, s));
  }
  return reduce_nodes(M, 3, 0, out, s);
}

// RK work buffers (stage state, direction, stage residual), allocated on
// first use by sbp_rrk_step or sbp_autotune.
int ensure_rk_buffers(sbp_mesh *M) {
  const size_t n = (size_t)M->n_dof;
  const size_t rsz = M->phys.precision == SBP_FP32 ? sizeof(float) : sizeof(double);
  if (!M->d_y) HIPCHK(hipMalloc((void **)&M->d_y, sizeof(double) * n));
  if (!M->d_d) HIPCHK(hipMalloc((void **)&M->d_d, sizeof(double) * n));
  if (!M->d_r) HIPCHK(hipMalloc(&M->d_r, rsz * n));
  return SBP_OK;
}

// The four RK stages of one step (Sec. 6.1): y_i = u + c_i dt r_{i-1},
// r_i = r(y_i) with its entropy rate, d = dt sum_i b_i r_i; dt is the device
// scalar SC_DT so that the same sequence can be captured once and replayed.
int rk_stages(sbp_mesh *M, const double *u, hipStream_t s) {
  const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  const double cst[4] = {0.0, 0.5, 0.5, 1.0};
  const long long n = M->n_dof;
  const int f32 = M->phys.precision == SBP_FP32;
  const double *dtp = M->d_scal + SC_DT;
  int rc;
  for (int i = 0; i < 4; ++i) {
    const double *y = u;
    if (i > 0) {
      HIPCHK(sbp::launch_axpy(M->d_y, u, M->d_r, f32, cst[i], n, s, dtp));
      y = M->d_y;
    }
    if ((rc = residual_impl(M, handle_work(M), y, M->d_r, M->d_scal + SC_ENT + i, s, M->d_scal + SC_T, dtp, cst[i])))
      return rc;
    if (i == 0)
      HIPCHK(sbp::launch_axpy(M->d_d, nullptr, M->d_r, f32, b[i], n, s, dtp));
    else
      HIPCHK(sbp::launch_accum(M->d_d, M->d_r, f32, b[i], n, s, dtp));
  }
  return SBP_OK;
}

// One relaxation RK4 step on the device (Sec. 6.1): the step size (Sec.
// 7.1; the requested one when positive), the four stages, e, kNewtonSteps
// safeguarded Newton steps for the relaxation root (the steps after the
// root is found do nothing), u += gamma d, and with a report the total
// entropy before and after.  No host round trip: the host reads the
// scalars once afterwards.
constexpr int kNewtonSteps = 8;

int rrk_device(sbp_mesh *M, double *u, bool report, hipStream_t s) {
  double *rk = M->d_scal;
  for (auto &c : M->cls) HIPCHK(sbp::launch_dt(node_args(M, c, u, nullptr), M->d_npart + c.node_off_blk, s, rk));
  HIPCHK(sbp::launch_reduce(M->d_npart, M->node_total, 1, 1, rk + sbp::RK_GAP, s));
  HIPCHK(sbp::launch_rrk_dt(rk + sbp::RK_GAP, rk, s));
  int rc;
  if ((rc = rk_stages(M, u, s))) return rc;
  HIPCHK(sbp::launch_rrk_init(rk, s));
  if (report) {
    for (auto &c : M->cls) HIPCHK(sbp::launch_diagnostics(node_args(M, c, u, nullptr), M->d_npart + c.node_off_blk, s));
    HIPCHK(sbp::launch_reduce(M->d_npart, M->node_total, 1, 0, rk + sbp::RK_S0, s));
  }
  for (int it = 0; it < kNewtonSteps; ++it) {
    for (auto &c : M->cls)
      HIPCHK(sbp::launch_entropy_gap(node_args(M, c, u, M->d_d), 0.0, M->d_npart + c.node_off_blk, s, rk));
    HIPCHK(sbp::launch_reduce(M->d_npart, M->node_total, 3, 0, rk + sbp::RK_GAP, s));
    HIPCHK(sbp::launch_rrk_newton(rk + sbp::RK_GAP, rk, s));
  }
  HIPCHK(sbp::launch_rrk_update(u, M->d_d, rk, M->d_err, M->n_dof, s));
  if (report) {
    for (auto &c : M->cls) HIPCHK(sbp::launch_diagnostics(node_args(M, c, u, nullptr), M->d_npart + c.node_off_blk, s));
    HIPCHK(sbp::launch_reduce(M->d_npart, M->node_total, 1, 0, rk + sbp::RK_S1, s));
  }
  return SBP_OK;
}

// The relaxation root on the host: Newton from g = 1, stopped once |r(g)| is
// at the rounding level of its evaluation (eps sum H |s|) or the step
// stalls; the bracket [0.5, 1.5] is evaluated if a Newton step leaves it
// (then bisection safeguards).  The fallback of the device solve; u is
// read, not changed.  iters receives the number of evaluations.
int relaxation_host(sbp_mesh *M, const double *u, double e, double &g, double &iters, hipStream_t s) {
  constexpr double eps = 2.220446049250313e-16;
  double lo = 0.5, hi = 1.5;
  g = 1.0;
  bool bracketed = false;
  double fv[3];
  int it = 0, rc;
  for (; it < 100; ++it) {
    if ((rc = entropy_gap(M, u, M->d_d, g, fv, s))) return rc;
    const double f = fv[0] - g * e;
    const double df = fv[1] - e;
    if (std::fabs(f) <= eps * fv[2]) break;
    if (bracketed) {
      if (f < 0.0) lo = g; else hi = g;
    }
    double gn = g - f / df;
    if (!(df > 0.0) || !(gn > lo && gn < hi)) {
      if (!bracketed) {
        double fb[3];
        if ((rc = entropy_gap(M, u, M->d_d, lo, fb, s))) return rc;
        const double flo = fb[0] - lo * e;
        if ((rc = entropy_gap(M, u, M->d_d, hi, fb, s))) return rc;
        const double fhi = fb[0] - hi * e;
        if (!(flo < 0.0 && fhi > 0.0)) return fail(SBP_ERRK, "relaxation root not bracketed in [0.5, 1.5]");
        bracketed = true;
        if (f < 0.0) lo = g; else hi = g;
      }
      if (!(df > 0.0) || !(gn > lo && gn < hi)) gn = 0.5 * (lo + hi);
    }
    if (gn == g || std::fabs(gn - g) <= eps * g || (bracketed && hi - lo <= 4.0 * eps * g)) {
      g = gn;
      break;
    }
    g = gn;
  }
  if (it >= 100) return fail(SBP_ERRK, "relaxation root solve did not converge");
  if (!(g > 0.5 && g < 1.5)) return fail(SBP_ERRK, "relaxation parameter outside [0.5, 1.5]");
  iters = it + 1;
  return SBP_OK;
}

void drop_rk_graph(sbp_mesh *M) {
  if (M->rk_exec) (void)hipGraphExecDestroy(M->rk_exec);
  M->rk_exec = nullptr;
  M->rk_u = nullptr;
  M->rk_rep = -1;
}

int rrk_device_graph(sbp_mesh *M, double *u, bool report, hipStream_t s) {
  if (!M->use_graphs) return rrk_device(M, u, report, s);
  if (M->rk_exec && (M->rk_u != (const void *)u || M->rk_rep != (int)report)) drop_rk_graph(M);
  if (!M->rk_exec) {
    if (!M->cap_stream) HIPCHK(hipStreamCreateWithFlags(&M->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(M->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = rrk_device(M, u, report, M->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(M->cap_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    HIPCHK(ec);
    const hipError_t ei = hipGraphInstantiate(&M->rk_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(ei);
    M->rk_u = u;
    M->rk_rep = (int)report;
  }
  HIPCHK(hipGraphLaunch(M->rk_exec, s));
  return SBP_OK;
}

// The first nv of the n_c + 2 diagnostics (total entropy, conserved sums,
// kinetic energy) into out[0..nv).
int diagnostics_impl(sbp_mesh *M, const double *u, double *out, hipStream_t s, int nv) {
  for (auto &c : M->cls) {
    sbp::NodeArgs A = node_args(M, c, u, nullptr);
    HIPCHK(sbp::launch_diagnostics(A, M->d_npart + c.node_off_blk, s));
  }
  return reduce_nodes(M, nv, 0, out, s);
}

// --------------------------------------------------------------------------
// Autotuner.  Every kernel slot of a handle (one degree class of the
// residual or of the VJP, or the batched launch of all classes of a 2D mesh)
// has a launch shape (kernel variant x grid, sbp::LaunchCfg).  sbp_autotune
// times each candidate on the caller's state and keeps the fastest; the
// choice is remembered for the process per workload key, and handles set up
// later with the same key start from it.
enum { TUNE_RES = 0, TUNE_VJP = 1 };

typedef std::array<long long, 9> TuneKey;

std::mutex g_tune_mu;
std::map<TuneKey, sbp::LaunchCfg> g_tune;

TuneKey tune_key(const sbp_mesh *M, int kind, int p, long long n_elem) {
  const sbp_physics &ph = M->phys;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  return {kind, M->dim, p, ph.precision, ph.form, ph.viscous, ph.dissipation, n_elem, dev};
}

bool tune_lookup(const TuneKey &k, sbp::LaunchCfg &cfg) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const auto it = g_tune.find(k);
  if (it == g_tune.end()) return false;
  cfg = it->second;
  return true;
}

void tune_store(const TuneKey &k, const sbp::LaunchCfg &cfg) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[k] = cfg;
}

// launch shapes remembered for this workload (called at the end of setup)
void apply_tuned(sbp_mesh *M) {
  sbp::LaunchCfg cfg;
  if (M->batch_blocks > 0) {
    if (tune_lookup(tune_key(M, TUNE_RES, 0, M->n_elem), cfg)) M->batch_grid = cfg.grid;
    if (tune_lookup(tune_key(M, TUNE_VJP, 0, M->n_elem), cfg)) M->vjp_batch_grid = cfg.grid;
  }
  for (auto &c : M->cls) {
    if (tune_lookup(tune_key(M, TUNE_RES, c.p, c.n_elem), cfg)) c.res_cfg = cfg;
    if (tune_lookup(tune_key(M, TUNE_VJP, c.p, c.n_elem), cfg)) c.vjp_cfg = cfg;
  }
}

// mean time in ms of `reps` launches after two untimed ones; < 0 on error
template <typename F>
double time_launches(F launch, hipStream_t s, int reps) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  double ms = -1.0;
  bool ok = launch() == hipSuccess && launch() == hipSuccess && hipEventRecord(e0, s) == hipSuccess;
  for (int i = 0; ok && i < reps; ++i) ok = launch() == hipSuccess;
  float t = 0.0f;
  if (ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
      hipEventElapsedTime(&t, e0, e1) == hipSuccess)
    ms = (double)t / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

// Try every (variant, grid) of one slot; `run(cfg)` launches it.  Returns
// SBP_OK and fills the report slot, or the launch error.
// Each shape is timed over back-to-back launches (5, then 20 more when one
// launch takes under 0.5 ms, so that short kernels are timed over at least
// about 2 ms); a shape replaces the best so far only when it is faster by
// more than 1% (the built-in shape is timed first), so that timing noise
// does not flip the choice between shapes of equal speed.
template <typename F>
int tune_slot(int nvar, F run, hipStream_t s, sbp::LaunchCfg &best, sbp_tune_slot *out) {
  constexpr int kReps = 5, kMoreReps = 20;
  double best_ms = -1.0, builtin_ms = -1.0;
  int n = 0;
  sbp::LaunchCfg pick = best;
  for (int v = 0; v < nvar; ++v)
    for (int g : sbp::kGridChoices) {
      const sbp::LaunchCfg cfg{v, g};
      double ms = time_launches([&]() { return run(cfg); }, s, kReps);
      if (ms >= 0.0 && ms < 0.5) ms = time_launches([&]() { return run(cfg); }, s, kMoreReps);
      if (ms < 0.0) {
        const hipError_t e = hipGetLastError();
        return fail(SBP_EDEVICE, std::string("autotune launch failed: ") + hipGetErrorString(e));
      }
      ++n;
      if (v == 0 && g == 1) builtin_ms = ms;
      if (best_ms < 0.0 || ms < 0.99 * best_ms) {
        best_ms = ms;
        pick = cfg;
      }
    }
  best = pick;
  if (out) {
    out->variant = pick.variant;
    out->grid = pick.grid;
    out->n_candidates = n;
    out->ms_builtin = builtin_ms;
    out->ms_best = best_ms;
  }
  return SBP_OK;
}

int autotune_impl(sbp_mesh *M, const double *u, const double *lam, sbp_tune_report *rep, hipStream_t s) {
  const sbp_physics &ph = M->phys;
  const int f32 = ph.precision == SBP_FP32;
  const int form_eff = form_eff_of(M);
  sbp_tune_report local{};
  sbp_tune_report &R = rep ? *rep : local;
  R.n_slots = 0;
  int rc;
  // outputs of the timed launches go to the RK work buffers
  if ((rc = ensure_rk_buffers(M))) return rc;
  auto next_slot = [&](int kind, int p) -> sbp_tune_slot * {
    if (R.n_slots >= (int)(sizeof(R.slot) / sizeof(R.slot[0]))) return nullptr;
    sbp_tune_slot *t = &R.slot[R.n_slots++];
    *t = sbp_tune_slot{};
    t->kind = kind;
    t->p = p;
    return t;
  };
  if (ph.viscous)  // the Navier-Stokes kernel reads the facet fluxes of this state
    for (auto &c : M->cls) {
      if (!f32)
        HIPCHK(sbp::launch_visc_q(M->dim, c.p, kargs<double>(M, c, u, M->d_r, c.op64), s));
      else
        HIPCHK(sbp::launch_visc_q(M->dim, c.p, kargs<float>(M, c, u, M->d_r, c.op32), s));
    }
  if (M->batch_blocks > 0 && ph.form == SBP_FORM_SPLIT && !ph.viscous) {
    sbp::KArgs<double> a64[4];
    sbp::KArgs<float> a32[4];
    const sbp::KArgs<double> *p64[4] = {nullptr, nullptr, nullptr, nullptr};
    const sbp::KArgs<float> *p32[4] = {nullptr, nullptr, nullptr, nullptr};
    for (auto &c : M->cls) {
      a64[c.p - 1] = kargs<double>(M, c, u, M->d_r, c.op64);
      a32[c.p - 1] = kargs<float>(M, c, u, M->d_r, c.op32);
      p64[c.p - 1] = &a64[c.p - 1];
      p32[c.p - 1] = &a32[c.p - 1];
    }
    sbp::LaunchCfg cfg{0, M->batch_grid};
    auto run = [&](sbp::LaunchCfg k) {
      return f32 ? sbp::launch_residual2_batch(p32, M->d_bcls32, M->d_part, s, k.grid)
                 : sbp::launch_residual2_batch(p64, M->d_bcls64, M->d_part, s, k.grid);
    };
    if ((rc = tune_slot(1, run, s, cfg, next_slot(TUNE_RES, 0)))) return rc;
    M->batch_grid = cfg.grid;
    tune_store(tune_key(M, TUNE_RES, 0, M->n_elem), cfg);
  } else {
    for (auto &c : M->cls) {
      const sbp::KArgs<double> A64 = kargs<double>(M, c, u, M->d_r, c.op64);
      const sbp::KArgs<float> A32 = kargs<float>(M, c, u, M->d_r, c.op32);
      auto run = [&](sbp::LaunchCfg k) {
        return f32 ? sbp::launch_residual(M->dim, c.p, ph.form, A32, s, k)
                   : sbp::launch_residual(M->dim, c.p, ph.form, A64, s, k);
      };
      if ((rc = tune_slot(sbp::residual_variants(M->dim, c.p, ph.precision, form_eff), run, s, c.res_cfg,
                          next_slot(TUNE_RES, c.p))))
        return rc;
      tune_store(tune_key(M, TUNE_RES, c.p, c.n_elem), c.res_cfg);
    }
  }
  if (lam && !ph.viscous && ph.form == SBP_FORM_SPLIT) {
    auto vargs = [&](DegreeClass &c) {
      sbp::KArgs<double> A = kargs<double>(M, c, u, nullptr, c.op64);
      A.lam = lam;
      A.ubar = M->d_y;
      A.Hn = c.d_Hn;
      return A;
    };
    if (M->dim == 2 && M->cls.size() > 1) {
      sbp::KArgs<double> a[4];
      const sbp::KArgs<double> *pa[4] = {nullptr, nullptr, nullptr, nullptr};
      for (auto &c : M->cls) {
        a[c.p - 1] = vargs(c);
        pa[c.p - 1] = &a[c.p - 1];
      }
      sbp::LaunchCfg cfg{0, M->vjp_batch_grid};
      auto run = [&](sbp::LaunchCfg k) { return sbp::launch_vjp2_batch(pa, M->d_bcls64, s, k.grid); };
      if ((rc = tune_slot(1, run, s, cfg, next_slot(TUNE_VJP, 0)))) return rc;
      M->vjp_batch_grid = cfg.grid;
      tune_store(tune_key(M, TUNE_VJP, 0, M->n_elem), cfg);
    } else {
      for (auto &c : M->cls) {
        const sbp::KArgs<double> A = vargs(c);
        auto run = [&](sbp::LaunchCfg k) { return sbp::launch_vjp(M->dim, c.p, A, s, k); };
        if ((rc = tune_slot(sbp::vjp_variants(M->dim, c.p), run, s, c.vjp_cfg, next_slot(TUNE_VJP, c.p)))) return rc;
        tune_store(tune_key(M, TUNE_VJP, c.p, c.n_elem), c.vjp_cfg);
      }
    }
  }
  // the captured RK stages hold the old launch shapes
  drop_rk_graph(M);
  HIPCHK(hipStreamSynchronize(s));
  return check_err(M, s);
}

// Scratch of sbp_residual_noalloc: a fixed device array that every
// allocation-free residual on a GPU shares (each device holds its own copy
// until the process ends).  In host code `scratch` names a host-side shadow,
// not device memory: only the address hipGetSymbolAddress returns for the
// current device may be handed to kernels.
constexpr size_t kScratchDoubles = (size_t)1 << 17;  // 1 MiB per device
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per device
// (at mesh setup, or at the first allocation-free call on a device).
int vjp_euler(sbp_mesh *M, const void *u, const void *lam, void *ubar, hipStream_t stream);

int scratch_address(double **out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SBP_EDEVICE, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SBP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = (double *)p;
  }
  *out = g_scratch_dev[dev];
  return SBP_OK;
}

}  // namespace

extern "C" {

const char *sbp_last_error(void) { return g_err.c_str(); }

int sbp_setup_mesh(const sbp_mesh_desc *desc, const sbp_physics *phys, void *hip_stream, sbp_mesh **out) {
  if (!desc || !phys || !out) return fail(SBP_EINVAL, "null argument");
  *out = nullptr;
  if (desc->dim != 2 && desc->dim != 3) return fail(SBP_EINVAL, "dim must be 2 or 3");
  if (desc->n_elem <= 0 || desc->n_vert <= 0 || !desc->vert_xyz || !desc->elem_vert || !desc->period ||
      !desc->elem_degree)
    return fail(SBP_EINVAL, "incomplete mesh description");
  if (desc->p_geom != 1 && !(desc->p_geom == 2 && desc->geom_nodes))
    return fail(SBP_ENOTSUP, "p_geom must be 1, or 2 with geom_nodes");
  if (desc->dim == 3 && desc->p_geom == 2) {
    // Assumption 1: a quadratic map in 3D needs p >= 2 (p_geom <= floor(p/2) + 1)
    for (int e = 0; e < desc->n_elem; ++e)
      if (desc->elem_degree[e] < 2)
        return fail(SBP_EINVAL, "quadratic tetrahedral maps need degree p >= 2 (Assumption 1)");
  }
  if (desc->n_problems < 1) return fail(SBP_EINVAL, "n_problems must be >= 1");
  for (int i = 0; i < desc->dim; ++i)
    if (!(desc->period[i] > 0)) return fail(SBP_EINVAL, "period must be positive");
  if (!(phys->gamma > 1.0) || !(phys->beta > 0.0)) return fail(SBP_EINVAL, "need gamma > 1 and beta > 0");
  if (phys->form != SBP_FORM_SPLIT && phys->form != SBP_FORM_HADAMARD) return fail(SBP_EINVAL, "bad form");
  if (phys->precision != SBP_FP64 && phys->precision != SBP_FP32) return fail(SBP_EINVAL, "bad precision");
  if (phys->viscous && phys->form != SBP_FORM_SPLIT)
    return fail(SBP_ENOTSUP, "viscous terms are available for the entropy-split form");
  if (phys->viscous && !(phys->mu >= 0.0 && phys->Pr > 0.0 && phys->R > 0.0))
    return fail(SBP_EINVAL, "viscous terms need mu >= 0, Pr > 0, R > 0");
  sbp_mesh *M = new (std::nothrow) sbp_mesh();
  if (!M) return fail(SBP_ENOMEM, "host allocation failed");
  int rc;
  try {
    rc = setup_impl(desc, phys, (hipStream_t)hip_stream, M);
  } catch (const std::exception &ex) {
    rc = fail(SBP_EINVAL, std::string("setup: ") + ex.what());
  }
  if (rc != SBP_OK) {
    sbp_destroy_mesh(M);
    return rc;
  }
  for (int i = 0; i < desc->dim; ++i) M->period[i] = desc->period[i];
  double *scr = nullptr;  // the allocation-free residual's scratch on this device
  if ((rc = scratch_address(&scr))) {
    sbp_destroy_mesh(M);
    return rc;
  }
  *out = M;
  return SBP_OK;
}

int sbp_mesh_info(sbp_mesh *M, sbp_info *out) {
  if (!M || !out) return fail(SBP_EINVAL, "null argument");
  out->dim = M->dim;
  out->n_c = M->nc;
  out->n_elem = M->n_elem;
  out->n_nodes = M->n_nodes;
  out->node_off = M->node_off.data();
  out->elem_np = M->elem_np.data();
  out->node_xyz = M->d_node_xyz;
  out->node_h = M->d_node_h;
  out->t = M->t;
  return check_err(M, nullptr);
}

int sbp_residual(sbp_mesh *M, const void *u, void *r, double *ent_dev, void *stream) {
  if (!M || !u || !r) return fail(SBP_EINVAL, "null argument");
  M->timing_call = M->t_cap > 0;
  const int rc = residual_impl(M, handle_work(M), (const double *)u, r, ent_dev, (hipStream_t)stream);
  M->timing_call = false;
  return rc;
}

namespace {
// slots of the launch timing back to {no start yet, no end yet}
int reset_tstamp(sbp_mesh *M) {
  if (M->t_cap <= 0) return SBP_OK;
  std::vector<unsigned long long> init(2 * (size_t)M->t_cap);
  for (size_t i = 0; i < init.size(); i += 2) {
    init[i] = ~0ull;
    init[i + 1] = 0ull;
  }
  HIPCHK(hipMemcpy(M->d_tstamp, init.data(), init.size() * sizeof(unsigned long long), hipMemcpyHostToDevice));
  M->t_n = 0;
  return SBP_OK;
}
}  // namespace

int sbp_time_launches(sbp_mesh *M, int capacity) {
  if (!M || capacity < 0 || capacity > 65536) return fail(SBP_EINVAL, "null handle or capacity outside 0..65536");
  const sbp_physics &ph = M->phys;
  if (capacity > 0 && (M->dim != 2 || ph.form != SBP_FORM_SPLIT || ph.viscous))
    return fail(SBP_ENOTSUP, "launch timing covers the entropy-split kernels of triangle meshes (Euler terms)");
  HIPCHK(hipDeviceSynchronize());
  (void)hipFree(M->d_tstamp);
  M->d_tstamp = nullptr;
  M->t_cap = M->t_n = 0;
  if (capacity == 0) return SBP_OK;
  HIPCHK(hipMalloc((void **)&M->d_tstamp, sizeof(unsigned long long) * 2 * (size_t)capacity));
  M->t_cap = capacity;
  return reset_tstamp(M);
}

int sbp_launch_times(sbp_mesh *M, double *ms_out, int max, int *n_out) {
  if (!M || !n_out || (max > 0 && !ms_out)) return fail(SBP_EINVAL, "null argument");
  *n_out = 0;
  if (M->t_cap <= 0) return SBP_OK;
  HIPCHK(hipDeviceSynchronize());
  const int n = std::min(M->t_n, std::max(0, max));
  std::vector<unsigned long long> ts(2 * (size_t)std::max(1, M->t_n));
  if (M->t_n > 0)
    HIPCHK(hipMemcpy(ts.data(), M->d_tstamp, sizeof(unsigned long long) * 2 * (size_t)M->t_n, hipMemcpyDeviceToHost));
  int dev = 0, khz = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) return fail(SBP_EDEVICE, "device clock rate unknown");
  for (int i = 0; i < n; ++i)
    ms_out[i] = ts[2 * i + 1] >= ts[2 * i] ? (double)(ts[2 * i + 1] - ts[2 * i]) / (double)khz : -1.0;
  *n_out = n;
  return reset_tstamp(M);
}

int sbp_residual_noalloc(sbp_mesh *M, const void *u, void *r, double *ent_dev, void *stream) {
  if (!M || !u || !r) return fail(SBP_EINVAL, "null argument");
  const size_t need = work_doubles(M);
  if (need > kScratchDoubles)
    return fail(SBP_EINVAL, "sbp_residual_noalloc: the mesh needs " + std::to_string(need) +
                                " scratch doubles, more than the " + std::to_string(kScratchDoubles) +
                                " of the static scratch array; use sbp_residual");
  double *scr = nullptr;
  int rc;
  if ((rc = scratch_address(&scr))) return rc;
  // layout: [part_total partials | SC_TOTAL scalars | node partials (source only)]
  const size_t np = (size_t)std::max(1, M->part_total);
  const Work W{scr, scr + np, scr + np + SC_TOTAL};
  return residual_impl(M, W, (const double *)u, r, ent_dev, (hipStream_t)stream);
}

int sbp_residual_vjp(sbp_mesh *M, const void *u, const void *lam, void *ubar, void *stream) {
  if (!M || !u || !lam || !ubar) return fail(SBP_EINVAL, "null argument");
  const sbp_physics &ph = M->phys;
  int rc = vjp_euler(M, u, lam, ubar, (hipStream_t)stream);
  if (rc || !ph.viscous) return rc;
  // the Navier-Stokes terms add their VJP to the Euler terms'
  for (auto &c : M->cls) {
    sbp::KArgs<double> A = kargs<double>(M, c, (const double *)u, nullptr, c.op64);
    A.lam = (const double *)lam;
    A.ubar = (double *)ubar;
    A.Hn = c.d_Hn;
    HIPCHK(sbp::launch_vjp_viscous(M->dim, c.p, A, c.d_vq, (hipStream_t)stream));
  }
  return SBP_OK;
}

}  // extern "C"

namespace {

// ubar = (dr/du)^T lambda of the Euler terms (both volume forms, hybrid flags,
// dissipation).
int vjp_euler(sbp_mesh *M, const void *u, const void *lam, void *ubar, hipStream_t stream) {
  const sbp_physics &ph = M->phys;
  if (M->eform || ph.form == SBP_FORM_HADAMARD) {
    // Hadamard form, or the hybrid scheme: each form's kernel takes the
    // elements flagged with it (both kernels for every class)
    const hipStream_t s = (hipStream_t)stream;
    for (auto &c : M->cls) {
      sbp::KArgs<double> A = kargs<double>(M, c, (const double *)u, nullptr, c.op64);
      A.lam = (const double *)lam;
      A.ubar = (double *)ubar;
      A.Hn = c.d_Hn;
      A.eform = M->eform;
      for (int form : {SBP_FORM_SPLIT, SBP_FORM_HADAMARD}) {
        if (!M->eform && form != ph.form) continue;
        A.form_id = form;
        if (form == SBP_FORM_HADAMARD)
          HIPCHK(sbp::launch_vjp_hadamard(M->dim, c.p, A, s));
        else
          HIPCHK(sbp::launch_vjp(M->dim, c.p, A, s, c.vjp_cfg));
      }
    }
    return SBP_OK;
  }
  if (M->dim == 2 && M->cls.size() > 1) {
    // every degree class in one persistent launch
    sbp::KArgs<double> a[4];
    const sbp::KArgs<double> *pa[4] = {nullptr, nullptr, nullptr, nullptr};
    for (auto &c : M->cls) {
      sbp::KArgs<double> &A = a[c.p - 1];
      A = kargs<double>(M, c, (const double *)u, nullptr, c.op64);
      A.lam = (const double *)lam;
      A.ubar = (double *)ubar;
      A.Hn = c.d_Hn;
      pa[c.p - 1] = &A;
    }
    HIPCHK(sbp::launch_vjp2_batch(pa, M->d_bcls64, (hipStream_t)stream, M->vjp_batch_grid));
    return SBP_OK;
  }
  for (auto &c : M->cls) {
    sbp::KArgs<double> A = kargs<double>(M, c, (const double *)u, nullptr, c.op64);
    A.lam = (const double *)lam;
    A.ubar = (double *)ubar;
    A.Hn = c.d_Hn;
    HIPCHK(sbp::launch_vjp(M->dim, c.p, A, (hipStream_t)stream, c.vjp_cfg));
  }
  return SBP_OK;
}

}  // namespace

extern "C" {

int sbp_diagnostics(sbp_mesh *M, const void *u, double *out_host, void *stream) {
  if (!M || !u || !out_host) return fail(SBP_EINVAL, "null argument");
  return diagnostics_impl(M, (const double *)u, out_host, (hipStream_t)stream, M->nc + 2);
}

int sbp_check_device(sbp_mesh *M, void *stream) {
  if (!M) return fail(SBP_EINVAL, "null argument");
  return check_err(M, (hipStream_t)stream);
}

int sbp_use_graphs(sbp_mesh *M, int enable) {
  if (!M) return fail(SBP_EINVAL, "null argument");
  M->use_graphs = enable ? 1 : 0;
  if (!M->use_graphs) drop_rk_graph(M);
  return SBP_OK;
}

int sbp_autotune(sbp_mesh *M, const void *u, const void *lam, sbp_tune_report *rep, void *stream) {
  if (!M || !u) return fail(SBP_EINVAL, "null argument");
  return autotune_impl(M, (const double *)u, (const double *)lam, rep, (hipStream_t)stream);
}

namespace {

// the slot (kind, p) of the handle: its config, or nullptr; grid-only slots
// (batched launches) report nvar = 1
sbp::LaunchCfg *find_slot(sbp_mesh *M, int kind, int p, int &nvar, int *&grid_only) {
  grid_only = nullptr;
  const sbp_physics &ph = M->phys;
  const int form_eff = form_eff_of(M);
  if (kind == TUNE_VJP && (ph.viscous || ph.form != SBP_FORM_SPLIT)) return nullptr;
  const bool batched = kind == TUNE_RES ? (M->batch_blocks > 0 && ph.form == SBP_FORM_SPLIT && !ph.viscous)
                                        : (M->dim == 2 && M->cls.size() > 1);
  if (batched) {
    if (p != 0) return nullptr;
    nvar = 1;
    grid_only = kind == TUNE_RES ? &M->batch_grid : &M->vjp_batch_grid;
    return nullptr;
  }
  for (auto &c : M->cls)
    if (c.p == p) {
      nvar = kind == TUNE_RES ? sbp::residual_variants(M->dim, p, ph.precision, form_eff) : sbp::vjp_variants(M->dim, p);
      return kind == TUNE_RES ? &c.res_cfg : &c.vjp_cfg;
    }
  return nullptr;
}

}  // namespace

int sbp_set_volume_form(sbp_mesh *M, const uint8_t *form_dev) {
  if (!M) return fail(SBP_EINVAL, "null handle");
  if (form_dev && M->phys.viscous)
    return fail(SBP_ENOTSUP, "the hybrid scheme covers the Euler terms (no viscous terms)");
  M->eform = form_dev;
  // the captured RK stages hold the previous launches
  drop_rk_graph(M);
  return SBP_OK;
}

int sbp_set_source(sbp_mesh *M, int32_t kind, const double *params) {
  if (!M) return fail(SBP_EINVAL, "null handle");
  if (kind != SBP_SOURCE_NONE && kind != SBP_SOURCE_NS_MMS && kind != SBP_SOURCE_VORTEX3D &&
      kind != SBP_SOURCE_VORTEX2D)
    return fail(SBP_EINVAL, "unknown source kind");
  if (kind == SBP_SOURCE_VORTEX3D && M->dim != 3) return fail(SBP_EINVAL, "the 3D vortex needs a 3D mesh");
  if (kind == SBP_SOURCE_VORTEX2D) {
    if (M->dim != 2) return fail(SBP_EINVAL, "the 2D vortex needs a 2D mesh");
    const double def[3] = {3.0, 5.0, 0.0};
    const double *q = params ? params : def;
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(q[k])) return fail(SBP_EINVAL, "vortex parameters must be finite");
    // T > 0 at the centre: alpha^2 (gamma-1) e^2 / (16 gamma pi^2) < 1
    const double g = M->phys.gamma, e = std::exp(1.0);
    if (!(q[0] * q[0] * (g - 1.0) * e * e / (16.0 * g * M_PI * M_PI) < 1.0))
      return fail(SBP_EINVAL, "vortex too strong (negative temperature at its centre)");
    M->src.alpha = q[0];
    M->src.xc = q[1];
    M->src.yc = q[2];
    M->src.px = M->period[0];
    M->src.py = M->period[1];
  }
  if (kind == SBP_SOURCE_NS_MMS) {
    const double def[4] = {2.0, 0.1, 0.6, 1.0};
    const double *q = params ? params : def;
    for (int k = 0; k < 4; ++k)
      if (!std::isfinite(q[k])) return fail(SBP_EINVAL, "source parameters must be finite");
    if (!(q[0] - std::fabs(q[1]) > 0.0)) return fail(SBP_EINVAL, "need rho0 > |a|");
    const double g = M->phys.gamma;
    if (!(q[0] - std::fabs(q[1]) > 0.5 * M->dim * q[3] * q[3])) return fail(SBP_EINVAL, "need rho0 - |a| > d V0^2 / 2 (p > 0)");
    for (int i = 0; i < M->dim; ++i) {
      const double k = M->period[i] / 2.0;
      if (!(std::fabs(k - std::round(k)) <= 1e-12 * k) || k < 0.5)
        return fail(SBP_EINVAL, "the manufactured fields have period 2: box sides must be multiples of 2");
    }
    M->src.rho0 = q[0];
    M->src.a = q[1];
    M->src.c = q[2];
    M->src.V0 = q[3];
    const sbp_physics &ph = M->phys;
    // kappa (gamma-1)/R with kappa = mu c_p / Pr, c_p = gamma R / (gamma-1)
    M->src.heat = (ph.viscous && ph.heat_flux) ? ph.mu * g / ph.Pr : 0.0;
  }
  M->src.kind = kind;
  M->src_kind = kind;
  // the captured RK stages hold the previous launches
  drop_rk_graph(M);
  return SBP_OK;
}

int sbp_source_state(sbp_mesh *M, double t, void *u_dev, void *stream) {
  if (!M || !u_dev) return fail(SBP_EINVAL, "null argument");
  if (!M->src_kind) return fail(SBP_EINVAL, "no source set");
  for (auto &c : M->cls) {
    sbp::NodeArgs A = node_args(M, c, nullptr, nullptr);
    HIPCHK(sbp::launch_source_state(A, M->src, t, (double *)u_dev, (hipStream_t)stream));
  }
  return SBP_OK;
}

// Device table of the error rule of class c: I [nq][np], w [nq] and, in 2D,
// the quadratic map's basis and derivatives at the points.
int ensure_error_rule(sbp_mesh *M, DegreeClass &c, hipStream_t s) {
  if (c.d_eq) return SBP_OK;
  const sbp::ErrRule &R = sbp::error_rule(M->dim, c.p);
  std::vector<double> tab(R.I);
  tab.insert(tab.end(), R.w.begin(), R.w.end());
  if (M->dim == 2) {
    std::vector<double> N((size_t)R.nq * 6), dN((size_t)2 * R.nq * 6);
    for (int q = 0; q < R.nq; ++q) {
      double n[6], d[2][6];
      p2_basis(R.xi[2 * q], R.xi[2 * q + 1], n);
      p2_dbasis(R.xi[2 * q], R.xi[2 * q + 1], d);
      for (int a = 0; a < 6; ++a) {
        N[(size_t)q * 6 + a] = n[a];
        dN[(size_t)q * 6 + a] = d[0][a];
        dN[(size_t)(R.nq + q) * 6 + a] = d[1][a];
      }
    }
    tab.insert(tab.end(), N.begin(), N.end());
    tab.insert(tab.end(), dN.begin(), dN.end());
  } else if (M->curved3) {
    std::vector<double> N((size_t)R.nq * 10), dN((size_t)3 * R.nq * 10);
    for (int q = 0; q < R.nq; ++q) {
      double n[10], d[3][10];
      p2t_basis(&R.xi[(size_t)3 * q], n, d);
      for (int a = 0; a < 10; ++a) {
        N[(size_t)q * 10 + a] = n[a];
        for (int l = 0; l < 3; ++l) dN[((size_t)l * R.nq + q) * 10 + a] = d[l][a];
      }
    }
    tab.insert(tab.end(), N.begin(), N.end());
    tab.insert(tab.end(), dN.begin(), dN.end());
  }
  int rc;
  if ((rc = upload(c.d_eq, tab, s))) return rc;
  HIPCHK(hipStreamSynchronize(s));  // tab is freed on return
  c.eq_nq = R.nq;
  return SBP_OK;
}

int sbp_source_error(sbp_mesh *M, const void *u_dev, double t, int32_t norm, double *out_host, void *stream) {
  if (!M || !u_dev || !out_host) return fail(SBP_EINVAL, "null argument");
  if (!M->src_kind) return fail(SBP_EINVAL, "no source set");
  if (norm != SBP_NORM_NODAL && norm != SBP_NORM_QUADRATURE) return fail(SBP_EINVAL, "unknown norm");
  hipStream_t s = (hipStream_t)stream;
  for (auto &c : M->cls) {
    sbp::NodeArgs A = node_args(M, c, (const double *)u_dev, nullptr);
    if (norm == SBP_NORM_NODAL) {
      HIPCHK(sbp::launch_source_error(A, M->src, t, M->d_npart + c.node_off_blk, s));
    } else {
      int rc;
      if ((rc = ensure_error_rule(M, c, s))) return rc;
      HIPCHK(sbp::launch_source_error_quad(A, M->src, t, c.d_eq, c.eq_nq, c.d_geo, M->curved3,
                                           M->d_npart + c.node_off_blk, s));
    }
  }
  return reduce_nodes(M, M->nc, 0, out_host, s);
}

int sbp_get_launch_shape(sbp_mesh *M, int32_t kind, int32_t p, int32_t *variant, int32_t *grid) {
  if (!M || (kind != 0 && kind != 1)) return fail(SBP_EINVAL, "bad handle or kind");
  int nvar = 0, *g = nullptr;
  sbp::LaunchCfg *c = find_slot(M, kind, p, nvar, g);
  if (!c && !g) return fail(SBP_EINVAL, "no such kernel slot");
  if (variant) *variant = c ? c->variant : 0;
  if (grid) *grid = c ? c->grid : *g;
  return SBP_OK;
}

int sbp_set_launch_shape(sbp_mesh *M, int32_t kind, int32_t p, int32_t variant, int32_t grid) {
  if (!M || (kind != 0 && kind != 1)) return fail(SBP_EINVAL, "bad handle or kind");
  int nvar = 0, *g = nullptr;
  sbp::LaunchCfg *c = find_slot(M, kind, p, nvar, g);
  if (!c && !g) return fail(SBP_EINVAL, "no such kernel slot");
  if (variant < 0 || variant >= nvar) return fail(SBP_EINVAL, "variant out of range");
  if (grid < 0 || grid > 64) return fail(SBP_EINVAL, "grid must be 0..64");
  if (c) *c = sbp::LaunchCfg{variant, grid};
  else *g = grid;
  drop_rk_graph(M);
  return SBP_OK;
}

int sbp_set_time(sbp_mesh *M, double t) {
  if (!M) return fail(SBP_EINVAL, "null argument");
  M->t = t;
  return SBP_OK;
}

int sbp_rrk_step(sbp_mesh *M, void *u_dev, double dt, double cfl, sbp_rrk_report *rep, void *stream) {
  if (!M || !u_dev) return fail(SBP_EINVAL, "null argument");
  if (!(dt > 0.0) && !(cfl > 0.0)) return fail(SBP_EINVAL, "need dt > 0 or cfl > 0");
  hipStream_t s = (hipStream_t)stream;
  double *u = (double *)u_dev;
  int rc;
  if ((rc = ensure_rk_buffers(M))) return rc;
  // the whole step on the device (one captured graph), then one read-back
  HIPCHK(sbp::launch_scalar_set(M->d_scal + sbp::RK_DTIN, dt > 0.0 ? dt : 0.0, s));
  HIPCHK(sbp::launch_scalar_set(M->d_scal + sbp::RK_CFL, cfl, s));
  HIPCHK(sbp::launch_scalar_set(M->d_scal + SC_T, M->t, s));
  if ((rc = rrk_device_graph(M, u, rep != nullptr, s))) return rc;
  double k[sbp::RK_TOTAL];
  HIPCHK(hipMemcpyAsync(k, M->d_scal, sizeof(k), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if ((rc = check_err(M, s))) return rc;
  if (k[sbp::RK_BAD] != 0.0) return fail(SBP_ENONPHYS, "time step is not positive (non-physical state)");
  dt = k[sbp::RK_DT];
  const double e = k[sbp::RK_E];
  double g = k[sbp::RK_G];
  const double done = k[sbp::RK_DONE];
  int iters = (int)k[sbp::RK_IT];
  double ent0 = k[sbp::RK_S0], ent1 = k[sbp::RK_S1];
  if (!((done == 1.0 || done == 2.0) && g > 0.5 && g < 1.5)) {
    // the device steps did not settle inside the bracket: the host solve
    // (Newton with bisection on an evaluated bracket), u still unchanged
    double extra = 0;
    if ((rc = relaxation_host(M, u, e, g, extra, s))) return rc;
    iters += (int)extra;
    if (rep && (rc = diagnostics_impl(M, u, &ent0, s, 1))) return rc;
    HIPCHK(sbp::launch_accum(u, M->d_d, 0, g, M->n_dof, s));
    if (rep && (rc = diagnostics_impl(M, u, &ent1, s, 1))) return rc;
  }
  M->t += g * dt;
  if (rep) {
    rep->gamma_n = g;
    rep->dt = dt;
    rep->t = M->t;
    rep->entropy_before = ent0;
    rep->entropy_after = ent1;
    rep->entropy_rate_e = e;
    rep->newton_iters = iters;
  }
  HIPCHK(hipStreamSynchronize(s));
  return check_err(M, s);
}

int sbp_destroy_mesh(sbp_mesh *M) {
  if (!M) return SBP_OK;
  (void)hipFree(M->d_tstamp);
  for (auto &c : M->cls) {
    (void)hipFree(c.d_uoff);
    (void)hipFree(c.d_gid);
    (void)hipFree(c.d_geo);
    (void)hipFree(c.d_eq);
    (void)hipFree(c.d_nbr);
    (void)hipFree(c.d_Hn);
    (void)hipFree(c.d_hmin);
    (void)hipFree(c.d_ops);
    (void)hipFree(c.d_nbrq);
    (void)hipFree(c.d_q);
    (void)hipFree(c.d_vq);
  }
  (void)hipFree(M->d_node_xyz);
  (void)hipFree(M->d_node_h);
  (void)hipFree(M->d_part);
  (void)hipFree(M->d_npart);
  (void)hipFree(M->d_scal);
  (void)hipFree(M->d_eac);
  (void)hipFree(M->d_bcls64);
  (void)hipFree(M->d_bcls32);
  (void)hipFree(M->d_err);
  (void)hipFree(M->d_y);
  (void)hipFree(M->d_d);
  (void)hipFree(M->d_r);
  if (M->rk_exec) (void)hipGraphExecDestroy(M->rk_exec);
  if (M->cap_stream) (void)hipStreamDestroy(M->cap_stream);
  delete M;
  return SBP_OK;
}

int sbp_reference_operator(int32_t dim, int32_t p, int32_t *n_p, int32_t *n_f, double *nodes, double *h,
                           double *Q, double *E, int32_t *facet_nodes, double *facet_w) {
  try {
    const sbp::RefOp &op = sbp::reference_operator(dim, p);
    if (n_p) *n_p = op.np;
    if (n_f) *n_f = op.nf;
    if (nodes) std::memcpy(nodes, op.nodes.data(), op.nodes.size() * sizeof(double));
    if (h) std::memcpy(h, op.h.data(), op.h.size() * sizeof(double));
    if (Q) std::memcpy(Q, op.Q.data(), op.Q.size() * sizeof(double));
    if (E) std::memcpy(E, op.E.data(), op.E.size() * sizeof(double));
    if (facet_nodes)
      for (size_t k = 0; k < op.facet_nodes.size(); ++k) facet_nodes[k] = op.facet_nodes[k];
    if (facet_w) std::memcpy(facet_w, op.facet_w.data(), op.facet_w.size() * sizeof(double));
  } catch (const std::invalid_argument &ex) {
    return fail(SBP_ENOTSUP, ex.what());
  } catch (const std::exception &ex) {
    return fail(SBP_EINVAL, ex.what());
  }
  return SBP_OK;
}

}  // extern "C"
