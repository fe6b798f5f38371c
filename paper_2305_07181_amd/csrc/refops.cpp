// Reference-element diagonal-E SBP operators (host side of sbp_setup_mesh).
//
// Def. 1 and Sec. 2.1 of the paper fix the requirements: D = H^{-1} Q exact
// on P^p, H a positive quadrature of degree >= 2p-1, Q = S + E/2 with S skew,
// E = sum_f R_f^T B_f N_f R_f diagonal (facet nodes collocated with volume
// nodes, facet quadrature of degree >= 2p with positive weights).
//
// Node sets (shared with the test oracle by convention, solved independently):
//   triangle: (p+1)-point Gauss-Legendre nodes on each edge (ascending along
//     edge f from vertex (f+1)%3 to (f+2)%3) + interior orbits
//       p=1 none | p=2 centroid | p=3 6-orbit | p=4 centroid, two 3-orbits
//   tetrahedron: a symmetric degree-2p triangle rule on each face (face f
//     opposite vertex f, face vertices ascending) + interior orbits
//       p=1 none | p=2 centroid | p=3 one 12-orbit (a,a,b,1-2a-b)
// Facet nodes come first (facet by facet), interior nodes last; each orbit
// lists its distinct permutations in ascending lexicographic order.
//
// Construction here: orbit parameters and weights by Gauss-Newton on the
// moment equations (complex-step Jacobian), S as the minimum-norm skew
// solution of S V = H V_l - E_l V / 2 in closed form from a Householder QR of
// the Vandermonde matrix: with V = QR and B = A R^{-1},
//   S = B Q^T - Q B^T - Q (Q^T B) Q^T.
#include "refops.hpp"

#include <algorithm>
#include <complex>
#include <map>
#include <mutex>
#include <stdexcept>

#include "dense.hpp"

namespace sbp {
namespace {

using LD = long double;
using cplx = std::complex<LD>;

double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// Monomial exponents of total degree <= deg in `dim` variables, in the order
// (a, b[, c]) nested loops.
std::vector<std::vector<int>> monomials(int deg, int dim) {
  std::vector<std::vector<int>> out;
  if (dim == 2) {
    for (int a = 0; a <= deg; ++a)
      for (int b = 0; b <= deg - a; ++b) out.push_back({a, b});
  } else {
    for (int a = 0; a <= deg; ++a)
      for (int b = 0; b <= deg - a; ++b)
        for (int c = 0; c <= deg - a - b; ++c) out.push_back({a, b, c});
  }
  return out;
}

LD simplex_moment(const std::vector<int> &e) {
  int s = 0;
  LD num = 1.0L;
  for (int k : e) { s += k; num *= (LD)factorial(k); }
  return num / (LD)factorial(s + (int)e.size());
}

// Orbit description: symbol ids of the base barycentric tuple and how the
// symbol values follow from the orbit parameters.
struct Orbit {
  char kind;                 // '1', '3', '6', 'T' (12-orbit)
  std::vector<double> guess;
};

int orbit_npar(char k) { return k == '1' ? 0 : (k == '3' ? 1 : 2); }

// Symbol values of the base tuple (complex for the complex-step Jacobian).
std::vector<cplx> orbit_symbols(char kind, const cplx *x, int nb) {
  switch (kind) {
    case '1': return {cplx(1.0L / nb)};
    case '3': return {x[0], (LD)1 - (LD)2 * x[0]};
    case '6': return {x[0], x[1], (LD)1 - x[0] - x[1]};
    case 'T': return {x[0], x[1], (LD)1 - (LD)2 * x[0] - x[1]};
  }
  throw std::runtime_error("orbit kind");
}

std::vector<int> orbit_pattern(char kind, int nb) {
  switch (kind) {
    case '1': return std::vector<int>(nb, 0);
    case '3': return {0, 0, 1};
    case '6': return {0, 1, 2};
    case 'T': return {0, 0, 1, 2};
  }
  throw std::runtime_error("orbit kind");
}

// Distinct permutations of the symbol pattern -> points (complex barycentric).
std::vector<std::vector<cplx>> orbit_points(char kind, const cplx *x, int nb) {
  auto sym = orbit_symbols(kind, x, nb);
  auto pat = orbit_pattern(kind, nb);
  std::sort(pat.begin(), pat.end());
  std::vector<std::vector<cplx>> pts;
  do {
    std::vector<cplx> q(nb);
    for (int i = 0; i < nb; ++i) q[i] = sym[pat[i]];
    pts.push_back(q);
  } while (std::next_permutation(pat.begin(), pat.end()));
  // ascending lexicographic order of the (real) barycentric tuples
  std::sort(pts.begin(), pts.end(), [](const std::vector<cplx> &a, const std::vector<cplx> &b) {
    for (size_t i = 0; i < a.size(); ++i) {
      if (a[i].real() < b[i].real()) return true;
      if (a[i].real() > b[i].real()) return false;
    }
    return false;
  });
  return pts;
}

// Orbit points in double arithmetic from double parameters.
std::vector<std::vector<double>> orbit_points_d(char kind, const double *x, int nb) {
  std::vector<double> sym;
  switch (kind) {
    case '1': sym = {1.0 / nb}; break;
    case '3': sym = {x[0], 1.0 - 2.0 * x[0]}; break;
    case '6': sym = {x[0], x[1], 1.0 - x[0] - x[1]}; break;
    case 'T': sym = {x[0], x[1], 1.0 - 2.0 * x[0] - x[1]}; break;
    default: throw std::runtime_error("orbit kind");
  }
  auto pat = orbit_pattern(kind, nb);
  std::sort(pat.begin(), pat.end());
  std::vector<std::vector<double>> pts;
  do {
    std::vector<double> q(nb);
    for (int i = 0; i < nb; ++i) q[i] = sym[pat[i]];
    pts.push_back(q);
  } while (std::next_permutation(pat.begin(), pat.end()));
  std::sort(pts.begin(), pts.end());
  return pts;
}

// A quadrature rule being solved: fixed point groups (known points, unknown
// common weight) followed by orbits (unknown parameters and weight).
struct RuleProblem {
  int sdim;  // simplex dimension (2: triangle, 3: tetrahedron)
  int deg;
  std::vector<std::vector<std::vector<double>>> fixed_groups;  // [g][pt][nb]
  std::vector<Orbit> orbits;
};

struct RuleSolution {
  std::vector<std::vector<double>> pts;  // barycentric, group order
  std::vector<double> w;                 // per point
  std::vector<double> params;
  double residual;
};

// Moment residual R_q = sum_g w_g sum_{pt in g} mono_q(pt) - mom_q as a
// function of the orbit parameters and group weights, solved by Gauss-Newton
// in 80-bit extended precision (complex-step Jacobian) so that the parameters
// round to the nearest doubles; the points are then formed in double
// arithmetic and the weights re-solved (extended precision) for those points.
RuleSolution solve_rule(const RuleProblem &P) {
  const int nb = P.sdim + 1;
  auto mons = monomials(P.deg, P.sdim);
  const int nq = (int)mons.size();
  std::vector<LD> mom(nq);
  for (int q = 0; q < nq; ++q) mom[q] = simplex_moment(mons[q]);
  int npar = 0;
  for (auto &o : P.orbits) npar += orbit_npar(o.kind);
  const int ng = (int)P.fixed_groups.size() + (int)P.orbits.size();
  std::vector<LD> x;
  for (auto &o : P.orbits)
    for (double g : o.guess) x.push_back((LD)g);

  auto mono_val = [&](const std::vector<cplx> &pt, int q) {
    cplx v = 1.0L;
    for (int i = 0; i < P.sdim; ++i)
      for (int k = 0; k < mons[q][i]; ++k) v *= pt[1 + i];
    return v;
  };
  // group sums of monomials with complex parameters
  auto group_sums = [&](const std::vector<cplx> &xc) {
    std::vector<std::vector<cplx>> G(nq, std::vector<cplx>(ng, 0.0L));
    int g = 0;
    for (auto &fg : P.fixed_groups) {
      for (auto &pt : fg) {
        std::vector<cplx> pc(pt.begin(), pt.end());
        for (int q = 0; q < nq; ++q) G[q][g] += mono_val(pc, q);
      }
      ++g;
    }
    int k = 0;
    for (auto &o : P.orbits) {
      for (auto &pt : orbit_points(o.kind, xc.data() + k, nb))
        for (int q = 0; q < nq; ++q) G[q][g] += mono_val(pt, q);
      k += orbit_npar(o.kind);
      ++g;
    }
    return G;
  };
  auto real_G = [&](const std::vector<LD> &xr) {
    std::vector<cplx> xc(xr.begin(), xr.end());
    auto G = group_sums(xc);
    MatT<LD> M(nq, ng);
    for (int q = 0; q < nq; ++q)
      for (int gi = 0; gi < ng; ++gi) M(q, gi) = G[q][gi].real();
    return M;
  };
  std::vector<LD> w = lstsq(real_G(x), mom);
  const LD h = 1e-40L;
  for (int it = 0; it < 200; ++it) {
    MatT<LD> G = real_G(x);
    std::vector<LD> R(nq);
    for (int q = 0; q < nq; ++q) {
      LD s = -mom[q];
      for (int gi = 0; gi < ng; ++gi) s += G(q, gi) * w[gi];
      R[q] = -s;
    }
    MatT<LD> J(nq, npar + ng);
    for (int j = 0; j < npar; ++j) {
      std::vector<cplx> xc(x.begin(), x.end());
      xc[j] += cplx(0.0L, h);
      auto Gc = group_sums(xc);
      for (int q = 0; q < nq; ++q) {
        LD s = 0.0L;
        for (int gi = 0; gi < ng; ++gi) s += Gc[q][gi].imag() / h * w[gi];
        J(q, j) = s;
      }
    }
    for (int q = 0; q < nq; ++q)
      for (int gi = 0; gi < ng; ++gi) J(q, npar + gi) = G(q, gi);
    std::vector<LD> dz = lstsq(J, R);
    LD step = 0.0L;
    for (int j = 0; j < npar; ++j) { x[j] += dz[j]; step = std::max(step, std::fabs(dz[j])); }
    for (int gi = 0; gi < ng; ++gi) { w[gi] += dz[npar + gi]; step = std::max(step, std::fabs(dz[npar + gi])); }
    if (step < 1e-21L) break;
  }
  RuleSolution sol;
  for (LD v : x) sol.params.push_back((double)v);
  // points in double arithmetic from the rounded parameters
  std::vector<std::vector<std::vector<double>>> gpts;
  for (auto &fg : P.fixed_groups) gpts.push_back(fg);
  {
    int k = 0;
    for (auto &o : P.orbits) {
      gpts.push_back(orbit_points_d(o.kind, sol.params.data() + k, nb));
      k += orbit_npar(o.kind);
    }
  }
  MatT<LD> G(nq, ng);
  for (int gi = 0; gi < ng; ++gi)
    for (auto &pt : gpts[gi]) {
      std::vector<cplx> pc(pt.begin(), pt.end());
      for (int q = 0; q < nq; ++q) G(q, gi) += mono_val(pc, q).real();
    }
  w = lstsq(G, mom);
  LD res = 0.0L;
  for (int q = 0; q < nq; ++q) {
    LD s = -mom[q];
    for (int gi = 0; gi < ng; ++gi) s += G(q, gi) * w[gi];
    res = std::max(res, std::fabs(s));
  }
  sol.residual = (double)res;
  for (int gi = 0; gi < ng; ++gi)
    for (auto &pt : gpts[gi]) {
      sol.pts.push_back(pt);
      sol.w.push_back((double)w[gi]);
    }
  return sol;
}

// Gauss-Legendre on [0,1] (ascending), Newton on P_n from the Chebyshev-like
// initial guesses, weights 1/((1-x^2) P_n'(x)^2) on [0,1].
void gauss_legendre01(int n, std::vector<double> &t, std::vector<double> &w) {
  // Newton on P_n in extended precision from cos(pi (i + 3/4)/(n + 1/2)),
  // weights 1/((1 - x^2) P_n'(x)^2) on [0,1]; rounded to double, ascending.
  std::vector<std::pair<double, double>> tw;
  const LD pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    LD x = std::cos(pi * ((LD)i + 0.75L) / ((LD)n + 0.5L));
    LD dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      LD p0 = 1.0L, p1 = x;
      for (int k = 2; k <= n; ++k) {
        LD p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / (LD)k;
        p0 = p1;
        p1 = p2;
      }
      dp = (LD)n * (x * p1 - p0) / (x * x - 1.0L);
      LD dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-21L) break;
    }
    LD p0 = 1.0L, p1 = x;
    for (int k = 2; k <= n; ++k) {
      LD p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / (LD)k;
      p0 = p1;
      p1 = p2;
    }
    dp = (LD)n * (x * p1 - p0) / (x * x - 1.0L);
    tw.push_back({(double)(0.5L * (x + 1.0L)), (double)(1.0L / ((1.0L - x * x) * dp * dp))});
  }
  std::sort(tw.begin(), tw.end());
  t.clear();
  w.clear();
  for (auto &q : tw) { t.push_back(q.first); w.push_back(q.second); }
}

std::vector<Orbit> face_rule_spec(int p) {
  switch (p) {
    case 1: return {{'3', {1.0 / 6.0}}};
    case 2: return {{'3', {0.4459}}, {'3', {0.0916}}};
    case 3: return {{'3', {0.2493}}, {'3', {0.0631}}, {'6', {0.0531, 0.3104}}};
  }
  throw std::runtime_error("no tetrahedron face rule for this degree");
}

std::vector<Orbit> interior_spec(int dim, int p) {
  if (dim == 2) {
    switch (p) {
      case 1: return {};
      case 2: return {{'1', {}}};
      case 3: return {{'6', {0.2288, 0.1871}}};
      case 4: return {{'1', {}}, {'3', {0.1394}}, {'3', {0.4384}}};
    }
  } else {
    switch (p) {
      case 1: return {};
      case 2: return {{'1', {}}};
      case 3: return {{'T', {0.1910, 0.1173}}};
    }
  }
  throw std::runtime_error("no operator for this degree");
}

RefOp build(int dim, int p) {
  RefOp op;
  op.dim = dim;
  op.p = p;
  const int nb = dim + 1;
  op.nfac = nb;
  // facet rule in facet barycentrics (nb-1 entries), weights summing to one
  std::vector<std::vector<double>> fb;
  std::vector<double> fw;
  if (dim == 2) {
    std::vector<double> t, w;
    gauss_legendre01(p + 1, t, w);
    for (int j = 0; j <= p; ++j) fb.push_back({1.0 - t[j], t[j]});
    fw = w;
  } else {
    RuleProblem fp;
    fp.sdim = 2;
    fp.deg = 2 * p;
    fp.orbits = face_rule_spec(p);
    RuleSolution fs = solve_rule(fp);
    if (fs.residual > 1e-14) throw std::runtime_error("face rule did not converge");
    fb = fs.pts;
    for (double v : fs.w) fw.push_back(2.0 * v);  // weights of the unit-area rule
  }
  op.nf = (int)fw.size();
  // facet vertex lists
  std::vector<std::vector<int>> fverts(nb);
  for (int f = 0; f < nb; ++f) {
    if (dim == 2) fverts[f] = {(f + 1) % 3, (f + 2) % 3};
    else
      for (int i = 0; i < nb; ++i)
        if (i != f) fverts[f].push_back(i);
  }
  // facet nodes and their symmetry groups (equal facet-rule weights and equal
  // sorted barycentric multisets form one orbit of the element's symmetries)
  std::vector<std::vector<double>> bary;
  std::vector<std::vector<std::vector<double>>> groups;
  std::vector<std::vector<double>> group_keys;
  op.facet_nodes.assign((size_t)nb * op.nf, 0);
  for (int f = 0; f < nb; ++f)
    for (int j = 0; j < op.nf; ++j) {
      std::vector<double> lam(nb, 0.0);
      for (int c = 0; c < nb - 1; ++c) lam[fverts[f][c]] = fb[j][c];
      op.facet_nodes[(size_t)f * op.nf + j] = (int)bary.size();
      bary.push_back(lam);
      std::vector<double> key = fb[j];
      std::sort(key.begin(), key.end());
      int gi = -1;
      for (size_t g = 0; g < group_keys.size(); ++g) {
        bool same = true;
        for (size_t c = 0; c < key.size(); ++c)
          if (std::fabs(key[c] - group_keys[g][c]) > 1e-10) same = false;
        if (same) gi = (int)g;
      }
      if (gi < 0) { group_keys.push_back(key); groups.push_back({}); gi = (int)groups.size() - 1; }
      groups[gi].push_back(lam);
    }
  RuleProblem vp;
  vp.sdim = dim;
  vp.deg = 2 * p - 1;
  vp.fixed_groups = groups;
  vp.orbits = interior_spec(dim, p);
  RuleSolution vs = solve_rule(vp);
  if (vs.residual > 1e-14) throw std::runtime_error("volume rule did not converge");
  // map group-ordered solution points back to node order: facet nodes in
  // facet order, then interior points as returned
  auto near = [](const std::vector<double> &a, const std::vector<double> &b) {
    for (size_t i = 0; i < a.size(); ++i)
      if (std::fabs(a[i] - b[i]) > 1e-13) return false;
    return true;
  };
  std::vector<double> hw(bary.size(), -1.0);
  size_t nfixed = 0;
  for (auto &g : groups) nfixed += g.size();
  for (size_t i = 0; i < nfixed; ++i)
    for (size_t m = 0; m < bary.size(); ++m)
      if (near(vs.pts[i], bary[m])) hw[m] = vs.w[i];
  for (size_t i = nfixed; i < vs.pts.size(); ++i) {
    bary.push_back(vs.pts[i]);
    hw.push_back(vs.w[i]);
  }
  op.np = (int)bary.size();
  for (double v : hw)
    if (!(v > 0.0)) throw std::runtime_error("non-positive norm weight");
  op.h = hw;
  op.nodes.assign((size_t)op.np * dim, 0.0);
  for (int m = 0; m < op.np; ++m)
    for (int i = 0; i < dim; ++i) op.nodes[(size_t)m * dim + i] = bary[m][1 + i];
  // facet area-normals of the reference simplex: -d |T| grad(lambda_f)
  const double inv_dm1 = 1.0 / factorial(dim - 1);
  op.facet_normal.assign((size_t)nb * dim, 0.0);
  std::vector<double> area(nb);
  for (int f = 0; f < nb; ++f) {
    std::vector<double> an(dim);
    for (int i = 0; i < dim; ++i) an[i] = (f == 0) ? inv_dm1 : (i == f - 1 ? -inv_dm1 : 0.0);
    double a = 0.0;
    for (double v : an) a += v * v;
    a = std::sqrt(a);
    area[f] = a;
    for (int i = 0; i < dim; ++i) op.facet_normal[(size_t)f * dim + i] = an[i] / a;
  }
  op.facet_w.assign((size_t)nb * op.nf, 0.0);
  op.E.assign((size_t)dim * op.np, 0.0);
  for (int f = 0; f < nb; ++f)
    for (int j = 0; j < op.nf; ++j) {
      double bw = fw[j] * area[f];
      op.facet_w[(size_t)f * op.nf + j] = bw;
      int m = op.facet_nodes[(size_t)f * op.nf + j];
      for (int l = 0; l < dim; ++l) op.E[(size_t)l * op.np + m] += bw * op.facet_normal[(size_t)f * dim + l];
    }
  // Vandermonde of P^p in centred coordinates; S in extended precision
  auto mons = monomials(p, dim);
  const int nm = (int)mons.size();
  const LD cen = 1.0L / nb;
  auto ipow = [](LD x, int k) { LD v = 1.0L; for (int i = 0; i < k; ++i) v *= x; return v; };
  const int np = op.np;
  MatT<LD> V(np, nm);
  for (int m = 0; m < np; ++m)
    for (int k = 0; k < nm; ++k) {
      LD v = 1.0L;
      for (int i = 0; i < dim; ++i) v *= ipow((LD)op.nodes[(size_t)m * dim + i] - cen, mons[k][i]);
      V(m, k) = v;
    }
  MatT<LD> Qm, Rm;
  qr_thin(V, Qm, Rm);
  op.Q.assign((size_t)dim * np * np, 0.0);
  for (int l = 0; l < dim; ++l) {
    // A = H V_l - E_l V / 2, B = A R^{-1} (forward substitution on rows)
    MatT<LD> B(np, nm);
    for (int m = 0; m < np; ++m)
      for (int k = 0; k < nm; ++k) {
        LD dv = 0.0L;
        if (mons[k][l] > 0) {
          dv = (LD)mons[k][l];
          for (int i = 0; i < dim; ++i)
            dv *= ipow((LD)op.nodes[(size_t)m * dim + i] - cen, mons[k][i] - (i == l ? 1 : 0));
        }
        LD a = (LD)op.h[m] * dv - 0.5L * (LD)op.E[(size_t)l * np + m] * V(m, k);
        for (int j = 0; j < k; ++j) a -= B(m, j) * Rm(j, k);
        B(m, k) = a / Rm(k, k);
      }
    // C = Q^T B (nm x nm)
    MatT<LD> Cm(nm, nm);
    for (int a = 0; a < nm; ++a)
      for (int b2 = 0; b2 < nm; ++b2) {
        LD s2 = 0.0L;
        for (int m = 0; m < np; ++m) s2 += Qm(m, a) * B(m, b2);
        Cm(a, b2) = s2;
      }
    // S = B Q^T - Q B^T - Q C Q^T, then exact skew symmetry and Q = S + E/2
    MatT<LD> QC(np, nm);
    for (int i = 0; i < np; ++i)
      for (int b2 = 0; b2 < nm; ++b2) {
        LD s2 = 0.0L;
        for (int a = 0; a < nm; ++a) s2 += Qm(i, a) * Cm(a, b2);
        QC(i, b2) = s2;
      }
    for (int i = 0; i < np; ++i)
      for (int j = i + 1; j < np; ++j) {
        LD sij = 0.0L, sji = 0.0L;
        for (int k = 0; k < nm; ++k) {
          sij += B(i, k) * Qm(j, k) - Qm(i, k) * B(j, k) - QC(i, k) * Qm(j, k);
          sji += B(j, k) * Qm(i, k) - Qm(j, k) * B(i, k) - QC(j, k) * Qm(i, k);
        }
        const double v = (double)(0.5L * (sij - sji));
        op.Q[((size_t)l * np + i) * np + j] = v;
        op.Q[((size_t)l * np + j) * np + i] = -v;
      }
    for (int i = 0; i < np; ++i) op.Q[((size_t)l * np + i) * np + i] = 0.5 * op.E[(size_t)l * np + i];
  }
  return op;
}

}  // namespace

const RefOp &reference_operator(int dim, int p) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, RefOp> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto key = std::make_pair(dim, p);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  if (!((dim == 2 && p >= 1 && p <= 4) || (dim == 3 && p >= 1 && p <= 3)))
    throw std::invalid_argument("unsupported (dim, p)");
  auto res = cache.emplace(key, build(dim, p));
  return res.first->second;
}

// Error rule of the grid studies (Sec. 7.3: the nodal solution interpolated
// to a quadrature of degree 3p + 1).  Points of the collapsed Gauss-Legendre
// product rule on the unit simplex, q points per direction with
// 2q - 1 >= 3p + 1 + dim - 1 (the collapse adds dim - 1 to the degree in the
// last variable); the map from nodal values is the degree-p least-squares
// fit weighted by h, solved from its normal equations in long double.
static ErrRule build_error_rule(int dim, int p) {
  const RefOp &op = reference_operator(dim, p);
  ErrRule R;
  const int k = 3 * p + 1, q = (k + dim + 1) / 2;
  std::vector<double> t, w;
  gauss_legendre01(q, t, w);
  if (dim == 2) {
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        R.xi.push_back(t[i] * (1.0 - t[j]));
        R.xi.push_back(t[j]);
        R.w.push_back(w[i] * w[j] * (1.0 - t[j]));
      }
  } else {
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j)
        for (int l = 0; l < q; ++l) {
          R.xi.push_back(t[i] * (1.0 - t[j]) * (1.0 - t[l]));
          R.xi.push_back(t[j] * (1.0 - t[l]));
          R.xi.push_back(t[l]);
          R.w.push_back(w[i] * w[j] * w[l] * (1.0 - t[j]) * (1.0 - t[l]) * (1.0 - t[l]));
        }
  }
  R.nq = (int)R.w.size();
  const auto mon = monomials(p, dim);
  const int N = (int)mon.size(), np = op.np;
  auto vand = [&](const double *x, int m) {
    LD v = 1.0L;
    for (int d = 0; d < dim; ++d)
      for (int e = 0; e < mon[m][d]; ++e) v *= (LD)x[d];
    return v;
  };
  // normal equations A c = V^T h f for all unit nodal vectors f at once:
  // A = V^T h V [N][N], B = V^T h [N][np]
  std::vector<LD> A((size_t)N * N, 0.0L), B((size_t)N * np, 0.0L);
  for (int j = 0; j < np; ++j) {
    const double *x = &op.nodes[(size_t)j * dim];
    for (int a = 0; a < N; ++a) {
      const LD va = vand(x, a) * (LD)op.h[j];
      B[(size_t)a * np + j] = va;
      for (int b = 0; b < N; ++b) A[(size_t)a * N + b] += va * vand(x, b);
    }
  }
  // Gaussian elimination with partial pivoting: B <- A^-1 B
  for (int c = 0; c < N; ++c) {
    int piv = c;
    for (int r = c + 1; r < N; ++r)
      if (std::fabs(A[(size_t)r * N + c]) > std::fabs(A[(size_t)piv * N + c])) piv = r;
    if (piv != c) {
      for (int b = 0; b < N; ++b) std::swap(A[(size_t)c * N + b], A[(size_t)piv * N + b]);
      for (int b = 0; b < np; ++b) std::swap(B[(size_t)c * np + b], B[(size_t)piv * np + b]);
    }
    const LD d = A[(size_t)c * N + c];
    for (int r = 0; r < N; ++r) {
      if (r == c) continue;
      const LD f = A[(size_t)r * N + c] / d;
      if (f == 0.0L) continue;
      for (int b = 0; b < N; ++b) A[(size_t)r * N + b] -= f * A[(size_t)c * N + b];
      for (int b = 0; b < np; ++b) B[(size_t)r * np + b] -= f * B[(size_t)c * np + b];
    }
  }
  for (int c = 0; c < N; ++c)
    for (int b = 0; b < np; ++b) B[(size_t)c * np + b] /= A[(size_t)c * N + c];
  R.I.assign((size_t)R.nq * np, 0.0);
  for (int m = 0; m < R.nq; ++m)
    for (int j = 0; j < np; ++j) {
      LD s = 0.0L;
      for (int a = 0; a < N; ++a) s += vand(&R.xi[(size_t)m * dim], a) * B[(size_t)a * np + j];
      R.I[(size_t)m * np + j] = (double)s;
    }
  return R;
}

const ErrRule &error_rule(int dim, int p) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, ErrRule> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto key = std::make_pair(dim, p);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  auto res = cache.emplace(key, build_error_rule(dim, p));
  return res.first->second;
}

}  // namespace sbp
