// Reference-element diagonal-E SBP operator (host).  See refops.cpp.
#pragma once
#include <vector>

namespace sbp {

struct RefOp {
  int dim = 0, p = 0, np = 0, nf = 0, nfac = 0;
  std::vector<double> nodes;         // [np][dim] reference coordinates
  std::vector<double> h;             // [np] diagonal of H
  std::vector<double> Q;             // [dim][np][np]
  std::vector<double> E;             // [dim][np] diagonal of E
  std::vector<int> facet_nodes;      // [nfac][nf] volume-node indices
  std::vector<double> facet_w;       // [nfac][nf] facet weights (reference measure)
  std::vector<double> facet_normal;  // [nfac][dim] unit outward normals
};

// Cached, thread-safe.  Throws std::invalid_argument for unsupported (dim,p).
const RefOp &reference_operator(int dim, int p);

// Quadrature of degree 3p + 1 on the unit simplex and the map from nodal
// values to its points (the error norm of the grid studies).
struct ErrRule {
  int nq = 0;
  std::vector<double> xi;  // [nq][dim] reference coordinates
  std::vector<double> w;   // [nq]
  std::vector<double> I;   // [nq][np]: degree-p fit weighted by h, at xi
};
// Cached, thread-safe; same (dim, p) range as reference_operator.
const ErrRule &error_rule(int dim, int p);

}  // namespace sbp
