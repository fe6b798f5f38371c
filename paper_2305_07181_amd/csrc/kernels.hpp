// Kernel-side shapes and argument blocks shared by the HIP translation units
// and the host launch code.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_physics.hpp"

namespace sbp {

constexpr int ru(int x, int m) { return (x + m - 1) / m * m; }

// Node counts of the operators built by refops.cpp.
template <int DIM, int P>
struct Shape;
template <> struct Shape<2, 1> { static constexpr int NP = 6, NF = 2; };
template <> struct Shape<2, 2> { static constexpr int NP = 10, NF = 3; };
template <> struct Shape<2, 3> { static constexpr int NP = 18, NF = 4; };
template <> struct Shape<2, 4> { static constexpr int NP = 22, NF = 5; };
template <> struct Shape<3, 1> { static constexpr int NP = 12, NF = 3; };
template <> struct Shape<3, 2> { static constexpr int NP = 25, NF = 6; };
template <> struct Shape<3, 3> { static constexpr int NP = 60, NF = 12; };

// Device tables of one degree class (pointers into one device allocation).
template <typename T>
struct OpTables {
  const T *S;   // skew parts S_xi_l = Q_xi_l - E_xi_l / 2, [dim][NP][NP]
  const T *h;   // [NP]
  const T *E;   // [dim][NP] diagonal of E_xi_l
  const T *dN;  // derivatives of the quadratic map basis at the nodes: 2D [2][6][NP], 3D [3][10][NP]
};

template <typename T>
struct KArgs {
  const double *u;     // state (FP64)
  T *r;                // residual (T)
  const double *geo;   // 2D: [n_elem][12] map nodes; 3D affine: [n_elem][10] Lambda (row i,
                       // col l), J; 3D curved: [n_elem][10][3] quadratic map nodes
  const int *nbr;      // [n_elem][NFAC*NF] u offset of the matching neighbour node (component 0)
  const int *uoff;     // [n_elem] u offset of each element of the class
  int u_dense, u_base; // u_dense: uoff[e] == u_base + e n_c n_p for every e (no lookup needed)
  int n_elem;
  int diss;
  OpTables<T> op;
  GasC<T> G;
  double *ent_part;    // [gridDim.x] partial sums of w^T H r (may be null)
  int *err;            // non-physical state flag
  // Navier-Stokes terms (Baumann-Oden SATs)
  int visc;
  int curved;          // 3D: quadratic maps (metrics from geo and op.dN per node)
  ViscC<T> V;
  const T *q;          // [n_elem][NFAC*NF][n_c] facet normal viscous fluxes B n . F^V
  T *qout;             // written by the facet-flux pre-pass
  const int *nbrq;     // [n_elem][NFAC*NF] index (elem*NFAC*NF + node) of the neighbour's q
  // vector-Jacobian product
  const double *lam;   // cotangent (state layout)
  double *ubar;        // result (state layout)
  const double *Hn;    // [n_elem*NP] diagonal of H_k
  // hybrid scheme: volume form of every element of the mesh (0 entropy split,
  // 1 Hadamard) in the mesh's element order, or null; the kernel of form
  // form_id then skips the elements of the other form
  const unsigned char *eform;
  const int *gid;      // [n_elem] mesh element id of each element of the class
  int form_id;
  // the exponential-average constants of G (G.e1, G.e2) in device memory:
  // kernels that read them at their use instead of holding them in scalar
  // registers for the whole launch
  const ExpAvgC<T> *eac;
  const JumpC<T> *jc;  // binomial coefficients of the node powers (node_near)
  // launch timing (2D entropy split): [0] earliest workgroup start, [1] latest
  // workgroup end on the device's constant-rate clock, or null
  unsigned long long *tstamp;
};

// Map-node coordinate idx of an element (g: its FP64 map nodes) for the
// metric sums F = sum_a dN_a g_a, with `first` the index of the same
// coordinate of the element's first map node.  In FP32 the coordinate is
// taken relative to that node, in FP64 before rounding: the basis
// derivatives sum to zero, so F is unchanged in exact arithmetic, and the
// small differences keep FP32's digits (absolute coordinates of O(10)
// against an element size of O(0.1) would lose about seven bits of every
// metric term).  FP64 takes the coordinates as they are.
template <typename T>
__device__ __forceinline__ T map_node(const double *g, int idx, int first) {
  if constexpr (sizeof(T) == 4)
    return (T)(g[idx] - g[first]);
  else
    return (T)g[idx];
}

// Tile order of a persistent workgroup.  The chip dispatches workgroups to
// its 8 XCDs (each with its own L2) round-robin by workgroup index, so
// workgroup b runs on XCD b mod 8.  When the grid is a multiple of 8, each
// XCD takes one contiguous eighth of the tiles: an element's facet
// neighbours (nearby element indices on the structured grids) are then read
// by the same XCD, from its L2, instead of from another XCD's memory.
constexpr int kXcds = 8;
struct TileSeq {
  int t, step, end;
  __device__ __forceinline__ explicit TileSeq(int ntiles) {
    const int b = blockIdx.x, G = gridDim.x;
    if (G % kXcds == 0) {
      const int per = (ntiles + kXcds - 1) / kXcds;
      const int x = b % kXcds;
      t = x * per + b / kXcds;
      step = G / kXcds;
      end = min(ntiles, (x + 1) * per);
    } else {
      t = b;
      step = G;
      end = ntiles;
    }
  }
};

// Whether element e of the class runs in this kernel (hybrid scheme).  Any
// nonzero flag byte selects the Hadamard form, so exactly one of the two
// kernels writes each element's residual whatever the caller's bytes are.
template <typename T>
__device__ __forceinline__ bool elem_on(const KArgs<T> &A, int e) {
  return !A.eform || (A.eform[A.gid[e]] != 0) == (A.form_id != 0);
}

// Whether any element of [e0, e0 + ne) runs in this kernel; the same answer
// in every lane, so a workgroup may skip the tile as a whole.
template <typename T>
__device__ __forceinline__ bool tile_on(const KArgs<T> &A, int e0, int ne) {
  if (!A.eform) return true;
  for (int e = 0; e < ne; ++e)
    if (elem_on(A, e0 + e)) return true;
  return false;
}

// All degree classes of a 2D mesh in one launch: cls[p-1] (device memory,
// written at mesh setup) holds the argument block of the class of degree p
// (n_elem = 0 if absent) without the per-call pointers, which follow here;
// g0[p-1] is the class's first group in the launch-wide group index, g0[4]
// the number of groups.  Reading the blocks from memory where a tile needs
// them keeps the four classes' arguments out of the scalar registers.
template <typename T>
struct Batch2 {
  const KArgs<T> *cls;
  const double *u;
  T *r;
  const unsigned char *eform;
  const double *lam;
  double *ubar;
  int g0[5];
  double *ent_part;  // [gridDim.x] partial sums of w^T H r (may be null)
  unsigned long long *tstamp;  // launch timing as KArgs::tstamp, or null
};

// A pointer read from memory, marked as one into global memory (the device
// allocations of a mesh handle).  The compiler takes a pointer it loads for a
// flat one, and flat loads also count against the LDS wait counter, so every
// LDS wait would wait for them as well.  The route through an integer is one
// the address-space inference follows and later passes do not fold away.
template <typename P>
__device__ __forceinline__ P *as_global(P *p) {
  return (P *)(__attribute__((address_space(1))) P *)(unsigned long long)p;
}

// The argument block of class q of a batched launch with the call's pointers.
template <typename T>
__device__ __forceinline__ KArgs<T> batch_args(const Batch2<T> &Bt, int q) {
  KArgs<T> A = Bt.cls[q];
  A.geo = as_global(A.geo);
  A.nbr = as_global(A.nbr);
  A.nbrq = as_global(A.nbrq);
  A.uoff = as_global(A.uoff);
  A.gid = as_global(A.gid);
  A.Hn = as_global(A.Hn);
  A.op.S = as_global(A.op.S);
  A.op.h = as_global(A.op.h);
  A.op.E = as_global(A.op.E);
  A.op.dN = as_global(A.op.dN);
  A.err = as_global(A.err);
  A.eac = as_global(A.eac);
  A.jc = as_global(A.jc);
  A.u = Bt.u;
  A.r = Bt.r;
  A.eform = Bt.eform;
  A.lam = Bt.lam;
  A.ubar = Bt.ubar;
  return A;
}

}  // namespace sbp
