// Forward-mode dual numbers for the device vector-Jacobian product: a value
// and one directional derivative.  The pointwise physics templates of
// device_physics.hpp instantiate with Dual<double> unchanged; comparisons and
// branch choices use the value part.
#pragma once
#include <hip/hip_runtime.h>

#include "device_physics.hpp"

namespace sbp {

template <typename T>
struct Dual {
  T v, d;
  __host__ __device__ Dual() : v(0), d(0) {}
  __host__ __device__ Dual(T a) : v(a), d(0) {}
  __host__ __device__ Dual(T a, T b) : v(a), d(b) {}
  __host__ __device__ explicit Dual(int a) : v((T)a), d(0) {}
  __host__ __device__ Dual &operator+=(const Dual &o) { v += o.v; d += o.d; return *this; }
  __host__ __device__ Dual &operator-=(const Dual &o) { v -= o.v; d -= o.d; return *this; }
  __host__ __device__ Dual &operator*=(const Dual &o) { d = d * o.v + v * o.d; v *= o.v; return *this; }
};

template <typename T> __device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator/(Dual<T> a, Dual<T> b) {
  const T ib = drcp(b.v);
  const T q = a.v * ib;
  return {q, (a.d - q * b.d) * ib};
}
template <typename T> __device__ __forceinline__ bool operator<(Dual<T> a, Dual<T> b) { return a.v < b.v; }
template <typename T> __device__ __forceinline__ bool operator>(Dual<T> a, Dual<T> b) { return a.v > b.v; }
template <typename T> __device__ __forceinline__ bool operator<=(Dual<T> a, Dual<T> b) { return a.v <= b.v; }
template <typename T> __device__ __forceinline__ bool operator>=(Dual<T> a, Dual<T> b) { return a.v >= b.v; }

__device__ __forceinline__ Dual<double> dexp(Dual<double> a) {
  const double e = exp(a.v);
  return {e, e * a.d};
}
__device__ __forceinline__ Dual<double> dlog(Dual<double> a) { return {log(a.v), a.d * drcp(a.v)}; }
__device__ __forceinline__ Dual<double> dsqrt(Dual<double> a) {
  const double s = sqrt(a.v);
  return {s, 0.5 * a.d * drcp(s)};
}
// |x| with derivative sign(x) (0 at x = 0)
__device__ __forceinline__ Dual<double> dabs(Dual<double> a) {
  const double sg = a.v > 0.0 ? 1.0 : (a.v < 0.0 ? -1.0 : 0.0);
  return {fabs(a.v), sg * a.d};
}

template <typename T>
__host__ __device__ GasC<Dual<T>> dual_gas(const GasC<T> &G) {
  GasC<Dual<T>> H;
  H.g = G.g;
  H.gm1 = G.gm1;
  H.a = G.a;
  H.cb = G.cb;
  H.inv_apg = G.inv_apg;
  H.r1 = G.r1;
  H.r2 = G.r2;
  H.wfirst = G.wfirst;
  H.ja = G.ja;
  H.jb_inv = G.jb_inv;
  H.sfac = G.sfac;
  H.ggm1 = G.ggm1;
  H.gm1_a = G.gm1_a;
  const ExpAvgC<T> *src[2] = {&G.e1, &G.e2};
  ExpAvgC<Dual<T>> *dst[2] = {&H.e1, &H.e2};
  for (int q = 0; q < 2; ++q) {
    dst[q]->r = src[q]->r;
    for (int k = 0; k < 4; ++k) dst[q]->c[k] = src[q]->c[k];
    for (int k = 0; k < 9; ++k) dst[q]->bn[k] = src[q]->bn[k];
  }
  return H;
}

}  // namespace sbp
