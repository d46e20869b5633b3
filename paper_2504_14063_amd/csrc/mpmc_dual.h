// mpmc_dual.h -- forward-mode dual numbers with N tangent directions.
//
// Used by the discrete adjoint for the small blocks with few inputs (the
// per-cell equilibrium and auxiliaries, the face-average equilibrium): their
// Jacobians are obtained by running the very same templated forward code on
// Dual<N> with one unit tangent per input.  Every branch is decided on the
// value part, so decisions are those of the unperturbed state.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#ifndef MPMC_HD
#define MPMC_HD __host__ __device__ __forceinline__
#endif

namespace mpmc {

template <int N> struct Dual {
  double v;
  double d[N];
  __host__ __device__ Dual() : v(0.0) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
  __host__ __device__ Dual(double x) : v(x) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
  // value x with unit tangent along direction k
  static __host__ __device__ Dual seed(double x, int k) {
    Dual r(x);
    r.d[k] = 1.0;
    return r;
  }
};

MPMC_HD double val(double x) { return x; }
MPMC_HD float val(float x) { return x; }
template <int N> MPMC_HD double val(const Dual<N>& x) { return x.v; }

template <int N> MPMC_HD Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v + b.v);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N> MPMC_HD Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v - b.v);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N> MPMC_HD Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r(-a.v);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N> MPMC_HD Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v * b.v);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N> MPMC_HD Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  const double q = a.v / b.v, ib = 1.0 / b.v;
  Dual<N> r(q);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - q * b.d[i]) * ib;
  return r;
}
template <int N> MPMC_HD Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> MPMC_HD Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> MPMC_HD Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> MPMC_HD Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> MPMC_HD Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r(a.v * b);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int N> MPMC_HD Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> MPMC_HD Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> MPMC_HD Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> MPMC_HD Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { return a = a + b; }
template <int N> MPMC_HD Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { return a = a - b; }
template <int N> MPMC_HD Dual<N>& operator*=(Dual<N>& a, const Dual<N>& b) { return a = a * b; }
template <int N> MPMC_HD bool operator<(const Dual<N>& a, const Dual<N>& b) { return a.v < b.v; }
template <int N> MPMC_HD bool operator>(const Dual<N>& a, const Dual<N>& b) { return a.v > b.v; }
template <int N> MPMC_HD bool operator<=(const Dual<N>& a, const Dual<N>& b) { return a.v <= b.v; }
template <int N> MPMC_HD bool operator>=(const Dual<N>& a, const Dual<N>& b) { return a.v >= b.v; }
template <int N> MPMC_HD bool operator==(const Dual<N>& a, const Dual<N>& b) { return a.v == b.v; }

template <int N> MPMC_HD Dual<N> sqrt(const Dual<N>& a) {
  const double s = ::sqrt(a.v), h = 0.5 / s;
  Dual<N> r(s);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * h;
  return r;
}
template <int N> MPMC_HD Dual<N> log(const Dual<N>& a) {
  const double ia = 1.0 / a.v;
  Dual<N> r(::log(a.v));
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * ia;
  return r;
}
template <int N> MPMC_HD Dual<N> tanh(const Dual<N>& a) {
  const double t = ::tanh(a.v), g = 1.0 - t * t;
  Dual<N> r(t);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * g;
  return r;
}
// |x| with the arm of the value's sign (x >= 0 keeps x)
template <int N> MPMC_HD Dual<N> fabs(const Dual<N>& a) { return a.v >= 0.0 ? a : -a; }

}  // namespace mpmc
