// dual_dev.h -- forward-mode numbers (value + one tangent) for the adjoint
// kernels: the local Jacobians of the Riemann solver and of the Hancock
// predictor are taken by running the same device functions on these numbers,
// one input direction at a time.
#pragma once
#include <hip/hip_runtime.h>

#include "mhd_dev.h"

namespace dsp {

template <class R> struct Dual {
  R v, d;
  __device__ Dual() : v(R(0)), d(R(0)) {}
  __device__ Dual(R a) : v(a), d(R(0)) {}
  __device__ Dual(R a, R b) : v(a), d(b) {}
};

template <class R> __device__ __forceinline__ Dual<R> operator+(Dual<R> a, Dual<R> b) {
  return Dual<R>(a.v + b.v, a.d + b.d);
}
template <class R> __device__ __forceinline__ Dual<R> operator-(Dual<R> a, Dual<R> b) {
  return Dual<R>(a.v - b.v, a.d - b.d);
}
template <class R> __device__ __forceinline__ Dual<R> operator-(Dual<R> a) { return Dual<R>(-a.v, -a.d); }
template <class R> __device__ __forceinline__ Dual<R> operator*(Dual<R> a, Dual<R> b) {
  return Dual<R>(a.v * b.v, a.d * b.v + a.v * b.d);
}
template <class R> __device__ __forceinline__ Dual<R> operator/(Dual<R> a, Dual<R> b) {
  const R q = a.v / b.v;
  return Dual<R>(q, (a.d - q * b.d) / b.v);
}
// mixed forms (a plain number is a constant)
template <class R> __device__ __forceinline__ Dual<R> operator*(R a, Dual<R> b) { return Dual<R>(a * b.v, a * b.d); }
template <class R> __device__ __forceinline__ Dual<R> operator*(Dual<R> a, R b) { return Dual<R>(a.v * b, a.d * b); }
template <class R> __device__ __forceinline__ bool operator<(Dual<R> a, Dual<R> b) { return a.v < b.v; }
template <class R> __device__ __forceinline__ bool operator>(Dual<R> a, Dual<R> b) { return a.v > b.v; }
template <class R> __device__ __forceinline__ bool operator<=(Dual<R> a, Dual<R> b) { return a.v <= b.v; }
template <class R> __device__ __forceinline__ bool operator>=(Dual<R> a, Dual<R> b) { return a.v >= b.v; }
template <class R> __device__ __forceinline__ Dual<R> fabs(Dual<R> a) { return a.v < R(0) ? -a : a; }

template <> struct Eps<Dual<float>> { static constexpr float deg = Eps<float>::deg; };
template <> struct Eps<Dual<double>> { static constexpr double deg = Eps<double>::deg; };

// IEEE arithmetic on dual numbers; the square root's tangent at 0 is taken
// as 0 (its symmetric derivative), as the oracle's forward mode does.
template <class R> struct DualExact {
  static __device__ __forceinline__ Dual<R> rcp(Dual<R> x) { return Dual<R>(R(1)) / x; }
  static __device__ __forceinline__ Dual<R> div(Dual<R> a, Dual<R> b) { return a / b; }
  static __device__ __forceinline__ Dual<R> root(Dual<R> x) {
    const R s = sqrt(x.v);
    if (s == R(0)) return Dual<R>(R(0), R(0));
    return Dual<R>(s, x.d / (R(2) * s));
  }
};

}  // namespace dsp
