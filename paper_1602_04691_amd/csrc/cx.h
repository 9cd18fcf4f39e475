// Minimal complex arithmetic for device code (interleaved {re, im}).
//
// The library is compiled without automatic contraction of a * b + c into
// fused multiply-adds (-ffp-contract=off): which of two products the
// compiler would fuse in a * b - c * d depends on the code around it, so
// the same expression could round differently in two kernels.  The fused
// operations are written out instead (fmadd), so every kernel that runs a
// piece of arithmetic rounds it the same way.
#pragma once

#include <hip/hip_runtime.h>

namespace ori {

__host__ __device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__host__ __device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

using cxd = cx<double>;
using cxf = cx<float>;

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) {
  return cx<T>{a, b};
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {fmadd(a.re, b.re, -(a.im * b.im)), fmadd(a.re, b.im, a.im * b.re)};
}
// y + a b and y - a b
template <typename T>
__device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> y) {
  return {fmadd(a.re, b.re, fmadd(-a.im, b.im, y.re)), fmadd(a.re, b.im, fmadd(a.im, b.re, y.im))};
}
template <typename T>
__device__ __forceinline__ cx<T> cfms(cx<T> a, cx<T> b, cx<T> y) {
  return {fmadd(-a.re, b.re, fmadd(a.im, b.im, y.re)), fmadd(-a.re, b.im, fmadd(-a.im, b.re, y.im))};
}
// y + s x
template <typename T>
__device__ __forceinline__ cx<T> axpy(cx<T> y, cx<T> x, T s) {
  return {fmadd(x.re, s, y.re), fmadd(x.im, s, y.im)};
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) {
  return {a.re * s, a.im * s};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) {
  return {a.re, -a.im};
}
// a * conj(w) when INV, a * w otherwise (twiddles are stored for the forward sign)
template <bool INV, typename T>
__device__ __forceinline__ cx<T> twiddle(cx<T> a, cx<T> w) {
  if (INV) return {fmadd(a.re, w.re, a.im * w.im), fmadd(a.im, w.re, -(a.re * w.im))};
  return a * w;
}
template <typename To, typename From>
__device__ __forceinline__ cx<To> cvt(cx<From> a) {
  return {static_cast<To>(a.re), static_cast<To>(a.im)};
}
template <typename T>
__device__ __forceinline__ double norm2(cx<T> a) {
  const double re = a.re, im = a.im;
  return fmadd(re, re, im * im);
}

}  // namespace ori
