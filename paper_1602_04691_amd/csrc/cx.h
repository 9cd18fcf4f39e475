// Minimal complex arithmetic for device code (interleaved {re, im}).
#pragma once

#include <hip/hip_runtime.h>

namespace ori {

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
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
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
  if (INV) return {a.re * w.re + a.im * w.im, a.im * w.re - a.re * w.im};
  return {a.re * w.re - a.im * w.im, a.re * w.im + a.im * w.re};
}
template <typename To, typename From>
__device__ __forceinline__ cx<To> cvt(cx<From> a) {
  return {static_cast<To>(a.re), static_cast<To>(a.im)};
}
template <typename T>
__device__ __forceinline__ double norm2(cx<T> a) {
  return static_cast<double>(a.re) * a.re + static_cast<double>(a.im) * a.im;
}

}  // namespace ori
