// Device helpers shared by the FFT pass kernels of every padded length:
// deterministic workgroup sums, raw buffer accesses, the two-level row
// addressing of the work arrays and the XCD-aware workgroup order.
#pragma once

#include <cstdint>

#include "cx.h"

namespace ori {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic sum of 4 values over the workgroup; thread 0 writes them.
template <int NT>
__device__ __forceinline__ void block_partials(double (&v)[4], void* lds_scratch, double* out) {
  constexpr int NW = NT / 64;
  double* sh = static_cast<double*>(lds_scratch);
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = wave_sum(v[j]);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) sh[w * 4 + j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int i = 0; i < NW; ++i) s += sh[i * 4 + j];
      out[j] = s;
    }
  }
}

// Raw buffer accesses: the base address in a buffer resource (scalar
// registers; no stride, num_records bytes of range, dword 3 as on every
// gfx9 part) and a 32-bit byte offset per lane, so that per-tile address
// arithmetic stays off the vector ALU.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, int32_t bytes) {
  // the base is uniform over the workgroup: read it from the first lane so
  // that the resource is built in scalar registers
  const uint64_t b = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b >> 32));
  void* p = reinterpret_cast<void*>((static_cast<uint64_t>(hi) << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, 0, bytes, 0x00020000);
}

// off: the lane's byte offset; soff: a byte offset the same for every lane
// (a scalar register)
template <typename T>
__device__ __forceinline__ cx<T> buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0) {
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(off),
                                                                             static_cast<int>(soff), 0));
  } else {
    return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(off),
                                                                            static_cast<int>(soff), 0));
  }
}

template <typename T>
__device__ __forceinline__ void buffer_store(__amdgpu_buffer_rsrc_t r, uint32_t off, cx<T> v, uint32_t soff = 0) {
  using V4 = __attribute__((ext_vector_type(4))) unsigned int;
  using V2 = __attribute__((ext_vector_type(2))) unsigned int;
  if constexpr (sizeof(T) == 8) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, v), r, static_cast<int>(off),
                                           static_cast<int>(soff), 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, static_cast<int>(off),
                                          static_cast<int>(soff), 0);
  }
}

__device__ __forceinline__ int64_t two_level(int64_t o, int lg, int64_t hi, int64_t lo) {
  return (o >> lg) * hi + (o & ((int64_t{1} << lg) - 1)) * lo;
}

// Workgroups go round-robin over the 8 XCDs (workgroup b runs on XCD b % 8,
// each XCD with its own L2).  xcd_order renumbers them so that each XCD walks
// one contiguous range of tiles: neighbouring tiles, which share cache lines
// and spectrum rows, then meet in the same L2.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t G) {
  constexpr int64_t X = 8;
  const int64_t q = G / X, r = G % X, x = b % X, j = b / X;
  return x * q + (x < r ? x : r) + j;
}

}  // namespace ori
