// FFT plans for the padded length L = 2n of each axis (Section 3 pads every
// axis before the convolution theorem, eq. 3.3.8).  Shared by host and device
// code: everything here is constexpr.
#pragma once

#include <cstdint>

namespace ori {

// Every supported padded length, one translation unit of FFT kernels each.
#define ORI_FOR_EACH_L(X) \
  X(2) X(4) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) \
  X(128) X(192) X(256) X(384) X(512) X(1024)

struct RadixPlan {
  int n;     // number of Stockham stages
  int r[4];  // forward radix order; the inverse runs them in reverse
};

// The first forward radix is even so that the zero upper half of a padded
// input is skipped at compile time.  Radix 8 is the sweet spot on gfx950 in
// complex128: 8 values (32 VGPRs) per butterfly leave room for the spectrum
// and twiddles of the fused Z pass at 4 waves per SIMD, where radix 16 needs
// over 200 VGPRs.  L = 16 is 4 x 4 (four threads per pencil), so that its
// pass bodies fit the register budget of the multi-problem launches.
constexpr RadixPlan radix_plan(int L) {
  switch (L) {
    case 2: return {1, {2, 0, 0, 0}};
    case 4: return {1, {4, 0, 0, 0}};
    case 6: return {2, {2, 3, 0, 0}};
    case 8: return {1, {8, 0, 0, 0}};
    case 10: return {2, {2, 5, 0, 0}};
    case 12: return {2, {4, 3, 0, 0}};
    case 16: return {2, {4, 4, 0, 0}};
    case 20: return {2, {4, 5, 0, 0}};
    case 24: return {2, {8, 3, 0, 0}};
    case 32: return {2, {8, 4, 0, 0}};
    case 40: return {2, {8, 5, 0, 0}};
    case 48: return {3, {8, 2, 3, 0}};
    case 64: return {2, {8, 8, 0, 0}};
    case 80: return {3, {8, 2, 5, 0}};
    case 96: return {3, {8, 4, 3, 0}};
    case 128: return {3, {8, 4, 4, 0}};
    case 192: return {3, {8, 8, 3, 0}};
    case 256: return {3, {8, 8, 4, 0}};
    case 384: return {4, {8, 4, 4, 3}};
    case 512: return {3, {8, 8, 8, 0}};
    case 1024: return {4, {8, 8, 4, 4}};
    default: return {0, {0, 0, 0, 0}};
  }
}

// Alternative plans of the fused Z pass (its radix-plan knob, `zplan`):
// variant 1 factors L into another radix order, or other radices, with the
// same threads per pencil (the smallest butterfly count of a stage), so
// that the Z workgroup shape is unchanged; the first radix stays even.  At
// L = 1024 variant 1 is 16 x 8 x 8: two exchanges per transform instead of
// three with the same 64 threads per pencil (complex128 Z 6.04 vs 6.52 ms
// at n = 512, its default there).  Lengths without an alternative (L = 64
// and most short ones) have variant 1 equal to the default.
constexpr RadixPlan radix_plan(int L, int variant) {
  if (variant == 1) switch (L) {
      case 32: return {2, {4, 8, 0, 0}};
      case 48: return {3, {8, 3, 2, 0}};
      case 80: return {3, {8, 5, 2, 0}};
      case 96: return {3, {4, 8, 3, 0}};
      case 128: return {3, {4, 4, 8, 0}};
      case 192: return {3, {8, 3, 8, 0}};
      case 256: return {3, {4, 8, 8, 0}};
      case 384: return {4, {8, 3, 4, 4}};
      case 512: return {4, {8, 4, 4, 4}};
      case 1024: return {3, {16, 8, 8, 0}};
      default: break;
    }
  return radix_plan(L);
}

constexpr bool same_plan(const RadixPlan& a, const RadixPlan& b) {
  if (a.n != b.n) return false;
  for (int s = 0; s < a.n; ++s)
    if (a.r[s] != b.r[s]) return false;
  return true;
}

// whether the Z pass has a second plan at L
constexpr bool has_plan_variant(int L) { return !same_plan(radix_plan(L, 1), radix_plan(L)); }

constexpr bool supported_length(int L) { return radix_plan(L).n > 0; }

// Threads per pencil: the smallest butterfly count over the stages, so that
// no stage leaves threads idle in its widest configuration, capped at two
// wavefronts (L = 1024: one radix-8 butterfly per thread keeps a complex128
// thread within 128 registers).
constexpr int threads_per_pencil(int L, int variant = 0) {
  RadixPlan p = radix_plan(L, variant);
  int t = L;
  for (int s = 0; s < p.n; ++s) {
    int b = L / p.r[s];
    if (b < t) t = b;
  }
  return t > 128 ? 128 : t;
}

constexpr int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

// Pencils per workgroup.  Strided passes need several adjacent pencils per
// row so that each row read/written is a contiguous run (8 x 16 B = 128 B for
// complex128, 16 x 8 B for complex64); contiguous passes only need enough
// threads to fill the workgroup.
// Workgroups are whole wavefronts (64 lanes): the reductions use full-wave
// shuffles.
constexpr int whole_waves(int np, int tpp) {
  while ((np * tpp) % 64 != 0) np *= 2;
  return np;
}

constexpr int pencils_strided(int L, int elem_bytes) {
  int tpp = threads_per_pencil(L);
  int np = pow2_floor(256 / tpp);
  int lo = elem_bytes == 16 ? 8 : 16;
  if (np < lo) np = lo;
  if (np > 64) np = 64;
  while (np > 1 && np * tpp > 1024) np /= 2;  // at most 1024 threads per workgroup
  return whole_waves(np, tpp);
}

constexpr int pencils_contig(int L) {
  int tpp = threads_per_pencil(L);
  int np = pow2_floor(256 / tpp);
  if (np < 1) np = 1;
  return whole_waves(np, tpp);
}

}  // namespace ori
