// Register/LDS Stockham FFT engine for one workgroup of pencils (gfx950).
//
// The product with the Green's matrix is a 3-D convolution (Section 3,
// eqs. 3.3.4-3.3.7), evaluated with the convolution theorem (eq. 3.3.8) on
// a grid padded to L = 2n per axis.  Each pass of that evaluation is a batch
// of length-L DFTs along one axis ("pencils").  A workgroup owns NP pencils
// and TPP threads per pencil; each thread holds whole radix-R butterflies in
// registers.  Stage s reads its inputs at  b + r * (L / R)  and writes its
// outputs at  (b - k) R + k + j Ns  (k = b mod Ns, Ns = product of earlier
// radices): the self-sorting Stockham order, so the last stage writes the
// natural order and no bit reversal pass is needed.  The first stage reads
// and the last stage writes global memory directly (the pattern
// b + r * (L/R) is coalesced both along a contiguous pencil and across
// adjacent strided pencils); the stages in between exchange through LDS.
#pragma once

#include <type_traits>

#include "cx.h"
#include "plan.h"

namespace ori {

// f(integral_constant<int, I>) for I = 0 .. N-1
template <int N, int I = 0, class F>
__device__ __forceinline__ void unroll(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    unroll<N, I + 1>(f);
  }
}

// ---------------------------------------------------------------------------
// DFT butterflies, natural order in and out.  Forward uses exp(-2 pi i/R).
// ---------------------------------------------------------------------------
template <bool INV, typename T>
__device__ __forceinline__ cx<T> mul_w4(cx<T> a) {  // * exp(-+ i pi/2)
  return INV ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

// multiply by exp(-+ 2 pi i m / 16) for m = 0..7 (compile-time m)
template <bool INV, int M, typename T>
__device__ __forceinline__ cx<T> mul_w16(cx<T> a) {
  constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
  constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
  constexpr double H = 0.70710678118654752440;   // cos(pi/4)
  constexpr double cs[8] = {1.0, C1, H, S1, 0.0, -S1, -H, -C1};
  constexpr double sn[8] = {0.0, S1, H, C1, 1.0, C1, H, S1};
  if constexpr (M == 0) return a;
  if constexpr (M == 4) return mul_w4<INV>(a);
  const T c = static_cast<T>(cs[M]);
  const T s = INV ? static_cast<T>(sn[M]) : static_cast<T>(-sn[M]);
  return {fmadd(a.re, c, -(a.im * s)), fmadd(a.re, s, a.im * c)};
}

// (a, b) <- (a + t b, a - t b) in six fused multiply-adds: a - t b is formed
// as 2a - (a + t b), so the product t b is never rounded on its own.
template <typename T>
__device__ __forceinline__ void bfly_tw(cx<T>& a, cx<T>& b, cx<T> t) {
  const T pr = fmadd(-t.im, b.im, fmadd(t.re, b.re, a.re));
  const T pi = fmadd(t.im, b.re, fmadd(t.re, b.im, a.im));
  b = {fmadd(static_cast<T>(2), a.re, -pr), fmadd(static_cast<T>(2), a.im, -pi)};
  a = {pr, pi};
}

template <bool INV, int R, typename T>
struct Dft;

template <bool INV, typename T>
struct Dft<INV, 2, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    cx<T> a = v[0];
    v[0] = a + v[1];
    v[1] = a - v[1];
  }
  __device__ __forceinline__ static void run_half(cx<T>* v) { v[1] = v[0]; }
};

template <bool INV, typename T>
struct Dft<INV, 4, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
    cx<T> t2 = v[1] + v[3], t3 = mul_w4<INV>(v[1] - v[3]);
    v[0] = t0 + t2;
    v[2] = t0 - t2;
    v[1] = t1 + t3;
    v[3] = t1 - t3;
  }
  // inputs 2, 3 are zero
  __device__ __forceinline__ static void run_half(cx<T>* v) {
    cx<T> a = v[0], b = v[1], bw = mul_w4<INV>(v[1]);
    v[0] = a + b;
    v[2] = a - b;
    v[1] = a + bw;
    v[3] = a - bw;
  }
};

// (a, b) <- (a + t b, a - t b) for t = exp(-+2 pi i M/8), M = 0..3: one
// addition per component (M even), or for M odd (t = c (+-1 +- i), c =
// cos(pi/4)) two additions and four fused multiply-adds.
template <bool INV, int M, typename T>
__device__ __forceinline__ void bfly_w8(cx<T>& a, cx<T>& b) {
  if constexpr (M % 2 == 0) {
    const cx<T> tb = M == 0 ? b : mul_w4<INV>(b);
    b = a - tb;
    a = a + tb;
  } else {
    const T c = static_cast<T>(0.70710678118654752440);
    // t / c = sr + i si
    constexpr T sr = M == 1 ? 1 : -1;
    constexpr T si = INV ? 1 : -1;
    const T u = sr * b.re - si * b.im;  // re(t b) / c
    const T v = sr * b.im + si * b.re;  // im(t b) / c
    b = {fmadd(-c, u, a.re), fmadd(-c, v, a.im)};
    a = {fmadd(c, u, a.re), fmadd(c, v, a.im)};
  }
}

template <bool INV, typename T>
struct Dft<INV, 8, T> {
  // Radix 8 as three layers of radix-2 butterflies, splitting the input
  // index by its top bit first: (v_m, v_(m+4)), then (v_m, v_(m+2)) with
  // the factors 1 and W^2, then neighbours with 1, W^2, W, W^3 (W =
  // exp(-+2 pi i/8)).  The outputs y0..y7 come out in bit-reversed slots.
  __device__ __forceinline__ static void layers23(cx<T>* v) {
    bfly_w8<INV, 0>(v[0], v[2]);
    bfly_w8<INV, 0>(v[1], v[3]);
    bfly_w8<INV, 2>(v[4], v[6]);
    bfly_w8<INV, 2>(v[5], v[7]);
    bfly_w8<INV, 0>(v[0], v[1]);
    bfly_w8<INV, 2>(v[2], v[3]);
    bfly_w8<INV, 1>(v[4], v[5]);
    bfly_w8<INV, 3>(v[6], v[7]);
  }
  __device__ __forceinline__ static void natural(cx<T>* v) {
    const cx<T> y1 = v[4], y3 = v[6], y4 = v[1], y6 = v[3];
    v[1] = y1;
    v[3] = y3;
    v[4] = y4;
    v[6] = y6;
  }
  __device__ __forceinline__ static void run(cx<T>* v) {
#pragma unroll
    for (int m = 0; m < 4; ++m) bfly_w8<INV, 0>(v[m], v[m + 4]);
    layers23(v);
    natural(v);
  }
  // inputs 4..7 are zero
  __device__ __forceinline__ static void run_half(cx<T>* v) {
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m + 4] = v[m];
    layers23(v);
    natural(v);
  }
  // the DFT of (s_m v_m): the products with the first four factors, then
  // the first layer as bfly_tw with the other four
  __device__ __forceinline__ static void run_scaled(cx<T>* v, const cx<T>* sc) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      v[m] = v[m] * sc[m];
      bfly_tw(v[m], v[m + 4], sc[m + 4]);
    }
    layers23(v);
    natural(v);
  }
  // y_j = sum_m v_m w^m W^(jm) (W = exp(-+2 pi i/8)): the twiddled butterfly
  // of a Stockham stage as three layers of bfly_tw.  Splitting m by its top
  // bit gives y_(2j') from A_m = v_m + w^4 v_(m+4) and y_(2j'+1) from B_m =
  // v_m - w^4 v_(m+4), two twiddled 4-point DFTs with twiddle bases w and
  // wW; splitting again gives 2-point DFTs with twiddles w^2, w^2 W^2, w,
  // wW^2, wW and wW^3.  W^2 = -+i costs nothing, so the stage needs w, w^2,
  // w^4 and wW (forward sign; the inverse conjugates them) and 12 butterflies
  // of 6 operations, against 7 complex products and the plain butterfly.
  __device__ __forceinline__ static void run_tw(cx<T>* v, cx<T> w1, cx<T> w2, cx<T> w4, cx<T> w1w) {
    if constexpr (INV) {
      w1 = conj(w1);
      w2 = conj(w2);
      w4 = conj(w4);
      w1w = conj(w1w);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) bfly_tw(v[m], v[m + 4], w4);
    const cx<T> w2v = mul_w4<INV>(w2);
    bfly_tw(v[0], v[2], w2);
    bfly_tw(v[1], v[3], w2);
    bfly_tw(v[4], v[6], w2v);
    bfly_tw(v[5], v[7], w2v);
    bfly_tw(v[0], v[1], w1);
    bfly_tw(v[2], v[3], mul_w4<INV>(w1));
    bfly_tw(v[4], v[5], w1w);
    bfly_tw(v[6], v[7], mul_w4<INV>(w1w));
    natural(v);
  }
  // w exp(-2 pi i/8), w given with the forward sign
  __device__ __forceinline__ static cx<T> times_w8(cx<T> w) {
    const T c = static_cast<T>(0.70710678118654752440);
    return {(w.re + w.im) * c, (w.im - w.re) * c};
  }
};

template <bool INV, typename T>
struct Dft<INV, 16, T> {
  __device__ __forceinline__ static void combine(cx<T>* v, cx<T>* e, cx<T>* o) {
    o[1] = mul_w16<INV, 1>(o[1]);
    o[2] = mul_w16<INV, 2>(o[2]);
    o[3] = mul_w16<INV, 3>(o[3]);
    o[4] = mul_w16<INV, 4>(o[4]);
    o[5] = mul_w16<INV, 5>(o[5]);
    o[6] = mul_w16<INV, 6>(o[6]);
    o[7] = mul_w16<INV, 7>(o[7]);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      v[k] = e[k] + o[k];
      v[k + 8] = e[k] - o[k];
    }
  }
  __device__ __forceinline__ static void run(cx<T>* v) {
    cx<T> e[8], o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      e[k] = v[2 * k];
      o[k] = v[2 * k + 1];
    }
    Dft<INV, 8, T>::run(e);
    Dft<INV, 8, T>::run(o);
    combine(v, e, o);
  }
  __device__ __forceinline__ static void run_half(cx<T>* v) {
    cx<T> e[8] = {v[0], v[2], v[4], v[6], {}, {}, {}, {}};
    cx<T> o[8] = {v[1], v[3], v[5], v[7], {}, {}, {}, {}};
    Dft<INV, 8, T>::run_half(e);
    Dft<INV, 8, T>::run_half(o);
    combine(v, e, o);
  }
  // y_j = sum_m v_m w^m W^(jm) (W = exp(-+2 pi i/16)): splitting m by its
  // top bit gives y_(2j') from A_m = v_m + w^8 v_(m+8), a twiddled 8-point
  // DFT with base w, and y_(2j'+1) from B_m = v_m - w^8 v_(m+8), one with
  // base w exp(-2 pi i/16) (Dft<8>::run_tw for both).  Twiddles w, w^2, w^4,
  // w^8 with the forward sign (the inverse conjugates them): 8 + 24
  // butterflies of 6 operations and 4 products by constants, against 15
  // complex products (11 of them to derive the powers) and the plain
  // butterfly.
  __device__ __forceinline__ static void run_tw(cx<T>* v, cx<T> w1, cx<T> w2, cx<T> w4, cx<T> w8) {
    using D8 = Dft<INV, 8, T>;
    const cx<T> t8 = INV ? conj(w8) : w8;
#pragma unroll
    for (int m = 0; m < 8; ++m) bfly_tw(v[m], v[m + 8], t8);
    D8::run_tw(v, w1, w2, w4, D8::times_w8(w1));
    // the powers 1, 2, 4 of w exp(-2 pi i/16), and its product with exp(-2 pi i/8)
    D8::run_tw(v + 8, mul_w16<false, 1>(w1), D8::times_w8(w2), mul_w4<false>(w4), mul_w16<false, 3>(w1));
    cx<T> y[16];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      y[2 * j] = v[j];
      y[2 * j + 1] = v[8 + j];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = y[j];
  }
};

template <bool INV, typename T>
struct Dft<INV, 3, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    constexpr double C = -0.5;
    constexpr double S = 0.86602540378443864676;  // sin(2 pi / 3)
    const T sg = INV ? static_cast<T>(S) : static_cast<T>(-S);
    cx<T> s = v[1] + v[2], d = v[1] - v[2];
    cx<T> m = {fmadd(static_cast<T>(C), s.re, v[0].re), fmadd(static_cast<T>(C), s.im, v[0].im)};
    cx<T> id = {-sg * d.im, sg * d.re};  // i * sg * d
    v[0] = v[0] + s;
    v[1] = m + id;
    v[2] = m - id;
  }
};

template <bool INV, typename T>
struct Dft<INV, 5, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    constexpr double C1 = 0.30901699437494742410;   // cos(2 pi/5)
    constexpr double C2 = -0.80901699437494742410;  // cos(4 pi/5)
    constexpr double S1 = 0.95105651629515357212;   // sin(2 pi/5)
    constexpr double S2 = 0.58778525229247312917;   // sin(4 pi/5)
    const T s1 = INV ? static_cast<T>(S1) : static_cast<T>(-S1);
    const T s2 = INV ? static_cast<T>(S2) : static_cast<T>(-S2);
    const T c1 = static_cast<T>(C1), c2 = static_cast<T>(C2);
    cx<T> b1 = v[1] + v[4], b2 = v[2] + v[3];
    cx<T> d1 = v[1] - v[4], d2 = v[2] - v[3];
    cx<T> m1 = {fmadd(c2, b2.re, fmadd(c1, b1.re, v[0].re)), fmadd(c2, b2.im, fmadd(c1, b1.im, v[0].im))};
    cx<T> m2 = {fmadd(c1, b2.re, fmadd(c2, b1.re, v[0].re)), fmadd(c1, b2.im, fmadd(c2, b1.im, v[0].im))};
    // i * (s1 d1 + s2 d2) and i * (s2 d1 - s1 d2)
    cx<T> n1 = {-fmadd(s1, d1.im, s2 * d2.im), fmadd(s1, d1.re, s2 * d2.re)};
    cx<T> n2 = {-fmadd(s2, d1.im, -(s1 * d2.im)), fmadd(s2, d1.re, -(s1 * d2.re))};
    v[0] = v[0] + b1 + b2;
    v[1] = m1 + n1;
    v[4] = m1 - n1;
    v[2] = m2 + n2;
    v[3] = m2 - n2;
  }
};

// ---------------------------------------------------------------------------
// Stage bookkeeping
// ---------------------------------------------------------------------------
template <int L, bool INV, int TP = threads_per_pencil(L), int PV = 0>
struct Stages {
  static constexpr RadixPlan plan = radix_plan(L, PV);  // PV: plan variant (plan.h)
  static constexpr int NS = plan.n;
  static constexpr int TPP = TP;  // threads per pencil
  static constexpr int radix(int s) { return INV ? plan.r[NS - 1 - s] : plan.r[s]; }
  static constexpr int ns(int s) {  // product of the radices before stage s
    int p = 1;
    for (int i = 0; i < s; ++i) p *= radix(i);
    return p;
  }
  static constexpr int nbf(int s) { return L / radix(s); }            // butterflies per pencil
  static constexpr int cnt(int s) { return (nbf(s) + TPP - 1) / TPP; }  // per thread
  static constexpr bool radices_ok() {
    for (int s = 0; s < NS; ++s) {
      int r = plan.r[s];
      if (r != 2 && r != 3 && r != 4 && r != 5 && r != 8 && r != 16) return false;
    }
    return true;
  }
  static_assert(NS > 0 && ns(NS) == L && radices_ok(), "plan must factor L into radices 2, 3, 4, 5, 8, 16");
  // Largest twiddle table index any stage reads: the powers r = 1, 2, 4, 8
  // below R of w^(k TS), k < ns(s), TS = L / (ns(s) R).  Below L/2 when every
  // radix is a power of two, so a table staged in LDS can stop there.
  static constexpr int max_twiddle_index() {
    int m = 0;
    for (int s = 1; s < NS; ++s) {
      const int R = radix(s), TS = L / (ns(s) * R);
      int p = 1;
      while (p * 2 < R) p *= 2;
      const int v = p * (ns(s) - 1) * TS;
      if (v > m) m = v;
    }
    return m;
  }
};

// One thread's view of its pencil in LDS.  Strided passes interleave NP
// pencils element by element (element e at base[e * es], es = NP): every
// LDS access of a wavefront is then a run of NP consecutive slots.  Contiguous
// passes keep each pencil in one row with one padding slot after every 8
// elements (element e at base[e + e / 8]), which breaks the power-of-two
// strides of the Stockham writes across the LDS banks.
//
// Narrow interleaves (NP pencils of fewer than 128 bytes per element row)
// add one padding row after every 8 rows (element e at base[(e + e/8) es],
// pad = 1).  A group of lanes served together then spans two butterflies b
// and b + 1 of its NP pencils: their rows differ by 1 in every read and in
// every write after the first stage, and by the radix R = 8 in the first
// stage's writes, which the padding turns into 9 -- an odd number of rows,
// so the two runs fall on disjoint banks instead of the same ones.  Every
// offset between the accesses of one thread stays a compile-time constant.
template <typename T>
struct LdsPencil {
  cx<T>* base;
  int es;   // 0: padded contiguous row; otherwise the interleave stride
  int pad;  // interleave: one padding row after every 8 rows
  __device__ __forceinline__ cx<T>& at(int e) const {
    return es ? base[(pad ? e + (e >> 3) : e) * es] : base[e + (e >> 3)];
  }
  // Element b + C for a compile-time C.  SPLIT: the caller guarantees
  // (b + C) / 8 = b / 8 + C / 8 (C a multiple of 8, or b % 8 + C % 8 < 8),
  // so the padded position is the thread's own b + b / 8 plus a constant,
  // and every access of a butterfly shares one address register.
  template <int C, bool SPLIT>
  __device__ __forceinline__ cx<T>& at(int b) const {
    if (es && !pad) return base[(b + C) * es];
    const int row = SPLIT ? b + (b >> 3) + (C + (C >> 3)) : (b + C) + ((b + C) >> 3);
    return es ? base[row * es] : base[row];
  }
};

// LDS slots of one padded contiguous pencil row
constexpr int padded_row(int L) { return L + L / 8; }
// LDS rows of an interleave of length L, with or without the padding rows
constexpr int interleave_rows(int L, bool pad) { return pad ? L + L / 8 : L; }

enum Keep : int { KEEP_ALL = 0, KEEP_HALF = 1, KEEP_HALF1 = 2 };

// Stage data: cnt(s) butterflies of radix(s) complex values.
template <typename T, int C, int R>
struct Regs {
  cx<T> v[C][R];
};

// TWM selects where the twiddles of a stage come from:
//  0: tw is the length-L table exp(-2 pi i m / L); the powers w, w^2, w^4,
//     w^8 are read, the other powers are products of two of them;
//  1: tw is the stage-major table (stage_table): every twiddle a stage
//     uses is read, no products (fewer vector instructions, more table);
//  2: tw is the stage-major table of the powers of two only: w, w^2, w^4,
//     w^8 are read, the others are products as in 0.  The lanes of a
//     wavefront read adjacent entries (in the length-L table a stage with
//     few butterflies reads entries TS apart, which share LDS banks), and
//     the table holds only what the stages read.
// A radix-8 stage with twiddles runs Dft<8>::run_tw, which uses w, w^2, w^4
// and w exp(-2 pi i/8): the last is a table entry in mode 1 (entry
// k TS + L/8 of the length-L table) and a product by a constant otherwise.
template <typename T, int L, bool INV, int TP = threads_per_pencil(L), int PV = 0, int TWM = 0>
struct Engine {
  using St = Stages<L, INV, TP, PV>;
  static constexpr int NS = St::NS;
  static constexpr int TPP = St::TPP;

  // Stage-major twiddle table: stage s >= 1 holds w^(r k TS) for the powers
  // r it reads (TWM 1: r = 1..R-1, or for R = 8 the powers 1, 2, 4 and then
  // w exp(-2 pi i/8); TWM 2: r = 1, 2, 4, 8 below R) and k < ns(s) (TS = L /
  // (ns(s) R)), power by power: the q-th power read at stage_offset(s) +
  // q ns(s) + k, forward sign (the inverse conjugates on use).  Consecutive
  // k of one r are adjacent, so the lanes of a wavefront read adjacent
  // entries.
  static constexpr int powers_read(int R) {
    if (TWM == 1) return R == 8 ? 4 : R - 1;
    int c = 0;
    for (int r = 1; r < R; r *= 2) ++c;
    return c;
  }
  static constexpr int stage_offset(int s) {
    int o = 0;
    for (int q = 1; q < s; ++q) o += powers_read(St::radix(q)) * St::ns(q);
    return o;
  }
  static constexpr int stage_table_size() { return stage_offset(NS); }

  // Fill the stage-major table from the length-L table (every thread of the
  // workgroup takes entries tid, tid + nthreads, ... of each stage).
  __device__ __forceinline__ static void build_stage_table(cx<T>* dst, const cx<T>* __restrict__ tw_full, int tid,
                                                           int nthreads) {
    unroll<NS>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      if constexpr (q >= 1) {
        constexpr int nsq = St::ns(q), R = St::radix(q), TS = L / (nsq * R);
        for (int idx = tid; idx < powers_read(R) * nsq; idx += nthreads) {
          const int p = idx / nsq, k = idx % nsq;
          int e;
          if (TWM == 1 && R == 8)
            e = p < 3 ? (k * TS) << p : k * TS + L / 8;
          else
            e = (TWM == 2 ? 1 << p : p + 1) * k * TS;
          dst[stage_offset(q) + idx] = tw_full[e];
        }
      }
    });
  }

  template <int s>
  using RegsOf = Regs<T, St::cnt(s), St::radix(s)>;

  // Twiddles w^r, r = 1..R-1, of butterfly b in stage s, w = exp(-2 pi i k / (Ns R)),
  // k = b mod Ns: the powers r = 1, 2, 4, 8 come from the table, the others
  // are products of two of them (a few ulps), which cuts the table loads from
  // R - 1 to log2 R per butterfly.
  template <int R, int TS>
  __device__ __forceinline__ static void twiddles(cx<T> (&w)[R], int k, const cx<T>* __restrict__ tw) {
#pragma unroll
    for (int r = 1; r < R; ++r) {
      if ((r & (r - 1)) == 0) {
        w[r] = tw[r * k * TS];
      } else {
        const int low = r & -r;
        w[r] = w[r - low] * w[low];
      }
    }
  }

  // twiddle + butterfly of stage s, in registers
  template <int s, bool HALF_IN>
  __device__ __forceinline__ static void compute(RegsOf<s>& g, int bt, const cx<T>* __restrict__ tw) {
    constexpr int R = St::radix(s);
    constexpr int NSs = St::ns(s);
    constexpr int TS = L / (NSs * R);
#pragma unroll
    for (int i = 0; i < St::cnt(s); ++i) {
      const int b = bt + i * TPP;
      if (St::nbf(s) % TPP != 0 && b >= St::nbf(s)) continue;
      if constexpr (NSs > 1 && R == 8) {
        const int k = b % NSs;
        cx<T> w1, w2, w4, w1w;
        if constexpr (TWM == 1 || TWM == 2) {
          constexpr int o = stage_offset(s);
          w1 = tw[o + k];
          w2 = tw[o + NSs + k];
          w4 = tw[o + 2 * NSs + k];
          if constexpr (TWM == 1) w1w = tw[o + 3 * NSs + k];
        } else {
          w1 = tw[k * TS];
          w2 = tw[2 * k * TS];
          w4 = tw[4 * k * TS];
        }
        if constexpr (TWM != 1) w1w = Dft<INV, 8, T>::times_w8(w1);
        Dft<INV, 8, T>::run_tw(g.v[i], w1, w2, w4, w1w);
        continue;
      }
      if constexpr (NSs > 1 && R == 16) {
        const int k = b % NSs;
        cx<T> w1, w2, w4, w8;
        if constexpr (TWM == 1 || TWM == 2) {
          // the powers 1, 2, 4, 8: positions 0, 1, 2, 3 of the powers of two
          // (TWM 2) or 0, 1, 3, 7 of every power (TWM 1)
          constexpr int o = stage_offset(s);
          constexpr int q4 = TWM == 2 ? 2 : 3, q8 = TWM == 2 ? 3 : 7;
          w1 = tw[o + k];
          w2 = tw[o + NSs + k];
          w4 = tw[o + q4 * NSs + k];
          w8 = tw[o + q8 * NSs + k];
        } else {
          w1 = tw[k * TS];
          w2 = tw[2 * k * TS];
          w4 = tw[4 * k * TS];
          w8 = tw[8 * k * TS];
        }
        Dft<INV, 16, T>::run_tw(g.v[i], w1, w2, w4, w8);
        continue;
      }
      if constexpr (NSs > 1) {
        const int k = b % NSs;
        cx<T> w[R];
        if constexpr (TWM == 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) w[r] = tw[stage_offset(s) + (r - 1) * NSs + k];
        } else if constexpr (TWM == 2) {
#pragma unroll
          for (int r = 1, q = 0; r < R; ++r) {
            if ((r & (r - 1)) == 0) {
              w[r] = tw[stage_offset(s) + q * NSs + k];
              ++q;
            } else {
              const int low = r & -r;
              w[r] = w[r - low] * w[low];
            }
          }
        } else {
          twiddles<R, TS>(w, k, tw);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) g.v[i][r] = twiddle<INV>(g.v[i][r], w[r]);
      }
      if constexpr (HALF_IN && s == 0 && (R % 2 == 0)) {
        Dft<INV, R, T>::run_half(g.v[i]);
      } else {
        Dft<INV, R, T>::run(g.v[i]);
      }
    }
  }

  // outputs of stage s -> LDS (Stockham positions)
  template <int s>
  __device__ __forceinline__ static void write_lds(const RegsOf<s>& g, int bt, LdsPencil<T> p) {
    constexpr int R = St::radix(s);
    constexpr int NSs = St::ns(s);
#pragma unroll
    for (int i = 0; i < St::cnt(s); ++i) {
      const int b = bt + i * TPP;
      if (St::nbf(s) % TPP != 0 && b >= St::nbf(s)) continue;
      const int k = b % NSs;
      const int base = (b - k) * R + k;
      // (base + j NSs) / 8 splits when NSs is a multiple of 8, or in the
      // first stage (NSs = 1, base = b R) for a power-of-two R
      constexpr bool SPLIT = NSs % 8 == 0 || (NSs == 1 && (R & (R - 1)) == 0);
      unroll<R>([&](auto J) {
        constexpr int j = decltype(J)::value;
        p.template at<j * NSs, SPLIT>(base) = g.v[i][j];
      });
    }
  }

  // inputs of stage s <- LDS
  template <int s>
  __device__ __forceinline__ static void read_lds(RegsOf<s>& g, int bt, LdsPencil<T> p) {
    constexpr int R = St::radix(s);
    constexpr int STRIDE = L / R;
#pragma unroll
    for (int i = 0; i < St::cnt(s); ++i) {
      const int b = bt + i * TPP;
      if (St::nbf(s) % TPP != 0 && b >= St::nbf(s)) continue;
      unroll<R>([&](auto J) {
        constexpr int r = decltype(J)::value;
        g.v[i][r] = p.template at<r * STRIDE, STRIDE % 8 == 0>(b);
      });
    }
  }

  // Stage 0 inputs from a functor: load(e) for e = b + r L/R0.  With HALF_IN
  // the upper half (e >= L/2) is zero and never loaded.
  template <bool HALF_IN, class Load>
  __device__ __forceinline__ static void load_first(RegsOf<0>& g, int bt, Load&& load) {
    constexpr int R = St::radix(0);
    constexpr int STRIDE = L / R;
    constexpr bool SKIP = HALF_IN && (R % 2 == 0);
#pragma unroll
    for (int i = 0; i < St::cnt(0); ++i) {
      const int b = bt + i * TPP;
      if (St::nbf(0) % TPP != 0 && b >= St::nbf(0)) continue;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (SKIP && r >= R / 2) {
          g.v[i][r] = cx<T>{};
        } else if (HALF_IN && !SKIP) {
          const int e = b + r * STRIDE;
          g.v[i][r] = e < L / 2 ? load(e) : cx<T>{};
        } else {
          g.v[i][r] = load(b + r * STRIDE);
        }
      }
    }
  }

  // The same loads with the index of each value in the thread's registers:
  // load(slot, e), slot = i * R0 + r (a compile-time constant once unrolled).
  template <bool HALF_IN, class Load>
  __device__ __forceinline__ static void load_first_slots(RegsOf<0>& g, int bt, Load&& load) {
    constexpr int R = St::radix(0);
    constexpr int STRIDE = L / R;
    constexpr bool SKIP = HALF_IN && (R % 2 == 0);
#pragma unroll
    for (int i = 0; i < St::cnt(0); ++i) {
      const int b = bt + i * TPP;
      if (St::nbf(0) % TPP != 0 && b >= St::nbf(0)) continue;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (SKIP && r >= R / 2) {
          g.v[i][r] = cx<T>{};
        } else if (HALF_IN && !SKIP) {
          const int e = b + r * STRIDE;
          g.v[i][r] = e < L / 2 ? load(i * R + r, e) : cx<T>{};
        } else {
          g.v[i][r] = load(i * R + r, b + r * STRIDE);
        }
      }
    }
  }

  // Every element index e that load_first<HALF_IN> reads, with its slot:
  // f(slot, e) (slots as in load_first_slots).
  template <bool HALF_IN, class F>
  __device__ __forceinline__ static void first_slots(int bt, F&& f) {
    constexpr int R = St::radix(0);
    constexpr int STRIDE = L / R;
#pragma unroll
    for (int i = 0; i < St::cnt(0); ++i) {
      const int b = bt + i * TPP;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = b + r * STRIDE;
        if (HALF_IN && (R % 2 == 0) && r >= R / 2) continue;
        f(i * R + r, e);
      }
    }
  }

  // Last-stage outputs to a functor: store(e, value) for e = b + j L/R_last.
  // KEEP selects the outputs: KEEP_ALL, KEEP_HALF (e < L/2: the discarded
  // half of a padded inverse is never written) or KEEP_HALF1 (e <= L/2: the
  // octant of an even sequence).
  template <int KEEP, class Store>
  __device__ __forceinline__ static void store_last(const RegsOf<NS - 1>& g, int bt, Store&& store) {
    constexpr int s = NS - 1;
    constexpr int R = St::radix(s);
    constexpr int STRIDE = L / R;
#pragma unroll
    for (int i = 0; i < St::cnt(s); ++i) {
      const int b = bt + i * TPP;
      if (St::nbf(s) % TPP != 0 && b >= St::nbf(s)) continue;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int e = b + j * STRIDE;
        if (KEEP == KEEP_HALF && (R % 2 == 0) && j >= R / 2) continue;
        if (KEEP == KEEP_HALF && e >= L / 2) continue;
        if (KEEP == KEEP_HALF1 && e > L / 2) continue;
        store(e, g.v[i][j]);
      }
    }
  }

  // The same stores with the slot of each value: store(slot, e, value),
  // slot = i * R_last + j.
  template <int KEEP, class Store>
  __device__ __forceinline__ static void store_last_slots(const RegsOf<NS - 1>& g, int bt, Store&& store) {
    constexpr int s = NS - 1;
    constexpr int R = St::radix(s);
    constexpr int STRIDE = L / R;
#pragma unroll
    for (int i = 0; i < St::cnt(s); ++i) {
      const int b = bt + i * TPP;
      if (St::nbf(s) % TPP != 0 && b >= St::nbf(s)) continue;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int e = b + j * STRIDE;
        if (KEEP == KEEP_HALF && (R % 2 == 0) && j >= R / 2) continue;
        if (KEEP == KEEP_HALF && e >= L / 2) continue;
        if (KEEP == KEEP_HALF1 && e > L / 2) continue;
        store(i * R + j, e, g.v[i][j]);
      }
    }
  }

  // Every element index e that store_last<KEEP> may write (bounds on b
  // aside), with its slot: f(slot, e).
  template <int KEEP, class F>
  __device__ __forceinline__ static void last_slots(int bt, F&& f) {
    constexpr int s = NS - 1;
    constexpr int R = St::radix(s);
    constexpr int STRIDE = L / R;
#pragma unroll
    for (int i = 0; i < St::cnt(s); ++i) {
      const int b = bt + i * TPP;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (KEEP == KEEP_HALF && (R % 2 == 0) && j >= R / 2) continue;
        f(i * R + j, b + j * STRIDE);
      }
    }
  }

  // Run stages s..NS-1 starting from inputs already in LDS; hand the last
  // stage's outputs (natural order, element b + j L/R) to fin(regs).
  template <int s, class Fin>
  __device__ __forceinline__ static void run_from_lds(int bt, LdsPencil<T> p, const cx<T>* __restrict__ tw,
                                                      Fin&& fin) {
    RegsOf<s> g;
    read_lds<s>(g, bt, p);
    __syncthreads();
    compute<s, false>(g, bt, tw);
    if constexpr (s + 1 < NS) {
      write_lds<s>(g, bt, p);
      __syncthreads();
      run_from_lds<s + 1>(bt, p, tw, fin);
    } else {
      fin(g);
    }
  }

  // The whole transform of the elementwise product of g0 and sc (both laid
  // out as stage 0's registers): for radix 8 the products are folded into
  // the first butterfly layer (Dft<8>::run_scaled).  fin as in run.
  template <class Fin>
  __device__ __forceinline__ static void run_scaled(RegsOf<0>& g0, const RegsOf<0>& sc, int bt, LdsPencil<T> p,
                                                    const cx<T>* __restrict__ tw, Fin&& fin) {
    constexpr int R = St::radix(0);
#pragma unroll
    for (int i = 0; i < St::cnt(0); ++i) {
      const int b = bt + i * TPP;
      if (St::nbf(0) % TPP != 0 && b >= St::nbf(0)) continue;
      if constexpr (R == 8) {
        Dft<INV, 8, T>::run_scaled(g0.v[i], sc.v[i]);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) g0.v[i][r] = g0.v[i][r] * sc.v[i][r];
        Dft<INV, R, T>::run(g0.v[i]);
      }
    }
    if constexpr (NS > 1) {
      write_lds<0>(g0, bt, p);
      __syncthreads();
      run_from_lds<1>(bt, p, tw, fin);
    } else {
      fin(g0);
    }
  }

  // Whole transform: stage 0 from registers g0 (already loaded), the rest
  // through LDS; fin(regs of the last stage).
  template <bool HALF_IN, class Fin>
  __device__ __forceinline__ static void run(RegsOf<0>& g0, int bt, LdsPencil<T> p,
                                             const cx<T>* __restrict__ tw, Fin&& fin) {
    compute<0, HALF_IN>(g0, bt, tw);
    if constexpr (NS > 1) {
      write_lds<0>(g0, bt, p);
      __syncthreads();
      run_from_lds<1>(bt, p, tw, fin);
    } else {
      fin(g0);
    }
  }
};

}  // namespace ori
