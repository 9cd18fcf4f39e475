// FFT pass kernels for one padded length L (compiled once per L with
// -DORI_L=<L>).
//
// One product with the Green's matrix (Section 3: eq. 3.3.4 as the 3-D
// convolution of eq. 3.3.7, evaluated by eq. 3.3.8 on a grid padded to
// L = 2n per axis) is five passes over the data:
//
//   F1  contiguous axis i3, forward; prologue p = r + beta p, v = S p; input
//       n of L per pencil (the zero padding is never read)       n*n pencils
//   F2  axis i2, forward, input n of L                            n*L pencils
//   Z   axis i1: forward, times the kernel spectrum, inverse,
//       keep n                                                     L*L pencils
//   I2  axis k2, inverse, keep n                                  n*L pencils
//   I1  contiguous axis k3, inverse, keep n; epilogue
//       q = p + S conv and the bilinear partials p^T q             n*n pencils
//
// The work arrays are  A[i1][i2][k3]  (n*n*L)  and  B[i1][k2][k3]  (n*L*L).
// L is the padded length of the plan; any n with 2n - 1 <= L gives the
// linear convolution (offsets lie in (-n, n)).  Kernels with EX = true take
// n = L/2 exactly; EX = false guards every read and write at n.
#include "fft_engine.h"
#include "kernels.h"
#include "launch.h"

#ifndef ORI_L
#error "compile once per padded length with -DORI_L=<L>"
#endif

namespace ori {
namespace {

constexpr int L = ORI_L;
constexpr int TPP = threads_per_pencil(L);
constexpr int NPC = pencils_contig(L);
constexpr int BLOCK_C = NPC * TPP;
template <typename T>
constexpr int nps() {
  return pencils_strided(L, int(sizeof(cx<T>)));
}
template <typename T>
constexpr int block_s() {
  return nps<T>() * TPP;
}

__host__ __device__ __forceinline__ int64_t contig_blocks_per_rhs(int64_t ppr) { return (ppr + NPC - 1) / NPC; }

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

// ---------------------------------------------------------------------------
// F1 (and the first spectrum pass): contiguous forward with prologue
// ---------------------------------------------------------------------------
template <typename V, typename T, bool EX>
__global__ void __launch_bounds__(BLOCK_C) k_contig_fwd(ContigFwdArgs a) {
  __shared__ cx<T> lds[NPC * padded_row(L)];
  using E = Engine<T, L, false>;
  const int tid = threadIdx.x;
  const int bt = tid % TPP, t = tid / TPP;
  const int64_t bpr = contig_blocks_per_rhs(a.ppr);
  const int64_t rhs = blockIdx.x / bpr;
  const int64_t lp_id = (blockIdx.x % bpr) * NPC + t;  // pencil within its right-hand side
  const bool act = lp_id < a.ppr;
  const int64_t pid = rhs * a.ppr + lp_id;
  const cx<T>* __restrict__ tw = static_cast<const cx<T>*>(a.tw);
  const cx<V>* __restrict__ x = static_cast<const cx<V>*>(a.x);
  cx<V>* pv = static_cast<cx<V>*>(a.pvec);
  const cx<V>* __restrict__ s = static_cast<const cx<V>*>(a.s_in);
  cx<T>* __restrict__ out = static_cast<cx<T>*>(a.out);
  const int64_t ib = pid * a.in_pitch;
  const int64_t db = lp_id * a.in_pitch;  // shared diagonal
  const int64_t ob = pid * a.out_pitch;
  cx<V>* xv = static_cast<cx<V>*>(a.xvec);
  cx<double> beta = {0.0, 0.0}, alpha = {0.0, 0.0};
  if (a.mode == 1 && !a.first) {
    beta = cx<double>{a.sc[rhs].beta_re, a.sc[rhs].beta_im};
    alpha = cx<double>{a.sc[rhs].alpha_re, a.sc[rhs].alpha_im};
  }
  const bool x_moves = xv && (alpha.re != 0.0 || alpha.im != 0.0);

  auto load = [&](int e) -> cx<T> {
    if (!act) return cx<T>{};
    if constexpr (!EX) {
      if (e >= a.in_pitch) return cx<T>{};  // zero padding between n and L/2
    }
    const int64_t i = ib + e;
    cx<double> v;
    if (a.mode == 1) {
      v = cvt<double>(x[i]);
      if (!a.first) {
        const cx<double> po = cvt<double>(pv[i]);
        // the previous iteration's x += alpha p, folded into this pass
        if (x_moves) xv[i] = cvt<V>(cvt<double>(xv[i]) + alpha * po);
        v = v + beta * po;
      }
      pv[i] = cvt<V>(v);
    } else {
      v = cvt<double>(x[i]);
    }
    if (s) v = v * cvt<double>(s[db + e]);
    return cvt<T>(v);
  };
  typename E::template RegsOf<0> g;
  E::template load_first<true>(g, bt, load);
  LdsPencil<T> lp{lds + t * padded_row(L), 0};
  E::template run<true>(g, bt, lp, tw, [&](auto& gl) {
    E::template store_last<KEEP_ALL>(gl, bt, [&](int e, cx<T> v) {
      if (act) out[ob + e] = v;
    });
  });
}

// ---------------------------------------------------------------------------
// I1: contiguous inverse, keep e < out_pitch (= n), epilogue and partials
// ---------------------------------------------------------------------------
template <typename V, typename T, bool EX>
__global__ void __launch_bounds__(BLOCK_C) k_contig_inv(ContigInvArgs a) {
  __shared__ cx<T> lds[NPC * padded_row(L)];
  using E = Engine<T, L, true>;
  const int tid = threadIdx.x;
  const int bt = tid % TPP, t = tid / TPP;
  const int64_t bpr = contig_blocks_per_rhs(a.ppr);
  const int64_t rhs = blockIdx.x / bpr;
  const int64_t lp_id = (blockIdx.x % bpr) * NPC + t;
  const bool act = lp_id < a.ppr;
  const int64_t pid = rhs * a.ppr + lp_id;
  const cx<T>* __restrict__ tw = static_cast<const cx<T>*>(a.tw);
  const cx<T>* __restrict__ in = static_cast<const cx<T>*>(a.in);
  cx<V>* __restrict__ y = static_cast<cx<V>*>(a.y);
  const cx<V>* __restrict__ a0 = static_cast<const cx<V>*>(a.a0);
  const cx<V>* __restrict__ a1 = static_cast<const cx<V>*>(a.a1);
  const cx<V>* __restrict__ so = static_cast<const cx<V>*>(a.s_out);
  const int64_t ib = pid * a.in_pitch;
  const int64_t ob = pid * a.out_pitch;
  const int64_t db = lp_id * a.out_pitch;  // shared diagonal
  double acc[4] = {0.0, 0.0, 0.0, 0.0};

  auto load = [&](int e) -> cx<T> { return act ? in[ib + e] : cx<T>{}; };
  typename E::template RegsOf<0> g;
  E::template load_first<false>(g, bt, load);
  LdsPencil<T> lp{lds + t * padded_row(L), 0};
  E::template run<false>(g, bt, lp, tw, [&](auto& gl) {
    E::template store_last<KEEP_HALF>(gl, bt, [&](int e, cx<T> c) {
      if (!act) return;
      if constexpr (!EX) {
        if (e >= a.out_pitch) return;
      }
      const int64_t i = ob + e;
      cx<double> conv = cvt<double>(c);
      if (so) conv = conv * cvt<double>(so[db + e]);
      cx<double> yv = scale(conv, a.cc);
      cx<double> av = {0.0, 0.0};
      if (a0) {
        av = cvt<double>(a0[i]);
        yv = yv + scale(av, a.c0);
      }
      if (a1) yv = yv + scale(cvt<double>(a1[i]), a.c1);
      y[i] = cvt<V>(yv);
      if (a.partials) {
        const cx<double> d = a.dot_self ? yv * yv : av * yv;
        acc[0] += d.re;
        acc[1] += d.im;
        acc[2] += norm2(yv);
        acc[3] += norm2(av);
      }
    });
  });
  if (a.partials) block_partials<BLOCK_C>(acc, lds, a.partials + 4 * static_cast<int64_t>(blockIdx.x));
}

// ---------------------------------------------------------------------------
// F2 / I2: strided axis, NP adjacent pencils per workgroup
// ---------------------------------------------------------------------------
// Workgroups go round-robin over the 8 XCDs (workgroup b runs on XCD b % 8,
// each XCD with its own L2).  xcd_order renumbers them so that each XCD walks
// one contiguous range of tiles: neighbouring tiles, which share cache lines
// and spectrum rows, then meet in the same L2.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t G) {
  constexpr int64_t X = 8;
  const int64_t q = G / X, r = G % X, x = b % X, j = b / X;
  return x * q + (x < r ? x : r) + j;
}

template <typename T, int NP, bool INV, bool HIN, bool HOUT, bool EX>
__global__ void __launch_bounds__(NP * TPP) k_strided(StridedArgs a) {
  constexpr bool PADL = NP * int(sizeof(cx<T>)) < 128 && L <= 512;  // narrow interleave: padding rows (LdsPencil)
  __shared__ cx<T> lds[NP * interleave_rows(L, PADL)];
  using E = Engine<T, L, INV>;
  const int tid = threadIdx.x;
  const int t = tid % NP, bt = tid / NP;
  const int64_t CT = (a.C + NP - 1) / NP;
  const int64_t w = xcd_order(blockIdx.x, gridDim.x);
  const int64_t o = w / CT;
  const int64_t c = (w % CT) * NP + t;
  const bool act = c < a.C;
  // complex64: the twiddles are staged in LDS (measured faster; for
  // complex128 the extra LDS traffic costs more than the loads it saves)
  constexpr bool TW_LDS = sizeof(T) == 4;
  __shared__ cx<T> twl[TW_LDS ? L : 1];
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw);
  if constexpr (TW_LDS) {
    for (int i = tid; i < L; i += NP * TPP) twl[i] = tw[i];
    tw = twl;  // first read after the first exchange barrier
  }
  const cx<T>* in = static_cast<const cx<T>*>(a.in);
  cx<T>* out = static_cast<cx<T>*>(a.out);
  const int64_t ib = two_level(o, a.in_lg, a.in_hi, a.in_lo) + c;
  const int64_t ob = two_level(o, a.out_lg, a.out_hi, a.out_lo) + c;

  auto load = [&](int e) -> cx<T> {
    if constexpr (HIN && !EX) {
      if (e >= a.nv) return cx<T>{};
    }
    return act ? in[ib + e * a.in_axis] : cx<T>{};
  };
  typename E::template RegsOf<0> g;
  E::template load_first<HIN>(g, bt, load);
  LdsPencil<T> lp{lds + t, NP, PADL ? 1 : 0};
  E::template run<HIN>(g, bt, lp, tw, [&](auto& gl) {
    E::template store_last<HOUT ? KEEP_HALF : KEEP_ALL>(gl, bt, [&](int e, cx<T> v) {
      if constexpr (HOUT && !EX) {
        if (e >= a.nv) return;
      }
      if (act) out[ob + e * a.out_axis] = v;
    });
  });
}

// ---------------------------------------------------------------------------
// Z: forward along i1 (n inputs), times the spectrum, inverse, keep n
// ---------------------------------------------------------------------------
// The spectrum is even along every axis, so the pencils (k2, k3) and
// (L - k2, k3) multiply by the same values K(m1, m2, k3), m = min(k, L - k).
// A workgroup takes the octant row m2 and a tile of NP consecutive k3: it
// loads its K values once into registers (the shape of the last forward
// stage, so element e = b + j L/R of the transform meets K(min(e, L-e), m2,
// k3) in place) and runs the tiles (k2 = m2 | L - m2) x (the right-hand
// sides of its slice: small grids split a batch over several workgroups)
// one after the other (with PF, the loads of the next tile are issued before
// the current one is transformed).  The spectrum is read from its octant: the
// tiles k3 and L - k3 of a row m2 need the same values; the workgroups of a
// row take the tiles in the order 0, last, 1, last - 1, ... so that the two
// run back to back on one XCD and the second read is served by its L2.
//
// Threads per pencil of the Z pass: the length's default, except at
// L >= 1024, where one wavefront per pencil (two butterflies per thread)
// measured faster than two: complex128 6.6 vs 6.9 ms (it spills on two),
// complex64 on narrow tiles 3.9 vs 4.6 ms at n = 512.
template <typename T>
constexpr int z_tpp() {
  return (L >= 1024 && TPP > 64) ? 64 : TPP;
}

// Waves per SIMD that the register allocation must allow.  At L = 512 the
// complex64 pass on 512-thread workgroups (default plan) fits three
// workgroups per CU within 80 VGPRs: 0.366 vs 0.441 ms at n = 256 when it
// needed 81 (it now needs 61, and four workgroups fit its LDS).  The
// alternative plan would spill under that bound and gets none.
template <typename T, int NP, bool PF, int PV>
constexpr int z_min_waves() {
  if (L == 512 && sizeof(T) == 4 && !PF && PV == 0 && NP * z_tpp<T>() == 512) return 6;
  return 1;
}

// Twiddle source of the Z pass (fft_engine.h, TWM): the complex64 pass is
// bound by vector instructions, so up to L = 512 it reads every power of
// each twiddle from a stage-major table in LDS instead of multiplying two
// of them; the complex128 pass reads the powers of two from a stage-major
// table (its LDS is full: that table is smaller than the entries of the
// length-L table below the largest index read, and its lanes read adjacent
// entries where the length-L table has them TS apart, on shared banks).
template <typename T>
constexpr int z_twm() {
  if (L > 512) return 0;
  return sizeof(T) == 4 ? 1 : 2;
}

template <typename T, int PV>
using ZRegs = typename Engine<T, L, false, z_tpp<T>(), PV, z_twm<T>()>::template RegsOf<
    Stages<L, false, z_tpp<T>(), PV>::NS - 1>;

// The Z pass's plan variants (plan.h) keep the threads per pencil of the
// length's default plan, so that its workgroup shape does not depend on the
// plan.
static_assert(L >= 1024 || threads_per_pencil(L, 1) == threads_per_pencil(L), "Z plan variant changes the tile");

// log2 of the largest power of two that divides every C of the elements
// bt + C a thread reads in the first forward stage and writes in the last
// inverse stage of the Z pass (the inverse ends with the radix the forward
// transform starts with; only the lower half of either is touched).  With
// the B layout's i1 block 2^e_lg no larger, element bt + C lies a fixed
// (C >> e_lg) e_hi elements after element bt for every lane.
template <typename T, int PV>
constexpr int z_align_lg() {
  using St = Stages<L, false, z_tpp<T>(), PV>;
  constexpr int R = St::radix(0), STRIDE = L / R;
  int lg = 30;
  for (int i = 0; i < St::cnt(0); ++i)
    for (int r = 0; r < (R % 2 == 0 ? R / 2 : R); ++r) {
      const int c = i * St::TPP + r * STRIDE;
      int z = 0;
      while (c != 0 && ((c >> z) & 1) == 0) ++z;
      if (c != 0 && z < lg) lg = z;
    }
  return lg;
}

// SOFF: every element of a tile is addressed as one per-lane 32-bit offset
// plus a scalar one (L <= 512, e_lg <= z_align_lg); otherwise each thread
// addresses its elements from its own base in 64 bits.  PV: the radix plan
// (plan.h, radix_plan(L, PV)).
template <typename T, int NP, bool PF, bool EX, bool SOFF, int PV>
__global__ void __launch_bounds__(NP * z_tpp<T>(), (z_min_waves<T, NP, PF, PV>())) k_zpass(ZArgs a) {
  constexpr int half = L / 2;
  constexpr int ZT = z_tpp<T>();
  constexpr int TWM = z_twm<T>();
  using EF = Engine<T, L, false, ZT, PV, TWM>;
  using EI = Engine<T, L, true, ZT, PV, TWM>;
  using St = Stages<L, false, ZT, PV>;
  using G0 = typename EF::template RegsOf<0>;
  constexpr int SL = St::NS - 1;
  constexpr int RL = St::radix(SL);
  constexpr int STRIDE = L / RL;
  constexpr int64_t CT = (L + NP - 1) / NP;
  // NP interleaved pencils, with padding rows when a row of the interleave
  // is narrower than 128 bytes (the lanes served together then span two
  // butterflies; see LdsPencil).  Up to L = 512 only: longer pencils give a
  // thread several butterflies per stage, whose padded rows each take an
  // address register (at L = 1024 the pass then loses occupancy).
  constexpr bool PADL = NP * int(sizeof(cx<T>)) < 128 && L <= 512;
  __shared__ cx<T> lds[NP * interleave_rows(L, PADL)];
  const int tid = threadIdx.x;
  const int t = tid % NP, bt = tid / NP;
  // workgroup w takes right-hand-side slice w % RS of the tile w / RS, so the
  // slices of a tile, which read the same spectrum values, run side by side
  const uint32_t RS = static_cast<uint32_t>(a.rhs_slices);
  const uint32_t w = static_cast<uint32_t>(xcd_order(blockIdx.x, gridDim.x));
  const uint32_t wt = RS == 1 ? w : w / RS;
  const uint32_t slice = w - wt * RS;
  const int64_t m2 = wt / CT;
  // tiles of a row in the order 0, CT-1, 1, CT-2, ...: a tile and its mirror
  // (which reads the same spectrum values) run back to back
  const int64_t j = wt % CT;
  const int64_t tile = (j & 1) ? CT - 1 - (j >> 1) : (j >> 1);
  const int64_t k3 = tile * NP + t;
  const bool act = k3 < L;
  const int64_t m3 = k3 <= L - k3 ? k3 : L - k3;  // the octant holds k3 and its mirror
  const uint32_t nrhs = static_cast<uint32_t>(a.nrhs);
  const uint32_t rper = RS == 1 ? nrhs : (nrhs + RS - 1) / RS;
  const int64_t r_lo = static_cast<int64_t>(slice) * rper;
  const int64_t r_hi = r_lo + rper < a.nrhs ? r_lo + rper : a.nrhs;
  const cx<T>* __restrict__ kh = static_cast<const cx<T>*>(a.khat);
  // The twiddles are staged in LDS: read from global memory inside a stage,
  // a twiddle would wait behind every tile load still in flight
  // (vector-memory completions are counted in order).  TWM 0: the entries of
  // the length-L table the stages read (below L/2 for power-of-two
  // radices); TWM 1: the stage-major tables of the forward and inverse
  // transforms (one table when the plan reads the same forwards and
  // backwards).
  constexpr bool SAME_TW = [] {
    for (int q = 0; q < EF::NS; ++q)
      if (EF::St::radix(q) != EI::St::radix(q)) return false;
    return true;
  }();
  constexpr int NTW0 = (EF::St::max_twiddle_index() > EI::St::max_twiddle_index() ? EF::St::max_twiddle_index()
                                                                                   : EI::St::max_twiddle_index()) + 1;
  constexpr int NTW_F = TWM ? EF::stage_table_size() : NTW0;
  constexpr int NTW_I = TWM ? (SAME_TW ? 0 : EI::stage_table_size()) : 0;
  __shared__ cx<T> twl[NTW_F + NTW_I > 0 ? NTW_F + NTW_I : 1];
  {
    const cx<T>* __restrict__ src = static_cast<const cx<T>*>(a.tw);
    if constexpr (TWM) {
      EF::build_stage_table(twl, src, tid, NP * ZT);
      if constexpr (!SAME_TW) EI::build_stage_table(twl + NTW_F, src, tid, NP * ZT);
    } else {
      for (int i = tid; i < NTW0; i += NP * ZT) twl[i] = src[i];
    }
  }
  const cx<T>* tw = twl;
  const cx<T>* twi = (TWM && !SAME_TW) ? twl + NTW_F : twl;
  cx<T>* buf = static_cast<cx<T>*>(a.buf);
  // the spectrum values of this thread: octant entry (m1, m2, m3), m1 from
  // the element of the last forward stage it holds (32-bit index: the octant
  // has (L/2 + 1)^3 < 2^31 entries)
  constexpr uint32_t KP = L / 2 + 1;
  const uint32_t krow = static_cast<uint32_t>(m2) * KP + static_cast<uint32_t>(m3);
  ZRegs<T, PV> kv;
#pragma unroll
  for (int i = 0; i < St::cnt(SL); ++i) {
    const int b = bt + i * ZT;
#pragma unroll
    for (int j = 0; j < RL; ++j) {
      const int e = b + j * STRIDE;
      const uint32_t m1 = static_cast<uint32_t>(e <= L - e ? e : L - e);
      const bool ok = act && (St::nbf(SL) % ZT == 0 || b < St::nbf(SL));
      kv.v[i][j] = ok ? kh[m1 * (KP * KP) + krow] : cx<T>{};
    }
  }
  const int64_t nvar = (m2 != 0 && m2 != half) ? 2 : 1;  // uniform over the workgroup
  const int64_t ntile = r_lo < r_hi ? nvar * (r_hi - r_lo) : 0;
  const int64_t emask = (int64_t{1} << a.e_lg) - 1;
  // tiles in the order (k2 = m2, rhs r_lo..r_hi-1), (k2 = L - m2, the same
  // right-hand sides), walked with counters (no division per tile).  A
  // tile's base (its first column, tile * NP) is the same for the whole
  // workgroup; each thread adds its column t and the offset of each element.
  // Up to L = 512 one right-hand side's work array is below 4 GB, so the
  // offset of each element within a tile is a 32-bit byte count, the same
  // for every tile.  The elements a thread reads and writes are bt + C with
  // C a compile-time multiple of 2^e_lg (the host keeps e_lg within
  // z_align_lg), so element bt + C sits (C >> e_lg) e_hi elements after
  // element bt: one per-lane offset (that of bt, computed once) plus a
  // part the same for every lane (a scalar register).  Longer lengths
  // address each element from the thread's own base (k3 included) in 64
  // bits.
  constexpr bool A32 = SOFF;
  static_assert(!SOFF || L <= 512, "32-bit tile offsets need L <= 512");
  int64_t nx_rhs = r_lo, nx_var = 0;
  auto next_base = [&]() -> int64_t {
    const int64_t k2 = nx_var ? L - m2 : m2;
    const int64_t base = nx_rhs * a.batch_stride + k2 * a.o_stride + (A32 ? tile * NP : k3);
    if (++nx_rhs == r_hi) {
      nx_rhs = r_lo;
      ++nx_var;
    }
    return base;
  };
  // offset of element e of this thread's pencil from the tile's base (32
  // bits: A32 below)
  auto elem_off32 = [&](int e) -> uint32_t {
    return static_cast<uint32_t>(t) + (static_cast<uint32_t>(e) >> a.e_lg) * static_cast<uint32_t>(a.e_hi) +
           (static_cast<uint32_t>(e) & static_cast<uint32_t>(emask)) * static_cast<uint32_t>(a.e_lo);
  };
  auto addr = [&](int64_t base, int e) -> int64_t {
    return base + (e >> a.e_lg) * a.e_hi + (e & emask) * a.e_lo;
  };
  const uint32_t off0 = A32 ? elem_off32(bt) * static_cast<uint32_t>(sizeof(cx<T>)) : 0;
  // the part of element e's offset beyond element bt's (e - bt is a
  // compile-time constant once the stage loops are unrolled)
  auto uoff = [&](int e) -> uint32_t {
    return (static_cast<uint32_t>(e - bt) >> a.e_lg) * static_cast<uint32_t>(a.e_hi) *
           static_cast<uint32_t>(sizeof(cx<T>));
  };
  // range of a tile's buffer resource: one right-hand side's work array
  const int32_t range = A32 ? static_cast<int32_t>(a.batch_stride * int64_t{sizeof(cx<T>)}) : 0;
  auto fetch = [&](G0& g, int64_t base) {
    if constexpr (A32) {
      const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(buf + base, range);
      EF::template load_first<true>(g, bt, [&](int e) -> cx<T> {
        if constexpr (!EX) {
          if (e >= a.n) return cx<T>{};  // zero padding between n and L/2
        }
        return act ? buffer_load<T>(rs, off0, uoff(e)) : cx<T>{};
      });
    } else {
      EF::template load_first<true>(g, bt, [&](int e) -> cx<T> {
        if constexpr (!EX) {
          if (e >= a.n) return cx<T>{};
        }
        return act ? buf[addr(base, e)] : cx<T>{};
      });
    }
  };
  LdsPencil<T> lp{lds + t, NP, PADL ? 1 : 0};
  auto transform = [&](G0& g, int64_t base) {
    EF::template run<true>(g, bt, lp, tw, [&](auto& gl) {
#pragma unroll
      for (int i = 0; i < St::cnt(SL); ++i) {
#pragma unroll
        for (int j = 0; j < RL; ++j) gl.v[i][j] = gl.v[i][j] * kv.v[i][j];
      }
      EI::template run<false>(gl, bt, lp, twi, [&](auto& gi) {
        if constexpr (A32) {
          const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(buf + base, range);
          EI::template store_last<KEEP_HALF>(gi, bt, [&](int e, cx<T> v) {
            if constexpr (!EX) {
              if (e >= a.n) return;
            }
            if (act) buffer_store<T>(rs, off0, v, uoff(e));
          });
        } else {
          EI::template store_last<KEEP_HALF>(gi, bt, [&](int e, cx<T> v) {
            if constexpr (!EX) {
              if (e >= a.n) return;
            }
            if (act) buf[addr(base, e)] = v;
          });
        }
      });
    });
    __syncthreads();
  };
  if (ntile == 0) return;  // an empty right-hand-side slice (uniform over the workgroup)
  if constexpr (PF) {
    // two register sets in turn: the loads of tile it + 1 are in flight while
    // tile it is transformed
    G0 ga, gb;
    int64_t ba = next_base(), bb = 0;
    fetch(ga, ba);
#pragma unroll 1
    for (int64_t it = 0; it < ntile; it += 2) {
      if (it + 1 < ntile) {
        bb = next_base();
        fetch(gb, bb);
      }
      transform(ga, ba);
      if (it + 1 < ntile) {
        if (it + 2 < ntile) {
          ba = next_base();
          fetch(ga, ba);
        }
        transform(gb, bb);
      }
    }
  } else {
    G0 g;
#pragma unroll 1
    for (int64_t it = 0; it < ntile; ++it) {
      const int64_t base = next_base();
      fetch(g, base);
      transform(g, base);
    }
  }
}

// ---------------------------------------------------------------------------
// kernel spectrum on its octant (SpectrumArgs)
// ---------------------------------------------------------------------------
// The Green's table on the padded grid: c(m) = G(spacing |d|), wrapped
// offsets d_i = m_i (m_i <= L/2) or m_i - L (m_i > L/2); zero at m = 0 (the
// excluded self term, eq. 2.19) and wherever some |d_i| >= n (offsets that
// two of the n points per axis never have).
__device__ __forceinline__ cxd green_table(int m1, int m2, int m3, double k, double spacing, int n) {
  constexpr int half = L / 2;
  const int d1i = m1 <= half ? m1 : m1 - L;
  const int d2i = m2 <= half ? m2 : m2 - L;
  const int d3i = m3 <= half ? m3 : m3 - L;
  if (abs(d1i) >= n || abs(d2i) >= n || abs(d3i) >= n || (m1 | m2 | m3) == 0) return cxd{0.0, 0.0};
  const double d1 = d1i, d2 = d2i, d3 = d3i;
  const double r = spacing * sqrt(d1 * d1 + d2 * d2 + d3 * d3);
  double sn, cs;
  sincos(k * r, &sn, &cs);
  const double inv = 1.0 / (12.566370614359172954 * r);  // 1 / (4 pi r), eq. 2.6a
  return cxd{cs * inv, sn * inv};
}

// pass 1: pencils (m1, m2) in [0..n]^2 along the contiguous m3
__global__ void __launch_bounds__(BLOCK_C) k_spectrum_first(SpectrumArgs a) {
  constexpr int n = L / 2, kp = n + 1;
  __shared__ cxd lds[NPC * padded_row(L)];
  using E = Engine<double, L, false>;
  const int tid = threadIdx.x;
  const int bt = tid % TPP, t = tid / TPP;
  const int64_t pid = static_cast<int64_t>(blockIdx.x) * NPC + t;
  const bool act = pid < static_cast<int64_t>(kp) * kp;  // one pencil per (m1, m2)
  const int m1 = act ? static_cast<int>(pid / kp) : 0;
  const int m2 = act ? static_cast<int>(pid % kp) : 0;
  cxd* __restrict__ kh = static_cast<cxd*>(a.kh);
  auto load = [&](int e) -> cxd { return act ? green_table(m1, m2, e, a.k, a.spacing, static_cast<int>(a.n)) : cxd{}; };
  typename E::template RegsOf<0> g;
  E::template load_first<false>(g, bt, load);
  LdsPencil<double> lp{lds + t * padded_row(L), 0};
  E::template run<false>(g, bt, lp, static_cast<const cxd*>(a.tw), [&](auto& gl) {
    E::template store_last<KEEP_HALF1>(gl, bt, [&](int e, cxd v) {
      if (act) kh[pid * kp + e] = v;
    });
  });
}

// passes 2 and 3: pencils (o, c) in [0..n]^2 along m2 (pass 2) or m1 (pass 3)
__global__ void __launch_bounds__(block_s<double>()) k_spectrum_strided(SpectrumArgs a) {
  constexpr int n = L / 2, kp = n + 1;
  constexpr int NP = nps<double>();
  constexpr int64_t CT = (kp + NP - 1) / NP;
  __shared__ cxd lds[NP * L];
  using E = Engine<double, L, false>;
  const int tid = threadIdx.x;
  const int t = tid % NP, bt = tid / NP;
  // neighbouring column tiles share cache lines (rows of kp = n + 1 values
  // are not line aligned), so they run on one XCD
  const int64_t w = xcd_order(blockIdx.x, gridDim.x);
  const int64_t o = w / CT;
  const int64_t c = (w % CT) * NP + t;
  const bool act = c < kp;
  const int64_t ostride = a.pass == 2 ? int64_t{kp} * kp : kp;
  const int64_t axis = a.pass == 2 ? kp : int64_t{kp} * kp;
  const int64_t base = o * ostride + c;
  cxd* kh = static_cast<cxd*>(a.kh);
  cxd* kout = static_cast<cxd*>(a.kout);
  cxf* koutf = static_cast<cxf*>(a.koutf);
  auto load = [&](int e) -> cxd {
    const int em = e <= n ? e : L - e;  // even sequence: mirror
    return act ? kh[base + em * axis] : cxd{};
  };
  typename E::template RegsOf<0> g;
  E::template load_first<false>(g, bt, load);
  LdsPencil<double> lp{lds + t, NP};
  E::template run<false>(g, bt, lp, static_cast<const cxd*>(a.tw), [&](auto& gl) {
    E::template store_last<KEEP_HALF1>(gl, bt, [&](int e, cxd v) {
      if (!act) return;
      if (a.pass == 2) {
        kh[base + e * axis] = v;
        return;
      }
      // pass 3: K(k1 = e, k2 = o, k3 = c), scaled, into the octant the Z pass reads
      v = scale(v, a.scale);
      const int64_t at = (static_cast<int64_t>(e) * kp + o) * kp + c;
      kout[at] = v;
      if (koutf) koutf[at] = cvt<float>(v);
    });
  });
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// Tile widths: "wide" (nps, 128-byte rows) and "narrow" (half as many pencils
// per workgroup, twice as many workgroups per CU).
template <typename T>
constexpr int np_narrow() {
  return whole_waves(nps<T>() / 2 > 0 ? nps<T>() / 2 : 1, TPP);
}
template <typename T>
int np_of(int sel) {
  return sel ? np_narrow<T>() : nps<T>();
}

int64_t strided_blocks(int fprec, int np_sel, int64_t n_outer, int64_t C) {
  const int np = fprec == PREC_F64 ? np_of<double>(np_sel) : np_of<float>(np_sel);
  return n_outer * ((C + np - 1) / np);
}

template <bool EX>
hipError_t contig_fwd_t(int vp, int fp, const ContigFwdArgs& a, hipStream_t st) {
  hipError_t e = hipSuccess;
  const dim3 grid(static_cast<unsigned>(a.nrhs * contig_blocks_per_rhs(a.ppr))), block(BLOCK_C);
  if (vp == PREC_F64 && fp == PREC_F64) {
    e = launch_kernel((k_contig_fwd<double, double, EX>), grid, block, st, a);
  } else if (vp == PREC_F32 && fp == PREC_F32) {
    e = launch_kernel((k_contig_fwd<float, float, EX>), grid, block, st, a);
  } else if (vp == PREC_F64 && fp == PREC_F32) {
    e = launch_kernel((k_contig_fwd<double, float, EX>), grid, block, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return e;
}

hipError_t contig_fwd(int vp, int fp, const ContigFwdArgs& a, hipStream_t st) {
  // the input is the first n <= L/2 entries of each pencil (zero padding)
  if (!a.half_in || a.in_pitch < 1 || 2 * a.in_pitch - 1 > L || a.out_pitch != L) return hipErrorInvalidValue;
  return 2 * a.in_pitch == L ? contig_fwd_t<true>(vp, fp, a, st) : contig_fwd_t<false>(vp, fp, a, st);
}

template <bool EX>
hipError_t contig_inv_t(int vp, int fp, const ContigInvArgs& a, hipStream_t st) {
  hipError_t e = hipSuccess;
  const dim3 grid(static_cast<unsigned>(a.nrhs * contig_blocks_per_rhs(a.ppr))), block(BLOCK_C);
  if (vp == PREC_F64 && fp == PREC_F64)
    e = launch_kernel((k_contig_inv<double, double, EX>), grid, block, st, a);
  else if (vp == PREC_F32 && fp == PREC_F32)
    e = launch_kernel((k_contig_inv<float, float, EX>), grid, block, st, a);
  else if (vp == PREC_F64 && fp == PREC_F32)
    e = launch_kernel((k_contig_inv<double, float, EX>), grid, block, st, a);
  else
    return hipErrorInvalidValue;
  return e;
}

hipError_t contig_inv(int vp, int fp, const ContigInvArgs& a, hipStream_t st) {
  // the output is the first n <= L/2 entries of each inverse transform
  if (a.out_pitch < 1 || 2 * a.out_pitch - 1 > L || a.in_pitch != L) return hipErrorInvalidValue;
  return 2 * a.out_pitch == L ? contig_inv_t<true>(vp, fp, a, st) : contig_inv_t<false>(vp, fp, a, st);
}

template <typename T, int NP>
hipError_t strided_t(const StridedArgs& a, hipStream_t st) {
  hipError_t e = hipSuccess;
  const dim3 grid(static_cast<unsigned>(a.n_outer * ((a.C + NP - 1) / NP))), block(NP * TPP);
  if (a.nv < 1 || 2 * a.nv - 1 > L) return hipErrorInvalidValue;
  const bool ex = 2 * a.nv == L;
  if (!a.inverse && a.half_in && !a.half_out)
    e = ex ? launch_kernel((k_strided<T, NP, false, true, false, true>), grid, block, st, a)
           : launch_kernel((k_strided<T, NP, false, true, false, false>), grid, block, st, a);
  else if (a.inverse && !a.half_in && a.half_out)
    e = ex ? launch_kernel((k_strided<T, NP, true, false, true, true>), grid, block, st, a)
           : launch_kernel((k_strided<T, NP, true, false, true, false>), grid, block, st, a);
  else
    return hipErrorInvalidValue;
  return e;
}

hipError_t strided(int fp, const StridedArgs& a, hipStream_t st) {
  if (fp == PREC_F64)
    return a.np_sel ? strided_t<double, np_narrow<double>()>(a, st) : strided_t<double, nps<double>()>(a, st);
  return a.np_sel ? strided_t<float, np_narrow<float>()>(a, st) : strided_t<float, nps<float>()>(a, st);
}

// Z workgroups per right-hand-side slice: octant rows m2 in [0, L/2] times
// the tiles of k3 in [0, L)
int64_t zpass_blocks(int fprec, int np_sel) {
  const int64_t np = fprec == PREC_F64 ? np_of<double>(np_sel) : np_of<float>(np_sel);
  return (L / 2 + 1) * ((L + np - 1) / np);
}

template <typename T, int NP, bool SOFF, int PV>
hipError_t zpass_s(const ZArgs& a, const dim3& grid, const dim3& block, hipStream_t st) {
  const bool ex = 2 * a.n == L;
  if (a.prefetch)
    return ex ? launch_kernel((k_zpass<T, NP, true, true, SOFF, PV>), grid, block, st, a)
              : launch_kernel((k_zpass<T, NP, true, false, SOFF, PV>), grid, block, st, a);
  return ex ? launch_kernel((k_zpass<T, NP, false, true, SOFF, PV>), grid, block, st, a)
            : launch_kernel((k_zpass<T, NP, false, false, SOFF, PV>), grid, block, st, a);
}

template <typename T, int NP, int PV>
hipError_t zpass_p(const ZArgs& a, const dim3& grid, const dim3& block, hipStream_t st) {
  if constexpr (L <= 512) {
    if (a.e_lg <= z_align_lg<T, PV>()) return zpass_s<T, NP, true, PV>(a, grid, block, st);
  }
  return zpass_s<T, NP, false, PV>(a, grid, block, st);
}

template <typename T, int NP>
hipError_t zpass_t(const ZArgs& a, hipStream_t st) {
  if (a.rhs_slices < 1 || a.rhs_slices > a.nrhs) return hipErrorInvalidValue;
  if (a.plan != 0 && (a.plan != 1 || !has_plan_variant(L))) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>((L / 2 + 1) * ((L + NP - 1) / NP) * a.rhs_slices)), block(NP * z_tpp<T>());
  if constexpr (has_plan_variant(L)) {
    if (a.plan == 1) return zpass_p<T, NP, 1>(a, grid, block, st);
  }
  return zpass_p<T, NP, 0>(a, grid, block, st);
}

hipError_t spectrum(const SpectrumArgs& a, hipStream_t st) {
  if (a.n < 1 || 2 * a.n - 1 > L) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  constexpr int64_t kp = L / 2 + 1;
  if (a.pass == 1) {
    e = launch_kernel(k_spectrum_first, dim3(static_cast<unsigned>(contig_blocks_per_rhs(kp * kp))), dim3(BLOCK_C), st,
                       a);
  } else if (a.pass == 2 || a.pass == 3) {
    const int64_t np = nps<double>();
    const dim3 grid(static_cast<unsigned>(kp * ((kp + np - 1) / np)));
    e = launch_kernel(k_spectrum_strided, grid, dim3(block_s<double>()), st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return e;
}

hipError_t zpass(int fp, const ZArgs& a, hipStream_t st) {
  if (a.n < 1 || 2 * a.n - 1 > L || a.kp != L / 2 + 1) return hipErrorInvalidValue;
  if (fp == PREC_F64) return a.np_sel ? zpass_t<double, np_narrow<double>()>(a, st) : zpass_t<double, nps<double>()>(a, st);
  return a.np_sel ? zpass_t<float, np_narrow<float>()>(a, st) : zpass_t<float, nps<float>()>(a, st);
}

}  // namespace

#define ORI_CAT2(a, b) a##b
#define ORI_CAT(a, b) ORI_CAT2(a, b)

const LengthKernels* ORI_CAT(kernels_L, ORI_L)() {
  static const LengthKernels k = {L, contig_fwd, contig_inv, strided, zpass, contig_blocks_per_rhs, strided_blocks,
                                  zpass_blocks, spectrum};
  return &k;
}

}  // namespace ori
