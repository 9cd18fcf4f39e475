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
#include "fft_engine.h"
#include "kernels.h"

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

__device__ __forceinline__ int64_t two_level(int64_t o, int lg, int64_t hi, int64_t lo) {
  return (o >> lg) * hi + (o & ((int64_t{1} << lg) - 1)) * lo;
}

// ---------------------------------------------------------------------------
// F1 (and the first spectrum pass): contiguous forward with prologue
// ---------------------------------------------------------------------------
template <typename V, typename T, bool HALF>
__global__ void __launch_bounds__(BLOCK_C) k_contig_fwd(ContigFwdArgs a) {
  __shared__ cx<T> lds[NPC * L];
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
  cx<double> beta = {0.0, 0.0};
  if (a.mode == 1 && !a.first) beta = cx<double>{a.sc[rhs].beta_re, a.sc[rhs].beta_im};

  auto load = [&](int e) -> cx<T> {
    if (!act) return cx<T>{};
    const int64_t i = ib + e;
    cx<double> v;
    if (a.mode == 1) {
      v = cvt<double>(x[i]);
      if (!a.first) v = v + beta * cvt<double>(pv[i]);
      pv[i] = cvt<V>(v);
    } else {
      v = cvt<double>(x[i]);
    }
    if (s) v = v * cvt<double>(s[db + e]);
    return cvt<T>(v);
  };
  typename E::template RegsOf<0> g;
  E::template load_first<HALF>(g, bt, load);
  LdsPencil<T> lp{lds + t * L, 1};
  E::template run<HALF>(g, bt, lp, tw, [&](auto& gl) {
    E::template store_last<KEEP_ALL>(gl, bt, [&](int e, cx<T> v) {
      if (act) out[ob + e] = v;
    });
  });
}

// ---------------------------------------------------------------------------
// I1: contiguous inverse, keep e < out_pitch (= n), epilogue and partials
// ---------------------------------------------------------------------------
template <typename V, typename T>
__global__ void __launch_bounds__(BLOCK_C) k_contig_inv(ContigInvArgs a) {
  __shared__ cx<T> lds[NPC * L];
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
  LdsPencil<T> lp{lds + t * L, 1};
  E::template run<false>(g, bt, lp, tw, [&](auto& gl) {
    E::template store_last<KEEP_HALF>(gl, bt, [&](int e, cx<T> c) {
      if (!act) return;
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
// F2 / I2 / spectrum passes: strided axis, NP adjacent pencils per workgroup
// ---------------------------------------------------------------------------
template <typename T, bool INV, bool HIN, bool HOUT>
__global__ void __launch_bounds__(block_s<T>()) k_strided(StridedArgs a) {
  constexpr int NP = nps<T>();
  __shared__ cx<T> lds[NP * L];
  using E = Engine<T, L, INV>;
  const int tid = threadIdx.x;
  const int t = tid % NP, bt = tid / NP;
  const int64_t CT = (a.C + NP - 1) / NP;
  const int64_t o = blockIdx.x / CT;
  const int64_t c = (blockIdx.x % CT) * NP + t;
  const bool act = c < a.C;
  const cx<T>* __restrict__ tw = static_cast<const cx<T>*>(a.tw);
  const cx<T>* in = static_cast<const cx<T>*>(a.in);
  cx<T>* out = static_cast<cx<T>*>(a.out);
  const int64_t ib = two_level(o, a.in_lg, a.in_hi, a.in_lo) + c;
  const int64_t ob = two_level(o, a.out_lg, a.out_hi, a.out_lo) + c;

  auto load = [&](int e) -> cx<T> { return act ? in[ib + e * a.in_axis] : cx<T>{}; };
  typename E::template RegsOf<0> g;
  E::template load_first<HIN>(g, bt, load);
  LdsPencil<T> lp{lds + t, NP};
  E::template run<HIN>(g, bt, lp, tw, [&](auto& gl) {
    E::template store_last<HOUT ? KEEP_HALF : KEEP_ALL>(gl, bt, [&](int e, cx<T> v) {
      if (act) out[ob + e * a.out_axis] = v;
    });
  });
}

// ---------------------------------------------------------------------------
// Z: forward along i1 (n inputs), times the spectrum octant, inverse, keep n
// ---------------------------------------------------------------------------
// One pencil tile: NP pencils (k2, k3_t) of one workgroup, t = thread's
// pencil.  kb is the thread's octant offset m2 * kp + m3.
template <typename T>
__device__ __forceinline__ void z_tile(const ZArgs& a, cx<T>* lds, int t, int bt, bool act, int64_t rhs, int64_t k2,
                                       int64_t k3, int64_t kb) {
  constexpr int NP = nps<T>();
  using EF = Engine<T, L, false>;
  using EI = Engine<T, L, true>;
  using St = Stages<L, false>;
  constexpr int SL = St::NS - 1;
  constexpr int RL = St::radix(SL);
  constexpr int STRIDE = L / RL;
  const cx<T>* __restrict__ tw = static_cast<const cx<T>*>(a.tw);
  const cx<T>* __restrict__ kh = static_cast<const cx<T>*>(a.khat);
  cx<T>* buf = static_cast<cx<T>*>(a.buf);
  const int64_t base = rhs * a.batch_stride + k2 * a.o_stride + k3;
  const int64_t emask = (int64_t{1} << a.e_lg) - 1;
  auto addr = [&](int e) -> int64_t { return base + (e >> a.e_lg) * a.e_hi + (e & emask) * a.e_lo; };
  auto load = [&](int e) -> cx<T> { return act ? buf[addr(e)] : cx<T>{}; };
  typename EF::template RegsOf<0> g;
  EF::template load_first<true>(g, bt, load);
  LdsPencil<T> lp{lds + t, NP};
  EF::template run<true>(g, bt, lp, tw, [&](auto& gl) {
    if (act) {
#pragma unroll
      for (int i = 0; i < St::cnt(SL); ++i) {
        const int b = bt + i * TPP;
        if (St::nbf(SL) % TPP != 0 && b >= St::nbf(SL)) continue;
#pragma unroll
        for (int j = 0; j < RL; ++j) {
          const int e = b + j * STRIDE;
          const int m1 = e <= L - e ? e : L - e;
          gl.v[i][j] = gl.v[i][j] * kh[m1 * a.kp * a.kp + kb];
        }
      }
    }
    EI::template run<false>(gl, bt, lp, tw, [&](auto& gi) {
      EI::template store_last<KEEP_HALF>(gi, bt, [&](int e, cx<T> v) {
        if (act) buf[addr(e)] = v;
      });
    });
  });
}

// zmap 0: workgroup = (k2, tile of NP consecutive k3)
template <typename T>
__global__ void __launch_bounds__(block_s<T>()) k_zpass(ZArgs a) {
  constexpr int NP = nps<T>();
  __shared__ cx<T> lds[NP * L];
  const int tid = threadIdx.x;
  const int t = tid % NP, bt = tid / NP;
  constexpr int64_t CT = (L + NP - 1) / NP;
  const int64_t k2 = blockIdx.x / CT;
  const int64_t k3 = (blockIdx.x % CT) * NP + t;
  const bool act = k3 < L;
  const int64_t m2 = k2 <= L - k2 ? k2 : L - k2;
  const int64_t m3 = act ? (k3 <= L - k3 ? k3 : L - k3) : 0;
#pragma unroll 1
  for (int64_t rhs = 0; rhs < a.nrhs; ++rhs) {
    z_tile<T>(a, lds, t, bt, act, rhs, k2, k3, m2 * a.kp + m3);
    __syncthreads();
  }
}

// zmap 1: workgroup = (m2, tile of NP consecutive m3) of the octant; it runs
// the pencils (m2 | L-m2) x (m3 | L-m3) one after the other, so the octant
// rows it reads serve up to four pencils from cache.
template <typename T>
__global__ void __launch_bounds__(block_s<T>()) k_zpass_octant(ZArgs a) {
  constexpr int NP = nps<T>();
  constexpr int n = L / 2;
  __shared__ cx<T> lds[NP * L];
  const int tid = threadIdx.x;
  const int t = tid % NP, bt = tid / NP;
  constexpr int64_t CT = (n + 1 + NP - 1) / NP;
  const int64_t m2 = blockIdx.x / CT;
  const int64_t m3 = (blockIdx.x % CT) * NP + t;
  const bool in_oct = m3 <= n;
  const int64_t kb = m2 * a.kp + (in_oct ? m3 : 0);
  const bool mirror2 = m2 != 0 && m2 != n;
  const bool mirror3 = m3 != 0 && m3 < n;
#pragma unroll 1
  for (int v = 0; v < 4; ++v) {
    if ((v & 2) && !mirror2) continue;  // uniform over the workgroup
    const int64_t k2 = (v & 2) ? L - m2 : m2;
    const int64_t k3 = (v & 1) ? L - m3 : m3;
    const bool act = in_oct && (!(v & 1) || mirror3);
#pragma unroll 1
    for (int64_t rhs = 0; rhs < a.nrhs; ++rhs) {
      z_tile<T>(a, lds, t, bt, act, rhs, k2, k3, kb);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// kernel spectrum on its octant (SpectrumArgs)
// ---------------------------------------------------------------------------
// The Green's table on the padded grid: c(m) = G(spacing |d|), wrapped
// offsets d_i = m_i (m_i < n) or m_i - L (m_i > n); zero at m = 0 (the
// excluded self term, eq. 2.19) and where some m_i = n (never reached).
__device__ __forceinline__ cxd green_table(int m1, int m2, int m3, double k, double spacing) {
  constexpr int n = L / 2;
  if (m1 == n || m2 == n || m3 == n || (m1 | m2 | m3) == 0) return cxd{0.0, 0.0};
  const double d1 = m1 < n ? m1 : m1 - L;
  const double d2 = m2 < n ? m2 : m2 - L;
  const double d3 = m3 < n ? m3 : m3 - L;
  const double r = spacing * sqrt(d1 * d1 + d2 * d2 + d3 * d3);
  double sn, cs;
  sincos(k * r, &sn, &cs);
  const double inv = 1.0 / (12.566370614359172954 * r);  // 1 / (4 pi r), eq. 2.6a
  return cxd{cs * inv, sn * inv};
}

// pass 1: pencils (m1, m2) in [0..n]^2 along the contiguous m3
__global__ void __launch_bounds__(BLOCK_C) k_spectrum_first(SpectrumArgs a) {
  constexpr int n = L / 2, kp = n + 1;
  __shared__ cxd lds[NPC * L];
  using E = Engine<double, L, false>;
  const int tid = threadIdx.x;
  const int bt = tid % TPP, t = tid / TPP;
  const int64_t pid = static_cast<int64_t>(blockIdx.x) * NPC + t;
  const bool act = pid < static_cast<int64_t>(kp) * kp;  // one pencil per (m1, m2)
  const int m1 = act ? static_cast<int>(pid / kp) : 0;
  const int m2 = act ? static_cast<int>(pid % kp) : 0;
  cxd* __restrict__ kh = static_cast<cxd*>(a.kh);
  auto load = [&](int e) -> cxd { return act ? green_table(m1, m2, e, a.k, a.spacing) : cxd{}; };
  typename E::template RegsOf<0> g;
  E::template load_first<false>(g, bt, load);
  LdsPencil<double> lp{lds + t * L, 1};
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
  const int64_t o = blockIdx.x / CT;
  const int64_t c = (blockIdx.x % CT) * NP + t;
  const bool act = c < kp;
  const int64_t ostride = a.pass == 2 ? int64_t{kp} * kp : kp;
  const int64_t axis = a.pass == 2 ? kp : int64_t{kp} * kp;
  const int64_t base = o * ostride + c;
  cxd* kh = static_cast<cxd*>(a.kh);
  cxf* khf = static_cast<cxf*>(a.khf);
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
      const int64_t i = base + e * axis;
      if (a.pass == 3) {
        v = scale(v, a.scale);
        if (khf) khf[i] = cvt<float>(v);
      }
      kh[i] = v;
    });
  });
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int64_t strided_blocks(int fprec, int64_t n_outer, int64_t C) {
  const int np = fprec == PREC_F64 ? nps<double>() : nps<float>();
  return n_outer * ((C + np - 1) / np);
}

hipError_t contig_fwd(int vp, int fp, const ContigFwdArgs& a, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(a.nrhs * contig_blocks_per_rhs(a.ppr))), block(BLOCK_C);
  if (!a.half_in) return hipErrorInvalidValue;
  if (vp == PREC_F64 && fp == PREC_F64) {
    hipLaunchKernelGGL((k_contig_fwd<double, double, true>), grid, block, 0, st, a);
  } else if (vp == PREC_F32 && fp == PREC_F32) {
    hipLaunchKernelGGL((k_contig_fwd<float, float, true>), grid, block, 0, st, a);
  } else if (vp == PREC_F64 && fp == PREC_F32) {
    hipLaunchKernelGGL((k_contig_fwd<double, float, true>), grid, block, 0, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t contig_inv(int vp, int fp, const ContigInvArgs& a, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(a.nrhs * contig_blocks_per_rhs(a.ppr))), block(BLOCK_C);
  if (vp == PREC_F64 && fp == PREC_F64)
    hipLaunchKernelGGL((k_contig_inv<double, double>), grid, block, 0, st, a);
  else if (vp == PREC_F32 && fp == PREC_F32)
    hipLaunchKernelGGL((k_contig_inv<float, float>), grid, block, 0, st, a);
  else if (vp == PREC_F64 && fp == PREC_F32)
    hipLaunchKernelGGL((k_contig_inv<double, float>), grid, block, 0, st, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t strided(int fp, const StridedArgs& a, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(strided_blocks(fp, a.n_outer, a.C)));
  if (fp == PREC_F64) {
    const dim3 block(block_s<double>());
    if (!a.inverse && a.half_in && !a.half_out)
      hipLaunchKernelGGL((k_strided<double, false, true, false>), grid, block, 0, st, a);
    else if (a.inverse && !a.half_in && a.half_out)
      hipLaunchKernelGGL((k_strided<double, true, false, true>), grid, block, 0, st, a);
    else
      return hipErrorInvalidValue;
  } else {
    const dim3 block(block_s<float>());
    if (!a.inverse && a.half_in && !a.half_out)
      hipLaunchKernelGGL((k_strided<float, false, true, false>), grid, block, 0, st, a);
    else if (a.inverse && !a.half_in && a.half_out)
      hipLaunchKernelGGL((k_strided<float, true, false, true>), grid, block, 0, st, a);
    else
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int64_t zpass_blocks(int fprec, int64_t n, int zmap) {
  const int64_t np = fprec == PREC_F64 ? nps<double>() : nps<float>();
  if (zmap == 1) return (n + 1) * ((n + 1 + np - 1) / np);
  return (2 * n) * ((2 * n + np - 1) / np);
}

hipError_t spectrum(const SpectrumArgs& a, hipStream_t st) {
  constexpr int64_t kp = L / 2 + 1;
  if (a.pass == 1) {
    hipLaunchKernelGGL(k_spectrum_first, dim3(static_cast<unsigned>(contig_blocks_per_rhs(kp * kp))), dim3(BLOCK_C), 0, st,
                       a);
  } else if (a.pass == 2 || a.pass == 3) {
    const int64_t np = nps<double>();
    const dim3 grid(static_cast<unsigned>(kp * ((kp + np - 1) / np)));
    hipLaunchKernelGGL(k_spectrum_strided, grid, dim3(block_s<double>()), 0, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t zpass(int fp, const ZArgs& a, hipStream_t st) {
  if (a.n != L / 2) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(zpass_blocks(fp, a.n, a.zmap)));
  if (fp == PREC_F64) {
    if (a.zmap == 1)
      hipLaunchKernelGGL((k_zpass_octant<double>), grid, dim3(block_s<double>()), 0, st, a);
    else
      hipLaunchKernelGGL((k_zpass<double>), grid, dim3(block_s<double>()), 0, st, a);
  } else {
    if (a.zmap == 1)
      hipLaunchKernelGGL((k_zpass_octant<float>), grid, dim3(block_s<float>()), 0, st, a);
    else
      hipLaunchKernelGGL((k_zpass<float>), grid, dim3(block_s<float>()), 0, st, a);
  }
  return hipGetLastError();
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
