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

// ---------------------------------------------------------------------------
// F1 (and the first spectrum pass): contiguous forward with prologue
// ---------------------------------------------------------------------------
template <typename V, typename T, bool HALF>
__global__ void __launch_bounds__(BLOCK_C) k_contig_fwd(ContigFwdArgs a) {
  __shared__ cx<T> lds[NPC * L];
  using E = Engine<T, L, false>;
  const int tid = threadIdx.x;
  const int bt = tid % TPP, t = tid / TPP;
  const int64_t pid = static_cast<int64_t>(blockIdx.x) * NPC + t;
  const bool act = pid < a.npencils;
  const cx<T>* __restrict__ tw = static_cast<const cx<T>*>(a.tw);
  const cx<V>* __restrict__ x = static_cast<const cx<V>*>(a.x);
  cx<V>* pv = static_cast<cx<V>*>(a.pvec);
  const cx<V>* __restrict__ s = static_cast<const cx<V>*>(a.s_in);
  cx<T>* __restrict__ out = static_cast<cx<T>*>(a.out);
  const int64_t ib = pid * a.in_pitch;
  const int64_t ob = pid * a.out_pitch;
  cx<double> beta = {0.0, 0.0};
  if (a.mode == 1 && !a.first) beta = cx<double>{a.sc->beta_re, a.sc->beta_im};

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
    if (s) v = v * cvt<double>(s[i]);
    return cvt<T>(v);
  };
  typename E::template RegsOf<0> g;
  E::template load_first<HALF>(g, bt, load);
  LdsPencil<T> lp{lds + t * L, 1};
  E::template run<HALF>(g, bt, lp, tw, [&](auto& gl) {
    E::template store_last<false>(gl, bt, [&](int e, cx<T> v) {
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
  const int64_t pid = static_cast<int64_t>(blockIdx.x) * NPC + t;
  const bool act = pid < a.npencils;
  const cx<T>* __restrict__ tw = static_cast<const cx<T>*>(a.tw);
  const cx<T>* __restrict__ in = static_cast<const cx<T>*>(a.in);
  cx<V>* __restrict__ y = static_cast<cx<V>*>(a.y);
  const cx<V>* __restrict__ a0 = static_cast<const cx<V>*>(a.a0);
  const cx<V>* __restrict__ a1 = static_cast<const cx<V>*>(a.a1);
  const cx<V>* __restrict__ so = static_cast<const cx<V>*>(a.s_out);
  const int64_t ib = pid * a.in_pitch;
  const int64_t ob = pid * a.out_pitch;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};

  auto load = [&](int e) -> cx<T> { return act ? in[ib + e] : cx<T>{}; };
  typename E::template RegsOf<0> g;
  E::template load_first<false>(g, bt, load);
  LdsPencil<T> lp{lds + t * L, 1};
  E::template run<false>(g, bt, lp, tw, [&](auto& gl) {
    E::template store_last<true>(gl, bt, [&](int e, cx<T> c) {
      if (!act) return;
      const int64_t i = ob + e;
      cx<double> conv = cvt<double>(c);
      if (so) conv = conv * cvt<double>(so[i]);
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
  const int64_t ib = o * a.in_outer + c;
  const int64_t ob = o * a.out_outer + c;

  auto load = [&](int e) -> cx<T> { return act ? in[ib + e * a.in_axis] : cx<T>{}; };
  typename E::template RegsOf<0> g;
  E::template load_first<HIN>(g, bt, load);
  LdsPencil<T> lp{lds + t, NP};
  E::template run<HIN>(g, bt, lp, tw, [&](auto& gl) {
    E::template store_last<HOUT>(gl, bt, [&](int e, cx<T> v) {
      if (act) out[ob + e * a.out_axis] = v;
    });
  });
}

// ---------------------------------------------------------------------------
// Z: forward along i1 (n inputs), times the spectrum octant, inverse, keep n
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(block_s<T>()) k_zpass(ZArgs a) {
  constexpr int NP = nps<T>();
  __shared__ cx<T> lds[NP * L];
  using EF = Engine<T, L, false>;
  using EI = Engine<T, L, true>;
  using St = Stages<L, false>;
  constexpr int SL = St::NS - 1;
  constexpr int RL = St::radix(SL);
  constexpr int STRIDE = L / RL;
  const int tid = threadIdx.x;
  const int t = tid % NP, bt = tid / NP;
  const int64_t CT = (a.C + NP - 1) / NP;
  const int64_t o = blockIdx.x / CT;
  const int64_t c = (blockIdx.x % CT) * NP + t;
  const bool act = c < a.C;
  const cx<T>* __restrict__ tw = static_cast<const cx<T>*>(a.tw);
  const cx<T>* __restrict__ kh = static_cast<const cx<T>*>(a.khat);
  cx<T>* buf = static_cast<cx<T>*>(a.buf);
  const int64_t base = o * a.outer + c;
  const int64_t m2 = o <= L - o ? o : L - o;
  const int64_t m3 = act ? (c <= L - c ? c : L - c) : 0;
  const int64_t kb = m2 * a.kp + m3;

  auto load = [&](int e) -> cx<T> { return act ? buf[base + e * a.axis] : cx<T>{}; };
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
      EI::template store_last<true>(gi, bt, [&](int e, cx<T> v) {
        if (act) buf[base + e * a.axis] = v;
      });
    });
  });
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int64_t contig_blocks(int64_t npencils) { return (npencils + NPC - 1) / NPC; }

int64_t strided_blocks(int fprec, int64_t n_outer, int64_t C) {
  const int np = fprec == PREC_F64 ? nps<double>() : nps<float>();
  return n_outer * ((C + np - 1) / np);
}

hipError_t contig_fwd(int vp, int fp, const ContigFwdArgs& a, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(contig_blocks(a.npencils))), block(BLOCK_C);
  if (vp == PREC_F64 && fp == PREC_F64) {
    if (a.half_in)
      hipLaunchKernelGGL((k_contig_fwd<double, double, true>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_contig_fwd<double, double, false>), grid, block, 0, st, a);
  } else if (vp == PREC_F32 && fp == PREC_F32 && a.half_in) {
    hipLaunchKernelGGL((k_contig_fwd<float, float, true>), grid, block, 0, st, a);
  } else if (vp == PREC_F64 && fp == PREC_F32 && a.half_in) {
    hipLaunchKernelGGL((k_contig_fwd<double, float, true>), grid, block, 0, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t contig_inv(int vp, int fp, const ContigInvArgs& a, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(contig_blocks(a.npencils))), block(BLOCK_C);
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
    else if (!a.inverse && !a.half_in && !a.half_out)
      hipLaunchKernelGGL((k_strided<double, false, false, false>), grid, block, 0, st, a);
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

hipError_t zpass(int fp, const ZArgs& a, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(strided_blocks(fp, a.n_outer, a.C)));
  if (fp == PREC_F64)
    hipLaunchKernelGGL((k_zpass<double>), grid, dim3(block_s<double>()), 0, st, a);
  else
    hipLaunchKernelGGL((k_zpass<float>), grid, dim3(block_s<float>()), 0, st, a);
  return hipGetLastError();
}

}  // namespace

#define ORI_CAT2(a, b) a##b
#define ORI_CAT(a, b) ORI_CAT2(a, b)

const LengthKernels* ORI_CAT(kernels_L, ORI_L)() {
  static const LengthKernels k = {L, contig_fwd, contig_inv, strided, zpass, contig_blocks, strided_blocks};
  return &k;
}

}  // namespace ori
