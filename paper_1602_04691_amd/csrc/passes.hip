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
#include "pass_common.h"

#ifndef ORI_L
#error "compile once per padded length with -DORI_L=<L>"
#endif

namespace ori {
namespace {

constexpr int L = ORI_L;

#include "pass_bodies.inc"

// The kernels of this length: one workgroup of the pass each.
template <typename V, typename T, bool EX>
__global__ void __launch_bounds__(BLOCK_C) k_contig_fwd(ContigFwdArgs a) {
  __shared__ __align__(16) unsigned char smem[contig_smem<T>()];
  contig_fwd_body<V, T, EX>(a, blockIdx.x, smem);
}

template <typename V, typename T, bool EX>
__global__ void __launch_bounds__(BLOCK_C) k_contig_inv(ContigInvArgs a) {
  __shared__ __align__(16) unsigned char smem[contig_smem<T>()];
  contig_inv_body<V, T, EX>(a, blockIdx.x, smem);
}

template <typename T, int NP, bool INV, bool HIN, bool HOUT, bool EX>
__global__ void __launch_bounds__(NP * TPP) k_strided(StridedArgs a) {
  __shared__ __align__(16) unsigned char smem[strided_smem<T, NP>()];
  strided_body<T, NP, INV, HIN, HOUT, EX>(a, blockIdx.x, gridDim.x, smem);
}

template <typename T, int NP, bool PF, bool EX, bool SOFF, int PV>
__global__ void __launch_bounds__(NP * z_tpp<T>(), (z_min_waves<T, NP, PF, PV, SOFF>())) k_zpass(ZArgs a) {
  __shared__ __align__(16) unsigned char smem[z_smem<T, NP, PV>()];
  zpass_body<T, NP, PF, EX, SOFF, PV>(a, blockIdx.x, gridDim.x, smem);
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
