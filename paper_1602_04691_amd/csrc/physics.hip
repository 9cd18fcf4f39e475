// What the solution of eq. 2.19 is used for.
//
//  * Charges (eq. 2.13 summed over the particles of a cell with eq. 2.18):
//    Q_p = -c_S h_p N_p |Delta_p| u_p = -D_p u_p.
//  * The scattered field anywhere (eq. 2.10, the particles of each cell at
//    x_p): v(x) = sum_p G(x, x_p) Q_p, G of eq. 2.6a; a cell point at distance
//    exactly 0 is left out, as the sum of eq. 2.19 leaves out p = q.
//  * Its far-field amplitude: v(r beta) = A(beta) e^{ikr} / r + O(1/r^2) with
//    A(beta) = (1 / 4 pi) sum_p e^{-ik beta.x_p} Q_p.
//  * The refraction recipe (eqs. 2.24-2.26, 4.1-4.2): n = [n0^2 - c_S h N /
//    k^2]^{1/2} with the branch arg in [0, 2 pi), and the h that creates a
//    desired n.
//  * The solution difference of Section 4 (Table 4) between a fine and a
//    coarse grid: the sup over coarse cells of the mean |x_i - y_q| over the
//    fine points x_i inside the cell.
//
// The sums over cells are direct (M points x P cells, FP64): workgroup
// (chunk of cells, point, right-hand side) writes one partial; a second
// kernel adds the partials of each point in a fixed order, so results are
// deterministic.
#include "cx.h"
#include "kernels.h"
#include "launch.h"

namespace ori {
namespace {

constexpr int kFieldThreads = 256;
constexpr double kFourPi = 12.566370614359172954;

__device__ __forceinline__ cxd block_sum_cx(cxd v) {
  __shared__ double sh[2 * (kFieldThreads / 64)];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_xor(v.re, off, 64);
    v.im += __shfl_xor(v.im, off, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[2 * w] = v.re;
    sh[2 * w + 1] = v.im;
  }
  __syncthreads();
  cxd s{0.0, 0.0};
  if (threadIdx.x == 0)
    for (int i = 0; i < kFieldThreads / 64; ++i) s = s + cxd{sh[2 * i], sh[2 * i + 1]};
  return s;
}

// floor(v / n) for 0 <= v < 2^31 and n <= 1024 without an integer division:
// (v + 1/2) / n lies at least 1/(2n) from an integer, and its FP64 product
// with the rounded reciprocal of n is off by less than 2^-21, so truncation
// gives the quotient exactly
__device__ __forceinline__ int32_t quot(int32_t v, double inv_n) {
  return static_cast<int32_t>((static_cast<double>(v) + 0.5) * inv_n);
}

constexpr int kFieldMaxN = 512;

// grid (chunks, points, right-hand sides): partial sum over one chunk of cells.
// The cell points lie on a grid, so a workgroup first tabulates the
// coordinate origin + side (i + offset) / n of every index along each axis
// and, for the far field, the phase e^{-ik beta_d x_d} of each (the phase of
// a cell is the product of its three axis phases): no division and no sine
// per cell.
template <bool FAR>
__global__ void __launch_bounds__(kFieldThreads) k_field_partial(FieldArgs a) {
  const int64_t chunk = blockIdx.x, m = blockIdx.y, rhs = blockIdx.z;
  const double* y = a.pts + 3 * (a.m0 + m);
  const double y0 = y[0], y1 = y[1], y2 = y[2];
  const cxd* __restrict__ u = a.u + rhs * a.P;
  const int64_t p0 = chunk * a.chunk, p1 = p0 + a.chunk < a.P ? p0 + a.chunk : a.P;
  const int n = static_cast<int>(a.n);
  __shared__ double xs[3 * kFieldMaxN];
  __shared__ cxd ph[FAR ? 3 * kFieldMaxN : 1];
  for (int t = threadIdx.x; t < 3 * n; t += kFieldThreads) {
    const int d = t / n, i = t - d * n;
    const double x = a.origin[d] + a.side * (static_cast<double>(i) + a.offset) / a.dn;
    xs[t] = x;
    if constexpr (FAR) {
      const double yd = d == 0 ? y0 : d == 1 ? y1 : y2;
      double s, c;
      sincos(-a.k * (yd * x), &s, &c);
      ph[t] = cxd{c, s};
    }
  }
  __syncthreads();
  const double inv_n = 1.0 / a.dn;
  cxd acc{0.0, 0.0};
  for (int64_t p = p0 + threadIdx.x; p < p1; p += kFieldThreads) {
    // p = (i1 n + i2) n + i3
    const int32_t pp = static_cast<int32_t>(p);
    const int32_t r = quot(pp, inv_n), i3 = pp - r * n;
    const int32_t i1 = quot(r, inv_n), i2 = r - i1 * n;
    const cxd q = scale(a.D[p] * u[p], -1.0);  // Q_p
    if (FAR) {
      // e^{-ik beta.x_p} Q_p
      acc = acc + (ph[i1] * ph[n + i2]) * ph[2 * n + i3] * q;
    } else {
      const double d0 = y0 - xs[i1], d1 = y1 - xs[n + i2], d2 = y2 - xs[2 * n + i3];
      const double rsq = d0 * d0 + d1 * d1 + d2 * d2;
      if (rsq > 0.0) {
        // r and 1 / (4 pi r) from one reciprocal square root
        const double ir = rsqrt(rsq), r = rsq * ir;
        double s, c;
        sincos(a.k * r, &s, &c);
        const double g = ir * (1.0 / kFourPi);  // G = e^{ikr} / (4 pi r)
        acc = acc + cxd{c * g, s * g} * q;
      }
    }
  }
  const cxd t = block_sum_cx(acc);
  if (threadIdx.x == 0) a.part[(rhs * a.mb + m) * a.nchunk + chunk] = t;
}

// one thread per (point, right-hand side): chunks in order
__global__ void __launch_bounds__(64) k_field_finalize(FieldArgs a, int32_t far) {
  const int64_t m = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x, rhs = blockIdx.y;
  if (m >= a.mb) return;
  const cxd* part = a.part + (rhs * a.mb + m) * a.nchunk;
  cxd s{0.0, 0.0};
  for (int64_t c = 0; c < a.nchunk; ++c) s = s + part[c];
  if (far) s = scale(s, 1.0 / kFourPi);
  a.out[rhs * a.M + a.m0 + m] = s;
}

__global__ void __launch_bounds__(256) k_charges(const cxd* __restrict__ D, const cxd* __restrict__ u, int64_t P,
                                                 cxd* __restrict__ q) {
  const int64_t off = static_cast<int64_t>(blockIdx.y) * P;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < P;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    q[off + i] = scale(D[i] * u[off + i], -1.0);
}

// z^{1/2} with arg z in [0, 2 pi) (eq. 4.2): the root with Im >= 0, and the
// positive root on the cut [0, +inf).  The larger component comes from a
// square root, the smaller one from |Im z| / (2 * larger), so neither loses
// digits to cancellation.
__device__ __forceinline__ cxd sqrt_upper(cxd z) {
  if (z.re == 0.0 && z.im == 0.0) return cxd{0.0, 0.0};
  const double r = hypot(z.re, z.im), ay = fabs(z.im);
  double re, im;
  if (z.re >= 0.0) {
    re = sqrt(0.5 * (r + z.re));
    im = ay / (2.0 * re);
  } else {
    im = sqrt(0.5 * (r - z.re));
    re = ay / (2.0 * im);
  }
  if (z.im < 0.0) re = -re;  // arg in (pi, 2 pi): Re < 0
  return cxd{re, im};
}

// partials[block] = number of bad entries (N <= 0 or a non-finite input)
__global__ void __launch_bounds__(256) k_refraction(RefractionArgs a) {
  __shared__ double sh[4];
  double bad = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.P;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const cxd n0 = a.n0[i], x = a.in[i];
    const double N = a.N ? a.N[i] : 1.0;
    const bool ok = isfinite(n0.re) && isfinite(n0.im) && isfinite(x.re) && isfinite(x.im) && isfinite(N) &&
                    (a.design ? N > 0.0 : N >= 0.0);
    cxd out{0.0, 0.0};
    if (ok) {
      if (a.design) {
        // h = k^2 (n0^2 - n^2) / (c_S N)  (eqs. 2.25, 2.26)
        out = scale(n0 * n0 - x * x, a.k * a.k / (a.c_s * N));
      } else {
        // n = [n0^2 - c_S h N / k^2]^{1/2}  (eq. 4.1)
        out = sqrt_upper(n0 * n0 - scale(x, a.c_s * N / (a.k * a.k)));
      }
    }
    a.out[i] = out;
    bad += ok ? 0.0 : 1.0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = bad;
  __syncthreads();
  if (threadIdx.x == 0) a.bad[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// One workgroup per coarse cell q: the fine points inside it are those whose
// index i (per axis) has floor((i + off) nc / nf) = q; they lie in a box of
// a few more than nf / nc indices per axis around q nf / nc.
__global__ void __launch_bounds__(kFieldThreads) k_cell_difference(DiffArgs a) {
  const int64_t q = blockIdx.x;
  const int64_t qq[3] = {q / (a.nc * a.nc), (q / a.nc) % a.nc, q % a.nc};
  int64_t lo[3], len[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double dn = static_cast<double>(a.nf), dc = static_cast<double>(a.nc);
    int64_t l = static_cast<int64_t>(floor(static_cast<double>(qq[d]) * dn / dc - a.off)) - 1;
    int64_t h = static_cast<int64_t>(ceil(static_cast<double>(qq[d] + 1) * dn / dc - a.off)) + 2;
    l = l < 0 ? 0 : l;
    h = h > a.nf ? a.nf : h;
    lo[d] = l;
    len[d] = h > l ? h - l : 0;
  }
  const cxd yq = a.y[q];
  const int64_t box = len[0] * len[1] * len[2];
  double sum = 0.0, cnt = 0.0;
  for (int64_t t = threadIdx.x; t < box; t += kFieldThreads) {
    const int64_t i[3] = {lo[0] + t / (len[1] * len[2]), lo[1] + (t / len[2]) % len[1], lo[2] + t % len[2]};
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      in = in && static_cast<int64_t>(floor((static_cast<double>(i[d]) + a.off) * static_cast<double>(a.nc) /
                                            static_cast<double>(a.nf))) == qq[d];
    if (in) {
      const cxd x = a.x[(i[0] * a.nf + i[1]) * a.nf + i[2]];
      sum += hypot(x.re - yq.re, x.im - yq.im);
      cnt += 1.0;
    }
  }
  const cxd t = block_sum_cx(cxd{sum, cnt});
  if (threadIdx.x == 0) a.means[q] = t.im > 0.0 ? t.re / t.im : -1.0;
}

__global__ void __launch_bounds__(256) k_max(const double* __restrict__ v, int64_t P, double* __restrict__ part) {
  __shared__ double sh[4];
  double m = -1.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < P;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    m = fmax(m, v[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

}  // namespace

hipError_t launch_field(const FieldArgs& a, bool far, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (a.n < 1 || a.n > kFieldMaxN || a.n * a.n * a.n != a.P) return hipErrorInvalidValue;  // the axis tables
  const dim3 grid(static_cast<unsigned>(a.nchunk), static_cast<unsigned>(a.mb), static_cast<unsigned>(a.nrhs));
  if (far)
    e = launch_kernel((k_field_partial<true>), grid, dim3(kFieldThreads), st, a);
  else
    e = launch_kernel((k_field_partial<false>), grid, dim3(kFieldThreads), st, a);
  if (e != hipSuccess) return e;
  e = launch_kernel(k_field_finalize, dim3(static_cast<unsigned>((a.mb + 63) / 64), static_cast<unsigned>(a.nrhs)),
                     dim3(64), st, a, far ? 1 : 0);
  return e;
}

hipError_t launch_charges(const void* D, const void* u, int64_t P, int64_t nrhs, void* q, hipStream_t st) {
  hipError_t e = hipSuccess;
  int64_t g = (P + 255) / 256;
  if (g > 8192) g = 8192;
  e = launch_kernel(k_charges, dim3(static_cast<unsigned>(g), static_cast<unsigned>(nrhs)), dim3(256), st,
                     static_cast<const cxd*>(D), static_cast<const cxd*>(u), P, static_cast<cxd*>(q));
  return e;
}

int64_t refraction_blocks(int64_t P) {
  const int64_t g = (P + 255) / 256;
  return g < 1 ? 1 : (g > 1024 ? 1024 : g);
}

hipError_t launch_refraction(const RefractionArgs& a, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_refraction, dim3(static_cast<unsigned>(refraction_blocks(a.P))), dim3(256), st, a);
  return e;
}

int64_t max_blocks(int64_t P) {
  const int64_t g = (P + 255) / 256;
  return g < 1 ? 1 : (g > 1024 ? 1024 : g);
}

hipError_t launch_cell_difference(const DiffArgs& a, int64_t P_coarse, double* part, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_cell_difference, dim3(static_cast<unsigned>(P_coarse)), dim3(kFieldThreads), st, a);
  if (e != hipSuccess) return e;
  e = launch_kernel(k_max, dim3(static_cast<unsigned>(max_blocks(P_coarse))), dim3(256), st, a.means, P_coarse,
                     part);
  return e;
}

}  // namespace ori
