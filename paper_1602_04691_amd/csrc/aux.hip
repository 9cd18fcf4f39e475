// Elementwise and reduction kernels: coefficients (eq. 2.19), the Green's
// table for the spectrum (eqs. 2.6a, 3.3.7 and the padding of Section 3), and
// the COCG vector updates with their bilinear reductions.
#include "cx.h"
#include "kernels.h"

namespace ori {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic workgroup sum of 4 values (kRedThreads threads).
__device__ __forceinline__ void block_sum4(double (&v)[4], double* out) {
  __shared__ double sh[(kRedThreads / 64) * 4];
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = wave_sum(v[j]);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) sh[w * 4 + j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int i = 0; i < kRedThreads / 64; ++i) s += sh[i * 4 + j];
      out[j] = s;
    }
  }
}

// Principal square root of a + ib.
__device__ __forceinline__ cxd csqrt(cxd z) {
  if (z.re == 0.0 && z.im == 0.0) return cxd{0.0, 0.0};
  const double r = hypot(z.re, z.im);
  if (z.re >= 0.0) {
    const double t = sqrt(0.5 * (r + z.re));
    return cxd{t, z.im / (2.0 * t)};
  }
  const double t = sqrt(0.5 * (r - z.re));
  return cxd{fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

__device__ __forceinline__ bool finite_cx(cxd z) { return isfinite(z.re) && isfinite(z.im); }

// a1: D = 4 pi h N vol, S = sqrt(D), b = S u0
__global__ void __launch_bounds__(kRedThreads)
    k_coefficients(const cxd* __restrict__ h, const double* __restrict__ N, const cxd* __restrict__ u0,
                   double vol, int64_t P, cxd* __restrict__ D, cxd* __restrict__ S, cxf* __restrict__ Sf,
                   cxd* __restrict__ b, cxd* __restrict__ u0c, double* __restrict__ partials) {
  constexpr double FOUR_PI = 12.566370614359172954;  // c_S for spheres
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < P; i += stride) {
    const cxd hv = h[i];
    const double nv = N ? N[i] : 1.0;
    const cxd uv = u0[i];
    const bool bad = !finite_cx(hv) || !isfinite(nv) || nv < 0.0 || !finite_cx(uv);
    const cxd d = bad ? cxd{0.0, 0.0} : scale(hv, FOUR_PI * nv * vol);
    const cxd s = csqrt(d);
    const cxd bv = bad ? cxd{0.0, 0.0} : s * uv;
    D[i] = d;
    S[i] = s;
    if (Sf) Sf[i] = cvt<float>(s);
    b[i] = bv;
    u0c[i] = bad ? cxd{0.0, 0.0} : uv;
    acc[0] += norm2(bv);
    acc[1] += bad ? 0.0 : norm2(uv);
    acc[2] += bad ? 1.0 : 0.0;
  }
  block_sum4(acc, partials + 4 * static_cast<int64_t>(blockIdx.x));
}

// Green's table on the padded grid: c(m) = G(spacing |d(m)|) with the
// wrapped offset d_i = m_i (m_i < n), m_i - L (m_i > n); zero at m = 0 (the
// excluded self term) and where some m_i = n (never reached by |j - m| < n).
__global__ void __launch_bounds__(256) k_embed(cxd* __restrict__ g, int L, double k, double spacing) {
  const int n = L / 2;
  const int64_t total = static_cast<int64_t>(L) * L * L;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int m3 = static_cast<int>(idx % L);
    const int m2 = static_cast<int>((idx / L) % L);
    const int m1 = static_cast<int>(idx / (static_cast<int64_t>(L) * L));
    cxd v{0.0, 0.0};
    if (m1 != n && m2 != n && m3 != n && (m1 | m2 | m3) != 0) {
      const double d1 = m1 < n ? m1 : m1 - L;
      const double d2 = m2 < n ? m2 : m2 - L;
      const double d3 = m3 < n ? m3 : m3 - L;
      const double r = spacing * sqrt(d1 * d1 + d2 * d2 + d3 * d3);
      double sn, cs;
      sincos(k * r, &sn, &cs);
      const double inv = 1.0 / (12.566370614359172954 * r);
      v = cxd{cs * inv, sn * inv};
    }
    g[idx] = v;
  }
}

__global__ void __launch_bounds__(256)
    k_octant(const cxd* __restrict__ g, int L, double scale_, cxd* __restrict__ kh, cxf* __restrict__ khf) {
  const int n = L / 2, kp = n + 1;
  const int64_t total = static_cast<int64_t>(kp) * kp * kp;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int64_t m3 = idx % kp, m2 = (idx / kp) % kp, m1 = idx / (static_cast<int64_t>(kp) * kp);
    const cxd v = scale(g[(m1 * L + m2) * L + m3], scale_);
    kh[idx] = v;
    if (khf) khf[idx] = cvt<float>(v);
  }
}

// Reduce nblk partial quadruples in a fixed order and update the scalars.
__global__ void __launch_bounds__(kRedThreads)
    k_finalize(const double* __restrict__ part, int64_t nblk, ScalarBlock* sc, int32_t mode, double eps) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = threadIdx.x; i < nblk; i += kRedThreads) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] += part[4 * i + j];
  }
  __shared__ double tot[4];
  block_sum4(acc, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double s0 = tot[0], s1 = tot[1], s2 = tot[2], s3 = tot[3];
  switch (mode) {
    case FIN_SETUP:
      sc->bb = s0;
      sc->aux = s1;
      sc->flags = s2 > 0.0 ? FLAG_BAD_INPUT : 0;
      break;
    case FIN_INIT: {
      sc->rho_re = s0;
      sc->rho_im = s1;
      sc->rr = s2;
      sc->beta_re = 0.0;
      sc->beta_im = 0.0;
      int f = 0;
      if (s2 == 0.0) f |= FLAG_ZERO_RESIDUAL;
      else if (hypot(s0, s1) <= eps * s2) f |= FLAG_BREAKDOWN_RHO;
      sc->flags = f;
      break;
    }
    case FIN_MU: {
      sc->mu_re = s0;
      sc->mu_im = s1;
      sc->pp = s3;
      sc->qq = s2;
      const double mag = hypot(s0, s1);
      if (s3 == 0.0 || (sc->flags & (FLAG_BREAKDOWN_RHO | FLAG_BREAKDOWN_MU | FLAG_ZERO_RESIDUAL))) {
        sc->alpha_re = 0.0;  // nothing left to do (r = p = 0) or already broken down
        sc->alpha_im = 0.0;
      } else if (mag <= eps * sqrt(s2 * s3)) {
        sc->flags |= FLAG_BREAKDOWN_MU;
        sc->alpha_re = 0.0;
        sc->alpha_im = 0.0;
      } else {
        // alpha = rho / mu
        const double den = s0 * s0 + s1 * s1;
        sc->alpha_re = (sc->rho_re * s0 + sc->rho_im * s1) / den;
        sc->alpha_im = (sc->rho_im * s0 - sc->rho_re * s1) / den;
      }
      break;
    }
    case FIN_RHO: {
      int f = sc->flags;
      if (f & (FLAG_BREAKDOWN_RHO | FLAG_BREAKDOWN_MU)) {
        sc->beta_re = 0.0;
        sc->beta_im = 0.0;
        break;
      }
      const double ro = sc->rho_re, io = sc->rho_im;
      sc->rr = s2;
      if (s2 == 0.0) {
        f |= FLAG_ZERO_RESIDUAL;
        sc->beta_re = 0.0;
        sc->beta_im = 0.0;
      } else if (hypot(s0, s1) <= eps * s2) {
        f |= FLAG_BREAKDOWN_RHO;
        sc->beta_re = 0.0;
        sc->beta_im = 0.0;
      } else {
        const double den = ro * ro + io * io;  // beta = rho' / rho
        sc->beta_re = (s0 * ro + s1 * io) / den;
        sc->beta_im = (s1 * ro - s0 * io) / den;
      }
      sc->rho_re = s0;
      sc->rho_im = s1;
      sc->flags = f;
      break;
    }
    case FIN_NORM:
      sc->aux = s2;
      break;
  }
}

template <typename V>
__global__ void __launch_bounds__(kRedThreads)
    k_update(cx<V>* __restrict__ x, const cx<V>* __restrict__ p, cx<V>* __restrict__ r,
             const cx<V>* __restrict__ q, int64_t P, const ScalarBlock* __restrict__ sc,
             double* __restrict__ partials) {
  const cxd al = {sc->alpha_re, sc->alpha_im};
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < P; i += stride) {
    const cxd pv = cvt<double>(p[i]);
    const cxd xv = cvt<double>(x[i]) + al * pv;
    const cxd rv = cvt<double>(r[i]) - al * cvt<double>(q[i]);
    x[i] = cvt<V>(xv);
    const cx<V> rs = cvt<V>(rv);
    r[i] = rs;
    const cxd rd = cvt<double>(rs);  // reduce what was stored
    const cxd rr = rd * rd;
    acc[0] += rr.re;
    acc[1] += rr.im;
    acc[2] += norm2(rd);
  }
  block_sum4(acc, partials + 4 * static_cast<int64_t>(blockIdx.x));
}

template <typename V>
__global__ void __launch_bounds__(kRedThreads)
    k_init(const cxd* __restrict__ b, double bscale, cx<V>* __restrict__ x, cx<V>* __restrict__ r, int64_t P,
           double* __restrict__ partials) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < P; i += stride) {
    const cx<V> rs = cvt<V>(scale(b[i], bscale));
    r[i] = rs;
    x[i] = cx<V>{};
    const cxd rd = cvt<double>(rs);
    const cxd rr = rd * rd;
    acc[0] += rr.re;
    acc[1] += rr.im;
    acc[2] += norm2(rd);
  }
  block_sum4(acc, partials + 4 * static_cast<int64_t>(blockIdx.x));
}

template <typename VO>
__global__ void __launch_bounds__(256) k_scale_into(const cxd* __restrict__ x, double a, cx<VO>* __restrict__ y,
                                                    int64_t P) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < P; i += stride)
    y[i] = cvt<VO>(scale(x[i], a));
}

template <typename VI>
__global__ void __launch_bounds__(256) k_axpy_d(double a, const cx<VI>* __restrict__ x, cxd* __restrict__ y,
                                                int64_t P) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < P; i += stride)
    y[i] = y[i] + scale(cvt<double>(x[i]), a);
}

__global__ void __launch_bounds__(256) k_mul(const cxd* __restrict__ s, const cxd* __restrict__ x,
                                             cxd* __restrict__ y, int64_t P) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < P; i += stride)
    y[i] = s[i] * x[i];
}

unsigned grid_for(int64_t P, int threads, int64_t cap) {
  int64_t g = (P + threads - 1) / threads;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return static_cast<unsigned>(g);
}

}  // namespace

hipError_t launch_coefficients(const void* h, const double* N, const void* u0, double vol, int64_t P, void* D,
                               void* S, void* Sf, void* b, void* u0c, double* partials, hipStream_t st) {
  hipLaunchKernelGGL(k_coefficients, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<const cxd*>(h), N,
                     static_cast<const cxd*>(u0), vol, P, static_cast<cxd*>(D), static_cast<cxd*>(S),
                     static_cast<cxf*>(Sf), static_cast<cxd*>(b), static_cast<cxd*>(u0c), partials);
  return hipGetLastError();
}

hipError_t launch_embed(void* grid, int L, double k, double spacing, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(L) * L * L;
  hipLaunchKernelGGL(k_embed, dim3(grid_for(total, 256, 1 << 16)), dim3(256), 0, st, static_cast<cxd*>(grid), L, k,
                     spacing);
  return hipGetLastError();
}

hipError_t launch_octant(const void* grid, int L, double scale_, void* kh, void* khf, hipStream_t st) {
  const int64_t kp = L / 2 + 1;
  hipLaunchKernelGGL(k_octant, dim3(grid_for(kp * kp * kp, 256, 1 << 16)), dim3(256), 0, st,
                     static_cast<const cxd*>(grid), L, scale_, static_cast<cxd*>(kh), static_cast<cxf*>(khf));
  return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int64_t nblk, ScalarBlock* sc, int32_t mode, double eps,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, st, partials, nblk, sc, mode, eps);
  return hipGetLastError();
}

hipError_t launch_update(int prec, void* x, const void* p, void* r, const void* q, int64_t P, const ScalarBlock* sc,
                         double* partials, hipStream_t st) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(k_update<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<cxd*>(x),
                       static_cast<const cxd*>(p), static_cast<cxd*>(r), static_cast<const cxd*>(q), P, sc, partials);
  else
    hipLaunchKernelGGL(k_update<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<cxf*>(x),
                       static_cast<const cxf*>(p), static_cast<cxf*>(r), static_cast<const cxf*>(q), P, sc, partials);
  return hipGetLastError();
}

hipError_t launch_init(int prec, const void* b, double bscale, void* x, void* r, int64_t P, double* partials,
                       hipStream_t st) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(k_init<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<const cxd*>(b), bscale,
                       static_cast<cxd*>(x), static_cast<cxd*>(r), P, partials);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<const cxd*>(b), bscale,
                       static_cast<cxf*>(x), static_cast<cxf*>(r), P, partials);
  return hipGetLastError();
}

hipError_t launch_scale_into(int prec_out, const void* x, double a, void* y, int64_t P, hipStream_t st) {
  const dim3 g(grid_for(P, 256, 8192));
  if (prec_out == PREC_F64)
    hipLaunchKernelGGL(k_scale_into<double>, g, dim3(256), 0, st, static_cast<const cxd*>(x), a,
                       static_cast<cxd*>(y), P);
  else
    hipLaunchKernelGGL(k_scale_into<float>, g, dim3(256), 0, st, static_cast<const cxd*>(x), a,
                       static_cast<cxf*>(y), P);
  return hipGetLastError();
}

hipError_t launch_axpy_d(int prec_in, double a, const void* x, void* y, int64_t P, hipStream_t st) {
  const dim3 g(grid_for(P, 256, 8192));
  if (prec_in == PREC_F64)
    hipLaunchKernelGGL(k_axpy_d<double>, g, dim3(256), 0, st, a, static_cast<const cxd*>(x), static_cast<cxd*>(y), P);
  else
    hipLaunchKernelGGL(k_axpy_d<float>, g, dim3(256), 0, st, a, static_cast<const cxf*>(x), static_cast<cxd*>(y), P);
  return hipGetLastError();
}

hipError_t launch_mul(const void* s, const void* x, void* y, int64_t P, hipStream_t st) {
  hipLaunchKernelGGL(k_mul, dim3(grid_for(P, 256, 8192)), dim3(256), 0, st, static_cast<const cxd*>(s),
                     static_cast<const cxd*>(x), static_cast<cxd*>(y), P);
  return hipGetLastError();
}

}  // namespace ori
