// Elementwise and reduction kernels: coefficients of eq. 2.19, the
// right-hand sides, and the COCG vector updates with their bilinear
// reductions.  Reductions are two-stage and deterministic: fixed-order
// per-workgroup partials, then one workgroup per right-hand side
// (k_finalize) in a fixed order.
#include "cx.h"
#include "kernels.h"
#include "launch.h"

namespace ori {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic workgroup sum of 4 values (kRedThreads threads); thread 0
// writes out[0..3].
template <int NT = kRedThreads>
__device__ __forceinline__ void block_sum4(double (&v)[4], double* out) {
  __shared__ double sh[(NT / 64) * 4];
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
      for (int i = 0; i < NT / 64; ++i) s += sh[i * 4 + j];
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

// grid-stride loop over [0, P) within the right-hand side blockIdx.y
#define ORI_RHS_LOOP(i)                                                                                \
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < P;                 \
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)

// a1, operator part: D = 4 pi h N vol, S = sqrt(D), c = 4 pi N vol.
// Partials per workgroup: {bad-input count, min |S|^2, max |S|^2, 0}.
__global__ void __launch_bounds__(kRedThreads)
    k_coefficients(const cxd* __restrict__ h, const double* __restrict__ N, double vol, int64_t P,
                   cxd* __restrict__ D, cxd* __restrict__ S, cxf* __restrict__ Sf, double* __restrict__ cN,
                   double* __restrict__ partials) {
  constexpr double FOUR_PI = 12.566370614359172954;  // c_S for spheres
  double bad_n = 0.0, mn = INFINITY, mx = 0.0;
  ORI_RHS_LOOP(i) {
    const cxd hv = h[i];
    const double nv = N ? N[i] : 1.0;
    const bool bad = !finite_cx(hv) || !isfinite(nv) || nv < 0.0;
    const double c = bad ? 0.0 : FOUR_PI * nv * vol;
    const cxd d = scale(bad ? cxd{0.0, 0.0} : hv, c);
    const cxd s = csqrt(d);
    D[i] = d;
    S[i] = s;
    if (Sf) Sf[i] = cvt<float>(s);
    cN[i] = c;
    bad_n += bad ? 1.0 : 0.0;
    const double s2 = norm2(s);
    mn = fmin(mn, s2);
    mx = fmax(mx, s2);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    bad_n += __shfl_xor(bad_n, off, 64);
    mn = fmin(mn, __shfl_xor(mn, off, 64));
    mx = fmax(mx, __shfl_xor(mx, off, 64));
  }
  __shared__ double sh[(kRedThreads / 64) * 3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[3 * w] = bad_n;
    sh[3 * w + 1] = mn;
    sh[3 * w + 2] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kRedThreads / 64; ++i) {
      sh[0] += sh[3 * i];
      sh[1] = fmin(sh[1], sh[3 * i + 1]);
      sh[2] = fmax(sh[2], sh[3 * i + 2]);
    }
    double* out = partials + 4 * static_cast<int64_t>(blockIdx.x);
    out[0] = sh[0];
    out[1] = sh[1];
    out[2] = sh[2];
    out[3] = 0.0;
  }
}

// {bad count, min |S|^2, max |S|^2} over nblk partials -> sc[0]; one
// workgroup, strided over the partials, then a fixed-order combine (the
// count is a sum of small integers, so the order does not matter anyway)
__global__ void __launch_bounds__(kRedThreads) k_finalize_coeff(const double* __restrict__ part, int64_t nblk,
                                                                ScalarBlock* sc) {
  double bad = 0.0, mn = INFINITY, mx = 0.0;
  for (int64_t i = threadIdx.x; i < nblk; i += kRedThreads) {
    bad += part[4 * i];
    mn = fmin(mn, part[4 * i + 1]);
    mx = fmax(mx, part[4 * i + 2]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    bad += __shfl_xor(bad, off, 64);
    mn = fmin(mn, __shfl_xor(mn, off, 64));
    mx = fmax(mx, __shfl_xor(mx, off, 64));
  }
  __shared__ double sh[(kRedThreads / 64) * 3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[3 * w] = bad;
    sh[3 * w + 1] = mn;
    sh[3 * w + 2] = mx;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = 1; i < kRedThreads / 64; ++i) {
    sh[0] += sh[3 * i];
    sh[1] = fmin(sh[1], sh[3 * i + 1]);
    sh[2] = fmax(sh[2], sh[3 * i + 2]);
  }
  sc->flags = sh[0] > 0.0 ? FLAG_BAD_COEFF : 0;
  sc->s2_min = sh[1];
  sc->s2_max = sh[2];
}

// u = w / S, per right-hand side (S shared)
__global__ void __launch_bounds__(256) k_div(const cxd* __restrict__ w, const cxd* __restrict__ s,
                                             cxd* __restrict__ u, int64_t P) {
  const int64_t off = static_cast<int64_t>(blockIdx.y) * P;
  ORI_RHS_LOOP(i) {
    const cxd d = s[i];
    const double inv = 1.0 / norm2(d);
    u[off + i] = scale(w[off + i] * conj(d), inv);
  }
}

// q = (z + r) / S (one right-hand side; S nonzero), the division as in k_div
__global__ void __launch_bounds__(256) k_add_div(const cxd* __restrict__ z, const cxd* __restrict__ r,
                                                 const cxd* __restrict__ s, cxd* __restrict__ q, int64_t P) {
  ORI_RHS_LOOP(i) {
    const cxd d = s[i];
    const double inv = 1.0 / norm2(d);
    q[i] = scale((z[i] + r[i]) * conj(d), inv);
  }
}

// u = w / S as k_div, and the partials {-, -, ||r / S||^2, -} per
// right-hand side (red_grid): with r = b - (I + S G0 S) w and b = S u0,
// r / S = u0 - u - G0 D u, the residual of eq. 2.19 for u = w / S
__global__ void __launch_bounds__(kRedThreads)
    k_div_res(const cxd* __restrict__ w, const cxd* __restrict__ r, const cxd* __restrict__ s, cxd* __restrict__ u,
              int64_t P, double* __restrict__ partials) {
  const int64_t off = static_cast<int64_t>(blockIdx.y) * P;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  ORI_RHS_LOOP(i) {
    const cxd d = s[i];
    const double inv = 1.0 / norm2(d);
    u[off + i] = scale(w[off + i] * conj(d), inv);
    acc[2] += norm2(scale(r[off + i] * conj(d), inv));
  }
  block_sum4(acc, partials + 4 * (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x));
}

// a1, right-hand sides: b = S u0 (one batch row per blockIdx.y)
__global__ void __launch_bounds__(kRedThreads)
    k_rhs(const cxd* __restrict__ u0, const cxd* __restrict__ S, int64_t P, cxd* __restrict__ b,
          cxd* __restrict__ u0c, double* __restrict__ partials) {
  const int64_t off = static_cast<int64_t>(blockIdx.y) * P;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  ORI_RHS_LOOP(i) {
    const cxd uv = u0[off + i];
    const bool bad = !finite_cx(uv);
    const cxd bv = bad ? cxd{0.0, 0.0} : S[i] * uv;
    b[off + i] = bv;
    u0c[off + i] = bad ? cxd{0.0, 0.0} : uv;
    acc[0] += norm2(bv);
    acc[1] += bad ? 0.0 : norm2(uv);
    acc[2] += bad ? 1.0 : 0.0;
  }
  block_sum4(acc, partials + 4 * (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x));
}

// One workgroup per right-hand side: reduce its nblk partial quadruples in a
// fixed order and update its scalars.  1024 threads: after the I1 pass there
// is one quadruple per I1 workgroup (16 384 at n = 256).
constexpr int kFinThreads = 1024;
__device__ __forceinline__ void finalize_body(const double* __restrict__ partials, int64_t nblk, ScalarBlock* scb,
                                              int64_t rhs, int32_t mode, double eps, double tol2, int32_t tol2_of_bb,
                                              const double* __restrict__ tol2_rhs) {
  const double* part = partials + 4 * nblk * rhs;
  ScalarBlock* sc = scb + rhs;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = threadIdx.x; i < nblk; i += kFinThreads) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] += part[4 * i + j];
  }
  __shared__ double tot[4];
  block_sum4<kFinThreads>(acc, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double s0 = tot[0], s1 = tot[1], s2 = tot[2], s3 = tot[3];
  switch (mode) {
    case FIN_SETUP:
      sc->bb = s0;
      sc->aux = s1;
      // keeps the coefficient check of sc[0] (k_finalize_coeff, earlier on
      // the stream), so that one copy to the host brings both
      sc->flags = (sc->flags & FLAG_BAD_COEFF) | (s2 > 0.0 ? FLAG_BAD_INPUT : 0);
      break;
    case FIN_INIT: {
      sc->rho_re = s0;
      sc->rho_im = s1;
      sc->rr = s2;
      sc->rr0 = s2;
      sc->beta_re = 0.0;
      sc->beta_im = 0.0;
      sc->alpha_re = 0.0;
      sc->alpha_im = 0.0;
      sc->iters = 0;
      sc->rr_target = (tol2_rhs ? tol2_rhs[rhs] : tol2) * (tol2_of_bb ? sc->bb : s2);
      int f = 0;
      if (s2 == 0.0) f |= FLAG_ZERO_RESIDUAL;
      else if (s2 <= sc->rr_target) f |= FLAG_CONVERGED;
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
      if (s3 == 0.0 || (sc->flags & FLAG_DONE)) {
        sc->alpha_re = 0.0;  // converged, r = p = 0, or broken down: nothing moves
        sc->alpha_im = 0.0;
      } else if (mag <= eps * sqrt(s2 * s3)) {
        sc->flags |= FLAG_BREAKDOWN_MU;
        sc->alpha_re = 0.0;
        sc->alpha_im = 0.0;
      } else {
        const double den = s0 * s0 + s1 * s1;  // alpha = rho / mu
        sc->alpha_re = (sc->rho_re * s0 + sc->rho_im * s1) / den;
        sc->alpha_im = (sc->rho_im * s0 - sc->rho_re * s1) / den;
      }
      break;
    }
    case FIN_RHO: {
      int f = sc->flags;
      if (f & FLAG_DONE) {  // frozen
        sc->beta_re = 0.0;
        sc->beta_im = 0.0;
        break;
      }
      sc->iters += 1;
      const double ro = sc->rho_re, io = sc->rho_im;
      sc->rr = s2;
      sc->beta_re = 0.0;
      sc->beta_im = 0.0;
      if (s2 == 0.0) {
        f |= FLAG_ZERO_RESIDUAL;
      } else if (s2 <= sc->rr_target) {
        f |= FLAG_CONVERGED;
      } else if (hypot(s0, s1) <= eps * s2) {
        f |= FLAG_BREAKDOWN_RHO;
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

__global__ void __launch_bounds__(kFinThreads)
    k_finalize(const double* __restrict__ partials, int64_t nblk, ScalarBlock* scb, int32_t mode, double eps,
               double tol2, int32_t tol2_of_bb, const double* __restrict__ tol2_rhs) {
  finalize_body(partials, nblk, scb, blockIdx.x, mode, eps, tol2, tol2_of_bb, tol2_rhs);
}

// workgroup bid of nb over right-hand side rhs
template <typename V>
__device__ __forceinline__ void update_body(cx<V>* __restrict__ x, const cx<V>* __restrict__ p, cx<V>* __restrict__ r,
                                            const cx<V>* __restrict__ q, int64_t P,
                                            const ScalarBlock* __restrict__ scb, double* __restrict__ partials,
                                            int64_t bid, int64_t nb, int64_t rhs) {
  const ScalarBlock* sc = scb + rhs;
  const int64_t off = rhs * P;
  const cxd al = {sc->alpha_re, sc->alpha_im};
  const bool moving = al.re != 0.0 || al.im != 0.0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = bid * blockDim.x + threadIdx.x; i < P; i += nb * blockDim.x) {
    cxd rd;
    if (moving) {
      if (x) x[off + i] = cvt<V>(cfma(al, cvt<double>(p[off + i]), cvt<double>(x[off + i])));
      const cx<V> rs = cvt<V>(cfms(al, cvt<double>(q[off + i]), cvt<double>(r[off + i])));
      r[off + i] = rs;
      rd = cvt<double>(rs);  // reduce what was stored
    } else {
      rd = cvt<double>(r[off + i]);
    }
    const cxd rr = rd * rd;
    acc[0] += rr.re;
    acc[1] += rr.im;
    acc[2] += norm2(rd);
  }
  block_sum4(acc, partials + 4 * (rhs * nb + bid));
}

template <typename V>
__global__ void __launch_bounds__(kRedThreads)
    k_update(cx<V>* __restrict__ x, const cx<V>* __restrict__ p, cx<V>* __restrict__ r,
             const cx<V>* __restrict__ q, int64_t P, const ScalarBlock* __restrict__ scb,
             double* __restrict__ partials) {
  update_body<V>(x, p, r, q, P, scb, partials, blockIdx.x, gridDim.x, blockIdx.y);
}

// The finalisation and the update of several problems in one launch
// (MultiFin, MultiUpd): workgroup b belongs to the problem whose range of
// workgroups holds it, and runs that problem's workgroup b - first_block.
template <typename E>
__device__ __forceinline__ int find_problem(const E* __restrict__ tab, int32_t np, int64_t b) {
  int p = 0;
  while (p + 1 < np && tab[p + 1].first_block <= b) ++p;
  return p;
}

__global__ void __launch_bounds__(kFinThreads)
    k_multi_finalize(const MultiFin* __restrict__ tab, int32_t np, int32_t mode, double eps) {
  const MultiFin& m = tab[find_problem(tab, np, blockIdx.x)];
  finalize_body(m.partials, m.nblk, m.sc, blockIdx.x - m.first_block, mode, eps, 0.0, 0, nullptr);
}

// Every guard band of a workspace block in one launch: workgroup i fills
// band i with 16-byte stores (kGuardBandBytes / 16 = 256 threads).
static_assert(kGuardBandBytes == 256 * 16, "one 16-byte store per thread and band");
__global__ void __launch_bounds__(256) k_fill_guards(GuardBands g) {
  const uint32_t b = g.v & 0xFFu;
  const uint32_t w = b | (b << 8) | (b << 16) | (b << 24);
  uint4* band = reinterpret_cast<uint4*>(static_cast<unsigned char*>(g.base) + g.off[blockIdx.x]);
  band[threadIdx.x] = make_uint4(w, w, w, w);
}

// The scalar blocks of several problems (one right-hand side each, the sc
// of each MultiFin entry) copied into out[0..np), host memory the device
// writes, so that one wait brings every problem's scalars to the host.
static_assert(sizeof(ScalarBlock) % sizeof(double) == 0, "scalar blocks are whole doubles");
__global__ void __launch_bounds__(64) k_gather_scalars(const MultiFin* __restrict__ tab, int32_t np, ScalarBlock* out) {
  constexpr int W = static_cast<int>(sizeof(ScalarBlock) / sizeof(double));
  for (int i = threadIdx.x; i < np * W; i += blockDim.x) {
    const int p = i / W, w = i - p * W;
    reinterpret_cast<double*>(out + p)[w] = reinterpret_cast<const double*>(tab[p].sc)[w];
  }
}

template <typename V>
__global__ void __launch_bounds__(kRedThreads) k_multi_update(const MultiUpd* __restrict__ tab, int32_t np) {
  const MultiUpd& m = tab[find_problem(tab, np, blockIdx.x)];
  update_body<V>(nullptr, static_cast<const cx<V>*>(m.p), static_cast<cx<V>*>(m.r), static_cast<const cx<V>*>(m.q),
                 m.P, m.sc, m.partials, blockIdx.x - m.first_block, m.nblocks, 0);
}

template <typename V>
__global__ void __launch_bounds__(256)
    k_x_flush(cx<V>* __restrict__ x, const cx<V>* __restrict__ p, int64_t P, const ScalarBlock* __restrict__ scb) {
  const ScalarBlock* sc = scb + blockIdx.y;
  const int64_t off = static_cast<int64_t>(blockIdx.y) * P;
  const cxd al = {sc->alpha_re, sc->alpha_im};
  if (al.re == 0.0 && al.im == 0.0) return;
  ORI_RHS_LOOP(i) x[off + i] = cvt<V>(cfma(al, cvt<double>(p[off + i]), cvt<double>(x[off + i])));
}

template <typename V>
__global__ void __launch_bounds__(kRedThreads)
    k_init(const cxd* __restrict__ b, const double* __restrict__ m, cx<V>* __restrict__ x, cx<V>* __restrict__ r,
           int64_t P, double* __restrict__ partials) {
  const int64_t off = static_cast<int64_t>(blockIdx.y) * P;
  double sc = 1.0;
  if (m) sc = m[blockIdx.y] > 0.0 ? 1.0 / m[blockIdx.y] : 0.0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  ORI_RHS_LOOP(i) {
    const cx<V> rs = cvt<V>(scale(b[off + i], sc));
    r[off + i] = rs;
    x[off + i] = cx<V>{};
    const cxd rd = cvt<double>(rs);
    const cxd rr = rd * rd;
    acc[0] += rr.re;
    acc[1] += rr.im;
    acc[2] += norm2(rd);
  }
  block_sum4(acc, partials + 4 * (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x));
}

template <typename VI>
__global__ void __launch_bounds__(256)
    k_axpy_batch(const double* __restrict__ m, const cx<VI>* __restrict__ x, cxd* __restrict__ y, int64_t P) {
  const int64_t off = static_cast<int64_t>(blockIdx.y) * P;
  const double a = m[blockIdx.y];
  if (a == 0.0) return;
  ORI_RHS_LOOP(i) y[off + i] = y[off + i] + scale(cvt<double>(x[off + i]), a);
}

__global__ void __launch_bounds__(256) k_mul(const cxd* __restrict__ s, const cxd* __restrict__ x,
                                             cxd* __restrict__ y, int64_t P) {
  const int64_t off = static_cast<int64_t>(blockIdx.y) * P;
  ORI_RHS_LOOP(i) y[off + i] = s[i] * x[off + i];
}

__global__ void __launch_bounds__(kRedThreads)
    k_conj_diff(const cxd* __restrict__ u, const cxd* __restrict__ t, cxd* __restrict__ f, int64_t P,
                double* __restrict__ partials) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  ORI_RHS_LOOP(i) {
    const cxd e = u[i] - t[i];
    f[i] = conj(e);
    acc[2] += norm2(e);
  }
  block_sum4(acc, partials + 4 * static_cast<int64_t>(blockIdx.x));
}

__global__ void __launch_bounds__(256) k_gradient(const double* __restrict__ c, const cxd* __restrict__ u,
                                                  const cxd* __restrict__ q, double alpha, cxd* __restrict__ g,
                                                  int64_t P) {
  ORI_RHS_LOOP(i) g[i] = scale(u[i] * q[i], alpha * c[i]);
}

__global__ void __launch_bounds__(256) k_sub_mul(const cxd* __restrict__ f, const cxd* __restrict__ s,
                                                 const cxd* __restrict__ x, cxd* __restrict__ y, int64_t P) {
  ORI_RHS_LOOP(i) y[i] = f[i] - s[i] * x[i];
}

// Twiddles exp(-2 pi i m / L), m < L, in FP64 and FP32, exact at the
// quarter turns (the device counterpart of the host's long double table).
__global__ void __launch_bounds__(256) k_twiddles(int64_t L, cxd* __restrict__ twd, cxf* __restrict__ twf) {
  const int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= L) return;
  double cs, sn;
  if ((4 * m) % L == 0) {
    const int64_t q = 4 * m / L;
    cs = q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0);
    sn = q == 1 ? 1.0 : (q == 3 ? -1.0 : 0.0);
  } else {
    sincospi(2.0 * static_cast<double>(m) / static_cast<double>(L), &sn, &cs);
  }
  twd[m] = cxd{cs, -sn};
  twf[m] = cxf{static_cast<float>(cs), static_cast<float>(-sn)};
}

unsigned grid_for(int64_t P, int threads, int64_t cap) {
  int64_t g = (P + threads - 1) / threads;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return static_cast<unsigned>(g);
}

dim3 red_grid(int64_t P, int64_t nrhs, int64_t cap = kRedBlocksMax) {
  return dim3(static_cast<unsigned>(red_blocks(P, cap)), static_cast<unsigned>(nrhs));
}

}  // namespace

hipError_t launch_coefficients(const void* h, const double* N, double vol, int64_t P, void* D, void* S, void* Sf,
                               double* cN, double* partials, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_coefficients, red_grid(P, 1), dim3(kRedThreads), st, static_cast<const cxd*>(h), N, vol, P,
                     static_cast<cxd*>(D), static_cast<cxd*>(S), static_cast<cxf*>(Sf), cN, partials);
  return e;
}

hipError_t launch_finalize_coeff(const double* partials, int64_t nblk, ScalarBlock* sc, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_finalize_coeff, dim3(1), dim3(kRedThreads), st, partials, nblk, sc);
  return e;
}

hipError_t launch_div(const void* w, const void* s, void* u, int64_t P, int64_t nrhs, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_div, dim3(grid_for(P, 256, 8192), static_cast<unsigned>(nrhs)), dim3(256), st,
                     static_cast<const cxd*>(w), static_cast<const cxd*>(s), static_cast<cxd*>(u), P);
  return e;
}

hipError_t launch_add_div(const void* z, const void* r, const void* s, void* q, int64_t P, hipStream_t st) {
  return launch_kernel(k_add_div, dim3(grid_for(P, 256, 8192), 1u), dim3(256), st, static_cast<const cxd*>(z),
                       static_cast<const cxd*>(r), static_cast<const cxd*>(s), static_cast<cxd*>(q), P);
}

hipError_t launch_div_res(const void* w, const void* r, const void* s, void* u, int64_t P, int64_t nrhs,
                          double* partials, hipStream_t st) {
  return launch_kernel(k_div_res, red_grid(P, nrhs), dim3(kRedThreads), st, static_cast<const cxd*>(w),
                       static_cast<const cxd*>(r), static_cast<const cxd*>(s), static_cast<cxd*>(u), P, partials);
}

hipError_t launch_rhs(const void* u0, const void* S, int64_t P, int64_t nrhs, void* b, void* u0c, double* partials,
                      hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_rhs, red_grid(P, nrhs), dim3(kRedThreads), st, static_cast<const cxd*>(u0),
                     static_cast<const cxd*>(S), P, static_cast<cxd*>(b), static_cast<cxd*>(u0c), partials);
  return e;
}

hipError_t launch_finalize(const double* partials, int64_t nblk, int64_t nrhs, ScalarBlock* sc, int32_t mode,
                           double eps, double tol2, int32_t tol2_of_bb, const double* tol2_rhs, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_finalize, dim3(static_cast<unsigned>(nrhs)), dim3(kFinThreads), st, partials, nblk, sc,
                     mode, eps, tol2, tol2_of_bb, tol2_rhs);
  return e;
}

hipError_t launch_update(int prec, void* x, const void* p, void* r, const void* q, int64_t P, int64_t nrhs,
                         const ScalarBlock* sc, double* partials, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (prec == PREC_F64)
    e = launch_kernel(k_update<double>, red_grid(P, nrhs), dim3(kRedThreads), st, static_cast<cxd*>(x),
                       static_cast<const cxd*>(p), static_cast<cxd*>(r), static_cast<const cxd*>(q), P, sc, partials);
  else
    e = launch_kernel(k_update<float>, red_grid(P, nrhs, kUpdateBlocksMaxF32), dim3(kRedThreads), st, static_cast<cxf*>(x),
                       static_cast<const cxf*>(p), static_cast<cxf*>(r), static_cast<const cxf*>(q), P, sc, partials);
  return e;
}

hipError_t launch_multi_finalize(const MultiFin* tab, int32_t np, int64_t blocks, int32_t mode, double eps,
                                 hipStream_t st) {
  if (np < 1 || blocks < 1) return hipErrorInvalidValue;
  return launch_kernel(k_multi_finalize, dim3(static_cast<unsigned>(blocks)), dim3(kFinThreads), st, tab, np, mode,
                       eps);
}

hipError_t launch_fill_guards(const GuardBands& g, hipStream_t st) {
  if (g.count < 0 || g.count > kMaxGuardBands || !g.base) return hipErrorInvalidValue;
  for (int i = 0; i < g.count; ++i)
    if (g.off[i] < 0 || g.off[i] % 16 != 0) return hipErrorInvalidValue;
  if (g.count == 0) return hipSuccess;
  return launch_kernel(k_fill_guards, dim3(static_cast<unsigned>(g.count)), dim3(256), st, g);
}

hipError_t launch_gather_scalars(const MultiFin* tab, int32_t np, ScalarBlock* out, hipStream_t st) {
  if (np < 1) return hipErrorInvalidValue;
  return launch_kernel(k_gather_scalars, dim3(1), dim3(64), st, tab, np, out);
}

hipError_t launch_multi_update(int prec, const MultiUpd* tab, int32_t np, int64_t blocks, hipStream_t st) {
  if (np < 1 || blocks < 1) return hipErrorInvalidValue;
  if (prec == PREC_F64)
    return launch_kernel(k_multi_update<double>, dim3(static_cast<unsigned>(blocks)), dim3(kRedThreads), st, tab, np);
  return launch_kernel(k_multi_update<float>, dim3(static_cast<unsigned>(blocks)), dim3(kRedThreads), st, tab, np);
}

hipError_t launch_x_flush(int prec, void* x, const void* p, int64_t P, int64_t nrhs, const ScalarBlock* sc,
                          hipStream_t st) {
  hipError_t e = hipSuccess;
  const dim3 g(static_cast<unsigned>(grid_for(P, 256, 8192)), static_cast<unsigned>(nrhs));
  if (prec == PREC_F64)
    e = launch_kernel(k_x_flush<double>, g, dim3(256), st, static_cast<cxd*>(x), static_cast<const cxd*>(p), P,
                       sc);
  else
    e = launch_kernel(k_x_flush<float>, g, dim3(256), st, static_cast<cxf*>(x), static_cast<const cxf*>(p), P,
                       sc);
  return e;
}

hipError_t launch_init(int prec, const void* b, const double* m, void* x, void* r, int64_t P, int64_t nrhs,
                       double* partials, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (prec == PREC_F64)
    e = launch_kernel(k_init<double>, red_grid(P, nrhs), dim3(kRedThreads), st, static_cast<const cxd*>(b), m,
                       static_cast<cxd*>(x), static_cast<cxd*>(r), P, partials);
  else
    e = launch_kernel(k_init<float>, red_grid(P, nrhs), dim3(kRedThreads), st, static_cast<const cxd*>(b), m,
                       static_cast<cxf*>(x), static_cast<cxf*>(r), P, partials);
  return e;
}

hipError_t launch_axpy_batch(int prec_in, const double* m, const void* x, void* y, int64_t P, int64_t nrhs,
                             hipStream_t st) {
  hipError_t e = hipSuccess;
  const dim3 g(grid_for(P, 256, 8192), static_cast<unsigned>(nrhs));
  if (prec_in == PREC_F64)
    e = launch_kernel(k_axpy_batch<double>, g, dim3(256), st, m, static_cast<const cxd*>(x),
                       static_cast<cxd*>(y), P);
  else
    e = launch_kernel(k_axpy_batch<float>, g, dim3(256), st, m, static_cast<const cxf*>(x), static_cast<cxd*>(y),
                       P);
  return e;
}

hipError_t launch_mul(const void* s, const void* x, void* y, int64_t P, int64_t nrhs, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_mul, dim3(grid_for(P, 256, 8192), static_cast<unsigned>(nrhs)), dim3(256), st,
                     static_cast<const cxd*>(s), static_cast<const cxd*>(x), static_cast<cxd*>(y), P);
  return e;
}

hipError_t launch_conj_diff(const void* u, const void* t, void* f, int64_t P, double* partials, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_conj_diff, red_grid(P, 1), dim3(kRedThreads), st, static_cast<const cxd*>(u),
                     static_cast<const cxd*>(t), static_cast<cxd*>(f), P, partials);
  return e;
}

hipError_t launch_gradient(const double* c, const void* u, const void* q, double alpha, void* g, int64_t P,
                           hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_gradient, dim3(grid_for(P, 256, 8192)), dim3(256), st, c, static_cast<const cxd*>(u),
                     static_cast<const cxd*>(q), alpha, static_cast<cxd*>(g), P);
  return e;
}

hipError_t launch_sub_mul(const void* f, const void* s, const void* x, void* lam, int64_t P, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_sub_mul, dim3(grid_for(P, 256, 8192)), dim3(256), st, static_cast<const cxd*>(f),
                     static_cast<const cxd*>(s), static_cast<const cxd*>(x), static_cast<cxd*>(lam), P);
  return e;
}

hipError_t launch_twiddles(int64_t L, void* twd, void* twf, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = launch_kernel(k_twiddles, dim3(static_cast<unsigned>((L + 255) / 256)), dim3(256), st, L, static_cast<cxd*>(twd),
                    static_cast<cxf*>(twf));
  return e;
}

}  // namespace ori
