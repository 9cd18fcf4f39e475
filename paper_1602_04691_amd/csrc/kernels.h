// Launch interface between the host runtime and the kernel translation units.
// Plain structs of device pointers and sizes; no torch types.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ori {

// COCG scalars, resident in device memory for the whole solve (the host only
// reads them at convergence checks).  rho = r^T r and mu = p^T A p use the
// unconjugated bilinear form of COCG.
struct ScalarBlock {
  double rho_re, rho_im;      // r^T r of the current residual
  double mu_re, mu_im;        // p^T q
  double alpha_re, alpha_im;  // rho / mu
  double beta_re, beta_im;    // rho_new / rho_old
  double rr;                  // ||r||^2
  double bb;                  // ||b||^2 (set by the init reduction)
  double pp, qq;              // ||p||^2, ||q||^2 of the last product
  double aux;                 // free slot for one-off reductions (||u0||^2, residual norms)
  double pad0, pad1, pad2;
  int32_t flags;              // FLAG_* below
  int32_t pad3;
};

enum : int32_t {
  FLAG_BREAKDOWN_RHO = 1,  // r^T r ~ 0 while r != 0
  FLAG_BREAKDOWN_MU = 2,   // p^T A p ~ 0 while p != 0
  FLAG_ZERO_RESIDUAL = 4,  // r == 0 exactly: converged
  FLAG_BAD_INPUT = 8,      // NaN / Inf / negative N met in ori_load
};

enum Prec : int { PREC_F64 = 0, PREC_F32 = 1 };

// F1: forward DFT along the contiguous axis, with the prologue
//   PLAIN: v = s_in * x            (s_in NULL means 1)
//   COCG : p = r + beta p (p = r on the first iteration), stored; v = s_in * p
struct ContigFwdArgs {
  const void* x;        // PLAIN input / COCG residual r        (vector type V)
  void* pvec;           // COCG search direction, updated in place (V)
  const void* s_in;     // diagonal scale (V) or NULL
  const ScalarBlock* sc;
  int32_t mode;         // 0 PLAIN, 1 COCG
  int32_t first;        // COCG: first iteration
  int32_t half_in;      // 1: only the first L/2 entries of each pencil are input (zero padding)
  int32_t pad;
  void* out;            // FFT type T, out[pencil * out_pitch + e]
  int64_t npencils, in_pitch, out_pitch;
  const void* tw;       // L twiddles exp(-2 pi i m / L) in type T
};

// I1: inverse DFT along the contiguous axis, keep e < n, epilogue
//   y = c0 a0 + c1 a1 + cc (s_out * conv)     (NULL operands are skipped; s_out NULL = 1)
// and optional per-workgroup partials {dot.re, dot.im, |y|^2, |a0|^2}, with
// dot = sum a0_j y_j (dot_self = 0) or sum y_j y_j (dot_self = 1), unconjugated.
struct ContigInvArgs {
  const void* in;       // T, in[pencil * in_pitch + e]
  void* y;              // V, y[pencil * out_pitch + e], e < out_pitch
  const void* a0;
  const void* a1;
  const void* s_out;
  double c0, c1, cc;
  double* partials;     // 4 doubles per workgroup, or NULL
  int32_t dot_self;
  int32_t pad;
  int64_t npencils, in_pitch, out_pitch;
  const void* tw;
};

// F2 / I2 / the spectrum passes: DFT along a strided axis.  Pencil (o, c)
// element e lives at  o * outer + e * axis + c,  c in [0, C) contiguous.
struct StridedArgs {
  const void* in;
  void* out;
  int64_t n_outer, C;
  int64_t in_outer, in_axis, out_outer, out_axis;
  int32_t inverse, half_in, half_out, pad;
  const void* tw;
};

// Z: forward DFT along the slowest axis (first n inputs), multiply by the
// kernel spectrum, inverse DFT, keep the first n outputs; in place.
// Pencil (o = k2, c = k3), element e = i1 / k1 at  e * axis + o * outer + c.
struct ZArgs {
  void* buf;
  int64_t n_outer, C, axis, outer;
  const void* khat;     // octant [0..n]^3 of the spectrum (T), pitch kp = n + 1
  int64_t kp;
  const void* tw;
};

// Per-length launchers (one translation unit per L, see passes.hip).
struct LengthKernels {
  int L;
  hipError_t (*contig_fwd)(int vprec, int fprec, const ContigFwdArgs&, hipStream_t);
  hipError_t (*contig_inv)(int vprec, int fprec, const ContigInvArgs&, hipStream_t);
  hipError_t (*strided)(int fprec, const StridedArgs&, hipStream_t);
  hipError_t (*zpass)(int fprec, const ZArgs&, hipStream_t);
  int64_t (*contig_blocks)(int64_t npencils);
  int64_t (*strided_blocks)(int fprec, int64_t n_outer, int64_t C);
};

const LengthKernels* kernels_for_length(int L);

// ---------------------------------------------------------------------------
// Elementwise / reduction kernels (aux.hip)
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;  // fixed grid of the reduction kernels
constexpr int kRedThreads = 256;

// a1: D = 4 pi h N vol, S = sqrt(D), b = S u0; copies u0; partials
// {||b||^2, ||u0||^2, bad-input count, 0}; also complex64 copies of S.
hipError_t launch_coefficients(const void* h, const double* N, const void* u0, double vol, int64_t P,
                               void* D, void* S, void* Sf, void* b, void* u0c, double* partials,
                               hipStream_t st);
// kernel table c(m) on the L^3 grid [m1][m2][m3] (zero at m = 0 and where a
// wrapped offset equals n)
hipError_t launch_embed(void* grid, int L, double k, double spacing, hipStream_t st);
// kh[m1][m2][m3] = grid[m] * scale for m in [0, n]^3; complex64 copy too
hipError_t launch_octant(const void* grid, int L, double scale, void* kh, void* khf, hipStream_t st);
// reduce 4-double partials of nblk workgroups; mode says where the sums go
enum FinalizeMode : int32_t {
  FIN_SETUP = 0,   // sums = {||b||^2, ||u0||^2, bad, -}: bb, aux, flags
  FIN_INIT = 1,    // sums = {rho.re, rho.im, rr, -}: rho, rr, beta = 0
  FIN_MU = 2,      // sums = {mu.re, mu.im, qq, pp}: mu, alpha = rho / mu
  FIN_RHO = 3,     // sums = {rho'.re, rho'.im, rr, -}: beta = rho'/rho, rho = rho', rr
  FIN_NORM = 4,    // sums = {-, -, ||y||^2, -}: aux
};
hipError_t launch_finalize(const double* partials, int64_t nblk, ScalarBlock* sc, int32_t mode,
                           double eps, hipStream_t st);
// x += alpha p; r -= alpha q; partials {r^T r, ||r||^2} (vector type by prec)
hipError_t launch_update(int prec, void* x, const void* p, void* r, const void* q, int64_t P,
                         const ScalarBlock* sc, double* partials, hipStream_t st);
// r = b (converted to prec), x = 0; partials {r^T r, ||r||^2}
hipError_t launch_init(int prec, const void* b, double bscale, void* x, void* r, int64_t P,
                       double* partials, hipStream_t st);
// y = a * x (complex128 x, a real)  -- elementwise helpers
hipError_t launch_scale_into(int prec_out, const void* x, double a, void* y, int64_t P, hipStream_t st);
// y += a * x with x of type prec_in, y complex128
hipError_t launch_axpy_d(int prec_in, double a, const void* x, void* y, int64_t P, hipStream_t st);
// y = s * x (complex128, elementwise)
hipError_t launch_mul(const void* s, const void* x, void* y, int64_t P, hipStream_t st);

}  // namespace ori
