// Launch interface between the host runtime and the kernel translation units.
// Plain structs of device pointers and sizes; no torch types.
//
// Every vector may carry a batch of right-hand sides sharing one operator
// (same k, h, N): vectors are [nrhs][P], the work arrays [nrhs][...], and the
// diagonals D, S and the spectrum are shared.  Each right-hand side has its
// own ScalarBlock and its own range of reduction partials.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace ori {

// COCG scalars of one right-hand side, resident in device memory for the
// whole solve (the host only reads them at convergence checks).  rho = r^T r
// and mu = p^T A p use the unconjugated bilinear form of COCG.
struct ScalarBlock {
  double rho_re, rho_im;      // r^T r of the current residual
  double mu_re, mu_im;        // p^T q
  double alpha_re, alpha_im;  // rho / mu
  double beta_re, beta_im;    // rho_new / rho_old
  double rr;                  // ||r||^2
  double bb;                  // ||b||^2 of the forward right-hand side (set at load)
  double pp, qq;              // ||p||^2, ||q||^2 of the last product
  double aux;                 // one-off reductions (||u0||^2 at load, residual norms)
  double rr_target;           // converged once rr <= rr_target (set by FIN_INIT)
  double rr0;                 // rr at FIN_INIT
  double s2_min, s2_max;      // min / max |S_p|^2 over the grid (operator coefficients, sc[0])
  int32_t flags;              // FLAG_* below
  int32_t iters;              // COCG iterations done while not converged
};

enum : int32_t {
  FLAG_BREAKDOWN_RHO = 1,  // r^T r ~ 0 while r != 0
  FLAG_BREAKDOWN_MU = 2,   // p^T A p ~ 0 while p != 0
  FLAG_ZERO_RESIDUAL = 4,  // r == 0 exactly
  FLAG_BAD_INPUT = 8,      // NaN / Inf in a right-hand side u0, met in ori_load
  FLAG_BAD_COEFF = 32,     // NaN / Inf in h or N, or N < 0, met in ori_load (sc[0])
  FLAG_CONVERGED = 16,     // rr <= rr_target: alpha = 0 from now on
};
constexpr int32_t FLAG_DONE = FLAG_BREAKDOWN_RHO | FLAG_BREAKDOWN_MU | FLAG_ZERO_RESIDUAL | FLAG_CONVERGED;

enum Prec : int { PREC_F64 = 0, PREC_F32 = 1 };

// F1: forward DFT along the contiguous axis, with the prologue
//   PLAIN: v = s_in * x            (s_in NULL means 1)
//   COCG : p = r + beta p (p = r on the first iteration), stored; v = s_in * p
// Pencils: nrhs * ppr (ppr = n*n per right-hand side); element e of pencil
// (rhs, l) is vector entry (rhs * ppr + l) * in_pitch + e, and diagonal entry
// l * in_pitch + e (diagonals are shared by the batch).
struct ContigFwdArgs {
  const void* x;        // PLAIN input / COCG residual r        (vector type V)
  void* pvec;           // COCG search direction, updated in place (V)
  void* xvec;           // COCG iterate (V): x += alpha p with the alpha and p of the
                        // previous iteration, before p is replaced (NULL: no update)
  const void* s_in;     // diagonal scale (V) or NULL
  const ScalarBlock* sc;  // [nrhs]
  int32_t mode;         // 0 PLAIN, 1 COCG
  int32_t first;        // COCG: first iteration
  int32_t half_in;      // 1: only the first L/2 entries of each pencil are input (zero padding)
  int32_t pad;
  void* out;            // FFT type T, out[pencil * out_pitch + e]
  int64_t nrhs, ppr, in_pitch, out_pitch;
  const void* tw;       // L twiddles exp(-2 pi i m / L) in type T
};

// I1: inverse DFT along the contiguous axis, keep e < n, epilogue
//   y = c0 a0 + c1 a1 + cc (s_out * conv)     (NULL operands are skipped; s_out NULL = 1)
// and optional per-workgroup partials {dot.re, dot.im, |y|^2, |a0|^2}, with
// dot = sum a0_j y_j (dot_self = 0) or sum y_j y_j (dot_self = 1), unconjugated.
// y, a0, a1 are batch vectors; s_out is a shared diagonal.  The workgroups of
// one right-hand side are consecutive: rhs owns partials [rhs*bpr, (rhs+1)*bpr).
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
  int64_t nrhs, ppr, in_pitch, out_pitch;
  const void* tw;
};

// F2 / I2: DFT along a strided axis.  Pencil (o, c) element e lives at
// off(o) + e * axis + c,  c in [0, C) contiguous, with a two-level outer
// offset  off(o) = (o >> lg) * hi + (o & (2^lg - 1)) * lo  (lg = 0: o * hi).
// The two levels express the blocked layout of the B array (see ZArgs); a
// batch of right-hand sides is simply more outer rows (o = rhs * n + i1).
struct StridedArgs {
  const void* in;
  void* out;
  int64_t n_outer, C;
  int64_t nv;  // entries present along the axis: inputs e < nv (half_in), outputs e < nv (half_out)
  int32_t in_lg, out_lg;
  int64_t in_hi, in_lo, in_axis;
  int64_t out_hi, out_lo, out_axis;
  int32_t inverse, half_in, half_out, np_sel;  // np_sel: 0 wide tiles, 1 narrow tiles
  const void* tw;
};

// Z: forward DFT along i1 (first n inputs), multiply by the kernel spectrum,
// inverse DFT, keep the first n outputs; in place on B.  B element
// (rhs, i1, k2, k3) lives at
//   rhs * batch_stride + (i1 >> e_lg) * e_hi + (i1 & (2^e_lg - 1)) * e_lo + k2 * o_stride + k3
// i.e. i1 is split into blocks of 2^e_lg rows stored next to each other, so
// that one pencil of the Z pass spans n / 2^e_lg far-apart regions instead
// of n.  The spectrum is even along every axis and stored as its octant:
// khat[(m1 * kp + m2) * kp + m3], kp = L / 2 + 1, m = min(k, L - k) per axis,
// so a tile of consecutive k3 reads one run, ascending below L / 2 and
// descending above.  plan: the radix plan of the transforms (0 the length's
// default, 1 its alternative where plan.h defines one).
struct ZArgs {
  void* buf;
  int64_t n;
  int32_t e_lg, np_sel;  // np_sel: 0 wide tiles, 1 narrow tiles
  int64_t e_hi, e_lo, o_stride;
  int64_t nrhs, batch_stride;
  int32_t prefetch;    // 1: load the next tile while transforming the current one
  int32_t rhs_slices;  // workgroups per (m2, k3 tile), each taking a contiguous share of the right-hand sides
  const void* khat;     // spectrum (T), octant [kp][kp][kp]
  int64_t kp;
  const void* tw;
  int32_t plan;
};

// Kernel spectrum: passes 1 and 2 in place on an octant scratch
// kh[(m1 kp + m2) kp + m3], kp = n + 1 (the Green's table of the padded grid
// is even along every axis, so are its transforms, and [0..n] per axis
// determines everything); pass 3 writes the scaled octant kout (ZArgs):
//   pass 1: generate the table along m3 for (m1, m2) in [0..n]^2, forward DFT,
//           keep k3 in [0..n]
//   pass 2: along m2 for (m1, k3): read [0..n], mirror, DFT, keep [0..n]
//   pass 3: along m1 for (k2, k3): same, times `scale`, stored in kout
//           (complex128) and koutf (complex64, or NULL).
struct SpectrumArgs {
  void* kh;
  void* kout;
  void* koutf;
  int64_t n;  // points per axis: the table is zero at offsets |d_i| >= n
  double k, spacing, scale;
  int32_t pass, pad;
  const void* tw;      // complex128 twiddles
};

// Per-length launchers (one translation unit per L, see passes.hip).
struct LengthKernels {
  int L;
  hipError_t (*contig_fwd)(int vprec, int fprec, const ContigFwdArgs&, hipStream_t);
  hipError_t (*contig_inv)(int vprec, int fprec, const ContigInvArgs&, hipStream_t);
  hipError_t (*strided)(int fprec, const StridedArgs&, hipStream_t);
  hipError_t (*zpass)(int fprec, const ZArgs&, hipStream_t);
  int64_t (*contig_blocks_per_rhs)(int64_t ppr);
  int64_t (*strided_blocks)(int fprec, int np_sel, int64_t n_outer, int64_t C);
  int64_t (*zpass_blocks)(int fprec, int np_sel);
  hipError_t (*spectrum)(const SpectrumArgs&, hipStream_t);
};

const LengthKernels* kernels_for_length(int L);

// ---------------------------------------------------------------------------
// One pass of several problems of different padded lengths in one launch
// (multi_passes.hip).  The problems' workgroup ranges follow each other:
// launch workgroup b belongs to the problem p with first_block(p) <= b <
// first_block(p + 1) and runs that problem's workgroup b - first_block(p),
// with the pass body its length L compiles for the single-problem kernels,
// on the tile shape below.  Lanes beyond that body's workgroup size (the
// launch uses the largest of the problems') leave at once.  So every
// problem computes exactly what its own launch computes.
// ---------------------------------------------------------------------------
struct MultiProblem {
  int64_t first_block, nblocks;
  int32_t L;
  int32_t ex;    // n = L / 2 exactly (the EX bodies)
  int32_t soff;  // Z: per-lane plus scalar tile offsets (blk_lg <= the length's alignment)
  int32_t pad;
  union {
    ContigFwdArgs f1;
    StridedArgs s;
    ZArgs z;
    ContigInvArgs i1;
  } a;
};
enum MultiPass : int32_t { MP_F1 = 0, MP_F2 = 1, MP_Z = 2, MP_I2 = 3, MP_I1 = 4, MP_NPASS = 5 };
// The padded lengths that have multi-problem bodies: 8 to 256 (L = 16 is
// planned as 4 x 4: a single radix-16 stage would hold 16 values per thread,
// and its complex128 Z body of 188 VGPRs would set the register budget of
// every problem's Z workgroups in the launch).
constexpr bool multi_length(int L) { return L >= 8 && L <= 256 && radix_plan(L).n > 0; }
// Their tile shape: wide strided tiles, no Z prefetch, the default Z plan,
// and Z tiles narrow for complex64 and wide for complex128 (the library's
// default layout up to L = 256).  A problem whose layout differs runs its
// own launches.
constexpr int kMultiZNarrow[2] = {0, 1};  // [PREC_F64, PREC_F32]
// Workgroup size of pass `pass` (MultiPass) at length L in precision prec,
// or 0 if L has no multi-problem bodies.
int multi_pass_threads(int L, int prec, int pass);
// whether the Z pass of that length addresses its tiles with scalar offsets
// at i1 block 2^e_lg (MultiProblem::soff, as the single-problem launch decides)
bool multi_z_soff(int L, int prec, int e_lg);
// LDS bytes of that pass and length
int multi_pass_smem(int L, int prec, int pass);
// tab: device array of np problems (first_block ascending), blocks = the
// sum of their nblocks; threads and smem = the largest multi_pass_threads
// and multi_pass_smem of them.
hipError_t launch_multi_pass(int prec, int pass, const MultiProblem* tab, int32_t np, int64_t blocks, int threads,
                             int smem, hipStream_t st);

// finalisation of several problems: problem p's right-hand sides are
// workgroups [first_block, first_block + nrhs) of the launch
struct MultiFin {
  const double* partials;
  int64_t nblk;  // partial quadruples per right-hand side
  ScalarBlock* sc;
  int64_t first_block;
};
// COCG update (r -= alpha q, partials) of several problems, one right-hand
// side each, on their own update_blocks(P, prec) workgroups
struct MultiUpd {
  const void* p;
  void* r;
  const void* q;
  int64_t P;
  const ScalarBlock* sc;
  double* partials;
  int64_t first_block, nblocks;
};
hipError_t launch_multi_finalize(const MultiFin* tab, int32_t np, int64_t blocks, int32_t mode, double eps,
                                 hipStream_t st);
hipError_t launch_multi_update(int prec, const MultiUpd* tab, int32_t np, int64_t blocks, hipStream_t st);
// out[p] = *tab[p].sc for p < np; out is host memory the device can write
hipError_t launch_gather_scalars(const MultiFin* tab, int32_t np, ScalarBlock* out, hipStream_t st);

// ---------------------------------------------------------------------------
// Elementwise / reduction kernels (aux.hip).  Batched kernels run a grid of
// (red_blocks(P), nrhs) workgroups; right-hand side rhs writes partials
// [rhs * red_blocks(P), (rhs + 1) * red_blocks(P)).
// ---------------------------------------------------------------------------
// Field sums over the cells (eq. 2.10): points a.pts[m0 .. m0 + mb) of M,
// cells in chunks of `chunk`, partials [nrhs][mb][nchunk], results
// out[nrhs][M].
struct FieldArgs {
  const cxd* u;      // [nrhs][P] solution of eq. 2.19
  const cxd* D;      // [P]
  const double* pts; // [M][3] points (field) or unit directions (far field)
  cxd* part;
  cxd* out;
  int64_t n, P, M, m0, mb, nchunk, chunk, nrhs;
  double dn, side, offset, k;
  double origin[3];
};
hipError_t launch_field(const FieldArgs& a, bool far, hipStream_t st);
// q = -D u over the batch
hipError_t launch_charges(const void* D, const void* u, int64_t P, int64_t nrhs, void* q, hipStream_t st);

// Refraction recipe, elementwise over P entries: design = 1 gives
// h = k^2 (n0^2 - n^2) / (c_S N) from in = n; design = 0 gives
// n = [n0^2 - c_S h N / k^2]^{1/2} (arg in [0, 2 pi)) from in = h.
// bad[refraction_blocks(P)] counts rejected entries per workgroup.
struct RefractionArgs {
  const cxd* n0;
  const cxd* in;
  const double* N;  // NULL: N = 1
  cxd* out;
  double* bad;
  int64_t P;
  double k, c_s;
  int32_t design, pad;
};
int64_t refraction_blocks(int64_t P);
hipError_t launch_refraction(const RefractionArgs& a, hipStream_t st);

// Section 4 solution difference: x fine [nf^3], y coarse [nc^3]; means
// [nc^3] (mean |x_i - y_q| per coarse cell, -1 for a cell without fine
// points); part[max_blocks(nc^3)] receives block maxima of the means.
struct DiffArgs {
  const cxd* x;
  const cxd* y;
  double* means;
  int64_t nf, nc;
  double off;  // offset of the fine points in their cells
};
int64_t max_blocks(int64_t P);
hipError_t launch_cell_difference(const DiffArgs& a, int64_t P_coarse, double* part, hipStream_t st);

constexpr int kRedThreads = 256;
constexpr int64_t kRedBlocksMax = 1024;
inline int64_t red_blocks(int64_t P, int64_t cap = kRedBlocksMax) {
  int64_t b = (P + kRedThreads * 4 - 1) / (kRedThreads * 4);
  if (b > cap) b = cap;
  return b < 1 ? 1 : b;
}
// The complex64 COCG update (r -= alpha q with the partials of r^T r and
// |r|^2) runs on up to 4096 workgroups: on 8-byte elements 1024 of them leave
// too few loads in flight (0.113 vs 0.079 ms at n = 256, 0.93 vs 0.65 ms at
// n = 512).  The complex128 update and the other reductions measured faster
// on 1024.  The update's partials are finalised with the same count.
constexpr int64_t kUpdateBlocksMaxF32 = 4096;
inline int64_t update_blocks(int64_t P, int prec) {
  return red_blocks(P, prec == PREC_F32 ? kUpdateBlocksMaxF32 : kRedBlocksMax);
}

// a1 (operator): D = 4 pi h N vol, S = sqrt(D), complex64 S, c = 4 pi N vol;
// partials {bad-input count, min |S|^2, max |S|^2, 0} (one range), reduced
// into sc[0] by launch_finalize_coeff
hipError_t launch_coefficients(const void* h, const double* N, double vol, int64_t P, void* D, void* S, void* Sf,
                               double* cN, double* partials, hipStream_t st);
hipError_t launch_finalize_coeff(const double* partials, int64_t nblk, ScalarBlock* sc, hipStream_t st);
// u = w / S (w, u batch vectors; S shared, nonzero)
hipError_t launch_div(const void* w, const void* s, void* u, int64_t P, int64_t nrhs, hipStream_t st);
// q = (z + r) / S (one right-hand side; S nonzero)
hipError_t launch_add_div(const void* z, const void* r, const void* s, void* q, int64_t P, hipStream_t st);
// u = w / S as launch_div, and partials {-, -, ||r / S||^2, -} per
// right-hand side on red_blocks(P) workgroups each (FIN_NORM)
hipError_t launch_div_res(const void* w, const void* r, const void* s, void* u, int64_t P, int64_t nrhs,
                          double* partials, hipStream_t st);
// a1 (right-hand sides): b = S u0, u0 copied; partials {||b||^2, ||u0||^2, bad, 0} per rhs
hipError_t launch_rhs(const void* u0, const void* S, int64_t P, int64_t nrhs, void* b, void* u0c,
                      double* partials, hipStream_t st);
// reduce partials (nblk per right-hand side) into sc[rhs]; mode says where
// the sums go
enum FinalizeMode : int32_t {
  FIN_SETUP = 0,   // sums = {||b||^2, ||u0||^2, bad, -}: bb, aux, flags
  FIN_INIT = 1,    // sums = {rho.re, rho.im, rr, -}: rho, rr, rr0, beta = 0, flags, rr_target
  FIN_MU = 2,      // sums = {mu.re, mu.im, qq, pp}: mu, alpha = rho / mu
  FIN_RHO = 3,     // sums = {rho'.re, rho'.im, rr, -}: beta = rho'/rho, rho = rho', rr, flags
  FIN_NORM = 4,    // sums = {-, -, ||y||^2, -}: aux
};
// FIN_INIT: rr_target = t2 * (tol2_of_bb ? bb : rr), t2 = tol2_rhs[rhs] when
// tol2_rhs is not NULL, else tol2
hipError_t launch_finalize(const double* partials, int64_t nblk, int64_t nrhs, ScalarBlock* sc, int32_t mode,
                           double eps, double tol2, int32_t tol2_of_bb, const double* tol2_rhs, hipStream_t st);
// r -= alpha q (and x += alpha p when x is not NULL); partials
// {r^T r, ||r||^2} on (update_blocks(P, prec), nrhs) workgroups; converged
// right-hand sides (alpha = 0) stay as they are
hipError_t launch_update(int prec, void* x, const void* p, void* r, const void* q, int64_t P, int64_t nrhs,
                         const ScalarBlock* sc, double* partials, hipStream_t st);
// x += alpha p per right-hand side (the update left pending by the last
// COCG iteration, whose F1 would have applied it)
hipError_t launch_x_flush(int prec, void* x, const void* p, int64_t P, int64_t nrhs, const ScalarBlock* sc,
                          hipStream_t st);
// r = m_inv[rhs] * b (converted to prec; m NULL: 1), x = 0; partials {r^T r, ||r||^2}
hipError_t launch_init(int prec, const void* b, const double* m, void* x, void* r, int64_t P, int64_t nrhs,
                       double* partials, hipStream_t st);
// y += m[rhs] * x with x of type prec_in, y complex128
hipError_t launch_axpy_batch(int prec_in, const double* m, const void* x, void* y, int64_t P, int64_t nrhs,
                             hipStream_t st);
// y = s * x (s shared diagonal, x and y batch vectors)
hipError_t launch_mul(const void* s, const void* x, void* y, int64_t P, int64_t nrhs, hipStream_t st);
// f = conj(u - t); partials {0, 0, |u - t|^2, 0} (one right-hand side)
hipError_t launch_conj_diff(const void* u, const void* t, void* f, int64_t P, double* partials, hipStream_t st);
// g = alpha * c * u * q  (c real)
hipError_t launch_gradient(const double* c, const void* u, const void* q, double alpha, void* g, int64_t P,
                           hipStream_t st);
// twd[m] = exp(-2 pi i m / L) (complex128) and twf[m] the same in complex64, m < L
hipError_t launch_twiddles(int64_t L, void* twd, void* twf, hipStream_t st);

// Guard bands of a workspace block: count bands of kGuardBandBytes at
// base + off[i] (each 16-byte aligned) filled with the byte v.
constexpr int kMaxGuardBands = 32;
constexpr int kGuardBandBytes = 4096;
struct GuardBands {
  void* base;
  int32_t count;
  uint32_t v;
  int64_t off[kMaxGuardBands];
};
hipError_t launch_fill_guards(const GuardBands& g, hipStream_t st);
// lam = f - s * x
hipError_t launch_sub_mul(const void* f, const void* s, const void* x, void* lam, int64_t P, hipStream_t st);

}  // namespace ori
