// Host runtime and C ABI (include/ori.h): context, workspaces, the FFT
// product with the Green's matrix (Section 3), COCG (van der Vorst &
// Melissen, cited by the paper) and mixed-precision refinement.
#include "ori.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "cx.h"
#include "kernels.h"
#include "plan.h"

namespace ori {
#define ORI_DECL(L) const LengthKernels* kernels_L##L();
ORI_FOR_EACH_L(ORI_DECL)
#undef ORI_DECL

const LengthKernels* kernels_for_length(int L) {
  switch (L) {
#define ORI_CASE(L) \
  case L:           \
    return kernels_L##L();
    ORI_FOR_EACH_L(ORI_CASE)
#undef ORI_CASE
    default:
      return nullptr;
  }
}
}  // namespace ori

using namespace ori;

namespace {

constexpr double kBreakdownEps = 1e-13;

enum ProfKind : int {
  K_F1,
  K_F2,
  K_Z,
  K_I2,
  K_I1,
  K_UPDATE,
  K_FINALIZE,
  K_INIT,
  K_COEFF,
  K_EMBED,
  K_SPEC_FFT,
  K_OCTANT,
  K_ELEMWISE,
  K_NKIND
};
const char* const kKindNames[K_NKIND] = {"f1", "f2", "zpass", "i2", "i1", "update", "finalize",
                                         "init", "coefficients", "embed", "spectrum_fft", "octant",
                                         "elementwise"};

thread_local std::string g_last_error = "no error";

struct ProfPending {
  int slot;  // kind * 2 + (fprec == F32)
  int ev;
};

}  // namespace

struct ori_ctx_s {
  ori_grid grid{};
  int64_t n = 0, L = 0, P = 0;
  int provision = 0;
  double k = 0.0;
  bool loaded = false;
  bool poisoned = false;
  hipStream_t stream = nullptr;
  int device = 0;
  const LengthKernels* K = nullptr;
  std::string err = "no error";
  double u0norm2 = 0.0, bnorm2 = 0.0;

  void* arena = nullptr;  // L^3 complex128: spectrum grid, then the A/B work arrays
  cxd *D = nullptr, *S = nullptr, *b = nullptr, *u0 = nullptr;
  cxd *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
  cxf *Sf = nullptr, *xf = nullptr, *rf = nullptr, *pf = nullptr, *qf = nullptr;
  cxd* kh = nullptr;
  cxf* khf = nullptr;
  cxd* twd = nullptr;
  cxf* twf = nullptr;
  double* partials = nullptr;
  int64_t npartials = 0;  // quadruples
  ScalarBlock* sc = nullptr;
  ScalarBlock* sc_host = nullptr;  // pinned
  std::vector<void*> allocs;

  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev;  // pairs
  std::vector<ProfPending> pend;
  double prof_ms[2 * K_NKIND] = {};
  int64_t prof_n[2 * K_NKIND] = {};
};

namespace {

ori_status set_err(ori_ctx c, ori_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) {
    c->err = buf;
    if (st == ORI_ERR_DEVICE) c->poisoned = true;
  } else {
    g_last_error = buf;
  }
  return st;
}

#define ORI_HIP(c, call)                                                                            \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) return set_err((c), ORI_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define ORI_TRY(expr)               \
  do {                              \
    ori_status s_ = (expr);         \
    if (s_ != ORI_OK) return s_;    \
  } while (0)

bool finite(double v) { return std::isfinite(v); }

ori_status check_grid(const ori_grid* g, int64_t* L_out) {
  if (!g) return set_err(nullptr, ORI_ERR_INVALID_ARG, "grid is NULL");
  if (g->n < 1) return set_err(nullptr, ORI_ERR_INVALID_ARG, "n = %lld must be >= 1", (long long)g->n);
  if (!(g->side > 0.0) || !finite(g->side))
    return set_err(nullptr, ORI_ERR_INVALID_ARG, "side must be finite and > 0");
  for (int i = 0; i < 3; ++i)
    if (!finite(g->origin[i])) return set_err(nullptr, ORI_ERR_INVALID_ARG, "origin must be finite");
  if (!finite(g->cell_offset)) return set_err(nullptr, ORI_ERR_INVALID_ARG, "cell_offset must be finite");
  if (g->n > 512 || !supported_length(static_cast<int>(2 * g->n)))
    return set_err(nullptr, ORI_ERR_UNSUPPORTED, "no FFT plan for n = %lld (padded length %lld)",
                   (long long)g->n, (long long)(2 * g->n));
  *L_out = 2 * g->n;
  return ORI_OK;
}

struct Layout {
  int64_t arena, vec_d, vec_f, kh, khf, tw, partials, nvec_d, nvec_f, npart;
  int64_t total;
};

int64_t align_up(int64_t v) { return (v + 255) / 256 * 256; }

Layout layout_for(int64_t n, int provision) {
  const int64_t L = 2 * n, P = n * n * n, kp = n + 1;
  Layout l{};
  l.arena = align_up(L * L * L * 16);
  l.vec_d = align_up(P * 16);
  l.vec_f = align_up(P * 8);
  l.nvec_d = 8;  // D, S, b, u0, x, r, p, q
  l.nvec_f = (provision & ORI_PROVISION_MIXED) ? 5 : 0;  // Sf, xf, rf, pf, qf
  l.kh = align_up(kp * kp * kp * 16);
  l.khf = (provision & ORI_PROVISION_MIXED) ? align_up(kp * kp * kp * 8) : 0;
  l.tw = align_up(L * 16) + align_up(L * 8);
  // partial quadruples: the largest grid of a reducing kernel (I1 has at
  // most n*n workgroups; the exact count is used at create time)
  l.npart = std::max<int64_t>(kRedBlocks, n * n);
  l.partials = align_up(l.npart * 4 * 8);
  l.total = l.arena + l.nvec_d * l.vec_d + l.nvec_f * l.vec_f + l.kh + l.khf + l.tw + l.partials +
            align_up(sizeof(ScalarBlock));
  return l;
}

ori_status check_dev_ptr(ori_ctx c, const void* ptr, int64_t bytes, const char* what) {
  if (!ptr) return set_err(c, ORI_ERR_INVALID_ARG, "%s is NULL", what);
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(c, ORI_ERR_INVALID_ARG, "%s is not a device pointer", what);
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    return set_err(c, ORI_ERR_INVALID_ARG, "%s is not device memory (memory type %d)", what, (int)at.type);
  if (at.device != c->device)
    return set_err(c, ORI_ERR_INVALID_ARG, "%s lives on device %d, the context on device %d", what, at.device,
                   c->device);
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(ptr)) == hipSuccess && base) {
    const char* b0 = static_cast<const char*>(base);
    const char* p0 = static_cast<const char*>(ptr);
    if (p0 + bytes > b0 + size)
      return set_err(c, ORI_ERR_INVALID_ARG, "%s holds %lld bytes from the pointer, %lld needed", what,
                     (long long)(b0 + size - p0), (long long)bytes);
  } else {
    (void)hipGetLastError();
  }
  if (reinterpret_cast<uintptr_t>(ptr) % 16 != 0 && bytes > 8)
    return set_err(c, ORI_ERR_INVALID_ARG, "%s is not 16-byte aligned", what);
  return ORI_OK;
}

// ---------------------------------------------------------------------------
// profiling wrapper
// ---------------------------------------------------------------------------
ori_status prof_fold(ori_ctx c) {
  if (c->pend.empty()) return ORI_OK;
  ORI_HIP(c, hipEventSynchronize(c->ev[c->pend.back().ev * 2 + 1]));
  for (const ProfPending& pp : c->pend) {
    float ms = 0.f;
    ORI_HIP(c, hipEventElapsedTime(&ms, c->ev[pp.ev * 2], c->ev[pp.ev * 2 + 1]));
    c->prof_ms[pp.slot] += ms;
    c->prof_n[pp.slot] += 1;
  }
  c->pend.clear();
  return ORI_OK;
}

template <class F>
ori_status launch(ori_ctx c, int kind, int fprec, F&& f) {
  int evi = -1;
  if (c->prof) {
    const int cap = 4096;
    if (static_cast<int>(c->pend.size()) >= cap) ORI_TRY(prof_fold(c));
    evi = static_cast<int>(c->pend.size());
    while (static_cast<int>(c->ev.size()) < 2 * (evi + 1)) {
      hipEvent_t e;
      ORI_HIP(c, hipEventCreate(&e));
      c->ev.push_back(e);
    }
    ORI_HIP(c, hipEventRecord(c->ev[2 * evi], c->stream));
  }
  hipError_t e = f();
  if (e != hipSuccess) return set_err(c, ORI_ERR_DEVICE, "kernel %s launch failed: %s", kKindNames[kind], hipGetErrorString(e));
  if (c->prof) {
    ORI_HIP(c, hipEventRecord(c->ev[2 * evi + 1], c->stream));
    c->pend.push_back(ProfPending{kind * 2 + (fprec == PREC_F32 ? 1 : 0), evi});
  }
  return ORI_OK;
}

ori_status sync_scalars(ori_ctx c) {
  ORI_HIP(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(ScalarBlock), hipMemcpyDeviceToHost, c->stream));
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  return ORI_OK;
}

ori_status finalize(ori_ctx c, int64_t nblk, int mode) {
  return launch(c, K_FINALIZE, PREC_F64,
                [&] { return launch_finalize(c->partials, nblk, c->sc, mode, kBreakdownEps, c->stream); });
}

// ---------------------------------------------------------------------------
// the FFT product: F1 -> F2 -> Z -> I2 -> I1 (prologue / epilogue in f1, i1)
// ---------------------------------------------------------------------------
ori_status matvec(ori_ctx c, int vprec, int fprec, ContigFwdArgs f1, ContigInvArgs i1, int64_t* nblk_out) {
  const int64_t n = c->n, L = c->L;
  const int64_t elem = fprec == PREC_F64 ? 16 : 8;
  char* A = static_cast<char*>(c->arena);
  char* B = A + n * n * L * elem;
  const void* tw = fprec == PREC_F64 ? static_cast<const void*>(c->twd) : static_cast<const void*>(c->twf);
  const void* kh = fprec == PREC_F64 ? static_cast<const void*>(c->kh) : static_cast<const void*>(c->khf);
  if (!kh) return set_err(c, ORI_ERR_INVALID_ARG, "complex64 workspaces were not provisioned");

  f1.half_in = 1;
  f1.out = A;
  f1.npencils = n * n;
  f1.in_pitch = n;
  f1.out_pitch = L;
  f1.tw = tw;
  ORI_TRY(launch(c, K_F1, fprec, [&] { return c->K->contig_fwd(vprec, fprec, f1, c->stream); }));

  StridedArgs f2{A, B, n, L, n * L, L, L * L, L, 0, 1, 0, 0, tw};
  ORI_TRY(launch(c, K_F2, fprec, [&] { return c->K->strided(fprec, f2, c->stream); }));

  ZArgs z{B, L, L, L * L, L, kh, n + 1, tw};
  ORI_TRY(launch(c, K_Z, fprec, [&] { return c->K->zpass(fprec, z, c->stream); }));

  StridedArgs i2{B, A, n, L, L * L, L, n * L, L, 1, 0, 1, 0, tw};
  ORI_TRY(launch(c, K_I2, fprec, [&] { return c->K->strided(fprec, i2, c->stream); }));

  i1.in = A;
  i1.npencils = n * n;
  i1.in_pitch = L;
  i1.out_pitch = n;
  i1.tw = tw;
  if (nblk_out) *nblk_out = c->K->contig_blocks(n * n);
  ORI_TRY(launch(c, K_I1, fprec, [&] { return c->K->contig_inv(vprec, fprec, i1, c->stream); }));
  return ORI_OK;
}

ContigFwdArgs plain_f1(const void* x, const void* s_in) {
  ContigFwdArgs a{};
  a.x = x;
  a.s_in = s_in;
  a.mode = 0;
  return a;
}

ContigInvArgs epi(void* y, const void* a0, double c0, const void* a1, double c1, const void* s_out, double cc,
                  double* partials, int dot_self) {
  ContigInvArgs a{};
  a.y = y;
  a.a0 = a0;
  a.c0 = c0;
  a.a1 = a1;
  a.c1 = c1;
  a.s_out = s_out;
  a.cc = cc;
  a.partials = partials;
  a.dot_self = dot_self;
  return a;
}

// ---------------------------------------------------------------------------
// setup: spectrum of the Green's table (a2) and the coefficients (a1)
// ---------------------------------------------------------------------------
ori_status compute_spectrum(ori_ctx c) {
  const int L = static_cast<int>(c->L);
  const int64_t L2 = c->L * c->L;
  const double spacing = c->grid.side / static_cast<double>(c->n);
  ORI_TRY(launch(c, K_EMBED, PREC_F64, [&] { return launch_embed(c->arena, L, c->k, spacing, c->stream); }));
  ContigFwdArgs f{};
  f.x = c->arena;
  f.mode = 0;
  f.half_in = 0;
  f.out = c->arena;
  f.npencils = L2;
  f.in_pitch = L;
  f.out_pitch = L;
  f.tw = c->twd;
  ORI_TRY(launch(c, K_SPEC_FFT, PREC_F64, [&] { return c->K->contig_fwd(PREC_F64, PREC_F64, f, c->stream); }));
  StridedArgs s2{c->arena, c->arena, L, L, L2, L, L2, L, 0, 0, 0, 0, c->twd};
  ORI_TRY(launch(c, K_SPEC_FFT, PREC_F64, [&] { return c->K->strided(PREC_F64, s2, c->stream); }));
  StridedArgs s1{c->arena, c->arena, L, L, L, L2, L, L2, 0, 0, 0, 0, c->twd};
  ORI_TRY(launch(c, K_SPEC_FFT, PREC_F64, [&] { return c->K->strided(PREC_F64, s1, c->stream); }));
  const double scale = 1.0 / (static_cast<double>(L) * L * L);  // inverse DFT normalisation, folded in once
  ORI_TRY(launch(c, K_OCTANT, PREC_F64, [&] { return launch_octant(c->arena, L, scale, c->kh, c->khf, c->stream); }));
  return ORI_OK;
}

void fill_twiddles(int64_t L, std::vector<cxd>& d, std::vector<cxf>& f) {
  d.resize(L);
  f.resize(L);
  const long double two_pi = 6.283185307179586476925286766559L;
  for (int64_t m = 0; m < L; ++m) {
    // exp(-2 pi i m / L), argument reduced to [0, pi/4] by symmetry for accuracy
    const long double a = two_pi * static_cast<long double>(m) / static_cast<long double>(L);
    long double cs = cosl(a), sn = sinl(a);
    // exact values where known
    if (4 * m % L == 0) {
      const int64_t q = 4 * m / L;
      cs = (q == 0) ? 1 : (q == 2) ? -1 : 0;
      sn = (q == 1) ? 1 : (q == 3) ? -1 : 0;
    }
    d[m] = cxd{static_cast<double>(cs), static_cast<double>(-sn)};
    f[m] = cxf{static_cast<float>(cs), static_cast<float>(-sn)};
  }
}

// ---------------------------------------------------------------------------
// COCG on (I + S G0 S) w = rhs, vectors of type vprec, FFTs of type fprec.
// Expects x, r initialised and the scalars set by FIN_INIT.
// ---------------------------------------------------------------------------
struct CocgOut {
  int iters = 0;
  int64_t matvecs = 0;
  double rr = 0.0;
  int flags = 0;
  bool converged = false;
};

ori_status run_cocg(ori_ctx c, int prec, void* x, void* r, void* p, void* q, const void* S, double rr_target,
                    int max_iter, int check_every, CocgOut* out) {
  ORI_TRY(sync_scalars(c));
  out->rr = c->sc_host->rr;
  out->flags = c->sc_host->flags;
  if ((out->flags & FLAG_ZERO_RESIDUAL) || out->rr <= rr_target) {
    out->converged = true;
    return ORI_OK;
  }
  if (out->flags & (FLAG_BREAKDOWN_RHO | FLAG_BREAKDOWN_MU)) return ORI_OK;
  const int64_t P = c->P;
  for (int it = 0; it < max_iter; ++it) {
    ContigFwdArgs f1{};
    f1.x = r;
    f1.pvec = p;
    f1.s_in = S;
    f1.sc = c->sc;
    f1.mode = 1;
    f1.first = it == 0;
    ContigInvArgs i1 = epi(q, p, 1.0, nullptr, 0.0, S, 1.0, c->partials, 0);
    int64_t nblk = 0;
    ORI_TRY(matvec(c, prec, prec, f1, i1, &nblk));
    out->matvecs++;
    ORI_TRY(finalize(c, nblk, FIN_MU));
    ORI_TRY(launch(c, K_UPDATE, prec, [&] { return launch_update(prec, x, p, r, q, P, c->sc, c->partials, c->stream); }));
    ORI_TRY(finalize(c, kRedBlocks, FIN_RHO));
    out->iters++;
    if ((it + 1) % check_every == 0 || it + 1 == max_iter) {
      ORI_TRY(sync_scalars(c));
      out->rr = c->sc_host->rr;
      out->flags = c->sc_host->flags;
      if (out->flags & (FLAG_BREAKDOWN_RHO | FLAG_BREAKDOWN_MU)) return ORI_OK;
      if ((out->flags & FLAG_ZERO_RESIDUAL) || out->rr <= rr_target) {
        out->converged = true;
        return ORI_OK;
      }
    }
  }
  return ORI_OK;
}

// r = b - (I + S G0 S) x in FP64; returns ||r||^2 and r^T r via FIN_INIT
ori_status true_residual_sym(ori_ctx c, const cxd* x, cxd* r) {
  int64_t nblk = 0;
  ORI_TRY(matvec(c, PREC_F64, PREC_F64, plain_f1(x, c->S), epi(r, c->b, 1.0, x, -1.0, c->S, -1.0, c->partials, 1),
                 &nblk));
  return finalize(c, nblk, FIN_INIT);
}

// u = u0 - G0 S w (recovery of the solution of eq. 2.19 from w)
ori_status recover(ori_ctx c, const cxd* w, cxd* u) {
  return matvec(c, PREC_F64, PREC_F64, plain_f1(w, c->S), epi(u, c->u0, 1.0, nullptr, 0.0, nullptr, -1.0, nullptr, 0),
                nullptr);
}

// ||u0 - u - G0 D u|| / ||u0||
ori_status true_residual_orig(ori_ctx c, const cxd* u, double* rel) {
  int64_t nblk = 0;
  ORI_TRY(matvec(c, PREC_F64, PREC_F64, plain_f1(u, c->D),
                 epi(c->q, c->u0, 1.0, u, -1.0, nullptr, -1.0, c->partials, 1), &nblk));
  ORI_TRY(finalize(c, nblk, FIN_NORM));
  ORI_TRY(sync_scalars(c));
  *rel = c->u0norm2 > 0 ? std::sqrt(c->sc_host->aux / c->u0norm2) : std::sqrt(c->sc_host->aux);
  return ORI_OK;
}

ori_status guard(ori_ctx c) {
  if (!c) return set_err(nullptr, ORI_ERR_INVALID_ARG, "context is NULL");
  if (c->poisoned) return set_err(c, ORI_ERR_DEVICE, "context is poisoned by an earlier device error: %s", c->err.c_str());
  ORI_HIP(c, hipSetDevice(c->device));
  return ORI_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void ori_default_opts(ori_solve_opts* o) {
  if (!o) return;
  o->tol = 1e-10;
  o->max_iter = 1000;
  o->precision = ORI_FP64;
  o->check_every = 1;
  o->use_x0 = 0;
  o->inner_tol = 1e-5;
  o->max_outer = 10;
  o->true_residual = 1;
}

const char* ori_version(void) { return "ori 0.1 (gfx950)"; }

ori_status ori_workspace_bytes(const ori_grid* g, int32_t provision, int64_t* bytes) {
  int64_t L = 0;
  ORI_TRY(check_grid(g, &L));
  if (!bytes) return set_err(nullptr, ORI_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = layout_for(g->n, provision | ORI_PROVISION_FP64).total;
  return ORI_OK;
}

ori_status ori_create(const ori_grid* g, int32_t provision, int64_t mem_limit_bytes, void* stream, ori_ctx* out) {
  if (!out) return set_err(nullptr, ORI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int64_t L = 0;
  ORI_TRY(check_grid(g, &L));
  provision |= ORI_PROVISION_FP64;
  const Layout lay = layout_for(g->n, provision);
  if (mem_limit_bytes > 0 && lay.total > mem_limit_bytes)
    return set_err(nullptr, ORI_ERR_OUT_OF_MEMORY, "workspace of %lld bytes exceeds the limit of %lld bytes",
                   (long long)lay.total, (long long)mem_limit_bytes);
  const LengthKernels* K = kernels_for_length(static_cast<int>(L));
  if (!K) return set_err(nullptr, ORI_ERR_UNSUPPORTED, "no kernels for padded length %lld", (long long)L);

  ori_ctx c = new ori_ctx_s();
  c->grid = *g;
  c->n = g->n;
  c->L = L;
  c->P = g->n * g->n * g->n;
  c->provision = provision;
  c->K = K;
  c->stream = static_cast<hipStream_t>(stream);
  auto fail = [&](ori_status st) {
    g_last_error = c->err;
    ori_destroy(c);
    return st;
  };
  if (hipGetDevice(&c->device) != hipSuccess) {
    set_err(c, ORI_ERR_DEVICE, "hipGetDevice failed (no GPU?)");
    return fail(ORI_ERR_DEVICE);
  }
  auto alloc = [&](int64_t bytes, void** p) -> ori_status {
    if (bytes <= 0) {
      *p = nullptr;
      return ORI_OK;
    }
    hipError_t e = hipMalloc(p, static_cast<size_t>(bytes));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return set_err(c, ORI_ERR_OUT_OF_MEMORY, "hipMalloc(%lld) failed: %s", (long long)bytes, hipGetErrorString(e));
    }
    c->allocs.push_back(*p);
    return ORI_OK;
  };
  ori_status st = ORI_OK;
  void* v = nullptr;
#define ORI_ALLOC(bytes, dst, type)                 \
  do {                                              \
    st = alloc((bytes), &v);                        \
    if (st != ORI_OK) return fail(st);              \
    dst = static_cast<type>(v);                     \
  } while (0)
  ORI_ALLOC(lay.arena, c->arena, void*);
  ORI_ALLOC(lay.vec_d, c->D, cxd*);
  ORI_ALLOC(lay.vec_d, c->S, cxd*);
  ORI_ALLOC(lay.vec_d, c->b, cxd*);
  ORI_ALLOC(lay.vec_d, c->u0, cxd*);
  ORI_ALLOC(lay.vec_d, c->x, cxd*);
  ORI_ALLOC(lay.vec_d, c->r, cxd*);
  ORI_ALLOC(lay.vec_d, c->p, cxd*);
  ORI_ALLOC(lay.vec_d, c->q, cxd*);
  if (provision & ORI_PROVISION_MIXED) {
    ORI_ALLOC(lay.vec_f, c->Sf, cxf*);
    ORI_ALLOC(lay.vec_f, c->xf, cxf*);
    ORI_ALLOC(lay.vec_f, c->rf, cxf*);
    ORI_ALLOC(lay.vec_f, c->pf, cxf*);
    ORI_ALLOC(lay.vec_f, c->qf, cxf*);
    ORI_ALLOC(lay.khf, c->khf, cxf*);
  }
  ORI_ALLOC(lay.kh, c->kh, cxd*);
  ORI_ALLOC(align_up(L * 16), c->twd, cxd*);
  ORI_ALLOC(align_up(L * 8), c->twf, cxf*);
  const int64_t npart = std::max<int64_t>(kRedBlocks, K->contig_blocks(c->n * c->n));
  c->npartials = npart;
  ORI_ALLOC(npart * 4 * 8, c->partials, double*);
  ORI_ALLOC(static_cast<int64_t>(sizeof(ScalarBlock)), c->sc, ScalarBlock*);
#undef ORI_ALLOC
  if (hipHostMalloc(reinterpret_cast<void**>(&c->sc_host), sizeof(ScalarBlock), hipHostMallocDefault) != hipSuccess) {
    c->sc_host = nullptr;
    set_err(c, ORI_ERR_OUT_OF_MEMORY, "hipHostMalloc of the scalar mirror failed");
    return fail(ORI_ERR_OUT_OF_MEMORY);
  }
  std::vector<cxd> twd;
  std::vector<cxf> twf;
  fill_twiddles(L, twd, twf);
  if (hipMemcpy(c->twd, twd.data(), L * sizeof(cxd), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->twf, twf.data(), L * sizeof(cxf), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemsetAsync(c->sc, 0, sizeof(ScalarBlock), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    set_err(c, ORI_ERR_DEVICE, "initial copies failed");
    return fail(ORI_ERR_DEVICE);
  }
  *out = c;
  return ORI_OK;
}

ori_status ori_load(ori_ctx c, double k, const void* h, const double* N, const void* u0) {
  ORI_TRY(guard(c));
  if (!(k > 0.0) || !std::isfinite(k)) return set_err(c, ORI_ERR_INVALID_ARG, "k must be finite and > 0");
  const int64_t P = c->P;
  ORI_TRY(check_dev_ptr(c, h, P * 16, "h"));
  if (N) ORI_TRY(check_dev_ptr(c, N, P * 8, "N"));
  ORI_TRY(check_dev_ptr(c, u0, P * 16, "u0"));
  c->loaded = false;
  c->k = k;
  ORI_TRY(compute_spectrum(c));
  const double vol = std::pow(c->grid.side / static_cast<double>(c->n), 3);
  ORI_TRY(launch(c, K_COEFF, PREC_F64, [&] {
    return launch_coefficients(h, N, u0, vol, P, c->D, c->S, c->Sf, c->b, c->u0, c->partials, c->stream);
  }));
  ORI_TRY(finalize(c, kRedBlocks, FIN_SETUP));
  ORI_TRY(sync_scalars(c));
  if (c->sc_host->flags & FLAG_BAD_INPUT)
    return set_err(c, ORI_ERR_INVALID_ARG, "h, N or u0 holds NaN/Inf, or N < 0");
  c->bnorm2 = c->sc_host->bb;
  c->u0norm2 = c->sc_host->aux;
  c->loaded = true;
  return ORI_OK;
}

ori_status ori_setup(const ori_grid* g, double k, const void* h, const double* N, const void* u0, void* stream,
                     ori_ctx* out) {
  ORI_TRY(ori_create(g, ORI_PROVISION_FP64 | ORI_PROVISION_MIXED, 0, stream, out));
  ori_status st = ori_load(*out, k, h, N, u0);
  if (st != ORI_OK) {
    g_last_error = (*out)->err;
    ori_destroy(*out);
    *out = nullptr;
  }
  return st;
}

ori_status ori_matvec(ori_ctx c, int32_t op, int32_t precision, const void* x, void* y) {
  ORI_TRY(guard(c));
  if (!c->loaded) return set_err(c, ORI_ERR_INVALID_ARG, "ori_load has not succeeded on this context");
  if (precision != ORI_FP64 && precision != ORI_MIXED) return set_err(c, ORI_ERR_INVALID_ARG, "bad precision");
  if (precision == ORI_MIXED && !(c->provision & ORI_PROVISION_MIXED))
    return set_err(c, ORI_ERR_INVALID_ARG, "complex64 workspaces were not provisioned");
  ORI_TRY(check_dev_ptr(c, x, c->P * 16, "x"));
  ORI_TRY(check_dev_ptr(c, y, c->P * 16, "y"));
  const int fp = precision == ORI_MIXED ? PREC_F32 : PREC_F64;
  ContigFwdArgs f1;
  ContigInvArgs i1;
  switch (op) {
    case ORI_OP_SYSTEM:
      f1 = plain_f1(x, c->D);
      i1 = epi(y, x, 1.0, nullptr, 0.0, nullptr, 1.0, nullptr, 0);
      break;
    case ORI_OP_SYMMETRIC:
      f1 = plain_f1(x, c->S);
      i1 = epi(y, x, 1.0, nullptr, 0.0, c->S, 1.0, nullptr, 0);
      break;
    case ORI_OP_GREEN:
      f1 = plain_f1(x, nullptr);
      i1 = epi(y, nullptr, 0.0, nullptr, 0.0, nullptr, 1.0, nullptr, 0);
      break;
    default:
      return set_err(c, ORI_ERR_INVALID_ARG, "unknown operator %d", op);
  }
  ORI_TRY(matvec(c, PREC_F64, fp, f1, i1, nullptr));
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  return ORI_OK;
}

ori_status ori_solve(ori_ctx c, const ori_solve_opts* opts_in, void* u_out, ori_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  ORI_TRY(guard(c));
  if (!c->loaded) return set_err(c, ORI_ERR_INVALID_ARG, "ori_load has not succeeded on this context");
  ori_solve_opts o;
  if (opts_in)
    o = *opts_in;
  else
    ori_default_opts(&o);
  if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) return set_err(c, ORI_ERR_INVALID_ARG, "tol must be finite and >= 0");
  if (o.max_iter < 0) return set_err(c, ORI_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (o.precision != ORI_FP64 && o.precision != ORI_MIXED) return set_err(c, ORI_ERR_INVALID_ARG, "bad precision");
  if (o.precision == ORI_MIXED && !(c->provision & ORI_PROVISION_MIXED))
    return set_err(c, ORI_ERR_INVALID_ARG, "complex64 workspaces were not provisioned");
  if (o.check_every < 0) return set_err(c, ORI_ERR_INVALID_ARG, "check_every must be >= 0");
  const int check_every = o.check_every == 0 ? 1 : o.check_every;
  const double inner_tol = o.inner_tol > 0.0 ? o.inner_tol : 1e-5;
  if (!std::isfinite(inner_tol) || inner_tol >= 1.0) return set_err(c, ORI_ERR_INVALID_ARG, "inner_tol must be in (0, 1)");
  const int max_outer = o.max_outer > 0 ? o.max_outer : 10;
  ORI_TRY(check_dev_ptr(c, u_out, c->P * 16, "u"));
  cxd* u = static_cast<cxd*>(u_out);
  const int64_t P = c->P;

  ori_solve_info inf{};
  inf.rel_res_true = -1.0;
  const double bb = c->bnorm2;
  const double rr_target = o.tol * o.tol * bb;
  bool breakdown = false, converged = false;

  // initial residual r = b - A_sym x0
  if (o.use_x0) {
    ORI_TRY(launch(c, K_ELEMWISE, PREC_F64, [&] { return launch_mul(c->S, u, c->x, P, c->stream); }));
    ORI_TRY(true_residual_sym(c, c->x, c->r));
    inf.matvecs++;
  } else {
    ORI_TRY(launch(c, K_INIT, PREC_F64, [&] { return launch_init(PREC_F64, c->b, 1.0, c->x, c->r, P, c->partials, c->stream); }));
    ORI_TRY(finalize(c, kRedBlocks, FIN_INIT));
  }

  if (o.precision == ORI_FP64) {
    CocgOut co;
    ORI_TRY(run_cocg(c, PREC_F64, c->x, c->r, c->p, c->q, c->S, rr_target, o.max_iter, check_every, &co));
    inf.iterations = co.iters;
    inf.matvecs += co.matvecs;
    inf.rel_res_recursive = bb > 0 ? std::sqrt(co.rr / bb) : 0.0;
    converged = co.converged;
    breakdown = !converged && (co.flags & (FLAG_BREAKDOWN_RHO | FLAG_BREAKDOWN_MU));
  } else {
    // iterative refinement: FP64 true residual, complex64 inner COCG on the correction
    ORI_TRY(sync_scalars(c));
    double rr = c->sc_host->rr;
    int flags = c->sc_host->flags;
    if (flags & FLAG_BREAKDOWN_RHO) breakdown = true;
    int inner_left = o.max_iter;
    for (int outer = 0; !breakdown; ++outer) {
      if (rr <= rr_target || (flags & FLAG_ZERO_RESIDUAL)) {
        converged = true;
        break;
      }
      if (outer >= max_outer || inner_left <= 0) break;
      const double scale = 1.0 / std::sqrt(rr);
      ORI_TRY(launch(c, K_INIT, PREC_F32,
                     [&] { return launch_init(PREC_F32, c->r, scale, c->xf, c->rf, P, c->partials, c->stream); }));
      ORI_TRY(finalize(c, kRedBlocks, FIN_INIT));
      CocgOut co;
      ORI_TRY(run_cocg(c, PREC_F32, c->xf, c->rf, c->pf, c->qf, c->Sf, inner_tol * inner_tol, inner_left,
                       check_every, &co));
      inner_left -= co.iters;
      inf.iterations += co.iters;
      inf.matvecs += co.matvecs;
      inf.matvecs_c64 += co.matvecs;
      if (co.iters == 0 && (co.flags & (FLAG_BREAKDOWN_RHO | FLAG_BREAKDOWN_MU))) {
        breakdown = true;
        break;
      }
      ORI_TRY(launch(c, K_ELEMWISE, PREC_F32,
                     [&] { return launch_axpy_d(PREC_F32, 1.0 / scale, c->xf, c->x, P, c->stream); }));
      ORI_TRY(true_residual_sym(c, c->x, c->r));
      inf.matvecs++;
      inf.refinements++;
      ORI_TRY(sync_scalars(c));
      rr = c->sc_host->rr;
      flags = c->sc_host->flags & ~(FLAG_BREAKDOWN_RHO | FLAG_BREAKDOWN_MU);
    }
    inf.rel_res_recursive = bb > 0 ? std::sqrt(rr / bb) : 0.0;
  }

  ORI_TRY(recover(c, c->x, u));
  inf.matvecs++;
  if (o.true_residual) {
    ORI_TRY(true_residual_orig(c, u, &inf.rel_res_true));
    inf.matvecs++;
  }
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  if (breakdown) return set_err(c, ORI_ERR_BREAKDOWN, "COCG breakdown after %d iterations", inf.iterations);
  if (!converged)
    return set_err(c, ORI_ERR_NOT_CONVERGED, "not converged: relative residual %.3e after %d iterations",
                   inf.rel_res_recursive, inf.iterations);
  return ORI_OK;
}

ori_status ori_profile_enable(ori_ctx c, int32_t enable) {
  ORI_TRY(guard(c));
  if (enable) {
    ORI_TRY(prof_fold(c));
    std::fill(std::begin(c->prof_ms), std::end(c->prof_ms), 0.0);
    std::fill(std::begin(c->prof_n), std::end(c->prof_n), 0);
    c->prof = true;
  } else {
    ORI_TRY(prof_fold(c));
    c->prof = false;
  }
  return ORI_OK;
}

ori_status ori_profile_read(ori_ctx c, int32_t max, const char** names, double* avg_ms, int64_t* launches,
                            int32_t* count) {
  ORI_TRY(guard(c));
  ORI_TRY(prof_fold(c));
  static const char* const full[2 * K_NKIND] = {
      "f1.c128", "f1.c64", "f2.c128", "f2.c64", "zpass.c128", "zpass.c64", "i2.c128", "i2.c64",
      "i1.c128", "i1.c64", "update.c128", "update.c64", "finalize", "finalize.c64", "init.c128", "init.c64",
      "coefficients", "coefficients.c64", "embed", "embed.c64", "spectrum_fft", "spectrum_fft.c64",
      "octant", "octant.c64", "elementwise.c128", "elementwise.c64"};
  int w = 0;
  for (int s = 0; s < 2 * K_NKIND; ++s) {
    if (c->prof_n[s] == 0) continue;
    if (w < max) {
      if (names) names[w] = full[s];
      if (avg_ms) avg_ms[w] = c->prof_ms[s] / static_cast<double>(c->prof_n[s]);
      if (launches) launches[w] = c->prof_n[s];
    }
    ++w;
  }
  if (count) *count = w;
  return ORI_OK;
}

void ori_destroy(ori_ctx c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->sc_host) (void)hipHostFree(c->sc_host);
  delete c;
}

const char* ori_last_error(ori_ctx c) { return c ? c->err.c_str() : g_last_error.c_str(); }

}  // extern "C"
