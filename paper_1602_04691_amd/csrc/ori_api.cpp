// Host runtime and C ABI (include/ori.h): context, workspaces, the FFT
// product with the Green's matrix (Section 3), COCG (van der Vorst &
// Melissen, cited by the paper) with HIP-graph replay of its iterations,
// mixed-precision refinement, batches of right-hand sides, the adjoint, the
// layout autotuner, and the physics of the solution (charges, field, far
// field, refraction recipe, and the Table 4 comparison of Section 4).
#include "ori.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <memory>
#include <vector>

#include "cx.h"
#include "kernels.h"
#include "launch.h"
#include "plan.h"

namespace ori {
namespace {
thread_local GraphBuild* t_graph = nullptr;
}
GraphBuild* graph_being_built() { return t_graph; }

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
constexpr int64_t kMaxRhs = 1024;
// Z-pass workgroups below which a batch is split over its right-hand sides
constexpr int64_t kZMinWorkgroups = 4096;

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
  K_SPEC_FFT,
  K_ELEMWISE,
  K_NKIND
};
const char* const kKindNames[K_NKIND] = {"f1", "f2", "zpass", "i2", "i1", "update", "finalize",
                                         "init", "coefficients", "spectrum", "elementwise"};

thread_local std::string g_last_error = "no error";

constexpr int64_t kGuardBytes = kGuardBandBytes;
constexpr unsigned char kGuardByte = 0xA5;

// Blocks of destroyed contexts and groups, kept for the next ones of the
// same size: device workspaces, pinned host mirrors and group streams.
// Contexts made and destroyed in a loop (a group per batch of problems) then
// skip hipMalloc, hipFree (which waits for the device), hipHostMalloc and
// stream creation and destruction.  A block is reused only on its own device
// and at its exact size.  At most kPoolBytes of memory per kind are kept;
// larger blocks, and blocks beyond that, are freed at once.  A block comes
// back only after its owner's work has finished (ori_destroy and
// ori_group_destroy wait for their streams first), and a block taken again
// holds whatever its last owner left: every workspace is initialised by the
// code that uses it.  ori_release_cached_memory frees every kept block.
constexpr size_t kPoolBytes = size_t{4} << 30;
constexpr size_t kPoolStreams = 64;

class BlockPool {
 public:
  enum Kind { DEVICE, HOST };
  explicit BlockPool(Kind kind) : kind_(kind) {}
  // a kept block of exactly `bytes` on `device`, or NULL
  void* take(int device, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = free_.find({device, bytes});
    if (it == free_.end() || it->second.empty()) return nullptr;
    void* p = it->second.back();
    it->second.pop_back();
    kept_ -= bytes;
    return p;
  }
  // keeps p for a later take, or frees it
  void give(int device, size_t bytes, void* p) {
    if (!p) return;
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (kept_ + bytes <= kPoolBytes) {
        free_[{device, bytes}].push_back(p);
        kept_ += bytes;
        return;
      }
    }
    free_block(device, p);
  }
  void release_all() {
    std::map<std::pair<int, size_t>, std::vector<void*>> all;
    {
      std::lock_guard<std::mutex> lk(mu_);
      all.swap(free_);
      kept_ = 0;
    }
    for (auto& kv : all)
      for (void* p : kv.second) free_block(kv.first.first, p);
  }

 private:
  void free_block(int device, void* p) {
    if (kind_ == HOST) {
      (void)hipHostFree(p);
      return;
    }
    int cur = 0;
    const bool switch_dev = hipGetDevice(&cur) == hipSuccess && cur != device;
    if (switch_dev) (void)hipSetDevice(device);
    (void)hipFree(p);
    if (switch_dev) (void)hipSetDevice(cur);
  }
  Kind kind_;
  std::mutex mu_;
  std::map<std::pair<int, size_t>, std::vector<void*>> free_;
  size_t kept_ = 0;
};

// process-wide pools (never destroyed: blocks still kept at exit go with the
// process)
BlockPool& device_pool() {
  static BlockPool* p = new BlockPool(BlockPool::DEVICE);
  return *p;
}
BlockPool& host_pool() {
  static BlockPool* p = new BlockPool(BlockPool::HOST);
  return *p;
}

// device memory of `bytes` on the current device `device`: a kept block, or
// hipMalloc
hipError_t pool_malloc(int device, size_t bytes, void** p) {
  *p = device_pool().take(device, bytes);
  if (*p) return hipSuccess;
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) *p = nullptr;
  return e;
}
// pinned host memory of `bytes`: a kept block, or hipHostMalloc
hipError_t pool_host_malloc(size_t bytes, void** p) {
  *p = host_pool().take(-1, bytes);
  if (*p) return hipSuccess;
  const hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
  if (e != hipSuccess) *p = nullptr;
  return e;
}

// Non-blocking streams for group members, kept per device.
struct StreamPool {
  std::mutex mu;
  std::map<int, std::vector<hipStream_t>> free;
};
StreamPool& stream_pool() {
  static StreamPool* p = new StreamPool();
  return *p;
}
hipError_t pool_stream(int device, hipStream_t* s) {
  {
    std::lock_guard<std::mutex> lk(stream_pool().mu);
    auto& v = stream_pool().free[device];
    if (!v.empty()) {
      *s = v.back();
      v.pop_back();
      return hipSuccess;
    }
  }
  return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}
// s has no work left (the caller waited for it)
void pool_stream_give(int device, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(stream_pool().mu);
    auto& v = stream_pool().free[device];
    if (v.size() < kPoolStreams) {
      v.push_back(s);
      return;
    }
  }
  (void)hipStreamDestroy(s);
}

// Layout knobs of the FFT passes (performance only)
struct Knobs {
  int blk_lg = 4;  // log2 of the i1 block of the B layout (n divisible by 2^blk_lg)
  int np_sel = 0;  // strided tile width: 0 wide, 1 narrow
  int zpf = 0;     // Z pass: prefetch the next tile
  int z_np = 0;    // Z tile width: 0 wide, 1 narrow
  int zplan = 0;   // Z radix plan: 0 the length's default, 1 its alternative (plan.h)
  bool operator==(const Knobs& o) const {
    return blk_lg == o.blk_lg && np_sel == o.np_sel && zpf == o.zpf && z_np == o.z_np && zplan == o.zplan;
  }
};

// Tuned layouts, process-wide, by (device, n, nrhs): a context created on a
// tuned key starts from the tuned layout.
struct TuneKey {
  int device;
  int64_t n, nrhs;
  bool operator<(const TuneKey& o) const {
    return device != o.device ? device < o.device : n != o.n ? n < o.n : nrhs < o.nrhs;
  }
};
struct Tuned {
  Knobs k[2];
  bool have[2] = {false, false};
};
std::mutex g_tune_mu;

std::map<TuneKey, Tuned> g_tuned;

// Cached HIP graphs of COCG iteration blocks, the most recently used last.
// An entry holds `iters` iterations (the first of them the first COCG
// iteration when `first`) of every context in `members`, one independent
// chain per context.  A few entries are kept, so that every block shape of
// a solve stays cached across solves: the first block, full blocks, and the
// blocks of the members left running once others are done.
struct IterGraph {
  struct Entry {
    hipGraphExec_t exec = nullptr;
    int iters = 0;
    bool first = false;
    std::vector<ori_ctx> members;
    const void* multi = nullptr;  // the MultiSet its launches serve, or NULL (one chain per member)
  };
  std::vector<Entry> entries;
  hipEvent_t done = nullptr;  // recorded after a replay, waited on by each member's stream
  void release() {
    for (auto& e : entries)
      if (e.exec) (void)hipGraphExecDestroy(e.exec);
    entries.clear();
    if (done) (void)hipEventDestroy(done);
    done = nullptr;
  }
};
constexpr size_t kGraphCacheEntries = 8;

struct ProfPending {
  int slot;  // kind * 2 + (fprec == F32)
  int ev;
};

}  // namespace

struct ori_ctx_s {
  ori_grid grid{};
  int64_t n = 0, L = 0, P = 0;
  int64_t nrhs = 1;  // right-hand sides per solve (fixed at create)
  int provision = 0;
  double k = 0.0;
  bool loaded = false;
  bool poisoned = false;
  // the kernel spectrum depends only on (n, side, k): ori_load keeps it while
  // k is unchanged (spectrum_k), unless the cache is switched off
  bool spectrum_cache = true;
  bool spectrum_valid = false;
  double spectrum_k = 0.0;
  hipStream_t stream = nullptr;
  int device = 0;
  const LengthKernels* K = nullptr;
  Knobs knob[2];   // layout of the FFT passes, [0] complex128 FFTs, [1] complex64
  bool recover_by_division = false;  // u = w / S (no S_p near zero)
  std::string err = "no error";
  std::vector<double> u0norm2, bnorm2;     // per right-hand side
  std::vector<ori_solve_info> last_info;  // per right-hand side, last solve

  void* arena = nullptr;                      // A/B work arrays of the FFT passes, nrhs of them
  cxd *D = nullptr, *S = nullptr;             // shared diagonals
  double* cN = nullptr;                       // 4 pi N |Delta| (real, shared)
  cxf* Sf = nullptr;
  cxd *b = nullptr, *u0 = nullptr;            // [nrhs][P]
  cxd *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;  // [nrhs][P]
  cxf *xf = nullptr, *rf = nullptr, *pf = nullptr, *qf = nullptr;
  cxd *t1 = nullptr, *t2 = nullptr;           // adjoint work vectors (one right-hand side)
  cxd* kh = nullptr;
  cxf* khf = nullptr;
  cxd* twd = nullptr;
  cxf* twf = nullptr;
  double* partials = nullptr;
  ScalarBlock* sc = nullptr;       // [nrhs]
  ScalarBlock* sc_host = nullptr;  // pinned mirror
  double* outer_m = nullptr;       // [2 nrhs]: refinement multipliers, then inner tolerances^2
  double* outer_m_host = nullptr;  // pinned
  // every device workspace is carved from one block (device_pool), the two
  // pinned mirrors from one pinned block (host_pool)
  void* ws_block = nullptr;
  size_t ws_bytes = 0;
  void* pin_block = nullptr;
  size_t pin_bytes = 0;
  // guard band after every workspace: kGuardBytes of kGuardByte, checked by
  // ori_check_guards and, with ORI_CHECK_GUARDS=1 in the environment at
  // create, after every kernel launch
  std::vector<unsigned char*> guards;
  bool check_guards = false;
  // ORI_TRACE=1 in the environment at create: the residual of every
  // right-hand side on stderr after every check of a solve
  bool trace = false;

  // COCG iteration blocks as HIP graphs, one per vector precision
  IterGraph graphs[2];

  // profiling
  bool prof = false;
  uint32_t prof_mask = ~0u;  // bit per kernel kind that is timed
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

#define ORI_HIP(c, call)                                                                                     \
  do {                                                                                                       \
    hipError_t e_ = (call);                                                                                  \
    if (e_ != hipSuccess) return set_err((c), ORI_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define ORI_TRY(expr)            \
  do {                           \
    ori_status s_ = (expr);      \
    if (s_ != ORI_OK) return s_; \
  } while (0)

bool finite(double v) { return std::isfinite(v); }

// Padded length per axis: the shortest planned length L >= 2n - 1, so that
// the cyclic convolution of length L holds every offset in (-n, n) without
// wrap-around (the zero padding of Section 3, eq. 3.3.5); 0 beyond n = 512.
int64_t padded_length(int64_t n) {
  if (n < 1 || n > 512) return 0;
  int64_t best = 0;
#define ORI_PICK(Lc) \
  if ((Lc) >= 2 * n - 1 && (best == 0 || (Lc) < best)) best = (Lc);
  ORI_FOR_EACH_L(ORI_PICK)
#undef ORI_PICK
  return best;
}

ori_status check_grid(const ori_grid* g, int64_t* L_out) {
  if (!g) return set_err(nullptr, ORI_ERR_INVALID_ARG, "grid is NULL");
  if (g->n < 1) return set_err(nullptr, ORI_ERR_INVALID_ARG, "n = %lld must be >= 1", (long long)g->n);
  if (!(g->side > 0.0) || !finite(g->side))
    return set_err(nullptr, ORI_ERR_INVALID_ARG, "side must be finite and > 0");
  for (int i = 0; i < 3; ++i)
    if (!finite(g->origin[i])) return set_err(nullptr, ORI_ERR_INVALID_ARG, "origin must be finite");
  if (!finite(g->cell_offset)) return set_err(nullptr, ORI_ERR_INVALID_ARG, "cell_offset must be finite");
  const int64_t L = padded_length(g->n);
  if (L == 0)
    return set_err(nullptr, ORI_ERR_UNSUPPORTED, "n = %lld: no FFT plan of length >= 2n - 1 (n <= 512 is supported)",
                   (long long)g->n);
  *L_out = L;
  return ORI_OK;
}

int64_t align_up(int64_t v) { return (v + 255) / 256 * 256; }

struct Layout {
  int64_t arena, vec_d, vec_f, kh, khf, npart, total;
};

// Device bytes for n and a batch of nrhs.  Partial quadruples cover the
// largest reducing grid: I1 (at most n*n workgroups per right-hand side) and
// the reduction kernels (red_blocks(P), update_blocks(P, prec) per right-hand side).
Layout layout_for(int64_t n, int64_t nrhs, int provision) {
  const int64_t L = padded_length(n);
  const int64_t P = n * n * n, kp = L / 2 + 1;
  const bool mixed = provision & ORI_PROVISION_MIXED;
  Layout l{};
  // A (n*n*L) + B (n*L*L) complex128 per right-hand side; also the octant
  // scratch of the spectrum passes at load time
  l.arena = align_up(std::max<int64_t>(nrhs * (n * n * L + n * L * L), kp * kp * kp) * 16);
  l.vec_d = align_up(P * 16);
  l.vec_f = align_up(P * 8);
  l.kh = align_up(kp * kp * kp * 16);  // octant [L/2+1]^3
  l.khf = mixed ? align_up(kp * kp * kp * 8) : 0;
  l.npart = nrhs * std::max({red_blocks(P), update_blocks(P, PREC_F32), n * n});
  const int64_t shared = 2 * l.vec_d + l.vec_f /* cN */ + (mixed ? l.vec_f : 0) /* Sf */ + 2 * l.vec_d /* t1, t2 */;
  const int64_t batch = nrhs * (6 * l.vec_d + (mixed ? 4 * l.vec_f : 0));
  // the context's device block (ori_create: every workspace followed by its
  // guard band; the twiddle tables are shared per length)
  l.total = l.arena + shared + batch + l.kh + l.khf + align_up(l.npart * 4 * 8) +
            align_up(nrhs * (int64_t)sizeof(ScalarBlock)) + align_up(2 * nrhs * 8) + (mixed ? 22 : 16) * kGuardBytes;
  return l;
}

// align: the element alignment the kernels need (16 for complex128 arrays,
// 8 for real ones)
ori_status check_dev_ptr(ori_ctx c, const void* ptr, int64_t bytes, const char* what, int align = 16) {
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
  if (reinterpret_cast<uintptr_t>(ptr) % align != 0)
    return set_err(c, ORI_ERR_INVALID_ARG, "%s is not %d-byte aligned", what, align);
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

// number of workspaces whose guard band no longer holds kGuardByte
ori_status count_damaged_guards(ori_ctx c, int64_t* damaged) {
  std::vector<unsigned char> h(kGuardBytes);
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  int64_t bad = 0;
  for (unsigned char* g : c->guards) {
    ORI_HIP(c, hipMemcpy(h.data(), g, kGuardBytes, hipMemcpyDeviceToHost));
    for (unsigned char v : h)
      if (v != kGuardByte) {
        ++bad;
        break;
      }
  }
  *damaged = bad;
  return ORI_OK;
}

template <class F>
ori_status launch(ori_ctx c, int kind, int fprec, F&& f) {
  int evi = -1;
  const bool timed = c->prof && ((c->prof_mask >> kind) & 1u);
  if (timed) {
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
  (void)hipGetLastError();  // the launch reports its own error, not an earlier call's
  const hipError_t e = f();
  if (e != hipSuccess)
    return set_err(c, ORI_ERR_DEVICE, "kernel %s %s failed: %s", kKindNames[kind],
                   graph_being_built() ? "graph node" : "launch", hipGetErrorString(e));
  if (c->check_guards) {
    int64_t bad = 0;
    ORI_TRY(count_damaged_guards(c, &bad));
    if (bad) return set_err(c, ORI_ERR_DEVICE, "kernel %s wrote past the end of %lld workspace(s)", kKindNames[kind],
                            (long long)bad);
  }
  if (timed) {
    ORI_HIP(c, hipEventRecord(c->ev[2 * evi + 1], c->stream));
    c->pend.push_back(ProfPending{kind * 2 + (fprec == PREC_F32 ? 1 : 0), evi});
  }
  return ORI_OK;
}

ori_status sync_scalars(ori_ctx c) {
  ORI_HIP(c, hipMemcpyAsync(c->sc_host, c->sc, c->nrhs * sizeof(ScalarBlock), hipMemcpyDeviceToHost, c->stream));
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  return ORI_OK;
}

ori_status finalize(ori_ctx c, int64_t nblk, int mode, double tol2 = 0.0, int tol2_of_bb = 0,
                    const double* tol2_rhs = nullptr) {
  return launch(c, K_FINALIZE, PREC_F64, [&] {
    return launch_finalize(c->partials, nblk, c->nrhs, c->sc, mode, kBreakdownEps, tol2, tol2_of_bb, tol2_rhs,
                           c->stream);
  });
}

int64_t rblocks(ori_ctx c) { return red_blocks(c->P); }

// ---------------------------------------------------------------------------
// the FFT product: F1 -> F2 -> Z -> I2 -> I1 (prologue / epilogue in f1, i1),
// over all right-hand sides of the context at once
// ---------------------------------------------------------------------------

// The arguments of the five passes of one product of context c with FFTs
// of precision fprec, from the prologue f1 and the epilogue i1, and the
// workgroups of each pass.
struct PassArgs {
  ContigFwdArgs f1;
  StridedArgs f2;
  ZArgs z;
  StridedArgs i2;
  ContigInvArgs i1;
  int64_t blocks[MP_NPASS];
  int64_t i1_blocks_per_rhs;
};

ori_status pass_args(ori_ctx c, int fprec, ContigFwdArgs f1, ContigInvArgs i1, PassArgs* out) {
  const int64_t n = c->n, L = c->L, R = c->nrhs;
  const int64_t elem = fprec == PREC_F64 ? 16 : 8;
  char* A = static_cast<char*>(c->arena);
  char* B = A + R * n * n * L * elem;
  const void* tw = fprec == PREC_F64 ? static_cast<const void*>(c->twd) : static_cast<const void*>(c->twf);
  const void* kh = fprec == PREC_F64 ? static_cast<const void*>(c->kh) : static_cast<const void*>(c->khf);
  if (!kh) return set_err(c, ORI_ERR_INVALID_ARG, "complex64 workspaces were not provisioned");

  f1.half_in = 1;
  f1.out = A;
  f1.nrhs = R;
  f1.ppr = n * n;
  f1.in_pitch = n;
  f1.out_pitch = L;
  f1.tw = tw;
  out->f1 = f1;

  // B layout: i1 split into blocks of 2^lg rows (see ZArgs); the batch is
  // just more outer rows
  const Knobs& kn = c->knob[fprec == PREC_F32 ? 1 : 0];
  const int lg = kn.blk_lg;
  const int64_t Bk = int64_t{1} << lg;
  const int ns = kn.np_sel;
  out->f2 = StridedArgs{A, B, R * n, L, n, 0, lg, n * L, 0, L, L * L * Bk, L, Bk * L, 0, 1, 0, ns, tw};

  // Small grids (a batch at small n) are split over the right-hand sides,
  // so that the pass has enough workgroups to fill the chip; no slice is
  // left empty.
  const int64_t zbase = c->K->zpass_blocks(fprec, kn.z_np);
  int64_t rs = std::min<int64_t>(R, (kZMinWorkgroups + zbase - 1) / zbase);
  if (rs > 1) rs = (R + (R + rs - 1) / rs - 1) / ((R + rs - 1) / rs);
  out->z = ZArgs{B,  n,  lg, kn.z_np, L * L * Bk, L, Bk * L, R, n * L * L, kn.zpf, static_cast<int32_t>(rs),
                 kh, L / 2 + 1, tw, kn.zplan};

  out->i2 = StridedArgs{B, A, R * n, L, n, lg, 0, L * L * Bk, L, Bk * L, n * L, 0, L, 1, 0, 1, ns, tw};

  i1.in = A;
  i1.nrhs = R;
  i1.ppr = n * n;
  i1.in_pitch = L;
  i1.out_pitch = n;
  i1.tw = tw;
  out->i1 = i1;

  const int64_t cb = c->K->contig_blocks_per_rhs(n * n);
  out->i1_blocks_per_rhs = cb;
  out->blocks[MP_F1] = R * cb;
  out->blocks[MP_F2] = c->K->strided_blocks(fprec, ns, R * n, L);
  out->blocks[MP_Z] = zbase * rs;
  out->blocks[MP_I2] = c->K->strided_blocks(fprec, ns, R * n, L);
  out->blocks[MP_I1] = R * cb;
  return ORI_OK;
}

ori_status matvec(ori_ctx c, int vprec, int fprec, ContigFwdArgs f1, ContigInvArgs i1, int64_t* nblk_out) {
  PassArgs pa;
  ORI_TRY(pass_args(c, fprec, f1, i1, &pa));
  ORI_TRY(launch(c, K_F1, fprec, [&] { return c->K->contig_fwd(vprec, fprec, pa.f1, c->stream); }));
  ORI_TRY(launch(c, K_F2, fprec, [&] { return c->K->strided(fprec, pa.f2, c->stream); }));
  ORI_TRY(launch(c, K_Z, fprec, [&] { return c->K->zpass(fprec, pa.z, c->stream); }));
  ORI_TRY(launch(c, K_I2, fprec, [&] { return c->K->strided(fprec, pa.i2, c->stream); }));
  if (nblk_out) *nblk_out = pa.i1_blocks_per_rhs;
  ORI_TRY(launch(c, K_I1, fprec, [&] { return c->K->contig_inv(vprec, fprec, pa.i1, c->stream); }));
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
// setup: the kernel spectrum (a2), three in-place passes on its octant
// ---------------------------------------------------------------------------
ori_status compute_spectrum(ori_ctx c) {
  const double L = static_cast<double>(c->L);
  // the octant scratch of passes 1-2 lives in the (idle) FFT work arena
  SpectrumArgs a{c->arena, c->kh, c->khf, c->n, c->k, c->grid.side / static_cast<double>(c->n), 1.0 / (L * L * L), 1,
                 0, c->twd};
  for (int pass = 1; pass <= 3; ++pass) {  // 1/L^3 of the inverse DFT is folded in by pass 3
    a.pass = pass;
    ORI_TRY(launch(c, K_SPEC_FFT, PREC_F64, [&] { return c->K->spectrum(a, c->stream); }));
  }
  return ORI_OK;
}

void fill_twiddles(int64_t L, std::vector<cxd>& d, std::vector<cxf>& f) {
  d.resize(L);
  f.resize(L);
  const long double two_pi = 6.283185307179586476925286766559L;
  for (int64_t m = 0; m < L; ++m) {
    // exp(-2 pi i m / L) in long double, exact at the quarter turns
    const long double a = two_pi * static_cast<long double>(m) / static_cast<long double>(L);
    long double cs = cosl(a), sn = sinl(a);
    if (4 * m % L == 0) {
      const int64_t q = 4 * m / L;
      cs = (q == 0) ? 1 : (q == 2) ? -1 : 0;
      sn = (q == 1) ? 1 : (q == 3) ? -1 : 0;
    }
    d[m] = cxd{static_cast<double>(cs), static_cast<double>(-sn)};
    f[m] = cxf{static_cast<float>(cs), static_cast<float>(-sn)};
  }
}

// The twiddle tables of padded length L on a device (fill_twiddles), made
// on first use and shared, read only, by every context of that length on
// that device for the rest of the process.
ori_status shared_twiddles(int device, int64_t L, cxd** twd, cxf** twf) {
  static std::mutex mu;
  static auto* tabs = new std::map<std::pair<int, int64_t>, std::pair<cxd*, cxf*>>();
  std::lock_guard<std::mutex> lk(mu);
  auto it = tabs->find({device, L});
  if (it == tabs->end()) {
    std::vector<cxd> d;
    std::vector<cxf> f;
    fill_twiddles(L, d, f);
    void* pd = nullptr;
    void* pf = nullptr;
    if (hipMalloc(&pd, L * sizeof(cxd)) != hipSuccess || hipMalloc(&pf, L * sizeof(cxf)) != hipSuccess ||
        hipMemcpy(pd, d.data(), L * sizeof(cxd), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pf, f.data(), L * sizeof(cxf), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      if (pd) (void)hipFree(pd);
      if (pf) (void)hipFree(pf);
      g_last_error = "twiddle tables: allocation or copy failed";
      return ORI_ERR_DEVICE;
    }
    it = tabs->emplace(std::make_pair(device, L), std::make_pair(static_cast<cxd*>(pd), static_cast<cxf*>(pf))).first;
  }
  *twd = it->second.first;
  *twf = it->second.second;
  return ORI_OK;
}

// ---------------------------------------------------------------------------
// COCG on (I + S G0 S) w = rhs for every right-hand side in lockstep,
// vectors of type prec (FFTs too).  Expects x, r initialised and FIN_INIT
// done (per right-hand side targets set); a right-hand side that converges
// or breaks down is frozen on the device (alpha = 0) while the others go on.
// ---------------------------------------------------------------------------

bool all_done(ori_ctx c) {
  for (int64_t i = 0; i < c->nrhs; ++i)
    if (!(c->sc_host[i].flags & FLAG_DONE)) return false;
  return true;
}

// One COCG iteration on every right-hand side: x += alpha p (the previous
// iteration's step) and p = r + beta p (p = r when first) in F1, q = (I +
// S G0 S) p with <p,q>, then alpha, r and rho.  The step x += alpha p of
// the last iteration is left pending for flush_x.  No memset and no host
// work, so its launches can also be built into a graph (iteration_graph).
ori_status cocg_iteration(ori_ctx c, int prec, void* x, void* r, void* p, void* q, const void* S, bool first) {
  ContigFwdArgs f1{};
  f1.x = r;
  f1.pvec = p;
  f1.xvec = x;  // applies the previous iteration's x += alpha p
  f1.s_in = S;
  f1.sc = c->sc;
  f1.mode = 1;
  f1.first = first;
  ContigInvArgs i1 = epi(q, p, 1.0, nullptr, 0.0, S, 1.0, c->partials, 0);
  int64_t nblk = 0;
  ORI_TRY(matvec(c, prec, prec, f1, i1, &nblk));
  ORI_TRY(finalize(c, nblk, FIN_MU));
  ORI_TRY(launch(c, K_UPDATE, prec, [&] {
    return launch_update(prec, nullptr, p, r, q, c->P, c->nrhs, c->sc, c->partials, c->stream);
  }));
  return finalize(c, update_blocks(c->P, prec), FIN_RHO);
}

// The COCG vectors of precision prec of a context (the FFTs run in the same
// precision).
struct PrecVecs {
  void *x, *r, *p, *q;
  const void* S;
};
PrecVecs vecs(ori_ctx c, int prec) {
  if (prec == PREC_F32) return PrecVecs{c->xf, c->rf, c->pf, c->qf, c->Sf};
  return PrecVecs{c->x, c->r, c->p, c->q, c->S};
}

ori_status iteration(ori_ctx c, int prec, bool first) {
  const PrecVecs v = vecs(c, prec);
  return cocg_iteration(c, prec, v.x, v.r, v.p, v.q, v.S, first);
}

// Several contexts solved in lockstep: the members of an ori_group (a
// stream each), or a single context.
using Members = std::vector<ori_ctx>;

// ---------------------------------------------------------------------------
// The COCG iteration of several problems in one launch per kernel
// (kernels.h, MultiProblem; the uneven batch of an ori_group).  A MultiSet
// holds the device tables of one set of members in one precision: the five
// passes (F1 twice: the first iteration and the others), the finalisations
// of the product and of the update, and the update.  The tables hold the
// arguments each member's own launches take, so every member computes what
// its own solve computes.
// ---------------------------------------------------------------------------
struct MultiSet {
  Members members;
  int prec = 0;
  void* dev = nullptr;  // every table, one block (device_pool)
  size_t dev_bytes = 0;
  int device = 0;
  const MultiProblem* f1_first = nullptr;
  const MultiProblem* pass[MP_NPASS] = {};
  int64_t blocks[MP_NPASS] = {};
  int threads[MP_NPASS] = {};
  int smem[MP_NPASS] = {};
  const MultiFin* fin_mu = nullptr;
  const MultiFin* fin_rho = nullptr;
  const MultiUpd* upd = nullptr;
  int64_t fin_blocks = 0, upd_blocks = 0;
};

// The MultiSets of an ori_group, built on first use and kept (a later
// solve of the same members reuses them).  Cached graphs of either
// precision point into them, so they go together: release() drops the
// group's graphs (graphs[2]) first.
struct MultiCache {
  std::vector<std::unique_ptr<MultiSet>> sets;
  IterGraph* graphs = nullptr;  // the group's graph caches, [2]
  int64_t iterations = 0;       // COCG iterations run this way (per member set, not per member)
  ScalarBlock* gathered = nullptr;      // pinned, one block per member: the scalars after a block of iterations
  ScalarBlock* gathered_dev = nullptr;  // its device address
  void release() {
    if (graphs) {
      graphs[0].release();
      graphs[1].release();
    }
    for (auto& m : sets) device_pool().give(m->device, m->dev_bytes, m->dev);
    sets.clear();
  }
};
constexpr size_t kMultiSetsMax = 32;
// problems in one ori_group (and scalar blocks in MultiCache::gathered)
constexpr int32_t kGroupMaxProblems = 64;

// whether the members can run in one launch per kernel in precision prec:
// lengths with multi-problem bodies, one right-hand side each, the tile
// shape of those bodies, no per-kernel profiling or guard checks
bool multi_ok(const Members& ms, int prec) {
  if (ms.size() < 2) return false;
  const int f = prec == PREC_F32 ? 1 : 0;
  for (ori_ctx c : ms) {
    const Knobs& k = c->knob[f];
    if (!multi_length(static_cast<int>(c->L)) || c->nrhs != 1 || c->prof || c->check_guards || k.np_sel != 0 ||
        k.zpf != 0 || k.zplan != 0 || k.z_np != kMultiZNarrow[f])
      return false;
  }
  return true;
}

template <class E>
size_t table_bytes(size_t n) {
  return (n * sizeof(E) + 255) / 256 * 256;
}

ori_status multi_set(MultiCache& mc, const Members& act, int prec, const MultiSet** out) {
  for (auto& m : mc.sets)
    if (m->prec == prec && m->members == act) {
      *out = m.get();
      return ORI_OK;
    }
  ori_ctx c0 = act.front();
  const size_t M = act.size();
  auto ms = std::make_unique<MultiSet>();
  ms->members = act;
  ms->prec = prec;
  std::vector<MultiProblem> tp[MP_NPASS + 1];  // [MP_NPASS]: F1 of the first iteration
  std::vector<MultiFin> fmu(M), frho(M);
  std::vector<MultiUpd> up(M);
  int64_t first[MP_NPASS] = {};
  for (size_t i = 0; i < M; ++i) {
    ori_ctx c = act[i];
    const PrecVecs v = vecs(c, prec);
    ContigFwdArgs f1{};  // as cocg_iteration
    f1.x = v.r;
    f1.pvec = v.p;
    f1.xvec = v.x;
    f1.s_in = v.S;
    f1.sc = c->sc;
    f1.mode = 1;
    PassArgs pa;
    ORI_TRY(pass_args(c, prec, f1, epi(v.q, v.p, 1.0, nullptr, 0.0, v.S, 1.0, c->partials, 0), &pa));
    const int L = static_cast<int>(c->L);
    for (int p = 0; p < MP_NPASS; ++p) {
      MultiProblem e{};
      e.first_block = first[p];
      e.nblocks = pa.blocks[p];
      e.L = L;
      e.ex = 2 * c->n == c->L;
      e.soff = multi_z_soff(L, prec, pa.z.e_lg);
      if (p == MP_F1) e.a.f1 = pa.f1;
      if (p == MP_F2) e.a.s = pa.f2;
      if (p == MP_Z) e.a.z = pa.z;
      if (p == MP_I2) e.a.s = pa.i2;
      if (p == MP_I1) e.a.i1 = pa.i1;
      tp[p].push_back(e);
      if (p == MP_F1) {
        e.a.f1.first = 1;
        tp[MP_NPASS].push_back(e);
      }
      first[p] += pa.blocks[p];
      ms->threads[p] = std::max(ms->threads[p], multi_pass_threads(L, prec, p));
      ms->smem[p] = std::max(ms->smem[p], multi_pass_smem(L, prec, p));
      ms->blocks[p] = first[p];
    }
    const int64_t ub = update_blocks(c->P, prec);
    fmu[i] = MultiFin{c->partials, pa.i1_blocks_per_rhs, c->sc, static_cast<int64_t>(i)};
    frho[i] = MultiFin{c->partials, ub, c->sc, static_cast<int64_t>(i)};
    up[i] = MultiUpd{v.p, v.r, v.q, c->P, c->sc, c->partials, ms->upd_blocks, ub};
    ms->upd_blocks += ub;
  }
  ms->fin_blocks = static_cast<int64_t>(M);
  // one host image of every table, copied once
  const size_t bp = table_bytes<MultiProblem>(M), bf = table_bytes<MultiFin>(M), bu = table_bytes<MultiUpd>(M);
  std::vector<unsigned char> img((MP_NPASS + 1) * bp + 2 * bf + bu, 0);
  for (int p = 0; p <= MP_NPASS; ++p) std::memcpy(img.data() + p * bp, tp[p].data(), M * sizeof(MultiProblem));
  unsigned char* tail = img.data() + (MP_NPASS + 1) * bp;
  std::memcpy(tail, fmu.data(), M * sizeof(MultiFin));
  std::memcpy(tail + bf, frho.data(), M * sizeof(MultiFin));
  std::memcpy(tail + 2 * bf, up.data(), M * sizeof(MultiUpd));
  ms->device = c0->device;
  ORI_HIP(c0, pool_malloc(ms->device, img.size(), &ms->dev));
  ms->dev_bytes = img.size();
  const hipError_t e = hipMemcpy(ms->dev, img.data(), img.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    device_pool().give(ms->device, ms->dev_bytes, ms->dev);
    return set_err(c0, ORI_ERR_DEVICE, "copy of the multi-problem tables failed: %s", hipGetErrorString(e));
  }
  unsigned char* d = static_cast<unsigned char*>(ms->dev);
  for (int p = 0; p < MP_NPASS; ++p) ms->pass[p] = reinterpret_cast<const MultiProblem*>(d + p * bp);
  ms->f1_first = reinterpret_cast<const MultiProblem*>(d + MP_NPASS * bp);
  d += (MP_NPASS + 1) * bp;
  ms->fin_mu = reinterpret_cast<const MultiFin*>(d);
  ms->fin_rho = reinterpret_cast<const MultiFin*>(d + bf);
  ms->upd = reinterpret_cast<const MultiUpd*>(d + 2 * bf);
  mc.sets.push_back(std::move(ms));
  *out = mc.sets.back().get();
  return ORI_OK;
}

// The scalar blocks of every member of m on the host after work that ran
// on the first member's stream: one gather into pinned memory, one wait,
// then each member's mirror.
ori_status multi_sync_scalars(MultiCache& mc, const MultiSet& m) {
  ori_ctx c0 = m.members.front();
  const int32_t np = static_cast<int32_t>(m.members.size());
  if (np > kGroupMaxProblems) return set_err(c0, ORI_ERR_INVALID_ARG, "%d problems in one group", np);
  if (!mc.gathered) {
    if (pool_host_malloc(kGroupMaxProblems * sizeof(ScalarBlock), reinterpret_cast<void**>(&mc.gathered)) !=
        hipSuccess) {
      mc.gathered = nullptr;
      return set_err(c0, ORI_ERR_OUT_OF_MEMORY, "hipHostMalloc of the gathered scalars failed");
    }
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&mc.gathered_dev), mc.gathered, 0) != hipSuccess) {
      host_pool().give(-1, kGroupMaxProblems * sizeof(ScalarBlock), mc.gathered);
      mc.gathered = nullptr;
      mc.gathered_dev = nullptr;
      return set_err(c0, ORI_ERR_DEVICE, "hipHostGetDevicePointer of the gathered scalars failed");
    }
  }
  ORI_HIP(c0, launch_gather_scalars(m.fin_mu, np, mc.gathered_dev, c0->stream));
  ORI_HIP(c0, hipStreamSynchronize(c0->stream));
  for (int32_t i = 0; i < np; ++i) m.members[i]->sc_host[0] = mc.gathered[i];
  return ORI_OK;
}

// One COCG iteration of every member of m on stream st: the launches of
// cocg_iteration, one for all members each.
ori_status multi_iteration(const MultiSet& m, bool first, hipStream_t st) {
  ori_ctx c0 = m.members.front();
  const int32_t np = static_cast<int32_t>(m.members.size());
  for (int p = 0; p < MP_NPASS; ++p) {
    const MultiProblem* tab = (p == MP_F1 && first) ? m.f1_first : m.pass[p];
    ORI_HIP(c0, launch_multi_pass(m.prec, p, tab, np, m.blocks[p], m.threads[p], m.smem[p], st));
  }
  ORI_HIP(c0, launch_multi_finalize(m.fin_mu, np, m.fin_blocks, FIN_MU, kBreakdownEps, st));
  ORI_HIP(c0, launch_multi_update(m.prec, m.upd, np, m.upd_blocks, st));
  ORI_HIP(c0, launch_multi_finalize(m.fin_rho, np, m.fin_blocks, FIN_RHO, kBreakdownEps, st));
  return ORI_OK;
}

// The graph of `iters` non-first iterations of every context of `active`,
// cached in `cache`.  It is built node by node: with graph_being_built()
// set, every launch of an iteration appends a kernel node after the previous
// node of the same context (launch.h), so each context is one chain holding
// exactly the kernels and arguments of its eager launches, in order; the
// chains of different contexts are independent, so the GPU runs them side
// by side.  No stream is put into capture mode.
ori_status iteration_graph(const Members& active, int prec, int iters, bool first, const MultiSet* multi,
                           IterGraph& cache, hipGraphExec_t* out) {
  *out = nullptr;
  ori_ctx c0 = active.front();
  auto& ents = cache.entries;
  for (size_t i = 0; i < ents.size(); ++i) {
    if (ents[i].iters == iters && ents[i].first == first && ents[i].members == active && ents[i].multi == multi) {
      std::rotate(ents.begin() + i, ents.begin() + i + 1, ents.end());
      *out = ents.back().exec;
      return ORI_OK;
    }
  }
  if (!cache.done) ORI_HIP(c0, hipEventCreateWithFlags(&cache.done, hipEventDisableTiming));
  if (ents.size() >= kGraphCacheEntries) {
    ORI_HIP(c0, hipGraphExecDestroy(ents.front().exec));
    ents.erase(ents.begin());
  }
  GraphBuild gb;
  ORI_HIP(c0, hipGraphCreate(&gb.graph, 0));
  t_graph = &gb;
  ori_status st = ORI_OK;
  if (multi) {
    // one chain: the launches of every member together
    for (int it = 0; it < iters && st == ORI_OK; ++it) st = multi_iteration(*multi, first && it == 0, c0->stream);
  } else {
    for (ori_ctx c : active) {
      gb.last = nullptr;  // a chain of its own
      for (int it = 0; it < iters && st == ORI_OK; ++it) st = iteration(c, prec, first && it == 0);
      if (st != ORI_OK) {
        if (c != c0) set_err(c0, st, "%s", c->err.c_str());
        break;
      }
    }
  }
  t_graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (st == ORI_OK) {
    const hipError_t e = hipGraphInstantiateWithFlags(&exec, gb.graph, 0);
    if (e != hipSuccess) {
      exec = nullptr;
      st = set_err(c0, ORI_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
  }
  (void)hipGraphDestroy(gb.graph);
  if (st != ORI_OK) return st;
  ents.push_back(IterGraph::Entry{exec, iters, first, active, multi});
  *out = exec;
  return ORI_OK;
}

// x += alpha p left pending by the last iteration
ori_status flush_x(ori_ctx c, int prec, void* x, const void* p) {
  return launch(c, K_UPDATE, prec, [&] { return launch_x_flush(prec, x, p, c->P, c->nrhs, c->sc, c->stream); });
}

// one line per right-hand side: its iterations so far, ||r|| and ||r|| / ||r0||
// (r0 the residual this COCG run started from)
void trace_cocg(ori_ctx c, int prec) {
  if (!c->trace) return;
  for (int64_t i = 0; i < c->nrhs; ++i) {
    const ScalarBlock& s = c->sc_host[i];
    std::fprintf(stderr, "[ori] cocg %s rhs %lld iter %d res %.6e rel %.6e%s\n", prec == PREC_F32 ? "c64" : "c128",
                 (long long)i, s.iters, std::sqrt(s.rr), s.rr0 > 0.0 ? std::sqrt(s.rr / s.rr0) : 0.0,
                 (s.flags & FLAG_DONE) ? " done" : "");
  }
}

// The scalar blocks of every member on the host: one copy each on the
// member's stream, then one wait per stream.
ori_status sync_members(const Members& ms) {
  for (ori_ctx c : ms)
    ORI_HIP(c, hipMemcpyAsync(c->sc_host, c->sc, c->nrhs * sizeof(ScalarBlock), hipMemcpyDeviceToHost, c->stream));
  for (size_t i = 0; i < ms.size(); ++i) {
    bool seen = false;
    for (size_t j = 0; j < i; ++j) seen = seen || ms[j]->stream == ms[i]->stream;
    if (!seen) ORI_HIP(ms[i], hipStreamSynchronize(ms[i]->stream));
  }
  return ORI_OK;
}

// COCG on every member in lockstep, vectors (and FFTs) of precision prec.
// Expects each member's x, r initialised and FIN_INIT done.  Member i runs
// at most budget[i] iterations and leaves when all its right-hand sides are
// done (a right-hand side that converges or breaks down is frozen on the
// device, alpha = 0, while the others of its context go on); ran[i]
// receives the iterations it ran.  Every full block of check_every
// iterations (the first one starting with the first COCG iteration) is one
// replay of a graph over the members still running; a shorter block (an
// iteration budget running out) runs eagerly.  Each member runs exactly the
// kernels of its own solve, so results do not depend on the other members.
ori_status group_cocg(const Members& ms, int prec, const std::vector<int>& budget, int check_every, bool use_graph,
                      IterGraph& cache, MultiCache* mc, std::vector<int>* ran) {
  ran->assign(ms.size(), 0);
  ORI_TRY(sync_members(ms));
  for (ori_ctx c : ms) {
    trace_cocg(c, prec);
    use_graph = use_graph && !c->prof && !c->check_guards;
  }
  std::vector<size_t> act;
  for (size_t i = 0; i < ms.size(); ++i)
    if (!all_done(ms[i]) && budget[i] > 0) act.push_back(i);
  int it = 0;
  while (!act.empty()) {
    int blk = check_every;
    for (size_t i : act) blk = std::min(blk, budget[i] - (*ran)[i]);
    Members active;
    for (size_t i : act) active.push_back(ms[i]);
    // members that fit run in one launch per kernel (multi_ok)
    const MultiSet* mset = nullptr;
    if (mc && multi_ok(active, prec)) {
      if (mc->sets.size() >= kMultiSetsMax) mc->release();  // with every graph that points into them
      ORI_TRY(multi_set(*mc, active, prec, &mset));
    }
    hipGraphExec_t exec = nullptr;
    if (use_graph && blk == check_every) ORI_TRY(iteration_graph(active, prec, blk, it == 0, mset, cache, &exec));
    ori_ctx c0 = active.front();
    if (mset) mc->iterations += blk;
    if (exec) {
      ORI_HIP(c0, hipGraphLaunch(exec, c0->stream));
    } else if (mset) {
      for (int j = 0; j < blk; ++j) ORI_TRY(multi_iteration(*mset, it + j == 0, c0->stream));
    } else {
      for (int j = 0; j < blk; ++j)
        for (ori_ctx c : active) ORI_TRY(iteration(c, prec, it + j == 0));
    }
    if (exec || mset) {
      // a replay, or the multi-problem launches, ran every member's work on
      // the first member's stream; the other members' streams wait for it
      // before their next work
      if (!cache.done) ORI_HIP(c0, hipEventCreateWithFlags(&cache.done, hipEventDisableTiming));
      ORI_HIP(c0, hipEventRecord(cache.done, c0->stream));
      for (ori_ctx c : active)
        if (c->stream != c0->stream) ORI_HIP(c, hipStreamWaitEvent(c->stream, cache.done, 0));
    }
    it += blk;
    for (size_t i : act) (*ran)[i] += blk;
    if (mset)
      ORI_TRY(multi_sync_scalars(*mc, *mset));  // the block ran on the first member's stream
    else
      ORI_TRY(sync_members(active));
    std::vector<size_t> next;
    for (size_t i : act) {
      trace_cocg(ms[i], prec);
      if (!all_done(ms[i]) && (*ran)[i] < budget[i]) next.push_back(i);
    }
    act.swap(next);
  }
  for (size_t i = 0; i < ms.size(); ++i) {
    if ((*ran)[i] == 0) continue;
    const PrecVecs v = vecs(ms[i], prec);
    ORI_TRY(flush_x(ms[i], prec, v.x, v.p));
  }
  return ORI_OK;
}

// r = rhs - (I + S G0 S) x in FP64 (batch), then FIN_INIT (rr, rho, targets)
ori_status true_residual_sym(ori_ctx c, const cxd* rhs, const cxd* x, cxd* r, double tol2, int tol2_of_bb) {
  int64_t nblk = 0;
  ORI_TRY(matvec(c, PREC_F64, PREC_F64, plain_f1(x, c->S), epi(r, rhs, 1.0, x, -1.0, c->S, -1.0, c->partials, 1),
                 &nblk));
  return finalize(c, nblk, FIN_INIT, tol2, tol2_of_bb);
}

// Recovery of the solution of eq. 2.19 from w = S u: u = w / S when every
// |S_p| is within 1e3 of the largest, else u = u0 - G0 S w (one product,
// valid for any S, zeros included).  Returns the products used.
ori_status recover(ori_ctx c, const cxd* w, cxd* u, int* products) {
  if (c->recover_by_division) {
    *products = 0;
    return launch(c, K_ELEMWISE, PREC_F64, [&] { return launch_div(w, c->S, u, c->P, c->nrhs, c->stream); });
  }
  *products = 1;
  return matvec(c, PREC_F64, PREC_F64, plain_f1(w, c->S), epi(u, c->u0, 1.0, nullptr, 0.0, nullptr, -1.0, nullptr, 0),
                nullptr);
}

// ||u0 - u - G0 D u|| / ||u0|| per right-hand side
// (launched; true_residual_orig_read reads it once the scalars are on the host)
ori_status true_residual_orig(ori_ctx c, const cxd* u) {
  int64_t nblk = 0;
  ORI_TRY(matvec(c, PREC_F64, PREC_F64, plain_f1(u, c->D),
                 epi(c->q, c->u0, 1.0, u, -1.0, nullptr, -1.0, c->partials, 1), &nblk));
  return finalize(c, nblk, FIN_NORM);
}

std::vector<double> true_residual_orig_read(ori_ctx c) {
  std::vector<double> rel(c->nrhs);
  for (int64_t i = 0; i < c->nrhs; ++i) {
    const double a = c->sc_host[i].aux;
    rel[i] = c->u0norm2[i] > 0 ? std::sqrt(a / c->u0norm2[i]) : std::sqrt(a);
  }
  return rel;
}

// Layout knobs: the i1 blocking of the B work array (ZArgs), the tile widths
// of the strided and of the Z passes and the Z-pass prefetch.  Start from the
// measured defaults, or from the tuned layout of this (device, n, nrhs);
// ORI_TUNE_BLK_LG / ORI_TUNE_NP / ORI_TUNE_ZPF / ORI_TUNE_ZNP / ORI_TUNE_ZPLAN override both
// for tuning runs.  Narrow Z tiles by default where they measured faster:
// complex64 at every length (at L = 512 its wide workgroup of 16 wavefronts
// fits once per CU, the narrow one three times) and complex128 from L = 512
// on (0.57 vs 0.65 ms at n = 256, while wide tiles win at L = 256).
bool valid_knobs(int64_t n, int64_t L, const Knobs& k) {
  return k.blk_lg >= 0 && k.blk_lg <= 6 && n % (int64_t{1} << k.blk_lg) == 0 && (k.np_sel == 0 || k.np_sel == 1) &&
         (k.zpf == 0 || k.zpf == 1) && (k.z_np == 0 || k.z_np == 1) &&
         (k.zplan == 0 || (k.zplan == 1 && has_plan_variant(static_cast<int>(L))));
}

// The Z pass's radix plan by default: the alternative (16 x 8 x 8) for the
// complex128 pass at L = 1024, where it measured faster, else the length's
// default.
int default_zplan(int64_t L, int f) { return (L == 1024 && f == 0) ? 1 : 0; }

void choose_layout(ori_ctx c) {
  for (int f = 0; f < 2; ++f) {
    Knobs k;
    k.z_np = (f == 1 || c->L >= 512) ? 1 : 0;
    k.zplan = default_zplan(c->L, f);
    while (k.blk_lg > 0 && (c->n % (int64_t{1} << k.blk_lg)) != 0) --k.blk_lg;
    c->knob[f] = k;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(TuneKey{c->device, c->n, c->nrhs});
    if (it != g_tuned.end())
      for (int f = 0; f < 2; ++f)
        if (it->second.have[f]) c->knob[f] = it->second.k[f];
  }
  for (int f = 0; f < 2; ++f) {
    Knobs k = c->knob[f];
    if (const char* e = std::getenv("ORI_TUNE_BLK_LG")) k.blk_lg = std::atoi(e);
    if (const char* e = std::getenv("ORI_TUNE_NP")) k.np_sel = std::atoi(e) ? 1 : 0;
    if (const char* e = std::getenv("ORI_TUNE_ZPF")) k.zpf = std::atoi(e) ? 1 : 0;
    if (const char* e = std::getenv("ORI_TUNE_ZNP")) k.z_np = std::atoi(e) ? 1 : 0;
    if (const char* e = std::getenv("ORI_TUNE_ZPLAN")) k.zplan = std::atoi(e) && has_plan_variant(c->L) ? 1 : 0;
    if (k.blk_lg < 0) k.blk_lg = 0;
    if (k.blk_lg > 6) k.blk_lg = 6;
    while (k.blk_lg > 0 && (c->n % (int64_t{1} << k.blk_lg)) != 0) --k.blk_lg;
    c->knob[f] = k;
  }
}

// Captured graphs bake the layout into their kernel arguments.
ori_status drop_graphs(ori_ctx c) {
  for (auto& g : c->graphs) g.release();
  return ORI_OK;
}

ori_status guard(ori_ctx c) {
  if (!c) return set_err(nullptr, ORI_ERR_INVALID_ARG, "context is NULL");
  if (c->poisoned)
    return set_err(c, ORI_ERR_DEVICE, "context is poisoned by an earlier device error: %s", c->err.c_str());
  ORI_HIP(c, hipSetDevice(c->device));
  return ORI_OK;
}

ori_status check_opts(ori_ctx c, const ori_solve_opts* in, ori_solve_opts* o) {
  if (!c->loaded) return set_err(c, ORI_ERR_INVALID_ARG, "ori_load has not succeeded on this context");
  if (in)
    *o = *in;
  else
    ori_default_opts(o);
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return set_err(c, ORI_ERR_INVALID_ARG, "tol must be finite and >= 0");
  if (o->max_iter < 0) return set_err(c, ORI_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (o->precision != ORI_FP64 && o->precision != ORI_MIXED) return set_err(c, ORI_ERR_INVALID_ARG, "bad precision");
  if (o->precision == ORI_MIXED && !(c->provision & ORI_PROVISION_MIXED))
    return set_err(c, ORI_ERR_INVALID_ARG, "complex64 workspaces were not provisioned");
  if (o->check_every < 0) return set_err(c, ORI_ERR_INVALID_ARG, "check_every must be >= 0");
  if (o->check_every == 0) o->check_every = 1;
  if (o->inner_tol <= 0.0) o->inner_tol = 1e-5;
  if (!std::isfinite(o->inner_tol) || o->inner_tol >= 1.0)
    return set_err(c, ORI_ERR_INVALID_ARG, "inner_tol must be in (0, 1)");
  if (o->max_outer <= 0) o->max_outer = 10;
  return ORI_OK;
}

// Per right-hand side outcome of a solve.
struct Outcome {
  std::vector<ori_solve_info> info;
  std::vector<int> state;  // 0 converged, 1 not converged, 2 breakdown
};

ori_status end_status(ori_ctx c, const Outcome& oc, const char* what) {
  int nb = 0, nn = 0;
  for (int s : oc.state) {
    nb += s == 2;
    nn += s == 1;
  }
  if (nb) return set_err(c, ORI_ERR_BREAKDOWN, "%s breakdown in %d of %zu right-hand sides", what, nb, oc.state.size());
  if (nn)
    return set_err(c, ORI_ERR_NOT_CONVERGED, "%s not converged in %d of %zu right-hand sides (relative residual %.3e)",
                   what, nn, oc.state.size(), oc.info.empty() ? 0.0 : oc.info[0].rel_res_recursive);
  return ORI_OK;
}

ori_solve_info aggregate(const Outcome& oc) {
  ori_solve_info a{};
  a.rel_res_true = -1.0;
  for (const ori_solve_info& i : oc.info) {
    a.iterations = std::max(a.iterations, i.iterations);
    a.refinements = std::max(a.refinements, i.refinements);
    a.matvecs = std::max(a.matvecs, i.matvecs);
    a.matvecs_c64 = std::max(a.matvecs_c64, i.matvecs_c64);
    a.rel_res_recursive = std::max(a.rel_res_recursive, i.rel_res_recursive);
    a.rel_res_true = std::max(a.rel_res_true, i.rel_res_true);
  }
  return a;
}

// One member of a lockstep solve of (I + S G0 S) w = rhs: its right-hand
// side (device), ||rhs_i||^2 per right-hand side (host) and its outcome.
struct SymJob {
  ori_ctx c;
  const cxd* rhs;
  std::vector<double> bb;
  Outcome* oc;
};

// Solve (I + S G0 S) w = rhs into c->x for every right-hand side of every
// member.  On entry each member's x and r hold the initial iterate and its
// residual, FIN_INIT done with the stopping targets; bb sets the same
// targets for the refinement loop.  Counts go to each member's outcome
// (added).  Every member runs the kernels of its own solve in the same
// order as alone, so its results do not depend on the others.
ori_status solve_sym_group(std::vector<SymJob>& jobs, const ori_solve_opts& o, IterGraph* cache,
                           MultiCache* mc = nullptr) {
  const size_t M = jobs.size();
  Members ms;
  for (auto& j : jobs) ms.push_back(j.c);
  std::vector<std::vector<double>> target(M);
  for (size_t m = 0; m < M; ++m) {
    target[m].resize(jobs[m].c->nrhs);
    for (int64_t i = 0; i < jobs[m].c->nrhs; ++i) target[m][i] = o.tol * o.tol * jobs[m].bb[i];
  }
  std::vector<int> ran;
  if (o.precision == ORI_FP64) {
    ORI_TRY(
        group_cocg(ms, PREC_F64, std::vector<int>(M, o.max_iter), o.check_every, o.graph != 0, cache[0], mc, &ran));
    for (auto& j : jobs) {
      for (int64_t i = 0; i < j.c->nrhs; ++i) {
        const ScalarBlock& s = j.c->sc_host[i];
        j.oc->info[i].iterations += s.iters;
        j.oc->info[i].matvecs += s.iters;
        j.oc->info[i].rel_res_recursive = j.bb[i] > 0 ? std::sqrt(s.rr / j.bb[i]) : 0.0;
        const bool conv = (s.flags & (FLAG_CONVERGED | FLAG_ZERO_RESIDUAL)) != 0;
        j.oc->state[i] = conv ? 0 : (s.flags & (FLAG_BREAKDOWN_RHO | FLAG_BREAKDOWN_MU)) ? 2 : 1;
      }
    }
    return ORI_OK;
  }
  // iterative refinement: FP64 true residual, complex64 inner COCG on the
  // normalised correction equation of every unconverged right-hand side;
  // a member leaves the loop when all its right-hand sides are done, its
  // inner iterations are spent, its inner solve made no progress or after
  // max_outer cycles
  ORI_TRY(sync_members(ms));
  std::vector<std::vector<int>> done(M);
  for (size_t m = 0; m < M; ++m) done[m].assign(jobs[m].c->nrhs, 0);
  std::vector<int> inner_left(M, o.max_iter);
  std::vector<bool> stopped(M, false);
  for (int outer = 0;; ++outer) {
    std::vector<size_t> act;
    for (size_t m = 0; m < M; ++m) {
      if (stopped[m]) continue;
      ori_ctx c = jobs[m].c;
      const int64_t R = c->nrhs;
      bool all = true;
      for (int64_t i = 0; i < R; ++i) {
        const ScalarBlock& s = c->sc_host[i];
        const double bbi = jobs[m].bb[i];
        jobs[m].oc->info[i].rel_res_recursive = bbi > 0 ? std::sqrt(s.rr / bbi) : 0.0;
        if (c->trace)
          std::fprintf(stderr, "[ori] refine %d rhs %lld fp64 rel %.6e\n", outer, (long long)i,
                       jobs[m].oc->info[i].rel_res_recursive);
        int& d = done[m][i];
        if (d == 0 && (s.rr <= target[m][i] || s.rr == 0.0)) d = 1;
        if (d == 0 && outer == 0 && (s.flags & FLAG_BREAKDOWN_RHO)) d = 2;
        c->outer_m_host[i] = d ? 0.0 : std::sqrt(s.rr);
        // inner tolerance: inner_tol, or looser when the outer tolerance
        // needs less (the correction reduces the residual by about the
        // inner tolerance; half of what is left is asked for)
        double t = o.inner_tol;
        if (!d && s.rr > 0.0) t = std::max(t, 0.5 * std::sqrt(target[m][i] / s.rr));
        c->outer_m_host[R + i] = std::min(t, 0.5) * std::min(t, 0.5);
        all = all && d;
      }
      if (all || outer >= o.max_outer || inner_left[m] <= 0)
        stopped[m] = true;
      else
        act.push_back(m);
    }
    if (act.empty()) break;
    Members am;
    std::vector<int> budget;
    for (size_t m : act) {
      ori_ctx c = jobs[m].c;
      const int64_t P = c->P, R = c->nrhs;
      ORI_HIP(c, hipMemcpyAsync(c->outer_m, c->outer_m_host, 2 * R * sizeof(double), hipMemcpyHostToDevice,
                                c->stream));
      ORI_TRY(launch(c, K_INIT, PREC_F32, [&] {
        return launch_init(PREC_F32, c->r, c->outer_m, c->xf, c->rf, P, R, c->partials, c->stream);
      }));
      ORI_TRY(finalize(c, rblocks(c), FIN_INIT, 0.0, 0, c->outer_m + R));
      am.push_back(c);
      budget.push_back(inner_left[m]);
    }
    ORI_TRY(group_cocg(am, PREC_F32, budget, o.check_every, o.graph != 0, cache[1], mc, &ran));
    for (size_t a = 0; a < act.size(); ++a) {
      const size_t m = act[a];
      ori_ctx c = jobs[m].c;
      const int64_t P = c->P, R = c->nrhs;
      inner_left[m] -= ran[a];
      bool progress = false;
      for (int64_t i = 0; i < R; ++i) {
        if (done[m][i]) continue;
        const ScalarBlock& s = c->sc_host[i];
        jobs[m].oc->info[i].iterations += s.iters;
        jobs[m].oc->info[i].matvecs += s.iters;
        jobs[m].oc->info[i].matvecs_c64 += s.iters;
        if (s.iters == 0 && (s.flags & (FLAG_BREAKDOWN_RHO | FLAG_BREAKDOWN_MU))) done[m][i] = 2;
        progress = progress || s.iters > 0;
      }
      ORI_TRY(launch(c, K_ELEMWISE, PREC_F32, [&] {
        return launch_axpy_batch(PREC_F32, c->outer_m, c->xf, c->x, P, R, c->stream);
      }));
      ORI_TRY(true_residual_sym(c, jobs[m].rhs, c->x, c->r, 0.0, 0));
      for (int64_t i = 0; i < R; ++i) {
        if (done[m][i]) continue;
        jobs[m].oc->info[i].matvecs++;
        jobs[m].oc->info[i].refinements++;
      }
      if (!progress) stopped[m] = true;
    }
    ORI_TRY(sync_members(am));
  }
  for (size_t m = 0; m < M; ++m)
    for (int64_t i = 0; i < jobs[m].c->nrhs; ++i)
      jobs[m].oc->state[i] = done[m][i] == 1 ? 0 : done[m][i] == 2 ? 2 : 1;
  return ORI_OK;
}

ori_status solve_sym(ori_ctx c, const ori_solve_opts& o, const cxd* rhs, const std::vector<double>& bb, Outcome* oc) {
  std::vector<SymJob> jobs{SymJob{c, rhs, bb, oc}};
  return solve_sym_group(jobs, o, c->graphs);
}

// Forward problem for every right-hand side of every context: w = S u
// (guess) or 0, solve (in lockstep), recover u (recover: w / S, or
// u0 - G0 S w), true residual.
ori_status forward_solve_group(const Members& ms, const ori_solve_opts& o, const std::vector<cxd*>& u,
                               std::vector<Outcome>* ocs, IterGraph* cache, MultiCache* mc = nullptr) {
  const double tol2 = o.tol * o.tol;
  ocs->resize(ms.size());
  std::vector<SymJob> jobs;
  for (size_t m = 0; m < ms.size(); ++m) {
    ori_ctx c = ms[m];
    const int64_t P = c->P, R = c->nrhs;
    Outcome* oc = &(*ocs)[m];
    oc->info.assign(R, ori_solve_info{});
    oc->state.assign(R, 1);
    if (o.use_x0) {
      ORI_TRY(launch(c, K_ELEMWISE, PREC_F64, [&] { return launch_mul(c->S, u[m], c->x, P, R, c->stream); }));
      ORI_TRY(true_residual_sym(c, c->b, c->x, c->r, tol2, 1));
      for (auto& i : oc->info) i.matvecs++;
    } else {
      ORI_TRY(launch(c, K_INIT, PREC_F64, [&] {
        return launch_init(PREC_F64, c->b, nullptr, c->x, c->r, P, R, c->partials, c->stream);
      }));
      ORI_TRY(finalize(c, rblocks(c), FIN_INIT, tol2, 1));
    }
    jobs.push_back(SymJob{c, c->b, c->bnorm2, oc});
  }
  ORI_TRY(solve_sym_group(jobs, o, cache, mc));
  // every member's recovery and true residual launched, then one wait per
  // stream
  // In mixed precision the refinement loop ends with r = b - (I + S G0 S) x
  // in FP64 for the final x = w (computed after the last correction, or r = b
  // for x = 0); with u = w / S that is r = S (u0 - u - G0 D u), so the
  // residual of eq. 2.19 is r / S and needs no product.
  std::vector<bool> from_r(ms.size(), false);
  for (size_t m = 0; m < ms.size(); ++m) {
    ori_ctx c = ms[m];
    Outcome* oc = &(*ocs)[m];
    for (auto& i : oc->info) i.rel_res_true = -1.0;
    from_r[m] = o.true_residual && o.precision == ORI_MIXED && c->recover_by_division;
    if (from_r[m]) {
      ORI_TRY(launch(c, K_ELEMWISE, PREC_F64, [&] {
        return launch_div_res(c->x, c->r, c->S, u[m], c->P, c->nrhs, c->partials, c->stream);
      }));
      ORI_TRY(finalize(c, rblocks(c), FIN_NORM));
      continue;
    }
    int rec = 0;
    ORI_TRY(recover(c, c->x, u[m], &rec));
    for (auto& i : oc->info) i.matvecs += rec;
    if (o.true_residual) ORI_TRY(true_residual_orig(c, u[m]));
  }
  if (!o.true_residual) return ORI_OK;
  ORI_TRY(sync_members(ms));
  for (size_t m = 0; m < ms.size(); ++m) {
    ori_ctx c = ms[m];
    const std::vector<double> rel = true_residual_orig_read(c);
    for (int64_t i = 0; i < c->nrhs; ++i) {
      if (!from_r[m]) (*ocs)[m].info[i].matvecs++;
      (*ocs)[m].info[i].rel_res_true = rel[i];
    }
  }
  return ORI_OK;
}

ori_status forward_solve(ori_ctx c, const ori_solve_opts& o, cxd* u, Outcome* oc) {
  std::vector<Outcome> ocs;
  ORI_TRY(forward_solve_group(Members{c}, o, std::vector<cxd*>{u}, &ocs, c->graphs));
  *oc = std::move(ocs[0]);
  return ORI_OK;
}

// Adjoint problem A^T lam = f with A^T = I + D G0 (one right-hand side),
// division free:
//   lam = f - S z,  (I + S G0 S) z = S G0 f,
//   G0 lam = G0 f - G0 S z,
//   g = -scale * c u (G0 lam),   c = 4 pi N |Delta|.
ori_status adjoint_solve(ori_ctx c, const ori_solve_opts& o, const cxd* u, const cxd* f, double scale, cxd* g,
                         cxd* lam, Outcome* oc) {
  const int64_t P = c->P;
  oc->info.assign(1, ori_solve_info{});
  oc->state.assign(1, 1);
  // t1 = G0 f
  ORI_TRY(matvec(c, PREC_F64, PREC_F64, plain_f1(f, nullptr),
                 epi(c->t1, nullptr, 0.0, nullptr, 0.0, nullptr, 1.0, nullptr, 0), nullptr));
  oc->info[0].matvecs++;
  // t2 = S t1 (right-hand side); x = 0, r = t2
  ORI_TRY(launch(c, K_ELEMWISE, PREC_F64, [&] { return launch_mul(c->S, c->t1, c->t2, P, 1, c->stream); }));
  ORI_TRY(launch(c, K_INIT, PREC_F64, [&] {
    return launch_init(PREC_F64, c->t2, nullptr, c->x, c->r, P, 1, c->partials, c->stream);
  }));
  ORI_TRY(finalize(c, rblocks(c), FIN_INIT, o.tol * o.tol, 0));
  ORI_TRY(sync_scalars(c));
  const std::vector<double> bb(1, c->sc_host[0].rr0);
  ORI_TRY(solve_sym(c, o, c->t2, bb, oc));
  // q = G0 lam = t1 - G0 S z.  In mixed precision the refinement loop ends
  // with r = t2 - (I + S G0 S) z in FP64, and t2 = S t1, so with no S_p
  // small G0 S z = t1 - (z + r) / S and q = (z + r) / S (to rounding)
  // without a product.
  if (o.precision == ORI_MIXED && c->recover_by_division) {
    ORI_TRY(launch(c, K_ELEMWISE, PREC_F64,
                   [&] { return launch_add_div(c->x, c->r, c->S, c->q, P, c->stream); }));
  } else {
    ORI_TRY(matvec(c, PREC_F64, PREC_F64, plain_f1(c->x, c->S),
                   epi(c->q, c->t1, 1.0, nullptr, 0.0, nullptr, -1.0, nullptr, 0), nullptr));
    oc->info[0].matvecs++;
  }
  if (g)
    ORI_TRY(launch(c, K_ELEMWISE, PREC_F64,
                   [&] { return launch_gradient(c->cN, u, c->q, -scale, g, P, c->stream); }));
  if (lam)
    ORI_TRY(launch(c, K_ELEMWISE, PREC_F64, [&] { return launch_sub_mul(f, c->S, c->x, lam, P, c->stream); }));
  return ORI_OK;
}

double elapsed(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

ori_status field_sum(ori_ctx c, const void* u, const double* pts, int64_t M, void* out, bool far) {
  ORI_TRY(guard(c));
  if (!c->loaded) return set_err(c, ORI_ERR_INVALID_ARG, "ori_load has not succeeded on this context");
  if (M < 0) return set_err(c, ORI_ERR_INVALID_ARG, "M = %lld must be >= 0", (long long)M);
  if (M == 0) return ORI_OK;
  ORI_TRY(check_dev_ptr(c, u, c->nrhs * c->P * 16, "u"));
  ORI_TRY(check_dev_ptr(c, pts, M * 3 * 8, far ? "beta" : "x", 8));
  ORI_TRY(check_dev_ptr(c, out, c->nrhs * M * 16, far ? "A" : "v"));
  FieldArgs a{};
  a.u = static_cast<const cxd*>(u);
  a.D = c->D;
  a.pts = pts;
  a.part = c->t1;  // P complex values of scratch
  a.out = static_cast<cxd*>(out);
  a.n = c->n;
  a.P = c->P;
  a.M = M;
  a.nrhs = c->nrhs;
  a.chunk = int64_t{1} << 16;
  a.nchunk = (c->P + a.chunk - 1) / a.chunk;
  a.dn = static_cast<double>(c->n);
  a.side = c->grid.side;
  a.offset = c->grid.cell_offset;
  a.k = c->k;
  for (int d = 0; d < 3; ++d) a.origin[d] = c->grid.origin[d];
  // points per launch: the partials [nrhs][mb][nchunk] fit the P-value scratch
  int64_t mb = c->P / (c->nrhs * a.nchunk);
  if (mb < 1) mb = 1;
  if (mb > 65535) mb = 65535;
  for (int64_t m0 = 0; m0 < M; m0 += mb) {
    a.m0 = m0;
    a.mb = std::min(mb, M - m0);
    if (c->nrhs * a.mb * a.nchunk > c->P) return set_err(c, ORI_ERR_UNSUPPORTED, "field scratch too small");
    ORI_TRY(launch(c, K_ELEMWISE, PREC_F64, [&] { return launch_field(a, far, c->stream); }));
  }
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  return ORI_OK;
}

ori_status refraction(ori_ctx c, double k, double c_s, const void* n0, const void* in, const double* N, void* out,
                      bool design) {
  ORI_TRY(guard(c));
  if (!(k > 0.0) || !std::isfinite(k)) return set_err(c, ORI_ERR_INVALID_ARG, "k must be finite and > 0");
  if (!(c_s > 0.0) || !std::isfinite(c_s)) return set_err(c, ORI_ERR_INVALID_ARG, "c_S must be finite and > 0");
  const int64_t bytes = c->P * 16;
  ORI_TRY(check_dev_ptr(c, n0, bytes, "n0"));
  ORI_TRY(check_dev_ptr(c, in, bytes, design ? "n" : "h"));
  if (N) ORI_TRY(check_dev_ptr(c, N, c->P * 8, "N", 8));
  ORI_TRY(check_dev_ptr(c, out, bytes, design ? "h" : "n"));
  RefractionArgs a{};
  a.n0 = static_cast<const cxd*>(n0);
  a.in = static_cast<const cxd*>(in);
  a.N = N;
  a.out = static_cast<cxd*>(out);
  a.bad = c->partials;
  a.P = c->P;
  a.k = k;
  a.c_s = c_s;
  a.design = design ? 1 : 0;
  ORI_TRY(launch(c, K_ELEMWISE, PREC_F64, [&] { return launch_refraction(a, c->stream); }));
  const int64_t nb = refraction_blocks(c->P);
  std::vector<double> bad(nb);
  ORI_HIP(c, hipMemcpyAsync(bad.data(), c->partials, nb * 8, hipMemcpyDeviceToHost, c->stream));
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  double nbad = 0.0;
  for (double b : bad) nbad += b;
  if (nbad > 0.0)
    return set_err(c, ORI_ERR_INVALID_ARG, "%.0f entries hold NaN/Inf or N %s 0 (their output is 0)", nbad,
                   design ? "<=" : "<");
  return ORI_OK;
}
// ---------------------------------------------------------------------------
// The Green's product without allocation (ori_green_noalloc): every
// workspace of the product -- the work arrays, the spectrum octant and the
// twiddle tables -- is a slice of one static device array.
// ---------------------------------------------------------------------------
constexpr int64_t kStaticBytes = int64_t{32} << 20;  // 32 MiB per device
constexpr int kMaxStaticDevices = 64;

struct StaticLayout {
  int64_t arena, kh, khf, twd, twf, total;
};

// The context layout_for gives one right-hand side, restricted to what the
// product needs: the arena (A and B, also the spectrum passes' octant
// scratch), the octant and its complex64 copy, and the two twiddle tables.
StaticLayout static_layout(int64_t n, int64_t L, bool mixed) {
  const int64_t kp = L / 2 + 1;
  StaticLayout s{};
  s.arena = 0;
  s.kh = align_up(std::max<int64_t>(n * n * L + n * L * L, kp * kp * kp) * 16);
  s.khf = s.kh + align_up(kp * kp * kp * 16);
  s.twd = s.khf + (mixed ? align_up(kp * kp * kp * 8) : 0);
  s.twf = s.twd + align_up(L * 16);
  s.total = s.twf + align_up(L * 8);
  return s;
}

std::mutex g_static_mu;
void* g_static_ptr[kMaxStaticDevices] = {};

}  // namespace

// The array itself.  In host code its name is only a stand-in: kernels get
// the device address that hipGetSymbolAddress returns for the current
// device, kept per device in g_static_ptr.
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

// Device address of the static array on device dev (looked up once per
// device, with that device current).
ori_status static_workspace(int dev, void** out) {
  if (dev < 0 || dev >= kMaxStaticDevices)
    return set_err(nullptr, ORI_ERR_UNSUPPORTED, "device %d: the static workspace covers devices 0..%d", dev,
                   kMaxStaticDevices - 1);
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_err(nullptr, ORI_ERR_DEVICE, "hipGetSymbolAddress of the static workspace failed: %s",
                     hipGetErrorString(e));
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return ORI_OK;
}

}  // namespace

// A group of independent problems solved together (ori_group_*).  Each
// member context has a stream of its own, so the members' eager launches run
// side by side; their COCG iteration blocks replay one graph with a chain
// per member.  Group calls start after the work already queued on the
// caller's stream (an event) and return after all of theirs is done.
struct ori_group_s {
  int device = 0;
  std::vector<ori_ctx> members;
  std::vector<hipStream_t> streams;  // one per member, owned by the group (stream_pool)
  hipStream_t caller = nullptr;
  hipEvent_t ready = nullptr;
  IterGraph graphs[2];  // per vector precision
  MultiCache multi;     // tables of the one-launch-per-kernel iterations
};

namespace {
// order member m's stream after the work queued on the caller's stream
ori_status group_wait_caller(ori_group g, size_t m) {
  ori_ctx c = g->members[m];
  ORI_HIP(c, hipEventRecord(g->ready, g->caller));
  ORI_HIP(c, hipStreamWaitEvent(c->stream, g->ready, 0));
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
  o->graph = 1;
  o->multi = 1;
}

const char* ori_version(void) { return "ori 0.2 (gfx950)"; }

ori_status ori_workspace_bytes(const ori_grid* g, int32_t nrhs, int32_t provision, int64_t* bytes) {
  int64_t L = 0;
  ORI_TRY(check_grid(g, &L));
  if (nrhs < 1 || nrhs > kMaxRhs) return set_err(nullptr, ORI_ERR_INVALID_ARG, "nrhs = %d out of [1, %lld]", nrhs,
                                                  (long long)kMaxRhs);
  if (!bytes) return set_err(nullptr, ORI_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = layout_for(g->n, nrhs, provision | ORI_PROVISION_FP64).total;
  return ORI_OK;
}

ori_status ori_create(const ori_grid* g, int32_t nrhs, int32_t provision, int64_t mem_limit_bytes, void* stream,
                      ori_ctx* out) {
  if (!out) return set_err(nullptr, ORI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int64_t L = 0;
  ORI_TRY(check_grid(g, &L));
  if (nrhs < 1 || nrhs > kMaxRhs)
    return set_err(nullptr, ORI_ERR_INVALID_ARG, "nrhs = %d out of [1, %lld]", nrhs, (long long)kMaxRhs);
  provision |= ORI_PROVISION_FP64;
  const Layout lay = layout_for(g->n, nrhs, provision);
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
  c->nrhs = nrhs;
  c->provision = provision;
  c->K = K;
  c->u0norm2.assign(nrhs, 0.0);
  c->bnorm2.assign(nrhs, 0.0);
  choose_layout(c);
  if (const char* e = std::getenv("ORI_CHECK_GUARDS")) c->check_guards = std::atoi(e) != 0;
  if (const char* e = std::getenv("ORI_TRACE")) c->trace = std::atoi(e) != 0;
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
  const bool mixed = provision & ORI_PROVISION_MIXED;
  const int64_t R = nrhs;
  // The workspaces, in order, carved from one block: each starts on a
  // 256-byte boundary and is followed by its guard band.  carve(take) calls
  // take(bytes, pointer) for every workspace; a first pass sums the sizes.
  auto carve = [&](auto&& take) {
    take(lay.arena, c->arena);
    take(lay.vec_d, c->D);
    take(lay.vec_d, c->S);
    take(lay.vec_f, c->cN);
    take(lay.vec_d, c->t1);
    take(lay.vec_d, c->t2);
    take(R * lay.vec_d, c->b);
    take(R * lay.vec_d, c->u0);
    take(R * lay.vec_d, c->x);
    take(R * lay.vec_d, c->r);
    take(R * lay.vec_d, c->p);
    take(R * lay.vec_d, c->q);
    if (mixed) {
      take(lay.vec_f, c->Sf);
      take(R * lay.vec_f, c->xf);
      take(R * lay.vec_f, c->rf);
      take(R * lay.vec_f, c->pf);
      take(R * lay.vec_f, c->qf);
      take(lay.khf, c->khf);
    }
    take(lay.kh, c->kh);
    take(align_up(lay.npart * 4 * 8), c->partials);
    take(align_up(R * (int64_t)sizeof(ScalarBlock)), c->sc);
    take(align_up(2 * R * 8), c->outer_m);
  };
  int64_t total = 0;
  carve([&](int64_t bytes, auto&) {
    if (bytes > 0) total = align_up(total + bytes + kGuardBytes);
  });
  if (total != lay.total) {  // layout_for and the list above describe the same block
    set_err(c, ORI_ERR_DEVICE, "internal: workspace of %lld bytes, layout says %lld", (long long)total,
            (long long)lay.total);
    return fail(ORI_ERR_DEVICE);
  }
  {
    const hipError_t e = pool_malloc(c->device, static_cast<size_t>(total), &c->ws_block);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_err(c, ORI_ERR_OUT_OF_MEMORY, "hipMalloc(%lld) failed: %s", (long long)total, hipGetErrorString(e));
      return fail(ORI_ERR_OUT_OF_MEMORY);
    }
    c->ws_bytes = static_cast<size_t>(total);
  }
  int64_t at = 0;
  unsigned char* base = static_cast<unsigned char*>(c->ws_block);
  carve([&](int64_t bytes, auto& dst) {
    using Ptr = std::remove_reference_t<decltype(dst)>;
    if (bytes <= 0) {
      dst = nullptr;
      return;
    }
    dst = static_cast<Ptr>(static_cast<void*>(base + at));
    c->guards.push_back(base + at + bytes);
    at = align_up(at + bytes + kGuardBytes);
  });
  // the guard bands, one launch on the context's stream (ori_check_guards
  // waits for it)
  {
    GuardBands gb{};
    gb.base = c->ws_block;
    gb.count = static_cast<int32_t>(c->guards.size());
    gb.v = kGuardByte;
    for (size_t i = 0; i < c->guards.size() && i < kMaxGuardBands; ++i) gb.off[i] = c->guards[i] - base;
    if (c->guards.size() > kMaxGuardBands || launch_fill_guards(gb, c->stream) != hipSuccess) {
      set_err(c, ORI_ERR_DEVICE, "setting the guard bands failed");
      return fail(ORI_ERR_DEVICE);
    }
  }
  // the pinned mirrors of sc and outer_m, one block
  const size_t sc_bytes = static_cast<size_t>(align_up(R * (int64_t)sizeof(ScalarBlock)));
  if (pool_host_malloc(sc_bytes + 2 * R * sizeof(double), &c->pin_block) != hipSuccess) {
    (void)hipGetLastError();
    set_err(c, ORI_ERR_OUT_OF_MEMORY, "hipHostMalloc of the scalar mirrors failed");
    return fail(ORI_ERR_OUT_OF_MEMORY);
  }
  c->pin_bytes = sc_bytes + 2 * R * sizeof(double);
  c->sc_host = static_cast<ScalarBlock*>(c->pin_block);
  c->outer_m_host = reinterpret_cast<double*>(static_cast<unsigned char*>(c->pin_block) + sc_bytes);
  std::memset(c->sc_host, 0, R * sizeof(ScalarBlock));
  {
    const ori_status ts = shared_twiddles(c->device, L, &c->twd, &c->twf);
    if (ts != ORI_OK) {
      set_err(c, ts, "%s", g_last_error.c_str());
      return fail(ts);
    }
  }
  if (hipMemsetAsync(c->sc, 0, R * sizeof(ScalarBlock), c->stream) != hipSuccess) {
    set_err(c, ORI_ERR_DEVICE, "clearing the scalar blocks failed");
    return fail(ORI_ERR_DEVICE);
  }
  *out = c;
  return ORI_OK;
}

namespace {
// ori_load in two halves: the checks of the arguments and every launch
// (load_launch), then one wait for the context's stream and the checks of
// the data (load_finish).  Several contexts can be loaded with their waits
// overlapping (ori_group_load_all).
ori_status load_launch(ori_ctx c, double k, const void* h, const double* N, const void* u0) {
  if (!(k > 0.0) || !std::isfinite(k)) return set_err(c, ORI_ERR_INVALID_ARG, "k must be finite and > 0");
  const int64_t P = c->P, R = c->nrhs;
  ORI_TRY(check_dev_ptr(c, h, P * 16, "h"));
  if (N) ORI_TRY(check_dev_ptr(c, N, P * 8, "N", 8));
  ORI_TRY(check_dev_ptr(c, u0, R * P * 16, "u0"));
  c->loaded = false;
  c->k = k;
  if (!(c->spectrum_cache && c->spectrum_valid && c->spectrum_k == k)) {
    c->spectrum_valid = false;
    ORI_TRY(compute_spectrum(c));
    c->spectrum_valid = true;
    c->spectrum_k = k;
  }
  const double vol = std::pow(c->grid.side / static_cast<double>(c->n), 3);
  // operator coefficients: the bad-input count lands in sc[0]
  ORI_TRY(launch(c, K_COEFF, PREC_F64, [&] {
    return launch_coefficients(h, N, vol, P, c->D, c->S, c->Sf, c->cN, c->partials, c->stream);
  }));
  ORI_HIP(c, hipMemsetAsync(c->sc, 0, R * sizeof(ScalarBlock), c->stream));
  ORI_TRY(launch(c, K_FINALIZE, PREC_F64,
                 [&] { return launch_finalize_coeff(c->partials, rblocks(c), c->sc, c->stream); }));
  // right-hand sides b = S u0 and their norms; the coefficient check stays
  // in sc[0] (FLAG_BAD_COEFF, |S|^2 range), so one wait covers both
  ORI_TRY(launch(c, K_COEFF, PREC_F64, [&] { return launch_rhs(u0, c->S, P, R, c->b, c->u0, c->partials, c->stream); }));
  return finalize(c, rblocks(c), FIN_SETUP);
}

ori_status load_finish(ori_ctx c) {
  const int64_t R = c->nrhs;
  ORI_TRY(sync_scalars(c));
  if (c->sc_host[0].flags & FLAG_BAD_COEFF) return set_err(c, ORI_ERR_INVALID_ARG, "h or N holds NaN/Inf, or N < 0");
  // u = w / S is exact and free when no S_p vanishes; with |S| spread over
  // more than 1e3 the division would amplify the error of w in small-S
  // cells, so the recovery u = u0 - G0 S w (one product) is used instead
  c->recover_by_division = c->sc_host[0].s2_min > 0.0 && c->sc_host[0].s2_min >= 1e-6 * c->sc_host[0].s2_max;
  for (int64_t i = 0; i < R; ++i) {
    if (c->sc_host[i].flags & FLAG_BAD_INPUT)
      return set_err(c, ORI_ERR_INVALID_ARG, "u0 (right-hand side %lld) holds NaN/Inf", (long long)i);
    c->bnorm2[i] = c->sc_host[i].bb;
    c->u0norm2[i] = c->sc_host[i].aux;
  }
  c->loaded = true;
  return ORI_OK;
}
}  // namespace

ori_status ori_load(ori_ctx c, double k, const void* h, const double* N, const void* u0) {
  ORI_TRY(guard(c));
  ORI_TRY(load_launch(c, k, h, N, u0));
  return load_finish(c);
}

ori_status ori_spectrum_cache(ori_ctx c, int32_t enable) {
  ORI_TRY(guard(c));
  c->spectrum_cache = enable != 0;
  if (!c->spectrum_cache) c->spectrum_valid = false;
  return ORI_OK;
}

ori_status ori_setup(const ori_grid* g, double k, const void* h, const double* N, const void* u0, void* stream,
                     ori_ctx* out) {
  ORI_TRY(ori_create(g, 1, ORI_PROVISION_FP64 | ORI_PROVISION_MIXED, 0, stream, out));
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
  ORI_TRY(check_dev_ptr(c, x, c->nrhs * c->P * 16, "x"));
  ORI_TRY(check_dev_ptr(c, y, c->nrhs * c->P * 16, "y"));
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

// ---------------------------------------------------------------------------
// physics of the solution: charges, field, far field, refraction recipe
// ---------------------------------------------------------------------------
ori_status ori_charges(ori_ctx c, const void* u, void* q) {
  ORI_TRY(guard(c));
  if (!c->loaded) return set_err(c, ORI_ERR_INVALID_ARG, "ori_load has not succeeded on this context");
  const int64_t bytes = c->nrhs * c->P * 16;
  ORI_TRY(check_dev_ptr(c, u, bytes, "u"));
  ORI_TRY(check_dev_ptr(c, q, bytes, "q"));
  ORI_TRY(launch(c, K_ELEMWISE, PREC_F64, [&] { return launch_charges(c->D, u, c->P, c->nrhs, q, c->stream); }));
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  return ORI_OK;
}

ori_status ori_scattered_field(ori_ctx c, const void* u, const double* x, int64_t M, void* v) {
  return field_sum(c, u, x, M, v, false);
}

ori_status ori_far_field(ori_ctx c, const void* u, const double* beta, int64_t M, void* A) {
  return field_sum(c, u, beta, M, A, true);
}

ori_status ori_refraction_index(ori_ctx c, double k, double c_s, const void* n0, const void* h, const double* N,
                                void* n) {
  return refraction(c, k, c_s, n0, h, N, n, false);
}

ori_status ori_design_impedance(ori_ctx c, double k, double c_s, const void* n0, const void* n, const double* N,
                                void* h) {
  return refraction(c, k, c_s, n0, n, N, h, true);
}

ori_status ori_interpolation_difference(ori_ctx c, const void* y, const void* x_fine, int64_t n_fine,
                                       double fine_offset, double* diff) {
  ORI_TRY(guard(c));
  if (!diff) return set_err(c, ORI_ERR_INVALID_ARG, "diff is NULL");
  if (n_fine < 1 || n_fine > 4096) return set_err(c, ORI_ERR_INVALID_ARG, "n_fine = %lld out of range", (long long)n_fine);
  if (!std::isfinite(fine_offset) || fine_offset < 0.0 || fine_offset >= 1.0)
    return set_err(c, ORI_ERR_INVALID_ARG, "fine_offset must lie in [0, 1)");
  ORI_TRY(check_dev_ptr(c, y, c->P * 16, "y"));
  ORI_TRY(check_dev_ptr(c, x_fine, n_fine * n_fine * n_fine * 16, "x_fine"));
  DiffArgs a{};
  a.x = static_cast<const cxd*>(x_fine);
  a.y = static_cast<const cxd*>(y);
  a.means = reinterpret_cast<double*>(c->t1);  // P doubles of scratch
  a.nf = n_fine;
  a.nc = c->n;
  a.off = fine_offset;
  ORI_TRY(launch(c, K_ELEMWISE, PREC_F64,
                 [&] { return launch_cell_difference(a, c->P, c->partials, c->stream); }));
  const int64_t nb = max_blocks(c->P);
  std::vector<double> part(nb);
  ORI_HIP(c, hipMemcpyAsync(part.data(), c->partials, nb * 8, hipMemcpyDeviceToHost, c->stream));
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  double m = -1.0;
  for (double v : part) m = std::max(m, v);
  *diff = m;
  return ORI_OK;
}

ori_status ori_green_noalloc(const ori_grid* g, double k, int32_t precision, const void* x, void* y, void* stream) {
  int64_t L = 0;
  ORI_TRY(check_grid(g, &L));
  if (!(k > 0.0) || !std::isfinite(k)) return set_err(nullptr, ORI_ERR_INVALID_ARG, "k must be finite and > 0");
  if (precision != ORI_FP64 && precision != ORI_MIXED) return set_err(nullptr, ORI_ERR_INVALID_ARG, "bad precision");
  const bool mixed = precision == ORI_MIXED;
  const StaticLayout sl = static_layout(g->n, L, mixed);
  if (sl.total > kStaticBytes)
    return set_err(nullptr, ORI_ERR_UNSUPPORTED,
                   "n = %lld needs %lld bytes of workspace; the static workspace holds %lld (n <= 64)",
                   (long long)g->n, (long long)sl.total, (long long)kStaticBytes);
  const LengthKernels* K = kernels_for_length(static_cast<int>(L));
  if (!K) return set_err(nullptr, ORI_ERR_UNSUPPORTED, "no kernels for padded length %lld", (long long)L);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_err(nullptr, ORI_ERR_DEVICE, "hipGetDevice failed (no GPU?)");
  void* base = nullptr;
  ORI_TRY(static_workspace(dev, &base));
  // A context on the stack that owns nothing: its workspaces are slices of
  // the static array, and it is never destroyed through ori_destroy.
  ori_ctx_s c;
  c.grid = *g;
  c.n = g->n;
  c.L = L;
  c.P = g->n * g->n * g->n;
  c.nrhs = 1;
  c.provision = ORI_PROVISION_FP64 | (mixed ? ORI_PROVISION_MIXED : 0);
  c.k = k;
  c.device = dev;
  c.K = K;
  c.stream = static_cast<hipStream_t>(stream);
  choose_layout(&c);
  char* b = static_cast<char*>(base);
  c.arena = b + sl.arena;
  c.kh = reinterpret_cast<cxd*>(b + sl.kh);
  c.khf = mixed ? reinterpret_cast<cxf*>(b + sl.khf) : nullptr;
  c.twd = reinterpret_cast<cxd*>(b + sl.twd);
  c.twf = reinterpret_cast<cxf*>(b + sl.twf);
  ori_status st = check_dev_ptr(&c, x, c.P * 16, "x");
  if (st == ORI_OK) st = check_dev_ptr(&c, y, c.P * 16, "y");
  if (st == ORI_OK)
    st = launch(&c, K_ELEMWISE, PREC_F64, [&] { return launch_twiddles(L, c.twd, c.twf, c.stream); });
  if (st == ORI_OK) st = compute_spectrum(&c);
  if (st == ORI_OK)
    st = matvec(&c, PREC_F64, mixed ? PREC_F32 : PREC_F64, plain_f1(x, nullptr),
                epi(y, nullptr, 0.0, nullptr, 0.0, nullptr, 1.0, nullptr, 0), nullptr);
  if (st != ORI_OK) g_last_error = c.err;
  return st;
}

ori_status ori_get_layout(ori_ctx c, int32_t precision, ori_layout* out) {
  ORI_TRY(guard(c));
  if (!out) return set_err(c, ORI_ERR_INVALID_ARG, "out is NULL");
  if (precision != ORI_FP64 && precision != ORI_MIXED) return set_err(c, ORI_ERR_INVALID_ARG, "bad precision");
  const Knobs& k = c->knob[precision == ORI_MIXED ? 1 : 0];
  *out = ori_layout{k.blk_lg, k.np_sel, k.zpf, k.z_np, k.zplan};
  return ORI_OK;
}

ori_status ori_set_layout(ori_ctx c, int32_t precision, const ori_layout* in) {
  ORI_TRY(guard(c));
  if (!in) return set_err(c, ORI_ERR_INVALID_ARG, "layout is NULL");
  if (precision != ORI_FP64 && precision != ORI_MIXED) return set_err(c, ORI_ERR_INVALID_ARG, "bad precision");
  const Knobs k{in->blk_lg, in->narrow, in->prefetch, in->znarrow, in->zplan};
  if (!valid_knobs(c->n, c->L, k))
    return set_err(c, ORI_ERR_INVALID_ARG,
                   "layout {blk_lg %d, narrow %d, prefetch %d, znarrow %d, zplan %d} is not valid for n = %lld "
                   "(padded length %lld%s)",
                   in->blk_lg, in->narrow, in->prefetch, in->znarrow, in->zplan, (long long)c->n, (long long)c->L,
                   has_plan_variant(static_cast<int>(c->L)) ? "" : ", one radix plan");
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  ORI_TRY(drop_graphs(c));
  c->knob[precision == ORI_MIXED ? 1 : 0] = k;
  return ORI_OK;
}

ori_status ori_tune(ori_ctx c, int32_t reps, ori_layout* best, double* ms_per_product) {
  ORI_TRY(guard(c));
  if (!c->loaded) return set_err(c, ORI_ERR_INVALID_ARG, "ori_load has not succeeded on this context");
  if (reps < 0) return set_err(c, ORI_ERR_INVALID_ARG, "reps must be >= 0");
  if (reps == 0) reps = 3;
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  ORI_TRY(drop_graphs(c));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ORI_HIP(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_err(c, ORI_ERR_DEVICE, "hipEventCreate failed");
  }
  ori_status st = ORI_OK;
  Tuned found;
  const bool mixed = c->provision & ORI_PROVISION_MIXED;
  for (int f = 0; f < (mixed ? 2 : 1) && st == ORI_OK; ++f) {
    // the COCG product of this precision: q = (I + S G0 S) x on the batch
    const int fp = f ? PREC_F32 : PREC_F64;
    void* x = f ? static_cast<void*>(c->xf) : static_cast<void*>(c->x);
    void* y = f ? static_cast<void*>(c->qf) : static_cast<void*>(c->q);
    const void* S = f ? static_cast<const void*>(c->Sf) : static_cast<const void*>(c->S);
    if (f) {
      ORI_HIP(c, hipMemsetAsync(x, 0, c->nrhs * c->P * 8, c->stream));
    } else {
      ORI_HIP(c, hipMemcpyAsync(x, c->b, c->nrhs * c->P * 16, hipMemcpyDeviceToDevice, c->stream));
    }
    const Knobs start = c->knob[f];
    Knobs win = start;
    double win_ms = INFINITY;
    for (int lg = 0; lg <= 6 && st == ORI_OK; ++lg)
      for (int np = 0; np <= 1 && st == ORI_OK; ++np)
        for (int pf = 0; pf <= 1 && st == ORI_OK; ++pf)
          for (int znp = 0; znp <= 1 && st == ORI_OK; ++znp)
            for (int zp = 0; zp <= 1 && st == ORI_OK; ++zp) {
            const Knobs k{lg, np, pf, znp, zp};
            if (!valid_knobs(c->n, c->L, k)) continue;
            c->knob[f] = k;
            auto product = [&] {
              return matvec(c, fp, fp, plain_f1(x, S), epi(y, x, 1.0, nullptr, 0.0, S, 1.0, nullptr, 0), nullptr);
            };
            st = product();  // warm-up
            if (st == ORI_OK && hipEventRecord(e0, c->stream) != hipSuccess)
              st = set_err(c, ORI_ERR_DEVICE, "hipEventRecord failed");
            for (int i = 0; i < reps && st == ORI_OK; ++i) st = product();
            if (st == ORI_OK && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
              st = set_err(c, ORI_ERR_DEVICE, "timing events failed");
            float ms = 0.f;
            if (st == ORI_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
              st = set_err(c, ORI_ERR_DEVICE, "hipEventElapsedTime failed");
            if (st == ORI_OK && ms / reps < win_ms) {
              win_ms = ms / reps;
              win = k;
            }
          }
    c->knob[f] = st == ORI_OK ? win : start;
    found.k[f] = win;
    found.have[f] = st == ORI_OK;
    if (best) best[f] = ori_layout{win.blk_lg, win.np_sel, win.zpf, win.z_np, win.zplan};
    if (ms_per_product) ms_per_product[f] = st == ORI_OK ? win_ms : -1.0;
  }
  if (!mixed) {
    if (best) best[1] = ori_layout{c->knob[1].blk_lg, c->knob[1].np_sel, c->knob[1].zpf, c->knob[1].z_np,
                                   c->knob[1].zplan};
    if (ms_per_product) ms_per_product[1] = -1.0;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ORI_OK) return st;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  Tuned& t = g_tuned[TuneKey{c->device, c->n, c->nrhs}];
  for (int f = 0; f < 2; ++f)
    if (found.have[f]) {
      t.k[f] = found.k[f];
      t.have[f] = true;
    }
  return ORI_OK;
}

ori_status ori_solve(ori_ctx c, const ori_solve_opts* opts_in, void* u_out, ori_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  ORI_TRY(guard(c));
  ori_solve_opts o;
  ORI_TRY(check_opts(c, opts_in, &o));
  ORI_TRY(check_dev_ptr(c, u_out, c->nrhs * c->P * 16, "u"));
  Outcome oc;
  ORI_TRY(forward_solve(c, o, static_cast<cxd*>(u_out), &oc));
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  const double secs = elapsed(t0);
  for (auto& i : oc.info) i.seconds = secs;
  c->last_info = oc.info;
  if (info) {
    *info = aggregate(oc);
    info->seconds = secs;
  }
  return end_status(c, oc, "COCG");
}

ori_status ori_group_create(const ori_grid* grids, int32_t nprob, int32_t provision, void* stream, ori_group* out) {
  if (!out) return set_err(nullptr, ORI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!grids) return set_err(nullptr, ORI_ERR_INVALID_ARG, "grids is NULL");
  if (nprob < 1 || nprob > kGroupMaxProblems)
    return set_err(nullptr, ORI_ERR_INVALID_ARG, "nprob = %d out of [1, %d]", nprob, kGroupMaxProblems);
  ori_group g = new ori_group_s();
  g->multi.graphs = g->graphs;
  g->caller = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&g->device) != hipSuccess || hipEventCreateWithFlags(&g->ready, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    g->ready = nullptr;
    ori_group_destroy(g);
    return set_err(nullptr, ORI_ERR_DEVICE, "hipEventCreate failed (no GPU?)");
  }
  for (int32_t i = 0; i < nprob; ++i) {
    hipStream_t sm = nullptr;
    if (pool_stream(g->device, &sm) != hipSuccess) {
      (void)hipGetLastError();
      ori_group_destroy(g);
      return set_err(nullptr, ORI_ERR_DEVICE, "problem %d: hipStreamCreate failed", i);
    }
    g->streams.push_back(sm);
    ori_ctx c = nullptr;
    const ori_status st = ori_create(&grids[i], 1, provision, 0, sm, &c);
    if (st != ORI_OK) {
      const std::string msg = g_last_error;
      ori_group_destroy(g);
      return set_err(nullptr, st, "problem %d: %s", i, msg.c_str());
    }
    g->members.push_back(c);
  }
  *out = g;
  return ORI_OK;
}

ori_status ori_group_load(ori_group g, int32_t i, double k, const void* h, const double* N, const void* u0) {
  if (!g) return set_err(nullptr, ORI_ERR_INVALID_ARG, "group is NULL");
  if (i < 0 || i >= static_cast<int32_t>(g->members.size()))
    return set_err(nullptr, ORI_ERR_INVALID_ARG, "problem %d out of [0, %zu)", i, g->members.size());
  ori_ctx c = g->members[i];
  ori_status st = guard(c);
  if (st == ORI_OK) st = group_wait_caller(g, i);
  if (st == ORI_OK) st = ori_load(c, k, h, N, u0);
  if (st != ORI_OK) set_err(nullptr, st, "problem %d: %s", i, c->err.c_str());
  return st;
}

ori_status ori_group_load_all(ori_group g, const double* k, const void* const* h, const double* const* N,
                              const void* const* u0) {
  if (!g) return set_err(nullptr, ORI_ERR_INVALID_ARG, "group is NULL");
  if (!k || !h || !u0) return set_err(nullptr, ORI_ERR_INVALID_ARG, "k, h and u0 must not be NULL");
  const size_t M = g->members.size();
  // every problem's launches first, then the waits: the problems' loads run
  // side by side on their streams
  for (size_t m = 0; m < M; ++m) {
    ori_ctx c = g->members[m];
    ori_status st = guard(c);
    if (st == ORI_OK) st = group_wait_caller(g, m);
    if (st == ORI_OK) st = load_launch(c, k[m], h[m], N ? N[m] : nullptr, u0[m]);
    if (st != ORI_OK) return set_err(nullptr, st, "problem %zu: %s", m, c->err.c_str());
  }
  for (size_t m = 0; m < M; ++m) {
    ori_ctx c = g->members[m];
    const ori_status st = load_finish(c);
    if (st != ORI_OK) return set_err(nullptr, st, "problem %zu: %s", m, c->err.c_str());
  }
  return ORI_OK;
}

ori_status ori_group_solve(ori_group g, const ori_solve_opts* opts_in, void* const* u, ori_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!g) return set_err(nullptr, ORI_ERR_INVALID_ARG, "group is NULL");
  if (!u) return set_err(nullptr, ORI_ERR_INVALID_ARG, "u is NULL");
  const size_t M = g->members.size();
  ori_solve_opts o{};
  std::vector<cxd*> us(M);
  for (size_t m = 0; m < M; ++m) {
    ori_ctx c = g->members[m];
    ori_status st = guard(c);
    if (st == ORI_OK) st = check_opts(c, opts_in, &o);
    if (st == ORI_OK) st = check_dev_ptr(c, u[m], c->nrhs * c->P * 16, "u");
    if (st == ORI_OK) st = group_wait_caller(g, m);
    if (st != ORI_OK) return set_err(nullptr, st, "problem %zu: %s", m, c->err.c_str());
    us[m] = static_cast<cxd*>(u[m]);
  }
  std::vector<Outcome> ocs;
  ori_status st = forward_solve_group(g->members, o, us, &ocs, g->graphs, o.multi ? &g->multi : nullptr);
  for (size_t m = 0; m < M && st == ORI_OK; ++m) {
    ori_ctx c = g->members[m];
    if (hipStreamSynchronize(c->stream) != hipSuccess) st = set_err(c, ORI_ERR_DEVICE, "hipStreamSynchronize failed");
  }
  if (st != ORI_OK) {
    for (ori_ctx c : g->members)
      if (c->err != "no error") return set_err(nullptr, st, "%s", c->err.c_str());
    return st;
  }
  const double secs = elapsed(t0);
  ori_status worst = ORI_OK;
  for (size_t m = 0; m < M; ++m) {
    ori_ctx c = g->members[m];
    for (auto& i : ocs[m].info) i.seconds = secs;
    c->last_info = ocs[m].info;
    if (info) {
      info[m] = aggregate(ocs[m]);
      info[m].seconds = secs;
    }
    const ori_status sm = end_status(c, ocs[m], "COCG");
    if (sm != ORI_OK && worst == ORI_OK) {
      worst = sm;
      set_err(nullptr, sm, "problem %zu: %s", m, c->err.c_str());
    }
  }
  return worst;
}

ori_status ori_group_multi_iterations(ori_group g, int64_t* iterations) {
  if (!g) return set_err(nullptr, ORI_ERR_INVALID_ARG, "group is NULL");
  if (!iterations) return set_err(nullptr, ORI_ERR_INVALID_ARG, "iterations is NULL");
  *iterations = g->multi.iterations;
  return ORI_OK;
}

void ori_group_destroy(ori_group g) {
  if (!g) return;
  for (ori_ctx c : g->members) (void)hipStreamSynchronize(c->stream);  // nothing of the group in flight
  g->multi.release();  // the graphs, then the tables their nodes point into
  if (g->multi.gathered) host_pool().give(-1, kGroupMaxProblems * sizeof(ScalarBlock), g->multi.gathered);
  for (ori_ctx c : g->members) ori_destroy(c);
  for (hipStream_t sm : g->streams) {
    (void)hipStreamSynchronize(sm);
    pool_stream_give(g->device, sm);
  }
  if (g->ready) (void)hipEventDestroy(g->ready);
  delete g;
}

ori_status ori_batch_info(ori_ctx c, int32_t i, ori_solve_info* info) {
  if (!c) return set_err(nullptr, ORI_ERR_INVALID_ARG, "context is NULL");
  if (!info) return set_err(c, ORI_ERR_INVALID_ARG, "info is NULL");
  if (i < 0 || i >= static_cast<int32_t>(c->last_info.size()))
    return set_err(c, ORI_ERR_INVALID_ARG, "no solve result for right-hand side %d", i);
  *info = c->last_info[i];
  return ORI_OK;
}

ori_status ori_adjoint(ori_ctx c, const ori_solve_opts* opts_in, const void* u_in, const void* f_in, void* g_out,
                       void* lam_out, ori_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  ORI_TRY(guard(c));
  if (c->nrhs != 1) return set_err(c, ORI_ERR_UNSUPPORTED, "the adjoint needs a context with one right-hand side");
  ori_solve_opts o;
  ORI_TRY(check_opts(c, opts_in, &o));
  o.use_x0 = 0;
  ORI_TRY(check_dev_ptr(c, u_in, c->P * 16, "u"));
  ORI_TRY(check_dev_ptr(c, f_in, c->P * 16, "f"));
  if (!g_out && !lam_out) return set_err(c, ORI_ERR_INVALID_ARG, "g and lam are both NULL");
  if (g_out) ORI_TRY(check_dev_ptr(c, g_out, c->P * 16, "g"));
  if (lam_out) ORI_TRY(check_dev_ptr(c, lam_out, c->P * 16, "lam"));
  Outcome oc;
  ORI_TRY(adjoint_solve(c, o, static_cast<const cxd*>(u_in), static_cast<const cxd*>(f_in), 1.0,
                        static_cast<cxd*>(g_out), static_cast<cxd*>(lam_out), &oc));
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  if (info) {
    *info = oc.info[0];
    info->seconds = elapsed(t0);
  }
  return end_status(c, oc, "adjoint COCG");
}

ori_status ori_gradient(ori_ctx c, const ori_solve_opts* opts_in, const void* target, void* u_out, double* J,
                        void* g_out, ori_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  ORI_TRY(guard(c));
  if (c->nrhs != 1) return set_err(c, ORI_ERR_UNSUPPORTED, "the gradient needs a context with one right-hand side");
  ori_solve_opts o;
  ORI_TRY(check_opts(c, opts_in, &o));
  ORI_TRY(check_dev_ptr(c, target, c->P * 16, "u_target"));
  ORI_TRY(check_dev_ptr(c, u_out, c->P * 16, "u"));
  ORI_TRY(check_dev_ptr(c, g_out, c->P * 16, "dJdh"));
  if (!J) return set_err(c, ORI_ERR_INVALID_ARG, "J is NULL");
  cxd* u = static_cast<cxd*>(u_out);
  Outcome fw;
  ORI_TRY(forward_solve(c, o, u, &fw));
  ori_solve_info inf = fw.info[0];
  if (fw.state[0] != 0) {
    ORI_HIP(c, hipStreamSynchronize(c->stream));
    inf.seconds = elapsed(t0);
    if (info) *info = inf;
    return end_status(c, fw, "forward COCG");
  }
  // f = conj(u - t) (in t2), J = ||u - t||^2
  ORI_TRY(launch(c, K_ELEMWISE, PREC_F64,
                 [&] { return launch_conj_diff(u, target, c->t2, c->P, c->partials, c->stream); }));
  ORI_TRY(finalize(c, rblocks(c), FIN_NORM));
  ORI_TRY(sync_scalars(c));
  *J = c->sc_host[0].aux;
  o.use_x0 = 0;
  Outcome ad;
  ORI_TRY(adjoint_solve(c, o, u, c->t2, 2.0, static_cast<cxd*>(g_out), nullptr, &ad));
  inf.iterations += ad.info[0].iterations;
  inf.refinements += ad.info[0].refinements;
  inf.matvecs += ad.info[0].matvecs;
  inf.matvecs_c64 += ad.info[0].matvecs_c64;
  ORI_HIP(c, hipStreamSynchronize(c->stream));
  inf.seconds = elapsed(t0);
  if (info) *info = inf;
  return end_status(c, ad, "adjoint COCG");
}

ori_status ori_profile_enable(ori_ctx c, int32_t enable) {
  ORI_TRY(guard(c));
  ORI_TRY(prof_fold(c));
  if (enable) {
    std::fill(std::begin(c->prof_ms), std::end(c->prof_ms), 0.0);
    std::fill(std::begin(c->prof_n), std::end(c->prof_n), 0);
  }
  c->prof = enable != 0;
  return ORI_OK;
}

ori_status ori_profile_kinds(ori_ctx c, const char* kinds) {
  ORI_TRY(guard(c));
  if (!kinds || !*kinds) {
    c->prof_mask = ~0u;
    return ORI_OK;
  }
  uint32_t mask = 0;
  std::string list(kinds);
  size_t pos = 0;
  while (pos <= list.size()) {
    const size_t end = std::min(list.find(',', pos), list.size());
    const std::string name = list.substr(pos, end - pos);
    int found = -1;
    for (int k = 0; k < K_NKIND; ++k)
      if (name == kKindNames[k]) found = k;
    if (found < 0) return set_err(c, ORI_ERR_INVALID_ARG, "unknown kernel kind '%s'", name.c_str());
    mask |= 1u << found;
    pos = end + 1;
  }
  c->prof_mask = mask;
  return ORI_OK;
}

ori_status ori_profile_read(ori_ctx c, int32_t max, const char** names, double* avg_ms, int64_t* launches,
                            int32_t* count) {
  ORI_TRY(guard(c));
  ORI_TRY(prof_fold(c));
  static const char* const full[2 * K_NKIND] = {
      "f1.c128",          "f1.c64",          "f2.c128",      "f2.c64",          "zpass.c128",       "zpass.c64",
      "i2.c128",          "i2.c64",          "i1.c128",      "i1.c64",          "update.c128",      "update.c64",
      "finalize",         "finalize.c64",    "init.c128",    "init.c64",        "coefficients",     "coefficients.c64",
      "spectrum",         "spectrum.c64",    "elementwise.c128", "elementwise.c64"};
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

ori_status ori_check_guards(ori_ctx c, int64_t* damaged) {
  ORI_TRY(guard(c));
  if (!damaged) return set_err(c, ORI_ERR_INVALID_ARG, "damaged is NULL");
  return count_damaged_guards(c, damaged);
}

void ori_destroy(ori_ctx c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);  // all of the context's work is on its stream
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  for (auto& g : c->graphs) g.release();
  device_pool().give(c->device, c->ws_bytes, c->ws_block);
  host_pool().give(-1, c->pin_bytes, c->pin_block);
  delete c;
}

void ori_release_cached_memory(void) {
  device_pool().release_all();
  host_pool().release_all();
  std::map<int, std::vector<hipStream_t>> streams;
  {
    std::lock_guard<std::mutex> lk(stream_pool().mu);
    streams.swap(stream_pool().free);
  }
  for (auto& kv : streams)
    for (hipStream_t sm : kv.second) (void)hipStreamDestroy(sm);
}

const char* ori_last_error(ori_ctx c) { return c ? c->err.c_str() : g_last_error.c_str(); }

}  // extern "C"
