// One FFT pass of several problems of different padded lengths in one
// launch (the uneven batch of independent problems; kernels.h, MultiProblem).
// Every length of multi_length() has its pass bodies compiled here, in a
// namespace of its own, from the same source as its single-problem kernels
// (pass_bodies.inc), with the tile shape of kernels.h; a launch runs each
// problem's workgroups on its own length's body.
#include "fft_engine.h"
#include "kernels.h"
#include "launch.h"
#include "pass_common.h"

namespace ori {

namespace ml8 {
constexpr int L = 8;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml8

namespace ml10 {
constexpr int L = 10;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml10

namespace ml12 {
constexpr int L = 12;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml12

namespace ml16 {
constexpr int L = 16;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml16

namespace ml20 {
constexpr int L = 20;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml20

namespace ml24 {
constexpr int L = 24;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml24

namespace ml32 {
constexpr int L = 32;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml32

namespace ml40 {
constexpr int L = 40;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml40

namespace ml48 {
constexpr int L = 48;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml48

namespace ml64 {
constexpr int L = 64;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml64

namespace ml80 {
constexpr int L = 80;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml80

namespace ml96 {
constexpr int L = 96;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml96

namespace ml128 {
constexpr int L = 128;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml128

namespace ml192 {
constexpr int L = 192;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml192

namespace ml256 {
constexpr int L = 256;
#include "pass_bodies.inc"
#include "multi_len.inc"
}  // namespace ml256

// every length with multi-problem bodies (multi_length in kernels.h)
#define ORI_MULTI_LENGTHS(X) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) X(192) X(256)

namespace {

#define ORI_MULTI_CHECK(Lv) static_assert(multi_length(Lv), "length without multi-problem bodies");
ORI_MULTI_LENGTHS(ORI_MULTI_CHECK)
#undef ORI_MULTI_CHECK

template <typename T, int PASS>
constexpr int max_threads() {
  int t = 0;
#define ORI_MT(Lv) t = ml##Lv::mp_threads<T, PASS>() > t ? ml##Lv::mp_threads<T, PASS>() : t;
  ORI_MULTI_LENGTHS(ORI_MT)
#undef ORI_MT
  return t;
}

// Launch workgroup b runs workgroup b - first_block of the problem whose
// range holds it (problems in ascending first_block), on its length's body.
// The LDS is dynamic: the largest the launch's problems need.
template <typename T, int PASS>
__global__ void __launch_bounds__((max_threads<T, PASS>())) k_multi_pass(const MultiProblem* __restrict__ tab,
                                                                       int32_t np) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t b = blockIdx.x;
  int p = 0;
  while (p + 1 < np && tab[p + 1].first_block <= b) ++p;
  const MultiProblem m = tab[p];
  const int64_t bid = b - m.first_block;
  switch (m.L) {
#define ORI_MC(Lv)                                \
  case Lv:                                        \
    ml##Lv::mp_run<T, PASS>(m, bid, smem);        \
    break;
    ORI_MULTI_LENGTHS(ORI_MC)
#undef ORI_MC
    default:
      break;
  }
}

// dynamic LDS of a launch: within the 64 KB a launch gets without asking
constexpr int kMaxDynSmem = 64 * 1024;

template <typename T, int PASS>
hipError_t launch_t(const MultiProblem* tab, int32_t np, int64_t blocks, int threads, int smem, hipStream_t st) {
  if (threads < 64 || threads > max_threads<T, PASS>() || threads % 64 != 0) return hipErrorInvalidValue;
  if (smem < 0 || smem > kMaxDynSmem) return hipErrorInvalidValue;
  return launch_kernel_smem(k_multi_pass<T, PASS>, dim3(static_cast<unsigned>(blocks)), dim3(threads),
                            static_cast<unsigned>(smem), st, tab, np);
}

template <typename T>
hipError_t launch_prec(int pass, const MultiProblem* tab, int32_t np, int64_t blocks, int threads, int smem,
                       hipStream_t st) {
  switch (pass) {
    case MP_F1: return launch_t<T, MP_F1>(tab, np, blocks, threads, smem, st);
    case MP_F2: return launch_t<T, MP_F2>(tab, np, blocks, threads, smem, st);
    case MP_Z: return launch_t<T, MP_Z>(tab, np, blocks, threads, smem, st);
    case MP_I2: return launch_t<T, MP_I2>(tab, np, blocks, threads, smem, st);
    case MP_I1: return launch_t<T, MP_I1>(tab, np, blocks, threads, smem, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
int smem_prec(int L, int pass) {
  switch (L) {
#define ORI_SM(Lv)                                                                \
  case Lv:                                                                        \
    switch (pass) {                                                               \
      case MP_F1: return ml##Lv::mp_smem<T, MP_F1>();                             \
      case MP_F2: return ml##Lv::mp_smem<T, MP_F2>();                             \
      case MP_Z: return ml##Lv::mp_smem<T, MP_Z>();                               \
      case MP_I2: return ml##Lv::mp_smem<T, MP_I2>();                             \
      case MP_I1: return ml##Lv::mp_smem<T, MP_I1>();                             \
      default: return 0;                                                          \
    }
    ORI_MULTI_LENGTHS(ORI_SM)
#undef ORI_SM
    default:
      return 0;
  }
}

#define ORI_SMEM_CHECK(Lv)                                                                              \
  static_assert(ml##Lv::mp_smem<double, MP_F1>() <= kMaxDynSmem && ml##Lv::mp_smem<double, MP_Z>() <= kMaxDynSmem && \
                    ml##Lv::mp_smem<double, MP_F2>() <= kMaxDynSmem,                                     \
                "multi-problem LDS above 64 KB");
ORI_MULTI_LENGTHS(ORI_SMEM_CHECK)
#undef ORI_SMEM_CHECK

template <typename T>
int threads_prec(int L, int pass) {
  switch (L) {
#define ORI_TH(Lv)                                                                \
  case Lv:                                                                        \
    switch (pass) {                                                               \
      case MP_F1: return ml##Lv::mp_threads<T, MP_F1>();                          \
      case MP_F2: return ml##Lv::mp_threads<T, MP_F2>();                          \
      case MP_Z: return ml##Lv::mp_threads<T, MP_Z>();                            \
      case MP_I2: return ml##Lv::mp_threads<T, MP_I2>();                          \
      case MP_I1: return ml##Lv::mp_threads<T, MP_I1>();                          \
      default: return 0;                                                          \
    }
    ORI_MULTI_LENGTHS(ORI_TH)
#undef ORI_TH
    default:
      return 0;
  }
}

template <typename T>
bool soff_prec(int L, int e_lg) {
  switch (L) {
#define ORI_SO(Lv) \
  case Lv:         \
    return ml##Lv::mz_soff_ok<T>(e_lg);
    ORI_MULTI_LENGTHS(ORI_SO)
#undef ORI_SO
    default:
      return false;
  }
}

}  // namespace

int multi_pass_threads(int L, int prec, int pass) {
  return prec == PREC_F64 ? threads_prec<double>(L, pass) : threads_prec<float>(L, pass);
}

int multi_pass_smem(int L, int prec, int pass) {
  return prec == PREC_F64 ? smem_prec<double>(L, pass) : smem_prec<float>(L, pass);
}

bool multi_z_soff(int L, int prec, int e_lg) {
  return prec == PREC_F64 ? soff_prec<double>(L, e_lg) : soff_prec<float>(L, e_lg);
}

hipError_t launch_multi_pass(int prec, int pass, const MultiProblem* tab, int32_t np, int64_t blocks, int threads,
                             int smem, hipStream_t st) {
  if (np < 1 || blocks < 1) return hipErrorInvalidValue;
  return prec == PREC_F64 ? launch_prec<double>(pass, tab, np, blocks, threads, smem, st)
                          : launch_prec<float>(pass, tab, np, blocks, threads, smem, st);
}

}  // namespace ori
