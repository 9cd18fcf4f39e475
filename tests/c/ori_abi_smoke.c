/* Standalone use of the C ABI (include/ori.h), no Python: the two-per-side
 * closed form of eq. 2.19, the error paths, and a group of two problems.
 *
 * With n = 2 and constant h, N, u0 = 1, cube symmetry makes all eight
 * unknowns equal, and eq. 2.19 reduces to
 *   u (1 + D (3 G(d) + 3 G(sqrt(2) d) + G(sqrt(3) d))) = 1,
 * D = 4 pi h N d^3, d = side / 2 the spacing of the cell centres and
 * G(r) = e^{ikr} / (4 pi r) (eq. 2.6a).
 *
 * Exit status 0 and a line "OK ..." on success. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ori.h"

typedef struct {
  double re, im;
} cplx;

static cplx cmul(cplx a, cplx b) { return (cplx){a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
static cplx cdiv1(cplx a) { /* 1 / a */
  const double d = a.re * a.re + a.im * a.im;
  return (cplx){a.re / d, -a.im / d};
}
static cplx green(double k, double r) {
  const double s = 1.0 / (4.0 * M_PI * r);
  return (cplx){cos(k * r) * s, sin(k * r) * s};
}

#define CHECK(cond, ...)              \
  do {                                \
    if (!(cond)) {                    \
      fprintf(stderr, "FAIL: ");      \
      fprintf(stderr, __VA_ARGS__);   \
      fprintf(stderr, "\n");          \
      return 1;                       \
    }                                 \
  } while (0)

int main(void) {
  const int64_t n = 2, P = 8;
  const double side = 1.3, k = 4.0, Nc = 2.5;
  const cplx hc = {0.7, -2.0};
  cplx h_host[8], u0_host[8], u_host[8];
  double N_host[8];
  for (int i = 0; i < 8; ++i) {
    h_host[i] = hc;
    u0_host[i] = (cplx){1.0, 0.0};
    N_host[i] = Nc;
  }
  void *h = NULL, *u0 = NULL, *u = NULL;
  double* N = NULL;
  CHECK(hipMalloc(&h, sizeof h_host) == hipSuccess && hipMalloc(&u0, sizeof u0_host) == hipSuccess &&
            hipMalloc(&u, sizeof u_host) == hipSuccess && hipMalloc((void**)&N, sizeof N_host) == hipSuccess,
        "hipMalloc");
  CHECK(hipMemcpy(h, h_host, sizeof h_host, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(u0, u0_host, sizeof u0_host, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(N, N_host, sizeof N_host, hipMemcpyHostToDevice) == hipSuccess,
        "hipMemcpy");

  ori_grid g = {n, side, {0.0, 0.0, 0.0}, 0.5};
  ori_ctx ctx = NULL;

  /* error paths: host memory is refused before any kernel runs */
  ori_status st = ori_setup(&g, k, h_host, N, u0, NULL, &ctx);
  CHECK(st == ORI_ERR_INVALID_ARG && ctx == NULL, "host pointer accepted (status %d)", (int)st);
  CHECK(strlen(ori_last_error(NULL)) > 0, "no error text");
  ori_grid bad = g;
  bad.n = 513; /* beyond the largest planned length (n <= 512) */
  CHECK(ori_setup(&bad, k, h, N, u0, NULL, &ctx) == ORI_ERR_UNSUPPORTED, "unsupported n accepted");

  st = ori_setup(&g, k, h, N, u0, NULL, &ctx);
  CHECK(st == ORI_OK, "ori_setup: %s", ori_last_error(NULL));
  ori_solve_opts o;
  ori_default_opts(&o);
  o.tol = 1e-14;
  ori_solve_info info;
  st = ori_solve(ctx, &o, u, &info);
  CHECK(st == ORI_OK, "ori_solve: %s", ori_last_error(ctx));
  CHECK(hipMemcpy(u_host, u, sizeof u_host, hipMemcpyDeviceToHost) == hipSuccess, "copy back");

  const double d = side / (double)n;
  const double D = 4.0 * M_PI * Nc * d * d * d;
  const cplx g1 = green(k, d), g2 = green(k, sqrt(2.0) * d), g3 = green(k, sqrt(3.0) * d);
  const cplx sum = {3.0 * g1.re + 3.0 * g2.re + g3.re, 3.0 * g1.im + 3.0 * g2.im + g3.im};
  const cplx hs = cmul(hc, sum);
  const cplx expect = cdiv1((cplx){1.0 + D * hs.re, D * hs.im});
  double err = 0.0;
  for (int i = 0; i < 8; ++i) {
    const double e = hypot(u_host[i].re - expect.re, u_host[i].im - expect.im);
    err = e > err ? e : err;
  }
  CHECK(err <= 1e-13, "closed form: max error %.3e", err);
  CHECK(info.rel_res_true >= 0.0 && info.rel_res_true < 1e-12, "true residual %.3e", info.rel_res_true);

  ori_destroy(ctx);

  /* a group of two problems (n = 4 and 5: padded lengths 8 and 10) solved
   * in one launch per kernel, bitwise each problem's own ori_solve */
  {
    const int64_t ns[2] = {4, 5};
    ori_grid gg[2] = {{4, side, {0.0, 0.0, 0.0}, 0.5}, {5, side, {0.0, 0.0, 0.0}, 0.5}};
    static cplx hb[125], ub[125], out_g[125], out_s[125];
    static double Nb[125];
    for (int i = 0; i < 125; ++i) {
      hb[i] = (cplx){hc.re * (1.0 + 0.01 * (i % 7)), hc.im};
      ub[i] = (cplx){cos(0.3 * i), sin(0.3 * i)};
      Nb[i] = Nc;
    }
    void *hg[2], *u0g[2], *ug[2], *us = NULL;
    double* Ng[2];
    double kk[2] = {k, 0.5 * k};
    for (int j = 0; j < 2; ++j) {
      const size_t P3 = (size_t)(ns[j] * ns[j] * ns[j]);
      CHECK(hipMalloc(&hg[j], P3 * sizeof(cplx)) == hipSuccess && hipMalloc(&u0g[j], P3 * sizeof(cplx)) == hipSuccess &&
                hipMalloc(&ug[j], P3 * sizeof(cplx)) == hipSuccess &&
                hipMalloc((void**)&Ng[j], P3 * sizeof(double)) == hipSuccess,
            "hipMalloc (group)");
      CHECK(hipMemcpy(hg[j], hb, P3 * sizeof(cplx), hipMemcpyHostToDevice) == hipSuccess &&
                hipMemcpy(u0g[j], ub, P3 * sizeof(cplx), hipMemcpyHostToDevice) == hipSuccess &&
                hipMemcpy(Ng[j], Nb, P3 * sizeof(double), hipMemcpyHostToDevice) == hipSuccess,
            "hipMemcpy (group)");
    }
    CHECK(hipMalloc(&us, 125 * sizeof(cplx)) == hipSuccess, "hipMalloc (single)");
    ori_group grp = NULL;
    st = ori_group_create(gg, 2, ORI_PROVISION_FP64, NULL, &grp);
    CHECK(st == ORI_OK, "ori_group_create: %s", ori_last_error(NULL));
    st = ori_group_load_all(grp, kk, (const void* const*)hg, (const double* const*)Ng, (const void* const*)u0g);
    CHECK(st == ORI_OK, "ori_group_load_all: %s", ori_last_error(NULL));
    ori_solve_info ginfo[2];
    st = ori_group_solve(grp, &o, ug, ginfo);
    CHECK(st == ORI_OK, "ori_group_solve: %s", ori_last_error(NULL));
    /* one launch per kernel for both problems, except under ORI_CHECK_GUARDS=1
       (guard checks after every launch: each problem's own launches) */
    const char* guards_env = getenv("ORI_CHECK_GUARDS");
    const int guards_on = guards_env && atoi(guards_env) != 0;
    int64_t multi_iters = 0;
    CHECK(ori_group_multi_iterations(grp, &multi_iters) == ORI_OK && (multi_iters > 0) == !guards_on,
          "multi-problem iterations: %lld", (long long)multi_iters);
    for (int j = 0; j < 2; ++j) {
      const size_t P3 = (size_t)(ns[j] * ns[j] * ns[j]);
      ori_ctx c1 = NULL;
      st = ori_setup(&gg[j], kk[j], hg[j], Ng[j], u0g[j], NULL, &c1);
      CHECK(st == ORI_OK, "ori_setup (n=%lld): %s", (long long)ns[j], ori_last_error(NULL));
      ori_solve_info i1;
      st = ori_solve(c1, &o, us, &i1);
      CHECK(st == ORI_OK, "ori_solve (n=%lld): %s", (long long)ns[j], ori_last_error(c1));
      CHECK(hipMemcpy(out_g, ug[j], P3 * sizeof(cplx), hipMemcpyDeviceToHost) == hipSuccess &&
                hipMemcpy(out_s, us, P3 * sizeof(cplx), hipMemcpyDeviceToHost) == hipSuccess,
            "copy back (group)");
      CHECK(memcmp(out_g, out_s, P3 * sizeof(cplx)) == 0, "group result of n=%lld differs from its own solve",
            (long long)ns[j]);
      CHECK(ginfo[j].iterations == i1.iterations, "iterations differ (n=%lld)", (long long)ns[j]);
      ori_destroy(c1);
    }
    ori_group_destroy(grp);
    for (int j = 0; j < 2; ++j) {
      hipFree(hg[j]);
      hipFree(u0g[j]);
      hipFree(ug[j]);
      hipFree(Ng[j]);
    }
    hipFree(us);
  }

  hipFree(h);
  hipFree(u0);
  hipFree(u);
  hipFree(N);
  /* the blocks and streams the destroyed contexts and group left behind */
  ori_release_cached_memory();
  printf("OK %s n=2 closed form max_err=%.3e iterations=%d; group n=4,5 bitwise\n", ori_version(), err,
         info.iterations);
  return 0;
}
