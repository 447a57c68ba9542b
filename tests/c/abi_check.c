/* Plain-C client of libfpw: compiles against include/fpw.h with a C compiler,
 * links the shared library and exercises the host-side argument checks
 * (no GPU needed).  With argument "gpu" it also runs one small pass on the
 * default device and checks a known peak. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fpw.h"

#define CHECK(cond, ...)                \
  do {                                  \
    if (!(cond)) {                      \
      fprintf(stderr, __VA_ARGS__);     \
      fprintf(stderr, "\n");            \
      return 1;                         \
    }                                   \
  } while (0)

int main(int argc, char** argv) {
  fpw_options o;
  fpw_options_default(&o);
  CHECK(o.n_bins == 10 && o.use_graph == 1 && o.baseline_scale == 1.0, "defaults");
  CHECK(strncmp(fpw_version(), "fpw ", 4) == 0, "version %s", fpw_version());

  enum { N = 300, NF = 2000 };
  int64_t off[2] = {0, N};
  double* t = malloc(sizeof(double) * N);
  double* y = malloc(sizeof(double) * N);
  double* dy = malloc(sizeof(double) * N);
  double* f = malloc(sizeof(double) * NF);
  unsigned s = 12345u;
  for (int i = 0; i < N; ++i) {
    s = s * 1664525u + 1013904223u;
    t[i] = 1000.0 * (double)(s >> 8) / 16777216.0;
    y[i] = 0.1 * sin(2.0 * 3.14159265358979323846 * t[i] / 0.37);
    dy[i] = 0.02;
  }
  for (int k = 0; k < NF; ++k) f[k] = 0.5 + 4.0 * k / (NF - 1);

  fpw_plan_t p = NULL;
  /* host-side checks run before any HIP call */
  o.n_bins = 0;
  CHECK(fpw_plan(&p, 1, off, t, y, dy, NF, f, &o, NULL) == FPW_EINVAL && p == NULL, "M = 0 accepted");
  CHECK(strlen(fpw_last_error()) > 0, "no error text");
  o.n_bins = FPW_MAX_BINS + 1;
  CHECK(fpw_plan(&p, 1, off, t, y, dy, NF, f, &o, NULL) == FPW_EUNSUPPORTED, "M too large accepted");
  o.n_bins = 20;
  dy[7] = -1.0;
  CHECK(fpw_plan(&p, 1, off, t, y, dy, NF, f, &o, NULL) == FPW_EINVAL, "negative dy accepted");
  dy[7] = 0.02;
  CHECK(fpw_plan_shared(&p, 1, 0, t, y, dy, NF, f, &o, NULL) == FPW_EINVAL, "empty shared plan accepted");
  CHECK(fpw_eval_batch(NULL, NULL, NULL, NULL, NULL) == FPW_EINVAL, "null plan accepted");
  fpw_plan_destroy(NULL);

  if (argc > 1 && strcmp(argv[1], "gpu") == 0) {
    o.topk = 3;
    fpw_status st = fpw_plan(&p, 1, off, t, y, dy, NF, f, &o, NULL);
    CHECK(st == FPW_OK, "plan: %s", fpw_last_error());
    fpw_plan_info info;
    CHECK(fpw_get_plan_info(p, &info) == FPW_OK && info.evals == (int64_t)N * NF, "plan info");
    /* device outputs: the library takes device pointers; hipMalloc comes from the
       HIP runtime the library links, declared here to keep this file plain C */
    extern int hipMalloc(void** ptr, size_t size);
    extern int hipMemcpy(void* dst, const void* src, size_t size, int kind);
    extern int hipFree(void* ptr);
    extern int hipDeviceSynchronize(void);
    int32_t* idx_d = NULL;
    float* val_d = NULL;
    CHECK(hipMalloc((void**)&idx_d, 3 * sizeof(int32_t)) == 0 && hipMalloc((void**)&val_d, 3 * sizeof(float)) == 0, "alloc");
    CHECK(fpw_eval_batch(p, NULL, idx_d, val_d, NULL) == FPW_OK, "eval: %s", fpw_last_error());
    CHECK(hipDeviceSynchronize() == 0, "sync");
    int32_t idx[3];
    CHECK(hipMemcpy(idx, idx_d, sizeof(idx), 2 /* device to host */) == 0, "copy");
    const double best = f[idx[0]];
    CHECK(fabs(best - 1.0 / 0.37) < 3.0 * (f[1] - f[0]), "top peak at %g, expected %g", best, 1.0 / 0.37);
    hipFree(idx_d);
    hipFree(val_d);
    fpw_plan_destroy(p);
    printf("gpu pass ok: top peak %.5f /d\n", best);
  }
  free(t);
  free(y);
  free(dy);
  free(f);
  printf("C ABI checks ok\n");
  return 0;
}
