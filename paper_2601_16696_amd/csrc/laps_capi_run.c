/*
 * A plain C consumer of the library's ABI (include/laps.h) with the HIP
 * runtime's C API and no other framework.
 *
 *   laps_capi_run IN OUT N D SEED
 *
 * IN holds a diagonal Gaussian's variances (D doubles) and the starts of N
 * chains (N x D doubles, row-major).  The program runs 12 unadjusted steps
 * with the switch at step 12, then 3 MAMS transitions, in FP64, and writes
 * the final positions (N x D doubles) followed by t, phase and eps to OUT.
 * Exit status 0 on success, else the number of the failing step.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "laps.h"

int main(int argc, char **argv) {
  if (argc < 6) return 1;
  const int64_t N = atoll(argv[3]), D = atoll(argv[4]);
  if (N < 2 || D < 2 || N > 65536 || D > 8192) return 1;
  const int64_t ld = laps_row_stride(D);
  double *s2 = malloc(sizeof(double) * D), *x = calloc((size_t)(N * ld), sizeof(double));
  if (!s2 || !x) return 2;
  FILE *f = fopen(argv[1], "rb");
  if (!f || fread(s2, sizeof(double), (size_t)D, f) != (size_t)D) return 2;
  for (int64_t m = 0; m < N; ++m)
    if (fread(x + m * ld, sizeof(double), (size_t)D, f) != (size_t)D) return 2;
  fclose(f);

  laps_config cfg;
  laps_config_default(&cfg, N, D);
  cfg.seed = (uint64_t)strtoull(argv[5], NULL, 10);
  cfg.switch_policy = 1;
  cfg.max_steps_unadj = 12;
  cfg.max_steps_total = 12 + 15 * 3;
  void *s2_dev = NULL, *x_dev = NULL, *ws_dev = NULL;
  if (hipMalloc(&s2_dev, sizeof(double) * D) != hipSuccess || hipMalloc(&x_dev, sizeof(double) * N * ld) != hipSuccess)
    return 3;
  if (hipMemcpy(s2_dev, s2, sizeof(double) * D, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(x_dev, x, sizeof(double) * N * ld, hipMemcpyHostToDevice) != hipSuccess)
    return 3;
  laps_target tg = {0};
  tg.kind = LAPS_GAUSS_DIAG;
  tg.d = D;
  tg.data[0] = s2_dev;
  size_t bytes = 0;
  if (laps_workspace_size(&cfg, &tg, &bytes) != LAPS_OK) return 4;
  if (hipMalloc(&ws_dev, bytes) != hipSuccess) return 5;
  laps_ctx *ctx = NULL;
  if (laps_init(&cfg, &tg, x_dev, NULL, ws_dev, bytes, NULL, &ctx) != LAPS_OK) return 6;
  if (laps_step_unadjusted(ctx, 12) != LAPS_OK) return 7;
  if (laps_step_adjusted(ctx, 3) != LAPS_OK) return 8;
  laps_stats st;
  if (laps_ensemble_stats(ctx, &st, NULL) != LAPS_OK) return 9;
  if (hipMemcpy(x, x_dev, sizeof(double) * N * ld, hipMemcpyDeviceToHost) != hipSuccess) return 10;
  f = fopen(argv[2], "wb");
  if (!f) return 11;
  for (int64_t m = 0; m < N; ++m) fwrite(x + m * ld, sizeof(double), (size_t)D, f);
  const double tail[3] = {(double)st.t, (double)st.phase, st.eps};
  fwrite(tail, sizeof(double), 3, f);
  fclose(f);
  laps_destroy(ctx);
  hipFree(ws_dev);
  hipFree(x_dev);
  hipFree(s2_dev);
  free(x);
  free(s2);
  return 0;
}
