/* A C program that drives the library through its C ABI alone: device
 * memory from the HIP runtime, no Python and no torch.  It steps a small
 * +-1 instance with the paper's defaults, reads the spins back and checks
 * the library's exact energies against Eq. (1) evaluated on the host for
 * those spins; it also checks two error paths.  Exit status 0 on success. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "spring_ising.h"

#define N 96
#define R 5
#define STEPS 300

static uint64_t splitmix64(uint64_t *state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

#define HIP_OK(expr)                                                   \
  do {                                                                 \
    if ((expr) != hipSuccess) {                                        \
      fprintf(stderr, "HIP call failed: %s\n", #expr);                 \
      return 2;                                                        \
    }                                                                  \
  } while (0)

int main(void) {
  static float hJ[N * N], hx[R * N];
  static int8_t hs[R * N];
  int32_t he[R];
  uint64_t st = 2305;
  memset(hJ, 0, sizeof hJ);
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) hJ[i * N + j] = hJ[j * N + i] = (splitmix64(&st) >> 63) ? 1.f : -1.f;
  for (int k = 0; k < R * N; ++k)
    hx[k] = (float)(-0.1 + 0.2 * (double)(splitmix64(&st) >> 11) * 0x1p-53);

  float *dJ = NULL, *dx = NULL;
  int8_t *ds = NULL;
  int32_t *de = NULL;
  HIP_OK(hipMalloc((void **)&dJ, sizeof hJ));
  HIP_OK(hipMalloc((void **)&dx, sizeof hx));
  HIP_OK(hipMalloc((void **)&ds, sizeof hs));
  HIP_OK(hipMalloc((void **)&de, sizeof he));
  HIP_OK(hipMemcpy(dJ, hJ, sizeof hJ, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dx, hx, sizeof hx, hipMemcpyHostToDevice));

  si_params prm;
  if (spring_ising_default_params(&prm, STEPS) != SI_OK) return 3;
  si_ctx *ctx = NULL;
  /* host memory where device memory is required is rejected */
  if (spring_ising_init(&ctx, N, R, hJ, dx, NULL, &prm, NULL) != SI_ERR_INVALID || ctx) {
    fprintf(stderr, "host J was not rejected\n");
    return 4;
  }
  if (spring_ising_init(&ctx, N, R, dJ, dx, NULL, &prm, NULL) != SI_OK) {
    fprintf(stderr, "init: %s\n", spring_ising_last_error());
    return 5;
  }
  if (spring_ising_run(ctx, STEPS) != SI_OK || spring_ising_spins(ctx, ds) != SI_OK ||
      spring_ising_energy(ctx, de, NULL) != SI_OK) {
    fprintf(stderr, "run: %s\n", spring_ising_last_error());
    return 6;
  }
  /* the schedule is exhausted */
  if (spring_ising_run(ctx, 1) != SI_ERR_RANGE || !spring_ising_last_error()[0]) return 7;
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(hs, ds, sizeof hs, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(he, de, sizeof he, hipMemcpyDeviceToHost));
  int bad = 0;
  printf("c-abi demo N=%d R=%d steps=%d energies", N, R, STEPS);
  for (int r = 0; r < R; ++r) {
    long e = 0;
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j)
        e -= (long)hJ[i * N + j] * hs[r * N + i] * hs[r * N + j];
    printf(" %d", he[r]);
    if (e != he[r]) bad = 1;
    for (int i = 0; i < N; ++i)
      if (hs[r * N + i] != 1 && hs[r * N + i] != -1) bad = 1;
  }
  printf("%s\n", bad ? " MISMATCH" : " (match Eq. (1) on the host)");
  if (spring_ising_destroy(ctx) != SI_OK) return 8;
  hipFree(dJ);
  hipFree(dx);
  hipFree(ds);
  hipFree(de);
  return bad ? 1 : 0;
}
