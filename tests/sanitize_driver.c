/*
 * Driver for the sanitizer test (tests/test_sanitizers.py): built with AddressSanitizer and
 * UndefinedBehaviorSanitizer, it runs
 *   - every oracle routine (oracle/wf_oracle.c, oracle/tridiag.c, oracle/softmin.c) on small
 *     random inputs, including the degenerate shapes (1 x 1, one row, one column), and
 *   - when linked with the library (-DWITH_LIB), the argument checks of every entry point of
 *     include/wf.h and include/tri.h on invalid arguments, which must return an error before
 *     any device work (no GPU is needed).
 * Exit status 0 and no sanitizer report = pass.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void wfo_forward_f64(int64_t, int64_t, const double*, int64_t, double*, int64_t, uint8_t*);
void wfo_forward_f32(int64_t, int64_t, const float*, int64_t, float*, int64_t, uint8_t*);
void wfo_forward_i64(int64_t, int64_t, const int64_t*, int64_t, int64_t*, int64_t, uint8_t*);
void wfo_backward_f64(int64_t, int64_t, const uint8_t*, const double*, int64_t, double, double*, int64_t);
void wfo_backward_f32(int64_t, int64_t, const uint8_t*, const float*, int64_t, float, float*, int64_t);
int tro_thomas_f64(int64_t, const double*, const double*, const double*, const double*, double*);
int tro_partition_f64(int64_t, int32_t, const int32_t*, const double*, const double*, const double*,
                      const double*, double*);
int tro_partition_f32(int64_t, int32_t, const int32_t*, const float*, const float*, const float*, const float*,
                      float*);
void wfo_soft_forward_f64(int64_t, int64_t, const double*, int64_t, double, double*, int64_t);
void wfo_soft_backward_f64(int64_t, int64_t, const double*, int64_t, const double*, int64_t, double, const double*,
                           int64_t, double, double*, int64_t);

static double rnd(void) { return (double)rand() / RAND_MAX; }

static int oracle_runs(void) {
  const int64_t shapes[][2] = {{1, 1}, {1, 9}, {7, 1}, {5, 6}, {33, 17}};
  for (int s = 0; s < 5; ++s) {
    const int64_t m = shapes[s][0], n = shapes[s][1];
    double* C = malloc(sizeof(double) * m * n);
    double* D = malloc(sizeof(double) * m * n);
    double* G = malloc(sizeof(double) * m * n);
    float* Cf = malloc(sizeof(float) * m * n);
    float* Df = malloc(sizeof(float) * m * n);
    float* Gf = malloc(sizeof(float) * m * n);
    int64_t* Ci = malloc(sizeof(int64_t) * m * n);
    int64_t* Di = malloc(sizeof(int64_t) * m * n);
    uint8_t* sel = malloc((size_t)(m * n));
    for (int64_t k = 0; k < m * n; ++k) {
      C[k] = rnd();
      Cf[k] = (float)C[k];
      Ci[k] = rand() % 1000;
    }
    wfo_forward_f64(m, n, C, n, D, n, sel);
    wfo_backward_f64(m, n, sel, D, n, 1.0, G, n);
    wfo_forward_f32(m, n, Cf, n, Df, n, sel);
    wfo_backward_f32(m, n, sel, NULL, n, 1.0f, Gf, n);
    wfo_forward_i64(m, n, Ci, n, Di, n, NULL);
    wfo_soft_forward_f64(m, n, C, n, 0.5, D, n);
    wfo_soft_backward_f64(m, n, C, n, D, n, 0.5, NULL, n, 1.0, G, n);
    if (!isfinite(G[0])) return 1;
    free(C), free(D), free(G), free(Cf), free(Df), free(Gf), free(Ci), free(Di), free(sel);
  }
  const int64_t Ns[] = {1, 2, 3, 10, 101, 1000};
  const int32_t ms[] = {4, 10, 3};
  for (int s = 0; s < 6; ++s) {
    const int64_t N = Ns[s];
    double* v[5];
    float* f[5];
    for (int q = 0; q < 5; ++q) {
      v[q] = malloc(sizeof(double) * N);
      f[q] = malloc(sizeof(float) * N);
    }
    for (int64_t i = 0; i < N; ++i) {
      v[0][i] = i ? rnd() - 0.5 : 0.0;
      v[2][i] = i < N - 1 ? rnd() - 0.5 : 0.0;
      v[1][i] = 2.0 + rnd();
      v[3][i] = rnd();
      for (int q = 0; q < 4; ++q) f[q][i] = (float)v[q][i];
    }
    if (tro_thomas_f64(N, v[0], v[1], v[2], v[3], v[4])) return 2;
    for (int R = -1; R <= 2 && N >= 2; ++R) {
      if (tro_partition_f64(N, R, ms, v[0], v[1], v[2], v[3], v[4])) return 3;
      if (tro_partition_f32(N, R, ms, f[0], f[1], f[2], f[3], f[4])) return 4;
    }
    for (int q = 0; q < 5; ++q) free(v[q]), free(f[q]);
  }
  return 0;
}

#ifdef WITH_LIB
#include "../include/tri.h"
#include "../include/wf.h"

static int lib_checks(void) {
  void* P = (void*)0x1000; /* never dereferenced: every call below fails its checks first */
  int bad = 0;
  bad |= wf_forward(7, 4, 4, P, 4, P, 4, P, NULL, 0, NULL) != WF_E_ARG;
  bad |= wf_forward(0, 0, 4, P, 4, P, 4, P, NULL, 0, NULL) != WF_E_ARG;
  bad |= wf_forward(0, 4, 4, P, 3, P, 4, P, NULL, 0, NULL) != WF_E_ARG;
  bad |= wf_forward(0, (int64_t)1 << 40, (int64_t)1 << 31, P, (int64_t)1 << 31, NULL, 1, P, NULL, 0, NULL) != WF_E_ARG;
  bad |= wf_forward_noalloc(1, 16384, 16384, P, 16384, NULL, 16384, P, NULL, 0, NULL) != WF_E_UNSUPPORTED;
  bad |= wf_backward(2, 4, 4, P, 4, NULL, 0, P, 4, NULL, NULL, 4, P, 4, NULL) != WF_E_UNSUPPORTED;
  bad |= wf_backward(0, 4, 4, P, 4, P, 64, P, 4, NULL, NULL, 4, P, 4, NULL) != WF_E_ARG;
  bad |= wf_select(0, 4, 4, NULL, 4, NULL, 0, P, 4, NULL) != WF_E_ARG;
  bad |= wf_soft_forward(0, 4, 4, 0.0, P, 4, P, 4, P, NULL) != WF_E_ARG;
  bad |= wf_soft_forward(0, 4, 4, NAN, P, 4, P, 4, P, NULL) != WF_E_ARG;
  bad |= wf_soft_backward(2, 4, 4, 1.0, P, 4, P, 4, NULL, NULL, 4, P, 4, NULL) != WF_E_UNSUPPORTED;
  bad |= wf_ckpt_elems(0, 5, 64) != -1;
  bad |= wf_set_tile(8) != WF_E_ARG;
  bad |= wf_tile_predict(5, 10, 10, 0) != WF_E_ARG;
  bad |= tri_stage1(1, 0, 100, 4, P, P, P, P, P, P, P, P, NULL) != WF_E_ARG;
  bad |= tri_stage3(1, 1, 100, 1, P, P, P, P, P, P, NULL) != WF_E_ARG;
  bad |= tri_thomas(1, 1, 0, P, P, P, P, P, P, NULL) != WF_E_ARG;
  bad |= tri_subsystems(1, 4) != -1;
  tri_plan* h = NULL;
  bad |= tri_plan_create(&h, 1, 1, 100, 4, 9, NULL) != WF_E_ARG;
  bad |= tri_plan_create(&h, 1, 1, 100000, 3000, 0, NULL) != WF_E_UNSUPPORTED;
  bad |= h != NULL;
  int32_t m = 0, R = 0, msv[TRI_MAX_R];
  bad |= tri_predict(1, 100000000, &m, &R, msv) != WF_OK;
  bad |= tri_predict(9, 1000, &m, &R, msv) != WF_E_ARG;
  return bad;
}
#endif

int main(void) {
  srand(1);
  int rc = oracle_runs();
  if (rc) {
    fprintf(stderr, "oracle run failed: %d\n", rc);
    return 10 + rc;
  }
#ifdef WITH_LIB
  if (lib_checks()) {
    fprintf(stderr, "an argument check did not return the expected code\n");
    return 20;
  }
#endif
  printf("sanitized run ok\n");
  return 0;
}
