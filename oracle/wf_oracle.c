/*
 * CPU oracle for the anti-diagonal wavefront cell recurrence (test infrastructure only).
 *
 * This file is the plain, slow, row-by-row definition that the GPU sweep is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the product library never links or calls it, and it shares no code, header or
 * constant with the GPU path.
 *
 * What it computes (reading "R0"; the paper never states a cell recurrence, its only
 * trace being the unused preamble macros giving 2n-1 anti-diagonals for an n x n grid and
 * a 3 n^2 per-sweep byte count, so the recurrence below is a documented reading):
 *
 *   Forward.  For an m x n input C (row-major, leading dimension ldc >= n):
 *       D[i][j] = C[i][j] + min( D[i-1][j-1], D[i-1][j], D[i][j-1] )
 *   with the virtual boundary  D[-1][-1] = 0  and  D[-1][j] = D[i][-1] = +inf  otherwise,
 *   so D[0][0] = C[0][0] and row 0 / column 0 are prefix sums.  The score is D[m-1][n-1].
 *   Each cell records which predecessor it took, SEL[i][j] in {NW, N, W}; ties go to the
 *   first in the order NW, N, W (strict "<" comparisons).  Cell (0,0) records SEL = NONE.
 *
 *   Adjoint.  For the loss  L = sum(gD * D) + gscore * score  and a fixed SEL, the routed
 *   (sub)gradient A = dL/dD = dL/dC is, in reverse row-major order,
 *       A[i][j] = gD[i][j] + [i==m-1 && j==n-1] * gscore
 *               + [SEL[i+1][j+1] == NW] * A[i+1][j+1]
 *               + [SEL[i+1][j]   == N ] * A[i+1][j]
 *               + [SEL[i][j+1]   == W ] * A[i][j+1]
 *   summed left to right in exactly that order, and gC = A.  (The order of the three
 *   routed terms is a reading: the paper gives none.  This one adds the terms that come
 *   from the row below first and the term from the same row last, so that in a sweep by
 *   row bands every contribution from the band below is known before the row's own.)
 *
 * Precision: the f64 forms accumulate in double (inputs may be float data widened to
 * double, so input quantisation is not counted as error); the f32 forms perform exactly one
 * IEEE single-precision add per cell, which makes them the bitwise reference for a float
 * implementation of the same recurrence; the i64 form is exact integer arithmetic.
 * Build with -O2 and no fast-math, no FP contraction.
 */
#include <stdint.h>
#include <stddef.h>
#include <math.h>

enum { WFO_SEL_NONE = 0, WFO_SEL_NW = 1, WFO_SEL_N = 2, WFO_SEL_W = 3 };

/* --- forward, one definition per arithmetic type ------------------------------------- */

#define WFO_DEFINE_FORWARD(NAME, T, INF)                                                    \
  void NAME(int64_t m, int64_t n, const T* C, int64_t ldc, T* D, int64_t ldd,             \
            uint8_t* sel) {                                                                \
    for (int64_t i = 0; i < m; ++i) {                                                      \
      for (int64_t j = 0; j < n; ++j) {                                                    \
        T nw, no, w;                                                                       \
        if (i == 0 && j == 0) {                                                            \
          nw = (T)0; no = INF; w = INF;                                                    \
        } else {                                                                           \
          nw = (i > 0 && j > 0) ? D[(i - 1) * ldd + (j - 1)] : INF;                        \
          no = (i > 0) ? D[(i - 1) * ldd + j] : INF;                                       \
          w = (j > 0) ? D[i * ldd + (j - 1)] : INF;                                        \
        }                                                                                  \
        T v = nw;                                                                          \
        uint8_t s = WFO_SEL_NW;                                                            \
        if (no < v) { v = no; s = WFO_SEL_N; }                                             \
        if (w < v) { v = w; s = WFO_SEL_W; }                                               \
        if (i == 0 && j == 0) s = WFO_SEL_NONE;                                            \
        D[i * ldd + j] = C[i * ldc + j] + v;                                               \
        if (sel) sel[i * n + j] = s;                                                       \
      }                                                                                    \
    }                                                                                      \
  }

WFO_DEFINE_FORWARD(wfo_forward_f64, double, (double)INFINITY)
WFO_DEFINE_FORWARD(wfo_forward_f32, float, (float)INFINITY)

/* Exact integer form: int64 arithmetic, +inf represented by INT64_MAX (never added to). */
void wfo_forward_i64(int64_t m, int64_t n, const int64_t* C, int64_t ldc, int64_t* D,
                     int64_t ldd, uint8_t* sel) {
  const int64_t INF = INT64_MAX;
  for (int64_t i = 0; i < m; ++i) {
    for (int64_t j = 0; j < n; ++j) {
      int64_t nw, no, w;
      if (i == 0 && j == 0) {
        nw = 0; no = INF; w = INF;
      } else {
        nw = (i > 0 && j > 0) ? D[(i - 1) * ldd + (j - 1)] : INF;
        no = (i > 0) ? D[(i - 1) * ldd + j] : INF;
        w = (j > 0) ? D[i * ldd + (j - 1)] : INF;
      }
      int64_t v = nw;
      uint8_t s = WFO_SEL_NW;
      if (no < v) { v = no; s = WFO_SEL_N; }
      if (w < v) { v = w; s = WFO_SEL_W; }
      if (i == 0 && j == 0) s = WFO_SEL_NONE;
      D[i * ldd + j] = C[i * ldc + j] + v; /* every real cell has a finite predecessor */
      if (sel) sel[i * n + j] = s;
    }
  }
}

/* --- adjoint ----------------------------------------------------------------------------- */

#define WFO_DEFINE_BACKWARD(NAME, T)                                                        \
  void NAME(int64_t m, int64_t n, const uint8_t* sel, const T* gD, int64_t ldgd, T gscore, \
            T* gC, int64_t ldgc) {                                                         \
    for (int64_t i = m - 1; i >= 0; --i) {                                                 \
      for (int64_t j = n - 1; j >= 0; --j) {                                               \
        T a = gD ? gD[i * ldgd + j] : (T)0;                                                \
        if (i == m - 1 && j == n - 1) a = a + gscore;                                      \
        if (i + 1 < m && j + 1 < n && sel[(i + 1) * n + (j + 1)] == WFO_SEL_NW)            \
          a = a + gC[(i + 1) * ldgc + (j + 1)];                                            \
        if (i + 1 < m && sel[(i + 1) * n + j] == WFO_SEL_N) a = a + gC[(i + 1) * ldgc + j]; \
        if (j + 1 < n && sel[i * n + (j + 1)] == WFO_SEL_W) a = a + gC[i * ldgc + (j + 1)]; \
        gC[i * ldgc + j] = a;                                                              \
      }                                                                                    \
    }                                                                                      \
  }

WFO_DEFINE_BACKWARD(wfo_backward_f64, double)
WFO_DEFINE_BACKWARD(wfo_backward_f32, float)

/* Version tag so the Python wrapper can refuse a stale build. */
int wfo_version(void) { return 2; }
