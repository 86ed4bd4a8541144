/*
 * CPU oracle for the smooth (soft-min) variant of the wavefront recurrence (test
 * infrastructure only; the product library never links or calls it and shares no code with
 * it).
 *
 * The cell recurrence of reading R0 takes the minimum of the north-west, north and west
 * neighbours.  Its smooth variant replaces that minimum by the soft minimum of temperature
 * gamma > 0,
 *     softmin(x_1, x_2, x_3) = -gamma * log( exp(-x_1/gamma) + exp(-x_2/gamma) + exp(-x_3/gamma) ),
 * so that
 *     D[i][j] = C[i][j] + softmin( D[i-1][j-1], D[i-1][j], D[i][j-1] )
 * with the same virtual boundary as R0 (D[-1][-1] = 0, every other virtual cell +inf, whose
 * exponential is 0).  This is the published soft dynamic-time-warping recursion (Cuturi and
 * Blondel, 2017); as gamma -> 0 it tends to R0.  D[i][j] equals -gamma log of the sum, over
 * every monotone path from (0,0) to (i,j), of exp(-path cost / gamma) -- the tests check
 * that by enumerating the paths.
 *
 * Every softmin is evaluated about its smallest argument mn, which leaves the value
 * unchanged: softmin = mn - gamma * log( sum_k exp((mn - x_k) / gamma) ).
 *
 * Adjoint.  For L = sum(gD * D) + gscore * score (score = D[m-1][n-1]), the gradient
 * E = dL/dD = dL/dC is, in reverse row-major order,
 *     E[i][j] = gD[i][j] + [i==m-1 && j==n-1] gscore
 *             + w(i+1,j+1) E[i+1][j+1] + w(i+1,j) E[i+1][j] + w(i,j+1) E[i][j+1],
 * summed left to right in that order, where the weight of successor s = (p, q) of (i, j) is
 * the derivative of its softmin with respect to D[i][j]:
 *     w(p, q) = exp( (D[p][q] - C[p][q] - D[i][j]) / gamma ).
 * gC = E.  Inputs C must be finite (no blocked cells in this variant).  Double precision,
 * libm exp and log, -O2, no fast-math, no contraction.
 */
#include <math.h>
#include <stdint.h>

void wfo_soft_forward_f64(int64_t m, int64_t n, const double* C, int64_t ldc, double gamma, double* D,
                          int64_t ldd) {
  for (int64_t i = 0; i < m; ++i) {
    for (int64_t j = 0; j < n; ++j) {
      double x[3];
      x[0] = (i == 0 && j == 0) ? 0.0 : (i > 0 && j > 0) ? D[(i - 1) * ldd + (j - 1)] : INFINITY;
      x[1] = (i > 0) ? D[(i - 1) * ldd + j] : INFINITY;
      x[2] = (j > 0) ? D[i * ldd + (j - 1)] : INFINITY;
      double mn = x[0];
      if (x[1] < mn) mn = x[1];
      if (x[2] < mn) mn = x[2];
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += exp((mn - x[k]) / gamma);
      D[i * ldd + j] = C[i * ldc + j] + (mn - gamma * log(s));
    }
  }
}

void wfo_soft_backward_f64(int64_t m, int64_t n, const double* C, int64_t ldc, const double* D, int64_t ldd,
                           double gamma, const double* gD, int64_t ldgd, double gscore, double* gC, int64_t ldgc) {
  for (int64_t i = m - 1; i >= 0; --i) {
    for (int64_t j = n - 1; j >= 0; --j) {
      const double dij = D[i * ldd + j];
      double e = gD ? gD[i * ldgd + j] : 0.0;
      if (i == m - 1 && j == n - 1) e = e + gscore;
      if (i + 1 < m && j + 1 < n) {
        const int64_t p = i + 1, q = j + 1;
        e = e + exp((D[p * ldd + q] - C[p * ldc + q] - dij) / gamma) * gC[p * ldgc + q];
      }
      if (i + 1 < m) {
        const int64_t p = i + 1, q = j;
        e = e + exp((D[p * ldd + q] - C[p * ldc + q] - dij) / gamma) * gC[p * ldgc + q];
      }
      if (j + 1 < n) {
        const int64_t p = i, q = j + 1;
        e = e + exp((D[p * ldd + q] - C[p * ldc + q] - dij) / gamma) * gC[p * ldgc + q];
      }
      gC[i * ldgc + j] = e;
    }
  }
}
