/*
 * CPU oracle for the tridiagonal partition method (test infrastructure only).
 *
 * The same three stages as oracle/tridiag.py (which the tests pin to exact rational
 * arithmetic, a dense library solve and closed forms), written out in plain C so that the
 * systems of the benchmark's size (10^8 unknowns) can be checked in seconds.  The tests
 * hold this file to the Python oracle bit for bit, in float64 and float32, on every shape
 * they run.  Only the tests and the benchmark's CPU-baseline leg load it; the product
 * library never links or calls it and shares no code with it.
 *
 * System (the paper states no storage): a (sub-diagonal, a[0] unused), b, c (c[N-1]
 * unused), d; row i reads a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i].
 *
 * The method (the paper's Introduction, and its section on the recursive variant):
 *   - cut the rows into sub-systems of m rows: P = ceil(N/m), all of m rows but the last,
 *     which holds the rest; a last sub-system of one row joins the one before it;
 *   - Stage 1: each sub-system k (rows s .. e) yields interface row 2k, its rows eliminated
 *     upward onto row s with x_e kept apart (a[s], r, g, t), and interface row 2k+1, its
 *     rows eliminated downward onto row e with x_s kept apart (f, p, c[e], q);
 *   - Stage 2: the interface system (2P unknowns z, z[2k] = x_s, z[2k+1] = x_e) is solved by
 *     the Thomas algorithm, or cut again (R recursive steps with sizes m_1 .. m_R);
 *   - Stage 3: each sub-system's interior rows are solved from x_s and x_e by recomputing
 *     the downward elimination and substituting back from x_e.
 * Build with -O2, no fast-math, no FP contraction (one rounding per operation, in the
 * order written).
 */
#include <stdint.h>
#include <stdlib.h>

static int64_t tro_count(int64_t N, int64_t m) {
  int64_t P = (N + m - 1) / m;
  if (P > 1 && N - (P - 1) * m == 1) P -= 1;
  return P;
}

int64_t tro_subsystems(int64_t N, int64_t m) { return (N < 2 || m < 2) ? -1 : tro_count(N, m); }

#define TRO_DEFINE(SUF, T)                                                                      \
  /* Thomas: piv_i = b_i - a_i cp_{i-1}, cp_i = c_i / piv_i, dp_i = (d_i - a_i dp_{i-1})/piv_i; \
     x_{N-1} = dp_{N-1}, x_i = dp_i - cp_i x_{i+1}. */                                          \
  int tro_thomas_##SUF(int64_t N, const T* a, const T* b, const T* c, const T* d, T* x) {       \
    T* cp = (T*)malloc((size_t)N * sizeof(T));                                                  \
    T* dp = (T*)malloc((size_t)N * sizeof(T));                                                  \
    if (!cp || !dp) { free(cp); free(dp); return 1; }                                           \
    for (int64_t i = 0; i < N; ++i) {                                                           \
      T piv = i > 0 ? b[i] - a[i] * cp[i - 1] : b[i];                                           \
      cp[i] = i < N - 1 ? c[i] / piv : (T)0;                                                    \
      dp[i] = i > 0 ? (d[i] - a[i] * dp[i - 1]) / piv : d[i] / piv;                             \
    }                                                                                           \
    x[N - 1] = dp[N - 1];                                                                       \
    for (int64_t i = N - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];                       \
    free(cp);                                                                                   \
    free(dp);                                                                                   \
    return 0;                                                                                   \
  }                                                                                             \
                                                                                                \
  /* Stage 1 of one level: the interface system (A, B, C, D, 2P rows each). */                  \
  void tro_interface_##SUF(int64_t N, int64_t m, const T* a, const T* b, const T* c,            \
                           const T* d, T* A, T* B, T* C, T* D) {                                \
    const int64_t P = tro_count(N, m);                                                          \
    for (int64_t k = 0; k < P; ++k) {                                                           \
      const int64_t s = k * m, e = (k < P - 1) ? s + m - 1 : N - 1;                             \
      /* upward elimination onto row s, x_e kept apart */                                       \
      T g = c[e - 1], r = b[e - 1], t = d[e - 1];                                               \
      for (int64_t i = e - 2; i >= s; --i) {                                                    \
        T w = c[i] / r;                                                                         \
        g = -w * g;                                                                             \
        r = b[i] - w * a[i + 1];                                                                \
        t = d[i] - w * t;                                                                       \
      }                                                                                         \
      A[2 * k] = k > 0 ? a[s] : (T)0;                                                           \
      B[2 * k] = r;                                                                             \
      C[2 * k] = g;                                                                             \
      D[2 * k] = t;                                                                             \
      /* downward elimination onto row e, x_s kept apart */                                     \
      T f = a[s + 1], p = b[s + 1], q = d[s + 1];                                               \
      for (int64_t i = s + 2; i <= e; ++i) {                                                    \
        T w = a[i] / p;                                                                         \
        f = -w * f;                                                                             \
        p = b[i] - w * c[i - 1];                                                                \
        q = d[i] - w * q;                                                                       \
      }                                                                                         \
      A[2 * k + 1] = f;                                                                         \
      B[2 * k + 1] = p;                                                                         \
      C[2 * k + 1] = k < P - 1 ? c[e] : (T)0;                                                   \
      D[2 * k + 1] = q;                                                                         \
    }                                                                                           \
  }                                                                                             \
                                                                                                \
  /* Stage 3 of one level: x from the interface unknowns z. */                                  \
  int tro_back_solve_##SUF(int64_t N, int64_t m, const T* a, const T* b, const T* c,            \
                           const T* d, const T* z, T* x) {                                      \
    const int64_t P = tro_count(N, m);                                                          \
    T* f = (T*)malloc((size_t)(m + 1) * sizeof(T));                                             \
    T* p = (T*)malloc((size_t)(m + 1) * sizeof(T));                                             \
    T* q = (T*)malloc((size_t)(m + 1) * sizeof(T));                                             \
    if (!f || !p || !q) { free(f); free(p); free(q); return 1; }                                \
    for (int64_t k = 0; k < P; ++k) {                                                           \
      const int64_t s = k * m, e = (k < P - 1) ? s + m - 1 : N - 1;                             \
      const T xs = z[2 * k], xe = z[2 * k + 1];                                                 \
      x[s] = xs;                                                                                \
      x[e] = xe;                                                                                \
      /* f[j], p[j], q[j] belong to row s+1+j */                                                \
      f[0] = a[s + 1];                                                                          \
      p[0] = b[s + 1];                                                                          \
      q[0] = d[s + 1];                                                                          \
      for (int64_t i = s + 2; i <= e; ++i) {                                                    \
        const int64_t j = i - (s + 1);                                                          \
        T w = a[i] / p[j - 1];                                                                  \
        f[j] = -w * f[j - 1];                                                                   \
        p[j] = b[i] - w * c[i - 1];                                                             \
        q[j] = d[i] - w * q[j - 1];                                                             \
      }                                                                                         \
      for (int64_t i = e - 1; i > s; --i) {                                                     \
        const int64_t j = i - (s + 1);                                                          \
        x[i] = (q[j] - f[j] * xs - c[i] * x[i + 1]) / p[j];                                     \
      }                                                                                         \
    }                                                                                           \
    free(f);                                                                                    \
    free(p);                                                                                    \
    free(q);                                                                                    \
    return 0;                                                                                   \
  }                                                                                             \
                                                                                                \
  /* The recursive method with sizes ms[0..R] (ms[0] = m): Stage 1 on every level from the  \
     top, Thomas on the deepest interface system, Stage 3 on every level from the bottom.    \
     R = -1: the direct solve.  A one-row system is solved directly. */                         \
  int tro_partition_##SUF(int64_t N, int32_t R, const int32_t* ms, const T* a, const T* b,      \
                          const T* c, const T* d, T* x) {                                       \
    if (N == 1 || R < 0) return tro_thomas_##SUF(N, a, b, c, d, x);                             \
    int64_t n[16];                                                                              \
    T* lv[16][5];                                                                               \
    if (R > 14) return 2;                                                                       \
    n[0] = N;                                                                                   \
    for (int l = 0; l <= R; ++l) n[l + 1] = 2 * tro_count(n[l], ms[l]);                         \
    for (int l = 1; l <= R + 1; ++l)                                                            \
      for (int v = 0; v < 5; ++v) {                                                             \
        lv[l][v] = (T*)malloc((size_t)n[l] * sizeof(T));                                        \
        if (!lv[l][v]) return 1;                                                                \
      }                                                                                         \
    lv[0][0] = (T*)a; lv[0][1] = (T*)b; lv[0][2] = (T*)c; lv[0][3] = (T*)d; lv[0][4] = x;     \
    for (int l = 0; l <= R; ++l)                                                                \
      tro_interface_##SUF(n[l], ms[l], lv[l][0], lv[l][1], lv[l][2], lv[l][3], lv[l + 1][0],    \
                          lv[l + 1][1], lv[l + 1][2], lv[l + 1][3]);                            \
    int rc = tro_thomas_##SUF(n[R + 1], lv[R + 1][0], lv[R + 1][1], lv[R + 1][2],               \
                              lv[R + 1][3], lv[R + 1][4]);                                      \
    for (int l = R; l >= 0 && rc == 0; --l)                                                     \
      rc = tro_back_solve_##SUF(n[l], ms[l], lv[l][0], lv[l][1], lv[l][2], lv[l][3],            \
                                lv[l + 1][4], lv[l][4]);                                        \
    for (int l = 1; l <= R + 1; ++l)                                                            \
      for (int v = 0; v < 5; ++v) free(lv[l][v]);                                               \
    return rc;                                                                                  \
  }

TRO_DEFINE(f64, double)
TRO_DEFINE(f32, float)
