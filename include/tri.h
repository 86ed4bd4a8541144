/*
 * tri.h -- C ABI of the tridiagonal partition solver in libwf (MI355X, gfx950).
 *
 * The operation (the paper's Introduction and its section on the recursive method).  A
 * system A x = d with a tridiagonal coefficient matrix A of N unknowns is solved by the
 * parallel partition method:
 *
 *   Stage 1  the rows are cut into sub-systems of m unknowns; each sub-system is reduced,
 *            independently, to two interface equations in its first and last unknowns;
 *   Stage 2  the interface equations form a tridiagonal interface system of 2P unknowns
 *            (P sub-systems), which is solved -- directly, or by applying the method to it
 *            again (one "recursive step"), R times in all, with sub-system sizes
 *            m_1 .. m_R on the successive interface systems;
 *   Stage 3  with the interface unknowns known, every sub-system's remaining unknowns are an
 *            independent tridiagonal system, solved in parallel.
 *
 * The paper runs Stage 2 on the host.  Here every stage runs on the device: the deepest
 * interface system is solved by the Thomas algorithm (Gaussian elimination restricted to
 * the three diagonals, no pivoting) by one lane per system, staged through LDS.  Nothing
 * crosses PCIe.
 *
 * Storage (the paper states none).  A system is four arrays of N elements: a (sub-diagonal,
 * a[0] unused), b (main diagonal), c (super-diagonal, c[N-1] unused) and the right-hand side
 * d; row i reads a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i].  A batch of systems of one
 * size is packed: system s occupies elements [s N, (s+1) N) of every array.
 *
 * Partition of N rows into sub-systems of m rows: P = ceil(N / m) sub-systems, all of m rows
 * but the last, which holds the N - (P-1) m rows left over; a last sub-system of a single
 * row joins the one before it (it could not own two interface unknowns), so the last one
 * has 2 .. m+1 rows.  Needs N >= 2 and m >= 2.  Interface unknowns of sub-system k (rows
 * s .. e) are z[2k] = x[s] and z[2k+1] = x[e]; interface row 2k is the sub-system's rows
 * eliminated upward onto row s, row 2k+1 its rows eliminated downward onto row e.
 *
 * Conventions: as in wf.h.  Data pointers are DEVICE pointers owned by the caller, sizes are
 * in elements, 'stream' is a hipStream_t as void*, every call only enqueues work (no host
 * synchronisation), arguments are validated before any device work, and the return value is
 * WF_OK or one of the WF_E_* codes of wf.h.  Element types: WF_F32, WF_F64.  No pivoting:
 * the method, like the paper's, assumes systems for which elimination without pivoting is
 * stable (diagonally dominant ones); a zero pivot yields inf/NaN in the result, it is not
 * reported.
 */
#ifndef TRI_H
#define TRI_H

#include <stddef.h>
#include <stdint.h>

#include "wf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Deepest recursion supported by a plan. */
#define TRI_MAX_R 6

/*
 * Stage 1 alone: the interface systems of 'batch' packed systems of N unknowns cut into
 * sub-systems of m rows.
 *   a, b, c, d      [in]  batch * N elements each.
 *   A, B, C, D      [out] batch * 2P elements each (P = tri_subsystems(N, m)): the interface
 *                         system of every system, packed with stride 2P; A[0] and C[2P-1]
 *                         of each system are written as 0.
 * Returns WF_E_ARG for batch < 1, N < 2, m < 2, a NULL pointer or an invalid dtype, and
 * WF_E_UNSUPPORTED when m exceeds the largest sub-system a workgroup can hold in LDS
 * (2048 rows in float64, 4096 in float32).
 */
int tri_stage1(int dtype, int32_t batch, int64_t N, int32_t m, const void* a, const void* b,
               const void* c, const void* d, void* A, void* B, void* C, void* D, void* stream);

/*
 * Stage 3 alone: with the interface unknowns z (batch * 2P elements, z[2k] = x at the first
 * row and z[2k+1] = x at the last row of sub-system k of each system) known, solves every
 * sub-system's interior rows and writes the whole solution x (batch * N elements; the
 * interface rows receive the z values).  Same argument checks as tri_stage1.
 */
int tri_stage3(int dtype, int32_t batch, int64_t N, int32_t m, const void* a, const void* b,
               const void* c, const void* d, const void* z, void* x, void* stream);

/*
 * Direct solve (the Stage 2 solver of the deepest level): x = A^-1 d for 'batch' packed
 * systems of n unknowns by the Thomas algorithm, one workgroup per system, the system staged
 * through LDS in chunks while one lane runs the elimination and the back substitution.
 *   scratch  [tmp]  2 * batch * n elements of device memory for the eliminated
 *                   super-diagonal and right-hand side (caller-owned; contents undefined
 *                   on return).
 * n >= 1.
 */
int tri_thomas(int dtype, int32_t batch, int64_t n, const void* a, const void* b, const void* c,
               const void* d, void* x, void* scratch, void* stream);

/* Number of sub-systems of N rows cut into sub-systems of m rows (the partition above), or
 * -1 for N < 2 or m < 2. */
int64_t tri_subsystems(int64_t N, int32_t m);

/*
 * Plan of the full solver for 'batch' systems of N unknowns: sub-system size m of the
 * given system and m_1 .. m_R of the R recursive steps.
 *   m        0 = predicted for N (tri_predict), else >= 2.
 *   R        -1 = predicted for N, else 0 .. TRI_MAX_R.
 *   ms       NULL = the rule of tri_predict for the given (or predicted) m and R, else R
 *            sizes >= 2.
 * N = 1 is allowed (the plan is then a direct solve).  The plan owns device memory for the
 * interface systems of every level and the Thomas scratch (allocated here, synchronously);
 * tri_solve allocates nothing, so it may be captured in a graph.
 */
typedef struct tri_plan tri_plan;
int tri_plan_create(tri_plan** plan, int dtype, int32_t batch, int64_t N, int32_t m, int32_t R,
                    const int32_t* ms);
/* The plan's choice: m, R, ms[0..R-1] (ms may be NULL; else room for TRI_MAX_R entries) and
 * the size of every level's system, sizes[0] = N .. sizes[R+1] = the deepest interface
 * system (sizes may be NULL; else room for TRI_MAX_R + 2 entries).  For N = 1, R = -1 and
 * sizes[0] = 1. */
int tri_plan_config(const tri_plan* plan, int32_t* m, int32_t* R, int32_t* ms, int64_t* sizes);
/* Solves the plan's batch: x = A^-1 d.  All four inputs are read only; x may not alias
 * them.  Stage 1 on every level from the top, the Thomas solve of the deepest interface
 * system, Stage 3 on every level from the bottom: 2R + 3 kernel launches on 'stream'.
 * Calls with one plan on overlapping streams race on its interface buffers. */
int tri_solve(const tri_plan* plan, const void* a, const void* b, const void* c, const void* d,
              void* x, void* stream);
/* Copies level l's interface system (1 <= l <= R+1; the arrays of tri_stage1's output for
 * level l-1) of the LAST tri_solve into A, B, C, D (device pointers, batch * sizes[l]
 * elements each), on 'stream'. */
int tri_plan_level(const tri_plan* plan, int32_t level, void* A, void* B, void* C, void* D,
                   void* stream);
void tri_plan_destroy(tri_plan* plan);

/*
 * Sub-system size and recursion depth for a system of N unknowns, predicted by the
 * nearest-neighbour rule the paper fits to measured optima (k = 1 on the system size):
 *   m   the measured-fastest m of the nearest timed N;
 *   R   the measured-fastest R of the nearest timed N;
 *   ms  (room for TRI_MAX_R entries, may be NULL) the paper's rule for the recursive steps:
 *       m_1 = the predicted m of the first interface system's size when R = 1, else 10;
 *       m_l (l >= 2) = the predicted m of the l-th interface system's size.
 * The tables were timed on one MI355X (float64 and float32 columns).
 */
int tri_predict(int dtype, int64_t N, int32_t* m, int32_t* R, int32_t* ms);

#ifdef __cplusplus
}
#endif

#endif /* TRI_H */
