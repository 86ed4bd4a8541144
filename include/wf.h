/*
 * wf.h -- C ABI of libwf, the MI355X (gfx950) anti-diagonal wavefront sweep.
 *
 * The operation.  The paper this library accompanies (an arXiv study of sub-system sizes
 * for the GPU tridiagonal partition method) does not state a cell recurrence; its only
 * trace of one is a pair of unused preamble macros (2n-1 anti-diagonals of an n x n grid
 * and a 3 n^2 per-sweep byte count).  The library implements the documented reading "R0"
 * of a west / north / north-west cell recurrence:
 *
 *     D[i][j] = C[i][j] + min( D[i-1][j-1], D[i-1][j], D[i][j-1] ),   0 <= i < m, 0 <= j < n
 *
 * with the virtual boundary D[-1][-1] = 0 and D[-1][j] = D[i][-1] = +inf otherwise (row 0
 * and column 0 are prefix sums).  score = D[m-1][n-1].  Predecessor selection, used by the
 * adjoint, breaks ties in the order NW, N, W.  All m+n-1 anti-diagonals are swept on the
 * device by one persistent kernel; no launch per diagonal.
 *
 * Conventions shared by every entry point:
 *   - Sizes and leading dimensions are in ELEMENTS.  Matrices are row-major.
 *   - Data pointers (C, D, score, ckpt, g_*) are DEVICE pointers owned by the caller; the
 *     library never frees or retains them past the call's stream work.
 *   - 'stream' is a hipStream_t passed as void* (NULL = the legacy default stream).  Every
 *     entry point only enqueues work on 'stream' and returns; there is no host sync on the
 *     hot path.  Results are bitwise reproducible run to run.
 *   - Return value: WF_OK or an error code.  Arguments are validated before any device work;
 *     on an argument error nothing is enqueued.  A device-side failure (a bounded wait that
 *     expired) is reported by wf_last_async_error().
 *   - The library keeps one internal workspace per (device, stream) pair (control block,
 *     handoff words, selections), created on the first call on that stream and grown when a
 *     larger shape arrives (growing allocates and synchronizes the device).  Calls on one
 *     stream are ordered by it; calls on different streams of a device use different
 *     workspaces and may overlap.  A workspace lives until the process ends, keyed by the
 *     stream handle, so a program that creates streams without bound should reuse them.
 *     Plans own their control block; wf_forward_noalloc uses one array per device instead.
 *   - Leading dimensions are limited to (2^31 / 128 - 16) bytes (about 4.2 million float
 *     columns): larger values return WF_E_UNSUPPORTED.
 *   - Element types: WF_F32 (float, one IEEE add per cell, min exact), WF_F64 (double),
 *     WF_I32 (int32; the caller guarantees (m+n-1) * max|C| < 2^31 - 1 so no sum overflows).
 *     Inputs must be free of NaN and -inf; +inf marks a blocked cell.
 */
#ifndef WF_H
#define WF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { WF_F32 = 0, WF_F64 = 1, WF_I32 = 2 } wf_dtype;

enum {
  WF_OK = 0,
  WF_E_ARG = 1,         /* invalid argument (size, pointer, leading dimension, dtype)   */
  WF_E_UNSUPPORTED = 2, /* valid but not supported by this build (e.g. a tile width)    */
  WF_E_NOMEM = 3,       /* device allocation of the internal workspace failed           */
  WF_E_DEVICE = 4,      /* a HIP runtime call failed                                    */
  WF_E_TIMEOUT = 5      /* a bounded device-side wait expired (reported asynchronously) */
};

/*
 * Forward sweep of one m x n instance.
 *   C      [in]  m x n, leading dimension ldc >= n.
 *   D      [out] m x n table, leading dimension ldd >= n; NULL = score-only mode (the table
 *                is never written to memory; the sweep still runs over every cell).
 *   score  [out] one element, D[m-1][n-1].  Required.
 *   ckpt   [out] checkpoint grid for wf_backward, wf_ckpt_elems(m, n, ckpt_k) elements; NULL
 *                when ckpt_k == 0 (and allowed when that count is 0).  Layout: first the band rows -- D[64b+63][0..n-1] for
 *                b = 0 .. ceil(m/64)-2, row after row -- then the block columns --
 *                D[0..m-1][K q - 1] for q = 1 .. ceil(n/K)-1, column after column
 *                (K = ckpt_k).  Rows are every 64 because the device sweep works on bands of
 *                64 rows; K sets the column spacing.
 *   ckpt_k      column spacing K of the checkpoint grid, 0 = no checkpoints, else 1..4096.
 * Element type of every buffer is 'dtype'.
 */
int wf_forward(int dtype, int64_t m, int64_t n, const void* C, int64_t ldc, void* D,
               int64_t ldd, void* score, void* ckpt, int32_t ckpt_k, void* stream);

/*
 * wf_forward for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments, checks and results
 * as wf_forward; it calls no allocating routine.  Its launch control block and handoff words
 * live in a fixed 32 MiB device array of the library (one copy per GPU, held until the
 * process ends) instead of the growable workspace, so the shapes it takes are bounded:
 * (bands - 1) * n * w <= 4194272 handoff words, with bands = ceil(m / 64) and w = 2 for
 * WF_F64, else 1 (16384 x 16384 float32 fits, 16384 x 16384 float64 does not); larger shapes
 * return WF_E_UNSUPPORTED before any device work.  A one-thread preparation kernel runs before
 * the sweep on 'stream'.  Every call on a GPU shares that GPU's array: calls that overlap on
 * one GPU (streams not ordered with each other) race on it and must not be issued; calls
 * ordered on one stream are fine, eager or captured.  A bounded wait that expires is reported
 * by wf_last_async_error, as for wf_forward.
 */
int wf_forward_noalloc(int dtype, int64_t m, int64_t n, const void* C, int64_t ldc, void* D,
                       int64_t ldd, void* score, void* ckpt, int32_t ckpt_k, void* stream);

/* Number of elements of the checkpoint grid written by wf_forward (0 when ckpt_k == 0, or
 * -1 on invalid sizes). */
int64_t wf_ckpt_elems(int64_t m, int64_t n, int32_t ckpt_k);

/*
 * Adjoint sweep: writes g_C = dL/dC for  L = sum(g_D * D) + g_score * score, where D and
 * score are the forward results for C.  The derivative is the routed (sub)gradient of the
 * min: each cell passes its adjoint to the one predecessor it selected (ties NW, N, W), so
 * A[i][j] = g_D[i][j] + [i=m-1, j=n-1] g_score + [SEL(i+1,j+1)=NW] A[i+1][j+1]
 *         + [SEL(i+1,j)=N] A[i+1][j] + [SEL(i,j+1)=W] A[i][j+1]   (summed in that order)
 * and g_C = A.  The selections are recomputed on the device from the input and either the
 * checkpoint grid of wf_forward (its band rows; pass ckpt_k > 0 and D = NULL) or the saved
 * table D (pass ckpt = NULL, ckpt_k = 0).
 *   dtype       WF_F32 or WF_F64 (WF_I32 returns WF_E_UNSUPPORTED).
 *   C, ldc      the forward input, m x n.
 *   ckpt, ckpt_k  the checkpoint grid and K of the forward call, or NULL / 0 (ckpt may be
 *               NULL with ckpt_k > 0 when the grid is empty, i.e. m <= 64 and n <= K).
 *   D, ldd      the forward table, or NULL.
 *   g_score     one element, or NULL for 0.
 *   g_D, ldgd   m x n upstream gradient of the table, or NULL for 0.
 *   g_C, ldgc   m x n output.
 * With g_D given, the selections are recomputed and the reverse sweep runs band by band from
 * the bottom up (wf_select then wf_reverse); g_D and g_score must then be finite (and the
 * sums must not overflow): the pipeline forms every routed term as a 0/1 factor times the
 * successor's value, so an infinite or NaN value would also reach, as NaN, the cells its
 * cell did not select.  With g_D = NULL the adjoint is g_score on the
 * cells of the argmin path traced back from cell (m-1, n-1) and exactly zero elsewhere (each
 * value being 0 + g_score, the same in any summation order), and it is computed that way:
 * the selection recompute also labels every cell with the exit of its path from its 64-row
 * band, the labels of the bands' last rows are composed over groups of bands, and each band
 * writes its part of the path (g_C is zeroed first, so g_score = NaN or +-inf reaches the
 * path cells only).  The selections are left in the stream's workspace either way, so a
 * wf_reverse may follow.
 * Uses (and grows) the stream's workspace: 4 bits per cell for the selections (three
 * bit-planes and padding), plus handoff words (g_D given) or one 32-bit exit per column of
 * every band's last row (g_D = NULL).  Results are bitwise reproducible; in float the sums
 * round once per term in the order above.
 */
int wf_backward(int dtype, int64_t m, int64_t n, const void* C, int64_t ldc, const void* ckpt,
                int32_t ckpt_k, const void* D, int64_t ldd, const void* g_score, const void* g_D,
                int64_t ldgd, void* g_C, int64_t ldgc, void* stream);

/*
 * The two halves of the reverse pipeline, for callers that time or schedule them separately
 * (wf_backward with g_D given is exactly wf_select followed by wf_reverse on the same stream;
 * with g_D = NULL and a finite g_score wf_reverse gives the same g_C as wf_backward).
 * wf_select recomputes the predecessor selections of an m x n forward sweep (arguments as
 * for wf_backward) into the workspace of (current device, 'stream'); wf_reverse runs the
 * reverse sweep from them and writes g_C.  wf_reverse must be given the stream of its
 * wf_select: it returns WF_E_ARG unless the last wf_select enqueued on that stream of this
 * device was for the same dtype, m and n (a workspace holds one set of selections).
 */
int wf_select(int dtype, int64_t m, int64_t n, const void* C, int64_t ldc, const void* ckpt,
              int32_t ckpt_k, const void* D, int64_t ldd, void* stream);
int wf_reverse(int dtype, int64_t m, int64_t n, const void* g_score, const void* g_D, int64_t ldgd,
               void* g_C, int64_t ldgc, void* stream);

/*
 * Ragged batch.  A plan describes a batch of independent instances of different sizes
 * (instance i: m[i] x n[i], row-major with leading dimension n[i], at element offset
 * offsets[i] of one buffer) and owns a device work list of (instance, band) items.
 * wf_batch_forward sweeps every instance with ONE persistent launch; the launch is
 * captured in a hipGraph the first time it is called with a given (C, D, scores) and the
 * graph is replayed on later calls with the same pointers (other pointers re-capture,
 * which synchronizes the device once).  Inside a stream capture of the caller's own the
 * launch is recorded into the caller's graph instead.
 *
 * wf_plan_create(plan, dtype, batch, m, n, offsets, tile, rows, stream)
 *   m, n       HOST arrays of 'batch' sizes (each >= 1).
 *   offsets    HOST array of element offsets (instances must not overlap), or NULL to pack
 *              the instances in order with 256-byte aligned starts (wf_plan_offsets
 *              returns them).
 *   tile       columns per handoff unit, 16/32/64, or 0 to autotune.
 *   rows       64-row tiles held by one workgroup at a time (rows per band / 64): 1, 2
 *              (not for WF_F64), or 0 to autotune.
 *   stream     used by the autotuner.  Autotuning times every allowed (tile, rows) on
 *              scratch buffers of the batch's size (allocated and freed inside the call,
 *              which synchronizes 'stream'); results are cached per process and, if the
 *              environment variable WF_TUNE_CACHE names a file, in that file.
 *   Creates the plan (host and device memory owned by the library until
 *   wf_plan_destroy).  Returns WF_E_ARG for invalid sizes or overlapping offsets.
 * wf_plan_elems    number of elements the C (and D) buffer must hold, -1 for NULL.
 * wf_plan_offsets  copies the batch's element offsets into a host array of 'batch'.
 * wf_plan_config   the (tile, rows) the plan uses.
 * wf_batch_forward(plan, C, D, scores, stream)
 *   C       [in]  device buffer of wf_plan_elems elements holding every instance.
 *   D       [out] same layout as C, every instance's table; NULL = scores only.
 *   scores  [out] 'batch' elements, D_i[m_i-1][n_i-1].
 *   The plan's device of creation must be current.  Calls on one plan must be ordered (its
 *   control block and buffers are its own); different plans may run on different streams.
 * wf_plan_destroy  synchronizes the device and frees the plan (NULL is ignored).
 */
typedef struct wf_plan wf_plan;
int wf_plan_create(wf_plan** plan, int dtype, int32_t batch, const int64_t* m, const int64_t* n,
                   const int64_t* offsets, int32_t tile, int32_t rows, void* stream);
int64_t wf_plan_elems(const wf_plan* plan);
int wf_plan_offsets(const wf_plan* plan, int64_t* offsets);
int wf_plan_config(const wf_plan* plan, int32_t* tile, int32_t* rows);
int wf_batch_forward(wf_plan* plan, const void* C, void* D, void* scores, void* stream);
void wf_plan_destroy(wf_plan* plan);

/*
 * Differentiable ragged batch: the forward with checkpoint grids, and the batched adjoint.
 *
 * wf_plan_ckpt_elems(plan, K)   elements of the buffer holding every instance's checkpoint
 *                               grid for column spacing K (1..4096; 0 gives 0): instance i's
 *                               grid (wf_ckpt_elems(m_i, n_i, K) elements, layout as for
 *                               wf_forward) starts at element offset o_i, the grids packed in
 *                               instance order with 256-byte aligned starts; -1 on bad input.
 * wf_plan_ckpt_offsets(plan, K, offsets)  copies the o_i into a host array of 'batch'.
 * wf_batch_forward_ckpt(plan, C, D, scores, ckpt, ckpt_k, stream)
 *   wf_batch_forward that also writes every instance's checkpoint grid into 'ckpt'
 *   (wf_plan_ckpt_elems(plan, ckpt_k) elements; NULL with ckpt_k = 0 for none).  The first
 *   call with a new K rebuilds the plan's instance table (synchronizes the device); the
 *   captured graph is keyed on (C, D, scores, ckpt) as for wf_batch_forward.
 * wf_batch_backward(plan, C, ckpt, ckpt_k, D, g_scores, g_D, g_C, stream)
 *   For every instance i, g_C_i = dL/dC_i for L = sum_i (sum(g_D_i * D_i) + g_scores[i] *
 *   score_i), the routed adjoint of wf_backward, in two launches over all instances: the
 *   selection recompute (every 64-row band of every instance at once) and one persistent
 *   reverse sweep over a bottom-up (instance, band) work list.
 *   C, D, g_D, g_C  device buffers in the plan's layout (wf_plan_elems elements; D and g_D may
 *                   be NULL); the selections are recomputed from C and either the checkpoint
 *                   grids of wf_batch_forward_ckpt (ckpt, ckpt_k > 0, D = NULL) or the saved
 *                   tables (D, ckpt = NULL, ckpt_k = 0).
 *   g_scores        'batch' elements, or NULL for 0.
 *   WF_F32 and WF_F64 plans only (WF_E_UNSUPPORTED otherwise).  The first call allocates the
 *   plan's selection bit-planes (4 bits per cell) and handoff words and synchronizes the
 *   device; a call with another K than the previous one synchronizes it too.  Calls on one
 *   plan must be ordered (the plan holds one set of selections).  Bitwise reproducible; each
 *   instance's g_C equals wf_backward's on that instance.
 */
int64_t wf_plan_ckpt_elems(const wf_plan* plan, int32_t ckpt_k);
int wf_plan_ckpt_offsets(const wf_plan* plan, int32_t ckpt_k, int64_t* offsets);
int wf_batch_forward_ckpt(wf_plan* plan, const void* C, void* D, void* scores, void* ckpt, int32_t ckpt_k,
                          void* stream);
int wf_batch_backward(wf_plan* plan, const void* C, const void* ckpt, int32_t ckpt_k, const void* D,
                      const void* g_scores, const void* g_D, void* g_C, void* stream);

/*
 * Force the tile width (columns per handoff unit, 64 rows per band) used by later calls on
 * this process: 16, 32 or 64, or 0 to return to the automatic choice (wf_tile_predict).
 * Returns WF_E_ARG for any other value.  Used by the autotuner and the tests.
 */
int wf_set_tile(int32_t tile);

/*
 * The automatic choice: the tile G (16, 32 or 64) that wf_forward (reverse = 0) or
 * wf_reverse / wf_backward (reverse = 1) use for an m x n instance of element type dtype,
 * by nearest-neighbour classification (k = 1, as the paper's kNN heuristic for its
 * sub-system size in the section "Building a heuristic for the optimum sub-system size"):
 * the fastest tile of the closest shape, in (log2 m, log2 n), of a table of shapes timed on
 * MI355X in float32 and in float64 (ties go to the earlier table row; WF_I32 uses the
 * float32 forward column).  Host-only, needs no device.  Returns the tile, or an error code
 * (all error codes are below 16): WF_E_ARG if dtype is not a wf_dtype, m < 1, n < 1 or
 * reverse is not 0 or 1; WF_E_UNSUPPORTED for WF_I32 with reverse = 1 (there is no integer
 * adjoint).
 */
int32_t wf_tile_predict(int32_t dtype, int64_t m, int64_t n, int32_t reverse);

/*
 * Tracing (for profiling the pipeline, off by default).  wf_trace_enable(B) allocates a
 * device buffer of B records on the current device; later forward calls and reverse sweeps
 * of wf_backward on that device whose band count is <= B fill record b for band b (a later
 * call overwrites earlier records).  wf_trace_enable(0) frees it.  wf_trace_fetch synchronizes the device and
 * copies up to max_bands records (8 uint64 each: claim time, first sub-chunk ready,
 * compute done, store done -- 100 MHz ticks --, sub-chunks the compute wave found not yet
 * loaded, sub-chunks whose top row had not yet arrived, XCC id, workgroup id) into 'host';
 * it returns the number of records copied, or minus an error code.
 */
int wf_trace_enable(int64_t max_bands);
int64_t wf_trace_fetch(uint64_t* host, int64_t max_bands);

/*
 * Synchronizes 'stream', then reports and clears the device-side error state of every
 * control block of the current device (the workspaces of all its streams, its plans and the
 * allocation-free array): WF_OK, or WF_E_TIMEOUT if a bounded wait expired in any call since
 * the last check (the outputs of such a call are undefined).  Work still running on other
 * streams is not waited for: synchronize them first to have their errors included.
 */
int wf_last_async_error(void* stream);

/*
 * Fault injection, for tests of the failure path only.  Sets the mode of every control block
 * of the current device (all streams, plans, the allocation-free array, and those created
 * later) for every later sweep on that device until it is set back to 0:
 *   0  no fault (the default);
 *   1  in wf_forward (and the ragged batch), band 0 publishes no boundary row: the band below
 *      waits until its bounded wait (2 s) expires, raises WF_E_TIMEOUT and every workgroup of
 *      the launch gives up and exits;
 *   2  in the reverse sweep (wf_reverse / wf_backward), the bottom band publishes no routed
 *      values, with the same effect.
 * Outputs of a sweep that timed out are undefined; wf_last_async_error reports WF_E_TIMEOUT
 * once, and later sweeps run normally.  Synchronizes the device.  Returns WF_E_ARG for any
 * other mode.
 */
int wf_fault_inject(int32_t mode);

/*
 * Smooth variant of the recurrence: the minimum replaced by the soft minimum of temperature
 * gamma > 0,
 *     D[i][j] = C[i][j] - gamma log( exp(-D[i-1][j-1]/gamma) + exp(-D[i-1][j]/gamma)
 *                                    + exp(-D[i][j-1]/gamma) ),
 * same boundary as above (the soft dynamic-time-warping recursion; gamma -> 0 gives the
 * min-plus table).  D[i][j] is -gamma log of the sum over all monotone paths from (0,0) to
 * (i,j) of exp(-path cost/gamma), so the table is smooth in C and its gradient is exact
 * (no selections, no ties).  C must be finite.  WF_F32 or WF_F64; the exponentials and
 * logarithms are the device's base-2 functions, so results agree with a float64 evaluation
 * to within rounding, not bit for bit.
 *
 * wf_soft_forward writes the full table D (m x n, ldd >= n; required, the adjoint reads it)
 * and score = D[m-1][n-1].
 * wf_soft_backward writes g_C = dL/dC for L = sum(g_D * D) + g_score * score from C and the
 * forward's D:
 *     A[i][j] = g_D[i][j] + [i=m-1, j=n-1] g_score + w(i+1,j+1) A[i+1][j+1]
 *             + w(i+1,j) A[i+1][j] + w(i,j+1) A[i][j+1],  g_C = A,
 * with w(s) = exp((D(s) - C(s) - D[i][j]) / gamma) the derivative of successor s's soft
 * minimum with respect to D[i][j].  g_score (one element) and g_D may be NULL (= 0).
 * Both are persistent band pipelines on the device workspace like wf_forward (same stream
 * ordering rules, bounded waits reported by wf_last_async_error).  gamma must be positive
 * and finite (WF_E_ARG otherwise); WF_I32 returns WF_E_UNSUPPORTED.
 */
int wf_soft_forward(int dtype, int64_t m, int64_t n, double gamma, const void* C, int64_t ldc,
                    void* D, int64_t ldd, void* score, void* stream);
int wf_soft_backward(int dtype, int64_t m, int64_t n, double gamma, const void* C, int64_t ldc,
                     const void* D, int64_t ldd, const void* g_score, const void* g_D,
                     int64_t ldgd, void* g_C, int64_t ldgc, void* stream);

/* Static, human-readable name of an error code. */
const char* wf_error_string(int code);

/* Library version (major*10000 + minor*100 + patch). */
int wf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WF_H */
