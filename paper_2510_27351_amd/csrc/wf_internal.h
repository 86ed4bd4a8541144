// Internal declarations shared by the device kernels and the host runtime of libwf.
// Nothing here is part of the public ABI (include/wf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wf {

// Rows per band: one band is swept by one 64-lane wavefront, lane r owning band row r.
constexpr int kBand = 64;
// Waves of a sweep workgroup: 0 = compute, 1 = input loader, 2 = top-boundary poller,
// 3 = output storer, 4 = boundary publisher.
constexpr int kWaves = 5;
constexpr int kThreads = kWaves * 64;

// Device-resident control block of a workspace.  It resets itself: the last workgroup of a
// launch clears 'claim' and 'done' and advances 'epoch', so a launch needs no host-side
// memset and may be captured in a graph and replayed.
struct Control {
  uint32_t claim;   // next band (or work item) to claim
  uint32_t done;    // workgroups that have finished this launch
  uint32_t epoch;   // tag carried by this launch's handoff words (never 0)
  uint32_t abort;   // set when a bounded wait expires; makes every wait give up
  uint32_t err;     // sticky error bits (kErrTimeout); read and cleared by the host
  uint32_t fault;   // injected fault for tests of the failure path (kFault*), 0 = none
  uint32_t pad[10];
};
constexpr uint32_t kErrTimeout = 1u;
// Injected faults (wf_fault_inject): a band withholds the boundary values another band
// waits for, so that the waiting band's bounded wait expires and the launch aborts.
constexpr uint32_t kFaultFwdWithhold = 1u;  // forward: band 0 publishes no boundary row
constexpr uint32_t kFaultRevWithhold = 2u;  // reverse: the bottom band publishes no routed values

// Arguments of the single-instance forward sweep.
struct FwdArgs {
  const void* C;
  void* D;          // may be null (score-only)
  void* score;
  void* ckpt;       // may be null
  int64_t ldc, ldd;
  int64_t m, n;
  int32_t ckpt_k;   // 0 = no checkpoints
  int32_t nb;       // bands of the sweep = ceil(m / forward_band_rows(dtype))
  Control* ctl;
  uint64_t* bnd;    // (nb-1) * n * words-per-element handoff words (last row of each band)
  uint64_t* trace;  // null, or kTraceWords words per band (see wf_trace_enable)
  // soft-min sweep only: kx = log2(e) / gamma scales C into the base-2 domain the cells run
  // in, gl = gamma ln 2 scales the results back to D
  double kx, gl;
};

// Per-band trace record, written when tracing is enabled (times in ticks of the 100 MHz
// real-time counter):
//   0 claim time        1 first sub-chunk ready   2 compute done     3 store done
//   4 sub-chunks the compute wave found not yet loaded
//   5 sub-chunks whose top row had not yet arrived
//   6 XCC id            7 workgroup id
//   8..11 ticks spent waiting by the compute, loader, top and storer waves
//   12 loader done      13 top done               18 ticks the publisher waited
//   14 time the storer published unit U1 = 62/G + 1, the one unit 0 of the band below needs
//   15 time the poller completed unit 0
//   16 time the compute wave finished unit U1
//   17 time the publisher saw unit U1 finished
//   19..23 reserved
constexpr int kTraceWords = 24;

// Arguments of the selection recompute (first half of the adjoint): every 64-row band is
// swept again from its top row -- a checkpoint row, or a row of the saved table -- and
// emits three bit-planes per band row (W selected, N selected, NW selected; one bit per
// cell).  For band b, 64-slot sub-chunk k (slot = row-in-band + column) and lane r, eight
// 32-bit words at sel[((b * Ks + k) * 64 + r) * 8]: W[0..1], N[0..1], NW[0..1], 0, 0, bit j
// of word h of a plane being slot 64k + 32h + j of row 64b + r; Ks = ceil((n + 63) / 64).
struct SelArgs {
  const void* C;
  const void* top;    // row 64b-1 of band b >= 1 is at top + (b-1) * ld_top
  int64_t ldc, ld_top;
  int64_t m, n;
  int32_t nb;         // 64-row bands
  uint32_t* sel;
  Control* ctl;
  // Column split (split > 0): each band is swept as 'pieces' pieces, columns
  // [p * split, (p + 1) * split) and the last one to n, split a multiple of 64; piece p >= 1
  // starts from column p * split - 1 of the forward table, D[i][p * split - 1] at
  // left + (p - 1) * left_pstride + i * ld_left (elements).
  int64_t split;
  const void* left;
  int64_t ld_left;
  int64_t left_pstride;
  int32_t pieces;
  int32_t pad;
};

// Arguments of the reverse adjoint sweep (second half): bands of 64 rows from the bottom
// up, each from right to left, reading the selection bit-planes and the upstream gradient.
struct AdjArgs {
  const uint32_t* sel;
  const void* gD;       // may be null (zero)
  const void* gscore;   // may be null (zero)
  void* gC;
  int64_t ldgd, ldgc;
  int64_t m, n;
  int32_t nb;           // 64-row bands
  Control* ctl;
  uint64_t* bnd;        // (nb-1) * n * 2 * words-per-element handoff words
  uint64_t* trace;
};

// Ragged batch of instances packed in one buffer.  Instance i is an m x n row-major matrix
// with leading dimension n at element offset 'off' of C (and of D); its handoff words start
// at word bnd_off of the plan's buffer.
struct BatchInst {
  int64_t off;
  int64_t m, n;
  int64_t bnd_off;
  int64_t ck_off;   // element offset of the instance's checkpoint grid (when one is written)
  int32_t nb;       // bands of the instance
  int32_t pad;
};
struct BatchItem {
  int32_t inst;
  int32_t band;
};
struct BatchArgs {
  const void* C;
  void* D;              // may be null (scores only)
  void* scores;         // one element per instance
  void* ckpt;           // may be null: every instance's checkpoint grid, at its ck_off
  int32_t ckpt_k;       // 0 = no checkpoints
  int32_t pad2;
  const BatchInst* inst;
  const BatchItem* items;
  int32_t n_items;
  int32_t pad;
  Control* ctl;
  uint64_t* bnd;
};

// Batched adjoint: instance i's C, D, gD and gC at element offset 'off' (leading dimension
// n), its checkpoint grid at ck_off, its selection bit-planes at word sel_off of the plan's
// selection buffer and its reverse handoff words at word bnd_off.
struct BwdInst {
  int64_t off;
  int64_t m, n;
  int64_t ck_off;
  int64_t sel_off;
  int64_t bnd_off;
  int32_t nb;       // 64-row bands
  int32_t pad;
};
// Work items of the batched adjoint are (instance, band) pairs (BatchItem), ordered from the
// bottom band up: every instance's last band, then every second-to-last band, and so on, so
// that in the reverse sweep a band always follows the band below it.  The selection
// recompute, whose bands are independent, takes the same list.
struct BwdBatchArgs {
  const void* C;
  const void* top;      // the checkpoint grids (ckpt_k > 0) or the saved tables (ckpt_k = 0)
  int32_t ckpt_k;
  int32_t n_items;
  const void* gD;       // may be null (zero)
  const void* gscores;  // one element per instance, or null (zero)
  void* gC;
  const BwdInst* inst;
  const BatchItem* items;
  uint32_t* sel;
  uint64_t* bnd;
  Control* ctl;
};

// Host-side launchers (defined in wf_fwd.hip).  'tile' is 16, 32 or 64.
hipError_t launch_forward(int dtype, int tile, const FwdArgs& a, int grid, hipStream_t s);
// Rows per band of the single-instance forward sweep for a dtype.
int forward_band_rows(int dtype);
// Batch sweep; 'rows' = 64-row sub-bands per band: 1, or 2 for the 4-byte types.
hipError_t launch_forward_batch(int dtype, int tile, int rows, const BatchArgs& b, int grid, hipStream_t s);
// Adjoint launchers (defined in wf_bwd.hip), float (dtype 0) and double (dtype 1) only.
hipError_t launch_select(int dtype, const SelArgs& a, int grid, hipStream_t s);
hipError_t launch_adjoint(int dtype, int tile, const AdjArgs& a, int grid, hipStream_t s);
hipError_t launch_select_batch(int dtype, const BwdBatchArgs& b, int grid, hipStream_t s);
hipError_t launch_adjoint_batch(int dtype, int tile, const BwdBatchArgs& b, int grid, hipStream_t s);

// ---------------------------------------------------------------------------------------
// Host runtime (defined in wf_api.hip).

// Per-device workspace, created on the first call on a device and grown on demand.
struct DeviceWs {
  Control* ctl = nullptr;     // device control block (zeroed, epoch = 1)
  uint64_t* bnd = nullptr;    // tagged handoff words
  size_t bnd_words = 0;
  uint32_t* sel = nullptr;    // selection codes of the adjoint
  size_t sel_words = 0;
  int sel_dtype = -1;         // dtype, m, n of the last selection recompute enqueued
  int64_t sel_m = 0, sel_n = 0;
  int num_cus = 0;
};
// Returns the workspace of device 'dev' with at least 'words' handoff words.
int ensure_ws(int dev, size_t words, DeviceWs** out);
int elem_size(int dtype);       // bytes per element, 0 for an invalid dtype
// Tile of the single-instance sweeps for a shape: the override (wf_set_tile, then WF_TILE),
// else the nearest-neighbour prediction (wf_tile_predict).  dtype, m and n must be valid.
int pick_tile(int dtype, int64_t m, int64_t n, bool reverse);
int words_per_elem(int dtype);  // 32-bit payload words per element in the handoff words

// Largest leading dimension, in bytes: a band of up to 128 rows is addressed with 32-bit
// byte offsets.
constexpr int64_t kMaxLd = ((int64_t)1 << 31) / 128 - 16;

}  // namespace wf
