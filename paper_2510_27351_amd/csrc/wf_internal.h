// Internal declarations shared by the device kernels and the host runtime of libwf.
// Nothing here is part of the public ABI (include/wf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wf {

// Rows per band: one band is swept by one 64-lane wavefront, lane r owning band row r.
constexpr int kBand = 64;
// Waves of a sweep workgroup: 0 = compute, 1 = input loader, 2 = top-boundary poller,
// 3 = output storer / boundary publisher.
constexpr int kWaves = 4;
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
  uint32_t pad[11];
};
constexpr uint32_t kErrTimeout = 1u;

// Arguments of the single-instance forward sweep.
struct FwdArgs {
  const void* C;
  void* D;          // may be null (score-only)
  void* score;
  void* ckpt;       // may be null
  int64_t ldc, ldd;
  int64_t m, n;
  int32_t ckpt_k;   // 0 = no checkpoints
  int32_t nb;       // bands = ceil(m / 64)
  Control* ctl;
  uint64_t* bnd;    // (nb-1) * n * words-per-element handoff words
};

// Host-side launchers (defined in wf_fwd.hip).  'tile' is 16, 32 or 64.
hipError_t launch_forward(int dtype, int tile, const FwdArgs& a, int grid, hipStream_t s);

}  // namespace wf
