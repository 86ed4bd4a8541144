// Launch arguments of the smooth (soft-min) sweeps (wf_soft.hip), shared with the host entry
// points (wf_api.hip).  Nothing here is part of the public ABI (include/wf.h).
#pragma once

#include "wf_internal.h"

namespace wf {

// Arguments of the smooth (soft-min) sweeps: the forward writes D (and the score) from C;
// the adjoint reads C and the forward's D (Din) and writes gC.  kx = log2(e) / gamma and
// gl = gamma ln 2 (the soft minimum in base-2 exponentials and logarithms).
struct SoftArgs {
  const void* C;
  const void* Din;
  void* D;
  void* score;
  const void* gD;       // may be null (zero)
  const void* gscore;   // may be null (zero)
  void* gC;
  int64_t ldc, ldd, ldgd, ldgc;
  int64_t m, n;
  int32_t nb;           // 64-row bands
  int32_t pad;
  double kx, gl;
  Control* ctl;
  uint64_t* bnd;        // forward: (nb-1) * n * W words; adjoint: twice that, (A, V) pairs
};
hipError_t launch_soft_forward(int dtype, const SoftArgs& a, int grid, hipStream_t s);
hipError_t launch_soft_backward(int dtype, const SoftArgs& a, int grid, hipStream_t s);

}  // namespace wf
