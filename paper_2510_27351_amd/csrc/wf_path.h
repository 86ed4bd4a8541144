// Adjoint of the score alone by the argmin path: declarations shared by wf_bwd.hip and
// wf_api.hip (not part of the public ABI).
//
// With no upstream gradient of the table, the routed adjoint of the score is the score's
// upstream value on the cells of the path the forward minimum traced back from the last
// cell (each cell routes its whole value to the one predecessor it selected) and zero on
// every other cell.  The path is found band-parallel:
//  1. the selection recompute also propagates, cell by cell, the exit of the cell's path
//     from its 64-row band: the column of the band above's last row at which the path
//     enters it (-1 if the path leaves the matrix);
//  2. the exits of the band's last row, composed over groups of bands, give every band the
//     column at which the path enters it;
//  3. each band walks its part of the path over the selection bit-planes and writes it
//     over the zeroed gradient.
#pragma once

#include "wf_internal.h"

namespace wf {

// Outputs of the labelled selection recompute.
//   exits  nb * n words: exits[b * n + p] is the exit of the path from cell (last row of
//          band b, column p), b < nb - 1; -1 if the path leaves the matrix; for a split band
//          -2 - ((q - 1) * 64 + r) if the path leaves piece q >= 1 through row r of its entry
//          column q * split - 1 (resolved by caps, possibly through several pieces).
//   caps   nb * kMaxPieces * 64 words: caps[(b * kMaxPieces + q) * 64 + r] = the label of
//          cell (r, c) of band b, with c = (q + 1) * split - 1 for a piece q that another
//          follows and c = n - 1 for the piece of the last band that holds column n - 1.
//   gC, ldgc  the gradient to zero in the same sweep (its loader wave stores zeros over
//          columns [64k, 64k + 64) of the band's rows with every sub-chunk k it stages), or
//          null when a pass of its own zeroes it.
constexpr int kMaxPieces = 4;  // column pieces a band's selection recompute is split into

struct PathLabels {
  int32_t* exits;
  int32_t* caps;
  void* gC;
  int64_t ldgc;
};

// The chase and the walk.  Bands are grouped by S (groups of bands [gS, gS + S) of the
// first nb - 1 bands); F[g * n + p] is where the path entering the last band of group g at
// column p enters the last band of group g - 1.
struct PathArgs {
  const int32_t* exits;
  const int32_t* caps;
  int32_t* F;
  const uint32_t* sel;
  const void* gscore;  // may be null (zero)
  void* gC;
  int64_t ldgc;
  int64_t m, n, split;
  int32_t nb, Ks, S, G;
  int32_t pieces, pad;
};

// Bands per group of the composition: the smallest S with S * S >= nb - 1.
__host__ __device__ inline int32_t path_group_size(int32_t nb) {
  int32_t s = 1;
  while ((int64_t)s * s < (int64_t)nb - 1) ++s;
  return s;
}

// Buffers of the batched path adjoint (a plan's): instance i's exits at word sel_off / 8 of
// 'exits', its captured labels at sel_off / 2 of 'caps' and its group maps at sel_off / 8 of
// 'F' (sel_off: the instance's offset in the selection buffer, whose nb * Ks * 512 words per
// instance bound all three).
struct PathBufs {
  int32_t* exits;
  int32_t* caps;
  int32_t* F;
  int32_t batch;
  int32_t pad;
  int64_t max_cols;  // the largest (G - 1) * n over the instances
};

// Defined in wf_bwd.hip, float (dtype 0) and double (dtype 1).
hipError_t launch_select_path(int dtype, const SelArgs& a, const PathLabels& p, int grid, hipStream_t s);
hipError_t launch_zero(int dtype, void* p, int64_t m, int64_t n, int64_t ld, int grid, hipStream_t s);
hipError_t launch_path(int dtype, const PathArgs& a, hipStream_t s);
// The batch: labelled selection recompute (which also zeroes every instance's gradient),
// composition and walk over the plan's (instance, band) work list.
hipError_t launch_path_batch(int dtype, const BwdBatchArgs& b, const PathBufs& pb, int grid, hipStream_t s);

}  // namespace wf
