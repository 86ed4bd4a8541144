// Launch arguments of the smooth (soft-min) sweeps (wf_soft.hip), shared with the host entry
// points (wf_api.hip).  Nothing here is part of the public ABI (include/wf.h).
#pragma once

#include "wf_internal.h"

namespace wf {

// Arguments of the smooth (soft-min) adjoint: it reads C and the forward's D (Din) and
// writes gC.  (The forward takes the min-plus forward's FwdArgs.)  kx = log2(e) / gamma (the
// weights as base-2 exponentials).
struct SoftArgs {
  const void* C;
  const void* Din;
  const void* gD;       // may be null (zero)
  const void* gscore;   // may be null (zero)
  void* gC;
  int64_t ldc, ldd, ldgd, ldgc;
  int64_t m, n;
  int32_t nb;           // 64-row bands
  int32_t pad;
  double kx;
  Control* ctl;
  uint64_t* bnd;        // adjoint: (nb-1) * n * 3 * W words, (A, D, C) per column
};
hipError_t launch_soft_backward(int dtype, const SoftArgs& a, int grid, hipStream_t s);
// The soft-min forward runs in the min-plus forward's band pipeline (wf_fwd.hip) with the
// soft-min cell: a.kx, a.gl set, no checkpoint grid.
hipError_t launch_forward_soft(int dtype, const FwdArgs& a, int grid, hipStream_t s);

// Base-2 exponential and logarithm of the soft minimum, and the adjoint's fused multiply-add,
// all in the element type.  float: the hardware functions (v_exp_f32, v_log_f32, about one
// ulp); the logarithm's argument is a sum in [1, 3] and an exponential that would be
// subnormal (a weight below 2^-126) reads as 0, which changes no sum it enters.
template <typename T>
struct SoftMath;
template <>
struct SoftMath<float> {
  __device__ static __forceinline__ float exp2_(float x) { return __builtin_amdgcn_exp2f(x); }
  __device__ static __forceinline__ float log2_(float x) { return __builtin_amdgcn_logf(x); }
  __device__ static __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
};
template <>
struct SoftMath<double> {
  __device__ static __forceinline__ double exp2_(double x) { return exp2(x); }
  __device__ static __forceinline__ double log2_(double x) { return log2(x); }
  __device__ static __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
};

// One cell in the scaled domain y = D log2(e) / gamma: the soft minimum of the scaled
// neighbours is ymn - log2(sum_k 2^(ymn - y_k)) with ymn their minimum, and the cell's value
// adds the scaled input yc.  Three inputs of +inf (the padding lanes before column 0) give
// +inf, not NaN.
template <typename T>
__device__ __forceinline__ T soft_cell(T yc, T ynw, T yn, T yw) {
  using M = SoftMath<T>;
  const T inf = __builtin_inf();
  const T ymn = ynw < yn ? (ynw < yw ? ynw : yw) : (yn < yw ? yn : yw);
  T s;
  if constexpr (sizeof(T) == 4) {
    // ordered as min <= median <= max, the minimum's term is exactly 1: two exponentials
    const T ymd = __builtin_amdgcn_fmed3f(ynw, yn, yw);
    const T ymx = __builtin_fmaxf(__builtin_fmaxf(ynw, yn), yw);
    s = (T)1 + M::exp2_(ymn - ymd) + M::exp2_(ymn - ymx);
  } else {
    s = M::exp2_(ymn - ynw) + M::exp2_(ymn - yn) + M::exp2_(ymn - yw);
  }
  const T y = yc + (ymn - M::log2_(s));
  return ymn < inf ? y : inf;
}

}  // namespace wf
