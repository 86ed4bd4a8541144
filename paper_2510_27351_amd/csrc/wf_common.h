// Device-side building blocks shared by the libwf sweep kernels (gfx950, wave64).
//
// Cell operation (reading R0 of the west / north / north-west recurrence; the paper states
// no recurrence, see include/wf.h):  D = C + min(NW, N, W).  The min is exact in every
// element type, and the float/double add rounds once, so any schedule reproduces the
// row-by-row result value for value.
#pragma once

#include "wf_internal.h"

namespace wf {

// ---------------------------------------------------------------------------------------
// Element traits.  'W' is the number of 32-bit payload words per element in the tagged
// handoff words; RING is the per-row length (in elements) of the LDS ring of a band and
// PITCH its row pitch, chosen so that the byte pitch is 16 mod 256: a 16-byte read by each
// lane of a different row then hits distinct LDS banks.
// ---------------------------------------------------------------------------------------
template <typename T>
struct Elem;

__device__ __forceinline__ uint32_t dpp_shr1_u32(uint32_t src, uint32_t old) {
  // wave_shr:1 -- lane r receives lane r-1's value; lane 0 keeps 'old' (bound_ctrl off).
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t dpp_shr1z_u32(uint32_t src) {
  // wave_shr:1 with bound_ctrl: lane 0 reads zero.  Feeding an add, the move folds into a
  // DPP add.
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)src, 0x138, 0xf, 0xf, true);
}

template <>
struct Elem<float> {
  static constexpr int W = 1;
  static constexpr int RING = 512;
  static constexpr int PITCH = RING + 4;
  __device__ static __forceinline__ float inf() { return __builtin_inff(); }
  __device__ static __forceinline__ float zero() { return 0.0f; }
  __device__ static __forceinline__ float shr1(float src, float old) {
    return __builtin_bit_cast(float, dpp_shr1_u32(__builtin_bit_cast(uint32_t, src),
                                                  __builtin_bit_cast(uint32_t, old)));
  }
  __device__ static __forceinline__ float shr1z(float src) {
    return __builtin_bit_cast(float, dpp_shr1z_u32(__builtin_bit_cast(uint32_t, src)));
  }
  __device__ static __forceinline__ float min3(float a, float b, float c) {
    return __builtin_fminf(__builtin_fminf(a, b), c);
  }
  // v_min3 on operands the compiler cannot prove canonical (DPP-shifted ones): fminf would
  // quieten each with an extra instruction first.  Inputs hold no NaN.
  __device__ static __forceinline__ float min3v(float a, float b, float c) {
    float r;
    asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
  }
  __device__ static __forceinline__ float min2(float a, float b) { return __builtin_fminf(a, b); }
  __device__ static __forceinline__ float add(float c, float v) { return c + v; }
  __device__ static __forceinline__ uint32_t word(float x, int) { return __builtin_bit_cast(uint32_t, x); }
  __device__ static __forceinline__ float from_words(const uint32_t* w) { return __builtin_bit_cast(float, w[0]); }
};

template <>
struct Elem<int32_t> {
  static constexpr int W = 1;
  static constexpr int RING = 512;
  static constexpr int PITCH = RING + 4;
  __device__ static __forceinline__ int32_t inf() { return 0x7fffffff; }
  __device__ static __forceinline__ int32_t zero() { return 0; }
  __device__ static __forceinline__ int32_t shr1(int32_t src, int32_t old) {
    return (int32_t)dpp_shr1_u32((uint32_t)src, (uint32_t)old);
  }
  __device__ static __forceinline__ int32_t shr1z(int32_t src) { return (int32_t)dpp_shr1z_u32((uint32_t)src); }
  __device__ static __forceinline__ int32_t min3(int32_t a, int32_t b, int32_t c) {
    int32_t x = a < b ? a : b;
    return x < c ? x : c;
  }
  __device__ static __forceinline__ int32_t min2(int32_t a, int32_t b) { return a < b ? a : b; }
  __device__ static __forceinline__ int32_t min3v(int32_t a, int32_t b, int32_t c) { return min3(a, b, c); }
  // Saturating, so that +inf (INT32_MAX) stays +inf on the virtual border; real cells
  // never saturate under the documented bound on |C|.
  __device__ static __forceinline__ int32_t add(int32_t c, int32_t v) { return __builtin_elementwise_add_sat(c, v); }
  __device__ static __forceinline__ uint32_t word(int32_t x, int) { return (uint32_t)x; }
  __device__ static __forceinline__ int32_t from_words(const uint32_t* w) { return (int32_t)w[0]; }
};

template <>
struct Elem<double> {
  static constexpr int W = 2;
  static constexpr int RING = 256;
  static constexpr int PITCH = RING + 2;
  __device__ static __forceinline__ double inf() { return __builtin_inf(); }
  __device__ static __forceinline__ double zero() { return 0.0; }
  __device__ static __forceinline__ double shr1(double src, double old) {
    uint64_t s = __builtin_bit_cast(uint64_t, src), o = __builtin_bit_cast(uint64_t, old);
    uint32_t lo = dpp_shr1_u32((uint32_t)s, (uint32_t)o);
    uint32_t hi = dpp_shr1_u32((uint32_t)(s >> 32), (uint32_t)(o >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  }
  __device__ static __forceinline__ double shr1z(double src) {
    const uint64_t s = __builtin_bit_cast(uint64_t, src);
    const uint32_t lo = dpp_shr1z_u32((uint32_t)s), hi = dpp_shr1z_u32((uint32_t)(s >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  }
  __device__ static __forceinline__ double min3(double a, double b, double c) {
    return __builtin_fmin(__builtin_fmin(a, b), c);
  }
  __device__ static __forceinline__ double min2(double a, double b) { return __builtin_fmin(a, b); }
  __device__ static __forceinline__ double min3v(double a, double b, double c) { return min3(a, b, c); }
  __device__ static __forceinline__ double add(double c, double v) { return c + v; }
  __device__ static __forceinline__ uint32_t word(double x, int k) {
    uint64_t b = __builtin_bit_cast(uint64_t, x);
    return k == 0 ? (uint32_t)b : (uint32_t)(b >> 32);
  }
  __device__ static __forceinline__ double from_words(const uint32_t* w) {
    return __builtin_bit_cast(double, ((uint64_t)w[1] << 32) | w[0]);
  }
};

// Value of lane 'l' (wave-uniform) in every lane.
template <typename T>
__device__ __forceinline__ T lane_value(T x, int l) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

// Four consecutive elements, as moved by one 16-byte (float/int) or two 16-byte (double)
// LDS accesses.
template <typename T>
struct alignas(16) Vec4 {
  T v[4];
};

// ---------------------------------------------------------------------------------------
// Synchronisation helpers.
//
// Inside a workgroup the four waves hand sub-chunks to each other through LDS counters: a
// producer writes its data to LDS, waits for those writes (lgkmcnt) and then stores the
// counter; a consumer spins on the counter.  Nothing here waits on global-memory counters,
// so the loader's prefetches stay in flight.
//
// Between workgroups, boundary values travel as 64-bit words (32 payload bits, 32 tag
// bits) stored and loaded with agent-scope relaxed atomics; a word is valid when its tag
// equals the launch epoch.  Each word validates itself, so no fences and no flag ordering
// are needed, and a stale word from an earlier launch can never be mistaken for a new one.
//
// Every wait is bounded: after kSpinTicks of the 100 MHz real-time counter (2 s) it records
// kErrTimeout, raises the workspace abort flag and gives up; every other wait then gives up
// at its next poll.  The outputs of such a launch are undefined but the kernel terminates.
// ---------------------------------------------------------------------------------------
constexpr uint64_t kSpinTicks = 200000000ull;

__device__ __forceinline__ void lds_wait_writes() { __builtin_amdgcn_s_waitcnt(0xC07F); }  // lgkmcnt(0) only

__device__ __forceinline__ uint32_t lds_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_publish(uint32_t* p, uint32_t v) {
  lds_wait_writes();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ bool global_aborted(const Control* ctl) {
  return __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

__device__ __forceinline__ void raise_timeout(Control* ctl) {
  __hip_atomic_fetch_or(&ctl->err, kErrTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-uniform wait until *p >= need; 'seen' receives the value that satisfied it.  Returns
// false if the launch is being aborted.  With check_global = false the wait never touches
// global memory (a global load would make the wave wait for all of its outstanding loads):
// the loader uses that form and learns of a global abort through the workgroup's LDS flag,
// which the other waves raise.  With nap = false the wave re-reads the counter without
// sleeping in between (for waits on the critical path).  'waited' accumulates the ticks
// spent spinning (for the optional trace); it is a register-resident reference once inlined.
template <bool check_global = true, bool nap = true>
__device__ __forceinline__ bool lds_wait_value(const uint32_t* p, uint32_t need, uint32_t* lds_abort,
                                               Control* ctl, uint64_t& waited, uint32_t& seen) {
  seen = lds_load(p);
  if (seen >= need) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return true;
  }
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  uint32_t polls = 0;
  bool ok = true;
  for (;;) {
    if (nap) __builtin_amdgcn_s_sleep(1);
    seen = lds_load(p);
    if (seen >= need) break;
    if ((++polls & 255u) == 0u) {
      if (lds_load(lds_abort) != 0u || (check_global && global_aborted(ctl))) {
        ok = false;
        break;
      }
      if (__builtin_amdgcn_s_memrealtime() - t0 > kSpinTicks) {
        raise_timeout(ctl);
        ok = false;
        break;
      }
    }
  }
  waited += __builtin_amdgcn_s_memrealtime() - t0;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return ok;
}

// Wave-uniform wait until ready() holds, for a condition on several LDS counters: ready()
// issues all of its counter reads before it compares, so a satisfied condition costs one LDS
// round trip rather than one per counter.  No sleep between polls (for the critical path);
// otherwise bounded like lds_wait_value.
template <typename Ready>
__device__ __forceinline__ bool lds_wait_until(Ready ready, uint32_t* lds_abort, Control* ctl, uint64_t& waited) {
  if (ready()) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return true;
  }
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  uint32_t polls = 0;
  bool ok = true;
  for (;;) {
    if (ready()) break;
    if ((++polls & 255u) == 0u) {
      if (lds_load(lds_abort) != 0u || global_aborted(ctl)) {
        ok = false;
        break;
      }
      if (__builtin_amdgcn_s_memrealtime() - t0 > kSpinTicks) {
        raise_timeout(ctl);
        ok = false;
        break;
      }
    }
  }
  waited += __builtin_amdgcn_s_memrealtime() - t0;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return ok;
}

// Wave-uniform wait until *p >= need.  Returns false if the launch is being aborted.
template <bool check_global = true>
__device__ __forceinline__ bool lds_wait_ge(const uint32_t* p, uint32_t need, uint32_t* lds_abort,
                                            Control* ctl, uint64_t& waited) {
  uint32_t seen;
  return lds_wait_value<check_global>(p, need, lds_abort, ctl, waited, seen);
}

// Counter store for a wave whose earlier LDS writes must be seen first by the readers of
// the counter.  LDS operations of one wave are performed in order, so the data written
// before the counter is visible to any wave that has seen the counter; no wait is needed.
__device__ __forceinline__ void lds_signal(uint32_t* p, uint32_t v) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Buffer resource over 'bytes' bytes at 'base' (raw, stride 0): loads beyond the range
// return zero instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ uint64_t tagged(uint32_t payload, uint32_t epoch) {
  return ((uint64_t)epoch << 32) | payload;
}
__device__ __forceinline__ void store_word(uint64_t* p, uint64_t w) {
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_word(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads a small struct that is the same for every lane and moves it word by word into scalar
// registers, so that its fields are wave-uniform values to the compiler (a work item's
// description, read from a table the kernel also writes near, would otherwise stay in vector
// registers).
template <typename S>
__device__ __forceinline__ S load_uniform(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "word-sized struct expected");
  constexpr int NW = (int)(sizeof(S) / 4);
  S v = *p;
  uint32_t w[NW];
  __builtin_memcpy(w, &v, sizeof(S));
#pragma unroll
  for (int i = 0; i < NW; ++i) w[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)w[i]);
  __builtin_memcpy(&v, w, sizeof(S));
  return v;
}

// Claims the next work index for the whole workgroup (thread 0 claims, LDS broadcasts).
// Also snapshots the abort flag so that the loop exit is uniform across the workgroup.
__device__ __forceinline__ void claim_next(Control* ctl, uint32_t* sh_item, uint32_t* sh_abort) {
  if (threadIdx.x == 0) {
    *sh_item = __hip_atomic_fetch_add(&ctl->claim, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (global_aborted(ctl)) *sh_abort = 1u;
  }
  __syncthreads();
}

// Last workgroup out resets the control block for the next launch.
__device__ __forceinline__ void finish_launch(Control* ctl, uint32_t epoch) {
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t d = __hip_atomic_fetch_add(&ctl->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (d == gridDim.x - 1) {
      __hip_atomic_store(&ctl->claim, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->abort, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint32_t next = epoch + 1u;
      __hip_atomic_store(&ctl->epoch, next == 0u ? 1u : next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace wf
