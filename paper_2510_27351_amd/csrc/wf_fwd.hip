// Persistent band-pipelined forward sweep (gfx950).
//
// Work decomposition.  The m x n table is cut into bands of H = 64*R rows.  A persistent
// workgroup claims bands in increasing order from a device counter and sweeps each band
// from left to right as a skewed wavefront.  Lane r of the compute wave owns row r of each
// of the band's R sub-bands of 64 rows (rows r, 64+r, ...).  Sub-band k runs 65*k steps
// behind sub-band 0: at step t lane r produces column t - r - 65k of row 64k + r, so the
// cells of one step lie on R anti-diagonals and all of a lane's chains are independent
// within the step.  The three inputs of a cell come from registers:
//   W  the lane's previous value in the same sub-band;
//   N  the previous value of lane r-1 moved by a DPP wave_shr:1; lane 0 of sub-band 0 takes
//      the row above the band (the "top" ring in LDS, published by the band above); lane 0
//      of sub-band k >= 1 takes lane 63 of sub-band k-1 from two steps back, moved by a
//      DPP wave_ror:1 one step ahead (the extra step of skew keeps that move off the chain);
//   NW the previous step's N.
// A band takes n + H + R - 2 steps and the band below trails it by H + R - 1 + G steps plus
// the handoff latency: all m+n-1 anti-diagonals in one launch, with one handoff through
// global memory per H rows.
//
// Skewed LDS ring.  Element (row i, column c) of the band lives at S[i][(i + c + i/64) mod
// RING]: at step t every lane touches slot t in every sub-band, so a lane's four
// consecutive steps are one aligned 16-byte LDS access per sub-band.  A 16-byte chunk of
// slots [4j, 4j+4) of row i holds four consecutive columns, which are also consecutive in
// global memory, so every global transfer is one (4-byte aligned) 16-byte access paired
// with one aligned 16-byte LDS access.  The row pitch is 16 mod 256 bytes, which keeps
// 16-byte accesses of different rows on distinct banks.  D overwrites C in place.
//
// Five waves per workgroup:
//   wave 0  compute   per 4 steps and sub-band: one 16-byte LDS read of C, 4 x (DPP shift,
//                     min3, add), one 16-byte LDS write of D; one broadcast read of the top;
//   wave 1  loader    64-slot sub-chunks of C: 16R x (16-byte buffer load, 16-byte LDS write)
//                     per lane, PF sub-chunks in flight in registers;
//   wave 2  top       polls the band above's tagged boundary words, 64 columns per pass,
//                     and fills the top ring with every complete unit of G columns;
//   wave 3  storer    every 64 steps writes the sub-chunk's D back (16-byte LDS read,
//                     16-byte global store), the checkpoint columns and the score;
//   wave 4  publisher publishes the values of the band's last row that became final since
//                     its previous pass (whole units of G steps, up to 64 columns) as tagged
//                     words for the band below, and the checkpoint rows.
// The publisher has a wave of its own so that nothing delays the handoff, which sits on
// the critical path of the whole sweep.  G (16/32/64, the "tile width") is the handoff
// granularity.
//
// The same pipeline runs the soft-min variant of the recurrence (wf_soft_forward): with the
// SOFT option the compute wave applies the soft-min cell to values in the scaled domain
// y = D log2(e) / gamma, the publisher hands the last row on in that domain, and the storer
// writes D = y gamma ln 2.
#include "wf_common.h"
#include "wf_soft.h"

namespace wf {
namespace {

constexpr int kSub = 64;  // slots per loader / storer sub-chunk

// Returns x unchanged, but hides its value from the optimiser at this point.
template <typename V>
__device__ __forceinline__ V opaque(V x) {
  asm volatile("" : "+s"(x));
  return x;
}

__device__ __forceinline__ uint32_t dpp_ror1_u32(uint32_t src) {
  // wave_ror:1 -- lane r receives lane r-1's value, lane 0 receives lane 63's.
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)src, 0x13C, 0xf, 0xf, false);
}

template <typename T>
__device__ __forceinline__ T ror1(T x) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp_ror1_u32(__builtin_bit_cast(uint32_t, x)));
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint64_t lo = dpp_ror1_u32((uint32_t)b), hi = dpp_ror1_u32((uint32_t)(b >> 32));
    return __builtin_bit_cast(T, (hi << 32) | lo);
  }
}

template <typename T, int G, int R>
struct FwdCfg {
  using E = Elem<T>;
  static constexpr int H = kBand * R;  // rows per band
  // LDS ring: H rows x RING slots, about 128 KiB.
  static constexpr int RING = (sizeof(T) == 4 ? 512 : 256) / R;
  static constexpr int PITCH = RING + 16 / (int)sizeof(T);
  static constexpr int MASK = RING - 1;
  // Sub-chunks the loader keeps in flight in registers (bounded by the 256 registers a wave
  // may use when two of the five waves share a SIMD).
  static constexpr int PF = sizeof(T) * R == 4 ? 2 : 1;
  static constexpr int GPS = kSub / G;  // handoff units per sub-chunk
  static constexpr int NG = G / 4;      // 4-step groups per unit
  static_assert(RING % kSub == 0 && kSub % G == 0, "bad tiling");
  static_assert(RING >= 4 * kSub, "ring too small");
  // Offset between the column of row i at step t and t itself: column = t - i - i/64.
  __device__ static __forceinline__ int skew(int i) { return i + i / kBand; }
};

struct alignas(8) Shared {
  uint32_t ctr[6];  // 0: C sub-chunks loaded, 1: top units loaded, 2: steps done, 3: sub-chunks stored,
                    // 4: units published, 5: unused
  uint32_t item;
  uint32_t abort;
};

// Both readiness counters of the compute wave in one 8-byte LDS read.
__device__ __forceinline__ uint64_t load_ready(const Shared& sh) {
  return __hip_atomic_load(reinterpret_cast<const uint64_t*>(&sh.ctr[0]), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Every role below launders the kernel-wide sizes it uses through opaque() first:
// otherwise the compiler hoists each role's per-row address arithmetic out of the band loop
// and keeps all of it live across every role, which does not fit 256 registers per wave.

// ---------------------------------------------------------------------------------------
// wave 0: the cell chains
template <typename T, int G, int R>
struct ComputeState {
  T X[R];   // previous value of each sub-band (W of the next cell)
  T NW[R];  // previous N of each sub-band (NW of the next cell)
  T Q[R];   // k >= 1: lane 63 of sub-band k-1 two steps back (rotated to lane 0)
};

// Per 4-step group: C of every sub-band, and the top row's values at the group's columns
// (read by every lane from the same LDS address; lane 0 takes them).
template <typename T, int G, int R>
struct GroupRegs {
  Vec4<T> c[R];
  Vec4<T> t;
};

template <typename T, int G, int R>
struct UnitRegs {
  GroupRegs<T, G, R> g[2];  // the unit's first two groups
};

template <typename T, int G, int R>
__device__ __forceinline__ void load_group(const T* __restrict__ S, const T* __restrict__ Tr, int slot, int lane,
                                           GroupRegs<T, G, R>& r) {
  using C = FwdCfg<T, G, R>;
#pragma unroll
  for (int k = 0; k < R; ++k) r.c[k] = *reinterpret_cast<const Vec4<T>*>(S + (k * kBand + lane) * C::PITCH + slot);
  r.t = *reinterpret_cast<const Vec4<T>*>(Tr + slot);
}

// Four steps, X = C + min(NW, N, W) per cell.  N is lane r-1's previous value moved by a
// DPP wave_shr:1 whose "old" operand fills lane 0: for sub-band 0 the top row's value, for
// sub-band k >= 1 lane 63 of sub-band k-1 from two steps back; NW is the previous N.  Per
// cell one DPP move, one v_min3, one add, all lanes' chains independent within the step.
//
// SOFT: the soft-min cell instead (one sub-band only), on values in the scaled domain
// y = D log2(e) / gamma; kx scales the cell's input C the same way.
template <typename T, int G, int R, bool SOFT>
__device__ __forceinline__ void cells4(ComputeState<T, G, R>& st, const GroupRegs<T, G, R>& r, Vec4<T> (&out)[R],
                                       T kx) {
  using E = Elem<T>;
  if constexpr (SOFT) {
    static_assert(R == 1, "the soft-min sweep uses one sub-band per band");
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T N = E::shr1(st.X[0], r.t.v[q]);
      st.X[0] = soft_cell<T>(r.c[0].v[q] * kx, st.NW[0], N, st.X[0]);
      st.NW[0] = N;
      out[0].v[q] = st.X[0];
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T N[R], Qn[R];
    N[0] = E::shr1(st.X[0], r.t.v[q]);  // lane 0 takes the top row
#pragma unroll
    for (int k = 1; k < R; ++k) {
      N[k] = E::shr1(st.X[k], st.Q[k]);  // lane 0 takes lane 63 of sub-band k-1
      Qn[k] = ror1(st.X[k - 1]);         // ... for the next step
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const T v = E::min3v(st.NW[k], N[k], st.X[k]);
      st.X[k] = E::add(r.c[k].v[q], v);
      st.NW[k] = N[k];
      out[k].v[q] = st.X[k];
    }
#pragma unroll
    for (int k = 1; k < R; ++k) st.Q[k] = Qn[k];
  }
}

// Whether the C sub-chunk and the top unit that unit u reads are in LDS, by the counters in
// 'ready'.
template <typename T, int G, int R>
__device__ __forceinline__ bool unit_in_lds(uint64_t ready, int u) {
  const uint32_t need_c = (uint32_t)((G * u) / kSub + 1);
  const uint32_t need_t = (uint32_t)(u + 1);
  return (uint32_t)ready >= need_c && (uint32_t)(ready >> 32) >= need_t;
}

// Waits until the C sub-chunk and the top unit that unit u reads are in LDS.
template <typename T, int G, int R>
__device__ __forceinline__ bool unit_wait(int u, Shared& sh, Control* ctl, uint64_t& waited) {
  return lds_wait_until([&] { return __all(unit_in_lds<T, G, R>(load_ready(sh), u)); }, &sh.abort, ctl, waited);
}

// One unit of G steps.  'in' holds the first two groups of unit u (already read); the reads
// of each later group are issued two groups ahead, and the last two groups issue the reads
// of unit u+1's first two groups into 'out' -- always, so that both paths below leave them
// in the same registers (conditional reads make the compiler copy every prefetched register
// at each unit boundary).  If unit u+1's inputs were not yet in LDS two groups before the
// end (by the counters read at the start of the unit), unit u is finished and signalled
// first and the wave then waits for unit u+1 and reads its first groups again.  Waiting
// earlier would hold back the last steps of unit u, and with them the band's last row,
// until the band above has delivered unit u+1: one unit of extra lag per band.  After the
// last unit the reads wrap around the ring and are not used.
template <typename T, int G, int R, bool SOFT>
__device__ __forceinline__ bool compute_unit(T* __restrict__ S, const T* __restrict__ Tr, Shared& sh, Control* ctl,
                                             int u, int Us, ComputeState<T, G, R>& st, const UnitRegs<T, G, R>& in,
                                             UnitRegs<T, G, R>& out, uint32_t& stall_c, uint32_t& stall_t,
                                             uint64_t& waited, bool trace, T kx) {
  using C = FwdCfg<T, G, R>;
  constexpr int NG = C::NG;
  const int lane = threadIdx.x & 63;
  const int base = (G * u) & C::MASK;
  const int next_base = (G * (u + 1)) & C::MASK;
  const bool has_next = u + 1 < Us;
  const uint64_t ready = load_ready(sh);  // for unit u+1, used two groups before the end
  __builtin_amdgcn_sched_barrier(0);
  GroupRegs<T, G, R> gr[NG + 2];
#pragma unroll
  for (int p = 0; p < 2; ++p) gr[p] = in.g[p];
  bool early = true;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (g + 2 < NG) {
      load_group<T, G, R>(S, Tr, base + 4 * (g + 2), lane, gr[g + 2]);
    } else {
      if (g + 2 == NG) {
        __builtin_amdgcn_sched_barrier(0);
        early = !has_next || __all(unit_in_lds<T, G, R>(ready, u + 1));
        if (trace && !early) {
          stall_c += (uint32_t)ready < (uint32_t)((G * (u + 1)) / kSub + 1);
          stall_t += (uint32_t)(ready >> 32) < (uint32_t)(u + 2);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      load_group<T, G, R>(S, Tr, next_base + 4 * (g + 2 - NG), lane, out.g[g + 2 - NG]);
    }
    // keeps every group's reads two groups ahead of their use (left alone, the scheduler
    // gathers the reads of several groups into one burst just before the first of them)
    __builtin_amdgcn_sched_barrier(0);
    Vec4<T> d[R];
    cells4<T, G, R, SOFT>(st, gr[g], d, kx);
#pragma unroll
    for (int k = 0; k < R; ++k) *reinterpret_cast<Vec4<T>*>(S + (k * kBand + lane) * C::PITCH + base + 4 * g) = d[k];
  }
  lds_signal(&sh.ctr[2], (uint32_t)(G * (u + 1)));
  __builtin_amdgcn_sched_barrier(0);
  if (!early) {
    if (!unit_wait<T, G, R>(u + 1, sh, ctl, waited)) return false;
    // The slot is hidden from the optimiser: through the restrict pointers it would take
    // these reads for repeats of the early ones above and drop them.
    const int nb = opaque(next_base);
#pragma unroll
    for (int p = 0; p < 2; ++p) load_group<T, G, R>(S, Tr, nb + 4 * p, lane, out.g[p]);
    __builtin_amdgcn_sched_barrier(0);
  }
  return true;
}

template <typename T, int G, int R, bool SOFT>
__device__ __forceinline__ void compute_band(T* __restrict__ S, const T* __restrict__ Tr, Shared& sh, Control* ctl,
                                             int Us, bool first_band, uint64_t* trace, T kx) {
  using E = Elem<T>;
  const int lane = threadIdx.x & 63;
  ComputeState<T, G, R> st;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    st.X[k] = E::inf();
    st.NW[k] = E::inf();
    st.Q[k] = E::inf();
  }
  // NW of the band's first cell: the virtual corner D[-1][-1] = 0 for the first band,
  // D[row0-1][-1] = +inf for the others
  if (first_band && lane == 0) st.NW[0] = E::zero();
  uint32_t stall_c = 0, stall_t = 0;
  uint64_t t_first = 0, waited = 0;
  const bool tr = trace != nullptr;
  UnitRegs<T, G, R> P;
  if (!unit_in_lds<T, G, R>(load_ready(sh), 0) && !unit_wait<T, G, R>(0, sh, ctl, waited)) {
    sh.abort = 1u;
    return;
  }
  if (tr) t_first = __builtin_amdgcn_s_memrealtime();
#pragma unroll
  for (int p = 0; p < 2; ++p) load_group<T, G, R>(S, Tr, 4 * p, lane, P.g[p]);
  // One unit per iteration: a unit reads its first groups from P and leaves the next
  // unit's there (they are dead by the time those reads are issued, so both use the same
  // registers and nothing is copied at the back edge).
  for (int u = 0; u < Us; ++u) {
    if (!compute_unit<T, G, R, SOFT>(S, Tr, sh, ctl, u, Us, st, P, P, stall_c, stall_t, waited, tr, kx)) {
      sh.abort = 1u;
      return;
    }
    if (tr && u == 62 / G + 1) trace[16] = __builtin_amdgcn_s_memrealtime();
  }
  if (tr && lane == 0) {
    trace[1] = t_first;
    trace[2] = __builtin_amdgcn_s_memrealtime();
    trace[4] = stall_c;
    trace[5] = stall_t;
    trace[8] = waited;
  }
}

// ---------------------------------------------------------------------------------------
// wave 1: global -> LDS loader.
//
// Vector k of a lane covers row i = 4k + lane/16 and slots [64s + 4j, 64s + 4j + 4) of
// sub-chunk s, j = lane % 16, i.e. columns c0 .. c0+3 with c0 = 64s + 4j - skew(i).
template <typename T, int G, int R>
__device__ __forceinline__ void load_sub(Vec4<T> (&buf)[16 * R], __amdgpu_buffer_rsrc_t rsrc, int64_t ldc, int s) {
  using C = FwdCfg<T, G, R>;
  const int lane = threadIdx.x & 63;
  // Loads of different sub-chunks stay in issue order, so the wait before a sub-chunk's
  // LDS write leaves the later sub-chunks in flight.  Columns outside [0, n) read
  // neighbouring row data; an offset below the band's start (possible only for a single
  // column, where i*ldc + c0 can reach -1) wraps to a huge unsigned value and, like reads
  // past the band's end, returns zeros from the range-checked buffer; store_sub_lds masks
  // all of them.
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < 16 * R; ++k) {
    const int i = 4 * k + (lane >> 4);
    const int c0 = kSub * s + 4 * (lane & 15) - C::skew(i);
    const uint32_t off = (uint32_t)((int64_t)i * ldc + c0) * (uint32_t)sizeof(T);
    if constexpr (sizeof(T) == 4) {
      buf[k] = __builtin_bit_cast(Vec4<T>, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)off, 0, 0));
    } else {
      struct Hf { T x[2]; };
      const Hf lo = __builtin_bit_cast(Hf, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)off, 0, 0));
      const Hf hi = __builtin_bit_cast(Hf, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(off + 16), 0, 0));
      buf[k].v[0] = lo.x[0]; buf[k].v[1] = lo.x[1]; buf[k].v[2] = hi.x[0]; buf[k].v[3] = hi.x[1];
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// A sub-chunk with every row real and every column in [0, n) needs no masking.
template <typename T, int G, int R>
__device__ __forceinline__ bool interior_sub(int s, int rows, int64_t n) {
  using C = FwdCfg<T, G, R>;
  return rows == C::H && kSub * s >= C::skew(C::H - 1) && (int64_t)kSub * s + kSub <= n;
}

template <typename T, int G, int R>
__device__ __forceinline__ void store_sub_lds(T* S, const Vec4<T> (&buf)[16 * R], int s, int rows, int64_t n) {
  using C = FwdCfg<T, G, R>;
  using E = typename C::E;
  const int lane = threadIdx.x & 63;
  const bool interior = interior_sub<T, G, R>(s, rows, n);
#pragma unroll
  for (int k = 0; k < 16 * R; ++k) {
    const int i = 4 * k + (lane >> 4);
    const int slot = (kSub * s + 4 * (lane & 15)) & C::MASK;
    Vec4<T> v = buf[k];
    if (!interior) {
      const int64_t c0 = (int64_t)kSub * s + 4 * (lane & 15) - C::skew(i);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (i >= rows || c0 + e < 0 || c0 + e >= n) v.v[e] = E::inf();
    }
    *reinterpret_cast<Vec4<T>*>(S + i * C::PITCH + slot) = v;
  }
}

template <typename T, int G, int R>
__device__ __forceinline__ void loader_band(T* S, Shared& sh, const FwdArgs& a, int band, int Ks, uint64_t* tr) {
  using C = FwdCfg<T, G, R>;
  const int64_t ldc = opaque(a.ldc), n = opaque(a.n);
  const int64_t row0 = (int64_t)band * C::H;
  const int rows = (int)(a.m - row0 < C::H ? a.m - row0 : C::H);
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(static_cast<const T*>(a.C) + row0 * ldc,
                                                (uint32_t)(((rows - 1) * ldc + n) * (int64_t)sizeof(T)));
  uint64_t waited = 0;
  Vec4<T> buf[C::PF][16 * R];
#pragma unroll
  for (int p = 0; p < C::PF; ++p) load_sub<T, G, R>(buf[p], rsrc, ldc, p);
  for (int s0 = 0; s0 < Ks; s0 += C::PF) {
#pragma unroll
    for (int p = 0; p < C::PF; ++p) {
      const int s = s0 + p;
      if (s < Ks) {
        // sub-chunk s reuses the slots of sub-chunk s - RING/64, which must be stored (by
        // the storer) and whose last rows must be read (by the publisher)
        const int older = s - C::RING / kSub;
        if (older >= 0 && (!lds_wait_ge<false>(&sh.ctr[3], (uint32_t)(older + 1), &sh.abort, a.ctl, waited) ||
                           !lds_wait_ge<false>(&sh.ctr[4], (uint32_t)(C::GPS * (older + 1)), &sh.abort, a.ctl,
                                               waited))) {
          sh.abort = 1u;
          return;
        }
        store_sub_lds<T, G, R>(S, buf[p], s, rows, n);
        lds_signal(&sh.ctr[0], (uint32_t)(s + 1));
        if (s + C::PF < Ks) load_sub<T, G, R>(buf[p], rsrc, ldc, s + C::PF);
      }
    }
  }
  if (tr && (threadIdx.x & 63) == 0) {
    tr[9] = waited;
    tr[12] = __builtin_amdgcn_s_memrealtime();
  }
}

// ---------------------------------------------------------------------------------------
// wave 2: top boundary poller.  Each pass fetches the band above's boundary words for the
// 64 columns from the first unit not yet handed over and hands over every unit of G columns
// that is complete, so one global round trip advances it by up to 64 columns whatever G is.
template <typename T, int G, int R>
__device__ __forceinline__ void top_band(const T* S, T* Tr, Shared& sh, const FwdArgs& a, int band, int Ut,
                                         uint32_t epoch, uint64_t* tr) {
  using C = FwdCfg<T, G, R>;
  using E = typename C::E;
  constexpr int W = E::W;
  const int lane = threadIdx.x & 63;
  const int64_t n = opaque(a.n);
  uint64_t waited = 0, t0 = 0;
  uint32_t polls = 0;
  int u = 0;  // units handed over
  while (u < Ut) {
    const int64_t j0 = (int64_t)G * u;
    // the top ring slot of column j is read at step j and reused RING steps later
    const int64_t need_steps = j0 + 64 - C::RING;
    if (need_steps > 0 && !lds_wait_ge(&sh.ctr[2], (uint32_t)need_steps, &sh.abort, a.ctl, waited)) {
      sh.abort = 1u;
      return;
    }
    const int64_t j = j0 + lane;
    const bool real = j < n;
    // Every lane loads on every pass (a lane with no word to read loads spare words of the
    // control block and ignores them): loads under a lane mask would make each wait drain
    // all of the wave's loads.
    const bool live = band > 0 && real;
    const uint64_t* src = live ? a.bnd + ((int64_t)(band - 1) * n + j) * W : reinterpret_cast<const uint64_t*>(a.ctl) + 4;
    // Two polls in flight: while one pass's words are checked, the next pass's are on their
    // way, so readiness is seen about half a round trip sooner than with one.
    uint64_t xa[W], xb[W];
    auto issue = [&](uint64_t (&x)[W]) {
#pragma unroll
      for (int q = 0; q < W; ++q) x[q] = load_word(src + q);
    };
    // units complete in x: the leading run of ready columns (columns past the matrix count
    // as ready), in whole units
    auto complete = [&](const uint64_t (&x)[W]) -> int {
      bool ok = true;
#pragma unroll
      for (int q = 0; q < W; ++q) ok = ok && (uint32_t)(x[q] >> 32) == epoch;
      ok = ok || !live;
      const uint64_t okm = __ballot(ok);
      const int run = ~okm == 0 ? 64 : __builtin_ctzll(~okm);
      const int k = run / G;
      return k < Ut - u ? k : Ut - u;
    };
    auto value = [&](const uint64_t (&x)[W]) -> T {
      if (!live) return E::inf();
      uint32_t w[W];
#pragma unroll
      for (int q = 0; q < W; ++q) w[q] = (uint32_t)x[q];
      return E::from_words(w);
    };
    // false when the wait has to give up
    auto pause = [&]() -> bool {
      if (polls == 0 && tr) t0 = __builtin_amdgcn_s_memrealtime();
      __builtin_amdgcn_s_sleep(1);
      if ((++polls & 63u) == 0u) {
        if (lds_load(&sh.abort) != 0u || global_aborted(a.ctl)) return false;
        const uint64_t now = __builtin_amdgcn_s_memrealtime();
        if (polls == 64u) {
          if (!tr) t0 = now;
        } else if (now - t0 > kSpinTicks) {
          raise_timeout(a.ctl);
          return false;
        }
      }
      return true;
    };
    T val;
    int k;
    if (band == 0 || j0 >= n) {
      // nothing to fetch (the first band's top row is virtual, and so are the columns past
      // the matrix): +inf without a round trip through memory, so that the first band --
      // whose pace every later band follows -- never waits for its poller
      k = (int)(kSub / G) < Ut - u ? (int)(kSub / G) : Ut - u;
      val = E::inf();
    } else {
      issue(xa);
      for (;;) {
        issue(xb);
        if ((k = complete(xa)) > 0) {
          val = value(xa);
          break;
        }
        if (!pause()) {
          sh.abort = 1u;
          return;
        }
        issue(xa);
        if ((k = complete(xb)) > 0) {
          val = value(xb);
          break;
        }
        if (!pause()) {
          sh.abort = 1u;
          return;
        }
      }
    }
    if (polls != 0u) {
      if (tr) waited += __builtin_amdgcn_s_memrealtime() - t0;
      polls = 0;
    }
    const int cols = k * G;
    if (lane < cols) Tr[(int)(j & C::MASK)] = real ? val : E::inf();
    u += k;
    lds_signal(&sh.ctr[1], (uint32_t)u);
    if (tr && u == k && lane == 0) tr[15] = __builtin_amdgcn_s_memrealtime();
  }
  if (tr && lane == 0) {
    tr[10] = waited;
    tr[13] = __builtin_amdgcn_s_memrealtime();
  }
}

// ---------------------------------------------------------------------------------------
// wave 3: storer.  SOFT: the ring holds scaled values; D = y * gl (gl = gamma ln 2).
template <typename T, int R, bool SOFT>
__device__ __forceinline__ void unscale(Vec4<T> (&v)[16], T gl) {
  if constexpr (SOFT) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) v[k].v[e] *= gl;
  }
}

template <typename T, int G, int R, bool SOFT>
__device__ __forceinline__ void store_sub(const T* S, __amdgpu_buffer_rsrc_t drs, int64_t ldd, int64_t n, int rows,
                                          int s, T gl) {
  using C = FwdCfg<T, G, R>;
  typedef int v4i __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int j4 = 4 * (lane & 15);
  const int slot = (kSub * s + j4) & C::MASK;
  if (interior_sub<T, G, R>(s, rows, n)) {
    // Interior sub-chunk: 16 LDS reads first, then one 16-byte store per 16 bytes.
#pragma unroll
    for (int h = 0; h < R; ++h) {
      Vec4<T> v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int i = 64 * h + 4 * k + (lane >> 4);
        v[k] = *reinterpret_cast<const Vec4<T>*>(S + i * C::PITCH + slot);
      }
      unscale<T, R, SOFT>(v, gl);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int i = 64 * h + 4 * k + (lane >> 4);
        const int off = (int)(((int64_t)i * ldd + kSub * s + j4 - C::skew(i)) * (int64_t)sizeof(T));
        if constexpr (sizeof(T) == 4) {
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, v[k]), drs, off, 0, 0);
        } else {
          struct Hf { v4i lo, hi; };
          const Hf hh = __builtin_bit_cast(Hf, v[k]);
          __builtin_amdgcn_raw_buffer_store_b128(hh.lo, drs, off, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b128(hh.hi, drs, off + 16, 0, 0);
        }
      }
    }
    return;
  }
  // Edge sub-chunk (first, last, or a partial band): the same 16 LDS reads first, then per
  // vector one 16-byte store if its four cells lie inside the matrix, else a store per cell
  // that does (one sub-band at a time: both at once would not fit the registers).
#pragma unroll 1
  for (int h = 0; h < R; ++h) {
    Vec4<T> v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = 64 * h + 4 * k + (lane >> 4);
      v[k] = *reinterpret_cast<const Vec4<T>*>(S + i * C::PITCH + slot);
    }
    unscale<T, R, SOFT>(v, gl);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = 64 * h + 4 * k + (lane >> 4);
      const int64_t c0 = (int64_t)kSub * s + j4 - C::skew(i);
      if (i >= rows) continue;
      const int off = (int)(((int64_t)i * ldd + c0) * (int64_t)sizeof(T));
      if (c0 >= 0 && c0 + 4 <= n) {
        if constexpr (sizeof(T) == 4) {
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, v[k]), drs, off, 0, 0);
        } else {
          struct Hf { v4i lo, hi; };
          const Hf hh = __builtin_bit_cast(Hf, v[k]);
          __builtin_amdgcn_raw_buffer_store_b128(hh.lo, drs, off, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b128(hh.hi, drs, off + 16, 0, 0);
        }
        continue;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (c0 + e >= 0 && c0 + e < n) {
          if constexpr (sizeof(T) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v[k].v[e]), drs, off + 4 * e, 0, 0);
          } else {
            typedef int v2i __attribute__((ext_vector_type(2)));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v[k].v[e]), drs, off + 8 * e, 0, 0);
          }
        }
      }
    }
  }
}

template <typename T, int G, int R, bool SOFT>
__device__ __forceinline__ void store_band(const T* S, Shared& sh, const FwdArgs& a, int band, int Ks,
                                           uint64_t* tr) {
  using C = FwdCfg<T, G, R>;
  const int lane = threadIdx.x & 63;
  const int64_t m = opaque(a.m), n = opaque(a.n), ldd = opaque(a.ldd);
  const int64_t row0 = (int64_t)band * C::H;
  const int rows = (int)(m - row0 < C::H ? m - row0 : C::H);
  T* ck_cols = a.ckpt ? static_cast<T*>(a.ckpt) + ((m + kBand - 1) / kBand - 1) * n : nullptr;
  const int K = a.ckpt_k;
  const int64_t sc_row = m - 1 - row0;  // band row of the score, if it lies in this band
  const T gl = SOFT ? (T)a.gl : T(1);
  const __amdgpu_buffer_rsrc_t drs =
      make_rsrc(a.D ? static_cast<T*>(a.D) + row0 * ldd : nullptr,
                a.D ? (uint32_t)(((rows - 1) * ldd + n) * (int64_t)sizeof(T)) : 0u);
  uint64_t waited = 0;
  for (int s = 0; s < Ks; ++s) {
    // sub-chunk s (slots [64s, 64s+64) of every row) is final after step 64s + 63; its D
    // goes out after the publisher has issued the boundary words of those steps, which
    // the band below waits for
    if (!lds_wait_ge(&sh.ctr[4], (uint32_t)(C::GPS * (s + 1)), &sh.abort, a.ctl, waited)) {
      sh.abort = 1u;
      return;
    }
    if (a.D) store_sub<T, G, R, SOFT>(S, drs, ldd, n, rows, s, gl);
    if (ck_cols) {
#pragma unroll
      for (int h = 0; h < R; ++h) {
        const int i = 64 * h + lane;
        if (i >= rows) continue;
        // checkpoint columns D[.][Kq-1] of row i held by sub-chunk s
        const int64_t lo = (int64_t)kSub * s - C::skew(i), hi = lo + kSub;
        for (int64_t j = ((lo > 0 ? lo : 0) + K) / K * K - 1; j < hi; j += K) {
          if (j >= lo && j + 1 < n)
            ck_cols[((j + 1) / K - 1) * m + row0 + i] = S[i * C::PITCH + ((int)(j + C::skew(i)) & C::MASK)];
        }
      }
    }
    if (sc_row >= 0 && sc_row < C::H && lane == (int)(sc_row % kBand)) {
      const int64_t slot = n - 1 + C::skew((int)sc_row);
      if (slot / kSub == s) {
        const T y = S[sc_row * C::PITCH + ((int)slot & C::MASK)];
        *static_cast<T*>(a.score) = SOFT ? y * gl : y;
      }
    }
    lds_publish(&sh.ctr[3], (uint32_t)(s + 1));
  }
  if (tr && lane == 0) tr[11] = waited;
}

// ---------------------------------------------------------------------------------------
// wave 4: publisher of the band's last row (and of the checkpoint rows)
template <typename T, int G, int R>
__device__ __forceinline__ void publish_band(const T* S, Shared& sh, const FwdArgs& a, int band, int Us,
                                             uint32_t epoch, uint64_t* tr) {
  using C = FwdCfg<T, G, R>;
  using E = typename C::E;
  constexpr int W = E::W;
  const int lane = threadIdx.x & 63;
  const int64_t m = opaque(a.m), n = opaque(a.n);
  const int nb64 = (int)((m + kBand - 1) / kBand);  // 64-row bands of the checkpoint grid
  const bool last_band = band == a.nb - 1;
  T* ck_rows = static_cast<T*>(a.ckpt);
  // an injected fault (tests of the failure path) makes band 0 withhold its boundary row
  const bool withhold =
      band == 0 && __hip_atomic_load(&a.ctl->fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == kFaultFwdWithhold;
  uint64_t waited = 0;
  for (int u = 0; u < Us;) {
    uint32_t done;
    if (!lds_wait_value<true, false>(&sh.ctr[2], (uint32_t)(G * (u + 1)), &sh.abort, a.ctl, waited, done)) {
      sh.abort = 1u;
      return;
    }
    // every unit finished by now goes out in this pass, up to 64 columns
    int k = (int)(done / G) - u;
    if (k > kSub / G) k = kSub / G;
    if (k > Us - u) k = Us - u;
    const int cols = k * G;
    const bool mark = tr && u <= 62 / G + 1 && 62 / G + 1 < u + k && lane == 0;
    if (mark) tr[17] = __builtin_amdgcn_s_memrealtime();
    if (lane < cols) {
      const int slot = (G * u + lane) & C::MASK;
      // the band's last row, row H-1, finished column Gu + lane - skew(H-1) at this step
      const int64_t j = (int64_t)G * u + lane - C::skew(C::H - 1);
      if (!last_band && !withhold && j >= 0 && j < n) {
        const T x = S[(C::H - 1) * C::PITCH + slot];
#pragma unroll
        for (int q = 0; q < W; ++q) store_word(a.bnd + ((int64_t)band * n + j) * W + q, tagged(E::word(x, q), epoch));
      }
      // checkpoint rows: the last row of every 64-row sub-band except the matrix's last one
      if (ck_rows) {
#pragma unroll
        for (int h = 0; h < R; ++h) {
          const int i = 64 * h + 63;
          const int b64 = band * R + h;
          const int64_t jc = (int64_t)G * u + lane - C::skew(i);
          if (b64 < nb64 - 1 && jc >= 0 && jc < n) ck_rows[(int64_t)b64 * n + jc] = S[i * C::PITCH + slot];
        }
      }
    }
    if (mark) tr[14] = __builtin_amdgcn_s_memrealtime();
    u += k;
    lds_publish(&sh.ctr[4], (uint32_t)u);
  }
  if (tr && lane == 0) tr[18] = waited;
}

// ---------------------------------------------------------------------------------------
// One band of one instance, all five roles.  The LDS counters must be zero on entry.
template <typename T, int G, int R, bool SOFT = false>
__device__ __forceinline__ void run_band(T* S, T* Tr, Shared& sh, const FwdArgs& a, int band, uint32_t epoch,
                                         uint64_t* tr) {
  using C = FwdCfg<T, G, R>;
  const int wave = threadIdx.x >> 6;
  // steps of a band: n + skew(H-1), rounded up to whole 64-slot sub-chunks
  const int Ks = (int)((a.n + C::skew(C::H - 1) + kSub - 1) / kSub);  // C sub-chunks
  const int Us = Ks * C::GPS;                                          // compute / publish units
  const int Ut = (int)((a.n + G - 1) / G);                             // top units holding real columns
  if (wave == 0) {
    compute_band<T, G, R, SOFT>(S, Tr, sh, a.ctl, Us, band == 0, tr, SOFT ? (T)a.kx : T(1));
  } else if (wave == 1) {
    loader_band<T, G, R>(S, sh, a, band, Ks, tr);
  } else if (wave == 2) {
    top_band<T, G, R>(S, Tr, sh, a, band, Ut, epoch, tr);
    // Top units beyond the last real column hold no values any real cell reads; mark
    // them loaded so that the compute wave's readiness test stays one comparison.
    if ((threadIdx.x & 63) == 0 && sh.abort == 0u) lds_signal(&sh.ctr[1], 0x7fffffffu);
  } else if (wave == 3) {
    store_band<T, G, R, SOFT>(S, sh, a, band, Ks, tr);
  } else {
    publish_band<T, G, R>(S, sh, a, band, Us, epoch, tr);
  }
}

// TRACE = false compiles every trace statement out (the production instance); the traced
// instance is launched only while tracing is enabled.
template <typename T, int G, int R, bool TRACE, bool SOFT = false>
__global__ __launch_bounds__(kThreads, 1) void fwd_kernel(FwdArgs a) {
  using C = FwdCfg<T, G, R>;
  if constexpr (!TRACE) a.trace = nullptr;
  __shared__ Vec4<T> S4[C::H * C::PITCH / 4];
  __shared__ Vec4<T> Tr4[C::RING / 4];
  __shared__ Shared sh;
  T* S = reinterpret_cast<T*>(S4);
  T* Tr = reinterpret_cast<T*>(Tr4);
  Control* ctl = a.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x < 6) sh.ctr[threadIdx.x] = 0u;
    claim_next(ctl, &sh.item, &sh.abort);
    const int band = (int)sh.item;
    if (band >= a.nb || sh.abort != 0u) break;
    uint64_t* tr = a.trace ? a.trace + (int64_t)band * kTraceWords : nullptr;
    if (tr && threadIdx.x == 0) {
      unsigned xcc;
      asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
      tr[0] = __builtin_amdgcn_s_memrealtime();
      tr[6] = xcc;
      tr[7] = blockIdx.x;
    }
    run_band<T, G, R, SOFT>(S, Tr, sh, a, band, epoch, tr);
    if (tr && threadIdx.x == 3 * 64) tr[3] = __builtin_amdgcn_s_memrealtime();
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

// Ragged batch: work items (instance, band) are claimed in list order; the host orders the
// list so that every band comes after the band above it of the same instance (and
// instances by decreasing critical path), so a claimed band only ever waits for bands
// that were claimed before it and are running or done.
template <typename T, int G, int R>
__global__ __launch_bounds__(kThreads, 1) void fwd_batch_kernel(BatchArgs b) {
  using C = FwdCfg<T, G, R>;
  __shared__ Vec4<T> S4[C::H * C::PITCH / 4];
  __shared__ Vec4<T> Tr4[C::RING / 4];
  __shared__ Shared sh;
  T* S = reinterpret_cast<T*>(S4);
  T* Tr = reinterpret_cast<T*>(Tr4);
  Control* ctl = b.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x < 6) sh.ctr[threadIdx.x] = 0u;
    claim_next(ctl, &sh.item, &sh.abort);
    const uint32_t item = sh.item;
    if (item >= (uint32_t)b.n_items || sh.abort != 0u) break;
    const BatchItem it = b.items[item];
    const BatchInst in = b.inst[it.inst];
    FwdArgs a;
    a.C = static_cast<const T*>(b.C) + in.off;
    a.D = b.D ? static_cast<T*>(b.D) + in.off : nullptr;
    a.score = static_cast<T*>(b.scores) + it.inst;
    a.ckpt = b.ckpt ? static_cast<T*>(b.ckpt) + in.ck_off : nullptr;
    a.ldc = in.n;
    a.ldd = in.n;
    a.m = in.m;
    a.n = in.n;
    a.ckpt_k = b.ckpt ? b.ckpt_k : 0;
    a.nb = in.nb;
    a.ctl = ctl;
    a.bnd = b.bnd + in.bnd_off;
    a.trace = nullptr;
    a.kx = a.gl = 1.0;
    run_band<T, G, R>(S, Tr, sh, a, it.band, epoch, nullptr);
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

template <typename T, int R, bool TRACE>
hipError_t launch_tt(int tile, const FwdArgs& a, int grid, hipStream_t s) {
  switch (tile) {
    case 16: hipLaunchKernelGGL((fwd_kernel<T, 16, R, TRACE>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 32: hipLaunchKernelGGL((fwd_kernel<T, 32, R, TRACE>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 64: hipLaunchKernelGGL((fwd_kernel<T, 64, R, TRACE>), dim3(grid), dim3(kThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int R>
hipError_t launch_t(int tile, const FwdArgs& a, int grid, hipStream_t s) {
  return a.trace ? launch_tt<T, R, true>(tile, a, grid, s) : launch_tt<T, R, false>(tile, a, grid, s);
}

template <typename T, int R>
hipError_t launch_batch_t(int tile, const BatchArgs& b, int grid, hipStream_t s) {
  switch (tile) {
    case 16: hipLaunchKernelGGL((fwd_batch_kernel<T, 16, R>), dim3(grid), dim3(kThreads), 0, s, b); break;
    case 32: hipLaunchKernelGGL((fwd_batch_kernel<T, 32, R>), dim3(grid), dim3(kThreads), 0, s, b); break;
    case 64: hipLaunchKernelGGL((fwd_batch_kernel<T, 64, R>), dim3(grid), dim3(kThreads), 0, s, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// 64-row sub-bands per band of the single-instance sweep for the 4-byte types.  One is the
// fastest at 16384 x 16384 on MI355X (two halve the handoffs but double the compute wave's
// work per step and leave half of the compute units idle at 256 bands); double always
// uses one.  The batch sweep lets its autotuner choose one or two.
constexpr int kRowsF = 1;

}  // namespace

int forward_band_rows(int dtype) { return dtype == 1 ? kBand : kBand * kRowsF; }

hipError_t launch_forward(int dtype, int tile, const FwdArgs& a, int grid, hipStream_t s) {
  switch (dtype) {
    case 0: return launch_t<float, kRowsF>(tile, a, grid, s);
    case 1: return launch_t<double, 1>(tile, a, grid, s);
    case 2: return launch_t<int32_t, kRowsF>(tile, a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// The soft-min sweep's steps cost several times a min-plus step (exponentials and a
// logarithm per cell), so the finest handoff unit, 16 columns, serves it best.
hipError_t launch_forward_soft(int dtype, const FwdArgs& a, int grid, hipStream_t s) {
  switch (dtype) {
    case 0: hipLaunchKernelGGL((fwd_kernel<float, 16, 1, false, true>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 1: hipLaunchKernelGGL((fwd_kernel<double, 16, 1, false, true>), dim3(grid), dim3(kThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_forward_batch(int dtype, int tile, int rows, const BatchArgs& b, int grid, hipStream_t s) {
  if (rows == 2 && dtype != 1) {
    return dtype == 0 ? launch_batch_t<float, 2>(tile, b, grid, s) : launch_batch_t<int32_t, 2>(tile, b, grid, s);
  }
  if (rows != 1) return hipErrorInvalidValue;
  switch (dtype) {
    case 0: return launch_batch_t<float, 1>(tile, b, grid, s);
    case 1: return launch_batch_t<double, 1>(tile, b, grid, s);
    case 2: return launch_batch_t<int32_t, 1>(tile, b, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wf
