// Adjoint (backward) sweep of the wavefront recurrence (gfx950).
//
// The routed adjoint of  L = sum(gD * D) + gscore * score  is
//     A[i][j] = gD[i][j] + [last] gscore + [SEL(i+1,j+1) = NW] A[i+1][j+1]
//             + [SEL(i,j+1) = W] A[i][j+1] + [SEL(i+1,j) = N] A[i+1][j],       gC = A,
// summed in exactly that order (reading R0; the paper states no recurrence).  SEL(i,j) is the
// predecessor cell (i,j) took in the forward min, ties broken NW, N, W.
//
// Two launches:
//  1. Selection recompute.  Every 64-row band is swept again left to right from its top
//     row, which the forward pass stored as a checkpoint row (or which the caller's saved
//     table provides).  The bands are therefore independent and all run at once.  The
//     sweep is the forward cell chain plus the two comparisons that name the predecessor;
//     it emits 2-bit codes, 16 per 32-bit word per lane.
//  2. Reverse sweep.  Bands from the bottom up, each a skewed wavefront from right to left:
//     lane r owns band row r and at reverse step t handles slot s = S - t (slot = row +
//     column), so lane r+1 handles a column one step before lane r does.  A cell's three
//     inputs are the routed values its successors pushed: from the south (lane r+1, one step
//     back, DPP wave_shl:1), from the east (the lane itself, one step back) and from the
//     south-east (lane r+1, two steps back).  Lane 63 takes the south and south-east values
//     from the band below, which publishes them (tagged 64-bit words, as in the forward
//     sweep).  After computing A a cell pushes it to the predecessor its code names and zero
//     to the others.
// Waves of the reverse sweep: compute; loader (gD and the selection words into LDS);
// poller (values from the band below); storer (gC); publisher (values for the band above).
#include "wf_common.h"

namespace wf {
namespace {

constexpr int kSub = 64;

template <typename V>
__device__ __forceinline__ V opaque(V x) {
  asm volatile("" : "+s"(x));
  return x;
}

enum : uint32_t { kSelNone = 0, kSelNW = 1, kSelN = 2, kSelW = 3 };

// wave_shl:1 -- lane r receives lane r+1's value; lane 63 keeps 'old'.
__device__ __forceinline__ uint32_t dpp_shl1_u32(uint32_t src, uint32_t old) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x130, 0xf, 0xf, false);
}
template <typename T>
__device__ __forceinline__ T shl1(T src, T old) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp_shl1_u32(__builtin_bit_cast(uint32_t, src), __builtin_bit_cast(uint32_t, old)));
  } else {
    const uint64_t s = __builtin_bit_cast(uint64_t, src), o = __builtin_bit_cast(uint64_t, old);
    const uint64_t lo = dpp_shl1_u32((uint32_t)s, (uint32_t)o), hi = dpp_shl1_u32((uint32_t)(s >> 32), (uint32_t)(o >> 32));
    return __builtin_bit_cast(T, (hi << 32) | lo);
  }
}

template <typename T>
struct BCfg {
  using E = Elem<T>;
  static constexpr int RING = E::RING;
  static constexpr int PITCH = E::PITCH;
  static constexpr int MASK = RING - 1;
  static constexpr int SW = RING / 16;   // selection words per lane in the ring
  static constexpr int SPITCH = SW + 4;  // their row pitch (16-byte aligned rows)
};

// Layout of the selection words in global memory: for band b, sub-chunk k (slots
// [64k, 64k+64)), lane r, the four words covering those slots are contiguous.
__device__ __forceinline__ int64_t sel_index(int band, int Ks, int k, int lane) {
  return (((int64_t)band * Ks + k) * 64 + lane) * 4;
}

// =======================================================================================
// 1. Selection recompute: two waves (compute, loader), one 64-row band per workgroup.
// =======================================================================================
struct alignas(8) SelShared {
  uint32_t loaded;  // sub-chunks of C and of the top row in LDS
  uint32_t steps;   // steps done by the compute wave
  uint32_t item;
  uint32_t abort;
};

template <typename T>
__device__ __forceinline__ void sel_compute(const T* __restrict__ S, const T* __restrict__ Tr, SelShared& sh,
                                            const SelArgs& a, int band, int Ks) {
  using C = BCfg<T>;
  using E = typename C::E;
  const int lane = threadIdx.x & 63;
  const int64_t n = opaque(a.n);
  const int rows = (int)(a.m - (int64_t)band * kBand < kBand ? a.m - (int64_t)band * kBand : kBand);
  T X = E::inf();
  T NW = (lane == 0 && band == 0) ? E::zero() : E::inf();  // virtual corner D[-1][-1] = 0
  uint32_t* out = a.sel;
  uint64_t waited = 0;
  for (int k = 0; k < Ks; ++k) {
    if (!lds_wait_ge(&sh.loaded, (uint32_t)(k + 1), &sh.abort, a.ctl, waited)) {
      sh.abort = 1u;
      return;
    }
    const int base = (kSub * k) & C::MASK;
    uint32_t words[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t word = 0;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int off = base + 16 * w + 4 * g;
        const Vec4<T> cv = *reinterpret_cast<const Vec4<T>*>(S + lane * C::PITCH + off);
        const Vec4<T> tv = *reinterpret_cast<const Vec4<T>*>(Tr + off);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const T N = E::shr1(X, tv.v[q]);
          // predecessor code with ties to NW, then N, then W (strict comparisons)
          const bool n_lt = N < NW;
          const T m1 = n_lt ? N : NW;
          const bool w_lt = X < m1;
          const uint32_t code = w_lt ? kSelW : (n_lt ? kSelN : kSelNW);
          word |= code << (2 * (4 * g + q));
          X = E::add(cv.v[q], w_lt ? X : m1);
          NW = N;
        }
      }
      // zero the codes of cells outside the matrix (and of cell (0,0), which has none)
      const int t0 = kSub * k + 16 * w;
      if (!(rows == kBand && t0 >= kBand - 1 && (int64_t)t0 + 16 <= n)) {
        const int64_t lo = lane - (int64_t)t0, hi = n + lane - (int64_t)t0;  // valid steps [lo, hi)
        const int a0 = (int)(lo < 0 ? 0 : (lo > 16 ? 16 : lo));
        const int a1 = (int)(hi < 0 ? 0 : (hi > 16 ? 16 : hi));
        uint64_t msk = a1 > a0 ? (((uint64_t)1 << (2 * a1)) - 1) & ~(((uint64_t)1 << (2 * a0)) - 1) : 0;
        if (lane >= rows) msk = 0;
        if (band == 0 && lane == 0 && t0 == 0) msk &= ~(uint64_t)3;
        word &= (uint32_t)msk;
      }
      words[w] = word;
    }
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i wv = {(int)words[0], (int)words[1], (int)words[2], (int)words[3]};
    __builtin_nontemporal_store(wv, reinterpret_cast<v4i*>(out + sel_index(band, Ks, k, lane)));
    lds_signal(&sh.steps, (uint32_t)(kSub * (k + 1)));
  }
}

// Sub-chunks of C the selection loader keeps in flight in registers (two waves per
// workgroup leave room for them).
template <typename T>
struct SelPF {
  static constexpr int PF = sizeof(T) == 4 ? 3 : 1;
};

// Issues the loads of sub-chunk k of C (16 lanes x 4 rows per vector, rows 0..63) and of
// the row above the band for slots [64k, 64k+64).
template <typename T>
__device__ __forceinline__ void sel_load_sub(Vec4<T> (&x)[16], T& tv, __amdgpu_buffer_rsrc_t rsrc, int64_t ldc,
                                             const T* top, int64_t n, int k) {
  const int lane = threadIdx.x & 63;
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = 4 * v + (lane >> 4);
    const int64_t c0 = (int64_t)kSub * k + 4 * (lane & 15) - i;
    const uint32_t off = (uint32_t)(i * ldc + c0) * (uint32_t)sizeof(T);
    if constexpr (sizeof(T) == 4) {
      x[v] = __builtin_bit_cast(Vec4<T>, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)off, 0, 0));
    } else {
      struct Hf { T y[2]; };
      const Hf lo = __builtin_bit_cast(Hf, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)off, 0, 0));
      const Hf hi = __builtin_bit_cast(Hf, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(off + 16), 0, 0));
      x[v].v[0] = lo.y[0]; x[v].v[1] = lo.y[1]; x[v].v[2] = hi.y[0]; x[v].v[3] = hi.y[1];
    }
  }
  const int64_t j = (int64_t)kSub * k + lane;
  tv = (top && j < n) ? top[j] : Elem<T>::inf();
  __builtin_amdgcn_sched_barrier(0);
}

template <typename T>
__device__ __forceinline__ void sel_store_sub(T* S, T* Tr, const Vec4<T> (&x)[16], T tv, int k, int rows,
                                              int64_t n) {
  using C = BCfg<T>;
  using E = typename C::E;
  const int lane = threadIdx.x & 63;
  const bool interior = rows == kBand && k > 0 && (int64_t)kSub * k + kSub <= n;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = 4 * v + (lane >> 4);
    const int64_t c0 = (int64_t)kSub * k + 4 * (lane & 15) - i;
    Vec4<T> y = x[v];
    if (!interior) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (i >= rows || c0 + e < 0 || c0 + e >= n) y.v[e] = E::inf();
    }
    *reinterpret_cast<Vec4<T>*>(S + i * C::PITCH + ((kSub * k + 4 * (lane & 15)) & C::MASK)) = y;
  }
  Tr[(kSub * k + lane) & C::MASK] = tv;
}

template <typename T>
__device__ __forceinline__ void sel_loader(T* S, T* Tr, SelShared& sh, const SelArgs& a, int band, int Ks) {
  using C = BCfg<T>;
  constexpr int PF = SelPF<T>::PF;
  const int64_t ldc = opaque(a.ldc), n = opaque(a.n), m = opaque(a.m);
  const int64_t row0 = (int64_t)band * kBand;
  const int rows = (int)(m - row0 < kBand ? m - row0 : kBand);
  // Loads outside the band's rows (or columns outside [0, n) on the last row) return zeros
  // from the range-checked buffer; sel_store_sub replaces them by +inf.
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(static_cast<const T*>(a.C) + row0 * ldc,
                                                (uint32_t)(((rows - 1) * ldc + n) * (int64_t)sizeof(T)));
  const T* top = band > 0 ? static_cast<const T*>(a.top) + (int64_t)(band - 1) * a.ld_top : nullptr;
  uint64_t waited = 0;
  Vec4<T> buf[PF][16];
  T tv[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p)
    if (p < Ks) sel_load_sub<T>(buf[p], tv[p], rsrc, ldc, top, n, p);
  for (int k0 = 0; k0 < Ks; k0 += PF) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int k = k0 + p;
      if (k >= Ks) break;
      // sub-chunk k reuses the ring slots of sub-chunk k - RING/64
      const int older = k - C::RING / kSub;
      if (older >= 0 &&
          !lds_wait_ge<false>(&sh.steps, (uint32_t)(kSub * (older + 1)), &sh.abort, a.ctl, waited)) {
        sh.abort = 1u;
        return;
      }
      sel_store_sub<T>(S, Tr, buf[p], tv[p], k, rows, n);
      lds_publish(&sh.loaded, (uint32_t)(k + 1));
      if (k + PF < Ks) sel_load_sub<T>(buf[p], tv[p], rsrc, ldc, top, n, k + PF);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(128, 1) void sel_kernel(SelArgs a) {
  using C = BCfg<T>;
  __shared__ Vec4<T> S4[kBand * C::PITCH / 4];
  __shared__ Vec4<T> Tr4[C::RING / 4];
  __shared__ SelShared sh;
  T* S = reinterpret_cast<T*>(S4);
  T* Tr = reinterpret_cast<T*>(Tr4);
  Control* ctl = a.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int Ks = (int)((a.n + kBand - 1 + kSub - 1) / kSub);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      sh.loaded = 0u;
      sh.steps = 0u;
    }
    claim_next(ctl, &sh.item, &sh.abort);
    const int band = (int)sh.item;
    if (band >= a.nb || sh.abort != 0u) break;
    if (threadIdx.x < 64)
      sel_compute<T>(S, Tr, sh, a, band, Ks);
    else
      sel_loader<T>(S, Tr, sh, a, band, Ks);
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

// =======================================================================================
// 2. Reverse sweep: five waves, one 64-row band per workgroup, bands from the bottom up.
// =======================================================================================
struct alignas(8) AdjShared {
  uint32_t ctr[6];  // 0: sub-chunks loaded (gD + selection), 1: bottom units loaded,
                    // 2: reverse steps done, 3: sub-chunks stored, 4: units published
  uint32_t item;
  uint32_t abort;
};

// Both readiness counters of the compute wave in one 8-byte LDS read.  'zero' is 0, but
// the compiler cannot tell: the value counts as per-lane data and is compared where it is
// used, so the wave waits for it there rather than right after the read (where it would
// also wait for every earlier LDS read, the prefetches).
__device__ __forceinline__ uint64_t adj_ready(const AdjShared& sh, int zero) {
  return __hip_atomic_load(reinterpret_cast<const uint64_t*>(&sh.ctr[0]) + zero, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int adj_opaque_zero() {
  int z = 0;
  asm volatile("" : "+v"(z));
  return z;
}

// wave 0: the reverse chain.  Slot group [b4, b4+4) is processed from b4+3 down to b4.
// The LDS reads of a group (the upstream values, the band-below values and the selection
// word) are issued PD groups ahead of their use: LDS latency under the other waves'
// traffic is longer than one group's compute.
template <typename T>
struct AdjGroup {
  Vec4<T> gv, bn, bnw;
  uint32_t word;
};

template <typename T, int G>
struct AdjCfg {
  static constexpr int NG = G / 4;
  static constexpr int PD = sizeof(T) == 4 ? 2 : 1;
};

template <typename T, int G>
struct AdjUnitRegs {
  AdjGroup<T> g[AdjCfg<T, G>::PD];
};

template <typename T>
__device__ __forceinline__ void adj_load_group(const T* __restrict__ S, const uint32_t* __restrict__ SelR,
                                               const T* __restrict__ Bn, const T* __restrict__ Bnw, int b4, int lane,
                                               AdjGroup<T>& r) {
  using C = BCfg<T>;
  r.gv = *reinterpret_cast<const Vec4<T>*>(S + lane * C::PITCH + b4);
  r.bn = *reinterpret_cast<const Vec4<T>*>(Bn + b4);
  r.bnw = *reinterpret_cast<const Vec4<T>*>(Bnw + b4);
  r.word = SelR[lane * C::SPITCH + (b4 >> 4)];
}

template <typename T>
struct AdjState {
  T toN, toW, toNW, SE;
};

template <typename T>
__device__ __forceinline__ void adj_cells4(AdjState<T>& st, const AdjGroup<T>& r, int b4, Vec4<T>& out) {
  using E = Elem<T>;
#pragma unroll
  for (int q = 3; q >= 0; --q) {
    const uint32_t code = (r.word >> (2 * ((b4 & 15) + q))) & 3u;
    const T sIn = shl1(st.toN, r.bn.v[q]);       // south: lane r+1 one step back; lane 63: band below
    const T seNext = shl1(st.toNW, r.bnw.v[q]);  // south-east for the next step
    T A = E::add(r.gv.v[q], st.SE);
    A = E::add(A, st.toW);
    A = E::add(A, sIn);
    st.toN = code == kSelN ? A : E::zero();
    st.toW = code == kSelW ? A : E::zero();
    st.toNW = code == kSelNW ? A : E::zero();
    st.SE = seNext;
    out.v[q] = A;
  }
}

// Unit u covers slots [S0 - G(u+1), S0 - Gu), groups in descending slot order.
template <typename T, int G>
__device__ __forceinline__ bool adj_unit(T* __restrict__ S, const uint32_t* __restrict__ SelR,
                                         const T* __restrict__ Bn, const T* __restrict__ Bnw, AdjShared& sh,
                                         Control* ctl, int zero, int u, int Us, int S0, AdjState<T>& st,
                                         const AdjUnitRegs<T, G>& in, AdjUnitRegs<T, G>& out, uint32_t& stall,
                                         uint64_t& waited) {
  using C = BCfg<T>;
  constexpr int NG = AdjCfg<T, G>::NG, PD = AdjCfg<T, G>::PD;
  const int lane = threadIdx.x & 63;
  const int top = S0 - G * u, next_top = top - G;
  const bool has_next = u + 1 < Us;
  const uint64_t ready = adj_ready(sh, zero);
  AdjGroup<T> gr[NG + PD];
#pragma unroll
  for (int p = 0; p < PD; ++p) gr[p] = in.g[p];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (g + PD < NG) {
      adj_load_group<T>(S, SelR, Bn, Bnw, (top - 4 * (g + PD + 1)) & C::MASK, lane, gr[g + PD]);
    } else if (has_next) {
      if (g + PD == NG) {
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t need_l = (uint32_t)((G * (u + 1)) / kSub + 1), need_b = (uint32_t)(u + 2);
        if (!__all((uint32_t)ready >= need_l && (uint32_t)(ready >> 32) >= need_b)) {
          ++stall;
          if (!lds_wait_ge(&sh.ctr[0], need_l, &sh.abort, ctl, waited) ||
              !lds_wait_ge(&sh.ctr[1], need_b, &sh.abort, ctl, waited))
            return false;
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      adj_load_group<T>(S, SelR, Bn, Bnw, (next_top - 4 * (g + PD - NG + 1)) & C::MASK, lane, out.g[g + PD - NG]);
    }
    __builtin_amdgcn_sched_barrier(0);
    const int b4 = (top - 4 * (g + 1)) & C::MASK;
    Vec4<T> o;
    adj_cells4<T>(st, gr[g], b4, o);
    *reinterpret_cast<Vec4<T>*>(S + lane * C::PITCH + b4) = o;
  }
  lds_signal(&sh.ctr[2], (uint32_t)(G * (u + 1)));
  __builtin_amdgcn_sched_barrier(0);
  return true;
}

template <typename T, int G>
__device__ __forceinline__ void adj_compute(T* __restrict__ S, const uint32_t* __restrict__ SelR,
                                            const T* __restrict__ Bn, const T* __restrict__ Bnw, AdjShared& sh,
                                            Control* ctl, int Ks, uint64_t* trace) {
  using C = BCfg<T>;
  using E = typename C::E;
  constexpr int PD = AdjCfg<T, G>::PD;
  const int lane = threadIdx.x & 63;
  const int S0 = kSub * Ks;  // slots [0, S0), processed from the top down
  const int Us = S0 / G;
  AdjState<T> st{E::zero(), E::zero(), E::zero(), E::zero()};
  uint64_t waited = 0, t_first = 0;
  uint32_t stall = 0;
  const int zero = adj_opaque_zero();
  {
    const uint64_t ready = adj_ready(sh, zero);
    if (!__all((uint32_t)ready >= 1u && (uint32_t)(ready >> 32) >= 1u)) {
      ++stall;
      if (!lds_wait_ge(&sh.ctr[0], 1u, &sh.abort, ctl, waited) || !lds_wait_ge(&sh.ctr[1], 1u, &sh.abort, ctl, waited)) {
        sh.abort = 1u;
        return;
      }
    }
  }
  if (trace) t_first = __builtin_amdgcn_s_memrealtime();
  AdjUnitRegs<T, G> P, Q;
#pragma unroll
  for (int p = 0; p < PD; ++p) adj_load_group<T>(S, SelR, Bn, Bnw, (S0 - 4 * (p + 1)) & C::MASK, lane, P.g[p]);
  // Units in pairs, so the next unit's prefetched registers alternate between P and Q.
  int u = 0;
  for (; u + 1 < Us; u += 2) {
    if (!adj_unit<T, G>(S, SelR, Bn, Bnw, sh, ctl, zero, u, Us, S0, st, P, Q, stall, waited) ||
        !adj_unit<T, G>(S, SelR, Bn, Bnw, sh, ctl, zero, u + 1, Us, S0, st, Q, P, stall, waited)) {
      sh.abort = 1u;
      return;
    }
  }
  if (u < Us && !adj_unit<T, G>(S, SelR, Bn, Bnw, sh, ctl, zero, u, Us, S0, st, P, Q, stall, waited)) {
    sh.abort = 1u;
    return;
  }
  if (trace && lane == 0) {
    trace[1] = t_first;
    trace[2] = __builtin_amdgcn_s_memrealtime();
    trace[4] = stall;
    trace[8] = waited;
  }
}

// wave 1: loader of gD (plus gscore on the last cell; zeros when gD is absent) and of the
// selection words, one 64-slot sub-chunk at a time from the top slot down.  The loads of
// the next PF sub-chunks are in flight in registers while one is written to LDS.
template <typename T>
struct AdjPF {
  static constexpr int PF = 1;                         // gD sub-chunks
  static constexpr int PFS = 4;                        // selection-word sub-chunks
};

template <typename T>
__device__ __forceinline__ void adj_load_g(Vec4<T> (&x)[16], __amdgpu_buffer_rsrc_t rsrc, int64_t ldg_, int k) {
  const int lane = threadIdx.x & 63;
  // recomputed per call: hoisted out of the loop, the 16 row offsets would stay live
  const int64_t ldg = opaque(ldg_);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = 4 * v + (lane >> 4);
    const int64_t c0 = (int64_t)kSub * k + 4 * (lane & 15) - i;
    const uint32_t off = (uint32_t)(i * ldg + c0) * (uint32_t)sizeof(T);
    if constexpr (sizeof(T) == 4) {
      x[v] = __builtin_bit_cast(Vec4<T>, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)off, 0, 0));
    } else {
      struct Hf { T y[2]; };
      const Hf lo = __builtin_bit_cast(Hf, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)off, 0, 0));
      const Hf hi = __builtin_bit_cast(Hf, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(off + 16), 0, 0));
      x[v].v[0] = lo.y[0]; x[v].v[1] = lo.y[1]; x[v].v[2] = hi.y[0]; x[v].v[3] = hi.y[1];
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

typedef int v4i_t __attribute__((ext_vector_type(4)));

template <typename T, int G>
__device__ __forceinline__ void adj_loader(T* S, uint32_t* SelR, AdjShared& sh, const AdjArgs& a, int band, int Ks) {
  using C = BCfg<T>;
  using E = typename C::E;
  constexpr int PF = AdjPF<T>::PF, PFS = AdjPF<T>::PFS;
  static_assert(PFS % PF == 0, "prefetch depths must nest");
  const int lane = threadIdx.x & 63;
  const int64_t ldg = opaque(a.ldgd), n = opaque(a.n), m = opaque(a.m);
  const int64_t row0 = (int64_t)band * kBand;
  const int rows = (int)(m - row0 < kBand ? m - row0 : kBand);
  const bool has_g = a.gD != nullptr;
  const __amdgpu_buffer_rsrc_t rsrc =
      make_rsrc(has_g ? static_cast<const T*>(a.gD) + row0 * ldg : nullptr,
                has_g ? (uint32_t)(((rows - 1) * ldg + n) * (int64_t)sizeof(T)) : 0u);
  // gscore lands on cell (m-1, n-1): band row m-1-row0, slot n-1 + that row
  const int64_t last_row = m - 1 - row0;
  const bool has_last = last_row >= 0 && last_row < kBand && a.gscore != nullptr;
  const T gs = has_last ? *static_cast<const T*>(a.gscore) : E::zero();
  const int64_t last_slot = n - 1 + last_row;
  const uint32_t* selp = a.sel + sel_index(band, Ks, 0, lane);  // + 256 words per sub-chunk
  uint64_t waited = 0;
  Vec4<T> gbuf[PF][16];
  v4i_t sbuf[PFS];
  // reverse order: the kr-th sub-chunk processed is k = Ks-1-kr
#pragma unroll
  for (int p = 0; p < PFS; ++p)
    if (p < Ks) sbuf[p] = __builtin_nontemporal_load(reinterpret_cast<const v4i_t*>(selp + (int64_t)(Ks - 1 - p) * 256));
  if (has_g) {
#pragma unroll
    for (int p = 0; p < PF; ++p)
      if (p < Ks) adj_load_g<T>(gbuf[p], rsrc, ldg, Ks - 1 - p);
  }
  for (int kr0 = 0; kr0 < Ks; kr0 += PFS) {
#pragma unroll
    for (int p = 0; p < PFS; ++p) {
      const int kr = kr0 + p;
      if (kr >= Ks) break;
      const int k = Ks - 1 - kr;  // sub-chunk (slots [64k, 64k+64))
      const int older = kr - C::RING / kSub;
      if (older >= 0 && (!lds_wait_ge<false>(&sh.ctr[3], (uint32_t)(older + 1), &sh.abort, a.ctl, waited) ||
                         !lds_wait_ge<false>(&sh.ctr[4], (uint32_t)((kSub / G) * (older + 1)), &sh.abort, a.ctl,
                                             waited))) {
        sh.abort = 1u;
        return;
      }
      const bool interior = rows == kBand && k > 0 && (int64_t)kSub * k + kSub <= n;
      Vec4<T>(&gx)[16] = gbuf[p % PF];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = 4 * v + (lane >> 4);
        const int slot = kSub * k + 4 * (lane & 15);
        const int64_t c0 = (int64_t)slot - i;
        Vec4<T> x;
        if (has_g) {
          x = gx[v];
          if (!interior) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (i >= rows || c0 + e < 0 || c0 + e >= n) x.v[e] = E::zero();
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) x.v[e] = E::zero();
        }
        if (has_last && i == (int)last_row) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (last_slot == slot + e) x.v[e] = E::add(x.v[e], gs);
        }
        *reinterpret_cast<Vec4<T>*>(S + i * C::PITCH + (slot & C::MASK)) = x;
      }
      *reinterpret_cast<v4i_t*>(SelR + lane * C::SPITCH + ((4 * k) & (C::SW - 1))) = sbuf[p];
      lds_publish(&sh.ctr[0], (uint32_t)(kr + 1));
      if (kr + PFS < Ks)
        sbuf[p] = __builtin_nontemporal_load(reinterpret_cast<const v4i_t*>(selp + (int64_t)(k - PFS) * 256));
      if (has_g && kr + PF < Ks) adj_load_g<T>(gx, rsrc, ldg, k - PF);
    }
  }
}

// wave 2: values pushed up by the band below (south and south-east of lane 63), G per unit
template <typename T, int G>
__device__ __forceinline__ void adj_poll(T* Bn, T* Bnw, AdjShared& sh, const AdjArgs& a, int band, int Ks,
                                         uint32_t epoch) {
  using C = BCfg<T>;
  using E = typename C::E;
  constexpr int W = E::W;
  const int lane = threadIdx.x & 63;
  const int64_t n = opaque(a.n);
  const int S0 = kSub * Ks, Us = S0 / G;
  const bool bottom = band == a.nb - 1;
  uint64_t waited = 0;
  for (int u = 0; u < Us; ++u) {
    const int64_t need_steps = (int64_t)G * u + G - C::RING;
    if (need_steps > 0 && !lds_wait_ge(&sh.ctr[2], (uint32_t)need_steps, &sh.abort, a.ctl, waited)) {
      sh.abort = 1u;
      return;
    }
    // ring index = slot of lane 63 = column + 63
    const int idx = S0 - G * (u + 1) + lane;
    const int64_t c = (int64_t)idx - (kBand - 1);
    T vn = E::zero(), vnw = E::zero();
    const bool mine = !bottom && lane < G && c >= 0 && c < n;
    if (!bottom) {
      const uint64_t* src = a.bnd + ((int64_t)band * n + (mine ? c : 0)) * 2 * W;
      uint32_t w[2 * W];
      bool ok = !mine;
      if (mine) {
        ok = true;
#pragma unroll
        for (int k = 0; k < 2 * W; ++k) {
          const uint64_t x = load_word(src + k);
          w[k] = (uint32_t)x;
          ok = ok && (uint32_t)(x >> 32) == epoch;
        }
      }
      if (!__all(ok)) {
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        uint32_t polls = 0;
        bool give_up = false;
        while (!__all(ok)) {
          __builtin_amdgcn_s_sleep(1);
          if (!ok) {
            ok = true;
#pragma unroll
            for (int k = 0; k < 2 * W; ++k) {
              const uint64_t x = load_word(src + k);
              w[k] = (uint32_t)x;
              ok = ok && (uint32_t)(x >> 32) == epoch;
            }
          }
          if ((++polls & 63u) == 0u) {
            if (lds_load(&sh.abort) != 0u || global_aborted(a.ctl)) { give_up = true; break; }
            if (__builtin_amdgcn_s_memrealtime() - t0 > kSpinTicks) { raise_timeout(a.ctl); give_up = true; break; }
          }
        }
        waited += __builtin_amdgcn_s_memrealtime() - t0;
        if (give_up) {
          sh.abort = 1u;
          return;
        }
      }
      if (mine) {
        vn = E::from_words(w);
        vnw = E::from_words(w + W);
      }
    }
    if (lane < G) {
      Bn[idx & C::MASK] = vn;
      Bnw[idx & C::MASK] = vnw;
    }
    lds_signal(&sh.ctr[1], (uint32_t)(u + 1));
  }
  (void)waited;
}

// wave 3: storer of gC (= A), one sub-chunk at a time from the top slot down
template <typename T, int G>
__device__ __forceinline__ void adj_store(const T* S, AdjShared& sh, const AdjArgs& a, int band, int Ks) {
  using C = BCfg<T>;
  typedef int v4i __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int64_t ldo = opaque(a.ldgc), n = opaque(a.n), m = opaque(a.m);
  const int64_t row0 = (int64_t)band * kBand;
  const int rows = (int)(m - row0 < kBand ? m - row0 : kBand);
  const __amdgpu_buffer_rsrc_t drs =
      make_rsrc(static_cast<T*>(a.gC) + row0 * ldo, (uint32_t)(((rows - 1) * ldo + n) * (int64_t)sizeof(T)));
  uint64_t waited = 0;
  for (int kr = 0; kr < Ks; ++kr) {
    const int k = Ks - 1 - kr;
    if (!lds_wait_ge(&sh.ctr[2], (uint32_t)(kSub * (kr + 1)), &sh.abort, a.ctl, waited)) {
      sh.abort = 1u;
      return;
    }
    const int j4 = 4 * (lane & 15);
    const int slot = (kSub * k + j4) & C::MASK;
    if (rows == kBand && k > 0 && (int64_t)kSub * k + kSub <= n) {
      Vec4<T> v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = *reinterpret_cast<const Vec4<T>*>(S + (4 * q + (lane >> 4)) * C::PITCH + slot);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = 4 * q + (lane >> 4);
        const int off = (int)(((int64_t)i * ldo + kSub * k + j4 - i) * (int64_t)sizeof(T));
        if constexpr (sizeof(T) == 4) {
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, v[q]), drs, off, 0, 0);
        } else {
          struct Hf { v4i lo, hi; };
          const Hf hh = __builtin_bit_cast(Hf, v[q]);
          __builtin_amdgcn_raw_buffer_store_b128(hh.lo, drs, off, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b128(hh.hi, drs, off + 16, 0, 0);
        }
      }
    } else {
      for (int q = 0; q < 16; ++q) {
        const int i = 4 * q + (lane >> 4);
        if (i >= rows) continue;
        const int64_t c0 = (int64_t)kSub * k + j4 - i;
        const Vec4<T> v = *reinterpret_cast<const Vec4<T>*>(S + i * C::PITCH + slot);
        const int off = (int)(((int64_t)i * ldo + c0) * (int64_t)sizeof(T));
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (c0 + e >= 0 && c0 + e < n) {
            if constexpr (sizeof(T) == 4) {
              __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v.v[e]), drs, off + 4 * e, 0, 0);
            } else {
              typedef int v2i __attribute__((ext_vector_type(2)));
              __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v.v[e]), drs, off + 8 * e, 0, 0);
            }
          }
        }
      }
    }
    lds_publish(&sh.ctr[3], (uint32_t)(kr + 1));
  }
}

// wave 4: publisher of lane 0's pushes to the band above (north and north-west)
template <typename T, int G>
__device__ __forceinline__ void adj_publish(const T* S, const uint32_t* SelR, AdjShared& sh, const AdjArgs& a,
                                            int band, int Ks, uint32_t epoch) {
  using C = BCfg<T>;
  using E = typename C::E;
  constexpr int W = E::W;
  const int lane = threadIdx.x & 63;
  const int64_t n = opaque(a.n);
  const int S0 = kSub * Ks, Us = S0 / G;
  uint64_t waited = 0;
  for (int u = 0; u < Us; ++u) {
    if (!lds_wait_ge(&sh.ctr[2], (uint32_t)(G * (u + 1)), &sh.abort, a.ctl, waited)) {
      sh.abort = 1u;
      return;
    }
    // lane 0 of the compute wave handled slots [S0 - G(u+1), S0 - Gu) = columns
    const int s = S0 - G * (u + 1) + lane;
    if (band > 0 && lane < G && s < n) {
      const T A = S[s & C::MASK];  // row 0
      const uint32_t code = (SelR[(s >> 4) & (C::SW - 1)] >> (2 * (s & 15))) & 3u;
      const T pn = code == kSelN ? A : E::zero();
      const T pnw = code == kSelNW ? A : E::zero();
      uint64_t* dst = a.bnd + ((int64_t)(band - 1) * n + s) * 2 * W;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        store_word(dst + k, tagged(E::word(pn, k), epoch));
        store_word(dst + W + k, tagged(E::word(pnw, k), epoch));
      }
    }
    lds_publish(&sh.ctr[4], (uint32_t)(u + 1));
  }
}

template <typename T, int G>
__global__ __launch_bounds__(kThreads, 1) void adj_kernel(AdjArgs a) {
  using C = BCfg<T>;
  __shared__ Vec4<T> S4[kBand * C::PITCH / 4];
  __shared__ Vec4<T> Bn4[C::RING / 4];
  __shared__ Vec4<T> Bnw4[C::RING / 4];
  __shared__ uint32_t SelR[64 * C::SPITCH];
  __shared__ AdjShared sh;
  T* S = reinterpret_cast<T*>(S4);
  T* Bn = reinterpret_cast<T*>(Bn4);
  T* Bnw = reinterpret_cast<T*>(Bnw4);
  const int wave = threadIdx.x >> 6;
  Control* ctl = a.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int Ks = (int)((a.n + kBand - 1 + kSub - 1) / kSub);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x < 6) sh.ctr[threadIdx.x] = 0u;
    claim_next(ctl, &sh.item, &sh.abort);
    if (sh.item >= (uint32_t)a.nb || sh.abort != 0u) break;
    const int band = a.nb - 1 - (int)sh.item;  // bottom band first
    uint64_t* tr = a.trace ? a.trace + (int64_t)band * kTraceWords : nullptr;
    if (tr && threadIdx.x == 0) tr[0] = __builtin_amdgcn_s_memrealtime();
    if (wave == 0)
      adj_compute<T, G>(S, SelR, Bn, Bnw, sh, ctl, Ks, tr);
    else if (wave == 1)
      adj_loader<T, G>(S, SelR, sh, a, band, Ks);
    else if (wave == 2)
      adj_poll<T, G>(Bn, Bnw, sh, a, band, Ks, epoch);
    else if (wave == 3)
      adj_store<T, G>(S, sh, a, band, Ks);
    else
      adj_publish<T, G>(S, SelR, sh, a, band, Ks, epoch);
    if (tr && threadIdx.x == 3 * 64) tr[3] = __builtin_amdgcn_s_memrealtime();
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

template <typename T>
hipError_t launch_adj_t(int tile, const AdjArgs& a, int grid, hipStream_t s) {
  switch (tile) {
    case 16: hipLaunchKernelGGL((adj_kernel<T, 16>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 32: hipLaunchKernelGGL((adj_kernel<T, 32>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 64: hipLaunchKernelGGL((adj_kernel<T, 64>), dim3(grid), dim3(kThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_select(int dtype, const SelArgs& a, int grid, hipStream_t s) {
  switch (dtype) {
    case 0: hipLaunchKernelGGL((sel_kernel<float>), dim3(grid), dim3(128), 0, s, a); break;
    case 1: hipLaunchKernelGGL((sel_kernel<double>), dim3(grid), dim3(128), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(int dtype, int tile, const AdjArgs& a, int grid, hipStream_t s) {
  switch (dtype) {
    case 0: return launch_adj_t<float>(tile, a, grid, s);
    case 1: return launch_adj_t<double>(tile, a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wf
