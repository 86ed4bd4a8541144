// Smooth (soft-min) variant of the wavefront recurrence on gfx950 (wf_soft_forward,
// wf_soft_backward in include/wf.h).
//
// The minimum of the north-west, north and west neighbours is replaced by the soft minimum
// of temperature gamma,  softmin(x) = -gamma log sum_k exp(-x_k / gamma),  evaluated about
// the smallest argument mn:  softmin = mn - gamma ln2 log2( sum_k 2^((mn - x_k) log2e / gamma) ).
// The adjoint of  L = sum(gD * D) + gscore * score  is
//     A[i][j] = gD[i][j] + [last] gscore + w(i+1,j+1) A[i+1][j+1] + w(i+1,j) A[i+1][j]
//             + w(i,j+1) A[i][j+1],       w(succ) = 2^((V(succ) - D[i][j]) log2e / gamma),
// with V(succ) = D(succ) - C(succ) the successor's soft minimum, so the weight is the
// derivative of the successor's soft minimum with respect to D[i][j].  gC = A.  The
// exponent is evaluated as (D(succ) - D[i][j]) log2e/gamma - C(succ) log2e/gamma, one fused
// multiply-add after the difference of two neighbouring table values, which is exact in
// floating point, so the weight's error is that of numbers of the size of C, not of the
// table.  (Forming V first would round it at the
// table's magnitude, and along a path of L cells those roundings add up: at 16384 x 16384
// in float32 that made the first cell's gradient 8% off.)
//
// The forward runs in the min-plus forward's band pipeline (wf_fwd.hip) with the soft-min
// cell in place of the minimum; this file holds the adjoint, a band pipeline of six waves
// per 64-row band (described with its kernel below).  Every wait is bounded.
#include "wf_common.h"
#include "wf_soft.h"

#include <type_traits>

namespace wf {
namespace {

constexpr int kRing = 512;   // handoff ring: columns
constexpr int kFill = 128;   // fill columns after the last one (at least the groups' overhang)

// Four consecutive columns of one row, as one (float) or two (double) 16-byte transfers.
template <typename T>
__device__ __forceinline__ Vec4<T> load4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  Vec4<T> v;
  if constexpr (sizeof(T) == 4) {
    v = __builtin_bit_cast(Vec4<T>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  } else {
    using H = struct alignas(16) { uint32_t w[4]; };
    H lo = __builtin_bit_cast(H, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    H hi = __builtin_bit_cast(H, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0));
    uint32_t w[8];
    for (int q = 0; q < 4; ++q) {
      w[q] = lo.w[q];
      w[4 + q] = hi.w[q];
    }
    __builtin_memcpy(&v, w, sizeof(v));
  }
  return v;
}

// wave_shl:1 -- lane r receives lane r+1's value; lane 63 keeps 'old'.
template <typename T>
__device__ __forceinline__ T shl1_(T src, T old) {
  auto mv = [](uint32_t s, uint32_t o) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)o, (int)s, 0x130, 0xf, 0xf, false);
  };
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, mv(__builtin_bit_cast(uint32_t, src), __builtin_bit_cast(uint32_t, old)));
  } else {
    const uint64_t s = __builtin_bit_cast(uint64_t, src), o = __builtin_bit_cast(uint64_t, old);
    const uint64_t lo = mv((uint32_t)s, (uint32_t)o), hi = mv((uint32_t)(s >> 32), (uint32_t)(o >> 32));
    return __builtin_bit_cast(T, (hi << 32) | lo);
  }
}

template <typename T>
__device__ __forceinline__ void store1(__amdgpu_buffer_rsrc_t r, uint32_t off, T x) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, off, 0, 0);
  } else {
    using V2 = __attribute__((ext_vector_type(2))) uint32_t;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, off, 0, 0);
  }
}

// Range-checked resource over rows [row0, row0 + rows) of a matrix with leading dimension
// ld: the last row ends at its n-th element, so nothing past the caller's data is touched.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t band_rsrc(const void* base, int64_t row0, int rows, int64_t ld,
                                                            int64_t n) {
  const T* p = static_cast<const T*>(base) + row0 * ld;
  const int64_t bytes = rows > 0 ? ((int64_t)(rows - 1) * ld + n) * (int64_t)sizeof(T) : 0;
  return make_rsrc(p, (uint32_t)bytes);
}

struct alignas(8) SoftShared {
  uint32_t avail;     // handoff columns in the ring, in the consumer's order
  uint32_t used;      // columns the compute wave has finished with
  uint32_t item;
  uint32_t abort;
  uint32_t produced;  // steps whose edge-row values the compute wave has put in the out ring
  uint32_t pubd;      // steps whose values the publisher has stored
  uint32_t ld[2];     // adjoint: sub-chunks of D and of C staged in LDS
  uint32_t done;      // adjoint: sub-chunks the compute wave has finished
  uint32_t stored;    // adjoint: sub-chunks of gC the storer has written back
};

// Out ring: the compute wave's edge-row values (NV per step) for the publisher wave, which
// turns them into coalesced tagged words; kPub steps.
constexpr int kPub = 256;

// The publisher wave: stores the values of steps [0, total) of the out ring as tagged words,
// 64 steps per pass, as the compute wave produces them.  Step s holds the values of column
// col(s) (or none, outside [0, n)); 'dst(c, v)' is the first word of value v of column c.
template <typename T, int NV, typename Col, typename Dst>
__device__ __forceinline__ bool publish_ring(const T* pub, SoftShared& sh, Control* ctl, int64_t n, uint32_t total,
                                             uint32_t epoch, Col col, Dst dst) {
  using E = Elem<T>;
  constexpr int W = E::W;
  const int lane = threadIdx.x & 63;
  uint64_t waited = 0;
  uint32_t ps = 0;
  while (ps < total) {
    uint32_t have;
    if (!lds_wait_value<true, false>(&sh.produced, ps + 1, &sh.abort, ctl, waited, have)) return false;
    const uint32_t pe = have < ps + 64 ? have : ps + 64;
    const uint32_t st = ps + (uint32_t)lane;
    if (st < pe) {
      const int64_t c = col((int64_t)st);
      if (c >= 0 && c < n) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const T x = pub[v * kPub + (int)(st & (kPub - 1))];
          uint64_t* d = dst(c, v);
#pragma unroll
          for (int w = 0; w < W; ++w) store_word(d + w, tagged(E::word(x, w), epoch));
        }
      }
    }
    ps = pe;
    lds_signal(&sh.pubd, ps);
  }
  return true;
}

// ---------------------------------------------------------------------------------------
// The poller: fetches the producer band's tagged words, 64 columns per pass from the first
// one not yet handed over, and hands over the leading run of complete columns.  NV values
// per column (the adjoint's A, D and scaled C), each of W payload words; 'word_at(k)' is the
// address of the first word of consumer column k.  After the last column it writes 'fill'
// into the next kFill columns of the ring and counts them as delivered.
template <typename T, int NV, typename WordAt>
__device__ __forceinline__ bool poll_ring(T* ring, SoftShared& sh, Control* ctl, int64_t n, uint32_t epoch,
                                          const T (&fill)[NV], WordAt word_at) {
  using E = Elem<T>;
  constexpr int W = E::W;
  const int lane = threadIdx.x & 63;
  uint64_t waited = 0, t0 = 0;
  uint32_t polls = 0;
  int64_t u = 0;
  while (u < n) {
    // ring slots of columns u .. u+63 are free once the compute wave is past column u+63-kRing
    const int64_t need = u + 64 - kRing;
    if (need > 0 && !lds_wait_ge(&sh.used, (uint32_t)need, &sh.abort, ctl, waited)) return false;
    const int64_t k = u + lane;
    const bool real = k < n;
    const uint64_t* src = real ? word_at(k) : reinterpret_cast<const uint64_t*>(ctl) + 4;
    // Two polls in flight: while one pass's words are checked, the next pass's are on their
    // way, so readiness is seen about half a round trip sooner than with one.
    uint64_t xa[NV * W], xb[NV * W];
    auto issue = [&](uint64_t (&x)[NV * W]) {
#pragma unroll
      for (int q = 0; q < NV * W; ++q) x[q] = load_word(src + q);
    };
    // the leading run of complete columns in x (columns past the matrix count as complete)
    auto complete = [&](const uint64_t (&x)[NV * W]) -> int {
      bool ok = true;
#pragma unroll
      for (int q = 0; q < NV * W; ++q) ok = ok && (uint32_t)(x[q] >> 32) == epoch;
      ok = ok || !real;
      const uint64_t okm = __ballot(ok);
      const int run = ~okm == 0 ? 64 : __builtin_ctzll(~okm);
      return (int)(run < n - u ? run : n - u);
    };
    // false when the wait has to give up
    auto pause = [&]() -> bool {
      if (polls == 0) t0 = __builtin_amdgcn_s_memrealtime();
      __builtin_amdgcn_s_sleep(1);
      if ((++polls & 63u) == 0u) {
        if (lds_load(&sh.abort) != 0u || global_aborted(ctl)) return false;
        if (__builtin_amdgcn_s_memrealtime() - t0 > kSpinTicks) {
          raise_timeout(ctl);
          return false;
        }
      }
      return true;
    };
    auto deliver = [&](const uint64_t (&x)[NV * W], int take) {
      if (lane < take) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          uint32_t w[W];
#pragma unroll
          for (int q = 0; q < W; ++q) w[q] = (uint32_t)x[v * W + q];
          ring[v * kRing + (int)((u + lane) & (kRing - 1))] = E::from_words(w);
        }
      }
      u += take;
      lds_publish(&sh.avail, (uint32_t)u);
    };
    issue(xa);
    for (;;) {
      issue(xb);
      int take = complete(xa);
      if (take > 0) {
        deliver(xa, take);
        break;
      }
      if (!pause()) return false;
      issue(xa);
      take = complete(xb);
      if (take > 0) {
        deliver(xb, take);
        break;
      }
      if (!pause()) return false;
    }
    polls = 0;
  }
  // the kFill columns after the last one hold 'fill', so that the consumer's vector reads of
  // them need no selects; they count as delivered once written
  if (n + kFill - kRing > 0 && !lds_wait_ge(&sh.used, (uint32_t)(n + kFill - kRing), &sh.abort, ctl, waited))
    return false;
  for (int c = lane; c < kFill; c += 64) {
#pragma unroll
    for (int v = 0; v < NV; ++v) ring[v * kRing + (int)((n + c) & (kRing - 1))] = fill[v];
  }
  lds_publish(&sh.avail, (uint32_t)(n + kFill));
  return true;
}

// ---------------------------------------------------------------------------------------
// Adjoint: a band pipeline of six waves per 64-row band, bands claimed bottom-up.
//
// Lane r owns band row r and at step t handles column n + 62 - r - t (the bottom row leads,
// right to left).  D and C are staged in two skewed LDS rings: element (row r, column c) sits
// at slot (n + 62 - r - c) mod RING, the step that uses it, so at step t every lane touches
// slot t and four steps are one aligned 16-byte LDS read per ring.  Slots [4j, 4j+4) of a row
// hold four consecutive columns in descending order, one (4-byte aligned) 16-byte global
// transfer with its elements reversed.  The compute wave writes A over C in place; a storer
// wave writes it back as gC.
//   wave 0  compute   per 4 steps: the D and C vectors (read one group ahead), the band
//                     below's (A, D, C log2e/gamma) from the handoff ring, 3 x 4 weights,
//                     the A vector back to LDS, and row 0's (A, D, C log2e/gamma) into the
//                     out ring;
//   wave 1  loader    sub-chunks of D (SUB slots of every row), one in flight in registers;
//   wave 2  loader    the same for C;
//   wave 3  poller    the band below's row-0 (A, D, C log2e/gamma) words into the handoff ring;
//   wave 4  storer    each finished sub-chunk's A back to gC;
//   wave 5  publisher this band's row-0 (A, D, C log2e/gamma) words for the band above.
// With an upstream gD the compute wave reads it straight from global memory along its own
// row, issued PD groups ahead (a third ring does not fit in LDS).
template <typename T>
struct SbCfg {
  static constexpr int RING = sizeof(T) == 4 ? 256 : 128;   // slots per row (about 64 KiB a ring)
  static constexpr int SUB = sizeof(T) == 4 ? 64 : 32;      // slots per sub-chunk
  static constexpr int PITCH = RING + 16 / (int)sizeof(T);  // row pitch 16 mod 256 bytes
  static constexpr int MASK = RING - 1;
  static constexpr int CPR = SUB / 4;                       // 4-slot chunks per row of a sub-chunk
  static constexpr int RPV = 64 / CPR;                      // rows one vector index spans across the wave
  static constexpr int NV = CPR;                            // vectors per lane per sub-chunk
  static constexpr int GPS = SUB / 4;                       // 4-step groups per sub-chunk
  static constexpr int NSUB = RING / SUB;                   // sub-chunks the ring holds
  static constexpr int PF = 1;                              // sub-chunks a loader keeps in flight
  static constexpr int PD = sizeof(T) == 4 ? 8 : 2;         // gD groups in flight (divides GPS)
  static_assert(NSUB >= 4 && GPS % PD == 0, "bad tiling");
};

constexpr int kSbThreads = 6 * 64;

// Returns x unchanged, but hides its value from the optimiser at this point: each role
// launders the kernel-wide sizes it uses, or the compiler hoists every role's address
// arithmetic out of the band loop and keeps all of it live across all roles.
template <typename V>
__device__ __forceinline__ V opaque(V x) {
  asm volatile("" : "+s"(x));
  return x;
}
// The same for a per-lane value.
__device__ __forceinline__ int opaque_lane() {
  int x = (int)(threadIdx.x & 63);
  asm volatile("" : "+v"(x));
  return x;
}

template <typename T>
__device__ __forceinline__ void store4(__amdgpu_buffer_rsrc_t r, uint32_t off, const Vec4<T>& v) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, v), r, off, 0, 0);
  } else {
    struct Hf { v4i lo, hi; };
    const Hf h = __builtin_bit_cast(Hf, v);
    __builtin_amdgcn_raw_buffer_store_b128(h.lo, r, off, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b128(h.hi, r, off + 16, 0, 0);
  }
}

template <typename T>
__device__ __forceinline__ Vec4<T> reversed(const Vec4<T>& v) {
  Vec4<T> o;
#pragma unroll
  for (int e = 0; e < 4; ++e) o.v[e] = v.v[3 - e];
  return o;
}

// Vector k of a lane in sub-chunk s: row i, slots t0 .. t0+3, which hold columns c_lo+3 down
// to c_lo.  32-bit arithmetic: a band spans less than 2^30 bytes (the leading-dimension
// limit of the entry points), so every element offset within it fits.
template <typename T>
struct SbVec {
  int i;
  int t0;
  int c_lo;
  __device__ __forceinline__ SbVec(int lane, int k, int s, int n) {
    using K = SbCfg<T>;
    i = K::RPV * k + lane / K::CPR;
    t0 = K::SUB * s + 4 * (lane % K::CPR);
    c_lo = n + 59 - i - t0;
  }
  __device__ __forceinline__ int lds(int pitch) const { return i * pitch + (t0 & SbCfg<T>::MASK); }
};

template <typename T>
__device__ __forceinline__ T load1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
}

// Four consecutive elements from element offset e of a resource.  Offsets below 0 (columns
// below 0, near the left edge only) read element 0 instead: those positions hold no data
// that a real cell uses.
template <typename T>
__device__ __forceinline__ Vec4<T> sb_load4(__amdgpu_buffer_rsrc_t r, int e) {
  if (__all(e >= 0)) return load4<T>(r, (uint32_t)e * (uint32_t)sizeof(T));
  Vec4<T> v;
#pragma unroll
  for (int q = 0; q < 4; ++q) v.v[q] = load1<T>(r, (uint32_t)(e + q > 0 ? e + q : 0) * (uint32_t)sizeof(T));
  return v;
}

// Loads sub-chunk s of one input.  Columns past the row's end read the next row (or zeros
// past the band's end), columns below 0 the row before (or nothing, before the band's
// start); none of them reaches a real cell.
template <typename T>
__device__ __forceinline__ void sb_load_sub(Vec4<T> (&buf)[SbCfg<T>::NV], __amdgpu_buffer_rsrc_t rsrc, int ld, int n,
                                            int s, int lane) {
  using K = SbCfg<T>;
  __builtin_amdgcn_sched_barrier(0);
  // an element offset is at least n + 63 - SUB (s+1): below 0 in the last sub-chunks only
  if (n + 63 >= K::SUB * (s + 1)) {
#pragma unroll
    for (int k = 0; k < K::NV; ++k) {
      const SbVec<T> v(lane, k, s, n);
      buf[k] = load4<T>(rsrc, (uint32_t)(v.i * ld + v.c_lo) * (uint32_t)sizeof(T));
    }
  } else {
#pragma unroll
    for (int k = 0; k < K::NV; ++k) {
      const SbVec<T> v(lane, k, s, n);
      buf[k] = sb_load4<T>(rsrc, v.i * ld + v.c_lo);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// waves 1 and 2: one input into its ring.  Sub-chunk s reuses the slots of sub-chunk
// s - NSUB, which 'freed' must have released.
template <typename T>
__device__ __forceinline__ bool sb_loader(T* P, SoftShared& sh, const SoftArgs& a, const void* src, int64_t ld64,
                                          int band, int Ks, uint32_t* cnt, const uint32_t* freed) {
  using K = SbCfg<T>;
  const int n = (int)opaque(a.n);
  const int ld = (int)opaque(ld64);
  const int lane = opaque_lane();
  const int64_t row0 = (int64_t)band * kBand;
  const int rows = (int)(a.m - row0 < kBand ? a.m - row0 : kBand);
  const __amdgpu_buffer_rsrc_t rsrc = band_rsrc<T>(src, row0, rows, ld, n);
  uint64_t waited = 0;
  Vec4<T> buf[K::PF][K::NV];
#pragma unroll
  for (int p = 0; p < K::PF; ++p) sb_load_sub<T>(buf[p], rsrc, ld, n, p, lane);
  for (int s0 = 0; s0 < Ks; s0 += K::PF) {
#pragma unroll
    for (int p = 0; p < K::PF; ++p) {
      const int s = s0 + p;
      if (s < Ks) {
        const int older = s - K::NSUB;
        if (older >= 0 && !lds_wait_ge<false>(freed, (uint32_t)(older + 1), &sh.abort, a.ctl, waited)) return false;
#pragma unroll
        for (int k = 0; k < K::NV; ++k) {
          const SbVec<T> v(lane, k, s, n);
          *reinterpret_cast<Vec4<T>*>(P + v.lds(K::PITCH)) = reversed(buf[p][k]);
        }
        lds_signal(cnt, (uint32_t)(s + 1));
        if (s + K::PF < Ks) sb_load_sub<T>(buf[p], rsrc, ld, n, s + K::PF, lane);
      }
    }
  }
  return true;
}

// wave 4: gC from the C ring (which the compute wave overwrote with A).
template <typename T>
__device__ __forceinline__ bool sb_store(const T* P, SoftShared& sh, const SoftArgs& a, int band, int Ks) {
  using K = SbCfg<T>;
  const int n = (int)opaque(a.n);
  const int lane = opaque_lane();
  const int64_t row0 = (int64_t)band * kBand;
  const int rows = (int)(a.m - row0 < kBand ? a.m - row0 : kBand);
  const int ldgc = (int)opaque(a.ldgc);
  const __amdgpu_buffer_rsrc_t ro = band_rsrc<T>(a.gC, row0, rows, ldgc, n);
  constexpr uint32_t es = sizeof(T);
  uint64_t waited = 0;
  for (int s = 0; s < Ks; ++s) {
    if (!lds_wait_ge(&sh.done, (uint32_t)(s + 1), &sh.abort, a.ctl, waited)) return false;
    // every row real and every column in [0, n): columns n - SUB(s+1) .. n + 62 - SUB s
    if (rows == kBand && K::SUB * s >= 63 && K::SUB * (s + 1) <= n) {
      Vec4<T> v[K::NV];
#pragma unroll
      for (int k = 0; k < K::NV; ++k) {
        const SbVec<T> q(lane, k, s, n);
        v[k] = reversed(*reinterpret_cast<const Vec4<T>*>(P + q.lds(K::PITCH)));
      }
#pragma unroll
      for (int k = 0; k < K::NV; ++k) {
        const SbVec<T> q(lane, k, s, n);
        store4<T>(ro, (uint32_t)(q.i * ldgc + q.c_lo) * es, v[k]);
      }
    } else {
      // the edge sub-chunks at a band's two ends: one vector at a time, in a loop (one copy
      // of this code instead of sixteen)
#pragma unroll 1
      for (int k = 0; k < K::NV; ++k) {
        const SbVec<T> q(lane, k, s, n);
        if (q.i >= rows) continue;
        const Vec4<T> x = reversed(*reinterpret_cast<const Vec4<T>*>(P + q.lds(K::PITCH)));
        if (q.c_lo >= 0 && q.c_lo + 4 <= n) {
          store4<T>(ro, (uint32_t)(q.i * ldgc + q.c_lo) * es, x);
          continue;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = q.c_lo + e;
          if (c >= 0 && c < n) store1<T>(ro, (uint32_t)(q.i * ldgc + c) * es, x.v[e]);
        }
      }
    }
    lds_publish(&sh.stored, (uint32_t)(s + 1));
  }
  return true;
}

// Both loader counters in one 8-byte LDS read: sub-chunk s of D and of C is in LDS.
__device__ __forceinline__ bool sb_loaded(const SoftShared& sh, int s) {
  const uint64_t w =
      __hip_atomic_load(reinterpret_cast<const uint64_t*>(&sh.ld[0]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)w);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(w >> 32));
  return lo >= (uint32_t)(s + 1) && hi >= (uint32_t)(s + 1);  // wave-uniform
}

// wave 0: the adjoint chain.  BOTTOM: the matrix's last band, whose successors below lie
// outside (A = 0, V = -inf) and which reads no handoff.
template <typename T, bool HAS_GD, bool BOTTOM>
__device__ __forceinline__ bool sb_compute(const T* __restrict__ Dp, T* __restrict__ Cp, const T* ring, T* pub,
                                           SoftShared& sh, const SoftArgs& a, int band, int Ks) {
  using E = Elem<T>;
  using M = SoftMath<T>;
  using K = SbCfg<T>;
  constexpr int PD = K::PD;
  const int lane = opaque_lane();
  const int64_t m = opaque(a.m), n = opaque(a.n);
  const int64_t row0 = (int64_t)band * kBand;
  const int rows = (int)(m - row0 < kBand ? m - row0 : kBand);
  const bool live = lane < rows;
  const int n32 = (int)n;
  const bool score_lane = lane == rows - 1;  // in the last band: the matrix's last row
  const T kx = (T)a.kx;
  const bool pubband = band > 0;  // a band above reads this band's first row
  const bool publish = lane == 0 && pubband;
  const T gs = a.gscore ? *static_cast<const T*>(a.gscore) : E::zero();
  const T NEG = -E::inf();
  const int64_t groups = (int64_t)Ks * K::GPS;
  // groups [g_lo, g_hi) have every lane's four columns inside the matrix (a full band only):
  // lane 0's highest column n+62-4g <= n-1 needs g >= 16, lane 63's lowest n-4-4g >= 0 needs
  // g <= (n-4)/4
  const int64_t g_lo = rows == kBand ? 16 : groups, g_hi = rows == kBand && n >= 4 ? (n - 4) / 4 + 1 : 0;
  __amdgpu_buffer_rsrc_t rg;
  Vec4<T> gb[PD];
  int gbase = 0;  // element offset of this lane's column n + 59 - lane (32-bit: see SbVec)
  if constexpr (HAS_GD) {
    const int ldgd = (int)opaque(a.ldgd);
    rg = band_rsrc<T>(a.gD, row0, rows, ldgd, n);
    gbase = lane * ldgd + (int)n + 59 - lane;
#pragma unroll
    for (int k = 0; k < PD; ++k) gb[k] = sb_load4<T>(rg, gbase - 4 * k);
  }
  // A, D and C log2(e)/gamma of the east successor (this lane's previous cell) and of the
  // south successor of the previous step (the south-east one now); a weight's exponent is
  // (D(succ) - D) log2(e)/gamma - C(succ) log2(e)/gamma, one fused multiply-add after an
  // exact difference.  A successor outside the matrix has A = 0, D = -inf, C = 0: its weight
  // is exactly 0.
  T Ae = E::zero(), De = NEG, Ce = E::zero();
  T Aso = E::zero(), Dso = NEG, Cso = E::zero();
  uint64_t waited = 0;
  // Consumer columns of the band below's first row known to be in the handoff ring
  // (wave-uniform); 'pend' is the counter read issued one group earlier, so that no group
  // waits for it.  Group g reads the ring's columns 4g .. 4g+3, which past the last column
  // hold the fill values the poller writes after it (counted as kFill more columns).
  uint32_t have = 0u, pend = 0u;
  auto need_of = [&](int64_t g) -> int64_t { return 4 * g + 4 <= n ? 4 * g + 4 : n + kFill; };
  auto avail_for = [&](int64_t g) -> bool {
    const int64_t need = need_of(g);
    if (need <= (int64_t)have) return true;
    uint32_t seen;
    if (!lds_wait_value<true, false>(&sh.avail, (uint32_t)need, &sh.abort, a.ctl, waited, seen)) return false;
    have = (uint32_t)__builtin_amdgcn_readfirstlane((int)seen);
    return true;
  };
  // the band below's row-0 (A, D, C) at lane 63's columns n-1-4g-q, consumer order 4g+q: one
  // aligned vector per plane, read unconditionally (a read under a condition would make the
  // wave wait for it where the paths join)
  auto read_bottom = [&](int64_t g, Vec4<T>& va, Vec4<T>& vd, Vec4<T>& vc) {
    const int sl = (int)((4 * g) & (kRing - 1));
    va = *reinterpret_cast<const Vec4<T>*>(ring + sl);
    vd = *reinterpret_cast<const Vec4<T>*>(ring + kRing + sl);
    vc = *reinterpret_cast<const Vec4<T>*>(ring + 2 * kRing + sl);
  };
  Vec4<T> ba, bd, bc;
  if constexpr (BOTTOM) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ba.v[q] = E::zero();
      bd.v[q] = NEG;
      bc.v[q] = E::zero();
    }
  } else {
    if (!avail_for(0)) return false;
    read_bottom(0, ba, bd, bc);
  }
  const T* Drow = Dp + lane * K::PITCH;
  T* Crow = Cp + lane * K::PITCH;
  auto wait_loaded = [&](int s) -> bool {
    return lds_wait_until([&] { return sb_loaded(sh, s); }, &sh.abort, a.ctl, waited);
  };
  if (!wait_loaded(0)) return false;
  Vec4<T> dn = *reinterpret_cast<const Vec4<T>*>(Drow), cn = *reinterpret_cast<const Vec4<T>*>(Crow);
  for (int s = 0; s < Ks; ++s) {
    for (int64_t g0 = (int64_t)s * K::GPS; g0 < (int64_t)(s + 1) * K::GPS; g0 += PD) {
      // the batch's out-ring slots must have been published
      if (pubband && 4 * (g0 + PD) > kPub &&
          !lds_wait_ge(&sh.pubd, (uint32_t)(4 * (g0 + PD) - kPub), &sh.abort, a.ctl, waited))
        return false;
      // One 4-step group; false when a wait has to give up.  PATH: 0 picks the interior or
      // the edge path per group, 1 takes the interior path, 2 the edge path (which is right
      // for every group, only slower).
      auto group = [&](int k, auto path) -> bool {
        constexpr int PATH = decltype(path)::value;
        const int64_t g = g0 + k;
        if constexpr (!BOTTOM) {
          // The counter read issued a group ago, into a scalar before any of this group's
          // reads are issued: waiting for it then waits for nothing recent.
          const uint32_t p = (uint32_t)__builtin_amdgcn_readfirstlane((int)pend);
          have = p > have ? p : have;
          __builtin_amdgcn_sched_barrier(0);
        }
        const Vec4<T> dg = dn;
        Vec4<T> cg;  // C log2(e)/gamma
#pragma unroll
        for (int q = 0; q < 4; ++q) cg.v[q] = cn.v[q] * kx;
        // the next group's D and C: in this sub-chunk, or in the next one if already loaded
        const bool next_sub = (g + 1) % K::GPS == 0;
        const bool pre = g + 1 < groups && (!next_sub || sb_loaded(sh, s + 1));
        if (pre) {
          const int sl = (int)((4 * (g + 1)) & K::MASK);
          dn = *reinterpret_cast<const Vec4<T>*>(Drow + sl);
          cn = *reinterpret_cast<const Vec4<T>*>(Crow + sl);
        }
        Vec4<T> gg;
        if constexpr (HAS_GD) {
          gg = gb[k];
          gb[k] = sb_load4<T>(rg, gbase - 4 * (int)(g + PD));
        }
        // the next group's handoff values, valid if the counter read before them covers them
        Vec4<T> na = ba, nd = bd, nc = bc;
        bool n_ready = true;
        if constexpr (!BOTTOM) {
          n_ready = need_of(g + 1) <= (int64_t)have;
          read_bottom(g + 1, na, nd, nc);
          pend = lds_load(&sh.avail);
          // keeps later ring reads after this counter read (the LDS performs one wave's
          // accesses in order)
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        // this lane's column at step 4g (32-bit: n < 2^31, and the edge path below runs in
        // every band's first and last groups, on the critical path of the band below's start)
        const int j0 = n32 + 62 - lane - 4 * (int)g;
        const bool interior = PATH == 1 || (PATH == 0 && g >= g_lo && g < g_hi);
        Vec4<T> out;
        if (interior) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const T As = shl1_(Ae, ba.v[q]), Ds = shl1_(De, bd.v[q]), Cs = shl1_(Ce, bc.v[q]);
            const T dd = dg.v[q], cc = cg.v[q];
            T acc = HAS_GD ? gg.v[3 - q] : E::zero();
            acc = M::fma_(M::exp2_(M::fma_(Dso - dd, kx, -Cso)), Aso, acc);
            acc = M::fma_(M::exp2_(M::fma_(Ds - dd, kx, -Cs)), As, acc);
            acc = M::fma_(M::exp2_(M::fma_(De - dd, kx, -Ce)), Ae, acc);
            Aso = As;
            Dso = Ds;
            Cso = Cs;
            Ae = acc;
            De = dd;
            Ce = cc;
            out.v[q] = acc;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = j0 - q;
            const bool valid = live && (uint32_t)j < (uint32_t)n32;
            const T As = shl1_(Ae, ba.v[q]), Ds = shl1_(De, bd.v[q]), Cs = shl1_(Ce, bc.v[q]);
            const T dd = dg.v[q], cc = cg.v[q];
            T acc = HAS_GD ? gg.v[3 - q] : E::zero();
            if constexpr (BOTTOM) {
              // the score's cell: the matrix's last row, last column
              if (score_lane && j == n32 - 1) acc = acc + gs;
            }
            acc = M::fma_(M::exp2_(M::fma_(Dso - dd, kx, -Cso)), Aso, acc);
            acc = M::fma_(M::exp2_(M::fma_(Ds - dd, kx, -Cs)), As, acc);
            acc = M::fma_(M::exp2_(M::fma_(De - dd, kx, -Ce)), Ae, acc);
            Aso = As;
            Dso = Ds;
            Cso = Cs;
            Ae = valid ? acc : E::zero();
            De = valid ? dd : NEG;
            Ce = valid ? cc : E::zero();
            out.v[q] = Ae;
          }
        }
        *reinterpret_cast<Vec4<T>*>(Crow + ((4 * g) & K::MASK)) = out;
        if (publish) {
          // lane 0's (A, D, C) of steps 4g .. 4g+3 (columns j0 .. j0-3) to the out ring
          const int ps = (int)((4 * g) & (kPub - 1));
          *reinterpret_cast<Vec4<T>*>(pub + ps) = out;
          *reinterpret_cast<Vec4<T>*>(pub + kPub + ps) = dg;
          *reinterpret_cast<Vec4<T>*>(pub + 2 * kPub + ps) = cg;
          lds_signal(&sh.produced, (uint32_t)(4 * g + 4));
        }
        if constexpr (!BOTTOM) {
          if (!n_ready && g + 1 < groups) {
            if (!avail_for(g + 1)) return false;
            read_bottom(g + 1, na, nd, nc);
          }
        }
        ba = na;
        bd = nd;
        bc = nc;
        if (!pre && g + 1 < groups) {
          if (!wait_loaded(s + 1)) return false;
          const int sl = (int)((4 * (g + 1)) & K::MASK);
          dn = *reinterpret_cast<const Vec4<T>*>(Drow + sl);
          cn = *reinterpret_cast<const Vec4<T>*>(Crow + sl);
        }
        return true;
      };
      if constexpr (HAS_GD) {
        // the g_D registers need constant indices: every group of the block unrolled
#pragma unroll
        for (int k = 0; k < PD; ++k)
          if (!group(k, std::integral_constant<int, 0>())) return false;
      } else if (g0 >= g_lo && g0 + PD <= g_hi) {
        // Interior blocks, nearly all of them, unrolled with the interior path only; the few
        // edge blocks at a band's two ends loop over one copy of the edge path.  Half the
        // code of unrolling both paths: a band starts on a compute unit whose instruction
        // cache has never held the loop, and the fetch of each new line is on the critical
        // path of the band above.
#pragma unroll
        for (int k = 0; k < PD; ++k)
          if (!group(k, std::integral_constant<int, 1>())) return false;
      } else {
#pragma unroll 1
        for (int k = 0; k < PD; ++k)
          if (!group(k, std::integral_constant<int, 2>())) return false;
      }
      if (!BOTTOM && lane == 0) lds_signal(&sh.used, (uint32_t)(4 * (g0 + PD) < n ? 4 * (g0 + PD) : n));
    }
    lds_signal(&sh.done, (uint32_t)(s + 1));
  }
  return true;
}

template <typename T, bool HAS_GD>
__global__ __launch_bounds__(kSbThreads, 1) void soft_bwd_kernel(SoftArgs a) {
  using E = Elem<T>;
  using K = SbCfg<T>;
  __shared__ Vec4<T> D4[kBand * K::PITCH / 4];
  __shared__ Vec4<T> C4[kBand * K::PITCH / 4];
  __shared__ alignas(16) T ring[3 * kRing];
  __shared__ alignas(16) T pub[3 * kPub];
  __shared__ SoftShared sh;
  T* Dp = reinterpret_cast<T*>(D4);
  T* Cp = reinterpret_cast<T*>(C4);
  Control* ctl = a.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      sh.avail = 0u;
      sh.used = 0u;
      sh.produced = 0u;
      sh.pubd = 0u;
      sh.ld[0] = 0u;
      sh.ld[1] = 0u;
      sh.done = 0u;
      sh.stored = 0u;
    }
    claim_next(ctl, &sh.item, &sh.abort);
    // bands from the bottom up
    const int band = a.nb - 1 - (int)sh.item;
    if ((int)sh.item >= a.nb || sh.abort != 0u) break;
    bool ok = true;
    const int64_t n = a.n;
    const int Ks = (int)((n + 63 + K::SUB - 1) / K::SUB);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform branches below
    if (wave == 0) {
      ok = band == a.nb - 1 ? sb_compute<T, HAS_GD, true>(Dp, Cp, ring, pub, sh, a, band, Ks)
                            : sb_compute<T, HAS_GD, false>(Dp, Cp, ring, pub, sh, a, band, Ks);
    } else if (wave == 1) {
      ok = sb_loader<T>(Dp, sh, a, a.Din, a.ldd, band, Ks, &sh.ld[0], &sh.done);
    } else if (wave == 2) {
      ok = sb_loader<T>(Cp, sh, a, a.C, a.ldc, band, Ks, &sh.ld[1], &sh.stored);
    } else if (wave == 3) {
      // consumer column k is matrix column n-1-k of the band below's first row
      if (band < a.nb - 1)
        ok = poll_ring<T, 3>(ring, sh, ctl, n, epoch, {E::zero(), -E::inf(), E::zero()}, [&](int64_t k) {
          return a.bnd + ((int64_t)band * n + (n - 1 - k)) * 3 * E::W;
        });
    } else if (wave == 4) {
      ok = sb_store<T>(Cp, sh, a, band, Ks);
    } else if (band > 0) {
      // the first row (lane 0 handles column n + 62 - s at step s) for the band above
      const uint32_t total = (uint32_t)(4 * (int64_t)Ks * K::GPS);
      ok = publish_ring<T, 3>(pub, sh, ctl, n, total, epoch, [n](int64_t st) { return n + 62 - st; },
                              [&](int64_t c, int v) { return a.bnd + ((int64_t)(band - 1) * n + c) * 3 * E::W + v * E::W; });
    }
    if (!ok) sh.abort = 1u;
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

}  // namespace

hipError_t launch_soft_backward(int dtype, const SoftArgs& a, int grid, hipStream_t s) {
  const bool gd = a.gD != nullptr;
  if (dtype == 0) {
    if (gd) hipLaunchKernelGGL((soft_bwd_kernel<float, true>), dim3(grid), dim3(kSbThreads), 0, s, a);
    else hipLaunchKernelGGL((soft_bwd_kernel<float, false>), dim3(grid), dim3(kSbThreads), 0, s, a);
  } else if (dtype == 1) {
    if (gd) hipLaunchKernelGGL((soft_bwd_kernel<double, true>), dim3(grid), dim3(kSbThreads), 0, s, a);
    else hipLaunchKernelGGL((soft_bwd_kernel<double, false>), dim3(grid), dim3(kSbThreads), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace wf
