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
// derivative of the successor's soft minimum with respect to D[i][j].  gC = A.
//
// The forward runs in the min-plus forward's band pipeline (wf_fwd.hip) with the soft-min
// cell in place of the minimum; this file holds the adjoint.  It is a persistent band
// pipeline in a lighter form: a workgroup of three waves per 64-row band, claimed bottom-up.
// The compute wave runs the skewed wavefront (lane r owns band row r; at step t it handles
// column n - 1 - t + 63 - r), taking the lane-shifted neighbour values through DPP and
// reading its inputs straight from global memory as 16-byte range-checked buffer loads of
// four consecutive columns, issued two 4-step groups ahead.  The band's first row goes to
// the band above as epoch-tagged 64-bit (A, V) word pairs: the compute wave writes it to an
// LDS out ring and a publisher wave stores it; a poller wave reads the band below's words
// into an LDS ring that the compute wave reads.  Every wait is bounded.
#include "wf_common.h"
#include "wf_soft.h"

namespace wf {
namespace {

constexpr int kRing = 1024;  // handoff ring: columns

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

// Four columns col .. col+3 of this lane's row (lane * ld elements into the resource).  A
// start before the resource (only lane 0 near the left edge of the adjoint's last groups,
// columns below 0) loads from offset 0 and moves the columns into place; the slots before
// column 0 hold no data and are never used.
template <typename T>
__device__ __forceinline__ Vec4<T> load4_at(__amdgpu_buffer_rsrc_t r, int64_t ld, int lane, int64_t col) {
  const int64_t e = (int64_t)lane * ld + col;
  const Vec4<T> v = load4<T>(r, e >= 0 ? (uint32_t)(e * (int64_t)sizeof(T)) : 0u);
  if (!__any(e < 0)) return v;  // wave-uniform: the shift is needed in the last groups only
  const int sh = e < 0 ? (int)-e : 0;
  Vec4<T> o = v;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T x = v.v[0];
#pragma unroll
    for (int p = 0; p < q; ++p)
      if (q - sh == p) x = v.v[p];
    if (sh == 0) x = v.v[q];
    o.v[q] = x;
  }
  return o;
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
// per column (1 forward, 2 backward), each of W payload words; 'word_at(k)' is the address
// of the first word of consumer column k.
template <typename T, int NV, typename WordAt>
__device__ __forceinline__ bool poll_ring(T* ring, SoftShared& sh, Control* ctl, int64_t n, uint32_t epoch,
                                          WordAt word_at) {
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
    uint64_t x[NV * W];
#pragma unroll
    for (int q = 0; q < NV * W; ++q) x[q] = load_word(src + q);
    bool ok = true;
#pragma unroll
    for (int q = 0; q < NV * W; ++q) ok = ok && (uint32_t)(x[q] >> 32) == epoch;
    ok = ok || !real;
    const uint64_t okm = __ballot(ok);
    const int run = ~okm == 0 ? 64 : __builtin_ctzll(~okm);
    const int take = (int)(run < n - u ? run : n - u);
    if (take == 0) {
      if (polls == 0) t0 = __builtin_amdgcn_s_memrealtime();
      __builtin_amdgcn_s_sleep(1);
      if ((++polls & 63u) == 0u) {
        if (lds_load(&sh.abort) != 0u || global_aborted(ctl)) return false;
        if (__builtin_amdgcn_s_memrealtime() - t0 > kSpinTicks) {
          raise_timeout(ctl);
          return false;
        }
      }
      continue;
    }
    polls = 0;
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
  }
  return true;
}

// ---------------------------------------------------------------------------------------
// Forward.

// 4-step groups of inputs in flight: the chain takes tens of nanoseconds per step, so the
// loads must be issued a memory latency (1-2 us under load) ahead of their use.
template <typename T>
struct SoftPF {
  static constexpr int PD = sizeof(T) == 4 ? 8 : 4;
};

// Handoff values of 4 consecutive consumer columns k0 .. k0+3 from the ring (vector NV-th
// plane), or 'fill' past the last column.
template <typename T>
__device__ __forceinline__ Vec4<T> ring4(const T* ring, int64_t k0, int64_t n, T fill) {
  // k0 is a multiple of 4: four whole columns are one aligned vector of the ring
  if (k0 + 4 <= n) return *reinterpret_cast<const Vec4<T>*>(ring + (int)(k0 & (kRing - 1)));
  Vec4<T> v;
#pragma unroll
  for (int q = 0; q < 4; ++q) v.v[q] = k0 + q < n ? ring[(int)((k0 + q) & (kRing - 1))] : fill;
  return v;
}

// ---------------------------------------------------------------------------------------
// Adjoint.

template <typename T>
__device__ __forceinline__ bool soft_bwd_compute(T* ring, T* pub, SoftShared& sh, const SoftArgs& a, int band) {
  using E = Elem<T>;
  using M = SoftMath<T>;
  constexpr int W = E::W;
  constexpr int PD = SoftPF<T>::PD;
  const int lane = threadIdx.x & 63;
  const int64_t m = a.m, n = a.n;
  const int64_t row0 = (int64_t)band * kBand;
  const int rows = (int)(m - row0 < kBand ? m - row0 : kBand);
  const int64_t i = row0 + lane;
  const bool live = lane < rows;
  const auto rc = band_rsrc<T>(a.C, row0, rows, a.ldc, n);
  const auto rd = band_rsrc<T>(a.Din, row0, rows, a.ldd, n);
  const auto rg = band_rsrc<T>(a.gD, row0, a.gD ? rows : 0, a.ldgd, n);
  const auto ro = band_rsrc<T>(a.gC, row0, rows, a.ldgc, n);
  const bool has_gd = a.gD != nullptr;
  const T kx = (T)a.kx;
  const bool bottom = band == a.nb - 1;  // no band below: successors below are outside
  const bool pubband = band > 0;  // a band above reads this band's first row
  const bool publish = lane == 0 && pubband;
  const T gs = a.gscore ? *static_cast<const T*>(a.gscore) : E::zero();
  const T NEG = -E::inf();
  // this lane's column at step t is n - 1 - t + 63 - lane; group g covers steps 4g .. 4g+3,
  // columns j0 - 3 .. j0 with j0 = n + 62 - lane - 4g, loaded as one 4-column vector
  const int64_t groups = (n + 63 + 3) / 4;
  // groups [g_lo, g_hi) have every lane's four columns inside the matrix (a full band only):
  // lane 0's highest column n+62-4g <= n-1 needs g >= 16, lane 63's lowest n-4-4g >= 0 needs
  // g <= (n-4)/4
  const int64_t g_lo = rows == kBand ? 16 : groups, g_hi = rows == kBand && n >= 4 ? (n - 4) / 4 + 1 : 0;
  auto first_col = [&](int64_t g) -> int64_t { return n + 62 - lane - 4 * g - 3; };
  auto off = [&](int64_t ld, int64_t col) -> uint32_t { return (uint32_t)(((int64_t)lane * ld + col) * sizeof(T)); };
  Vec4<T> db[PD], cb[PD], gb[PD];
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    db[k] = load4_at<T>(rd, a.ldd, lane, first_col(k));
    cb[k] = load4_at<T>(rc, a.ldc, lane, first_col(k));
    if (has_gd) gb[k] = load4_at<T>(rg, a.ldgd, lane, first_col(k));
  }
  T Ae = E::zero(), Ve = NEG;        // east successor: this lane's previous cell
  T Aso = E::zero(), Vso = NEG;      // south successor of the previous step (south-east now)
  uint64_t waited = 0;
  // columns of the band below's first row known to be in the ring (wave-uniform)
  uint32_t have = bottom ? 0xffffffffu : 0u;
  auto avail_for = [&](int64_t g) -> bool {
    const int64_t need = 4 * g + 4 < n ? 4 * g + 4 : n;
    if (need <= (int64_t)have) return true;
    have = lds_load(&sh.avail);
    if (need <= (int64_t)have) return true;
    uint32_t seen;
    if (!lds_wait_value<true, false>(&sh.avail, (uint32_t)need, &sh.abort, a.ctl, waited, seen)) return false;
    have = seen;
    return true;
  };
  // the band below's row-0 (A, V) at lane 63's columns n-1-4g-q, consumer order 4g+q
  Vec4<T> ba, bv;
  auto read_bottom = [&](int64_t g, Vec4<T>& va, Vec4<T>& vv) {
    va = ring4<T>(ring, 4 * g, n, E::zero());
    vv = ring4<T>(ring + kRing, 4 * g, n, NEG);
  };
  if (bottom) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ba.v[q] = E::zero();
      bv.v[q] = NEG;
    }
  } else {
    if (!avail_for(0)) return false;
    read_bottom(0, ba, bv);
  }
  for (int64_t g0 = 0; g0 < groups; g0 += PD) {
    // the batch's out-ring slots must have been published
    if (pubband && 4 * (g0 + PD) > kPub &&
        !lds_wait_ge(&sh.pubd, (uint32_t)(4 * (g0 + PD) - kPub), &sh.abort, a.ctl, waited))
      return false;
#pragma unroll
    for (int k = 0; k < PD; ++k) {
      const int64_t g = g0 + k;
      if (g < groups) {
        const Vec4<T> dg = db[k], cg = cb[k];
        db[k] = load4_at<T>(rd, a.ldd, lane, first_col(g + PD));
        cb[k] = load4_at<T>(rc, a.ldc, lane, first_col(g + PD));
        Vec4<T> gg;
        if (has_gd) {
          gg = gb[k];
          gb[k] = load4_at<T>(rg, a.ldgd, lane, first_col(g + PD));
        }
        Vec4<T> na = ba, nv = bv;
        bool n_ready = bottom;
        if (!bottom && g + 1 < groups && 4 * g + 8 <= (int64_t)have) {
          read_bottom(g + 1, na, nv);
          n_ready = true;
        }
        const int64_t j0 = n + 62 - lane - 4 * g;
        // interior group (full band, every lane's columns j0-3 .. j0 inside the matrix, the
        // last cell not among them): no validity selects, one vector store
        const bool interior = g >= g_lo && g < g_hi;
        Vec4<T> out;
        if (interior) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const T As = shl1_(Ae, ba.v[q]), Vs = shl1_(Ve, bv.v[q]);
            const T dd = dg.v[3 - q], cc = cg.v[3 - q];
            T acc = has_gd ? gg.v[3 - q] : E::zero();
            acc = __builtin_fma(M::exp2_((Vso - dd) * kx), Aso, acc);
            acc = __builtin_fma(M::exp2_((Vs - dd) * kx), As, acc);
            acc = __builtin_fma(M::exp2_((Ve - dd) * kx), Ae, acc);
            Aso = As;
            Vso = Vs;
            Ae = acc;
            Ve = dd - cc;
            out.v[q] = acc;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t j = j0 - q;
            const bool valid = live && j >= 0 && j < n;
            const T As = shl1_(Ae, ba.v[q]), Vs = shl1_(Ve, bv.v[q]);
            const T dd = dg.v[3 - q], cc = cg.v[3 - q];
            T acc = has_gd ? gg.v[3 - q] : E::zero();
            if (i == m - 1 && j == n - 1) acc = acc + gs;
            acc = __builtin_fma(M::exp2_((Vso - dd) * kx), Aso, acc);
            acc = __builtin_fma(M::exp2_((Vs - dd) * kx), As, acc);
            acc = __builtin_fma(M::exp2_((Ve - dd) * kx), Ae, acc);
            const T vown = dd - cc;
            Aso = As;
            Vso = Vs;
            Ae = valid ? acc : E::zero();
            Ve = valid ? vown : NEG;
            out.v[q] = Ae;
          }
        }
        if (live) {
          // the group's columns are j0-3 .. j0, out.v[q] at column j0 - q
          bool whole = false;
          if constexpr (sizeof(T) == 4) {
            if (interior || (j0 - 3 >= 0 && j0 < n)) {
              Vec4<T> asc;
#pragma unroll
              for (int q = 0; q < 4; ++q) asc.v[q] = out.v[3 - q];
              __builtin_amdgcn_raw_buffer_store_b128(
                  __builtin_bit_cast(__attribute__((ext_vector_type(4))) uint32_t, asc), ro, off(a.ldgc, j0 - 3), 0,
                  0);
              whole = true;
            }
          }
          if (!whole) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int64_t j = j0 - q;
              if (j >= 0 && j < n) store1<T>(ro, off(a.ldgc, j), out.v[q]);
            }
          }
        }
        if (publish) {
          // lane 0's (A, V) of steps 4g .. 4g+3 (columns j0 .. j0-3) to the out ring
          Vec4<T> vs;
#pragma unroll
          for (int q = 0; q < 4; ++q) vs.v[q] = dg.v[3 - q] - cg.v[3 - q];
          *reinterpret_cast<Vec4<T>*>(pub + (int)((4 * g) & (kPub - 1))) = out;
          *reinterpret_cast<Vec4<T>*>(pub + kPub + (int)((4 * g) & (kPub - 1))) = vs;
          lds_signal(&sh.produced, (uint32_t)(4 * g + 4));
        }
        if (!n_ready && g + 1 < groups) {
          if (!avail_for(g + 1)) return false;
          read_bottom(g + 1, na, nv);
        }
        ba = na;
        bv = nv;
      }
    }
    if (!bottom && lane == 0) lds_signal(&sh.used, (uint32_t)(4 * (g0 + PD) < n ? 4 * (g0 + PD) : n));
  }
  return true;
}

template <typename T>
__global__ __launch_bounds__(192) void soft_bwd_kernel(SoftArgs a) {
  using E = Elem<T>;
  __shared__ alignas(16) T ring[2 * kRing];
  __shared__ alignas(16) T pub[2 * kPub];
  __shared__ SoftShared sh;
  Control* ctl = a.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      sh.avail = 0u;
      sh.used = 0u;
      sh.produced = 0u;
      sh.pubd = 0u;
    }
    claim_next(ctl, &sh.item, &sh.abort);
    // bands from the bottom up
    const int band = a.nb - 1 - (int)sh.item;
    if ((int)sh.item >= a.nb || sh.abort != 0u) break;
    bool ok = true;
    const int64_t n = a.n;
    if (threadIdx.x < 64) {
      ok = soft_bwd_compute<T>(ring, pub, sh, a, band);
    } else if (threadIdx.x < 128) {
      // consumer column k is matrix column n-1-k of the band below's first row
      if (band < a.nb - 1)
        ok = poll_ring<T, 2>(ring, sh, ctl, n, epoch, [&](int64_t k) {
          return a.bnd + ((int64_t)band * n + (n - 1 - k)) * 2 * E::W;
        });
    } else if (band > 0) {
      // the first row (lane 0 handles column n + 62 - s at step s) for the band above
      const uint32_t total = (uint32_t)(4 * ((n + 63 + 3) / 4));
      ok = publish_ring<T, 2>(pub, sh, ctl, n, total, epoch, [n](int64_t st) { return n + 62 - st; },
                              [&](int64_t c, int v) { return a.bnd + ((int64_t)(band - 1) * n + c) * 2 * E::W + v * E::W; });
    }
    if (!ok) sh.abort = 1u;
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

}  // namespace

hipError_t launch_soft_backward(int dtype, const SoftArgs& a, int grid, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(soft_bwd_kernel<float>, dim3(grid), dim3(192), 0, s, a);
  else if (dtype == 1)
    hipLaunchKernelGGL(soft_bwd_kernel<double>, dim3(grid), dim3(192), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace wf
