// Persistent band-pipelined forward sweep (gfx950).
//
// Work decomposition.  The m x n table is cut into bands of 64 rows.  A persistent
// workgroup claims bands in increasing order from a device counter and sweeps each band
// from left to right as a skewed wavefront: lane r of the compute wave owns band row r and,
// at step t, produces column t - r, so the 64 cells of one step lie on one anti-diagonal.
// The three inputs of a cell come from registers: W is the lane's previous value, N is the
// previous value of lane r-1 moved by a DPP wave_shr:1, NW is the previous step's N.  Lane 0
// takes N from the row above the band (the "top" ring in LDS), which the band above
// published.  A band therefore takes n + 63 steps and the band below can follow 64 steps
// (plus the handoff latency) behind: all m+n-1 anti-diagonals are processed by one launch.
//
// Inside a workgroup four waves split the work so that the compute wave issues little
// besides its cell chain:
//   wave 0  compute   per 4 steps: one 16-byte LDS read of C, one broadcast read of the top
//                     boundary, 4 x (DPP shift, min3, add), one 16-byte LDS write of D;
//   wave 1  loader    coalesced row-major global loads of C (16 bytes per lane), kept in
//                     registers PF sub-chunks ahead, scattered into the skewed LDS ring;
//   wave 2  top       polls the band above's tagged boundary words and fills the top ring;
//   wave 3  storer    publishes the band's last row (tagged words) as soon as it is final,
//                     writes D back coalesced, the checkpoint grid and the score.
// The LDS ring stores element (r, c) at S[r][(r + c) mod RING]: all lanes touch the same
// slot index at a given step, 16-byte reads/writes per lane are aligned, and the row pitch
// (16 mod 256 bytes) keeps them free of bank conflicts.  D overwrites C in place.
//
// Sub-chunks of G columns ("tile width", 16/32/64) are the unit of every handoff.
#include "wf_common.h"

namespace wf {
namespace {

template <typename T, int G>
struct FwdCfg {
  using E = Elem<T>;
  static constexpr int RING = E::RING;
  static constexpr int PITCH = E::PITCH;
  static constexpr int MASK = RING - 1;
  static constexpr int VPR = G / 4;             // 4-element vectors per row per sub-chunk
  static constexpr int VPL = (kBand * VPR) / 64; // vectors per lane per sub-chunk (= VPR)
  // Sub-chunks the loader keeps in flight in registers (about 48 KiB per band).
  static constexpr int PF = (48 * 1024) / (kBand * G * (int)sizeof(T)) < 1
                                ? 1
                                : (48 * 1024) / (kBand * G * (int)sizeof(T));
  static_assert(RING % G == 0, "tile must divide the ring");
  static_assert(RING >= 2 * G + kBand, "ring too small for the handoff distance");
};

struct Shared {
  uint32_t ctr[4];  // 0: C sub-chunks loaded, 1: top sub-chunks loaded, 2: steps done, 3: stored
  uint32_t item;
  uint32_t abort;
};

// ---------------------------------------------------------------------------------------
// wave 0: the cell chain
template <typename T, int G>
__device__ __forceinline__ void compute_band(T* S, const T* Tr, Shared& sh, Control* ctl, int band,
                                             int Us, int Uc) {
  using C = FwdCfg<T, G>;
  using E = typename C::E;
  const int lane = threadIdx.x & 63;
  T D = E::inf();
  T NW = (lane == 0 && band == 0) ? E::zero() : E::inf();  // virtual corner D[-1][-1] = 0
  for (int u = 0; u < Us; ++u) {
    const uint32_t need = (uint32_t)(u + 1 < Uc ? u + 1 : Uc);
    if (!lds_wait_ge(&sh.ctr[0], need, &sh.abort, ctl) || !lds_wait_ge(&sh.ctr[1], need, &sh.abort, ctl)) {
      sh.abort = 1u;
      return;
    }
    // Steps past the last loaded column still write D in place into slots whose previous
    // lap (sub-chunk u - RING/G) must have been stored first.  For u < Uc the loader has
    // already waited for exactly that before publishing sub-chunk u.
    const int lap = u - C::RING / G;
    if (u >= Uc && lap >= 0 && !lds_wait_ge(&sh.ctr[3], (uint32_t)(lap + 1), &sh.abort, ctl)) {
      sh.abort = 1u;
      return;
    }
    const int base = (G * u) & C::MASK;
    T* srow = S + lane * C::PITCH + base;
    const T* trow = Tr + base;
#pragma unroll
    for (int g = 0; g < G / 4; ++g) {
      const Vec4<T> cv = *reinterpret_cast<const Vec4<T>*>(srow + 4 * g);
      const Vec4<T> tv = *reinterpret_cast<const Vec4<T>*>(trow + 4 * g);
      Vec4<T> out;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T N = E::shr1(D, tv.v[q]);   // lane 0 takes the row above the band
        const T v = E::min3(NW, N, D);
        D = E::add(cv.v[q], v);
        NW = N;
        out.v[q] = D;
      }
      *reinterpret_cast<Vec4<T>*>(srow + 4 * g) = out;
    }
    lds_publish(&sh.ctr[2], (uint32_t)(G * (u + 1)));
  }
}

// ---------------------------------------------------------------------------------------
// wave 1: global -> LDS loader
template <typename T, int G>
__device__ __forceinline__ void load_sub(Vec4<T> (&buf)[G / 4], const FwdArgs& a, int64_t row0,
                                         int u) {
  using C = FwdCfg<T, G>;
  using E = typename C::E;
  const int lane = threadIdx.x & 63;
  const T* Cp = static_cast<const T*>(a.C);
#pragma unroll
  for (int k = 0; k < C::VPL; ++k) {
    const int idx = k * 64 + lane;
    const int r = idx / C::VPR;
    const int64_t col = (int64_t)G * u + 4 * (idx % C::VPR);
    const int64_t row = row0 + r;
    Vec4<T> v;
    if (row < a.m && col + 3 < a.n) {
      __builtin_memcpy(&v, Cp + row * a.ldc + col, sizeof(v));
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        v.v[e] = (row < a.m && col + e < a.n) ? Cp[row * a.ldc + col + e] : E::inf();
    }
    buf[k] = v;
  }
}

template <typename T, int G>
__device__ __forceinline__ void store_sub_lds(T* S, const Vec4<T> (&buf)[G / 4], int u) {
  using C = FwdCfg<T, G>;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < C::VPL; ++k) {
    const int idx = k * 64 + lane;
    const int r = idx / C::VPR;
    const int col = G * u + 4 * (idx % C::VPR);
    T* srow = S + r * C::PITCH;
#pragma unroll
    for (int e = 0; e < 4; ++e) srow[(r + col + e) & C::MASK] = buf[k].v[e];
  }
}

template <typename T, int G>
__device__ __forceinline__ bool loader_slot(T* S, const Vec4<T> (&buf)[G / 4], Shared& sh,
                                            Control* ctl, int u) {
  using C = FwdCfg<T, G>;
  // Sub-chunk u reuses the slots of sub-chunk u - RING/G, which must be stored already.  On
  // the first lap the slots that wrap around belong to negative columns (row r, slots
  // < r), which the compute wave writes at steps < 64: it must have passed the last of
  // them, step G*u + G - 1 + 63 - RING.
  const int older = u - C::RING / G;
  if (older >= 0) {
    if (!lds_wait_ge(&sh.ctr[3], (uint32_t)(older + 1), &sh.abort, ctl)) return false;
  } else {
    const int steps = G * u + G + kBand - 1 - C::RING;
    if (steps > 0 && !lds_wait_ge(&sh.ctr[2], (uint32_t)steps, &sh.abort, ctl)) return false;
  }
  store_sub_lds<T, G>(S, buf, u);
  lds_publish(&sh.ctr[0], (uint32_t)(u + 1));
  return true;
}

template <typename T, int G>
__device__ __forceinline__ void loader_band(T* S, Shared& sh, const FwdArgs& a, int band, int Uc) {
  using C = FwdCfg<T, G>;
  using E = typename C::E;
  const int lane = threadIdx.x & 63;
  const int64_t row0 = (int64_t)band * kBand;
  // negative columns: row r reads slots 0 .. r-1 before its first real column
  Vec4<T> inf4;
#pragma unroll
  for (int e = 0; e < 4; ++e) inf4.v[e] = E::inf();
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int idx = k * 64 + lane;
    *reinterpret_cast<Vec4<T>*>(S + (idx >> 4) * C::PITCH + 4 * (idx & 15)) = inf4;
  }
  Vec4<T> buf[C::PF][C::VPL];
#pragma unroll
  for (int p = 0; p < C::PF; ++p)
    if (p < Uc) load_sub<T, G>(buf[p], a, row0, p);
  for (int u0 = 0; u0 < Uc; u0 += C::PF) {
#pragma unroll
    for (int p = 0; p < C::PF; ++p) {
      const int u = u0 + p;
      if (u < Uc) {
        if (!loader_slot<T, G>(S, buf[p], sh, a.ctl, u)) {
          sh.abort = 1u;
          return;
        }
        if (u + C::PF < Uc) load_sub<T, G>(buf[p], a, row0, u + C::PF);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// wave 2: top boundary poller
template <typename T, int G>
__device__ __forceinline__ void top_band(T* Tr, Shared& sh, const FwdArgs& a, int band, int Uc,
                                         uint32_t epoch) {
  using C = FwdCfg<T, G>;
  using E = typename C::E;
  constexpr int W = E::W;
  const int lane = threadIdx.x & 63;
  const int64_t n = a.n;
  for (int u = 0; u < Uc; ++u) {
    // the top ring slot of column j is reused RING steps later
    const int64_t need_steps = (int64_t)G * u + G - C::RING;
    if (need_steps > 0 && !lds_wait_ge(&sh.ctr[2], (uint32_t)need_steps, &sh.abort, a.ctl)) {
      sh.abort = 1u;
      return;
    }
    const int64_t j = (int64_t)G * u + lane;
    T val = E::inf();
    if (band > 0) {
      const bool mine = lane < G && j < n;
      const uint64_t* src = a.bnd + ((int64_t)(band - 1) * n + (mine ? j : 0)) * W;
      uint32_t w[W];
      bool ok = !mine;
      if (mine) {
        ok = true;
#pragma unroll
        for (int k = 0; k < W; ++k) {
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
            for (int k = 0; k < W; ++k) {
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
        if (give_up) {
          sh.abort = 1u;
          return;
        }
      }
      if (mine) val = E::from_words(w);
    }
    if (lane < G) Tr[(G * u + lane) & C::MASK] = val;
    lds_publish(&sh.ctr[1], (uint32_t)(u + 1));
  }
}

// ---------------------------------------------------------------------------------------
// wave 3: storer / publisher
template <typename T, int G>
__device__ __forceinline__ void store_band(const T* S, Shared& sh, const FwdArgs& a, int band, int Uc,
                                           uint32_t epoch) {
  using C = FwdCfg<T, G>;
  using E = typename C::E;
  constexpr int W = E::W;
  const int lane = threadIdx.x & 63;
  const int64_t m = a.m, n = a.n;
  const int64_t row0 = (int64_t)band * kBand;
  const bool last_band = band == a.nb - 1;
  T* Dp = static_cast<T*>(a.D);
  T* ck_rows = static_cast<T*>(a.ckpt);
  T* ck_cols = ck_rows ? ck_rows + (int64_t)(a.nb - 1) * n : nullptr;
  const int K = a.ckpt_k;
  for (int v = 0; v < Uc; ++v) {
    const int64_t j0 = (int64_t)G * v;
    const int64_t jend = j0 + G < n ? j0 + G : n;
    if (!lds_wait_ge(&sh.ctr[2], (uint32_t)(jend + kBand - 1), &sh.abort, a.ctl)) {
      sh.abort = 1u;
      return;
    }
    // 1. the band's last row, latency critical: it unblocks the band below
    if (!last_band && lane < G && j0 + lane < n) {
      const int64_t j = j0 + lane;
      const T x = S[(kBand - 1) * C::PITCH + ((kBand - 1 + (int)j) & C::MASK)];
#pragma unroll
      for (int k = 0; k < W; ++k) store_word(a.bnd + ((int64_t)band * n + j) * W + k, tagged(E::word(x, k), epoch));
      if (ck_rows) ck_rows[(int64_t)band * n + j] = x;
    }
    // 2. the table, coalesced
    if (Dp) {
#pragma unroll
      for (int k = 0; k < C::VPL; ++k) {
        const int idx = k * 64 + lane;
        const int r = idx / C::VPR;
        const int64_t col = j0 + 4 * (idx % C::VPR);
        const int64_t row = row0 + r;
        if (row < m && col < n) {
          const T* srow = S + r * C::PITCH;
          Vec4<T> x;
#pragma unroll
          for (int e = 0; e < 4; ++e) x.v[e] = srow[(r + (int)col + e) & C::MASK];
          T* dst = Dp + row * a.ldd + col;
          if (col + 3 < n) {
            __builtin_memcpy(dst, &x, sizeof(x));
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (col + e < n) dst[e] = x.v[e];
          }
        }
      }
    }
    // 3. checkpoint columns: D[.][Kq-1] for 1 <= q < ceil(n/K)
    if (ck_cols) {
      const int64_t row = row0 + lane;
      for (int64_t j = ((j0 + K) / K) * K - 1; j < jend; j += K) {
        if (j + 1 < n && row < m)
          ck_cols[((j + 1) / K - 1) * m + row] = S[lane * C::PITCH + ((lane + (int)j) & C::MASK)];
      }
    }
    // 4. the score
    if (last_band && v == Uc - 1 && lane == (int)(m - 1 - row0))
      *static_cast<T*>(a.score) = S[lane * C::PITCH + ((lane + (int)(n - 1)) & C::MASK)];
    lds_publish(&sh.ctr[3], (uint32_t)(v + 1));
  }
}

// ---------------------------------------------------------------------------------------
template <typename T, int G>
__global__ __launch_bounds__(kThreads, 1) void fwd_kernel(FwdArgs a) {
  using C = FwdCfg<T, G>;
  __shared__ Vec4<T> S4[kBand * C::PITCH / 4];
  __shared__ Vec4<T> Tr4[C::RING / 4];
  __shared__ Shared sh;
  T* S = reinterpret_cast<T*>(S4);
  T* Tr = reinterpret_cast<T*>(Tr4);
  const int wave = threadIdx.x >> 6;
  Control* ctl = a.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int Uc = (int)((a.n + G - 1) / G);
  const int Us = (int)((a.n + kBand - 1 + G - 1) / G);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x < 4) sh.ctr[threadIdx.x] = 0u;
    claim_next(ctl, &sh.item, &sh.abort);
    const int band = (int)sh.item;
    if (band >= a.nb || sh.abort != 0u) break;
    if (wave == 0)
      compute_band<T, G>(S, Tr, sh, ctl, band, Us, Uc);
    else if (wave == 1)
      loader_band<T, G>(S, sh, a, band, Uc);
    else if (wave == 2)
      top_band<T, G>(Tr, sh, a, band, Uc, epoch);
    else
      store_band<T, G>(S, sh, a, band, Uc, epoch);
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

template <typename T>
hipError_t launch_t(int tile, const FwdArgs& a, int grid, hipStream_t s) {
  switch (tile) {
    case 16: hipLaunchKernelGGL((fwd_kernel<T, 16>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 32: hipLaunchKernelGGL((fwd_kernel<T, 32>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 64: hipLaunchKernelGGL((fwd_kernel<T, 64>), dim3(grid), dim3(kThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_forward(int dtype, int tile, const FwdArgs& a, int grid, hipStream_t s) {
  switch (dtype) {
    case 0: return launch_t<float>(tile, a, grid, s);
    case 1: return launch_t<double>(tile, a, grid, s);
    case 2: return launch_t<int32_t>(tile, a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wf
