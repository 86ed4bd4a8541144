// Adjoint (backward) sweep of the wavefront recurrence (gfx950).
//
// The routed adjoint of  L = sum(gD * D) + gscore * score  is
//     A[i][j] = gD[i][j] + [last] gscore + [SEL(i+1,j+1) = NW] A[i+1][j+1]
//             + [SEL(i+1,j) = N] A[i+1][j] + [SEL(i,j+1) = W] A[i][j+1],       gC = A,
// summed in exactly that order (reading R0; the paper states no recurrence and no order for
// the routed terms: the two from the row below come first, the one from the same row last).
// SEL(i,j) is the predecessor cell (i,j) took in the forward min, ties broken NW, N, W.
//
// Two launches:
//  1. Selection recompute.  Every 64-row band is swept again left to right from its top
//     row, which the forward pass stored as a checkpoint row (or which the caller's saved
//     table provides).  The bands are therefore independent and all run at once.  The
//     sweep is the forward cell chain plus the comparisons that name the predecessor; it
//     emits three bit-planes per row (selected W, selected N, selected NW), one bit per
//     cell.
//  2. Reverse sweep.  Bands from the bottom up, each a skewed wavefront from right to left:
//     lane r owns band row r and at reverse step t handles slot s = S - t (slot = row +
//     column), so lane r+1 handles a column one step before lane r does.  A cell's routed
//     inputs come from the south-east (lane r+1, two steps back), the south (lane r+1, one
//     step back) and the east (the lane itself, one step back); each is the successor's A
//     times a 0/1 factor (did that successor select this cell?), so every term is one
//     fused multiply-add, and the lane-shifted ones take their operand through DPP
//     wave_shl:1.  The loader turns the bit-planes into those factors, already aligned to
//     the receiving cell, as bytes in LDS.  Lane 63's inputs come from the band below, which
//     publishes them (tagged 64-bit words, as in the forward sweep); the poller adds them to
//     lane 63's upstream value before the compute wave reads it.
// Waves of the reverse sweep: compute; value loader (gD); factor loader (bit-planes ->
// factors); poller (values from the band below); storer (gC); publisher (values for the
// band above).
#include <algorithm>

#include "wf_common.h"
#include "wf_path.h"

namespace wf {
namespace {

constexpr int kSub = 64;

template <typename V>
__device__ __forceinline__ V opaque(V x) {
  asm volatile("" : "+s"(x));
  return x;
}

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

// LDS rings of the adjoint kernels: RING slots per row.  The value ring's row pitch is 16 mod
// 256 bytes (conflict-free 16-byte accesses of 64 rows); the factor ring holds one word per
// slot (4 one-byte factors per 4-slot group and word) with the same property.
template <typename T>
struct BCfg {
  using E = Elem<T>;
  static constexpr int RING = sizeof(T) == 4 ? 256 : 128;
  static constexpr int PITCH = RING + 16 / (int)sizeof(T);
  static constexpr int FPITCH = RING + 4;
  static constexpr int MASK = RING - 1;
  static constexpr int NSUB = RING / kSub;  // 64-slot sub-chunks in a ring
};

// LDS ring of the selection recompute: 256 slots per row for 4-byte elements, 128 for 8-byte
// ones (two workgroups per CU either way).  A 128-slot ring for 4-byte elements lets four
// workgroups share a CU, but four compute waves per CU swept a band's pieces no faster in
// total than two (measured on MI355X), and the smaller ring stalled the plain recompute on
// its loader.  The row pitch keeps the 64 rows' 16-byte accesses conflict-free.
template <typename T>
struct SCfg {
  using E = Elem<T>;
  static constexpr int RING = sizeof(T) == 4 ? 256 : 128;
  static constexpr int PITCH = RING + 16 / (int)sizeof(T);
  static constexpr int MASK = RING - 1;
};

// Layout of the selection bit-planes in global memory: for band b, sub-chunk k (slots
// [64k, 64k+64)) and lane r, eight words: W[0..1], N[0..1], NW[0..1], 0, 0 -- bit j of word
// h of a plane is slot 64k + 32h + j of row r.
__device__ __forceinline__ int64_t sel_index(int band, int Ks, int k, int lane) {
  return (((int64_t)band * Ks + k) * 64 + lane) * 8;
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

// min of two values without the quieting of signalling NaNs that fminf implies for operands
// the compiler cannot prove canonical (here the DPP-shifted ones): inputs hold no NaN.
__device__ __forceinline__ float sel_min(float a, float b) {
  float r;
  asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double sel_min(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// bits = 2 bits + (x < y): for 4-byte elements one compare into VCC and one add with VCC as
// the carry in (the compiler's form takes a select, an or and a shift besides).
__device__ __forceinline__ void sel_bit(uint32_t& bits, float x, float y) {
  asm("v_cmp_lt_f32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, %0, %0, vcc" : "+v"(bits) : "v"(x), "v"(y) : "vcc");
}
__device__ __forceinline__ void sel_bit(uint32_t& bits, double x, double y) { bits = bits + bits + (uint32_t)(x < y); }

// One 4-step group's operands: C of the lane's row and the top row's values (a broadcast).
template <typename T>
struct SelGroup {
  Vec4<T> c;
  Vec4<T> t;
};

template <typename T>
__device__ __forceinline__ void sel_load_group(const T* __restrict__ S, const T* __restrict__ Tr, int slot, int lane,
                                               SelGroup<T>& r) {
  using C = SCfg<T>;
  r.c = *reinterpret_cast<const Vec4<T>*>(S + lane * C::PITCH + slot);
  r.t = *reinterpret_cast<const Vec4<T>*>(Tr + slot);
}

// Sub-chunks [k0, k1) of the band that one piece of it sweeps: the whole band, or with
// column splits every w = split columns (a multiple of 64) sub-chunks [p w/64, (p+1) w/64]
// for piece p and [p w/64, Ks) for the last.  Sub-chunk (p+1) w/64 is swept by pieces p
// and p+1; only piece p stores it (its cells of columns >= (p+1) w are plain cells of piece
// p's sweep too).
struct SelPiece {
  int k0, k1;
  bool second;  // piece >= 1: enters from column k0 * 64 - 1
  int piece;
};
__device__ __forceinline__ SelPiece sel_piece(const SelArgs& a, int piece, int Ks) {
  const int ks = (int)(a.split / kSub);
  if (a.split == 0) return {0, Ks, false, 0};
  return SelPiece{piece * ks, piece == a.pieces - 1 ? Ks : (piece + 1) * ks + 1, piece > 0, piece};
}

// One sub-chunk of the compute wave (see sel_compute); ENTRY: the first sub-chunk of a
// band's second piece, where each row takes its left value and nothing is stored.
// Cache policy of the gradient's zero stores (gfx950 buffer instructions: bit 1 = nt).
constexpr int kZeroAux = 2;

// Label state of the path variant (LAB): the exit of the lane's previous cell (W of the next
// cell), the previous N label, lane 0's N label (the cell's column below a band, -1 in band
// 0) and its step, lane 63's labels of the sub-chunk shifted in one per step, and the label
// captured at slot cbase + lane (CAP sub-chunks).
struct LabState {
  int32_t LX, LNW, tcol, inc, acc, cap, cbase, entry;
};

// The label a split band's piece p >= 1 gives row r at its entry column: the label of
// (r, entry column) in piece p - 1, which that piece captures (caps slot (p - 1) * 64 + r).
__device__ __forceinline__ int32_t sym_label(int piece, int r) { return -2 - ((piece - 1) * 64 + r); }

// Selection bits and the label of one cell: N if N < NW, W if W < min(N, NW), else NW.
__device__ __forceinline__ void sel_bits_lab(uint32_t& pn, uint32_t& pw, float N, float NW, float X, float m,
                                             int32_t LN, int32_t LNW, int32_t LX, int32_t& L) {
  int32_t t;
  asm("v_cmp_lt_f32 vcc, %4, %5\n\t"
      "v_cndmask_b32 %0, %8, %7, vcc\n\t"
      "v_addc_co_u32 %2, vcc, %2, %2, vcc\n\t"
      "v_cmp_lt_f32 vcc, %6, %10\n\t"
      "v_cndmask_b32 %1, %0, %9, vcc\n\t"
      "v_addc_co_u32 %3, vcc, %3, %3, vcc"
      : "=&v"(t), "=&v"(L), "+v"(pn), "+v"(pw)
      : "v"(N), "v"(NW), "v"(X), "v"(LN), "v"(LNW), "v"(LX), "v"(m)
      : "vcc");
}
__device__ __forceinline__ void sel_bits_lab(uint32_t& pn, uint32_t& pw, double N, double NW, double X, double m,
                                             int32_t LN, int32_t LNW, int32_t LX, int32_t& L) {
  const bool nl = N < NW, wl = X < m;
  pn = pn + pn + (uint32_t)nl;
  pw = pw + pw + (uint32_t)wl;
  L = wl ? LX : (nl ? LN : LNW);
}

template <typename T, bool ENTRY, bool LAB = false, bool CAP = false>
__device__ __forceinline__ void sel_sub(const T* __restrict__ S, const T* __restrict__ Tr, const SelArgs& a, int band,
                                        int Ks, int k, int rows, int64_t n, T& X, T& NW, T left,
                                        SelGroup<T> (&P)[2], LabState& ls, const PathLabels& po) {
  using C = SCfg<T>;
  using E = typename C::E;
  typedef int v4i __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  uint32_t* out = a.sel;
  const int base = (kSub * k) & C::MASK;
  const int next = (kSub * (k + 1)) & C::MASK;  // past the last sub-chunk: read, not used
  __builtin_amdgcn_sched_barrier(0);
  SelGroup<T> gr[18];
  gr[0] = P[0];
  gr[1] = P[1];
  uint32_t pl[3][2];
  uint32_t pw = 0, pn = 0;
  // CAP: lane r captures its label at slot cbase + r, i.e. at step 4g + q == cl of the sub-chunk
  const int cl = CAP ? lane - (kSub * k - ls.cbase) : 0;
#pragma unroll
  for (int g = 0; g < 16; ++g) {
    if (g + 2 < 16)
      sel_load_group<T>(S, Tr, base + 4 * (g + 2), lane, gr[g + 2]);
    else
      sel_load_group<T>(S, Tr, next + 4 * (g - 14), lane, P[g - 14]);
    __builtin_amdgcn_sched_barrier(0);
    // per step two bits, first step in the most significant bit: W strictly smaller than
    // both others, N strictly smaller than NW
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T N = E::shr1(X, gr[g].t.v[q]);
      const T m = sel_min(NW, N);
      if constexpr (LAB) {
        const int32_t LN = Elem<int32_t>::shr1(ls.LX, ls.tcol);
        int32_t L;
        sel_bits_lab(pn, pw, N, NW, X, m, LN, ls.LNW, ls.LX, L);
        ls.LNW = LN;
        ls.LX = L;
        ls.acc = (int32_t)dpp_shl1_u32((uint32_t)ls.acc, (uint32_t)L);
        ls.tcol += ls.inc;
        if (CAP && 4 * g + q == cl) ls.cap = L;
      } else {
        sel_bit(pn, N, NW);
        sel_bit(pw, X, m);
      }
      X = E::add(gr[g].c.v[q], sel_min(m, X));
      NW = N;
      if (ENTRY && 4 * g + q == lane - 1) {
        X = left;
        if constexpr (LAB) ls.LX = ls.entry - lane;
      }
    }

    if ((g & 7) == 7) {
      const int h = g >> 3;
      pw = __builtin_bitreverse32(pw);
      pn = __builtin_bitreverse32(pn);
      // predecessor: NW unless N is strictly smaller; W if strictly smaller than both
      uint32_t pnw = ~pn & ~pw;
      pn &= ~pw;
      // clear the bits of cells outside the matrix (and of cell (0,0), which selects nothing)
      const int t0 = kSub * k + 32 * h;
      if (!(rows == kBand && t0 >= kBand - 1 && (int64_t)t0 + 32 <= n)) {
        const int64_t lo = lane - (int64_t)t0, hi = n + lane - (int64_t)t0;  // valid steps [lo, hi)
        const int a0 = (int)(lo < 0 ? 0 : (lo > 32 ? 32 : lo));
        const int a1 = (int)(hi < 0 ? 0 : (hi > 32 ? 32 : hi));
        uint64_t msk = a1 > a0 ? (((uint64_t)1 << a1) - 1) & ~(((uint64_t)1 << a0) - 1) : 0;
        if (lane >= rows) msk = 0;
        if (band == 0 && lane == 0 && t0 == 0) msk &= ~(uint64_t)1;
        pw &= (uint32_t)msk;
        pn &= (uint32_t)msk;
        pnw &= (uint32_t)msk;
      }
      pl[0][h] = pw;
      pl[1][h] = pn;
      pl[2][h] = pnw;
      pw = 0;
      pn = 0;
    }
  }
  if (!ENTRY) {
    const v4i w0 = {(int)pl[0][0], (int)pl[0][1], (int)pl[1][0], (int)pl[1][1]};
    const v4i w1 = {(int)pl[2][0], (int)pl[2][1], 0, 0};
    v4i* dst = reinterpret_cast<v4i*>(out + sel_index(band, Ks, k, lane));
    __builtin_nontemporal_store(w0, dst);
    __builtin_nontemporal_store(w1, dst + 1);
    if constexpr (LAB) {
      // lane r holds lane 63's label of slot 64k + r: the last row's cell of column 64k + r - 63
      const int64_t col = (int64_t)kSub * k + lane - 63;
      if (col >= 0 && col < n) po.exits[(int64_t)band * n + col] = ls.acc;
    }
  }
}

// The compute wave.  Sub-chunk k (64 steps, 16 groups) starts once sub-chunks k and k+1 are
// in LDS; each group's reads are issued two groups ahead of its steps, the last two groups
// issuing the next sub-chunk's first two (left in 'P', the same registers every time).
// The second piece of a split band starts at slot 'split' (column split - r for row r):
// row r's state enters as column split-1 of the forward table, which the wave sets at step
// r-1 (row 0 before the first step, its NW from the row above); the cells before it are
// none of this piece's and their selections are not stored.
template <typename T, bool LAB>
__device__ __forceinline__ void sel_compute(const T* __restrict__ S, const T* __restrict__ Tr, SelShared& sh,
                                            const SelArgs& a, int band, int Ks, SelPiece pc, const PathLabels& po) {
  using C = SCfg<T>;
  using E = typename C::E;
  const int lane = threadIdx.x & 63;
  const int64_t n = opaque(a.n);
  const int rows = (int)(a.m - (int64_t)band * kBand < kBand ? a.m - (int64_t)band * kBand : kBand);
  T X = E::inf();
  T NW = (lane == 0 && band == 0) ? E::zero() : E::inf();  // virtual corner D[-1][-1] = 0
  T left = E::inf();
  if (pc.second) {
    const T* lp = static_cast<const T*>(a.left) + (int64_t)(pc.piece - 1) * a.left_pstride;
    const int64_t c = opaque(a.split) * pc.piece - 1;
    if (lane < rows) left = lp[((int64_t)band * kBand + lane) * a.ld_left];
    if (lane == 0) {
      X = left;
      NW = band > 0 ? static_cast<const T*>(a.top)[(int64_t)(band - 1) * a.ld_top + c] : E::inf();
    }
  }
  // labels (LAB): -1 (leaves the matrix) before the first column; lane 0's N label is the
  // cell's own column below band 0; the second piece's rows enter with -2 - r
  LabState ls;
  bool has_cap = false;
  if constexpr (LAB) {
    const int64_t c0 = pc.second ? opaque(a.split) * pc.piece : 0;
    ls.inc = band > 0 ? 1 : 0;
    ls.tcol = band > 0 ? (int32_t)c0 : -1;
    ls.LX = (pc.second && lane == 0) ? sym_label(pc.piece, 0) : -1;
    ls.LNW = (pc.second && lane == 0 && band > 0) ? (int32_t)(c0 - 1) : -1;
    ls.acc = 0;
    ls.cap = -1;
    ls.cbase = 0;
    ls.entry = pc.second ? sym_label(pc.piece, 0) : 0;
    if (a.split > 0 && pc.piece < a.pieces - 1) {
      has_cap = true;
      ls.cbase = (int32_t)(a.split * (pc.piece + 1) - 1);
    } else if (band == a.nb - 1) {
      has_cap = true;
      ls.cbase = (int32_t)(n - 1);
    }
  }
  uint64_t waited = 0;
  SelGroup<T> P[2];
  const int nk = pc.k1 - pc.k0;
  for (int k = pc.k0; k < pc.k1; ++k) {
    const int kl = k - pc.k0;  // sub-chunks counted from the piece's first
    // LDS-only wait: a global load in this wave (the abort flag) would make the compiler wait
    // for the wave's plane stores as well before reusing their registers.  A launch-wide
    // abort reaches it through the wait's own time limit.
    if (!lds_wait_ge<false>(&sh.loaded, (uint32_t)(kl + 2 < nk ? kl + 2 : nk), &sh.abort, a.ctl, waited)) {
      sh.abort = 1u;
      return;
    }
    if (k == pc.k0) {
      const int base = (kSub * k) & C::MASK;
#pragma unroll
      for (int p = 0; p < 2; ++p) sel_load_group<T>(S, Tr, base + 4 * p, lane, P[p]);
    }
    if (pc.second && k == pc.k0)
      sel_sub<T, true, LAB>(S, Tr, a, band, Ks, k, rows, n, X, NW, left, P, ls, po);
    else if (LAB && has_cap && (int64_t)kSub * k + 63 >= ls.cbase && (int64_t)kSub * k <= (int64_t)ls.cbase + 63)
      sel_sub<T, false, LAB, true>(S, Tr, a, band, Ks, k, rows, n, X, NW, left, P, ls, po);
    else
      sel_sub<T, false, LAB>(S, Tr, a, band, Ks, k, rows, n, X, NW, left, P, ls, po);
    lds_signal(&sh.steps, (uint32_t)(kSub * (kl + 1)));
  }
  if constexpr (LAB) {
    if (has_cap) po.caps[((int64_t)band * kMaxPieces + pc.piece) * 64 + lane] = ls.cap;
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
  // Every call issues the same loads (no branch around any of them), so the compiler can
  // count the loads in flight and wait for the oldest sub-chunk only.
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
  tv = top[j < n ? j : n - 1];  // replaced by +inf in sel_store_sub where not a real column
  __builtin_amdgcn_sched_barrier(0);
}

template <typename T>
__device__ __forceinline__ void sel_store_sub(T* S, T* Tr, const Vec4<T> (&x)[16], T tv, bool has_top, int k,
                                              int rows, int64_t n) {
  using C = SCfg<T>;
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
  const int64_t j = (int64_t)kSub * k + lane;
  Tr[(kSub * k + lane) & C::MASK] = (has_top && j < n) ? tv : E::inf();
}

// Zeros over the gradient's columns [64k, 64k + 64) of the band's rows (path adjoint with a
// gradient to zero): 16-byte streaming stores when the columns all lie in the matrix (rows
// past the band's last fall outside the buffer range and are dropped), else element by
// element.
template <typename T>
__device__ __forceinline__ void sel_zero_sub(const PathLabels& po, int band, int rows, int64_t n, int k) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)kSub * k + 4 * (lane & 15);
  T* gb = static_cast<T*>(po.gC) + (int64_t)band * kBand * po.ldgc;
  if ((int64_t)kSub * k + kSub <= n) {
    const __amdgpu_buffer_rsrc_t zrs = make_rsrc(gb, (uint32_t)(((rows - 1) * po.ldgc + n) * (int64_t)sizeof(T)));
    const v4i z = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int off = (int)(((int64_t)(4 * q + (lane >> 4)) * po.ldgc + c0) * (int64_t)sizeof(T));
      __builtin_amdgcn_raw_buffer_store_b128(z, zrs, off, 0, kZeroAux);
      if constexpr (sizeof(T) == 8) __builtin_amdgcn_raw_buffer_store_b128(z, zrs, off + 16, 0, kZeroAux);
    }
  } else {
    for (int q = 0; q < 16; ++q) {
      const int i = 4 * q + (lane >> 4);
      if (i >= rows) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (c0 + e < n) gb[(int64_t)i * po.ldgc + c0 + e] = T(0);
    }
  }
}

template <typename T>
__device__ __forceinline__ void sel_loader(T* S, T* Tr, SelShared& sh, const SelArgs& a, int band, int Ks,
                                           SelPiece pc, const PathLabels& po) {
  using C = SCfg<T>;
  constexpr int PF = SelPF<T>::PF;
  const int64_t ldc = opaque(a.ldc), n = opaque(a.n), m = opaque(a.m);
  const int64_t row0 = (int64_t)band * kBand;
  const int rows = (int)(m - row0 < kBand ? m - row0 : kBand);
  // Loads outside the band's rows (or columns outside [0, n) on the last row) return zeros
  // from the range-checked buffer; sel_store_sub replaces them by +inf.
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(static_cast<const T*>(a.C) + row0 * ldc,
                                                (uint32_t)(((rows - 1) * ldc + n) * (int64_t)sizeof(T)));
  // the first band has no row above: its loads read row 0 of C and are replaced by +inf
  const bool has_top = band > 0;
  const T* top = has_top ? static_cast<const T*>(a.top) + (int64_t)(band - 1) * a.ld_top : static_cast<const T*>(a.C);
  uint64_t waited = 0;
  Vec4<T> buf[PF][16];
  T tv[PF];
  const int k0 = pc.k0, k1 = pc.k1;
  // The loads of sub-chunk k+PF are issued right after sub-chunk k is stored, unconditionally
  // (clamped to the piece's last sub-chunk), so that PF sub-chunks are in flight at every wait.
#pragma unroll
  for (int p = 0; p < PF; ++p) sel_load_sub<T>(buf[p], tv[p], rsrc, ldc, top, n, k0 + p < k1 ? k0 + p : k1 - 1);
  auto store = [&](int p, int k) -> bool {
    // sub-chunk k reuses the ring slots of sub-chunk k - RING/64 (counted from the piece's first)
    const int older = k - k0 - C::RING / kSub;
    if (older >= 0 &&
        !lds_wait_ge<false>(&sh.steps, (uint32_t)(kSub * (older + 1)), &sh.abort, a.ctl, waited)) {
      sh.abort = 1u;
      return false;
    }
    sel_store_sub<T>(S, Tr, buf[p], tv[p], has_top, k, rows, n);
    lds_publish(&sh.loaded, (uint32_t)(k - k0 + 1));
    // a piece's first sub-chunk is the previous piece's last: zeroed there
    if (po.gC != nullptr && !(pc.second && k == k0)) sel_zero_sub<T>(po, band, rows, n, k);
    return true;
  };
  // Whole groups of PF sub-chunks carry no condition around the stores, which keeps the
  // compiler's wait counts at PF - 1 sub-chunks in flight; the last partial group follows.
  int kk = k0;
  for (; kk + PF <= k1; kk += PF) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int k = kk + p;
      if (!store(p, k)) return;
      sel_load_sub<T>(buf[p], tv[p], rsrc, ldc, top, n, k + PF < k1 ? k + PF : k1 - 1);
    }
  }
#pragma unroll
  for (int p = 0; p < PF; ++p)
    if (kk + p < k1 && !store(p, kk + p)) return;
}

template <typename T>
struct SelLds {
  Vec4<T> S4[kBand * SCfg<T>::PITCH / 4];
  Vec4<T> Tr4[SCfg<T>::RING / 4];
};

// One work item: band 'band' (piece 'piece' of it when the band is split) of the instance
// 'a' describes.  The LDS counters must be zero on entry.
template <typename T, bool LAB = false>
__device__ __forceinline__ void sel_item(SelLds<T>& L, SelShared& sh, const SelArgs& a, int band, int piece,
                                         const PathLabels& po = PathLabels{nullptr, nullptr, nullptr, 0}) {
  T* S = reinterpret_cast<T*>(L.S4);
  T* Tr = reinterpret_cast<T*>(L.Tr4);
  const int Ks = (int)((a.n + kBand - 1 + kSub - 1) / kSub);
  const SelPiece pc = sel_piece(a, piece, Ks);
  if (threadIdx.x < 64)
    sel_compute<T, LAB>(S, Tr, sh, a, band, Ks, pc, po);
  else
    sel_loader<T>(S, Tr, sh, a, band, Ks, pc, po);
}

template <typename T>
__global__ __launch_bounds__(128, 1) void sel_kernel(SelArgs a) {
  __shared__ SelLds<T> L;
  __shared__ SelShared sh;
  Control* ctl = a.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      sh.loaded = 0u;
      sh.steps = 0u;
    }
    claim_next(ctl, &sh.item, &sh.abort);
    // work items: bands, or (band, piece) pairs of split bands
    const int pieces = a.split > 0 ? a.pieces : 1;
    const int item = (int)sh.item;
    if (item >= a.nb * pieces || sh.abort != 0u) break;
    sel_item<T>(L, sh, a, item / pieces, item % pieces);
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

// Batched selection recompute: one (instance, band) item at a time, bands whole.
template <typename T>
__global__ __launch_bounds__(128, 1) void sel_batch_kernel(BwdBatchArgs b) {
  __shared__ SelLds<T> L;
  __shared__ SelShared sh;
  Control* ctl = b.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      sh.loaded = 0u;
      sh.steps = 0u;
    }
    claim_next(ctl, &sh.item, &sh.abort);
    // the same for every lane: read it into a scalar register, so that the item's fields are
    // scalar loads and kernel-wide values for the roles
    const uint32_t item = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.item);
    if (item >= (uint32_t)b.n_items || sh.abort != 0u) break;
    const BatchItem it = load_uniform(b.items + item);
    const BwdInst in = load_uniform(b.inst + it.inst);
    SelArgs a;
    a.C = static_cast<const T*>(b.C) + in.off;
    if (b.ckpt_k > 0) {  // band rows of the instance's checkpoint grid
      a.top = static_cast<const T*>(b.top) + in.ck_off;
      a.ld_top = in.n;
    } else {  // rows 64b+63 of the instance's saved table
      a.top = static_cast<const T*>(b.top) + in.off + 63 * in.n;
      a.ld_top = 64 * in.n;
    }
    a.ldc = in.n;
    a.m = in.m;
    a.n = in.n;
    a.nb = in.nb;
    a.sel = b.sel + in.sel_off;
    a.ctl = ctl;
    a.split = 0;
    a.left = nullptr;
    a.ld_left = 0;
    a.left_pstride = 0;
    a.pieces = 1;
    a.pad = 0;
    sel_item<T>(L, sh, a, it.band, 0);
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

// =======================================================================================
// 2. Reverse sweep: six waves, one 64-row band per workgroup, bands from the bottom up.
// =======================================================================================
struct alignas(8) AdjShared {
  uint32_t ctr[7];  // 0: sub-chunks of upstream values loaded, 1: units whose lane-63 inputs
                    // from the band below are added in, 2: reverse steps done, 3: sub-chunks
                    // stored, 4: units published, 5: unused, 6: sub-chunks of factors loaded
  uint32_t item;
  uint32_t abort;
};
constexpr int kAdjCounters = 7;
constexpr int kAdjThreads = 6 * 64;

// Both readiness counters of the compute wave in one 8-byte LDS read.  'zero' is 0, but
// the compiler cannot tell: the value counts as per-lane data and is compared where it is
// used, so the wave waits for it there rather than right after the read (where it would
// also wait for every earlier LDS read, the prefetches).
__device__ __forceinline__ uint64_t adj_ready(const AdjShared& sh, int zero) {
  return __hip_atomic_load(reinterpret_cast<const uint64_t*>(&sh.ctr[0]) + zero, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t adj_ready_f(const AdjShared& sh, int zero) {
  return __hip_atomic_load(&sh.ctr[6] + zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Whether the compute wave's inputs are in LDS: need_l sub-chunks of values and of factors,
// need_b units of the band below's inputs (all three counters read before any compare).
__device__ __forceinline__ bool adj_inputs_ready(const AdjShared& sh, int zero, uint32_t need_l, uint32_t need_b) {
  const uint64_t r = adj_ready(sh, zero);
  const uint32_t f = adj_ready_f(sh, zero);
  return __all((uint32_t)r >= need_l && (uint32_t)(r >> 32) >= need_b && f >= need_l);
}
__device__ __forceinline__ int adj_opaque_zero() {
  int z = 0;
  asm volatile("" : "+v"(z));
  return z;
}

// wave_shl:1 with bound_ctrl: lane r receives lane r+1's value, lane 63 reads zero.  Feeding
// a multiply or a fused multiply-add, the move folds into a DPP form of that instruction.
template <typename T>
__device__ __forceinline__ T shl1z(T src) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, src), 0x130, 0xf, 0xf, true));
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, src);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x130, 0xf, 0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}
__device__ __forceinline__ uint32_t shl1z_u32(uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)src, 0x130, 0xf, 0xf, true);
}

// 0/1 factor held in byte q of a factor word, as an element value (one v_cvt_f32_ubyteN).
template <typename T, int q>
__device__ __forceinline__ T factor(uint32_t w) {
  return (T)(float)((w >> (8 * q)) & 0xFFu);
}

// wave 0: the reverse chain.  Slot group [b4, b4+4) is processed from b4+3 down to b4.
// The LDS reads of a group (upstream values and factor words) are issued PD groups ahead of
// their use: LDS latency under the other waves' traffic is longer than one group's compute.
template <typename T>
struct AdjGroup {
  Vec4<T> gv;      // upstream value gD (+ gscore; lane 63: + the band below's inputs)
  uint32_t f[3];   // factor words: [0] W (east), [1] N (south), [2] NW (south-east)
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
__device__ __forceinline__ void adj_load_group(const T* __restrict__ S, const uint32_t* __restrict__ F, int b4,
                                               int lane, AdjGroup<T>& r) {
  using C = BCfg<T>;
  r.gv = *reinterpret_cast<const Vec4<T>*>(S + lane * C::PITCH + b4);
  // three words: a read of the unused fourth would leave a register that the compiler
  // reuses as a temporary while the read is still in flight
  typedef uint32_t v3u __attribute__((ext_vector_type(3)));
  const v3u f = *reinterpret_cast<const v3u*>(F + lane * C::FPITCH + b4);
  r.f[0] = f.x;
  r.f[1] = f.y;
  r.f[2] = f.z;
}

template <typename T>
struct AdjState {
  T A1;  // A of the previous step (slot + 1)
  T A2;  // A two steps back (slot + 2)
};

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T, int q>
__device__ __forceinline__ T adj_cell(AdjState<T>& st, const AdjGroup<T>& r) {
  // ((gv + NW-routed) + N-routed) + W-routed, one rounding per term: a factor is 0 or 1,
  // so each product is exact and each fused multiply-add rounds once.
  const T p = fma_t(shl1z(st.A2), factor<T, q>(r.f[2]), r.gv.v[q]);
  const T s = fma_t(shl1z(st.A1), factor<T, q>(r.f[1]), p);
  const T A = fma_t(st.A1, factor<T, q>(r.f[0]), s);
  st.A2 = st.A1;
  st.A1 = A;
  return A;
}

template <typename T>
__device__ __forceinline__ void adj_cells4(AdjState<T>& st, const AdjGroup<T>& r, Vec4<T>& out) {
  out.v[3] = adj_cell<T, 3>(st, r);
  out.v[2] = adj_cell<T, 2>(st, r);
  out.v[1] = adj_cell<T, 1>(st, r);
  out.v[0] = adj_cell<T, 0>(st, r);
}

// Unit u covers slots [S0 - G(u+1), S0 - Gu), groups in descending slot order.  The last
// PD groups always read unit u+1's first groups into 'out' (so that both paths below leave
// them in the same registers; conditional reads make the compiler copy every prefetched
// register at each unit boundary).  If unit u+1's inputs were not yet in LDS PD groups
// before the end (by the counters read at the start of the unit), unit u is finished and
// signalled first and the wave then waits for unit u+1 and reads its first groups again.
// Waiting earlier would hold back the last steps of unit u, and with them row 0's values
// for the band above, until the band below has delivered unit u+1: one unit of extra lag
// per band.  After the last unit the reads wrap around the ring and are not used.
template <typename T, int G>
__device__ __forceinline__ bool adj_unit(T* __restrict__ S, const uint32_t* __restrict__ F, AdjShared& sh,
                                         Control* ctl, int zero, int u, int Us, int S0, AdjState<T>& st,
                                         const AdjUnitRegs<T, G>& in, AdjUnitRegs<T, G>& out, uint32_t& stall,
                                         uint64_t& waited) {
  using C = BCfg<T>;
  constexpr int NG = AdjCfg<T, G>::NG, PD = AdjCfg<T, G>::PD;
  const int lane = threadIdx.x & 63;
  const int top = S0 - G * u, next_top = top - G;
  const bool has_next = u + 1 < Us;
  const uint32_t need_l = (uint32_t)((G * (u + 1)) / kSub + 1), need_b = (uint32_t)(u + 2);
  const uint64_t ready = adj_ready(sh, zero);
  const uint32_t ready_f = adj_ready_f(sh, zero);
  AdjGroup<T> gr[NG + PD];
#pragma unroll
  for (int p = 0; p < PD; ++p) gr[p] = in.g[p];
  bool early = true;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (g + PD < NG) {
      adj_load_group<T>(S, F, (top - 4 * (g + PD + 1)) & C::MASK, lane, gr[g + PD]);
    } else {
      if (g + PD == NG) {
        __builtin_amdgcn_sched_barrier(0);
        early = !has_next || __all((uint32_t)ready >= need_l && (uint32_t)(ready >> 32) >= need_b && ready_f >= need_l);
        stall += !early;
        __builtin_amdgcn_sched_barrier(0);
      }
      adj_load_group<T>(S, F, (next_top - 4 * (g + PD - NG + 1)) & C::MASK, lane, out.g[g + PD - NG]);
    }
    __builtin_amdgcn_sched_barrier(0);
    const int b4 = (top - 4 * (g + 1)) & C::MASK;
    Vec4<T> o;
    adj_cells4<T>(st, gr[g], o);
    *reinterpret_cast<Vec4<T>*>(S + lane * C::PITCH + b4) = o;
  }
  lds_signal(&sh.ctr[2], (uint32_t)(G * (u + 1)));
  __builtin_amdgcn_sched_barrier(0);
  if (!early) {
    if (!lds_wait_until([&] { return adj_inputs_ready(sh, zero, need_l, need_b); }, &sh.abort, ctl, waited))
      return false;
    // The slot is hidden from the optimiser: through the restrict pointers it would take
    // these reads for repeats of the early ones above and drop them.
    const int nt = opaque(next_top);
#pragma unroll
    for (int p = 0; p < PD; ++p) adj_load_group<T>(S, F, (nt - 4 * (p + 1)) & C::MASK, lane, out.g[p]);
    __builtin_amdgcn_sched_barrier(0);
  }
  return true;
}

template <typename T, int G>
__device__ __forceinline__ void adj_compute(T* __restrict__ S, const uint32_t* __restrict__ F, AdjShared& sh,
                                            Control* ctl, int Ks, uint64_t* trace) {
  using C = BCfg<T>;
  using E = typename C::E;
  constexpr int PD = AdjCfg<T, G>::PD;
  const int lane = threadIdx.x & 63;
  const int S0 = kSub * Ks;  // slots [0, S0), processed from the top down
  const int Us = S0 / G;
  AdjState<T> st{E::zero(), E::zero()};
  uint64_t waited = 0, t_first = 0;
  uint32_t stall = 0;
  const int zero = adj_opaque_zero();
  {
    if (!adj_inputs_ready(sh, zero, 1u, 1u)) {
      ++stall;
      if (!lds_wait_until([&] { return adj_inputs_ready(sh, zero, 1u, 1u); }, &sh.abort, ctl, waited)) {
        sh.abort = 1u;
        return;
      }
    }
  }
  if (trace) t_first = __builtin_amdgcn_s_memrealtime();
  AdjUnitRegs<T, G> P;
#pragma unroll
  for (int p = 0; p < PD; ++p) adj_load_group<T>(S, F, (S0 - 4 * (p + 1)) & C::MASK, lane, P.g[p]);
  // One unit per iteration: a unit reads its first groups from P and leaves the next
  // unit's there (they are dead by the time those reads are issued, so both use the same
  // registers and nothing is copied at the back edge).
  for (int u = 0; u < Us; ++u) {
    if (!adj_unit<T, G>(S, F, sh, ctl, zero, u, Us, S0, st, P, P, stall, waited)) {
      sh.abort = 1u;
      return;
    }
    // the first unit whose row 0 the band above's first unit needs is done
    if (trace && u == (G + kBand - 1) / G) trace[16] = __builtin_amdgcn_s_memrealtime();
  }
  if (trace && lane == 0) {
    trace[1] = t_first;
    trace[2] = __builtin_amdgcn_s_memrealtime();
    trace[4] = stall;
    trace[8] = waited;
  }
}

// waves 1 and 5: loaders, one 64-slot sub-chunk at a time from the top slot down.  Wave 1:
//  - upstream values gD (plus gscore on the last cell; zeros when gD is absent) into the
//    value ring.
// Wave 5:
//  - the factor words: for the cell of lane r at slot s, byte 0 of the W word says whether
//    cell (r, slot s+1) selected W, byte 0 of the N word whether (r+1, s+1) selected N, byte
//    0 of the NW word whether (r+1, s+2) selected NW -- i.e. whether that successor routes
//    its value here -- and bytes 1..3 the same for slots s+1..s+3 (the group of 4 slots);
//  - row 0's own N and NW planes, which the publisher needs.
// The loads of the next PF (gD) and PFS (planes) sub-chunks are in flight in registers.
template <typename T>
struct AdjPF {
  static constexpr int PF = 1;                         // gD sub-chunks
  static constexpr int PFS = 4;                        // bit-plane sub-chunks
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

// The four 0/1 bits of a 64-bit plane at slots [4g, 4g+4), spread to the four bytes of a word.
__device__ __forceinline__ uint32_t spread4(uint64_t bits, int g) {
  const uint32_t nib = (uint32_t)(bits >> (4 * g)) & 0xFu;
  return (nib * 0x00204081u) & 0x01010101u;
}

// Two waves share the loading: PART 0 writes the upstream values (HAS_G: whether gD is
// given; without it no loads are issued at all) and counts them in ctr[0], PART 1 the factor
// words and row 0's planes, counted in ctr[6].  One wave doing both falls behind the reverse
// chain: it spends longer per sub-chunk than the chain takes to consume it.
template <typename T, int G, bool HAS_G, int PART>
__device__ __forceinline__ void adj_loader(T* S, uint32_t* F, uint32_t* PubR, AdjShared& sh, const AdjArgs& a,
                                           int band, int Ks, uint64_t* tr) {
  using C = BCfg<T>;
  using E = typename C::E;
  constexpr int PF = AdjPF<T>::PF, PFS = AdjPF<T>::PFS;
  static_assert(PFS % PF == 0, "prefetch depths must nest");
  const int lane = threadIdx.x & 63;
  const int64_t ldg = opaque(a.ldgd), n = opaque(a.n), m = opaque(a.m);
  const int64_t row0 = (int64_t)band * kBand;
  const int rows = (int)(m - row0 < kBand ? m - row0 : kBand);
  const __amdgpu_buffer_rsrc_t rsrc =
      make_rsrc(HAS_G ? static_cast<const T*>(a.gD) + row0 * ldg : a.gC,
                HAS_G ? (uint32_t)(((rows - 1) * ldg + n) * (int64_t)sizeof(T)) : 0u);
  // gscore lands on cell (m-1, n-1): band row m-1-row0, slot n-1 + that row
  const int64_t last_row = m - 1 - row0;
  const bool has_last = last_row >= 0 && last_row < kBand && a.gscore != nullptr;
  const T gs = has_last ? *static_cast<const T*>(a.gscore) : E::zero();
  const int64_t last_slot = n - 1 + last_row;
  const uint32_t* selp = a.sel + sel_index(band, Ks, 0, lane);  // + 512 words per sub-chunk
  uint64_t waited = 0;
  constexpr bool LOAD_G = PART == 0 && HAS_G;
  Vec4<T> gbuf[LOAD_G ? PF : 1][16];
  v4i_t sbuf[PART == 1 ? PFS : 1][2];
  // bits of the slots just above the current sub-chunk (the one processed before it)
  uint64_t carry_w = 0, carry_n = 0, carry_nw = 0;
  // reverse order: the kr-th sub-chunk processed is k = Ks-1-kr
  // Loads are issued unconditionally (indices clamped to sub-chunk 0), PFS / PF sub-chunks
  // ahead, so that the number in flight is the same at every wait.
  if constexpr (PART == 1) {
#pragma unroll
    for (int p = 0; p < PFS; ++p) {
      const v4i_t* src = reinterpret_cast<const v4i_t*>(selp + (int64_t)(Ks - 1 - p >= 0 ? Ks - 1 - p : 0) * 512);
      sbuf[p][0] = __builtin_nontemporal_load(src);
      sbuf[p][1] = __builtin_nontemporal_load(src + 1);
    }
  }
  if constexpr (LOAD_G) {
#pragma unroll
    for (int p = 0; p < PF; ++p) adj_load_g<T>(gbuf[p], rsrc, ldg, Ks - 1 - p >= 0 ? Ks - 1 - p : 0);
  }
  for (int kr0 = 0; kr0 < Ks; kr0 += PFS) {
#pragma unroll
    for (int p = 0; p < PFS; ++p) {
      const int kr = kr0 + p;
      const int k = Ks - 1 - kr;  // sub-chunk (slots [64k, 64k+64))
      Vec4<T>(&gx)[16] = gbuf[LOAD_G ? p % PF : 0];
      if (kr < Ks) {
      const int older = kr - C::NSUB;
      if (older >= 0 && (!lds_wait_ge<false>(&sh.ctr[3], (uint32_t)(older + 1), &sh.abort, a.ctl, waited) ||
                         !lds_wait_ge<false>(&sh.ctr[4], (uint32_t)((kSub / G) * (older + 1)), &sh.abort, a.ctl,
                                             waited))) {
        sh.abort = 1u;
        return;
      }
      if constexpr (PART == 0) {
      // upstream values
      const bool interior = rows == kBand && k > 0 && (int64_t)kSub * k + kSub <= n;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = 4 * v + (lane >> 4);
        const int slot = kSub * k + 4 * (lane & 15);
        const int64_t c0 = (int64_t)slot - i;
        Vec4<T> x;
        if constexpr (HAS_G) {
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
      lds_publish(&sh.ctr[0], (uint32_t)(kr + 1));
      } else {
      // factors, aligned to the receiving cell
      const v4i_t w0 = sbuf[p % PFS][0], w1 = sbuf[p % PFS][1];
      const uint64_t pw = (uint32_t)w0.x | ((uint64_t)(uint32_t)w0.y << 32);
      const uint64_t pn_own = (uint32_t)w0.z | ((uint64_t)(uint32_t)w0.w << 32);
      const uint64_t pnw_own = (uint32_t)w1.x | ((uint64_t)(uint32_t)w1.y << 32);
      const uint64_t pn = shl1z_u32((uint32_t)pn_own) | ((uint64_t)shl1z_u32((uint32_t)(pn_own >> 32)) << 32);
      const uint64_t pnw = shl1z_u32((uint32_t)pnw_own) | ((uint64_t)shl1z_u32((uint32_t)(pnw_own >> 32)) << 32);
      const uint64_t fw = (pw >> 1) | (carry_w << 63);       // W selected at slot s+1, own row
      const uint64_t fn = (pn >> 1) | (carry_n << 63);       // N selected at slot s+1, row r+1
      const uint64_t fnw = (pnw >> 2) | (carry_nw << 62);    // NW selected at slot s+2, row r+1
      carry_w = pw & 1u;
      carry_n = pn & 1u;
      carry_nw = pnw & 3u;
      uint32_t* frow = F + lane * C::FPITCH + ((kSub * k) & C::MASK);
#pragma unroll
      for (int g = 0; g < 16; ++g) {
        typedef uint32_t v4u __attribute__((ext_vector_type(4)));
        const v4u f = {spread4(fw, g), spread4(fn, g), spread4(fnw, g), 0u};
        *reinterpret_cast<v4u*>(frow + 4 * g) = f;
      }
      if (lane == 0) {
        typedef uint32_t v4u __attribute__((ext_vector_type(4)));
        const v4u r0 = {(uint32_t)pn_own, (uint32_t)(pn_own >> 32), (uint32_t)pnw_own, (uint32_t)(pnw_own >> 32)};
        *reinterpret_cast<v4u*>(PubR + 4 * (k & (C::NSUB - 1))) = r0;
      }
      lds_publish(&sh.ctr[6], (uint32_t)(kr + 1));
      }
      }
      if constexpr (PART == 1) {
        const v4i_t* src = reinterpret_cast<const v4i_t*>(selp + (int64_t)(k - PFS >= 0 ? k - PFS : 0) * 512);
        sbuf[p][0] = __builtin_nontemporal_load(src);
        sbuf[p][1] = __builtin_nontemporal_load(src + 1);
      }
      if constexpr (LOAD_G) adj_load_g<T>(gx, rsrc, ldg, k - PF >= 0 ? k - PF : 0);
    }
  }
  if (PART == 0 && tr && lane == 0) {
    tr[9] = waited;
    tr[12] = __builtin_amdgcn_s_memrealtime();
  }
}

// wave 2: inputs from the band below.  For lane 63 (band row 63) at slot s, column c = s-63,
// the band below routes pn[c] (its row 0 at column c selected N) and pnw[c+1] (its row 0 at
// column c+1 selected NW).  The poller folds them into lane 63's upstream value in the value
// ring, in the order of the sum: (gv + pnw[c+1]) + pn[c].  Each pass fetches the words of
// the 64 slots below the last unit handed over and hands over every complete unit of G
// slots, so one global round trip advances it by up to 64 slots whatever G is.
template <typename T, int G>
__device__ __forceinline__ void adj_poll(T* S, AdjShared& sh, const AdjArgs& a, int band, int Ks, uint32_t epoch,
                                         uint64_t* tr) {
  using C = BCfg<T>;
  using E = typename C::E;
  constexpr int W = E::W;
  const int lane = threadIdx.x & 63;
  const int64_t n = opaque(a.n);
  const int S0 = kSub * Ks, Us = S0 / G;
  if (band == a.nb - 1) {  // the bottom band has nothing below it
    if (lane == 0) lds_signal(&sh.ctr[1], 0x7fffffffu);
    return;
  }
  uint64_t waited = 0, t0 = 0;
  uint32_t polls = 0;
  T carry_pnw = E::zero();  // pnw of the lowest slot handed over so far
  int u = 0;                // units handed over
  while (u < Us) {
    const int s = S0 - G * u - kSub + lane;  // the window: the 64 slots below slot S0 - Gu
    const int64_t c = (int64_t)s - (kBand - 1);
    const bool real = c >= 0 && c < n;
    // Every lane loads on every pass (a lane with no word to read loads spare words of the
    // control block and ignores them): loads under a lane mask would make each wait drain
    // all of the wave's loads.  Two polls are in flight: while one pass's words are checked
    // the next pass's are on their way.
    const uint64_t* src = real ? a.bnd + ((int64_t)band * n + c) * 2 * W : reinterpret_cast<const uint64_t*>(a.ctl) + 4;
    uint64_t xa[2 * W], xb[2 * W];
    auto issue = [&](uint64_t (&x)[2 * W]) {
#pragma unroll
      for (int q = 0; q < 2 * W; ++q) x[q] = load_word(src + q);
    };
    // units complete in x: the run of ready slots from the top of the window down (slots
    // outside the matrix count as ready), in whole units
    auto complete = [&](const uint64_t (&x)[2 * W]) -> int {
      bool ok = true;
#pragma unroll
      for (int q = 0; q < 2 * W; ++q) ok = ok && (uint32_t)(x[q] >> 32) == epoch;
      ok = ok || !real;
      const uint64_t okm = __ballot(ok);
      const int run = ~okm == 0 ? 64 : __builtin_clzll(~okm);
      const int k = run / G;
      return k < Us - u ? k : Us - u;
    };
    // false when the wait has to give up
    auto pause = [&]() -> bool {
      if (polls == 0 && a.trace) t0 = __builtin_amdgcn_s_memrealtime();
      __builtin_amdgcn_s_sleep(1);
      if ((++polls & 63u) == 0u) {
        if (lds_load(&sh.abort) != 0u || global_aborted(a.ctl)) return false;
        const uint64_t now = __builtin_amdgcn_s_memrealtime();
        if (polls == 64u) {
          if (!a.trace) t0 = now;
        } else if (now - t0 > kSpinTicks) {
          raise_timeout(a.ctl);
          return false;
        }
      }
      return true;
    };
    uint32_t w[2 * W];
    auto take = [&](const uint64_t (&x)[2 * W]) {
#pragma unroll
      for (int q = 0; q < 2 * W; ++q) w[q] = (uint32_t)x[q];
    };
    int k;
    issue(xa);
    for (;;) {
      issue(xb);
      if ((k = complete(xa)) > 0) {
        take(xa);
        break;
      }
      if (!pause()) {
        sh.abort = 1u;
        return;
      }
      issue(xa);
      if ((k = complete(xb)) > 0) {
        take(xb);
        break;
      }
      if (!pause()) {
        sh.abort = 1u;
        return;
      }
    }
    if (polls != 0u) {
      if (a.trace) waited += __builtin_amdgcn_s_memrealtime() - t0;
      polls = 0;
    }
    T vn = E::zero(), vnw = E::zero();
    if (real) {
      vn = E::from_words(w);
      vnw = E::from_words(w + W);
    }
    const int cols = k * G;
    // pnw of column c+1: the next lane's, or for the window's top lane the carried value
    T nw_next = shl1z(vnw);
    if (lane == kSub - 1) nw_next = carry_pnw;
    carry_pnw = lane_value(vnw, kSub - cols);
    // the value ring must hold the upstream values of the units handed over
    const uint32_t need_l = (uint32_t)((G * (u + k - 1)) / kSub + 1);
    if (!lds_wait_ge(&sh.ctr[0], need_l, &sh.abort, a.ctl, waited)) {
      sh.abort = 1u;
      return;
    }
    if (real && lane >= kSub - cols) {
      T* cell = S + (kBand - 1) * C::PITCH + (s & C::MASK);
      *cell = E::add(E::add(*cell, nw_next), vn);
    }
    u += k;
    lds_signal(&sh.ctr[1], (uint32_t)u);
    if (tr && lane == 0 && u == k) tr[15] = __builtin_amdgcn_s_memrealtime();
  }
  if (tr && lane == 0) tr[10] = waited;
}

// wave 3: storer of gC (= A), one sub-chunk at a time from the top slot down
template <typename T, int G>
__device__ __forceinline__ void adj_store(const T* S, AdjShared& sh, const AdjArgs& a, int band, int Ks, uint64_t* tr) {
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
    if (!lds_wait_ge(&sh.ctr[4], (uint32_t)((kSub / G) * (kr + 1)), &sh.abort, a.ctl, waited)) {
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
      // edge sub-chunk: the same 16 LDS reads first, then per vector one 16-byte store if its
      // four cells lie inside the matrix, else a store per cell that does
      Vec4<T> v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = *reinterpret_cast<const Vec4<T>*>(S + (4 * q + (lane >> 4)) * C::PITCH + slot);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = 4 * q + (lane >> 4);
        if (i >= rows) continue;
        const int64_t c0 = (int64_t)kSub * k + j4 - i;
        const int off = (int)(((int64_t)i * ldo + c0) * (int64_t)sizeof(T));
        if (c0 >= 0 && c0 + 4 <= n) {
          if constexpr (sizeof(T) == 4) {
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, v[q]), drs, off, 0, 0);
          } else {
            struct Hf { v4i lo, hi; };
            const Hf hh = __builtin_bit_cast(Hf, v[q]);
            __builtin_amdgcn_raw_buffer_store_b128(hh.lo, drs, off, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b128(hh.hi, drs, off + 16, 0, 0);
          }
          continue;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (c0 + e >= 0 && c0 + e < n) {
            if constexpr (sizeof(T) == 4) {
              __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v[q].v[e]), drs, off + 4 * e, 0, 0);
            } else {
              typedef int v2i __attribute__((ext_vector_type(2)));
              __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v[q].v[e]), drs, off + 8 * e, 0, 0);
            }
          }
        }
      }
    }
    lds_publish(&sh.ctr[3], (uint32_t)(kr + 1));
  }
  if (tr && lane == 0) tr[11] = waited;
}

// wave 4: publisher of row 0's routed values for the band above: at column c (slot c of
// row 0), A times "selected N" and A times "selected NW".
template <typename T, int G>
__device__ __forceinline__ void adj_publish(const T* S, const uint32_t* PubR, AdjShared& sh, const AdjArgs& a,
                                            int band, int Ks, uint32_t epoch, uint64_t* tr) {
  using C = BCfg<T>;
  using E = typename C::E;
  constexpr int W = E::W;
  const int lane = threadIdx.x & 63;
  const int64_t n = opaque(a.n);
  const int S0 = kSub * Ks, Us = S0 / G;
  // an injected fault (tests of the failure path) makes the bottom band withhold its values
  const bool withhold = band == a.nb - 1 && __hip_atomic_load(&a.ctl->fault, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT) == kFaultRevWithhold;
  uint64_t waited = 0;
  for (int u = 0; u < Us;) {
    uint32_t done;
    if (!lds_wait_value<true, false>(&sh.ctr[2], (uint32_t)(G * (u + 1)), &sh.abort, a.ctl, waited, done)) {
      sh.abort = 1u;
      return;
    }
    // every unit finished by now goes out in this pass, up to 64 slots
    int k = (int)(done / G) - u;
    if (k > kSub / G) k = kSub / G;
    if (k > Us - u) k = Us - u;
    const int cols = k * G;
    const bool mark = tr && lane == 0 && u <= (G + kBand - 1) / G && (G + kBand - 1) / G < u + k;
    if (mark) tr[17] = __builtin_amdgcn_s_memrealtime();
    // lane 0 of the compute wave handled slots [S0 - G(u+k), S0 - Gu) = columns
    const int s = S0 - G * (u + k) + lane;
    if (band > 0 && !withhold && lane < cols && s < n) {
      const T A = S[s & C::MASK];  // row 0
      const uint32_t* pr = PubR + 4 * ((s >> 6) & (C::NSUB - 1));
      const int h = (s >> 5) & 1, bit = s & 31;
      const T pn = ((pr[h] >> bit) & 1u) ? A : E::zero();
      const T pnw = ((pr[2 + h] >> bit) & 1u) ? A : E::zero();
      uint64_t* dst = a.bnd + ((int64_t)(band - 1) * n + s) * 2 * W;
#pragma unroll
      for (int q = 0; q < W; ++q) {
        store_word(dst + q, tagged(E::word(pn, q), epoch));
        store_word(dst + W + q, tagged(E::word(pnw, q), epoch));
      }
    }
    if (mark) tr[14] = __builtin_amdgcn_s_memrealtime();
    u += k;
    lds_publish(&sh.ctr[4], (uint32_t)u);
  }
  if (tr && lane == 0) tr[18] = waited;
}

template <typename T>
struct AdjLds {
  Vec4<T> S4[kBand * BCfg<T>::PITCH / 4];
  uint32_t F[kBand * BCfg<T>::FPITCH];
  uint32_t PubR[4 * BCfg<T>::NSUB];
};

// One band of the instance 'a' describes, all six roles.  The LDS counters must be zero on
// entry.
template <typename T, int G>
__device__ __forceinline__ void adj_band(AdjLds<T>& L, AdjShared& sh, const AdjArgs& a, int band, uint32_t epoch,
                                         uint64_t* tr) {
  T* S = reinterpret_cast<T*>(L.S4);
  const int wave = threadIdx.x >> 6;
  const int Ks = (int)((a.n + kBand - 1 + kSub - 1) / kSub);
  if (wave == 0)
    adj_compute<T, G>(S, L.F, sh, a.ctl, Ks, tr);
  else if (wave == 1)
    a.gD ? adj_loader<T, G, true, 0>(S, L.F, L.PubR, sh, a, band, Ks, tr)
         : adj_loader<T, G, false, 0>(S, L.F, L.PubR, sh, a, band, Ks, tr);
  else if (wave == 2)
    adj_poll<T, G>(S, sh, a, band, Ks, epoch, tr);
  else if (wave == 3)
    adj_store<T, G>(S, sh, a, band, Ks, tr);
  else if (wave == 4)
    adj_publish<T, G>(S, L.PubR, sh, a, band, Ks, epoch, tr);
  else
    adj_loader<T, G, false, 1>(S, L.F, L.PubR, sh, a, band, Ks, tr);
}

// TRACE = false compiles every trace statement out (the production instance); the traced
// instance is launched only while tracing is enabled.
template <typename T, int G, bool TRACE>
__global__ __launch_bounds__(kAdjThreads, 1) void adj_kernel(AdjArgs a) {
  if constexpr (!TRACE) a.trace = nullptr;
  __shared__ AdjLds<T> L;
  __shared__ AdjShared sh;
  Control* ctl = a.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x < kAdjCounters) sh.ctr[threadIdx.x] = 0u;
    claim_next(ctl, &sh.item, &sh.abort);
    if (sh.item >= (uint32_t)a.nb || sh.abort != 0u) break;
    const int band = a.nb - 1 - (int)sh.item;  // bottom band first
    uint64_t* tr = a.trace ? a.trace + (int64_t)band * kTraceWords : nullptr;
    if (tr && threadIdx.x == 0) tr[0] = __builtin_amdgcn_s_memrealtime();
    adj_band<T, G>(L, sh, a, band, epoch, tr);
    if (tr && threadIdx.x == 3 * 64) tr[3] = __builtin_amdgcn_s_memrealtime();
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

// Batched reverse sweep: (instance, band) items claimed in list order, which puts every
// band after the band below it of the same instance, so a claimed band only ever waits for
// bands that were claimed before it and are running or done.
template <typename T, int G>
__global__ __launch_bounds__(kAdjThreads, 1) void adj_batch_kernel(BwdBatchArgs b) {
  __shared__ AdjLds<T> L;
  __shared__ AdjShared sh;
  Control* ctl = b.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x < kAdjCounters) sh.ctr[threadIdx.x] = 0u;
    claim_next(ctl, &sh.item, &sh.abort);
    // the same for every lane: read it into a scalar register, so that the item's fields are
    // scalar loads and kernel-wide values for the roles
    const uint32_t item = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.item);
    if (item >= (uint32_t)b.n_items || sh.abort != 0u) break;
    const BatchItem it = load_uniform(b.items + item);
    const BwdInst in = load_uniform(b.inst + it.inst);
    AdjArgs a;
    a.sel = b.sel + in.sel_off;
    a.gD = b.gD ? static_cast<const T*>(b.gD) + in.off : nullptr;
    a.gscore = b.gscores ? static_cast<const T*>(b.gscores) + it.inst : nullptr;
    a.gC = static_cast<T*>(b.gC) + in.off;
    a.ldgd = in.n;
    a.ldgc = in.n;
    a.m = in.m;
    a.n = in.n;
    a.nb = in.nb;
    a.ctl = ctl;
    a.bnd = b.bnd + in.bnd_off;
    a.trace = nullptr;
    adj_band<T, G>(L, sh, a, it.band, epoch, nullptr);
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

// =======================================================================================
// 3. Adjoint of the score alone by the argmin path (no upstream gradient of the table).
// =======================================================================================

// The selection recompute with the exits of every band's last row (and the captured
// labels) besides the bit-planes; otherwise sel_kernel.
template <typename T>
__global__ __launch_bounds__(128, 1) void sel_path_kernel(SelArgs a, PathLabels po) {
  __shared__ SelLds<T> L;
  __shared__ SelShared sh;
  Control* ctl = a.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      sh.loaded = 0u;
      sh.steps = 0u;
    }
    claim_next(ctl, &sh.item, &sh.abort);
    const int pieces = a.split > 0 ? a.pieces : 1;
    const int item = (int)sh.item;
    if (item >= a.nb * pieces || sh.abort != 0u) break;
    sel_item<T, true>(L, sh, a, item / pieces, item % pieces, po);
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

// Zeroes an m x n matrix of leading dimension ld: rows over the grid, 16-byte stores along a
// row when the rows are 16-byte aligned.
template <typename T>
__global__ __launch_bounds__(256) void zero_kernel(T* __restrict__ p, int64_t m, int64_t n, int64_t ld, int vec) {
  for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
    T* row = p + i * ld;
    int64_t j0 = 0;
    if (vec) {
      const int64_t nv = n * (int64_t)sizeof(T) / 16;
      uint4* r4 = reinterpret_cast<uint4*>(row);
      for (int64_t j = threadIdx.x; j < nv; j += blockDim.x) r4[j] = make_uint4(0u, 0u, 0u, 0u);
      j0 = nv * 16 / (int64_t)sizeof(T);
    }
    for (int64_t j = j0 + threadIdx.x; j < n; j += blockDim.x) row[j] = T(0);
  }
}

// An exit as stored (a column, -1, or -2 - r of a split band's second piece) made a column
// or -1; anything out of range reads as -1.
__device__ __forceinline__ int32_t path_resolve(const PathArgs& a, int b, int32_t v) {
  // a label of piece p >= 1 names a row of piece p - 1's capture, which may name one of
  // piece p - 2's, and so on
  for (int hop = 0; hop < kMaxPieces && v <= -2; ++hop)
    v = v >= -1 - 64 * (kMaxPieces - 1) ? a.caps[(int64_t)b * kMaxPieces * 64 + (-2 - v)] : -1;
  return (v >= 0 && v < a.n) ? v : -1;
}

// F[g][p] for the groups g >= 1: the path entering the last band of group g at column p,
// followed up through the group's bands.
__device__ __forceinline__ void compose_one(const PathArgs& a, int g, int64_t p) {
  const int lo = g * a.S;
  const int hi = (lo + a.S < a.nb - 1 ? lo + a.S : a.nb - 1) - 1;
  int32_t v = (int32_t)p;
  for (int b = hi; b >= lo && v >= 0; --b) v = path_resolve(a, b, a.exits[(int64_t)b * a.n + v]);
  a.F[(int64_t)g * a.n + p] = v;
}

__global__ __launch_bounds__(256) void compose_kernel(PathArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < a.n) compose_one(a, (int)blockIdx.y + 1, p);
}

// One wave per band: the column at which the path enters the band's last row (the last
// cell for the last band; otherwise the end cell's exit followed down through the groups
// and then through the bands of the band's own group), then the walk up the band along the
// selections, writing the score's upstream value on every cell of the path.  The rows'
// runs of path cells are written by the lanes at once.
template <typename T>
__device__ __forceinline__ void walk_band(const PathArgs& a, int b) {
  const int lane = (int)threadIdx.x;
  T gv = a.gscore ? *static_cast<const T*>(a.gscore) : T(0);
  gv = gv + T(0);  // the last cell's value is 0 + gscore
  if (gv == T(0)) return;
  const int nb = a.nb;
  const int64_t n = a.n;
  const int rows_last = (int)(a.m - (int64_t)(nb - 1) * kBand);
  int32_t q = (int32_t)(n - 1);
  if (b < nb - 1) {
    const int endp = a.split > 0 ? a.pieces - 1 : 0;
    q = path_resolve(a, nb - 1, a.caps[((int64_t)(nb - 1) * kMaxPieces + endp) * 64 + rows_last - 1]);
    const int gb = b / a.S;
    for (int g = (nb - 2) / a.S; g > gb && q >= 0; --g) {
      q = a.F[(int64_t)g * n + q];
      q = (q >= 0 && q < n) ? q : -1;
    }
    const int btop = (gb * a.S + a.S < nb - 1 ? gb * a.S + a.S : nb - 1) - 1;
    for (int bb = btop; bb > b && q >= 0; --bb) q = path_resolve(a, bb, a.exits[(int64_t)bb * n + q]);
  }
  q = __builtin_amdgcn_readfirstlane(q);
  if (q < 0) return;
  const int rows = b == nb - 1 ? rows_last : kBand;
  T* g0 = static_cast<T*>(a.gC) + (int64_t)b * kBand * a.ldgc;
  const uint32_t* planes = a.sel;
  int r = rows - 1;
  int64_t col = q;
  int64_t run_hi = col;
  int kcur = -1;
  uint32_t w[6] = {0u, 0u, 0u, 0u, 0u, 0u};
  auto flush = [&](int row, int64_t lo, int64_t hi) {
    for (int64_t c = lo + lane; c <= hi; c += 64) g0[(int64_t)row * a.ldgc + c] = gv;
  };
  for (;;) {
    const int64_t s = col + r;
    const int k = (int)(s >> 6);
    if (k != kcur) {
      const uint4* src = reinterpret_cast<const uint4*>(planes + sel_index(b, a.Ks, k, lane));
      const uint4 x0 = src[0], x1 = src[1];
      w[0] = x0.x; w[1] = x0.y; w[2] = x0.z; w[3] = x0.w; w[4] = x1.x; w[5] = x1.y;
      kcur = k;
    }
    const int j = (int)(s & 63), h = j >> 5, bit = j & 31;
    const uint32_t sw = (uint32_t)__builtin_amdgcn_readlane((int)(h ? w[1] : w[0]), r);
    const uint32_t sn = (uint32_t)__builtin_amdgcn_readlane((int)(h ? w[3] : w[2]), r);
    const uint32_t snw = (uint32_t)__builtin_amdgcn_readlane((int)(h ? w[5] : w[4]), r);
    if ((sw >> bit) & 1u) {
      if (col == 0) break;  // never selected: W of column 0 is outside the matrix
      --col;
      continue;
    }
    flush(r, col, run_hi);
    if ((sn >> bit) & 1u) {
      if (r == 0) break;  // into the band above
      --r;
    } else if ((snw >> bit) & 1u) {
      if (r == 0 || col == 0) break;  // into the band above, or outside the matrix
      --r;
      --col;
    } else {
      break;  // cell (0, 0)
    }
    run_hi = col;
  }
}

template <typename T>
__global__ __launch_bounds__(64) void walk_kernel(PathArgs a) {
  walk_band<T>(a, (int)blockIdx.x);
}

// The path arguments of instance 'inst' of a batch (no split bands in a batch).
template <typename T>
__device__ __forceinline__ PathArgs inst_path(const BwdBatchArgs& b, const PathBufs& pb, const BwdInst& in, int inst) {
  PathArgs a;
  a.exits = pb.exits + in.sel_off / 8;
  a.caps = pb.caps + in.sel_off / 2;
  a.F = pb.F + in.sel_off / 8;
  a.sel = b.sel + in.sel_off;
  a.gscore = b.gscores ? static_cast<const T*>(b.gscores) + inst : nullptr;
  a.gC = static_cast<T*>(b.gC) + in.off;
  a.ldgc = in.n;
  a.m = in.m;
  a.n = in.n;
  a.split = 0;
  a.pieces = 1;
  a.nb = in.nb;
  a.Ks = (int32_t)((in.n + kBand - 1 + kSub - 1) / kSub);
  a.S = path_group_size(in.nb);
  a.G = in.nb > 1 ? (in.nb - 1 + a.S - 1) / a.S : 0;
  return a;
}

// Batched labelled selection recompute: sel_batch_kernel with every instance's exits and
// captured labels, and its gradient zeroed.
template <typename T>
__global__ __launch_bounds__(128, 1) void sel_path_batch_kernel(BwdBatchArgs b, PathBufs pb) {
  __shared__ SelLds<T> L;
  __shared__ SelShared sh;
  Control* ctl = b.ctl;
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) sh.abort = 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      sh.loaded = 0u;
      sh.steps = 0u;
    }
    claim_next(ctl, &sh.item, &sh.abort);
    const uint32_t item = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.item);
    if (item >= (uint32_t)b.n_items || sh.abort != 0u) break;
    const BatchItem it = load_uniform(b.items + item);
    const BwdInst in = load_uniform(b.inst + it.inst);
    SelArgs a;
    a.C = static_cast<const T*>(b.C) + in.off;
    if (b.ckpt_k > 0) {
      a.top = static_cast<const T*>(b.top) + in.ck_off;
      a.ld_top = in.n;
    } else {
      a.top = static_cast<const T*>(b.top) + in.off + 63 * in.n;
      a.ld_top = 64 * in.n;
    }
    a.ldc = in.n;
    a.m = in.m;
    a.n = in.n;
    a.nb = in.nb;
    a.sel = b.sel + in.sel_off;
    a.ctl = ctl;
    a.split = 0;
    a.left = nullptr;
    a.ld_left = 0;
    a.left_pstride = 0;
    a.pieces = 1;
    a.pad = 0;
    const PathLabels po{pb.exits + in.sel_off / 8, pb.caps + in.sel_off / 2, static_cast<T*>(b.gC) + in.off, in.n};
    sel_item<T, true>(L, sh, a, it.band, 0, po);
    __syncthreads();
  }
  finish_launch(ctl, epoch);
}

template <typename T>
__global__ __launch_bounds__(256) void compose_batch_kernel(BwdBatchArgs b, PathBufs pb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int i = (int)blockIdx.y; i < pb.batch; i += (int)gridDim.y) {
    const BwdInst in = b.inst[i];
    const PathArgs a = inst_path<T>(b, pb, in, i);
    if (a.G < 2 || t >= (int64_t)(a.G - 1) * a.n) continue;
    compose_one(a, 1 + (int)(t / a.n), t % a.n);
  }
}

template <typename T>
__global__ __launch_bounds__(64) void walk_batch_kernel(BwdBatchArgs b, PathBufs pb) {
  const BatchItem it = load_uniform(b.items + blockIdx.x);
  const BwdInst in = load_uniform(b.inst + it.inst);
  walk_band<T>(inst_path<T>(b, pb, in, it.inst), it.band);
}

template <typename T, bool TRACE>
hipError_t launch_adj_tt(int tile, const AdjArgs& a, int grid, hipStream_t s) {
  switch (tile) {
    case 16: hipLaunchKernelGGL((adj_kernel<T, 16, TRACE>), dim3(grid), dim3(kAdjThreads), 0, s, a); break;
    case 32: hipLaunchKernelGGL((adj_kernel<T, 32, TRACE>), dim3(grid), dim3(kAdjThreads), 0, s, a); break;
    case 64: hipLaunchKernelGGL((adj_kernel<T, 64, TRACE>), dim3(grid), dim3(kAdjThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_t(int tile, const AdjArgs& a, int grid, hipStream_t s) {
  return a.trace ? launch_adj_tt<T, true>(tile, a, grid, s) : launch_adj_tt<T, false>(tile, a, grid, s);
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

hipError_t launch_select_path(int dtype, const SelArgs& a, const PathLabels& p, int grid, hipStream_t s) {
  switch (dtype) {
    case 0: hipLaunchKernelGGL((sel_path_kernel<float>), dim3(grid), dim3(128), 0, s, a, p); break;
    case 1: hipLaunchKernelGGL((sel_path_kernel<double>), dim3(grid), dim3(128), 0, s, a, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zero(int dtype, void* p, int64_t m, int64_t n, int64_t ld, int grid, hipStream_t s) {
  const int es = dtype == 1 ? 8 : 4;
  const int vec = ((uintptr_t)p % 16 == 0 && (ld * es) % 16 == 0) ? 1 : 0;
  const int g = (int)std::min<int64_t>(m, grid);
  switch (dtype) {
    case 0: hipLaunchKernelGGL((zero_kernel<float>), dim3(g), dim3(256), 0, s, static_cast<float*>(p), m, n, ld, vec); break;
    case 1: hipLaunchKernelGGL((zero_kernel<double>), dim3(g), dim3(256), 0, s, static_cast<double*>(p), m, n, ld, vec); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_path(int dtype, const PathArgs& a, hipStream_t s) {
  if (a.G > 1) {
    hipLaunchKernelGGL(compose_kernel, dim3((unsigned)((a.n + 255) / 256), (unsigned)(a.G - 1)), dim3(256), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  switch (dtype) {
    case 0: hipLaunchKernelGGL((walk_kernel<float>), dim3(a.nb), dim3(64), 0, s, a); break;
    case 1: hipLaunchKernelGGL((walk_kernel<double>), dim3(a.nb), dim3(64), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_path_batch_t(const BwdBatchArgs& b, const PathBufs& pb, int grid, hipStream_t s) {
  hipLaunchKernelGGL((sel_path_batch_kernel<T>), dim3(grid), dim3(128), 0, s, b, pb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (pb.max_cols > 0) {
    const unsigned gy = (unsigned)std::min<int32_t>(pb.batch, 65535);
    hipLaunchKernelGGL((compose_batch_kernel<T>), dim3((unsigned)((pb.max_cols + 255) / 256), gy), dim3(256), 0, s, b,
                       pb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((walk_batch_kernel<T>), dim3((unsigned)b.n_items), dim3(64), 0, s, b, pb);
  return hipGetLastError();
}

hipError_t launch_path_batch(int dtype, const BwdBatchArgs& b, const PathBufs& pb, int grid, hipStream_t s) {
  switch (dtype) {
    case 0: return launch_path_batch_t<float>(b, pb, grid, s);
    case 1: return launch_path_batch_t<double>(b, pb, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_select_batch(int dtype, const BwdBatchArgs& b, int grid, hipStream_t s) {
  switch (dtype) {
    case 0: hipLaunchKernelGGL((sel_batch_kernel<float>), dim3(grid), dim3(128), 0, s, b); break;
    case 1: hipLaunchKernelGGL((sel_batch_kernel<double>), dim3(grid), dim3(128), 0, s, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_batch_t(int tile, const BwdBatchArgs& b, int grid, hipStream_t s) {
  switch (tile) {
    case 16: hipLaunchKernelGGL((adj_batch_kernel<T, 16>), dim3(grid), dim3(kAdjThreads), 0, s, b); break;
    case 32: hipLaunchKernelGGL((adj_batch_kernel<T, 32>), dim3(grid), dim3(kAdjThreads), 0, s, b); break;
    case 64: hipLaunchKernelGGL((adj_batch_kernel<T, 64>), dim3(grid), dim3(kAdjThreads), 0, s, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_batch(int dtype, int tile, const BwdBatchArgs& b, int grid, hipStream_t s) {
  switch (dtype) {
    case 0: return launch_adj_batch_t<float>(tile, b, grid, s);
    case 1: return launch_adj_batch_t<double>(tile, b, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wf
