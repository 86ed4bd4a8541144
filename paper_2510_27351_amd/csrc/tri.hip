// The tridiagonal partition method on gfx950 (declared in include/tri.h): the Stage 1 and
// Stage 3 kernels, the Thomas solve of the deepest interface system, plans over the
// recursive levels, the sub-system-size / recursion-depth predictor and the C ABI.
//
// Data-parallel structure (the paper's Introduction): every sub-system is handled by one
// lane.  A workgroup is one wave that owns S consecutive sub-systems of one system; their
// rows are contiguous in memory, so the wave stages them into LDS with coalesced loads (one
// element per lane per load, 64 consecutive elements per instruction) into a layout with
// one odd-pitched row of LDS per sub-system.  Lanes then read "their" sub-system at a
// stride the banks can serve without conflicts, and the results go back out through the
// same layout with coalesced stores.  All of a sub-system's arithmetic is in the order of
// the method's elimination, with the same operations as the plain definitions, so the
// interface systems and the solution are those of a row-by-row evaluation bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/tri.h"

namespace tri {
namespace {

constexpr int kLanes = 64;                // the stage kernels run one wave per workgroup
constexpr int kLdsBudget = 20 * 1024;     // LDS bytes a stage workgroup aims at (8 per CU)
constexpr int kLdsMax = 64 * 1024;        // LDS bytes a stage workgroup may take at most

// The LDS budget of a stage workgroup: kLdsBudget, or TRI_LDS_BUDGET (bytes, 4 KiB .. 64 KiB)
// from the environment, read once.
int lds_budget() {
  static const int b = [] {
    const char* e = std::getenv("TRI_LDS_BUDGET");
    const int v = e ? std::atoi(e) : 0;
    return v >= 4096 && v <= kLdsMax ? v : kLdsBudget;
  }();
  return b;
}
constexpr int kThomasThreads = 256;

int elem_bytes(int dtype) { return dtype == WF_F64 ? 8 : dtype == WF_F32 ? 4 : 0; }

// Row pitch, in elements, of one sub-system in LDS: at least m+1 (the last sub-system of a
// system may hold m+1 rows) and odd, so that 64 lanes reading row i of 64 consecutive
// sub-systems touch distinct banks.
int pitch_of(int m) {
  const int p = m + 1;
  return (p & 1) ? p : p + 1;
}

// Sub-systems per workgroup: at most 'cap' (32 for Stage 1, whose sub-systems take two lanes
// each, 64 for Stage 3), and as many as the LDS budget allows for four arrays; at least one.
int subsystems_per_group(int m, int es, int cap) {
  const int per = 4 * pitch_of(m) * es;
  int s = lds_budget() / per;
  if (s > cap) s = cap;
  if (s < 1) s = 1;
  return s;
}

int max_m(int dtype) {
  // one sub-system of four arrays must fit in kLdsMax
  const int es = elem_bytes(dtype);
  int m = kLdsMax / (4 * es) - 2;
  while (4 * pitch_of(m) * es > kLdsMax) --m;
  return m;
}

}  // namespace

int64_t partition_count(int64_t N, int64_t m) {
  if (N < 2 || m < 2) return -1;
  int64_t P = (N + m - 1) / m;
  if (P > 1 && N - (P - 1) * m == 1) --P;  // a one-row remainder joins the sub-system before
  return P;
}

// Arguments of the two stage kernels.
struct StageArgs {
  const void* a;
  const void* b;
  const void* c;
  const void* d;
  void* A;          // Stage 1: interface system out (batch * 2P each)
  void* B;
  void* C;
  void* D;
  const void* z;    // Stage 3: interface unknowns in (batch * 2P)
  void* x;          // Stage 3: solution out (batch * N)
  int64_t n;        // rows per system
  int64_t P;        // sub-systems per system
  int64_t groups;   // workgroups per system = ceil(P / S)
  int32_t m;        // sub-system size
  int32_t S;        // sub-systems per workgroup
  int32_t pitch;    // LDS row pitch per sub-system (elements)
  float rm;         // 1 / m, for the row -> sub-system mapping
};

// Sub-system of row q (0-based inside the workgroup's block of rows), clamped to the block's
// last sub-system, which takes the extra row of a merged remainder.
__device__ __forceinline__ int block_sub(int q, int m, float rm, int last) {
  int k = (int)((float)q * rm);
  if (k * m > q) --k;
  else if ((k + 1) * m <= q) ++k;
  return k < last ? k : last;
}

// The workgroup's block: system 'inst', sub-systems [k0, k0 + Sb), rows [r0, r0 + cnt) of
// the system.
struct Block {
  int64_t inst, k0, r0;
  int Sb, cnt;
};

__device__ __forceinline__ Block block_of(const StageArgs& g) {
  Block bl;
  bl.inst = (int64_t)blockIdx.x / g.groups;
  const int64_t grp = (int64_t)blockIdx.x - bl.inst * g.groups;
  bl.k0 = grp * g.S;
  const int64_t left = g.P - bl.k0;
  bl.Sb = (int)(left < g.S ? left : g.S);
  bl.r0 = bl.k0 * g.m;
  const int64_t r1 = (bl.k0 + bl.Sb == g.P) ? g.n : (bl.k0 + bl.Sb) * g.m;
  bl.cnt = (int)(r1 - bl.r0);
  return bl;
}

// Rows of sub-system gk of a system.
__device__ __forceinline__ int sub_rows(int64_t gk, const StageArgs& g) {
  return gk == g.P - 1 ? (int)(g.n - (g.P - 1) * g.m) : g.m;
}

// Stages the block's rows of the four arrays into LDS (sub-system k's row i at k*pitch + i).
// Sixteen rows per lane per round, all loads of a round issued before their LDS writes: a
// block within the LDS budget holds about 600 rows, so its loads leave in one round and
// wait out one memory latency.
template <typename T>
__device__ __forceinline__ void stage_in(const StageArgs& g, const Block& bl, T* la, T* lb, T* lc, T* ld) {
  const T* __restrict__ ga = static_cast<const T*>(g.a) + bl.inst * g.n + bl.r0;
  const T* __restrict__ gb = static_cast<const T*>(g.b) + bl.inst * g.n + bl.r0;
  const T* __restrict__ gc = static_cast<const T*>(g.c) + bl.inst * g.n + bl.r0;
  const T* __restrict__ gd = static_cast<const T*>(g.d) + bl.inst * g.n + bl.r0;
  const int t = threadIdx.x;
  constexpr int U = 16;
  for (int q0 = 0; q0 < bl.cnt; q0 += kLanes * U) {
    T va[U], vb[U], vc[U], vd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * kLanes + t;
      if (q < bl.cnt) {
        va[u] = ga[q];
        vb[u] = gb[q];
        vc[u] = gc[q];
        vd[u] = gd[q];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * kLanes + t;
      if (q < bl.cnt) {
        const int k = block_sub(q, g.m, g.rm, bl.Sb - 1);
        const int s = k * g.pitch + (q - k * g.m);
        la[s] = va[u];
        lb[s] = vb[u];
        lc[s] = vc[u];
        ld[s] = vd[u];
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Stage 1: the two interface equations of every sub-system.
//
// Lane l < 32 eliminates sub-system l of the block downward (rows s+1 .. e, x_s kept as a
// spike): row s+1 is a x_s + b x + c x = d, and each next row i loses its x_{i-1} term by
// subtracting w = a[i]/p times the row above, which gives f_i x_s + p_i x_i + c[i] x_{i+1}
// = q_i with f_i = -w f, p_i = b[i] - w c[i-1], q_i = d[i] - w q.  The last row's (f, p,
// c[e], q) is interface row 2k+1.  Lane 32 + l eliminates the same sub-system upward (rows
// e-1 .. s, x_e kept), the mirror image with w = c[i]/r, g = -w g, r = b[i] - w a[i+1],
// t = d[i] - w t; row s's (a[s], r, g, t) is interface row 2k.  Both run the same
// instruction stream: the direction picks which LDS array plays "a" and which "c" and the
// sign of the row step, so the wave does not diverge.
template <typename T>
__global__ __launch_bounds__(64) void stage1_kernel(StageArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* la = reinterpret_cast<T*>(smem);
  T* lb = la + g.S * g.pitch;
  T* lc = lb + g.S * g.pitch;
  T* ld = lc + g.S * g.pitch;
  const Block bl = block_of(g);
  stage_in<T>(g, bl, la, lb, lc, ld);
  __syncthreads();

  const int lane = threadIdx.x;
  const bool down = lane < 32;
  const int k = down ? lane : lane - 32;
  if (k >= bl.Sb) return;
  const int64_t gk = bl.k0 + k;
  const int L = sub_rows(gk, g);
  const T* Ur = down ? la : lc;  // the coefficient eliminated at each step
  const T* Yr = down ? lc : la;  // the neighbour coefficient of the previous row
  const int base = k * g.pitch;
  const int dir = down ? 1 : -1;
  int i = down ? 1 : L - 2;
  T x1 = Ur[base + i], x2 = lb[base + i], x3 = ld[base + i];
  for (int j = 0; j < L - 2; ++j) {
    i += dir;
    const T w = Ur[base + i] / x2;
    x1 = -w * x1;
    x2 = lb[base + i] - w * Yr[base + i - dir];
    x3 = ld[base + i] - w * x3;
  }
  const int64_t row = bl.inst * 2 * g.P + 2 * gk + (down ? 1 : 0);
  const T zero = T(0);
  static_cast<T*>(g.A)[row] = down ? x1 : (gk > 0 ? la[base] : zero);
  static_cast<T*>(g.B)[row] = x2;
  static_cast<T*>(g.C)[row] = down ? (gk < g.P - 1 ? lc[base + L - 1] : zero) : x1;
  static_cast<T*>(g.D)[row] = x3;
}

// ---------------------------------------------------------------------------------------
// Stage 3: with x_s = z[2k] and x_e = z[2k+1] known, the interior rows s+1 .. e-1 of
// sub-system k.  The downward elimination of Stage 1 is recomputed (f, p, q per row) and
// back substitution runs from x_e: x_i = (q_i - f_i x_s - c[i] x_{i+1}) / p_i.  In LDS, row
// i's a slot receives p_i and its b slot q_i - f_i x_s during the elimination, and its d
// slot the solution, which then leaves through the coalesced store path.
template <typename T>
__global__ __launch_bounds__(64) void stage3_kernel(StageArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* la = reinterpret_cast<T*>(smem);
  T* lb = la + g.S * g.pitch;
  T* lc = lb + g.S * g.pitch;
  T* ld = lc + g.S * g.pitch;
  const Block bl = block_of(g);
  stage_in<T>(g, bl, la, lb, lc, ld);
  __syncthreads();

  const int k = threadIdx.x;
  if (k < bl.Sb) {
    const int64_t gk = bl.k0 + k;
    const int L = sub_rows(gk, g);
    const int base = k * g.pitch;
    const T* z = static_cast<const T*>(g.z) + bl.inst * 2 * g.P + 2 * gk;
    const T xs = z[0], xe = z[1];
    if (L >= 3) {
      T f = la[base + 1], p = lb[base + 1], q = ld[base + 1];
      la[base + 1] = p;
      lb[base + 1] = q - f * xs;
      for (int i = 2; i <= L - 2; ++i) {
        const T w = la[base + i] / p;
        f = -w * f;
        p = lb[base + i] - w * lc[base + i - 1];
        q = ld[base + i] - w * q;
        la[base + i] = p;
        lb[base + i] = q - f * xs;
      }
      T xn = xe;
      for (int i = L - 2; i >= 1; --i) {
        xn = (lb[base + i] - lc[base + i] * xn) / la[base + i];
        ld[base + i] = xn;
      }
    }
    ld[base] = xs;
    ld[base + L - 1] = xe;
  }
  __syncthreads();

  // the block's solution rows out, coalesced
  T* __restrict__ gx = static_cast<T*>(g.x) + bl.inst * g.n + bl.r0;
  for (int q = threadIdx.x; q < bl.cnt; q += kLanes) {
    const int kk = block_sub(q, g.m, g.rm, bl.Sb - 1);
    gx[q] = ld[kk * g.pitch + (q - kk * g.m)];
  }
}

// ---------------------------------------------------------------------------------------
// The Thomas algorithm for one system per workgroup: forward elimination
//   piv_i = b_i - a_i cp_{i-1},  cp_i = c_i / piv_i,  dp_i = (d_i - a_i dp_{i-1}) / piv_i
// (row 0: piv = b_0, dp_0 = d_0 / b_0; cp of the last row is 0), then back substitution
// x_{n-1} = dp_{n-1}, x_i = dp_i - cp_i x_{i+1}.  The recurrences are serial, so one lane
// runs them; the workgroup stages the rows through LDS in chunks with coalesced loads and
// writes cp, dp to the scratch arrays and the solution back with coalesced stores.
template <typename T>
struct ThomasCfg {
  static constexpr int CH = 8192 / sizeof(T);  // rows per chunk: 8 KiB per array
};

template <typename T>
__global__ __launch_bounds__(kThomasThreads) void thomas_kernel(const T* __restrict__ a, const T* __restrict__ b,
                                                                const T* __restrict__ c, const T* __restrict__ d,
                                                                T* __restrict__ x, T* __restrict__ cp,
                                                                T* __restrict__ dp, int64_t n) {
  constexpr int CH = ThomasCfg<T>::CH;
  __shared__ T sa[CH], sb[CH], sc[CH], sd[CH];
  const int64_t off = (int64_t)blockIdx.x * n;
  a += off;
  b += off;
  c += off;
  d += off;
  x += off;
  cp += off;
  dp += off;
  const int t = threadIdx.x;
  const int64_t nch = (n + CH - 1) / CH;

  T cprev = T(0), dprev = T(0);
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int64_t i0 = ch * CH;
    const int len = (int)std::min<int64_t>(CH, n - i0);
    for (int q = t; q < len; q += kThomasThreads) {
      sa[q] = a[i0 + q];
      sb[q] = b[i0 + q];
      sc[q] = c[i0 + q];
      sd[q] = d[i0 + q];
    }
    __syncthreads();
    if (t == 0) {
      // the chain runs through piv and the two divisions; the next rows' LDS reads are
      // issued a group ahead so that their latency stays off it
      constexpr int U = 8;
      T ra[U], rb[U], rc[U], rd[U];
      auto fetch = [&](int q0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int q = q0 + u < len ? q0 + u : len - 1;
          ra[u] = sa[q];
          rb[u] = sb[q];
          rc[u] = sc[q];
          rd[u] = sd[q];
        }
      };
      fetch(0);
      for (int q0 = 0; q0 < len; q0 += U) {
        T xa[U], xb[U], xc[U], xd[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          xa[u] = ra[u];
          xb[u] = rb[u];
          xc[u] = rc[u];
          xd[u] = rd[u];
        }
        fetch(q0 + U < len ? q0 + U : q0);
        T cpo[U], dpo[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t i = i0 + q0 + u;
          T piv, dpi;
          if (i == 0) {
            piv = xb[u];
            dpi = xd[u] / piv;
          } else {
            piv = xb[u] - xa[u] * cprev;
            dpi = (xd[u] - xa[u] * dprev) / piv;
          }
          const T cpi = i < n - 1 ? xc[u] / piv : T(0);
          cpo[u] = cpi;
          dpo[u] = dpi;
          cprev = cpi;
          dprev = dpi;
        }
        // the stored values go to the scratch arrays through LDS (the chunk's c and d slots,
        // already read)
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (q0 + u < len) {
            sc[q0 + u] = cpo[u];
            sd[q0 + u] = dpo[u];
          }
      }
    }
    __syncthreads();
    for (int q = t; q < len; q += kThomasThreads) {
      cp[i0 + q] = sc[q];
      dp[i0 + q] = sd[q];
    }
    __syncthreads();
  }

  T xnext = T(0);
  for (int64_t ch = nch - 1; ch >= 0; --ch) {
    const int64_t i0 = ch * CH;
    const int len = (int)std::min<int64_t>(CH, n - i0);
    for (int q = t; q < len; q += kThomasThreads) {
      sc[q] = cp[i0 + q];
      sd[q] = dp[i0 + q];
    }
    __syncthreads();
    if (t == 0) {
      constexpr int U = 8;
      for (int q1 = len; q1 > 0; q1 -= U) {
        T xc[U], xd[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int q = q1 - 1 - u >= 0 ? q1 - 1 - u : 0;
          xc[u] = sc[q];
          xd[u] = sd[q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int q = q1 - 1 - u;
          if (q >= 0) {
            const int64_t i = i0 + q;
            const T xi = i == n - 1 ? xd[u] : xd[u] - xc[u] * xnext;
            sa[q] = xi;
            xnext = xi;
          }
        }
      }
    }
    __syncthreads();
    for (int q = t; q < len; q += kThomasThreads) x[i0 + q] = sa[q];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Launchers.

namespace {

StageArgs stage_args(int dtype, int64_t n, int m, int cap) {
  StageArgs g;
  std::memset(&g, 0, sizeof(g));
  g.n = n;
  g.m = m;
  g.P = partition_count(n, m);
  g.S = subsystems_per_group(m, elem_bytes(dtype), cap);
  g.pitch = pitch_of(m);
  g.groups = (g.P + g.S - 1) / g.S;
  g.rm = 1.0f / (float)m;
  return g;
}

size_t stage_lds(int dtype, const StageArgs& g) { return (size_t)4 * g.S * g.pitch * elem_bytes(dtype); }

hipError_t launch_stage1(int dtype, int32_t batch, const StageArgs& g, hipStream_t s) {
  const dim3 grid((unsigned)(batch * g.groups)), block(kLanes);
  const size_t lds = stage_lds(dtype, g);
  if (dtype == WF_F64)
    hipLaunchKernelGGL(stage1_kernel<double>, grid, block, lds, s, g);
  else
    hipLaunchKernelGGL(stage1_kernel<float>, grid, block, lds, s, g);
  return hipGetLastError();
}

hipError_t launch_stage3(int dtype, int32_t batch, const StageArgs& g, hipStream_t s) {
  const dim3 grid((unsigned)(batch * g.groups)), block(kLanes);
  const size_t lds = stage_lds(dtype, g);
  if (dtype == WF_F64)
    hipLaunchKernelGGL(stage3_kernel<double>, grid, block, lds, s, g);
  else
    hipLaunchKernelGGL(stage3_kernel<float>, grid, block, lds, s, g);
  return hipGetLastError();
}

hipError_t launch_thomas(int dtype, int32_t batch, int64_t n, const void* a, const void* b, const void* c,
                         const void* d, void* x, void* scratch, hipStream_t s) {
  const dim3 grid((unsigned)batch), block(kThomasThreads);
  if (dtype == WF_F64) {
    double* cp = static_cast<double*>(scratch);
    hipLaunchKernelGGL(thomas_kernel<double>, grid, block, 0, s, static_cast<const double*>(a),
                       static_cast<const double*>(b), static_cast<const double*>(c), static_cast<const double*>(d),
                       static_cast<double*>(x), cp, cp + (int64_t)batch * n, n);
  } else {
    float* cp = static_cast<float*>(scratch);
    hipLaunchKernelGGL(thomas_kernel<float>, grid, block, 0, s, static_cast<const float*>(a),
                       static_cast<const float*>(b), static_cast<const float*>(c), static_cast<const float*>(d),
                       static_cast<float*>(x), cp, cp + (int64_t)batch * n, n);
  }
  return hipGetLastError();
}

// Shared checks of the stage entry points.  Grid sizes: batch * groups workgroups must fit a
// 32-bit grid dimension.
int check_stage(int dtype, int32_t batch, int64_t N, int32_t m) {
  if (elem_bytes(dtype) == 0) return WF_E_ARG;
  if (batch < 1 || N < 2 || m < 2) return WF_E_ARG;
  if (m > max_m(dtype)) return WF_E_UNSUPPORTED;
  if (N > INT64_MAX / batch / 2) return WF_E_ARG;
  const StageArgs g = stage_args(dtype, N, m, 32);
  if (g.groups > (int64_t)0x7fffffff / batch) return WF_E_UNSUPPORTED;
  return WF_OK;
}

}  // namespace
}  // namespace tri

// ---------------------------------------------------------------------------------------
// Plans and the predictor.

struct tri_plan {
  int dtype = 0;
  int32_t batch = 0;
  int64_t N = 0;
  int32_t R = 0;                             // recursive steps; -1 = direct solve (N = 1)
  int32_t m[TRI_MAX_R + 1] = {};             // m, m_1 .. m_R
  int64_t n[TRI_MAX_R + 2] = {};             // n[0] = N, n[l+1] = 2 P(n[l], m[l])
  void* lv[TRI_MAX_R + 2][5] = {};           // level l >= 1: A, B, C, D, X (batch * n[l] each)
  void* scratch = nullptr;                   // Thomas cp, dp of the deepest system
};

namespace tri {
namespace {

// Training set of the nearest-neighbour rule: for each of the paper's 37 system sizes N (its
// Table I), the fastest sub-system size m and recursion depth R of the device solver on one
// MI355X, in float64 and in float32, timed by python -m paper_2510_27351_amd.tri_sweep
// (m in {4, 8, 16, 20, 32, 40, 64, 128}, R in 0..4; best of 3 rounds of 10 solves).  A copy
// is in tests/golden/mi355x_tri_table.txt.
struct SizeObs {
  int64_t N;
  int32_t m64, R64, m32, R32;
};
const SizeObs kSizeTable[] = {
    {100, 16, 0, 20, 0},
    {200, 16, 0, 16, 0},
    {400, 20, 0, 20, 0},
    {500, 8, 1, 8, 1},
    {800, 16, 1, 16, 1},
    {1000, 16, 1, 16, 1},
    {2000, 16, 1, 16, 1},
    {4000, 20, 1, 16, 2},
    {4500, 16, 2, 16, 2},
    {5000, 16, 2, 16, 2},
    {8000, 16, 2, 16, 2},
    {10000, 16, 2, 16, 2},
    {20000, 20, 2, 20, 2},
    {25000, 20, 2, 16, 3},
    {30000, 16, 3, 8, 4},
    {40000, 16, 3, 16, 3},
    {50000, 16, 3, 16, 3},
    {60000, 16, 3, 16, 3},
    {70000, 16, 3, 16, 3},
    {75000, 16, 3, 16, 3},
    {80000, 16, 3, 16, 3},
    {100000, 16, 3, 16, 3},
    {200000, 20, 3, 16, 4},
    {400000, 16, 4, 16, 4},
    {500000, 16, 4, 16, 4},
    {800000, 20, 4, 16, 4},
    {1000000, 20, 4, 16, 4},
    {2000000, 20, 4, 20, 4},
    {4000000, 20, 4, 20, 4},
    {5000000, 20, 4, 20, 4},
    {8000000, 20, 4, 32, 4},
    {10000000, 32, 4, 32, 4},
    {20000000, 32, 4, 32, 4},
    {40000000, 32, 4, 32, 4},
    {50000000, 32, 4, 32, 4},
    {80000000, 32, 4, 32, 4},
    {100000000, 32, 4, 32, 4},
};

// Nearest timed size (distance |log N - log N_i|, ties to the earlier row).
const SizeObs& nearest(int64_t N) {
  const int cnt = (int)(sizeof(kSizeTable) / sizeof(kSizeTable[0]));
  int best = 0;
  double bd = 1e300;
  for (int i = 0; i < cnt; ++i) {
    const double dd = std::fabs(std::log((double)N) - std::log((double)kSizeTable[i].N));
    if (dd < bd) {
      bd = dd;
      best = i;
    }
  }
  return kSizeTable[best];
}

int32_t predict_m(int dtype, int64_t N) {
  const SizeObs& o = nearest(N);
  return dtype == WF_F64 ? o.m64 : o.m32;
}

void level_sizes(int64_t N, int32_t R, const int32_t* ms, int64_t* n) {
  n[0] = N;
  for (int l = 0; l <= R; ++l) n[l + 1] = 2 * partition_count(n[l], ms[l]);
}

void free_plan(tri_plan* p) {
  for (auto& lv : p->lv)
    for (void*& q : lv)
      if (q) {
        (void)hipFree(q);
        q = nullptr;
      }
  if (p->scratch) (void)hipFree(p->scratch);
  p->scratch = nullptr;
}

}  // namespace
}  // namespace tri

using namespace tri;

extern "C" {

int64_t tri_subsystems(int64_t N, int32_t m) { return partition_count(N, m); }

int tri_stage1(int dtype, int32_t batch, int64_t N, int32_t m, const void* a, const void* b, const void* c,
               const void* d, void* A, void* B, void* C, void* D, void* stream) {
  int rc = check_stage(dtype, batch, N, m);
  if (rc != WF_OK) return rc;
  if (!a || !b || !c || !d || !A || !B || !C || !D) return WF_E_ARG;
  StageArgs g = stage_args(dtype, N, m, 32);
  g.a = a;
  g.b = b;
  g.c = c;
  g.d = d;
  g.A = A;
  g.B = B;
  g.C = C;
  g.D = D;
  return launch_stage1(dtype, batch, g, static_cast<hipStream_t>(stream)) == hipSuccess ? WF_OK : WF_E_DEVICE;
}

int tri_stage3(int dtype, int32_t batch, int64_t N, int32_t m, const void* a, const void* b, const void* c,
               const void* d, const void* z, void* x, void* stream) {
  int rc = check_stage(dtype, batch, N, m);
  if (rc != WF_OK) return rc;
  if (!a || !b || !c || !d || !z || !x) return WF_E_ARG;
  StageArgs g = stage_args(dtype, N, m, 64);
  if (g.groups > (int64_t)0x7fffffff / batch) return WF_E_UNSUPPORTED;
  g.a = a;
  g.b = b;
  g.c = c;
  g.d = d;
  g.z = z;
  g.x = x;
  return launch_stage3(dtype, batch, g, static_cast<hipStream_t>(stream)) == hipSuccess ? WF_OK : WF_E_DEVICE;
}

int tri_thomas(int dtype, int32_t batch, int64_t n, const void* a, const void* b, const void* c, const void* d,
               void* x, void* scratch, void* stream) {
  if (elem_bytes(dtype) == 0 || batch < 1 || n < 1) return WF_E_ARG;
  if (n > INT64_MAX / batch / 2) return WF_E_ARG;
  if (!a || !b || !c || !d || !x || !scratch) return WF_E_ARG;
  return launch_thomas(dtype, batch, n, a, b, c, d, x, scratch, static_cast<hipStream_t>(stream)) == hipSuccess
             ? WF_OK
             : WF_E_DEVICE;
}

int tri_predict(int dtype, int64_t N, int32_t* m, int32_t* R, int32_t* ms) {
  if (elem_bytes(dtype) == 0 || N < 1) return WF_E_ARG;
  const SizeObs& o = nearest(N);
  const int32_t mm = dtype == WF_F64 ? o.m64 : o.m32;
  int32_t rr = dtype == WF_F64 ? o.R64 : o.R32;
  if (rr > TRI_MAX_R) rr = TRI_MAX_R;
  if (m) *m = mm;
  if (R) *R = rr;
  if (ms) {
    // the paper's rule for the recursive steps: m_1 = the predicted m of the first
    // interface system when R = 1, else 10; m_l = the predicted m of the l-th interface
    // system's size
    int64_t nl = N >= 2 ? 2 * partition_count(N, mm) : 2;
    for (int l = 1; l <= rr; ++l) {
      int32_t ml = (l == 1 && rr > 1) ? 10 : predict_m(dtype, nl);
      ms[l - 1] = ml;
      nl = 2 * partition_count(nl, ml);
    }
  }
  return WF_OK;
}

int tri_plan_create(tri_plan** out, int dtype, int32_t batch, int64_t N, int32_t m, int32_t R, const int32_t* ms) {
  if (!out) return WF_E_ARG;
  *out = nullptr;
  const int es = elem_bytes(dtype);
  if (es == 0 || batch < 1 || N < 1) return WF_E_ARG;
  if (N > INT64_MAX / batch / 8) return WF_E_ARG;
  if (m < 0 || m == 1 || R < -1 || R > TRI_MAX_R) return WF_E_ARG;
  tri_plan* p = new (std::nothrow) tri_plan;
  if (!p) return WF_E_NOMEM;
  p->dtype = dtype;
  p->batch = batch;
  p->N = N;
  if (N == 1) {
    p->R = -1;
    p->n[0] = 1;
  } else {
    int32_t pm = 0, pR = 0;
    (void)tri_predict(dtype, N, &pm, &pR, nullptr);
    const int32_t mm = m ? m : pm;
    const int32_t rr = R >= 0 ? R : pR;
    int32_t rule[TRI_MAX_R] = {};
    if (!ms) {
      // the rule for the recursive steps, for this m and R
      int64_t nl = 2 * partition_count(N, mm);
      for (int l = 1; l <= rr; ++l) {
        rule[l - 1] = (l == 1 && rr > 1) ? 10 : predict_m(dtype, nl);
        nl = 2 * partition_count(nl, rule[l - 1]);
      }
      ms = rule;
    }
    p->R = rr;
    p->m[0] = mm;
    for (int l = 1; l <= rr; ++l) p->m[l] = ms[l - 1];
    for (int l = 0; l <= rr; ++l)
      if (p->m[l] < 2 || p->m[l] > max_m(dtype)) {
        const int bad = p->m[l] < 2 ? WF_E_ARG : WF_E_UNSUPPORTED;
        delete p;
        return bad;
      }
    level_sizes(N, rr, p->m, p->n);
    for (int l = 0; l <= rr; ++l) {
      const StageArgs g = stage_args(dtype, p->n[l], p->m[l], 32);
      if (g.groups > (int64_t)0x7fffffff / batch) {
        delete p;
        return WF_E_UNSUPPORTED;
      }
    }
    for (int l = 1; l <= rr + 1; ++l)
      for (int q = 0; q < 5; ++q)
        if (hipMalloc(&p->lv[l][q], (size_t)batch * p->n[l] * es) != hipSuccess) {
          p->lv[l][q] = nullptr;
          free_plan(p);
          delete p;
          return WF_E_NOMEM;
        }
  }
  const int64_t deep = p->R >= 0 ? p->n[p->R + 1] : 1;
  if (hipMalloc(&p->scratch, (size_t)2 * batch * deep * es) != hipSuccess) {
    p->scratch = nullptr;
    free_plan(p);
    delete p;
    return WF_E_NOMEM;
  }
  *out = p;
  return WF_OK;
}

int tri_plan_config(const tri_plan* p, int32_t* m, int32_t* R, int32_t* ms, int64_t* sizes) {
  if (!p) return WF_E_ARG;
  if (m) *m = p->R >= 0 ? p->m[0] : 0;
  if (R) *R = p->R;
  if (ms)
    for (int l = 1; l <= p->R; ++l) ms[l - 1] = p->m[l];
  if (sizes)
    for (int l = 0; l <= p->R + 1; ++l) sizes[l] = p->n[l];
  return WF_OK;
}

int tri_solve(const tri_plan* p, const void* a, const void* b, const void* c, const void* d, void* x,
              void* stream) {
  if (!p || !a || !b || !c || !d || !x) return WF_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int dt = p->dtype;
  if (p->R < 0) return launch_thomas(dt, p->batch, 1, a, b, c, d, x, p->scratch, s) == hipSuccess ? WF_OK : WF_E_DEVICE;
  // Stage 1 on every level from the top
  for (int l = 0; l <= p->R; ++l) {
    StageArgs g = stage_args(dt, p->n[l], p->m[l], 32);
    g.a = l == 0 ? a : p->lv[l][0];
    g.b = l == 0 ? b : p->lv[l][1];
    g.c = l == 0 ? c : p->lv[l][2];
    g.d = l == 0 ? d : p->lv[l][3];
    g.A = p->lv[l + 1][0];
    g.B = p->lv[l + 1][1];
    g.C = p->lv[l + 1][2];
    g.D = p->lv[l + 1][3];
    if (launch_stage1(dt, p->batch, g, s) != hipSuccess) return WF_E_DEVICE;
  }
  // Stage 2: the deepest interface system, directly
  const int deep = p->R + 1;
  void* const* L = p->lv[deep];
  if (launch_thomas(dt, p->batch, p->n[deep], L[0], L[1], L[2], L[3], L[4], p->scratch, s) != hipSuccess)
    return WF_E_DEVICE;
  // Stage 3 on every level from the bottom
  for (int l = p->R; l >= 0; --l) {
    StageArgs g = stage_args(dt, p->n[l], p->m[l], 64);
    g.a = l == 0 ? a : p->lv[l][0];
    g.b = l == 0 ? b : p->lv[l][1];
    g.c = l == 0 ? c : p->lv[l][2];
    g.d = l == 0 ? d : p->lv[l][3];
    g.z = p->lv[l + 1][4];
    g.x = l == 0 ? x : p->lv[l][4];
    if (launch_stage3(dt, p->batch, g, s) != hipSuccess) return WF_E_DEVICE;
  }
  return WF_OK;
}

int tri_plan_level(const tri_plan* p, int32_t level, void* A, void* B, void* C, void* D, void* stream) {
  if (!p || level < 1 || level > p->R + 1 || !A || !B || !C || !D) return WF_E_ARG;
  const size_t bytes = (size_t)p->batch * p->n[level] * elem_bytes(p->dtype);
  void* dst[4] = {A, B, C, D};
  for (int q = 0; q < 4; ++q)
    if (hipMemcpyAsync(dst[q], p->lv[level][q], bytes, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)) !=
        hipSuccess)
      return WF_E_DEVICE;
  return WF_OK;
}

void tri_plan_destroy(tri_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  free_plan(p);
  delete p;
}

}  // extern "C"
