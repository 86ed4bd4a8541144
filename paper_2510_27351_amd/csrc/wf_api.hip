// Host runtime and C ABI of libwf (declared in include/wf.h).
//
// Responsibilities: argument validation before any device work, the per-device workspace
// (self-resetting control block + tagged handoff words), tile choice, launch, and the
// asynchronous error channel.  No allocation happens on the hot path once the workspace
// has reached the size of the largest shape seen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/wf.h"
#include "wf_host.h"
#include "wf_internal.h"
#include "wf_path.h"
#include "wf_soft.h"

namespace wf {
namespace {

std::mutex g_mu;
// One workspace per (device, stream): sweeps on different streams of a device never share a
// control block, handoff words or selections.  Map nodes keep their addresses.
std::map<std::pair<int, hipStream_t>, DeviceWs> g_ws;
std::vector<uint32_t> g_fault;                   // per device: injected fault mode (tests)
std::vector<std::pair<int, Control*>> g_plan_ctl;  // control blocks owned by plans
int g_tile_override = 0;
// optional per-band trace buffer (one, for the device that enabled it)
uint64_t* g_trace = nullptr;
int64_t g_trace_bands = 0;
int g_trace_dev = -1;

uint32_t fault_of(int dev) { return dev < (int)g_fault.size() ? g_fault[dev] : 0u; }

// A zeroed control block with epoch 1 (tag 0 is what never-written handoff words carry).
// Caller holds g_mu.
int alloc_control(int dev, Control** out) {
  Control init;
  std::memset(&init, 0, sizeof(init));
  init.epoch = 1u;
  init.fault = fault_of(dev);
  Control* c = nullptr;
  if (hipMalloc(&c, sizeof(Control)) != hipSuccess) return WF_E_NOMEM;
  if (hipMemcpy(c, &init, sizeof(init), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(c);
    return WF_E_DEVICE;
  }
  *out = c;
  return WF_OK;
}

}  // namespace

int ensure_ws_on(int dev, hipStream_t s, size_t words, DeviceWs** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceWs& w = g_ws[{dev, s}];
  if (!w.ctl) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      return WF_E_DEVICE;
    w.num_cus = cus;
    const int rc = alloc_control(dev, &w.ctl);
    if (rc != WF_OK) {
      w.ctl = nullptr;
      return rc;
    }
  }
  if (words > w.bnd_words) {
    // Growing: the old buffer may still be read by queued work, so drain the device first.
    if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
    if (w.bnd) (void)hipFree(w.bnd);
    w.bnd = nullptr;
    w.bnd_words = 0;
    size_t bytes = words * sizeof(uint64_t);
    if (hipMalloc(&w.bnd, bytes) != hipSuccess) { w.bnd = nullptr; return WF_E_NOMEM; }
    // tag 0 never equals a launch epoch, so zeroed words read as "not yet written"
    if (hipMemset(w.bnd, 0, bytes) != hipSuccess) return WF_E_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
    w.bnd_words = words;
  }
  *out = &w;
  return WF_OK;
}

int ensure_ws(int dev, size_t words, DeviceWs** out) { return ensure_ws_on(dev, nullptr, words, out); }

int new_control(int dev, Control** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int rc = alloc_control(dev, out);
  if (rc == WF_OK) g_plan_ctl.emplace_back(dev, *out);
  return rc;
}

void free_control(Control* ctl) {
  if (!ctl) return;
  std::lock_guard<std::mutex> lk(g_mu);
  for (size_t i = 0; i < g_plan_ctl.size(); ++i)
    if (g_plan_ctl[i].second == ctl) {
      g_plan_ctl.erase(g_plan_ctl.begin() + (long)i);
      break;
    }
  (void)hipFree(ctl);
}

// Buffers of the path adjoint of one (device, stream): exits, captured labels, group maps.
struct PathWs {
  int32_t* exits = nullptr;
  size_t exits_words = 0;
  int32_t* caps = nullptr;
  size_t caps_words = 0;
  int32_t* F = nullptr;
  size_t F_words = 0;
};
std::map<std::pair<int, hipStream_t>, PathWs> g_path;

// Grows a device buffer to at least 'words' 32-bit words (drains the device before freeing
// the old one, which queued work may still read).  Caller holds g_mu.
int grow_words(int32_t** p, size_t* have, size_t words) {
  if (words <= *have) return WF_OK;
  if (*p) {
    if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
    (void)hipFree(*p);
  }
  *p = nullptr;
  *have = 0;
  if (hipMalloc(p, words * sizeof(int32_t)) != hipSuccess) {
    *p = nullptr;
    return WF_E_NOMEM;
  }
  *have = words;
  return WF_OK;
}

int ensure_path(int dev, hipStream_t s, size_t exits, size_t caps, size_t F, PathWs** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  PathWs& w = g_path[{dev, s}];
  int rc = grow_words(&w.exits, &w.exits_words, exits);
  if (rc == WF_OK) rc = grow_words(&w.caps, &w.caps_words, caps);
  if (rc == WF_OK) rc = grow_words(&w.F, &w.F_words, F > 0 ? F : 1);
  *out = &w;
  return rc;
}

// Grows the adjoint's selection buffer of a workspace that ensure_ws has set up.
int ensure_sel(DeviceWs* w, size_t words) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (words <= w->sel_words) return WF_OK;
  if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
  if (w->sel) (void)hipFree(w->sel);
  w->sel = nullptr;
  w->sel_words = 0;
  if (hipMalloc(&w->sel, words * sizeof(uint32_t)) != hipSuccess) { w->sel = nullptr; return WF_E_NOMEM; }
  w->sel_words = words;
  return WF_OK;
}

int elem_size(int dtype) {
  switch (dtype) {
    case WF_F32: return 4;
    case WF_F64: return 8;
    case WF_I32: return 4;
    default: return 0;
  }
}

int words_per_elem(int dtype) { return dtype == WF_F64 ? 2 : 1; }

namespace {

// Tile of the single-instance sweeps for a shape: the caller's override (wf_set_tile, then
// WF_TILE), else the nearest-neighbour prediction from the tiles measured on MI355X.
int choose_tile(int dtype, int64_t m, int64_t n, bool reverse) {
  if (g_tile_override) return g_tile_override;
  if (const char* s = std::getenv("WF_TILE")) {
    int t = std::atoi(s);
    if (t == 16 || t == 32 || t == 64) return t;
  }
  // the callers have validated dtype, m and n, so this is a tile, never an error code
  return wf_tile_predict(dtype, m, n, reverse ? 1 : 0);
}

int64_t nbands(int64_t m) { return (m + kBand - 1) / kBand; }

}  // namespace

int pick_tile(int dtype, int64_t m, int64_t n, bool reverse) { return choose_tile(dtype, m, n, reverse); }

// ---------------------------------------------------------------------------------------
// Scratch of the allocation-free forward sweep (wf_forward_noalloc): a file-scope device
// array, one copy per GPU, held until the process ends.  Bytes [0, 256) are the launch
// control block; the tagged handoff words follow.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol): each device's address
// comes from hipGetSymbolAddress, taken once per device with that device current.
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;  // 32 MiB
constexpr size_t kScratchCtl = 256;                  // control block, then handoff words
constexpr size_t kScratchWords = (kScratchBytes - kScratchCtl) / sizeof(uint64_t);

__device__ __align__(256) uint64_t scratch[kScratchBytes / sizeof(uint64_t)];

struct ScratchDev {
  bool ready = false;
  char* ptr = nullptr;  // this device's copy of 'scratch'
  int num_cus = 0;
};
std::vector<ScratchDev> g_scratch;  // per device, guarded by g_mu

// The current device's scratch: address and CU count, looked up on the first call on it.
int scratch_of(int dev, ScratchDev* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1);
  ScratchDev& sd = g_scratch[dev];
  if (!sd.ready) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return WF_E_DEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      return WF_E_DEVICE;
    // an injected fault mode (tests only) applies to the array's control block as well
    const uint32_t f = fault_of(dev);
    if (f && hipMemcpy(&reinterpret_cast<Control*>(p)->fault, &f, sizeof(f), hipMemcpyHostToDevice) != hipSuccess)
      return WF_E_DEVICE;
    sd.ptr = static_cast<char*>(p);
    sd.num_cus = cus;
    sd.ready = true;
  }
  *out = sd;
  return WF_OK;
}

// The control block starts zeroed with the array; a launch needs a non-zero epoch (tag 0 is
// what never-written handoff words carry).  Enqueued before every sweep, so that the order
// of calls, eager or captured in a graph, never matters; later launches advance the epoch
// themselves.
__global__ void scratch_prepare(Control* ctl) {
  if (threadIdx.x == 0 && __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
    __hip_atomic_store(&ctl->epoch, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

}  // namespace wf

using namespace wf;

extern "C" {

int wf_version(void) { return 100; }

const char* wf_error_string(int code) {
  switch (code) {
    case WF_OK: return "ok";
    case WF_E_ARG: return "invalid argument";
    case WF_E_UNSUPPORTED: return "unsupported configuration";
    case WF_E_NOMEM: return "device allocation failed";
    case WF_E_DEVICE: return "HIP runtime error";
    case WF_E_TIMEOUT: return "device-side wait timed out";
    default: return "unknown error";
  }
}

// The fastest tile G of the forward sweep (table, score, checkpoint grid K = 64) and of the
// reverse sweep (timed behind the selection recompute, where it always runs) on MI355X for
// the 7 x 7 grid of shapes with m and n each a power of two from 256 to 16384, in float32 and
// in float64 (python -m paper_2510_27351_amd.tile_sweep [--dtype f64]: best of 3 rounds of
// 10 calls per tile).  The training set of the
// nearest-neighbour rule below; the two element types get a column pair each, since the
// float32 choices lose up to 18% when reused for float64.
struct TileObs {
  int64_t m, n;
  int32_t fwd32, rev32, fwd64, rev64;
};
static const TileObs kTileTable[] = {
    {256, 256, 64, 32, 32, 16},    {256, 512, 64, 64, 64, 64},    {256, 1024, 64, 64, 64, 64},   {256, 2048, 64, 64, 64, 64},
    {256, 4096, 64, 64, 64, 64},   {256, 8192, 64, 64, 64, 64},   {256, 16384, 64, 64, 64, 64},  {512, 256, 32, 32, 32, 16},
    {512, 512, 64, 32, 32, 16},    {512, 1024, 64, 64, 64, 64},   {512, 2048, 64, 64, 64, 64},   {512, 4096, 64, 64, 64, 64},
    {512, 8192, 64, 64, 64, 64},   {512, 16384, 64, 64, 64, 64},  {1024, 256, 32, 32, 32, 16},   {1024, 512, 64, 32, 32, 16},
    {1024, 1024, 64, 32, 64, 16},  {1024, 2048, 64, 64, 64, 64},  {1024, 4096, 64, 64, 64, 64},  {1024, 8192, 64, 64, 64, 64},
    {1024, 16384, 64, 64, 64, 64}, {2048, 256, 32, 32, 32, 16},   {2048, 512, 32, 32, 32, 16},   {2048, 1024, 64, 32, 32, 16},
    {2048, 2048, 64, 32, 64, 64},  {2048, 4096, 64, 32, 64, 64},  {2048, 8192, 64, 64, 32, 64},  {2048, 16384, 64, 64, 64, 64},
    {4096, 256, 32, 32, 32, 16},   {4096, 512, 32, 32, 32, 16},   {4096, 1024, 32, 32, 32, 16},  {4096, 2048, 64, 32, 32, 16},
    {4096, 4096, 64, 32, 32, 64},  {4096, 8192, 64, 32, 64, 64},  {4096, 16384, 64, 64, 64, 64}, {8192, 256, 32, 32, 32, 16},
    {8192, 512, 32, 32, 32, 16},   {8192, 1024, 32, 32, 32, 16},  {8192, 2048, 32, 32, 32, 16},  {8192, 4096, 64, 32, 32, 64},
    {8192, 8192, 64, 32, 64, 64},  {8192, 16384, 64, 64, 64, 64}, {16384, 256, 32, 32, 32, 16},  {16384, 512, 32, 32, 32, 16},
    {16384, 1024, 32, 32, 32, 16}, {16384, 2048, 32, 32, 32, 16}, {16384, 4096, 64, 32, 32, 16}, {16384, 8192, 64, 32, 64, 16},
    {16384, 16384, 64, 32, 64, 64},
};

int32_t wf_tile_predict(int32_t dtype, int64_t m, int64_t n, int32_t reverse) {
  if (dtype != WF_F32 && dtype != WF_F64 && dtype != WF_I32) return WF_E_ARG;
  if (m < 1 || n < 1 || (reverse != 0 && reverse != 1)) return WF_E_ARG;
  if (dtype == WF_I32 && reverse) return WF_E_UNSUPPORTED;
  const double lm = std::log2((double)m), ln = std::log2((double)n);
  int best = 0;
  double best_d = INFINITY;
  for (int i = 0; i < (int)(sizeof(kTileTable) / sizeof(kTileTable[0])); ++i) {
    const double dm = lm - std::log2((double)kTileTable[i].m), dn = ln - std::log2((double)kTileTable[i].n);
    const double d = dm * dm + dn * dn;
    if (d < best_d) {  // strictly nearer: ties go to the earlier row
      best = i;
      best_d = d;
    }
  }
  const TileObs& o = kTileTable[best];
  if (dtype == WF_F64) return reverse ? o.rev64 : o.fwd64;
  return reverse ? o.rev32 : o.fwd32;  // int32 has float32's element size and no reverse sweep
}

int64_t wf_ckpt_elems(int64_t m, int64_t n, int32_t ckpt_k) {
  if (m < 1 || n < 1 || ckpt_k < 0 || ckpt_k > 4096) return -1;
  if (ckpt_k == 0) return 0;
  const int64_t rows = nbands(m) - 1;
  const int64_t cols = (n + ckpt_k - 1) / ckpt_k - 1;
  return rows * n + cols * m;
}

int wf_set_tile(int32_t tile) {
  if (tile != 0 && tile != 16 && tile != 32 && tile != 64) return WF_E_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  g_tile_override = tile;
  return WF_OK;
}

int wf_forward(int dtype, int64_t m, int64_t n, const void* C, int64_t ldc, void* D, int64_t ldd,
               void* score, void* ckpt, int32_t ckpt_k, void* stream) {
  const int es = elem_size(dtype);
  if (es == 0) return WF_E_ARG;
  if (m < 1 || n < 1 || n > (int64_t)1 << 31 || m > (int64_t)1 << 40) return WF_E_ARG;
  if (m > INT64_MAX / n) return WF_E_ARG;
  if (!C || !score || ldc < n) return WF_E_ARG;
  if (D && ldd < n) return WF_E_ARG;
  if (ckpt_k < 0 || ckpt_k > 4096) return WF_E_ARG;
  if (ckpt_k == 0 && ckpt != nullptr) return WF_E_ARG;
  if (ckpt_k > 0 && ckpt == nullptr && wf_ckpt_elems(m, n, ckpt_k) > 0) return WF_E_ARG;
  if ((m - 1) > INT64_MAX / ldc) return WF_E_ARG;
  // a band of 64 rows is addressed with 32-bit byte offsets
  if (ldc > kMaxLd / es || (D && ldd > kMaxLd / es)) return WF_E_UNSUPPORTED;
  const int64_t band_rows = forward_band_rows(dtype);
  const int64_t nb = (m + band_rows - 1) / band_rows;
  if (nb > 0x7fffffff) return WF_E_ARG;

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  const size_t words = (size_t)(nb > 1 ? nb - 1 : 1) * (size_t)n * words_per_elem(dtype);
  DeviceWs* ws = nullptr;
  int rc = ensure_ws_on(dev, static_cast<hipStream_t>(stream), words, &ws);
  if (rc != WF_OK) return rc;

  FwdArgs a;
  a.C = C;
  a.D = D;
  a.score = score;
  a.ckpt = ckpt;
  a.ldc = ldc;
  a.ldd = D ? ldd : n;
  a.m = m;
  a.n = n;
  a.ckpt_k = ckpt_k;
  a.nb = (int32_t)nb;
  a.ctl = ws->ctl;
  a.bnd = ws->bnd;
  a.trace = (g_trace && dev == g_trace_dev && nb <= g_trace_bands) ? g_trace : nullptr;
  a.kx = a.gl = 1.0;
  const int grid = (int)std::min<int64_t>(nb, ws->num_cus);
  const int tile = choose_tile(dtype, m, n, false);
  hipError_t e = launch_forward(dtype, tile, a, grid, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? WF_OK : WF_E_DEVICE;
}

int wf_forward_noalloc(int dtype, int64_t m, int64_t n, const void* C, int64_t ldc, void* D, int64_t ldd,
                       void* score, void* ckpt, int32_t ckpt_k, void* stream) {
  const int es = elem_size(dtype);
  if (es == 0) return WF_E_ARG;
  if (m < 1 || n < 1 || n > (int64_t)1 << 31 || m > (int64_t)1 << 40) return WF_E_ARG;
  if (m > INT64_MAX / n) return WF_E_ARG;
  if (!C || !score || ldc < n) return WF_E_ARG;
  if (D && ldd < n) return WF_E_ARG;
  if (ckpt_k < 0 || ckpt_k > 4096) return WF_E_ARG;
  if (ckpt_k == 0 && ckpt != nullptr) return WF_E_ARG;
  if (ckpt_k > 0 && ckpt == nullptr && wf_ckpt_elems(m, n, ckpt_k) > 0) return WF_E_ARG;
  if ((m - 1) > INT64_MAX / ldc) return WF_E_ARG;
  if (ldc > kMaxLd / es || (D && ldd > kMaxLd / es)) return WF_E_UNSUPPORTED;
  const int64_t band_rows = forward_band_rows(dtype);
  const int64_t nb = (m + band_rows - 1) / band_rows;
  if (nb > 0x7fffffff) return WF_E_ARG;
  // the handoff words of every band boundary must fit in the scratch array
  const int64_t words = (nb - 1) * words_per_elem(dtype);
  if (words > 0 && n > (int64_t)kScratchWords / words) return WF_E_UNSUPPORTED;

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  ScratchDev sd;
  int rc = scratch_of(dev, &sd);
  if (rc != WF_OK) return rc;
  Control* ctl = reinterpret_cast<Control*>(sd.ptr);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(scratch_prepare, dim3(1), dim3(64), 0, st, ctl);
  if (hipGetLastError() != hipSuccess) return WF_E_DEVICE;

  FwdArgs a;
  a.C = C;
  a.D = D;
  a.score = score;
  a.ckpt = ckpt;
  a.ldc = ldc;
  a.ldd = D ? ldd : n;
  a.m = m;
  a.n = n;
  a.ckpt_k = ckpt_k;
  a.nb = (int32_t)nb;
  a.ctl = ctl;
  a.bnd = reinterpret_cast<uint64_t*>(sd.ptr + kScratchCtl);
  a.trace = nullptr;
  a.kx = a.gl = 1.0;
  const int grid = (int)std::min<int64_t>(nb, sd.num_cus);
  hipError_t e = launch_forward(dtype, choose_tile(dtype, m, n, false), a, grid, st);
  return e == hipSuccess ? WF_OK : WF_E_DEVICE;
}

}  // extern "C"

namespace {

// Checks the arguments of a selection recompute, sets up the stream's workspace and fills
// the launch's arguments and grid (wf_select and the path adjoint).
int prepare_select(int dtype, int64_t m, int64_t n, const void* C, int64_t ldc, const void* ckpt, int32_t ckpt_k,
                   const void* D, int64_t ldd, void* stream, DeviceWs** out, SelArgs* sel_args, int* grid_out) {
  if (dtype != WF_F32 && dtype != WF_F64) return dtype == WF_I32 ? WF_E_UNSUPPORTED : WF_E_ARG;
  const int es = elem_size(dtype);
  if (m < 1 || n < 1 || n > (int64_t)1 << 31 || m > (int64_t)1 << 40) return WF_E_ARG;
  if (m > INT64_MAX / n) return WF_E_ARG;
  if (!C || ldc < n) return WF_E_ARG;
  // exactly one source of the band top rows: the checkpoint grid (ckpt_k > 0) or the table
  if (ckpt_k < 0 || ckpt_k > 4096) return WF_E_ARG;
  if (ckpt_k > 0) {
    if (D != nullptr) return WF_E_ARG;
    if (ckpt == nullptr && wf_ckpt_elems(m, n, ckpt_k) > 0) return WF_E_ARG;
  } else {
    if (D == nullptr || ckpt != nullptr || ldd < n) return WF_E_ARG;
  }
  if (ldc > kMaxLd / es) return WF_E_UNSUPPORTED;
  const int64_t nb = nbands(m);
  if (nb > 0x7fffffff) return WF_E_ARG;
  const int64_t Ks = (n + kBand - 1 + 63) / 64;
  if (Ks > 0x7fffffff / 64) return WF_E_ARG;

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  const size_t words = (size_t)(nb > 1 ? nb - 1 : 1) * (size_t)n * 2 * words_per_elem(dtype);
  DeviceWs* ws = nullptr;
  int rc = ensure_ws_on(dev, static_cast<hipStream_t>(stream), words, &ws);
  if (rc != WF_OK) return rc;
  rc = ensure_sel(ws, (size_t)nb * (size_t)Ks * 64 * 8);
  if (rc != WF_OK) return rc;

  SelArgs sa;
  sa.C = C;
  sa.ldc = ldc;
  if (ckpt_k > 0) {  // band rows of the checkpoint grid: row 64b+63 is ckpt row b
    sa.top = ckpt;
    sa.ld_top = n;
  } else {     // rows 64b+63 of the saved table
    sa.top = static_cast<const char*>(D) + (size_t)63 * ldd * es;
    sa.ld_top = 64 * ldd;
  }
  // With fewer bands than the CUs' workgroup slots (two per CU: a workgroup's ring takes
  // half of the LDS), each band is swept as up to four column pieces, each but the first
  // starting from a column of the forward table that the source holds: a block column of the
  // checkpoint grid (a multiple of K) or any column of the saved table.  The pieces are w
  // columns wide (a multiple of lcm(K, 64)), the last one the rest, every piece at least 256
  // columns.
  const int64_t per_cu = 2;
  sa.split = 0;
  sa.left = nullptr;
  sa.ld_left = 0;
  sa.left_pstride = 0;
  sa.pieces = 1;
  sa.pad = 0;
  {
    const int64_t K = ckpt_k > 0 ? ckpt_k : 64;
    const int64_t L = K / std::gcd<int64_t>(K, 64) * 64;  // lcm(K, 64)
    for (int64_t P = std::min<int64_t>(kMaxPieces, per_cu * ws->num_cus / nb); P >= 2; --P) {
      const int64_t w = (n / P + L / 2) / L * L;
      if (w < 256 || n - (P - 1) * w < 256) continue;
      sa.split = w;
      sa.pieces = (int32_t)P;
      if (ckpt_k > 0) {  // block column q = w/K holds D[.][w-1]
        sa.left = static_cast<const char*>(ckpt) + ((size_t)(nb - 1) * n + (size_t)(w / K - 1) * m) * es;
        sa.ld_left = 1;
        sa.left_pstride = (w / K) * m;
      } else {
        sa.left = static_cast<const char*>(D) + (size_t)(w - 1) * es;
        sa.ld_left = ldd;
        sa.left_pstride = w;
      }
      break;
    }
  }
  const int64_t items = nb * sa.pieces;
  const int grid = (int)std::min<int64_t>(items, per_cu * (int64_t)ws->num_cus);
  sa.m = m;
  sa.n = n;
  sa.nb = (int32_t)nb;
  sa.sel = ws->sel;
  sa.ctl = ws->ctl;
  *out = ws;
  *sel_args = sa;
  *grid_out = grid;
  return WF_OK;
}

// Records that the stream's workspace now holds the selections of this shape and type.
void note_selections(DeviceWs* ws, int dtype, int64_t m, int64_t n) {
  std::lock_guard<std::mutex> lk(g_mu);
  ws->sel_dtype = dtype;
  ws->sel_m = m;
  ws->sel_n = n;
}

}  // namespace

extern "C" {

int wf_select(int dtype, int64_t m, int64_t n, const void* C, int64_t ldc, const void* ckpt, int32_t ckpt_k,
              const void* D, int64_t ldd, void* stream) {
  DeviceWs* ws = nullptr;
  SelArgs sa;
  int grid = 0;
  const int rc = prepare_select(dtype, m, n, C, ldc, ckpt, ckpt_k, D, ldd, stream, &ws, &sa, &grid);
  if (rc != WF_OK) return rc;
  if (launch_select(dtype, sa, grid, static_cast<hipStream_t>(stream)) != hipSuccess) return WF_E_DEVICE;
  note_selections(ws, dtype, m, n);
  return WF_OK;
}

int wf_reverse(int dtype, int64_t m, int64_t n, const void* g_score, const void* g_D, int64_t ldgd, void* g_C,
               int64_t ldgc, void* stream) {
  if (dtype != WF_F32 && dtype != WF_F64) return dtype == WF_I32 ? WF_E_UNSUPPORTED : WF_E_ARG;
  const int es = elem_size(dtype);
  if (m < 1 || n < 1 || n > (int64_t)1 << 31 || m > (int64_t)1 << 40) return WF_E_ARG;
  if (m > INT64_MAX / n) return WF_E_ARG;
  if (!g_C || ldgc < n) return WF_E_ARG;
  if (g_D && ldgd < n) return WF_E_ARG;
  if (ldgc > kMaxLd / es || (g_D && ldgd > kMaxLd / es)) return WF_E_UNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  DeviceWs* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find({dev, static_cast<hipStream_t>(stream)});
    if (it == g_ws.end()) return WF_E_ARG;
    ws = &it->second;
    // the selections in this stream's workspace must be those of this shape and type
    if (ws->sel_dtype != dtype || ws->sel_m != m || ws->sel_n != n) return WF_E_ARG;
  }
  const int64_t nb = nbands(m);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int grid = (int)std::min<int64_t>(nb, ws->num_cus);
  AdjArgs aa;
  aa.sel = ws->sel;
  aa.gD = g_D;
  aa.gscore = g_score;
  aa.gC = g_C;
  aa.ldgd = g_D ? ldgd : n;
  aa.ldgc = ldgc;
  aa.m = m;
  aa.n = n;
  aa.nb = (int32_t)nb;
  aa.ctl = ws->ctl;
  aa.bnd = ws->bnd;
  aa.trace = (g_trace && dev == g_trace_dev && nb <= g_trace_bands) ? g_trace : nullptr;
  hipError_t e = launch_adjoint(dtype, choose_tile(dtype, m, n, true), aa, grid, st);
  return e == hipSuccess ? WF_OK : WF_E_DEVICE;
}

int wf_backward(int dtype, int64_t m, int64_t n, const void* C, int64_t ldc, const void* ckpt, int32_t ckpt_k,
                const void* D, int64_t ldd, const void* g_score, const void* g_D, int64_t ldgd, void* g_C,
                int64_t ldgc, void* stream) {
  if (dtype != WF_F32 && dtype != WF_F64) return dtype == WF_I32 ? WF_E_UNSUPPORTED : WF_E_ARG;
  const int es = elem_size(dtype);
  // the arguments of both halves are checked before either enqueues work
  if (m < 1 || n < 1 || n > (int64_t)1 << 31 || m > (int64_t)1 << 40) return WF_E_ARG;
  if (m > INT64_MAX / n) return WF_E_ARG;
  if (!C || ldc < n || !g_C || ldgc < n) return WF_E_ARG;
  if (g_D && ldgd < n) return WF_E_ARG;
  if (ckpt_k < 0 || ckpt_k > 4096) return WF_E_ARG;
  if (ckpt_k > 0 ? (D != nullptr || (ckpt == nullptr && wf_ckpt_elems(m, n, ckpt_k) > 0))
                 : (D == nullptr || ckpt != nullptr || ldd < n))
    return WF_E_ARG;
  if (ldc > kMaxLd / es || ldgc > kMaxLd / es || (g_D && ldgd > kMaxLd / es)) return WF_E_UNSUPPORTED;
  if (g_D) {
    const int rc = wf_select(dtype, m, n, C, ldc, ckpt, ckpt_k, D, ldd, stream);
    if (rc != WF_OK) return rc;
    return wf_reverse(dtype, m, n, g_score, g_D, ldgd, g_C, ldgc, stream);
  }
  // The score alone: its upstream value on the argmin path, zero elsewhere.
  DeviceWs* ws = nullptr;
  SelArgs sa;
  int grid = 0;
  int rc = prepare_select(dtype, m, n, C, ldc, ckpt, ckpt_k, D, ldd, stream, &ws, &sa, &grid);
  if (rc != WF_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nb = sa.nb;
  const int32_t S = path_group_size(nb);
  const int32_t G = nb > 1 ? (nb - 1 + S - 1) / S : 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  PathWs* pw = nullptr;
  rc = ensure_path(dev, st, (size_t)nb * (size_t)n, (size_t)nb * kMaxPieces * 64, (size_t)G * (size_t)n, &pw);
  if (rc != WF_OK) return rc;
  // The gradient is zeroed by the sweep itself for float32 (its zero stores cost the sweep
  // less than a pass of their own) and by a pass of its own before it for float64 (twice the
  // bytes: the fused stores slowed the sweep by more than the pass takes).
  const bool fused = dtype == WF_F32;
  if (!fused && launch_zero(dtype, g_C, m, n, ldgc, 8 * ws->num_cus, st) != hipSuccess) return WF_E_DEVICE;
  if (launch_select_path(dtype, sa, PathLabels{pw->exits, pw->caps, fused ? g_C : nullptr, ldgc}, grid, st) !=
      hipSuccess)
    return WF_E_DEVICE;
  note_selections(ws, dtype, m, n);
  PathArgs pa;
  pa.exits = pw->exits;
  pa.caps = pw->caps;
  pa.F = pw->F;
  pa.sel = ws->sel;
  pa.gscore = g_score;
  pa.gC = g_C;
  pa.ldgc = ldgc;
  pa.m = m;
  pa.n = n;
  pa.split = sa.split;
  pa.pieces = sa.pieces;
  pa.pad = 0;
  pa.nb = nb;
  pa.Ks = (int32_t)((n + kBand - 1 + 63) / 64);
  pa.S = S;
  pa.G = G;
  return launch_path(dtype, pa, st) == hipSuccess ? WF_OK : WF_E_DEVICE;
}

namespace {

// Checks shared by the two smooth sweeps; fills the sizes of the launch.
int soft_check(int dtype, int64_t m, int64_t n, double gamma, int64_t* nb) {
  if (dtype != WF_F32 && dtype != WF_F64) return dtype == WF_I32 ? WF_E_UNSUPPORTED : WF_E_ARG;
  if (m < 1 || n < 1 || n > (int64_t)1 << 31 || m > (int64_t)1 << 40) return WF_E_ARG;
  if (m > INT64_MAX / n) return WF_E_ARG;
  if (!(gamma > 0.0) || !std::isfinite(gamma)) return WF_E_ARG;
  *nb = nbands(m);
  if (*nb > 0x7fffffff) return WF_E_ARG;
  return WF_OK;
}

}  // namespace

int wf_soft_forward(int dtype, int64_t m, int64_t n, double gamma, const void* C, int64_t ldc, void* D, int64_t ldd,
                    void* score, void* stream) {
  int64_t nb = 0;
  int rc = soft_check(dtype, m, n, gamma, &nb);
  if (rc != WF_OK) return rc;
  const int es = elem_size(dtype);
  if (!C || !D || !score || ldc < n || ldd < n) return WF_E_ARG;
  if (ldc > kMaxLd / es || ldd > kMaxLd / es) return WF_E_UNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  DeviceWs* ws = nullptr;
  rc = ensure_ws_on(dev, static_cast<hipStream_t>(stream), (size_t)(nb > 1 ? nb - 1 : 1) * (size_t)n * words_per_elem(dtype),
                    &ws);
  if (rc != WF_OK) return rc;
  // the min-plus forward's band pipeline with the soft-min cell (64-row bands)
  FwdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.C = C;
  a.D = D;
  a.score = score;
  a.ckpt = nullptr;
  a.ldc = ldc;
  a.ldd = ldd;
  a.m = m;
  a.n = n;
  a.ckpt_k = 0;
  a.nb = (int32_t)nb;
  a.ctl = ws->ctl;
  a.bnd = ws->bnd;
  a.trace = nullptr;
  a.kx = 1.0 / (gamma * std::log(2.0));
  a.gl = gamma * std::log(2.0);
  const int grid = (int)std::min<int64_t>(nb, ws->num_cus);
  return launch_forward_soft(dtype, a, grid, static_cast<hipStream_t>(stream)) == hipSuccess ? WF_OK : WF_E_DEVICE;
}

int wf_soft_backward(int dtype, int64_t m, int64_t n, double gamma, const void* C, int64_t ldc, const void* D,
                     int64_t ldd, const void* g_score, const void* g_D, int64_t ldgd, void* g_C, int64_t ldgc,
                     void* stream) {
  int64_t nb = 0;
  int rc = soft_check(dtype, m, n, gamma, &nb);
  if (rc != WF_OK) return rc;
  const int es = elem_size(dtype);
  if (!C || !D || !g_C || ldc < n || ldd < n || ldgc < n) return WF_E_ARG;
  if (g_D && ldgd < n) return WF_E_ARG;
  if (ldc > kMaxLd / es || ldd > kMaxLd / es || ldgc > kMaxLd / es || (g_D && ldgd > kMaxLd / es))
    return WF_E_UNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  DeviceWs* ws = nullptr;
  rc = ensure_ws_on(dev, static_cast<hipStream_t>(stream),
                    (size_t)(nb > 1 ? nb - 1 : 1) * (size_t)n * 3 * words_per_elem(dtype), &ws);
  if (rc != WF_OK) return rc;
  SoftArgs a;
  std::memset(&a, 0, sizeof(a));
  a.C = C;
  a.Din = D;
  a.gD = g_D;
  a.gscore = g_score;
  a.gC = g_C;
  a.ldc = ldc;
  a.ldd = ldd;
  a.ldgd = g_D ? ldgd : n;
  a.ldgc = ldgc;
  a.m = m;
  a.n = n;
  a.nb = (int32_t)nb;
  a.kx = 1.0 / (gamma * std::log(2.0));
  a.ctl = ws->ctl;
  a.bnd = ws->bnd;
  const int grid = (int)std::min<int64_t>(nb, 4 * (int64_t)ws->num_cus);
  return launch_soft_backward(dtype, a, grid, static_cast<hipStream_t>(stream)) == hipSuccess ? WF_OK : WF_E_DEVICE;
}

int wf_trace_enable(int64_t max_bands) {
  if (max_bands < 0 || max_bands > ((int64_t)1 << 32)) return WF_E_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_trace) {
    if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
    (void)hipFree(g_trace);
    g_trace = nullptr;
    g_trace_bands = 0;
    g_trace_dev = -1;
  }
  if (max_bands == 0) return WF_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  const size_t bytes = (size_t)max_bands * kTraceWords * sizeof(uint64_t);
  if (hipMalloc(&g_trace, bytes) != hipSuccess) { g_trace = nullptr; return WF_E_NOMEM; }
  if (hipMemset(g_trace, 0, bytes) != hipSuccess) return WF_E_DEVICE;
  g_trace_bands = max_bands;
  g_trace_dev = dev;
  return WF_OK;
}

int64_t wf_trace_fetch(uint64_t* host, int64_t max_bands) {
  if (!host || max_bands < 0) return -WF_E_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_trace) return 0;
  const int64_t k = std::min(max_bands, g_trace_bands);
  if (hipDeviceSynchronize() != hipSuccess) return -WF_E_DEVICE;
  if (hipMemcpy(host, g_trace, (size_t)k * kTraceWords * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
    return -WF_E_DEVICE;
  return k;
}

int wf_fault_inject(int32_t mode) {
  if (mode < 0 || mode > (int32_t)kFaultRevWithhold) return WF_E_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  // queued sweeps keep the mode they were launched under
  if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_fault.size() <= dev) g_fault.resize(dev + 1, 0u);
  g_fault[dev] = (uint32_t)mode;
  const uint32_t v = (uint32_t)mode;
  for (auto& kv : g_ws)
    if (kv.first.first == dev && kv.second.ctl &&
        hipMemcpy(&kv.second.ctl->fault, &v, sizeof(v), hipMemcpyHostToDevice) != hipSuccess)
      return WF_E_DEVICE;
  for (auto& pc : g_plan_ctl)
    if (pc.first == dev && hipMemcpy(&pc.second->fault, &v, sizeof(v), hipMemcpyHostToDevice) != hipSuccess)
      return WF_E_DEVICE;
  if (dev < (int)g_scratch.size() && g_scratch[dev].ready &&
      hipMemcpy(&reinterpret_cast<Control*>(g_scratch[dev].ptr)->fault, &v, sizeof(v), hipMemcpyHostToDevice) !=
          hipSuccess)
    return WF_E_DEVICE;
  return WF_OK;
}

int wf_last_async_error(void* stream) {
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return WF_E_DEVICE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  // every control block of the device: the streams' workspaces, the plans', the scratch array's
  std::vector<Control*> ctls;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_ws)
      if (kv.first.first == dev && kv.second.ctl) ctls.push_back(kv.second.ctl);
    for (auto& pc : g_plan_ctl)
      if (pc.first == dev) ctls.push_back(pc.second);
    if (dev < (int)g_scratch.size() && g_scratch[dev].ready) ctls.push_back(reinterpret_cast<Control*>(g_scratch[dev].ptr));
  }
  uint32_t any = 0;
  for (Control* c : ctls) {
    uint32_t err = 0;
    if (hipMemcpy(&err, &c->err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return WF_E_DEVICE;
    if (err == 0) continue;
    any |= err;
    const uint32_t zero = 0;
    if (hipMemcpy(&c->err, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) return WF_E_DEVICE;
  }
  return any ? WF_E_TIMEOUT : WF_OK;
}

}  // extern "C"
