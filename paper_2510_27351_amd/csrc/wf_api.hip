// Host runtime and C ABI of libwf (declared in include/wf.h).
//
// Responsibilities: argument validation before any device work, the per-device workspace
// (self-resetting control block + tagged handoff words), tile choice, launch, and the
// asynchronous error channel.  No allocation happens on the hot path once the workspace
// has reached the size of the largest shape seen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/wf.h"
#include "wf_internal.h"

namespace wf {
namespace {

struct DeviceWs {
  Control* ctl = nullptr;     // device control block (zeroed, epoch = 1)
  uint64_t* bnd = nullptr;    // tagged handoff words
  size_t bnd_words = 0;
  int num_cus = 0;
};

std::mutex g_mu;
std::vector<DeviceWs> g_ws;
int g_tile_override = 0;

int ensure_ws(int dev, size_t words, DeviceWs** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
  DeviceWs& w = g_ws[dev];
  if (!w.ctl) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return WF_E_DEVICE;
    w.num_cus = prop.multiProcessorCount;
    Control init;
    std::memset(&init, 0, sizeof(init));
    init.epoch = 1u;
    if (hipMalloc(&w.ctl, sizeof(Control)) != hipSuccess) { w.ctl = nullptr; return WF_E_NOMEM; }
    if (hipMemcpy(w.ctl, &init, sizeof(init), hipMemcpyHostToDevice) != hipSuccess) return WF_E_DEVICE;
  }
  if (words > w.bnd_words) {
    // Growing: the old buffer may still be read by queued work, so drain the device first.
    if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
    if (w.bnd) hipFree(w.bnd);
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

int elem_size(int dtype) {
  switch (dtype) {
    case WF_F32: return 4;
    case WF_F64: return 8;
    case WF_I32: return 4;
    default: return 0;
  }
}

int words_per_elem(int dtype) { return dtype == WF_F64 ? 2 : 1; }

// Tile width used when the caller has not forced one.
int choose_tile(int64_t m, int64_t n) {
  if (g_tile_override) return g_tile_override;
  if (const char* s = std::getenv("WF_TILE")) {
    int t = std::atoi(s);
    if (t == 16 || t == 32 || t == 64) return t;
  }
  (void)m;
  return n >= 1024 ? 64 : 32;
}

int64_t nbands(int64_t m) { return (m + kBand - 1) / kBand; }

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
  if ((ckpt_k > 0) != (ckpt != nullptr)) return WF_E_ARG;
  if ((m - 1) > INT64_MAX / ldc) return WF_E_ARG;
  const int64_t nb = nbands(m);
  if (nb > 0x7fffffff) return WF_E_ARG;

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  const size_t words = (size_t)(nb > 1 ? nb - 1 : 1) * (size_t)n * words_per_elem(dtype);
  DeviceWs* ws = nullptr;
  int rc = ensure_ws(dev, words, &ws);
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
  const int grid = (int)std::min<int64_t>(nb, ws->num_cus);
  const int tile = choose_tile(m, n);
  hipError_t e = launch_forward(dtype, tile, a, grid, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? WF_OK : WF_E_DEVICE;
}

int wf_last_async_error(void* stream) {
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return WF_E_DEVICE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  Control* ctl = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev < (int)g_ws.size()) ctl = g_ws[dev].ctl;
  }
  if (!ctl) return WF_OK;
  uint32_t err = 0;
  if (hipMemcpy(&err, &ctl->err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return WF_E_DEVICE;
  if (err == 0) return WF_OK;
  const uint32_t zero = 0;
  if (hipMemcpy(&ctl->err, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) return WF_E_DEVICE;
  return WF_E_TIMEOUT;
}

}  // extern "C"
