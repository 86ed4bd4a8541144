// Ragged-batch plans (declared in include/wf.h): a device work list over many instances of
// different sizes, swept by one persistent launch that is captured once in a hipGraph and
// replayed, plus the autotuner that picks the tile width and the rows per band.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/wf.h"
#include "wf_host.h"
#include "wf_internal.h"
#include "wf_path.h"

using namespace wf;

struct wf_plan {
  int dtype = 0;
  int dev = 0;
  int32_t batch = 0;
  std::vector<int64_t> m, n, off;
  int64_t elems = 0;
  int tile = 0, rows = 0;         // the configuration in use
  int num_cus = 0;
  Control* ctl = nullptr;         // the plan's own control block
  BatchInst* inst = nullptr;      // device copy of the instance table for 'rows'
  BatchItem* items = nullptr;     // device work list for 'rows'
  int32_t n_items = 0;
  int32_t ck_k = 0;               // checkpoint spacing K the instance table's ck_off is for
  uint64_t* bnd = nullptr;        // handoff words (sized for one row per band, the larger)
  hipStream_t cap = nullptr;      // private stream used only to capture the graph
  hipGraphExec_t exec = nullptr;  // captured launch, valid for the pointers below
  const void* g_C = nullptr;
  void* g_D = nullptr;
  void* g_scores = nullptr;
  void* g_ckpt = nullptr;
  // batched adjoint, set up by the first wf_batch_backward
  BwdInst* b_inst = nullptr;      // instance table (checkpoint offsets for b_k)
  BatchItem* b_items = nullptr;   // bottom-up work list
  int32_t b_n_items = 0;
  int32_t b_k = -1;               // K of b_inst's checkpoint offsets (-1: not built)
  uint32_t* b_sel = nullptr;      // selection bit-planes of every instance
  uint64_t* b_bnd = nullptr;      // reverse handoff words of every instance
  // the adjoint of the scores alone (no g_D): exits, captured labels, group maps
  int32_t* b_exits = nullptr;
  int32_t* b_caps = nullptr;
  int32_t* b_F = nullptr;
  int64_t b_max_cols = 0;         // the largest (G - 1) * n over the instances
};

namespace {

// Element offsets of every instance's checkpoint grid for spacing K, packed in instance order
// with 256-byte aligned starts; returns the total number of elements.
int64_t ckpt_layout(const wf_plan& p, int32_t K, std::vector<int64_t>* offs) {
  const int64_t align = 256 / elem_size(p.dtype);
  int64_t at = 0;
  if (offs) offs->resize(p.batch);
  for (int32_t i = 0; i < p.batch; ++i) {
    if (offs) (*offs)[i] = at;
    const int64_t e = K > 0 ? wf_ckpt_elems(p.m[i], p.n[i], K) : 0;
    at += (e + align - 1) / align * align;
  }
  return at;
}

// Work list for bands of 64*rows rows.  Items are ordered band index first: every band-0
// item of every instance, then every band-1 item, and so on; within one band index,
// instances with more bands left come first.  A band therefore always follows the band
// above it of the same instance (the persistent workgroups can never wait on an unclaimed
// item), and by the time it is claimed the band above has usually been running for a
// whole round of the grid, so little time is lost to pipeline fill.
void build_work(const wf_plan& p, int rows, int32_t K, std::vector<BatchInst>& inst,
                std::vector<BatchItem>& items, size_t& bnd_words) {
  const int64_t H = (int64_t)kBand * rows;
  const int W = words_per_elem(p.dtype);
  std::vector<int64_t> ck;
  ckpt_layout(p, K, &ck);
  inst.resize(p.batch);
  bnd_words = 0;
  int32_t max_nb = 0;
  for (int32_t i = 0; i < p.batch; ++i) {
    BatchInst& b = inst[i];
    b.off = p.off[i];
    b.m = p.m[i];
    b.n = p.n[i];
    b.nb = (int32_t)((p.m[i] + H - 1) / H);
    b.pad = 0;
    b.ck_off = ck[i];
    b.bnd_off = (int64_t)bnd_words;
    bnd_words += (size_t)(b.nb - 1) * (size_t)p.n[i] * W;
    max_nb = std::max(max_nb, b.nb);
  }
  std::vector<int32_t> order(p.batch);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    if (inst[x].nb != inst[y].nb) return inst[x].nb > inst[y].nb;
    return inst[x].n > inst[y].n;
  });
  items.clear();
  for (int32_t band = 0; band < max_nb; ++band)
    for (int32_t i : order)
      if (band < inst[i].nb) items.push_back(BatchItem{i, band});
  if (bnd_words == 0) bnd_words = 1;
}

int upload_work(wf_plan& p, int rows, int32_t K) {
  std::vector<BatchInst> inst;
  std::vector<BatchItem> items;
  size_t words = 0;
  build_work(p, rows, K, inst, items, words);
  if (p.inst) (void)hipFree(p.inst);
  if (p.items) (void)hipFree(p.items);
  p.inst = nullptr;
  p.items = nullptr;
  if (hipMalloc(&p.inst, inst.size() * sizeof(BatchInst)) != hipSuccess) { p.inst = nullptr; return WF_E_NOMEM; }
  if (hipMalloc(&p.items, items.size() * sizeof(BatchItem)) != hipSuccess) { p.items = nullptr; return WF_E_NOMEM; }
  if (hipMemcpy(p.inst, inst.data(), inst.size() * sizeof(BatchInst), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) != hipSuccess)
    return WF_E_DEVICE;
  p.n_items = (int32_t)items.size();
  p.rows = rows;
  p.ck_k = K;
  return WF_OK;
}

hipError_t launch_plan(const wf_plan& p, const void* C, void* D, void* scores, void* ckpt, hipStream_t s) {
  BatchArgs b;
  b.C = C;
  b.D = D;
  b.scores = scores;
  b.ckpt = ckpt;
  b.ckpt_k = ckpt ? p.ck_k : 0;
  b.pad2 = 0;
  b.inst = p.inst;
  b.items = p.items;
  b.n_items = p.n_items;
  b.pad = 0;
  b.ctl = p.ctl;
  b.bnd = p.bnd;
  const int grid = std::min(p.n_items, p.num_cus);
  return launch_forward_batch(p.dtype, p.tile, p.rows, b, grid, s);
}

// ---------------------------------------------------------------------------------------
// Autotuner cache: the best (tile, rows) per (device kind, dtype, shape list), kept for the
// process and, when WF_TUNE_CACHE names a file, in that file (one "key tile rows" line per
// entry, appended when a new entry is measured).
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune;
bool g_tune_file_read = false;

std::string tune_key(const wf_plan& p) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the shape list
  auto mix = [&](uint64_t v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (v >> (8 * k)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)p.batch);
  for (int32_t i = 0; i < p.batch; ++i) {
    mix((uint64_t)p.m[i]);
    mix((uint64_t)p.n[i]);
  }
  char buf[96];
  std::snprintf(buf, sizeof(buf), "cu%d-dt%d-b%d-%016llx", p.num_cus, p.dtype, (int)p.batch, (unsigned long long)h);
  return buf;
}

bool tune_lookup(const std::string& key, int& tile, int& rows) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const char* path = std::getenv("WF_TUNE_CACHE");
  if (path && !g_tune_file_read) {
    g_tune_file_read = true;
    if (FILE* f = std::fopen(path, "r")) {
      char k[128];
      int t, r;
      while (std::fscanf(f, "%127s %d %d", k, &t, &r) == 3)
        if ((t == 16 || t == 32 || t == 64) && (r == 1 || r == 2)) g_tune[k] = {t, r};
      std::fclose(f);
    }
  }
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  tile = it->second.first;
  rows = it->second.second;
  return true;
}

void tune_store(const std::string& key, int tile, int rows) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = {tile, rows};
  if (const char* path = std::getenv("WF_TUNE_CACHE")) {
    if (FILE* f = std::fopen(path, "a")) {
      std::fprintf(f, "%s %d %d\n", key.c_str(), tile, rows);
      std::fclose(f);
    }
  }
}

// Times every allowed (tile, rows) on scratch buffers of the plan's size (the sweep's time
// does not depend on the values) and keeps the fastest.  Synchronizes the stream.
int autotune(wf_plan& p, int want_tile, int want_rows, hipStream_t s) {
  const int es = elem_size(p.dtype);
  const size_t bytes = (size_t)std::max<int64_t>(p.elems, 1) * es;
  void* C = nullptr;
  void* D = nullptr;
  void* sc = nullptr;
  int rc = WF_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float best = 1e30f;
  int best_tile = 0, best_rows = 0;
  if (hipMalloc(&C, bytes) != hipSuccess || hipMalloc(&D, bytes) != hipSuccess ||
      hipMalloc(&sc, (size_t)p.batch * es) != hipSuccess) {
    rc = WF_E_NOMEM;
    goto done;
  }
  if (hipMemsetAsync(C, 0, bytes, s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    rc = WF_E_DEVICE;
    goto done;
  }
  for (int rows : {1, 2}) {
    if (want_rows && rows != want_rows) continue;
    if (rows == 2 && p.dtype == WF_F64) continue;
    if ((rc = upload_work(p, rows, 0)) != WF_OK) goto done;
    for (int tile : {16, 32, 64}) {
      if (want_tile && tile != want_tile) continue;
      p.tile = tile;
      float t_min = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        if (hipEventRecord(e0, s) != hipSuccess || launch_plan(p, C, D, sc, nullptr, s) != hipSuccess ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          rc = WF_E_DEVICE;
          goto done;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = WF_E_DEVICE;
          goto done;
        }
        if (rep > 0) t_min = std::min(t_min, ms);  // the first launch is a warm-up
      }
      if (t_min < best) {
        best = t_min;
        best_tile = tile;
        best_rows = rows;
      }
    }
  }
  p.tile = best_tile;
  p.rows = best_rows;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  if (C) (void)hipFree(C);
  if (D) (void)hipFree(D);
  if (sc) (void)hipFree(sc);
  return rc;
}

void free_plan(wf_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->inst) (void)hipFree(p->inst);
  if (p->items) (void)hipFree(p->items);
  if (p->bnd) (void)hipFree(p->bnd);
  if (p->b_inst) (void)hipFree(p->b_inst);
  if (p->b_items) (void)hipFree(p->b_items);
  if (p->b_sel) (void)hipFree(p->b_sel);
  if (p->b_exits) (void)hipFree(p->b_exits);
  if (p->b_caps) (void)hipFree(p->b_caps);
  if (p->b_F) (void)hipFree(p->b_F);
  if (p->b_bnd) (void)hipFree(p->b_bnd);
  free_control(p->ctl);
  delete p;
}

// Sets up (or, for another K, rebuilds) the batched adjoint's tables and buffers: instance
// table, bottom-up work list, selection bit-planes and reverse handoff words.  Allocates and
// synchronizes the device the first time.
int ensure_bwd(wf_plan& p, int32_t K) {
  if (p.b_k == K) return WF_OK;
  if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
  std::vector<int64_t> ck;
  ckpt_layout(p, K, &ck);
  const int W = words_per_elem(p.dtype);
  std::vector<BwdInst> inst(p.batch);
  int64_t sel_words = 0, bnd_words = 0;
  int32_t max_nb = 0;
  for (int32_t i = 0; i < p.batch; ++i) {
    BwdInst& b = inst[i];
    b.off = p.off[i];
    b.m = p.m[i];
    b.n = p.n[i];
    b.ck_off = ck[i];
    b.nb = (int32_t)((p.m[i] + kBand - 1) / kBand);
    b.pad = 0;
    b.sel_off = sel_words;
    b.bnd_off = bnd_words;
    const int64_t Ks = (p.n[i] + kBand - 1 + 63) / 64;
    sel_words += (int64_t)b.nb * Ks * 64 * 8;
    const int32_t S = path_group_size(b.nb);
    const int64_t G = b.nb > 1 ? (b.nb - 1 + S - 1) / S : 0;
    p.b_max_cols = std::max<int64_t>(p.b_max_cols, (G > 1 ? G - 1 : 0) * p.n[i]);
    bnd_words += (int64_t)(b.nb - 1) * p.n[i] * 2 * W;
    max_nb = std::max(max_nb, b.nb);
  }
  // bottom-up, band-major: the last band of every instance, then the one above it, ...;
  // within one step instances with more bands first
  std::vector<int32_t> order(p.batch);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    if (inst[x].nb != inst[y].nb) return inst[x].nb > inst[y].nb;
    return inst[x].n > inst[y].n;
  });
  std::vector<BatchItem> items;
  for (int32_t t = 0; t < max_nb; ++t)
    for (int32_t i : order)
      if (t < inst[i].nb) items.push_back(BatchItem{i, inst[i].nb - 1 - t});
  if (items.size() >= (size_t)INT32_MAX) return WF_E_ARG;
  const bool first = p.b_k < 0;
  if (p.b_inst) (void)hipFree(p.b_inst);
  p.b_inst = nullptr;
  if (hipMalloc(&p.b_inst, inst.size() * sizeof(BwdInst)) != hipSuccess) { p.b_inst = nullptr; return WF_E_NOMEM; }
  if (hipMemcpy(p.b_inst, inst.data(), inst.size() * sizeof(BwdInst), hipMemcpyHostToDevice) != hipSuccess)
    return WF_E_DEVICE;
  if (first) {
    if (hipMalloc(&p.b_items, items.size() * sizeof(BatchItem)) != hipSuccess) { p.b_items = nullptr; return WF_E_NOMEM; }
    if (hipMemcpy(p.b_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) != hipSuccess)
      return WF_E_DEVICE;
    p.b_n_items = (int32_t)items.size();
    if (hipMalloc(&p.b_sel, (size_t)sel_words * sizeof(uint32_t)) != hipSuccess) { p.b_sel = nullptr; return WF_E_NOMEM; }
    // the path adjoint's buffers, addressed from each instance's selection offset
    if (hipMalloc(&p.b_exits, (size_t)(sel_words / 8) * sizeof(int32_t)) != hipSuccess) {
      p.b_exits = nullptr;
      return WF_E_NOMEM;
    }
    if (hipMalloc(&p.b_caps, (size_t)(sel_words / 2) * sizeof(int32_t)) != hipSuccess) {
      p.b_caps = nullptr;
      return WF_E_NOMEM;
    }
    if (hipMalloc(&p.b_F, (size_t)(sel_words / 8) * sizeof(int32_t)) != hipSuccess) {
      p.b_F = nullptr;
      return WF_E_NOMEM;
    }
    const size_t bw = (size_t)std::max<int64_t>(bnd_words, 1);
    if (hipMalloc(&p.b_bnd, bw * sizeof(uint64_t)) != hipSuccess) { p.b_bnd = nullptr; return WF_E_NOMEM; }
    // tag 0 never equals a launch epoch, so zeroed words read as "not yet written"
    if (hipMemset(p.b_bnd, 0, bw * sizeof(uint64_t)) != hipSuccess) return WF_E_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
  }
  p.b_k = K;
  return WF_OK;
}

// Rebuilds the forward instance table for checkpoint spacing K (the checkpoint offsets
// depend on it).  Drains the device first: a queued replay may still read the old table.
int ensure_fwd_ckpt(wf_plan& p, int32_t K) {
  if (p.ck_k == K) return WF_OK;
  if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
  if (p.exec) {
    (void)hipGraphExecDestroy(p.exec);
    p.exec = nullptr;
  }
  return upload_work(p, p.rows, K);
}

}  // namespace

extern "C" {

int wf_plan_create(wf_plan** out, int dtype, int32_t batch, const int64_t* m, const int64_t* n,
                   const int64_t* offsets, int32_t tile, int32_t rows, void* stream) {
  if (!out) return WF_E_ARG;
  *out = nullptr;
  const int es = elem_size(dtype);
  if (es == 0 || batch < 1 || !m || !n) return WF_E_ARG;
  if (tile != 0 && tile != 16 && tile != 32 && tile != 64) return WF_E_ARG;
  if (rows < 0 || rows > 2) return WF_E_ARG;
  if (rows == 2 && dtype == WF_F64) return WF_E_UNSUPPORTED;
  wf_plan* p = new wf_plan();
  p->dtype = dtype;
  p->batch = batch;
  p->m.assign(m, m + batch);
  p->n.assign(n, n + batch);
  p->off.resize(batch);
  // sizes, then the layout: the caller's offsets, or packed with 256-byte aligned starts
  int64_t cells = 0;
  for (int32_t i = 0; i < batch; ++i) {
    if (m[i] < 1 || n[i] < 1 || n[i] > kMaxLd / es || m[i] > ((int64_t)1 << 40) || m[i] > INT64_MAX / n[i] ||
        m[i] * n[i] > INT64_MAX / 4 - cells) {
      delete p;
      return WF_E_ARG;
    }
    cells += m[i] * n[i];
  }
  const int64_t align = 256 / es;
  if (offsets) {
    std::vector<int32_t> order(batch);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return offsets[x] < offsets[y]; });
    int64_t end = 0;
    for (int32_t i : order) {
      // instances must not overlap: their tables are written in place of nothing shared
      if (offsets[i] < end) {
        delete p;
        return WF_E_ARG;
      }
      end = offsets[i] + m[i] * n[i];
      p->off[i] = offsets[i];
    }
    p->elems = end;
  } else {
    int64_t at = 0;
    for (int32_t i = 0; i < batch; ++i) {
      p->off[i] = at;
      at += (m[i] * n[i] + align - 1) / align * align;
    }
    p->elems = at;
  }
  if (hipGetDevice(&p->dev) != hipSuccess) {
    delete p;
    return WF_E_DEVICE;
  }
  DeviceWs* ws = nullptr;
  int rc = ensure_ws(p->dev, 1, &ws);
  if (rc != WF_OK) {
    delete p;
    return rc;
  }
  p->num_cus = ws->num_cus;
  rc = new_control(p->dev, &p->ctl);
  if (rc != WF_OK) {
    p->ctl = nullptr;
    free_plan(p);
    return rc;
  }
  // handoff words: the one-row-per-band layout needs the most
  {
    std::vector<BatchInst> inst;
    std::vector<BatchItem> items;
    size_t words = 0;
    build_work(*p, 1, 0, inst, items, words);
    if (items.size() >= (size_t)INT32_MAX) {
      delete p;
      return WF_E_ARG;
    }
    if (hipMalloc(&p->bnd, words * sizeof(uint64_t)) != hipSuccess) {
      p->bnd = nullptr;
      free_plan(p);
      return WF_E_NOMEM;
    }
    // tag 0 never equals a launch epoch, so zeroed words read as "not yet written"
    if (hipMemset(p->bnd, 0, words * sizeof(uint64_t)) != hipSuccess) {
      free_plan(p);
      return WF_E_DEVICE;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int want_tile = tile, want_rows = rows;
  if (tile == 0 || rows == 0) {
    const std::string key = tune_key(*p);
    int t = 0, r = 0;
    if (tune_lookup(key, t, r) && (!tile || t == tile) && (!rows || r == rows)) {
      want_tile = t;
      want_rows = r;
    } else {
      rc = autotune(*p, tile, rows, s);
      if (rc != WF_OK) {
        free_plan(p);
        return rc;
      }
      want_tile = p->tile;
      want_rows = p->rows;
      if (!tile && !rows) tune_store(key, want_tile, want_rows);
    }
  }
  p->tile = want_tile;
  rc = upload_work(*p, want_rows, 0);
  if (rc == WF_OK && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
    p->cap = nullptr;
    rc = WF_E_DEVICE;
  }
  if (rc != WF_OK) {
    free_plan(p);
    return rc;
  }
  *out = p;
  return WF_OK;
}

void wf_plan_destroy(wf_plan* plan) { free_plan(plan); }

int64_t wf_plan_elems(const wf_plan* plan) { return plan ? plan->elems : -1; }

int wf_plan_offsets(const wf_plan* plan, int64_t* offsets) {
  if (!plan || !offsets) return WF_E_ARG;
  std::memcpy(offsets, plan->off.data(), plan->off.size() * sizeof(int64_t));
  return WF_OK;
}

int wf_plan_config(const wf_plan* plan, int32_t* tile, int32_t* rows) {
  if (!plan) return WF_E_ARG;
  if (tile) *tile = plan->tile;
  if (rows) *rows = plan->rows;
  return WF_OK;
}

int64_t wf_plan_ckpt_elems(const wf_plan* plan, int32_t ckpt_k) {
  if (!plan || ckpt_k < 0 || ckpt_k > 4096) return -1;
  return ckpt_layout(*plan, ckpt_k, nullptr);
}

int wf_plan_ckpt_offsets(const wf_plan* plan, int32_t ckpt_k, int64_t* offsets) {
  if (!plan || !offsets || ckpt_k < 0 || ckpt_k > 4096) return WF_E_ARG;
  std::vector<int64_t> ck;
  ckpt_layout(*plan, ckpt_k, &ck);
  std::memcpy(offsets, ck.data(), ck.size() * sizeof(int64_t));
  return WF_OK;
}

int wf_batch_forward_ckpt(wf_plan* plan, const void* C, void* D, void* scores, void* ckpt, int32_t ckpt_k,
                          void* stream) {
  if (!plan || !C || !scores) return WF_E_ARG;
  if (ckpt_k < 0 || ckpt_k > 4096) return WF_E_ARG;
  if (ckpt_k == 0 && ckpt != nullptr) return WF_E_ARG;
  if (ckpt_k > 0 && ckpt == nullptr && ckpt_layout(*plan, ckpt_k, nullptr) > 0) return WF_E_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  if (dev != plan->dev) return WF_E_ARG;
  if (ckpt_k == 0) ckpt = nullptr;
  if (ckpt) {
    const int rc = ensure_fwd_ckpt(*plan, ckpt_k);
    if (rc != WF_OK) return rc;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return WF_E_DEVICE;
  if (cs == hipStreamCaptureStatusActive) {
    // the caller is building a graph of its own: record the launch into it
    return launch_plan(*plan, C, D, scores, ckpt, s) == hipSuccess ? WF_OK : WF_E_DEVICE;
  }
  if (!plan->exec || plan->g_C != C || plan->g_D != D || plan->g_scores != scores || plan->g_ckpt != ckpt) {
    if (plan->exec) {
      // an earlier replay may still be queued on some stream
      if (hipDeviceSynchronize() != hipSuccess) return WF_E_DEVICE;
      (void)hipGraphExecDestroy(plan->exec);
      plan->exec = nullptr;
    }
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return WF_E_DEVICE;
    const hipError_t le = launch_plan(*plan, C, D, scores, ckpt, plan->cap);
    const hipError_t ce = hipStreamEndCapture(plan->cap, &g);
    if (le != hipSuccess || ce != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return WF_E_DEVICE;
    }
    const hipError_t ie = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      plan->exec = nullptr;
      return WF_E_DEVICE;
    }
    plan->g_C = C;
    plan->g_D = D;
    plan->g_scores = scores;
    plan->g_ckpt = ckpt;
  }
  return hipGraphLaunch(plan->exec, s) == hipSuccess ? WF_OK : WF_E_DEVICE;
}

int wf_batch_forward(wf_plan* plan, const void* C, void* D, void* scores, void* stream) {
  return wf_batch_forward_ckpt(plan, C, D, scores, nullptr, 0, stream);
}

int wf_batch_backward(wf_plan* plan, const void* C, const void* ckpt, int32_t ckpt_k, const void* D,
                      const void* g_scores, const void* g_D, void* g_C, void* stream) {
  if (!plan) return WF_E_ARG;
  if (plan->dtype != WF_F32 && plan->dtype != WF_F64) return WF_E_UNSUPPORTED;
  if (!C || !g_C) return WF_E_ARG;
  if (ckpt_k < 0 || ckpt_k > 4096) return WF_E_ARG;
  // exactly one source of the band top rows: the checkpoint grids or the saved tables
  if (ckpt_k > 0 ? (D != nullptr || (ckpt == nullptr && ckpt_layout(*plan, ckpt_k, nullptr) > 0))
                 : (D == nullptr || ckpt != nullptr))
    return WF_E_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_E_DEVICE;
  if (dev != plan->dev) return WF_E_ARG;
  int rc = ensure_bwd(*plan, ckpt_k);
  if (rc != WF_OK) return rc;
  BwdBatchArgs b;
  b.C = C;
  b.top = ckpt_k > 0 ? ckpt : D;
  b.ckpt_k = ckpt_k;
  b.n_items = plan->b_n_items;
  b.gD = g_D;
  b.gscores = g_scores;
  b.gC = g_C;
  b.inst = plan->b_inst;
  b.items = plan->b_items;
  b.sel = plan->b_sel;
  b.bnd = plan->b_bnd;
  b.ctl = plan->ctl;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!g_D) {
    // the scores alone: each instance's upstream value on its argmin path, zero elsewhere
    const PathBufs pb{plan->b_exits, plan->b_caps, plan->b_F, plan->batch, 0, plan->b_max_cols};
    return launch_path_batch(plan->dtype, b, pb, std::min(b.n_items, 2 * plan->num_cus), st) == hipSuccess
               ? WF_OK
               : WF_E_DEVICE;
  }
  // the reverse tile of the batch's largest instance
  int32_t big = 0;
  for (int32_t i = 1; i < plan->batch; ++i)
    if (plan->m[i] * plan->n[i] > plan->m[big] * plan->n[big]) big = i;
  const int tile = pick_tile(plan->dtype, plan->m[big], plan->n[big], true);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the recompute's workgroups are small (two waves, half of a CU's LDS): two per CU
  if (launch_select_batch(plan->dtype, b, std::min(b.n_items, 2 * plan->num_cus), s) != hipSuccess)
    return WF_E_DEVICE;
  if (launch_adjoint_batch(plan->dtype, tile, b, std::min(b.n_items, plan->num_cus), s) != hipSuccess)
    return WF_E_DEVICE;
  return WF_OK;
}

}  // extern "C"
