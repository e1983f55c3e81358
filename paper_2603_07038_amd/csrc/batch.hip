// Batched design variants (etm_batch_* in include/etm.h).
//
// Many bound plans of uneven size advance together: each EM step is ONE
// launch of the batched march kernel over a (variant, tile x, tile y, z chunk)
// work list that covers every attached variant, so small variants share the
// machine instead of each under-filling it.  Between the steps where some
// variant has a thermal step, a history record or a scheduled mechanical
// solve, the run is a segment of plain EM steps; each segment length is
// captured once as a HIP graph (EM launch + step-counter increment per step)
// and replayed.  Variant descriptors live in device memory and are restaged
// at each segment boundary, so the graphs stay valid until the attached set
// changes.  Every variant computes with the same per-node code as its solo
// run, so its results are bitwise those of the solo run.
//
// The tile shape per variant -- its z-chunk length and, in mixed precision,
// its work layout (runs over the x-fastest plane or row segments) -- comes
// from a tuning table keyed by the variant's size class
// ("{\"kchunk\": {\"<log2 cells>\": k, ...}, \"layout\": {\"<log2 cells>\": 1 or 2},
// \"kchunk_fp64\": {...}}"; "kchunk" serves mixed precision),
// written by the package's autotuner; without an entry the automatic choice
// is used.
//
// etm_batch_advance_noalloc runs the same steps with the same kernels but
// allocates nothing: the descriptors, the work list and the step counter live
// in a fixed array of device memory (`scratch`, one copy per GPU), the work
// list is generated on the device, and every step is launched directly
// instead of from a graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "etm_internal.h"
#include "plan.h"

using namespace etm;

namespace {
constexpr int kStageRing = 8;
}

struct etm_batch {
  int32_t max_slots = 0;
  std::vector<etm_plan *> slots;
  std::map<int, int> kchunk_by_class;       // mixed precision
  std::map<int, int> kchunk_fp64_by_class;  // FP64
  std::map<int, int> layout_by_class;
  // device
  BatchVar *d_vars = nullptr;
  int4 *d_items = nullptr;
  size_t items_cap = 0;
  int n_items = 0;
  int64_t *d_ctr = nullptr;
  // pinned staging ring for descriptors
  BatchVar *h_vars = nullptr;
  hipEvent_t stage_ev[kStageRing] = {};
  bool stage_used[kStageRing] = {};
  int stage_next = 0;
  // work list / graphs
  bool dirty = true;
  int precision = -1;
  std::vector<int> order;  // slot of each compact variant
  std::map<int, hipGraphExec_t> graphs;
  hipStream_t run = nullptr;  // the batch's own stream (graphs are captured and replayed on it)
  int device = 0;             // device current at creation (that of `run`)
  hipEvent_t order_ev = nullptr;  // orders `run` against the caller's and the plans' streams
  // per compact variant, sized max_slots at creation: each plan's own stream
  // during an advance, and its state index one step back
  std::vector<hipStream_t> own;
  std::vector<int> old_cur;
};

namespace {

void drop_graphs(etm_batch *b) {
  for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

// Minimal reader of one integer map of the tuning table, e.g.
// {"kchunk": {"17": 8, ...}}: entries with a value outside [lo, hi] are
// ignored, as is anything malformed.
void parse_tune(const char *json, const char *name, int lo, int hi, std::map<int, int> &out) {
  if (!json) return;
  const std::string s(json);
  size_t p = s.find(name);
  if (p == std::string::npos) return;
  p = s.find('{', p);
  if (p == std::string::npos) return;
  const size_t e = s.find('}', p);
  while (p < e) {
    const size_t q0 = s.find('"', p);
    if (q0 == std::string::npos || q0 >= e) break;
    const size_t q1 = s.find('"', q0 + 1);
    const size_t c = s.find(':', q1);
    if (q1 == std::string::npos || c == std::string::npos || c >= e) break;
    const int key = std::atoi(s.substr(q0 + 1, q1 - q0 - 1).c_str());
    const int val = std::atoi(s.c_str() + c + 1);
    if (val >= lo && val <= hi) out[key] = val;
    p = s.find(',', c);
    if (p == std::string::npos || p > e) break;
  }
}

int size_class(const etm_plan *p) {
  const double cells = double(p->nx) * p->ny * p->nz;
  return int(std::floor(std::log2(std::max(cells, 1.0))));
}

// Compact list of the attached slots (b->order keeps its capacity of
// max_slots from creation, so this allocates nothing) and each variant's
// z-chunk from the tuning table.
void order_variants(etm_batch *b) {
  b->order.clear();
  for (int s = 0; s < b->max_slots; ++s)
    if (b->slots[s]) b->order.push_back(s);
  for (int slot : b->order) {
    etm_plan *p = b->slots[slot];
    auto lt = b->layout_by_class.find(size_class(p));
    p->layout = lt != b->layout_by_class.end() ? lt->second : kLayoutAuto;
    const std::map<int, int> &km = b->precision == ETM_PREC_FP64 ? b->kchunk_fp64_by_class : b->kchunk_by_class;
    auto it = km.find(size_class(p));
    p->kchunk = it != km.end() ? it->second : em_kchunk(p->dev_grid(), b->precision);
  }
}

// New work list after attach / detach.  Kernels and graph launches of the
// previous work list may still be running on the batch's own (non-blocking)
// stream: drain it before the list, the graphs or their buffers change.
etm_status rebuild(etm_batch *b) {
  HIP_TRY(hipStreamSynchronize(b->run));
  order_variants(b);
  std::vector<int4> items;
  for (size_t v = 0; v < b->order.size(); ++v) {
    etm_plan *p = b->slots[b->order[v]];
    const DevGrid g = p->dev_grid();
    int ntx, nty, nkc;
    em_tiles(g, b->precision, p->kchunk, &ntx, &nty, &nkc);
    for (int c = 0; c < nkc; ++c)
      for (int y = 0; y < nty; ++y)
        for (int x = 0; x < ntx; ++x) items.push_back(make_int4(int(v), x, y, c));
  }
  if (items.size() > size_t(0x7fffffff)) return fail(ETM_E_INVAL, "batch work list too large");
  if (items.size() > b->items_cap) {
    if (b->d_items) HIP_TRY(hipFree(b->d_items));
    b->d_items = nullptr;
    HIP_TRY(hipMalloc((void **)&b->d_items, std::max<size_t>(items.size(), 1) * sizeof(int4)));
    b->items_cap = items.size();
  }
  if (!items.empty()) {
    HIP_TRY(hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice, b->run));
    HIP_TRY(hipStreamSynchronize(b->run));
  }
  b->n_items = int(items.size());
  drop_graphs(b);
  b->dirty = false;
  return ETM_OK;
}

// Where the batched kernels find their descriptors, work list and step
// counter, and whether plain-step segments are replayed from graphs.
struct BatchDev {
  BatchVar *vars = nullptr;
  const int4 *items = nullptr;
  int n_items = 0;
  int64_t *ctr = nullptr;
  bool graphs = false;
};

// Stage the descriptors of every variant at its current state.
etm_status stage_vars(etm_batch *b, hipStream_t st, const BatchDev &D) {
  const int slot = b->stage_next;
  b->stage_next = (b->stage_next + 1) % kStageRing;
  if (b->stage_used[slot]) HIP_TRY(hipEventSynchronize(b->stage_ev[slot]));
  BatchVar *h = b->h_vars + size_t(slot) * b->max_slots;
  for (size_t v = 0; v < b->order.size(); ++v) {
    etm_plan *p = b->slots[b->order[v]];
    BatchVar &V = h[v];
    std::memset(&V, 0, sizeof(V));
    V.L = em_launch_template(p);
    for (int q = 0; q < 3; ++q)
      for (int d = 0; d < 3; ++d) V.e[q][d] = p->r_e[q][d].bytes ? p->ws + p->r_e[q][d].off : nullptr;
    if (p->prec == ETM_PREC_MIXED)
      for (int q = 0; q < 2; ++q)
        for (int d = 0; d < 3; ++d) V.h[q][d] = p->ws + p->r_h[q][d].off;
    V.theta[0] = p->ptr<double>(p->r_theta[0]);
    V.theta[1] = p->ptr<double>(p->r_theta[1]);
    V.theta32 = p->prec == ETM_PREC_MIXED ? p->ptr<float>(p->r_theta32) : nullptr;
    V.step0 = p->step;
    V.cur0 = p->cur;
    V.th0 = p->th_cur;
    V.R = p->R;
    V.kchunk = p->kchunk;
    V.acc_joule0 = p->joule_pending ? 1 : 0;
  }
  HIP_TRY(hipMemcpyAsync(D.vars, h, b->order.size() * sizeof(BatchVar), hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(b->stage_ev[slot], st));
  b->stage_used[slot] = true;
  HIP_TRY(launch_step_ctr(D.ctr, 0, 1, st));
  return ETM_OK;
}

etm_status enqueue_steps(etm_batch *b, int len, hipStream_t st, const BatchDev &D) {
  for (int q = 0; q < len; ++q) {
    HIP_TRY(launch_em_batched(D.vars, D.items, D.n_items, D.ctr, b->precision, st));
    HIP_TRY(launch_step_ctr(D.ctr, 1, 0, st));
  }
  return ETM_OK;
}

// A segment of len plain EM steps, from a captured graph when len > 1 and
// graphs are in use.
etm_status run_segment(etm_batch *b, int len, hipStream_t st, const BatchDev &D) {
  if (len <= 1 || !D.graphs) return enqueue_steps(b, len, st, D);
  auto it = b->graphs.find(len);
  if (it == b->graphs.end()) {
    hipGraph_t graph;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    etm_status s = enqueue_steps(b, len, st, D);
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (s != ETM_OK) return s;
    if (e != hipSuccess) return fail(ETM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t exec;
    HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    HIP_TRY(hipGraphDestroy(graph));
    it = b->graphs.emplace(len, exec).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, st));
  return ETM_OK;
}

// ---- the advance loop shared by both entry points ---------------------------
// Runs n steps of every variant in b->order on the batch's stream: segments
// of plain EM steps up to the next step at which some variant has a thermal
// step or a history record, then that host-side work per variant.  `D` says
// where the kernels find their descriptors, work list and counter.
etm_status advance_impl(etm_batch *b, int64_t n, hipStream_t caller, const BatchDev &D) {
  Range r_call("etm_batch_advance");
  hipStream_t st = b->run;
  const size_t nv = b->order.size();
  // the batch stream runs after the caller's stream and after each plan's own stream
  HIP_TRY(hipEventRecord(b->order_ev, caller));
  HIP_TRY(hipStreamWaitEvent(st, b->order_ev, 0));
  for (size_t v = 0; v < nv; ++v) {
    etm_plan *p = b->slots[b->order[v]];
    b->own[v] = p->stream;
    if (p->stream != caller) {
      HIP_TRY(hipEventRecord(b->order_ev, p->stream));
      HIP_TRY(hipStreamWaitEvent(st, b->order_ev, 0));
    }
    p->stream = st;
  }
  int64_t done = 0;
  etm_status s = ETM_OK;
  while (done < n && s == ETM_OK) {
    // next step at which some variant needs host-side work
    int64_t len = n - done;
    for (int slot : b->order) {
      etm_plan *p = b->slots[slot];
      const int64_t to_thermal = p->R - (p->step % p->R);
      len = std::min(len, to_thermal);
      if (p->opts.history_stride > 0)
        len = std::min<int64_t>(len, p->opts.history_stride - (p->step % p->opts.history_stride));
    }
    len = std::max<int64_t>(std::min<int64_t>(len, kWaveBlock), 1);
    // closed-form waves: each variant's sample table covers the segment
    for (int slot : b->order)
      if (s == ETM_OK) s = ensure_waves(b->slots[slot], len);
    if (s != ETM_OK) break;
    if ((s = stage_vars(b, st, D)) != ETM_OK) break;
    if ((s = run_segment(b, int(len), st, D)) != ETM_OK) break;
    for (size_t v = 0; v < nv; ++v) {
      etm_plan *p = b->slots[b->order[v]];
      for (int64_t q = 0; q < len; ++q) {
        b->old_cur[v] = p->cur;
        p->cur = p->prec == ETM_PREC_FP64 ? (p->cur + 1) % 3 : 1 - p->cur;
      }
      p->step += len;
      p->joule_pending = true;
    }
    done += len;
    for (size_t v = 0; v < nv && s == ETM_OK; ++v) {
      etm_plan *p = b->slots[b->order[v]];
      if (p->step % p->R == 0) {
        if ((s = thermal_one(p)) != ETM_OK) break;
        if (p->opts.mech_every_thermal > 0 && p->n_thermal % p->opts.mech_every_thermal == 0) {
          s = mech_solve_impl(p);
          if (s == ETM_E_NOCONV) s = ETM_OK;
          if (s != ETM_OK) break;
        }
      }
      if (p->opts.history_stride > 0 && p->step % p->opts.history_stride == 0) s = diag_record(p, b->old_cur[v]);
    }
  }
  for (size_t v = 0; v < nv; ++v) {
    etm_plan *p = b->slots[b->order[v]];
    if (s == ETM_OK) s = joule_flush(p);
  }
  // the caller's stream and each plan's own stream continue after the batch
  hipError_t e = hipEventRecord(b->order_ev, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(caller, b->order_ev, 0);
  for (size_t v = 0; v < nv; ++v) {
    etm_plan *p = b->slots[b->order[v]];
    if (e == hipSuccess && b->own[v] != caller) e = hipStreamWaitEvent(b->own[v], b->order_ev, 0);
    p->stream = b->own[v];
  }
  if (e != hipSuccess && s == ETM_OK) s = fail(ETM_E_HIP, std::string("stream ordering: ") + hipGetErrorString(e));
  return s;
}

// ---- fixed device scratch of the allocation-free advance ---------------------
// Layout: [step counter | descriptors of up to kScratchSlots variants | work
// list].  One copy per GPU, held until the process ends; its device address
// is looked up once per device (kernels take that address, never the name).
constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr int kScratchSlots = 64;
constexpr size_t kScratchVarsOff = 256;
constexpr size_t kScratchItemsOff = kScratchVarsOff + ((sizeof(BatchVar) * kScratchSlots + 255) & ~size_t(255));
constexpr int64_t kScratchMaxItems = int64_t((kScratchBytes - kScratchItemsOff) / sizeof(int4));
static_assert(kScratchItemsOff < kScratchBytes / 4, "descriptor area too large for the scratch array");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev` (looked up with dev current, once).
etm_status scratch_on(int dev, char **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ETM_E_INVAL, "device index out of range for the no-alloc scratch");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int prev = 0;
    HIP_TRY(hipGetDevice(&prev));
    if (prev != dev) HIP_TRY(hipSetDevice(dev));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != dev) HIP_TRY(hipSetDevice(prev));
    if (e != hipSuccess || !ptr)
      return fail(ETM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return ETM_OK;
}

// Work list of the variants, generated on the device in the order of the
// graph path: item i of variant v (prefix[v] <= i < prefix[v + 1]) is tile
// (x, y, z chunk) with local index (c * nty + y) * ntx + x.
struct ItemTable {
  int n_var;
  int prefix[kScratchSlots + 1];
  int ntx[kScratchSlots], nty[kScratchSlots];
};

__global__ __launch_bounds__(256) void batch_items_kernel(ItemTable T, int4 *items) {
  const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (i >= T.prefix[T.n_var]) return;
  int v = 0;
  while (v + 1 < T.n_var && T.prefix[v + 1] <= i) ++v;
  const int loc = i - T.prefix[v], ntx = T.ntx[v], nty = T.nty[v];
  items[i] = make_int4(v, loc % ntx, (loc / ntx) % nty, loc / (ntx * nty));
}

}  // namespace

extern "C" {

etm_status etm_batch_create(int32_t max_slots, const char *tune_json, etm_batch **out) {
  if (!out) return fail(ETM_E_INVAL, "null out");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 4096) return fail(ETM_E_INVAL, "max_slots must be in 1..4096");
  etm_batch *b = new etm_batch();
  b->max_slots = max_slots;
  b->slots.assign(max_slots, nullptr);
  b->order.reserve(max_slots);
  b->own.assign(max_slots, nullptr);
  b->old_cur.assign(max_slots, 0);
  parse_tune(tune_json, "\"kchunk\"", 1, 128, b->kchunk_by_class);
  parse_tune(tune_json, "\"kchunk_fp64\"", 1, 128, b->kchunk_fp64_by_class);
  parse_tune(tune_json, "\"layout\"", kLayoutRuns, kLayoutRows, b->layout_by_class);
  hipError_t e = hipGetDevice(&b->device);
  if (e == hipSuccess) e = hipMalloc((void **)&b->d_vars, sizeof(BatchVar) * max_slots);
  if (e == hipSuccess) e = hipMalloc((void **)&b->d_ctr, sizeof(int64_t));
  if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_vars, sizeof(BatchVar) * max_slots * kStageRing, hipHostMallocDefault);
  for (int q = 0; q < kStageRing && e == hipSuccess; ++q) e = hipEventCreateWithFlags(&b->stage_ev[q], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->order_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->run, hipStreamNonBlocking);
  if (e != hipSuccess) {
    etm_batch_destroy(b);
    return fail(ETM_E_HIP, std::string("batch allocation: ") + hipGetErrorString(e));
  }
  *out = b;
  return ETM_OK;
}

etm_status etm_batch_attach(etm_batch *b, etm_plan *p, int32_t *slot) {
  if (!b || !p) return fail(ETM_E_INVAL, "null batch or plan");
  if (!p->bound) return fail(ETM_E_STATE, "plan is not bound");
  int used = 0;
  for (etm_plan *q : b->slots) {
    if (q == p) return fail(ETM_E_INVAL, "plan already attached");
    if (q) ++used;
  }
  if (used > 0 && p->prec != b->precision) return fail(ETM_E_INVAL, "all variants of a batch share one precision");
  for (int s = 0; s < b->max_slots; ++s)
    if (!b->slots[s]) {
      b->slots[s] = p;
      b->precision = p->prec;
      b->dirty = true;
      if (slot) *slot = s;
      return ETM_OK;
    }
  return fail(ETM_E_NOMEM, "no free batch slot");
}

etm_status etm_batch_detach(etm_batch *b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot]) return fail(ETM_E_INVAL, "bad slot");
  b->slots[slot]->kchunk = 0;
  b->slots[slot]->layout = kLayoutAuto;
  b->slots[slot] = nullptr;
  b->dirty = true;
  return ETM_OK;
}

etm_status etm_batch_advance(etm_batch *b, int64_t n, void *stream) {
  if (!b) return fail(ETM_E_INVAL, "null batch");
  if (n < 0) return fail(ETM_E_INVAL, "negative step count");
  etm_status s;
  if (b->dirty && (s = rebuild(b)) != ETM_OK) return s;
  if (b->order.empty() || n == 0) return ETM_OK;
  BatchDev D;
  D.vars = b->d_vars;
  D.items = b->d_items;
  D.n_items = b->n_items;
  D.ctr = b->d_ctr;
  D.graphs = true;
  return advance_impl(b, n, static_cast<hipStream_t>(stream), D);
}

etm_status etm_batch_advance_noalloc(etm_batch *b, int64_t n, void *stream) {
  if (!b) return fail(ETM_E_INVAL, "null batch");
  if (n < 0) return fail(ETM_E_INVAL, "negative step count");
  int n_att = 0;
  for (etm_plan *p : b->slots)
    if (p) {
      ++n_att;
      if (p->opts.mech_every_thermal > 0)
        return fail(ETM_E_INVAL, "no-alloc advance: attached plans must not schedule mechanical solves "
                                 "(mech_every_thermal = 0; call etm_mech_solve after the march)");
    }
  if (n_att > kScratchSlots)
    return fail(ETM_E_INVAL, "no-alloc advance: " + std::to_string(n_att) + " attached variants, at most " +
                                 std::to_string(kScratchSlots));
  if (n_att == 0 || n == 0) return ETM_OK;
  // the work list of the current set (the graph path's list is left as it is)
  order_variants(b);
  ItemTable T;
  std::memset(&T, 0, sizeof(T));
  T.n_var = int(b->order.size());
  int64_t total = 0;
  for (int v = 0; v < T.n_var; ++v) {
    etm_plan *p = b->slots[b->order[v]];
    hipPointerAttribute_t attr;
    HIP_TRY(hipPointerGetAttributes(&attr, p->ws));
    if (attr.device != b->device)
      return fail(ETM_E_INVAL, "no-alloc advance: a plan's workspace is not on the batch's device");
    int ntx, nty, nkc;
    em_tiles(p->dev_grid(), b->precision, p->kchunk, &ntx, &nty, &nkc);
    T.prefix[v] = int(total);
    T.ntx[v] = ntx;
    T.nty[v] = nty;
    total += int64_t(ntx) * nty * nkc;
    if (total > kScratchMaxItems)
      return fail(ETM_E_INVAL, "no-alloc advance: the work list exceeds " + std::to_string(kScratchMaxItems) +
                                   " tiles (" + std::to_string(kScratchBytes) + " bytes of scratch)");
  }
  T.prefix[T.n_var] = int(total);
  char *base = nullptr;
  etm_status s = scratch_on(b->device, &base);
  if (s != ETM_OK) return s;
  BatchDev D;
  D.ctr = reinterpret_cast<int64_t *>(base);
  D.vars = reinterpret_cast<BatchVar *>(base + kScratchVarsOff);
  int4 *items = reinterpret_cast<int4 *>(base + kScratchItemsOff);
  D.items = items;
  D.n_items = int(total);
  D.graphs = false;
  // the list is written on the batch's stream, after the caller's work
  hipStream_t caller = static_cast<hipStream_t>(stream);
  HIP_TRY(hipEventRecord(b->order_ev, caller));
  HIP_TRY(hipStreamWaitEvent(b->run, b->order_ev, 0));
  if (total > 0) {
    hipLaunchKernelGGL(batch_items_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, b->run, T, items);
    HIP_TRY(hipGetLastError());
  }
  return advance_impl(b, n, caller, D);
}

void etm_batch_destroy(etm_batch *b) {
  if (!b) return;
  if (b->run) (void)hipStreamSynchronize(b->run);
  drop_graphs(b);
  for (int q = 0; q < kStageRing; ++q)
    if (b->stage_ev[q]) {
      if (b->stage_used[q]) (void)hipEventSynchronize(b->stage_ev[q]);
      (void)hipEventDestroy(b->stage_ev[q]);
    }
  if (b->order_ev) (void)hipEventDestroy(b->order_ev);
  if (b->d_vars) (void)hipFree(b->d_vars);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_ctr) (void)hipFree(b->d_ctr);
  if (b->run) (void)hipStreamDestroy(b->run);
  if (b->h_vars) (void)hipHostFree(b->h_vars);
  delete b;
}

}  // extern "C"
