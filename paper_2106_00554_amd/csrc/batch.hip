// Batched execution of many independent operators (uneven sizes, wavelet
// orders, q and element types) as one hipGraph launch per direction.
//
// The graph forks from the launch stream into B concurrent branches; the
// instances are dealt to the branches in a chosen order, each instance being
// its own stage kernels (the same kernels as the single-plan entry points), and
// the branches join before the graph ends.  Independent branches let small
// instances fill the CUs that a large one leaves idle and remove the per-launch
// host cost.  A graph is captured once per set of pointers and replayed; the
// schedule (B, order) is a batch property that wh2wav_batch_tune picks by
// timing every candidate on the caller's buffers.
//
// In the fused mode the small instances instead run as fused launches, one per
// round of their stages (fused_batch.h), on the graph's own stream beside the
// branches, which keep the other instances.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/wh2wav.h"
#include "abi_internal.h"
#include "fused_batch.h"

namespace {

constexpr int kMaxBranches = 8;
constexpr size_t kAlign = 256;
constexpr size_t kMaxGraphs = 8;

struct GraphEntry {
  int dir, branches, order, mode;
  const void* ws;
  std::vector<const void*> in, out;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;       // recorded after every launch of `exec`
  std::vector<void*> io_dev;       // fused mode: per program, its instances' (input, output) pointers
};

// Waits for the last launch of a cached graph, then frees it: a graph may
// still run on the caller's stream when it leaves the cache.
void drop_graph(GraphEntry& g) {
  if (g.done) {
    (void)hipEventSynchronize(g.done);
    (void)hipEventDestroy(g.done);
  }
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  for (void* p : g.io_dev)
    if (p) (void)hipFree(p);
  g.io_dev.clear();
  g.done = nullptr;
  g.exec = nullptr;
}

}  // namespace

struct wh2wav_batch_s {
  std::vector<wh2wav_plan_t> plans;
  std::vector<wh2wav::PlanShape> shape;
  std::vector<size_t> ws_off;
  size_t ws_total = 0;
  int branches = 4;
  int order = 1;  // 0: as given, 1: largest first
  hipStream_t cap = nullptr;
  hipStream_t side[kMaxBranches] = {};
  hipEvent_t fork = nullptr, join[kMaxBranches] = {};
  std::vector<GraphEntry> graphs;
  int mode = WH2WAV_BATCH_BRANCHES;
  std::vector<char> in_kernel;            // instance runs in the fused launches (fused mode)
  wh2wav_fused::Program prog[2][2];       // [dtype][direction]
};

namespace {

int fail(int code, const std::string& msg) { return wh2wav::set_error(code, msg); }

#define HIP_B(call)                                                              \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(WH2WAV_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

double cost_of(const wh2wav::PlanShape& s) {
  const double n = double(s.ntot);
  const double e = s.dtype == WH2WAV_F64 ? 2.0 : 1.0;
  return n * e;
}

std::vector<int> schedule_order(const wh2wav_batch_s* b) {
  std::vector<int> idx(b->plans.size());
  std::iota(idx.begin(), idx.end(), 0);
  if (b->order == 1)
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int a, int c) { return cost_of(b->shape[a]) > cost_of(b->shape[c]); });
  return idx;
}

void release_batch(wh2wav_batch_s* b) {
  for (auto& g : b->graphs) drop_graph(g);
  b->graphs.clear();
  for (auto& pd : b->prog)
    for (auto& pr : pd) wh2wav_fused::release(&pr);
  for (auto* p : b->plans) wh2wav_destroy(p);
  b->plans.clear();
  for (int k = 0; k < kMaxBranches; ++k) {
    if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
    if (b->join[k]) (void)hipEventDestroy(b->join[k]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->cap) (void)hipStreamDestroy(b->cap);
}

// Fused mode: the (input, output) pointer pairs of every program's
// instances, uploaded to device arrays kept with the graph that uses them.
int upload_io(wh2wav_batch_s* b, int dir, const void* const* in, void* const* out, GraphEntry* e) {
  for (auto& pd : b->prog) {
    const auto& pr = pd[dir];
    void* d = nullptr;
    if (pr.ninst > 0) {
      std::vector<const void*> io;
      for (int i : pr.members) io.push_back(in[i]), io.push_back(out[i]);
      HIP_B(hipMalloc(&d, sizeof(void*) * io.size()));
      e->io_dev.push_back(d);
      HIP_B(hipMemcpy(d, io.data(), sizeof(void*) * io.size(), hipMemcpyHostToDevice));
    } else {
      e->io_dev.push_back(nullptr);
    }
  }
  return WH2WAV_OK;
}

// Captures the instances' stage kernels into one executable graph.
int capture(wh2wav_batch_s* b, int dir, const void* const* in, void* const* out, void* ws, GraphEntry* ge) {
  hipGraphExec_t* exec = &ge->exec;
  const int nb = std::max(1, std::min(b->branches, kMaxBranches));
  const bool fused = b->mode == WH2WAV_BATCH_FUSED;
  if (fused) {
    int rc = upload_io(b, dir, in, out, ge);
    if (rc) return rc;
  }
  HIP_B(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  int rc = WH2WAV_OK;
  hipError_t he = hipEventRecord(b->fork, b->cap);
  for (int k = 0; k < nb && he == hipSuccess; ++k) he = hipStreamWaitEvent(b->side[k], b->fork, 0);
  if (he != hipSuccess) rc = fail(WH2WAV_EHIP, std::string("batch fork: ") + hipGetErrorString(he));
  // the fused launches run on the capture stream, beside the branches
  for (int d = 0; d < 2 && fused && rc == WH2WAV_OK; ++d)
    if (b->prog[d][dir].ninst > 0)
      rc = wh2wav_fused::launch(b->prog[d][dir], ws, static_cast<void* const*>(ge->io_dev[d]), b->cap);
  std::vector<int> idx;
  for (int i : schedule_order(b))
    if (!fused || !b->in_kernel[i]) idx.push_back(i);
  for (size_t t = 0; t < idx.size() && rc == WH2WAV_OK; ++t) {
    const int i = idx[t];
    void* wsi = static_cast<char*>(ws) + b->ws_off[i];
    hipStream_t st = b->side[t % nb];
    rc = dir == 0 ? wh2wav_forward(b->plans[i], in[i], out[i], wsi, st)
                  : wh2wav_adjoint(b->plans[i], in[i], out[i], wsi, st);
  }
  // join every branch even after a failure, so that no stream is left capturing
  for (int k = 0; k < nb; ++k) {
    he = hipEventRecord(b->join[k], b->side[k]);
    if (he == hipSuccess) he = hipStreamWaitEvent(b->cap, b->join[k], 0);
    if (he != hipSuccess && rc == WH2WAV_OK)
      rc = fail(WH2WAV_EHIP, std::string("batch join: ") + hipGetErrorString(he));
  }
  hipGraph_t g = nullptr;
  he = hipStreamEndCapture(b->cap, &g);
  if (rc != WH2WAV_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (he != hipSuccess) return fail(WH2WAV_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(he));
  he = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (he != hipSuccess) return fail(WH2WAV_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(he));
  return WH2WAV_OK;
}

int check_ptrs(const wh2wav_batch_s* b, int dir, const void* const* in, void* const* out, void* ws) {
  if (!in || !out) return fail(WH2WAV_EINVAL, "pointer arrays are NULL");
  if (!ws && b->ws_total) return fail(WH2WAV_EINVAL, "workspace is NULL");
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const auto& s = b->shape[i];
    const int64_t xlen = s.xlen;
    const int64_t inlen = dir == 0 ? xlen : s.m, outlen = dir == 0 ? s.m : xlen;
    if ((inlen && !in[i]) || (outlen && !out[i]))
      return fail(WH2WAV_EINVAL, "instance " + std::to_string(i) + ": NULL input or output");
  }
  return WH2WAV_OK;
}

int run(wh2wav_batch_s* b, int dir, const void* const* in, void* const* out, void* ws, void* stream) {
  int rc = check_ptrs(b, dir, in, out, ws);
  if (rc) return rc;
  const size_t n = b->plans.size();
  GraphEntry* hit = nullptr;
  for (auto& g : b->graphs) {
    if (g.dir != dir || g.branches != b->branches || g.order != b->order || g.mode != b->mode || g.ws != ws)
      continue;
    if (std::equal(g.in.begin(), g.in.end(), in) && std::equal(g.out.begin(), g.out.end(), out)) {
      hit = &g;
      break;
    }
  }
  if (!hit) {
    if (b->graphs.size() >= kMaxGraphs) {
      drop_graph(b->graphs.front());
      b->graphs.erase(b->graphs.begin());
    }
    GraphEntry e;
    e.dir = dir, e.branches = b->branches, e.order = b->order, e.mode = b->mode, e.ws = ws;
    e.in.assign(in, in + n);
    e.out.assign(out, out + n);
    HIP_B(hipEventCreateWithFlags(&e.done, hipEventDisableTiming));
    rc = capture(b, dir, in, out, ws, &e);
    if (rc) {
      drop_graph(e);
      return rc;
    }
    b->graphs.push_back(std::move(e));
    hit = &b->graphs.back();
  }
  HIP_B(hipGraphLaunch(hit->exec, static_cast<hipStream_t>(stream)));
  HIP_B(hipEventRecord(hit->done, static_cast<hipStream_t>(stream)));
  return WH2WAV_OK;
}

// A live batch handle (one returned by wh2wav_plan_batch and not destroyed).
int check_batch(const wh2wav_batch_s* b) {
  if (!b) return fail(WH2WAV_EINVAL, "batch is NULL");
  if (!wh2wav::handle_live(b)) return fail(WH2WAV_EINVAL, "not a live batch (destroyed, or never created)");
  return WH2WAV_OK;
}

void free_batch(wh2wav_batch_s* b) {
  release_batch(b);
  delete b;
}

int plan_batch_body(const wh2wav_desc* descs, int count, wh2wav_batch_t* out) {
  if (!out) return fail(WH2WAV_EINVAL, "out is NULL");
  *out = nullptr;
  if (!descs || count <= 0) return fail(WH2WAV_EINVAL, "need at least one descriptor");
  // owned by `hold` until it is handed out; free_batch releases every plan made so far
  std::unique_ptr<wh2wav_batch_s, void (*)(wh2wav_batch_s*)> hold(new wh2wav_batch_s(), free_batch);
  wh2wav_batch_s* b = hold.get();
  for (int i = 0; i < count; ++i) {
    wh2wav_plan_t p = nullptr;
    int rc = wh2wav_plan(&descs[i], &p);
    if (rc != WH2WAV_OK) return fail(rc, "instance " + std::to_string(i) + ": " + wh2wav_last_error());
    b->plans.push_back(p);
    b->shape.push_back(wh2wav::plan_shape(p));
    size_t bytes = 0;
    wh2wav_workspace_size(p, &bytes);
    b->ws_off.push_back(b->ws_total);
    b->ws_total += (bytes + kAlign - 1) / kAlign * kAlign;
  }
  // the fused programs of the eligible instances, per element type and direction
  std::vector<wh2wav::PlanView> views;
  for (auto* p : b->plans) views.push_back(wh2wav::plan_view(p));
  b->in_kernel.assign(views.size(), 0);
  for (int d = 0; d < 2; ++d) {
    std::vector<int> members;
    for (size_t i = 0; i < views.size(); ++i)
      if (views[i].dtype == d && wh2wav_fused::eligible(views[i])) members.push_back(int(i)), b->in_kernel[i] = 1;
    if (members.empty()) continue;
    for (int dir = 0; dir < 2; ++dir) {
      int rc = wh2wav_fused::build(views, b->ws_off, members, d, dir, &b->prog[d][dir]);
      if (rc) return rc;
    }
  }
  hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int k = 0; k < kMaxBranches && e == hipSuccess; ++k) {
    e = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) return fail(WH2WAV_EHIP, std::string("batch streams: ") + hipGetErrorString(e));
  wh2wav::handle_add(b);
  *out = hold.release();
  return WH2WAV_OK;
}

int batch_workspace_size_body(wh2wav_batch_t b, size_t* bytes) {
  if (int rc = check_batch(b)) return rc;
  if (!bytes) return fail(WH2WAV_EINVAL, "NULL argument");
  *bytes = b->ws_total;
  return WH2WAV_OK;
}

int forward_batch_body(wh2wav_batch_t b, const void* const* xs, void* const* ys, void* ws, void* stream) {
  if (int rc = check_batch(b)) return rc;
  return run(b, 0, xs, ys, ws, stream);
}

int adjoint_batch_body(wh2wav_batch_t b, const void* const* ys, void* const* xs, void* ws, void* stream) {
  if (int rc = check_batch(b)) return rc;
  return run(b, 1, ys, xs, ws, stream);
}

int batch_schedule_body(wh2wav_batch_t b, int* branches, int* order) {
  if (int rc = check_batch(b)) return rc;
  if (!branches || !order) return fail(WH2WAV_EINVAL, "NULL argument");
  *branches = b->branches;
  *order = b->order;
  return WH2WAV_OK;
}

int batch_set_schedule_body(wh2wav_batch_t b, int branches, int order) {
  if (int rc = check_batch(b)) return rc;
  if (branches < 1 || branches > kMaxBranches || (order != 0 && order != 1))
    return fail(WH2WAV_EINVAL, "branches must be 1..8 and order 0 or 1");
  b->branches = branches;
  b->order = order;
  return WH2WAV_OK;
}

int batch_tune_body(wh2wav_batch_t b, const void* const* xs, void* const* ys, void* const* xa, void* ws,
                      void* stream, int reps, float* best_ms) {
  if (int rc = check_batch(b)) return rc;
  if (reps < 1) return fail(WH2WAV_EINVAL, "reps must be >= 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  HIP_B(hipEventCreate(&t0));
  hipError_t he = hipEventCreate(&t1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(t0);
    return fail(WH2WAV_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(he));
  }
  const int cand_b[] = {1, 2, 4, 8};
  float best = -1.f;
  int bb = b->branches, bo = b->order, rc = WH2WAV_OK;
  for (int order = 0; order < 2 && rc == WH2WAV_OK; ++order) {
    for (int nb : cand_b) {
      b->branches = nb;
      b->order = order;
      // first pair captures and warms up; then `reps` timed pairs
      rc = run(b, 0, xs, ys, ws, stream);
      if (rc == WH2WAV_OK) rc = run(b, 1, ys, xa, ws, stream);
      if (rc) break;
      he = hipEventRecord(t0, st);
      for (int r = 0; r < reps && rc == WH2WAV_OK && he == hipSuccess; ++r) {
        rc = run(b, 0, xs, ys, ws, stream);
        if (rc == WH2WAV_OK) rc = run(b, 1, ys, xa, ws, stream);
      }
      if (he == hipSuccess) he = hipEventRecord(t1, st);
      if (he == hipSuccess) he = hipEventSynchronize(t1);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, t0, t1);
      if (he != hipSuccess) rc = fail(WH2WAV_EHIP, std::string("tune timing: ") + hipGetErrorString(he));
      if (rc) break;
      ms /= float(reps);
      if (best < 0.f || ms < best) best = ms, bb = nb, bo = order;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  b->branches = bb;
  b->order = bo;
  if (best_ms) *best_ms = best;
  return rc;
}

int batch_set_mode_body(wh2wav_batch_t b, int mode) {
  if (int rc = check_batch(b)) return rc;
  if (mode != WH2WAV_BATCH_BRANCHES && mode != WH2WAV_BATCH_FUSED)
    return fail(WH2WAV_EINVAL, "mode must be WH2WAV_BATCH_BRANCHES or WH2WAV_BATCH_FUSED");
  b->mode = mode;
  return WH2WAV_OK;
}

int batch_mode_body(wh2wav_batch_t b, int* mode, int* fused_instances, int* fused_launches) {
  if (int rc = check_batch(b)) return rc;
  if (!mode) return fail(WH2WAV_EINVAL, "mode is NULL");
  *mode = b->mode;
  if (fused_instances) *fused_instances = int(std::count(b->in_kernel.begin(), b->in_kernel.end(), 1));
  if (fused_launches) {
    *fused_launches = 0;
    for (auto& pd : b->prog) *fused_launches += int(pd[0].rounds.size());
  }
  return WH2WAV_OK;
}

int destroy_batch_body(wh2wav_batch_t b) {
  if (!b) return WH2WAV_OK;
  if (!wh2wav::handle_remove(b)) return fail(WH2WAV_EINVAL, "not a live batch (destroyed twice, or never created)");
  free_batch(b);
  return WH2WAV_OK;
}

}  // namespace

extern "C" {

int wh2wav_plan_batch(const wh2wav_desc* descs, int count, wh2wav_batch_t* out) {
  return wh2wav::guarded([&] { return plan_batch_body(descs, count, out); });
}

int wh2wav_batch_workspace_size(wh2wav_batch_t b, size_t* bytes) {
  return wh2wav::guarded([&] { return batch_workspace_size_body(b, bytes); });
}

int wh2wav_forward_batch(wh2wav_batch_t b, const void* const* xs, void* const* ys, void* ws, void* stream) {
  return wh2wav::guarded([&] { return forward_batch_body(b, xs, ys, ws, stream); });
}

int wh2wav_adjoint_batch(wh2wav_batch_t b, const void* const* ys, void* const* xs, void* ws, void* stream) {
  return wh2wav::guarded([&] { return adjoint_batch_body(b, ys, xs, ws, stream); });
}

int wh2wav_batch_schedule(wh2wav_batch_t b, int* branches, int* order) {
  return wh2wav::guarded([&] { return batch_schedule_body(b, branches, order); });
}

int wh2wav_batch_set_schedule(wh2wav_batch_t b, int branches, int order) {
  return wh2wav::guarded([&] { return batch_set_schedule_body(b, branches, order); });
}

int wh2wav_batch_tune(wh2wav_batch_t b, const void* const* xs, void* const* ys, void* const* xa, void* ws,
                      void* stream, int reps, float* best_ms) {
  return wh2wav::guarded([&] { return batch_tune_body(b, xs, ys, xa, ws, stream, reps, best_ms); });
}

int wh2wav_batch_set_mode(wh2wav_batch_t b, int mode) {
  return wh2wav::guarded([&] { return batch_set_mode_body(b, mode); });
}

int wh2wav_batch_mode(wh2wav_batch_t b, int* mode, int* fused_instances, int* fused_launches) {
  return wh2wav::guarded([&] { return batch_mode_body(b, mode, fused_instances, fused_launches); });
}

int wh2wav_destroy_batch(wh2wav_batch_t b) {
  return wh2wav::guarded([&] { return destroy_batch_body(b); });
}

}  // extern "C"
