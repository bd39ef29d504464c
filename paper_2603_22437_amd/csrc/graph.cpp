// HIP-graph capture of evaluation calls (hck_graph_*): the calls a caller
// makes on one or more contexts between hck_graph_begin and hck_graph_end are
// recorded into one HIP graph, with each context's calls on a branch of their
// own, and replayed by one hipGraphLaunch.  A window pipeline issues hundreds
// to thousands of launches, most of them short at the low levels it runs on;
// a replay issues them without the host in the loop, and windows of
// different rings (one context each) run side by side on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.h"

using namespace hck;

struct hck_graph {
  std::vector<hck_context *> ctxs;  // ctxs[0]: the capture's origin stream
  // per context: the allocation mark of the capture (buffers allocated
  // before it may be read) and how much of the context's log of released
  // old buffers has been checked
  std::vector<uint64_t> mark, checked;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipEvent_t> events;   // [n]: order events of the launch's fork and join
};

namespace {

// the capture in progress on a context group (at most one per process
// thread: HIP's thread-local capture mode)
struct Capture {
  std::vector<hck_context *> ctxs;
  std::vector<hipEvent_t> events;
};
thread_local Capture *g_capture = nullptr;

void destroy_events(std::vector<hipEvent_t> &ev) {
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  ev.clear();
}

int make_events(hck_context *ctx, std::vector<hipEvent_t> &ev, size_t n) {
  ev.assign(n, nullptr);
  for (auto &e : ev) HCK_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return HCK_OK;
}

void release_graph_exec(hck_graph *g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
  destroy_events(g->events);
}

// releases the graph when any of its contexts is destroyed: the executable
// graph goes, and the handle is detached from every context
void release_graph(void *p) {
  hck_graph *g = static_cast<hck_graph *>(p);
  if (!g->ctxs.empty()) (void)hipSetDevice(g->ctxs[0]->device);
  // a replay in flight still reads the executable graph
  for (hck_context *c : g->ctxs)
    if (c->stream) (void)hipStreamSynchronize(c->stream);
  release_graph_exec(g);
  for (hck_context *c : g->ctxs) untrack(c, g);
  g->ctxs.clear();
}

void end_capture_flags(Capture *cap) {
  for (hck_context *c : cap->ctxs) c->capturing = false;
}

}  // namespace

namespace hck {
// a context destroyed while its calls are captured: the capture ends and its
// graph is discarded
void abort_capture(hck_context *ctx) {
  Capture *cap = g_capture;
  if (!cap || std::find(cap->ctxs.begin(), cap->ctxs.end(), ctx) == cap->ctxs.end()) return;
  g_capture = nullptr;
  end_capture_flags(cap);
  hipGraph_t dead = nullptr;
  (void)hipStreamEndCapture(cap->ctxs[0]->stream, &dead);
  if (dead) (void)hipGraphDestroy(dead);
  (void)hipGetLastError();
  destroy_events(cap->events);
  delete cap;
}
}  // namespace hck

extern "C" {

int hck_graph_begin(hck_context *const *ctxs, uint32_t n) {
  if (!ctxs || n == 0) return set_error(HCK_EINVAL, "no context to capture");
  if (g_capture) return set_error(HCK_EINVAL, "a graph capture is already open on this thread");
  for (uint32_t i = 0; i < n; i++) {
    hck_context *c = ctxs[i];
    if (!c) return set_error(HCK_EINVAL, "null context");
    if (c->broken) return set_error(HCK_EDEVICE, "context unusable after an earlier HIP error");
    if (!c->stream)
      return set_error(HCK_EINVAL, "graph capture needs a context on a created stream, not "
                                   "the null stream (hck_context_set_stream)");
    if (c->timing || c->capturing)
      return set_error(HCK_EINVAL, "context is timing or already capturing");
    if (c->device != ctxs[0]->device) return set_error(HCK_EINVAL, "contexts on different GPUs");
    for (uint32_t j = 0; j < i; j++)
      if (ctxs[j] == c || ctxs[j]->stream == c->stream)
        return set_error(HCK_EINVAL, "contexts must be distinct and on distinct streams");
  }
  hck_context *c0 = ctxs[0];
  HCK_HIP(c0, hipSetDevice(c0->device));
  auto *cap = new Capture();
  cap->ctxs.assign(ctxs, ctxs + n);
  int rc = make_events(c0, cap->events, 1);
  if (!rc) {
    const hipError_t e = hipStreamBeginCapture(c0->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) rc = check_hip(c0, e, "hipStreamBeginCapture");
  }
  // the other contexts' streams join the capture behind a fork event
  if (!rc && n > 1) {
    hipError_t e = hipEventRecord(cap->events[0], c0->stream);
    for (uint32_t i = 1; i < n && e == hipSuccess; i++)
      e = hipStreamWaitEvent(ctxs[i]->stream, cap->events[0], 0);
    if (e != hipSuccess) {
      rc = check_hip(c0, e, "fork of the captured streams");
      hipGraph_t dead = nullptr;
      (void)hipStreamEndCapture(c0->stream, &dead);
      if (dead) (void)hipGraphDestroy(dead);
    }
  }
  if (rc) {
    destroy_events(cap->events);
    delete cap;
    return rc;
  }
  for (hck_context *c : cap->ctxs) c->capturing = true;
  g_capture = cap;
  return HCK_OK;
}

int hck_graph_end(hck_context *const *ctxs, uint32_t n, hck_graph **out) {
  if (out) *out = nullptr;
  Capture *cap = g_capture;
  if (!cap) return set_error(HCK_EINVAL, "no graph capture open on this thread");
  if (!ctxs || n != cap->ctxs.size() || !std::equal(ctxs, ctxs + n, cap->ctxs.begin()))
    return set_error(HCK_EINVAL, "contexts differ from those of hck_graph_begin");
  g_capture = nullptr;
  end_capture_flags(cap);
  hck_context *c0 = cap->ctxs[0];
  int rc = HCK_OK;
  // join: the origin stream waits for every other branch
  std::vector<hipEvent_t> joins;
  if (n > 1) rc = make_events(c0, joins, n - 1);
  for (uint32_t i = 1; i < n && !rc; i++) {
    hipError_t e = hipEventRecord(joins[i - 1], ctxs[i]->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(c0->stream, joins[i - 1], 0);
    if (e != hipSuccess) rc = check_hip(c0, e, "join of the captured streams");
  }
  hipGraph_t graph = nullptr;
  const hipError_t e_end = hipStreamEndCapture(c0->stream, &graph);
  if (!rc && e_end != hipSuccess)
    rc = set_error(HCK_EINVAL, std::string("graph capture failed (a captured call made a "
                                           "call that cannot be captured): ") +
                                   hipGetErrorString(e_end));
  (void)hipGetLastError();
  destroy_events(joins);
  destroy_events(cap->events);
  delete cap;
  if (!rc && !out) rc = set_error(HCK_EINVAL, "null output");
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  auto *g = new hck_graph();
  g->ctxs.assign(ctxs, ctxs + n);
  g->graph = graph;
  for (hck_context *c : g->ctxs) {
    g->mark.push_back(c->alloc_counter + 1);
    g->checked.push_back(c->freed_old.size());
    c->graph_mark = std::max(c->graph_mark, c->alloc_counter + 1);
  }
  hipError_t e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e == hipSuccess) rc = make_events(c0, g->events, n);
  else rc = check_hip(c0, e, "hipGraphInstantiate");
  if (rc) {
    release_graph_exec(g);
    delete g;
    return rc;
  }
  for (hck_context *c : g->ctxs) track(c, g, release_graph);
  *out = g;
  return HCK_OK;
}

int hck_graph_launch(hck_graph *g) {
  if (!g) return set_error(HCK_EINVAL, "null graph");
  if (!g->exec) return set_error(HCK_EINVAL, "graph released with one of its contexts");
  for (size_t i = 0; i < g->ctxs.size(); i++) {
    hck_context *c = g->ctxs[i];
    if (c->broken) return set_error(HCK_EDEVICE, "context unusable after an earlier HIP error");
    if (c->capturing) return set_error(HCK_EINVAL, "graph launch during a capture");
    for (size_t k = g->checked[i]; k < c->freed_old.size(); k++)
      if (c->freed_old[k] < g->mark[i])
        return set_error(HCK_EINVAL, "a device buffer that existed at the capture was given "
                                     "back since (the graph may read it); capture again");
  }
  // nothing released since the last check concerns this graph
  for (size_t i = 0; i < g->ctxs.size(); i++) g->checked[i] = g->ctxs[i]->freed_old.size();
  hck_context *c0 = g->ctxs[0];
  HCK_HIP(c0, hipSetDevice(c0->device));
  const size_t n = g->ctxs.size();
  // the replay follows earlier work on every context's stream, and later
  // work on every stream follows the replay
  for (size_t i = 1; i < n; i++) {
    HCK_HIP(c0, hipEventRecord(g->events[i], g->ctxs[i]->stream));
    HCK_HIP(c0, hipStreamWaitEvent(c0->stream, g->events[i], 0));
  }
  HCK_HIP(c0, hipGraphLaunch(g->exec, c0->stream));
  if (n > 1) {
    HCK_HIP(c0, hipEventRecord(g->events[0], c0->stream));
    for (size_t i = 1; i < n; i++)
      HCK_HIP(c0, hipStreamWaitEvent(g->ctxs[i]->stream, g->events[0], 0));
  }
  return HCK_OK;
}

int hck_graph_info(const hck_graph *g, uint32_t *contexts, size_t *nodes) {
  if (!g) return set_error(HCK_EINVAL, "null graph");
  if (contexts) *contexts = (uint32_t)g->ctxs.size();
  if (nodes) {
    *nodes = 0;
    if (g->graph && hipGraphGetNodes(g->graph, nullptr, nodes) != hipSuccess)
      return set_error(HCK_EDEVICE, "hipGraphGetNodes failed");
  }
  return HCK_OK;
}

int hck_graph_destroy(hck_graph *g) {
  if (!g) return HCK_OK;
  if (!g->ctxs.empty()) release_graph(g);
  delete g;
  return HCK_OK;
}

}  // extern "C"
