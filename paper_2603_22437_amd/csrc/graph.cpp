// HIP-graph capture of evaluation calls (hck_graph_*): the calls a caller
// makes on one or more contexts between hck_graph_begin and hck_graph_end are
// recorded, each context's calls into a graph of its own on the context's
// stream, and replayed together by hck_graph_launch.  A window pipeline
// issues hundreds of launches, most of them short at the low levels it runs
// on; a replay issues them without the host in the loop, and the contexts'
// replays (windows of different rings, or several groups of windows of one
// ring) run side by side on their streams.  One graph per stream, not one
// graph with a branch per context: replays of separate graphs on separate
// streams overlapped on the device, while the branches of one graph did not.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.h"

using namespace hck;

struct hck_graph {
  std::vector<hck_context *> ctxs;
  std::vector<hipGraph_t> graphs;        // [context]
  std::vector<hipGraphExec_t> execs;     // [context]
  // per context: the allocation mark of the capture (buffers allocated
  // before it may be read) and how much of the context's log of released
  // old buffers has been checked
  std::vector<uint64_t> mark, checked;
};

namespace {

// the capture in progress (HIP's thread-local capture mode: at most one
// group per host thread)
struct Capture {
  std::vector<hck_context *> ctxs;
};
thread_local Capture *g_capture = nullptr;

void release_graph_exec(hck_graph *g) {
  for (hipGraphExec_t e : g->execs)
    if (e) (void)hipGraphExecDestroy(e);
  for (hipGraph_t x : g->graphs)
    if (x) (void)hipGraphDestroy(x);
  g->execs.clear();
  g->graphs.clear();
}

// releases the graph when any of its contexts is destroyed: the executable
// graphs go, and the handle is detached from every context
void release_graph(void *p) {
  hck_graph *g = static_cast<hck_graph *>(p);
  if (!g->ctxs.empty()) (void)hipSetDevice(g->ctxs[0]->device);
  // a replay in flight still reads the executable graphs
  for (hck_context *c : g->ctxs)
    if (c->stream) (void)hipStreamSynchronize(c->stream);
  release_graph_exec(g);
  for (hck_context *c : g->ctxs) untrack(c, g);
  g->ctxs.clear();
}

// ends the capture on the first `n` streams of the group, discarding the
// graphs (failure paths)
void discard_captures(Capture *cap, size_t n) {
  for (size_t i = 0; i < n; i++) {
    hipGraph_t dead = nullptr;
    (void)hipStreamEndCapture(cap->ctxs[i]->stream, &dead);
    if (dead) (void)hipGraphDestroy(dead);
  }
  (void)hipGetLastError();
}

}  // namespace

namespace hck {
// a context destroyed while its calls are captured: the capture of the whole
// group ends and its graphs are discarded
void abort_capture(hck_context *ctx) {
  Capture *cap = g_capture;
  if (!cap || std::find(cap->ctxs.begin(), cap->ctxs.end(), ctx) == cap->ctxs.end()) return;
  g_capture = nullptr;
  for (hck_context *c : cap->ctxs) c->capturing = false;
  discard_captures(cap, cap->ctxs.size());
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
  HCK_HIP(ctxs[0], hipSetDevice(ctxs[0]->device));
  auto *cap = new Capture();
  cap->ctxs.assign(ctxs, ctxs + n);
  for (uint32_t i = 0; i < n; i++) {
    const hipError_t e = hipStreamBeginCapture(ctxs[i]->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      discard_captures(cap, i);
      delete cap;
      return check_hip(ctxs[i], e, "hipStreamBeginCapture");
    }
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
  for (hck_context *c : cap->ctxs) c->capturing = false;
  auto *g = new hck_graph();
  int rc = HCK_OK;
  for (uint32_t i = 0; i < n; i++) {
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(ctxs[i]->stream, &graph);
    if (e != hipSuccess && !rc)
      rc = set_error(HCK_EINVAL, std::string("graph capture failed (a recorded call made a "
                                             "call that cannot be captured): ") +
                                     hipGetErrorString(e));
    g->graphs.push_back(graph);
  }
  (void)hipGetLastError();
  delete cap;
  if (!rc && !out) rc = set_error(HCK_EINVAL, "null output");
  for (uint32_t i = 0; i < n && !rc; i++) {
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, g->graphs[i], nullptr, nullptr, 0);
    if (e != hipSuccess) rc = check_hip(ctxs[i], e, "hipGraphInstantiate");
    g->execs.push_back(exec);
  }
  if (rc) {
    release_graph_exec(g);
    delete g;
    return rc;
  }
  g->ctxs.assign(ctxs, ctxs + n);
  for (hck_context *c : g->ctxs) {
    g->mark.push_back(c->alloc_counter + 1);
    g->checked.push_back(c->freed_old.size());
    c->graph_mark = std::max(c->graph_mark, c->alloc_counter + 1);
    track(c, g, release_graph);
  }
  *out = g;
  return HCK_OK;
}

int hck_graph_launch(hck_graph *g) {
  if (!g) return set_error(HCK_EINVAL, "null graph");
  if (g->execs.empty()) return set_error(HCK_EINVAL, "graph released with one of its contexts");
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
  HCK_HIP(g->ctxs[0], hipSetDevice(g->ctxs[0]->device));
  for (size_t i = 0; i < g->ctxs.size(); i++)
    HCK_HIP(g->ctxs[i], hipGraphLaunch(g->execs[i], g->ctxs[i]->stream));
  return HCK_OK;
}

int hck_graph_info(const hck_graph *g, uint32_t *contexts, size_t *nodes) {
  if (!g) return set_error(HCK_EINVAL, "null graph");
  if (contexts) *contexts = (uint32_t)g->ctxs.size();
  if (nodes) {
    *nodes = 0;
    for (hipGraph_t x : g->graphs) {
      size_t k = 0;
      if (x && hipGraphGetNodes(x, nullptr, &k) != hipSuccess)
        return set_error(HCK_EDEVICE, "hipGraphGetNodes failed");
      *nodes += k;
    }
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
