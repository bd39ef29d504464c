// Serving runtime: encrypted windows from many tenants evaluated with
// continuous batching (the streaming deployment the paper leaves to future
// work, section 7; the cloud side of section 3.3 serving several clients).
//
// One worker thread owns the context.  Callers submit requests (one encrypted
// window of a registered tenant, in interchange form) at any time; the worker
//  * admits them in arrival order while the HBM budget allows: a tenant's
//    evaluation keys are loaded from host memory when it has none resident
//    (least recently used idle tenants are evicted to make room, never one
//    with admitted work), on a copy stream of their own so that the transfer
//    overlaps the evaluation already queued.  At most kMaxUploads tenants'
//    keys are in transfer at once; requests of resident tenants are admitted
//    past those waiting for an upload slot;
//  * launches admitted windows whose keys have arrived as soon as fewer than
//    two batches are queued on the device, up to max_batch windows of one
//    pipeline per batch (windows of different tenants share key-switch
//    batches, each with its own keys), so that requests arriving while others
//    run join the next batch and a key transfer never stalls the evaluation
//    of resident tenants;
//  * completes batches as their events fire, copying the results to the
//    caller's buffers and releasing their footprint.
// All device work is stream-ordered on the context stream; the host never
// waits for the device except on teardown.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "admission.h"
#include "internal.h"

using namespace hck;

#define TRY(expr)         \
  do {                    \
    int _rc = (expr);     \
    if (_rc) return _rc;  \
  } while (0)

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Tenant {
  uint32_t kind = 0;
  const void *plan = nullptr;
  std::vector<int32_t> steps;
  std::vector<const uint64_t *> gk_host;
  const uint64_t *rlk_host = nullptr;
  uint64_t key_bytes = 0;
  // resident keys (device) and the copy that filled them
  hck_galois_keys *gks = nullptr;
  hck_switch_key *rlk = nullptr;
  hipEvent_t copied = nullptr;
  bool converted = false;
};

struct Request {
  uint64_t id = 0;
  uint32_t tenant = 0, level = 0;
  double scale = 0;
  std::vector<uint64_t> in;  // re then im, [2][level+1][N] each
  uint64_t *out_user = nullptr;
  size_t out_cap = 0;
  uint64_t extra = 0;  // admitted working set
  int slot = -1;       // pinned staging slot
  hck_server_result res{};
  hck_ciphertext *ct_in[2] = {nullptr, nullptr};
  hck_ciphertext *ct_out[4] = {nullptr, nullptr, nullptr, nullptr};
};

struct Batch {
  std::vector<Request *> reqs;
  hipEvent_t done = nullptr;
};

uint32_t outputs_of(uint32_t kind) { return kind == HCK_SERVE_VITAL ? 4 : 1; }

// tenants whose keys may be in transfer at once
constexpr size_t kMaxUploads = 2;

}  // namespace

struct hck_server {
  hck_context *ctx = nullptr;
  hck_server_config cfg{};
  hipStream_t copy = nullptr;
  Residency res{0};
  size_t slot_in_words = 0, slot_out_words = 0;
  std::vector<uint64_t *> slots_in, slots_out;
  std::vector<int> free_slots;
  std::vector<hipEvent_t> free_events;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> incoming;                          // guarded by mu
  std::deque<std::pair<uint32_t, Tenant>> new_tenants;     // guarded by mu
  std::set<uint32_t> registered;                           // guarded by mu
  std::deque<hck_server_result> finished;                  // guarded by mu
  uint64_t outstanding = 0;                                // guarded by mu
  hck_server_stats stats{};                                // guarded by mu
  bool stop = false;                                       // guarded by mu

  // worker-only state
  std::map<uint32_t, Tenant> tenants;
  std::deque<Request *> pending, admitted;
  std::deque<Batch> inflight;
  std::vector<uint32_t> uploading;  // tenants whose key transfer may be running
  std::thread worker;
  int fatal = HCK_OK;
};

namespace {

// releases a tenant's device keys, stream-ordered after every use (uses are
// on the context stream, which also waits for the upload when it never did)
void free_key(hck_server *s, hck_switch_key *k) {
  if (!k) return;
  if (k->data) (void)hipFreeAsync(k->data, s->ctx->stream);
  delete k;
}

void drop_keys(hck_server *s, Tenant &t) {
  if (t.copied && !t.converted) (void)hipStreamWaitEvent(s->ctx->stream, t.copied, 0);
  if (t.gks) {
    for (auto &kv : t.gks->keys) free_key(s, kv.second);
    delete t.gks;
  }
  free_key(s, t.rlk);
  if (t.copied) (void)hipEventDestroy(t.copied);
  t.gks = nullptr;
  t.rlk = nullptr;
  t.copied = nullptr;
  t.converted = false;
}

// device copies of a tenant's keys, allocated and filled on the copy stream
// (their own stream-ordered allocations, whatever allocator the context uses;
// free_key releases them)
int load_keys(hck_server *s, Tenant &t) {
  hck_context *ctx = s->ctx;
  const size_t words = (size_t)ctx->dnum * 2 * (ctx->L + ctx->K) * ctx->n;
  auto one = [&](const uint64_t *host, hck_switch_key **out) -> int {
    hck_switch_key *k = new hck_switch_key();
    k->ctx = ctx;
    hipError_t e = hipMallocAsync((void **)&k->data, words * 8, s->copy);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      delete k;
      return set_error(HCK_ENOMEM, "device allocation for tenant keys failed");
    }
    e = hipMemcpyAsync(k->data, host, words * 8, hipMemcpyHostToDevice, s->copy);
    *out = k;
    return e == hipSuccess ? HCK_OK : check_hip(ctx, e, "key upload");
  };
  t.gks = new hck_galois_keys();
  t.gks->ctx = ctx;
  int rc = HCK_OK;
  for (size_t i = 0; !rc && i < t.steps.size(); i++) {
    hck_switch_key *k = nullptr;
    rc = one(t.gk_host[i], &k);
    if (k) t.gks->keys[galois_of_step(ctx, t.steps[i])] = k;
  }
  if (!rc) rc = one(t.rlk_host, &t.rlk);
  if (!rc) {
    hipError_t e = hipEventCreateWithFlags(&t.copied, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(t.copied, s->copy);
    if (e != hipSuccess) rc = check_hip(ctx, e, "key upload event");
  }
  if (rc) {
    // the partial upload must finish before its memory is released
    (void)hipStreamSynchronize(s->copy);
    drop_keys(s, t);
  }
  t.converted = false;
  return rc;
}

// the context stream waits for the copy, then converts the keys in place
int convert_keys(hck_server *s, Tenant &t) {
  if (t.converted) return HCK_OK;
  hck_context *ctx = s->ctx;
  HCK_HIP(ctx, hipStreamWaitEvent(ctx->stream, t.copied, 0));
  for (auto &kv : t.gks->keys) {
    int rc = key_rows_to_internal(ctx, kv.second->data);
    if (rc) return rc;
  }
  int rc = key_rows_to_internal(ctx, t.rlk->data);
  if (rc) return rc;
  t.converted = true;
  return HCK_OK;
}

// true once a tenant's key transfer has completed (or its keys are in use)
bool keys_arrived(Tenant &t) {
  if (t.converted || !t.copied) return true;
  return hipEventQuery(t.copied) != hipErrorNotReady;
}

uint64_t window_bytes(const hck_context *ctx, uint32_t kind) {
  // inputs (2) and outputs, each [2][L][N] on the device
  return (uint64_t)(2 + outputs_of(kind)) * 2 * ctx->L * ctx->n * 8;
}

// completes a request: results to the caller's buffer, footprint released
void finish(hck_server *s, Request *r, int status) {
  r->res.status = status;
  r->res.t_done = now_s();
  if (r->slot >= 0) {
    if (status == HCK_OK) {
      size_t words = 0;
      for (uint32_t i = 0; i < r->res.n_out; i++)
        words += (size_t)2 * (r->res.out_level[i] + 1) * s->ctx->n;
      std::memcpy(r->out_user, s->slots_out[r->slot], words * 8);
    }
    s->free_slots.push_back(r->slot);
  }
  if (r->extra) s->res.release(r->tenant, r->extra);
  std::lock_guard<std::mutex> g(s->mu);
  s->finished.push_back(r->res);
  s->outstanding--;
  if (status == HCK_OK) s->stats.completed++;
  else s->stats.failed++;
  delete r;
  s->cv_done.notify_all();
}

// enqueues one batch: inputs, pipeline, outputs, completion event
int launch(hck_server *s, std::vector<Request *> &reqs, Batch &b) {
  hck_context *ctx = s->ctx;
  const uint32_t n = (uint32_t)reqs.size();
  Tenant &t0 = s->tenants[reqs[0]->tenant];
  std::vector<const hck_ciphertext *> re(n), im(n);
  std::vector<const hck_galois_keys *> gks(n);
  std::vector<const hck_switch_key *> rlk(n);
  std::vector<hck_ciphertext *> outs;
  const double t = now_s();
  for (uint32_t k = 0; k < n; k++) {
    Request *r = reqs[k];
    Tenant &tn = s->tenants[r->tenant];
    TRY(convert_keys(s, tn));
    r->slot = s->free_slots.back();
    s->free_slots.pop_back();
    uint64_t *pin = s->slots_in[r->slot];
    std::memcpy(pin, r->in.data(), r->in.size() * 8);
    std::vector<uint64_t>().swap(r->in);
    const size_t half = (size_t)2 * (r->level + 1) * ctx->n;
    for (int i = 0; i < 2; i++) {
      r->ct_in[i] = pool_get(ctx);
      TRY(ct_from_host_async(ctx, r->ct_in[i], pin + i * half, 2, r->level, r->scale));
    }
    for (uint32_t i = 0; i < outputs_of(tn.kind); i++) {
      r->ct_out[i] = pool_get(ctx);
      outs.push_back(r->ct_out[i]);
    }
    re[k] = r->ct_in[0];
    im[k] = r->ct_in[1];
    gks[k] = tn.gks;
    rlk[k] = tn.rlk;
    r->res.t_launch = t;
    r->res.batch = n;
  }
  if (t0.kind == HCK_SERVE_VITAL) {
    TRY(vital_eval_batch(ctx, (const hck_vital_plan *)t0.plan, re.data(), im.data(), n,
                         gks.data(), rlk.data(), outs.data()));
  } else {
    for (uint32_t k = 0; k < n; k++)
      TRY(hck_gesture_eval(ctx, (const hck_gesture_plan *)t0.plan, re[k], im[k], gks[k],
                           rlk[k], reqs[k]->ct_out[0]));
  }
  for (Request *r : reqs) {
    const Tenant &tn = s->tenants[r->tenant];
    size_t off = 0, need = 0;
    r->res.n_out = outputs_of(tn.kind);
    for (uint32_t i = 0; i < r->res.n_out; i++)
      need += (size_t)2 * (r->ct_out[i]->level + 1) * ctx->n;
    if (need > r->out_cap) return set_error(HCK_EINVAL, "output buffer too small");
    for (uint32_t i = 0; i < r->res.n_out; i++) {
      hck_ciphertext *c = r->ct_out[i];
      r->res.out_level[i] = c->level;
      r->res.out_scale[i] = c->scale;
      TRY(ct_to_host_async(ctx, c, s->slots_out[r->slot] + off));
      off += (size_t)2 * (c->level + 1) * ctx->n;
    }
    // the stream orders every later use of these after the copies above
    for (int i = 0; i < 2; i++) pool_put(ctx, r->ct_in[i]);
    for (uint32_t i = 0; i < r->res.n_out; i++) pool_put(ctx, r->ct_out[i]);
    std::fill(r->ct_in, r->ct_in + 2, nullptr);
    std::fill(r->ct_out, r->ct_out + 4, nullptr);
  }
  if (s->free_events.empty()) {
    hipEvent_t e;
    HCK_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    s->free_events.push_back(e);
  }
  b.done = s->free_events.back();
  s->free_events.pop_back();
  HCK_HIP(ctx, hipEventRecord(b.done, ctx->stream));
  b.reqs = reqs;
  return HCK_OK;
}

// completes the oldest batches whose events have fired; true if any did
bool complete(hck_server *s, bool block) {
  bool any = false;
  while (!s->inflight.empty()) {
    Batch &b = s->inflight.front();
    hipError_t e = block ? hipEventSynchronize(b.done) : hipEventQuery(b.done);
    if (e == hipErrorNotReady) break;
    const int st = e == hipSuccess ? HCK_OK : check_hip(s->ctx, e, "batch completion");
    for (Request *r : b.reqs) finish(s, r, st);
    s->free_events.push_back(b.done);
    s->inflight.pop_front();
    any = true;
    if (block) break;
  }
  return any;
}

// admits pending requests in arrival order while the budget and the in-flight
// limit allow; a request whose tenant's keys must be loaded waits for an
// upload slot without holding back later requests of resident tenants.  True
// if any was admitted.
bool admit(hck_server *s) {
  bool any = false;
  const size_t cap = s->cfg.max_inflight;
  size_t flying = s->admitted.size();
  for (auto &b : s->inflight) flying += b.reqs.size();
  s->uploading.erase(std::remove_if(s->uploading.begin(), s->uploading.end(),
                                    [&](uint32_t t) { return keys_arrived(s->tenants[t]); }),
                     s->uploading.end());
  for (auto pit = s->pending.begin(); pit != s->pending.end() && flying < cap;) {
    Request *r = *pit;
    auto it = s->tenants.find(r->tenant);
    if (!s->res.resident(r->tenant) && s->uploading.size() >= kMaxUploads) {
      ++pit;
      continue;
    }
    const uint64_t extra = window_bytes(s->ctx, it->second.kind);
    std::vector<uint32_t> evict;
    bool load = false;
    const Residency::Decision d = s->res.admit(r->tenant, extra, evict, load);
    if (d == Residency::kWait) {
      ++pit;
      continue;
    }
    pit = s->pending.erase(pit);
    r->res.t_admit = now_s();
    if (d == Residency::kReject) {
      finish(s, r, HCK_ENOMEM);
      continue;
    }
    r->extra = extra;
    for (uint32_t v : evict) {
      drop_keys(s, s->tenants[v]);
      std::lock_guard<std::mutex> g(s->mu);
      s->stats.evictions++;
    }
    if (load) {
      const int rc = load_keys(s, it->second);
      if (rc) {
        const uint32_t tenant = r->tenant;
        finish(s, r, rc);  // releases the request's footprint
        s->res.evict(tenant);
        continue;
      }
      s->uploading.push_back(r->tenant);
      r->res.key_load = 1;
      std::lock_guard<std::mutex> g(s->mu);
      s->stats.key_loads++;
      s->stats.key_bytes_loaded += it->second.key_bytes;
    }
    s->admitted.push_back(r);
    flying++;
    any = true;
  }
  std::lock_guard<std::mutex> g(s->mu);
  s->stats.resident_bytes = s->res.used();
  return any;
}

// launches one batch of admitted windows (the oldest request's pipeline)
bool launch_next(hck_server *s) {
  if (s->admitted.empty() || s->inflight.size() >= 2) return false;
  // the oldest admitted request whose keys have arrived sets the pipeline
  auto ready = [&](Request *r) { return keys_arrived(s->tenants[r->tenant]); };
  auto fit = std::find_if(s->admitted.begin(), s->admitted.end(), ready);
  if (fit == s->admitted.end()) return false;
  Request *first = *fit;
  const Tenant &t0 = s->tenants[first->tenant];
  std::vector<Request *> reqs;
  for (auto it = fit; it != s->admitted.end() && reqs.size() < s->cfg.max_batch;) {
    const Tenant &t = s->tenants[(*it)->tenant];
    if (t.kind == t0.kind && t.plan == t0.plan && (*it)->level == first->level && ready(*it)) {
      reqs.push_back(*it);
      it = s->admitted.erase(it);
    } else {
      ++it;
    }
  }
  Batch b;
  const int rc = launch(s, reqs, b);
  if (rc) {
    for (Request *r : reqs) {
      for (auto *&c : r->ct_in)
        if (c) pool_put(s->ctx, c), c = nullptr;
      for (auto *&c : r->ct_out)
        if (c) pool_put(s->ctx, c), c = nullptr;
      finish(s, r, rc);
    }
    if (s->ctx->broken) s->fatal = rc;
    return true;
  }
  s->inflight.push_back(b);
  std::lock_guard<std::mutex> g(s->mu);
  s->stats.batches++;
  s->stats.windows += reqs.size();
  return true;
}

void worker_main(hck_server *s) {
  (void)hipSetDevice(s->ctx->device);
  for (;;) {
    bool stopping;
    {
      std::unique_lock<std::mutex> g(s->mu);
      while (!s->new_tenants.empty()) {
        auto &nt = s->new_tenants.front();
        s->res.add_tenant(nt.first, nt.second.key_bytes);
        s->tenants[nt.first] = nt.second;
        s->new_tenants.pop_front();
      }
      while (!s->incoming.empty()) {
        s->pending.push_back(s->incoming.front());
        s->incoming.pop_front();
      }
      stopping = s->stop;
    }
    bool progress = complete(s, false);
    if (!s->fatal) {
      progress = admit(s) || progress;
      progress = launch_next(s) || progress;
    } else {
      // the context is unusable: fail everything not yet launched
      while (!s->pending.empty()) {
        finish(s, s->pending.front(), s->fatal);
        s->pending.pop_front();
      }
      while (!s->admitted.empty()) {
        finish(s, s->admitted.front(), s->fatal);
        s->admitted.pop_front();
      }
    }
    if (stopping && s->pending.empty() && s->admitted.empty() && s->inflight.empty()) break;
    if (!progress) {
      if (!s->inflight.empty() && s->pending.empty() && s->admitted.empty()) {
        // nothing else to do: wait for the oldest batch, but wake for arrivals
        std::unique_lock<std::mutex> g(s->mu);
        s->cv_work.wait_for(g, std::chrono::microseconds(200),
                            [&] { return !s->incoming.empty() || !s->new_tenants.empty(); });
      } else {
        std::unique_lock<std::mutex> g(s->mu);
        const bool busy = !s->inflight.empty() || !s->admitted.empty() || !s->pending.empty();
        s->cv_work.wait_for(g, std::chrono::microseconds(busy ? 200 : 2000),
                            [&] {
                              return !s->incoming.empty() || !s->new_tenants.empty() || s->stop;
                            });
      }
    }
  }
}

// stops the worker and releases every resource of the server; the server
// record stays, detached from its context (the context's destroy call runs
// this for servers still alive, before it releases the other handles, which
// the tenants' plans reference)
void server_shutdown(void *p) {
  hck_server *s = static_cast<hck_server *>(p);
  if (!s->ctx) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  s->worker.join();
  hck_context *ctx = s->ctx;
  (void)hipSetDevice(ctx->device);
  for (auto &kv : s->tenants) drop_keys(s, kv.second);
  s->tenants.clear();
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipStreamSynchronize(s->copy);
  for (auto *q : s->slots_in) (void)hipHostFree(q);
  for (auto *q : s->slots_out) (void)hipHostFree(q);
  s->slots_in.clear();
  s->slots_out.clear();
  for (auto e : s->free_events) (void)hipEventDestroy(e);
  s->free_events.clear();
  (void)hipStreamDestroy(s->copy);
  s->copy = nullptr;
  s->ctx = nullptr;
}

}  // namespace

extern "C" {

int hck_server_create(hck_context *ctx, const hck_server_config *cfg, hck_server **out) {
  if (!ctx || !cfg || !out) return set_error(HCK_EINVAL, "null argument");
  if (cfg->max_batch == 0 || cfg->max_batch > 64 || cfg->max_inflight == 0 ||
      cfg->max_inflight > 256)
    return set_error(HCK_EINVAL, "max_batch must be 1..64 and max_inflight 1..256");
  HCK_HIP(ctx, hipSetDevice(ctx->device));
  hck_server *s = new hck_server();
  s->ctx = ctx;
  s->cfg = *cfg;
  s->res = Residency(cfg->hbm_budget);
  s->slot_in_words = (size_t)2 * 2 * ctx->L * ctx->n;
  s->slot_out_words = (size_t)4 * 2 * ctx->L * ctx->n;
  hipError_t e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
  for (uint32_t i = 0; e == hipSuccess && i < cfg->max_inflight; i++) {
    uint64_t *a = nullptr, *b = nullptr;
    e = hipHostMalloc((void **)&a, s->slot_in_words * 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b, s->slot_out_words * 8, hipHostMallocDefault);
    if (a) s->slots_in.push_back(a);
    if (b) s->slots_out.push_back(b);
    s->free_slots.push_back((int)i);
  }
  if (e != hipSuccess) {
    const int rc = check_hip(nullptr, e, "server set-up");
    for (auto *p : s->slots_in) (void)hipHostFree(p);
    for (auto *p : s->slots_out) (void)hipHostFree(p);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    delete s;
    return rc;
  }
  s->stats.budget = cfg->hbm_budget;
  s->worker = std::thread(worker_main, s);
  track_server(ctx, s, server_shutdown);
  *out = s;
  return HCK_OK;
}

int hck_server_add_tenant(hck_server *s, uint32_t tenant, uint32_t kind, const void *plan,
                          const int32_t *steps, const uint64_t *const *gk_words, uint32_t n_steps,
                          const uint64_t *rlk_words) {
  if (!s || !plan || !rlk_words || (n_steps && (!steps || !gk_words)))
    return set_error(HCK_EINVAL, "null argument");
  if (!s->ctx) return set_error(HCK_EINVAL, "the server's context was destroyed");
  if (kind != HCK_SERVE_VITAL && kind != HCK_SERVE_GESTURE)
    return set_error(HCK_EINVAL, "unknown pipeline kind");
  hck_context *ctx = s->ctx;
  // the pipeline's rotation steps must all have keys
  std::vector<int32_t> need(256);
  uint32_t nn = 0;
  int rc = kind == HCK_SERVE_VITAL
               ? hck_vital_required_steps(ctx, (const hck_vital_plan *)plan, need.data(), 256, &nn)
               : hck_gesture_required_steps(ctx, (const hck_gesture_plan *)plan, need.data(), 256,
                                            &nn);
  if (rc) return rc;
  std::set<uint32_t> have;
  for (uint32_t i = 0; i < n_steps; i++) {
    if (!gk_words[i]) return set_error(HCK_EINVAL, "null key words");
    have.insert(galois_of_step(ctx, steps[i]));
  }
  for (uint32_t i = 0; i < nn; i++)
    if (!have.count(galois_of_step(ctx, need[i])))
      return set_error(HCK_ENOKEY, "missing Galois key for step " + std::to_string(need[i]));
  Tenant t;
  t.kind = kind;
  t.plan = plan;
  t.steps.assign(steps, steps + n_steps);
  t.gk_host.assign(gk_words, gk_words + n_steps);
  t.rlk_host = rlk_words;
  t.key_bytes = (uint64_t)(n_steps + 1) * ctx->dnum * 2 * (ctx->L + ctx->K) * ctx->n * 8;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->registered.count(tenant)) return set_error(HCK_EINVAL, "tenant already registered");
  s->registered.insert(tenant);
  s->new_tenants.push_back({tenant, t});
  s->stats.tenants++;
  s->cv_work.notify_all();
  return HCK_OK;
}

int hck_server_submit(hck_server *s, uint64_t request, uint32_t tenant, const uint64_t *re_words,
                      const uint64_t *im_words, uint32_t level, double scale, uint64_t *out_words,
                      size_t out_capacity) {
  if (!s || !re_words || !im_words || !out_words) return set_error(HCK_EINVAL, "null argument");
  if (!s->ctx) return set_error(HCK_EINVAL, "the server's context was destroyed");
  hck_context *ctx = s->ctx;
  if (level >= ctx->L) return set_error(HCK_ELEVEL, "level beyond the chain");
  const size_t half = (size_t)2 * (level + 1) * ctx->n;
  Request *r = new Request();
  r->id = request;
  r->tenant = tenant;
  r->level = level;
  r->scale = scale;
  r->out_user = out_words;
  r->out_cap = out_capacity;
  r->in.resize(2 * half);
  std::memcpy(r->in.data(), re_words, half * 8);
  std::memcpy(r->in.data() + half, im_words, half * 8);
  // every row [ct][poly][limb] below its limb's prime
  bool ok = true;
  for (size_t row = 0; row < 4 * (size_t)(level + 1); row++) {
    const uint64_t q = ctx->mods[row % (level + 1)];
    const uint64_t *v = r->in.data() + row * ctx->n;
    uint64_t bad = 0;
    for (size_t c = 0; c < ctx->n; c++) bad |= (uint64_t)(v[c] >= q);
    ok = ok && !bad;
  }
  if (!ok) {
    delete r;
    return set_error(HCK_EINVAL, "residue not below its prime");
  }
  r->res.request = request;
  r->res.tenant = tenant;
  r->res.t_submit = now_s();
  std::lock_guard<std::mutex> g(s->mu);
  if (!s->registered.count(tenant)) {
    delete r;
    return set_error(HCK_EINVAL, "unknown tenant");
  }
  if (s->stop) {
    delete r;
    return set_error(HCK_EINVAL, "server is shutting down");
  }
  s->incoming.push_back(r);
  s->outstanding++;
  s->stats.submitted++;
  s->cv_work.notify_all();
  return HCK_OK;
}

int hck_server_poll(hck_server *s, uint32_t timeout_ms, hck_server_result *results, uint32_t cap,
                    uint32_t *n) {
  if (!s || !n || (cap && !results)) return set_error(HCK_EINVAL, "null argument");
  std::unique_lock<std::mutex> g(s->mu);
  if (s->finished.empty() && timeout_ms)
    s->cv_done.wait_for(g, std::chrono::milliseconds(timeout_ms),
                        [&] { return !s->finished.empty() || s->outstanding == 0; });
  uint32_t k = 0;
  while (k < cap && !s->finished.empty()) {
    results[k++] = s->finished.front();
    s->finished.pop_front();
  }
  *n = k;
  return HCK_OK;
}

int hck_server_stats_get(hck_server *s, hck_server_stats *out) {
  if (!s || !out) return set_error(HCK_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->stats;
  out->pending = s->outstanding;
  return HCK_OK;
}

int hck_server_destroy(hck_server *s) {
  if (!s) return HCK_OK;
  if (s->ctx) {
    untrack_server(s->ctx, s);
    server_shutdown(s);
  }
  delete s;
  return HCK_OK;
}

}  // extern "C"
