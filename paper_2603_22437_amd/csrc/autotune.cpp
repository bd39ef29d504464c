// Autotuner of the key-switch schedule: how many key switches one launch
// sequence takes at each level.  Small batches leave the chip idle at low
// levels (each slot has few limbs); large ones stream more data between the
// passes of a batch at high levels.  The best size depends on the ring, the
// level and the chip, so it is measured: for each level, batches of zero
// ciphertexts are key-switched with a zero key (the work does not depend on
// the values) in launch sequences of each candidate size, timed with HIP
// events, and the fastest per key switch is kept.
#include <algorithm>
#include <vector>

#include "internal.h"

using namespace hck;

namespace {

#define TRY(expr)         \
  do {                    \
    int _rc = (expr);     \
    if (_rc) return _rc;  \
  } while (0)

// microseconds per key switch of `count` rotations at `level` with the
// current cap (median of `reps` timed calls after one warm-up call)
int time_batch(hck_context *ctx, const std::vector<hck_ciphertext *> &in,
               const std::vector<hck_ciphertext *> &out, const hck_switch_key *key, uint32_t reps,
               hipEvent_t e0, hipEvent_t e1, double *us) {
  const uint32_t n = (uint32_t)in.size();
  const uint32_t g = galois_of_step(ctx, 1);
  std::vector<uint32_t> gs(n, g);
  std::vector<const hck_switch_key *> keys(n, key);
  std::vector<double> t;
  for (uint32_t r = 0; r <= reps; r++) {
    HCK_HIP(ctx, hipEventRecord(e0, ctx->stream));
    TRY(apply_galois_keys(ctx, in.data(), gs.data(), keys.data(), n, out.data()));
    HCK_HIP(ctx, hipEventRecord(e1, ctx->stream));
    HCK_HIP(ctx, hipEventSynchronize(e1));
    float ms = 0;
    HCK_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
    if (r) t.push_back(1e3 * ms / n);
  }
  std::sort(t.begin(), t.end());
  *us = t[t.size() / 2];
  return HCK_OK;
}

// zero switching key and `count` zero ciphertexts on a context (the work of a
// key switch does not depend on the values)
struct ZeroSetup {
  hck_context *ctx;
  hck_switch_key key;
  std::vector<hck_ciphertext *> in, out;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  explicit ZeroSetup(hck_context *c) : ctx(c) { key.ctx = c; }
  int init(uint32_t count) {
    TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
    const size_t kwords = (size_t)ctx->dnum * 2 * (ctx->L + ctx->K) * ctx->n;
    TRY(dev_alloc(ctx, &key.data, kwords));
    for (uint32_t i = 0; i < count; i++) {
      in.push_back(pool_get(ctx));
      out.push_back(pool_get(ctx));
      TRY(ensure_ct(ctx, in.back(), 2));
      TRY(ensure_ct(ctx, out.back(), 2));
      if (hipMemsetAsync(in.back()->data, 0, (size_t)2 * ctx->L * ctx->n * 8, ctx->stream) !=
          hipSuccess)
        return check_hip(ctx, hipGetLastError(), "autotune set-up");
      in.back()->size = 2;
      in.back()->scale = 1.0;
    }
    if (hipMemsetAsync(key.data, 0, kwords * 8, ctx->stream) != hipSuccess)
      return check_hip(ctx, hipGetLastError(), "autotune set-up");
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      return check_hip(ctx, hipGetLastError(), "autotune events");
    return HCK_OK;
  }
  void level(uint32_t l) {
    for (hck_ciphertext *c : in) c->level = l;
  }
  int time(double *us) { return time_batch(ctx, in, out, &key, 3, e0, e1, us); }
  ~ZeroSetup() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (hck_ciphertext *c : in) pool_put(ctx, c);
    for (hck_ciphertext *c : out) pool_put(ctx, c);
    dev_free(ctx, key.data);
  }
};

}  // namespace

extern "C" {

int hck_autotune_keyswitch(hck_context *ctx, const uint32_t *levels, uint32_t n_levels,
                           uint32_t count, uint32_t *caps, double *us_per_switch) {
  if (!ctx || (n_levels && !levels)) return set_error(HCK_EINVAL, "null argument");
  if (count == 0 || count > 256) return set_error(HCK_EINVAL, "count must be 1..256");
  for (uint32_t i = 0; i < n_levels; i++)
    if (levels[i] >= ctx->L) return set_error(HCK_ELEVEL, "level beyond the chain");
  HCK_HIP(ctx, hipSetDevice(ctx->device));
  ZeroSetup z(ctx);
  int rc = z.init(count);
  static const uint32_t kCand[] = {1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 24, 32};
  for (uint32_t li = 0; li < n_levels && !rc; li++) {
    const uint32_t level = levels[li];
    z.level(level);
    const uint32_t fit = ks_batch_fit(ctx, level);
    const uint8_t saved = ctx->ks_cap[level];
    // the built-in rule first: a candidate must beat it by 2 % to replace it
    ctx->ks_cap[level] = 0;
    const uint32_t rule = ks_batch_limit(ctx, level);
    double best_us = 0;
    rc = z.time(&best_us);
    uint32_t best = rule;
    for (uint32_t c : kCand) {
      if (rc || c > fit || c == rule) continue;
      ctx->ks_cap[level] = (uint8_t)c;
      double us = 0;
      rc = z.time(&us);
      if (!rc && us < 0.98 * best_us) {
        best_us = us;
        best = c;
      }
    }
    ctx->ks_cap[level] = rc ? saved : (uint8_t)best;
    if (caps) caps[li] = best;
    if (us_per_switch) us_per_switch[li] = best_us;
  }
  return rc;
}

int hck_autotune_dnum(const hck_params *candidates, uint32_t n, int device, void *hip_stream,
                      uint32_t level, uint32_t count, double *us_per_switch, double *key_bytes,
                      uint32_t *best) {
  if (!candidates || n == 0) return set_error(HCK_EINVAL, "no candidate parameter sets");
  if (count == 0 || count > 256) return set_error(HCK_EINVAL, "count must be 1..256");
  for (uint32_t i = 0; i < n; i++) {
    const hck_params &p = candidates[i];
    const hck_params &p0 = candidates[0];
    if (p.log_n != p0.log_n || p.num_q != p0.num_q || !p.q || !p0.q ||
        !std::equal(p.q, p.q + p.num_q, p0.q))
      return set_error(HCK_EINVAL, "candidates must share the ring and the q chain");
    if (level >= p.num_q) return set_error(HCK_ELEVEL, "level beyond the chain");
  }
  double best_us = 0;
  uint32_t best_i = 0;
  for (uint32_t i = 0; i < n; i++) {
    hck_context *ctx = nullptr;
    TRY(build_context(&candidates[i], device, hip_stream, &ctx));
    double us = 0;
    int rc = HCK_OK;
    {
      ZeroSetup z(ctx);
      rc = z.init(count);
      if (!rc) {
        z.level(level);
        rc = z.time(&us);
      }
    }
    destroy_context(ctx);
    if (rc) return rc;
    if (us_per_switch) us_per_switch[i] = us;
    if (key_bytes)
      key_bytes[i] = 8.0 * candidates[i].dnum * 2 * (candidates[i].num_q + candidates[i].num_p) *
                     (double)(1u << candidates[i].log_n);
    if (i == 0 || us < best_us) {
      best_us = us;
      best_i = i;
    }
  }
  if (best) *best = best_i;
  return HCK_OK;
}

int hck_autotune_ntt(hck_context *ctx, uint32_t rows, int32_t *splits, double *us_per_row,
                     uint32_t cap, uint32_t *n, int32_t *chosen) {
  if (!ctx) return set_error(HCK_EINVAL, "null context");
  if (rows == 0 || rows > (uint32_t)kMaxRows) return set_error(HCK_EINVAL, "rows must be 1..256");
  if (ctx->capturing) return set_error(HCK_EINVAL, "tuning during graph capture");
  HCK_HIP(ctx, hipSetDevice(ctx->device));
  const int a0 = (ctx->log_n + 1) / 2;
  std::vector<int> cand;
  for (int a : {a0, a0 - 1, a0 + 1})
    if (ntt_split_available(ctx->log_n, a)) cand.push_back(a);
  if (n) *n = (uint32_t)cand.size();
  if ((splits || us_per_row) && cap < cand.size())
    return set_error(HCK_EINVAL, "output arrays too small");
  uint64_t *buf = nullptr;
  TRY(dev_alloc(ctx, &buf, (size_t)rows * ctx->n));
  LimbMap map;
  map.n = rows;
  for (uint32_t r = 0; r < rows; r++) {
    map.row[r] = (uint16_t)r;
    map.mod[r] = (uint8_t)(r % (ctx->L + ctx->K));
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = HCK_OK;
  if (hipMemsetAsync(buf, 0, (size_t)rows * ctx->n * 8, ctx->stream) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = check_hip(ctx, hipGetLastError(), "NTT tuning set-up");
  const uint8_t saved = ctx->ntt_a;
  double best_us = 0;
  int best = a0;
  for (size_t i = 0; i < cand.size() && !rc; i++) {
    rc = set_ntt_split(ctx, cand[i]);
    std::vector<double> t;
    for (int r = 0; r <= 5 && !rc; r++) {
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) rc = check_hip(ctx, hipGetLastError(), "event");
      if (!rc) rc = ntt_forward(ctx, buf, map);
      if (!rc) rc = ntt_inverse(ctx, buf, map, nullptr);
      float ms = 0;
      if (!rc && (hipEventRecord(e1, ctx->stream) != hipSuccess ||
                  hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = check_hip(ctx, hipGetLastError(), "NTT tuning timing");
      if (!rc && r) t.push_back(1e3 * ms / rows);
    }
    if (rc) break;
    std::sort(t.begin(), t.end());
    const double us = t[t.size() / 2];
    if (splits) splits[i] = cand[i];
    if (us_per_row) us_per_row[i] = us;
    // the default split first: another must beat it by 2 % to replace it
    if (i == 0 || us < 0.98 * best_us) {
      best_us = us;
      best = cand[i];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  dev_free(ctx, buf);
  if (rc) {
    ctx->ntt_a = saved;
    return rc;
  }
  if (chosen) *chosen = best;
  return set_ntt_split(ctx, best);
}

int hck_set_ntt_split(hck_context *ctx, int32_t log_r1) {
  if (!ctx) return set_error(HCK_EINVAL, "null context");
  HCK_HIP(ctx, hipSetDevice(ctx->device));
  return set_ntt_split(ctx, log_r1);
}

int hck_ntt_split(const hck_context *ctx, int32_t *log_r1) {
  if (!ctx || !log_r1) return set_error(HCK_EINVAL, "null argument");
  *log_r1 = ctx->ntt_a ? ctx->ntt_a : (int32_t)((ctx->log_n + 1) / 2);
  return HCK_OK;
}

int hck_set_keyswitch_cap(hck_context *ctx, uint32_t level, uint32_t cap) {
  if (!ctx) return set_error(HCK_EINVAL, "null context");
  if (level >= ctx->L) return set_error(HCK_ELEVEL, "level beyond the chain");
  if (cap > (uint32_t)kMaxBatch) return set_error(HCK_EINVAL, "cap beyond the batch limit");
  ctx->ks_cap[level] = (uint8_t)cap;
  return HCK_OK;
}

int hck_keyswitch_batch_limit(const hck_context *ctx, uint32_t level, uint32_t *cap) {
  if (!ctx || !cap) return set_error(HCK_EINVAL, "null argument");
  if (level >= ctx->L) return set_error(HCK_ELEVEL, "level beyond the chain");
  *cap = ks_batch_limit(ctx, level);
  return HCK_OK;
}

}  // extern "C"
