// Workspace layout and the automorphism-then-switch rotation
// Rot(c, k) = (phi_g(c0), 0) + KeySwitch(phi_g(c1)), g = 5^k mod 2N; the key
// switch itself is in ks_fused.hip.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace hck {

size_t ws_ks_rows(const hck_context *ctx) {
  const size_t L = ctx->L, LK = ctx->L + ctx->K;
  return L + ctx->dnum * LK + 2 * LK + 2 * L;
}

uint32_t ks_slots(const hck_context *ctx) {
  const size_t rows = ws_ks_rows(ctx);
  const size_t by_size = std::max<size_t>(8, 8192 / rows);
  const size_t by_index = 65535 / rows;
  return (uint32_t)std::max<size_t>(1, std::min<size_t>({(size_t)kMaxBatch, by_size, by_index}));
}

// [ks_slots key-switch slots][ks_slots x L rows: copies of aliased inputs]
// [3 (L+K) rows: general temporary][kLtOut x 2 (L+K) rows: extended-basis sums]
size_t ws_words_needed(const hck_context *ctx) {
  const size_t n = ctx->n, L = ctx->L, LK = ctx->L + ctx->K, S = ks_slots(ctx);
  return n * (S * ws_ks_rows(ctx) + S * L + 3 * LK + kLtOut * 2 * LK);
}

uint64_t *ws_ks(hck_context *ctx) { return ctx->ws; }

uint64_t *ws_rot(hck_context *ctx) {
  return ctx->ws + (size_t)ctx->n * ks_slots(ctx) * ws_ks_rows(ctx);
}

uint64_t *ws_tmp(hck_context *ctx) {
  return ws_rot(ctx) + (size_t)ctx->n * ks_slots(ctx) * ctx->L;
}

uint64_t *ws_pq(hck_context *ctx) {
  return ws_tmp(ctx) + (size_t)ctx->n * 3 * (ctx->L + ctx->K);
}

int ntt_forward_rows(hck_context *ctx, uint64_t *buf,
                     const std::vector<std::pair<uint16_t, uint8_t>> &rows) {
  for (size_t s = 0; s < rows.size(); s += kMaxRows) {
    LimbMap m;
    m.n = (uint32_t)std::min(rows.size() - s, (size_t)kMaxRows);
    for (uint32_t r = 0; r < m.n; r++) {
      m.row[r] = rows[s + r].first;
      m.mod[r] = rows[s + r].second;
    }
    int rc = ntt_forward(ctx, buf, m);
    if (rc) return rc;
  }
  return HCK_OK;
}

int apply_galois_multi(hck_context *ctx, const hck_ciphertext *const *a, const uint32_t *g,
                       uint32_t n, const hck_galois_keys *gks, hck_ciphertext *const *out) {
  std::vector<const hck_switch_key *> keys(n);
  for (uint32_t i = 0; i < n; i++) {
    auto it = gks->keys.find(g[i]);
    if (it == gks->keys.end())
      return set_error(HCK_ENOKEY, "no Galois key for element " + std::to_string(g[i]));
    keys[i] = it->second;
  }
  return apply_galois_keys(ctx, a, g, keys.data(), n, out);
}

int apply_galois_keys(hck_context *ctx, const hck_ciphertext *const *a, const uint32_t *g,
                      const hck_switch_key *const *keys, uint32_t n,
                      hck_ciphertext *const *out) {
  if (n == 0) return HCK_OK;
  const uint32_t level = a[0]->level;
  for (uint32_t i = 0; i < n; i++) {
    if (a[i]->size != 2) return set_error(HCK_EINVAL, "rotation needs a 2-part ciphertext");
    if (a[i]->level != level) return set_error(HCK_ELEVEL, "batched rotations need one level");
    for (uint32_t k = 0; k < n; k++) {
      if (k < i && out[k] == out[i]) return set_error(HCK_EINVAL, "batched outputs must be distinct");
      if (k != i && out[k] == a[i])
        return set_error(HCK_EINVAL, "a batched output may alias only its own input");
    }
  }
  int rc = ensure_workspace(ctx, ws_words_needed(ctx));
  if (rc) return rc;
  const size_t ps = (size_t)ctx->L * ctx->n;
  const uint32_t limit = ks_batch_limit(ctx, level);
  for (uint32_t s = 0; s < n; s += even_batch(n - s, limit)) {
    KsBatch kb;
    kb.n = even_batch(n - s, limit);
    std::vector<double> scales(kb.n);
    for (uint32_t b = 0; b < kb.n; b++) {
      const hck_ciphertext *x = a[s + b];
      hck_ciphertext *y = out[s + b];
      scales[b] = x->scale;
      // (phi_g(c0), 0) + KeySwitch(phi_g(c1)).  c1 is only read by the
      // launches before the final one, but c0 is gathered through phi_g by the
      // final launch while it writes the outputs: an output that aliases this
      // input gets a copy of c0 to read instead
      if ((rc = ensure_ct(ctx, y, 2))) return rc;
      const uint64_t *c0 = x->data, *c1 = x->data + ps;
      kb.add0_src[b] = nullptr;
      if (y == x) {
        // the first launch copies c0 into the workspace for the last one
        kb.add0_src[b] = x->data;
        c0 = ws_rot(ctx) + (size_t)b * ps;
      }
      kb.key[b] = keys[s + b]->data;
      kb.galois[b] = g[s + b];
      kb.d[b] = c1;
      kb.out0[b] = y->data;
      kb.out1[b] = y->data + ps;
      kb.add0[b] = c0;
      kb.add1[b] = nullptr;
    }
    if ((rc = keyswitch_batch(ctx, kb, level))) return rc;
    for (uint32_t b = 0; b < kb.n; b++) {
      out[s + b]->size = 2;
      out[s + b]->level = level;
      out[s + b]->scale = scales[b];
    }
  }
  return HCK_OK;
}

int apply_galois_many(hck_context *ctx, const hck_ciphertext *const *a, uint32_t n, uint32_t g,
                      const hck_galois_keys *gks, hck_ciphertext *const *out) {
  std::vector<uint32_t> gs(n, g);
  return apply_galois_multi(ctx, a, gs.data(), n, gks, out);
}

int apply_galois_core(hck_context *ctx, const hck_ciphertext *a, uint32_t g,
                      const hck_galois_keys *gks, hck_ciphertext *out) {
  return apply_galois_many(ctx, &a, 1, g, gks, &out);
}

// Pooled scratch ciphertexts of the host-side evaluators (returned empty or
// with their last contents; the context frees them).
hck_ciphertext *pool_get(hck_context *ctx) {
  if (!ctx->ct_pool.empty()) {
    hck_ciphertext *ct = ctx->ct_pool.back();
    ctx->ct_pool.pop_back();
    return ct;
  }
  hck_ciphertext *ct = new hck_ciphertext();
  ct->ctx = ctx;
  ct->pooled = true;
  return ct;
}

void pool_put(hck_context *ctx, hck_ciphertext *ct) {
  if (ct) ctx->ct_pool.push_back(ct);
}

}  // namespace hck
