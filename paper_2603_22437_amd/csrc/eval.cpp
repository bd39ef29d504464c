// Workspace layout and the automorphism-then-switch rotation
// Rot(c, k) = (phi_g(c0), 0) + KeySwitch(phi_g(c1)), g = 5^k mod 2N; the key
// switch itself is in ks_fused.hip.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace hck {

size_t ws_words_needed(const hck_context *ctx) {
  const size_t n = ctx->n, L = ctx->L, LK = ctx->L + ctx->K;
  const size_t ks = L + ctx->dnum * LK + 2 * LK + 2 * L;
  return n * (ks + 2 * L + 3 * LK);
}

uint64_t *ws_ks(hck_context *ctx) { return ctx->ws; }

uint64_t *ws_rot(hck_context *ctx) {
  const size_t n = ctx->n, L = ctx->L, LK = ctx->L + ctx->K;
  return ctx->ws + n * (L + ctx->dnum * LK + 2 * LK + 2 * L);
}

uint64_t *ws_tmp(hck_context *ctx) { return ws_rot(ctx) + (size_t)ctx->n * 2 * ctx->L; }

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

int apply_galois_core(hck_context *ctx, const hck_ciphertext *a, uint32_t g,
                      const hck_galois_keys *gks, hck_ciphertext *out) {
  auto it = gks->keys.find(g);
  if (it == gks->keys.end())
    return set_error(HCK_ENOKEY, "no Galois key for element " + std::to_string(g));
  if (a->size != 2) return set_error(HCK_EINVAL, "rotation needs a 2-part ciphertext");
  int rc = ensure_workspace(ctx, ws_words_needed(ctx));
  if (rc) return rc;
  rc = ensure_ct(ctx, out, 2);
  if (rc) return rc;
  const size_t ps = (size_t)ctx->L * ctx->n;
  const uint32_t level = a->level;
  const double scale = a->scale;
  // (phi_g(c0), 0) + KeySwitch(phi_g(c1)); the automorphism is applied while
  // reading c1 and c0, so c0 must not be overwritten while it is gathered
  const uint64_t *c0 = a->data;
  if (out == a) {
    uint64_t *copy = ws_rot(ctx);
    if ((rc = launch_copy(ctx, copy, a->data, (size_t)(level + 1) * ctx->n))) return rc;
    c0 = copy;
  }
  rc = keyswitch_core(ctx, a->data + ps, g, level, it->second, out->data, out->data + ps, c0,
                      nullptr);
  if (rc) return rc;
  out->size = 2;
  out->level = level;
  out->scale = scale;
  return HCK_OK;
}

}  // namespace hck
