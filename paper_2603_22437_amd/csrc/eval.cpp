// Hybrid key switching and the automorphism-then-switch rotation.
//
// KeySwitch(d) at level l with a switching key swk(s' -> s), d in evaluation
// form over Q_l = q_0..q_l:
//   1. d is copied and brought to the coefficient domain by an inverse NTT
//      whose final scaling also multiplies limb i by (Q_j / q_i)^-1, q_i in
//      digit D_j = [j alpha, min((j+1) alpha, l+1)) (alpha = ceil(L / dnum));
//   2. ModUp: for every digit, fast basis conversion of its limbs to every
//      other limb of Q_l u P (P = p_0..p_(K-1)), then forward NTT of those
//      limbs; on its own limbs the extended digit is d itself;
//   3. inner product with the key: acc_{0,1}[t] = sum_j d~_j[t] swk_j[t];
//   4. ModDown with rounding: the P limbs of acc are inverse-transformed with
//      (P/p_k)^-1 folded in and ((P-1)/2) (P/p_k)^-1 added, converted to
//      Q_l with -(P-1)/2 added, forward-transformed, and
//      out_i = (acc_i - conv_i) P^-1 mod q_i.
// Every limb of one step runs in one launch (LimbMap).
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

int keyswitch_core(hck_context *ctx, const uint64_t *d, uint32_t level, const hck_switch_key *key,
                   uint64_t *out0, uint64_t *out1, const uint64_t *add0, const uint64_t *add1) {
  int rc = ensure_workspace(ctx, ws_words_needed(ctx));
  if (rc) return rc;
  const size_t n = ctx->n;
  const uint32_t L = ctx->L, K = ctx->K, A = ctx->alpha, nm = L + K;
  const uint32_t nq = level + 1, ne = nq + K;
  uint64_t *y = ws_ks(ctx);
  uint64_t *ext = y + (size_t)L * n;
  uint64_t *acc = ext + (size_t)ctx->dnum * nm * n;
  uint64_t *conv = acc + (size_t)2 * nm * n;
  auto mod_of = [&](uint32_t t) -> uint8_t { return (uint8_t)(t < nq ? t : L + (t - nq)); };

  // 1. coefficient form of d, times (Q_j / q_i)^-1
  if ((rc = launch_copy(ctx, y, d, (size_t)nq * n))) return rc;
  RowScale sc;
  for (uint32_t i = 0; i < nq; i++) {
    sc.w[i] = ctx->up_scale[level][i];
    sc.wp[i] = h_shoup(sc.w[i], ctx->mods[i]);
    sc.add[i] = 0;
  }
  if ((rc = ntt_inverse(ctx, y, qmap(ctx, level), &sc))) return rc;

  // 2. ModUp of every digit, then one batched forward NTT
  std::vector<std::pair<uint16_t, uint8_t>> ext_rows;
  for (uint32_t j = 0; j < ctx->dnum; j++) {
    const uint32_t lo = j * A;
    if (lo >= nq) break;
    const uint32_t hi = std::min(lo + A, nq);
    LimbMap min, mout;
    min.n = hi - lo;
    for (uint32_t a = 0; a < hi - lo; a++) {
      min.row[a] = (uint16_t)(lo + a);
      min.mod[a] = (uint8_t)(lo + a);
    }
    mout.n = 0;
    for (uint32_t t = 0; t < ne; t++) {
      if (t >= lo && t < hi) continue;
      mout.row[mout.n] = (uint16_t)(j * ne + t);
      mout.mod[mout.n] = mod_of(t);
      ext_rows.push_back({mout.row[mout.n], mout.mod[mout.n]});
      mout.n++;
    }
    const uint64_t *cm = ctx->d_up_conv + ((size_t)level * ctx->dnum + j) * A * nm;
    if ((rc = launch_bconv(ctx, ext, mout, y, min, cm, nm, nullptr))) return rc;
  }
  if ((rc = ntt_forward_rows(ctx, ext, ext_rows))) return rc;

  // 3. inner product with the key over Q_l u P
  if ((rc = launch_ks_inner(ctx, acc, ext, d, key->data, level))) return rc;

  // 4. ModDown of both accumulators
  LimbMap mp;
  RowScale sp;
  mp.n = 2 * K;
  for (uint32_t p = 0; p < 2; p++)
    for (uint32_t k = 0; k < K; k++) {
      const uint32_t r = p * K + k;
      mp.row[r] = (uint16_t)(p * ne + nq + k);
      mp.mod[r] = (uint8_t)(L + k);
      sp.w[r] = ctx->down_scale[k];
      sp.wp[r] = h_shoup(sp.w[r], ctx->mods[L + k]);
      sp.add[r] = ctx->down_add[k];
    }
  if ((rc = ntt_inverse(ctx, acc, mp, &sp))) return rc;
  std::vector<std::pair<uint16_t, uint8_t>> conv_rows;
  for (uint32_t p = 0; p < 2; p++) {
    LimbMap min, mout;
    min.n = K;
    for (uint32_t k = 0; k < K; k++) {
      min.row[k] = (uint16_t)(p * ne + nq + k);
      min.mod[k] = (uint8_t)(L + k);
    }
    mout.n = nq;
    for (uint32_t i = 0; i < nq; i++) {
      mout.row[i] = (uint16_t)(p * L + i);
      mout.mod[i] = (uint8_t)i;
      conv_rows.push_back({mout.row[i], mout.mod[i]});
    }
    if ((rc = launch_bconv(ctx, conv, mout, acc, min, ctx->d_down_conv, nm, ctx->d_down_hneg)))
      return rc;
  }
  if ((rc = ntt_forward_rows(ctx, conv, conv_rows))) return rc;
  if ((rc = launch_moddown_tail(ctx, out0, acc, conv, add0, level))) return rc;
  return launch_moddown_tail(ctx, out1, acc + (size_t)ne * n, conv + (size_t)L * n, add1, level);
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
  uint64_t *rot = ws_rot(ctx);
  if ((rc = launch_automorphism(ctx, rot, a->data, ps, 2, qmap(ctx, a->level), g))) return rc;
  const uint32_t level = a->level;
  const double scale = a->scale;
  rc = keyswitch_core(ctx, rot + ps, level, it->second, out->data, out->data + ps, rot, nullptr);
  if (rc) return rc;
  out->size = 2;
  out->level = level;
  out->scale = scale;
  return HCK_OK;
}

}  // namespace hck
