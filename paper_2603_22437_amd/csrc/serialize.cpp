// Interchange form of ciphertexts and switching keys: a 64-byte header naming
// the parameter set, then the residues in the export layout.  The paper's
// client uploads its evaluation keys once at enrollment and the cloud keeps
// them (section 5.4, communication and resource overhead); windows travel as
// ciphertexts.  The header lets either side refuse words made under another
// parameter set instead of computing garbage with them.
#include <cstring>
#include <vector>

#include "internal.h"

using namespace hck;

namespace {

constexpr char kMagic[8] = {'H', 'C', 'K', 'C', 'K', 'K', 'S', '1'};
static_assert(sizeof(hck_blob_header) == 64, "the blob header is 64 bytes");

// FNV-1a (64-bit) over the primes as little-endian 8-byte words
uint64_t fnv1a_primes(const uint64_t *a, size_t na, const uint64_t *b, size_t nb) {
  uint64_t h = 0xcbf29ce484222325ull;
  auto eat = [&](uint64_t w) {
    for (int i = 0; i < 8; i++) {
      h ^= (w >> (8 * i)) & 0xFF;
      h *= 0x100000001b3ull;
    }
  };
  for (size_t i = 0; i < na; i++) eat(a[i]);
  for (size_t i = 0; i < nb; i++) eat(b[i]);
  return h;
}

int check_against(const hck_context *ctx, const hck_blob_header &h, uint32_t kind) {
  if (h.kind != kind) return set_error(HCK_EINVAL, "blob holds another kind of object");
  if (h.log_n != ctx->log_n || h.num_q != ctx->L || h.num_p != ctx->K || h.dnum != ctx->dnum ||
      h.prime_hash != fnv1a_primes(ctx->mods.data(), ctx->L + ctx->K, nullptr, 0))
    return set_error(HCK_EPARAMS, "blob made under another parameter set");
  return HCK_OK;
}

hck_blob_header header_for(const hck_context *ctx, uint32_t kind, uint32_t level, uint32_t polys,
                           uint32_t rows, double scale) {
  hck_blob_header h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kMagic, 8);
  h.kind = kind;
  h.log_n = ctx->log_n;
  h.num_q = ctx->L;
  h.num_p = ctx->K;
  h.dnum = ctx->dnum;
  h.level = level;
  h.polys = polys;
  h.rows = rows;
  h.scale = scale;
  h.prime_hash = fnv1a_primes(ctx->mods.data(), ctx->L + ctx->K, nullptr, 0);
  h.words = (uint64_t)polys * rows * ctx->n;
  return h;
}

int emit(const hck_blob_header &h, void *buf, size_t cap, size_t *size, uint8_t **words) {
  *size = sizeof(h) + 8 * h.words;
  *words = nullptr;
  if (!buf) return HCK_OK;
  if (cap < *size) return set_error(HCK_EINVAL, "buffer too small");
  std::memcpy(buf, &h, sizeof(h));
  *words = (uint8_t *)buf + sizeof(h);
  return HCK_OK;
}

}  // namespace

extern "C" {

int hck_params_hash(const hck_params *p, uint64_t *hash) {
  if (!p || !hash || (p->num_q && !p->q) || (p->num_p && !p->p))
    return set_error(HCK_EINVAL, "null argument");
  *hash = fnv1a_primes(p->q, p->num_q, p->p, p->num_p);
  return HCK_OK;
}

int hck_blob_parse(const void *buf, size_t size, hck_blob_header *out) {
  if (!buf || !out) return set_error(HCK_EINVAL, "null argument");
  if (size < sizeof(hck_blob_header)) return set_error(HCK_EINVAL, "blob shorter than its header");
  hck_blob_header h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, kMagic, 8) != 0) return set_error(HCK_EINVAL, "not a hipckks blob");
  if (h.kind != HCK_BLOB_CIPHERTEXT && h.kind != HCK_BLOB_SWITCH_KEY)
    return set_error(HCK_EINVAL, "unknown blob kind");
  if (h.log_n < 11 || h.log_n > 17 || h.num_q == 0 || h.num_q + h.num_p > HCK_MAX_LIMBS ||
      h.dnum == 0 || h.level >= h.num_q)
    return set_error(HCK_EINVAL, "blob header out of range");
  const uint64_t n = 1ull << h.log_n;
  const bool ct = h.kind == HCK_BLOB_CIPHERTEXT;
  if (ct ? ((h.polys != 2 && h.polys != 3) || h.rows != h.level + 1)
         : (h.polys != 2 * h.dnum || h.rows != h.num_q + h.num_p || h.level != h.num_q - 1))
    return set_error(HCK_EINVAL, "blob shape inconsistent with its kind");
  if (h.words != (uint64_t)h.polys * h.rows * n || size != sizeof(h) + 8 * h.words)
    return set_error(HCK_EINVAL, "blob size inconsistent with its header");
  *out = h;
  return HCK_OK;
}

int hck_ciphertext_serialize(hck_context *ctx, const hck_ciphertext *ct, void *buf, size_t cap,
                             size_t *size) {
  if (!ctx || !ct || !size) return set_error(HCK_EINVAL, "null argument");
  if (ct->ctx != ctx) return set_error(HCK_EINVAL, "ciphertext of another (or a destroyed) context");
  if (ct->size == 0) return set_error(HCK_EINVAL, "empty ciphertext");
  const hck_blob_header h =
      header_for(ctx, HCK_BLOB_CIPHERTEXT, ct->level, ct->size, ct->level + 1, ct->scale);
  uint8_t *words = nullptr;
  int rc = emit(h, buf, cap, size, &words);
  if (rc || !words) return rc;
  std::vector<uint64_t> tmp(h.words);
  rc = hck_ciphertext_export(ctx, ct, tmp.data(), tmp.size(), nullptr, nullptr, nullptr);
  if (!rc) std::memcpy(words, tmp.data(), 8 * h.words);
  return rc;
}

int hck_ciphertext_deserialize(hck_context *ctx, const void *buf, size_t size,
                               hck_ciphertext **out) {
  if (!ctx || !out) return set_error(HCK_EINVAL, "null argument");
  hck_blob_header h;
  int rc = hck_blob_parse(buf, size, &h);
  if (!rc) rc = check_against(ctx, h, HCK_BLOB_CIPHERTEXT);
  if (rc) return rc;
  std::vector<uint64_t> w(h.words);
  std::memcpy(w.data(), (const uint8_t *)buf + sizeof(h), 8 * h.words);
  for (uint64_t r = 0; r < (uint64_t)h.polys * h.rows; r++) {
    const uint64_t q = ctx->mods[r % h.rows];
    for (uint64_t c = 0; c < ctx->n; c++)
      if (w[r * ctx->n + c] >= q) return set_error(HCK_EINVAL, "residue not below its prime");
  }
  return hck_ciphertext_import(ctx, w.data(), h.polys, h.level, h.scale, out);
}

int hck_switch_key_serialize(hck_context *ctx, const hck_switch_key *swk, void *buf, size_t cap,
                             size_t *size) {
  if (!ctx || !swk || !size) return set_error(HCK_EINVAL, "null argument");
  const hck_blob_header h = header_for(ctx, HCK_BLOB_SWITCH_KEY, ctx->L - 1, 2 * ctx->dnum,
                                       ctx->L + ctx->K, 0.0);
  uint8_t *words = nullptr;
  int rc = emit(h, buf, cap, size, &words);
  if (rc || !words) return rc;
  std::vector<uint64_t> tmp(h.words);
  rc = hck_switch_key_export(ctx, swk, tmp.data(), tmp.size());
  if (!rc) std::memcpy(words, tmp.data(), 8 * h.words);
  return rc;
}

int hck_switch_key_deserialize(hck_context *ctx, const void *buf, size_t size,
                               hck_switch_key **out) {
  if (!ctx || !out) return set_error(HCK_EINVAL, "null argument");
  hck_blob_header h;
  int rc = hck_blob_parse(buf, size, &h);
  if (!rc) rc = check_against(ctx, h, HCK_BLOB_SWITCH_KEY);
  if (rc) return rc;
  std::vector<uint64_t> w(h.words);
  std::memcpy(w.data(), (const uint8_t *)buf + sizeof(h), 8 * h.words);
  return hck_switch_key_import(ctx, w.data(), w.size(), out);
}

}  // extern "C"
