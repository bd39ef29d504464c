// The C ABI: keys, plaintexts, ciphertexts, evaluation, linear transforms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace hck;

namespace {

int enter(hck_context *ctx) {
  if (!ctx) return set_error(HCK_EINVAL, "null context");
  if (ctx->broken) return set_error(HCK_EDEVICE, "context unusable after an earlier HIP error");
  HCK_HIP(ctx, hipSetDevice(ctx->device));
  return HCK_OK;
}

#define ENTER(ctx)             \
  do {                         \
    int _rc = enter(ctx);      \
    if (_rc) return _rc;       \
  } while (0)
#define TRY(expr)              \
  do {                         \
    int _rc = (expr);          \
    if (_rc) return _rc;       \
  } while (0)

size_t poly_stride(const hck_context *ctx) { return (size_t)ctx->L * ctx->n; }

// Releases of caller handles (hck::track): the device memory goes back and
// the handle is detached from its context (ctx = null), so that its destroy
// call later frees only the host record.
template <class T>
void release_data(void *p) {
  T *x = static_cast<T *>(p);
  if (x->ctx) dev_free(x->ctx, x->data);
  x->data = nullptr;
  x->ctx = nullptr;
}

void release_ct(void *p) {
  hck_ciphertext *ct = static_cast<hck_ciphertext *>(p);
  release_data<hck_ciphertext>(ct);
  ct->cap_polys = ct->size = 0;
}

void release_gks(void *p) {
  hck_galois_keys *g = static_cast<hck_galois_keys *>(p);
  for (auto &kv : g->keys) release_data<hck_switch_key>(kv.second);
  g->ctx = nullptr;
}

void release_lt(void *p) {
  hck_linear_transform *lt = static_cast<hck_linear_transform *>(p);
  if (lt->ctx)
    for (uint64_t *q : lt->owned) dev_free(lt->ctx, q);
  lt->owned.clear();
  lt->groups.clear();
  lt->grid = nullptr;
  lt->ctx = nullptr;
}

// a handle given to a call must belong to the call's context (a handle whose
// context was destroyed has none)
#define OWNED(ctx, h)                                                                 \
  do {                                                                                \
    if ((h) && (h)->ctx != (ctx))                                                     \
      return set_error(HCK_EINVAL, #h " belongs to another (or a destroyed) context"); \
  } while (0)

// Host buffers are often locals of the caller, so uploads complete before
// returning (set-up paths only; evaluation never uploads).
int upload(hck_context *ctx, uint64_t *dst, const void *src, size_t bytes) {
  if (ctx->capturing) return set_error(HCK_EINVAL, "host transfer during graph capture");
  HCK_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
  HCK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return HCK_OK;
}

int download(hck_context *ctx, void *dst, const uint64_t *src, size_t bytes) {
  if (ctx->capturing) return set_error(HCK_EINVAL, "host transfer during graph capture");
  HCK_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
  HCK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return HCK_OK;
}

// rows (row, modulus) of a [polys][stride/N][N] buffer for limbs 0..level
std::vector<std::pair<uint16_t, uint8_t>> poly_rows(uint32_t polys, uint32_t rows_per_poly,
                                                    uint32_t nlimbs, uint32_t mod_base = 0) {
  std::vector<std::pair<uint16_t, uint8_t>> r;
  for (uint32_t p = 0; p < polys; p++)
    for (uint32_t i = 0; i < nlimbs; i++)
      r.push_back({(uint16_t)(p * rows_per_poly + i), (uint8_t)(mod_base + i)});
  return r;
}

LimbMap make_map(const std::vector<std::pair<uint16_t, uint8_t>> &rows, size_t start,
                 size_t cap = kMaxLimbs) {
  LimbMap m;
  m.n = (uint32_t)std::min(rows.size() - start, cap);
  for (uint32_t i = 0; i < m.n; i++) {
    m.row[i] = rows[start + i].first;
    m.mod[i] = rows[start + i].second;
  }
  return m;
}

int inverse_rows(hck_context *ctx, uint64_t *buf,
                 const std::vector<std::pair<uint16_t, uint8_t>> &rows) {
  for (size_t s = 0; s < rows.size(); s += kMaxRows) TRY(ntt_inverse(ctx, buf, make_map(rows, s, kMaxRows), nullptr));
  return HCK_OK;
}

int mont_rows(hck_context *ctx, uint64_t *buf,
              const std::vector<std::pair<uint16_t, uint8_t>> &rows, bool to) {
  for (size_t s = 0; s < rows.size(); s += kMaxRows)
    TRY(launch_to_mont(ctx, buf, make_map(rows, s, kMaxRows), to));
  return HCK_OK;
}

// Uniform limbs drawn in parallel host threads (each limb its own stream).
void sample_uniform_limbs(hck_context *ctx, const std::string &tag, uint64_t seed,
                          uint32_t nlimbs, const std::vector<uint32_t> &mod_of_limb,
                          std::vector<uint64_t> &out) {
  out.resize((size_t)nlimbs * ctx->n);
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned w = 0; w < nt; w++)
    th.emplace_back([&, w]() {
      for (uint32_t t = w; t < nlimbs; t += nt)
        sample_uniform(tag, seed, t, ctx->mods[mod_of_limb[t]], out.data() + (size_t)t * ctx->n,
                       ctx->n);
    });
  for (auto &t : th) t.join();
}

// Uploads N small integers and embeds them into `rows` of buf.
int embed_small_host(hck_context *ctx, uint64_t *buf, const std::vector<int32_t> &v,
                     const std::vector<std::pair<uint16_t, uint8_t>> &rows) {
  uint64_t *tmp = nullptr;
  TRY(dev_alloc(ctx, &tmp, (ctx->n + 1) / 2));
  int rc = upload(ctx, tmp, v.data(), v.size() * sizeof(int32_t));
  for (size_t s = 0; !rc && s < rows.size(); s += kMaxRows)
    rc = launch_embed_small(ctx, buf, (const int32_t *)tmp, make_map(rows, s, kMaxRows));
  dev_free(ctx, tmp);
  return rc;
}

bool scales_match(double a, double b) {
  return std::fabs(a - b) <= std::ldexp(std::max(std::fabs(a), std::fabs(b)), -30);
}

// residues (host, coefficient domain) -> evaluation form rows of buf, checked < q
int import_rows(hck_context *ctx, uint64_t *buf, const uint64_t *res, uint32_t polys,
                uint32_t rows_per_poly, uint32_t nlimbs) {
  const size_t n = ctx->n;
  for (uint32_t p = 0; p < polys; p++)
    for (uint32_t i = 0; i < nlimbs; i++) {
      const uint64_t *src = res + ((size_t)p * nlimbs + i) * n;
      const uint64_t q = ctx->mods[i];
      for (size_t c = 0; c < n; c++)
        if (src[c] >= q) return set_error(HCK_EINVAL, "residue not below its prime");
      TRY(upload(ctx, buf + ((size_t)p * rows_per_poly + i) * n, src, n * 8));
    }
  return ntt_forward_rows(ctx, buf, poly_rows(polys, rows_per_poly, nlimbs));
}

// evaluation-form rows -> host residues (compact [polys][nlimbs][N]); `mont`
// undoes the Montgomery form first.  Uses a temporary device copy.
int export_rows(hck_context *ctx, const uint64_t *buf, uint32_t polys, uint32_t rows_per_poly,
                uint32_t nlimbs, bool mont, uint32_t mod_base, uint64_t *out) {
  const size_t n = ctx->n;
  uint64_t *tmp = nullptr;
  TRY(dev_alloc(ctx, &tmp, (size_t)polys * nlimbs * n));
  int rc = HCK_OK;
  for (uint32_t p = 0; p < polys && !rc; p++)
    rc = launch_copy(ctx, tmp + (size_t)p * nlimbs * n, buf + (size_t)p * rows_per_poly * n,
                     (size_t)nlimbs * n);
  auto rows = poly_rows(polys, nlimbs, nlimbs, 0);
  // modulus of compact row (p, i) is the chain index of limb i (+ mod_base)
  for (auto &r : rows) r.second = (uint8_t)(mod_base + r.first % nlimbs);
  if (!rc && mont) rc = mont_rows(ctx, tmp, rows, false);
  if (!rc) rc = inverse_rows(ctx, tmp, rows);
  if (!rc) rc = download(ctx, out, tmp, (size_t)polys * nlimbs * n * 8);
  dev_free(ctx, tmp);
  return rc;
}

// key rows in chain order: limb t of a full-basis polynomial is modulus t
int export_key_rows(hck_context *ctx, const uint64_t *buf, uint32_t polys, uint64_t *out) {
  const size_t n = ctx->n;
  const uint32_t nm = ctx->L + ctx->K;
  uint64_t *tmp = nullptr;
  TRY(dev_alloc(ctx, &tmp, (size_t)polys * nm * n));
  int rc = launch_copy(ctx, tmp, buf, (size_t)polys * nm * n);
  auto rows = poly_rows(polys, nm, nm, 0);
  if (!rc) rc = mont_rows(ctx, tmp, rows, false);
  if (!rc) rc = inverse_rows(ctx, tmp, rows);
  if (!rc) rc = download(ctx, out, tmp, (size_t)polys * nm * n * 8);
  dev_free(ctx, tmp);
  return rc;
}

// swk(s' -> s): digit j = (-a_j s + e_j + [i in D_j] (P mod q_i) s'_i, a_j) on
// all L+K limbs, stored in evaluation + Montgomery form.  sp_m: s' as
// evaluation-form Montgomery rows [L+K][N].
int make_switch_key(hck_context *ctx, const hck_secret_key *sk, const uint64_t *sp_m,
                    const std::string &tag, uint64_t seed, hck_switch_key **out) {
  const size_t n = ctx->n;
  const uint32_t L = ctx->L, K = ctx->K, nm = L + K;
  hck_switch_key *key = new hck_switch_key();
  key->ctx = ctx;
  int rc = dev_alloc(ctx, &key->data, (size_t)ctx->dnum * 2 * nm * n);
  if (rc) {
    delete key;
    return rc;
  }
  uint64_t *tmp = ws_tmp(ctx);
  std::vector<uint32_t> mod_of(nm);
  for (uint32_t t = 0; t < nm; t++) mod_of[t] = t;
  std::vector<uint64_t> a;
  std::vector<int32_t> e(n);
  const LimbMap full = fullmap(ctx);
  for (uint32_t j = 0; j < ctx->dnum && !rc; j++) {
    uint64_t *b = key->data + (size_t)2 * j * nm * n;
    uint64_t *ak = b + (size_t)nm * n;
    sample_uniform_limbs(ctx, tag + "/a/" + std::to_string(j), seed, nm, mod_of, a);
    sample_gaussian(tag + "/e/" + std::to_string(j), seed, e.data(), n);
    rc = upload(ctx, ak, a.data(), a.size() * 8);
    if (!rc) rc = embed_small_host(ctx, b, e, poly_rows(1, nm, nm));
    if (!rc) rc = ntt_forward_rows(ctx, b, poly_rows(2, nm, nm));
    // b = e - a s
    if (!rc) rc = launch_mul_mont(ctx, tmp, ak, sk->data, full, 0);
    if (!rc) rc = launch_addsub(ctx, b, b, tmp, full, 1);
    // + (P mod q_i) s' on the limbs of digit j
    const uint32_t lo = j * ctx->alpha, hi = std::min(L, lo + ctx->alpha);
    if (!rc && lo < hi) {
      LimbMap m;
      RowScale sc;
      m.n = hi - lo;
      for (uint32_t i = lo; i < hi; i++) {
        const uint64_t q = ctx->mods[i];
        uint64_t pm = 1;
        for (uint32_t k = 0; k < K; k++) pm = h_mulmod(pm, ctx->mods[L + k] % q, q);
        m.row[i - lo] = (uint16_t)i;
        m.mod[i - lo] = (uint8_t)i;
        sc.w[i - lo] = pm;
        sc.wp[i - lo] = 0;
        sc.add[i - lo] = 0;
      }
      rc = launch_scalar_mac(ctx, b, sp_m, m, sc);
    }
    if (!rc) rc = mont_rows(ctx, b, poly_rows(2, nm, nm), true);
  }
  if (rc) {
    dev_free(ctx, key->data);
    delete key;
    return rc;
  }
  *out = key;
  return HCK_OK;
}

int lt_alloc_ct(hck_context *ctx, hck_ciphertext **ct) {
  *ct = new hck_ciphertext();
  (*ct)->ctx = ctx;
  return ensure_ct(ctx, *ct, 2);
}

}  // namespace

namespace hck {

int key_rows_to_internal(hck_context *ctx, uint64_t *buf) {
  const uint32_t nm = ctx->L + ctx->K;
  const auto rows = poly_rows(2 * ctx->dnum, nm, nm, 0);
  TRY(ntt_forward_rows(ctx, buf, rows));
  return mont_rows(ctx, buf, rows, true);
}

int ct_from_host_async(hck_context *ctx, hck_ciphertext *ct, const uint64_t *host,
                       uint32_t polys, uint32_t level, double scale) {
  if (level >= ctx->L) return set_error(HCK_ELEVEL, "level beyond the chain");
  if (ctx->capturing) return set_error(HCK_EINVAL, "host transfer during graph capture");
  TRY(ensure_ct(ctx, ct, polys));
  const size_t n = ctx->n, rows = level + 1;
  for (uint32_t p = 0; p < polys; p++)
    HCK_HIP(ctx, hipMemcpyAsync(ct->data + (size_t)p * ctx->L * n, host + p * rows * n,
                                rows * n * 8, hipMemcpyHostToDevice, ctx->stream));
  TRY(ntt_forward_rows(ctx, ct->data, poly_rows(polys, ctx->L, level + 1)));
  ct->size = polys;
  ct->level = level;
  ct->scale = scale;
  return HCK_OK;
}

int ct_to_host_async(hck_context *ctx, const hck_ciphertext *ct, uint64_t *host) {
  const size_t n = ctx->n, rows = ct->level + 1, words = (size_t)ct->size * rows * n;
  uint64_t *tmp = nullptr;
  TRY(dev_alloc(ctx, &tmp, words));
  int rc = HCK_OK;
  for (uint32_t p = 0; p < ct->size && !rc; p++)
    rc = launch_copy(ctx, tmp + p * rows * n, ct->data + (size_t)p * ctx->L * n, rows * n);
  if (!rc) rc = inverse_rows(ctx, tmp, poly_rows(ct->size, ct->level + 1, ct->level + 1));
  if (!rc) {
    hipError_t e = hipMemcpyAsync(host, tmp, words * 8, hipMemcpyDeviceToHost, ctx->stream);
    if (e != hipSuccess) rc = check_hip(ctx, e, "device-to-host copy");
  }
  dev_free(ctx, tmp);
  return rc;
}

int relinearize_keys(hck_context *ctx, const hck_ciphertext *const *a,
                     const hck_switch_key *const *rlk, uint32_t n, hck_ciphertext *const *out) {
  if (n == 0) return HCK_OK;
  for (uint32_t i = 0; i < n; i++) {
    if (!a[i] || !out[i] || !rlk[i]) return set_error(HCK_EINVAL, "null ciphertext or key");
    if (a[i]->size != 3) return set_error(HCK_EINVAL, "relinearization needs a 3-part ciphertext");
    if (a[i]->level != a[0]->level) return set_error(HCK_ELEVEL, "batched inputs need one level");
    for (uint32_t k = 0; k < n; k++)
      if ((k < i && out[k] == out[i]) || (k != i && out[k] == a[i]))
        return set_error(HCK_EINVAL, "outputs must be distinct and alias only their own input");
  }
  const uint32_t level = a[0]->level;
  const size_t ps = poly_stride(ctx);
  const uint32_t limit = ks_batch_limit(ctx, level);
  for (uint32_t s0 = 0; s0 < n; s0 += even_batch(n - s0, limit)) {
    KsBatch kb;
    kb.n = even_batch(n - s0, limit);
    std::vector<double> scales(kb.n);
    for (uint32_t b = 0; b < kb.n; b++) {
      const hck_ciphertext *x = a[s0 + b];
      hck_ciphertext *y = out[s0 + b];
      scales[b] = x->scale;
      TRY(ensure_ct(ctx, y, 2));
      // (d0, d1) + KeySwitch(d2): d2 is read before the final launch writes
      // the outputs, and the addends are read at the positions written
      kb.key[b] = rlk[s0 + b]->data;
      kb.galois[b] = 1;
      kb.d[b] = x->data + 2 * ps;
      kb.out0[b] = y->data;
      kb.out1[b] = y->data + ps;
      kb.add0[b] = x->data;
      kb.add1[b] = x->data + ps;
    }
    TRY(keyswitch_batch(ctx, kb, level));
    for (uint32_t b = 0; b < kb.n; b++) {
      out[s0 + b]->size = 2;
      out[s0 + b]->level = level;
      out[s0 + b]->scale = scales[b];
    }
  }
  return HCK_OK;
}

}  // namespace hck

extern "C" {

/* ---- keys -------------------------------------------------------------------- */

int hck_keygen_secret(hck_context *ctx, uint64_t seed, hck_secret_key **out) {
  ENTER(ctx);
  if (!out) return set_error(HCK_EINVAL, "null output");
  std::vector<int32_t> s(ctx->n);
  sample_ternary("sk", seed, s.data(), ctx->n);
  std::vector<int8_t> c(s.begin(), s.end());
  return hck_secret_key_import(ctx, c.data(), out);
}

int hck_secret_key_import(hck_context *ctx, const int8_t *coeffs, hck_secret_key **out) {
  ENTER(ctx);
  if (!coeffs || !out) return set_error(HCK_EINVAL, "null argument");
  const uint32_t nm = ctx->L + ctx->K;
  std::vector<int32_t> v(ctx->n);
  for (uint32_t i = 0; i < ctx->n; i++) {
    if (coeffs[i] < -1 || coeffs[i] > 1) return set_error(HCK_EINVAL, "secret not ternary");
    v[i] = coeffs[i];
  }
  TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
  hck_secret_key *sk = new hck_secret_key();
  sk->ctx = ctx;
  sk->coeffs.assign(coeffs, coeffs + ctx->n);
  int rc = dev_alloc(ctx, &sk->data, (size_t)nm * ctx->n);
  auto rows = poly_rows(1, nm, nm);
  if (!rc) rc = embed_small_host(ctx, sk->data, v, rows);
  if (!rc) rc = ntt_forward_rows(ctx, sk->data, rows);
  if (!rc) rc = mont_rows(ctx, sk->data, rows, true);
  if (rc) {
    dev_free(ctx, sk->data);
    delete sk;
    return rc;
  }
  track(ctx, sk, release_data<hck_secret_key>);
  *out = sk;
  return HCK_OK;
}

int hck_secret_key_destroy(hck_secret_key *sk) {
  if (sk) {
    if (sk->ctx) untrack(sk->ctx, sk);
    release_data<hck_secret_key>(sk);
    delete sk;
  }
  return HCK_OK;
}

int hck_keygen_public(hck_context *ctx, const hck_secret_key *sk, uint64_t seed,
                      hck_public_key **out) {
  ENTER(ctx);
  OWNED(ctx, sk);
  if (!sk || !out) return set_error(HCK_EINVAL, "null argument");
  TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
  const size_t n = ctx->n;
  const uint32_t L = ctx->L;
  hck_public_key *pk = new hck_public_key();
  pk->ctx = ctx;
  int rc = dev_alloc(ctx, &pk->data, (size_t)2 * L * n);
  std::vector<uint32_t> mod_of(L);
  for (uint32_t t = 0; t < L; t++) mod_of[t] = t;
  std::vector<uint64_t> a;
  std::vector<int32_t> e(n);
  sample_uniform_limbs(ctx, "pk_a", seed, L, mod_of, a);
  sample_gaussian("pk_e", seed, e.data(), n);
  uint64_t *b = pk->data, *ak = pk->data + (size_t)L * n, *tmp = ws_tmp(ctx);
  const LimbMap qm = qmap(ctx, L - 1);
  if (!rc) rc = upload(ctx, ak, a.data(), a.size() * 8);
  if (!rc) rc = embed_small_host(ctx, b, e, poly_rows(1, L, L));
  if (!rc) rc = ntt_forward_rows(ctx, b, poly_rows(2, L, L));
  if (!rc) rc = launch_mul_mont(ctx, tmp, ak, sk->data, qm, 0);
  if (!rc) rc = launch_addsub(ctx, b, b, tmp, qm, 1);
  if (!rc) rc = mont_rows(ctx, pk->data, poly_rows(2, L, L), true);
  if (rc) {
    dev_free(ctx, pk->data);
    delete pk;
    return rc;
  }
  track(ctx, pk, release_data<hck_public_key>);
  *out = pk;
  return HCK_OK;
}

int hck_public_key_export(hck_context *ctx, const hck_public_key *pk, uint64_t *out,
                          size_t n_words) {
  ENTER(ctx);
  OWNED(ctx, pk);
  if (!pk || !out) return set_error(HCK_EINVAL, "null argument");
  if (n_words != (size_t)2 * ctx->L * ctx->n) return set_error(HCK_EINVAL, "size mismatch");
  return export_rows(ctx, pk->data, 2, ctx->L, ctx->L, true, 0, out);
}

int hck_public_key_destroy(hck_public_key *pk) {
  if (pk) {
    if (pk->ctx) untrack(pk->ctx, pk);
    release_data<hck_public_key>(pk);
    delete pk;
  }
  return HCK_OK;
}

int hck_keygen_relin(hck_context *ctx, const hck_secret_key *sk, uint64_t seed,
                     hck_switch_key **out) {
  ENTER(ctx);
  OWNED(ctx, sk);
  if (!sk || !out) return set_error(HCK_EINVAL, "null argument");
  TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
  // s^2 in Montgomery form: REDC(s~ s~) = s^2 2^64
  uint64_t *s2 = ws_rot(ctx);  // [L+K][N] fits in [2][L][N] when K <= L
  uint64_t *own = nullptr;
  if (ctx->K > ctx->L) {
    TRY(dev_alloc(ctx, &own, (size_t)(ctx->L + ctx->K) * ctx->n));
    s2 = own;
  }
  int rc = launch_mul_mont(ctx, s2, sk->data, sk->data, fullmap(ctx), 0);
  if (!rc) rc = make_switch_key(ctx, sk, s2, "rlk", seed, out);
  dev_free(ctx, own);
  if (!rc) track(ctx, *out, release_data<hck_switch_key>);
  return rc;
}

int hck_switch_key_export(hck_context *ctx, const hck_switch_key *swk, uint64_t *out,
                          size_t n_words) {
  ENTER(ctx);
  OWNED(ctx, swk);
  if (!swk || !out) return set_error(HCK_EINVAL, "null argument");
  if (n_words != (size_t)ctx->dnum * 2 * (ctx->L + ctx->K) * ctx->n)
    return set_error(HCK_EINVAL, "size mismatch");
  return export_key_rows(ctx, swk->data, 2 * ctx->dnum, out);
}

int hck_switch_key_destroy(hck_switch_key *swk) {
  if (swk) {
    if (swk->ctx) untrack(swk->ctx, swk);
    release_data<hck_switch_key>(swk);
    delete swk;
  }
  return HCK_OK;
}

int hck_switch_key_import(hck_context *ctx, const uint64_t *words, size_t n_words,
                          hck_switch_key **out) {
  ENTER(ctx);
  if (!words || !out) return set_error(HCK_EINVAL, "null argument");
  const uint32_t nm = ctx->L + ctx->K;
  const size_t total = (size_t)ctx->dnum * 2 * nm * ctx->n;
  if (n_words != total) return set_error(HCK_EINVAL, "size mismatch");
  for (size_t r = 0; r < (size_t)ctx->dnum * 2 * nm; r++) {
    const uint64_t q = ctx->mods[r % nm];
    for (size_t c = 0; c < ctx->n; c++)
      if (words[r * ctx->n + c] >= q) return set_error(HCK_EINVAL, "residue not below its prime");
  }
  hck_switch_key *key = new hck_switch_key();
  key->ctx = ctx;
  int rc = dev_alloc(ctx, &key->data, total);
  if (!rc) rc = upload(ctx, key->data, words, total * 8);
  if (!rc) rc = key_rows_to_internal(ctx, key->data);
  if (rc) {
    hck_switch_key_destroy(key);
    return rc;
  }
  track(ctx, key, release_data<hck_switch_key>);
  *out = key;
  return HCK_OK;
}

int hck_galois_keys_create(hck_context *ctx, hck_galois_keys **out) {
  if (!ctx || !out) return set_error(HCK_EINVAL, "null argument");
  hck_galois_keys *gks = new hck_galois_keys();
  gks->ctx = ctx;
  track(ctx, gks, release_gks);
  *out = gks;
  return HCK_OK;
}

int hck_galois_keys_insert(hck_galois_keys *gks, uint32_t element, hck_switch_key *swk) {
  if (!gks || !swk) return set_error(HCK_EINVAL, "null argument");
  if ((element & 1) == 0 || element >= 2 * gks->ctx->n)
    return set_error(HCK_EINVAL, "Galois element must be odd and below 2N");
  if (!gks->ctx || swk->ctx != gks->ctx) return set_error(HCK_EINVAL, "key of another context");
  auto it = gks->keys.find(element);
  if (it != gks->keys.end() && it->second == swk) return HCK_OK;
  untrack(gks->ctx, swk);   // owned by the set from now on
  if (it != gks->keys.end()) hck_switch_key_destroy(it->second);
  gks->keys[element] = swk;
  return HCK_OK;
}

int hck_keygen_galois(hck_context *ctx, const hck_secret_key *sk, const uint32_t *elements,
                      uint32_t n, uint64_t seed, hck_galois_keys **out) {
  ENTER(ctx);
  OWNED(ctx, sk);
  if (!sk || !out || (n && !elements)) return set_error(HCK_EINVAL, "null argument");
  for (uint32_t i = 0; i < n; i++)
    if ((elements[i] & 1) == 0 || elements[i] >= 2 * ctx->n)
      return set_error(HCK_EINVAL, "Galois element must be odd and below 2N");
  TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
  const uint32_t nm = ctx->L + ctx->K;
  uint64_t *sg = nullptr;
  TRY(dev_alloc(ctx, &sg, (size_t)nm * ctx->n));
  hck_galois_keys *gks = new hck_galois_keys();
  gks->ctx = ctx;
  int rc = HCK_OK;
  for (uint32_t i = 0; i < n && !rc; i++) {
    const uint32_t g = elements[i];
    if (gks->keys.count(g)) continue;
    rc = launch_automorphism(ctx, sg, sk->data, 0, 1, fullmap(ctx), g);
    hck_switch_key *key = nullptr;
    if (!rc) rc = make_switch_key(ctx, sk, sg, "gk/" + std::to_string(g), seed, &key);
    if (!rc) gks->keys[g] = key;
  }
  dev_free(ctx, sg);
  if (rc) {
    hck_galois_keys_destroy(gks);
    return rc;
  }
  track(ctx, gks, release_gks);
  *out = gks;
  return HCK_OK;
}

int hck_keygen_rotation(hck_context *ctx, const hck_secret_key *sk, const int32_t *steps,
                        uint32_t n, uint64_t seed, hck_galois_keys **out) {
  ENTER(ctx);
  OWNED(ctx, sk);
  if (n && !steps) return set_error(HCK_EINVAL, "null steps");
  std::vector<uint32_t> el;
  for (uint32_t i = 0; i < n; i++)
    if (((int64_t)steps[i] % (ctx->n / 2)) != 0) el.push_back(galois_of_step(ctx, steps[i]));
  return hck_keygen_galois(ctx, sk, el.data(), (uint32_t)el.size(), seed, out);
}

int hck_galois_keys_export(hck_context *ctx, const hck_galois_keys *gks, uint32_t element,
                           uint64_t *out, size_t n_words) {
  ENTER(ctx);
  OWNED(ctx, gks);
  if (!gks) return set_error(HCK_EINVAL, "null keys");
  auto it = gks->keys.find(element);
  if (it == gks->keys.end()) return set_error(HCK_ENOKEY, "no key for this element");
  return hck_switch_key_export(ctx, it->second, out, n_words);
}

int hck_galois_keys_count(const hck_galois_keys *gks, uint32_t *n) {
  if (!gks || !n) return set_error(HCK_EINVAL, "null argument");
  *n = (uint32_t)gks->keys.size();
  return HCK_OK;
}

int hck_galois_keys_destroy(hck_galois_keys *gks) {
  if (gks) {
    if (gks->ctx) untrack(gks->ctx, gks);
    for (auto &kv : gks->keys) hck_switch_key_destroy(kv.second);
    delete gks;
  }
  return HCK_OK;
}

/* ---- plaintexts ------------------------------------------------------------- */

static int plaintext_from_rows(hck_context *ctx, const uint64_t *res, uint32_t level, double scale,
                               hck_plaintext **out) {
  hck_plaintext *pt = new hck_plaintext();
  pt->ctx = ctx;
  pt->level = level;
  pt->scale = scale;
  int rc = dev_alloc(ctx, &pt->data, (size_t)(level + 1) * ctx->n);
  if (!rc) rc = import_rows(ctx, pt->data, res, 1, level + 1, level + 1);
  if (!rc) rc = mont_rows(ctx, pt->data, poly_rows(1, level + 1, level + 1), true);
  if (rc) {
    dev_free(ctx, pt->data);
    delete pt;
    return rc;
  }
  track(ctx, pt, release_data<hck_plaintext>);
  *out = pt;
  return HCK_OK;
}

int hck_plaintext_import(hck_context *ctx, const uint64_t *res, uint32_t level, double scale,
                         hck_plaintext **out) {
  ENTER(ctx);
  if (!res || !out) return set_error(HCK_EINVAL, "null argument");
  if (level >= ctx->L) return set_error(HCK_ELEVEL, "level beyond the chain");
  return plaintext_from_rows(ctx, res, level, scale, out);
}

static void coeffs_to_residues(const hck_context *ctx, const std::vector<int64_t> &c,
                               uint32_t level, std::vector<uint64_t> &res) {
  const size_t n = ctx->n;
  res.resize((size_t)(level + 1) * n);
  for (uint32_t i = 0; i <= level; i++) {
    const uint64_t q = ctx->mods[i];
    for (size_t k = 0; k < n; k++) {
      const int64_t v = c[k];
      const uint64_t mag = (uint64_t)(v < 0 ? -v : v) % q;
      res[(size_t)i * n + k] = (v < 0 && mag) ? q - mag : mag;
    }
  }
}

int hck_encode_const(hck_context *ctx, double value, double scale, uint32_t level,
                     hck_plaintext **out) {
  ENTER(ctx);
  if (!out) return set_error(HCK_EINVAL, "null argument");
  if (level >= ctx->L) return set_error(HCK_ELEVEL, "level beyond the chain");
  const double v = value * scale;
  if (!(std::fabs(v) < 9.2e18)) return set_error(HCK_EINVAL, "constant times scale beyond 2^63");
  std::vector<int64_t> c(ctx->n, 0);
  c[0] = (int64_t)std::copysign(std::floor(std::fabs(v) + 0.5), v);  // half away from zero
  std::vector<uint64_t> res;
  coeffs_to_residues(ctx, c, level, res);
  return plaintext_from_rows(ctx, res.data(), level, scale, out);
}

int hck_encode(hck_context *ctx, const double *re, const double *im, uint32_t n_slots,
               double scale, uint32_t level, hck_plaintext **out) {
  ENTER(ctx);
  if (!re || !out) return set_error(HCK_EINVAL, "null argument");
  if (n_slots != ctx->n / 2) return set_error(HCK_EINVAL, "n_slots must be N/2");
  if (level >= ctx->L) return set_error(HCK_ELEVEL, "level beyond the chain");
  std::vector<int64_t> c;
  TRY(encode_coeffs(ctx->log_n, re, im, scale, c));
  std::vector<uint64_t> res;
  coeffs_to_residues(ctx, c, level, res);
  return plaintext_from_rows(ctx, res.data(), level, scale, out);
}

int hck_plaintext_export(hck_context *ctx, const hck_plaintext *pt, uint64_t *out,
                         size_t n_words, uint32_t *level, double *scale) {
  ENTER(ctx);
  OWNED(ctx, pt);
  if (!pt || !out) return set_error(HCK_EINVAL, "null argument");
  if (n_words < (size_t)(pt->level + 1) * ctx->n) return set_error(HCK_EINVAL, "buffer too small");
  if (level) *level = pt->level;
  if (scale) *scale = pt->scale;
  return export_rows(ctx, pt->data, 1, pt->level + 1, pt->level + 1, true, 0, out);
}

int hck_decode(hck_context *ctx, const hck_plaintext *pt, double *re, double *im,
               uint32_t n_slots) {
  ENTER(ctx);
  OWNED(ctx, pt);
  if (!pt) return set_error(HCK_EINVAL, "null plaintext");
  if (n_slots != ctx->n / 2) return set_error(HCK_EINVAL, "n_slots must be N/2");
  std::vector<uint64_t> res((size_t)(pt->level + 1) * ctx->n);
  TRY(hck_plaintext_export(ctx, pt, res.data(), res.size(), nullptr, nullptr));
  decode_residues(ctx->log_n, res.data(), ctx->mods.data(), pt->level + 1, pt->scale, re, im);
  return HCK_OK;
}

int hck_plaintext_destroy(hck_plaintext *pt) {
  if (pt) {
    if (pt->ctx) untrack(pt->ctx, pt);
    release_data<hck_plaintext>(pt);
    delete pt;
  }
  return HCK_OK;
}

/* ---- ciphertexts ---------------------------------------------------------- */

int hck_ciphertext_create(hck_context *ctx, hck_ciphertext **out) {
  ENTER(ctx);
  if (!out) return set_error(HCK_EINVAL, "null output");
  hck_ciphertext *ct = new hck_ciphertext();
  ct->ctx = ctx;
  track(ctx, ct, release_ct);
  *out = ct;
  return HCK_OK;
}

int hck_ciphertext_import(hck_context *ctx, const uint64_t *res, uint32_t size, uint32_t level,
                          double scale, hck_ciphertext **out) {
  ENTER(ctx);
  if (!res || !out) return set_error(HCK_EINVAL, "null argument");
  if (size != 2 && size != 3) return set_error(HCK_EINVAL, "size must be 2 or 3");
  if (level >= ctx->L) return set_error(HCK_ELEVEL, "level beyond the chain");
  hck_ciphertext *ct = new hck_ciphertext();
  ct->ctx = ctx;
  int rc = ensure_ct(ctx, ct, size);
  if (!rc) rc = import_rows(ctx, ct->data, res, size, ctx->L, level + 1);
  if (rc) {
    hck_ciphertext_destroy(ct);
    return rc;
  }
  ct->size = size;
  ct->level = level;
  ct->scale = scale;
  track(ctx, ct, release_ct);
  *out = ct;
  return HCK_OK;
}

int hck_ciphertext_export(hck_context *ctx, const hck_ciphertext *ct, uint64_t *out,
                          size_t n_words, uint32_t *size, uint32_t *level, double *scale) {
  ENTER(ctx);
  OWNED(ctx, ct);
  if (!ct || !out) return set_error(HCK_EINVAL, "null argument");
  if (ct->size == 0) return set_error(HCK_EINVAL, "empty ciphertext");
  if (n_words < (size_t)ct->size * (ct->level + 1) * ctx->n)
    return set_error(HCK_EINVAL, "buffer too small");
  if (size) *size = ct->size;
  if (level) *level = ct->level;
  if (scale) *scale = ct->scale;
  return export_rows(ctx, ct->data, ct->size, ctx->L, ct->level + 1, false, 0, out);
}

int hck_ciphertext_info(const hck_ciphertext *ct, uint32_t *size, uint32_t *level,
                        double *scale) {
  if (!ct) return set_error(HCK_EINVAL, "null ciphertext");
  if (size) *size = ct->size;
  if (level) *level = ct->level;
  if (scale) *scale = ct->scale;
  return HCK_OK;
}

int hck_ciphertext_destroy(hck_ciphertext *ct) {
  if (ct) {
    if (ct->ctx) untrack(ct->ctx, ct);
    release_ct(ct);
    delete ct;
  }
  return HCK_OK;
}

int hck_encrypt_sk(hck_context *ctx, const hck_secret_key *sk, const hck_plaintext *pt,
                   uint64_t seed, hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, sk);
  OWNED(ctx, pt);
  OWNED(ctx, out);
  if (!sk || !pt || !out) return set_error(HCK_EINVAL, "null argument");
  TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
  TRY(ensure_ct(ctx, out, 2));
  const size_t n = ctx->n, ps = poly_stride(ctx);
  const uint32_t nq = pt->level + 1;
  std::vector<uint32_t> mod_of(nq);
  for (uint32_t t = 0; t < nq; t++) mod_of[t] = t;
  std::vector<uint64_t> a;
  std::vector<int32_t> e(n);
  sample_uniform_limbs(ctx, "enc_a", seed, nq, mod_of, a);
  sample_gaussian("enc_e", seed, e.data(), n);
  uint64_t *c0 = out->data, *c1 = out->data + ps, *tmp = ws_tmp(ctx);
  const LimbMap qm = qmap(ctx, pt->level);
  TRY(upload(ctx, c1, a.data(), a.size() * 8));
  TRY(embed_small_host(ctx, c0, e, poly_rows(1, ctx->L, nq)));
  TRY(ntt_forward_rows(ctx, c0, poly_rows(2, ctx->L, nq)));
  // c0 = e + m - a s
  TRY(launch_mul_mont(ctx, tmp, c1, sk->data, qm, 0));
  TRY(launch_addsub(ctx, c0, c0, tmp, qm, 1));
  TRY(launch_copy(ctx, tmp, pt->data, (size_t)nq * n));
  TRY(launch_to_mont(ctx, tmp, qm, false));
  TRY(launch_addsub(ctx, c0, c0, tmp, qm, 0));
  out->size = 2;
  out->level = pt->level;
  out->scale = pt->scale;
  return HCK_OK;
}

int hck_encrypt_pk(hck_context *ctx, const hck_public_key *pk, const hck_plaintext *pt,
                   uint64_t seed, hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, pk);
  OWNED(ctx, pt);
  OWNED(ctx, out);
  if (!pk || !pt || !out) return set_error(HCK_EINVAL, "null argument");
  TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
  TRY(ensure_ct(ctx, out, 2));
  const size_t n = ctx->n, ps = poly_stride(ctx);
  const uint32_t nq = pt->level + 1;
  std::vector<int32_t> v(n), e0(n), e1(n);
  sample_ternary("enc_v", seed, v.data(), n);
  sample_gaussian("enc_e0", seed, e0.data(), n);
  sample_gaussian("enc_e1", seed, e1.data(), n);
  uint64_t *c0 = out->data, *c1 = out->data + ps, *tmp = ws_tmp(ctx);
  uint64_t *vv = tmp + (size_t)ctx->L * n;
  const LimbMap qm = qmap(ctx, pt->level);
  TRY(embed_small_host(ctx, vv, v, poly_rows(1, ctx->L, nq)));
  TRY(embed_small_host(ctx, c0, e0, poly_rows(1, ctx->L, nq)));
  TRY(embed_small_host(ctx, c1, e1, poly_rows(1, ctx->L, nq)));
  TRY(ntt_forward_rows(ctx, c0, poly_rows(2, ctx->L, nq)));
  TRY(ntt_forward_rows(ctx, vv, poly_rows(1, ctx->L, nq)));
  TRY(launch_mul_mont(ctx, c0, vv, pk->data, qm, 1));
  TRY(launch_mul_mont(ctx, c1, vv, pk->data + ps, qm, 1));
  TRY(launch_copy(ctx, tmp, pt->data, (size_t)nq * n));
  TRY(launch_to_mont(ctx, tmp, qm, false));
  TRY(launch_addsub(ctx, c0, c0, tmp, qm, 0));
  out->size = 2;
  out->level = pt->level;
  out->scale = pt->scale;
  return HCK_OK;
}

int hck_decrypt(hck_context *ctx, const hck_secret_key *sk, const hck_ciphertext *ct,
                hck_plaintext **out) {
  ENTER(ctx);
  OWNED(ctx, sk);
  OWNED(ctx, ct);
  if (!sk || !ct || !out) return set_error(HCK_EINVAL, "null argument");
  if (ct->size < 2) return set_error(HCK_EINVAL, "empty ciphertext");
  TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
  const size_t n = ctx->n, ps = poly_stride(ctx);
  const uint32_t nq = ct->level + 1;
  const LimbMap qm = qmap(ctx, ct->level);
  hck_plaintext *pt = new hck_plaintext();
  pt->ctx = ctx;
  pt->level = ct->level;
  pt->scale = ct->scale;
  int rc = dev_alloc(ctx, &pt->data, (size_t)nq * n);
  uint64_t *tmp = ws_tmp(ctx);
  // m = c0 + REDC(c1 s~) (+ REDC(c2 REDC(s~ s~)))
  if (!rc) rc = launch_copy(ctx, pt->data, ct->data, (size_t)nq * n);
  if (!rc) rc = launch_mul_mont(ctx, pt->data, ct->data + ps, sk->data, qm, 1);
  if (!rc && ct->size == 3) {
    rc = launch_mul_mont(ctx, tmp, sk->data, sk->data, qm, 0);
    if (!rc) rc = launch_mul_mont(ctx, pt->data, ct->data + 2 * ps, tmp, qm, 1);
  }
  if (!rc) rc = launch_to_mont(ctx, pt->data, qm, true);
  if (rc) {
    hck_plaintext_destroy(pt);
    return rc;
  }
  track(ctx, pt, release_data<hck_plaintext>);
  *out = pt;
  return HCK_OK;
}

/* ---- evaluation ---------------------------------------------------------------- */

static int addsub_ct(hck_context *ctx, const hck_ciphertext *a, const hck_ciphertext *b,
                     hck_ciphertext *out, int op) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, b);
  OWNED(ctx, out);
  if (!a || !b || !out) return set_error(HCK_EINVAL, "null argument");
  if (a->size == 0 || a->size != b->size) return set_error(HCK_EINVAL, "sizes differ");
  if (a->level != b->level) return set_error(HCK_ELEVEL, "levels differ");
  if (!scales_match(a->scale, b->scale)) return set_error(HCK_ESCALE, "scales differ");
  const uint32_t size = a->size, level = a->level;
  const double scale = a->scale;
  TRY(ensure_ct(ctx, out, size));
  const size_t ps = poly_stride(ctx);
  for (uint32_t p = 0; p < size; p++)
    TRY(launch_addsub(ctx, out->data + p * ps, a->data + p * ps, b->data + p * ps,
                      qmap(ctx, level), op));
  out->size = size;
  out->level = level;
  out->scale = scale;
  return HCK_OK;
}

int hck_add(hck_context *ctx, const hck_ciphertext *a, const hck_ciphertext *b,
            hck_ciphertext *out) {
  return addsub_ct(ctx, a, b, out, 0);
}

int hck_sub(hck_context *ctx, const hck_ciphertext *a, const hck_ciphertext *b,
            hck_ciphertext *out) {
  return addsub_ct(ctx, a, b, out, 1);
}

int hck_add_plain(hck_context *ctx, const hck_ciphertext *a, const hck_plaintext *pt,
                  hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, pt);
  OWNED(ctx, out);
  if (!a || !pt || !out) return set_error(HCK_EINVAL, "null argument");
  if (a->size == 0) return set_error(HCK_EINVAL, "empty ciphertext");
  if (pt->level < a->level) return set_error(HCK_ELEVEL, "plaintext level below ciphertext level");
  if (!scales_match(a->scale, pt->scale)) return set_error(HCK_ESCALE, "scales differ");
  TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
  const uint32_t size = a->size, level = a->level;
  const double scale = a->scale;
  TRY(ensure_ct(ctx, out, size));
  const size_t n = ctx->n, ps = poly_stride(ctx);
  uint64_t *tmp = ws_tmp(ctx);
  const LimbMap qm = qmap(ctx, level);
  TRY(launch_copy(ctx, tmp, pt->data, (size_t)(level + 1) * n));
  TRY(launch_to_mont(ctx, tmp, qm, false));
  TRY(launch_addsub(ctx, out->data, a->data, tmp, qm, 0));
  for (uint32_t p = 1; p < size; p++)
    TRY(launch_copy(ctx, out->data + p * ps, a->data + p * ps, (size_t)(level + 1) * n));
  out->size = size;
  out->level = level;
  out->scale = scale;
  return HCK_OK;
}

int hck_mul_plain(hck_context *ctx, const hck_ciphertext *a, const hck_plaintext *pt,
                  hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, pt);
  OWNED(ctx, out);
  if (!a || !pt || !out) return set_error(HCK_EINVAL, "null argument");
  if (a->size == 0) return set_error(HCK_EINVAL, "empty ciphertext");
  if (pt->level < a->level) return set_error(HCK_ELEVEL, "plaintext level below ciphertext level");
  const uint32_t size = a->size, level = a->level;
  const double scale = a->scale * pt->scale;
  TRY(ensure_ct(ctx, out, size));
  const size_t ps = poly_stride(ctx);
  for (uint32_t p = 0; p < size; p++)
    TRY(launch_mul_mont(ctx, out->data + p * ps, a->data + p * ps, pt->data, qmap(ctx, level),
                        0));
  out->size = size;
  out->level = level;
  out->scale = scale;
  return HCK_OK;
}

int hck_drop_level(hck_context *ctx, const hck_ciphertext *a, uint32_t level,
                   hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, out);
  if (!a || !out) return set_error(HCK_EINVAL, "null argument");
  if (a->size == 0) return set_error(HCK_EINVAL, "empty ciphertext");
  if (level > a->level) return set_error(HCK_ELEVEL, "cannot raise the level");
  const uint32_t size = a->size;
  const double scale = a->scale;
  if (out != a) {
    TRY(ensure_ct(ctx, out, size));
    const size_t ps = poly_stride(ctx);
    for (uint32_t p = 0; p < size; p++)
      TRY(launch_copy(ctx, out->data + p * ps, a->data + p * ps, (size_t)(level + 1) * ctx->n));
  }
  out->size = size;
  out->level = level;
  out->scale = scale;
  return HCK_OK;
}

int hck_mul(hck_context *ctx, const hck_ciphertext *a, const hck_ciphertext *b,
            hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, b);
  OWNED(ctx, out);
  if (!a || !b || !out) return set_error(HCK_EINVAL, "null argument");
  if (a->size != 2 || b->size != 2) return set_error(HCK_EINVAL, "mul needs 2-part ciphertexts");
  if (a->level != b->level) return set_error(HCK_ELEVEL, "levels differ");
  const uint32_t level = a->level;
  const double scale = a->scale * b->scale;
  TRY(ensure_ct(ctx, out, 3));
  TRY(launch_tensor(ctx, out->data, a->data, b->data, poly_stride(ctx), qmap(ctx, level)));
  out->size = 3;
  out->level = level;
  out->scale = scale;
  return HCK_OK;
}

int hck_relinearize(hck_context *ctx, const hck_ciphertext *a, const hck_switch_key *rlk,
                    hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, rlk);
  OWNED(ctx, out);
  if (!a || !rlk || !out) return set_error(HCK_EINVAL, "null argument");
  if (a->size != 3) return set_error(HCK_EINVAL, "relinearization needs a 3-part ciphertext");
  const uint32_t level = a->level;
  const double scale = a->scale;
  TRY(ensure_ct(ctx, out, 2));
  const size_t ps = poly_stride(ctx);
  TRY(keyswitch_core(ctx, a->data + 2 * ps, 1, level, rlk, out->data, out->data + ps, a->data,
                     a->data + ps));
  out->size = 2;
  out->level = level;
  out->scale = scale;
  return HCK_OK;
}

int hck_relinearize_many(hck_context *ctx, const hck_ciphertext *const *a, uint32_t n,
                         const hck_switch_key *rlk, hck_ciphertext *const *out) {
  ENTER(ctx);
  OWNED(ctx, rlk);
  if ((n && (!a || !out)) || !rlk) return set_error(HCK_EINVAL, "null argument");
  for (uint32_t i = 0; i < n; i++) {
    OWNED(ctx, a[i]);
    OWNED(ctx, out[i]);
  }
  std::vector<const hck_switch_key *> keys(n, rlk);
  return relinearize_keys(ctx, a, keys.data(), n, out);
}

int hck_rescale(hck_context *ctx, const hck_ciphertext *a, hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, out);
  if (!a || !out) return set_error(HCK_EINVAL, "null argument");
  if (a->size == 0) return set_error(HCK_EINVAL, "empty ciphertext");
  if (a->level == 0) return set_error(HCK_ELEVEL, "no level left to rescale");
  TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
  const uint32_t size = a->size, level = a->level;
  const double scale = a->scale / (double)ctx->mods[level];
  TRY(ensure_ct(ctx, out, size));
  const size_t n = ctx->n, ps = poly_stride(ctx);
  uint64_t *last = ws_tmp(ctx);
  uint64_t *lift = last + (size_t)size * n;
  std::vector<std::pair<uint16_t, uint8_t>> lrows;
  for (uint32_t p = 0; p < size; p++) {
    TRY(launch_copy(ctx, last + p * n, a->data + p * ps + (size_t)level * n, n));
    lrows.push_back({(uint16_t)p, (uint8_t)level});
  }
  // dropped limb to coefficient form; then per target limb its centred lift,
  // forward transform and (c_i - t) q_l^-1, in two fused passes
  TRY(ntt_inverse(ctx, last, make_map(lrows, 0), nullptr));
  TRY(rescale_fused(ctx, out->data, a->data, last, lift, level, size));
  out->size = size;
  out->level = level - 1;
  out->scale = scale;
  return HCK_OK;
}

int hck_rotate(hck_context *ctx, const hck_ciphertext *a, int32_t step,
               const hck_galois_keys *gks, hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, gks);
  OWNED(ctx, out);
  if (!a || !out) return set_error(HCK_EINVAL, "null argument");
  if ((int64_t)step % (ctx->n / 2) == 0) {
    if (a == out) return HCK_OK;
    TRY(ensure_ct(ctx, out, a->size));
    const size_t ps = poly_stride(ctx);
    for (uint32_t p = 0; p < a->size; p++)
      TRY(launch_copy(ctx, out->data + p * ps, a->data + p * ps, (size_t)(a->level + 1) * ctx->n));
    out->size = a->size;
    out->level = a->level;
    out->scale = a->scale;
    return HCK_OK;
  }
  if (!gks) return set_error(HCK_EINVAL, "null Galois keys");
  return apply_galois_core(ctx, a, galois_of_step(ctx, step), gks, out);
}

int hck_rotate_noalloc(hck_context *ctx, const hck_ciphertext *a, int32_t step,
                       const hck_galois_keys *gks, hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, gks);
  OWNED(ctx, out);
  if (!a || !out) return set_error(HCK_EINVAL, "null argument");
  return rotate_noalloc(ctx, a, step, gks, out);
}

size_t hck_rotate_noalloc_scratch(const hck_context *ctx) {
  return ctx ? noalloc_scratch_needed(ctx) : noalloc_scratch_bytes();
}

int hck_apply_galois(hck_context *ctx, const hck_ciphertext *a, uint32_t element,
                     const hck_galois_keys *gks, hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, gks);
  OWNED(ctx, out);
  if (!a || !gks || !out) return set_error(HCK_EINVAL, "null argument");
  return apply_galois_core(ctx, a, element, gks, out);
}

int hck_keyswitch(hck_context *ctx, const hck_ciphertext *a, const hck_switch_key *swk,
                  hck_ciphertext *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, swk);
  OWNED(ctx, out);
  if (!a || !swk || !out) return set_error(HCK_EINVAL, "null argument");
  if (a->size == 0) return set_error(HCK_EINVAL, "empty ciphertext");
  const uint32_t level = a->level;
  const double scale = a->scale;
  TRY(ensure_ct(ctx, out, 2));
  const size_t ps = poly_stride(ctx);
  if (out == a) return set_error(HCK_EINVAL, "keyswitch output must not alias its input");
  TRY(keyswitch_core(ctx, a->data, 1, level, swk, out->data, out->data + ps, nullptr, nullptr));
  out->size = 2;
  out->level = level;
  out->scale = scale;
  return HCK_OK;
}

/* ---- linear transforms ------------------------------------------------------------ */

static int lt_finish_create(hck_context *ctx, const std::vector<std::vector<uint64_t>> &res,
                            const int32_t *offsets, uint32_t n_diag, uint32_t baby_step,
                            double pt_scale, uint32_t level, hck_linear_transform **out) {
  hck_linear_transform *lt = new hck_linear_transform();
  lt->ctx = ctx;
  lt->n1 = baby_step;
  lt->level = level;
  lt->scale = pt_scale;
  std::vector<int32_t> gs(n_diag), bs(n_diag);
  for (uint32_t d = 0; d < n_diag; d++) {
    gs[d] = (int32_t)std::floor((double)offsets[d] / (double)baby_step);
    bs[d] = offsets[d] - gs[d] * (int32_t)baby_step;
  }
  lt->giants = gs;
  lt->babies = bs;
  for (auto *v : {&lt->giants, &lt->babies}) {
    std::sort(v->begin(), v->end());
    v->erase(std::unique(v->begin(), v->end()), v->end());
  }
  const size_t per = (size_t)(level + 1) * ctx->n;
  const size_t cells = lt->giants.size() * lt->babies.size();
  int rc = dev_alloc(ctx, &lt->grid, cells * per);
  if (!rc) {
    lt->owned.push_back(lt->grid);
    const hipError_t e = hipMemsetAsync(lt->grid, 0, cells * per * sizeof(uint64_t), ctx->stream);
    if (e != hipSuccess) rc = check_hip(ctx, e, "hipMemsetAsync");
  }
  for (uint32_t d = 0; d < n_diag && !rc; d++) {
    const size_t gi = std::lower_bound(lt->giants.begin(), lt->giants.end(), gs[d]) -
                      lt->giants.begin();
    const size_t bi = std::lower_bound(lt->babies.begin(), lt->babies.end(), bs[d]) -
                      lt->babies.begin();
    uint64_t *p = lt->grid + (gi * lt->babies.size() + bi) * per;
    rc = import_rows(ctx, p, res[d].data(), 1, level + 1, level + 1);
    if (!rc) rc = mont_rows(ctx, p, poly_rows(1, level + 1, level + 1), true);
    lt->groups[gs[d]].push_back({bs[d], p});
  }
  if (rc) {
    hck_lt_destroy(lt);
    return rc;
  }
  track(ctx, lt, release_lt);
  *out = lt;
  return HCK_OK;
}

static int lt_check(hck_context *ctx, const int32_t *offsets, uint32_t n_diag, uint32_t baby_step,
                    uint32_t level) {
  if (!offsets || n_diag == 0) return set_error(HCK_EINVAL, "no diagonals");
  if (baby_step == 0) return set_error(HCK_EINVAL, "baby step must be positive");
  if (level >= ctx->L) return set_error(HCK_ELEVEL, "level beyond the chain");
  const int32_t slots = (int32_t)(ctx->n / 2);
  for (uint32_t d = 0; d < n_diag; d++) {
    if (offsets[d] <= -slots || offsets[d] >= slots)
      return set_error(HCK_EINVAL, "diagonal offset out of range");
    for (uint32_t e = 0; e < d; e++)
      if (offsets[e] == offsets[d]) return set_error(HCK_EINVAL, "duplicate diagonal offset");
  }
  return HCK_OK;
}

int hck_lt_create(hck_context *ctx, const double *diag_re, const double *diag_im,
                  const int32_t *offsets, uint32_t n_diag, uint32_t n_slots, uint32_t baby_step,
                  double pt_scale, uint32_t level, hck_linear_transform **out) {
  ENTER(ctx);
  if (!diag_re || !out) return set_error(HCK_EINVAL, "null argument");
  if (n_slots != ctx->n / 2) return set_error(HCK_EINVAL, "n_slots must be N/2");
  TRY(lt_check(ctx, offsets, n_diag, baby_step, level));
  if (pt_scale == 0.0) pt_scale = (double)ctx->mods[level];
  std::vector<std::vector<uint64_t>> res(n_diag);
  std::vector<double> re(n_slots), im(n_slots);
  for (uint32_t d = 0; d < n_diag; d++) {
    const int64_t k = offsets[d];
    const int64_t g = (int64_t)std::floor((double)k / (double)baby_step);
    const int64_t shift = g * (int64_t)baby_step;  // diagonal rotated right by g n1
    for (uint32_t j = 0; j < n_slots; j++) {
      const int64_t src = (((int64_t)j - shift) % n_slots + n_slots) % n_slots;
      re[j] = diag_re[(size_t)d * n_slots + src];
      im[j] = diag_im ? diag_im[(size_t)d * n_slots + src] : 0.0;
    }
    std::vector<int64_t> c;
    TRY(encode_coeffs(ctx->log_n, re.data(), im.data(), pt_scale, c));
    coeffs_to_residues(ctx, c, level, res[d]);
  }
  return lt_finish_create(ctx, res, offsets, n_diag, baby_step, pt_scale, level, out);
}

int hck_lt_create_from_residues(hck_context *ctx, const uint64_t *res, const int32_t *offsets,
                                uint32_t n_diag, uint32_t baby_step, double pt_scale,
                                uint32_t level, hck_linear_transform **out) {
  ENTER(ctx);
  if (!res || !out) return set_error(HCK_EINVAL, "null argument");
  TRY(lt_check(ctx, offsets, n_diag, baby_step, level));
  const size_t per = (size_t)(level + 1) * ctx->n;
  std::vector<std::vector<uint64_t>> rows(n_diag);
  for (uint32_t d = 0; d < n_diag; d++) rows[d].assign(res + d * per, res + (d + 1) * per);
  return lt_finish_create(ctx, rows, offsets, n_diag, baby_step, pt_scale, level, out);
}

int hck_lt_required_steps(const hck_linear_transform *lt, int32_t *steps, uint32_t cap,
                          uint32_t *n) {
  if (!lt || !n) return set_error(HCK_EINVAL, "null argument");
  std::vector<int32_t> s;
  for (auto &kv : lt->groups) {
    if (kv.first != 0) s.push_back(kv.first * (int32_t)lt->n1);
    for (auto &bp : kv.second)
      if (bp.first != 0) s.push_back(bp.first);
  }
  std::sort(s.begin(), s.end());
  s.erase(std::unique(s.begin(), s.end()), s.end());
  *n = (uint32_t)s.size();
  if (steps) {
    if (cap < s.size()) return set_error(HCK_EINVAL, "steps buffer too small");
    std::copy(s.begin(), s.end(), steps);
  }
  return HCK_OK;
}


int hck_measure_mulmod_rate(hck_context *ctx, double *tera_per_s) {
  ENTER(ctx);
  if (!tera_per_s) return set_error(HCK_EINVAL, "null argument");
  return measure_mulmod_rate(ctx, tera_per_s);
}

int hck_rotate_steps(hck_context *ctx, const hck_ciphertext *const *a, const int32_t *steps,
                     uint32_t n, const hck_galois_keys *gks, hck_ciphertext *const *out) {
  ENTER(ctx);
  OWNED(ctx, gks);
  if ((n && (!a || !out || !steps)) || !gks) return set_error(HCK_EINVAL, "null argument");
  std::vector<const hck_ciphertext *> src;
  std::vector<hck_ciphertext *> dst;
  std::vector<uint32_t> gal;
  for (uint32_t i = 0; i < n; i++) {
    if (!a[i] || !out[i]) return set_error(HCK_EINVAL, "null ciphertext");
    OWNED(ctx, a[i]);
    OWNED(ctx, out[i]);
    for (uint32_t k = 0; k < n; k++)
      if ((k < i && out[k] == out[i]) || (k != i && out[k] == a[i]))
        return set_error(HCK_EINVAL, "outputs must be distinct and alias only their own input");
  }
  for (uint32_t i = 0; i < n; i++) {
    if ((int64_t)steps[i] % (ctx->n / 2) == 0) {
      TRY(hck_rotate(ctx, a[i], steps[i], gks, out[i]));
      continue;
    }
    src.push_back(a[i]);
    dst.push_back(out[i]);
    gal.push_back(galois_of_step(ctx, steps[i]));
  }
  return apply_galois_multi(ctx, src.data(), gal.data(), (uint32_t)src.size(), gks, dst.data());
}

int hck_rotate_many(hck_context *ctx, const hck_ciphertext *const *a, uint32_t n, int32_t step,
                    const hck_galois_keys *gks, hck_ciphertext *const *out) {
  ENTER(ctx);
  OWNED(ctx, gks);
  if ((n && (!a || !out)) || !gks) return set_error(HCK_EINVAL, "null argument");
  for (uint32_t i = 0; i < n; i++) {
    if (!a[i] || !out[i]) return set_error(HCK_EINVAL, "null ciphertext");
    OWNED(ctx, a[i]);
    OWNED(ctx, out[i]);
  }
  if ((int64_t)step % (ctx->n / 2) == 0) {
    for (uint32_t i = 0; i < n; i++) TRY(hck_rotate(ctx, a[i], step, gks, out[i]));
    return HCK_OK;
  }
  return apply_galois_many(ctx, a, n, galois_of_step(ctx, step), gks, out);
}

int hck_rotate_hoisted(hck_context *ctx, const hck_ciphertext *a, const int32_t *steps,
                       uint32_t n, const hck_galois_keys *gks, hck_ciphertext *const *out) {
  ENTER(ctx);
  OWNED(ctx, a);
  OWNED(ctx, gks);
  if (!a || !gks || (n && (!steps || !out))) return set_error(HCK_EINVAL, "null argument");
  if (a->size != 2) return set_error(HCK_EINVAL, "rotation needs a 2-part ciphertext");
  std::vector<uint32_t> gal;
  std::vector<const hck_switch_key *> keys;
  std::vector<hck_ciphertext *> dst;
  const int64_t slots = ctx->n / 2;
  bool alias = false;
  for (uint32_t i = 0; i < n; i++) {
    if (!out[i]) return set_error(HCK_EINVAL, "null output");
    OWNED(ctx, out[i]);
    for (uint32_t k = 0; k < i; k++)
      if (out[k] == out[i]) return set_error(HCK_EINVAL, "outputs must be distinct");
    alias = alias || out[i] == a;
    if ((int64_t)steps[i] % slots == 0) continue;
    const uint32_t g = galois_of_step(ctx, steps[i]);
    auto it = gks->keys.find(g);
    if (it == gks->keys.end())
      return set_error(HCK_ENOKEY, "missing Galois key for step " + std::to_string(steps[i]));
    gal.push_back(g);
    keys.push_back(it->second);
    dst.push_back(out[i]);
  }
  TRY(ensure_workspace(ctx, ws_words_needed(ctx)));
  const uint32_t level = a->level;
  const double scale = a->scale;
  const size_t ps = poly_stride(ctx), words = (size_t)(level + 1) * ctx->n;
  const uint64_t *c0 = a->data, *c1 = a->data + ps;
  if (alias) {  // read the input from a copy so that its handle can be written
    uint64_t *copy = ws_rot(ctx);
    TRY(launch_copy(ctx, copy, a->data, words));
    TRY(launch_copy(ctx, copy + ps, a->data + ps, words));
    c0 = copy;
    c1 = copy + ps;
  }
  std::vector<uint64_t *> o0, o1;
  for (hck_ciphertext *y : dst) {
    TRY(ensure_ct(ctx, y, 2));
    o0.push_back(y->data);
    o1.push_back(y->data + ps);
  }
  TRY(keyswitch_hoisted(ctx, c0, c1, level, gal.data(), keys.data(), (uint32_t)gal.size(),
                        o0.data(), o1.data()));
  for (uint32_t i = 0; i < n; i++) {
    if ((int64_t)steps[i] % slots == 0 && out[i] != a) {
      TRY(ensure_ct(ctx, out[i], 2));
      TRY(launch_copy(ctx, out[i]->data, c0, words));
      TRY(launch_copy(ctx, out[i]->data + ps, c1, words));
    }
    out[i]->size = 2;
    out[i]->level = level;
    out[i]->scale = scale;
  }
  return HCK_OK;
}

// Baby-step/giant-step evaluation of sums of transforms:
//   out[o] = sum over terms t with term_out[t] = o of sign_t lt_t(in[term_in[t]]).
// Baby rotations Rot(in, b) are computed once per (input, b) and key-switched
// in batches over the inputs; for every giant index g the inner sums of all
// outputs are formed first (Rot(A) + Rot(B) = Rot(A + B)) and then rotated
// by g n1 together, one key stream per batch.
int hck_lt_eval(hck_context *ctx, const hck_ciphertext *const *in, uint32_t n_in,
                const hck_linear_transform *const *lts, const uint32_t *term_in,
                const uint32_t *term_out, const int32_t *term_sign, uint32_t n_terms,
                const hck_galois_keys *gks, hck_ciphertext *const *out, uint32_t n_out,
                uint32_t flags) {
  ENTER(ctx);
  OWNED(ctx, gks);
  if (!in || !lts || !term_in || !term_out || !out || !gks || n_in == 0 || n_terms == 0 ||
      n_out == 0)
    return set_error(HCK_EINVAL, "null or empty argument");
  for (uint32_t i = 0; i < n_in; i++) OWNED(ctx, in[i]);
  for (uint32_t i = 0; i < n_out; i++) OWNED(ctx, out[i]);
  for (uint32_t t = 0; t < n_terms; t++) OWNED(ctx, lts[t]);
  const uint32_t level = in[0]->level;
  uint32_t n1 = 0;
  for (uint32_t i = 0; i < n_in; i++) {
    if (!in[i] || in[i]->size != 2) return set_error(HCK_EINVAL, "inputs must be 2-part ciphertexts");
    if (in[i]->level != level) return set_error(HCK_ELEVEL, "inputs at different levels");
  }
  for (uint32_t o = 0; o < n_out; o++)
    if (!out[o]) return set_error(HCK_EINVAL, "null output");
  std::vector<double> out_scale(n_out, 0.0);
  for (uint32_t t = 0; t < n_terms; t++) {
    const hck_linear_transform *lt = lts[t];
    if (!lt || term_in[t] >= n_in || term_out[t] >= n_out)
      return set_error(HCK_EINVAL, "bad term");
    if (term_sign && term_sign[t] != 1 && term_sign[t] != -1)
      return set_error(HCK_EINVAL, "term signs must be +1 or -1");
    if (lt->level != level) return set_error(HCK_ELEVEL, "transform level differs from input level");
    if (n1 == 0) n1 = lt->n1;
    if (lt->n1 != n1) return set_error(HCK_EINVAL, "transforms must share the baby step");
    const double sc = in[term_in[t]]->scale * lt->scale;
    double &os = out_scale[term_out[t]];
    if (os == 0.0) os = sc;
    else if (!scales_match(os, sc)) return set_error(HCK_ESCALE, "terms of one output differ in scale");
  }
  for (uint32_t o = 0; o < n_out; o++)
    if (out_scale[o] == 0.0) return set_error(HCK_EINVAL, "an output has no term");
  // keys needed, checked before any work
  std::map<int32_t, std::vector<uint32_t>> baby_inputs;  // b -> inputs
  std::map<int32_t, std::vector<uint32_t>> giant_outputs; // g -> outputs
  for (uint32_t t = 0; t < n_terms; t++)
    for (auto &kv : lts[t]->groups) {
      auto &go = giant_outputs[kv.first];
      if (std::find(go.begin(), go.end(), term_out[t]) == go.end()) go.push_back(term_out[t]);
      for (auto &bp : kv.second) {
        auto &bi = baby_inputs[bp.first];
        if (std::find(bi.begin(), bi.end(), term_in[t]) == bi.end()) bi.push_back(term_in[t]);
      }
    }
  const int64_t slots = ctx->n / 2;
  auto need = [&](int64_t step) -> int {
    if (step % slots == 0) return HCK_OK;
    if (!gks->keys.count(galois_of_step(ctx, (int32_t)step)))
      return set_error(HCK_ENOKEY, "missing Galois key for step " + std::to_string(step));
    return HCK_OK;
  };
  for (auto &kv : baby_inputs) TRY(need(kv.first));
  for (auto &kv : giant_outputs) TRY(need((int64_t)kv.first * n1));

  const size_t n = ctx->n, ps = poly_stride(ctx);
  const LimbMap qm = qmap(ctx, level);
  std::vector<hck_ciphertext *> scratch;
  auto get = [&]() {
    hck_ciphertext *c = pool_get(ctx);
    scratch.push_back(c);
    return c;
  };
  int rc = HCK_OK;
  // baby steps: baby[(input, b)]; b = 0 is the input itself
  std::map<std::pair<uint32_t, int32_t>, const hck_ciphertext *> baby;
  if (flags & HCK_LT_HOIST_BABY) {
    std::map<uint32_t, std::vector<int32_t>> per_input;
    for (auto &kv : baby_inputs)
      for (uint32_t i : kv.second) {
        if (kv.first == 0) baby[{i, 0}] = in[i];
        else per_input[i].push_back(kv.first);
      }
    for (auto &kv : per_input) {
      std::vector<hck_ciphertext *> dst;
      for (int32_t b : kv.second) {
        hck_ciphertext *c = get();
        dst.push_back(c);
        baby[{kv.first, b}] = c;
      }
      if (rc == HCK_OK)
        rc = hck_rotate_hoisted(ctx, in[kv.first], kv.second.data(), (uint32_t)kv.second.size(),
                                gks, dst.data());
    }
  } else {
    for (auto &kv : baby_inputs) {
      const int32_t b = kv.first;
      if (b == 0) {
        for (uint32_t i : kv.second) baby[{i, 0}] = in[i];
        continue;
      }
      std::vector<const hck_ciphertext *> src;
      std::vector<hck_ciphertext *> dst;
      for (uint32_t i : kv.second) {
        hck_ciphertext *c = get();
        src.push_back(in[i]);
        dst.push_back(c);
        baby[{i, b}] = c;
      }
      if (rc == HCK_OK)
        rc = hck_rotate_many(ctx, src.data(), (uint32_t)src.size(), b, gks, dst.data());
    }
  }
  if (n_in > (uint32_t)kLtIn || n_out > (uint32_t)kLtOut)
    rc = rc ? rc : set_error(HCK_EINVAL, "at most 4 inputs and 4 outputs per evaluation");
  // distinct transforms, in order of first use, processed two per launch
  std::vector<const hck_linear_transform *> uniq;
  std::vector<uint32_t> term_lt(n_terms);
  for (uint32_t t = 0; t < n_terms; t++) {
    auto it = std::find(uniq.begin(), uniq.end(), lts[t]);
    term_lt[t] = (uint32_t)(it - uniq.begin());
    if (it == uniq.end()) uniq.push_back(lts[t]);
  }
  std::vector<int32_t> giants, babies;
  for (auto &kv : giant_outputs) giants.push_back(kv.first);
  for (auto &kv : baby_inputs) babies.push_back(kv.first);
  if (giants.size() > (size_t)kLtMaxG)
    rc = rc ? rc : set_error(HCK_EINVAL, "more than 64 giant groups in one evaluation");
  const uint32_t ng = (uint32_t)giants.size();
  if (!rc) rc = ensure_lt_scratch(ctx, (size_t)ng * n_out * 2 * ps);
  if (!rc) rc = ensure_zero_rows(ctx);
  uint64_t *sums = ctx->lt_scratch;
  // inner sums of every (giant group, output), babies in chunks that fit LDS
  const uint32_t bchunk = std::min<uint32_t>((uint32_t)kLtB, 64 / n_in);
  bool first = true;
  for (size_t l0 = 0; l0 < uniq.size() && !rc; l0 += kLtLts)
    for (size_t b0 = 0; b0 < babies.size() && !rc; b0 += bchunk) {
      LtSumArgs la;
      std::memset(&la, 0, sizeof(la));
      la.nb = (uint32_t)std::min<size_t>(bchunk, babies.size() - b0);
      la.ng = ng;
      la.n_in = n_in;
      la.n_out = n_out;
      la.ps = ps;
      la.accumulate = first ? 0 : 1;
      la.sums = sums;
      la.zero = ctx->zero_rows;
      for (uint32_t l = 0; l < (uint32_t)kLtLts && l0 + l < uniq.size(); l++) {
        const hck_linear_transform *lt = uniq[l0 + l];
        la.grid[l] = lt->grid;
        la.grid_nb[l] = (uint32_t)lt->babies.size();
        la.grid_rows[l] = lt->level + 1;
        for (uint32_t g = 0; g < ng; g++) {
          auto git = std::lower_bound(lt->giants.begin(), lt->giants.end(), giants[g]);
          const bool has_g = git != lt->giants.end() && *git == giants[g];
          la.gmap[l][g] = has_g ? (int32_t)(git - lt->giants.begin()) : -1;
          auto grp = lt->groups.find(giants[g]);
          for (uint32_t b = 0; b < la.nb && has_g && grp != lt->groups.end(); b++)
            for (auto &bp : grp->second)
              if (bp.first == babies[b0 + b]) la.present[l][g] |= 1u << b;
        }
        for (uint32_t b = 0; b < la.nb; b++) {
          auto bit = std::lower_bound(lt->babies.begin(), lt->babies.end(), babies[b0 + b]);
          la.bmap[l][b] = (bit != lt->babies.end() && *bit == babies[b0 + b])
                              ? (int32_t)(bit - lt->babies.begin())
                              : -1;
        }
      }
      for (uint32_t i = 0; i < n_in; i++)
        for (uint32_t b = 0; b < la.nb; b++) {
          auto it = baby.find({i, babies[b0 + b]});
          if (it != baby.end()) la.baby[i][b] = it->second->data;
        }
      std::vector<uint32_t> per_out(n_out, 0);
      for (uint32_t t = 0; t < n_terms; t++) {
        if (term_lt[t] < l0 || term_lt[t] >= l0 + kLtLts) continue;
        int8_t &c = la.coef[term_lt[t] - l0][term_in[t]][term_out[t]];
        if (c != 0) {
          rc = set_error(HCK_EINVAL, "repeated (transform, input, output) term");
          break;
        }
        c = (term_sign && term_sign[t] < 0) ? -1 : 1;
        per_out[term_out[t]]++;
      }
      la.max_terms = std::max<uint32_t>(1, *std::max_element(per_out.begin(), per_out.end()));
      if (!rc) rc = launch_lt_sums(ctx, la, level);
      first = false;
    }
  // the (group, output) sums that have terms, as ciphertexts over the scratch
  std::deque<hck_ciphertext> views;
  std::vector<std::vector<hck_ciphertext *>> inner(ng, std::vector<hck_ciphertext *>(n_out, nullptr));
  for (uint32_t gi = 0; gi < ng; gi++)
    for (uint32_t o : giant_outputs[giants[gi]]) {
      views.emplace_back();
      hck_ciphertext &v = views.back();
      v.ctx = ctx;
      v.data = sums + ((size_t)gi * n_out + o) * 2 * ps;
      v.cap_polys = 2;
      inner[gi][o] = &v;
    }
  // every output is the sum over its groups g of Rot(inner_g, g n1); the
  // inputs are no longer read, so outputs may alias them
  struct Part {
    uint32_t o;
    uint32_t galois;  // 1: unrotated group
    hck_ciphertext *u;
  };
  std::vector<Part> parts;
  for (size_t gi = 0; gi < giants.size() && !rc; gi++)
    for (uint32_t o = 0; o < n_out; o++) {
      hck_ciphertext *u = inner[gi][o];
      if (!u) continue;
      u->size = 2;
      u->level = level;
      u->scale = out_scale[o];
      parts.push_back({o, giants[gi] == 0 ? 1u : galois_of_step(ctx, giants[gi] * (int32_t)n1), u});
    }
  const size_t words = (size_t)(level + 1) * n;
  if (!rc && (flags & HCK_LT_HOIST_GIANT)) {
    // shared ModDown: the rotated groups' key products are summed in Q u P
    // per output (ws_pq), the phi_g(c0) and the unrotated group in Q
    const uint32_t limit = ks_batch_limit(ctx, level);
    std::vector<bool> written(n_out, false);
    std::vector<Part> rot;
    for (const Part &pt : parts)
      if (pt.galois != 1) rot.push_back(pt);
    if (!rc) rc = ensure_workspace(ctx, ws_words_needed(ctx));
    const size_t pq_stride = (size_t)2 * (ctx->L + ctx->K) * n;
    for (size_t s0 = 0; s0 < rot.size() && !rc; s0 += even_batch(rot.size() - s0, limit)) {
      KsBatch kb;
      kb.n = even_batch(rot.size() - s0, limit);
      std::vector<uint64_t *> pq(kb.n);
      bool first[kMaxBatch];
      for (uint32_t b = 0; b < kb.n; b++) {
        const Part &pt = rot[s0 + b];
        auto it = gks->keys.find(pt.galois);
        kb.key[b] = it->second->data;
        kb.galois[b] = pt.galois;
        kb.d[b] = pt.u->data + ps;
        kb.out0[b] = kb.out1[b] = nullptr;
        kb.add0[b] = kb.add1[b] = nullptr;
        pq[b] = ws_pq(ctx) + pt.o * pq_stride;
        first[b] = !written[pt.o];
      }
      rc = keyswitch_pq(ctx, kb, level, pq.data(), first);
      for (uint32_t b = 0; b < kb.n; b++) written[rot[s0 + b].o] = true;
    }
    std::vector<hck_ciphertext *> c0sum(n_out, nullptr);
    KsBatch md;
    md.n = 0;
    std::vector<const uint64_t *> md_pq;
    for (uint32_t o = 0; o < n_out && !rc; o++) {
      rc = ensure_ct(ctx, out[o], 2);
      std::vector<const uint64_t *> c0s;
      std::vector<uint32_t> gs;
      const hck_ciphertext *plain = nullptr;
      for (const Part &pt : parts) {
        if (pt.o != o) continue;
        c0s.push_back(pt.u->data);
        gs.push_back(pt.galois);
        if (pt.galois == 1) plain = pt.u;
      }
      if (!written[o]) {  // no rotated group: the unrotated one is the output
        for (uint32_t p = 0; p < 2 && !rc && plain; p++)
          rc = launch_copy(ctx, out[o]->data + p * ps, plain->data + p * ps, words);
        continue;
      }
      c0sum[o] = get();
      if (!rc) rc = ensure_ct(ctx, c0sum[o], 2);
      if (!rc) rc = launch_gather_sum(ctx, c0sum[o]->data, c0s.data(), gs.data(),
                                      (uint32_t)c0s.size(), qm);
      const uint32_t b = md.n++;
      md.key[b] = nullptr;
      md.galois[b] = 1;
      md.d[b] = nullptr;
      md.out0[b] = out[o]->data;
      md.out1[b] = out[o]->data + ps;
      md.add0[b] = c0sum[o]->data;
      md.add1[b] = plain ? plain->data + ps : nullptr;
      md_pq.push_back(ws_pq(ctx) + o * pq_stride);
      if (md.n == limit && !rc) {
        rc = moddown_pq(ctx, md, level, md_pq.data());
        md.n = 0;
        md_pq.clear();
      }
    }
    if (!rc && md.n) rc = moddown_pq(ctx, md, level, md_pq.data());
  } else if (!rc) {
    // separate rotations, key-switched together in batches, then one sum per
    // output
    std::vector<const hck_ciphertext *> src;
    std::vector<hck_ciphertext *> dst;
    std::vector<uint32_t> gal;
    std::vector<std::vector<const hck_ciphertext *>> terms_of(n_out);
    for (const Part &pt : parts) {
      if (pt.galois == 1) {
        terms_of[pt.o].push_back(pt.u);
        continue;
      }
      hck_ciphertext *r = get();
      src.push_back(pt.u);
      dst.push_back(r);
      gal.push_back(pt.galois);
      terms_of[pt.o].push_back(r);
    }
    rc = apply_galois_multi(ctx, src.data(), gal.data(), (uint32_t)src.size(), gks, dst.data());
    for (uint32_t o = 0; o < n_out && !rc; o++) {
      rc = ensure_ct(ctx, out[o], 2);
      std::vector<const uint64_t *> polys;
      for (uint32_t p = 0; p < 2 && !rc; p++) {
        polys.clear();
        for (const hck_ciphertext *c : terms_of[o]) polys.push_back(c->data + p * ps);
        rc = launch_sum_many(ctx, out[o]->data + p * ps, polys.data(), (uint32_t)polys.size(),
                             qm);
      }
    }
  }
  for (uint32_t o = 0; o < n_out && !rc; o++) {
    out[o]->size = 2;
    out[o]->level = level;
    out[o]->scale = out_scale[o];
  }
  for (hck_ciphertext *s : scratch) pool_put(ctx, s);
  return rc;
}

int hck_lt_apply(hck_context *ctx, const hck_linear_transform *lt, const hck_ciphertext *a,
                 const hck_galois_keys *gks, hck_ciphertext *out) {
  const uint32_t zero = 0;
  const int32_t one = 1;
  return hck_lt_eval(ctx, &a, 1, &lt, &zero, &zero, &one, 1, gks, &out, 1, 0);
}

int hck_lt_destroy(hck_linear_transform *lt) {
  if (lt) {
    if (lt->ctx) untrack(lt->ctx, lt);
    release_lt(lt);
    delete lt;
  }
  return HCK_OK;
}

}  // extern "C"
