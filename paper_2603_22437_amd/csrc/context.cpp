// Context: parameter validation, device tables, memory, errors, timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "internal.h"

namespace hck {

namespace {
thread_local std::string g_last_error;

uint32_t bit_reverse(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

bool is_prime_u64(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int r = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    r++;
  }
  for (uint64_t a : small) {
    uint64_t x = h_powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r; i++) {
      x = h_mulmod(x, x, n);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

// A primitive 2N-th root of unity: psi = x^((q-1)/2N) for the first x >= 3
// with psi^N = -1 (q prime, q = 1 mod 2N).
// contiguous-pass twists (ntt_core.h) of one limb for the split 2^log_a x
// 2^(log_n - log_a): word g R2 + i gets beta_g^i (and beta_g^-i), beta_g =
// psi^(2 brv_a(g)); pw, ipw hold psi^k, psi^-k for k < N
void twist_rows(const std::vector<uint64_t> &pw, const std::vector<uint64_t> &ipw, uint64_t q,
                uint32_t log_n, int log_a, size_t base, std::vector<uint64_t> &ttw,
                std::vector<uint64_t> &ttws, std::vector<uint64_t> &ittw,
                std::vector<uint64_t> &ittws) {
  const uint64_t n = 1ull << log_n;
  const int log_b = (int)log_n - log_a;
  for (uint32_t g = 0; g < (1u << log_a); g++) {
    const uint64_t bg = 2ull * bit_reverse(g, log_a);
    for (uint32_t i = 0; i < (1u << log_b); i++) {
      const uint64_t e = bg * i % (2ull * n);   // psi^N = -1
      const uint64_t f = e < n ? pw[e] : (q - pw[e - n]) % q;
      const uint64_t fi = e < n ? ipw[e] : (q - ipw[e - n]) % q;
      const size_t w = base + ((size_t)g << log_b) + i;
      ttw[w] = f;
      ttws[w] = h_shoup(f, q);
      ittw[w] = fi;
      ittws[w] = h_shoup(fi, q);
    }
  }
}

uint64_t primitive_2n_root(uint64_t q, uint64_t n) {
  for (uint64_t x = 3;; x++) {
    uint64_t psi = h_powmod(x, (q - 1) / (2 * n), q);
    if (h_powmod(psi, n, q) == q - 1) return psi;
  }
}

}  // namespace

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int check_hip(hck_context *ctx, hipError_t e, const char *what) {
  if (ctx) ctx->broken = true;
  return set_error(HCK_EDEVICE, std::string("HIP error in ") + what + ": " + hipGetErrorString(e));
}

// one record of the launch trace (hck_trace_enable)
static void trace_note(hck_context *ctx, const char *name, dim3 grid, double bytes,
                       double mulmods) {
  hck_trace_record r{};
  std::strncpy(r.name, name, sizeof(r.name) - 1);
  r.grid[0] = grid.x;
  r.grid[1] = grid.y;
  r.grid[2] = grid.z;
  r.bytes = bytes;
  r.mulmods = mulmods;
  ctx->trace_log.push_back(r);
}

int dev_alloc(hck_context *ctx, uint64_t **p, size_t words) {
  *p = nullptr;
  if (words == 0) return HCK_OK;
  const size_t bytes = words * sizeof(uint64_t);
  if (ctx->capturing)
    return set_error(HCK_EINVAL, "device allocation of " + std::to_string(bytes) +
                                     " bytes during graph capture (run the calls once "
                                     "before capturing them)");
  if (ctx->alloc_fn) {
    *p = (uint64_t *)ctx->alloc_fn(bytes, (void *)ctx->stream, ctx->alloc_user);
    if (!*p)
      return set_error(HCK_ENOMEM, "the allocator hook returned no memory for " +
                                       std::to_string(bytes) + " bytes");
  } else {
    hipError_t e = hipMallocAsync((void **)p, bytes, ctx->stream);
    if (e != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
      return set_error(HCK_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
  }
  ctx->live_allocs++;
  ctx->alloc_seq[*p] = ++ctx->alloc_counter;
  if (ctx->trace) trace_note(ctx, "alloc", dim3(0, 0, 0), (double)bytes, 0);
  return HCK_OK;
}

void dev_free(hck_context *ctx, void *p) {
  if (!p) return;
  if (ctx->trace) trace_note(ctx, "free", dim3(0, 0, 0), 0, 0);
  if (ctx->free_fn) ctx->free_fn(p, (void *)ctx->stream, ctx->alloc_user);
  else (void)hipFreeAsync(p, ctx->stream);
  ctx->live_allocs--;
  auto it = ctx->alloc_seq.find(p);
  if (it != ctx->alloc_seq.end()) {
    if (it->second < ctx->graph_mark) ctx->freed_old.push_back(it->second);
    ctx->alloc_seq.erase(it);
  }
}

int ensure_ct(hck_context *ctx, hck_ciphertext *ct, uint32_t polys) {
  if (ct->cap_polys >= polys && ct->data) return HCK_OK;
  if (ct->pooled) polys = std::max(polys, 3u);
  uint64_t *p = nullptr;
  int rc = dev_alloc(ctx, &p, (size_t)polys * ctx->L * ctx->n);
  if (rc) return rc;
  if (ct->data && ct->size) {
    HCK_HIP(ctx, hipMemcpyAsync(p, ct->data, (size_t)ct->size * ctx->L * ctx->n * 8,
                                hipMemcpyDeviceToDevice, ctx->stream));
  }
  dev_free(ctx, ct->data);
  ct->data = p;
  ct->cap_polys = polys;
  return HCK_OK;
}

int ensure_workspace(hck_context *ctx, size_t words) {
  if (ctx->ws_words >= words) return HCK_OK;
  dev_free(ctx, ctx->ws);
  ctx->ws = nullptr;
  ctx->ws_words = 0;
  int rc = dev_alloc(ctx, &ctx->ws, words);
  if (rc) return rc;
  ctx->ws_words = words;
  return HCK_OK;
}

int ensure_lt_scratch(hck_context *ctx, size_t words) {
  if (ctx->lt_scratch_words >= words) return HCK_OK;
  dev_free(ctx, ctx->lt_scratch);
  ctx->lt_scratch = nullptr;
  ctx->lt_scratch_words = 0;
  int rc = dev_alloc(ctx, &ctx->lt_scratch, words);
  if (rc) return rc;
  ctx->lt_scratch_words = words;
  return HCK_OK;
}

int ensure_zero_rows(hck_context *ctx) {
  if (ctx->zero_rows) return HCK_OK;
  const size_t words = (size_t)ctx->L * ctx->n;
  int rc = dev_alloc(ctx, &ctx->zero_rows, words);
  if (rc) return rc;
  HCK_HIP(ctx, hipMemsetAsync(ctx->zero_rows, 0, words * sizeof(uint64_t), ctx->stream));
  return HCK_OK;
}

LimbMap qmap(const hck_context *ctx, uint32_t level) {
  LimbMap m;
  m.n = level + 1;
  for (uint32_t i = 0; i <= level; i++) {
    m.row[i] = (uint16_t)i;
    m.mod[i] = (uint8_t)i;
  }
  return m;
}

LimbMap fullmap(const hck_context *ctx) {
  LimbMap m;
  m.n = ctx->L + ctx->K;
  for (uint32_t i = 0; i < m.n; i++) {
    m.row[i] = (uint16_t)i;
    m.mod[i] = (uint8_t)i;
  }
  return m;
}

uint32_t galois_of_step(const hck_context *ctx, int32_t step) {
  const int64_t slots = ctx->n / 2;
  int64_t k = ((int64_t)step % slots + slots) % slots;
  return (uint32_t)h_powmod(5, (uint64_t)k, 2ull * ctx->n);
}

// ---- timing ----------------------------------------------------------------

void timing_begin(hck_context *ctx, const char *name, dim3 grid, double bytes, double mulmods) {
  if (ctx->trace) trace_note(ctx, name, grid, bytes, mulmods);
  if (!ctx->timing) return;
  hck_context::Timed t;
  t.name = name;
  t.bytes = bytes;
  t.mulmods = mulmods;
  for (hipEvent_t *ev : {&t.start, &t.stop}) {
    if (!ctx->event_pool.empty()) {
      *ev = ctx->event_pool.back();
      ctx->event_pool.pop_back();
    } else if (hipEventCreate(ev) != hipSuccess) {
      return;
    }
  }
  (void)hipEventRecord(t.start, ctx->stream);
  ctx->pending.push_back(t);
}

void timing_end(hck_context *ctx) {
  if (!ctx->timing || ctx->pending.empty()) return;
  (void)hipEventRecord(ctx->pending.back().stop, ctx->stream);
}

int timing_collect(hck_context *ctx) {
  if (ctx->pending.empty()) return HCK_OK;
  HCK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (auto &t : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
      auto &slot = ctx->timing_total[t.name];
      slot.ms += ms;
      slot.launches += 1;
      slot.bytes += t.bytes;
      slot.mulmods += t.mulmods;
    }
    ctx->event_pool.push_back(t.start);
    ctx->event_pool.push_back(t.stop);
  }
  ctx->pending.clear();
  return HCK_OK;
}

// ---- context construction ------------------------------------------------------

static int validate(const hck_params *p) {
  if (!p || !p->q || (p->num_p && !p->p)) return set_error(HCK_EINVAL, "null parameters");
  if (p->log_n < 11 || p->log_n > 17) return set_error(HCK_EPARAMS, "log_n must be in [11, 17]");
  if (p->num_q < 1 || p->num_p < 1) return set_error(HCK_EPARAMS, "need at least one q and one p");
  if (p->num_q + p->num_p > (uint32_t)kMaxLimbs)
    return set_error(HCK_EPARAMS, "L + K exceeds HCK_MAX_LIMBS");
  if (p->dnum < 1 || p->dnum > p->num_q) return set_error(HCK_EPARAMS, "dnum must be in [1, L]");
  const uint64_t two_n = 2ull << p->log_n;
  std::vector<uint64_t> all(p->q, p->q + p->num_q);
  all.insert(all.end(), p->p, p->p + p->num_p);
  uint64_t maxm = 0;
  for (size_t i = 0; i < all.size(); i++) {
    uint64_t m = all[i];
    if (m >= (1ull << 61)) return set_error(HCK_EPARAMS, "modulus not below 2^61");
    if (m % two_n != 1) return set_error(HCK_EPARAMS, "modulus is not 1 mod 2N");
    if (!is_prime_u64(m)) return set_error(HCK_EPARAMS, "modulus is not prime");
    for (size_t j = 0; j < i; j++)
      if (all[j] == m) return set_error(HCK_EPARAMS, "moduli must be distinct");
    maxm = std::max(maxm, m);
  }
  const uint32_t alpha = (p->num_q + p->dnum - 1) / p->dnum;
  if (alpha > 16 || p->num_p > 16)
    return set_error(HCK_EPARAMS, "a digit or the special basis has more than 16 primes");
  for (uint32_t j = 0; j * alpha < p->num_q; j++) {
    unsigned __int128 s = 0;
    for (uint32_t i = j * alpha; i < std::min(p->num_q, (j + 1) * alpha); i++) s += p->q[i];
    if (s >> 64) return set_error(HCK_EPARAMS, "a digit's primes sum to 2^64 or more");
  }
  unsigned __int128 sp = 0;
  for (uint32_t k = 0; k < p->num_p; k++) sp += p->p[k];
  if (sp >> 64) return set_error(HCK_EPARAMS, "the special primes sum to 2^64 or more");
  if ((unsigned __int128)p->dnum * maxm >> 64)
    return set_error(HCK_EPARAMS, "dnum times the largest modulus reaches 2^64");
  return HCK_OK;
}

int build_context(const hck_params *prm, int device, void *stream, hck_context **out) {
  int rc = validate(prm);
  if (rc) return rc;
  HCK_HIP(nullptr, hipSetDevice(device));
  hck_context *ctx = new hck_context();
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  ctx->log_n = prm->log_n;
  ctx->n = 1u << prm->log_n;
  ctx->L = prm->num_q;
  ctx->K = prm->num_p;
  ctx->dnum = prm->dnum;
  ctx->alpha = (ctx->L + ctx->dnum - 1) / ctx->dnum;
  ctx->mods.assign(prm->q, prm->q + prm->num_q);
  ctx->mods.insert(ctx->mods.end(), prm->p, prm->p + prm->num_p);
  ctx->bconv30 = std::all_of(ctx->mods.begin(), ctx->mods.end(),
                             [](uint64_t m) { return m < (1ull << 60); });
  const uint32_t nm = ctx->L + ctx->K, n = ctx->n, L = ctx->L, K = ctx->K;

  // per-modulus constants and twiddles
  std::vector<ModConst> mc(nm);
  std::vector<uint64_t> tw((size_t)nm * n), tws((size_t)nm * n), itw((size_t)nm * n),
      itws((size_t)nm * n);
  std::vector<uint64_t> ttw((size_t)nm * n), ttws((size_t)nm * n), ittw((size_t)nm * n),
      ittws((size_t)nm * n);
  std::vector<uint64_t> pw(n), ipw(n);
  // contiguous-pass twists (ntt_core.h): word w = g R2 + i of a limb gets
  // beta_g^i with beta_g = psi^(2 brv_a(g)), a = log2 of the strided radix
  const int log_a = (ctx->log_n + 1) / 2;
  for (uint32_t m = 0; m < nm; m++) {
    const uint64_t q = ctx->mods[m];
    ModConst &c = mc[m];
    c.q = q;
    c.qinv = h_inv64(q);
    c.r64 = h_r64(q);
    c.r64_shoup = h_shoup(c.r64, q);
    c.ninv = h_invmod(n % q, q);
    c.ninv_shoup = h_shoup(c.ninv, q);
    c.r2 = h_mulmod(c.r64, c.r64, q);
    c.one_shoup = h_shoup(1, q);
    c.nq = 0 - q;
    const uint64_t psi = primitive_2n_root(q, n), ipsi = h_invmod(psi, q);
    pw[0] = ipw[0] = 1;
    for (uint32_t i = 1; i < n; i++) {
      pw[i] = h_mulmod(pw[i - 1], psi, q);
      ipw[i] = h_mulmod(ipw[i - 1], ipsi, q);
    }
    for (uint32_t k = 0; k < n; k++) {
      const uint32_t b = bit_reverse(k, ctx->log_n);
      tw[(size_t)m * n + k] = pw[b];
      tws[(size_t)m * n + k] = h_shoup(pw[b], q);
      itw[(size_t)m * n + k] = ipw[b];
      itws[(size_t)m * n + k] = h_shoup(ipw[b], q);
    }
    twist_rows(pw, ipw, q, ctx->log_n, log_a, (size_t)m * n, ttw, ttws, ittw, ittws);
  }

  // ModUp tables: for each level l and digit j with limbs D = [lo, hi),
  // scale_i = N^-1 (Q_D / q_i)^-1 mod q_i and conv[a][m] = (Q_D / q_(lo+a)) 2^64 mod m.
  const uint32_t A = ctx->alpha;
  std::vector<uint64_t> up_conv((size_t)L * ctx->dnum * A * nm, 0);
  ctx->up_scale.assign(L, std::vector<uint64_t>(L, 0));
  for (uint32_t l = 0; l < L; l++) {
    for (uint32_t j = 0; j < ctx->dnum; j++) {
      const uint32_t lo = j * A;
      if (lo > l) break;
      const uint32_t hi = std::min(lo + A, l + 1);
      for (uint32_t a = 0; a < hi - lo; a++) {
        const uint32_t i = lo + a;
        uint64_t hat_i = 1;
        for (uint32_t k = lo; k < hi; k++)
          if (k != i) hat_i = h_mulmod(hat_i, ctx->mods[k] % ctx->mods[i], ctx->mods[i]);
        ctx->up_scale[l][i] =
            h_mulmod(h_invmod(hat_i, ctx->mods[i]), mc[i].ninv, ctx->mods[i]);
        for (uint32_t m = 0; m < nm; m++) {
          const uint64_t t = ctx->mods[m];
          uint64_t hat_t = 1;
          for (uint32_t k = lo; k < hi; k++)
            if (k != i) hat_t = h_mulmod(hat_t, ctx->mods[k] % t, t);
          up_conv[(((size_t)l * ctx->dnum + j) * A + a) * nm + m] = h_mulmod(hat_t, mc[m].r64, t);
        }
      }
    }
  }

  // ModDown tables over P = prod p_k, with the rounding addend h = (P-1)/2.
  std::vector<uint64_t> down_conv((size_t)K * nm, 0);
  ctx->down_scale.assign(K, 0);
  ctx->down_add.assign(K, 0);
  for (uint32_t k = 0; k < K; k++) {
    const uint32_t mk = L + k;
    const uint64_t pk = ctx->mods[mk];
    uint64_t hat = 1;
    for (uint32_t r = 0; r < K; r++)
      if (r != k) hat = h_mulmod(hat, ctx->mods[L + r] % pk, pk);
    const uint64_t hat_inv = h_invmod(hat, pk);
    ctx->down_scale[k] = h_mulmod(hat_inv, mc[mk].ninv, pk);
    // (P-1)/2 mod p_k = -2^-1 mod p_k
    const uint64_t h = pk - h_invmod(2, pk);
    ctx->down_add[k] = h_mulmod(h, hat_inv, pk);
    for (uint32_t m = 0; m < L; m++) {
      const uint64_t t = ctx->mods[m];
      uint64_t hat_t = 1;
      for (uint32_t r = 0; r < K; r++)
        if (r != k) hat_t = h_mulmod(hat_t, ctx->mods[L + r] % t, t);
      down_conv[(size_t)k * nm + m] = h_mulmod(hat_t, mc[m].r64, t);
    }
  }
  ctx->down_hneg.assign(L, 0);
  ctx->pinv.assign(L, 0);
  for (uint32_t i = 0; i < L; i++) {
    const uint64_t q = ctx->mods[i];
    uint64_t pm = 1;
    for (uint32_t k = 0; k < K; k++) pm = h_mulmod(pm, ctx->mods[L + k] % q, q);
    ctx->pinv[i] = h_invmod(pm, q);
    // (P-1)/2 mod q = (P mod q - 1) 2^-1 mod q; stored negated
    const uint64_t h = h_mulmod((pm + q - 1) % q, h_invmod(2, q), q);
    ctx->down_hneg[i] = h == 0 ? 0 : q - h;
  }
  ctx->rescale_inv.assign(L, std::vector<uint64_t>(L, 0));
  for (uint32_t l = 1; l < L; l++)
    for (uint32_t i = 0; i < l; i++)
      ctx->rescale_inv[l][i] = h_invmod(ctx->mods[l] % ctx->mods[i], ctx->mods[i]);

  // upload
  auto up = [&](uint64_t **dst, const void *src, size_t bytes) -> int {
    if (hipMalloc((void **)dst, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(HCK_ENOMEM, "table allocation failed");
    }
    if (hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
      return check_hip(ctx, hipGetLastError(), "table upload");
    return HCK_OK;
  };
  const size_t tb = (size_t)nm * n * 8;
  if ((rc = up((uint64_t **)&ctx->d_mod, mc.data(), nm * sizeof(ModConst))) ||
      (rc = up(&ctx->d_tw, tw.data(), tb)) || (rc = up(&ctx->d_tw_shoup, tws.data(), tb)) ||
      (rc = up(&ctx->d_itw, itw.data(), tb)) || (rc = up(&ctx->d_itw_shoup, itws.data(), tb)) ||
      (rc = up(&ctx->d_ttw, ttw.data(), tb)) || (rc = up(&ctx->d_ttw_shoup, ttws.data(), tb)) ||
      (rc = up(&ctx->d_ittw, ittw.data(), tb)) ||
      (rc = up(&ctx->d_ittw_shoup, ittws.data(), tb)) ||
      (rc = up(&ctx->d_up_conv, up_conv.data(), up_conv.size() * 8)) ||
      (rc = up(&ctx->d_down_conv, down_conv.data(), down_conv.size() * 8)) ||
      (rc = up(&ctx->d_down_hneg, ctx->down_hneg.data(), ctx->down_hneg.size() * 8))) {
    hck_context_destroy(ctx);
    return rc;
  }
  ctx->def_twist[0] = ctx->d_ttw;
  ctx->def_twist[1] = ctx->d_ttw_shoup;
  ctx->def_twist[2] = ctx->d_ittw;
  ctx->def_twist[3] = ctx->d_ittw_shoup;
  *out = ctx;
  return HCK_OK;
}

const uint64_t *const *split_twists(const hck_context *ctx, int a) {
  const int a0 = (ctx->log_n + 1) / 2;
  if (a == a0) return ctx->def_twist;
  if (a != a0 - 1 && a != a0 + 1) return nullptr;
  const auto &t = ctx->alt_twist[a == a0 + 1];
  return t[0] ? t : nullptr;
}

int set_ntt_split(hck_context *ctx, int a) {
  const int a0 = (ctx->log_n + 1) / 2;
  if (a == 0 || a == a0) {
    ctx->ntt_a = 0;
    return HCK_OK;
  }
  if (!ntt_split_available(ctx->log_n, a))
    return set_error(HCK_EINVAL, "NTT split " + std::to_string(a) + " not available at log N " +
                                     std::to_string(ctx->log_n));
  if (ctx->capturing) return set_error(HCK_EINVAL, "NTT split change during graph capture");
  auto &t = ctx->alt_twist[a == a0 + 1];
  if (!t[0]) {
    const uint32_t nm = ctx->L + ctx->K;
    const size_t n = ctx->n;
    std::vector<uint64_t> ttw(nm * n), ttws(nm * n), ittw(nm * n), ittws(nm * n), pw(n), ipw(n);
    for (uint32_t m = 0; m < nm; m++) {
      const uint64_t q = ctx->mods[m];
      const uint64_t psi = primitive_2n_root(q, n), ipsi = h_invmod(psi, q);
      pw[0] = ipw[0] = 1;
      for (size_t i = 1; i < n; i++) {
        pw[i] = h_mulmod(pw[i - 1], psi, q);
        ipw[i] = h_mulmod(ipw[i - 1], ipsi, q);
      }
      twist_rows(pw, ipw, q, ctx->log_n, a, (size_t)m * n, ttw, ttws, ittw, ittws);
    }
    const std::vector<uint64_t> *src[4] = {&ttw, &ttws, &ittw, &ittws};
    uint64_t *dev[4] = {};
    for (int k = 0; k < 4; k++) {
      hipError_t e = hipMalloc((void **)&dev[k], nm * n * 8);
      if (e == hipSuccess) e = hipMemcpy(dev[k], src[k]->data(), nm * n * 8, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        for (uint64_t *p : dev)
          if (p) (void)hipFree(p);
        (void)hipGetLastError();
        return set_error(HCK_ENOMEM, "NTT split tables: allocation or upload failed");
      }
    }
    for (int k = 0; k < 4; k++) t[k] = dev[k];
  }
  ctx->ntt_a = (uint8_t)a;
  return HCK_OK;
}

void track(hck_context *ctx, void *obj, void (*release)(void *)) { ctx->handles[obj] = release; }

void untrack(hck_context *ctx, void *obj) { ctx->handles.erase(obj); }

void track_server(hck_context *ctx, void *srv, void (*release)(void *)) {
  ctx->servers[srv] = release;
}

void untrack_server(hck_context *ctx, void *srv) { ctx->servers.erase(srv); }

void destroy_context(hck_context *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  abort_capture(ctx);
  // servers stop their workers first; then every live handle gives back its
  // device memory and is detached
  auto servers = std::move(ctx->servers);
  ctx->servers.clear();
  for (auto &kv : servers) kv.second(kv.first);
  auto handles = std::move(ctx->handles);
  ctx->handles.clear();
  for (auto &kv : handles) kv.second(kv.first);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, ctx->ws);
  dev_free(ctx, ctx->lt_scratch);
  dev_free(ctx, ctx->zero_rows);
  for (hck_ciphertext *ct : ctx->ct_pool) {
    dev_free(ctx, ct->data);
    delete ct;
  }
  ctx->ct_pool.clear();
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  for (void *p : {(void *)ctx->d_mod, (void *)ctx->d_tw, (void *)ctx->d_tw_shoup,
                  (void *)ctx->d_itw, (void *)ctx->d_itw_shoup, (void *)ctx->d_ttw,
                  (void *)ctx->d_ttw_shoup, (void *)ctx->d_ittw, (void *)ctx->d_ittw_shoup,
                  (void *)ctx->d_up_conv,
                  (void *)ctx->d_down_conv, (void *)ctx->d_down_hneg})
    if (p) (void)hipFree(p);
  for (auto &t : ctx->alt_twist)
    for (uint64_t *p : t)
      if (p) (void)hipFree(p);
  for (auto &t : ctx->pending) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  // the stream-ordered allocator keeps the freed buffers cached in the
  // device's pool; hand them back, so that a destroyed context's workspace
  // and keys (several GB at N = 2^16) do not crowd later allocations
  if (!ctx->alloc_fn) {
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, ctx->device) == hipSuccess && pool)
      (void)hipMemPoolTrimTo(pool, 0);
    (void)hipGetLastError();
  }
  delete ctx;
}

}  // namespace hck

extern "C" {

const char *hck_last_error(void) { return hck::g_last_error.c_str(); }

int hck_context_create(const hck_params *params, int device, void *hip_stream,
                       hck_context **out) {
  if (!out) return hck::set_error(HCK_EINVAL, "null output");
  *out = nullptr;
  return hck::build_context(params, device, hip_stream, out);
}

int hck_context_destroy(hck_context *ctx) {
  hck::destroy_context(ctx);
  return HCK_OK;
}

int hck_set_allocator(hck_context *ctx, void *(*alloc)(size_t, void *, void *),
                      void (*free_fn)(void *, void *, void *), void *user) {
  if (!ctx) return hck::set_error(HCK_EINVAL, "null context");
  if (!alloc != !free_fn)
    return hck::set_error(HCK_EINVAL, "give both allocator functions or neither");
  if (ctx->live_allocs)
    return hck::set_error(HCK_EINVAL, "the context still holds device buffers of the current "
                                      "allocator");
  ctx->alloc_fn = alloc;
  ctx->free_fn = free_fn;
  ctx->alloc_user = alloc ? user : nullptr;
  return HCK_OK;
}

int hck_context_set_stream(hck_context *ctx, void *hip_stream) {
  if (!ctx) return hck::set_error(HCK_EINVAL, "null context");
  if (ctx->capturing) return hck::set_error(HCK_EINVAL, "stream change during graph capture");
  ctx->stream = (hipStream_t)hip_stream;
  return HCK_OK;
}

int hck_synchronize(hck_context *ctx) {
  if (!ctx) return hck::set_error(HCK_EINVAL, "null context");
  if (ctx->capturing) return hck::set_error(HCK_EINVAL, "wait during graph capture");
  HCK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return HCK_OK;
}

uint32_t hck_galois_element(const hck_context *ctx, int32_t step) {
  return ctx ? hck::galois_of_step(ctx, step) : 0;
}

int hck_timing_enable(hck_context *ctx, int on) {
  if (!ctx) return hck::set_error(HCK_EINVAL, "null context");
  if (ctx->capturing) return hck::set_error(HCK_EINVAL, "timing during graph capture");
  int rc = hck::timing_collect(ctx);
  ctx->timing = on != 0;
  return rc;
}

int hck_timing_reset(hck_context *ctx) {
  if (!ctx) return hck::set_error(HCK_EINVAL, "null context");
  int rc = hck::timing_collect(ctx);
  ctx->timing_total.clear();
  return rc;
}

int hck_timing_read(hck_context *ctx, const char *name, double *total_ms, uint64_t *launches,
                    double *bytes, double *mulmods) {
  if (!ctx || !name) return hck::set_error(HCK_EINVAL, "null argument");
  int rc = hck::timing_collect(ctx);
  if (rc) return rc;
  hck_context::TimingTotal t;
  auto it = ctx->timing_total.find(name);
  if (it != ctx->timing_total.end()) t = it->second;
  if (total_ms) *total_ms = t.ms;
  if (launches) *launches = t.launches;
  if (bytes) *bytes = t.bytes;
  if (mulmods) *mulmods = t.mulmods;
  return HCK_OK;
}

int hck_trace_enable(hck_context *ctx, int on) {
  if (!ctx) return hck::set_error(HCK_EINVAL, "null context");
  if (on) ctx->trace_log.clear();
  ctx->trace = on != 0;
  return HCK_OK;
}

int hck_trace_read(hck_context *ctx, hck_trace_record *out, size_t cap, size_t *count) {
  if (!ctx || !count || (cap && !out)) return hck::set_error(HCK_EINVAL, "null argument");
  *count = ctx->trace_log.size();
  const size_t n = std::min(cap, ctx->trace_log.size());
  if (n) std::memcpy(out, ctx->trace_log.data(), n * sizeof(hck_trace_record));
  return HCK_OK;
}

int hck_timing_names(hck_context *ctx, char *buf, size_t cap) {
  if (!ctx || !buf || cap == 0) return hck::set_error(HCK_EINVAL, "null argument");
  int rc = hck::timing_collect(ctx);
  if (rc) return rc;
  std::string s;
  for (auto &kv : ctx->timing_total) {
    if (!s.empty()) s += ",";
    s += kv.first;
  }
  std::strncpy(buf, s.c_str(), cap - 1);
  buf[cap - 1] = 0;
  return s.size() < cap ? HCK_OK : hck::set_error(HCK_EINVAL, "buffer too small");
}

}  // extern "C"
