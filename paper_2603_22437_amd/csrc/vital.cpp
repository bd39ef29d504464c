// The paper's vital-sign pipeline (section 3.3.3 example pipelines:
// K1 -> K2 -> K4 -> K5 -> K7 -> K3 -> K1 -> K2) composed from the library's
// evaluation calls.  Every rotate-and-sum chain advances all its independent
// members (num/den, I/Q, real/imaginary parts of both bands) by one step per
// batched key switch (hck_rotate_many), so one window issues as few key-switch
// launch sequences as its dependency depth allows.
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

uint32_t pow2_at_least(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p *= 2;
  return p;
}

// Scratch ciphertexts returned to the context's pool on scope exit.
struct Scratch {
  hck_context *ctx;
  std::vector<hck_ciphertext *> held;
  explicit Scratch(hck_context *c) : ctx(c) {}
  ~Scratch() {
    for (hck_ciphertext *c : held) pool_put(ctx, c);
  }
  hck_ciphertext *get() {
    hck_ciphertext *c = pool_get(ctx);
    held.push_back(c);
    return c;
  }
};

int check_plan(const hck_context *ctx, const hck_vital_plan *p) {
  if (!p) return set_error(HCK_EINVAL, "null plan");
  if (p->frames == 0 || p->bins == 0 || (p->bins & (p->bins - 1)))
    return set_error(HCK_EINVAL, "bins must be a power of two");
  if ((uint64_t)pow2_at_least(p->frames) * p->bins > ctx->n / 2)
    return set_error(HCK_EINVAL, "frames x bins do not fit the slots");
  if (p->taylor_order != 1 && p->taylor_order != 3)
    return set_error(HCK_EINVAL, "Taylor order must be 1 or 3");
  if (p->lanes_resp == 0 || p->lanes_hr == 0 ||
      pow2_at_least(p->lanes_resp + p->lanes_hr) > p->bins)
    return set_error(HCK_EINVAL, "DFT lanes do not fit the range bins");
  if (!p->bin_index || !p->bin_mask || !p->fir_resp || !p->fir_hr || !p->dft_re_resp ||
      !p->dft_im_resp || !p->dft_re_hr || !p->dft_im_hr || !p->freq_resp || !p->mask_resp ||
      !p->freq_hr || !p->mask_hr || (p->taylor_order == 3 && !p->third))
    return set_error(HCK_EINVAL, "missing plan operand");
  return HCK_OK;
}

std::vector<int32_t> plan_steps(const hck_vital_plan *p) {
  std::vector<int32_t> s;
  const uint32_t r = p->bins, t2 = pow2_at_least(p->frames);
  const uint32_t c_all = pow2_at_least(p->lanes_resp + p->lanes_hr);
  for (uint32_t k = r; k < r * t2; k *= 2) s.push_back((int32_t)k);
  for (uint32_t k = 1; k < r; k *= 2) s.push_back((int32_t)k);
  s.push_back(-(int32_t)r);
  for (uint32_t k = 1; k < c_all; k *= 2) s.push_back(-(int32_t)k);
  for (const hck_linear_transform *lt : {p->fir_resp, p->fir_hr})
    for (auto &kv : lt->groups) {
      if (kv.first != 0) s.push_back(kv.first * (int32_t)lt->n1);
      for (auto &bp : kv.second)
        if (bp.first != 0) s.push_back(bp.first);
    }
  std::sort(s.begin(), s.end());
  s.erase(std::unique(s.begin(), s.end()), s.end());
  return s;
}

// c_i <- c_i + Rot(c_i, step) + ... over `count` (a power of two) shifts, for
// every member at once
int rotsum(hck_context *ctx, std::vector<hck_ciphertext *> cs, int32_t step, uint32_t count,
           const hck_galois_keys *gks, Scratch &sc) {
  std::vector<hck_ciphertext *> tmp;
  for (size_t i = 0; i < cs.size(); i++) tmp.push_back(sc.get());
  for (uint64_t s = (uint64_t)step; s < (uint64_t)step * count; s *= 2) {
    TRY(hck_rotate_many(ctx, cs.data(), (uint32_t)cs.size(), (int32_t)s, gks, tmp.data()));
    for (size_t i = 0; i < cs.size(); i++) TRY(hck_add(ctx, cs[i], tmp[i], cs[i]));
  }
  return HCK_OK;
}

// out = relin(a b) rescaled
int mul_rs(hck_context *ctx, const hck_ciphertext *a, const hck_ciphertext *b,
           const hck_switch_key *rlk, hck_ciphertext *out, Scratch &sc) {
  hck_ciphertext *t = sc.get();
  TRY(hck_mul(ctx, a, b, t));
  TRY(hck_relinearize(ctx, t, rlk, out));
  return hck_rescale(ctx, out, out);
}

// out = relin(a b + c d) (op 0) or relin(a b - c d) (op 1), rescaled
int mul2_rs(hck_context *ctx, const hck_ciphertext *a, const hck_ciphertext *b,
            const hck_ciphertext *c, const hck_ciphertext *d, int op, const hck_switch_key *rlk,
            hck_ciphertext *out, Scratch &sc) {
  hck_ciphertext *t = sc.get(), *u = sc.get();
  TRY(hck_mul(ctx, a, b, t));
  TRY(hck_mul(ctx, c, d, u));
  TRY(op ? hck_sub(ctx, t, u, t) : hck_add(ctx, t, u, t));
  TRY(hck_relinearize(ctx, t, rlk, out));
  return hck_rescale(ctx, out, out);
}

// out = (a pt) rescaled
int mulpt_rs(hck_context *ctx, const hck_ciphertext *a, const hck_plaintext *pt,
             hck_ciphertext *out) {
  TRY(hck_mul_plain(ctx, a, pt, out));
  return hck_rescale(ctx, out, out);
}

}  // namespace

extern "C" {

int hck_vital_required_steps(const hck_context *ctx, const hck_vital_plan *plan, int32_t *steps,
                             uint32_t cap, uint32_t *n) {
  if (!ctx || !n) return set_error(HCK_EINVAL, "null argument");
  TRY(check_plan(ctx, plan));
  const std::vector<int32_t> s = plan_steps(plan);
  *n = (uint32_t)s.size();
  if (steps) {
    if (cap < s.size()) return set_error(HCK_EINVAL, "steps buffer too small");
    std::copy(s.begin(), s.end(), steps);
  }
  return HCK_OK;
}

int hck_vital_eval(hck_context *ctx, const hck_vital_plan *p, const hck_ciphertext *re,
                   const hck_ciphertext *im, const hck_galois_keys *gks,
                   const hck_switch_key *rlk, hck_ciphertext *const *out) {
  if (!ctx || !re || !im || !gks || !rlk || !out) return set_error(HCK_EINVAL, "null argument");
  TRY(check_plan(ctx, p));
  for (int i = 0; i < 6; i++)
    if (!out[i]) return set_error(HCK_EINVAL, "null output");
  const uint32_t depth = p->taylor_order == 3 ? 11 : 9;
  if (re->level != im->level || re->level < depth)
    return set_error(HCK_ELEVEL, "inputs must share a level of at least the pipeline depth");
  for (int32_t s : plan_steps(p))
    if (!gks->keys.count(galois_of_step(ctx, s)))
      return set_error(HCK_ENOKEY, "missing Galois key for step " + std::to_string(s));
  Scratch sc(ctx);
  const int32_t r = (int32_t)p->bins;
  const uint32_t t2 = pow2_at_least(p->frames);
  const uint32_t c_resp = pow2_at_least(p->lanes_resp);
  const uint32_t c_all = pow2_at_least(p->lanes_resp + p->lanes_hr);

  // K1: p = Re^2 + Im^2, E = sum over frames
  hck_ciphertext *pw = sc.get(), *e = sc.get();
  TRY(mul2_rs(ctx, re, re, im, im, 0, rlk, pw, sc));
  TRY(hck_drop_level(ctx, pw, pw->level, e));  // a copy
  TRY(rotsum(ctx, {e}, r, t2, gks, sc));
  // K2 over bins (gamma = 2) and K4 (P_phi = 2) share their squarings' level
  hck_ciphertext *w = sc.get(), *m = sc.get();
  TRY(mul_rs(ctx, e, e, rlk, w, sc));
  TRY(mul_rs(ctx, pw, pw, rlk, m, sc));
  TRY(mulpt_rs(ctx, w, p->bin_index, out[0]));
  TRY(mulpt_rs(ctx, w, p->bin_mask, out[1]));
  hck_ciphertext *re2 = sc.get(), *im2 = sc.get(), *it = sc.get(), *qt = sc.get();
  TRY(hck_drop_level(ctx, re, m->level, re2));
  TRY(hck_drop_level(ctx, im, m->level, im2));
  TRY(mul_rs(ctx, m, re2, rlk, it, sc));
  TRY(mul_rs(ctx, m, im2, rlk, qt, sc));
  TRY(rotsum(ctx, {out[0], out[1], it, qt}, 1, (uint32_t)r, gks, sc));
  // K5: both bands' FIR of I and Q in one BSGS evaluation
  hck_ciphertext *f[4] = {sc.get(), sc.get(), sc.get(), sc.get()};
  {
    const hck_ciphertext *ins[2] = {it, qt};
    const hck_linear_transform *lts[4] = {p->fir_resp, p->fir_resp, p->fir_hr, p->fir_hr};
    const uint32_t tin[4] = {0, 1, 0, 1}, tout[4] = {0, 1, 2, 3};
    TRY(hck_lt_eval(ctx, ins, 2, lts, tin, tout, nullptr, 4, gks, f, 4,
                    HCK_LT_HOIST_BABY | HCK_LT_HOIST_GIANT));
    for (int i = 0; i < 4; i++) TRY(hck_rescale(ctx, f[i], f[i]));
  }
  // K7: the previous frame by a rotation of -R (all four in one batch)
  hck_ciphertext *f1[4] = {sc.get(), sc.get(), sc.get(), sc.get()};
  TRY(hck_rotate_many(ctx, f, 4, -r, gks, f1));
  hck_ciphertext *dphi[2] = {sc.get(), sc.get()};
  for (int b = 0; b < 2; b++) {
    hck_ciphertext *fi = f[2 * b], *fq = f[2 * b + 1], *fi1 = f1[2 * b], *fq1 = f1[2 * b + 1];
    hck_ciphertext *y = sc.get();
    TRY(mul2_rs(ctx, fq, fi1, fi, fq1, 1, rlk, y, sc));
    if (p->taylor_order == 1) {
      TRY(hck_drop_level(ctx, y, y->level, dphi[b]));
      continue;
    }
    hck_ciphertext *x = sc.get(), *x2 = sc.get(), *y6 = sc.get(), *a = sc.get();
    hck_ciphertext *y2 = sc.get(), *yc = sc.get(), *bb = sc.get();
    TRY(mul2_rs(ctx, fi, fi1, fq, fq1, 0, rlk, x, sc));
    TRY(mul_rs(ctx, x, x, rlk, x2, sc));
    TRY(hck_drop_level(ctx, y, x2->level, y6));
    TRY(mul_rs(ctx, y6, x2, rlk, a, sc));
    TRY(mul_rs(ctx, y, y, rlk, y2, sc));
    TRY(mulpt_rs(ctx, y, p->third, yc));
    TRY(mul_rs(ctx, yc, y2, rlk, bb, sc));
    TRY(hck_sub(ctx, a, bb, dphi[b]));
  }
  // K3: copy dphi into the band's lanes, weight, sum over frames
  for (uint32_t s = 1; s < c_all; s *= 2) {
    const uint32_t nb = s < c_resp ? 2 : 1;   // respiration needs fewer lanes
    hck_ciphertext *src[2] = {dphi[1], dphi[0]};
    hck_ciphertext *tmp[2] = {sc.get(), sc.get()};
    TRY(hck_rotate_many(ctx, src, nb, -(int32_t)s, gks, tmp));
    for (uint32_t i = 0; i < nb; i++) TRY(hck_add(ctx, src[i], tmp[i], src[i]));
  }
  hck_ciphertext *xs[4] = {sc.get(), sc.get(), sc.get(), sc.get()};
  TRY(mulpt_rs(ctx, dphi[0], p->dft_re_resp, xs[0]));
  TRY(mulpt_rs(ctx, dphi[0], p->dft_im_resp, xs[1]));
  TRY(mulpt_rs(ctx, dphi[1], p->dft_re_hr, xs[2]));
  TRY(mulpt_rs(ctx, dphi[1], p->dft_im_hr, xs[3]));
  TRY(rotsum(ctx, {xs[0], xs[1], xs[2], xs[3]}, r, t2, gks, sc));
  TRY(hck_add(ctx, xs[0], xs[2], xs[0]));
  TRY(hck_add(ctx, xs[1], xs[3], xs[1]));
  // K1 on the spectrum, K2: sharpening and weighted frequency averages
  hck_ciphertext *pspec = sc.get(), *sh = sc.get();
  TRY(mul2_rs(ctx, xs[0], xs[0], xs[1], xs[1], 0, rlk, pspec, sc));
  TRY(mul_rs(ctx, pspec, pspec, rlk, sh, sc));
  TRY(mulpt_rs(ctx, sh, p->freq_resp, out[2]));
  TRY(mulpt_rs(ctx, sh, p->mask_resp, out[3]));
  TRY(mulpt_rs(ctx, sh, p->freq_hr, out[4]));
  TRY(mulpt_rs(ctx, sh, p->mask_hr, out[5]));
  TRY(rotsum(ctx, {out[2], out[3], out[4], out[5]}, 1, c_all, gks, sc));
  return HCK_OK;
}

}  // extern "C"
