// The paper's gesture-classification pipeline (section 3.3.3 example
// pipelines: K3 -> K1 -> K2 + K6, frame accumulation, FC1 -> x^2 -> FC2 ->
// x^2 -> FC3) composed from the library's evaluation calls.
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

int check_plan(const hck_context *ctx, const hck_gesture_plan *p) {
  if (!p) return set_error(HCK_EINVAL, "null plan");
  if (!p->dft_c || !p->dft_s || !p->fc1 || !p->fc2 || !p->fc3 || !p->notch || !p->bias1 ||
      !p->bias2 || !p->bias3)
    return set_error(HCK_EINVAL, "missing plan operand");
  if (p->frames == 0 || p->bins == 0 || p->chirps == 0 || p->hidden1 == 0)
    return set_error(HCK_EINVAL, "empty layout");
  const uint64_t rd = (uint64_t)p->bins * p->chirps;
  if (pow2_at_least(p->frames) * rd != ctx->n / 2)
    return set_error(HCK_EINVAL, "pow2(frames) x bins x chirps must equal N/2");
  if (rd % p->hidden1 || ((rd / p->hidden1) & (rd / p->hidden1 - 1)))
    return set_error(HCK_EINVAL, "bins x chirps / hidden1 must be a power of two");
  return HCK_OK;
}

std::vector<int32_t> plan_steps(const hck_gesture_plan *p) {
  std::vector<int32_t> s;
  const uint32_t rd = p->bins * p->chirps, t2 = pow2_at_least(p->frames);
  for (uint32_t k = rd; k < rd * t2; k *= 2) s.push_back((int32_t)k);
  for (uint32_t k = p->hidden1; k < rd; k *= 2) s.push_back((int32_t)k);
  for (const hck_linear_transform *lt : {p->dft_c, p->dft_s, p->fc1, p->fc2, p->fc3})
    for (auto &kv : lt->groups) {
      if (kv.first != 0) s.push_back(kv.first * (int32_t)lt->n1);
      for (auto &bp : kv.second)
        if (bp.first != 0) s.push_back(bp.first);
    }
  std::sort(s.begin(), s.end());
  s.erase(std::unique(s.begin(), s.end()), s.end());
  return s;
}

int rotsum(hck_context *ctx, hck_ciphertext *c, uint32_t step, uint32_t count,
           const hck_galois_keys *gks, Scratch &sc) {
  hck_ciphertext *t = sc.get();
  for (uint64_t s = step; s < (uint64_t)step * count; s *= 2) {
    TRY(hck_rotate(ctx, c, (int32_t)s, gks, t));
    TRY(hck_add(ctx, c, t, c));
  }
  return HCK_OK;
}

int mul_rs(hck_context *ctx, const hck_ciphertext *a, const hck_ciphertext *b,
           const hck_switch_key *rlk, hck_ciphertext *out, Scratch &sc) {
  hck_ciphertext *t = sc.get();
  TRY(hck_mul(ctx, a, b, t));
  TRY(hck_relinearize(ctx, t, rlk, out));
  return hck_rescale(ctx, out, out);
}

// out = rescale(fc(x)) + bias
int dense(hck_context *ctx, const hck_linear_transform *fc, const hck_plaintext *bias,
          const hck_ciphertext *x, const hck_galois_keys *gks, hck_ciphertext *out,
          uint32_t sum_from, uint32_t sum_count, Scratch &sc) {
  const uint32_t zero = 0;
  TRY(hck_lt_eval(ctx, &x, 1, &fc, &zero, &zero, nullptr, 1, gks, &out, 1,
                  HCK_LT_HOIST_BABY | HCK_LT_HOIST_GIANT));
  TRY(hck_rescale(ctx, out, out));
  if (sum_count > 1) TRY(rotsum(ctx, out, sum_from, sum_count, gks, sc));
  return hck_add_plain(ctx, out, bias, out);
}

// K3 -> K1 -> K6 -> K2 of one ciphertext pair at the plan's level: feat =
// P P^4 in place (every frame block of the pair at once).  tap(i, c) records
// intermediate i.
template <class Tap>
int front_end(hck_context *ctx, const hck_gesture_plan *p, const hck_ciphertext *re,
              const hck_ciphertext *im, const hck_switch_key *rlk, const hck_galois_keys *gks,
              hck_ciphertext *feat, Tap &&tap) {
  Scratch sc(ctx);
  // K3: Doppler DFT (complex, Eq. dft_re form)
  hck_ciphertext *d[2] = {sc.get(), sc.get()};
  {
    const hck_ciphertext *ins[2] = {re, im};
    const hck_linear_transform *lts[4] = {p->dft_c, p->dft_s, p->dft_s, p->dft_c};
    const uint32_t tin[4] = {0, 1, 0, 1}, tout[4] = {0, 0, 1, 1};
    const int32_t sign[4] = {1, -1, 1, 1};
    TRY(hck_lt_eval(ctx, ins, 2, lts, tin, tout, sign, 4, gks, d, 2,
                    HCK_LT_HOIST_BABY | HCK_LT_HOIST_GIANT));
    TRY(hck_rescale(ctx, d[0], d[0]));
    TRY(hck_rescale(ctx, d[1], d[1]));
  }
  TRY(tap(0, d[0]));
  TRY(tap(1, d[1]));
  // K1: power, K6: notch
  hck_ciphertext *pw = sc.get(), *t = sc.get(), *u = sc.get();
  TRY(hck_mul(ctx, d[0], d[0], t));
  TRY(hck_mul(ctx, d[1], d[1], u));
  TRY(hck_add(ctx, t, u, t));
  TRY(hck_relinearize(ctx, t, rlk, pw));
  TRY(hck_rescale(ctx, pw, pw));
  TRY(tap(2, pw));
  TRY(hck_mul_plain(ctx, pw, p->notch, pw));
  TRY(hck_rescale(ctx, pw, pw));
  TRY(tap(3, pw));
  // K2: gamma = 4, feature = P w
  hck_ciphertext *p2 = sc.get(), *p4 = sc.get(), *pl = sc.get();
  TRY(mul_rs(ctx, pw, pw, rlk, p2, sc));
  TRY(mul_rs(ctx, p2, p2, rlk, p4, sc));
  TRY(tap(4, p4));
  TRY(hck_drop_level(ctx, pw, p4->level, pl));
  return mul_rs(ctx, pl, p4, rlk, feat, sc);
}

// the FC network with square activations on the accumulated features, which
// sit in every block of bins x chirps slots
template <class Tap>
int fc_tail(hck_context *ctx, const hck_gesture_plan *p, const hck_ciphertext *feat,
            const hck_switch_key *rlk, const hck_galois_keys *gks, hck_ciphertext *out,
            Tap &&tap) {
  Scratch sc(ctx);
  const uint32_t rd = p->bins * p->chirps;
  hck_ciphertext *y = sc.get(), *h = sc.get();
  TRY(dense(ctx, p->fc1, p->bias1, feat, gks, y, p->hidden1, rd / p->hidden1, sc));
  TRY(tap(6, y));
  TRY(mul_rs(ctx, y, y, rlk, h, sc));
  TRY(dense(ctx, p->fc2, p->bias2, h, gks, y, 0, 1, sc));
  TRY(tap(7, y));
  TRY(mul_rs(ctx, y, y, rlk, h, sc));
  return dense(ctx, p->fc3, p->bias3, h, gks, out, 0, 1, sc);
}

// checks shared by both packings: the plan, its keys and the inputs' level
int check_call(hck_context *ctx, const hck_gesture_plan *p, const hck_galois_keys *gks,
               uint32_t level) {
  TRY(check_plan(ctx, p));
  if (p->dft_c->level < 11) return set_error(HCK_ELEVEL, "plan encoded below the pipeline depth");
  if (level < p->dft_c->level)
    return set_error(HCK_ELEVEL, "inputs must share a level of at least the plan's level");
  for (int32_t s : plan_steps(p))
    if (!gks->keys.count(galois_of_step(ctx, s)))
      return set_error(HCK_ENOKEY, "missing Galois key for step " + std::to_string(s));
  return HCK_OK;
}

// ---- the CNN variant ----------------------------------------------------

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

int act_depth(uint32_t degree) {
  int bits = 0;
  while ((1u << bits) < degree) bits++;   // ceil(log2 degree)
  return bits + 1;
}

int check_cnn_plan(const hck_context *ctx, const hck_gesture_cnn_plan *p) {
  if (!p) return set_error(HCK_EINVAL, "null plan");
  if (!p->dft_c || !p->dft_s || !p->notch || !p->conv1 || !p->conv2 || !p->dense1 ||
      !p->dense2 || !p->bias1 || !p->bias2)
    return set_error(HCK_EINVAL, "missing plan operand");
  if (p->act_degree < 1 || p->act_degree > 15 || !p->act_coeffs)
    return set_error(HCK_EINVAL, "activation degree must be 1 .. 15 with its coefficients");
  if (!p->frames || !p->bins || !p->chirps || !p->c1 || !p->c2 || !p->hidden || !p->classes)
    return set_error(HCK_EINVAL, "empty layout");
  const uint64_t rd = (uint64_t)p->bins * p->chirps;
  if (pow2_at_least(p->frames) * rd != ctx->n / 2)
    return set_error(HCK_EINVAL, "pow2(frames) x bins x chirps must equal N/2");
  if (p->bins % 8 || p->chirps % 8)
    return set_error(HCK_EINVAL, "bins and chirps must be multiples of 8");
  const uint64_t blocks = ctx->n / 2 / rd;
  if (blocks % p->c1 || blocks % p->c2)
    return set_error(HCK_EINVAL, "the block count must be a multiple of both channel counts");
  const uint64_t period = p->c2 * rd;
  if (period % p->hidden || !is_pow2(period / p->hidden))
    return set_error(HCK_EINVAL, "c2 bins chirps / hidden must be a power of two");
  return HCK_OK;
}

std::vector<int32_t> cnn_plan_steps(const hck_gesture_cnn_plan *p) {
  std::vector<int32_t> s;
  const uint32_t rd = p->bins * p->chirps, t2 = pow2_at_least(p->frames);
  const uint32_t period = p->c2 * rd;
  for (uint32_t k = rd; k < rd * t2; k *= 2) s.push_back((int32_t)k);
  for (uint32_t k = p->hidden; k < period; k *= 2) s.push_back((int32_t)k);
  for (const hck_linear_transform *lt :
       {p->dft_c, p->dft_s, p->conv1, p->conv2, p->dense1, p->dense2})
    for (auto &kv : lt->groups) {
      if (kv.first != 0) s.push_back(kv.first * (int32_t)lt->n1);
      for (auto &bp : kv.second)
        if (bp.first != 0) s.push_back(bp.first);
    }
  std::sort(s.begin(), s.end());
  s.erase(std::unique(s.begin(), s.end()), s.end());
  return s;
}

// out = rescale(lt(x)), hoisted baby steps and one ModDown per giant step
int apply_lt(hck_context *ctx, const hck_linear_transform *lt, const hck_ciphertext *x,
             const hck_galois_keys *gks, hck_ciphertext *out) {
  const uint32_t zero = 0;
  TRY(hck_lt_eval(ctx, &x, 1, &lt, &zero, &zero, nullptr, 1, gks, &out, 1,
                  HCK_LT_HOIST_BABY | HCK_LT_HOIST_GIANT));
  return hck_rescale(ctx, out, out);
}

}  // namespace

extern "C" {

int hck_gesture_required_steps(const hck_context *ctx, const hck_gesture_plan *plan,
                               int32_t *steps, uint32_t cap, uint32_t *n) {
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

int hck_gesture_eval(hck_context *ctx, const hck_gesture_plan *p, const hck_ciphertext *re,
                     const hck_ciphertext *im, const hck_galois_keys *gks,
                     const hck_switch_key *rlk, hck_ciphertext *out) {
  return hck_gesture_eval_taps(ctx, p, re, im, gks, rlk, out, nullptr);
}

int hck_gesture_eval_taps(hck_context *ctx, const hck_gesture_plan *p, const hck_ciphertext *re,
                          const hck_ciphertext *im, const hck_galois_keys *gks,
                          const hck_switch_key *rlk, hck_ciphertext *out,
                          hck_ciphertext *const *taps) {
  if (!ctx || !re || !im || !gks || !rlk || !out) return set_error(HCK_EINVAL, "null argument");
  if (foreign(ctx, re) || foreign(ctx, im) || foreign(ctx, gks) || foreign(ctx, rlk) ||
      foreign(ctx, out))
    return set_error(HCK_EINVAL, "handle of another (or a destroyed) context");
  if (taps)
    for (int i = 0; i < HCK_GESTURE_TAPS; i++)
      if (taps[i] && (taps[i] == re || taps[i] == im))
        return set_error(HCK_EINVAL, "taps must not alias inputs");
  auto tap = [&](int i, const hck_ciphertext *c) {
    hck_ciphertext *t = taps ? taps[i] : nullptr;
    return t ? hck_drop_level(ctx, c, c->level, t) : HCK_OK;
  };
  if (re->level != im->level) return set_error(HCK_ELEVEL, "inputs must share a level");
  TRY(check_call(ctx, p, gks, re->level));
  // the plan's operands are encoded for inputs at the level of its Doppler
  // DFT; inputs above it are dropped to it
  const uint32_t l0 = p->dft_c->level;
  Scratch sc(ctx);
  if (re->level > l0) {
    hck_ciphertext *a = sc.get(), *b = sc.get();
    TRY(hck_drop_level(ctx, re, l0, a));
    TRY(hck_drop_level(ctx, im, l0, b));
    re = a;
    im = b;
  }
  const uint32_t rd = p->bins * p->chirps, t2 = pow2_at_least(p->frames);
  hck_ciphertext *feat = sc.get();
  TRY(front_end(ctx, p, re, im, rlk, gks, feat, tap));
  // frame accumulation: every block of rd slots ends with the sum of all
  TRY(rotsum(ctx, feat, rd, t2, gks, sc));
  TRY(tap(5, feat));
  return fc_tail(ctx, p, feat, rlk, gks, out, tap);
}

int hck_gesture_eval_frames(hck_context *ctx, const hck_gesture_plan *p,
                            const hck_ciphertext *const *re, const hck_ciphertext *const *im,
                            uint32_t n_frames, const hck_galois_keys *gks,
                            const hck_switch_key *rlk, hck_ciphertext *out) {
  if (!ctx || !re || !im || !gks || !rlk || !out) return set_error(HCK_EINVAL, "null argument");
  if (n_frames == 0 || n_frames > HCK_GESTURE_MAX_FRAMES)
    return set_error(HCK_EINVAL, "frame count out of range");
  if (foreign(ctx, gks) || foreign(ctx, rlk) || foreign(ctx, out))
    return set_error(HCK_EINVAL, "handle of another (or a destroyed) context");
  for (uint32_t f = 0; f < n_frames; f++) {
    if (!re[f] || !im[f]) return set_error(HCK_EINVAL, "null frame ciphertext");
    if (foreign(ctx, re[f]) || foreign(ctx, im[f]))
      return set_error(HCK_EINVAL, "handle of another (or a destroyed) context");
    if (re[f]->level != re[0]->level || im[f]->level != re[0]->level)
      return set_error(HCK_ELEVEL, "frame ciphertexts must share a level");
    if (re[f]->scale != re[0]->scale || im[f]->scale != re[0]->scale)
      return set_error(HCK_ESCALE, "frame ciphertexts must share a scale");
  }
  TRY(check_call(ctx, p, gks, re[0]->level));
  const uint32_t l0 = p->dft_c->level;
  auto no_tap = [](int, const hck_ciphertext *) { return HCK_OK; };
  Scratch sc(ctx);
  hck_ciphertext *acc = sc.get(), *feat = sc.get(), *a = sc.get(), *b = sc.get();
  for (uint32_t f = 0; f < n_frames; f++) {
    const hck_ciphertext *x = re[f], *y = im[f];
    if (x->level > l0) {
      TRY(hck_drop_level(ctx, x, l0, a));
      TRY(hck_drop_level(ctx, y, l0, b));
      x = a;
      y = b;
    }
    TRY(front_end(ctx, p, x, y, rlk, gks, f ? feat : acc, no_tap));
    if (f) TRY(hck_add(ctx, acc, feat, acc));
  }
  // the frame sum sits in the first block of rd slots; the FC network reads
  // it in every block, as the batched packing leaves it
  const uint32_t rd = p->bins * p->chirps;
  TRY(rotsum(ctx, acc, rd, (uint32_t)(ctx->n / 2 / rd), gks, sc));
  return fc_tail(ctx, p, acc, rlk, gks, out, no_tap);
}

int hck_gesture_cnn_required_steps(const hck_context *ctx, const hck_gesture_cnn_plan *plan,
                                   int32_t *steps, uint32_t cap, uint32_t *n) {
  if (!ctx || !n) return set_error(HCK_EINVAL, "null argument");
  TRY(check_cnn_plan(ctx, plan));
  const std::vector<int32_t> s = cnn_plan_steps(plan);
  *n = (uint32_t)s.size();
  if (steps) {
    if (cap < s.size()) return set_error(HCK_EINVAL, "steps buffer too small");
    std::copy(s.begin(), s.end(), steps);
  }
  return HCK_OK;
}

int hck_gesture_cnn_eval(hck_context *ctx, const hck_gesture_cnn_plan *p,
                         const hck_ciphertext *re, const hck_ciphertext *im,
                         const hck_galois_keys *gks, const hck_switch_key *rlk,
                         hck_ciphertext *out, hck_ciphertext *const *taps) {
  if (!ctx || !re || !im || !gks || !rlk || !out) return set_error(HCK_EINVAL, "null argument");
  if (foreign(ctx, re) || foreign(ctx, im) || foreign(ctx, gks) || foreign(ctx, rlk) ||
      foreign(ctx, out))
    return set_error(HCK_EINVAL, "handle of another (or a destroyed) context");
  TRY(check_cnn_plan(ctx, p));
  if (taps)
    for (int i = 0; i < HCK_GESTURE_CNN_TAPS; i++)
      if (taps[i] && (taps[i] == re || taps[i] == im || foreign(ctx, taps[i])))
        return set_error(HCK_EINVAL, "taps must be this context's and not alias inputs");
  if (re->level != im->level) return set_error(HCK_ELEVEL, "inputs must share a level");
  const uint32_t l0 = p->dft_c->level;
  const uint32_t a = (uint32_t)act_depth(p->act_degree);
  if (l0 < 10 + 3 * a) return set_error(HCK_ELEVEL, "plan encoded below the network's depth");
  if (re->level < l0)
    return set_error(HCK_ELEVEL, "inputs must share a level of at least the plan's level");
  if (p->conv1->level != l0 - 6 || p->conv2->level != l0 - 7 - a ||
      p->dense1->level != l0 - 8 - 2 * a || p->dense2->level != l0 - 9 - 3 * a)
    return set_error(HCK_ELEVEL, "plan transforms at levels other than the network's");
  for (int32_t s : cnn_plan_steps(p))
    if (!gks->keys.count(galois_of_step(ctx, s)))
      return set_error(HCK_ENOKEY, "missing Galois key for step " + std::to_string(s));
  auto tap = [&](int i, const hck_ciphertext *c) {
    hck_ciphertext *t = taps ? taps[i] : nullptr;
    return t ? hck_drop_level(ctx, c, c->level, t) : HCK_OK;
  };
  Scratch sc(ctx);
  if (re->level > l0) {
    hck_ciphertext *x = sc.get(), *y = sc.get();
    TRY(hck_drop_level(ctx, re, l0, x));
    TRY(hck_drop_level(ctx, im, l0, y));
    re = x;
    im = y;
  }
  // front end of the gesture pipeline (its plan fields read there)
  hck_gesture_plan fe{};
  fe.dft_c = p->dft_c;
  fe.dft_s = p->dft_s;
  fe.notch = p->notch;
  auto no_tap = [](int, const hck_ciphertext *) { return HCK_OK; };
  const uint32_t rd = p->bins * p->chirps, t2 = pow2_at_least(p->frames);
  hck_ciphertext *feat = sc.get(), *u = sc.get(), *v = sc.get();
  TRY(front_end(ctx, &fe, re, im, rlk, gks, feat, no_tap));
  TRY(rotsum(ctx, feat, rd, t2, gks, sc));
  TRY(tap(0, feat));
  const uint32_t deg = p->act_degree;
  TRY(apply_lt(ctx, p->conv1, feat, gks, u));
  TRY(hck_poly_eval(ctx, u, p->act_coeffs, deg, rlk, v));
  TRY(tap(1, v));
  TRY(apply_lt(ctx, p->conv2, v, gks, u));
  TRY(hck_poly_eval(ctx, u, p->act_coeffs, deg, rlk, v));
  TRY(tap(2, v));
  TRY(apply_lt(ctx, p->dense1, v, gks, u));
  TRY(rotsum(ctx, u, p->hidden, p->c2 * rd / p->hidden, gks, sc));
  TRY(hck_add_plain(ctx, u, p->bias1, u));
  TRY(hck_poly_eval(ctx, u, p->act_coeffs, deg, rlk, v));
  TRY(tap(3, v));
  TRY(apply_lt(ctx, p->dense2, v, gks, out));
  return hck_add_plain(ctx, out, p->bias2, out);
}

}  // extern "C"
