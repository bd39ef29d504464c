// Polynomial evaluation sum_k c_k x^k on ciphertexts, slot-wise: the
// building block of polynomial approximations (magnitudes, activations) in
// the pipelines of section 3.3.  Composed from the library's operations:
//   powers   x^(2^j) by squaring; any other x^k = x^a x^(k-a), a the largest
//            power of two below k, the factor on the higher level dropped to
//            the other's; every product relinearized and rescaled, so x^k
//            sits at level l - ceil(log2 k);
//   terms    each x^k with c_k != 0, dropped to level l_f + 1
//            (l_f = l - ceil(log2 d) - 1), times the constant c_k encoded at
//            scale s q_(l_f+1) / scale(x^k) (s: the input's scale), rescaled:
//            every term lands on level l_f at scale s;
//   sum      terms added in increasing k, then c_0 at the sum's scale.
#include <vector>

#include "internal.h"

using namespace hck;

namespace {

#define TRY(expr)         \
  do {                    \
    int _rc = (expr);     \
    if (_rc) return _rc;  \
  } while (0)

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

// a plaintext handle released on scope exit
struct Pt {
  hck_plaintext *p = nullptr;
  ~Pt() { hck_plaintext_destroy(p); }
};

uint32_t ceil_log2(uint32_t v) {
  uint32_t b = 0;
  while ((1u << b) < v) b++;
  return b;
}

}  // namespace

extern "C" {

int hck_poly_eval(hck_context *ctx, const hck_ciphertext *x, const double *coeffs,
                  uint32_t degree, const hck_switch_key *rlk, hck_ciphertext *out) {
  if (!ctx || !x || !coeffs || !rlk || !out) return set_error(HCK_EINVAL, "null argument");
  if (foreign(ctx, x) || foreign(ctx, rlk) || foreign(ctx, out))
    return set_error(HCK_EINVAL, "handle of another (or a destroyed) context");
  if (out == x) return set_error(HCK_EINVAL, "the output must not alias the input");
  if (degree < 1 || degree > 64) return set_error(HCK_EINVAL, "degree must be 1..64");
  bool any = false;
  for (uint32_t k = 1; k <= degree; k++) any = any || coeffs[k] != 0.0;
  if (!any) return set_error(HCK_EINVAL, "need a nonzero coefficient of degree >= 1");
  if (x->size != 2) return set_error(HCK_EINVAL, "need a 2-part ciphertext");
  const uint32_t depth = ceil_log2(degree) + 1;
  if (x->level < depth) return set_error(HCK_ELEVEL, "not enough levels for this degree");
  Scratch sc(ctx);
  std::vector<hck_ciphertext *> pw(degree + 1, nullptr);
  pw[1] = const_cast<hck_ciphertext *>(x);
  for (uint32_t k = 2; k <= degree; k++) {
    const uint32_t a = 1u << (ceil_log2(k) - 1);  // largest power of two below k
    const hck_ciphertext *u = pw[a], *v = pw[k - a];
    const uint32_t lv = u->level < v->level ? u->level : v->level;
    hck_ciphertext *ud = sc.get(), *vd = sc.get(), *t = sc.get();
    TRY(hck_drop_level(ctx, u, lv, ud));
    TRY(hck_drop_level(ctx, v, lv, vd));
    TRY(hck_mul(ctx, ud, vd, t));
    pw[k] = sc.get();
    TRY(hck_relinearize(ctx, t, rlk, pw[k]));
    TRY(hck_rescale(ctx, pw[k], pw[k]));
  }
  const uint32_t lf = x->level - depth;
  bool first = true;
  for (uint32_t k = 1; k <= degree; k++) {
    if (coeffs[k] == 0.0) continue;
    hck_ciphertext *t = sc.get(), *term = first ? out : sc.get();
    TRY(hck_drop_level(ctx, pw[k], lf + 1, t));
    Pt pt;
    TRY(hck_encode_const(ctx, coeffs[k], x->scale * (double)ctx->mods[lf + 1] / t->scale, lf + 1,
                         &pt.p));
    TRY(hck_mul_plain(ctx, t, pt.p, term));
    TRY(hck_rescale(ctx, term, term));
    if (!first) TRY(hck_add(ctx, out, term, out));
    first = false;
  }
  if (coeffs[0] != 0.0) {
    Pt pt;
    TRY(hck_encode_const(ctx, coeffs[0], out->scale, lf, &pt.p));
    TRY(hck_add_plain(ctx, out, pt.p, out));
  }
  return HCK_OK;
}

}  // extern "C"
