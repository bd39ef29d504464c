// The paper's vital-sign pipeline (section 3.3.3 example pipelines:
// K1 -> K2 -> K4 -> K5 -> K7 -> K3 -> K1 -> K2) composed from the library's
// evaluation calls.  Every rotate-and-sum chain advances all its independent
// members (num/den, I/Q, real/imaginary parts) by one step per
// batched key switch, so one window issues as few key-switch
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

// The bin branch (K1 -> K2) needs log2(gamma) + 1 more levels and ends at
// level 1, so its energy sums run on few limbs: at level 2 + log2(gamma), its
// plaintexts at level 2.
constexpr uint32_t kBinPlainLevel = 2;

uint32_t log2_gamma(const hck_vital_plan *p) { return p->gamma == 4 ? 2 : 1; }

// K4's mask exponent P_phi (0 means 2) and the levels its powers of p take
// beyond P_phi = 2: p^3 and p^4 one more, p^5 two more
uint32_t phase_power(const hck_vital_plan *p) { return p->phase_power ? p->phase_power : 2; }
uint32_t phase_extra(const hck_vital_plan *p) {
  const uint32_t e = phase_power(p);
  return e == 2 ? 0 : e == 5 ? 2 : 1;
}

uint32_t pow2_at_least(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p *= 2;
  return p;
}

// The DFT bins of the two bands sit in two lane groups of `group` lanes of
// every frame's R slots: respiration from lane 0, heart rate from lane group.
// Each band's phase is copied into the first copies_* lanes.
struct Lanes {
  uint32_t group, copies_resp, copies_hr;
};

Lanes lanes_of(const hck_vital_plan *p) {
  const uint32_t g = pow2_at_least(std::max(p->lanes_resp, p->lanes_hr));
  return {g, pow2_at_least(p->lanes_resp), pow2_at_least(g + p->lanes_hr)};
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
  if (p->lanes_resp == 0 || p->lanes_hr == 0 || p->lanes_resp > p->bins ||
      p->lanes_hr > p->bins || 2 * lanes_of(p).group > p->bins)
    return set_error(HCK_EINVAL, "the two DFT lane groups do not fit the range bins");
  if (!p->bin_index || !p->bin_mask || !p->fir_resp || !p->fir_hr || !p->dft_re_resp ||
      !p->dft_im_resp || !p->dft_re_hr || !p->dft_im_hr || !p->freq || !p->mask ||
      (p->taylor_order == 3 && !p->third))
    return set_error(HCK_EINVAL, "missing plan operand");
  if (p->gamma != 0 && p->gamma != 2 && p->gamma != 4)
    return set_error(HCK_EINVAL, "gamma must be 2 or 4");
  if (p->phase_power != 0 && (p->phase_power < 2 || p->phase_power > 5))
    return set_error(HCK_EINVAL, "phase mask exponent must be 2 .. 5");
  if (p->mag_degree > 15 || (p->mag_degree && !p->mag_coeffs))
    return set_error(HCK_EINVAL, "magnitude polynomial: degree 0 .. 15 with coefficients");
  return HCK_OK;
}

std::vector<int32_t> plan_steps(const hck_vital_plan *p) {
  std::vector<int32_t> s;
  const uint32_t r = p->bins, t2 = pow2_at_least(p->frames);
  for (uint32_t k = r; k < r * t2; k *= 2) s.push_back((int32_t)k);
  for (uint32_t k = 1; k < r; k *= 2) s.push_back((int32_t)k);
  s.push_back(-(int32_t)r);
  for (uint32_t k = 1; k < lanes_of(p).copies_hr; k *= 2) s.push_back(-(int32_t)k);
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

// the per-frame packing's steps: the plan's and -R, -2R, ..., -(T2/2) R,
// which move every frame's I and Q to slot t R
std::vector<int32_t> frame_steps(const hck_vital_plan *p) {
  std::vector<int32_t> s = plan_steps(p);
  for (uint32_t k = p->bins; k < (uint64_t)p->bins * pow2_at_least(p->frames); k *= 2)
    s.push_back(-(int32_t)k);
  std::sort(s.begin(), s.end());
  s.erase(std::unique(s.begin(), s.end()), s.end());
  return s;
}

// Window k of a batch rotates with gks[k] and relinearizes with rlk[k] (the
// windows may belong to different tenants).  A batch's members are listed
// with the window each belongs to.
struct WindowKeys {
  const hck_galois_keys *const *gks;
  const hck_switch_key *const *rlk;
};

// member i belongs to window i / per
std::vector<uint32_t> owners(size_t members, uint32_t per) {
  std::vector<uint32_t> w(members);
  for (size_t i = 0; i < members; i++) w[i] = (uint32_t)(i / per);
  return w;
}

// dst[i] = Rot(src[i], step), every member with its window's key, key-switched
// together
int rotate_members(hck_context *ctx, const std::vector<hck_ciphertext *> &src,
                   const std::vector<uint32_t> &win, int32_t step, const WindowKeys &wk,
                   const std::vector<hck_ciphertext *> &dst) {
  const uint32_t g = galois_of_step(ctx, step);
  std::vector<uint32_t> gs(src.size(), g);
  std::vector<const hck_switch_key *> keys(src.size());
  for (size_t i = 0; i < src.size(); i++) {
    auto it = wk.gks[win[i]]->keys.find(g);
    if (it == wk.gks[win[i]]->keys.end())
      return set_error(HCK_ENOKEY, "missing Galois key for step " + std::to_string(step));
    keys[i] = it->second;
  }
  return apply_galois_keys(ctx, src.data(), gs.data(), keys.data(), (uint32_t)src.size(),
                           dst.data());
}

// c_i <- c_i + Rot(c_i, step) + ... over `count` (a power of two) shifts, for
// every member at once
int rotsum(hck_context *ctx, const std::vector<hck_ciphertext *> &cs,
           const std::vector<uint32_t> &win, int32_t step, uint32_t count, const WindowKeys &wk,
           Scratch &sc) {
  std::vector<hck_ciphertext *> tmp;
  for (size_t i = 0; i < cs.size(); i++) tmp.push_back(sc.get());
  for (uint64_t s = (uint64_t)step; s < (uint64_t)step * count; s *= 2) {
    TRY(rotate_members(ctx, cs, win, (int32_t)s, wk, tmp));
    for (size_t i = 0; i < cs.size(); i++) TRY(hck_add(ctx, cs[i], tmp[i], cs[i]));
  }
  return HCK_OK;
}

// outs[i] = relin(ts[i]) rescaled, the relinearizations key-switched together
int relin_rs(hck_context *ctx, const std::vector<hck_ciphertext *> &ts,
             const std::vector<uint32_t> &win, const WindowKeys &wk,
             const std::vector<hck_ciphertext *> &outs) {
  std::vector<const hck_switch_key *> keys(ts.size());
  for (size_t i = 0; i < ts.size(); i++) keys[i] = wk.rlk[win[i]];
  TRY(relinearize_keys(ctx, ts.data(), keys.data(), (uint32_t)ts.size(), outs.data()));
  for (hck_ciphertext *o : outs) TRY(hck_rescale(ctx, o, o));
  return HCK_OK;
}

// outs[i] = ins[i]^(2^times) by repeated squaring, every square relinearized
// (key-switched together) and rescaled
int square_rs(hck_context *ctx, const std::vector<hck_ciphertext *> &ins, uint32_t times,
              const std::vector<uint32_t> &win, const WindowKeys &wk,
              const std::vector<hck_ciphertext *> &outs, Scratch &sc) {
  std::vector<hck_ciphertext *> cur = ins;
  for (uint32_t r = 0; r < times; r++) {
    std::vector<hck_ciphertext *> ts, dst = r + 1 == times ? outs : std::vector<hck_ciphertext *>();
    for (size_t i = 0; i < cur.size(); i++) {
      hck_ciphertext *t = sc.get();
      TRY(hck_mul(ctx, cur[i], cur[i], t));
      ts.push_back(t);
      if (r + 1 < times) dst.push_back(sc.get());
    }
    TRY(relin_rs(ctx, ts, win, wk, dst));
    cur = dst;
  }
  return HCK_OK;
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

}  // extern "C"

// The pipeline over n windows at once: every stage advances all windows, so
// their rotate-and-sum chains and relinearizations share key-switch batches.
// taps (optional, HCK_VITAL_TAPS per window, entries may be null) receive
// copies of the kernels' intermediate results.
// frames of the per-frame packing whose K1 and K4 run together (a power of
// two, so that the frame tree's levels inside a block are its first levels)
constexpr uint32_t kFrameBlock = 16;

// K1 and K4 on units (windows, or frames of one window) u < uw.size(), unit
// u belonging to window uw[u]: pw[u] = Re^2 + Im^2; en[u] = its copy for the
// bin branch (the power, or the polynomial magnitude) at bin_level; iq[2u],
// iq[2u + 1] = I and Q (mask p^P_phi times Re, Im, summed over the R bins
// into each frame's first slot).  Intermediates come from sc.
static int front_units(hck_context *ctx, const hck_vital_plan *p,
                       const hck_ciphertext *const *re, const hck_ciphertext *const *im,
                       const std::vector<uint32_t> &uw, const WindowKeys &wk, uint32_t bin_level,
                       Scratch &sc, std::vector<hck_ciphertext *> &pw,
                       std::vector<hck_ciphertext *> &en, std::vector<hck_ciphertext *> &iq) {
  const uint32_t U = (uint32_t)uw.size();
  auto fresh = [&](uint32_t count) {
    std::vector<hck_ciphertext *> v(count);
    for (auto &c : v) c = sc.get();
    return v;
  };
  std::vector<uint32_t> uw2(2 * U);
  for (uint32_t u = 0; u < U; u++) uw2[2 * u] = uw2[2 * u + 1] = uw[u];
  // K1: p = Re^2 + Im^2 (one batched relinearization)
  pw = fresh(U);
  en = fresh(U);
  std::vector<hck_ciphertext *> ts;
  for (uint32_t u = 0; u < U; u++) {
    hck_ciphertext *t = sc.get(), *v = sc.get();
    TRY(hck_mul(ctx, re[u], re[u], t));
    TRY(hck_mul(ctx, im[u], im[u], v));
    TRY(hck_add(ctx, t, v, t));
    ts.push_back(t);
  }
  TRY(relin_rs(ctx, ts, uw, wk, pw));
  for (uint32_t u = 0; u < U; u++) {
    if (p->mag_degree) {  // the polynomial magnitude ~ |z| instead of the power
      hck_ciphertext *mg = sc.get();
      TRY(hck_poly_eval(ctx, pw[u], p->mag_coeffs, p->mag_degree, wk.rlk[uw[u]], mg));
      TRY(hck_drop_level(ctx, mg, bin_level, en[u]));
    } else {
      TRY(hck_drop_level(ctx, pw[u], bin_level, en[u]));
    }
  }
  // K4's mask m = p^P_phi: p^2, then p^3 = p^2 p, p^4 = (p^2)^2 or
  // p^5 = (p^2)^2 p, every product relinearized and rescaled
  const uint32_t pe = phase_power(p);
  std::vector<hck_ciphertext *> m = fresh(U);
  TRY(square_rs(ctx, pw, 1, uw, wk, m, sc));
  if (pe >= 4) {
    std::vector<hck_ciphertext *> p4 = fresh(U);
    TRY(square_rs(ctx, m, 1, uw, wk, p4, sc));
    m = p4;
  }
  if (pe == 3 || pe == 5) {  // times p (dropped to the power's level)
    std::vector<hck_ciphertext *> tm, mo = fresh(U);
    for (uint32_t u = 0; u < U; u++) {
      hck_ciphertext *pl = sc.get(), *tp = sc.get();
      TRY(hck_drop_level(ctx, pw[u], m[u]->level, pl));
      TRY(hck_mul(ctx, m[u], pl, tp));
      tm.push_back(tp);
    }
    TRY(relin_rs(ctx, tm, uw, wk, mo));
    m = mo;
  }
  // I and Q: the mask times Re and Im (one batched relinearization), summed
  // over the range bins by rotations 1 .. R/2
  iq = fresh(2 * U);
  ts.clear();
  for (uint32_t u = 0; u < U; u++) {
    hck_ciphertext *re2 = sc.get(), *im2 = sc.get(), *ti = sc.get(), *tq = sc.get();
    TRY(hck_drop_level(ctx, re[u], m[u]->level, re2));
    TRY(hck_drop_level(ctx, im[u], m[u]->level, im2));
    TRY(hck_mul(ctx, m[u], re2, ti));
    TRY(hck_mul(ctx, m[u], im2, tq));
    ts.insert(ts.end(), {ti, tq});
  }
  TRY(relin_rs(ctx, ts, uw2, wk, iq));
  return rotsum(ctx, iq, uw2, 1, p->bins, wk, sc);
}

// Levels of the frame tree over the list cur = (I_0, Q_0, I_1, Q_1, ...) of
// one window: at each level every other entry, rotated by -shift, is added
// to its left neighbour, and shift doubles; cur ends as (I, Q).
static int frame_tree(hck_context *ctx, std::vector<hck_ciphertext *> &cur, int32_t shift,
                      const WindowKeys &wk, Scratch &sc) {
  for (; cur.size() > 2; shift *= 2) {
    std::vector<hck_ciphertext *> src, nxt;
    for (size_t i = 2; i + 1 < cur.size(); i += 4) src.insert(src.end(), {cur[i], cur[i + 1]});
    std::vector<hck_ciphertext *> rot(src.size());
    for (auto &c : rot) c = sc.get();
    TRY(rotate_members(ctx, src, std::vector<uint32_t>(src.size(), 0), -shift, wk, rot));
    for (size_t i = 0; i < cur.size(); i += 4) {
      if (i + 2 < cur.size()) {
        TRY(hck_add(ctx, cur[i], rot[i / 2], cur[i]));
        TRY(hck_add(ctx, cur[i + 1], rot[i / 2 + 1], cur[i + 1]));
      }
      nxt.insert(nxt.end(), {cur[i], cur[i + 1]});
    }
    cur = nxt;
  }
  return HCK_OK;
}

// frames > 0: per-frame packing (section 3.3.2) of one window (n = 1):
// re[t], im[t] (t < frames) hold frame t's R range bins in slots 0 .. R-1.
static int vital_eval_windows(hck_context *ctx, const hck_vital_plan *p,
                              const hck_ciphertext *const *re, const hck_ciphertext *const *im,
                              uint32_t n, const WindowKeys &wk, hck_ciphertext *const *out,
                              hck_ciphertext *const *taps, uint32_t frames = 0) {
  TRY(check_plan(ctx, p));
  const uint32_t sq = log2_gamma(p);  // squarings of each K2 stage
  const uint32_t extra = phase_extra(p);  // levels of p^P_phi beyond p^2
  const uint32_t depth = (p->taylor_order == 3 ? 11 : 9) + sq - 1 + extra;
  const uint32_t bin_level = kBinPlainLevel + sq;
  // the plan's operands are encoded for inputs at level l0 (the FIR
  // transforms at l0 - 3 - extra, the bin branch's plaintexts at level 2);
  // inputs above l0 are dropped to it, since the circuit uses only its first
  // depth + 1 primes anyway
  const uint32_t l0 = p->fir_resp->level + 3 + extra;
  if (l0 < depth || l0 >= ctx->L)
    return set_error(HCK_ELEVEL, "plan encoded below the pipeline depth");
  if (p->bin_index->level != kBinPlainLevel || p->bin_mask->level != kBinPlainLevel)
    return set_error(HCK_ELEVEL, "bin plaintexts must be encoded at level 2");
  if (frames && (n != 1 || frames != p->frames))
    return set_error(HCK_EINVAL, "per-frame packing: one window of the plan's frame count");
  const uint32_t n_in = frames ? frames : n;
  for (uint32_t k = 0; k < n_in; k++) {
    if (!re[k] || !im[k]) return set_error(HCK_EINVAL, "null input");
    if (re[k]->level != re[0]->level || im[k]->level != re[0]->level || re[0]->level < l0)
      return set_error(HCK_ELEVEL, "inputs must share a level of at least the plan's level");
  }
  for (uint32_t k = 0; k < n; k++) {
    if (!wk.gks[k] || !wk.rlk[k]) return set_error(HCK_EINVAL, "null key");
    for (int i = 0; i < 4; i++)
      if (!out[4 * k + i]) return set_error(HCK_EINVAL, "null output");
  }
  for (int32_t s : frames ? frame_steps(p) : plan_steps(p))
    for (uint32_t k = 0; k < n; k++)
      if (!wk.gks[k]->keys.count(galois_of_step(ctx, s)))
        return set_error(HCK_ENOKEY, "missing Galois key for step " + std::to_string(s));
  Scratch sc(ctx);
  const std::vector<uint32_t> one = owners(n, 1), two = owners(2 * n, 2),
                              four = owners(4 * n, 4);
  const int32_t r = (int32_t)p->bins;
  const uint32_t t2 = pow2_at_least(p->frames);
  const Lanes lanes = lanes_of(p);
  auto fresh = [&](uint32_t count) {
    std::vector<hck_ciphertext *> v(count);
    for (auto &c : v) c = sc.get();
    return v;
  };
  std::vector<const hck_ciphertext *> in_re(re, re + n_in), in_im(im, im + n_in);
  if (re[0]->level > l0)
    for (uint32_t k = 0; k < n_in; k++) {
      hck_ciphertext *a = sc.get(), *b = sc.get();
      TRY(hck_drop_level(ctx, re[k], l0, a));
      TRY(hck_drop_level(ctx, im[k], l0, b));
      in_re[k] = a;
      in_im[k] = b;
    }
  re = in_re.data();
  im = in_im.data();
  auto O = [&](uint32_t k, int i) { return out[4 * k + i]; };
  auto tap = [&](uint32_t k, int i, const hck_ciphertext *c) {
    hck_ciphertext *t = taps ? taps[HCK_VITAL_TAPS * k + i] : nullptr;
    return t ? hck_drop_level(ctx, c, c->level, t) : HCK_OK;
  };

  // K1 and K4, then K2 over bins, on the windows (batched packing: every
  // frame of a window in one ciphertext pair) or on the frames of the one
  // window (per-frame packing), which run in aligned blocks of kFrameBlock
  // frames so that only one block's intermediates are held at a time
  std::vector<hck_ciphertext *> pw, e = fresh(n), it(n), qt(n);
  if (!frames) {
    std::vector<hck_ciphertext *> en, iq;
    TRY(front_units(ctx, p, re, im, one, wk, bin_level, sc, pw, en, iq));
    for (uint32_t k = 0; k < n; k++) {
      TRY(hck_drop_level(ctx, en[k], en[k]->level, e[k]));
      it[k] = iq[2 * k];
      qt[k] = iq[2 * k + 1];
    }
    TRY(rotsum(ctx, e, one, r, t2, wk, sc));
  } else {
    // entries of the frame tree that holds every frame's I and Q at slot t R
    std::vector<hck_ciphertext *> tree;
    for (uint32_t b0 = 0; b0 < frames; b0 += kFrameBlock) {
      const uint32_t nb = std::min(kFrameBlock, frames - b0);
      Scratch blk(ctx);
      std::vector<hck_ciphertext *> bpw, en, iq;
      TRY(front_units(ctx, p, re + b0, im + b0, std::vector<uint32_t>(nb, 0), wk, bin_level, blk,
                      bpw, en, iq));
      // E: the frames' energy copies added in frame order
      for (uint32_t t = 0; t < nb; t++)
        TRY(b0 + t == 0 ? hck_drop_level(ctx, en[t], en[t]->level, e[0])
                        : hck_add(ctx, e[0], en[t], e[0]));
      // the tree's levels inside the block; its one entry survives the block
      TRY(frame_tree(ctx, iq, (int32_t)r, wk, blk));
      hck_ciphertext *bi = sc.get(), *bq = sc.get();
      TRY(hck_drop_level(ctx, iq[0], iq[0]->level, bi));
      TRY(hck_drop_level(ctx, iq[1], iq[1]->level, bq));
      tree.insert(tree.end(), {bi, bq});
    }
    TRY(frame_tree(ctx, tree, (int32_t)(r * kFrameBlock), wk, sc));
    it[0] = tree[0];
    qt[0] = tree[1];
  }
  for (uint32_t k = 0; k < n; k++) {
    if (!frames) TRY(tap(k, 0, pw[k]));
    TRY(tap(k, 1, e[k]));
  }
  // K2 over bins: w = E^gamma by squarings on the bin branch's level
  std::vector<hck_ciphertext *> w = fresh(n), ts, outs;
  TRY(square_rs(ctx, e, sq, one, wk, w, sc));
  for (uint32_t k = 0; k < n; k++) TRY(tap(k, 2, w[k]));
  {
    std::vector<hck_ciphertext *> bins;
    for (uint32_t k = 0; k < n; k++) {
      TRY(mulpt_rs(ctx, w[k], p->bin_index, O(k, 0)));
      TRY(mulpt_rs(ctx, w[k], p->bin_mask, O(k, 1)));
      bins.insert(bins.end(), {O(k, 0), O(k, 1)});
    }
    TRY(rotsum(ctx, bins, two, 1, (uint32_t)r, wk, sc));
  }
  for (uint32_t k = 0; k < n; k++) {
    TRY(tap(k, 3, it[k]));
    TRY(tap(k, 4, qt[k]));
  }
  // K5: both bands' FIR of I and Q, one BSGS evaluation per window
  std::vector<hck_ciphertext *> f = fresh(4 * n);
  for (uint32_t k = 0; k < n; k++) {
    const hck_ciphertext *ins[2] = {it[k], qt[k]};
    const hck_linear_transform *lts[4] = {p->fir_resp, p->fir_resp, p->fir_hr, p->fir_hr};
    const uint32_t tin[4] = {0, 1, 0, 1}, tout[4] = {0, 1, 2, 3};
    TRY(hck_lt_eval(ctx, ins, 2, lts, tin, tout, nullptr, 4, wk.gks[k], &f[4 * k], 4,
                    HCK_LT_HOIST_BABY | HCK_LT_HOIST_GIANT));
    for (int i = 0; i < 4; i++) {
      TRY(hck_rescale(ctx, f[4 * k + i], f[4 * k + i]));
      TRY(tap(k, 5 + i, f[4 * k + i]));
    }
  }
  // K7: the previous frame by a rotation of -R; both bands of every window
  // advance together, one batched relinearization per product level
  std::vector<hck_ciphertext *> f1 = fresh(4 * n);
  TRY(rotate_members(ctx, f, four, -r, wk, f1));
  std::vector<hck_ciphertext *> dphi = fresh(2 * n), y = fresh(2 * n), x = fresh(2 * n);
  ts.clear();
  outs.clear();
  for (uint32_t j = 0; j < 2 * n; j++) {
    hck_ciphertext *fi = f[2 * j], *fq = f[2 * j + 1], *fi1 = f1[2 * j], *fq1 = f1[2 * j + 1];
    hck_ciphertext *t1 = sc.get(), *t2 = sc.get();
    TRY(hck_mul(ctx, fq, fi1, t1));
    TRY(hck_mul(ctx, fi, fq1, t2));
    TRY(hck_sub(ctx, t1, t2, t1));
    ts.push_back(t1);
    outs.push_back(y[j]);
    if (p->taylor_order == 3) {
      hck_ciphertext *u1 = sc.get(), *u2 = sc.get();
      TRY(hck_mul(ctx, fi, fi1, u1));
      TRY(hck_mul(ctx, fq, fq1, u2));
      TRY(hck_add(ctx, u1, u2, u1));
      ts.push_back(u1);
      outs.push_back(x[j]);
    }
  }
  TRY(relin_rs(ctx, ts, owners(ts.size(), (uint32_t)(ts.size() / n)), wk, outs));
  if (p->taylor_order == 1) {
    for (uint32_t j = 0; j < 2 * n; j++) TRY(hck_drop_level(ctx, y[j], y[j]->level, dphi[j]));
  } else {
    // x^2 and y^2 (one batch), then y x^2 and (y / 3) y^2 (one batch)
    std::vector<hck_ciphertext *> x2 = fresh(2 * n), y2 = fresh(2 * n);
    ts.clear();
    outs.clear();
    for (uint32_t j = 0; j < 2 * n; j++) {
      hck_ciphertext *t1 = sc.get(), *t2 = sc.get();
      TRY(hck_mul(ctx, x[j], x[j], t1));
      TRY(hck_mul(ctx, y[j], y[j], t2));
      ts.insert(ts.end(), {t1, t2});
      outs.insert(outs.end(), {x2[j], y2[j]});
    }
    TRY(relin_rs(ctx, ts, owners(ts.size(), (uint32_t)(ts.size() / n)), wk, outs));
    std::vector<hck_ciphertext *> av = fresh(2 * n), bv = fresh(2 * n);
    ts.clear();
    outs.clear();
    for (uint32_t j = 0; j < 2 * n; j++) {
      hck_ciphertext *y6 = sc.get(), *yc = sc.get(), *t1 = sc.get(), *t2 = sc.get();
      TRY(hck_drop_level(ctx, y[j], x2[j]->level, y6));
      TRY(mulpt_rs(ctx, y[j], p->third, yc));
      TRY(hck_mul(ctx, y6, x2[j], t1));
      TRY(hck_mul(ctx, yc, y2[j], t2));
      ts.insert(ts.end(), {t1, t2});
      outs.insert(outs.end(), {av[j], bv[j]});
    }
    TRY(relin_rs(ctx, ts, owners(ts.size(), (uint32_t)(ts.size() / n)), wk, outs));
    for (uint32_t j = 0; j < 2 * n; j++) TRY(hck_sub(ctx, av[j], bv[j], dphi[j]));
  }
  for (uint32_t k = 0; k < n; k++) {
    TRY(tap(k, 9, dphi[2 * k]));
    TRY(tap(k, 10, dphi[2 * k + 1]));
  }
  // K3: copy each dphi into its band's lanes (dphi[2k]: respiration,
  // dphi[2k + 1]: heart rate), weight; the bands' products are added (disjoint
  // lanes) so that one sum over frames serves both
  for (uint32_t s = 1; s < lanes.copies_hr; s *= 2) {
    std::vector<hck_ciphertext *> src;
    std::vector<uint32_t> win;
    for (uint32_t k = 0; k < n; k++) {
      src.push_back(dphi[2 * k + 1]);
      win.push_back(k);
      if (s < lanes.copies_resp) {
        src.push_back(dphi[2 * k]);
        win.push_back(k);
      }
    }
    std::vector<hck_ciphertext *> tmp = fresh((uint32_t)src.size());
    TRY(rotate_members(ctx, src, win, -(int32_t)s, wk, tmp));
    for (size_t i = 0; i < src.size(); i++) TRY(hck_add(ctx, src[i], tmp[i], src[i]));
  }
  std::vector<hck_ciphertext *> xs = fresh(2 * n);
  for (uint32_t k = 0; k < n; k++) {
    hck_ciphertext *hr_re = sc.get(), *hr_im = sc.get();
    TRY(mulpt_rs(ctx, dphi[2 * k], p->dft_re_resp, xs[2 * k]));
    TRY(mulpt_rs(ctx, dphi[2 * k + 1], p->dft_re_hr, hr_re));
    TRY(hck_add(ctx, xs[2 * k], hr_re, xs[2 * k]));
    TRY(mulpt_rs(ctx, dphi[2 * k], p->dft_im_resp, xs[2 * k + 1]));
    TRY(mulpt_rs(ctx, dphi[2 * k + 1], p->dft_im_hr, hr_im));
    TRY(hck_add(ctx, xs[2 * k + 1], hr_im, xs[2 * k + 1]));
  }
  TRY(rotsum(ctx, xs, two, r, t2, wk, sc));
  for (uint32_t k = 0; k < n; k++) {
    TRY(tap(k, 11, xs[2 * k]));
    TRY(tap(k, 12, xs[2 * k + 1]));
  }
  // K1 on the spectrum, K2: sharpening and the weighted frequency averages of
  // both lane groups (respiration in slot 0, heart rate in slot `group`)
  std::vector<hck_ciphertext *> pspec = fresh(n), sh = fresh(n);
  ts.clear();
  for (uint32_t k = 0; k < n; k++) {
    hck_ciphertext *sq_re = sc.get(), *sq_im = sc.get();
    TRY(hck_mul(ctx, xs[2 * k], xs[2 * k], sq_re));
    TRY(hck_mul(ctx, xs[2 * k + 1], xs[2 * k + 1], sq_im));
    TRY(hck_add(ctx, sq_re, sq_im, sq_re));
    ts.push_back(sq_re);
  }
  TRY(relin_rs(ctx, ts, one, wk, pspec));
  for (uint32_t k = 0; k < n; k++) TRY(tap(k, 13, pspec[k]));
  TRY(square_rs(ctx, pspec, sq, one, wk, sh, sc));
  for (uint32_t k = 0; k < n; k++) TRY(tap(k, 14, sh[k]));
  std::vector<hck_ciphertext *> chain;
  for (uint32_t k = 0; k < n; k++) {
    TRY(mulpt_rs(ctx, sh[k], p->freq, O(k, 2)));
    TRY(mulpt_rs(ctx, sh[k], p->mask, O(k, 3)));
    chain.insert(chain.end(), {O(k, 2), O(k, 3)});
  }
  return rotsum(ctx, chain, two, 1, lanes.group, wk, sc);
}

namespace hck {

int vital_eval_batch(hck_context *ctx, const hck_vital_plan *p, const hck_ciphertext *const *re,
                     const hck_ciphertext *const *im, uint32_t n,
                     const hck_galois_keys *const *gks, const hck_switch_key *const *rlk,
                     hck_ciphertext *const *out) {
  if (n == 0) return HCK_OK;
  return vital_eval_windows(ctx, p, re, im, n, WindowKeys{gks, rlk}, out, nullptr);
}

}  // namespace hck

// outputs and taps must not alias an input, and all belong to the context
static int check_aliases(const hck_context *ctx, const hck_ciphertext *const *re,
                         const hck_ciphertext *const *im, uint32_t n, hck_ciphertext *const *out,
                         uint32_t n_out) {
  for (uint32_t k = 0; k < n; k++)
    if (foreign(ctx, re[k]) || foreign(ctx, im[k]))
      return set_error(HCK_EINVAL, "handle of another (or a destroyed) context");
  for (uint32_t i = 0; i < n_out; i++) {
    if (foreign(ctx, out[i]))
      return set_error(HCK_EINVAL, "handle of another (or a destroyed) context");
    for (uint32_t k = 0; k < n; k++)
      if (out[i] && (out[i] == re[k] || out[i] == im[k]))
        return set_error(HCK_EINVAL, "outputs must not alias inputs");
  }
  return HCK_OK;
}

extern "C" {

int hck_vital_eval(hck_context *ctx, const hck_vital_plan *p, const hck_ciphertext *re,
                   const hck_ciphertext *im, const hck_galois_keys *gks,
                   const hck_switch_key *rlk, hck_ciphertext *const *out) {
  return hck_vital_eval_taps(ctx, p, re, im, gks, rlk, out, nullptr);
}

int hck_vital_eval_taps(hck_context *ctx, const hck_vital_plan *p, const hck_ciphertext *re,
                        const hck_ciphertext *im, const hck_galois_keys *gks,
                        const hck_switch_key *rlk, hck_ciphertext *const *out,
                        hck_ciphertext *const *taps) {
  if (!ctx || !re || !im || !gks || !rlk || !out) return set_error(HCK_EINVAL, "null argument");
  if (foreign(ctx, gks) || foreign(ctx, rlk))
    return set_error(HCK_EINVAL, "handle of another (or a destroyed) context");
  TRY(check_aliases(ctx, &re, &im, 1, out, 4));
  if (taps) TRY(check_aliases(ctx, &re, &im, 1, taps, HCK_VITAL_TAPS));
  return vital_eval_windows(ctx, p, &re, &im, 1, WindowKeys{&gks, &rlk}, out, taps);
}

int hck_vital_frames_required_steps(const hck_context *ctx, const hck_vital_plan *plan,
                                    int32_t *steps, uint32_t cap, uint32_t *n) {
  if (!ctx || !n) return set_error(HCK_EINVAL, "null argument");
  TRY(check_plan(ctx, plan));
  const std::vector<int32_t> s = frame_steps(plan);
  *n = (uint32_t)s.size();
  if (steps) {
    if (cap < s.size()) return set_error(HCK_EINVAL, "steps buffer too small");
    std::copy(s.begin(), s.end(), steps);
  }
  return HCK_OK;
}

int hck_vital_eval_frames(hck_context *ctx, const hck_vital_plan *p,
                          const hck_ciphertext *const *re, const hck_ciphertext *const *im,
                          uint32_t frames, const hck_galois_keys *gks, const hck_switch_key *rlk,
                          hck_ciphertext *const *out) {
  if (!ctx || !re || !im || !gks || !rlk || !out || frames == 0)
    return set_error(HCK_EINVAL, "null argument");
  if (foreign(ctx, gks) || foreign(ctx, rlk))
    return set_error(HCK_EINVAL, "handle of another (or a destroyed) context");
  TRY(check_aliases(ctx, re, im, frames, out, 4));
  return vital_eval_windows(ctx, p, re, im, 1, WindowKeys{&gks, &rlk}, out, nullptr, frames);
}

int hck_vital_eval_many(hck_context *ctx, const hck_vital_plan *p,
                        const hck_ciphertext *const *re, const hck_ciphertext *const *im,
                        uint32_t n, const hck_galois_keys *gks, const hck_switch_key *rlk,
                        hck_ciphertext *const *out) {
  if (!ctx || !gks || !rlk || (n && (!re || !im || !out)))
    return set_error(HCK_EINVAL, "null argument");
  if (n == 0) return HCK_OK;
  if (foreign(ctx, gks) || foreign(ctx, rlk))
    return set_error(HCK_EINVAL, "handle of another (or a destroyed) context");
  TRY(check_aliases(ctx, re, im, n, out, 4 * n));
  std::vector<const hck_galois_keys *> g(n, gks);
  std::vector<const hck_switch_key *> rl(n, rlk);
  return vital_eval_windows(ctx, p, re, im, n, WindowKeys{g.data(), rl.data()}, out, nullptr);
}

}  // extern "C"
