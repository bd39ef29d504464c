// Internal declarations of the hipckks library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "hipckks.h"
#include "modarith.h"

namespace hck {

constexpr int kMaxLimbs = HCK_MAX_LIMBS;
constexpr int kMaxRows = 256;  // rows of one batched launch (e.g. every extended digit)
constexpr int kMaxBatch = 32;  // key switches run together in one sequence of launches

// Per-modulus constants, indexed by the modulus index of the full chain
// (0..L-1: q chain, L..L+K-1: special primes).
struct ModConst {
  uint64_t q;
  uint64_t qinv;        // q^-1 mod 2^64 (Montgomery)
  uint64_t r64;         // 2^64 mod q (into Montgomery form, Shoup constant)
  uint64_t r64_shoup;
  uint64_t ninv;        // N^-1 mod q
  uint64_t ninv_shoup;
  uint64_t r2;          // 2^128 mod q (Montgomery fix-up of a plain product)
  uint64_t one_shoup;   // floor(2^64 / q): Shoup companion of 1 (reduction of any word)
  uint64_t nq;          // 2^64 - q
};

// Which rows of a [row][N] buffer a launch processes (blockIdx.y indexes the
// list) and the modulus index of each row.  Passed by value as a kernel
// argument.
struct LimbMap {
  uint32_t n;
  uint16_t row[kMaxRows];
  uint8_t mod[kMaxRows];
};

// Per-row Shoup multiplier and additive constant applied at the end of an
// inverse NTT (x -> x w + a mod q); indexed like LimbMap rows (list index).
struct RowScale {
  uint64_t w[kMaxLimbs];
  uint64_t wp[kMaxLimbs];
  uint64_t add[kMaxLimbs];
};

}  // namespace hck

struct hck_context {
  int device = 0;
  hipStream_t stream = nullptr;
  uint32_t log_n = 0, n = 0, L = 0, K = 0, dnum = 0, alpha = 0;
  std::vector<uint64_t> mods;  // L + K primes: q chain then special primes

  // device tables
  hck::ModConst *d_mod = nullptr;    // [L+K]
  uint64_t *d_tw = nullptr;          // [L+K][N] psi^brv(k)
  uint64_t *d_tw_shoup = nullptr;
  uint64_t *d_itw = nullptr;         // [L+K][N] psi^-brv(k)
  uint64_t *d_itw_shoup = nullptr;
  uint64_t *d_ttw = nullptr;         // [L+K][N] contiguous-pass twist beta_g^i (ntt_core.h)
  uint64_t *d_ttw_shoup = nullptr;
  uint64_t *d_ittw = nullptr;        // [L+K][N] inverse twist beta_g^-i
  uint64_t *d_ittw_shoup = nullptr;
  // basis conversion matrices (Montgomery form, per (level, digit) or ModDown)
  uint64_t *d_up_conv = nullptr;     // [L][dnum][alpha][L+K]
  uint64_t *d_down_conv = nullptr;   // [K][L+K] (columns < L used)
  uint64_t *d_down_hneg = nullptr;   // [L]: -(P-1)/2 mod q_i

  // host copies of per-row scale factors
  // up_scale[level][i]: N^-1 (Q'_j / q_i)^-1 mod q_i, digit j of limb i at that level
  std::vector<std::vector<uint64_t>> up_scale;
  std::vector<uint64_t> down_scale;   // [K]: N^-1 (P/p_k)^-1 mod p_k
  std::vector<uint64_t> down_add;     // [K]: ((P-1)/2 mod p_k) (P/p_k)^-1 mod p_k
  std::vector<uint64_t> down_hneg;    // [L]: -(P-1)/2 mod q_i
  std::vector<uint64_t> pinv;         // [L]: P^-1 mod q_i
  std::vector<std::vector<uint64_t>> rescale_inv;  // [l][i<l]: q_l^-1 mod q_i

  // key-switch workspace (device)
  uint64_t *ws = nullptr;
  size_t ws_words = 0;
  uint64_t *lt_scratch = nullptr;   // inner sums of the linear-transform evaluator
  size_t lt_scratch_words = 0;
  uint64_t *zero_rows = nullptr;    // [L][N] zeros (absent diagonals of the BSGS grid)
  // scratch ciphertexts reused by linear transforms
  std::vector<struct hck_ciphertext *> ct_pool;
  // device allocator: the caller's hook (hck_set_allocator) or, when unset,
  // stream-ordered hipMallocAsync / hipFreeAsync; live_allocs counts the
  // buffers dev_alloc handed out and dev_free has not yet returned
  // split of the plain full NTTs (log2 of the strided radix R1; 0: the
  // default (log N + 1) / 2), chosen by hck_autotune_ntt; alt_twist[0] and
  // [1] are the contiguous pass's twist tables (forward, its Shoup
  // companions, inverse, its companions) of the splits one below and one
  // above the default, built when first chosen and kept until the context is
  // destroyed (recorded graphs may read them)
  uint8_t ntt_a = 0;
  // every modulus below 2^60: the basis conversions sum products of 30-bit
  // halves in carry-free 64-bit columns
  bool bconv30 = false;
  uint64_t *alt_twist[2][4] = {};
  uint64_t *def_twist[4] = {};
  // key switches per launch sequence at each level, chosen by the autotuner
  // (hck_autotune_keyswitch) or set by the caller; 0: the built-in rule
  uint8_t ks_cap[HCK_MAX_LIMBS] = {};
  void *(*alloc_fn)(size_t, void *, void *) = nullptr;
  void (*free_fn)(void *, void *, void *) = nullptr;
  void *alloc_user = nullptr;
  uint64_t live_allocs = 0;
  // Allocation sequence numbers, for the validity of captured graphs: a
  // graph may read any buffer allocated before its capture ended (sequence
  // below its mark) and none allocated later.  graph_mark is the highest mark
  // of the graphs captured so far; a buffer below it that is given back is
  // logged in freed_old, which hck_graph_launch checks.
  uint64_t alloc_counter = 0;
  std::unordered_map<void *, uint64_t> alloc_seq;
  uint64_t graph_mark = 0;
  std::vector<uint64_t> freed_old;
  // the context's stream is being captured into a HIP graph (hck_graph_begin):
  // allocation, host transfers and waits are refused until hck_graph_end
  bool capturing = false;

  bool broken = false;

  // Caller-owned objects made on this context and not yet destroyed, each
  // with the function that releases its device memory and detaches it
  // (sets its ctx to null).  hck_context_destroy releases servers first
  // (their workers use the context and the other handles), then every other
  // handle; a handle's own destroy call afterwards frees only its host
  // record.  So destroy calls may come in any order.
  std::unordered_map<void *, void (*)(void *)> handles;
  std::unordered_map<void *, void (*)(void *)> servers;

  // kernel timing
  bool timing = false;
  struct Timed {
    std::string name;
    hipEvent_t start, stop;
    double bytes, mulmods;
  };
  struct TimingTotal {
    double ms = 0, bytes = 0, mulmods = 0;
    uint64_t launches = 0;
  };
  std::vector<Timed> pending;
  std::vector<hipEvent_t> event_pool;
  std::map<std::string, TimingTotal> timing_total;

  // launch trace (hck_trace_*): every kernel launch and device allocation in
  // issue order, while `trace` is on
  bool trace = false;
  std::vector<hck_trace_record> trace_log;
};

namespace hck {
// one launch of the linear-transform inner sums (lt_kernels.hip)
constexpr int kLtLts = 2;    // distinct transforms per launch
constexpr int kLtIn = 4;     // inputs
constexpr int kLtOut = 4;    // outputs
constexpr int kLtB = 32;     // baby steps per launch
constexpr int kLtMaxG = 64;  // giant groups per evaluation
constexpr int kLtCoeffs = 64;  // coefficients per workgroup (one per lane)
struct LtSumArgs {
  uint32_t nb, ng, n_in, n_out, n_terms, max_terms, accumulate;
  size_t ps;                                 // polynomial stride of baby ciphertexts / sums
  const uint64_t *baby[kLtIn][kLtB];         // baby rotation (input, chunk baby) or null
  const uint64_t *grid[kLtLts];              // transform's diagonal grid [giant][baby][limb][N]
  uint32_t grid_nb[kLtLts];                  // babies of the transform's grid
  uint32_t grid_rows[kLtLts];                // limbs per diagonal (transform level + 1)
  int32_t gmap[kLtLts][kLtMaxG];             // evaluation giant -> transform giant, -1: none
  int32_t bmap[kLtLts][kLtB];                // chunk baby -> transform baby, -1: none
  uint32_t present[kLtLts][kLtMaxG];         // bit b: diagonal (giant, chunk baby b) exists
  uint64_t *sums;                            // [ng][n_out] ciphertexts of 2 polys (stride ps)
  const uint64_t *zero;                      // [L][N] zeros, read for absent diagonals
  // sign of the term (transform, input -> output), 0: no such term
  int8_t coef[kLtLts][kLtIn][kLtOut];
};
}  // namespace hck

struct hck_ciphertext {
  hck_context *ctx = nullptr;
  uint64_t *data = nullptr;  // [cap_polys][L][N], evaluation (NTT) domain, plain form
  uint32_t cap_polys = 0;
  // a scratch ciphertext of the context's pool: always allocated for 3
  // polynomials, so that a pool entry never grows in a later call whatever
  // role it takes (calls in graph capture cannot allocate)
  bool pooled = false;
  uint32_t size = 0;  // polynomials in use (0: empty)
  uint32_t level = 0;
  double scale = 1.0;
};

struct hck_plaintext {
  hck_context *ctx = nullptr;
  uint64_t *data = nullptr;  // [level+1][N], evaluation domain, Montgomery form
  uint32_t level = 0;
  double scale = 1.0;
};

struct hck_secret_key {
  hck_context *ctx = nullptr;
  std::vector<int8_t> coeffs;  // N ternary coefficients
  uint64_t *data = nullptr;    // [L+K][N] evaluation domain, Montgomery form
};

struct hck_public_key {
  hck_context *ctx = nullptr;
  uint64_t *data = nullptr;  // [2][L][N] evaluation domain, Montgomery form
};

struct hck_switch_key {
  hck_context *ctx = nullptr;
  uint64_t *data = nullptr;  // [dnum][2][L+K][N] evaluation domain, Montgomery form
};

struct hck_galois_keys {
  hck_context *ctx = nullptr;
  std::map<uint32_t, hck_switch_key *> keys;
};

struct hck_linear_transform {
  hck_context *ctx = nullptr;
  uint32_t n1 = 1, level = 0;
  double scale = 1.0;
  // giant index g -> list of (baby step b, diagonal plaintext [level+1][N])
  std::map<int32_t, std::vector<std::pair<int32_t, uint64_t *>>> groups;
  // the diagonals as one grid [giants][babies][level+1][N] (rows of absent
  // diagonals are zero); giants and babies ascending
  std::vector<int32_t> giants, babies;
  uint64_t *grid = nullptr;
  std::vector<uint64_t *> owned;
};

namespace hck {

// ---- error handling (errors.cpp) ----
int set_error(int code, const std::string &msg);
int check_hip(hck_context *ctx, hipError_t e, const char *what);
#define HCK_HIP(ctx, expr)                                          \
  do {                                                              \
    hipError_t _e = (expr);                                         \
    if (_e != hipSuccess) return ::hck::check_hip((ctx), _e, #expr); \
  } while (0)

// ---- contexts (context.cpp) ----
int build_context(const hck_params *prm, int device, void *stream, hck_context **out);
void destroy_context(hck_context *ctx);

// ---- graph capture (graph.cpp) ----
void abort_capture(hck_context *ctx);

// ---- ownership of caller handles (context.cpp) ----
void track(hck_context *ctx, void *obj, void (*release)(void *));
void untrack(hck_context *ctx, void *obj);   // no-op for an untracked object
void track_server(hck_context *ctx, void *srv, void (*release)(void *));
void untrack_server(hck_context *ctx, void *srv);

// true when a handle is not of this context (or was detached from a
// destroyed one)
template <class T>
inline bool foreign(const hck_context *ctx, const T *h) {
  return h && h->ctx != ctx;
}

// ---- device memory ----
int dev_alloc(hck_context *ctx, uint64_t **p, size_t words);
void dev_free(hck_context *ctx, void *p);
int ensure_ct(hck_context *ctx, hck_ciphertext *ct, uint32_t polys);
int ensure_workspace(hck_context *ctx, size_t words);
int ensure_lt_scratch(hck_context *ctx, size_t words);
int ensure_zero_rows(hck_context *ctx);

// ---- kernel timing ----
// Called before every kernel launch with the launch's grid, its algorithmic
// HBM traffic `bytes` and 64-bit modular multiplications `mulmods` (the
// method's own counts, not the implementation's).  With timing on it records
// events around the launch; with the launch trace on it appends a record.
void timing_begin(hck_context *ctx, const char *name, dim3 grid, double bytes = 0,
                  double mulmods = 0);
void timing_end(hck_context *ctx);
int timing_collect(hck_context *ctx);

// ---- launchers (kernels.hip / ntt.hip); all asynchronous on ctx->stream ----
// forward NTT, in place, rows of `buf` listed in map; input fully reduced,
// output fully reduced
int ntt_forward(hck_context *ctx, uint64_t *buf, const LimbMap &map);
// inverse NTT, in place; output x * scale.w + scale.add (fully reduced); when
// scale is null, multiplies by N^-1 only
int ntt_inverse(hck_context *ctx, uint64_t *buf, const LimbMap &map, const RowScale *scale);
// out-of-place variants: the first pass reads src, both passes write dst
int ntt_forward_oop(hck_context *ctx, uint64_t *dst, const uint64_t *src, const LimbMap &map);
int ntt_inverse_oop(hck_context *ctx, uint64_t *dst, const uint64_t *src, const LimbMap &map,
                    const RowScale *scale);
// one pass (strided or contiguous, forward or inverse) in place; an inverse
// strided pass with `scale` uses entry (row list index mod period) (period 0:
// the list index itself)
// Rescale of polys polynomials at `level` (in and out strided by the
// polynomial stride, out may be in): last holds each polynomial's dropped limb
// in coefficient form ([0, q_level)), tmp has room for polys x level limbs.
int rescale_fused(hck_context *ctx, uint64_t *out, const uint64_t *in, const uint64_t *last,
                  uint64_t *tmp, uint32_t level, uint32_t polys);
// whether the plain transforms of a ring can run on split a (the default or
// one step either side), and the twist tables of split a (null: not built)
bool ntt_split_available(uint32_t log_n, int a);
const uint64_t *const *split_twists(const hck_context *ctx, int a);
// selects the split of the plain full transforms (0: the default), building
// its twist tables on first use
int set_ntt_split(hck_context *ctx, int a);
int ntt_pass(hck_context *ctx, uint64_t *buf, const LimbMap &map, bool inverse, bool strided,
             const RowScale *scale, int period = 0);

int launch_copy(hck_context *ctx, uint64_t *dst, const uint64_t *src, size_t words);
// out[r] = a[r] (+|-) b[r] for rows in map; op 0 add, 1 sub, 2 negate a
// out = sum of in[0..n_in) mod q over the rows of map (out may be one of the inputs)
constexpr int kSumInputs = 32;
int launch_sum_many(hck_context *ctx, uint64_t *out, const uint64_t *const *in, uint32_t n_in,
                    const LimbMap &map);
// out = sum of phi_{galois[k]}(in[k]) (evaluation-domain automorphisms;
// galois 1 = identity); out must not overlap an input read through an
// automorphism
int launch_gather_sum(hck_context *ctx, uint64_t *out, const uint64_t *const *in,
                      const uint32_t *galois, uint32_t n_in, const LimbMap &map);
// measured rate of Shoup modular products on this device (T per second)
int measure_mulmod_rate(hck_context *ctx, double *tera_per_s);
int launch_addsub(hck_context *ctx, uint64_t *out, const uint64_t *a, const uint64_t *b,
                  const LimbMap &map, int op);
// out = [+-] REDC(a * bm) [+ out] (bm in Montgomery form): mode 0 set,
// 1 add to out, 2 subtract from out, 3 set negated
int launch_mul_mont(hck_context *ctx, uint64_t *out, const uint64_t *a, const uint64_t *bm,
                    const LimbMap &map, int mode);
// x -> x 2^64 mod q (into Montgomery form) or x 2^-64 (out of it), in place
int launch_to_mont(hck_context *ctx, uint64_t *buf, const LimbMap &map, bool to);
// tensor of (a0, a1) and (b0, b1) into out0..out2; poly stride given in words
int launch_tensor(hck_context *ctx, uint64_t *out, const uint64_t *a, const uint64_t *b,
                  size_t poly_stride, const LimbMap &map);
// NTT-domain Galois automorphism of `polys` polynomials (poly stride given)
int launch_automorphism(hck_context *ctx, uint64_t *out, const uint64_t *in, size_t poly_stride,
                        uint32_t polys, const LimbMap &map, uint32_t galois);
// small signed integers -> residues for rows in map
int launch_embed_small(hck_context *ctx, uint64_t *out, const int32_t *small, const LimbMap &map);
// rescale: lift the coefficient-domain last limbs last[p] (p < polys) into
// out[p][0..level-1]
int launch_rescale_lift(hck_context *ctx, uint64_t *out, const uint64_t *last, uint32_t level,
                        uint32_t polys);
// rescale tail: out_p,i = (c_p,i - t[p][i]) q_l^-1 mod q_i (poly stride L N)
int launch_rescale_tail(hck_context *ctx, uint64_t *out, const uint64_t *c, const uint64_t *t,
                        uint32_t level, uint32_t polys);
// out[r] += REDC(in[r] c_r) for rows in map, c_r = sc.w[list index]
int launch_scalar_mac(hck_context *ctx, uint64_t *out, const uint64_t *in, const LimbMap &map,
                      const RowScale &sc);

// ---- host helpers ----
LimbMap qmap(const hck_context *ctx, uint32_t level);     // rows 0..level of the q chain
LimbMap fullmap(const hck_context *ctx);                  // rows 0..L+K-1
uint32_t galois_of_step(const hck_context *ctx, int32_t step);

// ---- sampler (sampler.cpp) ----
void shake256(const uint8_t *msg, size_t len, uint8_t *out, size_t outlen);
std::vector<uint8_t> shake_stream(const std::string &tag, uint64_t seed, uint32_t index,
                                  size_t nbytes);
void sample_uniform(const std::string &tag, uint64_t seed, uint32_t index, uint64_t q, uint64_t *out,
                    size_t n);
void sample_ternary(const std::string &tag, uint64_t seed, int32_t *out, size_t n);
void sample_gaussian(const std::string &tag, uint64_t seed, int32_t *out, size_t n);

// ---- encoder (encoder.cpp) ----
// integer coefficients (as int64, |c| < 2^62) of the encoding of z
int encode_coeffs(uint32_t log_n, const double *re, const double *im, double scale,
                  std::vector<int64_t> &coeffs);
// slots from centred CRT of residues [nl][N] (host, coefficient domain)
void decode_residues(uint32_t log_n, const uint64_t *res, const uint64_t *mods, uint32_t nl,
                     double scale, double *re, double *im);

// ---- evaluation internals (eval.cpp) ----
// workspace regions (words from ctx->ws)
size_t ws_words_needed(const hck_context *ctx);
uint64_t *ws_ks(hck_context *ctx);    // key-switch internals
uint64_t *ws_rot(hck_context *ctx);   // [kMaxBatch][L][N]: copies of aliased inputs
uint64_t *ws_tmp(hck_context *ctx);   // [3][L+K][N]: general temporary
uint64_t *ws_pq(hck_context *ctx);    // [kLtOut][2][L+K][N]: extended-basis sums
// Up to kMaxBatch key switches at one level in one sequence of launches,
// slot b with its own switching key key[b] ([dnum][2][L+K][N], Montgomery
// form; slots that share a key read it through the cache):
// (out0[b], out1[b]) = KeySwitch(phi_g(d[b])) + (phi_g(add0[b]), phi_g(add1[b])).
// d and the addends are [level+1][N] in evaluation form; g = 1 for no
// automorphism; null addends are skipped.  out rows must not overlap d; with
// g != 1 they must not overlap the addends.  An output that aliases its
// input's c0 sets add0_src[b] = c0 and add0[b] = a workspace copy of
// [level+1][N] words: the first launch copies c0 there before the last
// launch overwrites it (null: add0 is read in place).
struct KsBatch {
  uint32_t n;
  const uint64_t *key[kMaxBatch];
  uint32_t galois[kMaxBatch];
  const uint64_t *d[kMaxBatch];
  uint64_t *out0[kMaxBatch];
  uint64_t *out1[kMaxBatch];
  const uint64_t *add0[kMaxBatch];
  const uint64_t *add1[kMaxBatch];
  const uint64_t *add0_src[kMaxBatch] = {};
};
int keyswitch_batch(hck_context *ctx, const KsBatch &batch, uint32_t level);
// keyswitch_batch in the given workspace (ws_ks_rows rows per batch slot;
// no allocation)
int keyswitch_batch_ws(hck_context *ctx, const KsBatch &batch, uint32_t level, uint64_t *ws);
// hck_rotate in the library's static scratch array (noalloc.hip)
int rotate_noalloc(hck_context *ctx, const hck_ciphertext *a, int32_t step,
                   const hck_galois_keys *gks, hck_ciphertext *out);
size_t noalloc_scratch_bytes();
size_t noalloc_scratch_needed(const hck_context *ctx);
// largest batch keyswitch_batch accepts at this level (row limits of one launch)
uint32_t ks_batch_limit(const hck_context *ctx, uint32_t level);
// the largest batch one launch sequence can take at this level (row limits)
uint32_t ks_batch_fit(const hck_context *ctx, uint32_t level);
// size of the next batch when `left` key switches remain and one launch takes
// at most `limit`: the batches of what remains are made as even as possible
inline uint32_t even_batch(size_t left, uint32_t limit) {
  const size_t batches = (left + limit - 1) / limit;
  return (uint32_t)((left + batches - 1) / batches);
}
// K1-K4 of keyswitch_batch without ModDown: slot b's key products
// (acc0, acc1) in Q_level u P are added into pq[b] ([2][level+1+K][N];
// Q limbs in evaluation form, P limbs after ModDown's inverse contiguous
// pass, a linear map, so sums stay consistent), or stored there when
// first[b]; slots may share a pq buffer.  out/add fields of the batch are
// unused.  Only moddown_pq reads pq.
int keyswitch_pq(hck_context *ctx, const KsBatch &batch, uint32_t level, uint64_t *const *pq,
                 const bool *first);
// ModDown of n extended-basis pairs pq[b] ([2][level+1+K][N]) to Q_level:
// (out0[b], out1[b]) = ModDown(pq[b]) + (add0[b], add1[b]) (galois fields of
// the batch apply to the addends as in keyswitch_batch; d and key unused)
int moddown_pq(hck_context *ctx, const KsBatch &batch, uint32_t level,
               const uint64_t *const *pq);
// Hoisted rotations of one ciphertext (c0, c1) by n Galois elements: ModUp of
// c1 once, then per element the automorphism of the extended digits, the key
// inner product and ModDown (batched over the elements), plus phi_g(c0).
// out0/out1 rows must not overlap c0 or c1.
int keyswitch_hoisted(hck_context *ctx, const uint64_t *c0, const uint64_t *c1, uint32_t level,
                      const uint32_t *galois, const hck_switch_key *const *keys, uint32_t n,
                      uint64_t *const *out0, uint64_t *const *out1);
// single key switch (batch of one)
int keyswitch_core(hck_context *ctx, const uint64_t *d, uint32_t galois, uint32_t level,
                   const hck_switch_key *key, uint64_t *out0, uint64_t *out1, const uint64_t *add0,
                   const uint64_t *add1);
// fused inner sums of the linear-transform evaluator over limbs 0..level
// inner sums of the linear-transform evaluator over limbs 0..level
int launch_lt_sums(hck_context *ctx, const LtSumArgs &a, uint32_t level);
// automorphisms a[i] -> phi_{g[i]}(a[i]) of n ciphertexts (same level), each
// key-switched with its Galois key, in batches of kMaxBatch; outputs are
// distinct and out[i] may alias a[i] (no other input)
int apply_galois_multi(hck_context *ctx, const hck_ciphertext *const *a, const uint32_t *g,
                       uint32_t n, const hck_galois_keys *gks, hck_ciphertext *const *out);
// the same with the switch keys given, one per ciphertext (they may differ in
// owner: batches across tenants)
int apply_galois_keys(hck_context *ctx, const hck_ciphertext *const *a, const uint32_t *g,
                      const hck_switch_key *const *keys, uint32_t n,
                      hck_ciphertext *const *out);
// relinearizations of n 3-part ciphertexts (one level), each with its own
// key, key-switched together; outputs distinct, out[i] may alias a[i]
int relinearize_keys(hck_context *ctx, const hck_ciphertext *const *a,
                     const hck_switch_key *const *rlk, uint32_t n, hck_ciphertext *const *out);
// switch-key rows in interchange form ([2 dnum][L+K][N] coefficient domain)
// -> evaluation + Montgomery form, in place, on the context stream
int key_rows_to_internal(hck_context *ctx, uint64_t *buf);
// interchange-form ciphertext words in host memory ([polys][level+1][N]) ->
// ct, stream-ordered with no synchronization (host memory pinned for a truly
// asynchronous copy; it must stay valid until the stream reaches the copy)
int ct_from_host_async(hck_context *ctx, hck_ciphertext *ct, const uint64_t *host,
                       uint32_t polys, uint32_t level, double scale);
// ct -> interchange form in host memory (as hck_ciphertext_export writes it),
// stream-ordered with no synchronization
int ct_to_host_async(hck_context *ctx, const hck_ciphertext *ct, uint64_t *host);
// the vital-sign pipeline (hck_vital_eval) over n windows evaluated
// together, window k with its own keys gks[k], rlk[k] (windows of different
// tenants share key-switch batches); out: 4 per window, not aliasing inputs
int vital_eval_batch(hck_context *ctx, const hck_vital_plan *p, const hck_ciphertext *const *re,
                     const hck_ciphertext *const *im, uint32_t n,
                     const hck_galois_keys *const *gks, const hck_switch_key *const *rlk,
                     hck_ciphertext *const *out);
// the same with one Galois element for all
int apply_galois_many(hck_context *ctx, const hck_ciphertext *const *a, uint32_t n, uint32_t g,
                      const hck_galois_keys *gks, hck_ciphertext *const *out);
size_t ws_ks_rows(const hck_context *ctx);   // rows of one batch slot of ws_ks
// key-switch slots of the workspace: up to kMaxBatch while the slots' rows
// stay addressable by 16-bit row indices and within 8192 rows (8 slots at
// least, as many as one launch can take)
uint32_t ks_slots(const hck_context *ctx);
// scratch ciphertexts owned by the context
hck_ciphertext *pool_get(hck_context *ctx);
void pool_put(hck_context *ctx, hck_ciphertext *ct);
int apply_galois_core(hck_context *ctx, const hck_ciphertext *a, uint32_t g,
                      const hck_galois_keys *gks, hck_ciphertext *out);
// runs ntt_forward / ntt_inverse over maps longer than one launch allows
int ntt_forward_rows(hck_context *ctx, uint64_t *buf, const std::vector<std::pair<uint16_t, uint8_t>> &rows);

}  // namespace hck
