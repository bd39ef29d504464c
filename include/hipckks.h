/*
 * hipckks.h -- C ABI of the MI355X (gfx950) RNS-CKKS evaluation library.
 *
 * The paper's encrypted sensing pipeline (section 3.3) is a fixed chain of
 * homomorphic kernels built from the CKKS operations of its primer (section
 * 3.2): KeyGen producing a secret key, a public key, a relinearization key and
 * one Galois key per rotation amount; encoding of up to N/2 slots; slot-wise
 * addition; slot-wise multiplication that consumes one level; and cyclic slot
 * rotation.  Its DFT, FIR and fully connected kernels multiply plaintext
 * matrices into ciphertexts with the diagonal method under baby-step /
 * giant-step scheduling (Kernel 3, Eq. dft_re; Appendix D.1), with the
 * encoded diagonals cached on the cloud GPU (section 5.4, Table 6
 * discussion).  This header is the boundary of that evaluation layer.
 *
 * Conventions (all functions):
 *   - Return HCK_OK (0) on success, a negative hck_status on failure; no C++
 *     exception crosses the ABI.  hck_last_error() gives a message for the
 *     calling thread's last failure.
 *   - Handles returned through a `**` argument are owned by the caller and
 *     freed with the matching *_destroy.  A context must outlive every object
 *     created from it.  Host buffers passed in are read during the call and
 *     never retained; host output buffers are written before the call returns.
 *   - Device memory is owned by the library (stream-ordered allocations on
 *     the context's HIP stream).  Evaluation calls are asynchronous on that
 *     stream; *_export, hck_decode and hck_synchronize wait for it.
 *   - Residue layouts at the boundary are little-endian uint64 words laid out
 *     [poly][limb][N], coefficient domain, every word fully reduced in
 *     [0, q_limb).  Limb i < L is the i-th prime of the q chain; in switching
 *     keys limbs L..L+K-1 are the special primes.
 *   - An output ciphertext may alias an input.  Handles are not thread safe.
 *   - HCK_EDEVICE is sticky: after a HIP runtime error the context refuses
 *     further work.
 */
#ifndef HIPCKKS_H
#define HIPCKKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HCK_MAX_LIMBS 64 /* L + K */

typedef enum hck_status {
  HCK_OK = 0,
  HCK_EINVAL = -1,  /* bad argument, null handle, size mismatch */
  HCK_ENOMEM = -2,  /* device or host allocation failed */
  HCK_EDEVICE = -3, /* HIP runtime error (sticky) */
  HCK_ELEVEL = -4,  /* level mismatch, or no level left */
  HCK_ESCALE = -5,  /* scales differ by more than 2^-30 (relative) */
  HCK_ENOKEY = -6,  /* no Galois key for the requested element */
  HCK_EPARAMS = -7  /* invalid parameter set */
} hck_status;

typedef struct hck_context hck_context;
typedef struct hck_secret_key hck_secret_key;
typedef struct hck_public_key hck_public_key;
typedef struct hck_switch_key hck_switch_key;
typedef struct hck_galois_keys hck_galois_keys;
typedef struct hck_plaintext hck_plaintext;
typedef struct hck_ciphertext hck_ciphertext;
typedef struct hck_linear_transform hck_linear_transform;

/* Parameter set of the ring Z_Q[X]/(X^N + 1) in RNS form (section 3.2: CKKS
 * over RLWE; Table 8: ring degree and depth).  log_n in [11, 17]; q holds the
 * L = num_q primes of the ciphertext modulus chain (q[0] first), p the
 * K = num_p special primes of hybrid key switching; dnum the number of digits
 * of the decomposition.  Every prime must be = 1 (mod 2N), below 2^61 and
 * distinct, with L + K <= HCK_MAX_LIMBS and 1 <= dnum <= L.  The primes of
 * any digit, and the special primes, must each sum to less than 2^64 (the
 * accumulation bound of the basis conversion).  Arrays are copied.
 * Errors: HCK_EPARAMS. */
typedef struct hck_params {
  uint32_t log_n;
  uint32_t num_q;
  uint32_t num_p;
  uint32_t dnum;
  const uint64_t *q;
  const uint64_t *p;
} hck_params;

/* ---- context ------------------------------------------------------------ */

/* Creates a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the device's default stream).  Builds the twiddle
 * and basis-conversion tables on the device.
 * Errors: HCK_EPARAMS, HCK_EDEVICE, HCK_ENOMEM. */
int hck_context_create(const hck_params *params, int device, void *hip_stream,
                       hck_context **out);
int hck_context_destroy(hck_context *ctx);
/* Switches the stream later work is issued on (the caller orders the two). */
int hck_context_set_stream(hck_context *ctx, void *hip_stream);
/* Routes the context's device buffers (ciphertexts, keys, plaintexts,
 * transforms, workspaces) through the caller's allocator, e.g. torch's
 * caching allocator: alloc(bytes, stream, user) returns device memory usable
 * in the order of `stream` (the context stream), or NULL (HCK_ENOMEM);
 * free(ptr, stream, user) returns it, stream-ordered after every use queued
 * on that stream.  Both NULL restores the default (hipMallocAsync /
 * hipFreeAsync on the context stream).  Allowed only while the context holds
 * no buffer of the current allocator (set it right after creation), else
 * HCK_EINVAL.  Constant tables made at creation and a server's resident
 * tenant keys use their own allocations. */
int hck_set_allocator(hck_context *ctx, void *(*alloc)(size_t bytes, void *stream, void *user),
                      void (*free)(void *ptr, void *stream, void *user), void *user);
/* Waits for all work issued on the context's stream. */
int hck_synchronize(hck_context *ctx);
/* Message of the calling thread's last failure ("" if none). */
const char *hck_last_error(void);
/* Galois element 5^(step mod N/2) mod 2N of a left rotation by `step` slots
 * (reading of section 3.2's Rot(Enc(a), k)); 0 for a null context. */
uint32_t hck_galois_element(const hck_context *ctx, int32_t step);

/* ---- keys (client side in the paper, section 3.2 "Key Generation") -------
 * Randomness comes from SHAKE-256 streams keyed by (tag, seed, index), so
 * the same seed gives the same key everywhere (uniform `a` drawn per limb in
 * the coefficient domain, secret ternary, errors discrete Gaussian with
 * sigma = 3.2 cut at 19). */
int hck_keygen_secret(hck_context *ctx, uint64_t seed, hck_secret_key **out);
/* Secret key from N ternary coefficients in {-1, 0, 1}.  Errors: HCK_EINVAL. */
int hck_secret_key_import(hck_context *ctx, const int8_t *coeffs, hck_secret_key **out);
int hck_secret_key_destroy(hck_secret_key *sk);
/* pk = (-a s + e, a) over the full q chain. */
int hck_keygen_public(hck_context *ctx, const hck_secret_key *sk, uint64_t seed,
                      hck_public_key **out);
/* Writes pk as [2][L][N] coefficient-domain words. n_words must be 2 L N. */
int hck_public_key_export(hck_context *ctx, const hck_public_key *pk, uint64_t *out,
                          size_t n_words);
int hck_public_key_destroy(hck_public_key *pk);
/* Relinearization key: switching key from s^2 to s. */
int hck_keygen_relin(hck_context *ctx, const hck_secret_key *sk, uint64_t seed,
                     hck_switch_key **out);
/* Writes a switching key as [dnum][2][L+K][N] coefficient-domain words
 * (b_j rows then a_j rows). n_words must be dnum 2 (L+K) N. */
int hck_switch_key_export(hck_context *ctx, const hck_switch_key *swk, uint64_t *out,
                          size_t n_words);
int hck_switch_key_destroy(hck_switch_key *swk);
/* Galois keys (switching keys from phi_g(s) to s) for n Galois elements
 * (odd, < 2N); duplicates are generated once. */
int hck_keygen_galois(hck_context *ctx, const hck_secret_key *sk, const uint32_t *elements,
                      uint32_t n, uint64_t seed, hck_galois_keys **out);
/* Same, for the elements of left rotations by `steps` slots. */
int hck_keygen_rotation(hck_context *ctx, const hck_secret_key *sk, const int32_t *steps,
                        uint32_t n, uint64_t seed, hck_galois_keys **out);
/* Exports the key of one element as hck_switch_key_export does.
 * Errors: HCK_ENOKEY. */
int hck_galois_keys_export(hck_context *ctx, const hck_galois_keys *gks, uint32_t element,
                           uint64_t *out, size_t n_words);
int hck_galois_keys_count(const hck_galois_keys *gks, uint32_t *n);
int hck_galois_keys_destroy(hck_galois_keys *gks);
/* Imports a switching key from the words hck_switch_key_export writes (the
 * form a client uploads its evaluation keys in; every residue below its
 * prime, else HCK_EINVAL).  The caller owns the result. */
int hck_switch_key_import(hck_context *ctx, const uint64_t *words, size_t n_words,
                          hck_switch_key **out);
/* An empty Galois key set, filled by hck_galois_keys_insert, which takes
 * ownership of swk as the key of `element` (odd, < 2N; a key already there is
 * destroyed). */
int hck_galois_keys_create(hck_context *ctx, hck_galois_keys **out);
int hck_galois_keys_insert(hck_galois_keys *gks, uint32_t element, hck_switch_key *swk);

/* ---- plaintexts (section 3.2 "Encoding and Batching") --------------------- */

/* Encodes N/2 complex slots (im may be NULL: real slots) at `scale` and
 * `level`: coefficients round(scale * m_i) of the real polynomial m with
 * m(zeta^(5^j)) = z_j, zeta = exp(i pi / N), rounded half away from zero.
 * n_slots must be N/2.  |scale * m_i| must stay below 2^62.
 * Errors: HCK_EINVAL, HCK_ELEVEL. */
int hck_encode(hck_context *ctx, const double *re, const double *im, uint32_t n_slots,
               double scale, uint32_t level, hck_plaintext **out);
/* Plaintext from residues [level+1][N] (coefficient domain, fully reduced).
 * Errors: HCK_EINVAL (a word >= its prime), HCK_ELEVEL. */
int hck_plaintext_import(hck_context *ctx, const uint64_t *res, uint32_t level, double scale,
                         hck_plaintext **out);
/* Writes [level+1][N] residues; n_words must be at least (level+1) N. */
int hck_plaintext_export(hck_context *ctx, const hck_plaintext *pt, uint64_t *out,
                         size_t n_words, uint32_t *level, double *scale);
/* Decodes N/2 slots: CRT to centred integers, divided by the scale, then
 * evaluated at the slot roots.  im may be NULL. */
int hck_decode(hck_context *ctx, const hck_plaintext *pt, double *re, double *im,
               uint32_t n_slots);
int hck_plaintext_destroy(hck_plaintext *pt);

/* ---- ciphertexts ---------------------------------------------------------- */

/* Empty ciphertext to be written by an evaluation call. */
int hck_ciphertext_create(hck_context *ctx, hck_ciphertext **out);
/* Ciphertext from residues [size][level+1][N], size 2 or 3. */
int hck_ciphertext_import(hck_context *ctx, const uint64_t *res, uint32_t size, uint32_t level,
                          double scale, hck_ciphertext **out);
/* Writes [size][level+1][N] residues (n_words at least that); waits. */
int hck_ciphertext_export(hck_context *ctx, const hck_ciphertext *ct, uint64_t *out,
                          size_t n_words, uint32_t *size, uint32_t *level, double *scale);
int hck_ciphertext_info(const hck_ciphertext *ct, uint32_t *size, uint32_t *level,
                        double *scale);
int hck_ciphertext_destroy(hck_ciphertext *ct);

/* Enc_sk: (-a s + e + m, a).  Enc_pk: (v pk0 + e0 + m, v pk1 + e1). */
int hck_encrypt_sk(hck_context *ctx, const hck_secret_key *sk, const hck_plaintext *pt,
                   uint64_t seed, hck_ciphertext *out);
int hck_encrypt_pk(hck_context *ctx, const hck_public_key *pk, const hck_plaintext *pt,
                   uint64_t seed, hck_ciphertext *out);
/* m = c0 + c1 s (+ c2 s^2). */
int hck_decrypt(hck_context *ctx, const hck_secret_key *sk, const hck_ciphertext *ct,
                hck_plaintext **out);

/* ---- interchange form ------------------------------------------------------
 * The paper's client uploads its evaluation keys once, at enrollment, and
 * the cloud keeps them; windows travel as ciphertexts (section 5.4,
 * communication and resource overhead).  A blob is a 64-byte header, little
 * endian, then the residues in the export layout (ciphertexts
 * [size][level+1][N], switching keys [dnum][2][L+K][N], coefficient domain).
 * The header names the parameter set: prime_hash is FNV-1a (64-bit) over the
 * L q primes then the K special primes, each as 8 little-endian bytes. */
#define HCK_BLOB_CIPHERTEXT 1u
#define HCK_BLOB_SWITCH_KEY 2u
typedef struct hck_blob_header {
  char magic[8];        /* "HCKCKKS1" */
  uint32_t kind;        /* HCK_BLOB_CIPHERTEXT or HCK_BLOB_SWITCH_KEY */
  uint32_t log_n;
  uint32_t num_q;       /* L */
  uint32_t num_p;       /* K */
  uint32_t dnum;
  uint32_t level;       /* ciphertext level; L - 1 for keys */
  uint32_t polys;       /* ciphertext size (2, 3); 2 dnum for keys */
  uint32_t rows;        /* limbs per polynomial: level + 1; L + K for keys */
  double scale;         /* ciphertext scale; 0 for keys */
  uint64_t prime_hash;
  uint64_t words;       /* residue words after the header: polys rows N */
} hck_blob_header;
/* The parameter set's prime hash (host only, no context). */
int hck_params_hash(const hck_params *params, uint64_t *hash);
/* Checks a blob's header against itself (magic, kind, ranges, shape, total
 * size == 64 + 8 words) and copies it out (host only).  Errors: HCK_EINVAL. */
int hck_blob_parse(const void *buf, size_t size, hck_blob_header *out);
/* Writes the blob of a ciphertext or switching key into buf (cap bytes);
 * *size receives its size.  buf NULL: only the size.  Waits for the stream.
 * Errors: HCK_EINVAL (buffer too small). */
int hck_ciphertext_serialize(hck_context *ctx, const hck_ciphertext *ct, void *buf, size_t cap,
                             size_t *size);
int hck_switch_key_serialize(hck_context *ctx, const hck_switch_key *swk, void *buf, size_t cap,
                             size_t *size);
/* Reads a blob into a new object owned by the caller.  Errors: HCK_EINVAL
 * (malformed blob, another kind, a residue not below its prime), HCK_EPARAMS
 * (made under another parameter set). */
int hck_ciphertext_deserialize(hck_context *ctx, const void *buf, size_t size,
                               hck_ciphertext **out);
int hck_switch_key_deserialize(hck_context *ctx, const void *buf, size_t size,
                               hck_switch_key **out);

/* ---- evaluation (section 3.2 "Three Primitive Operations") ----------------
 * All asynchronous on the context stream. */

/* Slot-wise sum / difference; equal level, scales within 2^-30.
 * Errors: HCK_ELEVEL, HCK_ESCALE, HCK_EINVAL. */
int hck_add(hck_context *ctx, const hck_ciphertext *a, const hck_ciphertext *b,
            hck_ciphertext *out);
int hck_sub(hck_context *ctx, const hck_ciphertext *a, const hck_ciphertext *b,
            hck_ciphertext *out);
int hck_add_plain(hck_context *ctx, const hck_ciphertext *a, const hck_plaintext *pt,
                  hck_ciphertext *out);
/* Slot-wise product with a plaintext of the same level; scales multiply. */
int hck_mul_plain(hck_context *ctx, const hck_ciphertext *a, const hck_plaintext *pt,
                  hck_ciphertext *out);
/* Keeps limbs 0..level. */
int hck_drop_level(hck_context *ctx, const hck_ciphertext *a, uint32_t level,
                   hck_ciphertext *out);
/* Tensor product of two 2-part ciphertexts: (a0 b0, a0 b1 + a1 b0, a1 b1). */
int hck_mul(hck_context *ctx, const hck_ciphertext *a, const hck_ciphertext *b,
            hck_ciphertext *out);
/* (d0, d1) + KeySwitch(d2, rlk) of a 3-part ciphertext. */
int hck_relinearize(hck_context *ctx, const hck_ciphertext *a, const hck_switch_key *rlk,
                    hck_ciphertext *out);
/* Relinearizations of n 3-part ciphertexts of one level, key-switched
 * together in batches (the key is streamed once per batch); residues equal
 * hck_relinearize's for every member.  out[i] may alias a[i] but no other
 * input; outputs must be distinct.  Errors: HCK_EINVAL, HCK_ELEVEL. */
int hck_relinearize_many(hck_context *ctx, const hck_ciphertext *const *a, uint32_t n,
                         const hck_switch_key *rlk, hck_ciphertext *const *out);
/* Divides by the last prime with a centred lift; level - 1, scale / q_level.
 * Errors: HCK_ELEVEL at level 0. */
int hck_rescale(hck_context *ctx, const hck_ciphertext *a, hck_ciphertext *out);
/* Left rotation by `step` slots: (phi_g(c0), 0) + KeySwitch(phi_g(c1), gk_g),
 * g = 5^step mod 2N.  A step = 0 (mod N/2) copies.  Errors: HCK_ENOKEY. */
int hck_rotate(hck_context *ctx, const hck_ciphertext *a, int32_t step,
               const hck_galois_keys *gks, hck_ciphertext *out);
/* Rotations of n ciphertexts (one level) by the same step: the key switches
 * run in batches that stream the Galois key once per batch.  out[i] may alias
 * a[i] but no other input; outputs must be distinct.  Errors as hck_rotate,
 * HCK_ELEVEL, HCK_EINVAL. */
int hck_rotate_many(hck_context *ctx, const hck_ciphertext *const *a, uint32_t n, int32_t step,
                    const hck_galois_keys *gks, hck_ciphertext *const *out);
/* Rotations of n ciphertexts (one level), a[i] by steps[i] (section 3.2
 * rotation, one Galois key per step): the key switches run together in
 * batches, each member with its own key.  Residues equal hck_rotate's for
 * every member.  out[i] may alias a[i] but no other input; outputs must be
 * distinct.  Errors as hck_rotate_many. */
int hck_rotate_steps(hck_context *ctx, const hck_ciphertext *const *a, const int32_t *steps,
                     uint32_t n, const hck_galois_keys *gks, hck_ciphertext *const *out);
/* Hoisted rotations of one ciphertext by n steps: c1 is extended to Q u P
 * once (ModUp) and every step applies its automorphism to the extended
 * digits before the key inner product and ModDown.  These are valid
 * rotations whose residues differ from hck_rotate's (the automorphism does
 * not commute bit-exactly with the basis conversion).  Outputs must be
 * distinct; one may alias a.  Errors: HCK_ENOKEY, HCK_EINVAL. */
int hck_rotate_hoisted(hck_context *ctx, const hck_ciphertext *a, const int32_t *steps,
                       uint32_t n, const hck_galois_keys *gks, hck_ciphertext *const *out);
/* hck_rotate without any allocation, for callers that cannot allocate
 * device memory (work under HIP stream capture, serving loops that forbid
 * hipMalloc).  Residues equal hck_rotate's.  The key switch runs in a static
 * device array of the library (160 MiB per GPU, held from the library's first
 * use of it on that GPU until the process ends) instead of the context's
 * workspace; no hipMalloc, hipFree or allocating library call is made (a few
 * hundred bytes of host memory hold launch tables).  `out` must already hold
 * room for two polynomials: the result or import of an earlier call (a fresh
 * hck_ciphertext_create handle has none: HCK_EINVAL).  out may alias a.
 * Every call on one GPU shares its array and overwrites it: calls that
 * overlap in time on one GPU (other streams, contexts or threads) race, and
 * the caller must serialize them.  Errors: HCK_EINVAL when the context needs
 * more than the array holds (hck_rotate_noalloc_scratch), HCK_ENOKEY,
 * HCK_EDEVICE. */
int hck_rotate_noalloc(hck_context *ctx, const hck_ciphertext *a, int32_t step,
                       const hck_galois_keys *gks, hck_ciphertext *out);
/* Bytes of the static array hck_rotate_noalloc needs for this context (one
 * key-switch slot of (L + dnum (L+K) + 2 (L+K) + 2L) limbs plus L limbs),
 * or the array's size for ctx = NULL. */
size_t hck_rotate_noalloc_scratch(const hck_context *ctx);
/* The same for an explicit Galois element (e.g. 2N-1: conjugation). */
int hck_apply_galois(hck_context *ctx, const hck_ciphertext *a, uint32_t element,
                     const hck_galois_keys *gks, hck_ciphertext *out);
/* Raw hybrid key switching of polynomial 0 of `a`: out = (u0, u1) with
 * u0 + u1 s ~ a0 s' for the key's source secret s'. */
int hck_keyswitch(hck_context *ctx, const hck_ciphertext *a, const hck_switch_key *swk,
                  hck_ciphertext *out);

/* ---- baby-step/giant-step linear transform (Kernel 3; Appendix D.1) --------
 * y = sum_g Rot(sum_b pt_{g,b} * Rot(x, b), g n1) over the generalized
 * diagonals diag_k[j] = A[j][(j + k) mod N/2], k = g n1 + b, 0 <= b < n1
 * (g = floor(k / n1)); pt_{g,b} encodes diag_k rotated right by g n1.  No
 * rescale is applied: the caller rescales. */

/* From n_diag diagonals of N/2 doubles each (rows of diag_re / diag_im, im
 * may be NULL) at offsets[] (|k| < N/2, distinct), encoded at pt_scale
 * (0 = q_level) and cached on the device in evaluation form.
 * Errors: HCK_EINVAL, HCK_ELEVEL. */
int hck_lt_create(hck_context *ctx, const double *diag_re, const double *diag_im,
                  const int32_t *offsets, uint32_t n_diag, uint32_t n_slots, uint32_t baby_step,
                  double pt_scale, uint32_t level, hck_linear_transform **out);
/* From already encoded, already pre-rotated diagonals: residues
 * [n_diag][level+1][N] (coefficient domain). */
int hck_lt_create_from_residues(hck_context *ctx, const uint64_t *res, const int32_t *offsets,
                                uint32_t n_diag, uint32_t baby_step, double pt_scale,
                                uint32_t level, hck_linear_transform **out);
/* Rotation steps the transform needs keys for, ascending.  `cap` is the
 * capacity of steps[]; *n receives the count (steps may be NULL to query). */
int hck_lt_required_steps(const hck_linear_transform *lt, int32_t *steps, uint32_t cap,
                          uint32_t *n);
/* Errors: HCK_ELEVEL (input level != transform level), HCK_ENOKEY. */
int hck_lt_apply(hck_context *ctx, const hck_linear_transform *lt, const hck_ciphertext *a,
                 const hck_galois_keys *gks, hck_ciphertext *out);
/* Sums of transforms over shared inputs, e.g. the complex DFT of Eq. dft_re
 * (d_re = C v_re - S v_im, d_im = S v_re + C v_im):
 *   out[o] = sum_{t : term_out[t] = o} term_sign[t] lts[t](in[term_in[t]]).
 * Every baby rotation Rot(in[i], b) is computed once and the inner sums of
 * all outputs are combined before the giant rotations (Rot(A) + Rot(B) =
 * Rot(A + B)); all giant rotations are key-switched together in batches.
 * All inputs share one level and all transforms that level and one baby
 * step; term_sign may be NULL (all +1) and holds +1 or -1; at most 4 inputs,
 * 4 outputs and 64 giant groups, and no (transform, input, output) twice.
 * Outputs may alias inputs.  flags:
 *   HCK_LT_HOIST_BABY   each input's baby rotations are hoisted rotations
 *                       (hck_rotate_hoisted);
 *   HCK_LT_HOIST_GIANT  an output's giant rotations share one ModDown: their
 *                       key products are summed in Q u P and reduced once,
 *                       and the phi_g(c0) are summed in Q (valid rotations
 *                       with less rounding noise and different residues
 *                       than separate ones).
 * Errors: HCK_EINVAL, HCK_ELEVEL, HCK_ESCALE (terms of one output with
 * different scales), HCK_ENOKEY. */
#define HCK_LT_HOIST_BABY 1u
#define HCK_LT_HOIST_GIANT 2u
int hck_lt_eval(hck_context *ctx, const hck_ciphertext *const *in, uint32_t n_in,
                const hck_linear_transform *const *lts, const uint32_t *term_in,
                const uint32_t *term_out, const int32_t *term_sign, uint32_t n_terms,
                const hck_galois_keys *gks, hck_ciphertext *const *out, uint32_t n_out,
                uint32_t flags);
int hck_lt_destroy(hck_linear_transform *lt);

/* ---- constants and polynomials ---------------------------------------------
 * The constant slot vector `value` at `scale` and `level`: its only nonzero
 * coefficient is m_0 = round(value * scale), half away from zero (a constant
 * has that single coefficient; no FFT rounding enters).  |value * scale|
 * must stay below 2^63 (HCK_EINVAL). */
int hck_encode_const(hck_context *ctx, double value, double scale, uint32_t level,
                     hck_plaintext **out);
/* out = sum_k coeffs[k] x^k slot-wise, k = 0 .. degree (1 <= degree <= 64;
 * some coeffs[k], k >= 1, nonzero), the building block of the polynomial
 * approximations in section 3.3's pipelines (magnitudes, activations).
 * Powers x^(2^j) by squaring, any other x^k = x^a x^(k-a) with a the largest
 * power of two below k (the factor on the higher level dropped to the
 * other's), each product relinearized and rescaled; every term with
 * c_k != 0 is dropped to level l_f + 1, multiplied by the constant c_k
 * encoded at scale s q_(l_f+1) / scale(x^k) and rescaled, so all land on
 * level l_f = level(x) - ceil(log2 degree) - 1 at the input's scale s; they
 * are added in increasing k, then c_0.  out must not alias x.
 * Errors: HCK_ELEVEL (level(x) below ceil(log2 degree) + 1), HCK_EINVAL. */
int hck_poly_eval(hck_context *ctx, const hck_ciphertext *x, const double *coeffs,
                  uint32_t degree, const hck_switch_key *rlk, hck_ciphertext *out);

/* ---- vital-sign pipeline -------------------------------------------------
 * The paper's encrypted vital-sign pipeline (section 3.3.3, example
 * pipelines: K1 -> K2 -> K4 -> K5 -> K7 -> K3 -> K1 -> K2) on one window of
 * F frames x R range bins, packed frame-major (slot t R + r) into a real
 * and an imaginary ciphertext at level l0 (the batched packing of section
 * 3.3.1).  Stages (level reached):
 *   K1  p = Re^2 + Im^2 (l0-1); E_r = sum_t p by rotations R, 2R, ... on a
 *       copy of p dropped to level 3 (the bin branch needs two more levels
 *       and one of headroom, so its rotations run on few limbs)
 *   K2  w = E^gamma by squarings (level 2; gamma below); num_bin =
 *       sum_r w_r bin_index_r, den_bin = sum_r w_r bin_mask_r (rotations
 *       1 .. R/2; level 1)
 *   K4  m = p^P_phi (phase_power below; p^2 at l0-2); I = sum_r m Re,
 *       Q = sum_r m Im per frame (l0-3 for P_phi = 2)
 *   K5  (If, Qf) per band = FIR transform (I, Q) (BSGS, hck_lt_eval; l0-4)
 *   K7  y = Qf[t] If[t-1] - If[t] Qf[t-1], x = If[t] If[t-1] + Qf[t] Qf[t-1]
 *       (l0-5); taylor_order 3: dphi = y x^2 - y^3 third (l0-7); 1: dphi = y
 *   K3  the two bands' DFT bins sit in two groups of G lanes per frame (G the
 *       first power of two >= lanes_resp and lanes_hr): respiration from
 *       lane 0, heart rate from lane G.  Each band's dphi is copied into its
 *       lanes by rotations -1, -2, ...; the bands' weighted products are
 *       added and summed over frames at once (rotations R, 2R, ...): X
 *   K1  P = Re X^2 + Im X^2;  K2  S = P^gamma;  num = sum S freq, den = sum S
 *       mask over each lane group (rotations 1 .. G/2; output level: dft
 *       level - 4).
 * Outputs: out[0] num_bin, out[1] den_bin (value in slot 0), out[2]
 * num_rates, out[3] den_rates (respiration in slot 0, heart rate in slot
 * G); the client's scalar divisions (section 3.3.4) give the target bin and
 * the two rates in beats per minute.
 * The operands are public plaintexts and transforms owned by the caller,
 * encoded for inputs at a base level l0 (fir_* at l0-3, the others as
 * above, at scale q_level so that a product keeps the ciphertext's scale).
 * Inputs may come at any level >= l0: the pipeline drops them to l0 first
 * (the circuit consumes only its depth), so a plan encoded at l0 = depth runs
 * on depth + 1 primes whatever level the client encrypted at.
 * Errors: HCK_EINVAL (bad layout or missing operand), HCK_ELEVEL (input
 * level too low for the depth, operand level too low), HCK_ENOKEY. */
typedef struct {
  uint32_t frames, bins;         /* F; R a power of two, pow2ceil(F) R <= N/2 */
  uint32_t taylor_order;         /* 1 or 3 */
  uint32_t lanes_resp, lanes_hr; /* DFT bins per band; 2 pow2ceil(max) <= R */
  const hck_plaintext *bin_index, *bin_mask;                    /* level 2 */
  const hck_linear_transform *fir_resp, *fir_hr;                /* l0-3 */
  const hck_plaintext *third;                                   /* l0-5 (order 3) */
  const hck_plaintext *dft_re_resp, *dft_im_resp, *dft_re_hr, *dft_im_hr; /* l0-7 / l0-5 */
  const hck_plaintext *freq, *mask;                             /* dft level - 3 */
  /* magnitude option (0: the paper's power): the bin estimate's energy sums
   * the polynomial magnitude sum_k mag_coeffs[k] p^k ~ |z| of degree
   * mag_degree (1 .. 15, evaluated by hck_poly_eval on p) instead of p */
  uint32_t mag_degree;
  const double *mag_coeffs; /* mag_degree + 1 coefficients, caller-owned */
  /* soft-attention exponent of both K2 stages (Eq. soft_power_weight):
   * 2 (0 also means 2) or 4, by one or two squarings; 4 adds one level to
   * the main chain (freq and mask at dft level - 4, outputs one level
   * lower) and one to the bin branch (its energy sums at level 4) */
  uint32_t gamma;
  /* K4's mask exponent P_phi (Eq. phase_mask): 2 (0 also means 2) to 5, by
   * p^2, p^3 = p^2 p, p^4 = (p^2)^2, p^5 = (p^2)^2 p.  3 and 4 take one level
   * more before K5 and 5 two more: every operand from fir_* on sits that
   * many levels lower (fir_* at l0 - 3 - e, e = 0, 1, 1, 2) */
  uint32_t phase_power;
} hck_vital_plan;
/* Rotation steps the pipeline needs Galois keys for (ascending; `cap` is the
 * capacity of steps[], *n receives the count; steps may be NULL). */
int hck_vital_required_steps(const hck_context *ctx, const hck_vital_plan *plan, int32_t *steps,
                             uint32_t cap, uint32_t *n);
/* One window; out[0..3] must not alias re or im. */
int hck_vital_eval(hck_context *ctx, const hck_vital_plan *plan, const hck_ciphertext *re,
                   const hck_ciphertext *im, const hck_galois_keys *gks,
                   const hck_switch_key *rlk, hck_ciphertext *const *out);
/* hck_vital_eval that also copies each kernel's intermediate result into
 * taps[i] (caller-owned; a null entry skips that copy), for the per-kernel
 * encryption-noise measurement of section 5.2 (Table 3: encrypted against
 * plaintext execution, cumulative after the preceding kernels):
 *   0 K1 p (slot t R + r)          1 K1 energy E (slot r)
 *   2 K2 w = E^2 (slot r)          3, 4 K4 I, Q (slot t R)
 *   5..8 K5 If, Qf of respiration, If, Qf of heart rate (slot t R)
 *   9, 10 K7 dphi of respiration, heart rate (slot t R)
 *   11, 12 K3 Re X, Im X (lane c of frame 0)
 *   13 K1 P = Re X^2 + Im X^2     14 K2 S = P^2 (lane c).
 * out[] receives hck_vital_eval's results, bit-identical to it.  Taps must
 * not alias re or im. */
#define HCK_VITAL_TAPS 15
int hck_vital_eval_taps(hck_context *ctx, const hck_vital_plan *plan, const hck_ciphertext *re,
                        const hck_ciphertext *im, const hck_galois_keys *gks,
                        const hck_switch_key *rlk, hck_ciphertext *const *out,
                        hck_ciphertext *const *taps);
/* The pipeline on per-frame packing (section 3.3.2): frame t of the window
 * in its own ciphertext pair re[t], im[t] (t < frames, frames = the plan's
 * F), its R range bins in slots 0 .. R-1, zeros elsewhere, every pair at one
 * level >= the plan's l0.  K1 and K4 run on each pair: p_t, and I_t, Q_t
 * summed into slot 0 by rotations 1 .. R/2; the bin branch sums the frames'
 * powers by additions (no rotation).  The frames' I_t and Q_t then go to slot
 * t R of one ciphertext each by a tree of rotations (step j: every other
 * entry rotated by -2^j R and added to its left neighbour), the batched
 * packing's layout, and K5 -> K2 run as in hck_vital_eval.  The four outputs
 * decode to the batched pipeline's values (their residues differ: other
 * operations reach them).  Galois keys: hck_vital_frames_required_steps
 * (the plan's steps and -R, -2R, ..., -(T2/2) R).  Errors as
 * hck_vital_eval; HCK_EINVAL if frames differs from the plan's F. */
int hck_vital_frames_required_steps(const hck_context *ctx, const hck_vital_plan *plan,
                                    int32_t *steps, uint32_t cap, uint32_t *n);
int hck_vital_eval_frames(hck_context *ctx, const hck_vital_plan *plan,
                          const hck_ciphertext *const *re, const hck_ciphertext *const *im,
                          uint32_t frames, const hck_galois_keys *gks, const hck_switch_key *rlk,
                          hck_ciphertext *const *out);
/* n windows with one plan, evaluated together: every stage advances all
 * windows, so their rotate-and-sum chains and relinearizations share batched
 * key switches (a throughput mode; each window's residues equal
 * hck_vital_eval's).  Window k reads re[k], im[k] and writes out[4k .. 4k+3];
 * outputs must not alias inputs. */
int hck_vital_eval_many(hck_context *ctx, const hck_vital_plan *plan,
                        const hck_ciphertext *const *re, const hck_ciphertext *const *im,
                        uint32_t n, const hck_galois_keys *gks, const hck_switch_key *rlk,
                        hck_ciphertext *const *out);

/* ---- gesture-classification pipeline --------------------------------------
 * The paper's encrypted gesture pipeline (section 3.3.3, example pipelines:
 * K3 -> K1 -> K2 + K6 per frame, frame accumulation, FC1 -> x^2 -> FC2 ->
 * x^2 -> FC3; depth 11, Table 1) on F range-processed frames of R range bins
 * x D chirps packed (t R + r) D + c into a real and an imaginary ciphertext
 * at level l0, with pow2ceil(F) R D = N/2.  Stages (level reached):
 *   K3  Doppler DFT of every D-chirp block by hck_lt_eval with the windowed
 *       fftshifted DFT's real and imaginary block-diagonal transforms dft_c,
 *       dft_s (hoisted baby steps, shared giant ModDown; l0-1)
 *   K1  P = d_re^2 + d_im^2 (l0-2);  K6  P notch (l0-3)
 *   K2  w = P^4 by two squarings (gamma = 4; l0-5); feature = P w (l0-6);
 *       frames summed by rotations R D, 2 R D, ...
 *   FC1 fc1 over the cyclic feature vector (H1 diagonals), blocks of H1
 *       slots summed by rotations H1, 2 H1, ..., R D / 2; + bias1; squared
 *   FC2 fc2 (rectangular diagonals) + bias2; squared;  FC3 fc3 + bias3.
 * The output holds the logits in slots 0 .. classes-1 at level l0-11.
 * Transforms and plaintexts are owned by the caller and encoded for inputs
 * at a base level l0 (dft l0, notch l0-2, fc1 l0-6, fc2 l0-8, fc3 l0-10;
 * bias_i at the level after its product, at the scale reached there).
 * Inputs at a level above l0 are dropped to l0 first.
 * Errors: HCK_EINVAL, HCK_ELEVEL, HCK_ESCALE, HCK_ENOKEY. */
typedef struct {
  uint32_t frames, bins, chirps; /* F, R, D */
  uint32_t hidden1;              /* FC1 outputs H1; R D / H1 a power of two */
  const hck_linear_transform *dft_c, *dft_s, *fc1, *fc2, *fc3;
  const hck_plaintext *notch, *bias1, *bias2, *bias3;
} hck_gesture_plan;
int hck_gesture_required_steps(const hck_context *ctx, const hck_gesture_plan *plan,
                               int32_t *steps, uint32_t cap, uint32_t *n);
int hck_gesture_eval(hck_context *ctx, const hck_gesture_plan *plan, const hck_ciphertext *re,
                     const hck_ciphertext *im, const hck_galois_keys *gks,
                     const hck_switch_key *rlk, hck_ciphertext *out);
/* hck_gesture_eval that also copies each stage's result into taps[i]
 * (caller-owned; null entries skipped), for the per-kernel encryption-noise
 * measurement of section 5.2 (Table 3):
 *   0, 1 K3 d_re, d_im (slot (t R + r) D + c)   2 K1 P   3 K6 P notch
 *   4 K2 w = P^4   5 feature P w summed over frames (slot r D + c)
 *   6 FC1 + bias1 (slots 0 .. H1-1)   7 FC2 + bias2 (slots 0 .. H2-1).
 * out receives hck_gesture_eval's logits, bit-identical to it.  Taps must
 * not alias re or im. */
#define HCK_GESTURE_TAPS 8
int hck_gesture_eval_taps(hck_context *ctx, const hck_gesture_plan *plan,
                          const hck_ciphertext *re, const hck_ciphertext *im,
                          const hck_galois_keys *gks, const hck_switch_key *rlk,
                          hck_ciphertext *out, hck_ciphertext *const *taps);
/* The same pipeline on per-frame packing (section 3.3.2, the layout before
 * batching: one ciphertext pair per frame).  re[f], im[f] (f < n_frames) hold
 * frame f's R range bins x D chirps in slots r D + c and zeros in every other
 * slot (the caller's packing; nonzero slots there would enter the frame sum).
 * Each pair runs K3 -> K1 -> K6 -> K2 on its own, exactly as one frame block
 * of hck_gesture_eval; the n_frames features are added in frame order, and
 * rotations R D, 2 R D, ..., N/4 copy the sum into every block of R D slots
 * before the FC network, as the batched packing leaves it.  So the logits
 * decode to those of hck_gesture_eval on the same frames packed together,
 * at the same level (l0-11), for 2 n_frames input ciphertexts instead of 2.
 * plan->frames is not used beyond the layout check; any 1 <= n_frames <=
 * HCK_GESTURE_MAX_FRAMES frames are accepted.  All frames share one level (at
 * least l0; higher ones are dropped to l0) and one scale.
 * Errors: HCK_EINVAL, HCK_ELEVEL, HCK_ESCALE, HCK_ENOKEY. */
#define HCK_GESTURE_MAX_FRAMES 4096
int hck_gesture_eval_frames(hck_context *ctx, const hck_gesture_plan *plan,
                            const hck_ciphertext *const *re, const hck_ciphertext *const *im,
                            uint32_t n_frames, const hck_galois_keys *gks,
                            const hck_switch_key *rlk, hck_ciphertext *out);

/* ---- gesture CNN variant ----------------------------------------------------
 * The gesture classifier's CNN variant: the front end of hck_gesture_eval
 * (K3 Doppler DFT -> K1 power -> K6 notch -> K2 P^4, feature P P^4, frame
 * accumulation; section 3.3.3), then on the R x D feature map (slot r D + c
 * of every block of R D slots):
 *   conv1  3 x 3, stride 2, zero padding, 1 -> c1 channels: block b computes
 *          channel b mod c1 at the even positions (r, c); one BSGS transform
 *          over the diagonals of offsets dy D + dx
 *   act    sum_k act_coeffs[k] x^k (hck_poly_eval)
 *   conv2  3 x 3, stride 2, c1 -> c2: block b computes channel b mod c2 at
 *          the positions that are multiples of 4, from channel (b + delta)
 *          mod c1 of block b + delta (offsets delta R D + 2 (dy D + dx))
 *   act
 *   dense1 2 x 2 average pooling folded into the hybrid diagonals of the
 *          hidden x (c2 (R/8) (D/8)) weights over the period c2 R D of the
 *          replicated channels (offsets 0 .. hidden-1), then rotations hidden,
 *          2 hidden, ..., c2 R D / 2 sum the sub-blocks; + bias1; act
 *   dense2 classes x hidden by its rectangular diagonals; + bias2: the logits
 *          in slots 0 .. classes-1.
 * Every transform is applied with hoisted baby steps and a shared ModDown
 * per giant step and followed by one rescale.  Levels, for the input level
 * l0 of dft_c and a = ceil(log2 act_degree) + 1: conv1 at l0-6, conv2 at
 * l0-7-a, dense1 at l0-8-2a, bias1 l0-9-2a, dense2 l0-9-3a, bias2 and the
 * logits l0-10-3a.  Requirements: pow2(frames) R D = N/2, R and D multiples
 * of 8, (N/2)/(R D) a multiple of c1 and of c2, c2 R D / hidden a power of
 * two.  Inputs above l0 are dropped to it. */
typedef struct {
  uint32_t frames, bins, chirps;      /* F x R x D, batched packing */
  uint32_t c1, c2, hidden, classes;
  const hck_linear_transform *dft_c, *dft_s;            /* level l0 */
  const hck_plaintext *notch;                           /* l0 - 2 */
  const hck_linear_transform *conv1, *conv2, *dense1, *dense2;
  const hck_plaintext *bias1, *bias2;
  uint32_t act_degree;                /* 1 .. 15 */
  const double *act_coeffs;           /* act_degree + 1, caller-owned */
} hck_gesture_cnn_plan;
int hck_gesture_cnn_required_steps(const hck_context *ctx, const hck_gesture_cnn_plan *plan,
                                   int32_t *steps, uint32_t cap, uint32_t *n);
/* The logits of one window.  taps (nullable; null entries skipped) receive
 * the intermediates: 0 the accumulated feature map, 1 conv1 + act, 2 conv2
 * + act, 3 dense1 + bias1 + act.  Errors: HCK_EINVAL, HCK_ELEVEL,
 * HCK_ENOKEY. */
#define HCK_GESTURE_CNN_TAPS 4
int hck_gesture_cnn_eval(hck_context *ctx, const hck_gesture_cnn_plan *plan,
                         const hck_ciphertext *re, const hck_ciphertext *im,
                         const hck_galois_keys *gks, const hck_switch_key *rlk,
                         hck_ciphertext *out, hck_ciphertext *const *taps);

/* ---- device calibration ---------------------------------------------------
 * Rate of 64-bit Shoup modular products (a w mod q for a fixed w, the product
 * of every NTT butterfly) that this device sustains on its vector ALUs, in
 * 10^12 per second, from one timed compute-only launch (about 2^30 products
 * in dependent chains, 8 per thread) on the context's stream.  A measured
 * integer ceiling for the evaluation kernels, reported beside the HBM
 * bandwidth.  Errors: HCK_EINVAL, HCK_EDEVICE. */
int hck_measure_mulmod_rate(hck_context *ctx, double *tera_per_s);

/* Autotuner of the key-switch schedule (the batching of section 3.3's
 * rotations on this chip): for each of n_levels levels it times key
 * switches of `count` zero ciphertexts at that level with a zero key.  Each
 * candidate number of key switches per launch sequence (1 .. 32, within the
 * launch row limits) is tried, and the context keeps the fastest per key
 * switch.  The built-in rule stays unless a candidate beats it by 2 %.
 * caps[i] and us_per_switch[i] (either may be NULL) receive the choice and
 * its time.  Synchronizes the stream; results of later calls do not depend
 * on the schedule (tested bit for bit).  Errors: HCK_ELEVEL, HCK_EINVAL. */
int hck_autotune_keyswitch(hck_context *ctx, const uint32_t *levels, uint32_t n_levels,
                           uint32_t count, uint32_t *caps, double *us_per_switch);
/* Autotuner of the digit count of hybrid key switching (dnum; section 3.2's
 * relinearization and Galois keys are the switching keys): more digits make
 * smaller keys' special-prime basis but more key-inner-product work and
 * larger keys.  candidates[0..n) share the ring and the q chain, each with its
 * own dnum and special primes.  For each, a context is built on `device` /
 * `hip_stream`, `count` key switches of zero ciphertexts at `level` are timed
 * with a zero key (median of 3 after a warm-up), and the context is
 * destroyed.  us_per_switch[i] and key_bytes[i] (a switching key's device
 * size) receive each candidate's figures, *best the fastest's index (any
 * output may be NULL).  Errors: HCK_EINVAL, HCK_ELEVEL, HCK_EPARAMS,
 * HCK_EDEVICE, HCK_ENOMEM. */
int hck_autotune_dnum(const hck_params *candidates, uint32_t n, int device, void *hip_stream,
                      uint32_t level, uint32_t count, double *us_per_switch, double *key_bytes,
                      uint32_t *best);
/* Autotuner of the NTT split (the radices of the two passes a full
 * negacyclic NTT takes on this chip, N = R1 x R2; section 3.2's encoding,
 * encryption and key material go through full transforms).  Candidates: the
 * default R1 = 2^ceil(log N / 2) and one step either side where both passes
 * fit a workgroup (at most 80 KiB of LDS each, a contiguous sub-transform in
 * one wavefront).  Each is timed on `rows` (1 .. 256) rows of zeros, forward
 * then inverse (median of 5 after a warm-up); splits[i] (log2 R1) and
 * us_per_row[i] receive each candidate (cap entries at least, NULL to skip),
 * *n their count, *chosen the split kept: the default unless another is 2 %
 * faster.  The choice applies to the context's full transforms (encoding,
 * encryption, imports, keys, rescale's dropped limb); the fused key-switch
 * passes keep the default split.  Results never change (tested bit for
 * bit).  Errors: HCK_EINVAL, HCK_ENOMEM, HCK_EDEVICE. */
int hck_autotune_ntt(hck_context *ctx, uint32_t rows, int32_t *splits, double *us_per_row,
                     uint32_t cap, uint32_t *n, int32_t *chosen);
/* Selects the split of the full transforms by log2 R1 (0: the default) and
 * reads the one in force.  Errors: HCK_EINVAL (not a candidate). */
int hck_set_ntt_split(hck_context *ctx, int32_t log_r1);
int hck_ntt_split(const hck_context *ctx, int32_t *log_r1);
/* Sets the key switches per launch sequence at `level` (a saved tuning; 0
 * restores the built-in rule), and reads the size in force. */
int hck_set_keyswitch_cap(hck_context *ctx, uint32_t level, uint32_t cap);
int hck_keyswitch_batch_limit(const hck_context *ctx, uint32_t level, uint32_t *cap);

/* ---- kernel timing --------------------------------------------------------
 * With timing on, every kernel launch is bracketed by HIP events on the
 * context stream and its duration added to a per-kernel-name total, read
 * (after waiting for the stream) with hck_timing_read, together with the
 * launches' summed algorithmic HBM bytes (each operand read once, each result
 * written once) and 64-bit modular multiplications.  `name` is one of the
 * names hck_timing_names lists (comma separated).  Any output may be NULL. */
int hck_timing_enable(hck_context *ctx, int on);
int hck_timing_reset(hck_context *ctx);
int hck_timing_read(hck_context *ctx, const char *name, double *total_ms, uint64_t *launches,
                    double *bytes, double *mulmods);
int hck_timing_names(hck_context *ctx, char *buf, size_t cap);

/* ---- graph capture -------------------------------------------------------
 * Batching of section 3.3's windows on this chip: the evaluation calls a
 * caller makes on one or more contexts (one per ring or parameter set, or
 * several per ring, each evaluating its own group of windows) are recorded
 * once, each context's calls into a HIP graph on its own stream, and replayed
 * together, so that the windows of the contexts run side by side on the
 * device and no launch waits for the host.
 *
 * hck_graph_begin starts recording every call on the n contexts (distinct,
 * same GPU, each on a created stream of its own, none timing).  Until
 * hck_graph_end, calls on them issue nothing to the device; they record.
 * Recorded calls must not allocate device memory (run the same calls once
 * before capturing: every workspace, scratch ciphertext and output then
 * exists), transfer host memory (encode, encrypt, import, export, decrypt) or
 * wait (hck_synchronize); such calls fail with HCK_EINVAL, and the capture
 * then fails at hck_graph_end.  One capture per host thread at a time.
 *
 * hck_graph_end (same contexts, same order) stops recording and instantiates
 * the graphs.  hck_graph_launch replays every context's graph on that
 * context's stream: after all work issued earlier on the stream, and before
 * any work issued later on it (the contexts' replays are not ordered with
 * respect to each other).  The outputs of the recorded calls are rewritten
 * from the current contents of their inputs (the ciphertext levels and
 * scales stay those of the capture).
 * A replay is refused (HCK_EINVAL) once a device buffer of the contexts that
 * existed when the capture ended has been given back (the graph may read
 * it): destroy no handle the recorded calls used, and capture again after a
 * workspace has grown.  Destroying
 * any of the contexts releases the graph (later launches: HCK_EINVAL); its
 * destroy call then frees the host record.  hck_graph_info gives the number
 * of contexts and of graph nodes.
 * Errors: HCK_EINVAL, HCK_EDEVICE. */
typedef struct hck_graph hck_graph;
int hck_graph_begin(hck_context *const *ctxs, uint32_t n);
int hck_graph_end(hck_context *const *ctxs, uint32_t n, hck_graph **out);
int hck_graph_launch(hck_graph *graph);
int hck_graph_info(const hck_graph *graph, uint32_t *contexts, size_t *nodes);
int hck_graph_destroy(hck_graph *graph);

/* ---- launch trace ----------------------------------------------------------
 * The execution trace of Theorem 2 (data obliviousness; proof in Appendix D):
 * what the cloud side does, in order, as the host issues it.  With the trace
 * on, the context appends one record per kernel launch (its name as the
 * timing names above, its grid in workgroups, its algorithmic bytes and
 * modular multiplications) and one per device allocation ("alloc", bytes) or
 * release ("free"), in issue order.  Nothing is timed and nothing waits on the
 * device.  Two runs of a pipeline on inputs of the same public configuration
 * must give identical records.  Turning the trace on clears the log; records
 * are kept until the next hck_trace_enable(ctx, 1). */
typedef struct hck_trace_record {
  char name[32];
  uint32_t grid[3];
  double bytes;
  double mulmods;
} hck_trace_record;
int hck_trace_enable(hck_context *ctx, int on);
/* Copies up to cap records into out (out may be NULL when cap is 0) and
 * stores the number of records held in *count.  Errors: HCK_EINVAL. */
int hck_trace_read(hck_context *ctx, hck_trace_record *out, size_t cap, size_t *count);

/* ---- client-side host utilities (no context, no device) -------------------
 * The paper's client encodes, encrypts and decodes (section 3.2 "Encoding and
 * Batching"; section 3.3.4 result recovery).  These run on the host only. */

/* SHAKE-256 (FIPS 202) of msg, outlen bytes. */
int hck_shake256(const uint8_t *msg, size_t len, uint8_t *out, size_t outlen);
/* The samplers behind key generation and encryption: stream
 * SHAKE-256("hipckks/" || tag || "/" || le64(seed) || le32(index)).
 * Uniform: 64-bit little-endian words masked to bitlen(q), kept when < q.
 * Ternary (stream index 0): bytes, 255 rejected, b mod 3 -> 0, +1, -1.
 * Gaussian (stream index 0): sigma = 3.2 cut at 19 by a cumulative table on
 * the top 63 bits of each 64-bit word, bit 0 the sign. */
int hck_sample_uniform(const char *tag, uint64_t seed, uint32_t index, uint64_t q,
                       uint64_t *out, size_t n);
int hck_sample_ternary(const char *tag, uint64_t seed, int32_t *out, size_t n);
int hck_sample_gaussian(const char *tag, uint64_t seed, int32_t *out, size_t n);
/* Integer coefficients [N] of the encoding of N/2 slots at `scale` (as
 * hck_encode, before reduction modulo the primes). */
int hck_encode_coeffs(uint32_t log_n, const double *re, const double *im, double scale,
                      int64_t *coeffs);
/* Slots [N/2] of coefficient-domain residues [nl][N] over mods[0..nl): centred
 * CRT, divided by scale, evaluated at the slot roots.  im may be NULL. */
int hck_decode_residues(uint32_t log_n, const uint64_t *res, const uint64_t *mods, uint32_t nl,
                        double scale, double *re, double *im);

/* ---- serving runtime ---------------------------------------------------------
 * Encrypted windows from many tenants (edge clients) evaluated with continuous
 * batching: the streaming deployment that section 7 names as future work,
 * with the cloud side of section 3.3 serving several clients at once.
 *
 * A server owns one context: after hck_server_create, the caller uses the
 * context only through the server until hck_server_destroy.  One worker
 * thread admits requests in arrival order while the HBM budget allows.  A
 * tenant's evaluation keys are loaded from the caller's host memory when it
 * has none resident, two tenants' transfers at a time, on a copy stream that
 * overlaps the evaluation.  To make room, idle tenants are evicted, least
 * recently used first; a tenant with admitted work is never evicted.  A
 * request waiting for its tenant's keys (or for budget) does not hold back
 * later requests of resident tenants.  The worker launches admitted windows
 * whose keys have arrived, up to max_batch of one pipeline per batch,
 * whenever fewer than two batches are queued on the device.  So requests
 * that arrive while others run join the next batch, and windows of different
 * tenants share key-switch launches, each with its own keys.  Every result
 * equals, bit for bit, the plain call's (hck_vital_eval / hck_gesture_eval)
 * on the same window and keys. */
#define HCK_SERVE_VITAL 1u
#define HCK_SERVE_GESTURE 2u
typedef struct hck_server hck_server;
typedef struct {
  uint64_t hbm_budget;   /* bytes for resident tenant keys + admitted windows'
                            input and output ciphertexts */
  uint32_t max_batch;    /* windows per batch, 1..64 */
  uint32_t max_inflight; /* windows admitted and not yet completed, 1..256
                            (also the number of pinned staging slots) */
} hck_server_config;
typedef struct {
  uint64_t request;      /* the caller's id */
  int32_t status;        /* HCK_OK or the error code of the failure */
  uint32_t tenant;
  uint32_t n_out;        /* 4 (vital) or 1 (gesture) */
  uint32_t batch;        /* windows in the batch the request ran in */
  uint32_t key_load;     /* 1 if admitting it loaded its tenant's keys */
  uint32_t out_level[4];
  double out_scale[4];
  double t_submit, t_admit, t_launch, t_done; /* seconds, host steady clock */
} hck_server_result;
typedef struct {
  uint64_t budget, resident_bytes; /* resident_bytes: keys + admitted windows */
  uint64_t tenants, submitted, completed, failed, pending;
  uint64_t batches, windows, key_loads, evictions, key_bytes_loaded;
} hck_server_stats;
int hck_server_create(hck_context *ctx, const hck_server_config *cfg, hck_server **out);
/* Registers tenant `tenant` running pipeline `kind` with `plan` (an
 * hck_vital_plan or hck_gesture_plan, caller-owned, may be shared by tenants)
 * and its keys in host memory as hck_switch_key_export writes them: the
 * Galois key of each of n_steps rotation steps (gk_words[i] for steps[i]) and
 * the relinearization key.  The host words are read whenever the keys are
 * loaded: they stay valid and unchanged until the server is destroyed (pinned
 * memory makes the loads asynchronous).  Errors: HCK_ENOKEY when a step the
 * pipeline needs has no key; HCK_EINVAL for a tenant id already registered. */
int hck_server_add_tenant(hck_server *srv, uint32_t tenant, uint32_t kind, const void *plan,
                          const int32_t *steps, const uint64_t *const *gk_words, uint32_t n_steps,
                          const uint64_t *rlk_words);
/* Queues one window of a registered tenant: re and im in interchange form
 * ([2][level+1][N] each, as hck_ciphertext_export writes; copied, so the
 * buffers may be reused on return).  When the request completes, its outputs
 * are written to out_words one after another, each [2][out_level[i]+1][N]
 * (vital: num_bin, den_bin, num_rates, den_rates; gesture: the logits);
 * out_capacity (words) must cover them, else the request fails with
 * HCK_EINVAL.  out_words stays valid until the request's result is polled. */
int hck_server_submit(hck_server *srv, uint64_t request, uint32_t tenant, const uint64_t *re_words,
                      const uint64_t *im_words, uint32_t level, double scale, uint64_t *out_words,
                      size_t out_capacity);
/* Returns up to cap completed requests in completion order, waiting up to
 * timeout_ms for the first (returning early once nothing is outstanding). */
int hck_server_poll(hck_server *srv, uint32_t timeout_ms, hck_server_result *results, uint32_t cap,
                    uint32_t *n);
int hck_server_stats_get(hck_server *srv, hck_server_stats *out);
/* Completes every queued request, frees the tenants' device keys and the
 * staging memory, and hands the context back to the caller. */
int hck_server_destroy(hck_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* HIPCKKS_H */
