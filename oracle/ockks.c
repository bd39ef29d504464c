/*
 * Oracle core: plain, slow, scalar RNS arithmetic for CKKS evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP library, and the HIP
 * library never calls it.
 *
 * The paper (section 3.2, "Homomorphic Encryption Primer") names the scheme
 * (CKKS over RLWE, with addition, multiplication with relinearization and
 * slot rotation with Galois keys) and defers the internals to its backend
 * libraries.  This file writes those internals out from their textbook
 * definitions, one function per definition, with no blocking, lazy reduction
 * or fused steps:
 *
 *   - residues of the ring Z_q[X]/(X^N + 1), one row of N words per prime;
 *   - every product is (unsigned __int128)a * b % q;
 *   - the negacyclic NTT evaluates a polynomial at the odd powers of a
 *     primitive 2N-th root psi: out[k] = a(psi^(2k+1)), via the twist by
 *     psi^i and a textbook iterative radix-2 cyclic DFT;
 *   - polynomial products are NTT -> pointwise -> inverse NTT;
 *   - the Galois automorphism X -> X^g is applied to coefficients by its
 *     definition (index i -> i*g mod 2N, negated past N);
 *   - fast basis conversion, hybrid key switching (digit decomposition,
 *     ModUp, inner product with the switching key, ModDown) and rescale by
 *     the last prime follow their formulas term by term.
 *
 * All arrays hold residues in [0, q); polynomials are in coefficient form,
 * laid out [limb][N].  Loops over limbs run under OpenMP; nothing else is
 * parallel.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef unsigned __int128 u128;

/* ---- scalar modular arithmetic (definition) ---------------------------- */

static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }
static u64 submod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + q - b) % q); }

static u64 powmod(u64 a, u64 e, u64 q) {
  u64 r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = mulmod(r, a, q);
    a = mulmod(a, a, q);
    e >>= 1;
  }
  return r;
}

/* q is prime: a^(q-2) is the inverse of a. */
static u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); }

u64 ock_mulmod(u64 a, u64 b, u64 q) { return mulmod(a, b, q); }
u64 ock_powmod(u64 a, u64 e, u64 q) { return powmod(a, e, q); }
u64 ock_invmod(u64 a, u64 q) { return invmod(a, q); }

/* A primitive 2N-th root of unity mod q (q = 1 mod 2N): the first x >= 2
 * whose power x^((q-1)/2N) satisfies psi^N = -1 (then its order is 2N). */
u64 ock_root_2n(u64 q, u64 n) {
  for (u64 x = 2;; x++) {
    u64 psi = powmod(x, (q - 1) / (2 * n), q);
    if (powmod(psi, n, q) == q - 1) return psi;
  }
}

/* ---- negacyclic NTT ------------------------------------------------------ */

static void bit_reverse(u64 *a, u64 n) {
  for (u64 i = 1, j = 0; i < n; i++) {
    u64 bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      u64 t = a[i];
      a[i] = a[j];
      a[j] = t;
    }
  }
}

/* Textbook cyclic DFT over Z_q with root w of order n, natural order in/out:
 * out[k] = sum_i a[i] w^(ik). */
static void cyclic_dft(u64 *a, u64 n, u64 w, u64 q) {
  bit_reverse(a, n);
  for (u64 len = 2; len <= n; len <<= 1) {
    u64 wlen = powmod(w, n / len, q);
    for (u64 i = 0; i < n; i += len) {
      u64 wk = 1;
      for (u64 j = 0; j < len / 2; j++) {
        u64 u = a[i + j];
        u64 v = mulmod(a[i + j + len / 2], wk, q);
        a[i + j] = addmod(u, v, q);
        a[i + j + len / 2] = submod(u, v, q);
        wk = mulmod(wk, wlen, q);
      }
    }
  }
}

/* out[k] = a(psi^(2k+1)) for k in [0, N): twist by psi^i, then cyclic DFT
 * with omega = psi^2. */
void ock_ntt(u64 *a, uint32_t log_n, u64 q) {
  u64 n = (u64)1 << log_n;
  u64 psi = ock_root_2n(q, n);
  u64 pw = 1;
  for (u64 i = 0; i < n; i++) {
    a[i] = mulmod(a[i], pw, q);
    pw = mulmod(pw, psi, q);
  }
  cyclic_dft(a, n, mulmod(psi, psi, q), q);
}

/* Inverse of ock_ntt: inverse cyclic DFT (root omega^-1, times N^-1), then
 * untwist by psi^-i. */
void ock_intt(u64 *a, uint32_t log_n, u64 q) {
  u64 n = (u64)1 << log_n;
  u64 psi = ock_root_2n(q, n);
  u64 psi_inv = invmod(psi, q);
  cyclic_dft(a, n, mulmod(psi_inv, psi_inv, q), q);
  u64 n_inv = invmod(n % q, q);
  u64 pw = n_inv;
  for (u64 i = 0; i < n; i++) {
    a[i] = mulmod(a[i], pw, q);
    pw = mulmod(pw, psi_inv, q);
  }
}

/* out = a * b in Z_q[X]/(X^N + 1), one product per limb.  out may alias. */
void ock_poly_mul(const u64 *a, const u64 *b, u64 *out, uint32_t log_n,
                  const u64 *mods, uint32_t nl) {
  u64 n = (u64)1 << log_n;
#pragma omp parallel for schedule(dynamic)
  for (uint32_t l = 0; l < nl; l++) {
    u64 q = mods[l];
    u64 *ta = (u64 *)malloc(n * sizeof(u64));
    u64 *tb = (u64 *)malloc(n * sizeof(u64));
    memcpy(ta, a + l * n, n * sizeof(u64));
    memcpy(tb, b + l * n, n * sizeof(u64));
    ock_ntt(ta, log_n, q);
    ock_ntt(tb, log_n, q);
    for (u64 i = 0; i < n; i++) ta[i] = mulmod(ta[i], tb[i], q);
    ock_intt(ta, log_n, q);
    memcpy(out + l * n, ta, n * sizeof(u64));
    free(ta);
    free(tb);
  }
}

/* Schoolbook negacyclic product of one limb, O(N^2): the ring's definition,
 * used to pin the NTT product on small rings. */
void ock_poly_mul_schoolbook(const u64 *a, const u64 *b, u64 *out, uint32_t log_n, u64 q) {
  u64 n = (u64)1 << log_n;
  for (u64 k = 0; k < n; k++) out[k] = 0;
  for (u64 i = 0; i < n; i++)
    for (u64 j = 0; j < n; j++) {
      u64 p = mulmod(a[i], b[j], q);
      if (i + j < n)
        out[i + j] = addmod(out[i + j], p, q);
      else
        out[i + j - n] = submod(out[i + j - n], p, q); /* X^N = -1 */
    }
}

void ock_add(const u64 *a, const u64 *b, u64 *out, uint32_t log_n, const u64 *mods,
             uint32_t nl) {
  u64 n = (u64)1 << log_n;
  for (uint32_t l = 0; l < nl; l++)
    for (u64 i = 0; i < n; i++) out[l * n + i] = addmod(a[l * n + i], b[l * n + i], mods[l]);
}

void ock_sub(const u64 *a, const u64 *b, u64 *out, uint32_t log_n, const u64 *mods,
             uint32_t nl) {
  u64 n = (u64)1 << log_n;
  for (uint32_t l = 0; l < nl; l++)
    for (u64 i = 0; i < n; i++) out[l * n + i] = submod(a[l * n + i], b[l * n + i], mods[l]);
}

/* Small signed integers embedded as residues of every limb. */
void ock_embed_small(const int64_t *v, u64 *out, uint32_t log_n, const u64 *mods,
                     uint32_t nl) {
  u64 n = (u64)1 << log_n;
  for (uint32_t l = 0; l < nl; l++) {
    u64 q = mods[l];
    for (u64 i = 0; i < n; i++) {
      int64_t x = v[i];
      u64 mag = (u64)(x < 0 ? -x : x) % q;
      out[l * n + i] = (x < 0) ? (mag ? q - mag : 0) : mag;
    }
  }
}

/* Galois automorphism a(X) -> a(X^g), g odd: coefficient i moves to
 * i*g mod 2N, and picks up a minus sign when that index is >= N. */
void ock_automorphism(const u64 *in, u64 *out, uint32_t log_n, const u64 *mods,
                      uint32_t nl, u64 g) {
  u64 n = (u64)1 << log_n;
  u64 two_n = 2 * n;
  for (uint32_t l = 0; l < nl; l++) {
    u64 q = mods[l];
    for (u64 i = 0; i < n; i++) {
      u64 j = (u64)(((u128)i * g) % two_n);
      u64 x = in[l * n + i];
      if (j < n)
        out[l * n + j] = x;
      else
        out[l * n + j - n] = submod(0, x, q);
    }
  }
}

/* Fast basis conversion of x (residues over src[0..ns)) to one modulus t:
 *   sum_i [x_i * (B/b_i)^-1]_{b_i} * (B/b_i) mod t,   B = prod src.
 * Writes one row of N words.  No overflow correction (the result may exceed
 * the exact residue by a multiple of B, as the definition allows). */
static void bconv_one(const u64 *x, const u64 *src, uint32_t ns, u64 t, u64 *out,
                      u64 n) {
  u64 *hat_inv = (u64 *)malloc(ns * sizeof(u64)); /* (B/b_i)^-1 mod b_i */
  u64 *hat_t = (u64 *)malloc(ns * sizeof(u64));   /* (B/b_i) mod t */
  for (uint32_t i = 0; i < ns; i++) {
    u64 hi = 1, ht = 1;
    for (uint32_t k = 0; k < ns; k++) {
      if (k == i) continue;
      hi = mulmod(hi, src[k] % src[i], src[i]);
      ht = mulmod(ht, src[k] % t, t);
    }
    hat_inv[i] = invmod(hi, src[i]);
    hat_t[i] = ht;
  }
  for (u64 c = 0; c < n; c++) {
    u64 acc = 0;
    for (uint32_t i = 0; i < ns; i++) {
      u64 y = mulmod(x[i * n + c], hat_inv[i], src[i]);
      acc = addmod(acc, mulmod(y % t, hat_t[i], t), t);
    }
    out[c] = acc;
  }
  free(hat_inv);
  free(hat_t);
}

void ock_bconv(const u64 *x, const u64 *src, uint32_t ns, u64 *out, const u64 *dst,
               uint32_t nd, uint32_t log_n) {
  u64 n = (u64)1 << log_n;
#pragma omp parallel for schedule(dynamic)
  for (uint32_t t = 0; t < nd; t++) bconv_one(x, src, ns, dst[t], out + t * n, n);
}

/* ModDown with rounding: u over Q_l (nq limbs) followed by P (np limbs).
 * The integer (P-1)/2 is added to u first, so that the result is
 *   round(u / P) - v  (v in [0, np) from the basis conversion),
 * i.e. per limb
 *   out_i = (u_i + h_i - BConv_{P -> q_i}(u_P + h_P)) * P^-1 mod q_i,
 * with h_m = (P-1)/2 mod m = (P mod m - 1) * 2^-1 mod m. */
void ock_moddown(const u64 *u, u64 *out, const u64 *q, uint32_t nq, const u64 *p,
                 uint32_t np, uint32_t log_n) {
  u64 n = (u64)1 << log_n;
  u64 *up = (u64 *)malloc((size_t)np * n * sizeof(u64));
  for (uint32_t k = 0; k < np; k++) {
    u64 pk = p[k];
    u64 pm = 1;
    for (uint32_t m = 0; m < np; m++) pm = mulmod(pm, p[m] % pk, pk);
    u64 h = mulmod(submod(pm, 1, pk), invmod(2, pk), pk);
    for (u64 c = 0; c < n; c++) up[k * n + c] = addmod(u[((u64)nq + k) * n + c], h, pk);
  }
#pragma omp parallel for schedule(dynamic)
  for (uint32_t i = 0; i < nq; i++) {
    u64 *conv = (u64 *)malloc(n * sizeof(u64));
    bconv_one(up, p, np, q[i], conv, n);
    u64 pm = 1;
    for (uint32_t k = 0; k < np; k++) pm = mulmod(pm, p[k] % q[i], q[i]);
    u64 p_inv = invmod(pm, q[i]);
    u64 h = mulmod(submod(pm, 1, q[i]), invmod(2, q[i]), q[i]);
    for (u64 c = 0; c < n; c++)
      out[i * n + c] =
          mulmod(submod(addmod(u[i * n + c], h, q[i]), conv[c], q[i]), p_inv, q[i]);
    free(conv);
  }
  free(up);
}

/* ModUp of d (coefficient form, limbs 0..level of the q chain) for hybrid
 * key switching: digits are the contiguous blocks D_j = [j*alpha,
 * (j+1)*alpha) of the q chain, alpha = ceil(L/dnum), cut to the limbs present
 * at this level; each present digit is extended by fast basis conversion to
 * every limb of Q_level u P (its own limbs are kept).  ext is laid out
 * [digit][level+1+K][N] (q limbs first, then the special primes); returns the
 * number of digits present. */
uint32_t ock_modup(const u64 *d, uint32_t level, const u64 *q, uint32_t L, const u64 *p,
                   uint32_t K, uint32_t dnum, uint32_t log_n, u64 *ext) {
  u64 n = (u64)1 << log_n;
  uint32_t nq = level + 1;
  uint32_t ne = nq + K;
  uint32_t alpha = (L + dnum - 1) / dnum;
  u64 *mods = (u64 *)malloc(ne * sizeof(u64));
  for (uint32_t t = 0; t < nq; t++) mods[t] = q[t];
  for (uint32_t k = 0; k < K; k++) mods[nq + k] = p[k];
  uint32_t digits = 0;
  for (uint32_t j = 0; j < dnum; j++) {
    uint32_t lo = j * alpha;
    uint32_t hi = (j + 1) * alpha < nq ? (j + 1) * alpha : nq;
    if (lo >= hi) continue;
    digits++;
#pragma omp parallel for schedule(dynamic)
    for (uint32_t t = 0; t < ne; t++) {
      u64 *row = ext + ((u64)j * ne + t) * n;
      if (t >= lo && t < hi)
        memcpy(row, d + (u64)t * n, n * sizeof(u64));
      else
        bconv_one(d + (u64)lo * n, q + lo, hi - lo, mods[t], row, n);
    }
  }
  free(mods);
  return digits;
}

/* Second half of hybrid key switching: given the extended digits (as
 * ock_modup lays them out), u_{0,1} = sum_j ext_j * (b_j, a_j) over
 * Q_level u P with the switching key swk [dnum][2][L+K][N] (rows 0..L-1 for
 * the q chain, L..L+K-1 for the special primes), then ModDown of both sums to
 * Q_level.  Outputs (out0, out1) have level+1 limbs. */
/* Key inner product in Q_level u P: acc_{0,1}[t] = sum_j ext_j[t] * swk_j[t]
 * (negacyclic products per limb; keys [dnum][2][L+K][N], b first), without
 * ModDown.  acc0/acc1 are [level+1+K][N]. */
void ock_ks_inner(const u64 *ext, uint32_t digits, uint32_t level, const u64 *swk,
                  const u64 *q, uint32_t L, const u64 *p, uint32_t K, uint32_t log_n,
                  u64 *acc0, u64 *acc1) {
  u64 n = (u64)1 << log_n;
  uint32_t nq = level + 1;
  uint32_t ne = nq + K;
  u64 *mods = (u64 *)malloc(ne * sizeof(u64));
  for (uint32_t t = 0; t < nq; t++) mods[t] = q[t];
  for (uint32_t k = 0; k < K; k++) mods[nq + k] = p[k];
  memset(acc0, 0, (size_t)ne * n * sizeof(u64));
  memset(acc1, 0, (size_t)ne * n * sizeof(u64));
  for (uint32_t j = 0; j < digits; j++) {
#pragma omp parallel for schedule(dynamic)
    for (uint32_t t = 0; t < ne; t++) {
      u64 *prod = (u64 *)malloc(n * sizeof(u64));
      const u64 *row = ext + ((u64)j * ne + t) * n;
      uint32_t key_row = t < nq ? t : L + (t - nq);
      const u64 *kb = swk + (((u64)j * 2 + 0) * (L + K) + key_row) * n;
      const u64 *ka = swk + (((u64)j * 2 + 1) * (L + K) + key_row) * n;
      ock_poly_mul(row, kb, prod, log_n, &mods[t], 1);
      for (u64 c = 0; c < n; c++) acc0[t * n + c] = addmod(acc0[t * n + c], prod[c], mods[t]);
      ock_poly_mul(row, ka, prod, log_n, &mods[t], 1);
      for (u64 c = 0; c < n; c++) acc1[t * n + c] = addmod(acc1[t * n + c], prod[c], mods[t]);
      free(prod);
    }
  }
  free(mods);
}

/* Inner product of the extended digits with the key, then ModDown of both
 * accumulators to Q_level. */
void ock_keyswitch_ext(const u64 *ext, uint32_t digits, uint32_t level, const u64 *swk,
                       const u64 *q, uint32_t L, const u64 *p, uint32_t K, uint32_t log_n,
                       u64 *out0, u64 *out1) {
  u64 n = (u64)1 << log_n;
  uint32_t ne = level + 1 + K;
  u64 *acc0 = (u64 *)malloc((size_t)ne * n * sizeof(u64));
  u64 *acc1 = (u64 *)malloc((size_t)ne * n * sizeof(u64));
  ock_ks_inner(ext, digits, level, swk, q, L, p, K, log_n, acc0, acc1);
  ock_moddown(acc0, out0, q, level + 1, p, K, log_n);
  ock_moddown(acc1, out1, q, level + 1, p, K, log_n);
  free(acc0);
  free(acc1);
}

/* Hybrid key switching of d: ModUp, then inner product and ModDown. */
void ock_keyswitch(const u64 *d, uint32_t level, const u64 *swk, const u64 *q, uint32_t L,
                   const u64 *p, uint32_t K, uint32_t dnum, uint32_t log_n, u64 *out0,
                   u64 *out1) {
  u64 n = (u64)1 << log_n;
  uint32_t ne = level + 1 + K;
  u64 *ext = (u64 *)malloc((size_t)dnum * ne * n * sizeof(u64));
  uint32_t digits = ock_modup(d, level, q, L, p, K, dnum, log_n, ext);
  ock_keyswitch_ext(ext, digits, level, swk, q, L, p, K, log_n, out0, out1);
  free(ext);
}

/* Rescale one polynomial of nq = level+1 limbs by the last prime ql:
 * t = centred lift of the last limb into (-ql/2, ql/2);
 * out_i = (c_i - t) * ql^-1 mod q_i for i < level. */
void ock_rescale(const u64 *c, u64 *out, const u64 *q, uint32_t level, uint32_t log_n) {
  u64 n = (u64)1 << log_n;
  u64 ql = q[level];
#pragma omp parallel for schedule(dynamic)
  for (uint32_t i = 0; i < level; i++) {
    u64 qi = q[i];
    u64 ql_inv = invmod(ql % qi, qi);
    for (u64 k = 0; k < n; k++) {
      u64 v = c[(u64)level * n + k];
      u64 t; /* centred lift of v, reduced mod q_i */
      if (v <= (ql - 1) / 2)
        t = v % qi;
      else
        t = submod(v % qi, ql % qi, qi); /* v - ql < 0 */
      out[i * n + k] = mulmod(submod(c[i * n + k], t, qi), ql_inv, qi);
    }
  }
}

#ifdef _OPENMP
#include <omp.h>
int ock_num_threads(void) { return omp_get_max_threads(); }
/* threads of the limb loops from now on (timing at one thread and at all) */
void ock_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
int ock_num_threads(void) { return 1; }
void ock_set_num_threads(int n) { (void)n; }
#endif
