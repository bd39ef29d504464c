// Canonical-embedding encoder and CRT decoder (host side; the paper's client
// encodes and decodes, section 3.2 "Encoding and Batching", section 3.3.4).
//
// Slot j is the value of the real polynomial m at zeta^(5^j mod 2N), zeta =
// exp(i pi / N).  Writing E[k] = m(zeta^(2k+1)) for all odd powers,
//   E[k] = sum_i (m_i zeta^i) w^(ik),   w = exp(2 pi i / N),
// so encoding fills E (slot values at k = (5^j - 1)/2 and their conjugates at
// N - 1 - k, which makes m real) and inverts this DFT; decoding evaluates it.
// The DFT is an iterative radix-2 complex FFT with twiddles taken from
// cos/sin directly.
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "internal.h"

namespace hck {

namespace {

using cd = std::complex<double>;

// In-place FFT of length n (power of two): a[k] <- sum_i a[i] exp(sign 2 pi i ik / n).
void fft(std::vector<cd> &a, int sign) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; i++) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    const size_t half = len / 2;
    std::vector<cd> w(half);
    for (size_t k = 0; k < half; k++) {
      const double ang = sign * 2.0 * M_PI * (double)k / (double)len;
      w[k] = cd(std::cos(ang), std::sin(ang));
    }
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < half; k++) {
        const cd u = a[i + k], v = a[i + k + half] * w[k];
        a[i + k] = u + v;
        a[i + k + half] = u - v;
      }
  }
}

std::vector<size_t> slot_positions(uint32_t log_n) {
  const uint64_t n = 1ull << log_n, two_n = 2 * n;
  std::vector<size_t> pos(n / 2);
  uint64_t e = 1;
  for (size_t j = 0; j < n / 2; j++) {
    pos[j] = (size_t)((e - 1) / 2);
    e = e * 5 % two_n;
  }
  return pos;
}

cd zeta_pow(uint64_t i, uint64_t n) {
  const double ang = M_PI * (double)i / (double)n;
  return cd(std::cos(ang), std::sin(ang));
}

// Small fixed-width unsigned big integers (little-endian 64-bit words).
struct Big {
  std::vector<uint64_t> w;
};

void big_mul_add(std::vector<uint64_t> &acc, const std::vector<uint64_t> &b, uint64_t m) {
  unsigned __int128 carry = 0;
  for (size_t i = 0; i < acc.size(); i++) {
    unsigned __int128 t = (unsigned __int128)(i < b.size() ? b[i] : 0) * m + acc[i] + carry;
    acc[i] = (uint64_t)t;
    carry = t >> 64;
  }
}

int big_cmp(const std::vector<uint64_t> &a, const std::vector<uint64_t> &b) {
  for (size_t i = a.size(); i-- > 0;) {
    const uint64_t bi = i < b.size() ? b[i] : 0;
    if (a[i] != bi) return a[i] < bi ? -1 : 1;
  }
  return 0;
}

void big_sub(std::vector<uint64_t> &a, const std::vector<uint64_t> &b) {
  uint64_t borrow = 0;
  for (size_t i = 0; i < a.size(); i++) {
    const uint64_t bi = i < b.size() ? b[i] : 0;
    const uint64_t t = a[i] - bi - borrow;
    borrow = (a[i] < bi || (a[i] == bi && borrow)) ? 1 : 0;
    a[i] = t;
  }
}

double big_to_double(const std::vector<uint64_t> &a) {
  double r = 0;
  for (size_t i = a.size(); i-- > 0;) r = r * 18446744073709551616.0 + (double)a[i];
  return r;
}

}  // namespace

int encode_coeffs(uint32_t log_n, const double *re, const double *im, double scale,
                  std::vector<int64_t> &coeffs) {
  const size_t n = (size_t)1 << log_n;
  const std::vector<size_t> pos = slot_positions(log_n);
  std::vector<cd> e(n);
  for (size_t j = 0; j < n / 2; j++) {
    const cd z(re[j], im ? im[j] : 0.0);
    e[pos[j]] = z;
    e[n - 1 - pos[j]] = std::conj(z);
  }
  fft(e, -1);
  coeffs.assign(n, 0);
  for (size_t i = 0; i < n; i++) {
    const double v = (e[i] / (double)n * std::conj(zeta_pow(i, n))).real() * scale;
    const double r = v < 0 ? -std::floor(-v + 0.5) : std::floor(v + 0.5);
    if (!(std::fabs(r) < 4611686018427387904.0))  // 2^62
      return set_error(HCK_EINVAL, "encoded coefficient exceeds 2^62");
    coeffs[i] = (int64_t)r;
  }
  return HCK_OK;
}

void decode_residues(uint32_t log_n, const uint64_t *res, const uint64_t *mods, uint32_t nl,
                     double scale, double *re, double *im) {
  const size_t n = (size_t)1 << log_n;
  // Q and Q / q_i as big integers; (Q / q_i)^-1 mod q_i
  const size_t words = nl + 2;
  std::vector<uint64_t> big_q(words, 0);
  big_q[0] = 1;
  for (uint32_t i = 0; i < nl; i++) {
    std::vector<uint64_t> t(words, 0);
    big_mul_add(t, big_q, mods[i]);
    big_q = t;
  }
  std::vector<std::vector<uint64_t>> hat(nl, std::vector<uint64_t>(words, 0));
  std::vector<uint64_t> hat_inv(nl);
  for (uint32_t i = 0; i < nl; i++) {
    hat[i][0] = 1;
    uint64_t r = 1;
    for (uint32_t k = 0; k < nl; k++) {
      if (k == i) continue;
      std::vector<uint64_t> t(words, 0);
      big_mul_add(t, hat[i], mods[k]);
      hat[i] = t;
      r = h_mulmod(r, mods[k] % mods[i], mods[i]);
    }
    hat_inv[i] = h_invmod(r, mods[i]);
  }
  std::vector<uint64_t> half_q = big_q;  // floor(Q / 2)
  for (size_t i = 0; i < words; i++)
    half_q[i] = (half_q[i] >> 1) | (i + 1 < words ? half_q[i + 1] << 63 : 0);
  std::vector<double> m(n);
  std::vector<uint64_t> acc(words);
  for (size_t c = 0; c < n; c++) {
    std::fill(acc.begin(), acc.end(), 0);
    for (uint32_t i = 0; i < nl; i++)
      big_mul_add(acc, hat[i], h_mulmod(res[(size_t)i * n + c], hat_inv[i], mods[i]));
    while (big_cmp(acc, big_q) >= 0) big_sub(acc, big_q);
    if (big_cmp(acc, half_q) > 0) {
      std::vector<uint64_t> neg = big_q;
      big_sub(neg, acc);
      m[c] = -big_to_double(neg);
    } else {
      m[c] = big_to_double(acc);
    }
  }
  std::vector<cd> e(n);
  for (size_t i = 0; i < n; i++) e[i] = (m[i] / scale) * zeta_pow(i, n);
  fft(e, +1);
  const std::vector<size_t> pos = slot_positions(log_n);
  for (size_t j = 0; j < n / 2; j++) {
    if (re) re[j] = e[pos[j]].real();
    if (im) im[j] = e[pos[j]].imag();
  }
}

}  // namespace hck

extern "C" {

/* Host utilities of the client side (no context, no device). */
int hck_encode_coeffs(uint32_t log_n, const double *re, const double *im, double scale,
                      int64_t *coeffs) {
  if (!re || !coeffs || log_n < 2 || log_n > 17) return hck::set_error(HCK_EINVAL, "bad argument");
  std::vector<int64_t> c;
  int rc = hck::encode_coeffs(log_n, re, im, scale, c);
  if (rc) return rc;
  std::memcpy(coeffs, c.data(), c.size() * sizeof(int64_t));
  return HCK_OK;
}

int hck_decode_residues(uint32_t log_n, const uint64_t *res, const uint64_t *mods, uint32_t nl,
                        double scale, double *re, double *im) {
  if (!res || !mods || nl == 0 || nl > HCK_MAX_LIMBS || log_n < 2 || log_n > 17)
    return hck::set_error(HCK_EINVAL, "bad argument");
  hck::decode_residues(log_n, res, mods, nl, scale, re, im);
  return HCK_OK;
}

}  // extern "C"
