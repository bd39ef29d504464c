// Randomness for key generation and encryption: SHAKE-256 (FIPS 202) streams.
//
// The paper's client runs KeyGen and encryption (section 3.2); the scheme
// needs a uniform polynomial per limb, a ternary secret and small Gaussian
// errors.  Every draw reads a SHAKE-256 stream keyed by
//   "hipckks/" || tag || "/" || le64(seed) || le32(index),
// so keys and ciphertexts are reproducible from their seeds:
//   * uniform mod q: 64-bit little-endian words masked to bitlen(q) bits,
//     kept when below q (stream index = limb index);
//   * ternary: bytes, 255 rejected, b mod 3 -> 0, +1, -1;
//   * Gaussian (sigma = 3.2, |e| <= 19): a 64-bit word w; u = w >> 1 selects
//     the magnitude as the first k with u < T[k], T[k] = floor(2^63 P(|e| <= k));
//     bit 0 of w is the sign (magnitude 0 is never negated).
//
// Keccak-f[1600] is written from FIPS 202: the round constants come from the
// rc() LFSR of its Algorithm 5 and the rho offsets from the (t+1)(t+2)/2 walk
// of its Algorithm 2, both computed here rather than tabulated.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace hck {

namespace {

inline uint64_t rotl(uint64_t x, unsigned r) { return r == 0 ? x : (x << r) | (x >> (64 - r)); }

// rc(t) of FIPS 202 Algorithm 5.
int rc_bit(int t) {
  if (t % 255 == 0) return 1;
  unsigned r = 0x01;  // R[0] = 1 (bit i of r is R[i])
  for (int i = 1; i <= t % 255; i++) {
    r <<= 1;  // R = 0 || R
    const unsigned r8 = (r >> 8) & 1;
    r ^= r8 | (r8 << 4) | (r8 << 5) | (r8 << 6);
    r &= 0xFF;
  }
  return r & 1;
}

struct KeccakTables {
  uint64_t rc[24];
  unsigned rho[25];  // lane index x + 5 y
  KeccakTables() {
    for (int ir = 0; ir < 24; ir++) {
      uint64_t v = 0;
      for (int j = 0; j <= 6; j++)
        if (rc_bit(j + 7 * ir)) v |= 1ull << ((1u << j) - 1);
      rc[ir] = v;
    }
    rho[0] = 0;
    int x = 1, y = 0;
    for (int t = 0; t < 24; t++) {
      rho[x + 5 * y] = (unsigned)(((t + 1) * (t + 2) / 2) % 64);
      const int nx = y, ny = (2 * x + 3 * y) % 5;
      x = nx;
      y = ny;
    }
  }
};

const KeccakTables &tables() {
  static const KeccakTables t;
  return t;
}

void keccak_f1600(uint64_t a[25]) {
  const KeccakTables &kt = tables();
  for (int round = 0; round < 24; round++) {
    uint64_t c[5], d[5], b[25];
    for (int x = 0; x < 5; x++) c[x] = a[x] ^ a[x + 5] ^ a[x + 10] ^ a[x + 15] ^ a[x + 20];
    for (int x = 0; x < 5; x++) d[x] = c[(x + 4) % 5] ^ rotl(c[(x + 1) % 5], 1);
    for (int i = 0; i < 25; i++) a[i] ^= d[i % 5];
    // rho and pi: B[y, 2x + 3y] = rot(A[x, y], r[x, y])
    for (int x = 0; x < 5; x++)
      for (int y = 0; y < 5; y++) b[y + 5 * ((2 * x + 3 * y) % 5)] = rotl(a[x + 5 * y], kt.rho[x + 5 * y]);
    // chi
    for (int y = 0; y < 5; y++)
      for (int x = 0; x < 5; x++)
        a[x + 5 * y] = b[x + 5 * y] ^ (~b[(x + 1) % 5 + 5 * y] & b[(x + 2) % 5 + 5 * y]);
    // iota
    a[0] ^= kt.rc[round];
  }
}

constexpr size_t kRate = 136;  // SHAKE256: 1600 - 2 * 256 bits

// Incremental SHAKE-256 squeezer.
class Shake256 {
 public:
  explicit Shake256(const std::vector<uint8_t> &msg) {
    std::memset(st_, 0, sizeof(st_));
    size_t off = 0;
    while (msg.size() - off >= kRate) {
      absorb_block(msg.data() + off);
      off += kRate;
    }
    uint8_t last[kRate];
    std::memset(last, 0, kRate);
    if (msg.size() > off) std::memcpy(last, msg.data() + off, msg.size() - off);
    last[msg.size() - off] ^= 0x1F;  // SHAKE domain bits 1111 then pad10*1's first 1
    last[kRate - 1] ^= 0x80;         // pad10*1's final 1
    absorb_block(last);
    pos_ = 0;
    fill();
  }
  void squeeze(uint8_t *out, size_t len) {
    while (len) {
      if (pos_ == kRate) {
        keccak_f1600(st_);
        fill();
        pos_ = 0;
      }
      const size_t take = std::min(len, kRate - pos_);
      std::memcpy(out, buf_ + pos_, take);
      out += take;
      len -= take;
      pos_ += take;
    }
  }

 private:
  void absorb_block(const uint8_t *blk) {
    for (size_t i = 0; i < kRate / 8; i++) {
      uint64_t lane = 0;
      for (int b = 0; b < 8; b++) lane |= (uint64_t)blk[8 * i + b] << (8 * b);
      st_[i] ^= lane;
    }
    keccak_f1600(st_);
  }
  void fill() {
    for (size_t i = 0; i < kRate / 8; i++)
      for (int b = 0; b < 8; b++) buf_[8 * i + b] = (uint8_t)(st_[i] >> (8 * b));
  }
  uint64_t st_[25];
  uint8_t buf_[kRate];
  size_t pos_ = 0;
};

std::vector<uint8_t> stream_key(const std::string &tag, uint64_t seed, uint32_t index) {
  std::string pre = "hipckks/" + tag + "/";
  std::vector<uint8_t> msg(pre.begin(), pre.end());
  for (int b = 0; b < 8; b++) msg.push_back((uint8_t)(seed >> (8 * b)));
  for (int b = 0; b < 4; b++) msg.push_back((uint8_t)(index >> (8 * b)));
  return msg;
}

struct Cdt {
  uint64_t t[20];
  Cdt() {
    const long double sigma = 3.2L;
    long double mass[20], total = 0;
    for (int k = 0; k < 20; k++) {
      const long double rho = expl(-(long double)(k * k) / (2 * sigma * sigma));
      mass[k] = k == 0 ? rho : 2 * rho;
      total += mass[k];
    }
    long double acc = 0;
    for (int k = 0; k < 19; k++) {
      acc += mass[k];
      t[k] = (uint64_t)floorl(acc / total * 9223372036854775808.0L);
    }
    t[19] = 1ull << 63;
  }
};

}  // namespace

void shake256(const uint8_t *msg, size_t len, uint8_t *out, size_t outlen) {
  Shake256 s(std::vector<uint8_t>(msg, msg + len));
  s.squeeze(out, outlen);
}

std::vector<uint8_t> shake_stream(const std::string &tag, uint64_t seed, uint32_t index,
                                  size_t nbytes) {
  std::vector<uint8_t> out(nbytes);
  Shake256 s(stream_key(tag, seed, index));
  s.squeeze(out.data(), nbytes);
  return out;
}

void sample_uniform(const std::string &tag, uint64_t seed, uint32_t index, uint64_t q,
                    uint64_t *out, size_t n) {
  Shake256 s(stream_key(tag, seed, index));
  unsigned bits = 64 - __builtin_clzll(q);
  const uint64_t mask = bits == 64 ? ~0ull : ((1ull << bits) - 1);
  size_t got = 0;
  uint8_t w[8 * 64];
  while (got < n) {
    s.squeeze(w, sizeof(w));
    for (int k = 0; k < 64 && got < n; k++) {
      uint64_t v = 0;
      for (int b = 0; b < 8; b++) v |= (uint64_t)w[8 * k + b] << (8 * b);
      v &= mask;
      if (v < q) out[got++] = v;
    }
  }
}

void sample_ternary(const std::string &tag, uint64_t seed, int32_t *out, size_t n) {
  Shake256 s(stream_key(tag, seed, 0));
  size_t got = 0;
  uint8_t buf[256];
  while (got < n) {
    s.squeeze(buf, sizeof(buf));
    for (size_t k = 0; k < sizeof(buf) && got < n; k++) {
      if (buf[k] == 255) continue;
      const int r = buf[k] % 3;
      out[got++] = r == 2 ? -1 : r;
    }
  }
}

void sample_gaussian(const std::string &tag, uint64_t seed, int32_t *out, size_t n) {
  static const Cdt cdt;
  Shake256 s(stream_key(tag, seed, 0));
  uint8_t w[8];
  for (size_t i = 0; i < n; i++) {
    s.squeeze(w, 8);
    uint64_t v = 0;
    for (int b = 0; b < 8; b++) v |= (uint64_t)w[b] << (8 * b);
    const uint64_t u = v >> 1;
    int mag = 0;
    while (mag < 19 && u >= cdt.t[mag]) mag++;
    out[i] = ((v & 1) && mag) ? -mag : mag;
  }
}

}  // namespace hck

extern "C" {

/* Host utilities of the client side (no context, no device). */
int hck_shake256(const uint8_t *msg, size_t len, uint8_t *out, size_t outlen) {
  if ((!msg && len) || (!out && outlen)) return hck::set_error(HCK_EINVAL, "null buffer");
  hck::shake256(msg, len, out, outlen);
  return HCK_OK;
}

int hck_sample_uniform(const char *tag, uint64_t seed, uint32_t index, uint64_t q, uint64_t *out,
                       size_t n) {
  if (!tag || !out || q < 2) return hck::set_error(HCK_EINVAL, "bad argument");
  hck::sample_uniform(tag, seed, index, q, out, n);
  return HCK_OK;
}

int hck_sample_ternary(const char *tag, uint64_t seed, int32_t *out, size_t n) {
  if (!tag || !out) return hck::set_error(HCK_EINVAL, "bad argument");
  hck::sample_ternary(tag, seed, out, n);
  return HCK_OK;
}

int hck_sample_gaussian(const char *tag, uint64_t seed, int32_t *out, size_t n) {
  if (!tag || !out) return hck::set_error(HCK_EINVAL, "bad argument");
  hck::sample_gaussian(tag, seed, out, n);
  return HCK_OK;
}

}  // extern "C"
