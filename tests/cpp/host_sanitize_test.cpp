// The library's host-only client code (SHAKE-256, the samplers, the encoder
// and the residue decoder) run under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Prints every result as text; the Python test
// compares it with the same calls in the normal build of the library.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "hipckks.h"

// error reporting of the library (context.cpp is not part of this program)
namespace hck {
int set_error(int code, const std::string &) { return code; }
}  // namespace hck

static uint64_t lcg(uint64_t &s) {
  s = s * 6364136223846793005ull + 1442695040888963407ull;
  return s >> 11;
}

// argv[1..3]: three distinct primes (the decoder's CRT basis; the first is
// also the uniform sampler's modulus)
int main(int argc, char **argv) {
  if (argc != 4) return 2;
  const uint64_t mods[3] = {std::strtoull(argv[1], nullptr, 10),
                            std::strtoull(argv[2], nullptr, 10),
                            std::strtoull(argv[3], nullptr, 10)};
  // SHAKE-256 of messages across the 136-byte rate
  for (size_t len : {0, 1, 135, 136, 137, 300}) {
    std::vector<uint8_t> msg(len);
    for (size_t i = 0; i < len; i++) msg[i] = (uint8_t)(i * 7 + 3);
    std::vector<uint8_t> out(200);
    if (hck_shake256(msg.data(), len, out.data(), out.size())) return 1;
    std::printf("shake %zu ", len);
    for (uint8_t b : out) std::printf("%02x", b);
    std::printf("\n");
  }
  // samplers
  const uint64_t q = mods[0];
  std::vector<uint64_t> u(1000);
  if (hck_sample_uniform("san", 7, 3, q, u.data(), u.size())) return 1;
  std::printf("uniform");
  for (uint64_t x : u) std::printf(" %llu", (unsigned long long)x);
  std::printf("\n");
  std::vector<int32_t> t(1000), g(1000);
  if (hck_sample_ternary("san", 8, t.data(), t.size())) return 1;
  if (hck_sample_gaussian("san", 9, g.data(), g.size())) return 1;
  std::printf("ternary");
  for (int32_t x : t) std::printf(" %d", x);
  std::printf("\ngaussian");
  for (int32_t x : g) std::printf(" %d", x);
  std::printf("\n");
  // encoder and decoder on rings 2^4 .. 2^12
  uint64_t s = 12345;
  for (uint32_t log_n = 4; log_n <= 12; log_n += 4) {
    const size_t n = (size_t)1 << log_n, slots = n / 2;
    std::vector<double> re(slots), im(slots);
    for (size_t i = 0; i < slots; i++) {
      re[i] = (double)(lcg(s) % 2000001) / 1e6 - 1.0;
      im[i] = (double)(lcg(s) % 2000001) / 1e6 - 1.0;
    }
    std::vector<int64_t> c(n);
    if (hck_encode_coeffs(log_n, re.data(), im.data(), 1099511627776.0, c.data())) return 1;
    std::printf("encode %u", log_n);
    for (int64_t x : c) std::printf(" %lld", (long long)x);
    std::printf("\n");
    std::vector<uint64_t> res(3 * n);
    for (int l = 0; l < 3; l++)
      for (size_t i = 0; i < n; i++) {
        const int64_t v = c[i];
        res[l * n + i] = v < 0 ? mods[l] - (uint64_t)(-v) % mods[l] : (uint64_t)v % mods[l];
      }
    std::vector<double> dre(slots), dim(slots);
    if (hck_decode_residues(log_n, res.data(), mods, 3, 1099511627776.0, dre.data(),
                            dim.data()))
      return 1;
    std::printf("decode %u", log_n);
    for (size_t i = 0; i < slots; i++) std::printf(" %.17g %.17g", dre[i], dim[i]);
    std::printf("\n");
  }
  // argument checks return errors without touching memory
  if (hck_sample_uniform(nullptr, 0, 0, q, u.data(), 1) == 0) return 1;
  if (hck_encode_coeffs(1, nullptr, nullptr, 1.0, nullptr) == 0) return 1;
  std::printf("all checks passed\n");
  return 0;
}
