// Modular arithmetic for residues below 2^61 on gfx950.
//
// Every 64x64-bit product is built from v_mad_u64_u32 (32x32+64 -> 64),
// which issues at full rate on CDNA4; the plain C++ forms would be lowered to
// v_mul_lo_u32 / v_mul_hi_u32, which issue at half rate.  Inline asm keeps the
// full-rate instruction (the carry-out SGPR pair is unused).
//
// Reduction schemes:
//   * Shoup, for a known constant w < q with w' = floor(w 2^64 / q):
//       a w mod q = a w - floor(a w' / 2^64) q   in [0, 2q) for any a < 2^64;
//   * Montgomery REDC for a 128-bit T < q 2^64 with qinv = q^-1 mod 2^64:
//       REDC(T) = T 2^-64 mod q  in [0, q);
//     used where a sum of products is reduced once (basis conversion, key
//     inner product): multiplying one factor by 2^64 mod q beforehand cancels
//     the 2^-64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hck {

struct u128 {
  uint64_t lo, hi;
};

#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ uint64_t mad32(uint32_t a, uint32_t b, uint64_t c) {
  uint64_t d;
  uint64_t carry;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(d), "=s"(carry) : "v"(a), "v"(b), "v"(c));
  return d;
}
#else
__host__ inline uint64_t mad32(uint32_t a, uint32_t b, uint64_t c) {
  return (uint64_t)a * b + c;
}
#endif

// High 64 bits of a * b.
__host__ __device__ __forceinline__ uint64_t mul_hi(uint64_t a, uint64_t b) {
  uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  uint64_t p00 = mad32(a0, b0, 0);
  uint64_t p01 = mad32(a0, b1, p00 >> 32);
  uint64_t p10 = mad32(a1, b0, (uint32_t)p01);
  return mad32(a1, b1, (p01 >> 32) + (p10 >> 32));
}

// Low 64 bits of a * b.
__host__ __device__ __forceinline__ uint64_t mul_lo(uint64_t a, uint64_t b) {
  uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  uint64_t p00 = mad32(a0, b0, 0);
  uint64_t h = mad32(a0, b1, p00 >> 32);
  h = mad32(a1, b0, h);
  return (h << 32) | (uint32_t)p00;
}

// Full 128-bit product.
__host__ __device__ __forceinline__ u128 mul_wide(uint64_t a, uint64_t b) {
  uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  uint64_t p00 = mad32(a0, b0, 0);
  uint64_t p01 = mad32(a0, b1, p00 >> 32);
  uint64_t p10 = mad32(a1, b0, (uint32_t)p01);
  uint64_t p11 = mad32(a1, b1, (p01 >> 32) + (p10 >> 32));
  u128 r;
  r.lo = (p10 << 32) | (uint32_t)p00;
  r.hi = p11;
  return r;
}

// acc += a * b (128-bit accumulate; the caller bounds the sum below 2^128).
__host__ __device__ __forceinline__ void mac_wide(u128 &acc, uint64_t a, uint64_t b) {
  u128 p = mul_wide(a, b);
  uint64_t lo = acc.lo + p.lo;
  acc.hi += p.hi + (lo < p.lo ? 1 : 0);
  acc.lo = lo;
}

// a w mod q in [0, 2q), for any a < 2^64 and q < 2^63.
__host__ __device__ __forceinline__ uint64_t shoup_lazy(uint64_t a, uint64_t w, uint64_t wp,
                                                        uint64_t q) {
  return mul_lo(a, w) - mul_lo(mul_hi(a, wp), q);
}

__host__ __device__ __forceinline__ uint64_t reduce2(uint64_t a, uint64_t q) {
  return a >= q ? a - q : a;
}

// a w mod q in [0, q).
__host__ __device__ __forceinline__ uint64_t shoup(uint64_t a, uint64_t w, uint64_t wp,
                                                   uint64_t q) {
  return reduce2(shoup_lazy(a, w, wp, q), q);
}

// T 2^-64 mod q in [0, q) for T < q 2^64.
__host__ __device__ __forceinline__ uint64_t redc(u128 t, uint64_t q, uint64_t qinv) {
  uint64_t m = mul_lo(t.lo, qinv);
  uint64_t mh = mul_hi(m, q);
  // T - m q has a zero low word, so its high word is t.hi - mh (no borrow).
  return t.hi >= mh ? t.hi - mh : t.hi + q - mh;
}

__host__ __device__ __forceinline__ uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {
  uint64_t s = a + b;
  return s >= q ? s - q : s;
}

__host__ __device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) {
  return a >= b ? a - b : a + q - b;
}

// ---- host-side constant helpers (exact, via unsigned __int128) -----------

inline uint64_t h_mulmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)((unsigned __int128)a * b % q);
}

inline uint64_t h_powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = h_mulmod(r, a, q);
    a = h_mulmod(a, a, q);
  }
  return r;
}

// Inverse modulo a prime.
inline uint64_t h_invmod(uint64_t a, uint64_t q) { return h_powmod(a % q, q - 2, q); }

// floor(w 2^64 / q), the Shoup companion of w < q.
inline uint64_t h_shoup(uint64_t w, uint64_t q) {
  return (uint64_t)(((unsigned __int128)w << 64) / q);
}

// q^-1 mod 2^64 for odd q (Newton iteration, 6 doublings of precision).
inline uint64_t h_inv64(uint64_t q) {
  uint64_t x = q;  // correct to 3 bits for odd q
  for (int i = 0; i < 6; i++) x *= 2 - q * x;
  return x;
}

// 2^64 mod q.
inline uint64_t h_r64(uint64_t q) { return (uint64_t)(((unsigned __int128)1 << 64) % q); }

}  // namespace hck
