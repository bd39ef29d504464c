// Register-blocked NTT pass stages shared by the plain and fused kernels.
//
// Forward transform: the merged Cooley-Tukey network whose stage m (m = 1, 2,
// ..., N/2; half-width t = N / 2m) combines x[j], x[j+t] with the twiddle
// psi^brv(m + j / 2t), psi a primitive 2N-th root of unity and brv the logN-bit
// reversal.  Slot j of the output holds the polynomial's value at
// psi^(2 brv(j) + 1) (bit-reversed evaluation order).  The inverse runs the
// Gentleman-Sande network with psi^-brv in the reverse stage order.
//
// A limb of N 64-bit words (512 KiB at N = 2^16) exceeds one CU's LDS, so a
// transform is two passes over memory, N = R1 x R2:
//   * strided pass: stages m < R1 touch only elements R2 apart, so the R2
//     columns (stride R2) are independent R1-point transforms;
//   * contiguous pass: stages m >= R1 stay inside the R1 blocks of R2
//     contiguous words, independent R2-point transforms.
// In a pass a thread owns P = 2^ceil(log2(R)/2) points of one R-point
// sub-transform and T = R/P threads share it:
//   interleaved layout: thread r holds points r + T i (i < P); the first
//     log2(P) stages pair registers i and i + h;
//   blocked layout: thread r holds points r P + v (v < P); the remaining
//     stages (half-width < T <= P) pair registers v and v + t.
// One LDS exchange switches layouts.
//
// The contiguous pass's sub-transform g (words g R2 .. g R2 + R2 - 1) would
// need its own twiddles: the twiddle of its stage s and group grp is
// psi^brv(2^(a+s) + g 2^s + grp) (a = log2 R1), which factors as sub-transform
// 0's twiddle times beta_g^(R2 / 2^(s+1)), beta_g = psi^(2 brv_a(g)).  So
// every sub-transform runs sub-transform 0's network on its input twisted
// by x_i <- x_i beta_g^i: by induction over the stages the values entering
// stage s are the untwisted ones times beta_g^(i mod R2/2^s), and after the
// last stage the factor is 1, so the outputs are the same residues.  The
// inverse network is untwisted at its end (x_i beta_g^-i).  A twist is one
// coalesced table read and one Shoup product per point; the butterflies'
// twiddles then depend on the stage and group only (uniform across the
// wavefront in the interleaved stages, a handful of cached words in the
// blocked ones) instead of one scattered load per butterfly.  Global accesses are coalesced in the
// interleaved layout for the contiguous pass and in either layout for the
// strided pass (adjacent threads own adjacent columns).  Butterflies are
// Harvey's lazy ones (values in [0, 4q) forward, [0, 2q) inverse, q < 2^61)
// with Shoup twiddle products.
#pragma once
#include "internal.h"

namespace hck {

constexpr int kNttThreads = 256;

__device__ __forceinline__ Qn qn(const ModConst &m) { return Qn{m.q, m.nq}; }

__device__ __forceinline__ void ct_bfly(uint64_t &x, uint64_t &y, uint64_t w, uint64_t wp,
                                        Qn m) {
  const uint64_t q2 = 2 * m.q;
  uint64_t a = csub(x, q2, 2 * m.nq);      // [0, 2q)
  uint64_t t = shoup_lazy(y, w, wp, m);    // [0, 2q)
  x = a + t;                               // [0, 4q)
  y = a - t + q2;                          // (0, 4q)
}

__device__ __forceinline__ void gs_bfly(uint64_t &x, uint64_t &y, uint64_t w, uint64_t wp,
                                        Qn m) {
  const uint64_t q2 = 2 * m.q;
  const uint64_t s = csub(x + y, q2, 2 * m.nq);  // [0, 2q)
  y = shoup_lazy(x - y + q2, w, wp, m);          // [0, 2q)
  x = s;
}

// Geometry of one pass: R-point sub-transforms of an N-point limb.
template <int LOGR, int LOGN, bool STRIDED>
struct Pass {
  static constexpr int R = 1 << LOGR;
  static constexpr int LOGP = (LOGR + 1) / 2;
  static constexpr int P = 1 << LOGP;
  static constexpr int T = R / P;                 // threads per sub-transform
  static constexpr int TR = kNttThreads / T;      // sub-transforms per workgroup
  static constexpr int N = 1 << LOGN;
  static constexpr int OTHER = N / R;             // sub-transforms per limb
  static constexpr int S = R + R / P + 1;         // LDS words per sub-transform
  static constexpr int LDS_WORDS = TR * S;
  static constexpr int BLOCKS = OTHER / TR;       // workgroups per limb

  __device__ static int lidx(int c, int p) { return c * S + p + (p >> LOGP); }
  // word offset in the limb of point p of sub-transform g
  __device__ static size_t gaddr(int g, int p) {
    return STRIDED ? (size_t)p * OTHER + g : (size_t)g * R + p;
  }
  __device__ static int sub(int tid) { return STRIDED ? tid % TR : tid / T; }
  __device__ static int lane(int tid) { return STRIDED ? tid / TR : tid % T; }
  // point held in register i (interleaved) / v (blocked)
  __device__ static int ipoint(int r, int i) { return r + T * i; }
  __device__ static int bpoint(int r, int v) { return r * P + v; }
  // global twiddle index of pass stage s for the butterfly with top point p
  // (the contiguous pass uses sub-transform 0's twiddles for every g, on
  // twisted inputs)
  __device__ static int tw(int s, int g, int p) {
    const int grp = p >> (LOGR - s);
    return STRIDED ? (1 << s) + grp : (1 << s) * OTHER + grp;
  }

  // the same for the interleaved stages (s < LOGP), where a thread's point
  // r + T i with r < T gives grp = i >> (LOGP - s): a compile-time index,
  // the same for every lane, so the twiddle comes through the scalar cache
  __device__ static constexpr int tw_interleaved(int s, int i) {
    return (STRIDED ? (1 << s) : (1 << s) * OTHER) + (i >> (LOGP - s));
  }

  // contiguous pass, interleaved layout: x_i <- x_i t[i] (t: the limb's twist
  // or inverse-twist table, indexed like the data), for any x_i < 2^64;
  // results in [0, 2q)
  __device__ static void twist(uint64_t (&x)[P], int g, int r, const uint64_t *t,
                               const uint64_t *ts, Qn q) {
    static_assert(!STRIDED, "twists belong to the contiguous pass");
#pragma unroll
    for (int i = 0; i < P; i++) {
      const size_t a = gaddr(g, ipoint(r, i));
      x[i] = shoup_lazy(x[i], t[a], ts[a], q);
    }
  }

  // A layout switch exchanges values among the T threads of one
  // sub-transform through its own LDS rows.  In the contiguous pass those
  // threads are consecutive and T divides 64, so they share one wavefront:
  // a wavefront-scope fence keeps the compiler from moving the LDS reads
  // above the writes (or the next writes above the reads), and a wavefront's
  // LDS operations complete in issue order, so no workgroup barrier is
  // needed.  The strided pass spreads a sub-transform over the workgroup.
  static_assert(STRIDED || (T <= 64 && 64 % T == 0), "sub-transform must fit one wavefront");
  __device__ static void exchange_sync() {
    if constexpr (STRIDED) {
      __syncthreads();
    } else {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  }
  __device__ static void to_blocked(uint64_t *lds, uint64_t (&x)[P], int c, int r) {
#pragma unroll
    for (int i = 0; i < P; i++) lds[lidx(c, ipoint(r, i))] = x[i];
    exchange_sync();
#pragma unroll
    for (int v = 0; v < P; v++) x[v] = lds[lidx(c, bpoint(r, v))];
    exchange_sync();
  }
  __device__ static void to_interleaved(uint64_t *lds, uint64_t (&x)[P], int c, int r) {
#pragma unroll
    for (int v = 0; v < P; v++) lds[lidx(c, bpoint(r, v))] = x[v];
    exchange_sync();
#pragma unroll
    for (int i = 0; i < P; i++) x[i] = lds[lidx(c, ipoint(r, i))];
    exchange_sync();
  }

  // forward stages: interleaved in, blocked out
  __device__ static void forward(uint64_t *lds, uint64_t (&x)[P], int c, int r, int g,
                                 const uint64_t *w, const uint64_t *wp, Qn q) {
#pragma unroll
    for (int s = 0; s < LOGP; s++) {
      const int h = P >> (s + 1);
#pragma unroll
      for (int i = 0; i < P; i++) {
        if (i & h) continue;
        const int k = tw_interleaved(s, i);
        ct_bfly(x[i], x[i + h], w[k], wp[k], q);
      }
    }
    to_blocked(lds, x, c, r);
#pragma unroll
    for (int s = LOGP; s < LOGR; s++) {
      const int t = R >> (s + 1);
#pragma unroll
      for (int v = 0; v < P; v++) {
        if (v & t) continue;
        const int k = tw(s, g, bpoint(r, v));
        ct_bfly(x[v], x[v + t], w[k], wp[k], q);
      }
    }
  }

  // inverse stages: blocked in, interleaved out
  __device__ static void inverse(uint64_t *lds, uint64_t (&x)[P], int c, int r, int g,
                                 const uint64_t *w, const uint64_t *wp, Qn q) {
#pragma unroll
    for (int s = LOGR - 1; s >= LOGP; s--) {
      const int t = R >> (s + 1);
#pragma unroll
      for (int v = 0; v < P; v++) {
        if (v & t) continue;
        const int k = tw(s, g, bpoint(r, v));
        gs_bfly(x[v], x[v + t], w[k], wp[k], q);
      }
    }
    to_interleaved(lds, x, c, r);
#pragma unroll
    for (int s = LOGP - 1; s >= 0; s--) {
      const int h = P >> (s + 1);
#pragma unroll
      for (int i = 0; i < P; i++) {
        if (i & h) continue;
        const int k = tw_interleaved(s, i);
        gs_bfly(x[i], x[i + h], w[k], wp[k], q);
      }
    }
  }
};

// [0, 4q) -> [0, q)
__device__ __forceinline__ uint64_t reduce4(uint64_t v, Qn m) {
  return csub(csub(v, 2 * m.q, 2 * m.nq), m.q, m.nq);
}

// Slot of the input that lands in slot j under X -> X^g (bit-reversed
// evaluation order: slot j holds the value at psi^(2 brv(j) + 1)).
__device__ __forceinline__ uint32_t galois_src(uint32_t j, uint32_t g, int log_n) {
  const uint32_t shift = 32 - log_n;
  const uint32_t e = 2 * (__brev(j) >> shift) + 1;
  const uint32_t se = (uint32_t)(((uint64_t)e * g) & ((2u << log_n) - 1));
  return __brev((se - 1) >> 1) >> shift;
}

// log2(R1), log2(R2) of the two-pass split
constexpr int split_a(int log_n) { return (log_n + 1) / 2; }
constexpr int split_b(int log_n) { return log_n / 2; }

}  // namespace hck
