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

// Geometry of one pass: R-point sub-transforms of an N-point limb, two
// layouts (interleaved, blocked) of P = 2^ceil(log2(R)/2) points a thread.
template <int LOGR, int LOGN, bool STRIDED>
struct Pass2 {
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

// Contiguous pass of R = 2^LOGR points, LOGR = 7..9, with P = 8 points a
// thread (T = R / 8 threads a sub-transform, inside one wavefront) in three
// layouts of the point index p (bits LOGR-1 .. 0), LM = LOGR - 6:
//   I (interleaved): thread r holds p = r + T k, so register k is the top 3
//     bits; stages 0..2 pair registers k, k + 4 / 2 / 1 with twiddles that
//     depend on k only (uniform across the wavefront);
//   M (middle): register k is bits LOGR-4 .. LOGR-6 and the thread the rest,
//     p = (r >> LM) R/8 + k 2^LM + (r mod 2^LM); stages 3 .. LOGR-4;
//   B (blocked): thread r holds p = 8 r + k, register k the low 3 bits;
//     stages LOGR-3 .. LOGR-1.
// The butterflies, their twiddles and their order per point are those of
// the two-layout pass, so the results are the same words; the pass takes two
// LDS exchanges each way instead of one, and in return a thread holds half
// the points (the fused key-switching passes keep three such arrays live)
// and a workgroup half the LDS.
template <int LOGR, int LOGN>
struct Pass3 {
  static_assert(LOGR >= 7 && LOGR <= 9, "three-layout pass covers 128..512 points");
  static constexpr int R = 1 << LOGR;
  static constexpr int P = 8;
  static constexpr int T = R / P;                 // threads per sub-transform
  static constexpr int TR = kNttThreads / T;      // sub-transforms per workgroup
  static constexpr int N = 1 << LOGN;
  static constexpr int OTHER = N / R;             // sub-transforms per limb
  static constexpr int LM = LOGR - 6;
  static constexpr int S = R + R / 8 + 1;         // LDS words per sub-transform
  static constexpr int LDS_WORDS = TR * S;
  static constexpr int BLOCKS = OTHER / TR;       // workgroups per limb
  static_assert(T <= 64 && 64 % T == 0, "sub-transform must fit one wavefront");

  __device__ static int lidx(int c, int p) { return c * S + p + (p >> 3); }
  __device__ static size_t gaddr(int g, int p) { return (size_t)g * R + p; }
  __device__ static int sub(int tid) { return tid / T; }
  __device__ static int lane(int tid) { return tid % T; }
  __device__ static int ipoint(int r, int k) { return r + T * k; }
  __device__ static int mpoint(int r, int k) {
    return (r >> LM) * (R / 8) + (k << LM) + (r & ((1 << LM) - 1));
  }
  __device__ static int bpoint(int r, int k) { return r * P + k; }
  template <int LAYOUT>
  __device__ static int point(int r, int k) {
    return LAYOUT == 0 ? ipoint(r, k) : LAYOUT == 1 ? mpoint(r, k) : bpoint(r, k);
  }
  // twiddle of stage s for the butterfly with top point p (sub-transform
  // 0's network, which every sub-transform runs on twisted inputs)
  __device__ static int tw(int s, int p) { return (1 << s) * OTHER + (p >> (LOGR - s)); }

  __device__ static void twist(uint64_t (&x)[P], int g, int r, const uint64_t *t,
                               const uint64_t *ts, Qn q) {
#pragma unroll
    for (int k = 0; k < P; k++) {
      const size_t a = gaddr(g, ipoint(r, k));
      x[k] = shoup_lazy(x[k], t[a], ts[a], q);
    }
  }

  // a wavefront's LDS operations complete in issue order; the fence keeps
  // the compiler from moving them across each other
  __device__ static void sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  template <int FROM, int TO>
  __device__ static void exchange(uint64_t *lds, uint64_t (&x)[P], int c, int r) {
#pragma unroll
    for (int k = 0; k < P; k++) lds[lidx(c, point<FROM>(r, k))] = x[k];
    sync();
#pragma unroll
    for (int k = 0; k < P; k++) x[k] = lds[lidx(c, point<TO>(r, k))];
    sync();
  }
  __device__ static void to_blocked(uint64_t *lds, uint64_t (&x)[P], int c, int r) {
    exchange<0, 2>(lds, x, c, r);
  }
  __device__ static void to_interleaved(uint64_t *lds, uint64_t (&x)[P], int c, int r) {
    exchange<2, 0>(lds, x, c, r);
  }

  // forward stages: interleaved in, blocked out
  __device__ static void forward(uint64_t *lds, uint64_t (&x)[P], int c, int r, int g,
                                 const uint64_t *w, const uint64_t *wp, Qn q) {
#pragma unroll
    for (int s = 0; s < 3; s++) {
      const int h = 4 >> s;
#pragma unroll
      for (int k = 0; k < P; k++) {
        if (k & h) continue;
        const int t = (1 << s) * OTHER + (k >> (3 - s));
        ct_bfly(x[k], x[k + h], w[t], wp[t], q);
      }
    }
    exchange<0, 1>(lds, x, c, r);
#pragma unroll
    for (int s = 3; s <= LOGR - 4; s++) {
      const int h = 1 << (LOGR - 1 - s - LM);
#pragma unroll
      for (int k = 0; k < P; k++) {
        if (k & h) continue;
        const int t = tw(s, mpoint(r, k));
        ct_bfly(x[k], x[k + h], w[t], wp[t], q);
      }
    }
    exchange<1, 2>(lds, x, c, r);
#pragma unroll
    for (int s = LOGR - 3; s < LOGR; s++) {
      const int h = 1 << (LOGR - 1 - s);
#pragma unroll
      for (int k = 0; k < P; k++) {
        if (k & h) continue;
        const int t = tw(s, bpoint(r, k));
        ct_bfly(x[k], x[k + h], w[t], wp[t], q);
      }
    }
  }

  // inverse stages: blocked in, interleaved out
  __device__ static void inverse(uint64_t *lds, uint64_t (&x)[P], int c, int r, int g,
                                 const uint64_t *w, const uint64_t *wp, Qn q) {
#pragma unroll
    for (int s = LOGR - 1; s >= LOGR - 3; s--) {
      const int h = 1 << (LOGR - 1 - s);
#pragma unroll
      for (int k = 0; k < P; k++) {
        if (k & h) continue;
        const int t = tw(s, bpoint(r, k));
        gs_bfly(x[k], x[k + h], w[t], wp[t], q);
      }
    }
    exchange<2, 1>(lds, x, c, r);
#pragma unroll
    for (int s = LOGR - 4; s >= 3; s--) {
      const int h = 1 << (LOGR - 1 - s - LM);
#pragma unroll
      for (int k = 0; k < P; k++) {
        if (k & h) continue;
        const int t = tw(s, mpoint(r, k));
        gs_bfly(x[k], x[k + h], w[t], wp[t], q);
      }
    }
    exchange<1, 0>(lds, x, c, r);
#pragma unroll
    for (int s = 2; s >= 0; s--) {
      const int h = 4 >> s;
#pragma unroll
      for (int k = 0; k < P; k++) {
        if (k & h) continue;
        const int t = (1 << s) * OTHER + (k >> (3 - s));
        gs_bfly(x[k], x[k + h], w[t], wp[t], q);
      }
    }
  }
};

// The pass geometry of a split: three layouts for contiguous passes of 128
// points or more, two otherwise.
template <bool THREE, int LOGR, int LOGN, bool STRIDED>
struct PassPick {
  using type = Pass2<LOGR, LOGN, STRIDED>;
};
template <int LOGR, int LOGN>
struct PassPick<true, LOGR, LOGN, false> {
  using type = Pass3<LOGR, LOGN>;
};
template <int LOGR, int LOGN, bool STRIDED>
using Pass = typename PassPick<!STRIDED && LOGR >= 7, LOGR, LOGN, STRIDED>::type;

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
