// Inner sums of the baby-step/giant-step linear transform (Kernel 3's
// diagonal method) in one pass over memory.
//
// For giant index g and output o the inner sum is
//   inner[g][o] = sum over terms t of o, baby steps b:
//                 sign_t pt_{lt_t, g, b} * Rot(x_{in_t}, b)
// (pt_{lt, g, b} is the transform's diagonal g n1 + b, pre-rotated and cached
// in evaluation + Montgomery form).  A thread owns one coefficient of one
// limb and walks the baby steps once: it loads every input's baby rotation
// once per pass, each cached diagonal exactly once, and keeps the sums of G
// giant groups x O outputs x 2 polynomials in 128-bit registers, reduced by
// one Montgomery REDC at the end (and at flushes, see below).  A negative
// sign is folded into the ciphertext operand (q - x).
#include "internal.h"

namespace hck {

namespace {

template <int G, int O, int I>
__global__ __launch_bounds__(256) void k_lt_inner(LtInnerArgs a, const ModConst *__restrict__ mc,
                                                  int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int limb = blockIdx.y;
  const ModConst m = mc[limb];
  const size_t off = (size_t)limb * n + i;
  // products of values below q accumulate safely while their count stays
  // below 2^64 / q (the REDC input bound); each baby step adds up to
  // max_terms products to one sum.  A flush reduces a sum to r in [0, q) and
  // restarts it from r 2^64 mod q, which REDC maps back to r.
  const uint64_t per_flush = ~0ull / m.q - 1;
  const uint32_t flush_b = (uint32_t)max<uint64_t>(1, per_flush / a.max_terms);
  u128 acc[G][O][2];
#pragma unroll
  for (int g = 0; g < G; g++)
#pragma unroll
    for (int o = 0; o < O; o++)
#pragma unroll
      for (int p = 0; p < 2; p++) {
        acc[g][o][p].lo = acc[g][o][p].hi = 0;
        if (a.accumulate && g < (int)a.ng && o < (int)a.n_out && a.inner[g][o])
          acc[g][o][p].lo = shoup(a.inner[g][o][off + p * a.ps], m.r64, m.r64_shoup, m.q);
      }
  uint32_t since = 0;
  for (uint32_t b = 0; b < a.n1; b++) {
    uint64_t x[I][2];
#pragma unroll
    for (int in = 0; in < I; in++) {
      x[in][0] = x[in][1] = 0;
      if (in < (int)a.n_in && a.baby[in][b]) {
        x[in][0] = a.baby[in][b][off];
        x[in][1] = a.baby[in][b][off + a.ps];
      }
    }
#pragma unroll
    for (int g = 0; g < G; g++) {
      if (g >= (int)a.ng) break;
#pragma unroll
      for (int l = 0; l < kLtLts; l++) {
        const uint64_t *pp = a.pt[g][l][b];
        if (!pp) continue;
        const uint64_t w = pp[off];
#pragma unroll
        for (int t = 0; t < kLtTerms; t++) {
          if (t >= (int)a.n_terms || a.term_lt[t] != l) continue;
          const int in = a.term_in[t], o = a.term_out[t];
#pragma unroll
          for (int ii = 0; ii < I; ii++) {
            if (ii != in) continue;
#pragma unroll
            for (int oo = 0; oo < O; oo++) {
              if (oo != o) continue;
              const uint64_t x0 = a.term_neg[t] ? m.q - x[ii][0] : x[ii][0];
              const uint64_t x1 = a.term_neg[t] ? m.q - x[ii][1] : x[ii][1];
              mac_wide(acc[g][oo][0], w, x0);
              mac_wide(acc[g][oo][1], w, x1);
            }
          }
        }
      }
    }
    if (++since == flush_b && b + 1 < a.n1) {
      since = 0;
#pragma unroll
      for (int g = 0; g < G; g++)
#pragma unroll
        for (int o = 0; o < O; o++)
#pragma unroll
          for (int p = 0; p < 2; p++) {
            acc[g][o][p].lo = shoup(redc(acc[g][o][p], m.q, m.qinv), m.r64, m.r64_shoup, m.q);
            acc[g][o][p].hi = 0;
          }
    }
  }
#pragma unroll
  for (int g = 0; g < G; g++)
#pragma unroll
    for (int o = 0; o < O; o++)
      if (g < (int)a.ng && o < (int)a.n_out && a.inner[g][o]) {
        a.inner[g][o][off] = redc(acc[g][o][0], m.q, m.qinv);
        a.inner[g][o][off + a.ps] = redc(acc[g][o][1], m.q, m.qinv);
      }
}

}  // namespace

int launch_lt_inner(hck_context *ctx, const LtInnerArgs &a, uint32_t level) {
  const uint32_t nq = level + 1;
  double loads = 0, macs = 0;
  for (uint32_t g = 0; g < a.ng; g++)
    for (int l = 0; l < kLtLts; l++)
      for (uint32_t b = 0; b < a.n1; b++)
        if (a.pt[g][l][b]) {
          loads += 1;
          for (uint32_t t = 0; t < a.n_terms; t++) macs += (a.term_lt[t] == l) ? 2 : 0;
        }
  double babies = 0;
  for (uint32_t in = 0; in < a.n_in; in++)
    for (uint32_t b = 0; b < a.n1; b++) babies += a.baby[in][b] ? 2 : 0;
  const double words = (double)ctx->n * nq;
  timing_begin(ctx, "lt_inner",
               8.0 * words * (loads + babies + 2.0 * a.ng * a.n_out * (a.accumulate ? 2 : 1)),
               words * (macs + 2.0 * a.ng * a.n_out));
  dim3 grid(ctx->n / 256, nq);
  if (a.n_in <= 1 && a.n_out <= 1)
    k_lt_inner<4, 1, 1><<<grid, 256, 0, ctx->stream>>>(a, ctx->d_mod, ctx->n);
  else if (a.n_in <= 2 && a.n_out <= 2 && a.ng <= 4)
    k_lt_inner<4, 2, 2><<<grid, 256, 0, ctx->stream>>>(a, ctx->d_mod, ctx->n);
  else if (a.n_in <= kLtIn && a.n_out <= kLtOut && a.ng <= 2)
    k_lt_inner<2, kLtOut, kLtIn><<<grid, 256, 0, ctx->stream>>>(a, ctx->d_mod, ctx->n);
  else
    return set_error(HCK_EINVAL, "linear-transform launch shape not supported");
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

}  // namespace hck
