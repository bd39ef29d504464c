// Inner sums of the baby-step/giant-step linear transform (Kernel 3's
// diagonal method), all giant groups in one pass over the diagonals.
//
// For giant group g and output o the inner sum is
//   sums[g][o] = sum over terms t of o, baby steps b:
//                sign_t pt_{lt_t, g, b} * Rot(x_{in_t}, b)
// (pt_{lt, g, b} is the transform's diagonal g n1 + b, pre-rotated and cached
// in evaluation + Montgomery form, in the transform's [giant][baby] grid).
//
// A workgroup owns kLtCoeffs consecutive coefficients of one limb.  It first
// stages the baby rotations of its coefficients (every input, every baby step
// of the launch, both polynomials) in LDS, read from HBM once for all giant
// groups; then each of its 4 waves takes giant groups w, w + 4, ... (GW at a
// time, round robin), one coefficient per lane, and streams those groups'
// diagonals once,
// keeping GW x O x 2 sums in registers that are reduced by one Montgomery
// REDC at the end (and at flushes, see below).  A limb whose prime is below
// 2^52 keeps each sum in three carry-free 64-bit columns (four 32-bit
// multiply-adds per product); a wider prime keeps it as one 128-bit value.
// The terms enter as a sign per (transform, input, output); a negative one
// multiplies by the negated diagonal (q - w).
#include "internal.h"

namespace hck {

namespace {

// One inner sum in a 128-bit register pair: any q < 2^62.  The count of
// products between reductions stays below 2^64 / q (the REDC input bound).
struct WideSum {
  u128 v;
  __device__ __forceinline__ void set(uint64_t r) {
    v.lo = r;
    v.hi = 0;
  }
  __device__ __forceinline__ void mac(uint64_t w, uint64_t x) { mac_wide(v, w, x); }
  __device__ __forceinline__ u128 total() const { return v; }
  static __device__ __forceinline__ uint64_t max_products(uint64_t q) { return ~0ull / q - 1; }
};

// One inner sum in three 64-bit columns, for q < 2^52.  Both factors split
// at bit 26 into halves below 2^26, so each of the four 32 x 32-bit partial
// products is below 2^52 and lands, without carry handling, in the column of
// weight 1, 2^26 or 2^52: four v_mad_u64_u32 per product in place of a
// 128-bit multiply and add.  The middle column takes two partial products
// per product, so up to 2^11 products fit.
struct ColSum {
  static constexpr uint32_t kLow = (1u << 26) - 1;
  uint64_t c0, c1, c2;
  __device__ __forceinline__ void set(uint64_t r) {
    c0 = r;
    c1 = c2 = 0;
  }
  __device__ __forceinline__ void mac(uint64_t w, uint64_t x) {
    const uint32_t w0 = (uint32_t)w & kLow, w1 = (uint32_t)(w >> 26);
    const uint32_t x0 = (uint32_t)x & kLow, x1 = (uint32_t)(x >> 26);
    c0 += (uint64_t)w0 * x0;
    c1 += (uint64_t)w0 * x1;
    c1 += (uint64_t)w1 * x0;
    c2 += (uint64_t)w1 * x1;
  }
  // c0 + c1 2^26 + c2 2^52 as a 128-bit value
  __device__ __forceinline__ u128 total() const {
    const uint64_t a = c1 << 26, b = c2 << 52;
    u128 t;
    t.lo = c0 + a;
    uint64_t carry = t.lo < a;
    t.lo += b;
    carry += t.lo < b;
    t.hi = (c1 >> 38) + (c2 >> 12) + carry;
    return t;
  }
  static __device__ __forceinline__ uint64_t max_products(uint64_t q) {
    return min<uint64_t>(~0ull / q - 1, 2047);
  }
};

// One pass of a wave over the staged baby rotations xs: giant groups g0,
// g0 + 4, ..., g0 + 4 (GW - 1) (those below ng); Sum is the accumulator kind.
template <class Sum, int GW, int O, int I>
__device__ __forceinline__ void lt_sums_pass(const LtSumArgs &a, const uint64_t *xs,
                                             const ModConst &m, size_t base, int n, int lane,
                                             int g0, int flush_b) {
  constexpr int C = kLtCoeffs;
  const int nb = (int)a.nb;
  const size_t off = base + lane;
  {
    Sum acc[GW][O][2];
#pragma unroll
    for (int gi = 0; gi < GW; gi++)
#pragma unroll
      for (int o = 0; o < O; o++)
#pragma unroll
        for (int p = 0; p < 2; p++) {
          uint64_t r = 0;
          if (a.accumulate && g0 + 4 * gi < (int)a.ng && o < (int)a.n_out)
            r = shoup(a.sums[((size_t)(g0 + 4 * gi) * a.n_out + o) * 2 * a.ps + p * a.ps + off],
                      m.r64, m.r64_shoup, m.q);
          acc[gi][o][p].set(r);
        }
    // an absent diagonal reads a row of zeros, so every step issues all its
    // loads without branches before any product; addresses are wave-uniform
    // bases (scalar) plus the lane
    auto load_rows = [&](uint64_t(&w)[GW][kLtLts], int b) {
#pragma unroll
      for (int l = 0; l < kLtLts; l++)
#pragma unroll
        for (int gi = 0; gi < GW; gi++) {
          const int g = g0 + 4 * gi;
          const bool on = g < (int)a.ng && ((a.present[l][g] >> b) & 1u);
          const uint64_t *row =
              on ? a.grid[l] +
                       (size_t)(a.gmap[l][g] * (int)a.grid_nb[l] + a.bmap[l][b]) * a.grid_rows[l] * n +
                       base
                 : a.zero + base;
          w[gi][l] = row[lane];
        }
    };
    int since = 0;
    for (int b = 0; b < nb; b++) {
      uint64_t w[GW][kLtLts];
      load_rows(w, b);
      uint64_t x[I][2];
#pragma unroll
      for (int in = 0; in < I; in++)
#pragma unroll
        for (int p = 0; p < 2; p++)
          x[in][p] = in < (int)a.n_in ? xs[((in * nb + b) * 2 + p) * C + lane] : 0;
      // a negative term multiplies by q - w (a transform's terms share w)
#pragma unroll
      for (int l = 0; l < kLtLts; l++) {
        bool neg = false;
#pragma unroll
        for (int ii = 0; ii < I; ii++)
#pragma unroll
          for (int oo = 0; oo < O; oo++) neg = neg || a.coef[l][ii][oo] < 0;
#pragma unroll
        for (int gi = 0; gi < GW; gi++) {
          const uint64_t wn = neg ? m.q - w[gi][l] : 0;
#pragma unroll
          for (int ii = 0; ii < I; ii++)
#pragma unroll
            for (int oo = 0; oo < O; oo++) {
              const int c = a.coef[l][ii][oo];
              if (c == 0) continue;
              const uint64_t ws = c < 0 ? wn : w[gi][l];
              acc[gi][oo][0].mac(ws, x[ii][0]);
              acc[gi][oo][1].mac(ws, x[ii][1]);
            }
        }
      }
      if (++since == flush_b && b + 1 < nb) {
        since = 0;
#pragma unroll
        for (int gi = 0; gi < GW; gi++)
#pragma unroll
          for (int o = 0; o < O; o++)
#pragma unroll
            for (int p = 0; p < 2; p++)
              acc[gi][o][p].set(
                  shoup(redc(acc[gi][o][p].total(), m.q, m.qinv), m.r64, m.r64_shoup, m.q));
      }
    }
#pragma unroll
    for (int gi = 0; gi < GW; gi++)
#pragma unroll
      for (int o = 0; o < O; o++)
        if (g0 + 4 * gi < (int)a.ng && o < (int)a.n_out) {
          uint64_t *dst = a.sums + ((size_t)(g0 + 4 * gi) * a.n_out + o) * 2 * a.ps + off;
          dst[0] = redc(acc[gi][o][0].total(), m.q, m.qinv);
          dst[a.ps] = redc(acc[gi][o][1].total(), m.q, m.qinv);
        }
  }
}

// The last R or fewer groups of a wave (rem of them, 1 <= rem <= R) in one
// pass of exactly rem slots.
template <class Sum, int R, int O, int I>
__device__ __forceinline__ void lt_sums_rest(const LtSumArgs &a, const uint64_t *xs,
                                             const ModConst &m, size_t base, int n, int lane,
                                             int g0, int rem, int flush_b) {
  if constexpr (R > 0) {
    if (rem == R)
      lt_sums_pass<Sum, R, O, I>(a, xs, m, base, n, lane, g0, flush_b);
    else
      lt_sums_rest<Sum, R - 1, O, I>(a, xs, m, base, n, lane, g0, rem, flush_b);
  }
}

// The giant groups of one wave: w, w + 4, w + 8, ..., GW at a time, so the
// four waves of a workgroup stay within one group of each other.  With REST
// the last fewer than GW take a pass of their own size (no idle slots, each
// of which loads a row of zeros); otherwise the last pass has idle slots.
template <class Sum, int GW, int O, int I, bool REST>
__device__ __forceinline__ void lt_sums_wave(const LtSumArgs &a, const uint64_t *xs,
                                             const ModConst &m, size_t base, int n, int wave,
                                             int lane) {
  // each baby step adds up to max_terms products to one sum.  A flush
  // reduces a sum to r in [0, q) and restarts it from r 2^64 mod q, which
  // REDC maps back to r.
  const int flush_b = (int)max<uint64_t>(1, Sum::max_products(m.q) / a.max_terms);
  const int ng = (int)a.ng;
  int g0 = wave;
  if constexpr (REST) {
    for (; g0 + 4 * (GW - 1) < ng; g0 += 4 * GW)
      lt_sums_pass<Sum, GW, O, I>(a, xs, m, base, n, lane, g0, flush_b);
    if (g0 < ng)
      lt_sums_rest<Sum, GW - 1, O, I>(a, xs, m, base, n, lane, g0, (ng - g0 + 3) / 4, flush_b);
  } else {
    for (; g0 < ng; g0 += 4 * GW) lt_sums_pass<Sum, GW, O, I>(a, xs, m, base, n, lane, g0, flush_b);
  }
}

// GW / GWN: giant groups a wave carries at a time with 128-bit / column sums
template <int GW, int GWN, int O, int I>
__global__ __launch_bounds__(256, 4) void k_lt_sums(LtSumArgs a, const ModConst *__restrict__ mc,
                                                 int n) {
  constexpr int C = kLtCoeffs;
  extern __shared__ uint64_t xs[];  // [in][b][poly][C]
  const int limb = blockIdx.y;
  const size_t base = (size_t)limb * n + (size_t)blockIdx.x * C;
  const int nb = (int)a.nb;
  const int total = (int)a.n_in * nb * 2 * C;
  for (int idx = threadIdx.x; idx < total; idx += 256) {
    const int c = idx % C;
    const int r = idx / C;
    const int p = r & 1, b = (r >> 1) % nb, in = (r >> 1) / nb;
    const uint64_t *src = a.baby[in][b];
    xs[idx] = src ? src[base + p * a.ps + c] : 0;
  }
  __syncthreads();
  // the wave index is uniform across the wave: readfirstlane lets the
  // compiler keep the giant tables, branches and diagonal addresses scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  const ModConst m = mc[limb];
  // the limb's modulus is uniform across the workgroup
  if (m.q < (1ull << 52))
    lt_sums_wave<ColSum, GWN, O, I, true>(a, xs, m, base, n, wave, lane);
  else
    lt_sums_wave<WideSum, GW, O, I, false>(a, xs, m, base, n, wave, lane);
}

template <int GW, int GWN, int O, int I>
void launch(hck_context *ctx, const LtSumArgs &a, uint32_t nq) {
  const size_t lds = (size_t)a.n_in * a.nb * 2 * kLtCoeffs * sizeof(uint64_t);
  k_lt_sums<GW, GWN, O, I><<<dim3(ctx->n / kLtCoeffs, nq), 256, lds, ctx->stream>>>(a, ctx->d_mod,
                                                                               ctx->n);
}

}  // namespace

int launch_lt_sums(hck_context *ctx, const LtSumArgs &a, uint32_t level) {
  const uint32_t nq = level + 1;
  if (a.nb == 0 || a.nb > (uint32_t)kLtB || a.ng > (uint32_t)kLtMaxG || a.n_in == 0 ||
      a.n_in > (uint32_t)kLtIn || a.n_out == 0 || a.n_out > (uint32_t)kLtOut ||
      (size_t)a.n_in * a.nb * 2 * kLtCoeffs * sizeof(uint64_t) > 65536)
    return set_error(HCK_EINVAL, "linear-transform launch shape not supported");
  double diags = 0, macs = 0;
  for (uint32_t g = 0; g < a.ng; g++)
    for (int l = 0; l < kLtLts; l++)
      for (uint32_t b = 0; b < a.nb; b++)
        if ((a.present[l][g] >> b) & 1u) {
          diags += 1;
          for (int i = 0; i < kLtIn; i++)
            for (int o = 0; o < kLtOut; o++) macs += a.coef[l][i][o] ? 2.0 : 0.0;
        }
  double babies = 0;
  for (uint32_t in = 0; in < a.n_in; in++)
    for (uint32_t b = 0; b < a.nb; b++) babies += a.baby[in][b] ? 2 : 0;
  const double words = (double)ctx->n * nq;
  timing_begin(ctx, "lt_inner", dim3(ctx->n / kLtCoeffs, nq),
               8.0 * words * (diags + babies + 2.0 * a.ng * a.n_out * (a.accumulate ? 2 : 1)),
               words * macs);
  if (a.n_out <= 1 && a.n_in <= 2)
    launch<8, 6, 1, 2>(ctx, a, nq);
  else if (a.n_out <= 2 && a.n_in <= 2)
    launch<5, 3, 2, 2>(ctx, a, nq);
  else
    launch<2, 1, kLtOut, kLtIn>(ctx, a, nq);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

}  // namespace hck
