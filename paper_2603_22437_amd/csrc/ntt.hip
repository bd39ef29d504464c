// Negacyclic NTT / inverse NTT over many limbs in one launch (gfx950).
//
// Forward transform: the merged Cooley-Tukey network whose stage m (m = 1, 2,
// ..., N/2; half-width t = N / 2m) combines x[j], x[j+t] with the twiddle
// psi^brv(m + j / 2t), psi a primitive 2N-th root of unity and brv the logN-bit
// reversal.  Slot j of the output holds the polynomial's value at
// psi^(2 brv(j) + 1) (bit-reversed evaluation order).  The inverse runs the
// Gentleman-Sande network with psi^-brv in the reverse stage order and scales
// by N^-1, optionally times a per-limb constant and plus a per-limb addend.
//
// A limb of N 64-bit words (512 KiB at N = 2^16) exceeds one CU's LDS, so
// each transform is two passes over HBM, N = R1 x R2:
//   * strided pass: stages m < R1 touch only elements R2 apart, so R1-point
//     columns are independent; a workgroup loads a tile of C adjacent
//     columns (C words contiguous per row), runs log2(R1) stages in LDS, and
//     writes the tile back;
//   * contiguous pass: stages m >= R1 stay inside blocks of R2 contiguous
//     words; a workgroup runs log2(R2) stages on ROWS such blocks.
// Butterflies are Harvey's lazy ones (values in [0, 4q) forward, [0, 2q)
// inverse, q < 2^61) with Shoup twiddle products.
#include "internal.h"

namespace hck {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 4096;  // words per workgroup tile (32 KiB of LDS)

__device__ __forceinline__ void ct_bfly(uint64_t &x, uint64_t &y, uint64_t w, uint64_t wp,
                                        uint64_t q) {
  const uint64_t q2 = 2 * q;
  uint64_t a = x >= q2 ? x - q2 : x;       // [0, 2q)
  uint64_t t = shoup_lazy(y, w, wp, q);    // [0, 2q)
  x = a + t;                               // [0, 4q)
  y = a - t + q2;                          // (0, 4q)
}

__device__ __forceinline__ void gs_bfly(uint64_t &x, uint64_t &y, uint64_t w, uint64_t wp,
                                        uint64_t q) {
  const uint64_t q2 = 2 * q;
  uint64_t s = x + y;
  s = s >= q2 ? s - q2 : s;                // [0, 2q)
  y = shoup_lazy(x - y + q2, w, wp, q);    // [0, 2q)
  x = s;
}

template <int LOG_R1, int LOG_R2>
__global__ __launch_bounds__(kThreads) void k_fwd_strided(uint64_t *__restrict__ buf, LimbMap map,
                                                          const ModConst *__restrict__ mc,
                                                          const uint64_t *__restrict__ tw,
                                                          const uint64_t *__restrict__ tws) {
  constexpr int R1 = 1 << LOG_R1, R2 = 1 << LOG_R2, N = R1 * R2;
  constexpr int C = (kTile / R1) < R2 ? (kTile / R1) : R2;
  constexpr int E = R1 * C;
  __shared__ uint64_t lds[E];
  const int mi = map.mod[blockIdx.y];
  const uint64_t q = mc[mi].q;
  uint64_t *p = buf + (size_t)map.row[blockIdx.y] * N + blockIdx.x * C;
  const uint64_t *w_ = tw + (size_t)mi * N;
  const uint64_t *wp_ = tws + (size_t)mi * N;
  for (int e = threadIdx.x; e < E; e += kThreads) lds[e] = p[(e / C) * R2 + (e % C)];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < LOG_R1; s++) {
    const int t = R1 >> (s + 1);
    for (int b = threadIdx.x; b < (R1 / 2) * C; b += kThreads) {
      const int c = b % C, k = b / C;
      const int grp = k / t;
      const int j = grp * 2 * t + (k % t);
      const int widx = (1 << s) + grp;
      uint64_t x = lds[j * C + c], y = lds[(j + t) * C + c];
      ct_bfly(x, y, w_[widx], wp_[widx], q);
      lds[j * C + c] = x;
      lds[(j + t) * C + c] = y;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < E; e += kThreads) p[(e / C) * R2 + (e % C)] = lds[e];
}

template <int LOG_R1, int LOG_R2>
__global__ __launch_bounds__(kThreads) void k_fwd_contig(uint64_t *__restrict__ buf, LimbMap map,
                                                         const ModConst *__restrict__ mc,
                                                         const uint64_t *__restrict__ tw,
                                                         const uint64_t *__restrict__ tws) {
  constexpr int R1 = 1 << LOG_R1, R2 = 1 << LOG_R2, N = R1 * R2;
  constexpr int ROWS = (kTile / R2) < R1 ? (kTile / R2) : R1;
  constexpr int E = ROWS * R2;
  __shared__ uint64_t lds[E];
  const int mi = map.mod[blockIdx.y];
  const uint64_t q = mc[mi].q;
  const int r0 = blockIdx.x * ROWS;
  uint64_t *p = buf + (size_t)map.row[blockIdx.y] * N + (size_t)r0 * R2;
  const uint64_t *w_ = tw + (size_t)mi * N;
  const uint64_t *wp_ = tws + (size_t)mi * N;
  for (int e = threadIdx.x; e < E; e += kThreads) lds[e] = p[e];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < LOG_R2; s++) {
    const int t = R2 >> (s + 1);
    for (int b = threadIdx.x; b < (R2 / 2) * ROWS; b += kThreads) {
      const int k = b % (R2 / 2), rr = b / (R2 / 2);
      const int grp = k / t;
      const int j = rr * R2 + grp * 2 * t + (k % t);
      const int widx = (1 << s) * (R1 + r0 + rr) + grp;
      uint64_t x = lds[j], y = lds[j + t];
      ct_bfly(x, y, w_[widx], wp_[widx], q);
      lds[j] = x;
      lds[j + t] = y;
    }
    __syncthreads();
  }
  const uint64_t q2 = 2 * q;
  for (int e = threadIdx.x; e < E; e += kThreads) {
    uint64_t v = lds[e];
    v = v >= q2 ? v - q2 : v;
    p[e] = v >= q ? v - q : v;
  }
}

template <int LOG_R1, int LOG_R2>
__global__ __launch_bounds__(kThreads) void k_inv_contig(uint64_t *__restrict__ buf, LimbMap map,
                                                         const ModConst *__restrict__ mc,
                                                         const uint64_t *__restrict__ itw,
                                                         const uint64_t *__restrict__ itws) {
  constexpr int R1 = 1 << LOG_R1, R2 = 1 << LOG_R2, N = R1 * R2;
  constexpr int ROWS = (kTile / R2) < R1 ? (kTile / R2) : R1;
  constexpr int E = ROWS * R2;
  __shared__ uint64_t lds[E];
  const int mi = map.mod[blockIdx.y];
  const uint64_t q = mc[mi].q;
  const int r0 = blockIdx.x * ROWS;
  uint64_t *p = buf + (size_t)map.row[blockIdx.y] * N + (size_t)r0 * R2;
  const uint64_t *w_ = itw + (size_t)mi * N;
  const uint64_t *wp_ = itws + (size_t)mi * N;
  for (int e = threadIdx.x; e < E; e += kThreads) lds[e] = p[e];
  __syncthreads();
#pragma unroll
  for (int s = LOG_R2 - 1; s >= 0; s--) {
    const int t = R2 >> (s + 1);
    for (int b = threadIdx.x; b < (R2 / 2) * ROWS; b += kThreads) {
      const int k = b % (R2 / 2), rr = b / (R2 / 2);
      const int grp = k / t;
      const int j = rr * R2 + grp * 2 * t + (k % t);
      const int widx = (1 << s) * (R1 + r0 + rr) + grp;
      uint64_t x = lds[j], y = lds[j + t];
      gs_bfly(x, y, w_[widx], wp_[widx], q);
      lds[j] = x;
      lds[j + t] = y;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < E; e += kThreads) p[e] = lds[e];  // [0, 2q)
}

template <int LOG_R1, int LOG_R2>
__global__ __launch_bounds__(kThreads) void k_inv_strided(uint64_t *__restrict__ buf, LimbMap map,
                                                          const ModConst *__restrict__ mc,
                                                          const uint64_t *__restrict__ itw,
                                                          const uint64_t *__restrict__ itws,
                                                          RowScale sc, int use_scale) {
  constexpr int R1 = 1 << LOG_R1, R2 = 1 << LOG_R2, N = R1 * R2;
  constexpr int C = (kTile / R1) < R2 ? (kTile / R1) : R2;
  constexpr int E = R1 * C;
  __shared__ uint64_t lds[E];
  const int mi = map.mod[blockIdx.y];
  const uint64_t q = mc[mi].q;
  uint64_t *p = buf + (size_t)map.row[blockIdx.y] * N + blockIdx.x * C;
  const uint64_t *w_ = itw + (size_t)mi * N;
  const uint64_t *wp_ = itws + (size_t)mi * N;
  for (int e = threadIdx.x; e < E; e += kThreads) lds[e] = p[(e / C) * R2 + (e % C)];
  __syncthreads();
#pragma unroll
  for (int s = LOG_R1 - 1; s >= 0; s--) {
    const int t = R1 >> (s + 1);
    for (int b = threadIdx.x; b < (R1 / 2) * C; b += kThreads) {
      const int c = b % C, k = b / C;
      const int grp = k / t;
      const int j = grp * 2 * t + (k % t);
      const int widx = (1 << s) + grp;
      uint64_t x = lds[j * C + c], y = lds[(j + t) * C + c];
      gs_bfly(x, y, w_[widx], wp_[widx], q);
      lds[j * C + c] = x;
      lds[(j + t) * C + c] = y;
    }
    __syncthreads();
  }
  uint64_t sw, swp, sa;
  if (use_scale) {
    sw = sc.w[blockIdx.y];
    swp = sc.wp[blockIdx.y];
    sa = sc.add[blockIdx.y];
  } else {
    sw = mc[mi].ninv;
    swp = mc[mi].ninv_shoup;
    sa = 0;
  }
  for (int e = threadIdx.x; e < E; e += kThreads) {
    uint64_t v = shoup(lds[e], sw, swp, q);
    p[(e / C) * R2 + (e % C)] = add_mod(v, sa, q);
  }
}

template <int A, int B>
int run_forward(hck_context *ctx, uint64_t *buf, const LimbMap &map) {
  constexpr int R1 = 1 << A, R2 = 1 << B, N = R1 * R2;
  constexpr int C = (kTile / R1) < R2 ? (kTile / R1) : R2;
  constexpr int ROWS = (kTile / R2) < R1 ? (kTile / R2) : R1;
  timing_begin(ctx, "ntt_fwd_strided", 16.0 * N * map.n, 0.5 * N * A * map.n);
  k_fwd_strided<A, B><<<dim3(R2 / C, map.n), kThreads, 0, ctx->stream>>>(
      buf, map, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
  timing_end(ctx);
  timing_begin(ctx, "ntt_fwd_contig", 16.0 * N * map.n, 0.5 * N * B * map.n);
  k_fwd_contig<A, B><<<dim3(R1 / ROWS, map.n), kThreads, 0, ctx->stream>>>(
      buf, map, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

template <int A, int B>
int run_inverse(hck_context *ctx, uint64_t *buf, const LimbMap &map, const RowScale *sc) {
  constexpr int R1 = 1 << A, R2 = 1 << B, N = R1 * R2;
  constexpr int C = (kTile / R1) < R2 ? (kTile / R1) : R2;
  constexpr int ROWS = (kTile / R2) < R1 ? (kTile / R2) : R1;
  timing_begin(ctx, "ntt_inv_contig", 16.0 * N * map.n, 0.5 * N * B * map.n);
  k_inv_contig<A, B><<<dim3(R1 / ROWS, map.n), kThreads, 0, ctx->stream>>>(
      buf, map, ctx->d_mod, ctx->d_itw, ctx->d_itw_shoup);
  timing_end(ctx);
  RowScale dummy;
  timing_begin(ctx, "ntt_inv_strided", 16.0 * N * map.n, (0.5 * A + 1) * N * map.n);
  k_inv_strided<A, B><<<dim3(R2 / C, map.n), kThreads, 0, ctx->stream>>>(
      buf, map, ctx->d_mod, ctx->d_itw, ctx->d_itw_shoup, sc ? *sc : dummy, sc ? 1 : 0);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

}  // namespace

int ntt_forward(hck_context *ctx, uint64_t *buf, const LimbMap &map) {
  if (map.n == 0) return HCK_OK;
  switch (ctx->log_n) {
    case 10: return run_forward<5, 5>(ctx, buf, map);
    case 11: return run_forward<6, 5>(ctx, buf, map);
    case 12: return run_forward<6, 6>(ctx, buf, map);
    case 13: return run_forward<7, 6>(ctx, buf, map);
    case 14: return run_forward<7, 7>(ctx, buf, map);
    case 15: return run_forward<8, 7>(ctx, buf, map);
    case 16: return run_forward<8, 8>(ctx, buf, map);
    case 17: return run_forward<9, 8>(ctx, buf, map);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

int ntt_inverse(hck_context *ctx, uint64_t *buf, const LimbMap &map, const RowScale *sc) {
  if (map.n == 0) return HCK_OK;
  if (sc && map.n > (uint32_t)kMaxLimbs) return set_error(HCK_EINVAL, "too many scaled rows");
  switch (ctx->log_n) {
    case 10: return run_inverse<5, 5>(ctx, buf, map, sc);
    case 11: return run_inverse<6, 5>(ctx, buf, map, sc);
    case 12: return run_inverse<6, 6>(ctx, buf, map, sc);
    case 13: return run_inverse<7, 6>(ctx, buf, map, sc);
    case 14: return run_inverse<7, 7>(ctx, buf, map, sc);
    case 15: return run_inverse<8, 7>(ctx, buf, map, sc);
    case 16: return run_inverse<8, 8>(ctx, buf, map, sc);
    case 17: return run_inverse<9, 8>(ctx, buf, map, sc);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

}  // namespace hck
