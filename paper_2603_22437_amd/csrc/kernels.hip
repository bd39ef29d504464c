// Element-wise, automorphism, basis-conversion and key-switch kernels.
//
// Layout: a polynomial is [limb][N] 64-bit words, limb-major, each limb
// contiguous; kernels index limbs through a LimbMap (row in the buffer,
// modulus index) so that one launch covers every limb of an operation.
#include "internal.h"

namespace hck {

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_copy(uint64_t *__restrict__ dst,
                                                   const uint64_t *__restrict__ src,
                                                   size_t words) {
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  size_t stride = (size_t)gridDim.x * kThreads;
  for (; i < words; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(kThreads) void k_addsub(uint64_t *out, const uint64_t *a,
                                                     const uint64_t *b, LimbMap map,
                                                     const ModConst *__restrict__ mc, int n,
                                                     int op) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const size_t off = (size_t)map.row[blockIdx.y] * n + i;
  const uint64_t q = mc[map.mod[blockIdx.y]].q;
  uint64_t x = a[off];
  uint64_t r;
  if (op == 0)
    r = add_mod(x, b[off], q);
  else if (op == 1)
    r = sub_mod(x, b[off], q);
  else
    r = x == 0 ? 0 : q - x;
  out[off] = r;
}

// out = sum of n inputs mod q, row by row (rows of `map`)
struct SumArgs {
  const uint64_t *in[kSumInputs];
  uint32_t n;
};

__global__ __launch_bounds__(kThreads) void k_sum_many(uint64_t *out, SumArgs sa, LimbMap map,
                                                       const ModConst *__restrict__ mc, int n) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const size_t off = (size_t)map.row[blockIdx.y] * n + i;
  const uint64_t q = mc[map.mod[blockIdx.y]].q;
  uint64_t acc = sa.in[0][off];
  for (uint32_t k = 1; k < sa.n; k++) acc = add_mod(acc, sa.in[k][off], q);
  out[off] = acc;
}

// out = sum of phi_{g_k}(in_k) mod q (NTT-domain automorphism gathers; g = 1
// reads in place), row by row
struct GatherSumArgs {
  const uint64_t *in[kSumInputs];
  uint32_t galois[kSumInputs];
  uint32_t n;
};

__global__ __launch_bounds__(kThreads) void k_gather_sum(uint64_t *out, GatherSumArgs ga,
                                                         LimbMap map,
                                                         const ModConst *__restrict__ mc,
                                                         int log_n) {
  const uint32_t n = 1u << log_n;
  const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
  const size_t row = (size_t)map.row[blockIdx.y] * n;
  const uint64_t q = mc[map.mod[blockIdx.y]].q;
  const uint32_t shift = 32 - log_n;
  const uint32_t e = 2 * (__brev(j) >> shift) + 1;
  uint64_t acc = 0;
  for (uint32_t k = 0; k < ga.n; k++) {
    const uint32_t src_e = (uint32_t)(((uint64_t)e * ga.galois[k]) & (2 * n - 1));
    const uint32_t src = __brev((src_e - 1) >> 1) >> shift;
    acc = add_mod(acc, ga.in[k][row + src], q);
  }
  out[row + j] = acc;
}

// Calibration: chains of dependent Shoup products a <- a w mod q (the
// modular product of every NTT butterfly), 8 independent chains per thread,
// results folded into one word per thread so nothing is optimized away.
__global__ __launch_bounds__(kThreads) void k_mulmod_rate(uint64_t *out, uint64_t q, uint64_t w,
                                                          uint64_t wp, int iters) {
  const uint64_t tid = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  uint64_t x[8];
#pragma unroll
  for (int k = 0; k < 8; k++) x[k] = (tid * 8 + k) % q;
  for (int i = 0; i < iters; i++) {
#pragma unroll
    for (int k = 0; k < 8; k++) x[k] = reduce2(shoup_lazy(x[k], w, wp, q), q);
  }
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) s ^= x[k];
  out[tid] = s;
}

// out = [+-] REDC(a * bm) [+ out]: mode 0 set, 1 add to out, 2 subtract from
// out, 3 set negated (bm in Montgomery form, so REDC gives a * b mod q)
__global__ __launch_bounds__(kThreads) void k_mul_mont(uint64_t *out, const uint64_t *a,
                                                       const uint64_t *bm, LimbMap map,
                                                       const ModConst *__restrict__ mc, int n,
                                                       int mode) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const size_t off = (size_t)map.row[blockIdx.y] * n + i;
  const ModConst m = mc[map.mod[blockIdx.y]];
  uint64_t r = redc(mul_wide(a[off], bm[off]), m.q, m.qinv);
  if (mode == 1) r = add_mod(out[off], r, m.q);
  else if (mode == 2) r = sub_mod(out[off], r, m.q);
  else if (mode == 3) r = r == 0 ? 0 : m.q - r;
  out[off] = r;
}

__global__ __launch_bounds__(kThreads) void k_to_mont(uint64_t *buf, LimbMap map,
                                                      const ModConst *__restrict__ mc, int n,
                                                      int to) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const size_t off = (size_t)map.row[blockIdx.y] * n + i;
  const ModConst m = mc[map.mod[blockIdx.y]];
  const uint64_t x = buf[off];
  if (to) {
    buf[off] = shoup(x, m.r64, m.r64_shoup, m.q);
  } else {
    u128 t;
    t.lo = x;
    t.hi = 0;
    buf[off] = redc(t, m.q, m.qinv);
  }
}

// (a0, a1) x (b0, b1) -> (a0 b0, a0 b1 + a1 b0, a1 b1); plain operands, so
// each REDC result (x 2^-64) is brought back by a REDC with 2^128 mod q.
__global__ __launch_bounds__(kThreads) void k_tensor(uint64_t *out, const uint64_t *a,
                                                     const uint64_t *b, size_t ps, LimbMap map,
                                                     const ModConst *__restrict__ mc, int n) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const size_t off = (size_t)map.row[blockIdx.y] * n + i;
  const ModConst m = mc[map.mod[blockIdx.y]];
  const uint64_t a0 = a[off], a1 = a[off + ps], b0 = b[off], b1 = b[off + ps];
  uint64_t d0 = redc(mul_wide(a0, b0), m.q, m.qinv);
  u128 x = mul_wide(a0, b1);
  mac_wide(x, a1, b0);
  uint64_t d1 = redc(x, m.q, m.qinv);
  uint64_t d2 = redc(mul_wide(a1, b1), m.q, m.qinv);
  out[off] = redc(mul_wide(d0, m.r2), m.q, m.qinv);
  out[off + ps] = redc(mul_wide(d1, m.r2), m.q, m.qinv);
  out[off + 2 * ps] = redc(mul_wide(d2, m.r2), m.q, m.qinv);
}

// Galois automorphism in the bit-reversed evaluation domain: slot j holds the
// value at psi^(2 brv(j) + 1), and phi_g(a)(x) = a(x^g), so slot j of the
// output is slot brv(((2 brv(j) + 1) g mod 2N - 1) / 2) of the input.
__global__ __launch_bounds__(kThreads) void k_automorphism(uint64_t *__restrict__ out,
                                                           const uint64_t *__restrict__ in,
                                                           size_t ps, LimbMap map, int log_n,
                                                           uint32_t g) {
  const uint32_t n = 1u << log_n;
  const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
  const uint32_t shift = 32 - log_n;
  const uint32_t e = 2 * (__brev(j) >> shift) + 1;
  const uint32_t src_e = (uint32_t)(((uint64_t)e * g) & (2 * n - 1));
  const uint32_t src = __brev((src_e - 1) >> 1) >> shift;
  const size_t row = (size_t)map.row[blockIdx.y] * n + blockIdx.z * ps;
  out[row + j] = in[row + src];
}

__global__ __launch_bounds__(kThreads) void k_embed_small(uint64_t *out, const int32_t *small,
                                                          LimbMap map,
                                                          const ModConst *__restrict__ mc,
                                                          int n) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const uint64_t q = mc[map.mod[blockIdx.y]].q;
  const int32_t v = small[i];
  out[(size_t)map.row[blockIdx.y] * n + i] = v < 0 ? q - (uint64_t)(-(int64_t)v) : (uint64_t)v;
}

// out[r] += REDC(in[r] c_r): adds a per-row constant multiple of a
// Montgomery-form operand.
__global__ __launch_bounds__(kThreads) void k_scalar_mac(uint64_t *out, const uint64_t *in,
                                                         LimbMap map, RowScale sc,
                                                         const ModConst *__restrict__ mc, int n) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const size_t off = (size_t)map.row[blockIdx.y] * n + i;
  const ModConst m = mc[map.mod[blockIdx.y]];
  out[off] = add_mod(out[off], redc(mul_wide(in[off], sc.w[blockIdx.y]), m.q, m.qinv), m.q);
}

dim3 grid_rows(const hck_context *ctx, uint32_t rows, uint32_t z = 1) {
  return dim3(ctx->n / kThreads, rows, z);
}

}  // namespace

int launch_copy(hck_context *ctx, uint64_t *dst, const uint64_t *src, size_t words) {
  if (words == 0 || dst == src) return HCK_OK;
  unsigned blocks = (unsigned)std::min<size_t>((words + kThreads - 1) / kThreads, 8192);
  timing_begin(ctx, "copy", dim3(blocks), 16.0 * words);
  k_copy<<<blocks, kThreads, 0, ctx->stream>>>(dst, src, words);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

int launch_addsub(hck_context *ctx, uint64_t *out, const uint64_t *a, const uint64_t *b,
                  const LimbMap &map, int op) {
  if (map.n == 0) return HCK_OK;
  timing_begin(ctx, "addsub", grid_rows(ctx, map.n), 24.0 * ctx->n * map.n);
  k_addsub<<<grid_rows(ctx, map.n), kThreads, 0, ctx->stream>>>(out, a, b, map, ctx->d_mod,
                                                                 ctx->n, op);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

int launch_sum_many(hck_context *ctx, uint64_t *out, const uint64_t *const *in, uint32_t n_in,
                    const LimbMap &map) {
  if (n_in == 0) return set_error(HCK_EINVAL, "empty sum");
  if (map.n == 0) return HCK_OK;
  // chunks of kSumInputs; later chunks add to the partial sum in `out`
  for (uint32_t s = 0; s < n_in;) {
    SumArgs sa;
    sa.n = 0;
    if (s > 0) sa.in[sa.n++] = out;
    while (s < n_in && sa.n < (uint32_t)kSumInputs) sa.in[sa.n++] = in[s++];
    timing_begin(ctx, "sum_many", grid_rows(ctx, map.n), 8.0 * ctx->n * map.n * (sa.n + 1));
    k_sum_many<<<grid_rows(ctx, map.n), kThreads, 0, ctx->stream>>>(out, sa, map, ctx->d_mod,
                                                                      ctx->n);
    timing_end(ctx);
    HCK_HIP(ctx, hipGetLastError());
  }
  return HCK_OK;
}

int launch_gather_sum(hck_context *ctx, uint64_t *out, const uint64_t *const *in,
                      const uint32_t *galois, uint32_t n_in, const LimbMap &map) {
  if (n_in == 0) return set_error(HCK_EINVAL, "empty sum");
  if (map.n == 0) return HCK_OK;
  // chunks of kSumInputs; later chunks add to the partial sum in `out`
  for (uint32_t s = 0; s < n_in;) {
    GatherSumArgs ga;
    ga.n = 0;
    if (s > 0) {
      ga.in[0] = out;
      ga.galois[0] = 1;
      ga.n = 1;
    }
    while (s < n_in && ga.n < (uint32_t)kSumInputs) {
      ga.in[ga.n] = in[s];
      ga.galois[ga.n++] = galois[s++];
    }
    timing_begin(ctx, "gather_sum", grid_rows(ctx, map.n), 8.0 * ctx->n * map.n * (ga.n + 1));
    k_gather_sum<<<grid_rows(ctx, map.n), kThreads, 0, ctx->stream>>>(out, ga, map, ctx->d_mod,
                                                                        (int)ctx->log_n);
    timing_end(ctx);
    HCK_HIP(ctx, hipGetLastError());
  }
  return HCK_OK;
}

int measure_mulmod_rate(hck_context *ctx, double *tera_per_s) {
  const unsigned blocks = 256 * 16;
  const int iters = 1024;
  uint64_t *buf = nullptr;
  int rc = dev_alloc(ctx, &buf, (size_t)blocks * kThreads);
  if (rc) return rc;
  const uint64_t q = ctx->mods[0];
  const uint64_t w = h_powmod(3, 12345, q), wp = h_shoup(w, q);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    k_mulmod_rate<<<blocks, kThreads, 0, ctx->stream>>>(buf, q, w, wp, iters);  // warm-up
    e = hipEventRecord(e0, ctx->stream);
  }
  if (e == hipSuccess) {
    k_mulmod_rate<<<blocks, kThreads, 0, ctx->stream>>>(buf, q, w, wp, iters);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  dev_free(ctx, buf);
  if (e != hipSuccess) return check_hip(ctx, e, "mulmod rate");
  *tera_per_s = (double)blocks * kThreads * iters * 8 / (ms * 1e-3) / 1e12;
  return HCK_OK;
}

int launch_mul_mont(hck_context *ctx, uint64_t *out, const uint64_t *a, const uint64_t *bm,
                    const LimbMap &map, int mode) {
  if (map.n == 0) return HCK_OK;
  timing_begin(ctx, "mul_plain", grid_rows(ctx, map.n),
               ((mode == 1 || mode == 2) ? 32.0 : 24.0) * ctx->n * map.n, (double)ctx->n * map.n);
  k_mul_mont<<<grid_rows(ctx, map.n), kThreads, 0, ctx->stream>>>(out, a, bm, map, ctx->d_mod,
                                                                   ctx->n, mode);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

int launch_to_mont(hck_context *ctx, uint64_t *buf, const LimbMap &map, bool to) {
  if (map.n == 0) return HCK_OK;
  timing_begin(ctx, "mont", grid_rows(ctx, map.n), 16.0 * ctx->n * map.n, (double)ctx->n * map.n);
  k_to_mont<<<grid_rows(ctx, map.n), kThreads, 0, ctx->stream>>>(buf, map, ctx->d_mod, ctx->n,
                                                                  to ? 1 : 0);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

int launch_tensor(hck_context *ctx, uint64_t *out, const uint64_t *a, const uint64_t *b,
                  size_t poly_stride, const LimbMap &map) {
  timing_begin(ctx, "tensor", grid_rows(ctx, map.n), 56.0 * ctx->n * map.n, 4.0 * ctx->n * map.n);
  k_tensor<<<grid_rows(ctx, map.n), kThreads, 0, ctx->stream>>>(out, a, b, poly_stride, map,
                                                                 ctx->d_mod, ctx->n);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

int launch_automorphism(hck_context *ctx, uint64_t *out, const uint64_t *in, size_t poly_stride,
                        uint32_t polys, const LimbMap &map, uint32_t galois) {
  timing_begin(ctx, "automorphism", grid_rows(ctx, map.n, polys), 16.0 * ctx->n * map.n * polys);
  k_automorphism<<<grid_rows(ctx, map.n, polys), kThreads, 0, ctx->stream>>>(
      out, in, poly_stride, map, (int)ctx->log_n, galois);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

int launch_embed_small(hck_context *ctx, uint64_t *out, const int32_t *small, const LimbMap &map) {
  timing_begin(ctx, "embed", grid_rows(ctx, map.n), (8.0 * map.n + 4.0) * ctx->n);
  k_embed_small<<<grid_rows(ctx, map.n), kThreads, 0, ctx->stream>>>(out, small, map, ctx->d_mod,
                                                                      ctx->n);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

int launch_scalar_mac(hck_context *ctx, uint64_t *out, const uint64_t *in, const LimbMap &map,
                      const RowScale &sc) {
  if (map.n == 0) return HCK_OK;
  if (map.n > (uint32_t)kMaxLimbs) return set_error(HCK_EINVAL, "too many rows");
  timing_begin(ctx, "scalar_mac", grid_rows(ctx, map.n), 24.0 * ctx->n * map.n,
               (double)ctx->n * map.n);
  k_scalar_mac<<<grid_rows(ctx, map.n), kThreads, 0, ctx->stream>>>(out, in, map, sc, ctx->d_mod,
                                                                     ctx->n);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

}  // namespace hck
