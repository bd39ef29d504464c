// Negacyclic NTT / inverse NTT over many limbs in one launch: the two
// passes of ntt_core.h, each a kernel over every listed limb.
#include "ntt_core.h"

namespace hck {

namespace {

// One pass over the rows of `map`.  Reads from src (or dst when src is null)
// and writes dst.  Forward strided: [0, 4q) in and out; forward contiguous:
// [0, 4q) in, [0, q) out; inverse contiguous: [0, 2q) in and out; inverse
// strided: [0, 2q) in, out = x N^-1 fully reduced, or with scale_period > 0
// x sc.w[k] + sc.add[k], k = (row list index) mod scale_period.
template <int LOGR, int LOGN, bool STRIDED, bool INVERSE>
__global__ __launch_bounds__(kNttThreads) void k_ntt_pass(uint64_t *__restrict__ dst,
                                                          const uint64_t *__restrict__ src,
                                                          LimbMap map,
                                                          const ModConst *__restrict__ mc,
                                                          const uint64_t *__restrict__ tw,
                                                          const uint64_t *__restrict__ tws,
                                                          const uint64_t *__restrict__ tt,
                                                          const uint64_t *__restrict__ tts,
                                                          RowScale sc, int scale_period) {
  using G = Pass<LOGR, LOGN, STRIDED>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const int mi = map.mod[blockIdx.y];
  const uint64_t q = mc[mi].q;
  const Qn qm = qn(mc[mi]);
  const size_t roff = (size_t)map.row[blockIdx.y] * G::N;
  uint64_t *out = dst + roff;
  const uint64_t *in = (src ? src : dst) + roff;
  const uint64_t *w = tw + (size_t)mi * G::N;
  const uint64_t *wp = tws + (size_t)mi * G::N;
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  uint64_t x[P];
  if (!INVERSE) {
#pragma unroll
    for (int i = 0; i < P; i++) x[i] = in[G::gaddr(g, G::ipoint(r, i))];
    if constexpr (!STRIDED) G::twist(x, g, r, tt + (size_t)mi * G::N, tts + (size_t)mi * G::N, qm);
    G::forward(lds, x, c, r, g, w, wp, qm);
    if (STRIDED) {
#pragma unroll
      for (int v = 0; v < P; v++) out[G::gaddr(g, G::bpoint(r, v))] = x[v];
    } else {
#pragma unroll
      for (int v = 0; v < P; v++) x[v] = reduce4(x[v], qm);
      G::to_interleaved(lds, x, c, r);
#pragma unroll
      for (int i = 0; i < P; i++) out[G::gaddr(g, G::ipoint(r, i))] = x[i];
    }
  } else {
    if (STRIDED) {
#pragma unroll
      for (int v = 0; v < P; v++) x[v] = in[G::gaddr(g, G::bpoint(r, v))];
    } else {
#pragma unroll
      for (int i = 0; i < P; i++) x[i] = in[G::gaddr(g, G::ipoint(r, i))];
      G::to_blocked(lds, x, c, r);
    }
    G::inverse(lds, x, c, r, g, w, wp, qm);
    if constexpr (STRIDED) {
      uint64_t sw, swp, sa;
      if (scale_period) {
        const int k = blockIdx.y % scale_period;
        sw = sc.w[k];
        swp = sc.wp[k];
        sa = sc.add[k];
      } else {
        sw = mc[mi].ninv;
        swp = mc[mi].ninv_shoup;
        sa = 0;
      }
#pragma unroll
      for (int i = 0; i < P; i++)
        out[G::gaddr(g, G::ipoint(r, i))] = add_mod(shoup(x[i], sw, swp, q), sa, q);
    } else {
      G::twist(x, g, r, tt + (size_t)mi * G::N, tts + (size_t)mi * G::N, qm);
#pragma unroll
      for (int i = 0; i < P; i++) out[G::gaddr(g, G::ipoint(r, i))] = x[i];
    }
  }
}

// Rescale, forward half (strided pass): the dropped limb of polynomial
// blockIdx.z (coefficient form, [0, q_l)) is lifted to its centred value
// (v - q_l when v > (q_l - 1) / 2) modulo target limb i = blockIdx.y as it is
// loaded, then the forward strided pass of limb i runs on it.  last holds one
// limb per polynomial; tmp gets rows z level + i.  qmod.add[i] = q_l mod q_i.
template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_rescale_strided(
    uint64_t *__restrict__ tmp, const uint64_t *__restrict__ last, uint32_t level,
    RowScale qmod, const ModConst *__restrict__ mc, const uint64_t *__restrict__ tw,
    const uint64_t *__restrict__ tws) {
  using G = Pass<split_a(LOGN), LOGN, true>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const uint32_t i = blockIdx.y, z = blockIdx.z;
  const ModConst m = mc[i];
  const uint64_t half = (mc[level].q - 1) / 2, ql_i = qmod.add[i];
  const uint64_t *src = last + (size_t)z * G::N;
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  uint64_t x[P];
#pragma unroll
  for (int k = 0; k < P; k++) {
    const uint64_t v = src[G::gaddr(g, G::ipoint(r, k))];
    const uint64_t t = shoup(v, 1, m.one_shoup, m.q);
    x[k] = v > half ? sub_mod(t, ql_i, m.q) : t;
  }
  G::forward(lds, x, c, r, g, tw + (size_t)i * G::N, tws + (size_t)i * G::N, qn(m));
  uint64_t *out = tmp + ((size_t)z * level + i) * G::N;
#pragma unroll
  for (int v = 0; v < P; v++) out[G::gaddr(g, G::bpoint(r, v))] = x[v];
}

// Rescale, tail (contiguous pass): finishes the forward transform of the
// lifted limb t and writes out_i = (c_i - t) q_l^-1 mod q_i for i < level
// (inv.w / inv.wp: q_l^-1 mod q_i and its Shoup companion).  out may be c.
template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_rescale_contig_tail(
    uint64_t *out, const uint64_t *c_in, const uint64_t *__restrict__ tmp, size_t ps,
    uint32_t level, RowScale inv, const ModConst *__restrict__ mc,
    const uint64_t *__restrict__ tw, const uint64_t *__restrict__ tws,
    const uint64_t *__restrict__ tt, const uint64_t *__restrict__ tts) {
  using G = Pass<split_b(LOGN), LOGN, false>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const uint32_t i = blockIdx.y, z = blockIdx.z;
  const uint64_t q = mc[i].q;
  const Qn qm = qn(mc[i]);
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  const uint64_t *tin = tmp + ((size_t)z * level + i) * G::N;
  uint64_t x[P];
#pragma unroll
  for (int k = 0; k < P; k++) x[k] = tin[G::gaddr(g, G::ipoint(r, k))];
  G::twist(x, g, r, tt + (size_t)i * G::N, tts + (size_t)i * G::N, qm);
  G::forward(lds, x, c, r, g, tw + (size_t)i * G::N, tws + (size_t)i * G::N, qm);
#pragma unroll
  for (int v = 0; v < P; v++) x[v] = reduce4(x[v], qm);
  G::to_interleaved(lds, x, c, r);
  const size_t off = (size_t)z * ps + (size_t)i * G::N;
  const uint64_t w = inv.w[i], wp = inv.wp[i];
#pragma unroll
  for (int k = 0; k < P; k++) {
    const size_t pos = off + G::gaddr(g, G::ipoint(r, k));
    out[pos] = shoup(sub_mod(c_in[pos], x[k], q), w, wp, q);
  }
}

template <int LOGN>
int run_rescale(hck_context *ctx, uint64_t *out, const uint64_t *in, const uint64_t *last,
                uint64_t *tmp, uint32_t level, uint32_t polys) {
  constexpr int A = split_a(LOGN), B = split_b(LOGN);
  constexpr double N = (double)(1 << LOGN);
  using GA = Pass<A, LOGN, true>;
  using GB = Pass<B, LOGN, false>;
  RowScale qmod, inv;
  for (uint32_t i = 0; i < level; i++) {
    qmod.add[i] = ctx->mods[level] % ctx->mods[i];
    qmod.w[i] = qmod.wp[i] = 0;
    inv.w[i] = ctx->rescale_inv[level][i];
    inv.wp[i] = h_shoup(inv.w[i], ctx->mods[i]);
    inv.add[i] = 0;
  }
  const size_t ps = (size_t)ctx->L * ctx->n;
  timing_begin(ctx, "rescale_strided", dim3(GA::BLOCKS, level, polys),
               8.0 * N * polys * (1 + level), N * (1 + 0.5 * A) * polys * level);
  k_rescale_strided<LOGN><<<dim3(GA::BLOCKS, level, polys), kNttThreads, 0, ctx->stream>>>(
      tmp, last, level, qmod, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
  timing_end(ctx);
  timing_begin(ctx, "rescale_tail", dim3(GB::BLOCKS, level, polys), 24.0 * N * polys * level,
               N * (1 + 0.5 * B) * polys * level);
  k_rescale_contig_tail<LOGN><<<dim3(GB::BLOCKS, level, polys), kNttThreads, 0, ctx->stream>>>(
      out, in, tmp, ps, level, inv, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup, ctx->d_ttw,
      ctx->d_ttw_shoup);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

// One pass of the split N = 2^A x 2^(LOGN - A): the strided pass runs the
// first A stages (R1 = 2^A points per sub-transform), the contiguous pass the
// rest; tt/tts are the contiguous pass's twist tables for that split.
template <int LOGN, int A, bool STRIDED, bool INVERSE>
void launch_split(hck_context *ctx, uint64_t *dst, const uint64_t *src, const LimbMap &map,
                  const RowScale *sc, int period, const uint64_t *tt, const uint64_t *tts) {
  constexpr int LOGR = STRIDED ? A : LOGN - A;
  constexpr int N = 1 << LOGN;
  using G = Pass<LOGR, LOGN, STRIDED>;
  static const char *names[2][2] = {{"ntt_fwd_contig", "ntt_fwd_strided"},
                                    {"ntt_inv_contig", "ntt_inv_strided"}};
  const double mm = (0.5 * LOGR + (INVERSE && STRIDED ? 1 : 0)) * N * map.n;
  RowScale dummy;
  timing_begin(ctx, names[INVERSE][STRIDED], dim3(G::BLOCKS, map.n), 16.0 * N * map.n, mm);
  k_ntt_pass<LOGR, LOGN, STRIDED, INVERSE><<<dim3(G::BLOCKS, map.n), kNttThreads, 0, ctx->stream>>>(
      dst, src, map, ctx->d_mod, INVERSE ? ctx->d_itw : ctx->d_tw,
      INVERSE ? ctx->d_itw_shoup : ctx->d_tw_shoup, tt, tts, sc ? *sc : dummy,
      sc ? (period ? period : (int)map.n) : 0);
  timing_end(ctx);
}

template <int LOGN, bool STRIDED, bool INVERSE>
void launch_pass(hck_context *ctx, uint64_t *dst, const uint64_t *src, const LimbMap &map,
                 const RowScale *sc, int period = 0) {
  launch_split<LOGN, split_a(LOGN), STRIDED, INVERSE>(
      ctx, dst, src, map, sc, period, INVERSE ? ctx->d_ittw : ctx->d_ttw,
      INVERSE ? ctx->d_ittw_shoup : ctx->d_ttw_shoup);
}

// whether the split 2^A x 2^(LOGN - A) has both passes: at least one
// workgroup per limb, a contiguous sub-transform inside one wavefront, and
// each pass's LDS within a workgroup's share of gfx950's 160 KiB
template <int LOGN, int A>
constexpr bool split_ok() {
  if (A < 2 || LOGN - A < 2) return false;
  using S = Pass<A, LOGN, true>;
  using C = Pass<LOGN - A, LOGN, false>;
  return S::BLOCKS >= 1 && C::BLOCKS >= 1 && C::T <= 64 && 64 % C::T == 0 &&
         S::LDS_WORDS * 8 <= 80 * 1024 && C::LDS_WORDS * 8 <= 80 * 1024;
}

// full transforms on the split the context's NTT tuner chose (ctx->ntt_a;
// the default split_a(LOGN) when 0), one step either side of the default
template <int LOGN, int A>
int forward_split(hck_context *ctx, uint64_t *dst, const uint64_t *src, const LimbMap &map) {
  if constexpr (split_ok<LOGN, A>()) {
    const uint64_t *const *tt = split_twists(ctx, A);
    if (!tt) return set_error(HCK_EINVAL, "NTT split tables not built");
    launch_split<LOGN, A, true, false>(ctx, dst, src, map, nullptr, 0, nullptr, nullptr);
    launch_split<LOGN, A, false, false>(ctx, dst, nullptr, map, nullptr, 0, tt[0], tt[1]);
    HCK_HIP(ctx, hipGetLastError());
    return HCK_OK;
  } else {
    return set_error(HCK_EINVAL, "NTT split not available for this ring");
  }
}

template <int LOGN, int A>
int inverse_split(hck_context *ctx, uint64_t *dst, const uint64_t *src, const LimbMap &map,
                  const RowScale *sc) {
  if constexpr (split_ok<LOGN, A>()) {
    const uint64_t *const *tt = split_twists(ctx, A);
    if (!tt) return set_error(HCK_EINVAL, "NTT split tables not built");
    launch_split<LOGN, A, false, true>(ctx, dst, src, map, nullptr, 0, tt[2], tt[3]);
    launch_split<LOGN, A, true, true>(ctx, dst, nullptr, map, sc, 0, nullptr, nullptr);
    HCK_HIP(ctx, hipGetLastError());
    return HCK_OK;
  } else {
    return set_error(HCK_EINVAL, "NTT split not available for this ring");
  }
}

template <int LOGN>
int run_forward(hck_context *ctx, uint64_t *dst, const uint64_t *src, const LimbMap &map) {
  constexpr int A = split_a(LOGN);
  const int a = ctx->ntt_a ? ctx->ntt_a : A;
  if (a == A - 1) return forward_split<LOGN, A - 1>(ctx, dst, src, map);
  if (a == A + 1) return forward_split<LOGN, A + 1>(ctx, dst, src, map);
  return forward_split<LOGN, A>(ctx, dst, src, map);
}

template <int LOGN>
int run_inverse(hck_context *ctx, uint64_t *dst, const uint64_t *src, const LimbMap &map,
                const RowScale *sc) {
  constexpr int A = split_a(LOGN);
  const int a = ctx->ntt_a ? ctx->ntt_a : A;
  if (a == A - 1) return inverse_split<LOGN, A - 1>(ctx, dst, src, map, sc);
  if (a == A + 1) return inverse_split<LOGN, A + 1>(ctx, dst, src, map, sc);
  return inverse_split<LOGN, A>(ctx, dst, src, map, sc);
}

template <int LOGN>
int run_one(hck_context *ctx, uint64_t *buf, const LimbMap &map, bool inverse, bool strided,
            const RowScale *sc, int period) {
  if (!inverse && strided) launch_pass<LOGN, true, false>(ctx, buf, nullptr, map, nullptr);
  if (!inverse && !strided) launch_pass<LOGN, false, false>(ctx, buf, nullptr, map, nullptr);
  if (inverse && !strided) launch_pass<LOGN, false, true>(ctx, buf, nullptr, map, nullptr);
  if (inverse && strided) launch_pass<LOGN, true, true>(ctx, buf, nullptr, map, sc, period);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

}  // namespace

bool ntt_split_available(uint32_t log_n, int a) {
  switch (log_n) {
#define HCK_SPLITS(L)                                                                   \
  case L:                                                                                \
    return (a == split_a(L) - 1 && split_ok<L, split_a(L) - 1>()) || a == split_a(L) || \
           (a == split_a(L) + 1 && split_ok<L, split_a(L) + 1>());
    HCK_SPLITS(11)
    HCK_SPLITS(12)
    HCK_SPLITS(13)
    HCK_SPLITS(14)
    HCK_SPLITS(15)
    HCK_SPLITS(16)
    HCK_SPLITS(17)
#undef HCK_SPLITS
    default:
      return false;
  }
}

int ntt_forward(hck_context *ctx, uint64_t *buf, const LimbMap &map) {
  return ntt_forward_oop(ctx, buf, nullptr, map);
}

int ntt_forward_oop(hck_context *ctx, uint64_t *dst, const uint64_t *src, const LimbMap &map) {
  if (map.n == 0) return HCK_OK;
  switch (ctx->log_n) {
    case 11: return run_forward<11>(ctx, dst, src, map);
    case 12: return run_forward<12>(ctx, dst, src, map);
    case 13: return run_forward<13>(ctx, dst, src, map);
    case 14: return run_forward<14>(ctx, dst, src, map);
    case 15: return run_forward<15>(ctx, dst, src, map);
    case 16: return run_forward<16>(ctx, dst, src, map);
    case 17: return run_forward<17>(ctx, dst, src, map);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

int ntt_inverse(hck_context *ctx, uint64_t *buf, const LimbMap &map, const RowScale *sc) {
  return ntt_inverse_oop(ctx, buf, nullptr, map, sc);
}

int ntt_inverse_oop(hck_context *ctx, uint64_t *dst, const uint64_t *src, const LimbMap &map,
                    const RowScale *sc) {
  if (map.n == 0) return HCK_OK;
  if (sc && map.n > (uint32_t)kMaxLimbs) return set_error(HCK_EINVAL, "too many scaled rows");
  switch (ctx->log_n) {
    case 11: return run_inverse<11>(ctx, dst, src, map, sc);
    case 12: return run_inverse<12>(ctx, dst, src, map, sc);
    case 13: return run_inverse<13>(ctx, dst, src, map, sc);
    case 14: return run_inverse<14>(ctx, dst, src, map, sc);
    case 15: return run_inverse<15>(ctx, dst, src, map, sc);
    case 16: return run_inverse<16>(ctx, dst, src, map, sc);
    case 17: return run_inverse<17>(ctx, dst, src, map, sc);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

int rescale_fused(hck_context *ctx, uint64_t *out, const uint64_t *in, const uint64_t *last,
                  uint64_t *tmp, uint32_t level, uint32_t polys) {
  if (level == 0 || polys == 0) return HCK_OK;
  if (level > (uint32_t)kMaxLimbs) return set_error(HCK_EINVAL, "too many limbs");
  switch (ctx->log_n) {
    case 11: return run_rescale<11>(ctx, out, in, last, tmp, level, polys);
    case 12: return run_rescale<12>(ctx, out, in, last, tmp, level, polys);
    case 13: return run_rescale<13>(ctx, out, in, last, tmp, level, polys);
    case 14: return run_rescale<14>(ctx, out, in, last, tmp, level, polys);
    case 15: return run_rescale<15>(ctx, out, in, last, tmp, level, polys);
    case 16: return run_rescale<16>(ctx, out, in, last, tmp, level, polys);
    case 17: return run_rescale<17>(ctx, out, in, last, tmp, level, polys);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

int ntt_pass(hck_context *ctx, uint64_t *buf, const LimbMap &map, bool inverse, bool strided,
             const RowScale *sc, int period) {
  if (map.n == 0) return HCK_OK;
  const int per = period ? period : (int)map.n;
  if (sc && per > kMaxLimbs) return set_error(HCK_EINVAL, "too many scaled rows");
  switch (ctx->log_n) {
    case 11: return run_one<11>(ctx, buf, map, inverse, strided, sc, period);
    case 12: return run_one<12>(ctx, buf, map, inverse, strided, sc, period);
    case 13: return run_one<13>(ctx, buf, map, inverse, strided, sc, period);
    case 14: return run_one<14>(ctx, buf, map, inverse, strided, sc, period);
    case 15: return run_one<15>(ctx, buf, map, inverse, strided, sc, period);
    case 16: return run_one<16>(ctx, buf, map, inverse, strided, sc, period);
    case 17: return run_one<17>(ctx, buf, map, inverse, strided, sc, period);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

}  // namespace hck
