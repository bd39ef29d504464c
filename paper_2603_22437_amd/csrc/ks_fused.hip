// Hybrid key switching with the basis conversions, the key inner product and
// the ModDown tail fused into the NTT passes (ntt_core.h).
//
// KeySwitch(d) at level l with a switching key swk(s' -> s); d is read through
// the NTT-domain automorphism X -> X^g (g = 1: no automorphism), so a
// rotation never materializes phi_g(c):
//   K1  inverse contiguous pass of phi_g(d) over Q_l -> y          (gather)
//   K2  inverse strided pass, times N^-1 (Q_j / q_i)^-1 per limb    (digit scale)
//   K3  ModUp: per digit j and target limb t not in D_j, the fast basis
//       conversion of y's digit limbs computed at load time, then the
//       forward strided pass -> ext[j][t]
//   K4  per extended limb t: forward contiguous pass of every digit's ext
//       (or phi_g(d) itself on the digit's own limbs), then
//       acc_{0,1}[t] = sum_j d~_j[t] swk_j[t] (keys in Montgomery form)
//   K5  inverse passes of acc's P limbs, times N^-1 (P/p_k)^-1, plus
//       ((P-1)/2) (P/p_k)^-1 (the rounding term of ModDown)
//   K6  ModDown conversion P -> q_i (minus (P-1)/2) at load time, then the
//       forward strided pass -> conv
//   K7  forward contiguous pass of conv, then
//       out_i = (acc_i - conv_i) P^-1 (+ phi_g(addend)_i)
#include "ntt_core.h"

namespace hck {

namespace {

struct KsGeom {
  uint32_t level, nq, ne, L, K, dnum, alpha, nm;
};

struct ModUpRows {
  uint32_t n;
  uint16_t row[kMaxRows];
  uint8_t mod[kMaxRows];
  uint8_t digit[kMaxRows];
};

template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_ks_intt_gather(
    uint64_t *__restrict__ y, const uint64_t *__restrict__ d, uint32_t galois,
    const ModConst *__restrict__ mc, const uint64_t *__restrict__ itw,
    const uint64_t *__restrict__ itws) {
  using G = Pass<split_b(LOGN), LOGN, false>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const int li = blockIdx.y;  // limb i (modulus i)
  const uint64_t q = mc[li].q;
  const size_t roff = (size_t)li * G::N;
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  uint64_t x[P];
#pragma unroll
  for (int i = 0; i < P; i++)
    x[i] = d[roff + galois_src((uint32_t)G::gaddr(g, G::ipoint(r, i)), galois, LOGN)];
  G::to_blocked(lds, x, c, r);
  G::inverse(lds, x, c, r, g, itw + roff, itws + roff, q);
#pragma unroll
  for (int i = 0; i < P; i++) y[roff + G::gaddr(g, G::ipoint(r, i))] = x[i];
}

template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_modup_strided(
    uint64_t *__restrict__ ext, const uint64_t *__restrict__ y, ModUpRows rows,
    const uint64_t *__restrict__ conv, KsGeom kg, const ModConst *__restrict__ mc,
    const uint64_t *__restrict__ tw, const uint64_t *__restrict__ tws) {
  using G = Pass<split_a(LOGN), LOGN, true>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const int mi = rows.mod[blockIdx.y];
  const int j = rows.digit[blockIdx.y];
  const uint32_t lo = j * kg.alpha;
  const uint32_t na = min(kg.alpha, kg.nq - lo);
  const ModConst m = mc[mi];
  const uint64_t *cv = conv + (size_t)j * kg.alpha * kg.nm + mi;
  const uint64_t *src = y + (size_t)lo * G::N;
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  uint64_t x[P];
#pragma unroll
  for (int i = 0; i < P; i++) {
    const size_t pos = G::gaddr(g, G::ipoint(r, i));
    u128 acc;
    acc.lo = acc.hi = 0;
    for (uint32_t a = 0; a < na; a++) mac_wide(acc, src[(size_t)a * G::N + pos], cv[(size_t)a * kg.nm]);
    x[i] = redc(acc, m.q, m.qinv);
  }
  G::forward(lds, x, c, r, g, tw + (size_t)mi * G::N, tws + (size_t)mi * G::N, m.q);
  uint64_t *out = ext + (size_t)rows.row[blockIdx.y] * G::N;
#pragma unroll
  for (int v = 0; v < P; v++) out[G::gaddr(g, G::bpoint(r, v))] = x[v];
}

template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_ks_contig_inner(
    uint64_t *__restrict__ acc, const uint64_t *__restrict__ ext, const uint64_t *__restrict__ d,
    uint32_t galois, const uint64_t *__restrict__ key, KsGeom kg,
    const ModConst *__restrict__ mc, const uint64_t *__restrict__ tw,
    const uint64_t *__restrict__ tws) {
  using G = Pass<split_b(LOGN), LOGN, false>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const uint32_t t = blockIdx.y;
  const uint32_t mi = t < kg.nq ? t : kg.L + (t - kg.nq);
  const ModConst m = mc[mi];
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  const size_t krow = (size_t)kg.nm * G::N;
  uint64_t a0[P], a1[P], x[P];
#pragma unroll
  for (int i = 0; i < P; i++) a0[i] = a1[i] = 0;
  for (uint32_t j = 0; j < kg.dnum; j++) {
    const uint32_t lo = j * kg.alpha;
    if (lo >= kg.nq) break;
    const uint32_t hi = min(lo + kg.alpha, kg.nq);
    if (t >= lo && t < hi) {
#pragma unroll
      for (int i = 0; i < P; i++)
        x[i] = d[(size_t)t * G::N +
                 galois_src((uint32_t)G::gaddr(g, G::ipoint(r, i)), galois, LOGN)];
    } else {
      const uint64_t *e = ext + ((size_t)j * kg.ne + t) * G::N;
#pragma unroll
      for (int i = 0; i < P; i++) x[i] = e[G::gaddr(g, G::ipoint(r, i))];
      G::forward(lds, x, c, r, g, tw + (size_t)mi * G::N, tws + (size_t)mi * G::N, m.q);
#pragma unroll
      for (int v = 0; v < P; v++) x[v] = reduce4(x[v], m.q);
      G::to_interleaved(lds, x, c, r);
    }
    const uint64_t *kb = key + 2 * j * krow + (size_t)mi * G::N;
    const uint64_t *ka = kb + krow;
#pragma unroll
    for (int i = 0; i < P; i++) {
      const size_t pos = G::gaddr(g, G::ipoint(r, i));
      a0[i] = add_mod(a0[i], redc(mul_wide(x[i], kb[pos]), m.q, m.qinv), m.q);
      a1[i] = add_mod(a1[i], redc(mul_wide(x[i], ka[pos]), m.q, m.qinv), m.q);
    }
  }
  uint64_t *o0 = acc + (size_t)t * G::N;
  uint64_t *o1 = acc + ((size_t)kg.ne + t) * G::N;
#pragma unroll
  for (int i = 0; i < P; i++) {
    const size_t pos = G::gaddr(g, G::ipoint(r, i));
    o0[pos] = a0[i];
    o1[pos] = a1[i];
  }
}

template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_moddown_strided(
    uint64_t *__restrict__ conv_out, const uint64_t *__restrict__ acc,
    const uint64_t *__restrict__ down_conv, const uint64_t *__restrict__ hneg, KsGeom kg,
    const ModConst *__restrict__ mc, const uint64_t *__restrict__ tw,
    const uint64_t *__restrict__ tws) {
  using G = Pass<split_a(LOGN), LOGN, true>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const uint32_t p = blockIdx.y / kg.nq, li = blockIdx.y % kg.nq;
  const ModConst m = mc[li];
  const uint64_t h = hneg[li];
  const uint64_t *src = acc + ((size_t)p * kg.ne + kg.nq) * G::N;
  const uint64_t *cv = down_conv + li;
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  uint64_t x[P];
#pragma unroll
  for (int i = 0; i < P; i++) {
    const size_t pos = G::gaddr(g, G::ipoint(r, i));
    u128 s;
    s.lo = s.hi = 0;
    for (uint32_t k = 0; k < kg.K; k++) mac_wide(s, src[(size_t)k * G::N + pos], cv[(size_t)k * kg.nm]);
    x[i] = add_mod(redc(s, m.q, m.qinv), h, m.q);
  }
  G::forward(lds, x, c, r, g, tw + (size_t)li * G::N, tws + (size_t)li * G::N, m.q);
  uint64_t *out = conv_out + ((size_t)p * kg.L + li) * G::N;
#pragma unroll
  for (int v = 0; v < P; v++) out[G::gaddr(g, G::bpoint(r, v))] = x[v];
}

template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_moddown_contig_tail(
    uint64_t *__restrict__ out0, uint64_t *__restrict__ out1, const uint64_t *__restrict__ conv_in,
    const uint64_t *__restrict__ acc, const uint64_t *add0, const uint64_t *add1,
    uint32_t galois, RowScale pinv, KsGeom kg, const ModConst *__restrict__ mc,
    const uint64_t *__restrict__ tw, const uint64_t *__restrict__ tws) {
  using G = Pass<split_b(LOGN), LOGN, false>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const uint32_t p = blockIdx.y / kg.nq, li = blockIdx.y % kg.nq;
  const uint64_t q = mc[li].q;
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  const uint64_t *cin = conv_in + ((size_t)p * kg.L + li) * G::N;
  uint64_t x[P];
#pragma unroll
  for (int i = 0; i < P; i++) x[i] = cin[G::gaddr(g, G::ipoint(r, i))];
  G::forward(lds, x, c, r, g, tw + (size_t)li * G::N, tws + (size_t)li * G::N, q);
#pragma unroll
  for (int v = 0; v < P; v++) x[v] = reduce4(x[v], q);
  G::to_interleaved(lds, x, c, r);
  const uint64_t *u = acc + ((size_t)p * kg.ne + li) * G::N;
  const uint64_t *add = p == 0 ? add0 : add1;
  uint64_t *out = (p == 0 ? out0 : out1) + (size_t)li * G::N;
  const uint64_t w = pinv.w[li], wp = pinv.wp[li];
#pragma unroll
  for (int i = 0; i < P; i++) {
    const size_t pos = G::gaddr(g, G::ipoint(r, i));
    uint64_t v = shoup(sub_mod(u[pos], x[i], q), w, wp, q);
    if (add) v = add_mod(v, add[(size_t)li * G::N + galois_src((uint32_t)pos, galois, LOGN)], q);
    out[pos] = v;
  }
}

template <int LOGN>
int ks_run(hck_context *ctx, const uint64_t *d, uint32_t galois, uint32_t level,
           const hck_switch_key *key, uint64_t *out0, uint64_t *out1, const uint64_t *add0,
           const uint64_t *add1) {
  constexpr int A = split_a(LOGN), B = split_b(LOGN);
  constexpr double N = (double)(1 << LOGN);
  using GA = Pass<A, LOGN, true>;
  using GB = Pass<B, LOGN, false>;
  const size_t n = ctx->n;
  const uint32_t L = ctx->L, K = ctx->K, nm = L + K, alpha = ctx->alpha;
  const uint32_t nq = level + 1, ne = nq + K;
  const KsGeom kg{level, nq, ne, L, K, ctx->dnum, alpha, nm};
  uint64_t *y = ws_ks(ctx);
  uint64_t *ext = y + (size_t)L * n;
  uint64_t *acc = ext + (size_t)ctx->dnum * nm * n;
  uint64_t *conv = acc + (size_t)2 * nm * n;
  int rc;

  // K1, K2: coefficient form of phi_g(d) times N^-1 (Q_j / q_i)^-1
  timing_begin(ctx, "ks_intt_gather", 16.0 * N * nq, 0.5 * N * B * nq);
  k_ks_intt_gather<LOGN><<<dim3(GB::BLOCKS, nq), kNttThreads, 0, ctx->stream>>>(
      y, d, galois, ctx->d_mod, ctx->d_itw, ctx->d_itw_shoup);
  timing_end(ctx);
  RowScale sc;
  for (uint32_t i = 0; i < nq; i++) {
    sc.w[i] = ctx->up_scale[level][i];
    sc.wp[i] = h_shoup(sc.w[i], ctx->mods[i]);
    sc.add[i] = 0;
  }
  if ((rc = ntt_pass(ctx, y, qmap(ctx, level), true, true, &sc))) return rc;

  // K3: ModUp conversion + forward strided pass of every extended limb
  std::vector<std::pair<uint32_t, uint32_t>> ext_rows;  // (digit, t)
  for (uint32_t j = 0; j < ctx->dnum; j++) {
    const uint32_t lo = j * alpha;
    if (lo >= nq) break;
    const uint32_t hi = std::min(lo + alpha, nq);
    for (uint32_t t = 0; t < ne; t++)
      if (t < lo || t >= hi) ext_rows.push_back({j, t});
  }
  const uint64_t *up_conv = ctx->d_up_conv + (size_t)level * ctx->dnum * alpha * nm;
  for (size_t s = 0; s < ext_rows.size(); s += kMaxRows) {
    ModUpRows mr;
    mr.n = (uint32_t)std::min(ext_rows.size() - s, (size_t)kMaxRows);
    double srcs = 0;
    for (uint32_t k = 0; k < mr.n; k++) {
      const uint32_t j = ext_rows[s + k].first, t = ext_rows[s + k].second;
      mr.row[k] = (uint16_t)(j * ne + t);
      mr.mod[k] = (uint8_t)(t < nq ? t : L + (t - nq));
      mr.digit[k] = (uint8_t)j;
      srcs += std::min(alpha, nq - j * alpha);
    }
    timing_begin(ctx, "ks_modup_strided", 8.0 * N * (srcs + mr.n), N * (srcs + 0.5 * A * mr.n));
    k_modup_strided<LOGN><<<dim3(GA::BLOCKS, mr.n), kNttThreads, 0, ctx->stream>>>(
        ext, y, mr, up_conv, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
    timing_end(ctx);
  }

  // K4: forward contiguous pass of the extended digits + key inner product
  const double digits = (double)((nq + alpha - 1) / alpha);
  const double ext_limbs = (double)ext_rows.size();
  timing_begin(ctx, "ks_contig_inner", 8.0 * N * (ext_limbs + nq + 2 * digits * ne + 2 * ne),
               N * (0.5 * B * ext_limbs + 2 * digits * ne));
  k_ks_contig_inner<LOGN><<<dim3(GB::BLOCKS, ne), kNttThreads, 0, ctx->stream>>>(
      acc, ext, d, galois, key->data, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
  timing_end(ctx);

  // K5: inverse transform of the P limbs of both accumulators (+ ModDown scale)
  LimbMap mp;
  RowScale sp;
  mp.n = 2 * K;
  for (uint32_t p = 0; p < 2; p++)
    for (uint32_t k = 0; k < K; k++) {
      const uint32_t r = p * K + k;
      mp.row[r] = (uint16_t)(p * ne + nq + k);
      mp.mod[r] = (uint8_t)(L + k);
      sp.w[r] = ctx->down_scale[k];
      sp.wp[r] = h_shoup(sp.w[r], ctx->mods[L + k]);
      sp.add[r] = ctx->down_add[k];
    }
  if ((rc = ntt_pass(ctx, acc, mp, true, false, nullptr))) return rc;
  if ((rc = ntt_pass(ctx, acc, mp, true, true, &sp))) return rc;

  // K6: ModDown conversion + forward strided pass
  timing_begin(ctx, "ks_moddown_strided", 8.0 * N * (K + 1) * 2 * nq, N * (K + 0.5 * A) * 2 * nq);
  k_moddown_strided<LOGN><<<dim3(GA::BLOCKS, 2 * nq), kNttThreads, 0, ctx->stream>>>(
      conv, acc, ctx->d_down_conv, ctx->d_down_hneg, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
  timing_end(ctx);

  // K7: forward contiguous pass + (acc - conv) P^-1 + addend
  RowScale pinv;
  for (uint32_t i = 0; i < nq; i++) {
    pinv.w[i] = ctx->pinv[i];
    pinv.wp[i] = h_shoup(ctx->pinv[i], ctx->mods[i]);
    pinv.add[i] = 0;
  }
  const double adds = (add0 ? nq : 0) + (add1 ? nq : 0);
  timing_begin(ctx, "ks_moddown_tail", 8.0 * N * (3.0 * 2 * nq + adds), N * (0.5 * B + 1) * 2 * nq);
  k_moddown_contig_tail<LOGN><<<dim3(GB::BLOCKS, 2 * nq), kNttThreads, 0, ctx->stream>>>(
      out0, out1, conv, acc, add0, add1, galois, pinv, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

}  // namespace

int keyswitch_core(hck_context *ctx, const uint64_t *d, uint32_t galois, uint32_t level,
                   const hck_switch_key *key, uint64_t *out0, uint64_t *out1, const uint64_t *add0,
                   const uint64_t *add1) {
  int rc = ensure_workspace(ctx, ws_words_needed(ctx));
  if (rc) return rc;
  if (level + 1 > (uint32_t)kMaxLimbs) return set_error(HCK_EINVAL, "level too high");
  switch (ctx->log_n) {
    case 11: return ks_run<11>(ctx, d, galois, level, key, out0, out1, add0, add1);
    case 12: return ks_run<12>(ctx, d, galois, level, key, out0, out1, add0, add1);
    case 13: return ks_run<13>(ctx, d, galois, level, key, out0, out1, add0, add1);
    case 14: return ks_run<14>(ctx, d, galois, level, key, out0, out1, add0, add1);
    case 15: return ks_run<15>(ctx, d, galois, level, key, out0, out1, add0, add1);
    case 16: return ks_run<16>(ctx, d, galois, level, key, out0, out1, add0, add1);
    case 17: return ks_run<17>(ctx, d, galois, level, key, out0, out1, add0, add1);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

}  // namespace hck
