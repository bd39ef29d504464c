// Hybrid key switching with the basis conversions, the key inner product and
// the ModDown tail fused into the NTT passes (ntt_core.h), for a batch of up
// to ks_slots inputs, each with its own switching key.
//
// KeySwitch(d) at level l with a switching key swk(s' -> s); d is read through
// the NTT-domain automorphism X -> X^g (g = 1: no automorphism), so a
// rotation never materializes phi_g(c):
//   K1  inverse contiguous pass of phi_g(d) over Q_l -> y          (gather;
//       also the copy of c0 for an output that aliases its input)
//   K2  inverse strided pass, times N^-1 (Q_j / q_i)^-1 per limb    (digit scale)
//   K3  ModUp: per digit j and target limb t not in D_j, the fast basis
//       conversion of y's digit limbs computed at load time, then the
//       forward strided pass -> ext[j][t]
//   K4  per extended limb t: forward contiguous pass of every digit's ext
//       (or phi_g(d) itself on the digit's own limbs), then
//       acc_{0,1}[t] = sum_j d~_j[t] swk_j[t] (keys in Montgomery form); slots
//       that share a key re-read its tiles from cache; on the P limbs the
//       inverse contiguous pass of K5 follows in the same kernel
//   K5  inverse passes of acc's P limbs, times N^-1 (P/p_k)^-1, plus
//       ((P-1)/2) (P/p_k)^-1 (the rounding term of ModDown)
//   K6  ModDown conversion P -> q_i (minus (P-1)/2) at load time, then the
//       forward strided pass -> conv
//   K7  forward contiguous pass of conv, then
//       out_i = (acc_i - conv_i) P^-1 (+ phi_g(addend)_i)
//
// Workspace: batch slot b occupies rows [b R, (b+1) R) of ws_ks (R rows of N
// words): y [L] | ext [dnum][L+K] | acc [2][L+K] | conv [2][L].
#include <algorithm>

#include "ntt_core.h"

namespace hck {

namespace {

struct KsGeom;
// the largest kernel argument list (ModDown tail: batch table, row scales,
// geometry, pointers) stays within the 4 KiB a kernel can take
static_assert(sizeof(KsBatch) + sizeof(RowScale) + 128 + 64 <= 4096,
              "kernel arguments beyond 4 KiB");

struct KsGeom {
  uint32_t level, nq, ne, L, K, dnum, alpha, nm;
  uint32_t slot_rows;                       // rows per batch slot
  uint32_t off_ext, off_acc, off_conv;      // row offsets inside a slot
};

// One launch of the ModUp: entry k converts digit digit[k] (source rows from
// src[k]) into target modulus mod[k] (output row row[k]) and, where row2[k] is
// not kNoRow, into mod2[k] (row2[k]) from the same reads of the sources.
constexpr uint16_t kNoRow = 0xffff;
// workgroups (at one target each) from which the basis conversions pair
// targets: halved, they still fill the chip twice over at the paired kernel's
// occupancy (about 3 workgroups of 256 threads per CU)
constexpr size_t kPairMinBlocks = 3072;
struct ModUpRows {
  uint32_t n;
  uint16_t row[kMaxRows];     // output row (workspace row)
  uint16_t row2[kMaxRows];    // second output row or kNoRow
  uint16_t src[kMaxRows];     // workspace row of the digit's first source limb
  uint8_t mod[kMaxRows];
  uint8_t mod2[kMaxRows];
  uint8_t digit[kMaxRows];
};

template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_ks_intt_gather(
    uint64_t *__restrict__ ws, KsBatch kb, KsGeom kg,
    const ModConst *__restrict__ mc, const uint64_t *__restrict__ itw,
    const uint64_t *__restrict__ itws, const uint64_t *__restrict__ itt,
    const uint64_t *__restrict__ itts) {
  using G = Pass<split_b(LOGN), LOGN, false>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const int li = blockIdx.z;  // limb i (modulus i)
  const uint32_t b = blockIdx.y;
  const uint64_t q = mc[li].q;
  const Qn qm = qn(mc[li]);
  const size_t roff = (size_t)li * G::N;
  const uint64_t *d = kb.d[b];
  const uint32_t galois = kb.galois[b];
  uint64_t *y = ws + (size_t)b * kg.slot_rows * G::N;
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  if (const uint64_t *c0 = kb.add0_src[b]) {
    // an output aliasing its input: copy this tile of c0 for the last launch
    uint64_t *cp = const_cast<uint64_t *>(kb.add0[b]);
#pragma unroll
    for (int i = 0; i < P; i++) {
      const size_t a = roff + G::gaddr(g, G::ipoint(r, i));
      cp[a] = c0[a];
    }
  }
  uint64_t x[P];
#pragma unroll
  for (int i = 0; i < P; i++)
    x[i] = d[roff + galois_src((uint32_t)G::gaddr(g, G::ipoint(r, i)), galois, LOGN)];
  G::to_blocked(lds, x, c, r);
  G::inverse(lds, x, c, r, g, itw + roff, itws + roff, qm);
  G::twist(x, g, r, itt + roff, itts + roff, qm);
#pragma unroll
  for (int i = 0; i < P; i++) y[roff + G::gaddr(g, G::ipoint(r, i))] = x[i];
}

// Fast basis conversion of a thread's P points (interleaved layout of the
// strided pass) at load time, into NT target moduli at once:
//   x[t][i] = REDC(sum_{a < na} src[a N + pos_i] cv[t][a cstride]) in [0, q_t)
// (constants in Montgomery form; the sum stays below q_t 2^64).  Points are
// taken CH at a time, with the CH loads of one source limb issued together
// so that their latencies overlap (one load, then a wait, per product
// leaves the conversion latency-bound); each loaded word serves every
// target.
template <class G, int NT>
__device__ __forceinline__ void bconv_points(uint64_t (&x)[NT][G::P],
                                             const uint64_t *__restrict__ src,
                                             const uint64_t *const (&cv)[NT], uint32_t cstride,
                                             uint32_t na, int g, int r,
                                             const ModConst (&m)[NT]) {
  constexpr int P = G::P;
  constexpr int CH = NT == 1 ? P : P / 2;
#pragma unroll
  for (int c0 = 0; c0 < P; c0 += CH) {
    u128 acc[NT][CH];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int k = 0; k < CH; k++) acc[t][k].lo = acc[t][k].hi = 0;
    for (uint32_t a = 0; a < na; a++) {
      uint64_t v[CH];
#pragma unroll
      for (int k = 0; k < CH; k++) v[k] = src[(size_t)a * G::N + G::gaddr(g, G::ipoint(r, c0 + k))];
#pragma unroll
      for (int t = 0; t < NT; t++) {
        const uint64_t c = cv[t][(size_t)a * cstride];
#pragma unroll
        for (int k = 0; k < CH; k++) mac_wide(acc[t][k], v[k], c);
      }
    }
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int k = 0; k < CH; k++) x[t][c0 + k] = redc(acc[t][k], m[t].q, m[t].qinv);
  }
}

// The same sums for moduli below 2^60 (sources v and constants c below
// 2^60), with both factors split into 30-bit halves, v = v1 2^30 + v0 and
// c = c1 2^30 + c0:
//   sum_a v c = L + 2^30 (M1 + M2) + 2^60 H,
//   L = sum v0 c0, M1 = sum v0 c1, M2 = sum v1 c0, H = sum v1 c1.
// Each column is below na (2^30 - 1)^2 < 2^64 for na <= 16 sources (a
// digit or the special basis holds at most 16 primes), so every partial
// product is one 32 x 32 + 64-bit multiply-add into its column, with no
// carries between columns; the columns are combined into the 128-bit sum
// (the same integer as above, so the same REDC result) once per point.
// Four 64-bit columns take twice the registers of one 128-bit sum, so the
// points are taken in chunks of half the size.
template <class G, int NT, bool UNROLL2>
__device__ __forceinline__ void bconv_points30(uint64_t (&x)[NT][G::P],
                                               const uint64_t *__restrict__ src,
                                               const uint64_t *const (&cv)[NT], uint32_t cstride,
                                               uint32_t na, int g, int r,
                                               const ModConst (&m)[NT]) {
  constexpr int P = G::P;
  constexpr int CH = NT == 1 ? P / 2 : P / 4;
  constexpr uint32_t kLow30 = (1u << 30) - 1;
#pragma unroll
  for (int c0 = 0; c0 < P; c0 += CH) {
    uint64_t lo[NT][CH], m1[NT][CH], m2[NT][CH], hi[NT][CH];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int k = 0; k < CH; k++) lo[t][k] = m1[t][k] = m2[t][k] = hi[t][k] = 0;
    // one source limb: its CH words, split, into every target's columns
    auto source = [&](uint32_t a) {
      uint32_t v0[CH], v1[CH];
#pragma unroll
      for (int k = 0; k < CH; k++) {
        const uint64_t v = src[(size_t)a * G::N + G::gaddr(g, G::ipoint(r, c0 + k))];
        v0[k] = (uint32_t)v & kLow30;
        v1[k] = (uint32_t)(v >> 30);
      }
#pragma unroll
      for (int t = 0; t < NT; t++) {
        const uint64_t c = cv[t][(size_t)a * cstride];
        const uint32_t cl = (uint32_t)c & kLow30, ch = (uint32_t)(c >> 30);
#pragma unroll
        for (int k = 0; k < CH; k++) {
          lo[t][k] += (uint64_t)v0[k] * cl;
          m1[t][k] += (uint64_t)v0[k] * ch;
          m2[t][k] += (uint64_t)v1[k] * cl;
          hi[t][k] += (uint64_t)v1[k] * ch;
        }
      }
    };
    // two source limbs per iteration put twice the loads in flight; the
    // paired ModUp, held to 128 registers for a fourth wave per SIMD, takes
    // one (the unrolled loop would spill more there)
    if constexpr (UNROLL2) {
#pragma unroll 2
      for (uint32_t a = 0; a < na; a++) source(a);
    } else {
      for (uint32_t a = 0; a < na; a++) source(a);
    }
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int k = 0; k < CH; k++) {
        const wide_t mid = (wide_t)m1[t][k] + m2[t][k];
        const wide_t y = (wide_t)lo[t][k] + (mid << 30) + ((wide_t)hi[t][k] << 60);
        u128 s;
        s.lo = (uint64_t)y;
        s.hi = (uint64_t)(y >> 64);
        x[t][c0 + k] = redc(s, m[t].q, m[t].qinv);
        // reduce this chunk before the next chunk's loads (the empty asm
        // takes the result and orders memory accesses, and emits nothing), so
        // that one chunk's columns are live at a time, not every chunk's
        asm volatile("" ::"v"(x[t][c0 + k]) : "memory");
      }
  }
}

template <class G, int NT, bool S30, bool UNROLL2 = true>
__device__ __forceinline__ void bconv(uint64_t (&x)[NT][G::P], const uint64_t *__restrict__ src,
                                      const uint64_t *const (&cv)[NT], uint32_t cstride,
                                      uint32_t na, int g, int r, const ModConst (&m)[NT]) {
  if constexpr (S30)
    bconv_points30<G, NT, UNROLL2>(x, src, cv, cstride, na, g, r, m);
  else
    bconv_points<G, NT>(x, src, cv, cstride, na, g, r, m);
}

// the paired 30-bit ModUp is held to 128 VGPRs (4 waves per SIMD instead of
// 3, at 8 bytes of spill a lane): measured 6 % faster
template <int LOGN, bool PAIR, bool S30>
__global__ __launch_bounds__(kNttThreads)
__attribute__((amdgpu_waves_per_eu(PAIR && S30 ? 4 : 1))) void k_modup_strided(
    uint64_t *__restrict__ ws, ModUpRows rows, const uint64_t *__restrict__ conv, KsGeom kg,
    const ModConst *__restrict__ mc, const uint64_t *__restrict__ tw,
    const uint64_t *__restrict__ tws) {
  using G = Pass<split_a(LOGN), LOGN, true>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const int k = blockIdx.y;
  const int j = rows.digit[k];
  const uint32_t na = min(kg.alpha, kg.nq - j * kg.alpha);
  const int mi = rows.mod[k];
  const ModConst m = mc[mi];
  const uint64_t *cv = conv + (size_t)j * kg.alpha * kg.nm + mi;
  const uint64_t *src = ws + (size_t)rows.src[k] * G::N;
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  if constexpr (!PAIR) {
    uint64_t x[1][P];
    const uint64_t *const cvs[1] = {cv};
    const ModConst ms[1] = {m};
    bconv<G, 1, S30>(x, src, cvs, kg.nm, na, g, r, ms);
    G::forward(lds, x[0], c, r, g, tw + (size_t)mi * G::N, tws + (size_t)mi * G::N, qn(m));
    uint64_t *out = ws + (size_t)rows.row[k] * G::N;
#pragma unroll
    for (int v = 0; v < P; v++) out[G::gaddr(g, G::bpoint(r, v))] = x[0][v];
  } else {
    const bool two = rows.row2[k] != kNoRow;
    const int mi2 = two ? rows.mod2[k] : mi;
    const ModConst m2 = mc[mi2];
    const uint64_t *cv2 = conv + (size_t)j * kg.alpha * kg.nm + mi2;
    uint64_t x[2][P];
    const uint64_t *const cvs[2] = {cv, cv2};
    const ModConst ms[2] = {m, m2};
    bconv<G, 2, S30, false>(x, src, cvs, kg.nm, na, g, r, ms);
    G::forward(lds, x[0], c, r, g, tw + (size_t)mi * G::N, tws + (size_t)mi * G::N, qn(m));
    uint64_t *out = ws + (size_t)rows.row[k] * G::N;
#pragma unroll
    for (int v = 0; v < P; v++) out[G::gaddr(g, G::bpoint(r, v))] = x[0][v];
    if (!two) return;
    G::forward(lds, x[1], c, r, g, tw + (size_t)mi2 * G::N, tws + (size_t)mi2 * G::N, qn(m2));
    uint64_t *out2 = ws + (size_t)rows.row2[k] * G::N;
#pragma unroll
    for (int v = 0; v < P; v++) out2[G::gaddr(g, G::bpoint(r, v))] = x[1][v];
  }
}

template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_ks_contig_inner(
    uint64_t *__restrict__ ws, KsBatch kb, KsGeom kg, const ModConst *__restrict__ mc,
    const uint64_t *__restrict__ tw, const uint64_t *__restrict__ tws,
    const uint64_t *__restrict__ tt, const uint64_t *__restrict__ tts,
    const uint64_t *__restrict__ itw, const uint64_t *__restrict__ itws,
    const uint64_t *__restrict__ itt, const uint64_t *__restrict__ itts) {
  using G = Pass<split_b(LOGN), LOGN, false>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  // With 8 points a thread (three-layout passes) a workgroup covers TILE
  // consecutive words of a row, a wavefront 512 of them.  Each digit's two
  // key rows over those words are copied into LDS by direct global-to-LDS
  // loads issued before the digit's forward pass, so the copy runs under the
  // transform without holding registers; each wavefront reads only the words
  // it copied (no workgroup barrier).  The two rows take 32 KiB, which still
  // leaves room for as many workgroups per CU as the registers allow.
  constexpr bool KEY_LDS = G::P == 8 && G::T * G::TR == kNttThreads && split_b(LOGN) >= 7;
  constexpr int TILE = kNttThreads * P;
  __shared__ uint64_t ktile[KEY_LDS ? 2 * TILE : 1];
  // the special limbs, which also run an inverse pass, are dispatched first
  // so that the shorter workgroups fill in behind them
  const uint32_t t = blockIdx.z < kg.K ? kg.nq + blockIdx.z : blockIdx.z - kg.K;
  const uint32_t b = blockIdx.y;
  const uint32_t mi = t < kg.nq ? t : kg.L + (t - kg.nq);
  const ModConst m = mc[mi];
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  const size_t krow = (size_t)kg.nm * G::N;
  uint64_t *slot = ws + (size_t)b * kg.slot_rows * G::N;
  const uint64_t *d = kb.d[b];
  const uint64_t *key = kb.key[b];
  const uint32_t galois = kb.galois[b];
  uint64_t a0[P], a1[P], x[P];
#pragma unroll
  for (int i = 0; i < P; i++) a0[i] = a1[i] = 0;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const size_t tile0 = (size_t)blockIdx.x * TILE;  // first word of the tile in a row
  for (uint32_t j = 0; j < kg.dnum; j++) {
    const uint32_t lo = j * kg.alpha;
    if (lo >= kg.nq) break;
    const uint32_t hi = min(lo + kg.alpha, kg.nq);
    const uint64_t *kbp = key + 2 * j * krow + (size_t)mi * G::N;
    const uint64_t *kap = kbp + krow;
    // this wavefront's 512 words of each key row: 4 loads of 16 bytes a lane
    // (1 KiB a load), lane l's bytes landing at 16 l.  Loads complete in
    // issue order, so the copy is issued after the digit's own loads (a wait
    // for those does not wait for it) and before the transform it hides under.
    auto copy_keys = [&]() {
      if constexpr (KEY_LDS) {
#pragma unroll
        for (int rr = 0; rr < 2; rr++) {
          const uint64_t *src = (rr ? kap : kbp) + tile0 + wave * 512 + 2 * (threadIdx.x % 64);
#pragma unroll
          for (int i = 0; i < 4; i++)
            __builtin_amdgcn_global_load_lds(
                (const void *)(src + 128 * i),
                (__attribute__((address_space(3))) void *)&ktile[rr * TILE + wave * 512 + 128 * i],
                16, 0, 0);
        }
      }
    };
    if (t >= lo && t < hi) {
      copy_keys();
#pragma unroll
      for (int i = 0; i < P; i++)
        x[i] = d[(size_t)t * G::N +
                 galois_src((uint32_t)G::gaddr(g, G::ipoint(r, i)), galois, LOGN)];
    } else {
      const uint64_t *e = slot + ((size_t)kg.off_ext + j * kg.ne + t) * G::N;
#pragma unroll
      for (int i = 0; i < P; i++) x[i] = e[G::gaddr(g, G::ipoint(r, i))];
      G::twist(x, g, r, tt + (size_t)mi * G::N, tts + (size_t)mi * G::N, qn(m));
      copy_keys();
      G::forward(lds, x, c, r, g, tw + (size_t)mi * G::N, tws + (size_t)mi * G::N, qn(m));
#pragma unroll
      for (int v = 0; v < P; v++) x[v] = reduce4(x[v], qn(m));
      G::to_interleaved(lds, x, c, r);
    }
#pragma unroll
    for (int i = 0; i < P; i++) {
      const size_t pos = G::gaddr(g, G::ipoint(r, i));
      uint64_t kv0, kv1;
      if constexpr (KEY_LDS) {
        kv0 = ktile[pos - tile0];
        kv1 = ktile[TILE + pos - tile0];
      } else {
        kv0 = kbp[pos];
        kv1 = kap[pos];
      }
      a0[i] = add_mod(a0[i], redc(mul_wide(x[i], kv0), m.q, m.qinv), m.q);
      a1[i] = add_mod(a1[i], redc(mul_wide(x[i], kv1), m.q, m.qinv), m.q);
    }
  }
  if (t >= kg.nq) {
    // special limb: ModDown's inverse contiguous pass, while the limb's
    // blocks are at hand
    const size_t toff = (size_t)mi * G::N;
    G::to_blocked(lds, a0, c, r);
    G::inverse(lds, a0, c, r, g, itw + toff, itws + toff, qn(m));
    G::twist(a0, g, r, itt + toff, itts + toff, qn(m));
    G::to_blocked(lds, a1, c, r);
    G::inverse(lds, a1, c, r, g, itw + toff, itws + toff, qn(m));
    G::twist(a1, g, r, itt + toff, itts + toff, qn(m));
  }
  uint64_t *o0 = slot + ((size_t)kg.off_acc + t) * G::N;
  uint64_t *o1 = slot + ((size_t)kg.off_acc + kg.ne + t) * G::N;
#pragma unroll
  for (int i = 0; i < P; i++) {
    const size_t pos = G::gaddr(g, G::ipoint(r, i));
    o0[pos] = a0[i];
    o1[pos] = a1[i];
  }
}

template <int LOGN, bool PAIR, bool S30>
__global__ __launch_bounds__(kNttThreads) void k_moddown_strided(
    uint64_t *__restrict__ ws, const uint64_t *__restrict__ down_conv,
    const uint64_t *__restrict__ hneg, KsGeom kg, const ModConst *__restrict__ mc,
    const uint64_t *__restrict__ tw, const uint64_t *__restrict__ tws) {
  using G = Pass<split_a(LOGN), LOGN, true>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  // with PAIR workgroup y converts target limbs li and li + 1 (if below nq)
  // of poly p from one read of the K special limbs, else limb li alone
  const uint32_t per = PAIR ? (kg.nq + 1) / 2 : kg.nq;
  const uint32_t p = blockIdx.y / per, li = (PAIR ? 2 : 1) * (blockIdx.y % per);
  uint64_t *slot = ws + (size_t)blockIdx.z * kg.slot_rows * G::N;
  const ModConst m = mc[li];
  const uint64_t h = hneg[li];
  const uint64_t *src = slot + ((size_t)kg.off_acc + p * kg.ne + kg.nq) * G::N;
  const uint64_t *cv = down_conv + li;
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  if constexpr (!PAIR) {
    uint64_t x[1][P];
    const uint64_t *const cvs[1] = {cv};
    const ModConst ms[1] = {m};
    bconv<G, 1, S30>(x, src, cvs, kg.nm, kg.K, g, r, ms);
#pragma unroll
    for (int i = 0; i < P; i++) x[0][i] = add_mod(x[0][i], h, m.q);
    G::forward(lds, x[0], c, r, g, tw + (size_t)li * G::N, tws + (size_t)li * G::N, qn(m));
    uint64_t *out = slot + ((size_t)kg.off_conv + p * kg.L + li) * G::N;
#pragma unroll
    for (int v = 0; v < P; v++) out[G::gaddr(g, G::bpoint(r, v))] = x[0][v];
  } else {
    const bool two = li + 1 < kg.nq;
    const uint32_t li2 = two ? li + 1 : li;
    const ModConst m2 = mc[li2];
    const uint64_t h2 = hneg[li2];
    const uint64_t *cv2 = down_conv + li2;
    uint64_t x[2][P];
    const uint64_t *const cvs[2] = {cv, cv2};
    const ModConst ms[2] = {m, m2};
    bconv<G, 2, S30>(x, src, cvs, kg.nm, kg.K, g, r, ms);
#pragma unroll
    for (int i = 0; i < P; i++) {
      x[0][i] = add_mod(x[0][i], h, m.q);
      x[1][i] = add_mod(x[1][i], h2, m2.q);
    }
    G::forward(lds, x[0], c, r, g, tw + (size_t)li * G::N, tws + (size_t)li * G::N, qn(m));
    uint64_t *out = slot + ((size_t)kg.off_conv + p * kg.L + li) * G::N;
#pragma unroll
    for (int v = 0; v < P; v++) out[G::gaddr(g, G::bpoint(r, v))] = x[0][v];
    if (!two) return;
    G::forward(lds, x[1], c, r, g, tw + (size_t)li2 * G::N, tws + (size_t)li2 * G::N, qn(m2));
    uint64_t *out2 = slot + ((size_t)kg.off_conv + p * kg.L + li2) * G::N;
#pragma unroll
    for (int v = 0; v < P; v++) out2[G::gaddr(g, G::bpoint(r, v))] = x[1][v];
  }
}

template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_moddown_contig_tail(
    uint64_t *__restrict__ ws, KsBatch kb, RowScale pinv, KsGeom kg,
    const ModConst *__restrict__ mc, const uint64_t *__restrict__ tw,
    const uint64_t *__restrict__ tws, const uint64_t *__restrict__ tt,
    const uint64_t *__restrict__ tts) {
  using G = Pass<split_b(LOGN), LOGN, false>;
  constexpr int P = G::P;
  __shared__ uint64_t lds[G::LDS_WORDS];
  const uint32_t p = blockIdx.z & 1, li = blockIdx.z >> 1;
  const uint32_t b = blockIdx.y;
  const uint64_t *slot = ws + (size_t)b * kg.slot_rows * G::N;
  const uint64_t q = mc[li].q;
  const Qn qm = qn(mc[li]);
  const int c = G::sub(threadIdx.x), r = G::lane(threadIdx.x);
  const int g = blockIdx.x * G::TR + c;
  const uint64_t *cin = slot + ((size_t)kg.off_conv + p * kg.L + li) * G::N;
  uint64_t x[P];
#pragma unroll
  for (int i = 0; i < P; i++) x[i] = cin[G::gaddr(g, G::ipoint(r, i))];
  G::twist(x, g, r, tt + (size_t)li * G::N, tts + (size_t)li * G::N, qm);
  G::forward(lds, x, c, r, g, tw + (size_t)li * G::N, tws + (size_t)li * G::N, qm);
#pragma unroll
  for (int v = 0; v < P; v++) x[v] = reduce4(x[v], qm);
  G::to_interleaved(lds, x, c, r);
  const uint64_t *u = slot + ((size_t)kg.off_acc + p * kg.ne + li) * G::N;
  const uint64_t *add = p == 0 ? kb.add0[b] : kb.add1[b];
  const uint32_t galois = kb.galois[b];
  uint64_t *out = (p == 0 ? kb.out0[b] : kb.out1[b]) + (size_t)li * G::N;
  const uint64_t w = pinv.w[li], wp = pinv.wp[li];
#pragma unroll
  for (int i = 0; i < P; i++) {
    const size_t pos = G::gaddr(g, G::ipoint(r, i));
    uint64_t v = shoup(sub_mod(u[pos], x[i], q), w, wp, q);
    if (add) v = add_mod(v, add[(size_t)li * G::N + galois_src((uint32_t)pos, galois, LOGN)], q);
    out[pos] = v;
  }
}

// inner product of hoisted rotations: for extended limb t,
// acc_{0,1}[t] = sum_j phi_g(d~_j)[t] swk_j[t], with d~_j fully transformed in
// slot 0's ext rows (own limbs: phi_g(c1)) and the result in slot b's acc rows
template <int LOGN>
__global__ __launch_bounds__(256) void k_ks_inner_gather(
    uint64_t *__restrict__ ws, const uint64_t *__restrict__ c1, uint32_t galois, uint32_t b,
    const uint64_t *__restrict__ key, KsGeom kg, const ModConst *__restrict__ mc) {
  constexpr int N = 1 << LOGN;
  const uint32_t pos = blockIdx.x * 256 + threadIdx.x;
  const uint32_t t = blockIdx.y;
  const uint32_t mi = t < kg.nq ? t : kg.L + (t - kg.nq);
  const ModConst m = mc[mi];
  const uint32_t src = galois_src(pos, galois, LOGN);
  const size_t krow = (size_t)kg.nm * N;
  u128 s0, s1;
  s0.lo = s0.hi = s1.lo = s1.hi = 0;
  for (uint32_t j = 0; j < kg.dnum; j++) {
    const uint32_t lo = j * kg.alpha;
    if (lo >= kg.nq) break;
    const uint32_t hi = min(lo + kg.alpha, kg.nq);
    const uint64_t x = (t >= lo && t < hi)
                           ? c1[(size_t)t * N + src]
                           : ws[((size_t)kg.off_ext + j * kg.ne + t) * N + src];
    const uint64_t *kbp = key + 2 * j * krow + (size_t)mi * N;
    mac_wide(s0, x, kbp[pos]);
    mac_wide(s1, x, kbp[krow + pos]);
  }
  uint64_t *slot = ws + (size_t)b * kg.slot_rows * N;
  slot[((size_t)kg.off_acc + t) * N + pos] = redc(s0, m.q, m.qinv);
  slot[((size_t)kg.off_acc + kg.ne + t) * N + pos] = redc(s1, m.q, m.qinv);
}

KsGeom make_geom(const hck_context *ctx, uint32_t level) {
  KsGeom kg;
  kg.level = level;
  kg.nq = level + 1;
  kg.ne = level + 1 + ctx->K;
  kg.L = ctx->L;
  kg.K = ctx->K;
  kg.dnum = ctx->dnum;
  kg.alpha = ctx->alpha;
  kg.nm = ctx->L + ctx->K;
  kg.slot_rows = (uint32_t)ws_ks_rows(ctx);
  kg.off_ext = ctx->L;
  kg.off_acc = ctx->L + ctx->dnum * kg.nm;
  kg.off_conv = kg.off_acc + 2 * kg.nm;
  return kg;
}

// K1-K3 for batch slots 0..nb-1 (ModUp into each slot's ext rows)
template <int LOGN>
int ks_modup(hck_context *ctx, const KsBatch &kb, const KsGeom &kg, uint64_t *ws) {
  constexpr int A = split_a(LOGN), B = split_b(LOGN);
  constexpr double N = (double)(1 << LOGN);
  using GA = Pass<A, LOGN, true>;
  using GB = Pass<B, LOGN, false>;
  const uint32_t L = kg.L, nm = kg.nm, alpha = kg.alpha, nq = kg.nq, ne = kg.ne, nb = kb.n;
  const uint32_t level = kg.level;
  int rc;
  double copies = 0;   // c0 tiles copied for outputs that alias their input
  for (uint32_t b = 0; b < nb; b++) copies += kb.add0_src[b] ? nq : 0;
  timing_begin(ctx, "ks_intt_gather", dim3(GB::BLOCKS, nb, nq), 16.0 * N * (nq * nb + copies),
               0.5 * N * B * nq * nb);
  k_ks_intt_gather<LOGN><<<dim3(GB::BLOCKS, nb, nq), kNttThreads, 0, ctx->stream>>>(
      ws, kb, kg, ctx->d_mod, ctx->d_itw, ctx->d_itw_shoup, ctx->d_ittw, ctx->d_ittw_shoup);
  timing_end(ctx);
  RowScale sc;
  for (uint32_t i = 0; i < nq; i++) {
    sc.w[i] = ctx->up_scale[level][i];
    sc.wp[i] = h_shoup(sc.w[i], ctx->mods[i]);
    sc.add[i] = 0;
  }
  {
    LimbMap m;
    m.n = nq * nb;
    for (uint32_t b = 0; b < nb; b++)
      for (uint32_t i = 0; i < nq; i++) {
        m.row[b * nq + i] = (uint16_t)(b * kg.slot_rows + i);
        m.mod[b * nq + i] = (uint8_t)i;
      }
    if ((rc = ntt_pass(ctx, ws, m, true, true, &sc, (int)nq))) return rc;
  }
  struct Row {
    uint16_t row, src;
    uint8_t mod, digit;
    uint32_t na;
  };
  std::vector<Row> ext_rows;
  for (uint32_t b = 0; b < nb; b++)
    for (uint32_t j = 0; j < kg.dnum; j++) {
      const uint32_t lo = j * alpha;
      if (lo >= nq) break;
      const uint32_t hi = std::min(lo + alpha, nq);
      for (uint32_t t = 0; t < ne; t++) {
        if (t >= lo && t < hi) continue;
        Row rw;
        rw.row = (uint16_t)(b * kg.slot_rows + kg.off_ext + j * ne + t);
        rw.src = (uint16_t)(b * kg.slot_rows + lo);
        rw.mod = (uint8_t)(t < nq ? t : L + (t - nq));
        rw.digit = (uint8_t)j;
        rw.na = hi - lo;
        ext_rows.push_back(rw);
      }
    }
  const uint64_t *up_conv = ctx->d_up_conv + (size_t)level * kg.dnum * alpha * nm;
  // in a launch large enough to fill the chip at half the workgroups,
  // consecutive targets of one digit share a workgroup (one read of the
  // digit's limbs for both); small launches keep one target per workgroup
  // and the kernel's lower register count
  const bool paired = ext_rows.size() * GA::BLOCKS >= kPairMinBlocks;
  std::vector<std::pair<size_t, size_t>> groups;  // (first row, second row or SIZE_MAX)
  for (size_t i = 0; i < ext_rows.size();) {
    const bool pair = paired && i + 1 < ext_rows.size() &&
                      ext_rows[i + 1].src == ext_rows[i].src &&
                      ext_rows[i + 1].digit == ext_rows[i].digit;
    groups.push_back({i, pair ? i + 1 : SIZE_MAX});
    i += pair ? 2 : 1;
  }
  for (size_t s = 0; s < groups.size(); s += kMaxRows) {
    ModUpRows mr;
    mr.n = (uint32_t)std::min(groups.size() - s, (size_t)kMaxRows);
    // algorithmic bytes: every digit limb a launch converts is read once
    // (the targets sharing it re-read it from cache), every output written
    double srcs = 0, outs = 0, macs = 0;
    std::vector<uint16_t> seen;
    for (uint32_t k = 0; k < mr.n; k++) {
      const Row &rw = ext_rows[groups[s + k].first];
      if (std::find(seen.begin(), seen.end(), rw.src) == seen.end()) {
        seen.push_back(rw.src);
        srcs += rw.na;
      }
      mr.row[k] = rw.row;
      mr.src[k] = rw.src;
      mr.mod[k] = rw.mod;
      mr.digit[k] = rw.digit;
      mr.row2[k] = kNoRow;
      mr.mod2[k] = rw.mod;
      outs += 1;
      macs += rw.na;
      if (groups[s + k].second != SIZE_MAX) {
        const Row &r2 = ext_rows[groups[s + k].second];
        mr.row2[k] = r2.row;
        mr.mod2[k] = r2.mod;
        outs += 1;
        macs += rw.na;
      }
    }
    timing_begin(ctx, "ks_modup_strided", dim3(GA::BLOCKS, mr.n), 8.0 * N * (srcs + outs),
                 N * (macs + 0.5 * A * outs));
    const dim3 grid(GA::BLOCKS, mr.n);
    if (paired && ctx->bconv30)
      k_modup_strided<LOGN, true, true><<<grid, kNttThreads, 0, ctx->stream>>>(
          ws, mr, up_conv, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
    else if (paired)
      k_modup_strided<LOGN, true, false><<<grid, kNttThreads, 0, ctx->stream>>>(
          ws, mr, up_conv, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
    else if (ctx->bconv30)
      k_modup_strided<LOGN, false, true><<<grid, kNttThreads, 0, ctx->stream>>>(
          ws, mr, up_conv, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
    else
      k_modup_strided<LOGN, false, false><<<grid, kNttThreads, 0, ctx->stream>>>(
          ws, mr, up_conv, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
    timing_end(ctx);
  }
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

// K6 launch: the basis conversion on 30-bit halves where every modulus is
// below 2^60, on whole words otherwise
template <int LOGN, bool PAIR>
void launch_moddown_strided(hck_context *ctx, uint64_t *ws, const KsGeom &kg, uint32_t per,
                            uint32_t nb) {
  using GA = Pass<split_a(LOGN), LOGN, true>;
  const dim3 grid(GA::BLOCKS, 2 * per, nb);
  if (ctx->bconv30)
    k_moddown_strided<LOGN, PAIR, true><<<grid, kNttThreads, 0, ctx->stream>>>(
        ws, ctx->d_down_conv, ctx->d_down_hneg, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
  else
    k_moddown_strided<LOGN, PAIR, false><<<grid, kNttThreads, 0, ctx->stream>>>(
        ws, ctx->d_down_conv, ctx->d_down_hneg, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup);
}

// K5-K7 for batch slots 0..nb-1 (ModDown of each slot's acc rows)
template <int LOGN>
int ks_moddown(hck_context *ctx, const KsBatch &kb, const KsGeom &kg, uint64_t *ws,
               bool special_contig_done) {
  constexpr int A = split_a(LOGN), B = split_b(LOGN);
  constexpr double N = (double)(1 << LOGN);
  using GA = Pass<A, LOGN, true>;
  using GB = Pass<B, LOGN, false>;
  const uint32_t L = kg.L, K = kg.K, nq = kg.nq, ne = kg.ne, nb = kb.n;
  int rc;
  {
    LimbMap mp;
    RowScale sp;
    mp.n = 2 * K * nb;
    for (uint32_t b = 0; b < nb; b++)
      for (uint32_t p = 0; p < 2; p++)
        for (uint32_t k = 0; k < K; k++) {
          const uint32_t r = (b * 2 + p) * K + k;
          mp.row[r] = (uint16_t)(b * kg.slot_rows + kg.off_acc + p * ne + nq + k);
          mp.mod[r] = (uint8_t)(L + k);
        }
    for (uint32_t p = 0; p < 2; p++)
      for (uint32_t k = 0; k < K; k++) {
        sp.w[p * K + k] = ctx->down_scale[k];
        sp.wp[p * K + k] = h_shoup(ctx->down_scale[k], ctx->mods[L + k]);
        sp.add[p * K + k] = ctx->down_add[k];
      }
    // the inverse contiguous pass of the special limbs is fused into the
    // inner-product kernel's epilogue, except on the hoisted path
    if (!special_contig_done && (rc = ntt_pass(ctx, ws, mp, true, false, nullptr))) return rc;
    if ((rc = ntt_pass(ctx, ws, mp, true, true, &sp, (int)(2 * K)))) return rc;
  }
  // in a launch large enough to fill the chip at half the workgroups, the K
  // special limbs are read once per pair of target limbs
  const bool paired = (size_t)2 * nq * nb * GA::BLOCKS >= kPairMinBlocks;
  const uint32_t per = paired ? (nq + 1) / 2 : nq;
  // algorithmic bytes: each output's K special limbs read once, its target
  // limbs written
  timing_begin(ctx, "ks_moddown_strided", dim3(GA::BLOCKS, 2 * per, nb),
               8.0 * N * (K + nq) * 2 * nb, N * (K + 0.5 * A) * 2 * nq * nb);
  if (paired)
    launch_moddown_strided<LOGN, true>(ctx, ws, kg, per, nb);
  else
    launch_moddown_strided<LOGN, false>(ctx, ws, kg, per, nb);
  timing_end(ctx);
  RowScale pinv;
  for (uint32_t i = 0; i < nq; i++) {
    pinv.w[i] = ctx->pinv[i];
    pinv.wp[i] = h_shoup(ctx->pinv[i], ctx->mods[i]);
    pinv.add[i] = 0;
  }
  double adds = 0;
  for (uint32_t b = 0; b < nb; b++) adds += (kb.add0[b] ? nq : 0) + (kb.add1[b] ? nq : 0);
  timing_begin(ctx, "ks_moddown_tail", dim3(GB::BLOCKS, nb, 2 * nq),
               8.0 * N * (3.0 * 2 * nq * nb + adds), N * (0.5 * B + 1) * 2 * nq * nb);
  k_moddown_contig_tail<LOGN><<<dim3(GB::BLOCKS, nb, 2 * nq), kNttThreads, 0, ctx->stream>>>(
      ws, kb, pinv, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup, ctx->d_ttw, ctx->d_ttw_shoup);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

template <int LOGN>
int ks_run(hck_context *ctx, const KsBatch &kb, uint32_t level, uint64_t *ws) {
  constexpr int B = split_b(LOGN);
  constexpr double N = (double)(1 << LOGN);
  using GB = Pass<B, LOGN, false>;
  const KsGeom kg = make_geom(ctx, level);
  const uint32_t nq = kg.nq, ne = kg.ne, nb = kb.n, alpha = kg.alpha;
  int rc;
  if ((rc = ks_modup<LOGN>(ctx, kb, kg, ws))) return rc;
  const double digits = (double)((nq + alpha - 1) / alpha);
  const double ext_limbs = nb * (digits * ne - nq);
  double keys = 0;  // distinct keys in the batch
  for (uint32_t b = 0; b < nb; b++) {
    bool seen = false;
    for (uint32_t k = 0; k < b; k++) seen = seen || kb.key[k] == kb.key[b];
    keys += seen ? 0 : 1;
  }
  timing_begin(ctx, "ks_contig_inner", dim3(GB::BLOCKS, nb, ne),
               8.0 * N * (ext_limbs + nb * (nq + 2.0 * ne) + 2 * digits * ne * keys),
               N * (0.5 * B * (ext_limbs + 2.0 * kg.K * nb) + 2 * digits * ne * nb));
  k_ks_contig_inner<LOGN><<<dim3(GB::BLOCKS, nb, ne), kNttThreads, 0, ctx->stream>>>(
      ws, kb, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup, ctx->d_ttw, ctx->d_ttw_shoup,
      ctx->d_itw, ctx->d_itw_shoup, ctx->d_ittw, ctx->d_ittw_shoup);
  timing_end(ctx);
  return ks_moddown<LOGN>(ctx, kb, kg, ws, true);
}

template <int LOGN>
int ks_hoisted(hck_context *ctx, const uint64_t *c0, const uint64_t *c1, uint32_t level,
               const uint32_t *galois, const hck_switch_key *const *keys, uint32_t n,
               uint64_t *const *out0, uint64_t *const *out1) {
  constexpr double N = (double)(1 << LOGN);
  const KsGeom kg = make_geom(ctx, level);
  const uint32_t nq = kg.nq, ne = kg.ne, alpha = kg.alpha;
  int rc;
  KsBatch up;
  up.n = 1;
  up.galois[0] = 1;
  up.d[0] = c1;
  if ((rc = ks_modup<LOGN>(ctx, up, kg, ws_ks(ctx)))) return rc;
  // finish the forward transform of slot 0's extended digits in place
  std::vector<std::pair<uint16_t, uint8_t>> rows;
  for (uint32_t j = 0; j < kg.dnum; j++) {
    const uint32_t lo = j * alpha;
    if (lo >= nq) break;
    const uint32_t hi = std::min(lo + alpha, nq);
    for (uint32_t t = 0; t < ne; t++)
      if (t < lo || t >= hi)
        rows.push_back({(uint16_t)(kg.off_ext + j * ne + t),
                        (uint8_t)(t < nq ? t : kg.L + (t - nq))});
  }
  for (size_t s = 0; s < rows.size(); s += kMaxRows) {
    LimbMap m;
    m.n = (uint32_t)std::min(rows.size() - s, (size_t)kMaxRows);
    for (uint32_t r = 0; r < m.n; r++) {
      m.row[r] = rows[s + r].first;
      m.mod[r] = rows[s + r].second;
    }
    if ((rc = ntt_pass(ctx, ws_ks(ctx), m, false, false, nullptr))) return rc;
  }
  const double digits = (double)((nq + alpha - 1) / alpha);
  const uint32_t limit = ks_batch_limit(ctx, level);
  for (uint32_t s = 0; s < n; s += even_batch(n - s, limit)) {
    KsBatch kb;
    kb.n = even_batch(n - s, limit);
    for (uint32_t b = 0; b < kb.n; b++) {
      kb.key[b] = keys[s + b]->data;
      kb.galois[b] = galois[s + b];
      kb.d[b] = c1;
      kb.out0[b] = out0[s + b];
      kb.out1[b] = out1[s + b];
      kb.add0[b] = c0;
      kb.add1[b] = nullptr;
      timing_begin(ctx, "ks_inner_gather", dim3((1 << LOGN) / 256, ne),
                   8.0 * N * ne * (3 * digits + 2), 2 * digits * N * ne);
      k_ks_inner_gather<LOGN><<<dim3((1 << LOGN) / 256, ne), 256, 0, ctx->stream>>>(
          ws_ks(ctx), c1, galois[s + b], b, keys[s + b]->data, kg, ctx->d_mod);
      timing_end(ctx);
    }
    if ((rc = ks_moddown<LOGN>(ctx, kb, kg, ws_ks(ctx), false))) return rc;
  }
  HCK_HIP(ctx, hipGetLastError());
  return HCK_OK;
}

// K1-K4, then each slot's accumulators added into its extended-basis sum
template <int LOGN>
int ks_pq(hck_context *ctx, const KsBatch &kb, uint32_t level, uint64_t *const *pq,
          const bool *first) {
  constexpr int B = split_b(LOGN);
  constexpr double N = (double)(1 << LOGN);
  using GB = Pass<B, LOGN, false>;
  const KsGeom kg = make_geom(ctx, level);
  const uint32_t nq = kg.nq, ne = kg.ne, nb = kb.n, alpha = kg.alpha;
  int rc;
  if ((rc = ks_modup<LOGN>(ctx, kb, kg, ws_ks(ctx)))) return rc;
  const double digits = (double)((nq + alpha - 1) / alpha);
  const double ext_limbs = nb * (digits * ne - nq);
  timing_begin(ctx, "ks_contig_inner", dim3(GB::BLOCKS, nb, ne),
               8.0 * N * (ext_limbs + nb * (nq + 2.0 * ne) + 2 * digits * ne * nb),
               N * (0.5 * B * (ext_limbs + 2.0 * kg.K * nb) + 2 * digits * ne * nb));
  k_ks_contig_inner<LOGN><<<dim3(GB::BLOCKS, nb, ne), kNttThreads, 0, ctx->stream>>>(
      ws_ks(ctx), kb, kg, ctx->d_mod, ctx->d_tw, ctx->d_tw_shoup, ctx->d_ttw,
      ctx->d_ttw_shoup, ctx->d_itw, ctx->d_itw_shoup, ctx->d_ittw, ctx->d_ittw_shoup);
  timing_end(ctx);
  HCK_HIP(ctx, hipGetLastError());
  LimbMap rows;
  rows.n = 2 * ne;
  for (uint32_t r = 0; r < 2 * ne; r++) {
    const uint32_t t = r % ne;
    rows.row[r] = (uint16_t)r;
    rows.mod[r] = (uint8_t)(t < nq ? t : kg.L + (t - nq));
  }
  std::vector<bool> done(nb, false);
  for (uint32_t b = 0; b < nb; b++) {
    if (done[b]) continue;
    std::vector<const uint64_t *> in;
    if (!first[b]) in.push_back(pq[b]);
    for (uint32_t k = b; k < nb; k++)
      if (pq[k] == pq[b]) {
        done[k] = true;
        in.push_back(ws_ks(ctx) + ((size_t)k * kg.slot_rows + kg.off_acc) * (size_t)N);
      }
    if ((rc = launch_sum_many(ctx, pq[b], in.data(), (uint32_t)in.size(), rows))) return rc;
  }
  return HCK_OK;
}

template <int LOGN>
int md_pq(hck_context *ctx, const KsBatch &kb, uint32_t level, const uint64_t *const *pq) {
  const KsGeom kg = make_geom(ctx, level);
  int rc;
  for (uint32_t b = 0; b < kb.n; b++)
    if ((rc = launch_copy(ctx, ws_ks(ctx) + ((size_t)b * kg.slot_rows + kg.off_acc) * ctx->n,
                          pq[b], (size_t)2 * kg.ne * ctx->n)))
      return rc;
  return ks_moddown<LOGN>(ctx, kb, kg, ws_ks(ctx), true);
}

}  // namespace

// Batches grow where each slot is small (low levels), so that a launch still
// fills the chip; at high levels 8 slots of 24 limbs already do, and larger
// batches measured slower there (more data between the passes of a batch).
uint32_t ks_batch_fit(const hck_context *ctx, uint32_t level) {
  const uint32_t by_rows = (uint32_t)kMaxRows / std::max<uint32_t>(level + 1, 2 * ctx->K);
  return std::max<uint32_t>(1, std::min(ks_slots(ctx), by_rows));
}

uint32_t ks_batch_limit(const hck_context *ctx, uint32_t level) {
  const uint32_t fit = ks_batch_fit(ctx, level);
  if (level < (uint32_t)HCK_MAX_LIMBS && ctx->ks_cap[level])
    return std::min<uint32_t>(fit, ctx->ks_cap[level]);
  return std::min<uint32_t>(fit, std::max<uint32_t>(1, 192 / (level + 1)));
}

int keyswitch_batch(hck_context *ctx, const KsBatch &kb, uint32_t level) {
  if (kb.n == 0) return HCK_OK;
  if (kb.n > ks_slots(ctx)) return set_error(HCK_EINVAL, "batch too large");
  int rc = ensure_workspace(ctx, ws_words_needed(ctx));
  if (rc) return rc;
  return keyswitch_batch_ws(ctx, kb, level, ws_ks(ctx));
}

int keyswitch_batch_ws(hck_context *ctx, const KsBatch &kb, uint32_t level, uint64_t *ws) {
  if (kb.n == 0) return HCK_OK;
  if (level + 1 > (uint32_t)kMaxLimbs || (level + 1) * kb.n > (uint32_t)kMaxRows ||
      2 * ctx->K * kb.n > (uint32_t)kMaxRows)
    return set_error(HCK_EINVAL, "level too high for one batched launch");
  switch (ctx->log_n) {
    case 11: return ks_run<11>(ctx, kb, level, ws);
    case 12: return ks_run<12>(ctx, kb, level, ws);
    case 13: return ks_run<13>(ctx, kb, level, ws);
    case 14: return ks_run<14>(ctx, kb, level, ws);
    case 15: return ks_run<15>(ctx, kb, level, ws);
    case 16: return ks_run<16>(ctx, kb, level, ws);
    case 17: return ks_run<17>(ctx, kb, level, ws);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

int keyswitch_core(hck_context *ctx, const uint64_t *d, uint32_t galois, uint32_t level,
                   const hck_switch_key *key, uint64_t *out0, uint64_t *out1, const uint64_t *add0,
                   const uint64_t *add1) {
  KsBatch kb;
  kb.n = 1;
  kb.key[0] = key->data;
  kb.galois[0] = galois;
  kb.d[0] = d;
  kb.out0[0] = out0;
  kb.out1[0] = out1;
  kb.add0[0] = add0;
  kb.add1[0] = add1;
  return keyswitch_batch(ctx, kb, level);
}

int keyswitch_hoisted(hck_context *ctx, const uint64_t *c0, const uint64_t *c1, uint32_t level,
                      const uint32_t *galois, const hck_switch_key *const *keys, uint32_t n,
                      uint64_t *const *out0, uint64_t *const *out1) {
  if (n == 0) return HCK_OK;
  int rc = ensure_workspace(ctx, ws_words_needed(ctx));
  if (rc) return rc;
  if (level + 1 > (uint32_t)kMaxLimbs || 2 * ctx->K > (uint32_t)kMaxRows)
    return set_error(HCK_EINVAL, "level too high for one batched launch");
  switch (ctx->log_n) {
    case 11: return ks_hoisted<11>(ctx, c0, c1, level, galois, keys, n, out0, out1);
    case 12: return ks_hoisted<12>(ctx, c0, c1, level, galois, keys, n, out0, out1);
    case 13: return ks_hoisted<13>(ctx, c0, c1, level, galois, keys, n, out0, out1);
    case 14: return ks_hoisted<14>(ctx, c0, c1, level, galois, keys, n, out0, out1);
    case 15: return ks_hoisted<15>(ctx, c0, c1, level, galois, keys, n, out0, out1);
    case 16: return ks_hoisted<16>(ctx, c0, c1, level, galois, keys, n, out0, out1);
    case 17: return ks_hoisted<17>(ctx, c0, c1, level, galois, keys, n, out0, out1);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

}  // namespace hck

namespace hck {

int keyswitch_pq(hck_context *ctx, const KsBatch &kb, uint32_t level, uint64_t *const *pq,
                 const bool *first) {
  if (kb.n == 0) return HCK_OK;
  if (kb.n > ks_batch_limit(ctx, level)) return set_error(HCK_EINVAL, "batch too large");
  int rc = ensure_workspace(ctx, ws_words_needed(ctx));
  if (rc) return rc;
  switch (ctx->log_n) {
    case 11: return ks_pq<11>(ctx, kb, level, pq, first);
    case 12: return ks_pq<12>(ctx, kb, level, pq, first);
    case 13: return ks_pq<13>(ctx, kb, level, pq, first);
    case 14: return ks_pq<14>(ctx, kb, level, pq, first);
    case 15: return ks_pq<15>(ctx, kb, level, pq, first);
    case 16: return ks_pq<16>(ctx, kb, level, pq, first);
    case 17: return ks_pq<17>(ctx, kb, level, pq, first);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

int moddown_pq(hck_context *ctx, const KsBatch &kb, uint32_t level, const uint64_t *const *pq) {
  if (kb.n == 0) return HCK_OK;
  if (kb.n > ks_batch_limit(ctx, level)) return set_error(HCK_EINVAL, "batch too large");
  int rc = ensure_workspace(ctx, ws_words_needed(ctx));
  if (rc) return rc;
  switch (ctx->log_n) {
    case 11: return md_pq<11>(ctx, kb, level, pq);
    case 12: return md_pq<12>(ctx, kb, level, pq);
    case 13: return md_pq<13>(ctx, kb, level, pq);
    case 14: return md_pq<14>(ctx, kb, level, pq);
    case 15: return md_pq<15>(ctx, kb, level, pq);
    case 16: return md_pq<16>(ctx, kb, level, pq);
    case 17: return md_pq<17>(ctx, kb, level, pq);
    default: return set_error(HCK_EPARAMS, "unsupported ring degree");
  }
}

}  // namespace hck
