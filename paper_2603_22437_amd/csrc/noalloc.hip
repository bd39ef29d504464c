// Rotation that allocates nothing (hck_rotate_noalloc): the key switch runs
// in a static device array instead of the context's allocated workspace, for
// callers that cannot allocate device memory (code under stream capture,
// serving loops that forbid allocation).
//
// The array holds one key-switch batch slot (ws_ks_rows rows of N words) and
// a copy of c0 for an output that aliases its input.  Every rotation on a GPU
// shares that GPU's array: calls that overlap in time on one GPU (two
// streams, two contexts, two threads) race and must be serialized by the
// caller.  Nothing in it has to start at zero: each key-switch stage writes
// the rows it later reads, so the last call's contents are never used.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace hck {

namespace {

// one slot at the largest shape used here (N = 2^16, L = 30, K = 10,
// dnum = 3: 290 + 30 rows of 512 KiB) fits exactly
constexpr size_t kScratchBytes = (size_t)160 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint64_t scratch[kScratchBytes / sizeof(uint64_t)];

std::mutex g_scratch_mu;
uint64_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's array (the caller made ctx->device current).
// The array's name in host code is only a host-side stand-in; the address
// comes from the runtime, once per device.
int scratch_address(hck_context *ctx, uint64_t **out) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return set_error(HCK_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(HCK_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                        hipGetErrorString(e));
    g_scratch_ptr[ctx->device] = static_cast<uint64_t *>(p);
  }
  *out = g_scratch_ptr[ctx->device];
  return HCK_OK;
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

size_t noalloc_scratch_needed(const hck_context *ctx) {
  return (ws_ks_rows(ctx) + ctx->L) * (size_t)ctx->n * sizeof(uint64_t);
}

int rotate_noalloc(hck_context *ctx, const hck_ciphertext *a, int32_t step,
                   const hck_galois_keys *gks, hck_ciphertext *out) {
  if (a->size != 2) return set_error(HCK_EINVAL, "rotation needs a 2-part ciphertext");
  if (!out->data || out->cap_polys < 2)
    return set_error(HCK_EINVAL,
                     "output must already hold two polynomials (an earlier result or import)");
  const size_t need = noalloc_scratch_needed(ctx);
  if (need > kScratchBytes)
    return set_error(HCK_EINVAL, "this context needs " + std::to_string(need >> 20) +
                                     " MiB of rotation scratch, above the " +
                                     std::to_string(kScratchBytes >> 20) + " MiB maximum");
  const uint32_t level = a->level;
  const size_t n = ctx->n, ps = (size_t)ctx->L * n;
  if ((int64_t)step % (int64_t)(n / 2) == 0) {
    if (out != a) {
      for (uint32_t p = 0; p < 2; p++) {
        const int rc = launch_copy(ctx, out->data + p * ps, a->data + p * ps, (level + 1) * n);
        if (rc) return rc;
      }
    }
  } else {
    if (!gks) return set_error(HCK_EINVAL, "null Galois keys");
    const uint32_t g = galois_of_step(ctx, step);
    auto it = gks->keys.find(g);
    if (it == gks->keys.end())
      return set_error(HCK_ENOKEY, "no Galois key for element " + std::to_string(g));
    uint64_t *ws = nullptr;
    int rc = scratch_address(ctx, &ws);
    if (rc) return rc;
    // (phi_g(c0), 0) + KeySwitch(phi_g(c1)); the final launch gathers c0
    // while it writes the output, so an output aliasing the input reads a
    // copy of c0 placed after the key-switch slot
    KsBatch kb;
    const uint64_t *c0 = a->data;
    if (out == a) {
      kb.add0_src[0] = a->data;    // copied by the first launch
      c0 = ws + ws_ks_rows(ctx) * n;
    }
    kb.n = 1;
    kb.key[0] = it->second->data;
    kb.galois[0] = g;
    kb.d[0] = a->data + ps;
    kb.out0[0] = out->data;
    kb.out1[0] = out->data + ps;
    kb.add0[0] = c0;
    kb.add1[0] = nullptr;
    if ((rc = keyswitch_batch_ws(ctx, kb, level, ws))) return rc;
  }
  out->size = 2;
  out->level = level;
  out->scale = a->scale;
  return HCK_OK;
}

}  // namespace hck
