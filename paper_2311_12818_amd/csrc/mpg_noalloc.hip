// Allocation-free variant of manifold_walk_batch for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc): the persistent form's bucket order,
// queue heads and class bytes live in a file-scope device array instead of
// an mpg_workspace, and every per-length kernel runs on the caller's stream
// (the internal worker streams are created lazily by the other entry
// points, which is a resource allocation this variant avoids).
#include "mpg_internal.h"

namespace {

constexpr int kCounterWords = MPG_WS_COUNTERS;
constexpr int kPermWords = MPG_NOALLOC_MAX_CHAINS + KMAX * 64;
constexpr int kClassWords = (MPG_NOALLOC_MAX_CHAINS + 64 + 3) / 4;
constexpr size_t kScratchWords = (size_t)kCounterWords + kPermWords + kClassWords;

// One copy per device, held until the process ends.  Host code never passes
// this name to a kernel or a copy: it is only resolved to the device's own
// address with hipGetSymbolAddress below.
static __device__ __align__(256) int32_t scratch[kScratchWords];

std::mutex g_mu;
int32_t* g_addr[64] = {};

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
mpg_status scratch_address(int32_t** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MPG_ERR_UNSUPPORTED, "manifold_walk_batch_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MPG_ERR_HIP, "manifold_walk_batch_noalloc: no device address for the scratch array");
    g_addr[dev] = (int32_t*)p;
  }
  *out = g_addr[dev];
  return MPG_OK;
}

}  // namespace

extern "C" mpg_status manifold_walk_batch_noalloc(const mpg_scene* s, const mpg_walk_params* p,
                                                  const mpg_endpoints* ep, const mpg_chains* seeds,
                                                  const int8_t* d_seed_status, mpg_chains* out,
                                                  const mpg_walk_out* wout, void* stream) {
  if (!p || !ep) return fail(MPG_ERR_INVALID_ARG, "manifold_walk_batch_noalloc: NULL params or endpoints");
  if (ep->N > MPG_NOALLOC_MAX_CHAINS)
    return fail(MPG_ERR_INVALID_ARG, "manifold_walk_batch_noalloc: N exceeds MPG_NOALLOC_MAX_CHAINS (" +
                                         std::to_string(MPG_NOALLOC_MAX_CHAINS) + ")");
  if (p->form == MPG_FORM_PERSISTENT && p->bucketing >= 2)
    return fail(MPG_ERR_UNSUPPORTED, "manifold_walk_batch_noalloc: spatial bucketing (2, 3) needs a workspace");
  int32_t* base = nullptr;
  mpg_status st = scratch_address(&base);
  if (st != MPG_OK) return st;
  mpg_workspace ws;
  ws.cap = MPG_NOALLOC_MAX_CHAINS;
  ws.counters = base;
  ws.perm = base + kCounterWords;
  ws.aux = base + kCounterWords + kPermWords;
  ws.cells = nullptr;
  ws.single_stream = 1;
  return manifold_walk_batch(s, p, ep, seeds, d_seed_status, out, wout, &ws, stream);
}
