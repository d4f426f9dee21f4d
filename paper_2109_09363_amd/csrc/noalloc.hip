// Projection for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc): the
// same planning and projection kernels as hyp_plan + hyp_project, with the
// workspace taken from one static device array per GPU instead of a
// caller-owned buffer.
//
// The array lives for the whole process on every GPU the library runs on.
// Its device address is obtained once per device with hipGetSymbolAddress
// (with that device current) and only that address is handed to kernels,
// memsets or copies; the array's name is a host-side stand-in.  Every call
// on one GPU shares that GPU's array and leaves its contents behind: each
// call re-plans the flags, and every kernel of the projection clears what
// it needs to start at zero, as with a fresh workspace.  Two calls that
// overlap on one GPU (two streams, two threads) race on the array.
#include <mutex>

#include "../../include/hyproj.h"
#include "internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;  // HYP_NOALLOC_MAX_BYTES
static_assert(kScratchBytes == (size_t)HYP_NOALLOC_MAX_BYTES, "header and library agree");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up once per device).
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HYP_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HYP_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HYP_OK;
}

}  // namespace

extern "C" int hyp_project_noalloc(hyp_ctx* ctx, const hyp_grid* g, const hyp_fields* f,
                                   double threshold, const hyp_opts* o, hipStream_t stream,
                                   hyp_result* res) {
  if (!ctx || !g || !f || !o || !res || !f->flags) return HYP_EINVAL;
  size_t need = 0;
  int rc = hyp_workspace_size(ctx, g, &need);
  if (rc != HYP_OK) return rc;
  if (need > kScratchBytes) return HYP_EWORKSPACE;
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc != HYP_OK) return rc;
  return hyp::project_checked(ctx, g, f, threshold, o, ws, kScratchBytes, stream, res, true);
}
