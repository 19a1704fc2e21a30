// clak_run_block_static: clak_run_block with the block's scratch buffers in a
// file-scope device array of the library instead of a workspace slot, for
// callers that cannot allocate device memory around a call.
//
// The scratch of one SNP block (the int8 genotype panel, the per-SNP
// statistics, the ingest partials, and the rotated SNPs and their digit
// planes or the single-trait partials) is carved from `scratch`, one copy per
// GPU.  In host code `scratch` names a host-side stand-in, not device memory,
// so its device address is looked up once per device with
// hipGetSymbolAddress and only that address is used from then on.  Every
// call on a GPU shares that GPU's copy, which keeps the last call's contents;
// the per-block kernels write every scratch byte they later read, so nothing
// needs clearing.  Calls that overlap on one GPU race on the array.
#include <mutex>

#include "clak_internal.hpp"

using namespace clak;

namespace {

constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) char scratch[CLAK_STATIC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

// Device address of this device's copy of `scratch` (the device must be current).
clak_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(CLAK_E_DEVICE, "run_block_static: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CLAK_E_DEVICE, "run_block_static: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return CLAK_OK;
}

}  // namespace

extern "C" {

clak_status clak_plan_block_scratch_size(clak_plan_t h, size_t* bytes) {
  Plan* p = reinterpret_cast<Plan*>(h);
  if (!p || !bytes) return fail(CLAK_E_ARG, "plan_block_scratch_size: null argument");
  *bytes = slot_bytes(*p, nullptr, nullptr);
  return ok();
}

clak_status clak_run_block_static(clak_plan_t h, int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg,
                                  void* d_b, void* d_se, int out_dtype, int64_t ldo, uint8_t* d_flags,
                                  void* d_pval) {
  Plan* p = reinterpret_cast<Plan*>(h);
  clak_status s = need_state(p, ST_READY, "run_block_static");
  if (s) return s;
  if (p->flags & CLAK_STAGE_GENOTYPES)
    return fail(CLAK_E_UNSUPPORTED, "run_block_static: CLAK_STAGE_GENOTYPES plans stage through their workspace");
  if (p->profiling != CLAK_PROFILE_OFF)
    return fail(CLAK_E_STATE, "run_block_static: the stage profiler creates events; turn it off first");
  s = validate_block(p, m_blk, d_G, g_dtype, ldg, d_b, d_se, out_dtype, ldo, d_flags, d_pval);
  if (s) return s;
  const size_t need = slot_bytes(*p, nullptr, nullptr);
  if (need > (size_t)CLAK_STATIC_SCRATCH_BYTES)
    return fail(CLAK_E_UNSUPPORTED, "run_block_static: the plan's block scratch needs %zu bytes, the library's "
                "array holds %zu (smaller max_block or n)", need, (size_t)CLAK_STATIC_SCRATCH_BYTES);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(CLAK_E_DEVICE, "run_block_static: the plan's device must be current");
  void* base = nullptr;
  s = scratch_address(dev, &base);
  if (s) return s;
  // slot 0 of the plan points at the array for this call only
  const Slot saved = p->ws.slot[0];
  slot_bytes(*p, &p->ws.slot[0], (char*)base);
  s = enqueue_block(p, 0, p->stream, p->stream, nullptr, m_blk, d_G, g_dtype, ldg,
                    cell_out(d_b, d_se, d_pval, d_flags, ldo, out_dtype));
  p->ws.slot[0] = saved;
  select_slot(*p, 0);
  if (s) return s;
  return ok();
}

}  // extern "C"
