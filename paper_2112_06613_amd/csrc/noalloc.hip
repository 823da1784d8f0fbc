// A device build that allocates nothing: every intermediate buffer of the
// pipeline (records, sort keys, masks, plan, edge staging, counters) is
// carved from one static device array per GPU instead of the context's
// grow-only workspace.  For callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid
// hipMalloc).
#define TCRNET_BUILDING 1
#include <mutex>

#include "api_internal.h"

namespace tcr {

namespace {

constexpr size_t kScratchBytes = (size_t)TCRNET_NOALLOC_SCRATCH_BYTES;
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

// The array lives in every GPU's memory from the time the code object is
// loaded on it until the process ends.  In host code its name is a host-side
// stand-in, never a device address: device code is handed the address that
// hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace

// Look up this device's copy of the scratch array (once per device; the
// device must be current).  Called when a context is created.
hipError_t scratch_attach(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_ptr[device] = p;
  return hipSuccess;
}

static void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace tcr

using namespace tcr;

extern "C" int32_t tcrnet_build_device_noalloc(tcrnet_ctx* ctx, const char* d_data, const uint64_t* d_offsets,
                                               uint32_t n, int32_t k, void* stream, uint32_t* d_pairs,
                                               uint64_t pair_capacity, int32_t* d_degree, uint64_t* n_edges) {
  if (!ctx || !n_edges) return set_error(TCRNET_EINVAL, "NULL context or n_edges");
  int32_t rc;
  if ((rc = check_k(k))) return rc;
  if (n > TCRNET_MAX_SEQS) return set_error(TCRNET_EINVAL, "more than 2^28 sequences");
  if (n && (!d_data || !d_offsets || !d_degree)) return set_error(TCRNET_EINVAL, "NULL device buffer");
  if (pair_capacity && !d_pairs) return set_error(TCRNET_EINVAL, "NULL pair buffer with nonzero capacity");
  (void)hipSetDevice(ctx->device);
  unsigned char* base = static_cast<unsigned char*>(scratch_ptr(ctx->device));
  if (!base) return set_error(TCRNET_EDEVICE, "no static scratch on device %d", ctx->device);
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : ctx->stream;

  // Lay the pipeline's buffers out in the scratch array, sized exactly as the
  // allocating build would size them (so run_pipeline finds them big enough
  // and allocates nothing); with no pair buffer from the caller (capacity 0)
  // the one-edge output slot comes from the scratch too.
  const Sched sched = pick_sched(ctx, n, k);
  const uint64_t capacity = pair_capacity ? pair_capacity : 1;
  size_t bytes[kPipeBufs];
  uint32_t max_desc = 0;
  pipeline_sizes(n, 1, k, sched.texts_per_item, capacity, 0, bytes, &max_desc);
  size_t need = 0;
  for (int i = 0; i < kPipeBufs; ++i) need += align_up(bytes[i]);
  const size_t own_pairs = pair_capacity ? 0 : align_up(8);
  need += own_pairs;
  if (need > kScratchBytes)
    return set_error(TCRNET_EINVAL,
                     "%u sequences with room for %llu edges need %llu bytes of scratch; the static scratch holds "
                     "%llu",
                     n, (unsigned long long)capacity, (unsigned long long)need, (unsigned long long)kScratchBytes);
  Pipeline pl;
  DevBuf* bufs[kPipeBufs];
  pipeline_buffers(pl, bufs);
  size_t pos = 0;
  for (int i = 0; i < kPipeBufs; ++i) {
    bufs[i]->borrow(base + pos, bytes[i]);
    pos += align_up(bytes[i]);
  }
  pl.n_cap = n ? n : 1;
  pl.e_cap = capacity;
  pl.desc_cap = max_desc;

  PipeParams pp;
  pp.d_data = d_data;
  pp.d_off = d_offsets;
  pp.n = n;
  pp.k = k;
  pp.capacity = capacity;
  pp.d_pairs = pair_capacity ? d_pairs : reinterpret_cast<uint32_t*>(base + pos);
  pp.d_deg = d_degree;
  uint64_t E = 0;
  tcrnet_build_info info{};
  rc = run_pipeline(ctx, pl, pp, st, false, nullptr, &E, &info);
  ctx->last = info;
  *n_edges = E;
  return rc;
}
