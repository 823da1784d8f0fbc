// Host-side orchestration shared by the build, batch and serving entry points.
#pragma once
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstddef>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"

namespace tcr {

// Device and pinned-host allocation with an optional injected failure
// (tcrnet_debug_fail_alloc): the allocation after the armed number of
// successful ones reports hipErrorOutOfMemory, once.
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t host_malloc(void** p, size_t bytes);
void arm_alloc_failure(int64_t after);  // -1: disarm

// Chunks of a host-side copy of `bytes` handed to host_parallel: one per MiB,
// at most 32 (starting and joining its threads costs about 0.2 ms, more than
// a copy of under a MiB takes on one thread).
constexpr uint32_t kHostChunks = 32;
inline uint32_t host_chunks(uint64_t bytes) {
  const uint64_t c = bytes >> 20;
  return c < 1 ? 1u : (c > kHostChunks ? kHostChunks : (uint32_t)c);
}

// Runs f(i) for every i in [0, n) on up to 8 host threads that take indices
// one at a time (the items of a batch differ in size).
template <class F>
void host_parallel(uint32_t n, F&& f) {
  const unsigned hc = std::thread::hardware_concurrency();
  const uint32_t nt = std::min<uint32_t>(n, std::min(8u, hc ? hc : 1u));
  if (nt <= 1) {
    for (uint32_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<uint32_t> next{0};
  auto worker = [&]() {
    for (uint32_t i = next.fetch_add(1); i < n; i = next.fetch_add(1)) f(i);
  };
  std::vector<std::thread> pool;
  pool.reserve(nt - 1);
  for (uint32_t t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (std::thread& t : pool) t.join();
}

// Page-locked host staging buffer, grow-only (copies from and to it run as
// direct DMA; freeing one synchronises the device, so it only grows).
struct Pinned {
  void* p = nullptr;
  size_t cap = 0;
  Pinned() = default;
  Pinned(const Pinned&) = delete;
  Pinned& operator=(const Pinned&) = delete;
  ~Pinned() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap && p) return hipSuccess;
    release();
    size_t nb = bytes < 4096 ? 4096 : bytes + bytes / 4;
    hipError_t e = host_malloc(&p, nb);
    if (e == hipSuccess) cap = nb;
    else p = nullptr;
    return e;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Grow-only device buffer, or a borrowed view of memory the buffer does not
// own (never freed, never grown).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool borrowed = false;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && !borrowed) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    borrowed = false;
  }
  void borrow(void* q, size_t bytes) {
    release();
    p = q;
    cap = bytes;
    borrowed = true;
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap && p) return hipSuccess;
    if (borrowed) return hipErrorOutOfMemory;
    release();
    const size_t nb = bytes < 256 ? 256 : bytes + bytes / 8;
    hipError_t e = dev_malloc(&p, nb);
    if (e == hipSuccess) cap = nb;
    else p = nullptr;
    return e;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Resident waves per SIMD of the pair kernel (its register count allows six).
constexpr uint32_t kPairWavesPerSimd = 6;

// Default texts per work item for a launch over n sequences at threshold k:
// about n / 195, rounded down to a power of two in [256, 16384], and one
// doubling more at k <= 1 from 150,000 sequences on.  Measured best: 256 at
// 50,000 (the launch lasts as long as its heaviest items, and 256 texts
// shorten them more than the extra items cost: 0.196 -> 0.172 ms at k = 1,
// 0.327 -> 0.304 at k = 2, while 128 and 64 are slower again), 512 at
// 100,000 (1,024: 0.230 -> 0.260 ms); at k = 1, 2,048 at 200,000 (0.427 ->
// 0.424 ms against 1,024), 4,096 at 400,000 (0.739 -> 0.729 against 2,048)
// and 8,192 at 800,000 (1.39 -> 1.30 ms against 4,096; 16,384: 1.33); at
// k = 2, 800,000 keeps 4,096 (11.32 ms, 11.47 at 8,192).
inline uint32_t default_texts_per_item(uint64_t n, int k) {
  uint32_t t = 256;
  while (t < 16384 && (uint64_t)(2 * t) * 195 <= n) t *= 2;
  if (k <= 1 && n >= 150000 && t < 16384) t *= 2;
  return t;
}

// Pair-kernel schedule.
struct Sched {
  uint32_t texts_per_item = 16384;
  uint32_t waves_per_simd = kPairWavesPerSimd;
  bool peq_lds = false;
  bool pack = true;  // two patterns per lane for patterns of <= 16 residues
  bool tuned = false;  // chosen by the autotuner
  bool count_work = false;  // pair kernel's counting variant (same traversal)
};

// Device buffers of one build pipeline (encode -> sort -> bucket -> plan ->
// pairs -> canonicalise).  One per context, one per serving slot.
struct Pipeline {
  DevBuf rec, key, key2, val, val2, srec, speq, off, descs, ibase, meta, tmp, edges, edist, ekeys, ekeys2;
  uint64_t n_cap = 0, e_cap = 0;
  uint32_t desc_cap = 0;
  Counters* cnt() const { return meta.as<Counters>(); }
  Plan* plan() const { return reinterpret_cast<Plan*>(meta.as<char>() + sizeof(Counters)); }
};

struct Meta {  // host copy of the counters and plan header
  Counters cnt;
  Plan plan;
};

// Inputs and outputs of one pipeline run.
struct PipeParams {
  const char* d_data = nullptr;
  const uint64_t* d_off = nullptr;
  uint32_t n = 0;
  const uint32_t* d_segoff = nullptr;  // NULL: one segment
  uint32_t n_seg = 1;
  uint32_t id_base = 0;
  int k = 1;
  Sched sched;
  uint64_t capacity = 0;               // edge capacity
  uint32_t* d_pairs = nullptr;         // 2 * capacity words (sorted output)
  int32_t* d_deg = nullptr;            // n words
  uint8_t* d_dist = nullptr;           // capacity bytes: edge distances (NULL: not kept)
};

uint32_t bits_for(uint64_t v);  // number of bits to hold values < v (>= 1)

// Bytes of each pipeline buffer for these sizes, in the order of
// pipeline_buffers() (max_desc: 0 = the bound of a self plan over n
// sequences in n_seg segments).
constexpr int kPipeBufs = 16;
void pipeline_sizes(uint64_t n, uint32_t n_seg, int k, uint32_t T, uint64_t capacity, uint32_t max_desc,
                    size_t bytes[kPipeBufs], uint32_t* max_desc_out);
void pipeline_buffers(Pipeline& pl, DevBuf* bufs[kPipeBufs]);

// Allocate every buffer the pipeline needs for these sizes.
hipError_t pipeline_reserve(Pipeline& pl, uint64_t n, uint32_t n_seg, int k, uint32_t T, uint64_t capacity,
                            uint32_t max_desc = 0);

// Stage 1 (steps a1-a2): encode, sort by (segment, length, residues), bucket
// bounds and gather into sorted records / bit masks.  Writes srec (n), speq
// (n) and off (n_seg * 64 + 1) -- the pipeline's own buffers unless other
// outputs are given.  Uses pl.rec/key/val/tmp as scratch.
struct SetOut {
  SeqRec* srec = nullptr;
  PeqRec* speq = nullptr;
  uint32_t* off = nullptr;
};
void stage_prepare(Pipeline& pl, const char* d_data, const uint64_t* d_off, uint32_t n, const uint32_t* d_segoff,
                   uint32_t n_seg, uint32_t id_base, uint32_t id_tag, const SetOut& out, hipStream_t st);
// The same from records already encoded (ids kept): sorts n records of `rec`.
void stage_prepare_records(Pipeline& pl, const SeqRec* rec, uint32_t n, const SetOut& out, hipStream_t st);

// Stage 2 (steps a3-a6): plan the parts and run the pair kernel into
// pl.edges (capacity edges).  Resets the work counters (not the input error).
void stage_pairs(Pipeline& pl, const PlanPart* d_parts, uint32_t n_parts, const PlanPart& inline_part, int k,
                 const Sched& sched, uint64_t capacity, uint32_t grid_blocks, hipStream_t st, hipEvent_t ev0,
                 hipEvent_t ev1, bool keep_dist = false);

// Stage 3 (steps a7-a8): canonical sorted pairs into d_pairs; mode 0 adds
// both ends to deg, mode 1 (query tag first) adds the first end; d_dist (may
// be NULL) receives the distances kept by stage_pairs(keep_dist).
void stage_canon(Pipeline& pl, int mode, int shift, uint64_t capacity, uint32_t* d_pairs, int32_t* d_deg,
                 hipStream_t st, uint8_t* d_dist = nullptr);

// Enqueue the whole build on `st` with no host synchronisation.  ev0/ev1 (may
// be NULL) bracket the pair kernel.
void pipeline_enqueue(Pipeline& pl, const PipeParams& pp, int device, hipStream_t st, hipEvent_t ev0,
                      hipEvent_t ev1);

// Copy counters and plan header to the host (synchronises `st`).
hipError_t pipeline_meta(const Pipeline& pl, Meta* host_meta, hipStream_t st);

// Error reporting (thread-local message).
int32_t set_error(int32_t code, const char* fmt, ...);
int32_t hip_error(hipError_t e, const char* what);
std::string input_error_message(unsigned long long err);

}  // namespace tcr
