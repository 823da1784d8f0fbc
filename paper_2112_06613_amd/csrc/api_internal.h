// Objects behind the C-ABI handles (library-internal).
#pragma once
#include <map>
#include <memory>
#include <utility>
#include <vector>

#include "pipeline.h"
#include "tcrnet.h"

namespace tcr {

// Identity of a captured batch graph: the shape, and the address and size of
// every device buffer the captured launches read or write (kernel arguments
// are baked into the graph, so any reallocation requires a new capture).
struct BatchKey {
  uint32_t n = 0, n_seg = 0;
  int k = 0;
  uint32_t T = 0, W = 0;
  bool lds = false, pack = false, count = false;
  uint64_t capacity = 0;
  uint32_t desc_cap = 0;
  std::vector<std::pair<const void*, size_t>> bufs;
  bool operator==(const BatchKey& o) const {
    return n == o.n && n_seg == o.n_seg && k == o.k && T == o.T && W == o.W && lds == o.lds && pack == o.pack && count == o.count &&
           capacity == o.capacity && desc_cap == o.desc_cap && bufs == o.bufs;
  }
};

// Launch forms the autotuner keeps separate tables for.
constexpr int kFormPlain = 0;  // one build (plain, device, weighted, index)
constexpr int kFormBatch = 1;  // one batched launch over many repertoires

// Autotuner table key: launch form, size class (bits of the sequence count)
// and threshold; the device's arch and CU count key the persisted file.
struct TuneKey {
  int form = 0, size_class = 0, k = 0;
  bool operator<(const TuneKey& o) const {
    if (form != o.form) return form < o.form;
    if (size_class != o.size_class) return size_class < o.size_class;
    return k < o.k;
  }
};
struct TuneEntry {
  Sched sched;
  double ms = 0.0;  // measured device time of the chosen schedule
};

// Uploaded input of a batched build.
struct BatchInput {
  std::vector<uint32_t> seg;  // repertoire r = global ids [seg[r], seg[r+1])
  uint32_t n = 0, n_reps = 0;
};

}  // namespace tcr

struct tcrnet_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  tcrnet_opts opts{};
  tcr::Pipeline pipe;
  tcr::DevBuf in_data, in_off, in_seg, out_pairs, out_deg, out_dist;
  tcr::DevBuf ana_ws, ana_out;  // network-analysis workspace
  hipEvent_t ev_p0 = nullptr, ev_p1 = nullptr, ev_b0 = nullptr, ev_b1 = nullptr;
  tcr::Meta* h_meta = nullptr;  // pinned host copy of a build's counters and plan
  std::map<tcr::TuneKey, tcr::TuneEntry> tuned;  // autotuner choices
  char arch[64] = {0};                           // gcnArchName of the device
  int cus = 0;                                   // compute units
  tcrnet_build_info last{};
  // batched build: captured launch sequence
  hipGraphExec_t batch_exec = nullptr;
  tcr::BatchKey batch_key;
  uint64_t batch_captures = 0;  // graphs captured so far (diagnostic)
  tcr::Pinned batch_in, batch_out;  // batched build: staging of inputs and results
};

namespace tcr {

// Schedule of a launch over n sequences (form: kFormPlain or kFormBatch).
Sched pick_sched(const tcrnet_ctx* ctx, uint64_t n, int k, int form = kFormPlain);
int32_t batch_upload(tcrnet_ctx* ctx, const tcrnet_seqs* reps, uint32_t n_reps, BatchInput* bi);
int32_t batch_launch(tcrnet_ctx* ctx, const BatchInput& bi, int32_t k, const Sched& sched, uint64_t* E,
                     tcrnet_build_info* info);
// Find this device's copy of the static scratch array of the allocation-free
// build (once per device, with the device current).
hipError_t scratch_attach(int device);
void note_work(const Sched& sched, const Meta& m, tcrnet_build_info* inf);
int32_t check_k(int32_t k);
int32_t check_host_seqs(const tcrnet_seqs* s, const char* what);
int32_t run_pipeline(tcrnet_ctx* ctx, Pipeline& pl, PipeParams pp, hipStream_t st, bool grow_ok,
                     DevBuf* pairs_buf, uint64_t* E, tcrnet_build_info* info, DevBuf* dist_buf = nullptr);

}  // namespace tcr
