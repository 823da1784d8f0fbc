// Objects behind the C-ABI handles (library-internal).
#pragma once
#include <map>
#include <memory>
#include <utility>
#include <vector>

#include "pipeline.h"
#include "tcrnet.h"

namespace tcr {

// Identity of a captured batch graph: the shape and every buffer address the
// captured launches use.
struct BatchKey {
  uint32_t n = 0, n_seg = 0;
  int k = 0;
  uint32_t T = 0, W = 0;
  bool lds = false, pack = false;
  uint64_t capacity = 0;
  void *rec = nullptr, *edges = nullptr, *tmp = nullptr, *pairs = nullptr, *data = nullptr;
  bool operator==(const BatchKey& o) const {
    return n == o.n && n_seg == o.n_seg && k == o.k && T == o.T && W == o.W && lds == o.lds && pack == o.pack &&
           capacity == o.capacity && rec == o.rec && edges == o.edges && tmp == o.tmp && pairs == o.pairs &&
           data == o.data;
  }
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
  std::map<std::pair<int, int>, tcr::Sched> tuned;  // (size class, k) -> schedule
  tcrnet_build_info last{};
  // batched build: captured launch sequence
  hipGraphExec_t batch_exec = nullptr;
  tcr::BatchKey batch_key;
  std::vector<char> batch_host;
};

namespace tcr {

// Schedule of a launch over n sequences.
Sched pick_sched(const tcrnet_ctx* ctx, uint64_t n, int k);
int32_t run_pipeline(tcrnet_ctx* ctx, Pipeline& pl, PipeParams pp, hipStream_t st, bool grow_ok,
                     DevBuf* pairs_buf, uint64_t* E, tcrnet_build_info* info, DevBuf* dist_buf = nullptr);

}  // namespace tcr
