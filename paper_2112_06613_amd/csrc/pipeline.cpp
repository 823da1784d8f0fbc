// Host orchestration of one build pipeline: buffer sizing and the launch
// sequence, with no host synchronisation inside (so the same sequence can be
// captured in a HIP graph).
#include "pipeline.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <atomic>
#include <cstdio>

namespace tcr {

// The gather writes the walk arrays' residue codes from a record's first
// word, which holds residues 0-5: the walk's sibling-loop depth cannot exceed
// six without that changing (a depth of 7 gave wrong edges; 5 was slower,
// 1.31 -> 1.43 ms at N = 800,000).
static_assert(kWalkDepth <= 6, "walk codes come from SeqRec::w[0] (six residues)");

namespace {
thread_local std::string g_last_error;
std::atomic<int64_t> g_fail_after{-1};  // successful allocations before an injected failure (-1: none)

// roctx range over the host-side launch sequence of one stage (shown by
// rocprofv3 --marker-trace beside the kernels the stage enqueues).
struct StageRange {
  explicit StageRange(const char* name) { roctxRangePushA(name); }
  ~StageRange() { roctxRangePop(); }
  StageRange(const StageRange&) = delete;
  StageRange& operator=(const StageRange&) = delete;
};

bool injected_failure() {
  int64_t v = g_fail_after.load();
  while (v >= 0) {
    if (g_fail_after.compare_exchange_weak(v, v - 1)) return v == 0;
  }
  return false;
}
}  // namespace

hipError_t dev_malloc(void** p, size_t bytes) {
  if (injected_failure()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

hipError_t host_malloc(void** p, size_t bytes) {
  if (injected_failure()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

void arm_alloc_failure(int64_t after) { g_fail_after.store(after < 0 ? -1 : after); }

const char* last_error_text() { return g_last_error.c_str(); }
void clear_error() { g_last_error.clear(); }

int32_t set_error(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int32_t hip_error(hipError_t e, const char* what) {
  return set_error(e == hipErrorOutOfMemory ? 2 : 3, "%s: %s", what, hipGetErrorString(e));
}

std::string input_error_message(unsigned long long err) {
  char buf[160];
  const unsigned long long idx = err >> 2;
  if ((err & 3u) == 1u)
    snprintf(buf, sizeof buf, "sequence %llu: residue outside the 20-letter amino-acid alphabet", idx);
  else
    snprintf(buf, sizeof buf, "sequence %llu: length must be 1..32", idx);
  return buf;
}

uint32_t bits_for(uint64_t v) {
  uint32_t b = 1;
  while (b < 64 && (1ull << b) < v) ++b;
  return b;
}

static uint32_t seg_bits_for(uint32_t n_seg) { return n_seg <= 1 ? 0 : bits_for(n_seg); }

void pipeline_buffers(Pipeline& pl, DevBuf* bufs[kPipeBufs]) {
  DevBuf* b[kPipeBufs] = {&pl.rec,   &pl.key,   &pl.key2,  &pl.val,  &pl.val2,  &pl.srec,  &pl.speq,  &pl.off,
                          &pl.descs, &pl.ibase, &pl.meta,  &pl.tmp,  &pl.edges, &pl.edist, &pl.ekeys, &pl.ekeys2};
  for (int i = 0; i < kPipeBufs; ++i) bufs[i] = b[i];
}

void pipeline_sizes(uint64_t n, uint32_t n_seg, int k, uint32_t T, uint64_t capacity, uint32_t max_desc,
                    size_t bytes[kPipeBufs], uint32_t* max_desc_out) {
  const uint64_t nn = n ? n : 1;
  if (!max_desc) max_desc = plan_max_desc_self(n_seg, k, T, n);
  const uint64_t cap = capacity ? capacity : 1;
  const size_t b[kPipeBufs] = {
      nn * sizeof(SeqRec),                          // rec
      nn * 8,                                       // key
      nn * 8,                                       // key2
      nn * 4,                                       // val
      nn * 4,                                       // val2
      sorted_rec_bytes(nn),                         // srec (records, then walk arrays)
      nn * sizeof(PeqRec),                          // speq
      ((uint64_t)n_seg * 64 + 1) * 4,               // off
      (uint64_t)max_desc * sizeof(Desc),            // descs
      (uint64_t)max_desc * 8,                       // ibase
      sizeof(Counters) + sizeof(Plan) + 64,         // meta
      radix_tmp_words(nn > cap ? nn : cap) * 4,     // tmp
      cap * 8,                                      // edges
      cap,                                          // edist
      cap * 8,                                      // ekeys
      cap * 8,                                      // ekeys2
  };
  for (int i = 0; i < kPipeBufs; ++i) bytes[i] = b[i];
  *max_desc_out = max_desc;
}

hipError_t pipeline_reserve(Pipeline& pl, uint64_t n, uint32_t n_seg, int k, uint32_t T, uint64_t capacity,
                            uint32_t max_desc) {
  size_t bytes[kPipeBufs];
  DevBuf* bufs[kPipeBufs];
  pipeline_sizes(n, n_seg, k, T, capacity, max_desc, bytes, &max_desc);
  pipeline_buffers(pl, bufs);
  for (int i = 0; i < kPipeBufs; ++i) {
    const hipError_t e = bufs[i]->ensure(bytes[i]);
    if (e != hipSuccess) return e;
  }
  pl.n_cap = n ? n : 1;
  pl.e_cap = capacity ? capacity : 1;
  pl.desc_cap = max_desc;
  return hipSuccess;
}

void stage_prepare(Pipeline& pl, const char* d_data, const uint64_t* d_off, uint32_t n, const uint32_t* d_segoff,
                   uint32_t n_seg, uint32_t id_base, uint32_t id_tag, const SetOut& out, hipStream_t st) {
  StageRange range("tcrnet:prepare");
  const uint32_t seg_bits = seg_bits_for(n_seg);
  SeqRec* srec = out.srec ? out.srec : pl.srec.as<SeqRec>();
  PeqRec* speq = out.speq ? out.speq : pl.speq.as<PeqRec>();
  uint32_t* off = out.off ? out.off : pl.off.as<uint32_t>();
  const uint32_t n_combo = n_seg * 64;
  if (n == 0) {
    launch_fill_u32(off, n_combo + 1, 0u, st);
    return;
  }
  launch_encode(d_data, d_off, n, d_segoff, n_seg, seg_bits, id_base, id_tag, pl.rec.as<SeqRec>(),
                pl.key.as<uint64_t>(), pl.val.as<uint32_t>(), pl.cnt(), st);
  const bool alt = radix_sort(pl.key.as<uint64_t>(), pl.key2.as<uint64_t>(), pl.val.as<uint32_t>(),
                              pl.val2.as<uint32_t>(), n, nullptr, encode_key_bits(seg_bits), pl.tmp.as<uint32_t>(),
                              &pl.cnt()->fault, st);
  const uint64_t* skey = alt ? pl.key2.as<uint64_t>() : pl.key.as<uint64_t>();
  const uint32_t* sval = alt ? pl.val2.as<uint32_t>() : pl.val.as<uint32_t>();
  launch_bucket_bounds(skey, n, encode_combo_shift(seg_bits), n_combo, off, st);
  launch_gather(pl.rec.as<SeqRec>(), sval, skey, n, seg_bits, srec, speq, st);
}

void stage_prepare_records(Pipeline& pl, const SeqRec* rec, uint32_t n, const SetOut& out, hipStream_t st) {
  StageRange range("tcrnet:prepare_records");
  SeqRec* srec = out.srec ? out.srec : pl.srec.as<SeqRec>();
  PeqRec* speq = out.speq ? out.speq : pl.speq.as<PeqRec>();
  uint32_t* off = out.off ? out.off : pl.off.as<uint32_t>();
  if (n == 0) {
    launch_fill_u32(off, 65, 0u, st);
    return;
  }
  launch_record_keys(rec, n, pl.key.as<uint64_t>(), pl.val.as<uint32_t>(), st);
  const bool alt = radix_sort(pl.key.as<uint64_t>(), pl.key2.as<uint64_t>(), pl.val.as<uint32_t>(),
                              pl.val2.as<uint32_t>(), n, nullptr, encode_key_bits(0), pl.tmp.as<uint32_t>(),
                              &pl.cnt()->fault, st);
  const uint64_t* skey = alt ? pl.key2.as<uint64_t>() : pl.key.as<uint64_t>();
  const uint32_t* sval = alt ? pl.val2.as<uint32_t>() : pl.val.as<uint32_t>();
  launch_bucket_bounds(skey, n, encode_combo_shift(0), 64, off, st);
  launch_gather(rec, sval, skey, n, 0, srec, speq, st);
}

void stage_pairs(Pipeline& pl, const PlanPart* d_parts, uint32_t n_parts, const PlanPart& inline_part, int k,
                 const Sched& sched, uint64_t capacity, uint32_t grid_blocks, hipStream_t st, hipEvent_t ev0,
                 hipEvent_t ev1, bool keep_dist) {
  StageRange range("tcrnet:pairs");
  Counters* cnt = pl.cnt();
  launch_reset_work(cnt, st);
  launch_plan(d_parts, n_parts, inline_part, k, sched.texts_per_item, sched.pack, pl.descs.as<Desc>(),
              pl.ibase.as<uint64_t>(),
              pl.desc_cap, pl.plan(), st);
  PairArgs a;
  a.descs = pl.descs.as<Desc>();
  a.item_base = pl.ibase.as<uint64_t>();
  a.plan = pl.plan();
  a.cnt = cnt;
  a.edges = pl.edges.as<uint32_t>();
  a.edist = keep_dist ? pl.edist.as<uint8_t>() : nullptr;
  a.capacity = capacity;
  a.texts_per_item = sched.texts_per_item;
  a.k = k;
  a.count_work = sched.count_work;
  if (ev0) (void)hipEventRecord(ev0, st);
  launch_pairs(a, grid_blocks, sched.peq_lds, st);
  if (ev1) (void)hipEventRecord(ev1, st);
}

void stage_canon(Pipeline& pl, int mode, int shift, uint64_t capacity, uint32_t* d_pairs, int32_t* d_deg,
                 hipStream_t st, uint8_t* d_dist) {
  StageRange range("tcrnet:canonicalise");
  Counters* cnt = pl.cnt();
  launch_edge_keys(pl.edges.as<uint32_t>(), d_dist ? pl.edist.as<uint8_t>() : nullptr, capacity, &cnt->edges, mode,
                   shift, pl.ekeys.as<uint64_t>(), st);
  const bool ealt = radix_sort(pl.ekeys.as<uint64_t>(), pl.ekeys2.as<uint64_t>(), nullptr, nullptr, capacity,
                               &cnt->edges, 2 * shift + (d_dist ? 5 : 0), pl.tmp.as<uint32_t>(), &cnt->fault, st);
  const uint64_t* sk = ealt ? pl.ekeys2.as<uint64_t>() : pl.ekeys.as<uint64_t>();
  launch_unpack(sk, capacity, &cnt->edges, mode, shift, d_pairs, d_deg, d_dist, st);
}

void pipeline_enqueue(Pipeline& pl, const PipeParams& pp, int device, hipStream_t st, hipEvent_t ev0,
                      hipEvent_t ev1) {
  const uint32_t n = pp.n;
  launch_reset_counters(pl.cnt(), st);
  if (pp.d_deg) launch_fill_u32(reinterpret_cast<uint32_t*>(pp.d_deg), n, 0u, st);
  if (n == 0) return;
  // a1-a2
  stage_prepare(pl, pp.d_data, pp.d_off, n, pp.d_segoff, pp.n_seg, pp.id_base, 0u, SetOut{}, st);
  // a3-a6: one self part over the sorted set
  PlanPart part{};
  part.a.srec = pl.srec.as<SeqRec>();
  part.a.speq = pl.speq.as<PeqRec>();
  part.a.off = pl.off.as<uint32_t>();
  part.a.n_seg = pp.n_seg;
  part.cross = 0;
  stage_pairs(pl, nullptr, 1, part, pp.k, pp.sched, pp.capacity, pair_grid_blocks(device, pp.sched.waves_per_simd),
              st, ev0, ev1, pp.d_dist != nullptr);
  // a7-a8
  stage_canon(pl, 0, (int)bits_for(n), pp.capacity, pp.d_pairs, pp.d_deg, st, pp.d_dist);
}

hipError_t pipeline_meta(const Pipeline& pl, Meta* host_meta, hipStream_t st) {
  // the plan header follows the counters on the device as in Meta: one copy
  static_assert(offsetof(Meta, plan) == sizeof(Counters), "Meta mirrors the device layout");
  hipError_t e = hipMemcpyAsync(host_meta, pl.cnt(), sizeof(Counters) + sizeof(Plan), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

}  // namespace tcr
