// Served form: a resident, length-bucketed repertoire on the device that
// answers query batches and absorbs insert batches, with continuous batching.
//
// Repertoire versions.  The repertoire is a list of immutable segments: the
// initial set (sorted into length buckets) plus one segment per admitted
// insert.  A request is admitted in FIFO order; at admission it takes a
// snapshot (the current segment list, shared ownership) and a sequence
// number, and an insert appends its own segment for every later admission to
// see.  When the list grows past kMaxDeltas extra segments, they are merged
// (re-sorted on the device, on a stream of its own): the insert segments
// among themselves, or, once they reach an eighth of the base, everything
// into a new base.  A merged segment replaces its inputs for later admissions
// once its work has finished; older snapshots keep their segments alive until
// their requests finish.
//
// Continuous batching.  kSlots-many requests are on the device at once, each
// on its own stream (default priority) with its own pipeline buffers;
// admission also needs room in the device-memory budget.  A scheduler thread
// admits requests as slots and budget free up, and advances each in-flight
// request through two host checkpoints: (1) after the pair kernel, read the
// edge count (re-run with a larger buffer on overflow), (2) after the result
// copies, hand the result over.  A request reads a segment only after the
// event recorded when that segment was written.
#define TCRNET_BUILDING 1
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "api_internal.h"

using namespace tcr;
using Clock = std::chrono::steady_clock;

struct tcrnet_result {
  std::vector<uint32_t> pairs;
  std::vector<int32_t> counts;
  tcrnet_result_info info{};
};

namespace {

constexpr uint32_t kMaxDeltas = 4;       // segments after the base before a merge
constexpr uint32_t kDegHeadroom = 1u << 22;  // inserted nodes the degree array holds
// Requests this large (and a threshold this high) find every buffer of their
// slot already allocated: device and pinned-host frees synchronise the whole
// device, so the serving loop must not grow buffers under load.
constexpr uint32_t kReserveSeqs = 4096;
constexpr int kReserveK = 2;
// Requests on the device at once: one per hardware queue of the HIP runtime
// (four by default).  With more slots than queues two requests share a queue,
// and a small request's kernels wait behind a large one's: at half of
// saturation, 8 slots gave a p99 of 1.99 ms, 4 slots 1.79 ms (at 11% less
// saturation throughput), 2 slots 1.62 ms (31% less).
constexpr uint32_t kDefaultSlots = 4;

struct Segment {
  uint32_t n = 0;
  uint32_t hcount[33] = {0};  // host copy of the length histogram (sizing only)
  DevBuf srec, speq, off;  // off: 65 entries (one segment)
  hipEvent_t ready = nullptr;
  Segment() { (void)hipEventCreateWithFlags(&ready, hipEventDisableTiming); }
  ~Segment() {
    if (ready) (void)hipEventDestroy(ready);
  }
  hipError_t alloc(uint32_t count) {
    n = count;
    hipError_t e;
    if ((e = srec.ensure(sorted_rec_bytes(count ? count : 1))) != hipSuccess) return e;
    if ((e = speq.ensure((uint64_t)(count ? count : 1) * sizeof(PeqRec))) != hipSuccess) return e;
    return off.ensure(65 * 4);
  }
  SetRef ref() const {
    SetRef r{};
    r.srec = srec.as<SeqRec>();
    r.speq = speq.as<PeqRec>();
    r.off = off.as<uint32_t>();
    r.n_seg = 1;
    return r;
  }
};
using SegPtr = std::shared_ptr<Segment>;

// Segments no request or snapshot uses any more keep their device buffers
// here for reuse: freeing them would synchronise the device mid-serving.  A
// segment returns here when its last owner drops it, which happens only
// after every request that read it has finished on the device (a request
// failing with work in flight first waits for its stream).
struct SegPool {
  std::mutex mu;
  std::vector<std::unique_ptr<Segment>> free;
};
using PoolPtr = std::shared_ptr<SegPool>;

// A segment for `count` sequences: the smallest pooled one that holds them,
// else a new one (sized with room to grow: merged bases grow with inserts).
hipError_t take_segment(const PoolPtr& pool, uint32_t count, uint32_t headroom_pct, SegPtr* out) {
  std::unique_ptr<Segment> got;
  {
    std::lock_guard<std::mutex> g(pool->mu);
    const uint64_t need_rec = sorted_rec_bytes(count ? count : 1);
    size_t best = pool->free.size();
    for (size_t i = 0; i < pool->free.size(); ++i) {
      const Segment& c = *pool->free[i];
      if (c.srec.cap >= need_rec && c.speq.cap >= (uint64_t)(count ? count : 1) * sizeof(PeqRec) &&
          (best == pool->free.size() || c.srec.cap < pool->free[best]->srec.cap))
        best = i;
    }
    if (best < pool->free.size()) {
      got = std::move(pool->free[best]);
      pool->free.erase(pool->free.begin() + (long)best);
    }
  }
  if (!got) got.reset(new Segment());
  const uint32_t grow = count + (uint32_t)((uint64_t)count * headroom_pct / 100);
  hipError_t e = got->alloc(grow);
  if (e == hipSuccess) e = got->alloc(count);
  memset(got->hcount, 0, sizeof got->hcount);
  if (e != hipSuccess) return e;
  PoolPtr keep = pool;
  *out = SegPtr(got.release(), [keep](Segment* sp) {
    std::lock_guard<std::mutex> g(keep->mu);
    keep->free.emplace_back(sp);
  });
  return hipSuccess;
}

struct Request {
  uint64_t ticket = 0;
  std::vector<char> data;
  std::vector<uint64_t> off;  // rebased to 0
  uint32_t m = 0;
  uint32_t hcount[33] = {0};  // length histogram of the batch (sizing only)
  int k = 1;
  bool insert = false;
  Clock::time_point t_submit, t_admit;
  double admit_ms = 0.0;
  // admission
  uint64_t seqno = 0;
  std::vector<SegPtr> snap;
  uint32_t n_snap = 0;
  SegPtr new_seg;
  bool published = false;  // insert: its segment is part of the repertoire
  uint64_t bytes = 0;
  // outcome
  bool done = false;
  bool taken = false;
  int32_t status = TCRNET_OK;
  std::string err;
  tcrnet_result* res = nullptr;
};

struct Slot {
  hipStream_t st = nullptr;
  Pipeline pl;
  DevBuf d_data, d_off, d_parts, d_pairs, d_counts;
  Pinned h_data, h_off, h_parts, h_meta, h_pairs, h_counts;
  hipEvent_t ev_meta = nullptr, ev_done = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  Request* req = nullptr;
  int phase = 0;  // 0 idle, 1 waiting for counters, 2 waiting for results
  uint32_t grid = 0;
  uint64_t capacity = 0;
  uint32_t n_parts = 0;
  int attempts = 0;
};

}  // namespace

struct tcrnet_index {
  tcrnet_ctx* ctx = nullptr;
  int device = 0;
  int k_index = 1;
  std::atomic<uint32_t> n_total{0};
  uint64_t n_promised = 0;  // resident sequences once every accepted insert is in (under mu)
  uint32_t deg_cap = 0;
  DevBuf deg;
  PoolPtr pool = std::make_shared<SegPool>();  // declared before every SegPtr holder
  std::vector<SegPtr> segs;
  std::vector<std::unique_ptr<Slot>> slots;
  uint64_t budget = 0, used = 0;
  Sched sched;
  uint32_t grid = 0;
  // merge machinery
  hipStream_t merge_st = nullptr;
  Pipeline merge_pl;
  DevBuf merge_rec;
  // a merged segment still being built on merge_st: it replaces segs[merge_lo,
  // merge_hi) once its work is done (until then admissions keep
  // snapshotting the unmerged list)
  SegPtr merging;
  size_t merge_lo = 0, merge_hi = 0;
  // request queue (guarded by mu)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_ticket = 1, next_seqno = 1;
  bool stop = false;
  // An insert whose segment was published but whose edges or degrees were
  // not (a failure after admission), or a failed merge, leaves the resident
  // network inconsistent: the index then fails every request admitted after
  // that point and every later call (TCRNET_ESTATE).
  uint64_t failed_seqno = 0;  // 0: healthy
  std::string failed_msg;
  uint32_t inflight = 0;
  std::thread worker;
  std::vector<int32_t> host_deg;
};

namespace {

// Residue and length checks of host input (argument validation before a
// request can change the repertoire; the kernels check again).
int32_t check_request_seqs(const tcrnet_seqs* s) {
  if (!s) return set_error(TCRNET_EINVAL, "NULL sequence set");
  if (s->n && (!s->offsets || !s->data)) return set_error(TCRNET_EINVAL, "NULL data or offsets");
  if (s->n > TCRNET_MAX_SEQS) return set_error(TCRNET_EINVAL, "more than 2^28 sequences");
  static const char kAlpha[] = "ARNDCQEGHILKMFPSTWYV";
  bool ok[256] = {false};
  for (const char* a = kAlpha; *a; ++a) ok[(unsigned char)*a] = true;
  for (uint32_t i = 0; i < s->n; ++i) {
    if (s->offsets[i + 1] < s->offsets[i] || s->offsets[i + 1] - s->offsets[i] == 0 ||
        s->offsets[i + 1] - s->offsets[i] > TCRNET_MAX_LEN)
      return set_error(TCRNET_EINVAL, "sequence %u: length must be 1..32", i);
    for (uint64_t q = s->offsets[i]; q < s->offsets[i + 1]; ++q)
      if (!ok[(unsigned char)s->data[q]])
        return set_error(TCRNET_EINVAL, "sequence %u: residue outside the 20-letter amino-acid alphabet", i);
  }
  return TCRNET_OK;
}

uint64_t request_bytes(uint32_t m, uint64_t capacity, uint32_t n_parts) {
  return (uint64_t)m * sizeof(SeqRec) + sorted_rec_bytes(m) + (uint64_t)m * (sizeof(PeqRec) + 40 + 64) +
         capacity * 40 +
         (uint64_t)n_parts * 160 * sizeof(Desc) + (1u << 16);
}

// Work items of a request against its snapshot, estimated from length
// histograms (sizes the persistent grid; the plan on the device is exact).
uint64_t estimate_items(const Request* r, uint32_t T) {
  uint64_t items = 0;
  auto rect = [&](uint64_t a, uint64_t b) {
    if (a && b) items += ((a + 63) / 64) * ((b + T - 1) / T);
  };
  for (const SegPtr& seg : r->snap)
    for (int L = 1; L <= 32; ++L)
      for (int d = -r->k; d <= r->k; ++d) {
        const int L2 = L + d;
        if (L2 >= 1 && L2 <= 32) rect(r->hcount[L], seg->hcount[L2]);
      }
  if (r->insert)
    for (int L = 1; L <= 32; ++L)
      for (int d = 0; d <= r->k && L + d <= 32; ++d) rect(r->hcount[L + d], r->hcount[L]);
  return items;
}

// Completion of r (held by slot s, or never admitted when s is NULL).
void finish(tcrnet_index* idx, Slot* s, Request* r) {
  r->snap.clear();
  std::lock_guard<std::mutex> g(idx->mu);
  if (s) {
    s->req = nullptr;
    s->phase = 0;
    idx->used -= r->bytes;
    idx->inflight--;
  }
  r->done = true;
  idx->cv_done.notify_all();
}

int32_t status_of(hipError_t e) { return e == hipErrorOutOfMemory ? TCRNET_ENOMEM : TCRNET_EDEVICE; }

// Mark the index failed from admission `seqno` on (under mu).
void mark_failed_locked(tcrnet_index* idx, uint64_t seqno, const std::string& why) {
  if (idx->failed_seqno == 0 || seqno < idx->failed_seqno) {
    idx->failed_seqno = seqno ? seqno : 1;
    idx->failed_msg = why;
  }
}

void fail_request(tcrnet_index* idx, Slot* s, Request* r, int32_t status, const std::string& msg) {
  // work already on the slot's stream may still read the snapshot's
  // segments, which go back to the pool once the request lets go of them
  if (s) (void)hipStreamSynchronize(s->st);
  if (r->insert && r->published) {
    std::lock_guard<std::mutex> g(idx->mu);
    mark_failed_locked(idx, r->seqno, "insert (admission " + std::to_string(r->seqno) + ") failed: " + msg);
  }
  r->status = status;
  r->err = msg;
  finish(idx, s, r);
}

// A request admitted after the index failed sees an inconsistent repertoire.
bool after_failure(tcrnet_index* idx, const Request* r, std::string* why) {
  std::lock_guard<std::mutex> g(idx->mu);
  if (idx->failed_seqno == 0 || r->seqno < idx->failed_seqno) return false;
  *why = "index failed: " + idx->failed_msg;
  return true;
}

// Stage 2+3 of a request on its slot: plan the parts, pair kernel, canonical
// pairs, then the counters to the host.
hipError_t enqueue_pairs(tcrnet_index* idx, Slot* s) {
  Request* r = s->req;
  hipError_t e;
  const uint32_t max_desc = (s->n_parts + 1) * plan_max_desc_cross(r->k) +
                            (r->insert ? plan_max_desc_self(1, r->k, idx->sched.texts_per_item, r->m) : 0);
  if ((e = pipeline_reserve(s->pl, r->m, 1, r->k, idx->sched.texts_per_item, s->capacity, max_desc)) != hipSuccess)
    return e;
  if ((e = s->d_pairs.ensure(s->capacity * 8)) != hipSuccess) return e;
  if ((e = s->d_counts.ensure((uint64_t)(r->m ? r->m : 1) * 4)) != hipSuccess) return e;
  if ((e = s->h_meta.ensure(sizeof(Meta))) != hipSuccess) return e;
  stage_pairs(s->pl, s->d_parts.as<PlanPart>(), s->n_parts, PlanPart{}, r->k, idx->sched, s->capacity, s->grid,
              s->st, nullptr, nullptr);
  launch_fill_u32(s->d_counts.as<uint32_t>(), r->m, 0u, s->st);
  const uint32_t ids = r->n_snap + (r->insert ? r->m : 0);
  const int shift = (int)bits_for(ids > r->m ? ids : r->m);
  stage_canon(s->pl, r->insert ? 0 : 1, shift, s->capacity, s->d_pairs.as<uint32_t>(),
              r->insert ? nullptr : s->d_counts.as<int32_t>(), s->st);
  // counters and plan header are adjacent on the device as in Meta: one copy
  if ((e = hipMemcpyAsync(s->h_meta.as<Meta>(), s->pl.cnt(), sizeof(Counters) + sizeof(Plan),
                          hipMemcpyDeviceToHost, s->st)) != hipSuccess)
    return e;
  (void)hipEventRecord(s->ev_meta, s->st);
  s->phase = 1;
  s->attempts++;
  return hipSuccess;
}

// Allocate a slot's buffers for requests of up to kReserveSeqs sequences at
// k <= kReserveK against a fully fragmented snapshot.
hipError_t reserve_slot(tcrnet_index* idx, Slot* s) {
  hipError_t e;
  const uint32_t m = kReserveSeqs;
  const uint64_t cap = (uint64_t)m * 16;
  const uint32_t n_parts = 2 * kMaxDeltas + 3;  // deltas keep coming while a merge is built
  const uint32_t max_desc = (n_parts + 1) * plan_max_desc_cross(kReserveK) +
                            plan_max_desc_self(1, kReserveK, idx->sched.texts_per_item, m);
  if ((e = pipeline_reserve(s->pl, m, 1, kReserveK, idx->sched.texts_per_item, cap, max_desc)) != hipSuccess)
    return e;
  if ((e = s->d_pairs.ensure(cap * 8)) != hipSuccess || (e = s->d_counts.ensure((uint64_t)m * 4)) != hipSuccess ||
      (e = s->d_data.ensure((uint64_t)m * TCRNET_MAX_LEN)) != hipSuccess ||
      (e = s->d_off.ensure((uint64_t)(m + 1) * 8)) != hipSuccess ||
      (e = s->d_parts.ensure((uint64_t)n_parts * sizeof(PlanPart))) != hipSuccess)
    return e;
  if ((e = s->h_data.ensure((uint64_t)m * TCRNET_MAX_LEN)) != hipSuccess ||
      (e = s->h_off.ensure((uint64_t)(m + 1) * 8)) != hipSuccess ||
      (e = s->h_parts.ensure((uint64_t)n_parts * sizeof(PlanPart))) != hipSuccess ||
      (e = s->h_meta.ensure(sizeof(Meta))) != hipSuccess || (e = s->h_pairs.ensure(cap * 8 + 8)) != hipSuccess ||
      (e = s->h_counts.ensure((uint64_t)m * 4 + 4)) != hipSuccess)
    return e;
  return hipSuccess;
}

// Admission of r onto slot s: snapshot, insert segment, stage 1, parts.
hipError_t admit(tcrnet_index* idx, Slot* s, Request* r) {
  hipError_t e;
  r->t_admit = Clock::now();
  r->seqno = idx->next_seqno++;
  r->snap = idx->segs;
  r->n_snap = idx->n_total;
  s->req = r;
  s->attempts = 0;
  s->capacity = std::max<uint64_t>(4096, (uint64_t)r->m * 16);
  {
    // one item per wave (4 per block) in the first round; never more than
    // the full persistent grid (an uncapped grid of short-lived blocks was
    // slower: 1.03 -> 1.26 ms for 4,096 queries at k = 2 against 800,000)
    const uint64_t want = (estimate_items(r, idx->sched.texts_per_item) + 3) / 4;
    s->grid = (uint32_t)std::min<uint64_t>(idx->grid, std::max<uint64_t>(16, want));
  }
  hipStream_t st = s->st;
  (void)hipEventRecord(s->ev_t0, st);
  const uint32_t n_parts_max = (uint32_t)r->snap.size() + 1;
  const uint32_t max_desc = n_parts_max * plan_max_desc_cross(r->k) +
                            (r->insert ? plan_max_desc_self(1, r->k, idx->sched.texts_per_item, r->m) : 0);
  if ((e = pipeline_reserve(s->pl, r->m, 1, r->k, idx->sched.texts_per_item, s->capacity, max_desc)) != hipSuccess)
    return e;
  launch_reset_counters(s->pl.cnt(), st);
  SetRef qref{};
  if (r->m) {
    const uint64_t bytes = r->off[r->m];
    if ((e = s->h_data.ensure(bytes ? bytes : 1)) != hipSuccess) return e;
    if ((e = s->h_off.ensure((uint64_t)(r->m + 1) * 8)) != hipSuccess) return e;
    if ((e = s->d_data.ensure(bytes ? bytes : 1)) != hipSuccess) return e;
    if ((e = s->d_off.ensure((uint64_t)(r->m + 1) * 8)) != hipSuccess) return e;
    memcpy(s->h_data.p, r->data.data(), bytes);
    memcpy(s->h_off.p, r->off.data(), (uint64_t)(r->m + 1) * 8);
    if ((e = hipMemcpyAsync(s->d_data.p, s->h_data.p, bytes, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(s->d_off.p, s->h_off.p, (uint64_t)(r->m + 1) * 8, hipMemcpyHostToDevice, st)) !=
        hipSuccess)
      return e;
    SetOut out;
    if (r->insert) {
      if ((e = take_segment(idx->pool, r->m, 0, &r->new_seg)) != hipSuccess) return e;
      out.srec = r->new_seg->srec.as<SeqRec>();
      out.speq = r->new_seg->speq.as<PeqRec>();
      out.off = r->new_seg->off.as<uint32_t>();
    }
    stage_prepare(s->pl, s->d_data.as<char>(), s->d_off.as<uint64_t>(), r->m, nullptr, 1,
                  r->insert ? r->n_snap : 0u, r->insert ? 0u : kQueryTag, out, st);
    if (r->insert) {
      memcpy(r->new_seg->hcount, r->hcount, sizeof r->hcount);
      (void)hipEventRecord(r->new_seg->ready, st);
      qref = r->new_seg->ref();
      idx->segs.push_back(r->new_seg);
      idx->n_total += r->m;
      r->published = true;
    } else {
      qref.srec = s->pl.srec.as<SeqRec>();
      qref.speq = s->pl.speq.as<PeqRec>();
      qref.off = s->pl.off.as<uint32_t>();
      qref.n_seg = 1;
    }
  }
  // parts: the request's set against every segment of its snapshot, and an
  // insert against itself
  const uint32_t n_parts = (uint32_t)r->snap.size() + (r->insert ? 1u : 0u);
  if ((e = s->h_parts.ensure((uint64_t)(n_parts ? n_parts : 1) * sizeof(PlanPart))) != hipSuccess) return e;
  if ((e = s->d_parts.ensure((uint64_t)(n_parts ? n_parts : 1) * sizeof(PlanPart))) != hipSuccess) return e;
  PlanPart* hp = s->h_parts.as<PlanPart>();
  uint32_t np = 0;
  if (r->m) {
    for (const SegPtr& seg : r->snap) {
      (void)hipStreamWaitEvent(st, seg->ready, 0);
      PlanPart p{};
      p.a = seg->ref();
      p.b = qref;
      p.cross = 1;
      hp[np++] = p;
    }
    if (r->insert) {
      PlanPart p{};
      p.a = qref;
      p.cross = 0;
      hp[np++] = p;
    }
  }
  s->n_parts = np;
  if (np && (e = hipMemcpyAsync(s->d_parts.p, hp, np * sizeof(PlanPart), hipMemcpyHostToDevice, st)) != hipSuccess)
    return e;
  return enqueue_pairs(idx, s);
}

// Start merging segments on the merge stream, tiered: the insert segments
// after the base are merged among themselves (a cost proportional to their
// size) until together they reach an eighth of the base; then everything is
// merged into a new base.  The result is published by publish_merge once its
// work has finished, so no admission ever waits for a merge.
hipError_t merge_segments(tcrnet_index* idx) {
  hipError_t e;
  uint64_t rest = 0;
  for (size_t i = 1; i < idx->segs.size(); ++i) rest += idx->segs[i]->n;
  const size_t lo = 8 * rest < (uint64_t)idx->segs[0]->n ? 1 : 0, hi = idx->segs.size();
  uint32_t n = 0;
  for (size_t i = lo; i < hi; ++i) n += idx->segs[i]->n;
  SegPtr merged;
  if ((e = take_segment(idx->pool, n, lo == 0 ? 25 : 100, &merged)) != hipSuccess) return e;
  for (size_t i = lo; i < hi; ++i)
    for (int L = 0; L <= 32; ++L) merged->hcount[L] += idx->segs[i]->hcount[L];
  // (reserved with room for growth when the index was made)
  if ((e = idx->merge_rec.ensure((uint64_t)(n ? n : 1) * sizeof(SeqRec))) != hipSuccess) return e;
  if ((e = pipeline_reserve(idx->merge_pl, n, 1, 1, idx->sched.texts_per_item, 1, 1)) != hipSuccess) return e;
  uint64_t pos = 0;
  for (size_t i = lo; i < hi; ++i) {
    const SegPtr& seg = idx->segs[i];
    (void)hipStreamWaitEvent(idx->merge_st, seg->ready, 0);
    if (seg->n &&
        (e = hipMemcpyAsync(idx->merge_rec.as<SeqRec>() + pos, seg->srec.p, (uint64_t)seg->n * sizeof(SeqRec),
                            hipMemcpyDeviceToDevice, idx->merge_st)) != hipSuccess) {
      (void)hipStreamSynchronize(idx->merge_st);  // before `merged` goes back to the pool
      return e;
    }
    pos += seg->n;
  }
  SetOut out;
  out.srec = merged->srec.as<SeqRec>();
  out.speq = merged->speq.as<PeqRec>();
  out.off = merged->off.as<uint32_t>();
  stage_prepare_records(idx->merge_pl, idx->merge_rec.as<SeqRec>(), n, out, idx->merge_st);
  (void)hipEventRecord(merged->ready, idx->merge_st);
  idx->merging = merged;
  idx->merge_lo = lo;
  idx->merge_hi = hi;
  return hipSuccess;
}

// Publish a finished merge: the merged segment replaces the segments it
// covers (snapshots of earlier admissions keep those alive); inserts
// admitted while it was built stay behind it.
void publish_merge(tcrnet_index* idx) {
  if (!idx->merging || hipEventQuery(idx->merging->ready) != hipSuccess) return;
  std::vector<SegPtr> segs(idx->segs.begin(), idx->segs.begin() + (long)idx->merge_lo);
  segs.push_back(idx->merging);
  segs.insert(segs.end(), idx->segs.begin() + (long)idx->merge_hi, idx->segs.end());
  idx->segs.swap(segs);
  idx->merging.reset();
  idx->merge_lo = idx->merge_hi = 0;
}

// Checkpoint 1: counters are on the host.
void on_meta(tcrnet_index* idx, Slot* s) {
  Request* r = s->req;
  std::string why;
  if (after_failure(idx, r, &why)) {
    fail_request(idx, s, r, TCRNET_ESTATE, why);
    return;
  }
  const Meta m = *s->h_meta.as<Meta>();
  if (m.cnt.fault) {
    fail_request(idx, s, r, TCRNET_EDEVICE, "device sort stalled (internal)");
    return;
  }
  if (m.cnt.err != kNoError) {
    fail_request(idx, s, r, TCRNET_EINVAL, input_error_message(m.cnt.err));
    return;
  }
  if (m.plan.pad) {
    fail_request(idx, s, r, TCRNET_EDEVICE, "work plan overflow (internal)");
    return;
  }
  const uint64_t E = m.cnt.edges;
  hipError_t e;
  if (E > s->capacity) {
    if (s->attempts >= 2) {
      fail_request(idx, s, r, TCRNET_EDEVICE, "edge count changed between runs (internal)");
      return;
    }
    s->capacity = E + E / 16 + 1024;
    {
      std::lock_guard<std::mutex> g(idx->mu);
      idx->used -= r->bytes;
      r->bytes = request_bytes(r->m, s->capacity, s->n_parts);
      idx->used += r->bytes;
    }
    if ((e = enqueue_pairs(idx, s)) != hipSuccess) fail_request(idx, s, r, status_of(e), hipGetErrorString(e));
    return;
  }
  if (r->insert)
    launch_insert_degrees(s->d_pairs.as<uint32_t>(), &s->pl.cnt()->edges, s->capacity, r->n_snap,
                          s->d_counts.as<int32_t>(), idx->deg.as<int32_t>(), s->st);
  if ((e = s->h_pairs.ensure(E * 8 + 8)) != hipSuccess || (e = s->h_counts.ensure((uint64_t)r->m * 4 + 4)) != hipSuccess) {
    fail_request(idx, s, r, TCRNET_ENOMEM, hipGetErrorString(e));
    return;
  }
  if (E) (void)hipMemcpyAsync(s->h_pairs.p, s->d_pairs.p, E * 8, hipMemcpyDeviceToHost, s->st);
  if (r->m) (void)hipMemcpyAsync(s->h_counts.p, s->d_counts.p, (uint64_t)r->m * 4, hipMemcpyDeviceToHost, s->st);
  (void)hipEventRecord(s->ev_t1, s->st);
  (void)hipEventRecord(s->ev_done, s->st);
  s->phase = 2;
  r->res = new tcrnet_result();
  r->res->pairs.resize(2 * E);
}

// Checkpoint 2: results are on the host.
void on_done(tcrnet_index* idx, Slot* s) {
  Request* r = s->req;
  tcrnet_result* res = r->res;
  std::string why;
  if (after_failure(idx, r, &why)) {
    delete res;
    r->res = nullptr;
    fail_request(idx, s, r, TCRNET_ESTATE, why);
    return;
  }
  if (!res->pairs.empty()) memcpy(res->pairs.data(), s->h_pairs.p, res->pairs.size() * 4);
  res->counts.assign(s->h_counts.as<int32_t>(), s->h_counts.as<int32_t>() + r->m);
  float dev_ms = 0.f;
  (void)hipEventElapsedTime(&dev_ms, s->ev_t0, s->ev_t1);
  res->info.seqno = r->seqno;
  res->info.snapshot_size = r->n_snap;
  res->info.is_insert = r->insert ? 1 : 0;
  res->info.device_ms = dev_ms;
  res->info.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
  res->info.queue_ms = std::chrono::duration<double, std::milli>(r->t_admit - r->t_submit).count();
  res->info.admit_ms = r->admit_ms;
  res->info.attempts = (uint32_t)s->attempts;
  res->info.parts = s->n_parts;
  finish(idx, s, r);
}

void worker_loop(tcrnet_index* idx) {
  (void)hipSetDevice(idx->device);
  for (;;) {
    bool progressed = false;
    // admissions, in FIFO order
    for (;;) {
      Request* r = nullptr;
      Slot* free_slot = nullptr;
      {
        std::unique_lock<std::mutex> lk(idx->mu);
        if (idx->pending.empty()) break;
        for (auto& sl : idx->slots)
          if (!sl->req) {
            free_slot = sl.get();
            break;
          }
        if (!free_slot) break;
        r = idx->pending.front();
        if (idx->failed_seqno) {
          idx->pending.pop_front();
          const std::string why = "index failed: " + idx->failed_msg;
          lk.unlock();
          fail_request(idx, nullptr, r, TCRNET_ESTATE, why);
          progressed = true;
          continue;
        }
        const uint32_t n_parts = (uint32_t)idx->segs.size() + 1;
        const uint64_t need = request_bytes(r->m, std::max<uint64_t>(4096, (uint64_t)r->m * 16), n_parts);
        if (need > idx->budget) {
          idx->pending.pop_front();
          lk.unlock();
          fail_request(idx, nullptr, r, TCRNET_ENOMEM, "request exceeds the serving memory budget");
          progressed = true;
          continue;
        }
        if (idx->used + need > idx->budget) break;
        if (r->insert && (uint64_t)idx->n_total + r->m > idx->deg_cap) {
          idx->pending.pop_front();
          lk.unlock();
          fail_request(idx, nullptr, r, TCRNET_ENOMEM, "insert exceeds the index's node capacity");
          progressed = true;
          continue;
        }
        idx->pending.pop_front();
        r->bytes = need;
        idx->used += need;
        idx->inflight++;
      }
      hipError_t e = admit(idx, free_slot, r);
      r->admit_ms = std::chrono::duration<double, std::milli>(Clock::now() - r->t_admit).count();
      if (e != hipSuccess) fail_request(idx, free_slot, r, status_of(e), hipGetErrorString(e));
      // a failed merge changes nothing (the unmerged list stays current);
      // it is tried again after the next admission
      if (idx->segs.size() > 1 + kMaxDeltas && !idx->merging) (void)merge_segments(idx);
      progressed = true;
    }
    // in-flight requests
    for (auto& sl : idx->slots) {
      Slot* s = sl.get();
      if (s->phase == 0) continue;
      const hipError_t q = hipEventQuery(s->phase == 1 ? s->ev_meta : s->ev_done);
      if (q == hipErrorNotReady) continue;
      progressed = true;
      if (q != hipSuccess) {
        fail_request(idx, s, s->req, TCRNET_EDEVICE, hipGetErrorString(q));
      } else if (s->phase == 1) {
        on_meta(idx, s);
      } else {
        on_done(idx, s);
      }
    }
    publish_merge(idx);
    if (progressed) continue;
    std::unique_lock<std::mutex> lk(idx->mu);
    if (idx->stop && idx->pending.empty() && idx->inflight == 0) break;
    if (idx->inflight > 0 || idx->merging) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    } else {
      idx->cv_work.wait_for(lk, std::chrono::milliseconds(50));
    }
  }
}

void copy_seqs(const tcrnet_seqs* q, Request* r) {
  r->m = q->n;
  r->off.resize(q->n + 1);
  if (!q->n) {
    r->off[0] = 0;
    return;
  }
  const uint64_t base = q->offsets[0];
  for (uint32_t i = 0; i <= q->n; ++i) r->off[i] = q->offsets[i] - base;
  for (uint32_t i = 0; i < q->n; ++i) r->hcount[r->off[i + 1] - r->off[i]]++;  // lengths checked: 1..32
  r->data.assign(q->data + base, q->data + q->offsets[q->n]);
}

}  // namespace

extern "C" {

int32_t tcrnet_index_create(tcrnet_ctx* ctx, const tcrnet_seqs* seqs, int32_t k_index, tcrnet_index** out) {
  if (!out) return set_error(TCRNET_EINVAL, "NULL output pointer");
  *out = nullptr;
  if (!ctx) return set_error(TCRNET_EINVAL, "NULL context");
  int32_t rc;
  if ((rc = check_k(k_index)) || (rc = check_request_seqs(seqs))) return rc;
  (void)hipSetDevice(ctx->device);
  std::unique_ptr<tcrnet_index> idx(new tcrnet_index());
  idx->ctx = ctx;
  idx->device = ctx->device;
  idx->k_index = k_index;
  const uint32_t n = seqs->n;
  idx->deg_cap = n + kDegHeadroom;
  hipError_t e;
  if ((e = idx->deg.ensure((uint64_t)idx->deg_cap * 4)) != hipSuccess) return hip_error(e, "degree array");
  launch_fill_u32(idx->deg.as<uint32_t>(), idx->deg_cap, 0u, ctx->stream);
  // base segment: the plain build at k_index gives the sorted set and degrees
  SegPtr base;
  if ((e = take_segment(idx->pool, n, 0, &base)) != hipSuccess) return hip_error(e, "segment allocation");
  for (uint32_t i = 0; i < n; ++i) base->hcount[seqs->offsets[i + 1] - seqs->offsets[i]]++;
  if (n) {
    const uint64_t b0 = seqs->offsets[0], bytes = seqs->offsets[n] - b0;
    std::vector<uint64_t> off(n + 1);
    for (uint32_t i = 0; i <= n; ++i) off[i] = seqs->offsets[i] - b0;
    if ((e = ctx->in_data.ensure(bytes)) != hipSuccess || (e = ctx->in_off.ensure((n + 1) * 8)) != hipSuccess)
      return hip_error(e, "input allocation");
    (void)hipMemcpyAsync(ctx->in_data.p, seqs->data + b0, bytes, hipMemcpyHostToDevice, ctx->stream);
    (void)hipMemcpyAsync(ctx->in_off.p, off.data(), (n + 1) * 8, hipMemcpyHostToDevice, ctx->stream);
    PipeParams pp;
    pp.d_data = ctx->in_data.as<char>();
    pp.d_off = ctx->in_off.as<uint64_t>();
    pp.n = n;
    pp.k = k_index;
    pp.capacity = ctx->opts.edge_capacity ? ctx->opts.edge_capacity : std::max<uint64_t>(65536, 4ull * n);
    pp.d_deg = idx->deg.as<int32_t>();
    uint64_t E = 0;
    tcrnet_build_info info{};
    rc = run_pipeline(ctx, ctx->pipe, pp, ctx->stream, true, &ctx->out_pairs, &E, &info);
    if (rc) return rc;
    // the sorted records and their walk arrays, which follow them
    (void)hipMemcpyAsync(base->srec.p, ctx->pipe.srec.p, sorted_rec_bytes(n), hipMemcpyDeviceToDevice,
                         ctx->stream);
    (void)hipMemcpyAsync(base->speq.p, ctx->pipe.speq.p, (uint64_t)n * sizeof(PeqRec), hipMemcpyDeviceToDevice,
                         ctx->stream);
    (void)hipMemcpyAsync(base->off.p, ctx->pipe.off.p, 65 * 4, hipMemcpyDeviceToDevice, ctx->stream);
  } else {
    launch_fill_u32(base->off.as<uint32_t>(), 65, 0u, ctx->stream);
  }
  (void)hipEventRecord(base->ready, ctx->stream);
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_error(e, "index build");
  idx->segs.push_back(base);
  idx->n_total = n;
  idx->n_promised = n;
  // serving schedule and budget
  idx->sched = pick_sched(ctx, n, k_index);
  // requests are small next to the resident set: short work items keep many
  // waves busy on each request (measured best for 1-4,096 queries against
  // 800,000 resident sequences: 3,425 queries at k = 2 in 0.854 ms at 512
  // texts per item, 0.877 at 1,024, 1.02 at 2,048)
  if (!ctx->opts.texts_per_item) idx->sched.texts_per_item = 512;
  // and such launches run mostly in their tail: pattern masks in VGPRs
  if (!(ctx->opts.flags & TCRNET_F_PEQ_LDS)) idx->sched.peq_lds = false;
  const uint32_t n_slots = ctx->opts.max_inflight ? ctx->opts.max_inflight : kDefaultSlots;
  idx->grid = pair_grid_blocks(ctx->device, idx->sched.waves_per_simd);  // upper bound per request
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  idx->budget = ctx->opts.hbm_budget ? ctx->opts.hbm_budget : free_b / 4;
  for (uint32_t i = 0; i < n_slots; ++i) {
    std::unique_ptr<Slot> s(new Slot());
    if ((e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking)) != hipSuccess) return hip_error(e, "stream");
    (void)hipEventCreateWithFlags(&s->ev_meta, hipEventDisableTiming);
    (void)hipEventCreateWithFlags(&s->ev_done, hipEventDisableTiming);
    (void)hipEventCreate(&s->ev_t0);
    (void)hipEventCreate(&s->ev_t1);
    if ((e = reserve_slot(idx.get(), s.get())) != hipSuccess) return hip_error(e, "serving slot allocation");
    idx->slots.push_back(std::move(s));
  }
  // merge scratch for the repertoire with room for a quarter more inserts,
  // and a spare segment of that size for the first full merge
  {
    SegPtr spare;
    if ((e = take_segment(idx->pool, n + n / 4 + kReserveSeqs, 0, &spare)) != hipSuccess)
      return hip_error(e, "merge workspace");
  }
  {
    const uint64_t nm = (uint64_t)n + n / 4 + kReserveSeqs;
    if ((e = idx->merge_rec.ensure(nm * sizeof(SeqRec))) != hipSuccess ||
        (e = pipeline_reserve(idx->merge_pl, nm, 1, 1, idx->sched.texts_per_item, 1, 1)) != hipSuccess)
      return hip_error(e, "merge workspace");
  }
  if ((e = hipStreamCreateWithFlags(&idx->merge_st, hipStreamNonBlocking)) != hipSuccess)
    return hip_error(e, "stream");
  tcrnet_index* raw = idx.release();
  raw->worker = std::thread(worker_loop, raw);
  *out = raw;
  return TCRNET_OK;
}

int32_t tcrnet_index_size(tcrnet_index* idx, uint32_t* n) {
  if (!idx || !n) return set_error(TCRNET_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(idx->mu);
  if (idx->failed_seqno) return set_error(TCRNET_ESTATE, "index failed: %s", idx->failed_msg.c_str());
  // admitted inserts are counted in n_total; queued ones are not yet part of it
  *n = idx->n_total;
  return TCRNET_OK;
}

int32_t tcrnet_index_degree(tcrnet_index* idx, const int32_t** degree, uint32_t* n) {
  if (!idx || !degree || !n) return set_error(TCRNET_EINVAL, "NULL argument");
  {
    std::unique_lock<std::mutex> lk(idx->mu);
    idx->cv_done.wait(lk, [&] { return idx->pending.empty() && idx->inflight == 0; });
    if (idx->failed_seqno) return set_error(TCRNET_ESTATE, "index failed: %s", idx->failed_msg.c_str());
  }
  (void)hipSetDevice(idx->device);
  const uint32_t total = idx->n_total;
  idx->host_deg.resize(total ? total : 1);
  hipError_t e = hipMemcpy(idx->host_deg.data(), idx->deg.p, (uint64_t)total * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(e, "degree copy");
  *degree = total ? idx->host_deg.data() : nullptr;
  *n = total;
  return TCRNET_OK;
}

void tcrnet_index_free(tcrnet_index* idx) {
  if (!idx) return;
  {
    std::lock_guard<std::mutex> g(idx->mu);
    idx->stop = true;
    idx->cv_work.notify_all();
  }
  if (idx->worker.joinable()) idx->worker.join();
  (void)hipSetDevice(idx->device);
  for (auto& s : idx->slots) {
    (void)hipStreamSynchronize(s->st);
    (void)hipEventDestroy(s->ev_meta);
    (void)hipEventDestroy(s->ev_done);
    (void)hipEventDestroy(s->ev_t0);
    (void)hipEventDestroy(s->ev_t1);
    (void)hipStreamDestroy(s->st);
  }
  (void)hipStreamSynchronize(idx->merge_st);
  (void)hipStreamDestroy(idx->merge_st);
  for (auto& kv : idx->reqs) {
    delete kv.second->res;
    delete kv.second;
  }
  delete idx;
}

int32_t tcrnet_submit(tcrnet_index* idx, const tcrnet_seqs* q, int32_t k, int32_t insert, uint64_t* ticket) {
  if (!idx || !ticket) return set_error(TCRNET_EINVAL, "NULL argument");
  *ticket = 0;
  int32_t rc;
  if (insert) k = idx->k_index;
  if ((rc = check_k(k)) || (rc = check_request_seqs(q))) return rc;
  Request* r = new Request();
  copy_seqs(q, r);
  r->k = k;
  r->insert = insert != 0;
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> g(idx->mu);
  if (idx->stop) {
    delete r;
    return set_error(TCRNET_ESTATE, "index is shutting down");
  }
  if (idx->failed_seqno) {
    delete r;
    return set_error(TCRNET_ESTATE, "index failed: %s", idx->failed_msg.c_str());
  }
  if (r->insert) {
    // every accepted insert will be resident: keep the total in range
    if ((uint64_t)idx->n_promised + r->m > TCRNET_MAX_SEQS) {
      delete r;
      return set_error(TCRNET_EINVAL, "insert would grow the index past 2^28 sequences");
    }
    idx->n_promised += r->m;
  }
  r->ticket = idx->next_ticket++;
  idx->reqs[r->ticket] = r;
  idx->pending.push_back(r);
  idx->cv_work.notify_all();
  *ticket = r->ticket;
  return TCRNET_OK;
}

int32_t tcrnet_wait(tcrnet_index* idx, uint64_t ticket, tcrnet_result** out) {
  if (!idx || !out) return set_error(TCRNET_EINVAL, "NULL argument");
  *out = nullptr;
  Request* r = nullptr;
  {
    std::unique_lock<std::mutex> lk(idx->mu);
    auto it = idx->reqs.find(ticket);
    if (it == idx->reqs.end()) return set_error(TCRNET_ESTATE, "unknown or already collected ticket %llu",
                                                (unsigned long long)ticket);
    r = it->second;
    idx->cv_done.wait(lk, [&] { return r->done; });
    idx->reqs.erase(it);
  }
  const int32_t status = r->status;
  if (status != TCRNET_OK) {
    std::string msg = r->err;
    delete r->res;
    delete r;
    return set_error(status, "%s", msg.c_str());
  }
  *out = r->res;
  delete r;
  return TCRNET_OK;
}

int32_t tcrnet_query(tcrnet_index* idx, const tcrnet_seqs* q, int32_t k, tcrnet_result** out) {
  if (out) *out = nullptr;
  uint64_t t = 0;
  int32_t rc = tcrnet_submit(idx, q, k, 0, &t);
  if (rc) return rc;
  return tcrnet_wait(idx, t, out);
}

int32_t tcrnet_insert(tcrnet_index* idx, const tcrnet_seqs* q, tcrnet_result** out) {
  if (out) *out = nullptr;
  uint64_t t = 0;
  int32_t rc = tcrnet_submit(idx, q, 0, 1, &t);
  if (rc) return rc;
  return tcrnet_wait(idx, t, out);
}

int32_t tcrnet_result_pairs(const tcrnet_result* r, const uint32_t** pairs, uint64_t* n) {
  if (!r || !pairs || !n) return set_error(TCRNET_EINVAL, "NULL argument");
  *pairs = r->pairs.empty() ? nullptr : r->pairs.data();
  *n = r->pairs.size() / 2;
  return TCRNET_OK;
}

int32_t tcrnet_result_counts(const tcrnet_result* r, const int32_t** counts, uint32_t* n) {
  if (!r || !counts || !n) return set_error(TCRNET_EINVAL, "NULL argument");
  *counts = r->counts.empty() ? nullptr : r->counts.data();
  *n = (uint32_t)r->counts.size();
  return TCRNET_OK;
}

int32_t tcrnet_result_info_get(const tcrnet_result* r, tcrnet_result_info* info) {
  if (!r || !info) return set_error(TCRNET_EINVAL, "NULL argument");
  *info = r->info;
  return TCRNET_OK;
}

void tcrnet_result_free(tcrnet_result* r) { delete r; }

}  // extern "C"
