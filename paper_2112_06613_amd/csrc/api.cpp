// C-ABI of libtcrnet: contexts, the plain / device / batched builds, graphs
// and the autotuner.  Serving lives in serve.cpp.
#define TCRNET_BUILDING 1
#include "api_internal.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

using namespace tcr;

namespace tcr {
const char* last_error_text();
void clear_error();
}  // namespace tcr

// Allocator whose default-insertion leaves elements uninitialised: a result
// array sized and then filled by copies on several host threads is first
// touched by those copies (no zero fill on one thread beforehand).
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
template <class T>
using ResultVec = std::vector<T, NoInitAlloc<T>>;

struct tcrnet_graph {
  uint32_t n = 0;
  ResultVec<uint32_t> pairs;
  ResultVec<int32_t> deg;
  ResultVec<uint8_t> dist;  // weighted builds only
  tcrnet_build_info info{};
};

namespace {
const char kVersion[] = "tcrnet 0.1.0 (gfx950)";
}  // namespace

namespace tcr {

int32_t check_k(int32_t k) {
  if (k < 0 || k > TCRNET_MAX_K) return set_error(TCRNET_EINVAL, "k = %d outside [0, %d]", k, TCRNET_MAX_K);
  return TCRNET_OK;
}

// Host-side argument checks that need no residue arithmetic: pointers and
// offset monotonicity (lengths themselves are validated on the device).
int32_t check_host_seqs(const tcrnet_seqs* s, const char* what) {
  if (!s) return set_error(TCRNET_EINVAL, "%s: NULL sequence set", what);
  if (s->n > TCRNET_MAX_SEQS) return set_error(TCRNET_EINVAL, "%s: more than 2^28 sequences", what);
  if (s->n && (!s->offsets || !s->data)) return set_error(TCRNET_EINVAL, "%s: NULL data or offsets", what);
  for (uint32_t i = 0; i < s->n; ++i)
    if (s->offsets[i + 1] < s->offsets[i])
      return set_error(TCRNET_EINVAL, "%s: offsets decrease at sequence %u", what, i);
  return TCRNET_OK;
}

}  // namespace tcr

namespace {

uint64_t default_capacity(const tcrnet_ctx* ctx, uint64_t n) {
  if (ctx->opts.edge_capacity) return ctx->opts.edge_capacity;
  uint64_t c = 4 * n;
  return c < 65536 ? 65536 : c;
}

}  // namespace

namespace tcr {

Sched pick_sched(const tcrnet_ctx* ctx, uint64_t n, int k, int form) {
  Sched s;
  // Pattern masks in VGPRs: the sibling loops then wait on no LDS read and
  // the walk-record prefetch is the only scalar-memory traffic in flight
  // (N = 800,000, k = 1: 1.59 ms against 1.66 with the masks in LDS; 50,000:
  // 0.207 against 0.220 ms).  The walk's registers allow six waves per SIMD,
  // so a persistent grid of six blocks per CU.  Work items shrink with the
  // launch (default_texts_per_item): its tail is then shorter (N = 50,000,
  // k = 2: 1.78 ms at 16,384 texts per item, 0.49 ms at 512).
  s.peq_lds = false;
  s.waves_per_simd = kPairWavesPerSimd;
  s.texts_per_item = default_texts_per_item(n, k);
  if (!(ctx->opts.flags & TCRNET_F_NO_AUTOTUNE)) {
    TuneKey key;
    key.form = form;
    key.size_class = (int)bits_for(n ? n : 1);
    key.k = k;
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) {
      s = it->second.sched;
      s.tuned = true;
    }
  }
  if (ctx->opts.texts_per_item) s.texts_per_item = ctx->opts.texts_per_item;
  if (ctx->opts.waves_per_simd) s.waves_per_simd = ctx->opts.waves_per_simd;
  if (ctx->opts.flags & TCRNET_F_PEQ_LDS) s.peq_lds = true;
  if (ctx->opts.flags & TCRNET_F_PEQ_VGPR) s.peq_lds = false;
  if (ctx->opts.flags & TCRNET_F_NO_PACK) s.pack = false;
  s.count_work = (ctx->opts.flags & TCRNET_F_COUNT_WORK) != 0;
  // whole waves of 64 texts per item keep triangle items non-empty
  s.texts_per_item = std::max<uint32_t>(64, (s.texts_per_item + 63) / 64 * 64);
  s.waves_per_simd = std::min<uint32_t>(8, std::max<uint32_t>(1, s.waves_per_simd));
  return s;
}

// Work counts of the pair kernel's counting variant into a build's info.
void note_work(const Sched& sched, const Meta& m, tcrnet_build_info* inf) {
  if (!sched.count_work) return;
  inf->work_counted = 1;
  inf->visited_texts = m.cnt.visits;
  inf->wave_steps = m.cnt.steps;
  inf->wave_steps_packed = m.cnt.steps_packed;
}

// Run one pipeline on device-resident input into (d_pairs, d_deg) with
// capacity `cap`, re-running with the exact capacity once if the edge buffer
// overflowed (when grow_ok).  Returns E in *E.
int32_t run_pipeline(tcrnet_ctx* ctx, Pipeline& pl, PipeParams pp, hipStream_t st, bool grow_ok,
                     DevBuf* pairs_buf, uint64_t* E, tcrnet_build_info* info, DevBuf* dist_buf) {
  Sched sched = pick_sched(ctx, pp.n, pp.k);
  pp.sched = sched;
  tcrnet_build_info inf{};
  inf.texts_per_item = sched.texts_per_item;
  inf.waves_per_simd = sched.waves_per_simd;
  inf.peq_lds = sched.peq_lds ? 1 : 0;
  inf.pack = sched.pack ? 1 : 0;
  inf.tuned = sched.tuned ? 1 : 0;
  if (pp.n == 0) {
    *E = 0;
    if (info) *info = inf;
    return TCRNET_OK;
  }
  for (int attempt = 0; attempt < 2; ++attempt) {
    hipError_t e = pipeline_reserve(pl, pp.n, pp.n_seg, pp.k, sched.texts_per_item, pp.capacity);
    if (e != hipSuccess) return hip_error(e, "workspace allocation");
    if (pairs_buf) {
      e = pairs_buf->ensure(pp.capacity * 8);
      if (e != hipSuccess) return hip_error(e, "edge buffer allocation");
      pp.d_pairs = pairs_buf->as<uint32_t>();
    }
    if (dist_buf) {
      e = dist_buf->ensure(pp.capacity ? pp.capacity : 1);
      if (e != hipSuccess) return hip_error(e, "distance buffer allocation");
      pp.d_dist = dist_buf->as<uint8_t>();
    }
    (void)hipEventRecord(ctx->ev_b0, st);
    pipeline_enqueue(pl, pp, ctx->device, st, ctx->ev_p0, ctx->ev_p1);
    (void)hipEventRecord(ctx->ev_b1, st);
    e = pipeline_meta(pl, ctx->h_meta, st);
    if (e != hipSuccess) return hip_error(e, "build");
    const Meta m = *ctx->h_meta;
    float pk = 0.f, bt = 0.f;
    (void)hipEventElapsedTime(&pk, ctx->ev_p0, ctx->ev_p1);
    (void)hipEventElapsedTime(&bt, ctx->ev_b0, ctx->ev_b1);
    inf.pair_kernel_ms += pk;
    inf.build_ms += bt;
    inf.pair_launches += 1;
    inf.evaluated_pairs = m.plan.evaluated_pairs;
    note_work(sched, m, &inf);
    if (m.cnt.fault) return set_error(TCRNET_EDEVICE, "device sort stalled (internal)");
    if (m.cnt.err != kNoError) return set_error(TCRNET_EINVAL, "%s", input_error_message(m.cnt.err).c_str());
    if (m.plan.pad) return set_error(TCRNET_EDEVICE, "work plan overflow (internal)");
    *E = m.cnt.edges;
    if (info) *info = inf;
    if (*E <= pp.capacity) return TCRNET_OK;
    if (!grow_ok) return set_error(TCRNET_ETRUNC, "edge list of %llu edges exceeds the capacity %llu",
                                   (unsigned long long)*E, (unsigned long long)pp.capacity);
    pp.capacity = *E + *E / 16 + 1024;
  }
  return set_error(TCRNET_EDEVICE, "edge count changed between runs (internal)");
}

}  // namespace tcr

// ---------------------------------------------------------------- context
extern "C" {

int32_t tcrnet_ctx_create(int32_t device, const tcrnet_opts* opts, tcrnet_ctx** out) {
  if (!out) return set_error(TCRNET_EINVAL, "NULL output pointer");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return set_error(TCRNET_EDEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return set_error(TCRNET_EDEVICE, "device %d out of range", device);
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_error(e, "hipGetDeviceProperties");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_error(TCRNET_EDEVICE, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_error(e, "hipSetDevice");
  // this device's copy of the static scratch of tcrnet_build_device_noalloc
  if ((e = scratch_attach(device)) != hipSuccess) return hip_error(e, "static scratch lookup");
  tcrnet_ctx* c = new tcrnet_ctx();
  c->device = device;
  snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
  c->cus = prop.multiProcessorCount;
  if (opts) c->opts = *opts;
  if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
    delete c;
    return hip_error(e, "hipStreamCreate");
  }
  (void)hipEventCreate(&c->ev_p0);
  (void)hipEventCreate(&c->ev_p1);
  (void)hipEventCreate(&c->ev_b0);
  (void)hipEventCreate(&c->ev_b1);
  if ((e = host_malloc((void**)&c->h_meta, sizeof(Meta))) != hipSuccess) {
    c->h_meta = nullptr;
    (void)tcrnet_ctx_destroy(c);
    return hip_error(e, "pinned host allocation");
  }
  *out = c;
  return TCRNET_OK;
}

int32_t tcrnet_ctx_destroy(tcrnet_ctx* ctx) {
  if (!ctx) return TCRNET_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->batch_exec) (void)hipGraphExecDestroy(ctx->batch_exec);
  (void)hipEventDestroy(ctx->ev_p0);
  (void)hipEventDestroy(ctx->ev_p1);
  (void)hipEventDestroy(ctx->ev_b0);
  (void)hipEventDestroy(ctx->ev_b1);
  if (ctx->h_meta) (void)hipHostFree(ctx->h_meta);
  (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return TCRNET_OK;
}

const char* tcrnet_last_error(void) { return last_error_text(); }

const char* tcrnet_status_string(int32_t s) {
  switch (s) {
    case TCRNET_OK: return "TCRNET_OK";
    case TCRNET_EINVAL: return "TCRNET_EINVAL";
    case TCRNET_ENOMEM: return "TCRNET_ENOMEM";
    case TCRNET_EDEVICE: return "TCRNET_EDEVICE";
    case TCRNET_ESTATE: return "TCRNET_ESTATE";
    case TCRNET_ETRUNC: return "TCRNET_ETRUNC";
    default: return "TCRNET_UNKNOWN";
  }
}

const char* tcrnet_version(void) { return kVersion; }

void tcrnet_debug_fail_alloc(int64_t after) { arm_alloc_failure(after); }

// ----------------------------------------------------------------- builds
static int32_t build_host(tcrnet_ctx* ctx, const tcrnet_seqs* seqs, int32_t k, bool weighted, tcrnet_graph** out) {
  if (!out) return set_error(TCRNET_EINVAL, "NULL output pointer");
  *out = nullptr;
  if (!ctx) return set_error(TCRNET_EINVAL, "NULL context");
  int32_t rc;
  if ((rc = check_k(k)) || (rc = check_host_seqs(seqs, "tcrnet_build"))) return rc;
  (void)hipSetDevice(ctx->device);
  const uint32_t n = seqs->n;
  std::unique_ptr<tcrnet_graph> g(new tcrnet_graph());
  g->n = n;
  if (n > 0) {
    const uint64_t base = seqs->offsets[0];
    const uint64_t bytes = seqs->offsets[n] - base;
    hipError_t e;
    // characters, then the offsets from 0 (8-aligned), in pinned staging
    // filled in chunks on a few host threads: the copies then run as direct
    // DMA (N = 800,000: 3.8 ms host to host with pageable copies)
    const uint64_t off_at = (bytes + 7) & ~7ull;
    if ((e = ctx->batch_in.ensure(off_at + (uint64_t)(n + 1) * 8)) != hipSuccess)
      return hip_error(e, "pinned input staging");
    char* hdata = ctx->batch_in.as<char>();
    uint64_t* off = reinterpret_cast<uint64_t*>(hdata + off_at);
    const uint32_t in_chunks = host_chunks(bytes + (uint64_t)(n + 1) * 8);
    host_parallel(in_chunks, [&](uint32_t c) {
      const uint64_t b0 = bytes * c / in_chunks, b1 = bytes * (c + 1) / in_chunks;
      if (b1 > b0) memcpy(hdata + b0, seqs->data + base + b0, b1 - b0);
      const uint64_t i0 = (uint64_t)(n + 1) * c / in_chunks, i1 = (uint64_t)(n + 1) * (c + 1) / in_chunks;
      for (uint64_t i = i0; i < i1; ++i) off[i] = seqs->offsets[i] - base;
    });
    if ((e = ctx->in_data.ensure(bytes ? bytes : 1)) != hipSuccess) return hip_error(e, "input allocation");
    if ((e = ctx->in_off.ensure((n + 1) * 8)) != hipSuccess) return hip_error(e, "input allocation");
    if ((e = ctx->out_deg.ensure((uint64_t)n * 4)) != hipSuccess) return hip_error(e, "output allocation");
    if (bytes && (e = hipMemcpyAsync(ctx->in_data.p, hdata, bytes, hipMemcpyHostToDevice, ctx->stream)) !=
                     hipSuccess)
      return hip_error(e, "input copy");
    if ((e = hipMemcpyAsync(ctx->in_off.p, off, (uint64_t)(n + 1) * 8, hipMemcpyHostToDevice, ctx->stream)) !=
        hipSuccess)
      return hip_error(e, "input copy");
    PipeParams pp;
    pp.d_data = ctx->in_data.as<char>();
    pp.d_off = ctx->in_off.as<uint64_t>();
    pp.n = n;
    pp.k = k;
    pp.capacity = default_capacity(ctx, n);
    pp.d_deg = ctx->out_deg.as<int32_t>();
    uint64_t E = 0;
    // (run_pipeline waits for the stream, so the input staging is free after it)
    rc = run_pipeline(ctx, ctx->pipe, pp, ctx->stream, true, &ctx->out_pairs, &E, &g->info,
                      weighted ? &ctx->out_dist : nullptr);
    if (rc) return rc;
    // results: edges, degrees (and distances) into pinned staging, then into
    // the graph's arrays in chunks on a few host threads
    const uint64_t deg_at = E * 8, dist_at = deg_at + (uint64_t)n * 4;
    if ((e = ctx->batch_out.ensure(dist_at + (weighted ? E : 0))) != hipSuccess)
      return hip_error(e, "pinned result staging");
    char* hres = ctx->batch_out.as<char>();
    if (E && (e = hipMemcpyAsync(hres, ctx->out_pairs.p, E * 8, hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess)
      return hip_error(e, "result copy");
    if ((e = hipMemcpyAsync(hres + deg_at, ctx->out_deg.p, (uint64_t)n * 4, hipMemcpyDeviceToHost,
                            ctx->stream)) != hipSuccess)
      return hip_error(e, "result copy");
    if (weighted && E &&
        (e = hipMemcpyAsync(hres + dist_at, ctx->out_dist.p, E, hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess)
      return hip_error(e, "result copy");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_error(e, "result copy");
    g->pairs.resize(2 * E);
    g->deg.resize(n);
    if (weighted) g->dist.resize(E);
    char* dst_pairs = reinterpret_cast<char*>(g->pairs.data());
    char* dst_deg = reinterpret_cast<char*>(g->deg.data());
    char* dst_dist = reinterpret_cast<char*>(g->dist.data());
    const uint32_t out_chunks = host_chunks(dist_at + (weighted ? E : 0));
    host_parallel(out_chunks, [&](uint32_t c) {
      auto part = [&](char* dst, const char* src, uint64_t len) {
        const uint64_t b0 = len * c / out_chunks, b1 = len * (c + 1) / out_chunks;
        if (b1 > b0) memcpy(dst + b0, src + b0, b1 - b0);
      };
      part(dst_pairs, hres, E * 8);
      part(dst_deg, hres + deg_at, (uint64_t)n * 4);
      if (weighted) part(dst_dist, hres + dist_at, E);
    });
  }
  ctx->last = g->info;
  *out = g.release();
  return TCRNET_OK;
}

int32_t tcrnet_build(tcrnet_ctx* ctx, const tcrnet_seqs* seqs, int32_t k, tcrnet_graph** out) {
  return build_host(ctx, seqs, k, false, out);
}

int32_t tcrnet_build_weighted(tcrnet_ctx* ctx, const tcrnet_seqs* seqs, int32_t k_max, tcrnet_graph** out) {
  if (out) *out = nullptr;
  return build_host(ctx, seqs, k_max, true, out);
}

int32_t tcrnet_graph_distances(const tcrnet_graph* g, const uint8_t** dist, uint64_t* n_edges) {
  if (!g || !dist || !n_edges) return set_error(TCRNET_EINVAL, "NULL argument");
  if (g->dist.size() != g->pairs.size() / 2)
    return set_error(TCRNET_ESTATE, "graph was not built with distances (tcrnet_build_weighted)");
  *dist = g->dist.empty() ? nullptr : g->dist.data();
  *n_edges = g->dist.size();
  return TCRNET_OK;
}

int32_t tcrnet_build_device(tcrnet_ctx* ctx, const char* d_data, const uint64_t* d_offsets, uint32_t n, int32_t k,
                            void* stream, uint32_t* d_pairs, uint64_t pair_capacity, int32_t* d_degree,
                            uint64_t* n_edges) {
  if (!ctx || !n_edges) return set_error(TCRNET_EINVAL, "NULL context or n_edges");
  int32_t rc;
  if ((rc = check_k(k))) return rc;
  if (n > TCRNET_MAX_SEQS) return set_error(TCRNET_EINVAL, "more than 2^28 sequences");
  if (n && (!d_data || !d_offsets || !d_degree)) return set_error(TCRNET_EINVAL, "NULL device buffer");
  if (pair_capacity && !d_pairs) return set_error(TCRNET_EINVAL, "NULL pair buffer with nonzero capacity");
  (void)hipSetDevice(ctx->device);
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
  PipeParams pp;
  pp.d_data = d_data;
  pp.d_off = d_offsets;
  pp.n = n;
  pp.k = k;
  pp.capacity = pair_capacity ? pair_capacity : 1;
  pp.d_pairs = d_pairs;
  pp.d_deg = d_degree;
  DevBuf scratch_pairs;  // only used when the caller passes no pair buffer
  uint64_t E = 0;
  tcrnet_build_info info{};
  rc = run_pipeline(ctx, ctx->pipe, pp, st, false, pair_capacity ? nullptr : &scratch_pairs, &E, &info);
  ctx->last = info;
  *n_edges = E;
  return rc;
}

int32_t tcrnet_graph_edges(const tcrnet_graph* g, const uint32_t** pairs, uint64_t* n_edges) {
  if (!g || !pairs || !n_edges) return set_error(TCRNET_EINVAL, "NULL argument");
  *pairs = g->pairs.empty() ? nullptr : g->pairs.data();
  *n_edges = g->pairs.size() / 2;
  return TCRNET_OK;
}

int32_t tcrnet_graph_degree(const tcrnet_graph* g, const int32_t** degree, uint32_t* n) {
  if (!g || !degree || !n) return set_error(TCRNET_EINVAL, "NULL argument");
  *degree = g->deg.empty() ? nullptr : g->deg.data();
  *n = g->n;
  return TCRNET_OK;
}

int32_t tcrnet_graph_info(const tcrnet_graph* g, tcrnet_build_info* info) {
  if (!g || !info) return set_error(TCRNET_EINVAL, "NULL argument");
  *info = g->info;
  return TCRNET_OK;
}

int32_t tcrnet_ctx_last_info(const tcrnet_ctx* ctx, tcrnet_build_info* info) {
  if (!ctx || !info) return set_error(TCRNET_EINVAL, "NULL argument");
  *info = ctx->last;
  return TCRNET_OK;
}

void tcrnet_graph_free(tcrnet_graph* g) { delete g; }

int32_t tcrnet_graphs_views(tcrnet_graph* const* graphs, uint32_t n, const uint32_t** pairs, uint64_t* n_edges,
                            const int32_t** degree, uint32_t* n_nodes, const uint8_t** dist) {
  if (n && (!graphs || !pairs || !n_edges || !degree || !n_nodes || !dist))
    return set_error(TCRNET_EINVAL, "NULL argument");
  for (uint32_t i = 0; i < n; ++i)
    if (!graphs[i]) return set_error(TCRNET_EINVAL, "graph %u is NULL", i);
  for (uint32_t i = 0; i < n; ++i) {
    const tcrnet_graph* g = graphs[i];
    pairs[i] = g->pairs.empty() ? nullptr : g->pairs.data();
    n_edges[i] = g->pairs.size() / 2;
    degree[i] = g->deg.empty() ? nullptr : g->deg.data();
    n_nodes[i] = g->n;
    dist[i] = g->dist.empty() || g->dist.size() != g->pairs.size() / 2 ? nullptr : g->dist.data();
  }
  return TCRNET_OK;
}

// ----------------------------------------------------------------- batch
int32_t tcrnet_build_batch(tcrnet_ctx* ctx, const tcrnet_seqs* reps, uint32_t n_reps, int32_t k,
                           tcrnet_graph** outs) {
  if (!ctx || !outs || (n_reps && !reps)) return set_error(TCRNET_EINVAL, "NULL argument");
  for (uint32_t r = 0; r < n_reps; ++r) outs[r] = nullptr;
  int32_t rc;
  if ((rc = check_k(k))) return rc;
  (void)hipSetDevice(ctx->device);
  BatchInput bi;
  if ((rc = batch_upload(ctx, reps, n_reps, &bi))) return rc;
  const Sched sched = pick_sched(ctx, bi.n, k, kFormBatch);
  tcrnet_build_info info{};
  uint64_t E = 0;
  if ((rc = batch_launch(ctx, bi, k, sched, &E, &info))) return rc;
  // split by repertoire: edges are sorted by global (i, j), so each
  // repertoire's edges are one contiguous run, found by binary search; the
  // results come back into pinned staging and are split on a few threads
  const uint32_t n = bi.n;
  const std::vector<uint32_t>& seg = bi.seg;
  hipError_t e;
  const uint64_t deg_at = E * 8;
  if ((e = ctx->batch_out.ensure(deg_at + (uint64_t)(n ? n : 1) * 4)) != hipSuccess)
    return hip_error(e, "pinned result staging");
  uint32_t* all = ctx->batch_out.as<uint32_t>();
  int32_t* deg = reinterpret_cast<int32_t*>(ctx->batch_out.as<char>() + deg_at);
  if (E) (void)hipMemcpyAsync(all, ctx->out_pairs.p, E * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (n) (void)hipMemcpyAsync(deg, ctx->out_deg.p, (uint64_t)n * 4, hipMemcpyDeviceToHost, ctx->stream);
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_error(e, "result copy");
  std::vector<uint64_t> first(n_reps + 1);
  host_parallel(n_reps + 1, [&](uint32_t r) {
    uint64_t lo = 0, hi = E;  // first edge whose smaller id is >= seg[r]
    while (lo < hi) {
      const uint64_t mid = (lo + hi) / 2;
      if (all[2 * mid] < seg[r]) lo = mid + 1; else hi = mid;
    }
    first[r] = lo;
  });
  std::vector<tcrnet_graph*> made(n_reps, nullptr);
  host_parallel(n_reps, [&](uint32_t r) {
    tcrnet_graph* g = new tcrnet_graph();
    const uint32_t b = seg[r], en = seg[r + 1];
    g->n = en - b;
    g->deg.assign(deg + b, deg + en);
    const uint64_t p0 = first[r], p1 = first[r + 1];
    g->pairs.resize(2 * (p1 - p0));
    for (uint64_t x = p0; x < p1; ++x) {
      g->pairs[2 * (x - p0)] = all[2 * x] - b;
      g->pairs[2 * (x - p0) + 1] = all[2 * x + 1] - b;
    }
    g->info = info;
    made[r] = g;
  });
  for (uint32_t r = 0; r < n_reps; ++r) outs[r] = made[r];
  ctx->last = info;
  return TCRNET_OK;
}

}  // extern "C"

namespace tcr {

// Concatenate the repertoires (segment r holds global ids [seg[r], seg[r+1]))
// and copy them to the context's input buffers.
int32_t batch_upload(tcrnet_ctx* ctx, const tcrnet_seqs* reps, uint32_t n_reps, BatchInput* bi) {
  int32_t rc;
  for (uint32_t r = 0; r < n_reps; ++r)
    if ((rc = check_host_seqs(&reps[r], "tcrnet_build_batch"))) return rc;
  std::vector<uint32_t>& seg = bi->seg;
  seg.assign(n_reps + 1, 0);
  uint64_t bytes = 0, total = 0;
  for (uint32_t r = 0; r < n_reps; ++r) {
    total += reps[r].n;
    if (total > TCRNET_MAX_SEQS) return set_error(TCRNET_EINVAL, "more than 2^28 sequences in one batch");
    seg[r + 1] = (uint32_t)total;
    if (reps[r].n) bytes += reps[r].offsets[reps[r].n] - reps[r].offsets[0];
  }
  const uint32_t n = (uint32_t)total;
  bi->n = n;
  bi->n_reps = n_reps;
  // characters then 8-aligned offsets, in pinned staging, filled on a few
  // threads (one repertoire at a time each)
  std::vector<uint64_t> boff(n_reps + 1, 0);
  for (uint32_t r = 0; r < n_reps; ++r)
    boff[r + 1] = boff[r] + (reps[r].n ? reps[r].offsets[reps[r].n] - reps[r].offsets[0] : 0);
  const uint64_t off_at = (bytes + 7) & ~7ull;
  if (hipError_t pe = ctx->batch_in.ensure(off_at + (uint64_t)(n + 1) * 8); pe != hipSuccess)
    return hip_error(pe, "pinned input staging");
  char* hdata = ctx->batch_in.as<char>();
  uint64_t* off = reinterpret_cast<uint64_t*>(hdata + off_at);
  host_parallel(n_reps, [&](uint32_t r) {
    const tcrnet_seqs& s = reps[r];
    if (!s.n) return;
    const uint64_t b0 = s.offsets[0], pos = boff[r];
    memcpy(hdata + pos, s.data + b0, boff[r + 1] - pos);
    uint64_t* o = off + seg[r];
    for (uint32_t q = 0; q < s.n; ++q) o[q] = pos + (s.offsets[q] - b0);
  });
  off[n] = bytes;
  hipError_t e;
  if ((e = ctx->in_data.ensure(bytes ? bytes : 1)) != hipSuccess) return hip_error(e, "input allocation");
  if ((e = ctx->in_off.ensure((uint64_t)(n + 1) * 8)) != hipSuccess) return hip_error(e, "input allocation");
  if ((e = ctx->in_seg.ensure((uint64_t)(n_reps + 1) * 4)) != hipSuccess) return hip_error(e, "input allocation");
  if ((e = ctx->out_deg.ensure((uint64_t)(n ? n : 1) * 4)) != hipSuccess) return hip_error(e, "output allocation");
  if (bytes && (e = hipMemcpyAsync(ctx->in_data.p, hdata, bytes, hipMemcpyHostToDevice, ctx->stream)) !=
                   hipSuccess)
    return hip_error(e, "input copy");
  if ((e = hipMemcpyAsync(ctx->in_off.p, off, (uint64_t)(n + 1) * 8, hipMemcpyHostToDevice, ctx->stream)) !=
      hipSuccess)
    return hip_error(e, "input copy");
  if ((e = hipMemcpyAsync(ctx->in_seg.p, seg.data(), (uint64_t)(n_reps + 1) * 4, hipMemcpyHostToDevice,
                          ctx->stream)) != hipSuccess)
    return hip_error(e, "input copy");
  // the staging buffers and the segment table are read by the copies above:
  // wait before they can be reused or go
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_error(e, "input copy");
  return TCRNET_OK;
}

// One batched launch of the uploaded input: the whole launch sequence
// (counters, encode, sort, plan, pairs, canonicalise) as one HIP graph,
// captured again only when the shape or a buffer changed, then replayed.
// Re-runs once with the exact edge capacity after an overflow.
int32_t batch_launch(tcrnet_ctx* ctx, const BatchInput& bi, int32_t k, const Sched& sched, uint64_t* E_out,
                     tcrnet_build_info* info_out) {
  const uint32_t n = bi.n;
  PipeParams pp;
  pp.d_data = ctx->in_data.as<char>();
  pp.d_off = ctx->in_off.as<uint64_t>();
  pp.n = n;
  pp.d_segoff = ctx->in_seg.as<uint32_t>();
  pp.n_seg = bi.n_reps ? bi.n_reps : 1;
  pp.k = k;
  pp.capacity = ctx->opts.edge_capacity ? ctx->opts.edge_capacity : std::max<uint64_t>(65536, 4ull * n);
  pp.d_deg = ctx->out_deg.as<int32_t>();
  pp.sched = sched;
  tcrnet_build_info info{};
  info.texts_per_item = sched.texts_per_item;
  info.waves_per_simd = sched.waves_per_simd;
  info.peq_lds = sched.peq_lds;
  info.pack = sched.pack;
  info.tuned = sched.tuned;
  uint64_t E = 0;
  hipError_t e;
  if (n > 0) {
    for (int attempt = 0; attempt < 2; ++attempt) {
      if ((e = pipeline_reserve(ctx->pipe, n, pp.n_seg, k, sched.texts_per_item, pp.capacity)) != hipSuccess)
        return hip_error(e, "workspace allocation");
      if ((e = ctx->out_pairs.ensure(pp.capacity * 8)) != hipSuccess) return hip_error(e, "output allocation");
      pp.d_pairs = ctx->out_pairs.as<uint32_t>();
      BatchKey key;
      key.n = n;
      key.n_seg = pp.n_seg;
      key.k = k;
      key.T = sched.texts_per_item;
      key.W = sched.waves_per_simd;
      key.lds = sched.peq_lds;
      key.pack = sched.pack;
      key.count = sched.count_work;
      key.capacity = pp.capacity;
      key.desc_cap = ctx->pipe.desc_cap;
      {
        Pipeline& pl = ctx->pipe;
        const DevBuf* used[] = {&pl.rec,   &pl.key,   &pl.key2,   &pl.val,     &pl.val2,       &pl.srec,
                                &pl.speq,  &pl.off,   &pl.descs,  &pl.ibase,   &pl.meta,       &pl.tmp,
                                &pl.edges, &pl.edist, &pl.ekeys,  &pl.ekeys2,  &ctx->in_data,  &ctx->in_off,
                                &ctx->in_seg, &ctx->out_pairs, &ctx->out_deg};
        for (const DevBuf* b : used) key.bufs.emplace_back(b->p, b->cap);
      }
      if (!ctx->batch_exec || !(key == ctx->batch_key)) {
        if (ctx->batch_exec) {
          (void)hipGraphExecDestroy(ctx->batch_exec);
          ctx->batch_exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        if ((e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
          return hip_error(e, "graph capture");
        pipeline_enqueue(ctx->pipe, pp, ctx->device, ctx->stream, nullptr, nullptr);
        if ((e = hipStreamEndCapture(ctx->stream, &graph)) != hipSuccess) return hip_error(e, "graph capture");
        e = hipGraphInstantiate(&ctx->batch_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
          ctx->batch_exec = nullptr;
          return hip_error(e, "graph instantiate");
        }
        ctx->batch_key = key;
        ctx->batch_captures++;
        info.graph_captured = 1;
      }
      (void)hipEventRecord(ctx->ev_b0, ctx->stream);
      if ((e = hipGraphLaunch(ctx->batch_exec, ctx->stream)) != hipSuccess) return hip_error(e, "graph launch");
      (void)hipEventRecord(ctx->ev_b1, ctx->stream);
      if ((e = pipeline_meta(ctx->pipe, ctx->h_meta, ctx->stream)) != hipSuccess) return hip_error(e, "batch build");
      const Meta m = *ctx->h_meta;
      float bt = 0.f;
      (void)hipEventElapsedTime(&bt, ctx->ev_b0, ctx->ev_b1);
      info.build_ms += bt;
      info.pair_launches += 1;
      info.evaluated_pairs = m.plan.evaluated_pairs;
      note_work(sched, m, &info);
      if (m.cnt.fault) return set_error(TCRNET_EDEVICE, "device sort stalled (internal)");
      if (m.cnt.err != kNoError) {
        const std::vector<uint32_t>& seg = bi.seg;
        const unsigned long long idx = m.cnt.err >> 2;
        const uint32_t r = (uint32_t)(std::upper_bound(seg.begin(), seg.end(), (uint32_t)idx) - seg.begin()) - 1;
        return set_error(TCRNET_EINVAL, "repertoire %u, %s", r,
                         input_error_message(((idx - seg[r]) << 2) | (m.cnt.err & 3u)).c_str());
      }
      if (m.plan.pad) return set_error(TCRNET_EDEVICE, "work plan overflow (internal)");
      E = m.cnt.edges;
      if (E <= pp.capacity) break;
      pp.capacity = E + E / 16 + 1024;
      if (attempt == 1) return set_error(TCRNET_EDEVICE, "edge count changed between runs (internal)");
    }
  }
  *E_out = E;
  *info_out = info;
  return TCRNET_OK;
}

}  // namespace tcr
