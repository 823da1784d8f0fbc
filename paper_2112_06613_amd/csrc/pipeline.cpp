// Host orchestration of one build pipeline: buffer sizing and the launch
// sequence, with no host synchronisation inside (so the same sequence can be
// captured in a HIP graph).
#include "pipeline.h"

#include <cstdio>

namespace tcr {

namespace {
thread_local std::string g_last_error;
}

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

hipError_t pipeline_reserve(Pipeline& pl, uint64_t n, uint32_t n_seg, int k, uint32_t T, uint64_t capacity) {
  const uint64_t nn = n ? n : 1;
  const uint32_t max_desc = plan_max_desc(n_seg, nullptr, k, T, n);
  const uint64_t cap = capacity ? capacity : 1;
  hipError_t e;
#define TCR_RESERVE(buf, bytes) \
  if ((e = (buf).ensure(bytes)) != hipSuccess) return e;
  TCR_RESERVE(pl.rec, nn * sizeof(SeqRec));
  TCR_RESERVE(pl.key, nn * 8);
  TCR_RESERVE(pl.key2, nn * 8);
  TCR_RESERVE(pl.val, nn * 4);
  TCR_RESERVE(pl.val2, nn * 4);
  TCR_RESERVE(pl.srec, nn * sizeof(SeqRec));
  TCR_RESERVE(pl.speq, nn * sizeof(PeqRec));
  TCR_RESERVE(pl.off, ((uint64_t)n_seg * 64 + 1) * 4);
  TCR_RESERVE(pl.descs, (uint64_t)max_desc * sizeof(Desc));
  TCR_RESERVE(pl.ibase, (uint64_t)max_desc * 8);
  TCR_RESERVE(pl.meta, 128);
  const uint64_t tw = radix_tmp_words(nn > cap ? nn : cap);
  TCR_RESERVE(pl.tmp, tw * 4);
  TCR_RESERVE(pl.edges, cap * 8);
  TCR_RESERVE(pl.ekeys, cap * 8);
  TCR_RESERVE(pl.ekeys2, cap * 8);
#undef TCR_RESERVE
  pl.n_cap = nn;
  pl.e_cap = cap;
  pl.desc_cap = max_desc;
  return hipSuccess;
}

void pipeline_enqueue(Pipeline& pl, const PipeParams& pp, int device, hipStream_t st, hipEvent_t ev0,
                      hipEvent_t ev1) {
  const uint32_t n = pp.n;
  const uint32_t seg_bits = seg_bits_for(pp.n_seg);
  Counters* cnt = pl.cnt();
  launch_reset_counters(cnt, st);
  if (pp.d_deg) launch_fill_u32(reinterpret_cast<uint32_t*>(pp.d_deg), n, 0u, st);
  if (n == 0) return;

  // a1: validate + encode, a2: sort by (segment, length, residues)
  launch_encode(pp.d_data, pp.d_off, n, pp.d_segoff, pp.n_seg, seg_bits, pp.id_base, 0u, pl.rec.as<SeqRec>(),
                pl.key.as<uint64_t>(), pl.val.as<uint32_t>(), cnt, st);
  const bool alt = radix_sort(pl.key.as<uint64_t>(), pl.key2.as<uint64_t>(), pl.val.as<uint32_t>(),
                              pl.val2.as<uint32_t>(), n, nullptr, encode_key_bits(seg_bits), pl.tmp.as<uint32_t>(),
                              st);
  const uint64_t* skey = alt ? pl.key2.as<uint64_t>() : pl.key.as<uint64_t>();
  const uint32_t* sval = alt ? pl.val2.as<uint32_t>() : pl.val.as<uint32_t>();
  const uint32_t n_combo = pp.n_seg * 64;
  launch_bucket_bounds(skey, n, encode_combo_shift(seg_bits), n_combo, pl.off.as<uint32_t>(), st);
  launch_gather(pl.rec.as<SeqRec>(), sval, n, pl.srec.as<SeqRec>(), pl.speq.as<PeqRec>(), st);

  // a3: bucket-pair plan
  launch_plan(pl.off.as<uint32_t>(), pp.n_seg, pp.k, pp.sched.texts_per_item, pl.descs.as<Desc>(),
              pl.ibase.as<uint64_t>(), pl.desc_cap, pl.plan(), st);

  // a4-a6: pairs
  PairArgs a;
  a.descs = pl.descs.as<Desc>();
  a.item_base = pl.ibase.as<uint64_t>();
  a.plan = pl.plan();
  a.prec = pl.srec.as<SeqRec>();
  a.ppeq = pl.speq.as<PeqRec>();
  a.trec = pl.srec.as<SeqRec>();
  a.cnt = cnt;
  a.edges = pl.edges.as<uint32_t>();
  a.capacity = pp.capacity;
  a.texts_per_item = pp.sched.texts_per_item;
  a.k = pp.k;
  if (ev0) (void)hipEventRecord(ev0, st);
  launch_pairs(a, pair_grid_blocks(device, pp.sched.waves_per_simd), pp.sched.peq_lds, st);
  if (ev1) (void)hipEventRecord(ev1, st);

  // a7-a8: canonical sorted edge list and degrees
  const int shift = (int)bits_for(n);
  launch_edge_keys(pl.edges.as<uint32_t>(), pp.capacity, &cnt->edges, 0, shift, pl.ekeys.as<uint64_t>(), st);
  const bool ealt = radix_sort(pl.ekeys.as<uint64_t>(), pl.ekeys2.as<uint64_t>(), nullptr, nullptr, pp.capacity,
                               &cnt->edges, 2 * shift, pl.tmp.as<uint32_t>(), st);
  const uint64_t* sk = ealt ? pl.ekeys2.as<uint64_t>() : pl.ekeys.as<uint64_t>();
  launch_unpack(sk, pp.capacity, &cnt->edges, 0, shift, pp.d_pairs, pp.d_deg, st);
}

hipError_t pipeline_meta(const Pipeline& pl, Meta* host_meta, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(&host_meta->cnt, pl.cnt(), sizeof(Counters), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(&host_meta->plan, pl.plan(), sizeof(Plan), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

}  // namespace tcr
