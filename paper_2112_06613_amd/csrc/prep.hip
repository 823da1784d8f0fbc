// Steps a1-a3 of the build: validate and encode the strings, bucket them by
// length, gather them into sorted order with their bit masks, and plan the
// bucket-pair work items.
#include "kernels.h"

namespace tcr {

namespace {

// Residue code of each byte: position in the paper's amino-acid list
// (Methods, "Combination of amino acids"), -1 for anything else.
struct CodeTable {
  int8_t v[256];
  constexpr CodeTable() : v() {
    for (int i = 0; i < 256; ++i) v[i] = -1;
    const char* a = "ARNDCQEGHILKMFPSTWYV";
    for (int c = 0; c < kAlpha; ++c) v[(unsigned char)a[c]] = (int8_t)c;
  }
};
__constant__ CodeTable kCodes = CodeTable();

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_reset_counters(Counters* c) {
  if (threadIdx.x == 0) {
    c->item_next = 0;
    c->edges = 0;
    c->err = kNoError;
    c->pad = 0;
  }
}

__global__ void k_encode(const char* __restrict__ data, const uint64_t* __restrict__ off, uint32_t n,
                         const uint32_t* __restrict__ seg_off, uint32_t n_seg, int nres, int len_shift,
                         int seg_shift, uint32_t id_base, uint32_t id_tag, SeqRec* __restrict__ rec,
                         uint64_t* __restrict__ key, uint32_t* __restrict__ val, Counters* cnt) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t b = off[i], e = off[i + 1];
  unsigned long long err = 0;
  uint32_t len = 1;
  if (e <= b || e - b > (uint64_t)kMaxLen) {
    err = 2;
  } else {
    len = (uint32_t)(e - b);
  }
  uint32_t w[6] = {0, 0, 0, 0, 0, 0};
  uint64_t lex = 0;
#pragma unroll
  for (int q = 0; q < kMaxLen; ++q) {
    if (q < (int)len && err != 2) {
      int c = kCodes.v[(unsigned char)data[b + q]];
      if (c < 0) {
        if (err == 0) err = 1;
        c = 0;
      }
      w[q / 6] |= (uint32_t)c << (5 * (q % 6));
      if (q < nres) lex |= (uint64_t)c << (5 * (nres - 1 - q));
    }
  }
  uint32_t seg = 0;
  if (n_seg > 1) {
    uint32_t lo = 0, hi = n_seg;  // seg_off[lo] <= i < seg_off[hi]
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (seg_off[mid] <= i) lo = mid; else hi = mid;
    }
    seg = lo;
  }
  SeqRec r;
#pragma unroll
  for (int q = 0; q < 6; ++q) r.w[q] = w[q];
  r.len = len;
  r.id = (id_base + i) | id_tag;
  rec[i] = r;
  key[i] = ((uint64_t)seg << seg_shift) | ((uint64_t)len << len_shift) | lex;
  val[i] = i;
  if (err) atomicMin(&cnt->err, ((unsigned long long)i << 2) | err);
}

__global__ void k_bounds(const uint64_t* __restrict__ key, uint64_t n, int shift, uint32_t n_combo,
                         uint32_t* __restrict__ off) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s > n) return;
  const uint32_t cur = s < n ? (uint32_t)(key[s] >> shift) : n_combo;
  const uint32_t first = s > 0 ? (uint32_t)(key[s - 1] >> shift) + 1 : 0;
  for (uint32_t c = first; c <= cur && c <= n_combo; ++c) off[c] = (uint32_t)s;
}

__global__ void k_gather(const SeqRec* __restrict__ rec, const uint32_t* __restrict__ val, uint64_t n,
                         SeqRec* __restrict__ srec, PeqRec* __restrict__ speq) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const SeqRec r = rec[val[s]];
  srec[s] = r;
  // bit planes of the residue codes, then Peq[c] = positions whose code is c
  uint32_t pl[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < kMaxLen; ++q) {
    const uint32_t c = (r.w[q / 6] >> (5 * (q % 6))) & 31u;
#pragma unroll
    for (int b = 0; b < 5; ++b) pl[b] |= ((c >> b) & 1u) << q;
  }
  const uint32_t lm = r.len >= 32 ? ~0u : ((1u << r.len) - 1u);
  PeqRec p;
#pragma unroll
  for (int c = 0; c < kAlpha; ++c) {
    uint32_t eq = lm;
#pragma unroll
    for (int b = 0; b < 5; ++b) eq &= ((c >> b) & 1) ? pl[b] : ~pl[b];
    p.eq[c] = eq;
  }
  speq[s] = p;
}

// One thread block.  Entries (segment, m, delta) in segment-major order;
// delta = 0 entries are split into row blocks of texts_per_item patterns so
// that every work item of the triangle holds at least one valid pair.
constexpr int kPlanThreads = 1024;

__device__ void entry_shape(const uint32_t* off, uint32_t e, int k, uint32_t T, uint32_t& seg, uint32_t& m,
                            uint32_t& n, uint32_t& np, uint32_t& nt, uint32_t& ndesc, uint64_t& items,
                            uint64_t& pairs) {
  const uint32_t per_seg = 32u * (uint32_t)(k + 1);
  seg = e / per_seg;
  const uint32_t rem = e - seg * per_seg;
  m = 1 + rem / (uint32_t)(k + 1);
  const uint32_t delta = rem % (uint32_t)(k + 1);
  ndesc = 0;
  items = 0;
  pairs = 0;
  np = nt = 0;
  if (delta >= m) return;
  n = m - delta;
  const uint32_t cm = seg * 64 + m, cn = seg * 64 + n;
  np = off[cm + 1] - off[cm];
  nt = off[cn + 1] - off[cn];
  if (delta > 0) {
    if (np == 0 || nt == 0) return;
    ndesc = 1;
    items = (uint64_t)((np + 63) / 64) * ((nt + T - 1) / T);
    pairs = (uint64_t)np * nt;
  } else {
    if (np < 2) return;
    ndesc = (np - 1 + T - 1) / T;  // row blocks b with b*T <= np-2
    for (uint32_t bk = 0; bk < ndesc; ++bk) {
      const uint32_t rows = min(T, np - bk * T);
      const uint32_t cols = np - bk * T;
      items += (uint64_t)((rows + 63) / 64) * ((cols + T - 1) / T);
    }
    pairs = (uint64_t)np * (np - 1) / 2;
  }
}

__device__ uint64_t block_excl_scan_u64(uint64_t v, uint64_t* sh, uint64_t& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < kPlanThreads; d <<= 1) {
    uint64_t x = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  total = sh[kPlanThreads - 1];
  uint64_t r = sh[t] - v;
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kPlanThreads) void k_plan(const uint32_t* __restrict__ off, uint32_t n_seg, int k,
                                                       uint32_t T, Desc* __restrict__ descs,
                                                       uint64_t* __restrict__ item_base, uint32_t max_desc,
                                                       Plan* plan) {
  __shared__ uint64_t sh[kPlanThreads];
  const uint32_t n_entries = n_seg * 32u * (uint32_t)(k + 1);
  uint64_t run_desc = 0, run_items = 0, run_pairs = 0;
  for (uint32_t e0 = 0; e0 < n_entries; e0 += kPlanThreads) {
    const uint32_t e = e0 + threadIdx.x;
    uint32_t seg = 0, m = 0, n = 0, np = 0, nt = 0, nd = 0;
    uint64_t items = 0, pairs = 0;
    if (e < n_entries) entry_shape(off, e, k, T, seg, m, n, np, nt, nd, items, pairs);
    uint64_t tot_d, tot_i, tot_p;
    const uint64_t dpos = run_desc + block_excl_scan_u64(nd, sh, tot_d);
    const uint64_t ipos = run_items + block_excl_scan_u64(items, sh, tot_i);
    block_excl_scan_u64(pairs, sh, tot_p);
    if (nd > 0 && dpos + nd <= max_desc) {
      const uint32_t pm = off[seg * 64 + m], pn = off[seg * 64 + n];
      if (m != n) {
        Desc d;
        d.p0 = pm; d.np = np; d.t0 = pn; d.nt = nt; d.m = m; d.n = n; d.tri = 0;
        d.chunks = (nt + T - 1) / T;
        d.item_base = ipos;
        d.items = items;
        descs[dpos] = d;
        item_base[dpos] = ipos;
      } else {
        uint64_t ib = ipos;
        for (uint32_t bk = 0; bk < nd; ++bk) {
          Desc d;
          const uint32_t rows = min(T, np - bk * T);
          d.p0 = pm + bk * T; d.np = rows;
          d.t0 = pm + bk * T; d.nt = np - bk * T;
          d.m = m; d.n = n; d.tri = 1;
          d.chunks = (d.nt + T - 1) / T;
          d.item_base = ib;
          d.items = (uint64_t)((rows + 63) / 64) * d.chunks;
          descs[dpos + bk] = d;
          item_base[dpos + bk] = ib;
          ib += d.items;
        }
      }
    }
    run_desc += tot_d;
    run_items += tot_i;
    run_pairs += tot_p;
  }
  if (threadIdx.x == 0) {
    Plan p;
    p.total_items = run_desc <= max_desc ? run_items : 0;
    p.evaluated_pairs = run_pairs;
    p.n_desc = (uint32_t)(run_desc <= max_desc ? run_desc : 0);
    p.pad = run_desc <= max_desc ? 0u : 1u;  // 1: descriptor overflow
    *plan = p;
  }
}

inline uint32_t blocks_for(uint64_t n, uint32_t bs) { return (uint32_t)((n + bs - 1) / bs); }

}  // namespace

void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return;
  uint32_t blocks = blocks_for(n, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, st, p, n, v);
}

void launch_reset_counters(Counters* c, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, st, c);
}

static int encode_nres(uint32_t seg_bits) { return (int)((58 - seg_bits) / 5); }
int encode_key_bits(uint32_t seg_bits) { return (int)seg_bits + 6 + 5 * encode_nres(seg_bits); }
int encode_combo_shift(uint32_t seg_bits) { return 5 * encode_nres(seg_bits); }

void launch_encode(const char* d_data, const uint64_t* d_off, uint32_t n, const uint32_t* seg_off,
                   uint32_t n_seg, uint32_t seg_bits, uint32_t id_base, uint32_t id_tag, SeqRec* rec,
                   uint64_t* key, uint32_t* val, Counters* cnt, hipStream_t st) {
  if (n == 0) return;
  const int nres = encode_nres(seg_bits);
  const int len_shift = 5 * nres;
  const int seg_shift = len_shift + 6;
  hipLaunchKernelGGL(k_encode, dim3(blocks_for(n, 256)), dim3(256), 0, st, d_data, d_off, n, seg_off, n_seg,
                     nres, len_shift, seg_shift, id_base, id_tag, rec, key, val, cnt);
}

void launch_bucket_bounds(const uint64_t* key, uint64_t n, int combo_shift, uint32_t n_combo, uint32_t* off,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_bounds, dim3(blocks_for(n + 1, 256)), dim3(256), 0, st, key, n, combo_shift, n_combo,
                     off);
}

void launch_gather(const SeqRec* rec, const uint32_t* val, uint64_t n, SeqRec* srec, PeqRec* speq,
                   hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, 256)), dim3(256), 0, st, rec, val, n, srec, speq);
}

uint32_t plan_max_desc(uint32_t n_seg, const uint32_t*, int k, uint32_t T, uint64_t n) {
  // rectangles: one per (segment, m, delta>0); triangles: sum over buckets of
  // ceil((np-1)/T) <= n/T + 32 per segment
  uint64_t v = (uint64_t)n_seg * 32u * (uint32_t)(k + 1) + n / T + (uint64_t)n_seg * 32u + 1;
  return (uint32_t)v;
}

void launch_plan(const uint32_t* off, uint32_t n_seg, int k, uint32_t T, Desc* descs, uint64_t* item_base,
                 uint32_t max_desc, Plan* plan, hipStream_t st) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, st, off, n_seg, k, T, descs, item_base, max_desc,
                     plan);
}

}  // namespace tcr
