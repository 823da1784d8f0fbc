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

// The same codes for the letters 'A' + u, u < 26, as 5-bit fields of three
// words (12 letters each; 31: not a residue), so a lane maps a byte with
// register arithmetic instead of a per-lane table read.
struct LetterCodes {
  uint64_t w[3];
  constexpr LetterCodes() : w() {
    const CodeTable t;
    for (int u = 0; u < 26; ++u) {
      const int c = t.v['A' + u];
      w[u / 12] |= (uint64_t)(c < 0 ? 31 : c) << (5 * (u % 12));
    }
  }
};
constexpr LetterCodes kLetters = LetterCodes();

__device__ __forceinline__ int residue_code(uint32_t byte) {
  const uint32_t u = byte - (uint32_t)'A';
  if (u >= 26u) return -1;
  const uint64_t word = u < 12u ? kLetters.w[0] : u < 24u ? kLetters.w[1] : kLetters.w[2];
  const uint32_t c = (uint32_t)(word >> (5u * (u % 12u))) & 31u;
  return c == 31u ? -1 : (int)c;
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_reset_counters(Counters* c) {
  if (threadIdx.x < kQueueStripes) c->queue[threadIdx.x].next = 0;
  if (threadIdx.x == 0) {
    c->edges = 0;
    c->err = kNoError;
    c->fault = 0;
    c->visits = c->steps = c->steps_packed = 0;
  }
}

__global__ void k_reset_work(Counters* c) {
  if (threadIdx.x < kQueueStripes) c->queue[threadIdx.x].next = 0;
  if (threadIdx.x == 0) {
    c->edges = 0;
    c->visits = c->steps = c->steps_packed = 0;
  }
}

__global__ void k_record_keys(const SeqRec* __restrict__ rec, uint32_t n, int nres, int len_shift,
                              uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const SeqRec r = rec[i];
  uint64_t lex = 0;
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    if (q < nres) {
      const uint32_t c = q < (int)(r.len & kLenMask) ? (r.w[q / 6] >> (5 * (q % 6))) & 31u : 0u;
      lex |= (uint64_t)c << (5 * (nres - 1 - q));
    }
  }
  key[i] = ((uint64_t)(r.len & kLenMask) << len_shift) | lex;
  val[i] = i;
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
  if (err != 2) {
    // the string's bytes as the aligned dwords that hold them (at most 9 for
    // 32 bytes; a dword holding a byte of the buffer lies in the same page)
    const uintptr_t a0 = (uintptr_t)(data + b) & ~(uintptr_t)3;
    const uint32_t lead = (uint32_t)((uintptr_t)(data + b) - a0);
    const uint32_t nw = (lead + len + 3) / 4;
    const __attribute__((address_space(1))) uint32_t* src =
        reinterpret_cast<const __attribute__((address_space(1))) uint32_t*>(a0);
    uint32_t dw[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) dw[j] = (uint32_t)j < nw ? src[j] : 0u;
    uint32_t al[8];  // the string's bytes 4j .. 4j+3
#pragma unroll
    for (int j = 0; j < 8; ++j) al[j] = __builtin_amdgcn_alignbit(dw[j + 1], dw[j], 8u * lead);
#pragma unroll
    for (int q = 0; q < kMaxLen; ++q) {
      if (q < (int)len) {
        int c = residue_code((al[q / 4] >> (8 * (q % 4))) & 255u);
        if (c < 0) {
          if (err == 0) err = 1;
          c = 0;
        }
        w[q / 6] |= (uint32_t)c << (5 * (q % 6));
        if (q < nres) lex |= (uint64_t)c << (5 * (nres - 1 - q));
      }
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
#pragma unroll
  for (int q = 0; q < kSkipDepths; ++q) r.nxt[q] = 0;
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

// Sorted record s with its prefix-group ends (deepest first: the group at
// depth d contains the one at depth d + 1, so each search starts from the last
// known member, galloping then bisecting over the sorted keys).
__global__ void k_gather(const SeqRec* __restrict__ rec, const uint32_t* __restrict__ val,
                         const uint64_t* __restrict__ skey, uint64_t n, int nres, SeqRec* __restrict__ srec,
                         PeqRec* __restrict__ speq) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  SeqRec r = rec[val[s]];
  const uint64_t key = skey[s];
  uint64_t lo = s;  // last position known to share the current prefix
  for (int d = kSkipDepths; d >= 1; --d) {
    if (d > nres) {
      r.nxt[d - 1] = (uint32_t)(s + 1);
      continue;
    }
    const int sh = 5 * (nres - d);
    const uint64_t pre = key >> sh;
    uint64_t hi = n, step = 1;
    for (;;) {
      const uint64_t p = lo + step;
      if (p >= n) break;
      if ((skey[p] >> sh) != pre) {
        hi = p;
        break;
      }
      lo = p;
      step <<= 1;
    }
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if ((skey[mid] >> sh) == pre) lo = mid; else hi = mid;
    }
    r.nxt[d - 1] = (uint32_t)hi;
  }
  // common prefix lengths with the next record and with each group end: the
  // groups are nested, so a position lies in the depth-d group of s exactly
  // when it is below nxt[d-1]
  uint32_t packed = r.len & kLenMask;
  uint32_t l_next = 0;
#pragma unroll
  for (int d = 1; d <= kSkipDepths; ++d) l_next += r.nxt[d - 1] > s + 1 ? 1u : 0u;
  packed |= l_next << 6;
#pragma unroll
  for (int d = 2; d <= kSkipDepths; ++d) {
    uint32_t l = 0;
#pragma unroll
    for (int q = 1; q < d; ++q) l += r.nxt[q - 1] > r.nxt[d - 1] ? 1u : 0u;
    packed |= l << (10 + 3 * (d - 2));
  }
  r.len = packed;
  srec[s] = r;
  {
    WalkEnt* walk = const_cast<WalkEnt*>(walk_of(srec, (uint32_t)n));
#pragma unroll
    for (int d = 0; d < kWalkDepth; ++d) {
      WalkEnt e;
      e.end8 = 8u * r.nxt[d];
      e.code = (r.w[0] >> (5 * d)) & 31u;
      walk[(uint64_t)d * (n + 1) + s] = e;
      if (s + 1 == n) walk[(uint64_t)d * (n + 1) + n] = WalkEnt{8u * (uint32_t)n, 0u};  // the extra entry
    }
  }
  // bit planes of the residue codes
  uint32_t pl[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < kMaxLen; ++q) {
    const uint32_t c = (r.w[q / 6] >> (5 * (q % 6))) & 31u;
#pragma unroll
    for (int b = 0; b < 5; ++b) pl[b] |= ((c >> b) & 1u) << q;
  }
  PeqRec p;
#pragma unroll
  for (int b = 0; b < 5; ++b) p.pl[b] = pl[b];
  speq[s] = p;
}

// One thread block plans every part.  Entries:
//   self part:  (segment, m, delta) with n = m - delta, 0 <= delta <= k;
//               delta = 0 entries are split into row blocks of texts_per_item
//               patterns so that every work item of a triangle holds at least
//               one valid pair;
//   cross part: (La, Lb) with |La - Lb| <= k; the longer length supplies the
//               patterns (for equal lengths the set with fewer sequences
//               when it has at least 64, else the other).
constexpr int kPlanThreads = 1024;
constexpr uint32_t kPlanPer = 4;  // entries per thread in a planning round

__device__ uint32_t part_entries(const PlanPart& p, int k) {
  return p.cross ? 32u * (uint32_t)(2 * k + 1) : p.a.n_seg * 32u * (uint32_t)(k + 1);
}

struct Entry {
  const SeqRec* prec;
  const PeqRec* ppeq;
  const SeqRec* trec;
  const WalkEnt* twalk;
  uint32_t tw_len;
  uint32_t p0, np, t0, nt, m, n, tri, ndesc, pack;
  uint64_t items, pairs;
};

// Patterns per lane of a bucket pair whose patterns have length m.  A masked
// half holds 16 set miss bits, which must exceed k.
__device__ __forceinline__ uint32_t pack_for(uint32_t m, int k, uint32_t pack_ok) {
  return pack_ok && m <= kPackMaxLen && k < 16 ? 2u : 1u;
}

__device__ Entry entry_shape(const PlanPart& part, uint32_t e, int k, uint32_t T, uint32_t pack_ok) {
  Entry r;
  r.ndesc = 0;
  r.pack = 1;
  r.items = 0;
  r.pairs = 0;
  r.tri = 0;
  r.np = r.nt = 0;
  r.p0 = r.t0 = 0;
  r.m = r.n = 0;
  r.prec = part.a.srec;
  r.ppeq = part.a.speq;
  r.trec = part.a.srec;
  r.tw_len = part.a.off[part.a.n_seg * 64] + 1;
  r.twalk = walk_of(part.a.srec, r.tw_len - 1);
  if (!part.cross) {
    const uint32_t per_seg = 32u * (uint32_t)(k + 1);
    const uint32_t seg = e / per_seg;
    const uint32_t rem = e - seg * per_seg;
    const uint32_t m = 1 + rem / (uint32_t)(k + 1);
    const uint32_t delta = rem % (uint32_t)(k + 1);
    if (delta >= m) return r;
    const uint32_t n = m - delta;
    const uint32_t* off = part.a.off;
    const uint32_t cm = seg * 64 + m, cn = seg * 64 + n;
    r.m = m;
    r.n = n;
    r.p0 = off[cm];
    r.np = off[cm + 1] - off[cm];
    r.t0 = off[cn];
    r.nt = off[cn + 1] - off[cn];
    r.pack = pack_for(m, k, pack_ok);
    const uint32_t G = 64u * r.pack;  // patterns per group
    if (delta > 0) {
      if (r.np == 0 || r.nt == 0) return r;
      r.ndesc = 1;
      r.items = (uint64_t)((r.np + G - 1) / G) * ((r.nt + T - 1) / T);
      r.pairs = (uint64_t)r.np * r.nt;
    } else {
      if (r.np < 2) return r;
      r.tri = 1;
      r.ndesc = (r.np - 1 + T - 1) / T;  // row blocks b with b*T <= np-2
      // (a triangle's items are counted per plan pass, by pass_counts)
      r.pairs = (uint64_t)r.np * (r.np - 1) / 2;
    }
  } else {
    const uint32_t span = (uint32_t)(2 * k + 1);
    const uint32_t La = 1 + e / span;
    const int Lb = (int)La + (int)(e % span) - k;
    if (Lb < 1 || Lb > kMaxLen) return r;
    const uint32_t na = part.a.off[La + 1] - part.a.off[La];
    const uint32_t nb = part.b.off[Lb + 1] - part.b.off[Lb];
    if (na == 0 || nb == 0) return r;
    // the longer strings are the patterns (the exit rule needs m >= n).  For
    // equal lengths the smaller set is, once it fills half a wave: the walk
    // then runs over the larger, denser set's prefix tree (a query batch
    // against a resident repertoire: 4,096 queries at k = 2 in 0.88 instead
    // of 0.96 ms); a handful of patterns would walk that whole tree in few
    // items, so below that the larger set supplies them (many short items)
    const bool a_small = na <= nb;
    const bool pat_a = (int)La > Lb || ((int)La == Lb && ((a_small ? na : nb) >= 64u ? a_small : !a_small));
    if (pat_a) {
      r.m = La; r.n = (uint32_t)Lb;
      r.p0 = part.a.off[La]; r.np = na;
      r.t0 = part.b.off[Lb]; r.nt = nb;
      r.prec = part.a.srec; r.ppeq = part.a.speq; r.trec = part.b.srec;
      r.tw_len = part.b.off[part.b.n_seg * 64] + 1;
      r.twalk = walk_of(part.b.srec, r.tw_len - 1);
    } else {
      r.m = (uint32_t)Lb; r.n = La;
      r.p0 = part.b.off[Lb]; r.np = nb;
      r.t0 = part.a.off[La]; r.nt = na;
      r.prec = part.b.srec; r.ppeq = part.b.speq; r.trec = part.a.srec;
      r.tw_len = part.a.off[part.a.n_seg * 64] + 1;
      r.twalk = walk_of(part.a.srec, r.tw_len - 1);
    }
    r.ndesc = 1;
    r.pack = pack_for(r.m, k, pack_ok);
    r.items = (uint64_t)((r.np + 64u * r.pack - 1) / (64u * r.pack)) * ((r.nt + T - 1) / T);
    r.pairs = (uint64_t)na * nb;
  }
  return r;
}

// Exclusive prefix sums over the block of three values at once (the
// barriers of one scan serve all three), and their block totals.
struct Scan3 {
  uint64_t v[3];
};
__device__ Scan3 block_excl_scan3(Scan3 in, uint64_t (*sh)[kPlanThreads], Scan3& total) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 3; ++q) sh[q][t] = in.v[q];
  __syncthreads();
  for (int d = 1; d < kPlanThreads; d <<= 1) {
    uint64_t x[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) x[q] = t >= d ? sh[q][t - d] : 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) sh[q][t] += x[q];
    __syncthreads();
  }
  Scan3 r;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    total.v[q] = sh[q][kPlanThreads - 1];
    r.v[q] = sh[q][t] - in.v[q];
  }
  __syncthreads();
  return r;
}

// Texts per work item of a triangle's diagonal chunk (its first texts_per_item
// texts, where the patterns share their prefixes with the texts and the walk
// goes deepest): an eighth of the rest.
__device__ __forceinline__ uint32_t diag_texts(uint32_t T) { return max(64u, T / 8u / 64u * 64u); }

// Text chunks of row block bk (patterns bk*T .. of a triangle over np sorted
// sequences) in plan pass `pass`: pass 0, its texts past its first T in
// chunks of T, ceil((np - bk*T - T) / T) = C - bk - 1; pass 1, its first
// min(np - bk*T, T) texts in chunks of Td: cT for a whole block, cr for the
// block of np mod T.  The divisions are taken once per triangle (one
// thread plans all of a triangle's row blocks).
struct TriChunks {
  uint32_t C, cT, cr;
};
__device__ __forceinline__ TriChunks tri_shape(uint32_t np, uint32_t T, uint32_t Td) {
  TriChunks c;
  c.C = (np + T - 1) / T;
  c.cT = (T + Td - 1) / Td;
  c.cr = (np % T + Td - 1) / Td;
  return c;
}
__device__ __forceinline__ uint32_t tri_chunks(const TriChunks& c, uint32_t np, uint32_t bk, int pass, uint32_t T) {
  if (pass == 0) return c.C - bk - 1;
  return np - bk * T >= T ? c.cT : c.cr;
}

// Descriptors and items of entry `en` in plan pass `pass`: pass 0 holds the
// rectangles and each triangle row block's texts past its first T (chunks
// of T); pass 1 the row blocks' first T texts (chunks of diag_texts(T)).
// Work items are handed out in plan order, so the diagonal chunks -- the
// most expensive items, cut 8 ways -- come last and fill the end of the
// launch while the big items drain.
__device__ void pass_counts(const Entry& en, int pass, uint32_t T, uint32_t& ndesc, uint64_t& items) {
  ndesc = 0;
  items = 0;
  if (en.ndesc == 0) return;
  const uint32_t G = 64u * en.pack;
  if (!en.tri) {
    if (pass == 0) {
      ndesc = 1;
      items = en.items;
    }
    return;
  }
  const uint32_t Td = diag_texts(T);
  const TriChunks tc = tri_shape(en.np, T, Td);
  for (uint32_t bk = 0; bk < en.ndesc; ++bk) {
    const uint32_t rows = min(T, en.np - bk * T);
    const uint32_t cols = en.np - bk * T;
    const uint64_t groups = (rows + G - 1) >> (en.pack == 2 ? 7u : 6u);
    if (pass == 0) {
      if (cols > T) {
        ndesc += 1;
        items += groups * tri_chunks(tc, en.np, bk, 0, T);
      }
    } else {
      ndesc += 1;
      items += groups * tri_chunks(tc, en.np, bk, 1, T);
    }
  }
}

// Entry order of plan pass 0: the same entries with the pattern lengths
// taken longest first.  Work items are handed out in plan order; started
// early, the longer buckets' items (more steps per visited text) leave a
// shorter end to the launch (N = 50,000, k = 2: 0.361 -> 0.353 ms; no change
// at 800,000, where the diagonal pass forms the end).
__device__ __forceinline__ uint32_t longest_first(const PlanPart& part, uint32_t e, int k) {
  const uint32_t span = part.cross ? (uint32_t)(2 * k + 1) : (uint32_t)(k + 1);
  const uint32_t per_seg = 32u * span;
  const uint32_t seg = e / per_seg, rem = e - seg * per_seg;
  const uint32_t li = rem / span;
  return seg * per_seg + (31u - li) * span + (rem - li * span);
}

// Descriptors of entry en in plan pass `pass` (nd of them, ni items) at
// descriptor position dpos and item position ipos, unless they would run
// past max_desc (the plan then reports an overflow).
__device__ void write_entry(const Entry& en, int pass, uint32_t nd, uint64_t ni, uint64_t dpos, uint64_t ipos,
                            uint32_t Td, uint32_t T, uint32_t max_desc, Desc* __restrict__ descs,
                            uint64_t* __restrict__ item_base) {
  if (dpos + nd <= max_desc) {
    Desc d;
    d.prec = en.prec;
    d.ppeq = en.ppeq;
    d.trec = en.trec;
    d.twalk = en.twalk;
    d.tw_len = en.tw_len;
    d.m = en.m;
    d.n = en.n;
    d.tri = en.tri;
    d.pack = en.pack;
    const uint32_t G = 64u * en.pack;
    if (!en.tri) {
      d.p0 = en.p0; d.np = en.np; d.t0 = en.t0; d.nt = en.nt;
      d.T = T;
      d.chunks = (en.nt + T - 1) / T;
      d.item_base = ipos;
      d.items = ni;
      descs[dpos] = d;
      item_base[dpos] = ipos;
    } else {
      uint64_t ib = ipos;
      uint32_t q = 0;
      const TriChunks tc = tri_shape(en.np, T, Td);
      for (uint32_t bk = 0; bk < en.ndesc; ++bk) {
        const uint32_t rows = min(T, en.np - bk * T);
        const uint32_t cols = en.np - bk * T;
        d.p0 = en.p0 + bk * T; d.np = rows;
        if (pass == 0) {
          if (cols <= T) continue;
          d.t0 = en.p0 + bk * T + T; d.nt = cols - T; d.T = T;
        } else {
          d.t0 = en.p0 + bk * T; d.nt = min(cols, T); d.T = Td;
        }
        d.chunks = tri_chunks(tc, en.np, bk, pass, T);
        d.item_base = ib;
        d.items = (uint64_t)((rows + G - 1) >> (en.pack == 2 ? 7u : 6u)) * d.chunks;
        descs[dpos + q] = d;
        item_base[dpos + q] = ib;
        ib += d.items;
        ++q;
      }
    }
  }
}

__global__ __launch_bounds__(kPlanThreads) void k_plan(const PlanPart* __restrict__ parts, uint32_t n_parts,
                                                       PlanPart inline_part, int k, uint32_t T,
                                                       uint32_t pack_ok, Desc* __restrict__ descs,
                                                       uint64_t* __restrict__ item_base, uint32_t max_desc,
                                                       Plan* plan) {
  __shared__ uint64_t sh[3][kPlanThreads];
  if (!parts) {
    parts = nullptr;
    n_parts = 1;
  }
  const uint32_t Td = diag_texts(T);
  uint64_t run_desc = 0, run_items = 0, run_pairs = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (uint32_t pi = 0; pi < n_parts; ++pi) {
      const PlanPart part = parts ? parts[pi] : inline_part;
      const uint32_t n_entries = part_entries(part, k);
      // a round plans `per` consecutive entries per thread: their counts
      // first, then one scan of each per-thread total over the block, then
      // the descriptors (the entry shapes taken again), in entry order.  A
      // part of many entries (a batch: 32 (k+1) per repertoire) takes
      // kPlanPer per thread, which divides its rounds and scans by kPlanPer
      // (256 repertoires: 229 -> 111 us); one round of a part that fits the
      // block keeps one entry per thread, whose shapes then take their loads
      // and loops side by side.
      const uint32_t per = n_entries > (uint32_t)kPlanThreads ? kPlanPer : 1u;
      for (uint32_t e0 = 0; e0 < n_entries; e0 += kPlanThreads * per) {
        const uint32_t eb = e0 + threadIdx.x * per;
        uint32_t nd_j[kPlanPer];
        uint64_t ni_j[kPlanPer];
        uint32_t td = 0;
        uint64_t ti = 0, tp = 0;
#pragma unroll
        for (uint32_t j = 0; j < kPlanPer; ++j) {
          nd_j[j] = 0;
          ni_j[j] = 0;
          if (j < per && eb + j < n_entries) {
            const Entry en = entry_shape(part, pass == 0 ? longest_first(part, eb + j, k) : eb + j, k, T, pack_ok);
            pass_counts(en, pass, T, nd_j[j], ni_j[j]);
            if (pass == 0) tp += en.pairs;
          }
          td += nd_j[j];
          ti += ni_j[j];
        }
        Scan3 tot;
        const Scan3 pre = block_excl_scan3(Scan3{{td, ti, tp}}, sh, tot);
        uint64_t dpos = run_desc + pre.v[0];
        uint64_t ipos = run_items + pre.v[1];
#pragma unroll
        for (uint32_t j = 0; j < kPlanPer; ++j) {
          const uint32_t nd = nd_j[j];
          const uint64_t ni = ni_j[j];
          if (nd > 0) write_entry(entry_shape(part, pass == 0 ? longest_first(part, eb + j, k) : eb + j, k, T,
                                              pack_ok),
                                  pass, nd, ni, dpos, ipos, Td, T, max_desc, descs, item_base);
          dpos += nd;
          ipos += ni;
        }
        run_desc += tot.v[0];
        run_items += tot.v[1];
        run_pairs += tot.v[2];
      }
    }
  }
  if (threadIdx.x == 0) {
    Plan p;
    const bool ok = run_desc <= max_desc;
    p.total_items = ok ? run_items : 0;
    p.evaluated_pairs = run_pairs;
    p.n_desc = (uint32_t)(ok ? run_desc : 0);
    p.pad = ok ? 0u : 1u;  // 1: descriptor overflow
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

void launch_reset_work(Counters* c, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_work, dim3(1), dim3(64), 0, st, c);
}

// Residues in the sort key: as many as the prefix-group ends need (kSkipDepths)
// -- sorting deeper only reorders texts inside a depth-8 group, which neither
// the jumps nor the resumed steps look at -- and never more than fit 58 bits
// beside the segment.
static int encode_nres(uint32_t seg_bits) {
  const int fit = (int)((58 - seg_bits) / 5);
  return fit < kSkipDepths ? fit : kSkipDepths;
}
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

void launch_record_keys(const SeqRec* rec, uint32_t n, uint64_t* key, uint32_t* val, hipStream_t st) {
  if (n == 0) return;
  const int nres = encode_nres(0);
  hipLaunchKernelGGL(k_record_keys, dim3(blocks_for(n, 256)), dim3(256), 0, st, rec, n, nres, 5 * nres, key, val);
}

void launch_bucket_bounds(const uint64_t* key, uint64_t n, int combo_shift, uint32_t n_combo, uint32_t* off,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_bounds, dim3(blocks_for(n + 1, 256)), dim3(256), 0, st, key, n, combo_shift, n_combo,
                     off);
}

void launch_gather(const SeqRec* rec, const uint32_t* val, const uint64_t* skey, uint64_t n, uint32_t seg_bits,
                   SeqRec* srec, PeqRec* speq, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, 256)), dim3(256), 0, st, rec, val, skey, n,
                     encode_nres(seg_bits), srec, speq);
}

uint32_t plan_max_desc_self(uint32_t n_seg, int k, uint32_t T, uint64_t n) {
  // rectangles: one per (segment, m, delta>0); triangles: sum over buckets of
  // ceil((np-1)/T) <= n/T + 32 per segment row blocks, each a diagonal and
  // (when it has more than T texts) an off-diagonal descriptor
  uint64_t v = (uint64_t)n_seg * 32u * (uint32_t)(k + 1) + 2 * (n / T + (uint64_t)n_seg * 32u) + 1;
  return (uint32_t)v;
}

uint32_t plan_max_desc_cross(int k) { return 32u * (uint32_t)(2 * k + 1); }

void launch_plan(const PlanPart* d_parts, uint32_t n_parts, const PlanPart& inline_part, int k, uint32_t T,
                 bool pack, Desc* descs, uint64_t* item_base, uint32_t max_desc, Plan* plan, hipStream_t st) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, st, d_parts, n_parts, inline_part, k, T,
                     pack ? 1u : 0u, descs, item_base, max_desc, plan);
}

}  // namespace tcr
