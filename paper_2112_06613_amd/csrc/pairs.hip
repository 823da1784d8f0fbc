// Steps a4-a6: the bucket-pair kernel.
//
// Distance: the bit-parallel global edit distance of Myers (J. ACM 46(3),
// 1999) in the formulation of Hyyro (2001/2003), one 32-bit word per pattern.
// Column j of the DP table (text prefix of length j) is held as vertical
// deltas VP (+1) and VN (-1); the top row is D[0][j] = j, so the horizontal
// delta entering row 1 is +1 at every step (the "+ 1" after the shift, which
// equals "| 1" because the shifted word has bit 0 clear).
//
// Early exit: D never decreases along a diagonal (Ukkonen 1985), so after
// text step j the cell on the final diagonal, D[j+delta][j] with
// delta = m - n >= 0, is a lower bound of lev = D[m][n].  Hyyro's D0 word has
// bit r-1 set exactly when D[r][j] = D[r-1][j-1] (a zero step along the
// diagonal).  Each step therefore ORs the complement of the diagonal's D0 bit
// into a per-lane miss word Z whose bits below delta start set:
//   popcount(Z) = D[j+delta][j]   after j steps, and = lev at the end.
// A lane is still within k while popcount(Z) <= k.  The paper aborts once the
// smallest entry of a DP row exceeds l_max ("GPU-based network generation");
// the diagonal cell is the tighter exact bound of the same kind.
//
// Prefix-group jumps: texts are visited in sorted order.  When no lane is
// within k after e residues of a text, the lanes' state depended only on the
// patterns and those e residues, so every following text that shares them
// ends the same way without an edge; the wave continues at the end of that
// prefix group (stored in the text's record for e <= 8).
//
// Layout of the work: a wave holds 64 consecutive patterns of one length
// bucket (one per lane, their Peq tables in VGPRs, or in LDS) and walks the
// texts of a chunk of another (or the same) bucket; each text is
// wave-uniform and is read with scalar loads into SGPRs.  Patterns of at
// most 16 residues go two to a lane (128 per wave, one in each 16-bit half
// of every word): the per-text bookkeeping, which is scalar and bounds the
// kernel, is then shared by twice the patterns.  Sequences are sorted by
// (length, residues), so the patterns of a wave share prefixes and leave a
// text at nearly the same step.  Pattern = the longer string of the pair
// when lengths differ (it exits earliest).
//
// Output: patterns whose final distance is <= k are compacted with a ballot
// per half, staged in LDS per wave, and take consecutive global edge slots
// with one atomic add per staged batch (coalesced writes).
#include "kernels.h"

namespace tcr {

namespace {

constexpr int kEdgeBuf = 128;  // staged edges per wave

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t rfl64(uint64_t v) {
  return ((uint64_t)rfl((uint32_t)(v >> 32)) << 32) | rfl((uint32_t)v);
}

__device__ __forceinline__ uint32_t low_mask(uint32_t r) { return r >= 32 ? ~0u : ((1u << r) - 1u); }

// Loads through address-space views of descriptor pointers: the wave-uniform
// text records are read-only for the whole launch, so they are read through
// the constant address space (scalar loads into SGPRs); pattern data through
// the global one.  (The host compilation pass only parses kernel bodies.)
// load_const_at reads at a 32-bit byte offset from a wave-uniform base (the
// offset stays a scalar register operand of the load: no 64-bit address
// arithmetic per text).
template <class T>
__device__ __forceinline__ T load_const_at(const void* base, uint32_t byte_off) {
#if defined(__HIP_DEVICE_COMPILE__)
  const __attribute__((address_space(4))) char* q = (const __attribute__((address_space(4))) char*)base;
  T v;
  __builtin_memcpy(&v, (const T*)(q + byte_off), sizeof(T));
  return v;
#else
  return *(const T*)((const char*)base + byte_off);
#endif
}

template <class T>
__device__ __forceinline__ T load_global(const T* p, uint32_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  const __attribute__((address_space(1))) T* q = (const __attribute__((address_space(1))) T*)p;
  T v;
  __builtin_memcpy(&v, (const T*)(q + i), sizeof(T));
  return v;
#else
  return p[i];
#endif
}

// 2x and 2x + 1 as integer adds (a shift by one is the same value; on gfx950
// the adds issue at twice the rate of shifts and funnel shifts).
__device__ __forceinline__ uint32_t twice(uint32_t x) {
  uint32_t r;
  asm("v_add_u32 %0, %1, %1" : "=v"(r) : "v"(x));
  return r;
}
__device__ __forceinline__ uint32_t twice_plus1(uint32_t x) {
  uint32_t r;
  asm("v_add3_u32 %0, %1, %1, 1" : "=v"(r) : "v"(x));
  return r;
}

// Two patterns per lane (patterns of at most 16 residues): pattern A in
// bits 0-15 and pattern B in bits 16-31 of every bit-vector word.  The
// bitwise operations of a step act on both halves alike; the one addition
// and the two shifts by one must not carry from bit 15 into bit 16, so they
// are 16-bit packed adds (v_pk_add_u16, one instruction for both halves).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}

// kPack: 1, one pattern per lane; 2, two per lane with 16-bit packed adds
// (patterns of 16 residues); 3, two per lane for patterns of at most 15
// residues, with plain 32-bit adds.  v_pk_add_u16 issues at half the rate of
// v_add_u32 on gfx950, and with at most 15 residues no plain add carries
// across the halves: bit 15 of Eq is clear, and VP is kept masked to the
// pattern's bits after every step, so (Eq & VP) + VP stays below 2^16 in each
// half and the doubling of HN = D0 & VP cannot reach bit 16; the doubling of
// HP may move a bit into bit 16 of X, which the step sets anyway.  The bits
// of a half above the pattern (which the add and the doubling can set) never
// flow down into the pattern's bits, as in the one-pattern form.
template <int kPack>
__device__ __forceinline__ uint32_t add_p(uint32_t a, uint32_t b) {
  if constexpr (kPack == 2) return pk_add(a, b);
  else return a + b;
}
template <int kPack>
__device__ __forceinline__ uint32_t dbl_p(uint32_t x) {
  if constexpr (kPack == 2) return pk_add(x, x);
  else return twice(x);
}

// popcount(z) <= k for one miss word, with the cheap forms for k = 1 (at
// most one bit set) and k = 2 (at most two) selected at compile time.
template <int kMode>
__device__ __forceinline__ bool within_k_word(uint32_t z, int k) {
  if (kMode == 1) return (z & (z - 1u)) == 0u;
  if (kMode == 2) {
    const uint32_t y = z & (z - 1u);
    return (y & (y - 1u)) == 0u;
  }
  return __popc(z) <= k;
}

// The lane has a pattern still within k: the word, or either 16-bit half of
// a two-pattern word (a half is zero after clearing its lowest k set bits).
// The halves' lowest set bits are cleared with one 32-bit subtraction of
// 0x10001 (twice the issue rate of a packed one): it borrows from the upper
// half only when the lower half is zero, and then the lane is within k
// whatever the upper half holds.
template <int kMode, int kPack>
__device__ __forceinline__ bool within_k_lane(uint32_t z, int k) {
  if constexpr (kPack == 1) {
    return within_k_word<kMode>(z, k);
  } else {
    if (kMode == 1 || kMode == 2) {
      uint32_t y = z & (z - 0x10001u);
      if (kMode == 2) y &= y - 0x10001u;
      return min(y & 0xFFFFu, y >> 16) == 0u;
    }
    return (int)min(__popc(z & 0xFFFFu), __popc(z >> 16)) <= k;
  }
}

template <int V>
struct Tag {
  static constexpr int value = V;
};

// Depth of the walk's sibling loops: residues 0 .. kLoopDepth-1 of a text are
// stepped one prefix-tree level at a time (every sibling group of a level in
// its own loop iteration, the parent's state resident in registers); texts
// that are still alive after kLoopDepth residues run the rest of their steps
// one text at a time.  Must not exceed kSkipDepths (the group ends a record
// holds).
constexpr int kLoopDepth = kWalkDepth;
static_assert(kLoopDepth <= kSkipDepths, "a sibling loop needs the group end of its depth");

// Byte offset of the id field in a SeqRec.
constexpr uint32_t kRecIdOff = 28;

// kMode: the within-k test on the miss word: 1 (k = 1), 2 (k = 2), 0 (any k:
// popcount).  kCount: also count visited texts and wave text steps (the
// work-counting variant; the traversal is the same).
template <bool kPeqLds, int kMode, bool kCount>
__global__ __launch_bounds__(kBlock) void k_pairs(const Desc* __restrict__ descs,
                                                  const uint64_t* __restrict__ item_base,
                                                  const Plan* __restrict__ plan, Counters* __restrict__ cnt,
                                                  uint32_t* __restrict__ edges, uint8_t* __restrict__ edist,
                                                  uint64_t capacity, int k) {
  __shared__ uint32_t lds_eq[kPeqLds ? (kBlock / kWave) * kAlpha * kWave : 1];
  // per-wave edge staging: hits collect here and take their global slots
  // with one atomic per kEdgeBuf edges instead of one per hitting text
  __shared__ uint2 lds_edge[kBlock / kWave][kEdgeBuf];
  __shared__ uint8_t lds_dist[kBlock / kWave][kEdgeBuf];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wid = threadIdx.x >> 6;
  const uint64_t total = plan->total_items;
  const uint32_t nd = plan->n_desc;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint32_t* wave_eq = lds_eq + (kPeqLds ? wid * kAlpha * kWave : 0);
  uint2* wave_edge = lds_edge[wid];
  uint8_t* wave_dist = lds_dist[wid];
  uint32_t staged = 0;  // edges in wave_edge (wave-uniform)
  // work counters of the counting variant (wave-uniform)
  uint32_t n_visits = 0, n_steps = 0, n_steps_packed = 0;

  // Move the staged edges to consecutive global slots (one atomic per wave).
  auto flush = [&]() {
    __builtin_amdgcn_wave_barrier();
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&cnt->edges, (unsigned long long)staged);
    base = rfl64(base);
    for (uint32_t i = lane; i < staged; i += kWave) {
      const uint64_t slot = base + i;
      if (slot < capacity) {
        *reinterpret_cast<uint2*>(edges + 2 * slot) = wave_edge[i];
        if (edist) edist[slot] = wave_dist[i];
      }
    }
    __builtin_amdgcn_wave_barrier();
    staged = 0;
  };

  // One work item: pattern group g (kPack * 64 patterns, kPack per lane)
  // against text chunk c of descriptor d.
  auto run_item = [&](auto pack_tag, const Desc& d, uint32_t g, uint32_t c) {
    constexpr int kPack = decltype(pack_tag)::value;
    constexpr bool kTwo = kPack >= 2;           // two patterns per lane
    constexpr uint32_t kGroup = kWave * (kTwo ? 2 : 1);  // patterns of a work item
    const SeqRec* prec = d.prec;
    const PeqRec* ppeq = d.ppeq;
    const SeqRec* trec = d.trec;
    const uint32_t gbase = d.p0 + g * kGroup;
    // lane's patterns: gbase + lane (bits 0-15 when packed), gbase + 64 + lane
    // (bits 16-31); a lane outside the item reads pattern d.p0 and is masked
    const bool ok0 = g * kGroup + lane < d.np;
    const bool ok1 = kTwo && g * kGroup + kWave + lane < d.np;
    const uint32_t p0 = ok0 ? gbase + lane : d.p0;
    const uint32_t p1 = ok1 ? gbase + kWave + lane : d.p0;
    const uint32_t tb0 = d.t0 + c * d.T;
    const uint32_t te = min(d.t0 + d.nt, tb0 + d.T);
    uint32_t tb = tb0;
    if (d.tri && tb < gbase + 1) tb = gbase + 1;
    if (tb >= te) return;  // a diagonal chunk wholly before the group's patterns

    const uint32_t m = d.m, n = d.n;  // m >= n: the pattern is the longer string
    const uint32_t Mm = kTwo ? low_mask(m) * 0x10001u : low_mask(m);
    // Myers' Peq table of the lane's pattern(s), built from their bit planes:
    // eq[a] = positions whose code is a (within the length)
    uint32_t eq[kAlpha];
    {
      const PeqRec pr = load_global(ppeq, p0);
      uint32_t pl[5];
#pragma unroll
      for (int b = 0; b < 5; ++b) pl[b] = pr.pl[b];
      if constexpr (kTwo) {
        const PeqRec ph = load_global(ppeq, p1);
#pragma unroll
        for (int b = 0; b < 5; ++b) pl[b] |= ph.pl[b] << 16;
      }
#pragma unroll
      for (int a = 0; a < kAlpha; ++a) {
        uint32_t e = Mm;
#pragma unroll
        for (int b = 0; b < 5; ++b) e &= ((a >> b) & 1) ? pl[b] : ~pl[b];
        eq[a] = e;
      }
    }
    if (kPeqLds) {
#pragma unroll
      for (int a = 0; a < kAlpha; ++a) wave_eq[a * kWave + lane] = eq[a];
      __builtin_amdgcn_wave_barrier();
    }

    const uint32_t delta = m - n;     // final diagonal: row = column + delta
    // Miss word: bit delta+J set when text step J missed on the final
    // diagonal, bits below delta set from the start, so popcount(Z) is the
    // diagonal cell D[delta+j][j] after j steps and D[m][n] = lev at the end
    // (per 16-bit half when packed).  A pattern outside the item starts with
    // all its bits set (never within k).
    uint32_t z_item, m_item;
    if constexpr (kTwo) {
      z_item = (ok0 ? (1u << delta) - 1u : 0xFFFFu) | ((ok1 ? (1u << delta) - 1u : 0xFFFFu) << 16);
      m_item = (1u << delta) * 0x10001u;
    } else {
      z_item = ok0 ? (1u << delta) - 1u : ~0u;
      m_item = 1u << delta;
    }
    // in a triangle item, texts before tri_end still have patterns at or
    // after them in the item (those patterns are masked off)
    const uint32_t tri_end = d.tri ? gbase + kGroup : 0u;
    const SeqRec* tbase = trec + tb0;  // this item's text records
    auto rec_at = [&](uint32_t t) { return load_const_at<SeqRec>(tbase, (t - tb0) * (uint32_t)sizeof(SeqRec)); };

    // Edges of the patterns whose final miss word fZ is within k, against
    // every text of [t_first, t_end) (a run of identical texts).
    auto emit = [&](uint32_t fZ, uint32_t t_first, uint32_t t_end) {
      const uint32_t fz0 = kTwo ? fZ & 0xFFFFu : fZ;
      const bool hit0 = within_k_word<kMode>(fz0, k);
      const bool hit1 = kTwo && within_k_word<kMode>(fZ >> 16, k);
      const uint64_t hm0 = __ballot(hit0);
      const uint64_t hm1 = kTwo ? __ballot(hit1) : 0ull;
      if (!(hm0 | hm1)) return;
      const uint32_t nh0 = (uint32_t)__popcll(hm0);
      const uint32_t nh = nh0 + (uint32_t)__popcll(hm1);
      const uint32_t* pid = reinterpret_cast<const uint32_t*>(prec);  // ids: word 7 of a record
      const uint32_t id0 = hit0 ? load_global(pid, 16 * p0 + 7) : 0u;  // pattern ids, read on a hit only
      const uint32_t id1 = hit1 ? load_global(pid, 16 * p1 + 7) : 0u;
      for (uint32_t u = t_first; u < t_end; ++u) {
        const uint32_t tid = load_const_at<uint32_t>(tbase, (u - tb0) * (uint32_t)sizeof(SeqRec) + kRecIdOff);
        if (staged + nh > (uint32_t)kEdgeBuf) flush();
        if (hit0) {
          const uint32_t pos = staged + (uint32_t)__popcll(hm0 & lt_mask);
          wave_edge[pos] = make_uint2(id0, tid);
          wave_dist[pos] = (uint8_t)__popc(fz0);
        }
        if (hit1) {
          const uint32_t pos = staged + nh0 + (uint32_t)__popcll(hm1 & lt_mask);
          wave_edge[pos] = make_uint2(id1, tid);
          wave_dist[pos] = (uint8_t)__popc(fZ >> 16);
        }
        staged += nh;
      }
      if constexpr (kCount) n_visits += t_end - t_first - 1;  // the identical texts after the first
    };

// One Myers/Hyyro text step on residue J of record `rec` from the state
// (VP, VN, Z), then the miss accounting: OR the diagonal row's miss bit
// (mj) into Z; alive: some lane still within k.
#define TCR_EQ(cc) (kPeqLds ? wave_eq[(cc) * kWave + lane] : eq[(cc)])
#define TCR_CODE(rr, q) (((rr).w[(q) / 6] >> (5 * ((q) % 6))) & 31u)
#define TCR_STEP(rr, J, mj) TCR_STEP_CODE(TCR_CODE(rr, J), mj)
#define TCR_STEP_CODE(code, mj) TCR_STEP_EQV(TCR_EQ(code), mj)
#define TCR_STEP_EQV(eqv, mj)                                                  \
  {                                                                            \
    const uint32_t Eq = (eqv);                                                 \
    uint32_t D0;                                                               \
    if constexpr (kTwo) {                                                      \
      D0 = (add_p<kPack>(Eq & VP, VP) ^ VP) | Eq | VN;                         \
      const uint32_t HP = VN | ~(D0 | VP);                                     \
      const uint32_t HN = D0 & VP;                                             \
      const uint32_t X = dbl_p<kPack>(HP) | 0x00010001u;                       \
      VN = X & D0;                                                             \
      VP = dbl_p<kPack>(HN) | ~(X | D0);                                       \
      if constexpr (kPack == 3) VP &= Mm;                                      \
    } else {                                                                   \
      D0 = (((Eq & VP) + VP) ^ VP) | Eq | VN;                                  \
      const uint32_t HP = VN | ~(D0 | VP);                                     \
      const uint32_t HN = D0 & VP;                                             \
      const uint32_t X = twice_plus1(HP);                                      \
      VN = X & D0;                                                             \
      VP = twice(HN) | ~(X | D0);                                              \
    }                                                                          \
    Z |= ~D0 & (mj);                                                           \
    alive = __ballot((within_k_lane<kMode, kPack>(Z, k))) != 0ull;             \
    if constexpr (kCount) {                                                    \
      ++n_steps;                                                               \
      if constexpr (kTwo) ++n_steps_packed;                                    \
    }                                                                          \
  }

    // The rest of one text's steps, kStart .. n-1, from the state (VP, VN,
    // Z) after kStart residues; stops after the step at which no lane is
    // within k.  Returns the exit (the step index, or 32 when all n steps ran)
    // and the next text to visit: after an exit at J < kSkipDepths (and not
    // in the ragged run) the end of the text's depth-(J+1) prefix group --
    // every text sharing those J+1 residues ends the same way --, else t + 1.
    // The steps are nested ifs (structured control flow: every exit is a
    // plain scalar or VCC branch); a per-text copy of the length that the
    // compiler cannot see through keeps the per-step tests from being hoisted
    // into registers.
    auto chain = [&](auto start_tag, auto rag_tag, const SeqRec& rec, uint32_t t, uint32_t VP, uint32_t VN,
                     uint32_t& Z) __attribute__((always_inline)) {
      constexpr int kStart = decltype(start_tag)::value;
      constexpr bool kRagged = decltype(rag_tag)::value;
      uint32_t nn = n;
      asm volatile("" : "+s"(nn));
      uint32_t ex = 32, tn = t + 1;
      bool alive = true;
      uint32_t mj = m_item << kStart;
#define TCR_OPEN(J)                                                            \
  if ((J) < kStart || (uint32_t)(J) < nn) {                                    \
    if constexpr ((J) >= kStart) {                                             \
      TCR_STEP(rec, J, mj)                                                     \
      mj = twice(mj);                                                          \
    }                                                                          \
    if ((J) < kStart || alive) {
#define TCR_CLOSE(J)                                                           \
    } else {                                                                   \
      ex = (J);                                                                \
      if constexpr ((J) < kSkipDepths && !kRagged) tn = max(rec.nxt[(J)], t + 1); \
    }                                                                          \
  }
      TCR_OPEN(0) TCR_OPEN(1) TCR_OPEN(2) TCR_OPEN(3) TCR_OPEN(4) TCR_OPEN(5) TCR_OPEN(6) TCR_OPEN(7)
      TCR_OPEN(8) TCR_OPEN(9) TCR_OPEN(10) TCR_OPEN(11) TCR_OPEN(12) TCR_OPEN(13) TCR_OPEN(14)
      TCR_OPEN(15) TCR_OPEN(16) TCR_OPEN(17) TCR_OPEN(18) TCR_OPEN(19) TCR_OPEN(20) TCR_OPEN(21)
      TCR_OPEN(22) TCR_OPEN(23) TCR_OPEN(24) TCR_OPEN(25) TCR_OPEN(26) TCR_OPEN(27) TCR_OPEN(28)
      TCR_OPEN(29) TCR_OPEN(30) TCR_OPEN(31)
      TCR_CLOSE(31) TCR_CLOSE(30) TCR_CLOSE(29) TCR_CLOSE(28) TCR_CLOSE(27) TCR_CLOSE(26)
      TCR_CLOSE(25) TCR_CLOSE(24) TCR_CLOSE(23) TCR_CLOSE(22) TCR_CLOSE(21) TCR_CLOSE(20)
      TCR_CLOSE(19) TCR_CLOSE(18) TCR_CLOSE(17) TCR_CLOSE(16) TCR_CLOSE(15) TCR_CLOSE(14)
      TCR_CLOSE(13) TCR_CLOSE(12) TCR_CLOSE(11) TCR_CLOSE(10) TCR_CLOSE(9) TCR_CLOSE(8)
      TCR_CLOSE(7) TCR_CLOSE(6) TCR_CLOSE(5) TCR_CLOSE(4) TCR_CLOSE(3) TCR_CLOSE(2) TCR_CLOSE(1)
      TCR_CLOSE(0)
#undef TCR_OPEN
#undef TCR_CLOSE
      return uint2{ex, tn};
    };

    // Texts of [t, t_end), all sharing their first kLoopDepth residues, one at
    // a time from the shared state after those residues.
    auto leaf = [&](uint32_t sVP, uint32_t sVN, uint32_t sZ, uint32_t t, uint32_t t_end)
                    __attribute__((always_inline)) {
      SeqRec rec = rec_at(t);
      for (;;) {
        uint32_t Z = sZ;
        const uint2 x = chain(Tag<kLoopDepth>{}, Tag<false>{}, rec, t, sVP, sVN, Z);
        if (x.x == 32) emit(Z, t, t + 1);
        const uint32_t tn = x.y;
        if (tn >= t_end) break;
        t = tn;
        rec = rec_at(t);
        if constexpr (kCount) ++n_visits;
      }
    };

    // The walk is a depth-first search over the implicit prefix tree of the
    // item's sorted texts.  Level D holds the state after D residues shared by
    // every text of [t, g_end) and iterates the level's sibling groups (texts
    // sharing D+1 residues; the group of t ends at nxt[D]): one text step on
    // the group's residue D; when no lane is within k the whole group is
    // skipped, otherwise the walk descends into it (or, with D+1 = n, the
    // group is a run of identical texts that all take the lanes' edges).
    //
    // Positions here are byte offsets into the walk arrays (8 * sorted
    // position): t8 is the group's first text, g_end8 the end of the range.
    auto level = [&](auto self, auto depth_tag, uint32_t pVP, uint32_t pVN, uint32_t pZ, uint32_t t8,
                     uint32_t g_end8) __attribute__((always_inline)) -> void {
      constexpr int D = decltype(depth_tag)::value;
      // the diagonal row of step D, kept in a VGPR (scalar registers are the
      // scarce ones across the nested loops)
      uint32_t mj = m_item << D;
      asm volatile("" : "+v"(mj));
      const WalkEnt* walk = d.twalk + (uint64_t)D * d.tw_len;  // this depth's walk array
      auto ent_at = [&](uint32_t u8) { return load_const_at<uint2>(walk, u8); };
      uint2 rec = ent_at(t8);  // the first group's text (the parent's current one)
      for (;;) {
        const uint32_t code = rec.y;
        // end of t's group (> t), opaque to the compiler so that the loop's
        // exit test reads it rather than the entry's own end: the entry is
        // then dead here and the next one loads into its registers
        uint32_t tn8 = min(rec.x, g_end8);
        asm volatile("" : "+s"(tn8));
        // the group's Eq row is read before the next entry is requested
        // (the barrier keeps the load after it), so the residue code needs
        // no copy out of the registers the load overwrites; these two save a
        // third of the loops' scalar moves (N = 800,000: 1.43 -> 1.39 ms)
        const uint32_t eq_c = TCR_EQ(code);
        if constexpr (!kPeqLds) asm volatile("" : : "v"(eq_c) : "memory");
        // the next group's entry is requested now (the array has an entry
        // at the end of every range), so that its latency overlaps this
        // group's step (requesting the next depth's entry as well, for a
        // descent, was slower: 1.47 -> 1.54 ms at 800,000 sequences)
        rec = ent_at(tn8);
        uint32_t VP = pVP, VN = pVN, Z = pZ;
        bool alive;
        TCR_STEP_EQV(eq_c, mj)
        if (alive) {
          // a per-iteration copy of n the compiler cannot see through: the
          // test is one compare here instead of a mask held per level
          uint32_t nn = n;
          asm volatile("" : "+s"(nn));
          if (nn == (uint32_t)D + 1u) {
            emit(Z, t8 >> 3, tn8 >> 3);
          } else if constexpr (D + 1 < kLoopDepth) {
            self(self, Tag<D + 1>{}, VP, VN, Z, t8, tn8);
          } else {
            leaf(VP, VN, Z, t8 >> 3, tn8 >> 3);
          }
        }
        if (tn8 >= g_end8) break;
        t8 = tn8;
        if constexpr (kCount) ++n_visits;
      }
    };

    uint32_t t = tb;
    if (d.tri) {
      // the ragged texts of a triangle item: patterns at or after the text
      // are masked, so neither jumps nor shared state apply
      const uint32_t rend = min(te, tri_end);
      for (; t < rend; ++t) {
        const SeqRec rec = rec_at(t);
        if constexpr (kCount) ++n_visits;
        const uint32_t dt = t - gbase;
        uint32_t Z = z_item;
        if constexpr (kTwo) {
          if (lane >= dt) Z |= 0xFFFFu;
          if (lane + kWave >= dt) Z |= 0xFFFF0000u;
        } else {
          if (lane >= dt) Z = ~0u;
        }
        const uint2 x = chain(Tag<0>{}, Tag<true>{}, rec, t, Mm, 0u, Z);
        if (x.x == 32) emit(Z, t, t + 1);
      }
    }
    if (t < te) {
      if constexpr (kCount) ++n_visits;
      level(level, Tag<0>{}, Mm, 0u, z_item, 8u * t, 8u * te);
    }
    if (kPeqLds) __builtin_amdgcn_wave_barrier();
#undef TCR_STEP
#undef TCR_STEP_CODE
#undef TCR_STEP_EQV
#undef TCR_EQ
#undef TCR_CODE
  };

  // a wave starts on a stripe of its own XCD (workgroups are dealt to the
  // XCDs round-robin) when items go to XCDs in blocks, else the four waves of
  // a workgroup start on four different stripes; a wave moves on when its
  // stripe runs dry and stops after finding every stripe empty in a row
  const uint32_t qlog = queue_block_log2(total);
  uint32_t stripe = qlog ? 2u * (blockIdx.x % (uint32_t)kXcds) + (rfl(wid) & 1u)
                         : (blockIdx.x * (kBlock / kWave) + rfl(wid)) % kQueueStripes;
  uint32_t empty = 0;
  uint32_t dcache = 0;  // descriptor of the wave's previous item
  for (;;) {
    uint64_t j = 0;
    if (lane == 0) j = atomicAdd(&cnt->queue[stripe].next, 1ull);
    j = rfl64(j);
    const uint64_t item = queue_item(stripe, j, qlog);
    if (item >= total) {
      if (++empty == (uint32_t)kQueueStripes) break;
      stripe = (stripe + 1) % kQueueStripes;
      continue;
    }
    empty = 0;

    // descriptor holding this item: largest di with item_base[di] <= item
    // (usually the previous item's; otherwise a binary search)
    uint32_t lo = dcache;
    if (!(item_base[lo] <= item && (lo + 1 >= nd || item < item_base[lo + 1]))) {
      lo = 0;
      uint32_t hi = nd;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (item_base[mid] <= item) lo = mid; else hi = mid;
      }
      dcache = lo;
    }
    const Desc d = descs[lo];
    // items of a descriptor run chunk-major: waves that take consecutive
    // items walk the same text chunk (its walk arrays stay in cache)
    const uint32_t local = (uint32_t)(item - d.item_base);
    const uint32_t groups = (d.np + 64u * d.pack - 1u) >> (d.pack == 2 ? 7u : 6u);
    const uint32_t c = local / groups;
    const uint32_t g = local - c * groups;
    if (d.pack == 2) {
      if (d.m <= 15u) run_item(Tag<3>{}, d, g, c);
      else run_item(Tag<2>{}, d, g, c);
    } else {
      run_item(Tag<1>{}, d, g, c);
    }
  }
  if (staged) flush();
  if constexpr (kCount) {
    if (lane == 0) {
      atomicAdd(&cnt->visits, (unsigned long long)n_visits);
      atomicAdd(&cnt->steps, (unsigned long long)n_steps);
      atomicAdd(&cnt->steps_packed, (unsigned long long)n_steps_packed);
    }
  }
}

}  // namespace

uint32_t pair_grid_blocks(int device, uint32_t waves_per_simd) {
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (waves_per_simd == 0) waves_per_simd = 8;
  // a block is 4 waves, one per SIMD of a CU
  return (uint32_t)cus * waves_per_simd;
}

void launch_pairs(const PairArgs& a, uint32_t grid_blocks, bool peq_lds, hipStream_t st) {
#define TCR_LAUNCH(LDS, MODE, COUNT)                                                                      \
  hipLaunchKernelGGL((k_pairs<LDS, MODE, COUNT>), dim3(grid_blocks), dim3(kBlock), 0, st, a.descs, a.item_base, \
                     a.plan, a.cnt, a.edges, a.edist, a.capacity, a.k)
  const int mode = a.k == 1 ? 1 : (a.k == 2 ? 2 : 0);
  if (a.count_work) {
    // the counting variant walks exactly as the others; one mask location
    if (mode == 1) TCR_LAUNCH(false, 1, true);
    else if (mode == 2) TCR_LAUNCH(false, 2, true);
    else TCR_LAUNCH(false, 0, true);
  } else if (peq_lds) {
    if (mode == 1) TCR_LAUNCH(true, 1, false);
    else if (mode == 2) TCR_LAUNCH(true, 2, false);
    else TCR_LAUNCH(true, 0, false);
  } else {
    if (mode == 1) TCR_LAUNCH(false, 1, false);
    else if (mode == 2) TCR_LAUNCH(false, 2, false);
    else TCR_LAUNCH(false, 0, false);
  }
#undef TCR_LAUNCH
}

}  // namespace tcr
