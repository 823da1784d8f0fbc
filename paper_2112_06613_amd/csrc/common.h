// Internal definitions shared by the library's host and device code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tcr {

constexpr int kMaxLen = 32;      // one 32-bit bit-vector word per pattern
constexpr int kAlpha = 20;       // amino-acid alphabet size
constexpr int kWave = 64;        // CDNA wavefront
constexpr int kBlock = 256;      // threads per block of the pair kernel (4 waves)
constexpr uint32_t kQueryTag = 0x80000000u;  // id bit marking the query side

constexpr int kSkipDepths = 8;   // prefix depths with a group-end pointer
constexpr uint32_t kPackMaxLen = 16;  // patterns this short go two to a lane
constexpr uint32_t kLenMask = 63u;  // length bits of SeqRec::len

// One sequence as the pair kernel reads it (64 bytes, read with one scalar
// load when the sequence is the wave-uniform text).
//   w[0..5]: 5-bit residue codes, 6 per word, code q in w[q/6] bits 5*(q%6)
//   len:     bits 0-5: number of residues (1..32); in sorted records also
//            bits 6-9: common prefix length (capped at 8) with the next
//            sorted record, and for d = 2..8 bits 10+3(d-2) .. +2: common
//            prefix length with nxt[d-1] (below d)
//   id:      caller-visible node id (input position; in query mode the query
//            side carries kQueryTag)
//   nxt[d-1] (sorted records only): the first sorted position after this one
//            whose (segment, length, first d residues) differ -- the end of
//            this sequence's depth-d prefix group; the position + 1 when the
//            sort key holds fewer than d residues.
struct alignas(64) SeqRec {
  uint32_t w[6];
  uint32_t len;
  uint32_t id;
  uint32_t nxt[kSkipDepths];
};

static_assert(sizeof(SeqRec) == 64, "one record = one 64-byte line");

// What the pair kernel's prefix-tree walk reads of a text at its first
// kWalkDepth residues: one dense array per depth d (8 bytes a text, eight to
// a 64-byte scalar-cache line), entry s = {8 * (end of s's depth-(d+1)
// prefix group), code of residue d}; the group end is a byte offset into the
// same array, so the walk moves through it with no index arithmetic.  Each
// array has one more entry than the set (a valid read one past the end).
constexpr int kWalkDepth = 6;
struct WalkEnt {
  uint32_t end8;  // 8 * group end (a sorted position <= n)
  uint32_t code;  // residue d of the text (0..19)
};
static_assert(sizeof(WalkEnt) == 8, "eight walk entries to a 64-byte line");

// A sorted sequence set's record buffer holds its n SeqRec, then the
// kWalkDepth walk arrays of n + 1 entries each.
__host__ __device__ inline const WalkEnt* walk_of(const SeqRec* srec, uint32_t n) {
  return reinterpret_cast<const WalkEnt*>(srec + n);
}
__host__ __device__ inline uint64_t sorted_rec_bytes(uint64_t n) {
  return n * sizeof(SeqRec) + (uint64_t)kWalkDepth * (n + 1) * sizeof(WalkEnt);
}

// The residue codes of one pattern as bit planes: bit q of pl[b] is bit b of
// residue q's code (positions past the length hold code 0).  Myers' Peq
// table follows from them: eq[c] = AND over b of (pl[b] or its complement, as
// bit b of c is 1 or 0), restricted to the length.  20 bytes: a work item's
// patterns are read as planes and their tables built in registers.
struct PeqRec {
  uint32_t pl[5];
};

// One pair of length buckets (pattern bucket of length m, text bucket of
// length n): a rectangle of work items, or an upper triangle when both are the
// same bucket of the same segment.  Items are (pattern group of 64, chunk of
// texts_per_item texts), numbered group-major.  The descriptor names the
// sequence sets its patterns and texts come from, so one launch can cover
// several sets (a query batch against a repertoire and its inserted parts).
struct alignas(16) Desc {
  const SeqRec* prec;    // pattern-side records (lane side)
  const PeqRec* ppeq;    // pattern-side bit masks
  const SeqRec* trec;    // text-side records (wave-uniform side)
  const WalkEnt* twalk;  // text-side walk arrays (depth 0; depth d at + d * tw_len)
  uint32_t tw_len;       // entries of one walk array (text set size + 1)
  uint32_t p0, np;       // pattern range (sorted positions in prec)
  uint32_t t0, nt;       // text range (sorted positions in trec)
  uint32_t m, n;         // lengths
  uint32_t tri;          // 1: pairs (p, t) with p < t only
  uint32_t chunks;       // ceil(nt / texts_per_item)
  uint32_t pack;         // patterns per lane: 2 (m <= kPackMaxLen) or 1;
                         // a group is 64 * pack patterns
  uint32_t T;            // texts per chunk
  uint64_t item_base;    // first item of this descriptor
  uint64_t items;        // groups * chunks
};

// A sorted, length-bucketed sequence set: records and masks in sorted order
// and its bucket table off[seg * 64 + L] (n_seg segments, n_seg * 64 + 1
// entries): bucket (seg, L) = [off[seg*64+L], off[seg*64+L+1]).
struct SetRef {
  const SeqRec* srec;
  const PeqRec* speq;
  const uint32_t* off;
  uint32_t n_seg;
  uint32_t pad;
};

// One part of a work plan.  self (cross == 0): all pairs inside each segment
// of set a, lengths at most k apart.  cross: all pairs between set a (one
// segment) and set b (one segment), lengths at most k apart; when the lengths
// are equal, the set with fewer sequences of that length supplies the
// patterns when it has at least 64 of them, else the other (a when the
// counts are equal).
struct PlanPart {
  SetRef a;
  SetRef b;
  uint32_t cross;
  uint32_t pad;
};

// Per-launch plan header written by the planning kernel.
struct Plan {
  uint64_t total_items;
  uint64_t evaluated_pairs;
  uint32_t n_desc;
  uint32_t pad;
};

// Work counters of one build (zeroed before the encode kernel).  Every wave
// takes work items with atomics, so the queue is split into kQueueStripes
// counters, each on a cache line of its own, and the edge counter sits on
// another: the atomics of thousands of waves do not serialise on one line.
// The items are dealt out in blocks of consecutive items (which mostly share
// one chunk of texts), block b to XCD b mod kXcds; the XCD's two stripes take
// alternate items of its blocks in increasing order.  A chunk's texts are
// then read by the waves of one XCD, from its own L2, and every XCD still
// works through the plan's order (largest items first).  The block is the
// largest power of two from 256 to 1,024 items that leaves every XCD at least
// 32 blocks (a short tail); launches of fewer than 65,536 items, whose texts
// fit the L2s anyway, take blocks of one item (plain striping: stripe s hands
// out items 16j + 8(s mod 2) + s/2).
constexpr int kXcds = 8;  // MI355X: 8 XCDs of 32 CUs, workgroups dealt round-robin
constexpr int kQueueStripes = 2 * kXcds;
__host__ __device__ inline uint32_t queue_block_log2(uint64_t total_items) {
  if (total_items < (1u << 16)) return 0;
  uint32_t l = 8;
  while (l < 10 && (total_items >> (l + 1)) >= 32u * kXcds) ++l;
  return l;
}
__host__ __device__ inline uint64_t queue_item(uint32_t stripe, uint64_t j, uint32_t block_log2) {
  const uint64_t jj = 2 * j + (stripe & 1u);  // the XCD's jj-th item
  const uint64_t mask = (1ull << block_log2) - 1ull;
  return ((((jj >> block_log2) * kXcds) + stripe / 2) << block_log2) + (jj & mask);
}
struct alignas(128) QueueLine {
  unsigned long long next;        // next index j of this stripe
  unsigned long long pad[15];
};
struct alignas(256) Counters {
  QueueLine queue[kQueueStripes];
  unsigned long long edges;       // edges found (may exceed the capacity)
  unsigned long long err;         // min over bad inputs of (index << 2 | code),
                                  // code 1: residue outside the alphabet,
                                  // code 2: length 0 or > 32; ~0: none
  unsigned long long fault;       // nonzero: a device sort pass stalled
  // work of the pair kernel's counting variant: visited texts, wave text
  // steps, and the steps with two patterns per lane among them
  unsigned long long visits, steps, steps_packed;
  unsigned long long pad1[10];
};
constexpr unsigned long long kNoError = ~0ull;

}  // namespace tcr
