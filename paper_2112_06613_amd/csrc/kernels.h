// Launchers of the library's HIP kernels (all asynchronous on `st`).
#pragma once
#include "common.h"

namespace tcr {

// Fill n 32-bit words with v (used instead of hipMemsetAsync so that the
// sequence can be captured in a HIP graph).
void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st);

// Zero the work counters and mark "no input error".
void launch_reset_counters(Counters* c, hipStream_t st);
// Zero only the item and edge counters (keeps the input error).
void launch_reset_work(Counters* c, hipStream_t st);

// Sort keys (segment 0, length, first residues) and values 0..n-1 of
// already-encoded records (layout of launch_encode with seg_bits = 0).
void launch_record_keys(const SeqRec* rec, uint32_t n, uint64_t* key, uint32_t* val, hipStream_t st);

// Step a1: validate + encode.  Sequence i of the concatenated input is
// d_data[d_off[i] .. d_off[i+1]).  Segment of i: seg_off[s] <= i < seg_off[s+1]
// (n_seg segments; the plain build has one).  Writes rec[i] (original order),
// a sort key (segment, length, first residues) and value i; records the first
// invalid sequence in cnt->err_first / err_code.  rec[i].id = (id_base + i) | id_tag.
// seg_off may be NULL when n_seg == 1.  The key is
//   segment << (6 + 5 * nres) | length << (5 * nres) | first nres residues,
// with nres = min(8, (58 - seg_bits) / 5), so key_bits = seg_bits + 6 + 5 * nres.
int encode_key_bits(uint32_t seg_bits);
int encode_combo_shift(uint32_t seg_bits);
void launch_encode(const char* d_data, const uint64_t* d_off, uint32_t n, const uint32_t* seg_off,
                   uint32_t n_seg, uint32_t seg_bits, uint32_t id_base, uint32_t id_tag, SeqRec* rec,
                   uint64_t* key, uint32_t* val, Counters* cnt, hipStream_t st);

// Stable LSD radix sort of (key, val) pairs by key bits [0, key_bits), 8 bits a
// pass, one kernel per pass after a counting kernel.  Buffers are
// ping-ponged; returns true if the result ended in the *_alt buffers.  val may
// be NULL (keys only).  tmp must hold radix_tmp_words(n) words (8-byte
// aligned).  The element count is min(n, *d_n) when d_n is not NULL (read on
// the device, so the launch sequence needs no host sync); grids are sized for
// n.  *fault is set to nonzero if a pass stalls (an internal error).
uint64_t radix_tmp_words(uint64_t n);
bool radix_sort(uint64_t* key, uint64_t* key_alt, uint32_t* val, uint32_t* val_alt, uint64_t n,
                const unsigned long long* d_n, int key_bits, uint32_t* tmp, unsigned long long* fault,
                hipStream_t st);

// Step a2: bucket boundaries.  key holds sorted keys; combo = key >> combo_shift
// is (segment * 33 + length).  off[c] = first sorted position whose combo >= c,
// for c in [0, n_combo]; off[n_combo] = n.
void launch_bucket_bounds(const uint64_t* key, uint64_t n, int combo_shift, uint32_t n_combo,
                          uint32_t* off, hipStream_t st);

// Gather records into sorted order (val: sorted position -> record; skey:
// the sorted keys of a sort with seg_bits segment bits), fill each record's
// prefix-group ends and build each pattern's bit masks.
void launch_gather(const SeqRec* rec, const uint32_t* val, const uint64_t* skey, uint64_t n, uint32_t seg_bits,
                   SeqRec* srec, PeqRec* speq, hipStream_t st);

// Step a3: bucket-pair work plan over a list of parts (device array d_parts
// of n_parts entries, or the single inline_part when d_parts is NULL).
// Writes descs (compacted, in item order), their item_base array and the
// plan header; more than max_desc descriptors sets plan->pad = 1.
uint32_t plan_max_desc_self(uint32_t n_seg, int k, uint32_t texts_per_item, uint64_t n);
uint32_t plan_max_desc_cross(int k);
// pack: bucket pairs whose patterns have at most kPackMaxLen residues run two
// patterns per lane (groups of 128).
void launch_plan(const PlanPart* d_parts, uint32_t n_parts, const PlanPart& inline_part, int k,
                 uint32_t texts_per_item, bool pack, Desc* descs, uint64_t* item_base, uint32_t max_desc,
                 Plan* plan, hipStream_t st);

// Steps a4-a6: the pair kernel (persistent grid).
struct PairArgs {
  const Desc* descs;
  const uint64_t* item_base;
  const Plan* plan;
  Counters* cnt;
  uint32_t* edges;      // 2 * capacity words
  uint8_t* edist;       // capacity bytes: distance of each edge (NULL: not kept)
  uint64_t capacity;
  uint32_t texts_per_item;
  int32_t k;
  bool count_work = false;  // run the counting variant (Counters::visits/steps)
};
void launch_pairs(const PairArgs& a, uint32_t grid_blocks, bool peq_lds, hipStream_t st);
uint32_t pair_grid_blocks(int device, uint32_t waves_per_simd);

// Step a8: canonical keys.  mode 0: (min, max) of the ids.  mode 1: the id
// carrying kQueryTag first (tag removed).  key = (first << shift) | second,
// followed by the 5-bit distance when edist is not NULL.
// The edge count is min(E_max, *dE) (dE may be NULL).
void launch_edge_keys(const uint32_t* edges, const uint8_t* edist, uint64_t E_max, const unsigned long long* dE,
                      int mode, int shift, uint64_t* keys, hipStream_t st);
// Degrees of an insert: for each of the E pairs (i, j) add 1 to deg[i] and
// deg[j], and to counts[x - n_old] for each end x >= n_old.
void launch_insert_degrees(const uint32_t* pairs, const unsigned long long* dE, uint64_t E_max, uint32_t n_old,
                           int32_t* counts, int32_t* deg, hipStream_t st);

// Step a7: unpack sorted keys to pairs and add both ends (mode 0) or the
// first end (mode 1) to deg (NULL: no degrees).
// With dist_out != NULL the keys carry a 5-bit distance (written there).
void launch_unpack(const uint64_t* keys, uint64_t E_max, const unsigned long long* dE, int mode, int shift,
                   uint32_t* pairs, int32_t* deg, uint8_t* dist_out, hipStream_t st);

}  // namespace tcr
