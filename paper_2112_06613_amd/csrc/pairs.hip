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
// text step j the cell D[r][j] on the final diagonal r = j + m - n is a lower
// bound of lev = D[m][n].  Hyyro's D0 word has bit r-1 set exactly when
// D[r][j] = D[r-1][j-1] (a zero step along the diagonal), so collecting, at
// each step, the D0 bit of the diagonal's current row into one word DG gives
//   D[r][j] = max(m - n, 0) + j - popcount(DG).
// The paper aborts once the smallest entry of a DP row exceeds l_max
// ("GPU-based network generation"); the diagonal cell is the tighter exact
// bound of the same kind.  A bound above k for every lane of a wave ends the
// wave's work on that text; no lane's answer depends on when the check runs.
//
// Layout of the work: a wave holds 64 consecutive patterns of one length
// bucket (one per lane, their Peq tables in VGPRs, or in LDS) and walks the
// texts of a chunk of another (or the same) bucket; each text is
// wave-uniform and is read with one scalar load into SGPRs.  Sequences are
// sorted by (length, residues), so the 64 patterns of a wave share prefixes
// and leave a text at nearly the same step.  Pattern = the longer string of
// the pair when lengths differ (it exits earliest).
//
// Output: lanes whose final distance is <= k are compacted with one ballot,
// one atomic add per wave, and consecutive edge slots (coalesced writes).
#include "kernels.h"

namespace tcr {

namespace {

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t rfl64(uint64_t v) {
  return ((uint64_t)rfl((uint32_t)(v >> 32)) << 32) | rfl((uint32_t)v);
}

__device__ __forceinline__ uint32_t low_mask(uint32_t r) { return r >= 32 ? ~0u : ((1u << r) - 1u); }

// (h << 1) | 1 as one funnel shift: the low 32 bits of (h:0xffffffff) >> 31.
__device__ __forceinline__ uint32_t shl1_or1(uint32_t h) { return __builtin_amdgcn_alignbit(h, 0xffffffffu, 31); }

// Loads through address-space views of descriptor pointers: the wave-uniform
// text records are read-only for the whole launch, so they are read through
// the constant address space (scalar loads into SGPRs); pattern data through
// the global one.  (The host compilation pass only parses kernel bodies.)
template <class T>
__device__ __forceinline__ T load_const(const T* p, uint32_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  const __attribute__((address_space(4))) T* q = (const __attribute__((address_space(4))) T*)p;
  T v;
  __builtin_memcpy(&v, (const T*)(q + i), sizeof(T));
  return v;
#else
  return p[i];
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

template <bool kPeqLds>
__global__ __launch_bounds__(kBlock) void k_pairs(const Desc* __restrict__ descs,
                                                  const uint64_t* __restrict__ item_base,
                                                  const Plan* __restrict__ plan, Counters* __restrict__ cnt,
                                                  uint32_t* __restrict__ edges, uint8_t* __restrict__ edist,
                                                  uint64_t capacity,
                                                  uint32_t T, int k) {
  __shared__ uint32_t lds_eq[kPeqLds ? (kBlock / kWave) * kAlpha * kWave : 1];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wid = threadIdx.x >> 6;
  const uint64_t total = plan->total_items;
  const uint32_t nd = plan->n_desc;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint32_t* wave_eq = lds_eq + (kPeqLds ? wid * kAlpha * kWave : 0);

  for (;;) {
    uint64_t item = 0;
    if (lane == 0) item = atomicAdd(&cnt->item_next, 1ull);
    item = rfl64(item);
    if (item >= total) break;

    // descriptor holding this item: largest di with item_base[di] <= item
    uint32_t lo = 0, hi = nd;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (item_base[mid] <= item) lo = mid; else hi = mid;
    }
    const Desc d = descs[lo];
    const SeqRec* prec = d.prec;
    const PeqRec* ppeq = d.ppeq;
    const SeqRec* trec = d.trec;
    const uint32_t local = (uint32_t)(item - d.item_base);
    const uint32_t g = local / d.chunks;
    const uint32_t c = local - g * d.chunks;
    const uint32_t gbase = d.p0 + g * kWave;
    const bool lane_ok = g * kWave + lane < d.np;
    const uint32_t p = lane_ok ? gbase + lane : d.p0;
    const uint64_t lane_mask = __ballot(lane_ok);

    uint32_t eq[kAlpha];
    {
      const PeqRec pr = load_global(ppeq, p);
#pragma unroll
      for (int a = 0; a < kAlpha; ++a) eq[a] = pr.eq[a];
    }
    if (kPeqLds) {
#pragma unroll
      for (int a = 0; a < kAlpha; ++a) wave_eq[a * kWave + lane] = eq[a];
      __builtin_amdgcn_wave_barrier();
    }
    const uint32_t pid = load_global(prec, p).id;

    const uint32_t m = d.m, n = d.n;
    const uint32_t Mm = low_mask(m);
    const int delta = (int)m - (int)n;    // final diagonal: row = column + delta
    const int dpos = delta > 0 ? delta : 0;
    const uint32_t diag0 = delta >= 0 ? (1u << delta) : 0u;  // diagonal row of text step 1
    uint32_t tb = d.t0 + c * T;
    const uint32_t te = min(d.t0 + d.nt, tb + T);
    if (d.tri && tb < gbase + 1) tb = gbase + 1;

    // the next text's record is loaded one text ahead (scalar loads overlap
    // the current text's steps)
    SeqRec nxt = load_const(trec, tb < te ? tb : 0u);
    for (uint32_t t = tb; t < te; ++t) {
      const SeqRec tr = nxt;
      if (t + 1 < te) nxt = load_const(trec, t + 1);
      uint64_t valid = lane_mask;
      if (d.tri) {
        const uint32_t lim = t - gbase;  // lanes with pattern < text
        if (lim < 64) valid &= (1ull << lim) - 1ull;
      }

#define TCR_EQ(cc) (kPeqLds ? wave_eq[(cc) * kWave + lane] : eq[(cc)])
#define TCR_CODE(q) ((tr.w[(q) / 6] >> (5 * ((q) % 6))) & 31u)
// One text step for character J (0-based, J >= 1), then the exit test on the
// final diagonal once it has entered the table (r >= 1).
#define TCR_STEP(J)                                                          \
  {                                                                          \
    if ((uint32_t)(J) >= n) goto final_check;                                \
    const uint32_t Eq = TCR_EQ(TCR_CODE(J));                                 \
    const uint32_t D0 = (((Eq & VP) + VP) ^ VP) | Eq | VN;                   \
    const uint32_t HP = VN | ~(D0 | VP);                                     \
    const uint32_t HN = D0 & VP;                                             \
    const uint32_t X = shl1_or1(HP);                                         \
    VN = X & D0;                                                             \
    VP = (HN << 1) | ~(X | D0);                                              \
    /* the final diagonal is at row r = J + 1 + delta (bit J + delta) */     \
    const int bit = (J) + delta;                                             \
    if (bit >= 0) {                                                          \
      DG |= D0 & (1u << bit);                                                \
      /* D[r][J+1] <= k  <=>  popcount(DG) >= J + 1 + max(delta,0) - k */   \
      const int thr = (J) + 1 + dpos - k;                                    \
      if (thr > 0 &&                                                         \
          (__ballot((uint32_t)__popc(DG) >= (uint32_t)thr) & valid) == 0ull) \
        goto next_text;                                                      \
    }                                                                        \
  }

      // text step for character 0, from VP = 1^m, VN = 0 (then Eq & VP = Eq)
      uint32_t VP, VN, DG = 0;
      {
        const uint32_t Eq = TCR_EQ(TCR_CODE(0));
        const uint32_t D0 = ((Eq + Mm) ^ Mm) | Eq;
        const uint32_t HP = ~(D0 | Mm);
        const uint32_t HN = D0 & Mm;
        const uint32_t X = shl1_or1(HP);
        VN = X & D0;
        VP = (HN << 1) | ~(X | D0);
        DG = D0 & diag0;
      }
      TCR_STEP(1) TCR_STEP(2) TCR_STEP(3) TCR_STEP(4) TCR_STEP(5) TCR_STEP(6) TCR_STEP(7)
      TCR_STEP(8) TCR_STEP(9) TCR_STEP(10) TCR_STEP(11) TCR_STEP(12) TCR_STEP(13) TCR_STEP(14)
      TCR_STEP(15) TCR_STEP(16) TCR_STEP(17) TCR_STEP(18) TCR_STEP(19) TCR_STEP(20) TCR_STEP(21)
      TCR_STEP(22) TCR_STEP(23) TCR_STEP(24) TCR_STEP(25) TCR_STEP(26) TCR_STEP(27) TCR_STEP(28)
      TCR_STEP(29) TCR_STEP(30) TCR_STEP(31)
    final_check : {
      const int dist = (int)n + __popc(VP & Mm) - __popc(VN & Mm);
      const bool hit = ((valid >> lane) & 1ull) && dist <= k;
      const uint64_t hm = __ballot(hit);
      if (hm) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&cnt->edges, (unsigned long long)__popcll(hm));
        base = rfl64(base);
        if (hit) {
          const uint64_t slot = base + (uint64_t)__popcll(hm & lt_mask);
          if (slot < capacity) {
            uint2 e;
            e.x = pid;
            e.y = tr.id;
            *reinterpret_cast<uint2*>(edges + 2 * slot) = e;
            if (edist) edist[slot] = (uint8_t)dist;
          }
        }
      }
    }
    next_text:;
#undef TCR_STEP
#undef TCR_EQ
#undef TCR_CODE
    }
    if (kPeqLds) __builtin_amdgcn_wave_barrier();
  }
}

}  // namespace

uint32_t pair_grid_blocks(int device, uint32_t waves_per_simd) {
  int cus = 256;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (waves_per_simd == 0) waves_per_simd = 8;
  // a block is 4 waves, one per SIMD of a CU
  return (uint32_t)cus * waves_per_simd;
}

void launch_pairs(const PairArgs& a, uint32_t grid_blocks, bool peq_lds, hipStream_t st) {
  if (peq_lds)
    hipLaunchKernelGGL(k_pairs<true>, dim3(grid_blocks), dim3(kBlock), 0, st, a.descs, a.item_base, a.plan,
                       a.cnt, a.edges, a.edist, a.capacity, a.texts_per_item, a.k);
  else
    hipLaunchKernelGGL(k_pairs<false>, dim3(grid_blocks), dim3(kBlock), 0, st, a.descs, a.item_base, a.plan,
                       a.cnt, a.edges, a.edist, a.capacity, a.texts_per_item, a.k);
}

}  // namespace tcr
