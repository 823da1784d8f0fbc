// Stable LSD radix sort of 64-bit keys (with optional 32-bit values), 8 bits
// per pass, one kernel per pass.
//
// A counting kernel reads every key once and forms the digit histograms of
// all passes.  Each pass kernel (a grid of at most two blocks per CU, so an
// edge buffer sized far above its fill launches no idle blocks) then takes
// tiles in order from an atomic ticket, ranks its keys by digit (wave
// ballots, stable), publishes the tile's per-digit counts, and adds up the
// counts of all earlier tiles by decoupled look-back (Merrill & Garland, "Single-pass parallel prefix scan
// with decoupled look-back", 2016; its use for radix sorting is the
// "Onesweep" sort of Adinets & Merrill, 2022).  Keys are staged in LDS in
// digit order, so each digit's run of a tile leaves with consecutive stores.
//
// Forward progress: a tile only waits for tiles with smaller tickets, which
// were taken by blocks already running (a block takes its next ticket only
// when it is done with the last); tile 0 waits for nothing.  A tile
// whose first key lies past the element count takes no part (neither
// publishes nor waits), and every tile before it publishes.  The wait is
// bounded all the same: a stall past the bound sets *fault and ends the
// look-back (the output is then wrong but stays in bounds).
#include <algorithm>

#include "kernels.h"

namespace tcr {

namespace {

constexpr int kRB = 256;                    // threads per block
constexpr int kRWaves = kRB / 64;
constexpr int kRRounds = 16;                // rounds of 64 keys per wave
constexpr int kRWaveKeys = 64 * kRRounds;   // consecutive keys of one wave
constexpr int kRTile = kRB * kRRounds;      // keys per tile
constexpr int kMaxPasses = 8;               // 64-bit keys
constexpr int kTicketWords = 32;            // one ticket per pass, padded
constexpr uint64_t kFlagAgg = 1ull << 62;   // status: the tile's own count
constexpr uint64_t kFlagPre = 1ull << 63;   // status: count through this tile
constexpr uint64_t kValMask = kFlagAgg - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ uint64_t eff_n(uint64_t n, const unsigned long long* dn) {
  if (!dn) return n;
  const uint64_t v = *dn;
  return v < n ? v : n;
}

__device__ __forceinline__ uint64_t status_load(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void status_store(unsigned long long* p, uint64_t v) {
  __hip_atomic_store(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Histograms and tickets start at zero.
__global__ __launch_bounds__(kRB) void k_radix_clear(unsigned long long* __restrict__ p, uint32_t words) {
  for (uint32_t i = threadIdx.x; i < words; i += kRB) p[i] = 0;
}

// Digit counts of every pass over the tiles blockIdx.x, blockIdx.x +
// gridDim.x, ...; also clears those tiles' look-back status words.
__global__ __launch_bounds__(kRB) void k_radix_count(const uint64_t* __restrict__ key, uint64_t n_max,
                                                     const unsigned long long* __restrict__ dn, int passes,
                                                     unsigned long long* __restrict__ hist,
                                                     unsigned long long* __restrict__ status, uint64_t nb) {
  __shared__ uint32_t h[kMaxPasses][256];
  const uint32_t tid = threadIdx.x;
  const uint64_t n = eff_n(n_max, dn);
  const uint64_t tiles = (n + kRTile - 1) / kRTile;
#pragma unroll
  for (int p = 0; p < kMaxPasses; ++p) h[p][tid] = 0;
  __syncthreads();
  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    for (int p = 0; p < passes; ++p) status[((uint64_t)p * nb + tile) * 256 + tid] = 0;
    const uint64_t base = tile * kRTile;
    uint64_t kv[kRRounds];
#pragma unroll
    for (int r = 0; r < kRRounds; ++r) {
      const uint64_t idx = base + (uint64_t)r * kRB + tid;
      kv[r] = idx < n ? key[idx] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < kRRounds; ++r) {
      if (base + (uint64_t)r * kRB + tid < n)
        for (int p = 0; p < passes; ++p) atomicAdd(&h[p][(kv[r] >> (8 * p)) & 255u], 1u);
    }
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p)
    if (h[p][tid]) atomicAdd(&hist[p * 256 + tid], (unsigned long long)h[p][tid]);
}

// One pass over digit (key >> shift) & 255.  hist: this pass's global digit
// counts; ticket: this pass's tile counter; status: this pass's look-back
// words, 256 per tile.
template <bool kVal>
__global__ __launch_bounds__(kRB) void k_radix_pass(const uint64_t* __restrict__ key,
                                                    const uint32_t* __restrict__ val, uint64_t* __restrict__ okey,
                                                    uint32_t* __restrict__ oval, uint64_t n_max,
                                                    const unsigned long long* __restrict__ dn, int shift,
                                                    const unsigned long long* __restrict__ hist,
                                                    unsigned long long* __restrict__ ticket,
                                                    unsigned long long* __restrict__ status,
                                                    unsigned long long* __restrict__ fault) {
  __shared__ uint64_t s_key[kRTile];
  __shared__ uint32_t s_val[kVal ? kRTile : 1];
  __shared__ uint32_t s_wc[kRWaves][256];   // per wave and digit: running count, then offset
  __shared__ uint64_t s_scan_g[256];
  __shared__ uint32_t s_scan_t[256];
  __shared__ uint64_t s_out[256];           // output index of a digit's run = s_out[d] + tile position
  __shared__ uint32_t s_texcl[256];         // tile position of a digit's run
  __shared__ uint32_t s_id;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  const uint32_t wid = tid >> 6;
  const uint64_t n = eff_n(n_max, dn);
  // global exclusive digit offsets (the same for every tile)
  s_scan_g[tid] = hist[tid];
  __syncthreads();
  for (int s = 1; s < 256; s <<= 1) {
    const uint64_t x = tid >= (uint32_t)s ? s_scan_g[tid - s] : 0ull;
    __syncthreads();
    s_scan_g[tid] += x;
    __syncthreads();
  }
  const uint64_t gexcl = s_scan_g[tid] - hist[tid];
  // tiles in ticket order until past the end
  for (;;) {
    if (tid == 0) s_id = (uint32_t)atomicAdd(ticket, 1ull);
#pragma unroll
    for (int w = 0; w < kRWaves; ++w) s_wc[w][tid] = 0;
    __syncthreads();
    const uint32_t id = s_id;
    const uint64_t base = (uint64_t)id * kRTile;
    if (base >= n) break;  // block-uniform: this tile is past the end

    // 1. stable ranks inside each wave's run of keys
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t wbase = base + (uint64_t)wid * kRWaveKeys;
    uint64_t kv[kRRounds];
    uint32_t vv[kRRounds];
    uint32_t rk[kRRounds];
    // all of the wave's loads first, so their latencies overlap
#pragma unroll
    for (int r = 0; r < kRRounds; ++r) {
      const uint64_t idx = wbase + (uint64_t)r * 64 + lane;
      const bool ok = idx < n;
      kv[r] = ok ? key[idx] : 0ull;
      vv[r] = (kVal && ok) ? val[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRRounds; ++r) {
      const uint64_t idx = wbase + (uint64_t)r * 64 + lane;
      const bool ok = idx < n;
      const uint32_t d = (uint32_t)(kv[r] >> shift) & 255u;
      uint64_t peers = __ballot(ok);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        peers &= bit ? bb : ~bb;
      }
      const uint32_t before = ok ? s_wc[wid][d] : 0u;
      rk[r] = before + (uint32_t)__popcll(peers & lt_mask);
      if (ok && (peers & lt_mask) == 0ull) s_wc[wid][d] = before + (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // 2. thread d: wave offsets of digit d, the tile's count, publish it
    const uint32_t d = tid;
    uint32_t cnt = 0;
#pragma unroll
    for (int w = 0; w < kRWaves; ++w) {
      const uint32_t c = s_wc[w][d];
      s_wc[w][d] = cnt;
      cnt += c;
    }
    unsigned long long* my_status = status + (uint64_t)id * 256 + d;
    status_store(my_status, (id == 0 ? kFlagPre : kFlagAgg) | cnt);

    // 3. exclusive scan over digits: tile positions
    s_scan_t[d] = cnt;
    __syncthreads();
    for (int s = 1; s < 256; s <<= 1) {
      const uint32_t xt = d >= (uint32_t)s ? s_scan_t[d - s] : 0u;
      __syncthreads();
      s_scan_t[d] += xt;
      __syncthreads();
    }
    const uint32_t texcl = s_scan_t[d] - cnt;

    // 4. look-back: keys of digit d in all earlier tiles
    uint64_t prefix = 0;
    if (id > 0) {
      uint32_t spins = 0;
      for (uint32_t j = id; j > 0;) {
        --j;
        uint64_t v;
        for (;;) {
          v = status_load(status + (uint64_t)j * 256 + d);
          if (v & (kFlagAgg | kFlagPre)) break;
          if (++spins >= kSpinLimit) {
            atomicOr(fault, 1ull);
            v = kFlagPre;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        prefix += v & kValMask;
        if (v & kFlagPre) break;
      }
      status_store(my_status, kFlagPre | (prefix + cnt));
    }
    s_texcl[d] = texcl;
    s_out[d] = gexcl + prefix - texcl;
    __syncthreads();

    // 5. stage the tile in digit order, then write each digit's run
#pragma unroll
    for (int r = 0; r < kRRounds; ++r) {
      const uint64_t idx = wbase + (uint64_t)r * 64 + lane;
      if (idx < n) {
        const uint32_t dr = (uint32_t)(kv[r] >> shift) & 255u;
        const uint32_t pos = s_texcl[dr] + s_wc[wid][dr] + rk[r];
        s_key[pos] = kv[r];
        if (kVal) s_val[pos] = vv[r];
      }
    }
    __syncthreads();
    const uint32_t tn = n - base < (uint64_t)kRTile ? (uint32_t)(n - base) : (uint32_t)kRTile;
    for (uint32_t i = tid; i < tn; i += kRB) {
      const uint64_t k = s_key[i];
      const uint64_t o = s_out[(uint32_t)(k >> shift) & 255u] + i;
      okey[o] = k;
      if (kVal) oval[o] = s_val[i];
    }
    __syncthreads();  // the next tile reuses the block's LDS
  }
}

}  // namespace

uint64_t radix_tmp_words(uint64_t n) {
  const uint64_t nb = (n + kRTile - 1) / kRTile;
  return 2 * ((uint64_t)kMaxPasses * 256 + kTicketWords + (uint64_t)kMaxPasses * (nb ? nb : 1) * 256);
}

bool radix_sort(uint64_t* key, uint64_t* key_alt, uint32_t* val, uint32_t* val_alt, uint64_t n,
                const unsigned long long* d_n, int key_bits, uint32_t* tmp, unsigned long long* fault,
                hipStream_t st) {
  if (n <= 1 || key_bits <= 0) return false;
  const int passes = key_bits > 8 * kMaxPasses ? kMaxPasses : (key_bits + 7) / 8;
  const uint64_t nb = (n + kRTile - 1) / kRTile;
  unsigned long long* hist = reinterpret_cast<unsigned long long*>(tmp);
  unsigned long long* ticket = hist + kMaxPasses * 256;
  unsigned long long* status = ticket + kTicketWords;
  hipLaunchKernelGGL(k_radix_clear, dim3(1), dim3(kRB), 0, st, hist, (uint32_t)(kMaxPasses * 256 + kTicketWords));
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const uint32_t grid = (uint32_t)std::min<uint64_t>(nb, 2ull * (uint64_t)cus);
  hipLaunchKernelGGL(k_radix_count, dim3(grid), dim3(kRB), 0, st, key, n, d_n, passes, hist, status, nb);
  bool alt = false;
  for (int p = 0; p < passes; ++p) {
    const uint64_t* ki = alt ? key_alt : key;
    uint64_t* ko = alt ? key : key_alt;
    unsigned long long* sp = status + (uint64_t)p * nb * 256;
    if (val) {
      hipLaunchKernelGGL(k_radix_pass<true>, dim3(grid), dim3(kRB), 0, st, ki, alt ? val_alt : val,
                         ko, alt ? val : val_alt, n, d_n, 8 * p, hist + p * 256, ticket + p, sp, fault);
    } else {
      hipLaunchKernelGGL(k_radix_pass<false>, dim3(grid), dim3(kRB), 0, st, ki, nullptr, ko, nullptr, n,
                         d_n, 8 * p, hist + p * 256, ticket + p, sp, fault);
    }
    alt = !alt;
  }
  return alt;
}

}  // namespace tcr
