// Stable LSD radix sort of 64-bit keys (with optional 32-bit values), 8 bits
// per pass: per-block digit histograms, one exclusive scan over
// (digit, block), and a stable scatter that ranks equal digits inside each
// wave with ballots.
#include "kernels.h"

namespace tcr {

namespace {

constexpr int kRB = 256;                 // threads per block
constexpr int kRItems = 16;              // keys per thread per tile
constexpr int kRTile = kRB * kRItems;    // keys per block
constexpr int kScanThreads = 1024;

__device__ __forceinline__ uint64_t eff_n(uint64_t n, const unsigned long long* dn) {
  if (!dn) return n;
  const uint64_t v = *dn;
  return v < n ? v : n;
}

__global__ __launch_bounds__(kRB) void k_radix_hist(const uint64_t* __restrict__ key, uint64_t n_max,
                                                    const unsigned long long* __restrict__ dn, int shift,
                                                    uint32_t* __restrict__ hist, uint32_t nblocks) {
  __shared__ uint32_t h[256];
  const uint64_t n = eff_n(n_max, dn);
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kRTile;
  for (int i = threadIdx.x; i < kRTile; i += kRB) {
    const uint64_t idx = base + i;
    if (idx < n) atomicAdd(&h[(key[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `total` counts in place, one block.
__global__ __launch_bounds__(kScanThreads) void k_radix_scan(uint32_t* __restrict__ hist, uint64_t total) {
  __shared__ uint32_t sums[kScanThreads];
  const uint64_t per = (total + kScanThreads - 1) / kScanThreads;
  const uint64_t lo = per * threadIdx.x;
  const uint64_t hi = lo + per < total ? lo + per : total;
  uint32_t s = 0;
  for (uint64_t i = lo; i < hi; ++i) s += hist[i];
  sums[threadIdx.x] = s;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    uint32_t x = threadIdx.x >= (unsigned)d ? sums[threadIdx.x - d] : 0;
    __syncthreads();
    sums[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = sums[threadIdx.x] - s;
  for (uint64_t i = lo; i < hi; ++i) {
    const uint32_t v = hist[i];
    hist[i] = run;
    run += v;
  }
}

// Large scans in three passes: chunk sums, a scan of the sums, then each
// chunk rescanned from its offset.  kScanChunk entries per block.
constexpr int kScanChunk = 4096;

__device__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t* sh, uint32_t& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < kRB; d <<= 1) {
    const uint32_t x = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  total = sh[kRB - 1];
  const uint32_t r = sh[t] - v;
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kRB) void k_scan_partials(const uint32_t* __restrict__ a, uint64_t total,
                                                       uint32_t* __restrict__ partial) {
  __shared__ uint32_t sh[kRB];
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk;
  uint32_t s = 0;
  for (int i = threadIdx.x; i < kScanChunk; i += kRB) {
    const uint64_t idx = base + i;
    if (idx < total) s += a[idx];
  }
  uint32_t tot;
  block_excl_scan_u32(s, sh, tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kRB) void k_scan_chunks(uint32_t* __restrict__ a, uint64_t total,
                                                     const uint32_t* __restrict__ partial_excl) {
  __shared__ uint32_t sh[kRB];
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk;
  // each thread owns kScanChunk / kRB consecutive entries
  constexpr int per = kScanChunk / kRB;
  const uint64_t lo = base + (uint64_t)threadIdx.x * per;
  uint32_t v[per];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    v[i] = lo + i < total ? a[lo + i] : 0u;
    s += v[i];
  }
  uint32_t tot;
  uint32_t run = partial_excl[blockIdx.x] + block_excl_scan_u32(s, sh, tot);
#pragma unroll
  for (int i = 0; i < per; ++i) {
    if (lo + i < total) a[lo + i] = run;
    run += v[i];
  }
}

__global__ __launch_bounds__(kRB) void k_radix_scatter(const uint64_t* __restrict__ key,
                                                       const uint32_t* __restrict__ val,
                                                       uint64_t* __restrict__ okey, uint32_t* __restrict__ oval,
                                                       uint64_t n_max, const unsigned long long* __restrict__ dn,
                                                       int shift, const uint32_t* __restrict__ offs,
                                                       uint32_t nblocks) {
  __shared__ uint32_t run[256];
  const uint64_t n = eff_n(n_max, dn);
  __shared__ uint32_t wcnt[kRB / 64][256];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  run[tid] = offs[(uint64_t)tid * nblocks + blockIdx.x];
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint64_t base = (uint64_t)blockIdx.x * kRTile;
  for (int it = 0; it < kRItems; ++it) {
    const uint64_t idx = base + (uint64_t)it * kRB + tid;
    const bool ok = idx < n;
    const uint64_t kv = ok ? key[idx] : 0;
    const uint32_t d = (uint32_t)(kv >> shift) & 255u;
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
#pragma unroll
    for (int w = 0; w < kRB / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    if (ok && rank == 0) wcnt[wid][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      uint32_t r = run[tid];
#pragma unroll
      for (int w = 0; w < kRB / 64; ++w) {
        const uint32_t c = wcnt[w][tid];
        wcnt[w][tid] = r;
        r += c;
      }
      run[tid] = r;
    }
    __syncthreads();
    if (ok) {
      const uint32_t pos = wcnt[wid][d] + rank;
      okey[pos] = kv;
      if (val) oval[pos] = val[idx];
    }
    __syncthreads();
  }
}

}  // namespace

uint64_t radix_tmp_words(uint64_t n) {
  const uint64_t nb = (n + kRTile - 1) / kRTile;
  const uint64_t hist = 256 * (nb ? nb : 1);
  return hist + (hist + kScanChunk - 1) / kScanChunk + 1;  // histogram + chunk sums
}

// Exclusive scan of `total` words in place (partial: scratch of
// ceil(total / kScanChunk) words).
static void scan_u32(uint32_t* a, uint64_t total, uint32_t* partial, hipStream_t st) {
  const uint64_t chunks = (total + kScanChunk - 1) / kScanChunk;
  if (chunks <= 8) {
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(kScanThreads), 0, st, a, total);
    return;
  }
  hipLaunchKernelGGL(k_scan_partials, dim3((uint32_t)chunks), dim3(kRB), 0, st, a, total, partial);
  hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(kScanThreads), 0, st, partial, chunks);
  hipLaunchKernelGGL(k_scan_chunks, dim3((uint32_t)chunks), dim3(kRB), 0, st, a, total, partial);
}

bool radix_sort(uint64_t* key, uint64_t* key_alt, uint32_t* val, uint32_t* val_alt, uint64_t n,
                const unsigned long long* d_n, int key_bits, uint32_t* tmp, hipStream_t st) {
  if (n <= 1 || key_bits <= 0) return false;
  const uint32_t nb = (uint32_t)((n + kRTile - 1) / kRTile);
  bool alt = false;
  for (int shift = 0; shift < key_bits; shift += 8) {
    const uint64_t* ki = alt ? key_alt : key;
    uint64_t* ko = alt ? key : key_alt;
    const uint32_t* vi = val ? (alt ? val_alt : val) : nullptr;
    uint32_t* vo = val ? (alt ? val : val_alt) : nullptr;
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kRB), 0, st, ki, n, d_n, shift, tmp, nb);
    scan_u32(tmp, (uint64_t)256 * nb, tmp + (uint64_t)256 * nb, st);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kRB), 0, st, ki, vi, ko, vo, n, d_n, shift, tmp, nb);
    alt = !alt;
  }
  return alt;
}

}  // namespace tcr
