// Steps a7-a8: canonical edge keys and degrees.
#include "kernels.h"

namespace tcr {

namespace {

__device__ __forceinline__ uint64_t eff_n(uint64_t n, const unsigned long long* dn) {
  if (!dn) return n;
  const uint64_t v = *dn;
  return v < n ? v : n;
}

// Grid-stride loops over the edge count read on the device: the grids are
// capped (kPostBlocks), so an edge buffer sized far above its fill launches
// no idle blocks.
constexpr uint32_t kPostBlocks = 2048;

__global__ void k_edge_keys(const uint32_t* __restrict__ edges, const uint8_t* __restrict__ edist, uint64_t E_max,
                            const unsigned long long* __restrict__ dE, int mode, int shift,
                            uint64_t* __restrict__ keys) {
  const uint64_t E = eff_n(E_max, dE);
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (uint64_t)gridDim.x * blockDim.x) {
    const uint2 p = reinterpret_cast<const uint2*>(edges)[e];
    uint32_t a, b;
    if (mode == 0) {
      a = min(p.x, p.y);
      b = max(p.x, p.y);
    } else {
      // the query-side id carries the tag; it goes first, untagged
      const bool x_is_q = (p.x & kQueryTag) != 0;
      a = (x_is_q ? p.x : p.y) & ~kQueryTag;
      b = x_is_q ? p.y : p.x;
    }
    uint64_t key = ((uint64_t)a << shift) | b;
    if (edist) key = (key << 5) | edist[e];
    keys[e] = key;
  }
}

__global__ void k_unpack(const uint64_t* __restrict__ keys, uint64_t E_max,
                         const unsigned long long* __restrict__ dE, int mode, int shift,
                         uint32_t* __restrict__ pairs, int32_t* __restrict__ deg, uint8_t* __restrict__ dist_out) {
  const uint64_t E = eff_n(E_max, dE);
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t kv = keys[e];
    if (dist_out) {
      dist_out[e] = (uint8_t)(kv & 31u);
      kv >>= 5;
    }
    const uint32_t a = (uint32_t)(kv >> shift);
    const uint32_t b = (uint32_t)(kv & ((1ull << shift) - 1ull));
    uint2 p;
    p.x = a;
    p.y = b;
    reinterpret_cast<uint2*>(pairs)[e] = p;
    if (deg) {
      // edges arrive sorted by a: one atomic per run of equal a in the wave
      const uint32_t lane = threadIdx.x & 63u;
      const uint32_t a_up = (uint32_t)__shfl_up((int)a, 1);
      const bool head = lane == 0 || a_up != a;
      const uint64_t heads = __ballot(head);
      const uint64_t valid = __ballot(true);  // lanes with e < E (the rest left the loop)
      if (head) {
        const uint64_t after = lane == 63 ? 0ull : (heads & ~((2ull << lane) - 1ull));
        const uint32_t end = after ? (uint32_t)__ffsll((long long)after) - 1u
                                   : 64u - (uint32_t)__clzll((long long)valid);
        atomicAdd(&deg[a], (int32_t)(end - lane));
      }
      if (mode == 0) atomicAdd(&deg[b], 1);
    }
  }
}

__global__ void k_insert_degrees(const uint32_t* __restrict__ pairs, const unsigned long long* __restrict__ dE,
                                 uint64_t E_max, uint32_t n_old, int32_t* __restrict__ counts,
                                 int32_t* __restrict__ deg) {
  const uint64_t E = eff_n(E_max, dE);
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (uint64_t)gridDim.x * blockDim.x) {
    const uint2 p = reinterpret_cast<const uint2*>(pairs)[e];
    atomicAdd(&deg[p.x], 1);
    atomicAdd(&deg[p.y], 1);
    if (p.x >= n_old) atomicAdd(&counts[p.x - n_old], 1);
    if (p.y >= n_old) atomicAdd(&counts[p.y - n_old], 1);
  }
}

inline uint32_t post_blocks(uint64_t E_max) {
  const uint64_t b = (E_max + 255) / 256;
  return (uint32_t)(b < kPostBlocks ? b : kPostBlocks);
}

}  // namespace

void launch_insert_degrees(const uint32_t* pairs, const unsigned long long* dE, uint64_t E_max, uint32_t n_old,
                           int32_t* counts, int32_t* deg, hipStream_t st) {
  if (E_max == 0) return;
  hipLaunchKernelGGL(k_insert_degrees, dim3(post_blocks(E_max)), dim3(256), 0, st, pairs, dE, E_max,
                     n_old, counts, deg);
}

void launch_edge_keys(const uint32_t* edges, const uint8_t* edist, uint64_t E_max, const unsigned long long* dE,
                      int mode, int shift, uint64_t* keys, hipStream_t st) {
  if (E_max == 0) return;
  hipLaunchKernelGGL(k_edge_keys, dim3(post_blocks(E_max)), dim3(256), 0, st, edges, edist, E_max, dE,
                     mode, shift, keys);
}

void launch_unpack(const uint64_t* keys, uint64_t E_max, const unsigned long long* dE, int mode, int shift,
                   uint32_t* pairs, int32_t* deg, uint8_t* dist_out, hipStream_t st) {
  if (E_max == 0) return;
  hipLaunchKernelGGL(k_unpack, dim3(post_blocks(E_max)), dim3(256), 0, st, keys, E_max, dE, mode,
                     shift, pairs, deg, dist_out);
}

}  // namespace tcr
