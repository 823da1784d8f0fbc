// Network analysis on the device edge list (paper, Methods, "Overview of
// network theory concepts" and "Computing LCC"): connected components, the
// largest connected component (LCC), cluster sizes, and site percolation
// (LCC after removing a fraction of the nodes).
//
// Components: lock-free union-find over the edges.  Every edge hooks the
// larger of its two roots under the smaller with one compare-and-swap
// (retrying from the new roots when another edge won the race), so each root
// is its component's smallest node id; a final pass points every node at its
// root.  Percolation runs P independent union-finds in one launch (one
// parent array per removal count), an edge taking part in q when both of its
// ends survive the first removed[q] nodes of the caller's removal order.
#include <algorithm>

#include "graph.h"

namespace tcr {

namespace {

__device__ __forceinline__ uint32_t load_parent(const uint32_t* parent, uint32_t x) {
  return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving (every write points a node at an ancestor).
__device__ uint32_t find_root(uint32_t* parent, uint32_t x) {
  uint32_t p = load_parent(parent, x);
  while (p != x) {
    const uint32_t gp = load_parent(parent, p);
    if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = p;
    p = gp;
  }
  return x;
}

// Element loops are grid-stride: a launch covers any count with a capped grid.
#define TCR_FOR(i, count) \
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (count); i += (uint64_t)gridDim.x * blockDim.x)

__global__ void k_cc_init(uint32_t* __restrict__ parent, uint64_t total, uint32_t n) {
  TCR_FOR(i, total) parent[i] = (uint32_t)(i % n);
}

// rank[order[t]] = t: position of each node in the removal order.
__global__ void k_cc_rank(const uint32_t* __restrict__ order, uint32_t n, uint32_t* __restrict__ rank) {
  TCR_FOR(t, n) rank[order[t]] = (uint32_t)t;
}

__global__ void k_cc_hook(const uint32_t* __restrict__ pairs, uint64_t E, uint32_t n, uint32_t* __restrict__ parent,
                          const uint32_t* __restrict__ rank, const uint32_t* __restrict__ removed, uint32_t P) {
  TCR_FOR(w, E * P) {
    const uint32_t q = (uint32_t)(w / E);
    const uint64_t e = w - (uint64_t)q * E;
    uint32_t u = pairs[2 * e], v = pairs[2 * e + 1];
    if (u >= n || v >= n) continue;
    if (rank) {
      const uint32_t r = removed[q];
      if (rank[u] < r || rank[v] < r) continue;
    }
    uint32_t* par = parent + (uint64_t)q * n;
    for (;;) {
      u = find_root(par, u);
      v = find_root(par, v);
      if (u == v) break;
      if (u < v) {
        const uint32_t t = u;
        u = v;
        v = t;
      }
      // u > v: hook root u under v
      if (atomicCAS(par + u, u, v) == u) break;
    }
  }
}

// labels[i] = root of i; sizes[root] counts the alive members; comps counts
// alive roots.  One thread per (q, i).
__global__ void k_cc_finish(uint32_t* __restrict__ parent, uint32_t n, uint32_t P, const uint32_t* __restrict__ rank,
                            const uint32_t* __restrict__ removed, uint32_t* __restrict__ sizes,
                            uint32_t* __restrict__ comps) {
  TCR_FOR(w, (uint64_t)n * P) {
    const uint32_t q = (uint32_t)(w / n);
    const uint32_t i = (uint32_t)(w - (uint64_t)q * n);
    if (rank && rank[i] < removed[q]) continue;
    uint32_t* par = parent + (uint64_t)q * n;
    const uint32_t r = find_root(par, i);
    atomicAdd(&sizes[(uint64_t)q * n + r], 1u);
    if (r == i) atomicAdd(&comps[q], 1u);
  }
}

// labels from the fully compressed forest (after k_cc_finish).
__global__ void k_cc_labels(const uint32_t* __restrict__ parent, uint32_t n, uint32_t* __restrict__ labels) {
  TCR_FOR(i, n) {
    uint32_t x = (uint32_t)i;
    while (parent[x] != x) x = parent[x];
    labels[i] = x;
  }
}

// lcc[q] = max over sizes of run q.
__global__ void k_cc_max(const uint32_t* __restrict__ sizes, uint32_t n, uint32_t P, uint32_t* __restrict__ lcc) {
  TCR_FOR(w, (uint64_t)n * P) {
    const uint32_t s = sizes[w];
    if (s) atomicMax(&lcc[w / n], s);
  }
}

// ---------------------------------------------------------- degree statistics
// Input: a canonical edge list (i < j, sorted by (i, j), distinct), so the
// neighbours j > i of node i are the contiguous run pairs[row[i] .. row[i+1]).

__global__ void k_deg(const uint32_t* __restrict__ pairs, uint64_t E, uint32_t* __restrict__ deg) {
  TCR_FOR(e, E) {
    atomicAdd(&deg[pairs[2 * e]], 1u);
    atomicAdd(&deg[pairs[2 * e + 1]], 1u);
  }
}

// row[i] = first edge whose first end is >= i, i in [0, n].
__global__ void k_row_start(const uint32_t* __restrict__ pairs, uint64_t E, uint32_t n, uint64_t* __restrict__ row) {
  TCR_FOR(i, (uint64_t)n + 1) {
    uint64_t lo = 0, hi = E;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (pairs[2 * mid] < i) lo = mid + 1; else hi = mid;
    }
    row[i] = lo;
  }
}

__global__ void k_deg_hist(const uint32_t* __restrict__ deg, uint32_t n, unsigned long long* __restrict__ count,
                           uint32_t hist_len, uint32_t* __restrict__ maxdeg) {
  TCR_FOR(i, n) {
    const uint32_t d = deg[i];
    atomicMax(maxdeg, d);
    if (d < hist_len) atomicAdd(&count[d], 1ull);
  }
}

// Per edge: neighbour-degree sums by degree class, and the three exact sums
// of the assortativity coefficient (sum jk, sum j+k, sum j^2+k^2).
__global__ __launch_bounds__(256) void k_edge_sums(const uint32_t* __restrict__ pairs, uint64_t E,
                                                   const uint32_t* __restrict__ deg, uint32_t hist_len,
                                                   unsigned long long* __restrict__ nbr_sum,
                                                   unsigned long long* __restrict__ sums) {
  __shared__ unsigned long long sh[3][256];
  unsigned long long jk = 0, jpk = 0, j2k2 = 0;
  TCR_FOR(e, E) {
    const uint64_t a = deg[pairs[2 * e]], b = deg[pairs[2 * e + 1]];
    if (a < hist_len) atomicAdd(&nbr_sum[a], (unsigned long long)b);
    if (b < hist_len) atomicAdd(&nbr_sum[b], (unsigned long long)a);
    jk += a * b;
    jpk += a + b;
    j2k2 += a * a + b * b;
  }
  sh[0][threadIdx.x] = jk;
  sh[1][threadIdx.x] = jpk;
  sh[2][threadIdx.x] = j2k2;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + d];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + d];
      sh[2][threadIdx.x] += sh[2][threadIdx.x + d];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&sums[0], sh[0][0]);
    atomicAdd(&sums[1], sh[1][0]);
    atomicAdd(&sums[2], sh[2][0]);
  }
}

// Triangles u < v < w: for each edge (u, v), the common entries of the
// forward lists of u and v (merge of two sorted runs).
__global__ void k_triangles(const uint32_t* __restrict__ pairs, uint64_t E, const uint64_t* __restrict__ row,
                            uint32_t* __restrict__ tri, unsigned long long* __restrict__ total) {
  unsigned long long c = 0;
  TCR_FOR(e, E) {
    const uint32_t u = pairs[2 * e], v = pairs[2 * e + 1];
    uint64_t a = e + 1, ae = row[u + 1];  // u's neighbours after v
    uint64_t b = row[v], be = row[v + 1];
    while (a < ae && b < be) {
      const uint32_t x = pairs[2 * a + 1], y = pairs[2 * b + 1];
      if (x < y) {
        ++a;
      } else if (y < x) {
        ++b;
      } else {
        atomicAdd(&tri[u], 1u);
        atomicAdd(&tri[v], 1u);
        atomicAdd(&tri[x], 1u);
        ++c;
        ++a;
        ++b;
      }
    }
  }
  if (c) atomicAdd(total, c);
}

// Local clustering and per-block partial sums (fixed order: deterministic).
__global__ __launch_bounds__(256) void k_clustering(const uint32_t* __restrict__ deg, const uint32_t* __restrict__ tri,
                                                    uint32_t n, double* __restrict__ clustering,
                                                    double* __restrict__ partial) {
  __shared__ double sh[256];
  double acc = 0.0;
  TCR_FOR(i, n) {
    const double d = (double)deg[i];
    const double c = deg[i] >= 2 ? 2.0 * (double)tri[i] / (d * (d - 1.0)) : 0.0;
    if (clustering) clustering[i] = c;
    acc += c;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// One block: sum the partials in a fixed order, then the scalar results.
__global__ __launch_bounds__(256) void k_stats_final(const double* __restrict__ partial, uint32_t n_partial,
                                                     uint32_t n, uint64_t E, const unsigned long long* __restrict__ sums,
                                                     double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (uint32_t q = threadIdx.x; q < n_partial; q += 256) s += partial[q];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[1] = n ? sh[0] / (double)n : 0.0;
    // Pearson correlation of end degrees over both orientations of each edge
    const double m2 = 2.0 * (double)E;
    const double mean = m2 > 0 ? (double)sums[1] / m2 : 0.0;
    const double var = m2 > 0 ? (double)sums[2] / m2 - mean * mean : 0.0;
    out[0] = var > 0 ? (2.0 * (double)sums[0] / m2 - mean * mean) / var : 0.0;
  }
}

// Blocks of 256 for count elements, capped (the element loops are grid-stride).
inline uint32_t blocks(uint64_t n) { return (uint32_t)std::min<uint64_t>((n + 255) / 256, 1u << 20); }

}  // namespace

size_t stats_workspace_bytes(uint32_t n) {
  const uint64_t nn = (uint64_t)n + 1;
  return nn * 4 /*deg*/ + nn * 4 /*tri*/ + nn * 8 /*row*/ + (nn / 256 + 2) * 8 /*partials*/ + 256;
}

void launch_graph_stats(const uint32_t* d_pairs, uint64_t E, uint32_t n, void* ws, uint32_t hist_len,
                        unsigned long long* d_count, unsigned long long* d_nbr_sum, double* d_clustering,
                        uint32_t* d_deg_out, GraphStatsDev* d_out, hipStream_t st) {
  const uint64_t nn = (uint64_t)n + 1;
  uint32_t* deg = d_deg_out ? d_deg_out : static_cast<uint32_t*>(ws);
  uint32_t* tri = static_cast<uint32_t*>(ws) + nn;
  uint64_t* row = reinterpret_cast<uint64_t*>(static_cast<char*>(ws) + nn * 8);
  double* partial = reinterpret_cast<double*>(static_cast<char*>(ws) + nn * 16);
  launch_fill_u32(deg, n, 0u, st);
  launch_fill_u32(tri, n, 0u, st);
  launch_fill_u32(reinterpret_cast<uint32_t*>(d_count), (uint64_t)hist_len * 2, 0u, st);
  launch_fill_u32(reinterpret_cast<uint32_t*>(d_nbr_sum), (uint64_t)hist_len * 2, 0u, st);
  launch_fill_u32(reinterpret_cast<uint32_t*>(d_out), sizeof(GraphStatsDev) / 4, 0u, st);
  if (E) hipLaunchKernelGGL(k_deg, dim3(blocks(E)), dim3(256), 0, st, d_pairs, E, deg);
  hipLaunchKernelGGL(k_row_start, dim3(blocks(nn)), dim3(256), 0, st, d_pairs, E, n, row);
  if (n) hipLaunchKernelGGL(k_deg_hist, dim3(blocks(n)), dim3(256), 0, st, deg, n, d_count, hist_len,
                            &d_out->max_degree);
  if (E) {
    hipLaunchKernelGGL(k_edge_sums, dim3(blocks(E)), dim3(256), 0, st, d_pairs, E, deg, hist_len, d_nbr_sum,
                       d_out->sums);
    hipLaunchKernelGGL(k_triangles, dim3(blocks(E)), dim3(256), 0, st, d_pairs, E, row, tri, &d_out->triangles);
  }
  const uint32_t nb = blocks(n ? n : 1);
  hipLaunchKernelGGL(k_clustering, dim3(nb), dim3(256), 0, st, deg, tri, n, d_clustering, partial);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(256), 0, st, partial, nb, n, E, d_out->sums, d_out->real);
}

size_t cc_workspace_bytes(uint32_t n, uint32_t P) {
  const uint64_t nn = n ? n : 1;
  return (uint64_t)P * nn * 8 + nn * 4 + (uint64_t)P * 8 + 256;
}

void launch_components(const uint32_t* d_pairs, uint64_t E, uint32_t n, const uint32_t* d_order,
                       const uint32_t* d_removed, uint32_t P, void* ws, uint32_t* d_labels, uint32_t* d_sizes_out,
                       uint32_t* d_lcc, uint32_t* d_comps, hipStream_t st) {
  if (n == 0 || P == 0) return;
  const uint64_t total = (uint64_t)n * P;
  uint32_t* parent = static_cast<uint32_t*>(ws);
  uint32_t* sizes = d_sizes_out ? d_sizes_out : parent + total;
  uint32_t* rank = parent + 2 * total;
  launch_fill_u32(sizes, total, 0u, st);
  launch_fill_u32(d_lcc, P, 0u, st);
  launch_fill_u32(d_comps, P, 0u, st);
  hipLaunchKernelGGL(k_cc_init, dim3(blocks(total)), dim3(256), 0, st, parent, total, n);
  if (d_order) hipLaunchKernelGGL(k_cc_rank, dim3(blocks(n)), dim3(256), 0, st, d_order, n, rank);
  const uint32_t* rk = d_order ? rank : nullptr;
  if (E) hipLaunchKernelGGL(k_cc_hook, dim3(blocks(E * P)), dim3(256), 0, st, d_pairs, E, n, parent, rk, d_removed, P);
  hipLaunchKernelGGL(k_cc_finish, dim3(blocks(total)), dim3(256), 0, st, parent, n, P, rk, d_removed, sizes, d_comps);
  hipLaunchKernelGGL(k_cc_max, dim3(blocks(total)), dim3(256), 0, st, sizes, n, P, d_lcc);
  if (d_labels) hipLaunchKernelGGL(k_cc_labels, dim3(blocks(n)), dim3(256), 0, st, parent, n, d_labels);
}

}  // namespace tcr
