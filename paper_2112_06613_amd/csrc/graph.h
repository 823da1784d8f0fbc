// Launchers of the network-analysis kernels (graph.hip).
#pragma once
#include "kernels.h"

namespace tcr {

// Workspace bytes of launch_components for n nodes and P runs.
size_t cc_workspace_bytes(uint32_t n, uint32_t P);

// P union-find runs over the E device pairs: run q uses only nodes whose
// position in d_order is >= d_removed[q] (d_order NULL: one run, all nodes).
// Writes d_lcc[q] (LCC size), d_comps[q] (number of components) and, when
// not NULL, d_labels (n; run 0; smallest id of each node's component) and
// d_sizes_out (P*n; size of the component whose label is i, else 0).
void launch_components(const uint32_t* d_pairs, uint64_t E, uint32_t n, const uint32_t* d_order,
                       const uint32_t* d_removed, uint32_t P, void* ws, uint32_t* d_labels, uint32_t* d_sizes_out,
                       uint32_t* d_lcc, uint32_t* d_comps, hipStream_t st);

// Device results of launch_graph_stats.
struct GraphStatsDev {
  unsigned long long sums[3];   // sum jk, sum j+k, sum j^2+k^2 over edges
  unsigned long long triangles;
  double real[2];               // assortativity, average clustering
  uint32_t max_degree;
  uint32_t pad;
};

size_t stats_workspace_bytes(uint32_t n);

// Degree statistics of a canonical edge list (i < j, sorted, distinct):
// degrees, degree histogram and neighbour-degree sums by degree class
// (hist_len entries; larger degrees are left out and visible as
// max_degree >= hist_len), triangles, local clustering (may be NULL), the
// degree assortativity and the average clustering.
void launch_graph_stats(const uint32_t* d_pairs, uint64_t E, uint32_t n, void* ws, uint32_t hist_len,
                        unsigned long long* d_count, unsigned long long* d_nbr_sum, double* d_clustering,
                        uint32_t* d_deg_out, GraphStatsDev* d_out, hipStream_t st);

}  // namespace tcr
