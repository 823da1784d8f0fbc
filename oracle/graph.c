/*
 * Network-analysis oracle -- TEST INFRASTRUCTURE ONLY (same rules as
 * oracle.c: only tests, the smoke check and the benchmark's CPU-baseline leg
 * use it; no code is shared with the HIP library).
 *
 * Plain breadth-first searches over an adjacency list built from the edge
 * list (paper, Methods, "Overview of network theory concepts": connected
 * subgraphs, the largest connected component (LCC), cluster sizes;
 * "Percolation transition": site percolation = removal of nodes;
 * "Computing LCC": LCC(p) of the network left after removing nodes).
 *
 * Conventions: undirected graph on nodes 0..n-1, edges as 2E uint32 pairs
 * (duplicates and self loops are tolerated and have no effect on
 * connectivity).  A component's label is its smallest node id.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint64_t* start; /* n+1 */
  uint32_t* adj;   /* 2E */
} csr;

static int build_csr(const uint32_t* pairs, uint64_t E, uint32_t n, csr* g) {
  g->start = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
  g->adj = (uint32_t*)malloc((2 * E ? 2 * E : 1) * sizeof(uint32_t));
  uint64_t* fill = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
  if (!g->start || !g->adj || !fill) {
    free(g->start);
    free(g->adj);
    free(fill);
    return -1;
  }
  for (uint64_t e = 0; e < E; ++e) {
    g->start[pairs[2 * e] + 1]++;
    g->start[pairs[2 * e + 1] + 1]++;
  }
  for (uint32_t i = 0; i < n; ++i) g->start[i + 1] += g->start[i];
  for (uint32_t i = 0; i <= n; ++i) fill[i] = g->start[i];
  for (uint64_t e = 0; e < E; ++e) {
    uint32_t a = pairs[2 * e], b = pairs[2 * e + 1];
    g->adj[fill[a]++] = b;
    g->adj[fill[b]++] = a;
  }
  free(fill);
  return 0;
}

/*
 * Components of the nodes with alive[i] != 0 (alive may be NULL: all alive),
 * using only edges between alive nodes.  labels[i] (may be NULL) = smallest
 * id of i's component, or 0xffffffff for a removed node; sizes[i] (may be
 * NULL) = size of the component labelled i, 0 if i is no label.  Returns the
 * LCC size (0 for no alive node) and the number of components in *n_comp.
 */
static int64_t bfs_components(const csr* g, uint32_t n, const uint8_t* alive, uint32_t* labels, uint32_t* sizes,
                              uint32_t* n_comp) {
  uint32_t* lab = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
  uint32_t* queue = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
  if (!lab || !queue) {
    free(lab);
    free(queue);
    return -1;
  }
  for (uint32_t i = 0; i < n; ++i) lab[i] = 0xffffffffu;
  if (sizes) memset(sizes, 0, sizeof(uint32_t) * n);
  uint32_t comps = 0, best = 0;
  for (uint32_t s = 0; s < n; ++s) {
    if ((alive && !alive[s]) || lab[s] != 0xffffffffu) continue;
    /* s is the smallest id of its component: every smaller alive node was
       already reached from its own component */
    uint32_t head = 0, tail = 0;
    queue[tail++] = s;
    lab[s] = s;
    while (head < tail) {
      uint32_t u = queue[head++];
      for (uint64_t q = g->start[u]; q < g->start[u + 1]; ++q) {
        uint32_t v = g->adj[q];
        if ((alive && !alive[v]) || lab[v] != 0xffffffffu) continue;
        lab[v] = s;
        queue[tail++] = v;
      }
    }
    comps++;
    if (sizes) sizes[s] = tail;
    if (tail > best) best = tail;
  }
  if (labels) memcpy(labels, lab, sizeof(uint32_t) * n);
  if (n_comp) *n_comp = comps;
  free(lab);
  free(queue);
  return best;
}

/* Whole-graph components.  Returns the LCC size, -1 on allocation failure. */
int64_t oracle_components(const uint32_t* pairs, uint64_t E, uint32_t n, uint32_t* labels, uint32_t* sizes,
                          uint32_t* n_comp) {
  csr g;
  if (build_csr(pairs, E, n, &g)) return -1;
  int64_t r = bfs_components(&g, n, NULL, labels, sizes, n_comp);
  free(g.start);
  free(g.adj);
  return r;
}

/*
 * Site percolation: for each q < P remove the nodes order[0 .. removed[q])
 * and store the LCC size of what is left in lcc[q].  order is a permutation
 * of 0..n-1 supplied by the caller (the random removal order).
 */
int oracle_robustness(const uint32_t* pairs, uint64_t E, uint32_t n, const uint32_t* order,
                      const uint32_t* removed, uint32_t P, uint32_t* lcc) {
  csr g;
  if (build_csr(pairs, E, n, &g)) return -1;
  uint8_t* alive = (uint8_t*)malloc(n ? n : 1);
  if (!alive) {
    free(g.start);
    free(g.adj);
    return -1;
  }
  int rc = 0;
  for (uint32_t q = 0; q < P; ++q) {
    memset(alive, 1, n);
    uint32_t r = removed[q] < n ? removed[q] : n;
    for (uint32_t t = 0; t < r; ++t) alive[order[t]] = 0;
    int64_t best = bfs_components(&g, n, alive, NULL, NULL, NULL);
    if (best < 0) {
      rc = -1;
      break;
    }
    lcc[q] = (uint32_t)best;
  }
  free(alive);
  free(g.start);
  free(g.adj);
  return rc;
}

/*
 * Degree statistics of a simple undirected graph given as distinct pairs
 * (paper, Methods, "Overview of network theory concepts": degree d(u), degree
 * distribution p_d, average neighbour degree <d_nn>, degree assortativity r
 * (Newman 2002), and the clustering coefficient used in Results, "Network
 * structure of TCR repertoires").  Plain definitions:
 *   degree[u]       = number of pairs naming u
 *   count[d]        = number of nodes of degree d                 (hist_len)
 *   nbr_sum[d]      = sum over nodes u of degree d of the degrees of u's
 *                     neighbours; <d_nn>(d) = nbr_sum[d] / (d * count[d])
 *   r               = Pearson correlation of the degrees at the two ends of
 *                     an edge, over both orientations of every edge
 *   tri[u]          = triangles through u (pairs of neighbours that are
 *                     adjacent), clustering[u] = 2 tri[u] / (d (d - 1)), 0
 *                     for d < 2; avg_clustering = mean over all nodes
 * Returns the maximum degree, or -1 on allocation failure, -2 if hist_len
 * is too small (count/nbr_sum then untouched).
 */
int64_t oracle_graph_stats(const uint32_t* pairs, uint64_t E, uint32_t n, int32_t* degree, uint64_t* count,
                           uint64_t* nbr_sum, uint32_t hist_len, uint64_t* tri, double* clustering, double* r_out,
                           double* avg_clustering, uint64_t* triangles) {
  csr g;
  if (build_csr(pairs, E, n, &g)) return -1;
  int64_t maxd = 0;
  for (uint32_t u = 0; u < n; ++u) {
    int64_t d = (int64_t)(g.start[u + 1] - g.start[u]);
    if (degree) degree[u] = (int32_t)d;
    if (d > maxd) maxd = d;
  }
  if ((uint64_t)maxd >= hist_len) {
    free(g.start);
    free(g.adj);
    return -2;
  }
  memset(count, 0, sizeof(uint64_t) * hist_len);
  memset(nbr_sum, 0, sizeof(uint64_t) * hist_len);
  for (uint32_t u = 0; u < n; ++u) {
    uint64_t d = g.start[u + 1] - g.start[u];
    count[d]++;
    for (uint64_t q = g.start[u]; q < g.start[u + 1]; ++q) {
      uint32_t v = g.adj[q];
      nbr_sum[d] += g.start[v + 1] - g.start[v];
    }
  }
  /* assortativity over both orientations of every edge */
  double sx = 0, sxx = 0, sxy = 0, m2 = 0;
  for (uint64_t e = 0; e < E; ++e) {
    double a = (double)(g.start[pairs[2 * e] + 1] - g.start[pairs[2 * e]]);
    double b = (double)(g.start[pairs[2 * e + 1] + 1] - g.start[pairs[2 * e + 1]]);
    sx += a + b;
    sxx += a * a + b * b;
    sxy += 2 * a * b;
    m2 += 2;
  }
  if (r_out) {
    double mean = m2 > 0 ? sx / m2 : 0;
    double var = m2 > 0 ? sxx / m2 - mean * mean : 0;
    *r_out = var > 0 ? (sxy / m2 - mean * mean) / var : 0.0;
  }
  /* triangles: neighbours v < w of u that are adjacent (adjacency test by a
     scan of v's list) */
  uint64_t total3 = 0;
  double csum = 0;
  for (uint32_t u = 0; u < n; ++u) {
    uint64_t t = 0;
    for (uint64_t a = g.start[u]; a < g.start[u + 1]; ++a)
      for (uint64_t b = a + 1; b < g.start[u + 1]; ++b) {
        uint32_t v = g.adj[a], w = g.adj[b];
        for (uint64_t q = g.start[v]; q < g.start[v + 1]; ++q)
          if (g.adj[q] == w) {
            ++t;
            break;
          }
      }
    if (tri) tri[u] = t;
    total3 += t;
    uint64_t d = g.start[u + 1] - g.start[u];
    double c = d >= 2 ? 2.0 * (double)t / ((double)d * (double)(d - 1)) : 0.0;
    if (clustering) clustering[u] = c;
    csum += c;
  }
  if (avg_clustering) *avg_clustering = n ? csum / n : 0.0;
  if (triangles) *triangles = total3 / 3;
  free(g.start);
  free(g.adj);
  return maxd;
}
