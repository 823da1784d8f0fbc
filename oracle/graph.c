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
