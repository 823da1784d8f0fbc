/*
 * TCR-network oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU code for what the GPU library computes.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library; the product path never does.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * What it computes (paper, Methods):
 *  - "Levenshtein distance", Eq. (levenshtein) with the indicator cost:
 *    unit-cost insertion, deletion and substitution.  The printed base case is
 *    written with shifted indices; it is read here as the textbook recursion
 *    with row and column 0 standing for the empty prefix:
 *        D[i][0] = i, D[0][j] = j,
 *        D[i][j] = min(D[i-1][j] + 1, D[i][j-1] + 1, D[i-1][j-1] + [a_i != b_j]).
 *    The full (m+1) x (n+1) table is filled for every pair: no length filter,
 *    no early abort.
 *  - "TCR network": nodes i and j are adjacent iff lev(s_i, s_j) <= l_max
 *    (the text's "does not exceed"; the printed listing's strict "<" is read as
 *    a slip).  One node per input position; equal strings are distinct nodes
 *    joined by a distance-0 edge; no self-pairs (zero diagonal of the
 *    adjacency matrix in "Adjacency matrix").
 *  - "Overview of network theory concepts": degree d(u) = sum_v A_uv.
 * Output convention: edges (i, j) with i < j, 0-based input positions, sorted
 * lexicographically; degree as int32.
 *
 * Strings are compared as raw bytes; the oracle imposes no alphabet or length
 * limit (the library's input validation is not the oracle's business).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- distance */
/* Fill the full (m+1) x (n+1) table D (row-major, width n+1) for rows a and
   columns b.  D must hold (m+1)*(n+1) ints. */
static void dp_fill(const uint8_t* a, int m, const uint8_t* b, int n, int* D) {
  int w = n + 1;
  for (int i = 0; i <= m; ++i) D[i * w + 0] = i;
  for (int j = 0; j <= n; ++j) D[0 * w + j] = j;
  for (int i = 1; i <= m; ++i) {
    for (int j = 1; j <= n; ++j) {
      int del = D[(i - 1) * w + j] + 1;
      int ins = D[i * w + (j - 1)] + 1;
      int sub = D[(i - 1) * w + (j - 1)] + (a[i - 1] != b[j - 1] ? 1 : 0);
      int best = del;
      if (ins < best) best = ins;
      if (sub < best) best = sub;
      D[i * w + j] = best;
    }
  }
}

int oracle_lev(const uint8_t* a, int m, const uint8_t* b, int n) {
  int stack_tab[33 * 33];
  int* D = stack_tab;
  if ((m + 1) * (n + 1) > 33 * 33) {
    D = (int*)malloc(sizeof(int) * (size_t)(m + 1) * (size_t)(n + 1));
    if (!D) return -1;
  }
  dp_fill(a, m, b, n, D);
  int r = D[m * (n + 1) + n];
  if (D != stack_tab) free(D);
  return r;
}

/* ------------------------------------------------------------ edge buffers */
typedef struct {
  uint64_t* key; /* (first << 32) | second */
  uint64_t n, cap;
} keybuf;

static int kb_push(keybuf* b, uint64_t k) {
  if (b->n == b->cap) {
    uint64_t nc = b->cap ? b->cap * 2 : 1024;
    uint64_t* p = (uint64_t*)realloc(b->key, nc * sizeof(uint64_t));
    if (!p) return -1;
    b->key = p;
    b->cap = nc;
  }
  b->key[b->n++] = k;
  return 0;
}

static int cmp_u64(const void* x, const void* y) {
  uint64_t a = *(const uint64_t*)x, b = *(const uint64_t*)y;
  return (a > b) - (a < b);
}

/* Merge per-thread key buffers, sort, and unpack into (first, second) pairs. */
static int finish_pairs(keybuf* bufs, int nb, uint32_t** out_pairs, uint64_t* out_n) {
  uint64_t tot = 0;
  for (int t = 0; t < nb; ++t) tot += bufs[t].n;
  uint64_t* all = (uint64_t*)malloc((tot ? tot : 1) * sizeof(uint64_t));
  uint32_t* pairs = (uint32_t*)malloc((tot ? tot : 1) * 2 * sizeof(uint32_t));
  if (!all || !pairs) {
    free(all);
    free(pairs);
    return -1;
  }
  uint64_t p = 0;
  for (int t = 0; t < nb; ++t) {
    if (bufs[t].n) memcpy(all + p, bufs[t].key, bufs[t].n * sizeof(uint64_t));
    p += bufs[t].n;
  }
  qsort(all, tot, sizeof(uint64_t), cmp_u64);
  for (uint64_t e = 0; e < tot; ++e) {
    pairs[2 * e] = (uint32_t)(all[e] >> 32);
    pairs[2 * e + 1] = (uint32_t)(all[e] & 0xffffffffu);
  }
  free(all);
  *out_pairs = pairs;
  *out_n = tot;
  return 0;
}

static int max_threads(int nthreads) {
#ifdef _OPENMP
  return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/*
 * Network of the rows i in [row_lo, row_hi): every pair (i, j) with
 * row_lo <= i < row_hi, i < j < n, lev <= k.  With row_lo = 0 and row_hi = n
 * this is the whole network.  Degrees (length n, caller-allocated, may be
 * NULL) are the row sums of the adjacency restricted to those edges, so they
 * are the true degrees only for the whole network.
 * Returns 0, or -1 on allocation failure.  *out_pairs is freed by oracle_free.
 */
int oracle_build_rows(const uint8_t* chars, const uint64_t* offsets, uint32_t n, int32_t k,
                      uint32_t row_lo, uint32_t row_hi, int nthreads,
                      uint32_t** out_pairs, uint64_t* out_n, int32_t* degree) {
  if (row_hi > n) row_hi = n;
  int nt = max_threads(nthreads);
  keybuf* bufs = (keybuf*)calloc((size_t)nt, sizeof(keybuf));
  if (!bufs) return -1;
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt) reduction(| : fail)
  for (int64_t i = row_lo; i < (int64_t)row_hi; ++i) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    const uint8_t* a = chars + offsets[i];
    int m = (int)(offsets[i + 1] - offsets[i]);
    for (uint32_t j = (uint32_t)i + 1; j < n; ++j) {
      const uint8_t* b = chars + offsets[j];
      int l = (int)(offsets[j + 1] - offsets[j]);
      if (oracle_lev(a, m, b, l) <= k) {
        if (kb_push(&bufs[tid], ((uint64_t)i << 32) | j)) fail = 1;
      }
    }
  }
  int rc = fail ? -1 : finish_pairs(bufs, nt, out_pairs, out_n);
  for (int t = 0; t < nt; ++t) free(bufs[t].key);
  free(bufs);
  if (rc == 0 && degree) {
    memset(degree, 0, sizeof(int32_t) * n);
    for (uint64_t e = 0; e < *out_n; ++e) {
      degree[(*out_pairs)[2 * e]] += 1;
      degree[(*out_pairs)[2 * e + 1]] += 1;
    }
  }
  return rc;
}

int oracle_build(const uint8_t* chars, const uint64_t* offsets, uint32_t n, int32_t k, int nthreads,
                 uint32_t** out_pairs, uint64_t* out_n, int32_t* degree) {
  return oracle_build_rows(chars, offsets, n, k, 0, n, nthreads, out_pairs, out_n, degree);
}

/*
 * Neighbours of a single node i in the network of n strings: every j != i with
 * lev(s_i, s_j) <= k, ascending.  out must hold n entries.  Returns the count.
 */
int64_t oracle_row(const uint8_t* chars, const uint64_t* offsets, uint32_t n, int32_t k, uint32_t i,
                   int nthreads, uint32_t* out) {
  int nt = max_threads(nthreads);
  uint8_t* hit = (uint8_t*)calloc(n ? n : 1, 1);
  if (!hit) return -1;
  const uint8_t* a = chars + offsets[i];
  int m = (int)(offsets[i + 1] - offsets[i]);
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t j = 0; j < (int64_t)n; ++j) {
    if (j == i) continue;
    const uint8_t* b = chars + offsets[j];
    int l = (int)(offsets[j + 1] - offsets[j]);
    hit[j] = oracle_lev(a, m, b, l) <= k;
  }
  int64_t c = 0;
  for (uint32_t j = 0; j < n; ++j)
    if (hit[j]) out[c++] = j;
  free(hit);
  return c;
}

/*
 * Query of q strings against a repertoire of r strings: every (qi, ri) with
 * lev <= k, sorted by (qi, ri); counts[qi] = number of such ri (may be NULL).
 */
int oracle_query(const uint8_t* rchars, const uint64_t* roffs, uint32_t r,
                 const uint8_t* qchars, const uint64_t* qoffs, uint32_t q, int32_t k, int nthreads,
                 uint32_t** out_pairs, uint64_t* out_n, int32_t* counts) {
  int nt = max_threads(nthreads);
  keybuf* bufs = (keybuf*)calloc((size_t)nt, sizeof(keybuf));
  if (!bufs) return -1;
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt) reduction(| : fail)
  for (int64_t i = 0; i < (int64_t)q; ++i) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    const uint8_t* a = qchars + qoffs[i];
    int m = (int)(qoffs[i + 1] - qoffs[i]);
    for (uint32_t j = 0; j < r; ++j) {
      const uint8_t* b = rchars + roffs[j];
      int l = (int)(roffs[j + 1] - roffs[j]);
      if (oracle_lev(a, m, b, l) <= k) {
        if (kb_push(&bufs[tid], ((uint64_t)i << 32) | j)) fail = 1;
      }
    }
  }
  int rc = fail ? -1 : finish_pairs(bufs, nt, out_pairs, out_n);
  for (int t = 0; t < nt; ++t) free(bufs[t].key);
  free(bufs);
  if (rc == 0 && counts) {
    memset(counts, 0, sizeof(int32_t) * q);
    for (uint64_t e = 0; e < *out_n; ++e) counts[(*out_pairs)[2 * e]] += 1;
  }
  return rc;
}

void oracle_free(void* p) { free(p); }

int oracle_threads(int nthreads) { return max_threads(nthreads); }

/*
 * Algorithmic-work model of the early-exit rule (used to price the work of a
 * network build, not to decide edges).  Rows are the longer string (m),
 * columns the shorter (n <= m).  Returns the first column j in [1, n] whose
 * cell on the final diagonal, D[j + m - n][j], exceeds k, or n if none does.
 * D does not decrease along a diagonal, so that cell bounds D[m][n] from
 * below: a pair with lev <= k always returns n.
 */
int oracle_exit_step(const uint8_t* a, int m, const uint8_t* b, int n, int k) {
  if (m < n) {
    const uint8_t* t = a;
    a = b;
    b = t;
    int q = m;
    m = n;
    n = q;
  }
  int stack_tab[33 * 33];
  int* D = stack_tab;
  int w = n + 1;
  if ((m + 1) * (n + 1) > 33 * 33) {
    D = (int*)malloc(sizeof(int) * (size_t)(m + 1) * (size_t)(n + 1));
    if (!D) return -1;
  }
  dp_fill(a, m, b, n, D);
  int s = n;
  for (int j = 1; j <= n; ++j) {
    if (D[(j + m - n) * w + j] > k) {
      s = j;
      break;
    }
  }
  if (D != stack_tab) free(D);
  return s;
}

/* oracle_exit_step over `count` pairs (pi[q], pj[q]) of one sequence set. */
void oracle_exit_steps(const uint8_t* chars, const uint64_t* offsets, const uint32_t* pi, const uint32_t* pj,
                       uint64_t count, int32_t k, int nthreads, int32_t* out) {
  int nt = max_threads(nthreads);
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t q = 0; q < (int64_t)count; ++q) {
    const uint32_t i = pi[q], j = pj[q];
    out[q] = oracle_exit_step(chars + offsets[i], (int)(offsets[i + 1] - offsets[i]), chars + offsets[j],
                              (int)(offsets[j + 1] - offsets[j]), k);
  }
}
