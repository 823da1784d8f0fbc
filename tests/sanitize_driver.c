/*
 * Runs the C code of the test oracle (oracle/*.c) and of the input generator
 * (synth/gen.c) under AddressSanitizer and UndefinedBehaviorSanitizer on the
 * host (built and run by tests/test_sanitize.py).  Every call goes through
 * the same entry points the Python bindings use, with the checks that pin
 * them repeated here so that the sanitized build is also a correct one:
 *   - the paper's worked example, lev(ACCA, ACGG) = 2 (Methods, "Levenshtein
 *     distance"), kitten/sitting = 3, empty strings, the metric axioms;
 *   - a generated repertoire: the DP network equals the k = 1 closed form,
 *     degrees sum to twice the edge count, row and query calls agree with the
 *     network, exit steps lie in [1, n];
 *   - components, site percolation and degree statistics of that network.
 * Exit status 0 on success; a sanitizer finding aborts with its report.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_lev(const uint8_t* a, int m, const uint8_t* b, int n);
int oracle_build(const uint8_t* chars, const uint64_t* offsets, uint32_t n, int32_t k, int nthreads,
                 uint32_t** out_pairs, uint64_t* out_n, int32_t* degree);
int64_t oracle_row(const uint8_t* chars, const uint64_t* offsets, uint32_t n, int32_t k, uint32_t i, int nthreads,
                   uint32_t* out);
int oracle_query(const uint8_t* rchars, const uint64_t* roffs, uint32_t r, const uint8_t* qchars,
                 const uint64_t* qoffs, uint32_t q, int32_t k, int nthreads, uint32_t** out_pairs, uint64_t* out_n,
                 int32_t* counts);
void oracle_free(void* p);
int oracle_exit_step(const uint8_t* a, int m, const uint8_t* b, int n, int k);
int k1_build(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t** out_pairs, uint64_t* out_n,
             int32_t* degree);
void k1_free(void* p);
int64_t oracle_components(const uint32_t* pairs, uint64_t E, uint32_t n, uint32_t* labels, uint32_t* sizes,
                          uint32_t* n_comp);
int oracle_robustness(const uint32_t* pairs, uint64_t E, uint32_t n, const uint32_t* order,
                      const uint32_t* removed, uint32_t P, uint32_t* lcc);
int64_t oracle_graph_stats(const uint32_t* pairs, uint64_t E, uint32_t n, int32_t* degree, uint64_t* count,
                           uint64_t* nbr_sum, uint32_t hist_len, uint64_t* tri, double* clustering, double* r_out,
                           double* avg_clustering, uint64_t* triangles);
uint64_t synth_max_bytes(uint32_t n_seqs);
int64_t synth_generate(uint64_t tseed, uint32_t n_templates, uint64_t sseed, uint32_t n_seqs, char* chars,
                       uint64_t* offsets);
int k1_adjacent(const uint8_t* a, int m, const uint8_t* b, int n);

static int failures = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                    \
    }                                                                \
  } while (0)

static int lev_s(const char* a, const char* b) {
  return oracle_lev((const uint8_t*)a, (int)strlen(a), (const uint8_t*)b, (int)strlen(b));
}

int main(void) {
  /* distances */
  CHECK(lev_s("ACCA", "ACGG") == 2);
  CHECK(lev_s("kitten", "sitting") == 3);
  CHECK(lev_s("", "") == 0 && lev_s("", "ACD") == 3 && lev_s("ACD", "") == 3);
  const char* w[] = {"CASSF", "ASSFC", "CASF", "CASSLGF", "C", "CAWSF"};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      CHECK((lev_s(w[i], w[j]) == 0) == (i == j));
      CHECK(lev_s(w[i], w[j]) == lev_s(w[j], w[i]));
      for (int l = 0; l < 6; ++l) CHECK(lev_s(w[i], w[l]) <= lev_s(w[i], w[j]) + lev_s(w[j], w[l]));
    }

  /* a generated repertoire */
  const uint32_t n = 600;
  uint8_t* chars = (uint8_t*)malloc(synth_max_bytes(n));
  uint64_t* offs = (uint64_t*)malloc((n + 1) * sizeof(uint64_t));
  CHECK(chars && offs);
  const int64_t nb = synth_generate(20211213, 60, 20211214, n, (char*)chars, offs);
  CHECK(nb > 0 && (uint64_t)nb == offs[n]);

  uint32_t *pairs = NULL, *kp = NULL;
  uint64_t E = 0, kE = 0;
  int32_t* deg = (int32_t*)calloc(n, sizeof(int32_t));
  int32_t* kdeg = (int32_t*)calloc(n, sizeof(int32_t));
  CHECK(oracle_build(chars, offs, n, 1, 2, &pairs, &E, deg) == 0);
  CHECK(k1_build(chars, offs, n, &kp, &kE, kdeg) == 0);
  CHECK(E == kE && E > 0);
  if (E == kE) CHECK(memcmp(pairs, kp, E * 2 * sizeof(uint32_t)) == 0);
  CHECK(memcmp(deg, kdeg, n * sizeof(int32_t)) == 0);
  int64_t dsum = 0;
  for (uint32_t i = 0; i < n; ++i) dsum += deg[i];
  CHECK(dsum == (int64_t)(2 * E));

  /* rows and queries against the network */
  uint32_t* row = (uint32_t*)malloc(n * sizeof(uint32_t));
  for (uint32_t i = 0; i < n; i += 97) CHECK(oracle_row(chars, offs, n, 1, i, 2, row) == deg[i]);
  uint32_t* qp = NULL;
  uint64_t qE = 0;
  int32_t counts[10];
  CHECK(oracle_query(chars, offs, n, chars, offs, 10, 1, 2, &qp, &qE, counts) == 0);
  for (int i = 0; i < 10; ++i) CHECK(counts[i] == deg[i] + 1); /* a query also meets itself */

  /* exit steps and the pairwise closed form */
  for (uint32_t i = 0; i + 1 < n; i += 13) {
    const uint8_t *a = chars + offs[i], *b = chars + offs[i + 1];
    const int m = (int)(offs[i + 1] - offs[i]), l = (int)(offs[i + 2] - offs[i + 1]);
    const int s = oracle_exit_step(a, m, b, l, 1);
    const int within = oracle_lev(a, m, b, l) <= 1;
    CHECK(s >= 1 && s <= (m < l ? m : l));
    if (within) CHECK(s == (m < l ? m : l));
    CHECK(k1_adjacent(a, m, b, l) == within);
  }
  /* longer than any generated text: the exit-step table then lives on the heap */
  {
    uint8_t x[48], y[40];
    for (int i = 0; i < 48; ++i) x[i] = (uint8_t)('A' + (i * 7) % 20);
    memcpy(y, x, 40);
    y[5] = 'Z';
    CHECK(oracle_lev(x, 48, y, 40) == 9);
    CHECK(oracle_exit_step(x, 48, y, 40, 1) >= 1);
    CHECK(oracle_exit_step(x, 40, y, 40, 1) == 40);
  }

  /* network analyses */
  uint32_t* labels = (uint32_t*)malloc(n * sizeof(uint32_t));
  uint32_t* sizes = (uint32_t*)malloc(n * sizeof(uint32_t));
  uint32_t nc = 0;
  const int64_t lcc = oracle_components(pairs, E, n, labels, sizes, &nc);
  CHECK(lcc >= 2 && nc >= 1 && nc <= n);
  uint32_t* order = (uint32_t*)malloc(n * sizeof(uint32_t));
  for (uint32_t i = 0; i < n; ++i) order[i] = (i * 7919u) % n; /* 7919 is prime to 600 */
  const uint32_t removed[3] = {0, n / 2, n};
  uint32_t curve[3];
  CHECK(oracle_robustness(pairs, E, n, order, removed, 3, curve) == 0);
  CHECK(curve[0] == (uint32_t)lcc && curve[2] == 0 && curve[1] <= curve[0]);
  int32_t sdeg[600];
  uint64_t cnt[601], nbr[601], tri[600], t3 = 0;
  double clu[600], r = 0.0, avg = 0.0;
  const int64_t maxd = oracle_graph_stats(pairs, E, n, sdeg, cnt, nbr, n + 1, tri, clu, &r, &avg, &t3);
  CHECK(maxd >= 1 && memcmp(sdeg, deg, n * sizeof(int32_t)) == 0);
  CHECK(r >= -1.0 && r <= 1.0 && avg >= 0.0 && avg <= 1.0);

  oracle_free(pairs);
  oracle_free(qp);
  k1_free(kp);
  free(chars);
  free(offs);
  free(deg);
  free(kdeg);
  free(row);
  free(labels);
  free(sizes);
  free(order);
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("sanitized oracle and generator: all checks passed\n");
  return 0;
}
