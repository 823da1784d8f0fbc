/*
 * Second, independent witness for the threshold l_max = 1 -- TEST
 * INFRASTRUCTURE ONLY (same rules as oracle.c; shares no code with it or with
 * the HIP library).
 *
 * Closed form (follows from the unit-cost recursion of the paper's Eq.
 * (levenshtein)): lev(a, b) <= 1 iff
 *   - a == b, or
 *   - |a| == |b| and a, b differ in exactly one position, or
 *   - ||a| - |b|| == 1 and deleting one character of the longer gives the
 *     shorter.
 * No dynamic programming is involved, so this witness cannot share a mistake
 * with the DP oracle.  It enumerates the whole network in O(N L log N) by
 * sorting three kinds of keys:
 *   exact keys     (the string itself)                 -> distance-0 pairs
 *   wildcard keys  (length, position p, string without
 *                   its p-th character)                 -> Hamming-1 pairs
 *   deletion keys  (string with one character removed) -> matched against the
 *                                                         exact keys of the
 *                                                         strings one shorter
 * Strings longer than 32 bytes are rejected (-2).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint8_t s[32];
  uint32_t len; /* length of the string in s (for wildcard keys: len + 256*pos) */
  uint32_t id;
} krec;

static int cmp_key(const void* x, const void* y) {
  const krec* a = (const krec*)x;
  const krec* b = (const krec*)y;
  if (a->len != b->len) return a->len < b->len ? -1 : 1;
  int c = memcmp(a->s, b->s, 32);
  if (c) return c;
  return (a->id > b->id) - (a->id < b->id);
}

static int same_key(const krec* a, const krec* b) {
  return a->len == b->len && memcmp(a->s, b->s, 32) == 0;
}

static int cmp_u64(const void* x, const void* y) {
  uint64_t a = *(const uint64_t*)x, b = *(const uint64_t*)y;
  return (a > b) - (a < b);
}

typedef struct {
  uint64_t* k;
  uint64_t n, cap;
} vec64;

static int push(vec64* v, uint32_t i, uint32_t j) {
  if (i > j) {
    uint32_t t = i;
    i = j;
    j = t;
  }
  if (v->n == v->cap) {
    uint64_t nc = v->cap ? 2 * v->cap : 4096;
    uint64_t* p = (uint64_t*)realloc(v->k, nc * sizeof(uint64_t));
    if (!p) return -1;
    v->k = p;
    v->cap = nc;
  }
  v->k[v->n++] = ((uint64_t)i << 32) | j;
  return 0;
}

/* Index of the first record >= key in sorted exact records (by len, s). */
static uint64_t lower_bound(const krec* r, uint64_t n, const krec* key) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) / 2;
    int c;
    if (r[mid].len != key->len)
      c = r[mid].len < key->len ? -1 : 1;
    else
      c = memcmp(r[mid].s, key->s, 32);
    if (c < 0)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

/*
 * Whole network at threshold 1.  Output as in oracle_build: sorted (i < j)
 * pairs freed with k1_free, degree (n entries, may be NULL).
 * Returns 0, -1 on allocation failure, -2 for a string longer than 32.
 */
int k1_build(const uint8_t* chars, const uint64_t* offsets, uint32_t n, uint32_t** out_pairs,
             uint64_t* out_n, int32_t* degree) {
  uint64_t tot = offsets[n] - offsets[0];
  for (uint32_t i = 0; i < n; ++i)
    if (offsets[i + 1] - offsets[i] > 32) return -2;
  krec* ex = (krec*)calloc(n ? n : 1, sizeof(krec));
  krec* wc = (krec*)calloc(tot ? tot : 1, sizeof(krec));
  krec* dl = (krec*)calloc(tot ? tot : 1, sizeof(krec));
  vec64 out = {0, 0, 0};
  int rc = -1;
  if (!ex || !wc || !dl) goto done;
  uint64_t nw = 0, nd = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const uint8_t* a = chars + offsets[i];
    uint32_t L = (uint32_t)(offsets[i + 1] - offsets[i]);
    memcpy(ex[i].s, a, L);
    ex[i].len = L;
    ex[i].id = i;
    for (uint32_t p = 0; p < L; ++p) {
      krec* w = &wc[nw++];
      memcpy(w->s, a, p);
      memcpy(w->s + p, a + p + 1, L - p - 1);
      w->len = L + 256u * p;
      w->id = i;
      krec* d = &dl[nd];
      memset(d->s, 0, sizeof d->s); /* the slot may hold a rejected duplicate */
      memcpy(d->s, w->s, L - 1);
      d->len = L - 1;
      d->id = i;
      /* one deletion key per distinct result string */
      int dup = 0;
      for (uint64_t q = nd; q > 0 && dl[q - 1].id == i; --q)
        if (same_key(&dl[q - 1], d)) dup = 1;
      if (!dup) ++nd;
    }
  }
  qsort(ex, n, sizeof(krec), cmp_key);
  qsort(wc, nw, sizeof(krec), cmp_key);
  /* distance 0: every pair inside a group of equal strings */
  for (uint64_t a = 0; a < n;) {
    uint64_t b = a + 1;
    while (b < n && same_key(&ex[a], &ex[b])) ++b;
    for (uint64_t x = a; x < b; ++x)
      for (uint64_t y = x + 1; y < b; ++y)
        if (push(&out, ex[x].id, ex[y].id)) goto done;
    a = b;
  }
  /* Hamming 1: same length, same wildcard position, equal elsewhere, and the
     two strings are not equal (they then differ exactly at that position) */
  for (uint64_t a = 0; a < nw;) {
    uint64_t b = a + 1;
    while (b < nw && same_key(&wc[a], &wc[b])) ++b;
    for (uint64_t x = a; x < b; ++x)
      for (uint64_t y = x + 1; y < b; ++y) {
        uint32_t i = wc[x].id, j = wc[y].id;
        uint32_t L = wc[x].len & 255u;
        if (memcmp(chars + offsets[i], chars + offsets[j], L) != 0)
          if (push(&out, i, j)) goto done;
      }
    a = b;
  }
  /* one insertion/deletion: a deletion key of s equal to a string t */
  for (uint64_t d = 0; d < nd; ++d) {
    uint64_t e = lower_bound(ex, n, &dl[d]);
    for (; e < n && same_key(&ex[e], &dl[d]); ++e)
      if (push(&out, dl[d].id, ex[e].id)) goto done;
  }
  qsort(out.k, out.n, sizeof(uint64_t), cmp_u64);
  {
    uint32_t* pairs = (uint32_t*)malloc((out.n ? out.n : 1) * 2 * sizeof(uint32_t));
    if (!pairs) goto done;
    uint64_t m = 0;
    for (uint64_t e = 0; e < out.n; ++e) {
      if (e && out.k[e] == out.k[e - 1]) continue; /* cannot happen; keep output a set */
      pairs[2 * m] = (uint32_t)(out.k[e] >> 32);
      pairs[2 * m + 1] = (uint32_t)out.k[e];
      ++m;
    }
    *out_pairs = pairs;
    *out_n = m;
    if (degree) {
      memset(degree, 0, sizeof(int32_t) * n);
      for (uint64_t e = 0; e < m; ++e) {
        degree[pairs[2 * e]]++;
        degree[pairs[2 * e + 1]]++;
      }
    }
  }
  rc = 0;
done:
  free(ex);
  free(wc);
  free(dl);
  free(out.k);
  return rc;
}

/* Pairwise form of the same closed form: 1 if lev(a, b) <= 1, else 0. */
int k1_adjacent(const uint8_t* a, int m, const uint8_t* b, int n) {
  if (m == n) {
    int diff = 0;
    for (int i = 0; i < m; ++i) diff += a[i] != b[i];
    return diff <= 1;
  }
  if (m + 1 == n) return k1_adjacent(b, n, a, m);
  if (m != n + 1) return 0;
  /* a is one longer: skip the first mismatch in a, the rest must be equal */
  int i = 0;
  while (i < n && a[i] == b[i]) ++i;
  return memcmp(a + i + 1, b + i, (size_t)(n - i)) == 0;
}

void k1_free(void* p) { free(p); }
