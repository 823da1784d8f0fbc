/*
 * Work model of the pair kernel's traversal -- BENCHMARK INFRASTRUCTURE ONLY.
 * It prices a launch (workmodel/__init__.py writes bench_model.json); it
 * decides no edge, and shares no code with the HIP library or the test
 * oracle (its distances come from its own plain DP table below).
 *
 * A work item is a group of up to `width` patterns (64, or 128 when two
 * patterns share a lane) and a run of texts of one length bucket, the texts
 * in sorted order (length, residues).  For each visited text the wave needs
 * as many text steps as its last lane needs before the final-diagonal bound
 * exceeds k (wm_exit_step), or all n steps when some lane ends within k.
 * When every lane ended early after e residues, all texts sharing those
 * first e residues end the same way, so the walk continues at the end of
 * that prefix group (group ends for e = 1..8, given by the caller); in a
 * triangle item this holds only once the text lies `width` positions past
 * the group start (every pattern of the group before it).  A visited text
 * whose first r residues equal those of the previous visited text of the
 * item starts at step r (r capped at `resume`; 0 for the item's first text
 * and after a text whose set of valid lanes differs from the next one's).
 */
#include <stdint.h>

/* Plain DP table of the edit distance with unit costs (rows: a, columns: b,
 * D[i][0] = i, D[0][j] = j), then the exit step of the exact final-diagonal
 * early exit with the longer string as rows: the first text step j after
 * which D[j + m - n][j] > k, or n when there is none.  *lev = D[m][n].
 * Lengths are at most 32. */
int wm_exit_step(const uint8_t* a, int m, const uint8_t* b, int n, int k, int* lev) {
  if (m < n) {
    const uint8_t* t = a;
    a = b;
    b = t;
    const int q = m;
    m = n;
    n = q;
  }
  int D[33][33];
  for (int i = 0; i <= m; ++i) D[i][0] = i;
  for (int j = 0; j <= n; ++j) D[0][j] = j;
  for (int i = 1; i <= m; ++i)
    for (int j = 1; j <= n; ++j) {
      int v = D[i - 1][j - 1] + (a[i - 1] != b[j - 1]);
      if (D[i - 1][j] + 1 < v) v = D[i - 1][j] + 1;
      if (D[i][j - 1] + 1 < v) v = D[i][j - 1] + 1;
      D[i][j] = v;
    }
  *lev = D[m][n];
  for (int j = 1; j <= n; ++j)
    if (D[j + m - n][j] > k) return j;
  return n;
}

#define WM_DEPTHS 8

/* Length of the common prefix of a and b (n residues each), at most cap. */
static int common_prefix(const uint8_t* a, const uint8_t* b, int n, int cap) {
  int q = 0;
  while (q < n && q < cap && a[q] == b[q]) ++q;
  return q;
}

/* One item: patterns at sorted positions [gbase, gbase + np), texts [tb, te),
 * tri: only pairs with pattern position < text position.  seq[s] = input id
 * of sorted position s; gend[s * 8 + d - 1] = end of s's depth-d prefix
 * group.  Returns the text steps; *texts = texts visited. */

static uint64_t wm_item(const uint8_t* chars, const uint64_t* offsets, const uint32_t* seq, const uint32_t* gend,
                        uint32_t gbase, uint32_t np, uint32_t tb, uint32_t te, int tri, uint32_t width, int k,
                        int resume, uint64_t* texts) {
  uint64_t steps = 0, visited = 0;
  uint32_t t = tb;
  int prev_ok = 0;       /* previous visited text may pass its state on */
  uint32_t prev = 0;
  while (t < te) {
    const uint32_t b = seq[t];
    const uint8_t* tb_ = chars + offsets[b];
    const int n = (int)(offsets[b + 1] - offsets[b]);
    int e = 0, full = 0;
    for (uint32_t p = gbase; p < gbase + np; ++p) {
      if (tri && p >= t) continue;
      const uint32_t a = seq[p];
      const uint8_t* pa = chars + offsets[a];
      const int m = (int)(offsets[a + 1] - offsets[a]);
      int lev = 0;
      const int s = wm_exit_step(pa, m, tb_, n, k, &lev);
      if (s == n && lev <= k) full = 1;
      if (s > e) e = s;
    }
    int r = 0;
    if (prev_ok) {
      r = common_prefix(chars + offsets[seq[prev]], tb_, n, WM_DEPTHS);
      if (r > resume) r = resume;
    }
    steps += (full ? (uint64_t)n : (uint64_t)e) - (uint64_t)r;
    visited += 1;
    const int can_skip = !tri || t - gbase >= width;
    prev_ok = can_skip;
    prev = t;
    uint32_t tn = t + 1;
    if (!full && e >= 1 && e <= WM_DEPTHS && can_skip) {
      tn = gend[(uint64_t)t * WM_DEPTHS + (uint64_t)(e - 1)];
      if (tn < t + 1) tn = t + 1;
    }
    t = tn;
  }
  *texts = visited;
  return steps;
}

/* count items, item q = (gbase, np, tb, te, tri, width) at items[6q..6q+5]. */
void wm_items(const uint8_t* chars, const uint64_t* offsets, const uint32_t* seq, const uint32_t* gend,
              const uint32_t* items, int64_t count, int k, int resume, uint64_t* steps, uint64_t* texts) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < count; ++q) {
    const uint32_t* it = items + 6 * q;
    steps[q] = wm_item(chars, offsets, seq, gend, it[0], it[1], it[2], it[3], (int)it[4], it[5], k, resume,
                       &texts[q]);
  }
}

/* wm_exit_step over `count` pairs (pi[q], pj[q]) of one sequence set. */
void wm_exit_steps(const uint8_t* chars, const uint64_t* offsets, const uint32_t* pi, const uint32_t* pj,
                   int64_t count, int k, int32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < count; ++q) {
    const uint32_t i = pi[q], j = pj[q];
    int lev = 0;
    out[q] = wm_exit_step(chars + offsets[i], (int)(offsets[i + 1] - offsets[i]), chars + offsets[j],
                          (int)(offsets[j + 1] - offsets[j]), k, &lev);
  }
}
