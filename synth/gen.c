/*
 * Seeded synthetic CDR3-beta repertoire generator.
 *
 * Shared input source for the test oracle and for the GPU library's tests and
 * benchmark.  It contains none of the edit-distance arithmetic: it only draws
 * strings.  The Python module next to this file holds a line-for-line
 * equivalent in pure Python, and a test checks that both emit identical bytes.
 *
 * Workload shape (stand-in for the paper's SONIA-generated and empirical
 * CDR3-beta repertoires, which are not available): T templates, each 'C' +
 * uniform residues + 'F' with total length round(N(14, 2)) clipped to [6, 25];
 * each sequence is a uniformly chosen template plus Poisson(1.5) random edits,
 * each edit uniformly a substitution, an insertion or a deletion at a uniform
 * position.  Residues come from the 20 amino acids in the order the paper lists
 * them (Methods, "Combination of amino acids").
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).
 *   uniform_below(n) = ((x >> 32) * n) >> 32             (multiply-shift)
 *   u01()            = (x >> 11) * 2^-53
 *   normal length    = Irwin-Hall sum of 12 uniforms of 24 bits, integer only
 *   Poisson(1.5)     = Knuth's product-of-uniforms method, exp(-1.5) literal
 * Draw order: templates from a stream seeded with tseed (for each template: 12
 * length draws, then len-2 residues); sequences from a stream seeded with
 * sseed (for each sequence: template index, edit count, then per edit: type,
 * position, and a residue for substitutions and insertions).  An insertion
 * that would exceed 32 residues or a deletion that would leave none is drawn
 * but not applied.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const char kAlphabet[21] = "ARNDCQEGHILKMFPSTWYV";
#define SYNTH_MAX_LEN 32

typedef struct { uint64_t s; } sm64;

static uint64_t sm64_next(sm64* r) {
  uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static uint32_t below(sm64* r, uint32_t n) {
  return (uint32_t)(((sm64_next(r) >> 32) * (uint64_t)n) >> 32);
}

static double u01(sm64* r) { return (double)(sm64_next(r) >> 11) * (1.0 / 9007199254740992.0); }

static uint32_t poisson15(sm64* r) {
  const double L = 0.22313016014842982; /* exp(-1.5) */
  uint32_t n = 0;
  double p = u01(r);
  while (p > L) {
    ++n;
    p *= u01(r);
  }
  return n;
}

static int template_len(sm64* r) {
  uint64_t s = 0;
  for (int t = 0; t < 12; ++t) s += sm64_next(r) >> 40;
  /* round(14 + 2 * (s / 2^24 - 6)) = floor(2 + 2 s / 2^24 + 1/2) */
  int64_t L = (int64_t)((2 * s + (2ull << 24) + (1ull << 23)) >> 24);
  if (L < 6) L = 6;
  if (L > 25) L = 25;
  return (int)L;
}

/* Number of bytes synth_generate writes for a (T, N) request is at most N*32. */
uint64_t synth_max_bytes(uint32_t n_seqs) { return (uint64_t)n_seqs * SYNTH_MAX_LEN; }

/*
 * Generate n_seqs sequences from n_templates templates.
 * chars: capacity >= n_seqs*32 bytes; offsets: n_seqs+1 entries.
 * Returns the number of bytes written, or -1 on bad arguments.
 */
int64_t synth_generate(uint64_t tseed, uint32_t n_templates, uint64_t sseed, uint32_t n_seqs,
                       char* chars, uint64_t* offsets) {
  if (n_templates == 0 || !offsets || (n_seqs && !chars)) return -1;
  /* templates: stored as codes, 26 bytes each (max template length 25) */
  enum { TSTRIDE = 26 };
  uint8_t* tbuf = (uint8_t*)malloc((size_t)n_templates * TSTRIDE);
  if (!tbuf) return -1;
  sm64 tr = {tseed};
  for (uint32_t t = 0; t < n_templates; ++t) {
    uint8_t* dst = tbuf + (size_t)t * TSTRIDE;
    int L = template_len(&tr);
    dst[0] = (uint8_t)L;
    dst[1] = 4; /* 'C' */
    for (int i = 1; i < L - 1; ++i) dst[1 + i] = (uint8_t)below(&tr, 20);
    dst[L] = 13; /* 'F' */
  }
  sm64 sr = {sseed};
  uint64_t pos = 0;
  offsets[0] = 0;
  for (uint32_t i = 0; i < n_seqs; ++i) {
    uint32_t t = below(&sr, n_templates);
    const uint8_t* src = tbuf + (size_t)t * TSTRIDE;
    uint8_t s[SYNTH_MAX_LEN + 1];
    int len = src[0];
    memcpy(s, src + 1, (size_t)len);
    uint32_t ne = poisson15(&sr);
    for (uint32_t e = 0; e < ne; ++e) {
      uint32_t type = below(&sr, 3);
      if (type == 0) { /* substitution by one of the 19 other residues */
        uint32_t p = below(&sr, (uint32_t)len);
        uint32_t c = below(&sr, 19);
        s[p] = (uint8_t)(c < s[p] ? c : c + 1);
      } else if (type == 1) { /* insertion before position p in [0, len] */
        uint32_t p = below(&sr, (uint32_t)len + 1);
        uint32_t c = below(&sr, 20);
        if (len < SYNTH_MAX_LEN) {
          memmove(s + p + 1, s + p, (size_t)(len - (int)p));
          s[p] = (uint8_t)c;
          ++len;
        }
      } else { /* deletion */
        uint32_t p = below(&sr, (uint32_t)len);
        if (len > 1) {
          memmove(s + p, s + p + 1, (size_t)(len - (int)p - 1));
          --len;
        }
      }
    }
    for (int q = 0; q < len; ++q) chars[pos + (uint64_t)q] = kAlphabet[s[q]];
    pos += (uint64_t)len;
    offsets[i + 1] = pos;
  }
  free(tbuf);
  return (int64_t)pos;
}
