/*
 * tcrnet -- thresholded all-pairs Levenshtein networks of CDR3-beta strings on
 * AMD Instinct MI355X (gfx950).
 *
 * What is computed (paper: Ehrlich et al., "Large-scale GPU-based network
 * analysis of the human T-cell receptor repertoire", Methods):
 *   - "Levenshtein distance", Eq. (levenshtein): unit-cost insertions,
 *     deletions and substitutions; row/column 0 of the recursion stand for the
 *     empty prefix.
 *   - "TCR network": one node per input sequence; nodes i and j are joined iff
 *     lev(s_i, s_j) <= l_max (here: k).  Equal strings are distinct nodes
 *     joined by a distance-0 edge.  No self-pairs.
 *   - "Adjacency matrix": undirected edges, reported once as (i, j), i < j.
 *   - "Overview of network theory concepts": degree d(u) = sum_v A_uv.
 *
 * Conventions for every call:
 *   - Node ids are 0-based input positions (the paper numbers from 1).
 *   - Edge lists are arrays of 2*E uint32 values (i0, j0, i1, j1, ...) with
 *     i < j, sorted lexicographically by (i, j), without duplicates.
 *   - Degrees are int32, one per node.
 *   - Sequences are ASCII over the 20 amino-acid letters
 *     A R N D C Q E G H I L K M F P S T W Y V (paper, Methods, "Combination of
 *     amino acids"); each has 1..32 residues (one 32-bit bit-vector word).
 *     Anything else is TCRNET_EINVAL.
 *   - 0 <= k <= 31.
 *   - Every call returns a status (TCRNET_OK = 0).  On error, output pointers
 *     are set to NULL, nothing is returned half-built, and
 *     tcrnet_last_error() describes the failure (thread-local).
 *   - Input buffers are borrowed only for the duration of a call and copied.
 *     Results are owned by the library until the matching *_free call.
 *   - A context may be used from one thread at a time.  An index may be used
 *     from several threads (its calls serialize internally where needed).
 */
#ifndef TCRNET_H
#define TCRNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(TCRNET_BUILDING)
#define TCRNET_API __attribute__((visibility("default")))
#else
#define TCRNET_API
#endif

/* ------------------------------------------------------------------ status */
#define TCRNET_OK 0
#define TCRNET_EINVAL 1  /* bad argument: NULL pointer, residue outside the
                            alphabet, length 0 or > 32, k outside [0, 31] */
#define TCRNET_ENOMEM 2  /* device or host allocation failed, or a request
                            does not fit the serving memory budget */
#define TCRNET_EDEVICE 3 /* HIP runtime error (message in tcrnet_last_error) */
#define TCRNET_ESTATE 4  /* call not valid in the object's current state
                            (unknown ticket, result already taken, ...) */
#define TCRNET_ETRUNC 5  /* caller-provided output buffer too small; the
                            required size is returned, the call may be
                            repeated with a larger buffer */

#define TCRNET_MAX_LEN 32
#define TCRNET_MAX_K 31
/* Largest sequence set: one build's input (all repertoires of a batched
 * build together), and a serving index including every insert. */
#define TCRNET_MAX_SEQS (1u << 28)

typedef struct tcrnet_ctx tcrnet_ctx;
typedef struct tcrnet_graph tcrnet_graph;
typedef struct tcrnet_index tcrnet_index;
typedef struct tcrnet_result tcrnet_result;

/* A set of n sequences: n+1 byte offsets into `data` (offsets[0] need not be
   0; sequence i is data[offsets[i] .. offsets[i+1])).  Host memory. */
typedef struct {
  const char* data;
  const uint64_t* offsets;
  uint32_t n;
} tcrnet_seqs;

/* Options; a zero field selects the default.  Pass NULL for all defaults. */
typedef struct {
  uint32_t texts_per_item;  /* texts per work item of the pair kernel
                               (0: autotuned table / about N/195 rounded
                               down to a power of two in 256..16384, N the
                               sequences of the launch, doubled at k <= 1
                               from N = 150,000; 512 for a serving index) */
  uint32_t waves_per_simd;  /* resident waves per SIMD of the persistent
                               pair kernel (0: autotuned table / 6, what
                               the kernel's registers allow) */
  uint64_t edge_capacity;   /* initial edge buffer capacity in edges (0: sized
                               from N); too small only costs one re-run */
  uint64_t hbm_budget;      /* serving: bytes of device memory that admitted
                               requests may hold at once (0: 1/4 of free) */
  uint32_t max_inflight;    /* serving: requests on the device at once (0: 4) */
  uint32_t flags;           /* TCRNET_F_* */
} tcrnet_opts;

#define TCRNET_F_NO_AUTOTUNE 1u   /* never consult or run the autotuner */
#define TCRNET_F_PEQ_LDS 2u       /* keep pattern bit masks in LDS (default: in
                                     VGPRs) */
#define TCRNET_F_NO_PACK 4u       /* one pattern per lane also for patterns of <= 16
                                     residues (default: two, in 16-bit halves) */
#define TCRNET_F_PEQ_VGPR 8u      /* keep pattern bit masks in VGPRs (the
                                     default) */
#define TCRNET_F_COUNT_WORK 16u   /* run the pair kernel's counting variant: the
                                     same walk, also counting visited texts and
                                     wave text steps (tcrnet_build_info); slower,
                                     for measurement only */

/* Create a context on HIP device `device` (stream, workspace, options).
   Fails with TCRNET_EDEVICE if the device is absent or not gfx950. */
TCRNET_API int32_t tcrnet_ctx_create(int32_t device, const tcrnet_opts* opts, tcrnet_ctx** out);
TCRNET_API int32_t tcrnet_ctx_destroy(tcrnet_ctx* ctx);

/* Message of the last failed call on this thread ("" if none). */
TCRNET_API const char* tcrnet_last_error(void);
/* Static name of a status code. */
TCRNET_API const char* tcrnet_status_string(int32_t status);
/* Library version string. */
TCRNET_API const char* tcrnet_version(void);
/* Failure injection for tests of the error paths: after `after` more
   successful device or pinned-host allocations made by the library (in any
   thread), the next one fails as if the memory were exhausted (once); the
   call then returns TCRNET_ENOMEM with no result.  after < 0 disarms. */
TCRNET_API void tcrnet_debug_fail_alloc(int64_t after);

/* ------------------------------------------------------------ plain build
 * The whole network of `seqs` at threshold k (paper, "TCR network" and
 * "GPU-based network generation": all pairs, thresholded, sparse output).
 * Inputs are copied to the device once; edges and degrees are copied back.
 * N = 0 and N = 1 are valid and give E = 0. */
TCRNET_API int32_t tcrnet_build(tcrnet_ctx* ctx, const tcrnet_seqs* seqs, int32_t k,
                                tcrnet_graph** out);

/* Same computation on device-resident input and output, with no host copy
 * of sequences or results and no device allocation once the context's
 * workspace has grown to the input size.
 *   d_data, d_offsets (n+1 entries): device pointers, valid during the call.
 *   stream: a hipStream_t the work is ordered on (NULL: the context's stream).
 *   d_pairs: device buffer of 2 * pair_capacity uint32 (edge list as above).
 *   d_degree: device buffer of n int32.
 *   *n_edges: receives E.  If E > pair_capacity the call returns
 *   TCRNET_ETRUNC and only *n_edges is meaningful (d_pairs and d_degree hold
 *   partial data); repeat the call with pair_capacity >= E.
 * The call returns after the work completes (it reads the edge count). */
TCRNET_API int32_t tcrnet_build_device(tcrnet_ctx* ctx, const char* d_data, const uint64_t* d_offsets,
                                       uint32_t n, int32_t k, void* stream, uint32_t* d_pairs,
                                       uint64_t pair_capacity, int32_t* d_degree, uint64_t* n_edges);

/* tcrnet_build_device for callers that cannot allocate device memory: code
 * under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, result and errors as tcrnet_build_device, but
 * the call allocates nothing (no device, pinned or library allocation): every
 * intermediate buffer is carved from one static device array of
 * TCRNET_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on
 * holds from the context's creation until the process ends.
 *   Limit: the intermediate buffers of n sequences and pair_capacity edges
 *   (about 232 bytes a sequence plus 25 bytes an edge slot, with the work
 *   plan and sort state) must fit the array; otherwise the call returns
 *   TCRNET_EINVAL before any device work, naming the bytes it would need.
 *   Every call on one GPU shares that GPU's array and leaves its contents
 *   behind (the call clears what must start at zero itself): calls that
 *   overlap on one GPU, from any thread, context or stream, race and give
 *   undefined results.  Serialise them. */
#define TCRNET_NOALLOC_SCRATCH_BYTES (64u << 20)
TCRNET_API int32_t tcrnet_build_device_noalloc(tcrnet_ctx* ctx, const char* d_data, const uint64_t* d_offsets,
                                               uint32_t n, int32_t k, void* stream, uint32_t* d_pairs,
                                               uint64_t pair_capacity, int32_t* d_degree, uint64_t* n_edges);

/* Multi-threshold build: every pair with lev <= k_max, with its exact
 * distance (paper, Results, "LCC transition": networks for several l_max).
 * The network at any k <= k_max is the set of edges with distance <= k.
 * Degrees are those at k_max.  The distances are read with
 * tcrnet_graph_distances. */
TCRNET_API int32_t tcrnet_build_weighted(tcrnet_ctx* ctx, const tcrnet_seqs* seqs, int32_t k_max,
                                         tcrnet_graph** out);

/* Many independent repertoires (each its own network, own 0-based ids) in
 * one launch sequence: one persistent pair kernel over all repertoires' work
 * items, captured in a HIP graph.  outs[r] receives repertoire r's graph;
 * every graph's tcrnet_graph_info is that of the one batched launch. */
TCRNET_API int32_t tcrnet_build_batch(tcrnet_ctx* ctx, const tcrnet_seqs* reps, uint32_t n_reps,
                                      int32_t k, tcrnet_graph** outs);

/* Host views of a graph (valid until tcrnet_graph_free). */
TCRNET_API int32_t tcrnet_graph_edges(const tcrnet_graph* g, const uint32_t** pairs, uint64_t* n_edges);
TCRNET_API int32_t tcrnet_graph_degree(const tcrnet_graph* g, const int32_t** degree, uint32_t* n);
/* The views of graphs[0 .. n) in one call, for callers that wrap the hundreds
 * of graphs of a batched build: entry i of each output array (n entries
 * each, caller-owned) is what tcrnet_graph_edges (pairs, n_edges),
 * tcrnet_graph_degree (degree, n_nodes) and tcrnet_graph_distances (dist:
 * NULL for a graph without distances) give graphs[i].  The views stay valid
 * until that graph is freed.  Errors: TCRNET_EINVAL for a NULL array (with
 * n > 0) or a NULL graph (then no output is written). */
TCRNET_API int32_t tcrnet_graphs_views(tcrnet_graph* const* graphs, uint32_t n, const uint32_t** pairs,
                                       uint64_t* n_edges, const int32_t** degree, uint32_t* n_nodes,
                                       const uint8_t** dist);
/* Edge distances (E bytes, aligned with the edge list) of a weighted build;
   TCRNET_ESTATE for other graphs. */
TCRNET_API int32_t tcrnet_graph_distances(const tcrnet_graph* g, const uint8_t** dist, uint64_t* n_edges);
/* Counters of the build that made `g`: evaluated (length-compatible) pairs,
   pair-kernel time in milliseconds (HIP events around the pair kernel on its
   stream), whole-build time in ms (events around all device work), the
   number of pipeline launches (more than 1 after an edge-buffer overflow),
   and the schedule used. */
typedef struct {
  uint64_t evaluated_pairs;
  double pair_kernel_ms;
  double build_ms;
  uint32_t pair_launches;
  uint32_t texts_per_item;
  uint32_t waves_per_simd;
  uint32_t peq_lds;
  uint32_t pack;         /* 1: patterns of <= 16 residues ran two per lane */
  uint32_t tuned;        /* 1: the schedule came from the autotuner */
  uint32_t graph_captured; /* batched builds: 1 if this call captured a new
                              HIP graph (first call, or a changed shape or
                              buffer), 0 if it replayed the previous one */
  uint32_t work_counted;   /* 1: the three counts below are valid
                              (TCRNET_F_COUNT_WORK) */
  uint64_t visited_texts;  /* texts the pair kernel's walk visited */
  uint64_t wave_steps;     /* wave text steps (Myers/Hyyro steps of a wave) */
  uint64_t wave_steps_packed; /* of which with two patterns per lane */
} tcrnet_build_info;
TCRNET_API int32_t tcrnet_graph_info(const tcrnet_graph* g, tcrnet_build_info* info);
/* Counters of the context's most recent build of any kind. */
TCRNET_API int32_t tcrnet_ctx_last_info(const tcrnet_ctx* ctx, tcrnet_build_info* info);
TCRNET_API void tcrnet_graph_free(tcrnet_graph* g);

/* --------------------------------------------------------------- autotune
 * Time candidate pair-kernel schedules and keep the fastest in the context
 * for later launches of the same form, size class (bits of the sequence
 * count) and k.  Candidates: texts per work item 256 .. 16384 (powers of
 * two) x resident waves per SIMD {4, 6, 8} x pattern masks in VGPRs or LDS x
 * two patterns per lane on or off (off only, with TCRNET_F_NO_PACK).  Each
 * candidate is timed as the device time of its whole launch sequence, the
 * fastest of two runs.  Results are exact for every candidate (the calls
 * fail with TCRNET_EDEVICE if two candidates disagree on the edge count);
 * only speed differs.  Explicit options (texts_per_item, waves_per_simd,
 * TCRNET_F_PEQ_*) still override a tuned choice; TCRNET_F_NO_AUTOTUNE
 * ignores the table.  The input is borrowed for the call. */
TCRNET_API int32_t tcrnet_autotune(tcrnet_ctx* ctx, const tcrnet_seqs* seqs, int32_t k);
/* The same for batched launches (tcrnet_build_batch): each candidate's
 * launch sequence is captured as a HIP graph and replayed, and its time is
 * that of a replay. */
TCRNET_API int32_t tcrnet_autotune_batch(tcrnet_ctx* ctx, const tcrnet_seqs* reps, uint32_t n_reps, int32_t k);

typedef struct {
  uint32_t texts_per_item;
  uint32_t waves_per_simd;
  uint32_t peq_lds;
  uint32_t pack;
  double ms;  /* measured device time of the chosen schedule */
} tcrnet_tune_entry;
/* The tuned schedule for (form: batch = 1 or plain = 0, n sequences, k);
   TCRNET_ESTATE if none. */
TCRNET_API int32_t tcrnet_autotune_get(const tcrnet_ctx* ctx, int32_t batch, uint64_t n, int32_t k,
                                       tcrnet_tune_entry* out);
/* Persist the context's table as JSON (written to path + ".tmp", then
   renamed); each entry names the device's arch (e.g. "gfx950") and CU
   count, the form, size class and k, and the schedule. */
TCRNET_API int32_t tcrnet_autotune_save(const tcrnet_ctx* ctx, const char* path);
/* Merge the entries of a saved table that were measured on a device of the
   same arch and CU count into the context's table; *n_loaded (may be NULL)
   receives their number.  TCRNET_EINVAL for an unreadable or malformed file
   (the context's table is then unchanged). */
TCRNET_API int32_t tcrnet_autotune_load(tcrnet_ctx* ctx, const char* path, uint32_t* n_loaded);

/* ------------------------------------------------------------- diagnostics
 * Measured 32-bit VALU issue rate of the context's device, in lane-
 * instructions per second: eight waves per SIMD on every CU run independent
 * chains of v_xor_b32 / v_add_u32 (plain 32-bit integer VALU instructions of
 * the bit-vector step's kind) for a few tens of ms, timed with events on the
 * context's stream.  On gfx950 two waves of a SIMD issue such instructions
 * in the same 4-clock window, so their nominal peak is CUs x 128 lanes x
 * clock; this call is its measured counterpart.
 * *seconds (may be NULL) receives the timed duration.  Allocates and frees a
 * 2 MB scratch buffer; errors: TCRNET_EINVAL (NULL ctx or rate pointer),
 * TCRNET_EDEVICE. */
TCRNET_API int32_t tcrnet_valu_peak(tcrnet_ctx* ctx, double* lane_instr_per_s, double* seconds);

/* Measured issue rate of each of a fixed list of 32-bit VALU instruction
 * forms, in lane-instructions per second, the same way as tcrnet_valu_peak
 * (eight waves per SIMD, eight independent chains a wave, one form at a
 * time): the forms the bit-vector step, its miss-word update and its within-k
 * tests compile to (v_xor_b32, v_add_u32, v_and_b32, v_bitop3_b32,
 * v_pk_add_u16, v_add3_u32, v_or3_b32, v_min_u32, v_min_u32 with an SDWA
 * operand, v_lshlrev_b32, v_bcnt_u32_b32, v_cmp_eq_u32 into VCC).  They price
 * the pair kernel's instruction mix: on gfx950 some forms issue at about twice
 * the rate of others.  rates[i] receives form i, named by
 * tcrnet_valu_form_name(i) (NULL past the last form); *n_forms receives the
 * number of forms.  Runs about 50 ms of kernels on the context's stream and
 * allocates a 2 MB scratch buffer.  Errors: TCRNET_EINVAL (NULL ctx or
 * n_forms, or capacity below the number of forms: *n_forms is still set),
 * TCRNET_EDEVICE. */
TCRNET_API const char* tcrnet_valu_form_name(uint32_t i);
TCRNET_API int32_t tcrnet_valu_rates(tcrnet_ctx* ctx, double* rates, uint32_t capacity, uint32_t* n_forms);

/* ------------------------------------------------------------------ serving
 * A resident repertoire on the device (sorted into length buckets), with its
 * degree array at threshold k_index.  Query batches compare new sequences
 * against the repertoire at their own k; insert batches also add their
 * sequences (new ids N_old .. N_old+M-1) and their edges at k_index.
 * (Paper, "Distinguishing antigens with network analysis": cognate sequences
 * are placed into an existing network.) */
TCRNET_API int32_t tcrnet_index_create(tcrnet_ctx* ctx, const tcrnet_seqs* seqs, int32_t k_index,
                                       tcrnet_index** out);
TCRNET_API int32_t tcrnet_index_size(tcrnet_index* idx, uint32_t* n);
/* Host copy of the current degree array (valid until the next call on idx). */
TCRNET_API int32_t tcrnet_index_degree(tcrnet_index* idx, const int32_t** degree, uint32_t* n);
TCRNET_API void tcrnet_index_free(tcrnet_index* idx);

/* Synchronous query: pairs (q, r) with lev(q_q, R_r) <= k, sorted; r are
   repertoire ids.  counts[q] = number of such r. */
TCRNET_API int32_t tcrnet_query(tcrnet_index* idx, const tcrnet_seqs* q, int32_t k, tcrnet_result** out);
/* Synchronous insert: adds q to the repertoire.  Result pairs are the new
   edges (i, j), i < j, at k_index (j is always a new id); counts[q] is the
   degree of new node N_old + q; the degrees of old nodes are updated. */
TCRNET_API int32_t tcrnet_insert(tcrnet_index* idx, const tcrnet_seqs* q, tcrnet_result** out);

/* Asynchronous form with continuous batching.  A request is admitted when a
   device slot and enough of the memory budget are free; requests admitted
   while others run overlap on the device.  Each request sees the repertoire
   as of its admission: the initial sequences plus every insert admitted
   before it.  `insert` = 1 makes it an insert (k is then ignored and the
   index's k is used). */
TCRNET_API int32_t tcrnet_submit(tcrnet_index* idx, const tcrnet_seqs* q, int32_t k, int32_t insert,
                                 uint64_t* ticket);
/* Block until the request finishes; hands over its result (once). */
TCRNET_API int32_t tcrnet_wait(tcrnet_index* idx, uint64_t ticket, tcrnet_result** out);

typedef struct {
  uint64_t seqno;         /* admission order */
  uint32_t snapshot_size; /* repertoire size the request saw */
  uint32_t is_insert;
  double latency_ms;      /* submit -> result ready on the host */
  double device_ms;       /* first launch -> last kernel done (HIP events on
                             the request's stream: includes time its kernels
                             waited for others to free the device) */
  double queue_ms;        /* submit -> admission (waiting for a slot or
                             device-memory budget, behind earlier requests) */
  double admit_ms;        /* host work of the admission (staging, launches) */
  uint32_t attempts;      /* pair-kernel launches (2 after an edge overflow) */
  uint32_t parts;         /* planned parts (snapshot segments + own set) */
} tcrnet_result_info;

TCRNET_API int32_t tcrnet_result_pairs(const tcrnet_result* r, const uint32_t** pairs, uint64_t* n);
TCRNET_API int32_t tcrnet_result_counts(const tcrnet_result* r, const int32_t** counts, uint32_t* n);
TCRNET_API int32_t tcrnet_result_info_get(const tcrnet_result* r, tcrnet_result_info* info);
TCRNET_API void tcrnet_result_free(tcrnet_result* r);

/* ---------------------------------------------------------------- analysis
 * Network analysis on an edge list of n nodes (host arrays; pairs may come
 * from any build above).  Paper, Methods, "Overview of network theory
 * concepts" (connected subgraphs, largest connected component, cluster
 * sizes), "Percolation transition" (site percolation: node removal) and
 * "Computing LCC" (LCC after removal).  Every pair must name nodes < n
 * (else TCRNET_EINVAL); duplicate pairs and self loops are allowed. */
typedef struct {
  uint32_t n_components; /* number of connected components */
  uint32_t lcc_size;     /* nodes in the largest one (0 when n = 0) */
} tcrnet_cc_info;

/* Components: labels[i] (n entries, may be NULL) = smallest node id of i's
   component; sizes[i] (n entries, may be NULL) = size of the component whose
   label is i, 0 if i is not a label.  The cluster-size distribution is the
   histogram of the nonzero sizes. */
TCRNET_API int32_t tcrnet_components(tcrnet_ctx* ctx, const uint32_t* pairs, uint64_t n_edges, uint32_t n,
                                     uint32_t* labels, uint32_t* sizes, tcrnet_cc_info* info);

/* Site percolation: order is a permutation of 0..n-1 (the random removal
   order, drawn by the caller); for each q < n_runs the nodes
   order[0 .. removed[q]) are removed (removed[q] <= n) and lcc[q] receives
   the size of the largest connected component of the rest. */
TCRNET_API int32_t tcrnet_robustness(tcrnet_ctx* ctx, const uint32_t* pairs, uint64_t n_edges, uint32_t n,
                                     const uint32_t* order, const uint32_t* removed, uint32_t n_runs, uint32_t* lcc);

/* Normalised LCC sizes of a percolation curve (paper, Methods, "Computing
   LCC"): with p = removed[q] / n,
     norm1[q] = LCC_norm,1(p) = lcc[q] / ((1 - p) n)   (0 when no node is left)
     norm2[q] = LCC_norm,2(p) = LCC_norm,1(p) / LCC_norm,1(0)
   (norm2 requires removed[0] = 0; if LCC_norm,1(0) = 0 it is norm1).
   Host arrays of n_runs entries; norm1 or norm2 may be NULL.  TCRNET_EINVAL
   if removed[q] > n or lcc[q] > n - removed[q].  Host arithmetic only. */
TCRNET_API int32_t tcrnet_lcc_norm(const uint32_t* lcc, const uint32_t* removed, uint32_t n_runs, uint32_t n,
                                   double* norm1, double* norm2);

/* Degree statistics of a canonical edge list (i < j, sorted by (i, j),
   distinct: the output of the builds), paper, Methods, "Overview of network
   theory concepts": degree d(u), degree distribution p_d, average neighbour
   degree <d_nn>, degree assortativity r; Results: clustering coefficient.
     degree[n]        d(u)                                      (may be NULL)
     deg_count[h]     number of nodes with degree d, d < hist_len
     nbr_deg_sum[h]   sum over nodes u of degree d of the degrees of u's
                      neighbours, so <d_nn>(d) = nbr_deg_sum[d] / (d count[d])
     clustering[n]    2 T(u) / (d (d - 1)), T(u) = triangles through u, 0 for
                      d < 2                                     (may be NULL)
   A maximum degree >= hist_len gives TCRNET_ETRUNC with out->max_degree set
   (the histogram arrays then miss the larger degrees). */
typedef struct {
  uint32_t max_degree;
  uint64_t triangles;
  double assortativity;   /* Pearson correlation of the end degrees of edges */
  double avg_clustering;  /* mean of clustering[] over all n nodes */
  uint64_t sum_jk;        /* exact sums behind r over edges (j, k) */
  uint64_t sum_j_plus_k;
  uint64_t sum_j2_plus_k2;
} tcrnet_stats;

TCRNET_API int32_t tcrnet_graph_stats(tcrnet_ctx* ctx, const uint32_t* pairs, uint64_t n_edges, uint32_t n,
                                      int32_t* degree, uint64_t* deg_count, uint64_t* nbr_deg_sum, uint32_t hist_len,
                                      double* clustering, tcrnet_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* TCRNET_H */
