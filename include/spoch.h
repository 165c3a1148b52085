/*
 * spoch.h -- C ABI of the MI355X (gfx950) contraction-hierarchy library.
 *
 * The library builds a contraction hierarchy (CH) of a directed graph with
 * non-negative integer arc weights by round-synchronous contraction, the
 * method of Wan et al., "Parallel Contraction Hierarchies Can Be Efficient
 * and Scalable" (ICS 2025), and answers batches of s-t distance queries on
 * it.  Every step runs as HIP kernels on the GPU; there is no CPU fallback.
 *
 * Problem statement followed (Sec. "Preliminaries" and "Contraction
 * Hierarchies"): input G = (V, E, w) with w: E -> non-negative weights; the
 * CH G_CH = (V, E_CH) preserves all pairwise distances; a query from s to t
 * is answered by a bidirectional search over upward arcs (Sec. "Query on
 * Contraction Hierarchies").
 *
 * Conventions for every entry point
 *   - Return value: CH_OK (0) or a negative CH_E_* code.  On error no
 *     out-parameter is written and ch_last_error() describes the failure
 *     (thread-local, valid until the next call on the same thread).
 *   - Vertex ids are uint32 in [0, n); n <= 0xFFFFFFFE.
 *   - Arc weights are uint32 in [0, 0xFFFFFFFE]; 0xFFFFFFFF is reserved.
 *     Every witness-search bound and shortcut weight must fit in
 *     [0, 0xFFFFFFFE], else CH_E_OVERFLOW.  Query distances are uint64.
 *   - "Host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device allocations on the current device.  Flags say which.
 *   - The caller owns every array it passes; the library reads inputs during
 *     the call only and never retains a caller pointer.
 *   - The library owns a ch_t from ch_build until ch_free.
 *   - Calls on different ch_t objects may run concurrently on different
 *     streams; calls on the same ch_t must not overlap.
 */
#ifndef SPOCH_H
#define SPOCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define CH_OK 0
#define CH_E_INVALID -1  /* bad argument: NULL, id >= n, weight 0xFFFFFFFF, labels not distinct */
#define CH_E_OOM -2      /* device or host allocation failed */
#define CH_E_OVERFLOW -3 /* a search bound or shortcut weight exceeds 0xFFFFFFFE */
#define CH_E_DEVICE -4   /* HIP runtime error (message in ch_last_error) */
#define CH_E_LIMIT -5    /* max_rounds reached with vertices still uncontracted */
#define CH_E_UNSUPPORTED -6 /* option not implemented by this build */

/* ---- witness-path-search modes ---- */
/* The paper bounds each search by a settled-vertex budget whose value it
 * does not give (Sec. "Step 1: Local Search with Memoization").  Both modes
 * search from source s up to radius D_s = the largest two-arc length
 * w(s,u) + w(u,v) over its targets.
 *   CH_WPS_EXACT: the exact overlay distance of every target.
 *   CH_WPS_HOP:   hop- and distance-bounded: the minimum length over walks
 *                 of at most hop_limit arcs within D_s, computed level by
 *                 level (level k uses only level k-1 values); a target no
 *                 such walk reaches gets no memo entry.  Distances of the
 *                 finished CH stay exact (a missing witness only adds a
 *                 shortcut). */
#define CH_WPS_EXACT 0
#define CH_WPS_HOP 1
/* The paper's literal bound (Sec. "Step 1: Local Search with Memoization",
 * Alg. 4): a search settles vertices in (distance, label) order, s first,
 * and stops after settle_limit settled vertices or once every target is
 * settled; only settled targets get a memo entry (a target left unsettled
 * gets a shortcut).  Radius D_s as above. */
#define CH_WPS_SETTLED 2

/* ---- flags ---- */
#define CH_F_INPUT_ON_DEVICE 0x1u /* ch_graph_t arrays are device pointers */
#define CH_F_STATS 0x2u           /* collect per-round counters and timings */
#define CH_F_NO_QUERY_INDEX 0x4u  /* skip the rank-space CSR (ch_query_batch then fails) */

#define CH_Q_ON_DEVICE 0x1u       /* s, t, dist of ch_query_batch are device pointers */
/* Waves that share one query in the first query tier (1, 2, 4
 * or 8; 0 = the default, 4).  Results do not depend on it. */
#define CH_Q_WAVES(nw) ((uint32_t)(nw) << 8)
/* Level window of the query's search steps (1 .. 254 levels; 0 or 255 =
 * none, every flagged vertex is expanded at once, the default).  A step expands the reached
 * vertices whose CH level is within the window above the lowest level
 * still to be expanded, so fewer vertices are expanded twice; a window
 * covering every level is the same as none.  Results do not depend on it. */
#define CH_Q_LEVEL_WINDOW(w) ((uint32_t)(w) << 12)
/* By default a query skips every vertex and arc whose distance from its end
 * is not below the shortest s-t path met so far (no such vertex can be on a
 * shorter path), and does not expand a vertex whose distance is beaten by a
 * path through a higher-ranked neighbour (stall-on-demand: such a distance
 * is not exact, so no shortest path leaves the vertex upward with it); both
 * keep distances exact.  CH_Q_FULL_CLOSURE expands
 * both upward search spaces completely instead; ch_query_batch_stats always
 * does, so its visited counts (the sizes of the two search spaces) do not
 * depend on timing. */
#define CH_Q_FULL_CLOSURE (1u << 20)
/* Count the adjacency rows and arcs the batch reads, and its core-table
 * reads (ch_get_query_stats); ch_query_batch_stats always counts. */
#define CH_Q_COUNT (1u << 21)
/* Tier a batch starts in: 1 = LDS tables for small search spaces, 2 = LDS
 * tables for large ones, 3 = tables in global memory; 0 = chosen by the
 * library (tier 2 for hierarchies deeper than 256 levels, else tier 1, and
 * one tier up for later batches when more than half of a batch moved on).
 * Queries that outgrow a tier still move on.  Results do not depend on it. */
#define CH_Q_FIRST_TIER(t) ((uint32_t)(t) << 22)
/* The first and second tiers normally stop both searches at the 1024 and
 * 4096 highest ranks and finish with a table of the exact distances among
 * them (built once per CH, 4 MB and 64 MB, at the first pruned batch in
 * which at least 4096 queries enter the tier, and used by every later one;
 * skipped when a distance in it could pass 32 bits; ch_query_batch_noalloc
 * uses it only if it exists).  CH_Q_NO_CORE searches without it.  Results
 * do not depend on it. */
#define CH_Q_NO_CORE (1u << 26)

/* Input graph in CSR form, arcs grouped by tail vertex.
 *   offsets[n+1]: offsets[0] = 0, non-decreasing, offsets[n] = m
 *   dst[m]:       head of each arc, < n
 *   w[m]:         weight of each arc, <= 0xFFFFFFFE
 *   labels[n]:    optional distinct tie-break labels (NULL: derived from
 *                 the vertex id and params.seed by the MurmurHash3 32-bit
 *                 finaliser, fmix32(v ^ lo32(seed) ^ hi32(seed))).
 * Self-loops are dropped and parallel arcs keep the smallest weight. */
typedef struct {
  uint32_t n;
  uint64_t m;
  const uint64_t *offsets;
  const uint32_t *dst;
  const uint32_t *w;
  const uint32_t *labels;
} ch_graph_t;

typedef struct {
  uint32_t wps_mode;   /* CH_WPS_EXACT, CH_WPS_HOP or CH_WPS_SETTLED             */
  uint32_t max_rounds; /* 0: no limit; else CH_E_LIMIT after that many rounds    */
  uint64_t seed;       /* seed of the default labels                            */
  uint32_t flags;      /* CH_F_*                                                */
  uint32_t group;      /* lanes per item in the round kernels: 0 = automatic,   */
                       /* else 4, 8, 16, 32 or 64 (changes speed, never results) */
  void *stream;        /* hipStream_t to run on (borrowed); NULL = the library's */
  /* First-tier witness-search kernel (lanes x LDS table slots) for rounds
   * whose overlay has average out-degree <= dense_deg10 / 10 ("sparse") and
   * for the others ("dense"): CH_LS_AUTO or one of CH_LS_16x128 ...
   * CH_LS_64x2048.  dense_deg10 = 0 means 50.  These change speed only. */
  uint32_t ls_sparse;
  uint32_t ls_dense;
  uint32_t dense_deg10;
  uint32_t priority;   /* CH_PRIO_PLAIN (edge difference, Alg. 5) or CH_PRIO_LEARNED */
  const float *mlp;    /* CH_PRIO_LEARNED: CH_MLP_PARAMS weights, host memory      */
  uint32_t hop_limit;  /* CH_WPS_HOP: arcs per witness walk, >= 1 (else ignored)  */
  /* Exact mode: once the overlay has at most dense_tail vertices, the
   * distances of all its pairs are computed once (contraction keeps them
   * unchanged for the rest of the build) and every later witness search is
   * answered from that table.  0 = 3584; CH_DENSE_TAIL_OFF keeps the
   * searches; at most 4096.  With the plain priority, one graph and no
   * recorded features, those rounds run as a device-driven sequence of
   * launches (CH_LS_TAIL; its scratch is about 24 bytes per vertex pair of
   * the table, e.g. 308 MB at 3584 vertices).  Changes speed only, never
   * results. */
  uint32_t dense_tail;
  /* Integer score weights, used with CH_F_SCORE_WEIGHTS (Sec. "Step 2:
   * Score": the score used in practice combines edge difference, vertex
   * degree, hop distance and hierarchy depth, with weights the paper does
   * not give).  P = k_ed * ED + k_cn * CN + k_depth * depth in 64-bit
   * integers, saturated to int32; ED = the edge difference of Alg. 5, CN =
   * the vertex's contracted neighbours, depth = 1 + the largest depth of a
   * contracted neighbour (0 before any).  Without the flag, and with the
   * learned priority, the weights are 1, 0, 0 (the pure edge difference).
   * Weights change the contraction order, never the distances. */
  int32_t k_ed, k_cn, k_depth;
  /* Tie-break labels when ch_graph_t.labels is NULL (Sec. "Step 3:
   * Select" breaks ties by vertex label): CH_TIE_HASHED_ID (0, the default:
   * fmix32 of the id and seed) or CH_TIE_RAW_ID (label = vertex id; the
   * graph must then carry no labels, else CH_E_INVALID). */
  uint32_t tiebreak;
  uint32_t settle_limit; /* CH_WPS_SETTLED: vertices settled per search (theta), >= 1 */
  /* Exact mode, searches run by a whole wave or block (dense rounds and the
   * larger-table tiers): a search step expands only the frontier vertices
   * whose distance is below the smallest frontier distance plus D_s >> ls_step
   * (distance buckets, so fewer vertices are expanded before their distance
   * is final); 0 = the default, 2; CH_LS_STEP_ALL (32) expands the whole
   * frontier every step.  At most 32.  Changes speed only, never results. */
  uint32_t ls_step;
  /* CH_PRIO_LEARNED: the priority is rint(y * 2^mlp_qbits) of the network
   * output y, saturated to int32; 0 = 16, at most 24.  Fewer bits make more
   * equal priorities (ties go to the label in Select), so more vertices are
   * local minima in a round. */
  uint32_t mlp_qbits;
} ch_params_t;
#define CH_LS_STEP_ALL 32u
#define CH_DENSE_TAIL_OFF 1u
#define CH_TIE_HASHED_ID 0u
#define CH_TIE_RAW_ID 1u

/* ---- learned priority ----
 * An MLP 8 -> 64 -> 64 -> 1 with GELU maps eight features of a rescored
 * vertex to its priority (replacing the edge difference; Select and the rest
 * of the round are unchanged, so distances stay exact).  Features, each
 * squashed as x / (x + c): 0 edge difference (signed, x / (|x| + 8)),
 * 1 contracted neighbours, 2 live in-degree, 3 live out-degree, 4 hierarchy
 * depth (max over contracted neighbours of their depth + 1), 5 vertices
 * reached by the vertex's latest witness search (c = 64), 6 |N(u)|, 7 pairs
 * needing a shortcut; c = 8 unless stated.  GELU(x) = x/2 (1 + T(0.7978845608
 * (x + 0.044715 x^3))), T the [7/6] Pade approximant of tanh, +-1 for
 * |t| >= 4.97.  Evaluated in single precision in a fixed order without fused
 * multiply-add; priority = output x 2^16 rounded to nearest even, saturated
 * to int32.  Weights: W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3. */
#define CH_PRIO_PLAIN 0u
#define CH_PRIO_LEARNED 1u
#define CH_MLP_PARAMS 4801
#define CH_F_RECORD_FEATURES 0x8u /* keep each vertex's features at contraction */
#define CH_F_TAIL_STEPWISE 0x10u  /* table rounds: one launch per step and a host round
                                    * trip per round, as in the earlier rounds (the
                                    * default runs them as one device-driven sequence;
                                    * same results) */
#define CH_F_SCORE_WEIGHTS 0x40u /* score = k_ed ED + k_cn CN + k_depth depth (ch_params_t) */
#define CH_F_PROGRESS 0x80u      /* ch_build prints a line to stderr at most every 5 s
                                  * (round, vertices left, shortcuts so far) */
#define CH_F_NO_GRAPH 0x100u     /* table rounds: launch each batch of rounds directly
                                  * instead of replaying it as a captured HIP graph
                                  * (same results) */
#define CH_F_KEEP_ORDER 0x20u  /* build on the input's vertex numbering (the default
                                * renumbers graphs of 4096 or more vertices into
                                * clusters of nearby vertices first and maps the
                                * result back; same results) */

#define CH_MLP_ON_DEVICE 0x1u     /* x, t, y, prio are device pointers */
#define CH_MLP_BF16 0x2u          /* bf16 weights, inputs, activations and deltas on the
                                   * matrix cores, fp32 accumulation (forward, gradient,
                                   * training) */

typedef struct {
  uint32_t batch;  /* samples per step (<= 2^20), drawn with replacement */
  uint32_t steps;  /* Adam steps */
  float lr, beta1, beta2, eps;
  uint64_t seed;   /* sample-index generator seed */
} ch_mlp_train_params_t;

#define CH_LS_AUTO 0u
#define CH_LS_16x128 1u
#define CH_LS_32x512 2u
#define CH_LS_64x512 3u
#define CH_LS_64x2048 4u
#define CH_LS_TABLE 5u  /* round stats only: searches answered from the all-pairs table */
#define CH_LS_TAIL 6u   /* round stats only: table rounds run as one device-driven sequence */

typedef struct ch_s ch_t;

/* Per-round counters (CH_F_STATS): the sets of one iteration of Alg. 3's
 * loop (Sec. "Our Parallel CH Construction Algorithm") -- the search sources
 * V_W, the rescored vertices V_A, the contracted set V_F and the shortcut set
 * E+ -- and the work of the round's witness searches. */
typedef struct {
  uint32_t alive_before;    /* |V_O| at the start of the round                */
  uint32_t n_sources;       /* |V_W|, witness-search sources                  */
  uint32_t n_affected;      /* |V_A|, vertices rescored                        */
  uint32_t n_selected;      /* |V_F|, vertices contracted                      */
  uint64_t n_targets;       /* sum over sources of the target-set size         */
  uint64_t n_pruned;        /* arcs deleted by the pruning rule                */
  uint64_t n_shortcuts;     /* distinct (v1, v2) shortcut pairs                */
  uint64_t overlay_arcs;    /* arcs in the overlay after the round             */
  /* the next four count the first-tier witness-search kernel only */
  uint64_t rows_expanded;   /* adjacency rows read by the witness searches     */
  uint64_t arcs_scanned;    /* arcs read by the witness searches               */
  uint64_t memo_probes;     /* memo slots read by the local search             */
  uint64_t memo_inserts;    /* memo entries written                            */
  uint32_t n_ls_fallback;   /* sources whose search outgrew the first-tier table */
  uint32_t ls_tier1;        /* first-tier search kernel used (CH_LS_16x128 ...)   */
  float ms_local_search;    /* device time of the first-tier witness-search kernel */
  float ms_total;           /* device time of the whole round (host gaps included) */
  uint32_t n_ls_global;     /* sources searched with tables in global memory   */
  /* the later search tiers: sources that outgrew the first tier's table run
   * again with a block of waves per source, in LDS (n_ls_fallback sources),
   * then with global-memory tables (n_ls_global sources) */
  float ms_ls_blk;          /* device time of the LDS block tier               */
  float ms_ls_global;       /* device time of the global-memory tier (0: none)  */
  uint64_t rows2, arcs2, probes2, inserts2; /* block tier counters, as above    */
  uint64_t rows3, arcs3, probes3, inserts3; /* global tier counters             */
} ch_round_stats_t;

/* Whole-build summary: the size of the CH (Sec. "Contraction Hierarchies":
 * G_CH holds the upward and downward arcs moved out of the overlay at
 * contraction, Alg. 7) and of the build. */
typedef struct {
  uint32_t n;
  uint32_t rounds;
  uint64_t m_input;         /* arcs after dropping self-loops and duplicates  */
  uint64_t up_arcs;         /* arcs of the upward graph                       */
  uint64_t down_arcs;       /* arcs of the downward graph                     */
  uint64_t shortcuts;       /* sum over rounds of n_shortcuts                 */
  uint64_t memo_entries;
  double ms_build;          /* device time of the build, upload excluded      */
} ch_summary_t;

/* Build the CH of `g`.  Sec. "Our Parallel CH Construction Algorithm",
 * Alg. 3: rounds of LocalSearch (Alg. 4), Score (Alg. 5), Select (Alg. 6)
 * and Contract (Alg. 7) until the overlay is empty, then Postprocessing
 * (rank by level, then score, then label).
 *   g:   input graph; host arrays, or device arrays with CH_F_INPUT_ON_DEVICE
 *   p:   parameters (NULL = defaults: exact mode, no round limit, seed 0)
 *   out: receives the new ch_t (library-owned; release with ch_free)
 * Runs on p->stream and returns after the build has finished on the GPU.
 * Errors: CH_E_INVALID (bad graph or parameters), CH_E_OVERFLOW, CH_E_OOM,
 * CH_E_DEVICE, CH_E_LIMIT, CH_E_UNSUPPORTED. */
int ch_build(const ch_graph_t *g, const ch_params_t *p, ch_t **out);

/* Build the CHs of k independent graphs in one pass of the round loop (the
 * graphs become one disjoint union; every rule is local to a graph and
 * every tie uses that graph's own labels).  outs[i] is exactly the CH that
 * ch_build gives gs[i] alone; its summary has that graph's rounds, arcs and
 * shortcuts (memo_entries 0, ms_build of the whole batch); per-round stats
 * are not kept.
 *   gs:   k graphs (host arrays, or device arrays with CH_F_INPUT_ON_DEVICE);
 *         either every graph has labels or none has (then each graph gets
 *         the default labels of its local ids); labels need only be
 *         distinct within a graph
 *   p:    parameters as for ch_build (NULL = defaults)
 *   outs: k entries receive library-owned CHs (each released with ch_free);
 *         they run on p->stream (NULL: the default stream)
 * Errors: as ch_build; also CH_E_UNSUPPORTED when the union has more than
 * 0xFFFFFFFE vertices or 2^32 - 1 arcs.  On error no CH is returned. */
int ch_build_batch(const ch_graph_t *gs, uint32_t k, const ch_params_t *p, ch_t **outs);

/* Distances of q s-t pairs on the CH (Sec. "Query on Contraction
 * Hierarchies"): dist[i] = min over v of d_up(s_i, v) + d_down(v, t_i),
 * which equals the shortest s_i -> t_i distance in the input graph;
 * 0 when s_i == t_i, UINT64_MAX when t_i is unreachable.
 *   s, t: q vertex ids each; dist: q entries written by the call (caller-
 *   owned).  All three on the host, or on the device with CH_Q_ON_DEVICE.
 *   stream: hipStream_t (NULL = the CH's stream).
 * Returns after the distances are written.  The CH keeps query scratch and
 * remembers which table size most of the last batch needed (a later batch
 * starts there), so calls on one CH must not overlap.
 * Errors: CH_E_INVALID (NULL, id >= n, no query index), CH_E_OOM,
 * CH_E_DEVICE. */
int ch_query_batch(const ch_t *ch, const uint32_t *s, const uint32_t *t, uint64_t q,
                   uint64_t *dist, uint32_t flags, void *stream);

/* As ch_query_batch, and visited[i] = the number of vertices in the two
 * upward search spaces of the i-th query (q uint32 entries, host or device
 * like dist); both search spaces are expanded completely (CH_Q_FULL_CLOSURE
 * is implied). */
int ch_query_batch_stats(const ch_t *ch, const uint32_t *s, const uint32_t *t, uint64_t q,
                         uint64_t *dist, uint32_t *visited, uint32_t flags, void *stream);

/* One-to-all distances (and many-to-many) on the CH by its two sweeps (Sec.
 * "Query on Contraction Hierarchies": vertices grouped by level as in
 * PHAST; an upward search from each source, then a downward pass over the
 * levels from the top, each vertex taking the minimum over its downward
 * arcs).  Every CH arc joins two levels, so each level's distances are final
 * before the next level reads them; the results are exact distances.
 *   s:    ks source ids
 *   t:    kt target ids, or NULL for every vertex (then kt is ignored and
 *         each row has n entries)
 *   dist: ks rows of (t ? kt : n) uint64 distances, row i for s[i], entry j
 *         for t[j] (or vertex j in original ids); UINT64_MAX = unreachable.
 *   s, t, dist on the host, or on the device with CH_Q_ON_DEVICE.
 * Up to 64 sources share one pass over the levels; the CH keeps a scratch of
 * n x 8 bytes per source of a pass (n x 512 bytes for 64).
 * Errors: CH_E_INVALID (NULL, id >= n, no query index), CH_E_OOM,
 * CH_E_DEVICE. */
int ch_one_to_all(const ch_t *ch, const uint32_t *s, uint32_t ks, const uint32_t *t, uint32_t kt,
                  uint64_t *dist, uint32_t flags, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ch_query_batch_stats
 * without any allocation, with the same results.  s, t, dist and visited
 * (visited may be NULL) must be device arrays: flags must include
 * CH_Q_ON_DEVICE, else CH_E_INVALID.  Every scratch array (counters,
 * overflow lists, the global-memory search tables) lives in one fixed device
 * array of CH_NOALLOC_SCRATCH_BYTES per GPU, reserved where the library is
 * loaded and held until the process ends.  All calls on one GPU share it and
 * it keeps the last call's contents, so calls that overlap on one GPU (from
 * other threads or on other streams) race; calls on one ch_t must not
 * overlap either.  Queries run in passes of 2^20.  Its tables hold upward
 * search spaces of up to 14,336 vertices per direction, then (one query at
 * a time) of up to 917,504 -- every search space of a CH with at most
 * 524,287 vertices; a query with a larger one makes the call return
 * CH_E_LIMIT (ch_query_batch has no such limit).  Distances of other queries
 * may have been written when the call fails.
 * Errors: CH_E_INVALID (NULL, host arrays, id >= n, no query index),
 * CH_E_LIMIT, CH_E_DEVICE. */
#define CH_NOALLOC_SCRATCH_BYTES (96u << 20)
int ch_query_batch_noalloc(const ch_t *ch, const uint32_t *s, const uint32_t *t, uint64_t q,
                           uint64_t *dist, uint32_t *visited, uint32_t flags, void *stream);

/* Counters of the last query batch on a CH (Sec. "Query on Contraction
 * Hierarchies": one forward and one backward upward search per query).
 * Queries start in the tier where most of the previous batch ended; a query
 * whose search outgrows a tier's tables moves to the next tier. */
typedef struct {
  uint64_t queries;          /* queries of the last batch                        */
  uint32_t first_tier;       /* tier (1-4) the batch started in                  */
  uint32_t counted;          /* 1: rows and arcs were counted (a stats batch)    */
  uint64_t tier_queries[4];  /* queries that entered each tier                   */
  float tier_ms[4];          /* device time of each tier's launch (0: not run;   */
                             /* not measured by ch_query_batch_noalloc)          */
  uint64_t rows;             /* adjacency rows read: vertices expanded and
                              * stall-checked, every tier and re-expansion      */
  uint64_t arcs;             /* arcs read (relaxed or stall-checked) plus
                              * core-table entries read, every tier             */
} ch_query_stats_t;

/* Copies the counters of the CH's last query batch into *out (host).
 * Errors: CH_E_INVALID (NULL). */
int ch_get_query_stats(const ch_t *ch, ch_query_stats_t *out);

/* The finished CH (Sec. "Contraction Hierarchies" and "Postprocessing":
 * levels, the rank order by level then score, and the upward and downward
 * arc sets E_up and E_down of Alg. 7, each arc with the middle vertex that
 * unpacks a shortcut).  Copies to host arrays, in original vertex ids.  Any pointer
 * may be NULL to skip that array.
 *   level[n]: round in which the vertex was contracted (0-based)
 *   score[n]: its score when it was selected
 *   rank[n]:  position in the order (level, score, label)
 *   up_*[up_arcs]:     upward arcs (tail -> head, weight, middle vertex or
 *                      UINT32_MAX for an input arc), sorted by (rank of
 *                      tail, rank of head)
 *   down_*[down_arcs]: downward arcs (tail -> head) with rank(tail) >
 *                      rank(head), sorted by (rank of head, rank of tail)
 * Sizes are those of ch_get_summary. */
int ch_export(const ch_t *ch, uint32_t *level, int32_t *score, uint32_t *rank,
              uint32_t *up_tail, uint32_t *up_head, uint32_t *up_w, uint32_t *up_mid,
              uint32_t *down_tail, uint32_t *down_head, uint32_t *down_w,
              uint32_t *down_mid);

/* Copies the whole-build summary into *out (host).  Errors: CH_E_INVALID
 * (NULL). */
int ch_get_summary(const ch_t *ch, ch_summary_t *out);

/* Copy min(cap, rounds) per-round records (filled only with CH_F_STATS)
 * into out (host, cap entries).  Errors: CH_E_INVALID (NULL). */
int ch_get_round_stats(const ch_t *ch, ch_round_stats_t *out, uint32_t cap);

/* Features (8 floats per vertex, original ids) each vertex had when it was
 * contracted; needs CH_F_RECORD_FEATURES at build time.  x: n*8 host floats.
 * Errors: CH_E_INVALID (NULL, or built without recording). */
int ch_export_features(const ch_t *ch, float *x);

/* The network on n feature vectors: y[i] (output, may be NULL) and prio[i]
 * (the int32 priority, may be NULL).  x: n*8 floats; w: CH_MLP_PARAMS
 * weights; host arrays, or device arrays with CH_MLP_ON_DEVICE.  With
 * CH_MLP_BF16 weights, inputs and activations are rounded to bf16
 * (accumulation stays fp32).  Errors: CH_E_INVALID, CH_E_OOM, CH_E_DEVICE. */
int ch_mlp_forward(const float *x, uint64_t n, const float *w, float *y, int32_t *prio,
                   uint32_t flags, void *stream);

/* Gradient of the mean squared error (1/n) sum (f(x_i) - t_i)^2 over all n
 * samples with respect to the weights: grad (CH_MLP_PARAMS host floats),
 * loss (host float, may be NULL).  fp32: sums run in sample order; with
 * CH_MLP_BF16 each wave sums its 32-sample tiles on the matrix cores and the
 * waves' sums are added in wave order; deterministic either way.
 * x (n*8), t (n): host, or device with CH_MLP_ON_DEVICE; w host. */
int ch_mlp_grad(const float *x, const float *t, uint32_t n, const float *w, float *grad,
                float *loss, uint32_t flags, void *stream);

/* Adam on the mean squared error, minibatches drawn with replacement by a
 * counter-based generator (splitmix64 of seed and sample counter).  w (host,
 * CH_MLP_PARAMS) holds the initial weights and receives the trained ones
 * (fp32 master weights and Adam state; CH_MLP_BF16 computes each step's
 * gradient in bf16 as ch_mlp_grad does); losses (host, p->steps floats, may
 * be NULL) receives each step's batch loss.  Deterministic for given inputs. */
int ch_mlp_train(const float *x, const float *t, uint64_t n, float *w,
                 const ch_mlp_train_params_t *p, float *losses, uint32_t flags, void *stream);

/* Release a CH (NULL is ignored). */
void ch_free(ch_t *ch);

/* Message of the last failed call on this thread ("" if none). */
const char *ch_last_error(void);

/* Library version string. */
const char *ch_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPOCH_H */
