/*
 * spoch_oracle.h -- interface of the CPU oracle for round-synchronous
 * contraction-hierarchy (CH) construction (Wan et al., "Parallel Contraction
 * Hierarchies Can Be Efficient and Scalable", ICS 2025).
 *
 * TEST INFRASTRUCTURE.  The oracle is a plain, sequential, deliberately slow
 * C implementation that defines the result the GPU library must reproduce
 * bit for bit.  Only the test-suite, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header, table or constant with the
 * GPU library, and the GPU library never calls it.
 *
 * All graph arithmetic is integer: arc weights are uint32 in
 * [0, 0xFFFFFFFE]; 0xFFFFFFFF is reserved as "infinite".  Witness-search and
 * shortcut weights must fit that range (else ORC_E_OVERFLOW); query
 * distances are uint64 with UINT64_MAX meaning "unreachable".
 */
#ifndef SPOCH_ORACLE_H
#define SPOCH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_E_INVALID = -1,  /* bad argument: id >= n, weight 0xFFFFFFFF, labels not distinct */
  ORC_E_OOM = -2,
  ORC_E_OVERFLOW = -3, /* a search bound or shortcut weight exceeds 0xFFFFFFFE */
  ORC_E_LIMIT = -4,    /* max_rounds reached with vertices still alive */
  ORC_E_STATE = -5     /* call not valid in the current state */
};

/* Witness-path-search modes (the paper leaves the search bound open). */
enum {
  ORC_WPS_EXACT = 0,   /* exact overlay distance, search radius D_s      */
  ORC_WPS_HOP = 1,     /* min over walks of <= hop_limit arcs, <= D_s      */
  ORC_WPS_SETTLED = 2  /* Dijkstra stopped after settle_limit pops         */
};

/* Tie-break labels when none are given. */
enum {
  ORC_TIE_HASHED_ID = 0, /* label[v] = fmix32(v ^ lo32(seed) ^ hi32(seed)) */
  ORC_TIE_RAW_ID = 1     /* label[v] = v                                   */
};

/* Priority functions. */
enum {
  ORC_PRIO_PLAIN = 0,   /* edge difference (Alg. 5)                       */
  ORC_PRIO_LEARNED = 1  /* MLP over per-vertex features (see below)       */
};

/* The learned priority is an MLP 8 -> 64 -> 64 -> 1 with GELU, evaluated in
 * IEEE single precision in a fixed order without fused multiply-add.  Its
 * 4801 weights are laid out as W1[64][8], b1[64], W2[64][64], b2[64],
 * W3[64], b3. */
#define ORC_MLP_PARAMS 4801

typedef struct {
  uint32_t wps_mode;
  uint32_t hop_limit;    /* ORC_WPS_HOP: H >= 1                          */
  uint32_t settle_limit; /* ORC_WPS_SETTLED: theta >= 1                  */
  uint32_t max_rounds;   /* 0: no limit                                  */
  uint32_t priority;     /* ORC_PRIO_PLAIN or ORC_PRIO_LEARNED            */
  uint32_t record;       /* keep each vertex's features at contraction   */
  const float *mlp;      /* ORC_MLP_PARAMS weights (learned priority)    */
  /* plain priority = k_ed * ED + k_cn * CN + k_depth * depth, evaluated in
   * 64-bit integers and saturated to int32; ED = edge difference (Alg. 5),
   * CN = contracted neighbours, depth = hierarchy depth (1 + the largest
   * depth of a contracted neighbour).  1, 0, 0 is the pure edge difference. */
  int32_t k_ed, k_cn, k_depth;
  uint32_t tiebreak;     /* ORC_TIE_*; ORC_TIE_RAW_ID needs labels == NULL */
  /* learned priority: P = rint(y * 2^mlp_qbits) of the network output y,
   * saturated to int32 (0 means 16; at most 24).  Fewer bits make more
   * equal priorities, broken by label in Select. */
  uint32_t mlp_qbits;
} orc_params;

typedef struct orc_state orc_state;

/* Per-round counters, one record per finished round. */
typedef struct {
  uint32_t alive_before;   /* |V_O| at the start of the round            */
  uint32_t n_sources;      /* |V_W|                                       */
  uint32_t n_affected;     /* |V_A|                                       */
  uint32_t n_searched;     /* sources with a non-empty target set        */
  uint64_t n_targets;      /* sum over sources of |V_n|                   */
  uint64_t n_pruned;       /* arcs deleted by the pruning rule            */
  uint32_t n_selected;     /* |V_F|                                       */
  uint64_t n_pairs_emitted;/* (v1,v2) pairs that asked for a shortcut     */
  uint64_t n_shortcuts;    /* distinct (v1,v2) in E+                      */
  uint64_t n_absent;       /* Score/Contract lookups with no memo entry   */
  uint64_t n_settled;      /* vertices settled/reached by all searches    */
  uint64_t overlay_arcs;   /* arcs in the overlay after the round         */
} orc_round_stats;

/* Create the oracle state for a graph in CSR form.  `labels` (n distinct
 * values) may be NULL, in which case label[v] = fmix32(v ^ lo32(seed) ^
 * hi32(seed)), fmix32 being the MurmurHash3 32-bit finaliser (a bijection,
 * so the labels are distinct).  Input arrays are copied; self-loops are
 * dropped and parallel arcs keep their minimum weight. */
int orc_create(uint32_t n, uint64_t m, const uint64_t *off, const uint32_t *dst,
               const uint32_t *w, const uint32_t *labels, uint64_t seed,
               const orc_params *p, orc_state **out);
void orc_free(orc_state *st);

/* One iteration of the main loop; returns 1 if vertices remain alive, 0 when
 * the overlay is empty, or a negative error code. */
int orc_round(orc_state *st);
/* Runs rounds until the overlay is empty, then postprocesses. */
int orc_run(orc_state *st);
/* Postprocess (rank by level, score, label; build upward/downward CSR). */
int orc_finish(orc_state *st);

/* ---- state inspection (copies into caller-owned arrays) ---- */
uint32_t orc_n(const orc_state *st);
uint32_t orc_rounds(const orc_state *st);
uint32_t orc_alive_count(const orc_state *st);
void orc_get_labels(const orc_state *st, uint32_t *label);
/* level[v] (round of contraction, UINT32_MAX if alive), score at
 * contraction Pc[v], current score P[v], alive flag. */
void orc_get_vertex_state(const orc_state *st, uint32_t *level, int32_t *pc,
                          int32_t *p, uint8_t *alive);
/* Features (8 floats per vertex) each vertex had when it was contracted
 * (needs params.record). */
int orc_get_features(const orc_state *st, float *x);
/* MLP helpers: the features -> priority map used by the learned priority. */
int32_t orc_mlp_priority(const float *w, const float *x, float *y_out);
/* The same with the output quantised to qbits fractional bits (1 .. 24). */
int32_t orc_mlp_priority_q(const float *w, const float *x, uint32_t qbits, float *y_out);
float orc_gelu(float x);
/* rank[v] after orc_finish. */
int orc_get_rank(const orc_state *st, uint32_t *rank);

/* Overlay arcs of alive vertices (tail, head, weight, mid id or UINT32_MAX). */
uint64_t orc_overlay_count(const orc_state *st);
void orc_get_overlay(const orc_state *st, uint32_t *tail, uint32_t *head,
                     uint32_t *w, uint32_t *mid);
/* Memo entries (source, target, distance), in unspecified order. */
uint64_t orc_memo_count(const orc_state *st);
void orc_get_memo(const orc_state *st, uint32_t *s, uint32_t *t, uint32_t *d);

/* CH arcs.  Upward set: arcs (u -> v) leaving u when u was contracted.
 * Downward set: arcs (v -> u) entering u when u was contracted.  Each record
 * is (tail, head, weight, mid); mid is the middle vertex of a shortcut or
 * UINT32_MAX for an input arc. */
uint64_t orc_up_count(const orc_state *st);
void orc_get_up(const orc_state *st, uint32_t *tail, uint32_t *head, uint32_t *w,
                uint32_t *mid);
uint64_t orc_down_count(const orc_state *st);
void orc_get_down(const orc_state *st, uint32_t *tail, uint32_t *head, uint32_t *w,
                  uint32_t *mid);

void orc_get_round_stats(const orc_state *st, orc_round_stats *out);

/* ---- queries ---- */
/* Bidirectional upward search on the finished CH; returns the distance
 * (UINT64_MAX if t is unreachable) and, if settled != NULL, the number of
 * queue pops of both directions. */
uint64_t orc_query(orc_state *st, uint32_t s, uint32_t t, uint64_t *settled);
int orc_query_batch(orc_state *st, uint64_t q, const uint32_t *s, const uint32_t *t,
                    uint64_t *dist, uint64_t *settled);

/* A finished CH given by its rank order and arc lists (as exported), for
 * queries only: upward arcs (tail -> head) with rank(tail) < rank(head),
 * downward arcs (tail -> head) with rank(tail) > rank(head). */
int orc_load(uint32_t n, const uint32_t *rank, uint64_t nup, const uint32_t *up_tail,
             const uint32_t *up_head, const uint32_t *up_w, uint64_t ndown,
             const uint32_t *dn_tail, const uint32_t *dn_head, const uint32_t *dn_w,
             orc_state **out);

/* Plain Dijkstra on a CSR graph: dist[v] for all v (UINT64_MAX unreachable). */
int orc_dijkstra(uint32_t n, const uint64_t *off, const uint32_t *dst,
                 const uint32_t *w, uint32_t s, uint64_t *dist);

/* Dijkstra that stops after settling max_settled vertices: dist[v] is the
 * distance of every settled vertex and UINT64_MAX for all others. */
int orc_dijkstra_settle(uint32_t n, const uint64_t *off, const uint32_t *dst,
                        const uint32_t *w, uint32_t s, uint64_t max_settled, uint64_t *dist,
                        uint64_t *n_settled);

/* Single-source Dijkstra on the oracle's current overlay (alive vertices). */
int orc_overlay_dijkstra(const orc_state *st, uint32_t s, uint64_t *dist);

/* The default tie-break label of vertex v for a given seed. */
uint32_t orc_default_label(uint32_t v, uint64_t seed);

#ifdef __cplusplus
}
#endif
#endif
