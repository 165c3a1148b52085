// builder.hpp -- internal definitions shared by the builder, the query code
// and the C ABI.
#pragma once

#include <string>
#include <vector>

#include "../../include/spoch.h"
#include "prim.hpp"

// The finished contraction hierarchy (library-owned, device-resident).
struct ch_s {
  uint32_t n = 0;
  uint64_t m_input = 0;
  uint32_t rounds = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;

  // per vertex, original ids
  sp::DBuf level, score, label, rank;

  // CH arcs in original ids, sorted as documented by ch_export
  uint64_t nup = 0, ndown = 0;
  sp::DBuf up_t, up_h, up_w, up_m;
  sp::DBuf dn_t, dn_h, dn_w, dn_m;

  // query index in rank space: upward arcs stored at their tail, downward
  // arcs stored at their head (walked head -> tail by the backward search)
  bool has_index = false;
  sp::DBuf q_upoff, q_uparc, q_dnoff, q_dnarc;  // offsets uint32[n+1], arcs uint2{other, w}
  sp::DBuf q_lstart;  // first rank of each level (nlev + 1 entries)
  uint32_t q_nlev = 0;
  sp::DBuf q_wend;    // end of the query's level window at each rank
  uint32_t q_wend_win = 0;  // its window (0: not computed)

  // query scratch
  sp::DBuf q_s, q_t, q_d, q_v, q_ovf, q_ovf2, q_tab, q_gtab, q_ctr;
  int q_first_tier = 1;  // query tier where the previous batch mostly ended
  sp::DBuf q_phast;  // one-to-all sweeps: distances, rank-major, KC sources per vertex
  // core table of the query: exact distances among the q_core_k highest
  // ranks (row-major, q_core_n columns, 0xFFFFFFFF = none); 0 = not built,
  // q_core_state: 0 not tried, 1 built, 2 not usable on this CH
  sp::DBuf q_core, q_core_max;
  uint32_t q_core_k = 0, q_core_n = 0;
  int q_core_state = 0;
  // the first tier's smaller core table (the highest q_core1_k ranks)
  sp::DBuf q_core1;
  uint32_t q_core1_k = 0, q_core1_n = 0;
  int q_core1_state = 0;
  ch_query_stats_t qstats{};              // counters of the last query batch

  // features at contraction (CH_F_RECORD_FEATURES), 8 floats per vertex
  bool has_rec = false;
  sp::DBuf rec;

  std::vector<ch_round_stats_t> stats;
  ch_summary_t summary{};

  ~ch_s();
};

namespace sp {

// Records the message and returns code (thread-local last error).
int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);

// Build entry (builder.hip).
int build_ch(const ch_graph_t *g, const ch_params_t *p, ch_t **out);
// Postprocess: rank, sorted arc lists, query index (post.hip).  With gof
// (graph of each vertex, kgraphs graphs) the graph id is the major rank key.
int postprocess(ch_s *ch, bool make_index, const uint32_t *gof = nullptr, uint32_t kgraphs = 0);
// Query index of a CH whose arc lists are already sorted by rank (post.hip).
int build_index(ch_s *ch);
// Batched build of k graphs as one disjoint union (builder.hip).
int build_batch(const ch_graph_t *gs, uint32_t k, const ch_params_t *p, ch_t **outs);
// Query batch (post.hip).
int query_batch(const ch_s *ch, const uint32_t *s, const uint32_t *t, uint64_t q,
                uint64_t *dist, uint32_t *visited, uint32_t flags, hipStream_t st);
// One-to-all / many-to-many distances by the CH's two sweeps (phast.hip).
int one_to_all(const ch_s *ch, const uint32_t *s, uint32_t ks, const uint32_t *t, uint32_t kt,
               uint64_t *dist, uint32_t flags, hipStream_t st);
// All-pairs closure of an N x N distance matrix in place (N a multiple of
// 64; 0xFFFFFFFF = none; sums clamped): blocked Floyd-Warshall (builder.hip,
// the kernels of the all-pairs table).  fw_init sets none everywhere and 0
// on the diagonal.
hipError_t fw_init(uint32_t *D, uint32_t N, hipStream_t st);
hipError_t fw_close(uint32_t *D, uint32_t N, hipStream_t st);
// Query batch with every scratch array in a fixed per-GPU array (post.hip).
int query_batch_noalloc(const ch_s *ch, const uint32_t *s, const uint32_t *t, uint64_t q,
                        uint64_t *dist, uint32_t *visited, uint32_t flags, hipStream_t st);

}  // namespace sp
