// builder.hip -- host driver of the round-synchronous CH construction
// (Alg. 3 of Wan et al.): ingest, then rounds of LocalSearch, Score, Select
// and Contract on a compacted overlay until no vertex is left, then the
// postprocessing in post.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>

#include "builder.hpp"
#include "mlp.hpp"
#include "round_kernels.hpp"
#include "dense_tail.hpp"
#include "tail.hpp"

namespace sp {

static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}
const char *last_error_msg() { return g_last_error.c_str(); }
void clear_error() { g_last_error.clear(); }

int hip_error(hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return set_error(CH_E_OOM, std::string(what) + ": " + hipGetErrorString(e));
  return set_error(CH_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_error(e_, #expr);  \
  } while (0)
#define TRY(expr)               \
  do {                          \
    int r_ = (expr);            \
    if (r_ != CH_OK) return r_; \
  } while (0)

static int bits_for(uint32_t n) {  // bits to hold values 0..n-1 (at least 1)
  int b = 1;
  while (b < 32 && (1ull << b) < (uint64_t)n) b++;
  return b;
}

static uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Device-side counters read back by the host (one struct, one copy).
struct DevCtr {
  LsCounters ls, ls2, ls3;  // first search tier; block tier; global tier
  unsigned long long bound, pruned, kept;
  uint32_t work1, work2, novf1, novf2;  // persistent scheduling and overflow counts
  uint32_t err, bad;
  uint32_t c32[8];  // scan totals and list counts
};
enum { C_NF = 0, C_UP, C_DN, C_PAIR, C_HEADS, C_NNEW, C_MF, C_MR };

struct OvBuf {
  DBuf foff, farc, fmid, roff, rarc, rmid, gid, P;
  uint32_t n = 0, m = 0;
  void release() {
    foff.release(); farc.release(); fmid.release(); roff.release(); rarc.release();
    rmid.release(); gid.release(); P.release();
  }
};

struct Builder {
  ch_s *ch = nullptr;
  hipStream_t st = nullptr;
  ch_params_t prm{};
  uint32_t n = 0;
  int cus = 256;

  OvBuf ov[2];
  int cur = 0;
  DBuf aflag, aflag_next, wflag, F, S, newA, key, paircnt, newid, cnt, cnt2, cnt3, vw, va, vf;
  DBuf rowb;  // shortcut-row bounds: 4 arrays of the overlay's vertex count
  DBuf memo, memo_spare, alive_g;
  uint64_t mcap = 0, mcount = 0, mwmask = 0;  // slots, entries (upper bound), region width - 1
  DBuf f_cn, f_depth, f_ws, f_feat, mlpw;  // learned-priority feature state
  DBuf cup, cdn, cpair;
  DBuf ekey, ekey_alt, eidx, eidx_alt, ew, elab, emid, ehead, eheads, ukey, uw, umid, rkey,
      rkey_alt, ridx, ridx_alt;
  DBuf ovf1, ovf2, gtabs;
  DBuf prw;  // weights of the arcs pruned in the current round (overlay arc index)
  // all-pairs table of the small overlay (exact mode): matrix tab_N^2,
  // table position of each original id, original id of each position
  DBuf tab_D, tab_pos, tab_gid, tab_posl;
  bool tab_on = false;
  uint32_t tab_N = 0, tab_n0 = 0;
  // device-driven tail (tail.hpp): bitmaps, W / MID, lists, list lengths,
  // SC, touched pairs, per-vertex arrays, flags, vertex lists, state, records
  DBuf t_bits, t_W, t_MID, t_ol, t_il, t_len, t_SC, t_touch, t_vert, t_flags, t_lists, t_ctr,
      t_rec;
  TailCtr *h_tail = nullptr;  // pinned, two copies (one per batch parity)
  // locality order: r_order[new] = input id, r_inv[input id] = new; the
  // input-order labels wait in r_lab until the build is mapped back
  bool renum = false;
  DBuf r_order, r_inv, r_a, r_b, r_c, r_key, r_key_alt, r_val_alt, r_lab;
  hipEvent_t ev_tail[2] = {nullptr, nullptr};
  DBuf dctr, tmp;
  DevCtr *hctr = nullptr;  // pinned
  // round timing: 1 start, 2/3 first search tier, 4 end, 5/6 block tier,
  // 7/8 global tier
  hipEvent_t ev[9] = {};
  hipEvent_t ev_rb = nullptr;  // readback completion
  uint64_t up_cap = 0, dn_cap = 0;
  // disjoint-union batch: graph of each original vertex, per-graph
  // shortcut counters (device), vertex bases (device, k+1)
  struct Batch {
    uint32_t k = 0;
    const uint32_t *gof = nullptr;
    unsigned long long *shortcuts = nullptr;  // per graph
    unsigned long long *m_in = nullptr;       // per graph, arcs after ingest
  };
  const Batch *batch = nullptr;

  ~Builder() {
    OvBuf *o = ov;
    o[0].release();
    o[1].release();
    DBuf *all[] = {&aflag, &aflag_next, &wflag, &F, &S, &newA, &key, &paircnt, &newid, &cnt,
                   &vw, &va, &vf, &cnt2, &cnt3, &rowb, &memo, &memo_spare, &alive_g, &cup, &cdn, &cpair, &ekey, &ekey_alt,
                   &eidx, &eidx_alt, &ew, &elab, &emid, &ehead, &eheads, &ukey, &uw, &umid,
                   &rkey, &rkey_alt, &ridx, &ridx_alt, &ovf1, &ovf2, &gtabs, &prw, &dctr, &tmp,
                   &f_cn, &f_depth, &f_ws, &f_feat, &mlpw, &tab_D, &tab_pos, &tab_gid, &tab_posl,
                   &t_bits, &t_W, &t_MID, &t_ol, &t_il, &t_len, &t_SC, &t_touch, &t_vert,
                   &t_flags, &t_lists, &t_ctr, &t_rec, &r_order, &r_inv, &r_a, &r_b, &r_c,
                   &r_key, &r_key_alt, &r_val_alt, &r_lab};
    for (DBuf *b : all) b->release();
    if (hctr) (void)hipHostFree(hctr);
    if (h_tail) (void)hipHostFree(h_tail);
    for (auto &e : ev_tail)
      if (e) (void)hipEventDestroy(e);
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
    if (ev_rb) (void)hipEventDestroy(ev_rb);
  }

  DevCtr *dc() { return dctr.as<DevCtr>(); }
  // the search bound of the mode: hop_limit (hop) or settle_limit
  // (settled); in exact mode the distance-bucket shift of a search step
  uint32_t mode_limit() const {
    if (prm.wps_mode == CH_WPS_EXACT) return prm.ls_step ? prm.ls_step : kLsStepDefault;
    return prm.wps_mode == CH_WPS_SETTLED ? prm.settle_limit : prm.hop_limit;
  }

  // the learned priority and recorded features need every feature; nonzero
  // k_cn or k_depth need the contracted-neighbour count and depth
  bool need_feat() const {
    return prm.priority == CH_PRIO_LEARNED || (prm.flags & CH_F_RECORD_FEATURES);
  }
  bool need_cn_depth() const { return need_feat() || prm.k_cn != 0 || prm.k_depth != 0; }

  FeatState fstate() {
    FeatState f;
    const bool cd = need_cn_depth(), ft = need_feat();
    f.cn = cd ? f_cn.as<uint32_t>() : nullptr;
    f.depth = cd ? f_depth.as<uint32_t>() : nullptr;
    f.ws = ft ? f_ws.as<uint32_t>() : nullptr;
    f.feat = ft ? f_feat.as<float>() : nullptr;
    f.rec = (prm.flags & CH_F_RECORD_FEATURES) ? ch->rec.as<float>() : nullptr;
    f.k_ed = prm.k_ed;
    f.k_cn = prm.k_cn;
    f.k_depth = prm.k_depth;
    return f;
  }

  unsigned grid(uint64_t items, unsigned block = 256) const {
    uint64_t g = (items + block - 1) / block;
    uint64_t cap = (uint64_t)cus * 16;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
  }
  template <int G>
  unsigned ggrid(uint64_t items) const {  // group kernels, 256-thread blocks
    return grid(items * G);
  }

  // Counters to the host.  The wait polls an event instead of blocking in
  // hipStreamSynchronize: the round loop waits here twice per round, and a
  // blocked host thread takes longer to resume than the copy takes.
  int readback() {
    HIP_TRY(hipMemcpyAsync(hctr, dctr.p, sizeof(DevCtr), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(ev_rb, st));
    hipError_t e;
    while ((e = hipEventQuery(ev_rb)) == hipErrorNotReady) {
    }
    HIP_TRY(e);
    return CH_OK;
  }

  int check_err() {
    if (hctr->err & kErrOverflow)
      return set_error(CH_E_OVERFLOW,
                       "a witness-search radius or shortcut weight exceeds 0xFFFFFFFE");
    if (hctr->err & kErrCapacity) return set_error(CH_E_DEVICE, "internal capacity check failed");
    return CH_OK;
  }

  // ---------------------------------------------------------------- ingest
  int ingest(const ch_graph_t *g) {
    const bool on_dev = prm.flags & CH_F_INPUT_ON_DEVICE;
    const uint64_t m = g->m;
    if (m >= 0xFFFFFFFFull)
      return set_error(CH_E_UNSUPPORTED, "graphs with 2^32 - 1 or more arcs are not supported");
    const uint32_t m32 = (uint32_t)m;
    const int kb = bits_for(n);
    DBuf d_off, d_dst, d_w;
    const uint64_t *off = g->offsets;
    const uint32_t *dst = g->dst, *w = g->w;
    if (!on_dev) {
      HIP_TRY(d_off.ensure((n + 1) * sizeof(uint64_t)));
      HIP_TRY(d_dst.ensure(std::max<uint64_t>(m, 1) * 4));
      HIP_TRY(d_w.ensure(std::max<uint64_t>(m, 1) * 4));
      HIP_TRY(hipMemcpyAsync(d_off.p, g->offsets, (n + 1) * sizeof(uint64_t),
                             hipMemcpyHostToDevice, st));
      if (m) {
        HIP_TRY(hipMemcpyAsync(d_dst.p, g->dst, m * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_w.p, g->w, m * 4, hipMemcpyHostToDevice, st));
      }
      off = d_off.as<uint64_t>();
      dst = d_dst.as<uint32_t>();
      w = d_w.as<uint32_t>();
    }
    HIP_TRY(ekey.ensure(std::max<uint64_t>(m, 1) * 8));
    HIP_TRY(ekey_alt.ensure(std::max<uint64_t>(m, 1) * 8));
    HIP_TRY(ew.ensure(std::max<uint64_t>(m, 1) * 4));
    HIP_TRY(elab.ensure(std::max<uint64_t>(m, 1) * 4));
    HIP_TRY(ehead.ensure(std::max<uint64_t>(m, 1)));
    HIP_TRY(eheads.ensure(std::max<uint64_t>(m, 1) * 4));
    HIP_TRY(ukey.ensure(std::max<uint64_t>(m, 1) * 8));
    HIP_TRY(uw.ensure(std::max<uint64_t>(m, 1) * 4));
    HIP_TRY(hipMemsetAsync(dctr.p, 0, sizeof(DevCtr), st));
    // first offset and last offset checks happen on the host copy
    uint64_t first = 0, last = 0;
    if (on_dev) {
      HIP_TRY(hipMemcpyAsync(&first, off, 8, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(&last, off + n, 8, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
    } else {
      first = g->offsets[0];
      last = g->offsets[n];
    }
    if (first != 0 || last != m)
      return set_error(CH_E_INVALID, "offsets[0] must be 0 and offsets[n] must equal m");
    // locality order: the build runs on a renumbering that keeps clusters of
    // nearby vertices together (one graph; not with recorded features)
    renum = !batch && n >= kRenumberMin && m &&
            !(prm.flags & (CH_F_RECORD_FEATURES | CH_F_KEEP_ORDER));
    if (renum) TRY(locality_order(off, dst, m));
    if (m) {
      k_ingest_keys<<<grid(n), 256, 0, st>>>(n, m, kb, off, dst, w, ekey.as<uint64_t>(),
                                             ew.as<uint32_t>(), &dc()->bad,
                                             renum ? r_inv.as<uint32_t>() : nullptr);
      HIP_TRY(hipGetLastError());
      HIP_TRY(radix_sort_u64(ekey.as<uint64_t>(), ew.as<uint32_t>(), ekey_alt.as<uint64_t>(),
                             elab.as<uint32_t>(), m32, 2 * kb, tmp, st));
      k_run_heads<<<grid(m), 256, 0, st>>>(ekey.as<uint64_t>(), m32, ehead.as<uint8_t>());
      HIP_TRY(hipGetLastError());
      HIP_TRY(select_flags(ehead.as<uint8_t>(), m32, eheads.as<uint32_t>(), &dc()->c32[C_HEADS],
                           tmp, st));
      k_run_min<<<grid(m), 256, 0, st>>>(ekey.as<uint64_t>(), ew.as<uint32_t>(), m32,
                                         eheads.as<uint32_t>(), &dc()->c32[C_HEADS],
                                         ukey.as<uint64_t>(), uw.as<uint32_t>());
      HIP_TRY(hipGetLastError());
    }
    TRY(readback());
    if (hctr->bad & 1) return set_error(CH_E_INVALID, "offsets are not non-decreasing");
    if (hctr->bad & 2)
      return set_error(CH_E_INVALID, "an arc has head >= n or weight 0xFFFFFFFF");
    const uint32_t mu = m ? hctr->c32[C_HEADS] : 0;
    if (!m) HIP_TRY(hipMemsetAsync(&dc()->c32[C_HEADS], 0, 4, st));
    ch->m_input = mu;
    OvBuf &O = ov[cur];
    O.n = n;
    O.m = mu;
    HIP_TRY(O.foff.ensure((n + 1) * 4));
    HIP_TRY(O.roff.ensure((n + 1) * 4));
    HIP_TRY(O.farc.ensure(std::max<uint64_t>(mu, 1) * 8));
    HIP_TRY(O.rarc.ensure(std::max<uint64_t>(mu, 1) * 8));
    HIP_TRY(O.fmid.ensure(std::max<uint64_t>(mu, 1) * 4));
    HIP_TRY(O.rmid.ensure(std::max<uint64_t>(mu, 1) * 4));
    HIP_TRY(O.gid.ensure(std::max<uint64_t>(n, 1) * 4));
    HIP_TRY(O.P.ensure(std::max<uint64_t>(n, 1) * 4));
    k_csr_from_sorted<<<grid(std::max<uint64_t>(n + 1, mu)), 256, 0, st>>>(
        ukey.as<uint64_t>(), uw.as<uint32_t>(), &dc()->c32[C_HEADS], n, kb, O.foff.as<uint32_t>(),
        O.farc.as<uint2>(), O.fmid.as<uint32_t>());
    HIP_TRY(hipGetLastError());
    if (mu) {
      k_swap_key<<<grid(mu), 256, 0, st>>>(ukey.as<uint64_t>(), &dc()->c32[C_HEADS], mu, kb,
                                           ekey.as<uint64_t>());
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(ew.p, uw.p, (size_t)mu * 4, hipMemcpyDeviceToDevice, st));
      HIP_TRY(radix_sort_u64(ekey.as<uint64_t>(), ew.as<uint32_t>(), ekey_alt.as<uint64_t>(),
                             elab.as<uint32_t>(), mu, 2 * kb, tmp, st));
    }
    k_csr_from_sorted<<<grid(std::max<uint64_t>(n + 1, mu)), 256, 0, st>>>(
        ekey.as<uint64_t>(), ew.as<uint32_t>(), &dc()->c32[C_HEADS], n, kb, O.roff.as<uint32_t>(),
        O.rarc.as<uint2>(), O.rmid.as<uint32_t>());
    HIP_TRY(hipGetLastError());
    HIP_TRY(iota_u32(O.gid.as<uint32_t>(), n, st));
    HIP_TRY(hipMemsetAsync(O.P.p, 0, (size_t)n * 4, st));

    // labels (a batch build prepares and validates them per graph)
    if (batch) return CH_OK;
    HIP_TRY(ch->label.ensure(std::max<uint64_t>(n, 1) * 4));
    if (g->labels) {
      HIP_TRY(hipMemcpyAsync(ch->label.p, g->labels, (size_t)n * 4,
                             on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
      HIP_TRY(ekey.ensure(std::max<uint64_t>(n, 1) * 8));
      HIP_TRY(ekey_alt.ensure(std::max<uint64_t>(n, 1) * 8));
      HIP_TRY(ew.ensure(std::max<uint64_t>(n, 1) * 4));
      HIP_TRY(elab.ensure(std::max<uint64_t>(n, 1) * 4));
      k_labels_to_keys<<<grid(n), 256, 0, st>>>(n, ch->label.as<uint32_t>(), ekey.as<uint64_t>());
      HIP_TRY(hipGetLastError());
      HIP_TRY(iota_u32(ew.as<uint32_t>(), n, st));
      HIP_TRY(radix_sort_u64(ekey.as<uint64_t>(), ew.as<uint32_t>(), ekey_alt.as<uint64_t>(),
                             elab.as<uint32_t>(), n, 32, tmp, st));
      k_adjacent_equal<<<grid(n), 256, 0, st>>>(n, ekey.as<uint64_t>(), &dc()->bad);
      HIP_TRY(hipGetLastError());
      TRY(readback());
      if (hctr->bad & 4) return set_error(CH_E_INVALID, "labels are not distinct");
    } else {
      const uint32_t mix = (uint32_t)prm.seed ^ (uint32_t)(prm.seed >> 32);
      k_default_labels<<<grid(n), 256, 0, st>>>(n, mix, prm.tiebreak == CH_TIE_RAW_ID,
                                                ch->label.as<uint32_t>());
      HIP_TRY(hipGetLastError());
    }
    if (renum) {  // labels in the build's order; the input-order ones wait in r_lab
      HIP_TRY(r_lab.ensure((size_t)n * 4));
      k_permute_u32<<<grid(n), 256, 0, st>>>(n, r_order.as<uint32_t>(), ch->label.as<uint32_t>(),
                                             r_lab.as<uint32_t>(), 0);
      HIP_TRY(hipGetLastError());
      std::swap(ch->label, r_lab);
    }
    return CH_OK;
  }

  // Locality order of the input graph (device arrays off, dst): sixteen
  // steps of min-label propagation along the arcs, starting from the vertex
  // ids; the labels after four steps (fine clusters) and after sixteen
  // (coarse) give each vertex the key (coarse, fine), and the stable sort of
  // the keys is the new order.  Changes speed only: every decision of the
  // build depends on labels and distances, never on the numbering, and the
  // results are mapped back to the input's ids.
  static constexpr uint32_t kRenumberMin = 4096;
  static constexpr int kFineSteps = 4, kCoarseSteps = 16;

  int locality_order(const uint64_t *off, const uint32_t *dst, uint64_t m) {
    const size_t nb = (size_t)n * 4;
    HIP_TRY(r_order.ensure(nb));
    HIP_TRY(r_inv.ensure(nb));
    HIP_TRY(r_a.ensure(nb));
    HIP_TRY(r_b.ensure(nb));
    HIP_TRY(r_c.ensure(nb));
    HIP_TRY(r_key.ensure((size_t)n * 8));
    HIP_TRY(r_key_alt.ensure((size_t)n * 8));
    HIP_TRY(r_val_alt.ensure(nb));
    uint32_t *A = r_a.as<uint32_t>(), *B = r_b.as<uint32_t>();
    HIP_TRY(iota_u32(A, n, st));
    for (int k = 1; k <= kCoarseSteps; k++) {
      // after the fine steps the labels go to r_c and stay there
      uint32_t *out = k == kFineSteps ? r_c.as<uint32_t>() : B;
      k_minlabel_step<<<grid(n), 256, 0, st>>>(n, m, off, dst, A, out);
      HIP_TRY(hipGetLastError());
      if (k == kFineSteps) {
        HIP_TRY(hipMemcpyAsync(A, out, nb, hipMemcpyDeviceToDevice, st));
      } else {
        std::swap(A, B);
      }
    }
    const int kb = bits_for(n);
    k_order_keys<<<grid(n), 256, 0, st>>>(n, kb, A, r_c.as<uint32_t>(), r_key.as<uint64_t>());
    HIP_TRY(hipGetLastError());
    HIP_TRY(sort_u64_index(r_key.as<uint64_t>(), r_order.as<uint32_t>(),
                           r_key_alt.as<uint64_t>(), r_val_alt.as<uint32_t>(), n, 2 * kb, tmp,
                           st));
    HIP_TRY(iota_u32(r_a.as<uint32_t>(), n, st));
    k_permute_u32<<<grid(n), 256, 0, st>>>(n, r_order.as<uint32_t>(), r_a.as<uint32_t>(),
                                           r_inv.as<uint32_t>(), 1);
    HIP_TRY(hipGetLastError());
    return CH_OK;
  }

  // The finished build back in the input's ids: level and score per vertex,
  // the labels, and the ends and middle vertices of the CH arcs.
  int restore_order() {
    const uint32_t *ord = r_order.as<uint32_t>();
    for (DBuf *b : {&ch->level, &ch->score}) {
      HIP_TRY(r_a.ensure((size_t)n * 4));
      k_permute_u32<<<grid(n), 256, 0, st>>>(n, ord, b->as<uint32_t>(), r_a.as<uint32_t>(), 1);
      HIP_TRY(hipGetLastError());
      std::swap(*b, r_a);
    }
    std::swap(ch->label, r_lab);
    DBuf *arcs[] = {&ch->up_t, &ch->up_h, &ch->up_m, &ch->dn_t, &ch->dn_h, &ch->dn_m};
    for (int i = 0; i < 6; i++) {
      const uint64_t cnt = i < 3 ? ch->nup : ch->ndown;
      if (!cnt) continue;
      k_map_ids<<<grid(cnt), 256, 0, st>>>(cnt, arcs[i]->as<uint32_t>(), ord);
      HIP_TRY(hipGetLastError());
    }
    renum = false;
    return CH_OK;
  }

  // ------------------------------------------------------------- helpers
  Overlay view(OvBuf &O) {
    Overlay v;
    v.n = O.n;
    v.m = O.m;
    v.foff = O.foff.as<uint32_t>();
    v.farc = O.farc.as<uint2>();
    v.fmid = O.fmid.as<uint32_t>();
    v.roff = O.roff.as<uint32_t>();
    v.rarc = O.rarc.as<uint2>();
    v.rmid = O.rmid.as<uint32_t>();
    v.gid = O.gid.as<uint32_t>();
    return v;
  }

  int grow_copy(DBuf &b, size_t used_bytes, size_t need_bytes) {
    if (need_bytes <= b.cap) return CH_OK;
    DBuf nb;
    HIP_TRY(nb.ensure(std::max(need_bytes, b.cap * 2)));
    if (used_bytes) HIP_TRY(hipMemcpyAsync(nb.p, b.p, used_bytes, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    b.release();
    b = nb;
    return CH_OK;
  }

  MemoRef mref() { return MemoRef{memo.as<MemoSlot>(), mcap / kMemoBucket - 1, mwmask}; }

  // Room for `extra` more memo entries with `alive` live vertices.  The table
  // is rebuilt from its live entries when it would pass half full, or when
  // the entries per live vertex outgrow the source regions (mcount bounds
  // the live entries, so mcount <= 12 W alive keeps a source's first buckets
  // from filling).  The rebuilt table has twice the room the live entries
  // and `extra` need, and regions of W = 2 x (live entries per live vertex)
  // / 8 buckets, so a region is a quarter full after the rebuild.
  int ensure_memo(uint64_t extra, uint32_t alive) {
    const uint64_t W = mwmask + 1, a = std::max<uint32_t>(alive, 1);
    // the round's bound counts paths s -> u -> v, but the memo holds at most
    // one entry per ordered pair of alive vertices
    extra = std::min<uint64_t>(extra, a * (a - 1));
    const bool grow = (mcount + extra) * 2 > mcap;
    const bool spread = mcap && mcount > 12 * W * a && W * 4 < mcap / kMemoBucket;
    if (!grow && !spread) return CH_OK;
    uint64_t live = 0;
    if (mcap) {
      HIP_TRY(hipMemsetAsync(&dc()->kept, 0, 8, st));
      k_memo_count_live<<<grid(mcap), 256, 0, st>>>(memo.as<MemoSlot>(), mcap,
                                                     alive_g.as<uint8_t>(), &dc()->kept);
      HIP_TRY(hipGetLastError());
      TRY(readback());
      live = hctr->kept;
    }
    const uint64_t ncap = next_pow2(std::max<uint64_t>((live + extra) * 2, 1024));
    const uint64_t per = (2 * live + 8 * a - 1) / (8 * a);
    const uint64_t nw = std::min<uint64_t>(next_pow2(std::max<uint64_t>(per, 1)),
                                           ncap / kMemoBucket / 4);
    HIP_TRY(memo_spare.ensure(ncap * sizeof(MemoSlot)));
    HIP_TRY(fill_u64(memo_spare.as<uint64_t>(), SP_EMPTY64, ncap * 2, st));
    const MemoRef nt{memo_spare.as<MemoSlot>(), ncap / kMemoBucket - 1, nw - 1};
    uint64_t kept = 0;
    if (mcap) {
      HIP_TRY(hipMemsetAsync(&dc()->kept, 0, 8, st));
      k_memo_rehash<<<grid(mcap), 256, 0, st>>>(memo.as<MemoSlot>(), mcap, alive_g.as<uint8_t>(),
                                                 nt, &dc()->kept);
      HIP_TRY(hipGetLastError());
      TRY(readback());
      kept = hctr->kept;
    }
    std::swap(memo, memo_spare);
    mcap = ncap;
    mwmask = nw - 1;
    mcount = kept;
    return CH_OK;
  }

  // Persistent launch: blocks_per_cu one-wave blocks per CU; a group takes
  // 4 sources per scheduling step while sources are plentiful, else 1.
  // All-pairs distances of the current overlay (blocked Floyd-Warshall over
  // 64 x 64 tiles; the matrix is padded to a multiple of 64).
  int build_table(const Overlay &v) {
    const uint32_t N = (v.n + kFwTile - 1) / kFwTile * kFwTile;
    const uint32_t nb = N / kFwTile;
    HIP_TRY(tab_D.ensure((size_t)N * N * 4));
    HIP_TRY(tab_pos.ensure((size_t)std::max<uint32_t>(n, 1) * 4));
    HIP_TRY(tab_gid.ensure((size_t)N * 4));
    HIP_TRY(tab_posl.ensure((size_t)N * 4));
    k_fw_init<<<grid((uint64_t)N * N), 256, 0, st>>>(tab_D.as<uint32_t>(), N);
    HIP_TRY(hipGetLastError());
    k_fw_arcs<<<grid(v.n), 256, 0, st>>>(v, N, tab_D.as<uint32_t>(), tab_pos.as<uint32_t>(),
                                          tab_gid.as<uint32_t>());
    HIP_TRY(hipGetLastError());
    for (uint32_t k = 0; k < nb; k++) {
      k_fw_diag<<<1, kFwDiagThreads, 0, st>>>(tab_D.as<uint32_t>(), N, k);
      HIP_TRY(hipGetLastError());
      if (nb > 1) {
        k_fw_panels<<<2 * nb, kFwThreads, 0, st>>>(tab_D.as<uint32_t>(), N, k);
        HIP_TRY(hipGetLastError());
        k_fw_rest<<<nb * nb, kFwThreads, 0, st>>>(tab_D.as<uint32_t>(), N, k);
        HIP_TRY(hipGetLastError());
      }
    }
    tab_on = true;
    tab_N = N;
    tab_n0 = v.n;
    return CH_OK;
  }

  // The rest of the build on the table positions (tail.hpp): five launches
  // per round, rounds enqueued kTailBatch at a time, the state read back
  // once per batch while the next batch runs.  Entered at the start of a
  // round, right after the table is built (positions = current local ids);
  // nw: this round's source count.
  static constexpr uint32_t kTailBatch = 8;
  // default table threshold: road1m builds fastest at about 3584 vertices
  // (a larger table costs more Floyd-Warshall, a smaller one more rounds on
  // the general path)
  static constexpr uint32_t kDenseTailDefault = 3584;

  int run_tail(uint32_t &round, uint32_t nw) {
    OvBuf &O = ov[cur];
    const uint32_t n0 = O.n;
    if (n0 == 0 || n0 > kTailMaxN || n0 != tab_n0)
      return set_error(CH_E_DEVICE, "tail entered without a matching table (internal error)");
    const bool stats = prm.flags & CH_F_STATS;
    const uint32_t rw = (n0 + 31) / 32;
    const size_t nn = (size_t)n0 * n0;
    // every vertex pair gives at most one upward and one downward CH arc
    const uint64_t pairs = (uint64_t)n0 * (n0 - 1) / 2 + 1;
    DBuf *ub[] = {&ch->up_t, &ch->up_h, &ch->up_w, &ch->up_m, &ch->dn_t, &ch->dn_h, &ch->dn_w,
                  &ch->dn_m};
    if (ch->nup + pairs > up_cap) {
      const uint64_t nc = ch->nup + pairs;
      for (int i = 0; i < 4; i++) TRY(grow_copy(*ub[i], ch->nup * 4, nc * 4));
      up_cap = nc;
    }
    if (ch->ndown + pairs > dn_cap) {
      const uint64_t nc = ch->ndown + pairs;
      for (int i = 4; i < 8; i++) TRY(grow_copy(*ub[i], ch->ndown * 4, nc * 4));
      dn_cap = nc;
    }
    HIP_TRY(t_bits.ensure(3 * (size_t)n0 * rw * 4));
    HIP_TRY(t_W.ensure(nn * 4));
    HIP_TRY(t_MID.ensure(nn * 4));
    HIP_TRY(t_ol.ensure(nn * 2));
    HIP_TRY(t_il.ensure(nn * 2));
    HIP_TRY(t_SC.ensure(nn * 8));
    HIP_TRY(t_touch.ensure(nn * 4));
    HIP_TRY(t_len.ensure(2 * (size_t)n0 * 4));
    HIP_TRY(t_vert.ensure(5 * (size_t)n0 * 4));
    HIP_TRY(t_flags.ensure(5 * (size_t)n0 * 4));
    HIP_TRY(t_lists.ensure(4 * (size_t)n0 * 2));
    HIP_TRY(t_ctr.ensure(sizeof(TailCtr)));
    HIP_TRY(t_rec.ensure((size_t)n0 * sizeof(TailRound)));
    if (!h_tail) HIP_TRY(hipHostMalloc((void **)&h_tail, 2 * sizeof(TailCtr), hipHostMallocDefault));
    for (auto &e : ev_tail)
      if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    TailArgs A;
    A.n0 = n0;
    A.rw = rw;
    A.D = tab_D.as<uint32_t>();
    A.N = tab_N;
    A.gidp = tab_gid.as<uint32_t>();
    uint32_t *vtx = t_vert.as<uint32_t>();
    A.lab = vtx;
    A.lrank = vtx + n0;
    A.plr = vtx + 2 * (size_t)n0;
    A.P = (int32_t *)(vtx + 3 * (size_t)n0);
    A.alive = vtx + 4 * (size_t)n0;
    A.ob = t_bits.as<uint32_t>();
    A.ib = A.ob + (size_t)n0 * rw;
    A.eb = A.ib + (size_t)n0 * rw;
    A.W = t_W.as<uint32_t>();
    A.MID = t_MID.as<uint32_t>();
    A.ol = t_ol.as<uint16_t>();
    A.il = t_il.as<uint16_t>();
    A.olen = t_len.as<uint32_t>();
    A.ilen = A.olen + n0;
    A.SC = t_SC.as<unsigned long long>();
    A.touched = t_touch.as<uint32_t>();
    uint32_t *fl = t_flags.as<uint32_t>();
    A.af0 = fl;
    A.af1 = fl + n0;
    A.wf0 = fl + 2 * (size_t)n0;
    A.wf1 = fl + 3 * (size_t)n0;
    A.sflag = fl + 4 * (size_t)n0;
    uint16_t *ls = t_lists.as<uint16_t>();
    A.la0 = ls;
    A.la1 = ls + n0;
    A.lw0 = ls + 2 * (size_t)n0;
    A.lw1 = ls + 3 * (size_t)n0;
    A.C = t_ctr.as<TailCtr>();
    A.err = &dc()->err;
    HIP_TRY(hipMemsetAsync(dctr.p, 0, sizeof(DevCtr), st));
    HIP_TRY(hipMemsetAsync(t_ctr.p, 0, sizeof(TailCtr), st));
    k_tail_clear<<<grid(nn), 256, 0, st>>>(A);
    HIP_TRY(hipGetLastError());
    k_tail_load<<<grid(n0), 256, 0, st>>>(A, view(O), O.P.as<int32_t>(), aflag.as<uint8_t>(),
                                          vw.as<uint32_t>(), nw, ch->label.as<uint32_t>());
    HIP_TRY(hipGetLastError());
    if (mcap) {
      k_tail_memo<<<grid(mcap), 256, 0, st>>>(A, memo.as<MemoSlot>(), mcap,
                                               alive_g.as<uint8_t>(), tab_pos.as<uint32_t>());
      HIP_TRY(hipGetLastError());
    }
    k_tail_lrank<<<grid(n0), 256, 0, st>>>(A);
    HIP_TRY(hipGetLastError());

    ArcOut up{ch->up_t.as<uint32_t>(), ch->up_h.as<uint32_t>(), ch->up_w.as<uint32_t>(),
              ch->up_m.as<uint32_t>()};
    ArcOut dn{ch->dn_t.as<uint32_t>(), ch->dn_h.as<uint32_t>(), ch->dn_w.as<uint32_t>(),
              ch->dn_m.as<uint32_t>()};
    const uint32_t max_r = prm.max_rounds ? prm.max_rounds - round : 0xFFFFFFFFu;
    TailRound *rec = t_rec.as<TailRound>();
    uint32_t live = n0;  // last known live count (sizes the grids)
    uint32_t r = 0, batches = 0;
    bool stop = false;
    // one batch of rounds: five launches per round with fixed arguments (the
    // kernels read the round's parity and number from the device)
    auto enqueue_batch = [&](unsigned wg) {
      for (uint32_t b = 0; b < kTailBatch; b++) {
        k_tail_search<<<wg, kTailBlock, 0, st>>>(A);
        k_tail_score<<<wg, kTailBlock, 0, st>>>(A);
        k_tail_selcon<<<wg, kTailBlock, 0, st>>>(A, round, up, dn, ch->nup, ch->ndown, up_cap,
                                                 dn_cap, ch->level.as<uint32_t>(),
                                                 ch->score.as<int32_t>(), alive_g.as<uint8_t>());
        k_tail_compact<<<wg, kTailBlock, 0, st>>>(A);
        k_tail_merge_end<<<wg, kTailBlock, 0, st>>>(A, max_r, rec, n0);
      }
    };
    // batches replay a captured graph, one per grid size (the live count
    // rounded up to a power of two); CH_F_NO_GRAPH launches them directly
    const bool use_graph = !(prm.flags & CH_F_NO_GRAPH);
    struct GraphSet {
      std::vector<std::pair<unsigned, hipGraphExec_t>> ex;
      ~GraphSet() {
        for (auto &e : ex) (void)hipGraphExecDestroy(e.second);
      }
    } graphs;
    while (!stop) {
      // one wave per item; items never exceed the live count at the batch start
      uint32_t lb = 64;
      while (lb < live && lb < n0) lb <<= 1;
      const unsigned wg = grid((uint64_t)lb * kWave, kTailBlock);
      if (use_graph) {
        hipGraphExec_t ex = nullptr;
        for (auto &e : graphs.ex)
          if (e.first == wg) ex = e.second;
        if (!ex) {
          hipGraph_t gr = nullptr;
          HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
          enqueue_batch(wg);
          const hipError_t le = hipGetLastError();
          const hipError_t ce = hipStreamEndCapture(st, &gr);
          HIP_TRY(le);
          HIP_TRY(ce);
          const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          HIP_TRY(ie);
          graphs.ex.emplace_back(wg, ex);
        }
        HIP_TRY(hipGraphLaunch(ex, st));
      } else {
        enqueue_batch(wg);
      }
      r += kTailBatch;
      HIP_TRY(hipGetLastError());
      const int slot = batches & 1;
      HIP_TRY(hipMemcpyAsync(&h_tail[slot], t_ctr.p, sizeof(TailCtr), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipEventRecord(ev_tail[slot], st));
      batches++;
      // the previous batch's state (this batch runs meanwhile); after the
      // first batch, wait for it directly
      const int prev = batches >= 2 ? (slot ^ 1) : slot;
      hipError_t e;
      while ((e = hipEventQuery(ev_tail[prev])) == hipErrorNotReady) {
      }
      HIP_TRY(e);
      live = h_tail[prev].live;
      stop = h_tail[prev].done != 0;
      if (!stop && r > n0 + 4 * kTailBatch)
        return set_error(CH_E_DEVICE, "tail did not finish (internal error)");
    }
    // the newest copy holds the final state (later launches return at once)
    const int last = (batches - 1) & 1;
    {
      hipError_t e;
      while ((e = hipEventQuery(ev_tail[last])) == hipErrorNotReady) {
      }
      HIP_TRY(e);
    }
    const TailCtr T = h_tail[last];
    TRY(readback());
    TRY(check_err());
    std::vector<TailRound> recs(T.rounds);
    if (T.rounds)
      HIP_TRY(hipMemcpy(recs.data(), rec, (size_t)T.rounds * sizeof(TailRound),
                        hipMemcpyDeviceToHost));
    int khz = 0;
    if (stats) {
      HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ch->device));
    }
    for (uint32_t i = 0; i < T.rounds; i++) {
      const TailRound &x = recs[i];
      ch_round_stats_t rs{};
      rs.alive_before = x.alive_before;
      rs.n_sources = x.n_sources;
      rs.n_affected = x.n_affected;
      rs.n_selected = x.n_selected;
      rs.n_targets = x.n_targets;
      rs.n_pruned = x.n_pruned;
      rs.n_shortcuts = x.n_shortcuts;
      rs.overlay_arcs = x.overlay_arcs;
      rs.rows_expanded = x.rows;
      rs.arcs_scanned = x.arcs;
      rs.memo_probes = x.probes;
      rs.memo_inserts = x.n_targets;
      rs.ls_tier1 = CH_LS_TAIL;
      const unsigned long long c0 = i ? recs[i - 1].clk : T.clk0;
      if (stats && khz > 0) rs.ms_total = (float)((double)(x.clk - c0) / khz);
      mcount += x.n_targets;
      ch->stats.push_back(rs);
    }
    ch->nup += T.up_n;
    ch->ndown += T.dn_n;
    round += T.rounds;
    if (T.live) {
      if (prm.max_rounds && round >= prm.max_rounds)
        return set_error(CH_E_LIMIT, "max_rounds reached before every vertex was contracted");
      return set_error(CH_E_DEVICE, "tail stopped with live vertices (internal error)");
    }
    O.n = 0;
    O.m = 0;
    return CH_OK;
  }

  // At most max_per_cu one-wave blocks per CU, and no more than the CU's
  // 160 KB of LDS holds (hop mode adds a second distance array to every
  // table).
  template <int G, int CAP>
  void launch_ls(const Overlay &v, const uint32_t *list, uint32_t nl, const uint32_t *nl_dev,
                 int tier, int max_per_cu) {
    const bool hop = prm.wps_mode != CH_WPS_EXACT;  // a second per-slot array
    const size_t lds = ls_lds_bytes(G, CAP, hop);
    const int blocks_per_cu = std::max(1, std::min(max_per_cu, (int)((160u << 10) / lds)));
    const uint32_t groups = (uint32_t)cus * blocks_per_cu * (kLsBlock / G);
    const uint32_t chunk = (!nl_dev && nl >= 16u * groups) ? 4u : 1u;
    DevCtr *d = dc();
    auto go = [&](auto kern) {
      kern<<<(unsigned)cus * blocks_per_cu, kLsBlock, 0, st>>>(
          v, list, nl, aflag.as<uint8_t>(), mref(),
          tier == 1 ? &d->ls : &d->ls2, nl_dev, tier == 1 ? &d->work1 : &d->work2,
          tier == 1 ? ovf1.as<uint32_t>() : ovf2.as<uint32_t>(),
          tier == 1 ? &d->novf1 : &d->novf2, chunk, fstate().ws, &d->err, mode_limit(),
          ch->label.as<uint32_t>());
    };
    if (prm.wps_mode == CH_WPS_HOP) go(k_local_search<G, CAP, kWpsHop>);
    else if (prm.wps_mode == CH_WPS_SETTLED) go(k_local_search<G, CAP, kWpsSettled>);
    else go(k_local_search<G, CAP, kWpsExact>);
  }
  // second tier: sources that outgrew the first tier's tables (list ovf1,
  // count on the device), a block of kLsBlkWaves waves and one
  // kLsBlkCap-slot LDS table per source, one block per CU; overflows go to
  // ovf2 for the global tier
  void launch_ls_blk(const Overlay &v) {
    DevCtr *d = dc();
    auto go = [&](auto kern) {
      kern<<<(unsigned)cus, kWave * kLsBlkWaves, 0, st>>>(
          v, ovf1.as<uint32_t>(), 0, aflag.as<uint8_t>(), mref(), &d->ls2, &d->novf1, &d->work2,
          ovf2.as<uint32_t>(), &d->novf2, fstate().ws, &d->err, mode_limit(),
          ch->label.as<uint32_t>());
    };
    if (prm.wps_mode == CH_WPS_HOP) go(k_local_search_blk<kLsBlkCap, kWpsHop, kLsBlkWaves>);
    else if (prm.wps_mode == CH_WPS_SETTLED)
      go(k_local_search_blk<kLsBlkCap, kWpsSettled, kLsBlkWaves>);
    else go(k_local_search_blk<kLsBlkCap, kWpsExact, kLsBlkWaves>);
  }
  template <int G>
  void launch_score(const Overlay &v, uint32_t na) {
    k_score<G><<<ggrid<G>(na), 256, 0, st>>>(v, va.as<uint32_t>(), na, mref(), ov[cur].P.as<int32_t>(),
                                              paircnt.as<uint32_t>(), fstate());
  }
  template <int G>
  void launch_prune(const Overlay &v, uint32_t nw) {
    k_prune<G><<<ggrid<G>(nw), 256, 0, st>>>(v, vw.as<uint32_t>(), nw, mref(), &dc()->pruned,
                                              prw.as<uint32_t>(), &dc()->err);
  }
  template <int G>
  void launch_select(const Overlay &v) {
    k_select<G><<<ggrid<G>(v.n), 256, 0, st>>>(v, key.as<uint64_t>(), F.as<uint8_t>());
  }
  // counts of the selected vertices (count on the device, at most v.n)
  template <int G>
  void launch_ccount(const Overlay &v, uint32_t cap) {
    k_contract_count<G><<<ggrid<G>(cap), 256, 0, st>>>(
        v, vf.as<uint32_t>(), &dc()->c32[C_NF], cap, aflag.as<uint8_t>(), paircnt.as<uint32_t>(),
        mref(), cup.as<uint32_t>(), cdn.as<uint32_t>(),
        cpair.as<uint32_t>());
  }
  // scanned positions at offset cap of cup, cdn, cpair
  template <int G>
  void launch_contract(const Overlay &v, uint32_t nf, uint32_t cap, uint32_t round, int kb) {
    ArcOut up{ch->up_t.as<uint32_t>(), ch->up_h.as<uint32_t>(), ch->up_w.as<uint32_t>(),
              ch->up_m.as<uint32_t>()};
    ArcOut dn{ch->dn_t.as<uint32_t>(), ch->dn_h.as<uint32_t>(), ch->dn_w.as<uint32_t>(),
              ch->dn_m.as<uint32_t>()};
    k_contract<G><<<ggrid<G>(nf), 256, 0, st>>>(
        v, vf.as<uint32_t>(), nf, ov[cur].P.as<int32_t>(), ch->label.as<uint32_t>(),
        mref(), round, ch->level.as<uint32_t>(), ch->score.as<int32_t>(),
        alive_g.as<uint8_t>(), cup.as<uint32_t>() + cap, cdn.as<uint32_t>() + cap,
        cpair.as<uint32_t>() + cap, up, dn, ch->nup, ch->ndown, cpair.as<uint32_t>(), kb,
        ekey.as<uint64_t>(), ew.as<uint32_t>(), elab.as<uint32_t>(), emid.as<uint32_t>(),
        S.as<uint8_t>(), newA.as<uint8_t>(), fstate(), &dc()->err);
  }

  // Row lengths of the new overlay (new ids < n2, zero up to O.n), their
  // offsets over O.n + 1 entries (foff[n2 .. O.n] all equal m2), then the
  // merged rows, both directions.  fb0/fb1 and rb0/rb1: shortcut-row bounds.
  int merge_err = CH_OK;
  template <int G>
  void merge_rows(OvBuf &O, OvBuf &N, int kb, const uint32_t *fb0, const uint32_t *fb1,
                  const uint32_t *rb0, const uint32_t *rb1) {
    merge_err = CH_OK;
    const dim3 gr(ggrid<G>(O.n), 2);  // y: forward, reverse
    MergeSide f{O.foff.as<uint32_t>(), O.farc.as<uint2>(), O.fmid.as<uint32_t>(),
                ukey.as<uint64_t>(), nullptr, fb0, fb1, cnt2.as<uint32_t>(),
                N.foff.as<uint32_t>(), N.farc.as<uint2>(), N.fmid.as<uint32_t>()};
    MergeSide r{O.roff.as<uint32_t>(), O.rarc.as<uint2>(), O.rmid.as<uint32_t>(),
                rkey.as<uint64_t>(), ridx.as<uint32_t>(), rb0, rb1, cnt3.as<uint32_t>(),
                N.roff.as<uint32_t>(), N.rarc.as<uint2>(), N.rmid.as<uint32_t>()};
    k_merge_rows<G, 0><<<gr, 256, 0, st>>>(O.n, kb, F.as<uint8_t>(), newid.as<uint32_t>(),
                                           uw.as<uint32_t>(), umid.as<uint32_t>(), f, r);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = scan3_u32(cnt2.as<uint32_t>(), N.foff.as<uint32_t>(), &dc()->c32[C_MF],
                    cnt3.as<uint32_t>(), N.roff.as<uint32_t>(), &dc()->c32[C_MR], nullptr,
                    nullptr, nullptr, O.n + 1, tmp, st);
    if (e == hipSuccess) {
      k_merge_rows<G, 1><<<gr, 256, 0, st>>>(O.n, kb, F.as<uint8_t>(), newid.as<uint32_t>(),
                                             uw.as<uint32_t>(), umid.as<uint32_t>(), f, r);
      e = hipGetLastError();
    }
    if (e != hipSuccess) merge_err = hip_error(e, "overlay merge");
  }

  static int pick_group(double work) {
    if (work <= 4) return 4;
    if (work <= 8) return 8;
    if (work <= 16) return 16;
    if (work <= 32) return 32;
    return 64;
  }

  template <typename F4, typename F8, typename F16, typename F32, typename F64>
  static void dispatch(int G, F4 f4, F8 f8, F16 f16, F32 f32, F64 f64) {
    switch (G) {
      case 4: f4(); break;
      case 8: f8(); break;
      case 16: f16(); break;
      case 32: f32(); break;
      default: f64(); break;
    }
  }

  // ------------------------------------------------------------- rounds
  int run(const ch_graph_t *g) {
    HIP_TRY(dctr.ensure(sizeof(DevCtr)));
    HIP_TRY(hipHostMalloc((void **)&hctr, sizeof(DevCtr), hipHostMallocDefault));
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipEventCreateWithFlags(&ev_rb, hipEventDisableTiming));
    const bool stats = prm.flags & CH_F_STATS;

    TRY(ingest(g));
    if (batch && n) {
      k_rowlen_by_graph<<<grid(n), 256, 0, st>>>(n, ov[cur].foff.as<uint32_t>(), batch->gof,
                                                 batch->m_in);
      HIP_TRY(hipGetLastError());
    }

    HIP_TRY(ch->level.ensure(std::max<uint64_t>(n, 1) * 4));
    HIP_TRY(ch->score.ensure(std::max<uint64_t>(n, 1) * 4));
    HIP_TRY(alive_g.ensure(std::max<uint64_t>(n, 1)));
    HIP_TRY(fill_u32(ch->level.as<uint32_t>(), SP_INF32, n, st));
    HIP_TRY(hipMemsetAsync(ch->score.p, 0, (size_t)n * 4, st));
    HIP_TRY(fill_u8(alive_g.as<uint8_t>(), 1, n, st));
    if (need_cn_depth()) {
      HIP_TRY(f_cn.ensure(std::max<uint64_t>(n, 1) * 4));
      HIP_TRY(f_depth.ensure(std::max<uint64_t>(n, 1) * 4));
      HIP_TRY(hipMemsetAsync(f_cn.p, 0, (size_t)n * 4, st));
      HIP_TRY(hipMemsetAsync(f_depth.p, 0, (size_t)n * 4, st));
    }
    if (need_feat()) {
      HIP_TRY(f_ws.ensure(std::max<uint64_t>(n, 1) * 4));
      HIP_TRY(f_feat.ensure(std::max<uint64_t>(n, 1) * 32));
      HIP_TRY(hipMemsetAsync(f_ws.p, 0, (size_t)n * 4, st));
      HIP_TRY(hipMemsetAsync(f_feat.p, 0, (size_t)n * 32, st));
    }
    if (prm.flags & CH_F_RECORD_FEATURES) {
      HIP_TRY(ch->rec.ensure(std::max<uint64_t>(n, 1) * 32));
      HIP_TRY(hipMemsetAsync(ch->rec.p, 0, (size_t)n * 32, st));
      ch->has_rec = true;
    }
    if (prm.priority == CH_PRIO_LEARNED) {
      HIP_TRY(mlpw.ensure(kMlpParams * 4));
      HIP_TRY(hipMemcpyAsync(mlpw.p, prm.mlp, kMlpParams * 4, hipMemcpyHostToDevice, st));
    }
    const size_t nn = std::max<uint64_t>(n, 1);
    HIP_TRY(aflag.ensure(nn));
    HIP_TRY(aflag_next.ensure(nn));
    HIP_TRY(wflag.ensure(nn));
    HIP_TRY(F.ensure(nn));
    HIP_TRY(S.ensure(nn));
    HIP_TRY(newA.ensure(nn));
    HIP_TRY(key.ensure(nn * 8));
    HIP_TRY(paircnt.ensure(nn * 4));
    HIP_TRY(newid.ensure(nn * 4));
    HIP_TRY(cnt.ensure((nn + 1) * 4));
    HIP_TRY(rowb.ensure(nn * 16));
    HIP_TRY(vw.ensure(nn * 4));
    HIP_TRY(va.ensure(nn * 4));
    HIP_TRY(vf.ensure(nn * 4));
    HIP_TRY(ovf1.ensure(nn * 4));
    HIP_TRY(ovf2.ensure(nn * 4));
    HIP_TRY(fill_u8(aflag.as<uint8_t>(), 1, n, st));
    HIP_TRY(iota_u32(vw.as<uint32_t>(), n, st));
    HIP_TRY(iota_u32(va.as<uint32_t>(), n, st));
    uint32_t nw = n, na = n;
    // CH arc buffers: start at the input size
    up_cap = dn_cap = std::max<uint64_t>(ch->m_input, 16);
    DBuf *ub[] = {&ch->up_t, &ch->up_h, &ch->up_w, &ch->up_m, &ch->dn_t, &ch->dn_h, &ch->dn_w,
                  &ch->dn_m};
    for (DBuf *b : ub) HIP_TRY(b->ensure(up_cap * 4));
    ch->nup = ch->ndown = 0;

    uint64_t next_bound = 0;
    if (n) {
      HIP_TRY(hipMemsetAsync(&dc()->bound, 0, 8, st));
      k_ls_bound_affected<<<grid(n), 256, 0, st>>>(view(ov[cur]), aflag.as<uint8_t>(),
                                                   &dc()->bound);
      HIP_TRY(hipGetLastError());
      TRY(readback());
      next_bound = hctr->bound;
    }
    uint32_t round = 0;
    unsigned long long sc_total = 0;  // shortcuts so far (progress lines)
    auto last_note = std::chrono::steady_clock::now();
    while (ov[cur].n > 0) {
      if (prm.max_rounds && round >= prm.max_rounds)
        return set_error(CH_E_LIMIT, "max_rounds reached before every vertex was contracted");
      OvBuf &O = ov[cur];
      Overlay v = view(O);
      ch_round_stats_t rs{};
      rs.alive_before = O.n;
      rs.n_sources = nw;
      rs.n_affected = na;
      if (stats) HIP_TRY(hipEventRecord(ev[1], st));
      const double avgdeg = O.n ? (double)O.m / O.n : 0.0;

      // exact mode, plain priority, one graph: once the overlay fits the
      // all-pairs table, the remaining rounds run on the device (tail.hpp)
      {
        const uint32_t lim = prm.dense_tail == 0 ? kDenseTailDefault : prm.dense_tail;
        const bool fused = prm.wps_mode == CH_WPS_EXACT && prm.dense_tail != CH_DENSE_TAIL_OFF &&
                           prm.priority == CH_PRIO_PLAIN && !batch && prm.k_ed == 1 &&
                           prm.k_cn == 0 && prm.k_depth == 0 &&
                           !(prm.flags & (CH_F_RECORD_FEATURES | CH_F_TAIL_STEPWISE));
        if (fused && !tab_on && O.n && O.n <= lim && O.n <= kTailMaxN) {
          TRY(build_table(v));
          TRY(run_tail(round, nw));
          break;
        }
      }
      // ---- Step 1: LocalSearch (Alg. 4) --------------------------------
      // memo capacity for this round's inserts (bound computed with the
      // previous round's final readback)
      TRY(ensure_memo(next_bound, O.n));
      HIP_TRY(hipMemsetAsync(dctr.p, 0, sizeof(DevCtr), st));
      const double thr = prm.dense_deg10 ? prm.dense_deg10 / 10.0 : 5.0;
      const bool sparse = avgdeg <= thr;
      // exact mode on a small overlay: all distances once, then lookups
      const uint32_t tail = prm.dense_tail == 0 ? kDenseTailDefault : prm.dense_tail;
      if (!tab_on && prm.wps_mode == CH_WPS_EXACT && tail != CH_DENSE_TAIL_OFF && O.n &&
          O.n <= tail)
        TRY(build_table(v));
      bool blk_ran = false;  // the block tier was launched (its events recorded)
      if (nw && tab_on) {
        rs.ls_tier1 = CH_LS_TABLE;
        if (stats) HIP_TRY(hipEventRecord(ev[2], st));
        k_tab_posl<<<grid(O.n), 256, 0, st>>>(O.n, O.gid.as<uint32_t>(), tab_pos.as<uint32_t>(),
                                               tab_posl.as<uint32_t>());
        HIP_TRY(hipGetLastError());
        k_ls_table<<<(unsigned)std::min<uint64_t>(nw, (uint64_t)cus * 8), 64, 0, st>>>(
            v, vw.as<uint32_t>(), nw, aflag.as<uint8_t>(), mref(), &dc()->ls, tab_D.as<uint32_t>(), tab_N, tab_n0,
            tab_pos.as<uint32_t>(), tab_gid.as<uint32_t>(), tab_posl.as<uint32_t>(),
            alive_g.as<uint8_t>(), fstate().ws, &dc()->err);
        HIP_TRY(hipGetLastError());
        if (stats) HIP_TRY(hipEventRecord(ev[3], st));
      } else if (nw) {
        // tier 1: LDS tables sized for the overlay's degree (16 lanes x 128
        // slots on sparse overlays, 64 lanes x 2048 slots on dense ones);
        // sources whose search outgrows them go to a 4096-slot LDS tier
        // (launched with its count on the device), then, after the next
        // readback, to tables in global memory
        uint32_t kind = sparse ? prm.ls_sparse : prm.ls_dense;
        if (kind == CH_LS_AUTO) kind = sparse ? CH_LS_16x128 : CH_LS_64x2048;
        rs.ls_tier1 = kind;
        if (stats) HIP_TRY(hipEventRecord(ev[2], st));
        switch (kind) {
          case CH_LS_16x128: launch_ls<16, 128>(v, vw.as<uint32_t>(), nw, nullptr, 1, 16); break;
          case CH_LS_32x512: launch_ls<32, 512>(v, vw.as<uint32_t>(), nw, nullptr, 1, 8); break;
          case CH_LS_64x512: launch_ls<64, 512>(v, vw.as<uint32_t>(), nw, nullptr, 1, 16); break;
          default: launch_ls<64, 2048>(v, vw.as<uint32_t>(), nw, nullptr, 1, 8); break;
        }
        HIP_TRY(hipGetLastError());
        if (stats) HIP_TRY(hipEventRecord(ev[3], st));
        if (stats) HIP_TRY(hipEventRecord(ev[5], st));
        blk_ran = true;
        launch_ls_blk(v);
        HIP_TRY(hipGetLastError());
        if (stats) HIP_TRY(hipEventRecord(ev[6], st));
      }
      // Steps 1 (pruning) to 4 (contraction counts) run before the searches
      // are known to be complete; when a source needed the global tier, the
      // pruning is undone (k_unprune) before that search and all of them run
      // again after it (the rest overwrite their outputs).
      const int Gp = prm.group ? (int)prm.group : pick_group(avgdeg);
      const int Gs = prm.group ? (int)prm.group : pick_group(avgdeg * avgdeg / 4.0);
      const int Gsel = prm.group ? (int)prm.group : pick_group(avgdeg);
      const uint32_t ncap = O.n;  // bound on the selected count
      HIP_TRY(prw.ensure(std::max<size_t>(O.m, 1) * 4));
      HIP_TRY(cup.ensure(((size_t)ncap * 2 + 1) * 4));
      HIP_TRY(cdn.ensure(((size_t)ncap * 2 + 1) * 4));
      HIP_TRY(cpair.ensure(((size_t)ncap * 2 + 1) * 4));
      auto after_search = [&]() -> int {
        // pruning at the end of Alg. 4
        if (nw) {
          dispatch(Gp, [&] { launch_prune<4>(v, nw); }, [&] { launch_prune<8>(v, nw); },
                   [&] { launch_prune<16>(v, nw); }, [&] { launch_prune<32>(v, nw); },
                   [&] { launch_prune<64>(v, nw); });
          HIP_TRY(hipGetLastError());
        }
        // ---- Step 2: Score (Alg. 5) ------------------------------------
        if (na) {
          dispatch(Gs, [&] { launch_score<4>(v, na); }, [&] { launch_score<8>(v, na); },
                   [&] { launch_score<16>(v, na); }, [&] { launch_score<32>(v, na); },
                   [&] { launch_score<64>(v, na); });
          HIP_TRY(hipGetLastError());
          if (prm.priority == CH_PRIO_LEARNED)
            HIP_TRY(launch_mlp_priority(va.as<uint32_t>(), na, O.gid.as<uint32_t>(),
                                        f_feat.as<float>(), mlpw.as<float>(), O.P.as<int32_t>(),
                                        prm.mlp_qbits, cus, st));
        }
        // ---- Step 3: Select (Alg. 6) -----------------------------------
        k_keys<<<grid(O.n), 256, 0, st>>>(O.n, O.P.as<int32_t>(), O.gid.as<uint32_t>(),
                                          ch->label.as<uint32_t>(), key.as<uint64_t>(),
                                          S.as<uint8_t>(), newA.as<uint8_t>(),
                                          rowb.as<uint32_t>());
        HIP_TRY(hipGetLastError());
        dispatch(Gsel, [&] { launch_select<4>(v); }, [&] { launch_select<8>(v); },
                 [&] { launch_select<16>(v); }, [&] { launch_select<32>(v); },
                 [&] { launch_select<64>(v); });
        HIP_TRY(hipGetLastError());
        HIP_TRY(select_flags(F.as<uint8_t>(), O.n, vf.as<uint32_t>(), &dc()->c32[C_NF], tmp, st));
        // ---- Step 4 counts (Alg. 7): arcs and shortcut pairs per selected
        // vertex, exclusive scans into the second halves
        dispatch(Gs, [&] { launch_ccount<4>(v, ncap); }, [&] { launch_ccount<8>(v, ncap); },
                 [&] { launch_ccount<16>(v, ncap); }, [&] { launch_ccount<32>(v, ncap); },
                 [&] { launch_ccount<64>(v, ncap); });
        HIP_TRY(hipGetLastError());
        HIP_TRY(scan3_u32(cup.as<uint32_t>(), cup.as<uint32_t>() + ncap, &dc()->c32[C_UP],
                          cdn.as<uint32_t>(), cdn.as<uint32_t>() + ncap, &dc()->c32[C_DN],
                          cpair.as<uint32_t>(), cpair.as<uint32_t>() + ncap, &dc()->c32[C_PAIR],
                          ncap, tmp, st));
        return CH_OK;
      };
      TRY(after_search());
      TRY(readback());
      TRY(check_err());
      rs.rows_expanded = hctr->ls.rows;
      rs.arcs_scanned = hctr->ls.arcs;
      rs.memo_probes = hctr->ls.probes;
      rs.memo_inserts = hctr->ls.inserts;
      rs.n_ls_fallback = hctr->novf1;
      const uint32_t novf = hctr->novf2;
      rs.n_ls_global = novf;
      if (novf) {
        const uint32_t cap = (uint32_t)std::min<uint64_t>(next_pow2(2ull * O.n + 2), 1ull << 31);
        const bool hop = prm.wps_mode != CH_WPS_EXACT;  // a seventh array
        const size_t per = ((size_t)cap * (hop ? 7 : 6) + 4) * 4;
        size_t ntab = std::max<size_t>(1, std::min<size_t>({(size_t)novf, (size_t)cus * 2,
                                                            (size_t)(4ull << 30) / per}));
        HIP_TRY(gtabs.ensure(ntab * per));
        // key, dist (and dist2) = all ones; bitmaps, lists, counters = 0
        k_gtab_init<<<grid(ntab * (per / 4)), 256, 0, st>>>(gtabs.as<uint32_t>(), ntab * (per / 4),
                                                            per / 4, cap, hop);
        HIP_TRY(hipGetLastError());
        // the global tier searches the overlay as the other searches saw it:
        // this round's optimistic pruning is undone first and redone (and
        // recounted) by the second pass below
        if (nw) {
          HIP_TRY(hipMemsetAsync(&dc()->pruned, 0, sizeof(unsigned long long), st));
          k_unprune<<<grid((uint64_t)nw * kWave), 256, 0, st>>>(v, vw.as<uint32_t>(), nw,
                                                               prw.as<uint32_t>(), &dc()->err);
          HIP_TRY(hipGetLastError());
        }
        auto global = prm.wps_mode == CH_WPS_HOP
                          ? k_local_search_global<kWpsHop, kLsBlkWaves>
                          : prm.wps_mode == CH_WPS_SETTLED
                                ? k_local_search_global<kWpsSettled, kLsBlkWaves>
                                : k_local_search_global<kWpsExact, kLsBlkWaves>;
        if (stats) HIP_TRY(hipEventRecord(ev[7], st));
        global<<<(unsigned)ntab, kWave * kLsBlkWaves, 0, st>>>(
            v, ovf2.as<uint32_t>(), novf, aflag.as<uint8_t>(), mref(), &dc()->ls3, gtabs.as<uint32_t>(), cap, fstate().ws,
            &dc()->err, mode_limit(), ch->label.as<uint32_t>());
        HIP_TRY(hipGetLastError());
        if (stats) HIP_TRY(hipEventRecord(ev[8], st));
        TRY(after_search());
        TRY(readback());
        TRY(check_err());
      }
      mcount += hctr->ls.inserts + hctr->ls2.inserts + hctr->ls3.inserts;
      rs.rows2 = hctr->ls2.rows;  // block tier
      rs.arcs2 = hctr->ls2.arcs;
      rs.probes2 = hctr->ls2.probes;
      rs.inserts2 = hctr->ls2.inserts;
      rs.rows3 = hctr->ls3.rows;  // global tier
      rs.arcs3 = hctr->ls3.arcs;
      rs.probes3 = hctr->ls3.probes;
      rs.inserts3 = hctr->ls3.inserts;
      rs.n_targets = hctr->ls.targets + hctr->ls2.targets + hctr->ls3.targets;
      const uint32_t nf = hctr->c32[C_NF];
      rs.n_selected = nf;
      rs.n_pruned = hctr->pruned;
      if (nf == 0) return set_error(CH_E_DEVICE, "no vertex selected in a round (internal error)");

      // ---- Step 4: Contract (Alg. 7) -----------------------------------
      const uint32_t tup = hctr->c32[C_UP], tdn = hctr->c32[C_DN], ne = hctr->c32[C_PAIR];
      if (ch->nup + tup > up_cap) {
        uint64_t nc = std::max<uint64_t>((ch->nup + tup) * 3 / 2, up_cap * 2);
        for (int i = 0; i < 4; i++) TRY(grow_copy(*ub[i], ch->nup * 4, nc * 4));
        up_cap = nc;
      }
      if (ch->ndown + tdn > dn_cap) {
        uint64_t nc = std::max<uint64_t>((ch->ndown + tdn) * 3 / 2, dn_cap * 2);
        for (int i = 4; i < 8; i++) TRY(grow_copy(*ub[i], ch->ndown * 4, nc * 4));
        dn_cap = nc;
      }
      const size_t ne1 = std::max<uint32_t>(ne, 1);
      uint32_t *fb0 = rowb.as<uint32_t>(), *fb1 = fb0 + O.n, *rb0 = fb0 + 2 * (size_t)O.n,
               *rb1 = fb0 + 3 * (size_t)O.n;  // shortcut-row bounds, forward and reverse
      HIP_TRY(ekey.ensure(ne1 * 8));
      HIP_TRY(ekey_alt.ensure(ne1 * 8));
      HIP_TRY(eidx.ensure(ne1 * 4));
      HIP_TRY(eidx_alt.ensure(ne1 * 4));
      HIP_TRY(ew.ensure(ne1 * 4));
      HIP_TRY(elab.ensure(ne1 * 4));
      HIP_TRY(emid.ensure(ne1 * 4));
      HIP_TRY(ehead.ensure(ne1));
      HIP_TRY(eheads.ensure(ne1 * 4));
      HIP_TRY(ukey.ensure(ne1 * 8));
      HIP_TRY(uw.ensure(ne1 * 4));
      HIP_TRY(umid.ensure(ne1 * 4));
      HIP_TRY(rkey.ensure(ne1 * 8));
      HIP_TRY(rkey_alt.ensure(ne1 * 8));
      HIP_TRY(ridx.ensure(ne1 * 4));
      HIP_TRY(ridx_alt.ensure(ne1 * 4));
      const int kb = bits_for(O.n);
      dispatch(Gs, [&] { launch_contract<4>(v, nf, ncap, round, kb); },
               [&] { launch_contract<8>(v, nf, ncap, round, kb); },
               [&] { launch_contract<16>(v, nf, ncap, round, kb); },
               [&] { launch_contract<32>(v, nf, ncap, round, kb); },
               [&] { launch_contract<64>(v, nf, ncap, round, kb); });
      HIP_TRY(hipGetLastError());
      ch->nup += tup;
      ch->ndown += tdn;

      // shortcut set E+: sort candidates by (v1, v2), keep the minimum; the
      // number U of distinct pairs stays on the device (C_HEADS)
      const uint32_t *dU = &dc()->c32[C_HEADS];
      if (ne) {
        HIP_TRY(sort_u64_index(ekey.as<uint64_t>(), eidx.as<uint32_t>(), ekey_alt.as<uint64_t>(),
                               eidx_alt.as<uint32_t>(), ne, 2 * kb, tmp, st));
        k_run_heads<<<grid(ne), 256, 0, st>>>(ekey.as<uint64_t>(), ne, ehead.as<uint8_t>());
        HIP_TRY(hipGetLastError());
        HIP_TRY(select_flags(ehead.as<uint8_t>(), ne, eheads.as<uint32_t>(), &dc()->c32[C_HEADS],
                             tmp, st));
        k_eplus_reduce<<<grid(ne), 256, 0, st>>>(
            ekey.as<uint64_t>(), eidx.as<uint32_t>(), ne, eheads.as<uint32_t>(), dU,
            ew.as<uint32_t>(), elab.as<uint32_t>(), emid.as<uint32_t>(), kb, ukey.as<uint64_t>(),
            uw.as<uint32_t>(), umid.as<uint32_t>(), rkey.as<uint64_t>());
        HIP_TRY(hipGetLastError());
        if (batch) {
          k_count_by_graph<<<grid(ne), 256, 0, st>>>(ukey.as<uint64_t>(), dU, kb,
                                                     O.gid.as<uint32_t>(), batch->gof,
                                                     batch->shortcuts);
          HIP_TRY(hipGetLastError());
        }
        // reverse order (v2, v1) over all ne entries (written by the
        // reduction); the U real keys sort in front of the padding
        HIP_TRY(sort_u64_index(rkey.as<uint64_t>(), ridx.as<uint32_t>(), rkey_alt.as<uint64_t>(),
                               ridx_alt.as<uint32_t>(), ne, 2 * kb, tmp, st));
        k_row_bounds<<<dim3(grid(ne), 2), 256, 0, st>>>(ukey.as<uint64_t>(), rkey.as<uint64_t>(),
                                                         dU, kb, fb0, fb1, rb0, rb1);
        HIP_TRY(hipGetLastError());
      }

      // ---- overlay rebuild: drop V_F, merge E+ ---------------------------
      // sized by bounds known here: n2 < O.n vertices, m2 <= O.m + ne arcs;
      // the exact counts come with the round's last readback
      HIP_TRY(cnt2.ensure(((size_t)O.n + 1) * 4));
      HIP_TRY(cnt3.ensure(((size_t)O.n + 1) * 4));
      // keep flags; zero the row counts and the next round's flags
      k_keep<<<grid(O.n + 1), 256, 0, st>>>(O.n, F.as<uint8_t>(), cnt.as<uint32_t>(),
                                            cnt2.as<uint32_t>(), cnt3.as<uint32_t>(),
                                            wflag.as<uint8_t>(), aflag_next.as<uint8_t>());
      HIP_TRY(hipGetLastError());
      HIP_TRY(scan_u32(cnt.as<uint32_t>(), newid.as<uint32_t>(), O.n, &dc()->c32[C_NNEW], tmp, st));
      OvBuf &N = ov[cur ^ 1];
      const uint64_t mcap2 = std::max<uint64_t>((uint64_t)O.m + ne, 1);
      HIP_TRY(N.foff.ensure(((size_t)O.n + 2) * 4));
      HIP_TRY(N.roff.ensure(((size_t)O.n + 2) * 4));
      HIP_TRY(N.gid.ensure(std::max<size_t>(O.n, 1) * 4));
      HIP_TRY(N.P.ensure(std::max<size_t>(O.n, 1) * 4));
      HIP_TRY(N.farc.ensure(mcap2 * 8));
      HIP_TRY(N.rarc.ensure(mcap2 * 8));
      HIP_TRY(N.fmid.ensure(mcap2 * 4));
      HIP_TRY(N.rmid.ensure(mcap2 * 4));
      // row lengths of the new overlay (new ids < n2, zero up to O.n), then
      // offsets over O.n + 1 entries: foff[n2 .. O.n] all equal m2
      const int gm = pick_group(avgdeg);
      dispatch(gm, [&] { merge_rows<4>(O, N, kb, fb0, fb1, rb0, rb1); },
               [&] { merge_rows<8>(O, N, kb, fb0, fb1, rb0, rb1); },
               [&] { merge_rows<16>(O, N, kb, fb0, fb1, rb0, rb1); },
               [&] { merge_rows<32>(O, N, kb, fb0, fb1, rb0, rb1); },
               [&] { merge_rows<64>(O, N, kb, fb0, fb1, rb0, rb1); });
      TRY(merge_err);
      // carry state; V_W' = V_S + N_in(V_S); V_A' = N(V_F) (flags zeroed by
      // k_keep, so they are zero beyond the new vertex count)
      k_carry<<<grid(O.n), 256, 0, st>>>(O.n, F.as<uint8_t>(), newid.as<uint32_t>(),
                                         O.gid.as<uint32_t>(), O.P.as<int32_t>(), S.as<uint8_t>(),
                                         newA.as<uint8_t>(), N.gid.as<uint32_t>(),
                                         N.P.as<int32_t>(), wflag.as<uint8_t>(),
                                         aflag_next.as<uint8_t>());
      HIP_TRY(hipGetLastError());
      k_mark_in_neighbours<<<grid(O.n), 256, 0, st>>>(O.n, F.as<uint8_t>(), S.as<uint8_t>(),
                                                      newid.as<uint32_t>(), N.roff.as<uint32_t>(),
                                                      N.rarc.as<uint2>(), wflag.as<uint8_t>());
      HIP_TRY(hipGetLastError());
      HIP_TRY(select_flags2(wflag.as<uint8_t>(), aflag_next.as<uint8_t>(), O.n, vw.as<uint32_t>(),
                            va.as<uint32_t>(), &dc()->c32[C_UP], &dc()->c32[C_DN], tmp, st));
      // upper bound on the next round's memo inserts: in-degree x out-degree
      // summed over the affected vertices (rows past the new vertex count
      // are empty)
      {
        Overlay vb = view(N);
        vb.n = O.n;
        // the bound accumulates into the counter cleared at the round start
        k_ls_bound_affected<<<grid(O.n), 256, 0, st>>>(vb, aflag_next.as<uint8_t>(),
                                                       &dc()->bound);
        HIP_TRY(hipGetLastError());
      }
      if (stats) HIP_TRY(hipEventRecord(ev[4], st));
      TRY(readback());
      TRY(check_err());
      const uint32_t n2 = hctr->c32[C_NNEW], m2 = hctr->c32[C_MF];
      if (hctr->c32[C_MR] != m2)
        return set_error(CH_E_DEVICE, "forward and reverse overlay disagree (internal error)");
      if (n2 >= O.n || m2 > mcap2)
        return set_error(CH_E_DEVICE, "overlay rebuild out of bounds (internal error)");
      N.n = n2;
      N.m = m2;
      rs.n_shortcuts = hctr->c32[C_HEADS];
      nw = hctr->c32[C_UP];
      na = hctr->c32[C_DN];
      next_bound = hctr->bound;
      std::swap(aflag, aflag_next);
      cur ^= 1;
      rs.overlay_arcs = m2;
      if (stats) {
        float ls = 0.f, tot = 0.f;
        if (rs.n_sources) HIP_TRY(hipEventElapsedTime(&ls, ev[2], ev[3]));
        HIP_TRY(hipEventElapsedTime(&tot, ev[1], ev[4]));
        rs.ms_local_search = ls;
        rs.ms_total = tot;
        if (blk_ran) HIP_TRY(hipEventElapsedTime(&rs.ms_ls_blk, ev[5], ev[6]));
        if (rs.n_ls_global) HIP_TRY(hipEventElapsedTime(&rs.ms_ls_global, ev[7], ev[8]));
      }
      ch->stats.push_back(rs);
      round++;
      sc_total += rs.n_shortcuts;
      if (prm.flags & CH_F_PROGRESS) {  // a line at most every 5 s
        const auto now = std::chrono::steady_clock::now();
        if (now - last_note > std::chrono::seconds(5)) {
          last_note = now;
          std::fprintf(stderr, "[ch_build] round %u: %u vertices left, %llu shortcuts\n", round,
                       n2, sc_total);
          std::fflush(stderr);
        }
      }
    }
    ch->rounds = round;
    if (renum) TRY(restore_order());
    return CH_OK;
  }
};

hipError_t fw_init(uint32_t *D, uint32_t N, hipStream_t st) {
  const uint64_t nn = (uint64_t)N * N;
  k_fw_init<<<(unsigned)std::max<uint64_t>(1, std::min<uint64_t>((nn + 255) / 256, 65535)), 256, 0,
              st>>>(D, N);
  return hipGetLastError();
}

hipError_t fw_close(uint32_t *D, uint32_t N, hipStream_t st) {
  const uint32_t nb = N / kFwTile;
  for (uint32_t k = 0; k < nb; k++) {
    k_fw_diag<<<1, kFwDiagThreads, 0, st>>>(D, N, k);
    if (nb > 1) {
      k_fw_panels<<<2 * nb, kFwThreads, 0, st>>>(D, N, k);
      k_fw_rest<<<nb * nb, kFwThreads, 0, st>>>(D, N, k);
    }
  }
  return hipGetLastError();
}

static int check_params(const ch_params_t *p, ch_params_t &prm) {
  prm = ch_params_t{};
  if (p) prm = *p;
  if (prm.wps_mode != CH_WPS_EXACT && prm.wps_mode != CH_WPS_HOP &&
      prm.wps_mode != CH_WPS_SETTLED)
    return set_error(CH_E_UNSUPPORTED, "unknown wps_mode");
  if (prm.wps_mode == CH_WPS_HOP && prm.hop_limit < 1)
    return set_error(CH_E_INVALID, "hop mode needs hop_limit >= 1");
  if (prm.wps_mode == CH_WPS_SETTLED && prm.settle_limit < 1)
    return set_error(CH_E_INVALID, "settled mode needs settle_limit >= 1");
  if (prm.ls_step > CH_LS_STEP_ALL) return set_error(CH_E_INVALID, "ls_step must be at most 32");
  if (prm.mlp_qbits > 24) return set_error(CH_E_INVALID, "mlp_qbits must be at most 24");
  if (!prm.mlp_qbits) prm.mlp_qbits = 16;
  if (prm.dense_tail > kTabMaxN)
    return set_error(CH_E_INVALID, "dense_tail must be at most 4096");
  if (prm.group && prm.group != 4 && prm.group != 8 && prm.group != 16 && prm.group != 32 &&
      prm.group != 64)
    return set_error(CH_E_INVALID, "group must be 0, 4, 8, 16, 32 or 64");
  if (prm.ls_sparse > CH_LS_64x2048 || prm.ls_dense > CH_LS_64x2048)
    return set_error(CH_E_INVALID, "unknown first-tier search kernel");
  if (prm.priority > CH_PRIO_LEARNED) return set_error(CH_E_INVALID, "unknown priority");
  if (prm.priority == CH_PRIO_LEARNED && !prm.mlp)
    return set_error(CH_E_INVALID, "the learned priority needs mlp weights");
  if (prm.tiebreak > CH_TIE_RAW_ID) return set_error(CH_E_INVALID, "unknown tiebreak");
  // without CH_F_SCORE_WEIGHTS the score is the plain edge difference; the
  // learned priority replaces the score, so it takes no weights
  if (!(prm.flags & CH_F_SCORE_WEIGHTS) || prm.priority == CH_PRIO_LEARNED) {
    prm.k_ed = 1;
    prm.k_cn = 0;
    prm.k_depth = 0;
  }
  return CH_OK;
}

static int new_ch(hipStream_t stream, bool create_stream, ch_s **out) {
  ch_s *ch = new (std::nothrow) ch_s();
  if (!ch) return set_error(CH_E_OOM, "out of host memory");
  hipError_t e = hipGetDevice(&ch->device);
  if (e != hipSuccess) {
    delete ch;
    return hip_error(e, "hipGetDevice");
  }
  if (stream || !create_stream) {
    ch->stream = stream;
  } else {
    e = hipStreamCreateWithFlags(&ch->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete ch;
      return hip_error(e, "hipStreamCreate");
    }
    ch->own_stream = true;
  }
  *out = ch;
  return CH_OK;
}

// Rounds + postprocessing of `g` into ch (timed with events on ch's stream).
static int run_build(ch_s *ch, const ch_graph_t *g, const ch_params_t &prm,
                     const Builder::Batch *batch) {
  int rc;
  Builder b;
  b.ch = ch;
  b.st = ch->stream;
  b.prm = prm;
  b.n = g->n;
  b.batch = batch;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ch->device) ==
          hipSuccess &&
      cus > 0)
    b.cus = cus;
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  (void)hipEventRecord(t0, b.st);
  rc = b.run(g);
  if (rc == CH_OK)
    rc = postprocess(ch, !batch && !(prm.flags & CH_F_NO_QUERY_INDEX), batch ? batch->gof : nullptr,
                     batch ? batch->k : 0);
  (void)hipEventRecord(t1, b.st);
  if (rc == CH_OK) {
    hipError_t se = hipEventSynchronize(t1);
    if (se != hipSuccess) rc = hip_error(se, "build");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    ch->summary.ms_build = ms;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (rc == CH_OK) ch->summary.memo_entries = b.mcount;
  if (rc != CH_OK) (void)hipStreamSynchronize(ch->stream);
  return rc;
}

static void fill_summary(ch_s *ch) {
  ch->summary.n = ch->n;
  ch->summary.rounds = ch->rounds;
  ch->summary.m_input = ch->m_input;
  ch->summary.up_arcs = ch->nup;
  ch->summary.down_arcs = ch->ndown;
  uint64_t sc = 0;
  for (auto &r : ch->stats) sc += r.n_shortcuts;
  ch->summary.shortcuts = sc;
}

int build_ch(const ch_graph_t *g, const ch_params_t *p, ch_t **out) {
  clear_error();
  if (!g || !out) return set_error(CH_E_INVALID, "graph and out must not be NULL");
  ch_params_t prm;
  TRY(check_params(p, prm));
  if (g->n == 0xFFFFFFFFu) return set_error(CH_E_INVALID, "n must be at most 0xFFFFFFFE");
  if (!g->offsets || (g->m && (!g->dst || !g->w)))
    return set_error(CH_E_INVALID, "offsets, dst and w must not be NULL");
  if (g->labels && prm.tiebreak == CH_TIE_RAW_ID)
    return set_error(CH_E_INVALID, "CH_TIE_RAW_ID takes no labels");
  ch_s *ch = nullptr;
  TRY(new_ch((hipStream_t)prm.stream, true, &ch));
  ch->n = g->n;
  int rc = run_build(ch, g, prm, nullptr);
  if (rc != CH_OK) {
    delete ch;
    return rc;
  }
  fill_summary(ch);
  *out = ch;
  return CH_OK;
}

// ---------------------------------------------------------------------------
// batched construction: the k graphs become one disjoint union (ids shifted
// by each graph's vertex base, labels kept per graph), the rounds run once,
// and the result is split.  Every rule of a round is local to a vertex's own
// graph and every tie is broken by the graph's own labels, so each graph's
// CH equals the one ch_build gives it alone.
// ---------------------------------------------------------------------------
int build_batch(const ch_graph_t *gs, uint32_t k, const ch_params_t *p, ch_t **outs) {
  clear_error();
  if (!gs || !outs || k == 0) return set_error(CH_E_INVALID, "graphs and outs must not be NULL");
  ch_params_t prm;
  TRY(check_params(p, prm));
  if (prm.flags & CH_F_RECORD_FEATURES)
    return set_error(CH_E_UNSUPPORTED, "feature recording is not available for batches");
  const bool on_dev = prm.flags & CH_F_INPUT_ON_DEVICE;
  std::vector<uint32_t> vb(k + 1, 0);
  std::vector<uint64_t> ab(k + 1, 0);
  bool any_labels = false, all_labels = true;
  for (uint32_t g = 0; g < k; g++) {
    const ch_graph_t &G = gs[g];
    if (!G.offsets || (G.m && (!G.dst || !G.w)))
      return set_error(CH_E_INVALID, "offsets, dst and w must not be NULL");
    if ((uint64_t)vb[g] + G.n > 0xFFFFFFFEull)
      return set_error(CH_E_UNSUPPORTED, "the batch has more than 0xFFFFFFFE vertices");
    vb[g + 1] = vb[g] + G.n;
    ab[g + 1] = ab[g] + G.m;
    any_labels |= G.labels != nullptr;
    all_labels &= G.labels != nullptr || G.n == 0;
  }
  if (any_labels && !all_labels)
    return set_error(CH_E_INVALID, "either every graph of a batch has labels or none has");
  if (any_labels && prm.tiebreak == CH_TIE_RAW_ID)
    return set_error(CH_E_INVALID, "CH_TIE_RAW_ID takes no labels");
  const uint32_t n = vb[k];
  const uint64_t m = ab[k];
  if (m >= 0xFFFFFFFFull)
    return set_error(CH_E_UNSUPPORTED, "the batch has 2^32 - 1 or more arcs");
  const size_t n1 = std::max<uint32_t>(n, 1), m1 = std::max<uint64_t>(m, 1);

  ch_s *U = nullptr;
  TRY(new_ch((hipStream_t)prm.stream, true, &U));
  U->n = n;
  hipStream_t st = U->stream;
  DBuf d_vb, d_ab, stage, off, dst, w, gof, sc, min, mx, dbad;
  auto cleanup = [&]() {
    DBuf *all[] = {&d_vb, &d_ab, &stage, &off, &dst, &w, &gof, &sc, &min, &mx, &dbad};
    for (DBuf *b : all) b->release();
  };
  auto fail = [&](int rc) {
    (void)hipStreamSynchronize(st);
    cleanup();
    delete U;
    return rc;
  };
#define BTRY(expr)                                              \
  do {                                                          \
    hipError_t e_ = (expr);                                     \
    if (e_ != hipSuccess) return fail(hip_error(e_, #expr));    \
  } while (0)
  const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  BTRY(d_vb.ensure((k + 1) * 4));
  BTRY(d_ab.ensure((k + 1) * 8));
  BTRY(stage.ensure(((size_t)n + k) * 8));
  BTRY(off.ensure((n1 + 1) * 8));
  BTRY(dst.ensure(m1 * 4));
  BTRY(w.ensure(m1 * 4));
  BTRY(gof.ensure(n1 * 4));
  BTRY(sc.ensure(k * 8));
  BTRY(min.ensure(k * 8));
  BTRY(mx.ensure(k * 4));
  BTRY(dbad.ensure(4));
  BTRY(U->label.ensure(n1 * 4));
  BTRY(hipMemcpyAsync(d_vb.p, vb.data(), (k + 1) * 4, hipMemcpyHostToDevice, st));
  BTRY(hipMemcpyAsync(d_ab.p, ab.data(), (k + 1) * 8, hipMemcpyHostToDevice, st));
  BTRY(hipMemsetAsync(sc.p, 0, k * 8, st));
  BTRY(hipMemsetAsync(min.p, 0, k * 8, st));
  BTRY(hipMemsetAsync(mx.p, 0, k * 4, st));
  BTRY(hipMemsetAsync(dbad.p, 0, 4, st));
  for (uint32_t g = 0; g < k; g++) {
    const ch_graph_t &G = gs[g];
    BTRY(hipMemcpyAsync(stage.as<uint64_t>() + vb[g] + g, G.offsets, ((size_t)G.n + 1) * 8, kind,
                        st));
    if (G.m) {
      BTRY(hipMemcpyAsync(dst.as<uint32_t>() + ab[g], G.dst, G.m * 4, kind, st));
      BTRY(hipMemcpyAsync(w.as<uint32_t>() + ab[g], G.w, G.m * 4, kind, st));
    }
    if (G.labels && G.n)
      BTRY(hipMemcpyAsync(U->label.as<uint32_t>() + vb[g], G.labels, (size_t)G.n * 4, kind, st));
  }
  const unsigned gr = 1024;
  if (n) {
    k_batch_offsets<<<gr, 256, 0, st>>>(n, k, d_vb.as<uint32_t>(), d_ab.as<uint64_t>(),
                                        stage.as<uint64_t>(), off.as<uint64_t>(),
                                        gof.as<uint32_t>(), dbad.as<uint32_t>());
    BTRY(hipGetLastError());
  }
  BTRY(hipMemcpyAsync(off.as<uint64_t>() + n, &ab[k], 8, hipMemcpyHostToDevice, st));
  if (m) {
    k_batch_arcs<<<gr, 256, 0, st>>>(m, k, d_vb.as<uint32_t>(), d_ab.as<uint64_t>(),
                                     dst.as<uint32_t>(), dbad.as<uint32_t>());
    BTRY(hipGetLastError());
  }
  if (!any_labels && n) {
    const uint32_t mix = (uint32_t)prm.seed ^ (uint32_t)(prm.seed >> 32);
    k_batch_default_labels<<<gr, 256, 0, st>>>(n, k, d_vb.as<uint32_t>(), mix,
                                               prm.tiebreak == CH_TIE_RAW_ID,
                                               U->label.as<uint32_t>());
    BTRY(hipGetLastError());
  }
  if (any_labels && n > 1) {  // distinct within each graph
    DBuf k1, k2, v1, v2, tmp;
    BTRY(k1.ensure(n1 * 8));
    BTRY(k2.ensure(n1 * 8));
    BTRY(v1.ensure(n1 * 4));
    BTRY(v2.ensure(n1 * 4));
    k_graph_label_keys<<<gr, 256, 0, st>>>(n, gof.as<uint32_t>(), U->label.as<uint32_t>(),
                                           k1.as<uint64_t>());
    BTRY(iota_u32(v1.as<uint32_t>(), n, st));
    int kbits = 1;
    while (kbits < 32 && (1u << kbits) < k) kbits++;
    BTRY(radix_sort_u64(k1.as<uint64_t>(), v1.as<uint32_t>(), k2.as<uint64_t>(),
                        v2.as<uint32_t>(), n, 32 + kbits, tmp, st));
    k_adjacent_equal<<<gr, 256, 0, st>>>(n, k1.as<uint64_t>(), dbad.as<uint32_t>());
    BTRY(hipGetLastError());
    BTRY(hipStreamSynchronize(st));
    DBuf *bb[] = {&k1, &k2, &v1, &v2, &tmp};
    for (DBuf *b : bb) b->release();
  }
  uint32_t bad = 0;
  BTRY(hipMemcpyAsync(&bad, dbad.p, 4, hipMemcpyDeviceToHost, st));
  BTRY(hipStreamSynchronize(st));
  if (bad & 8) return fail(set_error(CH_E_INVALID, "a graph's offsets[0] is not 0 or offsets[n] is not m"));
  if (bad & 1) return fail(set_error(CH_E_INVALID, "a graph's offsets exceed its arc count"));
  if (bad & 2) return fail(set_error(CH_E_INVALID, "an arc has head >= n or weight 0xFFFFFFFF"));
  if (bad & 4) return fail(set_error(CH_E_INVALID, "labels are not distinct within a graph"));

  ch_graph_t ug{n, m, off.as<uint64_t>(), dst.as<uint32_t>(), w.as<uint32_t>(), U->label.as<uint32_t>()};
  ch_params_t uprm = prm;
  uprm.flags |= CH_F_INPUT_ON_DEVICE;
  Builder::Batch binfo;
  binfo.k = k;
  binfo.gof = gof.as<uint32_t>();
  binfo.shortcuts = sc.as<unsigned long long>();
  binfo.m_in = min.as<unsigned long long>();
  int rc = run_build(U, &ug, uprm, &binfo);
  if (rc != CH_OK) return fail(rc);

  // split: arcs per graph (sorted by graph, then rank), rounds per graph
  std::vector<unsigned long long> up_cnt(k, 0), dn_cnt(k, 0), h_sc(k), h_min(k);
  std::vector<uint32_t> h_mx(k);
  {
    DBuf cu, cd;
    BTRY(cu.ensure(k * 8));
    BTRY(cd.ensure(k * 8));
    BTRY(hipMemsetAsync(cu.p, 0, k * 8, st));
    BTRY(hipMemsetAsync(cd.p, 0, k * 8, st));
    if (U->nup)
      k_arcs_by_graph<<<gr, 256, 0, st>>>(U->nup, U->up_t.as<uint32_t>(), gof.as<uint32_t>(),
                                          cu.as<unsigned long long>());
    if (U->ndown)
      k_arcs_by_graph<<<gr, 256, 0, st>>>(U->ndown, U->dn_h.as<uint32_t>(), gof.as<uint32_t>(),
                                          cd.as<unsigned long long>());
    if (n)
      k_level_max_by_graph<<<gr, 256, 0, st>>>(n, U->level.as<uint32_t>(), gof.as<uint32_t>(),
                                               mx.as<uint32_t>());
    BTRY(hipGetLastError());
    BTRY(hipMemcpyAsync(up_cnt.data(), cu.p, k * 8, hipMemcpyDeviceToHost, st));
    BTRY(hipMemcpyAsync(dn_cnt.data(), cd.p, k * 8, hipMemcpyDeviceToHost, st));
    BTRY(hipMemcpyAsync(h_sc.data(), sc.p, k * 8, hipMemcpyDeviceToHost, st));
    BTRY(hipMemcpyAsync(h_min.data(), min.p, k * 8, hipMemcpyDeviceToHost, st));
    BTRY(hipMemcpyAsync(h_mx.data(), mx.p, k * 4, hipMemcpyDeviceToHost, st));
    BTRY(hipStreamSynchronize(st));
    cu.release();
    cd.release();
  }
  std::vector<ch_s *> made;
  auto fail_split = [&](int rc2) {
    for (ch_s *c : made) delete c;
    return fail(rc2);
  };
  uint64_t ubase = 0, dbase = 0;
  for (uint32_t g = 0; g < k; g++) {
    ch_s *c = nullptr;
    int r2 = new_ch((hipStream_t)prm.stream, false, &c);
    if (r2 != CH_OK) return fail_split(r2);
    made.push_back(c);
    const uint32_t ng = vb[g + 1] - vb[g];
    c->n = ng;
    c->nup = up_cnt[g];
    c->ndown = dn_cnt[g];
    c->rounds = h_mx[g];
    c->m_input = h_min[g];
    const size_t ng1 = std::max<uint32_t>(ng, 1);
    hipStream_t cs = c->stream;
    hipError_t e2;
#define STRY(expr)                                   \
  do {                                               \
    if ((e2 = (expr)) != hipSuccess) return fail_split(hip_error(e2, #expr)); \
  } while (0)
    STRY(c->level.ensure(ng1 * 4));
    STRY(c->score.ensure(ng1 * 4));
    STRY(c->label.ensure(ng1 * 4));
    STRY(c->rank.ensure(ng1 * 4));
    STRY(hipStreamSynchronize(st));
    if (ng) {
      STRY(hipMemcpyAsync(c->level.p, U->level.as<uint32_t>() + vb[g], ng * 4,
                          hipMemcpyDeviceToDevice, cs));
      STRY(hipMemcpyAsync(c->score.p, U->score.as<int32_t>() + vb[g], ng * 4,
                          hipMemcpyDeviceToDevice, cs));
      STRY(hipMemcpyAsync(c->label.p, U->label.as<uint32_t>() + vb[g], ng * 4,
                          hipMemcpyDeviceToDevice, cs));
      k_sub_base<<<gr, 256, 0, cs>>>(ng, U->rank.as<uint32_t>() + vb[g], vb[g], false,
                                     c->rank.as<uint32_t>());
      STRY(hipGetLastError());
    }
    DBuf *cu_[] = {&c->up_t, &c->up_h, &c->up_w, &c->up_m};
    DBuf *uu_[] = {&U->up_t, &U->up_h, &U->up_w, &U->up_m};
    DBuf *cd_[] = {&c->dn_t, &c->dn_h, &c->dn_w, &c->dn_m};
    DBuf *ud_[] = {&U->dn_t, &U->dn_h, &U->dn_w, &U->dn_m};
    for (int q = 0; q < 4; q++) {
      STRY(cu_[q]->ensure(std::max<uint64_t>(c->nup, 1) * 4));
      STRY(cd_[q]->ensure(std::max<uint64_t>(c->ndown, 1) * 4));
      if (c->nup)
        k_sub_base<<<gr, 256, 0, cs>>>(c->nup, uu_[q]->as<uint32_t>() + ubase,
                                       q == 2 ? 0u : vb[g], q == 3, cu_[q]->as<uint32_t>());
      if (c->ndown)
        k_sub_base<<<gr, 256, 0, cs>>>(c->ndown, ud_[q]->as<uint32_t>() + dbase,
                                       q == 2 ? 0u : vb[g], q == 3, cd_[q]->as<uint32_t>());
      STRY(hipGetLastError());
    }
    ubase += c->nup;
    dbase += c->ndown;
    if (!(prm.flags & CH_F_NO_QUERY_INDEX)) {
      r2 = build_index(c);
      if (r2 != CH_OK) return fail_split(r2);
    }
    STRY(hipStreamSynchronize(cs));
#undef STRY
    c->summary.n = ng;
    c->summary.rounds = c->rounds;
    c->summary.m_input = c->m_input;
    c->summary.up_arcs = c->nup;
    c->summary.down_arcs = c->ndown;
    c->summary.shortcuts = h_sc[g];
    c->summary.memo_entries = 0;
    c->summary.ms_build = U->summary.ms_build;
  }
#undef BTRY
  for (uint32_t g = 0; g < k; g++) outs[g] = made[g];
  cleanup();
  delete U;
  return CH_OK;
}

}  // namespace sp

ch_s::~ch_s() {
  sp::DBuf *all[] = {&level, &score, &label, &rank, &up_t, &up_h, &up_w, &up_m, &dn_t, &dn_h,
                     &dn_w, &dn_m, &q_upoff, &q_uparc, &q_dnoff, &q_dnarc, &q_lstart, &q_wend, &q_s, &q_t, &q_d,
                     &q_ovf, &q_tab, &q_ctr, &rec, &q_v, &q_ovf2, &q_gtab, &q_phast,
                     &q_core, &q_core_max, &q_core1};
  for (sp::DBuf *b : all) b->release();
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}
