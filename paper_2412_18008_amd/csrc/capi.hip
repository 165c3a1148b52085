// capi.hip -- the extern "C" entry points declared in include/spoch.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "builder.hpp"
#include "mlp.hpp"

namespace sp {
const char *last_error_msg();
void clear_error();
}  // namespace sp

using sp::set_error;

extern "C" {

int ch_build(const ch_graph_t *g, const ch_params_t *p, ch_t **out) {
  return sp::build_ch(g, p, out);
}

int ch_build_batch(const ch_graph_t *gs, uint32_t k, const ch_params_t *p, ch_t **outs) {
  return sp::build_batch(gs, k, p, outs);
}

int ch_query_batch(const ch_t *ch, const uint32_t *s, const uint32_t *t, uint64_t q,
                   uint64_t *dist, uint32_t flags, void *stream) {
  sp::clear_error();
  if (!ch) return set_error(CH_E_INVALID, "ch must not be NULL");
  if (q && (!s || !t || !dist)) return set_error(CH_E_INVALID, "s, t and dist must not be NULL");
  return sp::query_batch(ch, s, t, q, dist, nullptr, flags, (hipStream_t)stream);
}

int ch_query_batch_stats(const ch_t *ch, const uint32_t *s, const uint32_t *t, uint64_t q,
                         uint64_t *dist, uint32_t *visited, uint32_t flags, void *stream) {
  sp::clear_error();
  if (!ch) return set_error(CH_E_INVALID, "ch must not be NULL");
  if (q && (!s || !t || !dist || !visited))
    return set_error(CH_E_INVALID, "s, t, dist and visited must not be NULL");
  return sp::query_batch(ch, s, t, q, dist, visited, flags, (hipStream_t)stream);
}

int ch_one_to_all(const ch_t *ch, const uint32_t *s, uint32_t ks, const uint32_t *t, uint32_t kt,
                  uint64_t *dist, uint32_t flags, void *stream) {
  sp::clear_error();
  if (!ch) return set_error(CH_E_INVALID, "ch must not be NULL");
  if (ks && (!s || !dist)) return set_error(CH_E_INVALID, "s and dist must not be NULL");
  if (t && !kt) return set_error(CH_E_INVALID, "a target list needs kt > 0");
  return sp::one_to_all(ch, s, ks, t, kt, dist, flags, (hipStream_t)stream);
}

int ch_query_batch_noalloc(const ch_t *ch, const uint32_t *s, const uint32_t *t, uint64_t q,
                           uint64_t *dist, uint32_t *visited, uint32_t flags, void *stream) {
  sp::clear_error();
  if (!ch) return set_error(CH_E_INVALID, "ch must not be NULL");
  if (q && (!s || !t || !dist)) return set_error(CH_E_INVALID, "s, t and dist must not be NULL");
  return sp::query_batch_noalloc(ch, s, t, q, dist, visited, flags, (hipStream_t)stream);
}

static int copy_out(void *dst, const sp::DBuf &src, uint64_t count, hipStream_t st) {
  if (!dst || !count) return CH_OK;
  hipError_t e = hipMemcpyAsync(dst, src.p, count * 4, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return sp::hip_error(e, "ch_export copy");
  return CH_OK;
}

int ch_export(const ch_t *ch, uint32_t *level, int32_t *score, uint32_t *rank, uint32_t *up_tail,
              uint32_t *up_head, uint32_t *up_w, uint32_t *up_mid, uint32_t *down_tail,
              uint32_t *down_head, uint32_t *down_w, uint32_t *down_mid) {
  sp::clear_error();
  if (!ch) return set_error(CH_E_INVALID, "ch must not be NULL");
  hipStream_t st = ch->stream;
  int rc;
  if ((rc = copy_out(level, ch->level, ch->n, st)) || (rc = copy_out(score, ch->score, ch->n, st)) ||
      (rc = copy_out(rank, ch->rank, ch->n, st)) || (rc = copy_out(up_tail, ch->up_t, ch->nup, st)) ||
      (rc = copy_out(up_head, ch->up_h, ch->nup, st)) ||
      (rc = copy_out(up_w, ch->up_w, ch->nup, st)) ||
      (rc = copy_out(up_mid, ch->up_m, ch->nup, st)) ||
      (rc = copy_out(down_tail, ch->dn_t, ch->ndown, st)) ||
      (rc = copy_out(down_head, ch->dn_h, ch->ndown, st)) ||
      (rc = copy_out(down_w, ch->dn_w, ch->ndown, st)) ||
      (rc = copy_out(down_mid, ch->dn_m, ch->ndown, st)))
    return rc;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return sp::hip_error(e, "ch_export");
  return CH_OK;
}

int ch_get_summary(const ch_t *ch, ch_summary_t *out) {
  sp::clear_error();
  if (!ch || !out) return set_error(CH_E_INVALID, "ch and out must not be NULL");
  *out = ch->summary;
  return CH_OK;
}

int ch_get_query_stats(const ch_t *ch, ch_query_stats_t *out) {
  sp::clear_error();
  if (!ch || !out) return set_error(CH_E_INVALID, "ch and out must not be NULL");
  *out = ch->qstats;
  return CH_OK;
}

int ch_get_round_stats(const ch_t *ch, ch_round_stats_t *out, uint32_t cap) {
  sp::clear_error();
  if (!ch || (cap && !out)) return set_error(CH_E_INVALID, "ch and out must not be NULL");
  const uint32_t k = (uint32_t)std::min<size_t>(cap, ch->stats.size());
  if (k) memcpy(out, ch->stats.data(), (size_t)k * sizeof(ch_round_stats_t));
  return CH_OK;
}

int ch_export_features(const ch_t *ch, float *x) {
  sp::clear_error();
  if (!ch || !x) return set_error(CH_E_INVALID, "ch and x must not be NULL");
  if (!ch->has_rec) return set_error(CH_E_INVALID, "the CH was built without CH_F_RECORD_FEATURES");
  if (!ch->n) return CH_OK;
  hipError_t e = hipMemcpyAsync(x, ch->rec.p, (size_t)ch->n * 32, hipMemcpyDeviceToHost, ch->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ch->stream);
  if (e != hipSuccess) return sp::hip_error(e, "ch_export_features");
  return CH_OK;
}

int ch_mlp_forward(const float *x, uint64_t n, const float *w, float *y, int32_t *prio,
                   uint32_t flags, void *stream) {
  sp::clear_error();
  if ((n && !x) || !w) return set_error(CH_E_INVALID, "x and w must not be NULL");
  return sp::mlp_forward(x, n, w, y, prio, flags, (hipStream_t)stream);
}

int ch_mlp_grad(const float *x, const float *t, uint32_t n, const float *w, float *grad,
                float *loss, uint32_t flags, void *stream) {
  sp::clear_error();
  if (!x || !t || !w || !grad) return set_error(CH_E_INVALID, "x, t, w and grad must not be NULL");
  return sp::mlp_grad(x, t, n, w, grad, loss, flags, (hipStream_t)stream);
}

int ch_mlp_train(const float *x, const float *t, uint64_t n, float *w,
                 const ch_mlp_train_params_t *p, float *losses, uint32_t flags, void *stream) {
  sp::clear_error();
  if (!x || !t || !w || !p) return set_error(CH_E_INVALID, "x, t, w and p must not be NULL");
  return sp::mlp_train(x, t, n, w, p, losses, flags, (hipStream_t)stream);
}

void ch_free(ch_t *ch) {
  if (!ch) return;
  (void)hipStreamSynchronize(ch->stream);
  delete ch;
}

const char *ch_last_error(void) { return sp::last_error_msg(); }

const char *ch_version(void) { return "spoch-gfx950 0.1"; }

}  // extern "C"
