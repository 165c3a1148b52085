/*
 * spoch_oracle.c -- CPU oracle for round-synchronous contraction-hierarchy
 * construction, following Wan et al., "Parallel Contraction Hierarchies Can
 * Be Efficient and Scalable" (ICS 2025).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain sequential C, written for readability,
 * not speed.  It defines the result the GPU library must reproduce bit for
 * bit, and it is used only by the tests, the smoke check and the
 * benchmark's CPU baseline.  It shares no code with the GPU library.
 *
 * Map of the paper onto this file (published numbering):
 *   orc_round()      one iteration of the main loop of Alg. 3
 *     local_search() Alg. 4, "Step 1: Local Search with Memoization"
 *     prune()        the deletion at the end of Alg. 4
 *     score()        Alg. 5, "Step 2: Score" (edge difference)
 *     select_set()   Alg. 6, "Step 3: Select"
 *     contract()     Alg. 7, "Step 4: Contract", plus the combination of
 *                    the shortcut set with the overlay ("Maintaining the
 *                    Overlay Graph Dynamically", keep the smaller weight)
 *   orc_finish()     "Postprocessing": re-index by level, then score
 *   orc_query()      "Query on Contraction Hierarchies": bidirectional
 *                    upward search
 *
 * Points the paper leaves open are fixed as marked "READING:"; each reading
 * makes the output a pure function of (graph, labels, parameters).
 */
#include "spoch_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define INF32 0xFFFFFFFFu
#define MAXW 0xFFFFFFFEu
#define NOMID 0xFFFFFFFFu
#define INF64 0xFFFFFFFFFFFFFFFFull

/* ------------------------------------------------------------------ */
/* small utilities                                                     */
/* ------------------------------------------------------------------ */

/* MurmurHash3 32-bit finaliser (Appleby), a bijection on uint32. */
static uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

uint32_t orc_default_label(uint32_t v, uint64_t seed) {
  return fmix32(v ^ (uint32_t)seed ^ (uint32_t)(seed >> 32));
}

typedef struct {
  uint32_t v;   /* the other endpoint */
  uint32_t w;   /* weight */
  uint32_t mid; /* middle vertex of a shortcut, NOMID for an input arc */
} arc_t;

typedef struct {
  arc_t *a;
  uint32_t n, cap;
} adj_t;

static int adj_push(adj_t *l, uint32_t v, uint32_t w, uint32_t mid) {
  if (l->n == l->cap) {
    uint32_t nc = l->cap ? 2 * l->cap : 4;
    arc_t *na = (arc_t *)realloc(l->a, (size_t)nc * sizeof(arc_t));
    if (!na) return ORC_E_OOM;
    l->a = na;
    l->cap = nc;
  }
  l->a[l->n].v = v;
  l->a[l->n].w = w;
  l->a[l->n].mid = mid;
  l->n++;
  return ORC_OK;
}

static arc_t *adj_find(adj_t *l, uint32_t v) {
  for (uint32_t i = 0; i < l->n; i++)
    if (l->a[i].v == v) return &l->a[i];
  return NULL;
}

static void adj_remove(adj_t *l, uint32_t v) {
  for (uint32_t i = 0; i < l->n; i++)
    if (l->a[i].v == v) {
      l->a[i] = l->a[l->n - 1];
      l->n--;
      return;
    }
}

/* Open-addressing map from a (u, v) vertex pair to a uint32 value.  Insert
 * only; used for the memo `dist` and for the per-round shortcut set E+. */
typedef struct {
  uint64_t *key; /* (u << 32) | v, INF64 = empty */
  uint32_t *val;
  uint64_t cap, size;
} pairmap_t;

static uint64_t pm_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  return k;
}

static int pm_init(pairmap_t *m, uint64_t cap) {
  uint64_t c = 16;
  while (c < cap) c <<= 1;
  m->key = (uint64_t *)malloc(c * sizeof(uint64_t));
  m->val = (uint32_t *)malloc(c * sizeof(uint32_t));
  if (!m->key || !m->val) return ORC_E_OOM;
  memset(m->key, 0xff, c * sizeof(uint64_t));
  m->cap = c;
  m->size = 0;
  return ORC_OK;
}

static void pm_free(pairmap_t *m) {
  free(m->key);
  free(m->val);
  m->key = NULL;
  m->val = NULL;
  m->cap = m->size = 0;
}

static int pm_get(const pairmap_t *m, uint32_t u, uint32_t v, uint32_t *out) {
  uint64_t k = ((uint64_t)u << 32) | v;
  uint64_t i = pm_hash(k) & (m->cap - 1);
  while (m->key[i] != INF64) {
    if (m->key[i] == k) {
      *out = m->val[i];
      return 1;
    }
    i = (i + 1) & (m->cap - 1);
  }
  return 0;
}

static int pm_put_raw(pairmap_t *m, uint64_t k, uint32_t val) {
  uint64_t i = pm_hash(k) & (m->cap - 1);
  while (m->key[i] != INF64) {
    if (m->key[i] == k) {
      m->val[i] = val;
      return ORC_OK;
    }
    i = (i + 1) & (m->cap - 1);
  }
  m->key[i] = k;
  m->val[i] = val;
  m->size++;
  return ORC_OK;
}

static int pm_grow(pairmap_t *m) {
  pairmap_t nm;
  int rc = pm_init(&nm, m->cap * 2);
  if (rc) return rc;
  for (uint64_t i = 0; i < m->cap; i++)
    if (m->key[i] != INF64) pm_put_raw(&nm, m->key[i], m->val[i]);
  pm_free(m);
  *m = nm;
  return ORC_OK;
}

/* Insert or overwrite (u, v) -> val. */
static int pm_put(pairmap_t *m, uint32_t u, uint32_t v, uint32_t val) {
  if (2 * (m->size + 1) > m->cap) {
    int rc = pm_grow(m);
    if (rc) return rc;
  }
  return pm_put_raw(m, ((uint64_t)u << 32) | v, val);
}

/* Binary min-heap of (key, vertex), lazy deletion. */
typedef struct {
  uint64_t *k;
  uint32_t *v;
  size_t n, cap;
} heap_t;

static int heap_push(heap_t *h, uint64_t k, uint32_t v) {
  if (h->n == h->cap) {
    size_t nc = h->cap ? 2 * h->cap : 64;
    uint64_t *nk = (uint64_t *)realloc(h->k, nc * sizeof(uint64_t));
    if (!nk) return ORC_E_OOM;
    h->k = nk;
    uint32_t *nv = (uint32_t *)realloc(h->v, nc * sizeof(uint32_t));
    if (!nv) return ORC_E_OOM;
    h->v = nv;
    h->cap = nc;
  }
  size_t i = h->n++;
  while (i > 0) {
    size_t p = (i - 1) / 2;
    if (h->k[p] <= k) break;
    h->k[i] = h->k[p];
    h->v[i] = h->v[p];
    i = p;
  }
  h->k[i] = k;
  h->v[i] = v;
  return ORC_OK;
}

static void heap_pop(heap_t *h, uint64_t *k, uint32_t *v) {
  *k = h->k[0];
  *v = h->v[0];
  h->n--;
  if (h->n == 0) return;
  uint64_t lk = h->k[h->n];
  uint32_t lv = h->v[h->n];
  size_t i = 0;
  for (;;) {
    size_t c = 2 * i + 1;
    if (c >= h->n) break;
    if (c + 1 < h->n && h->k[c + 1] < h->k[c]) c++;
    if (h->k[c] >= lk) break;
    h->k[i] = h->k[c];
    h->v[i] = h->v[c];
    i = c;
  }
  h->k[i] = lk;
  h->v[i] = lv;
}

/* ------------------------------------------------------------------ */
/* state                                                               */
/* ------------------------------------------------------------------ */

typedef struct {
  uint32_t tail, head, w, mid;
} rec_t;

typedef struct {
  uint32_t w, lab, mid;
} eplus_t;

struct orc_state {
  uint32_t n;
  orc_params p;
  uint32_t *label;

  /* overlay graph G_O: out[v] holds arcs (v -> x), in[v] holds (x -> v) */
  adj_t *out, *in;
  uint8_t *alive;
  uint32_t n_alive;

  int32_t *P;      /* current score */
  int32_t *Pc;     /* score when contracted */
  uint32_t *level; /* round of contraction */
  uint32_t round;

  pairmap_t memo; /* dist: (s, v) -> shortest distance found by a WPS */

  /* sets carried between rounds: V_W (WPS sources), V_A (affected) */
  uint32_t *VW, nVW;
  uint32_t *VA, nVA;

  /* CH arcs */
  rec_t *up, *down;
  uint64_t nup, ndown, capup, capdown;

  /* scratch */
  uint64_t *dist, *dist2;    /* search distances, INF64 = unreached */
  uint32_t *touched, ntouched;
  uint32_t *stamp, stampv;   /* generic marker array */
  uint32_t *stamp2, stamp2v;
  uint32_t *list1, *list2;
  heap_t heap;

  orc_round_stats *stats;
  uint32_t nstats, capstats;

  /* learned priority: per-vertex feature state */
  float *mlp;        /* ORC_MLP_PARAMS weights, or NULL */
  uint32_t *cn;      /* contracted neighbours so far */
  uint32_t *depth;   /* hierarchy depth: max over contracted neighbours + 1 */
  uint32_t *ws;      /* vertices reached by this vertex's latest witness search */
  float *feat;       /* current features, 8 per vertex */
  float *rec;        /* features at contraction (params.record) */

  int finished;
  uint32_t *rank;
  /* CH in rank space for queries */
  uint64_t *upoff, *dnoff;
  uint32_t *uphead, *upw, *dntail, *dnw;
  uint64_t *qdf, *qdb;
  uint32_t *qtouch;
};

static uint32_t next_stamp(uint32_t *stamp, uint32_t *sv, uint32_t n) {
  if (++(*sv) == 0) {
    memset(stamp, 0, (size_t)n * sizeof(uint32_t));
    *sv = 1;
  }
  return *sv;
}

static int rec_push(rec_t **arr, uint64_t *cnt, uint64_t *cap, uint32_t tail,
                    uint32_t head, uint32_t w, uint32_t mid) {
  if (*cnt == *cap) {
    uint64_t nc = *cap ? 2 * *cap : 1024;
    rec_t *na = (rec_t *)realloc(*arr, nc * sizeof(rec_t));
    if (!na) return ORC_E_OOM;
    *arr = na;
    *cap = nc;
  }
  rec_t *r = &(*arr)[(*cnt)++];
  r->tail = tail;
  r->head = head;
  r->w = w;
  r->mid = mid;
  return ORC_OK;
}

void orc_free(orc_state *st) {
  if (!st) return;
  if (st->out)
    for (uint32_t v = 0; v < st->n; v++) free(st->out[v].a);
  if (st->in)
    for (uint32_t v = 0; v < st->n; v++) free(st->in[v].a);
  free(st->out);
  free(st->in);
  free(st->label);
  free(st->alive);
  free(st->P);
  free(st->Pc);
  free(st->level);
  pm_free(&st->memo);
  free(st->VW);
  free(st->VA);
  free(st->up);
  free(st->down);
  free(st->dist);
  free(st->dist2);
  free(st->touched);
  free(st->stamp);
  free(st->stamp2);
  free(st->list1);
  free(st->list2);
  free(st->heap.k);
  free(st->heap.v);
  free(st->stats);
  free(st->rank);
  free(st->upoff);
  free(st->dnoff);
  free(st->uphead);
  free(st->upw);
  free(st->dntail);
  free(st->dnw);
  free(st->qdf);
  free(st->qdb);
  free(st->qtouch);
  free(st->mlp);
  free(st->cn);
  free(st->depth);
  free(st->ws);
  free(st->feat);
  free(st->rec);
  free(st);
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return (x > y) - (x < y);
}

int orc_create(uint32_t n, uint64_t m, const uint64_t *off, const uint32_t *dst,
               const uint32_t *w, const uint32_t *labels, uint64_t seed,
               const orc_params *p, orc_state **out) {
  if (!out || !p || (n > 0 && !off) || (m > 0 && (!dst || !w))) return ORC_E_INVALID;
  if (n == 0xFFFFFFFFu) return ORC_E_INVALID;
  if (p->wps_mode > ORC_WPS_SETTLED) return ORC_E_INVALID;
  if (p->wps_mode == ORC_WPS_HOP && p->hop_limit < 1) return ORC_E_INVALID;
  if (p->wps_mode == ORC_WPS_SETTLED && p->settle_limit < 1) return ORC_E_INVALID;
  if (p->priority > ORC_PRIO_LEARNED || (p->priority == ORC_PRIO_LEARNED && !p->mlp))
    return ORC_E_INVALID;
  if (p->tiebreak > ORC_TIE_RAW_ID || (p->tiebreak == ORC_TIE_RAW_ID && labels))
    return ORC_E_INVALID;
  if (p->mlp_qbits > 24) return ORC_E_INVALID;
  if (n > 0 && (off[0] != 0 || off[n] != m)) return ORC_E_INVALID;
  for (uint32_t v = 0; v < n; v++)
    if (off[v] > off[v + 1]) return ORC_E_INVALID;
  for (uint64_t e = 0; e < m; e++)
    if (dst[e] >= n || w[e] == INF32) return ORC_E_INVALID;

  orc_state *st = (orc_state *)calloc(1, sizeof(orc_state));
  if (!st) return ORC_E_OOM;
  st->n = n;
  st->p = *p;
  if (!st->p.mlp_qbits) st->p.mlp_qbits = 16;
  size_t nn = n ? n : 1;
  st->label = (uint32_t *)malloc(nn * sizeof(uint32_t));
  st->out = (adj_t *)calloc(nn, sizeof(adj_t));
  st->in = (adj_t *)calloc(nn, sizeof(adj_t));
  st->alive = (uint8_t *)malloc(nn);
  st->P = (int32_t *)calloc(nn, sizeof(int32_t));
  st->Pc = (int32_t *)calloc(nn, sizeof(int32_t));
  st->level = (uint32_t *)malloc(nn * sizeof(uint32_t));
  st->VW = (uint32_t *)malloc(nn * sizeof(uint32_t));
  st->VA = (uint32_t *)malloc(nn * sizeof(uint32_t));
  st->dist = (uint64_t *)malloc(nn * sizeof(uint64_t));
  st->dist2 = (uint64_t *)malloc(nn * sizeof(uint64_t));
  st->touched = (uint32_t *)malloc(nn * sizeof(uint32_t));
  st->stamp = (uint32_t *)calloc(nn, sizeof(uint32_t));
  st->stamp2 = (uint32_t *)calloc(nn, sizeof(uint32_t));
  st->list1 = (uint32_t *)malloc(nn * sizeof(uint32_t));
  st->list2 = (uint32_t *)malloc(nn * sizeof(uint32_t));
  st->cn = (uint32_t *)calloc(nn, sizeof(uint32_t));
  st->depth = (uint32_t *)calloc(nn, sizeof(uint32_t));
  st->ws = (uint32_t *)calloc(nn, sizeof(uint32_t));
  st->feat = (float *)calloc(nn * 8, sizeof(float));
  if (p->record) st->rec = (float *)calloc(nn * 8, sizeof(float));
  if (p->priority == ORC_PRIO_LEARNED) {
    st->mlp = (float *)malloc(ORC_MLP_PARAMS * sizeof(float));
    if (st->mlp) memcpy(st->mlp, p->mlp, ORC_MLP_PARAMS * sizeof(float));
  }
  if (!st->label || !st->out || !st->in || !st->alive || !st->P || !st->Pc ||
      !st->level || !st->VW || !st->VA || !st->dist || !st->dist2 ||
      !st->touched || !st->stamp || !st->stamp2 || !st->list1 || !st->list2 || !st->cn ||
      !st->depth || !st->ws || !st->feat || (p->record && !st->rec) ||
      (p->priority == ORC_PRIO_LEARNED && !st->mlp)) {
    orc_free(st);
    return ORC_E_OOM;
  }
  for (uint32_t v = 0; v < n; v++) {
    st->label[v] = labels ? labels[v]
                   : (p->tiebreak == ORC_TIE_RAW_ID ? v : orc_default_label(v, seed));
    st->dist[v] = INF64;
    st->dist2[v] = INF64;
    st->level[v] = INF32;
    st->alive[v] = 1;
  }
  if (labels && n > 1) { /* labels must be distinct: a strict total order */
    uint32_t *tmp = (uint32_t *)malloc(nn * sizeof(uint32_t));
    if (!tmp) {
      orc_free(st);
      return ORC_E_OOM;
    }
    memcpy(tmp, labels, nn * sizeof(uint32_t));
    qsort(tmp, n, sizeof(uint32_t), cmp_u32);
    int dup = 0;
    for (uint32_t i = 1; i < n; i++)
      if (tmp[i] == tmp[i - 1]) dup = 1;
    free(tmp);
    if (dup) {
      orc_free(st);
      return ORC_E_INVALID;
    }
  }
  /* READING: input hygiene.  Self-loops carry no path information and are
   * dropped; of parallel arcs only the lightest is kept, as for duplicate
   * shortcuts ("only the one with the smallest weight should be kept"). */
  for (uint32_t u = 0; u < n; u++) {
    for (uint64_t e = off[u]; e < off[u + 1]; e++) {
      uint32_t v = dst[e];
      if (v == u) continue;
      arc_t *a = adj_find(&st->out[u], v);
      if (a) {
        if (w[e] < a->w) {
          a->w = w[e];
          adj_find(&st->in[v], u)->w = w[e];
        }
        continue;
      }
      if (adj_push(&st->out[u], v, w[e], NOMID) || adj_push(&st->in[v], u, w[e], NOMID)) {
        orc_free(st);
        return ORC_E_OOM;
      }
    }
  }
  st->n_alive = n;
  /* Alg. 3 initialisation: V_A = V_W = V. */
  for (uint32_t v = 0; v < n; v++) {
    st->VW[v] = v;
    st->VA[v] = v;
  }
  st->nVW = n;
  st->nVA = n;
  if (pm_init(&st->memo, 1024)) {
    orc_free(st);
    return ORC_E_OOM;
  }
  *out = st;
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 1: LocalSearch (Alg. 4)                                        */
/* ------------------------------------------------------------------ */

static void reset_touched(orc_state *st) {
  for (uint32_t i = 0; i < st->ntouched; i++) {
    st->dist[st->touched[i]] = INF64;
    st->dist2[st->touched[i]] = INF64;
  }
  st->ntouched = 0;
}

static void touch(orc_state *st, uint32_t v) {
  if (st->dist[v] == INF64 && st->dist2[v] == INF64) st->touched[st->ntouched++] = v;
}

/* Exact mode: Dijkstra from s on the current overlay, relaxing only
 * distances <= bound.  Every vertex within distance `bound` of s ends with
 * its exact overlay distance in st->dist. */
static int wps_exact(orc_state *st, uint32_t s, uint64_t bound, uint64_t *settled) {
  heap_t *h = &st->heap;
  h->n = 0;
  touch(st, s);
  st->dist[s] = 0;
  if (heap_push(h, 0, s)) return ORC_E_OOM;
  while (h->n) {
    uint64_t d;
    uint32_t x;
    heap_pop(h, &d, &x);
    if (d != st->dist[x]) continue; /* stale entry */
    (*settled)++;
    adj_t *l = &st->out[x];
    for (uint32_t i = 0; i < l->n; i++) {
      uint64_t nd = d + l->a[i].w;
      uint32_t y = l->a[i].v;
      if (nd <= bound && nd < st->dist[y]) {
        touch(st, y);
        st->dist[y] = nd;
        if (heap_push(h, nd, y)) return ORC_E_OOM;
      }
    }
  }
  return ORC_OK;
}

/* hop(H) mode: hop-synchronous Bellman-Ford.  After step k, dist[v] is the
 * minimum length over walks s ~> v of at most k arcs whose length is <=
 * bound (the READING for a hop- and distance-bounded search).  Step k reads
 * only values of step k-1 (dist) and writes dist2, then copies back. */
static int wps_hop(orc_state *st, uint32_t s, uint64_t bound, uint32_t H, uint64_t *settled) {
  uint32_t *front = st->list1, *next = st->list2;
  uint32_t nf = 0, nn;
  touch(st, s);
  st->dist[s] = 0;
  st->dist2[s] = 0;
  front[nf++] = s;
  for (uint32_t k = 1; k <= H && nf; k++) {
    uint32_t sv = next_stamp(st->stamp2, &st->stamp2v, st->n);
    nn = 0;
    for (uint32_t i = 0; i < nf; i++) {
      uint32_t x = front[i];
      adj_t *l = &st->out[x];
      for (uint32_t j = 0; j < l->n; j++) {
        uint64_t nd = st->dist[x] + l->a[j].w;
        uint32_t y = l->a[j].v;
        if (nd <= bound && nd < st->dist2[y]) {
          touch(st, y);
          st->dist2[y] = nd;
          if (st->stamp2[y] != sv) {
            st->stamp2[y] = sv;
            next[nn++] = y;
          }
        }
      }
    }
    for (uint32_t i = 0; i < nn; i++) st->dist[next[i]] = st->dist2[next[i]];
    uint32_t *t = front;
    front = next;
    next = t;
    nf = nn;
  }
  *settled += st->ntouched;
  return ORC_OK;
}

/* settled(theta) mode, the paper's literal bound: Dijkstra popping in
 * (distance, label) order, the source counting as the first settled
 * vertex; stops after theta pops or once every target is settled.  Only
 * settled vertices keep a distance (dist2 holds settled values). */
static int wps_settled(orc_state *st, uint32_t s, uint64_t bound, uint32_t theta,
                       uint32_t ntargets, uint32_t tstamp, uint64_t *settled) {
  heap_t *h = &st->heap;
  h->n = 0;
  touch(st, s);
  st->dist[s] = 0;
  if (heap_push(h, ((uint64_t)0 << 32) | st->label[s], s)) return ORC_E_OOM;
  uint32_t pops = 0, tdone = 0;
  while (h->n && pops < theta && tdone < ntargets) {
    uint64_t key;
    uint32_t x;
    heap_pop(h, &key, &x);
    uint64_t d = key >> 32;
    if (st->dist2[x] != INF64 || d != st->dist[x]) continue;
    st->dist2[x] = d;
    pops++;
    if (st->stamp[x] == tstamp) tdone++;
    adj_t *l = &st->out[x];
    for (uint32_t i = 0; i < l->n; i++) {
      uint64_t nd = d + l->a[i].w;
      uint32_t y = l->a[i].v;
      if (nd <= bound && nd < st->dist[y] && st->dist2[y] == INF64) {
        touch(st, y);
        st->dist[y] = nd;
        if (heap_push(h, (nd << 32) | st->label[y], y)) return ORC_E_OOM;
      }
    }
  }
  *settled += pops;
  return ORC_OK;
}

/* Alg. 4.  For each source s in V_W, the target set V_n collects the
 * out-neighbours v of every affected out-neighbour u of s, except s itself
 * and pairs already in the memo.  One search from s then settles them all
 * and the distances go to the memo.  READING: the search radius is D_s, the
 * largest two-arc length w(s,u)+w(u,v) over the collected pairs; every
 * target's distance is at most its own two-arc length, so in exact mode
 * the radius never changes a value.  READING: a target the search leaves
 * unsettled gets no memo entry (absent means "no witness", so a shortcut is
 * generated).  READING: the memo is never overwritten or cleared. */
static int local_search(orc_state *st, orc_round_stats *rs) {
  uint8_t *isA = (uint8_t *)calloc(st->n ? st->n : 1, 1);
  if (!isA) return ORC_E_OOM;
  for (uint32_t i = 0; i < st->nVA; i++) isA[st->VA[i]] = 1;

  uint32_t *targets = (uint32_t *)malloc((size_t)(st->n ? st->n : 1) * sizeof(uint32_t));
  if (!targets) {
    free(isA);
    return ORC_E_OOM;
  }
  int rc = ORC_OK;
  for (uint32_t i = 0; i < st->nVW && rc == ORC_OK; i++) {
    uint32_t s = st->VW[i];
    uint32_t tst = next_stamp(st->stamp, &st->stampv, st->n);
    uint32_t nt = 0;
    uint64_t D = 0;
    adj_t *ls = &st->out[s];
    for (uint32_t a = 0; a < ls->n; a++) {
      uint32_t u = ls->a[a].v;
      if (!isA[u]) continue;
      adj_t *lu = &st->out[u];
      for (uint32_t b = 0; b < lu->n; b++) {
        uint32_t v = lu->a[b].v;
        uint32_t dummy;
        if (v == s || pm_get(&st->memo, s, v, &dummy)) continue;
        uint64_t via = (uint64_t)ls->a[a].w + lu->a[b].w;
        if (via > D) D = via;
        if (st->stamp[v] != tst) {
          st->stamp[v] = tst;
          targets[nt++] = v;
        }
      }
    }
    if (nt == 0) continue;
    if (D > MAXW) {
      rc = ORC_E_OVERFLOW;
      break;
    }
    rs->n_searched++;
    rs->n_targets += nt;
    uint64_t settled = 0;
    if (st->p.wps_mode == ORC_WPS_EXACT) {
      rc = wps_exact(st, s, D, &settled);
    } else if (st->p.wps_mode == ORC_WPS_HOP) {
      rc = wps_hop(st, s, D, st->p.hop_limit, &settled);
    } else {
      rc = wps_settled(st, s, D, st->p.settle_limit, nt, tst, &settled);
    }
    rs->n_settled += settled;
    st->ws[s] = (uint32_t)(settled > 0xFFFFFFFFull ? 0xFFFFFFFFull : settled);
    for (uint32_t k = 0; k < nt && rc == ORC_OK; k++) {
      uint32_t v = targets[k];
      uint64_t d = (st->p.wps_mode == ORC_WPS_SETTLED) ? st->dist2[v] : st->dist[v];
      if (d <= MAXW) rc = pm_put(&st->memo, s, v, (uint32_t)d);
    }
    reset_touched(st);
  }
  free(targets);
  free(isA);
  return rc;
}

/* Pruning at the end of Alg. 4: delete overlay arc (s, v) of a source s in
 * V_W when its weight exceeds the memoized distance.  READING: applied after
 * all searches of the round, with any memo entry (of this or an earlier
 * round) as the justification. */
static void prune(orc_state *st, orc_round_stats *rs) {
  for (uint32_t i = 0; i < st->nVW; i++) {
    uint32_t s = st->VW[i];
    adj_t *l = &st->out[s];
    uint32_t a = 0;
    while (a < l->n) {
      uint32_t d, v = l->a[a].v;
      if (pm_get(&st->memo, s, v, &d) && l->a[a].w > d) {
        adj_remove(&st->in[v], s);
        l->a[a] = l->a[l->n - 1];
        l->n--;
        rs->n_pruned++;
      } else {
        a++;
      }
    }
  }
}

/* ------------------------------------------------------------------ */
/* Step 2: Score (Alg. 5)                                              */
/* ------------------------------------------------------------------ */

/* |N(u)| with N(u) = N_in(u) union N_out(u) as a set of vertices. */
static uint32_t neighbour_count(orc_state *st, uint32_t u) {
  uint32_t sv = next_stamp(st->stamp, &st->stampv, st->n);
  uint32_t c = 0;
  for (uint32_t i = 0; i < st->out[u].n; i++) {
    st->stamp[st->out[u].a[i].v] = sv;
    c++;
  }
  for (uint32_t i = 0; i < st->in[u].n; i++)
    if (st->stamp[st->in[u].a[i].v] != sv) c++;
  return c;
}

/* ---- learned priority ------------------------------------------------
 * READING (the learned priority is not in the paper): the priority is an MLP
 * over eight features of the vertex, each squashed to [0, 1) (or (-1, 1))
 * by x / (x + c):
 *   0 edge difference (signed: x / (|x| + 8))   1 contracted neighbours
 *   2 live in-degree   3 live out-degree          4 hierarchy depth
 *   5 vertices reached by the vertex's latest witness search (c = 64)
 *   6 |N(u)|           7 pairs that need a shortcut
 * GELU uses tanh through its [7/6] Pade approximant (Lambert's continued
 * fraction), set to +-1 for |t| >= 4.97.  Everything is single precision,
 * evaluated left to right as written, with no fused multiply-add, so any
 * IEEE implementation gives the same bits.  The priority is the output
 * times 2^16, rounded to nearest even and saturated to int32. */
static float tanh_pade(float t) {
  if (t >= 4.97f) return 1.0f;
  if (t <= -4.97f) return -1.0f;
  float t2 = t * t;
  float num = t * (135135.0f + t2 * (17325.0f + t2 * (378.0f + t2)));
  float den = 135135.0f + t2 * (62370.0f + t2 * (3150.0f + t2 * 28.0f));
  float r = num / den;
  if (r > 1.0f) r = 1.0f;
  if (r < -1.0f) r = -1.0f;
  return r;
}

float orc_gelu(float x) {
  float x3 = (x * x) * x;
  float inner = x + 0.044715f * x3;
  float t = 0.7978845608f * inner;
  return (0.5f * x) * (1.0f + tanh_pade(t));
}

int32_t orc_mlp_priority(const float *w, const float *x, float *y_out) {
  return orc_mlp_priority_q(w, x, 16, y_out);
}

int32_t orc_mlp_priority_q(const float *w, const float *x, uint32_t qbits, float *y_out) {
  const float *W1 = w, *b1 = w + 512, *W2 = w + 576, *b2 = w + 4672, *W3 = w + 4736,
              *b3 = w + 4800;
  float a1[64], a2[64];
  for (int j = 0; j < 64; j++) {
    float h = b1[j];
    for (int i = 0; i < 8; i++) h = h + W1[j * 8 + i] * x[i];
    a1[j] = orc_gelu(h);
  }
  for (int j = 0; j < 64; j++) {
    float h = b2[j];
    for (int i = 0; i < 64; i++) h = h + W2[j * 64 + i] * a1[i];
    a2[j] = orc_gelu(h);
  }
  float y = b3[0];
  for (int i = 0; i < 64; i++) y = y + W3[i] * a2[i];
  if (y_out) *y_out = y;
  float z = y * (float)(1u << qbits); /* a power of two: exact */
  if (!(z < 2147483648.0f)) return INT32_MAX; /* also NaN */
  if (z < -2147483648.0f) return INT32_MIN;
  return (int32_t)rintf(z);
}

static float squash(uint64_t x, float c) { return (float)x / ((float)x + c); }

static void vertex_features(const orc_state *st, uint32_t u, int32_t ed, uint32_t din,
                            uint32_t dout, uint32_t nb, uint32_t pairs, float *f) {
  uint64_t mag = ed < 0 ? (uint64_t)(-(int64_t)ed) : (uint64_t)ed;
  f[0] = (float)ed / ((float)mag + 8.0f);
  f[1] = squash(st->cn[u], 8.0f);
  f[2] = squash(din, 8.0f);
  f[3] = squash(dout, 8.0f);
  f[4] = squash(st->depth[u], 8.0f);
  f[5] = squash(st->ws[u], 64.0f);
  f[6] = squash(nb, 8.0f);
  f[7] = squash(pairs, 8.0f);
}

/* Alg. 5: P[u] = -|N(u)| + number of pairs (v1, v2) in N_in(u) x N_out(u)
 * whose path through u is no longer than the memoized distance, or whose
 * distance is not memoized.  READING: pairs with v1 == v2 are skipped (a
 * shortcut would be a self-loop); the test is "<=" (the text's "equal to or
 * smaller than"), identical to "=" when the memo holds exact distances. */
static void score(orc_state *st, orc_round_stats *rs) {
  for (uint32_t i = 0; i < st->nVA; i++) {
    uint32_t u = st->VA[i];
    uint32_t nb = neighbour_count(st, u);
    int64_t p = -(int64_t)nb;
    uint32_t pairs = 0;
    adj_t *li = &st->in[u], *lo = &st->out[u];
    for (uint32_t a = 0; a < li->n; a++) {
      for (uint32_t b = 0; b < lo->n; b++) {
        uint32_t v1 = li->a[a].v, v2 = lo->a[b].v, d;
        if (v1 == v2) continue;
        uint64_t via = (uint64_t)li->a[a].w + lo->a[b].w;
        if (!pm_get(&st->memo, v1, v2, &d)) {
          rs->n_absent++;
          p++;
          pairs++;
        } else if (via <= d) {
          p++;
          pairs++;
        }
      }
    }
    /* READING: the score combines edge difference, contracted neighbours
     * and hierarchy depth (the paper names the terms, not their weights)
     * with integer weights k_ed, k_cn, k_depth; 1, 0, 0 is Alg. 5's edge
     * difference. */
    int64_t comb = (int64_t)st->p.k_ed * p + (int64_t)st->p.k_cn * st->cn[u] +
                   (int64_t)st->p.k_depth * st->depth[u];
    /* READING: the score is an int32; a count outside that range (degrees
     * above ~46k) saturates. */
    if (p > INT32_MAX) p = INT32_MAX;
    if (p < INT32_MIN) p = INT32_MIN;
    if (comb > INT32_MAX) comb = INT32_MAX;
    if (comb < INT32_MIN) comb = INT32_MIN;
    float *f = &st->feat[(size_t)u * 8];
    vertex_features(st, u, (int32_t)p, li->n, lo->n, nb, pairs, f);
    st->P[u] = st->mlp ? orc_mlp_priority_q(st->mlp, f, st->p.mlp_qbits, NULL) : (int32_t)comb;
  }
}

/* ------------------------------------------------------------------ */
/* Step 3: Select (Alg. 6)                                             */
/* ------------------------------------------------------------------ */

/* Strict order on (score, label); labels are distinct. */
static int key_less(const orc_state *st, uint32_t a, uint32_t b) {
  if (st->P[a] != st->P[b]) return st->P[a] < st->P[b];
  return st->label[a] < st->label[b];
}

/* Alg. 6: u is selected when its (score, label) is smaller than that of
 * every neighbour in N_in(u) union N_out(u).  A vertex with no neighbour is
 * selected.  Returns the selected set in list1. */
static uint32_t select_set(orc_state *st, uint32_t *sel) {
  uint32_t ns = 0;
  for (uint32_t u = 0; u < st->n; u++) {
    if (!st->alive[u]) continue;
    int ok = 1;
    for (uint32_t i = 0; i < st->out[u].n && ok; i++)
      if (!key_less(st, u, st->out[u].a[i].v)) ok = 0;
    for (uint32_t i = 0; i < st->in[u].n && ok; i++)
      if (!key_less(st, u, st->in[u].a[i].v)) ok = 0;
    if (ok) sel[ns++] = u;
  }
  return ns;
}

/* ------------------------------------------------------------------ */
/* Step 4: Contract (Alg. 7) and combination of E+ with the overlay    */
/* ------------------------------------------------------------------ */

static int contract(orc_state *st, const uint32_t *VF, uint32_t nF, orc_round_stats *rs) {
  int rc = ORC_OK;
  uint32_t r = st->round;
  /* E+ : (v1, v2) -> index into a record array of (w, label(mid), mid). */
  pairmap_t eidx;
  if (pm_init(&eidx, 64)) return ORC_E_OOM;
  eplus_t *erec = NULL;
  uint64_t ne = 0, ecap = 0;
  uint8_t *inS = (uint8_t *)calloc(st->n ? st->n : 1, 1);  /* V_S */
  uint8_t *newA = (uint8_t *)calloc(st->n ? st->n : 1, 1); /* V_A of next round */
  if (!inS || !newA) {
    rc = ORC_E_OOM;
    goto done;
  }

  for (uint32_t f = 0; f < nF && rc == ORC_OK; f++) {
    uint32_t u = VF[f];
    adj_t *li = &st->in[u], *lo = &st->out[u];
    st->level[u] = r;
    st->Pc[u] = st->P[u];
    if (st->rec) memcpy(&st->rec[(size_t)u * 8], &st->feat[(size_t)u * 8], 8 * sizeof(float));
    /* feature state of the neighbours: one more contracted neighbour each,
     * depth at least depth(u) + 1 */
    {
      uint32_t sv = next_stamp(st->stamp2, &st->stamp2v, st->n);
      for (uint32_t b = 0; b < lo->n; b++) {
        uint32_t v = lo->a[b].v;
        if (st->stamp2[v] == sv) continue;
        st->stamp2[v] = sv;
        st->cn[v]++;
        if (st->depth[v] < st->depth[u] + 1) st->depth[v] = st->depth[u] + 1;
      }
      for (uint32_t a = 0; a < li->n; a++) {
        uint32_t v = li->a[a].v;
        if (st->stamp2[v] == sv) continue;
        st->stamp2[v] = sv;
        st->cn[v]++;
        if (st->depth[v] < st->depth[u] + 1) st->depth[v] = st->depth[u] + 1;
      }
    }
    /* incident arcs move to the CH: out-arcs to the upward set, in-arcs to
     * the downward set */
    for (uint32_t b = 0; b < lo->n && rc == ORC_OK; b++)
      rc = rec_push(&st->up, &st->nup, &st->capup, u, lo->a[b].v, lo->a[b].w, lo->a[b].mid);
    for (uint32_t a = 0; a < li->n && rc == ORC_OK; a++)
      rc = rec_push(&st->down, &st->ndown, &st->capdown, li->a[a].v, u, li->a[a].w,
                    li->a[a].mid);
    /* V_A of the next round: N(V_F) on the overlay before contraction */
    for (uint32_t b = 0; b < lo->n; b++) newA[lo->a[b].v] = 1;
    for (uint32_t a = 0; a < li->n; a++) newA[li->a[a].v] = 1;
    /* shortcuts: same test as the score */
    for (uint32_t a = 0; a < li->n && rc == ORC_OK; a++) {
      for (uint32_t b = 0; b < lo->n && rc == ORC_OK; b++) {
        uint32_t v1 = li->a[a].v, v2 = lo->a[b].v, d;
        if (v1 == v2) continue;
        uint64_t via = (uint64_t)li->a[a].w + lo->a[b].w;
        int present = pm_get(&st->memo, v1, v2, &d);
        if (!present) rs->n_absent++;
        if (present && via > d) continue;
        if (via > MAXW) {
          rc = ORC_E_OVERFLOW;
          break;
        }
        rs->n_pairs_emitted++;
        inS[v1] = 1;
        /* READING: a duplicate (v1, v2) keeps the smallest (weight,
         * label of the middle vertex). */
        uint32_t idx;
        if (pm_get(&eidx, v1, v2, &idx)) {
          eplus_t *e = &erec[idx];
          if (via < e->w || (via == e->w && st->label[u] < e->lab)) {
            e->w = (uint32_t)via;
            e->lab = st->label[u];
            e->mid = u;
          }
        } else {
          if (ne == ecap) {
            uint64_t nc = ecap ? 2 * ecap : 256;
            eplus_t *na = (eplus_t *)realloc(erec, nc * sizeof(eplus_t));
            if (!na) {
              rc = ORC_E_OOM;
              break;
            }
            erec = na;
            ecap = nc;
          }
          erec[ne].w = (uint32_t)via;
          erec[ne].lab = st->label[u];
          erec[ne].mid = u;
          rc = pm_put(&eidx, v1, v2, (uint32_t)ne);
          ne++;
        }
      }
    }
  }
  if (rc) goto done;
  rs->n_shortcuts = ne;

  /* remove V_F and every incident arc from the overlay */
  for (uint32_t f = 0; f < nF; f++) {
    uint32_t u = VF[f];
    for (uint32_t b = 0; b < st->out[u].n; b++) adj_remove(&st->in[st->out[u].a[b].v], u);
    for (uint32_t a = 0; a < st->in[u].n; a++) adj_remove(&st->out[st->in[u].a[a].v], u);
    st->out[u].n = 0;
    st->in[u].n = 0;
    st->alive[u] = 0;
    st->n_alive--;
    newA[u] = 0;
  }
  /* combine E+ with the overlay: a new pair is inserted; an existing arc
   * takes the shortcut only if the shortcut is strictly lighter (READING:
   * on equal weight the existing arc and its middle vertex stay). */
  for (uint64_t i = 0; i < eidx.cap && rc == ORC_OK; i++) {
    if (eidx.key[i] == INF64) continue;
    uint32_t v1 = (uint32_t)(eidx.key[i] >> 32), v2 = (uint32_t)eidx.key[i];
    eplus_t *e = &erec[eidx.val[i]];
    arc_t *a = adj_find(&st->out[v1], v2);
    if (!a) {
      rc = adj_push(&st->out[v1], v2, e->w, e->mid);
      if (!rc) rc = adj_push(&st->in[v2], v1, e->w, e->mid);
    } else if (e->w < a->w) {
      arc_t *b = adj_find(&st->in[v2], v1);
      a->w = b->w = e->w;
      a->mid = b->mid = e->mid;
    }
  }
  if (rc) goto done;

  /* V_W of the next round: V_S together with N_in(V_S), on the combined
   * overlay. */
  {
    uint32_t sv = next_stamp(st->stamp, &st->stampv, st->n);
    uint32_t nw = 0;
    for (uint32_t v = 0; v < st->n; v++) {
      if (!inS[v]) continue;
      if (st->stamp[v] != sv) {
        st->stamp[v] = sv;
        st->VW[nw++] = v;
      }
      for (uint32_t a = 0; a < st->in[v].n; a++) {
        uint32_t x = st->in[v].a[a].v;
        if (st->stamp[x] != sv) {
          st->stamp[x] = sv;
          st->VW[nw++] = x;
        }
      }
    }
    st->nVW = nw;
    uint32_t na = 0;
    for (uint32_t v = 0; v < st->n; v++)
      if (newA[v]) st->VA[na++] = v;
    st->nVA = na;
  }
done:
  pm_free(&eidx);
  free(erec);
  free(inS);
  free(newA);
  return rc;
}

/* ------------------------------------------------------------------ */
/* main loop (Alg. 3)                                                  */
/* ------------------------------------------------------------------ */

static uint64_t overlay_arc_count(const orc_state *st) {
  uint64_t c = 0;
  for (uint32_t v = 0; v < st->n; v++) c += st->out[v].n;
  return c;
}

int orc_round(orc_state *st) {
  if (!st || st->finished) return ORC_E_STATE;
  if (st->n_alive == 0) return 0;
  if (st->p.max_rounds && st->round >= st->p.max_rounds) return ORC_E_LIMIT;
  orc_round_stats rs;
  memset(&rs, 0, sizeof(rs));
  rs.alive_before = st->n_alive;
  rs.n_sources = st->nVW;
  rs.n_affected = st->nVA;

  int rc = local_search(st, &rs);
  if (rc) return rc;
  prune(st, &rs);
  score(st, &rs);
  uint32_t nF = select_set(st, st->list1);
  rs.n_selected = nF;
  uint32_t *VF = (uint32_t *)malloc((size_t)(nF ? nF : 1) * sizeof(uint32_t));
  if (!VF) return ORC_E_OOM;
  memcpy(VF, st->list1, (size_t)nF * sizeof(uint32_t));
  rc = contract(st, VF, nF, &rs);
  free(VF);
  if (rc) return rc;
  rs.overlay_arcs = overlay_arc_count(st);
  if (st->nstats == st->capstats) {
    uint32_t nc = st->capstats ? 2 * st->capstats : 64;
    orc_round_stats *ns = (orc_round_stats *)realloc(st->stats, nc * sizeof(orc_round_stats));
    if (!ns) return ORC_E_OOM;
    st->stats = ns;
    st->capstats = nc;
  }
  st->stats[st->nstats++] = rs;
  st->round++;
  return st->n_alive ? 1 : 0;
}

/* ------------------------------------------------------------------ */
/* Postprocessing                                                      */
/* ------------------------------------------------------------------ */

typedef struct {
  uint32_t level;
  int32_t pc;
  uint32_t label, v;
} rkey_t;

static int cmp_rkey(const void *pa, const void *pb) {
  const rkey_t *a = (const rkey_t *)pa, *b = (const rkey_t *)pb;
  if (a->level != b->level) return a->level < b->level ? -1 : 1;
  if (a->pc != b->pc) return a->pc < b->pc ? -1 : 1;
  if (a->label != b->label) return a->label < b->label ? -1 : 1;
  return 0;
}

/* Vertices are ordered by level (round of contraction), then by score from
 * low to high.  READING: the score is the one the vertex had when it was
 * selected; remaining ties go to the label. */
int orc_finish(orc_state *st) {
  if (!st) return ORC_E_STATE;
  if (st->finished) return ORC_OK;
  if (st->n_alive) return ORC_E_STATE;
  uint32_t n = st->n;
  size_t nn = n ? n : 1;
  rkey_t *k = (rkey_t *)malloc(nn * sizeof(rkey_t));
  st->rank = (uint32_t *)malloc(nn * sizeof(uint32_t));
  st->upoff = (uint64_t *)calloc(nn + 1, sizeof(uint64_t));
  st->dnoff = (uint64_t *)calloc(nn + 1, sizeof(uint64_t));
  st->uphead = (uint32_t *)malloc((st->nup ? st->nup : 1) * sizeof(uint32_t));
  st->upw = (uint32_t *)malloc((st->nup ? st->nup : 1) * sizeof(uint32_t));
  st->dntail = (uint32_t *)malloc((st->ndown ? st->ndown : 1) * sizeof(uint32_t));
  st->dnw = (uint32_t *)malloc((st->ndown ? st->ndown : 1) * sizeof(uint32_t));
  st->qdf = (uint64_t *)malloc(nn * sizeof(uint64_t));
  st->qdb = (uint64_t *)malloc(nn * sizeof(uint64_t));
  st->qtouch = (uint32_t *)malloc(2 * nn * sizeof(uint32_t));
  if (!k || !st->rank || !st->upoff || !st->dnoff || !st->uphead || !st->upw ||
      !st->dntail || !st->dnw || !st->qdf || !st->qdb || !st->qtouch) {
    free(k);
    return ORC_E_OOM;
  }
  for (uint32_t v = 0; v < n; v++) {
    k[v].level = st->level[v];
    k[v].pc = st->Pc[v];
    k[v].label = st->label[v];
    k[v].v = v;
  }
  qsort(k, n, sizeof(rkey_t), cmp_rkey);
  for (uint32_t i = 0; i < n; i++) st->rank[k[i].v] = i;
  free(k);
  /* upward graph in rank space: arc rank(u) -> rank(v) stored at rank(u);
   * downward graph: arc rank(v) -> rank(u) stored at rank(u), so that the
   * backward search from t walks it from head to tail. */
  for (uint64_t i = 0; i < st->nup; i++) st->upoff[st->rank[st->up[i].tail] + 1]++;
  for (uint64_t i = 0; i < st->ndown; i++) st->dnoff[st->rank[st->down[i].head] + 1]++;
  for (uint32_t v = 0; v < n; v++) {
    st->upoff[v + 1] += st->upoff[v];
    st->dnoff[v + 1] += st->dnoff[v];
  }
  uint64_t *pu = (uint64_t *)malloc(nn * sizeof(uint64_t));
  uint64_t *pd = (uint64_t *)malloc(nn * sizeof(uint64_t));
  if (!pu || !pd) {
    free(pu);
    free(pd);
    return ORC_E_OOM;
  }
  memcpy(pu, st->upoff, nn * sizeof(uint64_t));
  memcpy(pd, st->dnoff, nn * sizeof(uint64_t));
  for (uint64_t i = 0; i < st->nup; i++) {
    uint64_t at = pu[st->rank[st->up[i].tail]]++;
    st->uphead[at] = st->rank[st->up[i].head];
    st->upw[at] = st->up[i].w;
  }
  for (uint64_t i = 0; i < st->ndown; i++) {
    uint64_t at = pd[st->rank[st->down[i].head]]++;
    st->dntail[at] = st->rank[st->down[i].tail];
    st->dnw[at] = st->down[i].w;
  }
  free(pu);
  free(pd);
  for (uint32_t v = 0; v < n; v++) st->qdf[v] = st->qdb[v] = INF64;
  st->finished = 1;
  return ORC_OK;
}

int orc_load(uint32_t n, const uint32_t *rank, uint64_t nup, const uint32_t *up_tail,
             const uint32_t *up_head, const uint32_t *up_w, uint64_t ndown,
             const uint32_t *dn_tail, const uint32_t *dn_head, const uint32_t *dn_w,
             orc_state **out) {
  if (!out || (n && !rank)) return ORC_E_INVALID;
  orc_state *st = (orc_state *)calloc(1, sizeof(orc_state));
  if (!st) return ORC_E_OOM;
  st->n = n;
  size_t nn = n ? n : 1;
  st->rank = (uint32_t *)malloc(nn * sizeof(uint32_t));
  st->upoff = (uint64_t *)calloc(nn + 1, sizeof(uint64_t));
  st->dnoff = (uint64_t *)calloc(nn + 1, sizeof(uint64_t));
  st->uphead = (uint32_t *)malloc((nup ? nup : 1) * sizeof(uint32_t));
  st->upw = (uint32_t *)malloc((nup ? nup : 1) * sizeof(uint32_t));
  st->dntail = (uint32_t *)malloc((ndown ? ndown : 1) * sizeof(uint32_t));
  st->dnw = (uint32_t *)malloc((ndown ? ndown : 1) * sizeof(uint32_t));
  st->qdf = (uint64_t *)malloc(nn * sizeof(uint64_t));
  st->qdb = (uint64_t *)malloc(nn * sizeof(uint64_t));
  st->qtouch = (uint32_t *)malloc(2 * nn * sizeof(uint32_t));
  uint64_t *pu = (uint64_t *)malloc(nn * sizeof(uint64_t));
  uint64_t *pd = (uint64_t *)malloc(nn * sizeof(uint64_t));
  if (!st->rank || !st->upoff || !st->dnoff || !st->uphead || !st->upw || !st->dntail ||
      !st->dnw || !st->qdf || !st->qdb || !st->qtouch || !pu || !pd) {
    free(pu);
    free(pd);
    orc_free(st);
    return ORC_E_OOM;
  }
  memcpy(st->rank, rank, (size_t)n * sizeof(uint32_t));
  for (uint64_t i = 0; i < nup; i++) st->upoff[st->rank[up_tail[i]] + 1]++;
  for (uint64_t i = 0; i < ndown; i++) st->dnoff[st->rank[dn_head[i]] + 1]++;
  for (uint32_t v = 0; v < n; v++) {
    st->upoff[v + 1] += st->upoff[v];
    st->dnoff[v + 1] += st->dnoff[v];
  }
  memcpy(pu, st->upoff, nn * sizeof(uint64_t));
  memcpy(pd, st->dnoff, nn * sizeof(uint64_t));
  for (uint64_t i = 0; i < nup; i++) {
    uint64_t at = pu[st->rank[up_tail[i]]]++;
    st->uphead[at] = st->rank[up_head[i]];
    st->upw[at] = up_w[i];
  }
  for (uint64_t i = 0; i < ndown; i++) {
    uint64_t at = pd[st->rank[dn_head[i]]]++;
    st->dntail[at] = st->rank[dn_tail[i]];
    st->dnw[at] = dn_w[i];
  }
  free(pu);
  free(pd);
  for (uint32_t v = 0; v < n; v++) st->qdf[v] = st->qdb[v] = INF64;
  st->finished = 1;
  *out = st;
  return ORC_OK;
}

int orc_run(orc_state *st) {
  int rc;
  while ((rc = orc_round(st)) == 1) {
  }
  if (rc < 0) return rc;
  return orc_finish(st);
}

/* ------------------------------------------------------------------ */
/* Query                                                               */
/* ------------------------------------------------------------------ */

/* Bidirectional search: forward from s over upward arcs, backward from t
 * over downward arcs; mu = min over met vertices of d_s(v) + d_t(v).
 * READING (the stopping sentence is garbled): a direction stops once its
 * queue minimum is >= mu; the query ends when both have stopped.  The side
 * with the smaller queue minimum is expanded (forward on a tie); queue keys
 * are (distance, rank).  "Settled" counts the pops of both sides. */
uint64_t orc_query(orc_state *st, uint32_t s, uint32_t t, uint64_t *settled) {
  if (!st || !st->finished || s >= st->n || t >= st->n) return INF64;
  uint32_t rs_ = st->rank[s], rt = st->rank[t];
  uint32_t nt = 0;
  uint64_t mu = INF64, pops = 0;
  st->qdf[rs_] = 0;
  st->qtouch[nt++] = rs_;
  if (rt != rs_) st->qtouch[nt++] = rt;
  st->qdb[rt] = 0;
  /* Query distances are uint64, so the queue holds (distance, rank) pairs
   * compared lexicographically. */
  typedef struct {
    uint64_t d;
    uint32_t v;
  } qe_t;
  qe_t *qf = NULL, *qb = NULL;
  size_t nf = 0, nb = 0, cf = 0, cb = 0;
#define QLESS(x, y) ((x).d < (y).d || ((x).d == (y).d && (x).v < (y).v))
#define QPUSH(Q, N, C, D, V)                                   \
  do {                                                         \
    if ((N) == (C)) {                                          \
      size_t nc_ = (C) ? 2 * (C) : 64;                         \
      qe_t *nq_ = (qe_t *)realloc((Q), nc_ * sizeof(qe_t));    \
      if (!nq_) goto oom;                                      \
      (Q) = nq_;                                               \
      (C) = nc_;                                               \
    }                                                          \
    qe_t e_ = {(D), (V)};                                      \
    size_t i_ = (N)++;                                         \
    while (i_ > 0) {                                           \
      size_t p_ = (i_ - 1) / 2;                                \
      if (!QLESS(e_, (Q)[p_])) break;                          \
      (Q)[i_] = (Q)[p_];                                       \
      i_ = p_;                                                 \
    }                                                          \
    (Q)[i_] = e_;                                              \
  } while (0)
#define QPOP(Q, N, OUT)                                        \
  do {                                                         \
    (OUT) = (Q)[0];                                            \
    (N)--;                                                     \
    if (N) {                                                   \
      qe_t l_ = (Q)[N];                                        \
      size_t i_ = 0;                                           \
      for (;;) {                                               \
        size_t c_ = 2 * i_ + 1;                                \
        if (c_ >= (N)) break;                                  \
        if (c_ + 1 < (N) && QLESS((Q)[c_ + 1], (Q)[c_])) c_++; \
        if (!QLESS((Q)[c_], l_)) break;                        \
        (Q)[i_] = (Q)[c_];                                     \
        i_ = c_;                                               \
      }                                                        \
      (Q)[i_] = l_;                                            \
    }                                                          \
  } while (0)
  QPUSH(qf, nf, cf, (uint64_t)0, rs_);
  QPUSH(qb, nb, cb, (uint64_t)0, rt);
  for (;;) {
    /* drop stale heads */
    while (nf && qf[0].d != st->qdf[qf[0].v]) {
      qe_t stale;
      QPOP(qf, nf, stale);
      (void)stale;
    }
    while (nb && qb[0].d != st->qdb[qb[0].v]) {
      qe_t stale;
      QPOP(qb, nb, stale);
      (void)stale;
    }
    int fa = nf && qf[0].d < mu, ba = nb && qb[0].d < mu;
    if (!fa && !ba) break;
    int fwd = fa && (!ba || qf[0].d <= qb[0].d);
    qe_t x;
    if (fwd) {
      QPOP(qf, nf, x); /* relaxation only pushes strict improvements, so
                          a (d, v) pair is popped at most once */
      pops++;
      if (st->qdb[x.v] != INF64 && x.d + st->qdb[x.v] < mu) mu = x.d + st->qdb[x.v];
      for (uint64_t e = st->upoff[x.v]; e < st->upoff[x.v + 1]; e++) {
        uint32_t y = st->uphead[e];
        uint64_t nd = x.d + st->upw[e];
        if (nd < st->qdf[y]) {
          if (st->qdf[y] == INF64 && st->qdb[y] == INF64) st->qtouch[nt++] = y;
          st->qdf[y] = nd;
          QPUSH(qf, nf, cf, nd, y);
        }
      }
    } else {
      QPOP(qb, nb, x);
      pops++;
      if (st->qdf[x.v] != INF64 && x.d + st->qdf[x.v] < mu) mu = x.d + st->qdf[x.v];
      for (uint64_t e = st->dnoff[x.v]; e < st->dnoff[x.v + 1]; e++) {
        uint32_t y = st->dntail[e];
        uint64_t nd = x.d + st->dnw[e];
        if (nd < st->qdb[y]) {
          if (st->qdf[y] == INF64 && st->qdb[y] == INF64) st->qtouch[nt++] = y;
          st->qdb[y] = nd;
          QPUSH(qb, nb, cb, nd, y);
        }
      }
    }
  }
  for (uint32_t i = 0; i < nt; i++) st->qdf[st->qtouch[i]] = st->qdb[st->qtouch[i]] = INF64;
  free(qf);
  free(qb);
  if (settled) *settled = pops;
  return mu;
oom:
  for (uint32_t i = 0; i < nt; i++) st->qdf[st->qtouch[i]] = st->qdb[st->qtouch[i]] = INF64;
  free(qf);
  free(qb);
  if (settled) *settled = pops;
  return INF64;
#undef QPUSH
#undef QPOP
#undef QLESS
}

int orc_query_batch(orc_state *st, uint64_t q, const uint32_t *s, const uint32_t *t,
                    uint64_t *dist, uint64_t *settled) {
  if (!st || !st->finished) return ORC_E_STATE;
  for (uint64_t i = 0; i < q; i++)
    if (s[i] >= st->n || t[i] >= st->n) return ORC_E_INVALID;
  for (uint64_t i = 0; i < q; i++) {
    uint64_t c = 0;
    dist[i] = orc_query(st, s[i], t[i], &c);
    if (settled) settled[i] = c;
  }
  return ORC_OK;
}

/* Textbook Dijkstra with a binary heap on a CSR graph. */
int orc_dijkstra(uint32_t n, const uint64_t *off, const uint32_t *dst,
                 const uint32_t *w, uint32_t s, uint64_t *dist) {
  if (s >= n) return ORC_E_INVALID;
  for (uint32_t v = 0; v < n; v++) dist[v] = INF64;
  heap_t h = {0};
  dist[s] = 0;
  if (heap_push(&h, 0, s)) return ORC_E_OOM;
  while (h.n) {
    uint64_t d;
    uint32_t x;
    heap_pop(&h, &d, &x);
    if (d != dist[x]) continue;
    for (uint64_t e = off[x]; e < off[x + 1]; e++) {
      uint64_t nd = d + w[e];
      if (nd < dist[dst[e]]) {
        dist[dst[e]] = nd;
        if (heap_push(&h, nd, dst[e])) {
          free(h.k);
          free(h.v);
          return ORC_E_OOM;
        }
      }
    }
  }
  free(h.k);
  free(h.v);
  return ORC_OK;
}

int orc_dijkstra_settle(uint32_t n, const uint64_t *off, const uint32_t *dst,
                        const uint32_t *w, uint32_t s, uint64_t max_settled, uint64_t *dist,
                        uint64_t *n_settled) {
  if (s >= n) return ORC_E_INVALID;
  uint8_t *done = (uint8_t *)calloc(n ? n : 1, 1);
  if (!done) return ORC_E_OOM;
  for (uint32_t v = 0; v < n; v++) dist[v] = INF64;
  heap_t h = {0};
  uint64_t cnt = 0;
  dist[s] = 0;
  int rc = heap_push(&h, 0, s) ? ORC_E_OOM : ORC_OK;
  while (rc == ORC_OK && h.n && cnt < max_settled) {
    uint64_t d;
    uint32_t x;
    heap_pop(&h, &d, &x);
    if (d != dist[x] || done[x]) continue;
    done[x] = 1;
    cnt++;
    for (uint64_t e = off[x]; e < off[x + 1]; e++) {
      uint64_t nd = d + w[e];
      if (nd < dist[dst[e]]) {
        dist[dst[e]] = nd;
        if (heap_push(&h, nd, dst[e])) {
          rc = ORC_E_OOM;
          break;
        }
      }
    }
  }
  /* tentative labels of unsettled vertices are not distances */
  for (uint32_t v = 0; v < n; v++)
    if (!done[v]) dist[v] = INF64;
  free(h.k);
  free(h.v);
  free(done);
  if (n_settled) *n_settled = cnt;
  return rc;
}

int orc_overlay_dijkstra(const orc_state *st, uint32_t s, uint64_t *dist) {
  if (!st || s >= st->n) return ORC_E_INVALID;
  for (uint32_t v = 0; v < st->n; v++) dist[v] = INF64;
  if (!st->alive[s]) return ORC_OK;
  heap_t h = {0};
  dist[s] = 0;
  if (heap_push(&h, 0, s)) return ORC_E_OOM;
  while (h.n) {
    uint64_t d;
    uint32_t x;
    heap_pop(&h, &d, &x);
    if (d != dist[x]) continue;
    const adj_t *l = &st->out[x];
    for (uint32_t i = 0; i < l->n; i++) {
      uint64_t nd = d + l->a[i].w;
      if (nd < dist[l->a[i].v]) {
        dist[l->a[i].v] = nd;
        if (heap_push(&h, nd, l->a[i].v)) {
          free(h.k);
          free(h.v);
          return ORC_E_OOM;
        }
      }
    }
  }
  free(h.k);
  free(h.v);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* accessors                                                           */
/* ------------------------------------------------------------------ */

uint32_t orc_n(const orc_state *st) { return st->n; }
uint32_t orc_rounds(const orc_state *st) { return st->round; }
uint32_t orc_alive_count(const orc_state *st) { return st->n_alive; }

void orc_get_labels(const orc_state *st, uint32_t *label) {
  memcpy(label, st->label, (size_t)st->n * sizeof(uint32_t));
}

void orc_get_vertex_state(const orc_state *st, uint32_t *level, int32_t *pc,
                          int32_t *p, uint8_t *alive) {
  for (uint32_t v = 0; v < st->n; v++) {
    if (level) level[v] = st->level[v];
    if (pc) pc[v] = st->Pc[v];
    if (p) p[v] = st->P[v];
    if (alive) alive[v] = st->alive[v];
  }
}

int orc_get_rank(const orc_state *st, uint32_t *rank) {
  if (!st->finished) return ORC_E_STATE;
  memcpy(rank, st->rank, (size_t)st->n * sizeof(uint32_t));
  return ORC_OK;
}

int orc_get_features(const orc_state *st, float *x) {
  if (!st->rec) return ORC_E_STATE;
  memcpy(x, st->rec, (size_t)st->n * 8 * sizeof(float));
  return ORC_OK;
}

uint64_t orc_overlay_count(const orc_state *st) { return overlay_arc_count(st); }

void orc_get_overlay(const orc_state *st, uint32_t *tail, uint32_t *head,
                     uint32_t *w, uint32_t *mid) {
  uint64_t k = 0;
  for (uint32_t v = 0; v < st->n; v++)
    for (uint32_t i = 0; i < st->out[v].n; i++, k++) {
      tail[k] = v;
      head[k] = st->out[v].a[i].v;
      w[k] = st->out[v].a[i].w;
      mid[k] = st->out[v].a[i].mid;
    }
}

uint64_t orc_memo_count(const orc_state *st) { return st->memo.size; }

void orc_get_memo(const orc_state *st, uint32_t *s, uint32_t *t, uint32_t *d) {
  uint64_t k = 0;
  for (uint64_t i = 0; i < st->memo.cap; i++) {
    if (st->memo.key[i] == INF64) continue;
    s[k] = (uint32_t)(st->memo.key[i] >> 32);
    t[k] = (uint32_t)st->memo.key[i];
    d[k] = st->memo.val[i];
    k++;
  }
}

static void copy_recs(const rec_t *r, uint64_t cnt, uint32_t *tail, uint32_t *head,
                      uint32_t *w, uint32_t *mid) {
  for (uint64_t i = 0; i < cnt; i++) {
    tail[i] = r[i].tail;
    head[i] = r[i].head;
    w[i] = r[i].w;
    mid[i] = r[i].mid;
  }
}

uint64_t orc_up_count(const orc_state *st) { return st->nup; }
void orc_get_up(const orc_state *st, uint32_t *tail, uint32_t *head, uint32_t *w,
                uint32_t *mid) {
  copy_recs(st->up, st->nup, tail, head, w, mid);
}
uint64_t orc_down_count(const orc_state *st) { return st->ndown; }
void orc_get_down(const orc_state *st, uint32_t *tail, uint32_t *head, uint32_t *w,
                  uint32_t *mid) {
  copy_recs(st->down, st->ndown, tail, head, w, mid);
}

void orc_get_round_stats(const orc_state *st, orc_round_stats *out) {
  memcpy(out, st->stats, (size_t)st->nstats * sizeof(orc_round_stats));
}
