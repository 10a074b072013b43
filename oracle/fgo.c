/*
 * fgo.c -- CPU oracle for the FGraft harvest (TEST INFRASTRUCTURE ONLY).
 *
 * Only tests, the smoke entry point and the benchmark's CPU-baseline leg may
 * load this library.  It is written from the paper alone and shares no code
 * with the HIP library.  It is deliberately plain: per-point loops, qsort,
 * insertion into sorted arrays, malloc'd lists.
 *
 * Paper references:
 *   Sec. 1 and Sec. 3: scaffold = union of T SAT trees' edges, symmetrised;
 *     blocks p mod B; harvest = beam search of width ef_h from the tree roots
 *     with the point itself as query; the expanded set is occlusion-pruned
 *     to at most R neighbours; S_{b+1} = S_b u {(p,u),(u,p)}; finalize
 *     symmetrises and re-prunes and adds the tree-0 spine.
 *   Prop. 1: keyed randomness, disjoint writes, canonical merges and a total
 *     order on candidates make the graph schedule independent.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -pthread -lm
 */
#define _GNU_SOURCE
#include "fgo.h"

#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------------ */
/* Distances.                                                               */
/* ------------------------------------------------------------------------ */

/* Squared L2 of two float32 rows in the declared order: chunk q of four
 * consecutive elements goes to partial sum q mod 16, each element adds
 * fmaf(delta, delta, partial) with delta = x - y rounded once; then the
 * partials are combined pairwise with offsets 8, 4, 2, 1. */
static float l2_f32_c16(const float* x, const float* y, int d) {
  float p[16];
  for (int s = 0; s < 16; s++) p[s] = 0.0f;
  for (int q = 0; q < d / 4; q++) {
    int s = q % 16;
    for (int c = 0; c < 4; c++) {
      float delta = x[4 * q + c] - y[4 * q + c];
      p[s] = fmaf(delta, delta, p[s]);
    }
  }
  for (int off = 8; off >= 1; off /= 2)
    for (int s = 0; s < off; s++) p[s] = p[s] + p[s + off];
  return p[0];
}

/* Cosine distance 1 - <x, y> of two float32 rows, same order. */
static float cos_f32_c16(const float* x, const float* y, int d) {
  float p[16];
  for (int s = 0; s < 16; s++) p[s] = 0.0f;
  for (int q = 0; q < d / 4; q++) {
    int s = q % 16;
    for (int c = 0; c < 4; c++) p[s] = fmaf(x[4 * q + c], y[4 * q + c], p[s]);
  }
  for (int off = 8; off >= 1; off /= 2)
    for (int s = 0; s < off; s++) p[s] = p[s] + p[s + off];
  return 1.0f - p[0];
}

static double l2_f64(const float* x, const float* y, int d) {
  double s = 0.0;
  for (int i = 0; i < d; i++) {
    double t = (double)x[i] - (double)y[i];
    s += t * t;
  }
  return s;
}

static double cos_f64(const float* x, const float* y, int d) {
  double s = 0.0;
  for (int i = 0; i < d; i++) s += (double)x[i] * (double)y[i];
  return 1.0 - s;
}

static int64_t l2_u8(const uint8_t* x, const uint8_t* y, int d) {
  int64_t s = 0;
  for (int i = 0; i < d; i++) {
    int64_t t = (int64_t)x[i] - (int64_t)y[i];
    s += t * t;
  }
  return s;
}

/* Distance between two rows of the data's type, returned as a double that
 * holds the working-precision value exactly. */
static double dist_rows(const fgo_data* D, const void* a, const void* b) {
  if (D->dtype == FGO_U8) return (double)l2_u8(a, b, D->d);
  if (D->prec == 1)
    return D->metric == FGO_COSINE ? cos_f64(a, b, D->d) : l2_f64(a, b, D->d);
  float r = D->metric == FGO_COSINE ? cos_f32_c16(a, b, D->d)
                                    : l2_f32_c16(a, b, D->d);
  return (double)r;
}

static const void* row(const fgo_data* D, int64_t i) {
  return (const char*)D->x + i * D->stride;
}

double fgo_dist(const fgo_data* D, int64_t i, int64_t j) {
  return dist_rows(D, row(D, i), row(D, j));
}

double fgo_dist_vec(const fgo_data* D, const void* q, int64_t j) {
  return dist_rows(D, q, row(D, j));
}

/* The prune's kill test, alpha * d(c*, c) <= d(p, c): in float32 with one
 * rounding for float32 and integer data, in float64 for the FP64 mode. */
static int occludes(const fgo_data* D, float alpha, double d_kept_c,
                    double d_p_c) {
  if (D->prec == 1 && D->dtype == FGO_F32)
    return (double)alpha * d_kept_c <= d_p_c;
  float prod = alpha * (float)d_kept_c;
  return (double)prod <= d_p_c;
}

static int data_ok(const fgo_data* D) {
  if (!D || !D->x || D->n < 1 || D->d < 1) return 0;
  if (D->dtype != FGO_F32 && D->dtype != FGO_U8) return 0;
  if (D->dtype == FGO_F32 && D->d % 4 != 0) return 0;
  if (D->dtype == FGO_U8 && D->metric != FGO_L2) return 0;
  if (D->metric != FGO_L2 && D->metric != FGO_COSINE) return 0;
  int64_t esz = D->dtype == FGO_F32 ? 4 : 1;
  if (D->stride < esz * D->d) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Keyed randomness and hashing.                                            */
/* ------------------------------------------------------------------------ */

/* Output k (0-based) of the SplitMix64 stream seeded with `seed`
 * (Steele, Lea and Flood 2014): state = seed + (k+1) * golden gamma, then
 * the published finaliser. */
uint64_t fgo_splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Root of tree t: the first draw splitmix64(seed, t * 2^32 + j) mod n,
 * j = 0, 1, ..., that is not already a root. */
int fgo_roots(uint64_t seed, int64_t n, uint32_t T, uint32_t* roots) {
  if (n < 1 || T < 1 || (int64_t)T > n || !roots) return -1;
  for (uint32_t t = 0; t < T; t++) {
    for (uint64_t j = 0;; j++) {
      uint32_t r = (uint32_t)(fgo_splitmix64(seed, ((uint64_t)t << 32) + j) %
                              (uint64_t)n);
      int dup = 0;
      for (uint32_t u = 0; u < t; u++) dup |= roots[u] == r;
      if (!dup) {
        roots[t] = r;
        break;
      }
    }
  }
  return 0;
}

/* FNV-1a, 64-bit (Fowler, Noll, Vo). */
uint64_t fgo_fnv1a64(const void* bytes, size_t len) {
  const uint8_t* b = bytes;
  uint64_t h = 0xCBF29CE484222325ull;
  for (size_t i = 0; i < len; i++) {
    h ^= b[i];
    h *= 0x100000001B3ull;
  }
  return h;
}

/* ------------------------------------------------------------------------ */
/* Candidates under the total order (distance, id).                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  double d;
  uint32_t id;
} cand;

static int key_less(double da, uint32_t ia, double db, uint32_t ib) {
  return da < db || (da == db && ia < ib);
}

static int cand_cmp(const void* a, const void* b) {
  const cand* x = a;
  const cand* y = b;
  if (key_less(x->d, x->id, y->d, y->id)) return -1;
  if (key_less(y->d, y->id, x->d, x->id)) return 1;
  return 0;
}

static int u32_cmp(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return x < y ? -1 : x > y;
}

/* ------------------------------------------------------------------------ */
/* A tiny parallel-for over host threads.  Items are claimed from an atomic */
/* counter; results never depend on which thread runs which item.           */
/* ------------------------------------------------------------------------ */

typedef void (*item_fn)(void* ctx, int64_t item, int tid);
typedef struct {
  item_fn fn;
  void* ctx;
  int64_t count;
  atomic_llong next;
  int tid;
} pf_shared;
typedef struct {
  pf_shared* s;
  int tid;
} pf_arg;

static void* pf_worker(void* arg) {
  pf_arg* a = arg;
  for (;;) {
    int64_t i = atomic_fetch_add(&a->s->next, 1);
    if (i >= a->s->count) break;
    a->s->fn(a->s->ctx, i, a->tid);
  }
  return NULL;
}

static void parallel_for(int64_t count, uint32_t threads, item_fn fn,
                         void* ctx) {
  if (threads < 1) threads = 1;
  pf_shared s;
  s.fn = fn;
  s.ctx = ctx;
  s.count = count;
  atomic_init(&s.next, 0);
  pthread_t* th = malloc(sizeof(pthread_t) * threads);
  pf_arg* args = malloc(sizeof(pf_arg) * threads);
  for (uint32_t t = 1; t < threads; t++) {
    args[t].s = &s;
    args[t].tid = (int)t;
    pthread_create(&th[t], NULL, pf_worker, &args[t]);
  }
  args[0].s = &s;
  args[0].tid = 0;
  pf_worker(&args[0]);
  for (uint32_t t = 1; t < threads; t++) pthread_join(th[t], NULL);
  free(th);
  free(args);
}

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------------------------------------ */
/* Spatial-approximation tree (Navarro 2002), classic variant.              */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint32_t a;     /* the node */
  uint32_t* bag;  /* its not-yet-placed descendants */
  int64_t m;
} sat_frame;

/* For node a with bag S: sort S by (d(v,a), id); walk it and accept v as a
 * neighbour of a iff d(v,a) < d(v,b) for every neighbour b accepted before
 * it; every other v joins the bag of its closest neighbour (ties by the
 * neighbour's id).  An explicit stack replaces recursion (degenerate data
 * can make the tree as deep as n). */
int fgo_sat_tree(const fgo_data* D, uint32_t root, uint32_t* parent,
                 uint64_t* evals) {
  if (!data_ok(D) || (int64_t)root >= D->n || !parent) return -1;
  int64_t n = D->n;
  uint64_t ev = 0;
  for (int64_t v = 0; v < n; v++) parent[v] = FGO_NONE;

  int64_t cap = 64, sp = 0;
  sat_frame* st = malloc(sizeof(sat_frame) * cap);
  uint32_t* bag0 = malloc(sizeof(uint32_t) * (n > 1 ? n - 1 : 1));
  int64_t m0 = 0;
  for (int64_t v = 0; v < n; v++)
    if ((uint32_t)v != root) bag0[m0++] = (uint32_t)v;
  st[sp++] = (sat_frame){root, bag0, m0};

  while (sp > 0) {
    sat_frame f = st[--sp];
    if (f.m == 0) {
      free(f.bag);
      continue;
    }
    const void* ra = row(D, f.a);
    cand* c = malloc(sizeof(cand) * f.m);
    for (int64_t i = 0; i < f.m; i++) {
      c[i].d = dist_rows(D, row(D, f.bag[i]), ra);
      c[i].id = f.bag[i];
      ev++;
    }
    qsort(c, f.m, sizeof(cand), cand_cmp);

    /* Neighbour acceptance, in sorted order. */
    int64_t* nb = malloc(sizeof(int64_t) * f.m); /* indices into c */
    int64_t nn = 0;
    for (int64_t i = 0; i < f.m; i++) {
      int ok = 1;
      for (int64_t k = 0; k < nn; k++) {
        double dvb = fgo_dist(D, c[i].id, c[nb[k]].id);
        ev++;
        if (!(c[i].d < dvb)) {
          ok = 0;
          break;
        }
      }
      if (ok) nb[nn++] = i;
    }

    /* Closest-neighbour bag for every non-neighbour. */
    int64_t* owner = malloc(sizeof(int64_t) * f.m);
    int64_t* size = calloc(nn, sizeof(int64_t));
    char* is_nb = calloc(f.m, 1);
    for (int64_t k = 0; k < nn; k++) is_nb[nb[k]] = 1;
    for (int64_t i = 0; i < f.m; i++) {
      owner[i] = -1;
      if (is_nb[i]) continue;
      double bd = 0.0;
      uint32_t bid = FGO_NONE;
      for (int64_t k = 0; k < nn; k++) {
        uint32_t b = c[nb[k]].id;
        double dv = fgo_dist(D, c[i].id, b);
        ev++;
        if (owner[i] < 0 || key_less(dv, b, bd, bid)) {
          owner[i] = k;
          bd = dv;
          bid = b;
        }
      }
      size[owner[i]]++;
    }

    for (int64_t k = 0; k < nn; k++) parent[c[nb[k]].id] = f.a;

    /* Children are pushed in neighbour order (the order does not matter). */
    if (sp + nn > cap) {
      while (sp + nn > cap) cap *= 2;
      st = realloc(st, sizeof(sat_frame) * cap);
    }
    uint32_t** bags = malloc(sizeof(uint32_t*) * (nn ? nn : 1));
    int64_t* fill = calloc(nn ? nn : 1, sizeof(int64_t));
    for (int64_t k = 0; k < nn; k++)
      bags[k] = malloc(sizeof(uint32_t) * (size[k] ? size[k] : 1));
    for (int64_t i = 0; i < f.m; i++)
      if (owner[i] >= 0) bags[owner[i]][fill[owner[i]]++] = c[i].id;
    for (int64_t k = 0; k < nn; k++)
      st[sp++] = (sat_frame){c[nb[k]].id, bags[k], size[k]};

    free(bags);
    free(fill);
    free(is_nb);
    free(size);
    free(owner);
    free(nb);
    free(c);
    free(f.bag);
  }
  free(st);
  if (evals) *evals += ev;
  return 0;
}

int64_t fgo_scaffold_csr(int64_t n, uint32_t T, const uint32_t* parents,
                         uint64_t* off, uint32_t* ids) {
  if (n < 1 || T < 1 || !parents || !off || !ids) return -1;
  /* Collect every directed edge (parent, child) and (child, parent). */
  uint64_t* deg = calloc(n, sizeof(uint64_t));
  for (uint32_t t = 0; t < T; t++)
    for (int64_t v = 0; v < n; v++) {
      uint32_t p = parents[(int64_t)t * n + v];
      if (p == FGO_NONE) continue;
      deg[v]++;
      deg[p]++;
    }
  uint64_t* start = malloc(sizeof(uint64_t) * (n + 1));
  start[0] = 0;
  for (int64_t v = 0; v < n; v++) start[v + 1] = start[v] + deg[v];
  uint32_t* tmp = malloc(sizeof(uint32_t) * (start[n] ? start[n] : 1));
  uint64_t* fill = calloc(n, sizeof(uint64_t));
  for (uint32_t t = 0; t < T; t++)
    for (int64_t v = 0; v < n; v++) {
      uint32_t p = parents[(int64_t)t * n + v];
      if (p == FGO_NONE) continue;
      tmp[start[v] + fill[v]++] = p;
      tmp[start[p] + fill[p]++] = (uint32_t)v;
    }
  /* Sort each row by id and drop repeats. */
  uint64_t nnz = 0;
  off[0] = 0;
  for (int64_t v = 0; v < n; v++) {
    uint32_t* r = tmp + start[v];
    uint64_t m = deg[v];
    qsort(r, m, sizeof(uint32_t), u32_cmp);
    for (uint64_t i = 0; i < m; i++)
      if (i == 0 || r[i] != r[i - 1]) ids[nnz++] = r[i];
    off[v + 1] = nnz;
  }
  free(fill);
  free(tmp);
  free(start);
  free(deg);
  return (int64_t)nnz;
}

/* ------------------------------------------------------------------------ */
/* Beam search (Sec. 3): a bounded list of the ef best visited vertices     */
/* under (distance, id).  Repeatedly expand the best unexpanded entry and   */
/* evaluate every not-yet-visited neighbour; stop when every entry of the   */
/* list has been expanded.  Every evaluated vertex counts once.             */
/* ------------------------------------------------------------------------ */

typedef struct {
  double d;
  uint32_t id;
  uint8_t expanded;
} bentry;

typedef struct {
  uint8_t* visited;   /* n flags, all zero between queries */
  uint32_t* vlist;    /* visited ids in visit order */
  int64_t vn;
  bentry* beam;       /* capacity ef + 1 */
  uint32_t bn;
  cand* E;            /* expanded entries in expansion order */
  int64_t En, Ecap;
} beam_scratch;

static void scratch_init(beam_scratch* s, int64_t n, uint32_t ef) {
  s->visited = calloc(n, 1);
  s->vlist = malloc(sizeof(uint32_t) * n);
  s->vn = 0;
  s->beam = malloc(sizeof(bentry) * (ef + 1));
  s->bn = 0;
  s->Ecap = 64;
  s->E = malloc(sizeof(cand) * s->Ecap);
  s->En = 0;
}

static void scratch_free(beam_scratch* s) {
  free(s->visited);
  free(s->vlist);
  free(s->beam);
  free(s->E);
}

static void scratch_reset(beam_scratch* s) {
  for (int64_t i = 0; i < s->vn; i++) s->visited[s->vlist[i]] = 0;
  s->vn = 0;
  s->bn = 0;
  s->En = 0;
}

/* Bounded insertion: keep the ef smallest keys seen. */
static void beam_insert(beam_scratch* s, uint32_t ef, double d, uint32_t id) {
  if (s->bn == ef) {
    bentry* last = &s->beam[s->bn - 1];
    if (!key_less(d, id, last->d, last->id)) return;
  }
  int64_t i = s->bn;
  while (i > 0 && key_less(d, id, s->beam[i - 1].d, s->beam[i - 1].id)) {
    s->beam[i] = s->beam[i - 1];
    i--;
  }
  s->beam[i].d = d;
  s->beam[i].id = id;
  s->beam[i].expanded = 0;
  if (s->bn < ef) s->bn++;
}

static void visit(const fgo_data* D, const void* q, beam_scratch* s,
                  uint32_t ef, uint32_t u) {
  if (s->visited[u]) return;
  s->visited[u] = 1;
  s->vlist[s->vn++] = u;
  beam_insert(s, ef, dist_rows(D, q, row(D, u)), u);
}

static void beam_run(const fgo_data* D, const void* q, const uint64_t* off,
                     const uint32_t* ids, const uint32_t* roots, uint32_t T,
                     uint32_t ef, beam_scratch* s) {
  for (uint32_t t = 0; t < T; t++) visit(D, q, s, ef, roots[t]);
  for (;;) {
    int64_t i = 0;
    while (i < s->bn && s->beam[i].expanded) i++;
    if (i == s->bn) break;
    s->beam[i].expanded = 1;
    uint32_t v = s->beam[i].id;
    if (s->En == s->Ecap) {
      s->Ecap *= 2;
      s->E = realloc(s->E, sizeof(cand) * s->Ecap);
    }
    s->E[s->En].d = s->beam[i].d;
    s->E[s->En].id = v;
    s->En++;
    for (uint64_t e = off[v]; e < off[v + 1]; e++) visit(D, q, s, ef, ids[e]);
  }
}

int64_t fgo_beam(const fgo_data* D, const void* q, int64_t q_index,
                 const uint64_t* off, const uint32_t* ids,
                 const uint32_t* roots, uint32_t T, uint32_t ef,
                 uint32_t* beam_ids, double* beam_d, uint32_t* beam_n,
                 uint32_t* E_ids, double* E_d, uint32_t* E_n,
                 uint32_t* V_ids, uint32_t* V_n) {
  if (!data_ok(D) || ef < 1 || T < 1 || !off || !ids || !roots) return -1;
  const void* qr = q_index >= 0 ? row(D, q_index) : q;
  if (!qr) return -1;
  beam_scratch s;
  scratch_init(&s, D->n, ef);
  beam_run(D, qr, off, ids, roots, T, ef, &s);
  if (beam_n) *beam_n = s.bn;
  for (uint32_t i = 0; i < s.bn; i++) {
    if (beam_ids) beam_ids[i] = s.beam[i].id;
    if (beam_d) beam_d[i] = s.beam[i].d;
  }
  if (E_n) *E_n = (uint32_t)s.En;
  for (int64_t i = 0; i < s.En; i++) {
    if (E_ids) E_ids[i] = s.E[i].id;
    if (E_d) E_d[i] = s.E[i].d;
  }
  if (V_n) *V_n = (uint32_t)s.vn;
  if (V_ids)
    for (int64_t i = 0; i < s.vn; i++) V_ids[i] = s.vlist[i];
  int64_t evals = s.vn;
  scratch_free(&s);
  return evals;
}

/* ------------------------------------------------------------------------ */
/* Occlusion prune (Sec. 3; FANNG / DiskANN rule).                          */
/* Candidates sorted by key; take the next live one, keep it, stop at R;    */
/* every later live candidate c with alpha * d(kept, c) <= d(p, c) dies.    */
/* ------------------------------------------------------------------------ */

static uint32_t prune_sorted(const fgo_data* D, const cand* c, int64_t m,
                             uint32_t R, float alpha, uint32_t* out,
                             uint64_t* pe) {
  char* alive = malloc(m ? m : 1);
  memset(alive, 1, m ? m : 1);
  uint32_t k = 0;
  uint64_t pairs = 0;
  for (int64_t i = 0; i < m && k < R; i++) {
    if (!alive[i]) continue;
    out[k++] = c[i].id;
    if (k == R) break;
    for (int64_t j = i + 1; j < m; j++) {
      if (!alive[j]) continue;
      pairs++;
      double dij = fgo_dist(D, c[i].id, c[j].id);
      if (occludes(D, alpha, dij, c[j].d)) alive[j] = 0;
    }
  }
  free(alive);
  if (pe) *pe += pairs;
  return k;
}

int32_t fgo_prune(const fgo_data* D, int64_t p, const uint32_t* cand_ids,
                  const double* cand_d, uint32_t m, uint32_t R, float alpha,
                  uint32_t* out, uint64_t* pair_evals) {
  (void)p;
  if (!data_ok(D) || R < 1 || !(alpha >= 1.0f) || !isfinite(alpha)) return -1;
  cand* c = malloc(sizeof(cand) * (m ? m : 1));
  for (uint32_t i = 0; i < m; i++) {
    c[i].id = cand_ids[i];
    c[i].d = cand_d[i];
  }
  qsort(c, m, sizeof(cand), cand_cmp);
  uint32_t k = prune_sorted(D, c, m, R, alpha, out, pair_evals);
  free(c);
  return (int32_t)k;
}

/* ------------------------------------------------------------------------ */
/* Harvest of one block.                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  const fgo_data* D;
  const uint64_t* off;
  const uint32_t* ids;
  const uint32_t* roots;
  const fgo_params* P;
  const uint32_t* points;
  uint32_t* rows;
  uint32_t* cnt;
  beam_scratch* scratch; /* one per thread */
  uint64_t* evals;       /* per thread */
  uint64_t* pe;
  uint64_t* expansions;
} harvest_ctx;

static void harvest_one(void* vctx, int64_t item, int tid) {
  harvest_ctx* h = vctx;
  const fgo_data* D = h->D;
  uint32_t p = h->points[item];
  beam_scratch* s = &h->scratch[tid];
  scratch_reset(s);
  beam_run(D, row(D, p), h->off, h->ids, h->roots, h->P->T, h->P->ef_h, s);
  h->evals[tid] += (uint64_t)s->vn;
  h->expansions[tid] += (uint64_t)s->En;
  /* Prune the expanded set without p itself. */
  cand* c = malloc(sizeof(cand) * (s->En ? s->En : 1));
  int64_t m = 0;
  for (int64_t i = 0; i < s->En; i++)
    if (s->E[i].id != p) c[m++] = s->E[i];
  qsort(c, m, sizeof(cand), cand_cmp);
  uint32_t R = h->P->R;
  uint32_t* out = h->rows + (int64_t)p * R;
  uint32_t k = prune_sorted(D, c, m, R, h->P->alpha, out, &h->pe[tid]);
  for (uint32_t i = k; i < R; i++) out[i] = FGO_NONE;
  h->cnt[p] = k;
  free(c);
}

static int params_ok(const fgo_params* P) {
  return P && P->T >= 1 && P->ef_h >= 1 && P->R >= 1 && isfinite(P->alpha) &&
         P->alpha >= 1.0f;
}

int fgo_harvest_block(const fgo_data* D, const uint64_t* off,
                      const uint32_t* ids, const uint32_t* roots,
                      const fgo_params* P, uint32_t b, const uint32_t* order,
                      int64_t order_len, uint32_t* rows, uint32_t* cnt,
                      fgo_counters* C) {
  if (!data_ok(D) || !params_ok(P) || !off || !ids || !roots || !rows || !cnt)
    return -1;
  uint32_t Be = P->B > 1 ? P->B : 1;
  if (b >= Be) return -1;
  int64_t n = D->n;
  int64_t np = n > b ? (n - b + Be - 1) / Be : 0;
  uint32_t* pts = malloc(sizeof(uint32_t) * (np ? np : 1));
  if (order) {
    if (order_len != np) {
      free(pts);
      return -1;
    }
    for (int64_t i = 0; i < np; i++) {
      if (order[i] >= n || order[i] % Be != b) {
        free(pts);
        return -1;
      }
      pts[i] = order[i];
    }
  } else {
    for (int64_t i = 0; i < np; i++) pts[i] = (uint32_t)(b + i * Be);
  }
  uint32_t th = P->threads ? P->threads : 1;
  harvest_ctx h = {D, off, ids, roots, P, pts, rows, cnt, NULL, NULL, NULL,
                   NULL};
  h.scratch = malloc(sizeof(beam_scratch) * th);
  h.evals = calloc(th, sizeof(uint64_t));
  h.pe = calloc(th, sizeof(uint64_t));
  h.expansions = calloc(th, sizeof(uint64_t));
  for (uint32_t t = 0; t < th; t++) scratch_init(&h.scratch[t], n, P->ef_h);
  parallel_for(np, th, harvest_one, &h);
  for (uint32_t t = 0; t < th; t++) {
    if (C) {
      C->harvest_evals += h.evals[t];
      C->prune_evals += h.pe[t];
      C->expansions += h.expansions[t];
    }
    scratch_free(&h.scratch[t]);
  }
  free(h.scratch);
  free(h.evals);
  free(h.pe);
  free(h.expansions);
  free(pts);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Union merge S_{b+1} = S_b u {(p,u),(u,p)} for the rows of block b.       */
/* ------------------------------------------------------------------------ */

int64_t fgo_merge_block(int64_t n, const uint64_t* off, const uint32_t* ids,
                        const uint32_t* rows, const uint32_t* cnt, uint32_t R,
                        uint32_t B, uint32_t b, uint64_t* off_out,
                        uint32_t* ids_out, uint64_t cap) {
  if (n < 1 || !off || !ids || !rows || !cnt || !off_out || !ids_out)
    return -1;
  uint32_t Be = B > 1 ? B : 1;
  uint64_t* deg = malloc(sizeof(uint64_t) * n);
  for (int64_t v = 0; v < n; v++) deg[v] = off[v + 1] - off[v];
  for (int64_t p = b; p < n; p += Be)
    for (uint32_t i = 0; i < cnt[p]; i++) {
      deg[p]++;
      deg[rows[p * R + i]]++;
    }
  uint64_t* start = malloc(sizeof(uint64_t) * (n + 1));
  start[0] = 0;
  for (int64_t v = 0; v < n; v++) start[v + 1] = start[v] + deg[v];
  uint32_t* tmp = malloc(sizeof(uint32_t) * (start[n] ? start[n] : 1));
  uint64_t* fill = calloc(n, sizeof(uint64_t));
  for (int64_t v = 0; v < n; v++)
    for (uint64_t e = off[v]; e < off[v + 1]; e++)
      tmp[start[v] + fill[v]++] = ids[e];
  for (int64_t p = b; p < n; p += Be)
    for (uint32_t i = 0; i < cnt[p]; i++) {
      uint32_t u = rows[p * R + i];
      tmp[start[p] + fill[p]++] = u;
      tmp[start[u] + fill[u]++] = (uint32_t)p;
    }
  uint64_t nnz = 0;
  int64_t rc = 0;
  off_out[0] = 0;
  for (int64_t v = 0; v < n; v++) {
    uint32_t* r = tmp + start[v];
    qsort(r, deg[v], sizeof(uint32_t), u32_cmp);
    for (uint64_t i = 0; i < deg[v]; i++) {
      if (i > 0 && r[i] == r[i - 1]) continue;
      if (nnz == cap) {
        rc = -2;
        break;
      }
      ids_out[nnz++] = r[i];
    }
    if (rc) break;
    off_out[v + 1] = nnz;
  }
  free(fill);
  free(tmp);
  free(start);
  free(deg);
  return rc ? rc : (int64_t)nnz;
}

/* ------------------------------------------------------------------------ */
/* Finalize: symmetrise the harvested rows and re-prune.                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  const fgo_data* D;
  const fgo_params* P;
  const uint32_t* rows;
  const uint32_t* cnt;
  const uint64_t* roff;  /* reverse lists: {u : p in A[u]} */
  const uint32_t* rids;
  uint32_t* g_nbrs;
  uint32_t* g_cnt;
  uint64_t* ev;  /* per thread */
} fin_ctx;

static void finalize_one(void* vctx, int64_t p, int tid) {
  fin_ctx* f = vctx;
  uint32_t R = f->P->R;
  int64_t m0 = f->cnt[p] + (f->roff[p + 1] - f->roff[p]);
  uint32_t* u = malloc(sizeof(uint32_t) * (m0 ? m0 : 1));
  int64_t m = 0;
  for (uint32_t i = 0; i < f->cnt[p]; i++) u[m++] = f->rows[p * R + i];
  for (uint64_t e = f->roff[p]; e < f->roff[p + 1]; e++) u[m++] = f->rids[e];
  qsort(u, m, sizeof(uint32_t), u32_cmp);
  cand* c = malloc(sizeof(cand) * (m ? m : 1));
  int64_t mc = 0;
  for (int64_t i = 0; i < m; i++) {
    if (i > 0 && u[i] == u[i - 1]) continue;
    c[mc].id = u[i];
    c[mc].d = fgo_dist(f->D, p, u[i]);
    f->ev[tid]++;
    mc++;
  }
  qsort(c, mc, sizeof(cand), cand_cmp);
  uint32_t* out = f->g_nbrs + p * R;
  uint32_t k;
  if (mc > (int64_t)R || f->P->reprune_all) {
    k = prune_sorted(f->D, c, mc, R, f->P->alpha, out, &f->ev[tid]);
  } else {
    k = (uint32_t)mc;
    for (int64_t i = 0; i < mc; i++) out[i] = c[i].id;
  }
  for (uint32_t i = k; i < R; i++) out[i] = FGO_NONE;
  f->g_cnt[p] = k;
  free(c);
  free(u);
}

int fgo_finalize(const fgo_data* D, const uint32_t* rows, const uint32_t* cnt,
                 const fgo_params* P, uint32_t* g_nbrs, uint32_t* g_cnt,
                 fgo_counters* C) {
  if (!data_ok(D) || !params_ok(P) || !rows || !cnt || !g_nbrs || !g_cnt)
    return -1;
  int64_t n = D->n;
  uint32_t R = P->R;
  uint64_t* roff = calloc(n + 1, sizeof(uint64_t));
  for (int64_t p = 0; p < n; p++)
    for (uint32_t i = 0; i < cnt[p]; i++) roff[rows[p * R + i] + 1]++;
  for (int64_t v = 0; v < n; v++) roff[v + 1] += roff[v];
  uint32_t* rids = malloc(sizeof(uint32_t) * (roff[n] ? roff[n] : 1));
  uint64_t* fill = calloc(n, sizeof(uint64_t));
  for (int64_t p = 0; p < n; p++)
    for (uint32_t i = 0; i < cnt[p]; i++) {
      uint32_t u = rows[p * R + i];
      rids[roff[u] + fill[u]++] = (uint32_t)p;
    }
  uint32_t th = P->threads ? P->threads : 1;
  fin_ctx f = {D, P, rows, cnt, roff, rids, g_nbrs, g_cnt, NULL};
  f.ev = calloc(th, sizeof(uint64_t));
  parallel_for(n, th, finalize_one, &f);
  for (uint32_t t = 0; t < th; t++)
    if (C) C->finalize_evals += f.ev[t];
  free(f.ev);
  free(fill);
  free(rids);
  free(roff);
  return 0;
}

/* Hash of the final graph: FNV-1a-64 over the little-endian bytes of n (u64),
 * R (u32), T (u32), then per point its count and ids, then tree 0's parent
 * array, then the roots. */
uint64_t fgo_graph_hash(int64_t n, uint32_t R, uint32_t T,
                        const uint32_t* g_nbrs, const uint32_t* g_cnt,
                        const uint32_t* parent0, const uint32_t* roots) {
  uint64_t h = 0xCBF29CE484222325ull;
#define FEED(ptr, len)                                   \
  do {                                                   \
    const uint8_t* b_ = (const uint8_t*)(ptr);           \
    for (size_t i_ = 0; i_ < (size_t)(len); i_++) {      \
      h ^= b_[i_];                                       \
      h *= 0x100000001B3ull;                             \
    }                                                    \
  } while (0)
  uint64_t n64 = (uint64_t)n;
  FEED(&n64, 8);
  FEED(&R, 4);
  FEED(&T, 4);
  for (int64_t p = 0; p < n; p++) {
    FEED(&g_cnt[p], 4);
    FEED(g_nbrs + p * R, 4 * (size_t)g_cnt[p]);
  }
  FEED(parent0, 4 * (size_t)n);
  FEED(roots, 4 * (size_t)T);
#undef FEED
  return h;
}

/* ------------------------------------------------------------------------ */
/* Whole build.                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
  const fgo_data* D;
  const uint32_t* roots;
  uint32_t* parents;
  uint64_t* ev;
} sat_ctx;

static void sat_one(void* vctx, int64_t t, int tid) {
  (void)tid;
  sat_ctx* s = vctx;
  s->ev[t] = 0;
  fgo_sat_tree(s->D, s->roots[t], s->parents + t * s->D->n, &s->ev[t]);
}

int fgo_build_graph(const fgo_data* D, uint64_t seed, const fgo_params* P,
                    uint32_t* g_nbrs, uint32_t* g_cnt, uint32_t* parent0,
                    uint32_t* roots, fgo_counters* C, uint64_t* hash) {
  if (!data_ok(D) || !params_ok(P) || !g_nbrs || !g_cnt || !parent0 || !roots)
    return -1;
  int64_t n = D->n;
  uint32_t T = P->T, R = P->R;
  if ((int64_t)T > n) return -1;
  fgo_counters local;
  memset(&local, 0, sizeof(local));
  if (!C) C = &local;
  uint32_t th = P->threads ? P->threads : 1;

  double t0 = now_s();
  fgo_roots(seed, n, T, roots);
  uint32_t* parents = malloc(sizeof(uint32_t) * (size_t)T * n);
  uint64_t* ev = calloc(T, sizeof(uint64_t));
  sat_ctx sc = {D, roots, parents, ev};
  parallel_for(T, th < T ? th : T, sat_one, &sc);
  for (uint32_t t = 0; t < T; t++) C->scaffold_evals += ev[t];
  free(ev);
  uint64_t cap = 2ull * T * (uint64_t)(n - 1) + 2ull * R * (uint64_t)n + 1;
  uint64_t* off = malloc(sizeof(uint64_t) * (n + 1));
  uint32_t* ids = malloc(sizeof(uint32_t) * cap);
  uint64_t* off2 = malloc(sizeof(uint64_t) * (n + 1));
  uint32_t* ids2 = malloc(sizeof(uint32_t) * cap);
  fgo_scaffold_csr(n, T, parents, off, ids);
  memcpy(parent0, parents, sizeof(uint32_t) * n);
  free(parents);
  double t1 = now_s();
  C->t_scaffold += t1 - t0;

  uint32_t* rows = malloc(sizeof(uint32_t) * (size_t)n * R);
  uint32_t* cnt = calloc(n, sizeof(uint32_t));
  for (int64_t i = 0; i < n * (int64_t)R; i++) rows[i] = FGO_NONE;
  uint32_t Be = P->B > 1 ? P->B : 1;
  for (uint32_t b = 0; b < Be; b++) {
    double ta = now_s();
    fgo_harvest_block(D, off, ids, roots, P, b, NULL, 0, rows, cnt, C);
    double tb = now_s();
    C->t_harvest += tb - ta;
    if (b + 1 < Be) {
      fgo_merge_block(n, off, ids, rows, cnt, R, Be, b, off2, ids2, cap);
      uint64_t* to = off;
      off = off2;
      off2 = to;
      uint32_t* ti = ids;
      ids = ids2;
      ids2 = ti;
      C->t_merge += now_s() - tb;
    }
  }
  double t2 = now_s();
  fgo_finalize(D, rows, cnt, P, g_nbrs, g_cnt, C);
  C->t_finalize += now_s() - t2;
  if (hash) *hash = fgo_graph_hash(n, R, T, g_nbrs, g_cnt, parent0, roots);
  free(rows);
  free(cnt);
  free(off);
  free(ids);
  free(off2);
  free(ids2);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Query search over G u spine, and brute-force ground truth.               */
/* ------------------------------------------------------------------------ */

typedef struct {
  const fgo_data* D;
  const uint64_t* off;
  const uint32_t* ids;
  const uint32_t* roots;
  uint32_t T, L, k;
  const uint8_t* queries;
  int64_t qstride;
  beam_scratch* scratch;
  uint32_t* out_ids;
  double* out_d;
  uint32_t* out_evals;
} search_ctx;

static void search_one(void* vctx, int64_t qi, int tid) {
  search_ctx* s = vctx;
  beam_scratch* b = &s->scratch[tid];
  scratch_reset(b);
  beam_run(s->D, s->queries + qi * s->qstride, s->off, s->ids, s->roots, s->T,
           s->L, b);
  for (uint32_t i = 0; i < s->k; i++) {
    s->out_ids[qi * s->k + i] = i < b->bn ? b->beam[i].id : FGO_NONE;
    s->out_d[qi * s->k + i] = i < b->bn ? b->beam[i].d : INFINITY;
  }
  if (s->out_evals) s->out_evals[qi] = (uint32_t)b->vn;
}

int fgo_search(const fgo_data* D, const uint32_t* g_nbrs, const uint32_t* g_cnt,
               uint32_t R, const uint32_t* parent0, const uint32_t* roots,
               uint32_t T, const void* queries, int64_t nq, uint32_t k,
               uint32_t L, uint32_t threads, uint32_t* out_ids,
               double* out_d, uint32_t* out_evals) {
  if (!data_ok(D) || !g_nbrs || !g_cnt || !parent0 || !roots || !queries ||
      nq < 0 || k < 1 || L < k || !out_ids || !out_d)
    return -1;
  int64_t n = D->n;
  /* Adjacency of the search graph: G's row, then tree 0's parent, then tree
   * 0's children. */
  uint64_t* off = calloc(n + 1, sizeof(uint64_t));
  for (int64_t v = 0; v < n; v++) {
    off[v + 1] += g_cnt[v];
    if (parent0[v] != FGO_NONE) {
      off[v + 1]++;
      off[parent0[v] + 1]++;
    }
  }
  for (int64_t v = 0; v < n; v++) off[v + 1] += off[v];
  uint32_t* ids = malloc(sizeof(uint32_t) * (off[n] ? off[n] : 1));
  uint64_t* fill = calloc(n, sizeof(uint64_t));
  for (int64_t v = 0; v < n; v++)
    for (uint32_t i = 0; i < g_cnt[v]; i++)
      ids[off[v] + fill[v]++] = g_nbrs[v * R + i];
  for (int64_t v = 0; v < n; v++)
    if (parent0[v] != FGO_NONE) ids[off[v] + fill[v]++] = parent0[v];
  for (int64_t v = 0; v < n; v++)
    if (parent0[v] != FGO_NONE) {
      uint32_t p = parent0[v];
      ids[off[p] + fill[p]++] = (uint32_t)v;
    }
  uint32_t th = threads ? threads : 1;
  search_ctx s = {D, off, ids, roots, T, L, k, queries, 0, NULL, out_ids,
                  out_d, out_evals};
  s.qstride = (int64_t)D->d * (D->dtype == FGO_F32 ? 4 : 1);
  s.scratch = malloc(sizeof(beam_scratch) * th);
  for (uint32_t t = 0; t < th; t++) scratch_init(&s.scratch[t], n, L);
  parallel_for(nq, th, search_one, &s);
  for (uint32_t t = 0; t < th; t++) scratch_free(&s.scratch[t]);
  free(s.scratch);
  free(fill);
  free(ids);
  free(off);
  return 0;
}

typedef struct {
  const fgo_data* D;
  const uint8_t* queries;
  int64_t qstride;
  uint32_t k;
  uint32_t* out_ids;
  double* out_d;
} knn_ctx;

static void knn_one(void* vctx, int64_t qi, int tid) {
  (void)tid;
  knn_ctx* s = vctx;
  int64_t n = s->D->n;
  cand* c = malloc(sizeof(cand) * n);
  for (int64_t j = 0; j < n; j++) {
    c[j].d = dist_rows(s->D, s->queries + qi * s->qstride, row(s->D, j));
    c[j].id = (uint32_t)j;
  }
  qsort(c, n, sizeof(cand), cand_cmp);
  for (uint32_t i = 0; i < s->k; i++) {
    s->out_ids[qi * s->k + i] = i < n ? c[i].id : FGO_NONE;
    s->out_d[qi * s->k + i] = i < n ? c[i].d : INFINITY;
  }
  free(c);
}

int fgo_knn_brute(const fgo_data* D, const void* queries, int64_t nq,
                  uint32_t k, uint32_t threads, uint32_t* out_ids,
                  double* out_d) {
  if (!data_ok(D) || !queries || nq < 0 || k < 1 || !out_ids || !out_d)
    return -1;
  knn_ctx s = {D, queries, (int64_t)D->d * (D->dtype == FGO_F32 ? 4 : 1), k,
               out_ids, out_d};
  parallel_for(nq, threads ? threads : 1, knn_one, &s);
  return 0;
}
