/*
 * fgo.h -- CPU oracle for the FGraft harvest (TEST INFRASTRUCTURE ONLY).
 *
 * A plain, slow, obviously correct C implementation of what the harvest
 * path computes: the SAT-forest scaffold, the block schedule, the self-query
 * beam search, the occlusion prune, the union merge, finalize, the graph
 * hash and query search (paper Sec. 3, Prop. 1).  It exists to check the
 * HIP library; only tests, the smoke entry point and the CPU-baseline leg of
 * the benchmark may load it.  It shares no source with the HIP library.
 *
 * Precision modes:
 *   prec = 0  float32 data: squared L2 / cosine in the declared order "C16"
 *             (16 strided partial sums, explicit fused multiply-add, then a
 *             pairwise tree 8,4,2,1); uint8 data: exact integer squared L2.
 *   prec = 1  float64 arithmetic in natural order, used only to state the
 *             error of the float32 result.
 *
 * Every array is host memory owned by the caller.  Functions return 0 on
 * success and a negative code on bad arguments (no partial output then).
 */
#ifndef FGO_H
#define FGO_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FGO_NONE 0xFFFFFFFFu

enum { FGO_F32 = 0, FGO_U8 = 1 };
enum { FGO_L2 = 0, FGO_COSINE = 1 };

typedef struct {
  const void* x;      /* n rows of d elements, row stride `stride` bytes */
  int64_t n;
  int32_t d;
  int32_t dtype;      /* FGO_F32 or FGO_U8 */
  int32_t metric;     /* FGO_L2 or FGO_COSINE (f32 only) */
  int32_t prec;       /* 0 = declared float32 order / exact int, 1 = float64 */
  int64_t stride;     /* bytes between rows */
} fgo_data;

typedef struct {
  uint32_t T, ef_h, R;
  float alpha;
  uint32_t B;            /* B = 0 and B = 1 both mean one frozen block */
  uint32_t reprune_all;  /* 0: re-prune only rows with more than R candidates */
  uint32_t threads;      /* host threads for the parallel loops (>= 1) */
} fgo_params;

typedef struct {
  uint64_t scaffold_evals;
  uint64_t harvest_evals;   /* |visited| summed over all harvested points */
  uint64_t prune_evals;     /* lazy pair count of the harvest prunes */
  uint64_t finalize_evals;  /* candidate distances + prune pairs of finalize */
  uint64_t expansions;
  double t_scaffold, t_harvest, t_merge, t_finalize;   /* seconds */
} fgo_counters;

/* --- primitives ---------------------------------------------------------- */
uint64_t fgo_splitmix64(uint64_t seed, uint64_t k);
int fgo_roots(uint64_t seed, int64_t n, uint32_t T, uint32_t* roots);
double fgo_dist(const fgo_data* D, int64_t i, int64_t j);
double fgo_dist_vec(const fgo_data* D, const void* q, int64_t j);
uint64_t fgo_fnv1a64(const void* bytes, size_t len);

/* --- scaffold ------------------------------------------------------------ */
/* One SAT tree rooted at `root`: parent[v] for every v (FGO_NONE at root). */
int fgo_sat_tree(const fgo_data* D, uint32_t root, uint32_t* parent,
                 uint64_t* evals);
/* Union of the T trees' parent-child edges, both directions, deduplicated,
 * rows sorted by id.  parents is T*n.  ids needs capacity 2*T*(n-1).
 * Returns nnz or a negative code. */
int64_t fgo_scaffold_csr(int64_t n, uint32_t T, const uint32_t* parents,
                         uint64_t* off, uint32_t* ids);

/* --- harvest ------------------------------------------------------------- */
/* Beam search of width ef over CSR (off, ids) from the T roots, for the
 * query row q (a data row when q_index >= 0, else the vector q).  Outputs:
 * final beam (ids, dists, count), expanded set E in expansion order,
 * visited set V in visit order.  Capacities must be >= n where unknown.
 * Returns |V| (the evaluation count). */
int64_t fgo_beam(const fgo_data* D, const void* q, int64_t q_index,
                 const uint64_t* off, const uint32_t* ids,
                 const uint32_t* roots, uint32_t T, uint32_t ef,
                 uint32_t* beam_ids, double* beam_d, uint32_t* beam_n,
                 uint32_t* E_ids, double* E_d, uint32_t* E_n,
                 uint32_t* V_ids, uint32_t* V_n);
/* Greedy occlusion prune of candidates (any order; sorted here by key) for
 * data point p.  Writes <= R ids in kept order.  Returns the count. */
int32_t fgo_prune(const fgo_data* D, int64_t p, const uint32_t* cand_ids,
                  const double* cand_d, uint32_t m, uint32_t R, float alpha,
                  uint32_t* out, uint64_t* pair_evals);
/* Harvest every p with p mod max(B,1) == b (in the order given by `order`
 * when not NULL, a permutation of those points).  rows is n*R (FGO_NONE
 * padding), cnt is n.  Writes only the rows of block b. */
int fgo_harvest_block(const fgo_data* D, const uint64_t* off,
                      const uint32_t* ids, const uint32_t* roots,
                      const fgo_params* P, uint32_t b, const uint32_t* order,
                      int64_t order_len, uint32_t* rows, uint32_t* cnt,
                      fgo_counters* C);
/* S_{b+1} = S_b u {(p,u),(u,p) : u in rows[p], p in block b}; rows sorted by
 * id, deduplicated.  Returns nnz or -2 when cap is too small. */
int64_t fgo_merge_block(int64_t n, const uint64_t* off, const uint32_t* ids,
                        const uint32_t* rows, const uint32_t* cnt, uint32_t R,
                        uint32_t B, uint32_t b, uint64_t* off_out,
                        uint32_t* ids_out, uint64_t cap);
/* Symmetrise and re-prune: G[p] = prune(A[p] u {u : p in A[u]}) when that
 * set exceeds R (or always with reprune_all), else the set sorted by key. */
int fgo_finalize(const fgo_data* D, const uint32_t* rows, const uint32_t* cnt,
                 const fgo_params* P, uint32_t* g_nbrs, uint32_t* g_cnt,
                 fgo_counters* C);
uint64_t fgo_graph_hash(int64_t n, uint32_t R, uint32_t T,
                        const uint32_t* g_nbrs, const uint32_t* g_cnt,
                        const uint32_t* parent0, const uint32_t* roots);
/* Whole build: roots from seed, T SAT trees, B blocks, finalize.
 * parent0 (n) is tree 0's parent array (the spine), roots (T). */
int fgo_build_graph(const fgo_data* D, uint64_t seed, const fgo_params* P,
                    uint32_t* g_nbrs, uint32_t* g_cnt, uint32_t* parent0,
                    uint32_t* roots, fgo_counters* C, uint64_t* hash);

/* --- search and ground truth ------------------------------------------- */
/* Beam of width L over G u spine from the roots; first k entries. Queries are
 * nq contiguous rows of d elements of the data's dtype. */
int fgo_search(const fgo_data* D, const uint32_t* g_nbrs, const uint32_t* g_cnt,
               uint32_t R, const uint32_t* parent0, const uint32_t* roots,
               uint32_t T, const void* queries, int64_t nq, uint32_t k,
               uint32_t L, uint32_t threads, uint32_t* out_ids,
               double* out_d, uint32_t* out_evals);
int fgo_knn_brute(const fgo_data* D, const void* queries, int64_t nq,
                  uint32_t k, uint32_t threads, uint32_t* out_ids,
                  double* out_d);

#ifdef __cplusplus
}
#endif
#endif
