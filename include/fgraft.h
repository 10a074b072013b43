/*
 * fgraft.h -- C-ABI of the MI355X FGraft harvest library (libfgraft.so).
 *
 * FGraft (Sec. 3 of the paper) builds a navigable graph in B synchronous
 * blocks.  S_0, the scaffold, is the union of the edges of T spatial-
 * approximation trees, symmetrised.  For b = 0..B-1 every point p with
 * p mod B == b beam-searches S_b with itself as the query (width ef_h, from
 * the tree roots); the vertices the search expands are occlusion-pruned to
 * at most R neighbours (slack alpha) into p's own row; then
 * S_{b+1} = S_b u {(p,u),(u,p) : u in A[p], p in block b}.  The final graph
 * is the harvested rows symmetrised and re-pruned, plus the tree-0 spine.
 * By Prop. 1 the graph is a function of (data, seed, params, B) alone.
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev are device (HIP) memory; everything else is host
 *     memory.  Every buffer is owned by the caller; the library keeps no
 *     allocation between calls.
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = default stream).
 *     Entry points that return data-dependent sizes or counters synchronise
 *     that stream before returning; they say so.
 *   - `ws_dev` / `ws_bytes` is caller-allocated device scratch of at least
 *     fg_workspace_size() bytes (256-byte aligned).  Two calls may run
 *     concurrently only with distinct workspaces.
 *   - Ids are uint32 (n < 2^32 - 1); 0xFFFFFFFF pads unused row slots.
 *     CSR offsets are uint64.
 *   - Errors: argument errors return before any work is enqueued; a HIP
 *     failure returns FG_EHIP; a device-side capacity overflow returns
 *     FG_ECAPACITY.  fg_last_error() gives a message for the calling thread.
 *
 * Distances (Sec. 3 does not fix the precision; the declared order makes the
 * graph reproducible bit for bit):
 *   FG_U8 + FG_L2SQ   exact int32 sum of squared differences;
 *   FG_F32 + FG_L2SQ  float32, element chunk q of 4 goes to partial q mod 16,
 *                     fused multiply-add per element, partials combined
 *                     pairwise with offsets 8, 4, 2, 1;
 *   FG_F32 + FG_COSINE  1 - <x, y> in the same order (rows pre-normalised).
 * Candidates are totally ordered by (distance, id).
 */
#ifndef FGRAFT_H
#define FGRAFT_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FG_OK = 0,
  FG_EINVAL = -1,        /* bad argument */
  FG_ENOMEM = -2,        /* workspace too small */
  FG_EHIP = -3,          /* a HIP runtime call failed */
  FG_ECAPACITY = -4,     /* a device-side bounded buffer overflowed */
  FG_EUNSUPPORTED = -5   /* a shape the library has no kernel for */
} fg_status;

typedef enum { FG_F32 = 0, FG_U8 = 1 } fg_dtype;
typedef enum { FG_L2SQ = 0, FG_COSINE = 1 } fg_metric;

/* Mixed-precision forms (Sec. 5.3: an adaptive evaluation costs the bytes
 * of one row).  FG_F32 data with d > 64 only.  A narrow copy of the rows
 * (made in the workspace by the harvest entry points) gives cheap values with
 * proven error margins; a decision the margin settles is taken from the
 * cheap value, every other one from the exact float32 distance, so graphs,
 * counts and hashes are those of FG_SCREEN_NONE.
 *   search screen (FG_SCREEN_BF16, FG_SCREEN_FP8E4M3, FG_SCREEN_INT8): a
 *     new candidate that provably cannot enter the full beam is not
 *     evaluated exactly;
 *   split prune tiles (FG_SCREEN_BF16, FG_SCREEN_BF16_PRUNE; 256 < d <= 1024):
 *     the occlusion prune's Gram tiles (harvest and finalize) come from a
 *     bfloat16 split x = hi + lo + e, |e| <= 2^-16 |x| elementwise, three
 *     bfloat16 matrix-core products per 16 elements instead of eight float32
 *     ones. */
typedef enum {
  FG_SCREEN_NONE = 0,
  FG_SCREEN_BF16 = 1,       /* bfloat16 copy, round to nearest even: search screen and split prune tiles */
  FG_SCREEN_FP8E4M3 = 2,    /* fp8 e4m3 (OCP) copy with a power-of-two scale per row: search screen */
  FG_SCREEN_BF16_PRUNE = 3, /* split prune tiles only (256 < d <= 1024) */
  FG_SCREEN_INT8 = 4        /* int8 codes of x / s, s = max|x_i| / 127 per row: search screen; for
                               FG_COSINE the candidate's dot product with the point's own codes is
                               exact in integers */
} fg_screen;

/* Row-major data in device memory.  FG_F32 needs d % 4 == 0; FG_U8 needs
 * d % 16 == 0 and FG_L2SQ.  row_stride_bytes is a multiple of 16 and at
 * least d * element size. */
typedef struct {
  const void* x_dev;
  int64_t n;
  int32_t d;
  int32_t dtype;   /* fg_dtype */
  int32_t metric;  /* fg_metric */
  int32_t reserved;
  int64_t row_stride_bytes;
} fg_data;

/* Build parameters (Sec. 3).  B = 0 and B = 1 both mean one frozen block
 * (frozen Graft).  reprune_all = 0 re-prunes in finalize only the rows whose
 * symmetrised candidate set exceeds R; 1 re-prunes every row.
 * beam_table_slots is a tuning knob that never changes the graph: the size
 * of each harvest search's on-chip visited table, 512, 1024, 2048 or 4096
 * (0 = 4096 for FG_F32 rows of more than 256 elements or ef_h > 128, else
 * 1024 for rows of at most 16 bytes per lane -- uint8 d <= 256 or FG_F32
 * d <= 64 -- and for the screened harvest (FG_SCREEN_BF16, _FP8E4M3, _INT8) of
 * rows of at most 256 elements, and 2048 for the rest; ef_h > 128 always
 * uses 4096; 512 and 1024 apply to the unscreened harvest with ef_h <= 128
 * and the library's lanes per row, and 1024 (also for a 512 request) to
 * the screened harvest with ef_h <= 128 of rows of at most 256 elements;
 * otherwise 2048 is used).  Smaller tables let more searches run
 * per compute unit; a search whose visits outgrow its table continues in a
 * device bitset.  A search's
 * expanded set is sorted and pruned on chip up to half the table's slots and
 * in the workspace beyond; a search that expands 8192 vertices or more fails
 * the call with FG_ECAPACITY (Sec. 3 bounds nothing: the bound is this
 * library's).
 * screen is an fg_screen; it never changes the graph either.  waves_per_cu
 * caps the resident harvest searches per compute unit (0 = as many as fit);
 * another knob that never changes the graph (see fg_autotune).  So is
 * lanes_per_row: how many lanes of a wave share one row's gather in the
 * plain harvest (0 = the library's choice: 8 for rows of at most 128
 * bytes, else 16; 4 for rows of at most 128 bytes and 8 for rows of
 * 129..512 bytes hold more rows in flight; any other combination uses the
 * library's choice).  The declared summation order gives the same bits for
 * every lane count. */
typedef struct {
  uint32_t T;
  uint32_t ef_h;
  uint32_t R;
  float alpha;
  uint32_t B;
  uint32_t reprune_all;
  uint32_t beam_table_slots;
  uint32_t screen;
  uint32_t waves_per_cu;
  uint32_t lanes_per_row;
} fg_params;

/* Compressed rows in device memory: row v is ids_dev[off_dev[v] ..
 * off_dev[v+1]), sorted by id, no repeats.  `cap` is the capacity of ids_dev
 * (elements); `nnz` is a host copy of off_dev[n]. */
typedef struct {
  uint64_t* off_dev;
  uint32_t* ids_dev;
  int64_t n;
  uint64_t nnz;
  uint64_t cap;
} fg_csr;

/* The final graph, device memory: nbrs_dev is n x R (row p sorted by
 * (d(p,.), id), 0xFFFFFFFF padded), cnt_dev[p] its length, spine_parent_dev
 * tree 0's parent array (0xFFFFFFFF at its root), roots_dev the T roots. */
typedef struct {
  uint32_t* nbrs_dev;
  uint32_t* cnt_dev;
  uint32_t* spine_parent_dev;
  uint32_t* roots_dev;
  int64_t n;
  uint32_t R;
  uint32_t T;
} fg_graph;

/* Work counters (Sec. 2, "Cost model": every distance evaluation counts).
 * harvest_evals is the number of vertices each harvest search visited
 * (= evaluated), summed over points; prune_evals the pair distances the
 * greedy prune needs (each later live candidate tested against each kept
 * one until it dies). */
typedef struct {
  uint64_t scaffold_evals;
  uint64_t harvest_evals;
  uint64_t prune_evals;
  uint64_t expansions;
  uint64_t finalize_evals;
  uint64_t spilled_queries; /* searches whose visited set left on-chip memory */
  uint64_t screen_rejected; /* harvest evaluations settled by the screen alone (included in harvest_evals) */
  uint64_t prune_rechecks;  /* pair tests of the harvest and finalize prunes (counted in
                               prune_evals / finalize_evals) that, for float32 rows longer than
                               256 elements, the matrix-core distance's margin left open and an
                               exact recomputation settled */
} fg_counters;

/* Per-phase device time (HIP events on `stream`), milliseconds. */
typedef struct {
  float scaffold_ms;
  float harvest_ms;      /* sum over blocks */
  float merge_ms;        /* sum over blocks */
  float finalize_ms;
  float screen_ms;       /* making the narrow copy (screened builds) */
  float block_harvest_ms[64];
  uint64_t block_evals[64];
  uint32_t nblocks;
} fg_timings;

/* Bytes of device scratch needed by every entry point below for this data
 * shape and these parameters (one workspace serves all of them).  FG_F32
 * rows of 257..1024 elements add 8 GiB of Gram-prune scratch (2048 wave
 * slots of 1024 x 1024 floats) and a float per row; a screened harvest adds
 * the narrow copy and three floats per row, the split tiles 4d bytes per
 * row. */
size_t fg_workspace_size(const fg_data* data, const fg_params* params);

/* Keyed roots (Prop. 1, "keyed randomness"): root of tree t is the first
 * draw splitmix64(seed, t * 2^32 + j) mod n, j = 0, 1, ..., not already a
 * root, where splitmix64(seed, k) is output k of the SplitMix64 stream
 * seeded with `seed`.  roots is a host array of T entries. */
fg_status fg_roots(uint64_t seed, int64_t n, uint32_t T, uint32_t* roots);

/* Scaffold S_0 (Sec. 1 and Sec. 3): T classic spatial-approximation trees
 * rooted at roots_dev (distinct, device), the union of their parent-child
 * edges in both directions.  Writes S0 (its off/ids buffers must hold n+1
 * and 2*T*(n-1) entries; sets S0->nnz) and, when tree_parent_dev is not
 * NULL, the T x n parent arrays.  Synchronises `stream`. */
fg_status fg_build_scaffold(const fg_data* data, const uint32_t* roots_dev,
                            uint32_t T, fg_csr* S0, uint32_t* tree_parent_dev,
                            void* ws_dev, size_t ws_bytes, void* stream,
                            fg_counters* counters);

/* Harvest of block b (Sec. 3): for every p with p mod max(B,1) == b, the
 * beam search of width ef_h over Sb from the T roots (roots_dev), then the
 * occlusion prune of the expanded set minus p into rows_dev[p*R ..] (n x R)
 * and row_cnt_dev[p].  Other rows are not touched.  counters (optional)
 * makes the call synchronise `stream`.  With params->screen set, the call
 * first (re)makes the narrow copy of the data in the workspace. */
fg_status fg_harvest_block(const fg_data* data, const fg_csr* Sb,
                           const uint32_t* roots_dev, const fg_params* params,
                           uint32_t b, uint32_t* rows_dev,
                           uint32_t* row_cnt_dev, void* ws_dev, size_t ws_bytes,
                           void* stream, fg_counters* counters);

/* Union merge (Sec. 3): Sb1 = Sb u {(p,u),(u,p) : u in rows[p], p in block
 * b}, rows sorted by id, deduplicated.  Sb1 must not alias Sb; its capacity
 * must hold the result.  Synchronises `stream` (sets Sb1->nnz). */
fg_status fg_merge_block(const fg_csr* Sb, const uint32_t* rows_dev,
                         const uint32_t* row_cnt_dev, const fg_params* params,
                         uint32_t b, fg_csr* Sb1, void* ws_dev, size_t ws_bytes,
                         void* stream);

/* Finalize (Sec. 3): for every p, Cand = A[p] u {u : p in A[u]}; when |Cand|
 * exceeds R (or reprune_all) the occlusion prune of Cand, else Cand sorted
 * by (d(p,.), id).  Writes graph->nbrs_dev and graph->cnt_dev only. */
fg_status fg_finalize(const fg_data* data, const uint32_t* rows_dev,
                      const uint32_t* row_cnt_dev, const fg_params* params,
                      fg_graph* graph, void* ws_dev, size_t ws_bytes,
                      void* stream, fg_counters* counters);

/* The whole build (Sec. 3): roots from seed, scaffold, B x (harvest, merge),
 * finalize.  Fills every array of `out` (its n, R, T must match).
 * Synchronises `stream`.  timings (optional) records per-phase device time. */
fg_status fg_build_graph(const fg_data* data, uint64_t seed,
                         const fg_params* params, fg_graph* out, void* ws_dev,
                         size_t ws_bytes, void* stream, fg_counters* counters,
                         fg_timings* timings);

/* Visit log of the harvest searches, for the lockstep-density measurement
 * (Sec. 5.5, Tab. 6: the density of a block of points is the sum of their
 * visited-set sizes over the block size times the size of the union).
 * slot_dev (n entries, device) selects the points: slot_dev[p] in
 * [0, nslots) logs p's own harvest search (in block p mod max(B,1), over
 * S_b) into that slot; any other value logs nothing.  Per slot: ids_dev[slot
 * * cap ..] receives the ids the search visits, in visit order (the roots in
 * order, then each expanded row's unvisited ids in row order), the first cap
 * of them; len_dev[slot] the total; marks_dev[slot * FG_LOG_MARKS + e] the
 * visit count after the roots (e = 0) and after expansion e (e = 1..16; after
 * the search's last expansion, its total).  Two points must not share a
 * slot.  All device memory, caller-owned. */
#define FG_LOG_MARKS 17
typedef struct {
  const int32_t* slot_dev;
  uint32_t nslots;
  uint32_t cap;
  uint32_t* ids_dev;
  uint32_t* len_dev;
  uint32_t* marks_dev;
} fg_visit_log;

/* fg_build_graph that also fills a visit log (the same graph, counters and
 * timings; its harvest always uses the 4096-slot visited table).  screen
 * must be FG_SCREEN_NONE (FG_EUNSUPPORTED otherwise). */
fg_status fg_build_graph_log(const fg_data* data, uint64_t seed,
                             const fg_params* params, fg_graph* out,
                             void* ws_dev, size_t ws_bytes, void* stream,
                             fg_counters* counters, fg_timings* timings,
                             const fg_visit_log* log);

/* Batched builds: count independent instances, each exactly the graph
 * fg_build_graph would give it (same hash), built together so that one
 * harvest launch per block serves every instance (uneven beam lengths and
 * small instances keep the whole device busy).  Instances share dtype,
 * metric, T, R, alpha, B, reprune_all and the tuning knobs of params[0]; n,
 * d, ef_h and the seed may differ; screen must be FG_SCREEN_NONE.  outs[i]
 * is shaped like instance i.  flags: FG_BATCH_HIPGRAPH captures the B
 * harvests and merges into one HIP graph (on a stream of the library's own,
 * ordered after and before `stream`) and replays it once; merges then
 * finish rows with more than 2048 additions on the device alone.
 * FG_BATCH_AUTOTUNE replaces params[0]'s lanes_per_row, beam_table_slots
 * and waves_per_cu by the fastest candidates timed on this batch's own
 * harvest launch (block 0 of every instance over S_0, best of two; the
 * choice is kept per batch shape in host memory for later calls); no
 * graph changes.  Synchronises `stream`.  The workspace must hold
 * fg_batched_workspace_size() bytes (0 = invalid arguments). */
#define FG_BATCH_HIPGRAPH 1
#define FG_BATCH_AUTOTUNE 2
size_t fg_batched_workspace_size(const fg_data* const* data,
                                 const fg_params* const* params, uint32_t count);
fg_status fg_build_graph_batched(const fg_data* const* data,
                                 const fg_params* const* params,
                                 const uint64_t* seeds, uint32_t count,
                                 fg_graph* const* outs, void* ws_dev,
                                 size_t ws_bytes, void* stream,
                                 int flags, fg_counters* counters);

/* Query search (Sec. 2, "quality"): beam of width L over G u spine from the
 * roots for nq query rows (queries_dev, contiguous rows of d elements of the
 * data's dtype); writes the first k entries per query: ids (nq x k), their
 * distances (float32 for FG_F32, uint32 for FG_U8) and the evaluation count
 * per query (optional).  Needs L >= k. */
fg_status fg_search(const fg_data* data, const fg_graph* graph,
                    const void* queries_dev, int64_t nq, uint32_t k,
                    uint32_t L, uint32_t* out_ids_dev, void* out_dists_dev,
                    uint32_t* out_evals_dev, void* ws_dev, size_t ws_bytes,
                    void* stream);

/* fg_search for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as fg_search, without a workspace: the
 * kernels' scratch (a control block, the G u spine CSR, per-search visited
 * bitsets) lives in a fixed array of fg_search_noalloc_scratch_bytes()
 * bytes (64 MiB) that the library holds on each GPU it runs on until the
 * process ends.  The call allocates nothing and does not synchronise; its
 * device address is looked up on the first call on each device.
 * Limit: 4096 + 8 (n + 1) + 4 (R n + 2 n + 1) + 4 n bytes (each rounded up
 * to 256) plus, for at least one search per compute unit, 4 ceil(n / 32) +
 * 8192 bytes per search must fit; otherwise FG_EINVAL with a message and
 * nothing enqueued (n = 100,000 with R = 64 fits).  Every call on one GPU
 * uses that GPU's one array: calls that overlap in time on the same GPU
 * (other streams, other threads) race and give wrong results.  Each call
 * clears what must start at zero on `stream` itself. */
size_t fg_search_noalloc_scratch_bytes(void);
fg_status fg_search_noalloc(const fg_data* data, const fg_graph* graph,
                            const void* queries_dev, int64_t nq, uint32_t k,
                            uint32_t L, uint32_t* out_ids_dev,
                            void* out_dists_dev, uint32_t* out_evals_dev,
                            void* stream);

/* FNV-1a-64 over the graph's little-endian byte image: n (u64), R, T (u32),
 * then per point its count and ids, then the spine parents, then the roots.
 * Copies the graph to the host; synchronises `stream`. */
fg_status fg_graph_hash(const fg_graph* graph, void* stream, uint64_t* out);

/* The blocked dense side of the random-access wall (Sec. 5.4, Tab. 5): for
 * every point, its R nearest other points (squared L2, ties by id) inside
 * its leaf of leaf_size consecutive ids ([l*leaf_size, (l+1)*leaf_size)),
 * all leaf_size^2 distances computed as |x|^2 + |y|^2 - 2<x,y> with the inner
 * products on matrix cores: float32 operands (use_bf16 = 0) or operands
 * rounded to bfloat16 (use_bf16 = 1, norms of the rounded rows), float32
 * accumulation.  FG_F32 + FG_L2SQ data only; leaf_size a multiple of 128;
 * 1 <= R <= 64.  Writes out_ids_dev / out_dists_dev (n x R, rows sorted,
 * 0xFFFFFFFF / +inf padded when a leaf has fewer than R + 1 points).
 * Asynchronous on `stream`. */
size_t fg_leaf_knn_workspace_size(const fg_data* data);
fg_status fg_leaf_knn(const fg_data* data, uint32_t leaf_size, uint32_t R,
                      int use_bf16, uint32_t* out_ids_dev, float* out_dists_dev,
                      void* ws_dev, size_t ws_bytes, void* stream);

/* The narrow copy a screened harvest reads (fg_screen), for inspection:
 * row i of the data as bfloat16 (round to nearest even), as fp8 e4m3 (OCP)
 * codes of x * 2^k, k the largest integer with max|x_i| * 2^k <= 448, or as
 * int8 codes rint(x / s) clamped to [-127, 127], s = fl(max|x_i| / 127), in
 * the data's element order, rows fg_screen_row_bytes(d, screen) bytes apart
 * (a whole number of 128-byte lines).  A row holds the codes (bfloat16: 2d
 * bytes rounded up to a multiple of 32, pad bytes written as zero; fp8 and
 * int8: d rounded up to a multiple of 16, pad bytes not written), then a
 * 16-byte trailer of four floats (err, norm, sinv, 0) equal to the values
 * below, then padding (zero for bfloat16, not written otherwise).
 * err_dev[i] >= |x^_i - x_i| and norm_dev[i] >= |x_i| (float32 sums of
 * scaled squares raised by their rounding bound), sinv_dev[i] = 2^-k (fp8),
 * s (int8), 1 (bfloat16), where x^_i is the copy read back (fp8: code * 2^-k;
 * int8: fl(code * s), each element's product rounded once).  FG_F32 data
 * with d > 64 only.  Asynchronous on `stream`. */
int64_t fg_screen_row_bytes(int32_t d, uint32_t screen);
fg_status fg_screen_copy(const fg_data* data, uint32_t screen, void* xs_dev,
                         float* err_dev, float* norm_dev, float* sinv_dev,
                         void* stream);

/* Autotuning of the harvest's knobs (none changes the graph): the
 * visited-table size (beam_table_slots 512 / 1024 / 2048 / 4096, where ef_h and
 * the row size allow), the resident searches per compute unit
 * (waves_per_cu) and the lanes that share one row (lanes_per_row: the
 * library's shape and the other one where it exists).  On the first
 * min(n, 50000) rows it builds a scaffold, then times block 0's harvest
 * for each candidate (best of two) and writes the fastest into *tuned (a
 * copy of *params with those three fields set).  With cache_path != NULL the
 * result is looked up in / appended to that text file, one line per
 * (dtype, metric, row chunks, ef_h, R, T, B, log2 n).  The workspace is the
 * one fg_workspace_size gives for data and params.  Synchronises `stream`. */
fg_status fg_autotune(const fg_data* data, const fg_params* params,
                      const char* cache_path, void* ws_dev, size_t ws_bytes,
                      void* stream, fg_params* tuned);

/* Message of the last failed call on this thread ("" if none). */
/* Device-side status of the last call made with workspace ws_dev, for
 * workspaces sized by fg_workspace_size() or fg_batched_workspace_size()
 * (each entry point taking one clears the status when it starts; not for
 * the fg_leaf_knn workspace): synchronises `stream`, then returns
 * FG_ECAPACITY if that call overflowed a bounded device buffer (the expanded
 * set of a search), else FG_OK.  fg_harvest_block and fg_finalize without
 * counters return before their kernels finish; this call reports what they
 * found (Sec. 3 bounds nothing: the capacities are this library's). */
fg_status fg_sync_status(void* ws_dev, void* stream);

const char* fg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
