// fg_internal.h -- host-side declarations shared by the library's sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fgraft.h"
#include "fg_beam.h"

namespace fg {

// Bounds of the beam kernels' on-chip structures.
constexpr int kHashSlotsMax = 4096;      // LDS visited table per wave (largest variant)
// Expanded entries per harvest search: up to half the visited table's
// slots are sorted and pruned on chip, longer sets in the slot's device
// buffer (kEcap keys, then kEcap bits of live flags); beyond kEcap the
// search fails with a capacity error.
constexpr int kEcap = 8192;
constexpr int kSpillCap = 8192;          // ids remembered for clearing the spill bitset
constexpr int kMaxWaveSlots = 4096;      // persistent grid bound (wave slots)
constexpr int kMaxEfHarvest = 256;
constexpr int kMaxEfSearch = 512;

void set_error(const std::string& msg);

// Data shape as the kernels see it.
struct Shape {
  const uint8_t* x;
  int64_t stride, n;
  int d, dk, Q;  // dk = DistKind, Q = 16-byte chunks per row
};
bool make_shape(const fg_data* d, Shape* s);  // validates, sets error

// Beam kernels (fg_beam.hip).  beam_grid() gives the persistent grid;
// hslots is the requested on-chip visited-table size (2048 or 4096),
// beam_table_slots() the size the chosen kernel really uses.
// screen (ScreenKind) selects the screened harvest kernels (fg_beam_sbf16.hip,
// fg_beam_sfp8.hip: float32 rows of more than 16 chunks only).
// lanes (0 = the default shape) asks for another lanes-per-row shape of the
// plain harvest kernels (fg_beam_lanes.hip) where one exists.
int beam_table_slots(int ef, bool search, int hslots, int nch);
int beam_chunks_per_lane(const Shape& s, int lanes = 0);  // NCH of the kernel the dispatch picks
int beam_grid(const Shape& s, int ef, bool search, int hslots, int screen = SCR_NONE, int waves_per_cu = 0,
              int lanes = 0);
hipError_t launch_beam(const Shape& s, BeamArgs& a, bool search, int grid, int hslots, hipStream_t st,
                       int screen = SCR_NONE, int lanes = 0);
// The lanes-per-row alternative for rows of Q chunks (false: none).
bool lanes_variant(int dk, int Q, int lanes, int* L, int* nch);
void* pick_lanes(int dk, int Q, int ef, int hslots, int lanes);
// The plain harvest kernels with a 512- or 1024-slot table (fg_beam_small.hip).
void* pick_small(int dk, int Q, int ef, int hslots);
int num_cus_host();  // compute units of the current device
// The harvest kernels with the visit log (fg_beam_log.hip): selected by
// passing kBeamLog as `screen` to beam_grid / launch_beam (4096 slots).
constexpr int kBeamLog = 16;
void* pick_log(int dk, int Q, int ef);
void* pick_screen_bf16(int dk, int Q, int ef, int hslots);
void* pick_screen_fp8(int dk, int Q, int ef, int hslots);
void* pick_screen_int8(int dk, int Q, int ef, int hslots);

// Narrow copies for the screened harvest (fg_screen.hip): row stride in
// bytes (whole 128-byte lines), the offset of each row's 16-byte trailer
// (float err, norm, sinv, 0) after its codes, and the copy with its per-row
// error norm, norm and fp8 factor.
int64_t screen_stride(int d, int screen);
int64_t screen_tail(int d, int screen);
// xs may be NULL (no plain copy), and so may err, norm and sinv (the
// trailers hold them); sp (bfloat16 only, may be NULL) receives the
// interleaved hi/lo split, rows split_stride(d) bytes apart.
int64_t split_stride(int d);
// |x_i|^2 of every float32 row (fg_sat.hip).
hipError_t row_sq_norms(const Shape& s, float* out, hipStream_t st);
hipError_t make_screen(const Shape& s, int screen, uint8_t* xs, float* err, float* norm, float* sinv,
                       hipStream_t st, uint8_t* sp = nullptr);

// Small utilities (fg_graph.hip).
hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t st);
// Batched builds (fg_graph.hip): rows of the shared graph back to one
// instance's ids.
hipError_t localize_graph(const uint32_t* nbrs, const uint32_t* cnt, const uint32_t* parent0, int64_t ni, int R,
                          int64_t o, uint32_t* out_nbrs, uint32_t* out_cnt, uint32_t* out_parent, hipStream_t st);
hipError_t fill_u64(uint64_t* p, uint64_t v, int64_t count, hipStream_t st);
// The points of every block b (p mod B == b) in the order they appear in
// `order` (len ids: every id of [0, n) but `last`, or with last =
// 0xFFFFFFFF any set of distinct ids), block after block into sched (n
// entries; block b starts at the sum of the earlier blocks' sizes in
// [0, n)); `last` closes its block; slots no id fills keep their contents.
// flags (len) and pos (len + 1) are scratch.
hipError_t block_schedule(const uint32_t* order, int64_t len, int64_t n, uint32_t B, uint32_t last,
                          uint32_t* sched, uint32_t* flags, uint64_t* pos, void* scratch, hipStream_t st);
// rank[order[i]] = i for i < len, rank[last] = len (order: every id but last;
// last = 0xFFFFFFFF: no last).
hipError_t rank_of(const uint32_t* order, int64_t len, uint32_t last, uint32_t* rank, hipStream_t st);
// The substrate's ids with each id's rank beside it (pairs[e] = (ids[e],
// rank[ids[e]]) for e < off[n], off[n] read on the device), for the
// harvest's rank-indexed visited bitsets.
hipError_t csr_rank_pairs(int64_t n, const uint64_t* off, const uint32_t* ids, const uint32_t* rank, uint2* pairs,
                          hipStream_t st);
// Exclusive scan of `count` uint32 values into uint64 offsets (count+1 entries).
size_t scan_scratch_bytes(int64_t count);
hipError_t exclusive_scan_u32_u64(const uint32_t* in, uint64_t* out, int64_t count,
                                  void* scratch, hipStream_t st);

// Edge lists from harvested rows (fg_graph.hip): points p = b + i*B.
hipError_t edges_count(int64_t n, const uint32_t* rows, const uint32_t* cnt, int R, int64_t b, int64_t B,
                       int64_t nitems, bool own, bool rev, uint32_t* deg, hipStream_t st);
hipError_t edges_scatter(int64_t n, const uint32_t* rows, const uint32_t* cnt, int R, int64_t b, int64_t B,
                         int64_t nitems, bool own, bool rev, const uint64_t* off, uint32_t* cursor,
                         uint32_t* out, hipStream_t st);
// Rows whose additions exceed the on-chip bound are listed in big[] (count
// in *nbig) and finished by merge_big_rows() (host-planned segmented sort)
// or by merge_big_rows_dev() (device only, for captured streams; scratch
// holds 2 * additions entries).
hipError_t merge_rows(int64_t n, const uint64_t* off, const uint32_t* ids, const uint64_t* addoff,
                      const uint32_t* addbuf, uint32_t* tmp, uint32_t* newlen, uint32_t* big, uint32_t* nbig,
                      uint32_t* mid, uint32_t* nmid, hipStream_t st);
struct KSeg {
  uint64_t start;
  uint32_t len, pad;
};
struct KTile {
  uint32_t seg, off;
};
constexpr int kSegTilePositions = 256;
// Sort each segment of keys (keys2: same-size scratch).  hsegs mirrors dsegs.
hipError_t segsort_u64(uint64_t* keys, uint64_t* keys2, const KSeg* dsegs, const std::vector<KSeg>& hsegs,
                       KTile* dtiles, size_t tile_cap, hipStream_t st);
hipError_t merge_big_rows_dev(const uint32_t* big, const uint32_t* nbig, const uint64_t* off, const uint32_t* ids,
                              const uint64_t* addoff, const uint32_t* addbuf, uint32_t* scratch, uint32_t* tmp,
                              uint32_t* newlen, hipStream_t st);
hipError_t merge_big_rows(const uint32_t* big, uint32_t nbig, const uint64_t* off, const uint32_t* ids,
                          const uint64_t* addoff, const uint32_t* addbuf, uint32_t* tmp, uint32_t* newlen,
                          KSeg* dsegs, KTile* dtiles, size_t tile_cap, uint64_t* keys, uint64_t* keys2,
                          uint32_t* uni, hipStream_t st);
hipError_t compact_rows(int64_t n, const uint64_t* off, const uint64_t* addoff, const uint32_t* tmp,
                        const uint64_t* noff, uint32_t* out, hipStream_t st);
hipError_t search_graph(int64_t n, int R, const uint32_t* nbrs, const uint32_t* cnt,
                        const uint32_t* parent0, uint32_t* deg, uint64_t* off, uint32_t* out,
                        void* scan_scratch, hipStream_t st);

// Finalize rows (fg_finalize.hip): symmetrised candidates -> sorted / pruned.
struct FinalizeArgs {
  RowSet X;
  int64_t n;
  int R;
  float alpha;
  int reprune_all;
  const uint32_t* rows;
  const uint32_t* cnt;
  const uint64_t* revoff;
  const uint32_t* rev;
  uint32_t* g_nbrs;
  uint32_t* g_cnt;
  unsigned long long* counters;  // [0] candidate distances, [1] prune pairs, [2] exact rechecks
  int* status;
  uint32_t* big;   // points whose candidates exceed the on-chip bound
  uint32_t* nbig;  // their count (device, zero on entry)
  uint32_t* mid;   // points for the second on-chip tier
  uint32_t* nmid;  // their count (device, zero on entry)
  int d;
  float* gram;     // float32 rows longer than 256 elements: Gram scratch per block (or NULL)
  GramSplit split; // the Gram tiles from the bfloat16 split (p NULL: from the rows)
  const float* norm;  // |x_i|^2 per row for the Gram prune (NULL: no Gram prune)
  // batched builds: each point's instance and the chunks of that instance's
  // own rows (NULL: every row has X.Q chunks)
  const uint16_t* inst_of;
  const int* inst_q;
  // the points in processing order (a permutation of [0, n); NULL: id order)
  const uint32_t* order;
};
struct FinalizeBig {
  KSeg* segs;
  KTile* tiles;
  size_t tile_cap;
  uint64_t* keys;
  uint64_t* keys2;
};
hipError_t launch_finalize(int dk, int Q, const FinalizeArgs& a, const FinalizeBig& big, hipStream_t st);

// Query search (fg_api.hip), shared by fg_search and fg_search_noalloc.
// Its device scratch: a 4096-byte control block (queue, counters, status),
// the G u spine CSR (n + 1 offsets, R n + 2 n + 1 ids), n degree words, the
// scan's scratch, `grid` visited bitsets of spill_words words each and
// `grid` spill lists of spill_cap ids each.
struct SearchScratch {
  void* ctl;
  uint64_t* sgoff;
  uint32_t* sgids;
  uint32_t* deg;
  void* scan;
  uint32_t* bits;
  int64_t spill_words;
  uint32_t* slist;
  int spill_cap;
};
fg_status check_search(const fg_data* data, const fg_graph* graph, const void* queries_dev, int64_t nq, uint32_t k,
                       uint32_t L, const uint32_t* out_ids_dev, const void* out_dists_dev, Shape* s);
// Clears the control block and the first `grid` bitsets, builds the CSR and
// launches the search kernel with `grid` wave slots.  Asynchronous.
fg_status search_run(const Shape& s, const fg_graph* graph, const void* queries_dev, int64_t nq, uint32_t k,
                     uint32_t L, uint32_t* out_ids, void* out_d, uint32_t* out_evals, const SearchScratch& w,
                     int grid, hipStream_t st);

// Leaf k-NN on MFMA (fg_dense.hip).
size_t leaf_knn_ws_bytes(int64_t n, int d);
hipError_t leaf_knn(const Shape& s, int S, int R, bool bf16, void* ws, uint32_t* out_ids, float* out_d,
                    hipStream_t st);

}  // namespace fg
