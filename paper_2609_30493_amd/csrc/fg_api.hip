// fg_api.hip -- the C-ABI of libfgraft.so: validation, workspace layout and
// the orchestration of the kernels (Sec. 3 of the paper).
#include <math.h>
#include <string.h>

#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <cstdio>
#include <cstring>

#include "fg_internal.h"
#include "fg_sat.h"

namespace fg {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }

bool make_shape(const fg_data* d, Shape* s) {
  if (!d || !d->x_dev) return set_error("data or data->x_dev is NULL"), false;
  if (d->n < 1 || d->n >= (int64_t)FG_NONE) return set_error("n out of range"), false;
  if (d->d < 1) return set_error("d must be positive"), false;
  int64_t esz;
  if (d->dtype == FG_F32) {
    if (d->d % 4) return set_error("float32 rows need d % 4 == 0 (pad with zeros)"), false;
    if (d->metric != FG_L2SQ && d->metric != FG_COSINE) return set_error("bad metric"), false;
    esz = 4;
    s->dk = d->metric == FG_COSINE ? F32COS : F32L2;
    s->Q = d->d / 4;
  } else if (d->dtype == FG_U8) {
    if (d->d % 16) return set_error("uint8 rows need d % 16 == 0"), false;
    if (d->metric != FG_L2SQ) return set_error("uint8 data supports squared L2 only"), false;
    esz = 1;
    s->dk = U8L2;
    s->Q = d->d / 16;
  } else {
    return set_error("bad dtype"), false;
  }
  if (d->row_stride_bytes < esz * d->d || d->row_stride_bytes % 16)
    return set_error("row_stride_bytes must be >= d * elem and a multiple of 16"), false;
  if (reinterpret_cast<uintptr_t>(d->x_dev) % 16) return set_error("x_dev must be 16-byte aligned"), false;
  s->x = static_cast<const uint8_t*>(d->x_dev);
  s->stride = d->row_stride_bytes;
  s->n = d->n;
  s->d = d->d;
  return true;
}

namespace {

bool check_params(const fg_params* p, int64_t n, bool need_ef = true) {
  if (!p) return set_error("params is NULL"), false;
  if (p->T < 1 || (int64_t)p->T > n) return set_error("need 1 <= T <= n"), false;
  if (p->T > 64) return set_error("T > 64 is not supported"), false;
  if (need_ef && (p->ef_h < 1 || p->ef_h > (uint32_t)kMaxEfHarvest))
    return set_error("need 1 <= ef_h <= 256"), false;
  if (p->R < 1 || p->R > 1024) return set_error("need 1 <= R <= 1024"), false;
  if (!isfinite(p->alpha) || p->alpha < 1.0f) return set_error("alpha must be finite and >= 1"), false;
  if (p->beam_table_slots != 0 && p->beam_table_slots != 512 && p->beam_table_slots != 1024 &&
      p->beam_table_slots != 2048 && p->beam_table_slots != 4096)
    return set_error("beam_table_slots must be 0, 512, 1024, 2048 or 4096"), false;
  if (p->screen > FG_SCREEN_INT8) return set_error("screen must be an fg_screen"), false;
  if (p->waves_per_cu > 64) return set_error("waves_per_cu must be 0..64"), false;
  if (p->lanes_per_row != 0 && p->lanes_per_row != 4 && p->lanes_per_row != 8 && p->lanes_per_row != 16)
    return set_error("lanes_per_row must be 0, 4, 8 or 16"), false;
  return true;
}

// The screened kernels exist for float32 rows of 17..256 chunks, the split
// Gram tiles for 65..256 chunks.
bool check_screen(const fg_params* p, const Shape& s) {
  if (p->screen == FG_SCREEN_NONE) return true;
  if (s.dk == U8L2) return set_error("screening applies to FG_F32 data only"), false;
  if (s.Q <= 16 || s.Q > 256) return set_error("screening needs 64 < d <= 1024"), false;
  if (p->screen == FG_SCREEN_BF16_PRUNE && s.Q <= 64)
    return set_error("FG_SCREEN_BF16_PRUNE needs 256 < d <= 1024"), false;
  return true;
}

// The narrow copy's kind, and whether the prune's Gram tiles come from the
// bfloat16 split (float32 rows of 257..1024 elements).
int copy_kind(uint32_t screen) {
  return screen == FG_SCREEN_FP8E4M3 ? SCR_FP8 : screen == FG_SCREEN_INT8 ? SCR_INT8 : SCR_BF16;
}
bool split_tiles(uint32_t screen, int d) {
  return (screen == FG_SCREEN_BF16 || screen == FG_SCREEN_BF16_PRUNE) && d > 256 && d <= 1024 && d % 4 == 0;
}
// The search-side screen's kernel variant (none for FG_SCREEN_BF16_PRUNE).
int search_screen(uint32_t screen) {
  return screen == FG_SCREEN_BF16 ? SCR_BF16
         : screen == FG_SCREEN_FP8E4M3 ? SCR_FP8
         : screen == FG_SCREEN_INT8 ? SCR_INT8
                                    : SCR_NONE;
}

uint32_t b_eff(const fg_params* p) { return p->B > 1 ? p->B : 1; }

// Visited-table size for the harvest: the caller's choice, else by row
// shape, from full-size sweeps of every size.  Rows of one chunk per lane
// with ef_h <= 128 take 1024 (four searches per SIMD; the 1M x 128 uint8
// harvest: 528 ms, against 523 at 512 and 559 at 2048); other rows with
// ef_h <= 128 take 2048 (the 1,183,514 x 100 cosine harvest: 3.65 s, against
// 3.78 at 512 and 3.69 at 4096); rows of more than 64 chunks (nch 16) take
// 4096: their registers already hold residency at two searches per SIMD and
// the larger table keeps searches off the device bitset (the 10^6 x 960
// harvest: 1.88 s, against 1.98 at 2048); ef_h > 128 takes 4096.
// The screened forms' kernels for rows of 2..4 chunks per lane take 1024
// (the 1,183,514 x 100 cosine harvest with the fp8 screen: 2.69 s against
// 2.86 at 2048; at three searches per SIMD the smaller table lets a twelfth
// search per compute unit fit, and the screen's rounds are latency-bound).
int table_request(const fg_params* p, int nch = 1) {
  if (p->beam_table_slots == 512 || p->beam_table_slots == 1024 || p->beam_table_slots == 2048 ||
      p->beam_table_slots == 4096)
    return (int)p->beam_table_slots;
  if (nch >= 16 || p->ef_h > 128) return 4096;
  if (search_screen(p->screen) != SCR_NONE) return nch <= 4 ? 1024 : 2048;
  return nch == 1 ? 1024 : 2048;
}

// ---------------------------------------------------------------- workspace
// One layout serves every entry point for a given (n, T, R, B).
struct WsMap {
  size_t ctl, bits, slist, ebuf;            // beam kernels
  size_t deg, cursor, newlen, aoff, noff, zoff, addbuf, tmp, scan;  // edge lists / merges
  size_t keys, keys2, uni, big, mid, ksegs, ktiles;  // rows too large for on-chip sorting
  size_t ktile_cap;
  size_t sgoff, sgids;                      // search graph
  size_t off[2], ids[2], rows, cnt, tparent, roots;  // the whole build
  size_t sat;
  size_t xs;                                // screened harvest (last: only they depend on d)
  size_t xsp;                               // the bfloat16 split (interleaved hi/lo)
  int64_t xsp_stride;
  size_t sched;                             // every block's points in scaffold order
  size_t rank;                              // each id's position in that order
  size_t gram;                              // Gram-tile prune scratch (float32, d > 256)
  size_t norm;                              // |x_i|^2 per row for it
  size_t pairs;                             // the substrate's (id, rank) pairs
  int64_t xs_stride;
  SatWs satw;
  size_t total;
  int64_t spill_words;
  uint64_t csr_cap, tmp_cap, add_cap;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WsMap ws_map(int64_t n, const fg_params* p, int d = 0) {
  WsMap m{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  const uint64_t T = p ? p->T : 1, R = p ? p->R : 1;
  const uint64_t un = (uint64_t)n;
  m.spill_words = (n + 31) / 32;
  m.csr_cap = 2 * T * (un - 1) + 2 * R * un + 1;
  m.add_cap = 2 * R * un + 2 * T * un + 1;
  m.tmp_cap = m.csr_cap + m.add_cap;
  m.ctl = take(4096);
  m.bits = take((size_t)kMaxWaveSlots * m.spill_words * 4);
  m.slist = take((size_t)kMaxWaveSlots * kSpillCap * 4);
  m.ebuf = take((size_t)kMaxWaveSlots * (kEcap + kEcap / 64) * 8);
  m.deg = take(un * 4);
  m.cursor = take(un * 4);
  m.newlen = take(un * 4);
  m.aoff = take((un + 1) * 8);
  m.noff = take((un + 1) * 8);
  m.zoff = take((un + 1) * 8);
  m.addbuf = take(m.add_cap * 4);
  m.tmp = take(m.tmp_cap * 4);
  m.scan = take(scan_scratch_bytes((int64_t)un + 1));
  m.keys = take(m.add_cap * 8);
  m.keys2 = take(m.add_cap * 8);
  m.uni = take(m.add_cap * 4);
  m.big = take(un * 4);
  m.mid = take(un * 4);
  m.ksegs = take(un * sizeof(KSeg));
  m.ktile_cap = m.add_cap / kSegTilePositions + un + 64;
  m.ktiles = take(m.ktile_cap * sizeof(KTile));
  m.sgoff = take((un + 1) * 8);
  m.sgids = take((R * un + 2 * un + 1) * 4);
  for (int i = 0; i < 2; i++) {
    m.off[i] = take((un + 1) * 8);
    m.ids[i] = take(m.csr_cap * 4);
  }
  m.rows = take(R * un * 4);
  m.cnt = take(un * 4);
  m.tparent = take(T * un * 4);
  m.roots = take(64 * 4);
  m.sched = take(un * 4);
  m.rank = take(un * 4);
  sat_workspace_bytes(n, (uint32_t)T, &m.satw);
  m.sat = take(m.satw.total);
  if (p && d > 256 && d % 4 == 0 && d <= 1024) {
    m.gram = take((size_t)kGramSlots * kGramMax * kGramMax * 4);
    m.norm = take(un * 4);
  }
  // rows of 68..256 float32 elements (2..4 chunks per lane) index the
  // harvest's visited bitsets by rank: the substrate's ids paired with ranks
  if (p && d >= 68 && d <= 256 && d % 4 == 0) m.pairs = take(m.csr_cap * 8);

  if (p && p->screen && d > 0) {
    m.xs_stride = screen_stride(d, copy_kind(p->screen));
    if (search_screen(p->screen) != SCR_NONE) m.xs = take(un * (uint64_t)m.xs_stride);
    if (split_tiles(p->screen, d)) {
      m.xsp_stride = split_stride(d);
      m.xsp = take(un * (uint64_t)m.xsp_stride);
    }
  }
  m.total = o;
  return m;
}

// ctl region: [0] queue, [1..4] beam counters, [8] status (int)
struct Ctl {
  unsigned long long queue;
  unsigned long long counters[6];    // beam: evals, expansions, prune pairs, spilled, screen-rejected, rechecks
  unsigned long long fin[3];         // finalize: candidate distances, prune pairs, exact rechecks
  uint32_t nbig, nmid;               // rows sent to the big-row paths / finalize's second tier
  int status;                        // 1 expanded-set overflow
  unsigned int xq[8];                // the ordered harvest's per-XCD queues
};

hipError_t g_last_hip = hipSuccess;
#define FG_HIP(call)                                                           \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      g_last_hip = e_;                                                         \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " + #call); \
      return FG_EHIP;                                                          \
    }                                                                          \
  } while (0)

bool check_ws(void* ws, size_t ws_bytes, const WsMap& m) {
  if (!ws) return set_error("workspace is NULL"), false;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return set_error("workspace must be 256-byte aligned"), false;
  if (ws_bytes < m.total) return set_error("workspace too small (see fg_workspace_size)"), false;
  return true;
}

char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

// Launch the harvest of block b.  The spill bitsets must be zero on entry
// (they are left zero on exit).
// Instances of a batched build sharing one id space (see fg_build_graph_batched).
struct BatchInfo {
  const uint16_t* inst_of;
  const uint32_t* inst_roots;
  const int* inst_ef;
  int ef_max;
  const int* inst_q;  // 16-byte chunks of each instance's own rows
};

fg_status harvest_launch(const Shape& s, const uint64_t* off, const uint32_t* ids,
                         const uint32_t* roots, const fg_params* P, uint32_t b, uint32_t* rows,
                         uint32_t* cnt, void* ws, const WsMap& m, hipStream_t st,
                         const BatchInfo* bi = nullptr, const uint32_t* order = nullptr,
                         const uint32_t* rank = nullptr, const fg_visit_log* log = nullptr) {
  const uint32_t Be = b_eff(P);
  int64_t nitems = s.n > (int64_t)b ? (s.n - (int64_t)b + Be - 1) / Be : 0;
  Ctl* ctl = reinterpret_cast<Ctl*>(at(ws, m.ctl));
  FG_HIP(fill_u64(reinterpret_cast<uint64_t*>(&ctl->queue), 0, 1, st));
  if (nitems == 0) return FG_OK;
  const int ef = bi ? bi->ef_max : (int)P->ef_h;
  // the logging kernels exist with the 4096-slot table only, the other
  // lanes-per-row shapes for the plain harvest only (none of these knobs
  // changes the graph)
  const int screen = log ? kBeamLog : search_screen(P->screen);
  const int lanes = screen == SCR_NONE ? (int)P->lanes_per_row : 0;
  const int nch = beam_chunks_per_lane(s, lanes);
  int hslots = log ? 4096 : beam_table_slots(ef, false, table_request(P, nch), nch);
  // the small tables exist for the plain kernels of the library's shape;
  // the screened kernels have 1024 for rows of up to 4 chunks per lane
  int Lv = 0, nv = 0;
  if (screen != SCR_NONE && screen != kBeamLog) {
    if (hslots < 1024) hslots = 1024;
    if (hslots == 1024 && nch > 4) hslots = 2048;
  } else if (hslots < 2048 && lanes_variant(s.dk, s.Q, lanes, &Lv, &nv)) {
    hslots = 2048;
  }
  int grid = beam_grid(s, ef, false, hslots, screen, (int)P->waves_per_cu, lanes);
  if (grid <= 0) return set_error("no beam kernel for this row size / ef_h"), FG_EUNSUPPORTED;
  BeamArgs a{};
  a.x = s.x;
  a.stride = s.stride;
  a.n = s.n;
  a.Q = s.Q;
  a.off = off;
  a.ids = ids;
  a.roots = roots;
  a.T = (int)P->T;
  a.ef = ef;
  a.R = (int)P->R;
  a.alpha = P->alpha;
  a.b = b;
  a.B = Be;
  a.rows = rows;
  a.cnt = cnt;
  a.nitems = nitems;
  a.order = order;
  a.rank = rank;
  if (rank && m.pairs && !bi && nch >= 2 && nch <= 4 && s.dk != U8L2) {
    uint2* pairs = reinterpret_cast<uint2*>(at(ws, m.pairs));
    FG_HIP(csr_rank_pairs(s.n, off, ids, rank, pairs, st));
    a.idr = pairs;
  }
  a.queue = &ctl->queue;
  if (order) {
    FG_HIP(fill_u32(ctl->xq, 0, 8, st));
    a.xqueue = ctl->xq;
  }
  a.Ebuf = reinterpret_cast<uint64_t*>(at(ws, m.ebuf));
  a.Ecap = kEcap;
  a.spill_bits = reinterpret_cast<uint32_t*>(at(ws, m.bits));
  a.spill_words = m.spill_words;
  a.spill_list = reinterpret_cast<uint32_t*>(at(ws, m.slist));
  a.spill_cap = kSpillCap;
  a.counters = ctl->counters;
  a.status = &ctl->status;
  a.d = s.d;
  if (m.gram && s.dk != U8L2 && s.Q > 64) {
    a.gram = reinterpret_cast<float*>(at(ws, m.gram));
    a.norm = reinterpret_cast<const float*>(at(ws, m.norm));
    grid = grid < kGramSlots ? grid : kGramSlots;
    if (m.xsp) a.split = GramSplit{reinterpret_cast<const uint8_t*>(at(ws, m.xsp)), m.xsp_stride};
  }
  if (bi) {
    a.inst_of = bi->inst_of;
    a.inst_roots = bi->inst_roots;
    a.inst_ef = bi->inst_ef;
    a.inst_q = bi->inst_q;
  }
  if (log) {
    a.log_slot = log->slot_dev;
    a.log_ids = log->ids_dev;
    a.log_len = log->len_dev;
    a.log_marks = log->marks_dev;
    a.log_cap = log->cap;
    a.log_nslots = (int)log->nslots;
  } else if (screen) {
    a.xs = reinterpret_cast<const uint8_t*>(at(ws, m.xs));
    a.xs_stride = m.xs_stride;
    a.xs_tail = screen_tail(s.d, copy_kind(P->screen));
  }
  FG_HIP(launch_beam(s, a, false, grid, hslots, st, screen, lanes));
  return FG_OK;
}

// Per-build preparation of the harvest's inputs beyond the rows: the row
// norms of the Gram prune, then the narrow copy of a screened harvest.
fg_status screen_launch(const Shape& s, const fg_params* P, void* ws, const WsMap& m, hipStream_t st) {
  if (m.norm && s.dk != U8L2) FG_HIP(row_sq_norms(s, reinterpret_cast<float*>(at(ws, m.norm)), st));
  if (!P->screen) return FG_OK;
  FG_HIP(make_screen(s, copy_kind(P->screen), m.xs ? reinterpret_cast<uint8_t*>(at(ws, m.xs)) : nullptr, nullptr,
                     nullptr, nullptr, st, m.xsp ? reinterpret_cast<uint8_t*>(at(ws, m.xsp)) : nullptr));
  return FG_OK;
}

fg_status reset_ctl(void* ws, const WsMap& m, hipStream_t st) {
  FG_HIP(fill_u64(reinterpret_cast<uint64_t*>(at(ws, m.ctl)), 0, 4096 / 8, st));
  return FG_OK;
}

fg_status read_ctl(void* ws, const WsMap& m, hipStream_t st, Ctl* out) {
  FG_HIP(hipMemcpyAsync(out, at(ws, m.ctl), sizeof(Ctl), hipMemcpyDeviceToHost, st));
  FG_HIP(hipStreamSynchronize(st));
  return FG_OK;
}

// Per-row union of sorted old rows with unsorted additions (see merge_rows);
// rows with too many additions for one wave's LDS take the global path.
//
// device_only: nothing waits for the host (for captured streams); big rows
// take the device-side path.
fg_status merge_rows_all(int64_t n, const uint64_t* off0, const uint32_t* ids0, const uint64_t* aoff,
                         const uint32_t* addbuf, uint32_t* tmp, uint32_t* newlen, void* ws, const WsMap& m,
                         hipStream_t st, bool device_only = false) {
  Ctl* ctl = reinterpret_cast<Ctl*>(at(ws, m.ctl));
  uint32_t* big = reinterpret_cast<uint32_t*>(at(ws, m.big));
  FG_HIP(fill_u32(&ctl->nbig, 0, 2, st));  // nbig and nmid
  FG_HIP(merge_rows(n, off0, ids0, aoff, addbuf, tmp, newlen, big, &ctl->nbig,
                    reinterpret_cast<uint32_t*>(at(ws, m.mid)), &ctl->nmid, st));
  if (device_only) {
    FG_HIP(merge_big_rows_dev(big, &ctl->nbig, off0, ids0, aoff, addbuf,
                              reinterpret_cast<uint32_t*>(at(ws, m.keys2)), tmp, newlen, st));
    return FG_OK;
  }
  uint32_t nbig = 0;
  FG_HIP(hipMemcpyAsync(&nbig, &ctl->nbig, 4, hipMemcpyDeviceToHost, st));
  FG_HIP(hipStreamSynchronize(st));
  FG_HIP(merge_big_rows(big, nbig, off0, ids0, aoff, addbuf, tmp, newlen,
                        reinterpret_cast<KSeg*>(at(ws, m.ksegs)), reinterpret_cast<KTile*>(at(ws, m.ktiles)),
                        m.ktile_cap, reinterpret_cast<uint64_t*>(at(ws, m.keys)),
                        reinterpret_cast<uint64_t*>(at(ws, m.keys2)), reinterpret_cast<uint32_t*>(at(ws, m.uni)),
                        st));
  return FG_OK;
}

// S_{b+1} = S_b u rows of block b (both directions), sorted and deduplicated
// per row.  Leaves the new offsets in off1 (off1[n] = nnz) and the ids in
// ids1; the caller guarantees the capacity.
fg_status merge_launch(int64_t n, const uint64_t* off0, const uint32_t* ids0, const uint32_t* rows,
                       const uint32_t* cnt, int R, uint32_t b, uint32_t Be, uint64_t* off1,
                       uint32_t* ids1, void* ws, const WsMap& m, hipStream_t st,
                       bool device_only = false) {
  int64_t nitems = n > (int64_t)b ? (n - (int64_t)b + Be - 1) / Be : 0;
  uint32_t* deg = reinterpret_cast<uint32_t*>(at(ws, m.deg));
  uint32_t* cursor = reinterpret_cast<uint32_t*>(at(ws, m.cursor));
  uint32_t* newlen = reinterpret_cast<uint32_t*>(at(ws, m.newlen));
  uint64_t* aoff = reinterpret_cast<uint64_t*>(at(ws, m.aoff));
  uint32_t* addbuf = reinterpret_cast<uint32_t*>(at(ws, m.addbuf));
  uint32_t* tmp = reinterpret_cast<uint32_t*>(at(ws, m.tmp));
  void* scan = at(ws, m.scan);
  Ctl* ctl = reinterpret_cast<Ctl*>(at(ws, m.ctl));
  FG_HIP(fill_u32(deg, 0, n, st));
  FG_HIP(edges_count(n, rows, cnt, R, b, Be, nitems, true, true, deg, st));
  FG_HIP(exclusive_scan_u32_u64(deg, aoff, n, scan, st));
  FG_HIP(fill_u32(cursor, 0, n, st));
  FG_HIP(edges_scatter(n, rows, cnt, R, b, Be, nitems, true, true, aoff, cursor, addbuf, st));
  fg_status r = merge_rows_all(n, off0, ids0, aoff, addbuf, tmp, newlen, ws, m, st, device_only);
  if (r) return r;
  FG_HIP(exclusive_scan_u32_u64(newlen, off1, n, scan, st));
  FG_HIP(compact_rows(n, off0, aoff, tmp, off1, ids1, st));
  return FG_OK;
}

// S_0 from the T parent arrays: both directions of every tree edge, sorted
// and deduplicated per row.
fg_status scaffold_csr_launch(int64_t n, uint32_t T, const uint32_t* tparent, uint64_t* off,
                              uint32_t* ids, void* ws, const WsMap& m, hipStream_t st) {
  uint32_t* deg = reinterpret_cast<uint32_t*>(at(ws, m.deg));
  uint32_t* cursor = reinterpret_cast<uint32_t*>(at(ws, m.cursor));
  uint32_t* newlen = reinterpret_cast<uint32_t*>(at(ws, m.newlen));
  uint64_t* aoff = reinterpret_cast<uint64_t*>(at(ws, m.aoff));
  uint64_t* zoff = reinterpret_cast<uint64_t*>(at(ws, m.zoff));
  uint32_t* addbuf = reinterpret_cast<uint32_t*>(at(ws, m.addbuf));
  uint32_t* tmp = reinterpret_cast<uint32_t*>(at(ws, m.tmp));
  void* scan = at(ws, m.scan);
  Ctl* ctl = reinterpret_cast<Ctl*>(at(ws, m.ctl));
  FG_HIP(tree_edges_csr(n, T, tparent, deg, aoff, cursor, addbuf, st, scan));
  FG_HIP(fill_u64(zoff, 0, n + 1, st));
  fg_status r = merge_rows_all(n, zoff, addbuf, aoff, addbuf, tmp, newlen, ws, m, st);
  if (r) return r;
  FG_HIP(exclusive_scan_u32_u64(newlen, off, n, scan, st));
  FG_HIP(compact_rows(n, zoff, aoff, tmp, off, ids, st));
  return FG_OK;
}

fg_status finalize_launch(const Shape& s, const uint32_t* rows, const uint32_t* cnt, const fg_params* P,
                          uint32_t* g_nbrs, uint32_t* g_cnt, void* ws, const WsMap& m, hipStream_t st,
                          const BatchInfo* bi = nullptr, const uint32_t* order = nullptr) {
  const int64_t n = s.n;
  const int R = (int)P->R;
  uint32_t* deg = reinterpret_cast<uint32_t*>(at(ws, m.deg));
  uint32_t* cursor = reinterpret_cast<uint32_t*>(at(ws, m.cursor));
  uint64_t* aoff = reinterpret_cast<uint64_t*>(at(ws, m.aoff));
  uint32_t* addbuf = reinterpret_cast<uint32_t*>(at(ws, m.addbuf));
  void* scan = at(ws, m.scan);
  Ctl* ctl = reinterpret_cast<Ctl*>(at(ws, m.ctl));
  FG_HIP(fill_u32(deg, 0, n, st));
  FG_HIP(edges_count(n, rows, cnt, R, 0, 1, n, false, true, deg, st));
  FG_HIP(exclusive_scan_u32_u64(deg, aoff, n, scan, st));
  FG_HIP(fill_u32(cursor, 0, n, st));
  FG_HIP(edges_scatter(n, rows, cnt, R, 0, 1, n, false, true, aoff, cursor, addbuf, st));
  FinalizeArgs f{};
  f.X = RowSet{s.x, s.stride, s.Q};
  f.n = n;
  f.R = R;
  f.alpha = P->alpha;
  f.reprune_all = P->reprune_all ? 1 : 0;
  f.rows = rows;
  f.cnt = cnt;
  f.revoff = aoff;
  f.rev = addbuf;
  f.g_nbrs = g_nbrs;
  f.g_cnt = g_cnt;
  f.counters = ctl->fin;
  f.d = s.d;
  f.gram = (m.gram && s.dk != U8L2 && s.Q > 64) ? reinterpret_cast<float*>(at(ws, m.gram)) : nullptr;
  f.norm = f.gram ? reinterpret_cast<const float*>(at(ws, m.norm)) : nullptr;
  if (bi) {
    f.inst_of = bi->inst_of;
    f.inst_q = bi->inst_q;
  }
  f.order = order;
  if (f.gram && m.xsp) f.split = GramSplit{reinterpret_cast<const uint8_t*>(at(ws, m.xsp)), m.xsp_stride};
  f.status = &ctl->status;
  f.big = reinterpret_cast<uint32_t*>(at(ws, m.big));
  f.nbig = &ctl->nbig;
  f.mid = reinterpret_cast<uint32_t*>(at(ws, m.mid));
  f.nmid = &ctl->nmid;
  FG_HIP(fill_u32(&ctl->nbig, 0, 2, st));  // nbig and nmid
  FinalizeBig fb{reinterpret_cast<KSeg*>(at(ws, m.ksegs)), reinterpret_cast<KTile*>(at(ws, m.ktiles)), m.ktile_cap,
                 reinterpret_cast<uint64_t*>(at(ws, m.keys)), reinterpret_cast<uint64_t*>(at(ws, m.keys2))};
  FG_HIP(launch_finalize(s.dk, s.Q, f, fb, st));
  return FG_OK;
}

fg_status status_error(int status) {
  if (status & 1) return set_error("a search expanded more vertices than its capacity"), FG_ECAPACITY;
  if (status & 8) return set_error("the tree builder's segment list overflowed"), FG_ECAPACITY;
  return FG_OK;
}

// Tuned knobs of batch shapes already tuned in this process (host memory).
std::mutex g_tune_mu;
std::map<std::string, std::array<uint32_t, 3>> g_tuned;

bool tuned_lookup(const std::string& key, uint32_t out[3]) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tuned.find(key);
  if (it == g_tuned.end()) return false;
  for (int i = 0; i < 3; i++) out[i] = it->second[i];
  return true;
}

void tuned_store(const std::string& key, const uint32_t v[3]) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tuned[key] = {v[0], v[1], v[2]};
}

uint64_t splitmix64(uint64_t seed, uint64_t k) {
  // Output k of the SplitMix64 stream (Steele, Lea and Flood 2014).
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

// The whole build (fg_build_graph, and fg_build_graph_log with a visit log).
fg_status build_graph_impl(const fg_data* data, uint64_t seed, const fg_params* params, fg_graph* out,
                           void* ws_dev, size_t ws_bytes, void* stream, fg_counters* counters,
                           fg_timings* timings, const fg_visit_log* log);

fg_status check_search(const fg_data* data, const fg_graph* graph, const void* queries_dev, int64_t nq, uint32_t k,
                       uint32_t L, const uint32_t* out_ids_dev, const void* out_dists_dev, Shape* s) {
  if (!make_shape(data, s)) return FG_EINVAL;
  if (!graph || !graph->nbrs_dev || !graph->cnt_dev || !graph->spine_parent_dev || !graph->roots_dev ||
      graph->n != s->n || graph->T < 1 || graph->T > 64 || graph->R < 1)
    return set_error("graph is incomplete or does not match the data"), FG_EINVAL;
  if (!queries_dev || nq < 0 || !out_ids_dev || !out_dists_dev)
    return set_error("queries and outputs are required"), FG_EINVAL;
  if (reinterpret_cast<uintptr_t>(queries_dev) % 16) return set_error("queries must be 16-byte aligned"), FG_EINVAL;
  if (k < 1 || L < k || L > (uint32_t)kMaxEfSearch) return set_error("need 1 <= k <= L <= 512"), FG_EINVAL;
  return FG_OK;
}

fg_status search_run(const Shape& s, const fg_graph* graph, const void* queries_dev, int64_t nq, uint32_t k,
                     uint32_t L, uint32_t* out_ids, void* out_d, uint32_t* out_evals, const SearchScratch& w,
                     int grid, hipStream_t st) {
  Ctl* ctl = static_cast<Ctl*>(w.ctl);
  FG_HIP(fill_u64(reinterpret_cast<uint64_t*>(ctl), 0, 4096 / 8, st));
  FG_HIP(search_graph(s.n, (int)graph->R, graph->nbrs_dev, graph->cnt_dev, graph->spine_parent_dev, w.deg,
                      w.sgoff, w.sgids, w.scan, st));
  FG_HIP(fill_u32(w.bits, 0, (int64_t)grid * w.spill_words, st));
  BeamArgs a{};
  a.x = s.x;
  a.stride = s.stride;
  a.n = s.n;
  a.Q = s.Q;
  a.off = w.sgoff;
  a.ids = w.sgids;
  a.roots = graph->roots_dev;
  a.T = (int)graph->T;
  a.ef = (int)L;
  a.queries = static_cast<const uint8_t*>(queries_dev);
  a.qstride = (int64_t)s.d * (s.dk == U8L2 ? 1 : 4);
  a.k = (int)k;
  a.out_ids = out_ids;
  a.out_d = out_d;
  a.out_evals = out_evals;
  a.nitems = nq;
  a.queue = &ctl->queue;
  a.Ebuf = nullptr;  // a search keeps no expanded list
  a.Ecap = 0;
  a.spill_bits = w.bits;
  a.spill_words = w.spill_words;
  a.spill_list = w.slist;
  a.spill_cap = w.spill_cap;
  a.counters = ctl->counters;
  a.status = &ctl->status;
  FG_HIP(launch_beam(s, a, true, grid, 4096, st));
  return FG_OK;
}

}  // namespace fg

using namespace fg;

extern "C" {

const char* fg_last_error(void) { return g_err.c_str(); }

size_t fg_leaf_knn_workspace_size(const fg_data* data) {
  if (!data || data->n < 1 || data->d < 1) return 0;
  return leaf_knn_ws_bytes(data->n, data->d);
}

fg_status fg_leaf_knn(const fg_data* data, uint32_t leaf_size, uint32_t R, int use_bf16, uint32_t* out_ids_dev,
                      float* out_dists_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  Shape s;
  if (!make_shape(data, &s)) return FG_EINVAL;
  if (data->dtype != FG_F32 || data->metric != FG_L2SQ)
    return set_error("fg_leaf_knn takes float32 squared-L2 data"), FG_EUNSUPPORTED;
  if (leaf_size < 128 || leaf_size % 128 || leaf_size > 65536)
    return set_error("leaf_size must be a multiple of 128 in [128, 65536]"), FG_EINVAL;
  if (R < 1 || R > 64) return set_error("need 1 <= R <= 64"), FG_EINVAL;
  if (!out_ids_dev || !out_dists_dev) return set_error("outputs are required"), FG_EINVAL;
  if (!ws_dev || ws_bytes < leaf_knn_ws_bytes(s.n, s.d) || reinterpret_cast<uintptr_t>(ws_dev) % 256)
    return set_error("workspace too small or misaligned (see fg_leaf_knn_workspace_size)"), FG_ENOMEM;
  FG_HIP(leaf_knn(s, (int)leaf_size, (int)R, use_bf16 != 0, ws_dev, out_ids_dev, out_dists_dev,
                  static_cast<hipStream_t>(stream)));
  return FG_OK;
}

int64_t fg_screen_row_bytes(int32_t d, uint32_t screen) {
  if (d < 1 || (screen != FG_SCREEN_BF16 && screen != FG_SCREEN_FP8E4M3 && screen != FG_SCREEN_INT8)) return 0;
  return screen_stride(d, copy_kind(screen));
}

fg_status fg_screen_copy(const fg_data* data, uint32_t screen, void* xs_dev, float* err_dev, float* norm_dev,
                         float* sinv_dev, void* stream) {
  Shape s;
  if (!make_shape(data, &s)) return FG_EINVAL;
  if (screen != FG_SCREEN_BF16 && screen != FG_SCREEN_FP8E4M3 && screen != FG_SCREEN_INT8)
    return set_error("screen must be FG_SCREEN_BF16, FG_SCREEN_FP8E4M3 or FG_SCREEN_INT8"), FG_EINVAL;
  fg_params P{};
  P.screen = screen;
  if (!check_screen(&P, s)) return FG_EUNSUPPORTED;
  if (!xs_dev || !err_dev || !norm_dev || !sinv_dev) return set_error("NULL output"), FG_EINVAL;
  if (reinterpret_cast<uintptr_t>(xs_dev) % 16) return set_error("xs_dev must be 16-byte aligned"), FG_EINVAL;
  FG_HIP(make_screen(s, copy_kind(screen), static_cast<uint8_t*>(xs_dev), err_dev, norm_dev, sinv_dev,
                     static_cast<hipStream_t>(stream)));
  return FG_OK;
}

fg_status fg_sync_status(void* ws_dev, void* stream) {
  if (!ws_dev) return set_error("ws_dev is NULL"), FG_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int status = 0;
  // the control block is the first region of every workspace layout
  FG_HIP(hipMemcpyAsync(&status, static_cast<char*>(ws_dev) + offsetof(Ctl, status), sizeof(int),
                        hipMemcpyDeviceToHost, st));
  FG_HIP(hipStreamSynchronize(st));
  return status_error(status);
}

size_t fg_workspace_size(const fg_data* data, const fg_params* params) {
  if (!data || data->n < 1) return 0;
  return ws_map(data->n, params, data->d).total;
}

fg_status fg_roots(uint64_t seed, int64_t n, uint32_t T, uint32_t* roots) {
  if (!roots || n < 1 || T < 1 || (int64_t)T > n) {
    set_error("fg_roots: need roots != NULL and 1 <= T <= n");
    return FG_EINVAL;
  }
  for (uint32_t t = 0; t < T; t++) {
    for (uint64_t j = 0;; j++) {
      uint32_t r = (uint32_t)(splitmix64(seed, ((uint64_t)t << 32) + j) % (uint64_t)n);
      bool dup = false;
      for (uint32_t u = 0; u < t; u++) dup = dup || roots[u] == r;
      if (!dup) {
        roots[t] = r;
        break;
      }
    }
  }
  return FG_OK;
}

fg_status fg_harvest_block(const fg_data* data, const fg_csr* Sb, const uint32_t* roots_dev,
                           const fg_params* params, uint32_t b, uint32_t* rows_dev,
                           uint32_t* row_cnt_dev, void* ws_dev, size_t ws_bytes, void* stream,
                           fg_counters* counters) {
  Shape s;
  if (!make_shape(data, &s)) return FG_EINVAL;
  if (!check_params(params, s.n)) return FG_EINVAL;
  if (!Sb || !Sb->off_dev || !Sb->ids_dev || Sb->n != s.n)
    return set_error("Sb must be a CSR over the data's n points"), FG_EINVAL;
  if (!roots_dev || !rows_dev || !row_cnt_dev) return set_error("NULL output or roots"), FG_EINVAL;
  if (b >= b_eff(params)) return set_error("need b < max(B, 1)"), FG_EINVAL;
  if (!check_screen(params, s)) return FG_EUNSUPPORTED;
  WsMap m = ws_map(s.n, params, s.d);
  if (!check_ws(ws_dev, ws_bytes, m)) return FG_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  fg_status r = reset_ctl(ws_dev, m, st);
  if (r) return r;
  r = screen_launch(s, params, ws_dev, m, st);
  if (r) return r;
  FG_HIP(fill_u32(reinterpret_cast<uint32_t*>(at(ws_dev, m.bits)), 0,
                  (int64_t)kMaxWaveSlots * m.spill_words, st));
  r = harvest_launch(s, Sb->off_dev, Sb->ids_dev, roots_dev, params, b, rows_dev, row_cnt_dev, ws_dev,
                     m, st);
  if (r) return r;
  if (counters) {
    Ctl c;
    r = read_ctl(ws_dev, m, st, &c);
    if (r) return r;
    counters->harvest_evals += c.counters[0];
    counters->expansions += c.counters[1];
    counters->prune_evals += c.counters[2];
    counters->spilled_queries += c.counters[3];
    counters->screen_rejected += c.counters[4];
    counters->prune_rechecks += c.counters[5] + c.fin[2];
    return status_error(c.status);
  }
  return FG_OK;
}

fg_status fg_build_scaffold(const fg_data* data, const uint32_t* roots_dev, uint32_t T, fg_csr* S0,
                            uint32_t* tree_parent_dev, void* ws_dev, size_t ws_bytes, void* stream,
                            fg_counters* counters) {
  Shape s;
  if (!make_shape(data, &s)) return FG_EINVAL;
  if (T < 1 || (int64_t)T > s.n || T > 64) return set_error("need 1 <= T <= min(n, 64)"), FG_EINVAL;
  if (!roots_dev || !S0 || !S0->off_dev || !S0->ids_dev || S0->n != s.n)
    return set_error("roots_dev and an S0 CSR over n points are required"), FG_EINVAL;
  if (S0->cap < 2ull * T * (uint64_t)(s.n - 1)) return set_error("S0->cap < 2*T*(n-1)"), FG_EINVAL;
  fg_params P{};
  P.T = T;
  P.ef_h = 1;
  P.R = 1;
  P.alpha = 1.0f;
  WsMap m = ws_map(s.n, &P);
  if (!check_ws(ws_dev, ws_bytes, m)) return FG_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  fg_status r = reset_ctl(ws_dev, m, st);
  if (r) return r;
  uint32_t* tparent = tree_parent_dev ? tree_parent_dev : reinterpret_cast<uint32_t*>(at(ws_dev, m.tparent));
  unsigned long long evals = 0;
  int status = 0;
  FG_HIP(sat_build(s, roots_dev, T, tparent, at(ws_dev, m.sat), m.satw, st, &evals, &status));
  if (status) return status_error(status);
  r = scaffold_csr_launch(s.n, T, tparent, S0->off_dev, S0->ids_dev, ws_dev, m, st);
  if (r) return r;
  Ctl c;
  r = read_ctl(ws_dev, m, st, &c);
  if (r) return r;
  FG_HIP(hipMemcpyAsync(&S0->nnz, S0->off_dev + s.n, 8, hipMemcpyDeviceToHost, st));
  FG_HIP(hipStreamSynchronize(st));
  if (counters) counters->scaffold_evals += evals;
  return status_error(c.status);
}

fg_status fg_merge_block(const fg_csr* Sb, const uint32_t* rows_dev, const uint32_t* row_cnt_dev,
                         const fg_params* params, uint32_t b, fg_csr* Sb1, void* ws_dev, size_t ws_bytes,
                         void* stream) {
  if (!Sb || !Sb1 || !Sb->off_dev || !Sb->ids_dev || !Sb1->off_dev || !Sb1->ids_dev)
    return set_error("Sb and Sb1 must be CSRs"), FG_EINVAL;
  if (Sb->n != Sb1->n || Sb->n < 1) return set_error("Sb and Sb1 must have the same n"), FG_EINVAL;
  if (Sb->ids_dev == Sb1->ids_dev || Sb->off_dev == Sb1->off_dev)
    return set_error("Sb1 must not alias Sb"), FG_EINVAL;
  if (!check_params(params, Sb->n, false)) return FG_EINVAL;
  if (!rows_dev || !row_cnt_dev) return set_error("rows and row counts are required"), FG_EINVAL;
  const uint32_t Be = b_eff(params);
  if (b >= Be) return set_error("need b < max(B, 1)"), FG_EINVAL;
  WsMap m = ws_map(Sb->n, params);
  if (!check_ws(ws_dev, ws_bytes, m)) return FG_ENOMEM;
  const int64_t n = Sb->n;
  int64_t nitems = n > (int64_t)b ? (n - (int64_t)b + Be - 1) / Be : 0;
  if (Sb->nnz + 2ull * params->R * (uint64_t)nitems > m.tmp_cap)
    return set_error("Sb->nnz exceeds what this workspace was sized for"), FG_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  fg_status r = reset_ctl(ws_dev, m, st);
  if (r) return r;
  uint64_t* noff = reinterpret_cast<uint64_t*>(at(ws_dev, m.noff));
  uint32_t* scratch_ids = reinterpret_cast<uint32_t*>(at(ws_dev, m.ids[0]));
  // merge into the workspace first, then check the caller's capacity
  r = merge_launch(n, Sb->off_dev, Sb->ids_dev, rows_dev, row_cnt_dev, (int)params->R, b, Be, noff,
                   scratch_ids, ws_dev, m, st);
  if (r) return r;
  uint64_t nnz = 0;
  Ctl c;
  FG_HIP(hipMemcpyAsync(&nnz, noff + n, 8, hipMemcpyDeviceToHost, st));
  r = read_ctl(ws_dev, m, st, &c);
  if (r) return r;
  if (c.status) return status_error(c.status);
  if (nnz > Sb1->cap) return set_error("Sb1->cap is too small for the merged substrate"), FG_ECAPACITY;
  FG_HIP(hipMemcpyAsync(Sb1->off_dev, noff, (n + 1) * 8, hipMemcpyDeviceToDevice, st));
  FG_HIP(hipMemcpyAsync(Sb1->ids_dev, scratch_ids, nnz * 4, hipMemcpyDeviceToDevice, st));
  FG_HIP(hipStreamSynchronize(st));
  Sb1->nnz = nnz;
  return FG_OK;
}

fg_status fg_finalize(const fg_data* data, const uint32_t* rows_dev, const uint32_t* row_cnt_dev,
                      const fg_params* params, fg_graph* graph, void* ws_dev, size_t ws_bytes, void* stream,
                      fg_counters* counters) {
  Shape s;
  if (!make_shape(data, &s)) return FG_EINVAL;
  if (!check_params(params, s.n, false)) return FG_EINVAL;
  if (!rows_dev || !row_cnt_dev || !graph || !graph->nbrs_dev || !graph->cnt_dev)
    return set_error("rows, counts and graph arrays are required"), FG_EINVAL;
  if (graph->n != s.n || graph->R != params->R) return set_error("graph shape mismatch"), FG_EINVAL;
  WsMap m = ws_map(s.n, params);
  if (!check_ws(ws_dev, ws_bytes, m)) return FG_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  fg_status r = reset_ctl(ws_dev, m, st);
  if (r) return r;
  r = finalize_launch(s, rows_dev, row_cnt_dev, params, graph->nbrs_dev, graph->cnt_dev, ws_dev, m, st);
  if (r) return r;
  if (counters) {
    Ctl c;
    r = read_ctl(ws_dev, m, st, &c);
    if (r) return r;
    counters->finalize_evals += c.fin[0] + c.fin[1];
    counters->prune_rechecks += c.fin[2];
    return status_error(c.status);
  }
  return FG_OK;
}

fg_status fg_search(const fg_data* data, const fg_graph* graph, const void* queries_dev, int64_t nq,
                    uint32_t k, uint32_t L, uint32_t* out_ids_dev, void* out_dists_dev,
                    uint32_t* out_evals_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  Shape s;
  fg_status r = check_search(data, graph, queries_dev, nq, k, L, out_ids_dev, out_dists_dev, &s);
  if (r) return r;
  fg_params P{};
  P.T = graph->T;
  P.R = graph->R;
  P.ef_h = 1;
  P.alpha = 1.0f;
  WsMap m = ws_map(s.n, &P);
  if (!check_ws(ws_dev, ws_bytes, m)) return FG_ENOMEM;
  if (nq == 0) return FG_OK;
  int grid = beam_grid(s, (int)L, true, 4096);
  if (grid <= 0) return set_error("no search kernel for this row size / L"), FG_EUNSUPPORTED;
  SearchScratch w{};
  w.ctl = at(ws_dev, m.ctl);
  w.sgoff = reinterpret_cast<uint64_t*>(at(ws_dev, m.sgoff));
  w.sgids = reinterpret_cast<uint32_t*>(at(ws_dev, m.sgids));
  w.deg = reinterpret_cast<uint32_t*>(at(ws_dev, m.deg));
  w.scan = at(ws_dev, m.scan);
  w.bits = reinterpret_cast<uint32_t*>(at(ws_dev, m.bits));
  w.spill_words = m.spill_words;
  w.slist = reinterpret_cast<uint32_t*>(at(ws_dev, m.slist));
  w.spill_cap = kSpillCap;
  return search_run(s, graph, queries_dev, nq, k, L, out_ids_dev, out_dists_dev, out_evals_dev, w, grid,
                    static_cast<hipStream_t>(stream));
}

fg_status fg_graph_hash(const fg_graph* graph, void* stream, uint64_t* out) {
  if (!graph || !out || !graph->nbrs_dev || !graph->cnt_dev || !graph->spine_parent_dev || !graph->roots_dev ||
      graph->n < 1)
    return set_error("incomplete graph"), FG_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = graph->n;
  const uint32_t R = graph->R, T = graph->T;
  std::vector<uint32_t> nb((size_t)n * R), cnt(n), par(n), roots(T);
  FG_HIP(hipMemcpyAsync(nb.data(), graph->nbrs_dev, nb.size() * 4, hipMemcpyDeviceToHost, st));
  FG_HIP(hipMemcpyAsync(cnt.data(), graph->cnt_dev, cnt.size() * 4, hipMemcpyDeviceToHost, st));
  FG_HIP(hipMemcpyAsync(par.data(), graph->spine_parent_dev, par.size() * 4, hipMemcpyDeviceToHost, st));
  FG_HIP(hipMemcpyAsync(roots.data(), graph->roots_dev, roots.size() * 4, hipMemcpyDeviceToHost, st));
  FG_HIP(hipStreamSynchronize(st));
  // FNV-1a, 64-bit, over the little-endian byte image.
  uint64_t h = 0xCBF29CE484222325ull;
  auto feed = [&](const void* p, size_t len) {
    const uint8_t* b = static_cast<const uint8_t*>(p);
    for (size_t i = 0; i < len; i++) {
      h ^= b[i];
      h *= 0x100000001B3ull;
    }
  };
  uint64_t n64 = (uint64_t)n;
  feed(&n64, 8);
  feed(&R, 4);
  feed(&T, 4);
  for (int64_t p = 0; p < n; p++) {
    if (cnt[p] > R) return set_error("row count above R"), FG_EINVAL;
    feed(&cnt[p], 4);
    feed(&nb[(size_t)p * R], (size_t)cnt[p] * 4);
  }
  feed(par.data(), par.size() * 4);
  feed(roots.data(), roots.size() * 4);
  *out = h;
  return FG_OK;
}

fg_status fg_build_graph(const fg_data* data, uint64_t seed, const fg_params* params, fg_graph* out,
                         void* ws_dev, size_t ws_bytes, void* stream, fg_counters* counters,
                         fg_timings* timings) {
  return build_graph_impl(data, seed, params, out, ws_dev, ws_bytes, stream, counters, timings, nullptr);
}

fg_status fg_build_graph_log(const fg_data* data, uint64_t seed, const fg_params* params, fg_graph* out,
                             void* ws_dev, size_t ws_bytes, void* stream, fg_counters* counters,
                             fg_timings* timings, const fg_visit_log* log) {
  if (!log || !log->slot_dev || !log->ids_dev || !log->len_dev || !log->marks_dev || log->nslots < 1 ||
      log->cap < 1 || log->nslots > (uint32_t)INT32_MAX)
    return set_error("fg_visit_log: slot, ids, len and marks arrays, nslots >= 1 and cap >= 1 are required"),
           FG_EINVAL;
  if (!params || params->screen != FG_SCREEN_NONE)
    return set_error("the visit log records the unscreened harvest (screen must be FG_SCREEN_NONE)"),
           FG_EUNSUPPORTED;
  return build_graph_impl(data, seed, params, out, ws_dev, ws_bytes, stream, counters, timings, log);
}

}  // extern "C"

namespace fg {
fg_status build_graph_impl(const fg_data* data, uint64_t seed, const fg_params* params, fg_graph* out,
                           void* ws_dev, size_t ws_bytes, void* stream, fg_counters* counters,
                           fg_timings* timings, const fg_visit_log* log) {
  Shape s;
  if (!make_shape(data, &s)) return FG_EINVAL;
  if (!check_params(params, s.n)) return FG_EINVAL;
  if (!out || !out->nbrs_dev || !out->cnt_dev || !out->spine_parent_dev || !out->roots_dev)
    return set_error("every array of the output graph is required"), FG_EINVAL;
  if (out->n != s.n || out->R != params->R || out->T != params->T)
    return set_error("output graph shape does not match data/params"), FG_EINVAL;
  const uint32_t Be = b_eff(params);
  if (timings && Be > 64) return set_error("timings record at most 64 blocks"), FG_EINVAL;
  if (!check_screen(params, s)) return FG_EUNSUPPORTED;
  WsMap m = ws_map(s.n, params, s.d);
  if (!check_ws(ws_dev, ws_bytes, m)) return FG_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = s.n;
  const uint32_t T = params->T, R = params->R;

  std::vector<hipEvent_t> ev;
  auto mark = [&]() -> fg_status {
    if (!timings) return FG_OK;
    hipEvent_t e;
    FG_HIP(hipEventCreate(&e));
    FG_HIP(hipEventRecord(e, st));
    ev.push_back(e);
    return FG_OK;
  };
  auto cleanup = [&]() {
    for (auto e : ev) hipEventDestroy(e);
  };
  fg_status r;
#define FG_TRY(x)       do {                    r = (x);              if (r) {                cleanup();            return r;           }                   } while (0)

  std::vector<uint32_t> hroots(T);
  FG_TRY(fg_roots(seed, n, T, hroots.data()));
  FG_TRY(reset_ctl(ws_dev, m, st));
  uint32_t* roots = out->roots_dev;
  FG_HIP(hipMemcpyAsync(roots, hroots.data(), T * 4, hipMemcpyHostToDevice, st));
  uint32_t* tparent = reinterpret_cast<uint32_t*>(at(ws_dev, m.tparent));
  uint64_t* off[2] = {reinterpret_cast<uint64_t*>(at(ws_dev, m.off[0])),
                      reinterpret_cast<uint64_t*>(at(ws_dev, m.off[1]))};
  uint32_t* ids[2] = {reinterpret_cast<uint32_t*>(at(ws_dev, m.ids[0])),
                      reinterpret_cast<uint32_t*>(at(ws_dev, m.ids[1]))};
  uint32_t* rows = reinterpret_cast<uint32_t*>(at(ws_dev, m.rows));
  uint32_t* cnt = reinterpret_cast<uint32_t*>(at(ws_dev, m.cnt));

  // Scaffold.
  FG_TRY(mark());
  unsigned long long sat_evals = 0;
  int status = 0;
  FG_HIP(sat_build(s, roots, T, tparent, at(ws_dev, m.sat), m.satw, st, &sat_evals, &status));
  if (status) {
    cleanup();
    return status_error(status);
  }
  FG_TRY(scaffold_csr_launch(n, T, tparent, off[0], ids[0], ws_dev, m, st));
  FG_HIP(hipMemcpyAsync(out->spine_parent_dev, tparent, n * 4, hipMemcpyDeviceToDevice, st));
  // Processing order of every block: tree 0's final bag layout, where each
  // subtree's points lie together, so that searches running at the same
  // time share targets in cache (the graph does not depend on it, Prop. 1).
  uint32_t* sched = reinterpret_cast<uint32_t*>(at(ws_dev, m.sched));
  FG_HIP(fill_u32(sched, FG_NONE, n, st));
  FG_HIP(block_schedule(reinterpret_cast<const uint32_t*>(at(ws_dev, m.sat) + m.satw.perm), n - 1, n, Be, hroots[0],
                        sched, reinterpret_cast<uint32_t*>(at(ws_dev, m.deg)),
                        reinterpret_cast<uint64_t*>(at(ws_dev, m.aoff)), at(ws_dev, m.scan), st));
  uint32_t* rank = reinterpret_cast<uint32_t*>(at(ws_dev, m.rank));
  FG_HIP(rank_of(reinterpret_cast<const uint32_t*>(at(ws_dev, m.sat) + m.satw.perm), n - 1, hroots[0], rank, st));
  FG_TRY(mark());
  FG_TRY(screen_launch(s, params, ws_dev, m, st));
  FG_TRY(mark());

  // Blocks.
  FG_HIP(fill_u32(rows, FG_NONE, n * (int64_t)R, st));
  FG_HIP(fill_u32(cnt, 0, n, st));
  FG_HIP(fill_u32(reinterpret_cast<uint32_t*>(at(ws_dev, m.bits)), 0, (int64_t)kMaxWaveSlots * m.spill_words, st));
  int cur = 0;
  std::vector<unsigned long long> blk_evals;
  Ctl* ctl = reinterpret_cast<Ctl*>(at(ws_dev, m.ctl));
  int64_t sched_base = 0;
  for (uint32_t b = 0; b < Be; b++) {
    FG_TRY(mark());
    FG_TRY(harvest_launch(s, off[cur], ids[cur], roots, params, b, rows, cnt, ws_dev, m, st, nullptr,
                          sched + sched_base, rank, log));
    sched_base += n > (int64_t)b ? (n - (int64_t)b + Be - 1) / Be : 0;
    FG_TRY(mark());
    if (timings) {
      unsigned long long e = 0;
      FG_HIP(hipMemcpyAsync(&e, &ctl->counters[0], 8, hipMemcpyDeviceToHost, st));
      FG_HIP(hipStreamSynchronize(st));
      blk_evals.push_back(e);
    }
    if (b + 1 < Be) {
      FG_TRY(merge_launch(n, off[cur], ids[cur], rows, cnt, (int)R, b, Be, off[cur ^ 1], ids[cur ^ 1], ws_dev,
                          m, st));
      cur ^= 1;
    }
    FG_TRY(mark());
  }

  // Finalize, in tree 0's layout order (neighbouring points together).
  if (n > 1)
    FG_HIP(hipMemcpyAsync(sched, at(ws_dev, m.sat) + m.satw.perm, (n - 1) * 4, hipMemcpyDeviceToDevice, st));
  FG_HIP(fill_u32(sched + n - 1, hroots[0], 1, st));
  FG_TRY(finalize_launch(s, rows, cnt, params, out->nbrs_dev, out->cnt_dev, ws_dev, m, st, nullptr, sched));
  FG_TRY(mark());
  Ctl c;
  FG_TRY(read_ctl(ws_dev, m, st, &c));
  if (counters) {
    counters->scaffold_evals += sat_evals;
    counters->harvest_evals += c.counters[0];
    counters->expansions += c.counters[1];
    counters->prune_evals += c.counters[2];
    counters->spilled_queries += c.counters[3];
    counters->screen_rejected += c.counters[4];
    counters->prune_rechecks += c.counters[5] + c.fin[2];
    counters->finalize_evals += c.fin[0] + c.fin[1];
  }
  if (timings) {
    memset(timings, 0, sizeof(*timings));
    auto ms = [&](int i, int j) {
      float t = 0.f;
      hipEventElapsedTime(&t, ev[i], ev[j]);
      return t;
    };
    timings->scaffold_ms = ms(0, 1);
    timings->screen_ms = ms(1, 2);
    timings->nblocks = Be;
    unsigned long long prev = 0;
    for (uint32_t b = 0; b < Be; b++) {
      int i0 = 3 + 3 * b;
      float h = ms(i0, i0 + 1);
      timings->block_harvest_ms[b] = h;
      timings->harvest_ms += h;
      timings->merge_ms += ms(i0 + 1, i0 + 2);
      timings->block_evals[b] = blk_evals[b] - prev;
      prev = blk_evals[b];
    }
    timings->finalize_ms = ms(2 + 3 * Be, 3 + 3 * Be);
  }
  cleanup();
#undef FG_TRY
  return status_error(c.status);
}

// Times block 0's harvest (over the substrate off/ids; a batched launch when
// bi is set) for every candidate of the knobs that never change the graph:
// the lanes per row (the library's shape, and the other one where the plain
// harvest has it), the visited-table size (where ef_h and the row allow)
// and the resident searches per compute unit (as many as fit, three
// quarters, half), best of two launches each; leaves the fastest in *P and
// its time in *best_ms.  The block's rows are overwritten.
fg_status tune_harvest(const Shape& s, const uint64_t* off, const uint32_t* ids, const uint32_t* roots,
                       fg_params* P, uint32_t* rows, uint32_t* cnt, void* ws, const WsMap& m, hipStream_t st,
                       const BatchInfo* bi, const uint32_t* order, const uint32_t* rank, float* best_ms) {
  const int ef = bi ? bi->ef_max : (int)P->ef_h;
  std::vector<unsigned> lanes_c = {0u};
  if (P->screen == FG_SCREEN_NONE)
    for (unsigned ln : {4u, 8u}) {
      int L = 0, nc = 0;
      if (lanes_variant(s.dk, s.Q, (int)ln, &L, &nc)) lanes_c.push_back(ln);
    }
  hipEvent_t e0, e1;
  FG_HIP(hipEventCreate(&e0));
  FG_HIP(hipEventCreate(&e1));
  float best = 3.0e38f;
  unsigned best_tb = 0, best_wv = 0, best_ln = 0;
  fg_params Q = *P;
  for (unsigned ln : lanes_c) {
    Q.lanes_per_row = ln;
    const int nch = beam_chunks_per_lane(s, (int)ln);
    std::vector<unsigned> tables;
    if (ef <= 128 && ln == 0 && Q.screen == FG_SCREEN_NONE) tables = {512, 1024, 2048, 4096};
    else if (ef <= 128 && search_screen(Q.screen) != SCR_NONE && nch <= 4) tables = {1024, 2048, 4096};
    else if (ef <= 128) tables = {2048, 4096};
    else tables = {4096};
    for (unsigned tb : tables) {
      Q.beam_table_slots = tb;
      Q.waves_per_cu = 0;
      const int hs = beam_table_slots(ef, false, table_request(&Q, nch), nch);
      const int lk = Q.screen == FG_SCREEN_NONE ? (int)ln : 0;
      int full = beam_grid(s, ef, false, hs, search_screen(Q.screen), 0, lk) / num_cus_host();
      if (full < 1) full = 1;
      for (unsigned wv : {0u, (unsigned)(full * 3 / 4), (unsigned)(full / 2)}) {
        if (wv != 0 && (wv < 1 || (int)wv >= full)) continue;
        Q.waves_per_cu = wv;
        float t_best = 3.0e38f;
        for (int rep = 0; rep < 2; rep++) {
          fg_status rr = FG_OK;
          if (hipEventRecord(e0, st) != hipSuccess) rr = FG_EHIP;
          if (!rr) rr = harvest_launch(s, off, ids, roots, &Q, 0, rows, cnt, ws, m, st, bi, order, rank);
          if (!rr && hipEventRecord(e1, st) != hipSuccess) rr = FG_EHIP;
          if (!rr && hipEventSynchronize(e1) != hipSuccess) rr = FG_EHIP;
          float ms = 0.f;
          if (!rr && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rr = FG_EHIP;
          if (rr) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rr;
          }
          t_best = ms < t_best ? ms : t_best;
        }
        if (t_best < best) {
          best = t_best;
          best_tb = tb;
          best_wv = wv;
          best_ln = ln;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->beam_table_slots = best_tb;
  P->waves_per_cu = best_wv;
  P->lanes_per_row = best_ln;
  *best_ms = best;
  return FG_OK;
}

}  // namespace fg

extern "C" {

// ---------------------------------------------------------------- autotune
fg_status fg_autotune(const fg_data* data, const fg_params* params, const char* cache_path, void* ws_dev,
                      size_t ws_bytes, void* stream, fg_params* tuned) {
  Shape s;
  if (!make_shape(data, &s)) return FG_EINVAL;
  if (!check_params(params, s.n)) return FG_EINVAL;
  if (!check_screen(params, s)) return FG_EUNSUPPORTED;
  if (!tuned) return set_error("tuned is NULL"), FG_EINVAL;
  int lg = 0;
  while ((1ll << (lg + 1)) <= s.n) lg++;
  char key[160];
  snprintf(key, sizeof(key), "dk=%d Q=%d ef=%u R=%u T=%u B=%u screen=%u lgn=%d", s.dk, s.Q, params->ef_h,
           params->R, params->T, b_eff(params), params->screen, lg);
  *tuned = *params;
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char line[256];
      bool hit = false;
      while (fgets(line, sizeof(line), f)) {
        unsigned tb = 0, wv = 0, ln = 0;
        const char* bar = strchr(line, '|');
        if (!bar || (size_t)(bar - line) != strlen(key) || strncmp(line, key, strlen(key))) continue;
        if (sscanf(bar + 1, " table=%u waves=%u lanes=%u", &tb, &wv, &ln) == 3 &&
            (tb == 1024 || tb == 2048 || tb == 4096) && wv <= 64 && (ln == 0 || ln == 4 || ln == 8 || ln == 16)) {
          tuned->beam_table_slots = tb;
          tuned->waves_per_cu = wv;
          tuned->lanes_per_row = ln;
          hit = true;
        }
      }
      fclose(f);
      if (hit) return FG_OK;
    }
  }
  // A prefix sample with its own scaffold; block 0 of its harvest is timed.
  Shape ss = s;
  ss.n = s.n < 50000 ? s.n : 50000;
  fg_params P = *params;
  const uint32_t T = P.T;
  if ((int64_t)T > ss.n) return set_error("fewer sample points than trees"), FG_EINVAL;
  WsMap m = ws_map(ss.n, &P, ss.d);
  if (!check_ws(ws_dev, ws_bytes, m)) return FG_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<uint32_t> hroots(T);
  fg_status r = fg_roots(1, ss.n, T, hroots.data());
  if (r) return r;
  uint32_t* roots = reinterpret_cast<uint32_t*>(at(ws_dev, m.roots));
  uint32_t* tparent = reinterpret_cast<uint32_t*>(at(ws_dev, m.tparent));
  uint64_t* off0 = reinterpret_cast<uint64_t*>(at(ws_dev, m.off[0]));
  uint32_t* ids0 = reinterpret_cast<uint32_t*>(at(ws_dev, m.ids[0]));
  uint32_t* rows = reinterpret_cast<uint32_t*>(at(ws_dev, m.rows));
  uint32_t* cnt = reinterpret_cast<uint32_t*>(at(ws_dev, m.cnt));
  r = reset_ctl(ws_dev, m, st);
  if (r) return r;
  FG_HIP(hipMemcpyAsync(roots, hroots.data(), T * 4, hipMemcpyHostToDevice, st));
  unsigned long long ev = 0;
  int status = 0;
  FG_HIP(sat_build(ss, roots, T, tparent, at(ws_dev, m.sat), m.satw, st, &ev, &status));
  if (status) return status_error(status);
  r = scaffold_csr_launch(ss.n, T, tparent, off0, ids0, ws_dev, m, st);
  if (r) return r;
  r = screen_launch(ss, &P, ws_dev, m, st);
  if (r) return r;
  FG_HIP(fill_u32(reinterpret_cast<uint32_t*>(at(ws_dev, m.bits)), 0, (int64_t)kMaxWaveSlots * m.spill_words, st));
  float best = 0.0f;
  unsigned best_tb = 0, best_wv = 0, best_ln = 0;
  r = tune_harvest(ss, off0, ids0, roots, &P, rows, cnt, ws_dev, m, st, nullptr, nullptr, nullptr, &best);
  if (r) return r;
  best_tb = P.beam_table_slots;
  best_wv = P.waves_per_cu;
  best_ln = P.lanes_per_row;
  Ctl c;
  r = read_ctl(ws_dev, m, st, &c);
  if (r) return r;
  r = status_error(c.status);
  if (r) return r;
  tuned->beam_table_slots = best_tb;
  tuned->waves_per_cu = best_wv;
  tuned->lanes_per_row = best_ln;
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "a")) {
      fprintf(f, "%s| table=%u waves=%u lanes=%u  (block-0 harvest of %lld points: %.3f ms)\n", key, best_tb,
              best_wv, best_ln, (long long)ss.n, best);
      fclose(f);
    }
  }
  return FG_OK;
}

// ---------------------------------------------------------------- batched
// Many independent instances in one id space: instance i owns ids
// [off_i, off_i + n_i) with off_i a multiple of B, so a point's block is the
// same as in its own build; rows are copied into one matrix whose stride fits
// the widest instance, zero-padded (zero chunks add exactly nothing in the
// declared order, so every distance is that of the instance alone).  One
// tree-builder pass grows every instance's trees; each block is one harvest
// launch over all
// instances (per-point instance, roots and beam width) and one merge over the
// whole id space; finalize runs once; each instance's graph is copied back
// in its own ids.
namespace {

struct BatchPlan {
  Shape s;
  fg_params P;
  int64_t N = 0, stride = 0;
  int ef_max = 0;
  std::vector<int64_t> off;
  WsMap m;
  size_t x_at = 0, inst_at = 0, roots_at = 0, ef_at = 0, q_at = 0, nbrs_at = 0, gcnt_at = 0;
  size_t total = 0;
};

bool plan_batch(const fg_data* const* data, const fg_params* const* params, uint32_t count, BatchPlan* bp) {
  if (!data || !params || count < 1 || count > 65535)
    return set_error("need 1 <= count <= 65535 instances and data/params arrays"), false;
  int dk = -1;
  for (uint32_t i = 0; i < count; i++) {
    Shape si;
    if (!data[i] || !params[i]) return set_error("NULL data or params entry"), false;
    if (!make_shape(data[i], &si)) return false;
    if (!check_params(params[i], si.n)) return false;
    if (params[i]->screen) return set_error("batched builds do not screen"), false;
    const fg_params* a = params[0];
    const fg_params* b = params[i];
    if (b->T != a->T || b->R != a->R || b->alpha != a->alpha || b_eff(b) != b_eff(a) ||
        b->reprune_all != a->reprune_all || b->beam_table_slots != a->beam_table_slots ||
        b->waves_per_cu != a->waves_per_cu)
      return set_error("batched instances must share T, R, alpha, B, reprune_all and the tuning knobs"), false;
    if (dk >= 0 && si.dk != dk) return set_error("batched instances must share dtype and metric"), false;
    dk = si.dk;
    const int64_t rb = (int64_t)si.Q * 16;
    bp->stride = rb > bp->stride ? rb : bp->stride;
    bp->ef_max = (int)b->ef_h > bp->ef_max ? (int)b->ef_h : bp->ef_max;
  }
  const int64_t Be = b_eff(params[0]);
  bp->off.assign(count + 1, 0);
  for (uint32_t i = 0; i < count; i++) bp->off[i + 1] = bp->off[i] + (data[i]->n + Be - 1) / Be * Be;
  bp->N = bp->off[count];
  if (bp->N >= (int64_t)0xFFFFFFFFu) return set_error("too many points in the batch"), false;
  bp->P = *params[0];
  bp->P.ef_h = (uint32_t)bp->ef_max;
  bp->s.x = nullptr;
  bp->s.stride = bp->stride;
  bp->s.n = bp->N;
  bp->s.dk = dk;
  bp->s.Q = (int)(bp->stride / 16);
  bp->s.d = dk == U8L2 ? (int)bp->stride : (int)(bp->stride / 4);
  bp->m = ws_map(bp->N, &bp->P);
  size_t o = bp->m.total;
  auto take = [&](size_t bytes) {
    size_t at_ = o;
    o += align256(bytes);
    return at_;
  };
  const uint64_t N = (uint64_t)bp->N, T = bp->P.T, R = bp->P.R;
  bp->x_at = take(N * (uint64_t)bp->stride);
  bp->inst_at = take(N * 2);
  bp->roots_at = take((uint64_t)count * T * 4);
  bp->ef_at = take((uint64_t)count * 4);
  bp->q_at = take((uint64_t)count * 4);
  bp->nbrs_at = take(N * R * 4);
  bp->gcnt_at = take(N * 4);
  bp->total = o;
  return true;
}

}  // namespace

size_t fg_batched_workspace_size(const fg_data* const* data, const fg_params* const* params, uint32_t count) {
  BatchPlan bp;
  if (!plan_batch(data, params, count, &bp)) return 0;
  return bp.total;
}

fg_status fg_build_graph_batched(const fg_data* const* data, const fg_params* const* params,
                                 const uint64_t* seeds, uint32_t count, fg_graph* const* outs, void* ws_dev,
                                 size_t ws_bytes, void* stream, int flags, fg_counters* counters) {
  const bool use_hipgraph = (flags & FG_BATCH_HIPGRAPH) != 0;
  BatchPlan bp;
  if (!plan_batch(data, params, count, &bp)) return FG_EINVAL;
  if (!seeds || !outs) return set_error("seeds and outs are required"), FG_EINVAL;
  const uint32_t T = bp.P.T, R = bp.P.R;
  for (uint32_t i = 0; i < count; i++) {
    const fg_graph* g = outs[i];
    if (!g || !g->nbrs_dev || !g->cnt_dev || !g->spine_parent_dev || !g->roots_dev)
      return set_error("every array of every output graph is required"), FG_EINVAL;
    if (g->n != data[i]->n || g->R != R || g->T != T)
      return set_error("an output graph's shape does not match its instance"), FG_EINVAL;
  }
  if (!ws_dev || reinterpret_cast<uintptr_t>(ws_dev) % 256) return set_error("workspace must be 256-byte aligned"), FG_EINVAL;
  if (ws_bytes < bp.total) return set_error("workspace too small (see fg_batched_workspace_size)"), FG_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const WsMap& m = bp.m;
  const int64_t N = bp.N;
  const uint32_t Be = b_eff(&bp.P);
  uint8_t* X = reinterpret_cast<uint8_t*>(at(ws_dev, bp.x_at));
  bp.s.x = X;
  uint16_t* inst_of = reinterpret_cast<uint16_t*>(at(ws_dev, bp.inst_at));
  uint32_t* inst_roots = reinterpret_cast<uint32_t*>(at(ws_dev, bp.roots_at));
  int* inst_ef = reinterpret_cast<int*>(at(ws_dev, bp.ef_at));
  int* inst_q = reinterpret_cast<int*>(at(ws_dev, bp.q_at));
  uint32_t* gnbrs = reinterpret_cast<uint32_t*>(at(ws_dev, bp.nbrs_at));
  uint32_t* gcnt = reinterpret_cast<uint32_t*>(at(ws_dev, bp.gcnt_at));
  uint32_t* tparent = reinterpret_cast<uint32_t*>(at(ws_dev, m.tparent));
  uint64_t* off[2] = {reinterpret_cast<uint64_t*>(at(ws_dev, m.off[0])),
                      reinterpret_cast<uint64_t*>(at(ws_dev, m.off[1]))};
  uint32_t* ids[2] = {reinterpret_cast<uint32_t*>(at(ws_dev, m.ids[0])),
                      reinterpret_cast<uint32_t*>(at(ws_dev, m.ids[1]))};
  uint32_t* rows = reinterpret_cast<uint32_t*>(at(ws_dev, m.rows));
  uint32_t* cnt = reinterpret_cast<uint32_t*>(at(ws_dev, m.cnt));

  // The shared matrix, the per-point instance and the per-instance tables.
  FG_HIP(fill_u32(reinterpret_cast<uint32_t*>(X), 0, N * bp.stride / 4, st));
  std::vector<uint16_t> hinst((size_t)N, 0xFFFFu);
  std::vector<uint32_t> hroots_all((size_t)count * T), hroots_local((size_t)count * T);
  std::vector<int> hef(count), hq(count);
  for (uint32_t i = 0; i < count; i++) {
    const fg_data* di = data[i];
    const int64_t esz = di->dtype == FG_U8 ? 1 : 4;
    FG_HIP(hipMemcpy2DAsync(X + bp.off[i] * bp.stride, (size_t)bp.stride, di->x_dev, (size_t)di->row_stride_bytes,
                            (size_t)(di->d * esz), (size_t)di->n, hipMemcpyDeviceToDevice, st));
    for (int64_t j = 0; j < di->n; j++) hinst[(size_t)(bp.off[i] + j)] = (uint16_t)i;
    fg_status r = fg_roots(seeds[i], di->n, T, &hroots_local[(size_t)i * T]);
    if (r) return r;
    for (uint32_t t = 0; t < T; t++)
      hroots_all[(size_t)i * T + t] = hroots_local[(size_t)i * T + t] + (uint32_t)bp.off[i];
    hef[i] = (int)params[i]->ef_h;
    hq[i] = bp.s.dk == U8L2 ? data[i]->d / 16 : data[i]->d / 4;
  }
  FG_HIP(hipMemcpyAsync(inst_of, hinst.data(), hinst.size() * 2, hipMemcpyHostToDevice, st));
  FG_HIP(hipMemcpyAsync(inst_roots, hroots_all.data(), hroots_all.size() * 4, hipMemcpyHostToDevice, st));
  FG_HIP(hipMemcpyAsync(inst_ef, hef.data(), hef.size() * 4, hipMemcpyHostToDevice, st));
  FG_HIP(hipMemcpyAsync(inst_q, hq.data(), hq.size() * 4, hipMemcpyHostToDevice, st));
  fg_status r = reset_ctl(ws_dev, m, st);
  if (r) return r;
  FG_HIP(hipStreamSynchronize(st));  // the host tables above must outlive their copies

  // Scaffold: every instance's T trees in one builder pass, in the shared ids.
  unsigned long long sat_evals = 0;
  {
    std::vector<SatInstance> si(count);
    for (uint32_t i = 0; i < count; i++) si[i] = SatInstance{bp.off[i], data[i]->n, &hroots_local[(size_t)i * T]};
    int status = 0;
    FG_HIP(sat_build_multi(bp.s, T, si, tparent, at(ws_dev, m.sat), m.satw, st, &sat_evals, &status, inst_of,
                           inst_q));
    if (status) return status_error(status);
  }
  r = scaffold_csr_launch(N, T, tparent, off[0], ids[0], ws_dev, m, st);
  if (r) return r;

  // Processing order: each instance's tree-0 layout and root, instance after
  // instance (the padding ids between instances are in no block's list), and
  // each id's position in it for the order-indexed visited bitsets.
  uint32_t* sched = reinterpret_cast<uint32_t*>(at(ws_dev, m.sched));
  uint32_t* rank = reinterpret_cast<uint32_t*>(at(ws_dev, m.rank));
  {
    uint32_t* ord = reinterpret_cast<uint32_t*>(at(ws_dev, m.deg));
    const uint32_t* perm0 = reinterpret_cast<const uint32_t*>(at(ws_dev, m.sat) + m.satw.perm);
    int64_t len = 0;
    for (uint32_t i = 0; i < count; i++) {
      const int64_t ni = data[i]->n;
      if (ni > 1)
        FG_HIP(hipMemcpyAsync(ord + len, perm0 + bp.off[i], (ni - 1) * 4, hipMemcpyDeviceToDevice, st));
      FG_HIP(fill_u32(ord + len + ni - 1, (uint32_t)bp.off[i] + hroots_local[(size_t)i * T], 1, st));
      len += ni;
    }
    FG_HIP(fill_u32(sched, FG_NONE, N, st));
    FG_HIP(block_schedule(ord, len, N, Be, FG_NONE, sched, reinterpret_cast<uint32_t*>(at(ws_dev, m.cursor)),
                          reinterpret_cast<uint64_t*>(at(ws_dev, m.aoff)), at(ws_dev, m.scan), st));
    FG_HIP(rank_of(ord, len, FG_NONE, rank, st));
  }

  // Blocks.
  const BatchInfo bi{inst_of, inst_roots, inst_ef, bp.ef_max, inst_q};
  auto init_rows = [&](hipStream_t s_) -> fg_status {
    FG_HIP(fill_u32(rows, FG_NONE, N * (int64_t)R, s_));
    FG_HIP(fill_u32(cnt, 0, N, s_));
    FG_HIP(fill_u32(reinterpret_cast<uint32_t*>(at(ws_dev, m.bits)), 0, (int64_t)kMaxWaveSlots * m.spill_words, s_));
    return FG_OK;
  };
  auto blocks = [&](hipStream_t s_, bool device_only) -> fg_status {
    int cur = 0;
    int64_t base = 0;
    for (uint32_t b = 0; b < Be; b++) {
      fg_status rr = harvest_launch(bp.s, off[cur], ids[cur], inst_roots, &bp.P, b, rows, cnt, ws_dev, m, s_, &bi,
                                    sched + base, rank);
      if (rr) return rr;
      base += N > (int64_t)b ? (N - (int64_t)b + Be - 1) / Be : 0;
      if (b + 1 < Be) {
        rr = merge_launch(N, off[cur], ids[cur], rows, cnt, (int)R, b, Be, off[cur ^ 1], ids[cur ^ 1], ws_dev, m,
                          s_, device_only);
        if (rr) return rr;
        cur ^= 1;
      }
    }
    return FG_OK;
  };
  // FG_BATCH_AUTOTUNE: the knobs that never change a graph (lanes per row,
  // visited-table size, resident searches per compute unit) timed on this
  // batch's own launch, block 0 of every instance over S_0; the choice is
  // kept per batch shape for later calls.
  if (flags & FG_BATCH_AUTOTUNE) {
    char key[256];
    snprintf(key, sizeof key, "batch count=%u N=%lld dk=%d Q=%d ef=%d T=%u R=%u B=%u", count, (long long)N, bp.s.dk,
             bp.s.Q, bp.ef_max, T, R, Be);
    uint32_t knobs[3];
    if (tuned_lookup(key, knobs)) {
      bp.P.beam_table_slots = knobs[0];
      bp.P.waves_per_cu = knobs[1];
      bp.P.lanes_per_row = knobs[2];
    } else {
      r = init_rows(st);
      if (r) return r;
      float ms = 0.0f;
      r = tune_harvest(bp.s, off[0], ids[0], inst_roots, &bp.P, rows, cnt, ws_dev, m, st, &bi, sched, rank, &ms);
      if (r) return r;
      const uint32_t got[3] = {bp.P.beam_table_slots, bp.P.waves_per_cu, bp.P.lanes_per_row};
      tuned_store(key, got);
      r = reset_ctl(ws_dev, m, st);  // the timing launches' counters are not the build's
      if (r) return r;
    }
  }
  r = init_rows(st);
  if (r) return r;
  if (use_hipgraph) {
    // Capture the blocks on a stream of our own (ordered after and before
    // the caller's stream) and replay the graph once.
    hipStream_t cs = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    auto release = [&]() {  // best effort: the first error is the one reported
      if (ge) (void)hipGraphExecDestroy(ge);
      if (g) (void)hipGraphDestroy(g);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      if (cs) (void)hipStreamDestroy(cs);
    };
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e0, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, e0, 0);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      release();
      FG_HIP(e);
    }
    fg_status rb = blocks(cs, true);
    e = hipStreamEndCapture(cs, &g);
    if (rb) {
      release();
      return rb;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(ge, cs);
    if (e == hipSuccess) e = hipEventRecord(e1, cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, e1, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    release();
    FG_HIP(e);
  } else {
    r = blocks(st, false);
    if (r) return r;
  }

  // Finalize over the shared id space, then each instance in its own ids.
  r = finalize_launch(bp.s, rows, cnt, &bp.P, gnbrs, gcnt, ws_dev, m, st, &bi);
  if (r) return r;
  for (uint32_t i = 0; i < count; i++) {
    FG_HIP(localize_graph(gnbrs, gcnt, tparent, data[i]->n, (int)R, bp.off[i], outs[i]->nbrs_dev, outs[i]->cnt_dev,
                          outs[i]->spine_parent_dev, st));
    FG_HIP(hipMemcpyAsync(outs[i]->roots_dev, &hroots_local[(size_t)i * T], T * 4, hipMemcpyHostToDevice, st));
  }
  Ctl c;
  r = read_ctl(ws_dev, m, st, &c);
  if (r) return r;
  if (counters) {
    counters->scaffold_evals += sat_evals;
    counters->harvest_evals += c.counters[0];
    counters->expansions += c.counters[1];
    counters->prune_evals += c.counters[2];
    counters->spilled_queries += c.counters[3];
    counters->finalize_evals += c.fin[0] + c.fin[1];
  }
  return status_error(c.status);
}

}  // extern "C"
