// fg_beam.h -- the beam-search wave (harvest and query search) and the
// occlusion prune, for gfx950.
//
// One wavefront serves one query at a time and takes queries from an atomic
// work queue until the block is exhausted (persistent grid), so uneven beam
// lengths do not idle the machine.
//
// Per query (Sec. 3): the beam is a sorted LDS array of at most ef keys
// (distance, id) with an "expanded" flag per entry.  The roots are evaluated
// first; then, repeatedly, the best unexpanded entry is expanded: its CSR row
// is read 64 ids at a time, every id not yet visited is evaluated (groups of
// L lanes gather one row each in 16-byte chunks), the new keys that can
// still enter the beam are sorted across the wave and merged into the beam
// by co-ranking.  The search ends when every beam entry is expanded.
//
// The visited set is exact: an LDS open-addressing table of HSLOTS ids; once
// it is 3/4 full, further ids go to a per-wave bitset in device memory (and a
// list of them, so the bitset can be cleared word by word afterwards).
//
// Screened harvest (float32 rows, Sec. 5.3's bytes-per-evaluation term): a
// narrow copy of the rows (bfloat16, or fp8-e4m3 with a power-of-two scale
// per row) gives each new candidate a cheap distance d~ and a rigorous error
// margin eps; once the beam is full, a candidate with d~ - eps above the
// beam's worst exact distance cannot enter it and is not evaluated exactly.
// Every other candidate gets its exact float32 distance, so the beam, the
// expanded set and the graph are those of the unscreened search.
//
// Harvest mode records the expanded entries and then prunes them (without
// the query point itself): sorted by key, the next live candidate is kept,
// and every later live candidate c with fl32(alpha * d(kept, c)) <= d(p, c)
// dies; at most R are kept.
#pragma once
#include "fg_device.h"

namespace fg {

// Phase timers for a profiling build (-DFG_PROFILE): shader-clock cycles
// spent by lane 0 of every wave in each phase of the beam loop, summed over
// the grid into fg_prof_cycles[].  Absent from normal builds.
#ifdef FG_PROFILE
// One array per translation unit; each unit exports its own reader.
static __device__ unsigned long long fg_prof_cycles[16];
#define FG_PROF_READER(name)                                                               \
  extern "C" int name(unsigned long long* out16) {                                        \
    if (hipMemcpyFromSymbol(out16, HIP_SYMBOL(fg::fg_prof_cycles), 16 * 8) != hipSuccess) \
      return -1;                                                                          \
    unsigned long long z[16] = {};                                                        \
    return hipMemcpyToSymbol(HIP_SYMBOL(fg::fg_prof_cycles), z, 16 * 8) == hipSuccess ? 0 : -1; \
  }
#define FG_T0() uint64_t fg_t0_ = __builtin_amdgcn_s_memtime()
#define FG_TICK(slot)                                        \
  do {                                                       \
    uint64_t fg_t1_ = __builtin_amdgcn_s_memtime();          \
    prof[slot] += fg_t1_ - fg_t0_;                           \
    fg_t0_ = fg_t1_;                                         \
  } while (0)
#else
#define FG_T0() \
  do {          \
  } while (0)
#define FG_TICK(slot) \
  do {                \
  } while (0)
#endif

// Rows x = hi + lo + e in bfloat16 (hi = x rounded to nearest even, lo = the
// remainder x - hi so rounded; |e| <= 2^-16 |x| elementwise), `stride` bytes
// per row in 64-byte steps of 16 elements (32 bytes of hi, then 32 of lo),
// zero-padded to whole steps.  p == NULL: the Gram tiles read the float32
// rows.
struct GramSplit {
  const uint8_t* p;
  int64_t stride;
};

struct BeamArgs {
  // data
  const uint8_t* x;
  int64_t stride;
  int64_t n;
  int Q;  // 16-byte chunks per row
  // graph
  const uint64_t* off;
  const uint32_t* ids;
  const uint32_t* roots;
  int T;
  int ef;
  // harvest
  int R;
  float alpha;
  int64_t b, B;  // points p = b + i * B
  uint32_t* rows;
  uint32_t* cnt;
  // search
  const uint8_t* queries;
  int64_t qstride;
  int k;
  uint32_t* out_ids;
  void* out_d;
  uint32_t* out_evals;
  // work
  int64_t nitems;
  // harvest: the block's points in processing order (NULL: p = b + item * B);
  // the graph does not depend on the order (Prop. 1), locality does
  const uint32_t* order;
  // visited bitsets indexed by position in the processing order instead of
  // by id (NULL: by id): a search's visits then cluster in fewer lines.
  // Used by rows of 2..4 chunks per lane, where it measured faster; the
  // extra dependent load costs more than it saves for one-chunk and
  // 16-chunk rows.
  const uint32_t* rank;
  // with rank: the CSR's ids paired with their ranks (idr[e] = (ids[e],
  // rank[ids[e]])), so a scanned id's bit needs no lookup in rank, whose
  // random reads compete with the rows for the L2 (NULL: look it up)
  const uint2* idr;
  unsigned long long* queue;
  // with order: eight counters, one slice of the order per XCD (workgroup i
  // runs on XCD i mod 8), so each L2 sees neighbouring points; a wave whose
  // slice is done takes from the next one (NULL: the single queue)
  unsigned int* xqueue;
  // scratch (per wave slot)
  uint64_t* Ebuf;
  int Ecap;
  uint32_t* spill_bits;
  int64_t spill_words;
  uint32_t* spill_list;
  int spill_cap;
  unsigned long long* counters;  // evals, expansions, prune pairs, spilled, screen-rejected, prune rechecks
  int* status;                   // bit 0: expanded-list overflow
  // screened harvest: the narrow copy (row stride xs_stride bytes, the
  // elements in data order), each row with a trailer at byte xs_tail:
  // the norm of its quantisation error |u^ - u|, its norm |u| (both rounded
  // up) and the fp8 dequantisation factor (a power of two)
  const uint8_t* xs;
  int64_t xs_stride;
  int64_t xs_tail;
  int d;
  // batched builds: many instances in one id space.  inst_of[p] is p's
  // instance (0xFFFF: an unused id, skipped), whose T roots are
  // inst_roots[i*T ..] and beam width inst_ef[i] (<= ef).  NULL otherwise.
  const uint16_t* inst_of;
  const uint32_t* inst_roots;
  const int* inst_ef;
  const int* inst_q;  // 16-byte chunks of instance i's own rows (the rest of a row is zero)
  // float32 rows of more than 64 chunks: per wave slot a kGramMax^2 float
  // scratch for the candidates' Gram matrix (NULL: exact prune only)
  float* gram;
  // the Gram tiles from the bfloat16 split of the rows (see GramSplit)
  GramSplit split;
  // |x_i|^2 of every row (any float32 summation order): the Gram prune's
  // diagonal (NULL: no Gram prune)
  const float* norm;
  // visit log (the logging instantiation only): points p with
  // log_slot[p] >= 0 record the ids their search visits, in visit order,
  // into log_ids[slot * log_cap ..] (the first log_cap of them), the total
  // into log_len[slot], and the visit count after the roots and after each
  // of the first kLogMarks - 1 expansions into log_marks[slot * kLogMarks ..]
  const int* log_slot;
  uint32_t* log_ids;
  uint32_t* log_len;
  uint32_t* log_marks;
  int64_t log_cap;
  int log_nslots;  // slots outside [0, log_nslots) are not logged
};

constexpr int kLogMarks = 17;

constexpr int kGramMax = 1024;   // candidates the Gram-tile prune takes
constexpr int kGramPF16 = 4;     // split-tile steps in flight
constexpr int kGramSlots = 2048; // wave slots that have Gram scratch

enum ScreenKind { SCR_NONE = 0, SCR_BF16 = 1, SCR_FP8 = 2, SCR_INT8 = 3 };

// One narrow row's codes as lane g of a group holds them: chunk q = g + L*i
// (four elements) as two words of bfloat16 or one word of fp8, zero past Q.
template <int NCH, int SCR>
struct NarrowChunks {
  uint32_t w[NCH * (SCR == SCR_BF16 ? 2 : 1)];
};

template <int L, int NCH, int SCR>
__device__ __forceinline__ void load_narrow(NarrowChunks<NCH, SCR>& r, const uint8_t* srow, int Q, int g) {
#pragma unroll
  for (int i = 0; i < NCH; i++) {
    const int q = g + L * i;
    if constexpr (SCR == SCR_BF16) {
      uint2 v = make_uint2(0, 0);
      if (q < Q) v = *reinterpret_cast<const uint2*>(srow + 8 * (size_t)q);
      r.w[2 * i] = v.x;
      r.w[2 * i + 1] = v.y;
    } else {
      r.w[i] = q < Q ? *reinterpret_cast<const uint32_t*>(srow + 4 * (size_t)q) : 0u;
    }
  }
}

// Screened sum between the query's exact float32 chunks `a` and a narrow
// row's chunks, reduced over the group (every lane of the group gets it):
// squared L2, the codes scaled by sinv element by element; cosine, the dot
// product with the unscaled codes (the caller forms 1 - sinv * sum: a power
// of two commutes with every rounding of the sum, and an overflow can only
// make the caller keep the candidate).  Any summation order: the margin
// below holds for all of them.
template <int DK, int L, int NCH, int SCR>
__device__ __forceinline__ float group_screen(const Chunks<L, NCH>& a, const NarrowChunks<NCH, SCR>& r, float sinv,
                                              int Q, int g) {
  float acc = 0.0f;
#pragma unroll
  for (int i = 0; i < NCH; i++) {
    const int q = g + L * i;
    if (q < Q) {
      const float4 xa = *reinterpret_cast<const float4*>(&a.c[i]);
      float4 xb;
      if constexpr (SCR == SCR_BF16) {
        const uint32_t w0 = r.w[2 * i], w1 = r.w[2 * i + 1];
        xb = make_float4(__uint_as_float(w0 << 16), __uint_as_float(w0 & 0xFFFF0000u), __uint_as_float(w1 << 16),
                         __uint_as_float(w1 & 0xFFFF0000u));
      } else if constexpr (SCR == SCR_INT8) {  // squared L2: each code read back as fl(code * s)
        const int w = (int)r.w[i];
        xb = make_float4((float)((w << 24) >> 24) * sinv, (float)((w << 16) >> 24) * sinv,
                         (float)((w << 8) >> 24) * sinv, (float)(w >> 24) * sinv);
      } else {
        const int w = (int)r.w[i];
        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
        if constexpr (DK == F32L2)
          xb = make_float4(lo[0] * sinv, lo[1] * sinv, hi[0] * sinv, hi[1] * sinv);
        else
          xb = make_float4(lo[0], lo[1], hi[0], hi[1]);
      }
      if constexpr (DK == F32L2) {
        const float d0 = xa.x - xb.x, d1 = xa.y - xb.y, d2 = xa.z - xb.z, d3 = xa.w - xb.w;
        acc = __builtin_fmaf(d0, d0, acc);
        acc = __builtin_fmaf(d1, d1, acc);
        acc = __builtin_fmaf(d2, d2, acc);
        acc = __builtin_fmaf(d3, d3, acc);
      } else {
        acc = __builtin_fmaf(xa.x, xb.x, acc);
        acc = __builtin_fmaf(xa.y, xb.y, acc);
        acc = __builtin_fmaf(xa.z, xb.z, acc);
        acc = __builtin_fmaf(xa.w, xb.w, acc);
      }
    }
  }
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) acc = acc + __shfl_xor(acc, off, 64);
  return acc;
}

// int8 codes of the point and of a candidate row, dot product over the
// group in exact integer arithmetic (|sum| <= 127^2 d < 2^24, so the result
// converts to float exactly).
template <int L, int NCH>
__device__ __forceinline__ int group_dot_i8(const NarrowChunks<NCH, SCR_INT8>& p,
                                            const NarrowChunks<NCH, SCR_INT8>& r) {
  int acc = 0;
#pragma unroll
  for (int i = 0; i < NCH; i++) acc = __builtin_amdgcn_sdot4((int)p.w[i], (int)r.w[i], acc, false);
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  return acc;
}

// Margin eps such that the exact (declared-order float32) distance is at
// least dt - eps, for a screened value dt (standard rounding-error analysis,
// unit roundoff u = 2^-24; gs bounds the screened sum's relative error over
// d + 12 roundings, gc the declared order's over d/16 + 8):
//   squared L2: with A = sqrt((dt + t) / (1 - gs)) >= |p - u^|,
//     |p - u| >= |p - u^| - E where E = |u^ - u|, so that
//     exact >= dt - (gs + gc) dt - 2 A E - t;
//   cosine: |<p,u^> - <p,u>| <= |p| E, both sums' errors are within
//     (gs + gc) |p| (|u| + E) + t, and the two roundings of 1 - s, with
//     the fp8 copy's power-of-two factor f, add 4u (1 + |p| (|u| + E)).
// t covers underflow: float32 subnormals are kept (IEEE mode, as built), so
// a product or fused multiply-add that underflows errs by at most 2^-150,
// d of them per sum: t = d 2^-149 for squared L2's two sums; for cosine
// t = d 2^-149 (1 + max(1, f) + |p|), the screened sum's errors scaled by
// f, and the fp8 read-back's underflow (at most 2^-150 per element) against
// |p|.  The result is raised by 2^-20 of itself, which covers the rounding
// of its own few operations (each at most u).
struct ScreenGammas {
  float gs, gc;
  float t;  // d 2^-149
};

__device__ __forceinline__ ScreenGammas screen_gammas(int d) {
  const float u = 5.9604645e-08f;  // 2^-24
  return {(d + 12) * u / (1.0f - (d + 12) * u), (d / 16 + 8) * u / (1.0f - (d / 16 + 8) * u),
          (float)d * 1.4012985e-45f};
}

constexpr float kEpsRaise = 1.0f + 9.5367432e-07f;  // 1 + 2^-20

template <int DK>
__device__ __forceinline__ float screen_eps(float dt, ScreenGammas k, float E, float np, float nu, float f) {
  const float u = 5.9604645e-08f;  // 2^-24
  const float gs = k.gs, gc = k.gc;
  float eps;
  if constexpr (DK == F32L2) {
    const float dd = dt > 0.0f ? dt : 0.0f;
    const float A = __builtin_sqrtf((dd + k.t) / (1.0f - gs)) * (1.0f + 4.0f * u);
    eps = (gs + gc) * dd + 2.0f * A * E + k.t;
  } else {
    const float pu = np * (nu + E);
    eps = np * E + (gs + gc) * pu + 4.0f * u * (1.0f + pu) + k.t * (1.0f + fmaxf(1.0f, f) + np);
  }
  return eps * kEpsRaise;
}

// The same for cosine over int8 codes of both rows: dt = 1 - fl(fl(s_p s_u) I)
// with I the exact integer dot product, so <p^,u^> = s_p s_u I with p^, u^
// the codes times their scales in exact arithmetic.  Their distances from p
// and u are at most E' = E + u (|x| + E) + d 2^-150 (E bounds the distance
// from the copy read back with one rounding per element, which may also
// underflow):
//   |<p,u> - <p^,u^>| <= E'_p |u| + |p^| E'_u, |p^| <= |p| + E'_p = P,
//   |u^| <= U; the two products round by at most 2.0001 u P U, 1 - x by
//   u (1 + P U); the declared order's sum errs by gc |p||u| and its 1 - s
//   by u (1 + |p||u|).  Underflow: fl(s_p s_u) errs by at most 2^-150,
//   times |I| <= 127^2 d, and the declared sum's d operations by 2^-150
//   each: below d 2^-136 together.  Raised by 2^-20 of itself as above.
__device__ __forceinline__ float screen_eps_i8(ScreenGammas k, float Ep, float np, float Eu, float nu) {
  const float u = 5.9604645e-08f;  // 2^-24
  const float fl = 0.5f * k.t;       // d 2^-150
  const float Epp = Ep + u * (np + Ep) + fl, Eup = Eu + u * (nu + Eu) + fl;
  const float P = np + Epp, U = nu + Eup;
  const float eps = Epp * nu + P * Eup + (k.gc + 4.0f * u) * P * U + 4.0f * u * (1.0f + P * U) + 8192.0f * k.t;
  return eps * kEpsRaise;
}

// Screen the cnt new ids in ids_lds (cnt <= 256) against the beam's worst
// exact distance w: ids that cannot enter the beam are dropped, the others
// are compacted to the front of ids_lds (in an order of their own: the
// beam's merge sorts by key).  Returns their number.  A narrow row is a
// quarter or half of the float32 row's bytes, so twice as many rows are
// kept in flight per round as in the exact gathers (rows of 16 chunks per
// lane and more take screen_filter_wide below).  Every row's loads of a
// round are issued before the first is used (with the loads inside the
// per-row arithmetic the compiler waited on each row in turn, and the
// screened harvest took 1.3-1.6x the plain one).  Lane g of a group owns
// row g of the group's rows in the round: it loads that row's trailer
// (err, norm, sinv) and decides it, so one ballot per round compacts the
// survivors.
template <int DK, int L, int NCH, int SCR>
__device__ __forceinline__ int screen_filter(const BeamArgs& A, const Chunks<L, NCH>& a, float np,
                                             const NarrowChunks<NCH, SCR>& pc, float p_err, float p_scale,
                                             uint32_t* ids_lds, int cnt, float w) {
  constexpr bool kIntDot = SCR == SCR_INT8 && DK == F32COS;  // the point's own codes against the row's
  constexpr int G = 64 / L;
  static_assert(NCH < 16, "longer rows take screen_filter_wide");
  constexpr int RB = 32 / NCH;
  static_assert(RB <= L, "a lane owns at most one row of a round");
  const int lane = lane_id();
  const int grp = lane / L, g = lane % L;
  const int base = grp * L;
  const ScreenGammas gam = screen_gammas(A.d);
  int kept = 0;
  for (int r0 = 0; r0 < cnt; r0 += G * RB) {
    uint32_t u[RB];
    float dt[RB];
    NarrowChunks<NCH, SCR> rc[RB];
#pragma unroll
    for (int t = 0; t < RB; t++) {
      const int r = r0 + t * G + grp;
      u[t] = ids_lds[r < cnt ? r : 0];
    }
    const int myr = r0 + g * G + grp;
    const bool mine = g < RB && myr < cnt;
    const uint32_t myid = ids_lds[mine ? myr : 0];
    // every row's loads are issued before any is used
    const float4 tr = *reinterpret_cast<const float4*>(A.xs + (size_t)myid * A.xs_stride + A.xs_tail);
#pragma unroll
    for (int t = 0; t < RB; t++) load_narrow<L, NCH, SCR>(rc[t], A.xs + (size_t)u[t] * A.xs_stride, A.Q, g);
#pragma unroll
    for (int t = 0; t < RB; t++) {
      if constexpr (kIntDot) {
        dt[t] = (float)group_dot_i8<L, NCH>(pc, rc[t]);
      } else {
        // squared L2 over fp8 or int8 codes scales each element by its
        // row's factor, which lane t of the group loaded
        const float sinv = ((SCR == SCR_FP8 || SCR == SCR_INT8) && DK == F32L2) ? __shfl(tr.z, base + t, 64) : 1.0f;
        dt[t] = group_screen<DK, L, NCH, SCR>(a, rc[t], sinv, A.Q, g);
      }
    }
    float own = dt[0];
#pragma unroll
    for (int t = 1; t < RB; t++)
      if (g == t) own = dt[t];
    float eps;
    if constexpr (kIntDot) {
      own = 1.0f - (p_scale * tr.z) * own;
      eps = screen_eps_i8(gam, p_err, np, tr.x, tr.y);
    } else {
      if constexpr (DK == F32COS) own = 1.0f - (SCR == SCR_FP8 ? tr.z * own : own);
      eps = screen_eps<DK>(own, gam, tr.x, np, DK == F32COS ? tr.y : 0.0f, SCR == SCR_FP8 ? tr.z : 1.0f);
    }
    const bool keep = mine && !(own - eps > w);
    wave_sync();  // every read of this round's ids precedes the compaction
    const uint64_t m = ballot(keep);
    if (keep) ids_lds[kept + popc64(m & lanes_below())] = myid;
    kept += popc64(m);
    wave_sync();
  }
  return kept;
}

// Rows of 16 chunks per lane and more (d > 256): the whole wave screens a
// narrow row, lane l taking its elements [16 l, 16 l + 16) -- one 16-byte
// load of fp8 or int8 codes, two of bfloat16 -- so a round keeps kWideRows
// rows in flight in 4 (8) registers each, where the group layout above
// holds a row in 16 (32) and the kernel's register budget allowed only one
// row per group (four per wave).  The point's own elements in this layout
// are read again at each call from its rows (cache hits, issued with the
// first round's loads), so nothing stays live across the search.  Lane 8t
// loads row t's trailer and decides row t; the eight partial sums are
// reduced together (three halving exchanges, then three plain ones), in an
// order of their own, which the margins allow.
constexpr int kWideRows = 8;

template <typename T>
__device__ __forceinline__ T reduce_wide_rows(const T (&v)[kWideRows]) {
  const int lane = lane_id();
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  T w4[4], w2[2];
#pragma unroll
  for (int t = 0; t < 4; t++) {  // w4[t]: row t + 4 b5
    const T send = b5 ? v[t] : v[t + 4], keep = b5 ? v[t + 4] : v[t];
    w4[t] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int t = 0; t < 2; t++) {  // w2[t]: row t + 2 b4 + 4 b5
    const T send = b4 ? w4[t] : w4[t + 2], keep = b4 ? w4[t + 2] : w4[t];
    w2[t] = keep + __shfl_xor(send, 16, 64);
  }
  const T send = b3 ? w2[0] : w2[1], keep = b3 ? w2[1] : w2[0];
  T s = keep + __shfl_xor(send, 8, 64);  // row b3 + 2 b4 + 4 b5 = lane / 8
  s = s + __shfl_xor(s, 4, 64);
  s = s + __shfl_xor(s, 2, 64);
  s = s + __shfl_xor(s, 1, 64);
  return s;
}

template <int SCR>
struct WideRow {
  uint4 w[SCR == SCR_BF16 ? 2 : 1];
};

// Lane l's 16 codes of a narrow row (zero for chunks at or past Q).
template <int SCR>
__device__ __forceinline__ void load_wide(WideRow<SCR>& r, const uint8_t* srow, int Q, int lane) {
  const int q0 = 4 * lane;
#pragma unroll
  for (int h = 0; h < (SCR == SCR_BF16 ? 2 : 1); h++) {
    uint4 v = make_uint4(0, 0, 0, 0);
    const int qh = q0 + 2 * h;  // first chunk of this 16-byte word (bfloat16: two chunks per word)
    if (qh < Q) v = *reinterpret_cast<const uint4*>(srow + (SCR == SCR_BF16 ? 32 : 16) * (size_t)lane + 16 * h);
    if constexpr (SCR == SCR_BF16) {
      if (qh + 1 >= Q) v.z = v.w = 0u;
    } else {
      if (q0 + 1 >= Q) v.y = 0u;
      if (q0 + 2 >= Q) v.z = 0u;
      if (q0 + 3 >= Q) v.w = 0u;
    }
    r.w[h] = v;
  }
}

// Chunk k (four elements) of a wide row: its codes as float32, scaled by
// sinv element by element for squared L2 over fp8 or int8.
template <int DK, int SCR>
__device__ __forceinline__ float4 wide_chunk(const WideRow<SCR>& r, int k, float sinv) {
  const uint4& v = r.w[SCR == SCR_BF16 ? k / 2 : 0];
  if constexpr (SCR == SCR_BF16) {
    const uint32_t w0 = (k & 1) ? v.z : v.x, w1 = (k & 1) ? v.w : v.y;
    return make_float4(__uint_as_float(w0 << 16), __uint_as_float(w0 & 0xFFFF0000u), __uint_as_float(w1 << 16),
                       __uint_as_float(w1 & 0xFFFF0000u));
  } else {
    const int w = (int)(k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w);
    if constexpr (SCR == SCR_INT8) {
      return make_float4((float)((w << 24) >> 24) * sinv, (float)((w << 16) >> 24) * sinv,
                         (float)((w << 8) >> 24) * sinv, (float)(w >> 24) * sinv);
    } else {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
      if constexpr (DK == F32L2) return make_float4(lo[0] * sinv, lo[1] * sinv, hi[0] * sinv, hi[1] * sinv);
      return make_float4(lo[0], lo[1], hi[0], hi[1]);
    }
  }
}

// The screen of screen_filter for rows of 16 chunks per lane and more, in
// the wave-per-row layout: qrow is the point's float32 row, prow its narrow
// row (whose codes the int8 cosine screen takes).  Same contract and margins.
template <int DK, int SCR>
__device__ __forceinline__ int screen_filter_wide(const BeamArgs& A, const uint8_t* qrow, const uint8_t* prow,
                                                  float np, float p_err, float p_scale, uint32_t* ids_lds, int cnt,
                                                  float w) {
  constexpr bool kIntDot = SCR == SCR_INT8 && DK == F32COS;
  const int lane = lane_id();
  const int Q = A.Q;
  const ScreenGammas gam = screen_gammas(A.d);
  float4 qv[4];
  uint4 qcode = make_uint4(0, 0, 0, 0);
  if constexpr (kIntDot) {
    WideRow<SCR> pr;
    load_wide<SCR>(pr, prow, Q, lane);
    qcode = pr.w[0];
  } else {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int q = 4 * lane + k;
      qv[k] = q < Q ? *reinterpret_cast<const float4*>(qrow + 16 * (size_t)q) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  const int myt = lane >> 3;
  int kept = 0;
  for (int r0 = 0; r0 < cnt; r0 += kWideRows) {
    uint32_t id[kWideRows];
#pragma unroll
    for (int t = 0; t < kWideRows; t++) id[t] = ids_lds[r0 + t < cnt ? r0 + t : r0];
    const bool dec = (lane & 7) == 0 && r0 + myt < cnt;
    const uint32_t myid = ids_lds[r0 + myt < cnt ? r0 + myt : r0];
    // every row's loads are issued before any is used
    const float4 tr = *reinterpret_cast<const float4*>(A.xs + (size_t)myid * A.xs_stride + A.xs_tail);
    WideRow<SCR> rw[kWideRows];
#pragma unroll
    for (int t = 0; t < kWideRows; t++) load_wide<SCR>(rw[t], A.xs + (size_t)id[t] * A.xs_stride, Q, lane);
    float own;
    float eps;
    if constexpr (kIntDot) {
      int acc[kWideRows];
#pragma unroll
      for (int t = 0; t < kWideRows; t++) {
        const uint4 v = rw[t].w[0];
        int s = __builtin_amdgcn_sdot4((int)qcode.x, (int)v.x, 0, false);
        s = __builtin_amdgcn_sdot4((int)qcode.y, (int)v.y, s, false);
        s = __builtin_amdgcn_sdot4((int)qcode.z, (int)v.z, s, false);
        acc[t] = __builtin_amdgcn_sdot4((int)qcode.w, (int)v.w, s, false);
      }
      own = 1.0f - (p_scale * tr.z) * (float)reduce_wide_rows<int>(acc);
      eps = screen_eps_i8(gam, p_err, np, tr.x, tr.y);
    } else {
      float acc[kWideRows];
#pragma unroll
      for (int t = 0; t < kWideRows; t++) {
        // squared L2 over fp8 or int8 codes scales each element by its
        // row's factor, which lane 8t loaded
        const float sinv = ((SCR == SCR_FP8 || SCR == SCR_INT8) && DK == F32L2)
                               ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tr.z), 8 * t))
                               : 1.0f;
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const float4 xb = wide_chunk<DK, SCR>(rw[t], k, sinv);
          if constexpr (DK == F32L2) {
            const float d0 = qv[k].x - xb.x, d1 = qv[k].y - xb.y, d2 = qv[k].z - xb.z, d3 = qv[k].w - xb.w;
            a = __builtin_fmaf(d0, d0, a);
            a = __builtin_fmaf(d1, d1, a);
            a = __builtin_fmaf(d2, d2, a);
            a = __builtin_fmaf(d3, d3, a);
          } else {
            a = __builtin_fmaf(qv[k].x, xb.x, a);
            a = __builtin_fmaf(qv[k].y, xb.y, a);
            a = __builtin_fmaf(qv[k].z, xb.z, a);
            a = __builtin_fmaf(qv[k].w, xb.w, a);
          }
        }
        acc[t] = a;
      }
      own = reduce_wide_rows<float>(acc);
      if constexpr (DK == F32COS) own = 1.0f - (SCR == SCR_FP8 ? tr.z * own : own);
      eps = screen_eps<DK>(own, gam, tr.x, np, DK == F32COS ? tr.y : 0.0f, SCR == SCR_FP8 ? tr.z : 1.0f);
    }
    const bool keep = dec && !(own - eps > w);
    wave_sync();  // every read of this round's ids precedes the compaction
    const uint64_t m = ballot(keep);
    if (keep) ids_lds[kept + popc64(m & lanes_below())] = myid;
    kept += popc64(m);
    wave_sync();
  }
  return kept;
}

template <int EFMAX, int HSLOTS>
struct WaveLDS {
  uint32_t htab[HSLOTS];  // visited ids; after the search, the prune's sort buffer
  uint64_t bkeys[2][EFMAX];
  uint8_t bflag[2][EFMAX];
  uint64_t ckey[64];
  uint32_t cid[64];
  uint32_t sid[256];   // new ids of one super-chunk of neighbours
  uint64_t skey[256];  // their keys
  uint32_t alive[HSLOTS / 64];
  uint32_t nspill;
};

// Fibonacci hashing: the top log2(HSLOTS) bits of u * 2^32 / golden ratio.
template <int HSLOTS>
__device__ __forceinline__ uint32_t hash_slot(uint32_t u) {
  return (u * 0x9E3779B1u) >> (32 - __builtin_ctz((unsigned)HSLOTS));
}

// Rows as the prune needs them.
struct RowSet {
  const uint8_t* x;
  int64_t stride;
  int Q;
};

// Distances from the register-resident row `a` (norm an) to the `cnt`
// (<= 64) rows whose ids are in ids_lds; writes keys into keys_lds.
template <int NCH, int L>
constexpr int default_rb() {
  return (NCH >= 8) ? 1 : ((8 / NCH) < L ? (8 / NCH) : L);
}

// RB rows per lane group are loaded before any is reduced, so a wave keeps
// (64 / L) * RB row gathers in flight.
template <int DK, int L, int NCH, int RB = default_rb<NCH, L>()>
__device__ __forceinline__ void batch_dists_rs(const RowSet& X, const Chunks<L, NCH>& a, uint32_t an,
                                               const uint32_t* ids_lds, int cnt, uint64_t* keys_lds) {
  constexpr int G = 64 / L;
  const int lane = lane_id();
  const int grp = lane / L, g = lane % L;
  for (int r0 = 0; r0 < cnt; r0 += G * RB) {
    Chunks<L, NCH> rc[RB];
    uint32_t u[RB];
#pragma unroll
    for (int t = 0; t < RB; t++) {
      int r = r0 + t * G + grp;
      u[t] = ids_lds[r < cnt ? r : 0];
      load_chunks<L, NCH>(rc[t], X.x + (size_t)u[t] * X.stride, X.Q, g);
    }
#pragma unroll
    for (int t = 0; t < RB; t++) {
      int r = r0 + t * G + grp;
      uint32_t hi = group_dist<DK, L, NCH>(a, an, rc[t], X.Q, g);
      if (r < cnt && g == 0) keys_lds[r] = make_key(hi, u[t]);
    }
  }
  wave_sync();
}

// Ascending bitonic sort of M (a power of two >= 64) entries in LDS by one wave.
template <typename T>
__device__ __forceinline__ void wave_sort_lds(T* a, int M) {
  const int lane = lane_id();
  for (int kb = 2; kb <= M; kb <<= 1) {
    for (int jb = kb >> 1; jb > 0; jb >>= 1) {
      for (int i = lane; i < M; i += 64) {
        int ixj = i ^ jb;
        if (ixj > i) {
          T a0 = a[i], a1 = a[ixj];
          bool up = (i & kb) == 0;
          if ((a0 > a1) == up) {
            a[i] = a1;
            a[ixj] = a0;
          }
        }
      }
      wave_sync();
    }
  }
}

// The same sort in device memory (the expanded sets longer than the
// on-chip bound): each pass's stores are made visible, and the vector L1's
// stale lines dropped, before the next pass reads them.
__device__ __forceinline__ void wave_sort_global(uint64_t* a, int M) {
  const int lane = lane_id();
  for (int kb = 2; kb <= M; kb <<= 1) {
    for (int jb = kb >> 1; jb > 0; jb >>= 1) {
      for (int i = lane; i < M; i += 64) {
        int ixj = i ^ jb;
        if (ixj > i) {
          uint64_t a0 = a[i], a1 = a[ixj];
          bool up = (i & kb) == 0;
          if ((a0 > a1) == up) {
            a[i] = a1;
            a[ixj] = a0;
          }
        }
      }
      __threadfence();
      wave_sync();
    }
  }
}

// A word of the prune's live-candidate bits: in LDS, or (GA) in device
// memory, where other lanes clear bits with atomics at L2, so the word is
// read past the vector L1.
template <bool GA>
__device__ __forceinline__ uint32_t alive_word(const uint32_t* alive, int w) {
  if constexpr (GA) return __hip_atomic_load(alive + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return alive[w];
}

// Greedy occlusion prune of the mc candidates sk[0..mc) (sorted by key; the
// key's high word is d(p, c)).  alive holds >= mc bits of LDS scratch, cid /
// ckey 64 entries each.  Writes the kept ids to out[0..kept) (lane 0) and
// returns kept; *pe counts the pair distances evaluated (each later live
// candidate against each kept one until it dies).
// GA: alive is in device memory (candidate sets beyond the on-chip bound).
template <int DK, int L, int NCH, bool GA = false>
__device__ int prune_wave(const RowSet& X, float alpha, int R, const uint64_t* sk, int mc,
                          uint32_t* alive, uint32_t* cid, uint64_t* ckey, uint32_t* out,
                          unsigned long long* pe) {
  const int lane = lane_id();
  const int g = lane % L;
  for (int w = lane; w < (mc + 31) / 32; w += 64) {
    int valid = mc - w * 32;
    const uint32_t v = valid >= 32 ? 0xFFFFFFFFu : ((1u << valid) - 1u);
    if constexpr (GA) __hip_atomic_store(alive + w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else alive[w] = v;
  }
  if constexpr (GA) __threadfence();
  wave_sync();
  int kept = 0, i = 0;
  while (kept < R) {
    int nxt = -1;
    for (int base = i & ~63; base < mc; base += 64) {
      int j = base + lane;
      bool live = j >= i && j < mc && ((alive_word<GA>(alive, j >> 5) >> (j & 31)) & 1u);
      uint64_t m = ballot(live);
      if (m) {
        nxt = base + __ffsll((long long)m) - 1;
        break;
      }
    }
    if (nxt < 0) break;
    i = nxt;
    uint32_t kid = key_id(sk[i]);
    if (lane == 0) out[kept] = kid;
    kept++;
    if (kept == R) break;
    Chunks<L, NCH> kc;
    load_chunks<L, NCH>(kc, X.x + (size_t)kid * X.stride, X.Q, g);
    uint32_t kn = 0;
    if constexpr (DK == U8L2) kn = group_sum_u32<L>(u8_selfdot<L, NCH>(kc));
    for (int base = i + 1; base < mc; base += 64) {
      int j = base + lane;
      bool live = j < mc && ((alive_word<GA>(alive, j >> 5) >> (j & 31)) & 1u);
      uint64_t m = ballot(live);
      int nl = popc64(m);
      if (nl == 0) continue;
      *pe += (unsigned long long)nl;
      int pos = popc64(m & lanes_below());
      if (live) cid[pos] = key_id(sk[j]);
      wave_sync();
      batch_dists_rs<DK, L, NCH>(X, kc, kn, cid, nl, ckey);
      if (live) {
        float dkc = hi_to_float<DK>(key_hi(ckey[pos]));
        float dpc = hi_to_float<DK>(key_hi(sk[j]));
        float scaled = alpha * dkc;
        if (scaled <= dpc) atomicAnd(&alive[j >> 5], ~(1u << (j & 31)));
      }
      if constexpr (GA) __threadfence();  // the cleared bits, before the next read
      wave_sync();
    }
    i++;
  }
  return kept;
}

// Waves per SIMD the register budget aims at: more searches in flight hide
// more gather latency.  Four for rows of one or two chunks per lane with a
// table of at most 1024 slots (at most about 10 KB of LDS per wave), three
// for such rows with larger tables and for the screened kernels of such
// rows (whose screen needs more than the 128 registers of four), two for
// the longest rows, else whatever the registers allow.
template <int NCH, int HS, int SCR = 0>
constexpr int beam_waves_per_eu() {
  return (NCH <= 2 && HS <= 1024 && SCR == 0) ? 4 : (NCH <= 2 ? 3 : (NCH >= 16 ? 2 : 1));
}

// ------------------------------------------------------------ Gram-tile prune
// Float32 rows of more than 64 chunks: the occlusion prune's pair distances
// come from the candidates' Gram matrix on matrix cores (each candidate row
// read once per 32-row block instead of once per kept candidate),
// d~(a,c) = G_aa + G_cc - 2 G_ac (cosine: 1 - G_ac).  A test whose outcome
// the rounding margin cannot settle is recomputed exactly in the declared
// order, so the kept lists and the pair count are those of prune_wave.

typedef float gram_f32x16 __attribute__((ext_vector_type(16)));

// Row of the 32x32 accumulator held in register r of lane l.
__device__ __forceinline__ int gram_acc_row(int r, int lane) { return (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3); }

// G[i * kGramMax + j] = <c_i, c_j> for j > i, candidates c_i = row of sk[i],
// one 32-row block-row at a time.  Lanes l and l+32 read chunks c and c+1 of
// the same row: the four elements
// of each 16-byte chunk are four k-steps of the 32x32x2 product.  Rows are
// taken in steps of eight chunks (one 128-byte line per row), double-
// buffered: a step's four loads per operand are issued together, one step
// ahead of the products, so each line is used up while it is in the vector
// L1.  Rows past mc read candidate 0 (in bounds; their results are not
// stored), so the loop has no per-lane branches.
__device__ __forceinline__ void gram_mfma4(gram_f32x16& acc, const float4& a, const float4& b) {
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, acc, 0, 0, 0);
}

__device__ __forceinline__ void gram_step_load(float4* fa, float4* fb, const uint8_t* pa, const uint8_t* pb,
                                               int s) {
#pragma unroll
  for (int j = 0; j < 4; j++) {
    fa[j] = *reinterpret_cast<const float4*>(pa + 128 * (size_t)s + 32 * j);
    fb[j] = *reinterpret_cast<const float4*>(pb + 128 * (size_t)s + 32 * j);
  }
}

__device__ __forceinline__ void gram_step_mfma(gram_f32x16& acc, const float4* fa, const float4* fb) {
#pragma unroll
  for (int j = 0; j < 4; j++) gram_mfma4(acc, fa[j], fb[j]);
}

// acc += the 32x32 tile <a_i, b_j>: lane l reads row a_(l & 31) at pa and
// row b_(l & 31) at pb (both already offset by 16 (l >> 5) bytes), Q chunks.
__device__ __forceinline__ void gram_tile_acc(gram_f32x16& acc, const uint8_t* pa, const uint8_t* pb, int Q) {
  const int h = lane_id() >> 5;
  const int NS = Q / 8;  // whole steps; the rest in pairs, an odd last chunk apart
  float4 a0[4], b0[4], a1[4], b1[4];
  if (NS > 0) gram_step_load(a0, b0, pa, pb, 0);
  int s = 0;
  for (; s + 1 < NS; s += 2) {
    gram_step_load(a1, b1, pa, pb, s + 1);
    gram_step_mfma(acc, a0, b0);
    if (s + 2 < NS) gram_step_load(a0, b0, pa, pb, s + 2);
    gram_step_mfma(acc, a1, b1);
  }
  if (s < NS) gram_step_mfma(acc, a0, b0);
  int c = 8 * NS;
  for (; c + 1 < Q; c += 2) {
    const float4 a = *reinterpret_cast<const float4*>(pa + 16 * (size_t)c);
    const float4 b = *reinterpret_cast<const float4*>(pb + 16 * (size_t)c);
    gram_mfma4(acc, a, b);
  }
  if (c < Q) {  // the last chunk: lanes of the upper half contribute zero
    float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a;
    if (h == 0) {
      a = *reinterpret_cast<const float4*>(pa + 16 * (size_t)c);
      b = *reinterpret_cast<const float4*>(pb + 16 * (size_t)c);
    }
    gram_mfma4(acc, a, b);
  }
}

// Block-row I of G: G[i * kGramMax + j] = <c_i, c_j> for i in block I and
// j > i (the tiles (I, J), J >= I).
__device__ __forceinline__ void gram_row_block(const RowSet& X, const uint64_t* sk, int mc, float* G, int I) {
  const int lane = lane_id();
  const int nb = (mc + 31) / 32;
  const int h = lane >> 5;
  {
    const int ra = 32 * I + (lane & 31);
    const uint8_t* pa = X.x + (size_t)key_id(sk[ra < mc ? ra : 0]) * X.stride + 16 * h;
    for (int J = I; J < nb; J++) {
      const int rb = 32 * J + (lane & 31);
      const uint8_t* pb = X.x + (size_t)key_id(sk[rb < mc ? rb : 0]) * X.stride + 16 * h;
      gram_f32x16 acc;
#pragma unroll
      for (int e = 0; e < 16; e++) acc[e] = 0.0f;
      gram_tile_acc(acc, pa, pb, X.Q);
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int i = 32 * I + gram_acc_row(r, lane);
        const int j = 32 * J + (lane & 31);
        if (i < mc && j < mc && j > i) G[i * kGramMax + j] = acc[r];
      }
    }
  }
}

typedef __bf16 gram_bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void gram_mfma_split(gram_f32x16& acc, const gram_bf16x8& ah, const gram_bf16x8& al,
                                                const gram_bf16x8& bh, const gram_bf16x8& bl) {
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
}

// gram_row_block from the split rows: <a,c> ~ <ah,ch> + <ah,cl> + <al,ch> (the
// dropped <al,cl> and the residuals e are covered by the margin).  A
// 16-element step is one 32x32x16 product per term: lane l reads the eight
// k-values at bytes 16 (l >> 5) of the step's hi and lo halves, so lanes l
// and l + 32 together take the step's whole 64 bytes of the row.  Same
// accumulator layout and stores as gram_row_block.
__device__ __forceinline__ void gram_row_block_split(const GramSplit& gs, const uint64_t* sk, int mc, float* G,
                                                     int I) {
  const int lane = lane_id();
  const int nb = (mc + 31) / 32;
  const int K = (int)(gs.stride / 64);
  const uint8_t* base = gs.p + 16 * (size_t)(lane >> 5);
  {
    const int ra = 32 * I + (lane & 31);
    const size_t oa = (size_t)key_id(sk[ra < mc ? ra : 0]) * gs.stride;
    for (int J = I; J < nb; J++) {
      const int rb = 32 * J + (lane & 31);
      const size_t ob = (size_t)key_id(sk[rb < mc ? rb : 0]) * gs.stride;
      gram_f32x16 acc;
#pragma unroll
      for (int e = 0; e < 16; e++) acc[e] = 0.0f;
      gram_bf16x8 ah[kGramPF16], al[kGramPF16], bh[kGramPF16], bl[kGramPF16];
#pragma unroll
      for (int u = 0; u < kGramPF16; u++)
        if (u < K) {
          ah[u] = *reinterpret_cast<const gram_bf16x8*>(base + oa + 64 * (size_t)u);
          al[u] = *reinterpret_cast<const gram_bf16x8*>(base + oa + 64 * (size_t)u + 32);
          bh[u] = *reinterpret_cast<const gram_bf16x8*>(base + ob + 64 * (size_t)u);
          bl[u] = *reinterpret_cast<const gram_bf16x8*>(base + ob + 64 * (size_t)u + 32);
        }
      int c = 0;
      for (; c + kGramPF16 <= K; c += kGramPF16) {
#pragma unroll
        for (int u = 0; u < kGramPF16; u++) {
          gram_mfma_split(acc, ah[u], al[u], bh[u], bl[u]);
          const int nx = c + u + kGramPF16;
          if (nx < K) {
            ah[u] = *reinterpret_cast<const gram_bf16x8*>(base + oa + 64 * (size_t)nx);
            al[u] = *reinterpret_cast<const gram_bf16x8*>(base + oa + 64 * (size_t)nx + 32);
            bh[u] = *reinterpret_cast<const gram_bf16x8*>(base + ob + 64 * (size_t)nx);
            bl[u] = *reinterpret_cast<const gram_bf16x8*>(base + ob + 64 * (size_t)nx + 32);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kGramPF16; u++)
        if (c + u < K) gram_mfma_split(acc, ah[u], al[u], bh[u], bl[u]);
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int i = 32 * I + gram_acc_row(r, lane);
        const int j = 32 * J + (lane & 31);
        if (i < mc && j < mc && j > i) G[i * kGramMax + j] = acc[r];
      }
    }
  }
}

// Margin for d~ against the exact declared-order distance (standard model:
// every elementary operation of the matrix-core sum is taken to err by up to
// 2^-23 relative, twice the float32 unit roundoff, since its internal order
// and rounding are the hardware's; the declared order errs by gc):
//   squared L2: |d~ - d| <= (gg + 2u)(1 + gg) (|a| + |c|)^2, with
//     (|a| + |c|)^2 <= 2 (G_aa + G_cc) / (1 - gg); the exact value adds
//     gc (|d~| + that);
//   cosine: |G_ac - <a,c>| <= gg |a||c|, the declared order gc |a||c|, two
//     roundings of 1 - s at most 2u (1 + |a||c|) each, |a||c| <=
//     sqrt(G_aa G_cc) / (1 - gg).
// From the bfloat16 split the entries are sums of 3d exact products whose
// magnitudes add up to at most (1 + 2^-8)^2 (1 + 2^-7 (1 + 2^-8)) |a||c| <=
// 1.016 |a||c|, and the terms left out (<al,cl> and the residuals) are at
// most 3.01 * 2^-16 |a||c|: gg = 3.1 * 2^-16 + 1.016 gamma(3d + 4).
// Underflow is outside the standard model: the matrix cores may flush
// operands and partial sums below 2^-126 to zero, and gradual underflow
// errs absolutely.  An operand flushed to zero drops a product of at most
// 2^-126 |c_k| (a sum over the row of at most 2^-126 sqrt(d) |c|, k of them
// per element with k = 3 for the split), and each of the nk flushed or
// underflowed partial results at most 2^-126; with |a| <= sqrt(|G_aa| +
// 2^-120) (the norm's own float32 sum underflows by at most d 2^-149), the
// three entries of d~ add 2^-124 (k sqrt(d) (|a| + |c|) + 2 nk), the one
// entry of 1 - G_ac 2^-125 (k sqrt(d) (|a| + |c|) + nk); negligible for
// rows of normal magnitude, it sends tests on tiny rows to the exact
// recomputation.  The result is doubled.
template <int DK>
__device__ __forceinline__ float gram_eps(float dt, float gaa, float gcc, int d, bool split) {
  const float u = 5.9604645e-08f;  // 2^-24
  const int nk = split ? 3 * d + 4 : d + 4;
  float gg = nk * (2.0f * u) / (1.0f - nk * (2.0f * u));
  if (split) gg = 3.1f * 1.5258789e-05f + 1.016f * gg;
  const float gc = (d / 16 + 8) * u / (1.0f - (d / 16 + 8) * u);
  const float sn = fabsf(gaa) + fabsf(gcc);
  float eps;
  if constexpr (DK == F32L2) {
    const float s2 = 2.0f * sn / (1.0f - gg);
    const float b = (gg + 2.0f * u) * (1.0f + gg) * s2;
    eps = b + gc * (fabsf(dt) + b);
  } else {
    const float nn = __builtin_sqrtf(fabsf(gaa) * fabsf(gcc)) / (1.0f - gg);
    eps = (gg + gc) * nn + 4.0f * u * (1.0f + nn);
  }
  // Underflow: flushed operands contribute at most 2^-126 sqrt(d) (|a| + |c|)
  // per product plane (k planes), bounded without roots by
  // sqrt(d) sqrt(y) <= (d + y) / 2 with y = |G| + 2^-120, and nk flushed or
  // underflowed partial results at most 2^-126 each (twice for L2's 2 G_ac):
  //   L2: 2^-124 (k (d + sn / 2 + 2^-120) + 2 nk), cosine: 2^-125 (k (...) + nk),
  // written as c1 sn + c0 with c0, c1 fixed by d (a square root per pair
  // here cost the 10^6 x 960 scaffold a tenth of its time).
  const float kf = split ? 3.0f : 1.0f;
  const float sc = DK == F32L2 ? 4.7019774e-38f : 2.3509887e-38f;  // 2^-124, 2^-125
  const float c0 = sc * (kf * ((float)d + 7.5231638e-37f) + (DK == F32L2 ? 2.0f : 1.0f) * (float)nk);
  const float c1 = sc * kf * 0.5f;
  eps += __builtin_fmaf(c1, sn, c0);
  return 2.0f * eps;
}

// Exact declared-order float32 distance between two rows read chunk by
// chunk (the same partial slots, tree and cross-lane levels as group_dist,
// so the same bits, without holding either row in registers).
template <int DK, int L, int NCH>
__device__ __forceinline__ float group_dist_stream(const uint8_t* ra, const uint8_t* rb, int Q, int g) {
  constexpr int S = 16 / L;
  float p[S];
#pragma unroll
  for (int s = 0; s < S; s++) p[s] = 0.0f;
#pragma unroll 4
  for (int i = 0; i < NCH; i++) {
    const int q = g + L * i;
    if (q < Q) {
      float& acc = p[i % S];
      const float4 xa = *reinterpret_cast<const float4*>(ra + 16 * (size_t)q);
      const float4 xb = *reinterpret_cast<const float4*>(rb + 16 * (size_t)q);
      if constexpr (DK == F32L2) {
        const float d0 = xa.x - xb.x, d1 = xa.y - xb.y, d2 = xa.z - xb.z, d3 = xa.w - xb.w;
        acc = __builtin_fmaf(d0, d0, acc);
        acc = __builtin_fmaf(d1, d1, acc);
        acc = __builtin_fmaf(d2, d2, acc);
        acc = __builtin_fmaf(d3, d3, acc);
      } else {
        acc = __builtin_fmaf(xa.x, xb.x, acc);
        acc = __builtin_fmaf(xa.y, xb.y, acc);
        acc = __builtin_fmaf(xa.z, xb.z, acc);
        acc = __builtin_fmaf(xa.w, xb.w, acc);
      }
    }
  }
#pragma unroll
  for (int off = S / 2; off >= 1; off >>= 1)
#pragma unroll
    for (int s = 0; s < off; s++) p[s] = p[s] + p[s + off];
  float v = p[0];
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
  if constexpr (DK == F32COS) v = 1.0f - v;
  return v;
}

// The greedy prune of prune_wave, its pair tests decided from the Gram
// matrix where the margin allows.  A block-row of G is computed (then
// fenced) when the greedy first keeps a candidate of that block: with
// candidates sorted by distance and at most R kept, later blocks often are
// never needed.  The diagonal comes from norm (|x|^2 of every row, any
// float32 order: within the same margin).  G is this wave's kGramMax^2
// scratch; *rc counts the exact recomputations.
template <int DK, int L, int NCH>
__device__ int prune_gram(const RowSet& X, int d, const GramSplit& split, const float* norm, float alpha, int R,
                          const uint64_t* sk, int mc, float* G, uint32_t* alive, uint32_t* cid, uint64_t* ckey,
                          uint32_t* out, unsigned long long* pe, unsigned long long* rc) {
  uint32_t rows_done = 0;  // block-rows of G computed so far (at most 32)
  const int lane = lane_id();
  const int g = lane % L;
  for (int w = lane; w < (mc + 31) / 32; w += 64) {
    int valid = mc - w * 32;
    alive[w] = valid >= 32 ? 0xFFFFFFFFu : ((1u << valid) - 1u);
  }
  wave_sync();
  const float u8 = 8.0f * 5.9604645e-08f;
  int kept = 0, i = 0;
  while (kept < R) {
    int nxt = -1;
    for (int base = i & ~63; base < mc; base += 64) {
      int j = base + lane;
      bool live = j >= i && j < mc && ((alive[j >> 5] >> (j & 31)) & 1u);
      uint64_t m = ballot(live);
      if (m) {
        nxt = base + __ffsll((long long)m) - 1;
        break;
      }
    }
    if (nxt < 0) break;
    i = nxt;
    uint32_t kid = key_id(sk[i]);
    if (lane == 0) out[kept] = kid;
    kept++;
    if (kept == R) break;
    if (!((rows_done >> (i >> 5)) & 1u)) {
      if (split.p)
        gram_row_block_split(split, sk, mc, G, i >> 5);
      else
        gram_row_block(X, sk, mc, G, i >> 5);
      // the tiles were written by other lanes, and this slot's scratch may
      // sit in the vector L1 from an earlier search: make the stores
      // visible and drop stale lines before reading them back
      __threadfence();
      rows_done |= 1u << (i >> 5);
    }
    const float gaa = norm[kid];
    const uint8_t* krow = X.x + (size_t)kid * X.stride;
    for (int base = i + 1; base < mc; base += 64) {
      int j = base + lane;
      bool live = j < mc && ((alive[j >> 5] >> (j & 31)) & 1u);
      uint64_t m = ballot(live);
      int nl = popc64(m);
      if (nl == 0) continue;
      *pe += (unsigned long long)nl;
      bool kill = false, unsure = false;
      float dpc = 0.0f;
      if (live) {
        dpc = hi_to_float<DK>(key_hi(sk[j]));
        const float gcc = norm[key_id(sk[j])], gac = G[i * kGramMax + j];
        const float dt = DK == F32L2 ? (gaa + gcc) - 2.0f * gac : 1.0f - gac;
        const float eps = gram_eps<DK>(dt, gaa, gcc, d, split.p != nullptr);
        // bounds on fl(alpha * exact), widened for their own roundings
        const float up = alpha * (dt + eps), lo = alpha * (dt - eps);
        if (up + fabsf(up) * u8 < dpc) kill = true;
        else if (!(lo - fabsf(lo) * u8 > dpc)) unsure = true;
      }
      const uint64_t mu = ballot(unsure);
      const int nu = popc64(mu);
      if (nu) {  // exact distances for the tests the margin left open
        *rc += (unsigned long long)nu;
        const int pos = popc64(mu & lanes_below());
        if (unsure) cid[pos] = key_id(sk[j]);
        wave_sync();
        constexpr int G4 = 64 / L;
        float* cd = reinterpret_cast<float*>(ckey);
        for (int r0 = 0; r0 < nu; r0 += G4) {
          const int r = r0 + lane / L;
          const uint32_t cu = cid[r < nu ? r : 0];
          const float v = group_dist_stream<DK, L, NCH>(krow, X.x + (size_t)cu * X.stride, X.Q, g);
          if (r < nu && g == 0) cd[r] = v;
        }
        wave_sync();
        if (unsure) kill = alpha * cd[pos] <= dpc;
      }
      if (kill) atomicAnd(&alive[j >> 5], ~(1u << (j & 31)));
      wave_sync();
    }
    i++;
  }
  return kept;
}

template <int DK, int L, int NCH, int EFMAX, int HSLOTS, bool SEARCH, int SCR = SCR_NONE, bool LOG = false>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(beam_waves_per_eu<NCH, HSLOTS, SCR>())))
k_beam(BeamArgs A) {
  __shared__ WaveLDS<EFMAX, HSLOTS> S;
  const int lane = lane_id();
  const int g = lane % L;
  const int64_t wslot = blockIdx.x;
  uint32_t* bits = A.spill_bits + wslot * A.spill_words;
  uint32_t* slist = A.spill_list + wslot * (int64_t)A.spill_cap;
  // this slot's expanded list: Ecap keys, then Ecap bits of prune scratch
  uint64_t* E = A.Ebuf + wslot * ((int64_t)A.Ecap + A.Ecap / 64);
  constexpr uint32_t HMASK = HSLOTS - 1;
  constexpr int HCAP = HSLOTS / 2 - 64;  // load <= 1/2; checked after every 64 insertions
  // rows in flight per lane group, sized to the register budget above
  constexpr int kRB = (NCH >= 16) ? 1 : (NCH == 1 ? (HSLOTS <= 1024 ? 8 : 12) : 16 / NCH);
  constexpr bool kRankBits = !SEARCH && NCH >= 2 && NCH <= 4;  // see BeamArgs::rank
  RowSet X{A.x, A.stride, A.Q};

  unsigned long long my_evals = 0, my_exp = 0, my_pe = 0, my_spilled = 0, my_rej = 0, my_rc = 0;
#ifdef FG_PROFILE
  unsigned long long prof[16] = {};
#endif
  FG_T0();

  // wave-uniform scalars (the slice walk stays in scalar registers)
  int xq = (int)(blockIdx.x & 7), xfail = 0;
  const int64_t xslice = (A.nitems + 7) / 8;
  for (;;) {
    unsigned long long item = 0;
    if (A.xqueue) {
      int64_t it = -1;
      while (xfail < 8) {
        unsigned int k = 0;
        if (lane == 0) k = atomicAdd(&A.xqueue[xq], 1u);
        k = (unsigned int)__builtin_amdgcn_readfirstlane((int)k);
        const int64_t c = (int64_t)xq * xslice + (int64_t)k;
        if ((int64_t)k < xslice && c < A.nitems) {
          it = c;
          break;
        }
        xq = (xq + 1) & 7;  // this slice is done: the next one (each is visited once)
        xfail++;
      }
      if (it < 0) break;
      item = (unsigned long long)it;
    } else {
      if (lane == 0) item = atomicAdd(A.queue, 1ull);
      item = __shfl(item, 0, 64);
      if ((int64_t)item >= A.nitems) break;
    }

    const int64_t p = SEARCH ? (int64_t)item : (A.order ? (int64_t)A.order[item] : A.b + (int64_t)item * A.B);
    if constexpr (!SEARCH)
      if (p >= A.n) continue;  // an order slot left empty (never, for a permutation)
    int ef = A.ef;
    const uint32_t* roots = A.roots;
    if constexpr (!SEARCH) {
      if (A.inst_of) {
        const uint32_t inst = A.inst_of[p];
        if (inst == 0xFFFFu) continue;  // an unused id between instances
        ef = A.inst_ef[inst];
        roots = A.inst_roots + (size_t)inst * A.T;
        // a query and its candidates share the instance: its zero chunks
        // add exactly nothing, so they are not read (rows of up to 64
        // chunks; longer rows keep the register budget of the Gram prune)
        if constexpr (NCH <= 4) X.Q = A.inst_q[inst];
      }
    }
    const uint8_t* qrow = SEARCH ? A.queries + (size_t)item * A.qstride : A.x + (size_t)p * A.stride;
    Chunks<L, NCH> qc;
    load_chunks<L, NCH>(qc, qrow, X.Q, g);
    uint32_t qn = 0;
    if constexpr (DK == U8L2) qn = group_sum_u32<L>(u8_selfdot<L, NCH>(qc));
    float qnorm = 0.0f;  // |p| for the cosine screen margin
    float qerr = 0.0f, qscale = 0.0f;
    NarrowChunks<NCH, SCR == SCR_NONE ? SCR_FP8 : SCR> qcodes{};  // the point's own codes (int8 cosine)
    if constexpr (SCR != SCR_NONE && DK == F32COS) {
      const uint8_t* prow = A.xs + (size_t)p * A.xs_stride;
      const float4 ptr = *reinterpret_cast<const float4*>(prow + A.xs_tail);
      qnorm = ptr.y;
      qerr = ptr.x;
      qscale = ptr.z;
      if constexpr (SCR == SCR_INT8 && NCH < 16) load_narrow<L, NCH, SCR>(qcodes, prow, X.Q, g);
    }

    for (int i = lane; i < HSLOTS; i += 64) S.htab[i] = FG_NONE;
    if (lane == 0) S.nspill = 0;
    wave_sync();
    int bsize = 0, cur = 0, hcount = 0, En = 0;
    bool spill = false, overflow = false;
    unsigned long long evals = 0;
    int lslot = -1;  // this point's visit-log slot
    if constexpr (LOG && !SEARCH) {
      lslot = A.log_slot[p];
      if (lslot >= A.log_nslots) lslot = -1;
    }

    // Visit then evaluate a list of candidate ids (roots or a CSR row), 256
    // ids per step: the id loads, the visited checks (and the device bitset
    // atomics once the LDS table is full) of all 256 are issued before any
    // result is waited for; the new ids' rows are gathered 64*RB/L at a time;
    // keys that can still enter the beam are merged 64 at a time.
    auto process = [&](const uint32_t* list, const uint2* plist, int64_t len) {
      for (int64_t base = 0; base < len; base += 256) {
        uint32_t u[4], rk[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
          int64_t j = base + k * 64 + lane;
          u[k] = FG_NONE;
          rk[k] = FG_NONE;
          if (j < len) {
            if (kRankBits && plist) {
              const uint2 pr = plist[j];
              u[k] = pr.x;
              rk[k] = pr.y;
            } else {
              u[k] = list[j];
            }
          }
        }
        bool isnew[4], need[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
          isnew[k] = false;
          need[k] = false;
          bool in_lds = false;
          if (u[k] < (uint64_t)A.n) {  // ids outside [0, n) are ignored
            if (spill) {
              need[k] = true;  // the bitset holds every visited id
            } else {
              uint32_t h = hash_slot<HSLOTS>(u[k]);
              for (;;) {
                uint32_t old = atomicCAS(&S.htab[h], FG_NONE, u[k]);
                if (old == FG_NONE) { isnew[k] = true; in_lds = true; break; }
                if (old == u[k]) break;
                h = (h + 1) & HMASK;
              }
            }
          }
          hcount += popc64(ballot(in_lds));
          if (!spill && hcount >= HCAP) {
            // Table full: move its ids into the device bitset (listed for
            // clearing), then use the bitset alone for this search.
            wave_sync();
            for (int i = lane; i < HSLOTS; i += 64) {
              uint32_t v = S.htab[i];
              if (v != FG_NONE) {
                if constexpr (kRankBits)
                  if (A.rank) v = A.rank[v];
                atomicOr(&bits[v >> 5], 1u << (v & 31));
                uint32_t idx = atomicAdd(&S.nspill, 1u);
                if ((int)idx < A.spill_cap) slist[idx] = v;
              }
            }
            spill = true;
          }
          wave_sync();
        }
        FG_TICK(0);
        uint32_t old[4];
        if constexpr (kRankBits) {
          uint32_t bi[4];
#pragma unroll
          for (int k = 0; k < 4; k++) {
            bi[k] = need[k] && A.rank ? (plist ? rk[k] : A.rank[u[k]]) : u[k];  // the bit of u
            if (need[k]) old[k] = atomicOr(&bits[bi[k] >> 5], 1u << (bi[k] & 31));
          }
#pragma unroll
          for (int k = 0; k < 4; k++)
            if (need[k] && !(old[k] & (1u << (bi[k] & 31)))) {
              isnew[k] = true;
              uint32_t idx = atomicAdd(&S.nspill, 1u);
              if ((int)idx < A.spill_cap) slist[idx] = bi[k];
            }
        } else {
#pragma unroll
          for (int k = 0; k < 4; k++)
            if (need[k]) old[k] = atomicOr(&bits[u[k] >> 5], 1u << (u[k] & 31));
#pragma unroll
          for (int k = 0; k < 4; k++)
            if (need[k] && !(old[k] & (1u << (u[k] & 31)))) {
              isnew[k] = true;
              uint32_t idx = atomicAdd(&S.nspill, 1u);
              if ((int)idx < A.spill_cap) slist[idx] = u[k];
            }
        }
        FG_TICK(1);
        int nnew = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
          uint64_t m = ballot(isnew[k]);
          if (isnew[k]) S.sid[nnew + popc64(m & lanes_below())] = u[k];
          nnew += popc64(m);
        }
        const unsigned long long before = evals;
        evals += (unsigned long long)nnew;
        if (nnew == 0) continue;
        wave_sync();
        if constexpr (LOG) {
          if (lslot >= 0)
            for (int i = lane; i < nnew; i += 64)
              if ((int64_t)(before + i) < A.log_cap) A.log_ids[lslot * A.log_cap + (int64_t)(before + i)] = S.sid[i];
        }
        if constexpr (SCR != SCR_NONE) {
          if (bsize == ef) {  // a full beam: its worst exact distance bounds entry
            const float w = ord_to_f32(key_hi(S.bkeys[cur][ef - 1]));
            int nx;
            if constexpr (NCH >= 16)
              nx = screen_filter_wide<DK, SCR>(A, qrow, A.xs + (size_t)p * A.xs_stride, qnorm, qerr, qscale, S.sid,
                                               nnew, w);
            else
              nx = screen_filter<DK, L, NCH, SCR>(A, qc, qnorm, qcodes, qerr, qscale, S.sid, nnew, w);
            my_rej += (unsigned long long)(nnew - nx);
            nnew = nx;
            FG_TICK(8);
            if (nnew == 0) continue;
          }
        }
        batch_dists_rs<DK, L, NCH, kRB>(X, qc, qn, S.sid, nnew, S.skey);
        FG_TICK(2);
        for (int c0 = 0; c0 < nnew; c0 += 64) {
          uint64_t ck = c0 + lane < nnew ? S.skey[c0 + lane] : FG_KEY_NONE;
          if (bsize == ef && ck >= S.bkeys[cur][ef - 1]) ck = FG_KEY_NONE;
          if (!ballot(ck != FG_KEY_NONE)) continue;
          ck = wave_sort64(ck);
          int nc = popc64(ballot(ck != FG_KEY_NONE));
          S.ckey[lane] = ck;
          wave_sync();
          // merge by co-ranking into the other buffer
          const uint64_t* Bk = S.bkeys[cur];
          const uint8_t* Bf = S.bflag[cur];
          uint64_t* Nk = S.bkeys[cur ^ 1];
          uint8_t* Nf = S.bflag[cur ^ 1];
          if (lane < nc) {
            int np = lane + lower_bound_lds<uint64_t>(Bk, bsize, ck);
            if (np < ef) { Nk[np] = ck; Nf[np] = 0; }
          }
          for (int jb = lane; jb < bsize; jb += 64) {
            uint64_t bk = Bk[jb];
            int np = jb + lower_bound_lds<uint64_t>(S.ckey, nc, bk);
            if (np < ef) { Nk[np] = bk; Nf[np] = Bf[jb]; }
          }
          bsize = bsize + nc < ef ? bsize + nc : ef;
          cur ^= 1;
          wave_sync();
        }
        FG_TICK(3);
      }
    };

    FG_TICK(6);
    process(roots, nullptr, A.T);
    if constexpr (LOG)
      if (lslot >= 0 && lane == 0) A.log_marks[(int64_t)lslot * kLogMarks] = (uint32_t)evals;
    for (;;) {
      int first = -1;
      for (int base = 0; base < bsize; base += 64) {
        int j = base + lane;
        uint64_t m = ballot(j < bsize && S.bflag[cur][j] == 0);
        if (m) { first = base + __ffsll((long long)m) - 1; break; }
      }
      if (first < 0) break;
      uint64_t key = S.bkeys[cur][first];
      wave_sync();
      if (lane == 0) S.bflag[cur][first] = 1;
      if constexpr (!SEARCH) {
        if (En >= A.Ecap) { overflow = true; break; }
        if (lane == 0) E[En] = key;
        En++;
      }
      my_exp++;
      uint32_t v = key_id(key);
      uint64_t s0 = A.off[v], s1 = A.off[v + 1];
      wave_sync();
      FG_TICK(5);
      process(A.ids + s0, kRankBits && A.idr ? A.idr + s0 : nullptr, (int64_t)(s1 - s0));
      if constexpr (LOG)
        if (lslot >= 0 && lane == 0 && En < kLogMarks) A.log_marks[(int64_t)lslot * kLogMarks + En] = (uint32_t)evals;
    }
    my_evals += evals;
    if constexpr (LOG)
      if (lslot >= 0 && lane == 0) {
        A.log_len[lslot] = (uint32_t)evals;
        for (int e = En + 1; e < kLogMarks; e++) A.log_marks[(int64_t)lslot * kLogMarks + e] = (uint32_t)evals;
      }

    if constexpr (SEARCH) {
      for (int i = lane; i < A.k; i += 64) {
        uint64_t kk = i < bsize ? S.bkeys[cur][i] : FG_KEY_NONE;
        A.out_ids[item * A.k + i] = i < bsize ? key_id(kk) : FG_NONE;
        if constexpr (DK == U8L2)
          reinterpret_cast<uint32_t*>(A.out_d)[item * A.k + i] = i < bsize ? key_hi(kk) : FG_NONE;
        else
          reinterpret_cast<float*>(A.out_d)[item * A.k + i] =
              i < bsize ? ord_to_f32(key_hi(kk)) : __builtin_inff();
      }
      if (lane == 0 && A.out_evals) A.out_evals[item] = (uint32_t)evals;
    } else {
      uint32_t* out = A.rows + (size_t)p * A.R;
      int kept = 0;
      if (overflow) {
        if (lane == 0) atomicOr(A.status, 1);
      } else {
        // Sort the expanded set (minus p), then prune it: in LDS (the
        // visited table's space) when it fits, else in place in this slot's
        // device buffer.
        const bool onchip = En <= HSLOTS / 2;
        uint64_t* sk = onchip ? reinterpret_cast<uint64_t*>(S.htab) : E;
        int M = 64;
        while (M < En) M <<= 1;  // <= Ecap: En < Ecap, a power of two
        wave_sync();
        for (int i = lane; i < M; i += 64) {
          uint64_t kk = FG_KEY_NONE;
          if (i < En) {
            kk = E[i];
            if (key_id(kk) == (uint32_t)p) kk = FG_KEY_NONE;
          }
          sk[i] = kk;
        }
        if (onchip) {
          wave_sync();
          wave_sort_lds<uint64_t>(sk, M);
        } else {
          __threadfence();
          wave_sync();
          wave_sort_global(sk, M);
        }
        int mc = 0;
        for (int base = 0; base < M; base += 64) mc += popc64(ballot(sk[base + lane] != FG_KEY_NONE));
        FG_TICK(5);
        bool gram = false;
        if constexpr (DK != U8L2 && NCH >= 16)
          gram = onchip && A.gram != nullptr && A.norm != nullptr && mc <= kGramMax && wslot < kGramSlots;
        if (gram) {
          float* G = A.gram + (size_t)wslot * kGramMax * kGramMax;
          kept = prune_gram<DK, L, NCH>(X, A.d, A.split, A.norm, A.alpha, A.R, sk, mc, G, S.alive, S.cid, S.ckey,
                                        out, &my_pe, &my_rc);
        } else if (onchip) {
          kept = prune_wave<DK, L, NCH>(X, A.alpha, A.R, sk, mc, S.alive, S.cid, S.ckey, out, &my_pe);
        } else {
          uint32_t* galive = reinterpret_cast<uint32_t*>(E + A.Ecap);
          kept = prune_wave<DK, L, NCH, true>(X, A.alpha, A.R, sk, mc, galive, S.cid, S.ckey, out, &my_pe);
        }
        FG_TICK(4);
      }
      for (int t = kept + lane; t < A.R; t += 64) out[t] = FG_NONE;
      if (lane == 0) A.cnt[p] = (uint32_t)kept;
    }

    FG_TICK(5);
    // Return the spill bitset to all-zero for the next query.
    if (spill) {
      my_spilled++;
      wave_sync();
      uint32_t ns = S.nspill;
      // Clear with atomics: the next query sets bits with atomics at L2, and
      // plain stores are not ordered against them.
      if ((int)ns <= A.spill_cap) {
        for (uint32_t t = lane; t < ns; t += 64) atomicAnd(&bits[slist[t] >> 5], 0u);  // listed bits' words
      } else {
        for (int64_t t = lane; t < A.spill_words; t += 64) atomicAnd(&bits[t], 0u);
      }
      __threadfence();
    }
    wave_sync();
    FG_TICK(7);
  }
  if (lane == 0) {
#ifdef FG_PROFILE
    for (int i = 0; i < 9; i++) atomicAdd(&fg_prof_cycles[i], prof[i]);
#endif
    atomicAdd(&A.counters[0], my_evals);
    atomicAdd(&A.counters[1], my_exp);
    atomicAdd(&A.counters[2], my_pe);
    atomicAdd(&A.counters[3], my_spilled);
    if (my_rej) atomicAdd(&A.counters[4], my_rej);
    if (my_rc) atomicAdd(&A.counters[5], my_rc);
  }
}

}  // namespace fg
