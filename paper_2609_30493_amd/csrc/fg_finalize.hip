// fg_finalize.hip -- finalize (Sec. 3): each point's harvested row united
// with its reverse edges, deduplicated, sorted by (d(p,.), id) and, when it
// holds more than R candidates (or always with reprune_all), occlusion-pruned
// to at most R.  One wave per point.
#include <vector>

#include "fg_internal.h"

namespace fg {

namespace {

constexpr int kFinCap = 2048;      // candidates per point held on chip (second tier)
constexpr int kFinSmall = 512;     // candidates held by the first tier
constexpr int kFinKeptMax = 1024;  // R bound of the big-row path

// One point: candidates gathered (ids outside [0, n) dropped), sorted,
// deduplicated, their distances to p, then sorted by key and pruned when
// more than R (or always with reprune_all).  m0 <= CAP.
template <int DK, int L, int NCH, int CAP>
__device__ void fin_point(const FinalizeArgs& A, int64_t p, uint32_t* cb, uint64_t* sk, uint32_t* alive,
                          uint32_t* cid, uint64_t* ckey, unsigned long long& ev, unsigned long long& pe,
                          unsigned long long& rcheck) {
  const int lane = lane_id();
  const int g = lane % L;
  RowSet X = A.X;  // a batched point and its candidates share the instance's own length
  if constexpr (DK != U8L2 && NCH <= 4)  // (uint8 rows: the register budget of five waves per SIMD)
    if (A.inst_q) X.Q = A.inst_q[A.inst_of[p]];
  uint32_t* out = A.g_nbrs + p * A.R;
  const int c = (int)min(A.cnt[p], (uint32_t)A.R);  // counts above R are not trusted
  const uint64_t r0 = A.revoff[p];
  const int m0 = c + (int)(A.revoff[p + 1] - r0);
  int M = 64;
  while (M < m0) M <<= 1;
  for (int i = lane; i < M; i += 64) {
    uint32_t v = i < c ? A.rows[p * A.R + i] : (i < m0 ? A.rev[r0 + (i - c)] : FG_NONE);
    cb[i] = v < (uint64_t)A.n ? v : FG_NONE;  // ids outside [0, n) are dropped
  }
  wave_sync();
  wave_sort_lds<uint32_t>(cb, M);
  // keep first occurrences (in place: a chunk is read before it is written)
  int m = 0;
  uint32_t carry = FG_NONE;  // last original value of the previous chunk
  for (int base = 0; base < M; base += 64) {
    int i = base + lane;
    uint32_t x = cb[i];
    uint32_t prev = __shfl(x, lane > 0 ? lane - 1 : 0, 64);
    if (lane == 0) prev = carry;
    carry = __shfl(x, 63, 64);
    bool keep = x != FG_NONE && x != prev;
    uint64_t msk = ballot(keep);
    wave_sync();
    if (keep) cb[m + popc64(msk & lanes_below())] = x;
    m += popc64(msk);
    wave_sync();
  }
  Chunks<L, NCH> qc;
  load_chunks<L, NCH>(qc, X.x + (size_t)p * X.stride, X.Q, g);
  uint32_t qn = 0;
  if constexpr (DK == U8L2) qn = group_sum_u32<L>(u8_selfdot<L, NCH>(qc));
  for (int base = 0; base < m; base += 64) {
    int cnt = m - base < 64 ? m - base : 64;
    batch_dists_rs<DK, L, NCH>(X, qc, qn, cb + base, cnt, sk + base);
  }
  ev += (unsigned long long)m;
  int Mk = 64;
  while (Mk < m) Mk <<= 1;
  for (int i = m + lane; i < Mk; i += 64) sk[i] = FG_KEY_NONE;
  wave_sync();
  wave_sort_lds<uint64_t>(sk, Mk);
  int kept;
  if (m > A.R || A.reprune_all) {
    bool gram = false;
    if constexpr (DK != U8L2 && NCH >= 16)
      gram = A.gram != nullptr && A.norm != nullptr && m <= kGramMax && blockIdx.x < kGramSlots;
    if (gram) {  // matrix-core pair distances with exact rechecks (see prune_gram)
      float* G = A.gram + (size_t)blockIdx.x * kGramMax * kGramMax;
      kept = prune_gram<DK, L, NCH>(X, A.d, A.split, A.norm, A.alpha, A.R, sk, m, G, alive, cid, ckey, out, &pe,
                                    &rcheck);
    } else {
      kept = prune_wave<DK, L, NCH>(X, A.alpha, A.R, sk, m, alive, cid, ckey, out, &pe);
    }
  } else {
    for (int i = lane; i < m; i += 64) out[i] = key_id(sk[i]);
    kept = m;
  }
  for (int t = kept + lane; t < A.R; t += 64) out[t] = FG_NONE;
  if (lane == 0) A.g_cnt[p] = (uint32_t)kept;
  wave_sync();
}

__device__ __forceinline__ void fin_flush(const FinalizeArgs& A, unsigned long long ev, unsigned long long pe,
                                          unsigned long long rcheck) {
  if (lane_id() == 0) {
    if (ev) atomicAdd(&A.counters[0], ev);
    if (pe) atomicAdd(&A.counters[1], pe);
    if (rcheck) atomicAdd(&A.counters[2], rcheck);
  }
}

// First tier: one wave per point with at most kFinSmall candidates (small
// LDS, many waves per compute unit); points with more are listed for the
// second tier (up to kFinCap) or for the big-row path.
template <int DK, int L, int NCH>
__global__ void __launch_bounds__(64) k_finalize(FinalizeArgs A) {
  __shared__ uint32_t cb[kFinSmall];
  __shared__ uint64_t sk[kFinSmall];
  __shared__ uint32_t alive[kFinSmall / 32];
  __shared__ uint32_t cid[64];
  __shared__ uint64_t ckey[64];
  unsigned long long ev = 0, pe = 0, rcheck = 0;
  for (int64_t i = blockIdx.x; i < A.n; i += gridDim.x) {
    // rows of more than 64 chunks (where it measured faster; shorter rows keep
    // their register budget of five waves per SIMD): the given order
    int64_t p = i;
    if constexpr (NCH >= 16)
      if (A.order) p = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)A.order[i]);
    if (p >= A.n) continue;  // an order slot left empty (never, for a permutation)
    const int m0 = (int)min(A.cnt[p], (uint32_t)A.R) + (int)(A.revoff[p + 1] - A.revoff[p]);
    if (m0 > kFinCap) {  // finished by the big-row path
      if (lane_id() == 0) A.big[atomicAdd(A.nbig, 1u)] = (uint32_t)p;
      continue;
    }
    if (m0 > kFinSmall) {  // finished by the second tier
      if (lane_id() == 0) A.mid[atomicAdd(A.nmid, 1u)] = (uint32_t)p;
      continue;
    }
    fin_point<DK, L, NCH, kFinSmall>(A, p, cb, sk, alive, cid, ckey, ev, pe, rcheck);
  }
  fin_flush(A, ev, pe, rcheck);
}

// Second tier: the listed points (count read on the device).
template <int DK, int L, int NCH>
__global__ void __launch_bounds__(64) k_finalize_mid(FinalizeArgs A) {
  __shared__ uint32_t cb[kFinCap];
  __shared__ uint64_t sk[kFinCap];
  __shared__ uint32_t alive[kFinCap / 32];
  __shared__ uint32_t cid[64];
  __shared__ uint64_t ckey[64];
  unsigned long long ev = 0, pe = 0, rcheck = 0;
  const uint32_t nm = *A.nmid;
  for (uint32_t k = blockIdx.x; k < nm; k += gridDim.x)
    fin_point<DK, L, NCH, kFinCap>(A, A.mid[k], cb, sk, alive, cid, ckey, ev, pe, rcheck);
  fin_flush(A, ev, pe, rcheck);
}

// ---------------------------------------------------------------- big rows
// A point with more than kFinCap candidates: its candidate keys live in a
// device segment [revoff[p] + p*R, + c + rc), sorted by segsort_u64, and are
// pruned in a stream of chunks of 64: each chunk is first tested against the
// rows kept so far (in order, stopping at the first that occludes), then
// resolved within itself.  Once R are kept, later chunks are still tested
// against the first R-1 kept rows, so the pair count equals that of the
// greedy prune run over the whole sorted list.
__global__ void k_fin_big_segs(FinalizeArgs A, KSeg* segs) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < *A.nbig; i += gridDim.x * blockDim.x) {
    uint32_t p = A.big[i];
    uint32_t c = min(A.cnt[p], (uint32_t)A.R);
    uint64_t rc = A.revoff[p + 1] - A.revoff[p];
    segs[i] = KSeg{A.revoff[p] + (uint64_t)p * A.R, (uint32_t)(c + rc), 0};
  }
}

template <int DK, int L, int NCH>
__global__ void __launch_bounds__(64) k_fin_big_keys(FinalizeArgs A, const KSeg* segs, uint64_t* keys) {
  __shared__ uint32_t cid[64];
  __shared__ uint64_t ckey[64];
  const int lane = lane_id(), g = lane % L;
  const uint32_t p = A.big[blockIdx.x];
  const KSeg sg = segs[blockIdx.x];
  const uint32_t c = min(A.cnt[p], (uint32_t)A.R);
  const uint64_t r0 = A.revoff[p];
  Chunks<L, NCH> qc;
  load_chunks<L, NCH>(qc, A.X.x + (size_t)p * A.X.stride, A.X.Q, g);
  uint32_t qn = 0;
  if constexpr (DK == U8L2) qn = group_sum_u32<L>(u8_selfdot<L, NCH>(qc));
  for (uint32_t base = 0; base < sg.len; base += 64) {
    uint32_t j = base + lane;
    uint32_t v = FG_NONE;
    if (j < sg.len) v = j < c ? A.rows[(uint64_t)p * A.R + j] : A.rev[r0 + (j - c)];
    bool ok = v < (uint64_t)A.n;
    uint64_t m = ballot(ok);
    int cnt = popc64(m);
    if (ok) cid[popc64(m & lanes_below())] = v;
    wave_sync();
    if (cnt) batch_dists_rs<DK, L, NCH>(A.X, qc, qn, cid, cnt, ckey);
    // keep each candidate at its own slot; invalid ids sort last
    uint64_t kk = FG_KEY_NONE;
    if (ok) kk = ckey[popc64(m & lanes_below())];
    if (j < sg.len) keys[sg.start + j] = kk;
    wave_sync();
  }
}

template <int DK, int L, int NCH>
__global__ void __launch_bounds__(64) k_fin_big_prune(FinalizeArgs A, const KSeg* segs, const uint64_t* keys,
                                                      uint32_t* segs_tail) {
  __shared__ uint32_t kept[kFinKeptMax];
  __shared__ uint64_t sk[64];
  __shared__ uint32_t alive[2];
  __shared__ uint32_t cid[64];
  __shared__ uint64_t ckey[64];
  const int lane = lane_id(), g = lane % L;
  const uint32_t p = A.big[blockIdx.x];
  const KSeg sg = segs[blockIdx.x];
  const int R = A.R;
  unsigned long long ev = 0, pe = 0;
  int kc = 0;
  bool full = false;
  uint32_t tail = sg.len;
  uint64_t carry = FG_KEY_NONE;
  for (uint32_t base = 0; base < sg.len; base += 64) {
    uint32_t j = base + lane;
    uint64_t x = j < sg.len ? keys[sg.start + j] : FG_KEY_NONE;
    uint64_t prev = shfl64(x, lane > 0 ? lane - 1 : 0);
    if (lane == 0) prev = carry;
    carry = shfl64(x, 63);
    bool uniq = x != FG_KEY_NONE && x != prev;
    uint64_t um = ballot(uniq);
    int k = popc64(um);
    ev += (unsigned long long)k;
    if (k == 0) continue;
    const int myslot = popc64(um & lanes_below());
    // filter against the kept rows (after R are kept, only the first R-1)
    const int nk = full ? R - 1 : kc;
    bool live = uniq;
    for (int i = 0; i < nk; i++) {
      uint64_t lm = ballot(live);
      int nl = popc64(lm);
      if (nl == 0) break;
      if (live) cid[popc64(lm & lanes_below())] = key_id(x);
      wave_sync();
      Chunks<L, NCH> kcn;
      load_chunks<L, NCH>(kcn, A.X.x + (size_t)kept[i] * A.X.stride, A.X.Q, g);
      uint32_t kn = 0;
      if constexpr (DK == U8L2) kn = group_sum_u32<L>(u8_selfdot<L, NCH>(kcn));
      batch_dists_rs<DK, L, NCH>(A.X, kcn, kn, cid, nl, ckey);
      pe += (unsigned long long)nl;
      if (live) {
        float dkc = hi_to_float<DK>(key_hi(ckey[popc64(lm & lanes_below())]));
        float dpc = hi_to_float<DK>(key_hi(x));
        if (A.alpha * dkc <= dpc) live = false;
      }
      wave_sync();
    }
    // resolve the chunk's survivors among themselves
    uint64_t lm = ballot(live);
    int nl = popc64(lm);
    if (nl) {
      if (live) sk[popc64(lm & lanes_below())] = x;
      wave_sync();
      int add = prune_wave<DK, L, NCH>(A.X, A.alpha, R - kc, sk, nl, alive, cid, ckey, kept + kc, &pe);
      kc += add;
      if (kc == R) full = true;
    }
    wave_sync();
    (void)myslot;
    if (full) {  // the rest only counts tests against the first R-1 kept rows
      tail = base + 64;
      break;
    }
  }
  uint32_t* out = A.g_nbrs + (uint64_t)p * R;
  for (int t = lane; t < R; t += 64) out[t] = t < kc ? kept[t] : FG_NONE;
  if (lane == 0) {
    A.g_cnt[p] = (uint32_t)kc;
    segs_tail[blockIdx.x] = tail;
    atomicAdd(&A.counters[0], ev);
    atomicAdd(&A.counters[1], pe);
  }
}

// The candidates after the chunk in which the R-th row was kept, spread
// over kTailBlocks workgroups per big row: each unique candidate is tested
// against kept rows 0..R-2 in order until one occludes it.  The tests and
// the candidates only feed the counters; the row is already final.
constexpr int kTailBlocks = 32;

template <int DK, int L, int NCH>
__global__ void __launch_bounds__(64) k_fin_big_tail(FinalizeArgs A, const KSeg* segs, const uint32_t* segs_tail,
                                                     const uint64_t* keys) {
  __shared__ uint32_t kept[kFinKeptMax];
  __shared__ uint32_t cid[64];
  __shared__ uint64_t ckey[64];
  const int lane = lane_id(), g = lane % L;
  const uint32_t r = blockIdx.x / kTailBlocks, q = blockIdx.x % kTailBlocks;
  const uint32_t p = A.big[r];
  const KSeg sg = segs[r];
  const uint32_t tail = segs_tail[r];
  const int R = A.R;
  if (tail >= sg.len) return;
  for (int t = lane; t < R - 1; t += 64) kept[t] = A.g_nbrs[(uint64_t)p * R + t];
  wave_sync();
  unsigned long long ev = 0, pe = 0;
  for (uint32_t base = tail + 64 * q; base < sg.len; base += 64 * kTailBlocks) {
    uint32_t j = base + lane;
    uint64_t x = j < sg.len ? keys[sg.start + j] : FG_KEY_NONE;
    uint64_t prev = shfl64(x, lane > 0 ? lane - 1 : 0);
    if (lane == 0) prev = base > 0 ? keys[sg.start + base - 1] : FG_KEY_NONE;
    bool live = x != FG_KEY_NONE && x != prev;
    ev += (unsigned long long)popc64(ballot(live));
    for (int i = 0; i < R - 1; i++) {
      uint64_t lm = ballot(live);
      int nl = popc64(lm);
      if (nl == 0) break;
      if (live) cid[popc64(lm & lanes_below())] = key_id(x);
      wave_sync();
      Chunks<L, NCH> kcn;
      load_chunks<L, NCH>(kcn, A.X.x + (size_t)kept[i] * A.X.stride, A.X.Q, g);
      uint32_t kn = 0;
      if constexpr (DK == U8L2) kn = group_sum_u32<L>(u8_selfdot<L, NCH>(kcn));
      batch_dists_rs<DK, L, NCH>(A.X, kcn, kn, cid, nl, ckey);
      pe += (unsigned long long)nl;
      if (live) {
        float dkc = hi_to_float<DK>(key_hi(ckey[popc64(lm & lanes_below())]));
        float dpc = hi_to_float<DK>(key_hi(x));
        if (A.alpha * dkc <= dpc) live = false;
      }
      wave_sync();
    }
  }
  if (lane == 0) {
    if (ev) atomicAdd(&A.counters[0], ev);
    if (pe) atomicAdd(&A.counters[1], pe);
  }
}

template <int DK, int L, int NCH>
hipError_t go(const FinalizeArgs& a, const FinalizeBig& big, hipStream_t st) {
  int grid = (int)(a.n < 65536 ? a.n : 65536);
  if (a.gram && grid > kGramSlots) grid = kGramSlots;  // one Gram scratch per block
  k_finalize<DK, L, NCH><<<grid, 64, 0, st>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int grid2 = grid < 2048 ? grid : 2048;
  k_finalize_mid<DK, L, NCH><<<grid2, 64, 0, st>>>(a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint32_t nbig = 0;
  e = hipMemcpyAsync(&nbig, a.nbig, 4, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess || nbig == 0) return e;
  k_fin_big_segs<<<(nbig + 255) / 256, 256, 0, st>>>(a, big.segs);
  std::vector<KSeg> hsegs(nbig);
  e = hipMemcpyAsync(hsegs.data(), big.segs, nbig * sizeof(KSeg), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  k_fin_big_keys<DK, L, NCH><<<nbig, 64, 0, st>>>(a, big.segs, big.keys);
  e = segsort_u64(big.keys, big.keys2, big.segs, hsegs, big.tiles, big.tile_cap, st);
  if (e != hipSuccess) return e;
  uint32_t* tails = reinterpret_cast<uint32_t*>(big.keys2);  // free after the sort
  k_fin_big_prune<DK, L, NCH><<<nbig, 64, 0, st>>>(a, big.segs, big.keys, tails);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_fin_big_tail<DK, L, NCH><<<nbig * kTailBlocks, 64, 0, st>>>(a, big.segs, tails, big.keys);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_finalize(int dk, int Q, const FinalizeArgs& a, const FinalizeBig& big, hipStream_t st) {
  if (dk == U8L2) {
    if (Q <= 8) return go<U8L2, 8, 1>(a, big, st);
    if (Q <= 16) return go<U8L2, 16, 1>(a, big, st);
    return hipErrorInvalidValue;
  }
#define FG_F32_ROWS(DKV)                              \
  if (Q <= 8) return go<DKV, 8, 1>(a, big, st);            \
  if (Q <= 16) return go<DKV, 16, 1>(a, big, st);          \
  if (Q <= 32) return go<DKV, 16, 2>(a, big, st);          \
  if (Q <= 64) return go<DKV, 16, 4>(a, big, st);          \
  if (Q <= 256) return go<DKV, 16, 16>(a, big, st);        \
  return hipErrorInvalidValue;
  if (dk == F32L2) { FG_F32_ROWS(F32L2) }
  if (dk == F32COS) { FG_F32_ROWS(F32COS) }
#undef FG_F32_ROWS
  return hipErrorInvalidValue;
}

}  // namespace fg
