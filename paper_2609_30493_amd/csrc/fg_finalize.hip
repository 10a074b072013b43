// fg_finalize.hip -- finalize (Sec. 3): each point's harvested row united
// with its reverse edges, deduplicated, sorted by (d(p,.), id) and, when it
// holds more than R candidates (or always with reprune_all), occlusion-pruned
// to at most R.  One wave per point.
#include "fg_internal.h"

namespace fg {

namespace {

constexpr int kFinCap = 2048;  // candidates per point held on chip

template <int DK, int L, int NCH>
__global__ void __launch_bounds__(64) k_finalize(FinalizeArgs A) {
  __shared__ uint32_t cb[kFinCap];
  __shared__ uint64_t sk[kFinCap];
  __shared__ uint32_t alive[kFinCap / 32];
  __shared__ uint32_t cid[64];
  __shared__ uint64_t ckey[64];
  const int lane = lane_id();
  const int g = lane % L;
  unsigned long long ev = 0, pe = 0;
  for (int64_t p = blockIdx.x; p < A.n; p += gridDim.x) {
    uint32_t* out = A.g_nbrs + p * A.R;
    const int c = (int)min(A.cnt[p], (uint32_t)A.R);  // counts above R are not trusted
    const uint64_t r0 = A.revoff[p];
    const int rc = (int)(A.revoff[p + 1] - r0);
    const int m0 = c + rc;
    if (m0 > kFinCap) {
      if (lane == 0) {
        atomicOr(A.status, 4);
        A.g_cnt[p] = 0;
      }
      for (int t = lane; t < A.R; t += 64) out[t] = FG_NONE;
      continue;
    }
    int M = 64;
    while (M < m0) M <<= 1;
    for (int i = lane; i < M; i += 64)
    {
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
    load_chunks<L, NCH>(qc, A.X.x + (size_t)p * A.X.stride, A.X.Q, g);
    uint32_t qn = 0;
    if constexpr (DK == U8L2) qn = group_sum_u32<L>(u8_selfdot<L, NCH>(qc));
    for (int base = 0; base < m; base += 64) {
      int cnt = m - base < 64 ? m - base : 64;
      batch_dists_rs<DK, L, NCH>(A.X, qc, qn, cb + base, cnt, sk + base);
    }
    ev += (unsigned long long)m;
    int Mk = 64;
    while (Mk < m) Mk <<= 1;
    for (int i = m + lane; i < Mk; i += 64) sk[i] = FG_KEY_NONE;
    wave_sync();
    wave_sort_lds<uint64_t>(sk, Mk);
    int kept;
    if (m > A.R || A.reprune_all) {
      kept = prune_wave<DK, L, NCH>(A.X, A.alpha, A.R, sk, m, alive, cid, ckey, out, &pe);
    } else {
      for (int i = lane; i < m; i += 64) out[i] = key_id(sk[i]);
      kept = m;
    }
    for (int t = kept + lane; t < A.R; t += 64) out[t] = FG_NONE;
    if (lane == 0) A.g_cnt[p] = (uint32_t)kept;
    wave_sync();
  }
  if (lane == 0) {
    atomicAdd(&A.counters[0], ev);
    atomicAdd(&A.counters[1], pe);
  }
}

template <int DK, int L, int NCH>
hipError_t go(const FinalizeArgs& a, hipStream_t st) {
  int grid = (int)(a.n < 65536 ? a.n : 65536);
  k_finalize<DK, L, NCH><<<grid, 64, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_finalize(int dk, int Q, const FinalizeArgs& a, hipStream_t st) {
  if (dk == U8L2) {
    if (Q <= 8) return go<U8L2, 8, 1>(a, st);
    if (Q <= 16) return go<U8L2, 16, 1>(a, st);
    return hipErrorInvalidValue;
  }
#define FG_F32_ROWS(DKV)                              \
  if (Q <= 8) return go<DKV, 8, 1>(a, st);            \
  if (Q <= 16) return go<DKV, 16, 1>(a, st);          \
  if (Q <= 32) return go<DKV, 16, 2>(a, st);          \
  if (Q <= 64) return go<DKV, 16, 4>(a, st);          \
  if (Q <= 256) return go<DKV, 16, 16>(a, st);        \
  return hipErrorInvalidValue;
  if (dk == F32L2) { FG_F32_ROWS(F32L2) }
  if (dk == F32COS) { FG_F32_ROWS(F32COS) }
#undef FG_F32_ROWS
  return hipErrorInvalidValue;
}

}  // namespace fg
