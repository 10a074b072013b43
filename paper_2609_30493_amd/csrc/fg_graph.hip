// fg_graph.hip -- fills and prefix scans used by the graph-building steps.
#include <vector>

#include "fg_internal.h"

namespace fg {

namespace {

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

// Inclusive scan of one value per thread across a 256-thread block.
__device__ uint64_t block_inclusive_scan(uint64_t v, uint64_t* sh) {
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint64_t o = shfl64(v, lane >= off ? lane - off : lane);
    if (lane >= off) v += o;
  }
  if (lane == 63) sh[w] = v;
  __syncthreads();
  uint64_t add = 0;
  for (int i = 0; i < w; i++) add += sh[i];
  __syncthreads();
  return v + add;
}

__global__ void k_scan_tiles(const uint32_t* in, int64_t count, uint64_t* tile_sums) {
  __shared__ uint64_t sh[4];
  int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanPer;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; i++)
    if (base + i < count) s += in[base + i];
  uint64_t inc = block_inclusive_scan(s, sh);
  if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = inc;
}

// One block scans the tile sums in place (exclusive), chunk by chunk.
__global__ void k_scan_sums(uint64_t* sums, int64_t ntiles, uint64_t* total) {
  __shared__ uint64_t sh[4];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < ntiles; base += kScanThreads) {
    int64_t i = base + threadIdx.x;
    uint64_t v = i < ntiles ? sums[i] : 0;
    uint64_t inc = block_inclusive_scan(v, sh);
    uint64_t c = carry;
    if (i < ntiles) sums[i] = c + inc - v;
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) carry = c + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_apply(const uint32_t* in, int64_t count, const uint64_t* tile_off,
                             uint64_t* out) {
  __shared__ uint64_t sh[4];
  int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; i++) {
    v[i] = base + i < count ? in[base + i] : 0;
    s += v[i];
  }
  uint64_t inc = block_inclusive_scan(s, sh);
  uint64_t run = tile_off[blockIdx.x] + inc - s;
#pragma unroll
  for (int i = 0; i < kScanPer; i++) {
    if (base + i < count) out[base + i] = run;
    run += v[i];
  }
}

int blocks_for(int64_t count, int per_block) {
  int64_t b = (count + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

// ------------------------------------------------------------------ edges
// The rows of the points p = b + i*B (i < nitems), R slots each, cnt[p]
// used.  Each used slot (p, u) contributes u to row p when `own` and p to
// row u when `rev`.
__global__ void k_edges_count(int64_t n, const uint32_t* rows, const uint32_t* cnt, int R, int64_t b,
                              int64_t B, int64_t nitems, bool own, bool rev, uint32_t* deg) {
  int64_t total = nitems * R;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / R;
    int s = (int)(t - i * R);
    int64_t p = b + i * B;
    if ((uint32_t)s >= cnt[p]) continue;
    uint32_t u = rows[p * R + s];
    if (u >= (uint64_t)n) continue;  // not a point id: ignored
    if (own) atomicAdd(&deg[p], 1u);
    if (rev) atomicAdd(&deg[u], 1u);
  }
}

__global__ void k_edges_scatter(int64_t n, const uint32_t* rows, const uint32_t* cnt, int R, int64_t b,
                                int64_t B, int64_t nitems, bool own, bool rev, const uint64_t* off,
                                uint32_t* cursor, uint32_t* out) {
  int64_t total = nitems * R;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / R;
    int s = (int)(t - i * R);
    int64_t p = b + i * B;
    if ((uint32_t)s >= cnt[p]) continue;
    uint32_t u = rows[p * R + s];
    if (u >= (uint64_t)n) continue;
    if (own) out[off[p] + atomicAdd(&cursor[p], 1u)] = u;
    if (rev) out[off[u] + atomicAdd(&cursor[u], 1u)] = (uint32_t)p;
  }
}

// ------------------------------------------------------------------ merge
// One wave per row v: the old row (sorted, unique) united with the row's
// additions (any order, repeats allowed) -> sorted unique, written at the
// row's upper-bound slot off[v] + addoff[v] of tmp; its length to newlen[v].
// Two on-chip tiers: rows with at most kMergeSmall additions first (small
// LDS, many waves per compute unit); rows up to kMergeAddMax are listed for
// the second tier; rows beyond that for the big-row paths.
constexpr int kMergeAddMax = 2048;
constexpr int kMergeSmall = 256;

template <int CAP>
__device__ void merge_row(int64_t v, const uint64_t* off, const uint32_t* ids, const uint64_t* addoff,
                          const uint32_t* addbuf, uint32_t* tmp, uint32_t* newlen, uint32_t* buf, uint32_t* uni) {
  const int lane = lane_id();
  const uint64_t o0 = off[v];
  const int64_t o = (int64_t)(off[v + 1] - o0);
  const uint64_t a0 = addoff[v];
  const int64_t a = (int64_t)(addoff[v + 1] - a0);
  uint32_t* dst = tmp + o0 + a0;
  int M = 64;
  while (M < a) M <<= 1;
  for (int i = lane; i < M; i += 64) buf[i] = i < a ? addbuf[a0 + i] : FG_NONE;
  wave_sync();
  wave_sort_lds<uint32_t>(buf, M);
  // keep first occurrences that are not already in the old row
  int u = 0;
  for (int base = 0; base < M; base += 64) {
    int i = base + lane;
    uint32_t x = buf[i];
    bool keep = x != FG_NONE && (i == 0 || buf[i - 1] != x);
    if (keep) {
      int lo = 0, hi = (int)o;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (ids[o0 + mid] < x) lo = mid + 1;
        else hi = mid;
      }
      keep = !(lo < o && ids[o0 + lo] == x);
    }
    uint64_t m = ballot(keep);
    if (keep) uni[u + popc64(m & lanes_below())] = x;
    u += popc64(m);
  }
  wave_sync();
  for (int64_t j = lane; j < o; j += 64) {
    uint32_t x = ids[o0 + j];
    dst[j + lower_bound_lds<uint32_t>(uni, u, x)] = x;
  }
  for (int i = lane; i < u; i += 64) {
    uint32_t x = uni[i];
    int lo = 0, hi = (int)o;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (ids[o0 + mid] < x) lo = mid + 1;
      else hi = mid;
    }
    dst[i + lo] = x;
  }
  if (lane == 0) newlen[v] = (uint32_t)(o + u);
  wave_sync();
}

__global__ void __launch_bounds__(64) k_merge_rows(int64_t n, const uint64_t* off, const uint32_t* ids,
                                                   const uint64_t* addoff, const uint32_t* addbuf,
                                                   uint32_t* tmp, uint32_t* newlen, uint32_t* big,
                                                   uint32_t* nbig, uint32_t* mid, uint32_t* nmid) {
  __shared__ uint32_t buf[kMergeSmall];
  __shared__ uint32_t uni[kMergeSmall];
  const int lane = lane_id();
  for (int64_t v = blockIdx.x; v < n; v += gridDim.x) {
    const uint64_t o0 = off[v];
    const int64_t o = (int64_t)(off[v + 1] - o0);
    const int64_t a = (int64_t)(addoff[v + 1] - addoff[v]);
    if (a == 0) {
      uint32_t* dst = tmp + o0 + addoff[v];
      for (int64_t j = lane; j < o; j += 64) dst[j] = ids[o0 + j];
      if (lane == 0) newlen[v] = (uint32_t)o;
      continue;
    }
    if (a > kMergeAddMax) {  // handled by the big-row path
      if (lane == 0) {
        uint32_t at = atomicAdd(nbig, 1u);
        big[at] = (uint32_t)v;
        newlen[v] = 0;
      }
      continue;
    }
    if (a > kMergeSmall) {  // handled by the second tier
      if (lane == 0) mid[atomicAdd(nmid, 1u)] = (uint32_t)v;
      continue;
    }
    merge_row<kMergeSmall>(v, off, ids, addoff, addbuf, tmp, newlen, buf, uni);
  }
}

__global__ void __launch_bounds__(64) k_merge_rows_mid(const uint64_t* off, const uint32_t* ids,
                                                       const uint64_t* addoff, const uint32_t* addbuf,
                                                       uint32_t* tmp, uint32_t* newlen, const uint32_t* mid,
                                                       const uint32_t* nmid) {
  __shared__ uint32_t buf[kMergeAddMax];
  __shared__ uint32_t uni[kMergeAddMax];
  const uint32_t nm = *nmid;
  for (uint32_t k = blockIdx.x; k < nm; k += gridDim.x)
    merge_row<kMergeAddMax>(mid[k], off, ids, addoff, addbuf, tmp, newlen, buf, uni);
}

// Rows with more than kMergeAddMax additions without the host: workgroups of
// 1024 threads take the rows listed in big[0..*nbig) in turn.  A row's
// additions are sorted by a bitonic network in global scratch (row v uses
// the 2 * a entries at scratch + 2 * addoff[v], enough for the power of two
// M >= a), reduced in place to the ids that are new (first occurrence, not
// in the old row), then merged with the old row by co-ranking into the
// row's upper-bound slot of tmp, as k_merge_rows does.
__global__ void __launch_bounds__(1024) k_merge_big_dev(const uint32_t* big, const uint32_t* nbig,
                                                        const uint64_t* off, const uint32_t* ids,
                                                        const uint64_t* addoff, const uint32_t* addbuf,
                                                        uint32_t* scratch, uint32_t* tmp, uint32_t* newlen) {
  __shared__ uint32_t wcount[16];
  __shared__ uint32_t carry;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nt = blockDim.x;
  const uint32_t nb = *nbig;
  for (uint32_t k = blockIdx.x; k < nb; k += gridDim.x) {
    const uint32_t v = big[k];
    const uint64_t o0 = off[v];
    const int64_t o = (int64_t)(off[v + 1] - o0);
    const uint64_t a0 = addoff[v];
    const int64_t a = (int64_t)(addoff[v + 1] - a0);
    int64_t M = 1;
    while (M < a) M <<= 1;
    uint32_t* buf = scratch + 2 * a0;
    for (int64_t i = tid; i < M; i += nt) buf[i] = i < a ? addbuf[a0 + i] : FG_NONE;
    __syncthreads();
    for (int64_t kb = 2; kb <= M; kb <<= 1) {
      for (int64_t jb = kb >> 1; jb > 0; jb >>= 1) {
        for (int64_t i = tid; i < M; i += nt) {
          const int64_t ixj = i ^ jb;
          if (ixj > i) {
            const uint32_t x0 = buf[i], x1 = buf[ixj];
            if ((x0 > x1) == ((i & kb) == 0)) {
              buf[i] = x1;
              buf[ixj] = x0;
            }
          }
        }
        __syncthreads();
      }
    }
    // in-place compaction: every read of a chunk precedes its writes, which
    // land at or before the chunk; the raw last value of the previous chunk
    // is carried for the repeat test
    int64_t u = 0;
    if (tid == 0) carry = FG_NONE;
    __syncthreads();
    for (int64_t c0 = 0; c0 < M; c0 += nt) {
      const int64_t i = c0 + tid;
      const uint32_t x = i < M ? buf[i] : FG_NONE;
      const uint32_t prev = tid == 0 ? carry : (i - 1 < M ? buf[i - 1] : FG_NONE);
      bool keep = x != FG_NONE && !(i > 0 && prev == x);
      if (keep) {
        int64_t lo = 0, hi = o;
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (ids[o0 + mid] < x) lo = mid + 1;
          else hi = mid;
        }
        keep = !(lo < o && ids[o0 + lo] == x);
      }
      const uint64_t m = ballot(keep);
      if (lane == 0) wcount[wv] = (uint32_t)popc64(m);
      __syncthreads();
      uint32_t before = 0, total = 0;
      for (int t = 0; t < nt / 64; t++) {
        before += t < wv ? wcount[t] : 0;
        total += wcount[t];
      }
      const uint32_t last = c0 + nt - 1 < M ? buf[c0 + nt - 1] : FG_NONE;
      __syncthreads();
      if (keep) buf[u + before + popc64(m & lanes_below())] = x;
      if (tid == 0) carry = last;
      u += total;
      __syncthreads();
    }
    uint32_t* dst = tmp + o0 + a0;
    for (int64_t j = tid; j < o; j += nt) {
      const uint32_t x = ids[o0 + j];
      int64_t lo = 0, hi = u;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (buf[mid] < x) lo = mid + 1;
        else hi = mid;
      }
      dst[j + lo] = x;
    }
    for (int64_t i = tid; i < u; i += nt) {
      const uint32_t x = buf[i];
      int64_t lo = 0, hi = o;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ids[o0 + mid] < x) lo = mid + 1;
        else hi = mid;
      }
      dst[i + lo] = x;
    }
    if (tid == 0) newlen[v] = (uint32_t)(o + u);
    __syncthreads();
  }
}

// Copy row v from its upper-bound slot to its final offset.
__global__ void __launch_bounds__(64) k_compact_rows(int64_t n, const uint64_t* off, const uint64_t* addoff,
                                                     const uint32_t* tmp, const uint64_t* noff,
                                                     uint32_t* out) {
  const int lane = lane_id();
  for (int64_t v = blockIdx.x; v < n; v += gridDim.x) {
    const uint32_t* src = tmp + off[v] + addoff[v];
    uint64_t d0 = noff[v];
    int64_t len = (int64_t)(noff[v + 1] - d0);
    for (int64_t j = lane; j < len; j += 64) out[d0 + j] = src[j];
  }
}

// ------------------------------------------------------------------ search graph
// Degree of v in G u spine: its row count, one for its tree-0 parent, one
// per tree-0 child.
__global__ void k_search_deg(int64_t n, int R, const uint32_t* nbrs, const uint32_t* cnt,
                             const uint32_t* parent0, uint32_t* deg) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c = min(cnt[v], (uint32_t)R);  // counts above R are not trusted
    uint32_t d = 0;
    for (uint32_t i = 0; i < c; i++) d += nbrs[v * R + i] < (uint64_t)n ? 1u : 0u;
    uint32_t pa = parent0[v];
    if (pa < (uint64_t)n) {
      d += 1;
      atomicAdd(&deg[pa], 1u);
    }
    atomicAdd(&deg[v], d);
  }
}

__global__ void k_search_fill(int64_t n, int R, const uint32_t* nbrs, const uint32_t* cnt,
                              const uint32_t* parent0, const uint64_t* off, uint32_t* cursor,
                              uint32_t* out) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c = min(cnt[v], (uint32_t)R);
    uint32_t pa = parent0[v];
    uint32_t own = pa < (uint64_t)n ? 1u : 0u;
    for (uint32_t i = 0; i < c; i++) own += nbrs[v * R + i] < (uint64_t)n ? 1u : 0u;
    uint32_t at = atomicAdd(&cursor[v], own);
    uint64_t w = off[v] + at;
    for (uint32_t i = 0; i < c; i++) {
      uint32_t u = nbrs[v * R + i];
      if (u < (uint64_t)n) out[w++] = u;
    }
    if (pa < (uint64_t)n) {
      out[w] = pa;
      out[off[pa] + atomicAdd(&cursor[pa], 1u)] = (uint32_t)v;
    }
  }
}

// ------------------------------------------------------------------ segmented sort
// Ascending sort of each segment [start, start + len) of a key array, for
// segments of any length: every tile of kSegTile keys is sorted by one wave
// in LDS, then runs of width 2^k * kSegTile are merged pairwise (each key's
// output slot is its rank in its own run plus its rank in the partner run).
constexpr int kSegTile = 256;

__global__ void __launch_bounds__(64) k_seg_tile_sort(const KSeg* segs, const KTile* tiles, uint64_t* keys) {
  __shared__ uint64_t sk[kSegTile];
  const int lane = lane_id();
  const KTile tl = tiles[blockIdx.x];
  const KSeg sg = segs[tl.seg];
  const uint32_t cnt = min((uint32_t)kSegTile, sg.len - tl.off);
  for (int i = lane; i < kSegTile; i += 64) sk[i] = i < (int)cnt ? keys[sg.start + tl.off + i] : FG_KEY_NONE;
  wave_sync();
  wave_sort_lds<uint64_t>(sk, kSegTile);
  for (int i = lane; i < (int)cnt; i += 64) keys[sg.start + tl.off + i] = sk[i];
}

__global__ void __launch_bounds__(64) k_seg_merge_pass(const KSeg* segs, const KTile* tiles, const uint64_t* src,
                                                       uint64_t* dst, uint32_t w) {
  const int lane = lane_id();
  const KTile tl = tiles[blockIdx.x];
  const KSeg sg = segs[tl.seg];
  const uint64_t* s = src + sg.start;
  uint64_t* d = dst + sg.start;
  const uint32_t hi = min(sg.len, tl.off + kSegTile);
  for (uint32_t j = tl.off + lane; j < hi; j += 64) {
    uint64_t k = s[j];
    uint32_t r = j / w;
    uint32_t pb = (r & ~1u) * w;
    uint32_t lo_o, hi_o, mine;
    if ((r & 1u) == 0) {
      mine = j - pb;
      lo_o = min(pb + w, sg.len);
      hi_o = min(pb + 2 * w, sg.len);
    } else {
      mine = j - pb - w;
      lo_o = pb;
      hi_o = pb + w;
    }
    // stable: the left run's keys go before equal keys of the right run
    const bool left = (r & 1u) == 0;
    uint32_t a = lo_o, b = hi_o;
    while (a < b) {
      uint32_t m = (a + b) >> 1;
      if (left ? (s[m] < k) : (s[m] <= k)) a = m + 1;
      else b = m;
    }
    d[pb + mine + (a - lo_o)] = k;
  }
}

__global__ void __launch_bounds__(64) k_seg_copy(const KSeg* segs, const KTile* tiles, const uint64_t* src,
                                                 uint64_t* dst) {
  const KTile tl = tiles[blockIdx.x];
  const KSeg sg = segs[tl.seg];
  const uint32_t hi = min(sg.len, tl.off + kSegTile);
  for (uint32_t j = tl.off + lane_id(); j < hi; j += 64) dst[sg.start + j] = src[sg.start + j];
}

// ------------------------------------------------------------------ big merge rows
// Segment descriptors of the rows listed in `big` (their additions).
__global__ void k_big_segs(const uint32_t* big, uint32_t nbig, const uint64_t* addoff, KSeg* segs) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nbig; i += gridDim.x * blockDim.x) {
    uint32_t v = big[i];
    segs[i] = KSeg{addoff[v], (uint32_t)(addoff[v + 1] - addoff[v]), 0};
  }
}

__global__ void __launch_bounds__(64) k_big_widen(const KSeg* segs, const KTile* tiles, const uint32_t* addbuf,
                                                  uint64_t* keys) {
  const KTile tl = tiles[blockIdx.x];
  const KSeg sg = segs[tl.seg];
  const uint32_t hi = min(sg.len, tl.off + kSegTile);
  for (uint32_t j = tl.off + lane_id(); j < hi; j += 64) keys[sg.start + j] = addbuf[sg.start + j];
}

// One wave per big row: the sorted additions (keys, id in the low word)
// deduplicated and stripped of ids already in the old row, compacted into
// uni (same offsets), then merged with the old row into tmp.
__global__ void __launch_bounds__(64) k_merge_big(const uint32_t* big, const KSeg* segs, const uint64_t* off,
                                                  const uint32_t* ids, const uint64_t* addoff, const uint64_t* keys,
                                                  uint32_t* uni, uint32_t* tmp, uint32_t* newlen) {
  const int lane = lane_id();
  const uint32_t v = big[blockIdx.x];
  const KSeg sg = segs[blockIdx.x];
  const uint64_t o0 = off[v];
  const int64_t o = (int64_t)(off[v + 1] - o0);
  uint32_t* u_out = uni + sg.start;
  auto in_old = [&](uint32_t x) {
    int64_t lo = 0, hi = o;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (ids[o0 + mid] < x) lo = mid + 1;
      else hi = mid;
    }
    return lo < o && ids[o0 + lo] == x;
  };
  uint32_t u = 0;
  uint32_t carry = FG_NONE;
  for (uint32_t base = 0; base < sg.len; base += 64) {
    uint32_t j = base + lane;
    uint32_t x = j < sg.len ? (uint32_t)keys[sg.start + j] : FG_NONE;
    uint32_t prev = __shfl(x, lane > 0 ? lane - 1 : 0, 64);
    if (lane == 0) prev = carry;
    carry = __shfl(x, 63, 64);
    bool keep = x != FG_NONE && x != prev && !in_old(x);
    uint64_t m = ballot(keep);
    if (keep) u_out[u + popc64(m & lanes_below())] = x;
    u += popc64(m);
  }
  wave_sync();
  __threadfence();
  uint32_t* dst = tmp + o0 + addoff[v];
  for (int64_t j = lane; j < o; j += 64) {
    uint32_t x = ids[o0 + j];
    uint32_t lo = 0, hi = u;
    while (lo < hi) {
      uint32_t mid = (lo + hi) >> 1;
      if (u_out[mid] < x) lo = mid + 1;
      else hi = mid;
    }
    dst[j + lo] = x;
  }
  for (uint32_t i = lane; i < u; i += 64) {
    uint32_t x = u_out[i];
    int64_t lo = 0, hi = o;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (ids[o0 + mid] < x) lo = mid + 1;
      else hi = mid;
    }
    dst[i + lo] = x;
  }
  if (lane == 0) newlen[v] = (uint32_t)(o + u);
}

}  // namespace

namespace {
__global__ void k_block_flags(const uint32_t* order, int64_t len, uint32_t B, uint32_t b, uint32_t* flags) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    flags[i] = order[i] % B == b ? 1u : 0u;
}
__global__ void k_block_scatter(const uint32_t* order, int64_t len, uint32_t B, uint32_t b, const uint64_t* pos,
                                uint32_t* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = order[i];
    if (p % B == b) out[pos[i]] = p;
  }
}
__global__ void k_rank_of(const uint32_t* order, int64_t len, uint32_t last, uint32_t* rank) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= len; i += (int64_t)gridDim.x * blockDim.x)
    if (i < len || last != FG_NONE) rank[i < len ? order[i] : last] = (uint32_t)i;
}
}  // namespace

namespace {
// pairs[e] = (ids[e], rank[ids[e]]) for e < off[n] (read on the device).
__global__ void k_csr_pairs(const uint64_t* off_n, const uint32_t* ids, const uint32_t* rank, uint2* pairs) {
  const uint64_t nnz = *off_n;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < nnz; e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t u = ids[e];
    pairs[e] = make_uint2(u, rank[u]);
  }
}
}  // namespace

hipError_t csr_rank_pairs(int64_t n, const uint64_t* off, const uint32_t* ids, const uint32_t* rank, uint2* pairs,
                          hipStream_t st) {
  k_csr_pairs<<<4096, 256, 0, st>>>(off + n, ids, rank, pairs);
  return hipGetLastError();
}

hipError_t rank_of(const uint32_t* order, int64_t len, uint32_t last, uint32_t* rank, hipStream_t st) {
  k_rank_of<<<blocks_for(len + 1, 1024), 256, 0, st>>>(order, len, last, rank);
  return hipGetLastError();
}

hipError_t block_schedule(const uint32_t* order, int64_t len, int64_t n, uint32_t B, uint32_t last,
                          uint32_t* sched, uint32_t* flags, uint64_t* pos, void* scratch, hipStream_t st) {
  int64_t base = 0;
  for (uint32_t b = 0; b < B; b++) {
    const int64_t nb = n > (int64_t)b ? (n - (int64_t)b + B - 1) / B : 0;
    if (len > 0) {
      k_block_flags<<<blocks_for(len, 1024), 256, 0, st>>>(order, len, B, b, flags);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = exclusive_scan_u32_u64(flags, pos, len, scratch, st);
      if (e != hipSuccess) return e;
      k_block_scatter<<<blocks_for(len, 1024), 256, 0, st>>>(order, len, B, b, pos, sched + base);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (last != FG_NONE && last % B == b && nb > 0) {  // the one id the order leaves out closes its block
      hipError_t e = fill_u32(sched + base + nb - 1, last, 1, st);
      if (e != hipSuccess) return e;
    }
    base += nb;
  }
  return hipSuccess;
}

hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_fill_u32<<<blocks_for(count, 1024), 256, 0, st>>>(p, v, count);
  return hipGetLastError();
}

__global__ void k_localize_graph(const uint32_t* nbrs, const uint32_t* cnt, const uint32_t* parent0, int64_t ni,
                                 int R, int64_t o, uint32_t* out_nbrs, uint32_t* out_cnt, uint32_t* out_parent) {
  const int64_t total = ni * R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = i / R;
    const uint32_t v = nbrs[o * R + i];
    out_nbrs[i] = v == FG_NONE ? FG_NONE : (uint32_t)(v - o);
    if (i - j * R == 0) {
      out_cnt[j] = cnt[o + j];
      const uint32_t p = parent0[o + j];
      out_parent[j] = p == FG_NONE ? FG_NONE : (uint32_t)(p - o);
    }
  }
}

hipError_t localize_graph(const uint32_t* nbrs, const uint32_t* cnt, const uint32_t* parent0, int64_t ni, int R,
                          int64_t o, uint32_t* out_nbrs, uint32_t* out_cnt, uint32_t* out_parent, hipStream_t st) {
  k_localize_graph<<<blocks_for(ni * R, 256), 256, 0, st>>>(nbrs, cnt, parent0, ni, R, o, out_nbrs, out_cnt,
                                                             out_parent);
  return hipGetLastError();
}

hipError_t fill_u64(uint64_t* p, uint64_t v, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_fill_u64<<<blocks_for(count, 1024), 256, 0, st>>>(p, v, count);
  return hipGetLastError();
}

size_t scan_scratch_bytes(int64_t count) {
  int64_t ntiles = (count + kScanTile - 1) / kScanTile + 1;
  return (size_t)ntiles * sizeof(uint64_t);
}

hipError_t exclusive_scan_u32_u64(const uint32_t* in, uint64_t* out, int64_t count,
                                  void* scratch, hipStream_t st) {
  int64_t ntiles = (count + kScanTile - 1) / kScanTile;
  uint64_t* sums = static_cast<uint64_t*>(scratch);
  if (ntiles == 0) return fill_u64(out, 0, 1, st);
  k_scan_tiles<<<(unsigned)ntiles, kScanThreads, 0, st>>>(in, count, sums);
  k_scan_sums<<<1, kScanThreads, 0, st>>>(sums, ntiles, out + count);
  k_scan_apply<<<(unsigned)ntiles, kScanThreads, 0, st>>>(in, count, sums, out);
  return hipGetLastError();
}

hipError_t edges_count(int64_t n, const uint32_t* rows, const uint32_t* cnt, int R, int64_t b, int64_t B,
                       int64_t nitems, bool own, bool rev, uint32_t* deg, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  k_edges_count<<<blocks_for(nitems * R, 1024), 256, 0, st>>>(n, rows, cnt, R, b, B, nitems, own, rev, deg);
  return hipGetLastError();
}

hipError_t edges_scatter(int64_t n, const uint32_t* rows, const uint32_t* cnt, int R, int64_t b, int64_t B,
                         int64_t nitems, bool own, bool rev, const uint64_t* off, uint32_t* cursor,
                         uint32_t* out, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  k_edges_scatter<<<blocks_for(nitems * R, 1024), 256, 0, st>>>(n, rows, cnt, R, b, B, nitems, own, rev,
                                                                off, cursor, out);
  return hipGetLastError();
}

hipError_t merge_big_rows_dev(const uint32_t* big, const uint32_t* nbig, const uint64_t* off, const uint32_t* ids,
                              const uint64_t* addoff, const uint32_t* addbuf, uint32_t* scratch, uint32_t* tmp,
                              uint32_t* newlen, hipStream_t st) {
  k_merge_big_dev<<<64, 1024, 0, st>>>(big, nbig, off, ids, addoff, addbuf, scratch, tmp, newlen);
  return hipGetLastError();
}

hipError_t merge_rows(int64_t n, const uint64_t* off, const uint32_t* ids, const uint64_t* addoff,
                      const uint32_t* addbuf, uint32_t* tmp, uint32_t* newlen, uint32_t* big, uint32_t* nbig,
                      uint32_t* mid, uint32_t* nmid, hipStream_t st) {
  int grid = (int)(n < 65536 ? n : 65536);
  k_merge_rows<<<grid, 64, 0, st>>>(n, off, ids, addoff, addbuf, tmp, newlen, big, nbig, mid, nmid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_merge_rows_mid<<<grid < 2048 ? grid : 2048, 64, 0, st>>>(off, ids, addoff, addbuf, tmp, newlen, mid, nmid);
  return hipGetLastError();
}

hipError_t segsort_u64(uint64_t* keys, uint64_t* keys2, const KSeg* dsegs, const std::vector<KSeg>& hsegs,
                       KTile* dtiles, size_t tile_cap, hipStream_t st) {
  std::vector<KTile> tiles;
  uint32_t maxlen = 0;
  for (uint32_t i = 0; i < hsegs.size(); i++) {
    for (uint32_t o = 0; o < hsegs[i].len; o += kSegTile) tiles.push_back(KTile{i, o});
    maxlen = maxlen > hsegs[i].len ? maxlen : hsegs[i].len;
  }
  if (tiles.empty()) return hipSuccess;
  if (tiles.size() > tile_cap) return hipErrorOutOfMemory;
  hipError_t e = hipMemcpyAsync(dtiles, tiles.data(), tiles.size() * sizeof(KTile), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  // the host vector must outlive the copy
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  const unsigned nt = (unsigned)tiles.size();
  k_seg_tile_sort<<<nt, 64, 0, st>>>(dsegs, dtiles, keys);
  uint64_t* src = keys;
  uint64_t* dst = keys2;
  for (uint32_t w = kSegTile; w < maxlen; w *= 2) {
    k_seg_merge_pass<<<nt, 64, 0, st>>>(dsegs, dtiles, src, dst, w);
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  if (src != keys) k_seg_copy<<<nt, 64, 0, st>>>(dsegs, dtiles, src, keys);
  return hipGetLastError();
}

hipError_t merge_big_rows(const uint32_t* big, uint32_t nbig, const uint64_t* off, const uint32_t* ids,
                          const uint64_t* addoff, const uint32_t* addbuf, uint32_t* tmp, uint32_t* newlen,
                          KSeg* dsegs, KTile* dtiles, size_t tile_cap, uint64_t* keys, uint64_t* keys2,
                          uint32_t* uni, hipStream_t st) {
  if (nbig == 0) return hipSuccess;
  k_big_segs<<<blocks_for(nbig, 256), 256, 0, st>>>(big, nbig, addoff, dsegs);
  std::vector<KSeg> hsegs(nbig);
  hipError_t e = hipMemcpyAsync(hsegs.data(), dsegs, nbig * sizeof(KSeg), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  std::vector<KTile> tiles;
  for (uint32_t i = 0; i < nbig; i++)
    for (uint32_t o = 0; o < hsegs[i].len; o += kSegTile) tiles.push_back(KTile{i, o});
  if (tiles.size() > tile_cap) return hipErrorOutOfMemory;
  e = hipMemcpyAsync(dtiles, tiles.data(), tiles.size() * sizeof(KTile), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  k_big_widen<<<(unsigned)tiles.size(), 64, 0, st>>>(dsegs, dtiles, addbuf, keys);
  e = segsort_u64(keys, keys2, dsegs, hsegs, dtiles, tile_cap, st);
  if (e != hipSuccess) return e;
  k_merge_big<<<nbig, 64, 0, st>>>(big, dsegs, off, ids, addoff, keys, uni, tmp, newlen);
  return hipGetLastError();
}

hipError_t compact_rows(int64_t n, const uint64_t* off, const uint64_t* addoff, const uint32_t* tmp,
                        const uint64_t* noff, uint32_t* out, hipStream_t st) {
  int grid = (int)(n < 65536 ? n : 65536);
  k_compact_rows<<<grid, 64, 0, st>>>(n, off, addoff, tmp, noff, out);
  return hipGetLastError();
}

hipError_t search_graph(int64_t n, int R, const uint32_t* nbrs, const uint32_t* cnt,
                        const uint32_t* parent0, uint32_t* deg, uint64_t* off, uint32_t* out,
                        void* scan_scratch, hipStream_t st) {
  hipError_t e = fill_u32(deg, 0, n, st);
  if (e != hipSuccess) return e;
  k_search_deg<<<blocks_for(n, 256), 256, 0, st>>>(n, R, nbrs, cnt, parent0, deg);
  e = exclusive_scan_u32_u64(deg, off, n, scan_scratch, st);
  if (e != hipSuccess) return e;
  e = fill_u32(deg, 0, n, st);
  if (e != hipSuccess) return e;
  k_search_fill<<<blocks_for(n, 256), 256, 0, st>>>(n, R, nbrs, cnt, parent0, off, deg, out);
  return hipGetLastError();
}

}  // namespace fg
