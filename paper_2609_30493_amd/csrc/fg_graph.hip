// fg_graph.hip -- fills and prefix scans used by the graph-building steps.
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
constexpr int kMergeAddMax = 2048;

__global__ void __launch_bounds__(64) k_merge_rows(int64_t n, const uint64_t* off, const uint32_t* ids,
                                                   const uint64_t* addoff, const uint32_t* addbuf,
                                                   uint32_t* tmp, uint32_t* newlen, int* status) {
  __shared__ uint32_t buf[kMergeAddMax];
  __shared__ uint32_t uni[kMergeAddMax];
  const int lane = lane_id();
  for (int64_t v = blockIdx.x; v < n; v += gridDim.x) {
    const uint64_t o0 = off[v];
    const int64_t o = (int64_t)(off[v + 1] - o0);
    const uint64_t a0 = addoff[v];
    const int64_t a = (int64_t)(addoff[v + 1] - a0);
    uint32_t* dst = tmp + o0 + a0;
    if (a == 0) {
      for (int64_t j = lane; j < o; j += 64) dst[j] = ids[o0 + j];
      if (lane == 0) newlen[v] = (uint32_t)o;
      continue;
    }
    if (a > kMergeAddMax) {
      if (lane == 0) {
        atomicOr(status, 2);
        newlen[v] = 0;
      }
      continue;
    }
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

}  // namespace

hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_fill_u32<<<blocks_for(count, 1024), 256, 0, st>>>(p, v, count);
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

hipError_t merge_rows(int64_t n, const uint64_t* off, const uint32_t* ids, const uint64_t* addoff,
                      const uint32_t* addbuf, uint32_t* tmp, uint32_t* newlen, int* status,
                      hipStream_t st) {
  int grid = (int)(n < 65536 ? n : 65536);
  k_merge_rows<<<grid, 64, 0, st>>>(n, off, ids, addoff, addbuf, tmp, newlen, status);
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
