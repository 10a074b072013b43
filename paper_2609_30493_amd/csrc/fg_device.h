// fg_device.h -- device helpers shared by the FGraft kernels (gfx950, wave64).
//
// Distances follow the library's declared order (see include/fgraft.h):
// a row is read as 16-byte chunks; a group of L lanes shares one row, lane g
// of the group reading chunks q = g, g+L, g+2L, ...  For float32 a chunk is
// four elements and chunk q feeds partial sum (q mod 16); lane g keeps the
// 16/L partials s = g (mod L) in registers, each updated with one fused
// multiply-add per element in chunk order.  The partials are then combined
// pairwise with offsets 8, 4, 2, 1 -- in registers while the offset is a
// multiple of L, by xor-shuffles inside the group below that.  Every group
// lane ends with the same bits, whatever L is.  uint8 rows use exact int32
// arithmetic: |x-y|^2 = |x|^2 + |y|^2 - 2<x,y> with 4-byte dot products.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FG_NONE 0xFFFFFFFFu
#define FG_KEY_NONE 0xFFFFFFFFFFFFFFFFull

namespace fg {

enum DistKind { U8L2 = 0, F32L2 = 1, F32COS = 2 };

// ---------------------------------------------------------------- keys
// A candidate key packs an order-preserving image of its distance in the
// high word and its id in the low word, so that (distance, id) order is
// unsigned 64-bit order.
__device__ __forceinline__ uint32_t f32_to_ord(float f) {
  uint32_t u = __float_as_uint(f + 0.0f);  // -0 -> +0
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_to_f32(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  return __uint_as_float(u);
}
template <int DK>
__device__ __forceinline__ float hi_to_float(uint32_t hi) {
  if constexpr (DK == U8L2) return (float)hi;  // exact below 2^24
  else return ord_to_f32(hi);
}
__device__ __forceinline__ uint64_t make_key(uint32_t hi, uint32_t id) {
  return ((uint64_t)hi << 32) | id;
}
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return (uint32_t)k; }
__device__ __forceinline__ uint32_t key_hi(uint64_t k) { return (uint32_t)(k >> 32); }

// ---------------------------------------------------------------- wave ops
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }
__device__ __forceinline__ uint64_t lanes_below() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  uint32_t lo = __shfl_xor((uint32_t)v, m, 64);
  uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  uint32_t lo = __shfl((uint32_t)v, src, 64);
  uint32_t hi = __shfl((uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}
template <typename T>
__device__ __forceinline__ T bcast0(T v) {
  return __shfl(v, 0, 64);
}

// Bitonic sort of one 64-bit key per lane, ascending across the wave.
__device__ __forceinline__ uint64_t wave_sort64(uint64_t key) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      uint64_t other = shfl_xor64(key, j);
      bool up = (lane & k) == 0;
      bool lower = (lane & j) == 0;
      uint64_t mn = key < other ? key : other;
      uint64_t mx = key < other ? other : key;
      key = (lower == up) ? mn : mx;
    }
  }
  return key;
}

// Number of entries of the sorted array a[0..n) strictly below v.
template <typename T>
__device__ __forceinline__ int lower_bound_lds(const T* a, int n, T v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------- distances
// A lane's view of one row: the 16-byte chunks q = g + L*i (i < NCH).
template <int L, int NCH>
struct Chunks {
  uint4 c[NCH];
};

template <int L, int NCH>
__device__ __forceinline__ void load_chunks(Chunks<L, NCH>& r, const uint8_t* row, int Q, int g) {
#pragma unroll
  for (int i = 0; i < NCH; i++) {
    int q = g + L * i;
    if (q < Q) r.c[i] = *reinterpret_cast<const uint4*>(row + 16 * (size_t)q);
    else r.c[i] = make_uint4(0, 0, 0, 0);
  }
}

__device__ __forceinline__ uint32_t udot4(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_udot4(a, b, c, false);
}

// uint8: this lane's contribution to |x|^2 (self-dot) of its chunks.
template <int L, int NCH>
__device__ __forceinline__ uint32_t u8_selfdot(const Chunks<L, NCH>& r) {
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < NCH; i++) {
    s = udot4(r.c[i].x, r.c[i].x, s);
    s = udot4(r.c[i].y, r.c[i].y, s);
    s = udot4(r.c[i].z, r.c[i].z, s);
    s = udot4(r.c[i].w, r.c[i].w, s);
  }
  return s;
}

template <int L>
__device__ __forceinline__ uint32_t group_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Distance between the query chunks `a` (with its full squared norm `an`
// for uint8) and the row chunks `b`, reduced over the group.  Returns the
// order-preserving image of the distance (identical in every group lane).
template <int DK, int L, int NCH>
__device__ __forceinline__ uint32_t group_dist(const Chunks<L, NCH>& a, uint32_t an,
                                               const Chunks<L, NCH>& b, int Q, int g) {
  if constexpr (DK == U8L2) {
    // int32 arithmetic is exact: the true value lies in [0, 128*255^2] per
    // 128 bytes and intermediate wrap-around cancels.
    uint32_t bb = 0, ab = 0;
#pragma unroll
    for (int i = 0; i < NCH; i++) {
      bb = udot4(b.c[i].x, b.c[i].x, bb);
      bb = udot4(b.c[i].y, b.c[i].y, bb);
      bb = udot4(b.c[i].z, b.c[i].z, bb);
      bb = udot4(b.c[i].w, b.c[i].w, bb);
      ab = udot4(a.c[i].x, b.c[i].x, ab);
      ab = udot4(a.c[i].y, b.c[i].y, ab);
      ab = udot4(a.c[i].z, b.c[i].z, ab);
      ab = udot4(a.c[i].w, b.c[i].w, ab);
    }
    uint32_t part = bb - 2u * ab;
    part = group_sum_u32<L>(part);
    return an + part;
  } else {
    constexpr int S = 16 / L;  // partials per lane
    static_assert(S >= 1, "L <= 16");
    float p[S];
#pragma unroll
    for (int s = 0; s < S; s++) p[s] = 0.0f;
#pragma unroll
    for (int i = 0; i < NCH; i++) {
      int q = g + L * i;
      if (q < Q) {
        // chunk q = g + L*i feeds partial (q mod 16) = g + L*(i mod S): slot i mod S
        float& acc = p[i % S];
        float4 xa = *reinterpret_cast<const float4*>(&a.c[i]);
        float4 xb = *reinterpret_cast<const float4*>(&b.c[i]);
        if constexpr (DK == F32L2) {
          float d0 = xa.x - xb.x, d1 = xa.y - xb.y, d2 = xa.z - xb.z, d3 = xa.w - xb.w;
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
    // in-register tree levels: offsets 8 .. L (in units of partials)
#pragma unroll
    for (int off = S / 2; off >= 1; off >>= 1)
#pragma unroll
      for (int s = 0; s < off; s++) p[s] = p[s] + p[s + off];
    float v = p[0];
    // cross-lane levels: offsets L/2 .. 1
#pragma unroll
    for (int off = L / 2; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
    if constexpr (DK == F32COS) v = 1.0f - v;
    return f32_to_ord(v);
  }
}

}  // namespace fg
