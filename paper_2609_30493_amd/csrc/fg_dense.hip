// fg_dense.hip -- the blocked dense side of the random-access wall (Sec. 5.3,
// Sec. 5.4): every point's R nearest neighbours inside its leaf of S
// consecutive points, with all S^2 distances of a leaf computed as
// |x|^2 + |y|^2 - 2<x,y> and the inner products on MFMA (float32 or bfloat16
// operands, float32 accumulation).  The pair set is fixed before evaluation,
// so the product is tiled: each loaded row serves 128 others.
//
// Workgroup: 256 threads (4 waves), 128 rows of one leaf.  For each block of
// 128 columns every wave accumulates a 32 x 128 tile (four 32x32 MFMA
// accumulators) over the dimension, staged through padded LDS with the next
// chunk prefetched into registers.  Each wave owns its 32 rows outright, so
// the selection needs no block barrier.  In the 32x32 accumulator layout,
// register r of the lower half-wave always holds one fixed row and of the
// upper half another; that row's sorted top-R list of (distance, id) keys
// lives in the same half-wave, keys 2l and 2l+1 in lane l.  A candidate is
// tested against its row's R-th key with one ballot; each half-wave's
// survivors are compacted into a small per-wave LDS queue and inserted one
// per half-wave per step, both halves at once, each key's new value
// depending only on itself and its predecessor (one DPP shift, no ballot).
#include <hip/hip_bf16.h>

#include "fg_internal.h"

namespace fg {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kRows = 128;   // rows per workgroup
constexpr int kCols = 128;   // columns per block
constexpr int kRMax = 64;    // longest per-row list (one key per lane)

template <bool BF16>
struct Stage;
template <>
struct Stage<false> {  // float32 operands, K step 2
  static constexpr int KC = 16;     // elements per staged chunk
  static constexpr int PAD = 1;     // elements of padding per LDS row
  using T = float;
};
template <>
struct Stage<true> {  // bfloat16 operands, K step 16
  static constexpr int KC = 32;
  static constexpr int PAD = 8;
  using T = __bf16;
};

// A staged chunk is kRows rows of the A side and kCols rows of the B side,
// KC elements each, read as 16-byte vectors: 4 vectors per row either way,
// 1024 vectors in all, 4 per thread.
constexpr int kVecPerThread = (kRows + kCols) * 4 / 256;

// Row i of the 32x32 MFMA output held in accumulator register r of lane l.
__device__ __forceinline__ int acc_row(int r, int lane) { return (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Lane l receives lane l-1's value (DPP wave shift right by one); lane 0
// keeps its own.
__device__ __forceinline__ uint64_t shift_up64(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)v, (int)(uint32_t)v, 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(v >> 32), (int)(uint32_t)(v >> 32), 0x138, 0xF, 0xF,
                                             false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// One insertion step into two sorted lists at once, one per half-wave: keys
// 2l and 2l+1 of a half's list are s0 and s1 of its lane l.  c is the half's
// candidate (all-ones: none).  Key e becomes c where e is c's rank, key e-1
// past it; the key past the list's end falls off, and a c above every key
// leaves the list as it was.
__device__ __forceinline__ void insert_pairs(uint64_t& s0, uint64_t& s1, uint64_t c, int l) {
  const uint64_t p = shift_up64(s1);  // key 2l-1 (lane l-1's s1)
  const bool lt0 = s0 < c, lt1 = s1 < c;
  const bool plt = l == 0 || p < c;
  const uint64_t n1 = lt1 ? s1 : (lt0 ? c : s0);
  s0 = lt0 ? s0 : (plt ? c : p);
  s1 = n1;
}

template <bool BF16>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_leaf_knn(const void* xv, int64_t n, int d, int64_t stride_elems, int S,
                                                  int R, const float* norms, uint32_t* out_ids, float* out_d) {
  using St = Stage<BF16>;
  using T = typename St::T;
  constexpr int KC = St::KC, LD = St::KC + St::PAD;
  __shared__ T As[kRows * LD];
  __shared__ T Bs[kCols * LD];
  __shared__ uint64_t queue[4][64];  // per wave: survivors, lower half then upper
  const T* X = static_cast<const T*>(xv);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t leaf0 = (int64_t)blockIdx.y * S;
  const int64_t leaf1 = leaf0 + S < n ? leaf0 + S : n;
  const int64_t r0 = leaf0 + (int64_t)blockIdx.x * kRows;
  if (r0 >= leaf1) return;
  // norms of this lane's accumulator rows
  float ni[16];
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const int64_t i = r0 + 32 * w + acc_row(r, lane);
    ni[r] = i < leaf1 ? norms[i] : 0.0f;
  }
  // Lists: for accumulator register r, s0[r] / s1[r] of this half-wave.
  uint64_t s0[16], s1[16];
#pragma unroll
  for (int r = 0; r < 16; r++) s0[r] = s1[r] = ~0ull;
  const int l = lane & 31;
  const bool upper = lane >= 32;
  const bool v0 = 2 * l < R, v1 = 2 * l + 1 < R;
  const int tlane = (R - 1) >> 1;      // lane of key R-1 in the lower half
  const bool tslot1 = ((R - 1) & 1) != 0;
  auto tau_of = [&](int r) -> uint64_t {  // this half's R-th key of list r
    const uint64_t a = readlane64(tslot1 ? s1[r] : s0[r], tlane);
    const uint64_t b = readlane64(tslot1 ? s1[r] : s0[r], 32 + tlane);
    return upper ? b : a;
  };

  // Global -> registers for chunk k0 of column block c0.  float32 rows are
  // checked against d (d % 4 == 0, so a vector is wholly in or out);
  // bfloat16 rows are zero-padded to a multiple of KC by the conversion.
  auto fetch = [&](int64_t c0, int k0, uint4 (&v)[kVecPerThread]) {
#pragma unroll
    for (int it = 0; it < kVecPerThread; it++) {
      const int idx = tid + 256 * it;
      const int side = idx >> 9, rem = idx & 511, row = rem >> 2, q = rem & 3;
      const int64_t g = (side ? c0 : r0) + row;
      const int k = k0 + q * (16 / (int)sizeof(T));
      v[it] = make_uint4(0, 0, 0, 0);
      if (g < leaf1 && (BF16 || k < d)) v[it] = *reinterpret_cast<const uint4*>(X + g * stride_elems + k);
    }
  };
  auto stash = [&](const uint4 (&v)[kVecPerThread]) {
#pragma unroll
    for (int it = 0; it < kVecPerThread; it++) {
      const int idx = tid + 256 * it;
      const int side = idx >> 9, rem = idx & 511, row = rem >> 2, q = rem & 3;
      T* dst = (side ? Bs : As) + row * LD + q * (16 / (int)sizeof(T));
      if constexpr (BF16) {
        *reinterpret_cast<uint4*>(dst) = v[it];
      } else {
        dst[0] = __uint_as_float(v[it].x);
        dst[1] = __uint_as_float(v[it].y);
        dst[2] = __uint_as_float(v[it].z);
        dst[3] = __uint_as_float(v[it].w);
      }
    }
  };

  const int nk = (d + KC - 1) / KC;
  uint4 pre[kVecPerThread];
  fetch(leaf0, 0, pre);
  for (int64_t c0 = leaf0; c0 < leaf1; c0 += kCols) {
    f32x16 acc[4];
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int e = 0; e < 16; e++) acc[t][e] = 0.0f;
    for (int kc = 0; kc < nk; kc++) {
      stash(pre);
      __syncthreads();
      // prefetch the next chunk (next column block's first chunk at the end)
      if (kc + 1 < nk)
        fetch(c0, (kc + 1) * KC, pre);
      else if (c0 + kCols < leaf1)
        fetch(c0 + kCols, 0, pre);
      if constexpr (!BF16) {
#pragma unroll 4
        for (int k = 0; k < KC; k += 2) {
          float a = As[(32 * w + (lane & 31)) * LD + k + (lane >> 5)];
#pragma unroll
          for (int t = 0; t < 4; t++) {
            float b = Bs[(32 * t + (lane & 31)) * LD + k + (lane >> 5)];
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[t], 0, 0, 0);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < KC; k += 16) {
          bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[(32 * w + (lane & 31)) * LD + k + 8 * (lane >> 5)]);
#pragma unroll
          for (int t = 0; t < 4; t++) {
            bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[(32 * t + (lane & 31)) * LD + k + 8 * (lane >> 5)]);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
          }
        }
      }
      __syncthreads();
    }
    // selection
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int64_t j = c0 + 32 * t + l;
      const float nj = j < leaf1 ? norms[j] : 0.0f;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int64_t i = r0 + 32 * w + acc_row(r, lane);
        const bool valid = i < leaf1 && j < leaf1 && i != j;
        const float dist = ni[r] + nj - 2.0f * acc[t][r];
        const uint64_t key = valid ? make_key(f32_to_ord(dist), (uint32_t)j) : ~0ull;
        const bool pass = key < tau_of(r);
        const uint64_t m = ballot(pass);
        if (m) {
          const uint32_t mA = (uint32_t)m, mB = (uint32_t)(m >> 32);
          const int cntA = __popc(mA), cntB = __popc(mB);
          const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo(mA, 0));
          uint64_t* q = queue[w] + (upper ? 32 : 0);
          wave_sync();
          if (pass) q[below - (upper ? cntA : 0)] = key;
          wave_sync();
          const int cnt = upper ? cntB : cntA, kmax = cntA > cntB ? cntA : cntB;
          // four queue entries per batch (k + 3 <= 31: always inside the
          // half's 32 slots); entries past this half's count insert nothing
          for (int k = 0; k < kmax; k += 4) {
            uint64_t c[4];
#pragma unroll
            for (int u = 0; u < 4; u++) c[u] = q[k + u];
#pragma unroll
            for (int u = 0; u < 4; u++)
              if (k + u < kmax) insert_pairs(s0[r], s1[r], k + u < cnt ? c[u] : ~0ull, l);
          }
        }
      }
    }
  }
  // write the lists; keys past the leaf's other points stay at the sentinel
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const int64_t i = r0 + 32 * w + acc_row(r, lane);
    if (i < leaf1) {
      if (v0) {
        out_ids[i * R + 2 * l] = s0[r] == ~0ull ? FG_NONE : key_id(s0[r]);
        out_d[i * R + 2 * l] = s0[r] == ~0ull ? __builtin_inff() : ord_to_f32(key_hi(s0[r]));
      }
      if (v1) {
        out_ids[i * R + 2 * l + 1] = s1[r] == ~0ull ? FG_NONE : key_id(s1[r]);
        out_d[i * R + 2 * l + 1] = s1[r] == ~0ull ? __builtin_inff() : ord_to_f32(key_hi(s1[r]));
      }
    }
  }
}

// One wave per row, lanes over 4-element chunks (d % 4 == 0); the norm is
// summed per lane, then across the wave.
__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(256) k_row_norms_f32(const float* X, int64_t n, int d, int64_t stride, float* out) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    float s = 0.0f;
    for (int c = lane; c < d / 4; c += 64) {
      const float4 v = *reinterpret_cast<const float4*>(X + i * stride + 4 * c);
      s = __builtin_fmaf(v.x, v.x, s);
      s = __builtin_fmaf(v.y, v.y, s);
      s = __builtin_fmaf(v.z, v.z, s);
      s = __builtin_fmaf(v.w, v.w, s);
    }
    s = wave_sum_f32(s);
    if (lane == 0) out[i] = s;
  }
}

// Rows rounded to bfloat16 (nearest even) into a copy whose row stride dp is
// d rounded up to the staged chunk, zero-filled past d; norms of the rounded
// rows.
__global__ void __launch_bounds__(256) k_to_bf16(const float* X, int64_t n, int d, int64_t stride, __bf16* Y, int dp,
                                                 float* norms) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    float s = 0.0f;
    for (int c = lane; c < dp / 4; c += 64) {
      float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (4 * c < d) v = *reinterpret_cast<const float4*>(X + i * stride + 4 * c);
      const __bf16 b0 = (__bf16)v.x, b1 = (__bf16)v.y, b2 = (__bf16)v.z, b3 = (__bf16)v.w;
      __bf16* y = Y + i * dp + 4 * c;
      y[0] = b0;
      y[1] = b1;
      y[2] = b2;
      y[3] = b3;
      const float f0 = (float)b0, f1 = (float)b1, f2 = (float)b2, f3 = (float)b3;
      s = __builtin_fmaf(f0, f0, s);
      s = __builtin_fmaf(f1, f1, s);
      s = __builtin_fmaf(f2, f2, s);
      s = __builtin_fmaf(f3, f3, s);
    }
    s = wave_sum_f32(s);
    if (lane == 0) norms[i] = s;
  }
}

int grid1(int64_t n) {  // four rows (waves) per 256-thread block
  int64_t b = (n + 3) / 4;
  return (int)(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}

}  // namespace

int bf16_stride(int d) { return (d + Stage<true>::KC - 1) / Stage<true>::KC * Stage<true>::KC; }

size_t leaf_knn_ws_bytes(int64_t n, int d) { return (size_t)n * 4 + 256 + (size_t)n * bf16_stride(d) * 2 + 256; }

hipError_t leaf_knn(const Shape& s, int S, int R, bool bf16, void* ws, uint32_t* out_ids, float* out_d,
                    hipStream_t st) {
  float* norms = static_cast<float*>(ws);
  __bf16* xb = reinterpret_cast<__bf16*>(static_cast<char*>(ws) + (((size_t)s.n * 4 + 255) & ~(size_t)255));
  const int64_t stride = s.stride / 4;
  const float* X = reinterpret_cast<const float*>(s.x);
  dim3 grid((unsigned)((S + kRows - 1) / kRows), (unsigned)((s.n + S - 1) / S));
  if (bf16) {
    const int dp = bf16_stride(s.d);
    k_to_bf16<<<grid1(s.n), 256, 0, st>>>(X, s.n, s.d, stride, xb, dp, norms);
    k_leaf_knn<true><<<grid, 256, 0, st>>>(xb, s.n, s.d, dp, S, R, norms, out_ids, out_d);
  } else {
    k_row_norms_f32<<<grid1(s.n), 256, 0, st>>>(X, s.n, s.d, stride, norms);
    k_leaf_knn<false><<<grid, 256, 0, st>>>(X, s.n, s.d, stride, S, R, norms, out_ids, out_d);
  }
  return hipGetLastError();
}

}  // namespace fg
