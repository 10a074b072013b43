// fg_screen.hip -- the narrow copy of float32 rows that the screened harvest
// reads first (Sec. 5.3: the harvest's cost per evaluation is the bytes of
// one row; a half- or quarter-width copy rejects most candidates at a
// fraction of them).
//
// One wave per row.  bfloat16: round to nearest even.  fp8-e4m3 (OCP): the
// row is scaled by the power of two 2^k that brings its largest magnitude
// to at most 448, converted by the hardware, and read back as
// code * 2^-k; int8: codes rint(x / s) with s = fl(max|x| / 127), read
// back as fl(code * s).  For every row the norm of the actual error |u^ - u| and the
// norm |u| are bounded from above in float32 (no float64 on the device): each
// element error is exact in float32, the squares of the row's elements and
// errors are summed after scaling by a power of two that keeps them below
// one, and the sum is raised by its rounding bound (standard model, any
// summation order: S <= (S~ + d 2^-125)(1 + gamma_d), the 2^-125 term
// covering squares and sums flushed to zero), so the margin the search uses
// bounds the copy that the search reads.  For bfloat16 an optional split
// copy holds hi and each element's remainder x - hi rounded to bfloat16
// (lo), so that hi + lo carries 16 significant bits, interleaved per
// 16-element step (32 bytes of hi, then 32 of lo): the prune tiles read both
// halves of a step from one 64-byte span.
//
// Each narrow row ends in a 16-byte trailer (err, norm, sinv, 0) right after
// its codes, and rows are a whole number of 128-byte lines apart: a screened
// evaluation reads the lines of one row and nothing else (at d = 100, one
// line for fp8 and two for bfloat16, against four for the float32 row).
#include "fg_internal.h"

namespace fg {

namespace {

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// An upper bound on sqrt(S) * 2^ex from the float32 sum s~ of the d squares
// that make up S / 2^(2 ex) (each square below one):
//   S / 2^(2 ex) <= (s~ + d 2^-125)(1 + gamma_d), gamma_d = d u / (1 - d u),
// u = 2^-24; the factor is evaluated as 1 + 2 gamma_d, whose excess over
// 1 + gamma_d (d u >= 4u here) covers the three roundings of the bound
// itself.  The root (correctly rounded) is raised by 2^-22 of itself and
// one unit in the last place.
__device__ __forceinline__ float norm_bound(float s, int d, int ex) {
  const float u = 5.9604645e-08f;
  const float g = (float)d * u / (1.0f - (float)d * u);
  const float S = (s + (float)d * 2.3509887e-38f) * (1.0f + 2.0f * g);  // 2^-125
  float r = __builtin_sqrtf(S);
  r = r * (1.0f + 2.3841858e-07f);                                         // 2^-22
  r = __uint_as_float(__float_as_uint(r) + 1u);
  return ldexpf(r, ex);
}

__device__ __forceinline__ float wave_max_f32(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  const uint32_t b = __float_as_uint(f);
  return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// Elements are handled four at a time (d % 4 == 0): element 4c..4c+3 by
// lane c mod 64.
template <int SCR>
__global__ void __launch_bounds__(256) k_make_screen(const uint8_t* x, int64_t stride, int64_t n, int d,
                                                     uint8_t* xs, int64_t xs_stride, int64_t xs_tail, float* err,
                                                     float* norm, float* sinv, uint8_t* sp, int64_t sp_stride) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int C = d / 4;
  for (int64_t i = wave; i < n; i += nwaves) {
    const float* row = reinterpret_cast<const float*>(x + i * stride);
    float mx = 0.0f;
    for (int c = lane; c < C; c += 64) {
      const float4 v = *reinterpret_cast<const float4*>(row + 4 * c);
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
    mx = wave_max_f32(mx);
    // mx < 2^ex: every element and every element error scaled by 2^-ex is
    // below one in magnitude (the errors are at most the elements' size)
    int ex = 0;
    if (mx > 0.0f) (void)frexpf(mx, &ex);
    float scale = 1.0f, inv = 1.0f;
    if constexpr (SCR == SCR_FP8) {
      int k = 0;
      if (mx > 0.0f) {
        // largest k with mx * 2^k <= 448 = 0.875 * 2^9, from mx = f 2^ex,
        // f in [1/2, 1); the products with powers of two are exact
        k = 9 - ex;
        while (ldexpf(mx, k) > 448.0f) k--;
        while (ldexpf(mx, k + 1) <= 448.0f) k++;
        if (k > 100) k = 100;
        if (k < -100) k = -100;
      }
      scale = ldexpf(1.0f, k);
      inv = ldexpf(1.0f, -k);
    }
    if constexpr (SCR == SCR_INT8) {  // symmetric: codes rint(x / s) in [-127, 127]
      scale = mx / 127.0f;
      inv = scale;  // the trailer's factor: a code reads back as fl(code * s)
    }
    float e2 = 0.0f, n2 = 0.0f;
    for (int c = lane; c < C; c += 64) {
      const float4 v = *reinterpret_cast<const float4*>(row + 4 * c);
      const float a[4] = {v.x, v.y, v.z, v.w};
      float back[4];
      if constexpr (SCR == SCR_BF16) {
        uint16_t h[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
          h[t] = bf16_rne(a[t]);
          back[t] = __uint_as_float((uint32_t)h[t] << 16);
        }
        uint2 w;
        w.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
        w.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
        if (xs) *reinterpret_cast<uint2*>(xs + i * xs_stride + 8 * (int64_t)c) = w;
        if (sp) {  // the remainder x - hi (exact in float32), rounded to bfloat16
          uint16_t lo[4];
#pragma unroll
          for (int t = 0; t < 4; t++) lo[t] = bf16_rne(a[t] - back[t]);
          uint2 wl;
          wl.x = (uint32_t)lo[0] | ((uint32_t)lo[1] << 16);
          wl.y = (uint32_t)lo[2] | ((uint32_t)lo[3] << 16);
          uint8_t* at = sp + i * sp_stride + 64 * (int64_t)(c >> 2) + 8 * (c & 3);
          *reinterpret_cast<uint2*>(at) = w;
          *reinterpret_cast<uint2*>(at + 32) = wl;
        }
      } else if constexpr (SCR == SCR_INT8) {
        uint32_t w = 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
          float q8 = scale > 0.0f ? __builtin_rintf(a[t] / scale) : 0.0f;
          q8 = fminf(fmaxf(q8, -127.0f), 127.0f);
          back[t] = q8 * scale;
          w |= ((uint32_t)(int)q8 & 0xFFu) << (8 * t);
        }
        *reinterpret_cast<uint32_t*>(xs + i * xs_stride + 4 * (int64_t)c) = w;
      } else {
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(a[0] * scale, a[1] * scale, 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(a[2] * scale, a[3] * scale, w, true);
        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
        back[0] = lo[0] * inv;
        back[1] = lo[1] * inv;
        back[2] = hi[0] * inv;
        back[3] = hi[1] * inv;
        *reinterpret_cast<int*>(xs + i * xs_stride + 4 * (int64_t)c) = w;
      }
#pragma unroll
      for (int t = 0; t < 4; t++) {
        // back and a are within a factor of two of each other (or back is
        // zero), so their difference is exact in float32 (Sterbenz; int8: a
        // code q != 0 comes from fl(x / s) > |q| - 1/2 >= 1/2, ties going
        // to even, so |x| > |q| s / 2 for |q| = 1 and within 0.8..1.34 of
        // fl(q s) for larger |q|)
        const float e = ldexpf(back[t] - a[t], -ex), y = ldexpf(a[t], -ex);
        e2 = __builtin_fmaf(e, e, e2);
        n2 = __builtin_fmaf(y, y, n2);
      }
    }
    if constexpr (SCR == SCR_BF16) {  // zero the padding (read by 16-element steps)
      if (xs)
        for (int64_t c = C + lane; c < xs_stride / 8; c += 64)
          if (8 * c < xs_tail || 8 * c >= xs_tail + 16)
            *reinterpret_cast<uint2*>(xs + i * xs_stride + 8 * c) = make_uint2(0, 0);
      if (sp)
        for (int64_t c = C + lane; c < sp_stride / 16; c += 64) {
          uint8_t* at = sp + i * sp_stride + 64 * (c >> 2) + 8 * (c & 3);
          *reinterpret_cast<uint2*>(at) = make_uint2(0, 0);
          *reinterpret_cast<uint2*>(at + 32) = make_uint2(0, 0);
        }
    }
    e2 = wave_sum_f32(e2);
    n2 = wave_sum_f32(n2);
    if (lane == 0) {  // an all-zero row is copied exactly
      const float eb = mx > 0.0f ? norm_bound(e2, d, ex) : 0.0f;
      const float nb = mx > 0.0f ? norm_bound(n2, d, ex) : 0.0f;
      if (xs) *reinterpret_cast<float4*>(xs + i * xs_stride + xs_tail) = make_float4(eb, nb, inv, 0.0f);
      if (err) err[i] = eb;
      if (norm) norm[i] = nb;
      if (sinv) sinv[i] = inv;
    }
  }
}

}  // namespace

int64_t screen_tail(int d, int screen) {
  if (screen == SCR_BF16) return (2 * (int64_t)d + 31) / 32 * 32;  // whole 16-element steps
  return ((int64_t)d + 15) / 16 * 16;
}

int64_t screen_stride(int d, int screen) { return (screen_tail(d, screen) + 16 + 127) / 128 * 128; }

int64_t split_stride(int d) { return (4 * (int64_t)d + 63) / 64 * 64; }

hipError_t make_screen(const Shape& s, int screen, uint8_t* xs, float* err, float* norm, float* sinv,
                       hipStream_t st, uint8_t* sp) {
  const int64_t xst = screen_stride(s.d, screen), tail = screen_tail(s.d, screen);
  int64_t blocks = (s.n + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (screen == SCR_BF16)
    k_make_screen<SCR_BF16><<<(unsigned)blocks, 256, 0, st>>>(s.x, s.stride, s.n, s.d, xs, xst, tail, err, norm, sinv,
                                                              sp, split_stride(s.d));
  else if (screen == SCR_INT8)
    k_make_screen<SCR_INT8><<<(unsigned)blocks, 256, 0, st>>>(s.x, s.stride, s.n, s.d, xs, xst, tail, err, norm,
                                                              sinv, nullptr, 0);
  else
    k_make_screen<SCR_FP8><<<(unsigned)blocks, 256, 0, st>>>(s.x, s.stride, s.n, s.d, xs, xst, tail, err, norm, sinv,
                                                             nullptr, 0);
  return hipGetLastError();
}

}  // namespace fg
