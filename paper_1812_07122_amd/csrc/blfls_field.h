// Device helpers shared by the kernels that write the residual fields.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blfls_internal.h"

namespace blfls {

// Global memory accessed in its own address space.  An access through a generic
// pointer is a flat access, which also counts against the LDS wait counter, so a
// kernel that stages through LDS would wait for its LDS work at every use of a load.
__device__ __forceinline__ float load_global(const float* base, int64_t idx) {
  return ((const __attribute__((address_space(1))) float*)base)[idx];
}

template <typename T>
__device__ __forceinline__ void store_global(T* base, int64_t idx, T v) {
  ((__attribute__((address_space(1))) T*)base)[idx] = v;
}

// Store v as element idx of a packed field of type ft (FP32, BF16 or FP16,
// rounded to nearest even).
__device__ __forceinline__ void store_field(void* base, int64_t idx, float v, int ft) {
  if (ft == kF32) {
    store_global(static_cast<float*>(base), idx, v);
  } else if (ft == kBF16) {
    uint32_t b = __float_as_uint(v);
    b += 0x7FFFu + ((b >> 16) & 1u);  // round to nearest even (values are finite)
    store_global(static_cast<uint16_t*>(base), idx, static_cast<uint16_t>(b >> 16));
  } else {
    store_global(static_cast<_Float16*>(base), idx, static_cast<_Float16>(v));  // round to nearest even
  }
}

// Reduce the minmax partials of one field to the range source's extrema
// (block-wide call: every thread of the workgroup must reach it).
__device__ inline void field_extrema(const float* partial, int field, float* lo_out, float* hi_out) {
  __shared__ float red[2];
  if (threadIdx.x < 64) {
    float lo = INFINITY, hi = -INFINITY;
    for (int i = threadIdx.x; i < kMinmaxBlocks; i += 64) {
      lo = fminf(lo, partial[i * 4 + field * 2 + 0]);
      hi = fmaxf(hi, partial[i * 4 + field * 2 + 1]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off));
      hi = fmaxf(hi, __shfl_xor(hi, off));
    }
    if (threadIdx.x == 0) { red[0] = lo; red[1] = hi; }
  }
  __syncthreads();
  *lo_out = red[0];
  *hi_out = red[1];
}

// FP16 storage of the residual fields r = filter(p) - p.  Every filter's output
// is a weighted mean of the field p, so |r| <= max p - min p; a field whose span
// exceeds 2^15 is stored times 2^-e, e the smallest exponent that brings the span
// to at most 2^15 (below the FP16 maximum 65504), and the right-hand side of the
// solve multiplies it back (exact: powers of two).  Spans up to 2^15 (images in
// [0, 1], 8-bit or 15-bit data) keep scale 1.
__device__ inline float store_scale_of_span(float span) {
  if (!(span > 32768.0f)) return 1.0f;
  int k = 0;
  (void)frexpf(span, &k);          // span = m 2^k, 0.5 <= m < 1
  return ldexpf(1.0f, 15 - k);     // span 2^(15 - k) < 2^15
}

// Store scales of both fields from the image's gradient extrema partials fmm
// (nullptr: no scaling).  Block-wide call: every thread of the workgroup must
// reach it; it has its own LDS word pair, so it may follow field_extrema.
__device__ inline float2 field_store_scales(const float* fmm) {
  __shared__ float2 sc;
  if (fmm == nullptr) return make_float2(1.0f, 1.0f);
  __syncthreads();   // an earlier call's readers are done with sc
  if (threadIdx.x < 64) {
    float lo0 = INFINITY, hi0 = -INFINITY, lo1 = INFINITY, hi1 = -INFINITY;
    for (int i = threadIdx.x; i < kMinmaxBlocks; i += 64) {
      lo0 = fminf(lo0, fmm[i * 4 + 0]);
      hi0 = fmaxf(hi0, fmm[i * 4 + 1]);
      lo1 = fminf(lo1, fmm[i * 4 + 2]);
      hi1 = fmaxf(hi1, fmm[i * 4 + 3]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      lo0 = fminf(lo0, __shfl_xor(lo0, off));
      hi0 = fmaxf(hi0, __shfl_xor(hi0, off));
      lo1 = fminf(lo1, __shfl_xor(lo1, off));
      hi1 = fmaxf(hi1, __shfl_xor(hi1, off));
    }
    if (threadIdx.x == 0) sc = make_float2(store_scale_of_span(hi0 - lo0), store_scale_of_span(hi1 - lo1));
  }
  __syncthreads();
  return sc;
}

// max - min of the range source field (block-wide call).
__device__ inline float field_span(const float* partial, int field) {
  float lo, hi;
  field_extrema(partial, field, &lo, &hi);
  return hi - lo;
}

}  // namespace blfls
