// HDR tone mapping in the log domain (the experiments section's use of
// BLF-LS: the framework of Durand and Dorsey 2002 with BLF-LS as the
// base/detail split), for gfx950.  Three pointwise or reduction passes around
// one blfls_smooth of the log intensity:
//   * tm_log_kernel:     L = log10(max((20 R + 40 G + B) / 61, floor));
//   * tm_extrema_kernel: min and max of the smoothed base, one partial per
//                        workgroup (rows strided over the workgroups);
//   * tm_combine_kernel: every workgroup reduces the partials, then
//                        out_c = c / I * 10^((base - max) cf + L - base),
//                        cf = log10(contrast) / (max - min) (1 for a constant base).
// All FP32; the exponentials and logarithms are the device's exp2 / log2.
#include "blfls_internal.h"
#include "blfls_launch.h"

#include <algorithm>

namespace blfls {

namespace {
constexpr int kThreads = 256;
constexpr float kLog10of2 = 0.30102999566398120f;   // log10(2)
constexpr float kLog2of10 = 3.32192809488736235f;   // log2(10)
}  // namespace

__global__ void __launch_bounds__(kThreads) tm_log_kernel(const float* __restrict__ rgb, int64_t pitch, int H, int W,
                                                         float floor_i, float* __restrict__ L) {
  const int64_t n = static_cast<int64_t>(H) * W;
  const int64_t chan = static_cast<int64_t>(H) * pitch;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int64_t i = e / W, j = e - i * W;
    const int64_t at = i * pitch + j;
    const float inten = fmaxf((20.0f * rgb[at] + 40.0f * rgb[chan + at] + rgb[2 * chan + at]) * (1.0f / 61.0f),
                              floor_i);
    L[e] = log2f(inten) * kLog10of2;
  }
}

// One partial (min, max) per workgroup: rows blk, blk + gridDim.x, ...
__global__ void __launch_bounds__(kThreads) tm_extrema_kernel(const float* __restrict__ base, int H, int W,
                                                             float* __restrict__ partial) {
  __shared__ float red[2][kThreads / 64];
  float lo = INFINITY, hi = -INFINITY;
  for (int i = blockIdx.x; i < H; i += gridDim.x) {
    const float* row = base + static_cast<int64_t>(i) * W;
    for (int j = threadIdx.x; j < W; j += kThreads) {
      lo = fminf(lo, row[j]);
      hi = fmaxf(hi, row[j]);
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, off));
    hi = fmaxf(hi, __shfl_xor(hi, off));
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = lo;
    red[1][threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      lo = fminf(lo, red[0][w]);
      hi = fmaxf(hi, red[1][w]);
    }
    partial[2 * blockIdx.x] = lo;
    partial[2 * blockIdx.x + 1] = hi;
  }
}

__global__ void __launch_bounds__(kThreads) tm_combine_kernel(const float* __restrict__ rgb, float* __restrict__ out,
                                                             int64_t pitch, int H, int W, float floor_i,
                                                             const float* __restrict__ L,
                                                             const float* __restrict__ base,
                                                             const float* __restrict__ partial, int nparts,
                                                             float log_contrast) {
  __shared__ float ext[2];
  if (threadIdx.x < 64) {
    float lo = INFINITY, hi = -INFINITY;
    for (int k = threadIdx.x; k < nparts; k += 64) {
      lo = fminf(lo, partial[2 * k]);
      hi = fmaxf(hi, partial[2 * k + 1]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off));
      hi = fmaxf(hi, __shfl_xor(hi, off));
    }
    if (threadIdx.x == 0) { ext[0] = lo; ext[1] = hi; }
  }
  __syncthreads();
  const float lo = ext[0], hi = ext[1];
  const float cf = hi > lo ? log_contrast / (hi - lo) : 1.0f;
  const int64_t n = static_cast<int64_t>(H) * W;
  const int64_t chan = static_cast<int64_t>(H) * pitch;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int64_t i = e / W, j = e - i * W;
    const int64_t at = i * pitch + j;
    const float r = rgb[at], g = rgb[chan + at], b = rgb[2 * chan + at];
    const float inten = fmaxf((20.0f * r + 40.0f * g + b) * (1.0f / 61.0f), floor_i);
    const float bs = base[e];
    const float lout = (bs - hi) * cf + (L[e] - bs);
    const float scale = exp2f(lout * kLog2of10) / inten;
    out[at] = r * scale;
    out[chan + at] = g * scale;
    out[2 * chan + at] = b * scale;
  }
}

int tm_extrema_blocks() { return kMinmaxBlocks; }

hipError_t launch_tm_log(const float* rgb, int64_t pitch, int H, int W, float floor_i, float* L, hipStream_t s) {
  const int64_t n = static_cast<int64_t>(H) * W;
  const int blocks = static_cast<int>(std::min<int64_t>((n + kThreads - 1) / kThreads, 8192));
  hipLaunchKernelGGL(tm_log_kernel, dim3(blocks), dim3(kThreads), 0, s, rgb, pitch, H, W, floor_i, L);
  return hipGetLastError();
}

hipError_t launch_tm_finish(const float* rgb, float* out, int64_t pitch, int H, int W, float floor_i, const float* L,
                            const float* base, float* partial, float log_contrast, hipStream_t s) {
  hipLaunchKernelGGL(tm_extrema_kernel, dim3(kMinmaxBlocks), dim3(kThreads), 0, s, base, H, W, partial);
  const int64_t n = static_cast<int64_t>(H) * W;
  const int blocks = static_cast<int>(std::min<int64_t>((n + kThreads - 1) / kThreads, 8192));
  hipLaunchKernelGGL(tm_combine_kernel, dim3(blocks), dim3(kThreads), 0, s, rgb, out, pitch, H, W, floor_i, L, base,
                     static_cast<const float*>(partial), static_cast<int>(kMinmaxBlocks), log_contrast);
  return hipGetLastError();
}

}  // namespace blfls
