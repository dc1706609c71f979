// Small kernels around the filter and the solve:
//  * descriptor upload from kernel arguments into device memory;
//  * gradient extrema of the range source for the normalisation flag (the
//    experiments section maps images and gradients to [0, 1] before smoothing;
//    for Eq. (1), whose weights see only differences, that is sigma_r scaled by
//    the field's span), reduced per workgroup with wavefront shuffles;
//  * the circular Gaussian that smooths the initial guidance of the rolling
//    guidance extension (Section III-D), as two separable passes.
#include "blfls_field.h"
#include "blfls_internal.h"
#include "blfls_launch.h"
#include "blfls_work.h"

namespace blfls {

__global__ void desc_copy_kernel(DescChunk chunk, uint32_t* __restrict__ dst, int nwords) {
  for (int i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = chunk.words[i];
}

hipError_t launch_desc_copy(const void* host_src, size_t bytes, void* dev_dst, hipStream_t s) {
  const uint8_t* src = static_cast<const uint8_t*>(host_src);
  uint8_t* dst = static_cast<uint8_t*>(dev_dst);
  constexpr size_t kChunkBytes = sizeof(DescChunk::words);
  for (size_t off = 0; off < bytes; off += kChunkBytes) {
    DescChunk c;
    const size_t n = bytes - off < kChunkBytes ? bytes - off : kChunkBytes;
    memcpy(c.words, src + off, n);
    const int nwords = static_cast<int>((n + 3) / 4);
    hipLaunchKernelGGL(desc_copy_kernel, dim3(1), dim3(256), 0, s, c,
                       reinterpret_cast<uint32_t*>(dst + off), nwords);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

constexpr int kMinmaxBatch = 8;   // columns per thread whose loads go out together

// partial[b] = (min D_x, max D_x, min D_y, max D_y) over the elements of block b
// (kMinmaxBlocks blocks per plane, each a contiguous band of rows, so a row's
// lower neighbour is mostly the band's own next row, already in cache).
__device__ __forceinline__ void minmax_item(const AuxPlane& P, int blk) {
  const int H = P.H, W = P.W;
  float lx = INFINITY, hx = -INFINITY, ly = INFINITY, hy = -INFINITY;
  // threads stride the columns, kMinmaxBatch at a time with every load issued
  // before the first use.  Columns past the row are clamped to its last one: a
  // repeated value leaves a min or max unchanged, so they need no guard.
  const int i_begin = static_cast<int>(static_cast<int64_t>(H) * blk / kMinmaxBlocks);
  const int i_end = static_cast<int>(static_cast<int64_t>(H) * (blk + 1) / kMinmaxBlocks);
  for (int i = i_begin; i < i_end; ++i) {
    const int64_t o = static_cast<int64_t>(i) * P.pitch;
    const int64_t on = static_cast<int64_t>(i + 1 == H ? 0 : i + 1) * P.pitch;
    for (int j0 = threadIdx.x; j0 < W; j0 += 256 * kMinmaxBatch) {
      float v[kMinmaxBatch], vr[kMinmaxBatch], vd[kMinmaxBatch];
#pragma unroll
      for (int u = 0; u < kMinmaxBatch; ++u) {
        const int j = min(j0 + 256 * u, W - 1);
        v[u] = load_global(P.src, o + j);
        vr[u] = load_global(P.src, o + (j + 1 == W ? 0 : j + 1));
        vd[u] = load_global(P.src, on + j);
      }
#pragma unroll
      for (int u = 0; u < kMinmaxBatch; ++u) {
        const float gx = vr[u] - v[u];
        const float gy = vd[u] - v[u];
        lx = fminf(lx, gx); hx = fmaxf(hx, gx);
        ly = fminf(ly, gy); hy = fmaxf(hy, gy);
      }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    lx = fminf(lx, __shfl_xor(lx, off));
    hx = fmaxf(hx, __shfl_xor(hx, off));
    ly = fminf(ly, __shfl_xor(ly, off));
    hy = fmaxf(hy, __shfl_xor(hy, off));
  }
  __shared__ float red[4][4];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[wave][0] = lx; red[wave][1] = hx; red[wave][2] = ly; red[wave][3] = hy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float o0 = red[0][0], o1 = red[0][1], o2 = red[0][2], o3 = red[0][3];
    for (int w = 1; w < 4; ++w) {
      o0 = fminf(o0, red[w][0]); o1 = fmaxf(o1, red[w][1]);
      o2 = fminf(o2, red[w][2]); o3 = fmaxf(o3, red[w][3]);
    }
    float* out = P.partial + blk * 4;
    out[0] = o0; out[1] = o1; out[2] = o2; out[3] = o3;
  }
  __syncthreads();
}

// work == nullptr: grid (kMinmaxBlocks, planes); else a fixed grid strides over
// the work header's planes x kMinmaxBlocks items.
__global__ void __launch_bounds__(256) minmax_kernel(const AuxPlane* __restrict__ planes,
                                                     WorkHeader* __restrict__ work) {
  if (work == nullptr) {
    minmax_item(planes[blockIdx.y], blockIdx.x);
    return;
  }
  const AuxPlane* pl = static_cast<const AuxPlane*>(work->planes);
  const int total = work->items;
  for (;;) {
    const int it = grab_item(work->next[0], total, false);
    if (it >= total) break;
    minmax_item(pl[it / kMinmaxBlocks], it % kMinmaxBlocks);
  }
}

hipError_t launch_minmax(const AuxPlane* planes, int nplanes, hipStream_t s, WorkHeader* work, int grid) {
  if (work != nullptr) {
    hipLaunchKernelGGL(minmax_kernel, dim3(grid), dim3(256), 0, s, planes, work);
    return hipGetLastError();
  }
  if (nplanes <= 0) return hipSuccess;
  hipLaunchKernelGGL(minmax_kernel, dim3(kMinmaxBlocks, nplanes), dim3(256), 0, s, planes, work);
  return hipGetLastError();
}

// Separable circular Gaussian: pass 0 rows (src -> tmp), pass 1 columns (tmp -> dst).
// Item (plane, chunk): chunk c of kGaussChunks covers pixels c*256 + k*kGaussChunks*256.
constexpr int kGaussChunks = 256;

__device__ __forceinline__ void gauss_item(const AuxPlane& P, int chunk, int pass) {
  const int H = P.H, W = P.W, rg = P.rg;
  const int64_t n = static_cast<int64_t>(H) * W;
  for (int64_t idx = static_cast<int64_t>(chunk) * 256 + threadIdx.x; idx < n;
       idx += static_cast<int64_t>(kGaussChunks) * 256) {
    const int i = static_cast<int>(idx / W);
    const int j = static_cast<int>(idx - static_cast<int64_t>(i) * W);
    float acc = 0.0f;
    if (pass == 0) {
      const float* row = P.src + static_cast<int64_t>(i) * P.pitch;
      for (int d = -rg; d <= rg; ++d) {
        int jj = (j + d) % W;
        if (jj < 0) jj += W;
        acc = fmaf(P.gw[kMaxR + d], row[jj], acc);
      }
      P.tmp[idx] = acc;
    } else {
      for (int d = -rg; d <= rg; ++d) {
        int ii = (i + d) % H;
        if (ii < 0) ii += H;
        acc = fmaf(P.gw[kMaxR + d], P.tmp[static_cast<int64_t>(ii) * W + j], acc);
      }
      P.dst[idx] = acc;
    }
  }
}

__global__ void __launch_bounds__(256) gauss_kernel(const AuxPlane* __restrict__ planes, int pass,
                                                    WorkHeader* __restrict__ work) {
  if (work == nullptr) {
    gauss_item(planes[blockIdx.y], blockIdx.x, pass);
    return;
  }
  const AuxPlane* pl = static_cast<const AuxPlane*>(work->planes);
  const int total = work->items;
  for (;;) {
    // pass 0 draws from counter [1], pass 1 from [2]: both start at zero
    const int it = grab_item(work->next[1 + pass], total, false);
    if (it >= total) break;
    gauss_item(pl[it / kGaussChunks], it % kGaussChunks, pass);
  }
}

hipError_t launch_gauss(const AuxPlane* planes, int nplanes, int64_t max_pixels, hipStream_t s,
                        WorkHeader* work, int grid) {
  (void)max_pixels;
  for (int pass = 0; pass < 2; ++pass) {
    if (work != nullptr)
      hipLaunchKernelGGL(gauss_kernel, dim3(grid), dim3(256), 0, s, planes, pass, work);
    else if (nplanes > 0)
      hipLaunchKernelGGL(gauss_kernel, dim3(kGaussChunks, nplanes), dim3(256), 0, s, planes, pass, work);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int gauss_chunks() { return kGaussChunks; }

}  // namespace blfls
