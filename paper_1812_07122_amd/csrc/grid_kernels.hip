// Bilateral-grid approximation of Eq. (1) on the gradient fields (the fast
// filter of Paris and Durand 2006 that the paper's experiments use in place of
// the exact one, Section III-B), for gfx950.
//
// The approximation is a 3-D linear filter in (x, y, range) followed by a
// division: p and 1 are splatted into cells of s x s pixels by one range cell,
// blurred with a Gaussian (taps to +-2 cells), and read back at each pixel's
// own (x / s, y / s, range position) by trilinear interpolation.  The image is
// periodic like the exact filter's window.
//
// No global grid is stored: a workgroup owns 10 x 10 output cells of one field
// and builds, in LDS, the 16 x 16 cells (+-3) that can reach them through the
// blur and the interpolation, with the range axis (the bins the plane can use,
// at most 32, plus 2 empty bins of padding at each end; dynamic LDS sized to
// them, so narrow range axes leave room for more workgroups per CU):
//   * splat: the threads walk the local region's pixels (wrapped into the image)
//     a row at a time, coalesced, and add each pixel to its cell's bin with integer
//     LDS atomics, the value in fixed point with a power-of-two scale: integer sums
//     do not depend on the order of the adds, so they are deterministic and the
//     result does not change between runs, graph replays or served batches;
//   * blur: along the range axis per cell, then along x and y per grid line,
//     each line held in registers (in place);
//   * slice: each output pixel interpolates num and den from the 8 cells
//     around it, and the residual g - p is written in the field type (threads
//     on consecutive pixels of a row, each keeping its columns).
// The range bin floor((q - qmin) inv + 1/2) is an integer decision: it is
// computed in FP32 one rounding per operation, as the oracle computes it.
// qmin and the span come from the gradient-extrema partials of the range
// source.
#include "blfls_field.h"
#include "blfls_internal.h"
#include "blfls_launch.h"

#include <algorithm>
#include <cmath>

namespace blfls {

namespace {

constexpr int kTileCells = 10;                  // output cells per tile side
constexpr int kLocal = kTileCells + 6;          // local grid cells per side (+-3)
constexpr int kCells = kLocal * kLocal;         // 256: one splatting thread per cell
constexpr int kZPad = 2;
constexpr int kGridThreads = 256;
constexpr int kSplatBatch = 8;                  // splat rows whose loads go out together
constexpr int kSliceBatch = 4;                  // slice rows whose loads go out together
static_assert(kCells <= kGridThreads, "one thread per local cell");

__device__ __forceinline__ int wrapi(int v, int n) {
  const int m = v % n;
  return m < 0 ? m + n : m;
}

// i wrapped into [0, n) for any i (the cheap test first: only tiles at the border wrap).
__device__ __forceinline__ int wrapc(int v, int n) { return v >= 0 && v < n ? v : wrapi(v, n); }

__device__ __forceinline__ int find_grid_plane(const GridPlane* planes, int nplanes, int item) {
  int lo = 0, hi = nplanes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (2 * planes[mid].tile_begin <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// In-place 5-tap blur of n values spaced `stride` apart, zero beyond the ends.
template <int N>
__device__ __forceinline__ void blur_line(float* base, int stride, int n, const float* w) {
  float v[N];
#pragma unroll
  for (int t = 0; t < N; ++t) v[t] = t < n ? base[t * stride] : 0.0f;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    if (t < n) {
      float acc = 0.0f;
#pragma unroll
      for (int k = -2; k <= 2; ++k) {
        const int u = t + k;
        if (u >= 0 && u < N) acc += w[k + 2] * v[u];
      }
      base[t * stride] = acc;
    }
  }
}

}  // namespace

// One workgroup: (plane, field, tile of kTileCells x kTileCells output cells).  The two
// local grids (sums of values and of counts) take kCells x zs floats each of dynamic
// LDS; zs, odd for the LDS banks, covers every range bin the launch's planes can use.
// SELF: the range source is the image itself (every plane of the launch has g ==
// nullptr), so the range-source loads and the tile maximum are not needed.
template <bool SELF>
__global__ void __launch_bounds__(kGridThreads) grid_filter_kernel(const GridPlane* __restrict__ planes,
                                                                   int nplanes, int field_type, int zs) {
  extern __shared__ float grids[];
  float* const snum = grids;
  float* const sden = grids + kCells * zs;
  __shared__ float taps[2][5];
  const int item = blockIdx.x;
  const GridPlane& P = planes[find_grid_plane(planes, nplanes, item)];
  const int local = item - 2 * P.tile_begin;
  const int field = local >= P.tile_count ? 1 : 0;
  const int tile = local - field * P.tile_count;
  const int H = P.H, W = P.W, s = P.s, half = s / 2;
  const int X0 = (tile % P.tiles_x) * kTileCells;   // first output cell of the tile
  const int Y0 = (tile / P.tiles_x) * kTileCells;
  const int tid = threadIdx.x;

  // range axis: origin, scale (capped to kGridZMax bins), bins in use, blur width
  float qmin, qmax;
  field_extrema(P.minmax, field, &qmin, &qmax);
  // FP16 fields: the residual's power-of-two store scale (1 otherwise)
  const float2 fsc = field_store_scales(P.fmm);
  const float ssc = field ? fsc.y : fsc.x;
  const float span = qmax - qmin;
  float inv = P.inv_r;
  float inv_span = 1.0f;
  const bool norm = P.normalize != 0 && inv != 0.0f && span > 0.0f;
  if (norm) {
    inv_span = __fdiv_rn(1.0f, span);
    inv = __fmul_rn(inv, inv_span);
  }
  if (__fmul_rn(span, inv) > static_cast<float>(kGridZMax - 1)) inv = __fdiv_rn(static_cast<float>(kGridZMax - 1), span);
  // (the host's stride bound makes the min a no-op; it keeps every access in the grids)
  const int nz = min(static_cast<int>(floorf(__fadd_rn(__fmul_rn(span, inv), 0.5f))) + 1, zs - 2 * kZPad);
  const int zt = nz + 2 * kZPad;
  if (tid < 5) {
    const float k = static_cast<float>(tid - 2);
    const float sz = inv == 0.0f ? 0.0f : (norm ? P.sigma_r * inv / inv_span : P.sigma_r * inv);
    taps[0][tid] = expf(-(k * k) / (2.0f * P.sig_xy * P.sig_xy));
    taps[1][tid] = sz > 0.0f ? expf(-(k * k) / (2.0f * sz * sz)) : (tid == 2 ? 1.0f : 0.0f);
  }
  const float* __restrict__ f = P.f;
  constexpr bool self = SELF;
  // (a plane without a range source read by the general kernel uses its image)
  const float* __restrict__ g = self || P.g == nullptr ? P.f : P.g;
  const int64_t gp = self || P.g == nullptr ? P.pitch : P.gpitch;

  // Splat, one pixel per thread and step: the local cells (cy, cx) are grid cells
  // (Y0 - 3 + cy, X0 - 3 + cx), covering the kLocal s x kLocal s pixels (extended
  // coordinates) from ((Y0 - 3) s - s/2, (X0 - 3) s - s/2).  Consecutive threads take
  // consecutive pixels of a row, so the loads are coalesced, and add to their bins
  // with integer LDS atomics: the gradient in fixed point (scale 2^e, |sum| < 2^31)
  // and the count.  Integer sums do not depend on the order of the adds, so the
  // grids, and the result, are deterministic.
  const int side = kLocal * s;                       // local region side in pixels
  const int wc = min(side, kGridThreads);            // threads across a row
  const int rows_per_step = kGridThreads / wc;
  const int tr = tid / wc, tc = tid - (tid / wc) * wc;
  const bool active = tr < rows_per_step;
  const int ybase = (Y0 - 3) * s - half, xbase = (X0 - 3) * s - half;
  // (v * inv_s16) >> 16 == v / s for 0 <= v < 512 and s <= 32
  const unsigned inv_s16 = (65536u + static_cast<unsigned>(s) - 1u) / static_cast<unsigned>(s);

  // fixed-point exponent: 2^e max|p| s^2 < 2^30.  For a self-guided plane max|p| is
  // the field's extremum; with a separate range source it is this tile's own maximum
  // (a reduction in a fixed order, so still deterministic).
  __shared__ float red[kGridThreads / 64];
  float amax = 0.0f;
  if (self) {
    amax = fmaxf(fabsf(qmin), fabsf(qmax));
  } else {
    float m = 0.0f;
    for (int c = tc; active && c < side; c += wc) {
      const int j = wrapc(xbase + c, W);
      const int j1 = field ? j : (j + 1 == W ? 0 : j + 1);
      for (int r = tr; r < side; r += rows_per_step) {
        const int i = wrapc(ybase + r, H);
        const int i1 = field ? (i + 1 == H ? 0 : i + 1) : i;
        const float pv = load_global(f, static_cast<int64_t>(i1) * P.pitch + j1) -
                         load_global(f, static_cast<int64_t>(i) * P.pitch + j);
        m = fmaxf(m, fabsf(pv));
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((tid & 63) == 0) red[tid >> 6] = m;
  }
  int* const ni = reinterpret_cast<int*>(snum);
  int* const di = reinterpret_cast<int*>(sden);
  for (int i = tid; i < kCells * zs; i += kGridThreads) {
    ni[i] = 0;
    di[i] = 0;
  }
  __syncthreads();
  if (!self) {
#pragma unroll
    for (int w = 0; w < kGridThreads / 64; ++w) amax = fmaxf(amax, red[w]);
  }
  int ex = 0;
  (void)frexpf(__fmul_rn(amax, static_cast<float>(s * s)), &ex);
  const int e = amax > 0.0f && amax < INFINITY ? min(max(30 - ex, -120), 120) : 0;
  const float scale = ldexpf(1.0f, e), unscale = ldexpf(1.0f, -e);

  for (int c = tc; active && c < side; c += wc) {
    // the forward difference reads (i, j) and its neighbour: row i1 at column j for
    // the y field, row i at column j + 1 (wrapped) for the x field
    const int j = wrapc(xbase + c, W);
    const int j1 = field ? j : (j + 1 == W ? 0 : j + 1);
    const int cx = static_cast<int>((static_cast<unsigned>(c) * inv_s16) >> 16);
    // rows in batches of kSplatBatch: every load of the batch is issued before the
    // first atomic, so one memory round trip covers the batch
    for (int r0 = tr; r0 < side; r0 += kSplatBatch * rows_per_step) {
      // raw loads first, unconditional (rows past the region reload its last row and
      // are skipped below), so no wait falls between them
      float a0[kSplatBatch], a1[kSplatBatch], b0[kSplatBatch], b1[kSplatBatch];
#pragma unroll
      for (int u = 0; u < kSplatBatch; ++u) {
        const int r = min(r0 + u * rows_per_step, side - 1);
        const int i = wrapc(ybase + r, H);
        const int i1 = field ? (i + 1 == H ? 0 : i + 1) : i;
        a0[u] = load_global(f, static_cast<int64_t>(i) * P.pitch + j);
        a1[u] = load_global(f, static_cast<int64_t>(i1) * P.pitch + j1);
        b0[u] = 0.0f;
        b1[u] = 0.0f;
        if (!self) {
          b0[u] = load_global(g, static_cast<int64_t>(i) * gp + j);
          b1[u] = load_global(g, static_cast<int64_t>(i1) * gp + j1);
        }
      }
#pragma unroll
      for (int u = 0; u < kSplatBatch; ++u) {
        const int r = r0 + u * rows_per_step;
        if (r < side) {
          const float pvu = a1[u] - a0[u];
          const float q = self ? pvu : b1[u] - b0[u];
          const float t = __fmul_rn(__fsub_rn(q, qmin), inv);
          const int z = static_cast<int>(floorf(__fadd_rn(t, 0.5f)));
          const int cy = static_cast<int>((static_cast<unsigned>(r) * inv_s16) >> 16);
          const int slot = (cy * kLocal + cx) * zs + kZPad + z;
          atomicAdd(ni + slot, __float2int_rn(__fmul_rn(pvu, scale)));
          atomicAdd(di + slot, 1);
        }
      }
    }
  }
  __syncthreads();
  // back to FP32: one rounding of the integer, then an exact scaling by 2^-e
  for (int i = tid; i < kCells * zs; i += kGridThreads) {
    ni[i] = __float_as_int(__fmul_rn(static_cast<float>(ni[i]), unscale));
    di[i] = __float_as_int(static_cast<float>(di[i]));
  }
  __syncthreads();

  // blur along the range axis (per cell), then x, then y (per grid line)
  if (tid < kCells) {
    blur_line<kGridZMax + 2 * kZPad>(snum + tid * zs, 1, zt, taps[1]);
    blur_line<kGridZMax + 2 * kZPad>(sden + tid * zs, 1, zt, taps[1]);
  }
  __syncthreads();
  for (int l = tid; l < kLocal * zt; l += kGridThreads) {   // line (cy, z) along x
    const int cy = l / zt, z = l - (l / zt) * zt;
    blur_line<kLocal>(snum + cy * kLocal * zs + z, zs, kLocal, taps[0]);
    blur_line<kLocal>(sden + cy * kLocal * zs + z, zs, kLocal, taps[0]);
  }
  __syncthreads();
  for (int l = tid; l < kLocal * zt; l += kGridThreads) {   // line (cx, z) along y
    const int cx = l / zt, z = l - (l / zt) * zt;
    blur_line<kLocal>(snum + cx * zs + z, kLocal * zs, kLocal, taps[0]);
    blur_line<kLocal>(sden + cx * zs + z, kLocal * zs, kLocal, taps[0]);
  }
  __syncthreads();

  // slice the output pixels of the tile: pixels whose cell lies in [Y0, Y0+T) x [X0, X0+T)
  const int y_lo = max(Y0 * s - half, 0), y_hi = min((Y0 + kTileCells) * s - half, H);
  const int x_lo = max(X0 * s - half, 0), x_hi = min((X0 + kTileCells) * s - half, W);
  const int tw = x_hi - x_lo, th = y_hi - y_lo;
  const float inv_s = 1.0f / static_cast<float>(s);
  void* out = field ? P.ry : P.rx;
  // consecutive threads take consecutive pixels of a row; a thread keeps its columns
  const int swc = min(max(tw, 1), kGridThreads);
  const int srows = kGridThreads / swc;
  const int sr0 = tid / swc, sc0 = tid - (tid / swc) * swc;
  for (int jj = sc0; th > 0 && sr0 < srows && jj < tw; jj += swc) {
    const int j = x_lo + jj;
    const int j1 = field ? j : (j + 1 == W ? 0 : j + 1);
    const float fx = static_cast<float>(j) * inv_s - static_cast<float>(X0 - 3);
    const int x0 = static_cast<int>(floorf(fx));
    const float ax = fx - static_cast<float>(x0);
    for (int ii0 = sr0; ii0 < th; ii0 += kSliceBatch * srows) {
      float a0[kSliceBatch], a1[kSliceBatch], b0[kSliceBatch], b1[kSliceBatch];
#pragma unroll
      for (int u = 0; u < kSliceBatch; ++u) {   // the batch's loads first, as in the splat
        const int i = y_lo + min(ii0 + u * srows, th - 1);
        const int i1 = field ? (i + 1 == H ? 0 : i + 1) : i;
        a0[u] = load_global(f, static_cast<int64_t>(i) * P.pitch + j);
        a1[u] = load_global(f, static_cast<int64_t>(i1) * P.pitch + j1);
        b0[u] = 0.0f;
        b1[u] = 0.0f;
        if (!self) {
          b0[u] = load_global(g, static_cast<int64_t>(i) * gp + j);
          b1[u] = load_global(g, static_cast<int64_t>(i1) * gp + j1);
        }
      }
#pragma unroll
      for (int u = 0; u < kSliceBatch; ++u) {
        const int ii = ii0 + u * srows;
        if (ii < th) {
          const int i = y_lo + ii;
          const float pvu = a1[u] - a0[u];
          const float q = self ? pvu : b1[u] - b0[u];
          const float fz = __fmul_rn(__fsub_rn(q, qmin), inv) + static_cast<float>(kZPad);
          const float fy = static_cast<float>(i) * inv_s - static_cast<float>(Y0 - 3);
          const int z0 = min(max(static_cast<int>(floorf(fz)), 0), zt - 2);
          const int y0 = static_cast<int>(floorf(fy));
          const float az = fz - static_cast<float>(z0), ay = fy - static_cast<float>(y0);
          float vn = 0.0f, vd = 0.0f;
#pragma unroll
          for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
              const float wxy = (dy ? ay : 1.0f - ay) * (dx ? ax : 1.0f - ax);
              const int c = ((y0 + dy) * kLocal + (x0 + dx)) * zs + z0;
              vn += wxy * ((1.0f - az) * snum[c] + az * snum[c + 1]);
              vd += wxy * ((1.0f - az) * sden[c] + az * sden[c + 1]);
            }
          store_field(out, static_cast<int64_t>(i) * W + j, (vn / vd - pvu) * ssc, field_type);
        }
      }
    }
  }
}

int grid_cell_size(float sigma_s) { return std::max(1, static_cast<int>(std::floor(static_cast<double>(sigma_s) + 0.5))); }

int grid_tiles_x(int W, int s) { return ((W - 1 + s / 2) / s + 1 + kTileCells - 1) / kTileCells; }
int grid_tiles_y(int H, int s) { return ((H - 1 + s / 2) / s + 1 + kTileCells - 1) / kTileCells; }

// Range slots per cell for a plane's parameters.  The kernel uses nz = round(span * inv)
// + 1 bins plus kZPad on each side.  With normalisation inv = inv_r / span up to three
// roundings, so nz <= round(inv_r) + 1; one bin of slack covers the roundings and the
// cap at kGridZMax bins holds in every case.  The stride is made odd for the LDS banks.
int grid_z_stride(const GridPlane& p) {
  int nz = kGridZMax;
  if (p.inv_r == 0.0f) {
    nz = 1;
  } else if (p.normalize) {
    const double b = std::floor(static_cast<double>(p.inv_r) * (1.0 + 1e-5) + 0.5) + 2.0;
    nz = static_cast<int>(std::min(b, static_cast<double>(kGridZMax)));
  }
  return (nz + 2 * kZPad) | 1;
}

size_t grid_lds_bytes(int zs) { return 2 * sizeof(float) * static_cast<size_t>(kCells) * zs; }

hipError_t grid_init_kernels() {
  const int max_lds = static_cast<int>(grid_lds_bytes(kGridZMax + 2 * kZPad + 1));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&grid_filter_kernel<true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&grid_filter_kernel<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  return e;
}

hipError_t launch_grid(const GridPlane* planes, int nplanes, int items, int zs, bool self, int field_type,
                       hipStream_t s) {
  if (items <= 0) return hipSuccess;
  if (zs < 1 + 2 * kZPad || zs > kGridZMax + 2 * kZPad + 1) return hipErrorInvalidValue;
  if (self)
    hipLaunchKernelGGL(grid_filter_kernel<true>, dim3(items), dim3(kGridThreads), grid_lds_bytes(zs), s, planes,
                       nplanes, field_type, zs);
  else
    hipLaunchKernelGGL(grid_filter_kernel<false>, dim3(items), dim3(kGridThreads), grid_lds_bytes(zs), s, planes,
                       nplanes, field_type, zs);
  return hipGetLastError();
}

}  // namespace blfls
