// Normalized-convolution filter of the domain transform on the gradient
// fields (NC-LS, Section III-D: the NC filter of Gastal and Oliveira 2011 in
// place of the bilateral filter of Eq. (1)), for gfx950.
//
// Along a line the domain transform advances by d(t) = 1 + a |q(t) - q(t-1)|
// per pixel (a = sigma_s / sigma_r, q the range source's gradient field of the
// same axis, times 1/span(q) with the normalise flag); a pass replaces each
// value by the mean of the values on its line whose transformed distance is at
// most r_k.  Round k = 1..N is a row pass then a column pass with
// r_k = 3 sigma_s 2^(N-k) / sqrt(4^N - 1); the increments come from the range
// source every time (the transform is not recomputed from intermediate
// results), and windows stop at the image borders.
//
// Since d >= 1, a window never reaches more than floor(r_k) pixels from its
// centre, so each pass is a halo-tile kernel like the bilateral filter's:
//   * row passes: a wave owns a 256-pixel row segment (four outputs per
//     lane); the segment plus an R-pixel halo of values and increments is
//     staged in LDS;
//   * column passes: a workgroup owns a 32-column x 32-row tile (a wave holds
//     32 columns x 2 row groups) with an R-row halo in LDS,
//     so global loads read whole 128-byte lines;
//   * each output walks outward from its pixel, accumulating the increments in
//     FP32 (one rounding per addition, no contraction) until the distance
//     exceeds r_k, and averages the values it passed.  Window membership is an
//     integer decision, so it is computed exactly as the oracle computes it.
// The first pass forms the gradient field from f; passes ping-pong between
// two FP32 buffers per field; the last pass writes the residual
// r = NC(p) - p in the field type, which the Fourier solve consumes as it does
// the bilateral filter's.
#include "blfls_field.h"
#include "blfls_internal.h"
#include "blfls_launch.h"

namespace blfls {

namespace {

constexpr int kColW = 32;       // columns of a column-pass tile
constexpr int kRowSeg = 256;    // pixels of a row segment (one wave, four per lane)
constexpr int kRowWaves = 4;    // row segments per row-pass workgroup
constexpr int kColRows = 32;    // rows of a column-pass tile (8 per wave)
constexpr int kLine = kRowSeg + 2 * kNcMaxR;
constexpr int kLineLoads = (kLine + 63) / 64;  // staged values per lane

__device__ __forceinline__ int next_wrap(int i, int n) { return i + 1 == n ? 0 : i + 1; }

// Circular forward difference of image x along the field's axis at (i, j).
__device__ __forceinline__ float grad_at(const float* __restrict__ x, int64_t pitch, int H, int W, int i, int j,
                                         int field) {
  const float v = load_global(x, static_cast<int64_t>(i) * pitch + j);
  if (field == 0) return load_global(x, static_cast<int64_t>(i) * pitch + next_wrap(j, W)) - v;
  return load_global(x, static_cast<int64_t>(next_wrap(i, H)) * pitch + j) - v;
}

// Domain-transform increment between neighbouring guide values q0 -> q1,
// one FP32 rounding per operation: 1 + (a |q1 - q0|) [* inv].
__device__ __forceinline__ float dt_increment(float q1, float q0, float a, float inv, bool scaled) {
  float t = __fmul_rn(a, fabsf(__fsub_rn(q1, q0)));
  if (scaled) t = __fmul_rn(t, inv);
  return __fadd_rn(1.0f, t);
}

template <bool COLS>
__device__ __forceinline__ int find_nc_plane(const NcPlane* planes, int nplanes, int item) {
  int lo = 0, hi = nplanes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int begin = COLS ? planes[mid].cbegin : planes[mid].rbegin;
    if (begin <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// 1 / span of the range-source field with the normalise flag (block-wide call).
__device__ __forceinline__ bool field_scale(const NcPlane& P, int field, float* inv) {
  *inv = 1.0f;
  if (P.minmax == nullptr || P.a == 0.0f) return false;
  const float span = field_span(P.minmax, field);
  if (!(span > 0.0f)) return false;
  *inv = __fdiv_rn(1.0f, span);
  return true;
}

// Mean of the values within transformed distance r of position t0 of a staged
// line (values v[], increments d[]: d[t] joins t-1 and t); `right` / `left`
// bound the walk (pixels to the image border and the halo radius).  The walk
// reads four steps' values and increments at a time (one LDS round trip per
// four steps) and then applies them strictly in order, so the FP32 distance
// is the same running sum as one step at a time.
__device__ __forceinline__ float nc_window_mean(const float* v, const float* d, int stride, int t0, int right,
                                                int left, float r) {
  constexpr int kU = 4;
  float sum = v[t0 * stride];
  int cnt = 1;
  float dist = 0.0f;
  bool live = right > 0;
  for (int k = 1; live; k += kU) {
    float dd[kU], vv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + min(k + u, right);
      dd[u] = d[t * stride];
      vv[u] = v[t * stride];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (live) {
        dist = __fadd_rn(dist, dd[u]);
        if (dist <= r) {
          sum += vv[u];
          ++cnt;
        } else {
          live = false;
        }
        if (k + u >= right) live = false;
      }
    }
  }
  dist = 0.0f;
  live = left > 0;
  for (int k = 1; live; k += kU) {
    float dd[kU], vv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int kk = min(k + u, left);
      dd[u] = d[(t0 - kk + 1) * stride];
      vv[u] = v[(t0 - kk) * stride];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (live) {
        dist = __fadd_rn(dist, dd[u]);
        if (dist <= r) {
          sum += vv[u];
          ++cnt;
        } else {
          live = false;
        }
        if (k + u >= left) live = false;
      }
    }
  }
  return sum / static_cast<float>(cnt);
}

}  // namespace

// Row pass: items (plane, field, 4-row band, 64-column segment).  FIRST forms
// the gradient field from f; otherwise reads buf[src].  Writes buf[src ^ 1].
template <bool FIRST>
__global__ void __launch_bounds__(256) nc_rows_kernel(const NcPlane* __restrict__ planes, int nplanes, int src,
                                                      float r, int R) {
  __shared__ float sv[kRowWaves][kLine];
  __shared__ float sd[kRowWaves][kLine];
  const int item = blockIdx.x;
  const NcPlane& P = planes[find_nc_plane<false>(planes, nplanes, item)];
  const int local = item - P.rbegin;
  const int per_field = P.rcount >> 1;
  const int field = local >= per_field ? 1 : 0;
  const int tile = local - field * per_field;
  const int H = P.H, W = P.W;
  const int segs = (W + kRowSeg - 1) / kRowSeg;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = (tile / segs) * kRowWaves + wave;
  const int j0 = (tile % segs) * kRowSeg;
  float inv;
  const bool scaled = field_scale(P, field, &inv);
  const float* __restrict__ f = P.f;
  const float* __restrict__ g = P.g ? P.g : P.f;
  const int64_t gp = P.g ? P.gpitch : P.pitch;
  const float* __restrict__ in = P.buf[src][field];
  if (i < H) {
    // every load of the staged line is issued before the first LDS store
    float vv[kLineLoads], dd[kLineLoads];
#pragma unroll
    for (int u = 0; u < kLineLoads; ++u) {
      const int t = lane + 64 * u;
      const int m = j0 - R + t;
      vv[u] = 0.0f;
      dd[u] = 0.0f;
      if (t < kRowSeg + 2 * R && m >= 0 && m < W) {
        vv[u] = FIRST ? grad_at(f, P.pitch, H, W, i, m, field) : load_global(in, static_cast<int64_t>(i) * W + m);
        if (m >= 1)
          dd[u] = dt_increment(grad_at(g, gp, H, W, i, m, field), grad_at(g, gp, H, W, i, m - 1, field), P.a, inv,
                               scaled);
      }
    }
#pragma unroll
    for (int u = 0; u < kLineLoads; ++u) {
      const int t = lane + 64 * u;
      if (t < kLine) {
        sv[wave][t] = vv[u];
        sd[wave][t] = dd[u];
      }
    }
  }
  __syncthreads();
  if (i < H) {
#pragma unroll
    for (int q = 0; q < kRowSeg / 64; ++q) {
      const int j = j0 + lane + 64 * q;
      if (j < W) {
        const float out = nc_window_mean(sv[wave], sd[wave], 1, lane + 64 * q + R, min(R, W - 1 - j), min(R, j), r);
        store_global(P.buf[src ^ 1][field], static_cast<int64_t>(i) * W + j, out);
      }
    }
  }
}

// Column pass: items (plane, field, 32-column x 32-row tile).  Reads buf[src];
// writes buf[src ^ 1], or with LAST the residual NC(p) - p in field type FT.
// Lane l of a wave takes column l mod 32 and, of the wave's 8 rows, the 4
// starting at 4 (l / 32).  Dynamic LDS: 2 x (32 + 2R) x 32 floats.
template <bool LAST>
__global__ void __launch_bounds__(256) nc_cols_kernel(const NcPlane* __restrict__ planes, int nplanes, int src,
                                                      float r, int R, int field_type) {
  extern __shared__ float smem[];
  constexpr int kRowsPerLoad = 256 / kColW;   // staged rows per load instruction of the workgroup
  const int rows = kColRows + 2 * R;
  float* sv = smem;
  float* sd = smem + rows * kColW;
  const int item = blockIdx.x;
  const NcPlane& P = planes[find_nc_plane<true>(planes, nplanes, item)];
  const int local = item - P.cbegin;
  const int per_field = P.ccount >> 1;
  const int field = local >= per_field ? 1 : 0;
  const int tile = local - field * per_field;
  const int H = P.H, W = P.W;
  const int tiles_x = (W + kColW - 1) / kColW;
  const int i0 = (tile / tiles_x) * kColRows;
  const int j0 = (tile % tiles_x) * kColW;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = threadIdx.x & (kColW - 1);
  const int j = j0 + c;
  float inv;
  const bool scaled = field_scale(P, field, &inv);
  // FP16 fields: the residual's power-of-two store scale (1 otherwise)
  float ssc = 1.0f;
  if (LAST) {
    const float2 fsc = field_store_scales(P.fmm);
    ssc = field ? fsc.y : fsc.x;
  }
  const float* __restrict__ g = P.g ? P.g : P.f;
  const int64_t gp = P.g ? P.gpitch : P.pitch;
  const float* __restrict__ in = P.buf[src][field];
  if (j < W) {
    // four staged rows per thread and round: all loads of a round are issued
    // before its LDS stores
    for (int tb = threadIdx.x / kColW; tb < rows; tb += 4 * kRowsPerLoad) {
      float fv[4], dv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = tb + kRowsPerLoad * u;
        const int m = i0 - R + t;
        fv[u] = 0.0f;
        dv[u] = 0.0f;
        if (t < rows && m >= 0 && m < H) {
          fv[u] = load_global(in, static_cast<int64_t>(m) * W + j);
          if (m >= 1)
            dv[u] = dt_increment(grad_at(g, gp, H, W, m, j, field), grad_at(g, gp, H, W, m - 1, j, field), P.a, inv,
                                 scaled);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = tb + kRowsPerLoad * u;
        const int m = i0 - R + t;
        if (t < rows && m >= 0 && m < H) {
          sv[t * kColW + c] = fv[u];
          if (m >= 1) sd[t * kColW + c] = dv[u];
        }
      }
    }
  }
  __syncthreads();
  if (j < W) {
    const int rbase = wave * (kColRows / 4) + (lane / kColW) * (kColRows / 8);
    for (int rr = 0; rr < kColRows / 8; ++rr) {
      const int i = i0 + rbase + rr;
      if (i >= H) break;
      const float out = nc_window_mean(sv + c, sd + c, kColW, i - i0 + R, min(R, H - 1 - i), min(R, i), r);
      const int64_t o = static_cast<int64_t>(i) * W + j;
      if (LAST) {
        const float res = out - grad_at(P.f, P.pitch, H, W, i, j, field);
        store_field(field ? P.ry : P.rx, o, res * ssc, field_type);
      } else {
        store_global(P.buf[src ^ 1][field], o, out);
      }
    }
  }
}

int nc_row_items(int H, int W) { return 2 * ((H + kRowWaves - 1) / kRowWaves) * ((W + kRowSeg - 1) / kRowSeg); }
int nc_col_items(int H, int W) { return 2 * ((H + kColRows - 1) / kColRows) * ((W + kColW - 1) / kColW); }

hipError_t nc_init_kernels() {
  // column passes stage up to 2 x 96 x 32 floats (24 KiB) of dynamic LDS
  const int kMax = 2 * (kColRows + 2 * kNcMaxR) * kColW * static_cast<int>(sizeof(float));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&nc_cols_kernel<true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kMax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&nc_cols_kernel<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMax);
  return e;
}

hipError_t launch_nc_pass(const NcPlane* planes, int nplanes, int items, int pass, int npasses, float r, int R,
                          int field_type, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  if (R < 0 || R > kNcMaxR) return hipErrorInvalidValue;
  const int src = pass & 1;
  if ((pass & 1) == 0) {
    if (pass == 0)
      hipLaunchKernelGGL(nc_rows_kernel<true>, dim3(items), dim3(256), 0, s, planes, nplanes, src, r, R);
    else
      hipLaunchKernelGGL(nc_rows_kernel<false>, dim3(items), dim3(256), 0, s, planes, nplanes, src, r, R);
  } else {
    const size_t lds = static_cast<size_t>(2) * (kColRows + 2 * R) * kColW * sizeof(float);
    if (pass == npasses - 1)
      hipLaunchKernelGGL(nc_cols_kernel<true>, dim3(items), dim3(256), lds, s, planes, nplanes, src, r, R,
                         field_type);
    else
      hipLaunchKernelGGL(nc_cols_kernel<false>, dim3(items), dim3(256), lds, s, planes, nplanes, src, r, R,
                         field_type);
  }
  return hipGetLastError();
}

}  // namespace blfls
