// Fourier-domain least-squares solve of Eq. (8), in residual form, for gfx950.
//
// Eq. (8)'s numerator F(f) + lam sum_* conj(F(d_*)) F(g_*) equals
// F(f) (1 + lam sum_* |F(d_*)|^2) + lam sum_* conj(F(d_*)) F(r_*) with
// r_* = g_* - D_* f, and conj(F(d_*)) F(v) is the transform of the adjoint
// D_*^T v.  Hence u = f + delta with
//     delta = F^-1( F(c) / (1 + lam (4 sin^2(pi kx/W) + 4 sin^2(pi ky/H))) ),
//     c = lam (D_x^T r_x + D_y^T r_y),   (D_x^T v)(i,j) = v(i,j-1) - v(i,j),
// where F(1) = 1 (the transform of the delta, Section II-C) and
// |exp(2 pi i k/N) - 1|^2 = 4 sin^2(pi k/N).  One forward and one inverse 2-D
// real transform per channel, in three passes over HBM:
//   rows_fwd : form c from r_x, r_y (rows i and i-1), real-to-complex FFT of
//              each row (a complex FFT of W/2 plus a split step), store the
//              half spectrum transposed, [W/2+1][H];
//   cols     : per spectrum column: forward FFT over H, multiply by
//              1/(H W den), inverse FFT over H, all in LDS (one read, one write);
//   rows_inv : complex-to-real inverse of each row, u = f + delta.
// Transforms are in-place Stockham passes in LDS with radices 2, 3, 4, 5;
// twiddles come from FP64 host tables rounded to FP32.
#include "blfls_internal.h"
#include "blfls_launch.h"

namespace blfls {

namespace {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by i*sg (sg = +-1)
__device__ __forceinline__ float2 cmul_isg(float2 a, float sg) { return make_float2(-sg * a.y, sg * a.x); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// DFT of R points, A_k = sum_t a_t exp(sg * 2 pi i t k / R)
template <int R>
__device__ __forceinline__ void butterfly(float2* a, float sg);

template <>
__device__ __forceinline__ void butterfly<2>(float2* a, float) {
  const float2 t = a[1];
  a[1] = csub(a[0], t);
  a[0] = cadd(a[0], t);
}

template <>
__device__ __forceinline__ void butterfly<3>(float2* a, float sg) {
  constexpr float kS3 = 0.86602540378443864676f;  // sin(2 pi/3)
  const float2 t1 = cadd(a[1], a[2]);
  const float2 b = make_float2(fmaf(-0.5f, t1.x, a[0].x), fmaf(-0.5f, t1.y, a[0].y));
  const float2 m = cscale(csub(a[1], a[2]), kS3);
  a[0] = cadd(a[0], t1);
  const float2 im = cmul_isg(m, sg);
  a[1] = cadd(b, im);
  a[2] = csub(b, im);
}

template <>
__device__ __forceinline__ void butterfly<4>(float2* a, float sg) {
  const float2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
  const float2 s13 = cadd(a[1], a[3]), d13 = cmul_isg(csub(a[1], a[3]), sg);
  a[0] = cadd(s02, s13);
  a[2] = csub(s02, s13);
  a[1] = cadd(d02, d13);
  a[3] = csub(d02, d13);
}

template <>
__device__ __forceinline__ void butterfly<5>(float2* a, float sg) {
  constexpr float c1 = 0.30901699437494742410f;   // cos(2 pi/5)
  constexpr float c2 = -0.80901699437494742410f;  // cos(4 pi/5)
  constexpr float s1 = 0.95105651629515357212f;   // sin(2 pi/5)
  constexpr float s2 = 0.58778525229247312917f;   // sin(4 pi/5)
  const float2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
  const float2 t3 = csub(a[1], a[4]), t4 = csub(a[2], a[3]);
  const float2 b1 = make_float2(a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y);
  const float2 b2 = make_float2(a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y);
  const float2 m1 = cmul_isg(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y), sg);
  const float2 m2 = cmul_isg(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y), sg);
  a[0] = cadd(a[0], cadd(t1, t2));
  a[1] = cadd(b1, m1);
  a[4] = csub(b1, m1);
  a[2] = cadd(b2, m2);
  a[3] = csub(b2, m2);
}

// One in-place Stockham stage over `batch` transforms of length N at
// buf[b * stride + n].  Input element j + t*N/R of a transform, output element
// (j - k) * R + k + t * Ns with k = j mod Ns (decimation in time).  All inputs
// are read into registers before the barrier, so the update is in place.
template <int R>
__device__ void fft_stage(float2* buf, int stride, int batch, int N, int Ns, const float2* __restrict__ tw,
                          float sg) {
  constexpr int kMaxB = (kFftLdsComplex / R + kFftThreads - 1) / kFftThreads;
  const int per = N / R;
  const int total = per * batch;
  float2 a[kMaxB][R];
  int base[kMaxB], jj[kMaxB];
#pragma unroll
  for (int m = 0; m < kMaxB; ++m) {
    const int gidx = threadIdx.x + m * kFftThreads;
    if (gidx < total) {
      const int b = gidx / per;
      const int j = gidx - b * per;
      base[m] = b * stride;
      jj[m] = j;
#pragma unroll
      for (int t = 0; t < R; ++t) a[m][t] = buf[base[m] + j + t * per];
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kMaxB; ++m) {
    const int gidx = threadIdx.x + m * kFftThreads;
    if (gidx < total) {
      const int j = jj[m];
      const int k = j % Ns;
      if (Ns > 1) {
        const float2* w = tw + k * (R - 1);
#pragma unroll
        for (int t = 1; t < R; ++t) {
          // the table holds exp(-2 pi i t k/(Ns R)); the inverse takes its conjugate
          float2 wt = w[t - 1];
          if (sg > 0.0f) wt.y = -wt.y;
          a[m][t] = cmul(a[m][t], wt);
        }
      }
      butterfly<R>(a[m], sg);
      const int o = base[m] + (j - k) * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) buf[o + t * Ns] = a[m][t];
    }
  }
  __syncthreads();
}

// Full transform: forward (sg = -1) or inverse without scaling (sg = +1).
__device__ void lds_fft(float2* buf, int stride, int batch, const FftSize& sz, const float2* __restrict__ tw,
                        float sg) {
  const int N = sz.n;
  for (int s = 0; s < sz.nstages; ++s) {
    const int R = sz.radix[s];
    const int Ns = sz.ns[s];
    const float2* w = tw + sz.tw_off[s];
    switch (R) {
      case 2: fft_stage<2>(buf, stride, batch, N, Ns, w, sg); break;
      case 3: fft_stage<3>(buf, stride, batch, N, Ns, w, sg); break;
      case 4: fft_stage<4>(buf, stride, batch, N, Ns, w, sg); break;
      default: fft_stage<5>(buf, stride, batch, N, Ns, w, sg); break;
    }
  }
}

__device__ __forceinline__ float load_field(const void* base, int64_t idx, int ft) {
  if (ft == kF32) return static_cast<const float*>(base)[idx];
  if (ft == kBF16) {
    const uint32_t b = static_cast<uint32_t>(static_cast<const uint16_t*>(base)[idx]) << 16;
    return __uint_as_float(b);
  }
  return static_cast<float>(static_cast<const _Float16*>(base)[idx]);
}

template <bool COLS>
__device__ __forceinline__ int find_fft_plane(const FftPlane* planes, int nplanes, int item) {
  int lo = 0, hi = nplanes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int begin = COLS ? planes[mid].col_begin : planes[mid].row_begin;
    if (begin <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace

// ---------------------------------------------------------------------------
// Pass 1: c = lam (D_x^T r_x + D_y^T r_y), real FFT of each row, transposed store
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kFftThreads)
fft_rows_fwd_kernel(const FftPlane* __restrict__ planes, int nplanes, int field_type) {
  extern __shared__ float2 buf[];
  const int item = blockIdx.x;
  const FftPlane& P = planes[find_fft_plane<false>(planes, nplanes, item)];
  const int blk = item - P.row_begin;
  if (blk >= P.row_count) return;
  const int H = P.H, W = P.W, M = W >> 1;
  const int i0 = blk * P.rb;
  const int nrows = min(P.rb, H - i0);
  const float lam = P.lambda;
  const int tid = threadIdx.x;

  for (int idx = tid; idx < nrows * M; idx += kFftThreads) {
    const int row = idx / M;
    const int n = idx - row * M;
    const int i = i0 + row;
    const int im1 = i == 0 ? H - 1 : i - 1;
    const int j0 = 2 * n, j1 = j0 + 1;
    const int jm = j0 == 0 ? W - 1 : j0 - 1;
    const int64_t ri = static_cast<int64_t>(i) * W;
    const int64_t rim1 = static_cast<int64_t>(im1) * W;
    const float xm = load_field(P.rx, ri + jm, field_type);
    const float x0 = load_field(P.rx, ri + j0, field_type);
    const float x1 = load_field(P.rx, ri + j1, field_type);
    const float y0m = load_field(P.ry, rim1 + j0, field_type);
    const float y1m = load_field(P.ry, rim1 + j1, field_type);
    const float y0 = load_field(P.ry, ri + j0, field_type);
    const float y1 = load_field(P.ry, ri + j1, field_type);
    const float c0 = lam * ((xm - x0) + (y0m - y0));
    const float c1 = lam * ((x0 - x1) + (y1m - y1));
    buf[row * M + n] = make_float2(c0, c1);
  }
  __syncthreads();
  lds_fft(buf, M, nrows, *P.szM, P.twM, -1.0f);

  // split step: X[k] = E[k] + exp(-2 pi i k/W) O[k], k = 0..M, Z[M] = Z[0]
  float2* spec = P.spec;
  for (int idx = tid; idx < (M + 1) * nrows; idx += kFftThreads) {
    const int k = idx / nrows;
    const int row = idx - k * nrows;
    const float2 zk = buf[row * M + (k == M ? 0 : k)];
    const float2 zm = buf[row * M + (k == 0 ? 0 : M - k)];
    const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    // o = (zk - conj(zm)) / (2i)
    const float2 o = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
    const float2 x = cadd(e, cmul(P.twW[k], o));
    spec[static_cast<int64_t>(k) * H + i0 + row] = x;
  }
}

// ---------------------------------------------------------------------------
// Pass 2: per spectrum column, forward FFT over H, divide, inverse FFT over H
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kFftThreads)
fft_cols_kernel(const FftPlane* __restrict__ planes, int nplanes) {
  extern __shared__ float2 buf[];
  const int item = blockIdx.x;
  const FftPlane& P = planes[find_fft_plane<true>(planes, nplanes, item)];
  const int blk = item - P.col_begin;
  if (blk >= P.col_count) return;
  const int H = P.H, W = P.W, M = W >> 1;
  const int k0 = blk * P.cb;
  const int ncols = min(P.cb, M + 1 - k0);
  const int tid = threadIdx.x;
  float2* spec = P.spec + static_cast<int64_t>(k0) * H;

  for (int idx = tid; idx < ncols * H; idx += kFftThreads) buf[idx] = spec[idx];
  __syncthreads();
  lds_fft(buf, H, ncols, *P.szH, P.twH, -1.0f);
  const float lam = P.lambda;
  const float inv_hw = 1.0f / (static_cast<float>(H) * static_cast<float>(W));
  for (int idx = tid; idx < ncols * H; idx += kFftThreads) {
    const int col = idx / H;
    const int ky = idx - col * H;
    const float den = fmaf(lam, P.sx[k0 + col] + P.sy[ky], 1.0f);
    const float s = inv_hw / den;
    buf[idx] = cscale(buf[idx], s);
  }
  __syncthreads();
  lds_fft(buf, H, ncols, *P.szH, P.twH, 1.0f);
  for (int idx = tid; idx < ncols * H; idx += kFftThreads) spec[idx] = buf[idx];
}

// ---------------------------------------------------------------------------
// Pass 3: complex-to-real inverse of each row, u = f + delta
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kFftThreads)
fft_rows_inv_kernel(const FftPlane* __restrict__ planes, int nplanes) {
  extern __shared__ float2 buf[];
  const int item = blockIdx.x;
  const FftPlane& P = planes[find_fft_plane<false>(planes, nplanes, item)];
  const int blk = item - P.row_begin;
  if (blk >= P.row_count) return;
  const int H = P.H, W = P.W, M = W >> 1;
  const int S = M + 1;  // LDS row stride
  const int i0 = blk * P.rb;
  const int nrows = min(P.rb, H - i0);
  const int tid = threadIdx.x;
  const float2* spec = P.spec;

  for (int idx = tid; idx < S * nrows; idx += kFftThreads) {
    const int k = idx / nrows;
    const int row = idx - k * nrows;
    buf[row * S + k] = spec[static_cast<int64_t>(k) * H + i0 + row];
  }
  __syncthreads();
  // Z[k] = (X[k] + conj X[M-k]) + i exp(2 pi i k/W) (X[k] - conj X[M-k]), k = 0..M-1;
  // one thread forms the pair (k, M-k) so the update is in place
  const int half = M / 2;
  for (int idx = tid; idx < (half + 1) * nrows; idx += kFftThreads) {
    const int k = idx / nrows;
    const int row = idx - k * nrows;
    float2* X = buf + row * S;
    const float2 a = X[k], b = X[M - k];
    const float2 wa = cconj(P.twW[k]);       // exp(+2 pi i k/W)
    const float2 wb = cconj(P.twW[M - k]);
    // Z[k]
    const float2 sa = cadd(a, cconj(b)), da = csub(a, cconj(b));
    const float2 za = cadd(sa, cmul_isg(cmul(wa, da), 1.0f));
    // Z[M-k]
    const float2 sb = cadd(b, cconj(a)), db = csub(b, cconj(a));
    const float2 zb = cadd(sb, cmul_isg(cmul(wb, db), 1.0f));
    X[k] = za;
    if (k != 0 && M - k != k) X[M - k] = zb;
  }
  __syncthreads();
  lds_fft(buf, S, nrows, *P.szM, P.twM, 1.0f);
  const float* f = P.f;
  float* u = P.u;
  const int64_t pitch = P.pitch;
  for (int idx = tid; idx < nrows * M; idx += kFftThreads) {
    const int row = idx / M;
    const int n = idx - row * M;
    const int64_t o = static_cast<int64_t>(i0 + row) * pitch + 2 * n;
    const float2 z = buf[row * S + n];
    u[o] = f[o] + z.x;
    u[o + 1] = f[o + 1] + z.y;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_fft_rows_fwd(const FftPlane* planes, int nplanes, int blocks, size_t lds_bytes,
                               int field_type, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(fft_rows_fwd_kernel, dim3(blocks), dim3(kFftThreads), lds_bytes, s, planes, nplanes,
                     field_type);
  return hipGetLastError();
}

hipError_t launch_fft_cols(const FftPlane* planes, int nplanes, int blocks, size_t lds_bytes, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(fft_cols_kernel, dim3(blocks), dim3(kFftThreads), lds_bytes, s, planes, nplanes);
  return hipGetLastError();
}

hipError_t launch_fft_rows_inv(const FftPlane* planes, int nplanes, int blocks, size_t lds_bytes,
                               hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(fft_rows_inv_kernel, dim3(blocks), dim3(kFftThreads), lds_bytes, s, planes, nplanes);
  return hipGetLastError();
}

}  // namespace blfls
