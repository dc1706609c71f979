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
//
// Every pass is a persistent loop over small work items (a few rows or
// columns, about 2048 complex values): while an item's transform runs in LDS,
// the loads of the workgroup's next item are already in flight into
// registers, so HBM sees a steady stream instead of load/compute/store
// phases.  Transforms are Stockham passes with radices 2, 3, 4, 5, 8, 9, 15
// and 16 (three stages for the usual lengths); twiddles come from two-level
// tables (built in FP64, rounded once; about 1 KiB) kept in LDS for the
// workgroup's lifetime, so nearly all LDS holds data; LDS is padded so that
// every stage after the first addresses its legs linearly.  Work items are
// handed out in contiguous ranges per XCD, so neighbouring rows meet in one
// L2 where the transposed spectrum is written and read.
#include <algorithm>

#include "blfls_internal.h"
#include "blfls_launch.h"
#include "blfls_work.h"

namespace blfls {

namespace {

constexpr int T = kFftThreads;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by i*sg (sg = +-1)
__device__ __forceinline__ float2 cmul_isg(float2 a, float sg) { return make_float2(-sg * a.y, sg * a.x); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv d) {
  return (__umulhi(n, d.mul) + n) >> d.shift;
}

// W_N^e from a two-level table in LDS (lo: W_N^j, j < 64; hi: W_N^(64 j)).
__device__ __forceinline__ float2 twiddle2(const float2* tab, int e) {
  return cmul(tab[kTwLo + (e >> 6)], tab[e & (kTwLo - 1)]);
}

// ---------------------------------------------------------------------------
// Butterflies: DFT of R points, A_k = sum_t a_t exp(sg * 2 pi i t k / R)
// ---------------------------------------------------------------------------
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

// Radix 8 as 2 x 4: with t = t1 + 4 t2 and k = 2 k1 + k2,
// A_{2k1+k2} = sum_{t1} w4^{t1 k1} [ w8^{t1 k2} (a_{t1} + (-1)^{k2} a_{t1+4}) ].
template <>
__device__ __forceinline__ void butterfly<8>(float2* a, float sg) {
  constexpr float kH = 0.70710678118654752440f;  // 1/sqrt(2)
  float2 e[4], o[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    e[t] = cadd(a[t], a[t + 4]);
    o[t] = csub(a[t], a[t + 4]);
  }
  // o[t] *= w8^t, w8 = (1 + i sg)/sqrt(2)
  o[1] = cscale(cadd(o[1], cmul_isg(o[1], sg)), kH);
  o[2] = cmul_isg(o[2], sg);
  o[3] = cscale(csub(cmul_isg(o[3], sg), o[3]), kH);
  butterfly<4>(e, sg);
  butterfly<4>(o, sg);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    a[2 * k1] = e[k1];
    a[2 * k1 + 1] = o[k1];
  }
}

// Radix 16 as 4 x 4: with t = t1 + 4 t2 and k = 4 k1 + k2,
// A_{4k1+k2} = sum_{t1} w4^{t1 k1} [ w16^{t1 k2} sum_{t2} a_{t1+4t2} w4^{t2 k2} ].
template <>
__device__ __forceinline__ void butterfly<16>(float2* a, float sg) {
  // cos and sin of 2 pi m / 16, m = 0..3
  constexpr float kC[4] = {1.0f, 0.92387953251128675613f, 0.70710678118654752440f, 0.38268343236508977173f};
  constexpr float kS[4] = {0.0f, 0.38268343236508977173f, 0.70710678118654752440f, 0.92387953251128675613f};
  float2 b[4][4];
#pragma unroll
  for (int t1 = 0; t1 < 4; ++t1) {
    float2 c[4] = {a[t1], a[t1 + 4], a[t1 + 8], a[t1 + 12]};
    butterfly<4>(c, sg);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      const int m = t1 * k2;  // w16^m, m <= 9
      float2 w;
      if (m < 4) w = make_float2(kC[m], sg * kS[m]);
      else if (m < 8) w = make_float2(-kS[m - 4], sg * kC[m - 4]);  // exp(i (pi/2 + x))
      else w = make_float2(-kC[m - 8], -sg * kS[m - 8]);           // exp(i (pi + x))
      b[k2][t1] = m == 0 ? c[k2] : cmul(c[k2], w);
    }
  }
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    butterfly<4>(b[k2], sg);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) a[4 * k1 + k2] = b[k2][k1];
  }
}

// Radix 9 as 3 x 3: with t = t1 + 3 t2 and k = 3 k1 + k2,
// A_{3k1+k2} = sum_{t1} w3^{t1 k1} [ w9^{t1 k2} sum_{t2} a_{t1+3t2} w3^{t2 k2} ].
template <>
__device__ __forceinline__ void butterfly<9>(float2* a, float sg) {
  // cos and sin of 2 pi m / 9 for m = 1, 2, 4
  constexpr float c1 = 0.76604444311897803520f, s1 = 0.64278760968653932632f;
  constexpr float c2 = 0.17364817766693034885f, s2 = 0.98480775301220805936f;
  constexpr float c4 = -0.93969262078590838405f, s4 = 0.34202014332566873304f;
  float2 b[3][3];
#pragma unroll
  for (int t1 = 0; t1 < 3; ++t1) {
    float2 c[3] = {a[t1], a[t1 + 3], a[t1 + 6]};
    butterfly<3>(c, sg);
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2) {
      const int m = t1 * k2;  // 0, 1, 2 or 4
      float2 w = make_float2(1.0f, 0.0f);
      if (m == 1) w = make_float2(c1, sg * s1);
      else if (m == 2) w = make_float2(c2, sg * s2);
      else if (m == 4) w = make_float2(c4, sg * s4);
      b[k2][t1] = m == 0 ? c[k2] : cmul(c[k2], w);
    }
  }
#pragma unroll
  for (int k2 = 0; k2 < 3; ++k2) {
    butterfly<3>(b[k2], sg);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) a[3 * k1 + k2] = b[k2][k1];
  }
}

// Radix 15 as 3 x 5 without twiddles (Good-Thomas, 3 and 5 coprime): input
// n = (5 n1 + 3 n2) mod 15, output k = (10 k1 + 6 k2) mod 15 (10 = 5 (5^-1 mod 3),
// 6 = 3 (3^-1 mod 5)), so W_15^(n k) = W_3^(n1 k1) W_5^(n2 k2).
template <>
__device__ __forceinline__ void butterfly<15>(float2* a, float sg) {
  float2 y[5][3];
#pragma unroll
  for (int n2 = 0; n2 < 5; ++n2) {
    float2 c[3];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) c[n1] = a[(5 * n1 + 3 * n2) % 15];
    butterfly<3>(c, sg);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) y[n2][k1] = c[k1];
  }
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    float2 d[5];
#pragma unroll
    for (int n2 = 0; n2 < 5; ++n2) d[n2] = y[n2][k1];
    butterfly<5>(d, sg);
#pragma unroll
    for (int k2 = 0; k2 < 5; ++k2) a[(10 * k1 + 6 * k2) % 15] = d[k2];
  }
}

// ---------------------------------------------------------------------------
// Padded LDS batches and stage destinations
// ---------------------------------------------------------------------------
struct Lds {
  float2* buf;
  int stride;  // complex values per transform (multiple of 16)
  int pshift;  // one spare slot per 2^pshift values (31: none)
  __device__ __forceinline__ int pad(int i) const { return i + (i >> pshift); }
};

// Output legs n0 + t ns of transform b.  put() stores all R legs of one
// butterfly; put1() one value (length-1 transforms).
struct LdsOut {
  static constexpr bool kLds = true;
  Lds l;
  template <int R>
  __device__ __forceinline__ void put(int b, int n0, const FftStage& S, const float2* v) const {
    float2* p = l.buf + l.pad(b * l.stride + n0);
#pragma unroll
    for (int t = 0; t < R; ++t) p[t * S.pout] = v[t];
  }
  __device__ __forceinline__ void put1(int b, int n, float2 v) const { l.buf[l.pad(b * l.stride + n)] = v; }
};

// LDS destination that applies the Eq. (8) divide, 1 / (H W (1 + lam (sx + sy))),
// with sy and the item's sx values staged in LDS (no global access while the
// next item's loads are in flight).
struct ScaledLds {
  static constexpr bool kLds = true;
  Lds l;
  const float* sy;   // LDS, [H]
  const float* sx;   // LDS, [cb]: sx of columns k0 + b
  float lam, inv_hw;
  __device__ __forceinline__ float scale(int b, int n) const {
    const float den = fmaf(lam, sx[b] + sy[n], 1.0f);
    return inv_hw * __builtin_amdgcn_rcpf(den);
  }
  template <int R>
  __device__ __forceinline__ void put(int b, int n0, const FftStage& S, const float2* v) const {
    float2* p = l.buf + l.pad(b * l.stride + n0);
    const float sxb = sx[b];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const float den = fmaf(lam, sxb + sy[n0 + t * S.ns], 1.0f);
      p[t * S.pout] = cscale(v[t], inv_hw * __builtin_amdgcn_rcpf(den));
    }
  }
  __device__ __forceinline__ void put1(int b, int n, float2 v) const {
    l.buf[l.pad(b * l.stride + n)] = cscale(v, scale(b, n));
  }
};

// Spectrum columns k0 + b in HBM ([W/2+1][H] layout).
struct ColOut {
  static constexpr bool kLds = false;
  float2* spec;  // column k0
  int H;
  template <int R>
  __device__ __forceinline__ void put(int b, int n0, const FftStage& S, const float2* v) const {
    float2* q = spec + static_cast<int64_t>(b) * H + n0;
#pragma unroll
    for (int t = 0; t < R; ++t) q[t * S.ns] = v[t];
  }
  __device__ __forceinline__ void put1(int b, int n, float2 v) const { spec[static_cast<int64_t>(b) * H + n] = v; }
};

// u = f + delta for row i0 + b; complex value n holds the reals at columns 2n, 2n+1.
struct RowOut {
  static constexpr bool kLds = false;
  const float* __restrict__ f;
  float* __restrict__ u;
  int64_t pitch;
  int i0;
  __device__ __forceinline__ void put1(int b, int n, float2 v) const {
    const int64_t o = static_cast<int64_t>(i0 + b) * pitch + 2 * n;
    u[o] = f[o] + v.x;
    u[o + 1] = f[o + 1] + v.y;
  }
  template <int R>
  __device__ __forceinline__ void put(int b, int n0, const FftStage& S, const float2* v) const {
#pragma unroll
    for (int t = 0; t < R; ++t) put1(b, n0 + t * S.ns, v[t]);
  }
};

// ---------------------------------------------------------------------------
// Stockham stages
// ---------------------------------------------------------------------------

// One stage over `batch` transforms held in `in`: input legs j + t per of
// butterfly j, output legs (j - k) R + k + t ns with k = j mod ns (decimation
// in time), twiddles W_N^(t k es) from the transform's two-level table `tw` in
// LDS (forward) or their conjugates (inverse).  The first stage (ns = 1, no twiddles) reads
// with the general padded index; later stages read their legs at a fixed
// padded stride.  Inputs are read into registers before a barrier, so an
// LDS destination may be the same buffer; a barrier follows any LDS write.
template <int R, bool FWD, bool FIRST, class DST>
__device__ __forceinline__ void fft_stage(const Lds& in, const DST& dst, int batch, const FftStage& S,
                                          const float2* tw) {
  constexpr int kMaxB = (kFftItemMax / R + T - 1) / T;
  constexpr float sg = FWD ? -1.0f : 1.0f;
  const int per = S.per;
  const int Ns = S.ns;
  const int total = per * batch;
  float2 a[kMaxB][R];
  int ob[kMaxB], on[kMaxB];
#pragma unroll
  for (int m = 0; m < kMaxB; ++m) {
    const int g = threadIdx.x + m * T;
    if (g < total) {
      const int b = static_cast<int>(fdiv(static_cast<uint32_t>(g), S.per_div));
      const int j = g - b * per;
      if (FIRST) {
#pragma unroll
        for (int t = 0; t < R; ++t) a[m][t] = in.buf[in.pad(b * in.stride + j + t * per)];
        ob[m] = b;
        on[m] = j * R;
      } else {
        const float2* p = in.buf + in.pad(b * in.stride + j);
#pragma unroll
        for (int t = 0; t < R; ++t) a[m][t] = p[t * S.pin];
        const int k = j - static_cast<int>(fdiv(static_cast<uint32_t>(j), S.ns_div)) * Ns;
        ob[m] = b;
        on[m] = (j - k) * R + k;
        const int ek = k * S.es;
#pragma unroll
        for (int t = 1; t < R; ++t) {
          const float2 w = twiddle2(tw, t * ek);
          a[m][t] = FWD ? cmul(a[m][t], w) : cmulc(a[m][t], w);
        }
      }
    }
  }
  if (DST::kLds) __syncthreads();
#pragma unroll
  for (int m = 0; m < kMaxB; ++m) {
    const int g = threadIdx.x + m * T;
    if (g < total) {
      butterfly<R>(a[m], sg);
      dst.template put<R>(ob[m], on[m], S, a[m]);
    }
  }
  if (DST::kLds) __syncthreads();
}

template <bool FWD, bool FIRST, class DST>
__device__ __forceinline__ void fft_stage_r(const Lds& in, const DST& dst, int batch, const FftStage& S,
                                            const float2* tw) {
  switch (S.radix) {
    case 2: fft_stage<2, FWD, FIRST>(in, dst, batch, S, tw); break;
    case 3: fft_stage<3, FWD, FIRST>(in, dst, batch, S, tw); break;
    case 4: fft_stage<4, FWD, FIRST>(in, dst, batch, S, tw); break;
    case 5: fft_stage<5, FWD, FIRST>(in, dst, batch, S, tw); break;
    case 8: fft_stage<8, FWD, FIRST>(in, dst, batch, S, tw); break;
    case 9: fft_stage<9, FWD, FIRST>(in, dst, batch, S, tw); break;
    case 15: fft_stage<15, FWD, FIRST>(in, dst, batch, S, tw); break;
    default: fft_stage<16, FWD, FIRST>(in, dst, batch, S, tw); break;
  }
}

// Whole transform of the batch in `l`, forward or inverse without scaling; the
// last stage writes `dst`, the others work in place.  Length 1 copies.
template <bool FWD, class DST>
__device__ __forceinline__ void fft_run(const FftSize& sz, const float2* tw, int batch, const Lds& l,
                                        const DST& dst) {
  const int n = sz.nstages;
  if (n == 0) {
    for (int b = threadIdx.x; b < batch; b += T) dst.put1(b, 0, l.buf[l.pad(b * l.stride)]);
    if (DST::kLds) __syncthreads();
    return;
  }
  if (n == 1) {
    fft_stage_r<FWD, true>(l, dst, batch, sz.st[0], tw);
    return;
  }
  const LdsOut mid{l};
  fft_stage_r<FWD, true>(l, mid, batch, sz.st[0], tw);
  for (int s = 1; s < n - 1; ++s) fft_stage_r<FWD, false>(l, mid, batch, sz.st[s], tw);
  fft_stage_r<FWD, false>(l, dst, batch, sz.st[n - 1], tw);
}

// ---------------------------------------------------------------------------
// Work-item sequences of a persistent workgroup
// ---------------------------------------------------------------------------

// Static: the items are split into 8 contiguous ranges, one per XCD
// (workgroup b runs on XCD b mod 8); the workgroups of an XCD take its range
// round-robin.  Every range with items has a workgroup when grid >= min(8, total).
struct StaticItems {
  int pos, end, step, total;
  __device__ __forceinline__ int first(int n) {
    total = n;
    const int x = static_cast<int>(blockIdx.x % kXcds);
    const int s = static_cast<int>(blockIdx.x / kXcds);
    const int q = n / kXcds, rem = n % kXcds;
    const int start = x * q + min(x, rem);
    end = start + q + (x < rem ? 1 : 0);
    step = (static_cast<int>(gridDim.x) - x + kXcds - 1) / kXcds;
    pos = start + s;
    return pos < end ? pos : total;
  }
  __device__ __forceinline__ int next() {
    pos += step;
    return pos < end ? pos : total;
  }
};

// Dynamic: per-XCD counters of the work header (zero when the header is uploaded).
struct CounterItems {
  int* counters;
  int total;
  __device__ __forceinline__ int first(int n) {
    total = n;
    return grab_item(counters, n, true);
  }
  __device__ __forceinline__ int next() { return grab_item(counters, total, true); }
};

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

template <class E>
__device__ __forceinline__ void copy_to_lds(E* dst, const E* __restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += T) dst[i] = src[i];
}

// Two consecutive field values at an even index, as one word (16-bit fields)
// or two floats.
template <int FT>
struct FieldPair {
  using type = uint32_t;
  __device__ __forceinline__ static type load(const void* base, int64_t idx) {
    return *reinterpret_cast<const uint32_t*>(static_cast<const uint16_t*>(base) + idx);
  }
  __device__ __forceinline__ static float lo(type w) {
    if (FT == kBF16) return __uint_as_float(w << 16);
    _Float16 h;
    const uint16_t v = static_cast<uint16_t>(w & 0xFFFFu);
    __builtin_memcpy(&h, &v, 2);
    return static_cast<float>(h);
  }
  __device__ __forceinline__ static float hi(type w) {
    if (FT == kBF16) return __uint_as_float(w & 0xFFFF0000u);
    _Float16 h;
    const uint16_t v = static_cast<uint16_t>(w >> 16);
    __builtin_memcpy(&h, &v, 2);
    return static_cast<float>(h);
  }
  using one = uint32_t;
  __device__ __forceinline__ static one load1(const void* base, int64_t idx) {
    return static_cast<const uint16_t*>(base)[idx];
  }
  __device__ __forceinline__ static float val1(one w) { return lo(w); }
};

template <>
struct FieldPair<kF32> {
  using type = float2;
  __device__ __forceinline__ static type load(const void* base, int64_t idx) {
    return *reinterpret_cast<const float2*>(static_cast<const float*>(base) + idx);
  }
  __device__ __forceinline__ static float lo(type w) { return w.x; }
  __device__ __forceinline__ static float hi(type w) { return w.y; }
  using one = float;
  __device__ __forceinline__ static one load1(const void* base, int64_t idx) {
    return static_cast<const float*>(base)[idx];
  }
  __device__ __forceinline__ static float val1(one w) { return w; }
};

// Prefetch slots per thread: items up to T * kPre complex values stream
// through registers (the row pass's residual inputs: T * kPre / 2); larger
// items load their remainder when committed.
constexpr int kPre = 8;

}  // namespace

// ---------------------------------------------------------------------------
// Pass 1: c = lam (D_x^T r_x + D_y^T r_y), real FFT of each row, transposed store
// ---------------------------------------------------------------------------
template <int FT>
struct RowsFwd {
  static constexpr int kRaw = kPre / 2;  // raw residual values take 7 registers per element
  using FP = FieldPair<FT>;
  typename FP::type x[kRaw], y[kRaw], yp[kRaw];
  typename FP::one xm[kRaw];

  __device__ __forceinline__ static const FftPlane& plane(const FftPlane* pl, int np, int item) {
    return pl[find_fft_plane<false>(pl, np, item)];
  }
  __device__ __forceinline__ static const void* table_key(const FftPlane& P) { return P.twM; }
  __device__ __forceinline__ static void load_tables(const FftPlane& P, float2* smem) {
    copy_to_lds(smem, P.twM, P.ntwM);
    copy_to_lds(smem + P.r_split, P.twW, P.ntwW);
  }
  // residual values of element e (row e / M, complex column e mod M) of item rows i0..
  __device__ __forceinline__ static void load_raw(const FftPlane& P, int i0, int e, typename FP::type& vx,
                                                  typename FP::type& vy, typename FP::type& vyp,
                                                  typename FP::one& vxm) {
    const int M = P.W >> 1;
    const int row = static_cast<int>(fdiv(static_cast<uint32_t>(e), P.m_div));
    const int n = e - row * M;
    const int i = i0 + row;
    const int im1 = i == 0 ? P.H - 1 : i - 1;
    const int j0 = 2 * n;
    const int jm = j0 == 0 ? P.W - 1 : j0 - 1;
    const int64_t ri = static_cast<int64_t>(i) * P.W;
    vx = FP::load(P.rx, ri + j0);
    vy = FP::load(P.ry, ri + j0);
    vyp = FP::load(P.ry, static_cast<int64_t>(im1) * P.W + j0);
    vxm = FP::load1(P.rx, ri + jm);
  }
  // c(i, j) = lam ((r_x(i, j-1) - r_x(i, j)) + (r_y(i-1, j) - r_y(i, j))) at j = 2n, 2n+1
  __device__ __forceinline__ static float2 rhs(float lam, typename FP::type vx, typename FP::type vy,
                                               typename FP::type vyp, typename FP::one vxm) {
    const float x0 = FP::lo(vx), x1 = FP::hi(vx);
    return make_float2(lam * ((FP::val1(vxm) - x0) + (FP::lo(vyp) - FP::lo(vy))),
                       lam * ((x0 - x1) + (FP::hi(vyp) - FP::hi(vy))));
  }
  __device__ __forceinline__ void prefetch(const FftPlane* pl, int np, int item) {
    const FftPlane& P = plane(pl, np, item);
    const int i0 = (item - P.row_begin) * P.rb;
    const int nel = min(P.rb, P.H - i0) * (P.W >> 1);
#pragma unroll
    for (int u = 0; u < kRaw; ++u) {
      const int e = threadIdx.x + u * T;
      if (e < nel) load_raw(P, i0, e, x[u], y[u], yp[u], xm[u]);
    }
  }
  __device__ __forceinline__ void commit(const FftPlane& P, int item, float2* smem) const {
    const int M = P.W >> 1;
    const int i0 = (item - P.row_begin) * P.rb;
    const int nel = min(P.rb, P.H - i0) * M;
    const Lds l{smem + P.r_data, P.sM, P.szM->pshift};
#pragma unroll
    for (int u = 0; u < kRaw; ++u) {
      const int e = threadIdx.x + u * T;
      if (e < nel) {
        const int row = static_cast<int>(fdiv(static_cast<uint32_t>(e), P.m_div));
        l.buf[l.pad(row * l.stride + e - row * M)] = rhs(P.lambda, x[u], y[u], yp[u], xm[u]);
      }
    }
    for (int e0 = threadIdx.x + kRaw * T; e0 < nel; e0 += kRaw * T) {
      typename FP::type vx[kRaw], vy[kRaw], vyp[kRaw];
      typename FP::one vxm[kRaw];
#pragma unroll
      for (int u = 0; u < kRaw; ++u)
        if (e0 + u * T < nel) load_raw(P, i0, e0 + u * T, vx[u], vy[u], vyp[u], vxm[u]);
#pragma unroll
      for (int u = 0; u < kRaw; ++u) {
        const int e = e0 + u * T;
        if (e < nel) {
          const int row = static_cast<int>(fdiv(static_cast<uint32_t>(e), P.m_div));
          l.buf[l.pad(row * l.stride + e - row * M)] = rhs(P.lambda, vx[u], vy[u], vyp[u], vxm[u]);
        }
      }
    }
  }
  __device__ __forceinline__ static void compute(const FftPlane& P, int item, float2* smem) {
    const int H = P.H, M = P.W >> 1;
    const int i0 = (item - P.row_begin) * P.rb;
    const int nrows = min(P.rb, H - i0);
    const Lds l{smem + P.r_data, P.sM, P.szM->pshift};
    fft_run<true>(*P.szM, smem, nrows, l, LdsOut{l});
    // split step: X[k] = E[k] + exp(-2 pi i k/W) O[k], k = 0..M, Z[M] = Z[0]
    const float2* twR = smem + P.r_split;
    float2* spec = P.spec;
    for (int idx = threadIdx.x; idx < (M + 1) * nrows; idx += T) {
      int k, row;
      if (nrows == P.rb) {
        k = static_cast<int>(fdiv(static_cast<uint32_t>(idx), P.rb_div));
        row = idx - k * nrows;
      } else {
        k = idx / nrows;
        row = idx - k * nrows;
      }
      const float2 zk = l.buf[l.pad(row * l.stride + (k == M ? 0 : k))];
      const float2 zm = l.buf[l.pad(row * l.stride + (k == 0 ? 0 : M - k))];
      const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
      // o = (zk - conj(zm)) / (2i)
      const float2 o = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
      spec[static_cast<int64_t>(k) * H + i0 + row] = cadd(e, cmul(twiddle2(twR, k), o));
    }
  }
};

// ---------------------------------------------------------------------------
// Pass 2: per spectrum column, forward FFT over H, divide, inverse FFT over H.
// ---------------------------------------------------------------------------
struct Cols {
  float2 v[kPre];

  __device__ __forceinline__ static const FftPlane& plane(const FftPlane* pl, int np, int item) {
    return pl[find_fft_plane<true>(pl, np, item)];
  }
  __device__ __forceinline__ static const void* table_key(const FftPlane& P) { return P.twH; }
  __device__ __forceinline__ static void load_tables(const FftPlane& P, float2* smem) {
    copy_to_lds(smem, P.twH, P.ntwH);
    copy_to_lds(reinterpret_cast<float*>(smem + P.c_sy), P.sy, P.H);
  }
  __device__ __forceinline__ void prefetch(const FftPlane* pl, int np, int item) {
    const FftPlane& P = plane(pl, np, item);
    const int k0 = (item - P.col_begin) * P.cb;
    const int nel = min(P.cb, (P.W >> 1) + 1 - k0) * P.H;
    const float2* src = P.spec + static_cast<int64_t>(k0) * P.H;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int e = threadIdx.x + u * T;
      if (e < nel) v[u] = src[e];
    }
  }
  __device__ __forceinline__ void commit(const FftPlane& P, int item, float2* smem) const {
    const int H = P.H;
    const int k0 = (item - P.col_begin) * P.cb;
    const int ncols = min(P.cb, (P.W >> 1) + 1 - k0);
    const int nel = ncols * H;
    const Lds l{smem + P.c_data, P.sH, P.szH->pshift};
    if (static_cast<int>(threadIdx.x) < ncols) reinterpret_cast<float*>(smem + P.c_sx)[threadIdx.x] = P.sx[k0 + threadIdx.x];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int e = threadIdx.x + u * T;
      if (e < nel) {
        const int b = static_cast<int>(fdiv(static_cast<uint32_t>(e), P.h_div));
        l.buf[l.pad(b * l.stride + e - b * H)] = v[u];
      }
    }
    const float2* src = P.spec + static_cast<int64_t>(k0) * H;
    for (int e0 = threadIdx.x + kPre * T; e0 < nel; e0 += kPre * T) {
      float2 w[kPre];
#pragma unroll
      for (int u = 0; u < kPre; ++u)
        if (e0 + u * T < nel) w[u] = src[e0 + u * T];
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int e = e0 + u * T;
        if (e < nel) {
          const int b = static_cast<int>(fdiv(static_cast<uint32_t>(e), P.h_div));
          l.buf[l.pad(b * l.stride + e - b * H)] = w[u];
        }
      }
    }
  }
  __device__ __forceinline__ static void compute(const FftPlane& P, int item, float2* smem) {
    const int H = P.H, W = P.W, M = W >> 1;
    const int k0 = (item - P.col_begin) * P.cb;
    const int ncols = min(P.cb, M + 1 - k0);
    const Lds l{smem + P.c_data, P.sH, P.szH->pshift};
    const ScaledLds scaled{l, reinterpret_cast<const float*>(smem + P.c_sy), reinterpret_cast<const float*>(smem + P.c_sx),
                           P.lambda, 1.0f / (static_cast<float>(H) * static_cast<float>(W))};
    fft_run<true>(*P.szH, smem, ncols, l, scaled);
    fft_run<false>(*P.szH, smem, ncols, l, ColOut{P.spec + static_cast<int64_t>(k0) * H, H});
  }
};

// ---------------------------------------------------------------------------
// Pass 3: complex-to-real inverse of each row, u = f + delta (written by the
// last stage of the inverse transform)
// ---------------------------------------------------------------------------
struct RowsInv {
  float2 v[kPre];

  __device__ __forceinline__ static const FftPlane& plane(const FftPlane* pl, int np, int item) {
    return pl[find_fft_plane<false>(pl, np, item)];
  }
  __device__ __forceinline__ static const void* table_key(const FftPlane& P) { return P.twM; }
  __device__ __forceinline__ static void load_tables(const FftPlane& P, float2* smem) {
    copy_to_lds(smem, P.twM, P.ntwM);
    copy_to_lds(smem + P.r_split, P.twW, P.ntwW);
  }
  // element e of the item: spectrum column k = e / nrows, row e mod nrows
  __device__ __forceinline__ static void coords(const FftPlane& P, int nrows, int e, int& k, int& row) {
    if (nrows == P.rb) {
      k = static_cast<int>(fdiv(static_cast<uint32_t>(e), P.rb_div));
    } else {
      k = e / nrows;
    }
    row = e - k * nrows;
  }
  __device__ __forceinline__ void prefetch(const FftPlane* pl, int np, int item) {
    const FftPlane& P = plane(pl, np, item);
    const int i0 = (item - P.row_begin) * P.rb;
    const int nrows = min(P.rb, P.H - i0);
    const int nel = ((P.W >> 1) + 1) * nrows;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int e = threadIdx.x + u * T;
      if (e < nel) {
        int k, row;
        coords(P, nrows, e, k, row);
        v[u] = P.spec[static_cast<int64_t>(k) * P.H + i0 + row];
      }
    }
  }
  __device__ __forceinline__ void commit(const FftPlane& P, int item, float2* smem) const {
    const int i0 = (item - P.row_begin) * P.rb;
    const int nrows = min(P.rb, P.H - i0);
    const int nel = ((P.W >> 1) + 1) * nrows;
    const Lds l{smem + P.r_data, P.sM, P.szM->pshift};
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int e = threadIdx.x + u * T;
      if (e < nel) {
        int k, row;
        coords(P, nrows, e, k, row);
        l.buf[l.pad(row * l.stride + k)] = v[u];
      }
    }
    for (int e0 = threadIdx.x + kPre * T; e0 < nel; e0 += kPre * T) {
      float2 w[kPre];
      int dst[kPre];
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int e = e0 + u * T;
        if (e < nel) {
          int k, row;
          coords(P, nrows, e, k, row);
          w[u] = P.spec[static_cast<int64_t>(k) * P.H + i0 + row];
          dst[u] = l.pad(row * l.stride + k);
        }
      }
#pragma unroll
      for (int u = 0; u < kPre; ++u)
        if (e0 + u * T < nel) l.buf[dst[u]] = w[u];
    }
  }
  __device__ __forceinline__ static void compute(const FftPlane& P, int item, float2* smem) {
    const int M = P.W >> 1;
    const int i0 = (item - P.row_begin) * P.rb;
    const int nrows = min(P.rb, P.H - i0);
    const Lds l{smem + P.r_data, P.sM, P.szM->pshift};
    const float2* twR = smem + P.r_split;
    // Z[k] = (X[k] + conj X[M-k]) + i exp(2 pi i k/W) (X[k] - conj X[M-k]), k = 0..M-1;
    // one thread forms the pair (k, M-k) so the update is in place
    const int half = M / 2;
    for (int idx = threadIdx.x; idx < (half + 1) * nrows; idx += T) {
      const int row = idx / (half + 1);
      const int k = idx - row * (half + 1);
      const int ia = l.pad(row * l.stride + k), ib = l.pad(row * l.stride + M - k);
      const float2 a = l.buf[ia], b = l.buf[ib];
      const float2 wa = cconj(twiddle2(twR, k));  // exp(+2 pi i k/W)
      const float2 wb = cconj(twiddle2(twR, M - k));
      const float2 sa = cadd(a, cconj(b)), da = csub(a, cconj(b));
      const float2 za = cadd(sa, cmul_isg(cmul(wa, da), 1.0f));
      const float2 sb = cadd(b, cconj(a)), db = csub(b, cconj(a));
      const float2 zb = cadd(sb, cmul_isg(cmul(wb, db), 1.0f));
      l.buf[ia] = za;
      if (k != 0 && M - k != k) l.buf[ib] = zb;
    }
    __syncthreads();
    fft_run<false>(*P.szM, smem, nrows, l, RowOut{P.f, P.u, P.pitch, i0});
  }
};

// ---------------------------------------------------------------------------
// Persistent driver: commit the prefetched item into LDS, start the next
// item's loads, transform the committed item.  Tables are (re)loaded when an
// item's plane uses other tables than the ones in LDS.
// ---------------------------------------------------------------------------
template <class PASS, class SEQ>
__device__ __forceinline__ void run_items(const FftPlane* __restrict__ planes, int nplanes, int total, SEQ& seq,
                                          float2* smem) {
  PASS pass;
  int item = seq.first(total);
  if (item < total) pass.prefetch(planes, nplanes, item);
  const void* loaded = nullptr;
  while (item < total) {
    const FftPlane& P = PASS::plane(planes, nplanes, item);
    const void* key = PASS::table_key(P);
    if (key != loaded) {
      PASS::load_tables(P, smem);
      loaded = key;
    }
    pass.commit(P, item, smem);
    __syncthreads();
    const int next = seq.next();
    if (next < total) pass.prefetch(planes, nplanes, next);
    PASS::compute(P, item, smem);
    __syncthreads();
    item = next;
  }
}

// With work == nullptr the launch covers `items` items of `planes` with a
// fixed grid and static ranges; otherwise (launches captured in a graph) the
// item counts and planes come from the work header in device memory and the
// items from its per-XCD counters.
template <int FT, bool DYN>
__global__ void __launch_bounds__(kFftThreads, 4)
fft_rows_fwd_kernel(const FftPlane* __restrict__ planes, int nplanes, int items, WorkHeader* __restrict__ work) {
  extern __shared__ float2 smem[];
  if (!DYN) {
    StaticItems seq;
    run_items<RowsFwd<FT>>(planes, nplanes, items, seq, smem);
  } else {
    CounterItems seq{work->next[0], 0};
    run_items<RowsFwd<FT>>(static_cast<const FftPlane*>(work->planes), work->nplanes, work->items, seq, smem);
  }
}

template <bool DYN>
__global__ void __launch_bounds__(kFftThreads, 4)
fft_cols_kernel(const FftPlane* __restrict__ planes, int nplanes, int items, WorkHeader* __restrict__ work) {
  extern __shared__ float2 smem[];
  if (!DYN) {
    StaticItems seq;
    run_items<Cols>(planes, nplanes, items, seq, smem);
  } else {
    CounterItems seq{work->next[1], 0};
    run_items<Cols>(static_cast<const FftPlane*>(work->planes), work->nplanes, work->items2, seq, smem);
  }
}

template <bool DYN>
__global__ void __launch_bounds__(kFftThreads, 4)
fft_rows_inv_kernel(const FftPlane* __restrict__ planes, int nplanes, int items, WorkHeader* __restrict__ work) {
  extern __shared__ float2 smem[];
  if (!DYN) {
    StaticItems seq;
    run_items<RowsInv>(planes, nplanes, items, seq, smem);
  } else {
    CounterItems seq{work->next[2], 0};
    run_items<RowsInv>(static_cast<const FftPlane*>(work->planes), work->nplanes, work->items, seq, smem);
  }
}

// ---------------------------------------------------------------------------
// Host side: LDS sizes, kernel attributes, occupancy, launchers
// ---------------------------------------------------------------------------
static int align16(int n) { return (n + 15) / 16 * 16; }
static int padded(int n, int pshift) { return n + (pshift >= 31 ? 0 : (n >> pshift)) + 1; }

int fft_lds_stride(int n) { return align16(n); }

void fft_rows_layout(int M, int rb, int pshift, int ntwM, int ntwW, int* r_split, int* r_data, size_t* bytes) {
  *r_split = align16(ntwM);
  *r_data = *r_split + align16(ntwW);
  *bytes = static_cast<size_t>(*r_data + padded(rb * align16(M + 1), pshift)) * sizeof(float2);
}

void fft_cols_layout(int H, int cb, int pshift, int ntwH, int* c_sy, int* c_sx, int* c_data, size_t* bytes) {
  *c_sy = align16(ntwH);
  *c_sx = *c_sy + align16((H + 1) / 2);
  *c_data = *c_sx + 16;
  *bytes = static_cast<size_t>(*c_data + padded(cb * align16(H), pshift)) * sizeof(float2);
}

static const void* fft_kernel_fn(int pass, int ft, bool dyn) {
  if (pass == 0) {
    if (ft == kF32) return dyn ? reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kF32, true>)
                               : reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kF32, false>);
    if (ft == kBF16) return dyn ? reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kBF16, true>)
                                : reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kBF16, false>);
    return dyn ? reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kF16, true>)
               : reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kF16, false>);
  }
  if (pass == 1) return dyn ? reinterpret_cast<const void*>(&fft_cols_kernel<true>)
                            : reinterpret_cast<const void*>(&fft_cols_kernel<false>);
  return dyn ? reinterpret_cast<const void*>(&fft_rows_inv_kernel<true>)
             : reinterpret_cast<const void*>(&fft_rows_inv_kernel<false>);
}

hipError_t fft_init_kernels() {
  const int kMax = 128 * 1024;  // largest need is about 84 KiB; static LDS comes on top
  for (int pass = 0; pass < 3; ++pass)
    for (int ft = 0; ft < 3; ++ft)
      for (int dyn = 0; dyn < 2; ++dyn) {
        if (pass > 0 && ft > 0) continue;
        const hipError_t e = hipFuncSetAttribute(fft_kernel_fn(pass, ft, dyn != 0),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, kMax);
        if (e != hipSuccess) return e;
      }
  return hipSuccess;
}

int fft_grid(int pass, int ft, size_t lds_bytes, int items) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fft_kernel_fn(pass, ft, false), kFftThreads,
                                                   lds_bytes) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  return std::max(1, std::min(items, cus * per_cu));
}

template <int FT>
static void rows_fwd(const FftPlane* planes, int nplanes, int items, int grid, size_t lds, hipStream_t s,
                     WorkHeader* work) {
  const dim3 g(grid), b(kFftThreads);
  if (work == nullptr)
    hipLaunchKernelGGL((fft_rows_fwd_kernel<FT, false>), g, b, lds, s, planes, nplanes, items, work);
  else
    hipLaunchKernelGGL((fft_rows_fwd_kernel<FT, true>), g, b, lds, s, planes, nplanes, items, work);
}

hipError_t launch_fft_rows_fwd(const FftPlane* planes, int nplanes, int items, int grid, size_t lds_bytes,
                               int field_type, hipStream_t s, WorkHeader* work) {
  if (grid <= 0) return hipSuccess;
  if (field_type == kF32) rows_fwd<kF32>(planes, nplanes, items, grid, lds_bytes, s, work);
  else if (field_type == kBF16) rows_fwd<kBF16>(planes, nplanes, items, grid, lds_bytes, s, work);
  else rows_fwd<kF16>(planes, nplanes, items, grid, lds_bytes, s, work);
  return hipGetLastError();
}

hipError_t launch_fft_cols(const FftPlane* planes, int nplanes, int items, int grid, size_t lds_bytes,
                           hipStream_t s, WorkHeader* work) {
  if (grid <= 0) return hipSuccess;
  const dim3 g(grid), b(kFftThreads);
  if (work == nullptr)
    hipLaunchKernelGGL((fft_cols_kernel<false>), g, b, lds_bytes, s, planes, nplanes, items, work);
  else
    hipLaunchKernelGGL((fft_cols_kernel<true>), g, b, lds_bytes, s, planes, nplanes, items, work);
  return hipGetLastError();
}

hipError_t launch_fft_rows_inv(const FftPlane* planes, int nplanes, int items, int grid, size_t lds_bytes,
                               hipStream_t s, WorkHeader* work) {
  if (grid <= 0) return hipSuccess;
  const dim3 g(grid), b(kFftThreads);
  if (work == nullptr)
    hipLaunchKernelGGL((fft_rows_inv_kernel<false>), g, b, lds_bytes, s, planes, nplanes, items, work);
  else
    hipLaunchKernelGGL((fft_rows_inv_kernel<true>), g, b, lds_bytes, s, planes, nplanes, items, work);
  return hipGetLastError();
}

}  // namespace blfls
