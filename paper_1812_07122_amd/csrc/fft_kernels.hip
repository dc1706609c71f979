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
// Transforms are in-place Stockham passes in LDS with radices 2, 3, 4, 5, 8, 9, 15, 16.
// Each workgroup first stages two-level twiddle tables of its transform lengths
// (FP64 host tables rounded to FP32, about 1.5 KiB) in LDS next to the data, so
// no stage waits on global memory and two workgroups fit on a CU; index
// arithmetic uses precomputed multiply-shift division; consecutive row blocks
// are placed on the same XCD so partial lines of the transposed spectrum meet
// in one L2.
#include "blfls_field.h"
#include "blfls_internal.h"
#include "blfls_launch.h"
#include "blfls_work.h"

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

// Product of two non-negative indices below 2^24 whose product fits 32 bits
// (every LDS and per-plane spectrum index here): one full-rate 24-bit multiply
// instead of the quarter-rate 32-bit one.
__device__ __forceinline__ int imul(int a, int b) {
  return static_cast<int>(__umul24(static_cast<uint32_t>(a), static_cast<uint32_t>(b)));
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv d) {
  return (__umulhi(n, d.mul) + n) >> d.shift;
}

// W_N^e from a two-level table in LDS (lo: W_N^j, j < 64; hi: W_N^(64 j)).
__device__ __forceinline__ float2 twiddle(const float2* tab, int e) {
  return cmul(tab[kTwLo + (e >> 6)], tab[e & (kTwLo - 1)]);
}

// Logical workgroup index such that consecutive logical indices run on the same
// XCD (workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2): neighbouring row blocks then share the L2 lines of the transposed spectrum.
__device__ __forceinline__ int xcd_remap(int b, int nblk) {
  constexpr int kXcd = 8;
  const int q = nblk / kXcd, rem = nblk % kXcd;
  const int x = b % kXcd;
  return x * q + min(x, rem) + b / kXcd;
}

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
  // cos and sin of 2 pi m / 9 for the products m = t1 k2 in {1, 2, 4}
  constexpr float kC[5] = {1.0f, 0.76604444311897803520f, 0.17364817766693034885f, 0.0f, -0.93969262078590838405f};
  constexpr float kS[5] = {0.0f, 0.64278760968653932632f, 0.98480775301220805936f, 0.0f, 0.34202014332566873304f};
  float2 b[3][3];
#pragma unroll
  for (int t1 = 0; t1 < 3; ++t1) {
    float2 c[3] = {a[t1], a[t1 + 3], a[t1 + 6]};
    butterfly<3>(c, sg);
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2) {
      const int m = t1 * k2;
      b[k2][t1] = m == 0 ? c[k2] : cmul(c[k2], make_float2(kC[m], sg * kS[m]));
    }
  }
#pragma unroll
  for (int k2 = 0; k2 < 3; ++k2) {
    butterfly<3>(b[k2], sg);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) a[3 * k1 + k2] = b[k2][k1];
  }
}

// Radix 15 as 3 x 5 by the prime-factor (Good-Thomas) mapping, no twiddles:
// input t = (5 t1 + 3 t2) mod 15, output k = (10 k1 + 6 k2) mod 15 (k = k1 mod 3,
// k = k2 mod 5), so A_k = sum_{t1} w3^{t1 k1} sum_{t2} w5^{t2 k2} a_t.
template <>
__device__ __forceinline__ void butterfly<15>(float2* a, float sg) {
  float2 b[3][5];
#pragma unroll
  for (int t1 = 0; t1 < 3; ++t1) {
#pragma unroll
    for (int t2 = 0; t2 < 5; ++t2) b[t1][t2] = a[(5 * t1 + 3 * t2) % 15];
    butterfly<5>(b[t1], sg);
  }
#pragma unroll
  for (int k2 = 0; k2 < 5; ++k2) {
    float2 c[3] = {b[0][k2], b[1][k2], b[2][k2]};
    butterfly<3>(c, sg);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) a[(10 * k1 + 6 * k2) % 15] = c[k1];
  }
}

// Padded LDS index: one spare slot per 16 complex values, so the stride-R
// writes of the early Stockham stages spread over the LDS banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// Element sources and destinations of a stage; b is the transform, n the element.
struct LdsIO {  // in-place LDS buffer (padded layout)
  static constexpr bool kLds = true;
  float2* buf;
  int stride;
  __device__ __forceinline__ float2 load(int b, int n) const { return buf[pad(imul(b, stride) + n)]; }
  __device__ __forceinline__ void store(int b, int n, float2 v) const { buf[pad(imul(b, stride) + n)] = v; }
};

// One Stockham stage over `batch` transforms of length N.  Input element
// j + t*N/R of a transform, output element (j - k) R + k + t Ns with
// k = j mod Ns (decimation in time).  The stage's twiddles
// exp(-2 pi i t k/(Ns R)) = W_N^(t k es) come from the transform's two-level
// table in LDS.  When both ends are the same LDS buffer the inputs are read
// into registers before a barrier, so the update is in place; a barrier
// follows any stage that writes LDS.
template <int R, int T, int MAXE, class SRC, class DST>
__device__ __forceinline__ void fft_stage(const SRC& src, const DST& dst, int batch, const FftStage& S,
                                          const float2* tw, float sg) {
  // butterflies per thread held across the barrier; radix 15 keeps one (the plan
  // bounds its workgroups to T radix-15 butterflies, kFftRadix15Elems elements)
  constexpr int kMaxB = R == 15 ? 1 : (MAXE / R + T - 1) / T;
  static_assert(R != 15 || T * 15 == kFftRadix15Elems, "radix-15 workgroup bound");
  const int per = S.per;
  const int Ns = S.ns;
  const int total = per * batch;
  float2 a[kMaxB][R];
  int outb[kMaxB], outn[kMaxB];
#pragma unroll
  for (int m = 0; m < kMaxB; ++m) {
    const int g = threadIdx.x + m * T;
    if (g < total) {
      const int b = static_cast<int>(fdiv(static_cast<uint32_t>(g), S.per_div));
      const int j = g - imul(b, per);
#pragma unroll
      for (int t = 0; t < R; ++t) a[m][t] = src.load(b, j + t * per);
      const int k = j - imul(static_cast<int>(fdiv(static_cast<uint32_t>(j), S.ns_div)), Ns);
      outb[m] = b;
      outn[m] = (j - k) * R + k;
      if (Ns > 1) {
        // w^t for t = 1..R-1 from one table lookup of w = W_N^(k es): squares
        // for even t, one more factor w for odd t (at most 2 log2 t products
        // deep, a few ulp), so a butterfly reads two table entries, not 2 (R-1)
        float2 w[R];
        w[1] = twiddle(tw, imul(k, S.es));
        w[1].y = sg > 0.0f ? -w[1].y : w[1].y;  // the inverse takes the conjugate
#pragma unroll
        for (int t = 2; t < R; ++t) w[t] = (t & 1) ? cmul(w[t - 1], w[1]) : cmul(w[t / 2], w[t / 2]);
#pragma unroll
        for (int t = 1; t < R; ++t) a[m][t] = cmul(a[m][t], w[t]);
      }
    }
  }
  if (SRC::kLds && DST::kLds) __syncthreads();
#pragma unroll
  for (int m = 0; m < kMaxB; ++m) {
    const int g = threadIdx.x + m * T;
    if (g < total) {
      butterfly<R>(a[m], sg);
#pragma unroll
      for (int t = 0; t < R; ++t) dst.store(outb[m], outn[m] + t * Ns, a[m][t]);
    }
  }
  if (DST::kLds) __syncthreads();
}

template <int T, int MAXE, class SRC, class DST>
__device__ __forceinline__ void fft_stage_r(const SRC& src, const DST& dst, int batch, const FftStage& S,
                                            const float2* tw, float sg) {
  switch (S.radix) {
    case 2: fft_stage<2, T, MAXE>(src, dst, batch, S, tw, sg); break;
    case 3: fft_stage<3, T, MAXE>(src, dst, batch, S, tw, sg); break;
    case 4: fft_stage<4, T, MAXE>(src, dst, batch, S, tw, sg); break;
    case 5: fft_stage<5, T, MAXE>(src, dst, batch, S, tw, sg); break;
    case 8: fft_stage<8, T, MAXE>(src, dst, batch, S, tw, sg); break;
    case 9: fft_stage<9, T, MAXE>(src, dst, batch, S, tw, sg); break;
    case 15: fft_stage<15, T, MAXE>(src, dst, batch, S, tw, sg); break;
    default: fft_stage<16, T, MAXE>(src, dst, batch, S, tw, sg); break;
  }
}

// Whole transform, forward (sg = -1) or inverse without scaling (sg = +1): the
// first stage reads `src`, the last writes `dst`, the others work in place in
// `lds`.  A length-1 transform copies.
template <int T, int MAXE, class SRC, class DST>
__device__ __forceinline__ void fft_run(const FftSize& sz, const float2* tw, float sg, int batch, const SRC& src,
                                        const LdsIO& lds, const DST& dst) {
  const int n = sz.nstages;
  if (n == 0) {
    for (int b = threadIdx.x; b < batch; b += T) dst.store(b, 0, src.load(b, 0));
    if (DST::kLds) __syncthreads();
    return;
  }
  if (n == 1) {
    fft_stage_r<T, MAXE>(src, dst, batch, sz.st[0], tw, sg);
    return;
  }
  fft_stage_r<T, MAXE>(src, lds, batch, sz.st[0], tw, sg);
  for (int s = 1; s < n - 1; ++s) fft_stage_r<T, MAXE>(lds, lds, batch, sz.st[s], tw, sg);
  fft_stage_r<T, MAXE>(lds, dst, batch, sz.st[n - 1], tw, sg);
}

// Global memory at a 32-bit byte offset from a base pointer: the load or store
// takes the (workgroup-uniform) base in scalar registers and the offset in one
// vector register, with no 64-bit address arithmetic per element.  Every plane,
// field and spectrum here is far below 4 GiB.
typedef float vf2 __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ T gload_raw(const void* base, uint32_t byte_off) {
  return *(const __attribute__((address_space(1))) T*)((const __attribute__((address_space(1))) char*)base +
                                                         byte_off);
}
template <class T>
__device__ __forceinline__ T gload(const void* base, uint32_t byte_off) {
  return gload_raw<T>(base, byte_off);
}
template <>
__device__ __forceinline__ float2 gload<float2>(const void* base, uint32_t byte_off) {
  const vf2 v = gload_raw<vf2>(base, byte_off);
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gstore(void* base, uint32_t byte_off, float2 v) {
  *(__attribute__((address_space(1))) vf2*)((__attribute__((address_space(1))) char*)base + byte_off) = vf2{v.x, v.y};
}

// Two consecutive field values at an even index, as FP32.
template <int FT>
__device__ __forceinline__ float2 load_pair(const void* base, uint32_t idx) {
  if (FT == kF32) return gload<float2>(base, idx * 4u);
  const uint32_t w = gload<uint32_t>(base, idx * 2u);
  if (FT == kBF16) return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xFFFF0000u));
  _Float16 h0, h1;
  const uint16_t lo = static_cast<uint16_t>(w & 0xFFFFu), hi = static_cast<uint16_t>(w >> 16);
  __builtin_memcpy(&h0, &lo, 2);
  __builtin_memcpy(&h1, &hi, 2);
  return make_float2(static_cast<float>(h0), static_cast<float>(h1));
}

template <int FT>
__device__ __forceinline__ float load_one(const void* base, uint32_t idx) {
  if (FT == kF32) return gload<float>(base, idx * 4u);
  const uint16_t v = gload<uint16_t>(base, idx * 2u);
  if (FT == kBF16) return __uint_as_float(static_cast<uint32_t>(v) << 16);
  _Float16 h;
  __builtin_memcpy(&h, &v, 2);
  return static_cast<float>(h);
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

template <int T>
__device__ __forceinline__ void stage_twiddles(float2* dst, const float2* __restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += T) dst[i] = src[i];
}

// Global -> LDS copies issue kLoadBatch loads per thread before storing any of
// them, so one memory round trip covers kLoadBatch elements instead of one.
constexpr int kLoadBatch = 8;

}  // namespace

// ---------------------------------------------------------------------------
// Stage sources and destinations of the three passes
// ---------------------------------------------------------------------------

// Right-hand side of the residual-form solve for row i0 + b, two reals per
// complex: c(i, j) = lam ((r_x(i, j-1) - r_x(i, j)) + (r_y(i-1, j) - r_y(i, j))).
// FP16 fields hold r_x s_x and r_y s_y (powers of two, see field_store_scales):
// then lam is lambda / s_x and ky = s_x / s_y.
template <int FT>
struct RhsSrc {
  static constexpr bool kLds = false;
  const void* rx;
  const void* ry;
  int i0, H, W;
  float lam;
  float ky;
  __device__ __forceinline__ float2 load(int b, int n) const {
    const int i = i0 + b;
    const int im1 = i == 0 ? H - 1 : i - 1;
    const int j0 = 2 * n;
    const int jm = j0 == 0 ? W - 1 : j0 - 1;
    const uint32_t ri = imul(i, W);
    const float2 x = load_pair<FT>(rx, ri + j0);
    const float2 y = load_pair<FT>(ry, ri + j0);
    const float2 yp = load_pair<FT>(ry, imul(im1, W) + j0);
    const float xm = load_one<FT>(rx, ri + jm);
    if (FT == kF16)
      return make_float2(lam * ((xm - x.x) + ky * (yp.x - y.x)), lam * ((x.x - x.y) + ky * (yp.y - y.y)));
    return make_float2(lam * ((xm - x.x) + (yp.x - y.x)), lam * ((x.x - x.y) + (yp.y - y.y)));
  }
};

// Spectrum columns in HBM ([W/2+1][H] layout, column b of the block).
struct ColIO {
  static constexpr bool kLds = false;
  float2* spec;
  int H;
  __device__ __forceinline__ float2 load(int b, int n) const { return gload<float2>(spec, 8u * (imul(b, H) + n)); }
  __device__ __forceinline__ void store(int b, int n, float2 v) const { gstore(spec, 8u * (imul(b, H) + n), v); }
};

// LDS destination that applies the Eq. (8) divide, 1 / (H W (1 + lam (sx + sy)))
// (times the detail gain's 1 - m on the last iteration: u + m (f - u) = f + (1 - m) delta).
struct ScaledLds {
  static constexpr bool kLds = true;
  float2* buf;
  int H, k0;
  const float* sx;
  const float* sy;
  float lam, inv_hw;
  __device__ __forceinline__ void store(int b, int n, float2 v) const {
    const float den = fmaf(lam, sx[k0 + b] + sy[n], 1.0f);
    // den >= 1: the hardware reciprocal (1 ulp) instead of a correctly rounded
    // division, which costs ten instructions per spectrum value
    buf[pad(imul(b, H) + n)] = cscale(v, inv_hw * __builtin_amdgcn_rcpf(den));
  }
};

// u = f + delta for row i0 + b; element n holds the reals at columns 2n, 2n+1.
struct OutDst {
  static constexpr bool kLds = false;
  const float* __restrict__ f;
  float* __restrict__ u;
  int64_t pitch;
  int i0;
  __device__ __forceinline__ void store(int b, int n, float2 v) const {
    const int64_t o = static_cast<int64_t>(i0 + b) * pitch + 2 * n;
    u[o] = f[o] + v.x;
    u[o + 1] = f[o + 1] + v.y;
  }
};

// ---------------------------------------------------------------------------
// Wave-resident transforms of length N = 64 L (L = 8, 16): one wave holds one
// transform, lane l the elements l + 64 m in registers m.  With k = k1 + L k2,
//   X[k1 + L k2] = sum_l W_64^(l k2) W_N^(l k1) sum_m x[l + 64 m] W_L^(m k1),
// so each lane takes an L-point DFT of its registers and a twiddle, and the
// 64-point DFTs over the lanes (one per k1) run as 8 x 8 (l = l1 + 8 l2,
// k2 = k2a + 8 k2b) through a wave-private LDS block: 8-point DFTs over l2,
// the twiddle W_64^(l1 k2a), 8-point DFTs over l1.  The inverse retraces the
// steps with conjugate twiddles.  A wave orders its own LDS accesses, so the
// exchanges need a wave-scope fence, not a workgroup barrier.
// ---------------------------------------------------------------------------
constexpr int kWaveCols = kFftThreads / 64;   // transforms (waves) per workgroup

// Slot of entry (row, col) of the 8 x 8 block k1 in a wave's LDS: a bijection
// on the block whose rows are rotated by k1 and whose columns are XOR-ed with
// the row, so the column reads, the row reads and the lane-order transposes
// each touch 16 distinct 8-byte bank pairs per 16 lanes.
__device__ __forceinline__ int wslot(int k1, int row, int col) {
  return k1 * 64 + (((row + k1) & 7) << 3) + (col ^ row);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Powers w^t for t < N (N a multiple of 4, at most 16) as w^(t & 3) w^(4 (t >> 2)):
// six or fewer products, at most four deep, and eight registers at N = 16.
template <int N>
struct Powers {
  float2 lo[4], hi[N / 4];   // w^0..w^3 and w^0, w^4, w^8, w^12
  __device__ __forceinline__ explicit Powers(float2 w) {
    lo[0] = make_float2(1.0f, 0.0f);
    lo[1] = w;
    lo[2] = cmul(w, w);
    lo[3] = cmul(lo[2], w);
    hi[0] = lo[0];
    if (N > 4) hi[1] = cmul(lo[2], lo[2]);
#pragma unroll
    for (int j = 2; j < N / 4; ++j) hi[j] = cmul(hi[j - 1], hi[1]);
  }
  // v w^t (t known at compile time after unrolling)
  __device__ __forceinline__ float2 mul(float2 v, int t) const {
    if (t & 3) v = cmul(v, lo[t & 3]);
    if (t >> 2) v = cmul(v, hi[t >> 2]);
    return v;
  }
  __device__ __forceinline__ float2 mul_conj(float2 v, int t) const {
    if (t & 3) v = cmul(v, cconj(lo[t & 3]));
    if (t >> 2) v = cmul(v, cconj(hi[t >> 2]));
    return v;
  }
};

// Forward transform of the wave's registers a (a[m] = x[l + 64 m]) with the
// two-level table tw of W_N.  On return d[q][k2b] = X[k1 + L (k2a + 8 k2b)]
// with p = l + 64 q, k1 = p / 8, k2a = p mod 8.
template <int L>
__device__ __forceinline__ void wave_fft_fwd(float2 (&a)[L], float2 (&d)[L / 8][8], float2* T, int l,
                                             const float2* tw) {
  butterfly<L>(a, -1.0f);
  {
    const Powers<L> pw(tw[l]);   // W_N^(l k1); entries below 64 of the table are W_N^j
#pragma unroll
    for (int k1 = 1; k1 < L; ++k1) a[k1] = pw.mul(a[k1], k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < L; ++k1) T[wslot(k1, l >> 3, l & 7)] = a[k1];
  wave_lds_sync();
  // 8-point DFTs over l2 for each (k1, l1), then W_64^(l1 k2a)
#pragma unroll
  for (int q = 0; q < L / 8; ++q) {
    const int p = l + 64 * q, k1 = p >> 3, l1 = p & 7;
    float2 b[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) b[r] = T[wslot(k1, r, l1)];
    butterfly<8>(b, -1.0f);
    const Powers<8> pv(twiddle(tw, l1 * L));   // W_64^l1 = W_N^(l1 L)
#pragma unroll
    for (int r = 1; r < 8; ++r) b[r] = pv.mul(b[r], r);
#pragma unroll
    for (int r = 0; r < 8; ++r) T[wslot(k1, r, l1)] = b[r];
  }
  wave_lds_sync();
  // 8-point DFTs over l1 for each (k1, k2a)
#pragma unroll
  for (int q = 0; q < L / 8; ++q) {
    const int p = l + 64 * q, k1 = p >> 3, k2a = p & 7;
#pragma unroll
    for (int col = 0; col < 8; ++col) d[q][col] = T[wslot(k1, k2a, col)];
    butterfly<8>(d[q], -1.0f);
  }
}

// Inverse (unscaled) of wave_fft_fwd: from d in its layout to a[m] = y[l + 64 m].
// The first writes go to the slots this lane's last forward reads came from.
template <int L>
__device__ __forceinline__ void wave_fft_inv(float2 (&d)[L / 8][8], float2 (&a)[L], float2* T, int l,
                                             const float2* tw) {
#pragma unroll
  for (int q = 0; q < L / 8; ++q) {
    const int p = l + 64 * q, k1 = p >> 3, k2a = p & 7;
    butterfly<8>(d[q], 1.0f);
#pragma unroll
    for (int col = 0; col < 8; ++col) T[wslot(k1, k2a, col)] = d[q][col];
  }
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < L / 8; ++q) {
    const int p = l + 64 * q, k1 = p >> 3, l1 = p & 7;
    float2 e[8];
    const Powers<8> pv(twiddle(tw, l1 * L));
#pragma unroll
    for (int r = 0; r < 8; ++r) e[r] = pv.mul_conj(T[wslot(k1, r, l1)], r);
    butterfly<8>(e, 1.0f);
#pragma unroll
    for (int r = 0; r < 8; ++r) T[wslot(k1, r, l1)] = e[r];
  }
  wave_lds_sync();
#pragma unroll
  for (int k1 = 0; k1 < L; ++k1) a[k1] = T[wslot(k1, l >> 3, l & 7)];
  {
    const Powers<L> pw(tw[l]);
#pragma unroll
    for (int k1 = 1; k1 < L; ++k1) a[k1] = pw.mul_conj(a[k1], k1);
  }
  butterfly<L>(a, 1.0f);
}

// ---------------------------------------------------------------------------
// Pass 1: c = lam (D_x^T r_x + D_y^T r_y), real FFT of each row, transposed store
// LDS: [table of W_{W/2}: kTwMax][table of W_W: kTwMax][rows: rb x (M+1), padded]
// ---------------------------------------------------------------------------
// Pass 1 for W/2 = 64 L: one wave per row (right-hand side, forward transform
// in registers, split step), then the workgroup's kWaveCols rows go out
// through LDS so each spectrum column receives kWaveCols consecutive values.
// LDS: kWaveCols exchange blocks of W/2 values, then [W/2 + 1][kWaveCols + 1].
template <int L, int FT>
__device__ __forceinline__ void rows_fwd_wave_item(const FftPlane& P, int blk, float2* smem, float lam, float ky) {
  constexpr int kS = kWaveCols + 1;   // staging row stride (one spare slot against bank conflicts)
  const int H = P.H, W = P.W, M = W >> 1;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int i0 = blk * kWaveCols;
  const int nrows = min(kWaveCols, H - i0);
  const bool live = wave < nrows;
  float2 x[L], xm = make_float2(0.0f, 0.0f);
  if (live) {
    float2* T = smem + wave * M;
    // c(i, j) = lam ((r_x(i, j-1) - r_x(i, j)) + (r_y(i-1, j) - r_y(i, j))) for the
    // pair j = 2n, 2n + 1, n = l + 64 m: r_x(i, 2n - 1) is the odd value of the lane
    // to the left (of lane 63 one register back for lane 0; column W - 1 at n = 0)
    const int i = i0 + wave;
    const uint32_t ri = imul(i, W), rp = imul(i == 0 ? H - 1 : i - 1, W);
    float2 a[L], d[L / 8][8];
    float carry = load_one<FT>(P.rx, ri + W - 1);
#pragma unroll
    for (int m = 0; m < L; ++m) {
      const uint32_t j0 = 2u * (l + 64 * m);
      const float2 x = load_pair<FT>(P.rx, ri + j0);
      const float2 y = load_pair<FT>(P.ry, ri + j0);
      const float2 yp = load_pair<FT>(P.ry, rp + j0);
      const float left = __shfl_up(x.y, 1);
      const float xm = l == 0 ? carry : left;
      carry = __shfl(x.y, 63);
      if (FT == kF16)
        a[m] = make_float2(lam * ((xm - x.x) + ky * (yp.x - y.x)), lam * ((x.x - x.y) + ky * (yp.y - y.y)));
      else
        a[m] = make_float2(lam * ((xm - x.x) + (yp.x - y.x)), lam * ((x.x - x.y) + (yp.y - y.y)));
    }
    wave_fft_fwd<L>(a, d, T, l, P.twM);
    wave_lds_sync();
    // Z in natural order, then X[k] = E[k] + exp(-2 pi i k / W) O[k], k = 0..M
#pragma unroll
    for (int q = 0; q < L / 8; ++q) {
      const int p = l + 64 * q, k1 = p >> 3, k2a = p & 7;
#pragma unroll
      for (int k2b = 0; k2b < 8; ++k2b) T[k1 + L * (k2a + 8 * k2b)] = d[q][k2b];
    }
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < L; ++q) {
      const int k = l + 64 * q;
      const float2 zk = T[k];
      const float2 zm = T[(M - k) & (M - 1)];
      const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
      const float2 o = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));   // (zk - conj zm) / (2i)
      x[q] = cadd(e, cmul(twiddle(P.twW, k), o));
    }
    if (l == 0) {   // k = M: Z[M] = Z[0]
      const float2 z0 = T[0];
      const float2 e = make_float2(z0.x, 0.0f);
      const float2 o = make_float2(z0.y, 0.0f);
      xm = cadd(e, cmul(twiddle(P.twW, M), o));
    }
  }
  __syncthreads();   // every wave is done with its block: the staging overlays them
  float2* S = smem;
  if (live) {
#pragma unroll
    for (int q = 0; q < L; ++q) S[(l + 64 * q) * kS + wave] = x[q];
    if (l == 0) S[M * kS + wave] = xm;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < (M + 1) * kWaveCols; idx += kFftThreads) {
    const int k = idx / kWaveCols, w = idx - k * kWaveCols;
    if (w < nrows) gstore(P.spec, 8u * (imul(k, H) + i0 + w), S[k * kS + w]);
  }
}

// WAVE: planes with roww take the one-row-per-wave transform (direct launches
// only, as for the column pass).
template <int FT, bool WAVE>
__device__ __forceinline__ void rows_fwd_item(const FftPlane* __restrict__ planes, int nplanes, int item,
                                              float2* smem) {
  constexpr int T = kFftThreads;
  const FftPlane& P = planes[find_fft_plane<false>(planes, nplanes, item)];
  const int blk = item - P.row_begin;
  if (blk >= P.row_count) return;
  // FP16 fields: undo the fields' power-of-two store scales in the right-hand side
  float lam = P.lambda, ky = 1.0f;
  if (FT == kF16) {
    const float2 fsc = field_store_scales(P.fmm);
    lam = P.lambda / fsc.x;
    ky = fsc.x / fsc.y;
  }
  if (WAVE && P.roww == 8) {
    rows_fwd_wave_item<8, FT>(P, blk, smem, lam, ky);
    return;
  }
  if (WAVE && P.roww == 16) {
    rows_fwd_wave_item<16, FT>(P, blk, smem, lam, ky);
    return;
  }
  const int H = P.H, W = P.W, M = W >> 1;
  const int i0 = blk * P.rb;
  const int nrows = min(P.rb, H - i0);
  const int tid = threadIdx.x;
  float2* twS = smem;
  float2* twR = smem + kTwMax;
  float2* buf = smem + 2 * kTwMax;
  stage_twiddles<T>(twS, P.twM, P.ntwM);
  stage_twiddles<T>(twR, P.twW, P.ntwW);
  __syncthreads();
  // the first stage forms the right-hand side straight from the residual fields
  const LdsIO lds{buf, M};
  fft_run<T, kFftLdsComplex>(*P.szM, twS, -1.0f, nrows, RhsSrc<FT>{P.rx, P.ry, i0, H, W, lam, ky}, lds, lds);

  // split step: X[k] = E[k] + exp(-2 pi i k/W) O[k], k = 0..M, Z[M] = Z[0]
  float2* spec = P.spec;
  for (int idx = tid; idx < (M + 1) * nrows; idx += T) {
    int k, row;
    if (nrows == P.rb) {
      k = static_cast<int>(fdiv(static_cast<uint32_t>(idx), P.rb_div));
      row = idx - k * nrows;
    } else {
      k = idx / nrows;
      row = idx - k * nrows;
    }
    const float2 zk = buf[pad(imul(row, M) + (k == M ? 0 : k))];
    const float2 zm = buf[pad(imul(row, M) + (k == 0 ? 0 : M - k))];
    const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    // o = (zk - conj(zm)) / (2i)
    const float2 o = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
    gstore(spec, 8u * (imul(k, H) + i0 + row), cadd(e, cmul(twiddle(twR, k), o)));
  }
}

// Pass 2 for H = 64 L: one wave per spectrum column (forward, divide, inverse
// in registers); a workgroup takes kWaveCols consecutive columns.
template <int L>
__device__ __forceinline__ void cols_wave_item(const FftPlane& P, int blk, float2* smem) {
  const int H = P.H, W = P.W, M = W >> 1;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int c = blk * kWaveCols + wave;
  if (c > M) return;   // no workgroup barrier follows
  float2* T = smem + wave * (L * 64);
  const uint32_t base = 8u * static_cast<uint32_t>(imul(c, H));
  float2 a[L], d[L / 8][8];
#pragma unroll
  for (int m = 0; m < L; ++m) a[m] = gload<float2>(P.spec, base + 8u * (l + 64 * m));
  wave_fft_fwd<L>(a, d, T, l, P.twH);
  // the Eq. (8) divide on X[k1 + L (k2a + 8 k2b)]
  const float sxc = P.sx[c];
  const float inv_hw = P.gain * (1.0f / (static_cast<float>(H) * static_cast<float>(W)));
#pragma unroll
  for (int q = 0; q < L / 8; ++q) {
    const int p = l + 64 * q, k1 = p >> 3, k2a = p & 7;
#pragma unroll
    for (int k2b = 0; k2b < 8; ++k2b) {
      const float den = fmaf(P.lambda, sxc + P.sy[k1 + L * (k2a + 8 * k2b)], 1.0f);
      d[q][k2b] = cscale(d[q][k2b], inv_hw * __builtin_amdgcn_rcpf(den));
    }
  }
  wave_fft_inv<L>(d, a, T, l, P.twH);
#pragma unroll
  for (int m = 0; m < L; ++m) gstore(P.spec, base + 8u * (l + 64 * m), a[m]);
}

// ---------------------------------------------------------------------------
// Pass 2: per spectrum column, forward FFT over H, divide, inverse FFT over H.
// The forward transform reads the columns from HBM in its first stage and
// applies the divide in its last; the inverse writes HBM in its last stage.
// LDS: [table of W_H: kTwMax][columns: cb x H, padded]
// ---------------------------------------------------------------------------
// WAVE: planes with colw take the one-column-per-wave transform (direct
// launches; the persistent kernel omits that path, which keeps it within its
// register budget, and the server launches such steps directly).
template <bool WAVE>
__device__ __forceinline__ void cols_item(const FftPlane* __restrict__ planes, int nplanes, int item,
                                          float2* smem) {
  constexpr int T = kFftThreads;
  const FftPlane& P = planes[find_fft_plane<true>(planes, nplanes, item)];
  const int blk = item - P.col_begin;
  if (blk >= P.col_count) return;
  if (WAVE && P.colw == 16) {
    cols_wave_item<16>(P, blk, smem);
    return;
  }
  if (WAVE && P.colw == 8) {
    cols_wave_item<8>(P, blk, smem);
    return;
  }
  const int H = P.H, W = P.W, M = W >> 1;
  const int k0 = blk * P.cb;
  const int ncols = min(P.cb, M + 1 - k0);
  float2* twS = smem;
  float2* buf = smem + kTwMax;
  stage_twiddles<T>(twS, P.twH, P.ntwH);
  __syncthreads();
  const ColIO col{P.spec + static_cast<int64_t>(k0) * H, H};
  const LdsIO lds{buf, H};
  const ScaledLds scaled{buf, H, k0, P.sx, P.sy, P.lambda,
                         P.gain * (1.0f / (static_cast<float>(H) * static_cast<float>(W)))};
  fft_run<T, kFftLdsComplex>(*P.szH, twS, -1.0f, ncols, col, lds, scaled);
  fft_run<T, kFftLdsComplex>(*P.szH, twS, 1.0f, ncols, lds, lds, col);
}

// ---------------------------------------------------------------------------
// Pass 3: complex-to-real inverse of each row, u = f + delta (written by the
// last stage of the inverse transform)
// LDS: [table of W_{W/2}: kTwMax][table of W_W: kTwMax][rows: rb x (M+1), padded]
// ---------------------------------------------------------------------------
// Pass 3 for W/2 = 64 L: the workgroup gathers kWaveCols rows of the half
// spectrum through LDS, then one wave per row forms Z (the inverse split step)
// in the forward transform's output layout, transforms back in registers and
// writes u = f + delta.
template <int L>
__device__ __forceinline__ void rows_inv_wave_item(const FftPlane& P, int blk, float2* smem) {
  constexpr int kS = kWaveCols + 1;
  const int H = P.H, W = P.W, M = W >> 1;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int i0 = blk * kWaveCols;
  const int nrows = min(kWaveCols, H - i0);
  const bool live = wave < nrows;
  float2* S = smem;
  const int ntot = (M + 1) * kWaveCols;
  for (int base = threadIdx.x; base < ntot; base += kFftThreads * kLoadBatch) {
    float2 v[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int idx = base + u * kFftThreads;
      const int k = idx / kWaveCols, w = idx - k * kWaveCols;
      v[u] = make_float2(0.0f, 0.0f);
      if (idx < ntot && w < nrows) v[u] = gload<float2>(P.spec, 8u * (imul(k, H) + i0 + w));
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int idx = base + u * kFftThreads;
      const int k = idx / kWaveCols, w = idx - k * kWaveCols;
      if (idx < ntot) S[k * kS + w] = v[u];
    }
  }
  __syncthreads();
  // Z[k] = (X[k] + conj X[M-k]) + i exp(2 pi i k / W) (X[k] - conj X[M-k])
  float2 d[L / 8][8];
  if (live) {
#pragma unroll
    for (int q = 0; q < L / 8; ++q) {
      const int p = l + 64 * q, k1 = p >> 3, k2a = p & 7;
#pragma unroll
      for (int k2b = 0; k2b < 8; ++k2b) {
        const int k = k1 + L * (k2a + 8 * k2b);
        const float2 xa = S[k * kS + wave], xb = S[(M - k) * kS + wave];
        const float2 sa = cadd(xa, cconj(xb)), da = csub(xa, cconj(xb));
        d[q][k2b] = cadd(sa, cmul_isg(cmul(cconj(twiddle(P.twW, k)), da), 1.0f));
      }
    }
  }
  __syncthreads();   // the staging is read: the exchange blocks overlay it
  if (live) {
    float2* T = smem + wave * M;
    float2 a[L];
    wave_fft_inv<L>(d, a, T, l, P.twM);
    const int64_t row = static_cast<int64_t>(i0 + wave) * P.pitch;
#pragma unroll
    for (int m = 0; m < L; ++m) {
      const int64_t o = row + 2 * (l + 64 * m);
      P.u[o] = P.f[o] + a[m].x;
      P.u[o + 1] = P.f[o + 1] + a[m].y;
    }
  }
}

template <bool WAVE>
__device__ __forceinline__ void rows_inv_item(const FftPlane* __restrict__ planes, int nplanes, int item,
                                              float2* smem) {
  constexpr int T = kFftThreads;
  const FftPlane& P = planes[find_fft_plane<false>(planes, nplanes, item)];
  const int blk = item - P.row_begin;
  if (blk >= P.row_count) return;
  if (WAVE && P.roww == 8) {
    rows_inv_wave_item<8>(P, blk, smem);
    return;
  }
  if (WAVE && P.roww == 16) {
    rows_inv_wave_item<16>(P, blk, smem);
    return;
  }
  const int H = P.H, W = P.W, M = W >> 1;
  const int S = M + 1;  // LDS row stride
  const int i0 = blk * P.rb;
  const int nrows = min(P.rb, H - i0);
  const int tid = threadIdx.x;
  float2* twS = smem;
  float2* twR = smem + kTwMax;
  float2* buf = smem + 2 * kTwMax;
  stage_twiddles<T>(twS, P.twM, P.ntwM);
  stage_twiddles<T>(twR, P.twW, P.ntwW);
  const float2* spec = P.spec;
  const int ntot = S * nrows;
  for (int base = tid; base < ntot; base += T * kLoadBatch) {
    float2 v[kLoadBatch];
    int dst[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int idx = base + u * T;
      if (idx < ntot) {
        int k, row;
        if (nrows == P.rb) {
          k = static_cast<int>(fdiv(static_cast<uint32_t>(idx), P.rb_div));
          row = idx - k * nrows;
        } else {
          k = idx / nrows;
          row = idx - k * nrows;
        }
        v[u] = gload<float2>(spec, 8u * (imul(k, H) + i0 + row));
        dst[u] = pad(imul(row, S) + k);
      }
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u)
      if (base + u * T < ntot) buf[dst[u]] = v[u];
  }
  __syncthreads();
  // Z[k] = (X[k] + conj X[M-k]) + i exp(2 pi i k/W) (X[k] - conj X[M-k]), k = 0..M-1;
  // one thread forms the pair (k, M-k) so the update is in place
  const int half = M / 2;
  for (int idx = tid; idx < (half + 1) * nrows; idx += T) {
    const int row = idx / (half + 1);
    const int k = idx - row * (half + 1);
    const int ia = pad(imul(row, S) + k), ib = pad(imul(row, S) + M - k);
    const float2 a = buf[ia], b = buf[ib];
    const float2 wa = cconj(twiddle(twR, k));  // exp(+2 pi i k/W)
    const float2 wb = cconj(twiddle(twR, M - k));
    const float2 sa = cadd(a, cconj(b)), da = csub(a, cconj(b));
    const float2 za = cadd(sa, cmul_isg(cmul(wa, da), 1.0f));
    const float2 sb = cadd(b, cconj(a)), db = csub(b, cconj(a));
    const float2 zb = cadd(sb, cmul_isg(cmul(wb, db), 1.0f));
    buf[ia] = za;
    if (k != 0 && M - k != k) buf[ib] = zb;
  }
  __syncthreads();
  const LdsIO lds{buf, S};
  fft_run<T, kFftLdsComplex>(*P.szM, twS, 1.0f, nrows, lds, lds, OutDst{P.f, P.u, P.pitch, i0});
}

// ---------------------------------------------------------------------------
// Kernels: with work == nullptr one workgroup per item; otherwise a fixed
// (persistent) grid draws the items of the work header, read from device
// memory when the kernel runs (launches captured in a graph), from one counter
// per XCD.  Either way consecutive row blocks run on the same XCD.
// ---------------------------------------------------------------------------
template <int FT, bool PERSIST>
__global__ void __launch_bounds__(kFftThreads, 4)
fft_rows_fwd_kernel(const FftPlane* __restrict__ planes, int nplanes, WorkHeader* __restrict__ work) {
  extern __shared__ float2 smem[];
  if (!PERSIST) {
    rows_fwd_item<FT, true>(planes, nplanes, xcd_remap(blockIdx.x, gridDim.x), smem);
    return;
  }
  const int total = work->items, np = work->nplanes;
  const FftPlane* pl = static_cast<const FftPlane*>(work->planes);
  for (;;) {
    const int item = grab_item(work->next[0], total, true);
    if (item >= total) break;
    rows_fwd_item<FT, false>(pl, np, item, smem);
    __syncthreads();
  }
}

template <bool PERSIST>
__global__ void __launch_bounds__(kFftThreads, 4)
fft_cols_kernel(const FftPlane* __restrict__ planes, int nplanes, WorkHeader* __restrict__ work) {
  extern __shared__ float2 smem[];
  if (!PERSIST) {
    cols_item<true>(planes, nplanes, xcd_remap(blockIdx.x, gridDim.x), smem);
    return;
  }
  const int total = work->items2, np = work->nplanes;
  const FftPlane* pl = static_cast<const FftPlane*>(work->planes);
  for (;;) {
    const int item = grab_item(work->next[1], total, true);
    if (item >= total) break;
    cols_item<false>(pl, np, item, smem);
    __syncthreads();
  }
}

template <bool PERSIST>
__global__ void __launch_bounds__(kFftThreads, 4)
fft_rows_inv_kernel(const FftPlane* __restrict__ planes, int nplanes, WorkHeader* __restrict__ work) {
  extern __shared__ float2 smem[];
  if (!PERSIST) {
    rows_inv_item<true>(planes, nplanes, xcd_remap(blockIdx.x, gridDim.x), smem);
    return;
  }
  const int total = work->items, np = work->nplanes;
  const FftPlane* pl = static_cast<const FftPlane*>(work->planes);
  for (;;) {
    const int item = grab_item(work->next[2], total, true);
    if (item >= total) break;
    rows_inv_item<false>(pl, np, item, smem);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static size_t padded(int n) { return static_cast<size_t>(n) + static_cast<size_t>(n) / 16 + 1; }
size_t fft_rows_lds_bytes(int M, int rb) { return (2 * kTwMax + padded(rb * (M + 1))) * sizeof(float2); }
size_t fft_cols_lds_bytes(int H, int cb) { return (kTwMax + padded(cb * H)) * sizeof(float2); }
int fft_cols_wave_per_block() { return kWaveCols; }
size_t fft_cols_wave_lds_bytes(int L) { return static_cast<size_t>(kWaveCols) * L * 64 * sizeof(float2); }
size_t fft_rows_wave_lds_bytes(int L) {
  const size_t exchange = static_cast<size_t>(kWaveCols) * L * 64;
  const size_t staging = static_cast<size_t>(L * 64 + 1) * (kWaveCols + 1);
  return (exchange > staging ? exchange : staging) * sizeof(float2);
}

hipError_t fft_init_kernels() {
  const int kMax = 128 * 1024;  // largest need is about 73 KiB; static LDS comes on top
  const void* fns[] = {reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kF32, false>),
                       reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kBF16, false>),
                       reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kF16, false>),
                       reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kF32, true>),
                       reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kBF16, true>),
                       reinterpret_cast<const void*>(&fft_rows_fwd_kernel<kF16, true>),
                       reinterpret_cast<const void*>(&fft_cols_kernel<false>),
                       reinterpret_cast<const void*>(&fft_cols_kernel<true>),
                       reinterpret_cast<const void*>(&fft_rows_inv_kernel<false>),
                       reinterpret_cast<const void*>(&fft_rows_inv_kernel<true>)};
  for (const void* fn : fns) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMax);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int FT>
static void rows_fwd(const FftPlane* planes, int nplanes, int blocks, size_t lds, hipStream_t s, WorkHeader* work) {
  const dim3 g(blocks), b(kFftThreads);
  if (work == nullptr)
    hipLaunchKernelGGL((fft_rows_fwd_kernel<FT, false>), g, b, lds, s, planes, nplanes, work);
  else
    hipLaunchKernelGGL((fft_rows_fwd_kernel<FT, true>), g, b, lds, s, planes, nplanes, work);
}

hipError_t launch_fft_rows_fwd(const FftPlane* planes, int nplanes, int blocks, size_t lds_bytes,
                               int field_type, hipStream_t s, WorkHeader* work) {
  if (blocks <= 0) return hipSuccess;
  if (field_type == kF32) rows_fwd<kF32>(planes, nplanes, blocks, lds_bytes, s, work);
  else if (field_type == kBF16) rows_fwd<kBF16>(planes, nplanes, blocks, lds_bytes, s, work);
  else rows_fwd<kF16>(planes, nplanes, blocks, lds_bytes, s, work);
  return hipGetLastError();
}

hipError_t launch_fft_cols(const FftPlane* planes, int nplanes, int blocks, size_t lds_bytes, hipStream_t s,
                           WorkHeader* work) {
  if (blocks <= 0) return hipSuccess;
  const dim3 g(blocks), b(kFftThreads);
  if (work == nullptr)
    hipLaunchKernelGGL((fft_cols_kernel<false>), g, b, lds_bytes, s, planes, nplanes, work);
  else
    hipLaunchKernelGGL((fft_cols_kernel<true>), g, b, lds_bytes, s, planes, nplanes, work);
  return hipGetLastError();
}

hipError_t launch_fft_rows_inv(const FftPlane* planes, int nplanes, int blocks, size_t lds_bytes,
                               hipStream_t s, WorkHeader* work) {
  if (blocks <= 0) return hipSuccess;
  const dim3 g(blocks), b(kFftThreads);
  if (work == nullptr)
    hipLaunchKernelGGL((fft_rows_inv_kernel<false>), g, b, lds_bytes, s, planes, nplanes, work);
  else
    hipLaunchKernelGGL((fft_rows_inv_kernel<true>), g, b, lds_bytes, s, planes, nplanes, work);
  return hipGetLastError();
}

}  // namespace blfls
