// Adaptive-manifold filter on the gradient fields (AMF-LS, Section III-D: the
// filter of Gastal and Oliveira 2012 in place of the bilateral filter of
// Eq. (1)), for gfx950.
//
// The filter approximates a Gaussian bilateral filter of p with range source q
// by splatting every pixel onto a few smooth manifolds eta_k with weight
// psi_k = exp(-(eta_k - q)^2 / sigma_r^2), blurring the splatted (psi p, psi)
// along each manifold, and reading them back with the same weight:
//   r = alpha (sum_k psi_k Bn_k / sum_k psi_k Bd_k - p),  alpha = max_k psi_k.
// The blur is the domain transform's first-order recursive filter
//   y_j = c_j y_{j-1} + (1 - c_j) x_j,  c_j = exp(-sqrt(2) d_j / sigma_s)
// left to right then right to left, along rows then columns, with
// d_j = 1 + (sigma_s sqrt(2) / sigma_r) |eta_j - eta_{j-1}| on a manifold and
// d_j = 1 for the spatial low-passes.  The root manifold is the low-pass of q;
// the two children of a manifold are the low-passes of (w q, w) over the pixels
// below / above it, w = 1 - psi, divided; a child is absent (NaN) where its
// low-passed weight is under tau.  The tree is walked depth first from the
// host, one launch sequence per manifold.
//
// Every recursion is a scan of affine maps y -> c y + (1 - c) x:
//   * rows: one workgroup holds a whole row (all channels and the step
//     coefficients) in LDS; each thread composes the maps of a contiguous
//     chunk, a wave-shuffle scan plus a 4-entry LDS step gives each thread its
//     carry, and the chunk is walked again with it (then the same from the
//     right).  One HBM read and one write per value.
//   * columns: 256 adjacent columns per workgroup (coalesced rows), the height
//     cut into 16-row segments: (0) each segment's composed map, (carry) a
//     fold of the maps down each column (eight threads per column, their
//     shares combined in LDS), (1) the forward scan
//     from the carry plus the backward map of the segment, (carry) the
//     backward fold, (2) both scans again and the consumer: the root manifold,
//     the slice into the running sums (the last slice writes the residual in
//     the field type), or the children manifolds.
#include "blfls_field.h"
#include "blfls_internal.h"
#include "blfls_launch.h"

#include <cmath>

namespace blfls {

namespace {

constexpr int kThreads = 256;
constexpr int kRoot = 0, kSplat = 1, kSplit = 2;

template <int MODE>
struct Chans { static constexpr int n = MODE == kRoot ? 1 : MODE == kSplat ? 2 : 4; };

__host__ __device__ __forceinline__ int pad32(int i) { return i + (i >> 5); }

__device__ __forceinline__ int next_wrap(int i, int n) { return i + 1 == n ? 0 : i + 1; }

// Circular forward difference of image x along the field's axis at (i, j).
__device__ __forceinline__ float grad_at(const float* __restrict__ x, int64_t pitch, int H, int W, int i, int j,
                                         int field) {
  const float v = x[static_cast<int64_t>(i) * pitch + j];
  if (field == 0) return x[static_cast<int64_t>(i) * pitch + next_wrap(j, W)] - v;
  return x[static_cast<int64_t>(next_wrap(i, H)) * pitch + j] - v;
}

// Splat / slice weight of a pixel with range value q on manifold value e (0 where absent).
__device__ __forceinline__ float amf_weight(float e, float q, float inv, float kpsi) {
  if (!(e == e)) return 0.0f;
  const float d = (e - q) * inv;
  return exp2f(-kpsi * d * d);
}

// Step coefficient between manifold samples e0 -> e1 (flat across absent samples).
__device__ __forceinline__ float amf_step(float e1, float e0, const AmfGeom& G, float inv) {
  const float de = (e1 == e1 && e0 == e0) ? fabsf(e1 - e0) * inv : 0.0f;
  return exp2f(G.c0 + G.c1 * de);
}

// Carry into each thread's chunk: the composition of the affine maps
// (A, B) of threads 0..t-1 (in thread order) applied to 0.  sh holds 4 x (1 + N)
// floats; the call ends with every read of sh done by the caller's next barrier.
template <int N>
__device__ __forceinline__ void block_carry(float A, float (&B)[N], float (&carry)[N], float* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const float Ap = __shfl_up(A, d);
    float Bp[N];
#pragma unroll
    for (int c = 0; c < N; ++c) Bp[c] = __shfl_up(B[c], d);
    if (lane >= d) {
#pragma unroll
      for (int c = 0; c < N; ++c) B[c] = fmaf(A, Bp[c], B[c]);
      A *= Ap;
    }
  }
  if (lane == 63) {
    sh[wave * (1 + N)] = A;
#pragma unroll
    for (int c = 0; c < N; ++c) sh[wave * (1 + N) + 1 + c] = B[c];
  }
  __syncthreads();
  float PB[N];
#pragma unroll
  for (int c = 0; c < N; ++c) PB[c] = 0.0f;
  for (int w = 0; w < wave; ++w) {
    const float tA = sh[w * (1 + N)];
#pragma unroll
    for (int c = 0; c < N; ++c) PB[c] = fmaf(tA, PB[c], sh[w * (1 + N) + 1 + c]);
  }
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const float incl = fmaf(A, PB[c], B[c]);
    const float up = __shfl_up(incl, 1);
    carry[c] = lane == 0 ? PB[c] : up;
  }
}

__device__ __forceinline__ size_t plane_size(const AmfGeom& G) { return static_cast<size_t>(G.H) * G.W; }

}  // namespace

// One workgroup per (row, field): the row's recursive filter both ways.
template <int MODE>
__global__ void __launch_bounds__(kThreads) amf_rows_kernel(AmfGeom G) {
  constexpr int N = Chans<MODE>::n;
  constexpr bool STEPS = MODE == kSplat;
  extern __shared__ float lds[];
  __shared__ float sh[4 * (1 + N)];
  const int i = blockIdx.x, p = blockIdx.y;
  const AmfPlane& P = G.planes[p];
  const int H = G.H, W = G.W, Wp = pad32(W - 1) + 1;
  float* v = lds;               // [N][Wp]
  float* al = lds + N * Wp;     // [Wp] step coefficients (manifold blur)
  const float* qimg = P.g ? P.g : P.f;
  const int64_t qp = P.g ? P.gpitch : P.pitch;
  const float inv = G.inv[p];
  const size_t PN = static_cast<size_t>(G.P) * plane_size(G);
  const size_t row = static_cast<size_t>(p) * plane_size(G) + static_cast<size_t>(i) * W;

  for (int j = threadIdx.x; j < W; j += kThreads) {
    const float qv = grad_at(qimg, qp, H, W, i, j, P.field);
    const int jj = pad32(j);
    if constexpr (MODE == kRoot) {
      v[jj] = qv;
    } else {
      const float e = G.eta[row + j];
      const float psi = amf_weight(e, qv, inv, G.kpsi);
      if constexpr (MODE == kSplat) {
        const float pv = grad_at(P.f, P.pitch, H, W, i, j, P.field);
        v[jj] = psi * pv;
        v[Wp + jj] = psi;
        al[jj] = j == 0 ? 0.0f : amf_step(e, G.eta[row + j - 1], G, inv);
      } else {
        const float w = (e == e) ? 1.0f - psi : 0.0f;
        const bool below = qv < e;
        const float wl = below ? w : 0.0f, wh = below ? 0.0f : w;
        v[jj] = wl * qv;
        v[Wp + jj] = wl;
        v[2 * Wp + jj] = wh * qv;
        v[3 * Wp + jj] = wh;
      }
    }
  }
  __syncthreads();

  const int cw = (W + kThreads - 1) / kThreads;
  auto coef = [&](int j) -> float {   // step into j from j - 1; 0 at both ends of the row
    if (j <= 0 || j >= W) return 0.0f;
    if constexpr (STEPS) return al[pad32(j)];
    return G.a;
  };

  // left to right
  {
    const int j0 = min(W, static_cast<int>(threadIdx.x) * cw), j1 = min(W, j0 + cw);
    float A = 1.0f, B[N], carry[N];
#pragma unroll
    for (int c = 0; c < N; ++c) B[c] = 0.0f;
    for (int j = j0; j < j1; ++j) {
      const float k = coef(j);
#pragma unroll
      for (int c = 0; c < N; ++c) B[c] = fmaf(k, B[c] - v[c * Wp + pad32(j)], v[c * Wp + pad32(j)]);
      A *= k;
    }
    block_carry<N>(A, B, carry, sh);
    for (int j = j0; j < j1; ++j) {
      const float k = coef(j);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const float x = v[c * Wp + pad32(j)];
        carry[c] = fmaf(k, carry[c] - x, x);
        v[c * Wp + pad32(j)] = carry[c];
      }
    }
  }
  __syncthreads();
  // right to left: thread t owns chunk 255 - t, so thread order is right-to-left order
  {
    const int k0 = min(W, (kThreads - 1 - static_cast<int>(threadIdx.x)) * cw), k1 = min(W, k0 + cw);
    float A = 1.0f, B[N], carry[N];
#pragma unroll
    for (int c = 0; c < N; ++c) B[c] = 0.0f;
    for (int j = k1 - 1; j >= k0; --j) {
      const float k = coef(j + 1);
#pragma unroll
      for (int c = 0; c < N; ++c) B[c] = fmaf(k, B[c] - v[c * Wp + pad32(j)], v[c * Wp + pad32(j)]);
      A *= k;
    }
    block_carry<N>(A, B, carry, sh);
    for (int j = k1 - 1; j >= k0; --j) {
      const float k = coef(j + 1);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const float x = v[c * Wp + pad32(j)];
        carry[c] = fmaf(k, carry[c] - x, x);
        v[c * Wp + pad32(j)] = carry[c];
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < W; j += kThreads) {
#pragma unroll
    for (int c = 0; c < N; ++c) G.tmp[c * PN + row + j] = v[c * Wp + pad32(j)];
  }
}

// Column scans.  PHASE 0: each segment's composed forward map -> sum.
// PHASE 1: forward scan from carry_f, then the segment's backward map -> sum.
// PHASE 2: both scans from carry_f / carry_b, then the consumer of MODE.
template <int MODE, int PHASE>
__global__ void __launch_bounds__(kThreads) amf_cols_kernel(AmfGeom G) {
  constexpr int N = Chans<MODE>::n;
  constexpr bool STEPS = MODE == kSplat;
  const int j = blockIdx.x * kThreads + threadIdx.x;
  const int s = blockIdx.y, p = blockIdx.z;
  if (j >= G.W) return;
  const int H = G.H, W = G.W, S = G.S;
  const int i0 = s * kAmfSeg, n = min(kAmfSeg, H - i0);
  const size_t HW = plane_size(G), PN = static_cast<size_t>(G.P) * HW;
  const size_t col = static_cast<size_t>(p) * HW + j;
  const float inv = G.inv[p];

  // kk(t): step into row i0 + t from the row above (0 at the image's first row
  // and below its last); t = n is the step into the next segment.  The
  // manifold blur keeps its per-column steps in registers; the low-passes'
  // uniform steps are formed where they are used (an array of them would sit
  // in scalar registers).
  float k[STEPS ? kAmfSeg + 1 : 1];
  float ev[STEPS ? kAmfSeg : 1];
  if constexpr (STEPS) {
    float e_prev = i0 > 0 ? G.eta[col + static_cast<size_t>(i0 - 1) * W] : 0.0f;
#pragma unroll
    for (int t = 0; t <= kAmfSeg; ++t) {
      if (t <= n && i0 + t < H) {
        const float e = G.eta[col + static_cast<size_t>(i0 + t) * W];
        k[t] = i0 + t == 0 ? 0.0f : amf_step(e, e_prev, G, inv);
        if (t < kAmfSeg) ev[t] = e;
        e_prev = e;
      } else {
        k[t] = 0.0f;
        if (t < kAmfSeg) ev[t] = 0.0f;
      }
    }
  }
  auto kk = [&](int t) -> float {
    if constexpr (STEPS) return k[t];
    return (i0 + t == 0 || i0 + t >= H) ? 0.0f : G.a;
  };

  float* sum = G.sum + static_cast<size_t>(p * S + s) * 5 * W + j;
  if constexpr (PHASE == 0) {
    float A = 1.0f, y[N];
#pragma unroll
    for (int c = 0; c < N; ++c) y[c] = 0.0f;
#pragma unroll
    for (int t = 0; t < kAmfSeg; ++t) {
      if (t < n) {
        const size_t idx = col + static_cast<size_t>(i0 + t) * W;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const float x = G.tmp[c * PN + idx];
          y[c] = fmaf(kk(t), y[c] - x, x);
        }
        A *= kk(t);
      }
    }
    sum[0] = A;
#pragma unroll
    for (int c = 0; c < N; ++c) sum[(1 + c) * W] = y[c];
    return;
  } else {
    const float* cf = G.carry_f + static_cast<size_t>(p * S + s) * 4 * W + j;
    float y[N], ys[kAmfSeg][N];
#pragma unroll
    for (int c = 0; c < N; ++c) y[c] = cf[c * W];
#pragma unroll
    for (int t = 0; t < kAmfSeg; ++t) {
      if (t < n) {
        const size_t idx = col + static_cast<size_t>(i0 + t) * W;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const float x = G.tmp[c * PN + idx];
          y[c] = fmaf(kk(t), y[c] - x, x);
          ys[t][c] = y[c];
        }
      }
    }
    if constexpr (PHASE == 1) {
      float A = 1.0f, z[N];
#pragma unroll
      for (int c = 0; c < N; ++c) z[c] = 0.0f;
#pragma unroll
      for (int t = kAmfSeg - 1; t >= 0; --t) {
        if (t < n) {
#pragma unroll
          for (int c = 0; c < N; ++c) z[c] = fmaf(kk(t + 1), z[c] - ys[t][c], ys[t][c]);
          A *= kk(t + 1);
        }
      }
      sum[0] = A;
#pragma unroll
      for (int c = 0; c < N; ++c) sum[(1 + c) * W] = z[c];
    } else {
      const float* cb = G.carry_b + static_cast<size_t>(p * S + s) * 4 * W + j;
      const AmfPlane& P = G.planes[p];
      float z[N];
#pragma unroll
      for (int c = 0; c < N; ++c) z[c] = cb[c * W];
#pragma unroll
      for (int t = kAmfSeg - 1; t >= 0; --t) {
        if (t < n) {
#pragma unroll
          for (int c = 0; c < N; ++c) z[c] = fmaf(kk(t + 1), z[c] - ys[t][c], ys[t][c]);
          const int i = i0 + t;
          const size_t idx = col + static_cast<size_t>(i) * W;
          if constexpr (MODE == kRoot) {
            G.eta_out[idx] = z[0];
          } else if constexpr (MODE == kSplit) {
            G.eta_out[idx] = z[1] >= G.tau ? z[0] / z[1] : __builtin_nanf("");
            G.eta_out[PN + idx] = z[3] >= G.tau ? z[2] / z[3] : __builtin_nanf("");
          } else {
            const float* qimg = P.g ? P.g : P.f;
            const int64_t qp = P.g ? P.gpitch : P.pitch;
            const float qv = grad_at(qimg, qp, H, W, i, j, P.field);
            const float psi = amf_weight(ev[t], qv, inv, G.kpsi);
            float num = psi * z[0], den = psi * z[1], amax = psi;
            if (!G.first) {
              num = fmaf(psi, z[0], G.acc[idx]);
              den = fmaf(psi, z[1], G.acc[PN + idx]);
              amax = fmaxf(G.acc[2 * PN + idx], psi);
            }
            if (G.last) {
              const float pv = grad_at(P.f, P.pitch, H, W, i, j, P.field);
              const float r = den > 0.0f ? amax * (num / den - pv) : 0.0f;
              store_field(P.out, static_cast<int64_t>(i) * W + j, r * G.inv[G.P + p], G.ft);
            } else {
              G.acc[idx] = num;
              G.acc[PN + idx] = den;
              G.acc[2 * PN + idx] = amax;
            }
          }
        }
      }
    }
  }
}

// Fold the segment maps of each column into the carry entering every segment.
// A workgroup takes 32 adjacent columns (coalesced rows of the map arrays)
// and splits each column's segments, in scan order, over 8 threads: each
// composes its share, the shares' compositions are combined in LDS, and each
// thread walks its share again from its carry, writing the carries.
constexpr int kCarryCols = 32;
constexpr int kCarryGroups = kThreads / kCarryCols;   // 8

template <int N, bool BACKWARD>
__global__ void __launch_bounds__(kThreads) amf_carry_kernel(AmfGeom G) {
  __shared__ float tot[kCarryGroups][1 + N][kCarryCols];
  const int jj = threadIdx.x % kCarryCols, g = threadIdx.x / kCarryCols;
  const int j = blockIdx.x * kCarryCols + jj, p = blockIdx.y;
  const bool live = j < G.W;
  const int S = G.S, W = G.W;
  const int share = (S + kCarryGroups - 1) / kCarryGroups;
  const int q0 = min(S, g * share), q1 = min(S, q0 + share);   // scan positions of this thread
  const float* __restrict__ sum = G.sum;
  float* __restrict__ carry = BACKWARD ? G.carry_b : G.carry_f;
  auto seg = [&](int q) { return BACKWARD ? S - 1 - q : q; };
  // composition of this thread's share
  float A = 1.0f, B[N];
#pragma unroll
  for (int c = 0; c < N; ++c) B[c] = 0.0f;
  if (live) {
#pragma unroll 4
    for (int q = q0; q < q1; ++q) {
      const float* sm = sum + static_cast<size_t>(p * S + seg(q)) * 5 * W + j;
      const float a = sm[0];
#pragma unroll
      for (int c = 0; c < N; ++c) B[c] = fmaf(a, B[c], sm[(1 + c) * W]);
      A *= a;
    }
  }
  tot[g][0][jj] = A;
#pragma unroll
  for (int c = 0; c < N; ++c) tot[g][1 + c][jj] = B[c];
  __syncthreads();
  if (!live) return;
  // carry into the share: the shares before it, in scan order, applied to 0
  float y[N];
#pragma unroll
  for (int c = 0; c < N; ++c) y[c] = 0.0f;
  for (int h = 0; h < g; ++h) {
    const float a = tot[h][0][jj];
#pragma unroll
    for (int c = 0; c < N; ++c) y[c] = fmaf(a, y[c], tot[h][1 + c][jj]);
  }
#pragma unroll 4
  for (int q = q0; q < q1; ++q) {
    const size_t at = static_cast<size_t>(p * S + seg(q));
    const float* sm = sum + at * 5 * W + j;
    float* cr = carry + at * 4 * W + j;
    const float a = sm[0];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      cr[c * W] = y[c];
      y[c] = fmaf(a, y[c], sm[(1 + c) * W]);
    }
  }
}

// Range scale of each field: 1/span of its range source with the normalise
// flag; and its FP16 store scale (1 for FP32 and BF16 fields).
__global__ void __launch_bounds__(64) amf_prep_kernel(AmfGeom G) {
  const AmfPlane& P = G.planes[blockIdx.x];
  float inv = 1.0f;
  if (P.minmax != nullptr) {
    const float span = field_span(P.minmax, P.field);
    if (span > 0.0f) inv = __fdiv_rn(1.0f, span);
  }
  const float2 fsc = field_store_scales(P.fmm);
  if (threadIdx.x == 0) {
    G.inv[blockIdx.x] = inv;
    G.inv[G.P + blockIdx.x] = P.field ? fsc.y : fsc.x;
  }
}

namespace {

size_t rows_lds(int mode, int W) {
  const int n = mode == kRoot ? 1 : mode == kSplat ? 3 : 4;   // channels (+ coefficients)
  return static_cast<size_t>(n) * (pad32(W - 1) + 1) * sizeof(float);
}

template <int MODE>
hipError_t launch_rows(const AmfGeom& G, hipStream_t s) {
  hipLaunchKernelGGL(amf_rows_kernel<MODE>, dim3(G.H, G.P), dim3(kThreads), rows_lds(MODE, G.W), s, G);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_cols(const AmfGeom& G, hipStream_t s) {
  constexpr int N = Chans<MODE>::n;
  const dim3 seg((G.W + kThreads - 1) / kThreads, G.S, G.P);
  const dim3 lines((G.W + kCarryCols - 1) / kCarryCols, G.P);
  hipLaunchKernelGGL((amf_cols_kernel<MODE, 0>), seg, dim3(kThreads), 0, s, G);
  hipLaunchKernelGGL((amf_carry_kernel<N, false>), lines, dim3(kThreads), 0, s, G);
  hipLaunchKernelGGL((amf_cols_kernel<MODE, 1>), seg, dim3(kThreads), 0, s, G);
  hipLaunchKernelGGL((amf_carry_kernel<N, true>), lines, dim3(kThreads), 0, s, G);
  hipLaunchKernelGGL((amf_cols_kernel<MODE, 2>), seg, dim3(kThreads), 0, s, G);
  return hipGetLastError();
}

struct Walk {
  AmfGeom G;
  float* slots;
  size_t PN;
  int height, visited, count;
  hipStream_t s;

  float* slot(int k) const { return slots + static_cast<size_t>(k) * PN; }

  // Splat, blur and slice manifold `k` of tree level `level`, then split it
  // and visit its children (below first).
  hipError_t visit(int level, int k) {
    G.eta = slot(k);
    G.first = visited == 0;
    G.last = visited == count - 1;
    ++visited;
    hipError_t e = launch_rows<kSplat>(G, s);
    if (e == hipSuccess) e = launch_cols<kSplat>(G, s);
    if (e != hipSuccess || level >= height) return e;
    const int child = 1 + 2 * (level - 1);   // the slot pair of level + 1
    G.eta = slot(k);
    G.eta_out = slot(child);
    e = launch_rows<kSplit>(G, s);
    if (e == hipSuccess) e = launch_cols<kSplit>(G, s);
    if (e == hipSuccess) e = visit(level + 1, child);
    if (e == hipSuccess) e = visit(level + 1, child + 1);
    return e;
  }
};

}  // namespace

int amf_slots(int height) { return 2 * height - 1; }

int amf_segments(int H) { return (H + kAmfSeg - 1) / kAmfSeg; }

hipError_t amf_init_kernels() {
  // a row of up to 8192 values in 4 channels (or 2 channels and the steps), padded
  const int kMax = static_cast<int>(rows_lds(kSplit, 8192));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amf_rows_kernel<kRoot>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kMax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amf_rows_kernel<kSplat>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amf_rows_kernel<kSplit>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMax);
  return e;
}

hipError_t launch_amf(const AmfGeom& geom, float* slots, int height, hipStream_t s) {
  if (geom.P <= 0 || height < 1 || height > kAmfMaxHeight) return hipErrorInvalidValue;
  if (geom.W > 8192 || geom.S != amf_segments(geom.H)) return hipErrorInvalidValue;
  Walk w{geom, slots, static_cast<size_t>(geom.P) * geom.H * geom.W, height, 0, (1 << height) - 1, s};
  hipLaunchKernelGGL(amf_prep_kernel, dim3(geom.P), dim3(64), 0, s, geom);
  hipError_t e = hipGetLastError();
  // root manifold: the low-pass of the range source
  w.G.eta = nullptr;
  w.G.eta_out = w.slot(0);
  if (e == hipSuccess) e = launch_rows<kRoot>(w.G, s);
  if (e == hipSuccess) e = launch_cols<kRoot>(w.G, s);
  if (e == hipSuccess) e = w.visit(1, 0);
  return e;
}

}  // namespace blfls
