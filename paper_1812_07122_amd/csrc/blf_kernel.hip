// Exact windowed bilateral filter on the gradient fields (Eq. (1) applied to
// D_x f and D_y f, Section III-A), for gfx950.
//
// One workgroup filters ONE gradient field over one 64 x (WAVES*K) tile:
//   * the tile plus an R-pixel halo of the field (and of its range source in
//     joint mode) is built in LDS from the image with circular wrap;
//   * lane l of wave w owns image column x0+l and the K rows
//     y0+w*K .. y0+w*K+K-1 (a vertical register strip), so one LDS read of a
//     window row serves up to K outputs and the 64 lanes of a wave read 64
//     consecutive LDS words (no bank conflicts);
//   * the window column offset dx is a runtime loop over [-r, r]; the row
//     offsets are unrolled over [-R, R] for the kernel's radius class R, with
//     rows beyond r weighted exactly 0 (log2 weight -inf);
//   * per tap: d = q_t - q_s (range values prescaled by sqrt(log2 e/(2 s_r^2))),
//     w = exp2(sy[dy] - d*d), accumulate w*value and w.  The spatial weight is
//     separable: the row part sits in the exponent, the column part 2^sx[dx]
//     scales each column's partial sums, so the tap costs one v_exp_f32 and
//     four VALU operations;
//   * the output is the residual r = BLF(p) - p, which keeps 16-bit storage
//     small away from edges and lets the solve run in residual form.
//
// Self-guided fields keep only q = c*p in LDS: sum w*d / (c sum w) is the
// residual directly.  Joint fields (guide image, rolling guidance, or range
// kernel off) keep p and q and form sum w*p / sum w - p_s.
#include "blfls_field.h"
#include "blfls_internal.h"
#include "blfls_launch.h"
#include "blfls_work.h"

namespace blfls {

namespace {

__device__ __forceinline__ int wrap_index(int v, int n) {
  int m = v % n;
  return m < 0 ? m + n : m;
}

// Logical item of a direct launch's workgroup such that consecutive items run on
// one XCD (workgroups go round-robin over the 8 XCDs, each with its own L2): the
// two fields of a tile and neighbouring tiles, which read overlapping halo rows,
// then meet in one L2.
__device__ __forceinline__ int xcd_item(int b, int nblk) {
  constexpr int kXcd = 8;
  const int q = nblk / kXcd, rem = nblk % kXcd;
  const int x = b % kXcd;
  return x * q + min(x, rem) + b / kXcd;
}

__device__ __forceinline__ int find_plane(const BlfPlane* planes, int nplanes, int item) {
  // items of plane p: [2*tile_begin, 2*(tile_begin+tile_count))
  int lo = 0, hi = nplanes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (2 * planes[mid].tile_begin <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace

// One work item: one gradient field of one tile of one plane.
template <int R, int K, int WAVES, bool JOINT>
__device__ __forceinline__ void blf_item(const BlfPlane* __restrict__ planes, int nplanes, int field_type,
                                         int item) {
  constexpr int TW = 64;
  constexpr int TH = WAVES * K;
  constexpr int LW = TW + 2 * R;
  constexpr int LH = TH + 2 * R;
  constexpr int T = 64 * WAVES;
  __shared__ float q_lds[LH * LW];
  __shared__ float p_lds[JOINT ? LH * LW : 1];
  __shared__ int rowmap[LH + 1];
  __shared__ int colmap[LW + 1];
  __shared__ float ex_lds[2 * R + 1];

  const int pi = find_plane(planes, nplanes, item);
  const BlfPlane& P = planes[pi];
  const int local = item - 2 * P.tile_begin;
  if (local >= 2 * P.tile_count) return;  // uniform: more items than work
  // the two fields of a tile are consecutive items: they read the same halo tile
  const int field = local & 1;
  const int tile = local >> 1;
  const int H = P.H, W = P.W;
  const int x0 = (tile % P.tiles_x) * TW;
  const int y0 = (tile / P.tiles_x) * TH;
  const int tid = threadIdx.x;

  float c = field ? P.cy : P.cx;
  if (P.minmax != nullptr && c != 0.0f) {
    const float span = field_span(P.minmax, field);
    if (span > 0.0f) c = c / span;
  }
  // FP16 fields: the residual's power-of-two store scale (1 otherwise)
  const float2 fsc = field_store_scales(P.fmm);
  const float ssc = field ? fsc.y : fsc.x;

  // circular index maps of the halo tile (one extra row/column for the differences)
  for (int a = tid; a < LH + 1; a += T) rowmap[a] = wrap_index(y0 - R + a, H);
  for (int b = tid; b < LW + 1; b += T) colmap[b] = wrap_index(x0 - R + b, W);
  // column weights in LDS: the dx loop reads them without a memory round trip
  if (tid < 2 * R + 1) ex_lds[tid] = P.spatial[kSpan + kMaxR - R + tid];
  __syncthreads();

  const float* __restrict__ f = P.f;
  const float* __restrict__ g = P.g ? P.g : P.f;
  const int64_t pitch = P.pitch;
  const int64_t gpitch = P.g ? P.gpitch : P.pitch;
  // gradients of the halo tile; each thread issues kFill element loads before
  // writing any of them to LDS, so one memory round trip covers kFill elements
  constexpr int kFill = 4;
  for (int base = tid; base < LH * LW; base += T * kFill) {
    float f0[kFill], f1[kFill], g0[kFill], g1[kFill];
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const int idx = base + u * T;
      if (idx < LH * LW) {
        const int a = idx / LW;
        const int b = idx - a * LW;
        const int ra = rowmap[a];
        const int c0 = colmap[b];
        // neighbour along the field's axis
        const int rn = field ? rowmap[a + 1] : ra;
        const int c1 = field ? c0 : colmap[b + 1];
        f0[u] = f[ra * pitch + c0];
        f1[u] = f[rn * pitch + c1];
        if (JOINT) {
          g0[u] = g[ra * gpitch + c0];
          g1[u] = g[rn * gpitch + c1];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const int idx = base + u * T;
      if (idx < LH * LW) {
        const float pv = f1[u] - f0[u];
        if (JOINT) {
          p_lds[idx] = pv;
          q_lds[idx] = c * (g1[u] - g0[u]);
        } else {
          q_lds[idx] = c * pv;
        }
      }
    }
  }
  __syncthreads();

  const int lane = tid & 63;
  const int row0 = (tid >> 6) * K;
  const float* __restrict__ spatial = P.spatial;

  // row weights are uniform over the workgroup: held in scalar registers
  float sy[2 * R + 1];
#pragma unroll
  for (int i = 0; i < 2 * R + 1; ++i)
    sy[i] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(spatial[kMaxR - R + i])));

  float qs[K], ps[K], acc_n[K], acc_d[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int o = (row0 + k + R) * LW + lane + R;
    qs[k] = q_lds[o];
    ps[k] = JOINT ? p_lds[o] : 0.0f;
    acc_n[k] = 0.0f;
    acc_d[k] = 0.0f;
  }

  const int r = P.r;
  for (int dx = -r; dx <= r; ++dx) {
    const int col = lane + R + dx;
    float tn[K], td[K];
#pragma unroll
    for (int t = 0; t < K + 2 * R; ++t) {
      const float v = q_lds[(row0 + t) * LW + col];
      const float pv = JOINT ? p_lds[(row0 + t) * LW + col] : 0.0f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int dy = t - k - R;
        if (dy < -R || dy > R) continue;
        const float d = v - qs[k];
        const float w = __builtin_amdgcn_exp2f(fmaf(-d, d, sy[dy + R]));
        const float val = JOINT ? pv : d;
        if (dy == -R) {
          tn[k] = w * val;
          td[k] = w;
        } else {
          tn[k] = fmaf(w, val, tn[k]);
          td[k] += w;
        }
      }
    }
    const float e = ex_lds[dx + R];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      acc_n[k] = fmaf(e, tn[k], acc_n[k]);
      acc_d[k] = fmaf(e, td[k], acc_d[k]);
    }
  }

  void* out = field ? P.ry : P.rx;
  const int x = x0 + lane;
  if (x < W) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int y = y0 + row0 + k;
      if (y < H) {
        // the centre tap has weight exactly 1, so acc_d >= 1
        const float res = JOINT ? acc_n[k] / acc_d[k] - ps[k] : acc_n[k] / (c * acc_d[k]);
        store_field(out, static_cast<int64_t>(y) * W + x, res * ssc, field_type);
      }
    }
  }
}

// Kernel (two instantiations, each with its own register allocation): direct,
// the grid has exactly one workgroup per item;
// otherwise (persistent launch from a captured graph) the work header in
// device memory gives the items and the plane array, and the workgroups of a
// fixed grid draw items from its counter.
template <int R, int K, int WAVES, bool JOINT, bool PERSIST>
__global__ void __launch_bounds__(64 * WAVES)
blf_field_kernel(const BlfPlane* __restrict__ planes, int nplanes, int field_type,
                 WorkHeader* __restrict__ work) {
  if (!PERSIST) {
    blf_item<R, K, WAVES, JOINT>(planes, nplanes, field_type, xcd_item(blockIdx.x, gridDim.x));
    return;
  }
  const int total = work->items;
  const int np = work->nplanes;
  const BlfPlane* pl = static_cast<const BlfPlane*>(work->planes);
  for (;;) {
    const int item = grab_item(work->next[0], total, false);
    if (item >= total) break;
    blf_item<R, K, WAVES, JOINT>(pl, np, field_type, item);
    __syncthreads();  // the next item refills the LDS tile
  }
}

// ---------------------------------------------------------------------------
// Launch: radius classes and tile shape
// ---------------------------------------------------------------------------

namespace {
constexpr int kK = 8;
constexpr int kWaves = 4;
constexpr int kRadii[] = {1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 14, 16, 20, 24, 28, 32};

template <int R>
hipError_t launch_r(const BlfPlane* planes, int nplanes, int total_items, bool joint, int ft, WorkHeader* work,
                    hipStream_t s) {
  dim3 grid(total_items), block(64 * kWaves);
  if (work == nullptr) {
    if (joint)
      hipLaunchKernelGGL((blf_field_kernel<R, kK, kWaves, true, false>), grid, block, 0, s, planes, nplanes, ft, work);
    else
      hipLaunchKernelGGL((blf_field_kernel<R, kK, kWaves, false, false>), grid, block, 0, s, planes, nplanes, ft, work);
  } else {
    if (joint)
      hipLaunchKernelGGL((blf_field_kernel<R, kK, kWaves, true, true>), grid, block, 0, s, planes, nplanes, ft, work);
    else
      hipLaunchKernelGGL((blf_field_kernel<R, kK, kWaves, false, true>), grid, block, 0, s, planes, nplanes, ft, work);
  }
  return hipGetLastError();
}
}  // namespace

int blf_radius_class(int r) {
  for (int R : kRadii)
    if (R >= r) return R;
  return -1;
}

int blf_tile_w() { return 64; }
int blf_tile_h() { return kK * kWaves; }

hipError_t launch_blf(int R, const BlfPlane* planes, int nplanes, int total_items, bool joint,
                      int field_type, hipStream_t s, WorkHeader* work) {
  if (total_items <= 0) return hipSuccess;
  switch (R) {
#define BLFLS_CASE(RR) case RR: return launch_r<RR>(planes, nplanes, total_items, joint, field_type, work, s);
    BLFLS_CASE(1) BLFLS_CASE(2) BLFLS_CASE(3) BLFLS_CASE(4) BLFLS_CASE(5) BLFLS_CASE(6)
    BLFLS_CASE(8) BLFLS_CASE(9) BLFLS_CASE(10) BLFLS_CASE(12) BLFLS_CASE(14) BLFLS_CASE(16)
    BLFLS_CASE(20) BLFLS_CASE(24) BLFLS_CASE(28) BLFLS_CASE(32)
#undef BLFLS_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace blfls
