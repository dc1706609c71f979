// Exact windowed bilateral filter on the gradient fields (Eq. (1) on D_x f and
// D_y f, Section III-A) with one exponential per UNORDERED pair of taps, for gfx950.
//
// The weight of Eq. (1) is symmetric for self- and joint-guided fields: the
// spatial term depends on |d| and the range term on (q(s+d) - q(s))^2, so
// w(s, s+d) = w(s+d, s).  Every unordered pair {s, t} is evaluated once, for the
// offset d = t - s in the half-plane {dy > 0} u {dy = 0, dx > 0}, and its weight
// enters the sums of both pixels.
//
// Work split.  The image is cut into bands of at most 64 columns and whole
// blocks of K rows (8 for R = 8, 9; 4 from R = 10); one wave sweeps a band block by block.  A pair is
// evaluated by the band that holds the column of its partner t and the block
// that holds the row of its source s.  Lane l owns image column x0+l:
//   * its partner sums A[j] (rows y..y+K+R-1 of its own column) stay in
//     registers: rows below the block carry over to the next blocks, rows past
//     the band are written out as the next row band's share;
//   * the source sums B[k] (rows y..y+K-1) travel: for column offset dx > 0 the
//     source sits dx columns left of the partner, and stepping dx = r, ..., 1
//     with a one-lane DPP wave shift per step keeps every B on the lane that
//     meets its next partner column; for dx < 0 the same to the right;
//   * a B that leaves the wave belongs to a pixel of the neighbouring band: one
//     lane stores it (K pairs of floats) and the merge pass adds it there.
// One exp, one VOP3 FMA and five VOP2 operations per pair, against one exp and
// four VALU operations per tap for the tile kernel (two taps per pair).
//
// Merge pass: per pixel, its band's sums, the row band above's carry-over rows,
// and the right and left neighbours' travelling sums, in a fixed order; then
// the centre tap and the residual r = BLF(p) - p in the field type.
//
// Self-guided fields keep q = c*p: the partner sum is sum w (q_s - q_t), and the
// source sums hold the negated sums (both are e * (q_s - q_t)); joint fields sum
// w * p of the other pixel on both sides.
#include <algorithm>
#include <type_traits>

#include "blfls_field.h"
#include "blfls_internal.h"
#include "blfls_launch.h"
#include "blfls_work.h"

namespace blfls {

namespace {

static_assert(kPairMaxR == kMaxR && kPairBandCols == 64, "pair classes and wave width");

constexpr float kHuge = 1e30f;   // range value of a source row / partner lane outside the band: weight 0
constexpr int kMergeSeg = kPairMergeSeg;  // columns per merge item
constexpr int kMergeThreads = 256;

__device__ __forceinline__ int wrap_i(int v, int n) {
  int m = v % n;
  return m < 0 ? m + n : m;
}

// Workgroup order of a direct launch such that consecutive items (neighbouring
// bands, which read overlapping halo columns) run on one XCD.
__device__ __forceinline__ int xcd_order(int b, int nblk) {
  constexpr int kXcd = 8;
  const int q = nblk / kXcd, rem = nblk % kXcd;
  const int x = b % kXcd;
  return x * q + min(x, rem) + b / kXcd;
}

__device__ __forceinline__ int plane_of_band(const BlfPlane* planes, int nplanes, int item) {
  int lo = 0, hi = nplanes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (2 * planes[mid].tile_begin <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int plane_of_merge(const BlfPlane* planes, int nplanes, int item) {
  int lo = 0, hi = nplanes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (2 * planes[mid].merge_begin <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) f2v g_f2v;
typedef __attribute__((address_space(1))) f4v g_f4v;

__device__ __forceinline__ void store2(float2* base, int64_t idx, float a, float b) {
  ((g_f2v*)base)[idx] = f2v{a, b};
}
// Accesses at a 32-bit byte offset from a uniform base (images and records stay
// under 4 GiB): scalar base + vector offset, no 64-bit per-lane address to keep.
__device__ __forceinline__ float load_at(const float* base, uint32_t byte_off) {
  typedef __attribute__((address_space(1))) const char g_cchar;
  return *(const __attribute__((address_space(1))) float*)((g_cchar*)base + byte_off);
}
__device__ __forceinline__ void store2_at(float2* base, uint32_t byte_off, float a, float b) {
  typedef __attribute__((address_space(1))) char g_char;
  *(g_f2v*)((g_char*)base + byte_off) = f2v{a, b};
}
__device__ __forceinline__ void store4(float2* base, int64_t idx2, float a, float b, float c, float d) {
  ((g_f4v*)(base + idx2))[0] = f4v{a, b, c, d};
}
__device__ __forceinline__ f2v load2(const float2* base, int64_t idx) {
  return ((const g_f2v*)base)[idx];
}

// DPP wave shifts by one lane (lanes shifted in read 0).
__device__ __forceinline__ float lanes_down(float v) {  // lane i <- lane i + 1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float lanes_up(float v) {    // lane i <- lane i - 1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

// Band geometry (identical on host and device): column band bx covers
// [bx W / nbx, (bx+1) W / nbx); row band by covers blocks [by T / nby, (by+1) T / nby)
// of T = ceil(H / K) blocks, rows clipped at H.
struct Band {
  int x0, wb, Y0, Y1, nblk;
};
__device__ __forceinline__ Band band_of(const BlfPlane& P, int bx, int by) {
  const int K = P.pair_k;
  const int T = (P.H + K - 1) / K;
  Band b;
  b.x0 = pair_band_x0(P.W, P.nbx, bx);
  b.wb = pair_band_x0(P.W, P.nbx, bx + 1) - b.x0;
  const int blk0 = pair_band_first_block(T, P.nby, by);
  b.nblk = pair_band_first_block(T, P.nby, by + 1) - blk0;
  b.Y0 = blk0 * K;
  b.Y1 = min(P.H, b.Y0 + b.nblk * K);
  return b;
}

// main region of band (bx, by): [max_nblk K + R][64] float2; the sums that left
// band (bx, by) through lane 0 (dir 0, sources in the band to the left) or the
// last lane (dir 1): [max_nblk][R][K] float2 (layout in blfls_pair_geom.h)
__device__ __forceinline__ int64_t main_off(const BlfPlane& P, int bx, int by) {
  return pair_main_off(P.nbx, P.max_nblk, P.pair_k, P.pair_r, bx, by);
}
__device__ __forceinline__ int64_t ovf_off(const BlfPlane& P, int bx, int by, int dir) {
  return pair_edge_off(P.nbx, P.nby, P.max_nblk, P.pair_k, P.pair_r, bx, by, dir);
}

// Range scale of a field: c = sqrt(log2 e / (2 sigma_r^2)), divided by the
// range source's span when normalising (block-wide).
__device__ __forceinline__ float field_range_scale(const BlfPlane& P, int field) {
  float c = field ? P.cy : P.cx;
  if (P.minmax != nullptr && c != 0.0f) {
    const float span = field_span(P.minmax, field);
    if (span > 0.0f) c = c / span;
  }
  return c;
}

}  // namespace

// One band of one field: the wave sweeps the band's blocks.
template <int R, bool JOINT>
__device__ __forceinline__ void pair_item(const BlfPlane* __restrict__ planes, int nplanes, int item) {
  constexpr int K = pair_block_rows(R);
  constexpr int LW = 64 + 2 * R;   // source columns x0-R .. x0+64+R-1
  constexpr int NJ = K + R;        // partner rows y .. y+K+R-1
  constexpr int kFill = 4;
  __shared__ float wq[K * LW];
  __shared__ float wp[JOINT ? K * LW : 1];
  __shared__ int colmap[LW + 1];
  __shared__ float pw_lds[(R + 1) * (R + 1)];

  const int pi = plane_of_band(planes, nplanes, item);
  const BlfPlane& P = planes[pi];
  const int local = item - 2 * P.tile_begin;
  if (local >= 2 * P.tile_count) return;  // uniform
  const int field = local & 1;
  const int band = local >> 1;
  const int bx = band % P.nbx, by = band / P.nbx;
  const Band G = band_of(P, bx, by);
  const int H = P.H, W = P.W;
  const int lane = threadIdx.x;
  const float c = field_range_scale(P, field);

  const float* __restrict__ f = P.f;
  const float* __restrict__ g = P.g ? P.g : P.f;
  const int64_t pitch = P.pitch;
  const int64_t gpitch = P.g ? P.gpitch : P.pitch;
  float2* __restrict__ rec = P.rec + field * P.rec_field;
  float2* __restrict__ rmain = rec + main_off(P, bx, by);
  float2* __restrict__ rleft = rec + ovf_off(P, bx, by, 0);
  float2* __restrict__ rright = rec + ovf_off(P, bx, by, 1);

  for (int a = lane; a < LW + 1; a += 64) colmap[a] = wrap_i(G.x0 - R + a, W);

  // log2 spatial weights pw[dx][dy] = -(dx^2 + dy^2) log2(e) / (2 sigma_s^2) of
  // the request (-inf beyond r), in LDS: each row offset's exponent addend is
  // one broadcast LDS read instead of a VALU add
  {
    const float* __restrict__ pw =
        P.spatial + (offsetof(RequestTables, pw) - offsetof(RequestTables, sy)) / sizeof(float);
    for (int i = lane; i < (R + 1) * (R + 1); i += 64) pw_lds[i] = pw[(i / (R + 1)) * (kMaxR + 1) + i % (R + 1)];
  }

  const bool lane_ok = lane < G.wb;
  const int xo = G.x0 + (lane_ok ? lane : 0);
  const int xn = field ? xo : (xo + 1 == W ? 0 : xo + 1);
  // forward difference along the field's axis at (row, own column); row in [0, H)
  auto grad_own = [&](const float* img, int64_t pit, int row) -> float {
    const int rn = field ? (row + 1 == H ? 0 : row + 1) : row;
    const uint32_t p32 = static_cast<uint32_t>(pit);
    return load_at(img, (rn * p32 + xn) * 4u) - load_at(img, (row * p32 + xo) * 4u);
  };

  float an[NJ], ad[NJ], vq[NJ], vp[JOINT ? NJ : 1];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    an[j] = 0.0f;
    ad[j] = 0.0f;
    vq[j] = 0.0f;
    if (JOINT) vp[j] = 0.0f;
  }
  // partner values: shift the rows down by K and read K new rows into the top
  // (rows base..base+K-1); the prologue runs it until all NJ rows are in
  auto advance_v = [&](int base) {
#pragma unroll
    for (int i = 0; i + K < NJ; ++i) {
      vq[i] = vq[i + K];
      if (JOINT) vp[i] = vp[i + K];
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int row = wrap_i(base + i, H);
      const float gq = grad_own(g, gpitch, row);
      vq[NJ - K + i] = lane_ok ? c * gq : -kHuge;
      if (JOINT) vp[NJ - K + i] = lane_ok ? grad_own(f, pitch, row) : 0.0f;
    }
  };
  constexpr int kPre = (NJ + K - 1) / K;
  for (int it = 0; it < kPre; ++it) advance_v(G.Y0 + NJ - K - (kPre - 1 - it) * K);

  const int r = P.r;
  for (int b = 0; b < G.nblk; ++b) {
    const int y = G.Y0 + b * K;
    // source window: rows y..y+K-1 (rows past the band: weight 0), LW columns
    __syncthreads();
    for (int base = lane; base < K * LW; base += 64 * kFill) {
      float q0[kFill], q1[kFill], p0[kFill], p1[kFill];
#pragma unroll
      for (int u = 0; u < kFill; ++u) {
        const int idx = base + u * 64;
        const int k = idx / LW;
        const int cc = idx - k * LW;
        const int row = y + k;
        if (idx < K * LW && row < G.Y1) {
          const int c0 = colmap[cc];
          const int rn = field ? (row + 1 == H ? 0 : row + 1) : row;
          const int cn = field ? c0 : colmap[cc + 1];
          const uint32_t gp32 = static_cast<uint32_t>(gpitch), fp32 = static_cast<uint32_t>(pitch);
          q0[u] = load_at(g, (row * gp32 + c0) * 4u);
          q1[u] = load_at(g, (rn * gp32 + cn) * 4u);
          if (JOINT) {
            p0[u] = load_at(f, (row * fp32 + c0) * 4u);
            p1[u] = load_at(f, (rn * fp32 + cn) * 4u);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kFill; ++u) {
        const int idx = base + u * 64;
        if (idx < K * LW) {
          const bool ok = y + idx / LW < G.Y1;
          wq[idx] = ok ? c * (q1[u] - q0[u]) : kHuge;
          if (JOINT) wp[idx] = ok ? p1[u] - p0[u] : 0.0f;
        }
      }
    }
    __syncthreads();

    float bn[K], bd[K];
    // The pairs of one step (source row k, partner row k + dy) for dy = dy0..R,
    // software pipelined: each pair's exp is issued before the previous pair's
    // four sums, so the transcendental unit works beside the VALU, and the next
    // row offset's spatial term is read from LDS one group ahead.  Scheduling
    // barriers keep this order (left to itself the scheduler groups the exps).
    auto step_pairs = [&](const float (&sq)[K], const float (&sp)[K], const float* S, int dy0) {
      float dprev = 0.0f, eprev = 0.0f;
      float s_cur = S[dy0];
#pragma unroll
      for (int dy = dy0; dy <= R + 1; ++dy) {
        const float s_next = dy + 1 <= R ? S[dy + 1] : 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (dy == R + 1 && k > 0) break;
          float d = 0.0f, e = 0.0f;
          if (dy <= R) {
            d = sq[k] - vq[k + dy];
            e = __builtin_amdgcn_exp2f(fmaf(-d, d, s_cur));
          }
          // the previous pair: (dy, k - 1), or (dy - 1, K - 1)
          const int pdy = k > 0 ? dy : dy - 1;
          const int pk = k > 0 ? k - 1 : K - 1;
          if (pdy >= dy0) {
            const int j = pk + pdy;
            if (JOINT) {
              an[j] = fmaf(eprev, sp[pk], an[j]);
              bn[pk] = fmaf(eprev, vp[j], bn[pk]);
            } else {
              an[j] = fmaf(eprev, dprev, an[j]);
              bn[pk] = fmaf(eprev, dprev, bn[pk]);
            }
            ad[j] += eprev;
            bd[pk] += eprev;
          }
          dprev = d;
          eprev = e;
          __builtin_amdgcn_sched_barrier(0);
        }
        s_cur = s_next;
      }
    };
    auto merge_b = [&]() {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        an[k] = JOINT ? an[k] + bn[k] : an[k] - bn[k];
        ad[k] += bd[k];
      }
    };

    // dx > 0, dy >= 0: the source is dx columns left of the partner.  Each
    // step's sums leave lane 0 and shift at the top of the next step (nothing
    // but the loop latch follows the pairs, so they are not sunk past a branch).
    auto leave_left = [&](int dxp) {
      if (lane == 0) {
        // sources of column x0 - dxp: the band to the left
        float2* o = rleft + (static_cast<int64_t>(b) * R + (dxp - 1)) * K;
#pragma unroll
        for (int k = 0; k < K; k += 2) store4(o, k, bn[k], bd[k], bn[k + 1], bd[k + 1]);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        bn[k] = lanes_down(bn[k]);
        bd[k] = lanes_down(bd[k]);
      }
    };
#pragma unroll
    for (int k = 0; k < K; ++k) { bn[k] = 0.0f; bd[k] = 0.0f; }
    for (int dx = r; dx >= 1; --dx) {
      if (dx < r) leave_left(dx + 1);
      const float* S = pw_lds + dx * (R + 1);
      float sq[K], sp[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        sq[k] = wq[k * LW + R + lane - dx];
        sp[k] = JOINT ? wp[k * LW + R + lane - dx] : 0.0f;
      }
      step_pairs(sq, sp, S, 0);
    }
    if (r >= 1) leave_left(1);
    merge_b();

    // dx < 0, dy > 0: the source is |dx| columns right of the partner
    auto leave_right = [&](int mp) {
      if (lane == G.wb - 1) {
        // sources of column x0 + wb - 1 + mp: the band to the right
        float2* o = rright + (static_cast<int64_t>(b) * R + (mp - 1)) * K;
#pragma unroll
        for (int k = 0; k < K; k += 2) store4(o, k, bn[k], bd[k], bn[k + 1], bd[k + 1]);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        bn[k] = lanes_up(bn[k]);
        bd[k] = lanes_up(bd[k]);
      }
    };
#pragma unroll
    for (int k = 0; k < K; ++k) { bn[k] = 0.0f; bd[k] = 0.0f; }
    // m = 0 last: dx = 0, dy > 0, source and partner in the own column
    for (int m = r; m >= 0; --m) {
      if (m < r) leave_right(m + 1);
      const float* S = pw_lds + m * (R + 1);
      float sq[K], sp[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        sq[k] = wq[k * LW + R + lane + m];
        sp[k] = JOINT ? wp[k * LW + R + lane + m] : 0.0f;
      }
      step_pairs(sq, sp, S, 1);
    }
    merge_b();

    // rows y..y+K-1 are complete for this band (rows past the band: the next
    // row band's share); carry the rest
#pragma unroll
    for (int k = 0; k < K; ++k)
      store2_at(rmain, static_cast<uint32_t>(((b * K + k) * 64 + lane) * 8), an[k], ad[k]);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      an[i] = i + K < NJ ? an[i + K] : 0.0f;
      ad[i] = i + K < NJ ? ad[i + K] : 0.0f;
    }
    if (b + 1 < G.nblk) advance_v(y + NJ);   // the next block's rows y+K .. y+K+NJ-1
  }
#pragma unroll
  for (int i = 0; i < R; ++i)
    store2_at(rmain, static_cast<uint32_t>(((G.nblk * K + i) * 64 + lane) * 8), an[i], ad[i]);
}

// Merge: one item is one field of a segment of kMergeSeg columns of one row.
template <bool JOINT>
__device__ __forceinline__ void pair_merge_item(const BlfPlane* __restrict__ planes, int nplanes, int item,
                                                int field_type) {
  const int pi = plane_of_merge(planes, nplanes, item);
  const BlfPlane& P = planes[pi];
  const int local = item - 2 * P.merge_begin;
  if (local >= 2 * P.merge_count) return;  // uniform
  const int field = local & 1;
  const int rest = local >> 1;
  const int H = P.H, W = P.W;
  const int nseg = (W + kMergeSeg - 1) / kMergeSeg;
  const int Y = rest / nseg;
  const int seg = rest - Y * nseg;
  const float c = field_range_scale(P, field);
  const float2 fsc = field_store_scales(P.fmm);
  const float ssc = field ? fsc.y : fsc.x;
  const int K = P.pair_k;
  const int T = (H + K - 1) / K;
  const int R = P.pair_r;
  const int r = P.r;

  const int by = ((Y / K + 1) * P.nby - 1) / T;
  const int Y0 = (by * T / P.nby) * K;
  const int ly = Y - Y0;
  // the row band above: its rows past its end (and wrapped, for one row band)
  const int bya = by == 0 ? P.nby - 1 : by - 1;
  const int blka = bya * T / P.nby;
  const int nblka = (bya + 1) * T / P.nby - blka;
  const int Y0a = blka * K;
  const int hba = min(H, Y0a + nblka * K) - Y0a;
  int la = Y - Y0a;
  if (la < 0) la += H;
  if (la < hba) la += H;
  const bool above = la < nblka * K + R;

  const float2* __restrict__ rec = P.rec + field * P.rec_field;
  void* out = field ? P.ry : P.rx;
  const float* __restrict__ f = P.f;
  const int64_t pitch = P.pitch;
  const int rn = field ? (Y + 1 == H ? 0 : Y + 1) : Y;
  const int ovf_row = (ly / K) * R;
  const int ovf_k = ly % K;

  // Every load of the thread's kPer pixels is issued before any is used, so the item
  // waits on memory once (a pixel past the image reads column W - 1).  Rows with and
  // without carry-over rows from the band above take separate loops.
  constexpr int kPer = kMergeSeg / kMergeThreads;
  static_assert(kMergeSeg % kMergeThreads == 0, "whole pixels per thread");
  const int xbeg = seg * kMergeSeg + static_cast<int>(threadIdx.x);
  const int xend = min(W, (seg + 1) * kMergeSeg);
  auto run = [&](auto has_above) {
    constexpr bool kAbove = decltype(has_above)::value;
    f2v v[kPer], a[kPer], o_r[kPer], o_l[kPer];
    float fo[kPer], fn[kPer];
    bool take_r[kPer], take_l[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int x = min(xbeg + i * kMergeThreads, W - 1);
      const int bx = ((x + 1) * P.nbx - 1) / W;
      const int x0 = bx * W / P.nbx;
      const int lx = x - x0;
      const int64_t own = main_off(P, bx, by) + static_cast<int64_t>(ly) * 64 + lx;
      // sources in the band to the right, carried out through its lane 0
      const int bxr = bx + 1 == P.nbx ? 0 : bx + 1;
      int dr = bxr * W / P.nbx - x;
      if (dr <= 0) dr += W;
      // sources in the band to the left, carried out through its last lane
      const int bxl = bx == 0 ? P.nbx - 1 : bx - 1;
      int dl = x - ((bxl + 1) * W / P.nbx - 1);
      if (dl <= 0) dl += W;
      take_r[i] = dr <= r;
      take_l[i] = dl <= r;
      v[i] = load2(rec, own);
      if (kAbove) a[i] = load2(rec, main_off(P, bx, bya) + static_cast<int64_t>(la) * 64 + lx);
      // (an edge sum a pixel does not take is read at the nearest offset, r, and dropped)
      const int er = max(1, min(dr, r)), el = max(1, min(dl, r));
      o_r[i] = load2(rec, ovf_off(P, bxr, by, 0) + static_cast<int64_t>(ovf_row + er - 1) * K + ovf_k);
      o_l[i] = load2(rec, ovf_off(P, bxl, by, 1) + static_cast<int64_t>(ovf_row + el - 1) * K + ovf_k);
      if (JOINT) {
        const int xn = field ? x : (x + 1 == W ? 0 : x + 1);
        fo[i] = load_global(f, Y * pitch + x);
        fn[i] = load_global(f, rn * pitch + xn);
      }
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int x = xbeg + i * kMergeThreads;
      if (x >= xend) break;
      f2v s = v[i];
      if (kAbove) {
        s.x += a[i].x;
        s.y += a[i].y;
      }
      if (take_r[i]) {
        s.x = JOINT ? s.x + o_r[i].x : s.x - o_r[i].x;
        s.y += o_r[i].y;
      }
      if (take_l[i]) {
        s.x = JOINT ? s.x + o_l[i].x : s.x - o_l[i].x;
        s.y += o_l[i].y;
      }
      // the centre tap (weight 1), then the residual
      const float den = 1.0f + s.y;
      float res;
      if (JOINT) {
        const float ps = fn[i] - fo[i];
        res = (ps + s.x) / den - ps;
      } else {
        res = s.x / (c * den);
      }
      store_field(out, static_cast<int64_t>(Y) * W + x, res * ssc, field_type);
    }
  };
  if (above) run(std::true_type{}); else run(std::false_type{});
}

// Waves per SIMD the register allocation targets (no spills at any radius class):
// the persistent loop and the joint fields' values hold more registers.
constexpr int pair_waves(int R, bool joint, bool persist) {
  if (persist) return joint && R >= 32 ? 1 : 2;
  if (joint) return R >= 28 ? 2 : (R >= 10 && R <= 14) ? 4 : 3;
  return R >= 28 ? 3 : (R >= 10 && R <= 14) ? 5 : 4;
}

template <int R, bool JOINT, bool PERSIST>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(pair_waves(R, JOINT, PERSIST), 8)))
blf_pair_kernel(const BlfPlane* __restrict__ planes, int nplanes,
                                                      WorkHeader* __restrict__ work) {
  if (!PERSIST) {
    pair_item<R, JOINT>(planes, nplanes, xcd_order(blockIdx.x, gridDim.x));
    return;
  }
  const int total = work->items;
  const int np = work->nplanes;
  const BlfPlane* pl = static_cast<const BlfPlane*>(work->planes);
  for (;;) {
    const int item = grab_item(work->next[0], total, false);
    if (item >= total) break;
    pair_item<R, JOINT>(pl, np, item);
  }
}

template <bool JOINT, bool PERSIST>
__global__ void __launch_bounds__(kMergeThreads) blf_pair_merge_kernel(const BlfPlane* __restrict__ planes,
                                                                       int nplanes, int field_type,
                                                                       WorkHeader* __restrict__ work) {
  if (!PERSIST) {
    pair_merge_item<JOINT>(planes, nplanes, blockIdx.x, field_type);
    return;
  }
  const int total = work->items2;
  const int np = work->nplanes;
  const BlfPlane* pl = static_cast<const BlfPlane*>(work->planes);
  for (;;) {
    const int item = grab_item(work->next[1], total, false);
    if (item >= total) break;
    pair_merge_item<JOINT>(pl, np, item, field_type);
  }
}

// ---------------------------------------------------------------------------
// Host side: geometry and launch
// ---------------------------------------------------------------------------

namespace {
template <int R>
hipError_t launch_pair_r(const BlfPlane* planes, int nplanes, int items, int merge_items, bool joint, int ft,
                         hipStream_t s, WorkHeader* work) {
  if (work == nullptr) {
    if (items > 0) {
      if (joint)
        hipLaunchKernelGGL((blf_pair_kernel<R, true, false>), dim3(items), dim3(64), 0, s, planes, nplanes, work);
      else
        hipLaunchKernelGGL((blf_pair_kernel<R, false, false>), dim3(items), dim3(64), 0, s, planes, nplanes, work);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (merge_items > 0) {
      if (joint)
        hipLaunchKernelGGL((blf_pair_merge_kernel<true, false>), dim3(merge_items), dim3(kMergeThreads), 0, s,
                           planes, nplanes, ft, work);
      else
        hipLaunchKernelGGL((blf_pair_merge_kernel<false, false>), dim3(merge_items), dim3(kMergeThreads), 0, s,
                           planes, nplanes, ft, work);
    }
    return hipGetLastError();
  }
  if (joint)
    hipLaunchKernelGGL((blf_pair_kernel<R, true, true>), dim3(items), dim3(64), 0, s, planes, nplanes, work);
  else
    hipLaunchKernelGGL((blf_pair_kernel<R, false, true>), dim3(items), dim3(64), 0, s, planes, nplanes, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (joint)
    hipLaunchKernelGGL((blf_pair_merge_kernel<true, true>), dim3(merge_items), dim3(kMergeThreads), 0, s, planes,
                       nplanes, ft, work);
  else
    hipLaunchKernelGGL((blf_pair_merge_kernel<false, true>), dim3(merge_items), dim3(kMergeThreads), 0, s, planes,
                       nplanes, ft, work);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_blf_pair(int R, const BlfPlane* planes, int nplanes, int items, int merge_items, bool joint,
                           int field_type, hipStream_t s, WorkHeader* work) {
  switch (R) {
#define BLFLS_PAIR_CASE(RR) \
  case RR: return launch_pair_r<RR>(planes, nplanes, items, merge_items, joint, field_type, s, work);
    BLFLS_PAIR_CASE(8) BLFLS_PAIR_CASE(9) BLFLS_PAIR_CASE(10) BLFLS_PAIR_CASE(12) BLFLS_PAIR_CASE(14)
    BLFLS_PAIR_CASE(16) BLFLS_PAIR_CASE(20) BLFLS_PAIR_CASE(24) BLFLS_PAIR_CASE(28) BLFLS_PAIR_CASE(32)
#undef BLFLS_PAIR_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace blfls
