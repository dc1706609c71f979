// Work split of the symmetric-pair bilateral filter (Eq. (1) with one exp per
// unordered pair of taps): bands of at most 64 columns and whole blocks of K
// rows, and the layout of their partial sums.  Host code (plan, workspace
// size, descriptors) and the kernels use these same formulas; the header needs
// nothing from HIP, so the host logic is also checked by a plain C++ test.
#pragma once

#include <stdint.h>

#include <algorithm>

namespace blfls {

constexpr int kPairMinR = 8;         // smallest radius class on the pair path
constexpr int kPairMaxR = 32;        // largest radius class
constexpr int kPairBandCols = 64;    // lanes of a wave: columns of a band at most
constexpr int kPairMergeSeg = 1024;  // columns per merge item
constexpr int kPairBandRows = 40;    // rows per row band before the occupancy rule

// Rows per block at radius class R.  Four from class 10 up: the partner sums
// (K + R rows) then leave room for four to five waves per SIMD (measured 2-6%
// faster than eight-row blocks at classes 10-16); classes 8 and 9 run faster
// with eight.  Always even (the edge sums leave in pairs of rows).
constexpr int pair_block_rows(int R) { return R >= 10 ? 4 : 8; }

struct BlfPairGeom {
  int nbx = 0, nby = 0;     // column and row bands
  int max_nblk = 0;         // most blocks in a row band
  int64_t field_elems = 0;  // float2 partial sums per field
  int merge_count = 0;      // merge items per field
};

// Column band bx covers [bx W / nbx, (bx + 1) W / nbx); row band by covers the
// blocks [by T / nby, (by + 1) T / nby) of T = ceil(H / K), rows clipped at H.
constexpr int pair_band_x0(int W, int nbx, int bx) { return bx * W / nbx; }
constexpr int pair_band_first_block(int T, int nby, int by) { return by * T / nby; }

// Partial sums of one field: per band (bx, by), in band order by * nbx + bx,
// a main region of max_nblk K + R rows of 64 float2 (its own rows, then the R
// rows past its end that belong to the row band below); after all main regions
// the sums that left each band through its edge lanes, direction 0 (lane 0)
// for every band and then direction 1 (the last lane), max_nblk x R x K float2
// per band.  (constexpr: the kernels call the same functions.)
constexpr int64_t pair_main_rows(int max_nblk, int K, int R) { return static_cast<int64_t>(max_nblk) * K + R; }
constexpr int64_t pair_main_off(int nbx, int max_nblk, int K, int R, int bx, int by) {
  return (static_cast<int64_t>(by) * nbx + bx) * pair_main_rows(max_nblk, K, R) * kPairBandCols;
}
constexpr int64_t pair_edge_off(int nbx, int nby, int max_nblk, int K, int R, int bx, int by, int dir) {
  const int64_t nb = static_cast<int64_t>(nbx) * nby;
  const int64_t per = static_cast<int64_t>(max_nblk) * R * K;
  return nb * pair_main_rows(max_nblk, K, R) * kPairBandCols + (dir * nb + static_cast<int64_t>(by) * nbx + bx) * per;
}

// Geometry of a C-channel H x W image at radius class R; false when the tile
// kernel filters this shape instead (R outside the pair classes, a band
// narrower than R, or a row band shorter than R + K - 1 rows).
inline bool blf_pair_geometry(int H, int W, int C, int R, BlfPairGeom* out) {
  if (R < kPairMinR || R > kPairMaxR || H < 1 || W < 1 || C < 1) return false;
  const int K = pair_block_rows(R);
  const int nbx = (W + kPairBandCols - 1) / kPairBandCols;
  if (W / nbx < R) return false;                    // every band at least R columns
  const int T = (H + K - 1) / K;
  const int min_blocks = (R + K - 1 + K - 1) / K;   // every row band at least R + K - 1 rows
  // blocks per row band: 40 rows' worth (measured at 3840x2160 RGB, r = 24: 40-row
  // bands 11.59 ms per step, 64-row 12.14, 32-row 11.62; shorter waves balance the
  // launch's last round), fewer while the launch would give the chip under 4096
  // waves (bands of both fields of every channel)
  int per = (kPairBandRows + K - 1) / K;
  while (per > min_blocks && 2L * C * nbx * std::max(1, T / per) < 4096) --per;
  per = std::max(per, min_blocks);
  // fewer row bands while the shortest is under R + K - 1 rows: the non-last
  // bands have at least floor(T / nby) full blocks, the last one ends at H
  int nby = std::max(1, T / per);
  auto min_height = [&](int n) { return std::min((T / n) * K, H - ((n - 1) * T / n) * K); };
  while (nby > 1 && min_height(nby) < R + K - 1) --nby;
  if (min_height(nby) < R + K - 1) return false;
  BlfPairGeom g;
  g.nbx = nbx;
  g.nby = nby;
  g.max_nblk = (T + nby - 1) / nby;
  g.field_elems = pair_edge_off(nbx, nby, g.max_nblk, K, R, 0, 0, 2);
  g.merge_count = H * ((W + kPairMergeSeg - 1) / kPairMergeSeg);
  *out = g;
  return true;
}

}  // namespace blfls
