// Host logic of the symmetric-pair filter's work split (blfls_pair_geom.h),
// checked without a GPU over many image shapes and every radius class:
//   * column bands tile [0, W) with widths in [R, 64];
//   * row bands partition the T = ceil(H / K) blocks, every band at least one
//     block and, clipped at H, at least R + K - 1 rows tall, so the R rows a
//     band carries past its end (and, for the last band, the rows of its last
//     block beyond H, which wrap to the top) all land in the next band;
//   * main regions and edge records are disjoint, in order, and end exactly at
//     field_elems; merge items cover every row segment;
//   * a rejected shape really violates a condition (radius class, band width,
//     band height);
//   * two launch shapes pinned to the dispatch sizes seen in kernel traces.
#include <cstdio>
#include <cstdlib>

#include "blfls_pair_geom.h"

using namespace blfls;

static int failures = 0;
#define CHECK(cond, ...)                                          \
  do {                                                            \
    if (!(cond)) {                                                \
      if (++failures <= 20) {                                     \
        std::printf("FAIL %s:%d: %s  [", __FILE__, __LINE__, #cond); \
        std::printf(__VA_ARGS__);                                 \
        std::printf("]\n");                                       \
      }                                                           \
    }                                                             \
  } while (0)

static int band_height(int H, int T, int K, int nby, int by) {
  const int b0 = pair_band_first_block(T, nby, by), b1 = pair_band_first_block(T, nby, by + 1);
  const int y0 = b0 * K, y1 = std::min(H, b1 * K);
  return y1 - y0;
}

static void check_shape(int H, int W, int C, int R) {
  BlfPairGeom g;
  const bool ok = blf_pair_geometry(H, W, C, R, &g);
  const bool class_ok = R >= kPairMinR && R <= kPairMaxR;
  if (!ok) {
    if (!class_ok) return;
    const int K = pair_block_rows(R);
    const int nbx = (W + 63) / 64;
    // rejected: bands too narrow, or even a single row band too short
    CHECK(W / nbx < R || H < R + K - 1, "H=%d W=%d R=%d rejected", H, W, R);
    return;
  }
  CHECK(class_ok, "R=%d accepted", R);
  const int K = pair_block_rows(R);
  CHECK(K % 2 == 0 && K >= 2, "K=%d", K);
  const int T = (H + K - 1) / K;
  // column bands
  CHECK(g.nbx == (W + 63) / 64, "nbx=%d W=%d", g.nbx, W);
  int x = 0;
  for (int bx = 0; bx < g.nbx; ++bx) {
    const int x0 = pair_band_x0(W, g.nbx, bx), x1 = pair_band_x0(W, g.nbx, bx + 1);
    CHECK(x0 == x, "band %d starts at %d, not %d", bx, x0, x);
    CHECK(x1 - x0 >= R && x1 - x0 <= kPairBandCols, "H=%d W=%d R=%d band width %d", H, W, R, x1 - x0);
    x = x1;
  }
  CHECK(x == W, "column bands end at %d, W=%d", x, W);
  // row bands
  CHECK(g.nby >= 1 && g.nby <= T, "nby=%d T=%d", g.nby, T);
  int blk = 0, most = 0;
  for (int by = 0; by < g.nby; ++by) {
    const int b0 = pair_band_first_block(T, g.nby, by), b1 = pair_band_first_block(T, g.nby, by + 1);
    CHECK(b0 == blk && b1 > b0, "row band %d blocks [%d, %d)", by, b0, b1);
    blk = b1;
    most = std::max(most, b1 - b0);
    CHECK(band_height(H, T, K, g.nby, by) >= R + K - 1, "H=%d W=%d R=%d band %d of %d: %d rows", H, W, R, by,
          g.nby, band_height(H, T, K, g.nby, by));
    // the rows past this band's blocks, plus the R carried rows, fit in the next band
    const int beyond = (b1 - b0) * K - band_height(H, T, K, g.nby, by);
    const int next = band_height(H, T, K, g.nby, (by + 1) % g.nby);
    CHECK(beyond + R <= next, "H=%d R=%d band %d carries %d rows into %d", H, R, by, beyond + R, next);
    CHECK(beyond == 0 || by == g.nby - 1, "only the last band reaches past H (band %d)", by);
  }
  CHECK(blk == T, "row bands end at block %d of %d", blk, T);
  CHECK(g.max_nblk == most, "max_nblk=%d, most=%d", g.max_nblk, most);
  // record layout: main regions in band order, then the edge records, to field_elems
  const int64_t main_rows = pair_main_rows(g.max_nblk, K, R);
  int64_t at = 0;
  for (int by = 0; by < g.nby; ++by)
    for (int bx = 0; bx < g.nbx; ++bx) {
      CHECK(pair_main_off(g.nbx, g.max_nblk, K, R, bx, by) == at, "main (%d,%d)", bx, by);
      at += main_rows * kPairBandCols;
    }
  const int64_t per = static_cast<int64_t>(g.max_nblk) * R * K;
  for (int dir = 0; dir < 2; ++dir)
    for (int by = 0; by < g.nby; ++by)
      for (int bx = 0; bx < g.nbx; ++bx) {
        CHECK(pair_edge_off(g.nbx, g.nby, g.max_nblk, K, R, bx, by, dir) == at, "edge (%d,%d,%d)", bx, by, dir);
        CHECK(pair_edge_off(g.nbx, g.nby, g.max_nblk, K, R, bx, by, dir) % 2 == 0, "edge records 16-byte aligned");
        at += per;
      }
  CHECK(at == g.field_elems, "records end at %lld, field_elems %lld", static_cast<long long>(at),
        static_cast<long long>(g.field_elems));
  CHECK(g.merge_count == H * ((W + kPairMergeSeg - 1) / kPairMergeSeg), "merge_count=%d", g.merge_count);
}

int main() {
  const int classes[] = {7, 8, 9, 10, 12, 14, 16, 20, 24, 28, 32, 33};
  long shapes = 0;
  for (int R : classes)
    for (int C = 1; C <= 3; ++C)
      for (int H = 1; H <= 700; H += (H < 80 ? 1 : 7))
        for (int W = 1; W <= 1100; W += (W < 140 ? 1 : 13)) {
          check_shape(H, W, C, R);
          ++shapes;
        }
  // the large workloads
  const int big[][2] = {{2160, 3840}, {1024, 1024}, {2048, 2048}, {1536, 2048}, {1080, 1920}, {720, 1280},
                        {480, 640}, {320, 480}};
  for (auto& hw : big)
    for (int R : classes)
      for (int C = 1; C <= 3; ++C) check_shape(hw[0], hw[1], C, R);
  // dispatch sizes in the kernel traces: 3840x2160 RGB at class 24 launches
  // 60 x 54 bands x 2 fields x 3 channels one-wave workgroups; 1024x1024 RGB at
  // class 9, 16 x 64 bands
  BlfPairGeom g;
  CHECK(blf_pair_geometry(2160, 3840, 3, 24, &g), "uhd");
  CHECK(g.nbx == 60 && g.nby == 54 && g.max_nblk == 10, "uhd geometry %d %d %d", g.nbx, g.nby, g.max_nblk);
  CHECK(g.field_elems == 19491840, "uhd field_elems %lld", static_cast<long long>(g.field_elems));
  CHECK(2 * 3 * g.nbx * g.nby * 64 == 1244160, "uhd grid");
  CHECK(g.merge_count == 8640, "uhd merge items %d", g.merge_count);
  CHECK(blf_pair_geometry(1024, 1024, 3, 9, &g), "rgb1024");
  CHECK(g.nbx == 16 && g.nby == 64 && g.max_nblk == 2, "rgb1024 geometry %d %d %d", g.nbx, g.nby, g.max_nblk);
  CHECK(g.field_elems == 1933312, "rgb1024 field_elems %lld", static_cast<long long>(g.field_elems));
  CHECK(2 * 3 * g.nbx * g.nby * 64 == 393216, "rgb1024 grid");
  CHECK(!blf_pair_geometry(2160, 3840, 3, 7, &g) && !blf_pair_geometry(2160, 3840, 3, 33, &g), "classes");
  std::printf("%ld shapes checked\n", shapes);
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("all pair geometry checks passed\n");
  return 0;
}
