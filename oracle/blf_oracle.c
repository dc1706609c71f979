/* FP64 bilateral filter of Eq. (1), written as plain loops in C.
 *
 * TEST INFRASTRUCTURE ONLY: the same definition as bilateral_filter() in
 * blfls_oracle.py, for images too large for the NumPy loops to finish in
 * seconds (the 3840x2160 and 2048x2048 workloads).  It is part of the oracle
 * and shares nothing with the GPU library.
 *
 * out(s) = sum_d Gs(d) Gr(q(s+d) - q(s)) p(s+d) / sum_d Gs(d) Gr(q(s+d) - q(s))
 * over every offset d = (dy, dx) of the square [-r, r]^2, s + d wrapping (the
 * circular boundaries of the method), Gs(d) = exp(-(dx^2 + dy^2) / (2 sigma_s^2)),
 * Gr(t) = exp(-t^2 / (2 sigma_r^2)) or 1 when sigma_r is infinite.  Offsets are
 * summed in the order dy = -r..r, dx = -r..r for every pixel, as the NumPy
 * version sums them.  Rows are shared among OpenMP threads; each pixel's sums
 * are one thread's. */
#include <math.h>
#include <stdlib.h>

static int wrap(int v, int n) {
  int m = v % n;
  return m < 0 ? m + n : m;
}

int blf_oracle_fp64(const double *p, const double *q, int H, int W, double sigma_s, double sigma_r,
                    int r, double *out) {
  if (H < 1 || W < 1 || r < 0 || !(sigma_s > 0.0)) return -1;
  const int n = 2 * r + 1;
  double *gs = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
  if (!gs) return -2;
  for (int dy = -r; dy <= r; ++dy)
    for (int dx = -r; dx <= r; ++dx)
      gs[(dy + r) * n + (dx + r)] = exp(-(double)(dx * dx + dy * dy) / (2.0 * sigma_s * sigma_s));
  const int range_on = isfinite(sigma_r);
  const double two_sr2 = 2.0 * sigma_r * sigma_r;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < H; ++i) {
    for (int j = 0; j < W; ++j) {
      const double qs = q[(size_t)i * W + j];
      double num = 0.0, den = 0.0;
      for (int dy = -r; dy <= r; ++dy) {
        const size_t row = (size_t)wrap(i + dy, H) * W;
        for (int dx = -r; dx <= r; ++dx) {
          const size_t t = row + (size_t)wrap(j + dx, W);
          double w = gs[(dy + r) * n + (dx + r)];
          if (range_on) {
            const double d = q[t] - qs;
            w *= exp(-(d * d) / two_sr2);
          }
          num += w * p[t];
          den += w;
        }
      }
      out[(size_t)i * W + j] = num / den;
    }
  }
  free(gs);
  return 0;
}
