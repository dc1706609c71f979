// C ABI of the BLF-LS library: plans, validation and the synchronous path.
//
// A plan holds what depends only on the image shape: the factorisation of the
// two transform lengths (W/2 and H), the FP64-built twiddle and denominator
// tables rounded to FP32, the tile and workgroup geometry, and the workspace
// layout.  blfls_smooth builds the per-call descriptors on the host, uploads
// them into the caller's workspace through kernel arguments, and queues the
// kernels on the caller's stream without synchronising.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/blfls.h"
#include "blfls_internal.h"
#include "blfls_launch.h"
#include "blfls_plan.h"
#include "blfls_profile.h"

namespace blfls {

namespace {
thread_local std::string g_last_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Factor n into radices up to max_pow2 (16 or 8) for the powers of two, then one
// 8, 4 or 2, then the odd part as 15s (3 x 5, prime-factor butterflies), 9s
// (3 x 3), 3s and 5s; false if another prime divides n.  Fewer, larger stages
// mean fewer LDS round trips, barriers and twiddle products per element (rows
// and columns both take radix 16: at 3840x2160 the row passes ran 7% faster
// with it than with radix 8).
bool factorize(int n, std::vector<int>* radices, int max_pow2 = 16) {
  radices->clear();
  int m = n;
  if (max_pow2 >= 16)
    while (m % 16 == 0) { radices->push_back(16); m /= 16; }
  while (m % 8 == 0) { radices->push_back(8); m /= 8; }
  if (m % 4 == 0) { radices->push_back(4); m /= 4; }
  if (m % 2 == 0) { radices->push_back(2); m /= 2; }
  while (m % 15 == 0) { radices->push_back(15); m /= 15; }
  while (m % 9 == 0) { radices->push_back(9); m /= 9; }
  while (m % 3 == 0) { radices->push_back(3); m /= 3; }
  while (m % 5 == 0) { radices->push_back(5); m /= 5; }
  return m == 1;
}

}  // namespace

FastDiv make_fastdiv(uint32_t d) {
  // l = ceil(log2 d); mul = floor(2^32 (2^l - d) / d) + 1
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  FastDiv f;
  f.mul = static_cast<uint32_t>(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  f.shift = l;
  return f;
}

namespace {

// Two-level table of W_N = exp(-2 pi i / N) for exponents e < emax, built in FP64
// and rounded once to FP32: lo[j] = W_N^j (j < 64), hi[j] = W_N^(64 j).
std::vector<float2> two_level_table(int n, int emax) {
  std::vector<float2> t(kTwLo + (emax + kTwLo - 1) / kTwLo);
  for (size_t j = 0; j < t.size(); ++j) {
    const double e = j < static_cast<size_t>(kTwLo) ? static_cast<double>(j) : static_cast<double>(kTwLo) * (j - kTwLo);
    const double ang = -2.0 * M_PI * e / static_cast<double>(n);
    t[j] = make_float2(static_cast<float>(std::cos(ang)), static_cast<float>(std::sin(ang)));
  }
  return t;
}

// Stage descriptors of one transform length and its twiddle table.
void build_fft_size(int n, FftSize* sz, std::vector<float2>* tw, int max_pow2) {
  std::vector<int> rad;
  factorize(n, &rad, max_pow2);
  std::memset(sz, 0, sizeof(*sz));
  sz->n = n;
  sz->nstages = static_cast<int>(rad.size());
  int ns = 1;
  for (size_t s = 0; s < rad.size(); ++s) {
    const int R = rad[s];
    FftStage& S = sz->st[s];
    S.radix = R;
    S.ns = ns;
    S.per = n / R;
    S.es = n / (ns * R);
    S.per_div = make_fastdiv(static_cast<uint32_t>(n / R));
    S.ns_div = make_fastdiv(static_cast<uint32_t>(ns));
    ns *= R;
  }
  *tw = two_level_table(n, n);
}

int floor_pow2(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
}  // namespace

// Box radius of NC round k of n (domain transform, iterated boxes):
// 3 sigma_s 2^(n-k) / sqrt(4^n - 1), formed in FP64 from the FP32 sigma_s.
double nc_box_radius(float sigma_s, int n, int k) {
  const double sk = static_cast<double>(sigma_s) * std::sqrt(3.0) * std::ldexp(1.0, n - k) /
                    std::sqrt(std::ldexp(1.0, 2 * n) - 1.0);
  return std::sqrt(3.0) * sk;
}

// Farthest pixel offset an NC box of FP32 radius r can reach (increments are >= 1).
int nc_pixel_radius(float r) { return static_cast<int>(std::floor(static_cast<double>(r))); }

// Manifold tree height: filter_iterations if set, else max(2, ceil(H_s L)) with
// H_s = floor(log2 sigma_s) - 1 and L = 1 - sigma_r, each clamped at 0, capped
// at kAmfMaxHeight (FP64 from the FP32 sigmas).
int amf_tree_height(const blfls_params& p) {
  if (p.filter_iterations > 0) return p.filter_iterations;
  const double hs = std::max(0.0, std::floor(std::log2(static_cast<double>(p.sigma_s))) - 1.0);
  const double lr = std::isinf(p.sigma_r) ? 0.0 : std::max(0.0, 1.0 - static_cast<double>(p.sigma_r));
  return static_cast<int>(std::min<double>(kAmfMaxHeight, std::max(2.0, std::ceil(hs * lr))));
}

namespace {
// Layout of the adaptive-manifold arrays after the plan's workspace: offsets
// in floats from the region's start (each array 64-float aligned).
struct AmfLayout {
  size_t acc, tmp, slots, sum, carry_f, carry_b, inv, floats;
};

AmfLayout amf_layout(const blfls_plan_s* plan, int height) {
  const size_t P = 2 * static_cast<size_t>(plan->C), N = static_cast<size_t>(plan->H) * plan->W;
  const size_t line = P * amf_segments(plan->H) * static_cast<size_t>(plan->W);
  AmfLayout L{};
  size_t w = 0;
  auto take = [&](size_t n) { const size_t at = w; w = (w + n + 63) / 64 * 64; return at; };
  L.acc = take(3 * P * N);
  L.tmp = take(4 * P * N);
  L.slots = take(static_cast<size_t>(amf_slots(height)) * P * N);
  L.sum = take(5 * line);
  L.carry_f = take(4 * line);
  L.carry_b = take(4 * line);
  L.inv = take(2 * P);   // range scales, then FP16 store scales
  L.floats = w;
  return L;
}
}  // namespace

// Symmetric-pair filter of a BLF request: its geometry, or false for the tile kernel.
static bool request_pair_geometry(const blfls_plan_s* plan, const blfls_params& p, BlfPairGeom* g) {
  if (p.filter != BLFLS_FILTER_BLF) return false;
  const int r = p.radius >= 0 ? p.radius : static_cast<int>(std::ceil(3.0 * static_cast<double>(p.sigma_s)));
  const int R = blf_radius_class(r);
  return R > 0 && blf_pair_geometry(plan->H, plan->W, plan->C, R, g);
}

size_t request_workspace_bytes(const blfls_plan_s* plan, const blfls_params& p) {
  BlfPairGeom pg;
  if (request_pair_geometry(plan, p, &pg))   // the pair filter's partial sums follow the plan's workspace
    return plan->ws_bytes + align_up(2 * static_cast<size_t>(plan->C) * pg.field_elems * sizeof(float2), 256);
  if (p.filter != BLFLS_FILTER_AMF) return plan->ws_bytes;
  return plan->ws_bytes + amf_layout(plan, amf_tree_height(p)).floats * sizeof(float);
}

blfls_status set_error(blfls_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

blfls_status hip_error(hipError_t e, const char* where) {
  return set_error(BLFLS_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

blfls_status check_shape(int H, int W, int C) {
  if (H < 1 || W < 1) return set_error(BLFLS_E_INVALID, "H and W must be >= 1");
  if (C < 1 || C > BLFLS_MAX_CHANNELS) return set_error(BLFLS_E_INVALID, "C must be in [1, 4]");
  if (W % 2 != 0) return set_error(BLFLS_E_UNSUPPORTED, "W must be even (real FFT of W via a complex FFT of W/2)");
  const int M = W / 2;
  if (M > kMaxFft || H > kMaxFft) return set_error(BLFLS_E_UNSUPPORTED, "W/2 and H must be at most 4096");
  std::vector<int> rad;
  if (!factorize(M, &rad) || !factorize(H, &rad))
    return set_error(BLFLS_E_UNSUPPORTED, "W/2 and H must factor into 2, 3 and 5 only");
  return BLFLS_OK;
}

blfls_status check_params(const blfls_params* p, int* radius_out) {
  if (p == nullptr) return set_error(BLFLS_E_INVALID, "params is NULL");
  if (!std::isfinite(p->lambda) || p->lambda < 0.0f) return set_error(BLFLS_E_INVALID, "lambda must be finite and >= 0");
  if (!std::isfinite(p->sigma_s) || p->sigma_s <= 0.0f) return set_error(BLFLS_E_INVALID, "sigma_s must be finite and > 0");
  if (std::isnan(p->sigma_r) || p->sigma_r <= 0.0f) return set_error(BLFLS_E_INVALID, "sigma_r must be > 0 (or +inf)");
  if (p->iterations < 1) return set_error(BLFLS_E_INVALID, "iterations must be >= 1");
  if (!std::isfinite(p->sigma_guide) || p->sigma_guide < 0.0f) return set_error(BLFLS_E_INVALID, "sigma_guide must be finite and >= 0");
  if (p->flags & ~BLFLS_F_NORMALIZE) return set_error(BLFLS_E_INVALID, "unknown flag bits");
  if (!std::isfinite(p->detail_gain)) return set_error(BLFLS_E_INVALID, "detail_gain must be finite");
  if (p->filter != BLFLS_FILTER_BLF && p->filter != BLFLS_FILTER_NC && p->filter != BLFLS_FILTER_GRID &&
      p->filter != BLFLS_FILTER_AMF)
    return set_error(BLFLS_E_INVALID, "unknown filter");
  if (p->filter_iterations < 0 || p->filter_iterations > 8)
    return set_error(BLFLS_E_INVALID, "filter_iterations must be in [0, 8]");
  if (p->filter == BLFLS_FILTER_AMF && p->filter_iterations > kAmfMaxHeight)
    return set_error(BLFLS_E_INVALID, "the AMF tree height (filter_iterations) must be in [0, 6]");
  if (p->filter != BLFLS_FILTER_NC && p->filter != BLFLS_FILTER_AMF && p->filter_iterations != 0)
    return set_error(BLFLS_E_INVALID, "filter_iterations applies to the NC and AMF filters only");
  if (p->filter == BLFLS_FILTER_GRID && grid_cell_size(p->sigma_s) > kGridMaxCell)
    return set_error(BLFLS_E_INVALID, "sigma_s too large for the bilateral grid (cell above 32 pixels)");
  int r = p->radius;
  if (r < -1) return set_error(BLFLS_E_INVALID, "radius must be >= 0 or -1");
  if (p->filter == BLFLS_FILTER_GRID || p->filter == BLFLS_FILTER_AMF) {
    r = 0;
  } else if (p->filter == BLFLS_FILTER_NC) {
    const int n = p->filter_iterations ? p->filter_iterations : 3;
    if (nc_pixel_radius(static_cast<float>(nc_box_radius(p->sigma_s, n, 1))) > kNcMaxR)
      return set_error(BLFLS_E_INVALID, "sigma_s too large for the NC filter (first box radius above 32 pixels)");
    r = 0;
  } else {
    if (r == -1) r = static_cast<int>(std::ceil(3.0 * static_cast<double>(p->sigma_s)));
    if (r > BLFLS_MAX_RADIUS) return set_error(BLFLS_E_INVALID, "radius exceeds BLFLS_MAX_RADIUS (32)");
  }
  if (p->sigma_guide > 0.0f && static_cast<int>(std::ceil(3.0 * static_cast<double>(p->sigma_guide))) > kMaxR)
    return set_error(BLFLS_E_INVALID, "sigma_guide too large (radius ceil(3 sigma_guide) must be <= 32)");
  *radius_out = r;
  return BLFLS_OK;
}

blfls_status plan_create(int H, int W, int C, blfls_precision prec, blfls_plan_s** out) {
  blfls_status st = check_shape(H, W, C);
  if (st != BLFLS_OK) return st;
  if (prec != BLFLS_FP32 && prec != BLFLS_MIXED_BF16 && prec != BLFLS_MIXED_FP16)
    return set_error(BLFLS_E_INVALID, "unknown precision");
  static std::once_flag init_once;
  static hipError_t init_err = hipSuccess;
  std::call_once(init_once, [] {
    init_err = fft_init_kernels();
    if (init_err == hipSuccess) init_err = nc_init_kernels();
    if (init_err == hipSuccess) init_err = amf_init_kernels();
    if (init_err == hipSuccess) init_err = grid_init_kernels();
  });
  if (init_err != hipSuccess) return hip_error(init_err, "kernel attributes");
  auto* p = new (std::nothrow) blfls_plan_s();
  if (!p) return set_error(BLFLS_E_NOMEM, "host allocation failed");
  p->H = H; p->W = W; p->C = C; p->M = W / 2; p->precision = prec;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { delete p; return hip_error(e, "hipGetDevice"); }
  const int M = p->M;

  // tables, built in FP64 and rounded once to FP32
  FftSize szM, szH;
  std::vector<float2> twM, twH;
  build_fft_size(M, &szM, &twM, 16);
  build_fft_size(H, &szH, &twH, 16);
  const std::vector<float2> twW = two_level_table(W, M + 1);
  std::vector<float> sx(M + 1), sy(H);
  for (int k = 0; k <= M; ++k) {
    const double s = std::sin(M_PI * k / static_cast<double>(W));
    sx[k] = static_cast<float>(4.0 * s * s);
  }
  for (int k = 0; k < H; ++k) {
    const double s = std::sin(M_PI * k / static_cast<double>(H));
    sy[k] = static_cast<float>(4.0 * s * s);
  }
  size_t off = 0;
  const size_t o_szM = off; off = align_up(off + sizeof(FftSize), 256);
  const size_t o_szH = off; off = align_up(off + sizeof(FftSize), 256);
  const size_t o_twM = off; off = align_up(off + twM.size() * sizeof(float2) + 8, 256);
  const size_t o_twH = off; off = align_up(off + twH.size() * sizeof(float2) + 8, 256);
  const size_t o_twW = off; off = align_up(off + twW.size() * sizeof(float2), 256);
  const size_t o_sx = off; off = align_up(off + sx.size() * sizeof(float), 256);
  const size_t o_sy = off; off = align_up(off + sy.size() * sizeof(float), 256);
  std::vector<uint8_t> blob(off, 0);
  std::memcpy(blob.data() + o_szM, &szM, sizeof(szM));
  std::memcpy(blob.data() + o_szH, &szH, sizeof(szH));
  if (!twM.empty()) std::memcpy(blob.data() + o_twM, twM.data(), twM.size() * sizeof(float2));
  if (!twH.empty()) std::memcpy(blob.data() + o_twH, twH.data(), twH.size() * sizeof(float2));
  std::memcpy(blob.data() + o_twW, twW.data(), twW.size() * sizeof(float2));
  std::memcpy(blob.data() + o_sx, sx.data(), sx.size() * sizeof(float));
  std::memcpy(blob.data() + o_sy, sy.data(), sy.size() * sizeof(float));
  e = hipMalloc(&p->dev_tables, off);
  if (e != hipSuccess) { delete p; return set_error(BLFLS_E_NOMEM, "hipMalloc of plan tables failed"); }
  // upload on a private non-blocking stream: a copy on the legacy stream would
  // have to order itself against streams another thread may be capturing
  hipStream_t up = nullptr;
  e = hipStreamCreateWithFlags(&up, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMemcpyAsync(p->dev_tables, blob.data(), off, hipMemcpyHostToDevice, up);
  if (e == hipSuccess) e = hipStreamSynchronize(up);
  if (up) (void)hipStreamDestroy(up);
  if (e != hipSuccess) { (void)hipFree(p->dev_tables); delete p; return hip_error(e, "plan table upload"); }
  uint8_t* base = static_cast<uint8_t*>(p->dev_tables);
  p->szM = reinterpret_cast<const FftSize*>(base + o_szM);
  p->szH = reinterpret_cast<const FftSize*>(base + o_szH);
  p->twM = reinterpret_cast<const float2*>(base + o_twM);
  p->twH = reinterpret_cast<const float2*>(base + o_twH);
  p->twW = reinterpret_cast<const float2*>(base + o_twW);
  p->ntwM = static_cast<int>(twM.size());
  p->ntwH = static_cast<int>(twH.size());
  p->ntwW = static_cast<int>(twW.size());
  p->sx = reinterpret_cast<const float*>(base + o_sx);
  p->sy = reinterpret_cast<const float*>(base + o_sy);

  // FFT geometry: rows per row-pass workgroup (a power of two, rb (W/2+1)
  // complex values in LDS) and spectrum columns per column-pass workgroup
  // (cb H), both within 64 KiB so two workgroups share a CU, split further
  // while the whole pass would not give every CU a workgroup
  int rb = floor_pow2(std::min(16, std::max(1, kFftLdsComplex / (M + 1))));
  while (rb > 4 && static_cast<long>(C) * ((H + rb - 1) / rb) < 256) rb /= 2;
  rb = std::min(rb, floor_pow2(H));
  int cb = std::min(16, std::max(1, kFftLdsComplex / H));
  while (cb > 1 && static_cast<long>(C) * ((M + 1 + cb - 1) / cb) < 256) cb = (cb + 1) / 2;
  // a radix-15 stage holds one butterfly per thread across its barrier
  if (M % 15 == 0) while (rb > 1 && static_cast<long>(rb) * M > kFftRadix15Elems) rb /= 2;
  if (H % 15 == 0) while (cb > 1 && static_cast<long>(cb) * H > kFftRadix15Elems) --cb;
  // H = 512 or 1024: one spectrum column per wave, held in registers; likewise
  // one row per wave for W/2 = 512 or 1024
  const int colw = (H == 512 || H == 1024) ? H / 64 : 0;
  if (colw) cb = fft_cols_wave_per_block();
  const int roww = (M == 512 || M == 1024) ? M / 64 : 0;
  if (roww) rb = fft_cols_wave_per_block();
  p->rb = rb;
  p->cb = cb;
  p->colw = colw;
  p->roww = roww;
  p->row_blocks = (H + rb - 1) / rb;
  p->col_blocks = (M + 1 + cb - 1) / cb;
  p->lds_rows = roww ? fft_rows_wave_lds_bytes(roww) : fft_rows_lds_bytes(M, rb);
  p->lds_cols = colw ? fft_cols_wave_lds_bytes(colw) : fft_cols_lds_bytes(H, cb);
  p->tiles_x = (W + blf_tile_w() - 1) / blf_tile_w();
  p->tiles_y = (H + blf_tile_h() - 1) / blf_tile_h();

  // workspace layout
  p->field_elem = prec == BLFLS_FP32 ? 4 : 2;
  const size_t plane = static_cast<size_t>(H) * W;
  size_t w = 0;
  p->off_desc = w; w = align_up(w + kDescBytes, 256);
  p->off_partial = w; w = align_up(w + static_cast<size_t>(C) * kMinmaxBlocks * 4 * sizeof(float), 256);
  // FP16 fields: extrema partials of the image's own gradients (the fields' store scales)
  p->off_fpartial = w; w = align_up(w + static_cast<size_t>(C) * kMinmaxBlocks * 4 * sizeof(float), 256);
  p->off_rx = w; w = align_up(w + C * plane * p->field_elem, 256);
  p->off_ry = w; w = align_up(w + C * plane * p->field_elem, 256);
  p->off_spec = w; w = align_up(w + static_cast<size_t>(C) * (M + 1) * H * sizeof(float2), 256);
  p->off_gauss = w; w = align_up(w + C * plane * sizeof(float), 256);
  p->off_tmp = w; w = align_up(w + C * plane * sizeof(float), 256);
  // NC filter passes: ping buffers of both fields here; the pong buffers
  // overlay the spectrum (x) and the Gaussian scratch (y), idle while filtering
  p->off_nc = w; w = align_up(w + 2 * C * plane * sizeof(float), 256);
  p->ws_bytes = w;
  *out = p;
  return BLFLS_OK;
}

void plan_free(blfls_plan_s* p) {
  if (!p) return;
  if (p->dev_tables) (void)hipFree(p->dev_tables);
  delete p;
}

void build_request(const blfls_plan_s* plan, const blfls_params& prm, int radius, const float* f,
                   const float* guide, float* u, int64_t pitch, void* ws, const void* dev_tables,
                   RequestDesc* out) {
  const int H = plan->H, W = plan->W, C = plan->C, M = plan->M;
  uint8_t* wsb = static_cast<uint8_t*>(ws);
  const size_t plane = static_cast<size_t>(H) * W;
  const double log2e = 1.4426950408889634074;
  const double ss = prm.sigma_s;

  RequestTables& T = out->tables;
  for (int d = -kMaxR; d <= kMaxR; ++d) {
    const double q = static_cast<double>(d) * d * log2e / (2.0 * ss * ss);
    T.sy[d + kMaxR] = std::abs(d) <= radius ? static_cast<float>(-q) : -std::numeric_limits<float>::infinity();
    T.ex[d + kMaxR] = static_cast<float>(std::exp2(-q));
    T.gw[d + kMaxR] = 0.0f;
  }
  for (int dx = 0; dx <= kMaxR; ++dx)
    for (int dy = 0; dy <= kMaxR; ++dy) {
      const double q = static_cast<double>(dx * dx + dy * dy) * log2e / (2.0 * ss * ss);
      T.pw[dx * (kMaxR + 1) + dy] =
          dx <= radius && dy <= radius ? static_cast<float>(-q) : -std::numeric_limits<float>::infinity();
    }
  int rg = 0;
  if (prm.sigma_guide > 0.0f) {
    const double sg = prm.sigma_guide;
    rg = static_cast<int>(std::ceil(3.0 * sg));
    double tot = 0.0;
    for (int d = -rg; d <= rg; ++d) tot += std::exp(-static_cast<double>(d) * d / (2.0 * sg * sg));
    for (int d = -rg; d <= rg; ++d)
      T.gw[d + kMaxR] = static_cast<float>(std::exp(-static_cast<double>(d) * d / (2.0 * sg * sg)) / tot);
  }
  const float* spatial = static_cast<const float*>(dev_tables);
  const float* gw = spatial + offsetof(RequestTables, gw) / sizeof(float);

  const bool range_on = std::isfinite(prm.sigma_r);
  const float c = range_on ? static_cast<float>(std::sqrt(log2e / (2.0 * static_cast<double>(prm.sigma_r) * prm.sigma_r)))
                           : 0.0f;
  out->R = blf_radius_class(radius);
  out->iterations = prm.iterations;
  out->normalize = (prm.flags & BLFLS_F_NORMALIZE) != 0 && range_on;
  out->smooth_guide = prm.sigma_guide > 0.0f;
  out->joint_first = guide != nullptr || out->smooth_guide || !range_on;
  const int tiles = plan->tiles_x * plan->tiles_y;
  BlfPairGeom pg;
  out->pair = request_pair_geometry(plan, prm, &pg);
  out->pair_items = out->pair ? 2 * C * pg.nbx * pg.nby : 0;
  out->merge_items = out->pair ? 2 * C * pg.merge_count : 0;
  float2* pair_rec = reinterpret_cast<float2*>(wsb + plan->ws_bytes);
  out->blf_first.assign(C, BlfPlane{});
  out->blf_next.assign(C, BlfPlane{});
  out->mm_first.assign(C, AuxPlane{});
  out->mm_next.assign(C, AuxPlane{});
  out->mm_f.assign(C, AuxPlane{});
  out->fp16_scale = plan->precision == BLFLS_MIXED_FP16;
  out->gauss.assign(C, AuxPlane{});
  out->fft.assign(C, FftPlane{});
  out->grid_first.assign(C, GridPlane{});
  out->grid_next.assign(C, GridPlane{});
  out->nc_first.assign(C, NcPlane{});
  out->nc_next.assign(C, NcPlane{});
  out->amf_first.assign(2 * C, AmfPlane{});
  out->amf_next.assign(2 * C, AmfPlane{});
  out->filter = prm.filter;
  out->nc_rounds = prm.filter == BLFLS_FILTER_NC ? (prm.filter_iterations ? prm.filter_iterations : 3) : 0;
  for (int k = 1; k <= out->nc_rounds; ++k) {
    out->nc_r[k - 1] = static_cast<float>(nc_box_radius(prm.sigma_s, out->nc_rounds, k));
    out->nc_R[k - 1] = nc_pixel_radius(out->nc_r[k - 1]);
  }
  float* gauss_base = reinterpret_cast<float*>(wsb + plan->off_gauss);
  float* tmp_base = reinterpret_cast<float*>(wsb + plan->off_tmp);
  float* partial_base = reinterpret_cast<float*>(wsb + plan->off_partial);
  float* fpartial_base = reinterpret_cast<float*>(wsb + plan->off_fpartial);
  for (int ch = 0; ch < C; ++ch) {
    const float* fc = f + static_cast<int64_t>(ch) * H * pitch;
    const float* gc = guide ? guide + static_cast<int64_t>(ch) * H * pitch : nullptr;
    float* uc = u + static_cast<int64_t>(ch) * H * pitch;
    void* rx = wsb + plan->off_rx + ch * plane * plan->field_elem;
    void* ry = wsb + plan->off_ry + ch * plane * plan->field_elem;
    float* partial = partial_base + static_cast<size_t>(ch) * kMinmaxBlocks * 4;
    float* gdst = gauss_base + ch * plane;

    // range source of iteration 1 (and its row pitch)
    const float* src1 = out->smooth_guide ? gdst : (gc ? gc : fc);
    const int64_t src1_pitch = out->smooth_guide ? W : pitch;

    AuxPlane& G = out->gauss[ch];
    G.src = gc ? gc : fc;
    G.dst = gdst;
    G.tmp = tmp_base + ch * plane;
    G.partial = nullptr;
    G.pitch = pitch;
    G.H = H; G.W = W; G.rg = rg; G.gw = gw;

    AuxPlane& A1 = out->mm_first[ch];
    A1 = AuxPlane{};
    A1.src = src1; A1.partial = partial; A1.pitch = src1_pitch; A1.H = H; A1.W = W;
    AuxPlane& A2 = out->mm_next[ch];
    A2 = AuxPlane{};
    A2.src = uc; A2.partial = partial; A2.pitch = pitch; A2.H = H; A2.W = W;
    float* fpartial = out->fp16_scale ? fpartial_base + static_cast<size_t>(ch) * kMinmaxBlocks * 4 : nullptr;
    AuxPlane& AF = out->mm_f[ch];
    AF = AuxPlane{};
    AF.src = fc; AF.partial = fpartial; AF.pitch = pitch; AF.H = H; AF.W = W;

    for (int it = 0; it < 2; ++it) {
      BlfPlane& B = it == 0 ? out->blf_first[ch] : out->blf_next[ch];
      B.f = fc;
      B.rx = rx;
      B.ry = ry;
      B.pitch = pitch;
      B.gpitch = it == 0 ? src1_pitch : pitch;
      B.H = H; B.W = W; B.r = radius;
      B.tiles_x = plan->tiles_x;
      B.tile_begin = ch * tiles;
      B.tile_count = tiles;
      B.cx = B.cy = c;
      if (out->pair) {
        B.tile_begin = ch * pg.nbx * pg.nby;
        B.tile_count = pg.nbx * pg.nby;
        B.nbx = pg.nbx;
        B.nby = pg.nby;
        B.max_nblk = pg.max_nblk;
        B.pair_r = out->R;
        B.pair_k = pair_block_rows(out->R);
        B.merge_begin = ch * pg.merge_count;
        B.merge_count = pg.merge_count;
        B.rec = pair_rec + 2 * ch * pg.field_elems;
        B.rec_field = pg.field_elems;
      }
      B.spatial = spatial;
      B.minmax = out->normalize ? partial : nullptr;
      B.fmm = fpartial;
      if (it == 0) {
        // joint when a guide (or its Gaussian-smoothed copy) is the range
        // source, and when the range kernel is off (q = 0: spatial weights only)
        B.g = out->joint_first ? src1 : nullptr;
      } else {
        B.g = uc;
      }
    }
    for (int it = 0; it < 2; ++it) {
      const BlfPlane& B = it == 0 ? out->blf_first[ch] : out->blf_next[ch];
      NcPlane& N = it == 0 ? out->nc_first[ch] : out->nc_next[ch];
      N.f = fc;
      N.g = B.g;
      N.pitch = pitch;
      N.gpitch = B.gpitch;
      float* ping = reinterpret_cast<float*>(wsb + plan->off_nc);
      N.buf[0][0] = ping + (0 * C + ch) * plane;
      N.buf[0][1] = ping + (1 * C + ch) * plane;
      N.buf[1][0] = reinterpret_cast<float*>(wsb + plan->off_spec) + ch * plane;
      N.buf[1][1] = tmp_base + ch * plane;
      N.rx = rx;
      N.ry = ry;
      N.minmax = B.minmax;
      N.fmm = fpartial;
      N.H = H; N.W = W;
      N.a = range_on ? static_cast<float>(static_cast<double>(prm.sigma_s) / static_cast<double>(prm.sigma_r)) : 0.0f;
      N.rcount = nc_row_items(H, W);
      N.rbegin = ch * N.rcount;
      N.ccount = nc_col_items(H, W);
      N.cbegin = ch * N.ccount;
    }
    for (int it = 0; it < 2; ++it) {
      const BlfPlane& B = it == 0 ? out->blf_first[ch] : out->blf_next[ch];
      GridPlane& G2 = it == 0 ? out->grid_first[ch] : out->grid_next[ch];
      const int sc = grid_cell_size(prm.sigma_s);
      G2.f = fc;
      G2.g = B.g;
      G2.pitch = pitch;
      G2.gpitch = B.gpitch;
      G2.rx = rx;
      G2.ry = ry;
      G2.minmax = partial;
      G2.H = H; G2.W = W;
      G2.s = sc;
      G2.tiles_x = grid_tiles_x(W, sc);
      G2.tile_count = G2.tiles_x * grid_tiles_y(H, sc);
      G2.tile_begin = ch * G2.tile_count;
      G2.inv_r = range_on ? static_cast<float>(1.0 / static_cast<double>(prm.sigma_r)) : 0.0f;
      G2.sigma_r = range_on ? prm.sigma_r : 0.0f;
      G2.sig_xy = static_cast<float>(static_cast<double>(prm.sigma_s) / sc);
      G2.normalize = (prm.flags & BLFLS_F_NORMALIZE) != 0 ? 1 : 0;
      G2.fmm = fpartial;
    }
    for (int it = 0; it < 2; ++it) {
      const BlfPlane& B = it == 0 ? out->blf_first[ch] : out->blf_next[ch];
      for (int field = 0; field < 2; ++field) {
        AmfPlane& A = (it == 0 ? out->amf_first : out->amf_next)[2 * ch + field];
        A.f = fc;
        A.g = B.g;
        A.pitch = pitch;
        A.gpitch = B.gpitch;
        A.out = field ? ry : rx;
        A.minmax = B.minmax;
        A.field = field;
        A.fmm = fpartial;
      }
    }
    FftPlane& F = out->fft[ch];
    F.rx = rx; F.ry = ry;
    F.spec = reinterpret_cast<float2*>(wsb + plan->off_spec) + static_cast<size_t>(ch) * (M + 1) * H;
    F.f = fc; F.u = uc; F.pitch = pitch;
    F.H = H; F.W = W; F.lambda = prm.lambda;
    F.rb = plan->rb; F.cb = plan->cb; F.colw = plan->colw; F.roww = plan->roww;
    F.row_begin = ch * plan->row_blocks; F.row_count = plan->row_blocks;
    F.col_begin = ch * plan->col_blocks; F.col_count = plan->col_blocks;
    F.szM = plan->szM; F.szH = plan->szH;
    F.twM = plan->twM; F.twH = plan->twH; F.twW = plan->twW;
    F.ntwM = plan->ntwM; F.ntwH = plan->ntwH; F.ntwW = plan->ntwW;
    F.sx = plan->sx; F.sy = plan->sy;
    F.m_div = make_fastdiv(static_cast<uint32_t>(M));
    F.h_div = make_fastdiv(static_cast<uint32_t>(H));
    F.rb_div = make_fastdiv(static_cast<uint32_t>(plan->rb));
    F.gain = 1.0f;
    F.fmm = fpartial;
  }
  out->fft_last = out->fft;
  for (FftPlane& F : out->fft_last) F.gain = static_cast<float>(1.0 - static_cast<double>(prm.detail_gain));
  if (prm.filter == BLFLS_FILTER_AMF) {
    // the manifold arrays follow the plan's workspace
    const int height = amf_tree_height(prm);
    const AmfLayout L = amf_layout(plan, height);
    float* base = reinterpret_cast<float*>(wsb + plan->ws_bytes);
    AmfGeom& G = out->amf_geom;
    G = AmfGeom{};
    G.P = 2 * C; G.H = H; G.W = W; G.S = amf_segments(H);
    G.a = static_cast<float>(std::exp(-std::sqrt(2.0) / ss));
    G.c0 = static_cast<float>(-std::sqrt(2.0) * log2e / ss);
    G.c1 = range_on ? static_cast<float>(-2.0 * log2e / static_cast<double>(prm.sigma_r)) : 0.0f;
    G.kpsi = range_on ? static_cast<float>(log2e / (static_cast<double>(prm.sigma_r) * prm.sigma_r)) : 0.0f;
    G.tau = 1e-20f;
    G.acc = base + L.acc;
    G.tmp = base + L.tmp;
    G.sum = base + L.sum;
    G.carry_f = base + L.carry_f;
    G.carry_b = base + L.carry_b;
    G.inv = base + L.inv;
    G.ft = plan->precision == BLFLS_FP32 ? kF32 : plan->precision == BLFLS_MIXED_BF16 ? kBF16 : kF16;
    out->amf_slots = base + L.slots;
    out->amf_height = height;
  }
}

hipError_t enqueue_request(const blfls_plan_s* plan, const RequestDesc& rd, const DeviceDesc& dev,
                           hipStream_t s) {
  const int C = plan->C;
  const int items = 2 * plan->tiles_x * plan->tiles_y * C;
  const int ft = plan->precision == BLFLS_FP32 ? kF32 : plan->precision == BLFLS_MIXED_BF16 ? kBF16 : kF16;
  hipError_t e;
  if (rd.fp16_scale) {
    // FP16 fields: the image's gradient extrema, which set the fields' store scales
    StageTimer t(BLFLS_STAGE_MINMAX, s);
    e = launch_minmax(dev.mm_f, C, s);
    if (e != hipSuccess) return e;
  }
  if (rd.smooth_guide) {
    StageTimer t(BLFLS_STAGE_GAUSS, s);
    e = launch_gauss(dev.gauss, C, static_cast<int64_t>(plan->H) * plan->W, s);
    if (e != hipSuccess) return e;
  }
  for (int it = 0; it < rd.iterations; ++it) {
    const bool first = it == 0;
    if (rd.normalize || rd.filter == BLFLS_FILTER_GRID) {
      StageTimer t(BLFLS_STAGE_MINMAX, s);
      e = launch_minmax(first ? dev.mm_first : dev.mm_next, C, s);
      if (e != hipSuccess) return e;
    }
    if (rd.filter == BLFLS_FILTER_GRID) {
      StageTimer t(BLFLS_STAGE_BLF, s);
      const GridPlane* gp = first ? dev.grid_first : dev.grid_next;
      const GridPlane& g0 = first ? rd.grid_first[0] : rd.grid_next[0];
      e = launch_grid(gp, C, 2 * C * g0.tile_count, grid_z_stride(g0), g0.g == nullptr, ft, s);
      if (e != hipSuccess) return e;
    } else if (rd.filter == BLFLS_FILTER_AMF) {
      StageTimer t(BLFLS_STAGE_BLF, s);
      AmfGeom G = rd.amf_geom;
      G.planes = first ? dev.amf_first : dev.amf_next;
      e = launch_amf(G, rd.amf_slots, rd.amf_height, s);
      if (e != hipSuccess) return e;
    } else if (rd.filter == BLFLS_FILTER_NC) {
      StageTimer t(BLFLS_STAGE_BLF, s);
      const NcPlane* np = first ? dev.nc_first : dev.nc_next;
      const int passes = 2 * rd.nc_rounds;
      for (int pass = 0; pass < passes; ++pass) {
        const int k = pass / 2;
        const int n_items = (pass & 1) ? C * nc_col_items(plan->H, plan->W) : C * nc_row_items(plan->H, plan->W);
        e = launch_nc_pass(np, C, n_items, pass, passes, rd.nc_r[k], rd.nc_R[k], ft, s);
        if (e != hipSuccess) return e;
      }
    } else {
      StageTimer t(BLFLS_STAGE_BLF, s);
      if (rd.pair)
        e = launch_blf_pair(rd.R, first ? dev.blf_first : dev.blf_next, C, rd.pair_items, rd.merge_items,
                            first ? rd.joint_first : true, ft, s);
      else
        e = launch_blf(rd.R, first ? dev.blf_first : dev.blf_next, C, items, first ? rd.joint_first : true, ft, s);
      if (e != hipSuccess) return e;
    }
    const FftPlane* fp = it + 1 == rd.iterations ? dev.fft_last : dev.fft;
    {
      StageTimer t(BLFLS_STAGE_ROWS_FWD, s);
      e = launch_fft_rows_fwd(fp, C, plan->row_blocks * C, plan->lds_rows, ft, s);
      if (e != hipSuccess) return e;
    }
    {
      StageTimer t(BLFLS_STAGE_COLS, s);
      e = launch_fft_cols(fp, C, plan->col_blocks * C, plan->lds_cols, s);
      if (e != hipSuccess) return e;
    }
    {
      StageTimer t(BLFLS_STAGE_ROWS_INV, s);
      e = launch_fft_rows_inv(fp, C, plan->row_blocks * C, plan->lds_rows, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace blfls

using namespace blfls;

extern "C" {

const char* blfls_last_error(void) { return g_last_error.c_str(); }

const char* blfls_version(void) { return "blfls 0.1.0 (gfx950)"; }

blfls_status blfls_plan(blfls_plan_t* out, int32_t H, int32_t W, int32_t C, blfls_precision precision,
                        size_t* workspace_bytes) {
  g_last_error.clear();
  if (out == nullptr) return set_error(BLFLS_E_INVALID, "out is NULL");
  *out = nullptr;
  blfls_plan_s* p = nullptr;
  const blfls_status st = plan_create(H, W, C, precision, &p);
  if (st != BLFLS_OK) return st;
  *out = p;
  if (workspace_bytes) *workspace_bytes = p->ws_bytes;
  return BLFLS_OK;
}

blfls_status blfls_plan_workspace_size(blfls_plan_t plan, size_t* workspace_bytes) {
  g_last_error.clear();
  if (plan == nullptr || workspace_bytes == nullptr) return set_error(BLFLS_E_INVALID, "NULL argument");
  *workspace_bytes = plan->ws_bytes;
  return BLFLS_OK;
}

blfls_status blfls_workspace_size(blfls_plan_t plan, const blfls_params* params, size_t* workspace_bytes) {
  g_last_error.clear();
  if (plan == nullptr || params == nullptr || workspace_bytes == nullptr)
    return set_error(BLFLS_E_INVALID, "NULL argument");
  int radius = 0;
  const blfls_status st = check_params(params, &radius);
  if (st != BLFLS_OK) return st;
  *workspace_bytes = request_workspace_bytes(plan, *params);
  return BLFLS_OK;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb);

// Tone-mapping workspace: the smooth's own, then L, the base and the partials.
static size_t tonemap_bytes(const blfls_plan_s* plan, const blfls_params& p, size_t* off_l, size_t* off_base,
                            size_t* off_part) {
  const size_t plane = align_up(static_cast<size_t>(plan->H) * plan->W * sizeof(float), 256);
  *off_l = align_up(request_workspace_bytes(plan, p), 256);
  *off_base = *off_l + plane;
  *off_part = *off_base + plane;
  return *off_part + align_up(2 * static_cast<size_t>(tm_extrema_blocks()) * sizeof(float), 256);
}

blfls_status blfls_tonemap_workspace_size(blfls_plan_t plan, const blfls_params* params, size_t* workspace_bytes) {
  g_last_error.clear();
  if (plan == nullptr || params == nullptr || workspace_bytes == nullptr)
    return set_error(BLFLS_E_INVALID, "NULL argument");
  int radius = 0;
  const blfls_status st = check_params(params, &radius);
  if (st != BLFLS_OK) return st;
  size_t a, b, c;
  *workspace_bytes = tonemap_bytes(plan, *params, &a, &b, &c);
  return BLFLS_OK;
}

blfls_status blfls_tonemap(blfls_plan_t plan, const blfls_params* params, const float* rgb, float* out,
                           int64_t pitch, float contrast, void* workspace, void* stream) {
  g_last_error.clear();
  if (plan == nullptr || params == nullptr) return set_error(BLFLS_E_INVALID, "NULL argument");
  if (rgb == nullptr || out == nullptr || workspace == nullptr) return set_error(BLFLS_E_INVALID, "NULL buffer");
  if (plan->C != 1) return set_error(BLFLS_E_INVALID, "tone mapping smooths one channel: the plan must have C = 1");
  if (!std::isfinite(contrast) || !(contrast > 1.0f)) return set_error(BLFLS_E_INVALID, "contrast must be finite and > 1");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return set_error(BLFLS_E_INVALID, "workspace must be 256-byte aligned");
  if (pitch < plan->W) return set_error(BLFLS_E_INVALID, "pitch must be >= W");
  int radius = 0;
  blfls_status st = check_params(params, &radius);
  if (st != BLFLS_OK) return st;
  size_t off_l, off_base, off_part;
  const size_t ws_bytes = tonemap_bytes(plan, *params, &off_l, &off_base, &off_part);
  const size_t img_bytes = 3 * static_cast<size_t>(plan->H) * pitch * sizeof(float);
  if (overlaps(out, img_bytes, rgb, img_bytes) || overlaps(out, img_bytes, workspace, ws_bytes))
    return set_error(BLFLS_E_INVALID, "out must not overlap rgb or the workspace");
  if (overlaps(rgb, img_bytes, workspace, ws_bytes))
    return set_error(BLFLS_E_INVALID, "rgb must not overlap the workspace");
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  float* L = reinterpret_cast<float*>(ws + off_l);
  float* base = reinterpret_cast<float*>(ws + off_base);
  float* part = reinterpret_cast<float*>(ws + off_part);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float floor_i = 1e-6f;
  hipError_t e = launch_tm_log(rgb, pitch, plan->H, plan->W, floor_i, L, s);
  if (e != hipSuccess) return hip_error(e, "kernel launch");
  st = blfls_smooth(plan, params, L, nullptr, base, plan->W, workspace, stream);
  if (st != BLFLS_OK) return st;
  e = launch_tm_finish(rgb, out, pitch, plan->H, plan->W, floor_i, L, base, part,
                       static_cast<float>(std::log10(static_cast<double>(contrast))), s);
  if (e != hipSuccess) return hip_error(e, "kernel launch");
  return BLFLS_OK;
}

blfls_status blfls_plan_destroy(blfls_plan_t plan) {
  g_last_error.clear();
  if (plan == nullptr) return set_error(BLFLS_E_INVALID, "plan is NULL");
  plan_free(plan);
  return BLFLS_OK;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

blfls_status blfls_smooth(blfls_plan_t plan, const blfls_params* params, const float* f, const float* guide,
                          float* u, int64_t pitch, void* workspace, void* stream) {
  g_last_error.clear();
  if (plan == nullptr) return set_error(BLFLS_E_INVALID, "plan is NULL");
  if (f == nullptr || u == nullptr) return set_error(BLFLS_E_INVALID, "f and u must not be NULL");
  if (workspace == nullptr) return set_error(BLFLS_E_INVALID, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return set_error(BLFLS_E_INVALID, "workspace must be 256-byte aligned");
  if (pitch < plan->W) return set_error(BLFLS_E_INVALID, "pitch must be >= W");
  int radius = 0;
  blfls_status st = check_params(params, &radius);
  if (st != BLFLS_OK) return st;
  const size_t img_bytes = static_cast<size_t>(plan->C) * plan->H * pitch * sizeof(float);
  if (overlaps(u, img_bytes, f, img_bytes) || (guide && overlaps(u, img_bytes, guide, img_bytes)) ||
      overlaps(u, img_bytes, workspace, request_workspace_bytes(plan, *params)))
    return set_error(BLFLS_E_INVALID, "u must not overlap f, guide or the workspace");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  if (dev != plan->device) return set_error(BLFLS_E_INVALID, "the current device differs from the plan's device");

  // descriptors: tables, then each array, 16-byte aligned, in the workspace
  RequestDesc rd;
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  uint8_t* dbase = ws + plan->off_desc;
  build_request(plan, *params, radius, f, guide, u, pitch, workspace, dbase, &rd);
  std::vector<uint8_t> blob;
  blob.reserve(8192);
  auto place = [&](const void* src, size_t n) {
    const size_t off = align_up(blob.size(), 16);
    blob.resize(off + n);
    std::memcpy(blob.data() + off, src, n);
    return off;
  };
  const int C = plan->C;
  place(&rd.tables, sizeof(RequestTables));
  const size_t o_b1 = place(rd.blf_first.data(), C * sizeof(BlfPlane));
  const size_t o_b2 = place(rd.blf_next.data(), C * sizeof(BlfPlane));
  const size_t o_m1 = place(rd.mm_first.data(), C * sizeof(AuxPlane));
  const size_t o_m2 = place(rd.mm_next.data(), C * sizeof(AuxPlane));
  const size_t o_mf = place(rd.mm_f.data(), C * sizeof(AuxPlane));
  const size_t o_g = place(rd.gauss.data(), C * sizeof(AuxPlane));
  const size_t o_f = place(rd.fft.data(), C * sizeof(FftPlane));
  const size_t o_fl = params->detail_gain != 0.0f ? place(rd.fft_last.data(), C * sizeof(FftPlane)) : o_f;
  size_t o_n1 = 0, o_n2 = 0;
  if (rd.filter == BLFLS_FILTER_NC) {
    o_n1 = place(rd.nc_first.data(), C * sizeof(NcPlane));
    o_n2 = place(rd.nc_next.data(), C * sizeof(NcPlane));
  } else if (rd.filter == BLFLS_FILTER_GRID) {
    o_n1 = place(rd.grid_first.data(), C * sizeof(GridPlane));
    o_n2 = place(rd.grid_next.data(), C * sizeof(GridPlane));
  } else if (rd.filter == BLFLS_FILTER_AMF) {
    o_n1 = place(rd.amf_first.data(), 2 * C * sizeof(AmfPlane));
    o_n2 = place(rd.amf_next.data(), 2 * C * sizeof(AmfPlane));
  }
  if (blob.size() > kDescBytes) return set_error(BLFLS_E_INVALID, "descriptor area overflow");
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    StageTimer t(BLFLS_STAGE_UPLOAD, s);
    e = launch_desc_copy(blob.data(), blob.size(), dbase, s);
  }
  if (e != hipSuccess) return hip_error(e, "descriptor upload");
  DeviceDesc dd;
  dd.blf_first = reinterpret_cast<const BlfPlane*>(dbase + o_b1);
  dd.blf_next = reinterpret_cast<const BlfPlane*>(dbase + o_b2);
  dd.mm_first = reinterpret_cast<const AuxPlane*>(dbase + o_m1);
  dd.mm_next = reinterpret_cast<const AuxPlane*>(dbase + o_m2);
  dd.mm_f = reinterpret_cast<const AuxPlane*>(dbase + o_mf);
  dd.gauss = reinterpret_cast<const AuxPlane*>(dbase + o_g);
  dd.fft = reinterpret_cast<const FftPlane*>(dbase + o_f);
  dd.fft_last = reinterpret_cast<const FftPlane*>(dbase + o_fl);
  if (rd.filter == BLFLS_FILTER_NC) {
    dd.nc_first = reinterpret_cast<const NcPlane*>(dbase + o_n1);
    dd.nc_next = reinterpret_cast<const NcPlane*>(dbase + o_n2);
  } else if (rd.filter == BLFLS_FILTER_GRID) {
    dd.grid_first = reinterpret_cast<const GridPlane*>(dbase + o_n1);
    dd.grid_next = reinterpret_cast<const GridPlane*>(dbase + o_n2);
  } else if (rd.filter == BLFLS_FILTER_AMF) {
    dd.amf_first = reinterpret_cast<const AmfPlane*>(dbase + o_n1);
    dd.amf_next = reinterpret_cast<const AmfPlane*>(dbase + o_n2);
  }
  e = enqueue_request(plan, rd, dd, s);
  if (e != hipSuccess) return hip_error(e, "kernel launch");
  return BLFLS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free variant: the workspace is a static device array of the
// library, so a call makes no device allocation at all.
// ---------------------------------------------------------------------------

// One copy per GPU, held from the module's load on that GPU until the process
// ends.  In host code `scratch` names a host-side stand-in, never the device
// memory: only the address hipGetSymbolAddress returns for the current device
// may be passed to kernels.
static __device__ __align__(256) unsigned char scratch[BLFLS_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device ordinal, nullptr until looked up
}  // namespace

// The device address of `scratch` on device `dev` (which must be current),
// looked up on the first call for that device.
static blfls_status scratch_for_device(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0) return set_error(BLFLS_E_INVALID, "no current device");
  if (g_scratch_ptr.size() <= static_cast<size_t>(dev)) g_scratch_ptr.resize(dev + 1, nullptr);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
    if (ptr == nullptr || reinterpret_cast<uintptr_t>(ptr) % 256 != 0)
      return set_error(BLFLS_E_HIP, "static scratch has no aligned device address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BLFLS_OK;
}

extern "C" {

blfls_status blfls_smooth_noalloc(blfls_plan_t plan, const blfls_params* params, const float* f,
                                  const float* guide, float* u, int64_t pitch, void* stream) {
  g_last_error.clear();
  if (plan == nullptr) return set_error(BLFLS_E_INVALID, "plan is NULL");
  if (params == nullptr) return set_error(BLFLS_E_INVALID, "params is NULL");
  int radius = 0;
  blfls_status st = check_params(params, &radius);
  if (st != BLFLS_OK) return st;
  const size_t need = request_workspace_bytes(plan, *params);
  if (need > BLFLS_NOALLOC_SCRATCH_BYTES)
    return set_error(BLFLS_E_NOMEM, "workspace of " + std::to_string(need) +
                                        " bytes exceeds the static scratch of BLFLS_NOALLOC_SCRATCH_BYTES (" +
                                        std::to_string(static_cast<size_t>(BLFLS_NOALLOC_SCRATCH_BYTES)) +
                                        "); use blfls_smooth with a caller workspace");
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  void* ws = nullptr;
  st = scratch_for_device(dev, &ws);
  if (st != BLFLS_OK) return st;
  // the workspace's contents on entry are ignored by every kernel of the call:
  // nothing in it needs clearing
  return blfls_smooth(plan, params, f, guide, u, pitch, ws, stream);
}

}  // extern "C"
