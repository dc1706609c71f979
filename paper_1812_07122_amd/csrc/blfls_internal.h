// Internal descriptors shared by the HIP kernels and the host runtime.
//
// Every heavy kernel reads its work from descriptor arrays in device memory.
// The synchronous path writes them into the caller's workspace with a tiny
// setup kernel; the server uploads them from pinned host memory.  The same
// kernels therefore serve one image or a batch of images of uneven sizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blfls_pair_geom.h"

namespace blfls {

constexpr int kMaxR = 32;               // largest filter radius
constexpr int kSpan = 2 * kMaxR + 1;    // window taps per axis at kMaxR
constexpr int kMaxStages = 16;          // FFT stages per transform length
constexpr int kMaxFft = 4096;           // longest transform (W/2 or H)
constexpr int kFftThreads = 512;        // threads per FFT workgroup
constexpr int kFftLdsComplex = 8192;    // complex values per FFT workgroup (64 KiB)
constexpr int kFftRadix15Elems = 7680;  // complex values per FFT workgroup when a stage has radix 15
                                        // (one radix-15 butterfly per thread)
constexpr int kMinmaxBlocks = 256;      // partial-reduction blocks per plane

enum FieldType : int { kF32 = 0, kBF16 = 1, kF16 = 2 };

// Division by an invariant n via multiply-high and shift (valid for numerators < 2^31):
// q = (umulhi(x, mul) + x) >> shift.
struct FastDiv {
  uint32_t mul;
  uint32_t shift;
};

// One radix stage of a Stockham transform: it combines `radix` sub-transforms
// of length `ns`; per = N / radix butterflies per transform.  Its twiddles are
// W_N^(t k es), W_N = exp(-2 pi i / N), es = N / (ns radix), t < radix, k < ns.
struct FftStage {
  int radix, ns, per, es;
  FastDiv per_div, ns_div;
};

// One transform length N = prod of the stage radices.  Powers of W_N come from
// a two-level table: W_N^e = hi[e >> 6] * lo[e & 63] (lo: W_N^j, j < 64;
// hi: W_N^(64 j)); kTwLo + ceil(N / 64) entries in all.
struct FftSize {
  int n;
  int nstages;
  FftStage st[kMaxStages];
};

constexpr int kTwLo = 64;
constexpr int kTwMax = kTwLo + (kMaxFft * 2) / kTwLo + 1;  // entries of a two-level table (N <= 2 * kMaxFft)

// One channel plane for the bilateral-filter kernel (Eq. (1) on both
// gradient fields of one channel).
struct BlfPlane {
  const float* f;        // image whose gradients are filtered, [H][pitch]
  const float* g;        // range-source image (guide / previous output) or nullptr = f
  void* rx;              // residual r_x = BLF(p_x) - p_x, packed [H][W], field type
  void* ry;              // residual r_y
  const float* minmax;   // range-source gradient extrema partials (normalise flag) or nullptr
  int64_t pitch;         // elements per row of f
  int64_t gpitch;        // elements per row of g
  int H, W;
  int r;                 // radius actually used (dx loop bound), r <= kernel R
  int tiles_x;           // tiles across W
  int tile_begin;        // first linear tile index of this plane in the launch
  int tile_count;        // tiles_x * tiles_y
  float cx, cy;          // range scales sqrt(log2(e) / (2 sigma_r^2)) per field; 0 = range off
  const float* spatial;  // RequestTables::sy then ::ex of the request
  const float* fmm;      // FP16 fields: the image's gradient extrema partials (store scale), else nullptr
  // Symmetric-pair decomposition (BlfPairGeom): the items of the plane are its
  // bands (tile_begin / tile_count count bands instead of tiles), the merge pass
  // has its own items, and the partial sums live in `rec`.
  int nbx, nby;          // column bands (at most 64 columns) and row bands (whole blocks of pair_k rows)
  int max_nblk;          // most blocks in a row band
  int pair_r;            // radius class of the record layout
  int pair_k;            // rows per block, pair_block_rows(pair_r)
  int merge_begin;       // first merge item / 2 (a plane has 2 * merge_count merge items)
  int merge_count;       // merge items per field
  float2* rec;           // partial sums of field 0; field 1 follows at rec + rec_field
  int64_t rec_field;     // float2 elements per field
};

// Per-request tables built in FP64 on the host and rounded to FP32.
struct RequestTables {
  float sy[kSpan];       // log2 spatial weight per row offset dy+kMaxR: -dy^2 log2(e)/(2 sigma_s^2), -inf beyond r
  float ex[kSpan];       // spatial weight per column offset dx+kMaxR: 2^(-dx^2 log2(e)/(2 sigma_s^2))
  float gw[kSpan];       // normalised 1-D Gaussian of the guide smoothing, index d+kMaxR
  float pw[(kMaxR + 1) * (kMaxR + 1)];  // log2 spatial weight at |offset| (dx, dy): pw[dx (kMaxR+1) + dy], -inf beyond r
};

// One channel plane for the three FFT passes (Eq. (8) in residual form).
struct FftPlane {
  const void* rx;        // residual fields, packed [H][W], field type
  const void* ry;
  float2* spec;          // half spectrum, transposed: [W/2+1][H] complex
  const float* f;        // input plane [H][pitch]
  float* u;              // output plane [H][pitch]
  int64_t pitch;
  int H, W;
  float lambda;
  float gain;            // scale of delta: 1, or 1 - m for detail gain m on the last iteration
  int rb;                // rows per row-pass workgroup
  int cb;                // spectrum columns per column-pass workgroup
  int colw;              // L when H = 64 L is done one column per wave (L = 8, 16), else 0
  int roww;              // L when W/2 = 64 L is done one row per wave (L = 8, 16), else 0
  int row_begin, row_count;   // workgroups of the row passes
  int col_begin, col_count;   // workgroups of the column pass
  const FftSize* szM;    // W/2 complex transform
  const FftSize* szH;    // H complex transform
  const float2* twM;     // two-level table of W_{W/2}
  const float2* twH;     // two-level table of W_H
  const float2* twW;     // two-level table of W_W (split step, exponents k in [0, W/2])
  int ntwM, ntwH, ntwW;  // entries of the three tables
  const float* sx;       // 4 sin^2(pi k / W), k in [0, W/2]
  const float* sy;       // 4 sin^2(pi k / H), k in [0, H)
  FastDiv m_div;         // division by W/2
  FastDiv h_div;         // division by H
  FastDiv rb_div;        // division by rb
  const float* fmm;      // FP16 fields: the image's gradient extrema partials (store scale), else nullptr
};

// One channel plane for the NC filter passes (NC-LS, Section III-D): both
// gradient fields of one channel.  Pass s of the 2N passes reads buf[s % 2]
// (the first pass forms the gradients from f instead) and writes
// buf[(s + 1) % 2]; the last pass writes the residual fields rx, ry.
constexpr int kNcMaxR = 32;             // largest NC box radius in pixels
struct NcPlane {
  const float* f;        // image whose gradients are filtered, [H][pitch]
  const float* g;        // range-source image (guide / previous output) or nullptr = f
  int64_t pitch;         // elements per row of f
  int64_t gpitch;        // elements per row of g
  float* buf[2][2];      // [ping/pong][field] FP32 fields, packed [H][W]
  void* rx;              // residual r_x = NC(p_x) - p_x, packed [H][W], field type
  void* ry;
  const float* minmax;   // range-source gradient extrema partials (normalise flag) or nullptr
  int H, W;
  float a;               // sigma_s / sigma_r rounded to FP32 (0: range term off)
  int rbegin, rcount;    // items of the row passes: 2 fields x ceil(H/4) x ceil(W/64)
  int cbegin, ccount;    // items of the column passes: 2 fields x ceil(H/64) x ceil(W/64)
  int pad_;
  const float* fmm;      // FP16 fields: the image's gradient extrema partials (store scale), else nullptr
};

// One gradient field of one channel for the adaptive-manifold filter.
constexpr int kAmfMaxHeight = 6;        // manifold tree height at most
constexpr int kAmfSeg = 16;             // rows per segment of the column scans
struct AmfPlane {
  const float* f;        // image whose gradients are filtered, [H][pitch]
  const float* g;        // range-source image or nullptr = f
  int64_t pitch;
  int64_t gpitch;
  void* out;             // residual r = AMF(p) - p of this field, packed [H][W], field type
  const float* minmax;   // range-source gradient extrema partials (normalise flag) or nullptr
  int field;             // 0: x, 1: y
  int pad_;
  const float* fmm;      // FP16 fields: the image's gradient extrema partials (store scale), else nullptr
};

// One launch's view of the adaptive-manifold workspace (passed by value).
// Every array holds the P = 2C fields back to back, [P][H][W] per plane.
struct AmfGeom {
  const AmfPlane* planes;
  int P, H, W, S;        // fields, image size, column-scan segments (ceil(H / kAmfSeg))
  float a;               // step coefficient of the low-passes, exp(-sqrt(2) / sigma_s)
  float c0, c1;          // manifold step exp2(c0 + c1 |d eta| inv)
  float kpsi;            // splat / slice weight exp2(-kpsi ((eta - q) inv)^2)
  float tau;             // a child manifold exists where its low-passed weight is >= tau
  float* acc;            // [3][P][H][W]: sum psi Bn, sum psi Bd, max psi
  float* tmp;            // [4][P][H][W]: row-pass outputs
  const float* eta;      // manifold being splatted or split
  float* eta_out;        // root pass: the root manifold; split: [2][P][H][W] children
  float* sum;            // [P][S][5][W] segment summaries of a column scan
  float* carry_f;        // [P][S][4][W] carries into each segment, top to bottom
  float* carry_b;        // [P][S][4][W] and bottom to top
  float* inv;            // [2P] range scale of each field (1/span with the normalise flag, else 1),
                         // then each field's FP16 store scale (1 for FP32 and BF16)
  int ft;                // residual field type
  int first, last;       // this slice starts / completes the sums
};

// One channel plane for the bilateral-grid approximation of Eq. (1): both
// gradient fields of one channel, tiles of 10 x 10 grid cells per field.
constexpr int kGridZMax = 32;           // range bins at most
constexpr int kGridMaxCell = 32;        // spatial cell size at most (pixels)
struct GridPlane {
  const float* f;        // image whose gradients are filtered, [H][pitch]
  const float* g;        // range-source image or nullptr = f
  int64_t pitch;
  int64_t gpitch;
  void* rx;              // residual r_x = grid(p_x) - p_x, packed [H][W], field type
  void* ry;
  const float* minmax;   // range-source gradient extrema partials (always)
  int H, W;
  int s;                 // spatial cell size in pixels
  int tiles_x;           // tiles across W (10 cells each)
  int tile_begin;        // first tile index of this plane in the launch
  int tile_count;        // tiles per field
  float inv_r;           // 1 / sigma_r rounded to FP32 (0: range term off)
  float sigma_r;         // sigma_r (FP32): the range blur is sigma_r * inv cells wide
  float sig_xy;          // sigma_s / s: the spatial blur width in cells
  int normalize;         // divide the range scale by the field's span
  const float* fmm;      // FP16 fields: the image's gradient extrema partials (store scale), else nullptr
};

// Minmax (normalise flag) and Gaussian-guide descriptors.
struct AuxPlane {
  const float* src;      // range-source image [H][pitch]
  float* dst;            // Gaussian output [H][W] (guide smoothing) or nullptr
  float* tmp;            // [H][W] scratch of the separable Gaussian
  float* partial;        // kMinmaxBlocks * 4 floats
  int64_t pitch;
  int H, W;
  int rg;                // Gaussian radius
  int pad_;
  const float* gw;       // RequestTables::gw
};

// Work of one kernel family in a persistent launch, read from device memory
// when the kernel runs (so a captured graph replays with new work): item
// counts, plane counts, the plane descriptor array, and the item counters the
// workgroups draw from (zero when uploaded; one per XCD for the FFT passes so
// consecutive row blocks stay on one XCD).
constexpr int kXcds = 8;
struct WorkHeader {
  int items;         // work items (FFT: row blocks)
  int nplanes;
  int items2;        // FFT column blocks
  int pad_;
  const void* planes;
  int next[3][kXcds];  // counters: [0] filter / rows_fwd / aux, [1] cols, [2] rows_inv
  uint64_t pad2_;
};
static_assert(sizeof(WorkHeader) == 128, "work header size");

}  // namespace blfls
