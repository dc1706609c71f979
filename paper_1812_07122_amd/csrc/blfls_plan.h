// Host-side plan and request building shared by the synchronous path and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/blfls.h"
#include "blfls_internal.h"

struct blfls_plan_s {
  int H = 0, W = 0, C = 0, M = 0;
  blfls_precision precision = BLFLS_FP32;
  int device = 0;
  // plan-owned device tables (one allocation)
  void* dev_tables = nullptr;
  const blfls::FftSize* szM = nullptr;
  const blfls::FftSize* szH = nullptr;
  const float2* twM = nullptr;
  const float2* twH = nullptr;
  const float2* twW = nullptr;
  const float* sx = nullptr;
  const float* sy = nullptr;
  int ntwM = 0, ntwH = 0, ntwW = 0;
  // FFT pass geometry
  int rb = 1, cb = 1;
  int colw = 0;                         // column pass one column per wave for H = 64 colw
  int roww = 0;                         // row passes one row per wave for W/2 = 64 roww
  int row_blocks = 0, col_blocks = 0;   // per channel
  size_t lds_rows = 0, lds_cols = 0;
  // BLF geometry
  int tiles_x = 0, tiles_y = 0;
  // workspace layout (bytes from the workspace base)
  size_t field_elem = 4;
  size_t off_desc = 0, off_partial = 0, off_fpartial = 0, off_rx = 0, off_ry = 0, off_spec = 0, off_gauss = 0, off_tmp = 0, off_nc = 0;
  size_t ws_bytes = 0;
};

namespace blfls {

constexpr size_t kDescBytes = 64 * 1024;

// Thread-local error message helpers.
blfls_status set_error(blfls_status st, const std::string& msg);
blfls_status hip_error(hipError_t e, const char* where);

FastDiv make_fastdiv(uint32_t d);

// NC filter geometry: box radius of round k of n, and the farthest pixel a
// box of FP32 radius r reaches.
double nc_box_radius(float sigma_s, int n, int k);
int nc_pixel_radius(float r);

// Size and parameter validation shared by the ABI entry points.
blfls_status check_shape(int H, int W, int C);
blfls_status check_params(const blfls_params* p, int* radius_out);

// Adaptive-manifold filter: tree height of a request (filter_iterations, or
// the default rule from sigma_s and sigma_r), and the workspace bytes a
// request needs (the plan's, plus the manifold arrays for the AMF).
int amf_tree_height(const blfls_params& p);
size_t request_workspace_bytes(const blfls_plan_s* plan, const blfls_params& p);

// Plans keyed by shape, created on demand (used by the server).
blfls_status plan_create(int H, int W, int C, blfls_precision prec, blfls_plan_s** out);
void plan_free(blfls_plan_s* p);

// Everything one request needs to queue its kernels.
struct RequestDesc {
  RequestTables tables;
  std::vector<BlfPlane> blf_first;   // iteration 1
  std::vector<BlfPlane> blf_next;    // iterations 2..n (range source = previous output)
  std::vector<AuxPlane> mm_first;    // normalise: extrema of iteration 1's range source
  std::vector<AuxPlane> mm_next;
  std::vector<AuxPlane> mm_f;        // FP16 fields: extrema of the image's own gradients (store scales)
  std::vector<AuxPlane> gauss;       // guide smoothing
  std::vector<FftPlane> fft;
  std::vector<FftPlane> fft_last;    // the last iteration's (detail gain folded in)
  std::vector<GridPlane> grid_first; // bilateral grid: iteration 1
  std::vector<GridPlane> grid_next;  // and iterations 2..n
  std::vector<NcPlane> nc_first;     // NC-LS: the NC passes of iteration 1
  std::vector<NcPlane> nc_next;      // and of iterations 2..n
  std::vector<AmfPlane> amf_first;   // AMF-LS: both fields of each channel, iteration 1
  std::vector<AmfPlane> amf_next;    // and iterations 2..n
  AmfGeom amf_geom{};                // workspace arrays and constants (planes set at launch)
  float* amf_slots = nullptr;        // manifold slots
  int amf_height = 0;                // manifold tree height
  int filter = BLFLS_FILTER_BLF;
  int nc_rounds = 0;                 // NC rounds (a row and a column pass each)
  float nc_r[8] = {};                // box radius of each round (FP32)
  int nc_R[8] = {};                  // farthest pixel offset of each round
  bool joint_first = false;
  int R = 0;                         // kernel radius class
  bool pair = false;                 // BLF by the symmetric-pair kernel (partial sums after the plan's workspace)
  int pair_items = 0;                // its band items, all channels
  int merge_items = 0;               // its merge items, all channels
  int iterations = 1;
  bool normalize = false;
  bool smooth_guide = false;
  bool fp16_scale = false;           // FP16 fields: the image's gradient extrema set the store scales
};

// Build the descriptors of one request whose workspace starts at `ws`; the
// request's RequestTables will live at device address `dev_tables`.  Plane
// tile/block offsets are set for a launch of this request alone; the server
// rebases them when it batches several requests into one launch.
void build_request(const blfls_plan_s* plan, const blfls_params& prm, int radius, const float* f,
                   const float* guide, float* u, int64_t pitch, void* ws, const void* dev_tables,
                   RequestDesc* out);

// Queue one request's kernels on `s`, reading descriptors already resident at
// the device addresses in `dev` (arrays laid out as in RequestDesc).
struct DeviceDesc {
  const BlfPlane* blf_first = nullptr;
  const BlfPlane* blf_next = nullptr;
  const AuxPlane* mm_first = nullptr;
  const AuxPlane* mm_next = nullptr;
  const AuxPlane* mm_f = nullptr;
  const AuxPlane* gauss = nullptr;
  const FftPlane* fft = nullptr;
  const FftPlane* fft_last = nullptr;
  const GridPlane* grid_first = nullptr;
  const GridPlane* grid_next = nullptr;
  const NcPlane* nc_first = nullptr;
  const NcPlane* nc_next = nullptr;
  const AmfPlane* amf_first = nullptr;
  const AmfPlane* amf_next = nullptr;
};
hipError_t enqueue_request(const blfls_plan_s* plan, const RequestDesc& rd, const DeviceDesc& dev,
                           hipStream_t s);

}  // namespace blfls
