// Host-side launchers of the HIP kernels (one per kernel family).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include "blfls_internal.h"

namespace blfls {

// Kernel-argument payload used to upload descriptors without host staging.
struct DescChunk {
  uint32_t words[768];
};

// Radius class (kernel instantiation) for radius r, or -1 if r > kMaxR.
int blf_radius_class(int r);
int blf_tile_w();
int blf_tile_h();

hipError_t launch_desc_copy(const void* host_src, size_t bytes, void* dev_dst, hipStream_t s);
// work == nullptr: one workgroup per item (grid = total_items).  Otherwise a
// persistent launch: grid = total_items workgroups stride over the items of
// the work header (items, planes, descriptor array), read from device memory
// when the kernel runs.
hipError_t launch_blf(int R, const BlfPlane* planes, int nplanes, int total_items, bool joint,
                      int field_type, hipStream_t s, WorkHeader* work = nullptr);

// Symmetric-pair filter (Eq. (1) with one exp per unordered pair of taps): bands
// of at most 64 columns and whole blocks of K rows (geometry and record layout in
// blfls_pair_geom.h), their partial sums, and the merge pass that adds the
// neighbours' partial sums and writes the fields.
// Both passes: `items` band items (2 per band and plane), then `merge_items`
// merge items.  Persistent launches (work != nullptr) read their counts from
// the header's items / items2 and use grids of `items` and `merge_items`.
hipError_t launch_blf_pair(int R, const BlfPlane* planes, int nplanes, int items, int merge_items, bool joint,
                           int field_type, hipStream_t s, WorkHeader* work = nullptr);
size_t fft_rows_lds_bytes(int M, int rb);
size_t fft_cols_lds_bytes(int H, int cb);
// Column pass with one column per wave (H = 64 L): columns per workgroup, LDS bytes.
int fft_cols_wave_per_block();
size_t fft_cols_wave_lds_bytes(int L);
// Row passes with one row per wave (W/2 = 64 L): LDS bytes (rows per workgroup as above).
size_t fft_rows_wave_lds_bytes(int L);
hipError_t fft_init_kernels();
hipError_t launch_fft_rows_fwd(const FftPlane* planes, int nplanes, int blocks, size_t lds_bytes,
                               int field_type, hipStream_t s, WorkHeader* work = nullptr);
hipError_t launch_fft_cols(const FftPlane* planes, int nplanes, int blocks, size_t lds_bytes, hipStream_t s,
                           WorkHeader* work = nullptr);
hipError_t launch_fft_rows_inv(const FftPlane* planes, int nplanes, int blocks, size_t lds_bytes,
                               hipStream_t s, WorkHeader* work = nullptr);
// NC filter passes (NC-LS).  Items per plane of a row pass / a column pass;
// pass s in [0, npasses) is a row pass when even, the last writes the
// residual fields in field type.
int nc_row_items(int H, int W);
int nc_col_items(int H, int W);
hipError_t nc_init_kernels();
hipError_t launch_nc_pass(const NcPlane* planes, int nplanes, int items, int pass, int npasses, float r, int R,
                          int field_type, hipStream_t s);
// Bilateral-grid approximation: cell size for sigma_s, tiles (8 x 8 cells)
// across W and down H, and the launch over 2 fields x tiles of every plane.
int grid_cell_size(float sigma_s);
int grid_tiles_x(int W, int s);
int grid_tiles_y(int H, int s);
int grid_z_stride(const GridPlane& host_plane);
hipError_t grid_init_kernels();
// self: every plane's range source is its image (GridPlane::g == nullptr)
hipError_t launch_grid(const GridPlane* planes, int nplanes, int items, int zs, bool self, int field_type,
                       hipStream_t s);

// Adaptive-manifold filter: manifold slots of a tree of the given height,
// column-scan segments of an image of H rows, the kernels' LDS limits, and
// the whole filter (prep, root low-pass, depth-first walk of the manifolds;
// the last slice writes the residual fields).
int amf_slots(int height);
int amf_segments(int H);
hipError_t amf_init_kernels();
hipError_t launch_amf(const AmfGeom& geom, float* slots, int height, hipStream_t s);

// Log-domain tone mapping around one smooth of the log intensity: the log
// intensity of an RGB image, then the base's extrema and the recombination.
int tm_extrema_blocks();
hipError_t launch_tm_log(const float* rgb, int64_t pitch, int H, int W, float floor_i, float* L, hipStream_t s);
hipError_t launch_tm_finish(const float* rgb, float* out, int64_t pitch, int H, int W, float floor_i, const float* L,
                            const float* base, float* partial, float log_contrast, hipStream_t s);
hipError_t launch_minmax(const AuxPlane* planes, int nplanes, hipStream_t s, WorkHeader* work = nullptr,
                         int grid = 0);
hipError_t launch_gauss(const AuxPlane* planes, int nplanes, int64_t max_pixels, hipStream_t s,
                        WorkHeader* work = nullptr, int grid = 0);
int gauss_chunks();  // items per plane of the Gaussian passes

}  // namespace blfls
