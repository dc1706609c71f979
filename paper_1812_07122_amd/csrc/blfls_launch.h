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
// FFT passes.  LDS layouts of a row-pass / column-pass workgroup (offsets in
// float2 units, total in bytes) and the persistent grid a pass gets on this
// device.  With work == nullptr a launch covers `items` items of `planes`
// (static per-XCD ranges); otherwise items and planes come from the work header.
int fft_lds_stride(int n);
void fft_rows_layout(int M, int rb, int pshift, int ntwM, int ntwW, int* r_split, int* r_data, size_t* bytes);
void fft_cols_layout(int H, int cb, int pshift, int ntwH, int* c_sy, int* c_sx, int* c_data, size_t* bytes);
int fft_grid(int pass, int field_type, size_t lds_bytes, int items);
hipError_t fft_init_kernels();
hipError_t launch_fft_rows_fwd(const FftPlane* planes, int nplanes, int items, int grid, size_t lds_bytes,
                               int field_type, hipStream_t s, WorkHeader* work = nullptr);
hipError_t launch_fft_cols(const FftPlane* planes, int nplanes, int items, int grid, size_t lds_bytes,
                           hipStream_t s, WorkHeader* work = nullptr);
hipError_t launch_fft_rows_inv(const FftPlane* planes, int nplanes, int items, int grid, size_t lds_bytes,
                               hipStream_t s, WorkHeader* work = nullptr);
hipError_t launch_minmax(const AuxPlane* planes, int nplanes, hipStream_t s, WorkHeader* work = nullptr,
                         int grid = 0);
hipError_t launch_gauss(const AuxPlane* planes, int nplanes, int64_t max_pixels, hipStream_t s,
                        WorkHeader* work = nullptr, int grid = 0);
int gauss_chunks();  // items per plane of the Gaussian passes

}  // namespace blfls
