// Internal declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvx {

// Read-only plan tables in device memory plus the scalar sizes.
// Spectra are stored as 2L complex values: slot 0 holds (Re X(0), Re X(2L)),
// slots 1 .. 2L-1 hold X(k). Offsets are in stored complex elements.
struct DevPlan {
  int32_t L;              // hop; transforms are 4L real = 2L complex points
  int32_t C, I, K;        // channels, inputs, IR slots per channel
  const int32_t* ch_input;     // [C]
  const int32_t* ch_M;         // [C] partitions per channel
  const int64_t* ch_bank_off;  // [C] start of channel c in the bank ([K][M_c][2L])
  const int32_t* in_M;         // [I] delay-line length per parity
  const int64_t* in_fdl_off;   // [I] start of input i in the delay line ([2][M_i][2L])
  const float2* tw;            // [4L] exp(-2 pi i t / 4L), from double precision
  const float* win;            // [2L] periodic Hann window, amplitude 1/2
};

// One unit of spectral-MAC work: a bin tile of up to 4 channels that share an
// input, over the partitions [m0, m1). Channel g of the item writes its partial
// spectrum tile to row (row + g) of the partial buffer.
struct WorkItem {
  int32_t input, n_ch, m0, m1;
  int32_t tile, row, pad0, pad1;
  int32_t ch[4];
};

struct MacShape {
  int32_t V;    // complex bins per lane (tile width = 64 V)
  int32_t G;    // channel capacity of a work item (1, 2 or 4)
  int32_t NW;   // waves per workgroup (split the partition range)
};

// Launchers (tvolap_kernels.hip). dtype: 0 = f32, 1 = bf16, 2 = f16.
hipError_t launch_fwd(const DevPlan& P, int dtype, const float* in, int64_t in_stride,
                      float* hist, void* fdl, const uint64_t* counter, hipStream_t s);
hipError_t launch_mac(const DevPlan& P, int dtype, const MacShape& shape, const WorkItem* items,
                      int n_items, const void* bank, const void* fdl, const int32_t* sel,
                      float2* ypart, const uint64_t* counter, hipStream_t s);
hipError_t launch_inv(const DevPlan& P, int tile_width, const float2* ypart, const int32_t* rows_ptr,
                      const int32_t* rows, float* ola, float* out, int64_t out_stride,
                      const int32_t* sel_in, int32_t* sel_store, uint64_t* counter, hipStream_t s);
hipError_t launch_irprep(const DevPlan& P, int dtype, const float* taps, int32_t n_taps, int32_t M,
                         void* dst, hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace tvx
