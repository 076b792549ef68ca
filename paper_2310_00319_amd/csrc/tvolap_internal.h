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
  const int32_t* ch_row_base;  // [C] first partial-spectrum row of channel c
  const int32_t* ch_nchunks;   // [C] partition chunks of channel c (rows per tile)
  const int32_t* in_ch_ptr;    // [I+1] channels of input i: in_ch[in_ch_ptr[i] .. in_ch_ptr[i+1])
  const int32_t* in_ch;        // [C]
  int32_t tile_width;          // bins per MAC tile (64 V)
  // Output buses: bus e is the sum of channels out_ch[out_ptr[e] .. out_ptr[e+1])
  // (without a mixdown, bus c is channel c alone).
  int32_t n_out;
  const int32_t* out_ptr;      // [n_out+1]
  const int32_t* out_ch;       // [C]
  float2* ybus;                // [n_out][2L] bus spectra of one block (mixdown only, else NULL)
};

// One unit of per-block work. kind 1: the new spectrum of input `input`.
// kind 0: spectral MAC of a bin tile of up to 4 channels that share an input,
// over the partitions [max(m0, 1), m1) (chunk `chunk` of the channels'
// partition range; the m = 0 term is added when the channel is completed).
// Channel g writes its partial spectrum tile to row[g] of the partial buffer;
// the rows of a channel are contiguous, ordered (tile, chunk), nch chunks per
// tile (the same for all channels of an item).
struct WorkItem {
  int32_t input, n_ch, m0, m1;
  int32_t tile, chunk, kind, nch;
  int32_t ch[4];
  int32_t row[4];
};

// Everything the fused per-block kernel touches.
struct BlockArgs {
  DevPlan P;
  const WorkItem* items;
  int32_t n_items;
  const void* bank;
  void* fdl;
  const int32_t* sel;          // slots of this block (caller's device array or the handle's)
  int32_t* sel_store;          // handle's selection, updated when sel is the caller's
  int32_t copy_sel;
  const float* in;
  int64_t in_stride;
  float* hist;                 // [2][I][L]
  float2* ypart;               // [rows][tile_width]
  int32_t* arrive;             // [C] work items finished per channel in this block
  const int32_t* needed;       // [C] work items per channel
  int32_t* done;               // [1] work items finished in this block
  float* ola;                  // [C][3L]
  float* out;
  int64_t out_stride;
  uint64_t* counter;           // calls processed so far
  int32_t inverse_inline;      // 1: last item of a channel transforms back; 0: a later kernel does
};

struct MacShape {
  int32_t V;    // complex bins per lane (tile width = 64 V)
  int32_t G;    // channel capacity of a work item (1, 2 or 4)
  int32_t NW;   // waves per workgroup (split the partition range)
  int32_t E = 0;  // batched MAC engine: 0 = vector ALU (k_tmac), 1 = matrix cores (k_tmfma)
};

// Launchers (tvolap_kernels.hip). dtype: 0 = f32, 1 = bf16, 2 = f16.
hipError_t launch_fwd(const DevPlan& P, int dtype, const float* in, int64_t in_stride,
                      float* hist, void* fdl, const uint64_t* counter, hipStream_t s);
hipError_t launch_mac(const DevPlan& P, int dtype, const MacShape& shape, const WorkItem* items,
                      int n_items, const void* bank, const void* fdl, const int32_t* sel,
                      float2* ypart, const uint64_t* counter, hipStream_t s);
hipError_t launch_inv(const DevPlan& P, int dtype, const float2* ypart, const void* bank, const void* fdl,
                      const int32_t* sel, float* ola, float* out, int64_t out_stride, int32_t copy_sel,
                      int32_t* sel_store, int32_t* done, uint64_t* counter, hipStream_t s);
hipError_t launch_block(const BlockArgs& A, int dtype, const MacShape& shape, int grid, hipStream_t s);

// Batches of consecutive blocks (k_batch_spectra, k_tmac / k_tmfma,
// k_batch_out in tvolap_kernels.hip).
struct BatchArgs {
  DevPlan P;
  const WorkItem* items;       // time-blocked MAC items (partitions from 0)
  int32_t n_mac;
  int32_t n_blocks;
  int32_t n_rows;              // partial rows of one block
  int32_t tile_width;          // bins per item tile (64 V NW)
  int32_t time_block;          // blocks of one parity per MAC time group (8 or 16)
  const int32_t* row_base;     // [C] first partial row of channel c (rows ordered tile, chunk)
  const int32_t* nchunks;      // [C] partition chunks of channel c
  const void* bank;
  void* fdl;
  const int32_t* sel;          // [n_blocks][sel_stride] slots (caller's or the handle's with stride 0)
  int64_t sel_stride;
  int32_t* sel_store;
  int32_t copy_sel;
  float2* ypart;               // [n_max][rows][tile_width]
  float* ola_state;            // [C][3L]
  int32_t* done;               // [1] workgroups of the batch's last launch finished
  uint64_t* counter;
  int32_t bus_rows;            // 1: mixdown; bus sums are formed in the partial rows before the inverse
  // Work units (time groups of an item) that the matrix-core MAC leaves to
  // the vector-ALU MAC: irregular slot patterns and ragged channel pairs.
  int32_t* defer_list;         // [units]
  int32_t* defer_count;        // [1], zeroed by the spectra kernel of each call
  int32_t from_list;           // k_tmac: process defer_list[0 .. *defer_count)
};
// ev (may be NULL): four events recorded before the spectra, before the MAC,
// after the MAC and after the overlap-add.
hipError_t launch_batch(const BatchArgs& B, int dtype, const MacShape& shape, int grid, const float* in,
                        int64_t in_stride, float* hist, float* ola, float* out, int64_t out_stride, hipStream_t s,
                        hipEvent_t* ev);
hipError_t launch_irprep(const DevPlan& P, int dtype, const float* taps, int32_t n_taps, int32_t M,
                         void* dst, hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// One slot of every channel from device taps [C][taps_stride] (part_base:
// [C+1] prefix sums of the partition counts; ch_taps: [C] taps per channel).
hipError_t launch_irprep_all(const DevPlan& P, int dtype, const int32_t* part_base, int32_t total_parts,
                             const int32_t* ch_taps, const float* taps, int64_t taps_stride, int32_t slot, void* bank,
                             hipStream_t s);

// The same launchers for one hop L and storage type DT, instantiated by the
// kernel file compiled for that pair; launch_fwd and the others above pick one
// by P.L and dtype.
template <int L, int DT>
hipError_t hop_fwd(const DevPlan& P, int dtype, const float* in, int64_t in_stride, float* hist, void* fdl,
                   const uint64_t* counter, hipStream_t s);
template <int L, int DT>
hipError_t hop_inv(const DevPlan& P, int dtype, const float2* ypart, const void* bank, const void* fdl,
                   const int32_t* sel, float* ola, float* out, int64_t out_stride, int32_t copy_sel,
                   int32_t* sel_store, int32_t* done, uint64_t* counter, hipStream_t s);
template <int L, int DT>
hipError_t hop_block(const BlockArgs& A, int dtype, const MacShape& shape, int grid, hipStream_t s);
template <int L, int DT>
hipError_t hop_batch(const BatchArgs& B, int dtype, const MacShape& shape, int grid, const float* in,
                     int64_t in_stride, float* hist, float* ola, float* out, int64_t out_stride, hipStream_t s,
                     hipEvent_t* ev);
template <int L, int DT>
hipError_t hop_irprep(const DevPlan& P, int dtype, const float* taps, int32_t n_taps, int32_t M, void* dst,
                      hipStream_t s);
template <int L, int DT>
hipError_t hop_irprep_all(const DevPlan& P, int dtype, const int32_t* part_base, int32_t total_parts,
                          const int32_t* ch_taps, const float* taps, int64_t taps_stride, int32_t slot, void* bank,
                          hipStream_t s);
template <int DT>
hipError_t mac_dt(const DevPlan& P, int dtype, const MacShape& shape, const WorkItem* items, int n_items,
                  const void* bank, const void* fdl, const int32_t* sel, float2* ypart, const uint64_t* counter,
                  hipStream_t s);

}  // namespace tvx
