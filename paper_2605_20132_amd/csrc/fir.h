// Launch interface of the realtime FIR kernel (fir.hip), used by api.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace filark {

// Tap chunk: taps are applied KC at a time from SGPRs; the device tap array
// is padded with zeros to a multiple of KC.
constexpr int kFirChunk = 32;

// One launch covers a window of rows [T0, T0 + n_rows) of the chunk, in
// workgroups of nw waves stacked in time over one group of 64 channels; each
// wave computes R consecutive output rows of its 64 channels.  Row numbers
// inside the kernel are relative to T0 ("window rows").
struct FirParams {
  const float *x;    // chunk row lo = max(0, T0 - (Mp - 1)): base of the input reads
  float *y;          // chunk row T0
  const float *h;    // taps [Mp], FP32, zero past the filter length
  float *hist0, *hist1;  // history buffers [M - 1][n_ch], oldest row first: a call
                         // reads the one ctl[0] names and writes the other
  const uint32_t *ctl;   // [0] & 1: which buffer holds the history (flipped by launch_fir_flip)
  int64_t n_ch;
  int32_t xoff;       // T0 - lo: window row 0 sits xoff rows past the input base
  int32_t n_rows;     // rows in this window
  int32_t range;      // readable input bytes from x (through the window's end)
  int32_t out_range;  // n_rows * n_ch * 4
  int32_t hrange;     // (M - 1) * n_ch * 4
  int32_t hm;         // M - 1
  int32_t n_chunks;   // Mp / kFirChunk
  int32_t hs;         // window row where the new history starts: n_t - (M - 1) - T0
  int32_t hcopy;      // history rows carried over unchanged (chunks shorter than M - 1)
  int32_t hsrc;       // first carried-over row of the history read (n_t)
  int32_t n_cg, n_tb;  // channel groups of 64, workgroups along the window's rows
  int32_t per_xcd, nw;
  int32_t chan_minor;  // workgroup order 0, 1 or 2 (fir_tile_of); for 2, per_xcd is the slab width in groups
};

// Output rows per wave that the kernels are compiled for.
inline bool fir_rows_ok(int R) { return R == 16 || R == 32 || R == 48; }

hipError_t launch_fir(const FirParams &p, int R, hipStream_t stream);

// FFT filtering (fft.hip): blocks of B = kFftN - (M - 1) output rows, each
// from a window of kFftN input rows (overlap-save); then the new history is
// written to the buffer ctl[0] does not name.  M <= 1024.
constexpr int kFftN = 2048;
struct FftParams {
  const float *x;         // chunk [n_t][n_ch]
  float *y;               // output [n_t][n_ch]
  const float2 *tw;       // [1024] W_1024^j, then [1024] W_2048^k (FP32 of FP64 values)
  const float2 *H;        // [1025] the taps' 2048-point spectrum, scaled by 1 / 4096
  float *hist0, *hist1;   // history buffers [M - 1][n_ch] (as FirParams)
  uint32_t *ctl;          // [0] & 1: the current history buffer; [1]: workgroups done (the last flips [0])
  int64_t n_ch, n_t;
  int32_t hm;             // M - 1
  int32_t B;              // output rows per block
  int32_t ch;             // channels per workgroup: 4 or 8
  int32_t threads;        // threads per workgroup: 256, or 512 with 8 channels
  int32_t per_xcd;        // channel groups per XCD slab (set by the launcher)
  uint32_t total;         // workgroups that do work (set by the launcher)
};
hipError_t launch_fir_fft(const FftParams &p, hipStream_t stream);

// Ends a call: the history buffer its launches wrote becomes the current one
// (a one-lane kernel, so that graph replays alternate the buffers too).
hipError_t launch_fir_flip(uint32_t *ctl, hipStream_t stream);

}  // namespace filark
