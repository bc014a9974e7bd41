// Internal declarations shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace filark {

constexpr int kWave = 64;        // CDNA wavefront
constexpr int kMaxSections = 8;  // cascade length supported by the kernels
constexpr int kMaxBlock = 64;    // samples per lane block L: 32 or 64
constexpr int kMaxWaves = 9;     // data waves + 1 carry wave per workgroup

// Control words of one state object (device memory, uint32 each).
//   [0] ticket counter, [1] finished-tile counter, [2] launch epoch,
//   [3] error bits, [4..5] int64 global sample counter (STA/LTA objects).
enum { kCtrlTicket = 0, kCtrlDone = 1, kCtrlEpoch = 2, kCtrlError = 3, kCtrlCounter = 4, kCtrlWords = 8 };
enum { kErrTimeout = 1 };

// Look-back flag encoding: (epoch << 2) | status.
enum { kFlagAggregate = 1, kFlagInclusive = 2 };

// Parameters of the fused forward kernel (SOS cascade and/or STA/LTA).
struct FwdParams {
  const float *x;      // input  [n_t][n_ch]
  float *y;            // filter output [n_t][n_ch] or nullptr
  float *cf;           // characteristic function [n_t][n_ch] or nullptr
  int64_t n_ch;        // channels = row stride
  int32_t n_t;         // rows in this chunk
  int32_t n_seg;       // time segments per chunk (one workgroup row each)
  int32_t n_grp;       // channel groups of 64
  int32_t seg_len;     // rows per segment = waves * L

  // SOS cascade
  double *zs;          // state, two parity buffers of [2K][n_ch]
  const double *coef;  // [K][5] = b0, b1, b2, -a1, -a2
  const double *G;     // [L][2K]: A^(L-1-j) B, block-end state of a unit sample at j
  const double *P;     // [2K][2K]: A^L (one block)
  const double *Q;     // [n_seg][2K][2K]: (A^S)^m, m = 0 .. n_seg-1
  uint32_t *sos_ctrl;  // control words of the SOS object (epoch -> zs parity)

  // STA/LTA
  double *sl;          // state, two parity buffers of [2][n_ch] = (sta, lta)
  double asd, ald;     // FP64 decay factors 1 - 1/nsta, 1 - 1/nlta
  const double *slq;   // [2 + 2 q_cap]: alpha_s^L, alpha_l^L, alpha_s^(S m) (m < q_cap), alpha_l^(S m)
  int32_t q_cap;       // power-table capacity (>= n_seg, >= 2)
  uint32_t *sl_ctrl;   // control words of the STA/LTA object (epoch, counter)
  int64_t nlta;
  double nsta_d, nlta_d;
  float as, al;        // FP32 decay factors 1 - 1/nsta, 1 - 1/nlta
  float kappa;         // nlta / nsta (cf = kappa * S / L in the scaled sums)

  // look-back workspace of the launching object
  double *rec;         // SOS records, then STA/LTA records
  uint32_t *flags;     // [2][n_seg][n_grp]
  uint32_t *ctrl;      // launch control words (tickets, done, epoch, error)
  int32_t spin_limit;  // bounded wait (iterations) before flagging a timeout
};

// Dynamic LDS bytes of a forward workgroup with `waves` data waves.
size_t fwd_lds_bytes(int K, int waves);

// Host-side launcher (defined in fwd.hip).  K = 0 means STA/LTA only;
// `waves` data waves (<= kMaxWaves - 1) plus one carry wave per workgroup.
hipError_t launch_fwd(const FwdParams &p, int K, int L, bool stalta, bool write_y, int waves,
                      hipStream_t stream);

}  // namespace filark
