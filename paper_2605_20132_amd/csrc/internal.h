// Internal declarations shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace filark {

constexpr int kWave = 64;        // CDNA wavefront
constexpr int kMaxSections = 8;  // cascade length supported by the kernels
constexpr int kMaxWaves = 8;     // waves per workgroup
constexpr int kMaxLevels = 9;    // scan levels: blocks per window <= 2^9

// Parameters of the fused forward kernel (SOS cascade and/or STA/LTA).
//
// Work split: channel group g (cw = 2^cw_log2 consecutive channels) belongs to
// one workgroup, which covers a window of up to NB = nw * 64 / cw blocks of L
// rows.  Lane (r, cl) of wave w holds channel g*cw + cl and block
// b = w * (64 / cw) + r.  Longer chunks are launched window by window.
struct FwdParams {
  const float *x;      // input  [n_t][n_ch]
  float *y;            // filter output [n_t][n_ch] or nullptr
  float *cf;           // characteristic function [n_t][n_ch] or nullptr
  int64_t n_ch;        // channels = row stride
  int32_t n_t;         // rows in this launch (1 .. NB * L)
  int32_t cw_log2;     // log2 of channels per group
  int32_t nw;          // waves per workgroup
  int32_t n_grp;       // channel groups
  int32_t per_xcd;     // channel groups per XCD slab (ceil(n_grp / 8))
  int32_t n_lev;       // scan levels (>= 1; level k spans 2^k blocks)
  int32_t range;       // bytes of one [n_t][n_ch] FP32 array (buffer range)
  int32_t out_range;   // buffer range of y and cf: `range`, or 0 to write neither (states only)
  int32_t nt;          // 1: y and cf stores carry the non-temporal hint (groups of >= 16 channels)
  int32_t order;       // channel-group order within an XCD (dev::group_of)
  // state checkpoints (for the adjoint): at the start of block b, for every
  // b that is a multiple of ck_blocks (b = 0 only if ck_first), the filter
  // state [2K][n_ch], the STA/LTA state [2][n_ch] and the sample counter
  // [n_ch] (int64 in a double slot) go to ck + (b / ck_blocks) * ck_stride;
  // ck_blocks = 0: none
  double *ck;
  int64_t ck_stride;
  int32_t ck_blocks;
  int32_t ck_first;

  // SOS cascade
  double *zs;          // carried state [2K][n_ch], updated in place
  const double *coef;  // [K][5] = b0, b1, b2, -a1, -a2
  const double *G;     // [L][2K]: A^(L-1-j) B, block-end state of a unit sample at row j
  const double *Pw;    // [n_lev][2K][2K]: A^(L 2^k)

  // STA/LTA
  double *sl;          // carried state [2][n_ch] = (sta, lta), updated in place
  int64_t *cnt;        // [n_ch] global sample counter (equal for all channels)
  const double *dpow;  // [n_lev][2] decays^(L 2^k), then [L + 1][2] decays^m
  double asd, ald;     // FP64 decay factors 1 - 1/nsta, 1 - 1/nlta
  double nsta_d, nlta_d;
  int64_t nlta;
  float as, al;        // FP32 decay factors
  float kappa;         // nlta / nsta (cf = kappa * S / L in the scaled sums)
};

// Parameters of the adjoint kernel: one window of a chunk, processed after
// the windows that follow it (reverse time).  Same work split as FwdParams.
// The forward state at the window start is a checkpoint (read only); the
// adjoint state is read as the adjoint after the window and overwritten with
// the adjoint before it.
struct AdjParams {
  const float *x;      // input [n_t][n_ch]
  const float *g;      // dL/dcf (mode 0) or the target cf (mode 1) [n_t][n_ch]
  float *gx;           // dL/dx [n_t][n_ch]
  int64_t n_ch;
  int32_t n_t;         // rows in this launch (1 .. NB * L)
  int32_t cw_log2, nw, n_grp, per_xcd, n_lev, range;
  int32_t mode;        // 0: g = dL/dcf;  1: g = target, loss = scale * sum (cf - g)^2
  double scale;
  const double *zs0;   // forward filter state at the window start [2K][n_ch]
  const double *sl0;   // forward (sta, lta) at the window start [2][n_ch]
  const int64_t *cnt0; // global sample index of the window start [n_ch]
  double *adj;         // adjoint state [2K + 2][n_ch]: (u1, u2) per section, then sta, lta
  double *gpart;       // [n_grp][5K] coefficient-gradient sums of each group, added to
  const double *coef, *G, *Pw;  // forward tables (as FwdParams)
  const double *rinv;  // [K]: 1 / (-a2), or 1 / (-a1) for a first-order section (rebuilding variant)
  int32_t first_order; // bit k: section k is first order (a2 = b2 = 0)
  int32_t recon;       // section signals: 0 stored, 1 rebuilt backwards (second-order sections only),
                       // 2 rebuilt with first-order sections among them (adj_kernel RC)
  const double *dpow;           // [n_lev][2] decays^(L 2^k), then [L + 1][2] decays^m
  double asd, ald;     // 1 - 1/nsta, 1 - 1/nlta
  double cs, cl;       // 1/nsta, 1/nlta
  int64_t nlta;
  // several windows in one launch (n_win > 1, default adjoint tile only):
  // x, g, gx, zs0, sl0, cnt0, n_t and `range` describe the launch's first
  // window (a full one); window i is offset by i * win_elems elements of x, g, gx and by
  // i * ck_stride doubles of the start-state slots (zs0, sl0, cnt0 alike)
  int32_t n_win;
  int64_t win_elems;
  int64_t ck_stride;
  // rows and buffer range of the launch's last window: n_t and range for a
  // launch of full windows, fewer for a chunk's partial last window
  int32_t n_t_last, range_last;
};

// The several-window adjoint kernel runs the default adjoint tile only
// (16-row blocks, 4 waves, 8 channels: 32 blocks, 5 scan levels), with all
// of its LDS static: an x prefetch buffer of 4 x 16 x 64 floats and the
// handed-over adjoint state of the group's 8 channels besides the exchanges.
constexpr int kMultiWaves = 4;
constexpr int kMultiGroup = 8;
constexpr int kMultiCwLog2 = 3;
constexpr int kMultiLevels = 5;
// Cascades of more sections spill registers in that kernel (and so run one
// launch per window).
constexpr int kMultiMaxSections = 4;
inline bool adj_multi_fits(int nw, int cw, int L, int n_lev) {
  return L == 16 && nw == kMultiWaves && cw == kMultiGroup && n_lev == kMultiLevels;
}

// Two-threshold trigger on cf (one window of a chunk).  Same work split as
// FwdParams with 48-row blocks.  Carried per channel: open flag, start of the
// open event (global sample index) and the global sample counter.  Events
// closing in the window are appended to ev[cap][3] = (channel, t_on, t_off)
// at positions reserved on *count (which counts every event, stored or not).
struct TrigParams {
  const float *cf;     // [n_t][n_ch]
  int64_t n_ch;
  int32_t n_t;         // rows in this launch (1 .. NB * 48)
  int32_t cw_log2, nw, n_grp, per_xcd, range;
  float on, off;
  int32_t *open;       // [n_ch] 0 / 1, updated in place
  int64_t *t_on;       // [n_ch], updated in place
  int64_t *cnt;        // [n_ch] global sample index of the window start, advanced
  int64_t *ev;         // [cap][3]
  int64_t cap;
  unsigned long long *count;
};

hipError_t launch_trig(const TrigParams &p, int L, hipStream_t stream);

// The monitor launch: one window of the fused forward (SOS + STA/LTA, y and
// cf optional) whose cf goes on in registers to the trigger; t describes the
// same window and channel groups (t.cf and t.range unused).
struct MonParams {
  FwdParams f;
  TrigParams t;
};
hipError_t launch_monitor(const MonParams &p, int K, bool write_y, bool unit, hipStream_t stream);

// Stateful exponential-average operator (running-mean removal or running
// AGC), one window of a chunk; same work split as FwdParams, 48-row blocks.
struct EmaParams {
  const float *x;      // [n_t][n_ch]
  float *y;            // [n_t][n_ch] (may equal x)
  int64_t n_ch;
  int32_t n_t;         // rows in this launch (1 .. NB * 48)
  int32_t cw_log2, nw, n_grp, per_xcd, n_lev, range;
  int32_t mode;        // 0: y = x - mean; 1: y = x / sqrt(mean of x^2)
  double *avg;         // [n_ch] carried average, updated in place
  const double *dpow;  // [n_lev] a^(48 2^k), then [49] a^m
  double a, c;         // decay 1 - 1/n_win and weight 1/n_win
};

hipError_t launch_ema(const EmaParams &p, int L, hipStream_t stream);

// Batched forward launch (SOS only), one persistent kernel: an item is one
// channel group of one stream over every window of that stream's chunk (the
// consecutive descriptors descs[desc0 .. desc0 + n_win)), walked in order by
// one workgroup, which carries the state from window to window.  Items sit in
// 8 queues, one per XCD (queue x = items[qoff[x] .. qoff[x + 1])); the
// workgroups on XCD x take them in order from an atomic counter heads[x]
// until the queue is empty.  At the end of an item the workgroup raises
// stamps[stream] to its completion time.
struct BatchItem {
  int32_t desc0;   // descriptor of the first window
  int32_t n_win;   // windows
  int32_t K;       // sections
  int32_t group;   // channel group
  int32_t stream;
  int32_t pad[3];
};
struct BatchParams {
  const FwdParams *descs;
  const BatchItem *items;
  uint32_t *heads;             // [8] queue counters, then [1] workgroups done; the last
                               // workgroup to leave sets all 9 back to 0 for the next launch
  unsigned long long *stamps;  // [n_streams + 1]: completion stamps (raised with atomic max,
                               // so a launch's stamps exceed every earlier one's), then the
                               // start stamp (the first item taken from XCD 0's queue)
  int32_t qoff[9];
  int32_t n_streams;
};

// Dynamic LDS bytes of a forward workgroup.
size_t fwd_lds_bytes(int K, int nw, int n_lev, int cw);

// Launchers of one block length (fwd_l32.hip, fwd_l48.hip, fwd_l64.hip).
hipError_t launch_fwd_l32(const FwdParams &p, int K, bool stalta, bool write_y, bool unit, bool rev,
                          hipStream_t stream);
hipError_t launch_fwd_l48(const FwdParams &p, int K, bool stalta, bool write_y, bool unit, bool rev,
                          hipStream_t stream);
hipError_t launch_fwd_l64(const FwdParams &p, int K, bool stalta, bool write_y, bool unit, bool rev,
                          hipStream_t stream);

// Host-side launcher (defined in fwd.hip).  K = 0 means STA/LTA only.
hipError_t launch_fwd(const FwdParams &p, int K, int L, bool stalta, bool write_y, bool unit, bool rev,
                      hipStream_t stream);

// Batched launch: the persistent kernel (it leaves the queue counters cleared
// for the next launch), grid workgroups of nw waves with lds bytes of dynamic
// LDS, for cascades of up to kmax sections and 48-row blocks.  The occupancy
// query gives the workgroups of that kernel resident per CU.
hipError_t launch_fwd_batch(const BatchParams &bp, int kmax, int grid, int nw, size_t lds, hipStream_t stream);
hipError_t batch_occupancy(int kmax, int nw, size_t lds, int *per_cu);

// Channel groups per XCD slab and workgroups launched for n_grp groups.
inline int per_xcd_for(int n_grp) { return (n_grp + 7) / 8; }
inline int grid_for(int per_xcd) { return 8 * per_xcd; }
inline int fwd_grid(const FwdParams &p) { return grid_for(p.per_xcd); }

// Adjoint: LDS bytes, launcher (defined in adj.hip; L = 8 or 16, K = 1 .. 8),
// and the fixed-order sum of the per-group coefficient gradients into
// gsos[5K] (added to), which also clears gpart.
size_t adj_lds_bytes(int K, int nw, int n_lev);
hipError_t launch_adj(const AdjParams &p, int K, int L, bool unit, hipStream_t stream);
hipError_t launch_adj_reduce(double *gpart, int n_grp, int n5, double *gsos, hipStream_t stream);

}  // namespace filark
