// Two-threshold trigger on a characteristic function: the monitor contract
// of Section 3.4 (a window of data goes in, a list of time-channel events
// comes out), as the classic hysteresis of an energy detector.  Per channel,
// while closed, the first sample whose cf exceeds `on` opens an event; while
// open, the first later sample whose cf is below `off` closes it and the
// event [t_on, t_off) is emitted.  An event open at the end of a call stays
// in the carried state (open flag, t_on), so any chunking emits the events of
// the one-shot run.
//
// Parallel form: the state of a channel at a row is a code s
//   s = -1: closed;   s = -2: open since before the window;   s = r >= 0: open since window row r
// and one row maps it by the same rule whatever it is:
//   s <- (s != -1) ? (cf < off ? -1 : s) : (cf > on ? r : -1).
// A block of rows is therefore summarised by what it does to the two kinds of
// entry, A = run(-1) and B = run(-2) (B = -2: still open from the entry), and
// the map of a block applied after a prefix P is
//   apply(S, s) = s == -1 ? S.A : (S.B == -2 ? s : S.B),
// which composes associatively.  The blocks of a window are combined by a
// Hillis-Steele scan in LDS.  The number of events closing in a block depends
// only on whether it is entered open or closed, so the summary pass counts
// both; each lane takes its slots from a workgroup counter in LDS, the
// workgroup reserves the total with one atomic add on the caller's counter,
// and a rerun of the block from its exact entry code writes the events.
// Rows past the end of the chunk change nothing.
#include "device.h"
#include "internal.h"

namespace filark {
namespace {

using namespace dev;
typedef const FILARK_CONST TrigParams *tparams_t;
__device__ __forceinline__ tparams_t tparams() { return dev::kparams<TrigParams>(); }

__device__ __forceinline__ int step(int s, float v, float on, float off, int r) {
  return (s != -1) ? (v < off ? -1 : s) : (v > on ? r : -1);
}

__device__ __forceinline__ int apply(int sa, int sb, int s) {
  return s == -1 ? sa : (sb == -2 ? s : sb);
}

template <int L>
__global__ void __launch_bounds__(kMaxWaves * kWave) trig_kernel(TrigParams) {
  __shared__ int xa[2][kMaxWaves * kWave], xb[2][kMaxWaves * kWave];  // scan exchange (double-buffered)
  __shared__ unsigned int wg_cnt;  // events of the workgroup
  __shared__ unsigned long long base_x;
  tparams_t p = tparams();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x / kWave);
  const int cwl = p->cw_log2, CW = 1 << cwl, R = kWave >> cwl, NB = p->nw * R;
  const int g = group_of(p->per_xcd);
  if (g >= p->n_grp) return;  // whole workgroup, before any barrier
  const int r = lane >> cwl, cl = lane & (CW - 1);
  const int b = w * R + r;
  const int my = w * kWave + lane;
  const int64_t n_ch = p->n_ch;
  const int64_t c = (int64_t)g * CW + cl;
  const bool cval = c < n_ch;
  const int n_t = p->n_t;
  const int row0 = b * L;
  const int nv = row0 >= n_t ? 0 : (n_t - row0 >= L ? L : n_t - row0);  // valid rows of the block
  const float on = p->on, off = p->off;

  // the carried state of the channel: read by the lanes of block 0 and
  // staged in LDS; the barrier below also waits for these reads, so the
  // write-back after the scan cannot overtake them
  __shared__ int s_x[kWave];
  __shared__ int64_t ton_x[kWave], g0_x[kWave];
  if (threadIdx.x == 0) wg_cnt = 0u;
  if (b == 0) {
    s_x[cl] = cval && p->open[c] ? -2 : -1;
    ton_x[cl] = cval ? p->t_on[c] : 0;
    g0_x[cl] = cval ? p->cnt[c] : 0;
  }

  float xv[L];
  {
    const __amdgpu_buffer_rsrc_t rx = rsrc(p->cf, p->range);
    const uint32_t rowb = (uint32_t)n_ch * 4u;
    const uint32_t vo = cval ? (uint32_t)(((int64_t)row0 * n_ch + c) * 4) : kOffInvalid;
#pragma unroll
    for (int j = 0; j < L; ++j) xv[j] = buf_ld<true>(rx, vo + (uint32_t)j * rowb);  // read once: non-temporal
  }
  __syncthreads();  // workgroup barrier with every wave's memory reads complete
  const int s_in = s_x[cl];
  const int64_t ton_in = ton_x[cl], g0 = g0_x[cl];

  // block summary: the code after the block from a closed and an open
  // entry, and the events that close in it in either case
  int sa = -1, sb = -2, ca = 0, cb = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    if (j < nv) {
      ca += (sa != -1 && xv[j] < off) ? 1 : 0;
      cb += (sb != -1 && xv[j] < off) ? 1 : 0;
      sa = step(sa, xv[j], on, off, row0 + j);
      sb = step(sb, xv[j], on, off, row0 + j);
    }
  }

  // inclusive scan over the blocks of the window (earlier blocks first)
  int lev = 0;
  for (int d = 1; d < NB; d <<= 1, ++lev) {
    const int k = lev & 1;
    xa[k][my] = sa;
    xb[k][my] = sb;
    lds_barrier();
    if (b >= d) {
      const int pa = xa[k][my - d * CW], pb = xb[k][my - d * CW];
      const int na = apply(sa, sb, pa), nb = apply(sa, sb, pb);
      sa = na;
      sb = nb;
    }
  }
  const int kf = lev & 1;
  xa[kf][my] = sa;
  xb[kf][my] = sb;
  lds_barrier();
  // entry code of the block: the blocks before it applied to the carried state
  int s = s_in;
  if (b > 0) s = apply(xa[kf][my - CW], xb[kf][my - CW], s_in);
  if (b == NB - 1 && cval) {  // the state after the window
    const int f = apply(sa, sb, s_in);
    p->open[c] = f != -1 ? 1 : 0;
    if (f >= 0) p->t_on[c] = g0 + f;
    p->cnt[c] = g0 + n_t;
  }

  // events closing in this block, and their slots within the workgroup
  const int n_ev = cval ? (s == -1 ? ca : cb) : 0;
  const unsigned int mine = n_ev > 0 ? atomicAdd(&wg_cnt, (unsigned int)n_ev) : 0u;
  __syncthreads();  // every lane's slots taken
  if (threadIdx.x == 0) {
    // one reservation per workgroup on the caller's counter
    base_x = wg_cnt > 0u ? atomicAdd(p->count, (unsigned long long)wg_cnt) : 0ull;
  }
  __syncthreads();  // base_x
  if (n_ev == 0) return;
  const int64_t cap = p->cap;
  int64_t pos = (int64_t)base_x + (int64_t)mine;
  int64_t *ev = p->ev;
  {
    int q = s;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      if (j < nv) {
        if (q != -1 && xv[j] < off) {
          if (pos < cap) {
            ev[3 * pos + 0] = c;
            ev[3 * pos + 1] = q == -2 ? ton_in : g0 + q;
            ev[3 * pos + 2] = g0 + row0 + j;
          }
          ++pos;
        }
        q = step(q, xv[j], on, off, row0 + j);
      }
    }
  }
}

}  // namespace

hipError_t launch_trig(const TrigParams &p, int L, hipStream_t stream) {
  if (p.nw < 1 || p.nw > kMaxWaves || p.n_t < 1 || p.cap < 0 || !p.count) return hipErrorInvalidValue;
  const dim3 grid((unsigned)grid_for(p.per_xcd));
  const dim3 block((unsigned)(p.nw * kWave));
  if (L == 48) {
    hipLaunchKernelGGL(trig_kernel<48>, grid, block, 0, stream, p);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace filark
