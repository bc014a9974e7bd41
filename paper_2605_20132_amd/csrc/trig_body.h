// Trigger body shared by the standalone trigger kernel (trig.hip) and the
// fused monitor launch (monitor.hip): the two-threshold hysteresis over one
// window of cf rows already in registers.  The operation and its parallel
// form are described at the top of trig.hip.
#pragma once

#include "device.h"
#include "internal.h"

namespace filark {
namespace trigk {

using namespace dev;
typedef const FILARK_CONST TrigParams *tparams_t;

__device__ __forceinline__ int step(int s, float v, float on, float off, int r) {
  return (s != -1) ? (v < off ? -1 : s) : (v > on ? r : -1);
}

__device__ __forceinline__ int apply(int sa, int sb, int s) {
  return s == -1 ? sa : (sb == -2 ? s : sb);
}

// One window of channel group g: lane (r, cl) of wave w holds block
// b = w * (64 / cw) + r of channel g * cw + cl, rows b * L .. b * L + L - 1 of
// the window in xv (rows past the window's end are ignored).  Reads and
// advances the carried state, appends the events that close in the window.
// Every wave of the workgroup calls it (it holds workgroup barriers).
template <int L>
__device__ __forceinline__ void trig_window(tparams_t p, int g, const float (&xv)[L]) {
  __shared__ int xa[2][kMaxWaves * kWave], xb[2][kMaxWaves * kWave];  // scan exchange (double-buffered)
  __shared__ unsigned int wg_cnt;  // events of the workgroup
  __shared__ unsigned long long base_x;
  __shared__ int s_x[kWave];
  __shared__ int64_t ton_x[kWave], g0_x[kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x / kWave);
  const int cwl = p->cw_log2, CW = 1 << cwl, R = kWave >> cwl, NB = p->nw * R;
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
  // staged in LDS (the LDS writes wait for the reads' data, so the
  // write-back after the scan cannot overtake them).  The barriers here are
  // LDS-only: the window's own loads and stores (the cf rows of the
  // standalone kernel, the fused launch's y and cf stores) stay in flight.
  if (threadIdx.x == 0) wg_cnt = 0u;
  if (b == 0) {
    s_x[cl] = cval && p->open[c] ? -2 : -1;
    ton_x[cl] = cval ? p->t_on[c] : 0;
    g0_x[cl] = cval ? p->cnt[c] : 0;
  }

  lds_barrier();
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
  lds_barrier();  // every lane's slots taken
  if (threadIdx.x == 0) {
    // one reservation per workgroup on the caller's counter
    base_x = wg_cnt > 0u ? atomicAdd(p->count, (unsigned long long)wg_cnt) : 0ull;
  }
  lds_barrier();  // base_x (written from the atomic's returned value)
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

}  // namespace trigk
}  // namespace filark
