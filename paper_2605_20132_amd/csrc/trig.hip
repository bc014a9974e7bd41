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
#include "trig_body.h"

namespace filark {
namespace {

using namespace dev;
using trigk::tparams_t;
__device__ __forceinline__ tparams_t tparams() { return dev::kparams<TrigParams>(); }

template <int L>
__global__ void __launch_bounds__(kMaxWaves * kWave) trig_kernel(TrigParams) {
  tparams_t p = tparams();
  const int g = group_of(p->per_xcd);
  if (g >= p->n_grp) return;  // whole workgroup, before any barrier
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x / kWave);
  const int cwl = p->cw_log2, CW = 1 << cwl, R = kWave >> cwl;
  const int64_t n_ch = p->n_ch;
  const int64_t c = (int64_t)g * CW + (lane & (CW - 1));
  const int row0 = (w * R + (lane >> cwl)) * L;
  float xv[L];
  {
    const __amdgpu_buffer_rsrc_t rx = rsrc(p->cf, p->range);
    const uint32_t rowb = (uint32_t)n_ch * 4u;
    const uint32_t vo = c < n_ch ? (uint32_t)(((int64_t)row0 * n_ch + c) * 4) : kOffInvalid;
#pragma unroll
    for (int j = 0; j < L; ++j) xv[j] = buf_ld<true>(rx, vo + (uint32_t)j * rowb);  // read once: non-temporal
  }
  trigk::trig_window<L>(p, g, xv);
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
