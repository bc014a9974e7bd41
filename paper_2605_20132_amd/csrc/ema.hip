// Stateful exponential-average operators (Table 1's running mean and running
// AGC rows, Section 3.4): per channel, with weight c = 1 / n_win and decay
// a = 1 - c,
//   running-mean removal (DEMEAN):  m = a m + c x;    y = x - m
//   running AGC:                    p = a p + c x^2;  y = x / sqrt(p) (0 where p = 0)
// from the carried average, which is left after the chunk's last sample.
//
// Parallel form as for the STA/LTA: each lane sums its block from zero in
// FP64 (s = a s + c e with e = x or x^2), a Hillis-Steele scan over the
// blocks of the window with the decays a^(L 2^k) gives every block its exact
// entry average (the carried one folded into block 0), and each lane reruns
// its rows from that entry, writing y.  The running mean's rerun is FP64
// (y = x - m cancels when the input has an offset); the AGC's gain is an
// FP32 reciprocal square root of the FP64 average.
#include "device.h"
#include "internal.h"

namespace filark {
namespace {

using namespace dev;
typedef const FILARK_CONST EmaParams *eparams_t;
__device__ __forceinline__ eparams_t eparams() { return dev::kparams<EmaParams>(); }

template <int L, bool DEMEAN>
__global__ void __launch_bounds__(kMaxWaves * kWave) ema_kernel(EmaParams) {
  __shared__ double xs[2][kMaxWaves * kWave];  // scan exchange (double-buffered)
  __shared__ double avg_x[kWave];              // carried averages of the group
  eparams_t p = eparams();
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
  const int64_t row0 = (int64_t)b * L;
  const uint32_t rowb = (uint32_t)n_ch * 4u;
  const uint32_t vo = cval ? (uint32_t)((row0 * n_ch + c) * 4) : kOffInvalid;

  // the carried average, read by the lanes of block 0 and staged in LDS; the
  // barrier below waits for the reads, so the write-back cannot overtake them
  if (b == 0) avg_x[cl] = cval ? p->avg[c] : 0.0;
  float xv[L];
  {
    const __amdgpu_buffer_rsrc_t rx = rsrc(p->x, p->range);
    const uint32_t rb = fresh(rowb);
#pragma unroll
    for (int j = 0; j < L; ++j) xv[j] = buf_ld<true>(rx, vo + (uint32_t)j * rb);  // read once: non-temporal
  }
  __syncthreads();
  const double avg_in = avg_x[cl];

  // the window's last row: wave and row within the block
  const int b_end = (n_t - 1) / L;
  const int w_end = b_end / R, r_end = b_end - w_end * R;
  const int jend = (n_t - 1) - b_end * L;
  const int jcap = uniform(w == w_end ? jend : -1);
  const bool end_lane = w == w_end && r == r_end && cval;

  // block sums from zero (rows past the chunk read 0 and add nothing)
  const double a = p->a, cw = p->c;
  double s = 0.0, s_cap = 0.0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const double v = (double)xv[j];
    s = fma(a, s, cw * (DEMEAN ? v : v * v));
    if (j == jcap) {
      asm volatile("");
      s_cap = s;
    }
  }

  // inclusive scan over the blocks; the carried average enters block 0
  cdouble *dp = as_const(p->dpow);
  if (b == 0) s = fma(dp[0], avg_in, s);
  int lev = 0;
  for (int d = 1; d < NB; d <<= 1, ++lev) {
    double *xl = xs[lev & 1];
    xl[my] = s;
    lds_barrier();
    if (b >= d) s = fma(dp[lev], xl[my - d * CW], s);
  }
  double *xf = xs[lev & 1];
  xf[my] = s;
  lds_barrier();
  const double s_in = b == 0 ? avg_in : xf[my - CW];
  if (end_lane) {
    cdouble *rp = as_const(p->dpow) + p->n_lev;  // a^m, m = 0 .. L
    p->avg[c] = fma(rp[jend + 1], s_in, s_cap);
  }

  // rerun from the exact entry, writing y
  const __amdgpu_buffer_rsrc_t ry = rsrc(p->y, p->range);
  const uint32_t rb = fresh(rowb);
  double m = s_in;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const double v = widen<1>(xv[j]);  // not the sum pass's conversion, held until now
    float out;
    if constexpr (DEMEAN) {
      m = fma(a, m, cw * v);
      out = (float)(v - m);
    } else {
      m = fma(a, m, cw * (v * v));
      const float mf = (float)m;  // averages below FP32's normal range give 0
      out = mf >= 1.17549435e-38f ? xv[j] * __builtin_amdgcn_rsqf(mf) : 0.0f;
    }
    buf_st(ry, vo + (uint32_t)j * rb, out);
    __builtin_amdgcn_sched_barrier(0);
  }
}

}  // namespace

hipError_t launch_ema(const EmaParams &p, int L, hipStream_t stream) {
  if (p.nw < 1 || p.nw > kMaxWaves || p.n_t < 1 || p.n_lev < 1 || p.n_lev > kMaxLevels) return hipErrorInvalidValue;
  const dim3 grid((unsigned)grid_for(p.per_xcd));
  const dim3 block((unsigned)(p.nw * kWave));
  if (L != 48) return hipErrorInvalidValue;
  if (p.mode == 0)
    hipLaunchKernelGGL((ema_kernel<48, true>), grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL((ema_kernel<48, false>), grid, block, 0, stream, p);
  return hipGetLastError();
}

}  // namespace filark
