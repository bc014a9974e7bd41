// Realtime FIR with carried history (Table 1's FIR row, a stateful operator
// of Section 3.4): per channel
//   y[t] = sum_{k < M} h[k] x[t - k],
// where the M - 1 samples before the chunk come from the carried history,
// which is left holding the chunk's last M - 1 samples (ping-pong buffers, so
// the rows read and the rows written never alias).
//
// Direct form, one lane per channel: a wave holds 64 neighbouring channels
// (one 256-byte segment of every row) and R consecutive output rows in FP32
// accumulators.  Taps are applied 32 at a time from SGPRs (one scalar fetch
// per wave); for each tap chunk the lane loads the R + 31 input rows that the
// chunk touches and does R x 32 FMAs.  Every output takes its taps in
// ascending order, whatever the chunking, so a chunked run equals the one-shot
// run bit for bit.  The kernel is bound by FMA issue at long filters and by
// HBM at short ones; halo rows that neighbouring waves share are re-read from
// L1/L2, not HBM.  By default each XCD owns an eighth of the channel groups
// and sweeps its rows block by block across them (3 KB of every row at 6000
// channels), so the halo of a block was read into the same L2 one sweep
// earlier.  Up to 64 taps a second, unrolled kernel loads each input row once
// per wave.
#include "device.h"
#include "fir.h"

namespace filark {
namespace {

using namespace dev;
typedef const FILARK_CONST float cfloat;

// Output stores carry the non-temporal hint: y is never read back, and
// streaming it keeps L2 for the input rows that later row blocks re-read as
// their halo (measured: 9 % off a 16-tap pass over the record, 2-3 % at 64
// taps on 1500-row chunks).
constexpr int kNonTemporal = 2;
__device__ __forceinline__ void buf_st_stream(__amdgpu_buffer_rsrc_t r, uint32_t voff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, 0, kNonTemporal);
}
typedef const FILARK_CONST FirParams *firparams_t;
__device__ __forceinline__ firparams_t firparams() { return dev::kparams<FirParams>(); }

// The history buffer a launch reads and the one it writes, by the parity in
// ctl[0] (flipped by fir_flip_kernel after a call's last launch).
struct Hist {
  const float *in;
  float *out;
};
__device__ __forceinline__ Hist fir_hist(firparams_t p) {
  const uint32_t par = uniform((int)(*p->ctl & 1u));
  return Hist{par ? p->hist1 : p->hist0, par ? p->hist0 : p->hist1};
}

// Channel group and row block of this workgroup; false past the grid's work.
// Order 0: XCD x takes a contiguous run of (group, block) pairs, blocks
// fastest.  Order 1: the same with groups fastest, so an XCD streams whole
// rows.  Order 2: XCD x takes the channel slab [x s, (x + 1) s) of s = per_xcd
// groups and sweeps its rows block by block across the slab, so the halo rows
// of a block were read into the same L2 by the block before.
__device__ __forceinline__ bool fir_tile_of(firparams_t p, int &cg, int &tb) {
  const int n_tb = p->n_tb, n_cg = p->n_cg, order = p->chan_minor;
  if (order == 2) {
    const int x = (int)blockIdx.x & 7, i = (int)blockIdx.x >> 3, s = p->per_xcd;
    const int c0 = x * s;
    const int cs = n_cg - c0 < s ? n_cg - c0 : s;  // groups in this XCD's slab
    if (cs <= 0 || i >= cs * n_tb) return false;
    tb = uniform(i / cs);
    cg = uniform(c0 + (i - tb * cs));
    return true;
  }
  const int g = group_of(p->per_xcd);
  if (g >= n_cg * n_tb) return false;
  if (order == 1) {
    tb = uniform(g / n_cg);
    cg = g - tb * n_cg;
  } else {
    cg = uniform(g / n_tb);
    tb = g - cg * n_tb;
  }
  return true;
}

template <int R>
__device__ __forceinline__ void fir_body(firparams_t p, const Hist &hh) {
  constexpr int KC = kFirChunk;
  constexpr int NX = R + KC - 1;  // input rows one tap chunk touches
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x / kWave);
  int cg, tb;
  if (!fir_tile_of(p, cg, tb)) return;
  const int t0 = uniform((tb * p->nw + w) * R);  // first output row of the wave
  if (t0 >= p->n_rows) return;                   // no barriers below: waves leave freely
  const int64_t c = (int64_t)cg * kWave + lane;
  const bool cval = c < p->n_ch;
  const uint32_t rowb = (uint32_t)p->n_ch * 4u;
  const uint32_t cb = (uint32_t)c * 4u;

  float acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0f;

  const int n_chunks = p->n_chunks;
  for (int q = 0; q < n_chunks; ++q) {
    const int k0 = q * KC;
    // input rows of this chunk: xw[i] is input row t0 - k0 - (KC - 1) + i,
    // u0 the same row counted from the input base
    const int u0 = uniform(t0 + p->xoff - k0 - (KC - 1));
    float xw[NX];
    const uint32_t rb = fresh(rowb);  // row offsets formed here, not held across chunks
    if (u0 >= 0) {
      const __amdgpu_buffer_rsrc_t rx = rsrc(p->x, p->range);
      const uint32_t vo = cval ? (uint32_t)u0 * rb + cb : kOffInvalid;
      // newest rows first: they are the ones the first taps need
#pragma unroll
      for (int i = NX - 1; i >= 0; --i) xw[i] = buf_ld(rx, vo + (uint32_t)i * rb);
    } else {
      // the chunk reaches back before the input: rows -(M - 1) .. -1 come from
      // the carried history, rows further back (zero taps only) read 0
      const __amdgpu_buffer_rsrc_t rx = rsrc(p->x, p->range);
      const __amdgpu_buffer_rsrc_t rh = rsrc(hh.in, p->hrange);
      const int hm = p->hm;
#pragma unroll
      for (int i = NX - 1; i >= 0; --i) {
        const int u = u0 + i;
        const uint32_t ox = cval && u >= 0 ? (uint32_t)u * rb + cb : kOffInvalid;
        const uint32_t oh = cval && u < 0 && u >= -hm ? (uint32_t)(u + hm) * rb + cb : kOffInvalid;
        const float a = buf_ld(rx, ox), b = buf_ld(rh, oh);
        xw[i] = u >= 0 ? a : b;
      }
    }
    if (q == 0) {
      // the wave's own rows (xw[KC - 1 + r]) that end the chunk become history
      const int hs = p->hs, n_rows = p->n_rows;
      if (t0 + R > hs) {
        const __amdgpu_buffer_rsrc_t ro = rsrc(hh.out, p->hrange);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int t = t0 + r;
          const uint32_t o = cval && t >= hs && t < n_rows ? (uint32_t)(t - hs) * rb + cb : kOffInvalid;
          buf_st(ro, o, xw[KC - 1 + r]);
        }
      }
      // a chunk shorter than M - 1 rows keeps the newest old history rows
      const int hcopy = p->hcopy;
      if (t0 == 0 && hcopy > 0) {
        const __amdgpu_buffer_rsrc_t rh = rsrc(hh.in, p->hrange);
        const __amdgpu_buffer_rsrc_t ro = rsrc(hh.out, p->hrange);
        const int src = p->hsrc;
        for (int j = 0; j < hcopy; ++j) {
          const float v = buf_ld(rh, cval ? (uint32_t)(src + j) * rowb + cb : kOffInvalid);
          buf_st(ro, cval ? (uint32_t)j * rowb + cb : kOffInvalid, v);
        }
      }
    }
    cfloat *hp = (cfloat *)p->h + k0;
    float hk[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) hk[k] = hp[k];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = __builtin_fmaf(hk[k], xw[KC - 1 + r - k], acc[r]);
    }
  }

  const __amdgpu_buffer_rsrc_t ry = rsrc(p->y, p->out_range);
  const uint32_t rb = fresh(rowb);
  const uint32_t vy = cval ? (uint32_t)t0 * rb + cb : kOffInvalid;
#pragma unroll
  for (int r = 0; r < R; ++r) buf_st_stream(ry, vy + (uint32_t)r * rb, acc[r]);
}

template <int R>
__global__ void __launch_bounds__(kMaxWaves * kWave) fir_kernel(FirParams) {
  firparams_t p = firparams();
  const Hist hh = fir_hist(p);
  fir_body<R>(p, hh);
}

// Input rows of the unrolled kernel by age: xr[j] is row t0 + R - 1 - j, so
// output row t0 + r takes tap kk from xr[R - 1 - r + kk].  Slab s holds
// xr[32 s .. 32 s + 31]; the rows before the input come from the history.
template <int R, int N>
__device__ __forceinline__ void fir_load_slab(firparams_t p, const float *hin, int t0, bool cval, uint32_t cb, int s,
                                              float (&xr)[N]) {
  constexpr int KC = kFirChunk;
  const uint32_t rb = fresh((uint32_t)p->n_ch * 4u);
  const int umax = uniform(t0 + p->xoff + R - 1 - KC * s);  // base row of xr[32 s]
  const int n = N - KC * s < KC ? N - KC * s : KC;
  const __amdgpu_buffer_rsrc_t rx = rsrc(p->x, p->range);
  if (umax - (KC - 1) >= 0) {
    // offsets step down by a row: an invalid lane starts 31 rows above 2^31
    const uint32_t vo = cval ? (uint32_t)umax * rb + cb : kOffInvalid + (uint32_t)(KC - 1) * rb;
#pragma unroll
    for (int i = 0; i < KC; ++i)
      if (i < n) xr[KC * s + i] = buf_ld(rx, vo - (uint32_t)i * rb);
  } else {
    const __amdgpu_buffer_rsrc_t rh = rsrc(hin, p->hrange);
    const int hm = p->hm;
#pragma unroll
    for (int i = 0; i < KC; ++i) {
      if (i < n) {
        const int u = umax - i;
        const uint32_t ox = cval && u >= 0 ? (uint32_t)u * rb + cb : kOffInvalid;
        const uint32_t oh = cval && u < 0 && u >= -hm ? (uint32_t)(u + hm) * rb + cb : kOffInvalid;
        const float a = buf_ld(rx, ox), b = buf_ld(rh, oh);
        xr[KC * s + i] = u >= 0 ? a : b;
      }
    }
  }
}

// Taps [KC/2 * h, KC/2 * (h + 1)) of chunk Q, in ascending order.
template <int R, int N, int Q, int H>
__device__ __forceinline__ void fir_half(const float (&hk)[kFirChunk], const float (&xr)[N], float (&acc)[R]) {
  constexpr int KC = kFirChunk;
#pragma unroll
  for (int k = H * KC / 2; k < (H + 1) * KC / 2; ++k) {
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = __builtin_fmaf(hk[k], xr[R - 1 - r + KC * Q + k], acc[r]);
  }
}

// Slabs chunk 0 needs beyond slab 0 (chunk Q reaches slab Q + this).
template <int R>
constexpr int fir_reach() {
  return (R + kFirChunk - 2) / kFirChunk;
}

// Chunk Q of NCH: first half of its taps, then the next chunk's last slab
// and taps are fetched, then the second half; the next chunk follows.
template <int NCH, int Q, int R, int N>
__device__ __forceinline__ void fir_chunk(firparams_t p, const float *hin, int t0, bool cval, uint32_t cb,
                                          float (&xr)[N], float (&hk)[kFirChunk], float (&acc)[R]) {
  constexpr int KC = kFirChunk, S = Q + 1 + fir_reach<R>();
  fir_half<R, N, Q, 0>(hk, xr, acc);
  float hn[KC];
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (Q + 1 < NCH && KC * S < N) fir_load_slab<R>(p, hin, t0, cval, cb, S, xr);
  if constexpr (Q + 1 < NCH) {
    cfloat *hp = (cfloat *)p->h + KC * (Q + 1);
#pragma unroll
    for (int e = 0; e < KC; ++e) hn[e] = hp[e];
  }
  __builtin_amdgcn_sched_barrier(0);
  fir_half<R, N, Q, 1>(hk, xr, acc);
  if constexpr (Q + 1 < NCH) {
#pragma unroll
    for (int e = 0; e < KC; ++e) hk[e] = hn[e];
    fir_chunk<NCH, Q + 1>(p, hin, t0, cval, cb, xr, hk, acc);
  }
}

// The same computation for NCH <= 2 tap chunks and R = 32 or 48 output rows,
// unrolled: consecutive chunks share 32-row slabs (so each input row is
// loaded once per wave), the next slab and the next chunk's taps are fetched
// halfway through a chunk, into the registers of rows that chunk no longer
// needs, and the FMAs keep the ascending tap order (same bits as fir_kernel).
template <int NCH, int R>
__device__ __forceinline__ void fir_body_u(firparams_t p, const Hist &hh) {
  constexpr int KC = kFirChunk, N = R + KC * NCH - 1;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x / kWave);
  int cg, tb;
  if (!fir_tile_of(p, cg, tb)) return;
  const int t0 = uniform((tb * p->nw + w) * R);
  if (t0 >= p->n_rows) return;
  const int64_t c = (int64_t)cg * kWave + lane;
  const bool cval = c < p->n_ch;
  const uint32_t cb = (uint32_t)c * 4u;

  float xr[N];
#pragma unroll
  for (int s = 0; s <= fir_reach<R>(); ++s)
    if (KC * s < N) fir_load_slab<R>(p, hh.in, t0, cval, cb, s, xr);
  {
    const int hs = p->hs, n_rows = p->n_rows;
    if (t0 + R > hs) {
      const uint32_t rb = fresh((uint32_t)p->n_ch * 4u);
      const __amdgpu_buffer_rsrc_t ro = rsrc(hh.out, p->hrange);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int t = t0 + r;
        const uint32_t o = cval && t >= hs && t < n_rows ? (uint32_t)(t - hs) * rb + cb : kOffInvalid;
        buf_st(ro, o, xr[R - 1 - r]);
      }
    }
    const int hcopy = p->hcopy;
    if (t0 == 0 && hcopy > 0) {
      const uint32_t rb = fresh((uint32_t)p->n_ch * 4u);
      const __amdgpu_buffer_rsrc_t rh = rsrc(hh.in, p->hrange);
      const __amdgpu_buffer_rsrc_t ro = rsrc(hh.out, p->hrange);
      const int src = p->hsrc;
      for (int j = 0; j < hcopy; ++j) {
        const float v = buf_ld(rh, cval ? (uint32_t)(src + j) * rb + cb : kOffInvalid);
        buf_st(ro, cval ? (uint32_t)j * rb + cb : kOffInvalid, v);
      }
    }
  }

  float acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0f;
  float hk[KC];
  {
    cfloat *hp = (cfloat *)p->h;
#pragma unroll
    for (int k = 0; k < KC; ++k) hk[k] = hp[k];
  }
  fir_chunk<NCH, 0>(p, hh.in, t0, cval, cb, xr, hk, acc);

  const uint32_t rb = fresh((uint32_t)p->n_ch * 4u);
  const __amdgpu_buffer_rsrc_t ry = rsrc(p->y, p->out_range);
  const uint32_t vy = cval ? (uint32_t)t0 * rb + cb : kOffInvalid;
#pragma unroll
  for (int r = 0; r < R; ++r) buf_st_stream(ry, vy + (uint32_t)r * rb, acc[r]);
}

// Waves per SIMD the unrolled kernel is held to (its register budget):
// 4 (128 VGPRs) at 32 rows, 3 (168) at 48.
template <int R>
constexpr int fir_waves_per_eu() {
  return R == 32 ? 4 : 3;
}

template <int NCH, int R>
__global__ void __launch_bounds__(kMaxWaves * kWave) __attribute__((amdgpu_waves_per_eu(fir_waves_per_eu<R>())))
fir_kernel_u(FirParams) {
  firparams_t p = firparams();
  const Hist hh = fir_hist(p);
  fir_body_u<NCH, R>(p, hh);
}

// After a call's last launch: the history it wrote becomes the current one.
// One lane; a vector load and store.
__global__ void __launch_bounds__(kWave) fir_flip_kernel(uint32_t *ctl) {
  if (threadIdx.x == 0) ctl[0] ^= 1u;
}

// The kernel a launch with R rows per wave and n_chunks tap chunks runs.
const void *fir_kernel_for(int R, int n_chunks) {
  if (R == 32 && n_chunks == 1) return (const void *)fir_kernel_u<1, 32>;
  if (R == 32 && n_chunks == 2) return (const void *)fir_kernel_u<2, 32>;
  if (R == 48 && n_chunks == 1) return (const void *)fir_kernel_u<1, 48>;
  if (R == 48 && n_chunks == 2) return (const void *)fir_kernel_u<2, 48>;
  if (R == 16) return (const void *)fir_kernel<16>;
  if (R == 32) return (const void *)fir_kernel<32>;
  if (R == 48) return (const void *)fir_kernel<48>;
  return nullptr;
}

}  // namespace

hipError_t launch_fir(const FirParams &p, int R, hipStream_t stream) {
  if (p.nw < 1 || p.nw > kMaxWaves || p.n_rows < 1 || p.n_chunks < 1 || p.n_cg < 1 || p.n_tb < 1 ||
      p.chan_minor < 0 || p.chan_minor > 2)
    return hipErrorInvalidValue;
  // order 2: per_xcd is the slab width in groups, each XCD runs slab x n_tb workgroups
  const int64_t per = p.chan_minor == 2 ? (int64_t)p.per_xcd * p.n_tb : p.per_xcd;
  if (p.chan_minor == 2 ? 8LL * p.per_xcd < p.n_cg : (int64_t)p.n_cg * p.n_tb > 8LL * p.per_xcd)
    return hipErrorInvalidValue;
  if (per > ((int64_t)1 << 28)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(8 * per));
  const dim3 block((unsigned)(p.nw * kWave));
  // unrolled up to 64 taps; beyond, its live rows would cost occupancy
  const void *k = fir_kernel_for(R, p.n_chunks);
  if (!k) return hipErrorInvalidValue;
  FirParams q = p;
  void *args[] = {&q};
  const hipError_t e = hipLaunchKernel(k, grid, block, args, 0, stream);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_fir_flip(uint32_t *ctl, hipStream_t stream) {
  hipLaunchKernelGGL(fir_flip_kernel, dim3(1), dim3(kWave), 0, stream, ctl);
  return hipGetLastError();
}

}  // namespace filark
