// FFT filtering of the realtime FIR (the overlap-add / overlap-save FFT
// filtering of Table 1's FIR row; Section 6.2 reports its GPU speed-up):
// y[t] = sum_k h[k] x[t - k] computed block by block in the frequency domain,
// the samples before the call taken from the carried history (the last M - 1
// input rows, the state the direct kernel carries too).
//
// Block.  A workgroup takes 8 (or 4) consecutive channels and one block of
// B = N - (M - 1) output rows, N = 2048: the window of N input rows that ends
// with the block (M - 1 rows before it, from the chunk or the history),
// whose circular convolution with the zero-padded taps equals the linear one
// at the window's last B positions (overlap-save; overlap-add gives the same
// sums with the tail carried instead of the history).  Per channel:
//   z[n] = x[2n] + i x[2n + 1]          two real samples per complex value
//   Z = FFT_1024(z)                      radix-4 stages (two at a time in
//                                        registers), in place in LDS (DIT:
//                                        the input is placed digit-reversed)
//   X[k] = E + W_2048^k O, E = (Z[k] + Z*[1024 - k]) / 2, O = (Z[k] - Z*[1024 - k]) / 2i
//   Y[k] = X[k] H[k]                     H: the taps' 2048-point spectrum
//   Z'[k] = E' + i O', E' = (Y[k] + Y*[1024 - k]) / 2, O' = W_2048^-k (Y[k] - Y*[1024 - k]) / 2
//   z' = IFFT_1024(Z')                   radix-4 DIF: digit-reversed output
//   y[2n] = Re z'[n], y[2n + 1] = Im z'[n]
// The factors 1/2 and the 1/1024 of the inverse are folded into H on the
// host.  FP32 throughout (twiddles and H rounded from FP64); the error bound
// is that of FP32 transforms, not the direct kernel's exact summation order.
// The workgroups of the call's last block also write the new history (the
// last M - 1 input rows) into the other history buffer as they load it, and
// the last workgroup to finish makes that buffer the current one.
#include "device.h"
#include "fir.h"

namespace filark {
namespace {

constexpr int kN2 = kFftN / 2;           // complex points per channel
constexpr int kPitch = kN2;              // LDS float2 per channel (8 KiB)

// LDS place of point i of a channel: the low five bits xor-ed with the next
// five (a permutation within each run of 32), so the strided accesses of the
// early radix-4 stages spread over the banks without padding.
__device__ __forceinline__ int pad(int i) { return i ^ ((i >> 5) & 31); }

// Base-4 digit reversal of a 10-bit index (5 digits).
__device__ __forceinline__ int rev4(int n) {
  int r = 0;
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    r = (r << 2) | (n & 3);
    n >>= 2;
  }
  return r;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conj2(float2 a) { return make_float2(a.x, -a.y); }
// multiplication by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_i(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// The twiddle W_1024^e (forward) or its conjugate (inverse).
template <bool INV>
__device__ __forceinline__ float2 tw(const float2 *__restrict__ w1024, int e) {
  const float2 v = w1024[e & (kN2 - 1)];
  return INV ? conj2(v) : v;
}

// 4-point DFT in place: b_m = sum_l a_l w^(l m), w = -i (forward) or +i.
template <bool INV>
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
  const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const float2 s13 = cadd(a1, a3), d13 = mul_i<INV>(csub(a1, a3));
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, d13);
  a3 = csub(d02, d13);
}

// Two consecutive radix-4 stages, s and s + 1 (spans S = 4^s and 4 S), as
// one radix-16 step in registers: a thread takes the 16 points
// g 16 S + j + m S + n 4 S (j < S; m, n < 4), which stage s combines over m
// and stage s + 1 over n.  Forward (DIT): twiddle W_4S^(j m), 4-point
// transform over m, then twiddle W_16S^((j + m S) n), transform over n.
// Inverse (DIF): the same steps in reverse order, transforms first and
// conjugate twiddles.  64 groups per transform.
template <bool INV, int s, int kTpc>
__device__ __forceinline__ void radix16(float2 *buf, const float2 *__restrict__ w1024, int tc) {
  constexpr int S = 1 << (2 * s);
  constexpr int step0 = kN2 / (4 * S), step1 = kN2 / (16 * S);
#pragma unroll
  for (int u = 0; u < 64 / kTpc; ++u) {
    const int t = tc + u * kTpc;  // group 0 .. 63
    const int j = t & (S - 1), g = t >> (2 * s);
    const int base = g * 16 * S + j;
    float2 P[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) P[m][n] = buf[pad(base + m * S + n * 4 * S)];
    if (!INV) {
#pragma unroll
      for (int n = 0; n < 4; ++n) {
#pragma unroll
        for (int m = 1; m < 4; ++m) P[m][n] = cmul(P[m][n], tw<false>(w1024, j * m * step0));
        dft4<false>(P[0][n], P[1][n], P[2][n], P[3][n]);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int jp = j + m * S;
#pragma unroll
        for (int n = 1; n < 4; ++n) P[m][n] = cmul(P[m][n], tw<false>(w1024, jp * n * step1));
        dft4<false>(P[m][0], P[m][1], P[m][2], P[m][3]);
      }
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int jp = j + m * S;
        dft4<true>(P[m][0], P[m][1], P[m][2], P[m][3]);
#pragma unroll
        for (int n = 1; n < 4; ++n) P[m][n] = cmul(P[m][n], tw<true>(w1024, jp * n * step1));
      }
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        dft4<true>(P[0][n], P[1][n], P[2][n], P[3][n]);
#pragma unroll
        for (int m = 1; m < 4; ++m) P[m][n] = cmul(P[m][n], tw<true>(w1024, j * m * step0));
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) buf[pad(base + m * S + n * 4 * S)] = P[m][n];
  }
}

// One radix-4 stage of span S = 4^s: 256 butterflies over points
// g 4 S + j + m S, twiddle W_4S^(j m) before (DIT) or after (DIF) the
// 4-point transform.
template <bool INV, int s, int kTpc>
__device__ __forceinline__ void radix4(float2 *buf, const float2 *__restrict__ w1024, int tc) {
  constexpr int S = 1 << (2 * s);
  constexpr int step = kN2 / (4 * S);
#pragma unroll
  for (int u = 0; u < 256 / kTpc; ++u) {
    const int b = tc + u * kTpc;  // butterfly 0 .. 255
    const int j = b & (S - 1), g = b >> (2 * s);
    const int base = g * 4 * S + j;
    float2 a0 = buf[pad(base)], a1 = buf[pad(base + S)], a2 = buf[pad(base + 2 * S)], a3 = buf[pad(base + 3 * S)];
    if (!INV) {
      a1 = cmul(a1, tw<false>(w1024, j * step));
      a2 = cmul(a2, tw<false>(w1024, 2 * j * step));
      a3 = cmul(a3, tw<false>(w1024, 3 * j * step));
      dft4<false>(a0, a1, a2, a3);
    } else {
      dft4<true>(a0, a1, a2, a3);
      a1 = cmul(a1, tw<true>(w1024, j * step));
      a2 = cmul(a2, tw<true>(w1024, 2 * j * step));
      a3 = cmul(a3, tw<true>(w1024, 3 * j * step));
    }
    buf[pad(base)] = a0;
    buf[pad(base + S)] = a1;
    buf[pad(base + 2 * S)] = a2;
    buf[pad(base + 3 * S)] = a3;
  }
}

// In-place radix-4 transform of 1024 points of one channel held by kTpc
// threads: DIT from digit-reversed input to natural output (forward: stages
// 0 + 1, 2 + 3, 4), or DIF from natural input to digit-reversed output
// (inverse: stages 4 + 3, 2 + 1, 0).  Three passes through LDS, a workgroup
// barrier after each.
template <bool INV, int kTpc>
__device__ __forceinline__ void fft1024(float2 *buf, const float2 *__restrict__ w1024, int tc) {
  if constexpr (!INV) {
    radix16<false, 0, kTpc>(buf, w1024, tc);
    __syncthreads();
    radix16<false, 2, kTpc>(buf, w1024, tc);
    __syncthreads();
    radix4<false, 4, kTpc>(buf, w1024, tc);
    __syncthreads();
  } else {
    radix16<true, 3, kTpc>(buf, w1024, tc);
    __syncthreads();
    radix16<true, 1, kTpc>(buf, w1024, tc);
    __syncthreads();
    radix4<true, 0, kTpc>(buf, w1024, tc);
    __syncthreads();
  }
}

// Row t of the chunk for channel c: the chunk (0 <= t < n_t), the history
// (-(M - 1) <= t < 0, oldest row first) or 0 (past the chunk, or an invalid
// channel).  Branch-free, so that a thread's loads are all issued before the
// first is waited for: where there is no sample, a valid address (the
// twiddle table) is read and the value replaced by 0.
__device__ __forceinline__ float fft_in(const FftParams &p, const float *hist, int64_t t, int64_t c, bool cval) {
  const bool in_x = cval && t >= 0 && t < p.n_t;
  const bool in_h = cval && t < 0 && t + p.hm >= 0;
  const float *src = in_x ? p.x + t * p.n_ch + c
                          : (in_h ? hist + (t + p.hm) * p.n_ch + c : reinterpret_cast<const float *>(p.tw));
  const float v = __builtin_nontemporal_load(src);
  return (in_x || in_h) ? v : 0.0f;
}

// kCh channels per workgroup of kThreads threads (kThreads / kCh per
// channel).  Channel groups are dealt to the XCDs in contiguous slabs, so the
// groups that share a row's cache lines meet in one L2.  The LDS (8 KiB per
// channel) allows two workgroups of 8 channels per CU; the register bound
// keeps that many waves resident.
template <int kCh, int kThreads>
__global__ void __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(kThreads * 2 / (4 * 64)))) fir_fft_kernel(FftParams p) {
  constexpr int kTpc = kThreads / kCh;
  __shared__ float2 lds[kCh * kPitch];
  __shared__ float2 twl[kN2];  // W_1024^j, read by every butterfly
  const int tid = (int)threadIdx.x;
  const int cg = dev::group_of(p.per_xcd), blk = (int)blockIdx.y;
  if ((int64_t)cg * kCh >= p.n_ch) return;  // whole workgroup, before any barrier
  const int64_t c0 = (int64_t)cg * kCh;
  const int64_t t_out = (int64_t)blk * p.B;      // first output row of the block
  const int64_t t_win = t_out - p.hm;            // chunk row of window position 0
  const bool odd = (p.ctl[0] & 1u) != 0;
  const float *hist = odd ? p.hist1 : p.hist0;
  float *hist_new = odd ? p.hist0 : p.hist1;
  const float2 *w2048 = p.tw + kN2;
  for (int i = tid; i < kN2; i += kThreads) twl[i] = p.tw[i];
  // the new history (the last M - 1 rows before the end of the call, from
  // the chunk or the old history) lies in the last block's window: its
  // workgroups write it from the values they load
  const bool last_blk = p.hm > 0 && (int64_t)(blk + 1) * p.B >= p.n_t;
  const int64_t h0 = p.n_t - p.hm;  // chunk row of the new history's first row

  // load: thread (row rr, channel cc); a wave covers 8 rows of 8 channels;
  // window sample r goes to complex n = r / 2 (real part for even r) at the
  // digit-reversed place
  {
    constexpr int kStep = kThreads / kCh, kIt = kN2 / kStep;
    const int cc = tid & (kCh - 1), rr0 = tid / kCh;
    const int64_t c = c0 + cc;
    const bool cval = c < p.n_ch;
    float2 *buf = lds + cc * kPitch;
    constexpr int kBatch = 8;  // row pairs in flight per thread
#pragma unroll 1
    for (int i0 = 0; i0 < kIt; i0 += kBatch) {
      float2 v[kBatch];
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        const int64_t t = t_win + 2 * (rr0 + (i0 + i) * kStep);
        v[i] = make_float2(fft_in(p, hist, t, c, cval), fft_in(p, hist, t + 1, c, cval));
      }
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        buf[pad(rev4(rr0 + (i0 + i) * kStep))] = v[i];
        if (last_blk && cval) {
          const int64_t t = t_win + 2 * (rr0 + (i0 + i) * kStep);
          if (t >= h0 && t < p.n_t) hist_new[(t - h0) * p.n_ch + c] = v[i].x;
          if (t + 1 >= h0 && t + 1 < p.n_t) hist_new[(t + 1 - h0) * p.n_ch + c] = v[i].y;
        }
      }
    }
  }
  __syncthreads();
  const int ch = tid / kTpc, tc = tid & (kTpc - 1);
  float2 *buf = lds + ch * kPitch;
  fft1024<false, kTpc>(buf, twl, tc);

  // spectrum: the real transform of the window times H, and the packing for
  // the inverse, pair (k, 1024 - k) at a time (k = 0 with 512 alone and 512
  // with itself: done by the thread of k = 0)
  for (int k = tc; k <= kN2 / 2; k += kTpc) {
    const float2 h_lo = p.H[k], h_hi = p.H[kN2 - k];
    if (k == 0) {
      const float2 z0 = buf[pad(0)];
      const float x0 = 2.0f * (z0.x + z0.y), xn = 2.0f * (z0.x - z0.y);  // 2 X[0], 2 X[1024] (real)
      const float y0 = x0 * h_lo.x, yn = xn * p.H[kN2].x;     // H[0], H[1024] are real
      buf[pad(0)] = make_float2(y0 + yn, y0 - yn);
      // k = 512 pairs with itself: 2 X = 2 conj(Z) (W_2048^512 = -i), and the
      // packing gives 2 conj(2 X H)
      const float2 zm = buf[pad(kN2 / 2)];
      const float2 ym = cmul(make_float2(2.0f * zm.x, -2.0f * zm.y), p.H[kN2 / 2]);
      buf[pad(kN2 / 2)] = make_float2(2.0f * ym.x, -2.0f * ym.y);
      continue;
    }
    if (k == kN2 / 2) continue;
    const float2 zk = buf[pad(k)], zm = buf[pad(kN2 - k)];
    const float2 wk = w2048[k];                               // W_2048^k
    const float2 wm = w2048[kN2 - k];                         // W_2048^(1024 - k)
    // 2 X[k] = (Z[k] + Z*[m]) - i W^k (Z[k] - Z*[m]), m = 1024 - k; likewise 2 X[m]
    const float2 xk = csub(cadd(zk, conj2(zm)), mul_i<true>(cmul(wk, csub(zk, conj2(zm)))));
    const float2 xm = csub(cadd(zm, conj2(zk)), mul_i<true>(cmul(wm, csub(zm, conj2(zk)))));
    const float2 yk = cmul(xk, h_lo), ym = cmul(xm, h_hi);
    // Z'[k] = (Y[k] + Y*[m]) + i W^-k (Y[k] - Y*[m]), likewise Z'[m]
    buf[pad(k)] = cadd(cadd(yk, conj2(ym)), mul_i<true>(cmul(conj2(wk), csub(yk, conj2(ym)))));
    buf[pad(kN2 - k)] = cadd(cadd(ym, conj2(yk)), mul_i<true>(cmul(conj2(wm), csub(ym, conj2(yk)))));
  }
  __syncthreads();
  fft1024<true, kTpc>(buf, twl, tc);

  // store the block's rows: window position r = hm + i, i < B; complex n = r / 2
  // sits at the digit-reversed place after the DIF transform
  {
    const int cc = tid & (kCh - 1), rr0 = tid / kCh;
    const float2 *b2 = lds + cc * kPitch;
    const int64_t c = c0 + cc;
    for (int i = rr0; i < p.B; i += kThreads / kCh) {
      const int64_t t = t_out + i;
      if (t >= p.n_t || c >= p.n_ch) continue;
      const int r = p.hm + i;
      const float2 v = b2[pad(rev4(r >> 1))];
      __builtin_nontemporal_store((r & 1) ? v.y : v.x, p.y + t * p.n_ch + c);
    }
  }
  // The call's last workgroup to finish names the other history buffer the
  // current one and clears the count: every workgroup read the old name
  // before its first barrier, and a graph replay finds the count at 0.
  if (tid == 0) {
    const uint32_t done = atomicAdd(p.ctl + 1, 1u);
    if (done + 1 == p.total) {
      atomicXor(p.ctl, 1u);
      atomicExch(p.ctl + 1, 0u);
    }
  }
}

}  // namespace

hipError_t launch_fir_fft(const FftParams &p_in, hipStream_t stream) {
  FftParams p = p_in;
  if (p.B < 1 || p.hm < 0 || p.hm >= kFftN) return hipErrorInvalidValue;
  const int ch = p.ch == 4 ? 4 : 8;
  const int thr = p.threads == 512 && ch == 8 ? 512 : 256;
  const int64_t n_blk = (p.n_t + p.B - 1) / p.B;
  const int64_t n_cg = (p.n_ch + ch - 1) / ch;
  if (n_blk > 65535 || n_cg > ((int64_t)1 << 28) || n_cg * n_blk >= ((int64_t)1 << 32)) return hipErrorInvalidValue;
  p.per_xcd = (int32_t)((n_cg + 7) / 8);
  p.total = (uint32_t)(n_cg * n_blk);
  const dim3 grid((unsigned)(8 * p.per_xcd), (unsigned)n_blk);
  if (ch == 4)
    hipLaunchKernelGGL((fir_fft_kernel<4, 256>), grid, dim3(256), 0, stream, p);
  else if (thr == 512)
    hipLaunchKernelGGL((fir_fft_kernel<8, 512>), grid, dim3(512), 0, stream, p);
  else
    hipLaunchKernelGGL((fir_fft_kernel<8, 256>), grid, dim3(256), 0, stream, p);
  return hipGetLastError();
}

}  // namespace filark
