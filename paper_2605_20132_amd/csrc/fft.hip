// FFT filtering of the realtime FIR (the overlap-add / overlap-save FFT
// filtering of Table 1's FIR row; Section 6.2 reports its GPU speed-up):
// y[t] = sum_k h[k] x[t - k] computed block by block in the frequency domain,
// the samples before the call taken from the carried history (the last M - 1
// input rows, the state the direct kernel carries too).
//
// Block.  A workgroup takes 8 consecutive channels and one block of
// B = N - (M - 1) output rows, N = 2048: the window of N input rows that ends
// with the block (M - 1 rows before it, from the chunk or the history),
// whose circular convolution with the zero-padded taps equals the linear one
// at the window's last B positions (overlap-save; overlap-add gives the same
// sums with the tail carried instead of the history).  Per channel:
//   z[n] = x[2n] + i x[2n + 1]          two real samples per complex value
//   Z = FFT_1024(z)                      radix-4, in place in LDS (DIT: the
//                                        input is placed digit-reversed)
//   X[k] = E + W_2048^k O, E = (Z[k] + Z*[1024 - k]) / 2, O = (Z[k] - Z*[1024 - k]) / 2i
//   Y[k] = X[k] H[k]                     H: the taps' 2048-point spectrum
//   Z'[k] = E' + i O', E' = (Y[k] + Y*[1024 - k]) / 2, O' = W_2048^-k (Y[k] - Y*[1024 - k]) / 2
//   z' = IFFT_1024(Z')                   radix-4 DIF: digit-reversed output
//   y[2n] = Re z'[n], y[2n + 1] = Im z'[n]
// The factors 1/2 and the 1/1024 of the inverse are folded into H on the
// host.  FP32 throughout (twiddles and H rounded from FP64); the error bound
// is that of FP32 transforms, not the direct kernel's exact summation order.
#include "device.h"
#include "fir.h"

namespace filark {
namespace {

constexpr int kN2 = kFftN / 2;           // complex points per channel
constexpr int kCh = 8;                   // channels per workgroup
constexpr int kThreads = 256;
constexpr int kTpc = kThreads / kCh;     // threads per channel
constexpr int kPitch = kN2;              // LDS float2 per channel (64 KB for the workgroup)

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

// In-place radix-4 transform of 1024 points of one channel held by kTpc
// threads: DIT from digit-reversed input to natural output (forward), or DIF
// from natural input to digit-reversed output (inverse).  Each stage runs
// 256 butterflies, 8 per thread, separated by workgroup barriers.
template <bool INV>
__device__ __forceinline__ void fft1024(float2 *buf, const float2 *__restrict__ w1024, int tc) {
#pragma unroll
  for (int st = 0; st < 5; ++st) {
    const int s = INV ? 4 - st : st;     // DIF runs the spans from 256 down to 1
    const int S = 1 << (2 * s);          // span: the sub-transforms combined have length 4 S
    const int step = kN2 / (4 * S);      // W_(4S)^j = W_1024^(j step)
#pragma unroll
    for (int u = 0; u < 256 / kTpc; ++u) {
      const int b = tc + u * kTpc;       // butterfly 0 .. 255
      const int j = b & (S - 1), g = b >> (2 * s);
      const int base = g * 4 * S + j;
      float2 a0 = buf[pad(base)], a1 = buf[pad(base + S)], a2 = buf[pad(base + 2 * S)], a3 = buf[pad(base + 3 * S)];
      if (!INV) {  // DIT: twiddle, then the 4-point transform
        a1 = cmul(a1, tw<INV>(w1024, j * step));
        a2 = cmul(a2, tw<INV>(w1024, 2 * j * step));
        a3 = cmul(a3, tw<INV>(w1024, 3 * j * step));
        dft4<INV>(a0, a1, a2, a3);
      } else {     // DIF: the 4-point transform, then the twiddle
        dft4<INV>(a0, a1, a2, a3);
        a1 = cmul(a1, tw<INV>(w1024, j * step));
        a2 = cmul(a2, tw<INV>(w1024, 2 * j * step));
        a3 = cmul(a3, tw<INV>(w1024, 3 * j * step));
      }
      buf[pad(base)] = a0;
      buf[pad(base + S)] = a1;
      buf[pad(base + 2 * S)] = a2;
      buf[pad(base + 3 * S)] = a3;
    }
    __syncthreads();
  }
}

// Row t of the chunk for channel c: the chunk (0 <= t < n_t), the history
// (-(M - 1) <= t < 0, oldest row first) or 0 (past the chunk).
__device__ __forceinline__ float fft_in(const FftParams &p, const float *hist, int64_t t, int64_t c) {
  if (c >= p.n_ch || t >= p.n_t) return 0.0f;
  if (t >= 0) return __builtin_nontemporal_load(p.x + t * p.n_ch + c);
  const int64_t r = t + p.hm;
  return r >= 0 ? hist[r * p.n_ch + c] : 0.0f;
}

__global__ void __launch_bounds__(kThreads) fir_fft_kernel(FftParams p) {
  __shared__ float2 lds[kCh * kPitch];
  const int tid = (int)threadIdx.x;
  const int cg = (int)blockIdx.x, blk = (int)blockIdx.y;
  const int64_t c0 = (int64_t)cg * kCh;
  const int64_t t_out = (int64_t)blk * p.B;      // first output row of the block
  const int64_t t_win = t_out - p.hm;            // chunk row of window position 0
  const float *hist = (p.ctl[0] & 1u) ? p.hist1 : p.hist0;
  const float2 *w1024 = p.tw;
  const float2 *w2048 = p.tw + kN2;

  // load: thread (row rr, channel cc); a wave covers 8 rows of 8 channels;
  // window sample r goes to complex n = r / 2 (real part for even r) at the
  // digit-reversed place
  {
    const int cc = tid & (kCh - 1), rr0 = tid / kCh;
    float2 *buf = lds + cc * kPitch;
    for (int n = rr0; n < kN2; n += kThreads / kCh) {
      const int64_t t = t_win + 2 * n;
      const float e = fft_in(p, hist, t, c0 + cc), o = fft_in(p, hist, t + 1, c0 + cc);
      buf[pad(rev4(n))] = make_float2(e, o);
    }
  }
  __syncthreads();
  const int ch = tid / kTpc, tc = tid & (kTpc - 1);
  float2 *buf = lds + ch * kPitch;
  fft1024<false>(buf, w1024, tc);

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
  fft1024<true>(buf, w1024, tc);

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
}

// The new history: row r of the M - 1 rows before the end of the call, from
// the chunk (chunk row n_t - (M - 1) + r >= 0) or the old history.
__global__ void __launch_bounds__(256) fir_hist_kernel(FftParams p) {
  const int64_t n = (int64_t)p.hm * p.n_ch;
  const float *old = (p.ctl[0] & 1u) ? p.hist1 : p.hist0;
  float *nw = (p.ctl[0] & 1u) ? p.hist0 : p.hist1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / p.n_ch, c = i - r * p.n_ch;
    const int64_t t = p.n_t - p.hm + r;
    nw[i] = t >= 0 ? p.x[t * p.n_ch + c] : old[(t + p.hm) * p.n_ch + c];
  }
}

}  // namespace

hipError_t launch_fir_fft(const FftParams &p, hipStream_t stream) {
  if (p.B < 1 || p.hm < 0 || p.hm >= kFftN) return hipErrorInvalidValue;
  const int64_t n_blk = (p.n_t + p.B - 1) / p.B;
  const int64_t n_cg = (p.n_ch + kCh - 1) / kCh;
  if (n_blk > 65535 || n_cg > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fir_fft_kernel, dim3((unsigned)n_cg, (unsigned)n_blk), dim3(kThreads), 0, stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.hm == 0) return e;
  const int64_t n = (int64_t)p.hm * p.n_ch;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fir_hist_kernel, dim3(grid), dim3(256), 0, stream, p);
  return hipGetLastError();
}

}  // namespace filark
