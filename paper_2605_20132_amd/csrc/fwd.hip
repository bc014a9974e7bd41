// Forward launches: the per-block-length dispatch (kernels instantiated in
// fwd_l32.hip, fwd_l48.hip, fwd_l64.hip) and the batched multi-stream launch.
#include "fwd_body.h"

namespace filark {

using namespace fwdk;

// Dynamic LDS of one workgroup, all FP64: STA/LTA exchange [2][nw * 64][2],
// filter scan exchange [1 or 2][nw * 64][2K + 1] (the odd row pitch spreads a
// wave's rows over the banks), level matrices [n_lev][2K][2K], and the staged
// carried state of the cw channels: filter [cw][2K + 1], STA/LTA sums [cw][2].
size_t fwd_lds_bytes(int K, int nw, int n_lev, int cw) {
  const int NS = 2 * K, NSP = NS + 1;
  const size_t n = (size_t)nw * kWave;
  return (n * (4 + NSP * (fwd_double_buffer(K, nw) ? 2 : 1)) + (size_t)n_lev * NS * NS + (size_t)cw * (NSP + 2)) *
         sizeof(double);
}

namespace {

// Batched launch: workgroup i runs item i of a host-built table, a channel
// group of one stream's window (its descriptor), or nothing (padding).  Items
// are laid out so that XCD i % 8 holds a contiguous slab of every stream's
// groups.  At its end each workgroup raises its stream's completion stamp
// (the device's 100 MHz clock) with an atomic max.
template <int K, int L>
__global__ void __launch_bounds__(kMaxWaves * kWave) __attribute__((amdgpu_waves_per_eu(L >= 48 ? 3 : 1)))
fwd_batch_kernel(BatchParams) {
  const FILARK_CONST BatchParams *bp = dev::kparams<BatchParams>();
  const FILARK_CONST BatchItem *it = (const FILARK_CONST BatchItem *)bp->items + blockIdx.x;
  const int desc = it->desc;
  if (desc < 0) return;  // padding, whole workgroup
  const PSrc ps{(kparams_t)(bp->descs + desc)};
  fwd_body<K, L, false, true, false, false, false>(ps, it->group);
  unsigned long long *stamps = bp->stamps;
  if (stamps) {
    __syncthreads();  // every wave's stores have completed
    if (threadIdx.x == 0) atomicMax(stamps + it->stream, (unsigned long long)__builtin_amdgcn_s_memrealtime());
  }
}

// Clear the completion stamps of n streams and record the start stamp in
// slot n (a fill kernel, so the reset can live in a captured graph).
__global__ void __launch_bounds__(256) stamp_reset_kernel(unsigned long long *stamps, int n) {
  for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) stamps[i] = 0ull;
  if (threadIdx.x == 0) stamps[n] = (unsigned long long)__builtin_amdgcn_s_memrealtime();
}

template <int K, int L>
hipError_t launch_batch_k(const BatchParams &bp, int n_items, int nw, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((fwd_batch_kernel<K, L>), dim3((unsigned)n_items), dim3((unsigned)(nw * kWave)), lds,
                     stream, bp);
  return hipGetLastError();
}

template <int L>
hipError_t launch_batch_l(const BatchParams &bp, int K, int n_items, int nw, size_t lds, hipStream_t stream) {
  switch (K) {
    case 1: return launch_batch_k<1, L>(bp, n_items, nw, lds, stream);
    case 2: return launch_batch_k<2, L>(bp, n_items, nw, lds, stream);
    case 3: return launch_batch_k<3, L>(bp, n_items, nw, lds, stream);
    case 4: return launch_batch_k<4, L>(bp, n_items, nw, lds, stream);
    case 5: return launch_batch_k<5, L>(bp, n_items, nw, lds, stream);
    case 6: return launch_batch_k<6, L>(bp, n_items, nw, lds, stream);
    case 7: return launch_batch_k<7, L>(bp, n_items, nw, lds, stream);
    case 8: return launch_batch_k<8, L>(bp, n_items, nw, lds, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_fwd_batch(const BatchParams &bp, int K, int L, int n_items, int nw, int max_lev,
                            hipStream_t stream) {
  if (n_items < 1 || nw < 1 || nw > kMaxWaves || max_lev < 1 || max_lev > kMaxLevels) return hipErrorInvalidValue;
  const size_t lds = fwd_lds_bytes(K, nw, max_lev, kWave);  // any stream's group
  if (L == 32) return launch_batch_l<32>(bp, K, n_items, nw, lds, stream);
  if (L == 48) return launch_batch_l<48>(bp, K, n_items, nw, lds, stream);
  if (L == 64) return launch_batch_l<64>(bp, K, n_items, nw, lds, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_stamp_reset(unsigned long long *stamps, int n, hipStream_t stream) {
  hipLaunchKernelGGL(stamp_reset_kernel, dim3(1), dim3(256), 0, stream, stamps, n);
  return hipGetLastError();
}

hipError_t launch_fwd(const FwdParams &p, int K, int L, bool stalta, bool write_y, bool unit, bool rev,
                      hipStream_t stream) {
  if (p.nw < 1 || p.nw > kMaxWaves || p.n_t < 1 || p.n_lev < 1 || p.n_lev > kMaxLevels)
    return hipErrorInvalidValue;
  if (L == 32) return launch_fwd_l32(p, K, stalta, write_y, unit, rev, stream);
  if (L == 48) return launch_fwd_l48(p, K, stalta, write_y, unit, rev, stream);
  if (L == 64) return launch_fwd_l64(p, K, stalta, write_y, unit, rev, stream);
  return hipErrorInvalidValue;
}

}  // namespace filark
