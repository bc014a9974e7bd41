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

// One item: channel group g of one stream, its windows in order.  The state a
// window's last-row lanes write is read by the next window's first-block
// lanes, other waves of this workgroup: the release / acquire fences at
// workgroup scope around the barrier order those global accesses (the
// workgroup's waves share one L1).
template <int K>
__device__ __forceinline__ void batch_walk(const FILARK_CONST BatchParams *bp, const FILARK_CONST BatchItem *it) {
  const int desc0 = it->desc0, n_win = it->n_win, g = it->group;
  for (int w = 0; w < n_win; ++w) {
    const PSrc ps{(kparams_t)(bp->descs + desc0 + w)};
    fwd_body<K, 48, false, true, false, false, false>(ps, g);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
}

// The persistent batched kernel for cascades of up to KMAX sections (the
// registers are those of the largest cascade compiled in, so the host picks
// the smallest KMAX that covers its streams).  Every workgroup leaves when
// its XCD's queue is empty; the last one to leave clears the counters for
// the next launch, so a launch is this one kernel (no reset kernel before
// it, in a graph or not).
template <int KMAX>
__global__ void __launch_bounds__(kMaxWaves * kWave) __attribute__((amdgpu_waves_per_eu(3)))
fwd_batch_kernel(BatchParams) {
  const FILARK_CONST BatchParams *bp = dev::kparams<BatchParams>();
  __shared__ int next;
  const int x = (int)blockIdx.x & 7;
  const int q0 = bp->qoff[x], q1 = bp->qoff[x + 1];
  const bool wave0 = uniform((int)(threadIdx.x / kWave)) == 0;  // a scalar branch
  const bool lane0 = (threadIdx.x & (kWave - 1)) == 0;
  // The loop holds no lane-divergent branch: one around the barriers of a
  // loop lets the compiler split it into nested loops in which the waves can
  // come back to the barriers without taking a new item.  So the whole of
  // wave 0 takes the next item (lane 0 adds 1, the others 0) and every lane
  // of it writes the same index.
  for (;;) {
    if (wave0) {
      const uint32_t old = atomicAdd(bp->heads + x, lane0 ? 1u : 0u);
      const int taken = __builtin_amdgcn_readfirstlane((int)old);
      next = q0 + taken;
      // the launch's start: the first item of XCD 0's queue (every lane
      // stores the same value)
      if (x == 0 && taken == 0) bp->stamps[bp->n_streams] = __builtin_amdgcn_s_memrealtime();
    }
    __syncthreads();
    const int i = uniform(next);
    __syncthreads();  // every wave has read `next` before it is written again
    if (i >= q1) {  // the whole workgroup: i is uniform
      if (wave0) {
        // workgroups leave once their last atomic on the queue counters is
        // done, so the last one to leave finds no other still using them
        const uint32_t done = atomicAdd(bp->heads + 8, lane0 ? 1u : 0u);
        if (__builtin_amdgcn_readfirstlane((int)done) + 1 == (int)gridDim.x && lane0) {
#pragma unroll
          for (int k = 0; k < 9; ++k) atomicExch(bp->heads + k, 0u);
        }
      }
      break;
    }
    const FILARK_CONST BatchItem *it = (const FILARK_CONST BatchItem *)bp->items + i;
    switch (it->K) {
      case 1: batch_walk<1>(bp, it); break;
      case 2: if constexpr (KMAX >= 2) batch_walk<2>(bp, it); break;
      case 3: if constexpr (KMAX >= 3) batch_walk<3>(bp, it); break;
      case 4: if constexpr (KMAX >= 4) batch_walk<4>(bp, it); break;
      case 5: if constexpr (KMAX >= 5) batch_walk<5>(bp, it); break;
      case 6: if constexpr (KMAX >= 6) batch_walk<6>(bp, it); break;
      case 7: if constexpr (KMAX >= 7) batch_walk<7>(bp, it); break;
      case 8: if constexpr (KMAX >= 8) batch_walk<8>(bp, it); break;
      default: break;
    }
    // batch_walk ends on a barrier: every wave's stores of the item are done
    if (wave0) {
      const unsigned long long now = __builtin_amdgcn_s_memrealtime();
      atomicMax(bp->stamps + it->stream, lane0 ? now : 0ull);
    }
  }
}

template <int KMAX>
hipError_t launch_batch_k(const BatchParams &bp, int grid, int nw, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((fwd_batch_kernel<KMAX>), dim3((unsigned)grid), dim3((unsigned)(nw * kWave)), lds, stream, bp);
  return hipGetLastError();
}

template <int KMAX>
hipError_t occupancy_k(int nw, size_t lds, int *per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, reinterpret_cast<const void *>(&fwd_batch_kernel<KMAX>),
                                                      nw * kWave, lds);
}

}  // namespace

hipError_t launch_fwd_batch(const BatchParams &bp, int kmax, int grid, int nw, size_t lds, hipStream_t stream) {
  if (grid < 1 || nw < 1 || nw > kMaxWaves) return hipErrorInvalidValue;
  switch (kmax) {
    case 1: return launch_batch_k<1>(bp, grid, nw, lds, stream);
    case 2: return launch_batch_k<2>(bp, grid, nw, lds, stream);
    case 3: return launch_batch_k<3>(bp, grid, nw, lds, stream);
    case 4: return launch_batch_k<4>(bp, grid, nw, lds, stream);
    case 5: return launch_batch_k<5>(bp, grid, nw, lds, stream);
    case 6: return launch_batch_k<6>(bp, grid, nw, lds, stream);
    case 7: return launch_batch_k<7>(bp, grid, nw, lds, stream);
    case 8: return launch_batch_k<8>(bp, grid, nw, lds, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t batch_occupancy(int kmax, int nw, size_t lds, int *per_cu) {
  switch (kmax) {
    case 1: return occupancy_k<1>(nw, lds, per_cu);
    case 2: return occupancy_k<2>(nw, lds, per_cu);
    case 3: return occupancy_k<3>(nw, lds, per_cu);
    case 4: return occupancy_k<4>(nw, lds, per_cu);
    case 5: return occupancy_k<5>(nw, lds, per_cu);
    case 6: return occupancy_k<6>(nw, lds, per_cu);
    case 7: return occupancy_k<7>(nw, lds, per_cu);
    case 8: return occupancy_k<8>(nw, lds, per_cu);
    default: return hipErrorInvalidValue;
  }
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
