// Device helpers shared by the forward and adjoint kernels (gfx950).
#pragma once

#include "internal.h"

#define FILARK_CONST __attribute__((address_space(4)))

namespace filark {
namespace dev {

typedef const FILARK_CONST double cdouble;

__device__ __forceinline__ cdouble *as_const(const double *p) { return (cdouble *)p; }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A copy of a uniform value that the compiler must treat as new.  Row offsets
// are formed from it in each phase right where they are used, instead of one
// set of per-row offsets being kept live in VGPRs across all phases.
__device__ __forceinline__ uint32_t fresh(uint32_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

// FP64 value of a register-resident float, opaque to the compiler: each call
// site (its TAG) converts afresh, so the conversions of one phase are not
// kept live (two registers each) to be reused by a later phase.
template <int TAG>
__device__ __forceinline__ double widen(float x) {
  asm("; widen %1" : "+v"(x) : "n"(TAG));
  return (double)x;
}

// Kernel parameters are read through the kernarg-segment pointer, taken
// afresh in every phase: each phase scalar-loads only the fields it uses,
// and nothing from the parameter block stays live across other phases.
template <class P>
__device__ __forceinline__ const FILARK_CONST P *kparams() {
  const FILARK_CONST P *k = (const FILARK_CONST P *)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(k));
  return k;
}

// Raw buffer resource over `range` bytes at `base` (stride 0, byte offsets).
// Offsets at or past `range` read zero and drop stores; lanes whose channel
// is past n_ch use an offset of 2^31, which is always out of range.
constexpr uint32_t kOffInvalid = 0x80000000u;
// s_waitcnt immediate that waits for LDS / scalar-memory results only
// (lgkmcnt 0; vmcnt and expcnt at their maxima)
constexpr int kWaitLgkm0 = 0xc07f;
// ... and for vector memory only (vmcnt 0; expcnt and lgkmcnt at their maxima)
constexpr int kWaitVm0 = 0x0f70;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, int range) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, range, 0x00020000);
}
// NT: the non-temporal hint, for inputs read once (the lines are not kept
// for reuse in L2).
template <bool NT = false>
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, NT ? 2 : 0));
}
// NT: the non-temporal hint, for outputs never read again.  It pays where a
// workgroup writes at least 64 contiguous bytes of a row (the lines go out
// without lingering in L2); with 32-byte row pieces the partial lines of
// neighbouring workgroups no longer merge in L2 and every piece becomes its
// own memory write, so narrow groups store without it.
template <bool NT = false>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t voff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, 0, NT ? 2 : 0);
}

// Row j of a lane's block through a buffer resource rebased to that row:
// base + j * rb with the range shortened by as much (never below zero), so
// the lane keeps its block-start offset for every row (no per-row vector
// address arithmetic; the rebasing is scalar) and the range check still
// drops exactly the rows past the end.  range and j * rb stay below 2^31.
struct RowBuf {
  const char *base;
  uint32_t range, rb;
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t at(int j) const {
    const uint32_t d = (uint32_t)j * rb;
    int r = (int)range - (int)d;
    r = r < 0 ? 0 : r;
    asm volatile("" : "+s"(r));  // scalar: a vector select here would make every access a loop over lanes
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(base + d), (short)0, r, 0x00020000);
  }
};

// Workgroup barrier for data exchanged through LDS only: each wave waits for
// its own LDS operations, then all waves meet.  Unlike __syncthreads() it
// does not wait for outstanding global loads and stores, which the kernels
// never exchange between waves of a workgroup (global values read before a
// barrier are consumed before it), so stores keep draining and prefetched
// loads keep arriving across the scans.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// acc += M v for a block-lower-triangular M [NS][NS] (2x2 diagonal blocks)
// held in LDS; all lanes read the same entries (broadcast).  The fences keep
// one row of M in registers at a time.
template <int NS>
__device__ __forceinline__ void mv_acc(const double *M, const double (&v)[NS], double (&acc)[NS]) {
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double s = acc[i];
#pragma unroll
    for (int j = 0; j < (i / 2 + 1) * 2; ++j) s = fma(M[i * NS + j], v[j], s);
    acc[i] = s;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Entries of the lower block triangle of a block-lower-triangular [NS][NS]
// matrix (2x2 blocks), row by row: 2K(K+1) for NS = 2K.
template <int NS>
constexpr int tri_count() {
  return (NS / 2) * (NS / 2 + 1) * 2;
}

// The lower block triangle of a wave-uniform matrix, scalar-loaded (SGPRs:
// one fetch per wave, where an LDS read would return 64 copies).
template <int NS>
__device__ __forceinline__ void tri_load(cdouble *M, double (&m)[tri_count<NS>()]) {
  int k = 0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
#pragma unroll
    for (int j = 0; j < (i / 2 + 1) * 2; ++j) m[k++] = M[i * NS + j];
  }
}

// acc += M v with M given by tri_load.
template <int NS>
__device__ __forceinline__ void tri_mv_acc(const double (&m)[tri_count<NS>()], const double (&v)[NS],
                                           double (&acc)[NS]) {
  int k = 0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double s = acc[i];
#pragma unroll
    for (int j = 0; j < (i / 2 + 1) * 2; ++j) s = fma(m[k++], v[j], s);
    acc[i] = s;
  }
}

// acc += M^T v with M given by tri_load.
template <int NS>
__device__ __forceinline__ void tri_mtv_acc(const double (&m)[tri_count<NS>()], const double (&v)[NS],
                                            double (&acc)[NS]) {
  int k = 0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
#pragma unroll
    for (int j = 0; j < (i / 2 + 1) * 2; ++j) acc[j] = fma(m[k++], v[i], acc[j]);
  }
}

// acc += M^T v for the same M (block-upper-triangular product).
template <int NS>
__device__ __forceinline__ void mtv_acc(const double *M, const double (&v)[NS], double (&acc)[NS]) {
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    double s = acc[j];
#pragma unroll
    for (int i = (j / 2) * 2; i < NS; ++i) s = fma(M[i * NS + j], v[i], s);
    acc[j] = s;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Zero-state block-end projection a = sum_j A^(L-1-j) B x_j = sum_j G_j x_j
// of a block of L samples held in registers (G: [L][2K], row j = A^(L-1-j) B).
// The
// rows of G are scalar-loaded (one fetch per wave) in batches of D rows.
// Scalar loads complete out of order, so any wait for one waits for all: the
// next batch is therefore issued only after the first use of the current one
// (which is where that wait sits), and arrives while the rest of the batch is
// applied.  The fences keep this order and stop the scheduler from hoisting
// the whole table into SGPRs.
template <int K, int L>
__device__ __forceinline__ void project(cdouble *G, const float (&xv)[L], double (&a)[2 * K]) {
  constexpr int NS = 2 * K;
  constexpr int D = NS >= 16 ? 1 : 16 / NS;  // two batches of D rows: 4 D NS SGPRs
  double cur[D][NS], nxt[D][NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) a[i] = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
#pragma unroll
    for (int i = 0; i < NS; ++i) cur[d][i] = d < L ? G[d * NS + i] : 0.0;
  }
#pragma unroll
  for (int jb = 0; jb < L; jb += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int j = jb + d;
      if (j < L) {
        const double xd = (double)xv[j];
        a[0] = fma(cur[d][0], xd, a[0]);
        if (d == 0) {
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int e = 0; e < D; ++e) {
#pragma unroll
            for (int i = 0; i < NS; ++i) nxt[e][i] = jb + D + e < L ? G[(jb + D + e) * NS + i] : 0.0;
          }
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int i = 1; i < NS; ++i) a[i] = fma(cur[d][i], xd, a[i]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
      for (int i = 0; i < NS; ++i) cur[d][i] = nxt[d][i];
    }
  }
}

// Channel group of a workgroup.  Workgroups are dealt to the 8 XCDs
// round-robin by index, so workgroup w runs on XCD w % 8; XCD x is given the
// contiguous slab of groups [x * per_xcd, (x + 1) * per_xcd), which keeps the
// rows of neighbouring groups, which share cache lines, in one L2.
//   order 0: the XCD's workgroups take the slab in dispatch order, so the
//            groups that share a line run side by side (their partial-line
//            writes merge in L2: needed by 32-byte row pieces);
//   order 1: dispatch position p takes the p-th of 0, 3, 6, ..., 1, 4, 7, ...,
//            2, 5, 8, ...: the workgroups each CU receives first then cover
//            every line of every row together, which measured faster for
//            groups writing 64-byte pieces with the non-temporal hint.
__device__ __forceinline__ int group_of(int per_xcd, int order = 0) {
  const int wg = (int)blockIdx.x;
  const int p = wg >> 3;
  int q = p;
  if (order == 1) {
    const int c0 = (per_xcd + 2) / 3, c1 = (per_xcd + 1) / 3;  // counts of 0 and 1 mod 3 below per_xcd
    q = p < c0 ? 3 * p : (p < c0 + c1 ? 3 * (p - c0) + 1 : 3 * (p - c0 - c1) + 2);
  }
  return uniform((wg & 7) * per_xcd + q);
}

}  // namespace dev
}  // namespace filark
