// Fused forward kernel: stateful SOS cascade and recursive STA/LTA over one
// chunk of a time-major channel x time record, in a single pass over HBM.
//
// The operation (FiLark Section 3.4): each channel's samples go through a
// cascade of second-order sections in direct-form-II-transposed state
// (z1, z2 per section); the state at the end of the chunk is the state the
// next chunk starts from, so any chunking gives the one-shot result.  The
// STA/LTA characteristic runs on the squared filter output with two
// exponential averages, whose state is carried the same way.
//
// Parallel form.  A section is linear: s_t = A s_{t-1} + B v_t, y_t = C s_{t-1}
// + D v_t with A = [[-a1, 1], [-a2, 0]], B = [b1 - a1 b0, b2 - a2 b0], C = [1 0],
// D = b0 (the DF2T delay pair is exactly s).  The cascade is one linear system
// with a 2K state and a block-lower-triangular transition.  The chunk is cut
// into blocks of L samples; the state entering block b satisfies the affine
// recurrence s_in(b+1) = A^L s_in(b) + a(b), where a(b) = sum_j A^(L-1-j) B x_j
// is the block's zero-state end state.  So:
//   pass 1   every lane projects its L samples onto a(b) (2K FMAs/sample);
//   carry    blocks are combined by that affine scan: inside a workgroup through
//            LDS, across workgroups (time segments) by a decoupled look-back on
//            per-segment records in global memory;
//   pass 2   every lane reruns the DF2T recurrence from its exact entry state
//            and emits y (and, for the chunk's last block, the carried state).
// STA/LTA repeats the same three steps with scalar decays on e = y^2.
//
// Mapping (gfx950): lanes are 64 consecutive channels, so every load and store
// of a row segment is one coalesced 256 B access through a buffer resource
// with the row offset in an SGPR; waves of a workgroup are consecutive time
// blocks; workgroups are (segment, channel group) tiles taken in segment-major
// ticket order, so a tile only ever waits on tiles that started before it.
// Filter arithmetic and all carries are FP64 (v_fma_f64 issues at the
// v_fma_f32 rate here); STA/LTA sums are FP32 within a block with FP64
// carries.  Coefficient and scan tables are read through the constant address
// space, i.e. scalar loads into SGPRs.  No MFMA: the path is HBM-bound.
#include "internal.h"

#define FILARK_CONST __attribute__((address_space(4)))

namespace filark {
namespace {

typedef const FILARK_CONST double cdouble;
typedef const FILARK_CONST float cfloat;

__device__ __forceinline__ cdouble *as_const(const double *p) { return (cdouble *)p; }
__device__ __forceinline__ cfloat *as_const(const float *p) { return (cfloat *)p; }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// A copy of a uniform value that the compiler must treat as new, so that values
// derived from it in one phase (row offsets) are recomputed by scalar ALU ops
// there instead of being kept live in SGPRs from an earlier phase.
__device__ __forceinline__ uint32_t fresh(uint32_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

__device__ __forceinline__ double ld_agent(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent_u32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_u32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// All of this wave's outstanding vector memory operations have completed.
// Record stores are agent-coherent atomics, so once they have completed a flag
// written afterwards can be relied on by any agent that reads it.
__device__ __forceinline__ void vm_drain() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Raw buffer resource at `base`: stride 0, byte offsets, 2^31 - 1 bytes in
// range.  Lanes whose channel is past n_ch use a byte offset of 2^31, which the
// hardware range check turns into a zero load and a dropped store.
constexpr uint32_t kOffInvalid = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, 0x7fffffff,
                                           0x00020000);
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                       float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 0);
}

// out = M v + add, M block-lower-triangular [NS][NS] with 2x2 diagonal blocks.
// Scheduling fences keep each row's scalar loads inside that row, so at most
// one row of M is live in SGPRs.
template <int NS>
__device__ __forceinline__ void mv_add(cdouble *M, const double (&v)[NS], const double (&add)[NS],
                                       double (&out)[NS]) {
  double r[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double s = add[i];
#pragma unroll
    for (int j = 0; j < (i / 2 + 1) * 2; ++j) s = fma(M[i * NS + j], v[j], s);
    r[i] = s;
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) out[i] = r[i];
}

// Decoupled look-back over the predecessors of segment `seg` in one channel
// group.  Lane q of the wave polls the flag of segment m - q; the nearest
// inclusive record (or the chunk's initial state, reached past segment 0)
// closes the sum, and every aggregate in front of it must be published:
//   prefix(seg) = sum_{q<d} W(q) agg(seg-1-q) + W(d) inc(seg-1-d),
// with W(q) the transition over q segments, applied by `comp`.  `init(v)`
// loads the chunk's initial state.  The wait is bounded by spin_limit polls;
// past it the error word is set and the (invalid) partial sum returned.
template <int R, class Comp, class Init>
__device__ void lookback(const FwdParams &p, const uint32_t *flags_g, const double *agg_g,
                         const double *inc_g, size_t seg_stride, int seg, uint32_t ep,
                         double (&acc)[R], Comp comp, Init init, int lane) {
#pragma unroll
  for (int i = 0; i < R; ++i) acc[i] = 0.0;
  int m = seg - 1;
  int pw = 0;
  int spins = 0;
  const uint32_t ep30 = ep & 0x3fffffffu;
  while (true) {
    const int idx = m - lane;
    uint32_t f = 0;
    if (idx >= 0) f = ld_agent_u32(flags_g + (size_t)idx * p.n_grp);
    const bool ready = idx < 0 || (((f >> 2) == ep30) && (f & 3u) != 0);
    const bool incl = idx < 0 || (ready && (f & 3u) == kFlagInclusive);
    const uint64_t ready_m = __ballot(ready);
    const uint64_t incl_m = __ballot(incl);
    const int d = incl_m ? __ffsll((unsigned long long)incl_m) - 1 : 64;
    const uint64_t need = d >= 63 ? ~0ull : ((2ull << d) - 1ull);
    if ((ready_m & need) != need) {
      if (++spins > p.spin_limit) {
        if (lane == 0) atomicOr(p.ctrl + kCtrlError, (uint32_t)kErrTimeout);
        return;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const int n_agg = d < 64 ? d : 64;
    for (int q = 0; q < n_agg; ++q) {
      const double *r = agg_g + (size_t)(m - q) * seg_stride;
      double v[R];
#pragma unroll
      for (int i = 0; i < R; ++i) v[i] = ld_agent(r + i * kWave + lane);
      comp(pw + q, v, acc);
    }
    if (d < 64) {
      const int mi = m - d;
      double v[R];
      if (mi >= 0) {
        const double *r = inc_g + (size_t)mi * seg_stride;
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = ld_agent(r + i * kWave + lane);
      } else {
        init(v);
      }
      comp(pw + d, v, acc);
      return;
    }
    m -= 64;
    pw += 64;
  }
}

template <int R>
__device__ __forceinline__ void publish(double *rec, const double (&v)[R], uint32_t *flag,
                                        uint32_t word, int lane) {
#pragma unroll
  for (int i = 0; i < R; ++i) st_agent(rec + i * kWave + lane, v[i]);
  vm_drain();
  if (lane == 0) st_agent_u32(flag, word);
}

template <int K, bool STALTA, bool WRITE_Y>
__global__ void __launch_bounds__(256) fwd_kernel(FwdParams p) {
  constexpr int L = kBlock;
  constexpr int NS = 2 * K;
  extern __shared__ double lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x / kWave);
  const int NW = blockDim.x / kWave;
  double *sh_agg = lds;                       // [NW][NS][64] block aggregates
  double *sh_pre = sh_agg + NW * NS * kWave;  // [NS][64]     segment aggregate, then prefix
  double *sh_sl = sh_pre + NS * kWave;        // [NW][2][64]  STA/LTA block sums
  double *sh_slp = sh_sl + NW * 2 * kWave;    // [2][64]      STA/LTA segment prefix
  uint32_t *sh_u = reinterpret_cast<uint32_t *>(sh_slp + 2 * kWave);  // [6]

  if (threadIdx.x == 0) {
    sh_u[0] = atomicAdd(p.ctrl + kCtrlTicket, 1u);
    sh_u[1] = ld_agent_u32(p.ctrl + kCtrlEpoch);
    sh_u[2] = K > 0 ? ld_agent_u32(p.sos_ctrl + kCtrlEpoch) : 0u;
    sh_u[3] = STALTA ? ld_agent_u32(p.sl_ctrl + kCtrlEpoch) : 0u;
    sh_u[4] = STALTA ? ld_agent_u32(p.sl_ctrl + kCtrlCounter) : 0u;
    sh_u[5] = STALTA ? ld_agent_u32(p.sl_ctrl + kCtrlCounter + 1) : 0u;
  }
  __syncthreads();
  const uint32_t ticket = (uint32_t)uniform((int)sh_u[0]);
  const uint32_t ep = (uint32_t)uniform((int)sh_u[1]);
  if (ticket >= (uint32_t)p.n_seg * (uint32_t)p.n_grp) {  // counters out of sync: never index with it
    if (threadIdx.x == 0) atomicOr(p.ctrl + kCtrlError, 2u);
    return;
  }
  const int seg = (int)(ticket / (uint32_t)p.n_grp);
  const int grp = (int)(ticket - (uint32_t)seg * (uint32_t)p.n_grp);
  const int64_t c = (int64_t)grp * kWave + lane;
  const bool cval = c < p.n_ch;
  const int row0 = seg * p.seg_len + w * L;
  const int nv = max(0, min(L, p.n_t - row0));
  const bool last_seg = seg == p.n_seg - 1;
  const bool last_rows = nv > 0 && row0 + nv == p.n_t;
  const size_t n_cells = (size_t)p.n_seg * (size_t)p.n_grp;
  // Byte offsets: the lane's channel (VGPR) and each row of the block (SGPR).
  const uint32_t voff = cval ? (uint32_t)c * 4u : kOffInvalid;
  const uint32_t rowb = (uint32_t)p.n_ch * 4u;
  const size_t blk_off = (size_t)row0 * (size_t)p.n_ch;

  // ---- load this wave's block: L rows x 64 channels, one 256 B segment per row
  float xv[L];
  {
    const __amdgpu_buffer_rsrc_t rx = rsrc(p.x + blk_off);
    const uint32_t rb = fresh(rowb);
    if (nv == L) {
#pragma unroll
      for (int j = 0; j < L; ++j) xv[j] = buf_ld(rx, voff, (uint32_t)j * rb);
    } else {
#pragma unroll
      for (int j = 0; j < L; ++j) xv[j] = j < nv ? buf_ld(rx, voff, (uint32_t)j * rb) : 0.0f;
    }
  }

  // STA/LTA block-end sums from zero, S = sum alpha_s^(n-1-j) e_j (same for L)
  double s_loc = 0.0, l_loc = 0.0;
  if constexpr (K > 0) {
    cdouble *G = as_const(p.G);
    cdouble *P = as_const(p.P);
    cdouble *Q = as_const(p.Q);
    cdouble *coef = as_const(p.coef);
    const int zpar = (int)(sh_u[2] & 1u);
    const double *zin = p.zs + (size_t)zpar * NS * p.n_ch;
    double *zout = p.zs + (size_t)(zpar ^ 1) * NS * p.n_ch;

    // ---- pass 1: zero-state block-end projection a = sum_j A^(L-1-j) B x_j.
    // Row j+1 of G is fetched into SGPRs while row j is applied; the fences
    // stop the scheduler from hoisting the whole table into SGPRs.
    {
      double a[NS], gn[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        a[i] = 0.0;
        gn[i] = G[i];
      }
#pragma unroll
      for (int j = 0; j < L; ++j) {
        double gc[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) gc[i] = gn[i];
        if (j + 1 < L) {
#pragma unroll
          for (int i = 0; i < NS; ++i) gn[i] = G[(j + 1) * NS + i];
        }
        const double xd = (double)xv[j];
#pragma unroll
        for (int i = 0; i < NS; ++i) a[i] = fma(gc[i], xd, a[i]);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int i = 0; i < NS; ++i) sh_agg[(w * NS + i) * kWave + lane] = a[i];
    }
    __syncthreads();

    // ---- segment carry: wave 0 publishes the segment aggregate and looks back
    if (w == 0) {
      const size_t rstride = (size_t)p.n_grp * NS * kWave;
      double *agg_g = p.rec + (size_t)grp * NS * kWave;
      double *inc_g = agg_g + n_cells * NS * kWave;
      uint32_t *flag_g = p.flags + grp;
      {
        double T[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) T[i] = sh_agg[i * kWave + lane];
        for (int v = 1; v < NW; ++v) {
          double av[NS];
#pragma unroll
          for (int i = 0; i < NS; ++i) av[i] = sh_agg[(v * NS + i) * kWave + lane];
          mv_add<NS>(P, T, av, T);
        }
        if (!last_seg)
          publish<NS>(agg_g + (size_t)seg * rstride, T, flag_g + (size_t)seg * p.n_grp,
                      (ep << 2) | kFlagAggregate, lane);
#pragma unroll
        for (int i = 0; i < NS; ++i) sh_pre[i * kWave + lane] = T[i];
      }
      double pre[NS];
      lookback<NS>(
          p, flag_g, agg_g, inc_g, rstride, seg, ep, pre,
          [Q](int m, const double (&v)[NS], double (&acc)[NS]) {
            mv_add<NS>(Q + (size_t)m * NS * NS, v, acc, acc);
          },
          [&](double (&v)[NS]) {
#pragma unroll
            for (int i = 0; i < NS; ++i) v[i] = cval ? zin[(size_t)i * p.n_ch + c] : 0.0;
          },
          lane);
      if (!last_seg) {
        double T[NS], inc[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) T[i] = sh_pre[i * kWave + lane];
        mv_add<NS>(Q + NS * NS, pre, T, inc);
        publish<NS>(inc_g + (size_t)seg * rstride, inc, flag_g + (size_t)seg * p.n_grp,
                    (ep << 2) | kFlagInclusive, lane);
      }
#pragma unroll
      for (int i = 0; i < NS; ++i) sh_pre[i * kWave + lane] = pre[i];
    }
    __syncthreads();

    // ---- this block's entry state: z = P^w pre + sum_{v<w} P^(w-1-v) a_v
    double z[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) z[i] = sh_pre[i * kWave + lane];
    for (int v = 0; v < w; ++v) {
      double av[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) av[i] = sh_agg[(v * NS + i) * kWave + lane];
      mv_add<NS>(P, z, av, z);
    }

    // ---- pass 2: DF2T recurrence from the exact entry state; y is stored as
    // it is produced.  A full block runs without per-row guards.
    double cb0[K], cb1[K], cb2[K], cna1[K], cna2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      cb0[k] = coef[5 * k + 0];
      cb1[k] = coef[5 * k + 1];
      cb2[k] = coef[5 * k + 2];
      cna1[k] = coef[5 * k + 3];
      cna2[k] = coef[5 * k + 4];
    }
    const __amdgpu_buffer_rsrc_t ry = rsrc(WRITE_Y ? (const void *)(p.y + blk_off) : (const void *)p.x);
    const uint32_t rb = fresh(rowb);
    auto step = [&](int j) {
      double v = (double)xv[j];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double yk = fma(cb0[k], v, z[2 * k]);
        z[2 * k] = fma(cna1[k], yk, fma(cb1[k], v, z[2 * k + 1]));
        z[2 * k + 1] = fma(cna2[k], yk, cb2[k] * v);
        v = yk;
      }
      const float yf = (float)v;
      xv[j] = yf;
      if constexpr (STALTA) {
        const double e = v * v;
        s_loc = fma(p.asd, s_loc, e);
        l_loc = fma(p.ald, l_loc, e);
      }
      if constexpr (WRITE_Y) buf_st(ry, voff, (uint32_t)j * rb, yf);
    };
    if (nv == L) {
#pragma unroll
      for (int j = 0; j < L; ++j) step(j);
    } else {
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (j < nv) step(j);
    }
    if (last_rows && cval) {
#pragma unroll
      for (int i = 0; i < NS; ++i) zout[(size_t)i * p.n_ch + c] = z[i];
    }
  } else {
    // STA/LTA only: the input is the filtered signal
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const double xd = (double)xv[j];
      const double e = xd * xd;
      s_loc = fma(p.asd, s_loc, e);
      l_loc = fma(p.ald, l_loc, e);
    }
  }

  if constexpr (STALTA) {
    cdouble *slq = as_const(p.slq);
    const int spar = (int)(sh_u[3] & 1u);
    const double *slin = p.sl + (size_t)spar * 2 * p.n_ch;
    double *slout = p.sl + (size_t)(spar ^ 1) * 2 * p.n_ch;
    const int64_t g0 = (int64_t)(((uint64_t)sh_u[5] << 32) | (uint64_t)sh_u[4]);
    const double aLs = slq[0], aLl = slq[1];
    cdouble *qs = slq + 2;
    cdouble *ql = slq + 2 + p.q_cap;

    sh_sl[(w * 2 + 0) * kWave + lane] = s_loc;
    sh_sl[(w * 2 + 1) * kWave + lane] = l_loc;
    __syncthreads();
    if (w == 0) {
      double T[2] = {sh_sl[0 * kWave + lane], sh_sl[1 * kWave + lane]};
      for (int v = 1; v < NW; ++v) {
        T[0] = fma(aLs, T[0], sh_sl[(v * 2 + 0) * kWave + lane]);
        T[1] = fma(aLl, T[1], sh_sl[(v * 2 + 1) * kWave + lane]);
      }
      const size_t rstride = (size_t)p.n_grp * 2 * kWave;
      double *agg_g = p.rec + n_cells * 2 * NS * kWave + (size_t)grp * 2 * kWave;
      double *inc_g = agg_g + n_cells * 2 * kWave;
      uint32_t *flag_g = p.flags + n_cells + grp;
      if (!last_seg)
        publish<2>(agg_g + (size_t)seg * rstride, T, flag_g + (size_t)seg * p.n_grp,
                   (ep << 2) | kFlagAggregate, lane);
      double pre[2];
      lookback<2>(
          p, flag_g, agg_g, inc_g, rstride, seg, ep, pre,
          [qs, ql](int m, const double (&v)[2], double (&acc)[2]) {
            acc[0] = fma(qs[m], v[0], acc[0]);
            acc[1] = fma(ql[m], v[1], acc[1]);
          },
          [&](double (&v)[2]) {
            v[0] = cval ? slin[c] * p.nsta_d : 0.0;
            v[1] = cval ? slin[p.n_ch + c] * p.nlta_d : 0.0;
          },
          lane);
      if (!last_seg) {
        double inc[2] = {fma(qs[1], pre[0], T[0]), fma(ql[1], pre[1], T[1])};
        publish<2>(inc_g + (size_t)seg * rstride, inc, flag_g + (size_t)seg * p.n_grp,
                   (ep << 2) | kFlagInclusive, lane);
      }
      sh_slp[lane] = pre[0];
      sh_slp[kWave + lane] = pre[1];
    }
    __syncthreads();
    double S = sh_slp[lane], Lg = sh_slp[kWave + lane];
    for (int v = 0; v < w; ++v) {
      S = fma(aLs, S, sh_sl[(v * 2 + 0) * kWave + lane]);
      Lg = fma(aLl, Lg, sh_sl[(v * 2 + 1) * kWave + lane]);
    }
    float Sf = (float)S, Lf = (float)Lg;
    const __amdgpu_buffer_rsrc_t rc = rsrc(p.cf + blk_off);
    const uint32_t rb = fresh(rowb);
    const int64_t gfirst = g0 + row0;
    auto stepb = [&](int j) {
      const float e = xv[j] * xv[j];
      Sf = fmaf(p.as, Sf, e);
      Lf = fmaf(p.al, Lf, e);
      const float r = Lf > 0.0f ? p.kappa * Sf * __builtin_amdgcn_rcpf(Lf) : 0.0f;
      const float out = (gfirst + j >= p.nlta) ? r : 0.0f;
      buf_st(rc, voff, (uint32_t)j * rb, out);
    };
    if (nv == L) {
#pragma unroll
      for (int j = 0; j < L; ++j) stepb(j);
    } else {
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (j < nv) stepb(j);
    }
    if (last_rows && cval) {
      slout[c] = (double)Sf / p.nsta_d;
      slout[p.n_ch + c] = (double)Lf / p.nlta_d;
    }
  }

  // ---- the last tile to finish resets the ticket counters and advances epochs
  if (threadIdx.x == 0) {
    const uint32_t total = (uint32_t)n_cells;
    const uint32_t prev = atomicAdd(p.ctrl + kCtrlDone, 1u);
    if (prev == total - 1) {
      st_agent_u32(p.ctrl + kCtrlTicket, 0u);
      st_agent_u32(p.ctrl + kCtrlDone, 0u);
      if (K > 0) st_agent_u32(p.sos_ctrl + kCtrlEpoch, sh_u[2] + 1u);
      if (STALTA) {
        st_agent_u32(p.sl_ctrl + kCtrlEpoch, sh_u[3] + 1u);
        const uint64_t g1 = (((uint64_t)sh_u[5] << 32) | (uint64_t)sh_u[4]) + (uint64_t)p.n_t;
        st_agent_u32(p.sl_ctrl + kCtrlCounter, (uint32_t)g1);
        st_agent_u32(p.sl_ctrl + kCtrlCounter + 1, (uint32_t)(g1 >> 32));
      }
    }
  }
}

template <int K, bool S, bool Y>
hipError_t launch_one(const FwdParams &p, int waves, hipStream_t stream) {
  constexpr int NS = 2 * K;
  const size_t lds = (size_t)(waves * NS * kWave + NS * kWave + waves * 2 * kWave + 2 * kWave) *
                         sizeof(double) + 8 * sizeof(uint32_t);
  const dim3 grid((unsigned)(p.n_seg * p.n_grp));
  const dim3 block((unsigned)(waves * kWave));
  hipLaunchKernelGGL((fwd_kernel<K, S, Y>), grid, block, lds, stream, p);
  return hipGetLastError();
}

template <int K>
hipError_t launch_k(const FwdParams &p, bool stalta, bool write_y, int waves, hipStream_t stream) {
  if (!stalta) return launch_one<K, false, true>(p, waves, stream);
  if (write_y) return launch_one<K, true, true>(p, waves, stream);
  return launch_one<K, true, false>(p, waves, stream);
}

}  // namespace

size_t fwd_lds_bytes(int K, int waves) {
  const int NS = 2 * K;
  return (size_t)(waves * NS * kWave + NS * kWave + waves * 2 * kWave + 2 * kWave) *
             sizeof(double) + 8 * sizeof(uint32_t);
}

hipError_t launch_fwd(const FwdParams &p, int K, bool stalta, bool write_y, int waves,
                      hipStream_t stream) {
  switch (K) {
    case 0: return launch_one<0, true, false>(p, waves, stream);
    case 1: return launch_k<1>(p, stalta, write_y, waves, stream);
    case 2: return launch_k<2>(p, stalta, write_y, waves, stream);
    case 3: return launch_k<3>(p, stalta, write_y, waves, stream);
    case 4: return launch_k<4>(p, stalta, write_y, waves, stream);
    case 5: return launch_k<5>(p, stalta, write_y, waves, stream);
    case 6: return launch_k<6>(p, stalta, write_y, waves, stream);
    case 7: return launch_k<7>(p, stalta, write_y, waves, stream);
    case 8: return launch_k<8>(p, stalta, write_y, waves, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace filark
