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
// recurrence s_in(b+1) = P s_in(b) + a(b), P = A^L, where a(b) =
// sum_j A^(L-1-j) B x_j is the block's zero-state end state.  So:
//   pass 1   every lane projects its L samples onto a(b) (2K FMAs/sample);
//   carry    blocks are combined by that affine scan: inside a workgroup by a
//            dedicated carry wave through LDS, across workgroups (time
//            segments) by a decoupled look-back on per-segment records;
//   pass 2   every lane reruns the DF2T recurrence from its exact entry state
//            and emits y (and, for the chunk's last block, the carried state).
// STA/LTA repeats the same three steps with scalar decays on e = y^2.
//
// Mapping (gfx950): lanes are 64 consecutive channels, so every load and store
// of a row segment is one coalesced 256 B access through a buffer resource
// with the row offset in an SGPR.  A workgroup holds NW data waves, which own
// consecutive time blocks of one segment, and one carry wave, which owns all
// cross-block and cross-segment arithmetic, so the data waves hold only
// their block and filter state and never wait on global memory.  Tiles are
// taken in segment-major ticket order, so a tile only ever waits on tiles that
// started before it.  Filter arithmetic and all carries are FP64 (v_fma_f64
// issues at the v_fma_f32 rate here); STA/LTA sums are FP32 within a block
// with FP64 carries.  No MFMA: the path is HBM-bound.
#include "internal.h"

#define FILARK_CONST __attribute__((address_space(4)))

namespace filark {

// Dynamic LDS of one workgroup with `waves` data waves:
//   block records [waves][2K][64], STA/LTA records [waves][2][64],
//   P and A^S [2][2K][2K], 8 control words.
size_t fwd_lds_bytes(int K, int waves) {
  const int NS = 2 * K;
  return (size_t)(waves * NS * kWave + waves * 2 * kWave + 2 * NS * NS) * sizeof(double) +
         8 * sizeof(uint32_t);
}

namespace {

typedef const FILARK_CONST double cdouble;

__device__ __forceinline__ cdouble *as_const(const double *p) { return (cdouble *)p; }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A copy of a uniform value that the compiler must treat as new: row offsets
// derived from it in one phase are recomputed there by scalar ALU ops instead
// of being held in SGPRs from an earlier phase.
__device__ __forceinline__ uint32_t fresh(uint32_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

// Kernel parameters are read through the kernarg-segment pointer, taken
// afresh in every phase: each phase scalar-loads only the fields it uses,
// and nothing from the parameter block stays live across other phases.
typedef const FILARK_CONST FwdParams *kparams_t;
__device__ __forceinline__ kparams_t kparams() {
  kparams_t k = (kparams_t)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(k));
  return k;
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

// out = M v + add for a block-lower-triangular M [NS][NS] (2x2 diagonal
// blocks) held in LDS; all lanes read the same entries (broadcast).  M is
// loop-invariant wherever this is called in a loop; the opaque index offset
// stops the compiler from hoisting all of M into registers, and the fences
// keep one row of M live at a time.
template <int NS>
__device__ __forceinline__ void mv_lds(const double *M, const double (&v)[NS],
                                       const double (&add)[NS], double (&out)[NS]) {
  int o = 0;
  asm volatile("" : "+s"(o));
  double r[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double s = add[i];
#pragma unroll
    for (int j = 0; j < (i / 2 + 1) * 2; ++j) s = fma(M[o + i * NS + j], v[j], s);
    r[i] = s;
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) out[i] = r[i];
}

// Decoupled look-back of the carry wave (lane = channel) over the
// predecessors of segment `seg` in one channel group.  Lane q polls the flag
// of segment seg-1-q, so one load covers a window of 64 predecessors.  The
// nearest inclusive record (or the chunk's initial state, reached past
// segment 0) at distance d closes the window once every aggregate in front
// of it is published; the prefix is then Horner's rule from the far end,
//   acc = inc(seg-1-d);  acc = W acc + agg(q) for q = seg-d .. seg-1,
// with W the transition over one segment.  Records are fetched B at a time.
// If none of the 64 nearest predecessors has an inclusive record yet, the
// poll repeats: segments 0..63 always close inside their window, and every
// tile publishes its inclusive record after its own look-back, so records
// propagate and the wait ends.  `first_poll()` runs once after the first
// poll returned; the tile's own aggregate flag is released there, so the
// drain of its record stores overlaps that round trip.  The wait is bounded
// by spin_limit polls; past it the error word is set and an invalid sum is
// returned (the kernel still terminates).
template <int R, int B, class Step, class Init, class First>
__device__ void lookback(const uint32_t *flags_g, int n_grp, const double *agg_g,
                         const double *inc_g, size_t seg_stride, int seg, uint32_t ep,
                         double (&acc)[R], Step step, Init init, First first_poll,
                         int spin_limit, uint32_t *err, int lane) {
  const uint32_t ep30 = ep & 0x3fffffffu;
  const int m = seg - 1;
  bool first = true;
  int spins = 0;
  int d;
#pragma unroll
  for (int i = 0; i < R; ++i) acc[i] = 0.0;
  while (true) {
    const int idx = m - lane;
    uint32_t f = 0;
    if (idx >= 0) f = ld_agent_u32(flags_g + (size_t)idx * n_grp);
    const bool ready = idx < 0 || (((f >> 2) == ep30) && (f & 3u) != 0);
    const bool incl = idx < 0 || (ready && (f & 3u) == kFlagInclusive);
    const uint64_t ready_m = __ballot(ready);
    const uint64_t incl_m = __ballot(incl);
    if (first) {
      first = false;
      first_poll();
    }
    if (incl_m) {
      d = __ffsll((unsigned long long)incl_m) - 1;
      const uint64_t need = d >= 63 ? ~0ull : ((2ull << d) - 1ull);
      if ((ready_m & need) == need) break;
    }
    if (++spins > spin_limit) {
      if (lane == 0) atomicOr(err, (uint32_t)kErrTimeout);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  if (m - d >= 0) {
    const double *r = inc_g + (size_t)(m - d) * seg_stride;
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = ld_agent(r + i * kWave + lane);
  } else {
    init(acc);
  }
  for (int q0 = d - 1; q0 >= 0; q0 -= B) {
    double v[B][R];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (q0 - b >= 0) {
        const double *r = agg_g + (size_t)(m - (q0 - b)) * seg_stride;
#pragma unroll
        for (int i = 0; i < R; ++i) v[b][i] = ld_agent(r + i * kWave + lane);
      }
    }
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (q0 - b >= 0) step(acc, v[b]);
  }
}

template <int R>
__device__ __forceinline__ void store_record(double *rec, const double (&v)[R], int lane) {
#pragma unroll
  for (int i = 0; i < R; ++i) st_agent(rec + i * kWave + lane, v[i]);
}

template <int R>
__device__ __forceinline__ void publish(double *rec, const double (&v)[R], uint32_t *flag,
                                        uint32_t word, int lane) {
  store_record<R>(rec, v, lane);
  vm_drain();
  if (lane == 0) st_agent_u32(flag, word);
}

// Pass 2 of one data wave: DF2T recurrence of the cascade from the exact entry
// state z over the block, y stored as produced.  Every row is computed (rows
// past the chunk end of a ragged block repeat its last sample and are not
// stored), so the recurrence has no per-row branches; the carried state of the
// chunk is produced separately by tail_state().
template <int K, int L, bool STALTA, bool WRITE_Y>
__device__ __forceinline__ void pass2(float (&xv)[L], double (&z)[2 * K], int nv,
                                      __amdgpu_buffer_rsrc_t ry, uint32_t voff, uint32_t rb,
                                      double &s_loc, double &l_loc) {
  kparams_t p = kparams();
  cdouble *coef = as_const(p->coef);
  const double asd = p->asd, ald = p->ald;
  double cb0[K], cb1[K], cb2[K], cna1[K], cna2[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    cb0[k] = coef[5 * k + 0];
    cb1[k] = coef[5 * k + 1];
    cb2[k] = coef[5 * k + 2];
    cna1[k] = coef[5 * k + 3];
    cna2[k] = coef[5 * k + 4];
  }
#pragma unroll
  for (int j = 0; j < L; ++j) {
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
      s_loc = fma(asd, s_loc, e);
      l_loc = fma(ald, l_loc, e);
    }
    if constexpr (WRITE_Y) {
      if (j < nv) buf_st(ry, voff, (uint32_t)j * rb, yf);
    }
  }
}

// Pass B of one data wave: the STA/LTA sums from their exact entry values and
// the characteristic function, stored as produced (rows < nv only).
template <int L>
__device__ __forceinline__ void passb(const float (&xv)[L], float Sf, float Lf, int nv,
                                      int jwarm, __amdgpu_buffer_rsrc_t rc, uint32_t voff,
                                      uint32_t rb) {
  kparams_t p = kparams();
  const float as = p->as, al = p->al, kappa = p->kappa;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const float e = xv[j] * xv[j];
    Sf = fmaf(as, Sf, e);
    Lf = fmaf(al, Lf, e);
    const float r = kappa * Sf * __builtin_amdgcn_rcpf(Lf);
    const float out = (Lf > 0.0f && j >= jwarm) ? r : 0.0f;
    if (j < nv) buf_st(rc, voff, (uint32_t)j * rb, out);
  }
}

// Carried state of the chunk, written by the wave that owns the chunk's last
// row: its nv rows are rerun once, in FP64, from the block's exact entry
// state (filter) and entry sums (STA/LTA), and the states after the last row
// are stored.  The filter steps are pass 2's operations in pass 2's order, so
// the carried filter state is bit-identical to pass 2's; the STA/LTA sums use
// the FP64 convention of the block sums (e from the unrounded y).
template <int K, bool STALTA>
__device__ __forceinline__ void tail_state(const float *xrow, int64_t n_ch, int nv,
                                        const double *zent, double *zout, const double *slent,
                                        double *slout, int lane_c) {
  kparams_t p = kparams();
  double z[2 * K > 0 ? 2 * K : 1];
#pragma unroll
  for (int i = 0; i < 2 * K; ++i) z[i] = zent[(size_t)i * kWave];
  double S = 0.0, Lg = 0.0;
  if constexpr (STALTA) {
    S = slent[0];
    Lg = slent[kWave];
  }
  const double asd = p->asd, ald = p->ald;
  for (int j = 0; j < nv; ++j) {
    double v = (double)xrow[(size_t)j * n_ch + lane_c];
    if constexpr (K > 0) {
      cdouble *coef = as_const(p->coef);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double yk = fma(coef[5 * k + 0], v, z[2 * k]);
        z[2 * k] = fma(coef[5 * k + 3], yk, fma(coef[5 * k + 1], v, z[2 * k + 1]));
        z[2 * k + 1] = fma(coef[5 * k + 4], yk, coef[5 * k + 2] * v);
        v = yk;
      }
    }
    if constexpr (STALTA) {
      const double e = v * v;  // as the block sums of pass 2 (unrounded y)
      S = fma(asd, S, e);
      Lg = fma(ald, Lg, e);
    }
  }
#pragma unroll
  for (int i = 0; i < 2 * K; ++i) zout[(size_t)i * n_ch] = z[i];
  if constexpr (STALTA) {
    slout[0] = S / p->nsta_d;
    slout[n_ch] = Lg / p->nlta_d;
  }
}

// Tile context shared by both roles of a workgroup.
struct Tile {
  int lane, w, NW;
  int seg, grp, n_seg, n_grp;
  uint32_t ep;               // launch epoch (look-back flags)
  uint32_t sos_ep, sl_ep;    // state-object epochs (state parities)
  uint64_t g0;               // global index of the chunk's first sample
  int64_t n_ch, c;
  bool cval, last_seg;
  size_t n_cells;
};

// Role of the carry wave: every cross-block and cross-segment step.  It runs
// the same sequence of workgroup barriers as the data waves (two for the
// filter, two for the STA/LTA), so each role is register-allocated alone.
template <int K, bool STALTA>
__device__ __forceinline__ void carry_role(const Tile &t, double *sh_blk, double *sh_sl,
                                           const double *sh_P, const double *sh_Q) {
  constexpr int NS = 2 * K;
  constexpr int NSA = NS > 0 ? NS : 1;
  constexpr int BATCH = NS >= 8 ? 1 : 2;
  const int lane = t.lane, NW = t.NW, seg = t.seg, grp = t.grp, n_grp = t.n_grp;
  const uint32_t ep = t.ep;
  const size_t n_cells = t.n_cells;
  __builtin_amdgcn_s_setprio(2);

  if constexpr (K > 0) {
    __syncthreads();  // (1) block aggregates are in LDS
    double inc[NSA];
    {
      kparams_t q = kparams();
      const size_t rstride = (size_t)n_grp * NS * kWave;
      double *agg_g = q->rec + (size_t)grp * NS * kWave;
      double *inc_g = agg_g + n_cells * NS * kWave;
      uint32_t *flag_g = q->flags + grp;
      // segment aggregate T = sum_w P^(NW-1-w) a_w (Horner), stored at once
      if (!t.last_seg) {
        double T[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) T[i] = sh_blk[i * kWave + lane];
        for (int v = 1; v < NW; ++v) {
          double av[NS];
#pragma unroll
          for (int i = 0; i < NS; ++i) av[i] = sh_blk[(v * NS + i) * kWave + lane];
          mv_lds<NS>(sh_P, T, av, T);
        }
        store_record<NS>(agg_g + (size_t)seg * rstride, T, lane);
      }
      const double *zin = q->zs + (size_t)(t.sos_ep & 1u) * NS * t.n_ch;
      const int64_t n_ch = t.n_ch, c = t.c;
      const bool cval = t.cval, last_seg = t.last_seg;
      double pre[NS];
      lookback<NS, BATCH>(
          flag_g, n_grp, agg_g, inc_g, rstride, seg, ep, pre,
          [&](double (&acc)[NS], const double (&v)[NS]) { mv_lds<NS>(sh_Q, acc, v, acc); },
          [&](double (&v)[NS]) {
#pragma unroll
            for (int i = 0; i < NS; ++i) v[i] = cval ? zin[(size_t)i * n_ch + c] : 0.0;
          },
          [&]() {
            if (!last_seg) {
              vm_drain();
              if (lane == 0) st_agent_u32(flag_g + (size_t)seg * n_grp, (ep << 2) | kFlagAggregate);
            }
          },
          q->spin_limit, q->ctrl + kCtrlError, lane);
      // entry state of every block: z_0 = prefix, z_{w+1} = P z_w + a_w; the
      // end of the chain is the segment's inclusive state
#pragma unroll
      for (int i = 0; i < NS; ++i) inc[i] = pre[i];
      for (int v = 0; v < NW; ++v) {
        double av[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          av[i] = sh_blk[(v * NS + i) * kWave + lane];
          sh_blk[(v * NS + i) * kWave + lane] = inc[i];
        }
        mv_lds<NS>(sh_P, inc, av, inc);
      }
    }
    __syncthreads();  // (2) entry states are in LDS; data waves run pass 2
    if (!t.last_seg) {
      kparams_t q = kparams();
      const size_t rstride = (size_t)n_grp * NS * kWave;
      double *inc_g = q->rec + n_cells * NS * kWave + (size_t)grp * NS * kWave;
      publish<NS>(inc_g + (size_t)seg * rstride, inc, q->flags + grp + (size_t)seg * n_grp,
                  (ep << 2) | kFlagInclusive, lane);
    }
  }

  if constexpr (STALTA) {
    __syncthreads();  // (3) STA/LTA block sums are in LDS
    const size_t rstride = (size_t)n_grp * 2 * kWave;
    double sinc[2];
    {
      kparams_t q = kparams();
      cdouble *slq = as_const(q->slq);
      const double aLs = slq[0], aLl = slq[1];
      const double aSs = slq[2 + 1], aSl = slq[2 + q->q_cap + 1];
      double *agg_g = q->rec + n_cells * 2 * NS * kWave + (size_t)grp * 2 * kWave;
      double *inc_g = agg_g + n_cells * 2 * kWave;
      uint32_t *flag_g = q->flags + n_cells + grp;
      const double *slin = q->sl + (size_t)(t.sl_ep & 1u) * 2 * t.n_ch;
      const double nsta_d = q->nsta_d, nlta_d = q->nlta_d;
      const int64_t n_ch = t.n_ch, c = t.c;
      const bool cval = t.cval, last_seg = t.last_seg;
      if (!last_seg) {
        double T[2] = {sh_sl[0 * kWave + lane], sh_sl[1 * kWave + lane]};
        for (int v = 1; v < NW; ++v) {
          T[0] = fma(aLs, T[0], sh_sl[(v * 2 + 0) * kWave + lane]);
          T[1] = fma(aLl, T[1], sh_sl[(v * 2 + 1) * kWave + lane]);
        }
        store_record<2>(agg_g + (size_t)seg * rstride, T, lane);
      }
      double pre[2];
      lookback<2, 8>(
          flag_g, n_grp, agg_g, inc_g, rstride, seg, ep, pre,
          [&](double (&acc)[2], const double (&v)[2]) {
            acc[0] = fma(aSs, acc[0], v[0]);
            acc[1] = fma(aSl, acc[1], v[1]);
          },
          [&](double (&v)[2]) {
            v[0] = cval ? slin[c] * nsta_d : 0.0;
            v[1] = cval ? slin[n_ch + c] * nlta_d : 0.0;
          },
          [&]() {
            if (!last_seg) {
              vm_drain();
              if (lane == 0) st_agent_u32(flag_g + (size_t)seg * n_grp, (ep << 2) | kFlagAggregate);
            }
          },
          q->spin_limit, q->ctrl + kCtrlError, lane);
      sinc[0] = pre[0];
      sinc[1] = pre[1];
      for (int v = 0; v < NW; ++v) {
        const double bs = sh_sl[(v * 2 + 0) * kWave + lane], bl = sh_sl[(v * 2 + 1) * kWave + lane];
        sh_sl[(v * 2 + 0) * kWave + lane] = sinc[0];
        sh_sl[(v * 2 + 1) * kWave + lane] = sinc[1];
        sinc[0] = fma(aLs, sinc[0], bs);
        sinc[1] = fma(aLl, sinc[1], bl);
      }
    }
    __syncthreads();  // (4) STA/LTA entries are in LDS; data waves run pass B
    if (!t.last_seg) {
      kparams_t q = kparams();
      double *inc_g = q->rec + n_cells * 2 * NS * kWave + n_cells * 2 * kWave + (size_t)grp * 2 * kWave;
      publish<2>(inc_g + (size_t)seg * rstride, sinc, q->flags + n_cells + grp + (size_t)seg * n_grp,
                 (ep << 2) | kFlagInclusive, lane);
    }
  }

  // the last tile to finish resets the ticket counters and advances epochs
  if (lane == 0) {
    kparams_t q = kparams();
    const uint32_t prev = atomicAdd(q->ctrl + kCtrlDone, 1u);
    if (prev == (uint32_t)n_cells - 1) {
      st_agent_u32(q->ctrl + kCtrlTicket, 0u);
      st_agent_u32(q->ctrl + kCtrlDone, 0u);
      if (K > 0) st_agent_u32(q->sos_ctrl + kCtrlEpoch, t.sos_ep + 1u);
      if (STALTA) {
        st_agent_u32(q->sl_ctrl + kCtrlEpoch, t.sl_ep + 1u);
        const uint64_t g1 = t.g0 + (uint64_t)q->n_t;
        st_agent_u32(q->sl_ctrl + kCtrlCounter, (uint32_t)g1);
        st_agent_u32(q->sl_ctrl + kCtrlCounter + 1, (uint32_t)(g1 >> 32));
      }
    }
  }
}

// Role of a data wave: its block of L rows x 64 channels, passes 1, 2 and B.
template <int K, int L, bool STALTA, bool WRITE_Y>
__device__ __forceinline__ void data_role(const Tile &t, double *sh_blk, double *sh_sl) {
  constexpr int NS = 2 * K;
  const int lane = t.lane, w = t.w;
  kparams_t p = kparams();
  const int row0 = uniform(t.seg * p->seg_len + w * L);
  const int nv = uniform(max(0, min(L, p->n_t - row0)));
  const bool last_rows = nv > 0 && row0 + nv == p->n_t;
  // Byte offsets: the lane's channel (VGPR) and each row of the block (SGPR).
  const uint32_t voff = t.cval ? (uint32_t)t.c * 4u : kOffInvalid;
  const uint32_t rowb = (uint32_t)t.n_ch * 4u;
  const size_t blk_off = (size_t)row0 * (size_t)t.n_ch;

  // ---- load: one 256 B row segment per row.  Rows past the chunk end of a
  // ragged block re-read its last row (a scalar clamp, no branch): nothing
  // computed from them is stored or published, the carried state of the chunk
  // comes from tail_state().  A wave with no rows touches no memory.
  float xv[L];
  {
    const __amdgpu_buffer_rsrc_t rx = rsrc(p->x + blk_off);
    const uint32_t rb = fresh(rowb);
    const int jmax = max(nv - 1, 0);
    const uint32_t vld = nv > 0 ? voff : kOffInvalid;
#pragma unroll
    for (int j = 0; j < L; ++j) xv[j] = buf_ld(rx, vld, (uint32_t)min(j, jmax) * rb);
  }
  double s_loc = 0.0, l_loc = 0.0;  // STA/LTA block-end sums from zero

  if constexpr (K > 0) {
    {
      // ---- pass 1: zero-state block-end projection a = sum_j A^(L-1-j) B x_j.
      // Row j+1 of G is fetched into SGPRs while row j is applied; the fences
      // stop the scheduler from hoisting the whole table into SGPRs.
      cdouble *G = as_const(kparams()->G);
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
      for (int i = 0; i < NS; ++i) sh_blk[(w * NS + i) * kWave + lane] = a[i];
    }
    __syncthreads();  // (1)
    __syncthreads();  // (2)
    double z[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) z[i] = sh_blk[(w * NS + i) * kWave + lane];
    {
      kparams_t q = kparams();
      const __amdgpu_buffer_rsrc_t ry =
          rsrc(WRITE_Y ? (const void *)(q->y + blk_off) : (const void *)q->x);
      pass2<K, L, STALTA, WRITE_Y>(xv, z, nv, ry, voff, fresh(rowb), s_loc, l_loc);
    }
  } else {
    // STA/LTA only: the input is the filtered signal
    kparams_t q = kparams();
    const double asd = q->asd, ald = q->ald;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const double xd = (double)xv[j];
      const double e = xd * xd;
      s_loc = fma(asd, s_loc, e);
      l_loc = fma(ald, l_loc, e);
    }
  }

  if constexpr (STALTA) {
    sh_sl[(w * 2 + 0) * kWave + lane] = s_loc;
    sh_sl[(w * 2 + 1) * kWave + lane] = l_loc;
    __syncthreads();  // (3)
    __syncthreads();  // (4)
    float Sf = (float)sh_sl[(w * 2 + 0) * kWave + lane];
    float Lf = (float)sh_sl[(w * 2 + 1) * kWave + lane];
    kparams_t q = kparams();
    const __amdgpu_buffer_rsrc_t rc = rsrc(q->cf + blk_off);
    // rows j < jwarm of this block precede the warm-up boundary (cf = 0)
    const int jwarm =
        uniform((int)max((int64_t)0, min((int64_t)L, q->nlta - ((int64_t)t.g0 + row0))));
    passb<L>(xv, Sf, Lf, nv, jwarm, rc, voff, fresh(rowb));
  }

  // ---- carried states after the chunk's last row (one wave per chunk)
  if (last_rows && t.cval) {
    kparams_t q = kparams();
    double *zout = K > 0 ? q->zs + (size_t)((t.sos_ep & 1u) ^ 1u) * NS * t.n_ch + t.c : nullptr;
    double *slout = STALTA ? q->sl + (size_t)((t.sl_ep & 1u) ^ 1u) * 2 * t.n_ch + t.c : nullptr;
    tail_state<K, STALTA>(q->x + blk_off, t.n_ch, nv, sh_blk + (size_t)w * NS * kWave + lane, zout,
                          sh_sl + (size_t)w * 2 * kWave + lane, slout, (int)t.c);
  }
}

// Workgroup = NW data waves + 1 carry wave.  Data wave w owns rows
// [seg*S + w*L, +L) of 64 channels; the carry wave (w == NW) owns all the
// cross-block and cross-segment arithmetic.
template <int K, int L, bool STALTA, bool WRITE_Y>
__global__ void __launch_bounds__(kMaxWaves * kWave) fwd_kernel(FwdParams) {
  constexpr int NS = 2 * K;
  extern __shared__ double lds[];
  Tile t;
  t.lane = threadIdx.x & (kWave - 1);
  t.w = uniform(threadIdx.x / kWave);
  t.NW = (int)(blockDim.x / kWave) - 1;
  const bool carry = t.w == t.NW;
  double *sh_blk = lds;                        // [NW][NS][64] block aggregates -> entry states
  double *sh_sl = sh_blk + t.NW * NS * kWave;  // [NW][2][64]  STA/LTA block sums -> entries
  double *sh_P = sh_sl + t.NW * 2 * kWave;     // [NS][NS] A^L
  double *sh_Q = sh_P + NS * NS;               // [NS][NS] A^S
  uint32_t *sh_u = reinterpret_cast<uint32_t *>(sh_Q + NS * NS);  // [6]

  kparams_t p = kparams();
  if (threadIdx.x == 0) {
    sh_u[0] = atomicAdd(p->ctrl + kCtrlTicket, 1u);
    sh_u[1] = ld_agent_u32(p->ctrl + kCtrlEpoch);
    sh_u[2] = K > 0 ? ld_agent_u32(p->sos_ctrl + kCtrlEpoch) : 0u;
    sh_u[3] = STALTA ? ld_agent_u32(p->sl_ctrl + kCtrlEpoch) : 0u;
    sh_u[4] = STALTA ? ld_agent_u32(p->sl_ctrl + kCtrlCounter) : 0u;
    sh_u[5] = STALTA ? ld_agent_u32(p->sl_ctrl + kCtrlCounter + 1) : 0u;
  }
  if constexpr (K > 0) {
    if (carry) {
      for (int i = t.lane; i < NS * NS; i += kWave) {
        sh_P[i] = p->P[i];
        sh_Q[i] = p->Q[NS * NS + i];
      }
    }
  }
  __syncthreads();
  const uint32_t ticket = (uint32_t)uniform((int)sh_u[0]);
  t.ep = (uint32_t)uniform((int)sh_u[1]);
  t.sos_ep = (uint32_t)uniform((int)sh_u[2]);
  t.sl_ep = (uint32_t)uniform((int)sh_u[3]);
  t.g0 = ((uint64_t)(uint32_t)uniform((int)sh_u[5]) << 32) | (uint64_t)(uint32_t)uniform((int)sh_u[4]);
  t.n_grp = p->n_grp;
  t.n_seg = p->n_seg;
  if (ticket >= (uint32_t)t.n_seg * (uint32_t)t.n_grp) {  // counters out of sync: never index with it
    if (threadIdx.x == 0) atomicOr(p->ctrl + kCtrlError, 2u);
    return;
  }
  t.seg = (int)(ticket / (uint32_t)t.n_grp);
  t.grp = (int)(ticket - (uint32_t)t.seg * (uint32_t)t.n_grp);
  t.n_ch = p->n_ch;
  t.c = (int64_t)t.grp * kWave + t.lane;
  t.cval = t.c < t.n_ch;
  t.last_seg = t.seg == t.n_seg - 1;
  t.n_cells = (size_t)t.n_seg * (size_t)t.n_grp;

  if (carry)
    carry_role<K, STALTA>(t, sh_blk, sh_sl, sh_P, sh_Q);
  else
    data_role<K, L, STALTA, WRITE_Y>(t, sh_blk, sh_sl);
}

template <int K, int L, bool S, bool Y>
hipError_t launch_one(const FwdParams &p, int waves, hipStream_t stream) {
  const size_t lds = fwd_lds_bytes(K, waves);
  const dim3 grid((unsigned)(p.n_seg * p.n_grp));
  const dim3 block((unsigned)((waves + 1) * kWave));
  hipLaunchKernelGGL((fwd_kernel<K, L, S, Y>), grid, block, lds, stream, p);
  return hipGetLastError();
}

template <int K, int L>
hipError_t launch_k(const FwdParams &p, bool stalta, bool write_y, int waves, hipStream_t stream) {
  if (K == 0) return launch_one<0, L, true, false>(p, waves, stream);
  if (!stalta) return launch_one<K, L, false, true>(p, waves, stream);
  if (write_y) return launch_one<K, L, true, true>(p, waves, stream);
  return launch_one<K, L, true, false>(p, waves, stream);
}

template <int L>
hipError_t launch_l(const FwdParams &p, int K, bool stalta, bool write_y, int waves,
                    hipStream_t stream) {
  switch (K) {
    case 0: return launch_k<0, L>(p, stalta, write_y, waves, stream);
    case 1: return launch_k<1, L>(p, stalta, write_y, waves, stream);
    case 2: return launch_k<2, L>(p, stalta, write_y, waves, stream);
    case 3: return launch_k<3, L>(p, stalta, write_y, waves, stream);
    case 4: return launch_k<4, L>(p, stalta, write_y, waves, stream);
    case 5: return launch_k<5, L>(p, stalta, write_y, waves, stream);
    case 6: return launch_k<6, L>(p, stalta, write_y, waves, stream);
    case 7: return launch_k<7, L>(p, stalta, write_y, waves, stream);
    case 8: return launch_k<8, L>(p, stalta, write_y, waves, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_fwd(const FwdParams &p, int K, int L, bool stalta, bool write_y, int waves,
                      hipStream_t stream) {
  if (waves < 1 || waves + 1 > kMaxWaves) return hipErrorInvalidValue;
  if (L == 32) return launch_l<32>(p, K, stalta, write_y, waves, stream);
  if (L == 64) return launch_l<64>(p, K, stalta, write_y, waves, stream);
  return hipErrorInvalidValue;
}

}  // namespace filark
