// Forward kernel body (device templates), included by the translation units
// that instantiate it: fwd_l32.hip, fwd_l48.hip, fwd_l64.hip (one block
// length each) and fwd.hip (the batched launch).
//
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
// into blocks of L samples; the state after block b is the affine recurrence
// s(b) = P s(b-1) + a(b), P = A^L, where a(b) = sum_j A^(L-1-j) B x_j is the
// block's zero-state end state.  So:
//   pass 1   every lane projects its L samples onto a(b) (2K FMAs/sample);
//   scan     the blocks of a window are combined by a Hillis-Steele inclusive
//            scan through LDS: at distance d, s(b) += P^d s(b-d), with the
//            carried state folded into block 0 first;
//   pass 2   every lane reruns the DF2T recurrence from its exact entry state
//            and emits y; the lane owning the chunk's last sample keeps the
//            state after it, which is the carried state.
// STA/LTA repeats the three steps with scalar decays on e = y^2.
//
// Mapping (gfx950).  A workgroup owns a group of cw consecutive channels over
// the whole chunk; lane (r, cl) of wave w takes channel cl and block
// b = w * (64/cw) + r, so the carries never leave the workgroup: no
// inter-workgroup waits, and the result does not depend on timing.  A wave
// load of one row index touches 64/cw runs of cw * 4 contiguous bytes; every
// XCD takes a contiguous slab of channel groups, so the groups that share
// cache lines (and DRAM pages) meet in one L2.
// Rows past the chunk end fall outside the buffer range: loads return zero,
// stores are dropped.  Filter arithmetic and all carries are FP64 (v_fma_f64
// issues at the v_fma_f32 rate here); STA/LTA sums are FP32 within a block
// with FP64 carries.  No MFMA: the path is HBM-bound.
#pragma once

#include "device.h"
#include "trig_body.h"

namespace filark {

// The scans alternate between two exchange buffers, so a step needs one
// barrier instead of two: a wave writes the buffer of step l + 1 only after
// the barrier of step l, which every wave reaches after its reads of step
// l - 1, the last reads of that buffer.  The filter exchange is doubled for
// up to 4 sections and 4 waves (three such workgroups still fit a CU's LDS);
// the STA/LTA exchange always.
__host__ __device__ constexpr bool fwd_double_buffer(int K, int nw) { return K <= 4 && nw <= 4; }

namespace fwdk {

using namespace dev;
typedef const FILARK_CONST FwdParams *kparams_t;

// Where a workgroup's parameter block lives: the kernarg segment (one stream
// per launch) or a descriptor in device memory (batched launches).  get()
// hands out a copy the compiler must treat as new, so each phase scalar-loads
// only the fields it uses.
struct PSrc {
  kparams_t base;
  __device__ __forceinline__ kparams_t get() const {
    kparams_t k = base;
    asm volatile("" : "+s"(k));
    return k;
  }
};

// Pass 1: zero-state block-end projection (dev::project).
template <int K, int L>
__device__ __forceinline__ void pass1(PSrc ps, const float (&xv)[L], double (&a)[2 * K]) {
  project<K, L>(as_const(ps.get()->G), xv, a);
}

// Byte offsets of a lane's rows.  In time order row j of the lane's block is
// at vo + j * rb (rows past the chunk and invalid channels fall past the
// buffer range, vo >= 2^31 for the latter).  Time-reversed (REV), the
// launch's rows are taken last to first: row row0 + j is memory row
// n_t - 1 - row0 - j, valid while j <= jmax = n_t - 1 - row0; every other
// row gets the out-of-range offset 2^31 explicitly, so no offset wraps.
template <bool REV>
struct Rows {
  uint32_t vo, rb;
  int jmax;
  __device__ __forceinline__ Rows(kparams_t p, int64_t row0, int64_t c, bool cval) {
    const uint32_t rowb = (uint32_t)p->n_ch * 4u;
    rb = fresh(rowb);
    if constexpr (REV) {
      const int64_t last = (int64_t)p->n_t - 1 - row0;  // memory row of j = 0
      jmax = cval ? (int)(last < -1 ? -1 : last) : -1;
      vo = jmax >= 0 ? (uint32_t)((last * p->n_ch + c) * 4) : kOffInvalid;
    } else {
      jmax = 0;
      vo = cval ? (uint32_t)((row0 * p->n_ch + c) * 4) : kOffInvalid;
    }
  }
  __device__ __forceinline__ uint32_t off(int j) const {
    if constexpr (REV)
      return j <= jmax ? vo - (uint32_t)j * rb : kOffInvalid;
    else
      return vo + (uint32_t)j * rb;
  }
};

// Pass 2: DF2T recurrence of the cascade from the exact entry state z over
// the block; y replaces x in xv and is stored as produced.  With STALTA the
// block's STA/LTA sums from zero are accumulated from the unrounded y.  After
// row jcap (wave-uniform; -1 for none) the filter state is written to LDS at
// `keep` and the sums so far are kept: in the block that holds the last row
// of the launch, that is the carried state.
template <int K, int L, bool STALTA, bool WRITE_Y, bool UNIT, bool REV, bool NT>
__device__ __forceinline__ void pass2(PSrc ps, float (&xv)[L], double (&z)[2 * K], __amdgpu_buffer_rsrc_t ry,
                                      const Rows<REV> &rw, double &s_loc, double &l_loc,
                                      int jcap, double *keep, double &sc, double &lc) {
  kparams_t p = ps.get();
  const RowBuf ryb{(const char *)(WRITE_Y ? (const void *)p->y : (const void *)p->x),
                   (uint32_t)(WRITE_Y ? p->out_range : 0), fresh((uint32_t)p->n_ch * 4u)};
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
    double v = widen<1>(xv[j]);  // not pass 1's conversion, held until now
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (UNIT && k > 0) {  // b0 = b2 = 1: the same values, one operation fewer
        const double yk = v + z[2 * k];
        z[2 * k] = fma(cna1[k], yk, fma(cb1[k], v, z[2 * k + 1]));
        z[2 * k + 1] = fma(cna2[k], yk, v);
        v = yk;
      } else {
        const double yk = fma(cb0[k], v, z[2 * k]);
        z[2 * k] = fma(cna1[k], yk, fma(cb1[k], v, z[2 * k + 1]));
        z[2 * k + 1] = fma(cna2[k], yk, cb2[k] * v);
        v = yk;
      }
    }
    const float yf = (float)v;
    xv[j] = yf;
    if constexpr (STALTA) {
      const double e = v * v;
      s_loc = fma(asd, s_loc, e);
      l_loc = fma(ald, l_loc, e);
    }
    if constexpr (WRITE_Y) {
      if constexpr (REV)
        buf_st<NT>(ry, rw.off(j), yf);
      else
        buf_st<NT>(ryb.at(j), rw.vo, yf);
    }
    if (j == jcap) {  // a scalar branch: the side effect keeps it from being if-converted
      asm volatile("");
#pragma unroll
      for (int i = 0; i < 2 * K; ++i) keep[i] = z[i];
      sc = s_loc;
      lc = l_loc;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// STA/LTA sums of a block of an already filtered input, from zero.
template <int L>
__device__ __forceinline__ void sums(PSrc ps, const float (&xv)[L], double &s_loc, double &l_loc, int jcap,
                                     double &sc, double &lc) {
  kparams_t p = ps.get();
  const double asd = p->asd, ald = p->ald;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const double xd = (double)xv[j];
    const double e = xd * xd;
    s_loc = fma(asd, s_loc, e);
    l_loc = fma(ald, l_loc, e);
    if (j == jcap) {
      asm volatile("");
      sc = s_loc;
      lc = l_loc;
    }
  }
}

// Pass B: the STA/LTA sums from their exact entry values and the
// characteristic function, stored as produced (not stored without a cf
// buffer).  Rows before the warm-up boundary (block row < jwarm) give zero.
// KEEP: cf replaces y in xv (for the trigger of the monitor launch).
template <int L, bool WARM, bool NT, bool KEEP = false>
__device__ __forceinline__ void passb(PSrc ps, float (&xv)[L], float Sf, float Lf, int jwarm,
                                      const Rows<false> &rw) {
  kparams_t p = ps.get();
  const float as = p->as, al = p->al, kappa = p->kappa;
  const RowBuf rcb{(const char *)(p->cf ? (const void *)p->cf : (const void *)p->x),
                   p->cf ? (uint32_t)p->out_range : 0u, fresh((uint32_t)p->n_ch * 4u)};
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const float e = xv[j] * xv[j];
    Sf = fmaf(as, Sf, e);
    Lf = fmaf(al, Lf, e);
    const float r = kappa * Sf * __builtin_amdgcn_rcpf(Lf);
    const float out = (Lf > 0.0f && (!WARM || j >= jwarm)) ? r : 0.0f;
    buf_st<NT>(rcb.at(j), rw.vo, out);
    if constexpr (KEEP) xv[j] = out;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// LDS regions of a forward workgroup (see fwd_lds_bytes).
struct FwdLds {
  // exchange k of a scan: xsl + k * sl_step, xch + k * ch_step (k = 0, 1)
  double *xsl, *xch, *pw, *zc, *slc;
  int sl_step, ch_step;
  __device__ __forceinline__ FwdLds(kparams_t p, int NS) {
    extern __shared__ double lds[];
    const int NSP = NS + 1, n = p->nw * kWave;
    xsl = lds;                        // [2][n][2]
    sl_step = 2 * n;
    xch = lds + 4 * n;                // [1 or 2][n][NSP]
    ch_step = fwd_double_buffer(NS / 2, p->nw) ? n * NSP : 0;
    pw = xch + ch_step + n * NSP;     // [n_lev][NS][NS]
    zc = pw + p->n_lev * NS * NS;     // [CW][NSP]
    slc = zc + (NSP << p->cw_log2);   // [CW][2]
  }
};

// The carried state of channel group g, read by the lanes of block 0 before
// any signal load is issued: a later wait for it then never waits for the
// signal loads or for stores (the vector-memory counter is in order).
template <int K, bool STALTA>
struct Staged {
  double z[2 * K > 0 ? 2 * K : 1];
  double s, l;
  __device__ __forceinline__ void read(PSrc ps, int g) {
    kparams_t p = ps.get();
    const int lane = threadIdx.x & (kWave - 1);
    const int cwl = p->cw_log2, CW = 1 << cwl;
    const int b = uniform(threadIdx.x / kWave) * (kWave >> cwl) + (lane >> cwl);
    const int64_t n_ch = p->n_ch;
    const int64_t c = (int64_t)g * CW + (lane & (CW - 1));
    const bool on = b == 0 && c < n_ch;
#pragma unroll
    for (int i = 0; i < 2 * K; ++i) z[i] = on ? p->zs[i * n_ch + c] : 0.0;
    s = 0.0;
    l = 0.0;
    if constexpr (STALTA) {
      if (on) {
        s = p->sl[c] * p->nsta_d;
        l = p->sl[n_ch + c] * p->nlta_d;
      }
    }
  }
  // into LDS (after the signal loads have been issued)
  __device__ __forceinline__ void write(PSrc ps, const FwdLds &m) const {
    kparams_t p = ps.get();
    const int lane = threadIdx.x & (kWave - 1);
    const int cwl = p->cw_log2, CW = 1 << cwl;
    const int b = uniform(threadIdx.x / kWave) * (kWave >> cwl) + (lane >> cwl);
    const int cl = lane & (CW - 1);
    constexpr int NSP = 2 * K + 1;
    if (b == 0) {
#pragma unroll
      for (int i = 0; i < 2 * K; ++i) m.zc[cl * NSP + i] = z[i];
      if constexpr (STALTA) {
        m.slc[cl * 2 + 0] = s;
        m.slc[cl * 2 + 1] = l;
      }
    }
  }
};

// Level matrices into LDS.  Up to kCap values per thread are read into
// registers before the signal loads are issued and written to LDS after, so
// no wait for these reads holds back the signal loads; any remainder (many
// levels on a narrow workgroup) is copied afterwards.
template <int K>
struct Levels {
  static constexpr int NS = 2 * K, kCap = 4;
  double v[kCap];
  __device__ __forceinline__ void read(PSrc ps) {
    if constexpr (K > 0) {
      kparams_t p = ps.get();
      const int n = p->n_lev * NS * NS;
#pragma unroll
      for (int i = 0; i < kCap; ++i) {
        const int k = (int)threadIdx.x + i * (int)blockDim.x;
        v[i] = k < n ? p->Pw[k] : 0.0;
      }
    }
  }
  __device__ __forceinline__ void write(PSrc ps, const FwdLds &m) const {
    if constexpr (K > 0) {
      kparams_t p = ps.get();
      const int n = p->n_lev * NS * NS;
#pragma unroll
      for (int i = 0; i < kCap; ++i) {
        const int k = (int)threadIdx.x + i * (int)blockDim.x;
        if (k < n) m.pw[k] = v[i];
      }
      for (int k = (int)threadIdx.x + kCap * (int)blockDim.x; k < n; k += (int)blockDim.x) m.pw[k] = p->Pw[k];
    }
  }
};

// Loads of channel group g's window into xv (issued, not waited for); with
// NT (groups of 16 channels or more, 64-byte row pieces) they carry the
// non-temporal hint, as the stores do: the signal is read once.
template <int L, bool REV, bool NT>
__device__ __forceinline__ void fwd_load(PSrc ps, int g, float (&xv)[L]) {
  kparams_t p = ps.get();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x / kWave);
  const int cwl = p->cw_log2;
  const int CW = 1 << cwl, R = kWave >> cwl;
  const int r = lane >> cwl, cl = lane & (CW - 1);
  const int b = w * R + r;
  const int64_t n_ch = p->n_ch;
  const int64_t c = (int64_t)g * CW + cl;
  const bool cval = c < n_ch;
  const int64_t row0 = (int64_t)b * L;
  const Rows<REV> rw(p, row0, c, cval);
  if constexpr (REV) {
    const __amdgpu_buffer_rsrc_t rx = rsrc(ps.get()->x, ps.get()->range);
#pragma unroll
    for (int j = 0; j < L; ++j) {
      xv[j] = buf_ld<NT>(rx, rw.off(j));
      if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    kparams_t q = ps.get();
    const RowBuf rb{(const char *)q->x, (uint32_t)q->range, fresh((uint32_t)q->n_ch * 4u)};
#pragma unroll
    for (int j = 0; j < L; ++j) {
      xv[j] = buf_ld<NT>(rb.at(j), rw.vo);
      if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Everything after the loads for channel group g of the stream described by
// ps, over one window of rows: carries, passes, stores, carried state.
// TRIG (monitor launch; ps points at a MonParams): the two-threshold trigger
// then runs on the window's cf, kept in registers.
template <int K, int L, bool STALTA, bool WRITE_Y, bool UNIT, bool REV, bool NT, bool TRIG = false>
__device__ __forceinline__ void fwd_compute(PSrc ps, int g, float (&xv)[L]) {
  constexpr int NS = 2 * K;
  extern __shared__ double lds[];
  kparams_t p = ps.get();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x / kWave);
  const int NW = p->nw;
  const int cwl = p->cw_log2;
  const int CW = 1 << cwl, R = kWave >> cwl, NB = NW * R;
  const int r = lane >> cwl, cl = lane & (CW - 1);
  const int b = w * R + r;                 // block within the window
  const int my = w * kWave + lane;         // = b * CW + cl, the lane's LDS row
  constexpr int NSP = NS + 1;              // LDS row pitch of a filter state
  const int64_t n_ch = p->n_ch;
  const int64_t c = (int64_t)g * CW + cl;
  const bool cval = c < n_ch;
  const FwdLds m(p, NS);

  double *pw = m.pw;                       // [n_lev][NS][NS]
  double *zc = m.zc;                       // [CW][NSP] carried state at the window start
  const double *slc = m.slc;               // [CW][2] carried STA/LTA sums
  double *xme = m.xch + my * NSP;          // this lane's row of exchange 0

  // the window's last row: block, wave and row within the block
  const int n_t = p->n_t;
  const int b_end = (n_t - 1) / L;
  const int w_end = b_end / R, r_end = b_end - w_end * R;
  const int jend = (n_t - 1) - b_end * L;
  const int jcap = uniform(w == w_end ? jend : -1);
  const bool end_lane = w == w_end && r == r_end && cval;
  const int64_t row0 = (int64_t)b * L;

  double s_loc = 0.0, l_loc = 0.0, sc = 0.0, lc = 0.0;
  lds_barrier();  // level matrices and the staged carried state are in LDS

  if constexpr (K > 0) {
    double a[NS];
    pass1<K, L>(ps, xv, a);
    if (b == 0) {  // fold in the carried state: a += P z0
      double z0[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) z0[i] = zc[cl * NSP + i];
      mv_acc<NS>(pw, z0, a);
    }
    // up to 4 sections the level matrix of each step is scalar-loaded (its
    // 2K(K+1) entries fit the SGPRs), issued before the exchange so the
    // fetch overlaps the barrier; larger cascades read it from LDS
    constexpr bool kSgprLevels = K <= 4;
    cdouble *Pg = as_const(ps.get()->Pw);
    int lev = 0;
    for (int d = 1; d < NB; d <<= 1, ++lev) {
      double mt[tri_count<NS>()];
      if constexpr (kSgprLevels) tri_load<NS>(Pg + lev * NS * NS, mt);
      double *xl = m.xch + (lev & 1) * m.ch_step + my * NSP;
#pragma unroll
      for (int i = 0; i < NS; ++i) xl[i] = a[i];
      lds_barrier();
      if (b >= d) {
        const double *src = xl - d * CW * NSP;
        double t[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) t[i] = src[i];
        if constexpr (kSgprLevels)
          tri_mv_acc<NS>(mt, t, a);
        else
          mv_acc<NS>(pw + lev * NS * NS, t, a);
      }
      if (m.ch_step == 0) lds_barrier();  // one exchange buffer: wait for the reads
    }
    // the block totals, in the buffer the last step did not read
    double *xf = m.xch + (lev & 1) * m.ch_step + my * NSP;
#pragma unroll
    for (int i = 0; i < NS; ++i) xf[i] = a[i];
    lds_barrier();
    // entry state of the block: the state after block b - 1
    double z[NS];
    {
      const double *src = b == 0 ? zc + cl * NSP : xf - CW * NSP;
#pragma unroll
      for (int i = 0; i < NS; ++i) z[i] = src[i];
    }
    lds_barrier();  // the capture below reuses the exchange
    {
      // checkpoints of the filter state at every ck_blocks-th block start
      // (the adjoint's window starts)
      kparams_t q = ps.get();
      const int ckb = q->ck_blocks;
      if (ckb > 0 && (b > 0 || q->ck_first) && b % ckb == 0 && (int64_t)b * L < (int64_t)q->n_t && cval) {
        double *ck = q->ck + (int64_t)(b / ckb) * q->ck_stride;
#pragma unroll
        for (int i = 0; i < NS; ++i) ck[i * n_ch + c] = z[i];
      }
    }
    {
      kparams_t q = ps.get();
      const __amdgpu_buffer_rsrc_t ry =
          rsrc(WRITE_Y ? (const void *)q->y : (const void *)q->x, WRITE_Y ? q->out_range : 0);
      const Rows<REV> rw(ps.get(), row0, c, cval);
      pass2<K, L, STALTA, WRITE_Y, UNIT, REV, NT>(ps, xv, z, ry, rw, s_loc, l_loc, jcap, xme, sc, lc);
    }
    if (end_lane) {  // the filter state after the last row, kept by pass 2
      double *zs = ps.get()->zs;
#pragma unroll
      for (int i = 0; i < NS; ++i) zs[i * n_ch + c] = xme[i];
    }
  } else {
    sums<L>(ps, xv, s_loc, l_loc, jcap, sc, lc);
  }

  if constexpr (STALTA) {
    // the sample counter is equal for all channels: one scalar load
    const int64_t g0 = ((const FILARK_CONST int64_t *)ps.get()->cnt)[(int64_t)g * CW];
    double S0 = 0.0, L0 = 0.0;
    if (b == 0) {
      S0 = slc[cl * 2 + 0];
      L0 = slc[cl * 2 + 1];
    }
    int lev = 0;
    {
      cdouble *dp = as_const(ps.get()->dpow);
      if (b == 0) {
        s_loc = fma(dp[0], S0, s_loc);
        l_loc = fma(dp[1], L0, l_loc);
      }
      for (int d = 1; d < NB; d <<= 1, ++lev) {
        double *xs = m.xsl + (lev & 1) * m.sl_step;
        xs[2 * my] = s_loc;
        xs[2 * my + 1] = l_loc;
        lds_barrier();
        if (b >= d) {
          const double ts = xs[2 * (my - d * CW)], tl = xs[2 * (my - d * CW) + 1];
          s_loc = fma(dp[2 * lev], ts, s_loc);
          l_loc = fma(dp[2 * lev + 1], tl, l_loc);
        }
      }
    }
    double *xs = m.xsl + (lev & 1) * m.sl_step;
    xs[2 * my] = s_loc;
    xs[2 * my + 1] = l_loc;
    lds_barrier();
    double Sin = S0, Lin = L0;
    if (b > 0) {
      Sin = xs[2 * (my - CW)];
      Lin = xs[2 * (my - CW) + 1];
    }
    kparams_t q = ps.get();
    {  // checkpoints of the STA/LTA state and the sample counter (as the filter's above)
      const int ckb = q->ck_blocks;
      if (ckb > 0 && (b > 0 || q->ck_first) && b % ckb == 0 && (int64_t)b * L < (int64_t)q->n_t && cval) {
        double *ck = q->ck + (int64_t)(b / ckb) * q->ck_stride + (int64_t)NS * n_ch;
        ck[c] = Sin / q->nsta_d;
        ck[n_ch + c] = Lin / q->nlta_d;
        reinterpret_cast<int64_t *>(ck + 2 * n_ch)[c] = g0 + row0;
      }
    }
    if (end_lane) {
      // sums after the last row, from the block entry and the partial block
      // sums kept at that row
      cdouble *rp = as_const(q->dpow) + 2 * (q->n_lev + jend + 1);
      const double Se = fma(rp[0], Sin, sc), Le = fma(rp[1], Lin, lc);
      q->sl[c] = Se / q->nsta_d;
      q->sl[n_ch + c] = Le / q->nlta_d;
      q->cnt[c] = g0 + n_t;
    }
    const int64_t jw = q->nlta - (g0 + row0);
    const int jwarm = jw <= 0 ? 0 : (jw >= L ? L : (int)jw);
    if (q->out_range == 0) return;  // states only: no characteristic to write
    // past the warm-up for every row of the wave (a wave-uniform test): no
    // per-row comparison with the warm-up boundary
    if (g0 + (int64_t)w * R * L >= q->nlta)
      passb<L, false, NT, TRIG>(ps, xv, (float)Sin, (float)Lin, 0, Rows<false>(q, row0, c, cval));
    else
      passb<L, true, NT, TRIG>(ps, xv, (float)Sin, (float)Lin, jwarm, Rows<false>(q, row0, c, cval));
    if constexpr (TRIG)
      trigk::trig_window<L>(&reinterpret_cast<const FILARK_CONST MonParams *>(ps.get())->t, g, xv);
  }
}

// Touch every 64-byte line of G with scalar loads (16 lines per wait) while
// the signal loads are in flight, so pass 1's batched row fetches hit the
// scalar cache instead of all waves of a CU missing on the same lines at once.
template <int K, int L>
__device__ __forceinline__ void warm_g(PSrc ps) {
  if constexpr (K > 0) {
    const FILARK_CONST uint32_t *Gw = (const FILARK_CONST uint32_t *)ps.get()->G;
    constexpr int kLines = (L * 2 * K * 8 + 63) / 64, kBatch = 16;
#pragma unroll
    for (int b0 = 0; b0 < kLines; b0 += kBatch) {
      uint32_t acc = 0;
#pragma unroll
      for (int i = b0; i < b0 + kBatch && i < kLines; ++i) acc |= Gw[i * 16];
      asm volatile("" ::"s"(acc));
    }
  }
}

template <int K, int L, bool STALTA, bool WRITE_Y, bool UNIT, bool REV, bool NT, bool TRIG = false>
__device__ __forceinline__ void fwd_body(PSrc ps, int g) {
  const FwdLds m(ps.get(), 2 * K);
  Staged<K, STALTA> sa;
  Levels<K> tb;
  sa.read(ps, g);
  tb.read(ps);
  float xv[L];
  fwd_load<L, REV, NT>(ps, g, xv);
  warm_g<K, L>(ps);
  sa.write(ps, m);
  tb.write(ps, m);
  fwd_compute<K, L, STALTA, WRITE_Y, UNIT, REV, NT, TRIG>(ps, g, xv);
}

// One channel group per workgroup.  At least three waves per SIMD for 48-
// and 64-sample blocks (at most 168 VGPRs), four (128) for 48-sample blocks
// of up to 4 sections, so that every workgroup of a 6000-channel chunk is
// resident at once with the default 8-wave workgroups.
template <int K, int L, bool STALTA, bool WRITE_Y, bool UNIT, bool REV, bool NT>
__global__ void __launch_bounds__(kMaxWaves * kWave)
__attribute__((amdgpu_waves_per_eu(L == 48 && K <= 4 ? 4 : (L >= 48 ? 3 : 1)))) fwd_kernel(FwdParams) {
  const PSrc ps{dev::kparams<FwdParams>()};
  const int g = group_of(ps.get()->per_xcd, ps.get()->order);
  if (g >= ps.get()->n_grp) return;  // whole workgroup, before any barrier
  fwd_body<K, L, STALTA, WRITE_Y, UNIT, REV, NT>(ps, g);
}

template <int K, int L, bool S, bool Y, bool U, bool V>
hipError_t launch_one(const FwdParams &p, hipStream_t stream) {
  const size_t lds = fwd_lds_bytes(K, p.nw, p.n_lev, 1 << p.cw_log2);
  const dim3 grid((unsigned)fwd_grid(p));
  const dim3 block((unsigned)(p.nw * kWave));
  if (p.nt)
    hipLaunchKernelGGL((fwd_kernel<K, L, S, Y, U, V, true>), grid, block, lds, stream, p);
  else
    hipLaunchKernelGGL((fwd_kernel<K, L, S, Y, U, V, false>), grid, block, lds, stream, p);
  return hipGetLastError();
}

template <int K, int L>
hipError_t launch_k(const FwdParams &p, bool stalta, bool write_y, bool unit, bool rev, hipStream_t stream) {
  if (K == 0) return rev ? hipErrorInvalidValue : launch_one<0, L, true, false, false, false>(p, stream);
  if constexpr (K >= 1 && L == 48) {
    if (rev) {  // time-reversed: SOS only, 48-row blocks (the zero-phase filter's backward pass)
      if (stalta || !write_y) return hipErrorInvalidValue;
      if constexpr (K >= 2) {
        if (unit) return launch_one<K, L, false, true, true, true>(p, stream);
      }
      return launch_one<K, L, false, true, false, true>(p, stream);
    }
  }
  if (rev) return hipErrorInvalidValue;
  // cascades whose later sections have b0 = b2 = 1 (every Butterworth design
  // here) get the shorter section step; no such variant for 32-sample blocks
  if constexpr (K >= 2 && L != 32) {
    if (unit) {
      if (!stalta) return launch_one<K, L, false, true, true, false>(p, stream);
      if (write_y) return launch_one<K, L, true, true, true, false>(p, stream);
      return launch_one<K, L, true, false, true, false>(p, stream);
    }
  }
  if (!stalta) return launch_one<K, L, false, true, false, false>(p, stream);
  if (write_y) return launch_one<K, L, true, true, false, false>(p, stream);
  return launch_one<K, L, true, false, false, false>(p, stream);
}

// Launch of one window with L-row blocks (instantiated per L in its own
// translation unit, so the kernels build in parallel).
template <int L>
hipError_t launch_l(const FwdParams &p, int K, bool stalta, bool write_y, bool unit, bool rev,
                    hipStream_t stream) {
  switch (K) {
    case 0: return launch_k<0, L>(p, stalta, write_y, unit, rev, stream);
    case 1: return launch_k<1, L>(p, stalta, write_y, unit, rev, stream);
    case 2: return launch_k<2, L>(p, stalta, write_y, unit, rev, stream);
    case 3: return launch_k<3, L>(p, stalta, write_y, unit, rev, stream);
    case 4: return launch_k<4, L>(p, stalta, write_y, unit, rev, stream);
    case 5: return launch_k<5, L>(p, stalta, write_y, unit, rev, stream);
    case 6: return launch_k<6, L>(p, stalta, write_y, unit, rev, stream);
    case 7: return launch_k<7, L>(p, stalta, write_y, unit, rev, stream);
    case 8: return launch_k<8, L>(p, stalta, write_y, unit, rev, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fwdk

}  // namespace filark
