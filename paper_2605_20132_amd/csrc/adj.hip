// Adjoint kernel: gradient of a loss on the STA/LTA characteristic with
// respect to the input and the section coefficients, one window of a chunk
// per launch, windows and chunks taken last to first.
//
// The loss reaches x through cf = sta / lta, the two exponential averages of
// e = y^2, and the DF2T cascade y = H x.  Reverse mode runs the forward
// recurrences backwards in time (the time-reversed, transposed recurrence):
//   STA/LTA   with (A, B) the adjoints of (sta, lta) after sample t,
//             q = dL/dcf where cf is live (else 0),
//               Sb = A + q / lta,  Lb = B - q sta / lta^2,
//               ybar = 2 y (cs Sb + cl Lb),  A <- (1 - cs) Sb,  B <- (1 - cl) Lb;
//   filter    the delay-pair adjoints u of each section, last section first:
//               yb = ybar - a1 u1 - a2 u2,  vbar = b0 yb + b1 u1 + b2 u2,
//               u1 <- yb,  u2 <- u1,
//             vbar feeding the section before; the first section's vbar is
//             dL/dx, and the coefficient gradients gather the products of
//             these adjoints with the forward section inputs and outputs.
// Both backward recurrences are linear in their state, so a window is
// parallelised like the forward: each lane owns a block of L samples of one
// channel, runs the block backwards from a zero end state (or, for the block
// holding the window's last row, from the adjoint state handed in), the
// blocks are combined by a reverse Hillis-Steele scan through LDS with the
// transposed block transitions (A^L)^T and (1 - c)^L, and every lane reruns
// its block from the exact end state.  The forward values the backward pass
// needs (section outputs, the STA/LTA averages) are recomputed from the
// window's checkpointed start state with the forward scan of fwd.hip; the
// averages are then run forward over each block from their exact entry
// values, and every row keeps the two terms it adds to the adjoints of
// (sta, lta), so the backward passes never divide by a decay (which is 0 for
// a one-sample window).
//
// Lanes past the window's last row, or past the last channel, hold zeros and
// contribute nothing.  Coefficient gradients are summed in FP64 per lane, then
// per wave by a fixed butterfly, per workgroup in wave order, and across
// workgroups by a separate fixed-order pass: results do not depend on timing.
#include "device.h"

namespace filark {

// LDS: exchanges [nw * 64][2] and [nw * 64][2K + 1], level matrices
// [n_lev][2K][2K], carried filter state [64][2K + 1] and the per-wave
// coefficient sums [nw][5K], all FP64.
constexpr size_t adj_lds_doubles(int K, int nw, int n_lev) {
  return (size_t)nw * kWave * (2 * K + 3) + (size_t)n_lev * 4 * K * K + (size_t)kWave * (2 * K + 1) +
         (size_t)nw * 5 * K;
}

size_t adj_lds_bytes(int K, int nw, int n_lev) { return adj_lds_doubles(K, nw, n_lev) * sizeof(double); }

namespace {

using namespace dev;
typedef const FILARK_CONST AdjParams *aparams_t;
__device__ __forceinline__ aparams_t aparams() { return dev::kparams<AdjParams>(); }

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  const int lo = __builtin_amdgcn_ds_bpermute(((threadIdx.x & 63) ^ m) << 2,
                                              (int)(__builtin_bit_cast(uint64_t, v) & 0xffffffffu));
  const int hi = __builtin_amdgcn_ds_bpermute(((threadIdx.x & 63) ^ m) << 2,
                                              (int)(__builtin_bit_cast(uint64_t, v) >> 32));
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// 1 / v for v > 0: the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - v r), each of which squares the relative error (the plain
// division expands to a longer sequence of scaling, fix-up and refinement).
__device__ __forceinline__ double recip(double v) {
  double r = __builtin_amdgcn_rcp(v);
  r = fma(r, fma(-v, r, 1.0), r);
  return fma(r, fma(-v, r, 1.0), r);
}

// STA/LTA at one row, forward: the scaled sums (S, Lg) advance over e = y^2,
// and the row's contributions to the adjoints of (sta, lta) are returned:
// alpha = q / lta and beta = q cf / lta, with q = dL/dcf where cf is live
// (else 0).  gq is dL/dcf (mode 0) or the target cf (mode 1).
struct SlFwd {
  double cs, cl, asd, ald, scale;
  int64_t nlta;
  int mode;
  __device__ __forceinline__ void step(double &S, double &Lg, double yd, double gq, int64_t gidx, float &alpha,
                                       float &beta) const {
    const double e = yd * yd;
    S = fma(asd, S, e);
    Lg = fma(ald, Lg, e);
    const double sta = S * cs, lta = Lg * cl;
    const bool live = gidx >= nlta && lta > 0.0;
    const double rl = live ? recip(lta) : 0.0;
    const double cf = sta * rl;
    const double q = live ? (mode ? 2.0 * scale * (cf - gq) : gq) : 0.0;
    const double a = q * rl;
    alpha = (float)a;
    beta = (float)(a * cf);
  }
};

// STA/LTA at one row, backward: (A, B), the adjoints of (sta, lta) after the
// row, become the adjoints before it; returns dL/dy of the row.
struct SlBack {
  double cs, cl, asd, ald;
  __device__ __forceinline__ double step(double &A, double &B, double yd, float alpha, float beta) const {
    const double Sb = A + (double)alpha;
    const double Lb = B - (double)beta;
    A = asd * Sb;
    B = ald * Lb;
    return 2.0 * yd * fma(cs, Sb, cl * Lb);
  }
};

// Sum of the coefficient gradients over the lanes of a wave by recursive
// halving: at each of five exchange steps a lane gives away half of its
// (zero-padded) 32 values and adds the half its partner gives away, so a
// lane ends with one value, index lane >> 1, summed over its 32-lane half,
// and a last exchange completes the sum over all 64 lanes: 32 exchanged
// values per lane instead of 6 per coefficient.  Fixed order, so the result
// does not depend on timing.  Returns the sum of value (lane >> 1).
template <int NC>
__device__ __forceinline__ double wave_sum_halving(const double (&gc)[NC]) {
  static_assert(NC <= 32, "at most 32 values");
  const int lane = threadIdx.x & (kWave - 1);
  double v[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) v[i] = i < NC ? gc[i] : 0.0;
#pragma unroll
  for (int n = 32, m = 32; n > 1; n >>= 1, m >>= 1) {
    const bool hi = (lane & m) != 0;
#pragma unroll
    for (int i = 0; i < n / 2; ++i) {
      const double give = hi ? v[i] : v[i + n / 2];
      const double keep = hi ? v[i + n / 2] : v[i];
      v[i] = keep + shfl_xor_d(give, m);
    }
  }
  return v[0] + shfl_xor_d(v[0], 1);
}

// UNIT: every section after the first has b0 = b2 = 1 (Butterworth designs),
// so those sections skip the multiplications by them (bit-identical results).
// RECON: the section inputs and outputs of each row, which the coefficient
// gradients need in reverse time, are rebuilt backwards from the forward
// state after the block's last row and the input x (each section's state
// update inverted: y = (z2' - b2 v) / (-a2), or (z1' - b1 v) / (-a1) for a
// first-order section), in FP64, instead of being stored per row during the
// forward recompute; the host selects it when every section is invertible
// with |a2| >= 1/4 (first order: |a1| >= 1/2, b2 = 0), which bounds the
// growth of rounding over a 16-row block by 2^16.
// FULL: the window fills every block (n_t = NB L), so no row is past its
// end and the row loops run without a per-row validity branch (which costs
// the exec-mask updates and the register copies at every join).
// x rows of one window into this wave's slice of the LDS prefetch buffer
// (row j of the wave's lanes at dst[j][lane]): buffer loads with an LDS
// destination, so they need no registers and complete while the current
// window is processed.  Out-of-range lanes receive zeros.
template <int L>
__device__ __forceinline__ void xpre_issue(float (*dst)[kWave], __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t rb) {
#pragma unroll
  for (int j = 0; j < L; ++j)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void *)dst[j], 4,
                                             vo + (uint32_t)j * rb, 0, 0, 0);
}

// One window of the adjoint (wi of the launch's n_win, last to first).
// FULL: every block of the window is full (no per-row validity tests);
// with MULTI a launch's last window may be partial (n_t_last rows) and
// is taken by the FULL = false instance, the others by FULL = true.
template <int K, int L, bool UNIT, int RC, bool FULL, bool MULTI>
__device__ __forceinline__ void adj_window(int wi, int n_win, double *const lds,
                                           float (*xpre)[MULTI ? L : 1][kWave], double (*hand)[2 * K + 2],
                                           double &gacc) {
  constexpr bool RECON = RC != 0;
  constexpr int NS = 2 * K, NSP = NS + 1, NC = 5 * K;
  constexpr bool kSgprLevels = K <= 4;
  // Everything per thread is derived afresh in each window from an opaque
  // copy of the thread index, so that nothing (masks, addresses) is hoisted
  // out of the window loop and held in registers across it.
  uint32_t tid = threadIdx.x;
  if constexpr (MULTI) asm volatile("" : "+v"(tid));
  aparams_t p = aparams();
  const int lane = tid & (kWave - 1);
  const int w = uniform(tid / kWave);
  // the several-window kernel has the geometry as constants: LDS addresses
  // are then constant offsets of one array, which the compiler's alias
  // analysis follows (it stops after a few chained offsets)
  const int NW = MULTI ? kMultiWaves : p->nw;
  const int cwl = MULTI ? kMultiCwLog2 : p->cw_log2;
  const int n_lev = MULTI ? kMultiLevels : p->n_lev;
  const int CW = 1 << cwl, R = kWave >> cwl, NB = NW * R;
  const int g = group_of(p->per_xcd);
  const int r = lane >> cwl, cl = lane & (CW - 1);
  const int b = w * R + r;
  const int my = w * kWave + lane;
  const int64_t n_ch = p->n_ch;
  const int64_t c = (int64_t)g * CW + cl;
  const bool cval = c < n_ch;
  double *xsl = lds;                       // [NW * 64][2]
  double *xch = xsl + 2 * NW * kWave;      // [NW * 64][NSP]
  double *pw = xch + NW * kWave * NSP;     // [n_lev][NS][NS]
  double *zc = pw + n_lev * NS * NS;       // [CW][NSP]
  double *wsum = zc + kWave * NSP;         // [NW][NC]
  double *xme = xch + my * NSP;
  if (wi == n_win - 1) {
    const int n = n_lev * NS * NS;
    for (int k = tid; k < n; k += blockDim.x) pw[k] = p->Pw[k];
  }
  // rows of this window and its buffer range (a several-window launch's
  // partial last window: n_t_last rows)
  const int n_t = (MULTI && !FULL) ? p->n_t_last : p->n_t;
  const int range_w = (MULTI && !FULL) ? p->range_last : p->range;
  const int b_end = (n_t - 1) / L;  // block holding the window's last row
  const int64_t row0 = (int64_t)b * L;
  const int nv = (int)(row0 >= n_t ? 0 : (n_t - row0 >= L ? L : n_t - row0));
  const uint32_t rowb = (uint32_t)n_ch * 4u;
  const uint32_t vo = cval ? (uint32_t)((row0 * n_ch + c) * 4) : kOffInvalid;

  // offsets of this window's rows and start-state slot (0 for one window)
  const size_t xoff = MULTI ? (size_t)wi * (size_t)p->win_elems : 0;
  const size_t ckoff = MULTI ? (size_t)wi * (size_t)p->ck_stride : 0;
  // the adjoint state after the window (MULTI: in LDS, put there by the
  // window after it or, for the launch's last window, by the prologue)
  auto adj_in = [&](int i) -> double {
    if constexpr (MULTI)
      return hand[cl][i];
    else
      return aparams()->adj[i * n_ch + c];
  };
  if (b == 0) {
    const double *zs0 = aparams()->zs0 + ckoff;
#pragma unroll
    for (int i = 0; i < NS; ++i) zc[cl * NSP + i] = cval ? zs0[i * n_ch + c] : 0.0;
  }

  // MULTI: the STA/LTA start values are loaded before the prefetch is
  // issued (vector loads complete in order, so a wait for a later load would
  // wait for the prefetch as well)
  int64_t g0 = 0;
  double sl_s = 0.0, sl_l = 0.0;
  if constexpr (MULTI) {
    if (cval) {
      const double *sl0 = aparams()->sl0 + ckoff;
      g0 = reinterpret_cast<const int64_t *>(reinterpret_cast<const double *>(aparams()->cnt0) + ckoff)[c];
      if (b == 0) {
        sl_s = sl0[c];
        sl_l = sl0[n_ch + c];
      }
    }
  }

  float xv[L], gv[L];
  if constexpr (MULTI) {
    // this window's x is in LDS once its loads are done; the target rows
    // load into registers, and once the LDS reads are done the window
    // before starts loading into the same buffer
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const float t = xpre[w][j][lane];
      xv[j] = cval ? t : 0.0f;
    }
    const __amdgpu_buffer_rsrc_t rg = rsrc(aparams()->g + xoff, range_w);
    const uint32_t rb = fresh(rowb);
#pragma unroll
    for (int j = 0; j < L; ++j) gv[j] = buf_ld(rg, vo + (uint32_t)j * rb);
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    // issued in every window (an empty range after the first window of the
    // record reads zeros and moves nothing), so the compiler's count of the
    // loads in flight is the same on every path and waits for the target
    // rows do not wait for the prefetch
    {
      const bool more = wi > 0;
      aparams_t q = aparams();
      xpre_issue<L>(xpre[w], rsrc(more ? q->x + xoff - (size_t)q->win_elems : q->x, more ? q->range : 0), vo, rb);
    }
  } else {
    const __amdgpu_buffer_rsrc_t rx = rsrc(aparams()->x, aparams()->range);
    const __amdgpu_buffer_rsrc_t rg = rsrc(aparams()->g, aparams()->range);
    const uint32_t rb = fresh(rowb);
#pragma unroll
    for (int j = 0; j < L; ++j) {
      xv[j] = buf_ld(rx, vo + (uint32_t)j * rb);
      gv[j] = buf_ld(rg, vo + (uint32_t)j * rb);
      if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
  lds_barrier();  // level matrices and the checkpointed state are in LDS

  // ---------------- forward recompute: filter ----------------
  float yk[RECON ? 1 : K][L];     // output of section k at each row of the block (stored variant)
  float yo[RECON ? L : 1];        // the cascade output at each row (rebuilding variant)
  double zend[RECON ? NS : 1];    // forward state after the block's last row (rebuilding variant)
  double s_loc = 0.0, l_loc = 0.0;  // STA/LTA sums from zero over the block's valid rows
  {
    double a[NS];
    project<K, L>(as_const(aparams()->G), xv, a);
    if (b == 0) {
      double z0[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) z0[i] = zc[cl * NSP + i];
      mv_acc<NS>(pw, z0, a);
    }
    // level matrices scalar-loaded up to 4 sections (as in the forward kernel)
    cdouble *Pg = as_const(aparams()->Pw);
    int lev = 0;
    for (int d = 1; d < NB; d <<= 1, ++lev) {
      double mt[tri_count<NS>()];
      if constexpr (kSgprLevels) tri_load<NS>(Pg + lev * NS * NS, mt);
#pragma unroll
      for (int i = 0; i < NS; ++i) xme[i] = a[i];
      lds_barrier();
      if (b >= d) {
        const double *src = xme - d * CW * NSP;
        double t[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) t[i] = src[i];
        if constexpr (kSgprLevels)
          tri_mv_acc<NS>(mt, t, a);
        else
          mv_acc<NS>(pw + lev * NS * NS, t, a);
      }
      lds_barrier();
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) xme[i] = a[i];
    lds_barrier();
    double z[NS];
    {
      // one address from an index (a select of two pointers hides the array)
      const double *src = lds + (b == 0 ? (int)(zc - lds) + cl * NSP : (int)(xme - lds) - CW * NSP);
#pragma unroll
      for (int i = 0; i < NS; ++i) z[i] = src[i];
    }
    lds_barrier();  // the exchange is reused below
    aparams_t q = aparams();
    cdouble *coef = as_const(q->coef);
    const double asd = q->asd, ald = q->ald;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      double v = widen<1>(xv[j]);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const bool unit = UNIT && k > 0;
        const double yy = unit ? v + z[2 * k] : fma(coef[5 * k + 0], v, z[2 * k]);
        z[2 * k] = fma(coef[5 * k + 3], yy, fma(coef[5 * k + 1], v, z[2 * k + 1]));
        z[2 * k + 1] = fma(coef[5 * k + 4], yy, unit ? v : coef[5 * k + 2] * v);
        if constexpr (!RECON) yk[k][j] = (float)yy;
        v = yy;
      }
      if constexpr (RECON) yo[j] = (float)v;
      // sums from the rounded output, the value the backward pass sees
      double yd;
      if constexpr (RECON)
        yd = widen<2>(yo[j]);
      else
        yd = widen<2>(yk[K - 1][j]);
      const double e = yd * yd;
      if (FULL || j < nv) {
        s_loc = fma(asd, s_loc, e);
        l_loc = fma(ald, l_loc, e);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (RECON) {
#pragma unroll
      for (int i = 0; i < NS; ++i) zend[i] = z[i];
    }
  }

  // the cascade output of row j, as the STA/LTA sees it
  auto yout = [&](int j) -> float {
    if constexpr (RECON)
      return yo[j];
    else
      return yk[K - 1][j];
  };

  // ---------------- forward recompute: STA/LTA sums at block starts ----------------
  double Sin, Lin;  // scaled sums before the block's first row
  {
    aparams_t q = aparams();
    double S0 = 0.0, L0 = 0.0;
    if (cval) {
      if constexpr (MULTI) {
        if (b == 0) {
          S0 = sl_s / q->cs;
          L0 = sl_l / q->cl;
        }
      } else {
        const double *sl0 = q->sl0;
        g0 = q->cnt0[c];
        if (b == 0) {
          S0 = sl0[c] / q->cs;
          L0 = sl0[n_ch + c] / q->cl;
        }
      }
    }
    cdouble *dp = as_const(q->dpow);
    double s = s_loc, l = l_loc;
    if (b == 0) {
      s = fma(dp[0], S0, s);
      l = fma(dp[1], L0, l);
    }
    int lev = 0;
    for (int d = 1; d < NB; d <<= 1, ++lev) {
      xsl[2 * my] = s;
      xsl[2 * my + 1] = l;
      lds_barrier();
      if (b >= d) {
        s = fma(dp[2 * lev], xsl[2 * (my - d * CW)], s);
        l = fma(dp[2 * lev + 1], xsl[2 * (my - d * CW) + 1], l);
      }
      lds_barrier();
    }
    xsl[2 * my] = s;
    xsl[2 * my + 1] = l;
    lds_barrier();
    Sin = S0;
    Lin = L0;
    if (b > 0) {
      Sin = xsl[2 * (my - CW)];
      Lin = xsl[2 * (my - CW) + 1];
    }
    lds_barrier();
  }

  // ---------------- STA/LTA: per-row adjoint terms, forward ----------------
  // gv[j] (dL/dcf or the target) is replaced by alpha, bt[j] holds beta
  float bt[L];
  {
    aparams_t q = aparams();
    const SlFwd sf{q->cs, q->cl, q->asd, q->ald, q->scale, q->nlta, q->mode};
    double S = Sin, Lg = Lin;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      float al = 0.0f, be = 0.0f;
      if (FULL || j < nv) sf.step(S, Lg, widen<3>(yout(j)), widen<4>(gv[j]), g0 + row0 + j, al, be);
      gv[j] = al;
      bt[j] = be;
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // ---------------- adjoint: STA/LTA ----------------
  float *yb = gv;  // dL/dy of the cascade output at each row, over alpha as it is consumed
  {
    aparams_t q = aparams();
    const SlBack sb{q->cs, q->cl, q->asd, q->ald};
    double A = 0.0, B = 0.0;
    if (b == b_end && cval) {
      A = adj_in(NS);
      B = adj_in(NS + 1);
    }
    // from the block end to its start, from zero (or the handed-in state)
#pragma unroll
    for (int j = L - 1; j >= 0; --j) {
      if (FULL || j < nv) (void)sb.step(A, B, widen<5>(yout(j)), gv[j], bt[j]);
      __builtin_amdgcn_sched_barrier(0);
    }
    cdouble *dp = as_const(q->dpow);
    int lev = 0;
    for (int d = 1; d < NB; d <<= 1, ++lev) {
      xsl[2 * my] = A;
      xsl[2 * my + 1] = B;
      lds_barrier();
      if (b + d < NB) {
        A = fma(dp[2 * lev], xsl[2 * (my + d * CW)], A);
        B = fma(dp[2 * lev + 1], xsl[2 * (my + d * CW) + 1], B);
      }
      lds_barrier();
    }
    xsl[2 * my] = A;
    xsl[2 * my + 1] = B;
    lds_barrier();
    // exact adjoint after the block: the next block's start, or the
    // handed-in state for the block holding the last row
    double Ax = 0.0, Bx = 0.0;
    if (b < b_end) {
      Ax = xsl[2 * (my + CW)];
      Bx = xsl[2 * (my + CW) + 1];
    } else if (b == b_end && cval) {
      Ax = adj_in(NS);
      Bx = adj_in(NS + 1);
    }
    lds_barrier();
#pragma unroll
    for (int j = L - 1; j >= 0; --j) {
      float v = 0.0f;
      if (FULL || j < nv) v = (float)sb.step(Ax, Bx, widen<6>(yout(j)), gv[j], bt[j]);
      yb[j] = v;
      __builtin_amdgcn_sched_barrier(0);
    }
    if (b == 0 && cval) {
      // adjoint of (sta, lta) before the window; the filter part follows
      xsl[2 * my] = Ax;
      xsl[2 * my + 1] = Bx;
    }
  }

  // ---------------- adjoint: filter ----------------
  {
    aparams_t q = aparams();
    cdouble *coef = as_const(q->coef);
    double u[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) u[i] = (b == b_end && cval) ? adj_in(i) : 0.0;
    // local pass: delay-pair adjoints at the block start (the table holds
    // -a1, -a2, so ys is ybar - a1 u1 - a2 u2)
#pragma unroll
    for (int j = L - 1; j >= 0; --j) {
      if (FULL || j < nv) {
        double ybar = (double)yb[j];
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
          const double u1 = u[2 * k], u2 = u[2 * k + 1];
          const double ys = fma(coef[5 * k + 4], u2, fma(coef[5 * k + 3], u1, ybar));
          ybar = (UNIT && k > 0) ? u2 + fma(coef[5 * k + 1], u1, ys)
                                 : fma(coef[5 * k + 2], u2, fma(coef[5 * k + 1], u1, coef[5 * k + 0] * ys));
          u[2 * k] = ys;
          u[2 * k + 1] = u1;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    cdouble *Pg = as_const(aparams()->Pw);
    int lev = 0;
    for (int d = 1; d < NB; d <<= 1, ++lev) {
      double mt[tri_count<NS>()];
      if constexpr (kSgprLevels) tri_load<NS>(Pg + lev * NS * NS, mt);
#pragma unroll
      for (int i = 0; i < NS; ++i) xme[i] = u[i];
      lds_barrier();
      if (b + d < NB) {
        const double *src = xme + d * CW * NSP;
        double t[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) t[i] = src[i];
        if constexpr (kSgprLevels)
          tri_mtv_acc<NS>(mt, t, u);
        else
          mtv_acc<NS>(pw + lev * NS * NS, t, u);
      }
      lds_barrier();
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) xme[i] = u[i];
    lds_barrier();
    if (b < b_end) {
      const double *src = xme + CW * NSP;
#pragma unroll
      for (int i = 0; i < NS; ++i) u[i] = src[i];
    } else {
#pragma unroll
      for (int i = 0; i < NS; ++i) u[i] = (b == b_end && cval) ? adj_in(i) : 0.0;
    }
    lds_barrier();  // the adjoint state is overwritten below

    // rerun from the exact end state: dL/dx and the coefficient gradients
    double gc[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) gc[i] = 0.0;
    const __amdgpu_buffer_rsrc_t rgx = rsrc(q->gx + xoff, range_w);
    const uint32_t rb = fresh(rowb);
    double zr[RECON ? NS : 1];  // rebuilding variant: forward state after the current row
    if constexpr (RECON) {
#pragma unroll
      for (int i = 0; i < NS; ++i) zr[i] = zend[i];
    }
#pragma unroll
    for (int j = L - 1; j >= 0; --j) {
      double ybar = widen<7>(yb[j]);
      // section inputs and outputs of the row
      double vk[K], yk_d[K];
      if constexpr (RECON) {
        // invert the forward step of each section, first to last: from the
        // state after the row and the section's input, its output and the
        // state before the row (rows past the end, x = 0, are undone too)
        double v = widen<8>(xv[j]);
        aparams_t qr = aparams();
        cdouble *ri = as_const(qr->rinv);
        const int first_order = qr->first_order;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double z1a = zr[2 * k], z2a = zr[2 * k + 1];
          const bool unit = UNIT && k > 0;
          double y;
          if (RC == 2 && ((first_order >> k) & 1)) {  // a2 = b2 = 0: z1' = b1 v - a1 y, z2 = 0
            y = fma(-coef[5 * k + 1], v, z1a) * ri[k];
            zr[2 * k] = unit ? y - v : fma(-coef[5 * k + 0], v, y);
            zr[2 * k + 1] = 0.0;
          } else {  // z2' = b2 v - a2 y
            y = (unit ? z2a - v : fma(-coef[5 * k + 2], v, z2a)) * ri[k];
            zr[2 * k] = unit ? y - v : fma(-coef[5 * k + 0], v, y);
            zr[2 * k + 1] = fma(-coef[5 * k + 3], y, fma(-coef[5 * k + 1], v, z1a));
          }
          vk[k] = v;
          yk_d[k] = y;
          v = y;
        }
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          vk[k] = k == 0 ? widen<8>(xv[j]) : widen<9>(yk[k - 1][j]);
          yk_d[k] = widen<9>(yk[k][j]);
        }
      }
      if (j < nv) {
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
          const double vin = vk[k];
          const double yout = yk_d[k];
          const double u1 = u[2 * k], u2 = u[2 * k + 1];
          const double ys = fma(coef[5 * k + 4], u2, fma(coef[5 * k + 3], u1, ybar));
          gc[5 * k + 0] = fma(ys, vin, gc[5 * k + 0]);
          gc[5 * k + 1] = fma(u1, vin, gc[5 * k + 1]);
          gc[5 * k + 2] = fma(u2, vin, gc[5 * k + 2]);
          gc[5 * k + 3] = fma(-u1, yout, gc[5 * k + 3]);
          gc[5 * k + 4] = fma(-u2, yout, gc[5 * k + 4]);
          ybar = (UNIT && k > 0) ? u2 + fma(coef[5 * k + 1], u1, ys)
                                 : fma(coef[5 * k + 2], u2, fma(coef[5 * k + 1], u1, coef[5 * k + 0] * ys));
          u[2 * k] = ys;
          u[2 * k + 1] = u1;
        }
      }
      buf_st(rgx, vo + (uint32_t)j * rb, (float)ybar);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (b == 0 && cval) {  // the adjoint state before the window
      if (MULTI && wi > 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) hand[cl][i] = u[i];
        hand[cl][NS] = xsl[2 * my];
        hand[cl][NS + 1] = xsl[2 * my + 1];
      } else {
        double *adj = q->adj;
#pragma unroll
        for (int i = 0; i < NS; ++i) adj[i * n_ch + c] = u[i];
        adj[NS * n_ch + c] = xsl[2 * my];
        adj[(NS + 1) * n_ch + c] = xsl[2 * my + 1];
      }
    }

    // coefficient gradients: over the wave (recursive halving up to 32
    // values, else a butterfly per value), then the waves in order
    if constexpr (NC <= 32) {
      const double v = wave_sum_halving<NC>(gc);
      if ((lane & 1) == 0 && (lane >> 1) < NC) wsum[w * NC + (lane >> 1)] = v;
    } else {
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        double v = gc[i];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
        if (lane == 0) wsum[w * NC + i] = v;
      }
    }
    lds_barrier();
    if (threadIdx.x < NC) {
      double s = 0.0;
      for (int v = 0; v < NW; ++v) s += wsum[v * NC + threadIdx.x];
      if constexpr (MULTI) {
        gacc += s;
      } else {
        double *gp = aparams()->gpart + (size_t)g * NC + threadIdx.x;
        *gp += s;
      }
    }
  }
}

// RC: 0 stores the section outputs, 1 rebuilds them (every section of
// second order), 2 rebuilds them with first-order sections among them (a
// per-section test on the host's mask).
// MULTI: the launch takes p->n_win windows, last to first (all full but
// possibly the last, of n_t_last rows).  The group
// keeps its channels from window to window, so the adjoint state handed
// from a window to the one before it stays in LDS and the coefficient sums
// in a register; x of the window before is prefetched into LDS while a
// window runs.  Same arithmetic, in the same order, as one launch per window.
template <int K, int L, bool UNIT, int RC, bool FULL, bool MULTI>
__global__ void __launch_bounds__(kMaxWaves * kWave) __attribute__((amdgpu_waves_per_eu(3))) adj_kernel(AdjParams) {
  constexpr bool RECON = RC != 0;
  constexpr int NS = 2 * K, NSP = NS + 1, NC = 5 * K;
  constexpr bool kSgprLevels = K <= 4;
  // several windows per launch (MULTI): x prefetch buffer, the adjoint state
  // between windows.  That kernel's LDS is all static (fixed tile), so the
  // compiler can tell the exchanges apart from the prefetch buffer and waits
  // for the prefetch only where the buffer is read.
  extern __shared__ double lds_dyn[];
  __shared__ double lds_fix[MULTI ? adj_lds_doubles(K, kMultiWaves, kMultiLevels) : 1];
  __shared__ float xpre[MULTI ? kMultiWaves : 1][MULTI ? L : 1][kWave];
  __shared__ double hand[MULTI ? kMultiGroup : 1][NS + 2];
  double *const lds = MULTI ? lds_fix : lds_dyn;
  if (group_of(aparams()->per_xcd) >= aparams()->n_grp) return;  // whole workgroup, before any barrier
  const int n_win = MULTI ? aparams()->n_win : 1;
  double gacc = 0.0;  // MULTI: the group's coefficient sums so far (threads < 5K)
  if constexpr (MULTI) {
    aparams_t p = aparams();
    const int lane = threadIdx.x & (kWave - 1);
    const int w = uniform(threadIdx.x / kWave);
    const int cwl = kMultiCwLog2;
    const int64_t n_ch = p->n_ch;
    const int64_t c = (int64_t)group_of(p->per_xcd) * (1 << cwl) + (lane & ((1 << cwl) - 1));
    const int64_t row0 = (int64_t)(w * (kWave >> cwl) + (lane >> cwl)) * L;
    const uint32_t vo = c < n_ch ? (uint32_t)((row0 * n_ch + c) * 4) : kOffInvalid;
    if (threadIdx.x < NC) gacc = p->gpart[(size_t)group_of(p->per_xcd) * NC + threadIdx.x];
    // the adjoint state handed in after the launch's last window goes to
    // LDS with the rest: no window then waits on a global load issued after
    // its prefetch (vector loads complete in order)
    if (w == 0 && lane < (1 << cwl) && c < n_ch) {
#pragma unroll
      for (int i = 0; i < NS + 2; ++i) hand[lane][i] = p->adj[i * n_ch + c];
    }
    xpre_issue<L>(xpre[w], rsrc(p->x + (size_t)(n_win - 1) * p->win_elems, p->range_last), vo,
                  fresh((uint32_t)n_ch * 4u));
  }

  for (int wi = n_win - 1; wi >= 0; --wi) {
    if constexpr (MULTI) {
      // the launch's last window may be partial: the instance with the
      // per-row validity tests takes it
      if (wi == n_win - 1 && aparams()->n_t_last != aparams()->n_t) {
        adj_window<K, L, UNIT, RC, false, true>(wi, n_win, lds, xpre, hand, gacc);
        continue;
      }
    }
    adj_window<K, L, UNIT, RC, FULL, MULTI>(wi, n_win, lds, xpre, hand, gacc);
  }  // windows
  if constexpr (MULTI) {
    if (threadIdx.x < NC) aparams()->gpart[(size_t)group_of(aparams()->per_xcd) * NC + threadIdx.x] = gacc;
    // the last window's (empty) prefetch is complete before the workgroup's
    // LDS is released
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
  }
}

template <int K, int L, bool U, int RC>
hipError_t launch_u(const AdjParams &p, hipStream_t stream) {
  const size_t lds = adj_lds_bytes(K, p.nw, p.n_lev);
  const dim3 grid((unsigned)grid_for(p.per_xcd)), block((unsigned)(p.nw * kWave));
  const int nb = p.nw * (kWave >> p.cw_log2);
  if constexpr (L == 16 && U && RC == 1) {  // the full-window variants for the default Butterworth path
    if (p.n_t == nb * L) {
      if (p.n_win > 1) {
        if constexpr (K <= kMultiMaxSections) {
          if (!adj_multi_fits(p.nw, 1 << p.cw_log2, L, p.n_lev)) return hipErrorInvalidValue;
          hipLaunchKernelGGL((adj_kernel<K, L, U, RC, true, true>), grid, block, 0, stream, p);
        } else {
          return hipErrorInvalidValue;
        }
      } else {
        hipLaunchKernelGGL((adj_kernel<K, L, U, RC, true, false>), grid, block, lds, stream, p);
      }
      return hipGetLastError();
    }
  }
  if (p.n_win > 1) return hipErrorInvalidValue;  // several windows: the default path only
  hipLaunchKernelGGL((adj_kernel<K, L, U, RC, false, false>), grid, block, lds, stream, p);
  return hipGetLastError();
}

template <int K, int L>
hipError_t launch_one(const AdjParams &p, bool unit, hipStream_t stream) {
  if constexpr (K >= 2 && L == 16) {  // the default adjoint block only
    if (unit) {
      if (p.recon == 1) return launch_u<K, L, true, 1>(p, stream);
      return p.recon ? launch_u<K, L, true, 2>(p, stream) : launch_u<K, L, true, 0>(p, stream);
    }
  }
  if (p.recon == 1) return launch_u<K, L, false, 1>(p, stream);
  return p.recon ? launch_u<K, L, false, 2>(p, stream) : launch_u<K, L, false, 0>(p, stream);
}

template <int L>
hipError_t launch_l(const AdjParams &p, int K, bool unit, hipStream_t stream) {
  switch (K) {
    case 1: return launch_one<1, L>(p, unit, stream);
    case 2: return launch_one<2, L>(p, unit, stream);
    case 3: return launch_one<3, L>(p, unit, stream);
    case 4: return launch_one<4, L>(p, unit, stream);
    case 5: return launch_one<5, L>(p, unit, stream);
    case 6: return launch_one<6, L>(p, unit, stream);
    case 7: return launch_one<7, L>(p, unit, stream);
    case 8: return launch_one<8, L>(p, unit, stream);
    default: return hipErrorInvalidValue;
  }
}

// gsos[i] += sum over groups of gpart[g][i]; gpart is cleared.  Workgroup i
// reduces column i: thread t sums groups t, t + 256, ... in order (loads
// independent, all in flight at once), then a fixed LDS tree combines the 256
// partial sums, so the result does not depend on timing.
constexpr int kReduceThreads = 256;
__global__ void __launch_bounds__(kReduceThreads) adj_reduce_kernel(double *gpart, int n_grp, int n5, double *gsos) {
  __shared__ double part[kReduceThreads];
  const int i = (int)blockIdx.x, t = (int)threadIdx.x;
  double s = 0.0;
  for (int g = t; g < n_grp; g += kReduceThreads) s += gpart[(size_t)g * n5 + i];
  for (int g = t; g < n_grp; g += kReduceThreads) gpart[(size_t)g * n5 + i] = 0.0;
  part[t] = s;
  __syncthreads();
  for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
    if (t < h) part[t] += part[t + h];
    __syncthreads();
  }
  if (t == 0) gsos[i] += part[0];
}

}  // namespace

hipError_t launch_adj(const AdjParams &p, int K, int L, bool unit, hipStream_t stream) {
  if (p.nw < 1 || p.nw > kMaxWaves || p.n_t < 1 || p.n_lev < 1 || p.n_lev > kMaxLevels)
    return hipErrorInvalidValue;
  if (L == 8) return launch_l<8>(p, K, unit, stream);
  if (L == 16) return launch_l<16>(p, K, unit, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_adj_reduce(double *gpart, int n_grp, int n5, double *gsos, hipStream_t stream) {
  if (n5 < 1 || n5 > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(adj_reduce_kernel, dim3((unsigned)n5), dim3(kReduceThreads), 0, stream, gpart, n_grp, n5, gsos);
  return hipGetLastError();
}

}  // namespace filark
