/*
 * FP64 CPU oracle for the stateful chunked SOS + STA/LTA path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header, table or helper with the HIP
 * library; its own design, filter, STA/LTA and gradient routines are written
 * out from their textbook definitions, one plain loop at a time.
 *
 * What it computes (the paper, Section 3.4 "Signal processing, pipelines,
 * and algorithm integration", and its performance Section 6.2):
 *   - stateful-compatible causal IIR filtering in second-order sections: a
 *     chunk goes in, an output of the same length comes out and the filter
 *     state is carried to the next call, so that a chunked run equals a
 *     one-shot run (Section 3.4; Table 1 "IIR ... SOS" row);
 *   - bandpass / lowpass / highpass wrappers (Section 3.4), designed here as
 *     Butterworth filters by the bilinear transform with pre-warping;
 *   - a threshold energy-detector characteristic (Section 3.4, monitors),
 *     taken as the recursive STA/LTA ratio on the squared filter output;
 *   - the operators beside it in Table 1, each stateful across chunks:
 *     the on/off trigger on that characteristic, zero-phase (forward-
 *     backward) filtering of a window, running-mean removal and running AGC,
 *     and the realtime FIR with carried history.
 * The paper gives no formula for any of these; the readings are the textbook
 * ones (Oppenheim & Schafer for the bilinear Butterworth design and the
 * direct-form-II-transposed section; the exponential recursive STA/LTA) and
 * are listed, with every other reading, in the design notes.
 *
 * Layout: records are time-major x[t * n_ch + c] (channel contiguous), the
 * paper's 'nt_nc' tape convention (Section 3.5).  Arithmetic is IEEE double,
 * built without fast-math and without FMA contraction.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_EUNSTABLE 5

enum { ORC_LOWPASS = 0, ORC_HIGHPASS = 1, ORC_BANDPASS = 2, ORC_BANDSTOP = 3 };

typedef double complex cplx;

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Butterworth design by the bilinear transform (textbook; paper silent).
 *   1. analog prototype poles p_k = exp(j pi (2k + N + 1) / (2N)), gain 1;
 *   2. pre-warp each band edge: W = 2 fs tan(pi f / fs);
 *   3. frequency transform (LP, HP, BP, BS);
 *   4. bilinear map z = (2 fs + s) / (2 fs - s), missing zeros go to z = -1;
 *   5. pair poles and zeros into sections.
 * ---------------------------------------------------------------------- */

static cplx prod_minus(const cplx *r, int n) {  /* prod(-r_i) */
  cplx a = 1.0;
  for (int i = 0; i < n; ++i) a *= -r[i];
  return a;
}

/* Analog zeros/poles/gain of the transformed prototype. Arrays hold up to 2N. */
static int analog_zpk(int N, int btype, double w1, double w2,
                      cplx *z, int *nz, cplx *p, int *np, double *k) {
  cplx proto[256];
  for (int i = 0; i < N; ++i) proto[i] = cexp(I * M_PI * (2.0 * i + N + 1.0) / (2.0 * N));
  *nz = 0;
  *np = 0;
  if (btype == ORC_LOWPASS) {
    for (int i = 0; i < N; ++i) p[(*np)++] = w1 * proto[i];
    *k = pow(w1, N);
  } else if (btype == ORC_HIGHPASS) {
    for (int i = 0; i < N; ++i) p[(*np)++] = w1 / proto[i];
    for (int i = 0; i < N; ++i) z[(*nz)++] = 0.0;
    *k = creal(1.0 / prod_minus(proto, N));
  } else if (btype == ORC_BANDPASS) {
    double w0sq = w1 * w2, bw = w2 - w1;
    for (int i = 0; i < N; ++i) {
      cplx a = proto[i] * bw / 2.0;
      cplx r = csqrt(a * a - w0sq);
      p[(*np)++] = a + r;
      p[(*np)++] = a - r;
    }
    for (int i = 0; i < N; ++i) z[(*nz)++] = 0.0;
    *k = pow(bw, N);
  } else if (btype == ORC_BANDSTOP) {
    double w0sq = w1 * w2, bw = w2 - w1, w0 = sqrt(w0sq);
    for (int i = 0; i < N; ++i) {
      cplx a = (bw / 2.0) / proto[i];
      cplx r = csqrt(a * a - w0sq);
      p[(*np)++] = a + r;
      p[(*np)++] = a - r;
    }
    for (int i = 0; i < N; ++i) {
      z[(*nz)++] = I * w0;
      z[(*nz)++] = -I * w0;
    }
    /* H(s) = 1/prod(s' - p) with s' = B s / (s^2 + W0^2) gives gain 1/prod(-p) */
    *k = creal(1.0 / prod_minus(proto, N));
  } else {
    return ORC_EINVAL;
  }
  return ORC_OK;
}

static int is_real(cplx v) { return fabs(cimag(v)) <= 1e-10 * (1.0 + cabs(v)); }

/* Pair poles/zeros into sections (reading R7): the pole closest to the unit
 * circle goes into the LAST remaining section, with its conjugate (or, for a
 * real pole, the next real pole closest to the circle), and with the zeros
 * nearest to it; sections therefore run from the best-damped to the
 * least-damped pole pair.  The overall gain multiplies section 1's
 * numerator. */
static int zpk_to_sos(const cplx *z, int nz, const cplx *p, int np, double k,
                      double *sos, int *n_sec_out) {
  int n_sec = (np + 1) / 2;
  int used_p[512], used_z[512];
  memset(used_p, 0, sizeof used_p);
  memset(used_z, 0, sizeof used_z);
  for (int s = n_sec - 1; s >= 0; --s) {
    int i1 = -1;
    for (int i = 0; i < np; ++i) {
      if (used_p[i]) continue;
      if (i1 < 0 || cabs(p[i]) > cabs(p[i1]) ||
          (cabs(p[i]) == cabs(p[i1]) && cimag(p[i]) > cimag(p[i1])))
        i1 = i;
    }
    used_p[i1] = 1;
    int i2 = -1;
    if (!is_real(p[i1])) {
      for (int i = 0; i < np; ++i) {
        if (used_p[i]) continue;
        if (i2 < 0 || cabs(p[i] - conj(p[i1])) < cabs(p[i2] - conj(p[i1]))) i2 = i;
      }
    } else {
      for (int i = 0; i < np; ++i) {
        if (used_p[i] || !is_real(p[i])) continue;
        if (i2 < 0 || cabs(p[i]) > cabs(p[i2])) i2 = i;
      }
    }
    if (i2 >= 0) used_p[i2] = 1;
    int n_poles = (i2 >= 0) ? 2 : 1;

    int j1 = -1, j2 = -1;
    if (n_poles == 2) {
      for (int j = 0; j < nz; ++j) {
        if (used_z[j]) continue;
        if (j1 < 0 || cabs(z[j] - p[i1]) < cabs(z[j1] - p[i1])) j1 = j;
      }
      if (j1 >= 0) {
        used_z[j1] = 1;
        if (!is_real(z[j1])) {
          for (int j = 0; j < nz; ++j) {
            if (used_z[j]) continue;
            if (j2 < 0 || cabs(z[j] - conj(z[j1])) < cabs(z[j2] - conj(z[j1]))) j2 = j;
          }
        } else {
          for (int j = 0; j < nz; ++j) {
            if (used_z[j] || !is_real(z[j])) continue;
            if (j2 < 0 || cabs(z[j] - p[i1]) < cabs(z[j2] - p[i1])) j2 = j;
          }
        }
        if (j2 >= 0) used_z[j2] = 1;
      }
    } else {
      for (int j = 0; j < nz; ++j) {
        if (used_z[j] || !is_real(z[j])) continue;
        if (j1 < 0 || cabs(z[j] - p[i1]) < cabs(z[j1] - p[i1])) j1 = j;
      }
      if (j1 >= 0) used_z[j1] = 1;
    }

    double *row = sos + 6 * s;
    /* numerator: prod (1 - z_i q^-1) over this section's zeros */
    if (j1 >= 0 && j2 >= 0) {
      row[0] = 1.0;
      row[1] = -creal(z[j1] + z[j2]);
      row[2] = creal(z[j1] * z[j2]);
    } else if (j1 >= 0) {
      row[0] = 1.0;
      row[1] = -creal(z[j1]);
      row[2] = 0.0;
    } else {
      row[0] = 1.0;
      row[1] = 0.0;
      row[2] = 0.0;
    }
    row[3] = 1.0;
    if (n_poles == 2) {
      row[4] = -creal(p[i1] + p[i2]);
      row[5] = creal(p[i1] * p[i2]);
    } else {
      row[4] = -creal(p[i1]);
      row[5] = 0.0;
    }
  }
  sos[0] *= k;
  sos[1] *= k;
  sos[2] *= k;
  *n_sec_out = n_sec;
  return ORC_OK;
}

/* order = total digital order (bandpass / bandstop: even, N = order / 2).
 * btype: 0 lowpass (f1), 1 highpass (f1), 2 bandpass (f1, f2), 3 bandstop.
 * sos_out: caller-owned [ceil(order/2)][6] rows {b0 b1 b2 1 a1 a2}. */
int oracle_butter_sos(int order, int btype, double f1, double f2, double fs,
                      double *sos_out, int *n_sec) {
  if (!sos_out || !n_sec || !(fs > 0.0) || order < 1 || order > 128) return ORC_EINVAL;
  double nyq = fs / 2.0;
  int N;
  if (btype == ORC_LOWPASS || btype == ORC_HIGHPASS) {
    if (!(f1 > 0.0 && f1 < nyq)) return ORC_EINVAL;
    N = order;
  } else if (btype == ORC_BANDPASS || btype == ORC_BANDSTOP) {
    if (order % 2 != 0) return ORC_EINVAL;
    if (!(f1 > 0.0 && f1 < f2 && f2 < nyq)) return ORC_EINVAL;
    N = order / 2;
  } else {
    return ORC_EINVAL;
  }
  double fs2 = 2.0 * fs;
  double w1 = fs2 * tan(M_PI * f1 / fs);
  double w2 = (btype >= ORC_BANDPASS) ? fs2 * tan(M_PI * f2 / fs) : 0.0;

  cplx za[256], pa[256];
  int nz, np;
  double k;
  int rc = analog_zpk(N, btype, w1, w2, za, &nz, pa, &np, &k);
  if (rc) return rc;

  /* bilinear transform */
  cplx zd[256], pd[256];
  cplx num = 1.0, den = 1.0;
  for (int i = 0; i < nz; ++i) {
    zd[i] = (fs2 + za[i]) / (fs2 - za[i]);
    num *= (fs2 - za[i]);
  }
  for (int i = 0; i < np; ++i) {
    pd[i] = (fs2 + pa[i]) / (fs2 - pa[i]);
    den *= (fs2 - pa[i]);
  }
  int nzd = nz;
  for (int i = nz; i < np; ++i) zd[nzd++] = -1.0;
  double kd = k * creal(num / den);
  for (int i = 0; i < np; ++i)
    if (!(cabs(pd[i]) < 1.0)) return ORC_EUNSTABLE;
  return zpk_to_sos(zd, nzd, pd, np, kd, sos_out, n_sec);
}

/* ------------------------------------------------------------------------
 * Direct-form-II-transposed cascade (reading of the stateful IIR-SOS
 * operator, Section 3.4).  For each channel and sample, with v the input of
 * section k:
 *     y  = b0 v + z1
 *     z1 = b1 v - a1 y + z2
 *     z2 = b2 v - a2 y
 * and y becomes the input of section k + 1.  zi[c][k][0..1] = (z1, z2) is read
 * at entry and written back at exit, so consecutive calls continue the
 * recurrence exactly (chunked == one-shot, bit for bit).
 * Rows of sos are {b0 b1 b2 a0 a1 a2}; they are divided by a0.
 * x and y may be the same array.
 * ---------------------------------------------------------------------- */
void oracle_sos_filter(const double *sos, int n_sec, const double *x, double *y,
                       int64_t n_ch, int64_t n_t, double *zi) {
  const int64_t CB = 8;  /* channels per task: one cache line of doubles */
  int64_t n_blk = (n_ch + CB - 1) / CB;
#pragma omp parallel for schedule(static)
  for (int64_t blk = 0; blk < n_blk; ++blk) {
    int64_t c0 = blk * CB, c1 = c0 + CB < n_ch ? c0 + CB : n_ch;
    for (int64_t t = 0; t < n_t; ++t) {
      for (int64_t c = c0; c < c1; ++c) {
        double v = x[t * n_ch + c];
        for (int s = 0; s < n_sec; ++s) {
          const double *r = sos + 6 * s;
          double a0 = r[3];
          double b0 = r[0] / a0, b1 = r[1] / a0, b2 = r[2] / a0;
          double a1 = r[4] / a0, a2 = r[5] / a0;
          double *z = zi + (c * n_sec + s) * 2;
          double out = b0 * v + z[0];
          z[0] = b1 * v - a1 * out + z[1];
          z[1] = b2 * v - a2 * out;
          v = out;
        }
        y[t * n_ch + c] = v;
      }
    }
  }
}

/* The same loop in x87 extended precision (64-bit significand), used only to
 * bound the double-precision oracle's own rounding error in the tests. */
void oracle_sos_filter_ld(const double *sos, int n_sec, const double *x, double *y,
                          int64_t n_ch, int64_t n_t, double *zi) {
  for (int64_t c = 0; c < n_ch; ++c) {
    long double z[2 * 128];
    for (int s = 0; s < n_sec; ++s) {
      z[2 * s] = zi[(c * n_sec + s) * 2];
      z[2 * s + 1] = zi[(c * n_sec + s) * 2 + 1];
    }
    for (int64_t t = 0; t < n_t; ++t) {
      long double v = x[t * n_ch + c];
      for (int s = 0; s < n_sec; ++s) {
        const double *r = sos + 6 * s;
        long double a0 = r[3];
        long double b0 = r[0] / a0, b1 = r[1] / a0, b2 = r[2] / a0;
        long double a1 = r[4] / a0, a2 = r[5] / a0;
        long double out = b0 * v + z[2 * s];
        z[2 * s] = b1 * v - a1 * out + z[2 * s + 1];
        z[2 * s + 1] = b2 * v - a2 * out;
        v = out;
      }
      y[t * n_ch + c] = (double)v;
    }
    for (int s = 0; s < n_sec; ++s) {
      zi[(c * n_sec + s) * 2] = (double)z[2 * s];
      zi[(c * n_sec + s) * 2 + 1] = (double)z[2 * s + 1];
    }
  }
}

/* ------------------------------------------------------------------------
 * Recursive STA/LTA characteristic function (reading: the exponential
 * recursive energy ratio; the paper names threshold energy detectors as
 * monitors, Section 3.4).  With e = y^2, cs = 1/nsta, cl = 1/nlta:
 *     sta = (1 - cs) sta + cs e
 *     lta = (1 - cl) lta + cl e
 *     cf  = sta / lta   if g >= nlta and lta > 0, else 0
 * where g is the 0-based global index of the sample since the state was
 * zeroed.  st[c][0..1] = (sta, lta) and *g0 (the index of this call's first
 * sample) are read at entry and advanced at exit.
 * ---------------------------------------------------------------------- */
void oracle_stalta(const double *y, double *cf, int64_t n_ch, int64_t n_t,
                   int64_t nsta, int64_t nlta, double *st, int64_t *g0) {
  const double cs = 1.0 / (double)nsta, cl = 1.0 / (double)nlta;
  const int64_t CB = 8;
  int64_t n_blk = (n_ch + CB - 1) / CB;
  int64_t gstart = *g0;
#pragma omp parallel for schedule(static)
  for (int64_t blk = 0; blk < n_blk; ++blk) {
    int64_t c0 = blk * CB, c1 = c0 + CB < n_ch ? c0 + CB : n_ch;
    for (int64_t t = 0; t < n_t; ++t) {
      for (int64_t c = c0; c < c1; ++c) {
        double v = y[t * n_ch + c];
        double e = v * v;
        double sta = (1.0 - cs) * st[2 * c] + cs * e;
        double lta = (1.0 - cl) * st[2 * c + 1] + cl * e;
        st[2 * c] = sta;
        st[2 * c + 1] = lta;
        cf[t * n_ch + c] = (gstart + t >= nlta && lta > 0.0) ? sta / lta : 0.0;
      }
    }
  }
  *g0 = gstart + n_t;
}

/* ------------------------------------------------------------------------
 * Reference gradient (reverse mode, written out by hand) of the chunk loss
 *     loss = scale * sum_{t,c} (cf[t][c] - tgt[t][c])^2
 * with respect to the input x and the normalised section coefficients
 * (b0, b1, b2, a1, a2) of every section.  The paper gives no gradient; the
 * derivative of the forward loops above is taken operation by operation, in
 * reverse order:
 *   STA/LTA at sample t, with q = 2 scale (cf - tgt) where cf is live
 *   (g >= nlta and lta > 0), else 0, and (A, B) the adjoints of (sta, lta)
 *   after sample t coming from later samples:
 *       S = A + q / lta,   Lb = B - q sta / lta^2,   e_bar = cs S + cl Lb,
 *       y_bar = 2 y e_bar,  then A <- (1 - cs) S,  B <- (1 - cl) Lb;
 *   each section, last to first, given the adjoint y_bar of its output and
 *   (u1, u2) of its delay pair after the sample:
 *       from z2' = b2 v - a2 y:        gb2 += u2 v, v_bar  = b2 u2, ga2 -= u2 y, y_bar -= a2 u2
 *       from z1' = b1 v - a1 y + z2:   gb1 += u1 v, v_bar += b1 u1, ga1 -= u1 y, y_bar -= a1 u1,
 *                                      u2 <- u1
 *       from y = b0 v + z1:            gb0 += y_bar v, v_bar += b0 y_bar, u1 <- y_bar
 *   and v_bar is the output adjoint of the section before (x_bar for the
 *   first).
 * A chunk is one call: the forward state at its start (zi0, st0, g0) is the
 * checkpoint, and adj[c] = (u1, u2 per section, A, B) carries the adjoint
 * of the state after the chunk in and the adjoint of the state before it
 * out, so chunks processed last-to-first give the one-shot gradient (the
 * adjoint after the record's last sample is zero).
 * gx [n_t][n_ch] is written; gsos [n_sec][5] and *loss are added to, in
 * channel order (independent of the thread count).
 * ---------------------------------------------------------------------- */
static void coef_row(const double *r, double *b0, double *b1, double *b2, double *a1, double *a2) {
  double a0 = r[3];
  *b0 = r[0] / a0;
  *b1 = r[1] / a0;
  *b2 = r[2] / a0;
  *a1 = r[4] / a0;
  *a2 = r[5] / a0;
}

/* Reverse through the cascade at one sample. v[k] is the input of section k,
 * v[n_sec] the cascade output; u[2k], u[2k+1] the adjoints of section k's
 * delay pair after the sample (replaced by the adjoints before it); g[5k..]
 * accumulates the coefficient gradients.  Returns the adjoint of x. */
static double cascade_reverse(const double *sos, int n_sec, const double *v, double ybar, double *u,
                              double *g) {
  for (int k = n_sec - 1; k >= 0; --k) {
    double b0, b1, b2, a1, a2;
    coef_row(sos + 6 * k, &b0, &b1, &b2, &a1, &a2);
    const double vin = v[k], yout = v[k + 1];
    const double u1 = u[2 * k], u2 = u[2 * k + 1];
    double yb = ybar;
    double vb;
    /* z2' = b2 v - a2 y */
    g[5 * k + 2] += u2 * vin;
    vb = b2 * u2;
    g[5 * k + 4] -= u2 * yout;
    yb -= a2 * u2;
    /* z1' = b1 v - a1 y + z2 */
    g[5 * k + 1] += u1 * vin;
    vb += b1 * u1;
    g[5 * k + 3] -= u1 * yout;
    yb -= a1 * u1;
    /* y = b0 v + z1 */
    g[5 * k + 0] += yb * vin;
    vb += b0 * yb;
    u[2 * k] = yb;   /* adjoint of z1 before the sample */
    u[2 * k + 1] = u1; /* adjoint of z2 before the sample */
    ybar = vb;
  }
  return ybar;
}

void oracle_sos_stalta_grad(const double *sos, int n_sec, const double *x, const double *tgt,
                            int64_t n_ch, int64_t n_t, int64_t nsta, int64_t nlta, int64_t g0,
                            double scale, const double *zi0, const double *st0, double *adj,
                            double *gx, double *gsos, double *loss) {
  const double cs = 1.0 / (double)nsta, cl = 1.0 / (double)nlta;
  const int na = 2 * n_sec + 2;
  double *gch = (double *)calloc((size_t)n_ch * (5 * n_sec + 1), sizeof(double));
#pragma omp parallel
  {
    /* per-thread tape of one channel: section inputs / output, sta, lta */
    double *tv = (double *)malloc((size_t)n_t * (n_sec + 1) * sizeof(double));
    double *ts = (double *)malloc((size_t)n_t * 2 * sizeof(double));
#pragma omp for schedule(static)
    for (int64_t c = 0; c < n_ch; ++c) {
      double z[2 * 128];
      for (int i = 0; i < 2 * n_sec; ++i) z[i] = zi0[c * 2 * n_sec + i];
      double sta = st0[2 * c], lta = st0[2 * c + 1];
      double *gc = gch + c * (5 * n_sec + 1);
      for (int64_t t = 0; t < n_t; ++t) {
        double v = x[t * n_ch + c];
        double *row = tv + t * (n_sec + 1);
        for (int k = 0; k < n_sec; ++k) {
          double b0, b1, b2, a1, a2;
          coef_row(sos + 6 * k, &b0, &b1, &b2, &a1, &a2);
          row[k] = v;
          double out = b0 * v + z[2 * k];
          z[2 * k] = b1 * v - a1 * out + z[2 * k + 1];
          z[2 * k + 1] = b2 * v - a2 * out;
          v = out;
        }
        row[n_sec] = v;
        double e = v * v;
        sta = (1.0 - cs) * sta + cs * e;
        lta = (1.0 - cl) * lta + cl * e;
        ts[2 * t] = sta;
        ts[2 * t + 1] = lta;
      }
      double u[2 * 128];
      for (int i = 0; i < 2 * n_sec; ++i) u[i] = adj[c * na + i];
      double A = adj[c * na + 2 * n_sec], B = adj[c * na + 2 * n_sec + 1];
      double lsum = 0.0;
      for (int64_t t = n_t - 1; t >= 0; --t) {
        const double s = ts[2 * t], l = ts[2 * t + 1];
        const int live = (g0 + t >= nlta && l > 0.0);
        const double cf = live ? s / l : 0.0;
        const double d = cf - tgt[t * n_ch + c];
        lsum += scale * d * d;
        const double q = live ? 2.0 * scale * d : 0.0;
        const double S = A + (live ? q / l : 0.0);
        const double Lb = B - (live ? q * s / (l * l) : 0.0);
        const double ebar = cs * S + cl * Lb;
        A = (1.0 - cs) * S;
        B = (1.0 - cl) * Lb;
        const double *row = tv + t * (n_sec + 1);
        const double ybar = 2.0 * row[n_sec] * ebar;
        gx[t * n_ch + c] = cascade_reverse(sos, n_sec, row, ybar, u, gc);
      }
      for (int i = 0; i < 2 * n_sec; ++i) adj[c * na + i] = u[i];
      adj[c * na + 2 * n_sec] = A;
      adj[c * na + 2 * n_sec + 1] = B;
      gc[5 * n_sec] = lsum;
    }
    free(tv);
    free(ts);
  }
  for (int64_t c = 0; c < n_ch; ++c) {
    const double *gc = gch + c * (5 * n_sec + 1);
    for (int i = 0; i < 5 * n_sec; ++i) gsos[i] += gc[i];
    *loss += gc[5 * n_sec];
  }
  free(gch);
}

/* Vector-Jacobian product of the cascade alone over one chunk: given the
 * adjoint gy [n_t][n_ch] of the filter output, gx = (d y / d x)^T gy and the
 * coefficient gradients sum_t gy . d y / d theta (gsos [n_sec][5], added to).
 * zi0 is the forward state at the chunk start; adjz [n_ch][n_sec][2] carries
 * the delay-pair adjoints in (after the chunk) and out (before it). */
void oracle_sos_vjp(const double *sos, int n_sec, const double *x, const double *gy, int64_t n_ch,
                    int64_t n_t, const double *zi0, double *adjz, double *gx, double *gsos) {
  double *gch = (double *)calloc((size_t)n_ch * 5 * n_sec, sizeof(double));
#pragma omp parallel
  {
    double *tv = (double *)malloc((size_t)n_t * (n_sec + 1) * sizeof(double));
#pragma omp for schedule(static)
    for (int64_t c = 0; c < n_ch; ++c) {
      double z[2 * 128];
      for (int i = 0; i < 2 * n_sec; ++i) z[i] = zi0[c * 2 * n_sec + i];
      for (int64_t t = 0; t < n_t; ++t) {
        double v = x[t * n_ch + c];
        double *row = tv + t * (n_sec + 1);
        for (int k = 0; k < n_sec; ++k) {
          double b0, b1, b2, a1, a2;
          coef_row(sos + 6 * k, &b0, &b1, &b2, &a1, &a2);
          row[k] = v;
          double out = b0 * v + z[2 * k];
          z[2 * k] = b1 * v - a1 * out + z[2 * k + 1];
          z[2 * k + 1] = b2 * v - a2 * out;
          v = out;
        }
        row[n_sec] = v;
      }
      double u[2 * 128];
      for (int i = 0; i < 2 * n_sec; ++i) u[i] = adjz[c * 2 * n_sec + i];
      double *gc = gch + c * 5 * n_sec;
      for (int64_t t = n_t - 1; t >= 0; --t)
        gx[t * n_ch + c] = cascade_reverse(sos, n_sec, tv + t * (n_sec + 1), gy[t * n_ch + c], u, gc);
      for (int i = 0; i < 2 * n_sec; ++i) adjz[c * 2 * n_sec + i] = u[i];
    }
    free(tv);
  }
  for (int64_t c = 0; c < n_ch; ++c)
    for (int i = 0; i < 5 * n_sec; ++i) gsos[i] += gch[c * 5 * n_sec + i];
  free(gch);
}

/* ------------------------------------------------------------------------
 * Threshold trigger on a characteristic function: the monitor contract of
 * Section 3.4 (a window of data goes in, a list of time-channel events comes
 * out), with the classic two-threshold hysteresis of an energy detector.
 * Per channel: while closed, the first sample whose cf exceeds `on` opens an
 * event at that sample; while open, the first sample whose cf is below `off`
 * closes it, and the event [t_on, t_off) is emitted.  Comparisons are made
 * in FP32, the precision cf is delivered in.  An event still open after the
 * last sample stays in the state (open flag and t_on), so any chunking emits
 * the events of the one-shot run.  Sample indices are global: g0 is the
 * index of the chunk's first sample.  Events are appended to ev[cap][3] as
 * (channel, t_on, t_off), channel by channel in time order; the return value
 * is the number found (events past cap are counted but not stored).
 * ------------------------------------------------------------------------ */
int64_t oracle_trigger(const float *cf, int64_t n_ch, int64_t n_t, float on, float off,
                       uint8_t *open, int64_t *t_on, int64_t g0, int64_t *ev, int64_t cap) {
  int64_t n = 0;
  for (int64_t c = 0; c < n_ch; ++c) {
    for (int64_t t = 0; t < n_t; ++t) {
      const float v = cf[t * n_ch + c];
      if (!open[c]) {
        if (v > on) {
          open[c] = 1;
          t_on[c] = g0 + t;
        }
      } else if (v < off) {
        if (n < cap) {
          ev[3 * n + 0] = c;
          ev[3 * n + 1] = t_on[c];
          ev[3 * n + 2] = g0 + t;
        }
        ++n;
        open[c] = 0;
      }
    }
  }
  return n;
}

/* ------------------------------------------------------------------------
 * Zero-phase filtering of a window (the display filter's zero-phase option,
 * Section 3.2): the cascade from rest forward over x, then from rest over the
 * result taken backward in time; no padding at either edge.  x and y may be
 * the same array.
 * ------------------------------------------------------------------------ */
static double cascade_sample(const double *sos, int n_sec, double *z, double v) {
  for (int s = 0; s < n_sec; ++s) {
    const double *r = sos + 6 * s;
    const double a0 = r[3];
    const double b0 = r[0] / a0, b1 = r[1] / a0, b2 = r[2] / a0;
    const double a1 = r[4] / a0, a2 = r[5] / a0;
    const double out = b0 * v + z[2 * s];
    z[2 * s] = b1 * v - a1 * out + z[2 * s + 1];
    z[2 * s + 1] = b2 * v - a2 * out;
    v = out;
  }
  return v;
}

void oracle_sos_filtfilt(const double *sos, int n_sec, const double *x, double *y, int64_t n_ch, int64_t n_t) {
#pragma omp parallel
  {
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n_t > 0 ? n_t : 1));
    double z[2 * 64];
#pragma omp for schedule(static)
    for (int64_t c = 0; c < n_ch; ++c) {
      for (int i = 0; i < 2 * n_sec; ++i) z[i] = 0.0;
      for (int64_t t = 0; t < n_t; ++t) tmp[t] = cascade_sample(sos, n_sec, z, x[t * n_ch + c]);
      for (int i = 0; i < 2 * n_sec; ++i) z[i] = 0.0;
      for (int64_t t = n_t - 1; t >= 0; --t) y[t * n_ch + c] = cascade_sample(sos, n_sec, z, tmp[t]);
    }
    free(tmp);
  }
}

/* ------------------------------------------------------------------------
 * Stateful exponential-average operators (Table 1's running mean and
 * running AGC rows, Section 3.4): per channel, with c = 1 / n_win,
 *   mode 0, running-mean removal:  m = (1 - c) m + c x;    y = x - m
 *   mode 1, running AGC:           p = (1 - c) p + c x^2;  y = x / sqrt(p) (0 where p = 0)
 * starting from the carried average avg[c] (0 at rest) and leaving the
 * average after the last sample in it, so any chunking gives the one-shot
 * result.  x and y may be the same array.
 * ------------------------------------------------------------------------ */
void oracle_ema_op(const double *x, double *y, int64_t n_ch, int64_t n_t, int64_t n_win, int mode,
                   double *avg) {
  const double c = 1.0 / (double)n_win;
#pragma omp parallel for schedule(static)
  for (int64_t ch = 0; ch < n_ch; ++ch) {
    double a = avg[ch];
    for (int64_t t = 0; t < n_t; ++t) {
      const double v = x[t * n_ch + ch];
      if (mode == 0) {
        a = (1.0 - c) * a + c * v;
        y[t * n_ch + ch] = v - a;
      } else {
        a = (1.0 - c) * a + c * v * v;
        y[t * n_ch + ch] = a > 0.0 ? v / sqrt(a) : 0.0;
      }
    }
    avg[ch] = a;
  }
}

/* ------------------------------------------------------------------------
 * Realtime FIR with carried history (Table 1's FIR row, Section 3.4):
 *   y[t] = sum_{k < M} h[k] x[t - k]
 * where samples before the chunk come from hist[M - 1][n_ch] (oldest first:
 * hist[i] is the sample M - 1 - i before the chunk's first), zero at rest;
 * hist is left holding the last M - 1 samples.  FP64 accumulation of the
 * taps and samples as given.  x and y must differ.
 * ------------------------------------------------------------------------ */
void oracle_fir(const double *h, int M, const double *x, double *y, int64_t n_ch, int64_t n_t, double *hist) {
  const int64_t H = M - 1;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < n_ch; ++c) {
    for (int64_t t = 0; t < n_t; ++t) {
      double acc = 0.0;
      for (int k = 0; k < M; ++k) {
        const int64_t s = t - k;
        const double v = s >= 0 ? x[s * n_ch + c] : hist[(H + s) * n_ch + c];
        acc += h[k] * v;
      }
      y[t * n_ch + c] = acc;
    }
    /* the last H samples, oldest first */
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(H > 0 ? H : 1));
    for (int64_t i = 0; i < H; ++i) {
      const int64_t s = n_t - H + i;
      tmp[i] = s >= 0 ? x[s * n_ch + c] : hist[(H + s) * n_ch + c];
    }
    for (int64_t i = 0; i < H; ++i) hist[i * n_ch + c] = tmp[i];
    free(tmp);
  }
}
