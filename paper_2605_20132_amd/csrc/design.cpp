// Butterworth second-order-section design by the bilinear transform.
//
// The paper's real-time IIR comes with bandpass / lowpass / highpass wrappers
// (FiLark Section 3.4) but states no design method; this is the textbook one:
// analog Butterworth prototype, band edges pre-warped with W = 2 fs tan(pi f/fs)
// so the -3 dB points land exactly on the requested edges, LP/HP/BP/BS
// frequency transform, bilinear map s -> 2 fs (z - 1)/(z + 1), then grouping of
// poles and zeros into sections.
//
// Section arrangement: every section holds a conjugate pole pair (or two real
// poles, or one real pole for an odd low/highpass), with the zeros nearest to
// its poles; sections run from the pair farthest from the unit circle to the
// pair closest to it, and the overall gain sits in the first numerator.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "../../include/filark.h"

namespace filark {

using cplx = std::complex<double>;

namespace {

bool real_valued(cplx v) { return std::abs(v.imag()) <= 1e-10 * (1.0 + std::abs(v)); }

struct Roots {
  std::vector<cplx> zeros, poles;
  double gain = 1.0;
};

// Analog Butterworth prototype: N poles at angle pi/2 + pi (2m+1)/(2N) on the
// unit circle (left half plane), no zeros, unit gain.
std::vector<cplx> prototype_poles(int N) {
  std::vector<cplx> p;
  for (int m = 0; m < N; ++m) {
    const double phi = M_PI * (2.0 * m + 1.0) / (2.0 * N);
    p.emplace_back(-std::sin(phi), std::cos(phi));
  }
  return p;
}

cplx product_neg(const std::vector<cplx> &r) {
  cplx a(1.0, 0.0);
  for (const cplx &v : r) a *= -v;
  return a;
}

Roots analog_filter(int N, int btype, double W1, double W2) {
  const std::vector<cplx> proto = prototype_poles(N);
  Roots out;
  switch (btype) {
    case FILARK_LOWPASS:
      for (const cplx &p : proto) out.poles.push_back(W1 * p);
      out.gain = std::pow(W1, N);
      break;
    case FILARK_HIGHPASS:
      for (const cplx &p : proto) out.poles.push_back(W1 / p);
      out.zeros.assign(N, cplx(0.0, 0.0));
      out.gain = (1.0 / product_neg(proto)).real();
      break;
    case FILARK_BANDPASS: {
      const double B = W2 - W1, W0sq = W1 * W2;
      for (const cplx &p : proto) {
        const cplx h = 0.5 * B * p;
        const cplx d = std::sqrt(h * h - W0sq);
        out.poles.push_back(h + d);
        out.poles.push_back(h - d);
      }
      out.zeros.assign(N, cplx(0.0, 0.0));
      out.gain = std::pow(B, N);
      break;
    }
    default: {  // bandstop
      const double B = W2 - W1, W0sq = W1 * W2, W0 = std::sqrt(W0sq);
      for (const cplx &p : proto) {
        const cplx h = 0.5 * B / p;
        const cplx d = std::sqrt(h * h - W0sq);
        out.poles.push_back(h + d);
        out.poles.push_back(h - d);
        out.zeros.emplace_back(0.0, W0);
        out.zeros.emplace_back(0.0, -W0);
      }
      out.gain = (1.0 / product_neg(proto)).real();
      break;
    }
  }
  return out;
}

// s -> z = (2fs + s) / (2fs - s); zeros at infinity map to z = -1.
Roots bilinear(const Roots &a, double fs) {
  const double k2 = 2.0 * fs;
  Roots d;
  cplx num(1.0, 0.0), den(1.0, 0.0);
  for (const cplx &z : a.zeros) {
    d.zeros.push_back((k2 + z) / (k2 - z));
    num *= (k2 - z);
  }
  for (const cplx &p : a.poles) {
    d.poles.push_back((k2 + p) / (k2 - p));
    den *= (k2 - p);
  }
  while (d.zeros.size() < d.poles.size()) d.zeros.emplace_back(-1.0, 0.0);
  d.gain = a.gain * (num / den).real();
  return d;
}

struct Section {
  std::vector<cplx> poles, zeros;
};

// Take the index of the candidate minimising key among unused entries.
template <class Key>
int pick(const std::vector<cplx> &v, const std::vector<bool> &used, Key key) {
  int best = -1;
  double bk = 0.0;
  for (int i = 0; i < (int)v.size(); ++i) {
    if (used[i]) continue;
    const double k = key(v[i]);
    if (best < 0 || k < bk) {
      best = i;
      bk = k;
    }
  }
  return best;
}

std::vector<Section> group_sections(const Roots &d) {
  const int np = (int)d.poles.size();
  std::vector<bool> pu(np, false), zu(d.zeros.size(), false);
  std::vector<Section> secs;  // built from the least damped pair outward
  for (int remaining = np; remaining > 0;) {
    // pole nearest the unit circle; among equals, larger imaginary part
    int i1 = -1;
    for (int i = 0; i < np; ++i) {
      if (pu[i]) continue;
      if (i1 < 0) { i1 = i; continue; }
      const double ri = std::abs(d.poles[i]), r1 = std::abs(d.poles[i1]);
      if (ri > r1 || (ri == r1 && d.poles[i].imag() > d.poles[i1].imag())) i1 = i;
    }
    pu[i1] = true;
    const cplx p1 = d.poles[i1];
    Section s;
    s.poles.push_back(p1);
    int i2;
    if (!real_valued(p1)) {
      i2 = pick(d.poles, pu, [&](cplx q) { return std::abs(q - std::conj(p1)); });
    } else {
      std::vector<bool> mask = pu;
      for (int i = 0; i < np; ++i)
        if (!real_valued(d.poles[i])) mask[i] = true;
      i2 = pick(d.poles, mask, [](cplx q) { return -std::abs(q); });
    }
    if (i2 >= 0) {
      pu[i2] = true;
      s.poles.push_back(d.poles[i2]);
    }
    remaining -= (int)s.poles.size();

    std::vector<bool> zreal = zu;
    for (size_t j = 0; j < d.zeros.size(); ++j)
      if (!real_valued(d.zeros[j])) zreal[j] = true;
    if (s.poles.size() == 2) {
      const int j1 = pick(d.zeros, zu, [&](cplx q) { return std::abs(q - p1); });
      if (j1 >= 0) {
        zu[j1] = true;
        zreal[j1] = true;
        s.zeros.push_back(d.zeros[j1]);
        int j2;
        if (!real_valued(d.zeros[j1])) {
          const cplx zc = std::conj(d.zeros[j1]);
          j2 = pick(d.zeros, zu, [&](cplx q) { return std::abs(q - zc); });
        } else {
          j2 = pick(d.zeros, zreal, [&](cplx q) { return std::abs(q - p1); });
        }
        if (j2 >= 0) {
          zu[j2] = true;
          s.zeros.push_back(d.zeros[j2]);
        }
      }
    } else {
      const int j1 = pick(d.zeros, zreal, [&](cplx q) { return std::abs(q - p1); });
      if (j1 >= 0) {
        zu[j1] = true;
        s.zeros.push_back(d.zeros[j1]);
      }
    }
    secs.push_back(s);
  }
  std::reverse(secs.begin(), secs.end());
  return secs;
}

// Monic polynomial in q = z^-1 with the given roots: prod (1 - r q).
void monic(const std::vector<cplx> &r, double *c3) {
  c3[0] = 1.0;
  c3[1] = 0.0;
  c3[2] = 0.0;
  if (r.size() == 1) {
    c3[1] = -r[0].real();
  } else if (r.size() == 2) {
    c3[1] = -(r[0] + r[1]).real();
    c3[2] = (r[0] * r[1]).real();
  }
}

}  // namespace

filark_status design_butterworth(int order, int btype, double f1, double f2, double fs,
                                 double *sos_out, int *n_sec, const char **why) {
  *why = nullptr;
  if (!sos_out || !n_sec) return *why = "null output pointer", FILARK_EINVAL;
  if (!(fs > 0.0) || !std::isfinite(fs)) return *why = "fs must be positive and finite", FILARK_EINVAL;
  if (order < 1 || order > 64) return *why = "order must be in [1, 64]", FILARK_EINVAL;
  const double nyq = 0.5 * fs;
  int N;
  if (btype == FILARK_LOWPASS || btype == FILARK_HIGHPASS) {
    if (!(f1 > 0.0 && f1 < nyq)) return *why = "cutoff must satisfy 0 < f1 < fs/2", FILARK_EINVAL;
    N = order;
  } else if (btype == FILARK_BANDPASS || btype == FILARK_BANDSTOP) {
    if (order % 2) return *why = "band filters need an even order", FILARK_EINVAL;
    if (!(f1 > 0.0 && f1 < f2 && f2 < nyq))
      return *why = "band edges must satisfy 0 < f1 < f2 < fs/2", FILARK_EINVAL;
    N = order / 2;
  } else {
    return *why = "unknown filter type", FILARK_EINVAL;
  }
  const double W1 = 2.0 * fs * std::tan(M_PI * f1 / fs);
  const double W2 = btype >= FILARK_BANDPASS ? 2.0 * fs * std::tan(M_PI * f2 / fs) : 0.0;
  const Roots d = bilinear(analog_filter(N, btype, W1, W2), fs);
  for (const cplx &p : d.poles)
    if (!(std::abs(p) < 1.0)) return *why = "designed pole on or outside the unit circle", FILARK_EUNSTABLE;
  const std::vector<Section> secs = group_sections(d);
  for (size_t k = 0; k < secs.size(); ++k) {
    double *row = sos_out + 6 * k;
    monic(secs[k].zeros, row);
    monic(secs[k].poles, row + 3);
  }
  for (int i = 0; i < 3; ++i) sos_out[i] *= d.gain;
  *n_sec = (int)secs.size();
  return FILARK_OK;
}

}  // namespace filark
