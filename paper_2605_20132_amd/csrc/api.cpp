// Host side of the C ABI (include/filark.h): state objects, FP64 scan tables,
// argument checks and kernel launches.
//
// Every operator follows process(chunk, state) -> (output, new_state)
// (FiLark Section 3.4): the device state a call leaves behind is where the
// next call starts.  Device state buffers are double-buffered by launch
// parity: a launch reads parity e & 1 and its last block writes parity
// (e & 1) ^ 1, where e is the object's launch epoch that the last finishing
// workgroup advances on the device.  Hence a chunk's initial state is never
// overwritten while tiles of the same launch may still read it, and repeated
// launches (including graph replays) need no host bookkeeping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/filark.h"
#include "internal.h"

namespace filark {
filark_status design_butterworth(int order, int btype, double f1, double f2, double fs,
                                 double *sos_out, int *n_sec, const char **why);
size_t fwd_lds_bytes(int K, int waves);
}  // namespace filark

using namespace filark;

namespace {

thread_local std::string g_err;

filark_status fail(filark_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(FILARK_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int kDefaultWaves = 3;
constexpr int kDefaultBlock = 64;
constexpr int kSpinLimit = 1 << 22;

// Dense row-major n x n matrices in FP64.
using Mat = std::vector<double>;

Mat identity(int n) {
  Mat m(n * n, 0.0);
  for (int i = 0; i < n; ++i) m[i * n + i] = 1.0;
  return m;
}

Mat matmul(const Mat &a, const Mat &b, int n) {
  Mat c(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double aik = a[i * n + k];
      if (aik == 0.0) continue;
      for (int j = 0; j < n; ++j) c[i * n + j] += aik * b[k * n + j];
    }
  return c;
}

std::vector<double> matvec(const Mat &a, const std::vector<double> &v, int n) {
  std::vector<double> r(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) r[i] += a[i * n + j] * v[j];
  return r;
}

// Normalised section coefficients b0 b1 b2 a1 a2.
struct Cascade {
  int K = 0;
  double c[kMaxSections][5];
};

// One direct-form-II-transposed step of the whole cascade.
double cascade_step(const Cascade &cs, double *s, double v) {
  for (int k = 0; k < cs.K; ++k) {
    const double *r = cs.c[k];
    const double y = r[0] * v + s[2 * k];
    const double z1 = r[1] * v - r[3] * y + s[2 * k + 1];
    const double z2 = r[2] * v - r[4] * y;
    s[2 * k] = z1;
    s[2 * k + 1] = z2;
    v = y;
  }
  return v;
}

// State-space form of the cascade: s' = A s + B v (state = DF2T delay pairs).
void cascade_matrices(const Cascade &cs, Mat &A, std::vector<double> &B) {
  const int n = 2 * cs.K;
  A.assign(n * n, 0.0);
  B.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    std::vector<double> s(n, 0.0);
    s[i] = 1.0;
    cascade_step(cs, s.data(), 0.0);
    for (int r = 0; r < n; ++r) A[r * n + i] = s[r];
  }
  std::vector<double> s(n, 0.0);
  cascade_step(cs, s.data(), 1.0);
  B = s;
}

bool section_stable(double a1, double a2) {
  // roots of z^2 + a1 z + a2
  const std::complex<double> disc = std::sqrt(std::complex<double>(a1 * a1 - 4.0 * a2, 0.0));
  const std::complex<double> r1 = (-a1 + disc) / 2.0, r2 = (-a1 - disc) / 2.0;
  return std::abs(r1) < 1.0 && std::abs(r2) < 1.0;
}

struct Workspace {
  double *rec = nullptr;
  uint32_t *flags = nullptr;
  size_t cells = 0;
  int ns = 0;
};

void ws_free(Workspace &w) {
  if (w.rec) (void)hipFree(w.rec);
  if (w.flags) (void)hipFree(w.flags);
  w = Workspace();
}

// Grow the look-back workspace to hold `cells` tiles with NS-wide SOS records.
filark_status ws_ensure(Workspace &w, size_t cells, int ns, hipStream_t stream) {
  if (w.rec && cells <= w.cells && ns <= w.ns) return FILARK_OK;
  const size_t c2 = std::max(cells, w.cells);
  const int n2 = std::max(ns, w.ns);
  HIP_TRY(hipStreamSynchronize(stream));
  ws_free(w);
  const size_t rec_doubles = c2 * (size_t)(2 * n2 * kWave + 2 * 2 * kWave);
  HIP_TRY(hipMalloc(&w.rec, rec_doubles * sizeof(double)));
  HIP_TRY(hipMalloc(&w.flags, 2 * c2 * sizeof(uint32_t)));
  HIP_TRY(hipMemsetAsync(w.flags, 0, 2 * c2 * sizeof(uint32_t), stream));
  HIP_TRY(hipStreamSynchronize(stream));
  w.cells = c2;
  w.ns = n2;
  return FILARK_OK;
}

int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

}  // namespace

struct filark_sos_state {
  int device = 0;
  int64_t n_ch = 0;
  Cascade cas;
  int waves = kDefaultWaves;
  int block = kDefaultBlock;
  double *d_state = nullptr;  // 2 parities x [2K][n_ch]
  uint32_t *d_ctrl = nullptr;
  double *d_tab = nullptr;    // coef | G | P | Q[q_cap]
  int q_cap = 0;
  size_t off_G = 0, off_P = 0, off_Q = 0;
  Workspace ws;
};

struct filark_stalta_state {
  int device = 0;
  int64_t n_ch = 0;
  int64_t nsta = 0, nlta = 0;
  int waves = kDefaultWaves;
  int block = kDefaultBlock;
  double *d_state = nullptr;  // 2 parities x [2][n_ch]
  uint32_t *d_ctrl = nullptr;
  double *d_tab = nullptr;    // aL_s, aL_l, qs[q_cap], ql[q_cap]
  int q_cap = 0;
  Workspace ws;
};

namespace {

filark_status sos_tables(filark_sos_state *st, int q_cap, hipStream_t stream) {
  const int K = st->cas.K, n = 2 * K, L = st->block;
  Mat A;
  std::vector<double> B;
  cascade_matrices(st->cas, A, B);
  std::vector<double> tab;
  for (int k = 0; k < K; ++k) {
    const double *r = st->cas.c[k];
    tab.insert(tab.end(), {r[0], r[1], r[2], -r[3], -r[4]});
  }
  while (tab.size() % 8) tab.push_back(0.0);
  st->off_G = tab.size();
  std::vector<std::vector<double>> G(L);
  G[L - 1] = B;
  for (int j = L - 2; j >= 0; --j) G[j] = matvec(A, G[j + 1], n);
  for (int j = 0; j < L; ++j) tab.insert(tab.end(), G[j].begin(), G[j].end());
  while (tab.size() % 8) tab.push_back(0.0);
  st->off_P = tab.size();
  Mat P = identity(n);
  for (int j = 0; j < L; ++j) P = matmul(A, P, n);
  tab.insert(tab.end(), P.begin(), P.end());
  while (tab.size() % 8) tab.push_back(0.0);
  st->off_Q = tab.size();
  Mat Qs = identity(n);
  for (int w = 0; w < st->waves; ++w) Qs = matmul(P, Qs, n);
  Mat Qm = identity(n);
  for (int m = 0; m < q_cap; ++m) {
    tab.insert(tab.end(), Qm.begin(), Qm.end());
    Qm = matmul(Qs, Qm, n);
  }
  if (st->d_tab) {
    HIP_TRY(hipStreamSynchronize(stream));
    (void)hipFree(st->d_tab);
    st->d_tab = nullptr;
  }
  HIP_TRY(hipMalloc(&st->d_tab, tab.size() * sizeof(double)));
  HIP_TRY(hipMemcpyAsync(st->d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice,
                         stream));
  HIP_TRY(hipStreamSynchronize(stream));
  st->q_cap = q_cap;
  return FILARK_OK;
}

filark_status stalta_tables(filark_stalta_state *st, int q_cap, hipStream_t stream) {
  const int L = st->block, S = st->waves * st->block;
  const double as = 1.0 - 1.0 / (double)st->nsta, al = 1.0 - 1.0 / (double)st->nlta;
  std::vector<double> tab(2 + 2 * (size_t)q_cap);
  tab[0] = std::pow(as, L);
  tab[1] = std::pow(al, L);
  for (int m = 0; m < q_cap; ++m) {
    tab[2 + m] = std::pow(as, (double)S * m);
    tab[2 + q_cap + m] = std::pow(al, (double)S * m);
  }
  if (st->d_tab) {
    HIP_TRY(hipStreamSynchronize(stream));
    (void)hipFree(st->d_tab);
    st->d_tab = nullptr;
  }
  HIP_TRY(hipMalloc(&st->d_tab, tab.size() * sizeof(double)));
  HIP_TRY(hipMemcpyAsync(st->d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice,
                         stream));
  HIP_TRY(hipStreamSynchronize(stream));
  st->q_cap = q_cap;
  return FILARK_OK;
}

int round_cap(int need) {
  int c = 16;
  while (c < need) c *= 2;
  return c;
}

filark_status alloc_ctrl(uint32_t **ctrl, hipStream_t stream) {
  HIP_TRY(hipMalloc(ctrl, kCtrlWords * sizeof(uint32_t)));
  HIP_TRY(hipMemsetAsync(*ctrl, 0, kCtrlWords * sizeof(uint32_t), stream));
  return FILARK_OK;
}

filark_status read_ctrl(const uint32_t *d_ctrl, uint32_t *h, hipStream_t stream) {
  HIP_TRY(hipStreamSynchronize(stream));
  HIP_TRY(hipMemcpy(h, d_ctrl, kCtrlWords * sizeof(uint32_t), hipMemcpyDeviceToHost));
  return FILARK_OK;
}

// Shared launch path of the three processing entry points.
filark_status run_forward(filark_sos_state *sos, filark_stalta_state *sl, const float *in,
                          float *y, float *cf, int64_t n_ch, int64_t n_t, hipStream_t stream) {
  if (n_t < 0 || n_t > 0x7fffffff) return fail(FILARK_EINVAL, "n_t out of range: %lld", (long long)n_t);
  if (n_ch < 1) return fail(FILARK_EINVAL, "n_ch must be >= 1");
  if (n_ch > (int64_t)1 << 24) return fail(FILARK_EINVAL, "n_ch above 2^24 is not supported");
  if (sos && sos->n_ch != n_ch)
    return fail(FILARK_ESHAPE, "n_ch %lld differs from the SOS state's %lld", (long long)n_ch,
                (long long)sos->n_ch);
  if (sl && sl->n_ch != n_ch)
    return fail(FILARK_ESHAPE, "n_ch %lld differs from the STA/LTA state's %lld", (long long)n_ch,
                (long long)sl->n_ch);
  if (n_t == 0) return FILARK_OK;
  if (!in) return fail(FILARK_EINVAL, "null input pointer");
  if (sos && !sl && !y) return fail(FILARK_EINVAL, "null output pointer");
  if (sl && !cf) return fail(FILARK_EINVAL, "null cf pointer");
  if (y && cf && (const void *)y == (const void *)cf) return fail(FILARK_EINVAL, "y and cf must differ");
  const int waves = sos ? sos->waves : sl->waves;
  const int block = sos ? sos->block : sl->block;
  if (sos && sl && (sos->waves != sl->waves || sos->block != sl->block))
    return fail(FILARK_EINVAL, "tile shapes of the states differ (set both with filark_tile_set)");
  if ((uint64_t)block * (uint64_t)n_ch * 4u >= 0x7fffffffull)
    return fail(FILARK_EINVAL, "row stride too large");
  const int K = sos ? sos->cas.K : 0;
  const int seg_len = waves * block;
  const int n_seg = (int)((n_t + seg_len - 1) / seg_len);
  const int n_grp = (int)((n_ch + kWave - 1) / kWave);
  const size_t cells = (size_t)n_seg * (size_t)n_grp;
  if (cells > 0x7fffffffull) return fail(FILARK_EINVAL, "too many tiles");

  int prev_dev = current_device();
  const int dev = sos ? sos->device : sl->device;
  if (prev_dev != dev) HIP_TRY(hipSetDevice(dev));

  filark_status rc = FILARK_OK;
  if (sos && n_seg > sos->q_cap) rc = sos_tables(sos, round_cap(n_seg), stream);
  if (rc == FILARK_OK && sl && n_seg > sl->q_cap) rc = stalta_tables(sl, round_cap(n_seg), stream);
  Workspace &ws = sos ? sos->ws : sl->ws;
  if (rc == FILARK_OK) rc = ws_ensure(ws, cells, 2 * K, stream);
  if (rc != FILARK_OK) {
    if (prev_dev != dev) (void)hipSetDevice(prev_dev);
    return rc;
  }

  FwdParams p;
  std::memset(&p, 0, sizeof p);
  p.x = in;
  p.y = y;
  p.cf = cf;
  p.n_ch = n_ch;
  p.n_t = (int32_t)n_t;
  p.n_seg = n_seg;
  p.n_grp = n_grp;
  p.seg_len = seg_len;
  if (sos) {
    p.zs = sos->d_state;
    p.coef = sos->d_tab;
    p.G = sos->d_tab + sos->off_G;
    p.P = sos->d_tab + sos->off_P;
    p.Q = sos->d_tab + sos->off_Q;
    p.sos_ctrl = sos->d_ctrl;
  }
  if (sl) {
    p.sl = sl->d_state;
    p.slq = sl->d_tab;
    p.q_cap = sl->q_cap;
    p.sl_ctrl = sl->d_ctrl;
    p.nlta = sl->nlta;
    p.nsta_d = (double)sl->nsta;
    p.nlta_d = (double)sl->nlta;
    p.asd = 1.0 - 1.0 / (double)sl->nsta;
    p.ald = 1.0 - 1.0 / (double)sl->nlta;
    p.as = (float)p.asd;
    p.al = (float)p.ald;
    p.kappa = (float)((double)sl->nlta / (double)sl->nsta);
  }
  p.rec = ws.rec;
  p.flags = ws.flags;
  p.ctrl = sos ? sos->d_ctrl : sl->d_ctrl;
  p.spin_limit = kSpinLimit;
  hipError_t e = launch_fwd(p, K, block, sl != nullptr, sl == nullptr || y != nullptr, waves, stream);
  if (prev_dev != dev) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) return fail(FILARK_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

}  // namespace

extern "C" {

const char *filark_last_error(void) { return g_err.c_str(); }

const char *filark_version(void) { return "filark-mi355x 0.1 (gfx950)"; }

filark_status filark_sos_design(int order, int btype, double f1, double f2, double fs,
                                double *sos_out, int *n_sec) {
  const char *why = nullptr;
  filark_status st = design_butterworth(order, btype, f1, f2, fs, sos_out, n_sec, &why);
  if (st != FILARK_OK) return fail(st, "filark_sos_design: %s", why ? why : "error");
  return FILARK_OK;
}

filark_status filark_sos_init(filark_sos_t *out, const double *sos, int n_sec, int64_t n_ch,
                              unsigned flags, hipStream_t stream) {
  if (!out) return fail(FILARK_EINVAL, "null state pointer");
  *out = nullptr;
  if (!sos) return fail(FILARK_EINVAL, "null sos pointer");
  if (n_sec < 1 || n_sec > kMaxSections) return fail(FILARK_EINVAL, "n_sec must be in [1, %d]", kMaxSections);
  if (n_ch < 1 || n_ch > (int64_t)1 << 24) return fail(FILARK_EINVAL, "n_ch must be in [1, 2^24]");
  if (flags != 0) return fail(FILARK_EINVAL, "unknown flags");
  Cascade cas;
  cas.K = n_sec;
  for (int k = 0; k < n_sec; ++k) {
    const double *r = sos + 6 * k;
    for (int i = 0; i < 6; ++i)
      if (!std::isfinite(r[i])) return fail(FILARK_EINVAL, "non-finite coefficient in section %d", k);
    if (r[3] == 0.0) return fail(FILARK_EINVAL, "a0 of section %d is zero", k);
    cas.c[k][0] = r[0] / r[3];
    cas.c[k][1] = r[1] / r[3];
    cas.c[k][2] = r[2] / r[3];
    cas.c[k][3] = r[4] / r[3];
    cas.c[k][4] = r[5] / r[3];
    if (!section_stable(cas.c[k][3], cas.c[k][4]))
      return fail(FILARK_EUNSTABLE, "section %d has a pole on or outside the unit circle", k);
  }
  filark_sos_state *st = new (std::nothrow) filark_sos_state();
  if (!st) return fail(FILARK_ENOMEM, "host allocation failed");
  st->device = current_device();
  st->n_ch = n_ch;
  st->cas = cas;
  const size_t bytes = 2 * (size_t)(2 * n_sec) * (size_t)n_ch * sizeof(double);
  filark_status rc = FILARK_OK;
  hipError_t e = hipMalloc(&st->d_state, bytes);
  if (e == hipSuccess) e = hipMemsetAsync(st->d_state, 0, bytes, stream);
  if (e != hipSuccess) rc = fail(FILARK_EHIP, "state allocation: %s", hipGetErrorString(e));
  if (rc == FILARK_OK) rc = alloc_ctrl(&st->d_ctrl, stream);
  if (rc == FILARK_OK) rc = sos_tables(st, 16, stream);
  if (rc != FILARK_OK) {
    filark_sos_destroy(st);
    return rc;
  }
  *out = st;
  return FILARK_OK;
}

filark_status filark_stalta_init(filark_stalta_t *out, double sta_s, double lta_s, double fs,
                                 int64_t n_ch, hipStream_t stream) {
  if (!out) return fail(FILARK_EINVAL, "null state pointer");
  *out = nullptr;
  if (!(fs > 0.0) || !(sta_s > 0.0) || !(lta_s > 0.0) || !std::isfinite(fs * sta_s) ||
      !std::isfinite(fs * lta_s))
    return fail(FILARK_EINVAL, "windows and fs must be positive and finite");
  const double ns = std::round(sta_s * fs), nl = std::round(lta_s * fs);
  if (ns < 1.0 || nl < 1.0 || nl > 9.0e15) return fail(FILARK_EINVAL, "window lengths must round to >= 1 sample");
  if (n_ch < 1 || n_ch > (int64_t)1 << 24) return fail(FILARK_EINVAL, "n_ch must be in [1, 2^24]");
  filark_stalta_state *st = new (std::nothrow) filark_stalta_state();
  if (!st) return fail(FILARK_ENOMEM, "host allocation failed");
  st->device = current_device();
  st->n_ch = n_ch;
  st->nsta = (int64_t)ns;
  st->nlta = (int64_t)nl;
  const size_t bytes = 2 * 2 * (size_t)n_ch * sizeof(double);
  filark_status rc = FILARK_OK;
  hipError_t e = hipMalloc(&st->d_state, bytes);
  if (e == hipSuccess) e = hipMemsetAsync(st->d_state, 0, bytes, stream);
  if (e != hipSuccess) rc = fail(FILARK_EHIP, "state allocation: %s", hipGetErrorString(e));
  if (rc == FILARK_OK) rc = alloc_ctrl(&st->d_ctrl, stream);
  if (rc == FILARK_OK) rc = stalta_tables(st, 16, stream);
  if (rc != FILARK_OK) {
    filark_stalta_destroy(st);
    return rc;
  }
  *out = st;
  return FILARK_OK;
}

filark_status filark_sos_process(filark_sos_t st, const float *in, float *out, int64_t n_ch,
                                 int64_t n_t, hipStream_t stream) {
  if (!st) return fail(FILARK_EINVAL, "null state");
  return run_forward(st, nullptr, in, out, nullptr, n_ch, n_t, stream);
}

filark_status filark_stalta_process(filark_stalta_t st, const float *in, float *cf, int64_t n_ch,
                                    int64_t n_t, hipStream_t stream) {
  if (!st) return fail(FILARK_EINVAL, "null state");
  return run_forward(nullptr, st, in, nullptr, cf, n_ch, n_t, stream);
}

filark_status filark_sos_stalta_process(filark_sos_t sos, filark_stalta_t sl, const float *in,
                                        float *y_or_null, float *cf, int64_t n_ch, int64_t n_t,
                                        hipStream_t stream) {
  if (!sos || !sl) return fail(FILARK_EINVAL, "null state");
  if (sos->device != sl->device) return fail(FILARK_EINVAL, "states live on different devices");
  return run_forward(sos, sl, in, y_or_null, cf, n_ch, n_t, stream);
}

filark_status filark_state_get(const void *obj, int kind, void *host_buf, size_t bytes,
                               hipStream_t stream) {
  if (!obj || !host_buf) return fail(FILARK_EINVAL, "null pointer");
  uint32_t ctrl[kCtrlWords];
  if (kind == FILARK_STATE_SOS) {
    const filark_sos_state *st = static_cast<const filark_sos_state *>(obj);
    const int n = 2 * st->cas.K;
    const size_t need = (size_t)st->n_ch * n * sizeof(double);
    if (bytes != need) return fail(FILARK_EINVAL, "state_get: need %zu bytes, got %zu", need, bytes);
    filark_status rc = read_ctrl(st->d_ctrl, ctrl, stream);
    if (rc) return rc;
    const int par = (int)(ctrl[kCtrlEpoch] & 1u);
    std::vector<double> tmp((size_t)n * st->n_ch);
    HIP_TRY(hipMemcpy(tmp.data(), st->d_state + (size_t)par * n * st->n_ch, tmp.size() * sizeof(double),
                      hipMemcpyDeviceToHost));
    double *o = static_cast<double *>(host_buf);
    for (int64_t c = 0; c < st->n_ch; ++c)
      for (int i = 0; i < n; ++i) o[c * n + i] = tmp[(size_t)i * st->n_ch + c];
    return FILARK_OK;
  }
  if (kind == FILARK_STATE_STALTA) {
    const filark_stalta_state *st = static_cast<const filark_stalta_state *>(obj);
    const size_t need = (size_t)st->n_ch * 2 * sizeof(double) + sizeof(int64_t);
    if (bytes != need) return fail(FILARK_EINVAL, "state_get: need %zu bytes, got %zu", need, bytes);
    filark_status rc = read_ctrl(st->d_ctrl, ctrl, stream);
    if (rc) return rc;
    const int par = (int)(ctrl[kCtrlEpoch] & 1u);
    std::vector<double> tmp(2 * (size_t)st->n_ch);
    HIP_TRY(hipMemcpy(tmp.data(), st->d_state + (size_t)par * 2 * st->n_ch, tmp.size() * sizeof(double),
                      hipMemcpyDeviceToHost));
    double *o = static_cast<double *>(host_buf);
    for (int64_t c = 0; c < st->n_ch; ++c) {
      o[2 * c] = tmp[c];
      o[2 * c + 1] = tmp[st->n_ch + c];
    }
    const int64_t g = (int64_t)(((uint64_t)ctrl[kCtrlCounter + 1] << 32) | ctrl[kCtrlCounter]);
    std::memcpy(o + 2 * st->n_ch, &g, sizeof g);
    return FILARK_OK;
  }
  return fail(FILARK_EINVAL, "unknown state kind %d", kind);
}

filark_status filark_state_set(void *obj, int kind, const void *host_buf, size_t bytes,
                               hipStream_t stream) {
  if (!obj || !host_buf) return fail(FILARK_EINVAL, "null pointer");
  uint32_t ctrl[kCtrlWords];
  if (kind == FILARK_STATE_SOS) {
    filark_sos_state *st = static_cast<filark_sos_state *>(obj);
    const int n = 2 * st->cas.K;
    const size_t need = (size_t)st->n_ch * n * sizeof(double);
    if (bytes != need) return fail(FILARK_EINVAL, "state_set: need %zu bytes, got %zu", need, bytes);
    const double *src = static_cast<const double *>(host_buf);
    for (size_t i = 0; i < (size_t)st->n_ch * n; ++i)
      if (!std::isfinite(src[i])) return fail(FILARK_EINVAL, "state_set: non-finite value");
    filark_status rc = read_ctrl(st->d_ctrl, ctrl, stream);
    if (rc) return rc;
    const int par = (int)(ctrl[kCtrlEpoch] & 1u);
    std::vector<double> tmp((size_t)n * st->n_ch);
    for (int64_t c = 0; c < st->n_ch; ++c)
      for (int i = 0; i < n; ++i) tmp[(size_t)i * st->n_ch + c] = src[c * n + i];
    HIP_TRY(hipMemcpy(st->d_state + (size_t)par * n * st->n_ch, tmp.data(), tmp.size() * sizeof(double),
                      hipMemcpyHostToDevice));
    return FILARK_OK;
  }
  if (kind == FILARK_STATE_STALTA) {
    filark_stalta_state *st = static_cast<filark_stalta_state *>(obj);
    const size_t need = (size_t)st->n_ch * 2 * sizeof(double) + sizeof(int64_t);
    if (bytes != need) return fail(FILARK_EINVAL, "state_set: need %zu bytes, got %zu", need, bytes);
    const double *src = static_cast<const double *>(host_buf);
    for (size_t i = 0; i < (size_t)st->n_ch * 2; ++i)
      if (!std::isfinite(src[i]) || src[i] < 0.0) return fail(FILARK_EINVAL, "state_set: invalid STA/LTA value");
    int64_t g;
    std::memcpy(&g, src + 2 * st->n_ch, sizeof g);
    if (g < 0) return fail(FILARK_EINVAL, "state_set: negative sample counter");
    filark_status rc = read_ctrl(st->d_ctrl, ctrl, stream);
    if (rc) return rc;
    const int par = (int)(ctrl[kCtrlEpoch] & 1u);
    std::vector<double> tmp(2 * (size_t)st->n_ch);
    for (int64_t c = 0; c < st->n_ch; ++c) {
      tmp[c] = src[2 * c];
      tmp[st->n_ch + c] = src[2 * c + 1];
    }
    HIP_TRY(hipMemcpy(st->d_state + (size_t)par * 2 * st->n_ch, tmp.data(), tmp.size() * sizeof(double),
                      hipMemcpyHostToDevice));
    const uint32_t gw[2] = {(uint32_t)((uint64_t)g & 0xffffffffu), (uint32_t)((uint64_t)g >> 32)};
    HIP_TRY(hipMemcpy(st->d_ctrl + kCtrlCounter, gw, sizeof gw, hipMemcpyHostToDevice));
    return FILARK_OK;
  }
  return fail(FILARK_EINVAL, "unknown state kind %d", kind);
}

filark_status filark_tile_set(void *obj, int kind, int block, int waves, hipStream_t stream) {
  if (!obj) return fail(FILARK_EINVAL, "null state");
  if (block != 32 && block != 64) return fail(FILARK_EINVAL, "block must be 32 or 64");
  if (waves < 1 || waves + 1 > kMaxWaves) return fail(FILARK_EINVAL, "waves must be in [1, %d]", kMaxWaves - 1);
  if (kind == FILARK_STATE_SOS) {
    filark_sos_state *st = static_cast<filark_sos_state *>(obj);
    if (st->block == block && st->waves == waves) return FILARK_OK;
    HIP_TRY(hipStreamSynchronize(stream));
    st->block = block;
    st->waves = waves;
    return sos_tables(st, std::max(16, st->q_cap), stream);
  }
  if (kind == FILARK_STATE_STALTA) {
    filark_stalta_state *st = static_cast<filark_stalta_state *>(obj);
    if (st->block == block && st->waves == waves) return FILARK_OK;
    HIP_TRY(hipStreamSynchronize(stream));
    st->block = block;
    st->waves = waves;
    return stalta_tables(st, std::max(16, st->q_cap), stream);
  }
  return fail(FILARK_EINVAL, "unknown state kind %d", kind);
}

filark_status filark_tile_get(const void *obj, int kind, int *block, int *waves) {
  if (!obj || !block || !waves) return fail(FILARK_EINVAL, "null pointer");
  if (kind == FILARK_STATE_SOS) {
    const filark_sos_state *st = static_cast<const filark_sos_state *>(obj);
    *block = st->block;
    *waves = st->waves;
    return FILARK_OK;
  }
  if (kind == FILARK_STATE_STALTA) {
    const filark_stalta_state *st = static_cast<const filark_stalta_state *>(obj);
    *block = st->block;
    *waves = st->waves;
    return FILARK_OK;
  }
  return fail(FILARK_EINVAL, "unknown state kind %d", kind);
}

filark_status filark_check(const void *obj, int kind, hipStream_t stream) {
  if (!obj) return fail(FILARK_EINVAL, "null state");
  uint32_t *d_ctrl;
  if (kind == FILARK_STATE_SOS) d_ctrl = static_cast<const filark_sos_state *>(obj)->d_ctrl;
  else if (kind == FILARK_STATE_STALTA) d_ctrl = static_cast<const filark_stalta_state *>(obj)->d_ctrl;
  else return fail(FILARK_EINVAL, "unknown state kind %d", kind);
  uint32_t ctrl[kCtrlWords];
  filark_status rc = read_ctrl(d_ctrl, ctrl, stream);
  if (rc) return rc;
  if (ctrl[kCtrlError]) {
    const uint32_t zero = 0;
    HIP_TRY(hipMemcpy(d_ctrl + kCtrlError, &zero, sizeof zero, hipMemcpyHostToDevice));
    return fail(FILARK_ETIMEOUT, "a look-back wait exceeded its bound (error bits 0x%x)", ctrl[kCtrlError]);
  }
  return FILARK_OK;
}

filark_status filark_sos_destroy(filark_sos_t st) {
  if (!st) return FILARK_OK;
  if (st->d_state) (void)hipFree(st->d_state);
  if (st->d_ctrl) (void)hipFree(st->d_ctrl);
  if (st->d_tab) (void)hipFree(st->d_tab);
  ws_free(st->ws);
  delete st;
  return FILARK_OK;
}

filark_status filark_stalta_destroy(filark_stalta_t st) {
  if (!st) return FILARK_OK;
  if (st->d_state) (void)hipFree(st->d_state);
  if (st->d_ctrl) (void)hipFree(st->d_ctrl);
  if (st->d_tab) (void)hipFree(st->d_tab);
  ws_free(st->ws);
  delete st;
  return FILARK_OK;
}

}  // extern "C"
