// Host side of the C ABI (include/filark.h): state objects, FP64 scan tables,
// argument checks and kernel launches.
//
// Every operator follows process(chunk, state) -> (output, new_state)
// (FiLark Section 3.4): the device state a call leaves behind is where the
// next call starts.  A workgroup owns its channels for the whole chunk, so it
// reads their state at its start and overwrites it at its end, in place; no
// other workgroup touches them, and repeated launches (including graph
// replays) need no host bookkeeping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/filark.h"
#include "fir.h"
#include "internal.h"

namespace filark {
filark_status design_butterworth(int order, int btype, double f1, double f2, double fs,
                                 double *sos_out, int *n_sec, const char **why);
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

// Default tile: 48-sample blocks, 4 waves, groups of 8 channels, i.e. one
// workgroup covers 1536 rows of 8 channels per window.  Three such
// workgroups fill a CU with 12 waves, three on each SIMD: the VALU-bound
// passes see no SIMD with more waves than the others.
constexpr int kDefaultBlock = 48;
constexpr int kBatchBlock = 48;  // the batched kernel's block length
constexpr int kDefaultWaves = 8;
constexpr int kDefaultGroup = 16;

struct Tile {
  int block = kDefaultBlock;  // L: samples per lane block
  int waves = kDefaultWaves;  // waves per workgroup
  int group = kDefaultGroup;  // channels per workgroup
  bool operator==(const Tile &o) const {
    return block == o.block && waves == o.waves && group == o.group;
  }
  int blocks() const { return waves * kWave / group; }  // NB: blocks per window
  int window() const { return blocks() * block; }       // rows per window
  int levels() const {
    int k = 0;
    while ((1 << k) < blocks()) ++k;
    return std::max(1, k);
  }
};

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
  // every section after the first has b0 = b2 = 1 exactly (Butterworth
  // designs: numerators [1, +-2, 1] after the gain section)
  bool unit_tail() const {
    if (K < 2) return false;
    for (int k = 1; k < K; ++k)
      if (c[k][0] != 1.0 || c[k][2] != 1.0) return false;
    return true;
  }
  // bit k: section k is first order (a2 = b2 = 0)
  int first_order_bits() const {
    int m = 0;
    for (int k = 0; k < K; ++k)
      if (c[k][4] == 0.0 && c[k][2] == 0.0) m |= 1 << k;
    return m;
  }
  // the adjoint may rebuild section signals backwards: every section's state
  // update is invertible with |a2| >= 1/4 (first order: |a1| >= 1/2), so
  // undoing 16 rows grows rounding by at most 2^16
  bool invertible() const {
    for (int k = 0; k < K; ++k) {
      const double b2 = c[k][2], a1 = c[k][3], a2 = c[k][4];
      if (a2 != 0.0) {
        if (!(std::fabs(a2) >= 0.25)) return false;
      } else if (b2 != 0.0 || !(std::fabs(a1) >= 0.5)) {
        return false;
      }
    }
    return true;
  }
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

int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

}  // namespace

// Scan tables of one tile shape: coef [K][5] = b0 b1 b2 -a1 -a2 |
// G [L][2K] = A^(L-1-j) B | Pw [levels][2K][2K] = A^(L 2^k) (filter), or
// [levels][2] = (as, al)^(L 2^k) then [L + 1][2] = (as, al)^m (STA/LTA).
struct Tables {
  Tile tile;
  double *d = nullptr;
  size_t off_G = 0, off_P = 0, off_R = 0;
};

struct filark_sos_state {
  int device = 0;
  int64_t n_ch = 0;
  Cascade cas;
  double *d_state = nullptr;  // [2K][n_ch]
  Tables fwd;                 // forward kernel
  Tables adj;                 // adjoint kernel
  Tables ckp;                 // forward pass that checkpoints the adjoint's window starts
  uint64_t gen = 0;           // bumped whenever the forward tables are rebuilt
  // adjoint workspace: window checkpoints and per-group coefficient sums
  double *d_ck = nullptr;
  size_t ck_bytes = 0;
  double *d_ff = nullptr;  // zero-phase filter: the passes' own filter state
  size_t ff_bytes = 0;
  double *d_gpart = nullptr;
  size_t gpart_bytes = 0;
  int adj_windows = 0;  // most adjoint windows per launch (0: no limit)
};

struct filark_stalta_state {
  int device = 0;
  int64_t n_ch = 0;
  int64_t nsta = 0, nlta = 0;
  double *d_state = nullptr;  // [2][n_ch] (sta, lta)
  int64_t *d_cnt = nullptr;   // [n_ch] global sample counter
  Tables fwd;
  Tables adj;
  Tables ckp;
};

struct filark_batch {
  int device = 0;
  std::vector<filark_sos_state *> st;
  std::vector<uint64_t> gen;  // each state's table generation when bound
  int nw = 0;                 // waves per workgroup (the states' common tile)
  FwdParams *d_descs = nullptr;
  size_t descs_bytes = 0;
  BatchItem *d_items = nullptr;
  size_t items_bytes = 0;
  uint32_t *d_heads = nullptr;              // [8] queue counters, [1] workgroups done
  unsigned long long *d_stamps = nullptr;   // [n + 1]
  BatchParams bp{};
  int kmax = 0, grid = 0;
  size_t lds = 0;
  bool bound = false;
  // the launch sequence captured in a graph (filark_batch_capture)
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct filark_ema_state {
  int device = 0;
  int64_t n_ch = 0, n_win = 0;
  int mode = 0;
  double *d_avg = nullptr;   // [n_ch]
  double *d_tab = nullptr;   // decay powers
  int n_lev = 0;
};

struct filark_fir_state {
  int device = 0;
  int64_t n_ch = 0;
  int n_taps = 0, n_pad = 0;      // M and M padded to the tap chunk
  float *d_h = nullptr;           // [n_pad] FP32 taps, zero past M
  float *d_hist[2] = {};          // [max(M - 1, 1)][n_ch] each; d_ctl[0] names the current one
  uint32_t *d_ctl = nullptr;      // [2]: [0] & 1 names the current history buffer; [1]: FFT workgroups done
  int rows = 0, waves = 1;        // output rows per wave (0: by launch), waves per workgroup
  int order = 2;                  // workgroup order: a channel slab per XCD, swept row block by row block
  int method = FILARK_FIR_DIRECT;
  float2 *d_fft = nullptr;        // FFT method: twiddles [2048], then the taps' spectrum [1025]
};

struct filark_trigger_state {
  int device = 0;
  int64_t n_ch = 0;
  float on = 0.f, off = 0.f;
  int32_t *d_open = nullptr;  // [n_ch]
  int64_t *d_ton = nullptr;   // [n_ch]
  int64_t *d_cnt = nullptr;   // [n_ch]
};

namespace {

// Trigger and exponential-average tile: 48-row blocks, 8 waves, groups of
// 16 channels (1536-row windows, so a 1500-row chunk is one launch; 64-byte
// row segments per group; the kernels are compiled for 48-row blocks only).
constexpr int kTrigBlock = 48, kTrigWaves = 8, kTrigGroup = 16;

// Default adjoint tile: 16-sample blocks, 4 waves, groups of 8 channels
// (windows of 512 rows; three workgroups per CU when the section signals are
// rebuilt rather than stored).
Tile default_adj_tile() {
  Tile t;
  t.block = 16;
  t.waves = 4;
  t.group = 8;
  return t;
}

// Tile of the forward pass that writes the adjoint's window checkpoints:
// 64-row blocks, so any adjoint window that is a multiple of 64 rows and
// divides the 2048-row window starts on a block.
Tile checkpoint_tile() {
  Tile t;
  t.block = 64;
  t.waves = 4;
  t.group = 8;
  return t;
}

// Checkpoint emission of a forward launch (FwdParams::ck).
struct CkSpec {
  double *base;     // slot of the checkpoint at the first launch's start
  int64_t stride;   // doubles per slot
  int rows;         // rows between checkpoints (a multiple of the block)
  bool first;       // also write the checkpoint at each launch's start
};

filark_status upload(double **dst, const std::vector<double> &tab, hipStream_t stream) {
  if (*dst) {
    HIP_TRY(hipStreamSynchronize(stream));
    (void)hipFree(*dst);
    *dst = nullptr;
  }
  HIP_TRY(hipMalloc(dst, tab.size() * sizeof(double)));
  HIP_TRY(hipMemcpyAsync(*dst, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return FILARK_OK;
}

filark_status sos_tables(const Cascade &cas, Tables &tb, hipStream_t stream) {
  const int K = cas.K, n = 2 * K, L = tb.tile.block;
  Mat A;
  std::vector<double> B;
  cascade_matrices(cas, A, B);
  std::vector<double> tab;
  for (int k = 0; k < K; ++k) {
    const double *r = cas.c[k];
    tab.insert(tab.end(), {r[0], r[1], r[2], -r[3], -r[4]});
  }
  while (tab.size() % 8) tab.push_back(0.0);
  tb.off_G = tab.size();
  std::vector<std::vector<double>> G(L);
  G[L - 1] = B;
  for (int j = L - 2; j >= 0; --j) G[j] = matvec(A, G[j + 1], n);
  for (int j = 0; j < L; ++j) tab.insert(tab.end(), G[j].begin(), G[j].end());
  while (tab.size() % 8) tab.push_back(0.0);
  tb.off_P = tab.size();
  Mat P = identity(n);
  for (int j = 0; j < L; ++j) P = matmul(A, P, n);
  for (int k = 0; k < tb.tile.levels(); ++k) {
    tab.insert(tab.end(), P.begin(), P.end());
    P = matmul(P, P, n);
  }
  // reciprocals that invert each section's state update (adjoint kernel):
  // 1 / (-a2), or 1 / (-a1) for a first-order section, 0 where undefined
  tb.off_R = tab.size();
  for (int k = 0; k < K; ++k) {
    const double a1 = cas.c[k][3], a2 = cas.c[k][4];
    tab.push_back(a2 != 0.0 ? -1.0 / a2 : (a1 != 0.0 ? -1.0 / a1 : 0.0));
  }
  return upload(&tb.d, tab, stream);
}

filark_status stalta_tables(int64_t nsta, int64_t nlta, Tables &tb, hipStream_t stream) {
  const int L = tb.tile.block;
  const double as = 1.0 - 1.0 / (double)nsta, al = 1.0 - 1.0 / (double)nlta;
  std::vector<double> tab;
  for (int k = 0; k < tb.tile.levels(); ++k) {
    const double e = (double)L * std::ldexp(1.0, k);
    tab.push_back(std::pow(as, e));
    tab.push_back(std::pow(al, e));
  }
  for (int m = 0; m <= L; ++m) {
    tab.push_back(std::pow(as, (double)m));
    tab.push_back(std::pow(al, (double)m));
  }
  return upload(&tb.d, tab, stream);
}

filark_status check_lds(size_t lds, const Tile &t, int K, int dev) {
  int lds_max = 0;
  HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (lds > (size_t)lds_max)
    return fail(FILARK_EINVAL, "tile %dx%dx%d needs %zu bytes of LDS for %d sections (device limit %d)",
                t.block, t.waves, t.group, lds, K, lds_max);
  return FILARK_OK;
}

int log2_exact(int v) {
  int k = 0;
  while ((1 << k) < v) ++k;
  return k;
}

// Rows per launch of a tile, or 0 if a window's padded extent would reach
// 2^31 bytes (byte offsets within a launch are 32-bit).
int64_t launch_rows(const Tile &t, int64_t n_ch) {
  const uint64_t rows = (uint64_t)t.window();
  return rows * (uint64_t)n_ch * 4u > 0x7fffffffull ? 0 : (int64_t)rows;
}

// Forward launches over n_t rows from `in`, one window each, with the state
// at (zs, sl, cnt) updated in place.  y / cf may be null; with neither (and
// `states_only`) nothing but the state is written.
// Parameters common to every window of a forward launch sequence (pointers
// and the window's row count are set per window).
FwdParams fwd_base(const filark_sos_state *sos, const filark_stalta_state *sl, const Tile &t, double *zs,
                   double *slst, int64_t *cnt, int64_t n_ch, bool ckp_tables) {
  FwdParams p;
  std::memset(&p, 0, sizeof p);
  p.n_ch = n_ch;
  p.cw_log2 = log2_exact(t.group);
  p.nw = t.waves;
  p.n_grp = (int)((n_ch + t.group - 1) / t.group);
  p.per_xcd = per_xcd_for(p.n_grp);
  p.n_lev = t.levels();
  p.nt = t.group >= 16 ? 1 : 0;
  p.order = t.group >= 16 ? 1 : 0;
  if (sos) {
    const Tables &tb = ckp_tables ? sos->ckp : sos->fwd;
    p.zs = zs;
    p.coef = tb.d;
    p.G = tb.d + tb.off_G;
    p.Pw = tb.d + tb.off_P;
  }
  if (sl) {
    p.sl = slst;
    p.cnt = cnt;
    p.dpow = (ckp_tables ? sl->ckp : sl->fwd).d;
    p.nlta = sl->nlta;
    p.nsta_d = (double)sl->nsta;
    p.nlta_d = (double)sl->nlta;
    p.asd = 1.0 - 1.0 / (double)sl->nsta;
    p.ald = 1.0 - 1.0 / (double)sl->nlta;
    p.as = (float)p.asd;
    p.al = (float)p.ald;
    p.kappa = (float)((double)sl->nlta / (double)sl->nsta);
  }
  return p;
}

hipError_t forward_launches(const filark_sos_state *sos, const filark_stalta_state *sl, const Tile &t,
                            double *zs, double *slst, int64_t *cnt, const float *in, float *y, float *cf,
                            bool states_only, int64_t n_ch, int64_t n_t, hipStream_t stream,
                            bool rev = false, const CkSpec *ck = nullptr, bool ckp_tables = false) {
  const uint64_t rowb = (uint64_t)n_ch * 4u;
  const int64_t rows = launch_rows(t, n_ch);
  const int K = sos ? sos->cas.K : 0;
  FwdParams p = fwd_base(sos, sl, t, zs, slst, cnt, n_ch, ckp_tables);
  hipError_t e = hipSuccess;
  // time-reversed: the windows last to first, each one's rows last to first
  const int64_t n_win = (n_t + rows - 1) / rows;
  for (int64_t k = 0; k < n_win && e == hipSuccess; ++k) {
    const int64_t t0 = (rev ? n_win - 1 - k : k) * rows;
    const int64_t nt = std::min(rows, n_t - t0);
    const size_t off = (size_t)t0 * (size_t)n_ch;
    p.x = in + off;
    p.y = y ? y + off : nullptr;
    p.cf = cf ? cf + off : nullptr;
    p.n_t = (int32_t)nt;
    p.range = (int32_t)((uint64_t)nt * rowb);
    p.out_range = states_only ? 0 : p.range;
    if (ck) {
      p.ck = ck->base + (t0 / ck->rows) * ck->stride;
      p.ck_stride = ck->stride;
      p.ck_blocks = ck->rows / t.block;
      p.ck_first = ck->first ? 1 : 0;
    }
    e = launch_fwd(p, K, t.block, sl != nullptr, !states_only && (sl == nullptr || y != nullptr),
                   sos != nullptr && sos->cas.unit_tail(), rev, stream);
  }
  return e;
}

// Shared launch path of the three processing entry points.
filark_status run_forward(filark_sos_state *sos, filark_stalta_state *sl, const float *in,
                          float *y, float *cf, int64_t n_ch, int64_t n_t, hipStream_t stream) {
  if (n_t < 0) return fail(FILARK_EINVAL, "n_t out of range: %lld", (long long)n_t);
  if (n_ch < 1) return fail(FILARK_EINVAL, "n_ch must be >= 1");
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
  const Tile t = sos ? sos->fwd.tile : sl->fwd.tile;
  if (sos && sl && !(sos->fwd.tile == sl->fwd.tile))
    return fail(FILARK_EINVAL, "tile shapes of the states differ (set both with filark_tile_set)");
  if (launch_rows(t, n_ch) == 0)
    return fail(FILARK_EINVAL, "n_ch %lld too large for a %d-row window (at most %lld channels)",
                (long long)n_ch, t.window(), (long long)(0x7fffffffull / (uint64_t)t.window() / 4u));
  const int K = sos ? sos->cas.K : 0;
  const int dev = sos ? sos->device : sl->device;
  filark_status rc = check_lds(fwd_lds_bytes(K, t.waves, t.levels(), t.group), t, K, dev);
  if (rc != FILARK_OK) return rc;
  const int prev_dev = current_device();
  if (prev_dev != dev) HIP_TRY(hipSetDevice(dev));
  hipError_t e = forward_launches(sos, sl, t, sos ? sos->d_state : nullptr, sl ? sl->d_state : nullptr,
                                  sl ? sl->d_cnt : nullptr, in, y, cf, false, n_ch, n_t, stream);
  if (prev_dev != dev) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) return fail(FILARK_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

filark_status grow(double **buf, size_t *have, size_t need, hipStream_t stream) {
  if (*buf && *have >= need) return FILARK_OK;
  HIP_TRY(hipStreamSynchronize(stream));
  if (*buf) (void)hipFree(*buf);
  *buf = nullptr;
  *have = 0;
  HIP_TRY(hipMalloc(buf, need));
  HIP_TRY(hipMemsetAsync(*buf, 0, need, stream));
  *have = need;
  return FILARK_OK;
}

template <class T>
filark_status grow_raw(T **buf, size_t *have, size_t need) {
  if (*buf && *have >= need) return FILARK_OK;
  if (*buf) (void)hipFree(*buf);
  *buf = nullptr;
  *have = 0;
  HIP_TRY(hipMalloc(reinterpret_cast<void **>(buf), std::max<size_t>(need, 256)));
  *have = std::max<size_t>(need, 256);
  return FILARK_OK;
}

filark_status check_tile(int block, int waves, int group, bool adjoint) {
  if (adjoint ? (block != 8 && block != 16) : (block != 32 && block != 48 && block != 64))
    return fail(FILARK_EINVAL, adjoint ? "adjoint block must be 8 or 16" : "block must be 32, 48 or 64");
  if (waves < 1 || waves > kMaxWaves) return fail(FILARK_EINVAL, "waves must be in [1, %d]", kMaxWaves);
  if (group != 4 && group != 8 && group != 16 && group != 32 && group != 64)
    return fail(FILARK_EINVAL, "group must be 4, 8, 16, 32 or 64 channels");
  return FILARK_OK;
}

// Scratch of the allocation-free zero-phase entry point: the two passes' own
// FP64 filter state [2K][n_ch], at most 1 MiB (2 * sections * channels <=
// 131072).  Each GPU the library runs on holds its own copy until the
// process ends; every call on one GPU shares it, so calls that overlap on a
// GPU race.  In host code `scratch` is only a stand-in for the symbol: the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current, and is the only form passed to
// kernels.
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) double scratch[131072];
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxScratchDevices] = {};

// The device address of `dev`'s scratch (dev must be current).
filark_status scratch_on(int dev, double **out) {
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(FILARK_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FILARK_EHIP, "scratch address on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return FILARK_OK;
}

// Zero n doubles (a fill kernel rather than hipMemsetAsync, so a captured
// graph replays it correctly).
__global__ void __launch_bounds__(256) fill_zero_kernel(double *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t fill_zero(double *p, size_t n, hipStream_t stream) {
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

filark_status filtfilt_check(const filark_sos_state *sos, const float *in, const float *out, int64_t n_ch,
                             int64_t n_t) {
  if (!sos) return fail(FILARK_EINVAL, "null state");
  if (n_t < 0) return fail(FILARK_EINVAL, "n_t out of range: %lld", (long long)n_t);
  if (n_ch != sos->n_ch)
    return fail(FILARK_ESHAPE, "n_ch %lld differs from the SOS state's %lld", (long long)n_ch, (long long)sos->n_ch);
  if (n_t == 0) return FILARK_OK;
  if (!in || !out) return fail(FILARK_EINVAL, "null input or output pointer");
  const Tile &t = sos->fwd.tile;
  if (t.block != 48) return fail(FILARK_EINVAL, "zero-phase filtering runs on 48-sample blocks (the default tile)");
  if (launch_rows(t, n_ch) == 0) return fail(FILARK_EINVAL, "n_ch %lld too large for the tile", (long long)n_ch);
  const int K = sos->cas.K;
  return check_lds(fwd_lds_bytes(K, t.waves, t.levels(), t.group), t, K, sos->device);
}

// Forward pass from rest, then the time-reversed pass over its output from
// rest (in place), with `work` [2K][n_ch] as the passes' filter state; the
// object's carried state is not touched.
hipError_t filtfilt_launches(const filark_sos_state *sos, const float *in, float *out, int64_t n_ch, int64_t n_t,
                             double *work, hipStream_t stream) {
  const Tile &t = sos->fwd.tile;
  const size_t n = (size_t)(2 * sos->cas.K) * (size_t)n_ch;
  hipError_t e = fill_zero(work, n, stream);
  if (e == hipSuccess)
    e = forward_launches(sos, nullptr, t, work, nullptr, nullptr, in, out, nullptr, false, n_ch, n_t, stream);
  if (e == hipSuccess) e = fill_zero(work, n, stream);
  if (e == hipSuccess)
    e = forward_launches(sos, nullptr, t, work, nullptr, nullptr, out, out, nullptr, false, n_ch, n_t, stream, true);
  return e;
}

void drop_graph(filark_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

}  // namespace

extern "C" {

const char *filark_last_error(void) { return g_err.c_str(); }

const char *filark_version(void) { return "filark-mi355x 0.3 (gfx950)"; }

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
  const size_t bytes = (size_t)(2 * n_sec) * (size_t)n_ch * sizeof(double);
  filark_status rc = FILARK_OK;
  hipError_t e = hipMalloc(&st->d_state, bytes);
  if (e == hipSuccess) e = hipMemsetAsync(st->d_state, 0, bytes, stream);
  if (e != hipSuccess) rc = fail(FILARK_EHIP, "state allocation: %s", hipGetErrorString(e));
  st->adj.tile = default_adj_tile();
  st->ckp.tile = checkpoint_tile();
  if (rc == FILARK_OK) rc = sos_tables(st->cas, st->fwd, stream);
  if (rc == FILARK_OK) rc = sos_tables(st->cas, st->adj, stream);
  if (rc == FILARK_OK) rc = sos_tables(st->cas, st->ckp, stream);
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
  if (ns < 1.0 || nl < 1.0 || ns > 9.0e15 || nl > 9.0e15)
    return fail(FILARK_EINVAL, "window lengths must round to 1 .. 9e15 samples");
  if (n_ch < 1 || n_ch > (int64_t)1 << 24) return fail(FILARK_EINVAL, "n_ch must be in [1, 2^24]");
  filark_stalta_state *st = new (std::nothrow) filark_stalta_state();
  if (!st) return fail(FILARK_ENOMEM, "host allocation failed");
  st->device = current_device();
  st->n_ch = n_ch;
  st->nsta = (int64_t)ns;
  st->nlta = (int64_t)nl;
  // (sta, lta) [2][n_ch] and the counter [n_ch] in one allocation, so a
  // device checkpoint of the whole state is one copy
  const size_t bytes = (size_t)n_ch * (2 * sizeof(double) + sizeof(int64_t));
  filark_status rc = FILARK_OK;
  hipError_t e = hipMalloc(&st->d_state, bytes);
  if (e == hipSuccess) e = hipMemsetAsync(st->d_state, 0, bytes, stream);
  if (e == hipSuccess) st->d_cnt = reinterpret_cast<int64_t *>(st->d_state + 2 * (size_t)n_ch);
  if (e != hipSuccess) rc = fail(FILARK_EHIP, "state allocation: %s", hipGetErrorString(e));
  st->adj.tile = default_adj_tile();
  st->ckp.tile = checkpoint_tile();
  if (rc == FILARK_OK) rc = stalta_tables(st->nsta, st->nlta, st->fwd, stream);
  if (rc == FILARK_OK) rc = stalta_tables(st->nsta, st->nlta, st->adj, stream);
  if (rc == FILARK_OK) rc = stalta_tables(st->nsta, st->nlta, st->ckp, stream);
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

filark_status filark_sos_filtfilt(filark_sos_t sos, const float *in, float *out, int64_t n_ch, int64_t n_t,
                                  hipStream_t stream) {
  filark_status rc = filtfilt_check(sos, in, out, n_ch, n_t);
  if (rc != FILARK_OK || n_t == 0) return rc;
  const int prev_dev = current_device();
  if (prev_dev != sos->device) HIP_TRY(hipSetDevice(sos->device));
  const size_t bytes = (size_t)(2 * sos->cas.K) * (size_t)n_ch * sizeof(double);
  rc = grow(&sos->d_ff, &sos->ff_bytes, bytes, stream);
  hipError_t e = hipSuccess;
  if (rc == FILARK_OK) e = filtfilt_launches(sos, in, out, n_ch, n_t, sos->d_ff, stream);
  if (prev_dev != sos->device) (void)hipSetDevice(prev_dev);
  if (rc != FILARK_OK) return rc;
  if (e != hipSuccess) return fail(FILARK_EHIP, "zero-phase launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

filark_status filark_sos_filtfilt_noalloc(filark_sos_t sos, const float *in, float *out, int64_t n_ch, int64_t n_t,
                                          hipStream_t stream) {
  filark_status rc = filtfilt_check(sos, in, out, n_ch, n_t);
  if (rc != FILARK_OK || n_t == 0) return rc;
  const size_t bytes = (size_t)(2 * sos->cas.K) * (size_t)n_ch * sizeof(double);
  if (bytes > sizeof(scratch))
    return fail(FILARK_EINVAL, "the work state of %d sections x %lld channels needs %zu bytes; the allocation-free "
                "entry point holds at most %zu (2 * sections * channels <= %zu)", sos->cas.K, (long long)n_ch,
                bytes, sizeof(scratch), sizeof(scratch) / sizeof(double));
  const int prev_dev = current_device();
  if (prev_dev != sos->device) HIP_TRY(hipSetDevice(sos->device));
  double *work = nullptr;
  rc = scratch_on(sos->device, &work);
  hipError_t e = hipSuccess;
  if (rc == FILARK_OK) e = filtfilt_launches(sos, in, out, n_ch, n_t, work, stream);
  if (prev_dev != sos->device) (void)hipSetDevice(prev_dev);
  if (rc != FILARK_OK) return rc;
  if (e != hipSuccess) return fail(FILARK_EHIP, "zero-phase launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
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
  if (kind == FILARK_STATE_SOS) {
    const filark_sos_state *st = static_cast<const filark_sos_state *>(obj);
    const int n = 2 * st->cas.K;
    const size_t need = (size_t)st->n_ch * n * sizeof(double);
    if (bytes != need) return fail(FILARK_EINVAL, "state_get: need %zu bytes, got %zu", need, bytes);
    HIP_TRY(hipStreamSynchronize(stream));
    std::vector<double> tmp((size_t)n * st->n_ch);
    HIP_TRY(hipMemcpy(tmp.data(), st->d_state, tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
    double *o = static_cast<double *>(host_buf);
    for (int64_t c = 0; c < st->n_ch; ++c)
      for (int i = 0; i < n; ++i) o[c * n + i] = tmp[(size_t)i * st->n_ch + c];
    return FILARK_OK;
  }
  if (kind == FILARK_STATE_STALTA) {
    const filark_stalta_state *st = static_cast<const filark_stalta_state *>(obj);
    const size_t need = (size_t)st->n_ch * 2 * sizeof(double) + sizeof(int64_t);
    if (bytes != need) return fail(FILARK_EINVAL, "state_get: need %zu bytes, got %zu", need, bytes);
    HIP_TRY(hipStreamSynchronize(stream));
    std::vector<double> tmp(2 * (size_t)st->n_ch);
    HIP_TRY(hipMemcpy(tmp.data(), st->d_state, tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
    int64_t g = 0;
    HIP_TRY(hipMemcpy(&g, st->d_cnt, sizeof g, hipMemcpyDeviceToHost));
    double *o = static_cast<double *>(host_buf);
    for (int64_t c = 0; c < st->n_ch; ++c) {
      o[2 * c] = tmp[c];
      o[2 * c + 1] = tmp[st->n_ch + c];
    }
    std::memcpy(o + 2 * st->n_ch, &g, sizeof g);
    return FILARK_OK;
  }
  return fail(FILARK_EINVAL, "unknown state kind %d", kind);
}

filark_status filark_state_set(void *obj, int kind, const void *host_buf, size_t bytes,
                               hipStream_t stream) {
  if (!obj || !host_buf) return fail(FILARK_EINVAL, "null pointer");
  if (kind == FILARK_STATE_SOS) {
    filark_sos_state *st = static_cast<filark_sos_state *>(obj);
    const int n = 2 * st->cas.K;
    const size_t need = (size_t)st->n_ch * n * sizeof(double);
    if (bytes != need) return fail(FILARK_EINVAL, "state_set: need %zu bytes, got %zu", need, bytes);
    const double *src = static_cast<const double *>(host_buf);
    for (size_t i = 0; i < (size_t)st->n_ch * n; ++i)
      if (!std::isfinite(src[i])) return fail(FILARK_EINVAL, "state_set: non-finite value");
    std::vector<double> tmp((size_t)n * st->n_ch);
    for (int64_t c = 0; c < st->n_ch; ++c)
      for (int i = 0; i < n; ++i) tmp[(size_t)i * st->n_ch + c] = src[c * n + i];
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipMemcpy(st->d_state, tmp.data(), tmp.size() * sizeof(double), hipMemcpyHostToDevice));
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
    std::vector<double> tmp(2 * (size_t)st->n_ch);
    for (int64_t c = 0; c < st->n_ch; ++c) {
      tmp[c] = src[2 * c];
      tmp[st->n_ch + c] = src[2 * c + 1];
    }
    const std::vector<int64_t> gv((size_t)st->n_ch, g);
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipMemcpy(st->d_state, tmp.data(), tmp.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(st->d_cnt, gv.data(), gv.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    return FILARK_OK;
  }
  return fail(FILARK_EINVAL, "unknown state kind %d", kind);
}

filark_status filark_tile_set(void *obj, int kind, int block, int waves, int group, hipStream_t stream) {
  if (!obj) return fail(FILARK_EINVAL, "null state");
  const bool adjoint = kind == FILARK_TILE_SOS_ADJOINT || kind == FILARK_TILE_STALTA_ADJOINT;
  filark_status rc = check_tile(block, waves, group, adjoint);
  if (rc != FILARK_OK) return rc;
  Tile t;
  t.block = block;
  t.waves = waves;
  t.group = group;
  if (kind == FILARK_STATE_SOS || kind == FILARK_TILE_SOS_ADJOINT) {
    filark_sos_state *st = static_cast<filark_sos_state *>(obj);
    Tables &tb = adjoint ? st->adj : st->fwd;
    if (tb.tile == t) return FILARK_OK;
    HIP_TRY(hipStreamSynchronize(stream));
    tb.tile = t;
    if (!adjoint) ++st->gen;  // batches bound to this state must be bound again
    return sos_tables(st->cas, tb, stream);
  }
  if (kind == FILARK_STATE_STALTA || kind == FILARK_TILE_STALTA_ADJOINT) {
    filark_stalta_state *st = static_cast<filark_stalta_state *>(obj);
    Tables &tb = adjoint ? st->adj : st->fwd;
    if (tb.tile == t) return FILARK_OK;
    HIP_TRY(hipStreamSynchronize(stream));
    tb.tile = t;
    return stalta_tables(st->nsta, st->nlta, tb, stream);
  }
  return fail(FILARK_EINVAL, "unknown state kind %d", kind);
}

filark_status filark_tile_get(const void *obj, int kind, int *block, int *waves, int *group) {
  if (!obj || !block || !waves || !group) return fail(FILARK_EINVAL, "null pointer");
  Tile t;
  if (kind == FILARK_STATE_SOS) t = static_cast<const filark_sos_state *>(obj)->fwd.tile;
  else if (kind == FILARK_STATE_STALTA) t = static_cast<const filark_stalta_state *>(obj)->fwd.tile;
  else if (kind == FILARK_TILE_SOS_ADJOINT) t = static_cast<const filark_sos_state *>(obj)->adj.tile;
  else if (kind == FILARK_TILE_STALTA_ADJOINT) t = static_cast<const filark_stalta_state *>(obj)->adj.tile;
  else return fail(FILARK_EINVAL, "unknown state kind %d", kind);
  *block = t.block;
  *waves = t.waves;
  *group = t.group;
  return FILARK_OK;
}

filark_status filark_adjoint_windows_set(filark_sos_t sos, int max_windows) {
  if (!sos) return fail(FILARK_EINVAL, "null state");
  if (max_windows < 0) return fail(FILARK_EINVAL, "max_windows must be >= 0, got %d", max_windows);
  sos->adj_windows = max_windows;
  return FILARK_OK;
}

filark_status filark_state_bytes(const void *obj, int kind, size_t *bytes) {
  if (!obj || !bytes) return fail(FILARK_EINVAL, "null pointer");
  if (kind == FILARK_STATE_SOS) {
    const filark_sos_state *st = static_cast<const filark_sos_state *>(obj);
    *bytes = (size_t)(2 * st->cas.K) * (size_t)st->n_ch * sizeof(double);
    return FILARK_OK;
  }
  if (kind == FILARK_STATE_STALTA) {
    const filark_stalta_state *st = static_cast<const filark_stalta_state *>(obj);
    *bytes = (size_t)st->n_ch * (2 * sizeof(double) + sizeof(int64_t));
    return FILARK_OK;
  }
  return fail(FILARK_EINVAL, "unknown state kind %d", kind);
}

filark_status filark_state_save(const void *obj, int kind, void *dev_dst, hipStream_t stream) {
  if (!obj || !dev_dst) return fail(FILARK_EINVAL, "null pointer");
  if (kind == FILARK_STATE_SOS) {
    const filark_sos_state *st = static_cast<const filark_sos_state *>(obj);
    HIP_TRY(hipMemcpyAsync(dev_dst, st->d_state, (size_t)(2 * st->cas.K) * st->n_ch * sizeof(double),
                           hipMemcpyDeviceToDevice, stream));
    return FILARK_OK;
  }
  if (kind == FILARK_STATE_STALTA) {
    const filark_stalta_state *st = static_cast<const filark_stalta_state *>(obj);
    HIP_TRY(hipMemcpyAsync(dev_dst, st->d_state, (size_t)st->n_ch * (2 * sizeof(double) + sizeof(int64_t)),
                           hipMemcpyDeviceToDevice, stream));
    return FILARK_OK;
  }
  return fail(FILARK_EINVAL, "unknown state kind %d", kind);
}

filark_status filark_state_load(void *obj, int kind, const void *dev_src, hipStream_t stream) {
  if (!obj || !dev_src) return fail(FILARK_EINVAL, "null pointer");
  if (kind == FILARK_STATE_SOS) {
    filark_sos_state *st = static_cast<filark_sos_state *>(obj);
    HIP_TRY(hipMemcpyAsync(st->d_state, dev_src, (size_t)(2 * st->cas.K) * st->n_ch * sizeof(double),
                           hipMemcpyDeviceToDevice, stream));
    return FILARK_OK;
  }
  if (kind == FILARK_STATE_STALTA) {
    filark_stalta_state *st = static_cast<filark_stalta_state *>(obj);
    HIP_TRY(hipMemcpyAsync(st->d_state, dev_src, (size_t)st->n_ch * (2 * sizeof(double) + sizeof(int64_t)),
                           hipMemcpyDeviceToDevice, stream));
    return FILARK_OK;
  }
  return fail(FILARK_EINVAL, "unknown state kind %d", kind);
}

namespace {

// Rows of an adjoint window and doubles of one checkpoint slot (filter state
// [2K][n_ch], STA/LTA state [2][n_ch], counter [n_ch] in a double slot).
int64_t adjoint_rows(const filark_sos_state *sos, int64_t n_ch) { return launch_rows(sos->adj.tile, n_ch); }
size_t ck_slot_doubles(const filark_sos_state *sos, int64_t n_ch) {
  return (size_t)(2 * sos->cas.K + 3) * (size_t)n_ch;
}

// A tape's forward: the checkpoint tile (64-row blocks, so that every
// adjoint window start that is a multiple of 64 rows falls on a block start;
// 4 waves and groups of 8 channels, so that with the 64-row kernel's
// registers every workgroup of a 6000-channel chunk is resident at once).
Tile tape_tile(const filark_sos_state *sos, int64_t) { return sos->ckp.tile; }

// Bytes of the tape of a chunk of n_t rows: one slot per adjoint window.
size_t tape_need(const filark_sos_state *sos, int64_t n_ch, int64_t n_t) {
  const int64_t rows = adjoint_rows(sos, n_ch);
  return rows > 0 ? (size_t)((n_t + rows - 1) / rows) * ck_slot_doubles(sos, n_ch) * sizeof(double) : 0;
}

// Why a tape cannot be used with these objects and this channel count, or null.
const char *tape_unusable(const filark_sos_state *sos, const filark_stalta_state *sl, int64_t n_ch) {
  const Tile tt = tape_tile(sos, n_ch);
  const int64_t rows = adjoint_rows(sos, n_ch);
  if (!(sl->ckp.tile == sos->ckp.tile)) return "the states' checkpoint tiles differ";
  if (!(sos->adj.tile == sl->adj.tile)) return "the adjoint tile shapes of the states differ";
  if (rows == 0 || launch_rows(tt, n_ch) == 0) return "too many channels for the tape's windows";
  if (rows % tt.block != 0 || tt.window() % rows != 0)
    return "the adjoint window must be a multiple of 64 rows that divides 2048";
  return nullptr;
}

filark_status adjoint_run(filark_sos_t sos, filark_stalta_t sl, const double *tape, const float *x,
                          const float *g, int mode, double scale, float *gx, double *adj, double *gsos,
                          int64_t n_ch, int64_t n_t, hipStream_t stream) {
  if (!sos || !sl) return fail(FILARK_EINVAL, "null state");
  if (sos->device != sl->device) return fail(FILARK_EINVAL, "states live on different devices");
  if (sos->n_ch != n_ch || sl->n_ch != n_ch) return fail(FILARK_ESHAPE, "n_ch differs from the states'");
  if (n_t < 0) return fail(FILARK_EINVAL, "n_t out of range: %lld", (long long)n_t);
  if (mode != FILARK_ADJ_GRAD && mode != FILARK_ADJ_MSE) return fail(FILARK_EINVAL, "unknown mode %d", mode);
  if (!std::isfinite(scale)) return fail(FILARK_EINVAL, "scale must be finite");
  if (n_t == 0) return FILARK_OK;
  if (!x || !g || !gx || !adj || !gsos) return fail(FILARK_EINVAL, "null pointer");
  if (!(sos->adj.tile == sl->adj.tile))
    return fail(FILARK_EINVAL, "adjoint tile shapes of the states differ");
  if (!(sos->fwd.tile == sl->fwd.tile))
    return fail(FILARK_EINVAL, "tile shapes of the states differ (set both with filark_tile_set)");
  const Tile ta = sos->adj.tile, tf = sos->fwd.tile;
  const int K = sos->cas.K;
  const int64_t rows = launch_rows(ta, n_ch);
  if (rows == 0 || launch_rows(tf, n_ch) == 0) return fail(FILARK_EINVAL, "n_ch %lld too large", (long long)n_ch);
  filark_status rc = check_lds(adj_lds_bytes(K, ta.waves, ta.levels()), ta, K, sos->device);
  if (rc == FILARK_OK) rc = check_lds(fwd_lds_bytes(K, tf.waves, tf.levels(), tf.group), tf, K, sos->device);
  if (rc != FILARK_OK) return rc;
  const int prev_dev = current_device();
  if (prev_dev != sos->device) HIP_TRY(hipSetDevice(sos->device));

  // workspace: forward state at every window start after the first (filter
  // [2K][n_ch], STA/LTA [2][n_ch], counter [n_ch]; the tape's slots instead
  // when there is one), per-group coefficient sums
  const int64_t n_win = (n_t + rows - 1) / rows;
  const size_t ck_doubles = ck_slot_doubles(sos, n_ch);
  const int n_grp = (int)((n_ch + ta.group - 1) / ta.group);
  rc = FILARK_OK;
  if (!tape) rc = grow(&sos->d_ck, &sos->ck_bytes, (size_t)n_win * ck_doubles * sizeof(double), stream);
  if (rc == FILARK_OK) rc = grow(&sos->d_gpart, &sos->gpart_bytes, (size_t)n_grp * 5 * K * sizeof(double), stream);
  if (rc != FILARK_OK) {
    if (prev_dev != sos->device) (void)hipSetDevice(prev_dev);
    return rc;
  }
  auto ck_z = [&](int64_t w) { return sos->d_ck + (size_t)w * ck_doubles; };
  auto ck_s = [&](int64_t w) { return ck_z(w) + (size_t)(2 * K) * n_ch; };
  auto ck_c = [&](int64_t w) { return reinterpret_cast<int64_t *>(ck_s(w) + 2 * (size_t)n_ch); };
  // window 0 starts from the objects' own state; slot w > 0 of the
  // workspace holds the state at the start of window w.  A forward pass runs
  // in place on the slot of its END (seeded with its start state), so the
  // slot of its start stays intact.
  const size_t z_bytes = (size_t)(2 * K) * n_ch * sizeof(double);
  const size_t s_bytes = (size_t)n_ch * (2 * sizeof(double) + sizeof(int64_t));  // (sta, lta) then the counter
  auto seed = [&](int64_t to, int64_t from) -> hipError_t {
    if (from == 0) {
      hipError_t r = hipMemcpyAsync(ck_z(to), sos->d_state, z_bytes, hipMemcpyDeviceToDevice, stream);
      if (r == hipSuccess) r = hipMemcpyAsync(ck_s(to), sl->d_state, s_bytes, hipMemcpyDeviceToDevice, stream);
      return r;
    }
    return hipMemcpyAsync(ck_z(to), ck_z(from), ck_doubles * sizeof(double), hipMemcpyDeviceToDevice, stream);
  };
  hipError_t e = hipSuccess;
  // forward states at the window starts: one states-only pass over the rows
  // before the last window, with 64-row blocks, writes them as it goes
  // (windows that are a multiple of 64 rows and divide its 2048-row window);
  // otherwise one states-only launch per window
  const Tile tck = sos->ckp.tile;
  const int64_t ck_win = tck.window();
  const bool one_pass = rows % tck.block == 0 && ck_win % rows == 0 && launch_rows(tck, n_ch) != 0 &&
                        sl->ckp.tile == tck &&
                        check_lds(fwd_lds_bytes(K, tck.waves, tck.levels(), tck.group), tck, K, sos->device) ==
                            FILARK_OK;
  if (tape) {
    // the tape holds every window's start state
  } else if (one_pass) {
    const int64_t r_end = (n_win - 1) * rows;
    for (int64_t t0 = 0; t0 < r_end && e == hipSuccess; t0 += ck_win) {
      const int64_t nt = std::min(ck_win, r_end - t0);
      const int64_t w0 = t0 / rows, w1 = (t0 + nt) / rows;
      e = seed(w1, w0);
      const CkSpec cks{ck_z(w0), (int64_t)ck_doubles, (int)rows, false};
      if (e == hipSuccess)
        e = forward_launches(sos, sl, tck, ck_z(w1), ck_s(w1), ck_c(w1), x + (size_t)t0 * n_ch, nullptr, nullptr,
                             true, n_ch, nt, stream, false, &cks, true);
    }
  } else {
    for (int64_t w = 0; w + 1 < n_win && e == hipSuccess; ++w) {
      e = seed(w + 1, w);
      if (e == hipSuccess)
        e = forward_launches(sos, sl, tf, ck_z(w + 1), ck_s(w + 1), ck_c(w + 1), x + (size_t)(w * rows) * n_ch,
                             nullptr, nullptr, true, n_ch, rows, stream);
    }
  }
  // windows last to first
  AdjParams p;
  std::memset(&p, 0, sizeof p);
  p.g = g;
  p.n_ch = n_ch;
  p.cw_log2 = log2_exact(ta.group);
  p.nw = ta.waves;
  p.n_grp = n_grp;
  p.per_xcd = per_xcd_for(n_grp);
  p.n_lev = ta.levels();
  p.mode = mode;
  p.scale = scale;
  p.adj = adj;
  p.gpart = sos->d_gpart;
  p.coef = sos->adj.d;
  p.G = sos->adj.d + sos->adj.off_G;
  p.Pw = sos->adj.d + sos->adj.off_P;
  p.rinv = sos->adj.d + sos->adj.off_R;
  p.first_order = sos->cas.first_order_bits();
  p.recon = sos->cas.invertible() ? (p.first_order ? 2 : 1) : 0;
  p.dpow = sl->adj.d;
  p.cs = 1.0 / (double)sl->nsta;
  p.cl = 1.0 / (double)sl->nlta;
  p.asd = 1.0 - p.cs;
  p.ald = 1.0 - p.cl;
  p.nlta = sl->nlta;
  const uint64_t rowb = (uint64_t)n_ch * 4u;
  // The windows of a chunk run several to a launch where the tile and the
  // cascade allow (the default adjoint tile on a Butterworth-shaped
  // cascade): the adjoint state then passes between them on chip.  The window starts are
  // addressed as evenly spaced slots, so on the checkpoint path slot 0 gets
  // a copy of the objects' state.
  const bool multi = adj_multi_fits(ta.waves, ta.group, ta.block, ta.levels()) && K >= 2 && K <= kMultiMaxSections &&
                     sos->cas.unit_tail() && p.recon == 1 && sos->adj_windows != 1;
  const int64_t cap = sos->adj_windows > 0 ? sos->adj_windows : n_win;
  if (multi && !tape && e == hipSuccess && n_win > 1) e = seed(0, 0);
  p.win_elems = rows * n_ch;
  p.ck_stride = (int64_t)ck_doubles;
  for (int64_t w = n_win - 1; w >= 0 && e == hipSuccess;) {
    const int64_t nt = std::min(rows, n_t - w * rows);
    // windows w_lo .. w in this launch, last to first; only the chunk's last
    // window (w, taken first) may be partial
    const int64_t w_lo = multi ? std::max<int64_t>(0, w - cap + 1) : w;
    const size_t off = (size_t)(w_lo * rows) * (size_t)n_ch;
    p.x = x + off;
    p.g = g + off;
    p.gx = gx + off;
    p.n_win = (int32_t)(w - w_lo + 1);
    p.n_t = (int32_t)(p.n_win > 1 ? rows : nt);
    p.range = (int32_t)((uint64_t)p.n_t * rowb);
    p.n_t_last = (int32_t)nt;
    p.range_last = (int32_t)((uint64_t)nt * rowb);
    if (tape) {
      const double *slot = tape + (size_t)w_lo * ck_doubles;
      p.zs0 = slot;
      p.sl0 = slot + (size_t)(2 * K) * n_ch;
      p.cnt0 = reinterpret_cast<const int64_t *>(slot + (size_t)(2 * K + 2) * n_ch);
    } else if (p.n_win > 1 || w_lo > 0) {
      p.zs0 = ck_z(w_lo);
      p.sl0 = ck_s(w_lo);
      p.cnt0 = ck_c(w_lo);
    } else {
      p.zs0 = sos->d_state;
      p.sl0 = sl->d_state;
      p.cnt0 = sl->d_cnt;
    }
    e = launch_adj(p, K, ta.block, sos->cas.unit_tail(), stream);
    w = w_lo - 1;
  }
  if (e == hipSuccess) e = launch_adj_reduce(sos->d_gpart, n_grp, 5 * K, gsos, stream);
  if (prev_dev != sos->device) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) return fail(FILARK_EHIP, "adjoint launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

}  // namespace

filark_status filark_sos_stalta_adjoint(filark_sos_t sos, filark_stalta_t sl, const float *x,
                                        const float *g, int mode, double scale, float *gx, double *adj,
                                        double *gsos, int64_t n_ch, int64_t n_t, hipStream_t stream) {
  return adjoint_run(sos, sl, nullptr, x, g, mode, scale, gx, adj, gsos, n_ch, n_t, stream);
}

filark_status filark_adjoint_tape_bytes(filark_sos_t sos, filark_stalta_t sl, int64_t n_t, size_t *bytes) {
  if (!sos || !sl || !bytes) return fail(FILARK_EINVAL, "null pointer");
  if (n_t < 0) return fail(FILARK_EINVAL, "n_t out of range: %lld", (long long)n_t);
  if (sos->n_ch != sl->n_ch) return fail(FILARK_ESHAPE, "the states' channel counts differ");
  const char *why = tape_unusable(sos, sl, sos->n_ch);
  if (why) return fail(FILARK_EINVAL, "no tape: %s", why);
  *bytes = tape_need(sos, sos->n_ch, n_t);
  return FILARK_OK;
}

filark_status filark_sos_stalta_process_tape(filark_sos_t sos, filark_stalta_t sl, const float *x, float *y,
                                             float *cf, void *tape, size_t tape_bytes, int64_t n_ch, int64_t n_t,
                                             hipStream_t stream) {
  if (!sos || !sl) return fail(FILARK_EINVAL, "null state");
  if (sos->device != sl->device) return fail(FILARK_EINVAL, "states live on different devices");
  if (sos->n_ch != n_ch || sl->n_ch != n_ch) return fail(FILARK_ESHAPE, "n_ch differs from the states'");
  if (n_t < 0) return fail(FILARK_EINVAL, "n_t out of range: %lld", (long long)n_t);
  if (n_t == 0) return FILARK_OK;
  if (!x || !cf || !tape) return fail(FILARK_EINVAL, "null pointer");
  if (y && (const void *)y == (const void *)cf) return fail(FILARK_EINVAL, "y and cf must differ");
  const char *why = tape_unusable(sos, sl, n_ch);
  if (why) return fail(FILARK_EINVAL, "no tape: %s", why);
  const size_t need = tape_need(sos, n_ch, n_t);
  if (tape_bytes < need) return fail(FILARK_EINVAL, "tape of %zu bytes, %zu needed", tape_bytes, need);
  const Tile tt = tape_tile(sos, n_ch);
  const int K = sos->cas.K;
  filark_status rc = check_lds(fwd_lds_bytes(K, tt.waves, tt.levels(), tt.group), tt, K, sos->device);
  if (rc != FILARK_OK) return rc;
  const int prev_dev = current_device();
  if (prev_dev != sos->device) HIP_TRY(hipSetDevice(sos->device));
  const CkSpec ck{static_cast<double *>(tape), (int64_t)ck_slot_doubles(sos, n_ch), (int)adjoint_rows(sos, n_ch),
                  true};
  hipError_t e = forward_launches(sos, sl, tt, sos->d_state, sl->d_state, sl->d_cnt, x, y, cf, false, n_ch, n_t,
                                  stream, false, &ck, true);
  if (prev_dev != sos->device) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) return fail(FILARK_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

filark_status filark_sos_stalta_adjoint_tape(filark_sos_t sos, filark_stalta_t sl, const void *tape,
                                             size_t tape_bytes, const float *x, const float *g, int mode,
                                             double scale, float *gx, double *adj, double *gsos, int64_t n_ch,
                                             int64_t n_t, hipStream_t stream) {
  if (!sos || !sl) return fail(FILARK_EINVAL, "null state");
  if (n_t > 0 && !tape) return fail(FILARK_EINVAL, "null tape");
  if (sos->n_ch == n_ch && sl->n_ch == n_ch && n_t > 0) {
    const char *why = tape_unusable(sos, sl, n_ch);
    if (why) return fail(FILARK_EINVAL, "no tape: %s", why);
    const size_t need = tape_need(sos, n_ch, n_t);
    if (tape_bytes < need) return fail(FILARK_EINVAL, "tape of %zu bytes, %zu needed", tape_bytes, need);
  }
  return adjoint_run(sos, sl, static_cast<const double *>(tape), x, g, mode, scale, gx, adj, gsos, n_ch, n_t,
                     stream);
}

filark_status filark_batch_create(filark_batch_t *out, int n, const filark_sos_t *states, hipStream_t stream) {
  if (!out) return fail(FILARK_EINVAL, "null batch pointer");
  *out = nullptr;
  if (n < 1 || n > 4096 || !states) return fail(FILARK_EINVAL, "need 1 .. 4096 states");
  for (int i = 0; i < n; ++i)
    if (!states[i]) return fail(FILARK_EINVAL, "null state %d", i);
  const Tile t0 = states[0]->fwd.tile;
  for (int i = 0; i < n; ++i) {
    if (states[i]->device != states[0]->device) return fail(FILARK_EINVAL, "states live on different devices");
    if (states[i]->fwd.tile.block != kBatchBlock || states[i]->fwd.tile.waves != t0.waves)
      return fail(FILARK_EINVAL, "state %d: block must be %d and waves must match state 0's (group may differ)", i,
                  kBatchBlock);
    for (int j = 0; j < i; ++j)
      if (states[j] == states[i]) return fail(FILARK_EINVAL, "state %d appears twice", i);
  }
  filark_batch *b = new (std::nothrow) filark_batch();
  if (!b) return fail(FILARK_ENOMEM, "host allocation failed");
  b->device = states[0]->device;
  b->st.assign(states, states + n);
  b->nw = t0.waves;
  const int prev_dev = current_device();
  if (prev_dev != b->device) HIP_TRY(hipSetDevice(b->device));
  hipError_t e = hipMalloc(&b->d_stamps, (size_t)(n + 1) * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemsetAsync(b->d_stamps, 0, (size_t)(n + 1) * sizeof(unsigned long long), stream);
  if (e == hipSuccess) e = hipMalloc(&b->d_heads, 9 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemsetAsync(b->d_heads, 0, 9 * sizeof(uint32_t), stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (prev_dev != b->device) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) {
    filark_batch_destroy(b);
    return fail(FILARK_EHIP, "batch allocation: %s", hipGetErrorString(e));
  }
  *out = b;
  return FILARK_OK;
}

filark_status filark_batch_bind(filark_batch_t b, const float *const *in, float *const *out, const int64_t *n_t,
                                hipStream_t stream) {
  if (!b || !in || !out || !n_t) return fail(FILARK_EINVAL, "null pointer");
  const int n = (int)b->st.size();
  std::vector<FwdParams> descs;
  std::vector<BatchItem> lists[8];
  int kmax = 1;
  size_t lds = 0;
  for (int s = 0; s < n; ++s) {
    filark_sos_state *st = b->st[s];
    const Tile &t = st->fwd.tile;
    if (t.block != kBatchBlock || t.waves != b->nw)
      return fail(FILARK_EINVAL, "stream %d: block %d and waves %d differ from the batch's %d and %d", s, t.block,
                  t.waves, kBatchBlock, b->nw);
    if (n_t[s] < 0) return fail(FILARK_EINVAL, "stream %d: negative n_t", s);
    if (n_t[s] > 0 && (!in[s] || !out[s])) return fail(FILARK_EINVAL, "stream %d: null pointer", s);
    const int64_t rows = launch_rows(t, st->n_ch);
    if (rows == 0) return fail(FILARK_EINVAL, "stream %d: n_ch too large for its tile", s);
    const int K = st->cas.K;
    const size_t l = fwd_lds_bytes(K, t.waves, t.levels(), t.group);
    filark_status rc = check_lds(l, t, K, b->device);
    if (rc != FILARK_OK) return rc;
    if (n_t[s] == 0) continue;
    kmax = std::max(kmax, K);
    lds = std::max(lds, l);
    const uint64_t rowb = (uint64_t)st->n_ch * 4u;
    const int desc0 = (int)descs.size();
    const int n_grp = (int)((st->n_ch + t.group - 1) / t.group);
    for (int64_t t0 = 0; t0 < n_t[s]; t0 += rows) {
      const int64_t nt = std::min(rows, n_t[s] - t0);
      FwdParams p;
      std::memset(&p, 0, sizeof p);
      const size_t off = (size_t)t0 * (size_t)st->n_ch;
      p.x = in[s] + off;
      p.y = out[s] + off;
      p.n_ch = st->n_ch;
      p.n_t = (int32_t)nt;
      p.cw_log2 = log2_exact(t.group);
      p.nw = t.waves;
      p.n_grp = n_grp;
      p.per_xcd = per_xcd_for(n_grp);
      p.n_lev = t.levels();
      p.range = (int32_t)((uint64_t)nt * rowb);
      p.out_range = p.range;
      p.zs = st->d_state;
      p.coef = st->fwd.d;
      p.G = st->fwd.d + st->fwd.off_G;
      p.Pw = st->fwd.d + st->fwd.off_P;
      descs.push_back(p);
    }
    const int n_win = (int)descs.size() - desc0;
    // groups dealt to the XCDs in contiguous slabs, so the groups that share
    // cache lines meet in one L2
    const int per = per_xcd_for(n_grp);
    for (int g = 0; g < n_grp; ++g) lists[g / per].push_back({desc0, n_win, K, g, s, {0, 0, 0}});
  }
  // each queue longest items first (windows x sections): the last items to
  // start are the shortest
  std::vector<BatchItem> items;
  int qoff[9] = {};
  size_t longest = 0;
  for (int x = 0; x < 8; ++x) {
    std::stable_sort(lists[x].begin(), lists[x].end(), [](const BatchItem &u, const BatchItem &v) {
      return (int64_t)u.n_win * (u.K + 2) > (int64_t)v.n_win * (v.K + 2);
    });
    qoff[x] = (int)items.size();
    items.insert(items.end(), lists[x].begin(), lists[x].end());
    longest = std::max(longest, lists[x].size());
  }
  qoff[8] = (int)items.size();
  const int prev_dev = current_device();
  if (prev_dev != b->device) HIP_TRY(hipSetDevice(b->device));
  int per_cu = 0, n_cu = 0;
  hipError_t e = batch_occupancy(kmax, b->nw, lds, &per_cu);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  drop_graph(b);
  filark_status rc = FILARK_OK;
  if (e == hipSuccess && per_cu < 1) rc = fail(FILARK_EINVAL, "the batch's tiles do not fit a CU");
  if (rc == FILARK_OK && e == hipSuccess)
    rc = grow_raw(&b->d_descs, &b->descs_bytes, std::max<size_t>(1, descs.size()) * sizeof(FwdParams));
  if (rc == FILARK_OK && e == hipSuccess)
    rc = grow_raw(&b->d_items, &b->items_bytes, std::max<size_t>(1, items.size()) * sizeof(BatchItem));
  if (rc == FILARK_OK && e == hipSuccess && !descs.empty())
    e = hipMemcpy(b->d_descs, descs.data(), descs.size() * sizeof(FwdParams), hipMemcpyHostToDevice);
  if (rc == FILARK_OK && e == hipSuccess && !items.empty())
    e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
  if (prev_dev != b->device) (void)hipSetDevice(prev_dev);
  if (rc != FILARK_OK) return rc;
  if (e != hipSuccess) return fail(FILARK_EHIP, "batch upload: %s", hipGetErrorString(e));
  // as many workgroups as stay resident (a multiple of 8, one share per
  // XCD), but no more than the longest queue needs
  const int resident = std::max(1, per_cu * n_cu / 8);
  b->grid = 8 * std::max(1, std::min(resident, (int)longest));
  b->kmax = kmax;
  b->lds = lds;
  b->bp.descs = b->d_descs;
  b->bp.items = b->d_items;
  b->bp.heads = b->d_heads;
  b->bp.stamps = b->d_stamps;
  for (int x = 0; x < 9; ++x) b->bp.qoff[x] = qoff[x];
  b->bp.n_streams = n;
  b->gen.resize(n);
  for (int s = 0; s < n; ++s) b->gen[s] = b->st[s]->gen;
  b->bound = true;
  return FILARK_OK;
}

filark_status filark_batch_launch(filark_batch_t b, hipStream_t stream) {
  if (!b) return fail(FILARK_EINVAL, "null batch");
  if (!b->bound) return fail(FILARK_EINVAL, "batch not bound (filark_batch_bind)");
  for (size_t s = 0; s < b->st.size(); ++s)
    if (b->st[s]->gen != b->gen[s])
      return fail(FILARK_EINVAL, "stream %zu: tile changed since filark_batch_bind; bind again", s);
  const int prev_dev = current_device();
  if (prev_dev != b->device) HIP_TRY(hipSetDevice(b->device));
  const hipError_t e = b->exec ? hipGraphLaunch(b->exec, stream)
                               : launch_fwd_batch(b->bp, b->kmax, b->grid, b->nw, b->lds, stream);
  if (prev_dev != b->device) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) return fail(FILARK_EHIP, "batch launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

filark_status filark_batch_capture(filark_batch_t b) {
  if (!b) return fail(FILARK_EINVAL, "null batch");
  if (!b->bound) return fail(FILARK_EINVAL, "batch not bound (filark_batch_bind)");
  const int prev_dev = current_device();
  if (prev_dev != b->device) HIP_TRY(hipSetDevice(b->device));
  drop_graph(b);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t le = launch_fwd_batch(b->bp, b->kmax, b->grid, b->nw, b->lds, b->cap);
    e = hipStreamEndCapture(b->cap, &g);
    if (e == hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e == hipSuccess) {
    b->graph = g;
  } else if (g) {
    (void)hipGraphDestroy(g);
    b->exec = nullptr;
  }
  if (prev_dev != b->device) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) return fail(FILARK_EHIP, "batch capture failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

filark_status filark_batch_stamps(filark_batch_t b, uint64_t *host, hipStream_t stream) {
  if (!b || !host) return fail(FILARK_EINVAL, "null pointer");
  HIP_TRY(hipStreamSynchronize(stream));
  HIP_TRY(hipMemcpy(host, b->d_stamps, (b->st.size() + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost));
  return FILARK_OK;
}

filark_status filark_batch_destroy(filark_batch_t b) {
  if (!b) return FILARK_OK;
  drop_graph(b);
  if (b->d_descs) (void)hipFree(b->d_descs);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_stamps) (void)hipFree(b->d_stamps);
  if (b->d_heads) (void)hipFree(b->d_heads);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return FILARK_OK;
}

filark_status filark_autotune(filark_sos_t st, int64_t n_t, int block, int waves, const char *cache,
                              int *out_block, int *out_waves, int *out_group, hipStream_t stream) {
  if (!st || !out_block || !out_waves || !out_group) return fail(FILARK_EINVAL, "null pointer");
  if (n_t < 1 || n_t > ((int64_t)1 << 31)) return fail(FILARK_EINVAL, "n_t out of range: %lld", (long long)n_t);
  if (block != 0 && block != 32 && block != 48 && block != 64)
    return fail(FILARK_EINVAL, "block must be 0 (search) or 32, 48, 64");
  if (waves < 0 || waves > kMaxWaves) return fail(FILARK_EINVAL, "waves must be 0 (search) or 1 .. %d", kMaxWaves);
  const int64_t n_ch = st->n_ch;
  const int K = st->cas.K;
  char key[160];
  std::snprintf(key, sizeof key, "n_ch=%lld n_t=%lld K=%d block=%d waves=%d", (long long)n_ch, (long long)n_t, K,
                block, waves);
  // the cache: one entry per line, "key": {"block": B, "waves": W, "group": G, "us": T}
  std::map<std::string, std::string> entries;
  if (cache) {
    std::ifstream f(cache);
    std::string line;
    while (std::getline(f, line)) {
      const size_t q0 = line.find('"'), q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
      const size_t b0 = line.find('{'), b1 = line.rfind('}');
      if (q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos || b1 < b0) continue;
      entries[line.substr(q0 + 1, q1 - q0 - 1)] = line.substr(b0, b1 - b0 + 1);
    }
    auto it = entries.find(key);
    int cb = 0, cw = 0, cg = 0;
    if (it != entries.end() &&
        std::sscanf(it->second.c_str(), "{\"block\": %d, \"waves\": %d, \"group\": %d", &cb, &cw, &cg) == 3 &&
        check_tile(cb, cw, cg, false) == FILARK_OK) {
      filark_status rc = filark_tile_set(st, FILARK_STATE_SOS, cb, cw, cg, stream);
      if (rc != FILARK_OK) return rc;
      *out_block = cb;
      *out_waves = cw;
      *out_group = cg;
      return FILARK_OK;
    }
  }
  // a scratch state of the same filter, and synthetic input of the shape
  std::vector<double> sos(6 * (size_t)K);
  for (int k = 0; k < K; ++k) {
    const double *c = st->cas.c[k];
    const double row[6] = {c[0], c[1], c[2], 1.0, c[3], c[4]};
    std::copy(row, row + 6, sos.begin() + 6 * k);
  }
  const int prev_dev = current_device();
  if (prev_dev != st->device) HIP_TRY(hipSetDevice(st->device));
  filark_sos_t tmp = nullptr;
  filark_status rc = filark_sos_init(&tmp, sos.data(), K, n_ch, 0, stream);
  float *buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSuccess;
  const size_t bytes = (size_t)n_t * (size_t)n_ch * sizeof(float);
  if (rc == FILARK_OK) e = hipMalloc(&buf, 2 * bytes);
  if (rc == FILARK_OK && e == hipSuccess) e = hipMemsetAsync(buf, 0, 2 * bytes, stream);
  if (rc == FILARK_OK && e == hipSuccess) e = hipEventCreate(&e0);
  if (rc == FILARK_OK && e == hipSuccess) e = hipEventCreate(&e1);
  const std::vector<int> blocks = block ? std::vector<int>{block} : std::vector<int>{32, 48, 64};
  const std::vector<int> wave_set = waves ? std::vector<int>{waves} : std::vector<int>{2, 4, 8};
  const int groups[5] = {4, 8, 16, 32, 64};
  constexpr int kReps = 3;
  float best = -1.0f;
  int bb = 0, bw = 0, bg = 0;
  for (const int blk : blocks) {
    for (const int wv : wave_set) {
      for (int ig = 0; ig < 5 && rc == FILARK_OK && e == hipSuccess; ++ig) {
        Tile t;
        t.block = blk;
        t.waves = wv;
        t.group = groups[ig];
        if (t.blocks() < 1 || launch_rows(t, n_ch) == 0) continue;
        if (check_lds(fwd_lds_bytes(K, t.waves, t.levels(), t.group), t, K, st->device) != FILARK_OK) continue;
        rc = filark_tile_set(tmp, FILARK_STATE_SOS, t.block, t.waves, t.group, stream);
        if (rc != FILARK_OK) break;
        rc = filark_sos_process(tmp, buf, buf + bytes / sizeof(float), n_ch, n_t, stream);  // warm-up
        if (rc != FILARK_OK) break;
        e = hipEventRecord(e0, stream);
        for (int r = 0; r < kReps && rc == FILARK_OK && e == hipSuccess; ++r)
          rc = filark_sos_process(tmp, buf, buf + bytes / sizeof(float), n_ch, n_t, stream);
        if (rc == FILARK_OK && e == hipSuccess) e = hipEventRecord(e1, stream);
        if (rc == FILARK_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (rc == FILARK_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (rc == FILARK_OK && e == hipSuccess && (best < 0.0f || ms < best)) {
          best = ms;
          bb = t.block;
          bw = t.waves;
          bg = t.group;
        }
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf) (void)hipFree(buf);
  if (tmp) filark_sos_destroy(tmp);
  if (prev_dev != st->device) (void)hipSetDevice(prev_dev);
  if (rc != FILARK_OK) return rc;
  if (e != hipSuccess) return fail(FILARK_EHIP, "autotune: %s", hipGetErrorString(e));
  if (best < 0.0f) return fail(FILARK_EINVAL, "no tile candidate fits %lld channels", (long long)n_ch);
  rc = filark_tile_set(st, FILARK_STATE_SOS, bb, bw, bg, stream);
  if (rc != FILARK_OK) return rc;
  *out_block = bb;
  *out_waves = bw;
  *out_group = bg;
  if (cache) {
    char val[128];
    std::snprintf(val, sizeof val, "{\"block\": %d, \"waves\": %d, \"group\": %d, \"us\": %.2f}", bb, bw, bg,
                  1e3 * best / kReps);
    entries[key] = val;
    const std::string tmp_path = std::string(cache) + ".tmp";
    std::ofstream f(tmp_path);
    f << "{\n";
    size_t i = 0;
    for (const auto &kv : entries) f << " \"" << kv.first << "\": " << kv.second << (++i < entries.size() ? ",\n" : "\n");
    f << "}\n";
    f.close();
    if (!f || std::rename(tmp_path.c_str(), cache) != 0)
      return fail(FILARK_EINVAL, "autotune: cannot write the cache %s", cache);
  }
  return FILARK_OK;
}

filark_status filark_check(const void *obj, int kind, hipStream_t stream) {
  if (!obj) return fail(FILARK_EINVAL, "null state");
  if (kind != FILARK_STATE_SOS && kind != FILARK_STATE_STALTA)
    return fail(FILARK_EINVAL, "unknown state kind %d", kind);
  HIP_TRY(hipStreamSynchronize(stream));
  HIP_TRY(hipGetLastError());
  return FILARK_OK;
}

filark_status filark_sos_destroy(filark_sos_t st) {
  if (!st) return FILARK_OK;
  if (st->d_state) (void)hipFree(st->d_state);
  if (st->fwd.d) (void)hipFree(st->fwd.d);
  if (st->adj.d) (void)hipFree(st->adj.d);
  if (st->ckp.d) (void)hipFree(st->ckp.d);
  if (st->d_ck) (void)hipFree(st->d_ck);
  if (st->d_ff) (void)hipFree(st->d_ff);
  if (st->d_gpart) (void)hipFree(st->d_gpart);
  delete st;
  return FILARK_OK;
}

filark_status filark_stalta_destroy(filark_stalta_t st) {
  if (!st) return FILARK_OK;
  if (st->d_state) (void)hipFree(st->d_state);  // holds the counter too
  if (st->fwd.d) (void)hipFree(st->fwd.d);
  if (st->adj.d) (void)hipFree(st->adj.d);
  if (st->ckp.d) (void)hipFree(st->ckp.d);
  delete st;
  return FILARK_OK;
}

filark_status filark_ema_init(filark_ema_t *out, int mode, double win_s, double fs, int64_t n_ch,
                              hipStream_t stream) {
  if (!out) return fail(FILARK_EINVAL, "null state pointer");
  *out = nullptr;
  if (mode != FILARK_EMA_DEMEAN && mode != FILARK_EMA_AGC) return fail(FILARK_EINVAL, "unknown mode %d", mode);
  if (!(fs > 0.0) || !(win_s > 0.0) || !std::isfinite(fs * win_s)) return fail(FILARK_EINVAL, "window and fs must be positive");
  const double nw = std::round(win_s * fs);
  if (nw < 1.0 || nw > 9.0e15) return fail(FILARK_EINVAL, "the window must round to >= 1 sample");
  if (n_ch < 1 || n_ch > (int64_t)1 << 24) return fail(FILARK_EINVAL, "n_ch must be in [1, 2^24]");
  filark_ema_state *st = new (std::nothrow) filark_ema_state();
  if (!st) return fail(FILARK_ENOMEM, "host allocation failed");
  st->device = current_device();
  st->n_ch = n_ch;
  st->n_win = (int64_t)nw;
  st->mode = mode;
  Tile t;
  t.block = kTrigBlock;
  t.waves = kTrigWaves;
  t.group = kTrigGroup;
  st->n_lev = t.levels();
  const double a = 1.0 - 1.0 / (double)st->n_win;
  std::vector<double> tab;
  for (int k = 0; k < st->n_lev; ++k) tab.push_back(std::pow(a, (double)t.block * std::ldexp(1.0, k)));
  for (int m = 0; m <= t.block; ++m) tab.push_back(std::pow(a, (double)m));
  filark_status rc = upload(&st->d_tab, tab, stream);
  hipError_t e = hipSuccess;
  if (rc == FILARK_OK) {
    e = hipMalloc(&st->d_avg, (size_t)n_ch * sizeof(double));
    if (e == hipSuccess) e = hipMemsetAsync(st->d_avg, 0, (size_t)n_ch * sizeof(double), stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) rc = fail(FILARK_EHIP, "state allocation: %s", hipGetErrorString(e));
  }
  if (rc != FILARK_OK) {
    filark_ema_destroy(st);
    return rc;
  }
  *out = st;
  return FILARK_OK;
}

filark_status filark_ema_process(filark_ema_t st, const float *in, float *out, int64_t n_ch, int64_t n_t,
                                 hipStream_t stream) {
  if (!st) return fail(FILARK_EINVAL, "null state");
  if (n_ch != st->n_ch) return fail(FILARK_ESHAPE, "n_ch %lld != the state's %lld", (long long)n_ch, (long long)st->n_ch);
  if (n_t < 0) return fail(FILARK_EINVAL, "negative n_t");
  if (n_t == 0) return FILARK_OK;
  if (!in || !out) return fail(FILARK_EINVAL, "null input or output pointer");
  Tile t;
  t.block = kTrigBlock;
  t.waves = kTrigWaves;
  t.group = kTrigGroup;
  const int64_t rows = launch_rows(t, n_ch);
  if (rows == 0) return fail(FILARK_EINVAL, "n_ch %lld too large", (long long)n_ch);
  const int prev_dev = current_device();
  if (prev_dev != st->device) HIP_TRY(hipSetDevice(st->device));
  EmaParams p;
  std::memset(&p, 0, sizeof p);
  p.n_ch = n_ch;
  p.cw_log2 = log2_exact(t.group);
  p.nw = t.waves;
  p.n_grp = (int)((n_ch + t.group - 1) / t.group);
  p.per_xcd = per_xcd_for(p.n_grp);
  p.n_lev = st->n_lev;
  p.mode = st->mode;
  p.avg = st->d_avg;
  p.dpow = st->d_tab;
  p.c = 1.0 / (double)st->n_win;
  p.a = 1.0 - p.c;
  hipError_t e = hipSuccess;
  for (int64_t t0 = 0; t0 < n_t && e == hipSuccess; t0 += rows) {
    const int64_t nt = std::min<int64_t>(rows, n_t - t0);
    p.x = in + t0 * n_ch;
    p.y = out + t0 * n_ch;
    p.n_t = (int32_t)nt;
    p.range = (int32_t)((uint64_t)nt * (uint64_t)n_ch * 4u);
    e = launch_ema(p, t.block, stream);
  }
  if (prev_dev != st->device) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) return fail(FILARK_EHIP, "launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

filark_status filark_ema_state_get(filark_ema_t st, double *avg, hipStream_t stream) {
  if (!st || !avg) return fail(FILARK_EINVAL, "null pointer");
  HIP_TRY(hipStreamSynchronize(stream));
  HIP_TRY(hipMemcpy(avg, st->d_avg, (size_t)st->n_ch * sizeof(double), hipMemcpyDeviceToHost));
  return FILARK_OK;
}

filark_status filark_ema_state_set(filark_ema_t st, const double *avg, hipStream_t stream) {
  if (!st || !avg) return fail(FILARK_EINVAL, "null pointer");
  for (int64_t c = 0; c < st->n_ch; ++c)
    if (!std::isfinite(avg[c]) || (st->mode == FILARK_EMA_AGC && avg[c] < 0.0))
      return fail(FILARK_EINVAL, "state_set: invalid average");
  HIP_TRY(hipStreamSynchronize(stream));
  HIP_TRY(hipMemcpy(st->d_avg, avg, (size_t)st->n_ch * sizeof(double), hipMemcpyHostToDevice));
  return FILARK_OK;
}

filark_status filark_ema_destroy(filark_ema_t st) {
  if (!st) return FILARK_OK;
  if (st->d_avg) (void)hipFree(st->d_avg);
  if (st->d_tab) (void)hipFree(st->d_tab);
  delete st;
  return FILARK_OK;
}

filark_status filark_trigger_init(filark_trigger_t *out, float on, float off, int64_t n_ch,
                                  hipStream_t stream) {
  if (!out) return fail(FILARK_EINVAL, "null trigger pointer");
  *out = nullptr;
  if (!std::isfinite(on) || !std::isfinite(off) || off > on)
    return fail(FILARK_EINVAL, "thresholds must be finite with off <= on");
  if (n_ch < 1 || n_ch > (int64_t)1 << 24) return fail(FILARK_EINVAL, "n_ch must be in [1, 2^24]");
  filark_trigger_state *st = new (std::nothrow) filark_trigger_state();
  if (!st) return fail(FILARK_ENOMEM, "host allocation failed");
  st->device = current_device();
  st->n_ch = n_ch;
  st->on = on;
  st->off = off;
  hipError_t e = hipMalloc(&st->d_open, (size_t)n_ch * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemsetAsync(st->d_open, 0, (size_t)n_ch * sizeof(int32_t), stream);
  if (e == hipSuccess) e = hipMalloc(&st->d_ton, (size_t)n_ch * sizeof(int64_t));
  if (e == hipSuccess) e = hipMemsetAsync(st->d_ton, 0, (size_t)n_ch * sizeof(int64_t), stream);
  if (e == hipSuccess) e = hipMalloc(&st->d_cnt, (size_t)n_ch * sizeof(int64_t));
  if (e == hipSuccess) e = hipMemsetAsync(st->d_cnt, 0, (size_t)n_ch * sizeof(int64_t), stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    filark_trigger_destroy(st);
    return fail(FILARK_EHIP, "trigger allocation: %s", hipGetErrorString(e));
  }
  *out = st;
  return FILARK_OK;
}

filark_status filark_trigger_process(filark_trigger_t st, const float *cf, int64_t n_ch, int64_t n_t,
                                     int64_t *events, int64_t cap, uint64_t *count, hipStream_t stream) {
  if (!st) return fail(FILARK_EINVAL, "null trigger");
  if (n_ch != st->n_ch) return fail(FILARK_ESHAPE, "n_ch %lld != trigger's %lld", (long long)n_ch, (long long)st->n_ch);
  if (n_t < 0 || cap < 0) return fail(FILARK_EINVAL, "negative n_t or capacity");
  if (!count || (cap > 0 && !events)) return fail(FILARK_EINVAL, "null count or events pointer");
  if (n_t == 0) return FILARK_OK;
  if (!cf) return fail(FILARK_EINVAL, "null cf pointer");
  Tile t;
  t.block = kTrigBlock;
  t.waves = kTrigWaves;
  t.group = kTrigGroup;
  const int64_t rows = launch_rows(t, n_ch);
  if (rows == 0) return fail(FILARK_EINVAL, "n_ch %lld too large", (long long)n_ch);
  const int prev_dev = current_device();
  if (prev_dev != st->device) HIP_TRY(hipSetDevice(st->device));
  TrigParams p;
  std::memset(&p, 0, sizeof p);
  p.n_ch = n_ch;
  p.cw_log2 = log2_exact(t.group);
  p.nw = t.waves;
  p.n_grp = (int)((n_ch + t.group - 1) / t.group);
  p.per_xcd = per_xcd_for(p.n_grp);
  p.on = st->on;
  p.off = st->off;
  p.open = st->d_open;
  p.t_on = st->d_ton;
  p.cnt = st->d_cnt;
  p.ev = events;
  p.cap = cap;
  p.count = reinterpret_cast<unsigned long long *>(count);
  hipError_t e = hipSuccess;
  for (int64_t t0 = 0; t0 < n_t && e == hipSuccess; t0 += rows) {
    const int64_t nt = std::min<int64_t>(rows, n_t - t0);
    p.cf = cf + t0 * n_ch;
    p.n_t = (int32_t)nt;
    p.range = (int32_t)((uint64_t)nt * (uint64_t)n_ch * 4u);
    e = launch_trig(p, t.block, stream);
  }
  if (prev_dev != st->device) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) return fail(FILARK_EHIP, "trigger launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

filark_status filark_monitor_process(filark_sos_t sos, filark_stalta_t sl, filark_trigger_t tr, const float *in,
                                     float *y_or_null, float *cf_or_null, int64_t *events, int64_t cap,
                                     uint64_t *count, int64_t n_ch, int64_t n_t, hipStream_t stream) {
  if (!sos || !sl || !tr) return fail(FILARK_EINVAL, "null state");
  if (sos->device != sl->device || sos->device != tr->device)
    return fail(FILARK_EINVAL, "states live on different devices");
  if (sos->n_ch != n_ch || sl->n_ch != n_ch || tr->n_ch != n_ch)
    return fail(FILARK_ESHAPE, "n_ch %lld differs from a state's", (long long)n_ch);
  if (n_t < 0 || cap < 0) return fail(FILARK_EINVAL, "negative n_t or capacity");
  if (!count || (cap > 0 && !events)) return fail(FILARK_EINVAL, "null count or events pointer");
  if (n_t == 0) return FILARK_OK;
  if (!in) return fail(FILARK_EINVAL, "null input pointer");
  if (y_or_null && cf_or_null && (const void *)y_or_null == (const void *)cf_or_null)
    return fail(FILARK_EINVAL, "y and cf must differ");
  const Tile t = sos->fwd.tile;
  if (!(sl->fwd.tile == t)) return fail(FILARK_EINVAL, "tile shapes of the states differ (set both with filark_tile_set)");
  if (t.block != 48) return fail(FILARK_EINVAL, "the monitor runs 48-row blocks (tile block %d)", t.block);
  const int64_t rows = launch_rows(t, n_ch);
  if (rows == 0) return fail(FILARK_EINVAL, "n_ch %lld too large", (long long)n_ch);
  const int K = sos->cas.K;
  filark_status rc = check_lds(fwd_lds_bytes(K, t.waves, t.levels(), t.group), t, K, sos->device);
  if (rc != FILARK_OK) return rc;
  const int prev_dev = current_device();
  if (prev_dev != sos->device) HIP_TRY(hipSetDevice(sos->device));
  MonParams m;
  std::memset(&m, 0, sizeof m);
  m.f = fwd_base(sos, sl, t, sos->d_state, sl->d_state, sl->d_cnt, n_ch, false);
  TrigParams &q = m.t;
  q.n_ch = n_ch;
  q.cw_log2 = m.f.cw_log2;
  q.nw = m.f.nw;
  q.n_grp = m.f.n_grp;
  q.per_xcd = m.f.per_xcd;
  q.on = tr->on;
  q.off = tr->off;
  q.open = tr->d_open;
  q.t_on = tr->d_ton;
  q.cnt = tr->d_cnt;
  q.ev = events;
  q.cap = cap;
  q.count = reinterpret_cast<unsigned long long *>(count);
  const uint64_t rowb = (uint64_t)n_ch * 4u;
  hipError_t e = hipSuccess;
  for (int64_t t0 = 0; t0 < n_t && e == hipSuccess; t0 += rows) {
    const int64_t nt = std::min(rows, n_t - t0);
    const size_t off = (size_t)t0 * (size_t)n_ch;
    m.f.x = in + off;
    m.f.y = y_or_null ? y_or_null + off : nullptr;
    m.f.cf = cf_or_null ? cf_or_null + off : nullptr;
    m.f.n_t = (int32_t)nt;
    m.f.range = (int32_t)((uint64_t)nt * rowb);
    m.f.out_range = m.f.range;
    q.n_t = (int32_t)nt;
    e = launch_monitor(m, K, y_or_null != nullptr, sos->cas.unit_tail(), stream);
  }
  if (prev_dev != sos->device) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) return fail(FILARK_EHIP, "monitor launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

filark_status filark_trigger_state_get(filark_trigger_t st, int64_t *open_ton, int64_t *counter,
                                       hipStream_t stream) {
  if (!st || !open_ton || !counter) return fail(FILARK_EINVAL, "null pointer");
  HIP_TRY(hipStreamSynchronize(stream));
  std::vector<int32_t> o((size_t)st->n_ch);
  std::vector<int64_t> t((size_t)st->n_ch);
  HIP_TRY(hipMemcpy(o.data(), st->d_open, o.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(t.data(), st->d_ton, t.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(counter, st->d_cnt, sizeof(int64_t), hipMemcpyDeviceToHost));
  for (int64_t c = 0; c < st->n_ch; ++c) {
    open_ton[2 * c] = o[c] ? 1 : 0;
    open_ton[2 * c + 1] = o[c] ? t[c] : 0;
  }
  return FILARK_OK;
}

filark_status filark_trigger_state_set(filark_trigger_t st, const int64_t *open_ton, int64_t counter,
                                       hipStream_t stream) {
  if (!st || !open_ton) return fail(FILARK_EINVAL, "null pointer");
  if (counter < 0) return fail(FILARK_EINVAL, "negative sample counter");
  std::vector<int32_t> o((size_t)st->n_ch);
  std::vector<int64_t> t((size_t)st->n_ch), g((size_t)st->n_ch, counter);
  for (int64_t c = 0; c < st->n_ch; ++c) {
    if (open_ton[2 * c] != 0 && open_ton[2 * c] != 1) return fail(FILARK_EINVAL, "open flag must be 0 or 1");
    if (open_ton[2 * c] && (open_ton[2 * c + 1] < 0 || open_ton[2 * c + 1] >= counter))
      return fail(FILARK_EINVAL, "open event must start before the counter");
    o[c] = (int32_t)open_ton[2 * c];
    t[c] = open_ton[2 * c + 1];
  }
  HIP_TRY(hipStreamSynchronize(stream));
  HIP_TRY(hipMemcpy(st->d_open, o.data(), o.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(st->d_ton, t.data(), t.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(st->d_cnt, g.data(), g.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  return FILARK_OK;
}

filark_status filark_trigger_destroy(filark_trigger_t st) {
  if (!st) return FILARK_OK;
  if (st->d_open) (void)hipFree(st->d_open);
  if (st->d_ton) (void)hipFree(st->d_ton);
  if (st->d_cnt) (void)hipFree(st->d_cnt);
  delete st;
  return FILARK_OK;
}

namespace {

// Rows per FIR launch: every byte offset the kernel forms (window rows plus
// the taps' reach back and one wave's rows of slack) stays below 2^31.  A
// multiple of 96 x waves, so that 16-, 32- and 48-row waves tile it.
constexpr int kFirMaxRows = 48;
int64_t fir_window_rows(const filark_fir_state *st) {
  const int64_t rowb = st->n_ch * 4;
  const int64_t span = (int64_t)96 * st->waves;
  const int64_t budget = ((int64_t)1 << 31) / rowb - (st->n_pad + kFirMaxRows + kFirChunk + 2);
  return std::max<int64_t>(0, (budget - (st->n_pad - 1)) / span * span);
}

}  // namespace

filark_status filark_fir_init(filark_fir_t *out, const double *taps, int n_taps, int64_t n_ch, hipStream_t stream) {
  if (!out) return fail(FILARK_EINVAL, "null state pointer");
  *out = nullptr;
  if (!taps) return fail(FILARK_EINVAL, "null taps");
  if (n_taps < 1 || n_taps > 1024) return fail(FILARK_EINVAL, "n_taps must be in [1, 1024]");
  for (int k = 0; k < n_taps; ++k)
    if (!std::isfinite(taps[k]) || std::fabs(taps[k]) > 3.0e38) return fail(FILARK_EINVAL, "taps must be finite FP32 values");
  if (n_ch < 1 || n_ch > (int64_t)1 << 24) return fail(FILARK_EINVAL, "n_ch must be in [1, 2^24]");
  filark_fir_state *st = new (std::nothrow) filark_fir_state();
  if (!st) return fail(FILARK_ENOMEM, "host allocation failed");
  st->device = current_device();
  st->n_ch = n_ch;
  st->n_taps = n_taps;
  st->n_pad = (n_taps + kFirChunk - 1) / kFirChunk * kFirChunk;
  if (fir_window_rows(st) < 1) {
    delete st;
    return fail(FILARK_EINVAL, "n_ch %lld too large for a %d-tap FIR", (long long)n_ch, n_taps);
  }
  std::vector<float> h((size_t)st->n_pad, 0.0f);
  for (int k = 0; k < n_taps; ++k) h[k] = (float)taps[k];
  const size_t hist_bytes = (size_t)std::max(n_taps - 1, 1) * (size_t)n_ch * sizeof(float);
  hipError_t e = hipMalloc(&st->d_h, h.size() * sizeof(float));
  if (e == hipSuccess) e = hipMemcpyAsync(st->d_h, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, stream);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipMalloc(&st->d_hist[i], hist_bytes);
    if (e == hipSuccess) e = hipMemsetAsync(st->d_hist[i], 0, hist_bytes, stream);
  }
  if (e == hipSuccess) e = hipMalloc(&st->d_ctl, 2 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemsetAsync(st->d_ctl, 0, 2 * sizeof(uint32_t), stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    filark_fir_destroy(st);
    return fail(FILARK_EHIP, "state allocation: %s", hipGetErrorString(e));
  }
  *out = st;
  return FILARK_OK;
}

filark_status filark_fir_set_tile(filark_fir_t st, int rows, int waves, int order) {
  if (!st) return fail(FILARK_EINVAL, "null state");
  if ((rows != 0 && !fir_rows_ok(rows)) || waves < 1 || waves > kMaxWaves || order < 0 || order > 2)
    return fail(FILARK_EINVAL, "FIR tile %dx%d order %d: rows must be 0 (by launch), 16, 32 or 48, waves 1..%d, "
                "order 0..2", rows, waves, order, kMaxWaves);
  const int r0 = st->rows, w0 = st->waves;
  st->rows = rows;
  st->waves = waves;
  if (fir_window_rows(st) < 1) {
    st->rows = r0;
    st->waves = w0;
    return fail(FILARK_EINVAL, "FIR tile %dx%d too tall for n_ch %lld", rows, waves, (long long)st->n_ch);
  }
  st->order = order;
  return FILARK_OK;
}

filark_status filark_fir_set_method(filark_fir_t st, int method, hipStream_t stream) {
  if (!st) return fail(FILARK_EINVAL, "null state");
  if (method != FILARK_FIR_DIRECT && method != FILARK_FIR_FFT) return fail(FILARK_EINVAL, "unknown method %d", method);
  if (method == FILARK_FIR_FFT && !st->d_fft) {
    // twiddles W_1024^j and W_2048^k, and H[k] = sum_n h[n] W_2048^(n k) / 4096
    // (the FP32 taps the direct kernel uses, summed in FP64; 1 / 4096 folds
    // the inverse's 1 / 1024 and the real-transform halves)
    constexpr int N = kFftN, N2 = kFftN / 2;
    std::vector<float2> tab((size_t)N + N2 + 1);
    const double two_pi = 6.283185307179586476925286766559;
    for (int j = 0; j < N2; ++j) {
      const double a = -two_pi * j / N2;
      tab[j] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    for (int k = 0; k < N2; ++k) {
      const double a = -two_pi * k / N;
      tab[N2 + k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    const int prev_dev = current_device();
    if (prev_dev != st->device) HIP_TRY(hipSetDevice(st->device));
    std::vector<double> h(st->n_taps);
    std::vector<float> hf((size_t)st->n_pad);
    hipError_t e = hipMemcpy(hf.data(), st->d_h, hf.size() * sizeof(float), hipMemcpyDeviceToHost);
    for (int n = 0; n < st->n_taps; ++n) h[n] = (double)hf[n];
    for (int k = 0; k <= N2; ++k) {
      double re = 0.0, im = 0.0;
      for (int n = 0; n < st->n_taps; ++n) {
        const double a = -two_pi * (double)(((int64_t)n * k) % N) / N;
        re += h[n] * std::cos(a);
        im += h[n] * std::sin(a);
      }
      tab[N + k] = make_float2((float)(re / 4096.0), (float)(im / 4096.0));
    }
    if (e == hipSuccess) e = hipMalloc(&st->d_fft, tab.size() * sizeof(float2));
    if (e == hipSuccess) e = hipMemcpy(st->d_fft, tab.data(), tab.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess && st->d_fft) {
      (void)hipFree(st->d_fft);
      st->d_fft = nullptr;
    }
    if (prev_dev != st->device) (void)hipSetDevice(prev_dev);
    if (e != hipSuccess) return fail(FILARK_EHIP, "FFT tables: %s", hipGetErrorString(e));
  }
  (void)stream;
  st->method = method;
  return FILARK_OK;
}

filark_status filark_fir_process(filark_fir_t st, const float *in, float *out, int64_t n_ch, int64_t n_t,
                                 hipStream_t stream) {
  if (!st) return fail(FILARK_EINVAL, "null state");
  if (n_ch != st->n_ch) return fail(FILARK_ESHAPE, "n_ch %lld != the state's %lld", (long long)n_ch, (long long)st->n_ch);
  if (n_t < 0 || n_t > ((int64_t)1 << 40)) return fail(FILARK_EINVAL, "n_t out of range");
  if (n_t == 0) return FILARK_OK;
  if (!in || !out) return fail(FILARK_EINVAL, "null input or output pointer");
  {
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out, n = (uintptr_t)(n_t * n_ch * 4);
    if (a < b + n && b < a + n) return fail(FILARK_EINVAL, "FIR input and output must not overlap");
  }
  if (st->method == FILARK_FIR_FFT) {
    FftParams q;
    std::memset(&q, 0, sizeof q);
    q.x = in;
    q.y = out;
    q.tw = st->d_fft;
    q.H = st->d_fft + kFftN;
    q.hist0 = st->d_hist[0];
    q.hist1 = st->d_hist[1];
    q.ctl = st->d_ctl;
    q.n_ch = n_ch;
    q.n_t = n_t;
    q.hm = st->n_taps - 1;
    q.B = kFftN - q.hm;
    q.ch = 8;
    q.threads = 512;
    if ((n_t + q.B - 1) / q.B > 65535) return fail(FILARK_EINVAL, "n_t too large for one FFT call");
    const int prev_dev = current_device();
    if (prev_dev != st->device) HIP_TRY(hipSetDevice(st->device));
    hipError_t e = launch_fir_fft(q, stream);  // it also flips the current history buffer
    if (prev_dev != st->device) (void)hipSetDevice(prev_dev);
    if (e != hipSuccess) return fail(FILARK_EHIP, "FFT launch failed: %s", hipGetErrorString(e));
    return FILARK_OK;
  }
  const int64_t W = fir_window_rows(st);
  if (W < 1) return fail(FILARK_EINVAL, "n_ch too large for this FIR tile");
  const int prev_dev = current_device();
  if (prev_dev != st->device) HIP_TRY(hipSetDevice(st->device));
  const int64_t rowb = n_ch * 4, hm = st->n_taps - 1;
  FirParams p;
  std::memset(&p, 0, sizeof p);
  p.h = st->d_h;
  p.hist0 = st->d_hist[0];
  p.hist1 = st->d_hist[1];
  p.ctl = st->d_ctl;
  p.n_ch = n_ch;
  p.hrange = (int32_t)(hm * rowb);
  p.hm = (int32_t)hm;
  p.n_chunks = st->n_pad / kFirChunk;
  p.n_cg = (int32_t)((n_ch + kWave - 1) / kWave);
  p.nw = st->waves;
  p.chan_minor = st->order;
  hipError_t e = hipSuccess;
  for (int64_t T0 = 0; T0 < n_t && e == hipSuccess; T0 += W) {
    const int64_t n_rows = std::min<int64_t>(W, n_t - T0);
    const int64_t lo = std::max<int64_t>(0, T0 - (st->n_pad - 1));
    p.x = in + lo * n_ch;
    p.y = out + T0 * n_ch;
    p.xoff = (int32_t)(T0 - lo);
    p.n_rows = (int32_t)n_rows;
    p.range = (int32_t)((T0 + n_rows - lo) * rowb);
    p.out_range = (int32_t)(n_rows * rowb);
    const int64_t hs = n_t - hm - T0;
    p.hs = (int32_t)std::max<int64_t>(std::min<int64_t>(hs, n_rows), -hm);
    p.hcopy = T0 == 0 ? (int32_t)std::max<int64_t>(0, hm - n_t) : 0;
    p.hsrc = (int32_t)std::min<int64_t>(n_t, hm);
    // by launch: 48-row waves (3 per SIMD) on long windows of the unrolled
    // kernels, where their lower halo share pays; 32-row waves (4 per SIMD)
    // on chunk-sized windows and on the looped kernel, where more waves per
    // SIMD hide more load latency
    const int R = st->rows ? st->rows : (n_rows >= 8192 && p.n_chunks <= 2 ? 48 : 32);
    const int64_t span = (int64_t)R * st->waves;
    p.n_tb = (int32_t)((n_rows + span - 1) / span);
    const int64_t n_wg = (int64_t)p.n_cg * p.n_tb;
    if (n_wg > ((int64_t)1 << 30)) {
      e = hipErrorInvalidValue;
      break;
    }
    p.per_xcd = st->order == 2 ? (p.n_cg + 7) / 8 : (int32_t)((n_wg + 7) / 8);
    e = launch_fir(p, R, stream);
  }
  if (e == hipSuccess) e = launch_fir_flip(st->d_ctl, stream);
  if (prev_dev != st->device) (void)hipSetDevice(prev_dev);
  if (e != hipSuccess) return fail(FILARK_EHIP, "launch failed: %s", hipGetErrorString(e));
  return FILARK_OK;
}

filark_status filark_fir_state_get(filark_fir_t st, float *hist, hipStream_t stream) {
  if (!st || !hist) return fail(FILARK_EINVAL, "null pointer");
  if (st->n_taps == 1) return FILARK_OK;
  HIP_TRY(hipStreamSynchronize(stream));
  uint32_t ctl = 0;
  HIP_TRY(hipMemcpy(&ctl, st->d_ctl, sizeof ctl, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hist, st->d_hist[ctl & 1u], (size_t)(st->n_taps - 1) * st->n_ch * sizeof(float),
                    hipMemcpyDeviceToHost));
  return FILARK_OK;
}

filark_status filark_fir_state_set(filark_fir_t st, const float *hist, hipStream_t stream) {
  if (!st || !hist) return fail(FILARK_EINVAL, "null pointer");
  if (st->n_taps == 1) return FILARK_OK;
  const size_t n = (size_t)(st->n_taps - 1) * st->n_ch;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(hist[i])) return fail(FILARK_EINVAL, "state_set: history must be finite");
  HIP_TRY(hipStreamSynchronize(stream));
  uint32_t ctl = 0;
  HIP_TRY(hipMemcpy(&ctl, st->d_ctl, sizeof ctl, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(st->d_hist[ctl & 1u], hist, n * sizeof(float), hipMemcpyHostToDevice));
  return FILARK_OK;
}

filark_status filark_fir_destroy(filark_fir_t st) {
  if (!st) return FILARK_OK;
  if (st->d_fft) (void)hipFree(st->d_fft);
  if (st->d_h) (void)hipFree(st->d_h);
  for (int i = 0; i < 2; ++i)
    if (st->d_hist[i]) (void)hipFree(st->d_hist[i]);
  if (st->d_ctl) (void)hipFree(st->d_ctl);
  delete st;
  return FILARK_OK;
}

}  // extern "C"
