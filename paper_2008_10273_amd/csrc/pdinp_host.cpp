// Host side of the C ABI declared in include/pdinp.h: context, per-shape
// tables, argument checks and kernel orchestration.  Every step of the
// decode itself runs in the kernels of pdinp_kernels.hip.
#include "../../include/pdinp.h"
#include "pdinp_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

namespace {

constexpr double kPi = 3.14159265358979323846;
// Batches of at least this many mask blocks (all frames) take the binned
// wave-level path for b <= 16.
constexpr long long kBinnedMinBlocks = 32768;

struct TableSet {
  float *tab32 = nullptr;
  double *tab64 = nullptr;
  size_t bytes = 0;
  int tab32_floats = 0;
  int nshapes = 0;
  pdi::ShapeDev s[pdi::kMaxShapes];
  int group_shape[pdi::kMaxGroups][4];
};

using TableKey = std::tuple<int, int, int, int, int, int, double>;  // W,H,fmt,b,shared,op,s
// Launch choice per geometry, operator, evaluation dtype and frames per
// launch (set by pdi_autotune / pdi_autotune_batch).
using TuneKey = std::tuple<int, int, int, int, int, int, double, int, int>;  // TableKey + eval + n

}  // namespace

// Device scratch of one stream: decodes on different streams run
// concurrently, so each stream gets its own.
struct Workspace {
  int *status = nullptr;    // device status word
  int *counters = nullptr;  // device counters [kNumCounters]
  int *deferred = nullptr;  // device list of deferred mask blocks
  int *binlist = nullptr;   // device queues of the binned paths (4 ints per mask block and frame)
  int deferred_cap = 0;
  float *slots = nullptr;   // global-memory bordered systems
  long long slot_floats = 0;
  int slot_count = 0;
  unsigned long long *bits = nullptr;  // mask selection: one mask word per block
  int *selx = nullptr;                 // and the packing's prefix scratch (blocks + tiles)
  int bits_cap = 0;
};

// Buffers of global homogeneous diffusion inpainting for one plane size:
// the pyramid (levels 1.. : mask, values, solution; level 0 reads the
// caller's mask and values and solves into the caller's output), the CG
// vectors of the finest level (reused by the coarser ones) and the FP64
// scalars GAM[0..max_iter], DEL[0..max_iter], BB (kHdSlots slots each) and
// ALPHA[0..max_iter].
struct DiffWork {
  static constexpr int kMaxLevels = 12;
  int levels = 0;
  int w[kMaxLevels] = {0}, h[kMaxLevels] = {0};
  uint8_t *m[kMaxLevels] = {nullptr};
  float *f[kMaxLevels] = {nullptr}, *u[kMaxLevels] = {nullptr};
  float *p = nullptr, *rv[2] = {nullptr}, *wv[2] = {nullptr}, *sv[2] = {nullptr};  // CG vectors, full size
  double *sc = nullptr;
  int sc_cap = 0;     // doubles in sc
  double *host = nullptr;  // pinned: the slots of GAM[i..] and BB, read back for the convergence test
  int host_cap = 0;        // doubles in host
  hipEvent_t ev = nullptr; // marks the completion of the read-back in flight
  // Iterations each level took in the previous solve of this plane size (0:
  // none yet); a guess that sizes the first batches of launches only.
  int hint[kMaxLevels] = {0};
};

static void free_diff(DiffWork &d) {
  for (int l = 1; l < d.levels; ++l) {
    if (d.m[l]) (void)hipFree(d.m[l]);
    if (d.f[l]) (void)hipFree(d.f[l]);
    if (d.u[l]) (void)hipFree(d.u[l]);
  }
  for (float *p : {d.p, d.rv[0], d.rv[1], d.wv[0], d.wv[1], d.sv[0], d.sv[1]})
    if (p) (void)hipFree(p);
  if (d.sc) (void)hipFree(d.sc);
  if (d.host) (void)hipHostFree(d.host);
  if (d.ev) (void)hipEventDestroy(d.ev);
  d = DiffWork();
}

struct pdi_ctx {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  std::string err;
  std::mutex mu;  // guards the maps and the byte count
  std::map<TableKey, TableSet> tables;
  std::map<hipStream_t, Workspace> ws;
  std::map<TuneKey, int> tune;  // blocks per workgroup of the wave-per-block path
  std::map<std::pair<int, int>, DiffWork> diff;  // per plane size (W, H)
  // decode_residual_batch_noalloc: this device's copy of the static scratch
  // (from hipGetSymbolAddress at pdi_create; null if that failed) and
  // whether a call used it (pdi_sync then reads its status word too)
  void *noalloc = nullptr;
  hipError_t noalloc_err = hipSuccess;
  bool noalloc_used = false;
  // streams and events of the batched wave-per-block path's parts (created
  // on the first such decode; captured decodes do not use them)
  pdi::WideFork wf = {};
  bool wf_ready = false;
};

namespace {

void destroy_wide_fork(pdi::WideFork &w) {
  for (hipStream_t &a : w.aux)
    if (a) (void)hipStreamDestroy(a);
  if (w.fork) (void)hipEventDestroy(w.fork);
  for (hipEvent_t &j : w.join)
    if (j) (void)hipEventDestroy(j);
  w = pdi::WideFork();
}

int set_err(pdi_ctx *c, int code, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

int hip_fail(pdi_ctx *c, hipError_t e, const char *what) {
  return set_err(c, PDI_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int dev_alloc(pdi_ctx *c, void **p, size_t bytes, const char *what) {
  if (c->budget && c->used + bytes > c->budget)
    return set_err(c, PDI_ENOMEM, "%s: %zu bytes exceed the HBM budget (%zu of %zu used)", what,
                   bytes, c->used, c->budget);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return set_err(c, PDI_ENOMEM, "%s: hipMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
  }
  c->used += bytes;
  return PDI_OK;
}

void dev_free(pdi_ctx *c, void *p, size_t bytes) {
  if (p) {
    (void)hipFree(p);
    c->used -= bytes;
  }
}

struct PlaneGeom {
  int W, H;
};

int planes_of(const pdi_frame *f, PlaneGeom *pg) {
  if (f->format == PDI_GRAY) {
    pg[0] = {f->width, f->height};
    return 1;
  }
  int cw = (f->width + 1) / 2, ch = (f->height + 1) / 2;
  pg[0] = {f->width, f->height};
  pg[1] = {cw, ch};
  pg[2] = {cw, ch};
  return 3;
}

// Mask-plane groups: (mask plane, value planes).
int groups_of(const pdi_frame *f, int shared, int mplane[3], int vpl[3][2], int nv[3]) {
  if (f->format == PDI_GRAY) {
    mplane[0] = 0; vpl[0][0] = 0; nv[0] = 1;
    return 1;
  }
  if (shared) {
    mplane[0] = 0; vpl[0][0] = 0; nv[0] = 1;
    mplane[1] = 1; vpl[1][0] = 1; vpl[1][1] = 2; nv[1] = 2;
    return 2;
  }
  for (int g = 0; g < 3; ++g) { mplane[g] = g; vpl[g][0] = g; nv[g] = 1; }
  return 3;
}

int check_geometry(const pdi_frame *f, int b) {
  if (!f) return PDI_EINVAL;
  if (f->width <= 0 || f->height <= 0) return PDI_EINVAL;
  if (f->format != PDI_GRAY && f->format != PDI_YUV420) return PDI_EINVAL;
  if (b != 8 && b != 16 && b != 32) return PDI_EINVAL;
  if ((long long)f->width * f->height > (1LL << 31) / 2) return PDI_EINVAL;
  return PDI_OK;
}

long long mask_blocks_of(const pdi_frame *f, int b, int shared) {
  PlaneGeom pg[3];
  planes_of(f, pg);
  int mp[3], vp[3][2], nv[3];
  int ng = groups_of(f, shared, mp, vp, nv);
  long long n = 0;
  for (int g = 0; g < ng; ++g)
    n += (long long)((pg[mp[g]].W + b - 1) / b) * ((pg[mp[g]].H + b - 1) / b);
  return n;
}

// ---------------------------------------------------------------- tables
//
// For a w x h block with mirrored boundaries the operator is diagonalised by
// the 2D DCT-II (Eq. 4); with the orthonormal basis
//   phi_p(x) = sqrt(om_p) cos(pi p (x + 1/2) / n),  om_0 = 1/n, om_p = 2/n,
// the Green's function is G(x, x') = sum_pq lam_pq phi_p(x) phi_p(x')
// phi_q(y) phi_q(y').  Because phi_p(x) phi_p(x') = om_p/2 [cos(pi p (x-x')/n)
// + cos(pi p (x+x'+1)/n)], G is a quarter of the sum of
//   Hc(alpha, beta) = sum_pq lam_pq om_p om_q cos(pi p alpha/w) cos(pi q beta/h)
// over the four (alpha, beta) pairs built from |x-x'| and x+x'+1 (the latter
// reflected into [0, n] by the 2n period) - the Toeplitz-plus-Hankel
// structure of Sec. 2.2.  The tables below store Hc/4.

double eig_mu(int op, int p, int q, int w, int h) {
  if (op == PDI_OP_CONTINUOUS)
    return kPi * kPi * ((double)p * p / ((double)w * w) + (double)q * q / ((double)h * h));
  double a = std::sin(kPi * p / (2.0 * w)), b = std::sin(kPi * q / (2.0 * h));
  return 4.0 * a * a + 4.0 * b * b;
}

void build_shape_tables(int w, int h, int op, double s, std::vector<double> &lam,
                        std::vector<double> &hc) {
  lam.assign((size_t)w * h, 0.0);
  for (int q = 0; q < h; ++q)
    for (int p = 0; p < w; ++p)
      lam[(size_t)q * w + p] = (p == 0 && q == 0) ? 0.0 : std::pow(eig_mu(op, p, q, w, h), -s);
  // separable evaluation: first over p for every (q, alpha), then over q
  std::vector<double> cw((size_t)(w + 1) * w), ch((size_t)(h + 1) * h);
  for (int a = 0; a <= w; ++a)
    for (int p = 0; p < w; ++p)
      cw[(size_t)a * w + p] = (p == 0 ? 1.0 : 2.0) / w * std::cos(kPi * p * a / w);
  for (int bb = 0; bb <= h; ++bb)
    for (int q = 0; q < h; ++q)
      ch[(size_t)bb * h + q] = (q == 0 ? 1.0 : 2.0) / h * std::cos(kPi * q * bb / h);
  std::vector<double> t((size_t)h * (w + 1));  // t[q][alpha] = sum_p lam_qp cw
  for (int q = 0; q < h; ++q)
    for (int a = 0; a <= w; ++a) {
      double acc = 0.0;
      for (int p = 0; p < w; ++p) acc += lam[(size_t)q * w + p] * cw[(size_t)a * w + p];
      t[(size_t)q * (w + 1) + a] = acc;
    }
  hc.assign((size_t)(w + 1) * (h + 1), 0.0);
  for (int bb = 0; bb <= h; ++bb)
    for (int a = 0; a <= w; ++a) {
      double acc = 0.0;
      for (int q = 0; q < h; ++q) acc += ch[(size_t)bb * h + q] * t[(size_t)q * (w + 1) + a];
      hc[(size_t)bb * (w + 1) + a] = 0.25 * acc;
    }
}

// Orthonormal DCT-II matrix of size n, rows = frequency, cols = position,
// zero padded to m x m, row stride ld >= m.
void dct_padded(int n, int m, int ld, float *out) {
  for (int p = 0; p < m; ++p)
    for (int x = 0; x < ld; ++x) {
      double v = 0.0;
      if (p < n && x < n) v = std::sqrt((p == 0 ? 1.0 : 2.0) / n) * std::cos(kPi * p * (x + 0.5) / n);
      out[p * ld + x] = (float)v;
    }
}

int get_tables(pdi_ctx *c, const pdi_frame *f, int b, int shared, const pdi_params &P,
               TableSet **out) {
  TableKey key{f->width, f->height, f->format, b, shared, P.op, P.s};
  auto it = c->tables.find(key);
  if (it != c->tables.end()) {
    *out = &it->second;
    return PDI_OK;
  }
  TableSet ts;
  PlaneGeom pg[3];
  planes_of(f, pg);
  int mp[3], vp[3][2], nv[3];
  int ng = groups_of(f, shared, mp, vp, nv);
  std::vector<std::pair<int, int>> shapes;
  for (int g = 0; g < ng; ++g) {
    int W = pg[mp[g]].W, H = pg[mp[g]].H;
    int rw = W % b ? W % b : b, rh = H % b ? H % b : b;
    int cand[4][2] = {{b < W ? b : W, b < H ? b : H}, {rw, b < H ? b : H}, {b < W ? b : W, rh}, {rw, rh}};
    for (int k = 0; k < 4; ++k) {
      int id = -1;
      for (size_t t = 0; t < shapes.size(); ++t)
        if (shapes[t].first == cand[k][0] && shapes[t].second == cand[k][1]) id = (int)t;
      if (id < 0) {
        if ((int)shapes.size() >= pdi::kMaxShapes) return set_err(c, PDI_EINVAL, "too many block shapes");
        shapes.push_back({cand[k][0], cand[k][1]});
        id = (int)shapes.size() - 1;
      }
      ts.group_shape[g][k] = id;
    }
  }
  ts.nshapes = (int)shapes.size();
  std::vector<float> t32;
  std::vector<double> t64;
  for (int k = 0; k < ts.nshapes; ++k) {
    int w = shapes[k].first, h = shapes[k].second;
    std::vector<double> lam, hc;
    build_shape_tables(w, h, P.op, P.s, lam, hc);
    pdi::ShapeDev &S = ts.s[k];
    S.w = w;
    S.h = h;
    S.hc32 = (int)t32.size();
    for (double v : hc) t32.push_back((float)v);
    while (t32.size() % 4) t32.push_back(0.f);
    S.hc64 = (int)t64.size();
    for (double v : hc) t64.push_back(v);
    if (b <= 16) {
      // Row-pair table: J[y*jrow + y'*(w+1) + a] = Hc(a,|y-y'|)/4 + Hc(a, refl(y+y'+1))/4,
      // so that G(x, x') = J[..][|x-x'|] + J[..][refl(x+x'+1)].
      const int W1 = w + 1;
      S.fast = (int)t32.size();
      const int JR = pdi::jrow(w, h);
      S.jt_floats = (h * JR + 3) & ~3;
      t32.resize(t32.size() + S.jt_floats + 3 * pdi::kDct16Floats, 0.f);
      float *J = &t32[S.fast];
      for (int y = 0; y < h; ++y)
        for (int y2 = 0; y2 < h; ++y2) {
          int dy = y > y2 ? y - y2 : y2 - y;
          int sy = y + y2 + 1;
          if (sy > h) sy = 2 * h - sy;
          for (int a = 0; a <= w; ++a)
            J[y * JR + y2 * W1 + a] = (float)(hc[(size_t)dy * W1 + a] + hc[(size_t)sy * W1 + a]);
        }
      float *D = J + S.jt_floats;
      dct_padded(w, 16, pdi::kDct16Ld, D);
      dct_padded(h, 16, pdi::kDct16Ld, D + pdi::kDct16Floats);
      for (int q = 0; q < h; ++q)
        for (int p = 0; p < w; ++p)
          D[2 * pdi::kDct16Floats + q * pdi::kDct16Ld + p] = (float)lam[(size_t)q * w + p];
    } else {
      // Compact table, then Dw, Dh and lam zero-padded to 32 x 32 (row stride 33).
      const int W1 = w + 1;
      S.fast = (int)t32.size();
      S.jt_floats = (W1 * (h + 1) + 3) & ~3;
      t32.resize(t32.size() + S.jt_floats + 3 * pdi::kDct32Floats, 0.f);
      float *Hq = &t32[S.fast];
      for (size_t i = 0; i < hc.size(); ++i) Hq[i] = (float)hc[i];
      float *D = Hq + S.jt_floats;
      dct_padded(w, 32, pdi::kDct32Ld, D);
      dct_padded(h, 32, pdi::kDct32Ld, D + pdi::kDct32Floats);
      for (int q = 0; q < h; ++q)
        for (int p = 0; p < w; ++p)
          D[2 * pdi::kDct32Floats + q * pdi::kDct32Ld + p] = (float)lam[(size_t)q * w + p];
    }
  }
  ts.tab32_floats = (int)t32.size();
  t32.resize(t32.size() + pdi::kTabPadFloats, 0.f);  // read-only padding for vector loads
  size_t b32 = t32.size() * sizeof(float), b64 = t64.size() * sizeof(double);
  ts.tab32_floats = (int)t32.size();
  int rc = dev_alloc(c, (void **)&ts.tab32, b32, "tables");
  if (rc) return rc;
  rc = dev_alloc(c, (void **)&ts.tab64, b64, "tables");
  if (rc) { dev_free(c, ts.tab32, b32); return rc; }
  ts.bytes = b32 + b64;
  hipError_t e = hipMemcpy(ts.tab32, t32.data(), b32, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ts.tab64, t64.data(), b64, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dev_free(c, ts.tab32, b32);
    dev_free(c, ts.tab64, b64);
    return hip_fail(c, e, "table upload");
  }
  auto res = c->tables.emplace(key, ts);
  *out = &res.first->second;
  return PDI_OK;
}

// The cached tables of a geometry and operator, or PDI_EINVAL when no call
// has built them yet (never allocates).
int find_tables(pdi_ctx *c, const pdi_frame *f, int b, int shared, const pdi_params &P, TableSet **out) {
  auto it = c->tables.find(TableKey{f->width, f->height, f->format, b, shared, P.op, P.s});
  if (it == c->tables.end())
    return set_err(c, PDI_EINVAL,
                   "no tables for this geometry and operator yet: one decode_residual or decode_residual_batch "
                   "call with them builds them (that call allocates)");
  *out = &it->second;
  return PDI_OK;
}

int get_workspace(pdi_ctx *c, hipStream_t stream, Workspace **out) {
  auto it = c->ws.find(stream);
  if (it != c->ws.end()) {
    *out = &it->second;
    return PDI_OK;
  }
  Workspace w;
  int rc = dev_alloc(c, (void **)&w.status, sizeof(int) * 4, "status");
  if (!rc) rc = dev_alloc(c, (void **)&w.counters, sizeof(int) * pdi::kNumCounters, "counters");
  if (rc) {
    dev_free(c, w.status, sizeof(int) * 4);
    return rc;
  }
  hipError_t e = hipMemset(w.status, 0, sizeof(int) * 4);
  if (e == hipSuccess) e = hipMemset(w.counters, 0, sizeof(int) * pdi::kNumCounters);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "workspace init");
  *out = &c->ws.emplace(stream, w).first->second;
  return PDI_OK;
}

// k_fast2 workgroups for n_items mask blocks x frames: 16 blocks each, every
// one of at most 8 kMaxSegs bins padded to whole workgroups.
long long f2_wgs_max(long long n_items) { return (n_items + 15) / 16 + 8ll * pdi::kMaxSegs; }

// Ints of the queue buffer for n_items mask blocks x frames.  Wave-per-block
// path: 2 per block.  Binned wave-level path: the entries (4 ints for each of
// the 16 slots of every k_fast2 workgroup), the workgroup descriptors (2
// ints), then the binning's per-workgroup bin counts (kMaxSegs * 8 bins for
// each workgroup of 256 blocks of one frame; at most 32 frames add a partial
// workgroup each).
long long f2_desc_ints(long long n_items) { return (2 * f2_wgs_max(n_items) + 3) & ~3ll; }
long long binlist_ints(long long n_items) {
  return 64 * f2_wgs_max(n_items) + f2_desc_ints(n_items) + 8ll * pdi::kMaxSegs * (n_items / 256 + 33);
}

int ensure_workspace(pdi_ctx *c, Workspace *W, int n_items, int b, int nslots) {
  if (n_items > W->deferred_cap) {
    dev_free(c, W->deferred, sizeof(int) * (size_t)W->deferred_cap);
    dev_free(c, W->binlist, sizeof(int) * (size_t)binlist_ints(W->deferred_cap));
    W->deferred = W->binlist = nullptr;
    W->deferred_cap = 0;
    int rc = dev_alloc(c, (void **)&W->deferred, sizeof(int) * (size_t)n_items, "deferred list");
    if (!rc) rc = dev_alloc(c, (void **)&W->binlist, sizeof(int) * (size_t)binlist_ints(n_items), "block queues");
    if (rc) return rc;
    W->deferred_cap = n_items;
  }
  // Global-memory bordered systems: (K+1) rows of K+1+2 floats with
  // K <= b*b (decodes copy the values when K = b*b; encodes solve), one slot
  // per workgroup that may need one.
  const int nmax = b * b;
  const long long need = (long long)(nmax + 1) * (nmax + 3);
  if (nslots < pdi::kDeferredGrid) nslots = pdi::kDeferredGrid;
  if (need > W->slot_floats || nslots > W->slot_count) {
    const long long nf = need > W->slot_floats ? need : W->slot_floats;
    const int ns = nslots > W->slot_count ? nslots : W->slot_count;
    dev_free(c, W->slots, sizeof(float) * (size_t)W->slot_floats * (size_t)W->slot_count);
    W->slots = nullptr;
    W->slot_floats = 0;
    W->slot_count = 0;
    int rc = dev_alloc(c, (void **)&W->slots, sizeof(float) * (size_t)nf * (size_t)ns, "system slots");
    if (rc) return rc;
    W->slot_floats = nf;
    W->slot_count = ns;
  }
  return PDI_OK;
}

}  // namespace

extern "C" {

void pdi_default_params(pdi_params *p) {
  if (!p) return;
  p->op = PDI_OP_DISCRETE;
  p->s = 1.0;
  p->eval_dtype = PDI_EVAL_FP32;
  p->refine = 1;
  p->validate = 0;
  p->out_int8 = 0;
  p->path = PDI_PATH_AUTO;
  p->refine_tau = 1.0 / 64.0;
}

int pdi_create(pdi_ctx **out, int device, size_t hbm_budget_bytes) {
  if (!out) return PDI_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PDI_EINVAL;
  pdi_ctx *c = new (std::nothrow) pdi_ctx();
  if (!c) return PDI_ENOMEM;
  c->device = device;
  c->budget = hbm_budget_bytes;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) { delete c; return PDI_EHIP; }
  // The device address of this device's static scratch (no allocation);
  // a failure only disables decode_residual_batch_noalloc.
  c->noalloc_err = pdi::noalloc_setup(device, &c->noalloc);
  if (c->noalloc_err != hipSuccess) c->noalloc = nullptr;
  *out = c;
  return PDI_OK;
}

void pdi_destroy(pdi_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  destroy_wide_fork(c->wf);
  for (auto &kv : c->tables) {
    (void)hipFree(kv.second.tab32);
    (void)hipFree(kv.second.tab64);
  }
  for (auto &kv : c->ws) {
    (void)hipFree(kv.second.status);
    (void)hipFree(kv.second.counters);
    (void)hipFree(kv.second.deferred);
    (void)hipFree(kv.second.binlist);
    (void)hipFree(kv.second.slots);
    (void)hipFree(kv.second.bits);
    (void)hipFree(kv.second.selx);
  }
  for (auto &kv : c->diff) free_diff(kv.second);
  delete c;
}

const char *pdi_last_error(pdi_ctx *c) { return c ? c->err.c_str() : "null context"; }

int pdi_frame_info(const pdi_frame *frame, int block_size, int chroma_shared,
                   int32_t *n_mask_blocks, int64_t *out_elems) {
  if (check_geometry(frame, block_size)) return PDI_EINVAL;
  PlaneGeom pg[3];
  int np = planes_of(frame, pg);
  if (n_mask_blocks) *n_mask_blocks = (int32_t)mask_blocks_of(frame, block_size, chroma_shared && frame->format == PDI_YUV420);
  if (out_elems) {
    int64_t n = 0;
    for (int i = 0; i < np; ++i) n += (int64_t)pg[i].W * pg[i].H;
    *out_elems = n;
  }
  return PDI_OK;
}

// Mask groups of a frame (the plane each mask lives on, its value planes,
// offsets of those planes in the concatenated planes and in consts[], block
// grid, shape ids) into F.g; F.chroma_first is the first chroma block.
static void fill_groups(const pdi_frame *frame, int block_size, int shared, const TableSet *ts, pdi::FrameDev &F) {
  PlaneGeom pg[3];
  planes_of(frame, pg);
  long long poff[3] = {0, 0, 0};
  int pbo[3] = {0, 0, 0};  // first block of each plane in consts[]
  for (int i = 1; i < 3; ++i) {
    poff[i] = poff[i - 1] + (long long)pg[i - 1].W * pg[i - 1].H;
    pbo[i] = pbo[i - 1] + ((pg[i - 1].W + block_size - 1) / block_size) * ((pg[i - 1].H + block_size - 1) / block_size);
  }
  int mp[3], vp[3][2], nv[3];
  F.ngroups = groups_of(frame, shared, mp, vp, nv);
  int first = 0;
  F.chroma_first = -1;
  for (int g = 0; g < F.ngroups; ++g) {
    pdi::GroupDev &G = F.g[g];
    G.first = first;
    G.W = pg[mp[g]].W;
    G.H = pg[mp[g]].H;
    G.nbx = (G.W + block_size - 1) / block_size;
    G.nby = (G.H + block_size - 1) / block_size;
    G.nv = nv[g];
    for (int k = 0; k < nv[g]; ++k) {
      G.vplane[k] = vp[g][k];
      G.out_off[k] = poff[vp[g][k]];
      G.cbase[k] = pbo[vp[g][k]];
    }
    for (int k = 0; k < 4; ++k) G.shape[k] = ts->group_shape[g][k];
    if (mp[g] == 1) F.chroma_first = first;
    first += G.nbx * G.nby;
  }
}

// Decode n frames of one geometry (one launch per kernel for all of them):
// residual decodes (values, qp == nullptr), stored-coefficient decodes
// (coefs + consts, qp != nullptr) or coefficient encodes (qouts + aouts).
// With `scratch` (residual decodes only) the decode's device scratch is
// carved from that static array and nothing is allocated.
static int decode_impl(pdi_ctx *c, int n, const pdi_frame *frame, const pdi_mask *masks,
                       const float *const *values, int block_size, const pdi_params *params,
                       float *const *outs, void *stream, const int8_t *const *coefs = nullptr,
                       const float *const *consts = nullptr, const pdi_coef_params *qp = nullptr,
                       int8_t *const *qouts = nullptr, float *const *aouts = nullptr, void *scratch = nullptr) {
  if (!c) return PDI_EINVAL;
  const bool enc = qouts != nullptr;        // coefficient encode: values in, codes + constants out
  const bool coef = qp != nullptr && !enc;  // stored-coefficient decode
  if (n < 1 || n > pdi::kMaxBatch) return set_err(c, PDI_EINVAL, "batch of %d frames (1..%d)", n, pdi::kMaxBatch);
  if (enc ? (!frame || !masks || !values || !aouts || !qp)
          : (!frame || !masks || !outs || (coef ? (!coefs || !consts) : !values)))
    return set_err(c, PDI_EINVAL, enc ? "null frame, mask, values, quantiser params, codes or constants"
                                  : coef ? "null frame, mask, coefficients, constants or out"
                                         : "null frame, mask, values or out");
  if (enc) {
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(qp->step[k]) || !(qp->step[k] > 0.f)) return set_err(c, PDI_EINVAL, "bad quantiser step");
  } else if (coef) {
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(qp->step[k]) || qp->step[k] < 0.f) return set_err(c, PDI_EINVAL, "bad quantiser step");
    if (!(qp->rho >= 0.f) || !(qp->rho < 1.f)) return set_err(c, PDI_EINVAL, "rho must be in [0, 1)");
  }
  const pdi_mask *mask = &masks[0];
  if (check_geometry(frame, block_size))
    return set_err(c, PDI_EINVAL, "bad geometry %dx%d format %d block %d", frame->width,
                   frame->height, frame->format, block_size);
  pdi_params P;
  pdi_default_params(&P);
  if (params) P = *params;
  if (P.op != PDI_OP_DISCRETE && P.op != PDI_OP_CONTINUOUS) return set_err(c, PDI_EINVAL, "bad op");
  if (!(P.s > 0.0) || !(P.s <= 8.0)) return set_err(c, PDI_EINVAL, "s must be in (0, 8]");
  if (P.eval_dtype < PDI_EVAL_FP32 || P.eval_dtype > PDI_EVAL_BF16X2) return set_err(c, PDI_EINVAL, "bad eval_dtype");
  if (P.refine < 0 || P.refine > 2) return set_err(c, PDI_EINVAL, "bad refine");
  if (P.path != PDI_PATH_AUTO && P.path != PDI_PATH_PLAIN) return set_err(c, PDI_EINVAL, "bad path");
  if (!(P.refine_tau >= 0.0) || !(P.refine_tau <= 1.0)) return set_err(c, PDI_EINVAL, "bad refine_tau");
  if (P.out_int8 != 0 && P.out_int8 != 1) return set_err(c, PDI_EINVAL, "bad out_int8");
  int shared = (frame->format == PDI_YUV420 && mask->chroma_shared) ? 1 : 0;
  long long nitems = mask_blocks_of(frame, block_size, shared);
  if (nitems > pdi::kDeferItemMask) return set_err(c, PDI_EINVAL, "%lld mask blocks (at most %d)", nitems, pdi::kDeferItemMask);
  for (int k = 0; k < n; ++k) {
    const pdi_mask &mk = masks[k];
    const int sh = (frame->format == PDI_YUV420 && mk.chroma_shared) ? 1 : 0;
    if (sh != shared) return set_err(c, PDI_EINVAL, "frame %d: chroma sharing differs within the batch", k);
    if (nitems != mk.n_mask_blocks)
      return set_err(c, PDI_EINVAL, "n_mask_blocks %d, geometry needs %lld", mk.n_mask_blocks, nitems);
    if (enc ? (!mk.block_ptr || !mk.pos || !values[k] || !qouts[k] || !aouts[k])
            : (!mk.block_ptr || !mk.pos || !outs[k] || (coef ? (!coefs[k] || !consts[k]) : !values[k])))
      return set_err(c, PDI_EINVAL, "frame %d: null block_ptr, pos, %s", k,
                     enc ? "values, codes or constants" : coef ? "coefficients, constants or out" : "values or out");
  }
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  std::lock_guard<std::mutex> lock(c->mu);
  hipStream_t s = (hipStream_t)stream;
  Workspace SW;  // static-scratch decodes: the pieces of the static array
  Workspace *W = &SW;
  if (!scratch) {
    int rcw = get_workspace(c, s, &W);
    if (rcw) return rcw;
  }

  TableSet *ts = nullptr;
  int rc = scratch ? find_tables(c, frame, block_size, shared, P, &ts) : get_tables(c, frame, block_size, shared, P, &ts);
  if (rc) return rc;

  pdi::FrameDev F;
  std::memset(&F, 0, sizeof F);
  F.b = block_size;
  F.n_items = (int)nitems;
  F.shared = shared;
  F.validate = P.validate ? 1 : 0;
  F.refine = P.refine;
  F.tau = (float)P.refine_tau;
  F.eval = P.eval_dtype;
  F.out_i8 = P.out_int8;
  F.coef = coef ? 1 : 0;
  F.enc = enc ? 1 : 0;
  if (coef || enc) {
    for (int k = 0; k < 3; ++k) F.qstep[k] = qp->step[k];
    F.qrho = qp->rho;
  }
  fill_groups(frame, block_size, shared, ts, F);
  F.nshapes = ts->nshapes;
  for (int k = 0; k < ts->nshapes; ++k) F.s[k] = ts->s[k];
  // Shape-homogeneous runs of blocks for the batched paths: k_fast (b <= 16,
  // 16 blocks per workgroup) or k_wide (b = 32, 4 blocks per workgroup).
  // Stored-coefficient decodes always take the batched paths (no solve);
  // encodes take k_fast for b <= 16 and the per-block path for b = 32.
  const bool fast = ((coef || P.path == PDI_PATH_AUTO) && block_size <= 16);
  const bool wide = ((coef || P.path == PDI_PATH_AUTO) && block_size == 32 && !enc);
  int ipw = fast ? pdi::kFastItemsPerWG : pdi::kWideItemsDefault;
  if (!coef && !enc) {
    auto it = c->tune.find(TuneKey{frame->width, frame->height, frame->format, block_size, shared, P.op, P.s,
                                   P.eval_dtype, n});
    if (it != c->tune.end()) ipw = it->second;
  }
  F.ipw = ipw;
  int shape_count[pdi::kMaxShapes] = {0};
  const int dct_floats = fast ? 3 * pdi::kDct16Floats : 3 * pdi::kDct32Floats;
  F.nsegs = 0;
  F.fast_wgs = 0;
  F.fast_lds = 0;
  for (int g = 0; g < F.ngroups; ++g) {
    const pdi::GroupDev &G = F.g[g];
    const int b = block_size, nbxf = G.W / b, nbyf = G.H / b;
    const int rw = G.W % b, rh = G.H % b;
    const int segs[4][4] = {{0, nbxf, 0, nbyf},                      // full
                            {nbxf, rw ? 1 : 0, 0, nbyf},             // right edge
                            {0, nbxf, nbyf, rh ? 1 : 0},             // bottom edge
                            {nbxf, rw ? 1 : 0, nbyf, rh ? 1 : 0}};   // corner
    for (int e = 0; e < 4; ++e) {
      const int nx = segs[e][1], ny = segs[e][3];
      if (nx <= 0 || ny <= 0) continue;
      F.qge[g][e] = F.nsegs;
      pdi::SegDev &S = F.seg[F.nsegs++];
      S.group = g;
      S.shape = G.shape[e];
      S.bx0 = segs[e][0];
      S.nx = nx;
      S.by0 = segs[e][2];
      S.count = nx * ny;
      S.first_wg = F.fast_wgs;
      F.fast_wgs += (S.count + ipw - 1) / ipw;
      shape_count[S.shape] += S.count;
      const pdi::ShapeDev &SH = ts->s[S.shape];
      const int need = (coef ? 0 : SH.jt_floats) + dct_floats;  // coef: the matrices only
      if (need > F.fast_lds) F.fast_lds = need;
    }
  }
  // Batched residual decodes with b <= 16 take the binned path (k_fbin +
  // k_fast2): one queue per segment (mask-plane group and edge kind) with
  // four regions of its blocks x frames entries (two size classes each),
  // k_fast2 workgroups for every queued block plus one partial workgroup
  // per bin.  A binned queue keeps its group in first_wg.
  // (A batch of few blocks keeps k_fast: its one launch costs less than the
  // binned path's five; config 0, 32 grey 256 x 256 frames = 8192 blocks:
  // 28 us per batch against 41 us.)
  const bool binned = fast && !coef && !enc && n > 1 && nitems * n >= kBinnedMinBlocks;
  if (binned) {
    F.nq = 0;
    for (int k = 0; k < F.nsegs; ++k) {
      const pdi::SegDev &S = F.seg[k];
      pdi::QueueDev &Q = F.q[F.nq];
      Q.shape = S.shape;
      Q.count = S.count;
      Q.base = 0;
      Q.first_wg = S.group;
      F.nq++;  // queue k is segment k (F.qge was filled with the segments)
    }
    F.fast_wgs = (int)((nitems * n + 15) / 16) + 8 * F.nq;  // k_fast2 takes 16 blocks per workgroup
  }
  if (wide) {
    // One queue per block shape, the smallest first so that the few edge
    // blocks start early; each queue's workgroups follow one another.
    int order[pdi::kMaxShapes], nq = 0;
    for (int sh = 0; sh < ts->nshapes; ++sh)
      if (shape_count[sh] > 0) order[nq++] = sh;
    std::sort(order, order + nq, [&](int a, int b) { return shape_count[a] < shape_count[b]; });
    int base = 0, wgs = 0;
    for (int i = 0; i < nq; ++i) {
      pdi::QueueDev &Q = F.q[i];
      Q.shape = order[i];
      Q.count = shape_count[order[i]];
      Q.base = base;
      Q.first_wg = wgs;
      base += Q.count;
      wgs += (Q.count + ipw - 1) / ipw;
      F.qof[order[i]] = i;
    }
    F.nq = nq;
    F.fast_wgs = wgs;
  }
  F.slot_wgs = pdi::kDeferredGrid;
  if (scratch) {
    // status word, counters, deferred list, queues (wave-per-block path),
    // then as many global-memory systems as fit, up to one per workgroup of
    // the deferred pass that takes them
    auto up = [](long long x) { return (x + 255) & ~255ll; };
    const long long items = nitems * n, nmax = (long long)block_size * block_size;
    const long long slot_floats = (nmax + 1) * (nmax + 3);
    long long off = pdi::kNoAllocHeadBytes;
    const long long def_off = off;
    off += up(4 * items);
    const long long bin_off = off;
    if (wide) off += up(8 * items);
    if (binned) off += up(4 * binlist_ints(items));
    const long long room = pdi::kNoAllocScratchBytes - off;
    const long long nsl = room > 0 ? std::min<long long>(pdi::kDeferredGrid, room / (4 * slot_floats)) : 0;
    if (nsl < 1)
      return set_err(c, PDI_ENOMEM,
                     "%d frames of %lld mask blocks with %dx%d blocks need %lld bytes of scratch; the static "
                     "scratch holds %lld", n, nitems, block_size, block_size, off + 4 * slot_floats,
                     (long long)pdi::kNoAllocScratchBytes);
    char *base = static_cast<char *>(scratch);
    W->status = reinterpret_cast<int *>(base);
    W->counters = reinterpret_cast<int *>(base + pdi::kNoAllocCountersOff);
    W->deferred = reinterpret_cast<int *>(base + def_off);
    W->binlist = (wide || binned) ? reinterpret_cast<int *>(base + bin_off) : nullptr;
    W->slots = reinterpret_cast<float *>(base + off);
    W->slot_floats = slot_floats;
    F.slot_wgs = (int)nsl;
  } else {
    rc = ensure_workspace(c, W, (int)nitems * n, block_size, fast ? F.fast_wgs : 0);
    if (rc) return rc;
  }
  F.tab32_floats = ts->tab32_floats;
  F.nframes = n;
  // A single frame's k_fast workgroups decode their leftover blocks in their
  // own global slots; static-scratch decodes hand them to the deferred pass.
  F.tail_in_wg = (n == 1 && !coef && !enc && !scratch) ? 1 : 0;
  for (int k = 0; k < n; ++k) {
    F.fp[k].block_ptr = masks[k].block_ptr;
    F.fp[k].pos = masks[k].pos;
    F.fp[k].values = coef ? nullptr : values[k];
    F.fp[k].out = enc ? nullptr : outs[k];
    F.fp[k].coef = coef ? coefs[k] : nullptr;
    F.fp[k].consts = coef ? consts[k] : nullptr;
    F.fp[k].qout = enc ? qouts[k] : nullptr;
    F.fp[k].aout = enc ? aouts[k] : nullptr;
  }
  F.tab32 = ts->tab32;
  F.tab64 = ts->tab64;
  F.deferred = W->deferred;
  F.binlist = W->binlist;
  F.fl = binned ? W->binlist : nullptr;
  F.wgdesc = binned ? F.fl + 64 * f2_wgs_max(nitems * n) : nullptr;
  F.hist = binned ? F.wgdesc + f2_desc_ints(nitems * n) : nullptr;
  F.counters = W->counters;
  F.status = W->status;
  F.slots = W->slots;
  F.slot_floats = W->slot_floats;

  if (coef) {
    // Batched kernels, then the blocks with more points than they stage.
    e = fast ? pdi::launch_fast(F, s) : pdi::launch_wide(F, s);
    if (e == hipSuccess) e = pdi::launch_coef_general(F, s);
  } else if (binned) {
    // binning, the binned wave-level kernel, then the deferred blocks
    e = pdi::launch_fast2(F, s);
    if (e == hipSuccess) e = pdi::launch_general_deferred(F, s);
  } else if (fast) {
    // A single frame: one launch, the workgroups also decode their leftover
    // blocks.  An encode: leftover blocks go to the deferred pass.
    e = pdi::launch_fast(F, s);
    if (e == hipSuccess && !F.tail_in_wg) e = pdi::launch_general_deferred(F, s);
  } else if (wide) {
    // Batches run the parts side by side on the context's streams, except
    // for static-scratch decodes and inside a graph capture (forking a
    // capture onto streams shared by every caller crashed the runtime when a
    // capture spanned several caller streams; captured decodes keep the
    // parts in order on the caller's stream).
    const pdi::WideFork *fork = nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusActive;
    if (n > 1 && !scratch && hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      if (!c->wf_ready) {
        pdi::WideFork w = {};
        hipError_t ce = hipSuccess;
        for (int i = 0; i < pdi::kWideAux && ce == hipSuccess; ++i)
          ce = hipStreamCreateWithFlags(&w.aux[i], hipStreamNonBlocking);
        if (ce == hipSuccess) ce = hipEventCreateWithFlags(&w.fork, hipEventDisableTiming);
        for (int i = 0; i < pdi::kWideAux && ce == hipSuccess; ++i)
          ce = hipEventCreateWithFlags(&w.join[i], hipEventDisableTiming);
        if (ce != hipSuccess) {
          destroy_wide_fork(w);
          return hip_fail(c, ce, "streams of the wave-per-block parts");
        }
        c->wf = w;
        c->wf_ready = true;
      }
      fork = &c->wf;
    }
    e = pdi::launch_wide(F, s, fork);  // leftover blocks go to the deferred list
    if (e == hipSuccess) e = pdi::launch_general_deferred(F, s);
  } else {
    e = pdi::launch_plain_all(F, s);
    if (e == hipSuccess) e = pdi::launch_general_deferred(F, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return PDI_OK;
}

int decode_residual(pdi_ctx *c, const pdi_frame *frame, const pdi_mask *mask, const float *values,
                    int block_size, const pdi_params *params, float *out, void *stream) {
  if (c && (!mask || !out)) return set_err(c, PDI_EINVAL, "null frame, mask or out");
  return decode_impl(c, 1, frame, mask, &values, block_size, params, &out, stream);
}

int decode_residual_batch(pdi_ctx *c, int n, const pdi_frame *frame, const pdi_mask *masks,
                          const float *const *values, int block_size, const pdi_params *params,
                          float *const *outs, void *stream) {
  return decode_impl(c, n, frame, masks, values, block_size, params, outs, stream);
}

int decode_residual_batch_noalloc(pdi_ctx *c, int n, const pdi_frame *frame, const pdi_mask *masks,
                                  const float *const *values, int block_size, const pdi_params *params,
                                  float *const *outs, void *stream) {
  if (!c) return PDI_EINVAL;
  if (!c->noalloc)
    return set_err(c, PDI_EHIP, "static scratch unavailable: %s", hipGetErrorString(c->noalloc_err));
  {
    std::lock_guard<std::mutex> lock(c->mu);
    c->noalloc_used = true;
  }
  return decode_impl(c, n, frame, masks, values, block_size, params, outs, stream, nullptr, nullptr, nullptr,
                     nullptr, nullptr, c->noalloc);
}

int decode_coefficients(pdi_ctx *c, const pdi_frame *frame, const pdi_mask *mask, const int8_t *coef,
                        const float *consts, const pdi_coef_params *qp, int block_size,
                        const pdi_params *params, float *out, void *stream) {
  if (c && (!mask || !out || !qp)) return set_err(c, PDI_EINVAL, "null mask, quantiser params or out");
  return decode_impl(c, 1, frame, mask, nullptr, block_size, params, &out, stream, &coef, &consts, qp);
}

int decode_coefficients_batch(pdi_ctx *c, int n, const pdi_frame *frame, const pdi_mask *masks,
                              const int8_t *const *coefs, const float *const *consts,
                              const pdi_coef_params *qp, int block_size, const pdi_params *params,
                              float *const *outs, void *stream) {
  if (c && !qp) return set_err(c, PDI_EINVAL, "null quantiser params");
  return decode_impl(c, n, frame, masks, nullptr, block_size, params, outs, stream, coefs, consts, qp);
}

int encode_coefficients(pdi_ctx *c, const pdi_frame *frame, const pdi_mask *mask, const float *values,
                        const pdi_coef_params *qp, int block_size, const pdi_params *params, int8_t *coef,
                        float *consts, void *stream) {
  if (c && (!mask || !coef || !consts)) return set_err(c, PDI_EINVAL, "null mask, codes or constants");
  return decode_impl(c, 1, frame, mask, &values, block_size, params, nullptr, stream, nullptr, nullptr, qp, &coef,
                     &consts);
}

int encode_coefficients_batch(pdi_ctx *c, int n, const pdi_frame *frame, const pdi_mask *masks,
                              const float *const *values, const pdi_coef_params *qp, int block_size,
                              const pdi_params *params, int8_t *const *coefs, float *const *consts, void *stream) {
  if (c && (!coefs || !consts)) return set_err(c, PDI_EINVAL, "null codes or constants");
  return decode_impl(c, n, frame, masks, values, block_size, params, nullptr, stream, nullptr, nullptr, qp, coefs,
                     consts);
}

void pdi_default_select_params(pdi_select_params *p) {
  if (!p) return;
  p->threshold[0] = 16.0f;
  p->threshold[1] = 32.0f;
  p->max_rounds = 16;
}

int select_mask(pdi_ctx *c, const pdi_frame *frame, int chroma_shared, const float *planes, int block_size,
                const pdi_select_params *sp, int32_t *block_ptr, uint16_t *pos, float *values, void *stream) {
  if (!c) return PDI_EINVAL;
  if (!frame || !planes || !block_ptr || !pos || !values)
    return set_err(c, PDI_EINVAL, "null frame, planes, block_ptr, pos or values");
  if (block_size != 8) return set_err(c, PDI_EINVAL, "mask selection takes 8x8 blocks (block %d)", block_size);
  if (check_geometry(frame, block_size))
    return set_err(c, PDI_EINVAL, "bad geometry %dx%d format %d", frame->width, frame->height, frame->format);
  pdi_select_params S;
  pdi_default_select_params(&S);
  if (sp) S = *sp;
  if (std::isnan(S.threshold[0]) || std::isnan(S.threshold[1])) return set_err(c, PDI_EINVAL, "NaN threshold");
  if (S.max_rounds < 0 || S.max_rounds > 64) return set_err(c, PDI_EINVAL, "max_rounds must be in [0, 64]");
  const int shared = (frame->format == PDI_YUV420 && chroma_shared) ? 1 : 0;
  const long long nitems = mask_blocks_of(frame, block_size, shared);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  std::lock_guard<std::mutex> lock(c->mu);
  hipStream_t s = (hipStream_t)stream;
  Workspace *W = nullptr;
  int rc = get_workspace(c, s, &W);
  if (rc) return rc;
  if (W->bits_cap < nitems) {
    dev_free(c, W->bits, sizeof(unsigned long long) * (size_t)W->bits_cap);
    dev_free(c, W->selx, sizeof(int) * (size_t)(W->bits_cap + W->bits_cap / 256 + 1));
    W->bits = nullptr;
    W->selx = nullptr;
    W->bits_cap = 0;
    rc = dev_alloc(c, (void **)&W->bits, sizeof(unsigned long long) * (size_t)nitems, "mask words");
    if (!rc) rc = dev_alloc(c, (void **)&W->selx, sizeof(int) * (size_t)(nitems + nitems / 256 + 1), "mask words");
    if (rc) return rc;
    W->bits_cap = (int)nitems;
  }
  pdi_params P;  // the residual operator: harmonic, discrete 5-point eigenvalues
  pdi_default_params(&P);
  TableSet *ts = nullptr;
  rc = get_tables(c, frame, block_size, shared, P, &ts);
  if (rc) return rc;
  pdi::FrameDev F;
  std::memset(&F, 0, sizeof F);
  F.b = block_size;
  F.n_items = (int)nitems;
  F.shared = shared;
  F.nframes = 1;
  fill_groups(frame, block_size, shared, ts, F);
  F.nshapes = ts->nshapes;
  for (int k = 0; k < ts->nshapes; ++k) F.s[k] = ts->s[k];
  F.tab32 = ts->tab32;
  F.tab64 = ts->tab64;
  F.tab32_floats = ts->tab32_floats;
  F.status = W->status;
  F.counters = W->counters;
  F.sel_planes = planes;
  F.sel_bits = W->bits;
  F.sel_x = W->selx;
  F.sel_bp = block_ptr;
  F.sel_pos = pos;
  F.sel_vals = values;
  F.sel_thr[0] = S.threshold[0];
  F.sel_thr[1] = S.threshold[1];
  F.sel_rounds = S.max_rounds;
  e = pdi::launch_select(F, s);
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return PDI_OK;
}

int pdi_sync(pdi_ctx *c, void *stream) {
  if (!c) return PDI_EINVAL;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  std::lock_guard<std::mutex> lock(c->mu);
  // the stream's workspace (if it decoded anything) and, once static-scratch
  // decodes ran, the status word of the device's static scratch
  int *status[2] = {nullptr, nullptr}, *counters[2] = {nullptr, nullptr};
  auto it = c->ws.find((hipStream_t)stream);
  if (it != c->ws.end()) {
    status[0] = it->second.status;
    counters[0] = it->second.counters;
  }
  if (c->noalloc_used) {
    status[1] = static_cast<int *>(c->noalloc);
    counters[1] = reinterpret_cast<int *>(static_cast<char *>(c->noalloc) + pdi::kNoAllocCountersOff);
  }
  int st = 0;
  for (int k = 0; k < 2; ++k) {
    if (!status[k]) continue;
    int sk = 0;
    e = hipMemcpy(&sk, status[k], sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "status read");
    if (!sk) continue;
    st |= sk;
    e = hipMemset(status[k], 0, sizeof(int));
    if (e == hipSuccess) e = hipMemset(counters[k], 0, sizeof(int) * pdi::kNumCounters);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "status reset");
  }
  if (st) {
    if (st & pdi::kStatusMask) return set_err(c, PDI_EMASK, "device validation: bad mask positions");
    if (st & pdi::kStatusValue) return set_err(c, PDI_EVALUE, "device validation: non-finite value");
    return set_err(c, PDI_ESOLVE, "a block system broke down (non-finite solution)");
  }
  return PDI_OK;
}

int pdi_autotune_batch(pdi_ctx *c, int n, const pdi_frame *frame, const pdi_mask *masks,
                       const float *const *values, int block_size, const pdi_params *params,
                       float *const *outs, void *stream, int *choice) {
  if (!c || !frame || !masks || !values || !outs) return PDI_EINVAL;
  if (n < 1 || n > pdi::kMaxBatch) return set_err(c, PDI_EINVAL, "batch of %d frames (1..%d)", n, pdi::kMaxBatch);
  pdi_params P;
  pdi_default_params(&P);
  if (params) P = *params;
  const int shared = (frame->format == PDI_YUV420 && masks[0].chroma_shared) ? 1 : 0;
  const TuneKey key{frame->width, frame->height, frame->format, block_size, shared, P.op, P.s, P.eval_dtype, n};
  if (choice) *choice = 0;
  // Launch choices: blocks per workgroup of the batched path (k_fast: up to
  // 16, fewer spread the blocks more evenly over the compute units; k_wide:
  // waves per workgroup, one block per wave).  The plain path has none.
  auto run = [&]() { return decode_impl(c, n, frame, masks, values, block_size, params, outs, stream); };
  if (P.path != PDI_PATH_AUTO) {
    int rc = run();
    return rc ? rc : pdi_sync(c, stream);
  }
  static const int fast_cands[] = {16, 14, 13, 12, 10, 8};
  static const int wide_cands[] = {1, 2, 4};
  const int *cands = block_size == 32 ? wide_cands : fast_cands;
  const int ncand = block_size == 32 ? 3 : 6;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(c, e, "autotune events");
  }
  // Two sweeps over the candidates, the fastest time of each kept, so that
  // a transient slowdown during one candidate's timing does not decide.
  float best_ms[8];
  for (int ci = 0; ci < ncand; ++ci) best_ms[ci] = 3.0e38f;
  int rc = PDI_OK;
  const int reps = 8;
  for (int sweep = 0; sweep < 2 && rc == PDI_OK && e == hipSuccess; ++sweep) {
    for (int ci = 0; ci < ncand; ++ci) {
      {
        std::lock_guard<std::mutex> lock(c->mu);
        c->tune[key] = cands[ci];
      }
      for (int r = 0; r < 2 && rc == PDI_OK; ++r) rc = run();
      if (rc == PDI_OK) rc = pdi_sync(c, stream);
      if (rc != PDI_OK) break;
      e = hipEventRecord(e0, s);
      for (int r = 0; r < reps && rc == PDI_OK; ++r) rc = run();
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess || rc != PDI_OK) break;
      best_ms[ci] = std::min(best_ms[ci], ms);
    }
  }
  int best = cands[0];
  float bms = best_ms[0];
  for (int ci = 1; ci < ncand; ++ci)
    if (best_ms[ci] < bms) {
      bms = best_ms[ci];
      best = cands[ci];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> lock(c->mu);
    c->tune[key] = best;
  }
  if (rc != PDI_OK) return rc;
  if (e != hipSuccess) return hip_fail(c, e, "autotune timing");
  if (choice) *choice = best;
  return pdi_sync(c, stream);
}

int pdi_autotune(pdi_ctx *c, const pdi_frame *frame, const pdi_mask *mask, const float *values,
                 int block_size, const pdi_params *params, float *out, void *stream, int *choice) {
  if (!c || !frame || !mask || !out) return PDI_EINVAL;
  return pdi_autotune_batch(c, 1, frame, mask, &values, block_size, params, &out, stream, choice);
}

int pdi_validate_host(const pdi_frame *frame, int block_size, const int32_t *block_ptr,
                      const uint16_t *pos, int32_t n_mask_blocks, int32_t chroma_shared,
                      const float *values) {
  if (check_geometry(frame, block_size) || !block_ptr) return PDI_EINVAL;
  int shared = (frame->format == PDI_YUV420 && chroma_shared) ? 1 : 0;
  if (mask_blocks_of(frame, block_size, shared) != n_mask_blocks) return PDI_EINVAL;
  PlaneGeom pg[3];
  planes_of(frame, pg);
  int mp[3], vp[3][2], nv[3];
  int ng = groups_of(frame, shared, mp, vp, nv);
  if (block_ptr[0] != 0) return PDI_EMASK;
  int m = 0;
  long long chroma_first_ptr = -1, chroma_nnz = 0;
  for (int g = 0; g < ng; ++g) {
    int W = pg[mp[g]].W, H = pg[mp[g]].H, b = block_size;
    if (mp[g] == 1) chroma_first_ptr = block_ptr[m];
    for (int by = 0; by < (H + b - 1) / b; ++by)
      for (int bx = 0; bx < (W + b - 1) / b; ++bx, ++m) {
        int w = W - bx * b < b ? W - bx * b : b, h = H - by * b < b ? H - by * b : b;
        int lo = block_ptr[m], hi = block_ptr[m + 1];
        if (hi < lo || hi - lo > w * h) return PDI_EMASK;
        if (!pos && hi > lo) return PDI_EINVAL;
        for (int i = lo; i < hi; ++i) {
          if (pos[i] >= w * h) return PDI_EMASK;
          if (i > lo && pos[i] <= pos[i - 1]) return PDI_EMASK;
        }
      }
  }
  long long nnz = block_ptr[n_mask_blocks];
  if (shared) chroma_nnz = nnz - chroma_first_ptr;
  long long nval = nnz + chroma_nnz;
  if (nval > 0 && !values) return PDI_EINVAL;
  for (long long i = 0; i < nval; ++i)
    if (!std::isfinite(values[i])) return PDI_EVALUE;
  return PDI_OK;
}

int pdi_pack_dense(const pdi_frame *frame, const uint8_t *m, const float *f, int block_size,
                   int chroma_shared, int32_t *block_ptr, uint16_t *pos, int64_t *pos_cap,
                   float *values, int64_t *val_cap) {
  if (check_geometry(frame, block_size) || !m || !f || !block_ptr || !pos || !pos_cap ||
      !values || !val_cap)
    return PDI_EINVAL;
  int shared = (frame->format == PDI_YUV420 && chroma_shared) ? 1 : 0;
  PlaneGeom pg[3];
  int np = planes_of(frame, pg);
  long long foff[3] = {0, 0, 0};
  for (int i = 1; i < np; ++i) foff[i] = foff[i - 1] + (long long)pg[i - 1].W * pg[i - 1].H;
  int mp[3], vp[3][2], nv[3];
  int ng = groups_of(frame, shared, mp, vp, nv);
  // mask planes back to back: Y, then C (shared) or Cb, Cr
  long long moff[3] = {0, 0, 0};
  for (int g = 1; g < ng; ++g) moff[g] = moff[g - 1] + (long long)pg[mp[g - 1]].W * pg[mp[g - 1]].H;
  long long np_ = 0, nvv = 0;
  int mb = 0;
  block_ptr[0] = 0;
  std::vector<float> cr;  // shared Cr values follow all other values
  for (int g = 0; g < ng; ++g) {
    int W = pg[mp[g]].W, H = pg[mp[g]].H, b = block_size;
    for (int by = 0; by < (H + b - 1) / b; ++by)
      for (int bx = 0; bx < (W + b - 1) / b; ++bx) {
        int w = W - bx * b < b ? W - bx * b : b, h = H - by * b < b ? H - by * b : b;
        for (int y = 0; y < h; ++y)
          for (int x = 0; x < w; ++x) {
            long long px = (long long)(by * b + y) * W + bx * b + x;
            if (!m[moff[g] + px]) continue;
            if (np_ >= *pos_cap || nvv >= *val_cap) return PDI_ENOMEM;
            pos[np_++] = (uint16_t)(y * w + x);
            values[nvv++] = f[foff[vp[g][0]] + px];
            if (nv[g] == 2) cr.push_back(f[foff[vp[g][1]] + px]);
          }
        block_ptr[++mb] = (int32_t)np_;
      }
  }
  for (float v : cr) {
    if (nvv >= *val_cap) return PDI_ENOMEM;
    values[nvv++] = v;
  }
  *pos_cap = np_;
  *val_cap = nvv;
  return PDI_OK;
}

}  // extern "C"

// ----------------------------------------------- homogeneous diffusion

void pdi_default_cg_params(pdi_cg_params *p) {
  if (!p) return;
  p->tol = 1e-6;
  p->max_iter = 4000;
  p->check = 8;
  p->coarse_tol = 1e-3;
}

int inpaint_homogeneous(pdi_ctx *c, int width, int height, const uint8_t *mask, const float *f,
                        const pdi_cg_params *cp, float *u, void *stream, int32_t *iterations) {
  if (!c) return PDI_EINVAL;
  if (iterations) *iterations = 0;
  if (!mask || !f || !u) return set_err(c, PDI_EINVAL, "null mask, values or output");
  if (width <= 0 || height <= 0 || (long long)width * height > (1LL << 30))
    return set_err(c, PDI_EINVAL, "bad plane size %dx%d", width, height);
  pdi_cg_params P;
  pdi_default_cg_params(&P);
  if (cp) P = *cp;
  if (!(P.tol > 0.0) || !(P.tol < 1.0)) return set_err(c, PDI_EINVAL, "tol must be in (0, 1)");
  if (P.max_iter < 1 || P.max_iter > (1 << 16)) return set_err(c, PDI_EINVAL, "max_iter must be in [1, 65536]");
  if (P.check < 1 || P.check > 1024) return set_err(c, PDI_EINVAL, "check must be in [1, 1024]");
  if (!(P.coarse_tol >= P.tol) || !(P.coarse_tol < 1.0)) return set_err(c, PDI_EINVAL, "coarse_tol must be in [tol, 1)");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  std::lock_guard<std::mutex> lock(c->mu);
  hipStream_t s = (hipStream_t)stream;
  DiffWork &D = c->diff[{width, height}];
  int rc = PDI_OK;
  if (D.levels == 0) {
    // Pyramid: halve (rounding up) while both sides stay >= 64 pixels.
    D.w[0] = width;
    D.h[0] = height;
    D.levels = 1;
    while (D.levels < DiffWork::kMaxLevels && D.w[D.levels - 1] >= 128 && D.h[D.levels - 1] >= 128) {
      D.w[D.levels] = (D.w[D.levels - 1] + 1) / 2;
      D.h[D.levels] = (D.h[D.levels - 1] + 1) / 2;
      ++D.levels;
    }
    const size_t n0 = (size_t)width * height;
    for (int l = 1; l < D.levels && !rc; ++l) {
      const size_t n = (size_t)D.w[l] * D.h[l];
      rc = dev_alloc(c, (void **)&D.m[l], n, "diffusion pyramid");
      if (!rc) rc = dev_alloc(c, (void **)&D.f[l], sizeof(float) * n, "diffusion pyramid");
      if (!rc) rc = dev_alloc(c, (void **)&D.u[l], sizeof(float) * n, "diffusion pyramid");
    }
    for (float **v : {&D.p, &D.rv[0], &D.rv[1], &D.wv[0], &D.wv[1], &D.sv[0], &D.sv[1]})
      if (!rc) rc = dev_alloc(c, (void **)v, sizeof(float) * n0, "diffusion vectors");
    if (rc) {
      free_diff(D);
      c->diff.erase({width, height});
      return rc;
    }
  }
  // GAM and DEL: slots per iteration; BB: one slotted scalar; ALPHA: one
  // double per iteration.
  const int need = (2 * (P.max_iter + 1) + 1) * pdi::kHdSlots + (P.max_iter + 1);
  const int hneed = (P.check + 2) * pdi::kHdSlots;  // GAM[i..i+check] and BB
  if (!D.ev && hipEventCreateWithFlags(&D.ev, hipEventDisableTiming) != hipSuccess)
    return set_err(c, PDI_EHIP, "event for the norm read-back");
  if (D.host_cap < hneed) {
    if (D.host) (void)hipHostFree(D.host);
    D.host = nullptr;
    D.host_cap = 0;
    if (hipHostMalloc((void **)&D.host, sizeof(double) * (size_t)hneed) != hipSuccess)
      return set_err(c, PDI_ENOMEM, "pinned read-back buffer");
    D.host_cap = hneed;
  }
  if (D.sc_cap < need) {
    if (D.sc) (void)hipFree(D.sc);
    D.sc = nullptr;
    D.sc_cap = 0;
    rc = dev_alloc(c, (void **)&D.sc, sizeof(double) * (size_t)need, "diffusion scalars");
    if (rc) return rc;
    D.sc_cap = need;
  }
  D.m[0] = const_cast<uint8_t *>(mask);
  D.f[0] = const_cast<float *>(f);
  D.u[0] = u;
  double *GAM = D.sc, *DEL = D.sc + (P.max_iter + 1) * pdi::kHdSlots, *BB = D.sc + 2 * (P.max_iter + 1) * pdi::kHdSlots,
         *ALPHA = BB + pdi::kHdSlots;
  for (int l = 1; l < D.levels && e == hipSuccess; ++l)
    e = pdi::hd_restrict(D.m[l - 1], D.f[l - 1], D.w[l - 1], D.h[l - 1], D.m[l], D.f[l], D.w[l], D.h[l], s);
  bool converged = true;
  int its0 = 0;
  for (int l = D.levels - 1; l >= 0 && e == hipSuccess; --l) {
    const int W = D.w[l], H = D.h[l];
    e = pdi::hd_init(D.m[l], D.f[l], W, H, l + 1 < D.levels ? D.u[l + 1] : nullptr, l + 1 < D.levels ? D.w[l + 1] : 0,
                     D.u[l], s);
    if (e == hipSuccess) e = pdi::hd_zero(D.sc, need, s);
    if (e == hipSuccess) e = pdi::hd_residual(D.m[l], D.f[l], D.u[l], W, H, D.rv[0], GAM, BB, s);
    if (e == hipSuccess) e = pdi::hd_start(D.m[l], D.rv[0], W, H, D.wv[0], DEL, s);
    // CG.  Each launch tests convergence on the device (GAM[it] against
    // tol^2 BB) and does nothing once it holds.  The host queues P.check
    // launches at a time, each batch behind a read-back of the norms the
    // previous batch produced, and examines a read-back only once the next
    // batch is queued, so the device never waits for the host; the first
    // converged iteration is found in the norms.
    int it = 0;           // iterations queued
    int lo = 0, hi = 0;   // the read-back in flight holds GAM[lo..hi]
    int its = 0;          // iterations of the level's result
    bool done = false;
    const double tol2 = l ? P.coarse_tol * P.coarse_tol : P.tol * P.tol;
    const size_t sb = sizeof(double) * pdi::kHdSlots;
    auto read_back = [&]() -> hipError_t {
      const int n = hi - lo + 1;
      hipError_t r = hipMemcpyAsync(D.host, GAM + (size_t)lo * pdi::kHdSlots, n * sb, hipMemcpyDeviceToHost, s);
      if (r == hipSuccess)
        r = hipMemcpyAsync(D.host + (size_t)n * pdi::kHdSlots, BB, sb, hipMemcpyDeviceToHost, s);
      if (r == hipSuccess) r = hipEventRecord(D.ev, s);
      return r;
    };
    auto queue = [&](int count) -> hipError_t {
      const int stop = std::min(P.max_iter, it + count);
      hipError_t r = hipSuccess;
      for (; it < stop && r == hipSuccess; ++it) {
        const int a = it & 1, b = a ^ 1;
        r = pdi::hd_iterate(D.m[l], W, H, GAM, DEL, ALPHA, BB, tol2, it, D.u[l], D.p, D.rv[a], D.wv[a], D.sv[a],
                            D.rv[b], D.wv[b], D.sv[b], s);
      }
      return r;
    };
    // First batch: the previous solve's count for this level when there is
    // one (the read-back after it then already holds the converged norm).
    const int hint = D.hint[l];
    if (e == hipSuccess) e = read_back();  // GAM[0]
    if (e == hipSuccess) e = queue(hint > 0 ? std::min(P.check, hint) : P.check);
    double g_prev = -1.0;  // last norm examined and its iteration
    int i_prev = -1;
    double g0 = -1.0;      // |r_0|^2 of the level (the first read-back holds it)
    while (e == hipSuccess) {
      e = hipEventSynchronize(D.ev);
      if (e != hipSuccess) break;
      const int n = hi - lo + 1;
      double bb = 0.0;
      for (int k = 0; k < pdi::kHdSlots; ++k) bb += D.host[(size_t)n * pdi::kHdSlots + k];
      bool bad = false;
      double g_first = -1.0, g = 0.0;
      for (int i = 0; i < n; ++i) {
        g = 0.0;
        for (int k = 0; k < pdi::kHdSlots; ++k) g += D.host[(size_t)i * pdi::kHdSlots + k];
        if (!(g == g)) {  // NaN: not converging
          bad = true;
          break;
        }
        if (i == 0) g_first = g;
        if (lo + i == 0) g0 = g;
        // the device's test: relative to |b| or, when the start is worse than
        // zero (|r_0| > |b|, e.g. b = 0), to |r_0|
        bb = std::max(bb, g0);
        if (g <= tol2 * bb) {
          done = true;
          its = lo + i;  // the launches after it did nothing
          break;
        }
      }
      if (done || bad) break;
      if (hi >= P.max_iter) {  // the norm after max_iter iterations did not meet tol
        its = hi;
        break;
      }
      // Next batch: the iterations the norm's decay so far says are left
      // beyond the batch in flight (+1), at most P.check, at least 1; with
      // no decay seen yet (only GAM[0]), those the hint leaves (+1).
      int next = P.check;
      {
        const double g0 = i_prev >= 0 ? g_prev : g_first;
        const int i0 = i_prev >= 0 ? i_prev : lo, span = hi - i0;
        if (span > 0 && g > 0.0 && g0 > g) {
          const double rate = std::log(g / g0) / span;  // per iteration, < 0
          const double left = std::log(tol2 * bb / g) / rate - (double)(it - hi);
          next = std::max(1, std::min(P.check, (int)std::ceil(left) + 1));
        } else if (span == 0 && hint > 0) {
          next = std::max(1, std::min(P.check, hint - it + 1));
        }
      }
      g_prev = g;
      i_prev = hi;
      lo = hi + 1;  // everything queued so far (it > hi: at least one batch went out)
      hi = it;
      e = read_back();
      if (e == hipSuccess) e = queue(next);
    }
    if (!done && its == 0) its = it;
    D.hint[l] = done ? std::max(1, its) : 0;
    if (l == 0) {
      its0 = its;
      converged = done;
    }
  }
  if (e != hipSuccess) return hip_fail(c, e, "diffusion inpainting");
  if (iterations) *iterations = its0;
  if (!converged) return set_err(c, PDI_ESOLVE, "CG did not reach tol %g within %d iterations", P.tol, P.max_iter);
  return PDI_OK;
}
