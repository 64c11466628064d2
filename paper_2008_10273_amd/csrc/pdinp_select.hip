// Per-block mask selection by rectangular subdivision: how the encoder
// picks the mask points of each 8x8 residual block (Sec. 2.3 of the paper,
// which takes the scheme from its cited rectangular-subdivision codec).
//
// A block's mask is the set of corners of a set of rectangles (inclusive
// pixel ranges that share their common edges).  Starting from the whole
// block, each round inpaints the block from the current corners with the
// Green's route of Sec. 2.2 (bordered system, then Eq. 2), takes every
// rectangle's mean squared error and halves each rectangle whose error
// exceeds the threshold along its longer side (x on ties), both halves
// keeping the middle line; rounds stop when nothing splits.
//
// One wave per block: lane p is pixel (p & 7, p >> 3); the bordered system
// (at most 64 rows: 63 points + the border) sits in the wave's LDS, row i
// updated by lane i (Gauss-Jordan without pivoting, as the decoder's
// general path).  The result is one 64-bit word per block (bit y*8 + x),
// turned into the packed mask (block_ptr, pos) and the values at the mask
// points by k_sel_scan and k_sel_pack.
#include "pdinp_device.h"

#include <hip/hip_runtime.h>

namespace pdi {

constexpr int kSelThreads = 128;  // 2 waves: 39 KB of LDS per workgroup
constexpr int kSelWaves = kSelThreads / 64;
constexpr int kSelLd = 67;  // row stride of the system: 64 columns + 2 right-hand sides + 1 (banks)

struct SelStage {
  float M[64 * kSelLd];  // bordered system, row-major
  float r[2][64];        // residual of the block's pixels per value plane (0 outside the block)
  float e[64];           // squared error per pixel, summed over the value planes
  float c[2][64];        // coefficients of point i
  float a[2];
  int pt[64];            // pixel of point i
  int rect[64];          // rectangles: x0 | x1 << 8 | y0 << 16 | y1 << 24
  float tab[81];         // compact Green table of the block's shape
};

__device__ __forceinline__ int rect_pack(int x0, int x1, int y0, int y1) {
  return x0 | (x1 << 8) | (y0 << 16) | (y1 << 24);
}

// Lanes that are a corner of one of the n rectangles.
__device__ __forceinline__ unsigned long long corner_bits(const SelStage &st, int n, int px, int py, bool valid) {
  bool k = false;
  for (int j = 0; j < n; ++j) {
    const int R = st.rect[j];
    const int x0 = R & 255, x1 = (R >> 8) & 255, y0 = (R >> 16) & 255, y1 = R >> 24;
    k |= (px == x0 || px == x1) && (py == y0 || py == y1);
  }
  return __ballot(k && valid);
}

__global__ __launch_bounds__(kSelThreads) void k_select8(FrameDev f) {
  __shared__ SelStage stage[kSelWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = blockIdx.x * kSelWaves + wv;  // mask block
  if (m >= f.n_items) return;                 // whole waves leave: nothing below synchronises the workgroup
  SelStage &st = stage[wv];
  int g = 0;
  if (f.ngroups > 1 && m >= f.g[1].first) g = 1;
  if (f.ngroups > 2 && m >= f.g[2].first) g = 2;
  const GroupDev &G = f.g[g];
  const int l = m - G.first, bx = l % G.nbx, by = l / G.nbx;
  const int x0 = bx * 8, y0 = by * 8;
  const int w = min(8, G.W - x0), h = min(8, G.H - y0);
  const int e = (w < 8 ? 1 : 0) + (h < 8 ? 2 : 0);
  const ShapeDev S = f.s[G.shape[e]];
  const int nv = G.nv;
  const float thr = f.sel_thr[g ? 1 : 0];

  const int px = lane & 7, py = lane >> 3;
  const bool valid = px < w && py < h;
  for (int v = 0; v < 2; ++v)
    st.r[v][lane] = (valid && v < nv) ? f.sel_planes[G.out_off[v] + (long long)(y0 + py) * G.W + x0 + px] : 0.f;
  for (int i = lane; i < (w + 1) * (h + 1); i += 64) st.tab[i] = f.tab32[S.hc32 + i];
  if (lane == 0) st.rect[0] = rect_pack(0, w - 1, 0, h - 1);
  const unsigned long long full = __ballot(valid);
  const int N = __popcll(full);
  int nl = 1;
  wave_sync();

  unsigned long long bits = 0;
  for (int round = 0;; ++round) {
    bits = corner_bits(st, nl, px, py, valid);
    if (round >= f.sel_rounds) break;
    const int K = __popcll(bits);
    if (K == N) break;  // every pixel known: no error left
    // points in ascending pixel order
    if ((bits >> lane) & 1ull) st.pt[__popcll(bits & ((1ull << lane) - 1ull))] = lane;
    wave_sync();
    // bordered system [G_K 1; 1^T 0 | r]: row i on lane i
    const int n = K + 1, ld = n + nv;
    if (lane < n) {
      int xi = 0, yi = 0;
      if (lane < K) {
        const int p = st.pt[lane];
        xi = p & 7;
        yi = p >> 3;
      }
      float *row = st.M + lane * kSelLd;
      for (int k = 0; k < K; ++k) {
        const int q = st.pt[k];
        row[k] = lane < K ? green_tab(st.tab, w, h, xi, yi, q & 7, q >> 3) : 1.f;
      }
      row[K] = lane < K ? 1.f : 0.f;
      for (int v = 0; v < nv; ++v) row[n + v] = lane < K ? st.r[v][st.pt[lane]] : 0.f;
    }
    // Gauss-Jordan without pivoting (leading block SPD, last pivot nonzero)
    for (int j = 0; j < n; ++j) {
      wave_sync();  // row j of the previous step is complete
      if (lane < n && lane != j) {
        const float *pr = st.M + j * kSelLd;
        float *row = st.M + lane * kSelLd;
        const float fct = row[j] / pr[j];
        for (int k = j + 1; k < ld; ++k) row[k] = fmaf(-fct, pr[k], row[k]);
      }
    }
    wave_sync();
    if (lane < n) {
      const float *row = st.M + lane * kSelLd;
      for (int v = 0; v < nv; ++v) {
        const float x = row[n + v] / row[lane];
        if (lane < K) st.c[v][lane] = x;
        else st.a[v] = x;
      }
    }
    wave_sync();
    // Eq. 2 at every pixel and its squared error
    float err = 0.f;
    if (valid) {
      for (int v = 0; v < nv; ++v) {
        float u = 0.f;
        for (int i = 0; i < K; ++i) {
          const int q = st.pt[i];
          u = fmaf(st.c[v][i], green_tab(st.tab, w, h, px, py, q & 7, q >> 3), u);
        }
        const float d = (u + st.a[v]) - st.r[v][lane];
        err = fmaf(d, d, err);
      }
    }
    st.e[lane] = err;
    wave_sync();
    // rectangles: mean error, split decision, new rectangles appended
    bool split = false;
    int R = 0, Rn = 0;
    if (lane < nl) {
      R = st.rect[lane];
      const int rx0 = R & 255, rx1 = (R >> 8) & 255, ry0 = (R >> 16) & 255, ry1 = R >> 24;
      float s = 0.f;
      for (int y = ry0; y <= ry1; ++y)
        for (int x = rx0; x <= rx1; ++x) s += st.e[y * 8 + x];
      const float mse = s / (float)((rx1 - rx0 + 1) * (ry1 - ry0 + 1) * nv);
      const int gx = rx1 - rx0, gy = ry1 - ry0;
      if (mse > thr && (gx >= 2 || gy >= 2)) {
        split = true;
        if (gx >= gy) {
          const int mid = (rx0 + rx1) >> 1;
          R = rect_pack(rx0, mid, ry0, ry1);
          Rn = rect_pack(mid, rx1, ry0, ry1);
        } else {
          const int mid = (ry0 + ry1) >> 1;
          R = rect_pack(rx0, rx1, ry0, mid);
          Rn = rect_pack(rx0, rx1, mid, ry1);
        }
      }
    }
    const unsigned long long sm = __ballot(split);
    if (sm == 0) break;
    if (split) {
      st.rect[lane] = R;
      st.rect[nl + __popcll(sm & ((1ull << lane) - 1ull))] = Rn;
    }
    nl += __popcll(sm);
    wave_sync();
  }
  if (lane == 0) f.sel_bits[m] = bits;
}

// block_ptr[m] = points of the blocks before m (one workgroup: per-thread
// chunks, then a scan of the chunk sums in LDS).
__global__ __launch_bounds__(1024) void k_sel_scan(FrameDev f) {
  __shared__ int sums[1024];
  const int n = f.n_items, t = threadIdx.x;
  const int ch = (n + 1023) / 1024, lo = min(n, t * ch), hi = min(n, lo + ch);
  int s = 0;
  for (int m = lo; m < hi; ++m) s += __popcll(f.sel_bits[m]);
  sums[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? sums[t - o] : 0;
    __syncthreads();
    sums[t] += v;
    __syncthreads();
  }
  int run = sums[t] - s;  // exclusive prefix of this chunk
  int32_t *bp = f.sel_bp;
  for (int m = lo; m < hi; ++m) {
    bp[m] = run;
    run += __popcll(f.sel_bits[m]);
  }
  if (t == 1023) bp[n] = sums[1023];
}

// Positions (in-block index y*w + x, ascending) and values at the mask
// points; a shared chroma mask's Cr values follow every other value.
__global__ __launch_bounds__(256) void k_sel_pack(FrameDev f) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= f.n_items) return;
  int g = 0;
  if (f.ngroups > 1 && m >= f.g[1].first) g = 1;
  if (f.ngroups > 2 && m >= f.g[2].first) g = 2;
  const GroupDev &G = f.g[g];
  const int l = m - G.first, bx = l % G.nbx, by = l / G.nbx;
  const int x0 = bx * 8, y0 = by * 8, w = min(8, G.W - x0);
  const int32_t *bp = f.sel_bp;
  uint16_t *pos = f.sel_pos;
  float *vals = f.sel_vals;
  const long long base0 = bp[m];
  const long long base1 = (G.nv > 1) ? (long long)bp[f.n_items] + (bp[m] - bp[f.chroma_first]) : base0;
  unsigned long long bits = f.sel_bits[m];
  int i = 0;
  while (bits) {
    const int p = __ffsll((long long)bits) - 1;
    bits &= bits - 1ull;
    const int x = p & 7, y = p >> 3;
    pos[base0 + i] = (uint16_t)(y * w + x);
    const long long px = (long long)(y0 + y) * G.W + x0 + x;
    vals[base0 + i] = f.sel_planes[G.out_off[0] + px];
    if (G.nv > 1) vals[base1 + i] = f.sel_planes[G.out_off[1] + px];
    ++i;
  }
}

hipError_t launch_select(const FrameDev &f, hipStream_t s) {
  if (f.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_select8, dim3((f.n_items + kSelWaves - 1) / kSelWaves), dim3(kSelThreads), 0, s, f);
  hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1024), 0, s, f);
  hipLaunchKernelGGL(k_sel_pack, dim3((f.n_items + 255) / 256), dim3(256), 0, s, f);
  return hipGetLastError();
}

}  // namespace pdi
