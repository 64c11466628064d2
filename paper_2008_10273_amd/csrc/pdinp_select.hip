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
// (at most 64 rows: 63 points + the border) has row i in lane i's registers
// (Gauss-Jordan without pivoting, as the decoder's general path, pivot rows
// broadcast by readlane); rectangle errors come from a summed-area table.  The result is one 64-bit word per block (bit y*8 + x),
// turned into the packed mask (block_ptr, pos) and the values at the mask
// points by k_sel_count and k_sel_pack.
#include "pdinp_device.h"

#include <hip/hip_runtime.h>

namespace pdi {

constexpr int kSelThreads = 256;
constexpr int kSelWaves = kSelThreads / 64;

struct SelStage {
  float r[2][64];  // residual of the block's pixels per value plane (0 outside the block)
  float sat[64];   // summed-area table of the squared error: sat[y*8+x] = sum over x' <= x, y' <= y
  float c[2][64];  // coefficients of point i
  float a[2];
  int pt[64];      // pixel of point i
  int rect[64];    // rectangles: x0 | x1 << 8 | y0 << 16 | y1 << 24
  float tab[81];   // compact Green table of the block's shape
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

// Value of x in lane `src` (src uniform across the wave).
__device__ __forceinline__ float lane_f(float x, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), src));
}

// Bordered system of the K points on lanes 0..K (row i on lane i, NC >= K+1
// columns in registers, the right-hand sides apart), Gauss-Jordan without
// pivoting with the pivot row broadcast by readlane (step j is unrolled, so
// every register index is a constant); stores c and a in the stage.
template <int NC>
__device__ __forceinline__ void sel_solve(SelStage &st, int lane, int K, int nv, int w, int h) {
  const int n = K + 1;
  float row[NC];
  float b0 = 0.f, b1 = 0.f, diag = 1.f;
  {
    int xi = 0, yi = 0;
    if (lane < K) {
      const int p = st.pt[lane];
      xi = p & 7;
      yi = p >> 3;
      b0 = st.r[0][p];
      b1 = st.r[1][p];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      float v = 0.f;
      if (k < K) {
        const int q = st.pt[k];
        v = lane < K ? green_tab(st.tab, w, h, xi, yi, q & 7, q >> 3) : (lane == K ? 1.f : 0.f);
      } else if (k == K) {
        v = lane < K ? 1.f : 0.f;
      }
      row[k] = v;
    }
  }
  const bool act = lane < n;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    if (j < n) {  // uniform
      const float piv = lane_f(row[j], j);
      if (lane == j) diag = row[j];
      const float fct = (act && lane != j) ? row[j] / piv : 0.f;
#pragma unroll
      for (int k = j + 1; k < NC; ++k) row[k] = fmaf(-fct, lane_f(row[k], j), row[k]);
      b0 = fmaf(-fct, lane_f(b0, j), b0);
      if (nv > 1) b1 = fmaf(-fct, lane_f(b1, j), b1);
    }
  }
  if (act) {
    const float x0 = b0 / diag, x1 = b1 / diag;
    if (lane < K) {
      st.c[0][lane] = x0;
      st.c[1][lane] = x1;
    } else {
      st.a[0] = x0;
      st.a[1] = x1;
    }
  }
}

// At most 96 VGPRs (5 waves per SIMD): the 64-column solve still fits without spills.
__global__ __launch_bounds__(kSelThreads) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_select8(FrameDev f) {
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
    // (this order of the tests keeps the kernel within 96 VGPRs without spills)
    if (K >= 32) sel_solve<64>(st, lane, K, nv, w, h);
    else if (K >= 16) sel_solve<32>(st, lane, K, nv, w, h);
    else if (K >= 8) sel_solve<16>(st, lane, K, nv, w, h);
    else sel_solve<8>(st, lane, K, nv, w, h);
    wave_sync();
    // Eq. 2 at every pixel and its squared error.  Point i's pixel and
    // coefficients sit in lane i's registers and are broadcast by readlane;
    // each Green's function value serves both value planes.  Steps go in
    // fours: lanes K .. K4-1 hold pixel 0 and zero coefficients, so the
    // padding adds exact zeros (K4 <= 64 as K <= 63).  Lane i holds point i
    // whatever its own pixel is, so the broadcasts run with the whole wave
    // active (uniform loop, scalar results); only the lanes of in-block
    // pixels then evaluate.
    const int myq = lane < K ? st.pt[lane] : 0;
    const float myc0 = lane < K ? st.c[0][lane] : 0.f;
    const float myc1 = lane < K ? st.c[1][lane] : 0.f;
    const int K4 = (K + 3) & ~3;
    float u0 = 0.f, u1 = 0.f;
    for (int i0 = 0; i0 < K4; i0 += 4) {
      int q[4];
      float c0[4], c1[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        q[t] = __builtin_amdgcn_readlane(myq, i0 + t);
        c0[t] = lane_f(myc0, i0 + t);
        c1[t] = lane_f(myc1, i0 + t);
      }
      if (valid) {
        float gv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) gv[t] = green_tab(st.tab, w, h, px, py, q[t] & 7, q[t] >> 3);
#pragma unroll
        for (int t = 0; t < 4; ++t) u0 = fmaf(c0[t], gv[t], u0);
        if (nv > 1) {
#pragma unroll
          for (int t = 0; t < 4; ++t) u1 = fmaf(c1[t], gv[t], u1);
        }
      }
    }
    float err = 0.f;
    if (valid) {
      const float d0 = (u0 + st.a[0]) - st.r[0][lane];
      err = d0 * d0;
      if (nv > 1) {
        const float d1 = (u1 + st.a[1]) - st.r[1][lane];
        err = fmaf(d1, d1, err);
      }
    }
    // summed-area table: prefix along x inside each row of 8 lanes, then along y
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      const float t = __shfl_up(err, o, 8);
      if (px >= o) err += t;
    }
#pragma unroll
    for (int o = 8; o < 64; o <<= 1) {
      const float t = __shfl_up(err, o, 64);
      if (lane >= o) err += t;
    }
    st.sat[lane] = err;
    wave_sync();
    // rectangles: mean error from the table, split decision, new rectangles appended
    bool split = false;
    int R = 0, Rn = 0;
    if (lane < nl) {
      R = st.rect[lane];
      const int rx0 = R & 255, rx1 = (R >> 8) & 255, ry0 = (R >> 16) & 255, ry1 = R >> 24;
      float s = st.sat[ry1 * 8 + rx1];
      if (rx0 > 0) s -= st.sat[ry1 * 8 + rx0 - 1];
      if (ry0 > 0) s -= st.sat[(ry0 - 1) * 8 + rx1];
      if (rx0 > 0 && ry0 > 0) s += st.sat[(ry0 - 1) * 8 + rx0 - 1];
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

// Packing in two passes over tiles of 256 blocks.  k_sel_count: each tile's
// exclusive prefix of the blocks' point counts (sel_x[m]) and its total
// (sel_x[n + tile]).
constexpr int kSelTile = 256;

__device__ __forceinline__ int tile_scan_excl(int c, int *wsum, int &total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  int off = 0;
  total = 0;
  for (int k = 0; k < kSelTile / 64; ++k) {
    off += k < wv ? wsum[k] : 0;
    total += wsum[k];
  }
  return off + x - c;
}

__global__ __launch_bounds__(kSelTile) void k_sel_count(FrameDev f) {
  __shared__ int wsum[kSelTile / 64];
  const int m = blockIdx.x * kSelTile + threadIdx.x;
  const int c = m < f.n_items ? __popcll(f.sel_bits[m]) : 0;
  int total;
  const int ex = tile_scan_excl(c, wsum, total);
  if (m < f.n_items) f.sel_x[m] = ex;
  if (threadIdx.x == 0) f.sel_x[f.n_items + blockIdx.x] = total;
}

// Sum of v over the workgroup (every thread gets it).
__device__ __forceinline__ int wg_sum(int v, int *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();  // red is free
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int s = 0;
  for (int k = 0; k < kSelTile / 64; ++k) s += red[k];
  return s;
}

// block_ptr, positions (in-block index y*w + x, ascending) and the values at
// the mask points; a shared chroma mask's Cr values follow every other value.
__global__ __launch_bounds__(kSelTile) void k_sel_pack(FrameDev f) {
  __shared__ int red[kSelTile / 64];
  const int n = f.n_items, ntiles = (n + kSelTile - 1) / kSelTile, tile = blockIdx.x;
  const int cf = f.chroma_first, tcf = cf >= 0 ? cf / kSelTile : 0;
  int before = 0, before_cf = 0, all = 0;
  for (int t = threadIdx.x; t < ntiles; t += kSelTile) {
    const int v = f.sel_x[n + t];
    before += t < tile ? v : 0;
    before_cf += t < tcf ? v : 0;
    all += v;
  }
  before = wg_sum(before, red);
  before_cf = wg_sum(before_cf, red);
  all = wg_sum(all, red);
  const int m = tile * kSelTile + threadIdx.x;
  if (m == n - 1 || (n == 0 && m == 0)) f.sel_bp[n] = all;
  if (m >= n) return;
  const int bpm = before + f.sel_x[m];
  f.sel_bp[m] = bpm;
  int g = 0;
  if (f.ngroups > 1 && m >= f.g[1].first) g = 1;
  if (f.ngroups > 2 && m >= f.g[2].first) g = 2;
  const GroupDev &G = f.g[g];
  const int l = m - G.first, bx = l % G.nbx, by = l / G.nbx;
  const int x0 = bx * 8, y0 = by * 8, w = min(8, G.W - x0);
  const long long base0 = bpm;
  const long long base1 = (G.nv > 1) ? (long long)all + (bpm - (before_cf + f.sel_x[cf])) : base0;
  unsigned long long bits = f.sel_bits[m];
  int i = 0;
  while (bits) {
    const int p = __ffsll((long long)bits) - 1;
    bits &= bits - 1ull;
    const int x = p & 7, y = p >> 3;
    f.sel_pos[base0 + i] = (uint16_t)(y * w + x);
    const long long px = (long long)(y0 + y) * G.W + x0 + x;
    f.sel_vals[base0 + i] = f.sel_planes[G.out_off[0] + px];
    if (G.nv > 1) f.sel_vals[base1 + i] = f.sel_planes[G.out_off[1] + px];
    ++i;
  }
}

hipError_t launch_select(const FrameDev &f, hipStream_t s) {
  if (f.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_select8, dim3((f.n_items + kSelWaves - 1) / kSelWaves), dim3(kSelThreads), 0, s, f);
  const int ntiles = (f.n_items + kSelTile - 1) / kSelTile;
  hipLaunchKernelGGL(k_sel_count, dim3(ntiles), dim3(kSelTile), 0, s, f);
  hipLaunchKernelGGL(k_sel_pack, dim3(ntiles), dim3(kSelTile), 0, s, f);
  return hipGetLastError();
}

}  // namespace pdi
