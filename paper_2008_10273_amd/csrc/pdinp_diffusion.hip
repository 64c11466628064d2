// Global homogeneous diffusion inpainting (Sec. 2.1 of the paper): Eq. (1)
// with A = -L (5-point Laplacian, reflecting boundaries) on one whole
// plane, solved coarse to fine with conjugate gradients, each level
// starting from the solution of the next coarser one (the cascadic scheme
// the paper uses).  The unknowns are the pixels off the mask.  Vectors are
// kept on the full grid with zeros on the mask, so that A_UU p is the
// 5-point operator applied to p with the mask pixels held at zero: every
// kernel is one coalesced pass over the plane.  Dot products accumulate in
// FP64, one atomic per workgroup into one of kHdSlots slots (workgroup
// index modulo kHdSlots: thousands of workgroups adding to one address
// serialise), and a scalar is the sum of its slots.
#include "pdinp_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace pdi {

constexpr int kHdThreads = 512;

// The value of a slotted scalar (uniform loads).
__device__ __forceinline__ double slot_sum(const double *a) {
  double s = 0.0;
#pragma unroll 16
  for (int k = 0; k < kHdSlots; ++k) s += a[k];
  return s;
}

// Sum v and w over the workgroup and add the totals to the workgroup's slot
// of the slotted scalars dst0, dst1 (dst1 may be null).  Every thread of
// the workgroup must call it.
__device__ __forceinline__ void wg_add2(double v, double w, double *dst0, double *dst1) {
  __shared__ double red[2][kHdThreads / 64];
  for (int o = 32; o > 0; o >>= 1) {
    v += __shfl_xor(v, o);
    w += __shfl_xor(w, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = v;
    red[1][threadIdx.x >> 6] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, t = 0.0;
    for (int i = 0; i < kHdThreads / 64; ++i) {
      s += red[0][i];
      t += red[1][i];
    }
    const int slot = (blockIdx.y * gridDim.x + blockIdx.x) % kHdSlots;  // linear workgroup id
    atomicAdd(dst0 + slot, s);
    if (dst1) atomicAdd(dst1 + slot, t);
  }
}

// Kernels run on 64 x 8 pixel tiles: thread (tx, ty) of tile (bx, by)
// owns pixel (64 bx + tx, 8 by + ty).  The per-level kernels take one tile
// per workgroup (a 2D grid); the per-iteration kernel is persistent (at
// most kHdWgs workgroups, each looping over tiles) so that the scalars are
// read and the partial sums added once per workgroup, not once per tile.
constexpr int kTx = 64, kTy = 8;
constexpr int kHdWgs = 1024;  // four 512-thread workgroups per compute unit
static_assert(kTx * kTy == kHdThreads, "one pixel per thread");

// Coarser level: a pixel is known when one of its (up to 4) children is,
// with the mean of the known children's values.
__global__ __launch_bounds__(kHdThreads) void k_hd_restrict(const uint8_t *mf, const float *ff, int Wf, int Hf,
                                                            uint8_t *mc, float *fc, int Wc, int Hc) {
  const int x = blockIdx.x * kTx + (threadIdx.x & (kTx - 1)), y = blockIdx.y * kTy + threadIdx.x / kTx;
  if (x >= Wc || y >= Hc) return;
  int n = 0;
  float s = 0.f;
  for (int dy = 0; dy < 2; ++dy)
    for (int dx = 0; dx < 2; ++dx) {
      const int xf = 2 * x + dx, yf = 2 * y + dy;
      if (xf < Wf && yf < Hf && mf[yf * Wf + xf]) {
        ++n;
        s += ff[yf * Wf + xf];
      }
    }
  mc[y * Wc + x] = n ? 1 : 0;
  fc[y * Wc + x] = n ? s / (float)n : 0.f;
}

// Initial guess of a level: the known values on the mask, the coarser
// level's solution (nearest parent) elsewhere, or 0 on the coarsest level.
__global__ __launch_bounds__(kHdThreads) void k_hd_init(const uint8_t *m, const float *f, int W, int H,
                                                        const float *uc, int Wc, float *u) {
  const int x = blockIdx.x * kTx + (threadIdx.x & (kTx - 1)), y = blockIdx.y * kTy + threadIdx.x / kTx;
  if (x >= W || y >= H) return;
  const int i = y * W + x;
  u[i] = m[i] ? f[i] : (uc ? uc[(y >> 1) * Wc + (x >> 1)] : 0.f);
}

// r = -(A u) off the mask, 0 on it; RR[0] += |r|^2 and BB += |b|^2 with b
// the right-hand side of the unknowns' system A_UU u_U = b (b_i = sum of
// the known neighbours' values).
__global__ __launch_bounds__(kHdThreads) void k_hd_residual(const uint8_t *m, const float *f, const float *u,
                                                            int W, int H, float *r, double *rr, double *bb) {
  const int x = blockIdx.x * kTx + (threadIdx.x & (kTx - 1)), y = blockIdx.y * kTy + threadIdx.x / kTx;
  double sr = 0.0, sb = 0.0;
  if (x < W && y < H) {
    const int i = y * W + x;
    float ri = 0.f;
    if (!m[i]) {
      const float ui = u[i];
      float au = 0.f, b = 0.f;
      const int nb[4] = {x > 0 ? i - 1 : -1, x + 1 < W ? i + 1 : -1, y > 0 ? i - W : -1, y + 1 < H ? i + W : -1};
      for (int k = 0; k < 4; ++k) {
        const int j = nb[k];
        if (j >= 0) {
          au += ui - u[j];
          if (m[j]) b += f[j];
        }
      }
      ri = -au;
      sr = (double)ri * ri;
      sb = (double)b * b;
    }
    r[i] = ri;
  }
  wg_add2(sr, sb, rr, bb);
}

// w = A_UU r (r is zero on the mask) and DEL[0] += w . r: the start of the
// single-reduction CG recurrences below (one 2D tile per workgroup, the
// neighbours read from global memory: once per level).
__global__ __launch_bounds__(kHdThreads) void k_hd_aw(const uint8_t *m, const float *r, int W, int H, float *w,
                                                      double *del) {
  const int x = blockIdx.x * kTx + (threadIdx.x & (kTx - 1)), y = blockIdx.y * kTy + threadIdx.x / kTx;
  double sd = 0.0;
  if (x < W && y < H) {
    const int i = y * W + x;
    float wi = 0.f;
    if (!m[i]) {
      const float ri = r[i];
      float nsum = 0.f, deg = 0.f;
      if (x > 0) { nsum += r[i - 1]; deg += 1.f; }
      if (x + 1 < W) { nsum += r[i + 1]; deg += 1.f; }
      if (y > 0) { nsum += r[i - W]; deg += 1.f; }
      if (y + 1 < H) { nsum += r[i + W]; deg += 1.f; }
      wi = deg * ri - nsum;
      sd = (double)wi * ri;
    }
    w[i] = wi;
  }
  wg_add2(sd, 0.0, del, nullptr);
}

// Tile t of the persistent kernel's k-th pass for workgroup b of G.  Each
// XCD (workgroups are dealt to the 8 XCDs in turn) takes one contiguous
// eighth of the tiles in raster order, so the halo lines a tile shares with
// its neighbours are mostly fetched by the same L2.  Every tile is taken
// exactly once whatever the dispatch order; G < 8 falls back to a stride.
struct TileWalk {
  int t, end, step;
  __device__ TileWalk(int ntiles) {
    const int G = gridDim.x, b = blockIdx.x;
    if (G < 8) {
      t = b;
      end = ntiles;
      step = G;
    } else {
      const int k = b & 7, nk = (G - k + 7) >> 3;  // workgroups on this XCD
      t = (int)((long long)ntiles * k / 8) + (b >> 3);
      end = (int)((long long)ntiles * (k + 1) / 8);
      step = nk;
    }
  }
};

// One CG iteration in the single-reduction form (Chronopoulos and Gear):
// with w = A r and s = A p carried as vectors, both dot products of an
// iteration come from the same pass, so an iteration is one launch.
//   beta = g_i / g_{i-1}, alpha = g_i / (d_i - beta g_i / alpha_{i-1})
//   (beta = 0, alpha = g_0 / d_0 for i = 0), with g_i = r.r, d_i = w.r;
//   p = r + beta p, s = w + beta s, u += alpha p, r' = r - alpha s,
//   w' = A r', and GAM[i+1] += r'.r', DEL[i+1] += w'.r'.
// r', formed once per pixel of a tile and its one-pixel halo in LDS, feeds
// the stencil; r, w and s are read at the halo, so they are double-buffered
// (ri, wi, si in, ro, wo, so out); u and p are updated in place.  All
// vectors are zero on the mask.  Workgroup 0 records alpha in ALPHA[i].
// Once g_i <= tol2 max(|b|^2, g_0) (BB; g_0 = |r_0|^2 of the level's start,
// which keeps the test reachable when b = 0 but the start is not) every
// workgroup returns at once, leaving GAM[i+1] = 0, so the launches queued
// after convergence do nothing.
__global__ __launch_bounds__(kHdThreads) void k_hd_cg(const uint8_t *m, int W, int H, double *GAM, double *DEL,
                                                      double *ALPHA, const double *BB, double tol2, int it, float *u, float *p,
                                                      const float *ri, const float *wi, const float *si, float *ro,
                                                      float *wo, float *so) {
  __shared__ float rs[kTy + 2][kTx + 2];
  const int tx = threadIdx.x & (kTx - 1), ty = threadIdx.x / kTx;
  const int ntx = (W + kTx - 1) / kTx, ntiles = ntx * ((H + kTy - 1) / kTy);
  float alpha = 0.f, beta = 0.f;
  {
    const double g = slot_sum(GAM + it * kHdSlots), d = slot_sum(DEL + it * kHdSlots);
    if (g <= tol2 * fmax(slot_sum(BB), slot_sum(GAM))) return;  // converged (uniform over the grid)
    double a = 0.0, bt = 0.0;
    if (it == 0) {
      if (d > 0.0) a = g / d;
    } else {
      const double gp = slot_sum(GAM + (it - 1) * kHdSlots), ap = ALPHA[it - 1];
      if (gp > 0.0 && ap > 0.0) {
        bt = g / gp;
        const double den = d - bt * g / ap;
        if (den > 0.0) a = g / den;
      }
    }
    alpha = (float)a;
    beta = (float)bt;
    if (blockIdx.x == 0 && threadIdx.x == 0) ALPHA[it] = a;  // 0 once converged exactly: the iterate stays put
  }
  const bool first = it == 0;
  double sg = 0.0, sd = 0.0;
  for (TileWalk tw(ntiles); tw.t < tw.end; tw.t += tw.step) {
    const int x0 = (tw.t % ntx) * kTx, y0 = (tw.t / ntx) * kTy;
    const int x = x0 + tx, y = y0 + ty;
    const bool in = x < W && y < H;
    const int i = y * W + x;
    bool free_px = false;
    __syncthreads();  // the previous tile's LDS reads are done
    // own pixel: coalesced rows of 64.  The vectors are read whatever the
    // mask says (zero at known pixels), so that no load waits for the mask.
    float rn = 0.f;
    if (in) {
      const bool known = m[i];
      const float rv = ri[i], wv = wi[i], uv = u[i];
      const float pv = first ? 0.f : p[i], sv = first ? 0.f : si[i];
      free_px = !known;
      float pn = 0.f, sn = 0.f;
      if (free_px) {
        pn = first ? rv : fmaf(beta, pv, rv);
        sn = first ? wv : fmaf(beta, sv, wv);
        rn = fmaf(-alpha, sn, rv);
        u[i] = fmaf(alpha, pn, uv);
      }
      p[i] = pn;
      so[i] = sn;
      ro[i] = rn;
    }
    rs[ty + 1][tx + 1] = rn;
    // halo: 64 above, 64 below, 18 left, 18 right (same arithmetic as the
    // owning tile, so both see the same r')
    if (threadIdx.x < 2 * kTx + 2 * (kTy + 2)) {
      int lx, ly;
      const int h = threadIdx.x;
      if (h < kTx) { lx = h + 1; ly = 0; }
      else if (h < 2 * kTx) { lx = h - kTx + 1; ly = kTy + 1; }
      else if (h < 2 * kTx + kTy + 2) { lx = 0; ly = h - 2 * kTx; }
      else { lx = kTx + 1; ly = h - 2 * kTx - (kTy + 2); }
      const int gx = x0 + lx - 1, gy = y0 + ly - 1;
      float v = 0.f;
      if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
        const int j = gy * W + gx;
        const bool known = m[j];
        const float rv = ri[j], wv = wi[j], sv = first ? 0.f : si[j];
        if (!known) {
          const float sn = first ? wv : fmaf(beta, sv, wv);
          v = fmaf(-alpha, sn, rv);
        }
      }
      rs[ly][lx] = v;
    }
    __syncthreads();
    if (in) {
      float wn = 0.f;
      if (free_px) {
        // neighbours inside the plane; a masked neighbour holds r' = 0
        float nsum = 0.f, deg = 0.f;
        if (x > 0) { nsum += rs[ty + 1][tx]; deg += 1.f; }
        if (x + 1 < W) { nsum += rs[ty + 1][tx + 2]; deg += 1.f; }
        if (y > 0) { nsum += rs[ty][tx + 1]; deg += 1.f; }
        if (y + 1 < H) { nsum += rs[ty + 2][tx + 1]; deg += 1.f; }
        wn = deg * rn - nsum;
        sg += (double)rn * rn;
        sd += (double)wn * rn;
      }
      wo[i] = wn;
    }
  }
  wg_add2(sg, sd, GAM + (it + 1) * kHdSlots, DEL + (it + 1) * kHdSlots);
}

__global__ __launch_bounds__(kHdThreads) void k_hd_zero(double *a, int n) {
  const int i = blockIdx.x * kHdThreads + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

static inline dim3 hd_grid(long long n) { return dim3((unsigned)((n + kHdThreads - 1) / kHdThreads)); }
static inline dim3 hd_tiles(int W, int H) { return dim3((unsigned)((W + kTx - 1) / kTx), (unsigned)((H + kTy - 1) / kTy)); }

hipError_t hd_restrict(const uint8_t *mf, const float *ff, int Wf, int Hf, uint8_t *mc, float *fc, int Wc, int Hc,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_hd_restrict, hd_tiles(Wc, Hc), dim3(kHdThreads), 0, s, mf, ff, Wf, Hf, mc, fc, Wc, Hc);
  return hipGetLastError();
}
hipError_t hd_init(const uint8_t *m, const float *f, int W, int H, const float *uc, int Wc, float *u, hipStream_t s) {
  hipLaunchKernelGGL(k_hd_init, hd_tiles(W, H), dim3(kHdThreads), 0, s, m, f, W, H, uc, Wc, u);
  return hipGetLastError();
}
hipError_t hd_residual(const uint8_t *m, const float *f, const float *u, int W, int H, float *r, double *rr,
                       double *bb, hipStream_t s) {
  hipLaunchKernelGGL(k_hd_residual, hd_tiles(W, H), dim3(kHdThreads), 0, s, m, f, u, W, H, r, rr, bb);
  return hipGetLastError();
}
hipError_t hd_start(const uint8_t *m, const float *r, int W, int H, float *w, double *del, hipStream_t s) {
  hipLaunchKernelGGL(k_hd_aw, hd_tiles(W, H), dim3(kHdThreads), 0, s, m, r, W, H, w, del);
  return hipGetLastError();
}
hipError_t hd_iterate(const uint8_t *m, int W, int H, double *GAM, double *DEL, double *ALPHA, const double *BB,
                      double tol2, int it, float *u, float *p, const float *ri, const float *wi, const float *si,
                      float *ro, float *wo, float *so, hipStream_t s) {
  const dim3 t = hd_tiles(W, H);
  const dim3 g(std::min<unsigned>(t.x * t.y, kHdWgs));
  hipLaunchKernelGGL(k_hd_cg, g, dim3(kHdThreads), 0, s, m, W, H, GAM, DEL, ALPHA, BB, tol2, it, u, p, ri, wi, si, ro,
                     wo, so);
  return hipGetLastError();
}
hipError_t hd_zero(double *a, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_hd_zero, hd_grid(n), dim3(kHdThreads), 0, s, a, n);
  return hipGetLastError();
}

}  // namespace pdi
