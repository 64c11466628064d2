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

constexpr int kHdThreads = 1024;

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

// Kernels run on 64 x 16 pixel tiles: thread (tx, ty) of tile (bx, by)
// owns pixel (64 bx + tx, 16 by + ty).  The per-level kernels take one tile
// per workgroup (a 2D grid); the per-iteration kernels are persistent (at
// most kHdWgs workgroups, each looping over tiles) so that the scalars are
// read and the partial sums added once per workgroup, not once per tile.
constexpr int kTx = 64, kTy = 16;
constexpr int kHdWgs = 512;  // two 1024-thread workgroups per compute unit
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

// One half of CG iteration it: p = r + beta p_old (beta = RR[it] / RR[it-1],
// 0 for it = 0), formed once per pixel of a tile and its one-pixel halo in
// LDS (0 on the mask and outside the plane); q = A_UU p from LDS;
// PQ[it] += p . q.  RR and PQ hold kHdSlots slots per iteration.
__global__ __launch_bounds__(kHdThreads) void k_hd_apply(const uint8_t *m, const float *r, const float *pold,
                                                         int W, int H, const double *RR, int it, float *pnew,
                                                         float *q, double *PQ) {
  __shared__ float ps[kTy + 2][kTx + 2];
  const int tx = threadIdx.x & (kTx - 1), ty = threadIdx.x / kTx;
  const int ntx = (W + kTx - 1) / kTx, ntiles = ntx * ((H + kTy - 1) / kTy);
  float beta = 0.f;
  if (it) {
    const double prev = slot_sum(RR + (it - 1) * kHdSlots);
    if (prev > 0.0) beta = (float)(slot_sum(RR + it * kHdSlots) / prev);  // 0 once converged exactly
  }
  double s = 0.0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int x0 = (t % ntx) * kTx, y0 = (t / ntx) * kTy;
    __syncthreads();  // the previous tile's LDS reads are done
    for (int k = threadIdx.x; k < (kTy + 2) * (kTx + 2); k += kHdThreads) {
      const int ly = k / (kTx + 2), lx = k - ly * (kTx + 2);
      const int gx = x0 + lx - 1, gy = y0 + ly - 1;
      float v = 0.f;
      if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
        const int j = gy * W + gx;
        if (!m[j]) v = r[j] + beta * pold[j];
      }
      ps[ly][lx] = v;
    }
    __syncthreads();
    const int x = x0 + tx, y = y0 + ty;
    if (x < W && y < H) {
      const int i = y * W + x;
      const float pi = ps[ty + 1][tx + 1];
      float qi = 0.f;
      if (!m[i]) {
        // neighbours inside the plane; a masked neighbour holds p = 0
        float nsum = 0.f, deg = 0.f;
        if (x > 0) { nsum += ps[ty + 1][tx]; deg += 1.f; }
        if (x + 1 < W) { nsum += ps[ty + 1][tx + 2]; deg += 1.f; }
        if (y > 0) { nsum += ps[ty][tx + 1]; deg += 1.f; }
        if (y + 1 < H) { nsum += ps[ty + 2][tx + 1]; deg += 1.f; }
        qi = deg * pi - nsum;
        s += (double)pi * qi;
      }
      pnew[i] = pi;
      q[i] = qi;
    }
  }
  wg_add2(s, 0.0, PQ + it * kHdSlots, nullptr);
}

// The other half: alpha = RR[it] / PQ[it]; u += alpha p; r -= alpha q;
// RR[it + 1] += |r|^2 (pointwise: the workgroups stride over the pixels).
__global__ __launch_bounds__(kHdThreads) void k_hd_update(const float *p, const float *q, int W, int H,
                                                          const double *RR, const double *PQ, int it, float *u,
                                                          float *r, double *RRn) {
  const double pq = slot_sum(PQ + it * kHdSlots);
  const float alpha = pq > 0.0 ? (float)(slot_sum(RR + it * kHdSlots) / pq) : 0.f;
  const int n = W * H;
  double s = 0.0;
  for (int i = blockIdx.x * kHdThreads + threadIdx.x; i < n; i += gridDim.x * kHdThreads) {
    const float ri = r[i] - alpha * q[i];
    u[i] += alpha * p[i];
    r[i] = ri;
    s += (double)ri * ri;
  }
  wg_add2(s, 0.0, RRn, nullptr);
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
hipError_t hd_iterate(const uint8_t *m, int W, int H, const double *RR, const double *PQ, int it, float *u, float *r,
                      const float *pold, float *pnew, float *q, hipStream_t s) {
  const dim3 t = hd_tiles(W, H);
  const dim3 g(std::min<unsigned>(t.x * t.y, kHdWgs));
  hipLaunchKernelGGL(k_hd_apply, g, dim3(kHdThreads), 0, s, m, r, pold, W, H, RR, it, pnew, q,
                     const_cast<double *>(PQ));
  hipLaunchKernelGGL(k_hd_update, g, dim3(kHdThreads), 0, s, pnew, q, W, H, RR, PQ, it, u, r,
                     const_cast<double *>(RR) + (it + 1) * kHdSlots);
  return hipGetLastError();
}
hipError_t hd_zero(double *a, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_hd_zero, hd_grid(n), dim3(kHdThreads), 0, s, a, n);
  return hipGetLastError();
}

}  // namespace pdi
