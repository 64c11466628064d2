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
    const int slot = blockIdx.x % kHdSlots;
    atomicAdd(dst0 + slot, s);
    if (dst1) atomicAdd(dst1 + slot, t);
  }
}

// Coarser level: a pixel is known when one of its (up to 4) children is,
// with the mean of the known children's values.
__global__ __launch_bounds__(kHdThreads) void k_hd_restrict(const uint8_t *mf, const float *ff, int Wf, int Hf,
                                                            uint8_t *mc, float *fc, int Wc, int Hc) {
  const int i = blockIdx.x * kHdThreads + threadIdx.x;
  if (i >= Wc * Hc) return;
  const int x = i % Wc, y = i / Wc;
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
  mc[i] = n ? 1 : 0;
  fc[i] = n ? s / (float)n : 0.f;
}

// Initial guess of a level: the known values on the mask, the coarser
// level's solution (nearest parent) elsewhere, or 0 on the coarsest level.
__global__ __launch_bounds__(kHdThreads) void k_hd_init(const uint8_t *m, const float *f, int W, int H,
                                                        const float *uc, int Wc, float *u) {
  const int i = blockIdx.x * kHdThreads + threadIdx.x;
  if (i >= W * H) return;
  const int x = i % W, y = i / W;
  u[i] = m[i] ? f[i] : (uc ? uc[(y >> 1) * Wc + (x >> 1)] : 0.f);
}

// r = -(A u) off the mask, 0 on it; RR[0] += |r|^2 and BB += |b|^2 with b
// the right-hand side of the unknowns' system A_UU u_U = b (b_i = sum of
// the known neighbours' values).
__global__ __launch_bounds__(kHdThreads) void k_hd_residual(const uint8_t *m, const float *f, const float *u,
                                                            int W, int H, float *r, double *rr, double *bb) {
  const int i = blockIdx.x * kHdThreads + threadIdx.x;
  double sr = 0.0, sb = 0.0;
  if (i < W * H) {
    float ri = 0.f;
    if (!m[i]) {
      const int x = i % W, y = i / W;
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
// 0 for it = 0), evaluated at the pixel and its neighbours; q = A_UU p;
// PQ[it] += p . q.  RR and PQ hold kHdSlots slots per iteration.
__global__ __launch_bounds__(kHdThreads) void k_hd_apply(const uint8_t *m, const float *r, const float *pold,
                                                         int W, int H, const double *RR, int it, float *pnew,
                                                         float *q, double *PQ) {
  const int i = blockIdx.x * kHdThreads + threadIdx.x;
  float beta = 0.f;
  if (it) {
    const double prev = slot_sum(RR + (it - 1) * kHdSlots);
    if (prev > 0.0) beta = (float)(slot_sum(RR + it * kHdSlots) / prev);  // 0 once converged exactly
  }
  double s = 0.0;
  if (i < W * H) {
    float pi = 0.f, qi = 0.f;
    if (!m[i]) {
      const int x = i % W, y = i / W;
      pi = r[i] + beta * pold[i];
      const int nb[4] = {x > 0 ? i - 1 : -1, x + 1 < W ? i + 1 : -1, y > 0 ? i - W : -1, y + 1 < H ? i + W : -1};
      for (int k = 0; k < 4; ++k) {
        const int j = nb[k];
        if (j >= 0) qi += pi - (m[j] ? 0.f : r[j] + beta * pold[j]);
      }
      s = (double)pi * qi;
    }
    pnew[i] = pi;
    q[i] = qi;
  }
  wg_add2(s, 0.0, PQ + it * kHdSlots, nullptr);
}

// The other half: alpha = RR[it] / PQ[it]; u += alpha p; r -= alpha q;
// RR[it + 1] += |r|^2.
__global__ __launch_bounds__(kHdThreads) void k_hd_update(const float *p, const float *q, int W, int H,
                                                          const double *RR, const double *PQ, int it, float *u,
                                                          float *r, double *RRn) {
  const int i = blockIdx.x * kHdThreads + threadIdx.x;
  const double pq = slot_sum(PQ + it * kHdSlots);
  const float alpha = pq > 0.0 ? (float)(slot_sum(RR + it * kHdSlots) / pq) : 0.f;
  double s = 0.0;
  if (i < W * H) {
    const float ri = r[i] - alpha * q[i];
    u[i] += alpha * p[i];
    r[i] = ri;
    s = (double)ri * ri;
  }
  wg_add2(s, 0.0, RRn, nullptr);
}

__global__ __launch_bounds__(kHdThreads) void k_hd_zero(double *a, int n) {
  const int i = blockIdx.x * kHdThreads + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

static inline dim3 hd_grid(long long n) { return dim3((unsigned)((n + kHdThreads - 1) / kHdThreads)); }

hipError_t hd_restrict(const uint8_t *mf, const float *ff, int Wf, int Hf, uint8_t *mc, float *fc, int Wc, int Hc,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_hd_restrict, hd_grid((long long)Wc * Hc), dim3(kHdThreads), 0, s, mf, ff, Wf, Hf, mc, fc, Wc, Hc);
  return hipGetLastError();
}
hipError_t hd_init(const uint8_t *m, const float *f, int W, int H, const float *uc, int Wc, float *u, hipStream_t s) {
  hipLaunchKernelGGL(k_hd_init, hd_grid((long long)W * H), dim3(kHdThreads), 0, s, m, f, W, H, uc, Wc, u);
  return hipGetLastError();
}
hipError_t hd_residual(const uint8_t *m, const float *f, const float *u, int W, int H, float *r, double *rr,
                       double *bb, hipStream_t s) {
  hipLaunchKernelGGL(k_hd_residual, hd_grid((long long)W * H), dim3(kHdThreads), 0, s, m, f, u, W, H, r, rr, bb);
  return hipGetLastError();
}
hipError_t hd_iterate(const uint8_t *m, int W, int H, const double *RR, const double *PQ, int it, float *u, float *r,
                      const float *pold, float *pnew, float *q, hipStream_t s) {
  const dim3 g = hd_grid((long long)W * H);
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
