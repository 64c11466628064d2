// Device helpers shared by the gfx950 kernel sources (HIP only).
#pragma once
#include "pdinp_internal.h"

#include <hip/hip_runtime.h>

namespace pdi {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i2 __attribute__((ext_vector_type(2)));

// Hand block m of frame fi to the general path: blocks whose bordered system
// fits in LDS are listed from the front of the deferred list, larger ones from
// the back (K = w*h is decoded by a copy, but solved when encoding).
__device__ __forceinline__ void push_deferred(const FrameDev &f, int fi, int m, int K, int w, int h) {
  const int e = (fi << kDeferFrameShift) | m;
  if (K > kLdsKMax && (K < w * h || f.enc)) {
    int idx = atomicAdd(&f.counters[1], 1);
    f.deferred[f.n_items * f.nframes - 1 - idx] = e;
  } else {
    int idx = atomicAdd(&f.counters[0], 1);
    f.deferred[idx] = e;
  }
}

// Output planes of one frame of a launch: FP32, or int8 = clamp(rint(u),
// -128, 127) with round-half-to-even when the frame asks for 8-bit output.
// Taken once per wave, so that the pixel stores need no reload of the
// frame's pointer; element offsets fit in 32 bits (the host limits a
// plane to 2^30 pixels).
struct PlaneOut {
  float *f32;   // FP32 planes, or null
  int8_t *i8;   // int8 planes, or null
};
__device__ __forceinline__ PlaneOut plane_out(const FrameDev &f, int fi) {
  float *o = f.fp[fi].out;
  PlaneOut po;
  po.f32 = f.out_i8 ? nullptr : o;
  po.i8 = f.out_i8 ? reinterpret_cast<int8_t *>(o) : nullptr;
  return po;
}
// FP32 pixel stores are non-temporal: the planes are written once and not
// read back by the decode, so they stream to HBM instead of displacing the
// tables, entries and point runs held in the caches.  int8 planes keep
// ordinary stores: a wave writes them in pieces of a few bytes per row,
// which the L2 must merge before they go to HBM.
__device__ __forceinline__ void store_px(const PlaneOut &po, unsigned idx, float u) {
  if (po.i8) {
    const float q = fminf(fmaxf(__builtin_rintf(u), -128.f), 127.f);
    po.i8[idx] = (int8_t)(int)q;
  } else {
    __builtin_nontemporal_store(u, po.f32 + idx);
  }
}

// Four consecutive pixels of one row: one 16-byte store (FP32 planes) or one
// 4-byte store (int8 planes) where the address is aligned for it, else one
// store per pixel; pixels from x0 + n on are outside the block (n <= 4).
__device__ __forceinline__ void store_px4(const PlaneOut &po, unsigned idx, const float u[4], int n) {
  if (po.i8) {
    int8_t q[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) q[r] = (int8_t)(int)fminf(fmaxf(__builtin_rintf(u[r]), -128.f), 127.f);
    if (n == 4 && (reinterpret_cast<uintptr_t>(po.i8 + idx) & 3u) == 0) {
      *reinterpret_cast<int *>(po.i8 + idx) =
          (int)((unsigned)(uint8_t)q[0] | ((unsigned)(uint8_t)q[1] << 8) | ((unsigned)(uint8_t)q[2] << 16) |
                ((unsigned)(uint8_t)q[3] << 24));
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (r < n) po.i8[idx + r] = q[r];
    }
  } else if (n == 4 && (reinterpret_cast<uintptr_t>(po.f32 + idx) & 15u) == 0) {
    __builtin_nontemporal_store(f4{u[0], u[1], u[2], u[3]}, reinterpret_cast<f4 *>(po.f32 + idx));
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (r < n) __builtin_nontemporal_store(u[r], po.f32 + idx + r);
  }
}

// Reconstruction of a stored code (dead-zone quantiser, Sec. 2.3 of the
// paper): 0 stays 0, else sign(q) (|q| + rho) step.
// Dead-zone quantisation of a coefficient (the inverse of coef_value's
// intervals): |c| in [k step, (k + 1) step) gives code sign(c) k, k <= 127;
// |c| < step gives 0.
__device__ __forceinline__ int quant_code(float c, float step) {
  const float k = fminf(floorf(fabsf(c) / step), 127.f);  // NaN -> 127: flagged by the caller
  return c < 0.f ? -(int)k : (int)k;
}

__device__ __forceinline__ float coef_value(int q, float step, float rho) {
  const float m = ((float)abs(q) + rho) * step;
  return q == 0 ? 0.f : (q > 0 ? m : -m);
}

// Green's function from the quarter-scaled compact table of a w x h shape:
// G(x_a, x_b) = sum over the 4 (alpha, beta) pairs from |x_a - x_b| and the
// reflected x_a + x_b + 1 per axis.
template <typename T>
__device__ __forceinline__ T green_tab(const T *tab, int w, int h, int xa, int ya, int xb, int yb) {
  const int W1 = w + 1;
  int dx = abs(xa - xb), dy = abs(ya - yb);
  int sx = xa + xb + 1, sy = ya + yb + 1;
  sx = min(sx, 2 * w - sx);
  sy = min(sy, 2 * h - sy);
  return (tab[dy * W1 + dx] + tab[dy * W1 + sx]) + (tab[sy * W1 + dx] + tab[sy * W1 + sx]);
}

// Make this lane's LDS writes visible to the other lanes of its wave (no
// instruction beyond the wait the writes need).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Broadcast lane `src` of every 16-lane row (DPP row_newbcast).  `src` must
// fold to a constant after unrolling.  Callers whose consumers are VOP2 ALU
// instructions pass the result through pin_v(): row_newbcast folded into
// other VOP2 instructions gave wrong results on gfx950, so every broadcast
// stays a standalone v_mov_b32_dpp (tests/test_isa.py checks the ISA).
__device__ __forceinline__ int bcast_i(int x, int src) {
#define PDI_NB(n) case n: return __builtin_amdgcn_mov_dpp(x, 0x150 + n, 0xF, 0xF, true);
  switch (src & 15) {
    PDI_NB(0) PDI_NB(1) PDI_NB(2) PDI_NB(3) PDI_NB(4) PDI_NB(5) PDI_NB(6) PDI_NB(7)
    PDI_NB(8) PDI_NB(9) PDI_NB(10) PDI_NB(11) PDI_NB(12) PDI_NB(13) PDI_NB(14) PDI_NB(15)
  }
#undef PDI_NB
  return x;
}
// Empty statement that takes and "returns" v: the value is materialised in a
// VGPR here, so its producer cannot be merged into its consumers.
__device__ __forceinline__ void pin_v(int &v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ float bcast_f(float x, int src) {
  return __builtin_bit_cast(float, bcast_i(__builtin_bit_cast(int, x), src));
}

}  // namespace pdi
