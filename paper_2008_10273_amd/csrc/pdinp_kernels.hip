// gfx950 kernels of the residual decoder.
//
// Per block (Sec. 2.2 of the paper): assemble the kernel matrix G_K over the
// K mask points from the Green's function, solve the bordered (K+1) system
// [G_K 1; 1^T 0][c; a] = [r; 0], and evaluate u(x) = sum_i c_i G(x, x_i) + a
// at every pixel of the block.
//
// Two paths:
//  * k_fast - wave-level, 4 blocks per wave, one 16-lane DPP row per block,
//    a lane holds one (K <= 15) or two (K <= 31) rows of the bordered
//    system in VGPRs.  Gauss-Jordan elimination without pivoting (the
//    leading K x K block is SPD, and the last pivot is -1^T G_K^-1 1 != 0);
//    pivot rows are broadcast with DPP row_newbcast.  The evaluation uses the
//    DCT-II factorisation of G (Eq. 4): V = Dw[:,X] diag(c) Dh[:,Y]^T (inner
//    dimension K), U = Dh^T (lam .* V^T) Dw, as chained 16x16x4 FP32 MFMAs.
//  * k_general - one 256-thread workgroup per block, system in LDS (or a
//    global slot for large K), Gauss-Jordan with barriers, direct
//    evaluation through the Green table.  It is the plain per-block path,
//    and the fallback for blocks the fast path does not take.
#include "pdinp_device.h"

#include <type_traits>

#include <hip/hip_runtime.h>

namespace pdi {

// ------------------------------------------------------------------ items

struct Item {
  int K, base, w, h, x0, y0, shape, nv, W, g, l;  // g: group, l: block index in its plane
  long long vbase0, vbase1, obase0, obase1;
  __device__ __forceinline__ long long vbase(int v) const { return v ? vbase1 : vbase0; }
  __device__ __forceinline__ long long obase(int v) const { return v ? obase1 : obase0; }
};

__device__ __forceinline__ Item load_item(const FrameDev &f, const int32_t *bp, int m) {
  Item it;
  int g = 0;
  if (f.ngroups > 1 && m >= f.g[1].first) g = 1;
  if (f.ngroups > 2 && m >= f.g[2].first) g = 2;
  const GroupDev &G = f.g[g];
  const int b = f.b;
  int l = m - G.first;
  it.g = g;
  it.l = l;
  int bx = l % G.nbx, by = l / G.nbx;
  it.x0 = bx * b;
  it.y0 = by * b;
  it.w = min(b, G.W - it.x0);
  it.h = min(b, G.H - it.y0);
  int e = ((bx == G.nbx - 1) && (G.W % b) ? 1 : 0) + ((by == G.nby - 1) && (G.H % b) ? 2 : 0);
  it.shape = G.shape[e];
  int lo = bp[m], hi = bp[m + 1];
  it.K = hi - lo;
  it.base = lo;
  it.nv = G.nv;
  it.W = G.W;
  const long long pix = (long long)it.y0 * G.W + it.x0;
  it.vbase0 = lo;
  it.obase0 = G.out_off[0] + pix;
  if (G.nv > 1) {
    // a shared chroma mask: the Cr run follows every other value
    it.vbase1 = f.shared ? (long long)bp[f.n_items] + (lo - bp[f.chroma_first]) : lo;
    it.obase1 = G.out_off[1] + pix;
  } else {
    it.vbase1 = it.vbase0;
    it.obase1 = it.obase0;
  }
  return it;
}


// ------------------------------------------------------- general per-block

constexpr int kGenThreads = 256;
constexpr int kGeneralGrid = 128;  // persistent workgroups over the deferred lists

// Workgroup scratch of the general path for blocks of at most B x B pixels.
template <int B>
struct GenScratch {
  float tab[(B + 1) * (B + 1)];
  short px[B * B], py[B * B];
  float c[2][B * B];
  float fcol[B * B + 1];
  float rho[B * B + 1];
  double red[kGenThreads / 64];
  float redf[2][kGenThreads / 64];
  int flag;
};

struct GenShared {
  float M[(kLdsKMax + 1) * (kLdsKMax + 3)];
  GenScratch<32> g;
};

__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kGenThreads / 64; ++i) s += red[i];
  return s;
}

// Coefficient encodes: the constant of value column v of item `it`, and
// codes 0 for its first n points (blocks that are not solved).
__device__ __forceinline__ void enc_zero(const FrameDev &f, const FramePtrs &fp, const Item &it, int n) {
  const GroupDev &G = f.g[it.g];
  if (threadIdx.x < it.nv) fp.aout[G.cbase[threadIdx.x] + it.l] = 0.f;
  for (int v = 0; v < it.nv; ++v)
    for (int i = threadIdx.x; i < n; i += kGenThreads) fp.qout[it.vbase(v) + i] = 0;
}

// Decode one block with a whole workgroup.  M points at LDS (K <= kLdsKMax)
// or at a global slot (ld = row stride).  Coefficient encodes (f.enc) stop
// after the solve and store the quantised c and a instead.
template <int B>
__device__ void general_block(const FrameDev &f, int fi, int m, GenScratch<B> &sh, float *M) {
  const int tid = threadIdx.x;
  fi = __builtin_amdgcn_readfirstlane(fi);
  const FramePtrs fp = f.fp[fi];
  const Item it = load_item(f, fp.block_ptr, m);
  const uint16_t *pos = fp.pos;
  const float *values = fp.values;
  const int K = it.K, w = it.w, h = it.h, N = w * h;
  const ShapeDev S = f.s[it.shape];
  const PlaneOut po = plane_out(f, fi);

  if (tid == 0) sh.flag = 0;
  __syncthreads();
  if (K < 0 || K > N) {
    if (tid == 0) atomicOr(f.status, kStatusMask);
    if (f.enc) {
      enc_zero(f, fp, it, 0);
      return;
    }
    for (int v = 0; v < it.nv; ++v)
      for (int p = tid; p < N; p += kGenThreads) store_px(po, (unsigned)(it.obase(v) + (p / w) * it.W + p % w), 0.f);
    return;
  }
  if (f.validate) {
    int bad = 0;
    for (int i = tid; i < K; i += kGenThreads) {
      int p = pos[it.base + i];
      if (p >= N || (i > 0 && pos[it.base + i - 1] >= p)) bad |= kStatusMask;
      for (int v = 0; v < it.nv; ++v)
        if (!isfinite(values[it.vbase(v) + i])) bad |= kStatusValue;
    }
    if (bad) { atomicOr(f.status, bad); atomicOr(&sh.flag, 1); }
    __syncthreads();
    if (sh.flag) {
      if (f.enc) {
        enc_zero(f, fp, it, K);
        return;
      }
      for (int v = 0; v < it.nv; ++v)
        for (int p = tid; p < N; p += kGenThreads) store_px(po, (unsigned)(it.obase(v) + (p / w) * it.W + p % w), 0.f);
      return;
    }
  }
  if (K == 0) {
    if (f.enc) {  // u = 0: a = 0
      enc_zero(f, fp, it, 0);
      return;
    }
    for (int v = 0; v < it.nv; ++v)
      for (int p = tid; p < N; p += kGenThreads) store_px(po, (unsigned)(it.obase(v) + (p / w) * it.W + p % w), 0.f);
    return;
  }
  // Every pixel known: u = r.  G_K is then the whole G, singular on the
  // constants; an encode solves with G + 1 1^T instead, which has the same
  // solution (sum c = 0) and is positive definite.
  const float shift = (f.enc && K == N) ? 1.f : 0.f;
  if (K == N && !f.enc) {
    for (int v = 0; v < it.nv; ++v)
      for (int i = tid; i < K; i += kGenThreads) {
        int p = min((int)pos[it.base + i], N - 1);
        store_px(po, (unsigned)(it.obase(v) + (p / w) * it.W + p % w), values[it.vbase(v) + i]);
      }
    return;
  }

  for (int i = tid; i < (w + 1) * (h + 1); i += kGenThreads) sh.tab[i] = f.tab32[S.hc32 + i];
  for (int i = tid; i < K; i += kGenThreads) {
    int p = min((int)pos[it.base + i], N - 1);
    sh.px[i] = (short)(p % w);
    sh.py[i] = (short)(p / w);
  }
  __syncthreads();

  // Bordered system, rows 0..K, columns 0..K then the value columns.
  const int n = K + 1, ld = n + it.nv;
  const int lane = tid & 63, wid = tid >> 6;
  for (int i = wid; i < n; i += kGenThreads / 64)
    for (int k = lane; k < ld; k += 64) {
      float v;
      if (k < K) v = (i < K) ? green_tab(sh.tab, w, h, sh.px[i], sh.py[i], sh.px[k], sh.py[k]) + shift : 1.f;
      else if (k == K) v = (i < K) ? 1.f : 0.f;
      else v = (i < K) ? values[it.vbase(k - n) + i] : 0.f;
      M[(long long)i * ld + k] = v;
    }

  // Gauss-Jordan without pivoting; the multiplier of row i at step j is kept
  // in M[i][j] for the refinement replay.
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    const float piv = M[(long long)j * ld + j];
    const float rp = 1.0f / piv;
    for (int i = tid; i < n; i += kGenThreads) sh.fcol[i] = (i == j) ? 0.f : M[(long long)i * ld + j] * rp;
    __syncthreads();
    for (int i = wid; i < n; i += kGenThreads / 64) {
      if (i == j) continue;
      const float fi = sh.fcol[i];
      for (int k = j + 1 + lane; k < ld; k += 64)
        M[(long long)i * ld + k] = fmaf(-fi, M[(long long)j * ld + k], M[(long long)i * ld + k]);
      if (lane == 0) M[(long long)i * ld + j] = fi;
    }
  }
  __syncthreads();

  // Solution and pivot ratio over the SPD block.
  float dmin = 3.0e38f, dmax = 0.f;
  for (int i = tid; i < K; i += kGenThreads) {
    float d = fabsf(M[(long long)i * ld + i]);
    dmin = fminf(dmin, d);
    dmax = fmaxf(dmax, d);
  }
  for (int o = 32; o > 0; o >>= 1) {
    dmin = fminf(dmin, __shfl_xor(dmin, o));
    dmax = fmaxf(dmax, __shfl_xor(dmax, o));
  }
  if (lane == 0) { sh.redf[0][wid] = dmin; sh.redf[1][wid] = dmax; }
  for (int v = 0; v < it.nv; ++v)
    for (int i = tid; i < n; i += kGenThreads) {
      float x = M[(long long)i * ld + n + v] / M[(long long)i * ld + i];
      if (i < K) sh.c[v][i] = x; else sh.rho[v] = x;  // rho[0..nv) holds a until reused
    }
  __syncthreads();
  dmin = fminf(fminf(sh.redf[0][0], sh.redf[0][1]), fminf(sh.redf[0][2], sh.redf[0][3]));
  dmax = fmaxf(fmaxf(sh.redf[1][0], sh.redf[1][1]), fmaxf(sh.redf[1][2], sh.redf[1][3]));
  float a0 = sh.rho[0], a1 = it.nv > 1 ? sh.rho[1] : 0.f;  // a of each value set
  const bool refine = (f.refine == 2) || (f.refine == 1 && !(dmin >= f.tau * dmax));

  if (refine) {
    const double *tab64 = f.tab64 + S.hc64;
    for (int v = 0; v < it.nv; ++v) {
      __syncthreads();
      // FP64 residual of the bordered system: rho_i = r_i - a - sum_k G_ik c_k,
      // rho_K = -sum_k c_k.
      double cs = 0.0;
      for (int i = tid; i < K; i += kGenThreads) cs += (double)sh.c[v][i];
      cs = block_sum(cs, sh.red);
      for (int i = tid; i < K; i += kGenThreads) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k)
          acc += green_tab(tab64, w, h, (int)sh.px[i], (int)sh.py[i], (int)sh.px[k], (int)sh.py[k]) *
                 (double)sh.c[v][k];
        double r = (double)values[it.vbase(v) + i];
        sh.rho[i] = (float)(r - (double)(v ? a1 : a0) - acc - (double)shift * cs);
      }
      if (tid == 0) sh.rho[K] = (float)(-cs);
      // Replay the elimination on rho, then divide by the pivots.
      for (int j = 0; j < n; ++j) {
        __syncthreads();
        const float tj = sh.rho[j];
        __syncthreads();
        for (int i = tid; i < n; i += kGenThreads)
          if (i != j) sh.rho[i] = fmaf(-M[(long long)i * ld + j], tj, sh.rho[i]);
      }
      __syncthreads();
      for (int i = tid; i < K; i += kGenThreads) sh.c[v][i] += sh.rho[i] / M[(long long)i * ld + i];
      const float da = sh.rho[K] / M[(long long)K * ld + K];
      if (v) a1 += da; else a0 += da;
    }
    __syncthreads();
  }

  if (f.enc) {  // quantised c and a; no evaluation
    const GroupDev &G = f.g[it.g];
    bool bad = false;
    for (int v = 0; v < it.nv; ++v) {
      const float step = f.qstep[G.vplane[v]];
      for (int i = tid; i < K; i += kGenThreads) {
        const float c = sh.c[v][i];
        bad |= !isfinite(c);
        fp.qout[it.vbase(v) + i] = (int8_t)quant_code(c, step);
      }
    }
    if (tid < it.nv) {
      const float a = tid ? a1 : a0;
      bad |= !isfinite(a);
      fp.aout[G.cbase[tid] + it.l] = a;
    }
    if (bad) atomicOr(f.status, kStatusSolve);
    return;
  }

  // Direct evaluation u(x) = sum_i c_i G(x, x_i) + a.
  bool bad = false;
  for (int p = tid; p < N; p += kGenThreads) {
    const int xx = p % w, yy = p / w;
    float acc0 = 0.f, acc1 = 0.f;
    for (int i = 0; i < K; ++i) {
      float g = green_tab(sh.tab, w, h, xx, yy, (int)sh.px[i], (int)sh.py[i]);
      acc0 = fmaf(sh.c[0][i], g, acc0);
      if (it.nv > 1) acc1 = fmaf(sh.c[1][i], g, acc1);
    }
    float u0 = acc0 + a0;
    bad |= !isfinite(u0);
    store_px(po, (unsigned)(it.obase0 + (long long)yy * it.W + xx), u0);
    if (it.nv > 1) {
      float u1 = acc1 + a1;
      bad |= !isfinite(u1);
      store_px(po, (unsigned)(it.obase1 + (long long)yy * it.W + xx), u1);
    }
  }
  if (bad) atomicOr(f.status, kStatusSolve);
}

// One workgroup per mask block (the plain per-block path).  Blocks whose
// system does not fit in LDS go to the large list.
__global__ __launch_bounds__(kGenThreads) void k_plain_all(FrameDev f) {
  __shared__ GenShared sh;
  const int m = blockIdx.x, fi = blockIdx.y;
  if (m >= f.n_items) return;
  const Item it = load_item(f, f.fp[fi].block_ptr, m);
  if (it.K > kLdsKMax && (it.K < it.w * it.h || f.enc)) {
    if (threadIdx.x == 0) push_deferred(f, fi, m, it.K, it.w, it.h);
    return;
  }
  general_block<32>(f, fi, m, sh.g, sh.M);
}

// Persistent pass over the deferred lists; the last workgroup clears the
// counters for the next decode on this context.
__global__ __launch_bounds__(kGenThreads) void k_general_deferred(FrameDev f) {
  __shared__ GenShared sh;
  const int nmed = f.counters[0];
  const int nlarge = f.counters[1];
  const int cap = f.n_items * f.nframes;
  // Nothing deferred and no queue counters in use: every counter is still
  // zero, so there is nothing to decode or clear.
  if (nmed + nlarge == 0 && f.nq == 0) return;
  for (int idx = blockIdx.x; idx < nmed; idx += gridDim.x) {
    __syncthreads();
    const int e = f.deferred[idx];
    general_block<32>(f, e >> kDeferFrameShift, e & kDeferItemMask, sh.g, sh.M);
  }
  if ((int)blockIdx.x < f.slot_wgs) {
    float *slot = f.slots + (long long)blockIdx.x * f.slot_floats;
    for (int idx = blockIdx.x; idx < nlarge; idx += f.slot_wgs) {
      __syncthreads();
      const int e = f.deferred[cap - 1 - idx];
      general_block<32>(f, e >> kDeferFrameShift, e & kDeferItemMask, sh.g, slot);
    }
  }
  // Every workgroup has read both counts before it gets here; the last one
  // to arrive clears every counter (these and the wave-per-block queues',
  // whose kernels ran before this one) for the next decode; the kernel
  // boundary orders these writes before any later kernel on the stream.
  __syncthreads();
  if (threadIdx.x == 0)
    sh.g.flag = __hip_atomic_fetch_add(&f.counters[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                (int)gridDim.x - 1;
  __syncthreads();
  if (sh.g.flag)
    for (int i = threadIdx.x; i < kNumCounters; i += kGenThreads)
      __hip_atomic_store(&f.counters[i], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// -------------------------------------------------------- wave-level path

// The 64-bit value v of lane `src` (uniform result).
__device__ __forceinline__ long long lane_i64(long long v, int src) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)v, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), src);
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// Minimum / maximum over the 16 lanes of a DPP row, in DPP lane moves
// (quad swaps, then the half-row and row mirrors): no LDS round trip.
__device__ __forceinline__ float row_dpp(float v, int ctrl) {
  int r = 0;
  switch (ctrl) {
    case 0: r = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false); break;   // quad [1,0,3,2]
    case 1: r = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false); break;   // quad [2,3,0,1]
    case 2: r = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false); break;  // row_half_mirror
    default: r = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false); break; // row_mirror
  }
  return __builtin_bit_cast(float, r);
}
__device__ __forceinline__ float row_min(float v) {
#pragma unroll
  for (int c = 0; c < 4; ++c) v = fminf(v, row_dpp(v, c));
  return v;
}
__device__ __forceinline__ float row_max(float v) {
#pragma unroll
  for (int c = 0; c < 4; ++c) v = fmaxf(v, row_dpp(v, c));
  return v;
}

constexpr int kFastThreads = 256;
constexpr int kFastWaves = kFastThreads / 64;
constexpr int kFastItems = kFastWaves * kWaveItems;  // blocks per workgroup
// 16-byte table loads per thread: J (16 jrow(16, 16) floats at most, rounded to 4)
// plus the DCT matrices and eigenvalues (3 kDct16Floats) of a b <= 16 shape.
constexpr int kTabVec = ((16 * jrow(16, 16) + 3) / 4 + 3 * kDct16Floats / 4 + kFastThreads - 1) / kFastThreads;
static_assert(kTabVec * kFastThreads * 4 <= kTabPadFloats, "table reads stay inside the padded buffer");

// A block of the workgroup, as staged by the prologue.
struct FastItem {
  int m, K, base, cls, nv;
  int fi;  // frame of the launch
  long long vb0, vb1, ob0, ob1;
};

// Evaluation operands of one mask point (16 bytes: one LDS read).
struct FastPoint {
  int x, y;
  float c0, c1;
};

struct FastStage {
  FastPoint p[kWaveItems][32];
  float a[kWaveItems][2];
  int e[kWaveItems];  // binned path: (frame << 24) | block of each row, kept over the solve
};

// Size class of a block for the wave-level path: 0, 1, 2, 3 -> R = 8, 16,
// 24, 32 rows (the bordered system of K points has K + 1 rows); kClassDefer
// -> not taken (general path); kClassNone marks an empty slot.  Only
// coefficient encodes (ENC8) use R = 8: instantiating it in the decoders
// grew their code past what their instruction cache holds, and decodes ran
// several times slower.  Stored-coefficient decodes (COEF) take K = 0
// (u = a) and K = w*h as well.
constexpr int kClassDefer = 4, kClassNone = 5;
template <bool COEF, bool ENC8>
__device__ __forceinline__ int fast_class(int K, int N) {
  if (COEF ? (K < 0 || K > N || K > kFastKMax) : (K < 1 || K >= N || K > kFastKMax)) return kClassDefer;
  return (ENC8 && K <= 7) ? 0 : (K <= 15 ? 1 : (K <= 23 ? 2 : 3));
}

// Stored-coefficient decodes: stage (x, y, c) of the wave's 4 blocks (codes
// dequantised, zeros up to R) and their constants, in place of the solve.
template <int R>
__device__ __forceinline__ void fast_coef_stage(const FrameDev &f, const FastItem *items, int slot, bool ok,
                                                int t, int gi, int w, int h, const GroupDev &G,
                                                FastStage &st) {
  constexpr int NS = (R + 15) / 16;
  const FramePtrs fp = f.fp[blockIdx.y];
  const int K = ok ? items[slot].K : 0, N = w * h, nv = ok ? items[slot].nv : 0;
  const int pl0 = G.vplane[0], pl1 = G.vplane[nv > 1 ? 1 : 0];
  int bad = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = t + 16 * s;
    FastPoint P{0, 0, 0.f, 0.f};
    if (i < K) {
      const int base = items[slot].base;
      int p = fp.pos[base + i];
      if (f.validate && (p >= N || (i > 0 && (int)fp.pos[base + i - 1] >= p))) bad |= kStatusMask;
      p = min(p, N - 1);
      P.x = p % w;
      P.y = p / w;
      const int q0 = fp.coef[items[slot].vb0 + i];
      const int q1 = nv > 1 ? (int)fp.coef[items[slot].vb1 + i] : 0;
      if (f.validate && (q0 == -128 || q1 == -128)) bad |= kStatusValue;
      P.c0 = coef_value(q0, f.qstep[pl0], f.qrho);
      P.c1 = coef_value(q1, f.qstep[pl1], f.qrho);
    }
    st.p[gi][i] = P;  // zeros past K up to 16 NS: 16-point chunks may read up to row 31
  }
  if (t < 2) {
    float a = 0.f;
    if (t < nv) {
      a = fp.consts[G.cbase[t] + (items[slot].m - G.first)];
      if (f.validate && !isfinite(a)) bad |= kStatusValue;
    }
    st.a[gi][t] = a;
  }
  if (bad) atomicOr(f.status, bad);
}

// The points of a wave-level block (row i < K of the system in lane
// t = i mod 16, slice i / 16): in-block coordinates and the value(s) at them.
template <int NS>
struct FastPts {
  int xr[NS], yr[NS];
  float T[NS][2];
};

// Loads the K points of a block (positions from posp[base..], values from
// vals[vb0..] and, with nv = 2, vals[vb1..]), checking them when the
// launch validates.
template <int R>
__device__ __forceinline__ FastPts<(R + 15) / 16> fast_load(const FrameDev &f, int K, int t, int w, int h,
                                                           const uint16_t *posp, const float *vals,
                                                           long long base, long long vb0, long long vb1, int nv) {
  constexpr int NS = (R + 15) / 16;
  // (the runs are in device memory: global loads, not flat ones)
  typedef const __attribute__((address_space(1))) uint16_t gpos_t;
  typedef const __attribute__((address_space(1))) float gval_t;
  gpos_t *gpos = (gpos_t *)posp;
  gval_t *gval = (gval_t *)vals;
  FastPts<NS> P;
  int pr[NS];
  // every slice's loads first (one wait for all of them)
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = t + 16 * s;
    pr[s] = 0;
    P.T[s][0] = P.T[s][1] = 0.f;
    if (i < K) {
      pr[s] = gpos[base + i];
      P.T[s][0] = gval[vb0 + i];
      if (nv > 1) P.T[s][1] = gval[vb1 + i];
    }
  }
  const int N = w * h;
  // y = floor(p / w) for p < 256, w <= 16: (p + 1/2) / w is at least 1/32
  // away from an integer, far beyond the rounding of the reciprocal
  const float rw = __builtin_amdgcn_rcpf((float)w);
  int bad = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = t + 16 * s;
    P.xr[s] = 0;
    P.yr[s] = 0;
    if (i < K) {
      int p = pr[s];
      if (f.validate) {
        if (p >= N || (i > 0 && (int)gpos[base + i - 1] >= p)) bad |= kStatusMask;
        if (!(isfinite(P.T[s][0]) && isfinite(P.T[s][1]))) bad |= kStatusValue;
      }
      p = min(p, N - 1);
      P.yr[s] = (int)(((float)p + 0.5f) * rw);
      P.xr[s] = p - P.yr[s] * w;
    }
  }
  if (bad) atomicOr(f.status, bad);
  return P;
}

// Solve the bordered systems of the wave's 4 blocks (R rows per block, two
// value columns; the points loaded by fast_load) and stage the evaluation
// operands.  J is the row-pair Green table of the workgroup's shape (LDS).
// Returns false for a block whose pivots call for FP64 refinement; such
// blocks are left to the general path, which refines.
//
// BIN: the wave's blocks come from one size class of the binned path, so
// every taken block has K >= R - 4 (columns and rows below R - 4 hold
// Green's-function entries only, and the first R - 4 elimination steps are
// never past a block's border).
template <int R, int KCH, bool BIN>
__device__ __forceinline__ bool fast_solve_pts(const FrameDev &f, bool ok, int K, int t, int gi, int Kw, int w,
                                               int h, const float *J, FastStage &st,
                                               FastPts<(R + 15) / 16> &pts) {
  constexpr int NS = (R + 15) / 16;
  constexpr int NV = 2;
  const int W1 = w + 1;
  int(&xr)[NS] = pts.xr;
  int(&yr)[NS] = pts.yr;
  float(&T)[NS][NV] = pts.T;

  // Assembly of row i of [G_K 1; 1^T 0] (identity on padding rows):
  // G(x_i, x_k) = J[y_i, y_k][|x_i - x_k|] + J[y_i, y_k][refl(x_i + x_k + 1)].
  // Indices are kept as byte offsets, so that |x_i - x_k| plus the row base
  // is one v_sad_u32 and no shift is needed per entry.
  int x4[NS], yrow[NS], ycol[NS], xi1[NS], xcr[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    x4[s] = 4 * xr[s];
    yrow[s] = 4 * yr[s] * jrow(w, h);
    ycol[s] = 4 * yr[s] * W1;
    xi1[s] = 4 * (xr[s] + 1);
    xcr[s] = 4 * (2 * w - 1 - xr[s]);
  }
  const char *Jb = reinterpret_cast<const char *>(J);
  // The table lookups are unconditional (every index is in range) so that
  // they issue back to back; the border and padding pattern is applied by
  // selects afterwards.
  float A[NS][R];
  constexpr int KC = KCH;  // columns whose lookups are issued together (R is a multiple of KC)
  static_assert(R % KC == 0 && (KC == 4 || KC == 8), "lookup chunks");
#pragma unroll
  for (int k0 = 0; k0 < R; k0 += KC) {
    float g1[NS][KC], g2[NS][KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int k = k0 + kk;
      int xk = bcast_i(x4[k >> 4], k & 15);
      int yk = bcast_i(ycol[k >> 4], k & 15);
      pin_v(xk);
      pin_v(yk);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int base = yrow[s] + yk;
        const int a1 = (int)__usad((unsigned)x4[s], (unsigned)xk, (unsigned)base);
        const int a2 = base + min(xi1[s] + xk, xcr[s] - xk);
        g1[s][kk] = *reinterpret_cast<const float *>(Jb + a1);
        g2[s][kk] = *reinterpret_cast<const float *>(Jb + a2);
      }
    }
    // Empty statements that take every looked-up value: the compiler keeps
    // all lookups of the chunk ahead of them (one wait instead of one per
    // entry).  They emit no instruction.
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if constexpr (KC == 8) {
        asm volatile("" : "+v"(g1[s][0]), "+v"(g1[s][1]), "+v"(g1[s][2]), "+v"(g1[s][3]),
                          "+v"(g1[s][4]), "+v"(g1[s][5]), "+v"(g1[s][6]), "+v"(g1[s][7]));
        asm volatile("" : "+v"(g2[s][0]), "+v"(g2[s][1]), "+v"(g2[s][2]), "+v"(g2[s][3]),
                          "+v"(g2[s][4]), "+v"(g2[s][5]), "+v"(g2[s][6]), "+v"(g2[s][7]));
      } else {
        asm volatile("" : "+v"(g1[s][0]), "+v"(g1[s][1]), "+v"(g1[s][2]), "+v"(g1[s][3]));
        asm volatile("" : "+v"(g2[s][0]), "+v"(g2[s][1]), "+v"(g2[s][2]), "+v"(g2[s][3]));
      }
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
      for (int s = 0; s < NS; ++s) A[s][k0 + kk] = g1[s][kk] + g2[s][kk];
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = t + 16 * s;
    const bool prow = i < K, brow = i == K;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if (BIN && k < R - 4 && 16 * s + 15 < R - 4) continue;  // every row and column a point's
      const float inner = prow ? A[s][k] : (brow ? 1.f : 0.f);            // columns k < K
      if (BIN && k < R - 4) {
        A[s][k] = inner;
        continue;
      }
      const float outer = ((k == K) && prow) || (i > K && i == k) ? 1.f : 0.f;  // columns k >= K
      A[s][k] = (k < K) ? inner : outer;
    }
  }

  // Gauss-Jordan elimination without pivoting.
  float diag[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) diag[s] = 1.f;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if ((BIN && j < R - 4) || j <= Kw) {
      const int jl = j & 15, js = j >> 4;
      const float piv = bcast_f(A[js][j], jl);
      const float rp = __builtin_amdgcn_rcpf(piv);
      float fs[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const bool isj = (s == js) && (t == jl);
        fs[s] = isj ? 0.f : A[s][j] * rp;
        if (isj) diag[s] = piv;
      }
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if (k > j) {
          const float bk = bcast_f(A[js][k], jl);
#pragma unroll
          for (int s = 0; s < NS; ++s) A[s][k] = fmaf(-fs[s], bk, A[s][k]);
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const float bt = bcast_f(T[js][v], jl);
#pragma unroll
        for (int s = 0; s < NS; ++s) T[s][v] = fmaf(-fs[s], bt, T[s][v]);
      }
    }
  }

  // Pivot ratio of the SPD part (rows < K) decides the FP64 refinement.
  float dmin = 3.0e38f, dmax = 0.f;
#pragma unroll
  for (int s = 0; s < NS; ++s)
    if (t + 16 * s < K) { dmin = fminf(dmin, fabsf(diag[s])); dmax = fmaxf(dmax, fabsf(diag[s])); }
  dmin = row_min(dmin);
  dmax = row_max(dmax);
  const bool need = ok && ((f.refine == 2) || (f.refine == 1 && !(dmin >= f.tau * dmax)));

  // Stage (x, y, c) of rows < K, zeros for the other rows up to R, and a.
  bool fin = true;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = t + 16 * s;
    const float rd = __builtin_amdgcn_rcpf(diag[s]);
    const float x0 = T[s][0] * rd, x1 = T[s][1] * rd;
    {  // every staged row past K holds zeros (16-point chunks may read up to row 31)
      FastPoint P;
      P.x = i < K ? xr[s] : 0;
      P.y = i < K ? yr[s] : 0;
      P.c0 = i < K ? x0 : 0.f;
      P.c1 = i < K ? x1 : 0.f;
      st.p[gi][i] = P;
    }
    if (i < K) fin &= isfinite(x0) && isfinite(x1);
    if (i == K) {
      st.a[gi][0] = x0;
      st.a[gi][1] = x1;
      fin &= isfinite(x0) && isfinite(x1);
    }
  }
  if (ok && !need && !fin) atomicOr(f.status, kStatusSolve);
  return !need;
}

template <int R, int KCH = (R % 8 == 0 ? 8 : 4), bool BIN = false>
__device__ __forceinline__ bool fast_solve(const FrameDev &f, const FastItem *items, int slot, bool ok,
                                           int t, int gi, int Kw, int w, int h, const float *J,
                                           FastStage &st, const uint16_t *posp, const float *vals) {
  const int K = ok ? items[slot].K : 0;
  FastPts<(R + 15) / 16> P = fast_load<R>(f, K, t, w, h, posp, vals, items[slot].base, items[slot].vb0,
                                          items[slot].vb1, items[slot].nv);
  return fast_solve_pts<R, KCH, BIN>(f, ok, K, t, gi, Kw, w, h, J, st, P);
}

// u = Dh^T (lam .* (Dw[:,X] diag(c) Dh[:,Y]^T)^T) Dw + a for the wave's 4
// blocks (one shape), as interleaved FP32 MFMA 16x16x4 chains: lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; the result D[4(l/16)+r][l%16] is register r.
// Both value planes of a shared chroma mask go through the point chunks
// together (they share every gathered operand but the coefficient).  The
// last product is taken as U^T = S^T Dh, so that lane l holds pixels
// x = 4(l/16) .. 4(l/16)+3 of row y = l%16: one 16-byte store per lane.
template <int R, bool UNR2 = true>
__device__ __forceinline__ void fast_eval(const FrameDev &f, const float *D, const FastStage &st,
                                          int lane, unsigned okmask, int nvw, int w, int h,
                                          int W, long long ob0, long long ob1, int fi) {
  constexpr int nch = R / 4;  // staged rows K..R-1 hold zero coefficients
  const float *Dw = D, *Dh = D + kDct16Floats, *lam = D + 2 * kDct16Floats;
  const int lo = lane & 15, hi = lane >> 4;
  float lam4[4], dwb[4], dha[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int pq = 4 * hi + j;
    lam4[j] = lam[lo * kDct16Ld + pq];  // lam[q][p], q = lo, p = 4 hi + j
    dwb[j] = Dw[pq * kDct16Ld + lo];    // Dw[p][x], p = 4 hi + j, x = lo
    dha[j] = Dh[pq * kDct16Ld + lo];    // Dh[q][y], q = 4 hi + j, y = lo
  }
  f4 acc[2][kWaveItems];
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int g = 0; g < kWaveItems; ++g) acc[v][g] = f4{0.f, 0.f, 0.f, 0.f};
  if (nvw > 1) {
#pragma unroll UNR2 ? 2 : 1
    for (int ch = 0; ch < nch; ++ch) {
      float a0[kWaveItems], a1[kWaveItems], bop[kWaveItems];
#pragma unroll
      for (int g = 0; g < kWaveItems; ++g) {
        const FastPoint P = st.p[g][ch * 4 + hi];
        const float dw = Dw[lo * kDct16Ld + P.x];
        a0[g] = P.c0 * dw;                      // A[p][i], p = lo
        a1[g] = P.c1 * dw;
        bop[g] = Dh[lo * kDct16Ld + P.y];       // B[i][q], q = lo
      }
#pragma unroll
      for (int g = 0; g < kWaveItems; ++g) {
        acc[0][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[g], bop[g], acc[0][g], 0, 0, 0);
        acc[1][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[g], bop[g], acc[1][g], 0, 0, 0);
      }
    }
  } else {
#pragma unroll UNR2 ? 2 : 1
    for (int ch = 0; ch < nch; ++ch) {
      float aop[kWaveItems], bop[kWaveItems];
#pragma unroll
      for (int g = 0; g < kWaveItems; ++g) {
        const FastPoint P = st.p[g][ch * 4 + hi];
        aop[g] = P.c0 * Dw[lo * kDct16Ld + P.x];
        bop[g] = Dh[lo * kDct16Ld + P.y];
      }
#pragma unroll
      for (int g = 0; g < kWaveItems; ++g)
        acc[0][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[g], bop[g], acc[0][g], 0, 0, 0);
    }
  }
  for (int v = 0; v < nvw; ++v) {
    // acc[v][g][j] = V^T[p = 4 hi + j][q = lo]; scale by lam[q][p], then
    // S[q][x] = sum_p U^[q][p] Dw[p][x] and U^T[x][y] = sum_q S[q][x] Dh[q][y].
    f4 Sx[kWaveItems], Ut[kWaveItems];
#pragma unroll
    for (int g = 0; g < kWaveItems; ++g) Sx[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int g = 0; g < kWaveItems; ++g)
        Sx[g] = __builtin_amdgcn_mfma_f32_16x16x4f32((v ? acc[1][g][j] : acc[0][g][j]) * lam4[j], dwb[j], Sx[g],
                                                     0, 0, 0);
#pragma unroll
    for (int g = 0; g < kWaveItems; ++g) Ut[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int g = 0; g < kWaveItems; ++g)
        Ut[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(Sx[g][j], dha[j], Ut[g], 0, 0, 0);
    const int y = lo, x0 = 4 * hi, n = min(4, w - x0);
    // full 16x16 blocks of FP32 planes whose rows start 16-byte aligned take
    // one 16-byte store per lane with the block's base in scalar registers
    // (a uniform test per block instead of per-lane address checks)
    const bool full = w == 16 && h == 16 && !f.out_i8 && (W & 3) == 0;
    const unsigned loff = (unsigned)(y * W + x0);
#pragma unroll
    for (int g = 0; g < kWaveItems; ++g) {
      if (!((okmask >> g) & 1u)) continue;
      const float a = st.a[g][v];
      const long long o = lane_i64(v ? ob1 : ob0, 16 * g);
      const PlaneOut po = plane_out(f, __builtin_amdgcn_readlane(fi, 16 * g));
      const float u[4] = {Ut[g][0] + a, Ut[g][1] + a, Ut[g][2] + a, Ut[g][3] + a};
      float *bp = po.f32 + o;
      if (full && (reinterpret_cast<uintptr_t>(bp) & 15u) == 0)
        __builtin_nontemporal_store(f4{u[0], u[1], u[2], u[3]}, reinterpret_cast<f4 *>(bp + loff));
      else if (y < h && n > 0)
        store_px4(po, (unsigned)(o + loff), u, n);
    }
  }
}

// The FP32 evaluation for blocks of at most 8 x 8 pixels: the wave's 4
// blocks share one 16 x 16 tile, block g in quadrant (g / 2, g % 2) of V
// (its p rows, its q columns), with the DCT matrices block-diagonal and lam
// repeated in every quadrant.  A point product of block g only reaches its
// quadrant and both transforms act quadrant by quadrant, so one tile does
// the work of four (fast_eval spends a zero-padded tile per block).  With
// the last product taken transposed, lane l, register r holds pixel
// (x = 4 (l/16) + r, y = l%16) of the tile: block 2 (x / 8) + y / 8, pixel
// (x % 8, y % 8).
// UNI: the wave's blocks are of one frame (k_fast), so the output planes are
// one scalar pointer.
template <int R, bool UNI = false>
__device__ __forceinline__ void fast_eval8(const FrameDev &f, const float *D, const FastStage &st,
                                           int lane, unsigned okmask, int nvw, int w, int h,
                                           int W, long long ob0, long long ob1, int fi) {
  constexpr int nch = R / 4;  // staged rows K..R-1 hold zero coefficients
  const float *Dw = D, *Dh = D + kDct16Floats, *lam = D + 2 * kDct16Floats;
  const int lo = lane & 15, hi = lane >> 4, l8 = lo & 7, half = lo >> 3;
  float lam4[4], dwb[4], dha[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int pq = 4 * hi + j;
    lam4[j] = lam[l8 * kDct16Ld + (pq & 7)];                            // lam[q % 8][p % 8], q = lo, p = pq
    dwb[j] = (pq >> 3) == half ? Dw[(pq & 7) * kDct16Ld + l8] : 0.f;  // block-diagonal Dw[p][x], x = lo
    dha[j] = (pq >> 3) == half ? Dh[(pq & 7) * kDct16Ld + l8] : 0.f;  // block-diagonal Dh[q][y], y = lo
  }
  for (int v = 0; v < nvw; ++v) {
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int ch = 0; ch < nch; ++ch) {
#pragma unroll
      for (int g = 0; g < kWaveItems; ++g) {
        const FastPoint P = st.p[g][ch * 4 + hi];
        const float aop = half == (g >> 1) ? (v ? P.c1 : P.c0) * Dw[l8 * kDct16Ld + P.x] : 0.f;  // A[p][i]
        const float bop = half == (g & 1) ? Dh[l8 * kDct16Ld + P.y] : 0.f;                      // B[i][q]
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bop, acc, 0, 0, 0);
      }
    }
    // the last product taken transposed (U^T = S^T Dh): lane l, register r
    // holds pixel (x = 4 (l/16) + r, y = l%16) of the tile, so each lane
    // writes four consecutive pixels of one block row with one store
    f4 Sx = f4{0.f, 0.f, 0.f, 0.f}, Ut = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; ++j) Sx = __builtin_amdgcn_mfma_f32_16x16x4f32(acc[j] * lam4[j], dwb[j], Sx, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) Ut = __builtin_amdgcn_mfma_f32_16x16x4f32(Sx[j], dha[j], Ut, 0, 0, 0);
    long long ob[kWaveItems];
    int fb[kWaveItems];
#pragma unroll
    for (int g = 0; g < kWaveItems; ++g) {
      ob[g] = lane_i64(v ? ob1 : ob0, 16 * g);
      fb[g] = __builtin_amdgcn_readlane(fi, 16 * g);
    }
    const int bt = 2 * (hi >> 1) + half;  // block of this lane's pixels (x / 8 = hi / 2, y / 8 = half)
    const long long o = bt == 0 ? ob[0] : bt == 1 ? ob[1] : bt == 2 ? ob[2] : ob[3];
    const PlaneOut po = plane_out(f, UNI ? fb[0] : bt == 0 ? fb[0] : bt == 1 ? fb[1] : bt == 2 ? fb[2] : fb[3]);
    if ((okmask >> bt) & 1u) {
      const float a = st.a[bt][v];
      const int y = l8, x0 = 4 * (hi & 1), n = min(4, w - x0);
      const float u[4] = {Ut[0] + a, Ut[1] + a, Ut[2] + a, Ut[3] + a};
      if (y < h && n > 0) store_px4(po, (unsigned)(o + (long long)y * W + x0), u, n);
    }
  }
}

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef __bf16 b4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

// MFMA operands of N values in the evaluation dtype EV: FP16 (1), BF16 (2),
// or split BF16 (3: x = hi + lo with hi = bf16(x), lo = bf16(x - hi)).
template <int EV, int N> struct RedOp {
  typedef _Float16 H __attribute__((ext_vector_type(N)));
  typedef __bf16 B __attribute__((ext_vector_type(N)));
  typedef typename std::conditional<EV == 1, H, B>::type T;
  T hi, lo;
};

template <int EV, int N>
__device__ __forceinline__ RedOp<EV, N> red_op(const float *x) {
  RedOp<EV, N> r;
  if constexpr (EV == 1) {
#pragma unroll
    for (int e = 0; e < N; ++e) r.hi[e] = (_Float16)x[e];
  } else if constexpr (EV == 2) {
#pragma unroll
    for (int e = 0; e < N; ++e) r.hi[e] = (__bf16)x[e];
  } else {
    // hi rounded to nearest, then the residual rounded again
#pragma unroll
    for (int e = 0; e < N; ++e) {
      r.hi[e] = (__bf16)x[e];
      r.lo[e] = (__bf16)(x[e] - (float)r.hi[e]);
    }
  }
  return r;
}

// acc += A B on a 16x16x16 MFMA (lane l: A[l%16][4(l/16)+e], B[4(l/16)+e][l%16])
// or a 16x16x32 one (8 values per lane, k = 8(l/16)+e); split BF16 adds the
// hi*lo and lo*hi products (lo*lo is below FP32 rounding of the sum).
template <int EV>
__device__ __forceinline__ f4 mma16(f4 acc, const RedOp<EV, 4> &a, const RedOp<EV, 4> &b) {
  if constexpr (EV == 1) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a.hi, b.hi, acc, 0, 0, 0);
  } else {
    if constexpr (EV == 3) {
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, b.hi, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.lo, acc, 0, 0, 0);
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, acc, 0, 0, 0);
  }
}
template <int EV>
__device__ __forceinline__ f4 mma32(f4 acc, const RedOp<EV, 8> &a, const RedOp<EV, 8> &b) {
  if constexpr (EV == 1) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.hi, acc, 0, 0, 0);
  } else {
    if constexpr (EV == 3) {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, acc, 0, 0, 0);
    }
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, acc, 0, 0, 0);
  }
}

// The evaluation of fast_eval with FP16 / BF16 / split-BF16 operands and
// FP32 accumulation, on gfx950's matrix forms: the points of a block (at
// most 32) in one 16x16x32 product (lane l supplies points 8(l/16) ..
// 8(l/16)+7; both chroma planes share the Dh operand), the two transforms as
// 16x16x16 products with the constant matrices converted once per wave, the
// last one transposed as in fast_eval (16-byte stores).
template <int R, int EV>
__device__ __forceinline__ void fast_eval16(const FrameDev &f, const float *D, const FastStage &st,
                                            int lane, unsigned okmask, int nvw, int w, int h,
                                            int W, long long ob0, long long ob1, int fi) {
  const float *Dw = D, *Dh = D + kDct16Floats, *lam = D + 2 * kDct16Floats;
  const int lo = lane & 15, hi = lane >> 4;
  float lam4[4], dwb[4], dha[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int pq = 4 * hi + j;
    lam4[j] = lam[lo * kDct16Ld + pq];
    dwb[j] = Dw[pq * kDct16Ld + lo];
    dha[j] = Dh[pq * kDct16Ld + lo];
  }
  const RedOp<EV, 4> dwo = red_op<EV, 4>(dwb), dho = red_op<EV, 4>(dha);
  const int y = lo, x0 = 4 * hi, n = min(4, w - x0);
#pragma unroll 1
  for (int g = 0; g < kWaveItems; ++g) {
    if (!((okmask >> g) & 1u)) continue;
    // V^T of both planes: points 8 hi .. 8 hi + 7 (staged rows past K hold
    // zero coefficients; rows past R are not staged: zeros here)
    float a0[8], a1[8], b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a0[e] = a1[e] = b[e] = 0.f;
      const int k = 8 * hi + e;
      if (k < R) {
        const FastPoint P = st.p[g][k];
        const float dw = Dw[lo * kDct16Ld + P.x];
        a0[e] = P.c0 * dw;
        a1[e] = P.c1 * dw;
        b[e] = Dh[lo * kDct16Ld + P.y];
      }
    }
    const RedOp<EV, 8> bo = red_op<EV, 8>(b);
    f4 acc[2];
    acc[0] = mma32<EV>(f4{0.f, 0.f, 0.f, 0.f}, red_op<EV, 8>(a0), bo);
    if (nvw > 1) acc[1] = mma32<EV>(f4{0.f, 0.f, 0.f, 0.f}, red_op<EV, 8>(a1), bo);
    for (int v = 0; v < nvw; ++v) {
      float u[4], sx[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) u[e] = (v ? acc[1][e] : acc[0][e]) * lam4[e];  // U^[q = lo][p = 4 hi + e]
      const f4 S = mma16<EV>(f4{0.f, 0.f, 0.f, 0.f}, red_op<EV, 4>(u), dwo);    // S[q = 4 hi + r][x = lo]
#pragma unroll
      for (int e = 0; e < 4; ++e) sx[e] = S[e];
      const f4 Ut = mma16<EV>(f4{0.f, 0.f, 0.f, 0.f}, red_op<EV, 4>(sx), dho);  // U[y = lo][x = 4 hi + r]
      const float av = st.a[g][v];
      const long long o = lane_i64(v ? ob1 : ob0, 16 * g);
      const PlaneOut po = plane_out(f, __builtin_amdgcn_readlane(fi, 16 * g));
      const float uu[4] = {Ut[0] + av, Ut[1] + av, Ut[2] + av, Ut[3] + av};
      if (y < h && n > 0) store_px4(po, (unsigned)(o + (long long)y * W + x0), uu, n);
    }
  }
}

// The evaluation in the launch's dtype EV (a template parameter of k_fast:
// each kernel holds one evaluation, which keeps its code small).
// B8: 8 x 8 blocks (the FP32 evaluation packs four per tile); a template
// parameter of the kernels, so that a kernel holds one FP32 evaluation and
// the register file it needs (the 16 x 16 one needs more).
template <int R, int EV, bool UNR2 = true, bool UNI = false, int B8 = 0>
__device__ __forceinline__ void fast_eval_any(const FrameDev &f, const float *D, const FastStage &st,
                                              int lane, unsigned okmask, int nvw, int w, int h, int W,
                                              long long ob0, long long ob1, int fi) {
  if constexpr (EV != 0) {
    fast_eval16<R, EV>(f, D, st, lane, okmask, nvw, w, h, W, ob0, ob1, fi);
  } else if constexpr (B8 != 0) {
    fast_eval8<R, UNI>(f, D, st, lane, okmask, nvw, w, h, W, ob0, ob1, fi);
  } else {
    fast_eval<R, UNR2>(f, D, st, lane, okmask, nvw, w, h, W, ob0, ob1, fi);
  }
}

// Coefficient encodes: the quantised c and the a of the wave's solved blocks
// (each lane stores the rows it solved).
template <int R>
__device__ __forceinline__ void fast_encode_store(const FrameDev &f, const FastItem *items, int slot, bool done,
                                                  int t, int gi, const GroupDev &G, const FastStage &st) {
  constexpr int NS = (R + 15) / 16;
  if (!done) return;
  const FramePtrs fp = f.fp[blockIdx.y];
  const int K = items[slot].K, nv = items[slot].nv;
  const float s0 = f.qstep[G.vplane[0]], s1 = f.qstep[G.vplane[nv > 1 ? 1 : 0]];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = t + 16 * s;
    if (i < K) {
      const FastPoint P = st.p[gi][i];
      fp.qout[items[slot].vb0 + i] = (int8_t)quant_code(P.c0, s0);
      if (nv > 1) fp.qout[items[slot].vb1 + i] = (int8_t)quant_code(P.c1, s1);
    }
  }
  if (t < nv) fp.aout[G.cbase[t] + (items[slot].m - G.first)] = st.a[gi][t];
}

// MODE 0: residual decode (solve, evaluate); 1: stored coefficients
// (evaluate only); 2: coefficient encode (solve, quantise, no evaluation).
// EV: evaluation dtype (PDI_EVAL_*; encodes take 0).
template <int MODE, int EV, int B8 = 0>
__global__ __launch_bounds__(kFastThreads) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_fast(FrameDev f) {
  constexpr bool COEF = MODE == 1, ENC = MODE == 2;
  extern __shared__ __attribute__((aligned(16))) float tabs[];  // J, Dw, Dh, lam of the workgroup's shape
  __shared__ FastItem items[kFastItems];
  __shared__ int order[kFastItems];
  __shared__ int defer[kFastItems];
  __shared__ FastStage stage[kFastWaves];
  __shared__ GenScratch<16> gs;
  const int tid = threadIdx.x;
  const int wg = blockIdx.x;
  int si = 0;
  while (si + 1 < f.nsegs && wg >= f.seg[si + 1].first_wg) ++si;
  const SegDev sg = f.seg[si];
  const ShapeDev S = f.s[sg.shape];
  const GroupDev &G = f.g[sg.group];
  const int w = S.w, h = S.h;

  // Prologue: the workgroup's blocks (geometry from the segment, counts from
  // block_ptr: these loads are issued first) and the shape's tables into LDS
  // (16-byte loads, all in flight before the first store).
  const int kk = (wg - sg.first_wg) * f.ipw + tid;
  const bool has = tid < f.ipw && kk < sg.count;
  int im = 0, ilo = 0, ihi = 0, ibx = 0, iby = 0;
  long long icr = 0;
  if (has) {
    ibx = sg.bx0 + kk % sg.nx;
    iby = sg.by0 + kk / sg.nx;
    im = G.first + iby * G.nbx + ibx;
    const int32_t *bp = f.fp[blockIdx.y].block_ptr;
    ilo = bp[im];
    ihi = bp[im + 1];
    if (G.nv > 1 && f.shared) icr = (long long)bp[f.n_items] - bp[f.chroma_first];
  }
  if constexpr (COEF) {  // the evaluation's matrices only
    const int n4 = (3 * kDct16Floats) >> 2;
    const f4 *src = reinterpret_cast<const f4 *>(f.tab32 + S.fast + S.jt_floats);
    f4 *dst = reinterpret_cast<f4 *>(tabs);
    for (int i = tid; i < n4; i += kFastThreads) dst[i] = src[i];
  } else {  // J and the evaluation's matrices (encodes: J only)
    const int n4 = (S.jt_floats + (ENC ? 0 : 3 * kDct16Floats)) >> 2;
    const f4 *src = reinterpret_cast<const f4 *>(f.tab32 + S.fast);
    f4 *dst = reinterpret_cast<f4 *>(tabs);
    f4 buf[kTabVec];
#pragma unroll
    for (int r = 0; r < kTabVec; ++r) buf[r] = src[tid + r * kFastThreads];  // buffer is padded
#pragma unroll
    for (int r = 0; r < kTabVec; ++r) asm volatile("" : "+v"(buf[r]));  // all loads before any store
#pragma unroll
    for (int r = 0; r < kTabVec; ++r) {
      const int i = tid + r * kFastThreads;
      if (i < n4) dst[i] = buf[r];
    }
  }
  if (tid < kFastItems) {
    FastItem r;
    r.cls = kClassNone;
    r.m = r.K = r.base = r.nv = 0;
    r.fi = blockIdx.y;
    r.vb0 = r.vb1 = r.ob0 = r.ob1 = 0;
    if (has) {
      r.m = im;
      r.K = ihi - ilo;
      r.base = ilo;
      r.nv = G.nv;
      r.cls = fast_class<COEF, ENC>(r.K, w * h);
      const long long pix = (long long)(iby * f.b) * G.W + ibx * f.b;
      r.vb0 = ilo;
      r.ob0 = G.out_off[0] + pix;
      if (G.nv > 1) {
        // a shared chroma mask: the Cr run follows every other value
        r.vb1 = f.shared ? icr + ilo : ilo;
        r.ob1 = G.out_off[1] + pix;
      }
    }
    items[tid] = r;
    // Blocks the waves do not take: decoded by this workgroup at its end
    // (single-frame launches) or handed to the deferred pass (batches).
    defer[tid] = (r.cls == kClassDefer && f.tail_in_wg) ? 1 : 0;
    if (r.cls == kClassDefer && !f.tail_in_wg) push_deferred(f, blockIdx.y, r.m, r.K, w, h);
  }
  __syncthreads();
  // Bin by size class so that every wave solves blocks of one class.
  if (tid < kFastItems) {
    const int c = items[tid].cls;
    int r = 0;
    for (int j = 0; j < kFastItems; ++j) {
      const int cj = items[j].cls;
      r += (cj < c) || (cj == c && j < tid);
    }
    order[r] = tid;
  }
  __syncthreads();

  const int lane = tid & 63, wv = tid >> 6;
  const int gi = lane >> 4, t = lane & 15;
  const int slot = order[wv * kWaveItems + gi];
  const bool ok = items[slot].cls < kClassDefer;
  int kw = ok ? items[slot].K : 0, nvw = ok ? items[slot].nv : 0;
  for (int o = 32; o > 0; o >>= 1) {
    kw = max(kw, __shfl_xor(kw, o));
    nvw = max(nvw, __shfl_xor(nvw, o));
  }
  const int Kw = __builtin_amdgcn_readfirstlane(kw);
  const int NVw = __builtin_amdgcn_readfirstlane(nvw);
  if (COEF || Kw > 0) {
    FastStage &st = stage[wv];
    bool solved = true;
    if constexpr (COEF) {
      if (Kw <= 15) fast_coef_stage<16>(f, items, slot, ok, t, gi, w, h, G, st);
      else if (Kw <= 23) fast_coef_stage<24>(f, items, slot, ok, t, gi, w, h, G, st);
      else fast_coef_stage<32>(f, items, slot, ok, t, gi, w, h, G, st);
    } else {
      const uint16_t *posp = f.fp[blockIdx.y].pos;
      const float *vals = f.fp[blockIdx.y].values;
      if (ENC && Kw <= 7) solved = fast_solve<8>(f, items, slot, ok, t, gi, Kw, w, h, tabs, st, posp, vals);
      else if (Kw <= 15) solved = fast_solve<16>(f, items, slot, ok, t, gi, Kw, w, h, tabs, st, posp, vals);
      else if (Kw <= 23) solved = fast_solve<24>(f, items, slot, ok, t, gi, Kw, w, h, tabs, st, posp, vals);
      else solved = fast_solve<32>(f, items, slot, ok, t, gi, Kw, w, h, tabs, st, posp, vals);
    }
    if (ok && !solved && t == 0) {
      if (f.tail_in_wg) defer[slot] = 1;
      else push_deferred(f, blockIdx.y, items[slot].m, items[slot].K, w, h);
    }
    const bool eval = ok && solved;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const unsigned long long em = __ballot(eval);
    unsigned okmask = 0;
#pragma unroll
    for (int g = 0; g < kWaveItems; ++g) okmask |= ((em >> (16 * g)) & 1ull) ? (1u << g) : 0u;
    const long long ob0 = items[slot].ob0, ob1 = items[slot].ob1;
    if constexpr (ENC) {
      if (Kw <= 7) fast_encode_store<8>(f, items, slot, eval, t, gi, G, st);
      else if (Kw <= 15) fast_encode_store<16>(f, items, slot, eval, t, gi, G, st);
      else if (Kw <= 23) fast_encode_store<24>(f, items, slot, eval, t, gi, G, st);
      else fast_encode_store<32>(f, items, slot, eval, t, gi, G, st);
    } else if (okmask) {
      const float *D = tabs + (COEF ? 0 : S.jt_floats);
      const int fi = blockIdx.y;
      if (Kw <= 15) fast_eval_any<16, EV, true, true, B8>(f, D, st, lane, okmask, NVw, w, h, G.W, ob0, ob1, fi);
      else if (Kw <= 23) fast_eval_any<24, EV, true, true, B8>(f, D, st, lane, okmask, NVw, w, h, G.W, ob0, ob1, fi);
      else fast_eval_any<32, EV, true, true, B8>(f, D, st, lane, okmask, NVw, w, h, G.W, ob0, ob1, fi);
    }
  }

  // Blocks the waves did not take (K = 0, K = w*h, K > 31, invalid counts)
  // or whose pivots asked for FP64 refinement: the whole workgroup runs the
  // general algorithm on them, one at a time, with the bordered system in
  // this workgroup's global slot.
  if constexpr (MODE == 0) {
    if (!f.tail_in_wg) return;
    __syncthreads();
    float *slot_mem = f.slots + (long long)blockIdx.x * f.slot_floats;
    for (int j = 0; j < kFastItems; ++j) {
      if (defer[j]) {
        __syncthreads();
        general_block<16>(f, 0, items[j].m, gs, slot_mem);
      }
    }
  }
}

// ------------------------------------------- binned wave-level path (b <= 16)

// Bordered-system size class of a block for k_fast2: R = 4 (c + 1) rows,
// the smallest multiple of 4 that holds the K + 1 rows (K = 1 .. 31).
__device__ __forceinline__ int fast2_class(int K) { return ((K + 4) >> 2) - 1; }

// Binning for k_fast2: every mask block of every frame of the launch whose
// system the wave-level path solves goes to the queue of its mask-plane
// group and edge kind (so a queue holds blocks of one shape, one plane width
// and one value-plane count), into the bin of its size class; the others
// (K = 0, K = w*h, K > 31, invalid counts) go to the general path's lists.
// Three passes without global atomics (counting, a scan per bin, placing):
// thousands of workgroups adding to a few dozen counters serialise.  The
// placing pass writes every block's entry straight into its k_fast2
// workgroup's slice of f.fl: bins in hand-out order (classes from the
// largest systems down, queues in order), each padded to whole workgroups of
// kF2Items entries, the order inside a bin that of the blocks (frame, then
// block index).  An entry carries everything a workgroup needs to start
// loading the block's points (frame, block, first point, K, first Cr value),
// and the first entry of each workgroup's slice writes the workgroup's
// descriptor (bin, valid entries), so k_fast2 reads its blocks with one load
// and no search.
constexpr int kBinThreads = 256;
constexpr int kMaxBins = 8 * kMaxSegs;
constexpr int kF2Threads = 256;                  // k_fast2: 4 waves per workgroup
constexpr int kScanRun = 8;                      // k_fbin_scan: counts per thread in one round
constexpr int kF2Waves = kF2Threads / 64;
constexpr int kF2Items = kF2Waves * kWaveItems;  // 16 blocks per workgroup

// The bin of mask block m of frame fi (-1: not queued), with its first
// point, point count and value-plane count.
__device__ __forceinline__ int fbin_key(const FrameDev &f, int fi, int m, bool defer, int &lo, int &K, int &nv) {
  lo = K = 0;
  nv = 1;
  if (m >= f.n_items) return -1;
  const int32_t *bp = f.fp[fi].block_ptr;
  int g = 0;
  if (f.ngroups > 1 && m >= f.g[1].first) g = 1;
  if (f.ngroups > 2 && m >= f.g[2].first) g = 2;
  const GroupDev &G = f.g[g];
  const int l = m - G.first, bx = l % G.nbx, by = l / G.nbx;
  const int e = ((bx == G.nbx - 1) && (G.W % f.b) ? 1 : 0) + ((by == G.nby - 1) && (G.H % f.b) ? 2 : 0);
  const int shape = G.shape[e];
  const int w = f.s[shape].w, h = f.s[shape].h;
  lo = bp[m];
  K = bp[m + 1] - lo;
  nv = G.nv;
  if (K < 1 || K >= w * h || K > kFastKMax) {
    if (defer) push_deferred(f, fi, m, K, w, h);
    return -1;
  }
  return 8 * f.qge[g][e] + fast2_class(K);
}

// Per wave: how many of its lanes fall in each bin (wc[wave][bin]) and each
// lane's rank among them (lanes in order).
__device__ __forceinline__ int fbin_wave_rank(int key, int (*wc)[kMaxBins]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int rank = 0;
  unsigned long long todo = __ballot(key >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int k = __shfl(key, leader);
    const unsigned long long mine = __ballot(key == k);
    todo &= ~mine;
    if (key == k) rank = __popcll(mine & ((1ull << lane) - 1ull));
    if (lane == leader) wc[wv][k] = __popcll(mine);
  }
  return rank;
}

// Pass 1: the count of every bin in each workgroup's 256 blocks (one frame);
// also marks every k_fast2 workgroup empty (pass 3 describes the used ones).
__global__ __launch_bounds__(kBinThreads) void k_fbin_count(FrameDev f) {
  __shared__ int wc[kBinThreads / 64][kMaxBins];
  const int nb = 8 * f.nq, tid = threadIdx.x;
  const int wgi = blockIdx.y * gridDim.x + blockIdx.x;
  for (int i = wgi * kBinThreads + tid; i < f.fast_wgs; i += gridDim.x * gridDim.y * kBinThreads) {
    f.wgdesc[2 * i] = -1;
    f.wgdesc[2 * i + 1] = 0;
  }
  for (int i = tid; i < (kBinThreads / 64) * kMaxBins; i += kBinThreads) (&wc[0][0])[i] = 0;
  __syncthreads();
  int lo, K, nv;
  const int key = fbin_key(f, blockIdx.y, blockIdx.x * kBinThreads + tid, true, lo, K, nv);
  fbin_wave_rank(key, wc);
  __syncthreads();
  if (tid < nb) {
    int t = 0;
#pragma unroll
    for (int w = 0; w < kBinThreads / 64; ++w) t += wc[w][tid];
    f.hist[(long long)wgi * nb + tid] = t;
  }
}

// Pass 2: one workgroup per bin: exclusive scan of its counts over the
// workgroups of pass 1 (in place) and the bin's total into its counter.
__global__ __launch_bounds__(kBinThreads) void k_fbin_scan(FrameDev f, int nwg) {
  __shared__ int wsum[kBinThreads / 64];
  const int nb = 8 * f.nq, bin = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // Exclusive scan of one value x per thread over the workgroup's 256
  // threads, starting at carry: returns this thread's offset; tot receives
  // carry plus the sum of every thread's x.
  auto block_scan = [&](int x, int carry, int &tot) {
    const int v = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int off = carry;
    tot = carry;
#pragma unroll
    for (int k = 0; k < kBinThreads / 64; ++k) {
      off += k < wv ? wsum[k] : 0;
      tot += wsum[k];
    }
    __syncthreads();
    return off + x - v;
  };
  int carry = 0;
  if (nwg <= kScanRun * kBinThreads) {
    // one round: each thread takes a run of up to kScanRun consecutive
    // counts, all loaded at once (the counts of a bin are nb ints apart)
    const int run = (nwg + kBinThreads - 1) / kBinThreads, w0 = tid * run;
    int v[kScanRun], sum = 0;
#pragma unroll
    for (int i = 0; i < kScanRun; ++i) {
      v[i] = (i < run && w0 + i < nwg) ? f.hist[(long long)(w0 + i) * nb + bin] : 0;
      sum += v[i];
    }
    int off = block_scan(sum, 0, carry);
#pragma unroll
    for (int i = 0; i < kScanRun; ++i) {
      if (i < run && w0 + i < nwg) f.hist[(long long)(w0 + i) * nb + bin] = off;
      off += v[i];
    }
  } else {  // more counting workgroups: round by round, 256 counts each
    for (int w0 = 0; w0 < nwg; w0 += kBinThreads) {
      const int w = w0 + tid;
      const int v = w < nwg ? f.hist[(long long)w * nb + bin] : 0;
      const int off = block_scan(v, carry, carry);
      if (w < nwg) f.hist[(long long)w * nb + bin] = off;
    }
  }
  if (tid == 0) f.counters[kQueueCounters + bin] = carry;
}

// Pass 3: every queued block's entry to its place in f.fl.
__global__ __launch_bounds__(kBinThreads) void k_fbin_place(FrameDev f) {
  __shared__ int wc[kBinThreads / 64][kMaxBins];
  __shared__ int bstart[kMaxBins], bcount[kMaxBins];
  const int nb = 8 * f.nq, tid = threadIdx.x, wv = tid >> 6;
  for (int i = tid; i < (kBinThreads / 64) * kMaxBins; i += kBinThreads) (&wc[0][0])[i] = 0;
  if (tid < 64) {
    // first entry of every bin: bins in hand-out order (class 7 .. 0, queues
    // in order), each a whole number of workgroup slices
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 64) {
      const int b = b0 + tid;
      int key = 0, cnt = 0;
      if (b < nb) {
        key = 8 * (b % f.nq) + 7 - b / f.nq;
        cnt = f.counters[kQueueCounters + key];
      }
      const int len = (cnt + kF2Items - 1) / kF2Items * kF2Items;
      int incl = len;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int x = __shfl_up(incl, o, 64);
        if (tid >= o) incl += x;
      }
      incl += carry;
      if (b < nb) {
        bstart[key] = incl - len;
        bcount[key] = cnt;
      }
      carry = __shfl(incl, 63, 64);
    }
  }
  __syncthreads();
  const int fi = blockIdx.y, m = blockIdx.x * kBinThreads + tid;
  int lo, K, nv;
  const int key = fbin_key(f, fi, m, false, lo, K, nv);
  const int rank = fbin_wave_rank(key, wc);
  __syncthreads();
  if (key >= 0) {
    int idx = f.hist[(long long)(blockIdx.y * gridDim.x + blockIdx.x) * nb + key] + rank;
    for (int w = 0; w < wv; ++w) idx += wc[w][key];
    const long long j = (long long)bstart[key] + idx;
    if (idx < bcount[key] && j < (long long)kF2Items * f.fast_wgs) {
      // a shared chroma mask: the Cr run follows every other value (-1:
      // one value plane)
      const int32_t *bp = f.fp[fi].block_ptr;
      const int vb1 = nv < 2 ? -1 : f.shared ? bp[f.n_items] - bp[f.chroma_first] + lo : lo;
      i4 ent;
      ent.x = (fi << kDeferFrameShift) | m;
      ent.y = lo;
      ent.z = K;
      ent.w = vb1;
      reinterpret_cast<i4 *>(f.fl)[j] = ent;
      if (idx % kF2Items == 0) {
        const ShapeDev &S = f.s[f.q[key >> 3].shape];
        i2 d;
        d.x = key | (min(kF2Items, bcount[key] - idx) << 8) | (((S.jt_floats + 3 * kDct16Floats) >> 2) << 16);
        d.y = S.fast;
        reinterpret_cast<i2 *>(f.wgdesc)[j / kF2Items] = d;
      }
    }
  }
}

// The wave-level solve and evaluation of one workgroup's blocks, all of one
// size class R (R rows per block system, four blocks per wave): d is the
// workgroup's descriptor, ent this row's entry.
constexpr int kTabVec2 = ((16 * jrow(16, 16) + 3) / 4 + 3 * kDct16Floats / 4 + kF2Threads - 1) / kF2Threads;
static_assert(kTabVec2 * kF2Threads * 4 <= kTabPadFloats, "table reads stay inside the padded buffer");
static_assert(kTabVec2 * kF2Threads < (1 << 15), "the table's 16-byte count fits a descriptor");

// The launch's FrameDev read in place in the kernel-argument segment (the
// kernels that use it take it as their only argument, at offset 0): data-
// dependent indexes into a by-value kernel argument can make the compiler
// copy all of it to private memory first.
__device__ __forceinline__ const __attribute__((address_space(4))) FrameDev *kernarg_frame() {
  return (const __attribute__((address_space(4))) FrameDev *)__builtin_amdgcn_kernarg_segment_ptr();
}

template <int R, int EV, int B8>
__device__ __forceinline__ void fast2_run(const FrameDev &f, int d, int tabo, const i4 ent, float *tabs,
                                          FastStage *stage) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int gi = lane >> 4, t = lane & 15;
  const int slot = wv * kWaveItems + gi;
  const int qi = (d & 0xff) >> 3, nval = (d >> 8) & 0xff, n4 = d >> 16;
  // the tables' loads: J and the evaluation's matrices (16-byte loads; the
  // buffer is padded)
  const f4 *src = reinterpret_cast<const f4 *>(f.tab32 + tabo);
  f4 buf[kTabVec2];
#pragma unroll
  for (int r = 0; r < kTabVec2; ++r) buf[r] = src[tid + r * kF2Threads];
  // this row's block: its point loads go out before the tables are stored,
  // so that the two latencies overlap
  const bool ok = slot < nval;
  const int K = ok ? ent.z : 0;
  // the frame's point runs: its index is uniform in each 16-lane row, so
  // the pointers come from the kernel arguments by scalar loads (a hit in
  // the scalar cache, not a vector round trip)
  const uint16_t *ppos;
  const float *pval;
  {
    const uint16_t *pr[kWaveItems];
    const float *vr[kWaveItems];
#pragma unroll
    for (int g = 0; g < kWaveItems; ++g) {
      const int fr = (__builtin_amdgcn_readfirstlane(wv) * kWaveItems + g < nval)
                         ? __builtin_amdgcn_readlane(ent.x, 16 * g) >> kDeferFrameShift : 0;
      pr[g] = f.fp[fr].pos;
      vr[g] = f.fp[fr].values;
    }
    ppos = gi == 0 ? pr[0] : gi == 1 ? pr[1] : gi == 2 ? pr[2] : pr[3];
    pval = gi == 0 ? vr[0] : gi == 1 ? vr[1] : gi == 2 ? vr[2] : vr[3];
  }
  const QueueDev Q = f.q[qi];
  const ShapeDev S = f.s[Q.shape];
  const int w = S.w, h = S.h;
  FastPts<(R + 15) / 16> P =
      fast_load<R>(f, K, t, w, h, ppos, pval, ent.y, ent.y, ent.w, ent.w < 0 ? 1 : 2);
  {  // the tables into LDS (all loads in flight before the first store)
    f4 *dst = reinterpret_cast<f4 *>(tabs);
#pragma unroll
    for (int r = 0; r < kTabVec2; ++r) asm volatile("" : "+v"(buf[r]));
#pragma unroll
    for (int r = 0; r < kTabVec2; ++r) {
      const int i = tid + r * kF2Threads;
      if (i < n4) dst[i] = buf[r];
    }
  }
  // (uniform in each 16-lane row: the wave's largest from one lane per row)
  const int Kw = max(max(__builtin_amdgcn_readlane(K, 0), __builtin_amdgcn_readlane(K, 16)),
                     max(__builtin_amdgcn_readlane(K, 32), __builtin_amdgcn_readlane(K, 48)));
  __syncthreads();
  if (Kw == 0) return;  // no block in this wave
  const GroupDev G = f.g[Q.first_wg];  // the queue's group (binned queues keep it in first_wg)
  const int nv = G.nv;
  FastStage &st = stage[wv];
  if (t == 0) st.e[gi] = ok ? ent.x : 0;  // (read back after the solve: two registers fewer)
  // (for two-slice systems the lookups go in chunks of 4 columns and the
  // evaluation's point chunks one at a time: the register file then holds
  // four waves per SIMD for every class)
  const bool solved = fast_solve_pts<R, R <= 16 ? (R % 8 == 0 ? 8 : 4) : 4, true>(f, ok, K, t, gi, Kw, w, h, tabs,
                                                                                   st, P);
  const int e = st.e[gi], fi = e >> kDeferFrameShift, m = e & kDeferItemMask;
  if (ok && !solved && t == 0) push_deferred(f, fi, m, K, w, h);
  const bool eval = ok && solved;
  wave_sync();
  const unsigned long long em = __ballot(eval);
  unsigned okmask = 0;
#pragma unroll
  for (int g = 0; g < kWaveItems; ++g) okmask |= ((em >> (16 * g)) & 1ull) ? (1u << g) : 0u;
  if (okmask) {  // (every block of the queue has its group's value-plane count)
    const int l = m - G.first, bx = l % G.nbx, by = l / G.nbx;
    const long long pix = (long long)(by * f.b) * G.W + bx * f.b;
    const long long ob0 = ok ? G.out_off[0] + pix : 0, ob1 = (ok && nv > 1) ? G.out_off[1] + pix : 0;
    // (FP32: the lane index recomputed, nothing to keep in a register over the solve)
    const int ln = EV == 0 ? (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)) : lane;
    fast_eval_any<R, EV, false, false, B8>(f, tabs + S.jt_floats, st, ln, okmask, nv, w, h, G.W, ob0, ob1, fi);
  }
}

// Residual decodes with b <= 16, binned (k_fbin_* first): each workgroup takes
// up to 16 blocks of one bin - one block shape and one size class - so
// every wave solves four systems of nearly the same size with code sized for
// them, and workgroups of one class run one after another (bins are handed
// out class by class, the largest systems first).  The block arithmetic is
// that of k_fast (same solve and evaluation, padding rows and columns are
// exact identities and zeros), so results do not depend on the path.
template <int EV, int B8 = 0>
__global__ __launch_bounds__(kF2Threads) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_fast2(FrameDev arg) {
  extern __shared__ __attribute__((aligned(16))) float tabs[];  // J, Dw, Dh, lam of the bin's shape
  __shared__ FastStage stage[kF2Waves];
  (void)arg;
  const FrameDev &f = *(const FrameDev *)kernarg_frame();  // (read in place: see kernarg_frame)
  const int wg = blockIdx.x, slot = (threadIdx.x >> 6) * kWaveItems + ((threadIdx.x & 63) >> 4);
  // the descriptor and the entries in one round trip (the 16 lanes of a row
  // read the same entry).  A workgroup no bin reaches (descriptor -1) runs
  // the smallest class with no valid entry: its waves leave after the
  // barrier (no branch ahead of the entry load, which then issues at once).
  const i2 dv = reinterpret_cast<const i2 *>(f.wgdesc)[wg];
  const i4 ent = reinterpret_cast<const i4 *>(f.fl)[(long long)wg * kF2Items + slot];
  const int d0 = __builtin_amdgcn_readfirstlane(dv.x), tabo = __builtin_amdgcn_readfirstlane(dv.y);
  const int d = d0 < 0 ? 0 : d0;
  switch (d & 7) {
    case 0: fast2_run<4, EV, B8>(f, d, tabo, ent, tabs, stage); break;
    case 1: fast2_run<8, EV, B8>(f, d, tabo, ent, tabs, stage); break;
    case 2: fast2_run<12, EV, B8>(f, d, tabo, ent, tabs, stage); break;
    case 3: fast2_run<16, EV, B8>(f, d, tabo, ent, tabs, stage); break;
    case 4: fast2_run<20, EV, B8>(f, d, tabo, ent, tabs, stage); break;
    case 5: fast2_run<24, EV, B8>(f, d, tabo, ent, tabs, stage); break;
    case 6: fast2_run<28, EV, B8>(f, d, tabo, ent, tabs, stage); break;
    default: fast2_run<32, EV, B8>(f, d, tabo, ent, tabs, stage); break;
  }
}

// ------------------------------------------- stored coefficients, general

// One stored-coefficient block with a whole workgroup: u = sum_i c_i
// G(., x_i) + a at every pixel (Eq. 2 summed directly, FP32), the points
// staged in LDS 256 at a time, G from the compact table in LDS.  For the
// blocks the batched kernels leave (more points than they stage).
__device__ void coef_block(const FrameDev &f, int fi, int m, FastPoint *pts, float *tab) {
  const int tid = threadIdx.x;
  fi = __builtin_amdgcn_readfirstlane(fi);
  const FramePtrs fp = f.fp[fi];
  const Item it = load_item(f, fp.block_ptr, m);
  const GroupDev &G = f.g[it.g];
  const int K = it.K, w = it.w, h = it.h, N = w * h;
  const ShapeDev S = f.s[it.shape];
  const PlaneOut po = plane_out(f, fi);
  __syncthreads();  // the previous block's readers are done
  for (int i = tid; i < (w + 1) * (h + 1); i += kGenThreads) tab[i] = f.tab32[S.hc32 + i];
  int bad = (K < 0 || K > N) ? kStatusMask : 0;
  const int Kc = (K < 0 || K > N) ? 0 : K;
  const int pl0 = G.vplane[0], pl1 = G.vplane[it.nv > 1 ? 1 : 0];
  float acc[4][2];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j][0] = acc[j][1] = 0.f;
  for (int k0 = 0; k0 < Kc; k0 += kGenThreads) {
    const int i = k0 + tid;
    FastPoint P{0, 0, 0.f, 0.f};
    if (i < Kc) {
      int p = fp.pos[it.base + i];
      if (f.validate && (p >= N || (i > 0 && (int)fp.pos[it.base + i - 1] >= p))) bad |= kStatusMask;
      p = min(p, N - 1);
      P.x = p % w;
      P.y = p / w;
      const int q0 = fp.coef[it.vbase0 + i];
      const int q1 = it.nv > 1 ? (int)fp.coef[it.vbase1 + i] : 0;
      if (f.validate && (q0 == -128 || q1 == -128)) bad |= kStatusValue;
      P.c0 = coef_value(q0, f.qstep[pl0], f.qrho);
      P.c1 = coef_value(q1, f.qstep[pl1], f.qrho);
    }
    __syncthreads();  // the previous chunk is consumed
    pts[tid] = P;
    __syncthreads();
    const int nk = min(kGenThreads, Kc - k0);
    for (int k = 0; k < nk; ++k) {
      const FastPoint Q = pts[k];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int px = tid + j * kGenThreads;
        if (px < N) {
          const float g = green_tab(tab, w, h, px % w, px / w, Q.x, Q.y);
          acc[j][0] = fmaf(Q.c0, g, acc[j][0]);
          acc[j][1] = fmaf(Q.c1, g, acc[j][1]);
        }
      }
    }
  }
  if (Kc == 0) __syncthreads();  // the table is in LDS (no chunk loop ran)
  for (int v = 0; v < it.nv; ++v) {
    const float a = fp.consts[G.cbase[v] + it.l];
    if (f.validate && !isfinite(a)) bad |= kStatusValue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int px = tid + j * kGenThreads;
      if (px < N) store_px(po, (unsigned)(it.obase(v) + (px / w) * it.W + px % w), (v ? acc[j][1] : acc[j][0]) + a);
    }
  }
  if (bad) atomicOr(f.status, bad);
}

// Persistent pass over both deferred lists of a stored-coefficient decode;
// the last workgroup clears the counters as in k_general_deferred.
__global__ __launch_bounds__(kGenThreads) void k_coef_general(FrameDev f) {
  __shared__ FastPoint pts[kGenThreads];
  __shared__ float tab[33 * 33];
  __shared__ int last;
  const int nmed = f.counters[0];
  const int nlarge = f.counters[1];
  const int cap = f.n_items * f.nframes;
  if (nmed + nlarge == 0 && f.nq == 0) return;  // as in k_general_deferred
  for (int idx = blockIdx.x; idx < nmed + nlarge; idx += gridDim.x) {
    const int e = idx < nmed ? f.deferred[idx] : f.deferred[cap - 1 - (idx - nmed)];
    coef_block(f, e >> kDeferFrameShift, e & kDeferItemMask, pts, tab);
  }
  __syncthreads();
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(&f.counters[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
           (int)gridDim.x - 1;
  __syncthreads();
  if (last)
    for (int i = threadIdx.x; i < kNumCounters; i += kGenThreads)
      __hip_atomic_store(&f.counters[i], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- launchers

hipError_t launch_fast(const FrameDev &f, hipStream_t stream) {
  if (f.fast_wgs == 0) return hipSuccess;
  const size_t lds = sizeof(float) * (size_t)f.fast_lds;
  const dim3 g(f.fast_wgs, f.nframes), b(kFastThreads);
  if (f.enc) {
    hipLaunchKernelGGL((k_fast<2, 0>), g, b, lds, stream, f);
  } else if (f.coef) {
    switch (f.eval) {
      case 1: hipLaunchKernelGGL((k_fast<1, 1>), g, b, lds, stream, f); break;
      case 2: hipLaunchKernelGGL((k_fast<1, 2>), g, b, lds, stream, f); break;
      case 3: hipLaunchKernelGGL((k_fast<1, 3>), g, b, lds, stream, f); break;
      default:
        if (f.b == 8) hipLaunchKernelGGL((k_fast<1, 0, 1>), g, b, lds, stream, f);
        else hipLaunchKernelGGL((k_fast<1, 0, 0>), g, b, lds, stream, f);
        break;
    }
  } else {
    switch (f.eval) {
      case 1: hipLaunchKernelGGL((k_fast<0, 1>), g, b, lds, stream, f); break;
      case 2: hipLaunchKernelGGL((k_fast<0, 2>), g, b, lds, stream, f); break;
      case 3: hipLaunchKernelGGL((k_fast<0, 3>), g, b, lds, stream, f); break;
      default:
        if (f.b == 8) hipLaunchKernelGGL((k_fast<0, 0, 1>), g, b, lds, stream, f);
        else hipLaunchKernelGGL((k_fast<0, 0, 0>), g, b, lds, stream, f);
        break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_fast2(const FrameDev &f, hipStream_t stream) {
  if (f.fast_wgs == 0) return hipSuccess;
  const dim3 bg((f.n_items + kBinThreads - 1) / kBinThreads, f.nframes);
  hipLaunchKernelGGL(k_fbin_count, bg, dim3(kBinThreads), 0, stream, f);
  hipLaunchKernelGGL(k_fbin_scan, dim3(8 * f.nq), dim3(kBinThreads), 0, stream, f, (int)(bg.x * bg.y));
  hipLaunchKernelGGL(k_fbin_place, bg, dim3(kBinThreads), 0, stream, f);
  const size_t lds = sizeof(float) * (size_t)f.fast_lds;
  const dim3 g(f.fast_wgs), b(kF2Threads);
  switch (f.eval) {
    case 1: hipLaunchKernelGGL((k_fast2<1>), g, b, lds, stream, f); break;
    case 2: hipLaunchKernelGGL((k_fast2<2>), g, b, lds, stream, f); break;
    case 3: hipLaunchKernelGGL((k_fast2<3>), g, b, lds, stream, f); break;
    default:
      if (f.b == 8) hipLaunchKernelGGL((k_fast2<0, 1>), g, b, lds, stream, f);
      else hipLaunchKernelGGL((k_fast2<0, 0>), g, b, lds, stream, f);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_plain_all(const FrameDev &f, hipStream_t stream) {
  if (f.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_plain_all, dim3(f.n_items, f.nframes), dim3(kGenThreads), 0, stream, f);
  return hipGetLastError();
}

hipError_t launch_general_deferred(const FrameDev &f, hipStream_t stream) {
  hipLaunchKernelGGL(k_general_deferred, dim3(kGeneralGrid), dim3(kGenThreads), 0, stream, f);
  return hipGetLastError();
}

hipError_t launch_coef_general(const FrameDev &f, hipStream_t stream) {
  hipLaunchKernelGGL(k_coef_general, dim3(kGeneralGrid), dim3(kGenThreads), 0, stream, f);
  return hipGetLastError();
}

}  // namespace pdi
