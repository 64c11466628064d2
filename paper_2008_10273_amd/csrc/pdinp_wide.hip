// Wave-per-block path for blocks of up to 32 x 32 pixels with K <= 103 mask
// points (Sec. 2.2 of the paper, per block: assemble G_K, solve the bordered
// system [G_K 1; 1^T 0][c; a] = [r; 0], evaluate u = sum_i c_i G(., x_i) + a).
//
// One 64-lane wave per block.  Lane i holds row i of the bordered system in
// VGPRs, and row i + 64 as well when K + 1 > 64.  The elimination runs in
// LDL^T order without pivoting: the leading K x K block is SPD and the last
// pivot is -1^T G_K^-1 1 != 0.  Every trailing submatrix of the symmetric
// bordered matrix is symmetric, so the multiplier of row i at step j,
// M[i][j] / M[j][j], is read from the pivot row (element i), which its owner
// lane publishes in LDS; the other lanes read it whole as broadcast vector
// loads.  A back substitution over the upper triangle left in the rows then
// gives (c, a).  The evaluation uses the DCT-II factorisation of G (Eq. 4)
// on 2 x 2 tiles of 16 x 16 matrix-core products.
#include "pdinp_device.h"

#include <hip/hip_runtime.h>

namespace pdi {

typedef float V32 __attribute__((ext_vector_type(32)));
typedef float V8 __attribute__((ext_vector_type(8)));

constexpr int kWideCap2 = kWideKMax + 1;       // n <= 104: rows i and i + 64 per lane
constexpr int kWideStagePts = 112;             // evaluation points staged (multiple of 16)
constexpr int kGroups = (kWideCap2 + 31) / 32; // 32-column groups of a row
constexpr int kProw = 132;                     // stride of a published row (floats, 16-byte multiple)
static_assert(kWideCap2 == 104, "row storage below holds 104 columns");

// The lane's rows of the bordered system in VGPRs: row i (columns 0..103)
// and row i + 64, of which only columns 64..103 are kept: its columns below
// 64 lie in the lower triangle, which the elimination never reads.  Indices
// are compile-time constants after unrolling.
struct WRow {
  V32 q0, q1, q2;
  V8 t0;
  __device__ __forceinline__ float get(int k) const {
    return k < 32 ? q0[k] : k < 64 ? q1[k - 32] : k < 96 ? q2[k - 64] : t0[k - 96];
  }
  __device__ __forceinline__ void set(int k, float v) {
    if (k < 32) q0[k] = v;
    else if (k < 64) q1[k - 32] = v;
    else if (k < 96) q2[k - 64] = v;
    else t0[k - 96] = v;
  }
};
struct WRowHi {
  V32 q2;
  V8 t0;
  __device__ __forceinline__ float get(int k) const { return k < 64 ? 0.f : k < 96 ? q2[k - 64] : t0[k - 96]; }
  __device__ __forceinline__ void set(int k, float v) {
    if (k >= 64 && k < 96) q2[k - 64] = v;
    else if (k >= 96) t0[k - 96] = v;
  }
};
struct WRows {
  WRow r0;
  WRowHi r1;
  __device__ __forceinline__ float get(int s, int k) const { return s ? r1.get(k) : r0.get(k); }
  __device__ __forceinline__ void set(int s, int k, float v) {
    if (s) r1.set(k, v); else r0.set(k, v);
  }
};

struct WidePoint {
  int x, y;
  float c0, c1;
};

// Per-wave LDS.
struct alignas(16) WideStage {
  float prow[4 * 132];  // published block rows (stride kProw): columns 0..103, values at 128, 129
  int xy[kWideCap2];    // mask points: x | (y * (w + 1)) << 16
  WidePoint p[kWideStagePts];
  float a[2];
};

struct WideJob {
  int K, base, nv;
  long long vb0, vb1, ob0, ob1;
};

__device__ __forceinline__ float lane_f(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Assemble, factor and solve the bordered system of one block; stage (x, y,
// c) of the K points and a for the evaluation.  Returns false when the pivots
// call for FP64 refinement (the general path refines).
__device__ __forceinline__ bool wide_solve(const FrameDev &f, const WideJob &jb, int lane, int w, int h,
                                           const float *Hc, WideStage &st) {
  constexpr int RS = 2, CAP = kWideCap2;
  const int K = jb.K, n = K + 1, N = w * h, W1 = w + 1;
  const bool two = n > 64;  // row set 1 (rows 64..) in use; otherwise its work is skipped
  int xr[RS], yr[RS], ywr[RS];
  float T[RS][2];
  int bad = 0;
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int i = lane + 64 * s;
    xr[s] = yr[s] = ywr[s] = 0;
    T[s][0] = T[s][1] = 0.f;
    if (i < K) {
      const uint16_t *pos = f.fp[blockIdx.y].pos;
      int p = pos[jb.base + i];
      if (f.validate && (p >= N || (i > 0 && (int)pos[jb.base + i - 1] >= p))) bad |= kStatusMask;
      p = min(p, N - 1);
      xr[s] = p % w;
      yr[s] = p / w;
      ywr[s] = yr[s] * W1;
      const float *vals = f.fp[blockIdx.y].values;
      T[s][0] = vals[jb.vb0 + i];
      if (jb.nv > 1) T[s][1] = vals[jb.vb1 + i];
      if (f.validate && !(isfinite(T[s][0]) && isfinite(T[s][1]))) bad |= kStatusValue;
    }
    if (i < kWideCap2) st.xy[i] = (i < K) ? (xr[s] | (ywr[s] << 16)) : 0;
  }
  if (bad) atomicOr(f.status, bad);
  wave_sync();

  // Assembly: row i = [G(x_i, x_k) for k < K | 1 | 0...] for i < K, the border
  // row [1 ... 1 | 0] for i = K, zero rows past K.  G is the sum of four
  // quarter-scaled compact-table entries: (|dx|, |dy|) and the reflections
  // x_i + x_k + 1, y_i + y_k + 1 folded into [0, w] and [0, h].
  WRows R;
  const int xcr = 2 * w - 1, ycr = (2 * h - 1) * W1;
#pragma unroll
  for (int c = 0; c < CAP / 8; ++c) {
    if (8 * c < n) {
      const f4 pa = *reinterpret_cast<const f4 *>(&st.xy[8 * c]);
      const f4 pb = *reinterpret_cast<const f4 *>(&st.xy[8 * c + 4]);
      float g[RS][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int pk = __builtin_bit_cast(int, e < 4 ? pa[e] : pb[e - 4]);
        const int xk = pk & 0xffff, ykw = pk >> 16;
#pragma unroll
        for (int s = 0; s < RS; ++s) {
          g[s][e] = 0.f;
          if (s == 1 && (c < 8 || !two)) continue;  // row set 1 needs columns >= 64 only
          const int dyw = (int)__usad((unsigned)ywr[s], (unsigned)ykw, 0u);
          const int syw = min(ywr[s] + ykw + W1, ycr - ywr[s] - ykw);
          const int dx = (int)__usad((unsigned)xr[s], (unsigned)xk, 0u);
          const int sx = min(xr[s] + xk + 1, xcr - xr[s] - xk);
          g[s][e] = (Hc[dyw + dx] + Hc[dyw + sx]) + (Hc[syw + dx] + Hc[syw + sx]);
        }
      }
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int i = lane + 64 * s;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = 8 * c + e;
          const float inner = (i < K) ? g[s][e] : (i == K ? 1.f : 0.f);  // columns k < K
          const float outer = (k == K && i < K) ? 1.f : 0.f;              // columns k >= K
          R.set(s, k, k < K ? inner : outer);
        }
      }
    }
  }

  // Forward elimination in blocks of 4 pivots (rows j .. j+3; fewer at the
  // end).  The 4 owner lanes publish their rows from the block's 32-column
  // group on, with the value columns.  Every lane factors the 4 x 4 diagonal
  // block A11 = L D L^T (the same arithmetic in every lane) and, with p_i =
  // the block rows' column i (= row i's columns j..j+3, by symmetry), solves
  // A11 c_i = p_i; a row inside the block uses only the pivots before it.
  // Then row i -= sum_t c_i[t] * (block row t): a rank-4 update that leaves
  // the Schur complement below the block and the U rows of the block.
  float d[RS];
#pragma unroll
  for (int s = 0; s < RS; ++s) d[s] = 1.f;
  float dmin = 3.0e38f, dmax = 0.f;
#pragma unroll
  for (int JS = 0; JS < RS; ++JS) {
    const int jend = min(n, 64 * JS + 64);
    for (int j = 64 * JS; j < jend; j += 4) {
      const int bk = min(4, n - j), jl = j & 63, jg = j >> 5;
      const int tw = lane - jl;  // this lane's row position in the block
      if (tw >= 0 && tw < 4) {   // rows past n are zero rows: they publish zeros
        float *dst = st.prow + tw * kProw;
#pragma unroll
        for (int g = 0; g < kGroups; ++g) {
          if (g >= jg && 32 * g < n) {
#pragma unroll
            for (int c = 4 * g; c < min(4 * g + 4, CAP / 8); ++c) {
              f4 a, b;
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                a[e] = R.get(JS, 8 * c + e);
                b[e] = R.get(JS, 8 * c + 4 + e);
              }
              reinterpret_cast<f4 *>(dst)[2 * c] = a;
              reinterpret_cast<f4 *>(dst)[2 * c + 1] = b;
            }
          }
        }
        dst[128] = T[JS][0];
        dst[129] = T[JS][1];
      }
      wave_sync();
      // A11 (identity rows past the block end), then A11 = L D L^T.
      float a[4][4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const f4 r = *reinterpret_cast<const f4 *>(st.prow + t * kProw + j);
#pragma unroll
        for (int u = 0; u < 4; ++u) a[t][u] = (t < bk) ? r[u] : (t == u ? 1.f : 0.f);
      }
      float D[4], rD[4], L[4][4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float s_ = a[t][t];
#pragma unroll
        for (int u = 0; u < t; ++u) s_ -= L[t][u] * L[t][u] * D[u];
        D[t] = s_;
        rD[t] = __builtin_amdgcn_rcpf(s_);
#pragma unroll
        for (int r = t + 1; r < 4; ++r) {
          float v = a[r][t];
#pragma unroll
          for (int u = 0; u < t; ++u) v -= L[r][u] * L[t][u] * D[u];
          L[r][t] = v * rD[t];
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < bk && j + t < K) {
          dmin = fminf(dmin, fabsf(D[t]));
          dmax = fmaxf(dmax, fabsf(D[t]));
        }
      // Coefficients of the lane's rows.
      float cf[RS][4];
#pragma unroll
      for (int s = 0; s < RS; ++s) {
#pragma unroll
        for (int t = 0; t < 4; ++t) cf[s][t] = 0.f;
        if (s < JS) continue;
        const int i = lane + 64 * s;
        const int m = (i < j || i >= n) ? 0 : min(i - j, bk);
        float z[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          float v = st.prow[t * kProw + min(i, 127)];
#pragma unroll
          for (int u = 0; u < t; ++u) v -= L[t][u] * z[u];
          z[t] = v;
        }
#pragma unroll
        for (int t = 3; t >= 0; --t) {
          float v = (t < m) ? z[t] * rD[t] : 0.f;
#pragma unroll
          for (int u = t + 1; u < 4; ++u) v -= L[u][t] * cf[s][u];
          cf[s][t] = v;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) d[s] = (i == j + t && t < bk) ? D[t] : d[s];
      }
      // Rank-4 update, 8 columns (4 rows x 2 vectors per row) per load batch.
      // Columns left of the block inside its first group belong to the lower
      // triangle, which no later step reads; row set 1 (rows 64..) never
      // needs its columns below 64.
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        if (g >= jg && 32 * g < n) {
#pragma unroll
          for (int c = 4 * g; c < min(4 * g + 4, CAP / 8); ++c) {
            f4 pv[4][2];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              pv[t][0] = *reinterpret_cast<const f4 *>(st.prow + t * kProw + 8 * c);
              pv[t][1] = *reinterpret_cast<const f4 *>(st.prow + t * kProw + 8 * c + 4);
            }
#pragma unroll
            for (int s = JS; s < RS; ++s) {
              if (s == 1 && (c < 8 || (JS == 0 && !two))) continue;
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                const int k = 8 * c + e;
                float v = R.get(s, k);
#pragma unroll
                for (int t = 0; t < 4; ++t) v = fmaf(-cf[s][t], pv[t][e >> 2][e & 3], v);
                R.set(s, k, v);
              }
            }
          }
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float t0 = st.prow[t * kProw + 128], t1 = st.prow[t * kProw + 129];
#pragma unroll
        for (int s = JS; s < RS; ++s) {
          T[s][0] = fmaf(-cf[s][t], t0, T[s][0]);
          T[s][1] = fmaf(-cf[s][t], t1, T[s][1]);
        }
      }
      wave_sync();  // every lane has read the block rows before the next are published
    }
  }
  const bool need = (f.refine == 2) || (f.refine == 1 && !(dmin >= f.tau * dmax));
  if (need) return false;

  // Back substitution: x_k = (y_k - sum_{j > k} U[k][j] x_j) / U[k][k],
  // accumulated into the rows above k as each x_k is broadcast.
  float rd[RS], acc[RS][2];
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    rd[s] = __builtin_amdgcn_rcpf(d[s]);
    acc[s][0] = acc[s][1] = 0.f;
  }
#pragma unroll
  for (int k = CAP - 1; k >= 0; --k) {
    if (k < n) {
      const int ks = k >> 6, kl = k & 63;
      float t0 = 0.f, t1 = 0.f;
#pragma unroll
      for (int s = 0; s < RS; ++s)
        if (s == ks) {
          t0 = (T[s][0] - acc[s][0]) * rd[s];
          t1 = (T[s][1] - acc[s][1]) * rd[s];
        }
      const float x0 = lane_f(t0, kl), x1 = lane_f(t1, kl);
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        if (64 * s < k) {
          const bool above = lane + 64 * s < k;
          const float u = R.get(s, k);
          acc[s][0] = above ? fmaf(u, x0, acc[s][0]) : acc[s][0];
          acc[s][1] = above ? fmaf(u, x1, acc[s][1]) : acc[s][1];
        }
      }
    }
  }

  // Stage the K points with their coefficients (zeros up to the next multiple
  // of 16) and a = x_K.
  bool fin = true;
  float aK0 = 0.f, aK1 = 0.f;
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int i = lane + 64 * s;
    const float c0 = (T[s][0] - acc[s][0]) * rd[s];
    const float c1 = (T[s][1] - acc[s][1]) * rd[s];
    if (i < kWideStagePts) {
      WidePoint P;
      P.x = i < K ? xr[s] : 0;
      P.y = i < K ? yr[s] : 0;
      P.c0 = i < K ? c0 : 0.f;
      P.c1 = i < K ? c1 : 0.f;
      st.p[i] = P;
    }
    if (i <= K) fin &= isfinite(c0) && isfinite(c1);
    if ((K >> 6) == s) {
      aK0 = c0;
      aK1 = c1;
    }
  }
  st.a[0] = lane_f(aK0, K & 63);
  st.a[1] = lane_f(aK1, K & 63);
  if (__ballot(!fin)) {
    if (lane == 0) atomicOr(f.status, kStatusSolve);
  }
  wave_sync();
  return true;
}

// u = Dh^T (lam .* (Dw[:,X] diag(c) Dh[:,Y]^T)^T) Dw + a over the 32 x 32
// block as 2 x 2 tiles of FP32 16x16x4 MFMA chains (lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; the result D[4(l/16)+r][l%16] is register
// r).  D holds Dw[p][x], Dh[q][y] and lam[q][p], 32 x 32 each, zero-padded.
__device__ __forceinline__ void wide_eval32(const FrameDev &f, const WideJob &jb, const float *D,
                                            const WideStage &st, int lane, int w, int h, int W) {
  const float *Dw = D, *Dh = D + 1024, *lam = D + 2048;
  const int lo = lane & 15, hi = lane >> 4;
  const int nch = (jb.K + 7) >> 3;  // pairs of 4-point chunks (staged points are zero past K)
  for (int v = 0; v < jb.nv; ++v) {
    f4 acc[2][2];
#pragma unroll
    for (int pt = 0; pt < 2; ++pt)
#pragma unroll
      for (int qt = 0; qt < 2; ++qt) acc[pt][qt] = f4{0.f, 0.f, 0.f, 0.f};
    for (int ch = 0; ch < nch; ++ch) {
      float ao[2][2], bo[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const WidePoint P = st.p[8 * ch + 4 * u + hi];
        const float cv = v ? P.c1 : P.c0;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          ao[u][t] = cv * Dw[(16 * t + lo) * 32 + P.x];  // A[p][i], p = 16 pt + lo
          bo[u][t] = Dh[(16 * t + lo) * 32 + P.y];       // B[i][q], q = 16 qt + lo
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int pt = 0; pt < 2; ++pt)
#pragma unroll
          for (int qt = 0; qt < 2; ++qt)
            acc[pt][qt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ao[u][pt], bo[u][qt], acc[pt][qt], 0, 0, 0);
    }
    // acc[pt][qt][j] = V^T[p = 16 pt + 4 hi + j][q = 16 qt + lo].
    // S[q][x] = sum_p lam[q][p] V^T[p][q] Dw[p][x]
    f4 S[2][2];
#pragma unroll
    for (int qt = 0; qt < 2; ++qt)
#pragma unroll
      for (int xt = 0; xt < 2; ++xt) {
        f4 s4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int pt = 0; pt < 2; ++pt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int p = 16 * pt + 4 * hi + j;
            const float a = acc[pt][qt][j] * lam[(16 * qt + lo) * 32 + p];
            s4 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Dw[p * 32 + 16 * xt + lo], s4, 0, 0, 0);
          }
        S[qt][xt] = s4;  // S[q = 16 qt + 4 hi + r][x = 16 xt + lo]
      }
    const float av = st.a[v];
    const long long ob = v ? jb.ob1 : jb.ob0;
#pragma unroll
    for (int yt = 0; yt < 2; ++yt)
#pragma unroll
      for (int xt = 0; xt < 2; ++xt) {
        f4 u4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int qt = 0; qt < 2; ++qt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int q = 16 * qt + 4 * hi + j;
            u4 = __builtin_amdgcn_mfma_f32_16x16x4f32(Dh[q * 32 + 16 * yt + lo], S[qt][xt][j], u4, 0, 0, 0);
          }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int y = 16 * yt + 4 * hi + r, x = 16 * xt + lo;
          if (x < w && y < h) store_px(f, blockIdx.y, ob + (long long)y * W + x, u4[r] + av);
        }
      }
  }
}

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef __bf16 b4 __attribute__((ext_vector_type(4)));

// acc += A B on a 16x16x16 MFMA with reduced-precision operands: lane l
// supplies A[l%16][4(l/16)+e] = a[e] and B[4(l/16)+e][l%16] = b[e].
template <int EV>
__device__ __forceinline__ f4 wmma16(f4 acc, const float a[4], const float b[4]) {
  if constexpr (EV == 1) {
    h4 ha, hb;
#pragma unroll
    for (int e = 0; e < 4; ++e) { ha[e] = (_Float16)a[e]; hb[e] = (_Float16)b[e]; }
    return __builtin_amdgcn_mfma_f32_16x16x16f16(ha, hb, acc, 0, 0, 0);
  } else if constexpr (EV == 2) {
    b4 ba, bb;
#pragma unroll
    for (int e = 0; e < 4; ++e) { ba[e] = (__bf16)a[e]; bb[e] = (__bf16)b[e]; }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ba, bb, acc, 0, 0, 0);
  } else {  // split BF16: x = hi + lo, A B ~ hi*hi + hi*lo + lo*hi
    b4 ah, al, bh, bl;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ah[e] = (__bf16)a[e];
      al[e] = (__bf16)(a[e] - (float)ah[e]);
      bh[e] = (__bf16)b[e];
      bl[e] = (__bf16)(b[e] - (float)bh[e]);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
  }
}

// The evaluation of wide_eval32 with FP16 / BF16 / split-BF16 operands and
// FP32 accumulation (k = 16 per product).
template <int EV>
__device__ __forceinline__ void wide_eval16(const FrameDev &f, const WideJob &jb, const float *D,
                                            const WideStage &st, int lane, int w, int h, int W) {
  const float *Dw = D, *Dh = D + 1024, *lam = D + 2048;
  const int lo = lane & 15, hi = lane >> 4;
  const int nch = (jb.K + 15) >> 4;
  for (int v = 0; v < jb.nv; ++v) {
    f4 acc[2][2];
#pragma unroll
    for (int pt = 0; pt < 2; ++pt)
#pragma unroll
      for (int qt = 0; qt < 2; ++qt) acc[pt][qt] = f4{0.f, 0.f, 0.f, 0.f};
    for (int ch = 0; ch < nch; ++ch) {
      float ao[2][4], bo[2][4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const WidePoint P = st.p[16 * ch + 4 * hi + e];
        const float cv = v ? P.c1 : P.c0;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          ao[t][e] = cv * Dw[(16 * t + lo) * 32 + P.x];
          bo[t][e] = Dh[(16 * t + lo) * 32 + P.y];
        }
      }
#pragma unroll
      for (int pt = 0; pt < 2; ++pt)
#pragma unroll
        for (int qt = 0; qt < 2; ++qt) acc[pt][qt] = wmma16<EV>(acc[pt][qt], ao[pt], bo[qt]);
    }
    // acc[pt][qt][e] = V^T[p = 16 pt + 4 hi + e][q = 16 qt + lo]
    f4 S[2][2];
#pragma unroll
    for (int qt = 0; qt < 2; ++qt)
#pragma unroll
      for (int xt = 0; xt < 2; ++xt) {
        f4 s4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int pt = 0; pt < 2; ++pt) {
          float a[4], b[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int p = 16 * pt + 4 * hi + e;
            a[e] = acc[pt][qt][e] * lam[(16 * qt + lo) * 32 + p];
            b[e] = Dw[p * 32 + 16 * xt + lo];
          }
          s4 = wmma16<EV>(s4, a, b);
        }
        S[qt][xt] = s4;
      }
    const float av = st.a[v];
    const long long ob = v ? jb.ob1 : jb.ob0;
#pragma unroll
    for (int yt = 0; yt < 2; ++yt)
#pragma unroll
      for (int xt = 0; xt < 2; ++xt) {
        f4 u4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int qt = 0; qt < 2; ++qt) {
          float a[4], b[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int q = 16 * qt + 4 * hi + e;
            a[e] = Dh[q * 32 + 16 * yt + lo];
            b[e] = S[qt][xt][e];
          }
          u4 = wmma16<EV>(u4, a, b);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int y = 16 * yt + 4 * hi + r, x = 16 * xt + lo;
          if (x < w && y < h) store_px(f, blockIdx.y, ob + (long long)y * W + x, u4[r] + av);
        }
      }
  }
}

// Binning: every mask block goes to its shape's queue, into one of 4 bins by
// point count, so that the long solves are handed out first; blocks the wave
// path does not take (K = 0, K = w*h, K > 103, invalid counts) go to the
// general path's lists.
__global__ __launch_bounds__(256) void k_bin(FrameDev f) {
  const int m = blockIdx.x * 256 + threadIdx.x, fi = blockIdx.y;
  const int32_t *bp = f.fp[fi].block_ptr;
  int *cnt = f.counters + kQueueCounters + 4 * kMaxShapes * fi;
  int *list = f.binlist + 2 * f.n_items * fi;
  int key = -1;  // 4 * queue + bin, or -1: not queued
  if (m < f.n_items) {
  int g = 0;
  if (f.ngroups > 1 && m >= f.g[1].first) g = 1;
  if (f.ngroups > 2 && m >= f.g[2].first) g = 2;
  const GroupDev &G = f.g[g];
  const int l = m - G.first, bx = l % G.nbx, by = l / G.nbx;
  const int e = ((bx == G.nbx - 1) && (G.W % f.b) ? 1 : 0) + ((by == G.nby - 1) && (G.H % f.b) ? 2 : 0);
  const int shape = G.shape[e];
  const int w = f.s[shape].w, h = f.s[shape].h;
  const int K = bp[m + 1] - bp[m];
  if (K < 1 || K >= w * h || K > kWideKMax) push_deferred(f, fi, m, K, w, h);
  else key = 4 * f.qof[shape] + (K >= kBinK0 ? 0 : K >= kBinK1 ? 1 : K >= kBinK2 ? 2 : 3);
  }
  // One atomic per distinct queue and bin in the wave: the lanes of a key
  // take consecutive slots after the leader's reservation.
  unsigned long long todo = __ballot(key >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int k = __shfl(key, leader);
    const unsigned long long mine = __ballot(key == k);
    todo &= ~mine;
    const int rank = __popcll(mine & ((1ull << (threadIdx.x & 63)) - 1ull));
    int base = 0;
    if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(&cnt[k], __popcll(mine));
    base = __shfl(base, leader);
    if (key == k) {
      const QueueDev &Q = f.q[k >> 2];
      const int bin = k & 3, idx = base + rank;
      const int half = 2 * Q.base + (bin >> 1) * Q.count;  // bins 0, 1 | bins 2, 3
      if (idx < Q.count) list[half + ((bin & 1) ? Q.count - 1 - idx : idx)] = m;
      else atomicOr(f.status, kStatusSolve);  // counters were not cleared by the previous decode
    }
  }
}

// One block per wave, WAVES waves per workgroup (the workgroup shares the
// shape's tables in LDS); each wave takes the next block of its queue.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_wide(FrameDev f) {
  extern __shared__ __attribute__((aligned(16))) float tabs[];  // Hc | Dw | Dh | lam of the shape
  __shared__ WideStage stage[WAVES];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform, so is all that follows
  const int wg = blockIdx.x;
  int qi = 0;
  while (qi + 1 < f.nq && wg >= f.q[qi + 1].first_wg) ++qi;
  const QueueDev Q = f.q[qi];
  const ShapeDev S = f.s[Q.shape];
  const int w = S.w, h = S.h;
  {
    const int n4 = (S.jt_floats + 3072) >> 2;
    const f4 *src = reinterpret_cast<const f4 *>(f.tab32 + S.fast);
    f4 *dst = reinterpret_cast<f4 *>(tabs);
    for (int i = tid; i < n4; i += 64 * WAVES) dst[i] = src[i];
  }
  __syncthreads();  // the only workgroup barrier: waves are independent from here on

  // Queue position of this wave's block: workgroups start in index order, so
  // the first ones take the large-K blocks at the front of the queue.
  const int p = (wg - Q.first_wg) * WAVES + wv;
  const int fi = blockIdx.y;
  const int32_t *bp = f.fp[fi].block_ptr;
  const int *cnt = f.counters + kQueueCounters + 4 * (kMaxShapes * fi + qi);
  const int n0 = cnt[0], n1 = cnt[1], n2 = cnt[2], n3 = cnt[3];
  if (p >= Q.count || n0 + n1 > Q.count || n2 + n3 > Q.count) return;
  const int *h0 = f.binlist + 2 * f.n_items * fi + 2 * Q.base, *h1 = h0 + Q.count;
  int m;
  if (p < n0) m = h0[p];
  else if (p < n0 + n1) m = h0[Q.count - 1 - (p - n0)];
  else if (p < n0 + n1 + n2) m = h1[p - n0 - n1];
  else if (p < n0 + n1 + n2 + n3) m = h1[Q.count - 1 - (p - n0 - n1 - n2)];
  else return;
  m = __builtin_amdgcn_readfirstlane(m);
  if ((unsigned)m >= (unsigned)f.n_items) return;
  int gi = 0;
  if (f.ngroups > 1 && m >= f.g[1].first) gi = 1;
  if (f.ngroups > 2 && m >= f.g[2].first) gi = 2;
  const GroupDev &G = f.g[gi];
  const int bl = m - G.first, bx = bl % G.nbx, by = bl / G.nbx;
  const int lo = bp[m], hi = bp[m + 1];
  WideJob jb;
  jb.K = hi - lo;
  jb.base = lo;
  jb.nv = G.nv;
  const long long pix = (long long)(by * f.b) * G.W + bx * f.b;
  jb.vb0 = lo;
  jb.ob0 = G.out_off[0] + pix;
  jb.vb1 = jb.vb0;
  jb.ob1 = jb.ob0;
  if (G.nv > 1) {
    jb.vb1 = f.shared ? (long long)bp[f.n_items] + (lo - bp[f.chroma_first]) : lo;
    jb.ob1 = G.out_off[1] + pix;
  }
  const int K = jb.K;  // 1 <= K <= min(w*h - 1, kWideKMax): binned
  WideStage &st = stage[wv];
  const bool solved = wide_solve(f, jb, lane, w, h, tabs, st);
  if (!solved) {
    if (lane == 0) push_deferred(f, fi, m, K, w, h);
    return;
  }
  const float *D = tabs + S.jt_floats;
  switch (f.eval) {
    case 1: wide_eval16<1>(f, jb, D, st, lane, w, h, G.W); break;
    case 2: wide_eval16<2>(f, jb, D, st, lane, w, h, G.W); break;
    case 3: wide_eval16<3>(f, jb, D, st, lane, w, h, G.W); break;
    default: wide_eval32(f, jb, D, st, lane, w, h, G.W); break;
  }
}

hipError_t launch_wide(const FrameDev &f, hipStream_t stream) {
  if (f.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin, dim3((f.n_items + 255) / 256, f.nframes), dim3(256), 0, stream, f);
  const size_t lds = sizeof(float) * (size_t)f.fast_lds;
  switch (f.ipw) {
    case 1: hipLaunchKernelGGL(k_wide<1>, dim3(f.fast_wgs, f.nframes), dim3(64), lds, stream, f); break;
    case 2: hipLaunchKernelGGL(k_wide<2>, dim3(f.fast_wgs, f.nframes), dim3(128), lds, stream, f); break;
    case 4: hipLaunchKernelGGL(k_wide<4>, dim3(f.fast_wgs, f.nframes), dim3(256), lds, stream, f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pdi
