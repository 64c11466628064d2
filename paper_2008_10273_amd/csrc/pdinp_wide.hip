// Wave-per-block path for blocks of up to 32 x 32 pixels with K <= 103 mask
// points (Sec. 2.2 of the paper, per block: assemble G_K, solve the bordered
// system [G_K 1; 1^T 0][c; a] = [r; 0], evaluate u = sum_i c_i G(., x_i) + a).
//
// One 64-lane wave per block.  The bordered matrix (n = K + 1 rows, padded
// with identity rows to a multiple of 16) is held as its upper triangle of
// 16 x 16 tiles in the matrix-core accumulator layout: lane l, register r
// holds row 4(l/16) + r, column l%16 of the tile.  Block LDL^T without
// pivoting (the leading K x K block is SPD and the last pivot is
// -1^T G_K^-1 1 != 0): per diagonal tile p the lanes factor A_pp = L D L^T
// row by row (16-lane rows, broadcasts within a row) and keep D and L^-1;
// W = L^-1 A_pj for the tiles right of it, A_ij -= W_pi^T D^-1 W_pj for the
// trailing tiles, and the right-hand sides alike, are matrix-core products.
// A back substitution over the tiles gives (c, a).  The evaluation uses the
// DCT-II factorisation of G (Eq. 4) on 2 x 2 tiles of 16 x 16 products.
#include "pdinp_device.h"

#include <hip/hip_runtime.h>

namespace pdi {

constexpr int kWideStagePts = 112;  // points staged (multiple of 16, > kWideKMax)
constexpr int kTileN = 7;           // 16 x 16 tiles per side: n = K + 1 <= 104 <= 112
constexpr int kTb = 20;             // row stride of the per-wave tile buffer (floats)
static_assert(16 * kTileN == kWideStagePts && kWideKMax + 1 <= kWideStagePts, "tile cover");
// Index of tile (i, j), i <= j, in the packed upper triangle of TN x TN tiles.
template <int TN>
__host__ __device__ constexpr int tixn(int i, int j) { return i * TN - i * (i - 1) / 2 + (j - i); }
template <int TN>
constexpr int kNumTilesN = tixn<TN>(TN - 1, TN - 1) + 1;
typedef int i4 __attribute__((ext_vector_type(4)));

struct WidePoint {
  int x, y;
  float c0, c1;
};

// Per-wave LDS.
struct alignas(16) WideStage {
  float tb[16 * kTb];                // rows of a diagonal tile
  float dv[kWideStagePts];           // reciprocal pivots
  float rv[2][kWideStagePts];        // right-hand sides
  int xy[kWideStagePts];             // points as table byte offsets: 4x | (4 y (w + 1)) << 16
  WidePoint p[kWideStagePts];        // points and coefficients for the evaluation
  float a[2];
};

struct WideJob {
  int K, base, nv;
  long long vb0, vb1, ob0, ob1;
  int pl0, pl1;     // value planes (stored-coefficient decodes)
  int cidx0, cidx1; // indices of the block's constants
};

// Stored-coefficient decodes: stage (x, y, c) of the block's points (codes
// dequantised; zeros past K) and its constants, in place of the solve.
__device__ __forceinline__ void wide_coef_stage(const FrameDev &f, const WideJob &jb, int lane, int w, int h,
                                                WideStage &st) {
  const FramePtrs fp = f.fp[blockIdx.y];
  const int K = jb.K, N = w * h;
  int bad = 0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int i = lane + 64 * s;
    WidePoint P{0, 0, 0.f, 0.f};
    if (i < K) {
      int p = fp.pos[jb.base + i];
      if (f.validate && (p >= N || (i > 0 && (int)fp.pos[jb.base + i - 1] >= p))) bad |= kStatusMask;
      p = min(p, N - 1);
      P.x = p % w;
      P.y = p / w;
      const int q0 = fp.coef[jb.vb0 + i];
      const int q1 = jb.nv > 1 ? (int)fp.coef[jb.vb1 + i] : 0;
      if (f.validate && (q0 == -128 || q1 == -128)) bad |= kStatusValue;
      P.c0 = coef_value(q0, f.qstep[jb.pl0], f.qrho);
      P.c1 = coef_value(q1, f.qstep[jb.pl1], f.qrho);
    }
    if (i < kWideStagePts) st.p[i] = P;
  }
  if (lane < 2) {
    float a = 0.f;
    if (lane < jb.nv) {
      a = fp.consts[lane ? jb.cidx1 : jb.cidx0];
      if (f.validate && !isfinite(a)) bad |= kStatusValue;
    }
    st.a[lane] = a;
  }
  if (bad) atomicOr(f.status, bad);
  wave_sync();
}

// c + X^T Y for 16 x 16 tiles X, Y in accumulator layout: the k-th product
// of the chain takes register r of both operands, so lane l supplies
// A[l%16][l/16] = X[4(l/16) + r][l%16] and B[l/16][l%16] = Y[4(l/16) + r][l%16].
__device__ __forceinline__ f4 mma_tn(const f4 &x, const f4 &y, f4 c) {
#pragma unroll
  for (int r = 0; r < 4; ++r) c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[r], y[r], c, 0, 0, 0);
  return c;
}

// x^T of a 16 x 16 tile in accumulator layout, through the wave's tile
// buffer (4 scalar LDS writes and one 16-byte read per lane; as a product
// with the identity it took four matrix-core steps in the elimination's
// dependent chain).
__device__ __forceinline__ f4 tile_t(const f4 &x, float *tb, int lo, int hi) {
  wave_sync();  // earlier reads of the buffer done
#pragma unroll
  for (int r = 0; r < 4; ++r) tb[(4 * hi + r) * kTb + lo] = x[r];
  wave_sync();
  return *reinterpret_cast<const f4 *>(tb + lo * kTb + 4 * hi);
}

// Row broadcast kept as a standalone move (see bcast_i).
__device__ __forceinline__ float bcast_pin(float x, int src) {
  int v = bcast_i(__builtin_bit_cast(int, x), src);
  pin_v(v);
  return __builtin_bit_cast(float, v);
}

__device__ __forceinline__ float tab_at(const float *Hc, int byte_off) {
  return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(Hc) + byte_off);
}

// Assemble, factor and solve the bordered system of one block; stage (x, y,
// c) of the K points and a for the evaluation.  Returns false when the pivots
// call for FP64 refinement (the general path refines).  TN: tiles per side
// at most (7: K <= 103; 6: K <= 95; 5: K <= 79; 4: K <= 63: fewer registers).
// (Making the tile count a compile-time constant for the bins of one tile
// count turns the elimination into one straight-line region; the scheduler
// then hoists so much that every part spills hundreds of registers.)
template <int TN>
__device__ __forceinline__ bool wide_solve(const FrameDev &f, const WideJob &jb, int lane, int w, int h,
                                           const float *Hc, WideStage &st) {
  const int K = jb.K, n = K + 1, N = w * h, W1 = w + 1;
  const int NT = (n + 15) >> 4;
  const int lo = lane & 15, hi = lane >> 4;

  // Points (as table byte offsets) and right-hand sides into LDS.
  int bad = 0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int i = lane + 64 * s;
    int x = 0, y = 0;
    float v0 = 0.f, v1 = 0.f;
    if (i < K) {
      const uint16_t *pos = f.fp[blockIdx.y].pos;
      int p = pos[jb.base + i];
      if (f.validate && (p >= N || (i > 0 && (int)pos[jb.base + i - 1] >= p))) bad |= kStatusMask;
      p = min(p, N - 1);
      x = p % w;
      y = p / w;
      const float *vals = f.fp[blockIdx.y].values;
      v0 = vals[jb.vb0 + i];
      if (jb.nv > 1) v1 = vals[jb.vb1 + i];
      if (f.validate && !(isfinite(v0) && isfinite(v1))) bad |= kStatusValue;
    }
    if (i < kWideStagePts) {
      st.xy[i] = (4 * x) | ((4 * y * W1) << 16);
      st.p[i] = WidePoint{x, y, 0.f, 0.f};
      st.rv[0][i] = v0;
      st.rv[1][i] = v1;
    }
  }
  if (bad) atomicOr(f.status, bad);
  wave_sync();

  // Assembly of the tiles (ti <= tj): entry (i, k) is G(x_i, x_k) for i, k
  // < K, 1 in the border row and column, 0 at (K, K), identity past K.  G is
  // the sum of four quarter-scaled compact-table entries: (|dx|, |dy|) and
  // the reflections x_i + x_k + 1, y_i + y_k + 1 folded into [0, w], [0, h].
  f4 T[kNumTilesN<TN>], R[TN];
  const int xcr = 4 * (2 * w - 1), ycr = 4 * (2 * h - 1) * W1, W4 = 4 * W1;
#pragma unroll
  for (int ti = 0; ti < TN; ++ti) {
    if (ti < NT) {
      const i4 rowp = *reinterpret_cast<const i4 *>(&st.xy[16 * ti + 4 * hi]);
#pragma unroll
      for (int tj = ti; tj < TN; ++tj) {
        if (tj < NT) {
          const int k = 16 * tj + lo, ck = st.xy[k];
          const int xk = ck & 0xffff, yk = ck >> 16;
          f4 t;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * ti + 4 * hi + r, ci = rowp[r];
            const int xi = ci & 0xffff, yi = ci >> 16;
            const int dy = (int)__usad((unsigned)yi, (unsigned)yk, 0u);
            const int sy = min(yi + yk + W4, ycr - yi - yk);
            const int dx = (int)__usad((unsigned)xi, (unsigned)xk, 0u);
            const int sx = min(xi + xk + 4, xcr - xi - xk);
            const float g = (tab_at(Hc, dy + dx) + tab_at(Hc, dy + sx)) + (tab_at(Hc, sy + dx) + tab_at(Hc, sy + sx));
            const bool one = (i == K && k < K) || (k == K && i < K) || (i == k && i > K);
            t[r] = (i < K && k < K) ? g : (one ? 1.f : 0.f);
          }
          T[tixn<TN>(ti, tj)] = t;
        }
      }
      const f4 rv = *reinterpret_cast<const f4 *>(&st.rv[lo & 1][16 * ti + 4 * hi]);
      R[ti] = lo < 2 ? rv : f4{0.f, 0.f, 0.f, 0.f};
    }
  }

  // Forward elimination, one diagonal tile p at a time.
  float dmin = 3.0e38f, dmax = 0.f;
#pragma unroll
  for (int p = 0; p < TN; ++p) {
    if (p < NT) {
      // Row lo of A_pp in every lane.
      float e[16];
      {
        const f4 t = T[tixn<TN>(p, p)];
#pragma unroll
        for (int r = 0; r < 4; ++r) st.tb[(4 * hi + r) * kTb + lo] = t[r];
        wave_sync();
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const f4 v = *reinterpret_cast<const f4 *>(st.tb + lo * kTb + 4 * c);
#pragma unroll
          for (int u = 0; u < 4; ++u) e[4 * c + u] = v[u];
        }
        wave_sync();  // read before the next tile is written
      }
      // Row reduction of [A_pp | I] without pivoting: lane lo keeps row lo of
      // the reduced A_pp and columns 4 hi .. 4 hi + 3 of row lo of L^-1; the
      // multiplier of row lo at step j is its own entry j over the pivot.
      f4 lv, ds;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        lv[c] = (lo == 4 * hi + c) ? 1.f : 0.f;
        ds[c] = 1.f;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const float dj = bcast_pin(e[j], j);
        const float rj = __builtin_amdgcn_rcpf(dj);
        if (16 * p + j < K) {
          dmin = fminf(dmin, fabsf(dj));
          dmax = fmaxf(dmax, fabsf(dj));
        }
        if (hi == (j >> 2)) ds[j & 3] = rj;
        const float fm = (lo > j) ? e[j] * rj : 0.f;
#pragma unroll
        for (int k = j + 1; k < 16; ++k) e[k] = fmaf(-fm, bcast_pin(e[k], j), e[k]);
#pragma unroll
        for (int c = 0; c < 4; ++c) lv[c] = fmaf(-fm, bcast_pin(lv[c], j), lv[c]);
      }
      // lv is (L^-1)^T in accumulator layout.  Keep L^-1 itself (for the back
      // substitution) in place of A_pp, and the reciprocal pivots in LDS.
      T[tixn<TN>(p, p)] = tile_t(lv, st.tb, lo, hi);
      if (lo == 0) *reinterpret_cast<f4 *>(&st.dv[16 * p + 4 * hi]) = ds;
      // W_pj = L^-1 A_pj in place of A_pj for the trailing updates.
#pragma unroll
      for (int j = p + 1; j < TN; ++j)
        if (j < NT) T[tixn<TN>(p, j)] = mma_tn(lv, T[tixn<TN>(p, j)], f4{0.f, 0.f, 0.f, 0.f});
      R[p] = mma_tn(lv, R[p], f4{0.f, 0.f, 0.f, 0.f});
      // A_ij -= W_pi^T D^-1 W_pj, r_i -= W_pi^T D^-1 r_p.
#pragma unroll
      for (int i = p + 1; i < TN; ++i) {
        if (i < NT) {
          f4 x;
#pragma unroll
          for (int r = 0; r < 4; ++r) x[r] = -ds[r] * T[tixn<TN>(p, i)][r];
#pragma unroll
          for (int j = i; j < TN; ++j)
            if (j < NT) T[tixn<TN>(i, j)] = mma_tn(x, T[tixn<TN>(p, j)], T[tixn<TN>(i, j)]);
          R[i] = mma_tn(x, R[p], R[i]);
        }
      }
      // W_pj^T kept for the back substitution.
#pragma unroll
      for (int j = p + 1; j < TN; ++j)
        if (j < NT) T[tixn<TN>(p, j)] = tile_t(T[tixn<TN>(p, j)], st.tb, lo, hi);
    }
  }
  const bool need = (f.refine == 2) || (f.refine == 1 && !(dmin >= f.tau * dmax));
  if (__ballot(need)) return false;
  wave_sync();  // reciprocal pivots written

  // Back substitution: x_p = L_p^-T D_p^-1 (r_p - sum_{j > p} W_pj x_j).
#pragma unroll
  for (int p = TN - 1; p >= 0; --p) {
    if (p < NT) {
      f4 y = R[p];
#pragma unroll
      for (int j = p + 1; j < TN; ++j) {
        if (j < NT) {
          f4 wt = T[tixn<TN>(p, j)];
#pragma unroll
          for (int r = 0; r < 4; ++r) wt[r] = -wt[r];
          y = mma_tn(wt, R[j], y);
        }
      }
      const f4 dv = *reinterpret_cast<const f4 *>(&st.dv[16 * p + 4 * hi]);
#pragma unroll
      for (int r = 0; r < 4; ++r) y[r] *= dv[r];
      R[p] = mma_tn(T[tixn<TN>(p, p)], y, f4{0.f, 0.f, 0.f, 0.f});
    }
  }

  // Stage the coefficients (column lo of the solution tiles, lo < 2) and
  // a = x_K; staged points past K keep c = 0.
  bool fin = true;
#pragma unroll
  for (int p = 0; p < TN; ++p) {
    if (p < NT) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int idx = 16 * p + 4 * hi + r;
        const float v = R[p][r];
        if (lo < 2) {
          if (idx < K) {
            if (lo == 0) st.p[idx].c0 = v;
            else st.p[idx].c1 = v;
          }
          if (idx == K) st.a[lo] = v;
          if (idx <= K) fin &= isfinite(v);
        }
      }
    }
  }
  if (__ballot(!fin)) {
    if (lane == 0) atomicOr(f.status, kStatusSolve);
  }
  wave_sync();
  return true;
}

// u = Dh^T (lam .* (Dw[:,X] diag(c) Dh[:,Y]^T)^T) Dw + a over the 32 x 32
// block as 2 x 2 tiles of FP32 16x16x4 MFMA chains (lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; the result D[4(l/16)+r][l%16] is register
// r).  D holds Dw[p][x], Dh[q][y] and lam[q][p], 32 x 32 each, zero-padded,
// row stride kDct32Ld.
__device__ __forceinline__ void wide_eval32(const FrameDev &f, const WideJob &jb, const float *D,
                                            const WideStage &st, int lane, int w, int h, int W) {
  const float *Dw = D, *Dh = D + kDct32Floats, *lam = D + 2 * kDct32Floats;
  const int lo = lane & 15, hi = lane >> 4;
  const int nch = (jb.K + 7) >> 3;
  const PlaneOut po = plane_out(f, blockIdx.y);  // pairs of 4-point chunks (staged points are zero past K)
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
          ao[u][t] = cv * Dw[(16 * t + lo) * kDct32Ld + P.x];  // A[p][i], p = 16 pt + lo
          bo[u][t] = Dh[(16 * t + lo) * kDct32Ld + P.y];       // B[i][q], q = 16 qt + lo
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
            const float a = acc[pt][qt][j] * lam[(16 * qt + lo) * kDct32Ld + p];
            s4 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Dw[p * kDct32Ld + 16 * xt + lo], s4, 0, 0, 0);
          }
        S[qt][xt] = s4;  // S[q = 16 qt + 4 hi + r][x = 16 xt + lo]
      }
    const float av = st.a[v];
    const long long ob = v ? jb.ob1 : jb.ob0;
#pragma unroll
    for (int yt = 0; yt < 2; ++yt)
#pragma unroll
      for (int xt = 0; xt < 2; ++xt) {
        // Taken transposed (u^T = S^T Dh), so that register r is pixel
        // (x = 16 xt + 4 hi + r, y = 16 yt + lo): four consecutive pixels of
        // a block row per lane, one 16-byte store.
        f4 u4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int qt = 0; qt < 2; ++qt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int q = 16 * qt + 4 * hi + j;
            u4 = __builtin_amdgcn_mfma_f32_16x16x4f32(S[qt][xt][j], Dh[q * kDct32Ld + 16 * yt + lo], u4, 0, 0, 0);
          }
        const int y = 16 * yt + lo, x0 = 16 * xt + 4 * hi;
        if (x0 < w && y < h) {
          const float u[4] = {u4[0] + av, u4[1] + av, u4[2] + av, u4[3] + av};
          store_px4(po, (unsigned)(ob + (long long)y * W + x0), u, min(4, w - x0));
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
  const float *Dw = D, *Dh = D + kDct32Floats, *lam = D + 2 * kDct32Floats;
  const int lo = lane & 15, hi = lane >> 4;
  const int nch = (jb.K + 15) >> 4;
  const PlaneOut po = plane_out(f, blockIdx.y);
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
          ao[t][e] = cv * Dw[(16 * t + lo) * kDct32Ld + P.x];
          bo[t][e] = Dh[(16 * t + lo) * kDct32Ld + P.y];
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
            a[e] = acc[pt][qt][e] * lam[(16 * qt + lo) * kDct32Ld + p];
            b[e] = Dw[p * kDct32Ld + 16 * xt + lo];
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
        // Transposed as in wide_eval32: register r is pixel
        // (x = 16 xt + 4 hi + r, y = 16 yt + lo).
        f4 u4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int qt = 0; qt < 2; ++qt) {
          float a[4], b[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int q = 16 * qt + 4 * hi + e;
            a[e] = S[qt][xt][e];
            b[e] = Dh[q * kDct32Ld + 16 * yt + lo];
          }
          u4 = wmma16<EV>(u4, a, b);
        }
        const int y = 16 * yt + lo, x0 = 16 * xt + 4 * hi;
        if (x0 < w && y < h) {
          const float u[4] = {u4[0] + av, u4[1] + av, u4[2] + av, u4[3] + av};
          store_px4(po, (unsigned)(ob + (long long)y * W + x0), u, min(4, w - x0));
        }
      }
  }
}

// Binning: every mask block goes to its shape's queue, into one of 4 bins by
// point count, so that the long solves are handed out first; blocks the wave
// path does not take (K = 0, K = w*h, K > 103, invalid counts) go to the
// general path's lists.
template <bool COEF>
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
  const bool take = COEF ? (K >= 0 && K <= w * h && K <= kWideKMax) : (K >= 1 && K < w * h && K <= kWideKMax);
  if (!take) push_deferred(f, fi, m, K, w, h);
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
// PART 0 takes the whole queue; batched residual decodes launch one part per
// bin, largest systems first: PART 1 bin 0 (7 tiles per side), PART 2 bin 1
// (6), PART 3 bin 2 (5), PART 4 bin 3 (at most 4): the smaller register file
// of the smaller systems lets more waves share a SIMD and hide the latency
// of the elimination's dependent steps.
template <int PART> struct WidePart {
  static constexpr int TN = PART == 2 ? 6 : PART == 3 ? 5 : PART == 4 ? 4 : kTileN;
  static constexpr int WMIN = TN >= 7 ? 2 : TN == 6 ? 3 : 4;  // waves per SIMD asked for
};
template <int WAVES, bool COEF, int PART>
__global__ __launch_bounds__(64 * WAVES)
__attribute__((amdgpu_waves_per_eu(COEF ? 2 : WidePart<PART>::WMIN, COEF ? 3 : 8))) void k_wide(FrameDev f) {
  constexpr int TN = WidePart<PART>::TN;
  static_assert(16 * 4 >= kBinK2 && 16 * 5 >= kBinK1 && 16 * 6 >= kBinK0, "each bin fits its part's tiles");
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
  // Queue position of this wave's block: workgroups start in index order, so
  // the first ones take the large-K blocks at the front of the queue.
  const int fi = blockIdx.y;
  const int32_t *bp = f.fp[fi].block_ptr;
  const int *cnt = f.counters + kQueueCounters + 4 * (kMaxShapes * fi + qi);
  const int n0 = cnt[0], n1 = cnt[1], n2 = cnt[2], n3 = cnt[3];
  const int p_lo = PART == 2 ? n0 : PART == 3 ? n0 + n1 : PART == 4 ? n0 + n1 + n2 : 0;
  const int p_hi = PART == 1 ? n0 : PART == 2 ? n0 + n1 : PART == 3 ? n0 + n1 + n2 : n0 + n1 + n2 + n3;
  const int p0 = p_lo + (wg - Q.first_wg) * WAVES;  // the workgroup's first position
  if (p0 >= p_hi || p0 >= Q.count) return;          // uniform: no wave of this workgroup has a block
  {  // stored-coefficient decodes need the evaluation's matrices only
    const int n4 = ((COEF ? 0 : S.jt_floats) + 3 * kDct32Floats) >> 2;
    const f4 *src = reinterpret_cast<const f4 *>(f.tab32 + S.fast + (COEF ? S.jt_floats : 0));
    f4 *dst = reinterpret_cast<f4 *>(tabs);
    for (int i = tid; i < n4; i += 64 * WAVES) dst[i] = src[i];
  }
  __syncthreads();  // the only workgroup barrier: waves are independent from here on
  const int p = p0 + wv;
  if (p >= p_hi || p >= Q.count || n0 + n1 > Q.count || n2 + n3 > Q.count) return;
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
  const int K = jb.K;  // binned: 1 <= K <= min(w*h - 1, kWideKMax) (COEF: 0 <= K <= ..)
  WideStage &st = stage[wv];
  if constexpr (COEF) {
    jb.pl0 = G.vplane[0];
    jb.pl1 = G.vplane[G.nv > 1 ? 1 : 0];
    jb.cidx0 = G.cbase[0] + bl;
    jb.cidx1 = G.cbase[1] + bl;
    wide_coef_stage(f, jb, lane, w, h, st);
  } else {
    const bool solved = wide_solve<TN>(f, jb, lane, w, h, tabs, st);
    if (!solved) {
      if (lane == 0) push_deferred(f, fi, m, K, w, h);
      return;
    }
  }
  const float *D = tabs + (COEF ? 0 : S.jt_floats);
  switch (f.eval) {
    case 1: wide_eval16<1>(f, jb, D, st, lane, w, h, G.W); break;
    case 2: wide_eval16<2>(f, jb, D, st, lane, w, h, G.W); break;
    case 3: wide_eval16<3>(f, jb, D, st, lane, w, h, G.W); break;
    default: wide_eval32(f, jb, D, st, lane, w, h, G.W); break;
  }
}

// One part of a batched residual decode (the workgroup size is the launch choice).
template <int PART>
hipError_t launch_wide_part(const FrameDev &f, dim3 grid, size_t lds, hipStream_t st) {
  switch (f.ipw) {
    case 1: hipLaunchKernelGGL((k_wide<1, false, PART>), grid, dim3(64), lds, st, f); break;
    case 2: hipLaunchKernelGGL((k_wide<2, false, PART>), grid, dim3(128), lds, st, f); break;
    case 4: hipLaunchKernelGGL((k_wide<4, false, PART>), grid, dim3(256), lds, st, f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_wide(const FrameDev &f, hipStream_t stream, const WideFork *fork) {
  if (f.n_items == 0) return hipSuccess;
  const dim3 bgrid((f.n_items + 255) / 256, f.nframes), grid(f.fast_wgs, f.nframes);
  const size_t lds = sizeof(float) * (size_t)f.fast_lds;
  if (f.coef) {
    hipLaunchKernelGGL(k_bin<true>, bgrid, dim3(256), 0, stream, f);
    switch (f.ipw) {
      case 1: hipLaunchKernelGGL((k_wide<1, true, 0>), grid, dim3(64), lds, stream, f); break;
      case 2: hipLaunchKernelGGL((k_wide<2, true, 0>), grid, dim3(128), lds, stream, f); break;
      case 4: hipLaunchKernelGGL((k_wide<4, true, 0>), grid, dim3(256), lds, stream, f); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    hipLaunchKernelGGL(k_bin<false>, bgrid, dim3(256), 0, stream, f);
    if (f.nframes > 1) {
      // batches: one launch per bin, the large-K bins first (longest solves
      // start first).  With a fork the parts run side by side, so the tail of
      // one (the few K >= 96 blocks at 2 waves per SIMD) overlaps the others:
      // part 1 on one stream, parts 2 and then 3 on another, part 4 on the
      // caller's (all four at once delays part 1, the longest).  A single
      // frame keeps one launch: with few blocks more launches would only add
      // their latency.
      hipStream_t st[kWideAux] = {stream, stream};
      hipError_t e = hipSuccess;
      if (fork) {
        e = hipEventRecord(fork->fork, stream);
        for (int i = 0; i < kWideAux && e == hipSuccess; ++i) {
          e = hipStreamWaitEvent(fork->aux[i], fork->fork, 0);
          st[i] = fork->aux[i];
        }
        if (e != hipSuccess) return e;
      }
      e = launch_wide_part<1>(f, grid, lds, st[0]);
      if (e == hipSuccess) e = launch_wide_part<2>(f, grid, lds, st[1]);
      if (e == hipSuccess) e = launch_wide_part<3>(f, grid, lds, st[1]);
      if (e == hipSuccess) e = launch_wide_part<4>(f, grid, lds, stream);
      if (fork) {  // join (also after a failed launch: the caller's stream waits for what was queued)
        for (int i = 0; i < kWideAux; ++i) {
          const hipError_t r = hipEventRecord(fork->join[i], fork->aux[i]);
          const hipError_t w = r == hipSuccess ? hipStreamWaitEvent(stream, fork->join[i], 0) : r;
          if (e == hipSuccess) e = w;
        }
      }
      if (e != hipSuccess) return e;
    } else {
      switch (f.ipw) {
        case 1: hipLaunchKernelGGL((k_wide<1, false, 0>), grid, dim3(64), lds, stream, f); break;
        case 2: hipLaunchKernelGGL((k_wide<2, false, 0>), grid, dim3(128), lds, stream, f); break;
        case 4: hipLaunchKernelGGL((k_wide<4, false, 0>), grid, dim3(256), lds, stream, f); break;
        default: return hipErrorInvalidValue;
      }
    }
  }
  return hipGetLastError();
}

}  // namespace pdi
