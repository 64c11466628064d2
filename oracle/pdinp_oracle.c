/*
 * FP64 CPU oracle for block-based pseudodifferential residual inpainting
 * (Andris, Peter, Kaja Mohideen, Weickert, Hoffmann: "Inpainting-based Video
 * Compression in FullHD", SSVM 2021, Sec. 2.1-2.2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can check the GPU library against a plain,
 * slow, obviously correct implementation.  It shares no code, header or
 * table with the GPU library.
 *
 * Two independent routes to the same result u of one block:
 *
 *  (1) orc_block_direct: the plain definition.  Eq. (1) of Sec. 2.1,
 *        M (u - f) - (I - M) A u = 0,
 *      on a w x h block treated as an independent image with reflecting
 *      (mirrored) boundary conditions (Sec. 2.2, last paragraph), with the
 *      harmonic operator A = -L (Sec. 2.1 and Sec. 2.3), L the 5-point
 *      Laplacian, or its square A = L^2 (s = 2).  The mask rows fix u = f,
 *      so the unknowns solve A_UU u_U = -A_UK f_K, an SPD banded system,
 *      solved here by banded Cholesky.
 *
 *  (2) orc_block_green: the Green's-function route of Sec. 2.2.
 *      u_k = sum_i m_i c_i (g_i)_k + a  (Eq. 2), where the Green's functions
 *      are the columns of G, the pseudo-inverse of A; G is diagonalised by
 *      the DCT-II, G = C^-1 diag(lambda) C (Eq. 4), and the eigenvalues
 *      lambda fully define the operator.  c and a solve a dense
 *      (K+1) x (K+1) system (Sec. 2.2, after Eq. 2): interpolation at the K
 *      mask points plus sum_i c_i = 0, the latter forced by A u = M c and
 *      1^T A = 0.  The system is solved by LU with partial pivoting.
 *      Entries of G are read from the Toeplitz-plus-Hankel table of
 *      Sec. 2.2: with mirrored boundaries G depends on x - y and x + y.
 *
 * Beside them: orc_decode_coef, the decoder of stored coefficients (Eq. 2
 * summed directly from dequantised codes), and orc_encode_coef, the encoder
 * side (c and a by route (2), dead-zone quantisation of c; Sec. 2.2-2.3).
 *
 * Readings where the paper is silent: K = 0 gives u = 0 on the block; the
 * eigenvalues are those of the discrete 5-point operator (op 0) unless the
 * continuous symbol is asked for (op 1); lambda = mu^(-s) with lambda_00 = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* (1) Plain definition: Eq. (1) with A = (-L)^s, s in {1, 2}.        */
/* ------------------------------------------------------------------ */

/* Row `k` of the graph Laplacian -L of the w x h block (reflecting
 * boundaries: an out-of-block neighbour mirrors the pixel itself and adds
 * nothing).  Writes up to 5 (index, weight) pairs, returns the count. */
static int neg_laplacian_row(int w, int h, int k, int *idx, double *wt)
{
    int x = k % w, y = k / w, n = 0;
    double diag = 0.0;
    if (x > 0)     { idx[n] = k - 1; wt[n] = -1.0; n++; diag += 1.0; }
    if (x < w - 1) { idx[n] = k + 1; wt[n] = -1.0; n++; diag += 1.0; }
    if (y > 0)     { idx[n] = k - w; wt[n] = -1.0; n++; diag += 1.0; }
    if (y < h - 1) { idx[n] = k + w; wt[n] = -1.0; n++; diag += 1.0; }
    idx[n] = k; wt[n] = diag; n++;
    return n;
}

/* Sparse row k of A = (-L)^s: up to 25 (index, weight) terms, duplicates
 * allowed (they add up).  Returns the count. */
static int operator_row(int w, int h, int s, int k, int *idx, double *wt)
{
    int i1[5], i2[5], n1, n2, a, b, n = 0;
    double w1[5], w2[5];
    n1 = neg_laplacian_row(w, h, k, i1, w1);
    if (s == 1) {
        for (a = 0; a < n1; a++) { idx[a] = i1[a]; wt[a] = w1[a]; }
        return n1;
    }
    /* s == 2: row k of (-L)(-L) = sum_j (-L)_kj row j of (-L). */
    for (a = 0; a < n1; a++) {
        n2 = neg_laplacian_row(w, h, i1[a], i2, w2);
        for (b = 0; b < n2; b++) { idx[n] = i2[b]; wt[n] = w1[a] * w2[b]; n++; }
    }
    return n;
}

/* Banded Cholesky solve of the SPD system B x = rhs, B stored by rows as
 * band[i*(bw+1) + (i-j)] for 0 <= i-j <= bw (lower half).  Returns 0 on
 * success, -1 on a non-positive pivot. */
static int banded_cholesky_solve(int n, int bw, double *band, double *rhs)
{
    int i, j, k, W = bw + 1;
    for (j = 0; j < n; j++) {
        double d = band[j * W];
        int kmin = j - bw < 0 ? 0 : j - bw;
        for (k = kmin; k < j; k++) { double l = band[j * W + (j - k)]; d -= l * l; }
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        band[j * W] = d;
        for (i = j + 1; i < n && i <= j + bw; i++) {
            double v = band[i * W + (i - j)];
            int kmin2 = i - bw < 0 ? 0 : i - bw;
            for (k = (kmin2 > kmin ? kmin2 : kmin); k < j; k++)
                v -= band[i * W + (i - k)] * band[j * W + (j - k)];
            band[i * W + (i - j)] = v / d;
        }
    }
    for (i = 0; i < n; i++) {                     /* L y = rhs */
        double v = rhs[i];
        int kmin = i - bw < 0 ? 0 : i - bw;
        for (k = kmin; k < i; k++) v -= band[i * W + (i - k)] * rhs[k];
        rhs[i] = v / band[i * W];
    }
    for (i = n - 1; i >= 0; i--) {                /* L^T x = y */
        double v = rhs[i];
        for (k = i + 1; k < n && k <= i + bw; k++) v -= band[k * W + (k - i)] * rhs[k];
        rhs[i] = v / band[i * W];
    }
    return 0;
}

/* Solve Eq. (1) on one w x h block with mask positions pos[0..K-1]
 * (in-block index y*w + x, distinct) and values r; u receives w*h values.
 * Returns 0, or -1 on bad arguments / failed factorisation. */
int orc_block_direct(int w, int h, int s, int K, const uint16_t *pos,
                     const double *r, double *u)
{
    int N = w * h, nU = 0, i, j, bw, rc = 0, nt, ridx[25];
    int *is_mask, *uidx, *uof;
    double *band, *rhs, rwt[25];
    if (w <= 0 || h <= 0 || K < 0 || K > N || (s != 1 && s != 2)) return -1;
    if (K == 0) { for (i = 0; i < N; i++) u[i] = 0.0; return 0; }
    is_mask = (int *)calloc((size_t)N, sizeof(int));
    uidx = (int *)malloc(sizeof(int) * (size_t)N);
    uof = (int *)malloc(sizeof(int) * (size_t)N);
    for (i = 0; i < K; i++) {
        if (pos[i] >= N || is_mask[pos[i]]) { rc = -1; goto done; }
        is_mask[pos[i]] = 1 + i;
    }
    for (i = 0; i < N; i++) {
        if (is_mask[i]) { u[i] = r[is_mask[i] - 1]; uof[i] = -1; }
        else { uof[i] = nU; uidx[nU++] = i; }
    }
    if (nU == 0) goto done;
    bw = s * w;
    band = (double *)calloc((size_t)nU * (size_t)(bw + 1), sizeof(double));
    rhs = (double *)calloc((size_t)nU, sizeof(double));
    /* Unknown rows of Eq. (1): (A u)_k = 0; known values move to the right. */
    for (i = 0; i < nU; i++) {
        nt = operator_row(w, h, s, uidx[i], ridx, rwt);
        for (j = 0; j < nt; j++) {
            int col = ridx[j];
            if (is_mask[col]) rhs[i] -= rwt[j] * r[is_mask[col] - 1];
            else if (uof[col] <= i) band[i * (bw + 1) + (i - uof[col])] += rwt[j];
        }
    }
    if (banded_cholesky_solve(nU, bw, band, rhs) != 0) rc = -1;
    else for (i = 0; i < nU; i++) u[uidx[i]] = rhs[i];
    free(band);
    free(rhs);
done:
    free(is_mask); free(uidx); free(uof);
    return rc;
}

/* ------------------------------------------------------------------ */
/* (2) Green's-function route: Eqs. (2)-(4).                          */
/* ------------------------------------------------------------------ */

/* Eigenvalues of the Green's functions for a w x h block, lam[q*w + p].
 * mu_pq are the eigenvalues of A under the DCT-II (Eq. 4): op 0, the
 * 5-point operator, mu = 4 sin^2(pi p / 2w) + 4 sin^2(pi q / 2h); op 1, the
 * continuous symbol mu = pi^2 (p^2/w^2 + q^2/h^2).  lam = mu^-s, and
 * lam_00 = 0 because G is the pseudo-inverse of A. */
void orc_eigenvalues(int w, int h, int op, double s, double *lam)
{
    int p, q;
    for (q = 0; q < h; q++)
        for (p = 0; p < w; p++) {
            double mu;
            if (op == 1)
                mu = ORC_PI * ORC_PI * ((double)p * p / ((double)w * w) + (double)q * q / ((double)h * h));
            else {
                double sp = sin(ORC_PI * p / (2.0 * w)), sq = sin(ORC_PI * q / (2.0 * h));
                mu = 4.0 * sp * sp + 4.0 * sq * sq;
            }
            lam[q * w + p] = (p == 0 && q == 0) ? 0.0 : pow(mu, -s);
        }
}

/* Toeplitz-plus-Hankel table of G.  With the orthonormal DCT-II basis
 * phi_p(x) = sqrt(om_p) cos(pi p (x + 1/2) / n), om_0 = 1/n, om_p = 2/n,
 * the product phi_p(x) phi_p(x') is (om_p / 2) [cos(pi p (x - x')/n) +
 * cos(pi p (x + x' + 1)/n)].  Hence G(x, x') is a quarter of the sum of
 * Htab over the four index pairs built from |x - x'| and x + x' + 1 per
 * axis, where
 *   Htab[beta*(w+1) + alpha] = sum_pq lam_pq om_p om_q cos(pi p alpha / w) cos(pi q beta / h)
 * for alpha in [0, w], beta in [0, h] (x + x' + 1 is reflected into
 * [0, n] by the period 2n of the cosines). */
void orc_green_table(int w, int h, const double *lam, double *Htab)
{
    int alpha, beta, p, q;
    for (beta = 0; beta <= h; beta++)
        for (alpha = 0; alpha <= w; alpha++) {
            double acc = 0.0;
            for (q = 0; q < h; q++) {
                double oq = (q == 0 ? 1.0 : 2.0) / h;
                double cq = cos(ORC_PI * q * beta / h);
                for (p = 0; p < w; p++) {
                    double op_ = (p == 0 ? 1.0 : 2.0) / w;
                    acc += lam[q * w + p] * op_ * oq * cos(ORC_PI * p * alpha / w) * cq;
                }
            }
            Htab[beta * (w + 1) + alpha] = acc;
        }
}

static int reflect(int v, int n) { return v <= n ? v : 2 * n - v; }

/* G(x_a, x_b) for pixels (xa, ya), (xb, yb) of a w x h block. */
double orc_green(int w, int h, const double *Htab, int xa, int ya, int xb, int yb)
{
    int dx = abs(xa - xb), dy = abs(ya - yb);
    int sx = reflect(xa + xb + 1, w), sy = reflect(ya + yb + 1, h);
    int W1 = w + 1;
    return 0.25 * (Htab[dy * W1 + dx] + Htab[sy * W1 + dx] +
                   Htab[dy * W1 + sx] + Htab[sy * W1 + sx]);
}

/* Dense LU with partial pivoting; solves M X = B in place for nrhs right
 * hand sides stored column-major in B (n x nrhs).  Returns -1 if singular. */
static int lu_solve(int n, double *Mx, int nrhs, double *B)
{
    int i, j, k, c;
    for (k = 0; k < n; k++) {
        int piv = k;
        double best = fabs(Mx[k * n + k]);
        for (i = k + 1; i < n; i++)
            if (fabs(Mx[i * n + k]) > best) { best = fabs(Mx[i * n + k]); piv = i; }
        if (best == 0.0) return -1;
        if (piv != k) {
            for (j = 0; j < n; j++) { double t = Mx[k * n + j]; Mx[k * n + j] = Mx[piv * n + j]; Mx[piv * n + j] = t; }
            for (c = 0; c < nrhs; c++) { double t = B[c * n + k]; B[c * n + k] = B[c * n + piv]; B[c * n + piv] = t; }
        }
        for (i = k + 1; i < n; i++) {
            double f = Mx[i * n + k] / Mx[k * n + k];
            if (f == 0.0) continue;
            for (j = k; j < n; j++) Mx[i * n + j] -= f * Mx[k * n + j];
            for (c = 0; c < nrhs; c++) B[c * n + i] -= f * B[c * n + k];
        }
    }
    for (c = 0; c < nrhs; c++)
        for (i = n - 1; i >= 0; i--) {
            double v = B[c * n + i];
            for (j = i + 1; j < n; j++) v -= Mx[i * n + j] * B[c * n + j];
            B[c * n + i] = v / Mx[i * n + i];
        }
    return 0;
}

/* Green's route on one block for nrhs value sets sharing one mask.
 * r is [nrhs][K]; c receives [nrhs][K], a [nrhs], u [nrhs][w*h].
 * Htab must come from orc_green_table for this shape.  Returns 0 / -1. */
int orc_block_green_tab(int w, int h, const double *Htab, int K, const uint16_t *pos,
                        int nrhs, const double *r, double *c, double *a, double *u)
{
    int N = w * h, n = K + 1, i, j, t, rc = 0;
    int *xs, *ys;
    double *Mx, *B;
    if (K < 0 || K > N || nrhs < 1) return -1;
    if (K == 0) {
        for (t = 0; t < nrhs; t++) { a[t] = 0.0; for (i = 0; i < N; i++) u[t * N + i] = 0.0; }
        return 0;
    }
    xs = (int *)malloc(sizeof(int) * (size_t)K);
    ys = (int *)malloc(sizeof(int) * (size_t)K);
    Mx = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    B = (double *)malloc(sizeof(double) * (size_t)n * (size_t)nrhs);
    for (i = 0; i < K; i++) {
        if (pos[i] >= N) { rc = -1; goto done; }
        xs[i] = pos[i] % w; ys[i] = pos[i] / w;
    }
    /* (K+1) system [G_K 1; 1^T 0] [c; a] = [r; 0]. */
    for (i = 0; i < K; i++) {
        for (j = 0; j < K; j++) Mx[i * n + j] = orc_green(w, h, Htab, xs[i], ys[i], xs[j], ys[j]);
        Mx[i * n + K] = 1.0;
        Mx[K * n + i] = 1.0;
    }
    Mx[K * n + K] = 0.0;
    for (t = 0; t < nrhs; t++) {
        for (i = 0; i < K; i++) B[t * n + i] = r[t * K + i];
        B[t * n + K] = 0.0;
    }
    if (lu_solve(n, Mx, nrhs, B) != 0) { rc = -1; goto done; }
    /* Eq. (2): u_k = sum_i c_i (g_i)_k + a for every pixel k of the block. */
    for (t = 0; t < nrhs; t++) {
        for (i = 0; i < K; i++) c[t * K + i] = B[t * n + i];
        a[t] = B[t * n + K];
        for (j = 0; j < N; j++) {
            int xk = j % w, yk = j / w;
            double acc = 0.0;
            for (i = 0; i < K; i++) acc += c[t * K + i] * orc_green(w, h, Htab, xk, yk, xs[i], ys[i]);
            u[t * N + j] = acc + a[t];
        }
    }
done:
    free(xs); free(ys); free(Mx); free(B);
    return rc;
}

int orc_block_green(int w, int h, int op, double s, int K, const uint16_t *pos,
                    int nrhs, const double *r, double *c, double *a, double *u)
{
    double *lam = (double *)malloc(sizeof(double) * (size_t)w * (size_t)h);
    double *Htab = (double *)malloc(sizeof(double) * (size_t)(w + 1) * (size_t)(h + 1));
    int rc;
    orc_eigenvalues(w, h, op, s, lam);
    orc_green_table(w, h, lam, Htab);
    rc = orc_block_green_tab(w, h, Htab, K, pos, nrhs, r, c, a, u);
    free(lam); free(Htab);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Whole frame: blocks independent (Sec. 2.2), planes per Sec. 2.3.   */
/* ------------------------------------------------------------------ */

typedef struct {
    int m;            /* mask-block index */
    int plane[2];     /* value planes (1 or 2) */
    int nplanes;
    int x0, y0, w, h, pw;
    long long vbase[2];
} orc_item;

/* Decode every block of a frame.
 * fmt 0: one W x H plane; fmt 1: 4:2:0, planes Y (W x H), Cb, Cr
 * (ceil(W/2) x ceil(H/2)).  Mask blocks: Y blocks, then chroma blocks once
 * (chroma_shared) or Cb then Cr, raster order inside each plane.
 * method 0 = plain definition (s must be 1 or 2, op 0), 1 = Green's route.
 * out receives all planes, row-major, concatenated.  nthreads <= 0 keeps the
 * OpenMP default.  Returns 0, or -1 if any block failed. */
int orc_decode(int width, int height, int fmt, int b, const int32_t *block_ptr,
               const uint16_t *pos, const float *values, int chroma_shared,
               int method, int op, double s, double *out, int nthreads)
{
    int PW[3], PH[3], np_, g, ngroups, mp[3], vp[3][2], nv[3];
    long long poff[3], nnz;
    int nitems = 0, cap, chroma_first = -1, m = 0, err = 0, it;
    orc_item *items;
    if (fmt == 0) { np_ = 1; PW[0] = width; PH[0] = height; }
    else { np_ = 3; PW[0] = width; PH[0] = height;
           PW[1] = PW[2] = (width + 1) / 2; PH[1] = PH[2] = (height + 1) / 2; }
    poff[0] = 0;
    for (g = 1; g < np_; g++) poff[g] = poff[g - 1] + (long long)PW[g - 1] * PH[g - 1];
    if (fmt == 0) { ngroups = 1; mp[0] = 0; vp[0][0] = 0; nv[0] = 1; }
    else if (chroma_shared) { ngroups = 2; mp[0] = 0; vp[0][0] = 0; nv[0] = 1;
                              mp[1] = 1; vp[1][0] = 1; vp[1][1] = 2; nv[1] = 2; }
    else { ngroups = 3; for (g = 0; g < 3; g++) { mp[g] = g; vp[g][0] = g; nv[g] = 1; } }
    cap = 0;
    for (g = 0; g < ngroups; g++)
        cap += ((PW[mp[g]] + b - 1) / b) * ((PH[mp[g]] + b - 1) / b);
    items = (orc_item *)malloc(sizeof(orc_item) * (size_t)cap);
    for (g = 0; g < ngroups; g++) {
        int W = PW[mp[g]], H = PH[mp[g]], bx, by;
        if (mp[g] == 1) chroma_first = m;
        for (by = 0; by < (H + b - 1) / b; by++)
            for (bx = 0; bx < (W + b - 1) / b; bx++) {
                orc_item *I = &items[nitems++];
                int k;
                I->m = m; I->x0 = bx * b; I->y0 = by * b;
                I->w = W - I->x0 < b ? W - I->x0 : b;
                I->h = H - I->y0 < b ? H - I->y0 : b;
                I->pw = W; I->nplanes = nv[g];
                for (k = 0; k < nv[g]; k++) I->plane[k] = vp[g][k];
                m++;
            }
    }
    nnz = block_ptr[m];
    for (it = 0; it < nitems; it++) {
        orc_item *I = &items[it];
        int k;
        for (k = 0; k < I->nplanes; k++) {
            if (I->plane[k] == 2 && chroma_shared)
                I->vbase[k] = nnz + (block_ptr[I->m] - block_ptr[chroma_first]);
            else
                I->vbase[k] = block_ptr[I->m];
        }
    }
    /* Green's route: one table per distinct block shape (at most 4 per plane). */
    int nshape = 0, shw[16], shh[16];
    double *shtab[16];
    if (method != 0) {
        for (it = 0; it < nitems; it++) {
            int k, found = 0;
            for (k = 0; k < nshape; k++)
                if (shw[k] == items[it].w && shh[k] == items[it].h) found = 1;
            if (!found && nshape < 16) {
                double *lam = (double *)malloc(sizeof(double) * (size_t)items[it].w * items[it].h);
                shw[nshape] = items[it].w; shh[nshape] = items[it].h;
                shtab[nshape] = (double *)malloc(sizeof(double) * (size_t)(items[it].w + 1) * (items[it].h + 1));
                orc_eigenvalues(items[it].w, items[it].h, op, s, lam);
                orc_green_table(items[it].w, items[it].h, lam, shtab[nshape]);
                free(lam);
                nshape++;
            }
        }
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(|:err)
#endif
    for (it = 0; it < nitems; it++) {
        orc_item *I = &items[it];
        int K = block_ptr[I->m + 1] - block_ptr[I->m];
        int N = I->w * I->h, k, t, j;
        const uint16_t *ps = pos + block_ptr[I->m];
        double *r = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1) * 2);
        double *u = (double *)malloc(sizeof(double) * (size_t)N * 2);
        double *c = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1) * 2);
        double a[2];
        for (k = 0; k < I->nplanes; k++)
            for (j = 0; j < K; j++) r[k * K + j] = (double)values[I->vbase[k] + j];
        if (method == 0) {
            for (k = 0; k < I->nplanes; k++)
                err |= (orc_block_direct(I->w, I->h, (int)s, K, ps, r + k * K, u + k * N) != 0);
        } else {
            const double *tab = 0;
            for (k = 0; k < nshape; k++)
                if (shw[k] == I->w && shh[k] == I->h) tab = shtab[k];
            err |= (tab == 0 || orc_block_green_tab(I->w, I->h, tab, K, ps, I->nplanes, r, c, a, u) != 0);
        }
        for (k = 0; k < I->nplanes; k++) {
            double *dst = out + poff[I->plane[k]];
            for (t = 0; t < I->h; t++)
                for (j = 0; j < I->w; j++)
                    dst[(long long)(I->y0 + t) * I->pw + I->x0 + j] = u[k * N + t * I->w + j];
        }
        free(r); free(u); free(c);
    }
    for (it = 0; it < nshape; it++) free(shtab[it]);
    free(items);
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* (3) The decoder of stored coefficients: when the encoder keeps c   */
/*     and a of every block (Sec. 2.2, last paragraph), the decoder   */
/*     only evaluates Eq. (2).  The coefficients are stored as codes  */
/*     in [-127, 127] of a uniform quantiser with a dead zone around  */
/*     zero, so that zero comes back as zero (Sec. 2.3).              */
/* ------------------------------------------------------------------ */

/* Reconstruction of one code: 0 for q = 0, else sign(q) (|q| + rho) step.
 * rho in [0, 1) places the value inside the quantiser interval (0: its
 * edge nearer zero, 0.5: its middle); step is the plane's step. */
double orc_dequant(int q, double step, double rho)
{
    if (q == 0) return 0.0;
    return (q > 0 ? 1.0 : -1.0) * ((double)abs(q) + rho) * step;
}

/* Decode every block of a frame from stored coefficients.  Geometry, mask
 * layout and chroma sharing as for orc_decode; coef[] is laid out like the
 * values of orc_decode (one code per mask point and value plane); consts[]
 * holds a for every block of every plane: the Y blocks, then Cb, then Cr,
 * raster order.  steps[plane] is the quantiser step of the plane.  Per
 * block, u_k = sum_i c_i G(x_k, x_i) + a over all pixels k (Eq. 2), G
 * from the table of orc_green_table, summed directly.  K = 0 gives u = a.
 * Returns 0, or -1 on a position outside its block. */
int orc_decode_coef(int width, int height, int fmt, int b, const int32_t *block_ptr,
                    const uint16_t *pos, const int8_t *coef, int chroma_shared,
                    const float *consts, const double *steps, double rho,
                    int op, double s, double *out, int nthreads)
{
    int PW[3], PH[3], NB[3], np_, g, ngroups, mp[3], vp[3][2], nv[3];
    long long poff[3], cbase[3], nnz;
    int nitems = 0, cap, chroma_first = -1, m = 0, err = 0, it, k;
    int nshape = 0, shw[16], shh[16];
    double *shtab[16];
    orc_item *items;
    int *pblock;
    if (fmt == 0) { np_ = 1; PW[0] = width; PH[0] = height; }
    else { np_ = 3; PW[0] = width; PH[0] = height;
           PW[1] = PW[2] = (width + 1) / 2; PH[1] = PH[2] = (height + 1) / 2; }
    poff[0] = 0;
    cbase[0] = 0;
    for (g = 0; g < np_; g++) NB[g] = ((PW[g] + b - 1) / b) * ((PH[g] + b - 1) / b);
    for (g = 1; g < np_; g++) {
        poff[g] = poff[g - 1] + (long long)PW[g - 1] * PH[g - 1];
        cbase[g] = cbase[g - 1] + NB[g - 1];
    }
    if (fmt == 0) { ngroups = 1; mp[0] = 0; vp[0][0] = 0; nv[0] = 1; }
    else if (chroma_shared) { ngroups = 2; mp[0] = 0; vp[0][0] = 0; nv[0] = 1;
                              mp[1] = 1; vp[1][0] = 1; vp[1][1] = 2; nv[1] = 2; }
    else { ngroups = 3; for (g = 0; g < 3; g++) { mp[g] = g; vp[g][0] = g; nv[g] = 1; } }
    cap = 0;
    for (g = 0; g < ngroups; g++) cap += NB[mp[g]];
    items = (orc_item *)malloc(sizeof(orc_item) * (size_t)cap);
    pblock = (int *)malloc(sizeof(int) * (size_t)cap);  /* block index inside its plane */
    for (g = 0; g < ngroups; g++) {
        int W = PW[mp[g]], H = PH[mp[g]], bx, by;
        if (mp[g] == 1) chroma_first = m;
        for (by = 0; by < (H + b - 1) / b; by++)
            for (bx = 0; bx < (W + b - 1) / b; bx++) {
                orc_item *I = &items[nitems];
                pblock[nitems++] = by * ((W + b - 1) / b) + bx;
                I->m = m; I->x0 = bx * b; I->y0 = by * b;
                I->w = W - I->x0 < b ? W - I->x0 : b;
                I->h = H - I->y0 < b ? H - I->y0 : b;
                I->pw = W; I->nplanes = nv[g];
                for (k = 0; k < nv[g]; k++) I->plane[k] = vp[g][k];
                m++;
            }
    }
    nnz = block_ptr[m];
    for (it = 0; it < nitems; it++) {
        orc_item *I = &items[it];
        for (k = 0; k < I->nplanes; k++) {
            if (I->plane[k] == 2 && chroma_shared)
                I->vbase[k] = nnz + (block_ptr[I->m] - block_ptr[chroma_first]);
            else
                I->vbase[k] = block_ptr[I->m];
        }
        for (k = 0; k < nshape; k++)
            if (shw[k] == I->w && shh[k] == I->h) break;
        if (k == nshape && nshape < 16) {
            double *lam = (double *)malloc(sizeof(double) * (size_t)I->w * I->h);
            shw[nshape] = I->w; shh[nshape] = I->h;
            shtab[nshape] = (double *)malloc(sizeof(double) * (size_t)(I->w + 1) * (I->h + 1));
            orc_eigenvalues(I->w, I->h, op, s, lam);
            orc_green_table(I->w, I->h, lam, shtab[nshape]);
            free(lam);
            nshape++;
        }
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(|:err)
#endif
    for (it = 0; it < nitems; it++) {
        orc_item *I = &items[it];
        int K = block_ptr[I->m + 1] - block_ptr[I->m];
        const uint16_t *ps = pos + block_ptr[I->m];
        const double *tab = 0;
        int t, i, j, kk;
        for (kk = 0; kk < nshape; kk++)
            if (shw[kk] == I->w && shh[kk] == I->h) tab = shtab[kk];
        if (tab == 0) { err |= 1; continue; }
        for (i = 0; i < K; i++)
            if (ps[i] >= I->w * I->h) err |= 1;
        if (err) continue;
        for (kk = 0; kk < I->nplanes; kk++) {
            int pl = I->plane[kk];
            double a = (double)consts[cbase[pl] + pblock[it]];
            double *dst = out + poff[pl];
            for (t = 0; t < I->h; t++)
                for (j = 0; j < I->w; j++) {
                    double acc = 0.0;
                    for (i = 0; i < K; i++) {
                        double c = orc_dequant(coef[I->vbase[kk] + i], steps[pl], rho);
                        acc += c * orc_green(I->w, I->h, tab, j, t, ps[i] % I->w, ps[i] / I->w);
                    }
                    dst[(long long)(I->y0 + t) * I->pw + I->x0 + j] = acc + a;
                }
        }
    }
    for (it = 0; it < nshape; it++) free(shtab[it]);
    free(items);
    free(pblock);
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* (4) The encoder side of that split: per block, c and a from the    */
/*     bordered system of Sec. 2.2 (the values at the mask points as  */
/*     right-hand side), c mapped to codes by dead-zone uniform       */
/*     quantisation (Sec. 2.3), a kept.                               */
/* ------------------------------------------------------------------ */

/* Code of one coefficient: the interval [k step, (k+1) step) of |c| gives
 * k, capped at 127, with the sign of c; |c| < step gives 0 (the dead zone
 * around zero, so that zero coefficients stay zero).  orc_dequant maps a
 * code back into its interval. */
int orc_quant(double c, double step)
{
    double k = floor(fabs(c) / step);
    if (k > 127.0) k = 127.0;
    return c < 0.0 ? -(int)k : (int)k;
}

/* Encode every block of a frame.  Geometry, mask layout and chroma sharing
 * as for orc_decode; values[] as for orc_decode.  Per block and value
 * plane: c and a by orc_block_green_tab (dense LU of the bordered system in
 * FP64); code[] (laid out like values) = orc_quant(c, steps[plane]);
 * c_exact[] (same layout) = c unquantised; consts[] = a of every block of
 * every plane (Y blocks, then Cb, then Cr, raster order; 0 for K = 0).
 * Returns 0, or -1 on a position outside its block or a failed solve. */
int orc_encode_coef(int width, int height, int fmt, int b, const int32_t *block_ptr,
                    const uint16_t *pos, const float *values, int chroma_shared,
                    const double *steps, int op, double s,
                    int8_t *code, double *c_exact, double *consts, int nthreads)
{
    int PW[3], PH[3], NB[3], np_, g, ngroups, mp[3], vp[3][2], nv[3];
    long long cbase[3], nnz;
    int nitems = 0, cap, chroma_first = -1, m = 0, err = 0, it, k;
    int nshape = 0, shw[16], shh[16];
    double *shtab[16];
    orc_item *items;
    int *pblock;
    if (fmt == 0) { np_ = 1; PW[0] = width; PH[0] = height; }
    else { np_ = 3; PW[0] = width; PH[0] = height;
           PW[1] = PW[2] = (width + 1) / 2; PH[1] = PH[2] = (height + 1) / 2; }
    cbase[0] = 0;
    for (g = 0; g < np_; g++) NB[g] = ((PW[g] + b - 1) / b) * ((PH[g] + b - 1) / b);
    for (g = 1; g < np_; g++) cbase[g] = cbase[g - 1] + NB[g - 1];
    if (fmt == 0) { ngroups = 1; mp[0] = 0; vp[0][0] = 0; nv[0] = 1; }
    else if (chroma_shared) { ngroups = 2; mp[0] = 0; vp[0][0] = 0; nv[0] = 1;
                              mp[1] = 1; vp[1][0] = 1; vp[1][1] = 2; nv[1] = 2; }
    else { ngroups = 3; for (g = 0; g < 3; g++) { mp[g] = g; vp[g][0] = g; nv[g] = 1; } }
    cap = 0;
    for (g = 0; g < ngroups; g++) cap += NB[mp[g]];
    items = (orc_item *)malloc(sizeof(orc_item) * (size_t)cap);
    pblock = (int *)malloc(sizeof(int) * (size_t)cap);
    for (g = 0; g < ngroups; g++) {
        int W = PW[mp[g]], H = PH[mp[g]], bx, by;
        if (mp[g] == 1) chroma_first = m;
        for (by = 0; by < (H + b - 1) / b; by++)
            for (bx = 0; bx < (W + b - 1) / b; bx++) {
                orc_item *I = &items[nitems];
                pblock[nitems++] = by * ((W + b - 1) / b) + bx;
                I->m = m; I->x0 = bx * b; I->y0 = by * b;
                I->w = W - I->x0 < b ? W - I->x0 : b;
                I->h = H - I->y0 < b ? H - I->y0 : b;
                I->pw = W; I->nplanes = nv[g];
                for (k = 0; k < nv[g]; k++) I->plane[k] = vp[g][k];
                m++;
            }
    }
    nnz = block_ptr[m];
    for (it = 0; it < nitems; it++) {
        orc_item *I = &items[it];
        for (k = 0; k < I->nplanes; k++) {
            if (I->plane[k] == 2 && chroma_shared)
                I->vbase[k] = nnz + (block_ptr[I->m] - block_ptr[chroma_first]);
            else
                I->vbase[k] = block_ptr[I->m];
        }
        for (k = 0; k < nshape; k++)
            if (shw[k] == I->w && shh[k] == I->h) break;
        if (k == nshape && nshape < 16) {
            double *lam = (double *)malloc(sizeof(double) * (size_t)I->w * I->h);
            shw[nshape] = I->w; shh[nshape] = I->h;
            shtab[nshape] = (double *)malloc(sizeof(double) * (size_t)(I->w + 1) * (I->h + 1));
            orc_eigenvalues(I->w, I->h, op, s, lam);
            orc_green_table(I->w, I->h, lam, shtab[nshape]);
            free(lam);
            nshape++;
        }
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(|:err)
#endif
    for (it = 0; it < nitems; it++) {
        orc_item *I = &items[it];
        int K = block_ptr[I->m + 1] - block_ptr[I->m];
        int N = I->w * I->h, j, kk;
        const uint16_t *ps = pos + block_ptr[I->m];
        const double *tab = 0;
        double *r = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1) * 2);
        double *u = (double *)malloc(sizeof(double) * (size_t)N * 2);
        double *c = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1) * 2);
        double a[2] = {0.0, 0.0};
        for (kk = 0; kk < nshape; kk++)
            if (shw[kk] == I->w && shh[kk] == I->h) tab = shtab[kk];
        for (kk = 0; kk < I->nplanes; kk++)
            for (j = 0; j < K; j++) r[kk * K + j] = (double)values[I->vbase[kk] + j];
        if (tab == 0 || orc_block_green_tab(I->w, I->h, tab, K, ps, I->nplanes, r, c, a, u) != 0) {
            err |= 1;
        } else {
            for (kk = 0; kk < I->nplanes; kk++) {
                int pl = I->plane[kk];
                for (j = 0; j < K; j++) {
                    code[I->vbase[kk] + j] = (int8_t)orc_quant(c[kk * K + j], steps[pl]);
                    c_exact[I->vbase[kk] + j] = c[kk * K + j];
                }
                consts[cbase[pl] + pblock[it]] = a[kk];
            }
        }
        free(r); free(u); free(c);
    }
    for (it = 0; it < nshape; it++) free(shtab[it]);
    free(items);
    free(pblock);
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* (5) Mask selection per block by rectangular subdivision (the       */
/*     encoder picks each 8x8 block's mask points this way, Sec. 2.3; */
/*     the scheme is cited there, this is the reading taken).         */
/* ------------------------------------------------------------------ */

/* One block (w x h pixels, nv value planes r[v][w*h] sharing the mask):
 * rectangles are inclusive pixel ranges [x0, x1] x [y0, y1] whose four
 * corners are mask points; neighbours share their common edge.  Starting
 * from the whole block, each round inpaints the block from the corners of
 * all current rectangles (Green's route, orc_block_green_tab), takes every
 * rectangle's mean squared error over its pixels (averaged over the value
 * planes) and halves every rectangle whose error exceeds thr and whose
 * longer side spans at least 2 pixel gaps: along x when x1 - x0 >= y1 - y0,
 * else along y, at mid = (lo + hi) / 2 (both halves keep the middle line).
 * Rounds repeat until no rectangle is split (at most max_rounds).
 * mask[w*h] receives 1 at the selected pixels.  Returns 0 / -1. */
int orc_select_block(int w, int h, const double *Htab, int nv, const double *r, double thr,
                     int max_rounds, uint8_t *mask)
{
    int N = w * h, nl = 1, round, i, j, v, rc = 0;
    int rx0[256], rx1[256], ry0[256], ry1[256];
    uint16_t pos[256];
    double *rv = (double *)malloc(sizeof(double) * (size_t)N * 2);
    double *c = (double *)malloc(sizeof(double) * (size_t)N * 2);
    double *u = (double *)malloc(sizeof(double) * (size_t)N * 2);
    double a[2];
    if (N > 256 || nv < 1 || nv > 2) { free(rv); free(c); free(u); return -1; }
    rx0[0] = 0; rx1[0] = w - 1; ry0[0] = 0; ry1[0] = h - 1;
    for (round = 0; ; round++) {
        int K = 0, nnew = 0;
        memset(mask, 0, (size_t)N);
        for (j = 0; j < nl; j++) {
            mask[ry0[j] * w + rx0[j]] = 1; mask[ry0[j] * w + rx1[j]] = 1;
            mask[ry1[j] * w + rx0[j]] = 1; mask[ry1[j] * w + rx1[j]] = 1;
        }
        if (round >= max_rounds) break;
        for (i = 0; i < N; i++)
            if (mask[i]) pos[K++] = (uint16_t)i;
        if (K == N) break;  /* every pixel known: no error left */
        for (v = 0; v < nv; v++)
            for (i = 0; i < K; i++) rv[v * K + i] = r[v * N + pos[i]];
        if (orc_block_green_tab(w, h, Htab, K, pos, nv, rv, c, a, u) != 0) { rc = -1; break; }
        {
            int n0 = nl;
            for (j = 0; j < n0; j++) {
                double e = 0.0;
                int x, y, cnt = (rx1[j] - rx0[j] + 1) * (ry1[j] - ry0[j] + 1);
                int gx = rx1[j] - rx0[j], gy = ry1[j] - ry0[j];
                for (v = 0; v < nv; v++)
                    for (y = ry0[j]; y <= ry1[j]; y++)
                        for (x = rx0[j]; x <= rx1[j]; x++) {
                            double d = u[v * N + y * w + x] - r[v * N + y * w + x];
                            e += d * d;
                        }
                e /= (double)cnt * nv;
                if (!(e > thr)) continue;
                if (gx >= gy && gx >= 2) {
                    int mid = (rx0[j] + rx1[j]) / 2;
                    rx0[nl] = mid; rx1[nl] = rx1[j]; ry0[nl] = ry0[j]; ry1[nl] = ry1[j];
                    rx1[j] = mid;
                    nl++; nnew++;
                } else if (gy > gx && gy >= 2) {
                    int mid = (ry0[j] + ry1[j]) / 2;
                    rx0[nl] = rx0[j]; rx1[nl] = rx1[j]; ry0[nl] = mid; ry1[nl] = ry1[j];
                    ry1[j] = mid;
                    nl++; nnew++;
                }
            }
        }
        if (nnew == 0) break;
    }
    free(rv); free(c); free(u);
    return rc;
}

/* Select the mask of every block of a frame.  fmt, width, height and b as
 * for orc_decode; planes[] holds the dense residual planes (Y, then Cb, Cr
 * for 4:2:0), row-major, concatenated.  chroma_shared: one chroma mask
 * chosen on both chroma planes (their errors averaged), else one per plane.
 * thr[0] is the luma threshold, thr[1] the chroma one.  mask[] receives the
 * dense masks of the mask planes (Y, then the chroma mask(s)), row-major,
 * concatenated.  Returns 0 / -1. */
int orc_select_mask(int width, int height, int fmt, int b, const double *planes, int chroma_shared,
                    const double *thr, int max_rounds, uint8_t *mask, int nthreads)
{
    int PW[3], PH[3], np_, g, ngroups, mp[3], vp[3][2], nv[3], err = 0;
    long long poff[3], moff[3];
    if (fmt == 0) { np_ = 1; PW[0] = width; PH[0] = height; }
    else { np_ = 3; PW[0] = width; PH[0] = height;
           PW[1] = PW[2] = (width + 1) / 2; PH[1] = PH[2] = (height + 1) / 2; }
    poff[0] = 0;
    for (g = 1; g < np_; g++) poff[g] = poff[g - 1] + (long long)PW[g - 1] * PH[g - 1];
    if (fmt == 0) { ngroups = 1; mp[0] = 0; vp[0][0] = 0; nv[0] = 1; }
    else if (chroma_shared) { ngroups = 2; mp[0] = 0; vp[0][0] = 0; nv[0] = 1;
                              mp[1] = 1; vp[1][0] = 1; vp[1][1] = 2; nv[1] = 2; }
    else { ngroups = 3; for (g = 0; g < 3; g++) { mp[g] = g; vp[g][0] = g; nv[g] = 1; } }
    moff[0] = 0;
    for (g = 1; g < ngroups; g++) moff[g] = moff[g - 1] + (long long)PW[mp[g - 1]] * PH[mp[g - 1]];
    for (g = 0; g < ngroups; g++) {
        int W = PW[mp[g]], H = PH[mp[g]], nbx = (W + b - 1) / b, nby = (H + b - 1) / b, blk;
        double t = thr[g == 0 ? 0 : 1];
#ifdef _OPENMP
        if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(|:err)
#endif
        for (blk = 0; blk < nbx * nby; blk++) {
            int x0 = (blk % nbx) * b, y0 = (blk / nbx) * b;
            int w = W - x0 < b ? W - x0 : b, h = H - y0 < b ? H - y0 : b;
            int N = w * h, v, x, y;
            double lam[256], Htab[17 * 17], r[512];
            uint8_t m[256];
            if (N > 256) { err |= 1; continue; }
            orc_eigenvalues(w, h, 0, 1.0, lam);
            orc_green_table(w, h, lam, Htab);
            for (v = 0; v < nv[g]; v++) {
                const double *P = planes + poff[vp[g][v]];
                for (y = 0; y < h; y++)
                    for (x = 0; x < w; x++) r[v * N + y * w + x] = P[(long long)(y0 + y) * W + x0 + x];
            }
            if (orc_select_block(w, h, Htab, nv[g], r, t, max_rounds, m) != 0) { err |= 1; continue; }
            for (y = 0; y < h; y++)
                for (x = 0; x < w; x++) mask[moff[g] + (long long)(y0 + y) * W + x0 + x] = m[y * w + x];
        }
    }
    return err ? -1 : 0;
}
