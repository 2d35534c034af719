// Device kernels of the multi-level solve (Fig. code:mg): level transfers,
// smoother construction and application, dense bottom solve, norms.
#include <algorithm>
#include <cfloat>

#include "mlcr_internal.h"
#include "solver_internal.h"
#include "block_dev.h"

namespace mlcr {

// ---------------------------------------------------------------------------
// packed-vector kernels, one workgroup per (m, RHS)
// ---------------------------------------------------------------------------
// dst[idx_H(l,m,.)] = w[l] * src[idx_h(l,m,.)]  for l <= lmax_H  (restriction I_h^H)
// or, with add = true, dst_h += w[l] * src_H                       (interpolation (I_h^H)^T)
__global__ __launch_bounds__(256) void k_transfer(const double *__restrict__ src, int lmax_src,
                                                  double *__restrict__ dst, int lmax_dst,
                                                  const double *__restrict__ w, int lmax_w,
                                                  int add) {
    const int m = blockIdx.x, r = blockIdx.y;
    if (m > lmax_w) return;
    const long long nsrc = (long long)(lmax_src + 1) * (lmax_src + 1);
    const long long ndst = (long long)(lmax_dst + 1) * (lmax_dst + 1);
    const int nls = lmax_src - m + 1, nld = lmax_dst - m + 1, nlw = lmax_w - m + 1;
    const long long bs = (long long)r * nsrc + cos_base(m, lmax_src);
    const long long bd = (long long)r * ndst + cos_base(m, lmax_dst);
    const int cnt = (m == 0) ? nlw : 2 * nlw;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const int cs = i >= nlw;
        const int dl = cs ? i - nlw : i;           // l - m
        const double v = w[m + dl] * src[bs + (cs ? nls : 0) + dl];
        double *p = dst + bd + (cs ? nld : 0) + dl;
        if (add) *p += v;
        else *p = v;
    }
    // entries of a larger destination above lmax_w are cleared on restriction
    if (!add && lmax_dst > lmax_w) {
        const int extra = nld - nlw;
        const int cnt2 = (m == 0) ? extra : 2 * extra;
        for (int i = threadIdx.x; i < cnt2; i += blockDim.x) {
            const int cs = i >= extra;
            const int dl = nlw + (cs ? i - extra : i);
            dst[bd + (cs ? nld : 0) + dl] = 0.0;
        }
    }
}

// x += c[l] * d[idx] * r   (d may be null: 1)
__global__ __launch_bounds__(256) void k_axpy_l(double *__restrict__ x, const double *__restrict__ r,
                                                const double *__restrict__ c,
                                                const double *__restrict__ d, int lmax) {
    const int m = blockIdx.x, rr = blockIdx.y;
    const long long nalm = (long long)(lmax + 1) * (lmax + 1);
    const int nl = lmax - m + 1;
    const int cnt = (m == 0) ? nl : 2 * nl;
    const long long off = cos_base(m, lmax);
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const int l = m + (i < nl ? i : i - nl);
        double v = c[l] * r[(long long)rr * nalm + off + i];
        if (d) v *= d[off + i];
        x[(long long)rr * nalm + off + i] += v;
    }
}

// r = b - y (flat), with optional mask per l (0 removes the mode)
__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ b,
                                                  const double *__restrict__ y,
                                                  double *__restrict__ r,
                                                  const double *__restrict__ act, int lmax) {
    const int m = blockIdx.x, rr = blockIdx.y;
    const long long nalm = (long long)(lmax + 1) * (lmax + 1);
    const int nl = lmax - m + 1;
    const int cnt = (m == 0) ? nl : 2 * nl;
    const long long off = (long long)rr * nalm + cos_base(m, lmax);
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const int l = m + (i < nl ? i : i - nl);
        const double v = b[off + i] - (y ? y[off + i] : 0.0);
        r[off + i] = act ? act[l] * v : v;
    }
}

// per RHS: out[2 r] = sum w[l] a^2, out[2 r + 1] = sum w[l] b^2  (S^-1 weighted norms)
__global__ __launch_bounds__(256) void k_wnorms(const double *__restrict__ a,
                                                const double *__restrict__ b,
                                                const double *__restrict__ w, int lmax,
                                                double *__restrict__ partial) {
    // grid (lmax+1, nrhs): partial[(r * (lmax+1) + m) * 2 + {0,1}]
    const int m = blockIdx.x, rr = blockIdx.y;
    const long long nalm = (long long)(lmax + 1) * (lmax + 1);
    const int nl = lmax - m + 1;
    const int cnt = (m == 0) ? nl : 2 * nl;
    const long long off = (long long)rr * nalm + cos_base(m, lmax);
    double sa = 0.0, sb = 0.0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const int l = m + (i < nl ? i : i - nl);
        const double va = a[off + i], vb = b ? b[off + i] : 0.0;
        sa = fma(w[l] * va, va, sa);
        sb = fma(w[l] * vb, vb, sb);
    }
    __shared__ double ra[256], rb[256];
    ra[threadIdx.x] = sa;
    rb[threadIdx.x] = sb;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ra[threadIdx.x] += ra[threadIdx.x + s];
            rb[threadIdx.x] += rb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[((long long)rr * (lmax + 1) + m) * 2] = ra[0];
        partial[((long long)rr * (lmax + 1) + m) * 2 + 1] = rb[0];
    }
}

// second stage: one block per RHS sums the per-m partials in a fixed order
__global__ __launch_bounds__(256) void k_wnorms_final(const double *__restrict__ partial, int nm,
                                                      double *__restrict__ out) {
    const int rr = blockIdx.x;
    double sa = 0.0, sb = 0.0;
    for (int i = threadIdx.x; i < nm; i += blockDim.x) {
        sa += partial[((long long)rr * nm + i) * 2];
        sb += partial[((long long)rr * nm + i) * 2 + 1];
    }
    __shared__ double ra[256], rb[256];
    ra[threadIdx.x] = sa;
    rb[threadIdx.x] = sb;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ra[threadIdx.x] += ra[threadIdx.x + s];
            rb[threadIdx.x] += rb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * rr] = ra[0];
        out[2 * rr + 1] = rb[0];
    }
}

// p[0..n) = 0 (a kernel, not a memset: the cycle may be captured into a graph)
__global__ __launch_bounds__(256) void k_fill_zero(double *__restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// per RHS: out[2 r] = <a, b>, out[2 r + 1] = <c, d> over all coefficients
// (c, d may be null: 0); partial sums per order m, then k_wnorms_final
__global__ __launch_bounds__(256) void k_dots(const double *__restrict__ a,
                                              const double *__restrict__ b,
                                              const double *__restrict__ c,
                                              const double *__restrict__ d, int lmax,
                                              double *__restrict__ partial) {
    const int m = blockIdx.x, rr = blockIdx.y;
    const long long nalm = (long long)(lmax + 1) * (lmax + 1);
    const int nl = lmax - m + 1;
    const int cnt = (m == 0) ? nl : 2 * nl;
    const long long off = (long long)rr * nalm + cos_base(m, lmax);
    double s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        s1 = fma(a[off + i], b[off + i], s1);
        if (c) s2 = fma(c[off + i], d[off + i], s2);
    }
    __shared__ double ra[256], rb[256];
    ra[threadIdx.x] = s1;
    rb[threadIdx.x] = s2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            ra[threadIdx.x] += ra[threadIdx.x + st];
            rb[threadIdx.x] += rb[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[((long long)rr * (lmax + 1) + m) * 2] = ra[0];
        partial[((long long)rr * (lmax + 1) + m) * 2 + 1] = rb[0];
    }
}

// per multipole l: out[l] = sum_r sum_{m <= l} a_lm b_lm over the cosine and
// sine entries of l (one workgroup per l, fixed summation order)
__global__ __launch_bounds__(256) void k_ell_dots(const double *__restrict__ a,
                                                  const double *__restrict__ b, int lmax, int nrhs,
                                                  double *__restrict__ out) {
    const int l = blockIdx.x;
    const long long nalm = (long long)(lmax + 1) * (lmax + 1);
    const int cnt = 2 * l + 1;                 // entry 0: m = 0; 2 m - 1, 2 m: cos, sin of m
    double acc = 0.0;
    for (int rr = 0; rr < nrhs; rr++)
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            const int m = (i + 1) / 2;
            long long idx = cos_base(m, lmax) + (l - m);
            if (m > 0 && (i & 1) == 0) idx += lmax - m + 1;      // sine block
            const long long o = (long long)rr * nalm + idx;
            acc = fma(a[o], b[o], acc);
        }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[l] = red[0];
}

// out = al[r] u + be[r] v per RHS r, flat (out may alias u or v)
__global__ __launch_bounds__(256) void k_lincomb(const double *u, const double *v, double *out,
                                                 const double *__restrict__ al,
                                                 const double *__restrict__ be, long long n) {
    const int rr = blockIdx.y;
    const double a = al[rr], b = be[rr];
    const long long base = (long long)rr * n;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[base + i] = a * u[base + i] + b * v[base + i];
}

// CR right-hand side, pixel part: pix = N^-1 d + N^-1/2 w2 (w2 may be null)
__global__ __launch_bounds__(256) void k_cr_pix(const double *__restrict__ d,
                                                const double *__restrict__ w2,
                                                const double *__restrict__ ninv,
                                                double *__restrict__ pix, long long npix) {
    const int rr = blockIdx.y;
    const long long base = (long long)rr * npix;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < npix;
         i += (long long)gridDim.x * blockDim.x) {
        const double w = ninv[i];
        double v = w * d[base + i];
        if (w2) v = fma(sqrt(w), w2[base + i], v);
        pix[base + i] = v;
    }
}

// CR right-hand side, harmonic part: b = bh[l] v + sqrt(dd[l]) w1 (w1 may be null)
__global__ __launch_bounds__(256) void k_cr_combine(const double *v,
                                                    const double *__restrict__ w1,
                                                    const double *__restrict__ bh,
                                                    const double *__restrict__ dd,
                                                    double *b, int lmax) {
    const int m = blockIdx.x, rr = blockIdx.y;
    const long long nalm = (long long)(lmax + 1) * (lmax + 1);
    const int nl = lmax - m + 1;
    const int cnt = (m == 0) ? nl : 2 * nl;
    const long long off = (long long)rr * nalm + cos_base(m, lmax);
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const int l = m + (i < nl ? i : i - nl);
        double o = bh[l] * v[off + i];
        if (w1) o = fma(sqrt(dd[l]), w1[off + i], o);
        b[off + i] = o;
    }
}

// ---------------------------------------------------------------------------
// top-level diagonal: the ring sums of eq. Ni-dense at frequencies 0 and 2m
// ---------------------------------------------------------------------------
// Xi holds, per ring, w_D (Re, Im) of sum_j xi_j e^{i D phi_j} for D <= 2 lmax
// (the adjoint ring step applied to the map xi).  Output per ring and m:
// (Re Xi(0) + Re Xi(2m), Re Xi(0) - Re Xi(2m)) for m >= 1 and (Re Xi(0), 0) for m = 0.
__global__ __launch_bounds__(256) void k_diag_pairs(const double2 *__restrict__ Xi, int ldx,
                                                    double2 *__restrict__ G, int lmax) {
    const int k = blockIdx.x;
    const double x0 = Xi[(long long)k * ldx].x;     // w_0 = 1
    for (int m = threadIdx.x; m <= lmax; m += blockDim.x) {
        double2 out;
        if (m == 0) {
            out = make_double2(x0, 0.0);
        } else {
            const double x2 = Xi[(long long)k * ldx + 2 * m].x * 0.70710678118654752440;
            out = make_double2(x0 + x2, x0 - x2);
        }
        G[(long long)k * (lmax + 1) + m] = out;
    }
}

// dinv[idx] = act / (d[l] + bh[l]^2 q[idx])  (0 for excluded modes)
__global__ __launch_bounds__(256) void k_diag_inverse(const double *__restrict__ q,
                                                      const double *__restrict__ d,
                                                      const double *__restrict__ bh,
                                                      double *__restrict__ dinv, int lmax) {
    const int m = blockIdx.x;
    const int nl = lmax - m + 1;
    const int cnt = (m == 0) ? nl : 2 * nl;
    const long long off = cos_base(m, lmax);
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const int l = m + (i < nl ? i : i - nl);
        const double a = d[l] + bh[l] * bh[l] * q[off + i];
        dinv[off + i] = (d[l] > 0.0 && a > 0.0) ? 1.0 / a : 0.0;
    }
}

// ---------------------------------------------------------------------------
// pixel-level smoother on k x k tiles (tiles = pixels of the grid N_side / k)
// ---------------------------------------------------------------------------
// probe maps: map[p][tilepix[t * kk + c0 + p]] = 1 for every tile t
// maps[p][tilepix[t * kk + c0 + p]] = 1 for every tile t of the list (one colour)
__global__ __launch_bounds__(256) void k_probe_maps(double *__restrict__ maps, long long npix,
                                                    const int *__restrict__ tilepix,
                                                    const int *__restrict__ tiles, int ntl,
                                                    int kk, int c0, int nprobe) {
    const long long n = (long long)ntl * nprobe;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int p = (int)(i / ntl), t = tiles[i % ntl];
        maps[(long long)p * npix + tilepix[(long long)t * kk + c0 + p]] = 1.0;
    }
}

// Read the probe responses of the tiles u of one colour (Sec. 3.5 block pattern):
// at u itself into its diagonal block diag[u][i][c] (row-major, float64) and at
// each neighbour t into the coupling block of the pair (t, u), off[slot][c][i]
// (column c = probe position in u, row i = pixel of t; the slot is the entry of
// u in t's neighbour list, rev[] of u's own slot).
__global__ __launch_bounds__(256) void k_probe_collect(const double *__restrict__ z,
                                                       long long npix,
                                                       const int *__restrict__ tilepix,
                                                       const int *__restrict__ tiles, int ntl,
                                                       const int *__restrict__ nbptr,
                                                       const int *__restrict__ nbs,
                                                       const int *__restrict__ rev, int max_nb,
                                                       int c0, int nprobe,
                                                       double *__restrict__ diag,
                                                       float *__restrict__ off) {
    const long long n = (long long)ntl * (max_nb + 1) * kTileK2 * nprobe;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const int p = (int)(e % nprobe);
        long long q = e / nprobe;
        const int i = (int)(q % kTileK2);
        q /= kTileK2;
        const int j = (int)(q % (max_nb + 1));
        const int u = tiles[q / (max_nb + 1)];
        const int c = c0 + p;
        if (j == 0) {
            diag[((long long)u * kTileK2 + i) * kTileK2 + c] =
                z[(long long)p * npix + tilepix[(long long)u * kTileK2 + i]];
            continue;
        }
        const int sl = nbptr[u] + j - 1;
        if (sl >= nbptr[u + 1]) continue;
        const int t = nbs[sl];
        off[((long long)rev[sl] * kTileK2 + c) * kTileK2 + i] =
            z[(long long)p * npix + tilepix[(long long)t * kTileK2 + i]];
    }
}

// Average each coupling block with the transpose of its partner:
// off(t,u)[c][i] and off(u,t)[i][c] come from different probes.
__global__ __launch_bounds__(256) void k_sym_off(const int *__restrict__ nbptr,
                                                 const int *__restrict__ nbs,
                                                 const int *__restrict__ rev,
                                                 float *__restrict__ off) {
    const int t = blockIdx.x;
    for (int sl = nbptr[t]; sl < nbptr[t + 1]; sl++) {
        const int u = nbs[sl];
        if (u < t) continue;
        float *A = off + (long long)sl * kTileK2 * kTileK2;
        float *B = off + (long long)rev[sl] * kTileK2 * kTileK2;
        for (int e = threadIdx.x; e < kTileK2 * kTileK2; e += blockDim.x) {
            const int c = e / kTileK2, i = e % kTileK2;
            const float v = 0.5f * (A[c * kTileK2 + i] + B[i * kTileK2 + c]);
            A[c * kTileK2 + i] = v;
            B[i * kTileK2 + c] = v;
        }
    }
}

// In-LDS Cholesky of a kk x kk SPD matrix (lower, row-major a[i*kk+j]);
// returns false if a pivot is not positive.  All threads of the block.

// Per tile: symmetrize the probed block, factor with the smallest ridge
// alpha (bisection in log alpha, then 1.5 alpha, Sec. 3.5) that makes the
// Cholesky succeed, and store the inverse in float32 (column-major; it is
// symmetric).  ridge_out[t] records the alpha used (relative to max |a_ii|).
__global__ __launch_bounds__(256) void k_tile_factor(const double *__restrict__ blocks, int kk,
                                                     float *__restrict__ minv,
                                                     float *__restrict__ ridge_out) {
    extern __shared__ double sm[];
    double *a = sm;                  // kk*kk
    double *inv = sm + kk * kk;      // kk*kk
    double *flag = inv + kk * kk;    // 1
    const int t = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const double *B = blocks + (long long)t * kk * kk;
    __shared__ double dmax;
    if (tid == 0) {
        double m = 0.0;
        for (int i = 0; i < kk; i++) m = fmax(m, fabs(B[i * kk + i]));
        dmax = m > 0.0 ? m : 1.0;
    }
    __syncthreads();
    auto load = [&](double alpha) {
        for (int e = tid; e < kk * kk; e += nt) {
            const int i = e / kk, j = e % kk;
            double v = 0.5 * (B[i * kk + j] + B[j * kk + i]);
            if (i == j) v += alpha * dmax;
            a[e] = v;
        }
        __syncthreads();
    };
    load(0.0);
    bool ok = lds_cholesky(a, kk, flag);
    double alpha = 0.0;
    if (!ok) {
        double lo = -16.0, hi = 0.0;            // log10 of alpha
        load(1.0);
        if (lds_cholesky(a, kk, flag)) {
            for (int it = 0; it < 30; it++) {
                const double mid = 0.5 * (lo + hi);
                load(pow(10.0, mid));
                if (lds_cholesky(a, kk, flag)) hi = mid;
                else lo = mid;
            }
            alpha = 1.5 * pow(10.0, hi);
        } else {
            alpha = 1.5;
        }
        load(alpha);
        ok = lds_cholesky(a, kk, flag);
    }
    // inverse from the factor: solve L L^T X = I column by column
    for (int e = tid; e < kk * kk; e += nt) inv[e] = (e / kk == e % kk) ? 1.0 : 0.0;
    __syncthreads();
    for (int c = tid; c < kk; c += nt) {
        // forward: L y = e_c ; backward: L^T x = y   (column c of inv, stored inv[i*kk + c])
        for (int i = 0; i < kk; i++) {
            double s = inv[i * kk + c];
            for (int j = 0; j < i; j++) s -= a[i * kk + j] * inv[j * kk + c];
            inv[i * kk + c] = s / a[i * kk + i];
        }
        for (int i = kk - 1; i >= 0; i--) {
            double s = inv[i * kk + c];
            for (int j = i + 1; j < kk; j++) s -= a[j * kk + i] * inv[j * kk + c];
            inv[i * kk + c] = s / a[i * kk + i];
        }
    }
    __syncthreads();
    float *M = minv + (long long)t * kk * kk;
    for (int e = tid; e < kk * kk; e += nt) {
        const int i = e / kk, j = e % kk;
        M[j * kk + i] = ok ? (float)(0.5 * (inv[i * kk + j] + inv[j * kk + i])) : 0.0f;
    }
    if (tid == 0) ridge_out[t] = ok ? (float)alpha : -1.0f;
}

// One colour of the multicolour block symmetric Gauss-Seidel sweep on the
// block-sparse pixel operator (Sec. 3.5 pattern: a tile and its neighbours).
// Tiles of one colour are never neighbours, so each workgroup updates one
// tile with no ordering among them.  Lane i of each wave owns pixel i of the
// tile; blocks are float32 (the paper's smoother precision), maps float64.
//   mode 0, forward  (colours ascending):  y_t = D_t^-1 (r_t - sum_{u earlier} A_tu y_u)
//   mode 1, backward (colours descending): y_t -= D_t^-1 sum_{u later} A_tu y_u
// so y ends as M r with M^-1 = (D + L) D^-1 (D + L^T).  The same kernel runs
// the triangular solves of a block incomplete Cholesky factor L L^T: mode 0
// with blocks L_tu (u earlier) and L_tt^-1 is the forward solve, and
//   mode 2, backward (colours descending): y_t = L_tt^-T (y_t - sum_{u later} L_ut^T y_u)
// (blocks L_ut^T stored at the slot t -> u) the backward solve.
// A tile's work is a chain of dependent block products, so it is spread over
// NW = 4 waves: wave w takes every NW-th neighbour block and a quarter of the
// columns of D_t^-1, and the partial sums are added in LDS (wave order).
template <int MODE>
__global__ __launch_bounds__(256) void k_sgs_color(const double *__restrict__ r,
                                                   double *__restrict__ y, long long npix,
                                                   int nrhs, const int *__restrict__ tilepix,
                                                   const int *__restrict__ tiles,
                                                   const int *__restrict__ nbptr,
                                                   const int *__restrict__ nbs,
                                                   const int *__restrict__ color, int kappa,
                                                   const float *__restrict__ off,
                                                   const float *__restrict__ minv) {
    constexpr int K2 = kTileK2, NQ = 8, NW = 4, JW = K2 / NW;
    constexpr bool FWD = MODE == 0;
    static_assert(NQ % NW == 0 && K2 % (NW * 16) == 0, "tile shape");
    __shared__ float v[NW][NQ][K2];              // per-wave neighbour values; then the right side
    __shared__ float part[NW][NQ][K2];           // per-wave partial sums
    const int t = tiles[blockIdx.x];
    const int wv = threadIdx.x >> 6, i = threadIdx.x & 63;
    const long long pix = tilepix[(long long)t * K2 + i];
    const int s0 = nbptr[t], s1 = nbptr[t + 1];
    const float *Mi = minv + (long long)t * K2 * K2;
    for (int r0 = 0; r0 < nrhs; r0 += NQ) {
        const int nq = min(NQ, nrhs - r0);
        float acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; q++) acc[q] = 0.0f;
        bool any = false;
        for (int sl = s0 + wv; sl < s1; sl += NW) {
            const int u = nbs[sl];
            const int cu = color[u];
            if (FWD ? !(cu < kappa) : !(cu > kappa)) continue;
            any = true;
            const long long pu = tilepix[(long long)u * K2 + i];
#pragma unroll
            for (int q = 0; q < NQ; q++)
                v[wv][q][i] = q < nq ? (float)y[(long long)(r0 + q) * npix + pu] : 0.0f;
            __builtin_amdgcn_s_waitcnt(0xc07f);     // this wave's LDS writes landed
            __builtin_amdgcn_wave_barrier();
            const float *Bs = off + (long long)sl * K2 * K2;
            // 16 block entries loaded before their products
#pragma unroll 1
            for (int j0 = 0; j0 < K2; j0 += 16) {
                float b[16];
#pragma unroll
                for (int jj = 0; jj < 16; jj++) b[jj] = Bs[(j0 + jj) * K2 + i];
#pragma unroll
                for (int jj = 0; jj < 16; jj++)
#pragma unroll
                    for (int q = 0; q < NQ; q++) acc[q] = fmaf(b[jj], v[wv][q][j0 + jj], acc[q]);
            }
            __builtin_amdgcn_wave_barrier();         // reads done before the next gather
        }
#pragma unroll
        for (int q = 0; q < NQ; q++) part[wv][q][i] = acc[q];
        if (!__syncthreads_or(any) && MODE == 1) continue;    // uniform over the workgroup
        // right side for RHS q = NQ / NW * wv + qq, into v[0]
#pragma unroll
        for (int qq = 0; qq < NQ / NW; qq++) {
            const int q = NQ / NW * wv + qq;
            float tot = part[0][q][i];
#pragma unroll
            for (int w = 1; w < NW; w++) tot += part[w][q][i];
            float rhs = tot;
            if (q < nq && MODE == 0) rhs = (float)r[(long long)(r0 + q) * npix + pix] - tot;
            if (q < nq && MODE == 2) rhs = (float)y[(long long)(r0 + q) * npix + pix] - tot;
            v[0][q][i] = q < nq ? rhs : 0.0f;
        }
        __syncthreads();
        // D_t^-1 times the right side: wave w takes columns JW w .. JW w + JW - 1
        float o[NQ];
#pragma unroll
        for (int q = 0; q < NQ; q++) o[q] = 0.0f;
#pragma unroll 1
        for (int j0 = JW * wv; j0 < JW * (wv + 1); j0 += 16) {
            float mm[16];
#pragma unroll
            for (int jj = 0; jj < 16; jj++)
                mm[jj] = MODE == 2 ? Mi[i * K2 + (j0 + jj)] : Mi[(j0 + jj) * K2 + i];
#pragma unroll
            for (int jj = 0; jj < 16; jj++)
#pragma unroll
                for (int q = 0; q < NQ; q++) o[q] = fmaf(mm[jj], v[0][q][j0 + jj], o[q]);
        }
#pragma unroll
        for (int q = 0; q < NQ; q++) part[wv][q][i] = o[q];
        __syncthreads();
#pragma unroll
        for (int qq = 0; qq < NQ / NW; qq++) {
            const int q = NQ / NW * wv + qq;
            if (q >= nq) continue;
            float tot = part[0][q][i];
#pragma unroll
            for (int w = 1; w < NW; w++) tot += part[w][q][i];
            double *dst = y + (long long)(r0 + q) * npix + pix;
            *dst = MODE == 1 ? *dst - (double)tot : (double)tot;
        }
        __syncthreads();                         // LDS free for the next RHS chunk
    }
}

// ---------------------------------------------------------------------------
// dense block of Y^T N^-1 Y from ring Fourier sums (eq. Ni-dense)
// ---------------------------------------------------------------------------
// lambda_lm(theta_k) for l <= L at one ring per workgroup, one thread per m:
// the textbook recurrence (Sec. 3.2) from lambda_mm; for L <= 64 nothing
// leaves the float64 range, so no scaling is needed.  lt[k][tri(l, m)].
__global__ __launch_bounds__(128) void k_dense_lambda(const double *__restrict__ rz,
                                                      const double *__restrict__ rs, int L,
                                                      double *__restrict__ lt) {
    const int k = blockIdx.x;
    const int m = threadIdx.x;
    if (m > L) return;
    const double z = rz[k], sn = rs[k];
    const long long tri = (long long)(L + 1) * (L + 2) / 2;
    double *out = lt + (long long)k * tri + ((long long)m * (L + 1) - (long long)m * (m - 1) / 2);
    double lmm = 0.28209479177387814347;            // 1 / sqrt(4 pi)
    for (int j = 1; j <= m; j++) lmm *= -sqrt((2.0 * j + 1.0) / (2.0 * j)) * sn;
    out[0] = lmm;
    if (m == L) return;
    double l2 = lmm, l1 = sqrt(2.0 * m + 3.0) * z * lmm;
    out[1] = l1;
    double aprev = sqrt(2.0 * m + 3.0);
    for (int l = m + 2; l <= L; l++) {
        const double a = sqrt((4.0 * l * l - 1.0) / ((double)(l - m) * (l + m)));
        const double v = a * (z * l1 - l2 / aprev);
        l2 = l1;
        l1 = v;
        aprev = a;
        out[l - m] = v;
    }
}

// A[i][j] = d_i delta_ij + bh_i bh_j K_ij over the active modes, with
// K_ij = sum_k w_i w_j lambda_i(k) lambda_j(k) T_k: for real basis functions
// with trigonometric parts t_i(m_i phi), t_j(m_j phi) the ring sum of
// xi t_i t_j is half a combination of the ring sums C_k(D) = sum_j xi cos D phi
// and S_k(D) = sum_j xi sin D phi at D = m_i - m_j and m_i + m_j:
//   cos cos: (C(-) + C(+)) / 2     sin sin: (C(-) - C(+)) / 2
//   cos sin: (S(+) - S(-)) / 2     sin cos: (S(+) + S(-)) / 2
// Xi[k][D] holds (w_D C_k(D), w_D S_k(D)) (the ring adjoint's weights
// w_0 = 1, w_D = sqrt 2).  mode[i] = l | m << 8 | sine << 16.
__global__ __launch_bounds__(256) void k_dense_ringdft(const double2 *__restrict__ Xi, int ldx,
                                                       const double *__restrict__ lt, int L,
                                                       int nrings, const int *__restrict__ mode,
                                                       int na, const double *__restrict__ d,
                                                       const double *__restrict__ bh,
                                                       double *__restrict__ A) {
    const long long tri = (long long)(L + 1) * (L + 2) / 2;
    const long long n = (long long)na * na;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / na), j = (int)(e % na);
        if (j < i) continue;
        const int li = mode[i] & 255, mi = (mode[i] >> 8) & 255, si = mode[i] >> 16;
        const int lj = mode[j] & 255, mj = (mode[j] >> 8) & 255, sj = mode[j] >> 16;
        const long long ti = (long long)mi * (L + 1) - (long long)mi * (mi - 1) / 2 + (li - mi);
        const long long tj = (long long)mj * (L + 1) - (long long)mj * (mj - 1) / 2 + (lj - mj);
        const int dm = mi - mj, adm = dm < 0 ? -dm : dm, sp = mi + mj;
        const double wdm = adm == 0 ? 1.0 : 0.70710678118654752440;
        const double wsp = sp == 0 ? 1.0 : 0.70710678118654752440;
        const double sgn = dm < 0 ? -1.0 : 1.0;
        double acc = 0.0;
        for (int k = 0; k < nrings; k++) {
            const double2 xd = Xi[(long long)k * ldx + adm], xs = Xi[(long long)k * ldx + sp];
            const double cm = xd.x * wdm, sm = sgn * xd.y * wdm;
            const double cp = xs.x * wsp, smp = xs.y * wsp;
            double t;
            if (si == 0 && sj == 0) t = cm + cp;
            else if (si == 1 && sj == 1) t = cm - cp;
            else if (si == 0) t = smp - sm;
            else t = smp + sm;
            acc = fma(lt[(long long)k * tri + ti] * lt[(long long)k * tri + tj], t, acc);
        }
        const double w = (mi == 0 ? 1.0 : 1.41421356237309504880) * (mj == 0 ? 1.0 : 1.41421356237309504880);
        const double v = bh[li] * bh[lj] * 0.5 * w * acc + (i == j ? d[li] : 0.0);
        A[(long long)i * na + j] = v;
        A[(long long)j * na + i] = v;
    }
}

// Right-looking Cholesky (lower, row-major) of an n x n matrix in global
// memory by one workgroup.  info[0] = 0 on success, j + 1 at a failed pivot.
__global__ __launch_bounds__(1024) void k_dense_cholesky(double *__restrict__ a, int n,
                                                         int *__restrict__ info) {
    const int tid = threadIdx.x, nt = blockDim.x;
    __shared__ int bad;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < n; j++) {
        if (tid == 0) {
            const double piv = a[(long long)j * n + j];
            if (!(piv > 0.0) && !bad) bad = j + 1;
            a[(long long)j * n + j] = piv > 0.0 ? sqrt(piv) : 1.0;
        }
        __syncthreads();
        const double djj = a[(long long)j * n + j];
        for (int i = j + 1 + tid; i < n; i += nt) a[(long long)i * n + j] /= djj;
        __syncthreads();
        const int rem = n - j - 1;
        const long long tot = (long long)rem * (rem + 1) / 2;
        for (long long e = tid; e < tot; e += nt) {
            // e -> (i, c) with j < c <= i, row-by-row over the lower triangle
            const long long rr = (long long)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
            long long row = rr, base = rr * (rr + 1) / 2;
            if (base > e) { row--; base = row * (row + 1) / 2; }
            else if (base + row + 1 <= e) { row++; base = row * (row + 1) / 2; }
            const int i = j + 1 + (int)row, c = j + 1 + (int)(e - base);
            a[(long long)i * n + c] -= a[(long long)i * n + j] * a[(long long)c * n + j];
        }
        __syncthreads();
    }
    if (tid == 0) info[0] = bad;
}

// Column c of (L L^T)^-1 (one workgroup per column), written to inv[c * n + i].
__global__ __launch_bounds__(256) void k_dense_inverse(const double *__restrict__ L, int n,
                                                       double *__restrict__ inv) {
    extern __shared__ double v[];
    __shared__ double red[256];
    const int c = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < n; i += nt) v[i] = (i == c) ? 1.0 : 0.0;
    __syncthreads();
    // forward substitution L y = e_c (column-oriented; rows above c stay 0)
    for (int j = c; j < n; j++) {
        if (tid == 0) v[j] /= L[(long long)j * n + j];
        __syncthreads();
        const double vj = v[j];
        for (int i = j + 1 + tid; i < n; i += nt) v[i] -= L[(long long)i * n + j] * vj;
        __syncthreads();
    }
    // backward substitution L^T x = y (row-oriented dot products)
    for (int i = n - 1; i >= 0; i--) {
        double s = 0.0;
        for (int j = i + 1 + tid; j < n; j += nt) s += L[(long long)j * n + i] * v[j];
        red[tid] = s;
        __syncthreads();
        for (int st = nt / 2; st > 0; st >>= 1) {
            if (tid < st) red[tid] += red[tid + st];
            __syncthreads();
        }
        if (tid == 0) v[i] = (v[i] - red[0]) / L[(long long)i * n + i];
        __syncthreads();
    }
    for (int i = tid; i < n; i += nt) inv[(long long)c * n + i] = v[i];
}

// x[act_idx[i]] = sum_j Ainv[j][i] b[act_idx[j]]  (Ainv symmetric; x pre-cleared)
// x = A^-1 b on the active modes, in three steps: gather the active entries
// of b (g[r][j]), partial products over kDenseJS column chunks (64 rows per
// workgroup, 4 column lanes per row added in LDS in lane order), then the
// chunk sums in chunk order, scattered into x.  Every row's sum is split
// over many workgroups: one thread per row walking all n columns was bound
// by its serial chain of loads.
constexpr int kDenseJS = 8;

__global__ __launch_bounds__(256) void k_dense_rhs(const double *__restrict__ b, long long nalm,
                                                   const int *__restrict__ act_idx, int n,
                                                   int nrhs, double *__restrict__ g) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)n * nrhs) return;
    const int r = (int)(e / n), j = (int)(e % n);
    g[e] = b[(long long)r * nalm + act_idx[j]];
}

__global__ __launch_bounds__(256) void k_dense_partial(const double *__restrict__ Ainv, int n,
                                                       const double *__restrict__ g, int nrhs,
                                                       double *__restrict__ part) {
    constexpr int NQ = 8;
    __shared__ double red[4][NQ][64];
    const int l = threadIdx.x & 63, jl = threadIdx.x >> 6;
    const int row = blockIdx.x * 64 + l, c = blockIdx.y, r0 = blockIdx.z * NQ;
    const int jb = (int)((long long)n * c / kDenseJS), je = (int)((long long)n * (c + 1) / kDenseJS);
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) acc[q] = 0.0;
    if (row < n) {
        for (int j = jb + jl; j < je; j += 4) {
            const double a = Ainv[(long long)j * n + row];
#pragma unroll
            for (int q = 0; q < NQ; q++)
                if (r0 + q < nrhs) acc[q] = fma(a, g[(long long)(r0 + q) * n + j], acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; q++) red[jl][q][l] = acc[q];
    __syncthreads();
    if (jl == 0 && row < n) {
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            if (r0 + q >= nrhs) break;
            const double s = ((red[0][q][l] + red[1][q][l]) + red[2][q][l]) + red[3][q][l];
            part[((long long)c * nrhs + r0 + q) * n + row] = s;
        }
    }
}

__global__ __launch_bounds__(256) void k_dense_finish(const double *__restrict__ part, int n,
                                                      int nrhs, const int *__restrict__ act_idx,
                                                      double *__restrict__ x, long long nalm) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)n * nrhs) return;
    const int r = (int)(e / n), i = (int)(e % n);
    double s = 0.0;
    for (int c = 0; c < kDenseJS; c++) s += part[((long long)c * nrhs + r) * n + i];
    x[(long long)r * nalm + act_idx[i]] = s;
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(long long n, int bs) {
    long long b = (n + bs - 1) / bs;
    return (unsigned)std::min<long long>(std::max<long long>(b, 1), 65535LL * 4);
}

int launch_fill_zero(double *p, long long n, hipStream_t s) {
    if (n <= 0) return MLCR_OK;
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_transfer(const double *src, int lmax_src, double *dst, int lmax_dst, const double *w,
                    int lmax_w, bool add, int nrhs, hipStream_t s) {
    const int grid_m = std::max(lmax_dst, lmax_w) + 1;
    hipLaunchKernelGGL(k_transfer, dim3(grid_m, nrhs), dim3(256), 0, s, src, lmax_src, dst,
                       lmax_dst, w, lmax_w, add ? 1 : 0);
    MLCR_HIP_CHECK(hipGetLastError());
    if (!add && lmax_dst > lmax_w) {
        // orders m > lmax_w of the destination are cleared as a whole
        const long long nd = (long long)(lmax_dst + 1) * (lmax_dst + 1);
        for (int r = 0; r < nrhs; r++) {
            const long long off = cos_base(lmax_w + 1, lmax_dst);
            const int rc = launch_fill_zero(dst + r * nd + off, nd - off, s);
            if (rc) return rc;
        }
    }
    return MLCR_OK;
}

int launch_axpy_l(double *x, const double *r, const double *c, const double *d, int lmax, int nrhs,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_l, dim3(lmax + 1, nrhs), dim3(256), 0, s, x, r, c, d, lmax);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_residual(const double *b, const double *y, double *r, const double *act, int lmax,
                    int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_residual, dim3(lmax + 1, nrhs), dim3(256), 0, s, b, y, r, act, lmax);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_wnorms(const double *a, const double *b, const double *w, int lmax, int nrhs,
                  double *partial, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_wnorms, dim3(lmax + 1, nrhs), dim3(256), 0, s, a, b, w, lmax, partial);
    MLCR_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_wnorms_final, dim3(nrhs), dim3(256), 0, s, partial, lmax + 1, out);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_diag_pairs(const double2 *Xi, int ldx, double2 *G, int lmax, int nrings,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_diag_pairs, dim3(nrings), dim3(256), 0, s, Xi, ldx, G, lmax);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_diag_inverse(const double *q, const double *d, const double *bh, double *dinv, int lmax,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_diag_inverse, dim3(lmax + 1), dim3(256), 0, s, q, d, bh, dinv, lmax);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_probe_maps(double *maps, long long npix, const int *tilepix, const int *tiles, int ntl,
                      int kk, int c0, int nprobe, hipStream_t s) {
    MLCR_HIP_CHECK(hipMemsetAsync(maps, 0, (size_t)nprobe * npix * sizeof(double), s));
    if (ntl <= 0) return MLCR_OK;
    hipLaunchKernelGGL(k_probe_maps, dim3(nblk((long long)ntl * nprobe, 256)), dim3(256), 0, s,
                       maps, npix, tilepix, tiles, ntl, kk, c0, nprobe);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_probe_collect(const double *z, long long npix, const int *tilepix, const int *tiles,
                         int ntl, const int *nbptr, const int *nbs, const int *rev, int max_nb,
                         int c0, int nprobe, double *diag, float *off, hipStream_t s) {
    if (ntl <= 0) return MLCR_OK;
    hipLaunchKernelGGL(k_probe_collect,
                       dim3(nblk((long long)ntl * (max_nb + 1) * kTileK2 * nprobe, 256)), dim3(256),
                       0, s, z, npix, tilepix, tiles, ntl, nbptr, nbs, rev, max_nb, c0, nprobe,
                       diag, off);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_sym_off(const int *nbptr, const int *nbs, const int *rev, float *off, int ntiles,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_sym_off, dim3(ntiles), dim3(256), 0, s, nbptr, nbs, rev, off);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_tile_factor(const double *blocks, int ntiles, int kk, float *minv, float *ridge,
                       hipStream_t s) {
    const size_t lds = (2 * (size_t)kk * kk + 1) * sizeof(double);
    int rc = ensure_dynamic_lds((const void *)k_tile_factor, lds);
    if (rc) return rc;
    hipLaunchKernelGGL(k_tile_factor, dim3(ntiles), dim3(256), lds, s, blocks, kk, minv, ridge);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_sgs_color(int mode, const double *r, double *y, long long npix, int nrhs,
                     const int *tilepix, const int *tiles, int ntl, const int *nbptr,
                     const int *nbs, const int *color, int kappa, const float *off,
                     const float *minv, hipStream_t s) {
    if (ntl <= 0) return MLCR_OK;
#define MLCR_SGS(MD)                                                                               \
    hipLaunchKernelGGL(k_sgs_color<MD>, dim3(ntl), dim3(256), 0, s, r, y, npix, nrhs, tilepix,     \
                       tiles, nbptr, nbs, color, kappa, off, minv)
    if (mode == 0) MLCR_SGS(0);
    else if (mode == 1) MLCR_SGS(1);
    else MLCR_SGS(2);
#undef MLCR_SGS
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_dense_lambda(const double *rz, const double *rs, int nrings, int L, double *lt,
                        hipStream_t s) {
    if (L > 127) return fail(MLCR_EUNSUPPORTED, "dense block band limit above 127");
    hipLaunchKernelGGL(k_dense_lambda, dim3(nrings), dim3(128), 0, s, rz, rs, L, lt);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_dense_ringdft(const double2 *Xi, int ldx, const double *lt, int L, int nrings,
                         const int *mode, int na, const double *d, const double *bh, double *A,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_dense_ringdft, dim3(nblk((long long)na * na, 256)), dim3(256), 0, s, Xi,
                       ldx, lt, L, nrings, mode, na, d, bh, A);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_dense_cholesky(double *a, int n, int *info, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_cholesky, dim3(1), dim3(1024), 0, s, a, n, info);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_dense_inverse(const double *L, int n, double *inv, hipStream_t s) {
    const size_t lds = (size_t)n * sizeof(double);
    if (lds > 150 * 1024) return fail(MLCR_EINVAL, "dense bottom level too large for LDS");
    int rc = ensure_dynamic_lds((const void *)k_dense_inverse, lds);
    if (rc) return rc;
    hipLaunchKernelGGL(k_dense_inverse, dim3(n), dim3(256), lds, s, L, n, inv);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

long long dense_apply_ws_doubles(int n, int nrhs) {
    return (long long)(1 + kDenseJS) * nrhs * n;
}

// ws: dense_apply_ws_doubles(n, nrhs) doubles.  x is cleared with a fill
// kernel (no memset node when a caller captures this in a graph).
int launch_dense_apply(const double *Ainv, int n, const int *act_idx, const double *b, double *x,
                       long long nalm, int nrhs, double *ws, hipStream_t s) {
    int rc;
    if ((rc = launch_fill_zero(x, (long long)nrhs * nalm, s))) return rc;
    double *g = ws, *part = ws + (long long)nrhs * n;
    const long long ne = (long long)n * nrhs;
    hipLaunchKernelGGL(k_dense_rhs, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, b, nalm,
                       act_idx, n, nrhs, g);
    hipLaunchKernelGGL(k_dense_partial, dim3((n + 63) / 64, kDenseJS, (nrhs + 7) / 8), dim3(256), 0,
                       s, Ainv, n, g, nrhs, part);
    hipLaunchKernelGGL(k_dense_finish, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, part, n,
                       nrhs, act_idx, x, nalm);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_dots(const double *a, const double *b, const double *c, const double *d, int lmax,
                int nrhs, double *partial, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_dots, dim3(lmax + 1, nrhs), dim3(256), 0, s, a, b, c, d, lmax, partial);
    MLCR_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_wnorms_final, dim3(nrhs), dim3(256), 0, s, partial, lmax + 1, out);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_ell_dots(const double *a, const double *b, int lmax, int nrhs, double *out,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_ell_dots, dim3(lmax + 1), dim3(256), 0, s, a, b, lmax, nrhs, out);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_lincomb(const double *u, const double *v, double *out, const double *al,
                   const double *be, long long n, int nrhs, hipStream_t s) {
    const long long blocks = std::min<long long>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_lincomb, dim3((unsigned)blocks, nrhs), dim3(256), 0, s, u, v, out, al, be,
                       n);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_cr_pix(const double *d, const double *w2, const double *ninv, double *pix,
                  long long npix, int nrhs, hipStream_t s) {
    const long long blocks = std::min<long long>((npix + 255) / 256, 4096);
    hipLaunchKernelGGL(k_cr_pix, dim3((unsigned)blocks, nrhs), dim3(256), 0, s, d, w2, ninv, pix,
                       npix);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_cr_combine(const double *v, const double *w1, const double *bh, const double *dd,
                      double *b, int lmax, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_cr_combine, dim3(lmax + 1, nrhs), dim3(256), 0, s, v, w1, bh, dd, b, lmax);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}


}  // namespace mlcr
