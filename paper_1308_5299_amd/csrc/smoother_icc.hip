// The paper's error-smoother construction (Sec. 3.5) on the GPU.
//
// The pixel-domain level operator A_hat_h = Y_h A_h Y_h^T = D_hat_h +
// B_hat_h^T N^-1 B_hat_h (eqs. pixel-domain, Dhat, Bhat) is approximated on the
// tile pattern -- a k x k tile and its neighbour tiles -- with the blocks
// computed directly:
//   * D_hat_h and B_hat_h are rotationally invariant, so an entry is the
//     addition-theorem sum g(theta) = sum_l (2l+1)/(4 pi) g_l P_l(cos theta)
//     (eq. addition-theorem) at the angle between the two pixel centres, with
//     g_l = f_l^2 / C_l (D_hat) or f_l b_l p_l (B_hat).  g is tabulated once per
//     level on a fine theta grid and read by four-point Lagrange interpolation.
//   * B_hat_h^T N^-1 B_hat_h is formed by block products without fill-in: the
//     block of tiles (t, u) sums over the observation pixels inside the tiles T
//     that are t or a neighbour of t and also u or a neighbour of u, i.e. only
//     through blocks (T, t) and (T, u) that lie in the pattern.
// The approximant is factored by a zero-fill block incomplete Cholesky in the
// order of the sweep colouring (tiles of one colour are never neighbours, so
// one colour is one parallel launch), with the smallest ridge alpha on the
// diagonal (found by bisection on the host) that lets every pivot succeed,
// times 1.5.  Blocks are float32 (the paper's smoother precision); products
// and the factorization of a block run in float64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "solver_internal.h"
#include "block_dev.h"

namespace mlcr {

constexpr int K2 = kTileK2;          // 64 pixels per tile

// g(theta_i), theta_i = i dth: Legendre series summed with the three-term
// recurrence of P_l (stable on [-1, 1]).
__global__ __launch_bounds__(256) void k_addthm_table(const double *__restrict__ gl, int lmax,
                                                      double dth, int ntab,
                                                      double *__restrict__ tab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntab) return;
    const double x = cos(i * dth);
    const double c = 0.07957747154594766788;      // 1 / (4 pi)
    double p0 = 1.0, p1 = x;
    double sum = c * gl[0];
    if (lmax >= 1) sum += 3.0 * c * gl[1] * x;
    for (int l = 2; l <= lmax; l++) {
        const double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
        sum += (2.0 * l + 1.0) * c * gl[l] * p2;
        p0 = p1;
        p1 = p2;
    }
    tab[i] = sum;
}

// g at the angle whose chord between unit vectors is ch (theta = 2 asin(ch/2),
// exact for close points), four-point Lagrange interpolation in theta
__device__ __forceinline__ double addthm(const AddThmTable &T, double ch) {
    const double th = 2.0 * asin(fmin(0.5 * ch, 1.0));
    const double u = th / T.dth;
    int i0 = (int)u - 1;
    i0 = min(max(i0, 0), T.n - 4);
    const double t = u - i0;
    const double *g = T.tab + i0;
    const double l0 = -(t - 1.0) * (t - 2.0) * (t - 3.0) / 6.0;
    const double l1 = t * (t - 2.0) * (t - 3.0) * 0.5;
    const double l2 = -t * (t - 1.0) * (t - 3.0) * 0.5;
    const double l3 = t * (t - 1.0) * (t - 2.0) / 6.0;
    return l0 * g[0] + l1 * g[1] + l2 * g[2] + l3 * g[3];
}

__device__ __forceinline__ double chord(const double *a, const double *b) {
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// One workgroup per block (t, u): job j < ntiles is the diagonal block of
// tile j, the others are the pairs in jobs[] (slot of t -> u with t < u; the
// block and its transpose are stored at slot and rev[slot]).  Thread tid owns
// entries (a = tid % 64, b = tid / 64 + 4 q), q < 16.
constexpr int kAsmCh = 64;           // observation pixels per staged chunk
__global__ __launch_bounds__(256) void k_smoother_assemble(
    int ntiles, const int *__restrict__ nbptr, const int *__restrict__ nbs,
    const int *__restrict__ rev, const int *__restrict__ jobs, const double *__restrict__ vlev,
    const double *__restrict__ vobs, const int *__restrict__ oring, const double *__restrict__ ninv,
    long long sub, AddThmTable gD, AddThmTable gB, float *__restrict__ diag,
    float *__restrict__ off) {
    __shared__ double vt[K2][3], vu[K2][3], vo[kAsmCh][3];
    __shared__ double wo[kAsmCh];
    __shared__ float bt[kAsmCh][K2], bu[kAsmCh][K2];
    __shared__ int cl[32];
    __shared__ int ncl;
    const int tid = threadIdx.x;
    const int j = blockIdx.x;
    int t, u, slot = -1;
    if (j < ntiles) {
        t = u = j;
    } else {
        slot = jobs[j - ntiles];
        // owner of the slot: the last t with nbptr[t] <= slot
        int lo = 0, hi = ntiles - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (nbptr[mid] <= slot) lo = mid;
            else hi = mid - 1;
        }
        t = lo;
        u = nbs[slot];
    }
    for (int e = tid; e < 3 * K2; e += blockDim.x) {
        vt[e / 3][e % 3] = vlev[(long long)t * K2 * 3 + e];
        vu[e / 3][e % 3] = vlev[(long long)u * K2 * 3 + e];
    }
    if (tid == 0) {
        // tiles T in ({t} + nb(t)) and ({u} + nb(u)), ascending
        int n = 0;
        auto in_u = [&](int T) {
            if (T == u) return true;
            for (int q = nbptr[u]; q < nbptr[u + 1]; q++)
                if (nbs[q] == T) return true;
            return false;
        };
        int q = nbptr[t];
        bool self = false;
        while (n < 32 && (q < nbptr[t + 1] || !self)) {
            int T;
            if (!self && (q >= nbptr[t + 1] || t < nbs[q])) {
                T = t;
                self = true;
            } else {
                T = nbs[q++];
            }
            if (in_u(T)) cl[n++] = T;
        }
        ncl = n;
    }
    __syncthreads();
    const int a = tid & (K2 - 1), b0 = tid >> 6;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; q++) acc[q] = addthm(gD, chord(vt[a], vu[b0 + 4 * q]));
    for (int c = 0; c < ncl; c++) {
        const long long base = (long long)cl[c] * sub;
        for (long long c0 = 0; c0 < sub; c0 += kAsmCh) {
            for (int e = tid; e < kAsmCh * 3; e += blockDim.x)
                vo[e / 3][e % 3] = vobs[(base + c0) * 3 + e];
            for (int e = tid; e < kAsmCh; e += blockDim.x) wo[e] = ninv[oring[base + c0 + e]];
            __syncthreads();
            for (int e = tid; e < kAsmCh * K2; e += blockDim.x) {
                const int i = e / K2, p = e % K2;
                bt[i][p] = (float)(wo[i] * addthm(gB, chord(vo[i], vt[p])));
                bu[i][p] = (float)addthm(gB, chord(vo[i], vu[p]));
            }
            __syncthreads();
            float part[16];
#pragma unroll
            for (int q = 0; q < 16; q++) part[q] = 0.f;
            for (int i = 0; i < kAsmCh; i++) {
                const float x = bt[i][a];
#pragma unroll
                for (int q = 0; q < 16; q++) part[q] = fmaf(x, bu[i][b0 + 4 * q], part[q]);
            }
#pragma unroll
            for (int q = 0; q < 16; q++) acc[q] += (double)part[q];
            __syncthreads();
        }
    }
    // column-major blocks: entry (a, b) at b * 64 + a
    if (slot < 0) {
        float *D = diag + (long long)t * K2 * K2;
#pragma unroll
        for (int q = 0; q < 16; q++) D[(b0 + 4 * q) * K2 + a] = (float)acc[q];
    } else {
        float *Bf = off + (long long)slot * K2 * K2;
        float *Br = off + (long long)rev[slot] * K2 * K2;
#pragma unroll
        for (int q = 0; q < 16; q++) {
            Bf[(b0 + 4 * q) * K2 + a] = (float)acc[q];
            Br[a * K2 + (b0 + 4 * q)] = (float)acc[q];
        }
    }
}

// slot of u -> k in u's neighbour list, or -1
__device__ __forceinline__ int find_slot(const int *nbptr, const int *nbs, int u, int k) {
    for (int q = nbptr[u]; q < nbptr[u + 1]; q++)
        if (nbs[q] == k) return q;
    return -1;
}

// One colour of the block ICC(0), one workgroup (256 threads) per tile t:
//   S = A_tt + shift I - sum_{k in nb(t), col(k) < col(t)} L_tk L_tk^T
//   L_tt = chol(S),  minv_t = L_tt^-1
//   for u in nb(t), col(u) > col(t):
//     L_ut = (A_ut - sum_{k in nb(t) and nb(u), col(k) < col(t)} L_uk L_tk^T) L_tt^-T
// Blocks in LDS in float64 (row-major), global blocks float32 column-major.
__global__ __launch_bounds__(256) void k_icc_color(const int *__restrict__ tiles,
                                                   const int *__restrict__ nbptr,
                                                   const int *__restrict__ nbs,
                                                   const int *__restrict__ rev,
                                                   const int *__restrict__ color, int kappa,
                                                   const float *__restrict__ adiag,
                                                   const float *__restrict__ aoff, double shift,
                                                   float *__restrict__ minv,
                                                   float *__restrict__ lslot,
                                                   int *__restrict__ fail) {
    extern __shared__ double smem[];
    double *S = smem;                       // K2 x K2
    double *X = S + K2 * K2;                // K2 x K2: L_tt^-1
    float *F1 = reinterpret_cast<float *>(X + K2 * K2);     // staged blocks
    float *F2 = F1 + K2 * K2;
    double *flag = reinterpret_cast<double *>(F2 + K2 * K2);
    const int t = tiles[blockIdx.x];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int a = tid & (K2 - 1), b0 = tid >> 6;
    // S from A_tt (column-major in global) with the ridge
    for (int e = tid; e < K2 * K2; e += nth) {
        const int r = e / K2, c = e % K2;
        S[e] = (double)adiag[(long long)t * K2 * K2 + c * K2 + r] + (r == c ? shift : 0.0);
    }
    __syncthreads();
    const int s0 = nbptr[t], s1 = nbptr[t + 1];
    for (int q0 = s0; q0 < s1; q0++) {
        if (!(color[nbs[q0]] < kappa)) continue;
        for (int e = tid; e < K2 * K2; e += nth) F1[e] = lslot[(long long)q0 * K2 * K2 + e];
        __syncthreads();
        // S[a][b] -= sum_j L_tk[a][j] L_tk[b][j]   (L_tk[r][c] = F1[c * K2 + r])
        for (int q = 0; q < 16; q++) {
            const int b = b0 + 4 * q;
            double sacc = 0.0;
            for (int jj = 0; jj < K2; jj++)
                sacc = fma((double)F1[jj * K2 + a], (double)F1[jj * K2 + b], sacc);
            S[a * K2 + b] -= sacc;
        }
        __syncthreads();
    }
    const bool ok = lds_cholesky(S, K2, flag);
    if (tid == 0 && !ok) fail[t] = 1;
    // X = L^-1: column c by forward substitution
    for (int e = tid; e < K2 * K2; e += nth) X[e] = 0.0;
    __syncthreads();
    for (int c = tid; c < K2; c += nth) {
        for (int i = c; i < K2; i++) {
            double sacc = (i == c) ? 1.0 : 0.0;
            for (int jj = c; jj < i; jj++) sacc -= S[i * K2 + jj] * X[jj * K2 + c];
            X[i * K2 + c] = sacc / S[i * K2 + i];
        }
    }
    __syncthreads();
    for (int e = tid; e < K2 * K2; e += nth) {
        const int r = e % K2, c = e / K2;              // column-major store
        minv[(long long)t * K2 * K2 + e] = (float)X[r * K2 + c];
    }
    // the later neighbours' blocks
    for (int q0 = s0; q0 < s1; q0++) {
        const int u = nbs[q0];
        if (!(color[u] > kappa)) continue;
        const int sut = rev[q0];                      // slot u -> t
        double racc[16];
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int b = b0 + 4 * q;
            racc[q] = (double)aoff[(long long)sut * K2 * K2 + b * K2 + a];   // A_ut[a][b]
        }
        for (int q1 = s0; q1 < s1; q1++) {
            const int k = nbs[q1];
            if (!(color[k] < kappa)) continue;
            const int suk = find_slot(nbptr, nbs, u, k);
            if (suk < 0) continue;
            __syncthreads();
            for (int e = tid; e < K2 * K2; e += nth) {
                F1[e] = lslot[(long long)suk * K2 * K2 + e];     // L_uk
                F2[e] = lslot[(long long)q1 * K2 * K2 + e];      // L_tk
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int b = b0 + 4 * q;
                double sacc = 0.0;
                for (int jj = 0; jj < K2; jj++)
                    sacc = fma((double)F1[jj * K2 + a], (double)F2[jj * K2 + b], sacc);
                racc[q] -= sacc;
            }
        }
        __syncthreads();
        // R into S (the factor is no longer needed), then L_ut = R X^T
#pragma unroll
        for (int q = 0; q < 16; q++) S[a * K2 + b0 + 4 * q] = racc[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int b = b0 + 4 * q;
            double sacc = 0.0;
            for (int jj = 0; jj <= b; jj++) sacc = fma(S[a * K2 + jj], X[b * K2 + jj], sacc);
            // L_ut at slot u -> t (column-major), its transpose at slot t -> u
            lslot[(long long)sut * K2 * K2 + b * K2 + a] = (float)sacc;
            lslot[(long long)q0 * K2 * K2 + a * K2 + b] = (float)sacc;
        }
        __syncthreads();
    }
}

// max over tiles of the largest diagonal entry of A_tt (one workgroup)
__global__ __launch_bounds__(1024) void k_max_diag(const float *__restrict__ adiag, int ntiles,
                                                   double *__restrict__ out) {
    __shared__ double red[1024];
    double m = 0.0;
    for (long long e = threadIdx.x; e < (long long)ntiles * K2; e += blockDim.x) {
        const long long t = e / K2, i = e % K2;
        m = fmax(m, fabs((double)adiag[t * K2 * K2 + i * K2 + i]));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

int launch_addthm_table(const double *gl, int lmax, double dth, int ntab, double *tab,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_addthm_table, dim3((ntab + 255) / 256), dim3(256), 0, s, gl, lmax, dth,
                       ntab, tab);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_smoother_assemble(int ntiles, const int *nbptr, const int *nbs, const int *rev,
                             const int *jobs, int njobs, const double *vlev, const double *vobs,
                             const int *oring, const double *ninv, long long sub, AddThmTable gD,
                             AddThmTable gB, float *diag, float *off, hipStream_t s) {
    if (sub % kAsmCh) return fail(MLCR_EINVAL, "observation pixels per tile not a multiple of 64");
    hipLaunchKernelGGL(k_smoother_assemble, dim3(ntiles + njobs), dim3(256), 0, s, ntiles, nbptr,
                       nbs, rev, jobs, vlev, vobs, oring, ninv, sub, gD, gB, diag, off);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_icc_color(const int *tiles, int ntl, const int *nbptr, const int *nbs, const int *rev,
                     const int *color, int kappa, const float *adiag, const float *aoff,
                     double shift, float *minv, float *lslot, int *failv, hipStream_t s) {
    if (ntl <= 0) return MLCR_OK;
    const size_t lds = 2 * (size_t)K2 * K2 * sizeof(double) + 2 * (size_t)K2 * K2 * sizeof(float) +
                       sizeof(double);
    int rc = ensure_dynamic_lds((const void *)k_icc_color, lds);
    if (rc) return rc;
    hipLaunchKernelGGL(k_icc_color, dim3(ntl), dim3(256), lds, s, tiles, nbptr, nbs, rev, color,
                       kappa, adiag, aoff, shift, minv, lslot, failv);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_max_diag(const float *adiag, int ntiles, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_max_diag, dim3(1), dim3(1024), 0, s, adiag, ntiles, out);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

}  // namespace mlcr
