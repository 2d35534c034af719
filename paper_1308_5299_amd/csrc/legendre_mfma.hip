// Legendre adjoint on the matrix cores.
//
// The transpose of the synthesis of Sec. 2.1 (eq. sh-synthesis), lambda_lm
// by the recurrence of Sec. 3.2, as per-order GEMMs contracting over rings:
//     V_m[l, c] = sum_ring Lambda_m[ring, l] G_m[ring, c]
// with c = (RHS, cos/sin), 16 columns (8 right-hand sides).  (The synthesis
// direction is in legendre_seg.hip.)  The recurrence
// seeds, the 2^-512 range scaling and the recurrence itself stay in
// float64 on the vector ALUs while the matrix cores contract: each lambda is
// staged through LDS and fed to v_mfma_f32_16x16x4f32 (T = float: float32
// products and accumulation, the mixed path) or v_mfma_f64_16x16x4f64
// (T = double: the float64 path).  Even and odd l - m are separate GEMMs
// (mirror-ring parity).
//
// MFMA 16x16x4 operand layout (lane = 0..63): A[i][k] in lane i + 16 k,
// B[k][j] in lane j + 16 k.  D[i][j] sits in lane j + 16 (i / 4), element
// i % 4 for float32, and in lane j + 16 (i % 4), element i / 4 for float64.
#include <algorithm>

#include "legendre_dev.h"

namespace mlcr {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;
template <>
struct Mma<float> {
    typedef f4 acc;
    static __device__ __forceinline__ acc zero() { return (f4){0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // row i of D held by lane group kq (= lane / 16) in element v
    static __device__ __forceinline__ int row(int kq, int v) { return 4 * kq + v; }
    static __device__ __forceinline__ float cvt(double v) { return (float)v; }
};
template <>
struct Mma<double> {
    typedef d4 acc;
    static __device__ __forceinline__ acc zero() { return (d4){0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int kq, int v) { return kq + 4 * v; }
    static __device__ __forceinline__ double cvt(double v) { return v; }
};

// complex element of G: float64 pairs on the float64 path, float32 pairs on
// the mixed path
template <typename T>
struct CplxOf;
template <>
struct CplxOf<float> {
    typedef float2 type;
};
template <>
struct CplxOf<double> {
    typedef double2 type;
};

// ---------------------------------------------------------------------------
// adjoint: one workgroup of W waves per (m, chunk of W ring-pair blocks, 8 RHS)
// ---------------------------------------------------------------------------
// Wave w owns ring-pair block chunk * W + w.  Per tile of 32 l (16 even +
// 16 odd l - m) every wave forms its block's contribution
//     D_even[l_i, c] = sum_k Lambda[ring_k, l_2i] g_even[ring_k, c]
// with 16 MFMAs of 4 ring pairs each (likewise odd): MFMA g takes ring pair
// 16 k + g as its k-th, so lane i + 16 k reads its 16 A values (row i,
// ring pairs 16 k .. 16 k + 15) with 16-byte LDS reads.  The W tiles are summed
// in LDS in the contraction type (float32 for the mixed path: 8 terms, about
// 5e-7 relative; float64 for the float64 path), and the chunk's partial sum
// is stored once (T layout, same type); the chunks are added in float64 in
// the unpack step.
// The float64 tile would take 135 KiB of LDS per 8-wave workgroup (one
// workgroup, 2 waves per SIMD): for T = double each tile runs the
// recurrence twice from the tile's start state, storing the 16 even steps
// and then the 16 odd steps in one half-size tile, so two workgroups fit
// per CU (4 waves per SIMD, registers held to 128).
template <typename T, int W>
__global__ __launch_bounds__(64 * W, sizeof(T) == 8 ? 4 : 1) void k_ladj_mfma(
    const typename CplxOf<T>::type *__restrict__ G, long long fstride, int nrhs,
    T *__restrict__ P, int lmax,
    const double *__restrict__ rz, const double *__restrict__ alpha,
    const long long *__restrict__ aboff, const double2 *__restrict__ st,
    const int *__restrict__ stsc, const int *__restrict__ lstab, int nb16, int nrings, int npairs,
    int npb, int nchunks, long long total) {
    typedef Mma<T> M;
    // lambda tile of one wave: row (parity p, index i) = 16 p + i, padded so
    // that rows stay 16-byte aligned and the 16 rows read by 16 lanes start
    // 4 banks apart
    constexpr int SL = sizeof(T) == 8 ? 66 : 68;
    constexpr bool TWO = sizeof(T) == 8;         // two passes, half-size tile
    constexpr int LS = (TWO ? 16 : 32) * SL;
    constexpr int VW = 16 / sizeof(T);           // values per 16-byte read
    // tiles per chunk sum: the float32 area holds 4 finished 32 x 16 tiles
    constexpr int KG = W < 2 ? 1 : (TWO ? 2 : 4);
    extern __shared__ __align__(16) unsigned char smem[];
    double *sab = reinterpret_cast<double *>(smem);
    T *lam_all = reinterpret_cast<T *>(smem + 2 * KG * kChunkM * sizeof(double));
    int m, chunk, rc;
    bool ok;
    decode_item_m<sizeof(T) == 8 ? kGroupF64 : kGroupF32>(total, lmax, nchunks, m, chunk, rc, ok);
    if (!ok) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T *lam = lam_all + wv * LS;
    const int nl = lmax - m + 1;
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    const int nrc = (nrhs + 7) / 8;
    const double *abm = alpha + aboff[m] - (m + 1);
    const int ld = lmax + 1;
    const int kq = lane >> 4, jc = lane & 15;
    T *Pm = P + (((long long)chunk * nrc + rc) * tri + tri_off_m(m, lmax)) * 16;
    const int rB = min(rc * 8 + (jc >> 1), nrhs - 1), csB = jc & 1;

    const int pb = chunk * W + wv;
    const bool active = pb < npb;                // wave-uniform
    // The recurrence starts at tile tw: the 32-aligned offset (start-state
    // table of the segment synthesis) below which every lambda of this block
    // is negligible, with the table's state there.  Tiles below t0 (the
    // workgroup's first) hold no contribution of any wave.
    Lane1 L;
    const int kp = pb * 64 + lane;
    const bool valid = active && kp < npairs;
    L.z = valid ? rz[kp] : 0.0;
    L.l1 = L.l2 = 0.0;
    L.sc = 1;
    const int ntile = (nl + 31) / 32;
    const int tw = active ? lstab[(long long)m * nb16 + 4 * pb] / 32 : ntile;
    int t0 = ntile;
    for (int w = 0; w < W; w++)
        if (chunk * W + w < npb) t0 = min(t0, lstab[(long long)m * nb16 + 4 * (chunk * W + w)] / 32);
    // B operands: ring pair 16 kq + g of this block, column jc
    T ge[16], go[16];
    {
        const T *Gr = reinterpret_cast<const T *>(G + (long long)rB * fstride);
#pragma unroll
        for (int g = 0; g < 16; g++) {
            const int p = pb * 64 + 16 * kq + g;
            double gn = 0.0, gs = 0.0;
            if (active && p < npairs) {
                const int north = p, south = nrings - 1 - p;
                gn = (double)Gr[((long long)north * ld + m) * 2 + csB];
                if (south != north) gs = (double)Gr[((long long)south * ld + m) * 2 + csB];
            }
            ge[g] = M::cvt(gn + gs);
            go[g] = M::cvt(gn - gs);
        }
    }
    // mode -1: before tw (or no block), 0: all lanes range-scaled, 1: some, 2: none
    int mode = -1;
    for (int o = threadIdx.x; o < min(32 * t0, nl) * 16; o += 64 * W) Pm[o] = (T)0;
    // coefficients of a group of KG tiles; group g + 1's are loaded while
    // group g computes
    auto coef_at = [&](int tg) {
        const int l = m + tg * 32 + (int)threadIdx.x;
        return ((int)threadIdx.x < KG * kChunkM && l + 1 <= lmax) ? abm[l + 1] : 0.0;
    };
    double cpre = coef_at(t0);
    if ((int)threadIdx.x < KG * kChunkM) sab[threadIdx.x] = cpre;
    if (t0 + KG < ntile) cpre = coef_at(t0 + KG);
    // the block's recurrence start state, read once here so that no global
    // load is pending inside the tile loop
    double2 s0 = make_double2(0.0, 0.0);
    int sc0 = 1;
    if (active && tw < ntile) {
        const long long tix = ((long long)m * nb16 + 4 * pb + (lane >> 4)) * 64 + (lane & 15);
        s0 = st[tix];
        sc0 = stsc[tix];
    }
    __builtin_amdgcn_s_waitcnt(0x0f70);         // vmcnt(0): G, the start state, coefficients
    __syncthreads();
    for (int tg = t0; tg < ntile; tg += KG) {
        // Coefficients of group gi sit in buffer gi & 1.  Those of group gi + 1
        // (loaded during group gi - 1's stores) go to the other buffer once this
        // group's tiles are done, before the first barrier: that buffer's last
        // readers (group gi - 1) are past the barriers that ended it, and by
        // then the load and the stores issued before it have long completed,
        // so the wait for it costs nothing.
        const int gi = (tg - t0) / KG;
        const double *sbg = sab + (gi & 1) * KG * kChunkM;
        typename M::acc DEg[KG], DOg[KG];
#pragma unroll
        for (int j = 0; j < KG; j++) {
            const int t = tg + j;
            const double *sb = sbg + j * kChunkM;
            typename M::acc DE = M::zero(), DO = DE;
            if (t < ntile) {
                if (t == tw) {
                    L.l1 = s0.x;
                    L.l2 = s0.y;
                    L.sc = sc0;
                    mode = wave_mode1(L);
                }
                if (mode <= 0) {
                    if (mode == 0) {
#pragma unroll
                        for (int q = 0; q < 8; q++) {
#pragma unroll
                            for (int s = 0; s < 4; s++) L.step(sb[4 * q + s]);
                            L.check_range();
                        }
                        mode = wave_mode1(L);
                    }
                } else if constexpr (TWO) {
                    // pass p stores the steps of parity p (rows 0..15), then its MFMAs
                    const Lane1 L0 = L;
#pragma unroll
                    for (int p = 0; p < 2; p++) {
                        if (p == 1) {
                            L = L0;
                            __builtin_amdgcn_wave_barrier();    // even rows read before rewriting
                        }
                        if (mode == 1) {
#pragma unroll 4
                            for (int s = 0; s < 32; s++) {
                                if ((s & 1) == p) lam[(s >> 1) * SL + lane] = L.w();
                                L.step_rescale(sb[s]);
                            }
                        } else {
#pragma unroll 8
                            for (int s = 0; s < 32; s++) {
                                if ((s & 1) == p) lam[(s >> 1) * SL + lane] = L.l1;
                                const double nv = fma(sb[s] * L.z, L.l1, -L.l2);
                                L.l2 = L.l1;
                                L.l1 = nv;
                            }
                        }
                        __builtin_amdgcn_s_waitcnt(0xc07f);     // this wave's LDS writes landed
                        __builtin_amdgcn_wave_barrier();
                        const T *rr = lam + jc * SL + 16 * kq;
#pragma unroll
                        for (int g0 = 0; g0 < 16; g0 += VW) {
                            typedef T v16 __attribute__((ext_vector_type(VW)));
                            const v16 a = *reinterpret_cast<const v16 *>(rr + g0);
#pragma unroll
                            for (int u = 0; u < VW; u++) {
                                if (p == 0) DE = M::mma(a[u], ge[g0 + u], DE);
                                else DO = M::mma(a[u], go[g0 + u], DO);
                            }
                        }
                    }
                    if (mode == 1) mode = wave_mode1(L);
                } else {
                    if (mode == 1) {
#pragma unroll 4
                        for (int s = 0; s < 32; s++) {
                            lam[((s & 1) * 16 + (s >> 1)) * SL + lane] = M::cvt(L.w());
                            L.step_rescale(sb[s]);
                        }
                        mode = wave_mode1(L);
                    } else {
                        // steady state: every lane in range, plain recurrence
#pragma unroll 8
                        for (int s = 0; s < 32; s++) {
                            lam[((s & 1) * 16 + (s >> 1)) * SL + lane] = M::cvt(L.l1);
                            const double nv = fma(sb[s] * L.z, L.l1, -L.l2);
                            L.l2 = L.l1;
                            L.l1 = nv;
                        }
                    }
                    __builtin_amdgcn_s_waitcnt(0xc07f);     // this wave's LDS writes landed
                    __builtin_amdgcn_wave_barrier();
                    const T *re = lam + jc * SL + 16 * kq;         // row (even, jc)
                    const T *ro = re + 16 * SL;                     // row (odd, jc)
#pragma unroll
                    for (int g0 = 0; g0 < 16; g0 += VW) {
                        typedef T v16 __attribute__((ext_vector_type(VW)));
                        const v16 ae = *reinterpret_cast<const v16 *>(re + g0);
                        const v16 ao = *reinterpret_cast<const v16 *>(ro + g0);
#pragma unroll
                        for (int u = 0; u < VW; u++) {
                            DE = M::mma(ae[u], ge[g0 + u], DE);
                            DO = M::mma(ao[u], go[g0 + u], DO);
                        }
                    }
                    // the next tile's lambdas overwrite this one's after its reads
                    __builtin_amdgcn_s_waitcnt(0xc07f);
                    __builtin_amdgcn_wave_barrier();
                }
            }
            DEg[j] = DE;
            DOg[j] = DO;
        }
        // the wave's KG tiles (32 l x 16 columns each) into its own LDS area;
        // the stores take the MFMA results, so they follow the wave's own
        // reads of its lambda tile; other waves read the area only between
        // the two barriers of a group
#pragma unroll
        for (int j = 0; j < KG; j++) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int i = M::row(kq, v);
                lam[j * 512 + (2 * i) * 16 + jc] = DEg[j][v];
                lam[j * 512 + (2 * i + 1) * 16 + jc] = DOg[j][v];
            }
        }
        // on every path: the coefficient load and the previous group's stores
        // are retired here, one group after they were issued, so that neither
        // the write below nor the next load waits on the stores issued next
        __builtin_amdgcn_s_waitcnt(0x0f70);     // vmcnt(0)
        if (tg + KG < ntile && (int)threadIdx.x < KG * kChunkM)
            sab[((gi + 1) & 1) * KG * kChunkM + threadIdx.x] = cpre;
        __syncthreads();
        // sum the W tiles; one store per output
        for (int o = threadIdx.x; o < 512 * KG; o += 64 * W) {
            const int j = o >> 9, lr = (o & 511) >> 4;
            const int lb = (tg + j) * 32 + lr;
            if (tg + j >= ntile || m + lb > lmax) continue;
            T a = (T)0;
#pragma unroll
            for (int w = 0; w < W; w++) a += lam_all[w * LS + o];
            Pm[(long long)lb * 16 + (o & 15)] = a;
        }
        // group gi + 2's coefficients, issued after this group's stores
        if (tg + 2 * KG < ntile) cpre = coef_at(tg + 2 * KG);
        __syncthreads();        // the tiles are read before the next lambdas overwrite them
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Waves per adjoint workgroup: one ring-pair block each, the path's tuned
// count (8 or 4), halved while it exceeds the number of blocks.
int adjoint_waves(const mlcr_geom *g, int prec) {
    const int npb = (g->npairs + 63) / 64;
    int w = g->tune[prec].adj_waves;
    while (w > 1 && w > npb) w >>= 1;
    return w;
}

// Split-K over ring-pair blocks: a workgroup sums W blocks for one order m,
// the chunks are added in the unpack step.
int adjoint_chunks_mfma(const mlcr_geom *g, int lmax, int prec) {
    (void)lmax;
    const int npb = (g->npairs + 63) / 64;
    const int W = adjoint_waves(g, prec);
    return (npb + W - 1) / W;
}

template <typename T, int W>
static int launch_ladj_wg(const LegendreArgs &a, const SegTable *st,
                          const typename CplxOf<T>::type *G, T *P,
                          int nchunks) {
    const mlcr_geom *g = a.g;
    const int npb = (g->npairs + 63) / 64;
    const int nrc = (a.nrhs + 7) / 8;
    const long long total = mitems<sizeof(T) == 8 ? kGroupF64 : kGroupF32>(a.lmax, nchunks, nrc);
    const long long grid = ((total + 7) / 8) * 8;
    const long long fstride = (long long)g->nrings * (a.lmax + 1);
    constexpr int KG = W < 2 ? 1 : (sizeof(T) == 8 ? 2 : 4);     // tiles per chunk sum
    const size_t lds = 2 * KG * kChunkM * sizeof(double) +
                       (size_t)W * (sizeof(T) == 8 ? 16 * 66 : 32 * 68) * sizeof(T);
    int rc = ensure_dynamic_lds((const void *)k_ladj_mfma<T, W>, lds);
    if (rc) return rc;
    hipLaunchKernelGGL((k_ladj_mfma<T, W>), dim3((unsigned)grid), dim3(64 * W), lds, a.stream, G,
                       fstride, a.nrhs, P, a.lmax, g->ring_z.as<double>(), g->alpha.as<double>(),
                       g->aboff.as<long long>(), st->st.as<double2>(), st->sc.as<int>(),
                       st->ls.as<int>(), 4 * npb, g->nrings, g->npairs, npb, nchunks, total);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

template <typename T>
static int launch_ladj_t(const LegendreArgs &a, const SegTable *st,
                         const typename CplxOf<T>::type *G, T *P,
                         int nchunks, int prec) {
    switch (adjoint_waves(a.g, prec)) {
    case 8: return launch_ladj_wg<T, 8>(a, st, G, P, nchunks);
    case 4: return launch_ladj_wg<T, 4>(a, st, G, P, nchunks);
    case 2: return launch_ladj_wg<T, 2>(a, st, G, P, nchunks);
    default: return launch_ladj_wg<T, 1>(a, st, G, P, nchunks);
    }
}

// P: double T layout with 8 RHS per chunk
int launch_legendre_adjoint_mfma(const LegendreArgs &a, const SegTable *st, const void *G,
                                 void *P, int *nchunks_out, bool dbl) {
    if (st->lmax != a.lmax) return fail(MLCR_EINVAL, "start-state table of another band limit");
    const int prec = dbl ? MLCR_FP64 : MLCR_FP32;
    const int nchunks = adjoint_chunks_mfma(a.g, a.lmax, prec);
    const int rc = dbl ? launch_ladj_t<double>(a, st, static_cast<const double2 *>(G), (double *)P,
                                               nchunks, prec)
                       : launch_ladj_t<float>(a, st, static_cast<const float2 *>(G), (float *)P,
                                              nchunks, prec);
    if (rc) return rc;
    *nchunks_out = nchunks;
    return MLCR_OK;
}

}  // namespace mlcr
