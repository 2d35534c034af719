// Legendre adjoint with split-bfloat16 products on the matrix cores.
//
// The same per-order GEMMs as the adjoint of legendre_mfma.hip (transpose of
// Sec. 2.1 eq. sh-synthesis, lambda_lm by the recurrence of Sec. 3.2), but each
// float32 operand f is carried as two bfloat16 numbers, hi = bf16(f) and
// lo = bf16(f - hi), and a product as hi*hi + hi*lo + lo*hi, three
// v_mfma_f32_16x16x32_bf16 with float32 accumulation.  |f - hi - lo| is at
// most 2^-18 |f| and the dropped lo*lo term at most 2^-18 of the product, so
// one product is good to about 3 * 2^-18 (1.1e-5) relative.  The recurrence,
// its seeds and its range scaling stay in float64 exactly as in the float32
// path; the split costs a few vector instructions per lambda, the contraction
// runs at the bfloat16 rate.
//
// v_mfma_f32_16x16x32_bf16 operands (lane = 0..63): A[i][k] in lane
// i + 16 (k / 8), element k % 8; B[k][j] in lane j + 16 (k / 8), element
// k % 8; D[i][j] in lane j + 16 (i / 4), element i % 4.  Even and odd l - m
// are separate GEMMs (mirror-ring parity); the contraction index k runs over
// 32 values of one parity.
#include <algorithm>

#include "legendre_dev.h"

namespace mlcr {

// ---------------------------------------------------------------------------
// adjoint: one workgroup of W waves per (m, chunk of W ring-pair blocks, 8 RHS)
// ---------------------------------------------------------------------------
// Wave w owns ring-pair block chunk * W + w.  Per tile of 32 l-steps each lane
// writes its ring's lambdas in float32 (row = (parity, l index), column =
// ring); lane i + 16 kg reads rings 32 c + 8 kg .. + 7 of row i (two 16-byte
// reads) and splits them into its hi and lo A operands; the B operand holds
// the split even/odd ring sums of G for the same rings; both 32-ring halves
// accumulate into one tile per parity.  The W tiles are summed in LDS in
// float32 (8 terms: about 5e-7 relative, well inside the split products'
// 1e-5) and the chunk's partial sum stored once (T layout, float32 partial
// sums, added in float64 by the unpack step).
template <int W>
__global__ __launch_bounds__(64 * W) void k_ladj_b3(
    const float2 *__restrict__ G, long long fstride, int nrhs, float *__restrict__ P, int lmax,
    const double *__restrict__ rz, const double *__restrict__ alpha,
    const long long *__restrict__ aboff, const double2 *__restrict__ st,
    const int *__restrict__ stsc, const int *__restrict__ lstab, int nb16, int nrings, int npairs,
    int npb, int nchunks, long long total) {
    constexpr int RW = 68;                      // floats per row: 64 rings + 4 pad; the
                                                // 16 rows read by 16 lanes start 4 banks apart
    constexpr int LSB = 32 * RW * 4;            // bytes per wave: [p * 16 + i][RW]
    // tiles per chunk sum: a wave's area holds 4 finished 32 x 16 tiles
    constexpr int KG = W < 2 ? 1 : 4;
    extern __shared__ __align__(16) unsigned char smem[];
    double *sab = reinterpret_cast<double *>(smem);
    unsigned char *lam_all = smem + 2 * KG * kChunkM * sizeof(double);
    int m, chunk, rc;
    bool ok;
    decode_item_m<kGroupF32>(total, lmax, nchunks, m, chunk, rc, ok);
    if (!ok) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float *lam = reinterpret_cast<float *>(lam_all + wv * LSB);
    float *tile = lam;
    const int nl = lmax - m + 1;
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    const int nrc = (nrhs + 7) / 8;
    const double *abm = alpha + aboff[m] - (m + 1);
    const int ld = lmax + 1;
    const int kg = lane >> 4, jc = lane & 15;
    float *Pm = P + (((long long)chunk * nrc + rc) * tri + tri_off_m(m, lmax)) * 16;
    const int rB = min(rc * 8 + (jc >> 1), nrhs - 1), csB = jc & 1;

    const int pb = chunk * W + wv;
    const bool active = pb < npb;               // wave-uniform
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
    // B operands [c][parity]: ring pairs 32 c + 8 kg + e of this block, column jc
    uint4 bh[2][2], bl[2][2];
    {
        const float *Gr = reinterpret_cast<const float *>(G + (long long)rB * fstride);
#pragma unroll
        for (int c = 0; c < 2; c++) {
            float ev[8], od[8];
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int p = pb * 64 + 32 * c + 8 * kg + e;
                double gn = 0.0, gs = 0.0;
                if (active && p < npairs) {
                    const int north = p, south = nrings - 1 - p;
                    gn = (double)Gr[((long long)north * ld + m) * 2 + csB];
                    if (south != north) gs = (double)Gr[((long long)south * ld + m) * 2 + csB];
                }
                ev[e] = (float)(gn + gs);
                od[e] = (float)(gn - gs);
            }
            split2(ev[0], ev[1], bh[c][0].x, bl[c][0].x);
            split2(ev[2], ev[3], bh[c][0].y, bl[c][0].y);
            split2(ev[4], ev[5], bh[c][0].z, bl[c][0].z);
            split2(ev[6], ev[7], bh[c][0].w, bl[c][0].w);
            split2(od[0], od[1], bh[c][1].x, bl[c][1].x);
            split2(od[2], od[3], bh[c][1].y, bl[c][1].y);
            split2(od[4], od[5], bh[c][1].z, bl[c][1].z);
            split2(od[6], od[7], bh[c][1].w, bl[c][1].w);
        }
    }
    // mode -1: before tw (or no block), 0: all lanes range-scaled, 1: some, 2: none
    int mode = -1;
    for (int o = threadIdx.x; o < min(32 * t0, nl) * 16; o += 64 * W) Pm[o] = 0.f;
    // coefficients of a group of KG tiles; group g + 1's are loaded while
    // group g computes
    auto coef_at = [&](int tg) {
        const int l = m + tg * 32 + (int)threadIdx.x;
        return ((int)threadIdx.x < KG * kChunkM && l + 1 <= lmax) ? abm[l + 1] : 0.0;
    };
    double cpre = coef_at(t0);
    if ((int)threadIdx.x < KG * kChunkM) sab[threadIdx.x] = cpre;
    if (t0 + KG < ntile) cpre = coef_at(t0 + KG);
    __syncthreads();
    for (int tg = t0; tg < ntile; tg += KG) {
        // coefficients of group gi in buffer gi & 1; those of group gi + 1 go
        // to the other buffer, whose last readers (group gi - 1) are past the
        // barriers that ended the previous group
        const int gi = (tg - t0) / KG;
        const double *sbg = sab + (gi & 1) * KG * kChunkM;
        if (tg + KG < ntile) {
            if ((int)threadIdx.x < KG * kChunkM) sab[((gi + 1) & 1) * KG * kChunkM + threadIdx.x] = cpre;
            if (tg + 2 * KG < ntile) cpre = coef_at(tg + 2 * KG);
        }
        f4b Dg[KG][2];
#pragma unroll
        for (int j = 0; j < KG; j++) {
            const int t = tg + j;
            const double *sb = sbg + j * kChunkM;
            f4b D[2] = {(f4b){0.f, 0.f, 0.f, 0.f}, (f4b){0.f, 0.f, 0.f, 0.f}};   // [parity]
            if (t < ntile) {
                if (t == tw) {
                    const long long tix = ((long long)m * nb16 + 4 * pb + (lane >> 4)) * 64 + (lane & 15);
                    const double2 s0 = st[tix];
                    L.l1 = s0.x;
                    L.l2 = s0.y;
                    L.sc = stsc[tix];
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
                } else {
                    // steps 2 i (even l - m, row i) and 2 i + 1 (odd, row 16 + i)
                    if (mode == 1) {
#pragma unroll 4
                        for (int i = 0; i < 16; i++) {
                            lam[i * RW + lane] = (float)L.w();
                            L.step_rescale(sb[2 * i]);
                            lam[(16 + i) * RW + lane] = (float)L.w();
                            L.step_rescale(sb[2 * i + 1]);
                        }
                        mode = wave_mode1(L);
                    } else {
#pragma unroll 8
                        for (int i = 0; i < 16; i++) {
                            lam[i * RW + lane] = (float)L.l1;
                            double nv = fma(sb[2 * i] * L.z, L.l1, -L.l2);
                            L.l2 = L.l1;
                            L.l1 = nv;
                            lam[(16 + i) * RW + lane] = (float)L.l1;
                            nv = fma(sb[2 * i + 1] * L.z, L.l1, -L.l2);
                            L.l2 = L.l1;
                            L.l1 = nv;
                        }
                    }
                    __builtin_amdgcn_s_waitcnt(0xc07f);     // this wave's LDS writes landed
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int p = 0; p < 2; p++)
#pragma unroll
                        for (int c = 0; c < 2; c++) {
                            const float4 *src = reinterpret_cast<const float4 *>(
                                lam + (16 * p + jc) * RW + 32 * c + 8 * kg);
                            const float4 f0 = src[0], f1 = src[1];
                            uint4 ah, al;
                            split2(f0.x, f0.y, ah.x, al.x);
                            split2(f0.z, f0.w, ah.y, al.y);
                            split2(f1.x, f1.y, ah.z, al.z);
                            split2(f1.z, f1.w, ah.w, al.w);
                            D[p] = mma_b3(ah, bh[c][p], D[p]);
                            D[p] = mma_b3(ah, bl[c][p], D[p]);
                            D[p] = mma_b3(al, bh[c][p], D[p]);
                        }
                    // the next tile's lambdas overwrite this one's after its reads
                    __builtin_amdgcn_s_waitcnt(0xc07f);
                    __builtin_amdgcn_wave_barrier();
                }
            }
            Dg[j][0] = D[0];
            Dg[j][1] = D[1];
        }
        // the wave's KG tiles (32 l x 16 columns each) into its own LDS area;
        // the stores take the MFMA results, so they follow the wave's own
        // reads of its lambda tile; other waves read the area only between
        // the two barriers of a group
#pragma unroll
        for (int j = 0; j < KG; j++) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int i = 4 * kg + v;
                tile[j * 512 + (2 * i) * 16 + jc] = Dg[j][0][v];
                tile[j * 512 + (2 * i + 1) * 16 + jc] = Dg[j][1][v];
            }
        }
        __syncthreads();
        // sum the W tiles; one store per output
        for (int o = threadIdx.x; o < 512 * KG; o += 64 * W) {
            const int j = o >> 9, lr = (o & 511) >> 4;
            const int lb = (tg + j) * 32 + lr;
            if (tg + j >= ntile || m + lb > lmax) continue;
            float a = 0.f;
#pragma unroll
            for (int w = 0; w < W; w++) a += reinterpret_cast<const float *>(lam_all + w * LSB)[o];
            Pm[(long long)lb * 16 + (o & 15)] = a;
        }
        __syncthreads();        // the tiles are read before the next lambdas overwrite them
    }
}

// ---------------------------------------------------------------------------
// adjoint over CB column blocks: one workgroup of W waves per (m, chunk of W
// ring-pair blocks, 8 CB RHS)
// ---------------------------------------------------------------------------
// As k_ladj_b3, but each lambda tile, written once and split once, meets the
// B operands of CB column blocks (RHS chunks CB rw + cb, 8 RHS each): 12 CB
// MFMAs per tile instead of 12, so the recurrence, the LDS transpose and the
// split of the A operands are shared by 8 CB right-hand sides.  Each chunk's
// partial sum goes to its own slice of P (the layout k_ladj_b3 writes, so the
// unpack step is unchanged); column blocks past the last chunk are skipped
// (wave-uniform).
template <int W, int CB>
__global__ __launch_bounds__(64 * W) void k_ladj_b3w(
    const float2 *__restrict__ G, long long fstride, int nrhs, float *__restrict__ P, int lmax,
    const double *__restrict__ rz, const double *__restrict__ alpha,
    const long long *__restrict__ aboff, const double2 *__restrict__ st,
    const int *__restrict__ stsc, const int *__restrict__ lstab, int nb16, int nrings, int npairs,
    int npb, int nchunks, long long total) {
    constexpr int RW = 68;
    constexpr int LSB = 32 * RW * 4;
    static_assert(CB * 512 <= 32 * RW, "the wave's tiles fit its lambda area");
    extern __shared__ __align__(16) unsigned char smem[];
    double *sab = reinterpret_cast<double *>(smem);
    unsigned char *lam_all = smem + kChunkM * sizeof(double2);
    int m, chunk, rw;
    bool ok;
    decode_item_m<kGroupF32>(total, lmax, nchunks, m, chunk, rw, ok);
    if (!ok) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float *lam = reinterpret_cast<float *>(lam_all + wv * LSB);
    float *tile = lam;
    const int nl = lmax - m + 1;
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    const int nrc = (nrhs + 7) / 8;
    const int ncb = min(CB, nrc - rw * CB);              // wave-uniform, >= 1
    const double *abm = alpha + aboff[m] - (m + 1);
    const int ld = lmax + 1;
    const int kg = lane >> 4, jc = lane & 15;
    auto Pm = [&](int cb) {
        return P + (((long long)chunk * nrc + rw * CB + cb) * tri + tri_off_m(m, lmax)) * 16;
    };

    const int pb = chunk * W + wv;
    const bool active = pb < npb;
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
    // B operands [cb][c][parity]: ring pairs 32 c + 8 kg + e of this block, column jc
    uint4 bh[CB][2][2], bl[CB][2][2];
#pragma unroll
    for (int cb = 0; cb < CB; cb++) {
        const int rB = min((rw * CB + cb) * 8 + (jc >> 1), nrhs - 1), csB = jc & 1;
        const float *Gr = reinterpret_cast<const float *>(G + (long long)rB * fstride);
#pragma unroll
        for (int c = 0; c < 2; c++) {
            float ev[8], od[8];
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int p = pb * 64 + 32 * c + 8 * kg + e;
                double gn = 0.0, gs = 0.0;
                if (cb < ncb && active && p < npairs) {
                    const int north = p, south = nrings - 1 - p;
                    gn = (double)Gr[((long long)north * ld + m) * 2 + csB];
                    if (south != north) gs = (double)Gr[((long long)south * ld + m) * 2 + csB];
                }
                ev[e] = (float)(gn + gs);
                od[e] = (float)(gn - gs);
            }
            split2(ev[0], ev[1], bh[cb][c][0].x, bl[cb][c][0].x);
            split2(ev[2], ev[3], bh[cb][c][0].y, bl[cb][c][0].y);
            split2(ev[4], ev[5], bh[cb][c][0].z, bl[cb][c][0].z);
            split2(ev[6], ev[7], bh[cb][c][0].w, bl[cb][c][0].w);
            split2(od[0], od[1], bh[cb][c][1].x, bl[cb][c][1].x);
            split2(od[2], od[3], bh[cb][c][1].y, bl[cb][c][1].y);
            split2(od[4], od[5], bh[cb][c][1].z, bl[cb][c][1].z);
            split2(od[6], od[7], bh[cb][c][1].w, bl[cb][c][1].w);
        }
    }
    int mode = -1;
    for (int cb = 0; cb < ncb; cb++) {
        float *pz = Pm(cb);
        for (int o = threadIdx.x; o < min(32 * t0, nl) * 16; o += 64 * W) pz[o] = 0.f;
    }
    auto coef_at = [&](int t) {
        const int l = m + t * 32 + (int)threadIdx.x;
        return (threadIdx.x < kChunkM && l + 1 <= lmax) ? abm[l + 1] : 0.0;
    };
    double cpre = coef_at(t0);
    if (threadIdx.x < kChunkM) sab[threadIdx.x] = cpre;
    if (t0 + 1 < ntile) cpre = coef_at(t0 + 1);
    __syncthreads();
    for (int t = t0; t < ntile; t++) {
        const double *sb = sab + ((t - t0) & 1) * kChunkM;
        if (t + 1 < ntile) {
            if (threadIdx.x < kChunkM) sab[((t + 1 - t0) & 1) * kChunkM + threadIdx.x] = cpre;
            if (t + 2 < ntile) cpre = coef_at(t + 2);
        }
        if (t == tw) {
            const long long tix = ((long long)m * nb16 + 4 * pb + (lane >> 4)) * 64 + (lane & 15);
            const double2 s0 = st[tix];
            L.l1 = s0.x;
            L.l2 = s0.y;
            L.sc = stsc[tix];
            mode = wave_mode1(L);
        }
        f4b D[CB][2];
#pragma unroll
        for (int cb = 0; cb < CB; cb++) D[cb][0] = D[cb][1] = (f4b){0.f, 0.f, 0.f, 0.f};
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
        } else {
            if (mode == 1) {
#pragma unroll 4
                for (int i = 0; i < 16; i++) {
                    lam[i * RW + lane] = (float)L.w();
                    L.step_rescale(sb[2 * i]);
                    lam[(16 + i) * RW + lane] = (float)L.w();
                    L.step_rescale(sb[2 * i + 1]);
                }
                mode = wave_mode1(L);
            } else {
#pragma unroll 8
                for (int i = 0; i < 16; i++) {
                    lam[i * RW + lane] = (float)L.l1;
                    double nv = fma(sb[2 * i] * L.z, L.l1, -L.l2);
                    L.l2 = L.l1;
                    L.l1 = nv;
                    lam[(16 + i) * RW + lane] = (float)L.l1;
                    nv = fma(sb[2 * i + 1] * L.z, L.l1, -L.l2);
                    L.l2 = L.l1;
                    L.l1 = nv;
                }
            }
            __builtin_amdgcn_s_waitcnt(0xc07f);     // this wave's LDS writes landed
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int p = 0; p < 2; p++)
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const float4 *src =
                        reinterpret_cast<const float4 *>(lam + (16 * p + jc) * RW + 32 * c + 8 * kg);
                    const float4 f0 = src[0], f1 = src[1];
                    uint4 ah, al;
                    split2(f0.x, f0.y, ah.x, al.x);
                    split2(f0.z, f0.w, ah.y, al.y);
                    split2(f1.x, f1.y, ah.z, al.z);
                    split2(f1.z, f1.w, ah.w, al.w);
#pragma unroll
                    for (int cb = 0; cb < CB; cb++)
                        if (cb < ncb) D[cb][p] = mma_b3(ah, bh[cb][c][p], D[cb][p]);
#pragma unroll
                    for (int cb = 0; cb < CB; cb++)
                        if (cb < ncb) D[cb][p] = mma_b3(ah, bl[cb][c][p], D[cb][p]);
#pragma unroll
                    for (int cb = 0; cb < CB; cb++)
                        if (cb < ncb) D[cb][p] = mma_b3(al, bh[cb][c][p], D[cb][p]);
                }
        }
        // the wave's CB tiles (32 l x 16 columns each) into its own LDS area;
        // the stores take the MFMA results, so they follow the wave's reads
#pragma unroll
        for (int cb = 0; cb < CB; cb++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int i = 4 * kg + v;
                tile[cb * 512 + (2 * i) * 16 + jc] = D[cb][0][v];
                tile[cb * 512 + (2 * i + 1) * 16 + jc] = D[cb][1][v];
            }
        __syncthreads();
        const int lb0 = t * 32;
        for (int o = threadIdx.x; o < 512 * ncb; o += 64 * W) {
            const int cb = o >> 9, oo = o & 511, lr = oo >> 4;
            if (m + lb0 + lr > lmax) continue;
            float a = 0.f;
#pragma unroll
            for (int w = 0; w < W; w++) a += reinterpret_cast<const float *>(lam_all + w * LSB)[o];
            Pm(cb)[(long long)(lb0 + lr) * 16 + (oo & 15)] = a;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int W>
static int launch_ladj_b3_w(const LegendreArgs &a, const SegTable *st, const float2 *G, float *P,
                            int nchunks) {
    const mlcr_geom *g = a.g;
    const int npb = (g->npairs + 63) / 64;
    const int nrc = (a.nrhs + 7) / 8;
    const long long total = mitems<kGroupF32>(a.lmax, nchunks, nrc);
    const long long grid = ((total + 7) / 8) * 8;
    const long long fstride = (long long)g->nrings * (a.lmax + 1);
    constexpr int KG = W < 2 ? 1 : 4;           // tiles per chunk sum
    const size_t lds = 2 * KG * kChunkM * sizeof(double) + (size_t)W * (32 * 68 * 4);
    int rc = ensure_dynamic_lds((const void *)k_ladj_b3<W>, lds);
    if (rc) return rc;
    hipLaunchKernelGGL((k_ladj_b3<W>), dim3((unsigned)grid), dim3(64 * W), lds, a.stream, G,
                       fstride, a.nrhs, P, a.lmax, g->ring_z.as<double>(), g->alpha.as<double>(),
                       g->aboff.as<long long>(), st->st.as<double2>(), st->sc.as<int>(),
                       st->ls.as<int>(), 4 * npb, g->nrings, g->npairs, npb, nchunks, total);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

template <int W, int CB>
static int launch_ladj_b3w(const LegendreArgs &a, const SegTable *st, const float2 *G, float *P,
                           int nchunks) {
    const mlcr_geom *g = a.g;
    const int npb = (g->npairs + 63) / 64;
    const int nrc = (a.nrhs + 7) / 8;
    const int nrw = (nrc + CB - 1) / CB;
    const long long total = mitems<kGroupF32>(a.lmax, nchunks, nrw);
    const long long grid = ((total + 7) / 8) * 8;
    const long long fstride = (long long)g->nrings * (a.lmax + 1);
    const size_t lds = kChunkM * sizeof(double2) + (size_t)W * (32 * 68 * 4);
    int rc = ensure_dynamic_lds((const void *)k_ladj_b3w<W, CB>, lds);
    if (rc) return rc;
    hipLaunchKernelGGL((k_ladj_b3w<W, CB>), dim3((unsigned)grid), dim3(64 * W), lds, a.stream, G,
                       fstride, a.nrhs, P, a.lmax, g->ring_z.as<double>(), g->alpha.as<double>(),
                       g->aboff.as<long long>(), st->st.as<double2>(), st->sc.as<int>(),
                       st->ls.as<int>(), 4 * npb, g->nrings, g->npairs, npb, nchunks, total);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

// Same split-K chunking (with this path's tuned waves per workgroup) and P
// layout as the float32 adjoint.
int launch_legendre_adjoint_b3(const LegendreArgs &a, const SegTable *st, const float2 *G,
                               float *P, int *nchunks_out) {
    if (st->lmax != a.lmax) return fail(MLCR_EINVAL, "start-state table of another band limit");
    const int nchunks = adjoint_chunks_mfma(a.g, a.lmax, MLCR_BF16X3);
    const int W = adjoint_waves(a.g, MLCR_BF16X3);
    int rc;
    if (bf16_synth_cols(a.nrhs) == 2 && W <= 4) {
        // two column blocks share each lambda tile; with 8-wave workgroups its
        // 143 registers leave one workgroup per CU, so the 8-wave shape keeps
        // the one-block kernel (the autotuner chooses between them)
        if (W == 4) rc = launch_ladj_b3w<4, 2>(a, st, G, P, nchunks);
        else if (W == 2) rc = launch_ladj_b3w<2, 2>(a, st, G, P, nchunks);
        else rc = launch_ladj_b3w<1, 2>(a, st, G, P, nchunks);
    } else if (W == 8) rc = launch_ladj_b3_w<8>(a, st, G, P, nchunks);
    else if (W == 4) rc = launch_ladj_b3_w<4>(a, st, G, P, nchunks);
    else if (W == 2) rc = launch_ladj_b3_w<2>(a, st, G, P, nchunks);
    else rc = launch_ladj_b3_w<1>(a, st, G, P, nchunks);
    if (rc) return rc;
    *nchunks_out = nchunks;
    return MLCR_OK;
}

}  // namespace mlcr
