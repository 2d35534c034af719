// Legendre step on the matrix cores (float32 contraction, float64 recurrence).
//
// Same transforms as legendre.hip (Sec. 2.1 eq. sh-synthesis and its
// transpose, lambda_lm of Sec. 3.2), written as per-order GEMMs:
//     synthesis  F_m[ring, c] = sum_l Lambda_m[ring, l] U_m[l, c]
//     adjoint    V_m[l, c]    = sum_ring Lambda_m[ring, l] G_m[ring, c]
// with c = (RHS, cos/sin), 16 columns (8 right-hand sides).  The recurrence
// seeds, the 2^-512 range scaling and the recurrence itself stay in
// float64 on the vector ALUs; each lambda is rounded once to float32, staged
// through LDS and fed to v_mfma_f32_16x16x4f32 (float32 products, float32
// accumulation).  Even and odd l - m are separate GEMMs (mirror-ring parity).
//
// MFMA 16x16x4 operand layout (lane = 0..63): A[i][k] in lane i + 16 k,
// B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i / 4), element i % 4.
#include <algorithm>

#include "mlcr_internal.h"

namespace mlcr {

typedef float f4 __attribute__((ext_vector_type(4)));

static constexpr int kScaleStepM = 512;
static constexpr int kSeedMinExpM = -112;
static constexpr int kChunkM = 32;

__device__ __forceinline__ void seed_lambda_m(double s, int m, double c, double &lam, int &k) {
    int es;
    const double fs = frexp(s, &es);
    double mant = 1.0, b = fs;
    int me = 0, be = es;
    for (int e = m; e;) {
        if (e & 1) {
            int t;
            mant = frexp(mant * b, &t);
            me += be + t;
        }
        e >>= 1;
        if (e) {
            int t;
            b = frexp(b * b, &t);
            be = 2 * be + t;
        }
    }
    int t;
    const double v = frexp(mant * c, &t);
    const int ex = me + t;
    if (ex >= kSeedMinExpM) {
        lam = ldexp(v, ex);
        k = 0;
    } else {
        k = (kSeedMinExpM - ex + kScaleStepM - 1) / kScaleStepM;
        lam = ldexp(v, ex + kScaleStepM * k);
    }
}

__device__ __forceinline__ void decode_item_m(long long total, int lmax, int npb, int &m, int &pb,
                                              int &rc, bool &ok) {
    const long long b = blockIdx.x;
    const long long per = (total + 7) / 8;
    const long long w = (b & 7) * per + (b >> 3);
    ok = w < total;
    if (!ok) return;
    const int nm = lmax + 1;
    const int mi = (int)(w % nm);
    const long long rest = w / nm;
    pb = (int)(rest % npb);
    rc = (int)(rest / npb);
    m = (mi & 1) ? (lmax - (mi >> 1)) : (mi >> 1);
}

__device__ __forceinline__ long long tri_off_m(int m, int lmax) {
    return (long long)m * (lmax + 1) - (long long)m * (m - 1) / 2;
}

// one ring pair per lane
struct Lane1 {
    int sc;
    double z, l1, l2;
    __device__ __forceinline__ void step_rescale(double2 c) {
        const double nv = fma(c.x, z * l1, -c.y * l2);
        l2 = l1;
        l1 = nv;
        if (sc > 0 && fabs(nv) >= 0x1p400) {
            l1 *= 0x1p-512;
            l2 *= 0x1p-512;
            sc--;
        }
    }
    __device__ __forceinline__ float w() const { return sc == 0 ? (float)l1 : 0.0f; }
};

__device__ __forceinline__ int wave_mode1(const Lane1 &L) {
    if (__all(L.sc == 0)) return 2;
    if (__all(L.sc > 0)) return 0;
    return 1;
}

// ---------------------------------------------------------------------------
// synthesis: one wave per (m, 64 ring pairs, 8 RHS)
// ---------------------------------------------------------------------------
// U32: float T layout [RHS chunk][m][l - m][8][cos, sin] (16 floats per l)
__global__ __launch_bounds__(64) void k_lsynth_mfma32(
    const float *__restrict__ U32, int nrhs, double2 *__restrict__ F, long long fstride, int lmax,
    const double *__restrict__ rz, const double *__restrict__ rs, const double2 *__restrict__ ab,
    const long long *__restrict__ aboff, const double *__restrict__ seedc, int nrings, int npairs,
    int npb, long long total) {
    __shared__ double2 sab[kChunkM];
    __shared__ float su[kChunkM * 16];
    __shared__ float lam[8][64];
    int m, pb, rc;
    bool ok;
    decode_item_m(total, lmax, npb, m, pb, rc, ok);
    if (!ok) return;
    const int lane = threadIdx.x;
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    const float *Um = U32 + ((long long)rc * tri + tri_off_m(m, lmax)) * 16;
    const double2 *abm = ab + aboff[m] - (m + 1);
    const int nl = lmax - m + 1;

    Lane1 L;
    const int kp = pb * 64 + lane;
    const bool valid = kp < npairs;
    L.z = valid ? rz[kp] : 0.0;
    seed_lambda_m(valid ? rs[kp] : 1.0, m, seedc[m], L.l1, L.sc);
    L.l2 = 0.0;

    f4 CE[4], CO[4];
#pragma unroll
    for (int b = 0; b < 4; b++) CE[b] = CO[b] = (f4){0.f, 0.f, 0.f, 0.f};
    int mode = wave_mode1(L);
    const int kq = lane >> 4, jc = lane & 15;

    const int nchunks = (nl + kChunkM - 1) / kChunkM;
    for (int k = 0; k < nchunks; k++) {
        // stage the chunk's coefficients (A, B of l -> l+1; U at l)
        __syncthreads();
        if (lane < kChunkM) {
            const int l = m + k * kChunkM + lane;
            sab[lane] = (l + 1 <= lmax) ? abm[l + 1] : make_double2(0.0, 0.0);
        }
        {
            const int base = k * kChunkM;
            // 32 l x 16 floats = 128 float4: two per lane
            for (int q = lane; q < kChunkM * 4; q += 64) {
                const int jl = q >> 2, part = q & 3;
                const float4 v = (base + jl < nl)
                                     ? reinterpret_cast<const float4 *>(Um + (long long)(base + jl) * 16)[part]
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
                reinterpret_cast<float4 *>(su + jl * 16)[part] = v;
            }
        }
        __syncthreads();
        const int jend = min(kChunkM, nl - k * kChunkM);
#pragma unroll 1
        for (int j0 = 0; j0 < jend; j0 += 8) {
            // 8 steps l = m + k*C + j0 + s, s = 0..7 (even s: even l - m)
            if (mode == 0) {
#pragma unroll
                for (int s = 0; s < 8; s++) L.step_rescale(sab[j0 + s]);
                mode = wave_mode1(L);
                continue;
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < 8; s++) {
                lam[s][lane] = L.w();
                L.step_rescale(sab[j0 + s]);
            }
            mode = wave_mode1(L);
            __syncthreads();
            const float be = su[(j0 + 2 * kq) * 16 + jc];
            const float bo = su[(j0 + 2 * kq + 1) * 16 + jc];
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const float ae = lam[2 * kq][16 * b + jc];
                const float ao = lam[2 * kq + 1][16 * b + jc];
                CE[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ae, be, CE[b], 0, 0, 0);
                CO[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ao, bo, CO[b], 0, 0, 0);
            }
        }
    }
    // D[i][j] of block b: ring pair 16 b + 4 kq + v, column j = jc = (rhs, cos/sin)
    const int r = rc * 8 + (jc >> 1), cs = jc & 1;
    const int ld = lmax + 1;
    if (r < nrhs) {
        double *Fr = reinterpret_cast<double *>(F + (long long)r * fstride);
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int p = pb * 64 + 16 * b + 4 * kq + v;
                if (p >= npairs) continue;
                const double e = (double)CE[b][v], o = (double)CO[b][v];
                const int north = p, south = nrings - 1 - p;
                Fr[((long long)north * ld + m) * 2 + cs] = e + o;
                if (south != north) Fr[((long long)south * ld + m) * 2 + cs] = e - o;
            }
    }
}

// ---------------------------------------------------------------------------
// adjoint: one wave per (m, chunk of ring-pair blocks, 8 RHS)
// ---------------------------------------------------------------------------
// Per tile of 32 l (16 even + 16 odd l - m) and 64 ring pairs:
// D_even[l_i, c] += sum_{k} Lambda[ring_k, l_2i] g_even[ring_k, c] over 16 MFMAs of
// 4 ring pairs each; likewise odd.  The tile result is stored (first block
// of the chunk) or added to the chunk's partial sums P (double, T layout).
__global__ __launch_bounds__(64) void k_ladj_mfma32(
    const double2 *__restrict__ G, long long fstride, int nrhs, double *__restrict__ P,
    int pb_per_chunk, int lmax, const double *__restrict__ rz, const double *__restrict__ rs,
    const double2 *__restrict__ ab, const long long *__restrict__ aboff,
    const double *__restrict__ seedc, int nrings, int npairs, int npb, int nchunks,
    long long total) {
    __shared__ double2 sab[kChunkM];
    __shared__ float lam[32][65];
    int m, chunk, rc;
    bool ok;
    decode_item_m(total, lmax, nchunks, m, chunk, rc, ok);
    if (!ok) return;
    const int lane = threadIdx.x;
    const int nl = lmax - m + 1;
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    const int nrc = (nrhs + 7) / 8;
    const double2 *abm = ab + aboff[m] - (m + 1);
    const int ld = lmax + 1;
    const int kq = lane >> 4, jc = lane & 15;
    double *Pm = P + (((long long)chunk * nrc + rc) * tri + tri_off_m(m, lmax)) * 16;
    const int rB = min(rc * 8 + (jc >> 1), nrhs - 1), csB = jc & 1;

    for (int pbi = 0; pbi < pb_per_chunk; pbi++) {
        const int pb = chunk * pb_per_chunk + pbi;
        if (pb >= npb) break;
        const bool first = (pbi == 0);
        Lane1 L;
        const int kp = pb * 64 + lane;
        const bool valid = kp < npairs;
        L.z = valid ? rz[kp] : 0.0;
        seed_lambda_m(valid ? rs[kp] : 1.0, m, seedc[m], L.l1, L.sc);
        L.l2 = 0.0;
        // B operands: ring pair 4 g + kq of this block, column jc
        float ge[16], go[16];
        {
            const double *Gr = reinterpret_cast<const double *>(G + (long long)rB * fstride);
#pragma unroll
            for (int g = 0; g < 16; g++) {
                const int p = pb * 64 + 4 * g + kq;
                double gn = 0.0, gs = 0.0;
                if (p < npairs) {
                    const int north = p, south = nrings - 1 - p;
                    gn = Gr[((long long)north * ld + m) * 2 + csB];
                    if (south != north) gs = Gr[((long long)south * ld + m) * 2 + csB];
                }
                ge[g] = (float)(gn + gs);
                go[g] = (float)(gn - gs);
            }
        }
        int mode = wave_mode1(L);
        // tiles of 32 l; a tile never spans two coefficient chunks (both 32)
        const int ntile = (nl + 31) / 32;
        for (int t = 0; t < ntile; t++) {
            __syncthreads();
            if (lane < kChunkM) {
                const int l = m + t * 32 + lane;
                sab[lane] = (l + 1 <= lmax) ? abm[l + 1] : make_double2(0.0, 0.0);
            }
            __syncthreads();
            const int lb0 = m + t * 32;
            if (mode == 0) {
#pragma unroll 4
                for (int s = 0; s < 32; s++) L.step_rescale(sab[s]);
                mode = wave_mode1(L);
                if (first) {
                    // no contribution from this block: store zeros for the tile
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int i = 4 * kq + v;
                        if (lb0 + 2 * i <= lmax) Pm[(long long)(2 * i + t * 32) * 16 + jc] = 0.0;
                        if (lb0 + 2 * i + 1 <= lmax) Pm[(long long)(2 * i + 1 + t * 32) * 16 + jc] = 0.0;
                    }
                }
                continue;
            }
#pragma unroll 4
            for (int s = 0; s < 32; s++) {
                lam[s][lane] = L.w();
                L.step_rescale(sab[s]);
            }
            mode = wave_mode1(L);
            __syncthreads();
            f4 DE = (f4){0.f, 0.f, 0.f, 0.f}, DO = DE;
#pragma unroll
            for (int g = 0; g < 16; g++) {
                const float ae = lam[2 * jc][4 * g + kq];
                const float ao = lam[2 * jc + 1][4 * g + kq];
                DE = __builtin_amdgcn_mfma_f32_16x16x4f32(ae, ge[g], DE, 0, 0, 0);
                DO = __builtin_amdgcn_mfma_f32_16x16x4f32(ao, go[g], DO, 0, 0, 0);
            }
            // D row i = l index within the parity, column jc = (rhs, cos/sin)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int i = 4 * kq + v;
                const int le = 2 * i, lo = 2 * i + 1;
                if (lb0 + le <= lmax) {
                    double *p = Pm + (long long)(le + t * 32) * 16 + jc;
                    if (first) *p = (double)DE[v];
                    else *p += (double)DE[v];
                }
                if (lb0 + lo <= lmax) {
                    double *p = Pm + (long long)(lo + t * 32) * 16 + jc;
                    if (first) *p = (double)DO[v];
                    else *p += (double)DO[v];
                }
            }
        }
    }
}

// float T layout: U32[rc][tri_off(m) + l - m][8][cs] = dl[l] x[...]
__global__ __launch_bounds__(256) void k_pack_t32(const double *__restrict__ x,
                                                  const double *__restrict__ dl,
                                                  float *__restrict__ U, int lmax, int nrhs) {
    const int m = blockIdx.x, rr = blockIdx.y;
    const long long nalm = (long long)(lmax + 1) * (lmax + 1);
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    const int nl = lmax - m + 1;
    const int rc = rr / 8, r = rr % 8;
    const long long ob = cos_base(m, lmax);
    float *Ub = U + ((long long)rc * tri + tri_off_m(m, lmax)) * 16 + 2 * r;
    for (int i = threadIdx.x; i < 2 * nl; i += blockDim.x) {
        const int dlm = i >> 1, cs = i & 1;
        double v = 0.0;
        if (rr < nrhs && !(m == 0 && cs == 1)) {
            v = x[(long long)rr * nalm + ob + (cs ? nl : 0) + dlm];
            if (dl) v *= dl[m + dlm];
        }
        Ub[(long long)dlm * 16 + cs] = (float)v;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
long long tlayout32_floats(int lmax, int nrhs) {
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    return (long long)((nrhs + 7) / 8) * 16 * tri;
}

int launch_pack_t32(int lmax, int nrhs, const double *x, const double *dl, float *U,
                    hipStream_t s) {
    const int nrc = (nrhs + 7) / 8;
    hipLaunchKernelGGL(k_pack_t32, dim3(lmax + 1, nrc * 8), dim3(256), 0, s, x, dl, U, lmax, nrhs);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_legendre_synth_mfma(const LegendreArgs &a, const float *U32, double2 *F) {
    const mlcr_geom *g = a.g;
    const int npb = (g->npairs + 63) / 64;
    const int nrc = (a.nrhs + 7) / 8;
    const long long total = (long long)(a.lmax + 1) * npb * nrc;
    const long long grid = ((total + 7) / 8) * 8;
    const long long fstride = (long long)g->nrings * (a.lmax + 1);
    hipLaunchKernelGGL(k_lsynth_mfma32, dim3((unsigned)grid), dim3(64), 0, a.stream, U32, a.nrhs,
                       F, fstride, a.lmax, g->ring_z.as<double>(), g->ring_s.as<double>(),
                       g->ab.as<double2>(), g->aboff.as<long long>(), g->seed.as<double>(),
                       g->nrings, g->npairs, npb, total);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int adjoint_chunks_mfma(const mlcr_geom *g, int lmax) {
    const int npb = (g->npairs + 63) / 64;
    int want = (8192 + lmax) / (lmax + 1);
    want = std::max(1, std::min(want, 8));
    return std::min(want, npb);
}

// P: double T layout with 8 RHS per chunk
int launch_legendre_adjoint_mfma(const LegendreArgs &a, const double2 *G, double *P,
                                 int *nchunks_out) {
    const mlcr_geom *g = a.g;
    const int npb = (g->npairs + 63) / 64;
    const int nchunks = adjoint_chunks_mfma(g, a.lmax);
    const int per = (npb + nchunks - 1) / nchunks;
    const int nrc = (a.nrhs + 7) / 8;
    const long long total = (long long)(a.lmax + 1) * nchunks * nrc;
    const long long grid = ((total + 7) / 8) * 8;
    const long long fstride = (long long)g->nrings * (a.lmax + 1);
    hipLaunchKernelGGL(k_ladj_mfma32, dim3((unsigned)grid), dim3(64), 0, a.stream, G, fstride,
                       a.nrhs, P, per, a.lmax, g->ring_z.as<double>(), g->ring_s.as<double>(),
                       g->ab.as<double2>(), g->aboff.as<long long>(), g->seed.as<double>(),
                       g->nrings, g->npairs, npb, nchunks, total);
    MLCR_HIP_CHECK(hipGetLastError());
    *nchunks_out = nchunks;
    return MLCR_OK;
}

}  // namespace mlcr
