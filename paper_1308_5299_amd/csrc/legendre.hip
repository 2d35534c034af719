// Legendre step of the spherical harmonic transforms (float64 path).
//
// Synthesis, per order m and ring pair (theta, pi - theta):
//     F_m(theta) = sum_{l >= m} lambda_lm(theta) u_lm          (cos and sin parts)
// Adjoint, per m:
//     v_lm = sum_rings lambda_lm(theta_k) G_m(theta_k)
// with lambda_lm the normalized associated Legendre function (Sec. 3.2,
// beside eq. Ni-dense) generated on the fly by the three-term recurrence in l.
// The mirror ring uses lambda_lm(-z) = (-1)^{l+m} lambda_lm(z), so each lane
// keeps even and odd partial sums and serves both rings of a pair.
//
// Range: sin^m(theta) underflows float64 near the poles for large m, so
// each lane carries its value as v * 2^{-512 k}.  While k > 0 the true value
// is below 2^-112 and is not accumulated (its contribution is far below
// float64 resolution); it is rescaled by 2^-512 whenever |v| reaches 2^400.
// A wave first runs the recurrence alone while all its lanes are scaled
// (the "l_start" skip), then mixes, then runs the plain loop.
//
// Mapping: one wave (one workgroup) per (m, block of 64*NR ring pairs,
// chunk of RC right-hand sides); lane j owns pairs j, j+64, ...  The per-l
// inputs shared by the wave -- recurrence coefficients and the RC x (cos,
// sin) harmonic coefficients -- stream through LDS in chunks of 32 l, loaded
// one chunk ahead with coalesced vector loads and read back as broadcasts,
// so the loop never waits on a scalar-cache round trip.  Harmonic inputs
// and adjoint partial sums use an l-major, RHS-interleaved layout
// ("T layout": [RHS chunk][m][l - m][RC][cos, sin]) written and read by the
// prologue/epilogue kernels.
//
// Orders are visited in the sequence 0, lmax, 1, lmax-1, ... so that any
// contiguous run of work items carries the same amount of work, and each
// XCD (workgroup id mod 8) receives one contiguous run.
#include <algorithm>

#include "mlcr_internal.h"

namespace mlcr {

static constexpr int kScaleStep = 512;
static constexpr int kSeedMinExp = -112;
static constexpr int kChunk = 32;           // l values per LDS chunk (even)

__device__ __forceinline__ void seed_lambda(double s, int m, double c, double &lam, int &k) {
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
    if (ex >= kSeedMinExp) {
        lam = ldexp(v, ex);
        k = 0;
    } else {
        k = (kSeedMinExp - ex + kScaleStep - 1) / kScaleStep;
        lam = ldexp(v, ex + kScaleStep * k);
    }
}

__device__ __forceinline__ void decode_item(long long total, int lmax, int npb, int &m, int &pb,
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

// ---------------------------------------------------------------------------
// per-lane recurrence state
// ---------------------------------------------------------------------------
template <int NR>
struct Lanes {
    int kp[NR], sc[NR];
    double z[NR], l1[NR], l2[NR];

    __device__ __forceinline__ void init(int pb, int lane, int m, int npairs,
                                         const double *__restrict__ rz,
                                         const double *__restrict__ rs, double seedc) {
#pragma unroll
        for (int j = 0; j < NR; j++) {
            kp[j] = pb * 64 * NR + j * 64 + lane;
            const bool valid = kp[j] < npairs;
            z[j] = valid ? rz[kp[j]] : 0.0;
            const double s = valid ? rs[kp[j]] : 1.0;
            seed_lambda(s, m, seedc, l1[j], sc[j]);
            l2[j] = 0.0;
        }
    }
    __device__ __forceinline__ bool all_scaled() const {
        bool a = true;
#pragma unroll
        for (int j = 0; j < NR; j++) a = a && (sc[j] > 0);
        return a;
    }
    __device__ __forceinline__ bool all_normal() const {
        bool a = true;
#pragma unroll
        for (int j = 0; j < NR; j++) a = a && (sc[j] == 0);
        return a;
    }
    // lambda_{l+1} from lambda_l, lambda_{l-1}; c = (A_{l+1}, B_{l+1})
    __device__ __forceinline__ void step(double2 c) {
#pragma unroll
        for (int j = 0; j < NR; j++) {
            const double nv = fma(c.x, z[j] * l1[j], -c.y * l2[j]);
            l2[j] = l1[j];
            l1[j] = nv;
        }
    }
    __device__ __forceinline__ void step_rescale(double2 c) {
#pragma unroll
        for (int j = 0; j < NR; j++) {
            const double nv = fma(c.x, z[j] * l1[j], -c.y * l2[j]);
            l2[j] = l1[j];
            l1[j] = nv;
            if (sc[j] > 0 && fabs(nv) >= 0x1p400) {
                l1[j] *= 0x1p-512;
                l2[j] *= 0x1p-512;
                sc[j]--;
            }
        }
    }
    // value to accumulate: lambda where in range, 0 where still scaled
    __device__ __forceinline__ double w(int j) const { return sc[j] == 0 ? l1[j] : 0.0; }
};

// wave mode: 0 every lane below range, 1 mixed, 2 every lane in range
template <int NR>
__device__ __forceinline__ int wave_mode(const Lanes<NR> &L) {
    if (__all(L.all_normal())) return 2;
    if (__all(L.all_scaled())) return 0;
    return 1;
}

// offset of order m's block in a T-layout triangle: sum_{m' < m} (lmax - m' + 1)
__device__ __forceinline__ long long tri_off(int m, int lmax) {
    return (long long)m * (lmax + 1) - (long long)m * (m - 1) / 2;
}

// ---------------------------------------------------------------------------
// per-l coefficients streamed through LDS
// ---------------------------------------------------------------------------
// Chunk k holds, for l = m + k*C + j (j < C): ab = (A, B) of the step
// l -> l+1 (zero past lmax) and NU values of the T-layout harmonic input at
// l (zero past lmax).  Lanes 0..C-1 load one entry each.
template <int NU>
struct Stream {
    double2 ab;
    double u[NU > 0 ? NU : 1];
    __device__ __forceinline__ void load(int k, int m, int lmax, const double2 *__restrict__ abm,
                                         const double *__restrict__ U) {
        const int j = threadIdx.x;
        const int l = m + k * kChunk + j;
        if (j < kChunk) {
            ab = (l + 1 <= lmax) ? abm[l + 1] : make_double2(0.0, 0.0);
            if constexpr (NU > 0) {
                const double2 *src = reinterpret_cast<const double2 *>(U + (long long)(l - m) * NU);
#pragma unroll
                for (int i = 0; i < NU / 2; i++) {
                    const double2 v = (l <= lmax) ? src[i] : make_double2(0.0, 0.0);
                    u[2 * i] = v.x;
                    u[2 * i + 1] = v.y;
                }
            }
        }
    }
    __device__ __forceinline__ void store(double2 *sab, double *su) const {
        const int j = threadIdx.x;
        if (j < kChunk) {
            sab[j] = ab;
            if constexpr (NU > 0) {
                double2 *dst = reinterpret_cast<double2 *>(su + j * NU);
#pragma unroll
                for (int i = 0; i < NU / 2; i++) dst[i] = make_double2(u[2 * i], u[2 * i + 1]);
            }
        }
    }
};

// ---------------------------------------------------------------------------
// synthesis
// ---------------------------------------------------------------------------
template <int NR, int RC>
__global__ __launch_bounds__(64) void k_lsynth_f64(
    const double *__restrict__ U, int nrhs, double2 *__restrict__ F, long long fstride, int lmax,
    const double *__restrict__ rz, const double *__restrict__ rs, const double2 *__restrict__ ab,
    const long long *__restrict__ aboff, const double *__restrict__ seedc, int nrings, int npairs,
    int npb, long long total) {
    constexpr int NU = 2 * RC;
    __shared__ double2 sab[2][kChunk];
    __shared__ double su[2][kChunk * NU];
    int m, pb, rc;
    bool ok;
    decode_item(total, lmax, npb, m, pb, rc, ok);
    if (!ok) return;
    const int lane = threadIdx.x;
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    const double *Um = U + ((long long)rc * tri + tri_off(m, lmax)) * NU;
    const double2 *abm = ab + aboff[m] - (m + 1);     // abm[l], l >= m+1
    const int r0 = rc * RC;

    Lanes<NR> L;
    L.init(pb, lane, m, npairs, rz, rs, seedc[m]);
    double Ec[NR][RC], Es[NR][RC], Oc[NR][RC], Os[NR][RC];
#pragma unroll
    for (int j = 0; j < NR; j++)
#pragma unroll
        for (int r = 0; r < RC; r++) Ec[j][r] = Es[j][r] = Oc[j][r] = Os[j][r] = 0.0;

    const int nl = lmax - m + 1;
    const int nchunks = (nl + kChunk - 1) / kChunk;
    Stream<NU> st;
    st.load(0, m, lmax, abm, Um);
    st.store(sab[0], su[0]);
    if (nchunks > 1) st.load(1, m, lmax, abm, Um);
    __syncthreads();
    int mode = wave_mode(L);

    for (int k = 0; k < nchunks; k++) {
        const int bi = k & 1;
        const int jend = min(kChunk, nl - k * kChunk);     // entries with l <= lmax
#pragma unroll 1
        for (int j = 0; j < jend; j += 2) {
            // pair (l, l+1) with l - m even; past lmax the streamed values are 0
            const double2 c0 = sab[bi][j], c1 = sab[bi][j + 1];
            if (mode == 0) {
                L.step_rescale(c0);
                L.step_rescale(c1);
                mode = wave_mode(L);
                continue;
            }
            const double *u0 = &su[bi][j * NU];
            const double *u1 = &su[bi][(j + 1) * NU];
            if (mode == 2) {
#pragma unroll
                for (int jj = 0; jj < NR; jj++)
#pragma unroll
                    for (int r = 0; r < RC; r++) {
                        Ec[jj][r] = fma(L.l1[jj], u0[2 * r], Ec[jj][r]);
                        Es[jj][r] = fma(L.l1[jj], u0[2 * r + 1], Es[jj][r]);
                    }
                L.step(c0);
#pragma unroll
                for (int jj = 0; jj < NR; jj++)
#pragma unroll
                    for (int r = 0; r < RC; r++) {
                        Oc[jj][r] = fma(L.l1[jj], u1[2 * r], Oc[jj][r]);
                        Os[jj][r] = fma(L.l1[jj], u1[2 * r + 1], Os[jj][r]);
                    }
                L.step(c1);
            } else {
#pragma unroll
                for (int jj = 0; jj < NR; jj++) {
                    const double v = L.w(jj);
#pragma unroll
                    for (int r = 0; r < RC; r++) {
                        Ec[jj][r] = fma(v, u0[2 * r], Ec[jj][r]);
                        Es[jj][r] = fma(v, u0[2 * r + 1], Es[jj][r]);
                    }
                }
                L.step_rescale(c0);
#pragma unroll
                for (int jj = 0; jj < NR; jj++) {
                    const double v = L.w(jj);
#pragma unroll
                    for (int r = 0; r < RC; r++) {
                        Oc[jj][r] = fma(v, u1[2 * r], Oc[jj][r]);
                        Os[jj][r] = fma(v, u1[2 * r + 1], Os[jj][r]);
                    }
                }
                L.step_rescale(c1);
                mode = wave_mode(L);
            }
        }
        if (k + 1 < nchunks) {
            st.store(sab[bi ^ 1], su[bi ^ 1]);
            if (k + 2 < nchunks) st.load(k + 2, m, lmax, abm, Um);
            __syncthreads();
        }
    }

    const int ld = lmax + 1;
#pragma unroll
    for (int j = 0; j < NR; j++) {
        if (L.kp[j] >= npairs) continue;
        const int north = L.kp[j], south = nrings - 1 - L.kp[j];
#pragma unroll
        for (int r = 0; r < RC; r++) {
            const int rr = r0 + r;
            if (rr >= nrhs) continue;
            double2 *Fr = F + (long long)rr * fstride;
            Fr[(long long)north * ld + m] = make_double2(Ec[j][r] + Oc[j][r], Es[j][r] + Os[j][r]);
            if (south != north)
                Fr[(long long)south * ld + m] =
                    make_double2(Ec[j][r] - Oc[j][r], Es[j][r] - Os[j][r]);
        }
    }
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
// Each lane forms, per l, t = sum_j lambda_l(theta_j) g_j over its NR ring
// pairs (g = G_N + G_S for even l-m, G_N - G_S for odd) and stores it in a
// wave-private LDS tile of LB consecutive l.  At the end of each tile the
// tile is reduced across the 64 lanes (each output by 64/NOUT lanes plus a
// shuffle) and stored (first block of the chunk) or added to the partial
// result of this chunk of ring pairs, in T layout (coalesced).  Every output
// address is owned by one lane, so partial sums form in a fixed order.
// With SQ, lambda^2 replaces lambda and the even ring sums serve every l.
template <int NR, int RC, int LB, bool SQ>
__global__ __launch_bounds__(64) void k_ladj_f64(
    const double2 *__restrict__ G, long long fstride, int nrhs, double *__restrict__ P,
    int pb_per_chunk, int lmax, const double *__restrict__ rz, const double *__restrict__ rs,
    const double2 *__restrict__ ab, const long long *__restrict__ aboff,
    const double *__restrict__ seedc, int nrings, int npairs, int npb, int nchunks,
    long long total) {
    constexpr int NC = 2 * RC;          // components per l: RHS x (cos, sin)
    constexpr int NOUT = LB * NC;
    static_assert(NOUT <= 64 && (64 % NOUT) == 0, "tile must map onto the wave");
    static_assert(LB % 2 == 0 && kChunk % LB == 0, "tile length must divide the chunk");
    constexpr int LPO = 64 / NOUT;      // lanes per output
    constexpr int SEG = 64 / LPO;       // lane values summed by one lane
    __shared__ double red[NOUT][65];
    __shared__ double2 sab[2][kChunk];

    int m, chunk, rc;
    bool ok;
    decode_item(total, lmax, nchunks, m, chunk, rc, ok);
    if (!ok) return;
    const int lane = threadIdx.x;
    const int nl = lmax - m + 1;
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    const int nrc = (nrhs + RC - 1) / RC;
    const double2 *abm = ab + aboff[m] - (m + 1);
    const int r0 = rc * RC;
    const int ld = lmax + 1;

    // output owned by this lane in a flush: o = slot * NC + comp (contiguous in T layout)
    const int o = lane / LPO, part = lane % LPO;
    const int o_slot = o / NC;
    double *Pm = P + (((long long)chunk * nrc + rc) * tri + tri_off(m, lmax)) * NC;
    const bool o_write = (part == 0);

    for (int pbi = 0; pbi < pb_per_chunk; pbi++) {
        const int pb = chunk * pb_per_chunk + pbi;
        if (pb >= npb) break;
        const bool first = (pbi == 0);

        Lanes<NR> L;
        L.init(pb, lane, m, npairs, rz, rs, seedc[m]);
        double gec[NR][RC], ges[NR][RC], goc[NR][RC], gos[NR][RC];
#pragma unroll
        for (int j = 0; j < NR; j++) {
            const bool valid = L.kp[j] < npairs;
            const int north = valid ? L.kp[j] : 0;
            const int south = nrings - 1 - north;
#pragma unroll
            for (int r = 0; r < RC; r++) {
                const int rr = min(r0 + r, nrhs - 1);
                const double2 *Gr = G + (long long)rr * fstride;
                double2 gn = valid ? Gr[(long long)north * ld + m] : make_double2(0.0, 0.0);
                double2 gs = (valid && south != north) ? Gr[(long long)south * ld + m]
                                                        : make_double2(0.0, 0.0);
                gec[j][r] = gn.x + gs.x;
                ges[j][r] = gn.y + gs.y;
                goc[j][r] = SQ ? gec[j][r] : gn.x - gs.x;
                gos[j][r] = SQ ? ges[j][r] : gn.y - gs.y;
            }
        }
        for (int t = lane; t < NOUT * 65; t += 64) (&red[0][0])[t] = 0.0;

        const int nchk = (nl + kChunk - 1) / kChunk;
        Stream<0> st;
        st.load(0, m, lmax, abm, nullptr);
        st.store(sab[0], nullptr);
        if (nchk > 1) st.load(1, m, lmax, abm, nullptr);
        __syncthreads();
        int mode = wave_mode(L);

        // end of a tile starting at lb0: reduce and store/add, or store zeros
        auto flush = [&](int lb0, bool have) {
            double a = 0.0;
            if (have) {
                __syncthreads();
                const int i0 = part * SEG;
#pragma unroll 8
                for (int i = 0; i < SEG; i++) a += red[o][i0 + ((i + lane) % SEG)];
#pragma unroll
                for (int off = 1; off < LPO; off <<= 1) a += __shfl_xor(a, off, 64);
            }
            if (o_write && lb0 + o_slot <= lmax && (have || first)) {
                double *p = Pm + (long long)(lb0 - m) * NC + o;
                if (first) *p = a;
                else *p += a;
            }
            if (have) {
                __syncthreads();
                for (int tt = lane; tt < NOUT * 65; tt += 64) (&red[0][0])[tt] = 0.0;
                __syncthreads();
            }
        };
        auto put = [&](int j, bool masked, double (*gc)[RC], double (*gs)[RC]) {
            double tc[RC], ts[RC];
#pragma unroll
            for (int r = 0; r < RC; r++) tc[r] = ts[r] = 0.0;
#pragma unroll
            for (int jj = 0; jj < NR; jj++) {
                double v = masked ? L.w(jj) : L.l1[jj];
                if (SQ) v = v * v;
#pragma unroll
                for (int r = 0; r < RC; r++) {
                    tc[r] = fma(v, gc[jj][r], tc[r]);
                    ts[r] = fma(v, gs[jj][r], ts[r]);
                }
            }
            const int slot = j % LB;
#pragma unroll
            for (int r = 0; r < RC; r++) {
                red[slot * NC + 2 * r][lane] = tc[r];
                red[slot * NC + 2 * r + 1][lane] = ts[r];
            }
        };

        bool tile_has = false;
        for (int k = 0; k < nchk; k++) {
            const int bi = k & 1;
            const int jend = min(kChunk, nl - k * kChunk);
#pragma unroll 1
            for (int j = 0; j < jend; j += 2) {
                const int l = m + k * kChunk + j;
                const double2 c0 = sab[bi][j], c1 = sab[bi][j + 1];
                if (mode == 0) {
                    L.step_rescale(c0);
                    L.step_rescale(c1);
                    mode = wave_mode(L);
                } else if (mode == 2) {
                    put(j, false, gec, ges);
                    L.step(c0);
                    put(j + 1, false, goc, gos);
                    L.step(c1);
                    tile_has = true;
                } else {
                    put(j, true, gec, ges);
                    L.step_rescale(c0);
                    put(j + 1, true, goc, gos);
                    L.step_rescale(c1);
                    mode = wave_mode(L);
                    tile_has = true;
                }
                if (((l + 2 - m) % LB) == 0 || l + 2 > lmax) {
                    flush(m + ((l - m) / LB) * LB, tile_has);
                    tile_has = false;
                }
            }
            if (k + 1 < nchk) {
                st.store(sab[bi ^ 1], nullptr);
                if (k + 2 < nchk) st.load(k + 2, m, lmax, abm, nullptr);
                __syncthreads();
            }
        }
    }
}

// ---------------------------------------------------------------------------
// T-layout packing (beam prologue) and unpacking (prior/beam epilogue)
// ---------------------------------------------------------------------------
// U[rc][tri_off(m) + l - m][r][cs] = dl[l] x[rc*RC + r][packed(l, m, cs)]  (0 for padded RHS)
__global__ __launch_bounds__(256) void k_pack_t(const double *__restrict__ x,
                                                const double *__restrict__ dl,
                                                double *__restrict__ U, int lmax, int nrhs,
                                                int RC) {
    const int m = blockIdx.x, rr = blockIdx.y;        // rr over nrc * RC padded RHS
    const long long nalm = (long long)(lmax + 1) * (lmax + 1);
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    const int nl = lmax - m + 1;
    const int rc = rr / RC, r = rr % RC;
    const long long ob = cos_base(m, lmax);
    double *Ub = U + ((long long)rc * tri + tri_off(m, lmax)) * 2 * RC + 2 * r;
    for (int i = threadIdx.x; i < 2 * nl; i += blockDim.x) {
        const int dlm = i >> 1, cs = i & 1;
        const int l = m + dlm;
        double v = 0.0;
        if (rr < nrhs && !(m == 0 && cs == 1)) {
            v = x[(long long)rr * nalm + ob + (cs ? nl : 0) + dlm];
            if (dl) v *= dl[l];
        }
        Ub[(long long)dlm * 2 * RC + cs] = v;
    }
}

// y[r][packed] = d[l] x + bh[l] cf_lm sum_c P[c][rc][tri_off(m) + l - m][r][cs]
// (d, x may be null; bh, cf null mean 1; cf_lm = cf[tri_off(m, glmax) + l - m],
// the scale of the matrix-core kernels' recurrence).  One workgroup per (m, RHS chunk):
// tiles of 64 l are read row by row (the T layout is contiguous in
// (l, r, cs)), summed over the chunks, transposed in LDS and written out
// along l, so both sides stream.
template <typename PT>
__global__ __launch_bounds__(256) void k_unpack_t(const PT *__restrict__ P, int nchunks,
                                                  int nrhs, int RC, const double *__restrict__ cf,
                                                  int glmax, const double *__restrict__ x,
                                                  const double *__restrict__ d,
                                                  const double *__restrict__ bh,
                                                  double *__restrict__ y, int lmax) {
    constexpr int TL = 64;
    __shared__ double tile[TL * 17];
    const int m = blockIdx.x, rc = blockIdx.y;
    const long long nalm = (long long)(lmax + 1) * (lmax + 1);
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    const int nrc = (nrhs + RC - 1) / RC;
    const int nl = lmax - m + 1;
    const int NC = 2 * RC;
    const long long ob = cos_base(m, lmax);
    const long long cstride = (long long)nrc * tri * NC;
    const PT *Pb = P + ((long long)rc * tri + tri_off(m, lmax)) * NC;
    for (int base = 0; base < nl; base += TL) {
        const int nt = min(TL, nl - base);
        for (int e = threadIdx.x; e < nt * NC; e += blockDim.x) {
            const int j = e / NC, comp = e % NC;
            const PT *src = Pb + (long long)base * NC + e;
            // chunks added in order; loads issued 4 at a time
            double acc = 0.0;
            int c = 0;
            for (; c + 4 <= nchunks; c += 4) {
                const PT v0 = src[c * cstride], v1 = src[(c + 1) * cstride];
                const PT v2 = src[(c + 2) * cstride], v3 = src[(c + 3) * cstride];
                acc += (double)v0;
                acc += (double)v1;
                acc += (double)v2;
                acc += (double)v3;
            }
            for (; c < nchunks; c++) acc += (double)src[c * cstride];
            tile[j * 17 + comp] = acc;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nt * NC; e += blockDim.x) {
            const int comp = e / nt, j = e % nt;
            const int r = rc * RC + comp / 2, cs = comp & 1;
            if (r >= nrhs || (m == 0 && cs == 1)) continue;
            const int l = m + base + j;
            double v = tile[j * 17 + comp];
            if (cf) v *= cf[tri_off(m, glmax) + l - m];
            if (bh) v *= bh[l];
            const long long idx = (long long)r * nalm + ob + (long long)cs * nl + base + j;
            if (d) v = fma(d[l], x[idx], v);
            y[idx] = v;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int synth_rc(int nrhs) { return nrhs >= 5 ? 8 : (nrhs >= 2 ? 4 : 1); }
int adj_rc(int nrhs) { return nrhs >= 2 ? 4 : 1; }
static constexpr int kAdjNR = 2;

// Split-K over ring-pair blocks: `per` consecutive blocks per chunk, and as
// many chunks as that takes, so that every chunk holds at least one block
// (each chunk's partial sums are stored by its first block; an empty chunk
// would leave its slice of P unwritten for the unpack step to add).
static int adjoint_per(const mlcr_geom *g, int lmax) {
    const int npb = (g->npairs + 64 * kAdjNR - 1) / (64 * kAdjNR);
    int want = (8192 + lmax) / (lmax + 1);
    want = std::max(1, std::min(std::min(want, 8), npb));
    return (npb + want - 1) / want;
}

int adjoint_chunks(const mlcr_geom *g, int lmax) {
    const int npb = (g->npairs + 64 * kAdjNR - 1) / (64 * kAdjNR);
    const int per = adjoint_per(g, lmax);
    return (npb + per - 1) / per;
}

long long tlayout_doubles(int lmax, int nrhs, int rc) {
    const long long tri = (long long)(lmax + 1) * (lmax + 2) / 2;
    return (long long)((nrhs + rc - 1) / rc) * rc * 2 * tri;
}

int launch_pack_t(int lmax, int nrhs, int RC, const double *x, const double *dl, double *U,
                  hipStream_t s) {
    const int nrc = (nrhs + RC - 1) / RC;
    hipLaunchKernelGGL(k_pack_t, dim3(lmax + 1, nrc * RC), dim3(256), 0, s, x, dl, U, lmax, nrhs,
                       RC);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_unpack_t(int lmax, int nrhs, int RC, int nchunks, const void *P, bool pf32,
                    const double *cf, int glmax, const double *x, const double *d,
                    const double *bh, double *y, hipStream_t s) {
    if (RC > 8) return fail(MLCR_EINVAL, "unpack supports at most 8 RHS per chunk");
    const int nrc = (nrhs + RC - 1) / RC;
    if (pf32)
        hipLaunchKernelGGL(k_unpack_t<float>, dim3(lmax + 1, nrc), dim3(256), 0, s,
                           (const float *)P, nchunks, nrhs, RC, cf, glmax, x, d, bh, y, lmax);
    else
        hipLaunchKernelGGL(k_unpack_t<double>, dim3(lmax + 1, nrc), dim3(256), 0, s,
                           (const double *)P, nchunks, nrhs, RC, cf, glmax, x, d, bh, y, lmax);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

template <int NR, int RC>
static int launch_synth_t(const LegendreArgs &a, const double *U, double2 *F) {
    const mlcr_geom *g = a.g;
    const int npb = (g->npairs + 64 * NR - 1) / (64 * NR);
    const int nrc = (a.nrhs + RC - 1) / RC;
    const long long total = (long long)(a.lmax + 1) * npb * nrc;
    const long long grid = ((total + 7) / 8) * 8;
    const long long fstride = (long long)g->nrings * (a.lmax + 1);
    hipLaunchKernelGGL((k_lsynth_f64<NR, RC>), dim3((unsigned)grid), dim3(64), 0, a.stream, U,
                       a.nrhs, F, fstride, a.lmax, g->ring_z.as<double>(), g->ring_s.as<double>(),
                       g->ab.as<double2>(), g->aboff.as<long long>(), g->seed.as<double>(),
                       g->nrings, g->npairs, npb, total);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

// U in T layout with synth_rc(nrhs) right-hand sides per chunk
int launch_legendre_synth(const LegendreArgs &a, const double *U, double2 *F) {
    switch (synth_rc(a.nrhs)) {
    case 8: return launch_synth_t<1, 8>(a, U, F);
    case 4: return launch_synth_t<2, 4>(a, U, F);
    default: return launch_synth_t<4, 1>(a, U, F);
    }
}

template <int RC, int LB, bool SQ>
static int launch_ladj(const LegendreArgs &a, const double2 *G, double *P, int *nchunks_out) {
    const mlcr_geom *g = a.g;
    const int npb = (g->npairs + 64 * kAdjNR - 1) / (64 * kAdjNR);
    const int nchunks = adjoint_chunks(g, a.lmax);
    const int per = adjoint_per(g, a.lmax);
    const int nrc = (a.nrhs + RC - 1) / RC;
    const long long total = (long long)(a.lmax + 1) * nchunks * nrc;
    const long long grid = ((total + 7) / 8) * 8;
    const long long fstride = (long long)g->nrings * (a.lmax + 1);
    hipLaunchKernelGGL((k_ladj_f64<kAdjNR, RC, LB, SQ>), dim3((unsigned)grid), dim3(64), 0,
                       a.stream, G, fstride, a.nrhs, P, per, a.lmax, g->ring_z.as<double>(),
                       g->ring_s.as<double>(), g->ab.as<double2>(), g->aboff.as<long long>(),
                       g->seed.as<double>(), g->nrings, g->npairs, npb, nchunks, total);
    MLCR_HIP_CHECK(hipGetLastError());
    *nchunks_out = nchunks;
    return MLCR_OK;
}

// P in T layout with adj_rc(nrhs) right-hand sides per chunk
int launch_legendre_adjoint(const LegendreArgs &a, const double2 *G, double *P, int *nchunks_out) {
    if (adj_rc(a.nrhs) == 4) return launch_ladj<4, 4, false>(a, G, P, nchunks_out);
    return launch_ladj<1, 8, false>(a, G, P, nchunks_out);
}

// Same reduction with lambda^2 in place of lambda and the even ring sums for
// every l (the parity sign squares away): sum_k lambda_lm(theta_k)^2 G_m(theta_k).
int launch_legendre_adjoint_sq(const LegendreArgs &a, const double2 *G, double *P,
                               int *nchunks_out) {
    if (adj_rc(a.nrhs) == 4) return launch_ladj<4, 4, true>(a, G, P, nchunks_out);
    return launch_ladj<1, 8, true>(a, G, P, nchunks_out);
}

}  // namespace mlcr
