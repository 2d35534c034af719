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
// chunk of RHS).  Lane j of the block owns ring pairs j, j+64, ...; the NR
// independent recurrences per lane give instruction-level parallelism.
// Orders are visited in the sequence 0, lmax, 1, lmax-1, ... so that any
// contiguous run of work items carries the same amount of work, and each
// XCD (workgroup id mod 8) receives one contiguous run, so neighbouring m
// values -- which share cache lines of the ring-major Fourier buffer --
// are resident in the same L2.
#include <algorithm>

#include "mlcr_internal.h"

namespace mlcr {

static constexpr int kScaleStep = 512;
static constexpr int kSeedMinExp = -112;

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
// shared pieces of the recurrence
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

// ---------------------------------------------------------------------------
// synthesis
// ---------------------------------------------------------------------------
template <int NR, int RC>
__global__ __launch_bounds__(64) void k_lsynth_f64(
    const double *__restrict__ u, long long nalm, int nrhs, double2 *__restrict__ F,
    long long fstride, int lmax, const double *__restrict__ rz, const double *__restrict__ rs,
    const double2 *__restrict__ ab, const long long *__restrict__ aboff,
    const double *__restrict__ seedc, const double *__restrict__ zeros, int nrings, int npairs,
    int npb, long long total) {
    int m, pb, rc;
    bool ok;
    decode_item(total, lmax, npb, m, pb, rc, ok);
    if (!ok) return;
    const int lane = threadIdx.x;
    const int nl = lmax - m + 1;
    const long long bc = cos_base(m, lmax);
    const double2 *abm = ab + aboff[m] - (m + 1);      // abm[l] = (A_lm, B_lm), l >= m+1
    const int r0 = rc * RC;

    const double *uc[RC];
    const double *us[RC];
#pragma unroll
    for (int r = 0; r < RC; r++) {
        const int rr = min(r0 + r, nrhs - 1);
        uc[r] = u + (long long)rr * nalm + bc - m;      // uc[r][l]
        us[r] = (m > 0) ? uc[r] + nl : zeros - m;       // m = 0 has no sine block
    }

    Lanes<NR> L;
    L.init(pb, lane, m, npairs, rz, rs, seedc[m]);
    double Ec[NR][RC], Es[NR][RC], Oc[NR][RC], Os[NR][RC];
#pragma unroll
    for (int j = 0; j < NR; j++)
#pragma unroll
        for (int r = 0; r < RC; r++) Ec[j][r] = Es[j][r] = Oc[j][r] = Os[j][r] = 0.0;

    auto acc = [&](int l, bool masked, double (*Ac)[RC], double (*As)[RC]) {
        double cu[RC], su[RC];
#pragma unroll
        for (int r = 0; r < RC; r++) {
            cu[r] = uc[r][l];
            su[r] = us[r][l];
        }
#pragma unroll
        for (int j = 0; j < NR; j++) {
            const double v = masked ? L.w(j) : L.l1[j];
#pragma unroll
            for (int r = 0; r < RC; r++) {
                Ac[j][r] = fma(v, cu[r], Ac[j][r]);
                As[j][r] = fma(v, su[r], As[j][r]);
            }
        }
    };

    int l = m;
    // phase A: every lane below range -- recurrence only
    while (l < lmax && __all(L.all_scaled())) {
        L.step_rescale(abm[l + 1]);
        l++;
    }
    // phase B: mixed -- masked accumulation plus rescaling
    while (l <= lmax && !__all(L.all_normal())) {
        if (((l - m) & 1) == 0) acc(l, true, Ec, Es);
        else acc(l, true, Oc, Os);
        if (l < lmax) L.step_rescale(abm[l + 1]);
        l++;
    }
    // phase C: plain recurrence and accumulation, two steps (even l-m, odd l-m) per trip
    if (l <= lmax && ((l - m) & 1)) {
        acc(l, false, Oc, Os);
        if (l < lmax) L.step(abm[l + 1]);
        l++;
    }
    if (l + 1 <= lmax) {
        double2 ca = abm[l + 1], cb = abm[min(l + 2, lmax)];
        double cu0[RC], su0[RC], cu1[RC], su1[RC];
#pragma unroll
        for (int r = 0; r < RC; r++) {
            cu0[r] = uc[r][l];
            su0[r] = us[r][l];
            cu1[r] = uc[r][l + 1];
            su1[r] = us[r][l + 1];
        }
        for (; l + 1 <= lmax; l += 2) {
            // prefetch the next pair
            const int ln = min(l + 2, lmax);
            const double2 na = abm[min(l + 3, lmax)], nb = abm[min(l + 4, lmax)];
            double ncu0[RC], nsu0[RC], ncu1[RC], nsu1[RC];
#pragma unroll
            for (int r = 0; r < RC; r++) {
                ncu0[r] = uc[r][ln];
                nsu0[r] = us[r][ln];
                ncu1[r] = uc[r][min(ln + 1, lmax)];
                nsu1[r] = us[r][min(ln + 1, lmax)];
            }
#pragma unroll
            for (int j = 0; j < NR; j++)
#pragma unroll
                for (int r = 0; r < RC; r++) {
                    Ec[j][r] = fma(L.l1[j], cu0[r], Ec[j][r]);
                    Es[j][r] = fma(L.l1[j], su0[r], Es[j][r]);
                }
            L.step(ca);
#pragma unroll
            for (int j = 0; j < NR; j++)
#pragma unroll
                for (int r = 0; r < RC; r++) {
                    Oc[j][r] = fma(L.l1[j], cu1[r], Oc[j][r]);
                    Os[j][r] = fma(L.l1[j], su1[r], Os[j][r]);
                }
            L.step(cb);     // harmless past lmax: the value is never used
            ca = na;
            cb = nb;
#pragma unroll
            for (int r = 0; r < RC; r++) {
                cu0[r] = ncu0[r];
                su0[r] = nsu0[r];
                cu1[r] = ncu1[r];
                su1[r] = nsu1[r];
            }
        }
    }
    if (l == lmax) acc(l, false, Ec, Es);

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
// pairs (g = G_N + G_S for even l-m, G_N - G_S for odd), and stores it in a
// wave-private LDS tile of LB consecutive l.  When the tile is full it is
// reduced across the 64 lanes (each output by 64/NOUT lanes plus a shuffle)
// and stored to (first block of the chunk) or added to the partial result
// of this chunk of ring pairs.  Every output address is owned by one lane,
// so the chunk's partial sums are formed in a fixed order.
template <int NR, int RC, int LB, bool SQ>
__global__ __launch_bounds__(64) void k_ladj_f64(
    const double2 *__restrict__ G, long long fstride, int nrhs, double *__restrict__ P,
    long long nalm, int pb_per_chunk, int lmax, const double *__restrict__ rz,
    const double *__restrict__ rs, const double2 *__restrict__ ab,
    const long long *__restrict__ aboff, const double *__restrict__ seedc, int nrings, int npairs,
    int npb, int nchunks, long long total) {
    constexpr int NC = 2 * RC;          // components per l: (cos, sin) x RHS
    constexpr int NOUT = LB * NC;
    static_assert(NOUT <= 64 && (64 % NOUT) == 0, "tile must map onto the wave");
    static_assert(LB % 2 == 0, "tile length must be even");
    constexpr int LPO = 64 / NOUT;      // lanes per output
    constexpr int SEG = 64 / LPO;       // lane values summed by one lane
    __shared__ double red[LB * NC][65];

    int m, chunk, rc;
    bool ok;
    decode_item(total, lmax, nchunks, m, chunk, rc, ok);
    if (!ok) return;
    const int lane = threadIdx.x;
    const int nl = lmax - m + 1;
    const long long bc = cos_base(m, lmax);
    const double2 *abm = ab + aboff[m] - (m + 1);
    const int r0 = rc * RC;
    const int ld = lmax + 1;

    // output owned by this lane in a flush
    const int o = lane / LPO, part = lane % LPO;
    const int o_slot = o / NC, o_comp = o % NC;
    const int o_r = o_comp >> 1, o_cs = o_comp & 1;
    const bool o_write = (part == 0) && (r0 + o_r < nrhs) && !(m == 0 && o_cs == 1);
    double *Pout = P + ((long long)chunk * nrhs + (r0 + o_r)) * nalm + bc + (o_cs ? nl : 0) - m;

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
                goc[j][r] = gn.x - gs.x;
                gos[j][r] = gn.y - gs.y;
            }
        }

        int l = m;
        while (l < lmax && __all(L.all_scaled())) {
            L.step_rescale(abm[l + 1]);
            l++;
        }
        const bool nothing = __all(L.all_scaled());     // still below range at l = lmax
        const int nblk = (nl + LB - 1) / LB;
        const int blk0 = nothing ? nblk : (l - m) / LB;   // first tile this block touches

        // tiles before blk0 receive nothing from this block of ring pairs
        if (first && o_write) {
            for (int b = 0; b < blk0; b++) {
                const int ll = m + b * LB + o_slot;
                if (ll <= lmax) Pout[ll] = 0.0;
            }
        }
        if (nothing) continue;

        for (int t = lane; t < LB * NC * 65; t += 64) (&red[0][0])[t] = 0.0;
        __syncthreads();

        auto flush = [&](int lb0) {
            __syncthreads();
            double a = 0.0;
            const int i0 = part * SEG;
#pragma unroll 8
            for (int i = 0; i < SEG; i++) a += red[o][i0 + ((i + lane) % SEG)];
#pragma unroll
            for (int off = 1; off < LPO; off <<= 1) a += __shfl_xor(a, off, 64);
            const int ll = lb0 + o_slot;
            if (o_write && ll <= lmax) {
                if (first) Pout[ll] = a;
                else Pout[ll] += a;
            }
            __syncthreads();
            for (int tt = lane; tt < LB * NC * 65; tt += 64) (&red[0][0])[tt] = 0.0;
            __syncthreads();
        };
        auto put = [&](int l_, bool masked, double (*gc)[RC], double (*gs)[RC]) {
            double tc[RC], ts[RC];
#pragma unroll
            for (int r = 0; r < RC; r++) tc[r] = ts[r] = 0.0;
#pragma unroll
            for (int j = 0; j < NR; j++) {
                double v = masked ? L.w(j) : L.l1[j];
                if (SQ) v = v * v;
#pragma unroll
                for (int r = 0; r < RC; r++) {
                    tc[r] = fma(v, gc[j][r], tc[r]);
                    ts[r] = fma(v, gs[j][r], ts[r]);
                }
            }
            const int slot = (l_ - m) % LB;
#pragma unroll
            for (int r = 0; r < RC; r++) {
                red[slot * NC + 2 * r][lane] = tc[r];
                red[slot * NC + 2 * r + 1][lane] = ts[r];
            }
            if (slot == LB - 1 || l_ == lmax) flush(l_ - slot);
        };

        // phase B: mixed
        while (l <= lmax && !__all(L.all_normal())) {
            if (((l - m) & 1) == 0) put(l, true, gec, ges);
            else put(l, true, SQ ? gec : goc, SQ ? ges : gos);
            if (l < lmax) L.step_rescale(abm[l + 1]);
            l++;
        }
        // phase C: align to even l-m, then two steps per trip
        if (l <= lmax && ((l - m) & 1)) {
            put(l, false, SQ ? gec : goc, SQ ? ges : gos);
            if (l < lmax) L.step(abm[l + 1]);
            l++;
        }
        if (l + 1 <= lmax) {
            double2 ca = abm[l + 1], cb = abm[min(l + 2, lmax)];
            for (; l + 1 <= lmax; l += 2) {
                const double2 na = abm[min(l + 3, lmax)], nb = abm[min(l + 4, lmax)];
                put(l, false, gec, ges);
                L.step(ca);
                put(l + 1, false, SQ ? gec : goc, SQ ? ges : gos);
                L.step(cb);
                ca = na;
                cb = nb;
            }
        }
        if (l == lmax) put(l, false, gec, ges);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static constexpr int kSynthNR = 4, kSynthRC = 1;
static constexpr int kAdjNR = 4, kAdjRC = 1, kAdjLB = 8;

int adjoint_chunks(const mlcr_geom *g, int lmax) {
    const int npb = (g->npairs + 64 * kAdjNR - 1) / (64 * kAdjNR);
    // enough waves to fill 256 CUs several times over, but few partial buffers
    int want = (8192 + lmax) / (lmax + 1);
    want = std::max(1, std::min(want, 8));
    return std::min(want, npb);
}

int launch_legendre_synth(const LegendreArgs &a, const double *u, double2 *F) {
    const mlcr_geom *g = a.g;
    const int npb = (g->npairs + 64 * kSynthNR - 1) / (64 * kSynthNR);
    const int nrc = (a.nrhs + kSynthRC - 1) / kSynthRC;
    const long long total = (long long)(a.lmax + 1) * npb * nrc;
    const long long grid = ((total + 7) / 8) * 8;
    const long long nalm = (long long)(a.lmax + 1) * (a.lmax + 1);
    const long long fstride = (long long)g->nrings * (a.lmax + 1);
    hipLaunchKernelGGL((k_lsynth_f64<kSynthNR, kSynthRC>), dim3((unsigned)grid), dim3(64), 0,
                       a.stream, u, nalm, a.nrhs, F, fstride, a.lmax, g->ring_z.as<double>(),
                       g->ring_s.as<double>(), g->ab.as<double2>(), g->aboff.as<long long>(),
                       g->seed.as<double>(), g->zeros.as<double>(), g->nrings, g->npairs, npb,
                       total);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

template <bool SQ>
static int launch_ladj(const LegendreArgs &a, const double2 *G, double *P, int *nchunks_out) {
    const mlcr_geom *g = a.g;
    const int npb = (g->npairs + 64 * kAdjNR - 1) / (64 * kAdjNR);
    const int nchunks = adjoint_chunks(g, a.lmax);
    const int per = (npb + nchunks - 1) / nchunks;
    const int nrc = (a.nrhs + kAdjRC - 1) / kAdjRC;
    const long long total = (long long)(a.lmax + 1) * nchunks * nrc;
    const long long grid = ((total + 7) / 8) * 8;
    const long long nalm = (long long)(a.lmax + 1) * (a.lmax + 1);
    const long long fstride = (long long)g->nrings * (a.lmax + 1);
    hipLaunchKernelGGL((k_ladj_f64<kAdjNR, kAdjRC, kAdjLB, SQ>), dim3((unsigned)grid), dim3(64), 0,
                       a.stream, G, fstride, a.nrhs, P, nalm, per, a.lmax,
                       g->ring_z.as<double>(), g->ring_s.as<double>(), g->ab.as<double2>(),
                       g->aboff.as<long long>(), g->seed.as<double>(), g->nrings, g->npairs, npb,
                       nchunks, total);
    MLCR_HIP_CHECK(hipGetLastError());
    *nchunks_out = nchunks;
    return MLCR_OK;
}

int launch_legendre_adjoint(const LegendreArgs &a, const double2 *G, double *P, int *nchunks_out) {
    return launch_ladj<false>(a, G, P, nchunks_out);
}

// Same reduction with lambda^2 in place of lambda and the even ring sums for
// every l (the parity sign squares away): sum_k lambda_lm(theta_k)^2 G_m(theta_k).
int launch_legendre_adjoint_sq(const LegendreArgs &a, const double2 *G, double *P,
                               int *nchunks_out) {
    return launch_ladj<true>(a, G, P, nchunks_out);
}

}  // namespace mlcr
