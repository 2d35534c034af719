// Device helpers shared by the matrix-core Legendre kernels (float32 /
// float64 contraction and split-bfloat16 contraction): the scaled seed of
// lambda_mm, the work-item order, and the per-lane three-term recurrence
// (Sec. 3.2) with its 2^-512 range scaling.
#pragma once

#include "mlcr_internal.h"

namespace mlcr {

constexpr int kScaleStepM = 512;
constexpr int kSeedMinExpM = -112;
constexpr int kChunkM = 32;

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

// Work item w = ((rc * (lmax+1)) + mi) * npb + pb: the ring-pair blocks of one
// order are adjacent, so they run together and share that order's
// coefficients (and U rows) through L2, while their F/G accesses spread over
// all rings (all memory channels).  Each XCD (workgroup id mod 8) gets one
// contiguous run of items; orders are visited 0, lmax, 1, lmax-1, ... so
// every run holds the same mix of long and short orders.
__host__ __device__ inline long long mitems(int lmax, int npb, int nrc) {
    return (long long)(lmax + 1) * npb * nrc;
}

__device__ __forceinline__ void decode_item_m(long long total, int lmax, int npb, int &m, int &pb,
                                              int &rc, bool &ok) {
    const long long b = blockIdx.x;
    const long long per = (total + 7) / 8;
    const long long w = (b & 7) * per + (b >> 3);
    ok = w < total;
    if (!ok) return;
    const int nm = lmax + 1;
    pb = (int)(w % npb);
    const long long rest = w / npb;
    const int mi = (int)(rest % nm);
    rc = (int)(rest / nm);
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
    __device__ __forceinline__ double w() const { return sc == 0 ? l1 : 0.0; }
    __device__ __forceinline__ void step(double2 c) {
        const double nv = fma(c.x, z * l1, -c.y * l2);
        l2 = l1;
        l1 = nv;
    }
    // Range check after a run of 4 plain steps taken while every lane of the
    // wave is still scaled (contributing nothing).  One step grows |lambda|
    // by at most 2 max A_lm < 2 sqrt(2 lmax + 2) (< 2^8.5 for lmax <= 16384),
    // so 4 steps stay far below overflow, and a lane that enters range inside
    // a run has values below 2^-112 * 2^34 = 2^-78 there, too small to
    // change any sum.
    __device__ __forceinline__ void check_range() {
        if (sc > 0 && fabs(l1) >= 0x1p400) {
            l1 *= 0x1p-512;
            l2 *= 0x1p-512;
            sc--;
        }
    }
};

__device__ __forceinline__ int wave_mode1(const Lane1 &L) {
    if (__all(L.sc == 0)) return 2;
    if (__all(L.sc > 0)) return 0;
    return 1;
}

}  // namespace mlcr
