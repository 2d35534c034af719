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

// Work item w = ((rc * ng + gi) * npb + pb) * GO + mo, order m = GO g + mo in
// groups g of GO consecutive orders (ng = ceil((lmax + 1) / GO) groups, items
// past lmax exit at once).  The GO orders of a group run side by side and
// share the 128-byte lines of F and G (16 B per order, ring and RHS on the
// float64 path, GO = 8; 8 B on the mixed paths, GO = 16), which are then
// fetched or written once; the ring-pair blocks of one order stay close and
// share its coefficients and U rows through L2.  Each XCD (workgroup id mod
// 8) gets one contiguous run of items; groups are visited 0, ng-1, 1, ng-2,
// ... so every run holds the same mix of long and short orders.
template <int GO = 8>
__host__ __device__ inline long long mitems(int lmax, int npb, int nrc) {
    return (long long)((lmax + GO) / GO) * GO * npb * nrc;
}

template <int GO = 8>
__device__ __forceinline__ void decode_item_m(long long total, int lmax, int npb, int &m, int &pb,
                                              int &rc, bool &ok) {
    static_assert((GO & (GO - 1)) == 0, "orders per group: a power of two");
    const long long b = blockIdx.x;
    const long long per = (total + 7) / 8;
    const long long w = (b & 7) * per + (b >> 3);
    ok = w < total;
    if (!ok) return;
    const int ng = (lmax + GO) / GO;
    const int mo = (int)(w & (GO - 1));
    long long rest = w / GO;
    pb = (int)(rest % npb);
    rest /= npb;
    const int gi = (int)(rest % ng);
    rc = (int)(rest / ng);
    const int g = (gi & 1) ? (ng - 1 - (gi >> 1)) : (gi >> 1);
    m = GO * g + mo;
    ok = m <= lmax;
}

// orders per work group: 16 when F / G hold complex float32 (mixed paths)
constexpr int kGroupF64 = 8, kGroupF32 = 16;

__device__ __forceinline__ long long tri_off_m(int m, int lmax) {
    return (long long)m * (lmax + 1) - (long long)m * (m - 1) / 2;
}

// one ring pair per lane, on the scaled recurrence mu_l = alpha_l z mu_{l-1} -
// mu_{l-2} (lambda_l = c_l mu_l; the coefficient tables hold alpha, the
// kernels' inputs and outputs carry c), values below range carried as
// v 2^{-512 sc}
struct Lane1 {
    int sc;
    double z, l1, l2;
    __device__ __forceinline__ void step_rescale(double a) {
        const double nv = fma(a * z, l1, -l2);
        l2 = l1;
        l1 = nv;
        if (sc > 0 && fabs(nv) >= 0x1p400) {
            l1 *= 0x1p-512;
            l2 *= 0x1p-512;
            sc--;
        }
    }
    __device__ __forceinline__ double w() const { return sc == 0 ? l1 : 0.0; }
    __device__ __forceinline__ void step(double a) {
        const double nv = fma(a * z, l1, -l2);
        l2 = l1;
        l1 = nv;
    }
    // Range check after a run of 4 plain steps taken while every lane of the
    // wave is still scaled (contributing nothing).  One step grows
    // max(|mu_l|, |mu_{l-1}|) by at most max alpha_lm + 1 (< 2^7.6 for
    // lmax <= 16384), so 4 steps stay far below overflow, and a lane that enters range inside
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

// U layout: per RHS chunk of 8 and order m, blocks of 16 l-steps (the element
// order inside a block depends on the arithmetic).  Order m has
// ceil((lmax - m + 1) / 16) blocks followed by kSegOrderPad zeroed ones.
__host__ __device__ inline long long b3_ceil16_sum(long long n) {   // sum_{k=1..n} ceil(k / 16)
    const long long q = n / 16, r = n % 16;
    return 8 * q * (q + 1) + r * (q + 1);
}
__host__ __device__ inline long long b3_qoff(int m, int lmax) {
    return b3_ceil16_sum(lmax + 1) - b3_ceil16_sum(lmax + 1 - m);
}

// Zeroed blocks after each order's last U block: the trailing segments of
// the segment-parallel synthesis run up to 63 steps past lmax, where the
// scaled recurrence does not vanish (mu_l = -mu_{l-2} once alpha is 0).
constexpr int kSegOrderPad = 3;
__host__ __device__ inline long long seg_qoff(int m, int lmax) {
    return b3_qoff(m, lmax) + (long long)kSegOrderPad * m;
}
__host__ __device__ inline long long seg_qtot(int lmax) { return seg_qoff(lmax + 1, lmax); }

// split-bfloat16 operands (v_mfma_f32_16x16x32_bf16)
typedef float f4b __attribute__((ext_vector_type(4)));
typedef float f2b __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// hi/lo bfloat16 pair of two float32 numbers a (low half) and b (high half)
__device__ __forceinline__ void split2(float a, float b, unsigned &h, unsigned &l) {
    h = __builtin_bit_cast(unsigned, __builtin_convertvector((f2b){a, b}, bf2));
    const float ah = __uint_as_float(h << 16), bh = __uint_as_float(h & 0xffff0000u);
    l = __builtin_bit_cast(unsigned, __builtin_convertvector((f2b){a - ah, b - bh}, bf2));
}

__device__ __forceinline__ f4b mma_b3(uint4 a, uint4 b, f4b c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                   __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

}  // namespace mlcr
