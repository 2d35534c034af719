// Segment-parallel Legendre synthesis on the matrix cores.
//
// Synthesis contracts over l (Sec. 2.1 eq. sh-synthesis): for each order m,
//     F_m[ring, c] = sum_l lambda_lm(ring) U_m[l, c].
// On the matrix cores a lane supplies the A operand of one row (ring pair) and
// a slice of the contraction index; here that slice is a contiguous
// l-segment, so a lane runs the float64 recurrence (Sec. 3.2) of its ring
// pairs over its own segment and its lambdas go straight into its A-operand
// registers, with no exchange between lanes.  A wave covers 64 ring pairs
// (32 with the 2-chain launch shape) and 4 segments (kg = lane / 16) of
// [m + ls, lmax]: lane i + 16 kg runs 4 chains, ring pairs 16 nb + i
// (nb = 0..3), which share the segment, the recurrence coefficients and the
// B operand.  The recurrence state at each segment start
// comes from a table made once per grid and band limit (k_seg_init), which
// also records ls: below m + ls every lambda of the 64 ring pairs is below
// 2^-112 (all lanes range-scaled) and contributes nothing, so those steps are
// skipped.
//
// Contraction arithmetic: float32 (v_mfma_f32_16x16x4f32), float64
// (v_mfma_f64_16x16x4f64) or split bfloat16 hi*hi + hi*lo + lo*hi
// (v_mfma_f32_16x16x32_bf16); K index = segment (16x16x4) or 8 values of one
// parity of the segment (16x16x32).
#include <algorithm>
#include <type_traits>

#include "legendre_dev.h"

namespace mlcr {

typedef double d4s __attribute__((ext_vector_type(4)));

constexpr int kSegP32 = 0, kSegP64 = 1, kSegPB3 = 2;

// ---------------------------------------------------------------------------
// start states: one wave per (m, 64 ring pairs) = 4 blocks of 16
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_seg_init(int lmax, const double *__restrict__ rz,
                                                 const double *__restrict__ rs,
                                                 const double *__restrict__ alpha,
                                                 const long long *__restrict__ aboff,
                                                 const double *__restrict__ seedc, int npairs,
                                                 int npb, int nb16, long long total,
                                                 double2 *__restrict__ st, int *__restrict__ sc,
                                                 int *__restrict__ lstab) {
    int m, pb, rc;
    bool ok;
    decode_item_m(total, lmax, npb, m, pb, rc, ok);
    if (!ok) return;
    const int lane = threadIdx.x;
    const int b16 = pb * 4 + (lane >> 4);
    const int kp = pb * 64 + lane;
    const bool valid = kp < npairs;
    const double *abm = alpha + aboff[m] - (m + 1);
    const int nl = lmax - m + 1;
    const int nu = (nl + 15) / 16;
    Lane1 L;
    L.z = valid ? rz[kp] : 0.0;
    seed_lambda_m(valid ? rs[kp] : 1.0, m, seedc[m], L.l1, L.sc);
    L.l2 = 0.0;
    const double l1s = L.l1;
    const int scs = L.sc;
    auto unit = [&](int u) {            // 16 steps from offset 16 u, range check every 4
#pragma unroll
        for (int s = 0; s < 16; s++) {
            const int l = m + 16 * u + s;
            L.step(l + 1 <= lmax ? abm[l + 1] : 0.0);
            if ((s & 3) == 3) L.check_range();
        }
    };
    // first unit boundary u (0..nu) at which the lane is in range; nu + 1: never
    int eu = nu + 1;
    for (int u = 0; u <= nu; u++) {
        if (eu > nu && L.sc == 0) eu = u;
        if (u == nu || __all(eu <= nu)) break;
        unit(u);
    }
    int mn = eu;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mn = min(mn, __shfl_xor(mn, o));
    // all 64 lanes range-scaled at boundary mn - 1 and at every check before it
    // (32-aligned: the adjoint's tiles start there too; dead blocks past nl)
    const int ls = mn > nu ? 32 * ((nl + 31) / 32) : 32 * ((16 * max(mn - 1, 0)) / 32);
    const int nlive = nl - ls;
    const int n4 = nlive > 0 ? 16 * ((nlive + 63) / 64) : 0;
    // states at the segment starts ls + k n4, k = 0..3
    L.l1 = l1s;
    L.l2 = 0.0;
    L.sc = scs;
    const long long tb = ((long long)m * nb16 + b16) * 64 + (lane & 15);
    int k = 0;
    for (int u = 0;; u++) {
        while (k < 4 && ls + k * n4 == 16 * u) {
            st[tb + 16 * k] = make_double2(L.l1, L.l2);
            sc[tb + 16 * k] = L.sc;
            k++;
        }
        if (k >= 4) break;
        unit(u);
    }
    if ((lane & 15) == 0) lstab[(long long)m * nb16 + b16] = ls;
}

// ---------------------------------------------------------------------------
// synthesis: one wave per (m, 64 ring pairs, 8 RHS)
// ---------------------------------------------------------------------------
// Lane i + 16 kg runs NB recurrence chains (NB = 4, or 2 as a tuning choice),
// ring pairs 16 nb + i of the wave's 16 NB (nb = 0..NB-1), over segment kg;
// the chains share the segment, the coefficients and the B operand, and feed
// NB MFMAs (one per 16 ring pairs).  With NB = 2 two waves cover one 64-pair
// block of the start-state table (its offset ls is the block's).
// U (per RHS chunk, order m, block q of 16 l-steps from m):
//   float32 / float64: [j][16] values, element s at l = m + 16 q + s;
//   split bf16: [p][hl][j][8], element e at l = m + 16 q + 2 e + p.
template <int P, int NB>
__global__ __launch_bounds__(64) void k_lsynth_seg(
    const void *__restrict__ Uv, int nrhs, void *__restrict__ F, long long fstride, int lmax,
    const double *__restrict__ rz, const double *__restrict__ alpha,
    const long long *__restrict__ aboff, const double2 *__restrict__ st,
    const int *__restrict__ stsc, const int *__restrict__ lstab, int nrings, int npairs, int nb16,
    int npb, long long total) {
    typedef typename std::conditional<P == kSegP64, double, float>::type T;
    typedef typename std::conditional<P == kSegP64, d4s, f4b>::type acc_t;
    static_assert(NB == 4 || NB == 2, "4 or 2 chains per lane");
    constexpr int NH = 4 / NB;                  // waves per 64-pair block
    constexpr int CS = 17;                      // padded coefficient row per segment
    __shared__ double sab[4 * CS];
    int m, pb, rc;
    bool ok;
    decode_item_m<P == kSegP64 ? kGroupF64 : kGroupF32>(total, lmax, npb * NH, m, pb, rc, ok);
    if (!ok) return;
    const int g0 = (pb % NH) * NB;              // first 16-pair group of the block
    pb /= NH;
    const int lane = threadIdx.x, kg = lane >> 4, jc = lane & 15;
    const int nl = lmax - m + 1;
    const int ls = lstab[(long long)m * nb16 + 4 * pb];
    const int nlive = nl - ls;
    const int n4 = nlive > 0 ? 16 * ((nlive + 63) / 64) : 0;
    const int nt = n4 / 16;
    // acc[nb][parity]
    acc_t acc[NB][2];
#pragma unroll
    for (int nb = 0; nb < NB; nb++) acc[nb][0] = acc[nb][1] = (acc_t){0, 0, 0, 0};
    if (nt > 0) {
        Lane1 L[NB];
#pragma unroll
        for (int nb = 0; nb < NB; nb++) {
            const int kp = pb * 64 + 16 * (g0 + nb) + jc;
            L[nb].z = kp < npairs ? rz[kp] : 0.0;
            const long long tix = ((long long)m * nb16 + 4 * pb + g0 + nb) * 64 + lane;
            const double2 s0 = st[tix];
            L[nb].l1 = s0.x;
            L[nb].l2 = s0.y;
            L[nb].sc = stsc[tix];
        }
        const int seg0 = ls + kg * n4;                  // this lane's segment, offset from m
        const long long ub = (long long)rc * seg_qtot(lmax) + seg_qoff(m, lmax);
        const double *abm = alpha + aboff[m] - (m + 1);
        // U block of step t: seg0 / 16 + t.  The last segment ends at most
        // 63 steps past lmax, inside the order's zeroed pad blocks.
        const int q0 = seg0 / 16;
        // Coefficients of step t: lane i + 16 kg holds the one for step i of
        // segment kg.  Loads for step t + 1 are issued before step t computes
        // (software pipelining), so their latency hides behind the recurrence.
        auto coef_at = [&](int t) {
            const int l = m + seg0 + 16 * t + jc;
            return (l + 1 <= lmax) ? abm[l + 1] : 0.0;
        };
        auto stage = [&](double c) {
            __syncthreads();
            sab[kg * CS + jc] = c;
            __syncthreads();
        };
        auto all_in_range = [&]() {
            bool in = true;
#pragma unroll
            for (int nb = 0; nb < NB; nb++) in = in && L[nb].sc == 0;
            return __all(in);
        };
        // lambda of chain nb at the current step (0 while range-scaled), then one step
        auto advance = [&](Lane1 &C, double c, int s, auto checked) -> double {
            double v;
            if constexpr (decltype(checked)::value) {
                v = C.sc == 0 ? C.l1 : 0.0;
                C.step(c);
                if ((s & 3) == 3) C.check_range();
            } else {
                v = C.l1;
                const double nv = fma(c * C.z, C.l1, -C.l2);
                C.l2 = C.l1;
                C.l1 = nv;
            }
            return v;
        };
        if constexpr (P == kSegPB3) {
            const uint4 *Ub = reinterpret_cast<const uint4 *>(Uv) + (ub + q0) * 64 + jc;
            auto load_u = [&](int t, uint4 (&bu)[4]) {
#pragma unroll
                for (int ph = 0; ph < 4; ph++) bu[ph] = Ub[(long long)t * 64 + ph * 16];
            };
            auto body = [&](const uint4 (&bu)[4], auto checked) {
                uint4 ah[NB][2], al[NB][2];
#pragma unroll
                for (int d = 0; d < 4; d++) {           // steps 4 d .. 4 d + 3
                    float f[NB][4];
#pragma unroll
                    for (int s4 = 0; s4 < 4; s4++) {
                        const int s = 4 * d + s4;
                        const double c = sab[kg * CS + s];
#pragma unroll
                        for (int nb = 0; nb < NB; nb++) f[nb][s4] = (float)advance(L[nb], c, s, checked);
                    }
                    // element 2 d (step 4 d + p) and 2 d + 1 (step 4 d + 2 + p) of parity p
#pragma unroll
                    for (int nb = 0; nb < NB; nb++)
#pragma unroll
                        for (int p = 0; p < 2; p++) {
                            unsigned h, l;
                            split2(f[nb][p], f[nb][2 + p], h, l);
                            reinterpret_cast<unsigned *>(&ah[nb][p])[d] = h;
                            reinterpret_cast<unsigned *>(&al[nb][p])[d] = l;
                        }
                }
#pragma unroll
                for (int nb = 0; nb < NB; nb++) {
                    acc[nb][0] = mma_b3(ah[nb][0], bu[0], acc[nb][0]);
                    acc[nb][1] = mma_b3(ah[nb][1], bu[2], acc[nb][1]);
                }
#pragma unroll
                for (int nb = 0; nb < NB; nb++) {
                    acc[nb][0] = mma_b3(ah[nb][0], bu[1], acc[nb][0]);
                    acc[nb][1] = mma_b3(ah[nb][1], bu[3], acc[nb][1]);
                }
#pragma unroll
                for (int nb = 0; nb < NB; nb++) {
                    acc[nb][0] = mma_b3(al[nb][0], bu[0], acc[nb][0]);
                    acc[nb][1] = mma_b3(al[nb][1], bu[2], acc[nb][1]);
                }
            };
            double cpre = coef_at(0);
            uint4 ucur[4], unext[4];
            load_u(0, ucur);
            auto iter = [&](int t, auto checked) {
                stage(cpre);
#pragma unroll
                for (int ph = 0; ph < 4; ph++) unext[ph] = ucur[ph];
                if (t + 1 < nt) {
                    cpre = coef_at(t + 1);
                    load_u(t + 1, unext);
                }
                body(ucur, checked);
#pragma unroll
                for (int ph = 0; ph < 4; ph++) ucur[ph] = unext[ph];
            };
            int t = 0;
            for (; t < nt && !all_in_range(); t++) iter(t, std::true_type{});
            for (; t < nt; t++) iter(t, std::false_type{});
        } else {
            constexpr int NV = 16 * (int)sizeof(T) / 16;     // uint4 per lane per block
            const uint4 *Ub = reinterpret_cast<const uint4 *>(reinterpret_cast<const T *>(Uv) +
                                                              ((ub + q0) * 16 + jc) * 16);
            auto load_u = [&](int t, uint4 (&raw)[NV]) {
#pragma unroll
                for (int v = 0; v < NV; v++) raw[v] = Ub[(long long)t * 16 * NV + v];
            };
            auto body = [&](const uint4 (&raw)[NV], auto checked) {
#pragma unroll
                for (int s = 0; s < 16; s++) {
                    const double c = sab[kg * CS + s];
                    const T u = reinterpret_cast<const T *>(raw)[s];
#pragma unroll
                    for (int nb = 0; nb < NB; nb++) {
                        const T a = (T)advance(L[nb], c, s, checked);
                        if constexpr (P == kSegP64)
                            acc[nb][s & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, u, acc[nb][s & 1], 0, 0, 0);
                        else
                            acc[nb][s & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u, acc[nb][s & 1], 0, 0, 0);
                    }
                }
            };
            // (U is not prefetched here: the extra registers cost these
            // wider-accumulator variants more occupancy than the latency they hide)
            double cpre = coef_at(0);
            auto iter = [&](int t, auto checked) {
                stage(cpre);
                uint4 ucur[NV];
                load_u(t, ucur);
                if (t + 1 < nt) cpre = coef_at(t + 1);
                body(ucur, checked);
            };
            int t = 0;
            for (; t < nt && !all_in_range(); t++) iter(t, std::true_type{});
            for (; t < nt; t++) iter(t, std::false_type{});
        }
    }
    // D[i][j] of chain nb: ring pair 64 pb + 16 (g0 + nb) + i, column j = jc = (rhs,
    // cos/sin); element v of lane j + 16 kg holds row i = 4 kg + v (float32
    // result) or kg + 4 v (float64)
    const int r = rc * 8 + (jc >> 1), cs = jc & 1;
    const int ld = lmax + 1;
    if (r < nrhs) {
        // F: complex float64 on the float64 path, complex float32 on the mixed paths
        typedef typename std::conditional<P == kSegP64, double, float>::type FO;
        FO *Fr = reinterpret_cast<FO *>(F) + 2 * (long long)r * fstride;
#pragma unroll
        for (int nb = 0; nb < NB; nb++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int i = P == kSegP64 ? kg + 4 * v : 4 * kg + v;
                const int p = pb * 64 + 16 * (g0 + nb) + i;
                if (p >= npairs) continue;
                const double e = (double)acc[nb][0][v], o = (double)acc[nb][1][v];
                const int north = p, south = nrings - 1 - p;
                Fr[((long long)north * ld + m) * 2 + cs] = (FO)(e + o);
                if (south != north) Fr[((long long)south * ld + m) * 2 + cs] = (FO)(e - o);
            }
    }
}

// ---------------------------------------------------------------------------
// split-bfloat16 synthesis over CB column blocks: one wave per (m, 16 NB
// ring pairs, 8 CB RHS)
// ---------------------------------------------------------------------------
// The same segment-parallel recurrence as k_lsynth_seg (NB chains per lane
// over segment kg = lane / 16), but each lambda, converted and split into
// bfloat16 hi/lo once, feeds CB column blocks of 16 (8 RHS x cos, sin each):
// 3 CB MFMAs per 8 values of one parity instead of 3, so the vector work of
// the recurrence and the split is shared by 8 CB right-hand sides.  The U
// block of column block cb is the block of RHS chunk CB rw + cb (the layout
// k_pack_seg writes); column blocks past the last chunk are skipped
// (wave-uniform).  Work item order as decode_item_m with rc = rw.
template <int NB, int CB>
__global__ __launch_bounds__(64) void k_lsynth_b3w(
    const uint4 *__restrict__ U, int nrhs, float2 *__restrict__ F, long long fstride, int lmax,
    const double *__restrict__ rz, const double *__restrict__ alpha,
    const long long *__restrict__ aboff, const double2 *__restrict__ st,
    const int *__restrict__ stsc, const int *__restrict__ lstab, int nrings, int npairs, int nb16,
    int npb, long long total) {
    static_assert(NB == 2 || NB == 4, "2 or 4 chains per lane");
    constexpr int NH = 4 / NB;
    constexpr int CS = 17;
    __shared__ double sab[4 * CS];
    int m, pb, rw;
    bool ok;
    decode_item_m<kGroupF32>(total, lmax, npb * NH, m, pb, rw, ok);
    if (!ok) return;
    const int g0 = (pb % NH) * NB;
    pb /= NH;
    const int lane = threadIdx.x, kg = lane >> 4, jc = lane & 15;
    const int nrc = (nrhs + 7) / 8;
    const int ncb = min(CB, nrc - rw * CB);          // column blocks holding RHS (wave-uniform)
    const int nl = lmax - m + 1;
    const int ls = lstab[(long long)m * nb16 + 4 * pb];
    const int nlive = nl - ls;
    const int n4 = nlive > 0 ? 16 * ((nlive + 63) / 64) : 0;
    const int nt = n4 / 16;
    f4b acc[CB][NB][2];
#pragma unroll
    for (int cb = 0; cb < CB; cb++)
#pragma unroll
        for (int nb = 0; nb < NB; nb++) acc[cb][nb][0] = acc[cb][nb][1] = (f4b){0, 0, 0, 0};
    if (nt > 0) {
        Lane1 L[NB];
#pragma unroll
        for (int nb = 0; nb < NB; nb++) {
            const int kp = pb * 64 + 16 * (g0 + nb) + jc;
            L[nb].z = kp < npairs ? rz[kp] : 0.0;
            const long long tix = ((long long)m * nb16 + 4 * pb + g0 + nb) * 64 + lane;
            const double2 s0 = st[tix];
            L[nb].l1 = s0.x;
            L[nb].l2 = s0.y;
            L[nb].sc = stsc[tix];
        }
        const int seg0 = ls + kg * n4;
        const long long qt = seg_qtot(lmax);
        const uint4 *Ub = U + ((long long)rw * CB * qt + seg_qoff(m, lmax) + seg0 / 16) * 64 + jc;
        const double *abm = alpha + aboff[m] - (m + 1);
        auto coef_at = [&](int t) {
            const int l = m + seg0 + 16 * t + jc;
            return (l + 1 <= lmax) ? abm[l + 1] : 0.0;
        };
        auto stage = [&](double c) {
            __syncthreads();
            sab[kg * CS + jc] = c;
            __syncthreads();
        };
        auto all_in_range = [&]() {
            bool in = true;
#pragma unroll
            for (int nb = 0; nb < NB; nb++) in = in && L[nb].sc == 0;
            return __all(in);
        };
        auto advance = [&](Lane1 &C, double c, int s, auto checked) -> double {
            double v;
            if constexpr (decltype(checked)::value) {
                v = C.sc == 0 ? C.l1 : 0.0;
                C.step(c);
                if ((s & 3) == 3) C.check_range();
            } else {
                v = C.l1;
                const double nv = fma(c * C.z, C.l1, -C.l2);
                C.l2 = C.l1;
                C.l1 = nv;
            }
            return v;
        };
        auto body = [&](int t, auto checked) {
            // the U blocks of every column block for these 16 steps (chunk CB rw + cb)
            uint4 bu[CB][4];
#pragma unroll
            for (int cb = 0; cb < CB; cb++)
                if (cb < ncb) {
#pragma unroll
                    for (int ph = 0; ph < 4; ph++)
                        bu[cb][ph] = Ub[((long long)cb * qt + t) * 64 + ph * 16];
                }
            // chain by chain: 16 steps, the split, then its 6 CB MFMAs (hi*hi,
            // hi*lo, lo*hi over the column blocks and parities), so only one
            // chain's operands are live at a time
#pragma unroll
            for (int nb = 0; nb < NB; nb++) {
                float f[16];
#pragma unroll
                for (int s = 0; s < 16; s++) f[s] = (float)advance(L[nb], sab[kg * CS + s], s, checked);
                uint4 ah[2], al[2];
#pragma unroll
                for (int d = 0; d < 4; d++)
#pragma unroll
                    for (int p = 0; p < 2; p++) {
                        unsigned h, l;
                        split2(f[4 * d + p], f[4 * d + 2 + p], h, l);
                        reinterpret_cast<unsigned *>(&ah[p])[d] = h;
                        reinterpret_cast<unsigned *>(&al[p])[d] = l;
                    }
#pragma unroll
                for (int cb = 0; cb < CB; cb++)
                    if (cb < ncb) {
                        acc[cb][nb][0] = mma_b3(ah[0], bu[cb][0], acc[cb][nb][0]);
                        acc[cb][nb][1] = mma_b3(ah[1], bu[cb][2], acc[cb][nb][1]);
                    }
#pragma unroll
                for (int cb = 0; cb < CB; cb++)
                    if (cb < ncb) {
                        acc[cb][nb][0] = mma_b3(ah[0], bu[cb][1], acc[cb][nb][0]);
                        acc[cb][nb][1] = mma_b3(ah[1], bu[cb][3], acc[cb][nb][1]);
                    }
#pragma unroll
                for (int cb = 0; cb < CB; cb++)
                    if (cb < ncb) {
                        acc[cb][nb][0] = mma_b3(al[0], bu[cb][0], acc[cb][nb][0]);
                        acc[cb][nb][1] = mma_b3(al[1], bu[cb][2], acc[cb][nb][1]);
                    }
            }
        };
        double cpre = coef_at(0);
        auto iter = [&](int t, auto checked) {
            stage(cpre);
            if (t + 1 < nt) cpre = coef_at(t + 1);
            body(t, checked);
        };
        int t = 0;
        for (; t < nt && !all_in_range(); t++) iter(t, std::true_type{});
        for (; t < nt; t++) iter(t, std::false_type{});
    }
    // D[i][j]: ring pair 64 pb + 16 (g0 + nb) + i (i = 4 kg + v), column j = jc
    const int ld = lmax + 1;
#pragma unroll
    for (int cb = 0; cb < CB; cb++) {
        const int r = (rw * CB + cb) * 8 + (jc >> 1), cs = jc & 1;
        if (cb >= ncb || r >= nrhs) continue;
        float *Fr = reinterpret_cast<float *>(F + (long long)r * fstride);
#pragma unroll
        for (int nb = 0; nb < NB; nb++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int i = 4 * kg + v;
                const int p = pb * 64 + 16 * (g0 + nb) + i;
                if (p >= npairs) continue;
                const double e = (double)acc[cb][nb][0][v], o = (double)acc[cb][nb][1][v];
                const int north = p, south = nrings - 1 - p;
                Fr[((long long)north * ld + m) * 2 + cs] = (float)(e + o);
                if (south != north) Fr[((long long)south * ld + m) * 2 + cs] = (float)(e - o);
            }
    }
}

// U from x, times c_lm (lambda = c mu) and the per-l weights dl (e.g. the
// beam): one workgroup per (m, RHS chunk); tiles of 64 l are read along l for
// each of the 16 columns (j = 2 r + cos/sin) into LDS and written as whole
// 16-step blocks, then the order's zeroed pad blocks.
template <int P>
__global__ __launch_bounds__(256) void k_pack_seg(const double *__restrict__ x,
                                                  const double *__restrict__ dl,
                                                  const double *__restrict__ cfac, int glmax,
                                                  void *__restrict__ Uv, int lmax, int nrhs) {
    constexpr int TL = 64;
    __shared__ double tile[16][TL + 1];
    const int m = blockIdx.x, rc = blockIdx.y;
    const long long nalm = (long long)(lmax + 1) * (lmax + 1);
    const int nl = lmax - m + 1;
    const long long ob = cos_base(m, lmax);
    const long long qb = (long long)rc * seg_qtot(lmax) + seg_qoff(m, lmax);
    const double *cm = cfac + tri_off_m(m, glmax) - m;   // c_lm at cm[l]
    constexpr int BU = P == kSegP64 ? 128 : 64;          // uint4 per 16-step block
    uint4 *U = reinterpret_cast<uint4 *>(Uv);
    {
        uint4 *pad = U + (qb + (nl + 15) / 16) * BU;
        for (int i = threadIdx.x; i < kSegOrderPad * BU; i += blockDim.x)
            pad[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    for (int base = 0; base < nl; base += TL) {
        for (int e = threadIdx.x; e < 16 * TL; e += blockDim.x) {
            const int j = e / TL, o = e % TL;
            const int r = rc * 8 + (j >> 1), cs = j & 1;
            double v = 0.0;
            if (base + o < nl && r < nrhs && !(m == 0 && cs == 1)) {
                v = x[(long long)r * nalm + ob + (long long)cs * nl + base + o] * cm[m + base + o];
                if (dl) v *= dl[m + base + o];
            }
            tile[j][o] = v;
        }
        __syncthreads();
        const int nqt = min(TL, nl - base + 15) / 16;    // blocks of this tile
        uint4 *Ut = U + (qb + base / 16) * BU;
        if constexpr (P == kSegPB3) {
            // [p][hl][j][8]: element e of parity p at step 2 e + p
            for (int w = threadIdx.x; w < nqt * 2 * 16; w += blockDim.x) {
                const int qq = w / 32, p = (w / 16) & 1, j = w & 15;
                uint4 h, l;
                const double *t = &tile[j][16 * qq + p];
                split2((float)t[0], (float)t[2], h.x, l.x);
                split2((float)t[4], (float)t[6], h.y, l.y);
                split2((float)t[8], (float)t[10], h.z, l.z);
                split2((float)t[12], (float)t[14], h.w, l.w);
                Ut[qq * 64 + (2 * p) * 16 + j] = h;
                Ut[qq * 64 + (2 * p + 1) * 16 + j] = l;
            }
        } else {
            // [j][16]: element s at step s, 4 (float32) or 2 (float64) per uint4
            constexpr int PER = P == kSegP64 ? 2 : 4;
            for (int w = threadIdx.x; w < nqt * BU; w += blockDim.x) {
                const int qq = w / BU, rem = w % BU;
                const int j = rem / (16 / PER), s0 = (rem % (16 / PER)) * PER;
                const double *t = &tile[j][16 * qq + s0];
                uint4 o;
                if constexpr (P == kSegP64) {
                    const double2 d = make_double2(t[0], t[1]);
                    o = *reinterpret_cast<const uint4 *>(&d);
                } else {
                    o = make_uint4(__float_as_uint((float)t[0]), __float_as_uint((float)t[1]),
                                   __float_as_uint((float)t[2]), __float_as_uint((float)t[3]));
                }
                Ut[w] = o;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Column blocks of 16 (8 RHS) that one split-bfloat16 wave takes: 4 from 32
// RHS on, 2 from 16, else 1 (the 8-RHS kernel).
int bf16_synth_cols(int nrhs) { return nrhs >= 16 ? 2 : 1; }

long long seg_u_bytes(int lmax, int nrhs, int prec) {
    return (long long)((nrhs + 7) / 8) * seg_qtot(lmax) * (prec == MLCR_FP64 ? 2048 : 1024);
}

int seg_table(mlcr_geom *g, int lmax, hipStream_t s, const SegTable **out) {
    for (const SegTable &t : g->seg)
        if (t.lmax == lmax) {
            *out = &t;
            return MLCR_OK;
        }
    const int npb = (g->npairs + 63) / 64;
    const int nb16 = 4 * npb;
    const size_t n = (size_t)(lmax + 1) * nb16 * 64;
    SegTable t;
    t.lmax = lmax;
    if (t.st.reserve(n * sizeof(double2)) || t.sc.reserve(n * sizeof(int)) ||
        t.ls.reserve((size_t)(lmax + 1) * nb16 * sizeof(int))) {
        t.st.release();
        t.sc.release();
        t.ls.release();
        return fail(MLCR_ENOMEM, "segment start-state table allocation failed");
    }
    const long long total = mitems(lmax, npb, 1);
    const long long grid = ((total + 7) / 8) * 8;
    hipLaunchKernelGGL(k_seg_init, dim3((unsigned)grid), dim3(64), 0, s, lmax, g->ring_z.as<double>(),
                       g->ring_s.as<double>(), g->alpha.as<double>(), g->aboff.as<long long>(),
                       g->seed.as<double>(), g->npairs, npb, nb16, total, t.st.as<double2>(),
                       t.sc.as<int>(), t.ls.as<int>());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        t.st.release();
        t.sc.release();
        t.ls.release();
        return fail(MLCR_EHIP, std::string("k_seg_init: ") + hipGetErrorString(e));
    }
    g->seg.push_back(std::move(t));
    *out = &g->seg.back();
    return MLCR_OK;
}

int launch_pack_seg(const mlcr_geom *g, int lmax, int nrhs, const double *x, const double *dl,
                    void *U, int prec, hipStream_t s) {
    const int nrc = (nrhs + 7) / 8;
    if (prec == MLCR_BF16X3)
        hipLaunchKernelGGL(k_pack_seg<kSegPB3>, dim3(lmax + 1, nrc), dim3(256), 0, s, x, dl,
                           g->cfac.as<double>(), g->lmax, U, lmax, nrhs);
    else if (prec == MLCR_FP64)
        hipLaunchKernelGGL(k_pack_seg<kSegP64>, dim3(lmax + 1, nrc), dim3(256), 0, s, x, dl,
                           g->cfac.as<double>(), g->lmax, U, lmax, nrhs);
    else
        hipLaunchKernelGGL(k_pack_seg<kSegP32>, dim3(lmax + 1, nrc), dim3(256), 0, s, x, dl,
                           g->cfac.as<double>(), g->lmax, U, lmax, nrhs);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_legendre_synth_seg(const LegendreArgs &a, const SegTable *t, const void *U, void *F,
                              int prec) {
    const mlcr_geom *g = a.g;
    if (t->lmax != a.lmax) return fail(MLCR_EINVAL, "segment table of another band limit");
    const int nb16 = 4 * ((g->npairs + 63) / 64);
    const int npb = (g->npairs + 63) / 64;
    const int nrc = (a.nrhs + 7) / 8;
    const int nb = g->tune[prec].synth_chains;          // chains per lane: 4 or 2
    const long long total = prec == MLCR_FP64 ? mitems<kGroupF64>(a.lmax, npb * (4 / nb), nrc)
                                              : mitems<kGroupF32>(a.lmax, npb * (4 / nb), nrc);
    const long long grid = ((total + 7) / 8) * 8;
    const long long fstride = (long long)g->nrings * (a.lmax + 1);
#define MLCR_SEG_ARGS                                                                           \
    U, a.nrhs, F, fstride, a.lmax, g->ring_z.as<double>(), g->alpha.as<double>(),               \
        g->aboff.as<long long>(), t->st.as<double2>(), t->sc.as<int>(), t->ls.as<int>(),         \
        g->nrings, g->npairs, nb16, npb, total
#define MLCR_SEG_LAUNCH(PP, NBV)                                                                \
    hipLaunchKernelGGL((k_lsynth_seg<PP, NBV>), dim3((unsigned)grid), dim3(64), 0, a.stream,     \
                       MLCR_SEG_ARGS)
    const int cbw = prec == MLCR_BF16X3 ? bf16_synth_cols(a.nrhs) : 1;
    if (prec == MLCR_BF16X3 && cbw > 1) {
        // CB column blocks per wave share each lambda (two chains per lane)
        const int nrw = (nrc + cbw - 1) / cbw;
        const long long tw = mitems<kGroupF32>(a.lmax, npb, nrw);
        const long long gw = ((tw + 7) / 8) * 8;
#define MLCR_B3W_LAUNCH(CBV)                                                                     \
    hipLaunchKernelGGL((k_lsynth_b3w<4, CBV>), dim3((unsigned)gw), dim3(64), 0, a.stream,          \
                       reinterpret_cast<const uint4 *>(U), a.nrhs, static_cast<float2 *>(F), fstride, \
                       a.lmax,                                                                      \
                       g->ring_z.as<double>(), g->alpha.as<double>(), g->aboff.as<long long>(),      \
                       t->st.as<double2>(), t->sc.as<int>(), t->ls.as<int>(), g->nrings, g->npairs,  \
                       nb16, npb, tw)
        MLCR_B3W_LAUNCH(2);
#undef MLCR_B3W_LAUNCH
    } else if (prec == MLCR_BF16X3) {
        if (nb == 2) MLCR_SEG_LAUNCH(kSegPB3, 2);
        else MLCR_SEG_LAUNCH(kSegPB3, 4);
    } else if (prec == MLCR_FP64) {
        if (nb == 2) MLCR_SEG_LAUNCH(kSegP64, 2);
        else MLCR_SEG_LAUNCH(kSegP64, 4);
    } else {
        if (nb == 2) MLCR_SEG_LAUNCH(kSegP32, 2);
        else MLCR_SEG_LAUNCH(kSegP32, 4);
    }
#undef MLCR_SEG_LAUNCH
#undef MLCR_SEG_ARGS
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

}  // namespace mlcr
