// Ring step of the spherical harmonic transforms, and the pixel diagonal.
//
// For ring k with N = 4i pixels at phi_j = phi0 + 2 pi j / N, synthesis is
//     f_j = sum_m w_m (F^c_m cos m phi_j + F^s_m sin m phi_j),  w_0 = 1, w_m = sqrt 2,
// the real part of a length-N inverse DFT of the coefficients
// H_m = w_m (F^c_m - i F^s_m) e^{i m phi0} folded modulo N (eq. sh-synthesis
// restricted to one iso-latitude ring; m >= N/2 is aliased exactly, which
// the method's under-pixelized grids need, Sec. 3.3).  Adjoint synthesis
// (Sec. 2.1) is its exact transpose:
//     G^c_m + i G^s_m = w_m e^{i m phi0} conj(Y_{m mod N}),  Y_q = sum_j y_j e^{-2 pi i q j / N}.
//
// Both directions use one complex DFT of length n = N/2 on the packed map
// z_t = f_2t + i f_2t+1.  When n is a power of two it is a radix-2 Stockham
// FFT in LDS; otherwise Bluestein's chirp-z convolution with a power-of-two
// FFT of size M >= 2n - 1 and a precomputed filter.  The phase e^{i m phi0}
// is e^{i pi m p / N} with p in {0, 1}, so every twiddle, phase and chirp of
// a ring comes from one table T_N[j] = e^{i pi j / N}.
//
// In the fused operator kernel the map never leaves LDS: F is read, the map
// is multiplied by N^-1 (0 in the mask, Sec. 2.3), and G is written over F.
// One workgroup per (ring, right-hand side): 512 threads, or 1024 for FFT
// sizes above 4096 (the default launch shape; 512 as a tuning choice).  Rings are
// launched in groups of similar FFT size, each with the LDS its largest ring
// needs; within a launch the rings are dealt round-robin to the eight XCDs
// (workgroup id mod 8) and the right-hand sides of one ring run back to back
// on the same XCD, so its tables are fetched into that L2 once.
#include "mlcr_internal.h"

namespace mlcr {

static constexpr int kRingThreads = 512;
// Rings of at most kFoldMax pixels fold their coefficients cooperatively
// (all threads of the block, partial sums in LDS): there the fold
// sum over m = q mod N has (lmax + 1) / N terms per residue q.
static constexpr int kFoldMax = 1024;
static constexpr double kSqrt2 = 1.4142135623730950488;

// Complex arithmetic on double2 (float64 path) and float2 (the float32 FFT of
// the mixed-precision operator step).
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

template <typename C>
struct ScalarOf;
template <>
struct ScalarOf<double2> {
    typedef double T;
};
template <>
struct ScalarOf<float2> {
    typedef float T;
};

template <typename C>
__device__ __forceinline__ C to_c(double2 v);
template <>
__device__ __forceinline__ double2 to_c<double2>(double2 v) { return v; }
template <>
__device__ __forceinline__ float2 to_c<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ double2 to_d(double2 v) { return v; }
__device__ __forceinline__ double2 to_d(float2 v) { return make_double2((double)v.x, (double)v.y); }

// Small DFTs in registers.  Forward: X_r = sum_j x_j e^{-2 pi i j r / R};
// INV flips the sign of the exponent.
template <bool INV, typename C>
__device__ __forceinline__ C mul_mi(C a) {      // a * (-i), or a * i if INV
    C o;
    o.x = INV ? -a.y : a.y;
    o.y = INV ? a.x : -a.x;
    return o;
}

template <bool INV, typename C>
__device__ __forceinline__ void dft4(C &x0, C &x1, C &x2, C &x3) {
    const C a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3);
    const C d = mul_mi<INV>(csub(x1, x3));
    x0 = cadd(a, c);
    x2 = csub(a, c);
    x1 = cadd(b, d);
    x3 = csub(b, d);
}

template <int R, bool INV, typename C>
__device__ __forceinline__ void dft(C (&x)[R]) {
    typedef typename ScalarOf<C>::T S;
    if constexpr (R == 2) {
        const C a = x[0];
        x[0] = cadd(a, x[1]);
        x[1] = csub(a, x[1]);
    } else if constexpr (R == 4) {
        dft4<INV>(x[0], x[1], x[2], x[3]);
    } else {
        // radix-2 split into even and odd 4-point DFTs, then w^r = e^{-2 pi i r / 8}
        C e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
        C o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
        dft4<INV>(e0, e1, e2, e3);
        dft4<INV>(o0, o1, o2, o3);
        constexpr S h = (S)0.70710678118654752440;
        C w1o, w3o;
        if (INV) {
            w1o.x = h * (o1.x - o1.y);
            w1o.y = h * (o1.x + o1.y);
            w3o.x = -h * (o3.x + o3.y);
            w3o.y = h * (o3.x - o3.y);
        } else {
            w1o.x = h * (o1.x + o1.y);
            w1o.y = h * (o1.y - o1.x);
            w3o.x = h * (o3.y - o3.x);
            w3o.y = -h * (o3.x + o3.y);
        }
        const C w2o = mul_mi<INV>(o2);
        x[0] = cadd(e0, o0);
        x[4] = csub(e0, o0);
        x[1] = cadd(e1, w1o);
        x[5] = csub(e1, w1o);
        x[2] = cadd(e2, w2o);
        x[6] = csub(e2, w2o);
        x[3] = cadd(e3, w3o);
        x[7] = csub(e3, w3o);
    }
}

// Twiddles of one radix-8 pass (stride p) for this thread's butterflies i
// (k = i mod p): w, w^2 and w^4 with w = e^{-2 pi i k / (8 p)} (conjugated
// for the inverse), read from W[j] = e^{-2 pi i j / Wmax}.  The other powers
// are products of these (at most two roundings past the table's).  They are
// loaded one pass ahead, so the table latency hides behind the current
// pass.
template <bool INV, int NT, typename C>
struct Tw8 {
    static constexpr int CM = 8192 / (8 * NT) > 0 ? 8192 / (8 * NT) : 1;
    C w1[CM], w2[CM], w4[CM];
    __device__ __forceinline__ void load(int M, int p, const C *__restrict__ W, int Wmax) {
        const int T = M / 8;
        const int ts = Wmax / (8 * p);
#pragma unroll
        for (int c = 0; c < CM; c++) {
            const int i = threadIdx.x + c * NT;
            if (i < T) {
                const int k = i & (p - 1);
                w1[c] = W[k * ts];
                w2[c] = W[2 * k * ts];
                w4[c] = W[4 * k * ts];
                if (INV) {
                    w1[c].y = -w1[c].y;
                    w2[c].y = -w2[c].y;
                    w4[c].y = -w4[c].y;
                }
            }
        }
    }
};

// One radix-R Stockham pass over the M values in LDS (stride p so far):
// butterfly i (k = i mod p) reads x[i + j M/R], scales input j by
// w^{j k} with w = e^{-2 pi i / (p R)}, does an R-point DFT and writes
// output r to x[(i - k) R + k + r p].  tw: the pass's twiddles (radix 8,
// p > 1), null for p = 1.
template <int R, bool INV, int NT, typename C>
__device__ __forceinline__ void fft_pass(C *buf, int M, int p, const Tw8<INV, NT, C> *tw) {
    constexpr int CMAX = 8192 / (R * NT) > 0 ? 8192 / (R * NT) : 1;
    const int T = M / R;
    C v[CMAX][R];
#pragma unroll
    for (int c = 0; c < CMAX; c++) {
        const int i = threadIdx.x + c * NT;
        if (i < T) {
#pragma unroll
            for (int j = 0; j < R; j++) v[c][j] = buf[i + j * T];
            if constexpr (R == 8) {
                if (tw) {
                    const C w1 = tw->w1[c], w2 = tw->w2[c], w4 = tw->w4[c];
                    const C w3 = cmul(w1, w2);
                    v[c][1] = cmul(v[c][1], w1);
                    v[c][2] = cmul(v[c][2], w2);
                    v[c][3] = cmul(v[c][3], w3);
                    v[c][4] = cmul(v[c][4], w4);
                    v[c][5] = cmul(v[c][5], cmul(w1, w4));
                    v[c][6] = cmul(v[c][6], cmul(w2, w4));
                    v[c][7] = cmul(v[c][7], cmul(w3, w4));
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CMAX; c++) {
        const int i = threadIdx.x + c * NT;
        if (i < T) {
            const int k = i & (p - 1);
            dft<R, INV>(v[c]);
            const int jo = (i - k) * R + k;
#pragma unroll
            for (int j = 0; j < R; j++) buf[jo + j * p] = v[c][j];
        }
    }
    __syncthreads();
}

// Unnormalized DFT of size M (a power of two, M <= 8192) held in LDS, in
// place, all threads of the block taking part: one radix-2, radix-4 or
// radix-8 pass with stride 1 (no twiddles), then radix-8 passes.
template <bool INV, int NT, typename C>
__device__ void lds_fft_t(C *buf, int M, const C *__restrict__ W, int Wmax) {
    if (M < 2) return;
    const int lg = 31 - __clz(M);
    const int p1 = lg % 3 == 1 ? 2 : (lg % 3 == 2 ? 4 : 8);   // stride after the first pass
    Tw8<INV, NT, C> tw{}, tn{};
    if (p1 < M) tw.load(M, p1, W, Wmax);
    if (p1 == 2) fft_pass<2, INV, NT>(buf, M, 1, (const Tw8<INV, NT, C> *)nullptr);
    else if (p1 == 4) fft_pass<4, INV, NT>(buf, M, 1, (const Tw8<INV, NT, C> *)nullptr);
    else fft_pass<8, INV, NT>(buf, M, 1, (const Tw8<INV, NT, C> *)nullptr);
    for (int p = p1; p < M; p *= 8) {
        if (8 * p < M) tn.load(M, 8 * p, W, Wmax);
        fft_pass<8, INV, NT>(buf, M, p, &tw);
        tw = tn;
    }
}

template <int NT, typename C>
__device__ __forceinline__ void lds_fft(C *buf, int M, bool inverse, const C *__restrict__ W,
                                        int Wmax) {
    if (inverse) lds_fft_t<true, NT>(buf, M, W, Wmax);
    else lds_fft_t<false, NT>(buf, M, W, Wmax);
}

// Folded, phased coefficient  Hhat_q = sum_{m = q mod N} H_m  for 0 <= q < N.
template <typename FT>
__device__ __forceinline__ double2 hhat(const FT *__restrict__ Fk, int q, int N, int p,
                                        int lmax, const double2 *__restrict__ TN) {
    double ax = 0.0, ay = 0.0;
    int j = 0;
    for (int m = q; m <= lmax; m += N, j++) {
        const double2 f = to_d(Fk[m]);
        double w = (m == 0) ? 1.0 : kSqrt2;
        if ((j * p) & 1) w = -w;        // e^{i pi (q + jN) p / N} = e^{i pi q p / N} (-1)^{jp}
        ax = fma(w, f.x, ax);
        ay = fma(-w, f.y, ay);
    }
    return cmul(make_double2(ax, ay), TN[(q * p) % (2 * N)]);
}

// Hhat_q for every q < N (N <= kFoldMax) into hb, all NT threads taking part:
// G = max(1, NT / N) threads per residue q sum every G-th term of its fold,
// and the G partial sums are added in a fixed order (deterministic).
template <int NT, typename FT>
__device__ void fold_coop(const FT *__restrict__ Fk, int N, int p, int lmax,
                          const double2 *__restrict__ TN, double2 *hb, double2 *pb) {
    const int G = N >= NT ? 1 : NT / N;
    for (int t = threadIdx.x; t < G * N; t += NT) {
        const int q = t % N, g = t / N;
        double ax = 0.0, ay = 0.0;
        int j = g;
        for (int m = q + g * N; m <= lmax; m += G * N, j += G) {
            const double2 f = to_d(Fk[m]);
            double w = (m == 0) ? 1.0 : kSqrt2;
            if ((j * p) & 1) w = -w;
            ax = fma(w, f.x, ax);
            ay = fma(-w, f.y, ay);
        }
        pb[t] = make_double2(ax, ay);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < N; q += NT) {
        double2 s = pb[q];
        for (int g = 1; g < G; g++) s = cadd(s, pb[g * N + q]);
        hb[q] = cmul(s, TN[(q * p) % (2 * N)]);
    }
    __syncthreads();
}

// chirp q_t = e^{i pi t^2 / n} = T_N[2 t^2 mod 2N]
__device__ __forceinline__ double2 chirp(const double2 *__restrict__ TN, int t, int N) {
    return TN[(int)((2LL * t * t) % (2LL * N))];
}

// MODE 0: F -> map.  MODE 1: map -> G.  MODE 2: F -> N^-1 map -> G (G over F).
// C: complex type of F and G in HBM, of the LDS buffer, the FFTs and the
// Bluestein filter (double2, or float2 on the mixed-precision paths); the fold
// and unfold with their phases run in float64 either way.
template <int MODE, int NT, typename C>
__global__ __launch_bounds__(NT) void k_ring(
    const C *Fin, C *Gout, const double *__restrict__ map_in,
    double *__restrict__ map_out, const double *__restrict__ ninv,
    const RingInfo *__restrict__ rings, const LenInfo *__restrict__ lens,
    const int *__restrict__ order, const double2 *__restrict__ T, const C *__restrict__ Bf,
    const C *__restrict__ W, int Wmax, int lmax, long long fstride, long long npix,
    int goff, int gcount, int nrhs, int hoff) {
    typedef typename ScalarOf<C>::T S;
    extern __shared__ __align__(16) unsigned char smem_ring[];
    C *buf = reinterpret_cast<C *>(smem_ring);
    const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
    const int jr = (seq / nrhs) * 8 + xcd;
    if (jr >= gcount) return;
    const int k = order[goff + jr];
    const int r = seq % nrhs;
    const int tid = threadIdx.x;
    const RingInfo ri = rings[k];
    const LenInfo L = lens[ri.tab];
    const int N = ri.nphi, n = N >> 1, p = ri.phase;
    const double2 *TN = T + L.toff;
    const bool blue = L.boff >= 0;
    const int M = L.M;
    const C *Bk = Bf + (blue ? L.boff : 0);
    const S invM = (S)(1.0 / (double)M);
    const int ld = lmax + 1;
    const long long pix0 = (long long)r * npix + ri.start;
    const C czero = to_c<C>(make_double2(0.0, 0.0));
    // Bluestein chirps of this thread's t < n, held in registers for the up
    // to three pointwise passes that use them (loaded here, ahead of use);
    // in the 1024-thread launches only, where the registers are free
    constexpr int KCH = NT >= 1024 ? 4 : 1;
    const bool cch = NT >= 1024 && blue && n <= KCH * NT;
    C chv[KCH];
    if (cch) {
#pragma unroll
        for (int c = 0; c < KCH; c++) {
            const int t = tid + c * NT;
            chv[c] = t < n ? to_c<C>(chirp(TN, t, N)) : czero;
        }
    }
    // buf[t] = op(buf[t], chirp_t) for t < n
    auto with_chirp = [&](auto op) {
        if (cch) {
#pragma unroll
            for (int c = 0; c < KCH; c++) {
                const int t = tid + c * NT;
                if (t < n) buf[t] = op(buf[t], chv[c]);
            }
        } else {
            for (int t = tid; t < n; t += NT) buf[t] = op(buf[t], to_c<C>(chirp(TN, t, N)));
        }
    };

    if (MODE != 1) {
        const C *Fk = Fin + (long long)r * fstride + (long long)k * ld;
        if (blue)
            for (int t = n + tid; t < M; t += NT) buf[t] = czero;
        // folded coefficients: in LDS for short rings (hoff: byte offset of
        // kFoldMax + max(NT, kFoldMax) double2 past the FFT buffer), else per
        // thread from F
        const bool coop = N <= kFoldMax;            // uniform over the block
        double2 *hb = reinterpret_cast<double2 *>(smem_ring + hoff);
        if (coop) fold_coop<NT>(Fk, N, p, lmax, TN, hb, hb + kFoldMax);
        auto H = [&](int q) { return coop ? hb[q] : hhat(Fk, q, N, p, lmax, TN); };
        // Z_k = (G_k + G_{k+n}) + i w^k (G_k - G_{k+n}),  G_q = (Hhat_q + conj Hhat_{N-q}) / 2,
        // w = e^{2 pi i / N}: the length-n DFT input whose inverse is z_t = f_2t + i f_2t+1.
        for (int kk = tid; 2 * kk <= n; kk += NT) {
            const int i1 = kk == 0 ? 0 : N - kk;
            const double2 H0 = H(kk);
            const double2 H1 = H(i1);
            const double2 H2 = H(kk + n);
            const double2 H3 = H(n - kk);
            {
                const double2 g0 = cscale(cadd(H0, cconj(H1)), 0.5);
                const double2 g1 = cscale(cadd(H2, cconj(H3)), 0.5);
                const double2 d = cmul(TN[2 * kk], csub(g0, g1));
                double2 Z = make_double2(g0.x + g1.x - d.y, g0.y + g1.y + d.x);
                if (blue) Z = cmul(Z, chirp(TN, kk, N));
                buf[kk] = to_c<C>(Z);
            }
            const int k2 = n - kk;
            if (kk > 0 && k2 > kk) {
                const double2 g0 = cscale(cadd(H3, cconj(H2)), 0.5);
                const double2 g1 = cscale(cadd(H1, cconj(H0)), 0.5);
                const double2 d = cmul(TN[2 * k2], csub(g0, g1));
                double2 Z = make_double2(g0.x + g1.x - d.y, g0.y + g1.y + d.x);
                if (blue) Z = cmul(Z, chirp(TN, k2, N));
                buf[k2] = to_c<C>(Z);
            }
        }
        __syncthreads();
        if (!blue) {
            lds_fft<NT>(buf, n, true, W, Wmax);
        } else {
            lds_fft<NT>(buf, M, false, W, Wmax);
            for (int t = tid; t < M; t += NT) buf[t] = cmul(buf[t], Bk[t]);
            __syncthreads();
            lds_fft<NT>(buf, M, true, W, Wmax);
            if constexpr (NT >= 1024) {
                with_chirp([&](C v, C ch) { return cscale(cmul(v, ch), invM); });
            } else {
                for (int t = tid; t < n; t += NT)
                    buf[t] = cscale(cmul(buf[t], to_c<C>(chirp(TN, t, N))), invM);
            }
            __syncthreads();
        }
        if (MODE == 0) {
            double2 *out = reinterpret_cast<double2 *>(map_out + pix0);
            for (int t = tid; t < n; t += NT) out[t] = to_d(buf[t]);
            return;
        }
        const double2 *ni = reinterpret_cast<const double2 *>(ninv + ri.start);
        for (int t = tid; t < n; t += NT) {
            const double2 w = ni[t];
            const C v = buf[t];
            C o;
            o.x = v.x * (S)w.x;
            o.y = v.y * (S)w.y;
            buf[t] = o;
        }
    } else {
        const double2 *in = reinterpret_cast<const double2 *>(map_in + pix0);
        for (int t = tid; t < n; t += NT) buf[t] = to_c<C>(in[t]);
    }
    // forward DFT of z (adjoint direction)
    if (!blue) {
        __syncthreads();
        lds_fft<NT>(buf, n, false, W, Wmax);
    } else {
        if (NT >= 1024 && cch) {
            for (int t = n + tid; t < M; t += NT) buf[t] = czero;
            with_chirp([&](C v, C ch) { return cmul(v, cconj(ch)); });
        } else {
            for (int t = tid; t < M; t += NT)
                buf[t] = (t < n) ? cmul(buf[t], to_c<C>(cconj(chirp(TN, t, N)))) : czero;
        }
        __syncthreads();
        lds_fft<NT>(buf, M, false, W, Wmax);
        for (int t = tid; t < M; t += NT) buf[t] = cmul(buf[t], cconj(Bk[t]));
        __syncthreads();
        lds_fft<NT>(buf, M, true, W, Wmax);
        if constexpr (NT >= 1024) {
            with_chirp([&](C v, C ch) { return cscale(cmul(v, cconj(ch)), invM); });
        } else {
            for (int t = tid; t < n; t += NT)
                buf[t] = cscale(cmul(buf[t], to_c<C>(cconj(chirp(TN, t, N)))), invM);
        }
        __syncthreads();
    }
    // unfold: Y_q from the half-length transform, then G_m for m = 0..lmax
    C *Gk = Gout + (long long)r * fstride + (long long)k * ld;
    for (int m = tid; m <= lmax; m += NT) {
        const int q = m % N;
        const int kq = q % n;
        const int kc = kq == 0 ? 0 : n - kq;
        const double2 A = to_d(buf[kq]), B = cconj(to_d(buf[kc]));
        const double2 E = cscale(cadd(A, B), 0.5);
        const double2 D = csub(A, B);
        const double2 O = make_double2(0.5 * D.y, -0.5 * D.x);     // (A - B) / (2i)
        const double2 t = cmul(cconj(TN[2 * kq]), O);
        const double2 Y = (q < n) ? cadd(E, t) : csub(E, t);
        const double2 V = cmul(TN[(m * p) % (2 * N)], cconj(Y));
        const double w = (m == 0) ? 1.0 : kSqrt2;
        Gk[m] = to_c<C>(make_double2(w * V.x, w * V.y));
    }
}

template <int MODE, int NT, typename C>
static int launch_group(const mlcr_geom *g, const RingGroup &grp, int lmax, int nrhs,
                        const C *F, C *G, const double *map_in, double *map_out,
                        const double *ninv, long long fstride, const C *Bf, const C *W,
                        hipStream_t s) {
    // FFT buffer, then (groups with short rings, synthesis direction) the
    // cooperative fold's coefficients and partial sums
    const size_t hoff = ((size_t)grp.mmax * sizeof(C) + 15) / 16 * 16;
    const bool fold = MODE != 1 && grp.nmin <= kFoldMax;
    const size_t lds = fold ? hoff + (size_t)(kFoldMax + std::max(NT, kFoldMax)) * sizeof(double2)
                            : (size_t)grp.mmax * sizeof(C);
    int rc = ensure_dynamic_lds((const void *)k_ring<MODE, NT, C>, lds);
    if (rc) return rc;
    const long long nblk = 8LL * ((grp.count + 7) / 8) * nrhs;
    hipLaunchKernelGGL((k_ring<MODE, NT, C>), dim3((unsigned)nblk), dim3(NT), lds, s, F, G, map_in,
                       map_out, ninv, g->rings.as<RingInfo>(), g->lens.as<LenInfo>(),
                       g->order.as<int>(), g->T.as<double2>(), Bf, W, g->Wmax, lmax, fstride,
                       g->npix, grp.off, grp.count, nrhs, (int)hoff);
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

// Groups with FFT size above 4096 use big_nt threads (1024 by default: one
// butterfly per thread and radix-8 pass, so a CU holding one 128 KiB float64
// workgroup still runs 16 waves); the others use 512.
template <int MODE, typename C>
static int launch_ring_t(const mlcr_geom *g, int lmax, int nrhs, const C *F, C *G,
                         const double *map_in, double *map_out, const double *ninv, const C *Bf,
                         const C *W, int big_nt, hipStream_t s) {
    const long long fstride = (long long)g->nrings * (lmax + 1);
    for (const RingGroup &grp : g->ring_groups) {
        const int rc = grp.mmax > 4096 && big_nt == 1024
                           ? launch_group<MODE, 1024>(g, grp, lmax, nrhs, F, G, map_in, map_out,
                                                      ninv, fstride, Bf, W, s)
                           : launch_group<MODE, kRingThreads>(g, grp, lmax, nrhs, F, G, map_in,
                                                              map_out, ninv, fstride, Bf, W, s);
        if (rc) return rc;
    }
    return MLCR_OK;
}

// F and G hold complex float64 on the float64 path, complex float32 on the
// mixed paths (the ring FFTs there run in float32)
template <int MODE>
static int launch_ring(const mlcr_geom *g, int lmax, int nrhs, const void *F, void *G,
                       const double *map_in, double *map_out, const double *ninv, int prec,
                       hipStream_t s) {
    const int big_nt = g->tune[prec].ring_threads;
    if (prec != MLCR_FP64)
        return launch_ring_t<MODE>(g, lmax, nrhs, static_cast<const float2 *>(F),
                                   static_cast<float2 *>(G), map_in, map_out, ninv,
                                   g->Bf32.as<float2>(), g->W32.as<float2>(), big_nt, s);
    return launch_ring_t<MODE>(g, lmax, nrhs, static_cast<const double2 *>(F),
                               static_cast<double2 *>(G), map_in, map_out, ninv,
                               g->Bf.as<double2>(), g->W.as<double2>(), big_nt, s);
}

int launch_ring_synth(const mlcr_geom *g, int lmax, int nrhs, const void *F, double *map,
                      int prec, hipStream_t s) {
    return launch_ring<0>(g, lmax, nrhs, F, nullptr, nullptr, map, nullptr, prec, s);
}
int launch_ring_adjoint(const mlcr_geom *g, int lmax, int nrhs, const double *map, void *G,
                        int prec, hipStream_t s) {
    return launch_ring<1>(g, lmax, nrhs, nullptr, G, map, nullptr, nullptr, prec, s);
}
// one workgroup per ring
__global__ __launch_bounds__(256) void k_ring_weight(const double *__restrict__ in,
                                                     double *__restrict__ out,
                                                     const RingInfo *__restrict__ rings,
                                                     const double *__restrict__ w) {
    const RingInfo ri = rings[blockIdx.x];
    const double wk = w[blockIdx.x];
    for (int j = threadIdx.x; j < ri.nphi; j += blockDim.x) out[ri.start + j] = wk * in[ri.start + j];
}

int launch_ring_weight(const mlcr_geom *g, const double *in, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_ring_weight, dim3(g->nrings), dim3(256), 0, s, in, out,
                       g->rings.as<RingInfo>(), g->ring_w.as<double>());
    MLCR_HIP_CHECK(hipGetLastError());
    return MLCR_OK;
}

int launch_ring_apply(const mlcr_geom *g, int lmax, int nrhs, void *FG, const double *ninv,
                      int prec, hipStream_t s) {
    return launch_ring<2>(g, lmax, nrhs, FG, FG, nullptr, nullptr, ninv, prec, s);
}

}  // namespace mlcr
