// Host-side tables of a geometry: HEALPix RING rings, per-length FFT tables
// and the coefficients of the normalized associated-Legendre recurrence.
// All values are formed in long double and rounded once to double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "mlcr_internal.h"

namespace mlcr {

using cld = std::complex<long double>;
static const long double kPi = 3.141592653589793238462643383279502884L;

static int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}
static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// In-place iterative radix-2 forward DFT, X_k = sum_j x_j e^{-2 pi i jk/M}.
static void fft_ld(std::vector<cld> &x) {
    const int M = (int)x.size();
    for (int i = 1, j = 0; i < M; i++) {
        int bit = M >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    for (int len = 2; len <= M; len <<= 1) {
        const int h = len / 2;
        std::vector<cld> w(h);
        for (int k = 0; k < h; k++) {
            long double a = -2.0L * kPi * (long double)k / (long double)len;
            w[k] = cld(cosl(a), sinl(a));
        }
        for (int i = 0; i < M; i += len)
            for (int k = 0; k < h; k++) {
                cld u = x[i + k], v = x[i + k + h] * w[k];
                x[i + k] = u + v;
                x[i + k + h] = u - v;
            }
    }
}

// Tables shared by every ring layout: per length class N = 4 i the twiddles
// T_N and Bluestein filters, the power-of-two twiddles W, the recurrence
// coefficients, the ring launch groups; then the upload.  ri[k].tab indexes
// classes (the ring counts N = 4 i of the layout's length classes).
static int finish_geometry(mlcr_geom *g, int lmax, const std::vector<double> &z,
                           const std::vector<double> &s, std::vector<RingInfo> &ri,
                           const std::vector<int> &classes);

int build_geometry(mlcr_geom *g, int nside, int lmax) {
    g->kind = 0;
    g->nside = nside;
    g->lmax = lmax;
    g->nrings = 4 * nside - 1;
    g->npairs = 2 * nside;
    g->npix = 12LL * nside * nside;
    const int nr = g->nrings;
    // ---- rings (Sec. 2.1; Gorski et al. 2005) ----
    std::vector<double> z(nr), s(nr);
    std::vector<RingInfo> ri(nr);
    long long start = 0;
    for (int i = 1; i <= nr; i++) {
        RingInfo &r = ri[i - 1];
        long double zabs, one_minus;
        int cls;
        if (i < nside || i > 3 * nside) {
            int ii = (i < nside) ? i : 4 * nside - i;
            one_minus = (long double)ii * ii / (3.0L * nside * nside);
            zabs = 1.0L - one_minus;
            r.nphi = 4 * ii;
            r.phase = 1;                       // phi0 = pi / (4 ii) = pi / N
            cls = ii;
        } else {
            long double zz = (long double)(4 * nside - 2 * i) / (3.0L * nside);
            zabs = fabsl(zz);
            one_minus = 1.0L - zabs;
            r.nphi = 4 * nside;
            // phi0 = pi / (4 nside) when i - nside is even, 0 when odd (base
            // pixel 4 of the HEALPix numbering is centred on phi = 0)
            r.phase = ((i - nside) % 2 == 0) ? 1 : 0;
            cls = nside;
        }
        z[i - 1] = (double)((i > 2 * nside) ? -zabs : zabs);
        s[i - 1] = (double)sqrtl(one_minus * (1.0L + zabs));
        r.start = start;
        r.tab = cls - 1;
        r.pad = 0;
        start += r.nphi;
    }

    std::vector<int> classes(nside);
    for (int i = 1; i <= nside; i++) classes[i - 1] = i;
    g->ring_w_host.assign(nr, 4.0 * (double)kPi / (double)g->npix);   // equal-area pixels
    return finish_geometry(g, lmax, z, s, ri, classes);
}

// Gauss-Legendre rings: nrings nodes z_k of P_nrings (north to south), nphi
// equispaced pixels per ring starting at phi = 0.  The quadrature
// sum_k sum_j W_k f(theta_k, phi_j), W_k = w_k 2 pi / nphi with w_k the
// Gauss-Legendre weights, integrates f exactly when f is a polynomial of
// degree < 2 nrings in cos theta and holds frequencies |m| < nphi in phi.
int build_geometry_gl(mlcr_geom *g, int lmax, int nrings, int nphi) {
    g->kind = 1;
    g->nside = 0;
    g->lmax = lmax;
    g->nrings = nrings;
    g->npairs = (nrings + 1) / 2;
    g->npix = (long long)nrings * nphi;
    const int nr = nrings;
    std::vector<long double> zl(nr), wl(nr);
    // Newton on P_n from the usual cosine guesses; the south half mirrors the north
    auto node = [&](int k) {
        long double x = cosl(kPi * ((long double)k + 0.75L) / ((long double)nr + 0.5L));
        long double dp = 1.0L;
        for (int it = 0; it < 100; it++) {
            long double p0 = 1.0L, p1 = x;
            for (int j = 2; j <= nr; j++) {
                const long double p2 = ((2.0L * j - 1.0L) * x * p1 - (j - 1.0L) * p0) / (long double)j;
                p0 = p1;
                p1 = p2;
            }
            if (nr == 1) { p1 = x; p0 = 1.0L; }
            dp = (long double)nr * (x * p1 - p0) / (x * x - 1.0L);
            const long double dx = p1 / dp;
            x -= dx;
            if (fabsl(dx) < 1e-19L * std::max(1.0L, fabsl(x))) break;
        }
        zl[k] = x;
        wl[k] = 2.0L / ((1.0L - x * x) * dp * dp);
    };
    {
        const int half = (nr + 1) / 2;
        unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; t++)
            th.emplace_back([&, t] {
                for (int k = (int)t; k < half; k += (int)nt) node(k);
            });
        for (auto &t : th) t.join();
        for (int k = 0; k < half; k++) {
            zl[nr - 1 - k] = -zl[k];
            wl[nr - 1 - k] = wl[k];
        }
        if (nr & 1) zl[nr / 2] = 0.0L;
    }
    std::vector<double> z(nr), s(nr);
    std::vector<RingInfo> ri(nr);
    g->ring_w_host.resize(nr);
    for (int k = 0; k < nr; k++) {
        z[k] = (double)zl[k];
        s[k] = (double)sqrtl((1.0L - zl[k]) * (1.0L + zl[k]));
        RingInfo &r = ri[k];
        r.start = (long long)k * nphi;
        r.nphi = nphi;
        r.phase = 0;            // phi0 = 0
        r.tab = 0;
        r.pad = 0;
        g->ring_w_host[k] = (double)(wl[k] * 2.0L * kPi / (long double)nphi);
    }
    return finish_geometry(g, lmax, z, s, ri, std::vector<int>{nphi / 4});
}

static int finish_geometry(mlcr_geom *g, int lmax, const std::vector<double> &z,
                           const std::vector<double> &s, std::vector<RingInfo> &ri,
                           const std::vector<int> &classes) {
    const int nr = g->nrings;
    const int ncls = (int)classes.size();
    // ---- length classes N = 4 i: twiddles T_N and Bluestein filters ----
    std::vector<LenInfo> li(ncls);
    long long toff = 0, boff = 0;
    int maxfft = 1;
    for (int c = 0; c < ncls; c++) {
        LenInfo &L = li[c];
        const int N = 4 * classes[c], n = N / 2;
        L.toff = toff;
        toff += 2LL * N;
        if (is_pow2(n)) {
            L.boff = -1;
            L.M = n;
        } else {
            L.M = next_pow2(2 * n - 1);
            L.boff = boff;
            boff += L.M;
        }
        L.pad = 0;
        maxfft = std::max(maxfft, L.M);
    }
    g->lds_cplx = maxfft;
    g->Wmax = maxfft;

    std::vector<double2> T(toff), Bf(std::max<long long>(boff, 1)), W(maxfft);
    auto fill_class = [&](int c) {
        const int N = 4 * classes[c], n = N / 2;
        const LenInfo &L = li[c];
        for (int j = 0; j < 2 * N; j++) {
            long double a = kPi * (long double)j / (long double)N;
            T[L.toff + j] = make_double2((double)cosl(a), (double)sinl(a));
        }
        if (L.boff >= 0) {
            // b_j = e^{-i pi j^2 / n} for |j| < n, wrapped cyclically into length M
            std::vector<cld> b(L.M, cld(0, 0));
            for (int j = 0; j < n; j++) {
                long long r2 = ((long long)j * j) % (2LL * n);
                long double a = -kPi * (long double)r2 / (long double)n;
                cld v(cosl(a), sinl(a));
                b[j] = v;
                if (j > 0) b[L.M - j] = v;
            }
            fft_ld(b);
            for (int k = 0; k < L.M; k++)
                Bf[L.boff + k] = make_double2((double)b[k].real(), (double)b[k].imag());
        }
    };
    {
        unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; t++)
            th.emplace_back([&, t] {
                for (int c = (int)t; c < ncls; c += (int)nt) fill_class(c);
            });
        for (auto &t : th) t.join();
    }
    for (int j = 0; j < maxfft; j++) {
        long double a = -2.0L * kPi * (long double)j / (long double)maxfft;
        W[j] = make_double2((double)cosl(a), (double)sinl(a));
    }

    // ---- Legendre recurrence (Sec. 3.2 normalization) ----
    // lambda_lm = A_lm z lambda_{l-1,m} - B_lm lambda_{l-2,m}, l >= m+1, with
    // A_lm = sqrt((4 l^2 - 1) / (l^2 - m^2)), B_lm = A_lm / A_{l-1,m}, B_{m+1,m} = 0.
    // The matrix-core kernels run the same recurrence on mu_lm = lambda_lm / c_lm,
    // c_mm = c_{m+1,m} = 1, c_lm = B_lm c_{l-2,m}, which has the two-operation form
    //     mu_lm = alpha_lm z mu_{l-1,m} - mu_{l-2,m},  alpha_lm = A_lm c_{l-1,m} / c_lm;
    // c is folded into their inputs and outputs (0.11 <= c <= 1.13, 1.5 <= alpha <= 182 for lmax <= 16384).
    const long long nab = (long long)lmax * (lmax + 1) / 2;
    const long long ntri = (long long)(lmax + 1) * (lmax + 2) / 2;
    std::vector<double2> ab(std::max<long long>(nab, 1));
    std::vector<double> alpha(std::max<long long>(nab, 1)), cfac(ntri);
    std::vector<long long> aboff(lmax + 1);
    std::vector<double> seed(lmax + 1);
    long double prod = 1.0L;     // prod_{k=1..m} (2k-1)/(2k)
    for (int m = 0; m <= lmax; m++) {
        if (m > 0) prod *= (long double)(2 * m - 1) / (long double)(2 * m);
        long double c = sqrtl((2.0L * m + 1.0L) / (4.0L * kPi) * prod);
        seed[m] = (double)((m & 1) ? -c : c);
        aboff[m] = (long long)m * lmax - (long long)m * (m - 1) / 2;
    }
    {
        auto fill_m = [&](int m) {
            long double aprev = 0.0L;
            long double c2 = 1.0L, c1 = 1.0L;          // c_{l-2}, c_{l-1}
            const long long to = (long long)m * (lmax + 1) - (long long)m * (m - 1) / 2;
            cfac[to] = 1.0;
            for (int l = m + 1; l <= lmax; l++) {
                long double a = sqrtl((4.0L * l * l - 1.0L) / ((long double)(l - m) * (l + m)));
                long double b = (l == m + 1) ? 0.0L : a / aprev;
                ab[aboff[m] + (l - m - 1)] = make_double2((double)a, (double)b);
                const long double c = (l == m + 1) ? 1.0L : b * c2;
                alpha[aboff[m] + (l - m - 1)] = (double)(a * c1 / c);
                cfac[to + (l - m)] = (double)c;
                c2 = c1;
                c1 = c;
                aprev = a;
            }
        };
        unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; t++)
            th.emplace_back([&, t] {
                for (int m = (int)t; m <= lmax; m += (int)nt) fill_m(m);
            });
        for (auto &t : th) t.join();
    }

    // ---- ring order for the FFT kernels: grouped by LDS need (FFT size M),
    // each group launched with its own LDS size; most expensive first ----
    std::vector<int> order(nr);
    {
        std::vector<double> cost(nr);
        for (int k = 0; k < nr; k++) {
            const LenInfo &L = li[ri[k].tab];
            const double M = (double)L.M;
            cost[k] = (L.boff >= 0 ? 3.0 : 1.0) * M * std::log2(std::max(2.0, M));
            order[k] = k;
        }
        auto bucket = [&](int k) {
            const int M = li[ri[k].tab].M;
            return M <= 1024 ? 0 : (M <= 2048 ? 1 : (M <= 4096 ? 2 : 3));
        };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            if (bucket(a) != bucket(b)) return bucket(a) > bucket(b);
            return cost[a] > cost[b];
        });
        g->ring_groups.clear();
        for (int j = 0; j < nr;) {
            const int b = bucket(order[j]);
            RingGroup grp{j, 0, 0, 1 << 30};
            while (j < nr && bucket(order[j]) == b) {
                grp.mmax = std::max(grp.mmax, li[ri[order[j]].tab].M);
                grp.nmin = std::min(grp.nmin, ri[order[j]].nphi);
                grp.count++;
                j++;
            }
            g->ring_groups.push_back(grp);
        }
    }

    // ---- upload ----
    auto up = [](DevBuf &b, const void *src, size_t bytes) -> int {
        if (b.reserve(bytes)) return fail(MLCR_ENOMEM, "geometry table allocation failed");
        MLCR_HIP_CHECK(hipMemcpy(b.ptr, src, bytes, hipMemcpyHostToDevice));
        return MLCR_OK;
    };
    int rc;
    if ((rc = up(g->ring_z, z.data(), nr * sizeof(double)))) return rc;
    if ((rc = up(g->ring_s, s.data(), nr * sizeof(double)))) return rc;
    if ((rc = up(g->ring_w, g->ring_w_host.data(), nr * sizeof(double)))) return rc;
    if ((rc = up(g->rings, ri.data(), nr * sizeof(RingInfo)))) return rc;
    if ((rc = up(g->lens, li.data(), ncls * sizeof(LenInfo)))) return rc;
    if ((rc = up(g->order, order.data(), nr * sizeof(int)))) return rc;
    if ((rc = up(g->T, T.data(), T.size() * sizeof(double2)))) return rc;
    if ((rc = up(g->Bf, Bf.data(), Bf.size() * sizeof(double2)))) return rc;
    if ((rc = up(g->W, W.data(), W.size() * sizeof(double2)))) return rc;
    {
        // float32 copies for the mixed-precision operator step's FFTs
        std::vector<float2> Bf32(Bf.size()), W32(W.size());
        for (size_t i = 0; i < Bf.size(); i++) Bf32[i] = make_float2((float)Bf[i].x, (float)Bf[i].y);
        for (size_t i = 0; i < W.size(); i++) W32[i] = make_float2((float)W[i].x, (float)W[i].y);
        if ((rc = up(g->Bf32, Bf32.data(), Bf32.size() * sizeof(float2)))) return rc;
        if ((rc = up(g->W32, W32.data(), W32.size() * sizeof(float2)))) return rc;
    }
    if ((rc = up(g->ab, ab.data(), ab.size() * sizeof(double2)))) return rc;
    if ((rc = up(g->alpha, alpha.data(), alpha.size() * sizeof(double)))) return rc;
    if ((rc = up(g->cfac, cfac.data(), cfac.size() * sizeof(double)))) return rc;
    if ((rc = up(g->aboff, aboff.data(), aboff.size() * sizeof(long long)))) return rc;
    if ((rc = up(g->seed, seed.data(), seed.size() * sizeof(double)))) return rc;
    std::vector<double> zeros(lmax + 1, 0.0);
    if ((rc = up(g->zeros, zeros.data(), zeros.size() * sizeof(double)))) return rc;
    return MLCR_OK;
}

}  // namespace mlcr
