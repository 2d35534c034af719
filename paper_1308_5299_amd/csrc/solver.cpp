// Multi-level CR solver (Sec. 3.2, Fig. code:mg) on top of the operator
// kernels: level ladder, smoother construction, the recursive CR-Cycle and
// the float64 outer CR-Solve loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "solver_internal.h"

namespace mlcr {

// ---------------------------------------------------------------------------
// HEALPix NESTED -> RING (Gorski et al. 2005): a nested index holds the base
// face and the bit-interleaved (x, y) position inside it; ring number and
// position in the ring follow from the face's row/column offsets.
// ---------------------------------------------------------------------------
long long nest2ring(int nside, long long ipnest) {
    static const int jrll[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
    static const int jpll[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};
    const long long npface = (long long)nside * nside;
    const int face = (int)(ipnest / npface);
    long long ipf = ipnest % npface;
    long long ix = 0, iy = 0;
    for (int b = 0; ipf; b++) {
        ix |= (ipf & 1LL) << b;
        ipf >>= 1;
        iy |= (ipf & 1LL) << b;
        ipf >>= 1;
    }
    const long long jr = (long long)jrll[face] * nside - ix - iy - 1;
    const long long npix = 12 * npface;
    long long nr, n_before;
    int kshift;
    if (jr < nside) {
        nr = jr;
        n_before = 2 * nr * (nr - 1);
        kshift = 0;
    } else if (jr > 3LL * nside) {
        nr = 4LL * nside - jr;
        n_before = npix - 2 * (nr + 1) * nr;
        kshift = 0;
    } else {
        nr = nside;
        n_before = 2LL * nside * (nside - 1) + (jr - nside) * 4LL * nside;
        kshift = (int)((jr - nside) & 1);
    }
    long long jp = (jpll[face] * nr + ix - iy + 1 + kshift) / 2;
    if (jp > 4 * nr) jp -= 4 * nr;
    if (jp < 1) jp += 4 * nr;
    return n_before + jp - 1;
}

// ---------------------------------------------------------------------------
// ladder (Sec. 3.2 level structure; Sec. 3.3 filters; Sec. 3.4 band limits)
// ---------------------------------------------------------------------------
static constexpr int kDenseL = 40;     // bottom level: dense solve for l <= 40 (Sec. 3.2)
static constexpr int kTile = kTileK;
static constexpr int kMaxNb = 12;       // neighbour tiles per tile (8 in a regular patch)
static const double kPi = 3.14159265358979323846;

struct Plan {
    int H = 0;
    int nside[8] = {0}, lmax[8] = {0}, nrec[8] = {0};
    int nrec_top = 1;
    int lmax_b = 0;
    std::vector<double> fl[8];
    std::vector<double> highpass;
    double omega = 1.0, omega_top = 1.0;
    bool gl = true;         // coarse levels on Gauss-Legendre grids when cheaper
    int smoother = 0;       // 0: probed blocks + block SGS; 1: addition theorem + block ICC(0)
    double ridge_min = 1e-4;  // smallest ridge alpha of the ICC(0) smoother
    double ridge_max = 1.0;   // largest ridge alpha the ICC(0) search may use
    bool keep = false;      // keep the assembled smoother blocks (mlcr_solver_level_blocks)
};

// q_l = exp(-l^2 (l+1)^2 lambda) with q_{lstar} = 0.1 (eq. fourth-power-beam)
static std::vector<double> qfilter(int lmax, int lstar) {
    std::vector<double> f(lmax + 1);
    const double ls = (double)lstar;
    const double lam = std::log(10.0) / (ls * ls * (ls + 1) * (ls + 1));
    for (int l = 0; l <= lmax; l++) {
        const double t = (double)l * l * (l + 1.0) * (l + 1.0) * lam;
        f[l] = std::exp(-t);
    }
    return f;
}

// Gaussian of FWHM two pixels of the level's grid (Sec. 3.3; p_l = 1)
static std::vector<double> gauss2px(int lmax, int nside) {
    std::vector<double> f(lmax + 1);
    const double pix = std::sqrt(4.0 * kPi / (12.0 * nside * nside));
    const double sig = 2.0 * pix / std::sqrt(8.0 * std::log(2.0));
    for (int l = 0; l <= lmax; l++) f[l] = std::exp(-0.5 * l * (l + 1.0) * sig * sig);
    return f;
}

static void default_plan(int nside_obs, int lmax, Plan &p) {
    p = Plan();
    if (lmax <= kDenseL) {
        p.H = 0;
        p.lmax_b = lmax;
        return;
    }
    int ns = nside_obs / 2, lprev = lmax;
    while (ns >= 32 && p.H < 8 && ns % kTile == 0) {
        // band limits (Sec. 3.3): the finest level keeps the full band; 4 N_side
        // suffices on a q_l-filtered level (N_side >= 512), the coarser,
        // high signal-to-noise Gaussian levels need 6 N_side against ringing
        int lh;
        if (p.H == 0) lh = lmax;
        else if (ns >= 512) lh = std::min(lprev, 4 * ns);
        else lh = std::min(lprev, 6 * ns);
        if (lh <= kDenseL) break;
        p.nside[p.H] = ns;
        p.lmax[p.H] = lh;
        p.nrec[p.H] = 2;
        p.H++;
        lprev = lh;
        ns /= 2;
    }
    if (p.H == 0) {
        p.lmax_b = lmax;
        return;
    }
    p.nrec[p.H - 1] = 1;          // the dense bottom solve is exact: one visit
    p.nrec_top = 1;               // finest level runs once down, once up
    // q_l filters on the fine, lower signal-to-noise levels (the paper's N_side
    // 1024 and 512 levels); Gaussians of FWHM two pixels on levels of
    // N_side <= 256, where the q_l ringing would make couplings non-local.
    for (int h = 0; h < p.H; h++) {
        if (h == 0 && p.nside[h] >= 512)
            p.fl[h] = qfilter(p.lmax[h], (int)std::lround(p.lmax[h] * 2570.0 / 3000.0));
        else if (h == 1 && p.nside[h] >= 512)
            p.fl[h] = qfilter(p.lmax[h], (int)std::lround(p.lmax[h] * 1536.0 / 2048.0));
        else
            p.fl[h] = gauss2px(p.lmax[h], p.nside[h]);
    }
    p.lmax_b = std::min(kDenseL, p.lmax[p.H - 1]);
    p.highpass.resize(lmax + 1);
    for (int l = 0; l <= lmax; l++) p.highpass[l] = 1.0 - (l <= p.lmax[0] ? p.fl[0][l] : 0.0);
}

// ---------------------------------------------------------------------------
// ladder from a caller's descriptor
// ---------------------------------------------------------------------------
static constexpr int kMaxDenseL = 64;   // largest dense bottom band limit

static int check_ladder(int nside_obs, int lmax, const mlcr_ladder_desc *d) {
    if (!d) return fail(MLCR_EINVAL, "ladder is NULL");
    const int H = d->nlevels;
    if (H < 0 || H > 8) return fail(MLCR_EINVAL, "ladder: nlevels must be in [0, 8]");
    if (d->nrec_top < 1 || d->nrec_top > 3) return fail(MLCR_EINVAL, "ladder: nrec_top must be in [1, 3]");
    if (d->gl_levels != 0 && d->gl_levels != 1) return fail(MLCR_EINVAL, "ladder: gl_levels must be 0 or 1");
    if (d->smoother != 0 && d->smoother != 1) return fail(MLCR_EINVAL, "ladder: smoother must be 0 or 1");
    if (d->keep_blocks != 0 && d->keep_blocks != 1)
        return fail(MLCR_EINVAL, "ladder: keep_blocks must be 0 or 1");
    if (!(d->ridge_max >= 0.0) || !std::isfinite(d->ridge_max))
        return fail(MLCR_EINVAL, "ladder: ridge_max must be finite and >= 0");
    if (!(d->ridge_min >= 0.0) || !(d->ridge_min <= d->ridge_max))
        return fail(MLCR_EINVAL, "ladder: ridge_min must be in [0, ridge_max]");
    if (H == 0) {
        if (d->lmax_dense != lmax || lmax > kMaxDenseL)
            return fail(MLCR_EINVAL, "ladder: without pixel levels the dense solve must cover the "
                                     "operator's lmax (<= 64)");
        return MLCR_OK;
    }
    for (int h = 0; h < H; h++) {
        const std::string lv = "ladder level " + std::to_string(h) + ": ";
        if (d->nside[h] < kTile || d->nside[h] > 2048 || d->nside[h] % kTile)
            return fail(MLCR_EINVAL, lv + "nside must be a multiple of 8 in [8, 2048]");
        const int up = h == 0 ? lmax : d->lmax[h - 1];
        if (d->lmax[h] < 1 || d->lmax[h] > up)
            return fail(MLCR_EINVAL, lv + "lmax must be in [1, " + std::to_string(up) + "]");
        if (d->nrec[h] < 1 || d->nrec[h] > 3) return fail(MLCR_EINVAL, lv + "nrec must be in [1, 3]");
        if (d->smoother == 1 && (nside_obs % d->nside[h] || ((nside_obs / d->nside[h]) &
                                                              (nside_obs / d->nside[h] - 1))))
            return fail(MLCR_EINVAL, lv + "the addition-theorem smoother needs N_side_obs / "
                                          "N_side^h a power of two");
        if (!d->filter[h]) return fail(MLCR_EINVAL, lv + "filter is NULL");
        const int lnext = h + 1 < H ? d->lmax[h + 1] : d->lmax_dense;
        for (int l = 0; l <= d->lmax[h]; l++) {
            const double f = d->filter[h][l];
            if (!std::isfinite(f)) return fail(MLCR_EINVAL, lv + "filter must be finite");
            if (l <= lnext && !(f > 0.0))
                return fail(MLCR_EINVAL, lv + "filter must be > 0 up to the next level's lmax (l = " +
                                             std::to_string(l) + ")");
        }
    }
    if (d->lmax_dense < 0 || d->lmax_dense > d->lmax[H - 1] || d->lmax_dense > kMaxDenseL)
        return fail(MLCR_EINVAL, "ladder: lmax_dense must be in [0, min(lmax[H-1], 64)]");
    if (d->highpass)
        for (int l = 0; l <= lmax; l++)
            if (!std::isfinite(d->highpass[l])) return fail(MLCR_EINVAL, "ladder: highpass must be finite");
    return MLCR_OK;
}

static void plan_from_desc(int lmax, const mlcr_ladder_desc *d, Plan &p) {
    p = Plan();
    p.H = d->nlevels;
    p.nrec_top = d->nrec_top;
    p.gl = d->gl_levels != 0;
    p.smoother = d->smoother;
    p.ridge_min = d->ridge_min;
    p.ridge_max = d->ridge_max;
    p.keep = d->keep_blocks != 0;
    if (p.H == 0) {
        p.lmax_b = lmax;
        return;
    }
    for (int h = 0; h < p.H; h++) {
        p.nside[h] = d->nside[h];
        p.lmax[h] = d->lmax[h];
        p.nrec[h] = d->nrec[h];
        p.fl[h].assign(d->filter[h], d->filter[h] + d->lmax[h] + 1);
    }
    p.lmax_b = d->lmax_dense;
    p.highpass.resize(lmax + 1);
    for (int l = 0; l <= lmax; l++)
        p.highpass[l] = d->highpass ? d->highpass[l] : 1.0 - (l <= p.lmax[0] ? p.fl[0][l] : 0.0);
}

static void desc_from_plan(const Plan &p, int lmax, mlcr_ladder_desc *d, double *buf) {
    std::memset(d, 0, sizeof(*d));
    d->nlevels = p.H;
    d->nrec_top = p.nrec_top;
    d->lmax_dense = p.lmax_b;
    d->gl_levels = p.gl ? 1 : 0;
    d->smoother = p.smoother;
    d->ridge_min = p.ridge_min;
    d->ridge_max = p.ridge_max;
    d->keep_blocks = p.keep ? 1 : 0;
    for (int h = 0; h < p.H; h++) {
        d->nside[h] = p.nside[h];
        d->lmax[h] = p.lmax[h];
        d->nrec[h] = p.nrec[h];
        double *f = buf + (size_t)h * (lmax + 1);
        std::copy(p.fl[h].begin(), p.fl[h].end(), f);
        d->filter[h] = f;
    }
    d->highpass = nullptr;
}

// ---------------------------------------------------------------------------
// One multi-level cycle (Fig. code:mg) as a flat schedule of steps.
// Levels: 0 = top spherical-harmonic level (diagonal smoother), 1..H pixel
// levels, B = H + 1 the dense bottom (0 when there is no pixel level).
// A level entered from above is smoothed, its residual restricted, and the
// next coarser level entered n_rec times (from a zero correction) before the
// correction is interpolated back and the level smoothed again.  The
// schedule unrolls that into a step list with an explicit stack of the
// levels that still owe visits to the level below them; the same list
// drives the GPU cycle, the operation counts and the per-level profile.
// ---------------------------------------------------------------------------
enum StepKind { kStepSmooth = 0, kStepDown = 1, kStepUp = 2, kStepBottom = 3 };
struct Step {
    int kind, h;
    bool xzero;     // kStepSmooth: the level's iterate is still zero (r = b)
    bool enter;     // first step of a visit of level h
};

static void build_schedule(int B, const std::vector<int> &nrec, std::vector<Step> &out) {
    out.clear();
    struct Owed {
        int h, left;
    };
    std::vector<Owed> stack;
    auto enter = [&](int h, bool xzero) {
        if (h == B) {
            out.push_back({kStepBottom, h, true, true});
            return;
        }
        out.push_back({kStepSmooth, h, xzero, true});
        out.push_back({kStepDown, h, false, false});
        stack.push_back({h, nrec[h]});
    };
    enter(0, true);
    while (!stack.empty()) {
        const int h = stack.back().h, left = stack.back().left;
        if (left > 0) {
            stack.back().left = left - 1;
            enter(h + 1, left == nrec[h]);      // the coarse correction starts at zero
        } else {
            stack.pop_back();
            out.push_back({kStepUp, h, false, false});
            out.push_back({kStepSmooth, h, false, false});
        }
    }
}

struct CycleOps {
    virtual ~CycleOps() {}
    virtual int residual(int h, bool xzero) = 0;   // r_h = b_h - A_h x_h
    virtual int smooth(int h) = 0;                 // x_h += M_h r_h
    virtual int restrict_down(int h) = 0;          // b_{h+1} = I r_h, x_{h+1} = 0
    virtual int prolong_up(int h) = 0;             // x_h += I^T x_{h+1}
    virtual int bottom(int h) = 0;                 // x_h = A_h^-1 b_h
    virtual void visit(int h) = 0;
};

static int run_schedule(CycleOps &o, const std::vector<Step> &sch) {
    int rc = MLCR_OK;
    for (const Step &st : sch) {
        if (st.enter) o.visit(st.h);
        switch (st.kind) {
        case kStepSmooth:
            if (!(rc = o.residual(st.h, st.xzero))) rc = o.smooth(st.h);
            break;
        case kStepDown:
            if (!(rc = o.residual(st.h, false))) rc = o.restrict_down(st.h);
            break;
        case kStepUp: rc = o.prolong_up(st.h); break;
        default: rc = o.bottom(st.h); break;
        }
        if (rc) return rc;
    }
    return MLCR_OK;
}

struct CountOps : CycleOps {
    // per level: visits, A_h applications, level-transfer SHTs (Y_h), smoother/bottom applications
    std::vector<long long> c;
    int B;
    explicit CountOps(int nl, int b) : c(4 * nl, 0), B(b) {}
    int residual(int h, bool xzero) override {
        if (!xzero) c[4 * h + 1]++;
        return 0;
    }
    int smooth(int h) override {
        c[4 * h + 3]++;
        if (h > 0) c[4 * h + 2] += 2;
        return 0;
    }
    int restrict_down(int) override { return 0; }
    int prolong_up(int) override { return 0; }
    int bottom(int h) override {
        c[4 * h + 3]++;
        return 0;
    }
    void visit(int h) override { c[4 * h]++; }
};

// Per-level profile: HIP event pairs around the steps of a cycle, added up
// per (level, kind of work) when the solve reads its residual norms.
struct Profile {
    bool on = false;
    std::vector<double> ms;             // [4 * levels]
    std::vector<long long> calls;
    struct Rec {
        int slot;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    void reset(int levels) {
        ms.assign(4 * levels, 0.0);
        calls.assign(4 * levels, 0);
    }
    void drain() {
        for (Rec &r : pending) {
            float t = 0.f;
            (void)hipEventSynchronize(r.b);
            (void)hipEventElapsedTime(&t, r.a, r.b);
            if (r.slot >= 0 && r.slot < (int)ms.size()) {
                ms[r.slot] += t;
                calls[r.slot]++;
            }
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        pending.clear();
    }
};

struct ProfScope {
    Profile *p;
    hipStream_t s;
    int slot;
    hipEvent_t a = nullptr;
    ProfScope(Profile *p_, hipStream_t s_, int level, int kind) : p(p_), s(s_), slot(4 * level + kind) {
        if (!p || !p->on) return;
        if (hipEventCreate(&a) != hipSuccess) {
            a = nullptr;
            return;
        }
        (void)hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return;
        }
        (void)hipEventRecord(b, s);
        p->pending.push_back({slot, a, b});
    }
};

}  // namespace mlcr

// ---------------------------------------------------------------------------
// solver object
// ---------------------------------------------------------------------------
using namespace mlcr;

struct PixLevel {
    int nside = 0, lmax = 0, opl = 0;
    mlcr_geom *geom = nullptr;
    int ntiles = 0, kk = kTile * kTile;
    // block-sparse smoother: neighbour lists (CSR), coupling blocks, inverse
    // diagonal blocks, sweep colours and the tiles of each colour
    int n_sweep = 0, n_probe = 0;
    std::vector<int> soff;              // host: offsets of the colours in stiles
    DevBuf wdown, act, one, tilepix, nbptr, nbs, off, scol, stiles, minv, ridge;
    int smoother = 0;                   // 0: block SGS; 1: block ICC(0) (off, minv hold L)
    int nslots = 0;
    DevBuf rev, adiag, aoff;            // reverse slots; assembled blocks (kept on request)
    DevBuf x, b, r, t, map, cmap;
};

struct mlcr_solver {
    mlcr_op *op = nullptr;
    int max_nrhs = 0;
    Plan plan;
    bool direct = false;
    std::vector<std::unique_ptr<PixLevel>> lev;       // pixel levels 1..H
    // top
    DevBuf top_wdown, top_dinv, top_hp, top_act, x0, b0, r0, t0;
    // bottom
    int lmax_b = 0, opl_b = 0, na = 0;
    DevBuf b_idx, b_inv, xb, bb;
    DevBuf b_A;                         // the assembled dense matrix (before factoring)
    DevBuf b_ws;                        // workspace of the dense bottom apply
    // outer loop
    DevBuf sinv, chalf, partial, norms, ro, to;
    // conjugate gradients: search direction, previous preconditioned residual,
    // per-RHS coefficients
    DevBuf pcg_p, pcg_zo, pcg_coef;
    std::vector<float> ridge_summary;
    std::vector<Step> sched;            // one cycle's steps (build_schedule)
    DevBuf vobs, oring;                 // observation pixel vectors and RING indices, NESTED order
    // the solver's own level operators A_h, index = level number (1..H
    // pixel levels, H + 1 the dense bottom; 0 unused: the top is the
    // operator's level 0), so solvers with different ladders can share op
    std::vector<std::unique_ptr<mlcr_level>> slev;
    Profile prof;
    int prior_version = 0;              // op->prior_version the norms were made for
    int mode = 0;
    int graph = 0;          // replay cycles 2.. of a solve from a captured graph
    long long graph_replays = 0, graph_fallbacks = 0;
    ~mlcr_solver() {
        for (auto &L : lev)
            if (L->geom) mlcr_geom_destroy(L->geom);
        for (auto &L : slev)
            if (L) release_level(*L);
    }
};

namespace mlcr {

static long long nalm_l(int lmax) { return (long long)(lmax + 1) * (lmax + 1); }

static int up(DevBuf &b, const void *src, size_t bytes) {
    if (b.reserve(bytes)) return fail(MLCR_ENOMEM, "solver allocation failed");
    MLCR_HIP_CHECK(hipMemcpy(b.ptr, src, bytes, hipMemcpyHostToDevice));
    return MLCR_OK;
}
static int alloc(DevBuf &b, size_t bytes) {
    if (b.reserve(bytes)) return fail(MLCR_ENOMEM, "solver allocation failed");
    return MLCR_OK;
}

// A_h of the solver's level opl (0: the operator's top level)
static int solver_apply(mlcr_solver *S, int opl, int nrhs, const double *x, double *y, int prec,
                        hipStream_t s) {
    if (opl == 0) return apply_level(S->op, 0, nrhs, x, y, prec, s);
    if (opl >= (int)S->slev.size() || !S->slev[opl]) return fail(MLCR_EINVAL, "solver level not built");
    return apply_level_on(S->op, *S->slev[opl], nrhs, x, y, prec, s);
}

struct GpuOps : CycleOps {
    mlcr_solver *S;
    int R, prec;
    hipStream_t s;
    GpuOps(mlcr_solver *s_, int r, int p, hipStream_t st) : S(s_), R(r), prec(p), s(st) {}
    int H() const { return S->plan.H; }
    void visit(int) override {}
    // profile slot kinds: A_h applications, level transforms, smoother, transfers
    Profile *P() { return S->prof.on ? &S->prof : nullptr; }
    int apply_h(int opl, int n, const double *x, double *y, int p) {
        return solver_apply(S, opl, n, x, y, p, s);
    }

    // buffers of level h
    double *X(int h) { return h == 0 ? S->x0.as<double>() : S->lev[h - 1]->x.as<double>(); }
    double *Bv(int h) { return h == 0 ? S->b0.as<double>() : S->lev[h - 1]->b.as<double>(); }
    double *Rv(int h) { return h == 0 ? S->r0.as<double>() : S->lev[h - 1]->r.as<double>(); }
    double *Tv(int h) { return h == 0 ? S->t0.as<double>() : S->lev[h - 1]->t.as<double>(); }
    int Lmax(int h) { return h == 0 ? S->op->lmax : S->lev[h - 1]->lmax; }
    int Opl(int h) { return h == 0 ? 0 : S->lev[h - 1]->opl; }
    const double *Act(int h) {
        return h == 0 ? S->top_act.as<double>() : S->lev[h - 1]->act.as<double>();
    }

    int residual(int h, bool xzero) override {
        int rc;
        if (xzero) {
            ProfScope ps(P(), s, h, 3);
            return launch_residual(Bv(h), nullptr, Rv(h), Act(h), Lmax(h), R, s);
        }
        ProfScope ps(P(), s, h, 0);
        if ((rc = apply_h(Opl(h), R, X(h), Tv(h), prec))) return rc;
        return launch_residual(Bv(h), Tv(h), Rv(h), Act(h), Lmax(h), R, s);
    }
    int smooth(int h) override {
        if (h == 0) {
            ProfScope ps(P(), s, 0, 2);
            return launch_axpy_l(X(0), Rv(0), S->top_hp.as<double>(), S->top_dinv.as<double>(),
                                 Lmax(0), R, s);
        }
        PixLevel &L = *S->lev[h - 1];
        int rc;
        // x_h += Y_h^T M_h Y_h r_h  (eqs. pixel-correction-1..3)
        {
            ProfScope ps(P(), s, h, 1);
            if ((rc = sht_synth(L.geom, L.lmax, R, L.r.as<double>(), L.map.as<double>(), prec, s)))
                return rc;
        }
        if ((rc = sweep(L, h))) return rc;
        {
            ProfScope ps(P(), s, h, 1);
            if ((rc = sht_adjoint(L.geom, L.lmax, R, L.cmap.as<double>(), L.t.as<double>(), prec, s)))
                return rc;
        }
        ProfScope ps(P(), s, h, 3);
        return launch_axpy_l(L.x.as<double>(), L.t.as<double>(), L.one.as<double>(), nullptr,
                             L.lmax, R, s);
    }
    // c = M r on the level's map: one multicolour block symmetric Gauss-Seidel
    // sweep over the tiles (Sec. 3.5 pattern)
    int sweep(PixLevel &L, int h) {
        int rc;
        ProfScope ps(P(), s, h, 2);
        if (L.smoother == 1) {
            // (L L^T)^-1: forward solve over the colours ascending, backward descending
            for (int pass = 0; pass < 2; pass++)
                for (int j = 0; j < L.n_sweep; j++) {
                    const int c = pass == 0 ? j : L.n_sweep - 1 - j;
                    if ((rc = launch_sgs_color(pass == 0 ? 0 : 2, L.map.as<double>(),
                                               L.cmap.as<double>(), L.geom->npix, R,
                                               L.tilepix.as<int>(), L.stiles.as<int>() + L.soff[c],
                                               L.soff[c + 1] - L.soff[c], L.nbptr.as<int>(),
                                               L.nbs.as<int>(), L.scol.as<int>(), c,
                                               L.off.as<float>(), L.minv.as<float>(), s)))
                        return rc;
                }
            return MLCR_OK;
        }
        for (int pass = 0; pass < 2; pass++)
            for (int j = 0; j < L.n_sweep; j++) {
                const int c = pass == 0 ? j : L.n_sweep - 1 - j;
                if (pass == 1 && c == L.n_sweep - 1) continue;     // no later neighbours
                if ((rc = launch_sgs_color(pass == 0 ? 0 : 1, L.map.as<double>(), L.cmap.as<double>(),
                                           L.geom->npix, R, L.tilepix.as<int>(),
                                           L.stiles.as<int>() + L.soff[c],
                                           L.soff[c + 1] - L.soff[c], L.nbptr.as<int>(),
                                           L.nbs.as<int>(), L.scol.as<int>(), c,
                                           L.off.as<float>(), L.minv.as<float>(), s)))
                    return rc;
            }
        return MLCR_OK;
    }
    int restrict_down(int h) override {
        ProfScope ps(P(), s, h, 3);
        const double *w = h == 0 ? S->top_wdown.as<double>() : S->lev[h - 1]->wdown.as<double>();
        int rc;
        if (h + 1 == H() + 1) {          // into the dense bottom level
            if ((rc = launch_transfer(Rv(h), Lmax(h), S->bb.as<double>(), S->lmax_b, w, S->lmax_b,
                                      false, R, s)))
                return rc;
            return MLCR_OK;
        }
        if ((rc = launch_transfer(Rv(h), Lmax(h), Bv(h + 1), Lmax(h + 1), w, Lmax(h + 1), false, R,
                                  s)))
            return rc;
        return launch_fill_zero(X(h + 1), (long long)R * nalm_l(Lmax(h + 1)), s);
    }
    int prolong_up(int h) override {
        ProfScope ps(P(), s, h, 3);
        const double *w = h == 0 ? S->top_wdown.as<double>() : S->lev[h - 1]->wdown.as<double>();
        if (h + 1 == H() + 1)
            return launch_transfer(S->xb.as<double>(), S->lmax_b, X(h), Lmax(h), w, S->lmax_b,
                                   true, R, s);
        return launch_transfer(X(h + 1), Lmax(h + 1), X(h), Lmax(h), w, Lmax(h + 1), true, R, s);
    }
    int bottom(int h) override {
        ProfScope ps(P(), s, h, 2);
        if (S->direct)       // the top level itself is dense: x_0 = A^-1 b_0
            return launch_dense_apply(S->b_inv.as<double>(), S->na, S->b_idx.as<int>(),
                                      S->b0.as<double>(), S->x0.as<double>(), nalm_l(S->lmax_b),
                                      R, S->b_ws.as<double>(), s);
        (void)h;
        return launch_dense_apply(S->b_inv.as<double>(), S->na, S->b_idx.as<int>(),
                                  S->bb.as<double>(), S->xb.as<double>(), nalm_l(S->lmax_b), R,
                                  S->b_ws.as<double>(), s);
    }
};

// ---- setup pieces ----------------------------------------------------------
static int setup_top_diag(mlcr_solver *S, hipStream_t s) {
    mlcr_op *op = S->op;
    mlcr_geom *g = op->g;
    const int lmax = op->lmax;
    const int l2 = 2 * lmax;
    // ring sums Xi_k(D), D <= 2 lmax, of the map xi = N^-1 (eq. Ni-dense)
    DevBuf Xi, G2, q;
    int rc;
    if ((rc = alloc(Xi, (size_t)g->nrings * (l2 + 1) * sizeof(double2)))) return rc;
    if ((rc = alloc(G2, (size_t)g->nrings * (lmax + 1) * sizeof(double2)))) return rc;
    if ((rc = alloc(q, (size_t)nalm_l(lmax) * sizeof(double)))) return rc;
    if (g->wsP.reserve((size_t)adjoint_chunks(g, lmax) * tlayout_doubles(lmax, 1, adj_rc(1)) *
                       sizeof(double)))
        return fail(MLCR_ENOMEM, "workspace allocation failed");
    if ((rc = launch_ring_adjoint(g, l2, 1, op->ninv, Xi.as<double2>(), MLCR_FP64, s))) return rc;
    if ((rc = launch_diag_pairs(Xi.as<double2>(), l2 + 1, G2.as<double2>(), lmax, g->nrings, s)))
        return rc;
    LegendreArgs a{g, lmax, 1, s};
    int nch = 0;
    if ((rc = launch_legendre_adjoint_sq(a, G2.as<double2>(), g->wsP.as<double>(), &nch))) return rc;
    if ((rc = launch_unpack_t(lmax, 1, adj_rc(1), nch, g->wsP.as<double>(), false, nullptr, 0,
                              nullptr, nullptr, nullptr, q.as<double>(), s)))
        return rc;
    if ((rc = alloc(S->top_dinv, (size_t)nalm_l(lmax) * sizeof(double)))) return rc;
    const mlcr_level &L0 = op->levels[0];
    if ((rc = launch_diag_inverse(q.as<double>(), L0.d.as<double>(), L0.bh.as<double>(),
                                  S->top_dinv.as<double>(), lmax, s)))
        return rc;
    MLCR_HIP_CHECK(hipStreamSynchronize(s));
    return MLCR_OK;
}

// tiles of each colour, grouped; off[c] .. off[c + 1] index list
static void group_by_color(const std::vector<int> &col, int ncol, std::vector<int> &list,
                           std::vector<int> &off) {
    off.assign(ncol + 1, 0);
    for (int c : col) off[c + 1]++;
    for (int c = 0; c < ncol; c++) off[c + 1] += off[c];
    list.resize(col.size());
    std::vector<int> pos(off.begin(), off.end() - 1);
    for (size_t t = 0; t < col.size(); t++) list[pos[col[t]]++] = (int)t;
}

// The paper's construction (Sec. 3.5): blocks of D_hat_h + B_hat_h^T N^-1 B_hat_h
// on the tile pattern from tabulated addition-theorem sums, the B_hat product
// without fill-in over the observation pixels, then a block incomplete
// Cholesky in the sweep-colour order with the smallest ridge (bisection in
// log alpha, relative to the largest diagonal entry, then 1.5 alpha) that
// lets every pivot succeed.  L.off / L.minv receive the factor.
static int setup_smoother_icc(mlcr_solver *S, PixLevel &L, const std::vector<int> &ptr,
                              const std::vector<int> &nbs, hipStream_t s) {
    mlcr_op *op = S->op;
    const Plan &p = S->plan;
    const int nt = L.ntiles, kk = L.kk;
    const long long nslots = L.nslots;
    int rc;
    if (op->g->kind != 0) return fail(MLCR_EINVAL, "the addition-theorem smoother needs a HEALPix grid");
    const int nobs = op->g->nside;
    if (nobs % L.nside || ((nobs / L.nside) & (nobs / L.nside - 1)))
        return fail(MLCR_EINVAL, "N_side_obs / N_side^h must be a power of two");
    const long long sub = (long long)kk * (nobs / L.nside) * (nobs / L.nside);
    // pixel centres in nested order: the level's (tile t = nested [64 t, 64 t + 64))
    // and, once per solver, the observation grid's with RING indices into N^-1
    DevBuf vlev;
    {
        std::vector<double> v;
        std::vector<int> r;
        nested_pixel_table(L.nside, v, r);
        if ((rc = up(vlev, v.data(), v.size() * sizeof(double)))) return rc;
    }
    if (!S->vobs.ptr) {
        std::vector<double> v;
        std::vector<int> r;
        nested_pixel_table(nobs, v, r);
        if ((rc = up(S->vobs, v.data(), v.size() * sizeof(double)))) return rc;
        if ((rc = up(S->oring, r.data(), r.size() * sizeof(int)))) return rc;
    }
    // addition-theorem kernels of the level: g_l = f^2 / C_l (D_hat), f b_l (B_hat)
    const int lh = L.lmax;
    const int hidx = L.opl - 1;
    std::vector<double> gd(lh + 1), gb(lh + 1);
    for (int l = 0; l <= lh; l++) {
        const double f = p.fl[hidx][l];
        gd[l] = op->cl[l] > 0 ? f * f / op->cl[l] : 0.0;
        gb[l] = op->cl[l] > 0 ? f * op->bl[l] : 0.0;
    }
    DevBuf dgd, dgb, tabD, tabB;
    if ((rc = up(dgd, gd.data(), gd.size() * sizeof(double)))) return rc;
    if ((rc = up(dgb, gb.data(), gb.size() * sizeof(double)))) return rc;
    // couplings within the pattern lie within a few tile widths: the table
    // covers 64 level pixel widths
    const int ntab = 16384;
    const double pxw = std::sqrt(4.0 * kPi / (12.0 * (double)L.nside * L.nside));
    const double thmax = std::min(kPi, 64.0 * pxw);
    const double dth = thmax / (ntab - 1);
    if ((rc = alloc(tabD, (size_t)ntab * sizeof(double))) || (rc = alloc(tabB, (size_t)ntab * sizeof(double))))
        return rc;
    if ((rc = launch_addthm_table(dgd.as<double>(), lh, dth, ntab, tabD.as<double>(), s))) return rc;
    if ((rc = launch_addthm_table(dgb.as<double>(), lh, dth, ntab, tabB.as<double>(), s))) return rc;
    AddThmTable TD{dth, ntab, tabD.as<double>()}, TB{dth, ntab, tabB.as<double>()};
    // assembly: diagonal blocks and the pairs t < u (each also stored transposed)
    std::vector<int> jobs;
    for (int t = 0; t < nt; t++)
        for (int j = ptr[t]; j < ptr[t + 1]; j++)
            if (nbs[j] > t) jobs.push_back(j);
    DevBuf djobs;
    if ((rc = up(djobs, jobs.data(), std::max<size_t>(1, jobs.size()) * sizeof(int)))) return rc;
    if ((rc = alloc(L.adiag, (size_t)nt * kk * kk * sizeof(float)))) return rc;
    if ((rc = alloc(L.aoff, (size_t)std::max(1LL, nslots) * kk * kk * sizeof(float)))) return rc;
    if ((rc = launch_smoother_assemble(nt, L.nbptr.as<int>(), L.nbs.as<int>(), L.rev.as<int>(),
                                       djobs.as<int>(), (int)jobs.size(), vlev.as<double>(),
                                       S->vobs.as<double>(), S->oring.as<int>(), op->ninv, sub, TD,
                                       TB, L.adiag.as<float>(), L.aoff.as<float>(), s)))
        return rc;
    // block ICC(0) with the ridge search
    if ((rc = alloc(L.off, (size_t)std::max(1LL, nslots) * kk * kk * sizeof(float)))) return rc;
    if ((rc = alloc(L.minv, (size_t)nt * kk * kk * sizeof(float)))) return rc;
    DevBuf dmx, dfail;
    if ((rc = alloc(dmx, sizeof(double))) || (rc = alloc(dfail, (size_t)nt * sizeof(int)))) return rc;
    if ((rc = launch_max_diag(L.adiag.as<float>(), nt, dmx.as<double>(), s))) return rc;
    double scale = 0.0;
    MLCR_HIP_CHECK(hipMemcpyAsync(&scale, dmx.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
    MLCR_HIP_CHECK(hipStreamSynchronize(s));
    if (!(scale > 0.0)) scale = 1.0;
    std::vector<int> hfail(nt);
    auto factor = [&](double alpha, int &nfail) -> int {
        MLCR_HIP_CHECK(hipMemsetAsync(dfail.ptr, 0, (size_t)nt * sizeof(int), s));
        for (int c = 0; c < L.n_sweep; c++) {
            int r2;
            if ((r2 = launch_icc_color(L.stiles.as<int>() + L.soff[c], L.soff[c + 1] - L.soff[c],
                                       L.nbptr.as<int>(), L.nbs.as<int>(), L.rev.as<int>(),
                                       L.scol.as<int>(), c, L.adiag.as<float>(), L.aoff.as<float>(),
                                       alpha * scale, L.minv.as<float>(), L.off.as<float>(),
                                       dfail.as<int>(), s)))
                return r2;
        }
        MLCR_HIP_CHECK(hipMemcpyAsync(hfail.data(), dfail.ptr, (size_t)nt * sizeof(int),
                                      hipMemcpyDeviceToHost, s));
        MLCR_HIP_CHECK(hipStreamSynchronize(s));
        nfail = 0;
        for (int v : hfail) nfail += v != 0;
        return MLCR_OK;
    };
    // the paper's rule: no ridge if the factorization succeeds, else 1.5 x the
    // smallest ridge that lets it succeed; then at least ridge_min.  A
    // smallest ridge below ridge_min / 1.5 ends at ridge_min either way, so
    // the search starts there (one factorization decides it) and bisects
    // log10 alpha to 1/300 of a decade above it.
    int nf = 0;
    double alpha = 0.0;
    bool refactor = false;
    if ((rc = factor(0.0, nf))) return rc;
    const double floor_lo = p.ridge_min / 1.5;
    if (nf > 0 && floor_lo > 0.0) {
        if ((rc = factor(floor_lo, nf))) return rc;
        if (nf == 0) alpha = floor_lo;          // raised to ridge_min below
    }
    if (nf > 0) {
        int nf_hi = 0;
        if ((rc = factor(p.ridge_max, nf_hi))) return rc;
        if (nf_hi > 0)
            return fail(MLCR_ENOTPD, "block incomplete Cholesky of the level N_side " +
                                         std::to_string(L.nside) + " smoother fails on " +
                                         std::to_string(nf_hi) + " of " + std::to_string(nt) +
                                         " tiles even with the largest ridge " +
                                         std::to_string(p.ridge_max) + " x max diagonal");
        double lo = floor_lo > 0.0 ? std::log10(floor_lo) : -12.0;
        double hi = std::log10(std::max(p.ridge_max, 1e-300));
        while (hi - lo > 1.0 / 300.0) {
            const double mid = 0.5 * (lo + hi);
            if ((rc = factor(std::pow(10.0, mid), nf))) return rc;
            if (nf == 0) hi = mid;
            else lo = mid;
        }
        alpha = std::min(p.ridge_max, 1.5 * std::pow(10.0, hi));
        refactor = true;
    }
    if (alpha < p.ridge_min) {
        alpha = p.ridge_min;
        refactor = true;
    }
    if (refactor) {
        if ((rc = factor(alpha, nf))) return rc;
        if (nf > 0) return fail(MLCR_ENOTPD, "block incomplete Cholesky failed at the chosen ridge");
    }
    S->ridge_summary.push_back((float)alpha);
    L.smoother = 1;
    if (!p.keep) {
        L.adiag.release();
        L.aoff.release();
    }
    MLCR_HIP_CHECK(hipStreamSynchronize(s));
    return MLCR_OK;
}

static int setup_smoother(mlcr_solver *S, PixLevel &L, hipStream_t s) {
    int rc;
    const int kk = L.kk;
    const int nt = 12 * (L.nside / kTile) * (L.nside / kTile);
    L.ntiles = nt;
    std::vector<int> tp((size_t)nt * kk);
    for (long long i = 0; i < (long long)nt * kk; i++) tp[i] = (int)nest2ring(L.nside, i);
    if ((rc = up(L.tilepix, tp.data(), tp.size() * sizeof(int)))) return rc;
    // tile graph: neighbour lists in CSR form, rev[slot] = slot of the reverse pair
    TileGraph G;
    if ((rc = build_tile_graph(L.nside, kTile, kMaxNb, G))) return rc;
    std::vector<int> ptr(nt + 1, 0), nbs, rev;
    for (int t = 0; t < nt; t++) {
        int n = 0;
        while (n < kMaxNb && G.nb[(size_t)t * kMaxNb + n] >= 0) n++;
        ptr[t + 1] = ptr[t] + n;
    }
    nbs.resize(ptr[nt]);
    rev.resize(ptr[nt]);
    for (int t = 0; t < nt; t++)
        for (int j = ptr[t]; j < ptr[t + 1]; j++) nbs[j] = G.nb[(size_t)t * kMaxNb + (j - ptr[t])];
    for (int t = 0; t < nt; t++)
        for (int j = ptr[t]; j < ptr[t + 1]; j++) {
            const int u = nbs[j];
            const auto b = nbs.begin() + ptr[u], e = nbs.begin() + ptr[u + 1];
            const auto it = std::lower_bound(b, e, t);
            if (it == e || *it != t) return fail(MLCR_EINVAL, "tile graph is not symmetric");
            rev[j] = (int)(it - nbs.begin());
        }
    const long long nslots = ptr[nt];
    if ((rc = up(L.nbptr, ptr.data(), ptr.size() * sizeof(int)))) return rc;
    if ((rc = up(L.nbs, nbs.data(), nbs.size() * sizeof(int)))) return rc;
    DevBuf drev;
    if ((rc = up(drev, rev.data(), rev.size() * sizeof(int)))) return rc;
    if ((rc = up(L.scol, G.sweep_color.data(), nt * sizeof(int)))) return rc;
    std::vector<int> slist, plist, poff;
    group_by_color(G.sweep_color, G.n_sweep, slist, L.soff);
    group_by_color(G.probe_color, G.n_probe, plist, poff);
    L.n_sweep = G.n_sweep;
    L.n_probe = G.n_probe;
    if ((rc = up(L.stiles, slist.data(), slist.size() * sizeof(int)))) return rc;
    DevBuf ptiles;
    if ((rc = up(ptiles, plist.data(), plist.size() * sizeof(int)))) return rc;
    L.nslots = (int)nslots;
    if (S->plan.smoother == 1) {
        L.rev = std::move(drev);
        return setup_smoother_icc(S, L, ptr, nbs, s);
    }

    const long long npix = L.geom->npix, na = nalm_l(L.lmax);
    const int P = 16;          // probes per batch
    DevBuf maps, U, V, blocks;
    if ((rc = alloc(maps, (size_t)P * npix * sizeof(double)))) return rc;
    if ((rc = alloc(U, (size_t)P * na * sizeof(double)))) return rc;
    if ((rc = alloc(V, (size_t)P * na * sizeof(double)))) return rc;
    if ((rc = alloc(blocks, (size_t)nt * kk * kk * sizeof(double)))) return rc;
    if ((rc = alloc(L.off, (size_t)std::max(1LL, nslots) * kk * kk * sizeof(float)))) return rc;
    // column c of the blocks of tile u: (Y_h A_h Y_h^T e_c) read at u and at its
    // neighbours, with e_c the indicator of position c in every tile of u's
    // probe colour
    for (int c = 0; c < L.n_probe; c++) {
        const int *tl = ptiles.as<int>() + poff[c];
        const int ntl = poff[c + 1] - poff[c];
        for (int c0 = 0; c0 < kk; c0 += P) {
            const int np = std::min(P, kk - c0);
            if ((rc = launch_probe_maps(maps.as<double>(), npix, L.tilepix.as<int>(), tl, ntl, kk,
                                        c0, np, s)))
                return rc;
            if ((rc = sht_adjoint(L.geom, L.lmax, np, maps.as<double>(), U.as<double>(), MLCR_FP64,
                                  s)))
                return rc;
            if ((rc = solver_apply(S, L.opl, np, U.as<double>(), V.as<double>(), MLCR_FP64, s)))
                return rc;
            if ((rc = sht_synth(L.geom, L.lmax, np, V.as<double>(), maps.as<double>(), MLCR_FP64,
                                s)))
                return rc;
            if ((rc = launch_probe_collect(maps.as<double>(), npix, L.tilepix.as<int>(), tl, ntl,
                                           L.nbptr.as<int>(), L.nbs.as<int>(), drev.as<int>(),
                                           kMaxNb, c0, np, blocks.as<double>(),
                                           L.off.as<float>(), s)))
                return rc;
        }
    }
    if (nslots > 0 &&
        (rc = launch_sym_off(L.nbptr.as<int>(), L.nbs.as<int>(), drev.as<int>(), L.off.as<float>(),
                             nt, s)))
        return rc;
    if ((rc = alloc(L.minv, (size_t)nt * kk * kk * sizeof(float)))) return rc;
    if ((rc = alloc(L.ridge, (size_t)nt * sizeof(float)))) return rc;
    if ((rc = launch_tile_factor(blocks.as<double>(), nt, kk, L.minv.as<float>(),
                                 L.ridge.as<float>(), s)))
        return rc;
    MLCR_HIP_CHECK(hipStreamSynchronize(s));
    std::vector<float> rg(nt);
    MLCR_HIP_CHECK(hipMemcpy(rg.data(), L.ridge.ptr, nt * sizeof(float), hipMemcpyDeviceToHost));
    float worst = 0.f;
    int nfail = 0, first_fail = -1;
    for (int t = 0; t < nt; t++) {
        if (rg[t] < 0) {
            if (first_fail < 0) first_fail = t;
            nfail++;
        }
        worst = std::max(worst, rg[t]);
    }
    if (nfail) {
        // describe the first failing block: non-finite entries, diagonal range, asymmetry
        std::vector<double> B((size_t)kk * kk);
        MLCR_HIP_CHECK(hipMemcpy(B.data(), blocks.as<double>() + (size_t)first_fail * kk * kk,
                                 B.size() * sizeof(double), hipMemcpyDeviceToHost));
        int nonfinite = 0;
        double dmin = 1e300, dmax = -1e300, asym = 0.0, amax = 0.0;
        for (int i = 0; i < kk; i++)
            for (int j = 0; j < kk; j++) {
                const double v = B[(size_t)i * kk + j];
                if (!std::isfinite(v)) nonfinite++;
                amax = std::max(amax, std::fabs(v));
                asym = std::max(asym, std::fabs(v - B[(size_t)j * kk + i]));
                if (i == j) {
                    dmin = std::min(dmin, v);
                    dmax = std::max(dmax, v);
                }
            }
        return fail(MLCR_ENOTPD,
                    "tile factorization failed even with a ridge: level N_side " +
                        std::to_string(L.nside) + ", " + std::to_string(nfail) + " of " +
                        std::to_string(nt) + " tiles; first tile " + std::to_string(first_fail) +
                        ": non-finite " + std::to_string(nonfinite) + ", diag [" +
                        std::to_string(dmin) + ", " + std::to_string(dmax) + "], max |a| " +
                        std::to_string(amax) + ", max asymmetry " + std::to_string(asym));
    }
    S->ridge_summary.push_back(worst);
    return MLCR_OK;
}

// The dense bottom level: A_B over its active modes l <= lmax_b, its entries
// from the ring Fourier sums of eq. Ni-dense on the level's grid -- the
// Gauss-Legendre grid of its downgraded N^-1 (Sec. 3.4) when the level uses
// one, which makes the cost O(lmax_b) per entry instead of O(lmax) -- then a
// Cholesky factor and the explicit inverse (one GEMV per visit).
static int setup_bottom(mlcr_solver *S, hipStream_t s) {
    mlcr_op *op = S->op;
    const int lb = S->lmax_b;
    // active modes of the bottom level in packed order, with (l, m, sine)
    const std::vector<double> &clb = op->cl;
    std::vector<int> idx, mode;
    {
        long long pos = 0;
        for (int l = 0; l <= lb; l++, pos++)
            if (clb[l] > 0) {
                idx.push_back((int)pos);
                mode.push_back(l);
            }
        for (int m = 1; m <= lb; m++)
            for (int cs = 0; cs < 2; cs++)
                for (int l = m; l <= lb; l++, pos++)
                    if (clb[l] > 0) {
                        idx.push_back((int)pos);
                        mode.push_back(l | (m << 8) | (cs << 16));
                    }
    }
    const int na = (int)idx.size();
    S->na = na;
    int rc;
    if (na == 0) return fail(MLCR_EINVAL, "no active modes at the bottom level");
    if ((rc = up(S->b_idx, idx.data(), idx.size() * sizeof(int)))) return rc;
    const mlcr_level &Lv = S->direct ? op->levels[0] : *S->slev[S->opl_b];
    mlcr_geom *gb = Lv.gl ? Lv.gl : op->g;
    const double *ninvb = Lv.gl ? Lv.gninv.as<double>() : op->ninv;
    const int ldx = 2 * lb + 1;
    DevBuf Xi, lt, dmode, Ad, info;
    if ((rc = alloc(Xi, (size_t)gb->nrings * ldx * sizeof(double2)))) return rc;
    if ((rc = alloc(lt, (size_t)gb->nrings * (lb + 1) * (lb + 2) / 2 * sizeof(double)))) return rc;
    if ((rc = up(dmode, mode.data(), mode.size() * sizeof(int)))) return rc;
    if ((rc = alloc(Ad, (size_t)na * na * sizeof(double)))) return rc;
    if ((rc = alloc(info, sizeof(int)))) return rc;
    // ring sums of the (downgraded) inverse-noise map at frequencies 0..2 lmax_b
    if ((rc = launch_ring_adjoint(gb, 2 * lb, 1, ninvb, Xi.as<double2>(), MLCR_FP64, s))) return rc;
    if ((rc = launch_dense_lambda(gb->ring_z.as<double>(), gb->ring_s.as<double>(), gb->nrings, lb,
                                  lt.as<double>(), s)))
        return rc;
    if ((rc = launch_dense_ringdft(Xi.as<double2>(), ldx, lt.as<double>(), lb, gb->nrings,
                                   dmode.as<int>(), na, Lv.d.as<double>(), Lv.bh.as<double>(),
                                   Ad.as<double>(), s)))
        return rc;
    if ((rc = alloc(S->b_A, (size_t)na * na * sizeof(double)))) return rc;
    MLCR_HIP_CHECK(hipMemcpyAsync(S->b_A.ptr, Ad.ptr, (size_t)na * na * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
    if ((rc = launch_dense_cholesky(Ad.as<double>(), na, info.as<int>(), s))) return rc;
    int hinfo = 0;
    MLCR_HIP_CHECK(hipMemcpyAsync(&hinfo, info.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    MLCR_HIP_CHECK(hipStreamSynchronize(s));
    if (hinfo) return fail(MLCR_ENOTPD, "dense bottom-level matrix is not positive definite");
    if ((rc = alloc(S->b_inv, (size_t)na * na * sizeof(double)))) return rc;
    if ((rc = alloc(S->b_ws, (size_t)dense_apply_ws_doubles(na, S->max_nrhs) * sizeof(double))))
        return rc;
    if ((rc = launch_dense_inverse(Ad.as<double>(), na, S->b_inv.as<double>(), s))) return rc;
    MLCR_HIP_CHECK(hipStreamSynchronize(s));
    return MLCR_OK;
}

// A coarse level evaluates Y^T N^-1 Y on a Gauss-Legendre grid (Sec. 3.4)
// when that grid -- 2 lmax_h + 1 rings of the smallest power of two >=
// 4 lmax_h + 1 pixels -- is the cheaper one; otherwise on the observation
// grid itself.  Both give the same operator (exactly, up to rounding); only
// the cost differs.  The Legendre steps scale with the number of rings, and
// the ring step costs less per pixel on rings of one power-of-two length than
// on the observation grid's mixed lengths, so fewer rings and at most twice
// the pixels is cheaper (lmax_h 2048 under N_side 2048: 4097 x 16384 pixels
// against 8191 rings and 50.3M pixels, 1.7x faster per application).
static int set_level_best(mlcr_solver *S, int h, int lmax_h, const double *fl, bool gl) {
    mlcr_op *op = S->op;
    long long nphi = 4;
    while (nphi < 4LL * lmax_h + 1) nphi <<= 1;
    const long long gl_rings = 2LL * lmax_h + 1;
    const long long gl_pix = gl_rings * nphi;
    const bool use_gl = gl && 2 * lmax_h <= op->g->lmax && nphi <= 16384 &&
                        gl_rings < op->g->nrings && gl_pix <= 2 * op->g->npix;
    if ((int)S->slev.size() <= h) S->slev.resize(h + 1);
    S->slev[h].reset(new (std::nothrow) mlcr_level());
    if (!S->slev[h]) return fail(MLCR_ENOMEM, "host allocation failed");
    return define_level(op, *S->slev[h], lmax_h, fl, use_gl);
}

static int solver_build(mlcr_solver *S, const Plan &p, hipStream_t s) {
    mlcr_op *op = S->op;
    const int R = S->max_nrhs;
    const int lmax = op->lmax;
    int rc;
    S->plan = p;
    S->direct = (p.H == 0);
    {
        std::vector<int> nr(p.H + 1);
        nr[0] = p.nrec_top;
        for (int h = 0; h < p.H; h++) nr[h + 1] = p.nrec[h];
        build_schedule(S->direct ? 0 : p.H + 1, nr, S->sched);
        S->prof.reset(p.H + 2);
        S->prior_version = op->prior_version;
    }
    std::vector<double> act0(lmax + 1);
    for (int l = 0; l <= lmax; l++) act0[l] = op->cl[l] > 0 ? 1.0 : 0.0;
    if ((rc = up(S->top_act, act0.data(), act0.size() * sizeof(double)))) return rc;
    const size_t top_bytes = (size_t)R * nalm_l(lmax) * sizeof(double);
    for (DevBuf *b : {&S->x0, &S->b0, &S->r0, &S->t0, &S->ro, &S->to})
        if ((rc = alloc(*b, top_bytes))) return rc;
    std::vector<double> sinv(lmax + 1), ch(lmax + 1);
    for (int l = 0; l <= lmax; l++) {
        sinv[l] = op->cl[l] > 0 ? 1.0 / op->cl[l] : 0.0;
        ch[l] = op->cl[l];
    }
    if ((rc = up(S->sinv, sinv.data(), sinv.size() * sizeof(double)))) return rc;
    if ((rc = up(S->chalf, ch.data(), ch.size() * sizeof(double)))) return rc;
    if ((rc = alloc(S->partial, (size_t)R * (lmax + 1) * 2 * sizeof(double)))) return rc;
    if ((rc = alloc(S->norms, (size_t)R * 2 * sizeof(double)))) return rc;

    if (S->direct) {
        S->lmax_b = lmax;
        S->opl_b = 0;
        return setup_bottom(S, s);
    }
    // The coarse levels are Galerkin products of the top operator, which
    // needs every mode in the unknowns: with C_l = 0 (a mode conditioned to
    // zero, e.g. C_0 = C_1 = 0) the pixel operators lose locality, and the
    // paper's wide prior C_0 = C_1 = C_2 is the supported form (Sec. 4.1).
    for (int l = 0; l <= lmax; l++)
        if (!(op->cl[l] > 0))
            return fail(MLCR_EINVAL, "the multi-level solver needs C_l > 0 for every l (l = " +
                                         std::to_string(l) +
                                         " has C_l = 0; use a wide prior such as C_0 = C_1 = C_2)");
    // pixel levels
    for (int h = 0; h < p.H; h++) {
        auto L = std::make_unique<PixLevel>();
        L->nside = p.nside[h];
        L->lmax = p.lmax[h];
        L->opl = h + 1;
        if ((rc = mlcr_geom_create(L->nside, L->lmax, &L->geom))) return rc;
        if ((rc = set_level_best(S, L->opl, L->lmax, p.fl[h].data(), p.gl))) return rc;
        std::vector<double> act(L->lmax + 1), one(L->lmax + 1);
        for (int l = 0; l <= L->lmax; l++) {
            act[l] = op->cl[l] > 0 ? 1.0 : 0.0;
            one[l] = p.omega * act[l];
        }
        if ((rc = up(L->act, act.data(), act.size() * sizeof(double)))) return rc;
        if ((rc = up(L->one, one.data(), one.size() * sizeof(double)))) return rc;
        const size_t vb = (size_t)R * nalm_l(L->lmax) * sizeof(double);
        for (DevBuf *b : {&L->x, &L->b, &L->r, &L->t})
            if ((rc = alloc(*b, vb))) return rc;
        const size_t mb = (size_t)R * L->geom->npix * sizeof(double);
        if ((rc = alloc(L->map, mb)) || (rc = alloc(L->cmap, mb))) return rc;
        S->lev.push_back(std::move(L));
    }
    // restriction weights f~^H / f~^h (Sec. 3.2, eq. f_l)
    {
        std::vector<double> w(p.lmax[0] + 1);
        for (int l = 0; l <= p.lmax[0]; l++) w[l] = p.fl[0][l];
        if ((rc = up(S->top_wdown, w.data(), w.size() * sizeof(double)))) return rc;
    }
    for (int h = 0; h < p.H; h++) {
        const bool last = (h == p.H - 1);
        const int ln = last ? p.lmax_b : p.lmax[h + 1];
        std::vector<double> w(ln + 1);
        for (int l = 0; l <= ln; l++) {
            const double fh = p.fl[h][l];
            const double fH = last ? fh : p.fl[h + 1][l];
            w[l] = fh > 0.0 ? fH / fh : 0.0;
        }
        if ((rc = up(S->lev[h]->wdown, w.data(), w.size() * sizeof(double)))) return rc;
    }
    {
        std::vector<double> hp(lmax + 1);
        for (int l = 0; l <= lmax; l++) hp[l] = p.omega_top * p.highpass[l];
        if ((rc = up(S->top_hp, hp.data(), hp.size() * sizeof(double)))) return rc;
    }
    // bottom level A_B = restriction of the last pixel level to l <= lmax_b
    S->lmax_b = p.lmax_b;
    S->opl_b = p.H + 1;
    {
        std::vector<double> fb(p.fl[p.H - 1].begin(), p.fl[p.H - 1].begin() + p.lmax_b + 1);
        if ((rc = set_level_best(S, S->opl_b, S->lmax_b, fb.data(), p.gl))) return rc;
    }
    const size_t bbytes = (size_t)R * nalm_l(S->lmax_b) * sizeof(double);
    if ((rc = alloc(S->xb, bbytes)) || (rc = alloc(S->bb, bbytes))) return rc;
    if ((rc = setup_top_diag(S, s))) return rc;
    for (auto &L : S->lev)
        if ((rc = setup_smoother(S, *L, s))) return rc;
    return setup_bottom(S, s);
}

}  // namespace mlcr

extern "C" {

int mlcr_nest2ring(int nside, long long n, const long long *nest, long long *ring) {
    if (nside < 1 || n < 0 || (n > 0 && (!nest || !ring))) return fail(MLCR_EINVAL, "bad argument");
    const long long npix = 12LL * nside * nside;
    for (long long i = 0; i < n; i++) {
        if (nest[i] < 0 || nest[i] >= npix) return fail(MLCR_EINVAL, "nested index out of range");
        ring[i] = nest2ring(nside, nest[i]);
    }
    return MLCR_OK;
}

int mlcr_tile_graph(int nside, int max_nb, int *nb, int *sweep_color, int *probe_color,
                    int *n_sweep, int *n_probe) {
    if (nside < kTile || nside % kTile || max_nb < 1 || !nb || !sweep_color || !probe_color ||
        !n_sweep || !n_probe)
        return fail(MLCR_EINVAL, "bad argument");
    TileGraph G;
    int rc = build_tile_graph(nside, kTile, max_nb, G);
    if (rc) return rc;
    std::copy(G.nb.begin(), G.nb.end(), nb);
    std::copy(G.sweep_color.begin(), G.sweep_color.end(), sweep_color);
    std::copy(G.probe_color.begin(), G.probe_color.end(), probe_color);
    *n_sweep = G.n_sweep;
    *n_probe = G.n_probe;
    return MLCR_OK;
}

int mlcr_ladder_plan(int nside, int lmax, int *nlevels, int *nsides, int *lmaxs, int *nrec,
                     int *nrec_top, int *lmax_bottom) {
    if (nside < 1 || lmax < 0 || !nlevels) return fail(MLCR_EINVAL, "bad argument");
    Plan p;
    default_plan(nside, lmax, p);
    *nlevels = p.H;
    for (int h = 0; h < p.H; h++) {
        if (nsides) nsides[h] = p.nside[h];
        if (lmaxs) lmaxs[h] = p.lmax[h];
        if (nrec) nrec[h] = p.nrec[h];
    }
    if (nrec_top) *nrec_top = p.nrec_top;
    if (lmax_bottom) *lmax_bottom = p.lmax_b;
    return MLCR_OK;
}

int mlcr_cycle_counts(int nlevels, const int *nrec, int nrec_top, int ncycles, long long *counts) {
    if (nlevels < 0 || nlevels > 8 || ncycles < 1 || !counts || (nlevels > 0 && !nrec))
        return fail(MLCR_EINVAL, "bad argument");
    const int B = nlevels == 0 ? 0 : nlevels + 1;
    std::vector<int> nr(nlevels + 1);
    nr[0] = nrec_top;
    for (int h = 0; h < nlevels; h++) nr[h + 1] = nrec[h];
    CountOps ops(B + 1, B);
    std::vector<Step> sch;
    build_schedule(B, nr, sch);
    for (int c = 0; c < ncycles; c++) {
        run_schedule(ops, sch);
        ops.c[1]++;     // float64 residual b - A x of CR-Solve at the top level
    }
    for (size_t i = 0; i < ops.c.size(); i++) counts[i] = ops.c[i];
    return MLCR_OK;
}

int mlcr_ladder_default(int nside, int lmax, mlcr_ladder_desc *out, double *filters) {
    if (nside < 1 || lmax < 0 || !out || !filters) return fail(MLCR_EINVAL, "bad argument");
    Plan p;
    default_plan(nside, lmax, p);
    desc_from_plan(p, lmax, out, filters);
    return MLCR_OK;
}

int mlcr_ladder_check(int nside, int lmax, const mlcr_ladder_desc *ladder) {
    if (nside < 1 || lmax < 0) return fail(MLCR_EINVAL, "bad grid or band limit");
    return check_ladder(nside, lmax, ladder);
}

int mlcr_solver_create(mlcr_op *op, const mlcr_ladder_desc *ladder, int max_nrhs,
                       mlcr_solver **out) {
    if (!out) return fail(MLCR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!op) return fail(MLCR_EINVAL, "operator is NULL");
    if (max_nrhs < 1) return fail(MLCR_EINVAL, "max_nrhs must be >= 1");
    Plan p;
    if (ladder) {
        int rc = check_ladder(op->g->nside, op->lmax, ladder);
        if (rc) return rc;
        plan_from_desc(op->lmax, ladder, p);
    } else {
        default_plan(op->g->nside, op->lmax, p);
    }
    mlcr_solver *S = new (std::nothrow) mlcr_solver();
    if (!S) return fail(MLCR_ENOMEM, "host allocation failed");
    S->op = op;
    S->max_nrhs = max_nrhs;
    int rc = solver_build(S, p, nullptr);
    if (rc) {
        (void)hipDeviceSynchronize();
        delete S;
        return rc;
    }
    *out = S;
    return MLCR_OK;
}

void mlcr_solver_destroy(mlcr_solver *S) {
    if (!S) return;
    (void)hipDeviceSynchronize();
    delete S;
}

int mlcr_solver_info(const mlcr_solver *S, int *nlevels, int *lmax_bottom, int *n_bottom,
                     float *max_ridge) {
    if (!S) return fail(MLCR_EINVAL, "solver is NULL");
    if (nlevels) *nlevels = S->plan.H;
    if (lmax_bottom) *lmax_bottom = S->lmax_b;
    if (n_bottom) *n_bottom = S->na;
    if (max_ridge) {
        float w = 0.f;
        for (float v : S->ridge_summary) w = std::max(w, v);
        *max_ridge = w;
    }
    return MLCR_OK;
}

int mlcr_solver_set_profile(mlcr_solver *S, int on) {
    if (!S) return fail(MLCR_EINVAL, "solver is NULL");
    S->prof.drain();
    S->prof.on = on != 0;
    S->prof.reset(S->plan.H + 2);
    return MLCR_OK;
}

int mlcr_solver_profile(const mlcr_solver *S, int nlevels_max, double *ms, long long *calls) {
    if (!S || nlevels_max < 0) return fail(MLCR_EINVAL, "bad argument");
    const_cast<mlcr_solver *>(S)->prof.drain();
    const int L = std::min(nlevels_max, S->plan.H + 2);
    for (int i = 0; i < 4 * L; i++) {
        if (ms) ms[i] = i < (int)S->prof.ms.size() ? S->prof.ms[i] : 0.0;
        if (calls) calls[i] = i < (int)S->prof.calls.size() ? S->prof.calls[i] : 0;
    }
    return S->plan.H + 2;
}

int mlcr_solver_level_blocks(const mlcr_solver *S, int level, int which, int *ntiles,
                             long long *nslots, float *dev_diag, float *dev_off) {
    if (!S || level < 1 || level > S->plan.H || (which != 0 && which != 1))
        return fail(MLCR_EINVAL, "bad solver, level or kind");
    const PixLevel &L = *S->lev[level - 1];
    if (L.smoother != 1) return fail(MLCR_EINVAL, "the level does not use the incomplete-Cholesky smoother");
    if (ntiles) *ntiles = L.ntiles;
    if (nslots) *nslots = L.nslots;
    const size_t bb = (size_t)L.kk * L.kk * sizeof(float);
    const DevBuf &dg = which == 0 ? L.adiag : L.minv;
    const DevBuf &of = which == 0 ? L.aoff : L.off;
    if ((dev_diag || dev_off) && which == 0 && !L.adiag.ptr)
        return fail(MLCR_EINVAL, "assembled blocks were not kept (ladder keep_blocks = 0)");
    if (dev_diag) MLCR_HIP_CHECK(hipMemcpy(dev_diag, dg.ptr, (size_t)L.ntiles * bb, hipMemcpyDeviceToDevice));
    if (dev_off && L.nslots > 0)
        MLCR_HIP_CHECK(hipMemcpy(dev_off, of.ptr, (size_t)L.nslots * bb, hipMemcpyDeviceToDevice));
    return MLCR_OK;
}

int mlcr_solver_bottom(const mlcr_solver *S, int *n, double *dev_A, int *host_idx) {
    if (!S) return fail(MLCR_EINVAL, "solver is NULL");
    if (n) *n = S->na;
    if (dev_A)
        MLCR_HIP_CHECK(hipMemcpy(dev_A, S->b_A.ptr, (size_t)S->na * S->na * sizeof(double),
                                 hipMemcpyDeviceToDevice));
    if (host_idx)
        MLCR_HIP_CHECK(hipMemcpy(host_idx, S->b_idx.ptr, (size_t)S->na * sizeof(int),
                                 hipMemcpyDeviceToHost));
    return MLCR_OK;
}

int mlcr_solver_top_dinv(const mlcr_solver *S, double *out, void *stream) {
    if (!S || !out) return fail(MLCR_EINVAL, "NULL argument");
    if (S->direct) return fail(MLCR_EINVAL, "solver has no top-level smoother (dense solve)");
    MLCR_HIP_CHECK(hipMemcpyAsync(out, S->top_dinv.ptr, (size_t)nalm_l(S->op->lmax) * sizeof(double),
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return MLCR_OK;
}

namespace mlcr {

// One CR-Solve (Fig. code:mg, correction form) split into steps that only
// enqueue work and steps that read the residual norms back, so that several
// solves on different streams can be interleaved cycle by cycle.
struct SolveRun {
    mlcr_solver *S;
    int nrhs, prec;
    const double *b;
    double *x;
    double rtol;
    hipStream_t s;
    std::vector<double> hn, rho0, rho;
    std::vector<int> done, cyc;
    int it = 0;
    bool all = false;

    SolveRun(mlcr_solver *S_, int n, const double *b_, double *x_, double rt, int p, hipStream_t st)
        : S(S_), nrhs(n), prec(p), b(b_), x(x_), rtol(rt), s(st), hn(2 * n), rho0(n), rho(n, 0.0),
          done(n, 0), cyc(n, 0) {}
    // r = b - A x in float64 and its S^-1 norms, copied to hn (not yet waited on)
    int enqueue_residual() {
        mlcr_op *op = S->op;
        int rc;
        {
            ProfScope ps(S->prof.on ? &S->prof : nullptr, s, 0, 0);
            if ((rc = apply_level(op, 0, nrhs, x, S->to.as<double>(), MLCR_FP64, s))) return rc;
        }
        if ((rc = launch_residual(b, S->to.as<double>(), S->ro.as<double>(), S->top_act.as<double>(),
                                  op->lmax, nrhs, s)))
            return rc;
        if ((rc = launch_wnorms(S->ro.as<double>(), b, S->sinv.as<double>(), op->lmax, nrhs,
                                S->partial.as<double>(), S->norms.as<double>(), s)))
            return rc;
        return MLCR_OK;
    }
    int read_norms(std::vector<double> &out) {
        MLCR_HIP_CHECK(hipMemcpyAsync(hn.data(), S->norms.ptr, 2 * nrhs * sizeof(double),
                                      hipMemcpyDeviceToHost, s));
        MLCR_HIP_CHECK(hipStreamSynchronize(s));
        for (int r = 0; r < nrhs; r++)
            out[r] = hn[2 * r + 1] > 0 ? std::sqrt(hn[2 * r] / hn[2 * r + 1]) : 0.0;
        return MLCR_OK;
    }
    // The start: x holds the start vector (excluded modes projected out).  Its
    // S^-1 norms decide whether r = b - A x needs the operator: from x = 0
    // (every RHS) the residual is b itself and the float64 apply is skipped.
    // Three steps so that a group of solves enqueues each step for all its
    // problems before waiting on any.
    int enqueue_start() {
        int rc;
        if ((rc = launch_residual(x, nullptr, x, S->top_act.as<double>(), S->op->lmax, nrhs, s)))
            return rc;
        if ((rc = launch_wnorms(x, nullptr, S->sinv.as<double>(), S->op->lmax, nrhs,
                                S->partial.as<double>(), S->norms.as<double>(), s)))
            return rc;
        MLCR_HIP_CHECK(hipMemcpyAsync(hn.data(), S->norms.ptr, 2 * nrhs * sizeof(double),
                                      hipMemcpyDeviceToHost, s));
        return MLCR_OK;
    }
    int enqueue_start_residual() {
        MLCR_HIP_CHECK(hipStreamSynchronize(s));
        bool xzero = true;
        for (int r = 0; r < nrhs; r++) xzero = xzero && hn[2 * r] == 0.0;
        if (!xzero) return enqueue_residual();
        int rc;
        mlcr_op *op = S->op;
        if ((rc = launch_residual(b, nullptr, S->ro.as<double>(), S->top_act.as<double>(), op->lmax,
                                  nrhs, s)))
            return rc;
        return launch_wnorms(S->ro.as<double>(), b, S->sinv.as<double>(), op->lmax, nrhs,
                             S->partial.as<double>(), S->norms.as<double>(), s);
    }
    int finish_start() {
        int rc;
        if ((rc = read_norms(rho0))) return rc;
        rho = rho0;
        all = true;
        for (int r = 0; r < nrhs; r++) all = all && rho[r] <= rtol;
        return MLCR_OK;
    }
    // one cycle: solve A c = r from c = 0, x += c, then the new residual.
    // Only kernels and device copies: in graph mode cycle 2 is captured
    // (every workspace has reached its size in cycle 1) and later cycles
    // replay it; a capture that fails falls back to direct launches.
    hipGraphExec_t exec = nullptr;
    bool graph_off = false;
    ~SolveRun() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
    int enqueue_cycle_body() {
        const int lmax = S->op->lmax;
        const long long na = nalm_l(lmax);
        int rc;
        MLCR_HIP_CHECK(hipMemcpyAsync(S->b0.ptr, S->ro.ptr, (size_t)nrhs * na * sizeof(double),
                                      hipMemcpyDeviceToDevice, s));
        if ((rc = launch_fill_zero(S->x0.as<double>(), (long long)nrhs * na, s))) return rc;
        GpuOps ops(S, nrhs, prec, s);
        if ((rc = run_schedule(ops, S->sched))) return rc;
        if ((rc = launch_axpy_l(x, S->x0.as<double>(), S->top_act.as<double>(), nullptr, lmax, nrhs,
                                s)))
            return rc;
        return enqueue_residual();
    }
    int enqueue_cycle() {
        int rc = MLCR_OK;
        if (!S->graph || graph_off || it == 0 || S->prof.on) {
            rc = enqueue_cycle_body();
        } else if (exec) {
            MLCR_HIP_CHECK(hipGraphLaunch(exec, s));
            S->graph_replays++;
        } else if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
            (void)hipGetLastError();
            graph_off = true;
            S->graph_fallbacks++;
            rc = enqueue_cycle_body();
        } else {
            rc = enqueue_cycle_body();
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            hipError_t ei = e;
            if (e == hipSuccess && graph) ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess || !graph || ei != hipSuccess) {
                (void)hipGetLastError();
                exec = nullptr;
                graph_off = true;
                S->graph_fallbacks++;
                rc = enqueue_cycle_body();      // the captured work did not run: run it now
            } else {
                MLCR_HIP_CHECK(hipGraphLaunch(exec, s));
                S->graph_replays++;
            }
        }
        if (rc) return rc;
        it++;
        return MLCR_OK;
    }
    int finish_cycle() {
        int rc;
        if ((rc = read_norms(rho))) return rc;
        S->prof.drain();
        all = true;
        for (int r = 0; r < nrhs; r++) {
            if (!done[r]) cyc[r] = it;
            if (rho[r] <= rtol) done[r] = 1;
            all = all && done[r];
        }
        return MLCR_OK;
    }
    // ||S^{1/2} r|| for the a-posteriori max-pixel-error bound, and the report
    int finish(mlcr_solve_info *info) {
        int rc;
        if ((rc = launch_wnorms(S->ro.as<double>(), nullptr, S->chalf.as<double>(), S->op->lmax,
                                nrhs, S->partial.as<double>(), S->norms.as<double>(), s)))
            return rc;
        MLCR_HIP_CHECK(hipMemcpyAsync(hn.data(), S->norms.ptr, 2 * nrhs * sizeof(double),
                                      hipMemcpyDeviceToHost, s));
        MLCR_HIP_CHECK(hipStreamSynchronize(s));
        if (info)
            for (int r = 0; r < nrhs; r++) {
                info[r].cycles = cyc[r];
                info[r].rho0 = rho0[r];
                info[r].rho = rho[r];
                info[r].s_half_res = std::sqrt(hn[2 * r]);
                info[r].converged = rho[r] <= rtol;
            }
        return MLCR_OK;
    }
};

static int check_solve_args(mlcr_solver *S, int nrhs, const double *b, double *x, double rtol,
                            int max_cycles, int prec) {
    if (!S || !b || !x) return fail(MLCR_EINVAL, "NULL argument");
    if (nrhs < 1 || nrhs > S->max_nrhs) return fail(MLCR_EINVAL, "nrhs out of [1, max_nrhs]");
    if (max_cycles < 1) return fail(MLCR_EINVAL, "max_cycles must be >= 1");
    if (!(rtol >= 0.0)) return fail(MLCR_EINVAL, "rtol must be >= 0");
    if (prec != MLCR_FP64 && prec != MLCR_FP32 && prec != MLCR_BF16X3)
        return fail(MLCR_EINVAL, "unknown precision");
    // after mlcr_op_set_prior: the stopping norm and the certificate follow
    // the operator's current spectrum (the hierarchy keeps its own)
    if (S->prior_version != S->op->prior_version) {
        const int lmax = S->op->lmax;
        std::vector<double> sinv(lmax + 1), ch(lmax + 1);
        for (int l = 0; l <= lmax; l++) {
            sinv[l] = S->op->cl[l] > 0 ? 1.0 / S->op->cl[l] : 0.0;
            ch[l] = S->op->cl[l];
        }
        int rc;
        if ((rc = up(S->sinv, sinv.data(), sinv.size() * sizeof(double)))) return rc;
        if ((rc = up(S->chalf, ch.data(), ch.size() * sizeof(double)))) return rc;
        for (auto &L : S->slev)
            if (L && (rc = refresh_level(S->op, *L))) return rc;
        S->prior_version = S->op->prior_version;
    }
    return MLCR_OK;
}

}  // namespace mlcr

int wcycle_solve(mlcr_solver *S, int nrhs, const double *b, double *x, double rtol, int max_cycles,
                 int prec, mlcr_solve_info *info, void *stream) {
    int rc;
    if ((rc = check_solve_args(S, nrhs, b, x, rtol, max_cycles, prec))) return rc;
    // graph mode runs on a pooled stream (the caller's may be the legacy
    // default stream, which cannot be captured), forked and joined by events
    StreamFork f;
    hipStream_t s = (hipStream_t)stream;
    if (S->graph) {
        if ((rc = f.begin(s, {S->op->g}))) return rc;
        s = f.item_stream[0];
    }
    {
        SolveRun run(S, nrhs, b, x, rtol, prec, s);
        if (!(rc = run.enqueue_start()) && !(rc = run.enqueue_start_residual()) &&
            !(rc = run.finish_start()))
            while (!run.all && run.it < max_cycles)
                if ((rc = run.enqueue_cycle()) || (rc = run.finish_cycle())) break;
        if (!rc) rc = run.finish(info);
        if (!rc && !run.all) rc = fail(MLCR_ENOCONV, "rtol not reached within max_cycles");
    }
    if (S->graph) {
        const int rj = f.join();
        if (!rc) rc = rj;
    }
    return rc;
}

int mlcr_solver_set_graph(mlcr_solver *S, int on) {
    if (!S) return fail(MLCR_EINVAL, "NULL argument");
    S->graph = on ? 1 : 0;
    return MLCR_OK;
}

int mlcr_solver_graph_stats(const mlcr_solver *S, long long *replays, long long *fallbacks) {
    if (!S) return fail(MLCR_EINVAL, "NULL argument");
    if (replays) *replays = S->graph_replays;
    if (fallbacks) *fallbacks = S->graph_fallbacks;
    return MLCR_OK;
}

}  // extern "C"

int wcycle_solve_grouped(int nprob, mlcr_solver *const *S, const int *nrhs, const double *const *b,
                         double *const *x, double rtol, int max_cycles, int prec,
                         mlcr_solve_info *info, void *stream) {
    if (nprob < 1) return fail(MLCR_EINVAL, "nprob must be >= 1");
    if (!S || !b || !x) return fail(MLCR_EINVAL, "NULL argument");
    int rc;
    std::vector<const void *> keys(nprob);
    for (int p = 0; p < nprob; p++) {
        if ((rc = check_solve_args(S[p], nrhs ? nrhs[p] : 1, b[p], x[p], rtol, max_cycles, prec)))
            return rc;
        for (int q = 0; q < p; q++)
            if (S[q] == S[p]) return fail(MLCR_EINVAL, "a solver appears twice in the group");
        keys[p] = S[p]->op->g;
    }
    StreamFork f;
    if ((rc = f.begin((hipStream_t)stream, keys))) return rc;
    std::vector<std::unique_ptr<SolveRun>> runs;
    for (int p = 0; p < nprob; p++)
        runs.emplace_back(new SolveRun(S[p], nrhs ? nrhs[p] : 1, b[p], x[p], rtol, prec,
                                       f.item_stream[p]));
    // all problems' work is enqueued before any result is read back
    for (auto &r : runs)
        if (!rc) rc = r->enqueue_start();
    for (auto &r : runs)
        if (!rc) rc = r->enqueue_start_residual();
    for (auto &r : runs)
        if (!rc) rc = r->finish_start();
    for (int c = 0; c < max_cycles && !rc; c++) {
        bool any = false;
        for (auto &r : runs)
            if (!rc && !r->all) {
                rc = r->enqueue_cycle();
                any = true;
            }
        if (!any) break;
        for (auto &r : runs)
            if (!rc && r->it == c + 1) rc = r->finish_cycle();
    }
    bool all = true;
    long long off = 0;
    for (auto &r : runs) {
        if (!rc) rc = r->finish(info ? info + off : nullptr);
        off += r->nrhs;
        all = all && r->all;
    }
    const int rj = f.join();
    if (rc) return rc;
    if (rj) return rj;
    if (!all) return fail(MLCR_ENOCONV, "rtol not reached within max_cycles (some problem)");
    return MLCR_OK;
}

// Flexible preconditioned conjugate gradients on A x = b in float64 with one
// CR-Cycle from zero (in `prec`) as the preconditioner (the alternative the
// caption of Fig. code:mg names).  beta = <r_new, z_new - z_old> / <r_old,
// z_old> (Polak-Ribiere form), which tolerates the small asymmetry a
// mixed-precision cycle has.
int pcg_solve(mlcr_solver *S, int nrhs, const double *b, double *x, double rtol, int max_iter,
              int prec, mlcr_solve_info *info, void *stream) {
    int rc;
    if ((rc = check_solve_args(S, nrhs, b, x, rtol, max_iter, prec))) return rc;
    hipStream_t s = (hipStream_t)stream;
    mlcr_op *op = S->op;
    const int lmax = op->lmax;
    const long long na = nalm_l(lmax);
    const size_t vbytes = (size_t)S->max_nrhs * na * sizeof(double);
    if (S->pcg_p.reserve(vbytes) || S->pcg_zo.reserve(vbytes) ||
        S->pcg_coef.reserve(4 * (size_t)S->max_nrhs * sizeof(double)))
        return fail(MLCR_ENOMEM, "conjugate-gradient workspace allocation failed");
    SolveRun run(S, nrhs, b, x, rtol, prec, s);
    if ((rc = run.enqueue_start()) || (rc = run.enqueue_start_residual()) ||
        (rc = run.finish_start()))
        return rc;
    double *r = S->ro.as<double>(), *q = S->to.as<double>(), *z = S->x0.as<double>();
    double *p = S->pcg_p.as<double>(), *zo = S->pcg_zo.as<double>();
    double *al = S->pcg_coef.as<double>(), *be = al + S->max_nrhs;
    std::vector<double> h(2 * nrhs), rz(nrhs, 0.0), ca(nrhs), cb(nrhs);
    const std::vector<double> ones(nrhs, 1.0);
    auto dots = [&](const double *a1, const double *b1, const double *c1, const double *d1) -> int {
        int r2;
        if ((r2 = launch_dots(a1, b1, c1, d1, lmax, nrhs, S->partial.as<double>(),
                              S->norms.as<double>(), s)))
            return r2;
        MLCR_HIP_CHECK(hipMemcpyAsync(h.data(), S->norms.ptr, 2 * nrhs * sizeof(double),
                                      hipMemcpyDeviceToHost, s));
        MLCR_HIP_CHECK(hipStreamSynchronize(s));
        return MLCR_OK;
    };
    auto coefs = [&](const std::vector<double> &a1, const std::vector<double> &b1) -> int {
        MLCR_HIP_CHECK(hipMemcpyAsync(al, a1.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, s));
        MLCR_HIP_CHECK(hipMemcpyAsync(be, b1.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, s));
        return MLCR_OK;
    };
    auto precond = [&]() -> int {     // z = M r: one cycle from zero on r
        MLCR_HIP_CHECK(hipMemcpyAsync(S->b0.ptr, r, (size_t)nrhs * na * sizeof(double),
                                      hipMemcpyDeviceToDevice, s));
        if (int r2 = launch_fill_zero(z, (long long)nrhs * na, s)) return r2;
        GpuOps ops(S, nrhs, prec, s);
        return run_schedule(ops, S->sched);
    };
    if (!run.all) {
        if ((rc = precond())) return rc;
        MLCR_HIP_CHECK(hipMemcpyAsync(p, z, (size_t)nrhs * na * sizeof(double),
                                      hipMemcpyDeviceToDevice, s));
        if ((rc = dots(r, z, nullptr, nullptr))) return rc;
        for (int k = 0; k < nrhs; k++) rz[k] = h[2 * k];
    }
    while (!run.all && run.it < max_iter) {
        // alpha = <r, z> / <p, A p>; x += alpha p; r -= alpha A p
        if ((rc = apply_level(op, 0, nrhs, p, q, MLCR_FP64, s))) return rc;
        if ((rc = dots(p, q, nullptr, nullptr))) return rc;
        for (int k = 0; k < nrhs; k++) ca[k] = (run.done[k] || !(h[2 * k] > 0)) ? 0.0 : rz[k] / h[2 * k];
        if ((rc = coefs(ca, ones))) return rc;
        if ((rc = launch_lincomb(p, x, x, al, be, na, nrhs, s))) return rc;
        for (int k = 0; k < nrhs; k++) ca[k] = -ca[k];
        if ((rc = coefs(ca, ones))) return rc;
        if ((rc = launch_lincomb(q, r, r, al, be, na, nrhs, s))) return rc;
        run.it++;
        if ((rc = launch_wnorms(r, b, S->sinv.as<double>(), lmax, nrhs, S->partial.as<double>(),
                                S->norms.as<double>(), s)))
            return rc;
        if ((rc = run.finish_cycle())) return rc;
        if (run.all) break;
        // z_new = M r; beta = <r, z_new - z_old> / <r_old, z_old>; p = z_new + beta p
        MLCR_HIP_CHECK(hipMemcpyAsync(zo, z, (size_t)nrhs * na * sizeof(double),
                                      hipMemcpyDeviceToDevice, s));
        if ((rc = precond())) return rc;
        if ((rc = dots(r, z, r, zo))) return rc;
        for (int k = 0; k < nrhs; k++) {
            cb[k] = (run.done[k] || !(rz[k] > 0)) ? 0.0 : (h[2 * k] - h[2 * k + 1]) / rz[k];
            rz[k] = h[2 * k];
        }
        if ((rc = coefs(ones, cb))) return rc;
        if ((rc = launch_lincomb(z, p, p, al, be, na, nrhs, s))) return rc;
    }
    if ((rc = run.finish(info))) return rc;
    if (!run.all) return fail(MLCR_ENOCONV, "rtol not reached within max_iter");
    return MLCR_OK;
}

int mlcr_prior_band_grad(mlcr_op *op, int nrhs, const double *lam, const double *x,
                         const int *band, int nbands, const double *q, double *out, void *stream) {
    if (!op || !lam || !x || !band || !out) return fail(MLCR_EINVAL, "NULL argument");
    if (nrhs < 1) return fail(MLCR_EINVAL, "nrhs must be >= 1");
    if (nbands < 1) return fail(MLCR_EINVAL, "nbands must be >= 1");
    const int lmax = op->lmax;
    for (int l = 0; l <= lmax; l++)
        if (band[l] < -1 || band[l] >= nbands) return fail(MLCR_EINVAL, "band index out of range");
    if (q)
        for (int k = 0; k < nbands; k++)
            if (!(q[k] > 0.0) || !std::isfinite(q[k])) return fail(MLCR_EINVAL, "q must be finite and > 0");
    hipStream_t s = (hipStream_t)stream;
    if (op->ell_ws.reserve((size_t)(lmax + 1) * sizeof(double)))
        return fail(MLCR_ENOMEM, "band-gradient workspace allocation failed");
    int rc;
    if ((rc = launch_ell_dots(lam, x, lmax, nrhs, op->ell_ws.as<double>(), s))) return rc;
    std::vector<double> per(lmax + 1);
    MLCR_HIP_CHECK(hipMemcpyAsync(per.data(), op->ell_ws.ptr, per.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
    MLCR_HIP_CHECK(hipStreamSynchronize(s));
    // dL/dq_beta = -lam^T (dA/dq_beta) x, dA/dq_beta = -S^-1 / q_beta on the band
    for (int k = 0; k < nbands; k++) out[k] = 0.0;
    for (int l = 0; l <= lmax; l++)
        if (band[l] >= 0 && op->cl[l] > 0.0) out[band[l]] += per[l] / op->cl[l];
    if (q)
        for (int k = 0; k < nbands; k++) out[k] /= q[k];
    return MLCR_OK;
}

int mlcr_cr_rhs(mlcr_op *op, int nrhs, const double *d, const double *w1, const double *w2,
                double *b, void *stream) {
    if (!op || !d || !b) return fail(MLCR_EINVAL, "NULL argument");
    if (nrhs < 1 || nrhs > op->max_nrhs) return fail(MLCR_EINVAL, "nrhs out of [1, max_nrhs]");
    hipStream_t s = (hipStream_t)stream;
    mlcr_geom *g = op->g;
    int rc;
    if (op->rhs_pix.reserve((size_t)nrhs * g->npix * sizeof(double)))
        return fail(MLCR_ENOMEM, "right-hand-side workspace allocation failed");
    double *pix = op->rhs_pix.as<double>();
    if ((rc = launch_cr_pix(d, w2, op->ninv, pix, g->npix, nrhs, s))) return rc;
    if ((rc = sht_adjoint(g, op->lmax, nrhs, pix, b, MLCR_FP64, s))) return rc;
    const mlcr_level &L = op->levels[0];
    return launch_cr_combine(b, w1, L.bh.as<double>(), L.d.as<double>(), b, op->lmax, nrhs, s);
}
