// C ABI: handles, argument checks and the sequence of launches of each
// entry point.  Every step of the computation runs in the library's HIP
// kernels; this file only validates, sizes workspaces and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>

#include "mlcr_internal.h"
#include "solver_internal.h"

namespace mlcr {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int DevBuf::reserve(size_t nbytes) {
    if (nbytes <= bytes && ptr) return MLCR_OK;
    if (ptr) {
        // a previous launch may still read the old buffer
        (void)hipDeviceSynchronize();
        (void)hipFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
    if (nbytes == 0) nbytes = 16;
    if (hipMalloc(&ptr, nbytes) != hipSuccess) {
        ptr = nullptr;
        return MLCR_ENOMEM;
    }
    bytes = nbytes;
    return MLCR_OK;
}

// Waits for the device first: a launch still queued may read the buffer
// (an owner can go out of scope right after enqueueing work on it).  Never
// called inside a captured region: buffers are made and dropped outside.
void DevBuf::release() {
    if (ptr) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
}

// (kernels already raised are remembered in a fixed table: no heap use, so
// the entry points that must not allocate can launch through here)
int ensure_dynamic_lds(const void *func, size_t bytes) {
    if (bytes <= 64 * 1024) return MLCR_OK;
    static std::pair<const void *, size_t> done[64];
    static int ndone = 0;
    for (int i = 0; i < ndone; i++)
        if (done[i].first == func && done[i].second >= bytes) return MLCR_OK;
    MLCR_HIP_CHECK(hipFuncSetAttribute(func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    if (ndone < 64) done[ndone++] = {func, bytes};
    return MLCR_OK;
}

static void release_geom(mlcr_geom *g) {
    DevBuf *bufs[] = {&g->ring_z, &g->ring_s, &g->ring_w, &g->rings, &g->lens, &g->order, &g->T, &g->Bf,
                      &g->W, &g->Bf32, &g->W32, &g->ab, &g->alpha, &g->cfac, &g->aboff, &g->seed, &g->zeros, &g->wsF, &g->wsP,
                      &g->wsU};
    for (DevBuf *b : bufs) b->release();
    for (SegTable &t : g->seg) {
        t.st.release();
        t.sc.release();
        t.ls.release();
    }
    g->seg.clear();
}

// Pixel kernels read maps and N^-1 ring by ring as 16-byte pairs.
static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

static long long nalm_of(int lmax) { return (long long)(lmax + 1) * (lmax + 1); }

// Workspaces of one transform of nrhs right-hand sides at band limit lmax.
static int reserve_ws(mlcr_geom *g, int lmax, int nrhs) {
    const size_t fbytes = (size_t)nrhs * g->nrings * (lmax + 1) * sizeof(double2);
    int mchunks = 0;                    // most matrix-core chunks of any path's tuning
    for (int p = 0; p < 3; p++) mchunks = std::max(mchunks, adjoint_chunks_mfma(g, lmax, p));
    const size_t pbytes =
        std::max((size_t)adjoint_chunks(g, lmax) * tlayout_doubles(lmax, nrhs, adj_rc(nrhs)),
                 (size_t)mchunks * tlayout_doubles(lmax, nrhs, 8)) *
        sizeof(double);
    const size_t ubytes =
        std::max((size_t)tlayout_doubles(lmax, nrhs, synth_rc(nrhs)) * sizeof(double),
                 (size_t)seg_u_bytes(lmax, nrhs, MLCR_FP64));
    if (g->wsF.reserve(fbytes)) return fail(MLCR_ENOMEM, "workspace allocation failed (F)");
    if (g->wsP.reserve(pbytes)) return fail(MLCR_ENOMEM, "workspace allocation failed (P)");
    if (g->wsU.reserve(ubytes)) return fail(MLCR_ENOMEM, "workspace allocation failed (U)");
    return MLCR_OK;
}

// ---------------------------------------------------------------------------
// optional per-kernel timing with HIP events on the launch stream
// ---------------------------------------------------------------------------
struct TimingRec {
    const char *name;
    hipEvent_t a, b;
};
static std::vector<TimingRec> g_pending;
static std::vector<std::pair<std::string, std::pair<double, long long>>> g_acc;
static bool g_timing = false;

struct KTimer {
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    KTimer(const char *n, hipStream_t st) : name(n), s(st) {
        if (!g_timing) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, s);
    }
    ~KTimer() {
        if (!a) return;
        (void)hipEventRecord(b, s);
        g_pending.push_back({name, a, b});
    }
};

static void drain_timing() {
    for (auto &t : g_pending) {
        float ms = 0.f;
        (void)hipEventSynchronize(t.b);
        (void)hipEventElapsedTime(&ms, t.a, t.b);
        bool found = false;
        for (auto &e : g_acc)
            if (e.first == t.name) {
                e.second.first += ms;
                e.second.second += 1;
                found = true;
            }
        if (!found) g_acc.push_back({t.name, {(double)ms, 1}});
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    g_pending.clear();
}

static int check_prec(int prec) {
    if (prec == MLCR_FP64 || prec == MLCR_FP32 || prec == MLCR_BF16X3) return MLCR_OK;
    return fail(MLCR_EINVAL, "unknown precision");
}

// Legendre step dispatch on the arithmetic of the contraction
// Float64 uses the matrix cores once a launch carries enough RHS to fill
// their 16 columns (8 RHS x cos/sin) at least half; below that the per-lane
// vector kernels do less work.
static constexpr int kMfmaF64MinRhs = 4;

static bool use_mfma(int prec, int nrhs) {
    return prec != MLCR_FP64 || nrhs >= kMfmaF64MinRhs;
}

// F: complex float64 on the float64 path, complex float32 on the mixed paths
static int legendre_synth_any(const LegendreArgs &a, const double *x, const double *dl, mlcr_geom *g,
                              void *F, int prec) {
    int rc;
    if (use_mfma(prec, a.nrhs)) {
        const SegTable *st = nullptr;
        if ((rc = seg_table(g, a.lmax, a.stream, &st))) return rc;
        void *U = g->wsU.ptr;
        {
            KTimer t("pack", a.stream);
            if ((rc = launch_pack_seg(a.g, a.lmax, a.nrhs, x, dl, U, prec, a.stream))) return rc;
        }
        KTimer t("legendre_synth", a.stream);
        return launch_legendre_synth_seg(a, st, U, F, prec);
    }
    double *U = g->wsU.as<double>();
    {
        KTimer t("pack", a.stream);
        if ((rc = launch_pack_t(a.lmax, a.nrhs, synth_rc(a.nrhs), x, dl, U, a.stream))) return rc;
    }
    KTimer t("legendre_synth", a.stream);
    return launch_legendre_synth(a, U, static_cast<double2 *>(F));
}

static int legendre_adjoint_any(const LegendreArgs &a, const void *G, mlcr_geom *g,
                                const double *x, const double *d, const double *bh, double *y,
                                int prec) {
    int rc, nch = 0;
    double *P = g->wsP.as<double>();
    const bool mm = use_mfma(prec, a.nrhs);
    const SegTable *st = nullptr;
    if (mm && (rc = seg_table(g, a.lmax, a.stream, &st))) return rc;
    {
        KTimer t("legendre_adjoint", a.stream);
        if (prec == MLCR_BF16X3)
            rc = launch_legendre_adjoint_b3(a, st, static_cast<const float2 *>(G), (float *)P, &nch);
        else if (mm) rc = launch_legendre_adjoint_mfma(a, st, G, P, &nch, prec == MLCR_FP64);
        else rc = launch_legendre_adjoint(a, static_cast<const double2 *>(G), P, &nch);
        if (rc) return rc;
    }
    KTimer t("unpack", a.stream);
    // the matrix-core adjoints of the mixed paths store float32 partial sums
    return launch_unpack_t(a.lmax, a.nrhs, mm ? 8 : adj_rc(a.nrhs), nch, P,
                           mm && prec != MLCR_FP64, mm ? a.g->cfac.as<double>() : nullptr,
                           a.g->lmax, x, d, bh, y, a.stream);
}

}  // namespace mlcr

namespace mlcr {

int apply_level(mlcr_op *op, int level, int nrhs, const double *x, double *y, int prec,
                hipStream_t s) {
    if (!op || !x || !y) return fail(MLCR_EINVAL, "NULL argument");
    if (level < 0 || level >= 16 || op->levels[level].lmax < 0)
        return fail(MLCR_EINVAL, "level not defined");
    return apply_level_on(op, op->levels[level], nrhs, x, y, prec, s);
}

int apply_level_on(mlcr_op *op, const mlcr_level &L, int nrhs, const double *x, double *y,
                   int prec, hipStream_t s) {
    if (!op || !x || !y) return fail(MLCR_EINVAL, "NULL argument");
    if (x == y) return fail(MLCR_EINVAL, "x and y must not alias");
    if (L.lmax < 0) return fail(MLCR_EINVAL, "level not defined");
    if (nrhs < 1) return fail(MLCR_EINVAL, "nrhs must be >= 1");
    int rc;
    if ((rc = check_prec(prec))) return rc;
    mlcr_geom *g = L.gl ? L.gl : op->g;
    const double *ninv = L.gl ? L.gninv.as<double>() : op->ninv;
    const int lmax = L.lmax;
    if ((rc = reserve_ws(g, lmax, nrhs))) return rc;
    void *F = g->wsF.ptr;
    LegendreArgs a{g, lmax, nrhs, s};
    if ((rc = legendre_synth_any(a, x, L.bh.as<double>(), g, F, prec))) return rc;
    {
        KTimer t("ring_apply", s);
        if ((rc = launch_ring_apply(g, lmax, nrhs, F, ninv, prec, s))) return rc;
    }
    if ((rc = legendre_adjoint_any(a, F, g, x, L.d.as<double>(), L.bh.as<double>(), y, prec)))
        return rc;
    return MLCR_OK;
}

}  // namespace mlcr

using namespace mlcr;

extern "C" {

const char *mlcr_last_error(void) { return g_err.c_str(); }
const char *mlcr_version(void) { return "mlcr 0.1 (gfx950)"; }

int mlcr_timing_enable(int on) {
    drain_timing();
    g_timing = on != 0;
    return MLCR_OK;
}

int mlcr_timing_reset(void) {
    drain_timing();
    g_acc.clear();
    return MLCR_OK;
}

int mlcr_timing_count(void) {
    drain_timing();
    return (int)g_acc.size();
}

int mlcr_timing_get(int i, char *name, int name_len, double *total_ms, long long *calls) {
    drain_timing();
    if (i < 0 || i >= (int)g_acc.size() || !name || name_len < 1)
        return fail(MLCR_EINVAL, "bad timing index or buffer");
    std::strncpy(name, g_acc[i].first.c_str(), (size_t)name_len - 1);
    name[name_len - 1] = 0;
    if (total_ms) *total_ms = g_acc[i].second.first;
    if (calls) *calls = g_acc[i].second.second;
    return MLCR_OK;
}

int mlcr_geom_create(int nside, int lmax, mlcr_geom **out) {
    if (!out) return fail(MLCR_EINVAL, "out is NULL");
    *out = nullptr;
    if (nside < 1 || nside > 2048)
        return fail(MLCR_EINVAL, "nside must be in [1, 2048] (ring FFT buffers must fit in LDS)");
    if (lmax < 0 || lmax > 16384) return fail(MLCR_EINVAL, "lmax must be in [0, 16384]");
    mlcr_geom *g = new (std::nothrow) mlcr_geom();
    if (!g) return fail(MLCR_ENOMEM, "host allocation failed");
    int rc = build_geometry(g, nside, lmax);
    if (rc) {
        release_geom(g);
        delete g;
        return rc;
    }
    *out = g;
    g_err.clear();
    return MLCR_OK;
}

int mlcr_geom_create_gl(int lmax, int nrings, int nphi, mlcr_geom **out) {
    if (!out) return fail(MLCR_EINVAL, "out is NULL");
    *out = nullptr;
    if (lmax < 0 || lmax > 16384) return fail(MLCR_EINVAL, "lmax must be in [0, 16384]");
    if (nrings < 1 || nrings > 32768) return fail(MLCR_EINVAL, "nrings must be in [1, 32768]");
    if (nphi < 4 || nphi % 4 || nphi > 8192 * 2)
        return fail(MLCR_EINVAL, "nphi must be a multiple of 4 in [4, 16384]");
    {
        // ring FFT buffers must fit in LDS: n = nphi/2 itself, or Bluestein size
        int n = nphi / 2, M = 1;
        while (M < n) M <<= 1;
        if (M != n) {
            M = 1;
            while (M < 2 * n - 1) M <<= 1;
        }
        if (M > 8192) return fail(MLCR_EINVAL, "nphi needs an FFT larger than 8192 points");
    }
    mlcr_geom *g = new (std::nothrow) mlcr_geom();
    if (!g) return fail(MLCR_ENOMEM, "host allocation failed");
    int rc = build_geometry_gl(g, lmax, nrings, nphi);
    if (rc) {
        release_geom(g);
        delete g;
        return rc;
    }
    *out = g;
    g_err.clear();
    return MLCR_OK;
}

int mlcr_geom_weights(const mlcr_geom *g, double *w) {
    if (!g || !w) return fail(MLCR_EINVAL, "NULL argument");
    std::copy(g->ring_w_host.begin(), g->ring_w_host.end(), w);
    return MLCR_OK;
}

void mlcr_geom_destroy(mlcr_geom *g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    release_geom(g);
    delete g;
}

int mlcr_geom_info(const mlcr_geom *g, int *nside, int *lmax, long long *npix, int *nrings) {
    if (!g) return fail(MLCR_EINVAL, "geometry is NULL");
    if (nside) *nside = g->nside;
    if (lmax) *lmax = g->lmax;
    if (npix) *npix = g->npix;
    if (nrings) *nrings = g->nrings;
    return MLCR_OK;
}

int mlcr_geom_set_tuning(mlcr_geom *g, int prec, int adjoint_waves, int synth_chains,
                         int ring_threads) {
    if (!g) return fail(MLCR_EINVAL, "geometry is NULL");
    int rc;
    if ((rc = check_prec(prec))) return rc;
    if (adjoint_waves != 4 && adjoint_waves != 8)
        return fail(MLCR_EINVAL, "adjoint_waves must be 4 or 8");
    if (synth_chains != 2 && synth_chains != 4)
        return fail(MLCR_EINVAL, "synth_chains must be 2 or 4");
    if (ring_threads != 512 && ring_threads != 1024)
        return fail(MLCR_EINVAL, "ring_threads must be 512 or 1024");
    Tuning &t = g->tune[prec];
    t.adj_waves = adjoint_waves;
    t.synth_chains = synth_chains;
    t.ring_threads = ring_threads;
    return MLCR_OK;
}

int mlcr_geom_get_tuning(const mlcr_geom *g, int prec, int *adjoint_waves, int *synth_chains,
                         int *ring_threads) {
    if (!g) return fail(MLCR_EINVAL, "geometry is NULL");
    int rc;
    if ((rc = check_prec(prec))) return rc;
    const Tuning &t = g->tune[prec];
    if (adjoint_waves) *adjoint_waves = t.adj_waves;
    if (synth_chains) *synth_chains = t.synth_chains;
    if (ring_threads) *ring_threads = t.ring_threads;
    return MLCR_OK;
}

int sht_synth(mlcr_geom *g, int lmax, int nrhs, const double *alm, double *map, int prec,
              void *stream) {
    if (!g || !alm || !map) return fail(MLCR_EINVAL, "NULL argument");
    if (!aligned16(map)) return fail(MLCR_EINVAL, "map must be 16-byte aligned");
    if (lmax < 0 || lmax > g->lmax) return fail(MLCR_EINVAL, "lmax exceeds the geometry's lmax");
    if (nrhs < 1) return fail(MLCR_EINVAL, "nrhs must be >= 1");
    int rc;
    if ((rc = check_prec(prec))) return rc;
    if ((rc = reserve_ws(g, lmax, nrhs))) return rc;
    hipStream_t s = (hipStream_t)stream;
    LegendreArgs a{g, lmax, nrhs, s};
    void *F = g->wsF.ptr;
    if ((rc = legendre_synth_any(a, alm, nullptr, g, F, prec))) return rc;
    {
        KTimer t("ring_synth", s);
        if ((rc = launch_ring_synth(g, lmax, nrhs, F, map, prec, s))) return rc;
    }
    return MLCR_OK;
}

int sht_adjoint(mlcr_geom *g, int lmax, int nrhs, const double *map, double *alm, int prec,
                void *stream) {
    if (!g || !alm || !map) return fail(MLCR_EINVAL, "NULL argument");
    if (!aligned16(map)) return fail(MLCR_EINVAL, "map must be 16-byte aligned");
    if (lmax < 0 || lmax > g->lmax) return fail(MLCR_EINVAL, "lmax exceeds the geometry's lmax");
    if (nrhs < 1) return fail(MLCR_EINVAL, "nrhs must be >= 1");
    int rc;
    if ((rc = check_prec(prec))) return rc;
    if ((rc = reserve_ws(g, lmax, nrhs))) return rc;
    hipStream_t s = (hipStream_t)stream;
    LegendreArgs a{g, lmax, nrhs, s};
    void *G = g->wsF.ptr;
    {
        KTimer t("ring_adjoint", s);
        if ((rc = launch_ring_adjoint(g, lmax, nrhs, map, G, prec, s))) return rc;
    }
    if ((rc = legendre_adjoint_any(a, G, g, nullptr, nullptr, nullptr, alm, prec))) return rc;
    return MLCR_OK;
}

// ---------------------------------------------------------------------------
// operator
// ---------------------------------------------------------------------------
static void drop_gl(mlcr_level &L) {
    if (L.gl) {
        (void)hipDeviceSynchronize();
        mlcr_geom_destroy(L.gl);
        L.gl = nullptr;
    }
    L.gninv.release();
}

// d = f^2 / C_l and bh = f b_l of a level (0 on excluded modes), from its
// stored filter
static int level_tables(mlcr_level &L, int lmax_h, const std::vector<double> &cl,
                        const std::vector<double> &bl) {
    const double *fl = L.fl.empty() ? nullptr : L.fl.data();
    std::vector<double> d(lmax_h + 1), bh(lmax_h + 1);
    for (int l = 0; l <= lmax_h; l++) {
        const double f = fl ? fl[l] : 1.0;
        if (cl[l] > 0.0) {
            d[l] = f * f / cl[l];
            bh[l] = f * bl[l];
        } else {
            d[l] = 0.0;
            bh[l] = 0.0;
        }
    }
    if (L.d.reserve(d.size() * sizeof(double)) || L.bh.reserve(bh.size() * sizeof(double)))
        return fail(MLCR_ENOMEM, "level table allocation failed");
    MLCR_HIP_CHECK(hipMemcpy(L.d.ptr, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice));
    MLCR_HIP_CHECK(hipMemcpy(L.bh.ptr, bh.data(), bh.size() * sizeof(double), hipMemcpyHostToDevice));
    return MLCR_OK;
}

static int upload_level(mlcr_level &L, int lmax_h, const std::vector<double> &cl,
                        const std::vector<double> &bl, const double *fl) {
    drop_gl(L);
    if (fl) L.fl.assign(fl, fl + lmax_h + 1);
    else L.fl.clear();
    int rc = level_tables(L, lmax_h, cl, bl);
    if (rc) return rc;
    L.lmax = lmax_h;
    return MLCR_OK;
}

}  // extern "C"

// Level h with a caller-chosen prior spectrum (the solver's hierarchy).
extern "C" {

int mlcr_op_create(mlcr_geom *g, int lmax, const double *cl, const double *bl, const double *ninv,
                   int max_nrhs, mlcr_op **out) {
    if (!out) return fail(MLCR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g || !cl || !bl || !ninv) return fail(MLCR_EINVAL, "NULL argument");
    if (!aligned16(ninv)) return fail(MLCR_EINVAL, "ninv must be 16-byte aligned");
    if (lmax < 0 || lmax > g->lmax) return fail(MLCR_EINVAL, "lmax exceeds the geometry's lmax");
    if (max_nrhs < 1) return fail(MLCR_EINVAL, "max_nrhs must be >= 1");
    for (int l = 0; l <= lmax; l++) {
        if (!(cl[l] >= 0.0) || !std::isfinite(cl[l]))
            return fail(MLCR_EINVAL, "C_l must be finite and >= 0");
        if (!std::isfinite(bl[l])) return fail(MLCR_EINVAL, "b_l must be finite");
    }
    mlcr_op *op = new (std::nothrow) mlcr_op();
    if (!op) return fail(MLCR_ENOMEM, "host allocation failed");
    op->g = g;
    op->lmax = lmax;
    op->max_nrhs = max_nrhs;
    op->ninv = ninv;
    op->cl.assign(cl, cl + lmax + 1);
    op->bl.assign(bl, bl + lmax + 1);
    int rc = upload_level(op->levels[0], lmax, op->cl, op->bl, nullptr);
    if (!rc) rc = reserve_ws(g, lmax, max_nrhs);
    if (rc) {
        mlcr_op_destroy(op);
        return rc;
    }
    *out = op;
    return MLCR_OK;
}

void mlcr_op_destroy(mlcr_op *op) {
    if (!op) return;
    (void)hipDeviceSynchronize();
    for (auto &L : op->levels) {
        drop_gl(L);
        L.d.release();
        L.bh.release();
    }
    op->rhs_pix.release();
    delete op;
}

int mlcr_op_set_level(mlcr_op *op, int h, int lmax_h, const double *fl) {
    if (!op || !fl) return fail(MLCR_EINVAL, "NULL argument");
    if (h < 1 || h >= 16) return fail(MLCR_EINVAL, "level index must be in [1, 15]");
    if (lmax_h < 0 || lmax_h > op->lmax) return fail(MLCR_EINVAL, "lmax_h out of range");
    for (int l = 0; l <= lmax_h; l++)
        if (!std::isfinite(fl[l])) return fail(MLCR_EINVAL, "filter must be finite");
    return upload_level(op->levels[h], lmax_h, op->cl, op->bl, fl);
}

int mlcr_op_set_level_gl(mlcr_op *op, int h, int lmax_h, const double *fl) {
    if (!op || !fl) return fail(MLCR_EINVAL, "NULL argument");
    if (h < 1 || h >= 16) return fail(MLCR_EINVAL, "level index must be in [1, 15]");
    if (lmax_h < 0 || lmax_h > op->lmax) return fail(MLCR_EINVAL, "lmax_h out of range");
    return define_level(op, op->levels[h], lmax_h, fl, true);
}

}  // extern "C"

namespace mlcr {

void release_level(mlcr_level &L) {
    drop_gl(L);
    L.d.release();
    L.bh.release();
    L.fl.clear();
    L.lmax = -1;
}

int refresh_level(mlcr_op *op, mlcr_level &L) {
    return L.lmax >= 0 ? level_tables(L, L.lmax, op->cl, op->bl) : MLCR_OK;
}

// Level tables of band limit lmax_h and filter fl into L (f = 1 if fl is
// NULL); with gl, Y^T N^-1 Y of the level on a Gauss-Legendre grid.
int define_level(mlcr_op *op, mlcr_level &L, int lmax_h, const double *fl, bool gl) {
    if (lmax_h < 0 || lmax_h > op->lmax) return fail(MLCR_EINVAL, "lmax_h out of range");
    for (int l = 0; fl && l <= lmax_h; l++)
        if (!std::isfinite(fl[l])) return fail(MLCR_EINVAL, "filter must be finite");
    if (!gl) return upload_level(L, lmax_h, op->cl, op->bl, fl);
    const int lx = 2 * lmax_h;            // band limit of the downgraded N^-1
    if (lx > op->g->lmax)
        return fail(MLCR_EINVAL, "2 lmax_h exceeds the observation geometry's lmax");
    int nphi = 4;
    while (nphi < 4 * lmax_h + 1) nphi <<= 1;
    if (nphi > 16384) return fail(MLCR_EINVAL, "lmax_h too large for a Gauss-Legendre level");
    int rc = upload_level(L, lmax_h, op->cl, op->bl, fl);
    if (rc) return rc;
    mlcr_geom *gg = nullptr;
    if ((rc = mlcr_geom_create_gl(lx, 2 * lmax_h + 1, nphi, &gg))) return rc;
    L.gl = gg;
    // xi = Y_obs^T N^-1 (Sec. 3.4): every coupling of Y_obs^T N^-1 Y_obs between
    // modes l, l' <= lmax_h sees only xi_LM with L <= 2 lmax_h; synthesized on
    // the Gauss-Legendre grid and weighted by its quadrature, it reproduces
    // those couplings exactly (up to rounding)
    DevBuf xi, map;
    const long long nx = (long long)(lx + 1) * (lx + 1);
    if (xi.reserve((size_t)nx * sizeof(double)) || map.reserve((size_t)gg->npix * sizeof(double)) ||
        L.gninv.reserve((size_t)gg->npix * sizeof(double)))
        return fail(MLCR_ENOMEM, "Gauss-Legendre level allocation failed");
    if ((rc = sht_adjoint(op->g, lx, 1, op->ninv, xi.as<double>(), MLCR_FP64, nullptr))) return rc;
    if ((rc = sht_synth(gg, lx, 1, xi.as<double>(), map.as<double>(), MLCR_FP64, nullptr))) return rc;
    if ((rc = launch_ring_weight(gg, map.as<double>(), L.gninv.as<double>(), nullptr))) return rc;
    MLCR_HIP_CHECK(hipDeviceSynchronize());
    return MLCR_OK;
}

}  // namespace mlcr

extern "C" {

int mlcr_op_set_prior(mlcr_op *op, const double *cl) {
    if (!op || !cl) return fail(MLCR_EINVAL, "NULL argument");
    for (int l = 0; l <= op->lmax; l++) {
        if (!std::isfinite(cl[l]) || cl[l] < 0.0) return fail(MLCR_EINVAL, "C_l must be finite and >= 0");
        if ((cl[l] > 0.0) != (op->cl[l] > 0.0))
            return fail(MLCR_EINVAL, "the new C_l must be > 0 exactly where the current one is (l = " +
                                         std::to_string(l) + ")");
    }
    MLCR_HIP_CHECK(hipDeviceSynchronize());      // queued applies may read the level tables
    op->cl.assign(cl, cl + op->lmax + 1);
    for (auto &L : op->levels)
        if (L.lmax >= 0) {
            int rc = level_tables(L, L.lmax, op->cl, op->bl);
            if (rc) return rc;
        }
    op->prior_version++;
    return MLCR_OK;
}

int mlcr_op_level_lmax(const mlcr_op *op, int h) {
    if (!op || h < 0 || h >= 16) return fail(MLCR_EINVAL, "bad operator or level");
    if (op->levels[h].lmax < 0) return fail(MLCR_EINVAL, "level not defined");
    return op->levels[h].lmax;
}

int apply_A(mlcr_op *op, int level, int nrhs, const double *x, double *y, int prec, void *stream) {
    if (!op || !x || !y) return fail(MLCR_EINVAL, "NULL argument");
    if (nrhs < 1 || nrhs > op->max_nrhs) return fail(MLCR_EINVAL, "nrhs out of [1, max_nrhs]");
    return apply_level(op, level, nrhs, x, y, prec, (hipStream_t)stream);
}

int apply_A_grouped(int nprob, mlcr_op *const *ops, const int *nrhs, const double *const *x,
                    double *const *y, int prec, void *stream) {
    if (nprob < 1) return fail(MLCR_EINVAL, "nprob must be >= 1");
    if (!ops || !x || !y) return fail(MLCR_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_prec(prec))) return rc;
    std::vector<const void *> keys(nprob);
    for (int p = 0; p < nprob; p++) {
        if (!ops[p] || !x[p] || !y[p]) return fail(MLCR_EINVAL, "NULL operator or vector in the group");
        if (nrhs && nrhs[p] < 1) return fail(MLCR_EINVAL, "nrhs must be >= 1");
        keys[p] = ops[p]->g;
    }
    StreamFork f;
    if ((rc = f.begin((hipStream_t)stream, keys))) return rc;
    for (int p = 0; p < nprob && rc == MLCR_OK; p++)
        rc = apply_level(ops[p], 0, nrhs ? nrhs[p] : 1, x[p], y[p], prec, f.item_stream[p]);
    const int rj = f.join();
    return rc ? rc : rj;
}

}  // extern "C"
