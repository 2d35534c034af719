// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mlcr.h"

namespace mlcr {

// ---------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define MLCR_HIP_CHECK(expr)                                                       \
    do {                                                                           \
        hipError_t _e = (expr);                                                    \
        if (_e != hipSuccess)                                                      \
            return ::mlcr::fail(MLCR_EHIP, std::string(#expr) + ": " +            \
                                               hipGetErrorString(_e));             \
    } while (0)

// ---------------------------------------------------------------------------
// device buffer with grow-on-demand semantics
// ---------------------------------------------------------------------------
// Owns one device allocation (released when the owner goes away); movable,
// not copyable.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes) {
        o.ptr = nullptr;
        o.bytes = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            ptr = o.ptr;
            bytes = o.bytes;
            o.ptr = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    int reserve(size_t nbytes);     // MLCR_OK or MLCR_ENOMEM
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Per-ring information used by the ring (FFT) kernels.
struct RingInfo {
    long long start;    // RING index of the first pixel
    int nphi;           // pixels in the ring, N = 4 i
    int phase;          // p: e^{i m phi0} = e^{i pi m p / N}
    int tab;            // index i - 1 of the length class N = 4 i
    int pad;
};

// Offset of the cosine block of order m >= 1 in a real packed vector
// (the m = 0 block starts at 0).
__host__ __device__ inline long long cos_base(int m, int lmax) {
    return m == 0 ? 0 : (long long)(lmax + 1) + (long long)(m - 1) * (2 * lmax - m + 2);
}

// Per length class N = 4 i (i = 1..nside): twiddle table and Bluestein filter.
struct LenInfo {
    long long toff;     // offset of T_N[j] = e^{i pi j / N}, j = 0..2N-1
    long long boff;     // offset of the Bluestein filter (-1: n = N/2 is a power of two)
    int M;              // Bluestein FFT size (power of two >= 2n - 1), or n when pow2
    int pad;
};

// rings order[off .. off+count) share one ring-kernel launch; mmax = largest FFT size
struct RingGroup {
    int off, count, mmax;
    int nmin;           // smallest ring length N in the group
};

// Recurrence start states of the matrix-core Legendre kernels at one band
// limit: per order m and block of 16 ring pairs, the offset ls (from m, a
// multiple of 32, the same for the 64 ring pairs of a wave) below which every
// lambda of those ring pairs is negligible, and for each of the 4 l-segments
// of [m + ls, lmax] the recurrence state (l1, l2, scale count) of each ring
// pair at the segment start (segment 0 starts at ls: the adjoint's start).
struct SegTable {
    int lmax = -1;
    DevBuf st;          // double2 [(lmax+1) * nb16 * 64]
    DevBuf sc;          // int     [(lmax+1) * nb16 * 64]
    DevBuf ls;          // int     [(lmax+1) * nb16]
};

// Launch shapes of the transform kernels, one set per arithmetic path
// (index MLCR_FP64 / MLCR_FP32 / MLCR_BF16X3), chosen by the caller (the
// autotuner) through mlcr_geom_set_tuning.  Results do not depend on them
// beyond rounding order.
struct Tuning {
    int adj_waves = 8;        // ring-pair blocks (waves) per matrix-core adjoint workgroup: 4, 8
    int synth_chains = 4;     // recurrence chains per lane, segment synthesis: 2, 4
    int ring_threads = 1024;  // threads per ring workgroup, FFT size above 4096: 512, 1024
};

}  // namespace mlcr

struct mlcr_geom {
    int kind = 0;           // 0: HEALPix RING grid; 1: Gauss-Legendre grid
    int nside = 0, lmax = 0, nrings = 0, npairs = 0;
    long long npix = 0;
    int lds_cplx = 0;       // largest complex FFT buffer of any ring
    int Wmax = 0;           // size of the power-of-two twiddle table
    mlcr::Tuning tune[3];   // launch shapes per arithmetic path

    // device tables
    mlcr::DevBuf ring_z, ring_s;        // per ring: cos, sin theta (double)
    mlcr::DevBuf ring_w;                // per ring: quadrature weight per pixel (double)
    mlcr::DevBuf rings;                 // RingInfo[nrings]
    mlcr::DevBuf lens;                  // LenInfo[nside]
    mlcr::DevBuf order;                 // int[nrings]: rings by FFT size group, then cost
    std::vector<mlcr::RingGroup> ring_groups;   // host: launch groups over order
    std::vector<double> ring_w_host;            // host: quadrature weight per pixel of each ring
    mlcr::DevBuf T;                     // double2, all twiddle tables
    mlcr::DevBuf Bf;                    // double2, all Bluestein filters
    mlcr::DevBuf W;                     // double2, e^{-2 pi i j / Wmax}, j < Wmax
    mlcr::DevBuf Bf32, W32;             // float2 copies of Bf and W (float32 operator FFTs)
    mlcr::DevBuf ab;                    // double2 (A_lm, B_lm) recurrence coefficients
    mlcr::DevBuf alpha;                 // double alpha_lm (same index as ab): mu recurrence
    mlcr::DevBuf cfac;                  // double c_lm, [tri_off(m) + l - m] for this lmax
    mlcr::DevBuf aboff;                 // long long per m
    mlcr::DevBuf seed;                  // double per m: seed constant of lambda_mm
    mlcr::DevBuf zeros;                 // double[lmax+1] of zeros (absent sine block of m = 0)

    // workspaces, grown on demand
    mlcr::DevBuf wsF;                   // ring-major Fourier coefficients
    mlcr::DevBuf wsP;                   // partial adjoint sums
    mlcr::DevBuf wsU;                   // beam-weighted input
    std::vector<mlcr::SegTable> seg;    // synthesis start states, one per band limit used
};

struct mlcr_level {
    int lmax = -1;
    std::vector<double> fl;     // host: the level's filter (empty: f = 1)
    mlcr::DevBuf d;     // double[lmax+1]: f^2 / C_l (0 for excluded modes)
    mlcr::DevBuf bh;    // double[lmax+1]: f b_l p_l (0 for excluded modes)
    // optional Gauss-Legendre evaluation of Y^T N^-1 Y (owned): the grid and
    // the quadrature-weighted downgraded inverse noise on it
    mlcr_geom *gl = nullptr;
    mlcr::DevBuf gninv;
};

struct mlcr_op {
    mlcr_geom *g = nullptr;
    int lmax = 0, max_nrhs = 0;
    const double *ninv = nullptr;
    std::vector<double> cl, bl;
    int prior_version = 0;  // bumped by mlcr_op_set_prior
    mlcr::DevBuf rhs_pix;   // workspace of mlcr_cr_rhs
    mlcr::DevBuf ell_ws;    // workspace of mlcr_prior_band_grad
    mlcr_level levels[16];
};

namespace mlcr {

// Independent work items on pooled streams (streams.cpp): items with the same
// key (the grid whose workspaces they use) share a stream.
struct StreamFork {
    hipStream_t parent = nullptr;
    std::vector<hipStream_t> item_stream;   // per item
    std::vector<hipStream_t> used;
    int begin(hipStream_t parent, const std::vector<const void *> &keys);
    int join();
};

// Raise a kernel's dynamic LDS limit to `bytes` when it exceeds the 64 KiB
// default (gfx950 allows up to 160 KiB per workgroup, static plus dynamic).
int ensure_dynamic_lds(const void *func, size_t bytes);

// geometry.cpp
int build_geometry(mlcr_geom *g, int nside, int lmax);
int build_geometry_gl(mlcr_geom *g, int lmax, int nrings, int nphi);

// launch wrappers (kernels.hip)
struct LegendreArgs {
    const mlcr_geom *g;
    int lmax;        // band limit of this transform (<= g->lmax)
    int nrhs;
    hipStream_t stream;
};
int launch_legendre_synth(const LegendreArgs &a, const double *u, double2 *F);
int launch_legendre_adjoint(const LegendreArgs &a, const double2 *G, double *P, int *nchunks_out);
// The Fourier coefficients F and G ([RHS][ring][m]) are complex float64
// (double2) on the float64 path and complex float32 (float2) on the mixed
// paths, whose ring FFTs run in float32 (as launch_ring_apply).
int launch_ring_synth(const mlcr_geom *g, int lmax, int nrhs, const void *F, double *map,
                      int prec, hipStream_t s);
int launch_ring_adjoint(const mlcr_geom *g, int lmax, int nrhs, const double *map, void *G,
                        int prec, hipStream_t s);
// prec: the arithmetic path; its FFTs run in float32 (LDS buffer and
// Bluestein filter) on the mixed paths, fold/unfold in float64 always
int launch_ring_apply(const mlcr_geom *g, int lmax, int nrhs, void *FG, const double *ninv,
                      int prec, hipStream_t s);
// out[p] = W_ring(p) in[p]: a map times the grid's quadrature weights
int launch_ring_weight(const mlcr_geom *g, const double *in, double *out, hipStream_t s);
int adjoint_chunks(const mlcr_geom *g, int lmax);
// matrix-core Legendre adjoint, 8 RHS per wave; dbl selects float64 MFMA
// (else float32).
// P holds float64 partial sums for dbl, float32 otherwise; G is double2 for
// dbl, float2 otherwise
int launch_legendre_adjoint_mfma(const LegendreArgs &a, const SegTable *st, const void *G,
                                 void *P, int *nchunks_out, bool dbl);
int adjoint_chunks_mfma(const mlcr_geom *g, int lmax, int prec);
int adjoint_waves(const mlcr_geom *g, int prec);
// split-bfloat16 matrix-core adjoint (legendre_b3.hip): P as for the float32 adjoint.
// segment-parallel synthesis (legendre_seg.hip); prec: MLCR_FP32 / FP64 / BF16X3
long long seg_u_bytes(int lmax, int nrhs, int prec);
// column blocks of 16 (8 RHS) per wave of the split-bfloat16 kernels: 2 from
// 16 RHS on (one lambda feeds both), else 1
int bf16_synth_cols(int nrhs);
int seg_table(mlcr_geom *g, int lmax, hipStream_t s, const SegTable **out);
int launch_pack_seg(const mlcr_geom *g, int lmax, int nrhs, const double *x, const double *dl,
                    void *U, int prec, hipStream_t s);
// F: double2 for MLCR_FP64, float2 for the mixed paths
int launch_legendre_synth_seg(const LegendreArgs &a, const SegTable *t, const void *U, void *F,
                              int prec);
int launch_legendre_adjoint_b3(const LegendreArgs &a, const SegTable *st, const float2 *G,
                               float *P, int *nchunks_out);
// T layout ([RHS chunk][m][l - m][RC][cos, sin]) of the Legendre kernels
int synth_rc(int nrhs);
int adj_rc(int nrhs);
long long tlayout_doubles(int lmax, int nrhs, int rc);
int launch_pack_t(int lmax, int nrhs, int RC, const double *x, const double *dl, double *U,
                  hipStream_t s);
// P: partial sums in float64, or float32 (pf32) from the mixed-precision adjoints;
// cf (optional): c_lm of a geometry of band limit glmax, multiplied into the sums
// (the matrix-core adjoints run the scaled recurrence mu = lambda / c)
int launch_unpack_t(int lmax, int nrhs, int RC, int nchunks, const void *P, bool pf32,
                    const double *cf, int glmax, const double *x, const double *d,
                    const double *bh, double *y, hipStream_t s);

}  // namespace mlcr
