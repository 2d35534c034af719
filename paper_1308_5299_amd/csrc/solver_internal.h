// Internal declarations of the multi-level solver.
#pragma once

#include <vector>

#include "mlcr_internal.h"

namespace mlcr {

// pixel-level tiles: k x k nested pixels, k = 8 on every level (Sec. 3.5)
constexpr int kTileK = 8;
constexpr int kTileK2 = kTileK * kTileK;

// solver_kernels.hip
int launch_transfer(const double *src, int lmax_src, double *dst, int lmax_dst, const double *w,
                    int lmax_w, bool add, int nrhs, hipStream_t s);
int launch_axpy_l(double *x, const double *r, const double *c, const double *d, int lmax, int nrhs,
                  hipStream_t s);
int launch_residual(const double *b, const double *y, double *r, const double *act, int lmax,
                    int nrhs, hipStream_t s);
int launch_wnorms(const double *a, const double *b, const double *w, int lmax, int nrhs,
                  double *partial, double *out, hipStream_t s);
int launch_diag_pairs(const double2 *Xi, int ldx, double2 *G, int lmax, int nrings,
                      hipStream_t s);
int launch_diag_inverse(const double *q, const double *d, const double *bh, double *dinv, int lmax,
                        hipStream_t s);
int launch_probe_maps(double *maps, long long npix, const int *tilepix, const int *tiles, int ntl,
                      int kk, int c0, int nprobe, hipStream_t s);
int launch_probe_collect(const double *z, long long npix, const int *tilepix, const int *tiles,
                         int ntl, const int *nbptr, const int *nbs, const int *rev, int max_nb,
                         int c0, int nprobe, double *diag, float *off, hipStream_t s);
int launch_sym_off(const int *nbptr, const int *nbs, const int *rev, float *off, int ntiles,
                   hipStream_t s);
int launch_tile_factor(const double *blocks, int ntiles, int kk, float *minv, float *ridge,
                       hipStream_t s);
// mode 0: block Gauss-Seidel / forward triangular solve y_t = M_t (r_t - sum_{earlier} B_tu y_u);
// 1: Gauss-Seidel backward y_t -= M_t sum_{later} B_tu y_u; 2: backward
// triangular solve y_t = M_t^T (y_t - sum_{later} B_tu y_u)
int launch_sgs_color(int mode, const double *r, double *y, long long npix, int nrhs,
                     const int *tilepix, const int *tiles, int ntl, const int *nbptr,
                     const int *nbs, const int *color, int kappa, const float *off,
                     const float *minv, hipStream_t s);
// dense block of A_h from ring Fourier sums (eq. Ni-dense): lambda table
// lt[nrings][(L+1)(L+2)/2] for l <= L (<= 127), then A over the active modes
// (mode[i] = l | m << 8 | sine << 16) with the level's d and bh per l
int launch_dense_lambda(const double *rz, const double *rs, int nrings, int L, double *lt,
                        hipStream_t s);
int launch_dense_ringdft(const double2 *Xi, int ldx, const double *lt, int L, int nrings,
                         const int *mode, int na, const double *d, const double *bh, double *A,
                         hipStream_t s);
int launch_dense_cholesky(double *a, int n, int *info, hipStream_t s);
int launch_dense_inverse(const double *L, int n, double *inv, hipStream_t s);
// ws: dense_apply_ws_doubles(n, nrhs) doubles of device workspace
long long dense_apply_ws_doubles(int n, int nrhs);
int launch_dense_apply(const double *Ainv, int n, const int *act_idx, const double *b, double *x,
                       long long nalm, int nrhs, double *ws, hipStream_t s);
int launch_fill_zero(double *p, long long n, hipStream_t s);
// per-RHS dot products (c, d may be null), out[2 r], out[2 r + 1]
int launch_dots(const double *a, const double *b, const double *c, const double *d, int lmax,
                int nrhs, double *partial, double *out, hipStream_t s);
// out[l] = sum over RHS and m of a_lm b_lm (cosine and sine entries of l)
int launch_ell_dots(const double *a, const double *b, int lmax, int nrhs, double *out,
                    hipStream_t s);
// out = al[r] u + be[r] v, n values per RHS (al, be: device arrays per RHS)
int launch_lincomb(const double *u, const double *v, double *out, const double *al,
                   const double *be, long long n, int nrhs, hipStream_t s);
// CR right-hand side: pix = N^-1 d + N^-1/2 w2; b = bh v + sqrt(dd) w1
int launch_cr_pix(const double *d, const double *w2, const double *ninv, double *pix,
                  long long npix, int nrhs, hipStream_t s);
int launch_cr_combine(const double *v, const double *w1, const double *bh, const double *dd,
                      double *b, int lmax, int nrhs, hipStream_t s);

// legendre.hip: adjoint with lambda^2 (diagonal of Y^T N^-1 Y)
int launch_legendre_adjoint_sq(const LegendreArgs &a, const double2 *G, double *P,
                               int *nchunks_out);

// api.cpp: operator apply without the max_nrhs limit (workspaces grow), on
// one of the operator's levels or on a level held elsewhere (a solver's)
int apply_level(mlcr_op *op, int level, int nrhs, const double *x, double *y, int prec,
                hipStream_t s);
int apply_level_on(mlcr_op *op, const mlcr_level &L, int nrhs, const double *x, double *y,
                   int prec, hipStream_t s);
// level tables (band limit, filter; gl: Gauss-Legendre evaluation of
// Y^T N^-1 Y) into L; refresh after a prior change; release everything
int define_level(mlcr_op *op, mlcr_level &L, int lmax_h, const double *fl, bool gl);
int refresh_level(mlcr_op *op, mlcr_level &L);
void release_level(mlcr_level &L);

// HEALPix NESTED -> RING index (Gorski et al. 2005)
long long nest2ring(int nside, long long ipnest);

// tiles.cpp: neighbour graph and colourings of the k x k nested tiles of a
// pixel level.  Tiles are neighbours when their nearest pixel centres are
// closer than kTileAdjPx pixel widths; tiles probed together keep all tiles
// they are read at kProbeSepPx pixel widths away from each other.
constexpr double kTileAdjPx = 4.0;
constexpr double kProbeSepPx = 6.0;
struct TileGraph {
    int nt = 0, max_nb = 0;
    std::vector<int> nb;             // [nt][max_nb] neighbour tiles, -1 padded, ascending
    std::vector<int> sweep_color;    // neighbours differ
    std::vector<int> probe_color;    // probe responses separate
    int n_sweep = 0, n_probe = 0;
};
int build_tile_graph(int nside, int k, int max_nb, TileGraph &G);
// pixel-centre unit vectors [npix][3] and RING indices [npix] in NESTED order
void nested_pixel_table(int nside, std::vector<double> &vec, std::vector<int> &ring);

// smoother_icc.hip: the paper's smoother construction (Sec. 3.5) --
// tabulated addition-theorem kernels g(theta) = sum_l (2l+1)/(4 pi) g_l P_l(cos theta),
// the blocks of D_hat_h and of B_hat_h^T N^-1 B_hat_h (no fill-in) on the tile
// pattern, multicolour block incomplete Cholesky and its triangular solves
struct AddThmTable {
    double dth = 0.0;       // table step in theta
    int n = 0;              // points theta_i = i dth, i < n
    const double *tab = nullptr;
};
int launch_addthm_table(const double *gl, int lmax, double dth, int ntab, double *tab,
                        hipStream_t s);
// Assembled blocks (float32, column-major 64 x 64): diag[t] = A_tt and
// off[slot] = A_tu for the CSR slots of the tile graph.  vlev: level pixel
// vectors (nested), vobs/oring/ninv: observation pixels (nested) with their
// RING index into ninv; sub = obs pixels per level tile.
int launch_smoother_assemble(int ntiles, const int *nbptr, const int *nbs, const int *rev,
                             const int *jobs, int njobs, const double *vlev, const double *vobs,
                             const int *oring, const double *ninv, long long sub, AddThmTable gD,
                             AddThmTable gB, float *diag, float *off, hipStream_t s);
// One colour of the block ICC(0) of the assembled blocks (adiag, aoff) with
// ridge alpha * scale on the diagonal: for each tile t of the colour, L_tt
// (its inverse into minv, column-major) and L_ut for later neighbours u
// (L_ut at lslot[rev], L_ut^T at lslot[slot]); fail[t] = 1 on a failed pivot.
int launch_icc_color(const int *tiles, int ntl, const int *nbptr, const int *nbs, const int *rev,
                     const int *color, int kappa, const float *adiag, const float *aoff,
                     double shift, float *minv, float *lslot, int *fail, hipStream_t s);
int launch_max_diag(const float *adiag, int ntiles, double *out, hipStream_t s);

}  // namespace mlcr
