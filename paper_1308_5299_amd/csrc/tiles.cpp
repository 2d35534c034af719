// Tile graph of the pixel-level error smoothers (Sec. 3.5).
//
// Each pixel level is cut into k x k tiles (nested blocks of k^2 pixels).  The
// smoother keeps the couplings of Y_h A_h Y_h^T inside a tile and between
// neighbouring tiles, and drops the rest, as in the paper's block-sparse
// pattern (every pixel sees at least k pixels around it).  Two colourings of
// the tile graph serve the GPU:
//
// * the sweep colouring: neighbouring tiles get different colours, so a
//   block Gauss-Seidel sweep can update all tiles of one colour at once;
// * the probe colouring: the blocks are read off by applying the operator to
//   indicator maps holding one pixel in every tile of a colour.  The response
//   of tile u's probe is read at u and at its neighbours; no other tile of the
//   same colour may come within sep pixel widths of any of them, so that the
//   response there is u's column alone.
//
// Distances are between pixel centres in units of the mean pixel width
// sqrt(4 pi / N_pix); the nearest pixels of two disjoint tiles lie on their
// boundaries, so only boundary pixels are compared.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "solver_internal.h"

namespace mlcr {

// Centre of RING pixel ip as a unit vector (Gorski et al. 2005, pixel
// centres of the polar caps and the equatorial belt).
static void pix_vec_ring(int nside, long long ip, double v[3]) {
    const long long ns = nside, npix = 12 * ns * ns, ncap = 2 * ns * (ns - 1);
    double z, phi;
    if (ip < ncap) {                         // north polar cap: ring i has 4 i pixels
        long long i = (long long)((1.0 + std::sqrt(1.0 + 2.0 * (double)ip)) / 2.0);
        while (2 * i * (i - 1) > ip) i--;
        while (2 * (i + 1) * i <= ip) i++;
        const long long j = ip - 2 * i * (i - 1);
        z = 1.0 - (double)(i * i) / (3.0 * (double)(ns * ns));
        phi = ((double)j + 0.5) * M_PI / (2.0 * (double)i);
    } else if (ip < npix - ncap) {           // equatorial belt: 4 nside pixels per ring
        const long long q = ip - ncap, i = q / (4 * ns) + ns, j = q % (4 * ns);
        const double shift = ((i + ns) & 1) ? 0.0 : 0.5;
        z = (4.0 / 3.0) - 2.0 * (double)i / (3.0 * (double)ns);
        phi = ((double)j + shift) * M_PI / (2.0 * (double)ns);
    } else {                                 // south polar cap, mirrored
        const long long q = npix - 1 - ip;
        long long i = (long long)((1.0 + std::sqrt(1.0 + 2.0 * (double)q)) / 2.0);
        while (2 * i * (i - 1) > q) i--;
        while (2 * (i + 1) * i <= q) i++;
        const long long j = 4 * i - 1 - (q - 2 * i * (i - 1));
        z = -1.0 + (double)(i * i) / (3.0 * (double)(ns * ns));
        phi = ((double)j + 0.5) * M_PI / (2.0 * (double)i);
    }
    const double st = std::sqrt((1.0 - z) * (1.0 + z));
    v[0] = st * std::cos(phi);
    v[1] = st * std::sin(phi);
    v[2] = z;
}

namespace {

struct Near {
    int u;
    float d;      // nearest pixel-centre distance in pixel widths
};

// all tiles u != t nearer than reach_px to tile t, with their distances
void near_lists(int nside, int k, double reach_px, std::vector<std::vector<Near>> &out) {
    const long long kk = (long long)k * k;
    const long long nt = 12LL * (nside / k) * (nside / k);
    std::vector<int> bnd;
    for (int c = 0; c < kk; c++) {
        int x = 0, y = 0;
        for (int b = 0; b < 15; b++) {
            x |= ((c >> (2 * b)) & 1) << b;
            y |= ((c >> (2 * b + 1)) & 1) << b;
        }
        if (x == 0 || y == 0 || x == k - 1 || y == k - 1) bnd.push_back(c);
    }
    const int nb = (int)bnd.size();
    std::vector<double> bv((size_t)nt * nb * 3), cen((size_t)nt * 3), rad(nt);
    for (long long t = 0; t < nt; t++) {
        double c3[3] = {0, 0, 0};
        for (int b = 0; b < nb; b++) {
            double *v = &bv[((size_t)t * nb + b) * 3];
            pix_vec_ring(nside, nest2ring(nside, t * kk + bnd[b]), v);
            for (int d = 0; d < 3; d++) c3[d] += v[d];
        }
        const double nrm = std::sqrt(c3[0] * c3[0] + c3[1] * c3[1] + c3[2] * c3[2]);
        for (int d = 0; d < 3; d++) cen[t * 3 + d] = c3[d] / nrm;
        double r = 0.0;
        for (int b = 0; b < nb; b++) {
            const double *v = &bv[((size_t)t * nb + b) * 3];
            double e = 0.0;
            for (int d = 0; d < 3; d++) e += (v[d] - cen[t * 3 + d]) * (v[d] - cen[t * 3 + d]);
            r = std::max(r, std::sqrt(e));
        }
        rad[t] = r;
    }
    const double px = std::sqrt(4.0 * M_PI / (12.0 * (double)nside * nside));
    const double dreach = reach_px * px;     // chord ~ angle at these scales
    double rmax = 0.0;
    for (long long t = 0; t < nt; t++) rmax = std::max(rmax, rad[t]);
    // spatial hash of tile centres; a cell is no smaller than the largest reach
    const double reach = 2.0 * rmax + dreach;
    const int nc = std::max(1, std::min(1 << 20, (int)(2.0 / reach)));
    const double cw = 2.0 / nc;
    auto cell = [&](double u) { return std::min(nc - 1, std::max(0, (int)((u + 1.0) / cw))); };
    auto key = [&](long long a, long long b, long long c) { return (a * nc + b) * nc + c; };
    std::vector<std::pair<long long, int>> cells(nt);
    for (long long t = 0; t < nt; t++)
        cells[t] = {key(cell(cen[t * 3]), cell(cen[t * 3 + 1]), cell(cen[t * 3 + 2])), (int)t};
    std::sort(cells.begin(), cells.end());
    out.assign(nt, {});
    auto work = [&](long long t0, long long t1) {
        for (long long t = t0; t < t1; t++) {
            const int cx = cell(cen[t * 3]), cy = cell(cen[t * 3 + 1]), cz = cell(cen[t * 3 + 2]);
            for (int ax = std::max(0, cx - 1); ax <= std::min(nc - 1, cx + 1); ax++)
                for (int ay = std::max(0, cy - 1); ay <= std::min(nc - 1, cy + 1); ay++)
                    for (int az = std::max(0, cz - 1); az <= std::min(nc - 1, cz + 1); az++) {
                        const long long kc = key(ax, ay, az);
                        auto it = std::lower_bound(cells.begin(), cells.end(),
                                                   std::make_pair(kc, -1));
                        for (; it != cells.end() && it->first == kc; ++it) {
                            const int u = it->second;
                            if (u == t) continue;
                            double e = 0.0;
                            for (int d = 0; d < 3; d++) {
                                const double q = cen[t * 3 + d] - cen[u * 3 + d];
                                e += q * q;
                            }
                            if (std::sqrt(e) >= rad[t] + rad[u] + dreach) continue;
                            double best = 1e300;
                            for (int a = 0; a < nb; a++) {
                                const double *va = &bv[((size_t)t * nb + a) * 3];
                                for (int b = 0; b < nb; b++) {
                                    const double *vb = &bv[((size_t)u * nb + b) * 3];
                                    const double dx = va[0] - vb[0], dy = va[1] - vb[1],
                                                 dz = va[2] - vb[2];
                                    best = std::min(best, dx * dx + dy * dy + dz * dz);
                                }
                            }
                            const double dpx = std::sqrt(best) / px;
                            if (dpx < reach_px) out[t].push_back({u, (float)dpx});
                        }
                    }
            std::sort(out[t].begin(), out[t].end(),
                      [](const Near &a, const Near &b) { return a.u < b.u; });
        }
    };
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nt < 4096) nth = 1;
    std::vector<std::thread> th;
    const long long chunk = (nt + nth - 1) / nth;
    for (unsigned i = 0; i < nth; i++) {
        const long long a = i * chunk, b = std::min<long long>(nt, a + chunk);
        if (a < b) th.emplace_back(work, a, b);
    }
    for (auto &x : th) x.join();
}

// smallest colour not marked
int first_free(std::vector<char> &used) {
    int c = 0;
    while ((size_t)c < used.size() && used[c]) c++;
    return c;
}

}  // namespace

int build_tile_graph(int nside, int k, int max_nb, TileGraph &G) {
    const long long nt = 12LL * (nside / k) * (nside / k);
    std::vector<std::vector<Near>> near;
    near_lists(nside, k, std::max(kTileAdjPx, kProbeSepPx), near);
    G.nt = (int)nt;
    G.max_nb = max_nb;
    G.nb.assign((size_t)nt * max_nb, -1);
    std::vector<std::vector<int>> adj(nt), sep(nt);
    for (long long t = 0; t < nt; t++)
        for (const Near &n : near[t]) {
            if (n.d < kTileAdjPx) adj[t].push_back(n.u);
            if (n.d < kProbeSepPx) sep[t].push_back(n.u);
        }
    for (long long t = 0; t < nt; t++) {
        if ((int)adj[t].size() > max_nb)
            return fail(MLCR_EINVAL, "tile " + std::to_string(t) + " has " +
                                         std::to_string(adj[t].size()) + " neighbours (limit " +
                                         std::to_string(max_nb) + ")");
        for (size_t j = 0; j < adj[t].size(); j++) G.nb[(size_t)t * max_nb + j] = adj[t][j];
    }
    // sweep colouring: greedy over the neighbour graph in nested order
    G.sweep_color.assign(nt, -1);
    std::vector<char> used;
    for (long long t = 0; t < nt; t++) {
        used.assign(used.size(), 0);
        for (int u : adj[t])
            if (G.sweep_color[u] >= 0) {
                if ((size_t)G.sweep_color[u] >= used.size()) used.resize(G.sweep_color[u] + 1, 0);
                used[G.sweep_color[u]] = 1;
            }
        G.sweep_color[t] = first_free(used);
    }
    // probe colouring: u and u' conflict when u' is within sep of a tile of
    // N[u] (u and its neighbours) or u is within sep of a tile of N[u']; with
    // symmetric near lists the second set is N[sep[u]]
    // visit order: the nine 3 x 3 sub-lattices of tiles inside each base face
    // one after another, so a regular patch needs nine colours and the extra
    // ones go only to tiles where faces meet
    std::vector<std::pair<int, int>> ord(nt);
    const long long tpf = nt / 12;
    for (long long t = 0; t < nt; t++) {
        long long q = t % tpf;
        int x = 0, y = 0;
        for (int b = 0; q; b++) {
            x |= (int)(q & 1) << b;
            q >>= 1;
            y |= (int)(q & 1) << b;
            q >>= 1;
        }
        ord[t] = {(x % 3) + 3 * (y % 3), (int)t};
    }
    std::stable_sort(ord.begin(), ord.end(),
                     [](const std::pair<int, int> &a, const std::pair<int, int> &b) {
                         return a.first < b.first;
                     });
    G.probe_color.assign(nt, -1);
    std::vector<int> mark(nt, -1);
    for (const auto &o : ord) {
        const long long u = o.second;
        used.assign(used.size(), 0);
        auto hit = [&](int w) {
            if (w == u || mark[w] == u) return;
            mark[w] = (int)u;
            const int c = G.probe_color[w];
            if (c < 0) return;
            if ((size_t)c >= used.size()) used.resize(c + 1, 0);
            used[c] = 1;
        };
        auto closed_adj_then = [&](int t, const std::vector<std::vector<int>> &rel) {
            hit(t);
            for (int w : rel[t]) hit(w);
        };
        // S(N[u]): tiles within sep of u or of a neighbour of u
        closed_adj_then((int)u, sep);
        for (int t : adj[u]) closed_adj_then(t, sep);
        // N[S(u)]: neighbours of tiles within sep of u
        for (int t : sep[u]) closed_adj_then(t, adj);
        G.probe_color[u] = first_free(used);
    }
    G.n_sweep = 0;
    G.n_probe = 0;
    for (long long t = 0; t < nt; t++) {
        G.n_sweep = std::max(G.n_sweep, G.sweep_color[t] + 1);
        G.n_probe = std::max(G.n_probe, G.probe_color[t] + 1);
    }
    return MLCR_OK;
}

// Unit vectors of the pixel centres of a grid in NESTED order (3 doubles per
// pixel), and the RING index of each nested pixel; filled by several threads.
void nested_pixel_table(int nside, std::vector<double> &vec, std::vector<int> &ring) {
    const long long npix = 12LL * nside * nside;
    vec.assign((size_t)npix * 3, 0.0);
    ring.assign((size_t)npix, 0);
    const int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int w = 0; w < nth; w++)
        th.emplace_back([&, w]() {
            for (long long n = w; n < npix; n += nth) {
                const long long r = nest2ring(nside, n);
                ring[n] = (int)r;
                pix_vec_ring(nside, r, &vec[(size_t)n * 3]);
            }
        });
    for (auto &t : th) t.join();
}

}  // namespace mlcr
