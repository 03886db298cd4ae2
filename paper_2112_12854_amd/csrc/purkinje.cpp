// Host precompute of the Purkinje graph (vertex-centred finite volumes on a
// branching 1D medium, Sec. 3.2) and of the Purkinje-muscle junction regions
// (Sec. 3.3).  All in FP64, caller numbering unless stated.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "prep.hpp"

namespace ep {

namespace {

struct Grid {
    double lo[3], G;
    std::unordered_map<uint64_t, std::vector<int32_t>> cells;
    std::array<int64_t, 3> key(const double *x) const {
        return {(int64_t)std::floor((x[0] - lo[0]) / G), (int64_t)std::floor((x[1] - lo[1]) / G),
                (int64_t)std::floor((x[2] - lo[2]) / G)};
    }
    // keys of far-away points may collide; every candidate is tested exactly
    static uint64_t pack(int64_t a, int64_t b, int64_t c) {
        const uint64_t m = (1u << 21) - 1;
        return (((uint64_t)a & m) << 42) | (((uint64_t)b & m) << 21) | ((uint64_t)c & m);
    }
};

}  // namespace

std::string prepare_purkinje(const PurkIn &in, const PrepIn &tin, const PrepOut &tout,
                             PurkOut &out) {
    const int64_t n = in.n;
    if (n < 0 || (n == 0 && in.pmjs.empty())) return "empty Purkinje graph";
    if (n > 0 && (in.n_edges < 0 || !in.xyz || (in.n_edges > 0 && !in.edges)))
        return "empty Purkinje graph";
    if (n > 0 && !(in.sigma > 0)) return "Purkinje conductivity must be positive";
    // slot offsets of the state arrays are 32-bit byte offsets
    if (n >= (int64_t)1 << 25) return "Purkinje graph too large";
    out.n = n;

    // ---- graph operator: node i owns half of each incident segment
    std::vector<int32_t> deg(n, 0);
    for (int64_t e = 0; e < in.n_edges; ++e) {
        const int32_t a = in.edges[2 * e], b = in.edges[2 * e + 1];
        if (a < 0 || a >= n || b < 0 || b >= n) return "Purkinje edge index out of range";
        if (a == b) return "Purkinje edge joins a node to itself";
        deg[a]++;
        deg[b]++;
    }
    out.off.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) out.off[i + 1] = out.off[i] + deg[i];
    out.nbr.assign(out.off[n], 0);
    std::vector<double> len(out.off[n]), sc(out.off[n]);
    std::vector<int32_t> fill(out.off.begin(), out.off.end() - 1);
    for (int64_t e = 0; e < in.n_edges; ++e) {
        const int32_t a = in.edges[2 * e], b = in.edges[2 * e + 1];
        const double *p = in.xyz + 3 * (int64_t)a, *q = in.xyz + 3 * (int64_t)b;
        const double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
        const double L = std::sqrt(dx * dx + dy * dy + dz * dz);
        if (!(L > 0)) return "Purkinje segment of zero length";
        const double k = in.edge_scale ? in.edge_scale[e] : 1.0;
        if (!(k >= 0.0) || !std::isfinite(k)) return "bad Purkinje segment conductivity scale";
        out.nbr[fill[a]] = b;
        sc[fill[a]] = k;
        len[fill[a]++] = L;
        out.nbr[fill[b]] = a;
        sc[fill[b]] = k;
        len[fill[b]++] = L;
    }
    out.g.assign(out.off[n], 0.0);
    double dtmax = HUGE_VAL;
    for (int64_t i = 0; i < n; ++i) {
        double ell = 0.0, inv = 0.0;
        for (int32_t e = out.off[i]; e < out.off[i + 1]; ++e) {
            ell += 0.5 * len[e];
            inv += sc[e] / len[e];
        }
        for (int32_t e = out.off[i]; e < out.off[i + 1]; ++e)
            out.g[e] = in.sigma * sc[e] / (in.chi * in.cm * ell * len[e]);
        if (inv > 0) dtmax = std::min(dtmax, in.chi * in.cm * ell / (in.sigma * inv));
    }
    // explicit substeps: 90 % of the Gershgorin bound of the graph operator
    // (nodes cut off by blocked segments on every side impose none); the
    // Adams-Bashforth 2 interval on the negative real axis is half as long
    int32_t ns = in.n_sub;
    if (ns <= 0) {
        const double lim = (in.ab2 ? 0.45 : 0.9) * dtmax;
        ns = 1;
        while (in.dt / ns > lim) {
            if (++ns > 100000) return "Purkinje graph needs more than 1e5 substeps";
        }
    }
    out.n_sub = ns;

    // ---- junction regions
    const int64_t nc = tin.n_tets;
    // cells: tetrahedra, or triangles (fourth node -1)
    auto nverts = [&](int64_t c) { return tin.tets[4 * c + 3] < 0 ? 3 : 4; };
    std::vector<double> cen(3 * nc);
    for (int64_t c = 0; c < nc; ++c) {
        const int32_t *t = tin.tets + 4 * c;
        const int nv = nverts(c);
        for (int a = 0; a < 3; ++a) {
            double x = 0.0;
            for (int k = 0; k < nv; ++k) x += tin.xyz[3 * (int64_t)t[k] + a];
            cen[3 * c + a] = x / nv;
        }
    }
    Grid grid;
    double hi[3];
    for (int a = 0; a < 3; ++a) { grid.lo[a] = HUGE_VAL; hi[a] = -HUGE_VAL; }
    for (int64_t c = 0; c < nc; ++c)
        for (int a = 0; a < 3; ++a) {
            grid.lo[a] = std::min(grid.lo[a], cen[3 * c + a]);
            hi[a] = std::max(hi[a], cen[3 * c + a]);
        }
    const double ext = std::max({hi[0] - grid.lo[0], hi[1] - grid.lo[1], hi[2] - grid.lo[2], 1e-300});
    grid.G = std::max(ext / 64.0, 1e-12);
    for (const PmjIn &p : in.pmjs) grid.G = std::max(grid.G, p.radius);
    for (int64_t c = 0; c < nc; ++c) {
        auto k = grid.key(&cen[3 * c]);
        grid.cells[Grid::pack(k[0], k[1], k[2])].push_back((int32_t)c);
    }
    // node -> incident cells (for the fallback region)
    std::vector<int32_t> noff(tin.n_nodes + 1, 0), ncell(4 * nc);
    for (int64_t c = 0; c < nc; ++c)
        for (int a = 0; a < nverts(c); ++a) noff[tin.tets[4 * c + a] + 1]++;
    for (int64_t i = 0; i < tin.n_nodes; ++i) noff[i + 1] += noff[i];
    {
        std::vector<int32_t> f(noff.begin(), noff.end() - 1);
        for (int64_t c = 0; c < nc; ++c)
            for (int a = 0; a < nverts(c); ++a) ncell[f[tin.tets[4 * c + a]]++] = (int32_t)c;
    }

    out.jroff.assign(1, 0);
    out.jcells.clear();
    out.jsrc.clear();
    for (const PmjIn &p : in.pmjs) {
        // source point and the kind of cell the region takes (0: any; a cell
        // source couples to the other medium)
        const double *x;
        int kind = 0;
        if (p.cell >= 0) {
            if (p.cell >= nc) return "junction source cell out of range";
            x = &cen[3 * (int64_t)p.cell];
            kind = nverts(p.cell) == 3 ? 4 : 3;
            out.jsrc.push_back(tout.iperm[p.cell]);
        } else {
            if (p.node < 0 || p.node >= n) return "junction node out of range";
            x = in.xyz + 3 * (int64_t)p.node;
            out.jsrc.push_back(-1);
        }
        auto ok = [&](int32_t c) { return kind == 0 || nverts(c) == kind; };
        auto dist = [&](int32_t c) {
            const double dx = cen[3 * (int64_t)c] - x[0], dy = cen[3 * (int64_t)c + 1] - x[1],
                         dz = cen[3 * (int64_t)c + 2] - x[2];
            return std::sqrt(dx * dx + dy * dy + dz * dz);
        };
        std::vector<int32_t> region;
        // bucket side >= radius: the 27 buckets around the node hold every candidate
        const auto kx = grid.key(x);
        for (int64_t a = -1; a <= 1; ++a)
            for (int64_t b = -1; b <= 1; ++b)
                for (int64_t c = -1; c <= 1; ++c) {
                    auto it = grid.cells.find(Grid::pack(kx[0] + a, kx[1] + b, kx[2] + c));
                    if (it == grid.cells.end()) continue;
                    for (int32_t q : it->second)
                        if (ok(q) && dist(q) <= p.radius) region.push_back(q);
                }
        std::sort(region.begin(), region.end());
        region.erase(std::unique(region.begin(), region.end()), region.end());
        if (region.empty()) {
            // the cells sharing a mesh node with the cell of nearest centroid
            // (smallest id among equals)
            double best = HUGE_VAL;
            int32_t bc = -1;
            auto consider = [&](int32_t c) {
                if (!ok(c)) return;
                const double d = dist(c);
                if (d < best || (d == best && c < bc)) { best = d; bc = c; }
            };
            const int64_t kmax = (int64_t)std::ceil(ext / grid.G) + 1;
            const bool inside = kx[0] >= -2 && kx[1] >= -2 && kx[2] >= -2 && kx[0] <= kmax + 2 &&
                                kx[1] <= kmax + 2 && kx[2] <= kmax + 2;
            if (inside) {
                // shells of buckets at Chebyshev distance r: cells not yet
                // seen after shell r lie at least r G away
                for (int64_t r = 0; r <= kmax + 4; ++r) {
                    for (int64_t a = -r; a <= r; ++a)
                        for (int64_t b = -r; b <= r; ++b)
                            for (int64_t c = -r; c <= r; ++c) {
                                if (std::max({std::llabs(a), std::llabs(b), std::llabs(c)}) != r) continue;
                                auto it = grid.cells.find(Grid::pack(kx[0] + a, kx[1] + b, kx[2] + c));
                                if (it == grid.cells.end()) continue;
                                for (int32_t q : it->second) consider(q);
                            }
                    if (bc >= 0 && best < (double)r * grid.G) break;
                }
            } else {
                for (int64_t c = 0; c < nc; ++c) consider((int32_t)c);
            }
            if (bc < 0) return p.cell >= 0 ? "no cell of the other medium for a junction"
                                           : "no tissue cell for a junction";
            for (int a = 0; a < nverts(bc); ++a) {
                const int32_t node = tin.tets[4 * (int64_t)bc + a];
                for (int32_t e = noff[node]; e < noff[node + 1]; ++e) region.push_back(ncell[e]);
            }
            std::sort(region.begin(), region.end());
            region.erase(std::unique(region.begin(), region.end()), region.end());
        }
        for (int32_t u : region) out.jcells.push_back(tout.iperm[u]);
        out.jroff.push_back((int32_t)out.jcells.size());
    }

    // ---- per cell: junctions pulsing it, in junction order (its regions'
    // pulses, and the two-way pulses of junctions it is the source of)
    out.cpmj.assign(nc, -1);
    std::vector<int32_t> cnt(nc, 0);
    for (int32_t c : out.jcells) cnt[c]++;
    for (size_t k = 0; k < in.pmjs.size(); ++k)
        if (out.jsrc[k] >= 0 && in.pmjs[k].two_way) cnt[out.jsrc[k]]++;
    out.cpmj_list.clear();
    for (int64_t c = 0; c < nc; ++c)
        if (cnt[c] > 0) {
            out.cpmj[c] = (int32_t)out.cpmj_list.size();
            out.cpmj_list.resize(out.cpmj_list.size() + cnt[c] + 1, -1);
            cnt[c] = out.cpmj[c];   // next free entry
        }
    for (size_t k = 0; k + 1 < out.jroff.size(); ++k) {
        for (int32_t q = out.jroff[k]; q < out.jroff[k + 1]; ++q)
            out.cpmj_list[cnt[out.jcells[q]]++] = (int32_t)k;
        if (out.jsrc[k] >= 0 && in.pmjs[k].two_way)
            out.cpmj_list[cnt[out.jsrc[k]]++] = (int32_t)k | kAntiBit;
    }
    if (out.cpmj_list.empty()) out.cpmj_list.push_back(-1);
    return "";
}

}  // namespace ep
