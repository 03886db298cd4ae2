// Host precompute of the cell-centred tetrahedral FV operator (Sec. 3.2 of
// the paper) in the form the device kernels consume.
//
// The paper evaluates, per step, (a) node values by inverse-distance
// weighting, (b) face values as node means, (c) Gauss-Green cell gradients,
// (d) face gradients interpolated with the weights alpha of the two cells,
// (e) the eq. gra2bis correction along the centre-to-centre unit vector e,
// (f) fluxes A (M_f g_f).n.  Steps (b)-(f) are linear in the node values and
// in the two cell values of each face, so for every cell they are folded
// here into 8 node coefficients (its 4 vertices and the 4 vertices opposite
// its faces in the neighbours) and 4 two-point coefficients:
//
//   g_c = sum_k v_{n_k} G_ck,  G_ck = -S_k / (3 V_c)   (S_k: outward area
//         vector of the face opposite vertex k; Gauss-Green with face values
//         equal to node means reduces to this),
//   F_f = a_f . (alpha g_c + (1-alpha) g_c') + b_f (v_c' - v_c),
//         w = M_f S_f,  a_f = w - (w.e) e,  b_f = (w.e)/d,
//   L_c = sum_f F_f / (chi Cm V_c).
//
// Only step (a) stays a separate gather, because its stencil (all cells
// around a node) is not local to one cell.  Everything is FP64 here; the
// FP32 path rounds the finished coefficients.
#include "prep.hpp"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>

namespace ep {
namespace {

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn) {
    unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    if (n < 20000 || nt == 1) {
        fn(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        int64_t a = t * chunk, b = std::min<int64_t>(n, a + chunk);
        if (a >= b) break;
        th.emplace_back(fn, a, b);
    }
    for (auto &t : th) t.join();
}

using V3 = std::array<double, 3>;
inline V3 sub(const V3 &a, const V3 &b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline double dot(const V3 &a, const V3 &b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline V3 cross(const V3 &a, const V3 &b) {
    return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
inline double len(const V3 &a) { return std::sqrt(dot(a, a)); }

struct Geo {
    std::vector<V3> cen;                 // centroid
    std::vector<double> vol;             // volume (tet) or area (triangle)
    std::vector<std::array<V3, 4>> S;    // outward area vector opposite vertex k
    std::vector<std::array<V3, 4>> Sf;   // area vector of the face's flux
    std::vector<std::array<int32_t, 4>> nb;  // face neighbour opposite vertex k
};

// Cells are tetrahedra, or triangles of a 2D medium when the fourth node is
// -1 (the paper's 2D Purkinje shell, Sec. 3.2): there a "face" is the edge
// opposite vertex k, its area vector the in-plane outward normal times the
// edge length, and the "volume" the area.
inline int nverts(const PrepIn &in, int64_t c) { return in.tets[4 * c + 3] < 0 ? 3 : 4; }

V3 node(const PrepIn &in, int32_t i) {
    return {in.xyz[3 * (int64_t)i], in.xyz[3 * (int64_t)i + 1], in.xyz[3 * (int64_t)i + 2]};
}

std::string validate(const PrepIn &in) {
    if (in.n_nodes <= 0 || in.n_tets <= 0) return "empty mesh";
    // device arrays of one instance are addressed with 32-bit byte offsets
    if (in.n_tets >= ((int64_t)1 << 25) || in.n_nodes >= ((int64_t)1 << 28))
        return "mesh too large for one instance (limit 2^25 tets)";
    for (int64_t i = 0; i < 4 * in.n_tets; ++i)
        if ((in.tets[i] < 0 && !(i % 4 == 3 && in.tets[i] == -1)) || in.tets[i] >= in.n_nodes)
            return "cell " + std::to_string(i / 4) + " references node out of range";
    // a node belongs to tetrahedra or to triangles, not both (separate media)
    std::vector<uint8_t> kind(in.n_nodes, 0);
    bool tris = false;
    for (int64_t c = 0; c < in.n_tets; ++c) {
        const int nv = nverts(in, c);
        tris = tris || nv == 3;
        for (int k = 0; k < nv; ++k) {
            uint8_t &m = kind[in.tets[4 * c + k]];
            m |= nv == 3 ? 2 : 1;
            if (m == 3) return "node " + std::to_string(in.tets[4 * c + k]) +
                               " belongs to both tetrahedra and triangles";
        }
    }
    if (tris && in.elliptic) return "the bidomain model takes tetrahedral meshes only";
    for (int64_t c = 0; c < in.n_tets; ++c) {
        const int32_t *t = in.tets + 4 * c;
        if (t[0] == t[1] || t[0] == t[2] || t[1] == t[2] ||
            (t[3] >= 0 && (t[0] == t[3] || t[1] == t[3] || t[2] == t[3])))
            return "cell " + std::to_string(c) + " repeats a node";
        if (in.model && in.model[c] > 5) return "bad model id at tet " + std::to_string(c);
        const double *f = in.fibre + 3 * c;
        double n2 = f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
        if (!(std::fabs(n2 - 1.0) < 1e-6)) return "fibre of tet " + std::to_string(c) + " not unit";
        if (in.scale && !(in.scale[c] >= 0.0 && std::isfinite(in.scale[c])))
            return "bad conductivity scale at tet " + std::to_string(c);
    }
    if (!(in.sigma_l >= 0 && in.sigma_t >= 0 && in.chi > 0 && in.cm > 0))
        return "conductivity, chi and cm must be positive";
    return "";
}

// Face matching: every face is keyed by its sorted vertex triple and bucketed
// by the smallest vertex; equal keys inside a bucket are the two sides.
std::string match_faces(const PrepIn &in, Geo &g, int64_t &n_int, int64_t &n_bnd) {
    const int64_t nc = in.n_tets, nn = in.n_nodes;
    std::vector<int64_t> cnt(nn + 1, 0);
    // a triangle's edge (two vertices) is keyed with d = -1; the node sets of
    // the two media are disjoint, so keys of the two kinds never meet
    for (int64_t c = 0; c < nc; ++c) {
        const int32_t *t = in.tets + 4 * c;
        const int nv = nverts(in, c);
        for (int k = 0; k < nv; ++k) {
            int32_t lo = INT32_MAX;
            for (int q = 0; q < nv; ++q) if (q != k) lo = std::min(lo, t[q]);
            cnt[lo + 1]++;
        }
    }
    for (int64_t i = 0; i < nn; ++i) cnt[i + 1] += cnt[i];
    struct E { int32_t b, d; int64_t id; };
    std::vector<E> ent(cnt[nn]);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t c = 0; c < nc; ++c) {
        const int32_t *t = in.tets + 4 * c;
        const int nv = nverts(in, c);
        for (int k = 0; k < nv; ++k) {
            int32_t v[3] = {0, 0, -1}, m = 0;
            for (int q = 0; q < nv; ++q) if (q != k) v[m++] = t[q];
            std::sort(v, v + m);
            ent[pos[v[0]]++] = E{v[1], m == 3 ? v[2] : -1, 4 * c + k};
        }
    }
    g.nb.assign(nc, {-1, -1, -1, -1});
    std::atomic<int64_t> bad{-1};
    parallel_for(nn, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            auto beg = ent.begin() + cnt[i], end = ent.begin() + cnt[i + 1];
            std::sort(beg, end, [](const E &x, const E &y) {
                return x.b != y.b ? x.b < y.b : (x.d != y.d ? x.d < y.d : x.id < y.id);
            });
            for (auto it = beg; it != end;) {
                auto jt = it + 1;
                while (jt != end && jt->b == it->b && jt->d == it->d) ++jt;
                if (jt - it == 2) {
                    g.nb[it->id / 4][it->id % 4] = (int32_t)((it + 1)->id / 4);
                    g.nb[(it + 1)->id / 4][(it + 1)->id % 4] = (int32_t)(it->id / 4);
                } else if (jt - it > 2) {
                    bad = i;
                }
                it = jt;
            }
        }
    });
    if (bad >= 0) return "non-manifold mesh: a face is shared by more than two cells";
    n_int = n_bnd = 0;
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < nverts(in, c); ++k) (g.nb[c][k] >= 0 ? n_int : n_bnd)++;
    n_int /= 2;
    // flux area vectors: a tetrahedron's own; across an edge between two
    // triangles (not coplanar on a bent surface) the edge length times the
    // unit bisector of the two outward in-plane normals, the same vector with
    // opposite signs on the two sides, so the flux stays conservative
    g.Sf = g.S;
    for (int64_t c = 0; c < nc; ++c) {
        if (nverts(in, c) != 3) continue;
        const int32_t *t = in.tets + 4 * c;
        for (int k = 0; k < 3; ++k) {
            const int32_t c2 = g.nb[c][k];
            if (c2 < 0) continue;
            const int32_t *t2 = in.tets + 4 * (int64_t)c2;
            int k2 = 0;
            for (int q = 0; q < 3; ++q)
                if (t2[q] != t[(k + 1) % 3] && t2[q] != t[(k + 2) % 3]) k2 = q;
            const V3 &a = g.S[c][k], &b = g.S[c2][k2];
            const double la = len(a), lb = len(b);
            V3 m{a[0] / la - b[0] / lb, a[1] / la - b[1] / lb, a[2] / la - b[2] / lb};
            const double lm = len(m);
            g.Sf[c][k] = {la * m[0] / lm, la * m[1] / lm, la * m[2] / lm};
        }
    }
    return "";
}

std::string geometry(const PrepIn &in, Geo &g) {
    const int64_t nc = in.n_tets;
    g.cen.resize(nc);
    g.vol.resize(nc);
    g.S.resize(nc);
    std::atomic<int64_t> degenerate{-1};
    parallel_for(nc, [&](int64_t a, int64_t b) {
        for (int64_t c = a; c < b; ++c) {
            const int32_t *t = in.tets + 4 * c;
            if (nverts(in, c) == 3) {
                V3 p[3];
                for (int k = 0; k < 3; ++k) p[k] = node(in, t[k]);
                V3 N = cross(sub(p[1], p[0]), sub(p[2], p[0]));
                const double twice = len(N);
                if (!(twice > 1e-12 * len(sub(p[1], p[0])) * len(sub(p[2], p[0])))) degenerate = c;
                g.vol[c] = 0.5 * twice;
                for (int i = 0; i < 3; ++i) g.cen[c][i] = (p[0][i] + p[1][i] + p[2][i]) / 3.0;
                N = {N[0] / twice, N[1] / twice, N[2] / twice};
                for (int k = 0; k < 3; ++k) {
                    const V3 &q0 = p[(k + 1) % 3], &q1 = p[(k + 2) % 3];
                    V3 Sk = cross(sub(q1, q0), N);           // |Sk| = edge length
                    const double sg = dot(Sk, sub(q0, p[k])) > 0 ? 1.0 : -1.0;
                    g.S[c][k] = {sg * Sk[0], sg * Sk[1], sg * Sk[2]};
                }
                g.S[c][3] = {0, 0, 0};
                continue;
            }
            V3 p[4];
            for (int k = 0; k < 4; ++k) p[k] = node(in, t[k]);
            V3 e1 = sub(p[1], p[0]), e2 = sub(p[2], p[0]), e3 = sub(p[3], p[0]);
            double det = dot(e1, cross(e2, e3));
            double scale = len(e1) * len(e2) * len(e3);
            if (!(std::fabs(det) > 1e-12 * scale)) degenerate = c;
            g.vol[c] = std::fabs(det) / 6.0;
            for (int i = 0; i < 3; ++i) g.cen[c][i] = 0.25 * (p[0][i] + p[1][i] + p[2][i] + p[3][i]);
            for (int k = 0; k < 4; ++k) {
                const V3 &q0 = p[(k + 1) & 3], &q1 = p[(k + 2) & 3], &q2 = p[(k + 3) & 3];
                V3 A = cross(sub(q1, q0), sub(q2, q0));
                double s = dot(A, sub(q0, p[k])) > 0 ? 0.5 : -0.5;   // away from vertex k
                g.S[c][k] = {s * A[0], s * A[1], s * A[2]};
            }
        }
    });
    if (degenerate >= 0) return "cell " + std::to_string((int64_t)degenerate) + " has zero volume or area";
    return "";
}

// Reverse Cuthill-McKee on the face-adjacency graph, component by component,
// each started from a pseudo-peripheral cell.
std::vector<int32_t> rcm_order(const Geo &g) {
    const int64_t nc = (int64_t)g.nb.size();
    std::vector<int32_t> order;
    order.reserve(nc);
    std::vector<int32_t> level(nc, -1);
    std::vector<char> done(nc, 0);
    auto deg = [&](int32_t c) {
        int d = 0;
        for (int k = 0; k < 4; ++k) d += g.nb[c][k] >= 0;
        return d;
    };
    std::vector<int32_t> q;
    auto bfs_last = [&](int32_t s) {   // farthest cell of a plain BFS
        q.clear();
        q.push_back(s);
        level[s] = 0;
        size_t h = 0;
        while (h < q.size()) {
            int32_t c = q[h++];
            for (int k = 0; k < 4; ++k) {
                int32_t n = g.nb[c][k];
                if (n >= 0 && level[n] < 0) { level[n] = level[c] + 1; q.push_back(n); }
            }
        }
        int32_t best = q.back();
        for (int32_t c : q) level[c] = -1;
        return best;
    };
    for (int64_t s0 = 0; s0 < nc; ++s0) {
        if (done[s0]) continue;
        int32_t s = bfs_last(bfs_last((int32_t)s0));
        size_t start = order.size();
        order.push_back(s);
        done[s] = 1;
        for (size_t h = start; h < order.size(); ++h) {
            int32_t c = order[h];
            int32_t nbr[4], m = 0;
            for (int k = 0; k < 4; ++k) {
                int32_t n = g.nb[c][k];
                if (n >= 0 && !done[n]) { nbr[m++] = n; done[n] = 1; }
            }
            std::sort(nbr, nbr + m, [&](int32_t a, int32_t b) {
                int da = deg(a), db = deg(b);
                return da != db ? da < db : a < b;
            });
            for (int i = 0; i < m; ++i) order.push_back(nbr[i]);
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// Morton (Z-curve) order of the centroids: compact 3D tiles of consecutive cells.
std::vector<int32_t> morton_order(const Geo &g) {
    const int64_t nc = (int64_t)g.cen.size();
    V3 lo = g.cen[0], hi = g.cen[0];
    for (auto &c : g.cen)
        for (int i = 0; i < 3; ++i) { lo[i] = std::min(lo[i], c[i]); hi[i] = std::max(hi[i], c[i]); }
    double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    auto spread = [](uint64_t x) {
        x &= 0x1fffff;
        x = (x | x << 32) & 0x1f00000000ffffULL;
        x = (x | x << 16) & 0x1f0000ff0000ffULL;
        x = (x | x << 8) & 0x100f00f00f00f00fULL;
        x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
        x = (x | x << 2) & 0x1249249249249249ULL;
        return x;
    };
    std::vector<std::pair<uint64_t, int32_t>> key(nc);
    parallel_for(nc, [&](int64_t a, int64_t b) {
        for (int64_t c = a; c < b; ++c) {
            uint64_t q[3];
            for (int i = 0; i < 3; ++i)
                q[i] = (uint64_t)std::min(2097151.0, (g.cen[c][i] - lo[i]) / ext * 2097151.0);
            key[c] = {spread(q[0]) | spread(q[1]) << 1 | spread(q[2]) << 2, (int32_t)c};
        }
    });
    std::sort(key.begin(), key.end());
    std::vector<int32_t> order(nc);
    for (int64_t i = 0; i < nc; ++i) order[i] = key[i].second;
    return order;
}

}  // namespace

std::string prepare(const PrepIn &in, PrepOut &out) {
    std::string err = validate(in);
    if (!err.empty()) return err;
    const int64_t nc = in.n_tets, nn = in.n_nodes;
    Geo g;
    if (!(err = geometry(in, g)).empty()) return err;
    if (!(err = match_faces(in, g, out.n_interior_faces, out.n_boundary_faces)).empty()) return err;

    // ---- cell order: models grouped (stable), then RCM / Morton / input
    std::vector<int32_t> order;
    if (in.ordering == ORDER_RCM) order = rcm_order(g);
    else if (in.ordering == ORDER_MORTON) order = morton_order(g);
    else { order.resize(nc); for (int64_t i = 0; i < nc; ++i) order[i] = (int32_t)i; }
    if (in.model || in.split_media) {
        auto cls = [&](int32_t c) {
            const int m = in.model ? in.model[c] : 0;
            const int medium = in.split_media && nverts(in, c) == 3 ? 1 : 0;
            return medium * 8 + (m <= 2 ? 0 : m);
        };
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return cls(a) < cls(b); });
    }
    out.cell_2d = nc;
    if (in.split_media)
        for (int64_t i = 0; i < nc; ++i)
            if (nverts(in, order[i]) == 3) { out.cell_2d = i; break; }
    {   // the 2D medium's forward-Euler bound from its two-point couplings
        double rmax = 0.0;
        const double smax = std::max(in.sigma_l, in.sigma_t);
        for (int64_t c = 0; c < nc; ++c) {
            if (nverts(in, c) != 3) continue;
            double r = 0.0;
            for (int k = 0; k < 3; ++k) {
                const int32_t c2 = g.nb[c][k];
                if (c2 < 0) continue;
                r += len(g.S[c][k]) / len(sub(g.cen[c2], g.cen[c]));
            }
            r *= smax * (in.scale ? in.scale[c] : 1.0) / (in.chi * in.cm * g.vol[c]);
            rmax = std::max(rmax, r);
        }
        out.dtmax_2d = rmax > 0.0 ? 1.0 / rmax : HUGE_VAL;
    }
    out.n_tets = nc;
    out.n_nodes = nn;
    out.perm = order;
    out.iperm.assign(nc, 0);
    for (int64_t i = 0; i < nc; ++i) out.iperm[order[i]] = (int32_t)i;

    // ---- node order: first touch along the cell order
    std::vector<int32_t> nperm(nn, -1);   // caller node -> internal node
    int32_t nnext = 0;
    for (int64_t i = 0; i < nc; ++i)
        for (int k = 0; k < nverts(in, order[i]); ++k) {
            int32_t n = in.tets[4 * (int64_t)order[i] + k];
            if (nperm[n] < 0) nperm[n] = nnext++;
        }
    for (int64_t n = 0; n < nn; ++n)      // nodes no tet uses go last
        if (nperm[n] < 0) nperm[n] = nnext++;
    // nodes belong to one medium: the 2D medium's, first touched by its
    // cells, follow the tets' (counted up to its first cell)
    out.node_2d = nn;
    if (in.split_media && out.cell_2d < nc) {
        int32_t first = nn;
        for (int k = 0; k < nverts(in, order[out.cell_2d]); ++k)
            first = std::min(first, nperm[in.tets[4 * (int64_t)order[out.cell_2d] + k]]);
        out.node_2d = first;
    }
    std::vector<int32_t> ninv(nn);
    for (int64_t n = 0; n < nn; ++n) ninv[nperm[n]] = (int32_t)n;
    {   // within windows of 1024 nodes, order by valence so that the 64-node
        // slices of the sliced-ELL gather hold nodes of equal valence (the
        // 5-tet lattice mixes valence-32 and valence-8 nodes)
        std::vector<int32_t> degree(nn, 0);
        for (int64_t c = 0; c < nc; ++c)
            for (int k = 0; k < nverts(in, c); ++k) degree[in.tets[4 * c + k]]++;
        const int64_t W = 1024;
        for (int64_t a = 0, b; a < nn; a = b) {
            b = std::min(nn, a + W);
            if (a < out.node_2d && b > out.node_2d) b = out.node_2d;   // windows stay in one medium
            std::stable_sort(ninv.begin() + a, ninv.begin() + b,
                             [&](int32_t x, int32_t y) { return degree[x] > degree[y]; });
        }
        for (int64_t i = 0; i < nn; ++i) nperm[ninv[i]] = (int32_t)i;
    }

    // ---- node gather: inverse-distance weights (step a), internal numbering
    std::vector<int64_t> ioff(nn + 1, 0);
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < nverts(in, c); ++k) ioff[nperm[in.tets[4 * c + k]] + 1]++;
    for (int64_t i = 0; i < nn; ++i) ioff[i + 1] += ioff[i];
    const int64_t n_inc = ioff[nn];
    std::vector<int32_t> icell(n_inc);
    {
        std::vector<int64_t> fill(ioff.begin(), ioff.end() - 1);
        for (int64_t i = 0; i < nc; ++i) {       // internal cell order
            int32_t c = order[i];
            for (int k = 0; k < nverts(in, c); ++k)
                icell[fill[nperm[in.tets[4 * (int64_t)c + k]]]++] = (int32_t)i;
        }
    }
    std::vector<double> iw(n_inc);
    parallel_for(nn, [&](int64_t a, int64_t b) {
        for (int64_t n = a; n < b; ++n) {
            V3 x = node(in, ninv[n]);
            double sum = 0;
            for (int64_t e = ioff[n]; e < ioff[n + 1]; ++e) {
                iw[e] = 1.0 / len(sub(x, g.cen[order[icell[e]]]));
                sum += iw[e];
            }
            for (int64_t e = ioff[n]; e < ioff[n + 1]; ++e) iw[e] /= sum;
        }
    });
    const int64_t nslice = (nn + 63) / 64;
    out.sell_off.assign(nslice + 1, 0);
    out.max_node_degree = 0;
    for (int64_t k = 0; k < nslice; ++k) {
        int64_t w = 0;
        for (int64_t n = 64 * k; n < std::min(nn, 64 * k + 64); ++n) w = std::max(w, ioff[n + 1] - ioff[n]);
        out.max_node_degree = std::max<int>(out.max_node_degree, (int)w);
        out.sell_off[k + 1] = out.sell_off[k] + 64 * w;
    }
    out.sell_padding = (double)out.sell_off[nslice] / (double)n_inc - 1.0;
    out.n_incidences = n_inc;
    out.sell_cell.assign(out.sell_off[nslice], 0);
    out.sell_w.assign(out.sell_off[nslice], 0.0);
    for (int64_t n = 0; n < nn; ++n) {
        int64_t k = n / 64, l = n % 64;
        for (int64_t e = ioff[n], s = 0; e < ioff[n + 1]; ++e, ++s) {
            out.sell_cell[out.sell_off[k] + 64 * s + l] = icell[e];
            out.sell_w[out.sell_off[k] + 64 * s + l] = iw[e];
        }
        // padding (weight 0) names a cell of the node's own medium, whose
        // potential the gather may read from that medium's substep buffers
        const int32_t pad = ioff[n + 1] > ioff[n] ? icell[ioff[n]]
                                                  : (int32_t)(n >= out.node_2d ? out.cell_2d : 0);
        const int64_t width = (out.sell_off[k + 1] - out.sell_off[k]) / 64;
        for (int64_t s = ioff[n + 1] - ioff[n]; s < width; ++s)
            out.sell_cell[out.sell_off[k] + 64 * s + l] = pad;
    }

    // ---- fused per-cell stencil (steps b-f)
    out.cnode.assign(8 * nc, 0);
    out.cbeta.assign(8 * nc, 0.0);
    out.cnbr.assign(4 * nc, 0);
    out.cb.assign(4 * nc, 0.0);
    out.vol.assign(nc, 0.0);
    out.model.assign(nc, 0);
    if (in.elliptic) {
        out.ebeta.assign(8 * nc, 0.0);
        out.eb.assign(4 * nc, 0.0);
    }
    // the stencil for the tensor of conductivities (sl, st); into L form
    // (divided by chi Cm V_c) for the time step, or flux-sum form
    struct Set { double sl, st; std::vector<double> *beta, *b; bool lform; };
    std::vector<Set> sets = {{in.sigma_l, in.sigma_t, &out.cbeta, &out.cb, true}};
    if (in.elliptic)
        sets.push_back({in.sigma_l + in.sigma_el, in.sigma_t + in.sigma_et, &out.ebeta, &out.eb, false});
    std::vector<double> rowsum(nc, 0.0);
    for (const Set &set : sets)
    parallel_for(nc, [&](int64_t a, int64_t b) {
        const double sl = set.sl, st = set.st;
        auto tensor = [&](int64_t c, double M[3][3]) {
            const double *f = in.fibre + 3 * c;
            const double s = in.scale ? in.scale[c] : 1.0;
            for (int a2 = 0; a2 < 3; ++a2)
                for (int b2 = 0; b2 < 3; ++b2)
                    M[a2][b2] = s * ((a2 == b2 ? st : 0.0) + (sl - st) * f[a2] * f[b2]);
        };
        std::vector<double> &obeta = *set.beta, &ob = *set.b;
        for (int64_t i = a; i < b; ++i) {
            const int64_t c = order[i];
            const int32_t *t = in.tets + 4 * c;
            const int nv = nverts(in, c);
            double Mc[3][3];
            tensor(c, Mc);
            // Gauss-Green with face values = means of the nv - 1 face
            // vertices: G_ck = -S_k / ((nv - 1) V_c)
            const double kvol = 1.0 / ((nv - 1) * g.vol[c]);
            double beta[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int32_t nodes[8];
            for (int k = 0; k < 4; ++k) { nodes[k] = nperm[t[k < nv ? k : 0]]; nodes[4 + k] = nodes[0]; }
            for (int f = 0; f < 4; ++f) {
                const int32_t c2 = f < nv ? g.nb[c][f] : -1;
                const int64_t slot = (int64_t)f * nc + i;
                if (c2 < 0) {                      // no-flux boundary face (or none)
                    out.cnbr[slot] = (int32_t)i;
                    ob[slot] = 0.0;
                    continue;
                }
                const int32_t *t2 = in.tets + 4 * (int64_t)c2;
                V3 xf{0, 0, 0};
                for (int k = 0; k < nv; ++k)
                    if (k != f) {
                        V3 p = node(in, t[k]);
                        for (int q = 0; q < 3; ++q) xf[q] += p[q] / (nv - 1);
                    }
                const double r1 = len(sub(g.cen[c], xf)), r2 = len(sub(g.cen[c2], xf));
                const double alpha = r2 / (r1 + r2);
                V3 dv = sub(g.cen[c2], g.cen[c]);
                const double d = len(dv);
                V3 e{dv[0] / d, dv[1] / d, dv[2] / d};
                double M2[3][3];
                tensor(c2, M2);
                V3 w{0, 0, 0};
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q)
                        w[p] += (alpha * Mc[p][q] + (1.0 - alpha) * M2[p][q]) * g.Sf[c][f][q];
                const double we = dot(w, e);
                V3 af{w[0] - we * e[0], w[1] - we * e[1], w[2] - we * e[2]};
                // own gradient
                for (int k = 0; k < nv; ++k) beta[k] -= alpha * dot(af, g.S[c][k]) * kvol;
                // neighbour gradient (same medium, so as many vertices)
                const double kvol2 = 1.0 / ((nv - 1) * g.vol[c2]);
                for (int k2 = 0; k2 < nv; ++k2) {
                    const double coef = -(1.0 - alpha) * dot(af, g.S[c2][k2]) * kvol2;
                    int own = -1;
                    for (int k = 0; k < nv; ++k) if (t[k] == t2[k2]) own = k;
                    if (own >= 0) beta[own] += coef;
                    else { beta[4 + f] = coef; nodes[4 + f] = nperm[t2[k2]]; }
                }
                out.cnbr[slot] = out.iperm[c2];
                ob[slot] = we / d;
            }
            if (!set.lform) {
                for (int s = 0; s < 8; ++s) obeta[(int64_t)s * nc + i] = beta[s];
                continue;
            }
            const double inv = 1.0 / (in.chi * in.cm * g.vol[c]);
            double rs = 0.0;
            for (int s = 0; s < 8; ++s) {
                out.cnode[(int64_t)s * nc + i] = nodes[s];
                obeta[(int64_t)s * nc + i] = beta[s] * inv;
                rs += std::fabs(beta[s] * inv);
            }
            for (int f = 0; f < 4; ++f) {
                ob[(int64_t)f * nc + i] *= inv;
                rs += 2.0 * std::fabs(ob[(int64_t)f * nc + i]);
            }
            rowsum[i] = rs;
            out.vol[i] = g.vol[c];
            out.model[i] = in.model ? in.model[c] : 0;
        }
    });
    out.max_abs_L_row = *std::max_element(rowsum.begin(), rowsum.end());
    return "";
}

}  // namespace ep
