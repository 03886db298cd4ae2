// Host-side checks of the library's precompute, built with AddressSanitizer
// and UndefinedBehaviorSanitizer (test infrastructure: it links the CPU
// oracle to check the library's host code against it).
//
//   operator   prepare() on jittered tetrahedral meshes with random fibres
//              and conductivity scales, alone and with a separate triangle
//              sheet, in the three cell orders and with the 2D medium split
//              off: the fused stencil (sliced-ELL node weights, eight node
//              coefficients, four two-point terms) applied here equals the
//              oracle's node values -> gradients -> face fluxes (Sec. 3.2,
//              eq. gra2bis) to 1e-12 of max |L|; the 2D medium's substep
//              count from prepare()'s bound equals the oracle's.
//   purkinje   prepare_purkinje() on a random branching graph with junctions:
//              the substep count equals the oracle's and every junction
//              region (mapped to caller ids) equals the oracle's.
//   coarse     build_coarse(): the aggregates partition the cells, the
//              inverse diagonal and the coarse inverse are finite.
//   admission  the server's admission rule on random queues: budget and
//              slots hold, arrival order is kept, and every skipped request
//              failed to fit at its turn.
//   errors     malformed meshes are refused with a reason, not a crash.
//
// Prints one line per check and exits nonzero on the first failure.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2112_12854_amd/csrc/admission.hpp"
#include "../../paper_2112_12854_amd/csrc/prep.hpp"
extern "C" {
#include "../../oracle/oracle.h"
}

namespace {

int g_fail = 0;

void check(bool ok, const std::string &what) {
    std::printf("%s %s\n", ok ? "ok  " : "FAIL", what.c_str());
    std::fflush(stdout);
    if (!ok) g_fail = 1;
}

// splitmix64: a small seeded generator of its own
struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed) {}
    uint64_t next() {
        uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        return z ^ (z >> 31);
    }
    double uni() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    double sym() { return 2.0 * uni() - 1.0; }
};

struct Mesh {
    std::vector<double> xyz;
    std::vector<int32_t> cells;     // 4 per cell, fourth -1 for a triangle
    std::vector<double> fibre, scale;
    std::vector<uint8_t> model;
    int64_t nn() const { return (int64_t)xyz.size() / 3; }
    int64_t nc() const { return (int64_t)cells.size() / 4; }
};

// nx*ny*nz hexes of side h, each split into six tets around its main
// diagonal (Kuhn), interior nodes moved by up to jit*h.
void add_box(Mesh &m, int nx, int ny, int nz, double h, double jit, Rng &rng) {
    const int64_t base = m.nn();
    auto id = [&](int i, int j, int k) { return (int32_t)(base + i + (nx + 1) * (j + (ny + 1) * k)); };
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                const bool inner = i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz;
                m.xyz.push_back(h * (i + (inner ? jit * rng.sym() : 0.0)));
                m.xyz.push_back(h * (j + (inner ? jit * rng.sym() : 0.0)));
                m.xyz.push_back(h * (k + (inner ? jit * rng.sym() : 0.0)));
            }
    static const int kuhn[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7},
                                   {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                for (const auto &t : kuhn)
                    for (int q = 0; q < 4; ++q) {
                        const int c = t[q];
                        m.cells.push_back(id(i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1)));
                    }
}

// a flat sheet of nx*ny squares of side h at height z0, two triangles each
void add_sheet(Mesh &m, int nx, int ny, double h, double z0, Rng &rng) {
    const int64_t base = m.nn();
    auto id = [&](int i, int j) { return (int32_t)(base + i + (nx + 1) * j); };
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            const bool inner = i > 0 && i < nx && j > 0 && j < ny;
            m.xyz.push_back(h * (i + (inner ? 0.15 * rng.sym() : 0.0)));
            m.xyz.push_back(h * (j + (inner ? 0.15 * rng.sym() : 0.0)));
            m.xyz.push_back(z0);
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int32_t a = id(i, j), b = id(i + 1, j), c = id(i, j + 1), d = id(i + 1, j + 1);
            for (int32_t v : {a, b, d, -1}) m.cells.push_back(v);
            for (int32_t v : {a, d, c, -1}) m.cells.push_back(v);
        }
}

void finish(Mesh &m, Rng &rng) {
    const int64_t nc = m.nc();
    m.fibre.resize(3 * nc);
    m.scale.resize(nc);
    m.model.assign(nc, 0);
    for (int64_t c = 0; c < nc; ++c) {
        double f[3], n = 0;
        for (double &x : f) { x = rng.sym(); n += x * x; }
        n = std::sqrt(n);
        const bool tri = m.cells[4 * c + 3] < 0;
        if (tri) { f[2] = 0.0; n = std::hypot(f[0], f[1]); }   // fibres in the sheet
        for (int a = 0; a < 3; ++a) m.fibre[3 * c + a] = f[a] / n;
        m.scale[c] = 0.5 + 1.5 * rng.uni();
        m.model[c] = (uint8_t)(rng.uni() < 0.3 ? 3 : 0);     // TP06 and CRN cells
    }
}

ep::PrepIn prep_in(const Mesh &m, int ordering, bool split) {
    ep::PrepIn in;
    in.n_nodes = m.nn();
    in.n_tets = m.nc();
    in.xyz = m.xyz.data();
    in.tets = m.cells.data();
    in.fibre = m.fibre.data();
    in.scale = m.scale.data();
    in.model = m.model.data();
    in.sigma_l = 0.17;
    in.sigma_t = 0.019;
    in.chi = 140.0;
    in.cm = 0.01;
    in.ordering = ordering;
    in.split_media = split;
    return in;
}

orc_sim *oracle_of(const Mesh &m, double dt = 0.02) {
    return orc_create(m.nn(), m.xyz.data(), m.nc(), m.cells.data(), m.fibre.data(), 0.17, 0.019,
                      m.scale.data(), m.model.data(), dt, 140.0, 0.01);
}

// The fused stencil of a prepared mesh applied to caller-order potentials v.
std::vector<double> fused_apply(const ep::PrepOut &P, const std::vector<double> &v) {
    const int64_t nc = P.n_tets, nn = P.n_nodes;
    std::vector<double> vi(nc), vn(nn, 0.0), L(nc);
    for (int64_t i = 0; i < nc; ++i) vi[i] = v[P.perm[i]];
    for (int64_t n = 0; n < nn; ++n) {
        const int64_t k = n / 64, l = n % 64;
        const int64_t w = (P.sell_off[k + 1] - P.sell_off[k]) / 64;
        double a = 0.0;
        for (int64_t s = 0; s < w; ++s) {
            const int64_t e = P.sell_off[k] + 64 * s + l;
            a += P.sell_w[e] * vi[P.sell_cell[e]];
        }
        vn[n] = a;
    }
    for (int64_t c = 0; c < nc; ++c) {
        double s = 0.0;
        for (int q = 0; q < 8; ++q) s += P.cbeta[q * nc + c] * vn[P.cnode[q * nc + c]];
        for (int f = 0; f < 4; ++f) s += P.cb[f * nc + c] * (vi[P.cnbr[f * nc + c]] - vi[c]);
        L[P.perm[c]] = s;
    }
    return L;
}

void check_operator(const char *name, const Mesh &m, Rng &rng) {
    orc_sim *o = oracle_of(m);
    std::vector<double> v(m.nc()), Lo(m.nc());
    for (double &x : v) x = -80.0 + 30.0 * rng.sym();
    orc_apply_diffusion(o, v.data(), Lo.data());
    double scale = 0.0;
    for (double x : Lo) scale = std::max(scale, std::fabs(x));
    for (int ord = 0; ord < 3; ++ord)
        for (int split = 0; split < 2; ++split) {
            ep::PrepOut P;
            const std::string e = ep::prepare(prep_in(m, ord, split != 0), P);
            if (!e.empty()) { check(false, std::string(name) + ": prepare: " + e); continue; }
            const std::vector<double> L = fused_apply(P, v);
            double err = 0.0;
            for (int64_t c = 0; c < m.nc(); ++c) err = std::max(err, std::fabs(L[c] - Lo[c]));
            char buf[200];
            std::snprintf(buf, sizeof buf, "%s order %d split %d: fused stencil vs oracle, max|dL|/max|L| = %.2e",
                          name, ord, split, err / scale);
            check(err <= 1e-12 * scale, buf);
            // the permutation is one, and the split keeps each medium together
            std::vector<int> seen(m.nc(), 0);
            bool perm_ok = true;
            for (int32_t c : P.perm) perm_ok = perm_ok && c >= 0 && c < m.nc() && !seen[c]++;
            bool media_ok = true;
            for (int64_t i = 0; i < m.nc(); ++i)
                media_ok = media_ok && ((m.cells[4 * (int64_t)P.perm[i] + 3] < 0) == (split && i >= P.cell_2d));
            check(perm_ok && (media_ok || !split || P.cell_2d == m.nc()),
                  std::string(name) + ": permutation and media split");
            // every slot a node's gather reads, padding included, names a
            // cell of the node's own medium (the substep buffers of the 2D
            // medium hold only its cells)
            bool pad_ok = true;
            for (int64_t n = 0; n < P.n_nodes; ++n) {
                const int64_t k = n / 64, l = n % 64;
                for (int64_t e = P.sell_off[k] + l; e < P.sell_off[k + 1]; e += 64)
                    pad_ok = pad_ok && (P.sell_cell[e] >= P.cell_2d) == (n >= P.node_2d);
            }
            check(pad_ok, std::string(name) + ": node gathers stay in their medium");
        }
    // the 2D medium's derived substep count
    bool has_tri = false;
    for (int64_t c = 0; c < m.nc(); ++c) has_tri = has_tri || m.cells[4 * c + 3] < 0;
    if (has_tri) {
        ep::PrepOut P;
        ep::prepare(prep_in(m, 0, true), P);
        for (const double dt : {0.02, 0.005}) {
            int32_t k = 1;
            while (dt / k > 0.9 * P.dtmax_2d) ++k;
            orc_sim *q = oracle_of(m, dt);
            orc_set_medium_substeps(q, 0);
            char buf[160];
            std::snprintf(buf, sizeof buf, "%s: 2D substeps at dt %.3f: library %d, oracle %d", name, dt, k,
                          orc_medium_substeps(q));
            check(k == orc_medium_substeps(q), buf);
            orc_destroy(q);
        }
    }
    orc_destroy(o);
}

void check_purkinje(Rng &rng) {
    Mesh m;
    add_box(m, 10, 8, 3, 0.5, 0.2, rng);
    finish(m, rng);
    // a random branching graph above the box: each new node hangs off a
    // random earlier one, at 0.2-0.6 mm
    const int np = 300;
    std::vector<double> pxyz = {2.5, 2.0, 0.7};
    std::vector<int32_t> edges;
    for (int i = 1; i < np; ++i) {
        const int p = (int)(rng.uni() * i);
        const double len = 0.2 + 0.4 * rng.uni(), th = 6.283185307179586 * rng.uni();
        pxyz.push_back(std::min(4.9, std::max(0.1, pxyz[3 * p] + len * std::cos(th))));
        pxyz.push_back(std::min(3.9, std::max(0.1, pxyz[3 * p + 1] + len * std::sin(th))));
        pxyz.push_back(0.3 + 1.0 * rng.uni());
        edges.push_back(p);
        edges.push_back(i);
    }
    const std::vector<int32_t> pmj_nodes = {5, 77, 150, 299};
    orc_sim *o = oracle_of(m);
    orc_set_purkinje(o, np, pxyz.data(), (int64_t)edges.size() / 2, edges.data(), nullptr, 3.95, 4, 0);
    for (int32_t q : pmj_nodes) orc_add_pmj(o, q, 0.4, 5.0, 3.0, 1, -200.0, 0.5);
    ep::PrepIn tin = prep_in(m, 0, false);
    ep::PrepOut tout;
    check(ep::prepare(tin, tout).empty(), "purkinje: tissue prepared");
    ep::PurkIn pin;
    pin.n = np;
    pin.n_edges = (int64_t)edges.size() / 2;
    pin.xyz = pxyz.data();
    pin.edges = edges.data();
    pin.sigma = 3.95;
    pin.dt = 0.02;
    for (int32_t q : pmj_nodes) {
        ep::PmjIn j;
        j.node = q;
        j.radius = 0.4;
        j.two_way = 1;
        pin.pmjs.push_back(j);
    }
    ep::PurkOut pout;
    const std::string e = ep::prepare_purkinje(pin, tin, tout, pout);
    check(e.empty(), "purkinje: prepared " + e);
    if (!e.empty()) { orc_destroy(o); return; }
    char buf[160];
    std::snprintf(buf, sizeof buf, "purkinje: substeps library %d, oracle %d", pout.n_sub, orc_purkinje_n_sub(o));
    check(pout.n_sub == orc_purkinje_n_sub(o), buf);
    bool regions = pout.jroff.size() == pmj_nodes.size() + 1;
    for (size_t k = 0; regions && k < pmj_nodes.size(); ++k) {
        std::vector<int32_t> lib;
        for (int32_t i = pout.jroff[k]; i < pout.jroff[k + 1]; ++i) lib.push_back(tout.perm[pout.jcells[i]]);
        std::sort(lib.begin(), lib.end());
        std::vector<int32_t> ref(m.nc());
        ref.resize(orc_get_pmj_region(o, (int)k, ref.data(), m.nc()));
        std::sort(ref.begin(), ref.end());
        regions = regions && lib == ref && !lib.empty();
    }
    check(regions, "purkinje: every junction region equals the oracle's");
    orc_destroy(o);
}

void check_coarse(Rng &rng) {
    Mesh m;
    add_box(m, 12, 10, 4, 0.5, 0.2, rng);
    finish(m, rng);
    ep::PrepIn in = prep_in(m, 0, false);
    in.elliptic = true;
    in.sigma_el = 0.62;
    in.sigma_et = 0.24;
    ep::PrepOut P;
    check(ep::prepare(in, P).empty(), "coarse: bidomain operator prepared");
    ep::Coarse C;
    const std::string e = ep::build_coarse(in, P, 64, C);
    check(e.empty(), "coarse: aggregates built " + e);
    if (!e.empty()) return;
    const int64_t nc = m.nc();
    std::vector<int> seen(nc, 0);
    bool ok = C.n_agg > 1 && (int64_t)C.agg_of.size() == nc && (int)C.agg_off.size() == C.n_agg + 1 &&
              C.agg_off[0] == 0 && C.agg_off[C.n_agg] == nc;
    for (int32_t a = 0; ok && a < C.n_agg; ++a) {
        ok = C.agg_off[a + 1] > C.agg_off[a];
        for (int32_t i = C.agg_off[a]; ok && i < C.agg_off[a + 1]; ++i) {
            const int32_t c = C.agg_cells[i];
            ok = c >= 0 && c < nc && !seen[c]++ && C.agg_of[c] == a;
        }
    }
    // the flux-sum operator's diagonal has one sign (negative): D^-1 too
    for (double x : C.dinv) ok = ok && std::isfinite(x) && x * C.dinv[0] > 0.0;
    for (double x : C.cinv) ok = ok && std::isfinite(x);
    check(ok, "coarse: aggregates partition the cells, finite inverses (" + std::to_string(C.n_agg) + ")");
}

void check_admission(Rng &rng) {
    bool ok = true;
    for (int trial = 0; trial < 2000 && ok; ++trial) {
        const size_t n = (size_t)(rng.uni() * 20);
        const size_t budget = 1 + (size_t)(rng.uni() * 1000);
        size_t used0 = (size_t)(rng.uni() * budget);
        const size_t slots = (size_t)(rng.uni() * 8);
        std::vector<size_t> fp(n);
        for (size_t &f : fp) f = (size_t)(rng.uni() * 400);
        if (trial % 7 == 0 && n) fp[0] = (size_t)-1;   // beyond any budget
        size_t used = used0;
        const std::vector<size_t> pick = ep::admit_ready(fp, used, budget, slots);
        // budget, slots and order
        size_t sum = used0;
        for (size_t i = 0; i < pick.size(); ++i) {
            ok = ok && pick[i] < n && (i == 0 || pick[i] > pick[i - 1]);
            if (ok) sum += fp[pick[i]];
        }
        ok = ok && sum == used && used <= budget && pick.size() <= slots;
        // a request skipped before the slots ran out did not fit at its turn
        size_t run = used0, k = 0;
        for (size_t i = 0; ok && i < n && k < slots; ++i) {
            if (k < pick.size() && pick[k] == i) { run += fp[i]; ++k; continue; }
            ok = fp[i] > budget || run + fp[i] > budget;
        }
    }
    check(ok, "admission: budget, slots, arrival order and skips on 2000 random queues");
}

void check_errors() {
    Mesh m;
    Rng rng(5);
    add_box(m, 2, 2, 1, 1.0, 0.0, rng);
    finish(m, rng);
    {   // a degenerate tet
        Mesh d = m;
        d.cells[1] = d.cells[0];
        ep::PrepOut P;
        check(!ep::prepare(prep_in(d, 0, false), P).empty(), "errors: a degenerate cell is refused");
    }
    {   // a face shared by three cells
        Mesh d = m;
        for (int q = 0; q < 4; ++q) d.cells.push_back(d.cells[q]);
        d.fibre.insert(d.fibre.end(), {1.0, 0.0, 0.0});
        d.scale.push_back(1.0);
        d.model.push_back(0);
        ep::PrepOut P;
        check(!ep::prepare(prep_in(d, 0, false), P).empty(), "errors: a non-manifold face is refused");
    }
    {   // a node shared by a tet and a triangle
        Mesh d = m;
        for (int32_t v : {d.cells[0], d.cells[1], d.cells[2], -1}) d.cells.push_back(v);
        d.fibre.insert(d.fibre.end(), {1.0, 0.0, 0.0});
        d.scale.push_back(1.0);
        d.model.push_back(0);
        ep::PrepOut P;
        check(!ep::prepare(prep_in(d, 0, false), P).empty(), "errors: a node of both media is refused");
    }
}

}  // namespace

int main() {
    orc_set_num_threads(1);
    Rng rng(20211224);
    {
        Mesh m;
        add_box(m, 9, 7, 4, 0.5, 0.2, rng);
        finish(m, rng);
        check_operator("tets", m, rng);
    }
    {
        Mesh m;
        add_box(m, 6, 5, 3, 0.5, 0.2, rng);
        add_sheet(m, 14, 9, 0.25, 2.5, rng);
        finish(m, rng);
        check_operator("tets+sheet", m, rng);
    }
    check_purkinje(rng);
    check_coarse(rng);
    check_admission(rng);
    check_errors();
    std::printf(g_fail ? "host checks FAILED\n" : "host checks passed\n");
    return g_fail;
}
