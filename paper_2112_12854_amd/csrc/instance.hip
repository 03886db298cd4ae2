// Building instances on the device and stepping sets of them.
#include "instance.hpp"

#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace ep {

using namespace epdev;

int model_ng(int m) {
    if (m <= 2) return tp06::NG;
    if (m == 3) return crn::NG;
    if (m == 4) return stewart::NG;
    return 0;
}
int model_nc(int m) {
    if (m <= 2) return tp06::NC;
    if (m == 3) return crn::NC;
    if (m == 4) return stewart::NC;
    return 0;
}
void model_init(int m, double *y) {
    for (int i = 0; i < EP_MAX_SLOTS; ++i) y[i] = 0.0;
    if (m <= 2) tp06::init(y);
    else if (m == 3) crn::init(y);
    else if (m == 4) stewart::init(y);
    else y[0] = -86.2;
}

namespace {

void *raw_alloc(Inst &in, size_t bytes) {
    void *p = nullptr;
    if (in.al.alloc) p = in.al.alloc(bytes, in.al.ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    return p;
}

void *dalloc(Inst &in, size_t bytes) {
    const size_t r = (std::max<size_t>(bytes, 256) + 255) / 256 * 256;
    if (in.arena && in.arena_used + r <= in.arena_size) {
        void *p = in.arena + in.arena_used;
        in.arena_used += r;
        return p;
    }
    void *p = raw_alloc(in, r);
    if (p) {
        in.allocs.push_back({p, r});
        in.footprint += r;
    }
    return p;
}

template <typename T>
bool up(Inst &in, void **dst, const std::vector<T> &src) {
    *dst = dalloc(in, src.size() * sizeof(T));
    if (!*dst) return false;
    // synchronous: sources are often temporaries
    return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

// Zero-filled device array (set-up only: a synchronous fill).
void *zalloc(Inst &in, size_t bytes) {
    void *p = dalloc(in, bytes);
    if (p && hipMemset(p, 0, bytes) != hipSuccess) return nullptr;
    return p;
}

template <typename R>
std::vector<R> conv(const std::vector<double> &v) {
    return std::vector<R>(v.begin(), v.end());
}

size_t round256(size_t b) { return (std::max<size_t>(b, 256) + 255) / 256 * 256; }

// Per 256-cell block, the smallest id over the S slot-major rows of `a`
// (into *base when given); false when some block's ids span more than 65,535.
bool block_bases(const std::vector<int32_t> &a, int S, int64_t n, std::vector<int32_t> *base) {
    const int64_t nb = (n + LB - 1) / LB;
    if (base) base->assign(nb, 0);
    for (int64_t b = 0; b < nb; ++b) {
        int32_t lo = INT32_MAX, hi = INT32_MIN;
        for (int s = 0; s < S; ++s)
            for (int64_t c = b * LB; c < std::min<int64_t>(n, (b + 1) * LB); ++c) {
                const int32_t x = a[(size_t)s * n + c];
                lo = std::min(lo, x);
                hi = std::max(hi, x);
            }
        if ((int64_t)hi - lo > 65535) return false;
        if (base) (*base)[b] = lo;
    }
    return true;
}

// tile-major 16-bit offsets of the ids of `a` from their block's base
std::vector<uint16_t> offsets16(const std::vector<int32_t> &a, int S, int64_t n,
                                const std::vector<int32_t> &base) {
    std::vector<uint16_t> t(tiled_len(n, S), 0);
    for (int s = 0; s < S; ++s)
        for (int64_t c = 0; c < n; ++c) t[tix(c, s, S)] = (uint16_t)(a[(size_t)s * n + c] - base[c / LB]);
    return t;
}

// slot-major [S][n] host array -> the device's tile-major layout
template <typename T>
std::vector<T> tiled(const std::vector<T> &a, int S, int64_t n) {
    std::vector<T> t(tiled_len(n, S), T(0));
    for (int s = 0; s < S; ++s)
        for (int64_t c = 0; c < n; ++c) t[tix(c, s, S)] = a[(size_t)s * n + c];
    return t;
}

}  // namespace

size_t estimate_footprint(int64_t nc, int64_t nn, int rs, int max_degree_hint) {
    (void)max_degree_hint;
    const size_t c = (size_t)nc, n = (size_t)nn, r = (size_t)rs;
    const size_t ent = (size_t)(4.4 * c) + 64 * 8;   // incidences incl. slice padding
    size_t b = 0;
    b += round256(((n + 63) / 64 + 1) * 8) + round256(ent * 4) + round256(ent * r);
    b += round256(tiled_len(c, 8) * 4) + round256(tiled_len(c, 8) * r) + round256(tiled_len(c, 4) * 4) +
         round256(tiled_len(c, 4) * r);
    b += round256(c) + round256(c * 8);                       // model, volume
    b += round256(c * 4) + round256(c * 4);                   // stimulus mask, permutation
    b += round256(tiled_len(c, NC_MAX) * 8) + round256(tiled_len(c, NG_MAX) * r);   // states
    b += 2 * round256(c * r) + 3 * round256(c * r) + round256(n * r);   // v0 v1 vrest vmax, vn
    b += round256(c) + 2 * round256(c * 8);                   // detection
    b += round256(((c + 63) / 64 + 12) * 8) + round256(8 * 4096) + round256(sizeof(Ctrl));
    return b;
}

std::string spec_set_purkinje(InstSpec &sp, int64_t n, const double *xyz, int64_t n_edges,
                              const int32_t *edges, double sigma, int32_t model, int32_t n_sub) {
    if (n <= 0 || n >= ((int64_t)1 << 25) || !xyz || n_edges < 0 || (n_edges > 0 && !edges))
        return "empty graph or null array";
    if (!(sigma > 0) || !std::isfinite(sigma)) return "sigma must be > 0";
    if (model < 0 || model > EP_PASSIVE) return "model id out of range";
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(xyz[i])) return "non-finite node coordinate";
    for (int64_t e = 0; e < 2 * n_edges; ++e)
        if (edges[e] < 0 || edges[e] >= n) return "edge node index out of range";
    // junctions of cells outlive a change of graph; those of graph nodes do not
    std::vector<PmjIn> keep;
    for (const PmjIn &q : sp.purk.pmjs)
        if (q.cell >= 0) keep.push_back(q);
    sp.purk = PurkSpec();
    sp.purk.pmjs = keep;
    sp.purk.n = n;
    sp.purk.xyz.assign(xyz, xyz + 3 * n);
    sp.purk.edges.assign(edges, edges + 2 * n_edges);
    sp.purk.sigma = sigma;
    sp.purk.model = model;
    sp.purk.n_sub = n_sub;
    return "";
}

std::string spec_set_purkinje_scale(InstSpec &sp, int64_t n_edges, const double *scale) {
    PurkSpec &pk = sp.purk;
    if (n_edges != (int64_t)pk.edges.size() / 2 || (n_edges > 0 && !scale))
        return "one scale per graph segment";
    for (int64_t e = 0; e < n_edges; ++e)
        if (!(scale[e] >= 0.0) || !std::isfinite(scale[e]))
            return "segment scales must be finite and >= 0";
    pk.edge_scale.assign(scale, scale + n_edges);
    return "";
}

namespace {
std::string add_junction(InstSpec &sp, int32_t node, int32_t cell, double radius, double delay_ortho,
                         double delay_anti, int32_t two_way, double amp, double dur) {
    PurkSpec &pk = sp.purk;
    if (!(radius >= 0) || !std::isfinite(radius) || !(delay_ortho >= 0) || !(delay_anti >= 0) ||
        !std::isfinite(delay_ortho) || !std::isfinite(delay_anti) || !std::isfinite(amp) ||
        !(dur >= 0) || !std::isfinite(dur))
        return "bad junction parameters";
    if (pk.pmjs.size() >= (size_t)1 << 24) return "too many junctions";
    PmjIn q;
    q.node = node;
    q.cell = cell;
    q.radius = radius;
    q.delay_ortho = delay_ortho;
    q.delay_anti = delay_anti;
    q.two_way = two_way ? 1 : 0;
    q.amp = amp;
    q.dur = dur;
    pk.pmjs.push_back(q);
    return "";
}
}  // namespace

std::string spec_add_pmj(InstSpec &sp, int32_t node, double radius, double delay_ortho,
                         double delay_anti, int32_t two_way, double amp, double dur) {
    if (node < 0 || node >= sp.purk.n) return "junction node out of range";
    return add_junction(sp, node, -1, radius, delay_ortho, delay_anti, two_way, amp, dur);
}

std::string spec_add_cell_junction(InstSpec &sp, int32_t cell, double radius, double delay_ortho,
                                   double delay_anti, int32_t two_way, double amp, double dur) {
    if (cell < 0 || cell >= sp.n_tets) return "junction source cell out of range";
    return add_junction(sp, -1, cell, radius, delay_ortho, delay_anti, two_way, amp, dur);
}

std::string spec_add_stimulus(InstSpec &sp, int domain, int64_t n_ids, const int32_t *ids,
                              double t0, double dur, double amp, double period, int32_t count) {
    if (domain != 0 && domain != 1) return "domain must be 0 (tissue) or 1 (graph)";
    if ((int)sp.stims.size() >= EP_MAX_STIMULI) return "too many stimuli";
    if (n_ids < 0 || (n_ids > 0 && !ids) || !(dur >= 0) || !std::isfinite(amp) || !(period >= 0) ||
        !std::isfinite(t0) || !std::isfinite(dur) || !std::isfinite(period))
        return "bad stimulus";
    const int64_t lim = domain == 0 ? sp.n_tets : sp.purk.n;
    for (int64_t i = 0; i < n_ids; ++i)
        if (ids[i] < 0 || ids[i] >= lim) return "stimulus id out of range";
    StimSpec st;
    st.domain = domain;
    st.ids.assign(ids, ids + n_ids);
    st.t0 = t0; st.dur = dur; st.amp = amp; st.period = period;
    st.count = count < 1 ? 1 : count;
    sp.stims.push_back(std::move(st));
    return "";
}

std::string prep_instance(const InstSpec &sp, Inst &I, ep_status &st) {
    st = EP_OK;
    PrepIn in;
    in.n_nodes = sp.n_nodes;
    in.n_tets = sp.n_tets;
    in.xyz = sp.xyz.data();
    in.tets = sp.tets.data();
    in.fibre = sp.fibre.data();
    in.scale = sp.has_scale ? sp.scale.data() : nullptr;
    in.model = sp.model.data();
    in.sigma_l = sp.sigma_l;
    in.sigma_t = sp.sigma_t;
    in.chi = sp.chi;
    in.cm = sp.cm;
    in.ordering = sp.ordering;
    in.elliptic = sp.bido;
    in.sigma_el = sp.sigma_el;
    in.sigma_et = sp.sigma_et;
    in.split_media = sp.medium_substeps != 1;
    std::string e = prepare(in, I.prep);
    if (!e.empty()) { st = EP_EINVAL; return e; }
    I.c2 = I.prep.cell_2d;
    I.n2 = I.prep.node_2d;
    I.sub2 = 1;
    if (I.c2 < I.prep.n_tets) {
        if (sp.bido) { st = EP_EINVAL; return "a 2D medium with substeps is not available with the bidomain model"; }
        if (sp.medium_substeps > 1) {
            I.sub2 = sp.medium_substeps;
        } else {
            const double lim = (sp.scheme >= 1 ? 0.45 : 0.9) * I.prep.dtmax_2d;
            int32_t k = 1;
            while (sp.dt / k > lim && k < (1 << 20)) ++k;
            I.sub2 = k;
        }
    }
    // 16-bit stencil ids when every block allows them (the elliptic operator
    // of the bidomain model reads the 32-bit ones)
    I.idx16 = !sp.bido && block_bases(I.prep.cnode, 8, I.prep.n_tets, nullptr) &&
              block_bases(I.prep.cnbr, 4, I.prep.n_tets, nullptr);
    I.coarse = Coarse();
    if (sp.bido && sp.bido_coarse > 0) {
        e = build_coarse(in, I.prep, sp.bido_coarse, I.coarse);
        if (!e.empty()) { st = EP_EINVAL; return e; }
    }
    I.pk = PurkOut();
    I.n_pmj = 0;
    if (sp.purk.n > 0 || !sp.purk.pmjs.empty()) {
        PurkIn pin;
        pin.n = sp.purk.n;
        pin.n_edges = (int64_t)sp.purk.edges.size() / 2;
        pin.xyz = sp.purk.xyz.data();
        pin.edges = sp.purk.edges.data();
        pin.edge_scale = sp.purk.edge_scale.empty() ? nullptr : sp.purk.edge_scale.data();
        pin.sigma = sp.purk.sigma;
        pin.dt = sp.dt;
        pin.chi = sp.chi;
        pin.cm = sp.cm;
        pin.n_sub = sp.purk.n_sub;
        pin.ab2 = sp.scheme >= 1;
        pin.pmjs = sp.purk.pmjs;
        e = prepare_purkinje(pin, in, I.prep, I.pk);
        if (!e.empty()) { st = EP_EINVAL; return e; }
        I.pmodel = sp.purk.model;
        I.n_pmj = (int64_t)sp.purk.pmjs.size();
    }
    return "";
}

namespace {

size_t purkinje_bytes(const Inst &I, int rs) {
    if (!has_junction_block(I)) return 0;
    const size_t np = (size_t)I.pk.n, E = I.pk.nbr.size(), r = (size_t)rs, c = (size_t)I.prep.n_tets;
    size_t b = round256((np + 1) * 4) + round256(E * 4) + round256(E * r);
    b += 2 * round256(np * r) + round256(tiled_len(np, NG_MAX) * r) + round256(tiled_len(np, NC_MAX) * 8);
    b += round256(np * 4) + round256(np) + round256(np * 8) + round256(np * 4);
    b += round256((np + (size_t)I.n_pmj + 1) * 4) + round256(std::max<size_t>(I.n_pmj, 1) * sizeof(Pmj));
    b += round256(std::max<size_t>(I.pk.jcells.size(), 1) * 4);
    b += round256(c * 4) + round256(I.pk.cpmj_list.size() * 4);
    return b;
}

}  // namespace

size_t instance_footprint(const Inst &I, int rs, const InstSpec &sp) {
    const PrepOut &P = I.prep;
    const size_t c = (size_t)P.n_tets, n = (size_t)P.n_nodes, r = (size_t)rs;
    const size_t ent = P.sell_cell.size();
    int64_t cap = 4096;
    if (sp.trace_every > 0 && sp.target != INT64_MAX) cap = std::max<int64_t>(2, sp.target / sp.trace_every + 2);
    else if (sp.trace_every > 0) cap = 1 << 16;
    size_t b = 0;
    b += round256(P.sell_off.size() * 8) + round256(ent * 4) + round256(ent * r);
    if (I.idx16)
        b += round256(tiled_len(c, 8) * 2) + round256(tiled_len(c, 4) * 2) + 2 * round256((c + LB - 1) / LB * 4);
    else
        b += round256(tiled_len(c, 8) * 4) + round256(tiled_len(c, 4) * 4);
    b += round256(tiled_len(c, 8) * r) + round256(tiled_len(c, 4) * r);
    b += round256(c) + round256(c * 8) + round256(c * 4) + round256(c * 4);
    b += round256(tiled_len(c, NC_MAX) * 8) + round256(tiled_len(c, NG_MAX) * r);
    b += 4 * round256(c * r) + round256(n * r);
    b += round256(c) + 2 * round256(c * 8);
    b += round256((size_t)cap * 8) + round256(((c + 63) / 64 + 12) * 8) + round256(sizeof(Ctrl));
    if (sp.bido) {
        const size_t m1 = (size_t)sp.bido_restart + 1;
        b += round256(tiled_len(c, 8) * 8) + round256(tiled_len(c, 4) * 8) + 3 * round256(c * 8) +
             round256(n * 8) + round256(m1 * c * 8);
        b += round256(2 * m1 * bido_part_cols((int64_t)c) * 8) + round256((2 * m1 + 2) * 8) + round256(m1 * 8) +
             round256(gmres_state_doubles((int)m1 - 1) * 8);
        const size_t na = (size_t)I.coarse.n_agg;
        if (na > 0)
            b += 2 * round256(c * 4) + round256((na + 1) * 4) + round256(c * 8) +
                 round256(na * na * 4) + 2 * round256(c * 8) + 2 * round256(na * 8);
    }
    if (sp.scheme >= 1) {
        b += round256(c * r) + round256(tiled_len(c, NC_MAX) * 8);
        if (I.pk.n > 0) b += round256((size_t)I.pk.n * r) + round256(tiled_len(I.pk.n, NC_MAX) * 8);
    }
    if (I.c2 < P.n_tets) b += 2 * round256((size_t)(P.n_tets - I.c2) * r);   // substep potentials
    return b + purkinje_bytes(I, rs);
}

namespace {

// Graph arrays, junction table and the muscle's junction lists.
std::string upload_purkinje(const InstSpec &sp, int rs, Inst &I, ep_status &st) {
    const PurkOut &K = I.pk;
    const int64_t np = K.n;
    PurkDesc &P = I.pdesc;
    std::memset(&P, 0, sizeof(P));
    auto fail_mem = [&]() { st = EP_ENOMEM; free_instance(I); return std::string("device allocation failed"); };
    std::vector<double> v0(np), gate(tiled_len(np, NG_MAX), 0.0), conc(tiled_len(np, NC_MAX), 0.0);
    {
        double y[EP_MAX_SLOTS];
        model_init(I.pmodel, y);
        const int ng = model_ng(I.pmodel), ncc = model_nc(I.pmodel);
        for (int64_t i = 0; i < np; ++i) {
            v0[i] = y[0];
            for (int k = 0; k < ng; ++k) gate[tix(i, k, NG_MAX)] = y[1 + k];
            for (int k = 0; k < ncc; ++k) conc[tix(i, k, NC_MAX)] = y[1 + ng + k];
        }
    }
    std::vector<uint32_t> pmask(np, 0);
    for (size_t k = 0; k < sp.stims.size(); ++k)
        if (sp.stims[k].domain == 1)
            for (int32_t id : sp.stims[k].ids) pmask[id] |= 1u << k;
    // per node: its two-way junctions, in junction order
    std::vector<int32_t> npmj(np, -1), nlist;
    {
        std::vector<std::vector<int32_t>> at(np);
        for (size_t k = 0; k < sp.purk.pmjs.size(); ++k)
            if (sp.purk.pmjs[k].two_way && sp.purk.pmjs[k].cell < 0)
                at[sp.purk.pmjs[k].node].push_back((int32_t)k);
        for (int64_t i = 0; i < np; ++i)
            if (!at[i].empty()) {
                npmj[i] = (int32_t)nlist.size();
                for (int32_t k : at[i]) nlist.push_back(k);
                nlist.push_back(-1);
            }
        if (nlist.empty()) nlist.push_back(-1);
    }
    std::vector<Pmj> pmj(std::max<size_t>(sp.purk.pmjs.size(), 1));
    for (size_t k = 0; k < sp.purk.pmjs.size(); ++k) {
        const PmjIn &q = sp.purk.pmjs[k];
        Pmj &J = pmj[k];
        J.fire_o = J.fire_a = INT64_MIN / 2;
        J.delay_o = std::llround(q.delay_ortho / sp.dt);
        J.delay_a = std::llround(q.delay_anti / sp.dt);
        J.ndur = std::llround(q.dur / sp.dt);
        J.amp = q.amp;
        J.vprev = q.cell >= 0 ? 0.0 : rs == 8 ? v0[q.node] : (double)(float)v0[q.node];
        J.node = q.node;
        J.src_cell = K.jsrc[k];
        J.two_way = q.two_way ? 1 : 0;
        J.roff = K.jroff[k];
        J.rcnt = K.jroff[k + 1] - K.jroff[k];
    }
    const double nan = std::numeric_limits<double>::quiet_NaN();
    std::vector<int32_t> jc = K.jcells;
    if (jc.empty()) jc.push_back(0);
    bool ok = up(I, (void **)&P.off, K.off) && up(I, (void **)&P.nbr, K.nbr) &&
              up(I, (void **)&P.conc, conc) && up(I, (void **)&P.pmask, pmask) &&
              up(I, (void **)&P.pstat, std::vector<uint8_t>(np, 0)) &&
              up(I, (void **)&P.pt_act, std::vector<double>(np, nan)) &&
              up(I, (void **)&P.npmj, npmj) && up(I, (void **)&P.npmj_list, nlist) &&
              up(I, (void **)&P.pmj, pmj) && up(I, (void **)&P.jcells, jc) &&
              up(I, (void **)&I.desc.cpmj, K.cpmj) && up(I, (void **)&I.desc.cpmj_list, K.cpmj_list);
    if (!ok) return fail_mem();
    if (rs == 8)
        ok = up(I, (void **)&P.g, K.g) && up(I, &P.pv[0], v0) && up(I, &P.pv[1], v0) &&
             up(I, &P.gate, gate);
    else
        ok = up(I, (void **)&P.g, conv<float>(K.g)) && up(I, &P.pv[0], conv<float>(v0)) &&
             up(I, &P.pv[1], conv<float>(v0)) && up(I, &P.gate, conv<float>(gate));
    if (!ok) return fail_mem();
    I.desc.pmj = P.pmj;
    P.np = np;
    P.n_sub = K.n_sub;
    P.n_pmj = (int32_t)sp.purk.pmjs.size();
    P.model = I.pmodel;
    P.tv[0] = I.desc.v[0];
    P.tv[1] = I.desc.v[1];
    if (sp.scheme >= 1) {
        P.hv = zalloc(I, (size_t)np * rs);
        P.hc = (double *)zalloc(I, tiled_len(np, NC_MAX) * 8);
        if (!P.hv || !P.hc) return fail_mem();
    }
    P.ctrl = I.d_ctrl;
    P.dtp = sp.dt / K.n_sub;
    P.thr = sp.thr;
    P.gs = I.desc.gs;
    return "";
}

}  // namespace

std::string upload_instance(const InstSpec &sp, int rs, const Allocator &al, Inst &I,
                            ep_status &st) {
    st = EP_OK;
    I.rs = rs;
    I.al = al;
    PrepOut &P = I.prep;
    I.arena_size = instance_footprint(I, rs, sp);
    I.arena_used = 0;
    I.arena = (char *)raw_alloc(I, I.arena_size);
    if (!I.arena) {
        st = EP_ENOMEM;
        I.arena_size = 0;
        return "device allocation failed";
    }
    I.footprint = I.arena_size;
    const int64_t nc = sp.n_tets, nn = sp.n_nodes;
    I.n_slices = (int64_t)P.sell_off.size() - 1;
    I.dt = sp.dt;
    I.trace_every = sp.trace_every;
    I.target = sp.target;
    int present = 0;
    for (uint8_t m : P.model) present |= m <= 2 ? 1 : (m == 3 ? 2 : (m == 4 ? 4 : 8));
    I.mset = present;
    // class ranges (the host groups cells by class: TP06, CRN, Stewart, passive)
    {   // per medium: [0, c2) and the 2D medium with substeps [c2, nc)
        auto cls = [](uint8_t m) { return m <= 2 ? 0 : (m == 3 ? 1 : (m == 4 ? 2 : 3)); };
        int64_t i = 0;
        for (int k = 0; k < 4; ++k) {
            I.cls_begin[k] = i;
            while (i < I.c2 && cls(P.model[i]) == k) ++i;
            I.cls_end[k] = i;
        }
        const int64_t i1 = i;
        for (int k = 0; k < 4; ++k) {
            I.cls2_begin[k] = i;
            while (i < nc && cls(P.model[i]) == k) ++i;
            I.cls2_end[k] = i;
        }
        if (i1 != I.c2 || i != nc) {
            st = EP_EINVAL;
            return "cells are not grouped by medium and model class";
        }
    }

    InstDesc &D = I.desc;
    std::memset(&D, 0, sizeof(D));
    D.nc = nc;
    D.nn = nn;
    auto fail_mem = [&]() { st = EP_ENOMEM; free_instance(I); return std::string("device allocation failed"); };
    if (!up(I, (void **)&D.sell_off, P.sell_off) || !up(I, (void **)&D.sell_cell, P.sell_cell) ||
        !up(I, (void **)&D.model, P.model) || !up(I, (void **)&D.vol, P.vol) ||
        !up(I, (void **)&I.d_perm, P.perm))
        return fail_mem();
    bool ok;
    if (I.idx16) {
        std::vector<int32_t> nbs, cbs;
        block_bases(P.cnode, 8, nc, &nbs);
        block_bases(P.cnbr, 4, nc, &cbs);
        ok = up(I, (void **)&D.cnode16, offsets16(P.cnode, 8, nc, nbs)) &&
             up(I, (void **)&D.cnbr16, offsets16(P.cnbr, 4, nc, cbs)) && up(I, (void **)&D.nbase, nbs) &&
             up(I, (void **)&D.cbase, cbs);
        D.idx16 = 1;
    } else {
        ok = up(I, (void **)&D.cnode, tiled(P.cnode, 8, nc)) && up(I, (void **)&D.cnbr, tiled(P.cnbr, 4, nc));
    }
    if (!ok) return fail_mem();
    ok = rs == 8 ? (up(I, (void **)&D.sell_w, P.sell_w) &&
                         up(I, (void **)&D.cbeta, tiled(P.cbeta, 8, nc)) &&
                         up(I, (void **)&D.cb, tiled(P.cb, 4, nc)))
                      : (up(I, (void **)&D.sell_w, conv<float>(P.sell_w)) &&
                         up(I, (void **)&D.cbeta, tiled(conv<float>(P.cbeta), 8, nc)) &&
                         up(I, (void **)&D.cb, tiled(conv<float>(P.cb), 4, nc)));
    if (!ok) return fail_mem();

    // initial state (tile-major slot arrays, internal order)
    std::vector<double> v0(nc), gate(tiled_len(nc, NG_MAX), 0.0), conc(tiled_len(nc, NC_MAX), 0.0);
    for (int64_t i = 0; i < nc; ++i) {
        double y[EP_MAX_SLOTS];
        const int m = P.model[i];
        model_init(m, y);
        v0[i] = y[0];
        const int ng = model_ng(m), ncc = model_nc(m);
        for (int k = 0; k < ng; ++k) gate[tix(i, k, NG_MAX)] = y[1 + k];
        for (int k = 0; k < ncc; ++k) conc[tix(i, k, NC_MAX)] = y[1 + ng + k];
    }
    std::vector<uint32_t> smask(nc, 0);
    for (size_t k = 0; k < sp.stims.size(); ++k)
        if (sp.stims[k].domain == 0)
            for (int32_t id : sp.stims[k].ids) smask[P.iperm[id]] |= 1u << k;
    if (!up(I, (void **)&D.smask, smask) || !up(I, (void **)&D.conc, conc)) return fail_mem();
    if (rs == 8) {
        ok = up(I, (void **)&D.gate, gate) && up(I, &D.v[0], v0) && up(I, &D.v[1], v0) &&
             up(I, (void **)&D.vrest, v0) && up(I, &D.vmax, v0) &&
             up(I, &D.vn, std::vector<double>(nn, 0.0));
    } else {
        ok = up(I, (void **)&D.gate, conv<float>(gate)) && up(I, &D.v[0], conv<float>(v0)) &&
             up(I, &D.v[1], conv<float>(v0)) && up(I, (void **)&D.vrest, conv<float>(v0)) &&
             up(I, &D.vmax, conv<float>(v0)) && up(I, &D.vn, std::vector<float>(nn, 0.0f));
    }
    if (!ok) return fail_mem();
    const double nan = std::numeric_limits<double>::quiet_NaN();
    if (!up(I, (void **)&D.dstat, std::vector<uint8_t>(nc, 0)) ||
        !up(I, (void **)&D.t_act, std::vector<double>(nc, nan)) ||
        !up(I, (void **)&D.t_rep, std::vector<double>(nc, nan)))
        return fail_mem();

    // vbar trace: sample 0 now, then one every trace_every steps; one partial
    // per cell tile (tiles do not straddle model classes)
    D.n_waves = 0;
    for (int k = 0; k < 4; ++k)
        D.n_waves += (int32_t)((I.cls_end[k] - I.cls_begin[k] + 63) / 64) +
                     (int32_t)((I.cls2_end[k] - I.cls2_begin[k] + 63) / 64);
    if (I.c2 < nc) {   // potentials between substeps, indexed by internal cell
        char *w0 = (char *)dalloc(I, (size_t)(nc - I.c2) * rs);
        char *w1 = (char *)dalloc(I, (size_t)(nc - I.c2) * rs);
        if (!w0 || !w1) return fail_mem();
        D.w[0] = w0 - (size_t)I.c2 * rs;
        D.w[1] = w1 - (size_t)I.c2 * rs;
    }
    I.trace_cap = 4096;
    if (sp.trace_every > 0 && sp.target != INT64_MAX)
        I.trace_cap = std::max<int64_t>(2, sp.target / sp.trace_every + 2);
    else if (sp.trace_every > 0)
        I.trace_cap = 1 << 16;
    double tv = 0.0, vt = 0.0;
    for (int64_t i = 0; i < nc; ++i) { tv += P.vol[i]; vt += P.vol[i] * v0[i]; }
    std::vector<double> trace(I.trace_cap, nan);
    trace[0] = vt / tv;
    if (!up(I, (void **)&D.trace, trace) ||
        !up(I, (void **)&D.part, std::vector<double>((nc + 63) / 64 + 12, 0.0)))
        return fail_mem();
    D.dt = sp.dt;
    D.dt2 = sp.dt / I.sub2;
    D.thr = sp.thr;
    D.repol = sp.repol;
    D.inv_total_vol = 1.0 / tv;
    D.gs = GScale{sp.gscale[0], sp.gscale[1], sp.gscale[2], sp.gscale[3]};
    D.trace_cap = I.trace_cap;
    D.trace_every = sp.trace_every;

    Ctrl ctrl;
    std::memset(&ctrl, 0, sizeof(ctrl));
    ctrl.step = 0;
    ctrl.target = sp.target;
    ctrl.n_stim = (int32_t)sp.stims.size();
    for (size_t k = 0; k < sp.stims.size(); ++k) {
        const StimSpec &q = sp.stims[k];
        ctrl.st_n0[k] = std::llround(q.t0 / sp.dt);
        ctrl.st_ndur[k] = std::llround(q.dur / sp.dt);
        ctrl.st_nper[k] = q.period > 0 ? std::llround(q.period / sp.dt) : 0;
        ctrl.st_count[k] = q.count;
        ctrl.st_amp[k] = q.amp;
    }
    I.d_ctrl = (Ctrl *)dalloc(I, sizeof(Ctrl));
    if (!I.d_ctrl) return fail_mem();
    if (hipMemcpy(I.d_ctrl, &ctrl, sizeof(ctrl), hipMemcpyHostToDevice) != hipSuccess) {
        st = EP_EDEVICE;
        free_instance(I);
        return "hipMemcpy of the control block failed";
    }
    D.ctrl = I.d_ctrl;
    I.host_step = 0;
    I.ab2 = sp.scheme >= 1;
    I.scheme = sp.scheme;
    if (I.ab2) {
        D.hv = zalloc(I, nc * (size_t)rs);
        D.hc = (double *)zalloc(I, tiled_len(nc, NC_MAX) * 8);
        if (!D.hv || !D.hc) return fail_mem();
    }
    I.bido = sp.bido;
    if (sp.bido) {
        Bido &B = I.bd;
        const size_t m1 = (size_t)sp.bido_restart + 1;
        B.restart = sp.bido_restart;
        B.max_iter = sp.bido_max_iter;
        B.tol = sp.bido_tol;
        B.chi_cm = sp.chi * sp.cm;
        B.total_vol = tv;
        B.last_iters = B.total_iters = 0;
        B.last_relres = 0;
        // phi_e^0 = 0: exact for a uniform initial potential
        if (!up(I, (void **)&B.phi, std::vector<double>(nc, 0.0)) ||
            !up(I, (void **)&B.ebeta, tiled(P.ebeta, 8, nc)) || !up(I, (void **)&B.eb, tiled(P.eb, 4, nc)))
            return fail_mem();
        B.b = (double *)dalloc(I, nc * 8);
        B.w = (double *)dalloc(I, nc * 8);
        B.xn = (double *)dalloc(I, nn * 8);
        B.V = (double *)dalloc(I, m1 * nc * 8);
        B.part = (double *)dalloc(I, 2 * m1 * bido_part_cols(nc) * 8);   // two passes' partials
        B.h = (double *)dalloc(I, (2 * m1 + 2) * 8);
        B.y = (double *)dalloc(I, m1 * 8);
        B.gm = (double *)dalloc(I, gmres_state_doubles((int)m1 - 1) * 8);
        if (!B.b || !B.w || !B.xn || !B.V || !B.part || !B.h || !B.y || !B.gm) return fail_mem();
        if (hipHostMalloc((void **)&B.h_host, std::max<size_t>((2 * m1 + 2) * 8, 64)) != hipSuccess)
            return fail_mem();
        D.phi = B.phi;
        const Coarse &Cs = I.coarse;
        B.n_agg = Cs.n_agg;
        B.precond = Cs.n_agg > 0;
        if (B.precond) {
            // A_c^{-1} in FP32: the preconditioner only has to be a fixed
            // linear map (GMRES reaches the same solution to its tolerance),
            // and its dense product is the largest read of an Arnoldi step
            const std::vector<float> cinv32(Cs.cinv.begin(), Cs.cinv.end());
            if (!up(I, (void **)&B.agg_of, Cs.agg_of) || !up(I, (void **)&B.agg_cells, Cs.agg_cells) ||
                !up(I, (void **)&B.agg_off, Cs.agg_off) || !up(I, (void **)&B.dinv, Cs.dinv) ||
                !up(I, (void **)&B.cinv, cinv32))
                return fail_mem();
            B.z = (double *)dalloc(I, nc * 8);
            B.t = (double *)dalloc(I, nc * 8);
            B.rc = (double *)dalloc(I, (size_t)Cs.n_agg * 8);
            B.zc = (double *)dalloc(I, (size_t)Cs.n_agg * 8);
            if (!B.z || !B.t || !B.rc || !B.zc) return fail_mem();
        }
        I.coarse = Coarse();               // the host copy is no longer needed
    }
    if (has_junction_block(I)) {
        std::string e = upload_purkinje(sp, rs, I, st);
        if (!e.empty()) return e;
    }
    return "";
}

std::string build_instance(const InstSpec &sp, int rs, const Allocator &al, Inst &I,
                           ep_status &st) {
    std::string e = prep_instance(sp, I, st);
    if (!e.empty()) return e;
    return upload_instance(sp, rs, al, I, st);
}

void free_instance(Inst &I) {
    for (auto &a : I.allocs) {
        if (I.al.free) I.al.free(a.first, I.al.ctx);
        else (void)hipFree(a.first);
    }
    I.allocs.clear();
    if (I.bd.h_host) (void)hipHostFree(I.bd.h_host);
    for (hipGraphExec_t g : I.bd.chunk_graphs)
        if (g) (void)hipGraphExecDestroy(g);
    I.bd.chunk_graphs.clear();
    I.bd = Bido();
    if (I.arena) {
        if (I.al.free) I.al.free(I.arena, I.al.ctx);
        else (void)hipFree(I.arena);
    }
    I.arena = nullptr;
    I.arena_size = I.arena_used = 0;
    I.footprint = 0;
    I.d_ctrl = nullptr;
}

// ================================================================ stepper
namespace {

void drop_graph(Stepper &s) {
    if (s.graph) { (void)hipGraphExecDestroy(s.graph); s.graph = nullptr; }
}

Tables tables(const Stepper &s) {
    return Tables{s.d_desc, s.d_ctiles, s.d_ntiles, s.d_ptiles, s.d_purk, s.d_counts};
}

int grid_for(int64_t n_tiles) { return (int)std::max<int64_t>(n_tiles, 1); }

// The launch's XCD remap mode as each kernel takes it: modes 0-2 apply to
// both kernels; mode 3 leaves the cell kernels unremapped (their streams do
// best with every XCD in one band of tiles) and gives the node gather the
// chunked ranges of mode 2 (neighbouring node tiles share cells, whose
// potentials then stay in one L2).
int cell_remap(int mode) { return mode == 3 ? 0 : mode; }
int node_remap(int mode) { return mode == 3 ? 2 : mode; }

// Events that a profiled launch sets from the dispatches' own timestamps:
// `start` at the first kernel's start, `stop` at the last one's end (both
// null: an ordinary launch, the only kind that graphs capture).
struct Span {
    hipEvent_t start = nullptr, stop = nullptr;
};

template <typename... A, typename... B>
void launch_k(void (*kern)(A...), int grid, int block, hipStream_t st, hipEvent_t e0,
              hipEvent_t e1, B... args) {
    if (e0 || e1) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, e0, e1, 0, args...);
    else kern<<<grid, block, 0, st>>>(args...);
}

// Cell kernels of step offset `off`, one launch per model class present:
// the step's tiles (sub < 0) or substep `sub` of the 2D media with
// substeps, on stream `st`.
template <typename R, bool BIDO, int SCH>
void launch_cells_v(Stepper &s, const Tables &tb, int32_t off, int32_t sub = -1,
                    hipStream_t st = nullptr, Span sp = {}) {
    if (!st) st = s.stream;
    const int64_t *base = sub < 0 ? s.cls_base : s.cls2_base;
    const int64_t *cnt = sub < 0 ? s.cls_tiles : s.cls2_tiles;
    Tables t[4] = {tb, tb, tb, tb};
    for (int k = 0; k < 4; ++k) t[k].cell_tiles = tb.cell_tiles + base[k];
    int first = -1, last = -1;
    for (int k = 0; k < 4; ++k)
        if (cnt[k]) {
            if (first < 0) first = k;
            last = k;
        }
    const int B = s.cell_threads;
    auto go = [&](void (*kern)(Tables, int32_t, int, int32_t), int k) {
        if (cnt[k])
            launch_k(kern, (int)cnt[k], B, st, k == first ? sp.start : nullptr,
                     k == last ? sp.stop : nullptr, t[k], off, cell_remap(s.remap), sub);
    };
    go(k_cell<R, 1, BIDO, SCH>, 0);
    go(k_cell<R, 2, BIDO, SCH>, 1);
    go(k_cell<R, 4, BIDO, SCH>, 2);
    go(k_cell<R, 8, BIDO, SCH>, 3);
}

// bidomain instances run in FP64 with forward Euler only (checked at
// creation); Adams-Bashforth 2 applies to every instance of a stepper or none
template <typename R>
void launch_cells(Stepper &s, const Tables &tb, int32_t off, Span sp = {}) {
    if constexpr (sizeof(R) == 8) {
        if (s.bido) { launch_cells_v<R, true, 0>(s, tb, off, -1, nullptr, sp); return; }
    }
    if (s.scheme == 2) launch_cells_v<R, false, 2>(s, tb, off, -1, nullptr, sp);
    else if (s.scheme == 1) launch_cells_v<R, false, 1>(s, tb, off, -1, nullptr, sp);
    else launch_cells_v<R, false, 0>(s, tb, off, -1, nullptr, sp);
}

template <typename R>
void launch_gather(Stepper &s, const Tables &tb, int32_t off, Span sp = {}) {
    if (s.n_nt == 0) return;
    if constexpr (sizeof(R) == 8) {
        if (s.bido) {
            launch_k(k_node_gather<R, true>, s.grid_node, TILE, s.stream, sp.start, sp.stop, tb, off,
                     node_remap(s.remap), -1);
            return;
        }
    }
    launch_k(k_node_gather<R, false>, s.grid_node, TILE, s.stream, sp.start, sp.stop, tb, off,
             node_remap(s.remap), -1);
}

// The substeps of step offset `off` of the 2D media that have them, on
// stream `st`: per substep their node values, then their cells.  They read
// and write only those media (and v^n of their cells), so they may run
// beside the other kernels of the step.
template <typename R>
void launch_medium2(Stepper &s, int32_t off, hipStream_t st) {
    if (s.sub2_max <= 0 || s.n_nt2 == 0) return;
    Tables tb = tables(s);
    Tables tn = tb;
    tn.node_tiles = tb.node_tiles + s.nt2_base;
    for (int32_t q = 0; q < s.sub2_max; ++q) {
        k_node_gather<R, false><<<(int)s.n_nt2, TILE, 0, st>>>(tn, off, node_remap(s.remap), q);
        if (s.scheme == 2) launch_cells_v<R, false, 2>(s, tb, off, q, st);
        else if (s.scheme == 1) launch_cells_v<R, false, 1>(s, tb, off, q, st);
        else launch_cells_v<R, false, 0>(s, tb, off, q, st);
    }
}

// Graph substeps of step offset `off` on stream `st`.  They read the graph,
// the junction table (pulses scheduled by earlier steps) and the control
// block, and write only the graph, so they may run beside the tissue kernels
// of the same step.
template <typename R>
void launch_substeps(Stepper &s, int32_t off, hipStream_t st) {
    const Tables tb = tables(s);
    for (int32_t sub = 0; sub < s.n_sub_max; ++sub) {
        if (s.scheme == 2) k_purkinje<R, 2><<<(int)s.n_pt, TILE, 0, st>>>(tb, off, sub);
        else if (s.scheme == 1) k_purkinje<R, 1><<<(int)s.n_pt, TILE, 0, st>>>(tb, off, sub);
        else k_purkinje<R, 0><<<(int)s.n_pt, TILE, 0, st>>>(tb, off, sub);
    }
}

// Junction events of step offset `off`: after the tissue and the substeps.
template <typename R>
void launch_junctions(Stepper &s, int32_t off) {
    k_junctions<R><<<(int)s.n_pk, TILE, 0, s.stream>>>(tables(s), off);
}

std::string enqueue(Stepper &s, int64_t k) {
    hipError_t e = hipSuccess;
    const Tables tb = tables(s);
    for (int64_t i = 0; i < k && e == hipSuccess; ++i) {
        // graph substeps (none when every junction has a source cell) and 2D
        // media with substeps go to the side stream after the node gather (its
        // tile 0 may reduce the vbar partials the substeps write)
        const bool graph = s.n_pk > 0 && s.n_pt > 0 && s.n_sub_max > 0;
        const bool med2 = s.sub2_max > 0 && s.n_nt2 > 0;
        const bool fork = graph || med2;
        if (s.rs == 8) launch_gather<double>(s, tb, (int32_t)i);
        else launch_gather<float>(s, tb, (int32_t)i);
        if (fork) {
            if ((e = hipEventRecord(s.ev_fork, s.stream)) != hipSuccess ||
                (e = hipStreamWaitEvent(s.side, s.ev_fork, 0)) != hipSuccess)
                break;
            if (med2) {
                if (s.rs == 8) launch_medium2<double>(s, (int32_t)i, s.side);
                else launch_medium2<float>(s, (int32_t)i, s.side);
            }
            if (graph) {
                if (s.rs == 8) launch_substeps<double>(s, (int32_t)i, s.side);
                else launch_substeps<float>(s, (int32_t)i, s.side);
            }
        }
        if (s.rs == 8) launch_cells<double>(s, tb, (int32_t)i);
        else launch_cells<float>(s, tb, (int32_t)i);
        if (fork && ((e = hipEventRecord(s.ev_join, s.side)) != hipSuccess ||
                     (e = hipStreamWaitEvent(s.stream, s.ev_join, 0)) != hipSuccess))
            break;
        if (s.n_pk > 0) {
            if (s.rs == 8) launch_junctions<double>(s, (int32_t)i);
            else launch_junctions<float>(s, (int32_t)i);
        }
    }
    if (e != hipSuccess) return std::string("graph substep stream: ") + hipGetErrorString(e);
    k_advance<<<1, 256, 0, s.stream>>>(tables(s), k);
    return "";
}

std::string hip_err(const char *what, hipError_t e) {
    return std::string(what) + ": " + hipGetErrorString(e);
}

}  // namespace

std::string stepper_init(Stepper &s, int device, hipStream_t stream, int rs) {
    s.device = device;
    s.stream = stream;
    s.rs = rs;
    hipError_t e = hipEventCreateWithFlags(&s.stage_done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_err("hipEventCreate", e);
    if ((e = hipEventCreateWithFlags(&s.ev_fork, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&s.ev_join, hipEventDisableTiming)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s.side, hipStreamNonBlocking)) != hipSuccess)
        return hip_err("stepper streams and events", e);
    e = hipMalloc((void **)&s.d_counts, 8 * sizeof(int32_t));
    if (e != hipSuccess) return hip_err("hipMalloc", e);
    return "";
}

void stepper_free(Stepper &s) {
    drop_graph(s);
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    if (s.d_desc) (void)hipFree(s.d_desc);
    if (s.d_ctiles) (void)hipFree(s.d_ctiles);
    if (s.d_ntiles) (void)hipFree(s.d_ntiles);
    if (s.d_counts) (void)hipFree(s.d_counts);
    if (s.d_ptiles) (void)hipFree(s.d_ptiles);
    if (s.d_purk) (void)hipFree(s.d_purk);
    s.d_ptiles = nullptr;
    s.d_purk = nullptr;
    if (s.h_stage) (void)hipHostFree(s.h_stage);
    if (s.stage_done) (void)hipEventDestroy(s.stage_done);
    if (s.side) (void)hipStreamSynchronize(s.side);
    if (s.side) (void)hipStreamDestroy(s.side);
    if (s.ev_fork) (void)hipEventDestroy(s.ev_fork);
    if (s.ev_join) (void)hipEventDestroy(s.ev_join);
    s.side = nullptr; s.ev_fork = s.ev_join = nullptr;
    s.d_desc = nullptr; s.d_ctiles = s.d_ntiles = nullptr; s.d_counts = nullptr;
    s.h_stage = nullptr; s.stage_done = nullptr;
}

std::string stepper_sync_tables(Stepper &s) {
    std::vector<InstDesc> desc;
    std::vector<Tile> ct, nt;
    std::vector<PTile> pt;
    std::vector<PurkDesc> pk;
    int32_t nsub = 0;
    s.bido = false;
    s.scheme = 0;
    for (const Inst *I : s.insts) {
        s.bido = s.bido || I->bido;
        s.scheme = std::max(s.scheme, I->scheme);
    }
    // cell tiles class by class, those of 2D media with substeps after the
    // others; wave partials numbered per instance over its class ranges in
    // the order medium 0 classes 0-3, medium 1 classes 0-3 (as n_waves)
    const int64_t TS = s.cell_threads;
    auto wave_base = [](const Inst &I, int medium, int k) {
        int64_t w = 0;
        for (int m = 0; m <= medium; ++m)
            for (int q = 0; q < 4 && (m < medium || q < k); ++q)
                w += m == 0 ? (I.cls_end[q] - I.cls_begin[q] + 63) / 64
                            : (I.cls2_end[q] - I.cls2_begin[q] + 63) / 64;
        return w;
    };
    for (int k = 0; k < 4; ++k) {
        s.cls_base[k] = (int64_t)ct.size();
        for (size_t i = 0; i < s.insts.size(); ++i) {
            const Inst &I = *s.insts[i];
            const int64_t w0 = wave_base(I, 0, k);
            for (int64_t b = I.cls_begin[k]; b < I.cls_end[k]; b += TS)
                ct.push_back(Tile{I.desc, b, (int32_t)std::min<int64_t>(TS, I.cls_end[k] - b), 0, 1,
                                  (int32_t)(w0 + (b - I.cls_begin[k]) / 64)});
        }
        s.cls_tiles[k] = (int64_t)ct.size() - s.cls_base[k];
    }
    s.sub2_max = 0;
    for (int k = 0; k < 4; ++k) {
        s.cls2_base[k] = (int64_t)ct.size();
        for (size_t i = 0; i < s.insts.size(); ++i) {
            const Inst &I = *s.insts[i];
            const int64_t w0 = wave_base(I, 1, k);
            for (int64_t b = I.cls2_begin[k]; b < I.cls2_end[k]; b += TS)
                ct.push_back(Tile{I.desc, b, (int32_t)std::min<int64_t>(TS, I.cls2_end[k] - b), 0,
                                  I.sub2, (int32_t)(w0 + (b - I.cls2_begin[k]) / 64)});
        }
        s.cls2_tiles[k] = (int64_t)ct.size() - s.cls2_base[k];
    }
    for (size_t i = 0; i < s.insts.size(); ++i) {
        const Inst &I = *s.insts[i];
        desc.push_back(I.desc);
        if (has_junction_block(I)) {
            pk.push_back(I.pdesc);
            nsub = std::max(nsub, I.pdesc.n_sub);
            for (int64_t b = 0, t = 0; b < I.pdesc.np; b += TILE, ++t)
                pt.push_back(PTile{I.pdesc, b, (int32_t)std::min<int64_t>(TILE, I.pdesc.np - b), (int32_t)t});
        }
    }
    // node tiles: the step's, then those of 2D media with substeps; local
    // numbers run over the instance (tile 0 reduces the vbar trace)
    std::vector<int32_t> next_node(s.insts.size(), 0);
    for (size_t i = 0; i < s.insts.size(); ++i) {
        const Inst &I = *s.insts[i];
        for (int64_t b = 0; b < I.n2; b += TILE)
            nt.push_back(Tile{I.desc, b, (int32_t)std::min<int64_t>(TILE, I.n2 - b), next_node[i]++, 1, 0});
    }
    s.nt2_base = (int64_t)nt.size();
    for (size_t i = 0; i < s.insts.size(); ++i) {
        const Inst &I = *s.insts[i];
        if (I.c2 < I.desc.nc) s.sub2_max = std::max(s.sub2_max, I.sub2);
        for (int64_t b = I.n2; b < I.desc.nn; b += TILE)
            nt.push_back(Tile{I.desc, b, (int32_t)std::min<int64_t>(TILE, I.desc.nn - b), next_node[i]++,
                              I.sub2, 0});
    }
    // grow device tables geometrically; growth invalidates the graph
    auto grow = [&](void **p, size_t &cap, size_t need, size_t elem) -> hipError_t {
        if (need <= cap && *p) return hipSuccess;
        size_t nc = std::max<size_t>(need, cap * 2);
        nc = std::max<size_t>(nc, 16);
        if (*p) { (void)hipStreamSynchronize(s.stream); (void)hipFree(*p); *p = nullptr; }
        drop_graph(s);
        cap = nc;
        return hipMalloc(p, nc * elem);
    };
    hipError_t e;
    if ((e = grow((void **)&s.d_desc, s.cap_inst, desc.size(), sizeof(InstDesc))) != hipSuccess ||
        (e = grow((void **)&s.d_ctiles, s.cap_ct, ct.size(), sizeof(Tile))) != hipSuccess ||
        (e = grow((void **)&s.d_ntiles, s.cap_nt, nt.size(), sizeof(Tile))) != hipSuccess ||
        (e = grow((void **)&s.d_ptiles, s.cap_pt, pt.size(), sizeof(PTile))) != hipSuccess ||
        (e = grow((void **)&s.d_purk, s.cap_pk, pk.size(), sizeof(PurkDesc))) != hipSuccess)
        return hip_err("hipMalloc(tables)", e);
    // pinned staging: wait until the previous upload has left it
    const size_t need = desc.size() * sizeof(InstDesc) + (ct.size() + nt.size()) * sizeof(Tile) +
                        pt.size() * sizeof(PTile) + pk.size() * sizeof(PurkDesc) + 64;
    if (s.h_stage) (void)hipEventSynchronize(s.stage_done);
    if (need > s.stage_bytes) {
        if (s.h_stage) (void)hipHostFree(s.h_stage);
        s.stage_bytes = need * 2;
        if ((e = hipHostMalloc(&s.h_stage, s.stage_bytes)) != hipSuccess) {
            s.h_stage = nullptr;
            s.stage_bytes = 0;
            return hip_err("hipHostMalloc", e);
        }
    }
    char *p = (char *)s.h_stage;
    int32_t counts[8] = {(int32_t)ct.size(), (int32_t)nt.size(), (int32_t)desc.size(),
                         (int32_t)pt.size(), (int32_t)pk.size(), 0, 0, 0};
    std::memcpy(p, counts, sizeof(counts));
    char *pd = p + 64;
    std::memcpy(pd, desc.data(), desc.size() * sizeof(InstDesc));
    char *pc = pd + desc.size() * sizeof(InstDesc);
    std::memcpy(pc, ct.data(), ct.size() * sizeof(Tile));
    char *pn = pc + ct.size() * sizeof(Tile);
    std::memcpy(pn, nt.data(), nt.size() * sizeof(Tile));
    char *pp = pn + nt.size() * sizeof(Tile);
    std::memcpy(pp, pt.data(), pt.size() * sizeof(PTile));
    char *pq = pp + pt.size() * sizeof(PTile);
    std::memcpy(pq, pk.data(), pk.size() * sizeof(PurkDesc));
    if ((e = hipMemcpyAsync(s.d_counts, p, sizeof(counts), hipMemcpyHostToDevice, s.stream)) != hipSuccess ||
        (!desc.empty() && (e = hipMemcpyAsync(s.d_desc, pd, desc.size() * sizeof(InstDesc),
                                              hipMemcpyHostToDevice, s.stream)) != hipSuccess) ||
        (!ct.empty() && (e = hipMemcpyAsync(s.d_ctiles, pc, ct.size() * sizeof(Tile),
                                            hipMemcpyHostToDevice, s.stream)) != hipSuccess) ||
        (!nt.empty() && (e = hipMemcpyAsync(s.d_ntiles, pn, nt.size() * sizeof(Tile),
                                            hipMemcpyHostToDevice, s.stream)) != hipSuccess) ||
        (!pt.empty() && (e = hipMemcpyAsync(s.d_ptiles, pp, pt.size() * sizeof(PTile),
                                            hipMemcpyHostToDevice, s.stream)) != hipSuccess) ||
        (!pk.empty() && (e = hipMemcpyAsync(s.d_purk, pq, pk.size() * sizeof(PurkDesc),
                                            hipMemcpyHostToDevice, s.stream)) != hipSuccess))
        return hip_err("hipMemcpyAsync(tables)", e);
    (void)hipEventRecord(s.stage_done, s.stream);
    s.n_ct = (int64_t)ct.size();
    s.n_nt = s.nt2_base;
    s.n_nt2 = (int64_t)nt.size() - s.nt2_base;
    s.n_pt = (int64_t)pt.size();
    s.n_pk = (int64_t)pk.size();
    s.n_sub_max = nsub;
    s.dirty = false;
    return "";
}

std::string stepper_run(Stepper &s, int64_t k) {
    if (k <= 0) return "";
    if (s.dirty) {
        std::string e = stepper_sync_tables(s);
        if (!e.empty()) return e;
    }
    if (s.insts.empty()) return "";
    // one block per tile; a graph is reused until the tile counts change
    s.grid_node = grid_for(s.n_nt);
    const int64_t glen = s.steps_per_graph > 0 ? s.steps_per_graph : 0;
    int64_t left = k;
    if (glen > 0 && left >= glen) {
        if (s.graph && (s.graph_k != glen || !std::equal(s.cls_tiles, s.cls_tiles + 4, s.graph_cls) ||
                        !std::equal(s.cls2_tiles, s.cls2_tiles + 4, s.graph_cls2) ||
                        s.graph_gn != s.grid_node || s.graph_remap != s.remap ||
                        s.graph_pt != s.n_pt || s.graph_pk != s.n_pk || s.graph_nsub != s.n_sub_max ||
                        s.graph_nt2 != s.n_nt2 || s.graph_sub2 != s.sub2_max ||
                        s.graph_threads != s.cell_threads))
            drop_graph(s);
        if (!s.graph) {
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_err("hipStreamBeginCapture", e);
            const std::string eq = enqueue(s, glen);
            e = hipStreamEndCapture(s.stream, &g);
            if (!eq.empty()) {
                if (g) (void)hipGraphDestroy(g);
                return eq;
            }
            if (e != hipSuccess) return hip_err("hipStreamEndCapture", e);
            e = hipGraphInstantiate(&s.graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) { s.graph = nullptr; return hip_err("hipGraphInstantiate", e); }
            s.graph_k = (int)glen;
            std::copy(s.cls_tiles, s.cls_tiles + 4, s.graph_cls);
            std::copy(s.cls2_tiles, s.cls2_tiles + 4, s.graph_cls2);
            s.graph_nt2 = s.n_nt2;
            s.graph_sub2 = s.sub2_max;
            s.graph_threads = s.cell_threads;
            s.graph_gn = s.grid_node;
            s.graph_remap = s.remap;
            s.graph_pt = s.n_pt;
            s.graph_pk = s.n_pk;
            s.graph_nsub = s.n_sub_max;
        }
        while (left >= glen) {
            hipError_t e = hipGraphLaunch(s.graph, s.stream);
            if (e != hipSuccess) return hip_err("hipGraphLaunch", e);
            left -= glen;
        }
    }
    if (left > 0) {
        const std::string eq = enqueue(s, left);
        if (!eq.empty()) return eq;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err("kernel launch", e);
    for (Inst *I : s.insts) I->host_step = std::min(I->host_step + k, std::max(I->host_step, I->target));
    return "";
}

std::string stepper_autotune(Stepper &s, int64_t trial_steps, TuneResult &out,
                             bool allow_direct) {
    if (trial_steps <= 0) return "trial_steps must be positive";
    static const int32_t kGraph[] = {0, 10, 25, 50, 100};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return "hipEventCreate failed";
    }
    out = TuneResult();
    double best = HUGE_VAL;
    std::string err;
    for (int32_t remap = 0; remap <= 3 && err.empty(); ++remap)
        for (int32_t k : kGraph) {
            if (k == 0 && !allow_direct) continue;
            s.steps_per_graph = k;
            s.remap = remap;
            const int64_t warm = k > 0 ? k : 1;
            // whole graphs, so that the trial times the schedule it names
            const int64_t n = k > 0 ? (trial_steps + k - 1) / k * k : trial_steps;
            err = stepper_run(s, warm);
            if (!err.empty()) break;
            (void)hipEventRecord(e0, s.stream);
            err = stepper_run(s, n);
            if (!err.empty()) break;
            (void)hipEventRecord(e1, s.stream);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            out.n_trials++;
            out.steps_used += warm + n;
            const double per = ms / n;
            if (per < best) {
                best = per;
                out.steps_per_graph = k;
                out.xcd_remap = remap;
            }
        }
    s.steps_per_graph = out.steps_per_graph;
    s.remap = out.xcd_remap;
    // cell tile sizes at that schedule; a new size rebuilds the tile tables
    static const int32_t kTile[] = {256, 128, 64};
    const int32_t t0 = s.cell_threads;
    out.cell_threads = t0;
    double best_shape = HUGE_VAL;
    for (const int32_t tile : kTile) {
        if (!err.empty()) break;
        if (s.cell_threads != tile) {
            s.cell_threads = tile;
            s.dirty = true;
        }
        const int32_t k = out.steps_per_graph;
        const int64_t warm = k > 0 ? k : 1;
        const int64_t n = k > 0 ? (trial_steps + k - 1) / k * k : trial_steps;
        err = stepper_run(s, warm);
        if (!err.empty()) break;
        (void)hipEventRecord(e0, s.stream);
        err = stepper_run(s, n);
        if (!err.empty()) break;
        (void)hipEventRecord(e1, s.stream);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        out.n_trials++;
        out.steps_used += warm + n;
        const double per = ms / n;
        if (per < best_shape) {
            best_shape = per;
            out.cell_threads = tile;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s.cell_threads != out.cell_threads) {
        s.cell_threads = out.cell_threads;
        s.dirty = true;
    }
    out.ms_per_step = std::min(best, best_shape);
    return err;
}

std::string stepper_profile(Stepper &s, int64_t n, int64_t every, double &cell_ms,
                            double &node_ms, double *step_ms) {
    if (s.dirty) {
        std::string e = stepper_sync_tables(s);
        if (!e.empty()) return e;
    }
    const int gn = grid_for(s.n_nt);
    s.grid_node = gn;
    // The timed steps are steps 0, every, 2 every, ... of the n (the others
    // are launched plainly).  A ring of six events per timed step, all but
    // one set from the dispatches' own timestamps (so a kernel's time is
    // its execution alone, as a kernel trace reports it, and no marker
    // packet sits between kernels): start and end of the node gather and of
    // the cell kernels, and the end of the step's last kernel; the step
    // starts at the node gather's start (a recorded event only when the
    // step has no node gather).  The host waits only for the timed step
    // RING places back before reusing its events, so the queue stays at
    // least RING - 1 steps deep and the kernels run back to back as in an
    // unprofiled run.
    constexpr int RING = 64, NE = 6;
    std::vector<hipEvent_t> ev(NE * RING, nullptr);
    for (auto &x : ev)
        if (hipEventCreate(&x) != hipSuccess) {
            for (auto &y : ev)
                if (y) (void)hipEventDestroy(y);
            return "hipEventCreate failed";
        }
    double tc = 0, tn = 0;
    const bool gathers = s.n_nt > 0;
    const bool cells = s.cls_tiles[0] + s.cls_tiles[1] + s.cls_tiles[2] + s.cls_tiles[3] > 0;
    auto collect = [&](int64_t i) {
        hipEvent_t *q = &ev[NE * (i % RING)];
        (void)hipEventSynchronize(q[5]);
        float a = 0, b = 0, c = 0;
        if (gathers) (void)hipEventElapsedTime(&a, q[1], q[2]);
        if (cells) (void)hipEventElapsedTime(&b, q[3], q[4]);
        (void)hipEventElapsedTime(&c, gathers ? q[1] : q[0], q[5]);
        tn += a;
        tc += b;
        if (step_ms) step_ms[i] = c;
    };
    // Steps go out as in enqueue(): at step offsets from the device's step
    // counter, which one k_advance moves on over the steps launched since the
    // previous one; here each timed step ends with that advance (its end is
    // the step's end), and the last step too.
    const Tables tb = tables(s);
    const int64_t nt = (n + every - 1) / every;     // timed steps
    int64_t pend = 0;                               // steps since the last advance
    for (int64_t i = 0; i < n; ++i) {
        const bool timed = i % every == 0;
        const int64_t j = i / every;
        if (timed && j >= RING) collect(j - RING);
        hipEvent_t *q = timed ? &ev[NE * (j % RING)] : nullptr;
        const Span g = timed ? Span{q[1], q[2]} : Span{}, c = timed ? Span{q[3], q[4]} : Span{};
        const int32_t off = (int32_t)pend;
        if (timed && !gathers) (void)hipEventRecord(q[0], s.stream);
        if (s.rs == 8) launch_gather<double>(s, tb, off, g);
        else launch_gather<float>(s, tb, off, g);
        if (s.rs == 8) launch_cells<double>(s, tb, off, c);
        else launch_cells<float>(s, tb, off, c);
        if (s.rs == 8) launch_medium2<double>(s, off, s.stream);
        else launch_medium2<float>(s, off, s.stream);
        if (s.n_pk > 0) {               // one stream here: the timings stay apart
            if (s.n_pt > 0 && s.rs == 8) launch_substeps<double>(s, off, s.stream);
            else if (s.n_pt > 0) launch_substeps<float>(s, off, s.stream);
            if (s.rs == 8) launch_junctions<double>(s, off);
            else launch_junctions<float>(s, off);
        }
        ++pend;
        if (timed || i == n - 1) {
            launch_k(k_advance, 1, 256, s.stream, nullptr, timed ? q[5] : nullptr, tb, pend);
            pend = 0;
        }
    }
    for (int64_t j = std::max<int64_t>(0, nt - RING); j < nt; ++j) collect(j);
    for (Inst *I : s.insts) I->host_step = std::min(I->host_step + n, std::max(I->host_step, I->target));
    for (auto &x : ev) (void)hipEventDestroy(x);
    cell_ms = tc / nt;
    node_ms = tn / nt;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? "" : hip_err("kernel launch", e);
}

}  // namespace ep
