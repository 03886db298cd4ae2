// C-ABI of the monodomain library: object lifecycle, upload, stepping
// (direct launches or replayed HIP graphs), readouts and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/ep.h"
#include "instance.hpp"

using namespace epdev;
using ep::model_nc;
using ep::model_ng;

namespace {

// "EPSMCHK9": states in the tile-major layout, header with the cell order,
// trace partials per wave of 64 cells
constexpr uint64_t CKPT_MAGIC = 0x4550534d43484b39ULL;

const char *const TP06_NAMES[] = {"V", "m", "h", "j", "xr1", "xr2", "xs", "r", "s", "d",
                                  "f", "f2", "fCass", "Rbar", "Ca_i", "Ca_SR", "Ca_SS",
                                  "Na_i", "K_i"};
const char *const CRN_NAMES[] = {"V", "m", "h", "j", "oa", "oi", "ua", "ui", "xr", "xs", "d",
                                 "f", "fCa", "u", "v", "w", "Ca_i", "Ca_up", "Ca_rel",
                                 "Na_i", "K_i"};
const char *const STEWART_NAMES[] = {"V", "m", "h", "j", "xr1", "xr2", "xs", "r", "s", "d",
                                     "f", "f2", "fCass", "y", "Rbar", "Ca_i", "Ca_SR",
                                     "Ca_SS", "Na_i", "K_i"};

}  // namespace

struct ep_sim {
    ep_options opt;
    std::string err;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    ep::InstSpec spec;
    bool has_cond = false;
    bool inited = false;
    ep::Inst inst;
    ep::Stepper stepper;
};

namespace {

ep_status fail(ep_sim *s, ep_status st, const std::string &msg) {
    if (s) s->err = msg;
    return st;
}

#define HIP_TRY(s, call)                                                              \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(s, EP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

ep_status run_err(ep_sim *s, const std::string &e) {
    return e.empty() ? EP_OK : fail(s, EP_EDEVICE, e);
}

}  // namespace

// ======================================================================= API
extern "C" {

void ep_default_options(ep_options *o) {
    std::memset(o, 0, sizeof(*o));
    o->prec = EP_FP64;
    o->device = 0;
    o->stream = nullptr;
    o->dt = 0.02;
    o->chi = 140.0;
    o->cm = 0.01;
    o->at_threshold = 0.0;
    o->repol_frac = 0.9;
    o->trace_every = 50;
}

ep_status ep_create(const ep_options *o, ep_sim **out) {
    if (!o || !out) return EP_EINVAL;
    *out = nullptr;
    if (!(o->dt > 0) || !(o->chi > 0) || !(o->cm > 0) || o->trace_every < 0 ||
        (o->prec != EP_FP64 && o->prec != EP_FP32_MIXED) ||
        ((o->dev_alloc == nullptr) != (o->dev_free == nullptr)))
        return EP_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0 || o->device < 0 || o->device >= ndev)
        return EP_EDEVICE;
    if (hipSetDevice(o->device) != hipSuccess) return EP_EDEVICE;
    ep_sim *s = new ep_sim();
    s->opt = *o;
    if (o->stream) {
        s->stream = (hipStream_t)o->stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return EP_EDEVICE;
        }
        s->own_stream = true;
    }
    if (!ep::stepper_init(s->stepper, o->device, s->stream, o->prec == EP_FP64 ? 8 : 4).empty()) {
        ep_destroy(s);
        return EP_EDEVICE;
    }
    s->spec.dt = o->dt;
    s->spec.chi = o->chi;
    s->spec.cm = o->cm;
    s->spec.thr = o->at_threshold;
    s->spec.repol = o->repol_frac;
    s->spec.trace_every = o->trace_every;
    *out = s;
    return EP_OK;
}

void ep_destroy(ep_sim *s) {
    if (!s) return;
    (void)hipSetDevice(s->opt.device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    ep::stepper_free(s->stepper);
    ep::free_instance(s->inst);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

const char *ep_last_error(const ep_sim *s) { return s ? s->err.c_str() : "null simulation"; }

ep_status ep_set_mesh(ep_sim *s, int64_t n_nodes, const double *xyz, int64_t n_tets,
                      const int32_t *tet_nodes) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "mesh is frozen after ep_init");
    if (n_nodes <= 0 || n_tets <= 0 || !xyz || !tet_nodes)
        return fail(s, EP_EINVAL, "empty mesh or null array");
    for (int64_t i = 0; i < 4 * n_tets; ++i)
        if ((tet_nodes[i] < 0 && !(i % 4 == 3 && tet_nodes[i] == -1)) || tet_nodes[i] >= n_nodes)
            return fail(s, EP_EINVAL, "tet node index out of range");
    ep::InstSpec &sp = s->spec;
    sp.xyz.assign(xyz, xyz + 3 * n_nodes);
    sp.tets.assign(tet_nodes, tet_nodes + 4 * n_tets);
    sp.n_nodes = n_nodes;
    sp.n_tets = n_tets;
    sp.model.assign(n_tets, EP_TP06_ENDO);
    sp.fibre.clear();
    sp.stims.clear();
    sp.purk = ep::PurkSpec();
    s->has_cond = false;
    return EP_OK;
}

ep_status ep_set_conductivity(ep_sim *s, const double *fibre, double sigma_l, double sigma_t,
                              const double *scale) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "frozen after ep_init");
    ep::InstSpec &sp = s->spec;
    if (sp.n_tets == 0) return fail(s, EP_ESTATE, "set the mesh first");
    if (!fibre || !(sigma_l >= 0) || !(sigma_t >= 0)) return fail(s, EP_EINVAL, "bad conductivity");
    sp.fibre.assign(fibre, fibre + 3 * sp.n_tets);
    sp.sigma_l = sigma_l;
    sp.sigma_t = sigma_t;
    sp.has_scale = scale != nullptr;
    if (scale) sp.scale.assign(scale, scale + sp.n_tets);
    else sp.scale.clear();
    s->has_cond = true;
    return EP_OK;
}

ep_status ep_set_models(ep_sim *s, const uint8_t *model) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "frozen after ep_init");
    ep::InstSpec &sp = s->spec;
    if (sp.n_tets == 0) return fail(s, EP_ESTATE, "set the mesh first");
    if (!model) return fail(s, EP_EINVAL, "null model array");
    for (int64_t c = 0; c < sp.n_tets; ++c)
        if (model[c] > EP_PASSIVE) return fail(s, EP_EINVAL, "model id out of range");
    sp.model.assign(model, model + sp.n_tets);
    return EP_OK;
}

ep_status ep_set_ionic_scale(ep_sim *s, const char *param, double scale) {
    if (!s || !param) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "ionic scales are frozen after ep_init");
    if (!(scale > 0) || !std::isfinite(scale)) return fail(s, EP_EINVAL, "scale must be > 0");
    const char *names[4] = {"GKr", "GKs", "GCaL", "GNa"};
    for (int i = 0; i < 4; ++i)
        if (std::strcmp(param, names[i]) == 0) {
            s->spec.gscale[i] = scale;
            return EP_OK;
        }
    return fail(s, EP_EINVAL, std::string("unknown conductance ") + param);
}

ep_status ep_add_stimulus(ep_sim *s, int domain, int64_t n_ids, const int32_t *ids, double t0,
                          double dur, double amp, double period, int32_t count) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "stimuli are frozen after ep_init");
    ep::InstSpec &sp = s->spec;
    if (sp.n_tets == 0) return fail(s, EP_ESTATE, "set the mesh first");
    if (domain == 1 && sp.purk.n == 0) return fail(s, EP_ESTATE, "set the Purkinje graph first");
    const std::string e = ep::spec_add_stimulus(sp, domain, n_ids, ids, t0, dur, amp, period, count);
    return e.empty() ? EP_OK : fail(s, EP_EINVAL, e);
}

ep_status ep_set_purkinje(ep_sim *s, int64_t n, const double *xyz, int64_t n_edges,
                          const int32_t *edges, double sigma, int32_t model, int32_t n_sub) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "the graph is frozen after ep_init");
    ep::InstSpec &sp = s->spec;
    if (sp.n_tets == 0) return fail(s, EP_ESTATE, "set the mesh first");
    for (const ep::StimSpec &st : sp.stims)
        if (st.domain == 1) return fail(s, EP_ESTATE, "graph stimuli refer to the previous graph");
    const std::string e = ep::spec_set_purkinje(sp, n, xyz, n_edges, edges, sigma, model, n_sub);
    return e.empty() ? EP_OK : fail(s, EP_EINVAL, e);
}

ep_status ep_set_purkinje_scale(ep_sim *s, int64_t n_edges, const double *scale) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "the graph is frozen after ep_init");
    if (s->spec.purk.n == 0) return fail(s, EP_ESTATE, "set the Purkinje graph first");
    const std::string e = ep::spec_set_purkinje_scale(s->spec, n_edges, scale);
    return e.empty() ? EP_OK : fail(s, EP_EINVAL, e);
}

ep_status ep_add_pmj(ep_sim *s, int32_t node, double radius, double delay_ortho,
                     double delay_anti, int32_t two_way, double amp, double dur) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "junctions are frozen after ep_init");
    if (s->spec.purk.n == 0) return fail(s, EP_ESTATE, "set the Purkinje graph first");
    const std::string e = ep::spec_add_pmj(s->spec, node, radius, delay_ortho, delay_anti,
                                           two_way, amp, dur);
    return e.empty() ? EP_OK : fail(s, EP_EINVAL, e);
}

ep_status ep_add_cell_junction(ep_sim *s, int32_t cell, double radius, double delay_ortho,
                               double delay_anti, int32_t two_way, double amp, double dur) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "junctions are frozen after ep_init");
    if (s->spec.n_tets == 0) return fail(s, EP_ESTATE, "set the mesh first");
    const std::string e = ep::spec_add_cell_junction(s->spec, cell, radius, delay_ortho, delay_anti,
                                                     two_way, amp, dur);
    return e.empty() ? EP_OK : fail(s, EP_EINVAL, e);
}

ep_status ep_set_bidomain(ep_sim *s, double sigma_el, double sigma_et, int32_t restart,
                          double tol, int32_t max_iter) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "the model is frozen after ep_init");
    if (s->opt.prec != EP_FP64) return fail(s, EP_EINVAL, "the bidomain model runs in EP_FP64 only");
    if (!(sigma_el >= 0) || !(sigma_et >= 0) || !std::isfinite(sigma_el) || !std::isfinite(sigma_et) ||
        restart < 1 || restart > ep::kBidoMaxRestart || !(tol > 0) || max_iter < 1)
        return fail(s, EP_EINVAL, "bad bidomain parameters");
    ep::InstSpec &sp = s->spec;
    if (sp.scheme != 0) return fail(s, EP_EINVAL, "the bidomain model steps by forward Euler only");
    sp.bido = true;
    sp.sigma_el = sigma_el;
    sp.sigma_et = sigma_et;
    sp.bido_restart = restart;
    sp.bido_tol = tol;
    sp.bido_max_iter = max_iter;
    return EP_OK;
}

ep_status ep_set_time_scheme(ep_sim *s, int32_t scheme) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "the scheme is frozen after ep_init");
    if (scheme != EP_SCHEME_FE && scheme != EP_SCHEME_AB2 && scheme != EP_SCHEME_RL2_AB2)
        return fail(s, EP_EINVAL, "unknown time scheme");
    if (scheme != EP_SCHEME_FE && s->spec.bido)
        return fail(s, EP_EINVAL, "the bidomain model steps by forward Euler only");
    s->spec.scheme = scheme;
    return EP_OK;
}

ep_status ep_set_medium_substeps(ep_sim *s, int32_t n_sub) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "the substeps are frozen after ep_init");
    if (n_sub > (1 << 20)) return fail(s, EP_EINVAL, "more than 2^20 substeps");
    s->spec.medium_substeps = n_sub;
    return EP_OK;
}

ep_status ep_get_medium_substeps(ep_sim *s, int32_t *n_sub) {
    if (!s || !n_sub) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    *n_sub = s->inst.c2 < s->inst.desc.nc ? s->inst.sub2 : 1;
    return EP_OK;
}

ep_status ep_set_cell_order(ep_sim *s, int32_t order) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "the cell order is frozen after ep_init");
    if (order != EP_ORDER_RCM && order != EP_ORDER_MORTON && order != EP_ORDER_INPUT)
        return fail(s, EP_EINVAL, "unknown cell order");
    s->spec.ordering = order;
    return EP_OK;
}

ep_status ep_init(ep_sim *s) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "already initialised");
    if (s->spec.n_tets == 0) return fail(s, EP_ESTATE, "no mesh");
    if (!s->has_cond) return fail(s, EP_ESTATE, "no conductivity");
    HIP_TRY(s, hipSetDevice(s->opt.device));
    ep::Allocator al{s->opt.dev_alloc, s->opt.dev_free, s->opt.alloc_ctx};
    ep_status st = EP_OK;
    std::string e = ep::build_instance(s->spec, s->stepper.rs, al, s->inst, st);
    if (!e.empty()) return fail(s, st, e);
    if (!(e = ep::diffusion_scratch_setup(s->opt.device)).empty()) {
        ep::free_instance(s->inst);
        return fail(s, EP_EDEVICE, e);
    }
    s->stepper.insts = {&s->inst};
    s->stepper.dirty = true;
    e = ep::stepper_sync_tables(s->stepper);
    if (!e.empty()) { ep::free_instance(s->inst); return fail(s, EP_EDEVICE, e); }
    s->inited = true;
    // inputs are no longer needed on the host
    s->spec.xyz.clear(); s->spec.xyz.shrink_to_fit();
    s->spec.tets.clear(); s->spec.tets.shrink_to_fit();
    s->spec.fibre.clear(); s->spec.fibre.shrink_to_fit();
    s->spec.purk.xyz.clear(); s->spec.purk.xyz.shrink_to_fit();
    s->spec.purk.edges.clear(); s->spec.purk.edges.shrink_to_fit();
    return EP_OK;
}

ep_status ep_footprint(const ep_sim *s, size_t *bytes) {
    if (!s || !bytes) return EP_EINVAL;
    if (!s->inited) return EP_ESTATE;
    *bytes = s->inst.footprint;
    return EP_OK;
}

ep_status ep_set_launch(ep_sim *s, int32_t block, int32_t steps_per_graph, int32_t xcd_remap) {
    if (!s) return EP_EINVAL;
    if (block != 0 && block != 64 && block != 128 && block != 256)
        return fail(s, EP_EINVAL, "block must be 0 (keep), 64, 128 or 256");
    if (steps_per_graph < 0) return fail(s, EP_EINVAL, "steps_per_graph must be >= 0");
    if (xcd_remap < 0 || xcd_remap > 3) return fail(s, EP_EINVAL, "xcd_remap must be 0, 1, 2 or 3");
    s->stepper.steps_per_graph = steps_per_graph;
    s->stepper.remap = xcd_remap;
    if (block && block != s->stepper.cell_threads) {
        s->stepper.cell_threads = block;
        s->stepper.dirty = true;
    }
    return EP_OK;
}

ep_status ep_set_tile_size(ep_sim *s, int32_t cells) {
    if (!s) return EP_EINVAL;
    if (cells != 64 && cells != 128 && cells != 256)
        return fail(s, EP_EINVAL, "a cell tile holds 64, 128 or 256 cells");
    if (cells != s->stepper.cell_threads) {
        s->stepper.cell_threads = cells;
        s->stepper.dirty = true;
    }
    return EP_OK;
}

ep_status ep_get_launch(ep_sim *s, int32_t *tile_cells, int32_t *steps_per_graph,
                        int32_t *xcd_remap) {
    if (!s) return EP_EINVAL;
    if (tile_cells) *tile_cells = s->stepper.cell_threads;
    if (steps_per_graph) *steps_per_graph = s->stepper.steps_per_graph;
    if (xcd_remap) *xcd_remap = s->stepper.remap;
    return EP_OK;
}

ep_status ep_step(ep_sim *s, int64_t n) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (n < 0) return fail(s, EP_EINVAL, "negative step count");
    if (n == 0) return EP_OK;
    HIP_TRY(s, hipSetDevice(s->opt.device));
    if (!s->inst.bido) return run_err(s, ep::stepper_run(s->stepper, n));
    // bidomain: the elliptic solve follows every step
    for (int64_t i = 0; i < n && s->inst.host_step < s->inst.target; ++i) {
        std::string e = ep::stepper_run(s->stepper, 1);
        if (e.empty()) e = ep::bidomain_solve(s->inst, s->stream);
        if (!e.empty()) return fail(s, EP_EDEVICE, e);
    }
    return EP_OK;
}

ep_status ep_sync(ep_sim *s) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    HIP_TRY(s, hipSetDevice(s->opt.device));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    int32_t flag = 0;
    HIP_TRY(s, hipMemcpy(&flag, &s->inst.d_ctrl->nan_flag, sizeof(flag), hipMemcpyDeviceToHost));
    if (flag) return fail(s, EP_ENUMERIC, "non-finite membrane potential");
    return EP_OK;
}

static ep_status read_cells(ep_sim *s, const void *dev, int bytes_per, std::vector<double> &host) {
    const int64_t nc = s->inst.desc.nc;
    host.resize(nc);
    if (bytes_per == 8) {
        HIP_TRY(s, hipMemcpy(host.data(), dev, nc * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(nc);
        HIP_TRY(s, hipMemcpy(tmp.data(), dev, nc * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < nc; ++i) host[i] = tmp[i];
    }
    return EP_OK;
}

static ep_status readout(ep_sim *s, const void *dev, int bytes_per, double *out, int64_t n) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (!out || n != s->inst.desc.nc) return fail(s, EP_EINVAL, "output length must equal n_tets");
    ep_status st = ep_sync(s);
    if (st != EP_OK && st != EP_ENUMERIC) return st;
    std::vector<double> h;
    ep_status st2 = read_cells(s, dev, bytes_per, h);
    if (st2 != EP_OK) return st2;
    for (int64_t i = 0; i < n; ++i) out[s->inst.prep.perm[i]] = h[i];
    return st;
}

static void *cur_v(ep_sim *s) { return s->inst.desc.v[s->inst.host_step & 1]; }

ep_status ep_get_vm(ep_sim *s, double *out, int64_t n) {
    if (!s) return EP_EINVAL;
    return readout(s, cur_v(s), s->inst.rs, out, n);
}

ep_status ep_get_activation(ep_sim *s, double *t_act, int64_t n) {
    if (!s) return EP_EINVAL;
    return readout(s, s->inst.desc.t_act, 8, t_act, n);
}

ep_status ep_get_apd90(ep_sim *s, double *apd, int64_t n) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (!apd || n != s->inst.desc.nc) return fail(s, EP_EINVAL, "output length must equal n_tets");
    std::vector<double> ta(n), tr(n);
    ep_status st = readout(s, s->inst.desc.t_act, 8, ta.data(), n);
    if (st != EP_OK && st != EP_ENUMERIC) return st;
    ep_status st2 = readout(s, s->inst.desc.t_rep, 8, tr.data(), n);
    if (st2 != EP_OK && st2 != EP_ENUMERIC) return st2;
    for (int64_t i = 0; i < n; ++i) apd[i] = tr[i] - ta[i];   // NaN propagates
    return st;
}

ep_status ep_get_mean_vm_trace(ep_sim *s, double *t, double *vbar, int64_t cap, int64_t *n_out) {
    if (!s || !n_out) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (cap < 0 || (cap > 0 && (!t || !vbar))) return fail(s, EP_EINVAL, "bad trace buffers");
    ep_status st = ep_sync(s);
    if (st != EP_OK && st != EP_ENUMERIC) return st;
    const int every = s->inst.trace_every;
    int64_t avail = every > 0 ? std::min<int64_t>(s->inst.trace_cap, s->inst.host_step / every + 1) : 1;
    int64_t m = std::min(cap, avail);
    std::vector<double> tr(std::max<int64_t>(m, 1));
    if (m > 0) HIP_TRY(s, hipMemcpy(tr.data(), s->inst.desc.trace, m * 8, hipMemcpyDeviceToHost));
    // the sample of the last step issued is still held as per-tile partials
    // (the next step's node gather would add them): add them here, in the
    // device's order
    const int64_t hs = s->inst.host_step;
    if (every > 0 && hs > 0 && hs % every == 0 && hs / every < m) {
        const int ng = (s->inst.desc.n_waves + 3) / 4;   // groups of four wave partials
        std::vector<double> part(4 * (size_t)ng);
        HIP_TRY(s, hipMemcpy(part.data(), s->inst.desc.part, part.size() * 8, hipMemcpyDeviceToHost));
        double red[epdev::TILE];
        for (int t = 0; t < epdev::TILE; ++t) {
            double acc = 0.0;
            for (int g = t; g < ng; g += epdev::TILE)
                acc += (part[4 * g] + part[4 * g + 1]) + (part[4 * g + 2] + part[4 * g + 3]);
            red[t] = acc;
        }
        for (int w = epdev::TILE / 2; w > 0; w >>= 1)
            for (int t = 0; t < w; ++t) red[t] += red[t + w];
        tr[hs / every] = red[0] * s->inst.desc.inv_total_vol;
    }
    for (int64_t i = 0; i < m; ++i) {
        t[i] = (double)(i * (int64_t)std::max(every, 1)) * s->inst.dt;
        vbar[i] = tr[i];
    }
    *n_out = m;
    return st;
}

static ep_status diffusion_args(ep_sim *s, const double *v, double *L, int64_t n) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (!v || !L || n != s->inst.desc.nc) return fail(s, EP_EINVAL, "v and L must hold n_tets values");
    if (v == L) return fail(s, EP_EINVAL, "L may not alias v");
    return EP_OK;
}

ep_status ep_apply_diffusion(ep_sim *s, const double *v, double *L, int64_t n) {
    ep_status st = diffusion_args(s, v, L, n);
    if (st != EP_OK) return st;
    HIP_TRY(s, hipSetDevice(s->opt.device));
    const size_t bytes = ep::diffusion_workspace_bytes(s->inst);
    void *ws = nullptr;
    if (s->opt.dev_alloc) ws = s->opt.dev_alloc(bytes, s->opt.alloc_ctx);
    else if (hipMalloc(&ws, bytes) != hipSuccess) ws = nullptr;
    if (!ws) return fail(s, EP_ENOMEM, "diffusion workspace allocation failed");
    std::string e = ep::diffusion_apply(s->inst, s->stream, v, L, ws);
    const hipError_t es = hipStreamSynchronize(s->stream);
    if (s->opt.dev_free) s->opt.dev_free(ws, s->opt.alloc_ctx);
    else (void)hipFree(ws);
    if (!e.empty()) return fail(s, EP_EDEVICE, e);
    if (es != hipSuccess) return fail(s, EP_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(es));
    return EP_OK;
}

ep_status ep_apply_diffusion_noalloc(ep_sim *s, const double *v, double *L, int64_t n) {
    ep_status st = diffusion_args(s, v, L, n);
    if (st != EP_OK) return st;
    HIP_TRY(s, hipSetDevice(s->opt.device));
    ep_status code = EP_OK;
    std::string e = ep::diffusion_apply_noalloc(s->inst, s->opt.device, s->stream, v, L, code);
    if (!e.empty()) return fail(s, code, e);
    return EP_OK;
}

ep_status ep_get_time(ep_sim *s, int64_t *step, double *t) {
    if (!s) return EP_EINVAL;
    if (step) *step = s->inst.host_step;
    if (t) *t = (double)s->inst.host_step * s->spec.dt;
    return EP_OK;
}

static const void *cur_pv(ep_sim *s) {
    return s->inst.pdesc.pv[(s->inst.host_step * s->inst.pdesc.n_sub) & 1];
}

static ep_status purkinje_readout(ep_sim *s, const void *dev, int bytes_per, double *out, int64_t n) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (s->inst.pk.n == 0) return fail(s, EP_ESTATE, "no Purkinje graph");
    if (!out || n != s->inst.pk.n) return fail(s, EP_EINVAL, "output length must equal the graph size");
    ep_status st = ep_sync(s);
    if (st != EP_OK && st != EP_ENUMERIC) return st;
    if (bytes_per == 8) {
        HIP_TRY(s, hipMemcpy(out, dev, n * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(n);
        HIP_TRY(s, hipMemcpy(tmp.data(), dev, n * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) out[i] = tmp[i];
    }
    return st;
}

ep_status ep_get_purkinje_vm(ep_sim *s, double *out, int64_t n) {
    if (!s) return EP_EINVAL;
    return purkinje_readout(s, s->inited ? cur_pv(s) : nullptr, s->inst.rs, out, n);
}

ep_status ep_get_purkinje_activation(ep_sim *s, double *out, int64_t n) {
    if (!s) return EP_EINVAL;
    return purkinje_readout(s, s->inst.pdesc.pt_act, 8, out, n);
}

ep_status ep_get_phi_e(ep_sim *s, double *out, int64_t n) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (!s->inst.bido) return fail(s, EP_ESTATE, "not a bidomain simulation");
    return readout(s, s->inst.bd.phi, 8, out, n);
}

ep_status ep_get_bidomain_stats(ep_sim *s, int64_t *last_iters, int64_t *total_iters,
                                double *last_relres) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (!s->inst.bido) return fail(s, EP_ESTATE, "not a bidomain simulation");
    if (last_iters) *last_iters = s->inst.bd.last_iters;
    if (total_iters) *total_iters = s->inst.bd.total_iters;
    if (last_relres) *last_relres = s->inst.bd.last_relres;
    return EP_OK;
}

ep_status ep_get_purkinje_substeps(ep_sim *s, int32_t *n_sub) {
    if (!s || !n_sub) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    *n_sub = s->inst.pk.n > 0 ? s->inst.pk.n_sub : 0;
    return EP_OK;
}

int ep_model_n_slots(int model) {
    switch (model) {
    case EP_TP06_ENDO: case EP_TP06_MID: case EP_TP06_EPI: return 19;
    case EP_CRN: return 21;
    case EP_STEWART: return 20;
    case EP_PASSIVE: return 1;
    default: return 0;
    }
}

const char *ep_model_slot_name(int model, int slot) {
    if (slot < 0 || slot >= ep_model_n_slots(model)) return nullptr;
    if (model <= 2) return TP06_NAMES[slot];
    if (model == 3) return CRN_NAMES[slot];
    if (model == 4) return STEWART_NAMES[slot];
    return "V";
}

ep_status ep_get_states(ep_sim *s, double *out, int64_t n, int32_t n_slots) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    const int64_t nc = s->inst.desc.nc;
    if (!out || n != nc || n_slots != EP_MAX_SLOTS) return fail(s, EP_EINVAL, "bad state buffer");
    ep_status st = ep_sync(s);
    if (st != EP_OK && st != EP_ENUMERIC) return st;
    std::vector<double> v, gate(tiled_len(nc, NG_MAX)), conc(tiled_len(nc, NC_MAX));
    ep_status e = read_cells(s, cur_v(s), s->inst.rs, v);
    if (e != EP_OK) return e;
    if (s->inst.rs == 8) {
        HIP_TRY(s, hipMemcpy(gate.data(), s->inst.desc.gate, gate.size() * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> g(gate.size());
        HIP_TRY(s, hipMemcpy(g.data(), s->inst.desc.gate, g.size() * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < g.size(); ++i) gate[i] = g[i];
    }
    HIP_TRY(s, hipMemcpy(conc.data(), s->inst.desc.conc, conc.size() * 8, hipMemcpyDeviceToHost));
    const double nan = std::numeric_limits<double>::quiet_NaN();
    for (int64_t i = 0; i < nc; ++i) {
        const int64_t u = s->inst.prep.perm[i];
        const int m = s->inst.prep.model[i];
        const int ng = model_ng(m), ncc = model_nc(m);
        for (int k = 0; k < EP_MAX_SLOTS; ++k) out[(size_t)k * nc + u] = nan;
        out[u] = v[i];
        for (int k = 0; k < ng; ++k) out[(size_t)(1 + k) * nc + u] = gate[tix(i, k, NG_MAX)];
        for (int k = 0; k < ncc; ++k) out[(size_t)(1 + ng + k) * nc + u] = conc[tix(i, k, NC_MAX)];
    }
    return st;
}

ep_status ep_set_states(ep_sim *s, const double *in, int64_t n, int32_t n_slots) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    const int64_t nc = s->inst.desc.nc;
    if (!in || n != nc || n_slots != EP_MAX_SLOTS) return fail(s, EP_EINVAL, "bad state buffer");
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    std::vector<double> v(nc), gate(tiled_len(nc, NG_MAX), 0.0), conc(tiled_len(nc, NC_MAX), 0.0);
    for (int64_t i = 0; i < nc; ++i) {
        const int64_t u = s->inst.prep.perm[i];
        const int m = s->inst.prep.model[i];
        const int ng = model_ng(m), ncc = model_nc(m);
        v[i] = in[u];
        for (int k = 0; k < ng; ++k) gate[tix(i, k, NG_MAX)] = in[(size_t)(1 + k) * nc + u];
        for (int k = 0; k < ncc; ++k) conc[tix(i, k, NC_MAX)] = in[(size_t)(1 + ng + k) * nc + u];
    }
    void *dv = cur_v(s);
    if (s->inst.rs == 8) {
        HIP_TRY(s, hipMemcpy(dv, v.data(), nc * 8, hipMemcpyHostToDevice));
        HIP_TRY(s, hipMemcpy(s->inst.desc.gate, gate.data(), gate.size() * 8, hipMemcpyHostToDevice));
        if (s->inst.host_step == 0)   // a state set before the first step defines v_rest
            HIP_TRY(s, hipMemcpy((void *)s->inst.desc.vrest, v.data(), nc * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> vf(v.begin(), v.end()), gf(gate.begin(), gate.end());
        HIP_TRY(s, hipMemcpy(dv, vf.data(), nc * 4, hipMemcpyHostToDevice));
        HIP_TRY(s, hipMemcpy(s->inst.desc.gate, gf.data(), gf.size() * 4, hipMemcpyHostToDevice));
        if (s->inst.host_step == 0)
            HIP_TRY(s, hipMemcpy((void *)s->inst.desc.vrest, vf.data(), nc * 4, hipMemcpyHostToDevice));
    }
    HIP_TRY(s, hipMemcpy(s->inst.desc.conc, conc.data(), conc.size() * 8, hipMemcpyHostToDevice));
    return EP_OK;
}

// ----------------------------------------------------------- checkpoints
struct CkptHeader {
    uint64_t magic;
    int64_t n_tets, n_nodes, step;
    int32_t rs, n_pmj;
    int64_t trace_cap, n_purkinje;
    int64_t bidomain;
    int64_t time_scheme;
    int64_t ordering;         // EP_ORDER_* the image was taken under
    uint64_t layout_hash;     // of the internal order and each cell's model
};

// FNV-1a over the internal-to-caller cell permutation and the per-cell
// model bytes in internal order: the arrays of an image are stored in that
// order, so an image restores only into a simulation with the same layout
// (another cell order or another model assignment over the same mesh size
// would scramble every per-cell array).
static uint64_t layout_hash(const ep_sim *s) {
    uint64_t h = 0xcbf29ce484222325ULL;
    auto mix = [&h](const void *p, size_t n) {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 0x100000001b3ULL; }
    };
    mix(s->inst.prep.perm.data(), s->inst.prep.perm.size() * sizeof(int32_t));
    mix(s->inst.prep.model.data(), s->inst.prep.model.size());
    mix(&s->inst.sub2, sizeof(s->inst.sub2));
    return h;
}

static std::vector<std::pair<void *, size_t>> ckpt_arrays(ep_sim *s) {
    const epdev::InstDesc &D = s->inst.desc;
    const size_t nc = D.nc, r = s->inst.rs;
    std::vector<std::pair<void *, size_t>> a = {
        {D.v[0], nc * r},           {D.v[1], nc * r},        {D.gate, tiled_len(nc, NG_MAX) * r},
        {D.conc, tiled_len(nc, NC_MAX) * 8},  {D.dstat, nc}, {D.t_act, nc * 8},
        {D.t_rep, nc * 8},          {D.vmax, nc * r},        {(void *)D.vrest, nc * r},
        {D.trace, (size_t)s->inst.trace_cap * 8}, {D.part, (size_t)(D.n_waves + 3) / 4 * 32},
        {s->inst.d_ctrl, sizeof(epdev::Ctrl)}};
    if (s->inst.bido) a.push_back({s->inst.bd.phi, nc * 8});
    if (s->inst.ab2) {
        a.push_back({D.hv, nc * r});
        a.push_back({D.hc, tiled_len(nc, NC_MAX) * 8});
    }
    if (ep::has_junction_block(s->inst)) {
        const epdev::PurkDesc &P = s->inst.pdesc;
        const size_t np = P.np;             // 0 when only cells are junction sources
        a.push_back({P.pv[0], np * r});
        a.push_back({P.pv[1], np * r});
        a.push_back({P.gate, tiled_len(np, NG_MAX) * r});
        a.push_back({P.conc, tiled_len(np, NC_MAX) * 8});
        a.push_back({P.pstat, np});
        a.push_back({P.pt_act, np * 8});
        a.push_back({P.pmj, std::max<size_t>(P.n_pmj, 1) * sizeof(epdev::Pmj)});
        if (s->inst.ab2) {
            a.push_back({P.hv, np * r});
            a.push_back({P.hc, tiled_len(np, NC_MAX) * 8});
        }
    }
    a.erase(std::remove_if(a.begin(), a.end(), [](const auto &x) { return x.second == 0; }), a.end());
    return a;
}

ep_status ep_state_size(ep_sim *s, size_t *bytes) {
    if (!s || !bytes) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    size_t b = sizeof(CkptHeader);
    for (auto &a : ckpt_arrays(s)) b += a.second;
    *bytes = b;
    return EP_OK;
}

ep_status ep_get_state(ep_sim *s, void *buf, size_t bytes) {
    size_t need = 0;
    ep_status st = ep_state_size(s, &need);
    if (st != EP_OK) return st;
    if (!buf || bytes < need) return fail(s, EP_EINVAL, "checkpoint buffer too small");
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    CkptHeader h{CKPT_MAGIC, s->inst.desc.nc, s->inst.desc.nn, s->inst.host_step, s->inst.rs,
                 (int32_t)s->inst.n_pmj, s->inst.trace_cap, s->inst.pk.n, s->inst.bido ? 1 : 0,
                 s->inst.scheme, s->spec.ordering, layout_hash(s)};
    char *p = (char *)buf;
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    for (auto &a : ckpt_arrays(s)) {
        HIP_TRY(s, hipMemcpy(p, a.first, a.second, hipMemcpyDeviceToHost));
        p += a.second;
    }
    return EP_OK;
}

ep_status ep_set_state(ep_sim *s, const void *buf, size_t bytes) {
    size_t need = 0;
    ep_status st = ep_state_size(s, &need);
    if (st != EP_OK) return st;
    if (!buf || bytes < need) return fail(s, EP_EINVAL, "checkpoint buffer too small");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof(h));
    if (h.magic != CKPT_MAGIC || h.n_tets != s->inst.desc.nc || h.n_nodes != s->inst.desc.nn ||
        h.rs != s->inst.rs || h.trace_cap != s->inst.trace_cap || h.n_purkinje != s->inst.pk.n ||
        h.n_pmj != (int32_t)s->inst.n_pmj || h.bidomain != (s->inst.bido ? 1 : 0) ||
        h.time_scheme != s->inst.scheme)
        return fail(s, EP_EINVAL, "checkpoint does not match this simulation");
    if (h.ordering != s->spec.ordering || h.layout_hash != layout_hash(s))
        return fail(s, EP_EINVAL, "checkpoint was taken under another cell order or model layout");
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const char *p = (const char *)buf + sizeof(h);
    for (auto &a : ckpt_arrays(s)) {
        HIP_TRY(s, hipMemcpy(a.first, p, a.second, hipMemcpyHostToDevice));
        p += a.second;
    }
    s->inst.host_step = h.step;
    return EP_OK;
}

// ------------------------------------------------------------- profiling
ep_status ep_autotune(ep_sim *s, int64_t trial_steps, int32_t *steps_per_graph,
                      int32_t *xcd_remap, double *ms_per_step) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (trial_steps <= 0) return fail(s, EP_EINVAL, "trial_steps must be positive");
    HIP_TRY(s, hipSetDevice(s->opt.device));
    ep::TuneResult r;
    std::string e = ep::stepper_autotune(s->stepper, trial_steps, r);
    if (!e.empty()) return fail(s, EP_EDEVICE, e);
    if (steps_per_graph) *steps_per_graph = r.steps_per_graph;
    if (xcd_remap) *xcd_remap = r.xcd_remap;
    if (ms_per_step) *ms_per_step = r.ms_per_step;
    return EP_OK;
}

ep_status ep_profile_steps(ep_sim *s, int64_t n, int32_t every, double *cell_ms,
                           double *node_ms, double *step_ms) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (n <= 0) return fail(s, EP_EINVAL, "n must be positive");
    if (every <= 0) return fail(s, EP_EINVAL, "every must be positive");
    HIP_TRY(s, hipSetDevice(s->opt.device));
    double a = 0, b = 0;
    std::string e = ep::stepper_profile(s->stepper, n, every, a, b, step_ms);
    if (!e.empty()) return fail(s, EP_EDEVICE, e);
    if (cell_ms) *cell_ms = a;
    if (node_ms) *node_ms = b;
    return EP_OK;
}

ep_status ep_algorithmic_bytes(const ep_sim *s, double *node_bytes, double *cell_bytes,
                               double *diffusion_bytes) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return EP_ESTATE;
    const double r = s->inst.rs, nc = (double)s->inst.desc.nc, nn = (double)s->inst.desc.nn;
    // node gather: every incidence (index + weight; 4 per tet, 3 per
    // triangle), every v once, vn write
    const double ninc = (double)s->inst.prep.n_incidences;
    const double gather = ninc * (4.0 + r) + nc * r + nn * r + 8.0 * s->inst.n_slices;
    if (node_bytes) *node_bytes = gather;
    // cell kernel: stencil (8 node ids + 8 coefficients + 4 neighbours + 4
    // coefficients; 16-bit ids plus two 32-bit bases per 256 cells when the
    // instance has them), vn once, v^n once, v^{n+1} write, model byte, state
    // read+write, detection status byte; with Adams-Bashforth 2 the previous
    // rates of v and of the non-gating states, read and written (none are
    // read on step 0)
    const double ids = s->inst.idx16 ? 12 * 2.0 + 8.0 / epdev::LB : 12 * 4.0;
    double b = nc * (ids + 8 * r + 4 * r + r + r + 1.0 + 1.0) + nn * r;
    for (uint8_t m : s->inst.prep.model) {
        b += 2.0 * (model_ng(m) * r + model_nc(m) * 8.0);
        if (s->inst.ab2) b += 2.0 * (r + model_nc(m) * 8.0);
    }
    if (cell_bytes) *cell_bytes = b;
    // ep_apply_diffusion: caller v (FP64) and the permutation in, internal
    // copy out; the node gather of that copy; the stencil, vn once, the
    // copy once, the permutation again and L (FP64) out
    if (diffusion_bytes)
        *diffusion_bytes = nc * (8.0 + 4.0 + r) + gather + nc * (ids + 12 * r + r + 4.0 + 8.0) + nn * r;
    return EP_OK;
}

}  // extern "C"
