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
#include "kernels.hpp"
#include "prep.hpp"

using namespace epdev;

namespace {

constexpr uint64_t CKPT_MAGIC = 0x4550534d43484b31ULL;   // "EPSMCHK1"

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

const char *const TP06_NAMES[] = {"V", "m", "h", "j", "xr1", "xr2", "xs", "r", "s", "d",
                                  "f", "f2", "fCass", "Rbar", "Ca_i", "Ca_SR", "Ca_SS",
                                  "Na_i", "K_i"};
const char *const CRN_NAMES[] = {"V", "m", "h", "j", "oa", "oi", "ua", "ui", "xr", "xs", "d",
                                 "f", "fCa", "u", "v", "w", "Ca_i", "Ca_up", "Ca_rel",
                                 "Na_i", "K_i"};
const char *const STEWART_NAMES[] = {"V", "m", "h", "j", "xr1", "xr2", "xs", "r", "s", "d",
                                     "f", "f2", "fCass", "y", "Rbar", "Ca_i", "Ca_SR",
                                     "Ca_SS", "Na_i", "K_i"};

struct Stim {
    std::vector<int32_t> ids;   // caller numbering
    double t0, dur, amp, period;
    int32_t count;
};

}  // namespace

struct ep_sim {
    ep_options opt;
    std::string err;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // inputs
    std::vector<double> xyz, fibre, scale;
    std::vector<int32_t> tets;
    std::vector<uint8_t> model;
    double sigma_l = 0.17, sigma_t = 0.019;
    bool has_scale = false, has_cond = false;
    double gscale[4] = {1, 1, 1, 1};
    std::vector<Stim> stims;
    int ordering = ep::ORDER_RCM;
    // geometry
    int64_t nn = 0, nc = 0;
    bool inited = false;
    ep::PrepOut prep;
    int mset = 0;
    int64_t n_slices = 0;
    double inv_total_vol = 0.0;
    // device memory
    std::vector<std::pair<void *, size_t>> allocs;
    size_t footprint = 0;
    int rs = 8;                       // sizeof(R)
    void *d_sell_off = nullptr, *d_sell_cell = nullptr, *d_sell_w = nullptr;
    void *d_cnode = nullptr, *d_cbeta = nullptr, *d_cnbr = nullptr, *d_cb = nullptr;
    void *d_vn = nullptr, *d_v[2] = {nullptr, nullptr};
    void *d_gate = nullptr, *d_conc = nullptr, *d_model = nullptr, *d_smask = nullptr;
    void *d_dstat = nullptr, *d_tact = nullptr, *d_trep = nullptr, *d_vmax = nullptr;
    void *d_vrest = nullptr, *d_vol = nullptr, *d_part = nullptr, *d_trace = nullptr;
    Ctrl *d_ctrl = nullptr;
    int n_parts = 0;
    int64_t trace_cap = 0;
    // stepping
    int64_t host_step = 0;            // mirror of ctrl->step after queued work
    int parity = 0;                   // which v buffer holds v^n
    int block = 256;
    int steps_per_graph = 50;
    int remap = 1;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_k = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
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

void *dev_alloc(ep_sim *s, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (s->opt.dev_alloc) {
        p = s->opt.dev_alloc(bytes, s->opt.alloc_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) {
        s->allocs.push_back({p, bytes});
        s->footprint += bytes;
    }
    return p;
}

void free_all(ep_sim *s) {
    for (auto &a : s->allocs) {
        if (s->opt.dev_free) s->opt.dev_free(a.first, s->opt.alloc_ctx);
        else (void)hipFree(a.first);
    }
    s->allocs.clear();
    s->footprint = 0;
    for (int i = 0; i < 2; ++i)
        if (s->graph[i]) { (void)hipGraphExecDestroy(s->graph[i]); s->graph[i] = nullptr; }
}

template <typename T>
ep_status upload(ep_sim *s, void **dst, const std::vector<T> &src) {
    *dst = dev_alloc(s, src.size() * sizeof(T));
    if (!*dst) return fail(s, EP_ENOMEM, "device allocation failed");
    // synchronous: the sources are often temporaries
    HIP_TRY(s, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return EP_OK;
}

template <typename R>
std::vector<R> cast(const std::vector<double> &v) {
    return std::vector<R>(v.begin(), v.end());
}

template <typename R>
CellArgs<R> cell_args(ep_sim *s, int p) {
    CellArgs<R> a;
    a.n = s->nc;
    a.cnode = (const int32_t *)s->d_cnode;
    a.cbeta = (const R *)s->d_cbeta;
    a.cnbr = (const int32_t *)s->d_cnbr;
    a.cb = (const R *)s->d_cb;
    a.vn = (const R *)s->d_vn;
    a.vin = (const R *)s->d_v[p];
    a.vout = (R *)s->d_v[p ^ 1];
    a.gate = (R *)s->d_gate;
    a.conc = (double *)s->d_conc;
    a.model = (const uint8_t *)s->d_model;
    a.smask = (const uint32_t *)s->d_smask;
    a.dstat = (uint8_t *)s->d_dstat;
    a.t_act = (double *)s->d_tact;
    a.t_rep = (double *)s->d_trep;
    a.vmax = (R *)s->d_vmax;
    a.vrest = (const R *)s->d_vrest;
    a.ctrl = s->d_ctrl;
    a.dt = R(s->opt.dt);
    a.dtd = s->opt.dt;
    a.thr = R(s->opt.at_threshold);
    a.repol = R(s->opt.repol_frac);
    a.gs = GScale{s->gscale[0], s->gscale[1], s->gscale[2], s->gscale[3]};
    return a;
}

template <typename R>
void launch_cell(ep_sim *s, int p, int32_t off) {
    const int64_t nb = (s->nc + s->block - 1) / s->block;
    CellArgs<R> a = cell_args<R>(s, p);
    switch (s->mset) {
    case 1: k_cell<R, 1><<<nb, s->block, 0, s->stream>>>(a, off, s->remap); break;
    case 8: k_cell<R, 8><<<nb, s->block, 0, s->stream>>>(a, off, s->remap); break;
    default: k_cell<R, 15><<<nb, s->block, 0, s->stream>>>(a, off, s->remap); break;
    }
}

template <typename R>
void launch_nodes(ep_sim *s, int p) {
    const int64_t nb = (s->nn + s->block - 1) / s->block;
    k_node_gather<R><<<nb, s->block, 0, s->stream>>>(
        s->nn, (const int64_t *)s->d_sell_off, (const int32_t *)s->d_sell_cell,
        (const R *)s->d_sell_w, (const R *)s->d_v[p], (R *)s->d_vn, s->remap);
}

template <typename R>
void launch_trace(ep_sim *s, int p, int32_t off) {
    k_vsum_partial<R><<<s->n_parts, 256, 0, s->stream>>>(s->nc, (const R *)s->d_v[p],
                                                         (const double *)s->d_vol,
                                                         (double *)s->d_part);
    k_vsum_final<<<1, 256, 0, s->stream>>>(s->n_parts, (const double *)s->d_part,
                                           s->inv_total_vol, s->d_ctrl, off,
                                           s->opt.trace_every, s->trace_cap,
                                           (double *)s->d_trace);
}

// Enqueue k steps starting from buffer parity p and a step counter that
// stands at `base` when they run (base is only used to place trace samples).
void enqueue_steps(ep_sim *s, int p, int64_t base, int64_t k) {
    for (int64_t i = 0; i < k; ++i) {
        const int q = (p + (int)(i & 1)) & 1;
        if (s->rs == 8) { launch_nodes<double>(s, q); launch_cell<double>(s, q, (int32_t)i); }
        else { launch_nodes<float>(s, q); launch_cell<float>(s, q, (int32_t)i); }
        const int32_t every = s->opt.trace_every;
        if (every > 0 && (base + i + 1) % every == 0) {
            if (s->rs == 8) launch_trace<double>(s, q ^ 1, (int32_t)(i + 1));
            else launch_trace<float>(s, q ^ 1, (int32_t)(i + 1));
        }
    }
    k_advance<<<1, 1, 0, s->stream>>>(s->d_ctrl, k);
}

ep_status capture_graph(ep_sim *s, int p) {
    hipGraph_t g = nullptr;
    HIP_TRY(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    // graph replays start on a multiple of the graph length, which is a
    // multiple of trace_every, so trace samples fall at fixed offsets
    enqueue_steps(s, p, 0, s->graph_k);
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    if (e != hipSuccess) return fail(s, EP_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&s->graph[p], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(s, EP_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    return EP_OK;
}

ep_status check_launch(ep_sim *s) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(s, EP_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return EP_OK;
}

int slot_count(uint8_t m) { return ep_model_n_slots(m); }

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
    s->rs = o->prec == EP_FP64 ? 8 : 4;
    if (o->stream) {
        s->stream = (hipStream_t)o->stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return EP_EDEVICE;
        }
        s->own_stream = true;
    }
    for (int i = 0; i < 4; ++i)
        if (hipEventCreate(&s->ev[i]) != hipSuccess) { ep_destroy(s); return EP_EDEVICE; }
    *out = s;
    return EP_OK;
}

void ep_destroy(ep_sim *s) {
    if (!s) return;
    (void)hipSetDevice(s->opt.device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    free_all(s);
    for (int i = 0; i < 4; ++i) if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
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
        if (tet_nodes[i] < 0 || tet_nodes[i] >= n_nodes)
            return fail(s, EP_EINVAL, "tet node index out of range");
    s->xyz.assign(xyz, xyz + 3 * n_nodes);
    s->tets.assign(tet_nodes, tet_nodes + 4 * n_tets);
    s->nn = n_nodes;
    s->nc = n_tets;
    s->model.assign(n_tets, EP_TP06_ENDO);
    s->fibre.clear();
    s->has_cond = false;
    s->stims.clear();
    return EP_OK;
}

ep_status ep_set_conductivity(ep_sim *s, const double *fibre, double sigma_l, double sigma_t,
                              const double *scale) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "frozen after ep_init");
    if (s->nc == 0) return fail(s, EP_ESTATE, "set the mesh first");
    if (!fibre || !(sigma_l >= 0) || !(sigma_t >= 0)) return fail(s, EP_EINVAL, "bad conductivity");
    s->fibre.assign(fibre, fibre + 3 * s->nc);
    s->sigma_l = sigma_l;
    s->sigma_t = sigma_t;
    s->has_scale = scale != nullptr;
    if (scale) s->scale.assign(scale, scale + s->nc);
    else s->scale.clear();
    s->has_cond = true;
    return EP_OK;
}

ep_status ep_set_models(ep_sim *s, const uint8_t *model) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "frozen after ep_init");
    if (s->nc == 0) return fail(s, EP_ESTATE, "set the mesh first");
    if (!model) return fail(s, EP_EINVAL, "null model array");
    for (int64_t c = 0; c < s->nc; ++c)
        if (model[c] > EP_PASSIVE) return fail(s, EP_EINVAL, "model id out of range");
    s->model.assign(model, model + s->nc);
    return EP_OK;
}

ep_status ep_set_ionic_scale(ep_sim *s, const char *param, double scale) {
    if (!s || !param) return EP_EINVAL;
    if (!(scale > 0) || !std::isfinite(scale)) return fail(s, EP_EINVAL, "scale must be > 0");
    const char *names[4] = {"GKr", "GKs", "GCaL", "GNa"};
    for (int i = 0; i < 4; ++i)
        if (std::strcmp(param, names[i]) == 0) {
            s->gscale[i] = scale;
            return EP_OK;
        }
    return fail(s, EP_EINVAL, std::string("unknown conductance ") + param);
}

ep_status ep_add_stimulus(ep_sim *s, int domain, int64_t n_ids, const int32_t *ids, double t0,
                          double dur, double amp, double period, int32_t count) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "stimuli are frozen after ep_init");
    if (domain != 0) return fail(s, EP_EINVAL, "only the tissue domain (0) takes stimuli");
    if (s->nc == 0) return fail(s, EP_ESTATE, "set the mesh first");
    if ((int)s->stims.size() >= EP_MAX_STIMULI) return fail(s, EP_EINVAL, "too many stimuli");
    if (n_ids < 0 || (n_ids > 0 && !ids) || !(dur >= 0) || !std::isfinite(amp) || period < 0)
        return fail(s, EP_EINVAL, "bad stimulus");
    for (int64_t i = 0; i < n_ids; ++i)
        if (ids[i] < 0 || ids[i] >= s->nc) return fail(s, EP_EINVAL, "stimulus id out of range");
    Stim st;
    st.ids.assign(ids, ids + n_ids);
    st.t0 = t0; st.dur = dur; st.amp = amp; st.period = period;
    st.count = count < 1 ? 1 : count;
    s->stims.push_back(std::move(st));
    return EP_OK;
}

static ep_status init_device(ep_sim *s);

ep_status ep_init(ep_sim *s) {
    if (!s) return EP_EINVAL;
    if (s->inited) return fail(s, EP_ESTATE, "already initialised");
    if (s->nc == 0) return fail(s, EP_ESTATE, "no mesh");
    if (!s->has_cond) return fail(s, EP_ESTATE, "no conductivity");
    HIP_TRY(s, hipSetDevice(s->opt.device));
    ep::PrepIn in;
    in.n_nodes = s->nn; in.n_tets = s->nc;
    in.xyz = s->xyz.data(); in.tets = s->tets.data(); in.fibre = s->fibre.data();
    in.scale = s->has_scale ? s->scale.data() : nullptr;
    in.model = s->model.data();
    in.sigma_l = s->sigma_l; in.sigma_t = s->sigma_t;
    in.chi = s->opt.chi; in.cm = s->opt.cm;
    in.ordering = s->ordering;
    std::string e = ep::prepare(in, s->prep);
    if (!e.empty()) return fail(s, EP_EINVAL, e);
    ep_status st = init_device(s);
    if (st != EP_OK) { free_all(s); return st; }
    s->inited = true;
    return EP_OK;
}

static ep_status init_device(ep_sim *s) {
    ep::PrepOut &P = s->prep;
    const int64_t nc = s->nc, nn = s->nn;
    s->n_slices = (int64_t)P.sell_off.size() - 1;
    ep_status st;
    if ((st = upload(s, &s->d_sell_off, P.sell_off)) != EP_OK) return st;
    if ((st = upload(s, &s->d_sell_cell, P.sell_cell)) != EP_OK) return st;
    if ((st = upload(s, &s->d_cnode, P.cnode)) != EP_OK) return st;
    if ((st = upload(s, &s->d_cnbr, P.cnbr)) != EP_OK) return st;
    if ((st = upload(s, &s->d_model, P.model)) != EP_OK) return st;
    if ((st = upload(s, &s->d_vol, P.vol)) != EP_OK) return st;
    if (s->rs == 8) {
        if ((st = upload(s, &s->d_sell_w, P.sell_w)) != EP_OK) return st;
        if ((st = upload(s, &s->d_cbeta, P.cbeta)) != EP_OK) return st;
        if ((st = upload(s, &s->d_cb, P.cb)) != EP_OK) return st;
    } else {
        if ((st = upload(s, &s->d_sell_w, cast<float>(P.sell_w))) != EP_OK) return st;
        if ((st = upload(s, &s->d_cbeta, cast<float>(P.cbeta))) != EP_OK) return st;
        if ((st = upload(s, &s->d_cb, cast<float>(P.cb))) != EP_OK) return st;
    }
    // models present -> kernel variant
    int present = 0;
    for (uint8_t m : P.model) present |= m <= 2 ? 1 : (m == 3 ? 2 : (m == 4 ? 4 : 8));
    s->mset = (present == 1 || present == 8) ? present : 15;

    // initial state, structure of arrays in internal order
    std::vector<double> v0(nc), gate((size_t)NG_MAX * nc, 0.0), conc((size_t)NC_MAX * nc, 0.0);
    for (int64_t i = 0; i < nc; ++i) {
        double y[EP_MAX_SLOTS];
        const int m = P.model[i];
        model_init(m, y);
        v0[i] = y[0];
        const int ng = model_ng(m), ncc = model_nc(m);
        for (int k = 0; k < ng; ++k) gate[(size_t)k * nc + i] = y[1 + k];
        for (int k = 0; k < ncc; ++k) conc[(size_t)k * nc + i] = y[1 + ng + k];
    }
    std::vector<uint32_t> smask(nc, 0);
    for (size_t k = 0; k < s->stims.size(); ++k)
        for (int32_t id : s->stims[k].ids) smask[P.iperm[id]] |= 1u << k;
    if ((st = upload(s, &s->d_smask, smask)) != EP_OK) return st;
    if ((st = upload(s, &s->d_conc, conc)) != EP_OK) return st;
    if (s->rs == 8) {
        if ((st = upload(s, &s->d_gate, gate)) != EP_OK) return st;
        if ((st = upload(s, &s->d_v[0], v0)) != EP_OK) return st;
        if ((st = upload(s, &s->d_v[1], v0)) != EP_OK) return st;
        if ((st = upload(s, &s->d_vrest, v0)) != EP_OK) return st;
        if ((st = upload(s, &s->d_vmax, v0)) != EP_OK) return st;
        if ((st = upload(s, &s->d_vn, std::vector<double>(nn, 0.0))) != EP_OK) return st;
    } else {
        if ((st = upload(s, &s->d_gate, cast<float>(gate))) != EP_OK) return st;
        if ((st = upload(s, &s->d_v[0], cast<float>(v0))) != EP_OK) return st;
        if ((st = upload(s, &s->d_v[1], cast<float>(v0))) != EP_OK) return st;
        if ((st = upload(s, &s->d_vrest, cast<float>(v0))) != EP_OK) return st;
        if ((st = upload(s, &s->d_vmax, cast<float>(v0))) != EP_OK) return st;
        if ((st = upload(s, &s->d_vn, std::vector<float>(nn, 0.0f))) != EP_OK) return st;
    }
    const double nan = std::numeric_limits<double>::quiet_NaN();
    if ((st = upload(s, &s->d_dstat, std::vector<uint8_t>(nc, 0))) != EP_OK) return st;
    if ((st = upload(s, &s->d_tact, std::vector<double>(nc, nan))) != EP_OK) return st;
    if ((st = upload(s, &s->d_trep, std::vector<double>(nc, nan))) != EP_OK) return st;

    // trace of vbar: sample 0 now, then every trace_every steps
    s->n_parts = (int)std::min<int64_t>(1024, (nc + 255) / 256);
    s->trace_cap = 1 << 16;
    double tv = 0.0, vt = 0.0;
    for (int64_t i = 0; i < nc; ++i) { tv += P.vol[i]; vt += P.vol[i] * v0[i]; }
    s->inv_total_vol = 1.0 / tv;
    std::vector<double> trace(s->trace_cap, nan);
    trace[0] = vt / tv;
    if ((st = upload(s, &s->d_trace, trace)) != EP_OK) return st;
    if ((st = upload(s, &s->d_part, std::vector<double>(s->n_parts, 0.0))) != EP_OK) return st;

    Ctrl ctrl;
    std::memset(&ctrl, 0, sizeof(ctrl));
    ctrl.n_stim = (int32_t)s->stims.size();
    for (size_t k = 0; k < s->stims.size(); ++k) {
        const Stim &q = s->stims[k];
        ctrl.st_n0[k] = std::llround(q.t0 / s->opt.dt);
        ctrl.st_ndur[k] = std::llround(q.dur / s->opt.dt);
        ctrl.st_nper[k] = q.period > 0 ? std::llround(q.period / s->opt.dt) : 0;
        ctrl.st_count[k] = q.count;
        ctrl.st_amp[k] = q.amp;
    }
    s->d_ctrl = (Ctrl *)dev_alloc(s, sizeof(Ctrl));
    if (!s->d_ctrl) return fail(s, EP_ENOMEM, "device allocation failed");
    HIP_TRY(s, hipMemcpy(s->d_ctrl, &ctrl, sizeof(ctrl), hipMemcpyHostToDevice));
    s->host_step = 0;
    s->parity = 0;
    return EP_OK;
}

ep_status ep_footprint(const ep_sim *s, size_t *bytes) {
    if (!s || !bytes) return EP_EINVAL;
    if (!s->inited) return EP_ESTATE;
    *bytes = s->footprint;
    return EP_OK;
}

ep_status ep_set_launch(ep_sim *s, int32_t block, int32_t steps_per_graph, int32_t xcd_remap) {
    if (!s) return EP_EINVAL;
    if (block < 64 || block > 1024 || block % 64) return fail(s, EP_EINVAL, "block must be a multiple of 64 in [64, 1024]");
    if (steps_per_graph < 0) return fail(s, EP_EINVAL, "steps_per_graph must be >= 0");
    if (block > 256) return fail(s, EP_EINVAL, "the cell kernel is compiled for blocks of at most 256");
    s->block = block;
    s->steps_per_graph = steps_per_graph;
    s->remap = xcd_remap ? 1 : 0;
    for (int i = 0; i < 2; ++i)
        if (s->graph[i]) { (void)hipGraphExecDestroy(s->graph[i]); s->graph[i] = nullptr; }
    return EP_OK;
}

ep_status ep_step(ep_sim *s, int64_t n) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (n < 0) return fail(s, EP_EINVAL, "negative step count");
    if (n == 0) return EP_OK;
    HIP_TRY(s, hipSetDevice(s->opt.device));
    const int every = s->opt.trace_every;
    // graph length: a multiple of the trace period and of 2 (buffer parity)
    int64_t k = 0;
    if (s->steps_per_graph > 0) {
        k = s->steps_per_graph;
        if (every > 0) k = ((k + every - 1) / every) * every;
        if (k % 2) k *= 2;
    }
    if (k != s->graph_k) {
        for (int i = 0; i < 2; ++i)
            if (s->graph[i]) { (void)hipGraphExecDestroy(s->graph[i]); s->graph[i] = nullptr; }
        s->graph_k = (int)k;
    }
    int64_t left = n;
    // head: direct launches up to a multiple of k
    if (k > 0 && left >= k) {
        int64_t head = (k - s->host_step % k) % k;
        if (head > 0) {
            enqueue_steps(s, s->parity, s->host_step, head);
            s->host_step += head;
            s->parity ^= (int)(head & 1);
            left -= head;
        }
        while (left >= k) {
            if (!s->graph[s->parity]) {
                ep_status st = capture_graph(s, s->parity);
                if (st != EP_OK) return st;
            }
            HIP_TRY(s, hipGraphLaunch(s->graph[s->parity], s->stream));
            s->host_step += k;
            left -= k;
        }
    }
    if (left > 0) {
        enqueue_steps(s, s->parity, s->host_step, left);
        s->host_step += left;
        s->parity ^= (int)(left & 1);
    }
    return check_launch(s);
}

ep_status ep_sync(ep_sim *s) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    HIP_TRY(s, hipSetDevice(s->opt.device));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    int32_t flag = 0;
    HIP_TRY(s, hipMemcpy(&flag, &s->d_ctrl->nan_flag, sizeof(flag), hipMemcpyDeviceToHost));
    if (flag) return fail(s, EP_ENUMERIC, "non-finite membrane potential");
    return EP_OK;
}

static ep_status read_cells(ep_sim *s, const void *dev, int bytes_per, std::vector<double> &host) {
    const int64_t nc = s->nc;
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
    if (!out || n != s->nc) return fail(s, EP_EINVAL, "output length must equal n_tets");
    ep_status st = ep_sync(s);
    if (st != EP_OK && st != EP_ENUMERIC) return st;
    std::vector<double> h;
    ep_status st2 = read_cells(s, dev, bytes_per, h);
    if (st2 != EP_OK) return st2;
    for (int64_t i = 0; i < s->nc; ++i) out[s->prep.perm[i]] = h[i];
    return st;
}

ep_status ep_get_vm(ep_sim *s, double *out, int64_t n) {
    if (!s) return EP_EINVAL;
    return readout(s, s->d_v[s->parity], s->rs, out, n);
}

ep_status ep_get_activation(ep_sim *s, double *t_act, int64_t n) {
    if (!s) return EP_EINVAL;
    return readout(s, s->d_tact, 8, t_act, n);
}

ep_status ep_get_apd90(ep_sim *s, double *apd, int64_t n) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (!apd || n != s->nc) return fail(s, EP_EINVAL, "output length must equal n_tets");
    std::vector<double> ta(n), tr(n);
    ep_status st = readout(s, s->d_tact, 8, ta.data(), n);
    if (st != EP_OK && st != EP_ENUMERIC) return st;
    ep_status st2 = readout(s, s->d_trep, 8, tr.data(), n);
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
    const int every = s->opt.trace_every;
    int64_t avail = every > 0 ? std::min<int64_t>(s->trace_cap, s->host_step / every + 1) : 1;
    int64_t m = std::min(cap, avail);
    std::vector<double> tr(std::max<int64_t>(m, 1));
    if (m > 0) HIP_TRY(s, hipMemcpy(tr.data(), s->d_trace, m * 8, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m; ++i) {
        t[i] = (double)(i * (int64_t)std::max(every, 1)) * s->opt.dt;
        vbar[i] = tr[i];
    }
    *n_out = m;
    return st;
}

ep_status ep_get_time(ep_sim *s, int64_t *step, double *t) {
    if (!s) return EP_EINVAL;
    if (step) *step = s->host_step;
    if (t) *t = (double)s->host_step * s->opt.dt;
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
    if (!out || n != s->nc || n_slots != EP_MAX_SLOTS) return fail(s, EP_EINVAL, "bad state buffer");
    ep_status st = ep_sync(s);
    if (st != EP_OK && st != EP_ENUMERIC) return st;
    const int64_t nc = s->nc;
    std::vector<double> v, gate((size_t)NG_MAX * nc), conc((size_t)NC_MAX * nc);
    ep_status e = read_cells(s, s->d_v[s->parity], s->rs, v);
    if (e != EP_OK) return e;
    if (s->rs == 8) {
        HIP_TRY(s, hipMemcpy(gate.data(), s->d_gate, gate.size() * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> g(gate.size());
        HIP_TRY(s, hipMemcpy(g.data(), s->d_gate, g.size() * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < g.size(); ++i) gate[i] = g[i];
    }
    HIP_TRY(s, hipMemcpy(conc.data(), s->d_conc, conc.size() * 8, hipMemcpyDeviceToHost));
    const double nan = std::numeric_limits<double>::quiet_NaN();
    for (int64_t i = 0; i < nc; ++i) {
        const int64_t u = s->prep.perm[i];
        const int m = s->prep.model[i];
        const int ng = model_ng(m), ncc = model_nc(m);
        for (int k = 0; k < EP_MAX_SLOTS; ++k) out[(size_t)k * nc + u] = nan;
        out[u] = v[i];
        for (int k = 0; k < ng; ++k) out[(size_t)(1 + k) * nc + u] = gate[(size_t)k * nc + i];
        for (int k = 0; k < ncc; ++k) out[(size_t)(1 + ng + k) * nc + u] = conc[(size_t)k * nc + i];
    }
    return st;
}

ep_status ep_set_states(ep_sim *s, const double *in, int64_t n, int32_t n_slots) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (!in || n != s->nc || n_slots != EP_MAX_SLOTS) return fail(s, EP_EINVAL, "bad state buffer");
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const int64_t nc = s->nc;
    std::vector<double> v(nc), gate((size_t)NG_MAX * nc, 0.0), conc((size_t)NC_MAX * nc, 0.0);
    for (int64_t i = 0; i < nc; ++i) {
        const int64_t u = s->prep.perm[i];
        const int m = s->prep.model[i];
        const int ng = model_ng(m), ncc = model_nc(m);
        v[i] = in[u];
        for (int k = 0; k < ng; ++k) gate[(size_t)k * nc + i] = in[(size_t)(1 + k) * nc + u];
        for (int k = 0; k < ncc; ++k) conc[(size_t)k * nc + i] = in[(size_t)(1 + ng + k) * nc + u];
    }
    void *dv = s->d_v[s->parity];
    if (s->rs == 8) {
        HIP_TRY(s, hipMemcpy(dv, v.data(), nc * 8, hipMemcpyHostToDevice));
        HIP_TRY(s, hipMemcpy(s->d_gate, gate.data(), gate.size() * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> vf(v.begin(), v.end()), gf(gate.begin(), gate.end());
        HIP_TRY(s, hipMemcpy(dv, vf.data(), nc * 4, hipMemcpyHostToDevice));
        HIP_TRY(s, hipMemcpy(s->d_gate, gf.data(), gf.size() * 4, hipMemcpyHostToDevice));
    }
    HIP_TRY(s, hipMemcpy(s->d_conc, conc.data(), conc.size() * 8, hipMemcpyHostToDevice));
    if (s->host_step == 0) {   // a state set before the first step defines v_rest
        if (s->rs == 8) {
            HIP_TRY(s, hipMemcpy(s->d_vrest, v.data(), nc * 8, hipMemcpyHostToDevice));
        } else {
            std::vector<float> vf(v.begin(), v.end());
            HIP_TRY(s, hipMemcpy(s->d_vrest, vf.data(), nc * 4, hipMemcpyHostToDevice));
        }
    }
    return EP_OK;
}

// ----------------------------------------------------------- checkpoints
struct CkptHeader {
    uint64_t magic;
    int64_t n_tets, n_nodes, step;
    int32_t rs, parity;
    int64_t trace_cap;
};

static std::vector<std::pair<void *, size_t>> ckpt_arrays(ep_sim *s) {
    const size_t nc = s->nc, r = s->rs;
    return {{s->d_v[0], nc * r},      {s->d_v[1], nc * r},   {s->d_gate, NG_MAX * nc * r},
            {s->d_conc, NC_MAX * nc * 8}, {s->d_dstat, nc},  {s->d_tact, nc * 8},
            {s->d_trep, nc * 8},      {s->d_vmax, nc * r},   {s->d_vrest, nc * r},
            {s->d_trace, (size_t)s->trace_cap * 8}, {s->d_ctrl, sizeof(Ctrl)}};
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
    CkptHeader h{CKPT_MAGIC, s->nc, s->nn, s->host_step, s->rs, s->parity, s->trace_cap};
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
    if (h.magic != CKPT_MAGIC || h.n_tets != s->nc || h.n_nodes != s->nn || h.rs != s->rs ||
        h.trace_cap != s->trace_cap)
        return fail(s, EP_EINVAL, "checkpoint does not match this simulation");
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const char *p = (const char *)buf + sizeof(h);
    for (auto &a : ckpt_arrays(s)) {
        HIP_TRY(s, hipMemcpy(a.first, p, a.second, hipMemcpyHostToDevice));
        p += a.second;
    }
    s->host_step = h.step;
    s->parity = h.parity;
    return EP_OK;
}

// ------------------------------------------------------------- profiling
ep_status ep_profile_steps(ep_sim *s, int64_t n, double *cell_ms, double *node_ms) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return fail(s, EP_ESTATE, "ep_init first");
    if (n <= 0) return fail(s, EP_EINVAL, "n must be positive");
    HIP_TRY(s, hipSetDevice(s->opt.device));
    double tc = 0.0, tn = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const int q = s->parity;
        HIP_TRY(s, hipEventRecord(s->ev[0], s->stream));
        if (s->rs == 8) launch_nodes<double>(s, q); else launch_nodes<float>(s, q);
        HIP_TRY(s, hipEventRecord(s->ev[1], s->stream));
        if (s->rs == 8) launch_cell<double>(s, q, 0); else launch_cell<float>(s, q, 0);
        HIP_TRY(s, hipEventRecord(s->ev[2], s->stream));
        const int every = s->opt.trace_every;
        if (every > 0 && (s->host_step + 1) % every == 0) {
            if (s->rs == 8) launch_trace<double>(s, q ^ 1, 1); else launch_trace<float>(s, q ^ 1, 1);
        }
        k_advance<<<1, 1, 0, s->stream>>>(s->d_ctrl, 1);
        s->host_step += 1;
        s->parity ^= 1;
        HIP_TRY(s, hipEventSynchronize(s->ev[2]));
        float a = 0.f, b = 0.f;
        HIP_TRY(s, hipEventElapsedTime(&a, s->ev[0], s->ev[1]));
        HIP_TRY(s, hipEventElapsedTime(&b, s->ev[1], s->ev[2]));
        tn += a;
        tc += b;
    }
    if (cell_ms) *cell_ms = tc / n;
    if (node_ms) *node_ms = tn / n;
    return check_launch(s);
}

ep_status ep_algorithmic_bytes(const ep_sim *s, double *node_bytes, double *cell_bytes) {
    if (!s) return EP_EINVAL;
    if (!s->inited) return EP_ESTATE;
    const double r = s->rs, nc = (double)s->nc, nn = (double)s->nn;
    // node gather: 4 incidences per tet (index + weight), every v once, vn write
    if (node_bytes) *node_bytes = 4.0 * nc * (4.0 + r) + nc * r + nn * r + 8.0 * s->n_slices;
    // cell kernel: stencil (8 node ids + 8 coefficients + 4 neighbours + 4
    // coefficients), vn once, v^n once, v^{n+1} write, model byte, state
    // read+write, detection status byte
    double b = nc * (8 * 4.0 + 8 * r + 4 * 4.0 + 4 * r + r + r + 1.0 + 1.0) + nn * r;
    for (uint8_t m : s->prep.model) b += 2.0 * (model_ng(m) * r + model_nc(m) * 8.0);
    if (cell_bytes) *cell_bytes = b;
    return EP_OK;
}

}  // extern "C"
