// Single-GPU serving loop: continuous batching of independent simulations.
//
// Requests are copied at submission, precomputed on host worker threads,
// then admitted by a driver thread in arrival order while their exact device
// footprint fits the budget and a slot is free (later, smaller requests may
// pass one that does not fit yet).  Live instances are stepped together by
// the batched kernels, k steps per HIP graph launch; membership changes only
// rewrite the device tables between launches.  An instance that reaches its
// last step is retired: its results are copied out on the same stream, it
// leaves the tables, and its memory is freed once an event shows that no
// queued launch can still touch it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ep.h"
#include "admission.hpp"
#include "instance.hpp"

namespace {

enum ReqState { Q_PREP = 0, Q_READY = 1, Q_RUNNING = 2, Q_DONE = 3 };

struct Req {
    int64_t id = 0;
    ep::InstSpec spec;
    ep::Inst inst;
    size_t footprint = 0;
    int state = Q_PREP;
    ep_status status = EP_OK;
    std::string err;
    double t_submit = 0, t_ready = 0, t_admit = 0, t_done = 0;
    void *h_res = nullptr;             // pinned: t_act, t_rep (f64), v (R), NaN flag,
                                       // then graph t_act (f64) and v (R)
    std::vector<double> vm, tact, apd, pvm, pact;
};

struct Retire {
    std::vector<Req *> reqs;
    hipEvent_t ev = nullptr;
    void *h_group = nullptr;           // pinned results of all of reqs
};

}  // namespace

struct ep_server {
    ep_options opt{};
    int rs = 8;
    size_t budget = 0;
    int max_slots = 1;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_prep, cv_driver, cv_done;
    std::deque<int64_t> prep_q;
    std::deque<int64_t> ready_q;
    std::map<int64_t, std::unique_ptr<Req>> reqs;
    std::vector<std::thread> workers;
    std::thread driver;
    bool stop = false;
    int64_t next_id = 1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    ep::Stepper stepper;
    size_t in_use = 0;
    ep_server_stats stats{};
    std::string err;
    std::string driver_err;
    int32_t want_k = 50, want_remap = 1;   // launch settings, applied by the driver
    int32_t tile_cells = 256;                // cell tile size in effect (set by the driver)
    int32_t scheme = 0;                    // time scheme of every request
    // autotuning requests, served by the driver on the live batch
    bool hold = false;                     // admit and upload, but do not step
    bool tune_pending = false, tune_retune = false;
    int64_t tune_trial = 0;
    size_t tuned_live = 0;
    // steps issued since the last tuning, and the steps that tuning took:
    // retuning waits until the batch has advanced ten times as far, so that
    // the trials (each ends in a wait for the device) stay a small share
    int64_t steps_since_tune = 0, tune_steps = 0;
};

namespace {

double now_s(ep_server *sv) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - sv->t0).count();
}

ep_status sfail(ep_server *sv, ep_status st, const std::string &m) {
    if (sv) {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->err = m;
    }
    return st;
}

void worker_main(ep_server *sv) {
    for (;;) {
        int64_t id;
        Req *r;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_prep.wait(lk, [&] { return sv->stop || !sv->prep_q.empty(); });
            if (sv->stop) return;
            id = sv->prep_q.front();
            sv->prep_q.pop_front();
            r = sv->reqs[id].get();
        }
        ep_status st = EP_OK;
        std::string e = ep::prep_instance(r->spec, r->inst, st);
        size_t fp = e.empty() ? ep::instance_footprint(r->inst, sv->rs, r->spec) : 0;
        // the mesh arrays are not needed after the precompute
        r->spec.xyz.clear(); r->spec.xyz.shrink_to_fit();
        r->spec.tets.clear(); r->spec.tets.shrink_to_fit();
        r->spec.fibre.clear(); r->spec.fibre.shrink_to_fit();
        r->spec.scale.clear(); r->spec.scale.shrink_to_fit();
        {
            std::lock_guard<std::mutex> g(sv->mu);
            if (!e.empty() || fp > sv->budget) {
                r->status = e.empty() ? EP_ENOMEM : st;
                r->err = e.empty() ? "request larger than the HBM budget" : e;
                r->state = Q_DONE;
                r->t_done = now_s(sv);
                sv->stats.queued--;
                sv->stats.completed++;
                sv->cv_done.notify_all();
            } else {
                r->footprint = fp;
                r->state = Q_READY;
                r->t_ready = now_s(sv);
                sv->ready_q.push_back(id);
                sv->cv_driver.notify_all();
            }
        }
    }
}

// Tissue part of a request's staged results: t_act, t_rep (f64), v (R), NaN
// flag; the graph part (t_act f64, v R) follows at this offset.
size_t tissue_bytes(const Req *r, int rs) {
    const size_t nc = (size_t)r->inst.desc.nc;
    return (nc * 16 + nc * (size_t)rs + 8 + 255) / 256 * 256;
}

// Copy the results of a group of finished instances into one pinned buffer
// (stream order).
void *stage_results(ep_server *sv, const std::vector<Req *> &fin) {
    auto bytes_of = [&](const Req *r) {
        const size_t np = (size_t)r->inst.pk.n;
        return tissue_bytes(r, sv->rs) + (np * 8 + np * (size_t)sv->rs + 255) / 256 * 256;
    };
    size_t total = 0;
    for (const Req *r : fin) total += bytes_of(r);
    void *grp = nullptr;
    if (hipHostMalloc(&grp, std::max<size_t>(total, 256)) != hipSuccess) {
        for (Req *r : fin) r->h_res = nullptr;
        return nullptr;
    }
    char *p = (char *)grp;
    for (Req *r : fin) {
        const size_t nc = (size_t)r->inst.desc.nc;
        const epdev::InstDesc &D = r->inst.desc;
        r->h_res = p;
        (void)hipMemcpyAsync(p, D.t_act, nc * 8, hipMemcpyDeviceToHost, sv->stream);
        (void)hipMemcpyAsync(p + nc * 8, D.t_rep, nc * 8, hipMemcpyDeviceToHost, sv->stream);
        (void)hipMemcpyAsync(p + nc * 16, D.v[r->inst.host_step & 1], nc * sv->rs,
                             hipMemcpyDeviceToHost, sv->stream);
        (void)hipMemcpyAsync(p + nc * 16 + nc * sv->rs, &r->inst.d_ctrl->nan_flag, sizeof(int32_t),
                             hipMemcpyDeviceToHost, sv->stream);
        if (r->inst.pk.n > 0) {
            const epdev::PurkDesc &P = r->inst.pdesc;
            const size_t np = (size_t)P.np;
            char *q = p + tissue_bytes(r, sv->rs);
            (void)hipMemcpyAsync(q, P.pt_act, np * 8, hipMemcpyDeviceToHost, sv->stream);
            (void)hipMemcpyAsync(q + np * 8, P.pv[(r->inst.host_step * P.n_sub) & 1],
                                 np * sv->rs, hipMemcpyDeviceToHost, sv->stream);
        }
        p += bytes_of(r);
    }
    return grp;
}

// Unpack the staged results of a request (after its group's copies are
// done) and release its device memory.
void finish(ep_server *sv, Req *r) {
    const int64_t nc = r->inst.desc.nc;
    int32_t nan_flag = 0;
    if (r->h_res) {
        const double *ta = (const double *)r->h_res;
        const double *tr = ta + nc;
        const char *vb = (const char *)(tr + nc);
        std::memcpy(&nan_flag, vb + nc * sv->rs, sizeof(nan_flag));
        r->vm.assign(nc, 0.0);
        r->tact.assign(nc, 0.0);
        r->apd.assign(nc, 0.0);
        for (int64_t i = 0; i < nc; ++i) {
            const int64_t u = r->inst.prep.perm[i];
            r->tact[u] = ta[i];
            r->apd[u] = tr[i] - ta[i];
            r->vm[u] = sv->rs == 8 ? ((const double *)vb)[i] : (double)((const float *)vb)[i];
        }
        const int64_t np = r->inst.pk.n;
        if (np > 0) {
            // graph nodes keep the caller's numbering
            const char *q = (const char *)r->h_res + tissue_bytes(r, sv->rs);
            r->pact.assign((const double *)q, (const double *)q + np);
            r->pvm.resize(np);
            for (int64_t i = 0; i < np; ++i)
                r->pvm[i] = sv->rs == 8 ? ((const double *)(q + np * 8))[i]
                                        : (double)((const float *)(q + np * 8))[i];
        }
        r->h_res = nullptr;                 // part of its group's buffer
    } else if (r->status == EP_OK) {
        r->status = EP_ENOMEM;
        r->err = "pinned result buffer allocation failed";
    }
    if (nan_flag && r->status == EP_OK) {
        r->status = EP_ENUMERIC;
        r->err = "non-finite membrane potential";
    }
    const size_t fp = r->footprint;
    ep::free_instance(r->inst);
    r->inst.prep = ep::PrepOut();
    std::lock_guard<std::mutex> g(sv->mu);
    sv->in_use -= fp;
    r->state = Q_DONE;
    r->t_done = now_s(sv);
    sv->stats.running--;
    sv->stats.completed++;
    sv->cv_done.notify_all();
    sv->cv_driver.notify_all();
}

void driver_main(ep_server *sv) {
    (void)hipSetDevice(sv->opt.device);
    std::vector<Req *> live;
    std::deque<Retire> retiring;
    std::deque<hipEvent_t> inflight;
    auto new_event = [&]() {
        hipEvent_t e = nullptr;
        (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
        return e;
    };
    for (;;) {
        // ---- admission (arrival order, smaller requests may pass)
        std::vector<Req *> admit;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->stop) break;
            sv->stepper.steps_per_graph = sv->want_k;
            sv->stepper.remap = sv->want_remap;
            size_t used = sv->in_use;
            const size_t slots = live.size();
            std::vector<size_t> fp;
            fp.reserve(sv->ready_q.size());
            for (int64_t id : sv->ready_q) fp.push_back(sv->reqs[id]->footprint);
            const size_t free_slots = (size_t)std::max<int64_t>(0, (int64_t)sv->max_slots - (int64_t)slots);
            const std::vector<size_t> pick = ep::admit_ready(fp, used, sv->budget, free_slots);
            std::deque<int64_t> rest;
            for (size_t i = 0, k = 0; i < sv->ready_q.size(); ++i) {
                if (k < pick.size() && pick[k] == i) {
                    admit.push_back(sv->reqs[sv->ready_q[i]].get());
                    ++k;
                } else {
                    rest.push_back(sv->ready_q[i]);
                }
            }
            sv->ready_q.swap(rest);
            sv->in_use = used;
        }
        bool changed = false;
        ep::Allocator al{sv->opt.dev_alloc, sv->opt.dev_free, sv->opt.alloc_ctx};
        for (Req *r : admit) {
            ep_status st = EP_OK;
            std::string e = ep::upload_instance(r->spec, sv->rs, al, r->inst, st);
            std::lock_guard<std::mutex> g(sv->mu);
            sv->stats.queued--;
            if (!e.empty()) {
                sv->in_use -= r->footprint;
                r->status = st;
                r->err = e;
                r->state = Q_DONE;
                r->t_done = now_s(sv);
                sv->stats.completed++;
                sv->cv_done.notify_all();
                continue;
            }
            r->state = Q_RUNNING;
            r->t_admit = now_s(sv);
            sv->stats.running++;
            live.push_back(r);
            changed = true;
        }
        // ---- retire instances that reached their last step
        std::vector<Req *> fin;
        for (Req *r : live)
            if (r->inst.host_step >= r->inst.target) fin.push_back(r);
        void *h_group = nullptr;
        if (!fin.empty()) {
            h_group = stage_results(sv, fin);
            live.erase(std::remove_if(live.begin(), live.end(),
                                      [&](Req *r) { return r->inst.host_step >= r->inst.target; }),
                       live.end());
            changed = true;
        }
        if (changed) {
            sv->stepper.insts.clear();
            for (Req *r : live) sv->stepper.insts.push_back(&r->inst);
            std::string e = ep::stepper_sync_tables(sv->stepper);
            if (!e.empty()) { std::lock_guard<std::mutex> g(sv->mu); sv->driver_err = e; }
            std::lock_guard<std::mutex> g(sv->mu);
            sv->stats.table_updates++;
        }
        if (!fin.empty()) {
            Retire rt;
            rt.reqs = fin;
            rt.h_group = h_group;
            rt.ev = new_event();
            (void)hipEventRecord(rt.ev, sv->stream);
            retiring.push_back(rt);
        }
        // ---- held: requests are admitted and uploaded, nothing steps
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->hold && !sv->stop) {
                sv->cv_driver.wait_for(lk, std::chrono::milliseconds(20), [&] {
                    return sv->stop || !sv->hold || !sv->ready_q.empty();
                });
                continue;
            }
        }
        // ---- autotune the schedule on the live batch when asked
        bool tune = false;
        int64_t trial = 0;
        {
            std::lock_guard<std::mutex> g(sv->mu);
            const size_t n = live.size(), m = sv->tuned_live;
            tune = n > 0 && sv->tune_trial > 0 &&
                   (sv->tune_pending ||
                    (sv->tune_retune && n >= 4 && (n >= 2 * m || 2 * n <= m) &&
                     sv->steps_since_tune >= 10 * sv->tune_steps));
            trial = sv->tune_trial;
        }
        // tet-steps issued by a stepping call (progress of the live batch)
        auto issued_since = [&](const std::vector<int64_t> &h0) {
            double c = 0;
            for (size_t i = 0; i < live.size(); ++i)
                c += (double)live[i]->inst.desc.nc * (double)(live[i]->inst.host_step - h0[i]);
            return c;
        };
        auto steps_now = [&]() {
            std::vector<int64_t> h(live.size());
            for (size_t i = 0; i < live.size(); ++i) h[i] = live[i]->inst.host_step;
            return h;
        };
        if (tune) {
            ep::TuneResult r;
            const std::vector<int64_t> h0 = steps_now();
            std::string e = ep::stepper_autotune(sv->stepper, trial, r, false);
            const double c = issued_since(h0);
            std::lock_guard<std::mutex> g(sv->mu);
            sv->stats.cell_steps += c;
            if (!e.empty()) sv->driver_err = e;
            sv->want_k = r.steps_per_graph;
            sv->want_remap = r.xcd_remap;
            sv->tile_cells = r.cell_threads;
            sv->tune_pending = false;
            sv->tuned_live = live.size();
            sv->steps_since_tune = 0;
            sv->tune_steps = r.steps_used;
            sv->stats.autotune_runs++;
            sv->stats.tuned_ms_per_step = r.ms_per_step;
            sv->stats.graph_launches += r.n_trials;
        }
        // ---- step every live instance
        if (!live.empty()) {
            const int64_t k = sv->stepper.steps_per_graph;
            const std::vector<int64_t> h0 = steps_now();
            std::string e = ep::stepper_run(sv->stepper, k);
            const double c = issued_since(h0);
            if (!e.empty()) { std::lock_guard<std::mutex> g(sv->mu); sv->driver_err = e; }
            hipEvent_t ev = new_event();
            (void)hipEventRecord(ev, sv->stream);
            inflight.push_back(ev);
            std::lock_guard<std::mutex> g(sv->mu);
            sv->stats.graph_launches++;
            sv->stats.cell_steps += c;
            sv->steps_since_tune += k;
        }
        // ---- keep at most two launches queued ahead of the host
        while (inflight.size() > 2) {
            (void)hipEventSynchronize(inflight.front());
            (void)hipEventDestroy(inflight.front());
            inflight.pop_front();
        }
        // ---- free retired instances whose copies are done
        while (!retiring.empty() &&
               (live.empty() || hipEventQuery(retiring.front().ev) == hipSuccess)) {
            (void)hipEventSynchronize(retiring.front().ev);
            for (Req *r : retiring.front().reqs) finish(sv, r);
            if (retiring.front().h_group) (void)hipHostFree(retiring.front().h_group);
            (void)hipEventDestroy(retiring.front().ev);
            retiring.pop_front();
        }
        if (live.empty()) {
            while (!inflight.empty()) {
                (void)hipEventSynchronize(inflight.front());
                (void)hipEventDestroy(inflight.front());
                inflight.pop_front();
            }
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_driver.wait(lk, [&] { return sv->stop || !sv->ready_q.empty(); });
        }
    }
    // shutdown: drain the stream, release everything still resident
    (void)hipStreamSynchronize(sv->stream);
    for (hipEvent_t e : inflight) (void)hipEventDestroy(e);
    for (Retire &rt : retiring) {
        for (Req *r : rt.reqs) finish(sv, r);
        if (rt.h_group) (void)hipHostFree(rt.h_group);
        (void)hipEventDestroy(rt.ev);
    }
    for (Req *r : live) {
        ep::free_instance(r->inst);
        std::lock_guard<std::mutex> g(sv->mu);
        r->status = EP_ESTATE;
        r->err = "server destroyed before the request finished";
        r->state = Q_DONE;
    }
}

ep_status copy_request(const ep_request *rq, const ep_options &o, int32_t scheme, ep::InstSpec &sp,
                       std::string &err) {
    if (!rq || rq->n_nodes <= 0 || rq->n_tets <= 0 || !rq->xyz || !rq->tet_nodes || !rq->fibre ||
        rq->n_steps <= 0 || rq->n_stimuli < 0 || rq->n_stimuli > EP_MAX_STIMULI ||
        (rq->n_stimuli > 0 && !rq->stimuli) || !(rq->sigma_l >= 0) || !(rq->sigma_t >= 0)) {
        err = "malformed request";
        return EP_EINVAL;
    }
    for (int64_t i = 0; i < 4 * rq->n_tets; ++i)
        if ((rq->tet_nodes[i] < 0 && !(i % 4 == 3 && rq->tet_nodes[i] == -1)) ||
            rq->tet_nodes[i] >= rq->n_nodes) {
            err = "tet node index out of range";
            return EP_EINVAL;
        }
    sp.n_nodes = rq->n_nodes;
    sp.n_tets = rq->n_tets;
    sp.xyz.assign(rq->xyz, rq->xyz + 3 * rq->n_nodes);
    sp.tets.assign(rq->tet_nodes, rq->tet_nodes + 4 * rq->n_tets);
    sp.fibre.assign(rq->fibre, rq->fibre + 3 * rq->n_tets);
    sp.sigma_l = rq->sigma_l;
    sp.sigma_t = rq->sigma_t;
    sp.has_scale = rq->scale != nullptr;
    if (rq->scale) sp.scale.assign(rq->scale, rq->scale + rq->n_tets);
    if (rq->model) {
        for (int64_t c = 0; c < rq->n_tets; ++c)
            if (rq->model[c] > EP_PASSIVE) { err = "model id out of range"; return EP_EINVAL; }
        sp.model.assign(rq->model, rq->model + rq->n_tets);
    } else {
        sp.model.assign(rq->n_tets, EP_TP06_ENDO);
    }
    for (int i = 0; i < 4; ++i) {
        const double g = rq->ionic_scale[i];
        if (g < 0 || !std::isfinite(g)) { err = "bad ionic scale"; return EP_EINVAL; }
        sp.gscale[i] = g > 0 ? g : 1.0;
    }
    if (const ep_purkinje *g = rq->purkinje) {
        err = ep::spec_set_purkinje(sp, g->n, g->xyz, g->n_edges, g->edges, g->sigma, g->model,
                                    g->n_sub);
        if (err.empty() && g->edge_scale)
            err = ep::spec_set_purkinje_scale(sp, g->n_edges, g->edge_scale);
        if (err.empty() && (g->n_pmj < 0 || (g->n_pmj > 0 && !g->pmj))) err = "bad junction list";
        for (int32_t k = 0; err.empty() && k < g->n_pmj; ++k) {
            const ep_pmj &q = g->pmj[k];
            err = ep::spec_add_pmj(sp, q.node, q.radius, q.delay_ortho, q.delay_anti, q.two_way,
                                   q.amp, q.dur);
        }
        if (!err.empty()) return EP_EINVAL;
    }
    if (rq->n_cell_junctions < 0 || (rq->n_cell_junctions > 0 && !rq->cell_junctions)) {
        err = "bad cell junction list";
        return EP_EINVAL;
    }
    for (int32_t k = 0; k < rq->n_cell_junctions; ++k) {
        const ep_cell_junction &q = rq->cell_junctions[k];
        err = ep::spec_add_cell_junction(sp, q.cell, q.radius, q.delay_ortho, q.delay_anti,
                                         q.two_way, q.amp, q.dur);
        if (!err.empty()) return EP_EINVAL;
    }
    sp.scheme = scheme;
    if (rq->medium_substeps > (1 << 20)) { err = "more than 2^20 substeps"; return EP_EINVAL; }
    sp.medium_substeps = rq->medium_substeps == 0 ? 1 : (rq->medium_substeps < 0 ? 0 : rq->medium_substeps);
    for (int k = 0; k < rq->n_stimuli; ++k) {
        const ep_stimulus &q = rq->stimuli[k];
        if (q.domain == 1 && sp.purk.n == 0) {
            err = "graph stimulus without a Purkinje graph";
            return EP_EINVAL;
        }
        err = ep::spec_add_stimulus(sp, q.domain, q.n_ids, q.ids, q.t0, q.dur, q.amp, q.period,
                                    q.count);
        if (!err.empty()) return EP_EINVAL;
    }
    sp.dt = o.dt;
    sp.chi = o.chi;
    sp.cm = o.cm;
    sp.thr = o.at_threshold;
    sp.repol = o.repol_frac;
    sp.trace_every = o.trace_every;
    sp.target = rq->n_steps;
    return EP_OK;
}

}  // namespace

extern "C" {

ep_status ep_server_create(const ep_options *o, size_t hbm_budget, int32_t max_slots,
                           ep_server **out) {
    if (!o || !out || max_slots <= 0 || !(o->dt > 0) || !(o->chi > 0) || !(o->cm > 0) ||
        (o->prec != EP_FP64 && o->prec != EP_FP32_MIXED) ||
        ((o->dev_alloc == nullptr) != (o->dev_free == nullptr)))
        return EP_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0 || o->device < 0 || o->device >= ndev)
        return EP_EDEVICE;
    if (hipSetDevice(o->device) != hipSuccess) return EP_EDEVICE;
    ep_server *sv = new ep_server();
    sv->opt = *o;
    sv->rs = o->prec == EP_FP64 ? 8 : 4;
    sv->max_slots = max_slots;
    sv->t0 = std::chrono::steady_clock::now();
    if (hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete sv; return EP_EDEVICE; }
        hbm_budget = (size_t)(0.9 * (double)fr);
    }
    sv->budget = hbm_budget;
    sv->stats.bytes_budget = hbm_budget;
    if (o->stream) {
        sv->stream = (hipStream_t)o->stream;
    } else {
        if (hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
            delete sv;
            return EP_EDEVICE;
        }
        sv->own_stream = true;
    }
    if (!ep::stepper_init(sv->stepper, o->device, sv->stream, sv->rs).empty()) {
        if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
        delete sv;
        return EP_EDEVICE;
    }
    unsigned nw = std::max(1u, std::min(8u, std::thread::hardware_concurrency() / 2));
    for (unsigned i = 0; i < nw; ++i) sv->workers.emplace_back(worker_main, sv);
    sv->driver = std::thread(driver_main, sv);
    *out = sv;
    return EP_OK;
}

ep_status ep_server_submit(ep_server *sv, const ep_request *rq, int64_t *id) {
    if (!sv || !id) return EP_EINVAL;
    auto r = std::make_unique<Req>();
    std::string err;
    int32_t scheme;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        scheme = sv->scheme;
    }
    ep_status st = copy_request(rq, sv->opt, scheme, r->spec, err);
    if (st != EP_OK) return sfail(sv, st, err);
    if (ep::estimate_footprint(rq->n_tets, rq->n_nodes, sv->rs) > sv->budget * 2)
        return sfail(sv, EP_ENOMEM, "request cannot fit the HBM budget");
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stop) return EP_ESTATE;
    r->id = sv->next_id++;
    r->t_submit = now_s(sv);
    *id = r->id;
    sv->prep_q.push_back(r->id);
    sv->reqs[r->id] = std::move(r);
    sv->stats.submitted++;
    sv->stats.queued++;
    sv->cv_prep.notify_one();
    return EP_OK;
}

static void fill_result(const Req *r, ep_result *res) {
    res->id = r->id;
    res->status = r->status;
    res->n_tets = r->inst.prep.n_tets > 0 ? r->inst.prep.n_tets : r->spec.n_tets;
    res->steps = r->spec.target;
    res->footprint = r->footprint;
    res->t_submit = r->t_submit;
    res->t_admit = r->t_admit;
    res->t_done = r->t_done;
    res->t_ready = r->t_ready;
}

ep_status ep_server_poll(ep_server *sv, int64_t id, ep_result *res) {
    if (!sv || !res) return EP_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) { sv->err = "unknown request id"; return EP_EINVAL; }
    if (it->second->state != Q_DONE) return EP_EBUSY;
    fill_result(it->second.get(), res);
    return EP_OK;
}

ep_status ep_server_wait(ep_server *sv, int64_t id, ep_result *res) {
    if (!sv || !res) return EP_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) { sv->err = "unknown request id"; return EP_EINVAL; }
    Req *r = it->second.get();
    sv->cv_done.wait(lk, [&] { return r->state == Q_DONE; });
    fill_result(r, res);
    return EP_OK;
}

static ep_status get_vec(ep_server *sv, int64_t id, double *out, int64_t n, int which) {
    if (!sv || !out) return EP_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) { sv->err = "unknown request id"; return EP_EINVAL; }
    Req *r = it->second.get();
    if (r->state != Q_DONE) return EP_EBUSY;
    const std::vector<double> &v = which == 0 ? r->vm : which == 1 ? r->tact : which == 2 ? r->apd
                                 : which == 3 ? r->pvm : r->pact;
    if (which >= 3 && r->spec.purk.n == 0) { sv->err = "request has no Purkinje graph"; return EP_ESTATE; }
    if (v.empty()) { sv->err = r->err.empty() ? "no results" : r->err; return EP_ESTATE; }
    if (n != (int64_t)v.size()) {
        sv->err = which >= 3 ? "output length must equal the graph size" : "output length must equal n_tets";
        return EP_EINVAL;
    }
    std::memcpy(out, v.data(), n * sizeof(double));
    return r->status == EP_ENUMERIC ? EP_ENUMERIC : EP_OK;
}

ep_status ep_server_get_vm(ep_server *sv, int64_t id, double *out, int64_t n) {
    return get_vec(sv, id, out, n, 0);
}
ep_status ep_server_get_purkinje_vm(ep_server *sv, int64_t id, double *out, int64_t n) {
    return get_vec(sv, id, out, n, 3);
}
ep_status ep_server_get_purkinje_activation(ep_server *sv, int64_t id, double *out, int64_t n) {
    return get_vec(sv, id, out, n, 4);
}
ep_status ep_server_get_activation(ep_server *sv, int64_t id, double *out, int64_t n) {
    return get_vec(sv, id, out, n, 1);
}
ep_status ep_server_get_apd90(ep_server *sv, int64_t id, double *out, int64_t n) {
    return get_vec(sv, id, out, n, 2);
}

ep_status ep_server_release(ep_server *sv, int64_t id) {
    if (!sv) return EP_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return EP_EINVAL;
    if (it->second->state != Q_DONE) return EP_EBUSY;
    sv->reqs.erase(it);
    return EP_OK;
}

ep_status ep_server_get_stats(ep_server *sv, ep_server_stats *st) {
    if (!sv || !st) return EP_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    *st = sv->stats;
    st->bytes_in_use = sv->in_use;
    st->steps_per_graph = sv->want_k;
    st->xcd_remap = sv->want_remap;
    st->tile_cells = sv->tile_cells;
    if (!sv->driver_err.empty()) { sv->err = sv->driver_err; return EP_EDEVICE; }
    return EP_OK;
}

ep_status ep_server_set_launch(ep_server *sv, int32_t steps_per_graph, int32_t xcd_remap) {
    if (!sv || steps_per_graph <= 0 || xcd_remap < 0 || xcd_remap > 3) return EP_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    sv->want_k = steps_per_graph;           // applied by the driver between launches
    sv->want_remap = xcd_remap;
    return EP_OK;
}

ep_status ep_server_set_time_scheme(ep_server *sv, int32_t scheme) {
    if (!sv) return EP_EINVAL;
    if (scheme < EP_SCHEME_FE || scheme > EP_SCHEME_RL2_AB2) return sfail(sv, EP_EINVAL, "unknown time scheme");
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stats.submitted > 0) { sv->err = "the scheme is fixed once requests arrive"; return EP_ESTATE; }
    sv->scheme = scheme;
    return EP_OK;
}

ep_status ep_server_hold(ep_server *sv, int32_t hold) {
    if (!sv) return EP_EINVAL;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->hold = hold != 0;
    }
    sv->cv_driver.notify_all();
    return EP_OK;
}

ep_status ep_server_autotune(ep_server *sv, int64_t trial_steps, int32_t retune) {
    if (!sv || trial_steps <= 0) return EP_EINVAL;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->tune_trial = trial_steps;
        sv->tune_pending = true;
        sv->tune_retune = retune != 0;
    }
    sv->cv_driver.notify_all();
    return EP_OK;
}

void ep_server_destroy(ep_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stop = true;
    }
    sv->cv_prep.notify_all();
    sv->cv_driver.notify_all();
    if (sv->driver.joinable()) sv->driver.join();
    for (auto &t : sv->workers)
        if (t.joinable()) t.join();
    ep::stepper_free(sv->stepper);
    if (sv->own_stream && sv->stream) (void)hipStreamDestroy(sv->stream);
    delete sv;
}

const char *ep_server_last_error(ep_server *sv) {
    if (!sv) return "null server";
    std::lock_guard<std::mutex> g(sv->mu);
    thread_local std::string copy;
    copy = sv->err;
    return copy.c_str();
}

}  // extern "C"
