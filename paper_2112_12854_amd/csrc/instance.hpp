// Host-side objects behind the C ABI: one simulation instance on the device
// and a stepper that advances a set of instances with batched kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ep.h"
#include "kernels.hpp"
#include "prep.hpp"

namespace ep {

struct StimSpec {
    std::vector<int32_t> ids;   // caller numbering (tets, or graph nodes for domain 1)
    double t0 = 0, dur = 0, amp = 0, period = 0;
    int32_t count = 1;
    int32_t domain = 0;         // 0 tissue, 1 Purkinje graph
};

// Purkinje graph coupled to the tissue through junctions.
struct PurkSpec {
    int64_t n = 0;
    std::vector<double> xyz;
    std::vector<int32_t> edges;
    std::vector<double> edge_scale;    // per segment, empty = 1
    double sigma = 3.95;
    int32_t model = 4;
    int32_t n_sub = 0;
    std::vector<PmjIn> pmjs;
};

// Everything needed to build an instance (copied from the caller).
struct InstSpec {
    std::vector<double> xyz, fibre, scale;
    std::vector<int32_t> tets;
    std::vector<uint8_t> model;
    int64_t n_nodes = 0, n_tets = 0;
    double sigma_l = 0.17, sigma_t = 0.019;
    bool has_scale = false;
    double gscale[4] = {1, 1, 1, 1};   // GKr, GKs, GCaL, GNa
    std::vector<StimSpec> stims;
    int ordering = ORDER_RCM;
    double dt = 0.02, chi = 140.0, cm = 0.01, thr = 0.0, repol = 0.9;
    int32_t trace_every = 50;
    int64_t target = INT64_MAX;        // stop stepping at this step index
    PurkSpec purk;                     // n == 0: no graph
    // bidomain (sigma_l / sigma_t become the intracellular conductivities)
    bool bido = false;
    double sigma_el = 0.62, sigma_et = 0.24, bido_tol = 1e-6;
    int32_t bido_restart = 30, bido_max_iter = 2000;
    int32_t bido_coarse = 2048;        // aggregates of the preconditioner (0: none)
    // time scheme: 0 Rush-Larsen + forward Euler, 1 with Adams-Bashforth 2
    // for the non-gating states, 2 also with midpoint-rate (second-order)
    // Rush-Larsen gates
    int scheme = 0;
    // the 2D medium's substeps per step: 1 none, > 1 given, <= 0 from its
    // forward-Euler bound (90 %, 45 % with Adams-Bashforth 2)
    int32_t medium_substeps = 1;
};

// Device arrays of the extracellular solve of one bidomain instance.
struct Bido {
    double *phi = nullptr;             // [nc] phi_e, zero volume-weighted mean
    const double *ebeta = nullptr;     // elliptic stencil (flux-sum form), tile-major, 8 slots
    const double *eb = nullptr;        // tile-major, 4 slots
    double *xn = nullptr;              // [nn] node values of the operand
    double *b = nullptr, *w = nullptr; // [nc] right-hand side, work vector
    double *V = nullptr;               // [(restart+1)][nc] Krylov basis
    double *part = nullptr;            // [2][(restart+1)][blocks] reduction partials (two passes)
    double *h = nullptr;               // [2 restart + 4] reduced dot products
    double *y = nullptr;               // [restart] update coefficients
    int32_t restart = 30, max_iter = 2000;
    double tol = 1e-6, total_vol = 0, chi_cm = 1.4;
    int64_t last_iters = 0, total_iters = 0;
    double last_relres = 0;
    double *h_host = nullptr;          // pinned readback of h
    // GMRES state on the device (control block, Hessenberg matrix, Givens
    // rotations, reduced right-hand side, update coefficients) and the
    // captured graphs of the Arnoldi-step chunks (built at the first solve)
    double *gm = nullptr;
    std::vector<hipGraphExec_t> chunk_graphs;
    // two-level preconditioner
    int32_t n_agg = 0;
    const int32_t *agg_of = nullptr, *agg_off = nullptr, *agg_cells = nullptr;
    const double *dinv = nullptr;
    const float *cinv = nullptr;       // [n_agg][n_agg] A_c^{-1}, FP32
    double *z = nullptr, *t = nullptr; // [nc] preconditioned vector, update
    double *rc = nullptr, *zc = nullptr;   // [n_agg] coarse residual, correction
    bool precond = true;
};

struct Allocator {
    void *(*alloc)(size_t, void *) = nullptr;
    void (*free)(void *, void *) = nullptr;
    void *ctx = nullptr;
};

// Device state of one simulation.
struct Inst {
    int rs = 8;                        // sizeof(R): 8 FP64, 4 mixed
    PrepOut prep;
    int mset = 0;                      // model-set bits present
    bool idx16 = false;                // 16-bit stencil ids (InstDesc::idx16)
    // internal cells of each model class (bits 1 TP06, 2 CRN, 4 Stewart,
    // 8 passive, in that order): cells are grouped by class on the host
    int64_t cls_begin[4] = {0, 0, 0, 0}, cls_end[4] = {0, 0, 0, 0};
    // a 2D medium with a time step of its own (sub2 substeps per step): its
    // cells [c2, nc), grouped by class likewise, and nodes [n2, nn); without
    // one c2 = nc, n2 = nn and sub2 = 1
    int64_t cls2_begin[4] = {0, 0, 0, 0}, cls2_end[4] = {0, 0, 0, 0};
    int64_t c2 = 0, n2 = 0;
    int32_t sub2 = 1;
    Allocator al;
    std::vector<std::pair<void *, size_t>> allocs;
    // one device block per instance, carved in 256-byte aligned pieces (one
    // allocation and one free per instance); pieces beyond it are allocated
    // on their own
    char *arena = nullptr;
    size_t arena_size = 0, arena_used = 0;
    size_t footprint = 0;
    epdev::InstDesc desc{};            // device pointers and parameters
    int32_t *d_perm = nullptr;         // [nc] internal cell -> caller cell (device)
    epdev::Ctrl *d_ctrl = nullptr;
    int64_t host_step = 0;             // step index once queued work is done
    int64_t target = INT64_MAX;
    int64_t trace_cap = 0;
    int32_t trace_every = 50;
    double dt = 0.02;
    int64_t n_slices = 0;
    // Purkinje graph (pk.n == 0: none)
    PurkOut pk;                        // graph (pk.n nodes, possibly 0) and junctions
    int pmodel = 4;
    int64_t n_pmj = 0;
    epdev::PurkDesc pdesc{};
    bool bido = false;
    Bido bd;
    Coarse coarse;                     // host copy until upload
    bool ab2 = false;                  // Adams-Bashforth 2 history allocated
    int scheme = 0;
};

// An instance with a Purkinje graph or with junctions (of graph nodes or of
// cells) carries a PurkDesc: graph substeps (none for an empty graph) and the
// junction events.
inline bool has_junction_block(const Inst &I) { return I.pk.n > 0 || I.n_pmj > 0; }

// Host precompute only (thread-safe, no HIP calls).
// Validated edits of a spec, shared by the single-simulation API and the
// server's request copy; an empty string means success (EP_EINVAL otherwise).
std::string spec_set_purkinje(InstSpec &sp, int64_t n, const double *xyz, int64_t n_edges,
                              const int32_t *edges, double sigma, int32_t model, int32_t n_sub);
std::string spec_set_purkinje_scale(InstSpec &sp, int64_t n_edges, const double *scale);
std::string spec_add_pmj(InstSpec &sp, int32_t node, double radius, double delay_ortho,
                         double delay_anti, int32_t two_way, double amp, double dur);
std::string spec_add_cell_junction(InstSpec &sp, int32_t cell, double radius, double delay_ortho,
                                   double delay_anti, int32_t two_way, double amp, double dur);
std::string spec_add_stimulus(InstSpec &sp, int domain, int64_t n_ids, const int32_t *ids,
                              double t0, double dur, double amp, double period, int32_t count);

std::string prep_instance(const InstSpec &spec, Inst &out, ep_status &st);
// Device bytes upload_instance will allocate for a prepared instance.
size_t instance_footprint(const Inst &inst, int rs, const InstSpec &spec);
// Allocate and upload a prepared instance.
std::string upload_instance(const InstSpec &spec, int rs, const Allocator &al, Inst &out,
                            ep_status &st);
// prep_instance + upload_instance; returns "" or the reason (st set).
std::string build_instance(const InstSpec &spec, int rs, const Allocator &al, Inst &out,
                           ep_status &st);
void free_instance(Inst &inst);
// Exact device bytes build_instance would allocate for a mesh of this size
// and precision (used for admission by footprint).
size_t estimate_footprint(int64_t n_tets, int64_t n_nodes, int rs, int max_degree_hint = 32);

// A set of instances stepped together on one stream.
struct Stepper {
    hipStream_t stream = nullptr;
    // the graph substeps of a step run on a second stream, beside the
    // tissue kernels of the same step (neither reads what the other writes);
    // the junction events wait for both
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int device = 0;
    int rs = 8;
    int grid_node = 0;                 // one block per tile (set when launching)
    // cell tiles are listed class by class; one cell-kernel launch per class
    // present, specialised to that class's cell model
    int64_t cls_tiles[4] = {0, 0, 0, 0}, cls_base[4] = {0, 0, 0, 0};
    // tiles of the 2D media with substeps (after the others in the tables):
    // cell tiles class by class, node tiles; sub2_max substep launches per
    // step, on the side stream
    int64_t cls2_tiles[4] = {0, 0, 0, 0}, cls2_base[4] = {0, 0, 0, 0};
    int64_t nt2_base = 0, n_nt2 = 0;
    int32_t sub2_max = 0;
    int remap = 1;
    int steps_per_graph = 50;
    // cell tile shape: tiles of cell_threads cells (64, 128 or 256), one
    // per lane of a block; node tiles are always TILE nodes
    int32_t cell_threads = 256;
    std::vector<Inst *> insts;
    // device tables
    epdev::InstDesc *d_desc = nullptr;
    epdev::Tile *d_ctiles = nullptr, *d_ntiles = nullptr;
    epdev::PTile *d_ptiles = nullptr;
    epdev::PurkDesc *d_purk = nullptr;
    int32_t *d_counts = nullptr;
    size_t cap_inst = 0, cap_ct = 0, cap_nt = 0, cap_pt = 0, cap_pk = 0;
    int64_t n_ct = 0, n_nt = 0, n_pt = 0, n_pk = 0;
    int32_t n_sub_max = 0;             // graph substeps per step (max over instances)
    bool bido = false;                 // the (single) instance is a bidomain one
    int scheme = 0;                    // time scheme of the instances (all the same)
    // pinned staging of the tables
    void *h_stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t stage_done = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_k = 0, graph_gn = -1, graph_remap = -1;
    int64_t graph_cls[4] = {-1, -1, -1, -1};
    int64_t graph_cls2[4] = {-1, -1, -1, -1};
    int64_t graph_nt2 = -1;
    int32_t graph_sub2 = -1;
    int32_t graph_threads = -1;
    int64_t graph_pt = -1, graph_pk = -1;
    int32_t graph_nsub = -1;
    bool dirty = true;
};

std::string stepper_init(Stepper &s, int device, hipStream_t stream, int rs);
void stepper_free(Stepper &s);
// Rebuild and upload the tables from s.insts (call after membership changes).
std::string stepper_sync_tables(Stepper &s);
// Enqueue k steps of every live instance (graphs for whole multiples of the
// graph length, direct launches for the rest).  Updates host_step.
std::string stepper_run(Stepper &s, int64_t k);
// n steps by direct launches, those of steps 0, every, 2 every, ... timed
// with events (ms): the average node gather and cell kernel durations over
// the timed steps, and (step_ms non-null, ceil(n / every) entries) each
// timed step's device time from its first launch to the end of its last.
std::string stepper_profile(Stepper &s, int64_t n, int64_t every, double &cell_ms,
                            double &node_ms, double *step_ms = nullptr);

// Launch-schedule autotuner.  Every candidate (steps per graph launch x XCD
// tile remap, then the cell tile sizes at the best of those) runs one
// untimed launch (graph capture, warm caches) and then `trial_steps` timed
// steps of the live instances; the fastest per step is kept in the stepper.
// Results do not depend on the schedule, so the trial steps are ordinary
// steps of the simulations.
struct TuneResult {
    int32_t steps_per_graph = 50, xcd_remap = 1;
    int32_t cell_threads = 256;
    double ms_per_step = 0;
    int32_t n_trials = 0;
    int64_t steps_used = 0;
};
std::string stepper_autotune(Stepper &s, int64_t trial_steps, TuneResult &out,
                             bool allow_direct = true);

// Doubles of the device GMRES state for restart length m.
inline size_t gmres_state_doubles(int m) {
    return 8 + (size_t)(m + 1) * m + 2 * (size_t)m + (m + 1) + m + (m + 1);
}

// Bidomain: solve the extracellular equation for the instance's current
// v^{n} (after a step), from its phi_e, enqueued on `stream` after the step:
// captured chunks of four Arnoldi steps, the host waiting for the stream
// once per chunk and once per restart cycle to read the stop flag.
std::string bidomain_solve(Inst &I, hipStream_t stream);
constexpr int kBidoBlocks = 1024;      // blocks of the reduction kernels
constexpr int kBidoMaxRestart = 64;    // longest GMRES restart (its state is staged in LDS)
// partial sums per dot-product row of the bidomain solve: one per block of
// 256 cells, at least kBidoBlocks
inline size_t bido_part_cols(int64_t nc) { return std::max<size_t>(kBidoBlocks, (size_t)((nc + 255) / 256)); }

int model_ng(int m);
int model_nc(int m);
void model_init(int m, double *y);

// The diffusion operator alone (diffusion.hip).  v and L are device arrays
// of nc doubles in caller order; ws is a device workspace of
// diffusion_workspace_bytes(I) bytes (internal-order potentials from offset
// 0, node values from diffusion_workspace_split).  Enqueued on `st`.
size_t diffusion_workspace_split(int64_t nc, size_t rs);
size_t diffusion_workspace_bytes(const Inst &I);
std::string diffusion_apply(const Inst &I, hipStream_t st, const double *v, double *L, void *ws);
// Once per device, with that device current: the device address of the
// library's fixed workspace.
std::string diffusion_scratch_setup(int device);
// diffusion_apply on the fixed workspace of `device`; fails if the operator
// needs more than EP_DIFFUSION_SCRATCH_MAX bytes.  Allocates nothing.  On
// failure `code` is the status to report.
std::string diffusion_apply_noalloc(const Inst &I, int device, hipStream_t st, const double *v,
                                    double *L, ep_status &code);

}  // namespace ep
