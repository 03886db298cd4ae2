/* ep.h -- C ABI of the MI355X monodomain library (libep.so).
 *
 * One explicit monodomain time step of Del Corso, Verzicco & Viola, "A fast
 * computational model for the electrophysiology of the whole human heart":
 *   - cell-centred finite volumes on tetrahedra (Sec. 3.2, eqs. electro5 and
 *     electro2_3dmono): node values by inverse-distance weighting of the
 *     surrounding cell values, face values as the mean of the three node
 *     values, Gauss-Green cell gradients, face gradients interpolated
 *     between the two cells and corrected along the centre-to-centre
 *     direction (eq. gra2bis), flux A_f (M_f grad v_f).n_f, no-flux outer
 *     boundary;
 *   - the fibre conductivity tensor M = A diag(m_l, m_t, m_t) A^T (Sec. 3.1,
 *     eq. tensor), optionally scaled per cell;
 *   - cell models (Sec. 3.1-3.2): ten Tusscher-Panfilov (endo/mid/epi),
 *     Courtemanche, Stewart; Rush-Larsen for gating variables, forward
 *     Euler for the other states and for v, every right-hand side at t^n;
 *   - the stimulus of eq. stimulus (amplitude, onset, duration, optional
 *     period and count) on a set of cells, as a whole-step window;
 *   - activation time = first upward crossing of at_threshold (0 mV, Sec. 4),
 *     linearly interpolated within the step; APD90 = time from activation
 *     to the downward crossing of v_max - repol_frac (v_max - v_rest);
 *   - the volume-averaged potential vbar(t) = int v dV / V (Sec. 4).
 *
 * Units: mm, ms, mV, mS/mm, 1/mm, uF/mm^2, pA/pF (= mV/ms).
 * Indices are 0-based in the caller's numbering; the library reorders
 * internally and every readout is returned in the caller's numbering.
 *
 * Ownership: every input array is owned by the caller, copied during the
 * call and never retained.  Output arrays are allocated by the caller, their
 * length is passed and checked.  Host pointers unless stated otherwise.
 *
 * Errors: every call returns an ep_status; on failure the object is left in
 * its previous valid state and ep_last_error() describes the failure.  Calls
 * that need an initialised simulation return EP_ESTATE before ep_init().  A
 * non-finite membrane potential surfaces as EP_ENUMERIC at the next ep_sync()
 * or readout.  Nothing throws across this interface.  A simulation object is
 * not thread-safe; distinct objects are independent.
 *
 * Device work runs on the stream given in ep_options (or on a stream the
 * library creates); ep_step() only enqueues.  There is no CPU fallback: if no
 * HIP device is usable, ep_create() fails with EP_EDEVICE.
 */
#ifndef EP_H
#define EP_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EP_OK = 0,
    EP_EINVAL = -1,   /* bad argument (null pointer, size, range, degenerate mesh) */
    EP_ENOMEM = -2,   /* device or host allocation failed / over budget       */
    EP_EDEVICE = -3,  /* HIP runtime error                                     */
    EP_ESTATE = -4,   /* call not valid in the current state                   */
    EP_ENUMERIC = -5, /* non-finite membrane potential detected                */
    EP_EBUSY = -6     /* (server) request still running                        */
} ep_status;

typedef enum { EP_FP64 = 0, EP_FP32_MIXED = 1 } ep_precision;

/* Cell models.  EP_PASSIVE has I_ion = 0 (diffusion only, for tests). */
typedef enum {
    EP_TP06_ENDO = 0, EP_TP06_MID = 1, EP_TP06_EPI = 2,
    EP_CRN = 3, EP_STEWART = 4, EP_PASSIVE = 5
} ep_model;

#define EP_MAX_SLOTS 21     /* state slots per cell in ep_get_states()        */
#define EP_MAX_STIMULI 32   /* stimuli per simulation                         */

typedef struct {
    ep_precision prec;  /* EP_FP64 or EP_FP32_MIXED (FP32 gates/currents/flux,
                           FP64 Na/K/Ca concentrations and buffering)         */
    int device;         /* HIP device ordinal                                  */
    void *stream;       /* hipStream_t to run on, or NULL for a library stream */
    double dt;          /* time step, ms                                       */
    double chi;         /* surface-to-volume ratio, 1/mm (paper: 140)          */
    double cm;          /* membrane capacitance, uF/mm^2 (paper: 0.01)         */
    double at_threshold;/* activation threshold, mV (paper: 0)                 */
    double repol_frac;  /* APD repolarisation fraction (0.9 = APD90)           */
    int32_t trace_every;/* record vbar every this many steps (0 = never)       */
    /* optional device allocator (e.g. a framework's caching allocator);
       both NULL = hipMalloc/hipFree */
    void *(*dev_alloc)(size_t bytes, void *ctx);
    void (*dev_free)(void *ptr, void *ctx);
    void *alloc_ctx;
} ep_options;

typedef struct ep_sim ep_sim;

/* Fill *o with the paper's parameters (chi 140, cm 0.01, dt 0.02, 0 mV,
 * 0.9, FP64, device 0, library stream, trace every 50 steps). */
void ep_default_options(ep_options *o);

/* Create an empty simulation bound to o->device.  EP_EDEVICE if HIP has no
 * usable device. */
ep_status ep_create(const ep_options *o, ep_sim **out);
void ep_destroy(ep_sim *s);                 /* frees host and device memory */

/* Mesh: n_nodes coordinates xyz[3*i+k] (mm) and n_tets cells
 * tet_nodes[4*c+k] (node ids, any orientation).  A cell is a tetrahedron of
 * the 3D myocardium, or, when tet_nodes[4*c+3] == -1, a triangle of a 2D
 * medium (the paper's Purkinje shell, Sec. 3.2), discretised by the same
 * cell-centred scheme on its edges: the area takes the volume's place, edge
 * values are the means of their two node values, and across an edge between
 * two triangles that are not coplanar the flux uses the edge length times the
 * unit bisector of the two in-plane outward normals (conservative).  The 2D
 * medium behaves as a sheet of unit thickness: its fluxes are sigma (mS/mm)
 * times gradients times edge lengths.  A node belongs to tetrahedra or to
 * triangles, not both; triangles do not couple to tetrahedra except through
 * junctions.  Every "tet" argument and count of this interface means a cell
 * of either kind, in this order.  EP_EINVAL on an index out of range, a
 * degenerate cell, a node shared by both kinds, or triangles in a bidomain
 * simulation. */
ep_status ep_set_mesh(ep_sim *s, int64_t n_nodes, const double *xyz,
                      int64_t n_tets, const int32_t *tet_nodes);

/* Conductivity (Sec. 3.1): per-tet unit fibre vectors fibre[3*c+k],
 * longitudinal / transverse conductivities (mS/mm), optional per-tet scale
 * (NULL = 1).  M_c = scale_c (sigma_t I + (sigma_l - sigma_t) f f^T). */
ep_status ep_set_conductivity(ep_sim *s, const double *fibre, double sigma_l,
                              double sigma_t, const double *scale);

/* Cell model of every tet (ep_model values); default EP_TP06_ENDO. */
ep_status ep_set_models(ep_sim *s, const uint8_t *model);

/* Multiply a maximal conductance of every cell model by s (> 0):
 * param = "GKr", "GKs", "GCaL" or "GNa". */
ep_status ep_set_ionic_scale(ep_sim *s, const char *param, double scale);

/* Stimulus (eq. stimulus) on n_ids tets: amp pA/pF (negative depolarises)
 * from t0 for dur ms, on whole steps [round(t0/dt), round(t0/dt) +
 * round(dur/dt)); repeated every period ms count times if period > 0.
 * domain 0: ids are tets; domain 1: ids are Purkinje graph nodes (the window
 * covers every graph substep of those tissue steps).  At most
 * EP_MAX_STIMULI over both domains. */
ep_status ep_add_stimulus(ep_sim *s, int domain, int64_t n_ids,
                          const int32_t *ids, double t0, double dur,
                          double amp, double period, int32_t count);

/* Purkinje network (Sec. 2.2, 3.2; a 1D graph in place of the paper's 2D
 * surface): n nodes xyz[3*i+k], n_edges segments edges[2*e], conductivity
 * sigma (mS/mm; the paper's Purkinje value is 3.95), cell model (normally
 * EP_STEWART).  Vertex-centred finite volumes: node i owns half of each
 * incident segment, l_i = sum_j L_ij / 2, and
 *   dv_i/dt = sigma / (chi Cm l_i) sum_j (v_j - v_i) / L_ij - I_ion - I_stim.
 * The graph advances in n_sub explicit substeps per tissue step (n_sub <= 0:
 * the smallest n_sub with dt / n_sub <= 0.9 min_i chi Cm l_i / (sigma
 * sum_j 1/L_ij), a sufficient stability bound).  Stimuli on the graph use
 * ep_add_stimulus with domain 1 and node ids.  Call before ep_init. */
ep_status ep_set_purkinje(ep_sim *s, int64_t n, const double *xyz, int64_t n_edges,
                          const int32_t *edges, double sigma, int32_t model,
                          int32_t n_sub);

/* Conductivity multiplier s_e >= 0 per graph segment (n_edges == the count
 * given to ep_set_purkinje, same order; caller-owned, copied): segment e
 * conducts with sigma * s_e, so the flux term above reads
 * sum_j s_ij (v_j - v_i) / L_ij while l_i is unchanged.  The paper models a
 * bundle-branch delay by lowering the bundles' conductivity in proportion to
 * its severity and a complete block by a null conductivity (Sec. 6); the
 * substep bound then uses sigma sum_j s_ij / L_ij (nodes whose segments are
 * all blocked impose none).  ep_set_purkinje resets every s_e to 1.
 * EP_EINVAL for a count mismatch or a negative or non-finite value.  Call
 * before ep_init. */
ep_status ep_set_purkinje_scale(ep_sim *s, int64_t n_edges, const double *scale);

/* Purkinje-muscle junction at graph node `node` (Sec. 3.3): when the node's
 * potential crosses at_threshold upward during tissue step n, the tissue
 * cells whose centroid lies within `radius` of the node (if none: the cells
 * sharing a mesh node with the cell of nearest centroid) receive amp pA/pF
 * for dur ms from step n + 1 + round(delay_ortho/dt).  With two_way, an
 * upward crossing of the mean potential of that region stimulates the node
 * from step n + 1 + round(delay_anti/dt) (antidromic conduction).  Each step
 * runs the tissue, then the graph substeps, then these events.  Call before
 * ep_init. */
ep_status ep_add_pmj(ep_sim *s, int32_t node, double radius, double delay_ortho,
                     double delay_anti, int32_t two_way, double amp, double dur);

/* Communication node whose source is a cell (Sec. 3.3: the 2D Purkinje
 * shell excites the 3D myocardium through such nodes, about 1 mm apart,
 * with a 0.1 mm range and the 5 ms junction delay): when cell `cell`
 * crosses at_threshold upward during step n, the cells of the other kind
 * (tets for a triangle, triangles for a tet) whose centroid lies within
 * `radius` of its centroid (if none: those sharing a mesh node with the
 * nearest one) receive amp for dur ms from step n + 1 + round(delay_ortho/dt);
 * with two_way the upward crossing of that region's mean pulses the source
 * cell from step n + 1 + round(delay_anti/dt).  Shares one index sequence
 * with ep_add_pmj (call order); needs no graph.  EP_EINVAL for a cell out of
 * range, bad parameters, or (at ep_init) no cell of the other kind.  Call
 * after ep_set_mesh and before ep_init. */
ep_status ep_add_cell_junction(ep_sim *s, int32_t cell, double radius, double delay_ortho,
                               double delay_anti, int32_t two_way, double amp, double dur);

/* Graph readouts (caller numbering of graph nodes, n == graph size):
 * potential and activation time (first upward threshold crossing, NaN if
 * none); and the substep count in use. */
ep_status ep_get_purkinje_vm(ep_sim *s, double *out, int64_t n);
ep_status ep_get_purkinje_activation(ep_sim *s, double *out, int64_t n);
ep_status ep_get_purkinje_substeps(ep_sim *s, int32_t *n_sub);

/* Time scheme of the non-gating states: the potential v of cells and graph
 * nodes, the concentrations and Stewart's Rbar.  EP_SCHEME_FE: forward
 * Euler, the paper's scheme (Sec. 3.2).  EP_SCHEME_AB2: the second-order
 * Adams-Bashforth step the paper names for a smaller time error (Sec. 4),
 *   y^{n+1} = y^n + dt (3/2 f^n - 1/2 f^{n-1}),
 * forward Euler on step 0 (graph: substep 0); the gates stay Rush-Larsen, so
 * the scheme as a whole stays first order.  EP_SCHEME_RL2_AB2: also the
 * second-order Rush-Larsen step the paper names for second order overall:
 * each gate's steady state and time constant are taken at the midpoint
 * predictions v^n + dt/2 f_v^n and c^n + dt/2 f_c^n of the potential and of
 * the calcium concentrations it depends on (CRN's release gates u, v keep
 * their level-n driver).  AB2 keeps one previous rate per
 * non-gating state (device memory, part of the checkpoint) and is stable on
 * half the interval of forward Euler: a derived graph substep count uses
 * half the bound, and dt itself must suit.  Not with the bidomain model
 * (EP_EINVAL).  Call before ep_init. */
typedef enum { EP_SCHEME_FE = 0, EP_SCHEME_AB2 = 1, EP_SCHEME_RL2_AB2 = 2 } ep_time_scheme;
ep_status ep_set_time_scheme(ep_sim *s, int32_t scheme);

/* Internal numbering of the cells, which is their order in device memory:
 * reverse Cuthill-McKee from a peripheral cell (the default), Morton order of
 * the centroids, or the caller's order; cells stay grouped by model class.
 * Results and readouts (always in the caller's order) are the same up to the
 * order of rounding; the memory traffic is not: with EP_ORDER_INPUT on an
 * unordered mesh the node and neighbour ids of a 256-cell block usually span
 * more than 16 bits, and the cell kernel then reads 32-bit ids
 * (ep_algorithmic_bytes shows which).  Call before ep_init; EP_EINVAL for an
 * unknown order. */
typedef enum { EP_ORDER_RCM = 0, EP_ORDER_MORTON = 1, EP_ORDER_INPUT = 2 } ep_cell_order;
ep_status ep_set_cell_order(ep_sim *s, int32_t order);

/* The 2D medium (the triangles, e.g. the Purkinje shell) at a time step of
 * its own, as the paper integrates its Purkinje networks at a step far
 * below the myocardium's (Sec. 4): each step of dt, its cells take n_sub
 * explicit substeps of dt / n_sub, each the whole monodomain update of the
 * medium (node values, face fluxes, cell model, v, activation / APD90
 * interpolated inside the substep); stimuli and junction pulses of the step
 * hold through its substeps, junction events see the medium's v^n and
 * v^{n+1}.  n_sub = 1: the medium steps with the rest (the default);
 * n_sub > 1: given; n_sub <= 0: the smallest count within 90 % (45 % with
 * Adams-Bashforth 2) of the medium's forward-Euler bound 1 / max_c r_c,
 * r_c = sum over its edges of sigma_max scale_c |S_f| / (d_f chi Cm V_c)
 * (sigma_max the larger conductivity, |S_f| the edge length, d_f the
 * distance of the triangle centroids).  The tets always step at dt.  Before
 * ep_init; set the time scheme first.  EP_EINVAL with the bidomain model
 * (at ep_init) or above 2^20 substeps.  The medium's cells take the last
 * internal indices (their own tiles, stepped beside the tets on a second
 * stream). */
ep_status ep_set_medium_substeps(ep_sim *s, int32_t n_sub);
/* Substeps per step of the 2D medium after ep_init (1: none). */
ep_status ep_get_medium_substeps(ep_sim *s, int32_t *n_sub);

/* Bidomain model (Sec. 3.1 eq. electro, Sec. 3.2 eq. electro2_3d) instead of
 * the monodomain one: the conductivities of ep_set_conductivity become the
 * intracellular ones M_i; sigma_el / sigma_et (mS/mm) give the extracellular
 * M_e with the same fibres and scale (the paper's ventricular values are
 * 0.62 / 0.24).  Each step advances v with the intracellular flux of
 * v + phi_e at level n, then solves
 *   sum_f A_f ((M_i + M_e) grad phi_e).n = -sum_f A_f (M_i grad v^{n+1}).n
 * for phi_e^{n+1} by restarted GMRES(restart) started from phi_e^n, until the
 * residual is at most tol times the right-hand side's norm or max_iter Arnoldi
 * steps, and shifts phi_e to zero volume-weighted mean (phi_e^0 = 0, exact for
 * a uniform initial potential).  1 <= restart <= 64, EP_FP64 and forward Euler
 * only (EP_EINVAL otherwise); call before ep_init.  The solve runs on the
 * device; each ep_step of a bidomain simulation waits for its stream once per
 * four Arnoldi steps and once per restart cycle, to read the solver's stop
 * flag. */
ep_status ep_set_bidomain(ep_sim *s, double sigma_el, double sigma_et, int32_t restart,
                          double tol, int32_t max_iter);
/* phi_e in caller numbering (n == n_tets) */
ep_status ep_get_phi_e(ep_sim *s, double *out, int64_t n);
/* Arnoldi steps of the last solve, their total, the last relative residual */
ep_status ep_get_bidomain_stats(ep_sim *s, int64_t *last_iters, int64_t *total_iters,
                                double *last_relres);

/* Precompute geometry and flux coefficients (FP64, host), reorder the mesh,
 * upload to the device and set the standard initial state of every model.
 * After this the mesh, conductivity and models are frozen. */
ep_status ep_init(ep_sim *s);

/* Device bytes the initialised simulation holds. */
ep_status ep_footprint(const ep_sim *s, size_t *bytes);

/* Enqueue n time steps (n >= 0) on the simulation's stream; returns at once. */
ep_status ep_step(ep_sim *s, int64_t n);

/* Wait for queued work; EP_ENUMERIC if a non-finite v appeared. */
ep_status ep_sync(ep_sim *s);

/* Readouts (synchronise first), caller numbering, length n == n_tets. */
ep_status ep_get_vm(ep_sim *s, double *out, int64_t n);
ep_status ep_get_activation(ep_sim *s, double *t_act, int64_t n); /* NaN = never */
ep_status ep_get_apd90(ep_sim *s, double *apd, int64_t n);        /* NaN = undefined */

/* The vbar(t) samples recorded so far (every trace_every steps, starting
 * with step 0): up to cap pairs (t ms, vbar mV); *n_out = number written. */
ep_status ep_get_mean_vm_trace(ep_sim *s, double *t, double *vbar,
                               int64_t cap, int64_t *n_out);

/* Current step index and time t = step * dt. */
ep_status ep_get_time(ep_sim *s, int64_t *step, double *t);

/* The diffusion operator alone (Sec. 3.2: node values by inverse-distance
 * weights, cell gradients, the face gradient of eq. gra2bis, the sum of the
 * face fluxes): L_c = (1 / (chi Cm V_c)) sum_f A_f (M_f g_f) . n_f in mV/ms
 * for the potential v, with this simulation's mesh, fibres, conductivities
 * and precision (FP32 in the mixed precision) - the L that ep_step adds to
 * v^n = v.  v and L are DEVICE arrays on the simulation's device, n ==
 * n_tets doubles each in caller order; L may not alias v; both stay the
 * caller's.  The simulation's state is not touched.  The library allocates
 * a workspace of 8 (FP64) or 4 (mixed) bytes per cell and per node (through
 * dev_alloc when set), runs on the simulation's stream, waits for it and
 * frees the workspace before returning.  EP_ESTATE before ep_init,
 * EP_EINVAL for a wrong n, null or aliased arrays, EP_ENOMEM when the
 * workspace cannot be allocated. */
ep_status ep_apply_diffusion(ep_sim *s, const double *v, double *L, int64_t n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ep_apply_diffusion with its workspace in a fixed device buffer of
 * EP_DIFFUSION_SCRATCH_MAX bytes that the library holds on every GPU it
 * runs on until the process ends (its address is taken at ep_init).  Same
 * arguments and result; allocates nothing, host or device, and does not
 * wait: the kernels are enqueued on the simulation's stream and L is ready
 * once that stream is synchronised.  Every call on one GPU shares that
 * GPU's buffer (nothing in it needs to start at zero; it keeps the last
 * call's contents), so calls whose kernels overlap on one GPU - from other
 * streams or simulations - race and must be ordered by the caller.
 * EP_EINVAL when the workspace (8 (FP64) or 4 (mixed) bytes per cell and per
 * node, the cell part rounded up to 256 bytes) exceeds the buffer, with the
 * other errors of ep_apply_diffusion. */
#define EP_DIFFUSION_SCRATCH_MAX (64u << 20)
ep_status ep_apply_diffusion_noalloc(ep_sim *s, const double *v, double *L, int64_t n);

/* Per-cell states as FP64, layout out[slot * n + cell] with n == n_tets,
 * n_slots == EP_MAX_SLOTS.  Slot 0 is V; the model's states follow in the
 * order of ep_model_slot_name(); unused slots read NaN and are ignored on
 * write.  In EP_FP32_MIXED the FP32 slots are rounded on write.  States set
 * before the first step also become the resting potential of the APD90
 * detection; with an Adams-Bashforth scheme the stored previous rates are
 * not recomputed, so set states before the first step (or restore a
 * checkpoint) for a clean second-order start.  Graph nodes keep theirs. */
ep_status ep_get_states(ep_sim *s, double *out, int64_t n, int32_t n_slots);
ep_status ep_set_states(ep_sim *s, const double *in, int64_t n, int32_t n_slots);
int ep_model_n_slots(int model);                         /* incl. V, 0 if bad */
const char *ep_model_slot_name(int model, int slot);     /* NULL if bad       */

/* Checkpoint: an opaque byte image of every state array, the detection
 * state, the step counter and the trace.  Restoring it into a simulation
 * built from the same inputs continues bitwise identically.  The image holds
 * the device layout, tagged by a version in its header: ep_set_state returns
 * EP_EINVAL for an image of another layout version, mesh size, precision,
 * time scheme, model configuration or cell order (the header carries the
 * EP_ORDER_* value and a hash of the internal permutation and of each
 * cell's model, since the per-cell arrays are stored in internal order). */
ep_status ep_state_size(ep_sim *s, size_t *bytes);
ep_status ep_get_state(ep_sim *s, void *buf, size_t bytes);
ep_status ep_set_state(ep_sim *s, const void *buf, size_t bytes);

/* Launch controls used by the autotuner: block is the cells (= lanes) of a
 * cell-kernel tile, 64, 128 or 256 (0 keeps the current; node tiles are
 * always 256 nodes), steps_per_graph is the number of steps captured per HIP graph
 * launch (0 = direct launches only), xcd_remap remaps blocks to tiles: 0
 * none (the hardware deals consecutive blocks to the 8 XCDs in turn), 1 each
 * XCD one contiguous range of tiles, 2 each XCD every eighth of 32 chunks of
 * contiguous tiles, 3 none for the cell kernels and the chunks of 2 for
 * the node gather (EP_EINVAL otherwise).  May be called any time after
 * ep_create(). */
ep_status ep_set_launch(ep_sim *s, int32_t block, int32_t steps_per_graph,
                        int32_t xcd_remap);

/* Cell tile size (batched scheduling, not the paper's): a cell-kernel block
 * takes a tile of 64, 128 or 256 consecutive cells of one model class, one
 * per lane.  No result depends on it: every cell's arithmetic is its own,
 * and the vbar trace is summed from partials of 64 cells in a fixed order.
 * EP_EINVAL for other sizes. */
ep_status ep_set_tile_size(ep_sim *s, int32_t cells);
/* The schedule in effect (after ep_autotune: the one it chose); any output
 * pointer may be NULL. */
ep_status ep_get_launch(ep_sim *s, int32_t *tile_cells, int32_t *steps_per_graph,
                        int32_t *xcd_remap);

/* Launch-schedule autotuner (batched scheduling is this library's, not the
 * paper's).  Tries every graph length in {0 (direct launches), 10, 25, 50,
 * 100} steps, each with the XCD tile remaps 0 to 3, then at the fastest
 * of those the cell tile sizes 256, 128 and 64: each candidate one untimed
 * launch (graph capture, warm caches), then trial_steps steps, rounded up to
 * whole graphs, timed with HIP events on the simulation's stream.  Keeps the
 * fastest schedule and tile size (as ep_set_launch / ep_set_tile_size would;
 * ep_get_launch reads them) and reports the schedule; any output pointer may
 * be NULL.  The trials are ordinary steps, with the same results as under
 * any fixed schedule: the simulation advances by 744 steps plus four times
 * the sum over the five graph lengths of their timed steps, plus three times
 * the chosen length's untimed and timed steps.  EP_ESTATE before ep_init, EP_EINVAL for
 * trial_steps <= 0. */
ep_status ep_autotune(ep_sim *s, int64_t trial_steps, int32_t *steps_per_graph,
                      int32_t *xcd_remap, double *ms_per_step);

/* Runs n steps by direct launches on the simulation's stream.  The
 * kernels of steps 0, every, 2 every, ... (the timed steps; every = 1 times
 * them all) carry HIP events that their launch sets from the dispatch's own
 * start and end (no marker between kernels); the other steps are launched
 * plainly.  The host waits only for the timed step 64 places back (the
 * kernels run back to back, as without the events).  Reports the average
 * device duration (ms) over the timed steps of the fused cell kernel(s) and
 * of the node gather kernel and, when step_ms is not NULL, each timed
 * step's device time from the start of its first kernel to the end of its
 * last (step_ms holds ceil(n / every) doubles, caller-owned).  The steps
 * are ordinary steps of the simulation.  Any output pointer may be NULL.
 * EP_EINVAL for n <= 0 or every <= 0, EP_ESTATE before ep_init. */
ep_status ep_profile_steps(ep_sim *s, int64_t n, int32_t every, double *cell_ms,
                           double *node_ms, double *step_ms);

/* Algorithmic bytes moved per step by the node gather and by the cell
 * kernel, and by one ep_apply_diffusion call, for this mesh, precision,
 * time scheme and stencil-id width (16-bit offsets from per-block bases
 * when every 256-cell block allows them, else 32-bit ids): the roofline
 * numerators.  Any output pointer may be NULL.  EP_ESTATE before ep_init. */
ep_status ep_algorithmic_bytes(const ep_sim *s, double *node_bytes,
                               double *cell_bytes, double *diffusion_bytes);

const char *ep_last_error(const ep_sim *s);

/* ------------------------------------------------------------- serving
 * A single-GPU server for the parametric and uncertainty-quantification
 * sweeps the paper motivates (Sec. 6): independent simulations arrive as
 * requests, are precomputed on host worker threads, admitted while their
 * device footprint fits the HBM budget and a slot is free (first come first
 * served; a request that does not fit lets smaller later ones pass), and
 * stepped together in batched kernels replayed as HIP graphs.  Requests
 * that arrive while others run join at the next graph boundary (continuous
 * batching).  Each result is bitwise the one the same request gives alone.
 * All server calls are thread-safe. */

typedef struct {
    int64_t n_ids;        /* tets (domain 0) or graph nodes (domain 1) of the
                             stimulus region, caller numbering              */
    const int32_t *ids;
    double t0, dur, amp;  /* ms, ms, pA/pF                                   */
    double period;        /* 0 = single pulse                               */
    int32_t count;
    int32_t domain;       /* 0 tissue, 1 Purkinje graph (as ep_add_stimulus) */
} ep_stimulus;

/* A Purkinje-muscle junction of a request (as ep_add_pmj). */
typedef struct {
    int32_t node;
    int32_t two_way;
    double radius, delay_ortho, delay_anti, amp, dur;
} ep_pmj;

/* A junction whose source is a cell, in a request (as ep_add_cell_junction). */
typedef struct {
    int32_t cell;
    int32_t two_way;
    double radius, delay_ortho, delay_anti, amp, dur;
} ep_cell_junction;

/* The Purkinje graph of a request (as ep_set_purkinje, ep_set_purkinje_scale
 * and ep_add_pmj; every array caller-owned and copied at submission). */
typedef struct {
    int64_t n;
    const double *xyz;            /* [3*n]                                   */
    int64_t n_edges;
    const int32_t *edges;         /* [2*n_edges]                             */
    const double *edge_scale;     /* [n_edges] or NULL (all 1)               */
    double sigma;                 /* mS/mm                                   */
    int32_t model;                /* ep_model, normally EP_STEWART           */
    int32_t n_sub;                /* <= 0: from the stability bound          */
    int32_t n_pmj;
    const ep_pmj *pmj;
} ep_purkinje;

typedef struct {
    int64_t n_nodes;
    const double *xyz;            /* [3*n_nodes]                             */
    int64_t n_tets;
    const int32_t *tet_nodes;     /* [4*n_tets]                              */
    const double *fibre;          /* [3*n_tets] unit vectors                 */
    double sigma_l, sigma_t;      /* mS/mm                                   */
    const double *scale;          /* [n_tets] or NULL                        */
    const uint8_t *model;         /* [n_tets] ep_model, NULL = TP06 endo     */
    int32_t n_stimuli;            /* <= EP_MAX_STIMULI                       */
    const ep_stimulus *stimuli;
    double ionic_scale[4];        /* GKr, GKs, GCaL, GNa multipliers (0 = 1) */
    int64_t n_steps;              /* steps to run (> 0)                      */
    const ep_purkinje *purkinje;  /* NULL: tissue only                       */
    int32_t n_cell_junctions;     /* junctions with a source cell, after the
                                     graph's (as ep_add_cell_junction)       */
    const ep_cell_junction *cell_junctions;
    int32_t medium_substeps;      /* the 2D medium's substeps per step (as
                                     ep_set_medium_substeps): 0 or 1 none,
                                     > 1 given, < 0 from its bound           */
} ep_request;

typedef struct {
    int64_t id;
    ep_status status;             /* EP_OK, EP_ENUMERIC (non-finite v), or an
                                     admission / device error                */
    int64_t n_tets, steps;
    size_t footprint;             /* device bytes while resident             */
    double t_submit, t_admit, t_done;   /* seconds since server creation     */
    double t_ready;               /* host precompute finished (0 if it failed):
                                     t_ready - t_submit is the precompute,
                                     t_admit - t_ready the wait for memory or
                                     a slot, t_done - t_admit the device run */
} ep_result;

typedef struct {
    int64_t submitted, completed, running, queued;
    double cell_steps;            /* tet-steps issued so far (finished
                                     requests and the progress of running ones) */
    size_t bytes_in_use, bytes_budget;
    int64_t graph_launches, table_updates;
    int32_t steps_per_graph, xcd_remap;   /* schedule in effect              */
    int64_t autotune_runs;
    double tuned_ms_per_step;     /* batch step time of the last tuning      */
    int32_t tile_cells;           /* cell tile size in effect (64/128/256)   */
    int32_t pad;
} ep_server_stats;

typedef struct ep_server ep_server;

/* o->prec, device, dt, chi, cm, thresholds and allocator apply to every
 * request.  hbm_budget: device bytes for resident requests (0 = 90 % of the
 * free device memory); max_slots: resident requests at most (> 0). */
ep_status ep_server_create(const ep_options *o, size_t hbm_budget, int32_t max_slots,
                           ep_server **out);
/* Copies the request; returns its id.  EP_EINVAL for malformed requests and
 * EP_ENOMEM if it could never fit the budget. */
ep_status ep_server_submit(ep_server *sv, const ep_request *rq, int64_t *id);
/* EP_EBUSY while queued or running, else fills *res (EP_EINVAL: unknown id). */
ep_status ep_server_poll(ep_server *sv, int64_t id, ep_result *res);
ep_status ep_server_wait(ep_server *sv, int64_t id, ep_result *res);
/* Results of a finished request, caller numbering, n == its n_tets. */
ep_status ep_server_get_vm(ep_server *sv, int64_t id, double *out, int64_t n);
ep_status ep_server_get_activation(ep_server *sv, int64_t id, double *out, int64_t n);
ep_status ep_server_get_apd90(ep_server *sv, int64_t id, double *out, int64_t n);
/* Graph results of a finished request with a Purkinje graph, n == its node
 * count: potential and activation time (NaN: none).  EP_ESTATE without a
 * graph. */
ep_status ep_server_get_purkinje_vm(ep_server *sv, int64_t id, double *out, int64_t n);
ep_status ep_server_get_purkinje_activation(ep_server *sv, int64_t id, double *out, int64_t n);
ep_status ep_server_release(ep_server *sv, int64_t id);   /* drop stored results */
ep_status ep_server_get_stats(ep_server *sv, ep_server_stats *st);
/* Graph length in steps (> 0) and XCD remap, as ep_set_launch. */
ep_status ep_server_set_launch(ep_server *sv, int32_t steps_per_graph, int32_t xcd_remap);
/* Time scheme of every request of the server (as ep_set_time_scheme; one
 * scheme per server because the batched kernels are specialised on it).
 * EP_ESTATE once a request has been submitted. */
ep_status ep_server_set_time_scheme(ep_server *sv, int32_t scheme);
/* hold != 0: keep admitting and uploading requests but step none, so that a
 * batch can start together (a UQ sweep); hold == 0 resumes stepping. */
ep_status ep_server_hold(ep_server *sv, int32_t hold);
/* Autotune the schedule (as ep_autotune, trial_steps per candidate, rounded
 * up to whole graphs) on the batch that is live when the driver next steps;
 * with retune != 0, tune again whenever at least 4 requests are live, their
 * number has doubled or halved since the last tuning, and the batch has
 * advanced at least ten times the steps that tuning took.  The trials are
 * ordinary steps of the live requests. */
ep_status ep_server_autotune(ep_server *sv, int64_t trial_steps, int32_t retune);
void ep_server_destroy(ep_server *sv);    /* waits for running requests */
const char *ep_server_last_error(ep_server *sv);

#ifdef __cplusplus
}
#endif
#endif
