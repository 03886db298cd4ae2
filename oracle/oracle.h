/* CPU FP64 oracle of one explicit monodomain time step on tetrahedra.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, slow, obviously
 * correct reference that the tests, the smoke check and the CPU-baseline leg
 * of the benchmark call to check the HIP library.  Nothing on the product
 * path may link, load or call it.  It shares no code with the HIP library.
 *
 * What it computes (Del Corso, Verzicco, Viola, "A fast computational model
 * for the electrophysiology of the whole human heart"):
 *   - the cell-centred finite-volume monodomain equation on tetrahedra
 *     (Sec. 3.2, eqs. electro5 and electro2_3dmono), with the node values,
 *     face values, Gauss-Green cell gradients, interpolated face gradients
 *     and the stabilised face gradient of eq. gra2bis;
 *   - the transversely isotropic fibre tensor M = A diag(m_l, m_t, m_t) A^T
 *     (Sec. 3.1, eq. tensor);
 *   - forward Euler for v and the non-gating cell states, Rush-Larsen for the
 *     gating variables, all right-hand sides at level n (Sec. 3.2);
 *   - the stimulus of eq. stimulus as an integer step window;
 *   - activation time (first upward crossing of 0 mV, Sec. 4) and APD90.
 * Units: mm, ms, mV, mS/mm, 1/mm, uF/mm^2, pA/pF.  All arithmetic is FP64.
 *
 * State slots (a per-cell exchange format): slot 0 is V; the cell model's
 * states follow in the order listed by orc_model_slot_name().
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_TP06_ENDO = 0, ORC_TP06_MID = 1, ORC_TP06_EPI = 2, ORC_CRN = 3,
       ORC_STEWART = 4, ORC_PASSIVE = 5 };
#define ORC_MAX_SLOTS 21

typedef struct orc_sim orc_sim;

/* ------------------------------------------------------------ cell models */
int         orc_model_n_slots(int model);              /* incl. V          */
const char *orc_model_slot_name(int model, int slot);
void        orc_model_init(int model, double *y);      /* standard state   */
/* One step of a single cell: currents at level n from y, Rush-Larsen gates,
 * forward-Euler concentrations.  y[0] (V) is read, not written.  gscale
 * holds the multipliers of G_Kr, G_Ks, G_CaL, G_Na (NULL = 1).
 * Returns the total ionic current I_ion at level n in pA/pF. */
double orc_model_step(int model, double *y, double dt, double istim,
                      const double *gscale);

/* ------------------------------------------------------------- tissue */
orc_sim *orc_create(int64_t n_nodes, const double *xyz, int64_t n_tets,
                    const int32_t *tets, const double *fibre, double sigma_l,
                    double sigma_t, const double *scale, const uint8_t *model,
                    double dt, double chi, double cm);
void orc_destroy(orc_sim *s);
void orc_set_ionic_scale(orc_sim *s, const double gscale[4]);
int  orc_add_stimulus(orc_sim *s, int64_t n_ids, const int32_t *ids, double t0,
                      double dur, double amp, double period, int32_t count);
void orc_set_detection(orc_sim *s, double threshold, double repol_frac);
void orc_step(orc_sim *s, int64_t n_steps);
int64_t orc_get_step(const orc_sim *s);
void orc_get_vm(const orc_sim *s, double *out);
void orc_get_activation(const orc_sim *s, double *out);   /* NaN = never   */
void orc_get_apd90(const orc_sim *s, double *out);        /* NaN = undef.  */
double orc_mean_vm(const orc_sim *s);                     /* int v dV / V  */
/* states as [ORC_MAX_SLOTS][n_tets]; unused slots are NaN on output */
void orc_get_states(const orc_sim *s, double *out);
void orc_set_states(orc_sim *s, const double *in);
void orc_set_step(orc_sim *s, int64_t step);
void orc_get_detect_state(const orc_sim *s, double *out);
void orc_set_detect_state(orc_sim *s, const double *in);

/* ------------------------------------------------- Purkinje graph, PMJs */
/* A 1D Purkinje graph discretised with vertex-centred finite volumes (the
 * paper's choice for branching 1D media, Sec. 3.2): node i owns half of every
 * incident segment, l_i = sum_j L_ij / 2, and
 *   dv_i/dt = sigma / (chi Cm l_i) sum_j s_ij (v_j - v_i) / L_ij - I_ion - I_stim,
 * with s_ij >= 0 the segment's conductivity multiplier (edge_scale, NULL = 1;
 * a reduced value models a bundle-branch delay, 0 a complete block, Sec. 6).
 * It advances in n_sub explicit substeps per tissue step (n_sub <= 0: the
 * smallest n_sub with dt/n_sub <= 0.9 min_i chi Cm l_i / (sigma sum_j s_ij/L_ij),
 * nodes whose segments are all blocked left out).
 * Junctions (Sec. 3.3): an upward crossing of the threshold at the junction
 * node during tissue step n stimulates its muscle region (cells whose
 * centroid lies within `radius`, else the cells sharing a node with the cell
 * of nearest centroid) with amp for dur ms from step n + 1 + round(delay/dt);
 * with two_way the upward crossing of the region's mean potential stimulates
 * the node after delay_anti.  Each step: tissue, then Purkinje substeps, then
 * junction events. */
int orc_set_purkinje(orc_sim *s, int64_t n, const double *xyz, int64_t n_edges,
                     const int32_t *edges, const double *edge_scale, double sigma,
                     int model, int32_t n_sub);
int orc_add_pmj(orc_sim *s, int32_t node, double radius, double delay_ortho,
                double delay_anti, int two_way, double amp, double dur);
int orc_add_purkinje_stimulus(orc_sim *s, int64_t n_ids, const int32_t *ids,
                              double t0, double dur, double amp, double period,
                              int32_t count);
int32_t orc_purkinje_n_sub(const orc_sim *s);

/* Time scheme of the non-gating states (the potential of cells and graph
 * nodes, the concentrations, Stewart's Rbar): 0 forward Euler (the paper's
 * scheme, Sec. 3.2), 1 second-order Adams-Bashforth, which the paper names
 * as the way to shrink the time error of those states (Sec. 4):
 * y^{n+1} = y^n + dt (3/2 f^n - 1/2 f^{n-1}), forward Euler on step 0 (and
 * graph substep 0).  Gates stay Rush-Larsen in both; 2 adds the
 * second-order Rush-Larsen step the paper names as the way to second order
 * overall: each gate's steady state and time constant are evaluated at the
 * midpoint predictions v^n + dt/2 f_v^n and c^n + dt/2 f_c^n of the potential
 * and of the calcium concentrations it depends on (CRN's release gates u, v
 * keep their level-n driver).  AB2 is stable on half
 * the interval of forward Euler, so a derived substep count uses half the
 * graph bound.  Call before stepping; returns -1 for an unknown scheme. */
int orc_set_time_scheme(orc_sim *s, int scheme);
/* Per-medium time step: the 2D medium (triangles) takes n_sub substeps of
 * dt / n_sub per step; n_sub <= 0 derives the count from the medium's
 * forward-Euler bound (90 %, 45 % with Adams-Bashforth 2).  Before the first
 * step only; set the time scheme first.  -1 after the first step. */
int orc_set_medium_substeps(orc_sim *s, int32_t n_sub);
int32_t orc_medium_substeps(const orc_sim *s);
void orc_get_purkinje_vm(const orc_sim *s, double *out);
void orc_get_purkinje_activation(const orc_sim *s, double *out);
/* Junction whose source is a cell (the coupling of the 2D Purkinje shell
 * to the 3D myocardium through communication nodes, Sec. 3.3): the region
 * is the cells of the other kind (tets for a triangle source, triangles for
 * a tet) whose centroid lies within `radius` of the source's centroid, else
 * the cells of that kind sharing a node with the nearest one; the source's
 * upward crossing during step n pulses the region from n + 1 + round(delay/dt),
 * and with two_way the region mean's crossing pulses the source cell.
 * Shares the index sequence of orc_add_pmj; -1 for a bad cell or no region. */
int orc_add_cell_junction(orc_sim *s, int32_t cell, double radius, double delay_ortho,
                          double delay_anti, int two_way, double amp, double dur);
/* muscle region of junction k (at most cap ids); returns its size */
int64_t orc_get_pmj_region(const orc_sim *s, int k, int32_t *out, int64_t cap);

/* ----------------------------------------------------------- bidomain */
/* Bidomain (Sec. 3.1 eq. electro, Sec. 3.2 eq. electro2_3d): the monodomain
 * conductivities become the intracellular ones M_i, sigma_el / sigma_et the
 * extracellular M_e (same fibres and scale).  Each step advances v with the
 * intracellular flux of v + phi_e at level n, then solves
 *   sum_f A_f ((M_i + M_e) grad phi).n = -sum_f A_f (M_i grad v^{n+1}).n
 * for phi_e^{n+1} by restarted GMRES(restart) from phi_e^n, to a residual of
 * tol ||rhs|| or max_iter Arnoldi steps, then shifts phi_e to zero
 * volume-weighted mean.  phi_e^0 = 0. */
int orc_set_bidomain(orc_sim *s, double sigma_el, double sigma_et, int restart, double tol,
                     int max_iter);
void orc_get_phi_e(const orc_sim *s, double *out);
/* Arnoldi steps of the last solve (total over all solves, last residual) */
int64_t orc_bidomain_iterations(const orc_sim *s, int64_t *total, double *relres);
/* y = the flux sums sum_f A_f (M_f grad x_f).n_f for conductivities (sl, st) */
void orc_apply_flux(const orc_sim *s, const double *x, double sl, double st, double *y);
/* GMRES on that operator (x: start in, solution out); returns Arnoldi steps */
int64_t orc_gmres(orc_sim *s, const double *b, double *x, double sl, double st, int restart,
                  double tol, int max_iter, double *relres);

/* ---------------------------------------- operator probes (for pinning) */
/* Per tet: volume, 4 outward area vectors S_j (face opposite local node j),
 * 4 face neighbours (-1 = boundary face). */
void orc_geometry(const orc_sim *s, double *vol, double *area_vec,
                  int32_t *nbr);
void orc_node_values(const orc_sim *s, const double *v, double *vn);
void orc_cell_gradients(const orc_sim *s, const double *v, double *g);
/* L_c = sum_faces A (M_f grad v_f).n / (chi cm V_c), mV/ms */
void orc_apply_diffusion(const orc_sim *s, const double *v, double *L);

/* Detection on one sampled waveform v[0..n-1] at spacing dt. */
void orc_detect_waveform(const double *v, int64_t n, double dt,
                         double threshold, double repol_frac, double *t_act,
                         double *apd90);
int orc_num_threads(void);
void orc_set_num_threads(int n);   /* OpenMP threads of later calls */

#ifdef __cplusplus
}
#endif
#endif
