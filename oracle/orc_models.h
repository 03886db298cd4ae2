/* Internal declarations of the oracle's cell models.
 * TEST INFRASTRUCTURE ONLY (see oracle.h). */
#ifndef ORC_MODELS_H
#define ORC_MODELS_H

/* Time integration of the non-gating states (the concentrations and, in
 * Stewart, Rbar): forward Euler, the paper's scheme (Sec. 3.2), when h is
 * NULL; otherwise the second-order Adams-Bashforth step the paper points to
 * (Sec. 4), y += dt (3/2 r^n - 1/2 r^(n-1)), with h->r holding each rate of
 * the previous step in the model's order of those states (forward Euler on
 * the first step, h->first != 0).  The gates stay Rush-Larsen. */
typedef struct {
    double *r;
    int first;
} orc_hist;

static inline double orc_rate(orc_hist *h, int k, double r)
{
    if (!h) return r;
    const double prev = h->first ? r : h->r[k];
    h->r[k] = r;
    return 1.5 * r - 0.5 * prev;
}

/* Second-order Rush-Larsen (with AB2 above): the gates' steady states and
 * time constants are evaluated at midpoint predictions of the states they
 * depend on, V + dt/2 (lmi - I_ion) with lmi = L - I_stim the rest of the
 * potential's rate, and c + dt/2 (rate) for the calcium concentrations
 * (through their buffered totals).  NULL: everything at level n. */
typedef struct {
    double lmi;
} orc_mid;

const char *orc_tp06_slot_name(int slot);
void orc_tp06_init(double *y);
double orc_tp06_step(int celltype, double *y, double dt, double istim,
                     const double *gs, orc_hist *h, const orc_mid *mid);

const char *orc_crn_slot_name(int slot);
void orc_crn_init(double *y);
double orc_crn_step(double *y, double dt, double istim, const double *gs, orc_hist *h,
                    const orc_mid *mid);

const char *orc_stewart_slot_name(int slot);
void orc_stewart_init(double *y);
double orc_stewart_step(double *y, double dt, double istim, const double *gs,
                        orc_hist *h, const orc_mid *mid);

#endif
