/* Internal declarations of the oracle's cell models.
 * TEST INFRASTRUCTURE ONLY (see oracle.h). */
#ifndef ORC_MODELS_H
#define ORC_MODELS_H

const char *orc_tp06_slot_name(int slot);
void orc_tp06_init(double *y);
double orc_tp06_step(int celltype, double *y, double dt, double istim,
                     const double *gs);

const char *orc_crn_slot_name(int slot);
void orc_crn_init(double *y);
double orc_crn_step(double *y, double dt, double istim, const double *gs);

const char *orc_stewart_slot_name(int slot);
void orc_stewart_init(double *y);
double orc_stewart_step(double *y, double dt, double istim, const double *gs);

#endif
