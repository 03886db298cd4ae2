/* Courtemanche-Ramirez-Nattel human atrial cell model, FP64 oracle version.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Model: M. Courtemanche, R.J. Ramirez, S. Nattel, "Ionic mechanisms
 * underlying human atrial action potential properties: insights from a
 * mathematical model", Am J Physiol 275 (1998) H301-H321.  The paper uses it
 * for the atria (Sec. 3.1) with 15 gating variables out of 21 states
 * (Sec. 3.2).  Gates are Rush-Larsen integrated; Na_i, K_i, Ca_i, Ca_up,
 * Ca_rel forward Euler, with the buffering of Ca_i (troponin, calmodulin)
 * and Ca_rel (calsequestrin) folded into their rate as in the article.
 * Ion fluxes into concentrations use the total current Cm * I (pA).
 *
 * Slot order: 0 V, 1 m, 2 h, 3 j, 4 oa, 5 oi, 6 ua, 7 ui, 8 xr, 9 xs, 10 d,
 * 11 f, 12 fCa, 13 u, 14 v, 15 w, 16 Ca_i, 17 Ca_up, 18 Ca_rel, 19 Na_i,
 * 20 K_i.  Units: mV, ms, mM, pA/pF.
 */
#include <math.h>
#include <stddef.h>
#include "orc_models.h"

static const double R_GAS = 8.3143, T_K = 310.0, F_C = 96.4867;
static const double CM = 100.0;                       /* pF            */
static const double V_I = 13668.0, V_UP = 1109.52, V_RELV = 96.48; /* um^3 */
static const double K_O = 5.4, NA_O = 140.0, CA_O = 1.8;
/* maximal conductances and pump rates as printed in the article's parameter
 * table (nS/pF, pA/pF); published code versions carry more digits */
static const double G_NA = 7.8, G_K1 = 0.09, G_TO = 0.1652;
static const double G_KR = 0.0294, G_KS = 0.129, G_CAL = 0.1238;
static const double G_BCA = 0.00113, G_BNA = 0.000674;
static const double INAK_MAX = 0.60, INACA_MAX = 1600.0, IPCA_MAX = 0.275;
static const double IUP_MAX = 0.005, KQ10 = 3.0, GAMMA = 0.35;
static const double KM_NAI = 10.0, KM_KO = 1.5, KM_NA = 87.5, KM_CA = 1.38;
static const double K_SAT = 0.1, K_REL = 30.0, K_UP = 0.00092;
static const double CAUP_MAX = 15.0, CMDN_MAX = 0.05, TRPN_MAX = 0.07;
static const double CSQN_MAX = 10.0, KM_CMDN = 0.00238, KM_TRPN = 0.0005;
static const double KM_CSQN = 0.8, TAU_TR = 180.0;

static const char *const SLOT_NAMES[21] = {
    "V", "m", "h", "j", "oa", "oi", "ua", "ui", "xr", "xs", "d", "f", "fCa",
    "u", "v", "w", "Ca_i", "Ca_up", "Ca_rel", "Na_i", "K_i"};

const char *orc_crn_slot_name(int slot)
{
    return (slot >= 0 && slot < 21) ? SLOT_NAMES[slot] : NULL;
}

void orc_crn_init(double *y)
{
    /* initial values listed in the article */
    y[0] = -81.18;
    y[1] = 2.908e-3; y[2] = 9.649e-1; y[3] = 9.775e-1;
    y[4] = 3.043e-2; y[5] = 9.992e-1; y[6] = 4.966e-3; y[7] = 9.986e-1;
    y[8] = 3.296e-5; y[9] = 1.869e-2; y[10] = 1.367e-4; y[11] = 9.996e-1;
    y[12] = 7.755e-1; y[13] = 0.0; y[14] = 1.0; y[15] = 9.992e-1;
    y[16] = 1.013e-4; y[17] = 1.488; y[18] = 1.488; y[19] = 11.17;
    y[20] = 139.0;
}

/* z / (exp(z) - 1), continuous at z = 0 */
static double z_over_expm1(double z)
{
    return (fabs(z) < 1e-12) ? 1.0 : z / expm1(z);
}

static double rush_larsen(double y, double yinf, double tau, double dt)
{
    return yinf + (y - yinf) * exp(-dt / tau);
}

double orc_crn_step(double *y, double dt, double istim, const double *gs, orc_hist *hist,
                    const orc_mid *mid)
{
    (void)istim;  /* the article's K_i balance carries no stimulus term */
    const double V = y[0];
    double m = y[1], h = y[2], j = y[3], oa = y[4], oi = y[5], ua = y[6];
    double ui = y[7], xr = y[8], xs = y[9], d = y[10], f = y[11], fca = y[12];
    double u = y[13], v = y[14], w = y[15];
    double cai = y[16], caup = y[17], carel = y[18], nai = y[19], ki = y[20];
    const double sKr = gs ? gs[0] : 1.0, sKs = gs ? gs[1] : 1.0;
    const double sCaL = gs ? gs[2] : 1.0, sNa = gs ? gs[3] : 1.0;
    const double RTF = R_GAS * T_K / F_C;

    const double E_Na = RTF * log(NA_O / nai);
    const double E_K = RTF * log(K_O / ki);
    const double E_Ca = 0.5 * RTF * log(CA_O / cai);

    /* currents (pA/pF) */
    const double I_Na = sNa * G_NA * m * m * m * h * j * (V - E_Na);
    const double I_K1 = G_K1 * (V - E_K) / (1.0 + exp(0.07 * (V + 80.0)));
    const double I_to = G_TO * oa * oa * oa * oi * (V - E_K);
    const double g_Kur = 0.005 + 0.05 / (1.0 + exp(-(V - 15.0) / 13.0));
    const double I_Kur = g_Kur * ua * ua * ua * ui * (V - E_K);
    const double I_Kr = sKr * G_KR * xr * (V - E_K) / (1.0 + exp((V + 15.0) / 22.4));
    const double I_Ks = sKs * G_KS * xs * xs * (V - E_K);
    const double I_CaL = sCaL * G_CAL * d * f * fca * (V - 65.0);
    const double sigma = (exp(NA_O / 67.3) - 1.0) / 7.0;
    const double f_NaK = 1.0 / (1.0 + 0.1245 * exp(-0.1 * V / RTF) +
                                0.0365 * sigma * exp(-V / RTF));
    const double I_NaK = INAK_MAX * f_NaK / (1.0 + pow(KM_NAI / nai, 1.5)) *
                         K_O / (K_O + KM_KO);
    const double I_NaCa =
        INACA_MAX *
        (exp(GAMMA * V / RTF) * nai * nai * nai * CA_O -
         exp((GAMMA - 1.0) * V / RTF) * NA_O * NA_O * NA_O * cai) /
        ((KM_NA * KM_NA * KM_NA + NA_O * NA_O * NA_O) * (KM_CA + CA_O) *
         (1.0 + K_SAT * exp((GAMMA - 1.0) * V / RTF)));
    const double I_bNa = G_BNA * (V - E_Na);
    const double I_bCa = G_BCA * (V - E_Ca);
    const double I_pCa = IPCA_MAX * cai / (0.0005 + cai);
    const double I_ion = I_Na + I_K1 + I_to + I_Kur + I_Kr + I_Ks + I_CaL +
                         I_pCa + I_NaK + I_NaCa + I_bNa + I_bCa;

    /* SR fluxes (mM/ms) */
    const double I_rel = K_REL * u * u * v * w * (carel - cai);
    const double I_tr = (caup - carel) / TAU_TR;
    const double I_up = IUP_MAX / (1.0 + K_UP / cai);
    const double I_upleak = IUP_MAX * caup / CAUP_MAX;

    /* concentration rates at level n */
    const double dNai = (-3.0 * I_NaK - 3.0 * I_NaCa - I_bNa - I_Na) * CM / (F_C * V_I);
    const double dKi = (2.0 * I_NaK - I_K1 - I_to - I_Kur - I_Kr - I_Ks) * CM / (F_C * V_I);
    const double B1 = (2.0 * I_NaCa - I_pCa - I_CaL - I_bCa) * CM / (2.0 * F_C * V_I) +
                      (V_UP * (I_upleak - I_up) + I_rel * V_RELV) / V_I;
    const double B2 = 1.0 + TRPN_MAX * KM_TRPN / ((cai + KM_TRPN) * (cai + KM_TRPN)) +
                      CMDN_MAX * KM_CMDN / ((cai + KM_CMDN) * (cai + KM_CMDN));
    const double dCai = B1 / B2;
    const double dCaup = I_up - I_upleak - I_tr * V_RELV / V_UP;
    const double dCarel = (I_tr - I_rel) /
                          (1.0 + CSQN_MAX * KM_CSQN / ((carel + KM_CSQN) * (carel + KM_CSQN)));

    /* release gating driver: SR release flux and sarcolemmal Ca influx */
    const double Fn = 1e-12 * V_RELV * I_rel -
                      5e-13 / F_C * (0.5 * CM * I_CaL - 0.2 * CM * I_NaCa);

    /* ---- gates, Rush-Larsen at level n, or at the midpoint predictions of
     * V and Ca_i (second-order variant; u and v keep the level-n release
     * driver Fn) ---- */
    const double Vg = mid ? V + 0.5 * dt * (mid->lmi - I_ion) : V;
    const double cai_g = mid ? cai + 0.5 * dt * dCai : cai;
    {
    const double V = Vg, cai = cai_g;
    double a, b, yinf, tau;
    /* m: alpha = 0.32 (V+47.13)/(1 - exp(-0.1 (V+47.13))) */
    a = 3.2 * z_over_expm1(-0.1 * (V + 47.13));
    b = 0.08 * exp(-V / 11.0);
    m = rush_larsen(m, a / (a + b), 1.0 / (a + b), dt);
    /* h, j */
    if (V >= -40.0) {
        a = 0.0;
        b = 1.0 / (0.13 * (1.0 + exp(-(V + 10.66) / 11.1)));
    } else {
        a = 0.135 * exp(-(V + 80.0) / 6.8);
        b = 3.56 * exp(0.079 * V) + 3.1e5 * exp(0.35 * V);
    }
    h = rush_larsen(h, a / (a + b), 1.0 / (a + b), dt);
    if (V >= -40.0) {
        a = 0.0;
        b = 0.3 * exp(-2.535e-7 * V) / (1.0 + exp(-0.1 * (V + 32.0)));
    } else {
        a = (-127140.0 * exp(0.2444 * V) - 3.474e-5 * exp(-0.04391 * V)) *
            (V + 37.78) / (1.0 + exp(0.311 * (V + 79.23)));
        b = 0.1212 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14)));
    }
    j = rush_larsen(j, a / (a + b), 1.0 / (a + b), dt);
    /* oa, ua share their rate constants */
    a = 0.65 / (exp(-(V + 10.0) / 8.5) + exp(-(V - 30.0) / 59.0));
    b = 0.65 / (2.5 + exp((V + 82.0) / 17.0));
    tau = 1.0 / ((a + b) * KQ10);
    oa = rush_larsen(oa, 1.0 / (1.0 + exp(-(V + 20.47) / 17.54)), tau, dt);
    ua = rush_larsen(ua, 1.0 / (1.0 + exp(-(V + 30.3) / 9.6)), tau, dt);
    /* oi */
    a = 1.0 / (18.53 + exp((V + 113.7) / 10.95));
    b = 1.0 / (35.56 + exp(-(V + 1.26) / 7.44));
    oi = rush_larsen(oi, 1.0 / (1.0 + exp((V + 43.1) / 5.3)), 1.0 / ((a + b) * KQ10), dt);
    /* ui */
    a = 1.0 / (21.0 + exp(-(V - 185.0) / 28.0));
    b = exp((V - 158.0) / 16.0);
    ui = rush_larsen(ui, 1.0 / (1.0 + exp((V - 99.45) / 27.48)), 1.0 / ((a + b) * KQ10), dt);
    /* xr: alpha = 3e-4 (V+14.1)/(1-exp(-(V+14.1)/5)),
     *     beta = 7.3898e-5 (V-3.3328)/(exp((V-3.3328)/5.1237)-1) */
    a = 0.0003 * 5.0 * z_over_expm1(-(V + 14.1) / 5.0);
    b = 7.3898e-5 * 5.1237 * z_over_expm1((V - 3.3328) / 5.1237);
    xr = rush_larsen(xr, 1.0 / (1.0 + exp(-(V + 14.1) / 6.5)), 1.0 / (a + b), dt);
    /* xs: alpha = 4e-5 (V-19.9)/(1-exp(-(V-19.9)/17)),
     *     beta = 3.5e-5 (V-19.9)/(exp((V-19.9)/9)-1) */
    a = 4e-5 * 17.0 * z_over_expm1(-(V - 19.9) / 17.0);
    b = 3.5e-5 * 9.0 * z_over_expm1((V - 19.9) / 9.0);
    xs = rush_larsen(xs, 1.0 / sqrt(1.0 + exp(-(V - 19.9) / 12.7)), 0.5 / (a + b), dt);
    /* d: tau = (1 - exp(-(V+10)/6.24)) / (0.035 (V+10) (1 + exp(-(V+10)/6.24))) */
    {
        const double zz = (V + 10.0) / 6.24;
        const double ratio = 1.0 / z_over_expm1(-zz);  /* (1-e^{-z})/z */
        tau = ratio / (0.035 * 6.24 * (1.0 + exp(-zz)));
        d = rush_larsen(d, 1.0 / (1.0 + exp(-(V + 10.0) / 8.0)), tau, dt);
    }
    /* f */
    tau = 9.0 / (0.0197 * exp(-0.0337 * 0.0337 * (V + 10.0) * (V + 10.0)) + 0.02);
    f = rush_larsen(f, 1.0 / (1.0 + exp((V + 28.0) / 6.9)), tau, dt);
    /* fCa (uses Ca_i at level n) */
    fca = rush_larsen(fca, 1.0 / (1.0 + cai / 0.00035), 2.0, dt);
    /* u, v: driven by Fn */
    yinf = 1.0 / (1.0 + exp(-(Fn - 3.4175e-13) / 13.67e-16));
    u = rush_larsen(u, yinf, 8.0, dt);
    tau = 1.91 + 2.09 / (1.0 + exp(-(Fn - 3.4175e-13) / 13.67e-16));
    yinf = 1.0 - 1.0 / (1.0 + exp(-(Fn - 6.835e-14) / 13.67e-16));
    v = rush_larsen(v, yinf, tau, dt);
    /* w: tau = 6 (1 - exp(-(V-7.9)/5)) / ((1 + 0.3 exp(-(V-7.9)/5)) (V-7.9)) */
    {
        const double zz = (V - 7.9) / 5.0;
        const double ratio = 1.0 / z_over_expm1(-zz);  /* (1-e^{-z})/z */
        tau = 6.0 * ratio / (5.0 * (1.0 + 0.3 * exp(-zz)));
        w = rush_larsen(w, 1.0 - 1.0 / (1.0 + exp(-(V - 40.0) / 17.0)), tau, dt);
    }

    }

    /* ---- concentrations, forward Euler or Adams-Bashforth 2 ---- */
    nai += dt * orc_rate(hist, 3, dNai);
    ki += dt * orc_rate(hist, 4, dKi);
    cai += dt * orc_rate(hist, 0, dCai);
    caup += dt * orc_rate(hist, 1, dCaup);
    carel += dt * orc_rate(hist, 2, dCarel);

    y[1] = m; y[2] = h; y[3] = j; y[4] = oa; y[5] = oi; y[6] = ua; y[7] = ui;
    y[8] = xr; y[9] = xs; y[10] = d; y[11] = f; y[12] = fca; y[13] = u;
    y[14] = v; y[15] = w; y[16] = cai; y[17] = caup; y[18] = carel;
    y[19] = nai; y[20] = ki;
    return I_ion;
}
