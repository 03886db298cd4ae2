/* ten Tusscher-Panfilov human ventricular cell model, FP64 oracle version.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Model: K.H.W.J. ten Tusscher, A.V. Panfilov, "Alternans and spiral breakup
 * in a human ventricular tissue model", Am J Physiol Heart Circ Physiol 291
 * (2006) H1088-H1100, which keeps the currents of K.H.W.J. ten Tusscher,
 * D. Noble, P.J. Noble, A.V. Panfilov, Am J Physiol Heart Circ Physiol 286
 * (2004) H1573-H1589 and replaces the L-type calcium current and the
 * calcium-induced calcium release.  The paper uses it for the ventricles
 * (Sec. 3.1) and counts 13 gating variables out of 19 states (Sec. 3.2):
 * the 12 Hodgkin-Huxley gates plus the RyR recovery variable Rbar, whose
 * equation is linear in Rbar at fixed Ca_SS and is therefore Rush-Larsen
 * integrated too.  The buffered concentrations Ca_i, Ca_SR, Ca_SS use the
 * rapid-buffering approximation of the 2004 article: forward Euler on the
 * total (free + bound) concentration, then the free concentration is the
 * positive root of the buffer equilibrium quadratic.
 *
 * Slot order: 0 V, 1 m, 2 h, 3 j, 4 xr1, 5 xr2, 6 xs, 7 r, 8 s, 9 d, 10 f,
 * 11 f2, 12 fCass, 13 Rbar, 14 Ca_i, 15 Ca_SR, 16 Ca_SS, 17 Na_i, 18 K_i.
 * Units: mV, ms, mM, pA/pF.
 */
#include <math.h>
#include <stddef.h>
#include "orc_models.h"

/* physical constants and cell geometry */
static const double R_GAS = 8314.472;    /* mJ/(K mol)   */
static const double T_K = 310.0;         /* K            */
static const double F_C = 96485.3415;    /* C/mol        */
static const double CAP = 0.185;         /* cell capacitance (uF scale)   */
static const double V_C = 0.016404;      /* cytoplasmic volume            */
static const double V_SR = 0.001094;     /* SR volume                     */
static const double V_SS = 0.00005468;   /* subspace volume               */
/* extracellular concentrations, mM */
static const double K_O = 5.4, NA_O = 140.0, CA_O = 2.0;
/* maximal conductances and pump/exchanger parameters */
static const double G_NA = 14.838, G_K1 = 5.405, G_KR = 0.153;
static const double P_KNA = 0.03, G_CAL = 3.980e-5;
static const double K_NACA = 1000.0, GAMMA_NACA = 0.35, KM_CA = 1.38;
static const double KM_NAI = 87.5, K_SAT = 0.1, ALPHA_NACA = 2.5;
static const double P_NAK = 2.724, KM_K = 1.0, KM_NA = 40.0;
static const double G_PK = 0.0146, G_PCA = 0.1238, K_PCA = 0.0005;
static const double G_BNA = 0.00029, G_BCA = 0.000592;
/* intracellular calcium handling */
static const double VMAX_UP = 0.006375, K_UP = 0.00025, V_REL = 0.102;
static const double K1P = 0.15, K2P = 0.045, K3 = 0.060, K4 = 0.005;
static const double EC = 1.5, MAX_SR = 2.5, MIN_SR = 1.0;
static const double V_LEAK = 0.00036, V_XFER = 0.0038;
static const double BUF_C = 0.2, K_BUFC = 0.001;
static const double BUF_SR = 10.0, K_BUFSR = 0.3;
static const double BUF_SS = 0.4, K_BUFSS = 0.00025;

static const char *const SLOT_NAMES[19] = {
    "V", "m", "h", "j", "xr1", "xr2", "xs", "r", "s", "d", "f", "f2",
    "fCass", "Rbar", "Ca_i", "Ca_SR", "Ca_SS", "Na_i", "K_i"};

const char *orc_tp06_slot_name(int slot)
{
    return (slot >= 0 && slot < 19) ? SLOT_NAMES[slot] : NULL;
}

void orc_tp06_init(double *y)
{
    /* the standard resting initial state of the model */
    y[0] = -86.2;
    y[1] = 0.0;      /* m     */
    y[2] = 0.75;     /* h     */
    y[3] = 0.75;     /* j     */
    y[4] = 0.0;      /* xr1   */
    y[5] = 1.0;      /* xr2   */
    y[6] = 0.0;      /* xs    */
    y[7] = 0.0;      /* r     */
    y[8] = 1.0;      /* s     */
    y[9] = 0.0;      /* d     */
    y[10] = 1.0;     /* f     */
    y[11] = 1.0;     /* f2    */
    y[12] = 1.0;     /* fCass */
    y[13] = 1.0;     /* Rbar  */
    y[14] = 0.00007; /* Ca_i  */
    y[15] = 1.3;     /* Ca_SR */
    y[16] = 0.00007; /* Ca_SS */
    y[17] = 7.67;    /* Na_i  */
    y[18] = 138.3;   /* K_i   */
}

/* Rush-Larsen: exact solution of dy/dt = (yinf - y)/tau over dt at fixed V */
static double rush_larsen(double y, double yinf, double tau, double dt)
{
    return yinf + (y - yinf) * exp(-dt / tau);
}

/* free concentration from the total under one rapid buffer of capacity B and
 * dissociation constant K: c + B c/(c + K) = total, positive root */
static double free_from_total(double total, double B, double K)
{
    double b = B + K - total;
    double disc = sqrt(b * b + 4.0 * K * total);
    /* both forms are the same root; pick the one without cancellation */
    return (b >= 0.0) ? (2.0 * K * total) / (disc + b) : 0.5 * (disc - b);
}

static double total_from_free(double c, double B, double K)
{
    return c + B * c / (c + K);
}

double orc_tp06_step(int celltype, double *y, double dt, double istim,
                     const double *gs, orc_hist *hist, const orc_mid *mid)
{
    const double V = y[0];
    double m = y[1], h = y[2], j = y[3], xr1 = y[4], xr2 = y[5], xs = y[6];
    double r = y[7], s = y[8], d = y[9], f = y[10], f2 = y[11];
    double fcass = y[12], rbar = y[13];
    double cai = y[14], casr = y[15], cass = y[16], nai = y[17], ki = y[18];
    const double sKr = gs ? gs[0] : 1.0, sKs = gs ? gs[1] : 1.0;
    const double sCaL = gs ? gs[2] : 1.0, sNa = gs ? gs[3] : 1.0;

    const double RTF = R_GAS * T_K / F_C;  /* mV */
    /* cell-type dependent parameters (2006 article, Table 1 of 2004) */
    double g_to, g_ks;
    if (celltype == 0) {          /* endocardial */
        g_to = 0.073; g_ks = 0.392;
    } else if (celltype == 1) {   /* mid-myocardial (M) */
        g_to = 0.294; g_ks = 0.098;
    } else {                      /* epicardial */
        g_to = 0.294; g_ks = 0.392;
    }

    /* reversal potentials */
    const double E_Na = RTF * log(NA_O / nai);
    const double E_K = RTF * log(K_O / ki);
    const double E_Ca = 0.5 * RTF * log(CA_O / cai);
    const double E_Ks = RTF * log((K_O + P_KNA * NA_O) / (ki + P_KNA * nai));

    /* fast sodium current */
    const double I_Na = sNa * G_NA * m * m * m * h * j * (V - E_Na);

    /* L-type calcium current (GHK form, voltage offset 15 mV) */
    const double x = 2.0 * (V - 15.0) / RTF;
    const double ghk = (fabs(x) < 1e-12) ? 1.0 : x / expm1(x);  /* x/(e^x-1) */
    const double I_CaL = sCaL * G_CAL * d * f * f2 * fcass * 2.0 * F_C * ghk *
                         (0.25 * cass * exp(x) - CA_O);

    /* transient outward current */
    const double I_to = g_to * r * s * (V - E_K);

    /* slow and rapid delayed rectifiers */
    const double I_Ks = sKs * g_ks * xs * xs * (V - E_Ks);
    const double I_Kr = sKr * G_KR * sqrt(K_O / 5.4) * xr1 * xr2 * (V - E_K);

    /* inward rectifier, instantaneous */
    const double a_K1 = 0.1 / (1.0 + exp(0.06 * (V - E_K - 200.0)));
    const double b_K1 = (3.0 * exp(0.0002 * (V - E_K + 100.0)) +
                         exp(0.1 * (V - E_K - 10.0))) /
                        (1.0 + exp(-0.5 * (V - E_K)));
    const double xK1_inf = a_K1 / (a_K1 + b_K1);
    const double I_K1 = G_K1 * sqrt(K_O / 5.4) * xK1_inf * (V - E_K);

    /* Na/Ca exchanger */
    const double e_g = exp(GAMMA_NACA * V / RTF);
    const double e_g1 = exp((GAMMA_NACA - 1.0) * V / RTF);
    const double I_NaCa =
        K_NACA * (e_g * nai * nai * nai * CA_O -
                  e_g1 * NA_O * NA_O * NA_O * cai * ALPHA_NACA) /
        ((KM_NAI * KM_NAI * KM_NAI + NA_O * NA_O * NA_O) * (KM_CA + CA_O) *
         (1.0 + K_SAT * e_g1));

    /* Na/K pump */
    const double I_NaK =
        P_NAK * K_O * nai /
        ((K_O + KM_K) * (nai + KM_NA) *
         (1.0 + 0.1245 * exp(-0.1 * V / RTF) + 0.0353 * exp(-V / RTF)));

    /* plateau and background currents */
    const double I_pCa = G_PCA * cai / (K_PCA + cai);
    const double I_pK = G_PK * (V - E_K) / (1.0 + exp((25.0 - V) / 5.98));
    const double I_bNa = G_BNA * (V - E_Na);
    const double I_bCa = G_BCA * (V - E_Ca);

    const double I_ion = I_Na + I_K1 + I_to + I_Kr + I_Ks + I_CaL + I_NaCa +
                         I_NaK + I_pCa + I_pK + I_bNa + I_bCa;

    /* ---- calcium dynamics at level n ---- */
    const double kcasr = MAX_SR - (MAX_SR - MIN_SR) / (1.0 + (EC / casr) * (EC / casr));
    const double k1 = K1P / kcasr;
    const double O = k1 * cass * cass * rbar / (K3 + k1 * cass * cass);
    const double I_rel = V_REL * O * (casr - cass);
    const double I_up = VMAX_UP / (1.0 + (K_UP * K_UP) / (cai * cai));
    const double I_leak = V_LEAK * (casr - cai);
    const double I_xfer = V_XFER * (cass - cai);

    const double dCaiT = -(I_bCa + I_pCa - 2.0 * I_NaCa) * CAP / (2.0 * V_C * F_C) +
                         (I_leak - I_up) * V_SR / V_C + I_xfer;
    const double dCasrT = I_up - I_rel - I_leak;
    const double dCassT = -I_CaL * CAP / (2.0 * V_SS * F_C) +
                          I_rel * V_SR / V_SS - I_xfer * V_C / V_SS;
    const double dNai = -(I_Na + I_bNa + 3.0 * I_NaK + 3.0 * I_NaCa) * CAP / (V_C * F_C);
    /* the stimulus current is carried by K+ (2004 article); the axial
     * (diffusive) current is not included */
    const double dKi = -(I_K1 + I_to + I_Kr + I_Ks - 2.0 * I_NaK + I_pK + istim) *
                       CAP / (V_C * F_C);

    /* ---- gating variables, Rush-Larsen at V^n, or at the midpoint
     * predictions of V, Ca_SS and Ca_SR (second-order variant) ---- */
    double Vg = V, cass_g = cass, casr_g = casr;
    if (mid) {
        Vg = V + 0.5 * dt * (mid->lmi - I_ion);
        cass_g = free_from_total(total_from_free(cass, BUF_SS, K_BUFSS) + 0.5 * dt * dCassT,
                                 BUF_SS, K_BUFSS);
        casr_g = free_from_total(total_from_free(casr, BUF_SR, K_BUFSR) + 0.5 * dt * dCasrT,
                                 BUF_SR, K_BUFSR);
    }
    {
    const double V = Vg, cass = cass_g;
    const double k2 = K2P * (MAX_SR - (MAX_SR - MIN_SR) / (1.0 + (EC / casr_g) * (EC / casr_g)));
    double yinf, tau, a, b, c;
    /* m */
    yinf = 1.0 / ((1.0 + exp((-56.86 - V) / 9.03)) * (1.0 + exp((-56.86 - V) / 9.03)));
    a = 1.0 / (1.0 + exp((-60.0 - V) / 5.0));
    b = 0.1 / (1.0 + exp((V + 35.0) / 5.0)) + 0.10 / (1.0 + exp((V - 50.0) / 200.0));
    m = rush_larsen(m, yinf, a * b, dt);
    /* h */
    yinf = 1.0 / ((1.0 + exp((V + 71.55) / 7.43)) * (1.0 + exp((V + 71.55) / 7.43)));
    if (V >= -40.0) {
        a = 0.0;
        b = 0.77 / (0.13 * (1.0 + exp(-(V + 10.66) / 11.1)));
    } else {
        a = 0.057 * exp(-(V + 80.0) / 6.8);
        b = 2.7 * exp(0.079 * V) + 3.1e5 * exp(0.3485 * V);
    }
    h = rush_larsen(h, yinf, 1.0 / (a + b), dt);
    /* j (same steady state as h) */
    if (V >= -40.0) {
        a = 0.0;
        b = 0.6 * exp(0.057 * V) / (1.0 + exp(-0.1 * (V + 32.0)));
    } else {
        a = (-2.5428e4 * exp(0.2444 * V) - 6.948e-6 * exp(-0.04391 * V)) *
            (V + 37.78) / (1.0 + exp(0.311 * (V + 79.23)));
        b = 0.02424 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14)));
    }
    j = rush_larsen(j, yinf, 1.0 / (a + b), dt);
    /* xr1 */
    yinf = 1.0 / (1.0 + exp((-26.0 - V) / 7.0));
    a = 450.0 / (1.0 + exp((-45.0 - V) / 10.0));
    b = 6.0 / (1.0 + exp((V + 30.0) / 11.5));
    xr1 = rush_larsen(xr1, yinf, a * b, dt);
    /* xr2 */
    yinf = 1.0 / (1.0 + exp((V + 88.0) / 24.0));
    a = 3.0 / (1.0 + exp((-60.0 - V) / 20.0));
    b = 1.12 / (1.0 + exp((V - 60.0) / 20.0));
    xr2 = rush_larsen(xr2, yinf, a * b, dt);
    /* xs */
    yinf = 1.0 / (1.0 + exp((-5.0 - V) / 14.0));
    a = 1400.0 / sqrt(1.0 + exp((5.0 - V) / 6.0));
    b = 1.0 / (1.0 + exp((V - 35.0) / 15.0));
    xs = rush_larsen(xs, yinf, a * b + 80.0, dt);
    /* r */
    yinf = 1.0 / (1.0 + exp((20.0 - V) / 6.0));
    tau = 9.5 * exp(-(V + 40.0) * (V + 40.0) / 1800.0) + 0.8;
    r = rush_larsen(r, yinf, tau, dt);
    /* s */
    if (celltype == 0) {
        yinf = 1.0 / (1.0 + exp((V + 28.0) / 5.0));
        tau = 1000.0 * exp(-(V + 67.0) * (V + 67.0) / 1000.0) + 8.0;
    } else {
        yinf = 1.0 / (1.0 + exp((V + 20.0) / 5.0));
        tau = 85.0 * exp(-(V + 45.0) * (V + 45.0) / 320.0) +
              5.0 / (1.0 + exp((V - 20.0) / 5.0)) + 3.0;
    }
    s = rush_larsen(s, yinf, tau, dt);
    /* d */
    yinf = 1.0 / (1.0 + exp((-8.0 - V) / 7.5));
    a = 1.4 / (1.0 + exp((-35.0 - V) / 13.0)) + 0.25;
    b = 1.4 / (1.0 + exp((V + 5.0) / 5.0));
    c = 1.0 / (1.0 + exp((50.0 - V) / 20.0));
    d = rush_larsen(d, yinf, a * b + c, dt);
    /* f */
    yinf = 1.0 / (1.0 + exp((V + 20.0) / 7.0));
    a = 1102.5 * exp(-(V + 27.0) * (V + 27.0) / 225.0);
    b = 200.0 / (1.0 + exp((13.0 - V) / 10.0));
    c = 180.0 / (1.0 + exp((V + 30.0) / 10.0)) + 20.0;
    f = rush_larsen(f, yinf, a + b + c, dt);
    /* f2: the time constant as printed in the 2006 article's appendix
     * (562, 27, 240, 80); the authors' distributed code uses another set */
    yinf = 0.67 / (1.0 + exp((V + 35.0) / 7.0)) + 0.33;
    a = 562.0 * exp(-(V + 27.0) * (V + 27.0) / 240.0);
    b = 31.0 / (1.0 + exp((25.0 - V) / 10.0));
    c = 80.0 / (1.0 + exp((V + 30.0) / 10.0));
    f2 = rush_larsen(f2, yinf, a + b + c, dt);
    /* fCass (calcium dependent, uses Ca_SS at level n) */
    {
        const double q = (cass / 0.05) * (cass / 0.05);
        yinf = 0.6 / (1.0 + q) + 0.4;
        tau = 80.0 / (1.0 + q) + 2.0;
        fcass = rush_larsen(fcass, yinf, tau, dt);
    }
    /* Rbar: dR/dt = k4 (1 - R) - k2 Ca_SS R, linear in R at fixed Ca_SS */
    {
        const double rate = k2 * cass + K4;
        rbar = rush_larsen(rbar, K4 / rate, 1.0 / rate, dt);
    }
    }

    /* ---- concentrations, forward Euler or Adams-Bashforth 2 (buffered
     * ones on the total) ---- */
    cai = free_from_total(total_from_free(cai, BUF_C, K_BUFC) + dt * orc_rate(hist, 0, dCaiT),
                          BUF_C, K_BUFC);
    casr = free_from_total(total_from_free(casr, BUF_SR, K_BUFSR) + dt * orc_rate(hist, 1, dCasrT),
                           BUF_SR, K_BUFSR);
    cass = free_from_total(total_from_free(cass, BUF_SS, K_BUFSS) + dt * orc_rate(hist, 2, dCassT),
                           BUF_SS, K_BUFSS);
    nai += dt * orc_rate(hist, 3, dNai);
    ki += dt * orc_rate(hist, 4, dKi);

    y[1] = m; y[2] = h; y[3] = j; y[4] = xr1; y[5] = xr2; y[6] = xs;
    y[7] = r; y[8] = s; y[9] = d; y[10] = f; y[11] = f2; y[12] = fcass;
    y[13] = rbar; y[14] = cai; y[15] = casr; y[16] = cass; y[17] = nai;
    y[18] = ki;
    return I_ion;
}
