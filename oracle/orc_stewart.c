/* Stewart et al. human Purkinje fibre cell model, FP64 oracle version.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Model: P. Stewart, O.V. Aslanidi, D. Noble, P.J. Noble, M.R. Boyett,
 * H. Zhang, "Mathematical models of the electrical action potential of
 * Purkinje fibre cells", Phil Trans R Soc A 367 (2009) 2225-2255.  It is the
 * ten Tusscher-Panfilov 2006 formulation with Purkinje conductances, a
 * hyperpolarisation-activated current I_f (gate y), a sustained potassium
 * current I_sus and modified I_to kinetics.  The paper uses it for the
 * Purkinje network (Sec. 3.1) with 13 gating variables out of 20 states
 * (Sec. 3.2): the 12 gates it shares with the ventricular model plus y.
 * The RyR recovery variable Rbar is therefore forward-Euler integrated here.
 *
 * Slot order: 0 V, 1 m, 2 h, 3 j, 4 xr1, 5 xr2, 6 xs, 7 r, 8 s, 9 d, 10 f,
 * 11 f2, 12 fCass, 13 y, 14 Rbar, 15 Ca_i, 16 Ca_SR, 17 Ca_SS, 18 Na_i,
 * 19 K_i.  Units: mV, ms, mM, pA/pF.
 */
#include <math.h>
#include <stddef.h>
#include "orc_models.h"

static const double R_GAS = 8314.472, T_K = 310.0, F_C = 96485.3415;
static const double CAP = 0.185, V_C = 0.016404, V_SR = 0.001094;
static const double V_SS = 0.00005468;
static const double K_O = 5.4, NA_O = 140.0, CA_O = 2.0;
static const double G_NA = 130.5744, G_K1 = 0.065, G_KR = 0.0918;
static const double G_KS = 0.2352, G_TO = 0.08184, G_SUS = 0.0227;
static const double G_FNA = 0.0145654, G_FK = 0.0234346;
static const double P_KNA = 0.03, G_CAL = 3.980e-5;
static const double K_NACA = 1000.0, GAMMA_NACA = 0.35, KM_CA = 1.38;
static const double KM_NAI = 87.5, K_SAT = 0.1, ALPHA_NACA = 2.5;
static const double P_NAK = 2.724, KM_K = 1.0, KM_NA = 40.0;
static const double G_PK = 0.0146, G_PCA = 0.1238, K_PCA = 0.0005;
static const double G_BNA = 0.00029, G_BCA = 0.000592;
static const double VMAX_UP = 0.006375, K_UP = 0.00025, V_REL = 0.102;
static const double K1P = 0.15, K2P = 0.045, K3 = 0.060, K4 = 0.005;
static const double EC = 1.5, MAX_SR = 2.5, MIN_SR = 1.0;
static const double V_LEAK = 0.00036, V_XFER = 0.0038;
static const double BUF_C = 0.2, K_BUFC = 0.001;
static const double BUF_SR = 10.0, K_BUFSR = 0.3;
static const double BUF_SS = 0.4, K_BUFSS = 0.00025;

static const char *const SLOT_NAMES[20] = {
    "V", "m", "h", "j", "xr1", "xr2", "xs", "r", "s", "d", "f", "f2",
    "fCass", "y", "Rbar", "Ca_i", "Ca_SR", "Ca_SS", "Na_i", "K_i"};

const char *orc_stewart_slot_name(int slot)
{
    return (slot >= 0 && slot < 20) ? SLOT_NAMES[slot] : NULL;
}

void orc_stewart_init(double *y)
{
    /* initial values listed in the article */
    y[0] = -69.1865;
    y[1] = 0.0417391; y[2] = 0.190678; y[3] = 0.238219;
    y[4] = 0.00550281; y[5] = 0.313298; y[6] = 0.00953708;
    y[7] = 0.00103693; y[8] = 0.96369; y[9] = 0.000287906;
    y[10] = 0.989361; y[11] = 0.995179; y[12] = 0.999656;
    y[13] = 0.0457562; y[14] = 0.991656; y[15] = 0.000101878;
    y[16] = 3.10836; y[17] = 0.000446818; y[18] = 8.80474; y[19] = 136.7809;
}

static double rush_larsen(double y, double yinf, double tau, double dt)
{
    return yinf + (y - yinf) * exp(-dt / tau);
}

static double free_from_total(double total, double B, double K)
{
    double b = B + K - total;
    double disc = sqrt(b * b + 4.0 * K * total);
    return (b >= 0.0) ? (2.0 * K * total) / (disc + b) : 0.5 * (disc - b);
}

static double total_from_free(double c, double B, double K)
{
    return c + B * c / (c + K);
}

double orc_stewart_step(double *y, double dt, double istim, const double *gs,
                        orc_hist *hist, const orc_mid *mid)
{
    const double V = y[0];
    double m = y[1], h = y[2], j = y[3], xr1 = y[4], xr2 = y[5], xs = y[6];
    double r = y[7], s = y[8], d = y[9], f = y[10], f2 = y[11];
    double fcass = y[12], yf = y[13], rbar = y[14];
    double cai = y[15], casr = y[16], cass = y[17], nai = y[18], ki = y[19];
    const double sKr = gs ? gs[0] : 1.0, sKs = gs ? gs[1] : 1.0;
    const double sCaL = gs ? gs[2] : 1.0, sNa = gs ? gs[3] : 1.0;
    const double RTF = R_GAS * T_K / F_C;

    const double E_Na = RTF * log(NA_O / nai);
    const double E_K = RTF * log(K_O / ki);
    const double E_Ca = 0.5 * RTF * log(CA_O / cai);
    const double E_Ks = RTF * log((K_O + P_KNA * NA_O) / (ki + P_KNA * nai));

    const double I_Na = sNa * G_NA * m * m * m * h * j * (V - E_Na);
    const double x = 2.0 * (V - 15.0) / RTF;
    const double ghk = (fabs(x) < 1e-12) ? 1.0 : x / expm1(x);
    const double I_CaL = sCaL * G_CAL * d * f * f2 * fcass * 2.0 * F_C * ghk *
                         (0.25 * cass * exp(x) - CA_O);
    const double I_to = G_TO * r * s * (V - E_K);
    const double a_sus = 1.0 / (1.0 + exp((5.0 - V) / 17.0));
    const double I_sus = G_SUS * a_sus * (V - E_K);
    const double I_Ks = sKs * G_KS * xs * xs * (V - E_Ks);
    const double I_Kr = sKr * G_KR * sqrt(K_O / 5.4) * xr1 * xr2 * (V - E_K);
    const double a_K1 = 0.1 / (1.0 + exp(0.06 * (V - E_K - 200.0)));
    const double b_K1 = (3.0 * exp(0.0002 * (V - E_K + 100.0)) +
                         exp(0.1 * (V - E_K - 10.0))) /
                        (1.0 + exp(-0.5 * (V - E_K)));
    const double I_K1 = G_K1 * sqrt(K_O / 5.4) * (a_K1 / (a_K1 + b_K1)) * (V - E_K);
    const double I_fNa = G_FNA * yf * (V - E_Na);
    const double I_fK = G_FK * yf * (V - E_K);
    const double e_g = exp(GAMMA_NACA * V / RTF);
    const double e_g1 = exp((GAMMA_NACA - 1.0) * V / RTF);
    const double I_NaCa =
        K_NACA * (e_g * nai * nai * nai * CA_O -
                  e_g1 * NA_O * NA_O * NA_O * cai * ALPHA_NACA) /
        ((KM_NAI * KM_NAI * KM_NAI + NA_O * NA_O * NA_O) * (KM_CA + CA_O) *
         (1.0 + K_SAT * e_g1));
    const double I_NaK =
        P_NAK * K_O * nai /
        ((K_O + KM_K) * (nai + KM_NA) *
         (1.0 + 0.1245 * exp(-0.1 * V / RTF) + 0.0353 * exp(-V / RTF)));
    const double I_pCa = G_PCA * cai / (K_PCA + cai);
    const double I_pK = G_PK * (V - E_K) / (1.0 + exp((25.0 - V) / 5.98));
    const double I_bNa = G_BNA * (V - E_Na);
    const double I_bCa = G_BCA * (V - E_Ca);
    const double I_ion = I_Na + I_K1 + I_to + I_sus + I_Kr + I_Ks + I_CaL +
                         I_NaCa + I_NaK + I_pCa + I_pK + I_bNa + I_bCa +
                         I_fNa + I_fK;

    const double kcasr = MAX_SR - (MAX_SR - MIN_SR) / (1.0 + (EC / casr) * (EC / casr));
    const double k1 = K1P / kcasr;
    const double k2 = K2P * kcasr;
    const double O = k1 * cass * cass * rbar / (K3 + k1 * cass * cass);
    const double I_rel = V_REL * O * (casr - cass);
    const double I_up = VMAX_UP / (1.0 + (K_UP * K_UP) / (cai * cai));
    const double I_leak = V_LEAK * (casr - cai);
    const double I_xfer = V_XFER * (cass - cai);
    const double dRbar = -k2 * cass * rbar + K4 * (1.0 - rbar);

    const double dCaiT = -(I_bCa + I_pCa - 2.0 * I_NaCa) * CAP / (2.0 * V_C * F_C) +
                         (I_leak - I_up) * V_SR / V_C + I_xfer;
    const double dCasrT = I_up - I_rel - I_leak;
    const double dCassT = -I_CaL * CAP / (2.0 * V_SS * F_C) +
                          I_rel * V_SR / V_SS - I_xfer * V_C / V_SS;
    const double dNai = -(I_Na + I_bNa + I_fNa + 3.0 * I_NaK + 3.0 * I_NaCa) *
                        CAP / (V_C * F_C);
    const double dKi = -(I_K1 + I_to + I_sus + I_fK + I_Kr + I_Ks - 2.0 * I_NaK +
                         I_pK + istim) * CAP / (V_C * F_C);

    /* gates at level n, or at the midpoint predictions of V and Ca_SS
     * (second-order variant) */
    const double Vg = mid ? V + 0.5 * dt * (mid->lmi - I_ion) : V;
    const double cass_g = mid ? free_from_total(total_from_free(cass, BUF_SS, K_BUFSS) +
                                                    0.5 * dt * dCassT, BUF_SS, K_BUFSS)
                              : cass;
    {
    const double V = Vg, cass = cass_g;
    double yinf, tau, a, b, c;
    yinf = 1.0 / ((1.0 + exp((-56.86 - V) / 9.03)) * (1.0 + exp((-56.86 - V) / 9.03)));
    a = 1.0 / (1.0 + exp((-60.0 - V) / 5.0));
    b = 0.1 / (1.0 + exp((V + 35.0) / 5.0)) + 0.10 / (1.0 + exp((V - 50.0) / 200.0));
    m = rush_larsen(m, yinf, a * b, dt);
    yinf = 1.0 / ((1.0 + exp((V + 71.55) / 7.43)) * (1.0 + exp((V + 71.55) / 7.43)));
    if (V >= -40.0) {
        a = 0.0;
        b = 0.77 / (0.13 * (1.0 + exp(-(V + 10.66) / 11.1)));
    } else {
        a = 0.057 * exp(-(V + 80.0) / 6.8);
        b = 2.7 * exp(0.079 * V) + 3.1e5 * exp(0.3485 * V);
    }
    h = rush_larsen(h, yinf, 1.0 / (a + b), dt);
    if (V >= -40.0) {
        a = 0.0;
        b = 0.6 * exp(0.057 * V) / (1.0 + exp(-0.1 * (V + 32.0)));
    } else {
        a = (-2.5428e4 * exp(0.2444 * V) - 6.948e-6 * exp(-0.04391 * V)) *
            (V + 37.78) / (1.0 + exp(0.311 * (V + 79.23)));
        b = 0.02424 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14)));
    }
    j = rush_larsen(j, yinf, 1.0 / (a + b), dt);
    yinf = 1.0 / (1.0 + exp((-26.0 - V) / 7.0));
    a = 450.0 / (1.0 + exp((-45.0 - V) / 10.0));
    b = 6.0 / (1.0 + exp((V + 30.0) / 11.5));
    xr1 = rush_larsen(xr1, yinf, a * b, dt);
    yinf = 1.0 / (1.0 + exp((V + 88.0) / 24.0));
    a = 3.0 / (1.0 + exp((-60.0 - V) / 20.0));
    b = 1.12 / (1.0 + exp((V - 60.0) / 20.0));
    xr2 = rush_larsen(xr2, yinf, a * b, dt);
    yinf = 1.0 / (1.0 + exp((-5.0 - V) / 14.0));
    a = 1400.0 / sqrt(1.0 + exp((5.0 - V) / 6.0));
    b = 1.0 / (1.0 + exp((V - 35.0) / 15.0));
    xs = rush_larsen(xs, yinf, a * b + 80.0, dt);
    /* I_to gates with the Purkinje kinetics */
    yinf = 1.0 / (1.0 + exp((20.0 - V) / 13.0));
    tau = 10.45 * exp(-(V + 40.0) * (V + 40.0) / 1800.0) + 7.3;
    r = rush_larsen(r, yinf, tau, dt);
    yinf = 1.0 / (1.0 + exp((V + 27.0) / 13.0));
    tau = 85.0 * exp(-(V + 25.0) * (V + 25.0) / 320.0) +
          5.0 / (1.0 + exp((V - 40.0) / 5.0)) + 42.0;
    s = rush_larsen(s, yinf, tau, dt);
    yinf = 1.0 / (1.0 + exp((-8.0 - V) / 7.5));
    a = 1.4 / (1.0 + exp((-35.0 - V) / 13.0)) + 0.25;
    b = 1.4 / (1.0 + exp((V + 5.0) / 5.0));
    c = 1.0 / (1.0 + exp((50.0 - V) / 20.0));
    d = rush_larsen(d, yinf, a * b + c, dt);
    yinf = 1.0 / (1.0 + exp((V + 20.0) / 7.0));
    a = 1102.5 * exp(-(V + 27.0) * (V + 27.0) / 225.0);
    b = 200.0 / (1.0 + exp((13.0 - V) / 10.0));
    c = 180.0 / (1.0 + exp((V + 30.0) / 10.0)) + 20.0;
    f = rush_larsen(f, yinf, a + b + c, dt);
    yinf = 0.67 / (1.0 + exp((V + 35.0) / 7.0)) + 0.33;
    a = 600.0 * exp(-(V + 25.0) * (V + 25.0) / 170.0);
    b = 31.0 / (1.0 + exp((25.0 - V) / 10.0));
    c = 16.0 / (1.0 + exp((V + 30.0) / 10.0));
    f2 = rush_larsen(f2, yinf, a + b + c, dt);
    {
        const double q = (cass / 0.05) * (cass / 0.05);
        fcass = rush_larsen(fcass, 0.6 / (1.0 + q) + 0.4, 80.0 / (1.0 + q) + 2.0, dt);
    }
    /* I_f gate */
    yinf = 1.0 / (1.0 + exp((V + 80.6) / 6.8));
    a = exp(-2.9 - 0.04 * V);
    b = exp(3.6 + 0.11 * V);
    yf = rush_larsen(yf, yinf, 4000.0 / (a + b), dt);
    }

    rbar += dt * orc_rate(hist, 0, dRbar);
    cai = free_from_total(total_from_free(cai, BUF_C, K_BUFC) + dt * orc_rate(hist, 1, dCaiT),
                          BUF_C, K_BUFC);
    casr = free_from_total(total_from_free(casr, BUF_SR, K_BUFSR) + dt * orc_rate(hist, 2, dCasrT),
                           BUF_SR, K_BUFSR);
    cass = free_from_total(total_from_free(cass, BUF_SS, K_BUFSS) + dt * orc_rate(hist, 3, dCassT),
                           BUF_SS, K_BUFSS);
    nai += dt * orc_rate(hist, 4, dNai);
    ki += dt * orc_rate(hist, 5, dKi);

    y[1] = m; y[2] = h; y[3] = j; y[4] = xr1; y[5] = xr2; y[6] = xs;
    y[7] = r; y[8] = s; y[9] = d; y[10] = f; y[11] = f2; y[12] = fcass;
    y[13] = yf; y[14] = rbar; y[15] = cai; y[16] = casr; y[17] = cass;
    y[18] = nai; y[19] = ki;
    return I_ion;
}
