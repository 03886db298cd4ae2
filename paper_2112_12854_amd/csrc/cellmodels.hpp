// Cell models of the monodomain step as device functions.
//
// Each model advances one cell by one step dt with every right-hand side
// taken at level n (Sec. 3.2 of the paper): gating variables by Rush-Larsen,
// the other states by forward Euler.  The function returns I_ion(t^n) in
// pA/pF; the caller forms v^{n+1} = v^n + dt (L - I_ion - I_stim).
//
// Precision policy R is the type of V, gates, currents and their kinetics
// (double for the FP64 path, float for the mixed path).  Intracellular
// concentrations, their rates and the rapid-buffering solves are always
// FP64: they integrate small increments over hundreds of thousands of steps.
//
// Rush-Larsen is written as y += (y_inf - y) * (-expm1(-dt k)), k = 1/tau,
// in FP32, which keeps the per-step increment of slow gates accurate where
// exp(-dt/tau) would round to 1; FP64 uses y_inf + (y - y_inf) exp(-dt k).
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace epdev {

struct GScale {
    double kr, ks, cal, na;  // multipliers of G_Kr, G_Ks, G_CaL, G_Na
};

// --------------------------------------------------------------- helpers
// FP64: exp64 and log64 below and the library expm1 and sqrt (within an
// ulp), and the refined reciprocal below (within an ulp).  FP32 (the
// mixed path, whose bar is activation time and APD90): the hardware exp2 / log2 /
// reciprocal instructions, a few ulp each, which cuts the instruction count
// of the cell kernel by about a fifth.

// e^x in FP64, within about an ulp for |x| < 700 (the model's arguments are
// voltages over a few mV, tens at most).  Cody and Waite's reduction
// x = n ln2 + r, |r| <= ln2 / 2, with ln2 split into a 53-bit head (so that
// the first fused multiply-add is exact) and its tail; e^r from the degree-11
// Chebyshev fit of e^r on |r| <= ln2 / 2 (truncation error 3.2e-18, well
// under the rounding of its Horner evaluation), coefficients rounded to
// FP64; then the scaling by 2^n, whose saturation gives inf and 0 (through
// the subnormals) at the ends of the range.  The library exp adds range
// tests with three selects around the same steps: 17 instructions here
// against 25.  NaN stays NaN; arguments beyond about 1e9 in size are
// outside its domain.
__host__ __device__ inline double exp64(double x) {
    const double n = rint(x * 0x1.71547652b82fep+0);          // x / ln2
    double r = fma(-n, 0x1.62e42fefa39efp-1, x);              // ln2 head
    r = fma(-n, 0x1.abc9e3b39803fp-56, r);                    // ln2 tail
    double p = 0x1.af631d00624dap-26;
    p = fma(p, r, 0x1.28b4057f4b090p-22);
    p = fma(p, r, 0x1.71ddf5749d0dcp-19);
    p = fma(p, r, 0x1.a01991ac87291p-16);
    p = fma(p, r, 0x1.a01a01b14378fp-13);
    p = fma(p, r, 0x1.6c16c187fbe02p-10);
    p = fma(p, r, 0x1.111111110f225p-7);
    p = fma(p, r, 0x1.555555554f0cfp-5);
    p = fma(p, r, 0x1.555555555555ap-3);
    p = fma(p, r, 0x1.0000000000011p-1);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}

// ln x in FP64 for positive finite x (NaN for 0, negative, infinite or NaN
// x; the models take it of concentrations), within an ulp.
// x = 2^k m with m in [sqrt(1/2), sqrt(2)), u = m - 1 (exact); ln m =
// 2 atanh f with f = u / (2 + u), |f| <= 0.1716, and 2 atanh f = 2f + f z Q(z),
// z = f^2, where Q is the degree-6 Chebyshev fit of
// 2 (atanh(sqrt z) / sqrt z - 1) / z on [0, 0.0295] (its share of the
// relative error of ln m is 5e-18).  Since 2f = u - f u, ln m = u - f (u - z Q):
// u carries no rounding and f's rounding enters only the correction, at most
// a fifth of u.  k ln2 is added with ln2 split into a 42-bit head, whose
// product with k is exact, and a tail that joins the correction.  About 30
// instructions, against about 90 for the library log, which carries a
// double-double evaluation.
__host__ __device__ inline double log64(double x) {
    int k;
    double m = frexp(x, &k);                            // x = m 2^k, m in [1/2, 1)
    if (m < 0x1.6a09e667f3bcdp-1) { m += m; --k; }      // m in [sqrt(1/2), sqrt(2))
    const double u = m - 1.0;
    const double f = u / (2.0 + u);
    const double z = f * f;
    double q = 0x1.2b584aaef00b2p-3;
    q = fma(q, z, 0x1.39fe606539350p-3);
    q = fma(q, z, 0x1.7462b4ab2f411p-3);
    q = fma(q, z, 0x1.c71c62e580090p-3);
    q = fma(q, z, 0x1.2492492df148dp-2);
    q = fma(q, z, 0x1.99999999952e2p-2);
    q = fma(q, z, 0x1.5555555555558p-1);
    const double kd = (double)k;
    // ln m + k ln2 tail = u - (f (u - z Q) - k ln2 tail), then + k ln2 head
    const double c = fma(f, fma(-z, q, u), -kd * 0x1.ef35793c76730p-45);
    const double r = fma(kd, 0x1.62e42fefa3800p-1, u - c);
    return (x > 0.0 && x < HUGE_VAL) ? r : __builtin_nan("");
}

__device__ __forceinline__ double xexp(double x) { return exp64(x); }
__device__ __forceinline__ float xexp(float x) { return __expf(x); }
__device__ __forceinline__ double xexpm1(double x) { return expm1(x); }
// e^x - 1 in FP32: below |x| = 1/8 the Taylor series to x^5 (relative
// truncation error under |x|^5/720 < 5e-8), else e^x - 1, whose rounding is
// small next to |e^x - 1| >= 0.117 there.
__device__ __forceinline__ float xexpm1(float x) {
    const float p = x * (1.0f + x * (0.5f + x * (1.0f / 6.0f + x * (1.0f / 24.0f + x * (1.0f / 120.0f)))));
    return fabsf(x) < 0.125f ? p : __expf(x) - 1.0f;
}
__device__ __forceinline__ double xlog(double x) { return log64(x); }
__device__ __forceinline__ float xlog(float x) { return __logf(x); }
__device__ __forceinline__ double xsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float xsqrt(float x) { return sqrtf(x); }
// FP64 reciprocal: the hardware estimate r0 (relative error e = 1 - x r0
// below 2^-22) refined by one third-order step r = r0 (1 + e + e^2), which
// takes the error to e^3 < 2^-66, so that the result is within an ulp of 1/x
// (the last fused multiply-add's rounding): four instructions, against
// about ten for the IEEE division.  x = 0 and x = +-inf give NaN (the step
// forms 0 * inf); every argument here is finite and nonzero (1 + e^z for
// bounded z, e^{V/k}, sums of positive concentrations), and a cell whose
// voltage leaves the range where that holds is reported by the step's
// finiteness check of V.
__device__ __forceinline__ double xrcp(double x) {
    const double r0 = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r0, 1.0);
    return fma(r0, fma(e, e, e), r0);
}
__device__ __forceinline__ float xrcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double xpow15(double x) { return pow(x, 1.5); }
__device__ __forceinline__ float xpow15(float x) { return x * sqrtf(x); }
__device__ __forceinline__ double xdiv(double a, double b) { return a * xrcp(b); }
__device__ __forceinline__ float xdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// ln(a / b) for a constant a (Nernst potentials): in FP64 ln a (folded at
// compile time) - ln b, which saves the division.
template <typename R> __device__ __forceinline__ R lnratio(double a, double b) {
    return xlog(xdiv(R(a), R(b)));
}
template <> __device__ __forceinline__ double lnratio(double a, double b) {
    return __builtin_log(a) - log64(b);
}

// logistic 1 / (1 + e^z).  In FP64 z is capped at 708 so that e^z stays
// finite for xrcp (the result there is below 1e-307 either way): the
// calcium-release gates of the CRN model scale a small flux by 1/1.367e-15,
// and their z passes 709 whenever that flux is slightly negative.
template <typename R> __device__ __forceinline__ R sig(R z) { return xrcp(R(1) + xexp(z)); }
template <> __device__ __forceinline__ double sig(double z) { return xrcp(1.0 + xexp(fmin(z, 708.0))); }

// Logistic terms of one voltage scale k from a single exponential:
// e^{(a - V)/k} = e^{a/k} e^{-V/k} and e^{(V - b)/k} = e^{-b/k} e^{V/k},
// the constant factors folded at compile time, so every gate term with the
// same k costs a multiply and a reciprocal instead of an exponential.
template <typename R> struct Vscale {
    R p, n;    // e^{V/k}, e^{-V/k}
    __device__ __forceinline__ Vscale(R V, double k) : p(xexp(V * R(1.0 / k))), n(xrcp(p)) {}
    // e^{(a - V)/k} and the logistic 1 / (1 + e^{(a - V)/k})
    __device__ __forceinline__ R edown(double a, double k) const { return R(__builtin_exp(a / k)) * n; }
    __device__ __forceinline__ R down(double a, double k) const { return xrcp(R(1) + edown(a, k)); }
    // 1 / (1 + e^{(V - b)/k})
    __device__ __forceinline__ R up(double b, double k) const {
        return xrcp(R(1) + R(__builtin_exp(-b / k)) * p);
    }
};

// Rush-Larsen with rate k = 1/tau
template <typename R>
__device__ __forceinline__ R rl(R y, R yinf, R k, R dt) {
    return y + (yinf - y) * (-xexpm1(-dt * k));
}
// FP64 has the digits for the plain form, and exp is cheaper than expm1
template <>
__device__ __forceinline__ double rl(double y, double yinf, double k, double dt) {
    return yinf + (y - yinf) * exp64(-dt * k);
}

// z / (e^z - 1), continuous at 0
template <typename R>
__device__ __forceinline__ R z_expm1(R z) {
    R e = xexpm1(z);
    return (fabs(z) < R(1e-6)) ? R(1) - R(0.5) * z : xdiv(z, e);
}

// Free concentration under one rapid buffer (capacity B, constant K) that
// carries the total T: positive root of c^2 + (B + K - T) c - K T = 0,
// evaluated in the form without cancellation.
__device__ __forceinline__ double buffered_free(double T, double B, double K) {
    const double b = B + K - T;
    const double q = sqrt(b * b + 4.0 * K * T);
    return b >= 0.0 ? xdiv(2.0 * K * T, q + b) : 0.5 * (q - b);
}
__device__ __forceinline__ double buffered_total(double c, double B, double K) {
    return c * (1.0 + xdiv(B, c + K));
}

// Rate of a non-gating state (concentrations; Stewart's Rbar) under the time
// scheme: forward Euler uses the rate of step n; Adams-Bashforth 2 uses
// 3/2 r^n - 1/2 r^{n-1}, h[k] holding r^{n-1} (forward Euler on the first
// step) and receiving r^n.
struct FwdEuler {
    __device__ __forceinline__ double operator()(double r, int) const { return r; }
};
struct AdamsBashforth2 {
    double *h;
    bool first;
    __device__ __forceinline__ double operator()(double r, int k) const {
        const double p = first ? r : h[k];
        h[k] = r;
        return 1.5 * r - 0.5 * p;
    }
};

// ===================================================================== TP06
// ten Tusscher & Panfilov, Am J Physiol Heart Circ Physiol 291:H1088 (2006),
// currents shared with ten Tusscher, Noble, Noble & Panfilov, AJP 286:H1573
// (2004).  Gates (13, Rush-Larsen): m h j xr1 xr2 xs r s d f f2 fCass Rbar.
// Concentrations (FP64, forward Euler): Ca_i Ca_SR Ca_SS Na_i K_i, the
// buffered ones advanced on their totals.  type: 0 endo, 1 M, 2 epi.
namespace tp06 {
constexpr int NG = 13, NC = 5;
constexpr double RTF = 8314.472 * 310.0 / 96485.3415;   // mV
constexpr double FARADAY = 96485.3415;
constexpr double KO = 5.4, NAO = 140.0, CAO = 2.0;
constexpr double CAP = 0.185, VC = 0.016404, VSR = 0.001094, VSS = 0.00005468;
constexpr double INV_VCF = CAP / (VC * FARADAY);          // mM/ms per pA/pF
constexpr double INV_2VCF = CAP / (2.0 * VC * FARADAY);
constexpr double INV_2VSSF = CAP / (2.0 * VSS * FARADAY);
constexpr double SQRT_KO = 1.0;                           // sqrt(KO / 5.4)

__host__ __device__ inline void init(double *y) {
    // V, m h j xr1 xr2 xs r s d f f2 fCass Rbar, Ca_i Ca_SR Ca_SS Na_i K_i
    const double s[19] = {-86.2, 0.0, 0.75, 0.75, 0.0, 1.0, 0.0, 0.0, 1.0,
                          0.0, 1.0, 1.0, 1.0, 1.0, 7e-5, 1.3, 7e-5, 7.67, 138.3};
    for (int i = 0; i < 19; ++i) y[i] = s[i];
}

template <typename R, bool RL2 = false, typename E = FwdEuler>
__device__ __forceinline__ R step(int type, R V, R *g, double *c, R dt,
                                  double dtd, R istim, const GScale &gs, const E &e = E(),
                                  R lmi = R(0)) {
    const R frt = R(1.0 / RTF);
    const double cai = c[0], casr = c[1], cass = c[2], nai = c[3], ki = c[4];
    const R rtf = R(RTF);
    const R ENa = rtf * lnratio<R>(NAO, nai);
    const R EK = rtf * lnratio<R>(KO, ki);
    const R ECa = R(0.5) * rtf * lnratio<R>(CAO, cai);
    const R EKs = rtf * lnratio<R>(KO + 0.03 * NAO, ki + 0.03 * nai);
    const R m = g[0], h = g[1], j = g[2], xr1 = g[3], xr2 = g[4], xs = g[5];
    const R r = g[6], s = g[7], d = g[8], f = g[9], f2 = g[10], fcass = g[11];
    const R rbar = g[12];
    const bool endo = (type == 0);
    const R Gto = endo ? R(0.073) : R(0.294);
    const R Gks = (type == 1) ? R(0.098) : R(0.392);

    // ---- currents at level n (pA/pF)
    const R INa = R(gs.na) * R(14.838) * m * m * m * h * j * (V - ENa);
    const R xca = R(2) * (V - R(15)) * frt;
    const R emx = xexpm1(xca);
    const R ghk = (fabs(xca) < R(1e-6)) ? R(1) - R(0.5) * xca : xdiv(xca, emx);
    const R ICaL = R(gs.cal) * R(3.980e-5 * 2.0 * FARADAY) * d * f * f2 * fcass * ghk *
                   (R(0.25) * R(cass) * (emx + R(1)) - R(CAO));
    const R dK = V - EK;
    const R Ito = Gto * r * s * dK;
    const R IKs = R(gs.ks) * Gks * xs * xs * (V - EKs);
    const R IKr = R(gs.kr) * R(0.153 * SQRT_KO) * xr1 * xr2 * dK;
    const R aK1 = R(0.1) * sig(R(0.06) * (dK - R(200)));
    const R bK1 = (R(3) * xexp(R(0.0002) * (dK + R(100))) + xexp(R(0.1) * (dK - R(10)))) *
                  sig(R(-0.5) * dK);
    const R IK1 = R(5.405 * SQRT_KO) * xdiv(aK1, aK1 + bK1) * dK;
    const R ev = xexp(-V * frt);                  // e^{-VF/RT}
    const R eg = xexp(R(0.35) * V * frt);         // e^{gamma VF/RT}
    const R eg1 = eg * ev;                        // e^{(gamma-1)VF/RT}
    const R nai3 = R(nai) * R(nai) * R(nai);
    const R INaCa = R(1000.0 / ((87.5 * 87.5 * 87.5 + NAO * NAO * NAO) * (1.38 + CAO))) *
                    xdiv(eg * nai3 * R(CAO) - eg1 * R(NAO * NAO * NAO * 2.5) * R(cai),
                         R(1) + R(0.1) * eg1);
    const R INaK = R(2.724 * KO / (KO + 1.0)) *
                   xdiv(R(nai), (R(nai) + R(40)) *
                                    (R(1) + R(0.1245) * xexp(R(-0.1) * V * frt) + R(0.0353) * ev));
    const R IpCa = R(0.1238) * xdiv(R(cai), R(0.0005) + R(cai));
    const R IpK = R(0.0146) * dK * sig((R(25) - V) * R(1.0 / 5.98));
    const R IbNa = R(0.00029) * (V - ENa);
    const R IbCa = R(0.000592) * (V - ECa);
    const R Iion = INa + IK1 + Ito + IKr + IKs + ICaL + INaCa + INaK + IpCa + IpK +
                   IbNa + IbCa;

    // ---- calcium handling at level n (FP64)
    const double ec = xdiv(1.5, casr);
    const double kcasr = 2.5 - xdiv(1.5, 1.0 + ec * ec);
    const double k1 = xdiv(0.15, kcasr), k2 = 0.045 * kcasr;
    const double cass2 = cass * cass;
    const double Irel = 0.102 * xdiv(k1 * cass2 * double(rbar), 0.060 + k1 * cass2) * (casr - cass);
    const double Iup = xdiv(0.006375, 1.0 + xdiv(0.00025 * 0.00025, cai * cai));
    const double Ileak = 0.00036 * (casr - cai);
    const double Ixfer = 0.0038 * (cass - cai);
    const double rCai = -double(IbCa + IpCa - R(2) * INaCa) * INV_2VCF +
                        (Ileak - Iup) * (VSR / VC) + Ixfer;
    const double rCasr = Iup - Irel - Ileak;
    const double rCass = -double(ICaL) * INV_2VSSF + Irel * (VSR / VSS) - Ixfer * (VC / VSS);
    const double rNai = -double(INa + IbNa + R(3) * (INaK + INaCa)) * INV_VCF;
    const double rKi = -double(IK1 + Ito + IKr + IKs - R(2) * INaK + IpK + istim) * INV_VCF;

    // ---- gates: Rush-Larsen at level n, or (second-order variant) with
    // their rates at the midpoint predictions of V, Ca_SS and Ca_SR
    R Vg = V;
    double cass_g = cass, k2g = k2;
    if constexpr (RL2) {
        Vg = V + R(0.5) * dt * (lmi - Iion);
        cass_g = buffered_free(buffered_total(cass, 0.4, 0.00025) + 0.5 * dtd * rCass, 0.4, 0.00025);
        const double casr_g = buffered_free(buffered_total(casr, 10.0, 0.3) + 0.5 * dtd * rCasr,
                                            10.0, 0.3);
        const double ecg = xdiv(1.5, casr_g);
        k2g = 0.045 * (2.5 - xdiv(1.5, 1.0 + ecg * ecg));
    }
    {
    const R V = Vg;
    const double cass = cass_g, k2 = k2g;
    // the voltage scales shared by several gate terms
    const Vscale<R> e5(V, 5.0), e6(V, 6.0), e7(V, 7.0), e10(V, 10.0), e20(V, 20.0);
    {   // m
        const R s1 = sig((R(-56.86) - V) * R(1.0 / 9.03));
        const R am = e5.down(-60.0, 5.0);
        const R bm = R(0.1) * e5.up(-35.0, 5.0) + R(0.1) * sig((V - R(50)) * R(0.005));
        g[0] = rl(m, s1 * s1, xrcp(am * bm), dt);
    }
    {   // h, j share the steady state
        const R s1 = sig((V + R(71.55)) * R(1.0 / 7.43));
        const R inf = s1 * s1;
        R kh, kj;
        if (V >= R(-40)) {
            kh = R(0.13 / 0.77) * (R(1) + xexp((V + R(10.66)) * R(-1.0 / 11.1)));
            kh = xrcp(kh);
            kj = R(0.6) * xexp(R(0.057) * V) * e10.down(-32.0, 10.0);
        } else {
            kh = R(0.057) * xexp((V + R(80)) * R(-1.0 / 6.8)) + R(2.7) * xexp(R(0.079) * V) +
                 R(3.1e5) * xexp(R(0.3485) * V);
            kj = (R(-2.5428e4) * xexp(R(0.2444) * V) - R(6.948e-6) * xexp(R(-0.04391) * V)) *
                     (V + R(37.78)) * sig(R(0.311) * (V + R(79.23))) +
                 R(0.02424) * xexp(R(-0.01052) * V) * sig(R(-0.1378) * (V + R(40.14)));
        }
        g[1] = rl(h, inf, kh, dt);
        g[2] = rl(j, inf, kj, dt);
    }
    {   // xr1
        const R a = R(450) * e10.down(-45.0, 10.0);
        const R b = R(6) * sig((V + R(30)) * R(1.0 / 11.5));
        g[3] = rl(xr1, e7.down(-26.0, 7.0), xrcp(a * b), dt);
    }
    {   // xr2
        const R a = R(3) * e20.down(-60.0, 20.0);
        const R b = R(1.12) * e20.up(60.0, 20.0);
        g[4] = rl(xr2, sig((V + R(88)) * R(1.0 / 24.0)), xrcp(a * b), dt);
    }
    {   // xs
        const R a = xdiv(R(1400), xsqrt(R(1) + e6.edown(5.0, 6.0)));
        const R b = sig((V - R(35)) * R(1.0 / 15.0));
        g[5] = rl(xs, sig((R(-5) - V) * R(1.0 / 14.0)), xrcp(a * b + R(80)), dt);
    }
    {   // r
        const R t = R(9.5) * xexp(-(V + R(40)) * (V + R(40)) * R(1.0 / 1800.0)) + R(0.8);
        g[6] = rl(r, e6.down(20.0, 6.0), xrcp(t), dt);
    }
    {   // s (endocardial cells have their own inactivation kinetics)
        R inf, t;
        if (endo) {
            inf = e5.up(-28.0, 5.0);
            t = R(1000) * xexp(-(V + R(67)) * (V + R(67)) * R(0.001)) + R(8);
        } else {
            inf = e5.up(-20.0, 5.0);
            t = R(85) * xexp(-(V + R(45)) * (V + R(45)) * R(1.0 / 320.0)) +
                R(5) * e5.up(20.0, 5.0) + R(3);
        }
        g[7] = rl(s, inf, xrcp(t), dt);
    }
    {   // d
        const R a = R(1.4) * sig((R(-35) - V) * R(1.0 / 13.0)) + R(0.25);
        const R b = R(1.4) * e5.up(-5.0, 5.0);
        const R cc = e20.down(50.0, 20.0);
        g[8] = rl(d, sig((R(-8) - V) * R(1.0 / 7.5)), xrcp(a * b + cc), dt);
    }
    const R up30 = e10.up(-30.0, 10.0);      // shared by f and f2
    {   // f
        const R t = R(1102.5) * xexp(-(V + R(27)) * (V + R(27)) * R(1.0 / 225.0)) +
                    R(200) * e10.down(13.0, 10.0) + R(180) * up30 + R(20);
        g[9] = rl(f, e7.up(-20.0, 7.0), xrcp(t), dt);
    }
    {   // f2 (time constant as printed in the 2006 article)
        const R t = R(562) * xexp(-(V + R(27)) * (V + R(27)) * R(1.0 / 240.0)) +
                    R(31) * e10.down(25.0, 10.0) + R(80) * up30;
        g[10] = rl(f2, R(0.67) * e7.up(-35.0, 7.0) + R(0.33), xrcp(t), dt);
    }
    {   // fCass, driven by Ca_SS^n
        const R q = R(cass * 400.0 * cass);     // (Ca_SS / 0.05)^2
        const R w = xrcp(R(1) + q);
        g[11] = rl(fcass, R(0.6) * w + R(0.4), xrcp(R(80) * w + R(2)), dt);
    }
    {   // Rbar: dR/dt = k4 (1 - R) - k2 Ca_SS R  (linear in R at fixed Ca_SS)
        const double kk = k2 * cass + 0.005;
        g[12] = rl(rbar, R(0.005 / kk), R(kk), dt);
    }

    }

    // ---- concentrations, forward Euler or Adams-Bashforth 2 (FP64)
    c[0] = buffered_free(buffered_total(cai, 0.2, 0.001) + dtd * e(rCai, 0), 0.2, 0.001);
    c[1] = buffered_free(buffered_total(casr, 10.0, 0.3) + dtd * e(rCasr, 1), 10.0, 0.3);
    c[2] = buffered_free(buffered_total(cass, 0.4, 0.00025) + dtd * e(rCass, 2), 0.4, 0.00025);
    c[3] = nai + dtd * e(rNai, 3);
    c[4] = ki + dtd * e(rKi, 4);
    return Iion;
}
}  // namespace tp06

// ==================================================================== CRN
// Courtemanche, Ramirez & Nattel, Am J Physiol 275:H301 (1998), with the
// conductances and pump rates of the article's parameter table.
// Gates (15): m h j oa oi ua ui xr xs d f fCa u v w.
// Concentrations (FP64): Ca_i Ca_up Ca_rel Na_i K_i, with troponin /
// calmodulin / calsequestrin buffering folded into the Ca rates.
namespace crn {
constexpr int NG = 15, NC = 5;
constexpr double RTF = 8.3143 * 310.0 / 96.4867;
constexpr double FARADAY = 96.4867;                      // C/mmol
constexpr double CM = 100.0, VI = 13668.0, VUP = 1109.52, VREL = 96.48;
constexpr double KO = 5.4, NAO = 140.0, CAO = 1.8;

__host__ __device__ inline void init(double *y) {
    const double s[21] = {-81.18, 2.908e-3, 9.649e-1, 9.775e-1, 3.043e-2,
                          9.992e-1, 4.966e-3, 9.986e-1, 3.296e-5, 1.869e-2,
                          1.367e-4, 9.996e-1, 7.755e-1, 0.0, 1.0, 9.992e-1,
                          1.013e-4, 1.488, 1.488, 11.17, 139.0};
    for (int i = 0; i < 21; ++i) y[i] = s[i];
}

template <typename R, bool RL2 = false, typename E = FwdEuler>
__device__ __forceinline__ R step(R V, R *g, double *c, R dt, double dtd,
                                  const GScale &gs, const E &e = E(), R lmi = R(0)) {
    const R frt = R(1.0 / RTF), rtf = R(RTF);
    const double cai = c[0], caup = c[1], carel = c[2], nai = c[3], ki = c[4];
    const R ENa = rtf * lnratio<R>(NAO, nai);
    const R EK = rtf * lnratio<R>(KO, ki);
    const R ECa = R(0.5) * rtf * lnratio<R>(CAO, cai);
    const R m = g[0], h = g[1], j = g[2], oa = g[3], oi = g[4], ua = g[5], ui = g[6];
    const R xr = g[7], xs = g[8], d = g[9], f = g[10], fca = g[11];
    const R u = g[12], vv = g[13], w = g[14];
    const R dK = V - EK;

    const R INa = R(gs.na) * R(7.8) * m * m * m * h * j * (V - ENa);
    const R IK1 = R(0.09) * dK * sig(R(0.07) * (V + R(80)));
    const R Ito = R(0.1652) * oa * oa * oa * oi * dK;
    const R IKur = (R(0.005) + R(0.05) * sig((V - R(15)) * R(-1.0 / 13.0))) * ua * ua * ua * ui * dK;
    const R IKr = R(gs.kr) * R(0.0294) * xr * dK * sig((V + R(15)) * R(1.0 / 22.4));
    const R IKs = R(gs.ks) * R(0.129) * xs * xs * dK;
    const R ICaL = R(gs.cal) * R(0.1238) * d * f * fca * (V - R(65));
    const R ev = xexp(-V * frt);
    const R sigma = R((std::exp(NAO / 67.3) - 1.0) / 7.0);
    const R fNaK = xrcp(R(1) + R(0.1245) * xexp(R(-0.1) * V * frt) + R(0.0365) * sigma * ev);
    const R INaK = R(0.60 * KO / (KO + 1.5)) * fNaK /
                   (R(1) + xpow15(xdiv(R(10), R(nai))));
    const R eg = xexp(R(0.35) * V * frt);
    const R eg1 = eg * ev;
    const R nai3 = R(nai) * R(nai) * R(nai);
    const R INaCa = R(1600.0 / ((87.5 * 87.5 * 87.5 + NAO * NAO * NAO) * (1.38 + CAO))) *
                    (eg * nai3 * R(CAO) - eg1 * R(NAO * NAO * NAO) * R(cai)) /
                    (R(1) + R(0.1) * eg1);
    const R IbNa = R(0.000674) * (V - ENa);
    const R IbCa = R(0.00113) * (V - ECa);
    const R IpCa = R(0.275) * R(cai) / (R(0.0005) + R(cai));
    const R Iion = INa + IK1 + Ito + IKur + IKr + IKs + ICaL + IpCa + INaK + INaCa +
                   IbNa + IbCa;

    // SR fluxes and concentration rates (FP64)
    const double Irel = 30.0 * double(u) * double(u) * double(vv) * double(w) * (carel - cai);
    const double Itr = (caup - carel) * (1.0 / 180.0);
    const double Iup = 0.005 / (1.0 + 0.00092 / cai);
    const double Iupleak = 0.005 * caup / 15.0;
    const double kc = CM / (FARADAY * VI);
    const double rNai = double(R(-3) * (INaK + INaCa) - IbNa - INa) * kc;
    const double rKi = double(R(2) * INaK - IK1 - Ito - IKur - IKr - IKs) * kc;
    const double b1 = double(R(2) * INaCa - IpCa - ICaL - IbCa) * (0.5 * kc) +
                      (VUP * (Iupleak - Iup) + Irel * VREL) * (1.0 / VI);
    const double t1 = cai + 0.0005, t2 = cai + 0.00238;
    const double b2 = 1.0 + 0.07 * 0.0005 / (t1 * t1) + 0.05 * 0.00238 / (t2 * t2);
    const double rCai = b1 / b2;
    const double rCaup = Iup - Iupleak - Itr * (VREL / VUP);
    const double t3 = carel + 0.8;
    const double rCarel = (Itr - Irel) / (1.0 + 10.0 * 0.8 / (t3 * t3));
    // release trigger: SR release flux and sarcolemmal Ca entry
    const double Fn = 1e-12 * VREL * Irel -
                      (5e-13 / FARADAY) * CM * (0.5 * double(ICaL) - 0.2 * double(INaCa));

    // gates: at level n, or (second-order variant) at the midpoint
    // predictions of V and Ca_i; u and v keep the level-n driver Fn
    R Vg = V;
    double cai_g = cai;
    if constexpr (RL2) {
        Vg = V + R(0.5) * dt * (lmi - Iion);
        cai_g = cai + 0.5 * dtd * rCai;
    }
    {
    const R V = Vg;
    const double cai = cai_g;
    {   // m: alpha = 0.32 (V+47.13) / (1 - e^{-0.1 (V+47.13)})
        const R a = R(3.2) * z_expm1(R(-0.1) * (V + R(47.13)));
        const R b = R(0.08) * xexp(-V * R(1.0 / 11.0));
        const R k = a + b;
        g[0] = rl(m, a / k, k, dt);
    }
    {
        R ah, bh, aj, bj;
        if (V >= R(-40)) {
            ah = R(0);
            bh = xrcp(R(0.13) * (R(1) + xexp((V + R(10.66)) * R(-1.0 / 11.1))));
            aj = R(0);
            bj = R(0.3) * xexp(R(-2.535e-7) * V) * sig(R(-0.1) * (V + R(32)));
        } else {
            ah = R(0.135) * xexp((V + R(80)) * R(-1.0 / 6.8));
            bh = R(3.56) * xexp(R(0.079) * V) + R(3.1e5) * xexp(R(0.35) * V);
            aj = (R(-127140) * xexp(R(0.2444) * V) - R(3.474e-5) * xexp(R(-0.04391) * V)) *
                 (V + R(37.78)) * sig(R(0.311) * (V + R(79.23)));
            bj = R(0.1212) * xexp(R(-0.01052) * V) * sig(R(-0.1378) * (V + R(40.14)));
        }
        g[1] = rl(h, ah / (ah + bh), ah + bh, dt);
        g[2] = rl(j, aj / (aj + bj), aj + bj, dt);
    }
    {   // oa, ua: common rate constants, temperature factor 3
        const R a = R(0.65) * xrcp(xexp((V + R(10)) * R(-1.0 / 8.5)) + xexp((V - R(30)) * R(-1.0 / 59.0)));
        const R b = R(0.65) * xrcp(R(2.5) + xexp((V + R(82)) * R(1.0 / 17.0)));
        const R k = (a + b) * R(3);
        g[3] = rl(oa, sig((V + R(20.47)) * R(-1.0 / 17.54)), k, dt);
        g[5] = rl(ua, sig((V + R(30.3)) * R(-1.0 / 9.6)), k, dt);
    }
    {   // oi
        const R a = xrcp(R(18.53) + xexp((V + R(113.7)) * R(1.0 / 10.95)));
        const R b = xrcp(R(35.56) + xexp((V + R(1.26)) * R(-1.0 / 7.44)));
        g[4] = rl(oi, sig((V + R(43.1)) * R(1.0 / 5.3)), (a + b) * R(3), dt);
    }
    {   // ui
        const R a = xrcp(R(21) + xexp((V - R(185)) * R(-1.0 / 28.0)));
        const R b = xexp((V - R(158)) * R(1.0 / 16.0));
        g[6] = rl(ui, sig((V - R(99.45)) * R(1.0 / 27.48)), (a + b) * R(3), dt);
    }
    {   // xr
        const R a = R(0.0003 * 5.0) * z_expm1((V + R(14.1)) * R(-0.2));
        const R b = R(7.3898e-5 * 5.1237) * z_expm1((V - R(3.3328)) * R(1.0 / 5.1237));
        g[7] = rl(xr, sig((V + R(14.1)) * R(-1.0 / 6.5)), a + b, dt);
    }
    {   // xs
        const R a = R(4e-5 * 17.0) * z_expm1((V - R(19.9)) * R(-1.0 / 17.0));
        const R b = R(3.5e-5 * 9.0) * z_expm1((V - R(19.9)) * R(1.0 / 9.0));
        const R inf = xrcp(xsqrt(R(1) + xexp((V - R(19.9)) * R(-1.0 / 12.7))));
        g[8] = rl(xs, inf, R(2) * (a + b), dt);
    }
    {   // d: tau = (1 - e^{-z}) / (0.035 * 6.24 z (1 + e^{-z})), z = (V+10)/6.24
        const R z = (V + R(10)) * R(1.0 / 6.24);
        const R k = R(0.035 * 6.24) * z_expm1(-z) * (R(1) + xexp(-z));
        g[9] = rl(d, sig((V + R(10)) * R(-0.125)), k, dt);
    }
    {   // f
        const R k = (R(0.0197) * xexp(R(-0.0337 * 0.0337) * (V + R(10)) * (V + R(10))) + R(0.02)) *
                    R(1.0 / 9.0);
        g[10] = rl(f, sig((V + R(28)) * R(1.0 / 6.9)), k, dt);
    }
    g[11] = rl(fca, xrcp(R(1) + R(cai * (1.0 / 0.00035))), R(0.5), dt);
    {   // u, v driven by Fn
        const R zu = R((Fn - 3.4175e-13) * (1.0 / 13.67e-16));
        const R zv = R((Fn - 6.835e-14) * (1.0 / 13.67e-16));
        g[12] = rl(u, sig(-zu), R(0.125), dt);
        const R tv = R(1.91) + R(2.09) * sig(-zu);
        g[13] = rl(vv, R(1) - sig(-zv), xrcp(tv), dt);
    }
    {   // w: tau = 6 (1 - e^{-z}) / ((1 + 0.3 e^{-z}) 5 z), z = (V-7.9)/5
        const R z = (V - R(7.9)) * R(0.2);
        const R k = R(5.0 / 6.0) * z_expm1(-z) * (R(1) + R(0.3) * xexp(-z));
        g[14] = rl(w, R(1) - sig((V - R(40)) * R(-1.0 / 17.0)), k, dt);
    }
    }
    c[0] = cai + dtd * e(rCai, 0);
    c[1] = caup + dtd * e(rCaup, 1);
    c[2] = carel + dtd * e(rCarel, 2);
    c[3] = nai + dtd * e(rNai, 3);
    c[4] = ki + dtd * e(rKi, 4);
    return Iion;
}
}  // namespace crn

// ================================================================ Stewart
// Stewart, Aslanidi, Noble, Noble, Boyett & Zhang, Phil Trans R Soc A
// 367:2225 (2009).  TP06 structure with Purkinje conductances, I_f (gate y),
// I_sus and modified I_to kinetics.  Gates (13, Rush-Larsen): m h j xr1 xr2
// xs r s d f f2 fCass y.  Forward Euler (FP64, with the concentrations
// because its increments are too small for FP32): Rbar Ca_i Ca_SR Ca_SS
// Na_i K_i.
namespace stewart {
constexpr int NG = 13, NC = 6;
constexpr double RTF = 8314.472 * 310.0 / 96485.3415;
constexpr double FARADAY = 96485.3415;
constexpr double KO = 5.4, NAO = 140.0, CAO = 2.0;
constexpr double CAP = 0.185, VC = 0.016404, VSR = 0.001094, VSS = 0.00005468;
constexpr double INV_VCF = CAP / (VC * FARADAY);
constexpr double INV_2VCF = CAP / (2.0 * VC * FARADAY);
constexpr double INV_2VSSF = CAP / (2.0 * VSS * FARADAY);

__host__ __device__ inline void init(double *y) {
    // V, m h j xr1 xr2 xs r s d f f2 fCass y Rbar, Ca_i Ca_SR Ca_SS Na_i K_i
    const double s[20] = {-69.1865, 0.0417391, 0.190678, 0.238219, 0.00550281,
                          0.313298, 0.00953708, 0.00103693, 0.96369,
                          0.000287906, 0.989361, 0.995179, 0.999656,
                          0.0457562, 0.991656, 0.000101878, 3.10836,
                          0.000446818, 8.80474, 136.7809};
    for (int i = 0; i < 20; ++i) y[i] = s[i];
}

template <typename R, bool RL2 = false, typename E = FwdEuler>
__device__ __forceinline__ R step(R V, R *g, double *c, R dt, double dtd,
                                  R istim, const GScale &gs, const E &e = E(), R lmi = R(0)) {
    const R frt = R(1.0 / RTF), rtf = R(RTF);
    const double rbar = c[0], cai = c[1], casr = c[2], cass = c[3], nai = c[4], ki = c[5];
    const R ENa = rtf * lnratio<R>(NAO, nai);
    const R EK = rtf * lnratio<R>(KO, ki);
    const R ECa = R(0.5) * rtf * lnratio<R>(CAO, cai);
    const R EKs = rtf * lnratio<R>(KO + 0.03 * NAO, ki + 0.03 * nai);
    const R m = g[0], h = g[1], j = g[2], xr1 = g[3], xr2 = g[4], xs = g[5];
    const R r = g[6], s = g[7], d = g[8], f = g[9], f2 = g[10], fcass = g[11];
    const R y = g[12];
    const R dK = V - EK;

    const R INa = R(gs.na) * R(130.5744) * m * m * m * h * j * (V - ENa);
    const R xca = R(2) * (V - R(15)) * frt;
    const R emx = xexpm1(xca);
    const R ghk = (fabs(xca) < R(1e-6)) ? R(1) - R(0.5) * xca : xdiv(xca, emx);
    const R ICaL = R(gs.cal) * R(3.980e-5 * 2.0 * FARADAY) * d * f * f2 * fcass * ghk *
                   (R(0.25) * R(cass) * (emx + R(1)) - R(CAO));
    const R Ito = R(0.08184) * r * s * dK;
    const R Isus = R(0.0227) * sig((R(5) - V) * R(1.0 / 17.0)) * dK;
    const R IKs = R(gs.ks) * R(0.2352) * xs * xs * (V - EKs);
    const R IKr = R(gs.kr) * R(0.0918) * xr1 * xr2 * dK;
    const R aK1 = R(0.1) * sig(R(0.06) * (dK - R(200)));
    const R bK1 = (R(3) * xexp(R(0.0002) * (dK + R(100))) + xexp(R(0.1) * (dK - R(10)))) *
                  sig(R(-0.5) * dK);
    const R IK1 = R(0.065) * aK1 / (aK1 + bK1) * dK;
    const R IfNa = R(0.0145654) * y * (V - ENa);
    const R IfK = R(0.0234346) * y * dK;
    const R ev = xexp(-V * frt);
    const R eg = xexp(R(0.35) * V * frt);
    const R eg1 = eg * ev;
    const R nai3 = R(nai) * R(nai) * R(nai);
    const R INaCa = R(1000.0 / ((87.5 * 87.5 * 87.5 + NAO * NAO * NAO) * (1.38 + CAO))) *
                    xdiv(eg * nai3 * R(CAO) - eg1 * R(NAO * NAO * NAO * 2.5) * R(cai),
                         R(1) + R(0.1) * eg1);
    const R INaK = R(2.724 * KO / (KO + 1.0)) *
                   xdiv(R(nai), (R(nai) + R(40)) *
                                    (R(1) + R(0.1245) * xexp(R(-0.1) * V * frt) + R(0.0353) * ev));
    const R IpCa = R(0.1238) * xdiv(R(cai), R(0.0005) + R(cai));
    const R IpK = R(0.0146) * dK * sig((R(25) - V) * R(1.0 / 5.98));
    const R IbNa = R(0.00029) * (V - ENa);
    const R IbCa = R(0.000592) * (V - ECa);
    const R Iion = INa + IK1 + Ito + Isus + IKr + IKs + ICaL + INaCa + INaK + IpCa +
                   IpK + IbNa + IbCa + IfNa + IfK;

    const double ec = xdiv(1.5, casr);
    const double kcasr = 2.5 - xdiv(1.5, 1.0 + ec * ec);
    const double k1 = xdiv(0.15, kcasr), k2 = 0.045 * kcasr;
    const double cass2 = cass * cass;
    const double Irel = 0.102 * (k1 * cass2 * rbar / (0.060 + k1 * cass2)) * (casr - cass);
    const double Iup = 0.006375 / (1.0 + (0.00025 * 0.00025) / (cai * cai));
    const double Ileak = 0.00036 * (casr - cai);
    const double Ixfer = 0.0038 * (cass - cai);
    const double rRbar = -k2 * cass * rbar + 0.005 * (1.0 - rbar);
    const double rCai = -double(IbCa + IpCa - R(2) * INaCa) * INV_2VCF +
                        (Ileak - Iup) * (VSR / VC) + Ixfer;
    const double rCasr = Iup - Irel - Ileak;
    const double rCass = -double(ICaL) * INV_2VSSF + Irel * (VSR / VSS) - Ixfer * (VC / VSS);
    const double rNai = -double(INa + IbNa + IfNa + R(3) * (INaK + INaCa)) * INV_VCF;
    const double rKi = -double(IK1 + Ito + Isus + IfK + IKr + IKs - R(2) * INaK + IpK + istim) *
                       INV_VCF;

    // gates: at level n, or (second-order variant) at the midpoint
    // predictions of V and Ca_SS
    R Vg = V;
    double cass_g = cass;
    if constexpr (RL2) {
        Vg = V + R(0.5) * dt * (lmi - Iion);
        cass_g = buffered_free(buffered_total(cass, 0.4, 0.00025) + 0.5 * dtd * rCass, 0.4, 0.00025);
    }
    {
    const R V = Vg;
    const double cass = cass_g;
    {
        const R s1 = sig((R(-56.86) - V) * R(1.0 / 9.03));
        const R am = sig((R(-60) - V) * R(0.2));
        const R bm = R(0.1) * sig((V + R(35)) * R(0.2)) + R(0.1) * sig((V - R(50)) * R(0.005));
        g[0] = rl(m, s1 * s1, xrcp(am * bm), dt);
    }
    {
        const R s1 = sig((V + R(71.55)) * R(1.0 / 7.43));
        const R inf = s1 * s1;
        R kh, kj;
        if (V >= R(-40)) {
            kh = xrcp(R(0.13 / 0.77) * (R(1) + xexp((V + R(10.66)) * R(-1.0 / 11.1))));
            kj = R(0.6) * xexp(R(0.057) * V) * sig(R(-0.1) * (V + R(32)));
        } else {
            kh = R(0.057) * xexp((V + R(80)) * R(-1.0 / 6.8)) + R(2.7) * xexp(R(0.079) * V) +
                 R(3.1e5) * xexp(R(0.3485) * V);
            kj = (R(-2.5428e4) * xexp(R(0.2444) * V) - R(6.948e-6) * xexp(R(-0.04391) * V)) *
                     (V + R(37.78)) * sig(R(0.311) * (V + R(79.23))) +
                 R(0.02424) * xexp(R(-0.01052) * V) * sig(R(-0.1378) * (V + R(40.14)));
        }
        g[1] = rl(h, inf, kh, dt);
        g[2] = rl(j, inf, kj, dt);
    }
    {
        const R a = R(450) * sig((R(-45) - V) * R(0.1));
        const R b = R(6) * sig((V + R(30)) * R(1.0 / 11.5));
        g[3] = rl(xr1, sig((R(-26) - V) * R(1.0 / 7.0)), xrcp(a * b), dt);
    }
    {
        const R a = R(3) * sig((R(-60) - V) * R(0.05));
        const R b = R(1.12) * sig((V - R(60)) * R(0.05));
        g[4] = rl(xr2, sig((V + R(88)) * R(1.0 / 24.0)), xrcp(a * b), dt);
    }
    {
        const R a = R(1400) / xsqrt(R(1) + xexp((R(5) - V) * R(1.0 / 6.0)));
        const R b = sig((V - R(35)) * R(1.0 / 15.0));
        g[5] = rl(xs, sig((R(-5) - V) * R(1.0 / 14.0)), xrcp(a * b + R(80)), dt);
    }
    {   // I_to gates, Purkinje kinetics
        const R tr = R(10.45) * xexp(-(V + R(40)) * (V + R(40)) * R(1.0 / 1800.0)) + R(7.3);
        g[6] = rl(r, sig((R(20) - V) * R(1.0 / 13.0)), xrcp(tr), dt);
        const R ts = R(85) * xexp(-(V + R(25)) * (V + R(25)) * R(1.0 / 320.0)) +
                     R(5) * sig((V - R(40)) * R(0.2)) + R(42);
        g[7] = rl(s, sig((V + R(27)) * R(1.0 / 13.0)), xrcp(ts), dt);
    }
    {
        const R a = R(1.4) * sig((R(-35) - V) * R(1.0 / 13.0)) + R(0.25);
        const R b = R(1.4) * sig((V + R(5)) * R(0.2));
        const R cc = sig((R(50) - V) * R(0.05));
        g[8] = rl(d, sig((R(-8) - V) * R(1.0 / 7.5)), xrcp(a * b + cc), dt);
    }
    {
        const R t = R(1102.5) * xexp(-(V + R(27)) * (V + R(27)) * R(1.0 / 225.0)) +
                    R(200) * sig((R(13) - V) * R(0.1)) + R(180) * sig((V + R(30)) * R(0.1)) + R(20);
        g[9] = rl(f, sig((V + R(20)) * R(1.0 / 7.0)), xrcp(t), dt);
    }
    {
        const R t = R(600) * xexp(-(V + R(25)) * (V + R(25)) * R(1.0 / 170.0)) +
                    R(31) * sig((R(25) - V) * R(0.1)) + R(16) * sig((V + R(30)) * R(0.1));
        g[10] = rl(f2, R(0.67) * sig((V + R(35)) * R(1.0 / 7.0)) + R(0.33), xrcp(t), dt);
    }
    {
        const R q = R(cass * 400.0 * cass);
        const R w = xrcp(R(1) + q);
        g[11] = rl(fcass, R(0.6) * w + R(0.4), xrcp(R(80) * w + R(2)), dt);
    }
    {   // I_f gate
        const R k = (xexp(R(-2.9) - R(0.04) * V) + xexp(R(3.6) + R(0.11) * V)) * R(1.0 / 4000.0);
        g[12] = rl(y, sig((V + R(80.6)) * R(1.0 / 6.8)), k, dt);
    }
    }
    c[0] = rbar + dtd * e(rRbar, 0);
    c[1] = buffered_free(buffered_total(cai, 0.2, 0.001) + dtd * e(rCai, 1), 0.2, 0.001);
    c[2] = buffered_free(buffered_total(casr, 10.0, 0.3) + dtd * e(rCasr, 2), 10.0, 0.3);
    c[3] = buffered_free(buffered_total(cass, 0.4, 0.00025) + dtd * e(rCass, 3), 0.4, 0.00025);
    c[4] = nai + dtd * e(rNai, 4);
    c[5] = ki + dtd * e(rKi, 5);
    return Iion;
}
}  // namespace stewart

}  // namespace epdev
