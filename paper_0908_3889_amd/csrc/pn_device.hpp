// pn_device.hpp -- device-side pieces of the gfx950 integrator: the
// per-inspiral coefficient row, the right-hand side of Eqs. (1)-(4), and the
// few FP64 special functions the path needs (cube root, natural log,
// z^(-1/10)), each built from a hardware FP32 seed and FP64 Newton steps.
//
// Every value here is computed by this file; nothing is shared with the CPU
// oracle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pn.h"

namespace pn {

// a*b + c as the three-address FP64 FMA.  For Horner steps whose addend is a
// constant held in a register: the compiler otherwise copies the constant
// and uses the two-address form.
__device__ __forceinline__ double fma3(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// max(|a|, |b|) as one instruction.  The compiler's fmax first quiets each
// operand (a signalling NaN must not pass through) at the cost of two more
// instructions; the operands here are results of arithmetic, never
// signalling NaNs.
__device__ __forceinline__ double fmax_abs(double a, double b) {
    double d;
    asm("v_max_f64 %0, |%1|, |%2|" : "=v"(d) : "v"(a), "v"(b));
    return d;
}

// a*b + k for a constant k, as the three-address FP64 FMA with k in a scalar
// register pair: Horner chains with constant coefficients otherwise keep the
// coefficients in vector registers and copy each before a two-address FMA.
__device__ __forceinline__ double fma_k(double a, double b, double k) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(k));
    return d;
}

// ---------------------------------------------------------------------------
// FP64 special functions.  Each states the range it accepts; the callers
// guarantee or clamp it.
// ---------------------------------------------------------------------------

// cube root of a in [2^-120, 2^120]: FP32 seed from the hardware log2/exp2,
// then two Newton steps x <- x - (x^3 - a) r with r ~ 1/(3 x0^2) from the FP32
// reciprocal.  The seed is good to ~3e-7, the first step to ~1e-13, the
// second to rounding.
__device__ __forceinline__ double cbrt_mid(double a) {
    const float af = (float)a;
    const float x0f = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(af) * (1.0f / 3.0f));
    const double r = (double)__builtin_amdgcn_rcpf(3.0f * x0f * x0f);
    double x = (double)x0f;
    double t = __builtin_fma(x * x, x, -a);
    x = __builtin_fma(-t, r, x);
    t = __builtin_fma(x * x, x, -a);
    x = __builtin_fma(-t, r, x);
    return x;
}

// real cube root of any finite v (negative v gives -cbrt(|v|)).  Magnitudes
// outside [2^-120, 2^120] are first scaled by 2^(3k) into range; lanes that
// never see such values skip that branch.
__device__ __forceinline__ double cbrt_real(double v) {
    double a = __builtin_fabs(v);
    int k = 0;
    if (!(a >= 0x1p-120 && a <= 0x1p120)) {
        const int e = __builtin_amdgcn_frexp_exp(a);
        k = (e >= 0 ? e : e - 2) / 3;                      // floor(e/3)
        a = __builtin_amdgcn_ldexp(a, -3 * k);
        if (!(a > 0.0) || !__builtin_isfinite(a)) return v;   // 0, inf or NaN
    }
    const double x = __builtin_amdgcn_ldexp(cbrt_mid(a), k);
    return __builtin_copysign(x, v);
}

// 1/d for d normal (either sign; the name records the callers' usual case):
// hardware reciprocal refined by two Newton steps.
__device__ __forceinline__ double rcp_pos(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// 1/d for d > 0 normal to about 12 ulp: hardware reciprocal (good to about
// 2^-24 relative) and one Newton step.  For the error norm, which only
// steers the step size.
__device__ __forceinline__ double rcp_1step(double d) {
    const double r = __builtin_amdgcn_rcp(d);
    return __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
}

// natural log of v > 0 (normal or subnormal): v = 2^e m with m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s), s = (m-1)/(m+1), |s| <= 0.1716, by its Taylor series
// sum_k s^(2k+1)/(2k+1) truncated after s^19 (relative remainder < 3e-17).
__device__ __forceinline__ double log_pos(double v) {
    double m = __builtin_amdgcn_frexp_mant(v);          // [0.5, 1)
    int e = __builtin_amdgcn_frexp_exp(v);
    const bool lo = m < 0.70710678118654752440;
    m = lo ? m * 2.0 : m;
    e = lo ? e - 1 : e;
    const double num = m - 1.0;                          // exact (Sterbenz)
    const double den = m + 1.0;
    const double rden = rcp_pos(den);
    double s = num * rden;
    s = __builtin_fma(__builtin_fma(-s, den, num), rden, s);   // one residual correction
    const double s2 = s * s;
    double p = 1.0 / 19.0;
    p = __builtin_fma(p, s2, 1.0 / 17.0);
    p = __builtin_fma(p, s2, 1.0 / 15.0);
    p = __builtin_fma(p, s2, 1.0 / 13.0);
    p = __builtin_fma(p, s2, 1.0 / 11.0);
    p = __builtin_fma(p, s2, 1.0 / 9.0);
    p = __builtin_fma(p, s2, 1.0 / 7.0);
    p = __builtin_fma(p, s2, 1.0 / 5.0);
    p = __builtin_fma(p, s2, 1.0 / 3.0);
    const double lnm = __builtin_fma(2.0 * s * s2, p, 2.0 * s);
    // ln 2 split so that e * LN2_HI is exact for |e| < 2^11
    const double LN2_HI = 6.93147180369123816490e-01;
    const double LN2_LO = 1.90821492927058770002e-10;
    const double de = (double)e;
    return __builtin_fma(de, LN2_HI, __builtin_fma(de, LN2_LO, lnm));
}

// max(a, k) and min(a, k) for a constant k as one instruction each (see
// fmax_abs: no quieting of the operands, which are never signalling NaNs).
__device__ __forceinline__ double fmax_k(double a, double k) {
    double d;
    asm("v_max_f64 %0, %1, %2" : "=v"(d) : "v"(a), "s"(k));
    return d;
}
__device__ __forceinline__ double fmin_k(double a, double k) {
    double d;
    asm("v_min_f64 %0, %1, %2" : "=v"(d) : "v"(a), "s"(k));
    return d;
}

// c z^(-1/10) for z in [2^-30, 2^30] (callers clamp): FP32 seed (relative
// error below 1e-7 over that range), then one Newton step of
// y <- y (11 - z y^10) / 10, which leaves 5.5 times its square (< 1e-13).
// The result only scales the next step size.
__device__ __forceinline__ double pow_m_tenth_scaled(double z, double c) {
    const float zf = (float)z;
    const double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf(zf) * -0.1f);
    const double y2 = y * y;
    const double y5 = (y2 * y2) * y;
    const double t = __builtin_fma(-z, y5 * y5, 11.0);
    return (y * t) * (0.1 * c);
}

// ---------------------------------------------------------------------------
// Per-inspiral coefficient row: everything in Eqs. (1)-(4) that depends only
// on (m1, m2) and the term switches.  Built once per inspiral.
// ---------------------------------------------------------------------------
enum RowIdx {
    R_M = 0,   // m1 + m2
    R_C2,      // -(743 + 924 eta)/336                                (M w)^{2/3}
    R_SO1,     // (113 m1^2/M^2 + 75 eta)/(12 m1^2)  [times L.S1]     (M w)^{1}
    R_SO2,     // (113 m2^2/M^2 + 75 eta)/(12 m2^2)  [times L.S2]
    R_C4,      // 34103/18144 + 13661/2016 eta + 59/18 eta^2          (M w)^{4/3}
    R_SSD,     // eta / (48 m1^2 m2^2) [times (247 S1.S2 - 721 L.S1 L.S2)]
    R_C5,      // -(4159 + 15876 eta) pi / 672                        (M w)^{5/3}
    R_C6,      // 3PN constant part, -(856/105) ln 16 included        (M w)^{2}
    R_C7,      // (-4415/4032 + 358675/6048 eta + 91495/1512 eta^2) pi (M w)^{7/3}
    R_K,       // (96/5) eta: d omega/dt = K omega^2 x^5 {...}
    R_G1,      // eta (4 + 3 m2/m1)
    R_G2,      // eta (4 + 3 m1/m2)
    R_SIGM,    // 1/M: (1/M^2)(M w) = w/M in the spin-spin part of Eq. (4)
    R_LAM,     // 1/(eta M^2)
    NROW
};

// the row held in registers (test kernels)
struct Row {
    double v[NROW];
    __device__ __forceinline__ double operator[](int i) const { return v[i]; }
    __device__ __forceinline__ void set(int i, double x) { v[i] = x; }
};

// the row held in LDS, one column per lane: entry i of this lane at p[i * 64].
// Reads are volatile so that every right-hand-side evaluation reads the row
// again instead of the compiler keeping 16 doubles in registers.
struct RowLds {
    volatile double* p;
    __device__ __forceinline__ double operator[](int i) const { return p[i * 64]; }
    __device__ __forceinline__ void set(int i, double x) const { p[i * 64] = x; }
};

// Launch-uniform switches folded into numbers: 4 pi and -1712/315 when the
// non-spinning PN terms are on, else 0.
struct TermConsts {
    double c3;     // 4 pi
    double c6lnv;  // coefficient of ln|M w| in the 3PN bracket: -(856/105)(2/3) = -1712/315
};

#define PN_PI 3.14159265358979323846
#define PN_GAMMA_E 0.57721566490153286061
#define PN_LN16 2.77258872223978123767

template <class RowT>
__device__ __forceinline__ void make_row(RowT& r, double m1, double m2, int terms, int theta_literal) {
    const double M = m1 + m2;
    const double iM = 1.0 / M;
    const double eta = m1 * m2 * iM * iM;
    const double pn = (terms & PN_TERM_PN) ? 1.0 : 0.0;
    const double fso = (terms & PN_TERM_SO_WDOT) ? 1.0 : 0.0;
    const double fss = (terms & PN_TERM_SS_WDOT) ? 1.0 : 0.0;
    r.set(R_M, M);
    r.set(R_C2, pn * (-(743.0 + 924.0 * eta) / 336.0));
    r.set(R_SO1, fso * (113.0 * m1 * m1 * iM * iM + 75.0 * eta) / (12.0 * m1 * m1));
    r.set(R_SO2, fso * (113.0 * m2 * m2 * iM * iM + 75.0 * eta) / (12.0 * m2 * m2));
    r.set(R_C4, pn * (34103.0 / 18144.0 + (13661.0 / 2016.0) * eta + (59.0 / 18.0) * eta * eta));
    r.set(R_SSD, fss * eta / (48.0 * m1 * m1 * m2 * m2));
    r.set(R_C5, pn * (-(4159.0 + 15876.0 * eta) * PN_PI / 672.0));
    // 3PN: theta_hat = 1039/4620 multiplies eta once (the expansion of
    // Eq. (1)'s source), or, with theta_literal, eta^2 as printed.
    const double theta_term = (88.0 / 3.0) * (1039.0 / 4620.0) * (theta_literal ? eta : 1.0);
    r.set(R_C6, pn * ((16447322263.0 / 139708800.0) - (1712.0 / 105.0) * PN_GAMMA_E
                      + (16.0 / 3.0) * PN_PI * PN_PI
                      + (-273811877.0 / 1088640.0 + (451.0 / 48.0) * PN_PI * PN_PI - theta_term) * eta
                      + (541.0 / 896.0) * eta * eta - (5605.0 / 2592.0) * eta * eta * eta
                      - (856.0 / 105.0) * PN_LN16));
    r.set(R_C7, pn * ((-4415.0 / 4032.0 + (358675.0 / 6048.0) * eta + (91495.0 / 1512.0) * eta * eta) * PN_PI));
    r.set(R_K, (terms & PN_TERM_RR) ? (96.0 / 5.0) * eta : 0.0);
    r.set(R_G1, (terms & PN_TERM_SO_PREC) ? eta * (4.0 + 3.0 * m2 / m1) : 0.0);
    r.set(R_G2, (terms & PN_TERM_SO_PREC) ? eta * (4.0 + 3.0 * m1 / m2) : 0.0);
    r.set(R_SIGM, (terms & PN_TERM_SS_PREC) ? iM : 0.0);
    r.set(R_LAM, 1.0 / (eta * M * M));
}

// The stage points of a step lie close to its base point: with
// u = (w_s - w_n)/w_n, |u| <= 1/16 on all but about 2 in 10^4 steps of the
// workloads (the rest take the full log and cube root).  There
//   (1+u)^{1/3} - 1 = w = u (1/3 + u Q(u)),
//   ln(1+u) = 3 ln(1+w) = w (3 + w R3(w)),
// with Q of degree 8 on [-1/16, 1/16] and R3 of degree 5 on the matching
// w in [-0.02130, 0.02041], each interpolated at its Chebyshev nodes in 60-digit
// arithmetic.  Largest errors: |u^2 dQ| < 2.5e-18 (relative, in the cube
// root) and |w^2 dR3| < 4.5e-16 (absolute, in ln|M w|, whose weight in
// Eq. (1) is at most (1712/315) x^6 < 0.014).
constexpr double kSmallU = 0.0625;

__device__ __forceinline__ double cbrt1p_small_m1(double u) {
    double q = -0.01177066091614973521624749;
    q = fma_k(q, u, 0.0135791980361245423248501);
    q = fma_k(q, u, -0.01583407049188512767371284);
    q = fma_k(q, u, 0.01900090236519766360899345);
    q = fma_k(q, u, -0.0234720319593868172360808);
    q = fma_k(q, u, 0.03017832676360298774987899);
    q = fma_k(q, u, -0.04115226337441031440928335);
    q = fma_k(q, u, 0.06172839506164371309340048);
    q = fma_k(q, u, -0.1111111111111111111111111);
    return u * fma_k(u, q, 1.0 / 3.0);
}

// 3 ln(1+w) / w = 3 + w R3(w)
__device__ __forceinline__ double log1p_cbrt_over_w(double w) {
    double r = 0.4297688281944602466457629;
    r = fma_k(r, w, -0.5002437143231824139713031);
    r = fma_k(r, w, 0.599999539072323222208094);
    r = fma_k(r, w, -0.7499999603441906901946652);
    r = fma_k(r, w, 1.000000000035512911627931);
    r = fma_k(r, w, -1.500000000000957520846056);
    return fma_k(r, w, 3.0);
}

// The base of the stage logs and cube roots at the start of a step: within
// a step the stage omegas stay close to omega_n, so with u = (w_s - w_n)/w_n
//   (M w_s)^{1/3} = (M w_n)^{1/3} (1 + w),  w = (1 + u)^{1/3} - 1,
//   ln|M w_s| = ln|M w_n| + 3 ln(1 + w),
// each from a short polynomial; |u| > 1/16 (rejected or very long steps) falls
// back to the full log and cube root.
struct LogBase {
    double lnv;    // ln|M w_n|
    double x;      // (M w_n)^{1/3}
    double w;      // w_n
    double iw;     // 1/w_n
};

// dy/dt of Eqs. (1)-(4) at y = (w, S1, S2, L) into d (d omega/dt in d[0]),
// given v = M w, x = v^{1/3} and ln|v|.
//
// With v = M w and x = v^{1/3}:
//   d w/dt = K w^2 x^5 B (formed as K w^2 x^2 v B),
//     B = 1 + x^2 (c2 + x (c3' + x (c4' + x (c5 + x (c6' + x c7)))))
//     c3' = 4 pi - so1 L.S1 - so2 L.S2,
//     c4' = c4 - ssd (247 S1.S2 - 721 (L.S1)(L.S2)),
//     c6' = c6 - (1712/105) ln x;
//   dS1/dt = Omega_1 x S1,  Omega_1 = p [ (g1 x^2 - 3 sv L.S2) L + sv S2 ],
//   dS2/dt = Omega_2 x S2,  Omega_2 = p [ (g2 x^2 - 3 sv L.S1) L + sv S1 ],
//     p = w/2 = (M w)/(2M),  sv = w/M  (Eq. (4) expanded; the eta (M w)^{-1/3}
//     term times (M w)^2/(2M) is p g_i x^2);
//   dL/dt = -lam x (dS1/dt + dS2/dt)   (Eq. (3)).
// Off the physical region (stage points of rejected or fixed steps) omega may
// be negative; x is then the real cube root and the log term uses
// ln(16 x^2) = ln 16 + (2/3) ln|v|, which is what Eq. (1) gives for any real x.
template <class RowT>
__device__ __forceinline__ void rhs_at(const RowT& r, const TermConsts& tc, const double* __restrict__ y,
                                       double v, double x, double lnv, double* __restrict__ d) {
    const double w = y[0];
    const double x2 = x * x;
    const double L0 = y[7], L1 = y[8], L2 = y[9];
    const double a0 = y[1], a1 = y[2], a2 = y[3];   // S1
    const double b0 = y[4], b1 = y[5], b2 = y[6];   // S2
    const double LS1 = __builtin_fma(L0, a0, __builtin_fma(L1, a1, L2 * a2));
    const double LS2 = __builtin_fma(L0, b0, __builtin_fma(L1, b1, L2 * b2));
    const double S12 = __builtin_fma(a0, b0, __builtin_fma(a1, b1, a2 * b2));

    const double c3p = __builtin_fma(-r[R_SO2], LS2, __builtin_fma(-r[R_SO1], LS1, tc.c3));
    const double ssb = __builtin_fma(247.0, S12, -721.0 * (LS1 * LS2));
    const double c4p = __builtin_fma(-r[R_SSD], ssb, r[R_C4]);
    const double c6p = __builtin_fma(tc.c6lnv, lnv, r[R_C6]);
    double B = __builtin_fma(x, r[R_C7], c6p);
    B = __builtin_fma(x, B, r[R_C5]);
    B = __builtin_fma(x, B, c4p);
    B = __builtin_fma(x, B, c3p);
    B = __builtin_fma(x, B, r[R_C2]);
    B = __builtin_fma(x2, B, 1.0);
    // x^5 = x^2 v (x^3 = v)
    d[0] = (r[R_K] * (w * w)) * (x2 * v) * B;

    const double p = 0.5 * w;
    const double sv = r[R_SIGM] * w;
    const double al1 = p * __builtin_fma(r[R_G1], x2, -3.0 * sv * LS2);
    const double al2 = p * __builtin_fma(r[R_G2], x2, -3.0 * sv * LS1);
    const double be = p * sv;
    // Omega_1 = al1 L + be S2, Omega_2 = al2 L + be S1
    const double o0 = __builtin_fma(al1, L0, be * b0), o1 = __builtin_fma(al1, L1, be * b1),
                 o2 = __builtin_fma(al1, L2, be * b2);
    const double g0 = __builtin_fma(al2, L0, be * a0), g1 = __builtin_fma(al2, L1, be * a1),
                 g2 = __builtin_fma(al2, L2, be * a2);
    d[1] = __builtin_fma(o1, a2, -o2 * a1);
    d[2] = __builtin_fma(o2, a0, -o0 * a2);
    d[3] = __builtin_fma(o0, a1, -o1 * a0);
    d[4] = __builtin_fma(g1, b2, -g2 * b1);
    d[5] = __builtin_fma(g2, b0, -g0 * b2);
    d[6] = __builtin_fma(g0, b1, -g1 * b0);
    const double q = -r[R_LAM] * x;
    d[7] = q * (d[1] + d[4]);
    d[8] = q * (d[2] + d[5]);
    d[9] = q * (d[3] + d[6]);
}

// x = v^{1/3} and ln|v| at a stage point (v = M w) from the step's base
// point: the polynomials in u = (w - w_n)/w_n, or in full on the rare lanes
// with |u| > 1/16 (a block the wave skips unless one of its lanes needs it).
__device__ __forceinline__ void stage_x_lnv(const LogBase& lb, double v, double w, double& x, double& lnv) {
    const double u = (w - lb.w) * lb.iw;
    const double c = cbrt1p_small_m1(u);
    x = __builtin_fma(lb.x, c, lb.x);
    lnv = fma3(c, log1p_cbrt_over_w(c), lb.lnv);
    const bool far = !(__builtin_fabs(u) <= kSmallU);
    if (__builtin_expect(__ballot(far) != 0, 0)) {
        if (far) {
            x = cbrt_real(v);
            lnv = log_pos(__builtin_fabs(v));
        }
    }
}

// dy/dt at y into d; returns ln|M w| as used, and x = (M w)^{1/3} as used in
// xo.  FAST_LOG: x and the log from the step's base point (LogBase).
template <class RowT, bool FAST_LOG>
__device__ __forceinline__ double rhs_x(const RowT& r, const TermConsts& tc, const LogBase& lb,
                                        const double* __restrict__ y, double* __restrict__ d, double& xo) {
    const double w = y[0];
    const double v = r[R_M] * w;
    double x, lnv;
    if (FAST_LOG) {
        stage_x_lnv(lb, v, w, x, lnv);
        rhs_at(r, tc, y, v, x, lnv, d);
    } else {
        x = cbrt_real(v);
        lnv = log_pos(__builtin_fabs(v));
        rhs_at(r, tc, y, v, x, lnv, d);
    }
    xo = x;
    return lnv;
}
template <class RowT, bool FAST_LOG>
__device__ __forceinline__ double rhs(const RowT& r, const TermConsts& tc, const LogBase& lb,
                                      const double* __restrict__ y, double* __restrict__ d) {
    double x;
    return rhs_x<RowT, FAST_LOG>(r, tc, lb, y, d, x);
}

// the base of the stage logs at the state y
template <class RowT>
__device__ __forceinline__ LogBase log_base(const RowT& r, const double* y) {
    LogBase lb;
    lb.w = y[0];
    lb.lnv = log_pos(__builtin_fabs(r[R_M] * y[0]));
    lb.x = cbrt_real(r[R_M] * y[0]);
    lb.iw = rcp_pos(y[0]);
    return lb;
}

// ---------------------------------------------------------------------------
// FP32 right-hand side (the FP32-split mode): the same Eqs. (1)-(4) in single
// precision, with the hardware FP32 log2/exp2/reciprocal.
// ---------------------------------------------------------------------------
struct RowF {
    float v[NROW];
    __device__ __forceinline__ float operator[](int i) const { return v[i]; }
};

__device__ __forceinline__ RowF to_f32(const Row& r) {
    RowF f;
#pragma unroll
    for (int i = 0; i < NROW; ++i) f.v[i] = (float)r.v[i];
    return f;
}

// real cube root in FP32: hardware seed and one Newton step (negative a ->
// -cbrt|a|; the seed handles the whole float range except 0).
__device__ __forceinline__ float cbrt_f32(float a) {
    const float m = __builtin_fabsf(a);
    float x = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(m) * (1.0f / 3.0f));
    const float t = __builtin_fmaf(x * x, x, -m);
    x = __builtin_fmaf(-t, __builtin_amdgcn_rcpf(3.0f * x * x), x);
    return __builtin_copysignf(x, a);
}

struct TermConstsF {
    float c3;      // 4 pi (or 0)
    float c6lnv;   // -1712/315 (or 0)
};

// Eqs. (1)-(4) in FP32, same expansion as rhs() above.
__device__ __forceinline__ void rhs_f32(const RowF& r, const TermConstsF& tc, const float* __restrict__ y,
                                        float* __restrict__ d) {
    const float w = y[0];
    const float v = r[R_M] * w;
    const float x = cbrt_f32(v);
    const float lnv = __builtin_amdgcn_logf(__builtin_fabsf(v)) * 0.69314718055994531f;
    const float x2 = x * x;
    const float L0 = y[7], L1 = y[8], L2 = y[9];
    const float a0 = y[1], a1 = y[2], a2 = y[3];
    const float b0 = y[4], b1 = y[5], b2 = y[6];
    const float LS1 = __builtin_fmaf(L0, a0, __builtin_fmaf(L1, a1, L2 * a2));
    const float LS2 = __builtin_fmaf(L0, b0, __builtin_fmaf(L1, b1, L2 * b2));
    const float S12 = __builtin_fmaf(a0, b0, __builtin_fmaf(a1, b1, a2 * b2));
    const float c3p = __builtin_fmaf(-r[R_SO2], LS2, __builtin_fmaf(-r[R_SO1], LS1, tc.c3));
    const float ssb = __builtin_fmaf(247.0f, S12, -721.0f * (LS1 * LS2));
    const float c4p = __builtin_fmaf(-r[R_SSD], ssb, r[R_C4]);
    const float c6p = __builtin_fmaf(tc.c6lnv, lnv, r[R_C6]);
    float B = __builtin_fmaf(x, r[R_C7], c6p);
    B = __builtin_fmaf(x, B, r[R_C5]);
    B = __builtin_fmaf(x, B, c4p);
    B = __builtin_fmaf(x, B, c3p);
    B = __builtin_fmaf(x, B, r[R_C2]);
    B = __builtin_fmaf(x2, B, 1.0f);
    d[0] = (r[R_K] * (w * w)) * (x2 * v) * B;     // x^5 = x^2 v
    const float p = 0.5f * w;
    const float sv = r[R_SIGM] * w;
    const float al1 = p * __builtin_fmaf(r[R_G1], x2, -3.0f * sv * LS2);
    const float al2 = p * __builtin_fmaf(r[R_G2], x2, -3.0f * sv * LS1);
    const float be = p * sv;
    // Omega_1 = al1 L + be S2, Omega_2 = al2 L + be S1
    const float o0 = __builtin_fmaf(al1, L0, be * b0), o1 = __builtin_fmaf(al1, L1, be * b1),
                o2 = __builtin_fmaf(al1, L2, be * b2);
    const float g0 = __builtin_fmaf(al2, L0, be * a0), g1 = __builtin_fmaf(al2, L1, be * a1),
                g2 = __builtin_fmaf(al2, L2, be * a2);
    d[1] = __builtin_fmaf(o1, a2, -o2 * a1);
    d[2] = __builtin_fmaf(o2, a0, -o0 * a2);
    d[3] = __builtin_fmaf(o0, a1, -o1 * a0);
    d[4] = __builtin_fmaf(g1, b2, -g2 * b1);
    d[5] = __builtin_fmaf(g2, b0, -g0 * b2);
    d[6] = __builtin_fmaf(g0, b1, -g1 * b0);
    const float q = -r[R_LAM] * x;
    d[7] = q * (d[1] + d[4]);
    d[8] = q * (d[2] + d[5]);
    d[9] = q * (d[3] + d[6]);
}

}  // namespace pn
