// pn_adjoint.hpp -- reverse-mode pieces of the discrete adjoint: the
// vector-Jacobian product of the right-hand side of Eqs. (1)-(4) (with
// respect to the state and to the 14-entry coefficient row), and the
// derivative of the coefficient row with respect to the masses.
#pragma once

#include "pn_device.hpp"

namespace pn {

// Adjoint of the coefficient row, accumulated over every stage of every step.
struct RowBar {
    double v[NROW];
};

// VJP of f = rhs(y) at y: given fbar = dL/df (10), writes (df/dy)^T fbar to
// ybar and adds (df/drow)^T fbar to rb.  The primal is recomputed here (same
// expansion as rhs(); the cube root and log of the stage from the step's base
// point lb, as the stage derivatives of the replay take them).
//
// Omega mode: the stage derivative is g = (1, f_1/f_0, ..., f_9/f_0) with
// dt/domega = 1/f_0.  With omega_mode set, gbar (slot 0 unused) and gtbar
// (the weight of dt/domega) are first turned into fbar:
//   s = 1/f_0,  sbar = gtbar + sum_{c>=1} gbar_c f_c,
//   fbar_c = gbar_c s (c >= 1),  fbar_0 = -s^2 sbar.
//
// gscale multiplies gbar_in (the step size of the RK adjoint recurrence).
__device__ __forceinline__ void rhs_vjp(const Row& r, const TermConsts& tc, const LogBase& lb,
                                        const double* __restrict__ y,
                                        const double* __restrict__ gbar_in, double gscale, double gtbar,
                                        bool omega_mode, double* __restrict__ ybar, RowBar& rb) {
    // ---------------- primal ----------------
    const double w = y[0];
    const double M = r[R_M];
    const double v = M * w;
    double x, lnv;
    stage_x_lnv(lb, v, w, x, lnv);
    const double x2 = x * x;
    const double L0 = y[7], L1 = y[8], L2 = y[9];
    const double a0 = y[1], a1 = y[2], a2 = y[3];
    const double b0 = y[4], b1 = y[5], b2 = y[6];
    const double LS1 = __builtin_fma(L0, a0, __builtin_fma(L1, a1, L2 * a2));
    const double LS2 = __builtin_fma(L0, b0, __builtin_fma(L1, b1, L2 * b2));
    const double S12 = __builtin_fma(a0, b0, __builtin_fma(a1, b1, a2 * b2));
    const double c3p = __builtin_fma(-r[R_SO2], LS2, __builtin_fma(-r[R_SO1], LS1, tc.c3));
    const double ssb = __builtin_fma(247.0, S12, -721.0 * (LS1 * LS2));
    const double c4p = __builtin_fma(-r[R_SSD], ssb, r[R_C4]);
    const double c6p = __builtin_fma(tc.c6lnv, lnv, r[R_C6]);
    const double B5 = __builtin_fma(x, r[R_C7], c6p);
    const double B4 = __builtin_fma(x, B5, r[R_C5]);
    const double B3 = __builtin_fma(x, B4, c4p);
    const double B2 = __builtin_fma(x, B3, c3p);
    const double B1 = __builtin_fma(x, B2, r[R_C2]);
    const double B = __builtin_fma(x2, B1, 1.0);
    const double x4 = x2 * x2;
    const double x5 = x4 * x;
    const double Kw2 = r[R_K] * (w * w);
    const double f0 = Kw2 * x5 * B;
    const double p = 0.5 * w;
    const double sv = r[R_SIGM] * w;
    const double A1 = __builtin_fma(r[R_G1], x2, -3.0 * sv * LS2);
    const double A2 = __builtin_fma(r[R_G2], x2, -3.0 * sv * LS1);
    const double al1 = p * A1, al2 = p * A2, be = p * sv;
    const double q = -r[R_LAM] * x;

    // ---------------- seed fbar ----------------
    double fb[10];
    if (omega_mode) {
        const double u0 = __builtin_fma(L1, a2, -L2 * a1), u1 = __builtin_fma(L2, a0, -L0 * a2),
                     u2 = __builtin_fma(L0, a1, -L1 * a0);
        const double w0 = __builtin_fma(L1, b2, -L2 * b1), w1 = __builtin_fma(L2, b0, -L0 * b2),
                     w2 = __builtin_fma(L0, b1, -L1 * b0);
        const double C0 = __builtin_fma(a1, b2, -a2 * b1), C1 = __builtin_fma(a2, b0, -a0 * b2),
                     C2 = __builtin_fma(a0, b1, -a1 * b0);
        const double dS1_0 = __builtin_fma(al1, u0, -be * C0), dS1_1 = __builtin_fma(al1, u1, -be * C1),
                     dS1_2 = __builtin_fma(al1, u2, -be * C2);
        const double dS2_0 = __builtin_fma(al2, w0, be * C0), dS2_1 = __builtin_fma(al2, w1, be * C1),
                     dS2_2 = __builtin_fma(al2, w2, be * C2);
        const double s = 1.0 / f0;
        double sbar = 0.0;
        sbar = __builtin_fma(gbar_in[1], dS1_0, sbar);
        sbar = __builtin_fma(gbar_in[2], dS1_1, sbar);
        sbar = __builtin_fma(gbar_in[3], dS1_2, sbar);
        sbar = __builtin_fma(gbar_in[4], dS2_0, sbar);
        sbar = __builtin_fma(gbar_in[5], dS2_1, sbar);
        sbar = __builtin_fma(gbar_in[6], dS2_2, sbar);
        sbar = __builtin_fma(gbar_in[7], q * (dS1_0 + dS2_0), sbar);
        sbar = __builtin_fma(gbar_in[8], q * (dS1_1 + dS2_1), sbar);
        sbar = __builtin_fma(gbar_in[9], q * (dS1_2 + dS2_2), sbar);
        sbar = __builtin_fma(gscale, sbar, gtbar);
        const double gs = gscale * s;
#pragma unroll
        for (int c = 1; c < 10; ++c) fb[c] = gbar_in[c] * gs;
        fb[0] = -(s * s) * sbar;
    } else {
#pragma unroll
        for (int c = 0; c < 10; ++c) fb[c] = gbar_in[c] * gscale;
    }

    // ---------------- reverse ----------------
    // The cross products and the spin derivatives are recomputed below rather
    // than kept from the primal pass (fewer registers live across the VJP);
    // the empty asm keeps the compiler from merging the two computations.
    double ra0 = a0, ra1 = a1, ra2 = a2, rb0_ = b0, rb1_ = b1, rb2_ = b2, rL0 = L0, rL1 = L1, rL2 = L2;
    __asm__ volatile("" : "+v"(ra0), "+v"(ra1), "+v"(ra2), "+v"(rb0_), "+v"(rb1_), "+v"(rb2_), "+v"(rL0),
                     "+v"(rL1), "+v"(rL2));
#define a0 ra0
#define a1 ra1
#define a2 ra2
#define b0 rb0_
#define b1 rb1_
#define b2 rb2_
#define L0 rL0
#define L1 rL1
#define L2 rL2
    const double u0 = __builtin_fma(L1, a2, -L2 * a1), u1 = __builtin_fma(L2, a0, -L0 * a2),
                 u2 = __builtin_fma(L0, a1, -L1 * a0);
    const double w0 = __builtin_fma(L1, b2, -L2 * b1), w1 = __builtin_fma(L2, b0, -L0 * b2),
                 w2 = __builtin_fma(L0, b1, -L1 * b0);
    const double C0 = __builtin_fma(a1, b2, -a2 * b1), C1 = __builtin_fma(a2, b0, -a0 * b2),
                 C2 = __builtin_fma(a0, b1, -a1 * b0);
    // dL = q (dS1 + dS2), dS1 + dS2 = al1 u + al2 w
    const double ds0 = __builtin_fma(al1, u0, al2 * w0), ds1 = __builtin_fma(al1, u1, al2 * w1),
                 ds2 = __builtin_fma(al1, u2, al2 * w2);
    const double qbar = fb[7] * ds0 + fb[8] * ds1 + fb[9] * ds2;
    const double s1b0 = __builtin_fma(q, fb[7], fb[1]), s1b1 = __builtin_fma(q, fb[8], fb[2]),
                 s1b2 = __builtin_fma(q, fb[9], fb[3]);
    const double s2b0 = __builtin_fma(q, fb[7], fb[4]), s2b1 = __builtin_fma(q, fb[8], fb[5]),
                 s2b2 = __builtin_fma(q, fb[9], fb[6]);
    // q = -lam x
    rb.v[R_LAM] = __builtin_fma(-x, qbar, rb.v[R_LAM]);
    double xbar = -r[R_LAM] * qbar;
    // dS1 = al1 u - be C ; dS2 = al2 w + be C
    const double al1b = s1b0 * u0 + s1b1 * u1 + s1b2 * u2;
    const double al2b = s2b0 * w0 + s2b1 * w1 + s2b2 * w2;
    const double beb = (s2b0 - s1b0) * C0 + (s2b1 - s1b1) * C1 + (s2b2 - s1b2) * C2;
    const double ub0 = al1 * s1b0, ub1 = al1 * s1b1, ub2 = al1 * s1b2;
    const double wb0 = al2 * s2b0, wb1 = al2 * s2b1, wb2 = al2 * s2b2;
    const double Cb0 = be * (s2b0 - s1b0), Cb1 = be * (s2b1 - s1b1), Cb2 = be * (s2b2 - s1b2);
    // C = a x b: abar += b x Cbar, bbar += Cbar x a
    double ab0 = __builtin_fma(b1, Cb2, -b2 * Cb1), ab1 = __builtin_fma(b2, Cb0, -b0 * Cb2),
           ab2 = __builtin_fma(b0, Cb1, -b1 * Cb0);
    double bb0 = __builtin_fma(Cb1, a2, -Cb2 * a1), bb1 = __builtin_fma(Cb2, a0, -Cb0 * a2),
           bb2 = __builtin_fma(Cb0, a1, -Cb1 * a0);
    // u = L x a: Lbar += a x ubar, abar += ubar x L
    double Lb0 = __builtin_fma(a1, ub2, -a2 * ub1), Lb1 = __builtin_fma(a2, ub0, -a0 * ub2),
           Lb2 = __builtin_fma(a0, ub1, -a1 * ub0);
    ab0 += __builtin_fma(ub1, L2, -ub2 * L1);
    ab1 += __builtin_fma(ub2, L0, -ub0 * L2);
    ab2 += __builtin_fma(ub0, L1, -ub1 * L0);
    // w = L x b: Lbar += b x wbar, bbar += wbar x L
    Lb0 += __builtin_fma(b1, wb2, -b2 * wb1);
    Lb1 += __builtin_fma(b2, wb0, -b0 * wb2);
    Lb2 += __builtin_fma(b0, wb1, -b1 * wb0);
    bb0 += __builtin_fma(wb1, L2, -wb2 * L1);
    bb1 += __builtin_fma(wb2, L0, -wb0 * L2);
    bb2 += __builtin_fma(wb0, L1, -wb1 * L0);
    // be = p sv ; al1 = p A1 ; al2 = p A2
    double pbar = __builtin_fma(sv, beb, __builtin_fma(A1, al1b, A2 * al2b));
    double svbar = p * beb;
    const double A1b = p * al1b, A2b = p * al2b;
    // A1 = g1 x2 - 3 sv LS2 ; A2 = g2 x2 - 3 sv LS1
    rb.v[R_G1] = __builtin_fma(x2, A1b, rb.v[R_G1]);
    rb.v[R_G2] = __builtin_fma(x2, A2b, rb.v[R_G2]);
    double x2bar = __builtin_fma(r[R_G1], A1b, r[R_G2] * A2b);
    svbar = __builtin_fma(-3.0 * LS2, A1b, __builtin_fma(-3.0 * LS1, A2b, svbar));
    double LS2bar = -3.0 * sv * A1b;
    double LS1bar = -3.0 * sv * A2b;
    // sv = sigM w ; p = w/2
    rb.v[R_SIGM] = __builtin_fma(w, svbar, rb.v[R_SIGM]);
    double wbar = __builtin_fma(r[R_SIGM], svbar, 0.5 * pbar);
    // f0 = K w^2 x5 B
    const double f0b = fb[0];
    rb.v[R_K] = __builtin_fma((w * w) * x5 * B, f0b, rb.v[R_K]);
    wbar = __builtin_fma(2.0 * r[R_K] * w * x5 * B, f0b, wbar);
    const double x5bar = Kw2 * B * f0b;
    const double Bbar = Kw2 * x5 * f0b;
    // x5 = x4 x, x4 = x2^2
    x2bar = __builtin_fma(2.0 * x2 * x, x5bar, x2bar);
    xbar = __builtin_fma(x4, x5bar, xbar);
    // B = 1 + x2 B1
    x2bar = __builtin_fma(B1, Bbar, x2bar);
    const double B1b = x2 * Bbar;
    // Horner chain
    xbar = __builtin_fma(B2, B1b, xbar);
    rb.v[R_C2] += B1b;
    const double B2b = x * B1b;
    xbar = __builtin_fma(B3, B2b, xbar);
    const double c3pb = B2b;
    const double B3b = x * B2b;
    xbar = __builtin_fma(B4, B3b, xbar);
    const double c4pb = B3b;
    const double B4b = x * B3b;
    xbar = __builtin_fma(B5, B4b, xbar);
    rb.v[R_C5] += B4b;
    const double B5b = x * B4b;
    xbar = __builtin_fma(r[R_C7], B5b, xbar);
    rb.v[R_C7] = __builtin_fma(x, B5b, rb.v[R_C7]);
    const double c6pb = B5b;
    // c6p = c6 + c6lnv lnv
    rb.v[R_C6] += c6pb;
    const double lnvbar = tc.c6lnv * c6pb;
    // c4p = c4 - ssd ssb ; ssb = 247 S12 - 721 LS1 LS2
    rb.v[R_C4] += c4pb;
    rb.v[R_SSD] = __builtin_fma(-ssb, c4pb, rb.v[R_SSD]);
    const double ssbb = -r[R_SSD] * c4pb;
    const double S12bar = 247.0 * ssbb;
    LS1bar = __builtin_fma(-721.0 * LS2, ssbb, LS1bar);
    LS2bar = __builtin_fma(-721.0 * LS1, ssbb, LS2bar);
    // c3p = c3 - so1 LS1 - so2 LS2
    rb.v[R_SO1] = __builtin_fma(-LS1, c3pb, rb.v[R_SO1]);
    rb.v[R_SO2] = __builtin_fma(-LS2, c3pb, rb.v[R_SO2]);
    LS1bar = __builtin_fma(-r[R_SO1], c3pb, LS1bar);
    LS2bar = __builtin_fma(-r[R_SO2], c3pb, LS2bar);
    // LS1 = L.a ; LS2 = L.b ; S12 = a.b
    Lb0 = __builtin_fma(a0, LS1bar, __builtin_fma(b0, LS2bar, Lb0));
    Lb1 = __builtin_fma(a1, LS1bar, __builtin_fma(b1, LS2bar, Lb1));
    Lb2 = __builtin_fma(a2, LS1bar, __builtin_fma(b2, LS2bar, Lb2));
    ab0 = __builtin_fma(L0, LS1bar, __builtin_fma(b0, S12bar, ab0));
    ab1 = __builtin_fma(L1, LS1bar, __builtin_fma(b1, S12bar, ab1));
    ab2 = __builtin_fma(L2, LS1bar, __builtin_fma(b2, S12bar, ab2));
    bb0 = __builtin_fma(L0, LS2bar, __builtin_fma(a0, S12bar, bb0));
    bb1 = __builtin_fma(L1, LS2bar, __builtin_fma(a1, S12bar, bb1));
    bb2 = __builtin_fma(L2, LS2bar, __builtin_fma(a2, S12bar, bb2));
    // x2 = x x ; lnv = ln|v| ; x = cbrt(v) ; v = M w
    xbar = __builtin_fma(2.0 * x, x2bar, xbar);
    // d lnv/dv = 1/v, dx/dv = 1/(3 x^2) = x/(3 v): one reciprocal of v
    // (hardware seed and two Newton steps; valid for either sign)
    const double rv = rcp_pos(v);
    const double vbar = rv * __builtin_fma(xbar, x * (1.0 / 3.0), lnvbar);
    rb.v[R_M] = __builtin_fma(w, vbar, rb.v[R_M]);
    wbar = __builtin_fma(M, vbar, wbar);

    ybar[0] = wbar;
    ybar[1] = ab0; ybar[2] = ab1; ybar[3] = ab2;
    ybar[4] = bb0; ybar[5] = bb1; ybar[6] = bb2;
    ybar[7] = Lb0; ybar[8] = Lb1; ybar[9] = Lb2;
#undef a0
#undef a1
#undef a2
#undef b0
#undef b1
#undef b2
#undef L0
#undef L1
#undef L2
}

// ---------------------------------------------------------------------------
// d(row)/d(m1), d(row)/d(m2): make_row() evaluated on dual numbers.
// ---------------------------------------------------------------------------
struct Dl {
    double v, d;
    __device__ Dl() : v(0), d(0) {}
    __device__ Dl(double a) : v(a), d(0) {}
    __device__ Dl(double a, double b) : v(a), d(b) {}
};
__device__ __forceinline__ Dl operator+(Dl a, Dl b) { return Dl(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dl operator-(Dl a, Dl b) { return Dl(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dl operator-(Dl a) { return Dl(-a.v, -a.d); }
__device__ __forceinline__ Dl operator*(Dl a, Dl b) { return Dl(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ Dl operator/(Dl a, Dl b) {
    const double q = a.v / b.v;
    return Dl(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ Dl operator*(double a, Dl b) { return Dl(a * b.v, a * b.d); }
__device__ __forceinline__ Dl operator*(Dl a, double b) { return Dl(a.v * b, a.d * b); }
__device__ __forceinline__ Dl operator+(double a, Dl b) { return Dl(a + b.v, b.d); }
__device__ __forceinline__ Dl operator/(Dl a, double b) { return Dl(a.v / b, a.d / b); }
__device__ __forceinline__ Dl operator/(double a, Dl b) { return Dl(a) / b; }

struct RowDual {
    Dl v[NROW];
    __device__ __forceinline__ void set(int i, Dl x) { v[i] = x; }
};

// make_row() again, written on dual numbers (same expressions).
__device__ __forceinline__ void make_row_dual(RowDual& r, Dl m1, Dl m2, int terms, int theta_literal) {
    const Dl M = m1 + m2;
    const Dl iM = 1.0 / M;
    const Dl eta = m1 * m2 * iM * iM;
    const double pn = (terms & PN_TERM_PN) ? 1.0 : 0.0;
    const double fso = (terms & PN_TERM_SO_WDOT) ? 1.0 : 0.0;
    const double fss = (terms & PN_TERM_SS_WDOT) ? 1.0 : 0.0;
    r.set(R_M, M);
    r.set(R_C2, pn * ((-(743.0 + 924.0 * eta)) / 336.0));
    r.set(R_SO1, fso * ((113.0 * m1 * m1 * iM * iM + 75.0 * eta) / (12.0 * m1 * m1)));
    r.set(R_SO2, fso * ((113.0 * m2 * m2 * iM * iM + 75.0 * eta) / (12.0 * m2 * m2)));
    r.set(R_C4, pn * (34103.0 / 18144.0 + (13661.0 / 2016.0) * eta + (59.0 / 18.0) * eta * eta));
    r.set(R_SSD, fss * (eta / (48.0 * m1 * m1 * m2 * m2)));
    r.set(R_C5, pn * ((-(4159.0 + 15876.0 * eta)) * (PN_PI / 672.0)));
    const Dl theta_term = (88.0 / 3.0) * (1039.0 / 4620.0) * (theta_literal ? eta : Dl(1.0));
    const double c6c = (16447322263.0 / 139708800.0) - (1712.0 / 105.0) * PN_GAMMA_E + (16.0 / 3.0) * PN_PI * PN_PI
                     - (856.0 / 105.0) * PN_LN16;
    r.set(R_C6, pn * (c6c + (-273811877.0 / 1088640.0 + (451.0 / 48.0) * PN_PI * PN_PI - theta_term) * eta
                      + (541.0 / 896.0) * eta * eta - (5605.0 / 2592.0) * eta * eta * eta));
    r.set(R_C7, pn * ((-4415.0 / 4032.0 + (358675.0 / 6048.0) * eta + (91495.0 / 1512.0) * eta * eta) * PN_PI));
    r.set(R_K, (terms & PN_TERM_RR) ? (96.0 / 5.0) * eta : Dl(0.0));
    r.set(R_G1, (terms & PN_TERM_SO_PREC) ? eta * (4.0 + 3.0 * m2 / m1) : Dl(0.0));
    r.set(R_G2, (terms & PN_TERM_SO_PREC) ? eta * (4.0 + 3.0 * m1 / m2) : Dl(0.0));
    r.set(R_SIGM, (terms & PN_TERM_SS_PREC) ? iM : Dl(0.0));
    r.set(R_LAM, 1.0 / (eta * M * M));
}

__device__ __forceinline__ Dl operator-(double a, Dl b) { return Dl(a - b.v, -b.d); }

}  // namespace pn
