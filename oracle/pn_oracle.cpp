/*
 * pn_oracle.cpp -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * The CPU oracle for batched integration of precessing post-Newtonian
 * binary-black-hole inspirals (Herrmann, Silberholz, Bellone, Guerberoff,
 * Tiglio, "Integrating Post-Newtonian Equations on Graphics Processing
 * Units", arXiv:0908.3889).  Plain, slow and written to be checked against
 * the paper by eye.  Only the tests, the smoke check and the benchmark's CPU
 * baseline load it.  It shares no code, header or constant table with the
 * GPU library.
 *
 * What it computes, and where the paper defines it:
 *   - the right-hand side of the ODE system for the state
 *       y = (omega, S1[3], S2[3], L_hat[3])
 *     Eq. (1) omega-dot, Eq. (2) spin precession, Eq. (3) L_hat-dot and
 *     Eq. (4) the precession vector Omega_1 (Omega_2 by exchanging 1 <-> 2);
 *     masses and the spin parametrisation S_i = chi_i m_i^2 S_hat_i are from
 *     Sec. II;
 *   - the integration of that system from omega0 to omega_f with the
 *     Dormand-Prince method, tolerance tol and initial step h = 10 (Sec. II);
 *   - the unit-vector scalar products S1_hat.S2_hat, S_i_hat.L_hat used to
 *     analyse the final states (Sec. V);
 *   - on request, the orbital phase Phi(t) = integral of omega dt from 0
 *     (not a quantity of the paper: an added output for waveform-style use),
 *     integrated by the same Dormand-Prince steps as a pure quadrature: its
 *     derivative omega does not depend on Phi, so only the stage values of
 *     omega enter, and Phi is left out of the error norm, so the step
 *     sequence is the one without it.
 *
 * Readings taken where the paper is silent or ambiguous:
 *   R1  the 3PN term: theta_hat multiplies eta once, i.e. the bracket is
 *       (-273811877/1088640 + 451/48 pi^2 - 88/3 theta_hat) eta; the literal
 *       printed form with an extra factor eta is available as a flag;
 *   R2  "log" is the natural logarithm;  R3  gamma_E to full double precision;
 *   R4  chi_i L_hat.S_hat_i is evaluated as L_hat.S_i / m_i^2 and
 *       chi_1 chi_2 (S_hat_1.S_hat_2) as S1.S2/(m1^2 m2^2) (equal on the
 *       exact flow, where |S_i| = chi_i m_i^2 is conserved);
 *   R5  Omega_2 swaps m1 <-> m2 and S1 <-> S2 everywhere in Eq. (4);
 *   R6  Dormand-Prince RK5(4)7M with FSAL, advancing with the 5th-order
 *       solution (Dormand & Prince 1980; Hairer, Norsett & Wanner vol. I);
 *   R7  atol = rtol = tol, root-mean-square mixed norm over the 10 state
 *       components;
 *   R8  step controller: safety 0.9, exponent 1/5, growth factor clamped to
 *       [0.2, 5], no growth right after a rejection;
 *   R9  h0 = 10 (units of M);
 *   R10 "integrate to omega_f": a t-step whose accepted candidate passes
 *       omega_f is discarded and the remaining stretch is integrated with
 *       omega as the independent variable, with the same Dormand-Prince
 *       stepper and controller, each omega-step clipped to the distance
 *       left, ending exactly at omega = omega_f;
 *   R11 no renormalisation of S_i or L_hat during the integration;
 *   R12 observables use the current vector norms and are 0 when a norm is 0;
 *   R21 the orbital phase (not a quantity of the paper) is the integral of
 *       omega dt from 0, taken on the accepted steps as described above.
 *
 * Pins of the step sequence: the paper prints no trajectory, no step count
 * and no controller constants.  The error norm and the controller (R7, R8)
 * are pinned by SciPy's RK45, an independent implementation of the same
 * pair and controller, whose accepted time steps and rejections the tests
 * compare with these.  The omega stretch (R10) is one step on every
 * workload (the first omega-step, the whole distance left, is accepted);
 * SciPy's RK45 in omega, started from the state after the recorded time
 * steps, takes the same single step to the same spins, L_hat and t.  The
 * stretch is also pinned through convergence to closed forms, an
 * event-located library integration and the paper's printed correlation
 * coefficients (Sec. V A).
 *
 * The stage sums skip the tableau's structural zeros (a_sj = 0, and
 * b_j = bhat_j = 0 in the error estimate): the method's sums run over the
 * nonzero weights only, so a stage derivative that is infinite where its
 * weight is structurally zero must not turn the sum into 0 * inf = NaN,
 * and the operation counts of the counting scalar are the method's.
 *
 * Build: g++ -O2 -std=c++17 -fno-fast-math -ffp-contract=off -shared -fPIC.
 */
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

/* ------------------------------------------------------------------ */
/* Scalar types: double, a forward-mode dual number and a counting type */
/* ------------------------------------------------------------------ */

inline double val(double x) { return x; }

/* Forward-mode dual number: v + d*eps with eps^2 = 0. */
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double a) : v(a), d(0) {}
    Dual(double a, double b) : v(a), d(b) {}
};
inline double val(const Dual& x) { return x.v; }
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
inline Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
inline Dual& operator*=(Dual& a, Dual b) { return a = a * b; }
inline Dual cbrt(Dual a) { double c = std::cbrt(a.v); return Dual(c, a.d / (3.0 * c * c)); }
inline Dual log(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
inline Dual pow(Dual a, double e) {
    double p = std::pow(a.v, e);
    return Dual(p, e * std::pow(a.v, e - 1.0) * a.d);
}
inline Dual fabs(Dual a) { return a.v < 0 ? -a : a; }
inline bool isfinite(Dual a) { return std::isfinite(a.v) && std::isfinite(a.d); }

/* Counting scalar: counts the floating-point operations whose result
 * depends on the integration state ("tainted"); operations between
 * per-inspiral constants (masses and numbers derived only from them) are
 * not counted.  add, sub, mul and div count one FLOP each; cbrt, log, sqrt
 * and pow are counted separately as special functions. */
struct OpCounts {
    long long add, mul, div, cbrt_, log_, sqrt_, pow_;
};
thread_local OpCounts g_ops;

struct Counted {
    double v;
    bool t;
    Counted() : v(0), t(false) {}
    Counted(double a) : v(a), t(false) {}
    Counted(double a, bool tt) : v(a), t(tt) {}
};
inline double val(const Counted& x) { return x.v; }
inline Counted operator+(Counted a, Counted b) {
    bool t = a.t || b.t; if (t) g_ops.add++; return Counted(a.v + b.v, t);
}
inline Counted operator-(Counted a, Counted b) {
    bool t = a.t || b.t; if (t) g_ops.add++; return Counted(a.v - b.v, t);
}
inline Counted operator-(Counted a) { return Counted(-a.v, a.t); }
inline Counted operator*(Counted a, Counted b) {
    bool t = a.t || b.t; if (t) g_ops.mul++; return Counted(a.v * b.v, t);
}
inline Counted operator/(Counted a, Counted b) {
    bool t = a.t || b.t; if (t) g_ops.div++; return Counted(a.v / b.v, t);
}
inline Counted& operator+=(Counted& a, Counted b) { return a = a + b; }
inline Counted& operator-=(Counted& a, Counted b) { return a = a - b; }
inline Counted& operator*=(Counted& a, Counted b) { return a = a * b; }
inline Counted cbrt(Counted a) { if (a.t) g_ops.cbrt_++; return Counted(std::cbrt(a.v), a.t); }
inline Counted log(Counted a) { if (a.t) g_ops.log_++; return Counted(std::log(a.v), a.t); }
inline Counted sqrt(Counted a) { if (a.t) g_ops.sqrt_++; return Counted(std::sqrt(a.v), a.t); }
inline Counted pow(Counted a, double e) { if (a.t) g_ops.pow_++; return Counted(std::pow(a.v, e), a.t); }
inline Counted fabs(Counted a) { return Counted(std::fabs(a.v), a.t); }
inline bool isfinite(Counted a) { return std::isfinite(a.v); }

template <class T> inline T tmax(const T& a, const T& b) { return val(a) >= val(b) ? a : b; }
template <class T> inline T tmin(const T& a, const T& b) { return val(a) <= val(b) ? a : b; }

/* ------------------------------------------------------------------ */
/* Constants of Eq. (1)                                                 */
/* ------------------------------------------------------------------ */

const double PI = 3.14159265358979323846264338327950288;
const double GAMMA_E = 0.57721566490153286060651209008240243; /* Euler's constant (R3) */
const double THETA_HAT = 1039.0 / 4620.0;                       /* given after Eq. (3) */

/* Term switches.  All on reproduces Eqs. (1)-(4); subsets serve the tests
 * (closed forms and conservation laws hold for some subsets only). */
enum {
    TERM_PN = 1,        /* non-spinning corrections of Eq. (1): (Mw)^{2/3} ... (Mw)^{7/3} */
    TERM_SO_WDOT = 2,   /* spin-orbit term of Eq. (1), the sum over i of chi_i L.S_hat_i */
    TERM_SS_WDOT = 4,   /* spin-spin term of Eq. (1), the chi_1 chi_2 (247 ... - 721 ...) term */
    TERM_RR = 8,        /* omega-dot itself (radiation reaction); off => omega constant */
    TERM_SO_PREC = 16,  /* the L_hat part of Eq. (4) */
    TERM_SS_PREC = 32,  /* the S_j - 3 (S_j.L_hat) L_hat part of Eq. (4) */
    TERM_ALL = 63
};

/* ------------------------------------------------------------------ */
/* Right-hand side, Eqs. (1)-(4)                                       */
/* ------------------------------------------------------------------ */

/* y[0] = omega, y[1..3] = S1, y[4..6] = S2, y[7..9] = L_hat.  Writes dy/dt. */
template <class T>
void rhs(const T& m1, const T& m2, const T* y, T* dy, int terms, int theta_literal) {
    using std::cbrt; using std::log;
    const T M = m1 + m2;
    const T eta = m1 * m2 / (M * M);                 /* symmetric mass ratio, Sec. II */
    const T omega = y[0];
    const T S1[3] = {y[1], y[2], y[3]};
    const T S2[3] = {y[4], y[5], y[6]};
    const T L[3] = {y[7], y[8], y[9]};

    const T Mw = M * omega;                          /* M omega */
    const T x = cbrt(Mw);                            /* (M omega)^{1/3} */
    const T x2 = x * x, x3 = x2 * x, x4 = x3 * x, x5 = x4 * x, x6 = x5 * x, x7 = x6 * x;

    const T LS1 = L[0] * S1[0] + L[1] * S1[1] + L[2] * S1[2];
    const T LS2 = L[0] * S2[0] + L[1] * S2[1] + L[2] * S2[2];
    const T S12 = S1[0] * S2[0] + S1[1] * S2[1] + S1[2] * S2[2];

    /* Eq. (1): the curly bracket, term by term in the printed order. */
    T B = T(1.0);
    if (terms & TERM_PN) {
        B = B - (743.0 + 924.0 * eta) / 336.0 * x2;                      /* (Mw)^{2/3} */
    }
    {
        T so = T(0.0);
        if (terms & TERM_SO_WDOT) {
            /* (1/12) sum_i chi_i L.S_hat_i (113 m_i^2/M^2 + 75 eta), with R4 */
            so = (LS1 / (m1 * m1) * (113.0 * m1 * m1 / (M * M) + 75.0 * eta) +
                  LS2 / (m2 * m2) * (113.0 * m2 * m2 / (M * M) + 75.0 * eta)) / 12.0;
        }
        T four_pi = (terms & TERM_PN) ? T(4.0 * PI) : T(0.0);
        B = B - (so - four_pi) * x3;                                     /* (Mw)^{1} */
    }
    if (terms & TERM_PN) {
        B = B + (34103.0 / 18144.0 + 13661.0 / 2016.0 * eta + 59.0 / 18.0 * eta * eta) * x4;
    }
    if (terms & TERM_SS_WDOT) {
        /* (1/48) eta chi_1 chi_2 (247 S_hat_1.S_hat_2 - 721 (L.S_hat_1)(L.S_hat_2)), with R4 */
        B = B - eta / 48.0 * (247.0 * S12 - 721.0 * LS1 * LS2) / (m1 * m1 * m2 * m2) * x4;
    }
    if (terms & TERM_PN) {
        B = B - (4159.0 + 15876.0 * eta) * PI / 672.0 * x5;               /* (Mw)^{5/3} */
        const T theta_fac = theta_literal ? eta : T(1.0);                /* R1 */
        const T c6 = (16447322263.0 / 139708800.0 - 1712.0 / 105.0 * GAMMA_E + 16.0 / 3.0 * PI * PI)
                   + (-273811877.0 / 1088640.0 + 451.0 / 48.0 * PI * PI - 88.0 / 3.0 * THETA_HAT * theta_fac) * eta
                   + 541.0 / 896.0 * eta * eta - 5605.0 / 2592.0 * eta * eta * eta
                   - 856.0 / 105.0 * log(16.0 * x2);                     /* log(16 (Mw)^{2/3}), R2 */
        B = B + c6 * x6;                                                 /* (Mw)^{2} */
        B = B + (-4415.0 / 4032.0 + 358675.0 / 6048.0 * eta + 91495.0 / 1512.0 * eta * eta) * PI * x7;
    }
    /* omega-dot = omega^2 (96/5) eta (M omega)^{5/3} {...} */
    dy[0] = (terms & TERM_RR) ? omega * omega * 96.0 / 5.0 * eta * x5 * B : T(0.0);

    /* Eq. (4): Omega_1 = ((Mw)^2 / (2M)) ( eta (Mw)^{-1/3} (4 + 3 m2/m1) L_hat
     *                                       + (1/M^2)(S2 - 3 (S2.L_hat) L_hat) );
     * Omega_2 by 1 <-> 2 (R5). */
    const T pre = Mw * Mw / (2.0 * M);
    const T so1 = (terms & TERM_SO_PREC) ? eta / x * (4.0 + 3.0 * m2 / m1) : T(0.0);
    const T so2 = (terms & TERM_SO_PREC) ? eta / x * (4.0 + 3.0 * m1 / m2) : T(0.0);
    const T ss = (terms & TERM_SS_PREC) ? 1.0 / (M * M) : T(0.0);
    T Om1[3], Om2[3];
    for (int c = 0; c < 3; ++c) {
        Om1[c] = pre * (so1 * L[c] + ss * (S2[c] - 3.0 * LS2 * L[c]));
        Om2[c] = pre * (so2 * L[c] + ss * (S1[c] - 3.0 * LS1 * L[c]));
    }
    /* Eq. (2): dS_i/dt = Omega_i x S_i */
    T dS1[3], dS2[3];
    dS1[0] = Om1[1] * S1[2] - Om1[2] * S1[1];
    dS1[1] = Om1[2] * S1[0] - Om1[0] * S1[2];
    dS1[2] = Om1[0] * S1[1] - Om1[1] * S1[0];
    dS2[0] = Om2[1] * S2[2] - Om2[2] * S2[1];
    dS2[1] = Om2[2] * S2[0] - Om2[0] * S2[2];
    dS2[2] = Om2[0] * S2[1] - Om2[1] * S2[0];
    /* Eq. (3): dL_hat/dt = -((Mw)^{1/3} / (eta M^2)) (dS1/dt + dS2/dt) */
    const T lpre = x / (eta * M * M);
    for (int c = 0; c < 3; ++c) {
        dy[1 + c] = dS1[c];
        dy[4 + c] = dS2[c];
        dy[7 + c] = T(0.0) - lpre * (dS1[c] + dS2[c]);
    }
}

/* ------------------------------------------------------------------ */
/* Dormand-Prince RK5(4)7M tableau (Dormand & Prince 1980), as exact     */
/* rationals (numerator, denominator)                                   */
/* ------------------------------------------------------------------ */

struct Rat { double num, den; };

/* A[s][j], stage s = 1..6 (0-based rows 1..6), j < s */
const Rat DP_A[7][6] = {
    {{0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
    {{1, 5}, {0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
    {{3, 40}, {9, 40}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
    {{44, 45}, {-56, 15}, {32, 9}, {0, 1}, {0, 1}, {0, 1}},
    {{19372, 6561}, {-25360, 2187}, {64448, 6561}, {-212, 729}, {0, 1}, {0, 1}},
    {{9017, 3168}, {-355, 33}, {46732, 5247}, {49, 176}, {-5103, 18656}, {0, 1}},
    {{35, 384}, {0, 1}, {500, 1113}, {125, 192}, {-2187, 6784}, {11, 84}},
};
const Rat DP_C[7] = {{0, 1}, {1, 5}, {3, 10}, {4, 5}, {8, 9}, {1, 1}, {1, 1}};
/* 5th-order weights (= last row of A, FSAL) and embedded 4th-order weights */
const Rat DP_B[7] = {{35, 384}, {0, 1}, {500, 1113}, {125, 192}, {-2187, 6784}, {11, 84}, {0, 1}};
const Rat DP_BHAT[7] = {{5179, 57600}, {0, 1}, {7571, 16695}, {393, 640},
                        {-92097, 339200}, {187, 2100}, {1, 40}};

inline double rv(const Rat& r) { return r.num / r.den; }

/* ------------------------------------------------------------------ */
/* Integration from omega0 to omega_f (Sec. II)                         */
/* ------------------------------------------------------------------ */

enum {
    ST_OK = 0, ST_DONE_AT_START = 1, ST_MAX_STEPS = -1, ST_H_UNDERFLOW = -2,
    ST_NONFINITE = -3, ST_BAD_INPUT = -4, ST_OMEGADOT_NONPOSITIVE = -5
};

struct Mode {
    double omega_f, tol, h0, h_fixed, t_end;
    long long max_steps;
    int terms, theta_literal;
    /* replay: accepted t-steps, then all omega-steps but the last (which goes
     * to omega_f); NULL when not replaying */
    const double* replay; int n_replay_t, n_replay_w;
    /* record of accepted steps (same layout as replay); NULL when not recording */
    double* record; long long record_cap;
    bool phase;        /* also integrate the orbital phase */
};

template <class T>
struct Result {
    T y[10];
    T t;
    T phase;           /* integral of omega dt (when requested) */
    long long acc, rej, nrhs;
    int status;
    int n_t, n_w;      /* accepted t-steps and omega-steps */
};

/* g = dy/dt (mode t) or dy/domega (mode omega): in omega mode the RHS is
 * divided by omega-dot and the omega component becomes 1; dt/domega =
 * 1/omega-dot is returned in *dt_dvar (1 in mode t). */
template <class T>
void deriv(const T& m1, const T& m2, const T* y, T* g, T* dt_dvar, bool omega_mode,
           const Mode& md) {
    rhs(m1, m2, y, g, md.terms, md.theta_literal);
    if (!omega_mode) { *dt_dvar = T(1.0); return; }
    const T inv = T(1.0) / g[0];
    for (int c = 1; c < 10; ++c) g[c] = g[c] * inv;
    g[0] = T(1.0);
    *dt_dvar = inv;
}

template <class T>
Result<T> integrate_one(const T& m1, const T& m2, const T* y0, const Mode& md) {
    using std::sqrt; using std::pow; using std::fabs; using std::isfinite;
    Result<T> r;
    for (int c = 0; c < 10; ++c) r.y[c] = y0[c];
    r.t = T(0.0); r.phase = T(0.0); r.acc = r.rej = r.nrhs = 0; r.status = ST_OK; r.n_t = r.n_w = 0;

    bool bad = !(val(m1) > 0.0) || !(val(m2) > 0.0) || !(val(y0[0]) > 0.0);
    for (int c = 0; c < 10; ++c) bad = bad || !std::isfinite(val(y0[c]));
    bad = bad || !std::isfinite(val(m1)) || !std::isfinite(val(m2));
    if (bad) { r.status = ST_BAD_INPUT; return r; }

    const bool t_end_mode = md.t_end > 0.0;
    const bool fixed = md.h_fixed > 0.0;
    const bool replay = md.replay != nullptr;
    if (!t_end_mode && !(val(y0[0]) < md.omega_f)) { r.status = ST_DONE_AT_START; return r; }

    T k[7][10], dtv[7];
    T kp[7];           /* d Phi / d(variable) = omega dt/d(variable) at each stage */
    T y[10], Y[10], y5[10];
    for (int c = 0; c < 10; ++c) y[c] = y0[c];
    bool omega_mode = false;
    deriv(m1, m2, y, k[0], &dtv[0], omega_mode, md);
    if (md.phase) kp[0] = y[0] * dtv[0];
    r.nrhs = 1;

    T h = T(fixed ? md.h_fixed : (md.h0 > 0.0 ? md.h0 : 10.0));   /* R9 */
    bool last_rejected = false;
    int replay_pos = 0;

    for (;;) {
        if (r.acc + r.rej >= md.max_steps) { r.status = ST_MAX_STEPS; break; }
        if (!omega_mode && (md.terms & TERM_RR) && val(k[0][0]) <= 0.0) {
            r.status = ST_OMEGADOT_NONPOSITIVE; break;
        }
        if (omega_mode && val(dtv[0]) <= 0.0) { r.status = ST_OMEGADOT_NONPOSITIVE; break; }

        /* the step to attempt */
        bool last = false;   /* this step ends the integration if accepted */
        T htry = h;
        if (replay) {
            if (!omega_mode) {
                if (replay_pos < md.n_replay_t) {
                    htry = T(md.replay[replay_pos]);
                } else if (t_end_mode || md.n_replay_w <= 0) {
                    break;                                    /* nothing left to replay */
                } else {
                    omega_mode = true;                        /* switch as the record did */
                    const T inv = T(1.0) / k[0][0];
                    dtv[0] = inv;
                    for (int c = 1; c < 10; ++c) k[0][c] = k[0][c] * inv;
                    k[0][0] = T(1.0);
                    if (md.phase) kp[0] = y[0] * inv;
                    continue;
                }
            }
            if (omega_mode) {
                int wpos = replay_pos - md.n_replay_t;
                if (wpos < md.n_replay_w - 1) {
                    htry = T(md.replay[replay_pos]);
                } else {
                    htry = T(md.omega_f) - y[0];
                    last = true;
                }
            }
        } else if (omega_mode) {
            const T remain = T(md.omega_f) - y[0];
            if (val(htry) >= val(remain)) { htry = remain; last = true; }
        } else if (t_end_mode) {
            const T remain = T(md.t_end) - r.t;
            if (val(htry) >= val(remain)) { htry = remain; last = true; }
        }

        /* Dormand-Prince stages 2..7: Y_s = y + h sum_{j<s} a_sj k_j */
        for (int s = 1; s < 7; ++s) {
            for (int c = 0; c < 10; ++c) {
                T acc = T(0.0);
                for (int j = 0; j < s; ++j) {
                    if (DP_A[s][j].num == 0) continue;          /* structural zero */
                    acc = acc + rv(DP_A[s][j]) * k[j][c];
                }
                Y[c] = y[c] + htry * acc;
            }
            deriv(m1, m2, Y, k[s], &dtv[s], omega_mode, md);
            if (md.phase) kp[s] = Y[0] * dtv[s];
            r.nrhs += 1;
        }
        for (int c = 0; c < 10; ++c) y5[c] = Y[c];   /* stage 7 point = 5th-order solution */

        /* embedded error estimate and its norm (R7) */
        T err = T(0.0);
        if (!fixed && !replay) {
            T sum = T(0.0);
            for (int c = 0; c < 10; ++c) {
                T e = T(0.0);
                for (int j = 0; j < 7; ++j) {
                    if (DP_B[j].num == 0 && DP_BHAT[j].num == 0) continue;   /* structural zero */
                    e = e + (rv(DP_B[j]) - rv(DP_BHAT[j])) * k[j][c];
                }
                e = htry * e;
                const T sc = md.tol + md.tol * tmax(fabs(y[c]), fabs(y5[c]));
                const T q = e / sc;
                sum = sum + q * q;
            }
            err = sqrt(sum / 10.0);
            /* a NaN error or a non-finite candidate is a failure; an infinite
             * error with a finite candidate is only a (very) rejected step */
            bool fin = !std::isnan(val(err));
            for (int c = 0; c < 10; ++c) fin = fin && std::isfinite(val(y5[c]));
            if (!fin) { r.status = ST_NONFINITE; break; }
        } else {
            bool fin = true;
            for (int c = 0; c < 10; ++c) fin = fin && std::isfinite(val(y5[c]));
            if (!fin) { r.status = ST_NONFINITE; break; }
        }

        if (val(err) <= 1.0) {
            /* candidate passes omega_f in time mode: discard it and finish in omega (R10) */
            if (!omega_mode && !t_end_mode && !replay && val(y5[0]) > md.omega_f) {
                omega_mode = true;
                const T inv = T(1.0) / k[0][0];
                dtv[0] = inv;
                for (int c = 1; c < 10; ++c) k[0][c] = k[0][c] * inv;
                k[0][0] = T(1.0);
                if (md.phase) kp[0] = y[0] * inv;
                h = T(md.omega_f) - y[0];
                last_rejected = false;
                continue;
            }
            /* accept */
            if (omega_mode) {
                T dt = T(0.0);
                for (int j = 0; j < 7; ++j) {
                    if (DP_B[j].num == 0) continue;
                    dt = dt + rv(DP_B[j]) * dtv[j];
                }
                r.t = r.t + htry * dt;
            } else {
                r.t = r.t + htry;
            }
            if (md.phase) {
                /* the 5th-order weights applied to d Phi / d(variable) */
                T dphi = T(0.0);
                for (int j = 0; j < 7; ++j) {
                    if (DP_B[j].num == 0) continue;
                    dphi = dphi + rv(DP_B[j]) * kp[j];
                }
                r.phase = r.phase + htry * dphi;
                kp[0] = kp[6];
            }
            for (int c = 0; c < 10; ++c) y[c] = y5[c];
            if (md.record && replay_pos < md.record_cap) md.record[replay_pos] = val(htry);
            replay_pos++;
            r.acc++;
            if (omega_mode) r.n_w++; else r.n_t++;
            for (int c = 0; c < 10; ++c) k[0][c] = k[6][c];
            dtv[0] = dtv[6];
            if (!omega_mode && !t_end_mode && val(y[0]) == md.omega_f) last = true;
            if (last) {
                if (omega_mode) y[0] = T(md.omega_f);
                break;
            }
            if (!fixed && !replay) {
                T fac = val(err) == 0.0 ? T(5.0)
                       : tmin(T(5.0), tmax(T(0.2), 0.9 * pow(err, -0.2)));     /* R8 */
                if (last_rejected) fac = tmin(fac, T(1.0));
                h = htry * fac;
                last_rejected = false;
            }
        } else {
            r.rej++;
            const T fac = tmax(T(0.2), 0.9 * pow(err, -0.2));
            h = htry * fac;
            last_rejected = true;
            const double scale = omega_mode ? std::fabs(val(y[0])) : std::max(1.0, std::fabs(val(r.t)));
            if (val(h) < 1e-14 * scale) { r.status = ST_H_UNDERFLOW; break; }
        }
    }
    for (int c = 0; c < 10; ++c) r.y[c] = y[c];
    return r;
}

/* Unit-vector scalar products of Sec. V (R12). */
void observables(const double* y, double* d) {
    const double* S1 = y + 1; const double* S2 = y + 4; const double* L = y + 7;
    const double n1 = std::sqrt(S1[0] * S1[0] + S1[1] * S1[1] + S1[2] * S1[2]);
    const double n2 = std::sqrt(S2[0] * S2[0] + S2[1] * S2[1] + S2[2] * S2[2]);
    const double nl = std::sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
    const double s12 = S1[0] * S2[0] + S1[1] * S2[1] + S1[2] * S2[2];
    const double s1l = S1[0] * L[0] + S1[1] * L[1] + S1[2] * L[2];
    const double s2l = S2[0] * L[0] + S2[1] * L[1] + S2[2] * L[2];
    d[0] = (n1 > 0 && n2 > 0) ? s12 / (n1 * n2) : 0.0;
    d[1] = (n1 > 0 && nl > 0) ? s1l / (n1 * nl) : 0.0;
    d[2] = (n2 > 0 && nl > 0) ? s2l / (n2 * nl) : 0.0;
}

template <class F>
void parallel_for(int64_t n, int nthreads, F f) {
    if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
    if (n < 2 || nthreads == 1) { for (int64_t i = 0; i < n; ++i) f(i); return; }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> pool;
    const int nt = (int)std::min<int64_t>(nthreads, n);
    for (int w = 0; w < nt; ++w) {
        pool.emplace_back([&]() {
            for (;;) {
                int64_t i = next.fetch_add(1);
                if (i >= n) break;
                f(i);
            }
        });
    }
    for (auto& th : pool) th.join();
}

} /* namespace */

/* ------------------------------------------------------------------ */
/* C interface (ctypes).  Arrays are structure-of-arrays, float64,      */
/* component c of inspiral i at p[c*n + i].                             */
/* ------------------------------------------------------------------ */

extern "C" {

typedef struct oracle_opts {
    double h0;            /* initial step; <= 0 -> 10 */
    double h_fixed;       /* > 0: fixed step, no error control */
    double t_end;         /* > 0: integrate to t = t_end, no omega_f termination */
    int64_t max_steps;    /* <= 0 -> 10,000,000 */
    int32_t terms;        /* <= 0 -> all terms */
    int32_t theta_literal;
    /* replay (may be NULL): per inspiral i, replay + i*replay_stride holds the
     * accepted t-steps then the omega-steps except the last */
    const double* replay;
    const int32_t* n_replay_t;
    const int32_t* n_replay_w;
    int64_t replay_stride;
    /* record (may be NULL): same layout */
    double* record;
    int64_t record_stride;
} oracle_opts;

static Mode make_mode(double omega_f, double tol, const oracle_opts* o) {
    Mode md;
    md.omega_f = omega_f; md.tol = tol;
    md.h0 = (o && o->h0 > 0) ? o->h0 : 10.0;
    md.h_fixed = o ? o->h_fixed : 0.0;
    md.t_end = o ? o->t_end : 0.0;
    md.max_steps = (o && o->max_steps > 0) ? o->max_steps : 10000000LL;
    md.terms = (o && o->terms > 0) ? o->terms : TERM_ALL;
    md.theta_literal = o ? o->theta_literal : 0;
    md.replay = nullptr; md.n_replay_t = 0; md.n_replay_w = 0;
    md.record = nullptr; md.record_cap = 0;
    md.phase = false;
    return md;
}

/* Eqs. (1)-(4) pointwise: y [10][n], m [2][n] -> dydt [10][n]. */
int oracle_rhs(int64_t n, const double* m, const double* y, double* dydt, int32_t terms,
               int32_t theta_literal) {
    if (terms <= 0) terms = TERM_ALL;
    for (int64_t i = 0; i < n; ++i) {
        double yy[10], dd[10];
        for (int c = 0; c < 10; ++c) yy[c] = y[c * n + i];
        rhs(m[i], m[n + i], yy, dd, terms, theta_literal);
        for (int c = 0; c < 10; ++c) dydt[c * n + i] = dd[c];
    }
    return 0;
}

/* Integrate n inspirals.  m [2][n], S0 [6][n], L0 [3][n], omega0 [n];
 * outputs y_final [10][n], t_final [n], steps [3][n] (accepted, rejected,
 * RHS evaluations), status [n], n_steps_tw [2][n] (accepted t-steps and
 * omega-steps; may be NULL), phase [n] (the orbital phase at t_final; may be
 * NULL, and then it is not integrated). */
int oracle_integrate(int64_t n, const double* m, const double* S0, const double* L0,
                     const double* omega0, double omega_f, double tol, const oracle_opts* o,
                     double* y_final, double* t_final, int64_t* steps, int32_t* status,
                     int32_t* n_steps_tw, double* phase, int32_t nthreads) {
    Mode base = make_mode(omega_f, tol, o);
    base.phase = phase != nullptr;
    parallel_for(n, nthreads, [&](int64_t i) {
        Mode md = base;
        if (o && o->replay) {
            md.replay = o->replay + i * o->replay_stride;
            md.n_replay_t = o->n_replay_t[i];
            md.n_replay_w = o->n_replay_w[i];
        }
        if (o && o->record) {
            md.record = o->record + i * o->record_stride;
            md.record_cap = o->record_stride;
        }
        double y0[10];
        y0[0] = omega0[i];
        for (int c = 0; c < 6; ++c) y0[1 + c] = S0[c * n + i];
        for (int c = 0; c < 3; ++c) y0[7 + c] = L0[c * n + i];
        Result<double> r = integrate_one<double>(m[i], m[n + i], y0, md);
        for (int c = 0; c < 10; ++c) y_final[c * n + i] = r.y[c];
        t_final[i] = r.t;
        steps[i] = r.acc; steps[n + i] = r.rej; steps[2 * n + i] = r.nrhs;
        status[i] = r.status;
        if (n_steps_tw) { n_steps_tw[i] = r.n_t; n_steps_tw[n + i] = r.n_w; }
        if (phase) phase[i] = r.phase;
    });
    return 0;
}

/* Forward-mode tangent of the replayed integration: directions dm [2][n],
 * dS0 [6][n], dL0 [3][n], domega0 [n] -> dy_final [10][n], dt_final [n].
 * The step sizes are the recorded ones (replay is required), so this is the
 * derivative of the discrete scheme with frozen steps. */
int oracle_tangent(int64_t n, const double* m, const double* S0, const double* L0,
                   const double* omega0, const double* dm, const double* dS0,
                   const double* dL0, const double* domega0, double omega_f, double tol,
                   const oracle_opts* o, double* y_final, double* dy_final, double* t_final,
                   double* dt_final, int32_t* status, int32_t nthreads) {
    if (!o || !o->replay) return -1;
    const Mode base = make_mode(omega_f, tol, o);
    parallel_for(n, nthreads, [&](int64_t i) {
        Mode md = base;
        md.replay = o->replay + i * o->replay_stride;
        md.n_replay_t = o->n_replay_t[i];
        md.n_replay_w = o->n_replay_w[i];
        Dual y0[10];
        y0[0] = Dual(omega0[i], domega0[i]);
        for (int c = 0; c < 6; ++c) y0[1 + c] = Dual(S0[c * n + i], dS0[c * n + i]);
        for (int c = 0; c < 3; ++c) y0[7 + c] = Dual(L0[c * n + i], dL0[c * n + i]);
        Result<Dual> r = integrate_one<Dual>(Dual(m[i], dm[i]), Dual(m[n + i], dm[n + i]), y0, md);
        for (int c = 0; c < 10; ++c) { y_final[c * n + i] = r.y[c].v; dy_final[c * n + i] = r.y[c].d; }
        t_final[i] = r.t.v; dt_final[i] = r.t.d;
        status[i] = r.status;
    });
    return 0;
}

/* Unit-vector scalar products: y [10][n] -> dots [3][n]. */
int oracle_observables(int64_t n, const double* y, double* dots) {
    for (int64_t i = 0; i < n; ++i) {
        double yy[10], d[3];
        for (int c = 0; c < 10; ++c) yy[c] = y[c * n + i];
        observables(yy, d);
        for (int c = 0; c < 3; ++c) dots[c * n + i] = d[c];
    }
    return 0;
}

/* Operation counts.  counts_rhs[7]: one RHS evaluation at the given state;
 * counts_run[7] and runinfo[3] (accepted, rejected, RHS evaluations): one
 * whole adaptive integration.  Order: add, mul, div, cbrt, log, sqrt, pow. */
int oracle_count_ops(const double* m2v, const double* y0, double omega_f, double tol,
                     const oracle_opts* o, int64_t* counts_rhs, int64_t* counts_run,
                     int64_t* runinfo) {
    const Mode md = make_mode(omega_f, tol, o);
    Counted m1(m2v[0]), m2(m2v[1]);
    Counted y[10], d[10];
    for (int c = 0; c < 10; ++c) y[c] = Counted(y0[c], true);
    g_ops = OpCounts{0, 0, 0, 0, 0, 0, 0};
    rhs(m1, m2, y, d, md.terms, md.theta_literal);
    const OpCounts a = g_ops;
    long long* cr = (long long*)counts_rhs;
    cr[0] = a.add; cr[1] = a.mul; cr[2] = a.div; cr[3] = a.cbrt_; cr[4] = a.log_;
    cr[5] = a.sqrt_; cr[6] = a.pow_;
    g_ops = OpCounts{0, 0, 0, 0, 0, 0, 0};
    Result<Counted> r = integrate_one<Counted>(m1, m2, y, md);
    const OpCounts b = g_ops;
    long long* cu = (long long*)counts_run;
    cu[0] = b.add; cu[1] = b.mul; cu[2] = b.div; cu[3] = b.cbrt_; cu[4] = b.log_;
    cu[5] = b.sqrt_; cu[6] = b.pow_;
    runinfo[0] = r.acc; runinfo[1] = r.rej; runinfo[2] = r.nrhs;
    return r.status;
}

/* The tableau as exact rationals, for the order-condition checks:
 * a [7][6][2], b [7][2], bhat [7][2], c [7][2] as (numerator, denominator). */
int oracle_tableau(double* a, double* b, double* bhat, double* c) {
    for (int s = 0; s < 7; ++s) {
        for (int j = 0; j < 6; ++j) { a[(s * 6 + j) * 2] = DP_A[s][j].num; a[(s * 6 + j) * 2 + 1] = DP_A[s][j].den; }
        b[2 * s] = DP_B[s].num; b[2 * s + 1] = DP_B[s].den;
        bhat[2 * s] = DP_BHAT[s].num; bhat[2 * s + 1] = DP_BHAT[s].den;
        c[2 * s] = DP_C[s].num; c[2 * s + 1] = DP_C[s].den;
    }
    return 0;
}

} /* extern "C" */
